"""Pins of the oracle's dynamics against the exact references.

Chain of pins, each link independent of the next:
  App. D closed form  <->  Lindblad (Eq. 1, exact matrix exponential, and RK4)
  Ito SSE (Eq. 2) ensemble  ->  Lindblad
  Stratonovich SSE (Eqs. 4-5) path  <->  Ito SSE path (same Brownian path, dt -> 0)
  otVMC (Eq. 8, enumeration, complete ansatz)  <->  Stratonovich SSE path (same dW)
  otVMC closed system at h = 0  ->  theta_eta(t) = -i J t exactly (any sample set)
  otVMC ensemble  ->  Lindblad / single-spin closed form
"""
import numpy as np
import pytest

import oracle.exact as ex


# ------------------------------------------------------------------ exact references
@pytest.mark.parametrize("n,alpha,kappa", [(4, 1.0, 0.5), (5, 1.0, 0.5), (6, 1.5, 0.3)])
def test_appendix_d_pbc_matches_lindblad(orc, n, alpha, kappa):
    J = orc.couplings("pbc", n, alpha, 1.0)
    jumps = [(0, i, kappa) for i in range(n)]
    for t, rho in zip((0.3, 0.8), ex.lindblad_evolve(J, 0.0, jumps, [0.3, 0.8])):
        M, C = ex.rho_observables(rho, n)
        Ma, Ca = ex.appd_pbc(n, alpha, 1.0, kappa, t)
        assert np.abs(M - Ma).max() < 1e-12 and np.abs(C - Ca).max() < 1e-12


@pytest.mark.parametrize("n", [5, 6])
def test_appendix_d_site_resolved_matches_lindblad_obc(orc, n):
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.3) for i in range(n)]
    for t, rho in zip((0.5, 1.0), ex.lindblad_evolve(J, 0.0, jumps, [0.5, 1.0])):
        M, C = ex.rho_observables(rho, n)
        Mg, Cg = ex.appd_general(J, 0.3, t)
        assert np.abs(M - Mg).max() < 1e-12 and np.abs(C - Cg).max() < 1e-12


def test_appendix_d_sign_convention(orc):
    # App. D as printed describes H = +sum J_ij sz sz; the opposite sign flips M_y, C_xy, C_yz
    n = 5
    J = orc.couplings("pbc", n, 1.0, 1.0)
    jumps = [(0, i, 0.5) for i in range(n)]
    rho_m = ex.lindblad_evolve(-J, 0.0, jumps, [0.8])[0]
    M, C = ex.rho_observables(rho_m, n)
    Ma, Ca = ex.appd_pbc(n, 1.0, 1.0, 0.5, 0.8)
    assert abs(M[1] + Ma[1]) < 1e-12 and abs(M[1]) > 1e-3
    assert abs(C[0, 1] + Ca[0, 1]) < 1e-12 and abs(C[1, 2] + Ca[1, 2]) < 1e-12
    assert abs(ex.xi2(M, C, n) - ex.xi2(Ma, Ca, n)) < 1e-12


def test_rk4_matches_matrix_exponential(orc):
    n = 3
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.2) for i in range(n)] + [(2, 1, 0.1)]
    r1 = ex.lindblad_evolve(J, 0.8, jumps, [0.5])[0]
    r2 = ex.lindblad_rk4(J, 0.8, jumps, 0.5, 1e-3)
    assert np.abs(r1 - r2).max() < 1e-11


def test_single_spin_decay_closed_form():
    # J = 0, h = 0, L = sqrt(kappa) sigma^-: <sz> = e^{-kappa t} - 1, <sx> = e^{-kappa t / 2}
    for t, rho in zip((0.2, 1.0, 3.0), ex.lindblad_evolve(np.zeros((1, 1)), 0.0, [(0, 0, 0.7)], [0.2, 1.0, 3.0])):
        M, _ = ex.rho_observables(rho, 1)
        assert abs(M[2] - (np.exp(-0.7 * t) - 1)) < 1e-13 and abs(M[0] - np.exp(-0.35 * t)) < 1e-13
        Ma, _ = ex.appd_pbc(2, 1.0, 0.0, 0.7, t)   # J = 0 reduces App. D to independent spins
        assert abs(Ma[2] - (np.exp(-0.7 * t) - 1)) < 1e-13 and abs(Ma[0] - np.exp(-0.35 * t)) < 1e-13


def test_closed_system_product_formula(orc):
    # kappa = 0, h = 0: Phi(a) = cos(2at), so M_x = prod_{d} cos(2 J_d t)
    n = 6
    J = orc.couplings("pbc", n, 1.0, 1.0)
    t = 0.7
    Ma, _ = ex.appd_pbc(n, 1.0, 1.0, 0.0, t)
    assert abs(Ma[0] - np.prod(np.cos(2 * J[0, 1:] * t))) < 1e-13


def test_coherent_state_squeezing_is_one(orc):
    n = 6
    M, C = ex.rho_observables(ex.lindblad_evolve(orc.couplings("obc", n, 1.5, 1.0), 0.5, [], [0.0])[0], n)
    assert abs(ex.xi2(M, C, n) - 1.0) < 1e-13


# ------------------------------------------------------------------ SSE references
def test_ito_sse_preserves_norm_and_averages_to_lindblad(orc):
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.5), (0, 1, 0.5)]
    H, Ls = ex.hamiltonian(J, 0.5), ex.jump_ops(n, jumps)
    psi0 = ex.product_state_x(n)
    rng = np.random.default_rng(2)
    dt, steps, nt = 2e-3, 250, 400
    mz, nrm = [], []
    for _ in range(nt):
        dws = rng.standard_normal((steps, 2)) * np.sqrt(dt)
        psi = ex.sse_path(psi0, H, Ls, dws, dt, "ito_em")[-1]
        nrm.append(np.vdot(psi, psi).real)
        mz.append(ex.psi_observables(psi, n)[2])
    # Eq. 2 preserves the norm; Euler-Maruyama does so up to a small random walk
    assert abs(np.mean(nrm) - 1) < 0.01 and np.max(np.abs(np.array(nrm) - 1)) < 0.1
    M, _ = ex.rho_observables(ex.lindblad_evolve(J, 0.5, jumps, [dt * steps])[0], n)
    assert abs(np.mean(mz) - M[2]) < 4 * np.std(mz) / np.sqrt(nt) + 0.01


@pytest.mark.parametrize("nch", [1, 2])
def test_stratonovich_path_matches_ito_path(orc, nch):
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.3), (0, 1, 0.3)][:nch]
    H, Ls = ex.hamiltonian(J, 0.6), ex.jump_ops(n, jumps)
    psi0 = ex.product_state_x(n)
    rng = np.random.default_rng(0)
    fine = rng.standard_normal((8000, nch)) * np.sqrt(0.5 / 8000)
    infid = []
    for coarse in (8, 1):   # same Brownian path, coarse and fine resolution
        dws = fine.reshape(-1, coarse, nch).sum(1)
        dt = 0.5 / dws.shape[0]
        pe = ex.sse_path(psi0, H, Ls, dws, dt, "ito_em")[-1]
        ph = ex.sse_path(psi0, H, Ls, dws, dt, "heun")[-1]
        infid.append(1 - abs(np.vdot(pe, ph)) ** 2 / (np.vdot(pe, pe).real * np.vdot(ph, ph).real))
    assert infid[1] < 2e-6 and infid[1] < infid[0]


# ------------------------------------------------------------------ otVMC oracle dynamics
def _fidelity(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


@pytest.mark.parametrize("nch,scheme", [(1, 0), (2, 0), (2, 1)])
def test_otvmc_complete_ansatz_follows_state_vector_sse(orc, nch, scheme):
    # N = 2 Jastrow (a_1, a_2, eta_12) spans every ray, so with exact averages otVMC is the
    # Stratonovich SSE in other coordinates: same dW, same scheme -> paths agree as dt -> 0.
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.3), (0, 1, 0.3)][:nch]
    H, Ls = ex.hamiltonian(J, 0.6), ex.jump_ops(n, jumps)
    pb = orc.Problem(J, 0.6, jumps)
    infid = []
    for dt in (4e-3, 1e-3):
        steps = int(round(0.4 / dt))
        cfg = orc.Config(enumerate=True, dt=dt, diag_shift=0.0, n_steps=steps, seed=7, scheme=scheme)
        th, _, st = orc.run(pb, 0, 0, cfg, np.zeros(3), 1, traj0=5)
        assert st == 0
        dws = np.array([orc.draw_dw(7, 5, s, nch, dt) for s in range(steps)])
        ph = ex.sse_path(ex.product_state_x(n), H, Ls, dws, dt, "heun" if scheme == 0 else "midpoint")[-1]
        infid.append(1 - _fidelity(ex.jastrow_psi(n)(th[0]), ph))
    assert infid[1] < 5e-8, infid


def test_otvmc_detects_wrong_noise_path(orc):
    # the previous comparison is sharp: a different noise path gives an O(1) infidelity
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.3), (0, 1, 0.3)]
    pb = orc.Problem(J, 0.6, jumps)
    dt, steps = 2e-3, 200
    th, _, _ = orc.run(pb, 0, 0, orc.Config(enumerate=True, dt=dt, diag_shift=0.0, n_steps=steps, seed=7), np.zeros(3), 1)
    dws = np.array([orc.draw_dw(8, 0, s, 2, dt) for s in range(steps)])
    ph = ex.sse_path(ex.product_state_x(n), ex.hamiltonian(J, 0.6), ex.jump_ops(n, jumps), dws, dt)[-1]
    assert 1 - _fidelity(ex.jastrow_psi(n)(th[0]), ph) > 1e-3


def test_closed_system_jastrow_closed_form(orc):
    # gamma = 0, h = 0: E_loc = sum_p J_p O_p, so F = S J exactly on any sample set and, with
    # eps = 0, delta = -i J dt: eta(t) = -i J t, a(t) = 0 (Monte Carlo mode, finite N_s).
    n = 6
    J = orc.couplings("obc", n, 1.5, 1.0)
    pb = orc.Problem(J, 0.0, [])
    m = orc.n_params(0, n)
    cfg = orc.Config(n_samples=512, n_chains=8, burn_sweeps=2, dt=0.01, diag_shift=0.0, n_steps=10, seed=3)
    th, _, st = orc.run(pb, 0, 0, cfg, np.zeros(m), 2)
    assert st == 0
    want = np.zeros(m, np.complex128)
    want[n:] = -1j * 0.1 * np.array([J[j, k] for j in range(n) for k in range(j + 1, n)])
    assert np.abs(th - want[None, :]).max() < 1e-12


def _single_spin_ensemble(orc, scheme, n_traj=800):
    # N = 1 (a only) spans every ray.  A transverse field keeps z = psi_dn/psi_up off the real
    # axis: at h = 0 the single-spin dynamics is real and z can cross 0, the pole of
    # a = -log(z)/2, where S -> 0 and no finite step can follow the trajectory.
    pb = orc.Problem(np.zeros((1, 1)), 1.0, [(0, 0, 0.5)])
    cfg = orc.Config(enumerate=True, dt=0.005, diag_shift=0.0, n_steps=200, obs_every=100, seed=11, scheme=scheme)
    _, obs, st = orc.run(pb, 0, 0, cfg, np.zeros(1), n_traj, n_threads=8)
    rhos = ex.lindblad_evolve(np.zeros((1, 1)), 1.0, [(0, 0, 0.5)], [0.0, 0.5, 1.0])
    z = []
    for io, rho in enumerate(rhos):
        M, _ = ex.rho_observables(rho, 1)
        mo = obs[:, io, :3]
        z.append((mo.mean(0) - M) / np.maximum(mo.std(0) / np.sqrt(n_traj), 1e-12))
    return st, np.array(z)


def test_single_spin_otvmc_ensemble_matches_lindblad(orc):
    st, z = _single_spin_ensemble(orc, 0)
    assert st == 0
    assert np.all(np.abs(z) < 4.5), z


def test_euler_is_not_stratonovich_consistent(orc):
    # App. C: a single Euler step on the Stratonovich form misses the noise-induced drift, and
    # its trajectory average drifts many standard errors away from the Lindblad result
    _, z = _single_spin_ensemble(orc, 2)
    assert np.abs(z[1:]).max() > 5, z


def test_ensemble_n2_matches_lindblad(orc):
    # Trajectory average (Eq. 3) of the complete N = 2 ansatz against Eq. 1.  A tiny diagonal
    # shift keeps every trajectory finite: without it a few percent of the paths reach the
    # poles of the log-parametrisation (S singular) and the survivors are a biased sample.
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.3), (0, 1, 0.3)]
    pb = orc.Problem(J, 1.0, jumps)
    cfg = orc.Config(enumerate=True, dt=0.005, diag_shift=1e-6, n_steps=160, obs_every=80, seed=2)
    _, obs, st = orc.run(pb, 0, 0, cfg, np.zeros(3), 1000, n_threads=8)
    assert st == 0
    rhos = ex.lindblad_evolve(J, 1.0, jumps, [0.0, 0.4, 0.8])
    for io, rho in enumerate(rhos):
        M, C = ex.rho_observables(rho, n)
        Mo, Co, _ = orc.ensemble(obs[:, io], n)
        se = obs[:, io, :3].std(0) / np.sqrt(obs.shape[0])
        assert np.all(np.abs(Mo - M) < 4.5 * se + 1e-3), (io, Mo, M)
        sse = obs[:, io, 3:].std(0) / np.sqrt(obs.shape[0])
        s_exact = np.array([C[0, 0], C[1, 1], C[2, 2], C[0, 1], C[0, 2], C[1, 2]]) + \
            np.array([M[0] ** 2, M[1] ** 2, M[2] ** 2, M[0] * M[1], M[0] * M[2], M[1] * M[2]])
        assert np.all(np.abs(obs[:, io, 3:].mean(0) - s_exact) < 4.5 * sse + 1e-3)
