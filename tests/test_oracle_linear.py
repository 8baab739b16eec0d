"""Pins of the oracle's linear SSE (App. B) against references it shares no code with.

  linear Ito SSE (state vector) ensemble  ->  Lindblad (Eq. 1), and E ||psi||^2 = 1
  linear Stratonovich SSE path  <->  linear Ito SSE path (same Brownian path, dt -> 0)
  otVMC linear (enumeration, complete ansatz)  <->  linear Stratonovich path: the ray, and the
      norm Q integrated from its own SDE against ||psi||^2 of the state vector
  F^lin - F and D^lin - D  ==  the relation App. B states, with dense expectations
  one step's increment of log Q  ==  dense <H_eff^{Strat,lin}> and <L_n>
  weighted trajectory average of App. B  ->  Lindblad (single spin)
"""
import numpy as np
import pytest

import oracle.exact as ex


def _fidelity(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def _n2_problem(orc, hx=0.6):
    # a decay and a dephasing channel: the dephasing channel's L^2 = rate * 1 term of
    # H_eff^{Strat,lin} changes only the norm
    n = 2
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.3), (2, 1, 0.3)]
    return n, J, jumps, hx


def test_linear_ito_sse_averages_to_lindblad():
    # the linear SSE's outer products average to rho: unnormalised <psi|A|psi> averages to
    # Tr(rho A), and the mean squared norm stays 1
    n = 2
    J = np.array([[0.0, 1.0], [1.0, 0.0]])
    jumps = [(0, 0, 0.5), (0, 1, 0.5)]
    H, Ls = ex.hamiltonian(J, 0.5), ex.jump_ops(n, jumps)
    rng = np.random.default_rng(4)
    dt, steps, nt = 2e-3, 250, 600
    mz, nrm = [], []
    for _ in range(nt):
        dws = rng.standard_normal((steps, 2)) * np.sqrt(dt)
        psi = ex.sse_path(ex.product_state_x(n), H, Ls, dws, dt, "ito_em", linear=True)[-1]
        q = np.vdot(psi, psi).real
        nrm.append(q)
        mz.append(ex.psi_observables(psi, n)[2] * q)
    nrm, mz = np.array(nrm), np.array(mz)
    assert nrm.std() > 0.05                      # the paths really lose their norm
    assert abs(nrm.mean() - 1) < 4 * nrm.std() / np.sqrt(nt)
    M, _ = ex.rho_observables(ex.lindblad_evolve(J, 0.5, jumps, [dt * steps])[0], n)
    assert abs(mz.mean() - M[2]) < 4 * mz.std() / np.sqrt(nt) + 0.01


def _ito_milstein_linear(psi0, H, Ls, dws, dt):
    # Milstein scheme on the linear Ito SSE for mutually commuting L_n (strong order 1):
    # psi += a dt + sum_n L_n psi dW_n + (1/2) sum_nm L_n L_m psi (dW_n dW_m - delta_nm dt)
    psi = np.array(psi0, dtype=np.complex128)
    for dw in dws:
        a = -1j * (H @ psi) - 0.5 * sum(L.conj().T @ (L @ psi) for L in Ls)
        inc = a * dt + sum(L @ psi * w for L, w in zip(Ls, dw))
        for i, Li in enumerate(Ls):
            for j, Lj in enumerate(Ls):
                inc = inc + 0.5 * (Li @ (Lj @ psi)) * (dw[i] * dw[j] - (dt if i == j else 0.0))
        psi = psi + inc
    return psi


def test_linear_stratonovich_path_matches_ito_path():
    # Heun on the Stratonovich form (App. B) against Milstein on the Ito form, same Brownian
    # path: both converge strongly, so agreement pins the -(1/2) L^2 conversion term (a
    # sigma_z channel, L^2 = rate * 1, makes it change the norm)
    n = 2
    J = np.array([[0.0, 1.0], [1.0, 0.0]])
    jumps = [(0, 0, 0.3), (2, 1, 0.3)]
    H, Ls = ex.hamiltonian(J, 0.6), ex.jump_ops(n, jumps)
    rng = np.random.default_rng(1)
    fine = rng.standard_normal((8000, 2)) * np.sqrt(0.5 / 8000)
    err = []
    for coarse in (8, 1):
        dws = fine.reshape(-1, coarse, 2).sum(1)
        dt = 0.5 / dws.shape[0]
        pe = _ito_milstein_linear(ex.product_state_x(n), H, Ls, dws, dt)
        ph = ex.sse_path(ex.product_state_x(n), H, Ls, dws, dt, "heun", linear=True)[-1]
        err.append(np.linalg.norm(pe - ph) / np.linalg.norm(ph))
    assert err[1] < 2e-4 and err[1] < 0.5 * err[0], err
    # negative controls: the nonlinear SSE, and the Ito drift read as a Stratonovich one
    pn = ex.sse_path(ex.product_state_x(n), H, Ls, fine, 0.5 / 8000, "heun")[-1]
    assert np.linalg.norm(pn - ph) / np.linalg.norm(ph) > 0.05
    pw = ex.sse_path(ex.product_state_x(n), H + 0.5j * sum(L @ L for L in Ls), Ls, fine, 0.5 / 8000, "heun",
                     linear=True)[-1]
    assert np.linalg.norm(pw - ph) / np.linalg.norm(ph) > 0.05


@pytest.mark.parametrize("scheme", [0, 1])
def test_otvmc_linear_complete_ansatz_follows_linear_sse(orc, scheme):
    # N = 2 Jastrow spans every ray: with exact averages the linear otVMC equations are the
    # linear Stratonovich SSE in other coordinates, and Q is that path's squared norm
    n, J, jumps, hx = _n2_problem(orc)
    H, Ls = ex.hamiltonian(J, hx), ex.jump_ops(n, jumps)
    pb = orc.Problem(J, hx, jumps)
    infid, qerr = [], []
    for dt in (4e-3, 1e-3):
        steps = int(round(0.4 / dt))
        cfg = orc.Config(enumerate=True, dt=dt, diag_shift=0.0, n_steps=steps, obs_every=steps, seed=9,
                         scheme=scheme, linear=True)
        th, _, st = orc.run(pb, 0, 0, cfg, np.zeros(3), 1, traj0=3)
        assert st == 0
        lq = orc.run.last_lognorm[0]
        assert lq[0] == 0.0
        dws = np.array([orc.draw_dw(9, 3, s, 2, dt) for s in range(steps)])
        ph = ex.sse_path(ex.product_state_x(n), H, Ls, dws, dt, "heun" if scheme == 0 else "midpoint",
                         linear=True)[-1]
        infid.append(1 - _fidelity(ex.jastrow_psi(n)(th[0]), ph))
        qerr.append(abs(np.exp(lq[1]) / np.vdot(ph, ph).real - 1))
    assert infid[1] < 5e-8, infid
    # Q and ||psi||^2 come from different discretisations of one Stratonovich solution (log Q
    # against the vector itself) on a different Brownian path per dt: both errors stay
    # O(dt)-small, while log Q itself moves by O(0.1 .. 1)
    assert qerr[0] < 2e-3 and qerr[1] < 3e-4, qerr
    assert abs(lq[1]) > 0.05


def test_nonlinear_run_keeps_log_norm_zero(orc):
    n, J, jumps, hx = _n2_problem(orc)
    cfg = orc.Config(enumerate=True, dt=0.01, diag_shift=0.0, n_steps=4, obs_every=2, seed=9)
    _, _, st = orc.run(orc.Problem(J, hx, jumps), 0, 0, cfg, np.zeros(3), 2)
    assert st == 0 and np.all(orc.run.last_lognorm == 0.0)


@pytest.mark.parametrize("kind,nh", [(0, 0), (1, 2)])
def test_linear_force_relation_and_log_norm_increment(orc, kind, nh):
    # F^lin = F - i sum_n <L_n + L_n^dag> N^n (App. B); hence D^lin = D - dt sum_n <L+L^dag> N^n.
    # The increment of log Q is 2 Im<E_eff^lin> dt + 2 sum_n Re<B^n> dW_n, here against dense
    # expectations of H_eff^{Strat,lin} and L_n on the represented state.
    n = 3
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, 0, 0.4), (1, 1, 0.3), (2, 2, 0.2)]
    pb = orc.Problem(J, 0.7, jumps)
    m = orc.n_params(kind, n, nh)
    rng = np.random.default_rng(5)
    th = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    dw = np.array([0.03, -0.05, 0.02])
    r0 = orc.evaluate(pb, kind, nh, orc.Config(enumerate=True, dt=0.01), th, None, dw=dw)
    r1 = orc.evaluate(pb, kind, nh, orc.Config(enumerate=True, dt=0.01, linear=True), th, None, dw=dw)
    psi = (ex.jastrow_psi(n) if kind == 0 else ex.rbm_psi(n, nh))(th)
    H, Ls = ex.hamiltonian(J, 0.7), ex.jump_ops(n, jumps)
    nrm = np.vdot(psi, psi).real
    lexp = np.array([np.vdot(psi, L @ psi) / nrm for L in Ls])
    c = 2 * lexp.real
    assert np.allclose(r1["bmean"], lexp, atol=1e-12)
    assert np.allclose(r1["F"], r0["F"] - 1j * (c[:, None] * r0["Nn"]).sum(0), atol=1e-10)
    assert np.allclose(r1["D"], r0["D"] - 0.01 * (c[:, None] * r0["Nn"]).sum(0), atol=1e-12)
    Heff = H - 0.5j * sum(L.conj().T @ L + L @ L for L in Ls)
    e = np.vdot(psi, Heff @ psi) / nrm
    want = 2 * e.imag * 0.01 + 2 * (lexp.real * dw).sum()
    assert abs(r1["dlognorm"] - want) < 1e-12
    assert r0["dlognorm"] == 0.0 or abs(r0["dlognorm"] - want) > 1e-6


def test_linear_weighted_ensemble_matches_lindblad(orc):
    pb = orc.Problem(np.zeros((1, 1)), 1.0, [(0, 0, 0.5)])
    cfg = orc.Config(enumerate=True, dt=0.005, diag_shift=0.0, n_steps=200, obs_every=100, seed=13, linear=True)
    nt = 800
    _, obs, st = orc.run(pb, 0, 0, cfg, np.zeros(1), nt, n_threads=8)
    assert st == 0
    q = np.exp(orc.run.last_lognorm)
    rhos = ex.lindblad_evolve(np.zeros((1, 1)), 1.0, [(0, 0, 0.5)], [0.0, 0.5, 1.0])
    for io, rho in enumerate(rhos):
        M, _ = ex.rho_observables(rho, 1)
        Mo, _, _ = orc.ensemble(obs[:, io], 1, weights=q[:, io])
        w = obs[:, io, :3] * q[:, io, None]
        se = w.std(0) / np.sqrt(nt)
        assert np.all(np.abs(Mo - M) < 4.5 * se + 1e-3), (io, Mo, M, se)
        assert abs(q[:, io].mean() - 1) < 4.5 * q[:, io].std() / np.sqrt(nt) + 1e-3
    assert q[:, 2].std() > 0.05
    # unweighted, the same trajectories are off: the weights carry the physics
    Mu, _, _ = orc.ensemble(obs[:, 2], 1)
    M2, _ = ex.rho_observables(rhos[2], 1)
    assert np.abs(Mu - M2).max() > 0.02
