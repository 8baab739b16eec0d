"""Pins of the oracle's estimator layer (definitions after Eq. 8) and of its solve.

* enumeration-mode S, F, N^n and <B^n> equal independent dense algebra on 2^N vectors
  (derivative vectors by finite differences, H_eff^Strat of Eq. 5 as an explicit matrix);
* D = -i F dt + sum_n N^n dW_n;
* Monte Carlo estimates converge to the enumeration values;
* the Jastrow S is an exact dyadic rational (O_k = +-1), so it is bitwise reproducible;
* delta solves (S + eps I) delta = D;
* App. A: the c-number terms of H_eff^Strat and the change to the non-normalised state leave F
  unchanged (checked on the dense side, where both forms can be written explicitly).
"""
import numpy as np
import pytest

import oracle.exact as ex


def _problem(orc, n, hx, extra=True):
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    if extra:
        jumps += [(2, i, 0.05) for i in range(n)] + [(1, 1, 0.07)]
    return J, jumps, orc.Problem(J, hx, jumps)


@pytest.mark.parametrize("kind,nh", [(0, 0), (1, 3)])
def test_enumeration_matches_dense_algebra(orc, kind, nh):
    rng = np.random.default_rng(11 + kind)
    n = 4
    J, jumps, pb = _problem(orc, n, 0.7)
    m = orc.n_params(kind, n, nh)
    th = 0.2 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    dw = 0.1 * rng.standard_normal(len(jumps))
    cfg = orc.Config(enumerate=True, dt=0.01, diag_shift=1e-4)
    r = orc.evaluate(pb, kind, nh, cfg, th, None, dw=dw)
    assert r["status"] == 0
    f = ex.jastrow_psi(n) if kind == 0 else ex.rbm_psi(n, nh)
    S, F, Nn, bm = ex.dense_sfn(f, th, J, 0.7, jumps)
    assert np.abs(r["S"] - S).max() < 1e-8 * max(1.0, np.abs(S).max())
    assert np.abs(r["F"] - F).max() < 1e-8 * max(1.0, np.abs(F).max())
    assert np.abs(r["Nn"] - Nn).max() < 1e-8
    assert np.abs(r["bmean"] - bm).max() < 1e-13
    D = -1j * r["F"] * cfg.dt + dw @ r["Nn"]
    assert np.abs(r["D"] - D).max() < 1e-15
    A = r["S"] + cfg.diag_shift * np.eye(m)
    assert np.abs(A @ r["delta"] - r["D"]).max() < 1e-12
    assert np.allclose(r["S"], r["S"].conj().T, atol=0)


def test_c_number_terms_do_not_change_F():
    # App. A: H~_eff = H - (i/2) sum (L^+L - 2<L+L^+>L + L^2) gives the same theta dynamics as
    # the full H_eff^Strat of Eq. 5 (which adds <L+L^+>^2 - <L^2 + 2L^+L + L^+^2>/2): F is a
    # covariance, so any multiple of the identity cancels.
    rng = np.random.default_rng(5)
    n = 3
    import oracle
    J = oracle.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.2) for i in range(n)] + [(2, 0, 0.1)]
    f = ex.jastrow_psi(n)
    m = n + n * (n - 1) // 2
    th = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    psi = f(th)
    H = ex.hamiltonian(J, 0.4).toarray()
    Ls = [L.toarray() for L in ex.jump_ops(n, jumps)]
    Hfull, Hred = H.copy(), H.copy()
    for L in Ls:
        Ld = L.conj().T
        c = 2 * np.real(np.vdot(psi, L @ psi) / np.vdot(psi, psi))
        cn = c * c - 0.5 * np.vdot(psi, (L @ L + 2 * Ld @ L + Ld @ Ld) @ psi) / np.vdot(psi, psi)
        Hred = Hred - 0.5j * (Ld @ L - 2 * c * L + L @ L)
        Hfull = Hfull - 0.5j * (Ld @ L - 2 * c * L + L @ L + cn * np.eye(psi.size))
    h = 1e-6
    dpsi = np.array([(f(th + h * np.eye(m)[k]) - f(th - h * np.eye(m)[k])) / (2 * h) for k in range(m)])
    nrm = np.vdot(psi, psi).real
    ob = dpsi.conj() @ psi / nrm

    def force(Hm):
        Hp = Hm @ psi
        return dpsi.conj() @ Hp / nrm - ob * np.vdot(psi, Hp) / nrm

    assert np.abs(force(Hfull) - force(Hred)).max() < 1e-12


def test_monte_carlo_converges_to_enumeration(orc):
    rng = np.random.default_rng(3)
    n = 5
    J, jumps, pb = _problem(orc, n, 0.5, extra=False)
    m = orc.n_params(0, n)
    th = 0.25 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    dw = 0.1 * rng.standard_normal(len(jumps))
    ex_r = orc.evaluate(pb, 0, 0, orc.Config(enumerate=True, dt=0.01), th, None, dw=dw)
    errs = []
    for ns in (1024, 16384):
        cfg = orc.Config(n_samples=ns, n_chains=16, burn_sweeps=20, dt=0.01, seed=1)
        ch = orc.init_chains(1, 0, n, 16)
        r = orc.evaluate(pb, 0, 0, cfg, th, ch, dw=dw, first=True)
        errs.append((np.abs(r["S"] - ex_r["S"]).max(), np.abs(r["F"] - ex_r["F"]).max(),
                     np.abs(r["bmean"] - ex_r["bmean"]).max()))
    # statistical error ~ N_s^-1/2: well inside 6/sqrt(N_s) at both sizes, and shrinking
    for (es, ef, eb), ns in zip(errs, (1024, 16384)):
        assert es < 6 / np.sqrt(ns) and ef < 12 / np.sqrt(ns) and eb < 3 / np.sqrt(ns)
    assert errs[1][0] < errs[0][0]


def test_jastrow_S_is_exact(orc):
    # O_k = +-1 and N_s = 2^10: every S entry is an integer combination of 2^-20, computed
    # exactly in double; rebuild it from integer sums and compare bitwise.
    rng = np.random.default_rng(9)
    n = 6
    J, jumps, pb = _problem(orc, n, 1.0, extra=False)
    m = orc.n_params(0, n)
    th = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    cfg = orc.Config(n_samples=1024, n_chains=16, burn_sweeps=3, dt=0.01, seed=4)
    ch = orc.init_chains(4, 2, n, 16)
    r = orc.evaluate(pb, 0, 0, cfg, th, ch, traj=2, dw=np.zeros(len(jumps)))
    s = r["samples"].astype(np.int64)
    pairs = [(j, k) for j in range(n) for k in range(j + 1, n)]
    O = np.concatenate([s, np.stack([s[:, j] * s[:, k] for j, k in pairs], 1)], 1)
    G = O.T @ O
    c = O.sum(0)
    S_exact = (1024 * G - np.outer(c, c)) / 1024.0 ** 2
    assert np.array_equal(r["S"].real, S_exact) and not np.any(r["S"].imag)


def test_metropolis_samples_follow_psi_squared(orc):
    # chi-square of the chain histogram against |psi|^2 / Z over all 2^N configurations
    rng = np.random.default_rng(21)
    n = 4
    J, jumps, pb = _problem(orc, n, 0.3, extra=False)
    m = orc.n_params(1, n, 3)
    th = 0.4 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    cfg = orc.Config(n_samples=32768, n_chains=32, burn_sweeps=20, thin_sweeps=2, dt=0.01, seed=8)
    r = orc.evaluate(pb, 1, 3, cfg, th, orc.init_chains(8, 0, n, 32), dw=np.zeros(len(jumps)), want_solve=False)
    idx = ((r["samples"] > 0).astype(np.int64) * (1 << np.arange(n))).sum(1)
    counts = np.bincount(idx, minlength=1 << n)
    p = np.abs(ex.rbm_psi(n, 3)(th)) ** 2
    p /= p.sum()
    e = p * idx.size
    chi2 = np.sum((counts - e) ** 2 / e)
    # 15 degrees of freedom; thinning leaves some autocorrelation, so allow a generous bound
    assert chi2 < 60, chi2


@pytest.mark.parametrize("kind,nh", [(0, 0), (1, 3)])
def test_moment_estimators_match_dense_expectations(orc, kind, nh):
    # local estimators of sigma^a_i and sigma^a_i sigma^b_j (one- and two-flip ratios) averaged
    # exactly over |psi|^2 must equal <psi|M_a|psi> and <psi|{M_a,M_b}/2|psi> from dense algebra
    rng = np.random.default_rng(31 + kind)
    n = 4
    J, jumps, pb = _problem(orc, n, 0.3, extra=False)
    m = orc.n_params(kind, n, nh)
    th = 0.35 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    r = orc.evaluate(pb, kind, nh, orc.Config(enumerate=True), th, None, want_solve=False)
    f = ex.jastrow_psi(n) if kind == 0 else ex.rbm_psi(n, nh)
    want = ex.psi_observables(f(th), n)
    assert np.abs(r["obs"] - want).max() < 1e-13
    assert np.abs(want[[1, 6, 8]]).min() > 1e-3     # the sigma^y terms are really exercised
