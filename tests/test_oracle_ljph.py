"""Pins of the oracle's LJPHd ansatz (partially inhomogeneous long-range Jastrow, LITF section):
own eta for pairs at distance <= d, one shared eta per farther distance, biases always own.

  parameter count against the open-chain count (and the printed count where they agree)
  log psi against an independent dense construction of the features
  flip ratios and O_k against brute force and finite differences
  d = N-1 is the all-pair Jastrow, parameter for parameter
  S, F, N^n against the all-pair Jastrow's through the chain rule, and against dense algebra
  closed system at h = 0 with distance-only couplings: eta_D(t) = -i J_D t exactly (LJH)
"""
import numpy as np
import pytest

import oracle.exact as ex

LJPH = 2


def _count(n, d):
    # biases + own pairs (sum over D <= d of N - D) + one shared eta per distance d+1 .. N-1
    return n + sum(n - D for D in range(1, d + 1)) + (n - 1 - d)


@pytest.mark.parametrize("n", [2, 5, 9, 64])
def test_parameter_count(orc, n):
    for d in range(n):
        assert orc.n_params(LJPH, n, d) == _count(n, d)
    # the printed count 2N - 1 - d + N d / 2 agrees at both ends: LJH and LJNH
    assert orc.n_params(LJPH, n, 0) == 2 * n - 1
    assert orc.n_params(LJPH, n, n - 1) == n * (n + 1) // 2


@pytest.mark.parametrize("n,d", [(5, 0), (5, 1), (6, 2), (7, 6)])
def test_log_psi_matches_dense_features(orc, n, d):
    rng = np.random.default_rng(n * 10 + d)
    m = orc.n_params(LJPH, n, d)
    th = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    psi = ex.ljph_psi(n, d)(th)
    s = ex.spins(n)
    lp = np.array([orc.logpsi(LJPH, n, d, th, s[x]) for x in range(1 << n)])
    assert np.allclose(np.exp(lp), psi, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,d", [(5, 0), (6, 1), (6, 3)])
def test_flip_ratios_and_log_derivatives(orc, n, d):
    rng = np.random.default_rng(7 + n + d)
    m = orc.n_params(LJPH, n, d)
    th = 0.3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    for _ in range(3):
        s = rng.choice([-1, 1], size=n).astype(np.int8)
        f1, f2, O = orc.local_quantities(LJPH, n, d, th, s)
        base = orc.logpsi(LJPH, n, d, th, s)
        for i in range(n):
            t = s.copy()
            t[i] = -t[i]
            assert np.exp(f1[i]) == pytest.approx(np.exp(orc.logpsi(LJPH, n, d, th, t) - base), rel=1e-11)
            for k in range(i + 1, n):
                u = t.copy()
                u[k] = -u[k]
                assert np.exp(f2[i, k]) == pytest.approx(np.exp(orc.logpsi(LJPH, n, d, th, u) - base), rel=1e-11)
        h = 1e-6
        for k in range(m):
            e = np.zeros(m, np.complex128)
            e[k] = h
            fd = (orc.logpsi(LJPH, n, d, th + e, s) - orc.logpsi(LJPH, n, d, th - e, s)) / (2 * h)
            assert O[k] == pytest.approx(fd, abs=1e-8)
        # shared parameters carry integer O: the number of agreeing minus disagreeing pairs
        for D in range(d + 1, n):
            assert O[n + _count(n, d) - n - (n - 1 - d) + D - d - 1] == sum(s[j] * s[j + D] for j in range(n - D))


def _expand(n, d, th):
    """LJPHd parameters -> the all-pair Jastrow parameters of the same state (psi_L(t) = psi_J(P t))."""
    full = np.zeros(n + n * (n - 1) // 2, np.complex128)
    full[:n] = th[:n]
    own = n
    shared = n + _count(n, d) - n - (n - 1 - d)
    P = np.zeros((full.size, th.size))
    P[np.arange(n), np.arange(n)] = 1
    idx = n
    for j in range(n):
        for k in range(j + 1, n):
            src = own if k - j <= d else shared + (k - j - d - 1)
            if k - j <= d:
                own += 1
            P[idx, src] = 1
            idx += 1
    return P @ th, P


def test_full_range_is_the_all_pair_jastrow(orc):
    n = 6
    rng = np.random.default_rng(1)
    m = orc.n_params(0, n)
    th = 0.2 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    J = orc.couplings("obc", n, 1.5, 1.0)
    pb = orc.Problem(J, 0.7, [(0, i, 0.1) for i in range(n)])
    cfg = orc.Config(n_samples=256, n_chains=8, dt=0.01, diag_shift=1e-4, seed=4)
    ch0 = orc.init_chains(4, 0, n, 8)
    ch1 = ch0.copy()
    dw = orc.draw_dw(4, 0, 0, n, 0.01)
    r0 = orc.evaluate(pb, 0, 0, cfg, th, ch0, dw=dw)
    r1 = orc.evaluate(pb, LJPH, n - 1, cfg, th, ch1, dw=dw)
    for key in ("samples", "eloc", "S", "F", "D", "delta"):
        assert np.array_equal(r0[key], r1[key]), key


@pytest.mark.parametrize("d", [0, 1, 2])
def test_chain_rule_against_the_all_pair_jastrow(orc, d):
    # with exact averages, S_L = P^T S_J P, F_L = P^T F_J, N^n_L = P^T N^n_J at theta_J = P theta_L
    n = 5
    rng = np.random.default_rng(3 + d)
    m = orc.n_params(LJPH, n, d)
    th = 0.25 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    thj, P = _expand(n, d, th)
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.2) for i in range(n)] + [(2, 1, 0.1)]
    pb = orc.Problem(J, 0.6, jumps)
    cfg = orc.Config(enumerate=True, dt=0.01, diag_shift=1e-4)
    dw = 0.1 * rng.standard_normal(len(jumps))
    rl = orc.evaluate(pb, LJPH, d, cfg, th, None, dw=dw)
    rj = orc.evaluate(pb, 0, 0, cfg, thj, None, dw=dw)
    assert np.abs(rl["S"] - P.T @ rj["S"] @ P).max() < 1e-12
    assert np.abs(rl["F"] - P.T @ rj["F"]).max() < 1e-12
    assert np.abs(rl["Nn"] - rj["Nn"] @ P).max() < 1e-12
    assert np.abs(rl["eloc"] - rj["eloc"]).max() < 1e-12
    # and against dense algebra on the independently built features
    S, F, Nn, bm = ex.dense_sfn(ex.ljph_psi(n, d), th, J, 0.6, jumps)
    assert np.abs(rl["S"] - S).max() < 1e-8 * max(1.0, np.abs(S).max())
    assert np.abs(rl["F"] - F).max() < 1e-8 * max(1.0, np.abs(F).max())
    assert np.abs(rl["Nn"] - Nn).max() < 1e-8


def test_closed_system_ljh_closed_form(orc):
    # gamma = 0, h = 0, open-chain couplings that depend on |j - k| only: E_loc = sum_D J_D O_D
    # with O_D the shared log-derivative of distance D, so F = S J exactly on any sample set
    # and, at eps = 0, delta = -i J dt: eta_D(t) = -i J_D t, a(t) = 0 (Monte Carlo mode)
    n = 7
    J = orc.couplings("obc", n, 1.5, 1.0)
    for D in range(1, n):
        assert np.allclose([J[j, j + D] for j in range(n - D)], J[0, D], rtol=0, atol=0)
    pb = orc.Problem(J, 0.0, [])
    m = orc.n_params(LJPH, n, 0)
    cfg = orc.Config(n_samples=512, n_chains=8, burn_sweeps=2, dt=0.01, diag_shift=0.0, n_steps=10, seed=3)
    th, _, st = orc.run(pb, LJPH, 0, cfg, np.zeros(m), 2)
    assert st == 0
    want = np.zeros(m, np.complex128)
    want[n:] = -1j * 0.1 * J[0, 1:]
    assert np.abs(th - want[None, :]).max() < 1e-11
