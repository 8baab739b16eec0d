"""Pins of the oracle's ansatz layer (Eqs. 11-12): flip log-ratios against brute-force
differences of log psi, two-flip ratios likewise, and O_k = d log psi / d theta_k against
central finite differences (psi is holomorphic in theta)."""
import numpy as np
import pytest


def _rand_theta(rng, m, scale=0.3):
    return scale * (rng.standard_normal(m) + 1j * rng.standard_normal(m))


@pytest.mark.parametrize("kind,n,nh", [(0, 5, 0), (0, 9, 0), (1, 5, 4), (1, 6, 9)])
def test_flip_ratios_and_log_derivatives(orc, kind, n, nh):
    rng = np.random.default_rng(kind * 100 + n)
    m = orc.n_params(kind, n, nh)
    assert m == (n + n * (n - 1) // 2 if kind == 0 else n + nh + n * nh)
    th = _rand_theta(rng, m)
    for _ in range(3):
        s = rng.choice([-1, 1], size=n).astype(np.int8)
        f1, f2, O = orc.local_quantities(kind, n, nh, th, s)
        base = orc.logpsi(kind, n, nh, th, s)
        for i in range(n):
            t = s.copy()
            t[i] = -t[i]
            # compare ratios, not logs: log-differences agree only modulo 2 pi i
            assert np.exp(f1[i]) == pytest.approx(np.exp(orc.logpsi(kind, n, nh, th, t) - base), rel=1e-11)
            for k in range(n):
                if k == i:
                    continue
                u = t.copy()
                u[k] = -u[k]
                assert np.exp(f2[i, k]) == pytest.approx(np.exp(orc.logpsi(kind, n, nh, th, u) - base), rel=1e-11)
        h = 1e-6
        for k in range(m):
            e = np.zeros(m, np.complex128)
            e[k] = h
            fd = (orc.logpsi(kind, n, nh, th + e, s) - orc.logpsi(kind, n, nh, th - e, s)) / (2 * h)
            assert O[k] == pytest.approx(fd, abs=1e-8)


def test_jastrow_layout(orc):
    # theta = [a_0..a_{N-1}, eta_01, eta_02, ..., eta_{N-2,N-1}] (row-major upper triangle)
    n = 4
    m = orc.n_params(0, n)
    pairs = [(j, k) for j in range(n) for k in range(j + 1, n)]
    s = np.array([1, -1, -1, 1], np.int8)
    for idx, (j, k) in enumerate(pairs):
        th = np.zeros(m, np.complex128)
        th[n + idx] = 0.25 + 0.5j
        assert orc.logpsi(0, n, 0, th, s) == pytest.approx((0.25 + 0.5j) * s[j] * s[k])


def test_zero_parameters_give_plus_x(orc):
    # all-zero parameters: |psi|^2 uniform, i.e. the +x coherent state (text after Eq. 12);
    # for the RBM every configuration has amplitude 2^N' (the product of 2 cosh 0)
    rng = np.random.default_rng(0)
    for kind, n, nh in [(0, 6, 0), (1, 6, 6)]:
        m = orc.n_params(kind, n, nh)
        vals = {orc.logpsi(kind, n, nh, np.zeros(m), rng.choice([-1, 1], size=n).astype(np.int8)) for _ in range(8)}
        assert len({round(v.real, 12) for v in vals}) == 1 and all(v.imag == 0 for v in vals)
