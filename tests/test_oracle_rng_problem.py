"""Pins of the oracle's random-number layer and problem construction.

Philox4x32-10 is pinned to the published known-answer vectors; the conversions are pinned to
their definitions by exhaustive bit checks and by distribution moments; the Kac factor is
pinned to brute-force sums and to the reduction K(0) = N/2 that follows from its definition.
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(orc, row):
    ctr, key, want = row
    assert list(orc.philox(ctr, key)) == want


def test_u53_bit_layout(orc):
    # ((a>>5) * 2^26 + (b>>6)) * 2^-53 uses the top 27 bits of a and the top 26 of b
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == (2.0 ** 53 - 1) / 2.0 ** 53
    assert orc.u53(0x1F, 0x3F) == 0.0
    assert orc.u53(1 << 5, 0) == 2.0 ** 26 / 2.0 ** 53
    assert orc.u53(0, 1 << 6) == 1.0 / 2.0 ** 53


def test_wiener_increments_moments(orc):
    dt = 0.01
    z = np.concatenate([orc.draw_dw(3, t, s, 64, dt) for t in range(20) for s in range(50)]) / np.sqrt(dt)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.15
    # distinct (traj, step) counters give independent streams
    a, b = orc.draw_dw(3, 0, 0, 8, dt), orc.draw_dw(3, 0, 1, 8, dt)
    assert not np.allclose(a, b)
    # odd channel counts keep the first of the Box-Muller pair
    assert np.array_equal(orc.draw_dw(3, 2, 5, 7, dt), orc.draw_dw(3, 2, 5, 8, dt)[:7])


def test_initial_chains_uniform(orc):
    c = orc.init_chains(0, 0, 200, 64).astype(np.float64)
    assert set(np.unique(c)) == {-1.0, 1.0}
    assert abs(c.mean()) < 5 / np.sqrt(c.size)
    # configurations beyond 128 spins come from the next counter block
    assert not np.array_equal(c[:, :72], c[:, 128:200])


def _kac_brute(dist, alpha, n):
    return sum(dist(i, j) ** (-alpha) for i in range(n) for j in range(i + 1, n)) / (n - 1)


@pytest.mark.parametrize("geom,n,alpha", [("obc", 8, 1.5), ("pbc", 10, 1.0), ("obc", 64, 1.5), ("pbc", 7, 2.0)])
def test_couplings_1d(orc, geom, n, alpha):
    J = orc.couplings(geom, n, alpha, 1.0)
    if geom == "obc":
        dist = lambda i, j: abs(i - j)  # noqa: E731
    else:
        dist = lambda i, j: min(abs(i - j), n - abs(i - j))  # noqa: E731
    kac = _kac_brute(dist, alpha, n)
    for i in range(n):
        assert J[i, i] == 0.0
        for j in range(n):
            if i != j:
                assert J[i, j] == pytest.approx(dist(i, j) ** (-alpha) / kac, rel=1e-13)
    assert np.array_equal(J, J.T)
    # Kac normalisation: sum_{i<j} J_ij = (N-1) J, by the definition of K(alpha)
    assert np.sum(np.triu(J, 1)) == pytest.approx(n - 1, rel=1e-13)


def test_couplings_alpha0_is_uniform(orc):
    # alpha = 0: every pair couples with r^0 = 1, so K = N(N-1)/2/(N-1) = N/2 and J_ij = 2/N
    n = 9
    J = orc.couplings("obc", n, 0.0, 1.0)
    off = J[~np.eye(n, dtype=bool)]
    assert np.allclose(off, 2.0 / n, rtol=1e-14)


def test_couplings_2d(orc):
    lx = ly = 4
    J = orc.couplings("2d", lx, 3.0, 1.0, ly=ly)
    n = lx * ly
    pos = [(i % lx, i // lx) for i in range(n)]
    d = lambda i, j: np.hypot(pos[i][0] - pos[j][0], pos[i][1] - pos[j][1])  # noqa: E731
    kac = _kac_brute(d, 3.0, n)
    assert J[0, 1] == pytest.approx(1.0 / kac, rel=1e-13)
    assert J[0, 5] == pytest.approx(2.0 ** -1.5 / kac, rel=1e-13)
    assert J[0, 15] == pytest.approx((18.0 ** -1.5) / kac, rel=1e-13)
