"""Pins of the oracle's sample-space solve (want_solve = 3).

* push-through identity: (A^H A + eps I)^-1 A^H = A^H (A A^H + eps I)^-1, so the sample-space
  increment equals the parameter-space one on the same samples, for M above and below N_s and
  both ansaetze;
* the sample-space kernel T against closed forms derived independently of the log-derivative
  sums: for the Jastrow ansatz sum_k O_k(x) O_k(y) = q + (q^2 - N) / 2 with q = s(x).s(y); for
  the RBM sum_k O_k(x) O_k(y)^* = (1 + q)(1 + g) - 1 with g = sum_j tanh(g_j(x)) tanh(g_j(y))^*;
  centring is H K H / N_s with H = I - 11^T / N_s.
"""
import numpy as np
import pytest

import workloads as wl


def _eval(orc, kind, nh, n, ns, nc, want, seed=3, eps=1e-3):
    J, hx, jumps = wl.random_problem(n, seed=20 + n)
    m = orc.n_params(kind, n, nh)
    th = wl.random_theta(m, 0.15, seed=7 + nh)
    pb = orc.Problem(J, hx, jumps)
    cfg = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=3, thin_sweeps=1, dt=0.01, diag_shift=eps, seed=seed)
    chains = orc.init_chains(seed, 0, n, nc)
    dw = orc.draw_dw(seed, 0, 0, len(jumps), 0.01)
    r = orc.evaluate(pb, kind, nh, cfg, th, chains, traj=0, first=True, dw=dw, want_solve=want, want_moments=False)
    assert r["status"] == 0
    return r, th


@pytest.mark.parametrize("kind,n,nh,ns,nc", [(0, 7, 0, 16, 4), (0, 6, 0, 64, 8), (1, 4, 5, 16, 4), (1, 5, 3, 64, 8)])
def test_push_through_matches_parameter_space(orc, kind, n, nh, ns, nc):
    r1, _ = _eval(orc, kind, nh, n, ns, nc, want=1)
    r3, _ = _eval(orc, kind, nh, n, ns, nc, want=3)
    assert np.array_equal(r1["samples"], r3["samples"])
    assert np.abs(r1["D"] - r3["D"]).max() == 0.0
    d1, d3 = r1["delta"], r3["delta"]
    assert np.abs(d1 - d3).max() < 1e-10 * np.abs(d1).max()


def _centre(K):
    ns = K.shape[0]
    H = np.eye(ns) - np.ones((ns, ns)) / ns
    return H @ K @ H / ns


def test_sample_space_kernel_jastrow_closed_form(orc):
    n, ns = 7, 32
    r, _ = _eval(orc, 0, 0, n, ns, 4, want=3)
    s = r["samples"].astype(np.float64)
    q = s @ s.T
    K = q + (q * q - n) / 2.0
    T = _centre(K)
    assert np.abs(r["S"] - T).max() < 1e-13 * np.abs(T).max()


def test_sample_space_kernel_rbm_closed_form(orc):
    n, nh, ns = 5, 4, 32
    r, th = _eval(orc, 1, nh, n, ns, 4, want=3)
    s = r["samples"].astype(np.float64)
    b, w = th[n:n + nh], th[n + nh:].reshape(n, nh)
    t = np.tanh(b[None, :] + s @ w)
    q = s @ s.T
    g = t @ t.conj().T
    K = (1.0 + q) * (1.0 + g) - 1.0
    T = _centre(K)
    assert np.abs(r["S"] - T).max() < 1e-13 * np.abs(T).max()
