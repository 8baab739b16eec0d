"""SNR-regularised solve on the GPU (parallel Jacobi, one workgroup per trajectory) against the
oracle (cyclic Jacobi).  The two eigen-decompositions order and sign their eigenvectors
differently, so the comparison is on what is unique: the sorted eigenvalues (1e-12 of the
largest: Jacobi is backward stable to a few ulps of ||S||), the SNR of the component with the
same eigenvalue (1e-8 relative), and delta and theta (1e-10 relative: eigenvector rounding
amplified by 1/lam_min with lam_min ~ eps; measured up to 1e-11).  With tau = 0 the solve is the Cholesky one.  M <= 196 runs
the LDS-resident Jacobi, M = 231 (N = 21) the global-memory one; the RBM (kind 1, FP64 S) the
complex Hermitian Jacobi."""
import numpy as np
import pytest
from parity_log import parity

import workloads as wl

pytestmark = pytest.mark.gpu
LJPH = 2


@pytest.fixture(scope="module")
def tv():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    import paper_2506_23928_amd as tv
    from paper_2506_23928_amd import tvmc
    tvmc.lib()
    return tv


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kind,n,d,ns,nc,tau,prec", [(0, 6, 0, 512, 8, 4.0, 0), (0, 7, 0, 320, 16, 4.0, 0),
                                                     (LJPH, 9, 2, 256, 8, 4.0, 1), (0, 6, 0, 256, 8, 0.0, 1),
                                                     (LJPH, 64, 1, 256, 8, 4.0, 1), (0, 21, 0, 256, 8, 4.0, 1),
                                                     (1, 5, 3, 256, 8, 4.0, 0), (1, 6, 6, 320, 8, 0.0, 0),
                                                     (1, 7, 9, 512, 16, 4.0, 0)])
def test_snr_evaluation_parity(tv, orc, kind, n, d, ns, nc, tau, prec):
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=n + 5)
    m = orc.n_params(kind, n, d)
    th0 = wl.random_theta(m, 0.05, seed=2)
    seed, dt, eps, TT = 4, 0.01, 1e-4, 2
    cfg = tv.make_config(TT, ns, nc, dt, eps, precision=prec, seed=seed, traj_offset=1, regulariser=T.REG_SNR,
                         snr_tau=tau)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=kind, n_hidden=d, theta0=th0)
    ctx.sample()
    ctx.estimate()
    ctx.sr_solve()
    ctx.synchronize()
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, dt=dt, diag_shift=eps, seed=seed, regulariser=orc.REG_SNR,
                       snr_tau=tau)
    cfg_c = orc.Config(n_samples=ns, n_chains=nc, dt=dt, diag_shift=eps, seed=seed)
    pb = orc.Problem(J, hx, jumps)
    for t in range(TT):
        chains = orc.init_chains(seed, 1 + t, n, nc)
        dw = orc.draw_dw(seed, 1 + t, 0, len(jumps), dt)
        r = orc.evaluate(pb, kind, d, cfg_o, th0, chains.copy(), traj=1 + t, first=True, dw=dw)
        assert r["status"] == 0
        assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), r["samples"])
        eg = ctx.get(T.Q_EIG, t)
        go, oo = np.argsort(eg[:, 0]), np.argsort(r["eig"][:, 0])
        lmax = r["eig"][:, 0].max()
        assert np.abs(eg[go, 0] - r["eig"][oo, 0]).max() < 1e-12 * lmax
        gap = np.diff(r["eig"][oo, 0])
        ok = np.ones(m, bool)            # SNR of well-separated eigenvalues only
        ok[1:] &= gap > 1e-6 * lmax
        ok[:-1] &= gap > 1e-6 * lmax
        assert _rel(eg[go, 1][ok], r["eig"][oo, 1][ok]) < 1e-8
        parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, t), r["delta"]), 1e-10)
        if tau == 0.0:
            rc = orc.evaluate(pb, kind, d, cfg_c, th0, chains.copy(), traj=1 + t, first=True, dw=dw)
            parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, t), rc["delta"]), 1e-10)


def test_snr_trajectory_parity(tv, orc):
    """10 Heun steps of an N = 6 Jastrow chain with the SNR solve (tau = 4, eps = 0), moments
    every 5 steps: theta and moments against the oracle's trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, TT, steps = 6, 512, 8, 3, 10
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    m = orc.n_params(0, n)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.01, diag_shift=0.0, seed=6, n_steps=steps,
                       obs_every=5, regulariser=orc.REG_SNR, snr_tau=4.0)
    th_o, obs_o, st = orc.run(orc.Problem(J, 0.8, jumps), 0, 0, cfg_o, np.zeros(m), TT, n_threads=3)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, 0.01, 0.0, 2, 1, 0, tv.HEUN, tv.PREC_MFMA, 5, 3, 6, regulariser=T.REG_SNR,
                         snr_tau=4.0)
    ctx = tv.Context(tv.Problem(J, 0.8, jumps), cfg)
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, 2]).max() < 1e-9


def test_snr_with_the_linear_sse(tv, orc):
    """The SNR solve on the linear unravelling (G without the <L + L^dag> drive): theta and
    log Q after 6 midpoint steps against the oracle."""
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, TT, steps = 6, 512, 8, 2, 6
    J, hx, jumps = wl.random_problem(n, seed=3)
    m = orc.n_params(0, n)
    th0 = wl.random_theta(m, 0.05, seed=8)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.01, diag_shift=1e-4, seed=9, n_steps=steps,
                       obs_every=steps, scheme=1, linear=True, regulariser=orc.REG_SNR, snr_tau=4.0)
    th_o, _, st = orc.run(orc.Problem(J, hx, jumps), 0, 0, cfg_o, th0, TT, n_threads=2)
    assert st == 0
    lq = orc.run.last_lognorm
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-4, 2, 1, 0, tv.MIDPOINT, tv.PREC_MFMA, steps, 2, 9,
                         unravelling=T.SSE_LINEAR, regulariser=T.REG_SNR, snr_tau=4.0)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, theta0=th0)
    ctx.sde_step(steps)
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        assert abs(ctx.get(T.Q_LOGNORM, t)[0] - lq[t, 1]) < 1e-9


def test_snr_rbm_trajectory_parity(tv, orc):
    """6 Heun steps of an N = 5 RBM (N' = 4) with the Hermitian SNR solve and FP64 S against the
    oracle's trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    n, nh, ns, nc, TT, steps = 5, 4, 512, 8, 2, 6
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.05, seed=12)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.01, diag_shift=1e-4, seed=4, n_steps=steps,
                       regulariser=orc.REG_SNR, snr_tau=4.0)
    th_o, _, st = orc.run(orc.Problem(J, 0.7, jumps), 1, nh, cfg_o, th0, TT, n_threads=2)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-4, 2, 1, 0, tv.HEUN, tv.PREC_FP64, 0, 0, 4, regulariser=T.REG_SNR,
                         snr_tau=4.0)
    ctx = tv.Context(tv.Problem(J, 0.7, jumps), cfg, kind=T.RBM, n_hidden=nh, theta0=th0)
    ctx.sde_step(steps)
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
