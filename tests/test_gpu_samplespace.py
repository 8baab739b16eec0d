"""The sample-space solve (M > N_s) on the GPU against the oracle.

Tolerances: T + eps I 1e-13 of its scale for the Jastrow ansatz (integer kernel, centring by
separately rounded operations on both sides) and 1e-12 for the RBM (tanh rows, different
summation order); increments 1e-10 against the oracle's sample-space solve and against
its parameter-space solve (the push-through identity holds exactly; the two solves round
differently, amplified by cond(T + eps I))."""
import numpy as np
import pytest
from parity_log import parity

import workloads as wl

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("kind,n,nh,ns,nc", [(0, 8, 0, 32, 8), (1, 6, 40, 200, 8), (1, 5, 7, 40, 4)])
def test_sample_space_evaluation(tv, orc, kind, n, nh, ns, nc):
    """One predictor evaluation per trajectory: T + eps I and the increment against the
    oracle's sample-space solve, and the increment against its parameter-space solve;
    N_s = 200 leaves a ragged 64-row tile in the RBM kernel."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=70 + n)
    m = orc.n_params(kind, n, nh)
    assert m > ns
    th0 = wl.random_theta(m, 0.1, seed=3 + nh)
    seed, dt, eps, TT = 6, 0.01, 1e-3, 2
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, thin_sweeps=1, dt=dt, diag_shift=eps, seed=seed)
    pb = orc.Problem(J, hx, jumps)
    cfg = tv.make_config(TT, ns, nc, dt, eps, seed=seed, traj_offset=5)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=kind, n_hidden=nh, theta0=th0)
    assert ctx.sample_space and ctx.solve_dim == ns
    ctx.sample()
    ctx.estimate()
    Ts = [ctx.get(T.Q_S, t) for t in range(TT)]
    ctx.sr_solve()
    ctx.synchronize()
    low = np.tril_indices(ns)
    for t in range(TT):
        traj = 5 + t
        dw = orc.draw_dw(seed, traj, 0, len(jumps), dt)
        r3 = orc.evaluate(pb, kind, nh, cfg_o, th0, orc.init_chains(seed, traj, n, nc), traj=traj, dw=dw,
                          want_solve=3, want_moments=False)
        r1 = orc.evaluate(pb, kind, nh, cfg_o, th0, orc.init_chains(seed, traj, n, nc), traj=traj, dw=dw,
                          want_solve=1, want_moments=False)
        assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), r3["samples"])
        want = r3["S"] + eps * np.eye(ns)
        tol = 1e-13 if kind == 0 else 1e-12
        assert np.abs(Ts[t][low] - want[low]).max() < tol * np.abs(want).max()
        d = ctx.get(T.Q_DELTA0, t)
        parity("delta_vs_oracle_sample_space", _rel(d, r3["delta"]), 1e-10)
        parity("delta_vs_oracle_param_space", _rel(d, r1["delta"]), 1e-10)


def test_sample_space_trajectory(tv, orc):
    """12 Heun steps of an N = 8 Jastrow chain with 32 samples (M = 36 > N_s) in sample space
    against the oracle's parameter-space trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, TT, steps = 8, 32, 8, 3, 12
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.01, diag_shift=1e-3, seed=8, n_steps=steps)
    th_o, _, st = orc.run(orc.Problem(J, 1.0, jumps), 0, 0, cfg_o, np.zeros(orc.n_params(0, n)), TT, n_threads=3)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-3, seed=8, solver=tv.tvmc.SOLVER_SAMPLE_SPACE)
    ctx = tv.Context(tv.Problem(J, 1.0, jumps), cfg)
    ctx.sde_step(steps)
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)


@pytest.mark.parametrize("name", ["chain64_rbm_wide", "lattice8x8_rbm_ss"])
def test_sample_space_full_size(tv, orc, name):
    """The wide RBM workloads (chain N = 64, N' = 256, M = 16704; 8x8 lattice, alpha = 3,
    N' = 128, M = 8384; 4096 samples, 32 trajectories) in the benchmark's launch configuration: for the last trajectory the samples bit for bit
    against the oracle, T against the closed form (1 + q)(1 + g) - 1 centred, built from the
    oracle's samples, and the increment against the parameter-space normal equations
    A^H (A delta) + eps delta = D with A = (O - <O>) / sqrt(N_s) from the oracle's
    log-derivatives (S itself, 16704^2, is never formed)."""
    from paper_2506_23928_amd import tvmc as T
    import bench
    w = dict(wl.WORKLOADS[name])
    ctx = bench.build_context(tv, w, tv.PREC_FP64)
    n, nh, ns, TT = w["n"], w["n_hidden"], w["n_samples"], w["n_traj"]
    m = orc.n_params(1, n, nh)
    assert ctx.sample_space
    ctx.sample()
    ctx.estimate()
    t = TT - 1
    Tg = ctx.get(T.Q_S, t)
    ctx.sr_solve()
    ctx.synchronize()
    th0 = wl.rbm_theta0(n, nh, w["w_scale"], w["seed"])
    lx, ly = wl.lattice(w)
    pb = orc.Problem(orc.couplings(w["geom"], lx, w["alpha"], w["jscale"], ly), w["h"], wl.jumps(w))
    cfg_o = orc.Config(n_samples=ns, n_chains=w["n_chains"], burn_sweeps=w["burn_sweeps"],
                       thin_sweeps=w["thin_sweeps"], dt=w["dt"], diag_shift=w["diag_shift"], seed=w["seed"])
    r = orc.evaluate(pb, 1, nh, cfg_o, th0, orc.init_chains(w["seed"], t, n, w["n_chains"]), traj=t,
                     first=True, want_solve=0, want_moments=False)
    smp = r["samples"]
    assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), smp)
    s = smp.astype(np.float64)
    b, wm = th0[n:n + nh], th0[n + nh:].reshape(n, nh)
    tt = np.tanh(b[None, :] + s @ wm)
    q = s @ s.T
    K = (1.0 + q) * (1.0 + tt @ tt.conj().T) - 1.0
    H = np.eye(ns) - 1.0 / ns
    Tc = H @ K @ H / ns + w["diag_shift"] * np.eye(ns)
    low = np.tril_indices(ns)
    assert np.abs(Tg[low] - Tc[low]).max() < 1e-12 * np.abs(Tc).max()
    del K, H, Tc, Tg
    O = np.empty((ns, m), np.complex128)
    for x in range(ns):
        O[x] = orc.local_quantities(1, n, nh, th0, smp[x], two_flip=False)[2]
    A = (O - O.mean(0)) / np.sqrt(ns)
    del O
    d = ctx.get(T.Q_DELTA0, t)
    D = ctx.get(T.Q_D, t)
    res = A.conj().T @ (A @ d) + w["diag_shift"] * d - D
    assert np.abs(res).max() < 1e-8 * np.abs(D).max()
