"""Uneven batches on the GPU (one context per system size, one problem per trajectory, each
size on its own stream) against the oracle run trajectory by trajectory.  Tolerances as in the
other parity tests: samples bit-exact, D 1e-12 relative, theta 1e-9 relative."""
import numpy as np
import pytest

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


def _problems(tv, orc, params, h):
    from paper_2506_23928_amd.problem import litf_problem
    gpu = [litf_problem(n, a, h, g) for n, a, g in params]
    ref = [orc.Problem(orc.couplings("obc", n, a, 1.0), h, [(0, i, g) for i in range(n)]) for n, a, g in params]
    return gpu, ref


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_trajectories_match_oracle(tv, orc, precision):
    """Nine trajectories with N in {4, 6, 8}, alpha and gamma drawn per trajectory, 12 Heun
    steps: every trajectory's theta against the oracle's driver with that trajectory's problem
    and random-number index."""
    from paper_2506_23928_amd.uneven import UnevenBatch
    from paper_2506_23928_amd import tvmc as T
    w = dict(wl.UNEVEN, sizes=(4, 6, 8))
    params = wl.uneven_params(9, seed=3, w=w)
    assert len({p[0] for p in params}) == 3
    gpu, ref = _problems(tv, orc, params, w["h"])
    ns, nc, dt, eps, seed, steps = 256, 8, 0.01, 1e-4, 2, 12
    ub = UnevenBatch(gpu, n_samples=ns, n_chains=nc, dt=dt, diag_shift=eps, seed=seed, precision=precision)
    ub.sde_step(steps)
    ub.synchronize()
    cfg = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, thin_sweeps=1, dt=dt, diag_shift=eps, seed=seed)
    cfg.n_steps = steps
    for i, (n, a, g) in enumerate(params):
        m = orc.n_params(0, n)
        th, _, st = orc.run(ref[i], 0, 0, cfg, np.zeros(m), 1, traj0=int(ub.rank[i]))
        assert st == 0
        assert _rel(ub.theta(i), th[0]) < 1e-9, (i, n)
    # every group has its own stream
    assert len({id(g[2].stream) for g in ub.groups}) == len(ub.groups)
    assert ub.get(T.Q_THETA, 0).shape == (orc.n_params(0, params[0][0]),)


def test_uneven_full_size_launch(tv, orc):
    """The 512-trajectory uneven batch (N in {16, 24, 32, 48, 64}, 2048 samples) in the
    benchmark's launch configuration: the first and last trajectory of each size against the
    oracle (samples, <B^n>, D) and the solve against its defining residual."""
    from paper_2506_23928_amd.uneven import UnevenBatch
    from paper_2506_23928_amd import tvmc as T
    w = wl.UNEVEN
    params = wl.uneven_params(w["n_traj"], seed=w["seed"])
    gpu, ref = _problems(tv, orc, params, w["h"])
    ub = UnevenBatch(gpu, n_samples=w["n_samples"], n_chains=w["n_chains"], dt=w["dt"], diag_shift=w["diag_shift"],
                     seed=w["seed"], precision=1)
    for _, _, ctx in ub.groups:
        ctx.sample()
        ctx.estimate()
    cfg = orc.Config(n_samples=w["n_samples"], n_chains=w["n_chains"], burn_sweeps=2, thin_sweeps=1, dt=w["dt"],
                     diag_shift=w["diag_shift"], seed=w["seed"])
    checked = []
    for n, members, ctx in ub.groups:
        for loc in (0, len(members) - 1):
            i = int(members[loc])
            traj = int(ub.rank[i])
            m = orc.n_params(0, n)
            chains = orc.init_chains(w["seed"], traj, n, w["n_chains"])
            dw = orc.draw_dw(w["seed"], traj, 0, n, w["dt"])
            r = orc.evaluate(ref[i], 0, 0, cfg, np.zeros(m), chains, traj=traj, first=True, dw=dw, want_solve=2,
                             want_moments=False)
            smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, loc), n)
            assert np.array_equal(smp, r["samples"]), (n, i)
            assert _rel(ctx.get(T.Q_BMEAN, loc), r["bmean"]) < 1e-13
            assert _rel(ctx.get(T.Q_D, loc), r["D"]) < 1e-12
            checked.append((n, loc, r["samples"], ctx.get(T.Q_D, loc)))
    for _, _, ctx in ub.groups:
        ctx.sr_solve()
    ub.synchronize()
    # the increment against the parameter-space normal equations A^T (A delta) + eps delta = D,
    # A = (O - <O>) / sqrt(N_s) from the oracle's samples (the N = 64 group, M = 2080 > 2048
    # samples, solves in sample space)
    for n, loc, smp, D in checked:
        ctx = [g[2] for g in ub.groups if g[0] == n][0]
        assert ctx.sample_space == (n == 64)
        d = ctx.get(T.Q_DELTA0, loc)
        s = smp.astype(np.float64)
        iu = np.triu_indices(n, 1)
        O = np.concatenate([s, s[:, iu[0]] * s[:, iu[1]]], axis=1)
        A = (O - O.mean(0)) / np.sqrt(O.shape[0])
        res = A.T @ (A @ d) + w["diag_shift"] * d - D
        assert np.abs(res).max() < 1e-9 * np.abs(D).max(), n
    assert sorted({c[0] for c in checked}) == list(w["sizes"])


def test_uneven_graph_replay_is_the_eager_run(tv, orc):
    """Each group's plain steps replayed from its captured HIP graph (every group on its own
    stream) give the eager run's theta bit for bit, with a tuned sampler workgroup shape."""
    from paper_2506_23928_amd.uneven import UnevenBatch
    w = dict(wl.UNEVEN, sizes=(8, 16, 24))
    params = wl.uneven_params(12, seed=5, w=w)
    gpu, _ = _problems(tv, orc, params, w["h"])
    conf = dict(n_samples=512, n_chains=16, dt=0.01, diag_shift=1e-4, seed=4, precision=1)
    eager = UnevenBatch(gpu, **conf)
    graph = UnevenBatch(gpu, use_graph=1, sampler_chains=4, **conf)
    for ub in (eager, graph):
        ub.sde_step(5)
        ub.synchronize()
    for i in range(len(params)):
        assert np.array_equal(eager.theta(i), graph.theta(i)), i
