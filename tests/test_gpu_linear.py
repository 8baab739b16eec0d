"""Linear SSE (App. B) on the GPU against the oracle, element by element.

The same bars as the nonlinear path: samples bit-exact, D to 1e-12 relative, theta to 1e-10
relative after several steps; log Q is a sum of 2 Re <G> increments, each as exact as D's
mean, so its history is held to 1e-10 absolute; the weighted ensemble to 1e-10.
"""
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


def _run_pair(tv, orc, kind, nh, J, hx, jumps, th0, TT, ns, nc, dt, eps, seed, steps, every, scheme, init=0,
              solver=0, tol=1e-10, otol=1e-10):
    from paper_2506_23928_amd import tvmc as T
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, init_sweeps=init, dt=dt, diag_shift=eps, seed=seed,
                       n_steps=steps, obs_every=every, scheme=scheme, linear=True)
    th_o, obs_o, st = orc.run(orc.Problem(J, hx, jumps), kind, nh, cfg_o, th0, TT, n_threads=4)
    assert st == 0
    lq_o = orc.run.last_lognorm.copy()
    nobs = steps // every + 1
    cfg = tv.make_config(TT, ns, nc, dt, eps, 2, 1, init, scheme, tv.PREC_FP64, every, nobs, seed, solver=solver,
                         unravelling=T.SSE_LINEAR)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=kind, n_hidden=nh, theta0=th0)
    ctx.sde_step(steps)
    ctx.sample()                      # final observation pass, as the oracle's driver does
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), tol)
        assert np.abs(ctx.get(T.Q_OBS_HIST, t)[:nobs - 1] - obs_o[t, :nobs - 1]).max() < otol
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, nobs - 1]).max() < otol
        lh = ctx.get(T.Q_LOGNORM_HIST, t)
        assert np.abs(lh[:nobs - 1] - lq_o[t, :nobs - 1]).max() < otol, (t, lh, lq_o[t])
        assert abs(ctx.get(T.Q_LOGNORM, t)[0] - lq_o[t, nobs - 1]) < otol
    assert np.abs(lq_o[:, -1]).max() > 1e-3           # the norms really moved
    # App. B's weighted average of the last moments against the oracle's
    Mg, Cg, x2g = ctx.ensemble()
    M, C, x2 = orc.ensemble(obs_o[:, nobs - 1], J.shape[0], weights=np.exp(lq_o[:, nobs - 1]))
    assert np.abs(Mg - M).max() < 10 * otol
    assert np.abs(Cg - C).max() < 10 * otol
    # xi^2 = N lambda_min / |M|^2 amplifies C's and M's errors by N / |M|^2
    assert abs(x2g - x2) < 10 * otol * J.shape[0] * (1.0 + abs(x2)) / np.dot(M, M), (x2g, x2)
    return ctx, th_o, lq_o


@pytest.mark.parametrize("scheme", [0, 1])
def test_linear_jastrow_trajectory_parity(tv, orc, scheme):
    """12 steps of a random N = 6 problem with sigma^-, sigma^+ and sigma^z channels (the
    sigma^z channels' L^2 = rate * 1 term moves only log Q), 3 trajectories."""
    n = 6
    J, hx, jumps = wl.random_problem(n, seed=11)
    m = orc.n_params(0, n)
    th0 = wl.random_theta(m, 0.1, seed=3)
    _run_pair(tv, orc, 0, 0, J, hx, jumps, th0, 3, 512, 8, 0.02, 1e-4, 5, 12, 6, scheme)


def test_linear_rbm_trajectory_parity(tv, orc):
    n, nh = 5, 3
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.2) for i in range(n)] + [(2, i, 0.1) for i in range(n)]
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.05, seed=7)
    _run_pair(tv, orc, 1, nh, J, 1.0, jumps, th0, 3, 256, 8, 0.01, 1e-4, 2, 8, 4, 0, init=5)


def test_linear_sample_space_parity(tv, orc):
    """The linear drive reaches the sample-space solve through the same G: an N = 8 Jastrow
    chain, M = 36 > N_s = 32, against the oracle's parameter-space driver (the push-through
    identity reorders the rounding, hence 1e-8 for the moments; theta stays within 1e-10)."""
    from paper_2506_23928_amd import tvmc as T
    n = 8
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)] + [(2, i, 0.05) for i in range(n)]
    ctx, _, _ = _run_pair(tv, orc, 0, 0, J, 1.0, jumps, np.zeros(orc.n_params(0, n)), 3, 32, 8, 0.01, 1e-3, 8,
                          8, 4, 0, solver=T.SOLVER_SAMPLE_SPACE, tol=1e-10, otol=1e-8)
    assert ctx.sample_space


def test_nonlinear_keeps_log_norm_zero_and_plain_average(tv, orc):
    from paper_2506_23928_amd import tvmc as T
    n = 6
    J, hx, jumps = wl.random_problem(n, seed=11)
    cfg = tv.make_config(2, 256, 8, 0.02, 1e-4, obs_every=2, n_obs_max=3, seed=5)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg)
    ctx.sde_step(4)
    ctx.sample()
    mom = ctx.observables()
    Mg, Cg, x2g = ctx.ensemble()
    for t in range(2):
        assert ctx.get(T.Q_LOGNORM, t)[0] == 0.0
        assert np.all(ctx.get(T.Q_LOGNORM_HIST, t) == 0.0)
    M, C, x2 = orc.ensemble(mom, n)
    assert np.abs(Mg - M).max() < 1e-12 and np.abs(Cg - C).max() < 1e-12
    assert abs(x2g - x2) < 1e-12 * n * (1.0 + abs(x2)) / np.dot(M, M), (x2g, x2)


def test_linear_ljph_trajectory_parity(tv, orc):
    """The linear SSE with the LJPH1 ansatz (shared-distance log-derivatives in D), Heun."""
    n, d = 8, 1
    J = orc.couplings("pbc", n, 1.0, 1.0)
    jumps = [(0, i, 0.15) for i in range(n)] + [(2, i, 0.05) for i in range(n)]
    m = orc.n_params(2, n, d)
    th0 = wl.random_theta(m, 0.05, seed=4)
    _run_pair(tv, orc, 2, d, J, 0.4, jumps, th0, 3, 512, 8, 0.01, 1e-4, 7, 8, 4, 0)


def test_ensemble_at_and_leave_one_out_match_oracle(orc):
    """tvmc_ensemble_at at every history record and at the last moments, and its jackknife (the
    leave-one-out xi^2 of every trajectory, formed on the GPU), against the oracle's ensemble of
    the same per-trajectory moments, with and without each trajectory in turn (1e-12)."""
    import torch
    assert torch.cuda.is_available()
    import paper_2506_23928_amd as tv
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, TT, steps, every = 6, 256, 8, 7, 6, 2
    J, hx, jumps = wl.random_problem(n, seed=21)
    nobs = steps // every
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-4, 2, 1, 0, tv.HEUN, tv.PREC_FP64, every, nobs + 1, 5)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg)
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    hist = np.stack([ctx.get(T.Q_OBS_HIST, t) for t in range(TT)])
    final = np.stack([ctx.get(T.Q_MOMENTS, t) for t in range(TT)])
    for slot, mom in [(k, hist[:, k]) for k in range(nobs)] + [(-1, final)]:
        M, C, x2, loo = ctx.ensemble_at(slot, jackknife=True)
        Mo, Co, xo = orc.ensemble(mom, n)
        assert np.abs(M - Mo).max() < 1e-12 and np.abs(C - Co).max() < 1e-12 and abs(x2 - xo) < 1e-12, slot
        want = np.array([orc.ensemble(np.delete(mom, d, axis=0), n)[2] for d in range(TT)])
        assert np.abs(loo - want).max() < 1e-12, (slot, loo, want)
