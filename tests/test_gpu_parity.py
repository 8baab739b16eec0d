"""GPU path (libtvmc through its C ABI) against the oracle, element by element.

Tolerances, derived in the design notes from the arithmetic:
  * samples, chain states, accept counts: bit-exact (same Philox stream, same accept rule;
    fields are sums of exact +-eta terms, so only an ulp-level tie of log(u) against the
    flip log-ratio could differ);
  * S + eps I (Jastrow): bit-exact (integer sums of +-1 divided by a power of two);
  * <O_k>: bit-exact;
  * local energies, <B^n>, dW: relative 1e-13 (exp/sincos/log ulps and summation order);
  * D: 1e-12 relative to max|D| (different but equally exact summation of the covariance);
  * delta, theta: 1e-10 relative to max|.| (D's rounding amplified by cond(S + eps I); the
    measured errors are 2e-15 - 3e-11).
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
    tvmc.lib()   # raises if the library was not built
    return tv


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _pair(tv, orc, J, hx, jumps, T, ns, nc, dt, eps, seed, precision=0, burn=2, thin=1, init=0, scheme=0, traj0=0,
          theta0=None, obs_every=0, nobs=0, solver=0):
    pb_o = orc.Problem(J, hx, jumps)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=burn, thin_sweeps=thin, init_sweeps=init, dt=dt,
                       diag_shift=eps, scheme=scheme, seed=seed, obs_every=obs_every)
    cfg_g = tv.make_config(T, ns, nc, dt, eps, burn, thin, init, scheme, precision, obs_every, nobs, seed, traj0,
                           solver=solver)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg_g, theta0=theta0)
    return pb_o, cfg_o, ctx


def _check_eval(tv, ctx, t, r, n, eps, tag):
    from paper_2506_23928_amd import tvmc as T
    smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n)
    assert np.array_equal(smp, r["samples"]), "%s: samples differ (traj %d)" % (tag, t)
    assert np.array_equal(ctx.get(T.Q_ACCEPTS, t).astype(np.int64), r["accepts"]), tag
    assert _rel(ctx.get(T.Q_ELOC, t), r["eloc"]) < 1e-13, tag


def test_stage_by_stage_parity(tv, orc):
    """One full Heun step, every intermediate of both stages, three trajectories, a random
    problem with sigma^-, sigma^+ and sigma^z channels and random initial parameters."""
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, dt, eps, seed, TT = 6, 512, 8, 0.02, 1e-4, 5, 3
    J, hx, jumps = wl.random_problem(n, seed=11)
    m = orc.n_params(0, n)
    th0 = wl.random_theta(m, 0.1, seed=3)
    pb, cfg, ctx = _pair(tv, orc, J, hx, jumps, TT, ns, nc, dt, eps, seed, theta0=th0, traj0=7)
    ctx.sample()
    ctx.estimate()
    ctx.sr_solve()
    ctx.update()
    res = {}
    for t in range(TT):
        traj = 7 + t
        chains = orc.init_chains(seed, traj, n, nc)
        dw = orc.draw_dw(seed, traj, 0, len(jumps), dt)
        r0 = orc.evaluate(pb, 0, 0, cfg, th0, chains, traj=traj, step=0, stage=0, first=True, dw=dw)
        assert r0["status"] == 0
        res[t] = (chains, dw, r0)
        assert _rel(ctx.get(T.Q_DW, t), dw) < 1e-13
        assert np.array_equal(ctx.get(T.Q_OBAR, t), r0["obar"].real)
        assert _rel(ctx.get(T.Q_BMEAN, t), r0["bmean"]) < 1e-13
        assert _rel(ctx.get(T.Q_D, t), r0["D"]) < 1e-12
        parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, t), r0["delta"]), 1e-10)
        assert _rel(ctx.get(T.Q_THETA_EVAL, t), th0 + r0["delta"]) < 1e-12
    # predictor samples are overwritten by the corrector: re-run the predictor on a second context
    pb2, cfg2, ctx2 = _pair(tv, orc, J, hx, jumps, TT, ns, nc, dt, eps, seed, theta0=th0, traj0=7)
    ctx2.sample()
    ctx2.estimate()
    for t in range(TT):
        _check_eval(tv, ctx2, t, res[t][2], n, eps, "predictor")
        S = ctx2.get(T.Q_S, t)
        want = res[t][2]["S"].real + eps * np.eye(m)
        low = np.tril_indices(m)
        assert np.array_equal(S[low], want[low]), "S + eps I differs"
    # corrector
    ctx.sample()
    ctx.estimate()
    for t in range(TT):
        chains, dw, r0 = res[t]
        th_e = th0 + r0["delta"]
        r1 = orc.evaluate(pb, 0, 0, cfg, th_e, chains, traj=7 + t, step=0, stage=1, first=False, dw=dw)
        _check_eval(tv, ctx, t, r1, n, eps, "corrector")
        assert np.array_equal(ctx.get(T.Q_CHAINS, t), _pack(chains))
        assert _rel(ctx.get(T.Q_D, t), r1["D"]) < 1e-12
        res[t] = (chains, dw, r0, r1)
    ctx.sr_solve()
    ctx.update()
    assert ctx.position() == (1, 0)
    for t in range(TT):
        _, _, r0, r1 = res[t]
        parity("Q_DELTA1", _rel(ctx.get(T.Q_DELTA1, t), r1["delta"]), 1e-10)
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th0 + 0.5 * (r0["delta"] + r1["delta"])), 1e-11)
    ctx.synchronize()


def _pack(chains):
    c = np.asarray(chains)
    bits = (c > 0).astype(np.uint64)
    return (bits << np.arange(c.shape[1], dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint64)


@pytest.mark.parametrize("scheme", [0, 1])
def test_trajectory_parity_chain8(tv, orc, scheme):
    """20 Heun (or midpoint) steps of the N = 8 chain workload, 4 trajectories, moments every
    10 steps: theta and the moment history against the oracle's trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    w = wl.WORKLOADS["chain8_fp64"]
    J = orc.couplings(w["geom"], w["n"], w["alpha"], w["jscale"])
    jumps = wl.jumps(w)
    steps, TT = 20, 4
    m = orc.n_params(0, w["n"])
    pb, cfg, ctx = _pair(tv, orc, J, w["h"], jumps, TT, w["n_samples"], w["n_chains"], w["dt"], w["diag_shift"],
                         w["seed"], scheme=scheme, obs_every=10, nobs=3)
    cfg.n_steps, cfg.obs_every = steps, 10
    th_o, obs_o, st = orc.run(pb, 0, 0, cfg, np.zeros(m), TT, n_threads=4)
    assert st == 0
    ctx.sde_step(steps)
    ctx.sample()                     # final observation pass, as the oracle's driver does
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        hist = ctx.get(T.Q_OBS_HIST, t)
        assert np.abs(hist[:2] - obs_o[t, :2]).max() < 1e-10
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, 2]).max() < 1e-10


def test_closed_system_closed_form_on_gpu(tv, orc):
    """No jumps, h = 0, eps = 0: eta(t) = -i J t exactly on any sample set (the local energy is
    linear in the pair log-derivatives), checked on the GPU path alone."""
    from paper_2506_23928_amd import tvmc as T
    n = 7
    J = orc.couplings("obc", n, 1.5, 1.0)
    cfg = tv.make_config(3, 512, 8, 0.01, 0.0, seed=4)
    ctx = tv.Context(tv.Problem(J, 0.0, []), cfg)
    ctx.sde_step(10)
    ctx.synchronize()
    m = orc.n_params(0, n)
    want = np.zeros(m, np.complex128)
    want[n:] = -1j * 0.1 * np.array([J[j, k] for j in range(n) for k in range(j + 1, n)])
    for t in range(3):
        assert np.abs(ctx.get(T.Q_THETA, t) - want).max() < 1e-12


@pytest.mark.parametrize("n,ns,nc", [(1, 256, 4), (2, 192, 3), (13, 1024, 16), (64, 256, 8), (33, 320, 2)])
def test_edge_shapes(tv, orc, n, ns, nc):
    """N = 1 (a single parameter), odd chain counts, ragged tiles (M = 91, 528), a full 64-bit
    word (N = 64, M = 2080) and sample counts that are not multiples of 256: one predictor
    evaluation against the oracle, MFMA and FP64 S-builds against each other, the one- and
    several-workgroup solvers each against the oracle."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=n) if n > 1 else (np.zeros((1, 1)), 0.7, [(0, 0, 0.2)])
    m = orc.n_params(0, n)
    th0 = wl.random_theta(m, 0.05, seed=n)
    seed, dt, eps = 9, 0.01, 1e-3
    S_by_prec = []
    for prec, solver in ([(0, 1), (1, 2)] if ns % 64 == 0 else [(0, 1), (0, 2)]):
        pb, cfg, ctx = _pair(tv, orc, J, hx, jumps, 2, ns, nc, dt, eps, seed, precision=prec, theta0=th0,
                             solver=solver)
        ctx.sample()
        ctx.estimate()
        S_by_prec.append(ctx.get(T.Q_S, 1))
        ctx.sr_solve()
        ctx.synchronize()
        chains = orc.init_chains(seed, 1, n, nc)
        dw = orc.draw_dw(seed, 1, 0, len(jumps), dt)
        r = orc.evaluate(pb, 0, 0, cfg, th0, chains, traj=1, first=True, dw=dw)
        _check_eval(tv, ctx, 1, r, n, eps, "edge")
        low = np.tril_indices(m)
        assert np.array_equal(S_by_prec[-1][low], (r["S"].real + eps * np.eye(m))[low])
        assert _rel(ctx.get(T.Q_D, 1), r["D"]) < 1e-12
        parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, 1), r["delta"]), 1e-10)
    low = np.tril_indices(m)
    assert np.array_equal(S_by_prec[0][low], S_by_prec[1][low])


def test_bad_arguments_are_rejected(tv):
    from paper_2506_23928_amd import tvmc as T
    J = np.zeros((4, 4))
    bad = [
        (tv.Problem(J, 0.1, [(0, 9, 0.1)]), tv.make_config(2, 64, 8, 0.01)),        # site out of range
        (tv.Problem(J, 0.1, [(5, 0, 0.1)]), tv.make_config(2, 64, 8, 0.01)),        # bad kind
        (tv.Problem(J, 0.1, [(0, 0, -1.0)]), tv.make_config(2, 64, 8, 0.01)),       # negative rate
        (tv.Problem(J, 0.1, []), tv.make_config(2, 65, 8, 0.01)),                   # samples % chains
        (tv.Problem(J, 0.1, []), tv.make_config(2, 64, 12, 0.01)),                  # chains not a multiple of 8
        (tv.Problem(J, 0.1, []), tv.make_config(2, 96, 8, 0.01, precision=1)),      # MFMA needs 64 | samples
        (tv.Problem(np.ones((4, 4)), 0.1, []), tv.make_config(2, 64, 8, 0.01)),     # nonzero diagonal
        (tv.Problem(np.zeros((193, 193)), 0.1, []), tv.make_config(2, 64, 8, 0.01)),  # N > 192
    ]
    for pb, cfg in bad:
        with pytest.raises(T.TvmcError):
            tv.Context(pb, cfg)
    ctx = tv.Context(tv.Problem(J, 0.1, []), tv.make_config(2, 64, 8, 0.01))
    with pytest.raises(T.TvmcError):
        ctx.estimate()                   # out of order
    with pytest.raises(T.TvmcError):
        ctx.set(T.Q_CHAINS, 0, np.full(8, 1 << 10, np.uint64))   # bits above N


def test_numeric_failure_is_reported(tv):
    """eps = 0 and a_0 = 20: spin 0 is up in every sample, so O_0 is constant, row 0 of S is
    exactly zero and the factorisation meets a zero pivot; the library reports it instead of
    returning garbage."""
    from paper_2506_23928_amd import tvmc as T
    n = 8
    J = np.zeros((n, n))
    th = np.zeros(n + n * (n - 1) // 2, np.complex128)
    th[0] = 20.0
    cfg = tv.make_config(1, 64, 8, 0.01, diag_shift=0.0, burn_sweeps=10)
    ctx = tv.Context(tv.Problem(J, 0.5, [(0, 0, 0.1)]), cfg, theta0=th)
    ctx.sde_step(1)
    with pytest.raises(T.TvmcError) as ei:
        ctx.synchronize()
    assert ei.value.status == T.TVMC_E_NUMERIC


def test_full_size_launch_configuration(tv, orc):
    """The N = 64 chain workload in the launch configuration the benchmark times (256
    trajectories, 4096 samples, 64 chains, 128 jump channels, MFMA S-build): sampled outputs
    of the first and last trajectories against the oracle, S entries against exact integer
    sums of the oracle's own samples, and the solve against its defining residual."""
    from paper_2506_23928_amd import tvmc as T
    w = wl.WORKLOADS["chain64_jastrow"]
    n, ns, nc, TT = w["n"], w["n_samples"], w["n_chains"], w["n_traj"]
    J = orc.couplings(w["geom"], n, w["alpha"], w["jscale"])
    jumps = wl.jumps(w)
    m = orc.n_params(0, n)
    pb, cfg, ctx = _pair(tv, orc, J, w["h"], jumps, TT, ns, nc, w["dt"], w["diag_shift"], w["seed"], precision=1)
    ctx.sample()
    ctx.estimate()
    rng = np.random.default_rng(0)
    for t in (0, TT - 1):
        chains = orc.init_chains(w["seed"], t, n, nc)
        dw = orc.draw_dw(w["seed"], t, 0, len(jumps), w["dt"])
        r = orc.evaluate(pb, 0, 0, cfg, np.zeros(m), chains, traj=t, first=True, dw=dw, want_solve=2,
                         want_moments=False)
        _check_eval(tv, ctx, t, r, n, w["diag_shift"], "full size")
        assert _rel(ctx.get(T.Q_BMEAN, t), r["bmean"]) < 1e-13
        assert _rel(ctx.get(T.Q_D, t), r["D"]) < 1e-12
        S = ctx.get(T.Q_S, t)
        s = r["samples"].astype(np.int64)
        pa = np.array(list(range(n)) + [j for j in range(n) for k in range(j + 1, n)])
        pbb = np.array([-1] * n + [k for j in range(n) for k in range(j + 1, n)])
        O = s[:, pa] * np.where(pbb[None, :] >= 0, s[:, np.maximum(pbb, 0)], 1)
        ks = rng.integers(0, m, 400)
        ls = np.minimum(rng.integers(0, m, 400), ks)
        ks[:4], ls[:4] = [0, m - 1, m - 1, 1000], [0, 0, m - 1, 999]
        c = O.sum(0)
        for k, l in zip(ks, ls):
            want = (ns * int(O[:, k] @ O[:, l]) - int(c[k]) * int(c[l])) / float(ns) ** 2 + (w["diag_shift"] if k == l else 0.0)
            assert S[k, l] == want, (k, l)
        if t == 0:
            S0 = np.tril(S) + np.tril(S, -1).T
            D0 = ctx.get(T.Q_D, t)
    ctx.sr_solve()
    ctx.synchronize()
    d = ctx.get(T.Q_DELTA0, 0)
    assert np.abs(S0 @ d - D0).max() < 1e-10 * np.abs(D0).max()
