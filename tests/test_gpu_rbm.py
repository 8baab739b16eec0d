"""GPU path with the RBM ansatz (Eq. 11) against the oracle.

Same tolerances as the Jastrow tests, except: the GPU updates the hidden angles g_j
incrementally at every accepted flip (the oracle recomputes them), so after ~1e3 accepted
flips they differ by ~1e3 ulp; tanh g_j, <O_k>, the local energies (ratios are products of N'
factors on the GPU, exponentials of sums of log-cosh differences in the oracle) and the
complex S, accumulated in different orders, are compared to 1e-12 of their scale.
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


def _hermitian(S):
    """The full Hermitian matrix from its lower triangle."""
    return np.tril(S) + np.tril(S, -1).conj().T


@pytest.mark.parametrize("n,nh,ns,nc,scheme", [(5, 3, 256, 8, 0), (6, 70, 128, 4, 1), (4, 1, 64, 2, 0),
                                               (9, 20, 192, 3, 0), (7, 12, 320, 16, 1), (6, 70, 256, 32, 0)])
def test_rbm_step_parity(tv, orc, n, nh, ns, nc, scheme):
    """Predictor and corrector of one step: samples, accepts, local energies, <B^n>, <O_k>, S,
    D, both increments and theta; N' = 70 takes two hidden units per lane.  Where M > N_s
    (M = 496 and 209) the library solves in sample space: T against the oracle's sample-space
    T, the increments against its sample-space solve."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=40 + n)
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.1, seed=nh)
    seed, dt, eps, TT = 21, 0.01, 1e-3, 2
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, thin_sweeps=1, init_sweeps=3, dt=dt,
                       diag_shift=eps, scheme=scheme, seed=seed)
    pb = orc.Problem(J, hx, jumps)
    cfg = tv.make_config(TT, ns, nc, dt, eps, 2, 1, 3, scheme, tv.PREC_FP64, seed=seed, traj_offset=3)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=tv.tvmc.RBM, n_hidden=nh, theta0=th0)
    ss = ctx.sample_space
    assert ss == (m > ns)
    want_solve, dim = (3, ns) if ss else (1, m)
    ref = {}
    for t in range(TT):
        traj = 3 + t
        chains = orc.init_chains(seed, traj, n, nc)
        dw = orc.draw_dw(seed, traj, 0, len(jumps), dt)
        ref[t] = [chains, dw, orc.evaluate(pb, 1, nh, cfg_o, th0, chains, traj=traj, first=True, dw=dw,
                                           want_solve=want_solve)]
    for stage in (0, 1):
        ctx.sample()
        ctx.estimate()
        for t in range(TT):
            r = ref[t][2 + stage]
            smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n)
            assert np.array_equal(smp, r["samples"]), (stage, t)
            assert np.array_equal(ctx.get(T.Q_ACCEPTS, t).astype(np.int64), r["accepts"])
            assert _rel(ctx.get(T.Q_ELOC, t), r["eloc"]) < 1e-12
            assert _rel(ctx.get(T.Q_BMEAN, t), r["bmean"]) < 1e-12
            assert _rel(ctx.get(T.Q_OBAR, t), r["obar"]) < 1e-12
            S = ctx.get(T.Q_S, t)
            want = r["S"] + eps * np.eye(dim)
            low = np.tril_indices(dim)
            assert np.abs(S[low] - want[low]).max() < 1e-12 * np.abs(want).max()
            parity("Q_D", _rel(ctx.get(T.Q_D, t), r["D"]), 1e-11)
        ctx.sr_solve()
        for t in range(TT):
            r = ref[t][2 + stage]
            parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0 if stage == 0 else T.Q_DELTA1, t), r["delta"]), 1e-10)
        ctx.update()
        if stage == 0:
            for t in range(TT):
                chains, dw, r0 = ref[t]
                th_e = th0 + (r0["delta"] if scheme == 0 else 0.5 * r0["delta"])
                parity("Q_THETA_EVAL", _rel(ctx.get(T.Q_THETA_EVAL, t), th_e), 1e-10)
                ref[t].append(orc.evaluate(pb, 1, nh, cfg_o, th_e, chains, traj=3 + t, stage=1, first=False, dw=dw,
                                           want_solve=want_solve))
    ctx.synchronize()
    for t in range(TT):
        r0, r1 = ref[t][2], ref[t][3]
        want = th0 + (0.5 * (r0["delta"] + r1["delta"]) if scheme == 0 else r1["delta"])
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), want), 1e-10)


def test_rbm_trajectory_and_moments(tv, orc):
    """10 Heun steps of an N = 6 RBM (N' = 6) with moments every 5 steps against the oracle's
    trajectory driver (two-flip ratios of the RBM in the moment estimators)."""
    from paper_2506_23928_amd import tvmc as T
    n, nh, ns, nc, TT = 6, 6, 512, 8, 3
    J = orc.couplings("obc", n, 1.5, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.01, seed=7)
    seed, dt, eps, steps = 2, 0.01, 1e-4, 10
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, init_sweeps=5, dt=dt, diag_shift=eps, seed=seed,
                       n_steps=steps, obs_every=5)
    th_o, obs_o, st = orc.run(orc.Problem(J, 1.0, jumps), 1, nh, cfg_o, th0, TT, n_threads=3)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, dt, eps, 2, 1, 5, tv.HEUN, tv.PREC_FP64, 5, 3, seed)
    ctx = tv.Context(tv.Problem(J, 1.0, jumps), cfg, kind=tv.tvmc.RBM, n_hidden=nh, theta0=th0)
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        assert np.abs(ctx.get(T.Q_OBS_HIST, t)[:2] - obs_o[t, :2]).max() < 1e-10
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, 2]).max() < 1e-10


def test_rbm_weights_from_global_memory(tv, orc):
    """N N' > 4096: the sampler reads w rows from global memory instead of LDS (N = 40,
    N' = 110, M = 4550); samples, local energies, <B^n> and D against the oracle."""
    from paper_2506_23928_amd import tvmc as T
    n, nh, ns, nc = 40, 110, 64, 8
    J, hx, jumps = wl.random_problem(n, seed=5)
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.02, seed=9)
    seed, dt = 4, 0.01
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, init_sweeps=2, dt=dt, diag_shift=1e-3, seed=seed)
    cfg = tv.make_config(1, ns, nc, dt, 1e-3, 2, 1, 2, tv.HEUN, tv.PREC_FP64, seed=seed)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=tv.tvmc.RBM, n_hidden=nh, theta0=th0)
    ctx.sample()
    ctx.estimate()
    ctx.synchronize()
    r = orc.evaluate(orc.Problem(J, hx, jumps), 1, nh, cfg_o, th0, orc.init_chains(seed, 0, n, nc), traj=0,
                     first=True, dw=orc.draw_dw(seed, 0, 0, len(jumps), dt), want_solve=2, want_moments=False)
    assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n), r["samples"])
    assert _rel(ctx.get(T.Q_ELOC, 0), r["eloc"]) < 1e-12
    assert _rel(ctx.get(T.Q_BMEAN, 0), r["bmean"]) < 1e-12
    parity("Q_D", _rel(ctx.get(T.Q_D, 0), r["D"]), 1e-11)


def _bf16_bound(Sref, ns):
    """Entry-wise bound of the BF16-split S-build: the split of each operand keeps 2^-17 of it,
    the dropped lo*lo term is below 2^-16 of a product, and the FP32 sum of N_s products adds
    at most N_s 2^-24 of the sum of magnitudes, which the centred second moments bound by
    Cauchy-Schwarz: |dS_kl| <= (2^-15 + N_s 2^-24) sqrt(S_kk S_ll)."""
    d = np.sqrt(np.abs(np.diag(Sref).real))
    return (2.0 ** -15 + ns * 2.0 ** -24) * np.outer(d, d) + 1e-15


@pytest.mark.parametrize("n,nh,ns,nc,solver", [(5, 3, 128, 4, 1), (6, 70, 256, 8, 2), (6, 70, 256, 8, 1)])
def test_rbm_bf16_sbuild_matches_oracle(tv, orc, n, nh, ns, nc, solver):
    """The matrix-core precision form of the RBM S against the oracle's FP64 S on the same
    (bit-exact) samples, entry by entry within the split/accumulation bound; one tile (M = 23)
    and a ragged 8x8 tile grid (M = 496)."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=60 + n)
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.2, seed=nh + 1)
    seed, dt, eps = 8, 0.01, 1e-3
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, thin_sweeps=1, dt=dt, diag_shift=eps, seed=seed)
    pb = orc.Problem(J, hx, jumps)
    cfg = tv.make_config(2, ns, nc, dt, eps, 2, 1, 0, tv.HEUN, tv.PREC_MFMA, seed=seed, solver=solver)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=tv.RBM, n_hidden=nh, theta0=th0)
    ctx.sample()
    ctx.estimate()
    Ss = [ctx.get(T.Q_S, t) for t in range(2)]      # the solve factorises S in place
    ctx.sr_solve()
    ctx.synchronize()
    for t in range(2):
        chains = orc.init_chains(seed, t, n, nc)
        dw = orc.draw_dw(seed, t, 0, len(jumps), dt)
        r = orc.evaluate(pb, 1, nh, cfg_o, th0, chains, traj=t, first=True, dw=dw, want_moments=False)
        assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), r["samples"])
        S = Ss[t]
        E = r["S"] + eps * np.eye(m)
        B = _bf16_bound(r["S"], ns)
        low = np.tril_indices(m)
        for part in (np.real, np.imag):
            err = np.abs(part(S[low]) - part(E[low]))
            assert np.all(err <= B[low]), (err / B[low]).max()
        assert _rel(ctx.get(T.Q_D, t), r["D"]) < 1e-12
        # the FP64 solve of the BF16 S: its own residual
        x = ctx.get(T.Q_DELTA0, t)
        assert np.abs(_hermitian(S) @ x - r["D"]).max() < 1e-9 * np.abs(r["D"]).max()


def test_rbm_bf16_full_size_launch(tv, orc):
    """The N = 64 RBM workload in the launch configuration the benchmark times (64
    trajectories, 8192 samples, N' = 64, M = 4224, BF16-split S), with single-flip proposals
    so that the oracle reproduces the samples: for the first and last trajectory the samples
    bit for bit, <O_k> and ~1800 S entries (60 sampled parameters, every pair) against FP64
    sums over the oracle's log-derivatives of its own samples, within the split/accumulation
    bound, and the solve against its residual."""
    from paper_2506_23928_amd import tvmc as T
    import bench
    w = dict(wl.WORKLOADS["chain64_rbm_learned"])
    ctx = bench.build_context(tv, w, tv.PREC_MFMA, proposal=tv.PROPOSAL_FLIP)
    n, nh, ns, TT = w["n"], w["n_hidden"], w["n_samples"], w["n_traj"]
    m = orc.n_params(1, n, nh)
    ctx.sample()
    ctx.estimate()
    Ss = {t: ctx.get(T.Q_S, t) for t in (0, TT - 1)}      # the solve factorises S in place
    ctx.sr_solve()
    ctx.synchronize()
    th0 = wl.rbm_theta0(n, nh, w["w_scale"], w["seed"])
    pb = orc.Problem(orc.couplings(w["geom"], n, w["alpha"], w["jscale"]), w["h"], wl.jumps(w))
    cfg_o = orc.Config(n_samples=ns, n_chains=w["n_chains"], burn_sweeps=w["burn_sweeps"],
                       thin_sweeps=w["thin_sweeps"], dt=w["dt"], diag_shift=w["diag_shift"], seed=w["seed"])
    rng = np.random.default_rng(1)
    for t in (0, TT - 1):
        r = orc.evaluate(pb, 1, nh, cfg_o, th0, orc.init_chains(w["seed"], t, n, w["n_chains"]), traj=t,
                         first=True, want_solve=0, want_moments=False)
        smp = r["samples"]
        assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), smp)
        O = np.zeros((ns, 60), np.complex128)
        ks = np.concatenate([[0, n, n + nh, m - 1], rng.integers(0, m, 56)])
        for s in range(ns):
            O[s] = orc.local_quantities(1, n, nh, th0, smp[s], two_flip=False)[2][ks]
        Oc = O - O.mean(0)
        Sref = Oc.conj().T @ Oc / ns
        S = Ss[t]
        B = _bf16_bound(Sref, ns)
        for a_ in range(60):
            for b_ in range(60):
                k, l = ks[a_], ks[b_]
                if l > k:
                    continue
                want = Sref[a_, b_] + (w["diag_shift"] if k == l else 0.0)
                assert abs(S[k, l].real - want.real) <= B[a_, b_], (k, l)
                assert abs(S[k, l].imag - want.imag) <= B[a_, b_], (k, l)
        assert _rel(ctx.get(T.Q_OBAR, t)[ks], O.mean(0)) < 1e-12
        x = ctx.get(T.Q_DELTA0, t)
        D = ctx.get(T.Q_D, t)
        assert np.abs(_hermitian(S) @ x - D).max() < 1e-9 * np.abs(D).max()


@pytest.mark.parametrize("n,nh,ns,nc", [(20, 256, 256, 8), (70, 3, 256, 8), (100, 48, 128, 8)])
def test_rbm_moments_with_global_tables(tv, orc, n, nh, ns, nc):
    """The moment estimators where the factored two-flip tables (2 N N' complex) leave LDS for the
    workspace: N N' > 4096 (N = 20, N' = 256) and two configuration words (N = 70 and 100):
    the moments of the first evaluation's samples against the oracle's (1e-10)."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=n + 3)
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.02, seed=nh + 1)
    seed, dt, eps = 5, 0.01, 1e-4
    cfg = tv.make_config(1, ns, nc, dt, eps, 2, 1, 3, seed=seed)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=tv.tvmc.RBM, n_hidden=nh, theta0=th0)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, init_sweeps=3, dt=dt, diag_shift=eps, seed=seed)
    r = orc.evaluate(orc.Problem(J, hx, jumps), 1, nh, cfg_o, th0, orc.init_chains(seed, 0, n, nc), traj=0,
                     first=True, dw=orc.draw_dw(seed, 0, 0, len(jumps), dt), want_solve=0, want_moments=True)
    assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n), r["samples"])
    assert np.abs(ctx.get(T.Q_MOMENTS, 0) - r["obs"]).max() < 1e-10, (ctx.get(T.Q_MOMENTS, 0), r["obs"])
