"""Configurations of 65 to 192 spins (two or three 64-bit words: site i in word i // 64) on the
GPU against the oracle.  The bars are those of the one-word tests: samples, accept counts,
<O_k> and the Jastrow S bit for bit, local energies and <B^n> 1e-13 (RBM 1e-12), D 1e-12,
increments and theta 1e-10 relative.  N = 65 leaves one site in the second word (the ragged
case), N = 128 fills both, N = 129 puts one site in a third word and N = 192 fills three."""
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


def _oracle_eval(orc, J, hx, jumps, kind, nh, th0, ns, nc, seed, t, dt, eps, want_solve=1):
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, dt=dt, diag_shift=eps, seed=seed, init_sweeps=3)
    return orc.evaluate(orc.Problem(J, hx, jumps), kind, nh, cfg_o, th0, orc.init_chains(seed, t, J.shape[0], nc),
                        traj=t, first=True, dw=orc.draw_dw(seed, t, 0, len(jumps), dt), want_solve=want_solve)


@pytest.mark.parametrize("n,ns,nc", [(65, 256, 8), (100, 320, 16), (128, 256, 8), (129, 256, 8), (160, 320, 16),
                                     (192, 256, 8)])
def test_ljph_two_words(tv, orc, n, ns, nc):
    """LJPH1 on a random problem (sigma^-, sigma^+, sigma^z channels), random parameters: one
    evaluation and solve, S from the FP64 and the int8 S-builds (shared-distance sums across the
    word boundary), both bit-exact."""
    from paper_2506_23928_amd import tvmc as T
    d = 1
    J, hx, jumps = wl.random_problem(n, seed=n)
    m = orc.n_params(LJPH, n, d)
    th0 = wl.random_theta(m, 0.03, seed=2)
    seed, dt, eps, TT = 6, 0.01, 1e-3, 2
    ref = [_oracle_eval(orc, J, hx, jumps, LJPH, d, th0, ns, nc, seed, 3 + t, dt, eps) for t in range(TT)]
    # int8 S-build (64-sample chunks): the shared-distance sums, up to N - d - 1 terms of +-1 (191
    # at N = 192), go in as their halves and the exact sums are rebuilt in the epilogue
    runs = [tv.PREC_FP64] + ([tv.PREC_MFMA] if ns % 64 == 0 else [])
    for prec in runs:
        cfg = tv.make_config(TT, ns, nc, dt, eps, 2, 1, 3, precision=prec, seed=seed, traj_offset=3)
        ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=LJPH, n_hidden=d, theta0=th0)
        words = (n + 63) // 64
        assert ctx.words == words
        ctx.sample()
        ctx.estimate()
        S = [ctx.get(T.Q_S, t) for t in range(TT)]
        ctx.sr_solve()
        ctx.synchronize()
        for t in range(TT):
            r = ref[t]
            smp = ctx.get(T.Q_SAMPLES, t)
            assert smp.shape == (ns, words)
            assert np.array_equal(tv.unpack_samples(smp, n), r["samples"])
            assert np.all(smp[:, -1] >> np.uint64(n - 64 * (words - 1)) == 0)          # no bits above N
            assert np.array_equal(ctx.get(T.Q_ACCEPTS, t).astype(np.int64), r["accepts"])
            assert _rel(ctx.get(T.Q_ELOC, t), r["eloc"]) < 1e-13
            assert np.array_equal(ctx.get(T.Q_OBAR, t), r["obar"].real)
            low = np.tril_indices(m)
            assert np.array_equal(S[t][low], (r["S"].real + eps * np.eye(m))[low])
            assert _rel(ctx.get(T.Q_D, t), r["D"]) < 1e-12
            # the forward error of a backward-stable FP64 solve is bounded by kappa(S + eps I) 2^-53;
            # these random problems reach kappa ~ 2e7 at N = 192
            kappa = np.linalg.cond(r["S"].real + eps * np.eye(m))
            parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, t), r["delta"]), max(1e-10, kappa * 2.0 ** -53))


def test_jastrow_two_words_sample_space(tv, orc):
    """The all-pair Jastrow at N = 70 (M = 2485 > N_s = 256: the sample-space solve, whose kernel
    K = q + (q^2 - N) / 2 counts overlaps across both words)."""
    from paper_2506_23928_amd import tvmc as T
    n, ns, nc, seed, dt, eps = 70, 256, 8, 4, 0.01, 1e-3
    J, hx, jumps = wl.random_problem(n, seed=7)
    m = orc.n_params(0, n)
    th0 = wl.random_theta(m, 0.01, seed=3)
    cfg = tv.make_config(1, ns, nc, dt, eps, 2, 1, 3, seed=seed, traj_offset=5)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, theta0=th0)
    assert ctx.sample_space
    ctx.sample()
    ctx.estimate()
    Tg = ctx.get(T.Q_S, 0)
    ctx.sr_solve()
    ctx.synchronize()
    r = _oracle_eval(orc, J, hx, jumps, 0, 0, th0, ns, nc, seed, 5, dt, eps, want_solve=3)
    assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n), r["samples"])
    assert _rel(ctx.get(T.Q_ELOC, 0), r["eloc"]) < 1e-13
    low = np.tril_indices(ns)
    Tw = r["S"].real + eps * np.eye(ns)
    assert np.abs(Tg[low] - Tw[low]).max() < 1e-13 * np.abs(Tw).max()
    assert _rel(ctx.get(T.Q_D, 0), r["D"]) < 1e-12
    parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, 0), r["delta"]), 1e-10)


@pytest.mark.parametrize("n,nh,ns,nc,prec,TT", [(100, 3, 512, 8, 0, 2), (100, 3, 512, 8, 1, 1), (66, 70, 256, 8, 0, 1),
                                                (127, 20, 256, 16, 0, 1), (150, 3, 512, 8, 0, 2), (150, 3, 640, 8, 1, 1),
                                                (192, 20, 256, 16, 0, 1)])
def test_rbm_two_words(tv, orc, n, nh, ns, nc, prec, TT):
    """The RBM at N = 100 (M = 403, parameter space, FP64 and BF16-split S), N = 66 with N' = 70
    (two hidden units per lane, M = 4756 > N_s: sample space), N = 127 (M = 2687, sample space),
    and on three words N = 150 (M = 603: sample space at 512 samples, the BF16-split S at 640) and
    N = 192 (M = 4052, sample space)."""
    from paper_2506_23928_amd import tvmc as T
    J, hx, jumps = wl.random_problem(n, seed=n + 1)
    m = orc.n_params(1, n, nh)
    th0 = wl.random_theta(m, 0.05, seed=nh)
    seed, dt, eps = 21, 0.01, 1e-3
    cfg = tv.make_config(TT, ns, nc, dt, eps, 2, 1, 3, precision=prec, seed=seed, traj_offset=1)
    ctx = tv.Context(tv.Problem(J, hx, jumps), cfg, kind=tv.RBM, n_hidden=nh, theta0=th0)
    ss = ctx.sample_space
    assert ss == (m > ns)
    ctx.sample()
    ctx.estimate()
    S = [ctx.get(T.Q_S, t) for t in range(TT)] if prec == 1 else None
    ctx.sr_solve()
    ctx.synchronize()
    for t in range(TT):
        r = _oracle_eval(orc, J, hx, jumps, 1, nh, th0, ns, nc, seed, 1 + t, dt, eps, want_solve=3 if ss else 1)
        assert np.array_equal(tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n), r["samples"])
        assert np.array_equal(ctx.get(T.Q_ACCEPTS, t).astype(np.int64), r["accepts"])
        assert _rel(ctx.get(T.Q_ELOC, t), r["eloc"]) < 1e-12
        assert _rel(ctx.get(T.Q_BMEAN, t), r["bmean"]) < 1e-12
        assert _rel(ctx.get(T.Q_OBAR, t), r["obar"]) < 1e-12
        assert _rel(ctx.get(T.Q_D, t), r["D"]) < 1e-11
        if prec == 0:
            parity("Q_DELTA0", _rel(ctx.get(T.Q_DELTA0, t), r["delta"]), 1e-10)
        else:   # BF16-split S: within its entry bound of the FP64 S, and delta solves that S
            Sg = np.tril(S[t]) + np.tril(S[t], -1).conj().T
            Sw = r["S"] + eps * np.eye(m)
            dg = np.sqrt(np.abs(np.diag(Sw).real))
            bound = (2.0 ** -15 + ns * 2.0 ** -24) * np.outer(dg, dg)
            assert np.all(np.abs(np.tril(Sg - Sw)) <= bound)
            d = ctx.get(T.Q_DELTA0, t)
            assert np.abs(Sg @ d - r["D"]).max() < 1e-9 * np.abs(r["D"]).max()


def test_ljph_two_words_trajectory(tv, orc):
    """Four steps of the N = 100 periodic LJPH1 chain (the paper's N = 100 setting, h = 0.3 so
    that every flip ratio enters), 2 trajectories, moments every 2 steps: theta and the moment
    history against the oracle's trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    n, d, ns, nc, TT, steps = 100, 1, 256, 8, 2, 4
    J = orc.couplings("pbc", n, 1.0, 1.0)
    jumps = [(0, i, 0.27) for i in range(n)]
    m = orc.n_params(LJPH, n, d)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.005, diag_shift=1e-4, seed=2, n_steps=steps,
                       obs_every=2)
    th_o, obs_o, st = orc.run(orc.Problem(J, 0.3, jumps), LJPH, d, cfg_o, np.zeros(m), TT, n_threads=2)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, 0.005, 1e-4, 2, 1, 0, 0, tv.PREC_MFMA, 2, 3, 2)
    ctx = tv.Context(tv.Problem(J, 0.3, jumps), cfg, kind=LJPH, n_hidden=d)
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        assert np.abs(ctx.get(T.Q_OBS_HIST, t)[:2] - obs_o[t, :2]).max() < 1e-10
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, 2]).max() < 1e-10


def test_ljph_three_words_trajectory(tv, orc):
    """Four steps of the N = 160 periodic LJPH1 chain (the setting of Fig. 2, h = 0.3 so that every
    flip ratio enters; the eta plane is read from global memory at three words; FP64 S-build, since
    the shared-distance sums outgrow the int8 operands), 2 trajectories, moments every 2 steps:
    theta and the moment history against the oracle's trajectory driver."""
    from paper_2506_23928_amd import tvmc as T
    n, d, ns, nc, TT, steps = 160, 1, 256, 8, 2, 4
    J = orc.couplings("pbc", n, 1.0, 1.0)
    jumps = [(0, i, 0.1) for i in range(n)]
    m = orc.n_params(LJPH, n, d)
    cfg_o = orc.Config(n_samples=ns, n_chains=nc, burn_sweeps=2, dt=0.005, diag_shift=1e-4, seed=3, n_steps=steps,
                       obs_every=2)
    th_o, obs_o, st = orc.run(orc.Problem(J, 0.3, jumps), LJPH, d, cfg_o, np.zeros(m), TT, n_threads=2)
    assert st == 0
    cfg = tv.make_config(TT, ns, nc, 0.005, 1e-4, 2, 1, 0, 0, tv.PREC_FP64, 2, 3, 3)
    ctx = tv.Context(tv.Problem(J, 0.3, jumps), cfg, kind=LJPH, n_hidden=d)
    assert ctx.words == 3
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    for t in range(TT):
        parity("Q_THETA", _rel(ctx.get(T.Q_THETA, t), th_o[t]), 1e-10)
        assert np.abs(ctx.get(T.Q_OBS_HIST, t)[:2] - obs_o[t, :2]).max() < 1e-10
        assert np.abs(ctx.get(T.Q_MOMENTS, t) - obs_o[t, 2]).max() < 1e-10


def test_two_word_limits(tv):
    """N = 193, the one-word-only options and an int8 LJPHd S-build whose int32 sums of the halved
    distance sums could pass 2^31 are refused on the host."""
    from paper_2506_23928_amd import tvmc as T
    J = np.zeros((193, 193))
    with pytest.raises(T.TvmcError):
        tv.Context(tv.Problem(J, 0.5, []), tv.make_config(1, 64, 8, 0.01))
    J = np.zeros((80, 80))
    with pytest.raises(T.TvmcError):
        tv.Context(tv.Problem(J, 0.5, []), tv.make_config(1, 64, 8, 0.01, proposal=T.PROPOSAL_LEARNED, ar_hidden=32))
    with pytest.raises(T.TvmcError):
        tv.Context(tv.Problem(J, 0.5, []), tv.make_config(1, 64, 8, 0.01, regulariser=T.REG_SNR))
    # LJH at N = 192: halves up to |h| = 96, so N_s 96^2 must stay below 2^31 (N_s < 233017)
    J = np.zeros((192, 192))
    with pytest.raises(T.TvmcError, match="2\\^31"):
        tv.Context(tv.Problem(J, 0.5, []), tv.make_config(1, 233024, 8, 0.01, precision=tv.PREC_MFMA), kind=LJPH,
                   n_hidden=0)
    tv.Context(tv.Problem(J, 0.5, []), tv.make_config(1, 64, 8, 0.01, precision=tv.PREC_MFMA), kind=LJPH, n_hidden=0)


def test_lattice10x10_full_size_launch(tv, orc):
    """The sample-space configuration at its stated shape (10 x 10 open lattice, N = 100 in two
    words, alpha = 3, RBM N' = 200, M = 20300, 4096 samples x 32 trajectories) in the benchmark's
    launch configuration.  For the last trajectory: the samples bit for bit against the oracle,
    T against the closed form (1 + q)(1 + g) - 1 centred, built from the oracle's samples, and the
    increment against the parameter-space normal equations A^H (A delta) + eps delta = D with
    A = (O - <O>) / sqrt(N_s), applied through the RBM's factored O = (s, t, s t^T) rather than
    the 4096 x 20300 matrix."""
    from paper_2506_23928_amd import tvmc as T
    import bench
    w = dict(wl.WORKLOADS["lattice10x10_rbm_ss"])
    ctx = bench.build_context(tv, w, tv.PREC_FP64)
    n, nh, ns, TT = w["n"], w["n_hidden"], w["n_samples"], w["n_traj"]
    assert ctx.sample_space and ctx.words == 2
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
    K = (1.0 + s @ s.T) * (1.0 + tt @ tt.conj().T) - 1.0
    H = np.eye(ns) - 1.0 / ns
    Tc = H @ K @ H / ns + w["diag_shift"] * np.eye(ns)
    low = np.tril_indices(ns)
    assert np.abs(Tg[low] - Tc[low]).max() < 1e-12 * np.abs(Tc).max()
    del K, H, Tc, Tg
    # A delta and A^H v with O(x) = (s(x), t(x), vec(s(x) t(x)^T)), centred, / sqrt(N_s)
    d = ctx.get(T.Q_DELTA0, t)
    D = ctx.get(T.Q_D, t)
    da, db, dw = d[:n], d[n:n + nh], d[n + nh:].reshape(n, nh)
    Od = s @ da + tt @ db + np.einsum("xi,ij,xj->x", s, dw, tt)
    Ad = (Od - Od.mean()) / np.sqrt(ns)
    v = Ad / np.sqrt(ns)
    ob_s, ob_t = s.mean(0), tt.mean(0)
    ob_w = (s.T @ tt) / ns
    vs = v.sum()
    AhAd = np.concatenate([s.T @ v - ob_s * vs, tt.conj().T @ v - ob_t.conj() * vs,
                           (s.T @ (v[:, None] * tt.conj()) - ob_w.conj() * vs).reshape(-1)])
    res = AhAd + w["diag_shift"] * d - D
    assert np.abs(res).max() < 1e-8 * np.abs(D).max()
