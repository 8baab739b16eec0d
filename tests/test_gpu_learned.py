"""Learned proposal (masked autoregressive network, independent Metropolis-Hastings moves) on
the GPU against the float64 numpy oracle (oracle/made.py).

Tolerances: the GPU network runs in FP32 (training forward/backward with FP32 weights), so
log q agrees with the float64 oracle to ~1e-5 and the batch gradient to 1e-4 of its scale;
one Adam step from the same gradient agrees to 1e-5 of the step.  The chain itself is checked
statistically (exactness) because its proposal runs on BF16 weights.
"""
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


def _params(flat, n, h):
    W1 = flat[:h * n].reshape(h, n).astype(np.float64)
    b1 = flat[h * n:h * n + h].astype(np.float64)
    W2 = flat[h * n + h:h * n + h + n * h].reshape(n, h).astype(np.float64)
    b2 = flat[h * n + h + n * h:].astype(np.float64)
    return [W1, b1, W2, b2]


def _ctx(tv, n, h, ns, nc, theta0=None, traj=1, seed=3, hx=0.6, burn=2, init=0, train_every=0, kind=0, nh=0):
    J, hxr, jumps = wl.random_problem(n, seed=n)
    cfg = tv.make_config(traj, ns, nc, 0.01, 1e-3, burn, 1, init, seed=seed, proposal=tv.tvmc.PROPOSAL_LEARNED,
                         ar_hidden=h, ar_train_every=train_every, ar_train_iters=20, ar_lr=1e-2)
    return tv.Context(tv.Problem(J, hx, jumps), cfg, kind=kind, n_hidden=nh, theta0=theta0)


def test_logq_gradient_and_adam_match_oracle(tv):
    import oracle.made as md
    from paper_2506_23928_amd import tvmc as T
    n, h, ns = 8, 24, 256
    ctx = _ctx(tv, n, h, ns, 8)
    ctx.sample()
    ctx.train_proposal(0)
    ctx.synchronize()
    p = _params(ctx.get(T.Q_AR_PARAMS, 0), n, h)
    m1, m2 = md.masks(n, h)
    assert np.all(p[0][m1 == 0] == 0) and np.all(p[2][m2 == 0] == 0)   # masked entries are zero
    s = tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n).astype(np.float64)
    logq, _ = md.forward(p, s)
    assert np.abs(ctx.get(T.Q_AR_LOGQ, 0) - logq).max() < 2e-5
    loss, grads = md.nll_and_grad(p, s)
    assert abs(ctx.get(T.Q_AR_LOSS, 0)[0] - loss) < 2e-5
    g = ctx.get(T.Q_AR_GRAD, 0).astype(np.float64)
    gw = np.concatenate([x.reshape(-1) for x in grads])
    assert np.abs(g - gw).max() < 1e-4 * np.abs(gw).max()
    # one Adam step from the GPU's own gradient (a tiny entry whose FP32 sign differs from the
    # float64 one would flip a whole +-lr step, so the step is checked on the same input)
    ctx.train_proposal(1)
    ctx.synchronize()
    newp = ctx.get(T.Q_AR_PARAMS, 0).astype(np.float64)
    z = [np.zeros_like(x) for x in p]
    want, _, _ = md.adam_step(p, _params(g, n, h), z, z, 1, lr=1e-2)
    wantf = np.concatenate([x.reshape(-1) for x in want])
    pf = np.concatenate([x.reshape(-1) for x in p])
    assert np.abs(newp - wantf).max() < 1e-5 * 1e-2 + 1e-6 * np.abs(pf).max()


@pytest.mark.parametrize("kind,d", [(0, 0), (2, 1)])
def test_learned_chain_samples_psi_squared(tv, orc, kind, d):
    """Train the proposal on predictor samples, then sample the corrector point with the mixture
    of learned independent moves and single flips: the histogram over all 2^N configurations
    must follow |psi(theta_eval)|^2 (chi-square), and learned moves must actually be accepted.
    All-pair Jastrow and LJPH1 (the same sampler, eta expanded from shared parameters)."""
    import oracle.exact as ex
    from paper_2506_23928_amd import tvmc as T
    n, h, ns, nc = 7, 32, 32768, 64
    m = orc.n_params(kind, n, d)
    th0 = wl.random_theta(m, 0.25, seed=11)
    ctx = _ctx(tv, n, h, ns, nc, theta0=th0, init=20, kind=kind, nh=d)
    ctx.sample()
    ctx.train_proposal(60)
    ctx.estimate()
    ctx.sr_solve()
    ctx.update()
    ctx.sample()
    ctx.synchronize()
    th_e = ctx.get(T.Q_THETA_EVAL, 0)
    smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n)
    idx = ((smp > 0).astype(np.int64) * (1 << np.arange(n))).sum(1)
    counts = np.bincount(idx, minlength=1 << n)
    p = np.abs((ex.jastrow_psi(n) if kind == 0 else ex.ljph_psi(n, d))(th_e)) ** 2
    p /= p.sum()
    e = p * ns
    chi2 = np.sum((counts - e) ** 2 / e)
    assert chi2 < 2.0 * (1 << n), chi2          # 127 degrees of freedom, correlated samples
    ar = ctx.get(T.Q_AR_ACCEPTS, 0)
    assert ar.sum() > 0.2 * nc * (ns // nc + 2), ar.sum()


def test_learned_proposal_crosses_modes_single_flips_cannot(tv):
    """A strongly ferromagnetic Jastrow state (eta_jk = 0.6, N = 16) has two modes (mostly up /
    mostly down) separated by a barrier single flips do not cross within an evaluation.  After
    training on the chains' own samples, learned independent moves carry chains across."""
    from paper_2506_23928_amd import tvmc as T
    n, h, ns, nc = 16, 64, 4096, 64
    m = n + n * (n - 1) // 2
    th0 = np.zeros(m, np.complex128)
    th0[n:] = 0.6
    switches = {}
    for learned in (False, True):
        J = np.zeros((n, n))
        cfg = tv.make_config(1, ns, nc, 0.01, 1e-3, 2, 1, 10, seed=5,
                             proposal=tv.tvmc.PROPOSAL_LEARNED if learned else tv.tvmc.PROPOSAL_FLIP,
                             ar_hidden=h, ar_train_every=0, ar_train_iters=0, ar_lr=1e-2)
        ctx = tv.Context(tv.Problem(J, 0.0, []), cfg, theta0=th0)
        ctx.sample()
        if learned:
            ctx.train_proposal(80)
        ctx.estimate()
        ctx.sr_solve()
        ctx.update()      # no Hamiltonian or jumps: theta stays put (up to eps)
        ctx.sample()
        ctx.synchronize()
        smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n).reshape(nc, ns // nc, n)
        mag = np.sign(smp.sum(axis=2) + 0.5)
        switches[learned] = int(np.sum(mag[:, 1:] != mag[:, :-1]))
    assert switches[False] <= 2, switches
    assert switches[True] > 100, switches


def test_learned_chain_rbm_samples_psi_squared(tv):
    """The same exactness check with the RBM ansatz (N = 7, N' = 5): the learned independent
    moves and the single flips together must sample |psi_RBM|^2."""
    import oracle.exact as ex
    from paper_2506_23928_amd import tvmc as T
    n, nh, h, ns, nc = 7, 5, 32, 32768, 64
    m = n + nh + n * nh
    th0 = wl.random_theta(m, 0.3, seed=12)
    J, _, jumps = wl.random_problem(n, seed=n)
    cfg = tv.make_config(1, ns, nc, 0.01, 1e-3, 2, 1, 20, seed=4, proposal=tv.PROPOSAL_LEARNED, ar_hidden=h,
                         ar_train_every=0, ar_train_iters=20, ar_lr=1e-2)
    ctx = tv.Context(tv.Problem(J, 0.6, jumps), cfg, kind=tv.RBM, n_hidden=nh, theta0=th0)
    ctx.sample()
    ctx.train_proposal(60)
    ctx.estimate()
    ctx.sr_solve()
    ctx.update()
    ctx.sample()       # the corrector point, sampled with the trained network
    ctx.synchronize()
    th_e = ctx.get(T.Q_THETA_EVAL, 0)
    smp = tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n)
    idx = ((smp > 0).astype(np.int64) * (1 << np.arange(n))).sum(1)
    counts = np.bincount(idx, minlength=1 << n)
    p = np.abs(ex.rbm_psi(n, nh)(th_e)) ** 2
    p /= p.sum()
    e = p * ns
    chi2 = np.sum((counts - e) ** 2 / e)
    assert chi2 < 2.0 * (1 << n), chi2
    ar = ctx.get(T.Q_AR_ACCEPTS, 0)
    assert ar.sum() > 0.2 * nc * (ns // nc + 2), ar.sum()


def _bf16(x):
    """float32 -> bfloat16 (round to nearest even) -> float64: the sampler's weight copies."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _fp32_logq_bound(p, s):
    """Worst-case error of log q evaluated in FP32 with the float64 values of its weights:
    each pre-activation sums N + 1 terms and each logit H + 1, so with g_K = K u / (1 - K u),
    u = 2^-24, |d a_k| <= g_{N+1} (|b1_k| + sum_j |W1_kj|), |d l_i| <= g_{H+1} sum_k |W2_ik| |h_k|
    + sum_k |W2_ik| |d a_k| + |b2_i| u, and log sigmoid is 1-Lipschitz (plus its own rounding
    and that of the sum over sites)."""
    import oracle.made as md
    W1, b1, W2, b2 = p
    n, h = W2.shape
    m1, m2 = md.masks(n, h)
    u = 2.0 ** -24
    g = lambda k: k * u / (1 - k * u)
    aw1, aw2 = np.abs(W1 * m1), np.abs(W2 * m2)
    da = g(n + 1) * (np.abs(b1) + aw1.sum(axis=1))                      # [H]
    logq, (_, a, hh, logits, _, _) = md.forward(p, s)
    dl = g(h + 1) * (np.abs(hh) @ aw2.T + np.abs(b2)) + da @ aw2.T      # [B, N]
    return dl.sum(axis=1) + g(n + 1) * np.abs(logq) + n * 4 * u


def test_made_benchmark_shape_matches_oracle(tv):
    """The network at the benchmark's shape: N = 64 inputs, H = 128 hidden units (so every
    kernel's second 64-lane chunk of hidden units is used), 4096 samples of a random N = 64
    problem, random masked parameters.  Training forward (FP32) against the float64 oracle within
    the worst-case FP32 bound, loss, gradient and one Adam step; and the BF16 log q that the
    samplers' acceptance test uses, element by element against a float64 evaluation of the same
    BF16-rounded weights, within the same bound."""
    import oracle.made as md
    from paper_2506_23928_amd import tvmc as T
    n, h, ns, nc = 64, 128, 4096, 64
    m = n + n * (n - 1) // 2
    ctx = _ctx(tv, n, h, ns, nc, theta0=wl.random_theta(m, 0.05, seed=21), init=4)
    ctx.sample()
    rng = np.random.default_rng(5)
    m1, m2 = md.masks(n, h)
    W1 = (rng.standard_normal((h, n)) * 0.3 * m1).astype(np.float32)
    W2 = (rng.standard_normal((n, h)) * 0.3 * m2).astype(np.float32)
    b1 = (rng.standard_normal(h) * 0.1).astype(np.float32)
    b2 = (rng.standard_normal(n) * 0.1).astype(np.float32)
    flat = np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2]).astype(np.float32)
    ctx.set(T.Q_AR_PARAMS, 0, flat)
    ctx.train_proposal(0)
    ctx.synchronize()
    p = _params(ctx.get(T.Q_AR_PARAMS, 0), n, h)
    assert np.array_equal(np.concatenate([x.reshape(-1) for x in p]), flat.astype(np.float64))
    s = tv.unpack_samples(ctx.get(T.Q_SAMPLES, 0), n).astype(np.float64)
    logq, (_, a, _, _, _, _) = md.forward(p, s)
    assert (a[:, 64:] > 0).mean() > 0.2          # hidden units 64..127 are active
    bound = _fp32_logq_bound(p, s)
    err = np.abs(ctx.get(T.Q_AR_LOGQ, 0) - logq)
    assert np.all(err <= bound), (err.max(), bound.min())
    loss, grads = md.nll_and_grad(p, s)
    assert abs(ctx.get(T.Q_AR_LOSS, 0)[0] - loss) <= bound.mean()
    g = ctx.get(T.Q_AR_GRAD, 0).astype(np.float64)
    gw = np.concatenate([x.reshape(-1) for x in grads])
    assert np.abs(g - gw).max() < 3e-4 * np.abs(gw).max(), np.abs(g - gw).max() / np.abs(gw).max()
    # the sampler's BF16 network (weights rounded to BF16, biases FP32, FP32 sums)
    pb = [_bf16(p[0]), p[1], _bf16(p[2]), p[3]]
    lqb, _ = md.forward(pb, s)
    errb = np.abs(ctx.get(T.Q_AR_LOGQ_BF16, 0) - lqb)
    assert np.all(errb <= _fp32_logq_bound(pb, s)), errb.max()
    assert np.abs(lqb - logq).max() > 10 * errb.max()      # the comparison sees the BF16 rounding
    # one Adam step from the GPU's own gradient
    ctx.train_proposal(1)
    ctx.synchronize()
    newp = ctx.get(T.Q_AR_PARAMS, 0).astype(np.float64)
    z = [np.zeros_like(x) for x in p]
    want, _, _ = md.adam_step(p, _params(g, n, h), z, z, 1, lr=1e-2)
    wantf = np.concatenate([x.reshape(-1) for x in want])
    pf = np.concatenate([x.reshape(-1) for x in p])
    assert np.abs(newp - wantf).max() < 1e-5 * 1e-2 + 1e-6 * np.abs(pf).max()
