"""Determinism and checkpoint/resume on the GPU.

Two runs of the same configuration give the same bits (every reduction has a fixed order and
every random number comes from a counter-based stream, so this also serves as a race check),
and a run saved at a step boundary and loaded into a fresh context continues bit for bit:
theta, chains, the moment and log Q histories, and the learned proposal's parameters."""
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


def _make(tv, kind, nh, linear, learned):
    from paper_2506_23928_amd import tvmc as T
    n = 6
    J, hx, jumps = wl.random_problem(n, seed=21)
    cfg = tv.make_config(3, 256, 8, 0.01, 1e-4, 2, 1, 3, tv.HEUN, tv.PREC_FP64, 2, 4, 17, traj_offset=2,
                         proposal=T.PROPOSAL_LEARNED if learned else T.PROPOSAL_FLIP, ar_hidden=16, ar_train_every=2,
                         ar_train_iters=5, unravelling=T.SSE_LINEAR if linear else T.SSE_NONLINEAR)
    m = tv.n_params(kind, n, nh)
    return tv.Context(tv.Problem(J, hx, jumps), cfg, kind=kind, n_hidden=nh, theta0=wl.random_theta(m, 0.05, seed=5))


def _snapshot(tv, ctx, learned):
    from paper_2506_23928_amd import tvmc as T
    out = []
    for t in range(3):
        out += [ctx.get(T.Q_THETA, t), ctx.get(T.Q_CHAINS, t), ctx.get(T.Q_OBS_HIST, t), ctx.get(T.Q_LOGNORM_HIST, t),
                ctx.get(T.Q_LOGNORM, t)]
        if learned:
            out.append(ctx.get(T.Q_AR_PARAMS, t))
    return out


@pytest.mark.parametrize("kind,nh,linear,learned", [(0, 0, False, False), (1, 3, True, True), (2, 1, False, True)])
def test_resume_is_bit_identical(tv, kind, nh, linear, learned):
    ref = _make(tv, kind, nh, linear, learned)
    ref.sde_step(6)
    ref.synchronize()
    want = _snapshot(tv, ref, learned)
    del ref
    a = _make(tv, kind, nh, linear, learned)
    a.sde_step(3)
    blob = a.save_state()
    del a
    b = _make(tv, kind, nh, linear, learned)
    b.load_state(blob)
    assert b.position() == (3, 0)
    b.sde_step(3)
    b.synchronize()
    got = _snapshot(tv, b, learned)
    for x, y in zip(got, want):
        assert np.array_equal(x, y)


def test_two_runs_give_the_same_bits(tv):
    from paper_2506_23928_amd import tvmc as T
    runs = []
    for _ in range(2):
        ctx = _make(tv, 1, 3, False, True)
        ctx.sde_step(4)
        ctx.sample()
        ctx.synchronize()
        runs.append([ctx.get(T.Q_THETA, t) for t in range(3)] + [ctx.get(T.Q_SAMPLES, t) for t in range(3)] +
                    [ctx.get(T.Q_ELOC, t) for t in range(3)])
        del ctx
    assert all(np.array_equal(x, y) for x, y in zip(*runs))


def test_checkpoint_errors(tv):
    from paper_2506_23928_amd import tvmc as T
    a = _make(tv, 0, 0, False, False)
    a.sde_step(1)
    blob = a.save_state()
    a.sample()
    with pytest.raises(T.TvmcError):
        a.save_state()                         # off a step boundary
    b = _make(tv, 2, 1, False, False)          # another parameter count
    with pytest.raises(T.TvmcError):
        b.load_state(blob)
    c = _make(tv, 0, 0, False, False)
    bad = blob.copy()
    bad[0] ^= 1                                # wrong magic
    with pytest.raises(T.TvmcError):
        c.load_state(bad)
    c.load_state(blob)
    assert c.position() == (1, 0)


def test_metrics_log(tv, tmp_path):
    """Per-step JSON-lines metrics (paper_2506_23928_amd.metrics) read back with sane values."""
    import json
    from paper_2506_23928_amd.metrics import JsonlLog
    ctx = _make(tv, 1, 3, True, True)
    ctx.set_timing(True)
    log = JsonlLog(str(tmp_path / "m.jsonl"))
    for _ in range(3):
        ctx.sde_step(1)
        log.write(ctx)
    log.close()
    recs = [json.loads(x) for x in open(tmp_path / "m.jsonl")]
    assert [r["step"] for r in recs] == [1, 2, 3]
    for r in recs:
        assert 0.0 < r["accept_flip"] <= 1.0 and 0.0 <= r["accept_learned"] <= 1.0
        assert np.isfinite(r["dtheta_norm_mean"]) and r["dtheta_norm_max"] >= r["dtheta_norm_mean"] > 0
        assert r["log_q_std"] > 0 and "solve" in r["kernel_ms"]
