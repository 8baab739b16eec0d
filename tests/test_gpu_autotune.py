"""Autotuner: candidates are timed on fresh contexts, the fastest is cached per shape bucket, and
the chosen form gives the default form's trajectory (the candidates differ only in speed)."""
import json

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


@pytest.mark.parametrize("n,ncand", [(12, 4 + 4), (24, 6 + 4)])
def test_tune_caches_and_keeps_the_numbers(tv, tmp_path, n, ncand):
    from paper_2506_23928_amd import tvmc as T
    from paper_2506_23928_amd.autotune import tune
    J, hx, jumps = wl.random_problem(n, seed=n)
    pb = tv.Problem(J, hx, jumps)
    conf = dict(n_traj=4, n_samples=256, n_chains=8, dt=0.01, diag_shift=1e-3, seed=3)
    cache = str(tmp_path / "tune.json")
    r = tune([pb], conf, cache=cache)
    assert len(r["ms_per_step"]) == ncand and all(v > 0 for v in r["ms_per_step"].values())
    assert r["choice"]["sampler_chains"] in (1, 2, 4, 8)          # the sampler's workgroup shape was tuned
    assert json.load(open(cache))[r["bucket"]] == r
    assert tune([pb], conf, cache=cache) == r                 # from the cache, nothing run
    th = []
    for extra in ({}, r["choice"]):
        ctx = tv.Context(pb, tv.make_config(**dict(conf, **extra)))
        ctx.sde_step(3)
        ctx.synchronize()
        th.append(np.array([ctx.get(T.Q_THETA, t) for t in range(4)]))
    assert np.abs(th[0] - th[1]).max() <= 1e-8 * np.abs(th[0]).max()


def test_uneven_batch_with_autotune(tv, tmp_path):
    from paper_2506_23928_amd import tvmc as T
    from paper_2506_23928_amd.uneven import UnevenBatch
    probs = []    # one batch shares N, hx and the jump channels; couplings and rates differ
    for i, n in enumerate([8, 16, 8, 16]):
        J, _, _ = wl.random_problem(n, seed=40 + i)
        probs.append(tv.Problem(J, 0.6, [(0, s, 0.05 + 0.02 * i) for s in range(n)]))
    conf = dict(n_samples=256, n_chains=8, dt=0.01, diag_shift=1e-3, seed=5)
    a = UnevenBatch(probs, autotune=str(tmp_path / "t.json"), **conf)
    b = UnevenBatch(probs, **conf)
    for x in (a, b):
        x.sde_step(2)
        x.synchronize()
    for i in range(4):
        ta, tb = a.theta(i), b.theta(i)
        assert np.abs(ta - tb).max() <= 1e-8 * np.abs(tb).max()
    assert len(json.load(open(tmp_path / "t.json"))) == 2
