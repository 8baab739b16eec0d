"""A trajectory's path does not depend on the batch it runs in.

Every random number is keyed by (seed, trajectory id, step, purpose) and every kernel works on
one trajectory's data with a fixed order of operations, so a trajectory integrated alone (the
plain form: one trajectory per launch) and the same trajectory inside a batch must agree bit for
bit in FP64 with single-flip proposals.  This is what lets the plain form's statistics be taken
from a batched FP64 run."""
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


@pytest.mark.parametrize("kind,nh,solver", [(1, 16, 0), (0, 0, 0), (0, 0, 1), (2, 1, 0)])
def test_alone_equals_batched(tv, kind, nh, solver):
    from paper_2506_23928_amd import tvmc as T
    from paper_2506_23928_amd.problem import kac_couplings
    n, ns, nc, TT, steps = 16, 1024, 16, 5, 3
    J = kac_couplings("obc", n, 1.5, 1.0)
    jumps = [(tv.SIGMA_MINUS, i, 0.1) for i in range(n)]
    m = tv.n_params(kind, n, nh)
    th0 = wl.rbm_theta0(n, nh, 0.01, 0) if kind == 1 else None
    prob = tv.Problem(J, 0.5, jumps)
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-4, 2, 1, 4 if kind == 1 else 0, tv.HEUN, tv.PREC_FP64, 1, steps + 1, 7,
                         solver=solver)
    batch = tv.Context(prob, cfg, kind=kind, n_hidden=nh, theta0=th0)
    batch.sde_step(steps)
    batch.synchronize()
    for traj in (0, 3):
        cfg1 = tv.make_config(1, ns, nc, 0.01, 1e-4, 2, 1, 4 if kind == 1 else 0, tv.HEUN, tv.PREC_FP64, 1,
                              steps + 1, 7, traj_offset=traj, solver=solver)
        alone = tv.Context(prob, cfg1, kind=kind, n_hidden=nh, theta0=th0)
        alone.sde_step(steps)
        alone.synchronize()
        assert np.array_equal(alone.get(T.Q_THETA, 0), batch.get(T.Q_THETA, traj)), (traj, m)
        assert np.array_equal(alone.get(T.Q_SAMPLES, 0), batch.get(T.Q_SAMPLES, traj))
        assert np.array_equal(alone.get(T.Q_OBS_HIST, 0), batch.get(T.Q_OBS_HIST, traj))
        del alone
