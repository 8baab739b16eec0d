"""tvmc_init_static: the same otVMC run on the library's static device workspace (no device
allocation) as on a caller-allocated one.  Two contexts in a row on the one static array, the
second smaller than the first, each bit-identical to tvmc_init's run of the same problem."""
import gc

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


def _run(tv, static, n, kind, nh, TT, ns, nc, steps, seed):
    from paper_2506_23928_amd import tvmc as T
    from paper_2506_23928_amd.problem import kac_couplings
    J = kac_couplings("obc", n, 1.5, 1.0)
    jumps = [(tv.SIGMA_MINUS, i, 0.1) for i in range(n)] + [(tv.SIGMA_Z, 0, 0.05)]
    th0 = wl.rbm_theta0(n, nh, 0.05, seed) if kind == tv.RBM else None
    cfg = tv.make_config(TT, ns, nc, 0.01, 1e-4, 2, 1, 3, tv.HEUN, tv.PREC_MFMA, 2, steps // 2 + 1, seed)
    ctx = tv.Context(tv.Problem(J, 0.7, jumps), cfg, kind=kind, n_hidden=nh, theta0=th0, static_workspace=static)
    ctx.sde_step(steps)
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    out = [(ctx.get(T.Q_THETA, t), ctx.get(T.Q_SAMPLES, t), ctx.get(T.Q_OBS_HIST, t), ctx.get(T.Q_MOMENTS, t))
           for t in range(TT)]
    M, C, x2 = ctx.ensemble()
    del ctx
    gc.collect()
    return out, (M, C, x2)


@pytest.mark.parametrize("case", [(8, 0, 0, 32, 1024, 16, 4, 3), (6, 1, 4, 4, 256, 8, 3, 5)])
def test_static_workspace_equals_caller_workspace(tv, case):
    n, kind, nh, TT, ns, nc, steps, seed = case
    got, eg = _run(tv, True, n, kind, nh, TT, ns, nc, steps, seed)
    want, ew = _run(tv, False, n, kind, nh, TT, ns, nc, steps, seed)
    for t in range(TT):
        for a, b in zip(got[t], want[t]):
            assert np.array_equal(a, b), t
    assert np.array_equal(eg[0], ew[0]) and np.array_equal(eg[1], ew[1]) and eg[2] == ew[2]


def test_static_workspace_limits(tv):
    from paper_2506_23928_amd import tvmc as T
    limit = T.tvmc_static_workspace_bytes()
    assert limit == 64 << 20
    J = np.zeros((64, 64))
    big = tv.make_config(256, 4096, 64, 0.01)          # ~10 GB of workspace
    with pytest.raises(T.TvmcError) as e:
        tv.Context(tv.Problem(J, 0.5, []), big, static_workspace=True)
    assert e.value.status == T.TVMC_E_NOMEM
    small = tv.make_config(2, 64, 8, 0.01)
    J8 = np.zeros((8, 8))
    a = tv.Context(tv.Problem(J8, 0.5, []), small, static_workspace=True)
    with pytest.raises(T.TvmcError) as e:             # one live context per device
        tv.Context(tv.Problem(J8, 0.5, []), small, static_workspace=True)
    assert e.value.status == T.TVMC_E_STATE
    del a
    gc.collect()
    b = tv.Context(tv.Problem(J8, 0.5, []), small, static_workspace=True)   # free again after destroy
    del b
    gc.collect()
