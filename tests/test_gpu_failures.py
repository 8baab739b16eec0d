"""Failure detection forced from the host: a singular S with no diagonal shift.

At the RBM's all-zero parameters every weight log-derivative s_i tanh(b_j + sum_i w_ij s_i) is
exactly 0 (and so is tanh b_j), so with eps = 0 the rows of S for the weights and hidden
biases vanish: the Cholesky solve meets a
zero pivot and the library reports TVMC_E_NUMERIC; the SNR solve drops the zero eigenvalues
instead and the step stays finite.  Every kernel runs to its end either way."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tv():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    import paper_2506_23928_amd as tv
    from paper_2506_23928_amd import tvmc
    tvmc.lib()
    return tv


def _ctx(tv, reg):
    from paper_2506_23928_amd import tvmc as T
    n, nh = 6, 3
    J = np.zeros((n, n))
    J[0, 1] = J[1, 0] = 0.5
    cfg = tv.make_config(2, 128, 8, 0.01, diag_shift=0.0, precision=tv.PREC_FP64, regulariser=reg)
    return tv.Context(tv.Problem(J, 0.4, [(0, i, 0.1) for i in range(n)]), cfg, kind=T.RBM, n_hidden=nh)


def test_zero_pivot_is_reported(tv):
    from paper_2506_23928_amd import tvmc as T
    ctx = _ctx(tv, T.REG_SHIFT)
    ctx.sde_step(1)
    with pytest.raises(T.TvmcError) as ei:
        ctx.synchronize()
    assert ei.value.status == T.TVMC_E_NUMERIC


def test_snr_solve_drops_the_null_space(tv):
    from paper_2506_23928_amd import tvmc as T
    ctx = _ctx(tv, T.REG_SNR)
    ctx.sample()
    ctx.estimate()
    ctx.sr_solve()
    ctx.synchronize()
    eig = ctx.get(T.Q_EIG, 0)
    assert (eig[:, 0] == 0).sum() == 21          # tanh 0 = 0: the 3 hidden biases and 18 weights
    d = ctx.get(T.Q_DELTA0, 0)
    assert np.all(np.isfinite(d)) and np.all(d[6:] == 0) and np.any(d[:6] != 0)
