"""Pins of the learned-proposal oracle (oracle/made.py): q normalises over all 2^N
configurations and is autoregressive (q(s_i | s_<i) does not change with s_>=i), the gradient
matches central finite differences, and Adam's first step moves every parameter by lr in the
direction of -sign(grad) (the bias-corrected ratio m/sqrt(v) is sign(g) at t = 1)."""
import numpy as np

import oracle.made as md


def _params(rng, n, h, scale=0.5):
    return [scale * rng.standard_normal((h, n)), scale * rng.standard_normal(h),
            scale * rng.standard_normal((n, h)), scale * rng.standard_normal(n)]


def test_made_normalises_and_is_autoregressive():
    rng = np.random.default_rng(0)
    for n, h in [(5, 8), (7, 16), (1, 4)]:
        p = _params(rng, n, h)
        allc = md.all_configs(n)
        logq, (_, _, _, logits, _, _) = md.forward(p, allc)
        assert abs(np.exp(logq).sum() - 1.0) < 1e-12
        # logit i must not depend on spins j >= i
        for i in range(n):
            flipped = allc.copy()
            flipped[:, i:] *= -1
            _, (_, _, _, lf, _, _) = md.forward(p, flipped)
            assert np.allclose(lf[:, i], logits[:, i], atol=1e-14)


def test_made_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    n, h = 6, 10
    p = _params(rng, n, h)
    s = rng.choice([-1.0, 1.0], size=(40, n))
    _, grads = md.nll_and_grad(p, s)
    m1, m2 = md.masks(n, h)
    eps = 1e-6
    for which, mask in [(0, m1), (1, None), (2, m2), (3, None)]:
        flat = p[which].reshape(-1)
        for idx in range(flat.size):
            if mask is not None and mask.reshape(-1)[idx] == 0:
                assert grads[which].reshape(-1)[idx] == 0.0
                continue
            q = [x.copy() for x in p]
            q[which].reshape(-1)[idx] += eps
            up, _ = md.nll_and_grad(q, s)
            q[which].reshape(-1)[idx] -= 2 * eps
            dn, _ = md.nll_and_grad(q, s)
            assert abs((up - dn) / (2 * eps) - grads[which].reshape(-1)[idx]) < 1e-7


def test_adam_first_step():
    rng = np.random.default_rng(2)
    p = [rng.standard_normal(5)]
    g = [rng.standard_normal(5)]
    z = [np.zeros(5)]
    newp, m, v = md.adam_step(p, g, z, z, 1, lr=0.01)
    assert np.allclose(newp[0] - p[0], -0.01 * np.sign(g[0]), rtol=1e-6)
    assert np.allclose(m[0], 0.1 * g[0]) and np.allclose(v[0], 0.001 * g[0] ** 2)
