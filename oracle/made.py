"""ORACLE -- test infrastructure, not product code.

Plain float64 numpy reference for the learned proposal: a two-layer masked autoregressive
network (MADE: Germain, Gregor, Murray, Larochelle, ICML 2015) over spin configurations,
q(s) = prod_i q(s_i | s_<i), used as an independent Metropolis-Hastings proposal for |psi|^2.
The paper has no learned proposal; this component, its degrees and masks are defined here:
  inputs s_j = +-1; hidden unit k has degree d(k) = 1 + (k mod (N-1)) and sees inputs j < d(k);
  output i sees hidden units with d(k) <= i (output 0 sees none: a bias only);
  a_k = b1_k + sum_{j < d(k)} W1[k, j] s_j,  h = relu(a),
  l_i = b2_i + sum_{d(k) <= i} W2[i, k] h_k,  q(s_i = +1 | s_<i) = sigmoid(l_i),
  log q(s) = sum_i log sigmoid(s_i l_i).
Training minimises the mean negative log-likelihood of a batch of configurations with Adam
(Kingma & Ba, 2015).
"""
from __future__ import annotations

import numpy as np


def degrees(n: int, h: int) -> np.ndarray:
    return 1 + (np.arange(h) % max(n - 1, 1))


def masks(n: int, h: int):
    d = degrees(n, h)
    m1 = (np.arange(n)[None, :] < d[:, None]).astype(np.float64)      # [H, N]
    m2 = (d[None, :] <= np.arange(n)[:, None]).astype(np.float64)     # [N, H]
    return m1, m2


def log_sigmoid(x):
    return -np.logaddexp(0.0, -x)


def forward(params, s):
    """log q(s) for a batch s [B, N] of +-1 spins; returns (logq [B], cache)."""
    W1, b1, W2, b2 = params
    n, h = W2.shape
    m1, m2 = masks(n, h)
    s = np.asarray(s, dtype=np.float64)
    a = s @ (W1 * m1).T + b1
    hh = np.maximum(a, 0.0)
    logits = hh @ (W2 * m2).T + b2
    logq = log_sigmoid(s * logits).sum(axis=1)
    return logq, (s, a, hh, logits, m1, m2)


def nll_and_grad(params, s):
    """Mean negative log-likelihood over the batch and its gradient (plain backprop)."""
    W1, b1, W2, b2 = params
    logq, (s, a, hh, logits, m1, m2) = forward(params, s)
    B = s.shape[0]
    # d(-log sigmoid(s l))/dl = -s sigmoid(-s l)
    g = -s * np.exp(log_sigmoid(-s * logits)) / B          # [B, N]
    gW2 = (g.T @ hh) * m2
    gb2 = g.sum(axis=0)
    dh = g @ (W2 * m2)
    da = dh * (a > 0.0)
    gW1 = (da.T @ s) * m1
    gb1 = da.sum(axis=0)
    return -logq.mean(), (gW1, gb1, gW2, gb2)


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of every array; returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** t)
        vh = vv / (1 - beta2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def all_configs(n: int) -> np.ndarray:
    x = np.arange(1 << n)
    return np.where((x[:, None] >> np.arange(n)[None, :]) & 1, 1, -1).astype(np.float64)
