"""Host-side construction of the LITF problem (Eq. 10) handed to the library.

Couplings are Kac-normalised power laws: J_ij = J r_ij^-alpha / K(alpha) with
K(alpha) = sum_{i<j} r_ij^-alpha / (N-1).  Geometries: open chain (r = |i-j|), periodic chain
keeping only the nearest replica (r = min(|i-j|, N-|i-j|)), open 2D lattice (Euclidean r).
The library itself takes any symmetric J with zero diagonal.
"""
from __future__ import annotations

import numpy as np

from .tvmc import SIGMA_MINUS, SIGMA_Z, Problem


def distances(geom: str, lx: int, ly: int = 1) -> np.ndarray:
    if geom == "2d":
        x = np.arange(lx * ly) % lx
        y = np.arange(lx * ly) // lx
        return np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    i = np.arange(lx)
    d = np.abs(i[:, None] - i[None, :]).astype(np.float64)
    if geom == "pbc":
        d = np.minimum(d, lx - d)
    elif geom != "obc":
        raise ValueError(geom)
    return d


def kac_couplings(geom: str, lx: int, alpha: float, jscale: float = 1.0, ly: int = 1) -> np.ndarray:
    r = distances(geom, lx, ly)
    n = r.shape[0]
    off = ~np.eye(n, dtype=bool)
    w = np.zeros_like(r)
    w[off] = r[off] ** (-alpha)
    kac = np.sum(np.triu(w, 1)) / (n - 1)
    return jscale * w / kac


def litf_problem(n: int, alpha: float, h: float, gamma_decay: float, gamma_dephase: float = 0.0, jscale: float = 1.0,
                 geom: str = "obc", ly: int = 1) -> Problem:
    """H = sum_{i<j} J_ij sz sz + h sum sx with local decay (and optional dephasing) on every site."""
    lx = n // ly if geom == "2d" else n
    J = kac_couplings(geom, lx, alpha, jscale, ly) if n > 1 else np.zeros((1, 1))
    jumps = [(SIGMA_MINUS, i, gamma_decay) for i in range(n)] if gamma_decay > 0 else []
    if gamma_dephase > 0:
        jumps += [(SIGMA_Z, i, gamma_dephase) for i in range(n)]
    return Problem(J, h, jumps)
