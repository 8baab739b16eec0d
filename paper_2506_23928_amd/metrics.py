"""Per-step run metrics as JSON lines (acceptance, increment norms, jump means, log Q, timings).

Reads what the library already exposes through tvmc_get / tvmc_timing; every read synchronises
the context's stream, so a run that logs every step is slower than one that does not.
"""
from __future__ import annotations

import json

import numpy as np

from . import tvmc as T


def step_metrics(ctx, trajectories=None) -> dict:
    """Metrics of the last completed step (read between steps, at stage 0)."""
    cfg = ctx.config
    n = ctx.problem.n
    traj = range(cfg.n_traj) if trajectories is None else trajectories
    per = cfg.n_samples // cfg.n_chains
    proposals = (cfg.burn_sweeps + per * cfg.thin_sweeps) * n      # single-flip proposals per chain
    acc, dnorm, bmean, lq, lacc = [], [], [], [], []
    for t in traj:
        acc.append(ctx.get(T.Q_ACCEPTS, t).mean() / proposals)
        d0, d1 = ctx.get(T.Q_DELTA0, t), ctx.get(T.Q_DELTA1, t)
        dnorm.append(float(np.linalg.norm(0.5 * (d0 + d1)) if cfg.scheme == T.HEUN else np.linalg.norm(d1)))
        if len(ctx.problem.jumps):
            bmean.append(np.abs(ctx.get(T.Q_BMEAN, t)).mean())
        lq.append(ctx.get(T.Q_LOGNORM, t)[0])
        if cfg.proposal == T.PROPOSAL_LEARNED:
            lacc.append(ctx.get(T.Q_AR_ACCEPTS, t).mean() / (cfg.burn_sweeps + per * cfg.thin_sweeps))
    step, _ = ctx.position()
    out = {"step": step, "t": step * cfg.dt, "accept_flip": float(np.mean(acc)),
           "dtheta_norm_mean": float(np.mean(dnorm)), "dtheta_norm_max": float(np.max(dnorm)),
           "abs_bmean": float(np.mean(bmean)) if bmean else None,
           "log_q_mean": float(np.mean(lq)), "log_q_std": float(np.std(lq))}
    if lacc:
        out["accept_learned"] = float(np.mean(lacc))
    timing = {}
    for g in ("sample", "estimate", "sbuild", "solve", "update", "observe", "train"):
        ms, cnt = ctx.timing(g)
        if cnt:
            timing[g] = ms
    if timing:
        out["kernel_ms"] = timing
    return out


class JsonlLog:
    """Append one JSON line of step_metrics per call."""

    def __init__(self, path: str):
        self.f = open(path, "a")

    def write(self, ctx, **extra):
        rec = step_metrics(ctx)
        rec.update(extra)
        self.f.write(json.dumps(rec) + "\n")
        self.f.flush()

    def close(self):
        self.f.close()
