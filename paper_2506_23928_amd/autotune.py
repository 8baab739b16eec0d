"""Launch-configuration autotuner.

For one problem shape (ansatz, N, M, samples, chains, trajectories) it times the library's
interchangeable forms of a step and keeps the fastest, cached in a JSON file per shape bucket:

  * the solve: one workgroup per trajectory, several per trajectory (two side streams), or, for
    M > N_s, the sample-space solve (the push-through identity gives the same increment);
  * for the Jastrow ansaetze the S-build: int8 matrix cores or FP64 (both exact, the same bits);
  * then, with the fastest of those, the sampler's workgroup shape: 1, 2, 4, 8 (or, for the RBM
    with N' <= 128, 16) Markov chains per workgroup, each chain one wavefront (the samples are
    the same bits for every shape).

Only forms with the same result are candidates, so tuning changes the speed of a run, never its
numbers beyond rounding of the solve.  Each candidate runs on a fresh context of its own (the
caller's run is untouched); the timing brackets whole steps with device synchronisation.
"""
from __future__ import annotations

import json
import os
import time

from . import tvmc


def bucket(kind, n, n_hidden, m, n_traj, n_samples, n_chains, regulariser=0) -> str:
    return "k%d_n%d_h%d_m%d_t%d_s%d_c%d_r%d" % (kind, n, n_hidden, m, n_traj, n_samples, n_chains, regulariser)


def candidates(kind, m, n_samples, regulariser=0):
    solvers = [tvmc.SOLVER_ONE_GROUP, tvmc.SOLVER_MULTI_GROUP]
    if m > n_samples and kind != tvmc.LJPH and regulariser == tvmc.REG_SHIFT:
        solvers.append(tvmc.SOLVER_SAMPLE_SPACE)
    precisions = [tvmc.PREC_MFMA, tvmc.PREC_FP64] if kind != tvmc.RBM else [None]
    return [{"solver": s, **({"precision": p} if p is not None else {})} for s in solvers for p in precisions]


def sampler_shapes(kind, n_hidden, n_chains):
    """Chains per sampler workgroup the library accepts for this shape."""
    shapes = [1, 2, 4, 8] + ([16] if kind == tvmc.RBM and n_hidden <= 128 else [])
    return [s for s in shapes if n_chains % s == 0]


def _time_steps(problems, kind, n_hidden, config, theta0, steps, device):
    import torch
    cfg = tvmc.make_config(**config)
    ctx = tvmc.Context(problems, cfg, kind=kind, n_hidden=n_hidden, theta0=theta0, device=device)
    ctx.sde_step(1)            # first step: chain burn-in and workspace first touch
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sde_step(steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    del ctx
    return el


def tune(problems, config: dict, kind=tvmc.JASTROW, n_hidden=0, theta0=None, steps=2, cache=None,
         device="cuda") -> dict:
    """Fastest candidate for this shape: {"bucket", "choice", "ms_per_step": {label: ms}}.

    `config` holds make_config's keyword arguments (n_traj, n_samples, n_chains, dt, ...);
    moments and proposal training are switched off while timing.  With `cache` (a JSON path) a
    bucket tuned before is returned without running anything."""
    problems = list(problems) if isinstance(problems, (list, tuple)) else [problems]
    n = problems[0].n
    m = tvmc.n_params(kind, n, n_hidden)
    reg = config.get("regulariser", tvmc.REG_SHIFT)
    key = bucket(kind, n, n_hidden, m, config["n_traj"], config["n_samples"], config["n_chains"], reg)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return table[key]
    base = dict(config, obs_every=0, n_obs_max=0, ar_train_every=0)
    times, last_err = {}, None
    for cand in candidates(kind, m, config["n_samples"], reg):
        label = ",".join("%s=%d" % kv for kv in sorted(cand.items()))
        try:
            times[label] = 1e3 * _time_steps(problems, kind, n_hidden, dict(base, **cand), theta0, steps, device)
        except tvmc.TvmcError as e:
            last_err = e           # a form the library rejects for this shape
    if not times:
        raise RuntimeError("no candidate form runs for bucket %s: %s" % (key, last_err))
    best = min(times, key=times.get)
    choice = {k: int(v) for k, v in (kv.split("=") for kv in best.split(","))}
    # the sampler's workgroup shape, with the fastest form
    for sc in sampler_shapes(kind, n_hidden, config["n_chains"]):
        label = best + ",sampler_chains=%d" % sc
        try:
            times[label] = 1e3 * _time_steps(problems, kind, n_hidden, dict(base, **choice, sampler_chains=sc), theta0,
                                             steps, device)
        except tvmc.TvmcError as e:
            last_err = e
    best = min(times, key=times.get)
    choice = {k: int(v) for k, v in (kv.split("=") for kv in best.split(","))}
    result = {"bucket": key, "choice": choice, "ms_per_step": times}
    if cache:
        table[key] = result
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return result
