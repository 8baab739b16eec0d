"""Uneven batches: trajectories of different system sizes, couplings and rates in one job.

Trajectories are grouped by N (the sampler, the S build and the solve are shaped by N and by
M(N)); each group is one library context holding one problem per trajectory, and every
group's steps are issued on its own HIP stream (default priority), so the groups' kernels run
side by side and together fill the device.  Trajectory i draws its random numbers with the
trajectory index rank(i) + traj_offset, where rank orders the trajectories by N, stably.
Each step runs entirely in the library's kernels; this module only marshals and issues calls.
"""
from __future__ import annotations

import numpy as np

from . import tvmc


class UnevenBatch:
    """autotune: None, or the path of a JSON cache: each group's solver form (and, for the
    Jastrow ansaetze, S-build precision) is then the fastest one measured for its shape."""

    def __init__(self, problems, kind=tvmc.JASTROW, n_hidden=0, device="cuda", streams=True, autotune=None,
                 **config):
        import torch
        self.problems = list(problems)
        self.kind, self.n_hidden = kind, n_hidden
        ns = np.array([p.n for p in self.problems])
        self.order = np.argsort(ns, kind="stable")
        self.rank = np.empty_like(self.order)
        self.rank[self.order] = np.arange(len(self.order))
        offset = config.pop("traj_offset", 0)
        self.groups = []
        start = 0
        for n in np.unique(ns):
            members = self.order[start:start + int((ns == n).sum())]
            gconf = dict(config, n_traj=len(members), traj_offset=offset + start)
            if autotune:
                from .autotune import tune
                gconf.update(tune([self.problems[i] for i in members], gconf, kind, n_hidden, cache=autotune,
                                  device=device)["choice"])
            cfg = tvmc.make_config(**gconf)
            stream = torch.cuda.Stream(device=device) if streams else None
            ctx = tvmc.Context([self.problems[i] for i in members], cfg, kind=kind, n_hidden=n_hidden,
                               device=device, stream=stream)
            self.groups.append((int(n), members, ctx))
            start += len(members)

    def sde_step(self, n_steps=1):
        """Issue n_steps steps for every group (asynchronous; each group on its own stream)."""
        for _, _, ctx in self.groups:
            ctx.sde_step(n_steps)

    def synchronize(self):
        for _, _, ctx in self.groups:
            ctx.synchronize()

    def set_theta(self, i, theta):
        n, members, ctx = self._where(i)
        ctx.set(tvmc.Q_THETA, int(np.nonzero(members == i)[0][0]), theta)

    def get(self, what, i):
        _, members, ctx = self._where(i)
        return ctx.get(what, int(np.nonzero(members == i)[0][0]))

    def theta(self, i):
        return self.get(tvmc.Q_THETA, i)

    def observables(self):
        """[n_traj][9] moments at the current parameters, in the caller's trajectory order."""
        out = np.zeros((len(self.problems), 9))
        for _, members, ctx in self.groups:
            out[members] = ctx.observables()
        return out

    def _where(self, i):
        for g in self.groups:
            if i in g[1]:
                return g
        raise IndexError(i)
