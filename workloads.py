"""Seeded synthetic workloads shaped like the paper's quenches (inputs only).

This module holds no arithmetic of the method: it names the problem parameters (geometry,
system size, power-law exponent, field, dissipation rates), the sampler and integrator
settings, and draws the random initial parameters that a workload starts from.  Both the GPU
library and the CPU oracle receive these inputs and build everything else themselves.
"""
from __future__ import annotations

import numpy as np

SIGMA_MINUS, SIGMA_PLUS, SIGMA_Z = 0, 1, 2

# Quench workloads: a +x coherent spin state evolved under the dissipative long-range Ising
# model.  Fields: geometry, n (spins), alpha, jscale (J), h (transverse field), decay and
# dephasing rates per site, ansatz, samples per evaluation, chains, trajectories, dt, t_end,
# diagonal shift, observation interval (steps), seed.
WORKLOADS = {
    # plain FP64 check: 1D open chain N=8, Jastrow (36 parameters), 32 trajectories
    "chain8_fp64": dict(geom="obc", n=8, alpha=1.5, jscale=1.0, h=1.0, decay=0.1, dephase=0.0, ansatz="jastrow",
                        n_samples=1024, n_chains=16, n_traj=32, dt=0.01, t_end=1.0, diag_shift=1e-4, obs_every=10,
                        burn_sweeps=2, thin_sweeps=1, seed=0),
    # N=64 open chain, decay + dephasing (128 jump channels), Jastrow with 2080 parameters
    "chain64_jastrow": dict(geom="obc", n=64, alpha=1.5, jscale=1.0, h=0.5, decay=0.05, dephase=0.02,
                            ansatz="jastrow", n_samples=4096, n_chains=64, n_traj=256, dt=0.005, t_end=2.0,
                            diag_shift=1e-4, obs_every=20, burn_sweeps=2, thin_sweeps=1, seed=0),
    # N=64 periodic chain (nearest replica), alpha = 1, h = 0, decay: the setting of the paper's
    # large-N quench with the LJPH1 ansatz (there at N = 160), at the largest N one 64-bit word
    # holds; M = 3N - 3 = 189; App. D is exact here
    "chain64_ljph1": dict(geom="pbc", n=64, alpha=1.0, jscale=1.0, h=0.0, decay=0.1, dephase=0.0, ansatz="ljph",
                          d=1, n_samples=4096, n_chains=64, n_traj=256, dt=0.005, t_end=1.0, diag_shift=1e-4,
                          obs_every=20, burn_sweeps=2, thin_sweeps=1, seed=0),
    # N=64 open chain at h = 0, where the site-resolved closed form of App. D is exact
    "chain64_jastrow_h0": dict(geom="obc", n=64, alpha=1.5, jscale=1.0, h=0.0, decay=0.1, dephase=0.0,
                               ansatz="jastrow", n_samples=4096, n_chains=64, n_traj=256, dt=0.005, t_end=1.0,
                               diag_shift=1e-4, obs_every=20, burn_sweeps=2, thin_sweeps=1, seed=1),
    # N=64 open chain, decay only, RBM with N' = 64 hidden units (4224 complex parameters),
    # 8192 samples x 64 trajectories, masked autoregressive proposal (128 hidden units) retrained
    # every 20 steps; h = 0 (App. D is exact there) and h = 0.5
    "chain64_rbm_learned": dict(geom="obc", n=64, alpha=1.5, jscale=1.0, h=0.0, decay=0.1, dephase=0.0,
                                ansatz="rbm", n_hidden=64, n_samples=8192, n_chains=64, n_traj=64, dt=0.01,
                                t_end=1.0, diag_shift=1e-4, obs_every=10, burn_sweeps=2, thin_sweeps=1, seed=0,
                                proposal="learned", ar_hidden=128, ar_train_every=20, ar_train_iters=50,
                                ar_lr=3e-3, w_scale=0.01),
    "chain64_rbm_learned_h05": dict(geom="obc", n=64, alpha=1.5, jscale=1.0, h=0.5, decay=0.1, dephase=0.0,
                                    ansatz="rbm", n_hidden=64, n_samples=8192, n_chains=64, n_traj=64, dt=0.01,
                                    t_end=1.0, diag_shift=1e-4, obs_every=10, burn_sweeps=2, thin_sweeps=1, seed=0,
                                    proposal="learned", ar_hidden=128, ar_train_every=20, ar_train_iters=50,
                                    ar_lr=3e-3, w_scale=0.01),
    # N=64 open chain, RBM with hidden density 4 (N' = 256, 16704 complex parameters) and 4096
    # samples x 32 trajectories: M > N_s, the sample-space solve
    "chain64_rbm_wide": dict(geom="obc", n=64, alpha=1.5, jscale=1.0, h=0.5, decay=0.1, dephase=0.0,
                             ansatz="rbm", n_hidden=256, n_samples=4096, n_chains=64, n_traj=32, dt=0.01,
                             t_end=1.0, diag_shift=1e-4, obs_every=10, burn_sweeps=2, thin_sweeps=1, seed=0,
                             proposal="flip", w_scale=0.01),
    # The sample-space configuration at its stated shape: 2D 10x10 open lattice (N = 100, two
    # configuration words), alpha = 3, h = 1, decay 0.1, RBM with hidden density 2 (N' = 200,
    # 20300 complex parameters, weights N(0, 0.01)), 4096 samples x 32 trajectories, solved through
    # the 4096 x 4096 sample-space kernel
    "lattice10x10_rbm_ss": dict(geom="2d", n=100, ly=10, alpha=3.0, jscale=1.0, h=1.0, decay=0.1, dephase=0.0,
                                ansatz="rbm", n_hidden=200, n_samples=4096, n_chains=64, n_traj=32, dt=0.01,
                                t_end=1.0, diag_shift=1e-4, obs_every=10, burn_sweeps=2, thin_sweeps=1, seed=0,
                                proposal="flip", w_scale=0.01),
    # The paper's N = 100 quench (the transverse-field figure's setting at h = 0, where App. D is
    # exact): periodic chain (nearest replica), alpha = 1, decay kappa = 0.27, LJPH1 (297
    # parameters), 4096 samples x 64 trajectories, dt = 0.005
    # The paper's N = 160 quench (Fig. 2, LJPH1, h = 0, App. D exact) at its middle decay kappa/J = 0.1;
    # the figure does not state alpha, taken as 1 as in the N = 100 runs; three configuration
    # words, 4096 samples x 64 trajectories, dt = 0.005
    "chain160_ljph1": dict(geom="pbc", n=160, alpha=1.0, jscale=1.0, h=0.0, decay=0.1, dephase=0.0, ansatz="ljph",
                           d=1, n_samples=4096, n_chains=64, n_traj=64, dt=0.005, t_end=1.0, diag_shift=1e-4,
                           obs_every=20, burn_sweeps=2, thin_sweeps=1, seed=0),
    "chain100_ljph1": dict(geom="pbc", n=100, alpha=1.0, jscale=1.0, h=0.0, decay=0.27, dephase=0.0, ansatz="ljph",
                           d=1, n_samples=4096, n_chains=64, n_traj=64, dt=0.005, t_end=1.0, diag_shift=1e-4,
                           obs_every=20, burn_sweeps=2, thin_sweeps=1, seed=0),
    # 2D 8x8 open lattice, alpha = 3, h = 1, decay 0.1, RBM with hidden density 2 (N' = 128, 8384
    # complex parameters, weights N(0, 0.01)), 4096 samples x 32 trajectories: M > N_s, the
    # sample-space solve through the 4096 x 4096 kernel (the 10x10 shape at one configuration word)
    "lattice8x8_rbm_ss": dict(geom="2d", n=64, ly=8, alpha=3.0, jscale=1.0, h=1.0, decay=0.1, dephase=0.0,
                              ansatz="rbm", n_hidden=128, n_samples=4096, n_chains=64, n_traj=32, dt=0.01,
                              t_end=1.0, diag_shift=1e-4, obs_every=10, burn_sweeps=2, thin_sweeps=1, seed=0,
                              proposal="flip", w_scale=0.01),
}


def lattice(w: dict):
    """(lx, ly) of a workload's geometry (ly = 1 for chains)."""
    ly = w.get("ly", 1)
    return w["n"] // ly, ly


def rbm_theta0(n: int, nh: int, scale: float, seed: int) -> np.ndarray:
    """RBM start: a = b = 0, w_ij = scale (z1 + i z2) with z standard normal (seeded); the same
    for every trajectory."""
    th = np.zeros(n + nh + n * nh, np.complex128)
    th[n + nh:] = random_theta(n * nh, scale, seed)
    return th


def jumps(w: dict):
    """Local decay sqrt(gamma) sigma^- (and dephasing sqrt(gamma_phi) sigma^z) on every site."""
    out = []
    if w["decay"] > 0:
        out += [(SIGMA_MINUS, i, w["decay"]) for i in range(w["n"])]
    if w["dephase"] > 0:
        out += [(SIGMA_Z, i, w["dephase"]) for i in range(w["n"])]
    return out


def n_steps(w: dict) -> int:
    return int(round(w["t_end"] / w["dt"]))


def random_theta(m: int, scale: float, seed: int) -> np.ndarray:
    """Complex parameters scale*(z1 + i z2), z standard normal (seeded)."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(m) + 1j * rng.standard_normal(m))


def random_problem(n: int, seed: int, n_extra: int = 3):
    """A small random LITF-like problem for parity tests: random symmetric couplings, random
    field, decay on every site plus a few sigma^z / sigma^+ channels on random sites."""
    rng = np.random.default_rng(seed)
    J = rng.standard_normal((n, n)) * 0.4
    J = np.triu(J, 1)
    J = J + J.T
    hx = float(rng.uniform(0.2, 1.2))
    js = [(SIGMA_MINUS, i, float(rng.uniform(0.02, 0.3))) for i in range(n)]
    for _ in range(n_extra):
        js.append((int(rng.choice([SIGMA_PLUS, SIGMA_Z])), int(rng.integers(n)), float(rng.uniform(0.01, 0.1))))
    return J, hx, js


# Uneven batch: open chains with N drawn uniformly from {16, 24, 32, 48, 64}, alpha ~ U[0.5, 3],
# decay rate gamma ~ U[0.01, 0.2], per trajectory; h = 1; Jastrow; 2048 samples; Heun dt = 0.01
# to t = 1.  The per-trajectory parameters come from numpy's seeded generator (they are inputs,
# not random numbers of the method).
UNEVEN = dict(sizes=(16, 24, 32, 48, 64), alpha=(0.5, 3.0), gamma=(0.01, 0.2), h=1.0, jscale=1.0, n_traj=512,
              n_samples=2048, n_chains=64, dt=0.01, t_end=1.0, diag_shift=1e-4, burn_sweeps=2, thin_sweeps=1,
              seed=0)


def uneven_params(n_traj: int, seed: int = 0, w: dict = UNEVEN):
    """Per-trajectory (N, alpha, gamma) of the uneven batch."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(w["sizes"]), size=n_traj)
    alpha = rng.uniform(*w["alpha"], size=n_traj)
    gamma = rng.uniform(*w["gamma"], size=n_traj)
    return [(int(n), float(a), float(g)) for n, a, g in zip(ns, alpha, gamma)]
