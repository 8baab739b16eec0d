"""Python binding of libtvmc (include/tvmc.h): argument marshalling only.

Every step of the path runs in the HIP kernels of ``csrc/``; PyTorch only provides the device
workspace and the stream.  The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtvmc.so")

TVMC_OK, TVMC_E_INVAL, TVMC_E_NOMEM, TVMC_E_DEVICE, TVMC_E_NUMERIC, TVMC_E_STATE, TVMC_E_UNSUPPORTED = range(7)
SIGMA_MINUS, SIGMA_PLUS, SIGMA_Z = 0, 1, 2
JASTROW, RBM, LJPH = 0, 1, 2
HEUN, MIDPOINT = 0, 1
PREC_FP64, PREC_MFMA = 0, 1
(Q_THETA, Q_THETA_EVAL, Q_DELTA0, Q_DELTA1, Q_SAMPLES, Q_ELOC, Q_S, Q_D, Q_OBAR, Q_BMEAN, Q_DW, Q_ACCEPTS,
 Q_CHAINS, Q_MOMENTS, Q_OBS_HIST, Q_AR_PARAMS, Q_AR_GRAD, Q_AR_LOGQ, Q_AR_LOSS, Q_AR_ACCEPTS, Q_LOGNORM,
 Q_LOGNORM_HIST, Q_EIG, Q_AR_LOGQ_BF16) = range(24)
PROPOSAL_FLIP, PROPOSAL_LEARNED = 0, 1
SOLVER_AUTO, SOLVER_ONE_GROUP, SOLVER_MULTI_GROUP, SOLVER_SAMPLE_SPACE = 0, 1, 2, 3
SSE_NONLINEAR, SSE_LINEAR = 0, 1
REG_SHIFT, REG_SNR = 0, 1

_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class tvmc_problem(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("J", _dp), ("hx", ctypes.c_double), ("n_jumps", ctypes.c_int32),
                ("jump_kind", _i32p), ("jump_site", _i32p), ("jump_rate", _dp)]


class tvmc_ansatz(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("range", ctypes.c_int32)]


class tvmc_config(ctypes.Structure):
    _fields_ = [("n_traj", ctypes.c_int32), ("traj_offset", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("burn_sweeps", ctypes.c_int32), ("thin_sweeps", ctypes.c_int32),
                ("init_sweeps", ctypes.c_int32), ("scheme", ctypes.c_int32), ("dt", ctypes.c_double),
                ("diag_shift", ctypes.c_double), ("precision", ctypes.c_int32), ("obs_every", ctypes.c_int32),
                ("n_obs_max", ctypes.c_int32), ("seed", ctypes.c_uint64), ("proposal", ctypes.c_int32),
                ("ar_hidden", ctypes.c_int32), ("ar_train_every", ctypes.c_int32), ("ar_train_iters", ctypes.c_int32),
                ("ar_lr", ctypes.c_double), ("solver", ctypes.c_int32), ("unravelling", ctypes.c_int32),
                ("regulariser", ctypes.c_int32), ("snr_tau", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("sampler_chains", ctypes.c_int32)]


class TvmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tvmc status %d: %s" % (status, msg))
        self.status = status


_lib = None
EXPORTED = ["tvmc_workspace_size", "tvmc_init", "tvmc_workspace_size_batch", "tvmc_init_batch", "tvmc_sample", "tvmc_estimate", "tvmc_sr_solve", "tvmc_update",
            "tvmc_sde_step", "tvmc_train_proposal", "tvmc_observables", "tvmc_ensemble", "tvmc_ensemble_at", "tvmc_get", "tvmc_set", "tvmc_position",
            "tvmc_synchronize", "tvmc_set_timing", "tvmc_timing", "tvmc_last_error", "tvmc_destroy",
            "tvmc_state_size", "tvmc_save_state", "tvmc_load_state", "tvmc_static_workspace_bytes",
            "tvmc_init_static"]


def lib():
    """Load libtvmc.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtvmc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.tvmc_last_error.restype = ctypes.c_char_p
        L.tvmc_last_error.argtypes = [ctypes.c_void_p]
        for name in EXPORTED:
            if name != "tvmc_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st, ctx=None):
    if st != TVMC_OK:
        msg = lib().tvmc_last_error(ctx).decode(errors="replace")
        raise TvmcError(st, msg)


class Problem:
    """H = sum_{i<j} J_ij sz_i sz_j + hx sum_i sx_i; jumps = [(kind, site, rate), ...]."""

    def __init__(self, J, hx, jumps):
        self.J = np.ascontiguousarray(J, dtype=np.float64)
        self.n = self.J.shape[0]
        self.hx = float(hx)
        self.jumps = [tuple(j) for j in jumps]
        self.kind = np.ascontiguousarray([j[0] for j in jumps] or [0], dtype=np.int32)
        self.site = np.ascontiguousarray([j[1] for j in jumps] or [0], dtype=np.int32)
        self.rate = np.ascontiguousarray([j[2] for j in jumps] or [0.0], dtype=np.float64)

    def c(self):
        return tvmc_problem(self.n, self.J.ctypes.data_as(_dp), self.hx, len(self.jumps),
                            self.kind.ctypes.data_as(_i32p), self.site.ctypes.data_as(_i32p),
                            self.rate.ctypes.data_as(_dp))


def make_ansatz(kind: int, n_hidden: int = 0) -> tvmc_ansatz:
    """The ansatz's second number is N' for the RBM and d for LJPHd."""
    return tvmc_ansatz(kind, n_hidden, 0) if kind != LJPH else tvmc_ansatz(kind, 0, n_hidden)


def n_params(kind: int, n: int, n_hidden: int = 0) -> int:
    if kind == RBM:
        return n + n_hidden + n * n_hidden
    if kind == LJPH:
        d = n_hidden
        return n + d * (2 * n - d - 1) // 2 + (n - 1 - d)
    return n + n * (n - 1) // 2


def make_config(n_traj, n_samples, n_chains, dt, diag_shift=1e-4, burn_sweeps=2, thin_sweeps=1, init_sweeps=0,
                scheme=HEUN, precision=PREC_FP64, obs_every=0, n_obs_max=0, seed=0, traj_offset=0,
                proposal=PROPOSAL_FLIP, ar_hidden=128, ar_train_every=20, ar_train_iters=50, ar_lr=3e-3,
                solver=0, unravelling=SSE_NONLINEAR, regulariser=REG_SHIFT, snr_tau=4.0, use_graph=0,
                sampler_chains=0):
    return tvmc_config(n_traj, traj_offset, n_samples, n_chains, burn_sweeps, thin_sweeps, init_sweeps, scheme, dt,
                       diag_shift, precision, obs_every, n_obs_max, ctypes.c_uint64(seed), proposal, ar_hidden,
                       ar_train_every, ar_train_iters, ar_lr, solver, unravelling, regulariser, snr_tau,
                       int(bool(use_graph)), sampler_chains)


# ---------------------------------------------------------------- functions named as in the C ABI
def tvmc_workspace_size(problem: Problem, ansatz: tvmc_ansatz, config: tvmc_config) -> int:
    b = ctypes.c_size_t(0)
    pc = problem.c()
    _check(lib().tvmc_workspace_size(ctypes.byref(pc), ctypes.byref(ansatz), ctypes.byref(config), ctypes.byref(b)))
    return b.value


def tvmc_init(problem, ansatz, config, theta0, workspace_ptr, workspace_bytes, stream):
    ctx = ctypes.c_void_p()
    pc = problem.c()
    th = None
    if theta0 is not None:
        th = np.ascontiguousarray(np.asarray(theta0, dtype=np.complex128)).view(np.float64)
    _check(lib().tvmc_init(ctypes.byref(pc), ctypes.byref(ansatz), ctypes.byref(config),
                           th.ctypes.data_as(_dp) if th is not None else None, ctypes.c_void_p(workspace_ptr),
                           ctypes.c_size_t(workspace_bytes), ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def tvmc_static_workspace_bytes() -> int:
    b = ctypes.c_size_t(0)
    _check(lib().tvmc_static_workspace_bytes(ctypes.byref(b)))
    return b.value


def tvmc_init_static(problem, ansatz, config, theta0, stream):
    """tvmc_init on the library's static device workspace (no device allocation)."""
    ctx = ctypes.c_void_p()
    pc = problem.c()
    th = None
    if theta0 is not None:
        th = np.ascontiguousarray(np.asarray(theta0, dtype=np.complex128)).view(np.float64)
    _check(lib().tvmc_init_static(ctypes.byref(pc), ctypes.byref(ansatz), ctypes.byref(config),
                                  th.ctypes.data_as(_dp) if th is not None else None, ctypes.c_void_p(stream),
                                  ctypes.byref(ctx)))
    return ctx


def _problem_array(problems):
    arr = (tvmc_problem * len(problems))(*[p.c() for p in problems])
    return arr


def tvmc_workspace_size_batch(problems, ansatz: tvmc_ansatz, config: tvmc_config) -> int:
    b = ctypes.c_size_t(0)
    arr = _problem_array(problems)
    _check(lib().tvmc_workspace_size_batch(arr, ctypes.c_int32(len(problems)), ctypes.byref(ansatz),
                                           ctypes.byref(config), ctypes.byref(b)))
    return b.value


def tvmc_init_batch(problems, ansatz, config, theta0, workspace_ptr, workspace_bytes, stream):
    ctx = ctypes.c_void_p()
    arr = _problem_array(problems)
    th = None
    if theta0 is not None:
        th = np.ascontiguousarray(np.asarray(theta0, dtype=np.complex128)).view(np.float64)
    _check(lib().tvmc_init_batch(arr, ctypes.c_int32(len(problems)), ctypes.byref(ansatz), ctypes.byref(config),
                                 th.ctypes.data_as(_dp) if th is not None else None, ctypes.c_void_p(workspace_ptr),
                                 ctypes.c_size_t(workspace_bytes), ctypes.c_void_p(stream), ctypes.byref(ctx)))
    return ctx


def tvmc_sample(ctx):
    _check(lib().tvmc_sample(ctx), ctx)


def tvmc_estimate(ctx):
    _check(lib().tvmc_estimate(ctx), ctx)


def tvmc_sr_solve(ctx):
    _check(lib().tvmc_sr_solve(ctx), ctx)


def tvmc_update(ctx):
    _check(lib().tvmc_update(ctx), ctx)


def tvmc_sde_step(ctx, n_steps: int):
    _check(lib().tvmc_sde_step(ctx, ctypes.c_int32(n_steps)), ctx)


def tvmc_train_proposal(ctx, n_iters: int):
    _check(lib().tvmc_train_proposal(ctx, ctypes.c_int32(n_iters)), ctx)


def tvmc_observables(ctx, n_traj: int, copy=True):
    out = np.zeros((n_traj, 9)) if copy else None
    _check(lib().tvmc_observables(ctx, out.ctypes.data_as(_dp) if copy else None), ctx)
    return out


def tvmc_ensemble(ctx):
    out = np.zeros(13)
    _check(lib().tvmc_ensemble(ctx, out.ctypes.data_as(_dp)), ctx)
    return out[0:3], out[3:12].reshape(3, 3), float(out[12])


def tvmc_ensemble_at(ctx, slot, n_traj=0):
    """(M, C, xi^2) at history record `slot` (slot < 0: the last moments) and, with n_traj > 1,
    the n_traj leave-one-out xi^2 values of a jackknife over the trajectories (else None)."""
    out = np.zeros(13)
    loo = np.zeros(n_traj) if n_traj > 1 else None
    _check(lib().tvmc_ensemble_at(ctx, ctypes.c_int32(slot), out.ctypes.data_as(_dp),
                                  loo.ctypes.data_as(_dp) if loo is not None else None), ctx)
    return out[0:3], out[3:12].reshape(3, 3), float(out[12]), loo


def tvmc_synchronize(ctx):
    _check(lib().tvmc_synchronize(ctx), ctx)


def tvmc_destroy(ctx):
    _check(lib().tvmc_destroy(ctx))


class Context:
    """One batch of trajectories with its workspace held as a torch tensor.  `problem` is one
    Problem shared by every trajectory, or a list of n_traj Problems (same N, hx and jump
    channels; couplings and rates may differ per trajectory).  `n_hidden` is N' for the RBM
    and d for LJPHd."""

    _shapes = {Q_THETA: ("c", "m"), Q_THETA_EVAL: ("c", "m"), Q_DELTA0: ("c", "m"), Q_DELTA1: ("c", "m"),
               Q_SAMPLES: ("u8", "ns_w"), Q_ELOC: ("c", "ns"), Q_S: ("d", "mm"), Q_D: ("c", "m"), Q_OBAR: ("d", "m"),
               Q_BMEAN: ("c", "nch"), Q_DW: ("d", "nch"), Q_ACCEPTS: ("u4", "nc"), Q_CHAINS: ("u8", "nc_w"),
               Q_MOMENTS: ("d", "9"), Q_OBS_HIST: ("d", "hist"), Q_AR_PARAMS: ("f", "arnp"), Q_AR_GRAD: ("f", "arnp"),
               Q_AR_LOGQ: ("f", "ns"), Q_AR_LOSS: ("d", "1"), Q_AR_ACCEPTS: ("u4", "nc"), Q_LOGNORM: ("d", "1"),
               Q_LOGNORM_HIST: ("d", "nobs"), Q_EIG: ("d", "2m"), Q_AR_LOGQ_BF16: ("f", "ns")}

    def __init__(self, problem: Problem, config: tvmc_config, kind=JASTROW, n_hidden=0, theta0=None, device="cuda",
                 stream=None, static_workspace=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        batch = isinstance(problem, (list, tuple))
        self.problems = list(problem) if batch else [problem]
        self.problem = self.problems[0]
        self.config = config
        self.ansatz = make_ansatz(kind, n_hidden)
        self.m = n_params(kind, self.problem.n, n_hidden)
        if static_workspace:        # the library's static device workspace: nothing is allocated here
            if batch:
                raise ValueError("the static workspace takes one shared problem")
            self.workspace = None
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            self.ctx = tvmc_init_static(self.problem, self.ansatz, config, theta0, self.stream.cuda_stream)
            self._lib = lib()
            return
        nbytes = tvmc_workspace_size_batch(self.problems, self.ansatz, config)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = self.workspace.data_ptr()
        ptr += (-ptr) % 256
        if stream is None and config.use_graph:   # a captured graph needs a stream of its own
            stream = torch.cuda.Stream(device=self.workspace.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device=self.workspace.device)
        self.ctx = tvmc_init_batch(self.problems, self.ansatz, config, theta0, ptr, nbytes, self.stream.cuda_stream)
        self._lib = lib()    # kept for __del__, which may run while the interpreter shuts down

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self._lib.tvmc_destroy(ctx)
            self.ctx = None

    # stage calls
    def sample(self):
        tvmc_sample(self.ctx)

    def estimate(self):
        tvmc_estimate(self.ctx)

    def sr_solve(self):
        tvmc_sr_solve(self.ctx)

    def update(self):
        tvmc_update(self.ctx)

    def sde_step(self, n_steps=1):
        tvmc_sde_step(self.ctx, n_steps)

    def observables(self):
        return tvmc_observables(self.ctx, self.config.n_traj)

    def ensemble(self):
        return tvmc_ensemble(self.ctx)

    def ensemble_at(self, slot, jackknife=False):
        return tvmc_ensemble_at(self.ctx, slot, self.config.n_traj if jackknife else 0)

    def synchronize(self):
        tvmc_synchronize(self.ctx)

    def position(self):
        s, g = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tvmc_position(self.ctx, ctypes.byref(s), ctypes.byref(g)), self.ctx)
        return s.value, g.value

    def set_timing(self, on=True):
        _check(lib().tvmc_set_timing(self.ctx, ctypes.c_int32(int(on))), self.ctx)

    def timing(self, group):
        ms, cnt = ctypes.c_double(), ctypes.c_int32()
        _check(lib().tvmc_timing(self.ctx, group.encode(), ctypes.byref(ms), ctypes.byref(cnt)), self.ctx)
        return ms.value, cnt.value

    @property
    def sample_space(self):
        """Whether the solve runs in sample space (the library's rule: requested, or M > N_s; never
        for LJPHd or the SNR solve, which work in parameter space)."""
        c = self.config
        if self.ansatz.kind == LJPH or c.regulariser == REG_SNR:
            return False
        return c.solver == SOLVER_SAMPLE_SPACE or (c.solver == SOLVER_AUTO and self.m > c.n_samples)

    @property
    def solve_dim(self):
        """Dimension of the system solved: M, or N_s in sample space (real symmetric for the
        Jastrow ansatz, complex Hermitian for the RBM)."""
        return self.config.n_samples if self.sample_space else self.m

    @property
    def words(self):
        """64-bit words per configuration (sites 64 q .. 64 q + 63 in word q)."""
        return (self.problem.n + 63) // 64

    def _count(self, key):
        c = self.config
        w = self.words
        return {"m": self.m, "ns": c.n_samples, "ns_w": c.n_samples * w, "nc_w": c.n_chains * w, "mm": self.solve_dim ** 2, "nch": len(self.problem.jumps),
                "nc": c.n_chains, "9": 9, "hist": 9 * c.n_obs_max, "nobs": c.n_obs_max, "1": 1, "2m": 2 * self.m,
                "arnp": 2 * self.problem.n * c.ar_hidden + self.problem.n + c.ar_hidden}[key]

    def get(self, what, traj=0):
        dt, key = self._shapes[what]
        if what in (Q_OBAR, Q_S) and self.ansatz.kind == RBM:
            dt = "c"
        cnt = self._count(key)
        np_dt = {"c": np.complex128, "d": np.float64, "u8": np.uint64, "u4": np.uint32, "f": np.float32}[dt]
        out = np.zeros(max(cnt, 1), dtype=np_dt)
        _check(lib().tvmc_get(self.ctx, ctypes.c_int32(what), ctypes.c_int32(traj), out.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_size_t(out.nbytes)), self.ctx)
        out = out[:cnt]
        if what in (Q_SAMPLES, Q_CHAINS) and self.words > 1:
            out = out.reshape(-1, self.words)
        if what == Q_S:
            out = out.reshape(self.solve_dim, self.solve_dim)
        if what == Q_OBS_HIST:
            out = out.reshape(-1, 9)
        if what == Q_EIG:
            out = out.reshape(-1, 2)
        return out

    def save_state(self) -> np.ndarray:
        """Checkpoint at a step boundary (tvmc_save_state) as a uint8 array."""
        n = ctypes.c_size_t(0)
        _check(lib().tvmc_state_size(self.ctx, ctypes.byref(n)), self.ctx)
        blob = np.zeros(n.value, np.uint8)
        _check(lib().tvmc_save_state(self.ctx, blob.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(blob.nbytes)),
               self.ctx)
        return blob

    def load_state(self, blob):
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(lib().tvmc_load_state(self.ctx, blob.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(blob.nbytes)),
               self.ctx)

    def train_proposal(self, n_iters):
        tvmc_train_proposal(self.ctx, n_iters)

    def set(self, what, traj, values):
        np_dt = {Q_THETA: np.complex128, Q_AR_PARAMS: np.float32}.get(what, np.uint64)
        arr = np.ascontiguousarray(np.asarray(values, dtype=np_dt))
        _check(lib().tvmc_set(self.ctx, ctypes.c_int32(what), ctypes.c_int32(traj), arr.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_size_t(arr.nbytes)), self.ctx)


def unpack_samples(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 configuration words ([count] or [count, words]: site i in bit i % 64 of word i // 64)
    -> int8 spins [count, n] (+1 where the bit is set)."""
    w = np.asarray(words, dtype=np.uint64)
    if w.ndim == 1:
        w = w[:, None]
    site = np.arange(n)
    bits = (w[:, site // 64] >> (site % 64).astype(np.uint64)[None, :]) & np.uint64(1)
    return np.where(bits == 1, 1, -1).astype(np.int8)
