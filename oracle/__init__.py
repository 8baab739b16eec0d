"""ORACLE -- test infrastructure, not product code.

Plain FP64 CPU reference for trajectory-unravelled tVMC (the otVMC equations, Eq. 8 of
"Unraveling Open Quantum Dynamics with Time-Dependent Variational Monte Carlo", with the
predictor-corrector solvers of App. C), plus exact references in :mod:`oracle.exact`.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may import
this package.  It shares no code with the GPU library (``paper_2506_23928_amd``) and never
imports it.  The C core (``otvmc_oracle.c``) is compiled with gcc by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "otvmc_oracle.c")
_LIB = os.path.join(_HERE, "libotvmc_oracle.so")

SIGMA_MINUS, SIGMA_PLUS, SIGMA_Z = 0, 1, 2
JASTROW, RBM, LJPH = 0, 1, 2
HEUN, MIDPOINT, EULER = 0, 1, 2
REG_SHIFT, REG_SNR = 0, 1

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.POINTER(ctypes.c_double)
_c_i8p = ctypes.POINTER(ctypes.c_int8)
_c_i64p = ctypes.POINTER(ctypes.c_int64)


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("J", _c_dp), ("hx", ctypes.c_double), ("n_ch", ctypes.c_int32),
                ("kind", _c_i32p), ("site", _c_i32p), ("rate", _c_dp)]


class _AnsatzC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("range", ctypes.c_int32)]


def _Ansatz(kind, n_hidden):
    """The ansatz's second number is N' for the RBM and d for LJPHd (LJPH0 = LJH, LJPH(N-1) =
    the all-pair Jastrow, the LJNH of the LITF section, in the same parameter order)."""
    if kind == LJPH:
        return _AnsatzC(kind, 0, n_hidden)
    return _AnsatzC(kind, n_hidden, 0)


class _Config(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("n_chains", ctypes.c_int32), ("burn_sweeps", ctypes.c_int32),
                ("thin_sweeps", ctypes.c_int32), ("init_sweeps", ctypes.c_int32), ("enumerate", ctypes.c_int32),
                ("dt", ctypes.c_double), ("diag_shift", ctypes.c_double), ("scheme", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("obs_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("linear", ctypes.c_int32), ("regulariser", ctypes.c_int32), ("snr_tau", ctypes.c_double)]


class _EvalOut(ctypes.Structure):
    _fields_ = [("samples", _c_i8p), ("eloc", _c_dp), ("S", _c_dp), ("F", _c_dp), ("Nn", _c_dp), ("D", _c_dp),
                ("bmean", _c_dp), ("obar", _c_dp), ("delta", _c_dp), ("accepts", _c_i64p), ("obs", _c_dp),
                ("seconds", _c_dp), ("dlognorm", _c_dp), ("eig", _c_dp), ("G", _c_dp)]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain IEEE double: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_u53.restype = ctypes.c_double
        L.orc_n_params.restype = ctypes.c_int32
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ problem description
class Problem:
    """H = sum_{i<j} J_ij sz_i sz_j + hx sum_i sx_i;  L_c = sqrt(rate_c) op(kind_c) on site_c."""

    def __init__(self, J, hx, jumps):
        self.J = np.ascontiguousarray(J, dtype=np.float64)
        self.n = self.J.shape[0]
        self.hx = float(hx)
        self.kind = np.ascontiguousarray([j[0] for j in jumps], dtype=np.int32)
        self.site = np.ascontiguousarray([j[1] for j in jumps], dtype=np.int32)
        self.rate = np.ascontiguousarray([j[2] for j in jumps], dtype=np.float64)
        self.jumps = [tuple(j) for j in jumps]

    @property
    def n_ch(self):
        return len(self.kind)

    def _c(self):
        k = self.kind if self.n_ch else np.zeros(1, np.int32)
        s = self.site if self.n_ch else np.zeros(1, np.int32)
        r = self.rate if self.n_ch else np.zeros(1, np.float64)
        self._keep = (k, s, r)
        return _Problem(self.n, _p(self.J, _c_dp), self.hx, self.n_ch, _p(k, _c_i32p), _p(s, _c_i32p), _p(r, _c_dp))


def couplings(geom: str, n_or_lx: int, alpha: float, jscale: float, ly: int = 1) -> np.ndarray:
    """Kac-normalised power-law couplings (Eq. 10).  geom: 'obc', 'pbc' (nearest replica), '2d'."""
    g = {"obc": 0, "pbc": 1, "2d": 2}[geom]
    n = n_or_lx * ly if g == 2 else n_or_lx
    J = np.zeros((n, n))
    st = lib().orc_couplings(ctypes.c_int32(g), ctypes.c_int32(n_or_lx), ctypes.c_int32(ly), ctypes.c_double(alpha),
                             ctypes.c_double(jscale), _p(J, _c_dp))
    if st:
        raise ValueError("bad geometry")
    return J


def n_params(kind: int, n: int, n_hidden: int = 0) -> int:
    a = _Ansatz(kind, n_hidden)
    return lib().orc_n_params(ctypes.byref(a), ctypes.c_int32(n))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p))
    return o


def u53(a: int, b: int) -> float:
    return lib().orc_u53(ctypes.c_uint32(a), ctypes.c_uint32(b))


def draw_dw(seed: int, traj: int, step: int, n_ch: int, dt: float) -> np.ndarray:
    o = np.zeros(max(n_ch, 1))
    lib().orc_draw_dw(ctypes.c_uint64(seed), ctypes.c_int32(traj), ctypes.c_int32(step), ctypes.c_int32(n_ch),
                      ctypes.c_double(dt), _p(o, _c_dp))
    return o[:n_ch]


def init_chains(seed: int, traj: int, n: int, n_chains: int) -> np.ndarray:
    o = np.zeros((n_chains, n), np.int8)
    lib().orc_init_chains(ctypes.c_uint64(seed), ctypes.c_int32(traj), ctypes.c_int32(n), ctypes.c_int32(n_chains),
                          _p(o, _c_i8p))
    return o


def _theta2(theta):
    t = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128))
    return t.view(np.float64)


def logpsi(kind, n, n_hidden, theta, sigma) -> complex:
    a = _Ansatz(kind, n_hidden)
    t = _theta2(theta)
    s = np.ascontiguousarray(sigma, dtype=np.int8)
    o = np.zeros(2)
    lib().orc_logpsi(ctypes.byref(a), ctypes.c_int32(n), _p(t, _c_dp), _p(s, _c_i8p), _p(o, _c_dp))
    return complex(o[0], o[1])


def local_quantities(kind, n, n_hidden, theta, sigma, two_flip=True):
    """(flip log-ratios [n], two-flip log-ratios [n,n] or None, O_k [M]) at one configuration."""
    a = _Ansatz(kind, n_hidden)
    m = n_params(kind, n, n_hidden)
    t = _theta2(theta)
    s = np.ascontiguousarray(sigma, dtype=np.int8)
    f1 = np.zeros(n, np.complex128)
    f2 = np.zeros((n, n), np.complex128) if two_flip else None
    O = np.zeros(m, np.complex128)
    lib().orc_local_quantities(ctypes.byref(a), ctypes.c_int32(n), _p(t, _c_dp), _p(s, _c_i8p),
                               _p(f1.view(np.float64), _c_dp),
                               _p(f2.view(np.float64), _c_dp) if two_flip else None,
                               _p(O.view(np.float64), _c_dp))
    return f1, f2, O


class Config:
    def __init__(self, n_samples=1024, n_chains=16, burn_sweeps=2, thin_sweeps=1, init_sweeps=0, enumerate=False,
                 dt=0.01, diag_shift=1e-4, scheme=HEUN, n_steps=1, obs_every=0, seed=0, linear=False,
                 regulariser=0, snr_tau=4.0):
        self.__dict__.update(locals())
        del self.__dict__["self"]

    def _c(self):
        return _Config(self.n_samples, self.n_chains, self.burn_sweeps, self.thin_sweeps, self.init_sweeps,
                       int(bool(self.enumerate)), self.dt, self.diag_shift, self.scheme, self.n_steps,
                       self.obs_every, ctypes.c_uint64(self.seed), int(bool(self.linear)), int(self.regulariser),
                       float(self.snr_tau))


def eigh_sym(A):
    """The oracle's cyclic-Jacobi eigen-decomposition of a real symmetric matrix -> (lam, V)."""
    A = np.array(A, dtype=np.float64, order="C")
    m = A.shape[0]
    V = np.zeros((m, m))
    lam = np.zeros(m)
    st = lib().orc_eigh_sym(ctypes.c_int32(m), _p(A, _c_dp), _p(V, _c_dp), _p(lam, _c_dp))
    if st:
        raise RuntimeError("Jacobi did not converge")
    return lam, V


def eigh_herm(A):
    """The oracle's cyclic-Jacobi eigen-decomposition of a complex Hermitian matrix -> (lam, V)."""
    A = np.array(A, dtype=np.complex128, order="C")
    m = A.shape[0]
    V = np.zeros((m, m), np.complex128)
    lam = np.zeros(m)
    st = lib().orc_eigh_herm(ctypes.c_int32(m), _p(A.view(np.float64), _c_dp), _p(V.view(np.float64), _c_dp),
                             _p(lam, _c_dp))
    if st:
        raise RuntimeError("Jacobi did not converge")
    return lam, V


def evaluate(problem: Problem, kind: int, n_hidden: int, cfg: Config, theta, chains, traj=0, step=0, stage=0,
             first=True, dw=None, want_solve=True, want_moments=True):
    """One evaluation of Eq. 8's right-hand side at theta; returns a dict of every quantity.

    ``chains`` (int8 [n_chains, N]) is advanced in place, as the sampler would.  want_solve:
    0 sampling and local quantities only, 1 everything, 2 everything but S and the solve,
    3 everything with the solve done in sample space (r["S"] then holds T = O_c O_c^H / ns)."""
    n, m, nch = problem.n, n_params(kind, problem.n, n_hidden), problem.n_ch
    ns = (1 << n) if cfg.enumerate else cfg.n_samples
    a = _Ansatz(kind, n_hidden)
    t = _theta2(theta)
    dwa = np.ascontiguousarray(np.zeros(max(nch, 1)) if dw is None else np.asarray(dw, np.float64))
    if dwa.size == 0:
        dwa = np.zeros(1)
    r = {
        "samples": np.zeros((ns, n), np.int8), "eloc": np.zeros(ns, np.complex128),
        "S": np.zeros((m, m) if int(want_solve) == 1 else (ns, ns) if int(want_solve) == 3 else (1, 1), np.complex128),
        "F": np.zeros(m, np.complex128),
        "Nn": np.zeros((max(nch, 1), m), np.complex128), "D": np.zeros(m, np.complex128),
        "bmean": np.zeros(max(nch, 1), np.complex128), "obar": np.zeros(m, np.complex128),
        "delta": np.zeros(m, np.complex128), "accepts": np.zeros(max(cfg.n_chains, 1), np.int64),
        "obs": np.zeros(9), "seconds": np.zeros(3), "dlognorm": np.zeros(1), "eig": np.zeros((m, 2)),
        "G": np.zeros(ns, np.complex128),
    }
    eo = _EvalOut(_p(r["samples"], _c_i8p), _p(r["eloc"].view(np.float64), _c_dp),
                  _p(r["S"].view(np.float64), _c_dp), _p(r["F"].view(np.float64), _c_dp),
                  _p(r["Nn"].view(np.float64), _c_dp), _p(r["D"].view(np.float64), _c_dp),
                  _p(r["bmean"].view(np.float64), _c_dp), _p(r["obar"].view(np.float64), _c_dp),
                  _p(r["delta"].view(np.float64), _c_dp), _p(r["accepts"], _c_i64p),
                  _p(r["obs"], _c_dp) if want_moments else None, _p(r["seconds"], _c_dp),
                  _p(r["dlognorm"], _c_dp), _p(r["eig"], _c_dp), _p(r["G"].view(np.float64), _c_dp))
    ch = chains if chains is not None else np.zeros((1, n), np.int8)
    assert ch.dtype == np.int8 and ch.flags.c_contiguous
    pc = problem._c()
    st = lib().orc_eval(ctypes.byref(pc), ctypes.byref(a), ctypes.byref(cfg._c()), _p(t, _c_dp), _p(ch, _c_i8p),
                        ctypes.c_int32(traj), ctypes.c_int32(step), ctypes.c_int32(stage), ctypes.c_int32(int(first)),
                        _p(dwa, _c_dp), ctypes.c_int32(int(want_solve)), ctypes.byref(eo))
    r["status"] = st
    r["dlognorm"] = float(r["dlognorm"][0])
    r["Nn"] = r["Nn"][:nch]
    r["bmean"] = r["bmean"][:nch]
    return r


def run(problem: Problem, kind: int, n_hidden: int, cfg: Config, theta0, n_traj: int, traj0: int = 0,
        n_threads: int = 1):
    """Integrate n_traj trajectories; returns (theta [n_traj, M], moments [n_traj, n_out, 9], status).

    ``status`` is 0 when every trajectory finished; the per-trajectory codes are kept in
    ``run.last_status``.  A failed trajectory's later moments are NaN.  For the linear SSE
    (cfg.linear) ``run.last_lognorm`` [n_traj, n_out] holds log Q at the output times."""
    m = n_params(kind, problem.n, n_hidden)
    n_out = cfg.n_steps // cfg.obs_every + 1 if cfg.obs_every > 0 else 0
    th = np.zeros((n_traj, m), np.complex128)
    obs = np.full((n_traj, max(n_out, 1), 9), np.nan)
    stat = np.zeros(n_traj, np.int32)
    a = _Ansatz(kind, n_hidden)
    t0 = _theta2(theta0)
    pc = problem._c()
    lq = np.zeros((n_traj, max(n_out, 1)))
    st = lib().orc_run(ctypes.byref(pc), ctypes.byref(a), ctypes.byref(cfg._c()), _p(t0, _c_dp),
                       ctypes.c_int32(n_traj), ctypes.c_int32(traj0), ctypes.c_int32(n_threads),
                       _p(th.view(np.float64), _c_dp), _p(obs, _c_dp), _p(stat, _c_i32p), _p(lq, _c_dp))
    run.last_status = stat
    run.last_lognorm = lq[:, :n_out]
    return th, obs[:, :n_out], st


def ensemble(moments: np.ndarray, n: int, weights=None):
    """Trajectory average (Eq. 3) of per-trajectory moments -> (M [3], C [3,3], xi^2).

    moments[..., :] = (mx, my, mz, sxx, syy, szz, sxy, sxz, syz) per trajectory, with
    s_ab = (1/2)<{M_a, M_b}>.  C_ab = avg s_ab - M_a M_b, so the spread between trajectories is
    part of C.  xi^2 = N min_perp Var(M_perp) / |M|^2 (observables paragraph of the LITF
    section): the smaller eigenvalue of C restricted to the plane orthogonal to M.
    weights [n_traj, ...] (the norms Q_j of the linear SSE): the weighted average of App. B,
    (1/N_T) sum_j <A>_j Q_j, in place of the plain mean."""
    mo = np.asarray(moments, dtype=np.float64)
    if weights is None:
        avg = mo.mean(axis=0)
    else:
        avg = (mo * np.asarray(weights, dtype=np.float64)[..., None]).mean(axis=0)
    M = avg[..., 0:3]
    s = np.zeros(avg.shape[:-1] + (3, 3))
    s[..., 0, 0], s[..., 1, 1], s[..., 2, 2] = avg[..., 3], avg[..., 4], avg[..., 5]
    s[..., 0, 1] = s[..., 1, 0] = avg[..., 6]
    s[..., 0, 2] = s[..., 2, 0] = avg[..., 7]
    s[..., 1, 2] = s[..., 2, 1] = avg[..., 8]
    C = s - M[..., :, None] * M[..., None, :]
    xi2 = squeezing(M, C, n)
    return M, C, xi2


def squeezing(M, C, n):
    M = np.asarray(M, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if M.ndim > 1:
        return np.array([squeezing(M[i], C[i], n) for i in range(M.shape[0])])
    norm = np.linalg.norm(M)
    u = M / norm
    # orthonormal basis of the plane perpendicular to M
    trial = np.eye(3)[np.argmin(np.abs(u))]
    e1 = trial - u * (u @ trial)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    P = np.stack([e1, e2])
    C2 = P @ C @ P.T
    return n * np.linalg.eigvalsh(C2)[0] / norm ** 2
