"""ORACLE -- exact references (test infrastructure, not product code).

Dense / sparse state-space references for small N, written from the paper:
  * the Lindblad master equation, Eq. 1, integrated exactly (matrix exponential action of
    the Liouvillian, scipy's ``expm_multiply``) or with classical RK4 as a cross-check;
  * the nonlinear Ito SSE, Eq. 2, with Euler-Maruyama;
  * its Stratonovich form, Eqs. 4-5, with the trapezoidal and midpoint predictor-correctors
    of App. C;
  * dense-algebra S, F, N^n (definitions after Eq. 8) from derivative vectors of psi;
  * the closed form of App. D for the LITF without transverse field, as printed for the
    periodic chain, and its site-resolved form for arbitrary couplings J_ij;
  * a second, vectorised statement of the SNR-regularised solve (the regulariser named after
    Eq. 9, in the reading the C oracle also takes) from per-sample O_k(x) and G(x), with LAPACK's
    eigen-decomposition, so that the C oracle's Jacobi-based form can be checked against it.
Basis convention: configuration index x, bit i of x set <=> sigma_i = +1 (spin up).
Only tests and the benchmark's CPU-baseline leg import this module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

SIGMA_MINUS, SIGMA_PLUS, SIGMA_Z = 0, 1, 2


# ------------------------------------------------------------------ operators
def spins(n):
    """s[x, i] = +-1 for every configuration x."""
    x = np.arange(1 << n)
    return np.where((x[:, None] >> np.arange(n)[None, :]) & 1, 1, -1).astype(np.int8)


def op(n, name, i):
    """Sparse single-site operator on site i: 'x', 'y', 'z', 'm' (sigma^-), 'p' (sigma^+)."""
    d = 1 << n
    x = np.arange(d)
    up = ((x >> i) & 1).astype(bool)
    s = np.where(up, 1.0, -1.0)
    y = x ^ (1 << i)
    if name == "z":
        return sp.csr_matrix((s.astype(np.complex128), (x, x)), shape=(d, d))
    if name == "x":
        return sp.csr_matrix((np.ones(d, np.complex128), (y, x)), shape=(d, d))
    if name == "y":   # <y|sigma^y|x> with y = x flipped: +i if x is up, -i if down
        return sp.csr_matrix((1j * s, (y, x)), shape=(d, d))
    if name == "m":   # |down><up|
        return sp.csr_matrix((np.ones(up.sum(), np.complex128), (y[up], x[up])), shape=(d, d))
    if name == "p":   # |up><down|
        return sp.csr_matrix((np.ones((~up).sum(), np.complex128), (y[~up], x[~up])), shape=(d, d))
    raise ValueError(name)


def hamiltonian(J, hx):
    """H = sum_{i<j} J_ij sz_i sz_j + hx sum_i sx_i (sparse)."""
    n = J.shape[0]
    s = spins(n).astype(np.float64)
    diag = 0.5 * np.einsum("xi,ij,xj->x", s, J, s)   # J symmetric with zero diagonal
    H = sp.diags(diag.astype(np.complex128))
    for i in range(n):
        H = H + hx * op(n, "x", i)
    return sp.csr_matrix(H)


def jump_ops(n, jumps):
    out = []
    for kind, site, rate in jumps:
        name = {SIGMA_MINUS: "m", SIGMA_PLUS: "p", SIGMA_Z: "z"}[kind]
        out.append(np.sqrt(rate) * op(n, name, site))
    return out


def collective(n):
    """Sparse M_a = (1/N) sum_i sigma^a_i for a = x, y, z."""
    return [sum(op(n, a, i) for i in range(n)) / n for a in "xyz"]


# ------------------------------------------------------------------ Lindblad (Eq. 1)
def liouvillian(H, Ls):
    """Superoperator acting on vec(rho) (row-major): drho = -i[H,rho] + sum L rho L^+ - {L^+L,rho}/2."""
    d = H.shape[0]
    I = sp.identity(d, dtype=np.complex128, format="csr")
    # row-major vec: vec(A rho B) = (A kron B^T) vec(rho)
    Lv = -1j * (sp.kron(H, I) - sp.kron(I, H.T))
    for L in Ls:
        LdL = (L.conj().T @ L).tocsr()
        Lv = Lv + sp.kron(L, L.conj()) - 0.5 * (sp.kron(LdL, I) + sp.kron(I, LdL.T))
    return sp.csr_matrix(Lv)


def product_state_x(n):
    """Coherent spin state along +x: every amplitude 2^{-N/2}."""
    return np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)


def lindblad_evolve(J, hx, jumps, times, psi0=None):
    """rho(t) = exp(t Lv) rho(0) at the requested times (list of d x d arrays)."""
    n = J.shape[0]
    H = hamiltonian(J, hx)
    Lv = liouvillian(H, jump_ops(n, jumps))
    psi = product_state_x(n) if psi0 is None else np.asarray(psi0, np.complex128)
    rho0 = np.outer(psi, psi.conj()).reshape(-1)
    times = np.asarray(times, dtype=np.float64)
    out = []
    for t in times:
        v = expm_multiply(Lv * t, rho0) if t != 0 else rho0.copy()
        out.append(v.reshape(psi.size, psi.size))
    return out


def lindblad_rk4(J, hx, jumps, t_end, dt, psi0=None):
    """Classical RK4 on Eq. 1 (cross-check of the matrix-exponential integration)."""
    n = J.shape[0]
    Lv = liouvillian(hamiltonian(J, hx), jump_ops(n, jumps))
    psi = product_state_x(n) if psi0 is None else np.asarray(psi0, np.complex128)
    v = np.outer(psi, psi.conj()).reshape(-1)
    steps = int(round(t_end / dt))
    for _ in range(steps):
        k1 = Lv @ v
        k2 = Lv @ (v + 0.5 * dt * k1)
        k3 = Lv @ (v + 0.5 * dt * k2)
        k4 = Lv @ (v + dt * k3)
        v = v + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return v.reshape(psi.size, psi.size)


def rho_observables(rho, n):
    """(M [3], C [3,3]) of a density matrix: M_a = Tr(rho M_a), C_ab = (1/2)<{M_a,M_b}> - M_a M_b."""
    Ms = collective(n)
    M = np.array([np.real(np.sum(rho * A.T.toarray())) for A in Ms])
    C = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            A = (0.5 * (Ms[a] @ Ms[b] + Ms[b] @ Ms[a])).toarray()
            C[a, b] = np.real(np.sum(rho * A.T)) - M[a] * M[b]
    return M, C


def psi_observables(psi, n):
    """Per-trajectory moments (mx,my,mz,sxx,syy,szz,sxy,sxz,syz) of a state vector."""
    psi = psi / np.linalg.norm(psi)
    rho = np.outer(psi, psi.conj())
    M, C = rho_observables(rho, n)
    s = C + np.outer(M, M)
    return np.array([M[0], M[1], M[2], s[0, 0], s[1, 1], s[2, 2], s[0, 1], s[0, 2], s[1, 2]])


# ------------------------------------------------------------------ App. D closed form
def _sinc(z):
    z = np.asarray(z, dtype=np.complex128)
    safe = np.where(z == 0, 1.0, z)
    return np.where(z == 0, 1.0, np.sin(safe) / safe)


# App. D writes sin(z)/(2a + i Gamma) with z = (2a + i Gamma) t; as t * sin(z)/z it has no
# removable 0/0 at a = Gamma = 0.
def _phi(a, t, G):
    z = 2 * a * t + 1j * G * t
    return np.exp(-G * t) * (np.cos(z) + G * t * _sinc(z))


def _psi_aux(a, t, G):
    z = 2 * a * t + 1j * G * t
    return 2 * np.exp(-G * t) * (-G + 1j * a) * t * _sinc(z)


def _assemble(M, Qpz, Qmz, Qpp, Qmp, Qpm, n):
    Mx, My, Mz = M
    C = np.zeros((3, 3))
    C[0, 0] = 1 / n + np.real(2 * Qpp + Qmp + Qpm) - Mx ** 2
    C[1, 1] = 1 / n + np.real(-2 * Qpp + Qmp + Qpm) - My ** 2
    C[0, 1] = C[1, 0] = 2 * np.imag(Qpp) - Mx * My
    C[0, 2] = C[2, 0] = np.real(Qpz + Qmz) - Mx * Mz
    C[1, 2] = C[2, 1] = np.imag(Qpz - Qmz) - My * Mz
    C[2, 2] = (1 / n) * (1 - Mz ** 2)
    return C


def appd_pbc(n, alpha, jscale, kappa, t):
    """App. D as printed: translation-invariant couplings J_d = (J/K) d^-alpha for 0<d<N/2,
    J_d = J_{N-d} for d >= N/2 (a single bond at d = N/2), J_0 = 0; Gamma = kappa/2.
    Returns (M [3], C [3,3])."""
    d = np.arange(n)
    dist = np.minimum(d, n - d).astype(np.float64)
    with np.errstate(divide="ignore"):
        w = np.where(dist > 0, dist ** (-alpha), 0.0)
    kac = sum(min(abs(i - j), n - abs(i - j)) ** (-alpha) for i in range(n) for j in range(i + 1, n)) / (n - 1)
    Jd = jscale * w / kac
    G = kappa / 2.0

    def Phi(a):
        return _phi(a, t, G)

    Phip = np.prod(Phi(Jd))
    Phim = np.prod(Phi(-Jd))

    def Qz(mu):
        Ph = Phip if mu > 0 else Phim
        return np.exp(-G * t) / (2 * n) * Ph * sum(_psi_aux(mu * Jd[k], t, G) / Phi(mu * Jd[k]) for k in range(1, n))

    def Qmn(mu, nu):
        tot = 0.0
        for D in range(1, n):
            prod = np.prod([Phi(mu * Jd[k] + nu * Jd[(D - k) % n]) for k in range(n)])
            tot = tot + prod / (Phi(mu * Jd[D]) * Phi(nu * Jd[D]))
        return np.exp(-2 * G * t) / (4 * n) * tot

    M = np.array([np.exp(-G * t) * np.real(Phip), np.exp(-G * t) * np.imag(Phip), np.exp(-2 * G * t) - 1])
    C = _assemble(M, Qz(1), Qz(-1), Qmn(1, 1), Qmn(-1, 1), Qmn(1, -1), n)
    return M, C


def appd_general(J, kappa, t):
    """Site-resolved form of App. D for arbitrary symmetric couplings J_ij (H = +sum_{i<j}
    J_ij sz_i sz_j, h = 0, decay on every site, +x initial state).  For translation-invariant
    couplings it reduces term by term to the printed periodic-chain formulas."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    G = kappa / 2.0

    def Phi(a):
        return _phi(a, t, G)

    mask = ~np.eye(n, dtype=bool)
    Pp = np.array([np.prod(Phi(J[i][mask[i]])) for i in range(n)])
    Pm = np.array([np.prod(Phi(-J[i][mask[i]])) for i in range(n)])
    Mxy = np.exp(-G * t) / n * Pp.sum()
    M = np.array([np.real(Mxy), np.imag(Mxy), np.exp(-2 * G * t) - 1])

    def Qz(mu):
        P = Pp if mu > 0 else Pm
        tot = 0.0
        for i in range(n):
            a = mu * J[i][mask[i]]
            tot += P[i] * np.sum(_psi_aux(a, t, G) / Phi(a))
        return np.exp(-G * t) / (2 * n * n) * tot

    def Qmn(mu, nu):
        tot = 0.0
        for i in range(n):
            for k in range(n):
                if i == k:
                    continue
                js = [j for j in range(n) if j != i and j != k]
                tot += np.prod(Phi(mu * J[i, js] + nu * J[k, js]))
        return np.exp(-2 * G * t) / (4 * n * n) * tot

    C = _assemble(M, Qz(1), Qz(-1), Qmn(1, 1), Qmn(-1, 1), Qmn(1, -1), n)
    return M, C


def xi2(M, C, n):
    norm = np.linalg.norm(M)
    u = M / norm
    trial = np.eye(3)[np.argmin(np.abs(u))]
    e1 = trial - u * (u @ trial)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    P = np.stack([e1, e2])
    return n * np.linalg.eigvalsh(P @ C @ P.T)[0] / norm ** 2


# ------------------------------------------------------------------ state-vector SSE
def _expect(psi, A):
    return np.vdot(psi, A @ psi) / np.vdot(psi, psi)


def sse_ito_drift_diff(psi, H, Ls):
    """Drift and diffusion vectors of the nonlinear Ito SSE, Eq. 2."""
    a = -1j * (H @ psi)
    bs = []
    for L in Ls:
        c = 2.0 * np.real(_expect(psi, L))          # <L + L^dag>
        Lp = L @ psi
        a = a - 0.5 * ((L.conj().T @ Lp) - c * Lp + 0.25 * c * c * psi)
        bs.append(Lp - 0.5 * c * psi)
    return a, bs


def sse_strat_drift_diff(psi, H, Ls):
    """Drift -i H_eff^Strat psi (Eq. 5, with its c-number terms) and the diffusion of Eq. 4."""
    a = -1j * (H @ psi)
    bs = []
    for L in Ls:
        Ld = L.conj().T
        c = 2.0 * np.real(_expect(psi, L))
        Lp = L @ psi
        LdL = Ld @ Lp
        L2 = L @ Lp
        cnum = c * c - 0.5 * _expect(psi, L @ L + 2 * (Ld @ L) + Ld @ Ld)
        a = a - 0.5 * (LdL - 2 * c * Lp + L2 + cnum * psi)
        bs.append(Lp - 0.5 * c * psi)
    return a, bs


def sse_lin_ito_drift_diff(psi, H, Ls):
    """Drift and diffusion of the linear Ito SSE (App. B): no expectation values anywhere."""
    a = -1j * (H @ psi)
    bs = []
    for L in Ls:
        Lp = L @ psi
        a = a - 0.5 * (L.conj().T @ Lp)
        bs.append(Lp)
    return a, bs


def sse_lin_strat_drift_diff(psi, H, Ls):
    """Drift -i H_eff^{Strat,lin} psi and diffusion L psi of the linear Stratonovich SSE (App. B)."""
    a = -1j * (H @ psi)
    bs = []
    for L in Ls:
        Lp = L @ psi
        a = a - 0.5 * (L.conj().T @ Lp + L @ Lp)
        bs.append(Lp)
    return a, bs


def sse_path(psi0, H, Ls, dws, dt, scheme="heun", linear=False):
    """Integrate one trajectory given the Wiener increments dws[step, channel].

    scheme: 'ito_em' (Euler-Maruyama on the Ito form), 'heun' (trapezoidal predictor-corrector
    on the Stratonovich form), 'midpoint' (midpoint predictor-corrector on the Stratonovich
    form), 'strat_em' (Euler on the Stratonovich form, not Stratonovich-consistent).
    linear=False: the nonlinear SSE (Ito Eq. 2, Stratonovich Eqs. 4-5); linear=True: the
    linear SSE of App. B, whose paths do not keep their norm."""
    ito = sse_lin_ito_drift_diff if linear else sse_ito_drift_diff
    strat = sse_lin_strat_drift_diff if linear else sse_strat_drift_diff
    psi = np.array(psi0, dtype=np.complex128)
    out = [psi.copy()]
    for dw in dws:
        if scheme == "ito_em":
            a, bs = ito(psi, H, Ls)
            psi = psi + a * dt + sum(b * w for b, w in zip(bs, dw))
        else:
            a, bs = strat(psi, H, Ls)
            inc0 = a * dt + sum(b * w for b, w in zip(bs, dw))
            if scheme == "strat_em":
                psi = psi + inc0
            elif scheme == "heun":
                pb = psi + inc0
                a1, b1 = strat(pb, H, Ls)
                psi = psi + 0.5 * (inc0 + a1 * dt + sum(b * w for b, w in zip(b1, dw)))
            elif scheme == "midpoint":
                pm = psi + 0.5 * inc0
                a1, b1 = strat(pm, H, Ls)
                psi = psi + a1 * dt + sum(b * w for b, w in zip(b1, dw))
            else:
                raise ValueError(scheme)
        out.append(psi.copy())
    return out


# ------------------------------------------------------------------ dense otVMC algebra
def dense_sfn(psi_fn, theta, J, hx, jumps, h=1e-6):
    """S, F, N^n and <B^n> from dense vectors (definitions after Eq. 8), independent of any
    local-estimator code: d_k psi by central differences of psi(theta) along theta_k (psi is
    holomorphic in theta), H_eff^Strat of Eq. 5 as an explicit matrix with exact <L+L^dag>."""
    n = J.shape[0]
    theta = np.asarray(theta, dtype=np.complex128)
    psi = psi_fn(theta)
    nrm = np.vdot(psi, psi).real
    m = theta.size
    dpsi = np.zeros((m, psi.size), np.complex128)
    for k in range(m):
        e = np.zeros(m, np.complex128)
        e[k] = h
        dpsi[k] = (psi_fn(theta + e) - psi_fn(theta - e)) / (2 * h)
    H = hamiltonian(J, hx)
    Ls = jump_ops(n, jumps)
    Heff = H.copy().astype(np.complex128)
    for L in Ls:
        Ld = L.conj().T
        c = 2.0 * np.real(_expect(psi, L))
        Heff = Heff - 0.5j * (Ld @ L - 2 * c * L + L @ L)
    ob = dpsi.conj() @ psi / nrm                       # <O_k^*> = <d_k psi|psi>/<psi|psi>
    S = (dpsi.conj() @ dpsi.T) / nrm - np.outer(ob, ob.conj())
    Hp = Heff @ psi
    F = dpsi.conj() @ Hp / nrm - ob * (np.vdot(psi, Hp) / nrm)
    Nn, bm = [], []
    for L in Ls:
        Lp = L @ psi
        bmean = np.vdot(psi, Lp) / nrm
        Nn.append(dpsi.conj() @ Lp / nrm - ob * bmean)
        bm.append(bmean)
    return S, F, np.array(Nn).reshape(len(Ls), m), np.array(bm)


def jastrow_psi(n):
    """psi_theta(x) of Eq. 12 as a vector over all configurations (for dense tests)."""
    s = spins(n).astype(np.float64)
    pairs = [(j, k) for j in range(n) for k in range(j + 1, n)]
    feats = np.concatenate([s, np.stack([s[:, j] * s[:, k] for j, k in pairs], axis=1)
                            if pairs else np.zeros((s.shape[0], 0))], axis=1)

    def f(theta):
        return np.exp(feats @ np.asarray(theta))
    return f


def ljph_features(n, d):
    """Features of the LJPHd ansatz (LITF section) as columns [s_i | own pairs | distances]:
    pairs (j, k), j < k, k - j <= d in row-major order, then for each distance D > d the sum of
    s_j s_{j+D} over the open chain."""
    s = spins(n).astype(np.float64)
    cols = [s[:, i] for i in range(n)]
    cols += [s[:, j] * s[:, k] for j in range(n) for k in range(j + 1, n) if k - j <= d]
    cols += [sum(s[:, j] * s[:, j + D] for j in range(n - D)) for D in range(d + 1, n)]
    return np.stack(cols, axis=1)


def ljph_psi(n, d):
    """psi_theta(x) of LJPHd as a vector over all configurations."""
    feats = ljph_features(n, d)

    def f(theta):
        return np.exp(feats @ np.asarray(theta))
    return f


def rbm_psi(n, nh):
    """psi_theta(x) of Eq. 11 as a vector over all configurations."""
    s = spins(n).astype(np.float64)

    def f(theta):
        theta = np.asarray(theta)
        a, b, w = theta[:n], theta[n:n + nh], theta[n + nh:].reshape(n, nh)
        g = b[None, :] + s @ w
        return np.exp(s @ a) * np.prod(2 * np.cosh(g), axis=1)
    return f


# ------------------------------------------------------------------ SNR-regularised solve
def snr_solve(O, G, eps, tau, weights=None, cut=1e-14, hermitian=None):
    """delta of the SNR-filtered solve of (S + eps I) delta = D from per-sample log-derivatives
    O [ns, M] and G(x) = -i dt E_eff(x) + sum_n B^n(x) dW_n [ns] (weights: normalised
    |psi|^2 weights in place of the sample mean).  The filter (text after Eq. 9, with the form
    of the scheme the paper cites): with S + eps I = V diag(lam) V^H,
      rho = V^H D,  u_k(x) = sum_l V_lk (O_l(x) - <O_l>),  q_k(x) = conj(u_k(x)) (G(x) - <G>),
      SNR_k = |rho_k| sqrt(ns) / sqrt(<|q_k|^2> - |rho_k|^2)   (<q_k> = rho_k),
      delta = sum_k V_k rho_k / lam_k / (1 + (tau / SNR_k)^6),  lam_k <= cut * lam_max dropped.
    Real O (the Jastrow ansaetze) gives a real symmetric S.  Returns (delta, lam, snr, S, D), the
    eigenvalues ascending."""
    O = np.asarray(O)
    G = np.asarray(G, dtype=np.complex128)
    ns, m = O.shape
    if hermitian is None:
        hermitian = np.iscomplexobj(O) and np.abs(O.imag).max() > 0
    if not hermitian:
        O = O.real.astype(np.float64)
    w = np.full(ns, 1.0 / ns) if weights is None else np.asarray(weights, np.float64) / np.sum(weights)
    Oc = O - w @ O
    Gc = G - w @ G
    S = (Oc.conj() * w[:, None]).T @ Oc
    D = (Oc.conj() * w[:, None]).T @ Gc
    lam, V = np.linalg.eigh(S + eps * np.eye(m))
    rho = V.conj().T @ D
    u = Oc @ V
    q = u.conj() * Gc[:, None]
    var = w @ np.abs(q) ** 2 - np.abs(rho) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        snr = np.where(var > 0, np.abs(rho) * np.sqrt(ns) / np.sqrt(np.maximum(var, 1e-300)), np.inf)
        keep = np.where((lam > cut * lam.max()) & (np.abs(rho) > 0), 1.0 / (1.0 + (tau / snr) ** 6), 0.0)
    delta = V @ (keep * rho / lam)
    return delta, lam, snr, S, D
