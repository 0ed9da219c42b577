"""Linear and eigen solvers of the Bloch-wave method (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* pcg            Algorithm "InvA" (Sec. 3.3): preconditioned conjugate gradient
                 on K(k) with the homogeneous-reference preconditioner, stopping
                 on the true residual ||K x - y|| <= TOL ||y|| (Euclidean norm of
                 the DFT coefficients; the paper leaves the norm open).
* subspace       Algorithm "subspace" (Sec. 3.3, Bathe's subspace iteration in
                 operator form); stops when both err1 and err2 are small.
* lanczos        shift-invert implicitly restarted Lanczos (Sec. 3.3): largest
                 beta of OP = K^-1 M in the M inner product, lambda = 1 / beta,
                 restarted with exact shifts.
* dense_modes    dense assembly + generalized Hermitian eigendecomposition
                 (the exact result the iterations converge to; tiny grids only).
* lowest_modes   per-k driver (Algorithm "Full algorithm") with the Gamma-point
                 deflation of the three rigid translations.

Readings of the paper that these functions take (ambiguities, silences):
  - the subspace loop stops only when err1 <= TOL and err2 <= 10 TOL;
  - err2 = max_p ||K U_p - lambda_p M U_p|| / (lambda_p ||M U_p||);
  - the cold start uses the lowest eigenvectors of the homogeneous reference
    medium (plane waves with the C0 acoustic-tensor polarizations);
  - at Gamma (some xi + k = 0) K is singular: the three constant translations
    are returned as omega = 0 and the rest is computed on their M-orthogonal
    complement;
  - the Lanczos operator is K^-1 M (so that the eigenvectors are shared with
    the original pencil for any rho(x)).
Pins: dense generalized eigendecomposition (LAPACK), homogeneous closed forms,
the laminate dispersion relation and the structural invariants
(tests/test_oracle_*.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operators import Operators, inner


# --------------------------------------------------------------------------
# Gamma-point deflation
# --------------------------------------------------------------------------
class Deflation:
    """M-orthogonal projector onto the complement of null(K) = rigid translations."""

    def __init__(self, ops: Operators):
        self.ops = ops
        idx = np.argwhere(ops.null_mask)
        self.active = idx.shape[0] > 0
        if not self.active:
            return
        j = tuple(idx[0])
        N = np.zeros((3, 3) + ops.n, dtype=np.complex128)
        for c in range(3):
            N[(c, c) + j] = 1.0
        self.N = N
        self.MN = ops.apply_M(N)
        G = np.einsum("ai,bi->ab", N.reshape(3, -1).conj(), self.MN.reshape(3, -1))
        self.Ginv = np.linalg.inv(G)
        # M-normalized rigid modes N G^-1/2
        w, V = np.linalg.eigh(G)
        S = V @ np.diag(w ** -0.5) @ V.conj().T
        self.modes = np.einsum("ab,b...->a...", S.T, N)

    def project(self, U: np.ndarray) -> np.ndarray:
        if not self.active:
            return U
        flat = U.reshape(1 if U.ndim == 4 else U.shape[0], -1)
        c = self.MN.reshape(3, -1).conj() @ flat.T                  # (3, batch): (M n)^H u
        corr = (self.Ginv @ c).T @ self.N.reshape(3, -1)
        return (flat - corr).reshape(U.shape)


# --------------------------------------------------------------------------
# PCG (Algorithm InvA)
# --------------------------------------------------------------------------
def pcg(ops: Operators, b: np.ndarray, tol: float, maxit: int = 5000, x0=None):
    """Solve K(k) x = b; returns (x, iterations, true relative residual)."""
    bn = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    if bn == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - ops.apply_K(x) if x0 is not None else b.copy()
    z = ops.precond(r)
    p = z.copy()
    rz = inner(r, z).real
    it = 0
    while it < maxit:
        if np.linalg.norm(r) <= tol * bn:
            rt = b - ops.apply_K(x)                                 # true residual check
            if np.linalg.norm(rt) <= tol * bn:
                break
            r = rt                                                  # residual replacement
            z = ops.precond(r)
            p = z.copy()
            rz = inner(r, z).real
        Ap = ops.apply_K(p)
        alpha = rz / inner(p, Ap).real
        x += alpha * p
        r -= alpha * Ap
        it += 1
        z = ops.precond(r)
        rz_new = inner(r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.linalg.norm(b - ops.apply_K(x)) / bn)


# --------------------------------------------------------------------------
# cold start: lowest plane waves of the homogeneous reference medium
# --------------------------------------------------------------------------
def reference_vectors(ops: Operators, count: int) -> np.ndarray:
    P = ops.acoustic_tensor(ops.C0) / ops.rho_bar                   # (N0,N1,N2,3,3)
    w, V = np.linalg.eigh(P.reshape(-1, 3, 3))
    qn = np.linalg.norm(ops.qvec.reshape(-1, 3), axis=1)
    nvox = qn.shape[0]
    lam = w.reshape(-1)
    vox = np.repeat(np.arange(nvox), 3)
    pol = np.tile(np.arange(3), nvox)
    keep = ~np.repeat(ops.null_mask.reshape(-1), 3)
    order = np.lexsort((pol[keep], vox[keep], qn[vox[keep]], lam[keep]))[:count]
    sel_v, sel_p = vox[keep][order], pol[keep][order]
    U = np.zeros((count, 3, nvox), dtype=np.complex128)
    for i, (v, p) in enumerate(zip(sel_v, sel_p)):
        U[i, :, v] = V[v, :, p]
    return U.reshape((count, 3) + ops.n)


# --------------------------------------------------------------------------
# small generalized Hermitian eigenproblem (library primitive)
# --------------------------------------------------------------------------
def small_geig(A: np.ndarray, B: np.ndarray):
    A = 0.5 * (A + A.conj().T)
    B = 0.5 * (B + B.conj().T)
    return sla.eigh(A, B)


def _gram(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """X^H Y for batches of vectors (q, 3, N0, N1, N2)."""
    return X.reshape(X.shape[0], -1).conj() @ Y.reshape(Y.shape[0], -1).T


# --------------------------------------------------------------------------
# subspace iteration (Algorithm "subspace")
# --------------------------------------------------------------------------
def subspace(ops: Operators, nmodes: int, block: int, tol_eig: float, tol_lin: float,
             U0=None, maxit: int = 200):
    """Lowest eigenpairs of K U = lambda M U on the complement of null(K).

    Returns (lam[nmodes'], U[block], info) where nmodes' = nmodes minus the
    rigid modes deflated at Gamma.
    """
    defl = Deflation(ops)
    n_want = nmodes - (3 if defl.active else 0)
    U = reference_vectors(ops, block) if U0 is None else U0.copy()
    U = defl.project(U)
    lam_old = None
    info = dict(outer=0, pcg_iters=0, err1=np.inf, err2=np.inf)
    for s in range(maxit):
        V = ops.apply_M(U)                                          # v_p = M U_p
        Ub = np.empty_like(U)
        for p in range(block):                                      # Ubar = K^-1 v
            Ub[p], it, _ = pcg(ops, V[p], tol_lin)
            info["pcg_iters"] += it
        Ub = defl.project(Ub)
        MUb = ops.apply_M(Ub)
        Kq = _gram(Ub, V)                                           # Ubar^H Kn
        Mq = _gram(Ub, MUb)                                         # Ubar^H Mn
        lam, Q = small_geig(Kq, Mq)
        U = np.einsum("pq,p...->q...", Q, Ub)                       # Ritz update
        info["outer"] = s + 1
        if lam_old is not None:
            info["err1"] = float(np.sqrt(np.sum((lam[:n_want] - lam_old[:n_want]) ** 2)
                                         / np.sum(lam_old[:n_want] ** 2)))
        KU = ops.apply_K(U[:n_want])
        MU = ops.apply_M(U[:n_want])
        res = [np.linalg.norm(KU[p] - lam[p] * MU[p]) / (lam[p] * np.linalg.norm(MU[p]))
               for p in range(n_want)]
        info["err2"] = float(max(res))
        lam_old = lam
        if info["err1"] <= tol_eig and info["err2"] <= 10.0 * tol_eig:
            break
    return lam[:n_want], U, info


# --------------------------------------------------------------------------
# shift-invert implicitly restarted Lanczos (Sec. 3.3)
# --------------------------------------------------------------------------
def lanczos(ops: Operators, nmodes: int, tol_eig: float, tol_lin: float, ncv=None,
            maxit: int = 300, v0=None):
    """Largest beta of OP = K^-1 M (M inner product) with exact-shift implicit restarts.

    Returns (lam[nmodes'], X[nmodes'], info) with lam = 1 / beta ascending.
    """
    defl = Deflation(ops)
    n_want = nmodes - (3 if defl.active else 0)
    m = ncv or max(2 * n_want + 1, 20)

    def mnorm(v):
        return np.sqrt(inner(v, ops.apply_M(v)).real)

    def op(v):
        x, it, _ = pcg(ops, ops.apply_M(v), tol_lin)
        info["pcg_iters"] += it
        return defl.project(x)

    info = dict(restarts=0, pcg_iters=0)
    if v0 is None:
        v0 = reference_vectors(ops, 1)[0] + 0.1 * reference_vectors(ops, 4).sum(axis=0)
    v = defl.project(v0[None])[0]
    V = np.zeros((m + 1,) + v.shape, dtype=np.complex128)
    V[0] = v / mnorm(v)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    f = None

    def extend(j0, f):
        # Lanczos steps j0..m-1 with full re-orthogonalization in the M inner product
        for j in range(j0, m):
            if j > 0:
                bj = mnorm(f)
                beta[j - 1] = bj
                V[j] = f / bj
            w = op(V[j])
            MV = ops.apply_M(V[:j + 1])
            alpha[j] = inner(MV[j], w).real                        # <v_j, w>_M
            f = w - alpha[j] * V[j] - (beta[j - 1] * V[j - 1] if j > 0 else 0.0)
            for _ in range(2):
                c = MV.reshape(j + 1, -1).conj() @ f.ravel()
                f = f - np.einsum("a,a...->...", c, V[:j + 1])
        return f

    f = extend(0, f)
    for it in range(maxit):
        T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
        theta, S = np.linalg.eigh(T)                                # ascending
        bm = mnorm(f)
        resid = np.abs(bm * S[m - 1, :])
        want = np.arange(m - n_want, m)
        if np.all(resid[want] <= tol_eig * np.abs(theta[want])):
            break
        info["restarts"] += 1
        # exact shifts: the unwanted Ritz values
        Qacc = np.eye(m)
        for mu in theta[:m - n_want]:
            Qs, Rs = np.linalg.qr(T - mu * np.eye(m))
            T = Rs @ Qs + mu * np.eye(m)
            Qacc = Qacc @ Qs
        k = n_want
        Vnew = np.einsum("ji,j...->i...", Qacc[:, :k + 1], V[:m])
        f = Vnew[k] * T[k, k - 1] + f * Qacc[m - 1, k - 1]
        V[:k] = Vnew[:k]
        alpha[:k] = np.diag(T)[:k]
        beta[:k - 1] = np.diag(T, -1)[:k - 1]
        f = extend(k, f)
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    theta, S = np.linalg.eigh(T)
    sel = np.arange(m - 1, m - 1 - n_want, -1)                      # largest beta first
    X = np.einsum("ji,j...->i...", S[:, sel], V[:m])
    return 1.0 / theta[sel], X, info


# --------------------------------------------------------------------------
# dense reference and the per-k driver
# --------------------------------------------------------------------------
def dense_modes(ops: Operators, nmodes: int):
    """Exact lowest eigenpairs of the pencil (K, M) by dense assembly (tiny grids)."""
    K = ops.dense("K")
    M = ops.dense("M")
    w, X = sla.eigh(0.5 * (K + K.conj().T), 0.5 * (M + M.conj().T),
                    subset_by_index=[0, nmodes - 1])
    return w, X.T.reshape((nmodes, 3) + ops.n)


def lowest_modes(rve, k_list, nmodes: int, method: str = "subspace", block=None,
                 tol_eig: float = 1e-12, tol_lin: float = 1e-12, dense_max: int = 3072,
                 warm_start: bool = True, stats=None):
    """omega (rad/s) of the lowest nmodes branches at every k (Algorithm "Full algorithm").

    Uses the dense pencil when 3 N^3 <= dense_max, else the chosen iteration.
    If `stats` is a list, one dict of iteration counts per k is appended to it.
    """
    nvox = int(np.prod(rve.n))
    block = block or min(2 * nmodes, nmodes + 8)
    out = np.zeros((len(k_list), nmodes))
    U_prev = None
    for r, k in enumerate(k_list):
        ops = Operators(rve, k)
        if 3 * nvox <= dense_max or method == "dense":
            lam, _ = dense_modes(ops, nmodes)
            lam = np.sort(lam)
            if Deflation(ops).active:
                # the rigid translations are exact zeros (dense eigh returns O(eps) values)
                assert np.all(np.abs(lam[:3]) <= 1e-10 * max(lam[-1], 1.0))
                lam[:3] = 0.0
        else:
            defl = Deflation(ops)
            if method == "subspace":
                lam, U, info = subspace(ops, nmodes, block, tol_eig, tol_lin,
                                        U0=U_prev if warm_start else None)
                U_prev = U
            else:
                lam, _, info = lanczos(ops, nmodes, tol_eig, tol_lin)
            if stats is not None:
                stats.append(dict(info))
            if defl.active:
                lam = np.concatenate([np.zeros(3), lam])
        out[r] = np.sqrt(np.maximum(lam[:nmodes], 0.0))
    return out
