"""Group velocity and long-wave speeds of the dispersion branches (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* dK_dk            derivative of K(k) along a direction d, written out from eq.
                   hatA: K depends on k only through the shifted frequencies
                   q = xi + k, through the strain B(q) and the divergence
                   B(q)^H, so dK/ds U = B(d)^H F C F^-1 B(q) U + B(q)^H F C F^-1 B(d) U
                   with B(v) the Voigt strain operator of a constant vector v.
* branch_slopes    group velocity (Sec. 5.1, eq. c_group) d omega / ds along d.
                   omega^2 is the eigenvalue of the pencil (K, M) and M does not
                   depend on k, so for a simple eigenvalue
                   d omega^2 / ds = U^H dK/ds U / U^H M U (first-order
                   perturbation); within a cluster of equal omega the slopes are
                   the eigenvalues of the pencil (U^H dK U, U^H M U) on the
                   cluster, each divided by 2 omega.
* long_wave_speeds the three acoustic branches' omega / |k| at k = +-h d and +-2h d
                   extrapolated to k -> 0.  The mean over +-k of omega^2 is even and
                   analytic in k, so it gives c + O(k^2) and (4 c(h) - c(2h)) / 3 =
                   c + O(h^4);
                   the long-wave limit is the speed of the equivalent homogeneous
                   medium (Sec. 5.1, the limit of d omega / dk for k -> 0).
* mode_fields      real-space fields of modes (Sec. 5.2, eigenvectors, eq.
                   rotate_eigenvector): u = e^{-i phi} F^-1 U^ with phi = arg(sum u.u)/2
                   (the phase that brings the field closest to real; the paper's common
                   phase when there is one), and the strain of the Bloch wave divided by
                   e^{i k.x}: e^{-i phi} F^-1[i B(xi + k) U^].
* effective_stiffness  static homogenization on the same discretization (the
                   long-wave limit of the Bloch problem): for each of the six unit
                   macro strains E, the periodic displacement solves
                   K(0) U^ = i B(xi)^H F[C(x) E] (equilibrium of C (E + eps(u)), the
                   factors i of the gradient kept: eps(u) = F^-1[i B(xi) U^]) by PCG
                   (Algorithm "InvA"), and the column of C_eff is the volume mean of
                   C(x) (E + eps(u)).  rho_bar c^2 of the long-wave speeds are then the
                   Christoffel eigenvalues of C_eff.
* voigt_reuss_bracket  Christoffel eigenvalues of the Voigt (mean stiffness) and
                   Reuss (inverse mean compliance) averages, which bound rho_bar c^2
                   of the long-wave limit from above and below.

Pins (tests/test_oracle_postproc.py): homogeneous isotropic and cubic closed
forms, including a folded branch omega = c |k + G|; central differences of
exact (dense) eigenvalues; the laminate's exact quasi-static moduli along its
normal (the Reuss averages of the P-wave and shear moduli); the Voigt/Reuss
bracket for a polycrystal; exact long-wave speeds along the axis of fibre
textures; the 1D polycrystal's matrix harmonic mean; for mode_fields, a real
field rotated by a known phase and the analytic strain of a trigonometric
displacement; for effective_stiffness, a homogeneous medium, Backus averages of
a laminate, Voigt/Reuss bounds as quadratic forms and the Christoffel
eigenvalues against the long-wave speeds of the eigen-solver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fourier import fft3, ifft3
from .operators import Operators
from .solvers import lowest_modes, pcg
from .voigt import voigt_to_tensor


def _strain_const(d, U):
    """Voigt strain (engineering shear) of U with the constant vector d in place of q."""
    U1, U2, U3 = U[..., 0, :, :, :], U[..., 1, :, :, :], U[..., 2, :, :, :]
    return np.stack([d[0] * U1, d[1] * U2, d[2] * U3,
                     d[2] * U2 + d[1] * U3, d[2] * U1 + d[0] * U3, d[1] * U1 + d[0] * U2], axis=-4)


def _div_const(d, S):
    """Divergence of the Voigt stress S with the constant vector d in place of q."""
    s11, s22, s33, s23, s13, s12 = (S[..., i, :, :, :] for i in range(6))
    return np.stack([d[0] * s11 + d[1] * s12 + d[2] * s13,
                     d[0] * s12 + d[1] * s22 + d[2] * s23,
                     d[0] * s13 + d[1] * s23 + d[2] * s33], axis=-4)


def _stress_hat(ops: Operators, E_hat):
    """F C(x) F^-1 applied to a Fourier-space Voigt strain field."""
    e = ifft3(E_hat)
    E = e.reshape(e.shape[:-3] + (-1,))
    S = np.empty_like(E)
    for gi, idx in ops.grain_voxels:
        if idx.size:
            S[..., idx] = ops.C6[gi] @ E[..., idx]
    return fft3(S.reshape(e.shape))


def dK_dk(ops: Operators, d, U):
    """(d/ds) K(k + s d) U at s = 0."""
    d = np.asarray(d, dtype=np.float64)
    return (_div_const(d, _stress_hat(ops, ops.strain(U)))
            + ops.divergence(_stress_hat(ops, _strain_const(d, U))))


def clusters(omega, tol):
    """Index groups of consecutive (ascending) omega within a relative gap tol."""
    groups, cur = [], [0]
    for p in range(1, len(omega)):
        if omega[p] - omega[p - 1] <= tol * max(omega[p], 1e-300):
            cur.append(p)
        else:
            groups.append(cur)
            cur = [p]
    groups.append(cur)
    return groups


def branch_slopes(rve, k, d, U, omega, cluster_tol=1e-6):
    """d omega / ds along the unit direction d at k for the modes U (nmodes, 3, N0, N1, N2)
    with frequencies omega (ascending); 0 for omega = 0 (rigid translations at Gamma)."""
    d = np.asarray(d, dtype=np.float64) / np.linalg.norm(d)
    ops = Operators(rve, k)
    nm = U.shape[0]
    flat = U.reshape(nm, -1)
    D = flat.conj() @ dK_dk(ops, d, U).reshape(nm, -1).T
    G = flat.conj() @ ops.apply_M(U).reshape(nm, -1).T
    D = 0.5 * (D + D.conj().T)
    G = 0.5 * (G + G.conj().T)
    out = np.zeros(nm)
    for c in clusters(np.asarray(omega, dtype=np.float64), cluster_tol):
        w = float(np.mean(np.asarray(omega)[c]))
        if w == 0.0:
            continue
        lam = sla.eigh(D[np.ix_(c, c)], G[np.ix_(c, c)], eigvals_only=True)
        out[c] = np.sort(lam) / (2.0 * w)
    return out


def long_wave_speeds(rve, d, h_frac=0.02, **kw):
    """The three acoustic long-wave speeds (ascending) along the unit direction d;
    h = h_frac pi / max(L).  omega / |k| is averaged over k and -k: on an even grid the
    frequency set is not symmetric (the Nyquist label -N/2 has no +N/2), so omega(k) and
    omega(-k) differ at O(|k|) and only their mean is even in k.  Keyword arguments go to
    solvers.lowest_modes."""
    d = np.asarray(d, dtype=np.float64) / np.linalg.norm(d)
    h = h_frac * np.pi / max(rve.L)
    w = lowest_modes(rve, [h * d, -h * d, 2 * h * d, -2 * h * d], 3, **kw)
    c1 = (np.sort(w[0]) + np.sort(w[1])) / (2 * h)
    c2 = (np.sort(w[2]) + np.sort(w[3])) / (4 * h)
    return (4 * c1 - c2) / 3


def voigt_reuss_bracket(rve, d):
    """(lower, upper) bounds on rho_bar c^2 of the three long-wave branches along d:
    sorted Christoffel eigenvalues of the Reuss and the Voigt averages."""
    d = np.asarray(d, dtype=np.float64) / np.linalg.norm(d)
    ops = Operators(rve, np.zeros(3))
    C = ops.C_field.reshape(-1, 6, 6)
    CV = C.mean(axis=0)
    CR = np.linalg.inv(np.linalg.inv(C).mean(axis=0))
    def christoffel(C6):
        T = voigt_to_tensor(C6)
        return np.sort(np.linalg.eigvalsh(np.einsum("ijkl,j,l->ik", T, d, d)))
    return christoffel(CR), christoffel(CV)


def mode_fields(rve, k, U):
    """(u, eps, phi) of the modes U (nmodes, 3, N0, N1, N2): displacement and Voigt strain
    (engineering shear) in real space, rotated by e^{-i phi}."""
    ops = Operators(rve, k)
    u = ifft3(U)
    phi = 0.5 * np.angle(np.sum(u * u, axis=(-4, -3, -2, -1)))
    rot = np.exp(-1j * phi)[..., None, None, None, None]
    eps = ifft3(1j * ops.strain(U))
    return u * rot, eps * rot, phi


def effective_stiffness(rve, tol=1e-12):
    """6 x 6 Voigt effective stiffness (engineering shear) by static homogenization."""
    ops = Operators(rve, np.zeros(3))
    n = ops.n
    Cf = ops.C_field                                               # (N0, N1, N2, 6, 6)
    Ceff = np.zeros((6, 6))
    for j in range(6):
        E = np.zeros(6)
        E[j] = 1.0
        s0 = np.moveaxis(Cf @ E, -1, 0).astype(np.complex128)      # (6, N0, N1, N2), C(x) E
        b = 1j * ops.divergence(fft3(s0))
        u, _, _ = pcg(ops, b, tol)
        eps = ifft3(1j * ops.strain(u))                            # (6, N0, N1, N2)
        # on an even grid the fluctuation is not real (the Nyquist label -N/2 has no +N/2);
        # the physical tensor is the real part of the mean stress
        tot = np.moveaxis(eps.real, 0, -1) + E
        sig = np.einsum("xyzab,xyzb->xyza", Cf, tot)
        Ceff[:, j] = sig.reshape(-1, 6).mean(axis=0)
    return 0.5 * (Ceff + Ceff.T)
