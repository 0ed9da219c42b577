"""Pins of the oracle's solvers: PCG (Algorithm InvA), subspace iteration
(Algorithm subspace), shift-invert IRL (Sec. 3.3), Gamma deflation, and the
1D closed forms of Secs. 2.1 (eq. disp_homo) and 4.2 (eq. laminate, with the
sign of the sine term taken as minus: the printed plus sign fails the
homogeneous limit p = 1, where the relation must reduce to cos kL = cos(omega L / c))."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import brentq

from paper_2106_12487_amd import inputs
from oracle.operators import Operators
from oracle import solvers

L = 1e-3


def _poly(n, grains=5, idx=0, cfg=99):
    return inputs.polycrystal((n, n, n), (L, L, L), grains, cfg, idx)


def test_pcg_matches_dense_solve():
    ops = Operators(_poly(4), np.array([0.2, 0.1, 0.05]) * np.pi / L)
    rng = np.random.default_rng(0)
    b = rng.standard_normal((3, 4, 4, 4)) + 1j * rng.standard_normal((3, 4, 4, 4))
    x, it, rel = solvers.pcg(ops, b, 1e-12)
    xd = np.linalg.solve(ops.dense("K"), b.ravel()).reshape(b.shape)
    assert rel <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    # the preconditioner matters: plain CG (identity preconditioner) needs more iterations
    assert it < 200


def test_pcg_at_gamma_stays_in_range():
    ops = Operators(_poly(4), [0.0, 0.0, 0.0])
    rng = np.random.default_rng(1)
    b = rng.standard_normal((3, 4, 4, 4)) + 0j
    b[:, 0, 0, 0] = 0.0                                   # consistent right-hand side
    x, it, rel = solvers.pcg(ops, b, 1e-12)
    assert rel <= 1e-12 and np.allclose(x[:, 0, 0, 0], 0.0)


def test_reference_vectors_are_exact_lowest_modes_of_a_one_grain_cell():
    """Pin of the oracle's cold start (the lowest plane waves of the reference medium
    C0, Sec. 3.3): in a one-grain cell C0 is the crystal's own stiffness, so those plane
    waves are exact eigenvectors of the pencil (K, M).  Every returned vector satisfies
    K u = lambda M u to rounding, the vectors are orthonormal, and their Rayleigh
    quotients are the lowest eigenvalues of the dense pencil."""
    ops = Operators(_poly(4, 1, 0), np.array([0.3, 0.2, 0.1]) * np.pi / L)
    n = 7
    lam_d, _ = solvers.dense_modes(ops, n)
    U = solvers.reference_vectors(ops, n)
    lam = []
    for u in U:
        Ku, Mu = ops.apply_K(u), ops.apply_M(u)
        lu = np.vdot(u, Ku).real / np.vdot(u, Mu).real
        assert np.linalg.norm(Ku - lu * Mu) <= 1e-10 * lu * np.linalg.norm(Mu)
        lam.append(lu)
    assert np.allclose(np.sort(lam), lam_d[:n], rtol=1e-10)
    G = U.reshape(n, -1).conj() @ U.reshape(n, -1).T
    assert np.allclose(G, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("k", [[0.35, 0.0, 0.0], [0.5, 0.5, 0.0], [0.0, 0.0, 0.0]])
def test_subspace_matches_dense(k):
    ops = Operators(_poly(4, 6, 1), np.array(k) * np.pi / L)
    lam_d, _ = solvers.dense_modes(ops, 9)
    lam_s, U, info = solvers.subspace(ops, 9, 16, 1e-12, 1e-13)
    d = Operators(_poly(4, 6, 1), np.array(k) * np.pi / L)
    if solvers.Deflation(d).active:
        lam_s = np.concatenate([np.zeros(3), lam_s])
        assert np.all(lam_d[:3] < 1e-10 * lam_d[3])
        assert np.allclose(lam_s[3:], lam_d[3:], rtol=1e-10)
    else:
        assert np.allclose(lam_s, lam_d, rtol=1e-10)
    assert info["err1"] <= 1e-12 and info["err2"] <= 1e-11


@pytest.mark.parametrize("k", [[0.2, 0.3, 0.1], [0.0, 0.0, 0.0]])
def test_lanczos_matches_dense(k):
    ops = Operators(_poly(4, 6, 2), np.array(k) * np.pi / L)
    lam_d, _ = solvers.dense_modes(ops, 8)
    lam_l, X, info = solvers.lanczos(ops, 8, 1e-12, 1e-13)
    off = 3 if solvers.Deflation(ops).active else 0
    assert np.allclose(lam_l, lam_d[off:], rtol=1e-10)
    # Ritz vectors satisfy the pencil and are M-orthonormal
    for p in range(len(lam_l)):
        r = ops.apply_K(X[p]) - lam_l[p] * ops.apply_M(X[p])
        assert np.linalg.norm(r) <= 1e-8 * lam_l[p] * np.linalg.norm(ops.apply_M(X[p]))
    G = np.array([[np.vdot(a, ops.apply_M(b)) for b in X] for a in X])
    assert np.allclose(G, np.eye(len(X)), atol=1e-9)


def test_lowest_modes_path_with_warm_start_matches_dense():
    rve = _poly(6, 5, 3)
    ks = inputs.kpath("GXM", 4, L)
    w_it = solvers.lowest_modes(rve, ks, 6, method="subspace", block=12, dense_max=0,
                                tol_eig=1e-12, tol_lin=1e-13)
    w_d = solvers.lowest_modes(rve, ks, 6, method="dense")
    assert np.all(w_it[0, :3] == 0.0)
    assert np.allclose(w_it[1:], w_d[1:], rtol=1e-10)
    assert np.allclose(w_it[0, 3:], w_d[0, 3:], rtol=1e-10)


def test_homogeneous_1d_six_points():
    """Sec. 4.1: 6 points, 6 eigenvalues, omega_n = c |xi_n + k| exactly (eq. disp_homo)."""
    E, rho = inputs.EPOXY["E"], inputs.EPOXY["rho"]
    rve = inputs.homogeneous((6, 1, 1), (L, L, L), inputs.isotropic_voigt(E, 0.0), rho)
    c = np.sqrt(E / rho)                                  # nu = 0: P-wave modulus = E
    for k in np.linspace(0.0, np.pi / L, 5):
        w, X = solvers.dense_modes(Operators(rve, [k, 0, 0]), 18)
        Xl = X.reshape(18, 3, 6)
        lon = np.sort(w[np.abs(Xl[:, 0]).sum(axis=1) > 0.5 * np.abs(Xl).sum(axis=(1, 2))])
        ref = np.sort((c * np.abs(2 * np.pi * np.array([0, 1, 2, -3, -2, -1]) / L + k)) ** 2)
        assert np.allclose(lon, ref, rtol=1e-12, atol=1e-3)


def _rytov_roots(k, E1, r1, E2, r2, nroots):
    c1, c2 = np.sqrt(E1 / r1), np.sqrt(E2 / r2)
    p = np.sqrt(E2 * r2 / (E1 * r1))

    def f(w):
        a, b = w * L / (2 * c1), w * L / (2 * c2)
        return np.cos(a) * np.cos(b) - (1 + p * p) / (2 * p) * np.sin(a) * np.sin(b) - np.cos(k * L)

    ws = np.linspace(1.0, 40 * 2 * np.pi / L * min(c1, c2), 400000)
    fv = f(ws)
    idx = np.nonzero(np.sign(fv[:-1]) != np.sign(fv[1:]))[0][:nroots]
    return np.array([brentq(f, ws[i], ws[i + 1], xtol=1e-12) for i in idx])


def test_laminate_converges_to_rytov():
    """Sec. 4.2: epoxy/carbon bilayer (Table 1), k along the layering normal.

    Longitudinal branches use the P-wave modulus lambda + 2 mu, transverse ones mu.
    The FFT discretization converges to the laminate relation at second order."""
    ep, ca = inputs.EPOXY, inputs.CARBON
    pw = lambda m: m["E"] * (1 - m["nu"]) / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
    mu = lambda m: m["E"] / (2 * (1 + m["nu"]))
    errs = []
    for N in (32, 64, 128):
        k = 0.3 * np.pi / L
        lam, _ = solvers.dense_modes(Operators(inputs.bilayer(N, L, ep, ca), [k, 0, 0]), 9)
        rl = _rytov_roots(k, pw(ep), ep["rho"], pw(ca), ca["rho"], 6)
        rt = _rytov_roots(k, mu(ep), ep["rho"], mu(ca), ca["rho"], 6)
        ref = np.sort(np.concatenate([rl, rt, rt]))[:9]
        errs.append(np.abs(np.sqrt(lam) - ref) / ref)
    errs = np.array(errs)
    assert errs[-1].max() < 1e-4
    assert np.all(errs[1] < 0.35 * errs[0]) and np.all(errs[2] < 0.35 * errs[1])


def test_laminate_plus_sign_reading_fails():
    """The relation as printed (plus sign) is not satisfied by the homogeneous limit."""
    c = 1000.0
    w = c * 0.3 * np.pi / L                               # exact homogeneous branch at k
    a = w * L / (2 * c)
    printed = np.cos(a) ** 2 + np.sin(a) ** 2              # (1 + p^2) / 2p = 1 at p = 1
    corrected = np.cos(a) ** 2 - np.sin(a) ** 2
    assert abs(corrected - np.cos(0.3 * np.pi)) < 1e-12
    assert abs(printed - np.cos(0.3 * np.pi)) > 0.1
