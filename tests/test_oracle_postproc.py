"""Pins of the oracle's group velocity and long-wave speeds (oracle/postproc.py)."""
import numpy as np
import pytest

from oracle import postproc, solvers
from oracle.operators import Operators
from paper_2106_12487_amd import inputs

L = 1e-3


def _dense(rve, k, nm):
    lam, U = solvers.dense_modes(Operators(rve, k), nm)
    return np.sqrt(np.maximum(lam, 0.0)), U


def _iso_speeds(mat):
    C = mat["C"]
    return np.sqrt(C[3, 3] / mat["rho"]), np.sqrt(C[0, 0] / mat["rho"])


def test_slopes_homogeneous_isotropic_and_folded_branch():
    """omega = c |k + G| for a homogeneous isotropic medium: along x at k = 0.3 pi/L the
    slopes are c_T, c_T, c_L on the G = 0 branches and -c_T on the transverse pair
    folded from G = -2 pi/L x; along y all five are 0."""
    al = inputs.AL
    cT, cL = _iso_speeds(al)
    rve = inputs.homogeneous((4, 4, 4), (L, L, L), al["C"], al["rho"])
    k = np.array([0.3 * np.pi / L, 0, 0])
    w, U = _dense(rve, k, 5)
    np.testing.assert_allclose(w, [0.3 * np.pi / L * cT] * 2 + [0.3 * np.pi / L * cL] + [1.7 * np.pi / L * cT] * 2,
                               rtol=1e-12)
    sx = postproc.branch_slopes(rve, k, [1, 0, 0], U, w)
    np.testing.assert_allclose(sx, [cT, cT, cL, -cT, -cT], rtol=1e-10)
    sy = postproc.branch_slopes(rve, k, [0, 1, 0], U, w)
    assert np.abs(sy).max() <= 1e-10 * cL


def test_slopes_match_central_differences_of_dense_eigenvalues():
    """Sec. 5.1 eq. c_group on a polycrystal at a generic k: slopes against central
    differences of the exact (dense) eigenvalues at k +- delta d."""
    rve = inputs.polycrystal((4, 4, 4), (L, L, L), 3, 94, 1)
    k = np.array([0.37, 0.21, 0.13]) * np.pi / L
    d = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])
    w, U = _dense(rve, k, 8)
    assert np.min(np.diff(w) / w[1:]) > 1e-3                       # simple eigenvalues
    s = postproc.branch_slopes(rve, k, d, U, w)
    delta = 1e-5 * np.pi / L
    wp, _ = _dense(rve, k + delta * d, 8)
    wm, _ = _dense(rve, k - delta * d, 8)
    fd = (wp - wm) / (2 * delta)
    scale = np.max(np.abs(fd))
    assert np.abs(s - fd).max() <= 1e-6 * scale
    assert np.abs(fd).min() > 1e-3 * scale                          # a discriminating direction


def test_slopes_of_rigid_modes_at_gamma_are_zero():
    rve = inputs.polycrystal((4, 4, 4), (L, L, L), 3, 94, 1)
    w = solvers.lowest_modes(rve, [np.zeros(3)], 6, method="dense")[0]
    _, U = _dense(rve, np.zeros(3), 6)
    s = postproc.branch_slopes(rve, np.zeros(3), [1, 0, 0], U, w)
    assert np.all(s[:3] == 0.0)


@pytest.mark.parametrize("d", [[1, 0, 0], [1, 1, 0]])
def test_long_wave_speeds_cubic_crystal_closed_form(d):
    """Homogeneous cubic crystal: Christoffel speeds, [100]: sqrt(C44/rho) (x2), sqrt(C11/rho);
    [110]: sqrt(C44/rho), sqrt((C11 - C12)/(2 rho)), sqrt((C11 + C12 + 2 C44)/(2 rho))."""
    ni = inputs.NI
    C, rho = ni["C"], ni["rho"]
    rve = inputs.homogeneous((4, 4, 4), (L, L, L), C, rho)
    c = postproc.long_wave_speeds(rve, d, method="dense")
    c11, c12, c44 = C[0, 0], C[0, 1], C[3, 3]
    if d == [1, 0, 0]:
        ref = np.sqrt([c44 / rho, c44 / rho, c11 / rho])
    else:
        ref = np.sqrt(np.sort([c44 / rho, (c11 - c12) / (2 * rho), (c11 + c12 + 2 * c44) / (2 * rho)]))
    np.testing.assert_allclose(c, ref, rtol=1e-9)


def test_long_wave_speeds_laminate_are_reuss_averages():
    """Epoxy/carbon bilayer (Table 1), waves along the layering normal: the quasi-static
    stress is uniform along x, so rho_bar c^2 is the harmonic mean of the P-wave modulus
    (longitudinal) and of the shear modulus (transverse)."""
    ep, ca = inputs.EPOXY, inputs.CARBON
    rve = inputs.bilayer(16, L, ep, ca)
    c = postproc.long_wave_speeds(rve, [1, 0, 0], method="dense")
    rho = 0.5 * (ep["rho"] + ca["rho"])
    pw = lambda m: m["C"][0, 0]
    mu = lambda m: m["C"][3, 3]
    cL = np.sqrt(1.0 / (0.5 / pw(ep) + 0.5 / pw(ca)) / rho)
    cT = np.sqrt(1.0 / (0.5 / mu(ep) + 0.5 / mu(ca)) / rho)
    np.testing.assert_allclose(c, [cT, cT, cL], rtol=1e-6)    # without the extrapolation: 5e-5
    cV = np.sqrt(0.5 * (mu(ep) + mu(ca)) / rho)                      # the Voigt value is far off
    assert cV > 2 * cT


@pytest.mark.parametrize("d", [[1, 0, 0], [1, 1, 0], [1, 1, 1], [0.3, -0.5, 0.8]])
def test_long_wave_speeds_polycrystal_within_voigt_reuss(d):
    rve = inputs.polycrystal((6, 6, 6), (L, L, L), 8, 94, 2)
    c = postproc.long_wave_speeds(rve, d, method="dense")
    lo, hi = postproc.voigt_reuss_bracket(rve, d)
    rho = float(np.mean(rve.rho[rve.grain_map]))
    e = rho * c ** 2
    assert np.all(e > lo * (1 + 1e-6)) and np.all(e < hi * (1 - 1e-6)), (lo, e, hi)


def test_clusters_groups_equal_frequencies():
    assert postproc.clusters(np.array([0.0, 0.0, 1.0, 1.0 + 1e-9, 2.0]), 1e-6) == [[0, 1], [2, 3], [4]]


def _christoffel(C6, d):
    T = inputs.voigt_to_tensor(C6)
    return np.einsum("ijkl,j,l->ik", T, d, d)


def test_long_wave_speeds_fibre100_texture_along_z_exact():
    """[100] fibre texture (Sec. 5.2, effect of texture): every grain has the cubic axis along
    z, so a uniform strain e_zz or e_xz / e_yz gives the same stress in every grain (rotations
    about a cube axis keep C33, C13, C44 and the zero couplings): the uniform field is the
    exact long-wave solution and c_L = sqrt(C11 / rho), c_T = sqrt(C44 / rho) (twice)."""
    ni = inputs.NI
    rve = inputs.polycrystal((6, 6, 6), (L, L, L), 8, 52, 0, texture="fibre100", phases=("ni",))
    c = postproc.long_wave_speeds(rve, [0, 0, 1], method="dense")
    ref = np.sqrt(np.array([ni["C"][3, 3], ni["C"][3, 3], ni["C"][0, 0]]) / ni["rho"])
    np.testing.assert_allclose(c, ref, rtol=1e-7)
    cx = postproc.long_wave_speeds(rve, [1, 0, 0], method="dense")          # not trivial across z
    assert np.abs(cx - ref).max() > 1e-3 * ref.max()


def test_long_wave_speeds_fibre111_texture_longitudinal_exact():
    """[111] fibre texture: rotations about a 3-fold axis keep C'3333 = (C11 + 2 C12 + 4 C44) / 3
    and C'13, and C'3323 = C'3313 = 0, so uniform e_zz is exact for the longitudinal wave."""
    ni = inputs.NI
    C = ni["C"]
    rve = inputs.polycrystal((6, 6, 6), (L, L, L), 8, 52, 1, texture="fibre111", phases=("ni",))
    c = postproc.long_wave_speeds(rve, [0, 0, 1], method="dense")
    cl = np.sqrt((C[0, 0] + 2 * C[0, 1] + 4 * C[3, 3]) / 3 / ni["rho"])
    np.testing.assert_allclose(c[2], cl, rtol=1e-7)


def test_long_wave_speeds_ni_bar_is_matrix_harmonic_mean():
    """1D polycrystal (Sec. 5.1) as layers normal to x: the traction on the layer planes is
    uniform in the long-wave limit, so rho c^2 are the eigenvalues of the matrix harmonic mean
    of the layers' Christoffel matrices along x (voxel average)."""
    rve = inputs.ni_bar(32, 8, 50e-6, 50e-6, 2.45, 0)
    c = postproc.long_wave_speeds(rve, [1, 0, 0], method="dense")
    C6 = np.stack([inputs.c21_to_voigt(x) for x in rve.C21])[rve.grain_map.ravel()]
    G = np.linalg.inv(np.mean([np.linalg.inv(_christoffel(Ci, np.array([1.0, 0, 0]))) for Ci in C6], axis=0))
    ref = np.sqrt(np.sort(np.linalg.eigvalsh(G)) / inputs.NI["rho"])
    np.testing.assert_allclose(c, ref, rtol=1e-6)
    Gv = np.mean([_christoffel(Ci, np.array([1.0, 0, 0])) for Ci in C6], axis=0)   # Voigt: off
    assert np.abs(np.sqrt(np.sort(np.linalg.eigvalsh(Gv)) / inputs.NI["rho"]) - ref).max() > 1e-3 * ref.max()


def test_mode_fields_recover_a_rotated_real_field():
    rng = np.random.default_rng(5)
    rve = inputs.polycrystal((6, 4, 5), (L, L, L), 3, 94, 1)
    w = rng.standard_normal((2, 3, 6, 4, 5))
    alpha = np.array([0.7, -1.1])
    from oracle.fourier import fft3
    U = fft3(w) * np.exp(1j * alpha)[:, None, None, None, None]
    u, _, phi = postproc.mode_fields(rve, [0.1 / L, 0, 0], U)
    for p in range(2):
        sgn = np.sign(np.real(u[p]).ravel() @ w[p].ravel())
        assert np.abs(u[p] - sgn * w[p]).max() <= 1e-12 * np.abs(w[p]).max()
        assert abs(np.angle(np.exp(2j * (phi[p] - alpha[p])))) <= 1e-12     # phi = alpha mod pi


def test_mode_fields_strain_of_trigonometric_displacement():
    """w = (sin 2pi x/L, 0.5 cos 2pi y/L, 0) on grid points x = i L/n: the strain of the
    Bloch wave w e^{ik.x} divided by e^{ik.x} is sym grad w + i sym(k (x) w)."""
    n = (8, 8, 4)
    rve = inputs.polycrystal(n, (L, L, L), 3, 94, 1)
    k = np.array([0.3, 0.1, 0.0]) * np.pi / L
    x = np.arange(n[0])[:, None, None] * L / n[0] + 0 * np.zeros(n)
    y = np.arange(n[1])[None, :, None] * L / n[1] + 0 * np.zeros(n)
    g = 2 * np.pi / L
    w = np.stack([np.sin(g * x), 0.5 * np.cos(g * y), np.zeros(n)])
    from oracle.fourier import fft3
    u, eps, phi = postproc.mode_fields(rve, k, fft3(w)[None])
    assert abs(phi[0]) <= 1e-12
    e11 = g * np.cos(g * x) + 1j * k[0] * w[0]
    e22 = -0.5 * g * np.sin(g * y) + 1j * k[1] * w[1]
    e12 = 1j * (k[1] * w[0] + k[0] * w[1])
    e13 = 1j * k[2] * w[0]
    for got, ref in ((eps[0, 0], e11), (eps[0, 1], e22), (eps[0, 5], e12), (eps[0, 4], e13), (eps[0, 2], 0 * x)):
        assert np.abs(got - ref).max() <= 1e-12 * g


def test_effective_stiffness_homogeneous_is_C():
    ni = inputs.NI
    rve = inputs.homogeneous((4, 4, 4), (L, L, L), inputs.rotate_voigt(ni["C"], inputs.haar_rotations(
        np.array([[0.3, 0.6, 0.1]]))[0]), ni["rho"])
    C = inputs.c21_to_voigt(rve.C21[0])
    np.testing.assert_allclose(postproc.effective_stiffness(rve), C, atol=1e-9 * np.abs(C).max())


def test_effective_stiffness_laminate_backus():
    """Epoxy/carbon layers normal to x (equal thickness): Backus averages.
    C11 = 1/<1/M>, C12 = C13 = <lam/M>/<1/M>, C22 = C33 = <M - lam^2/M> + <lam/M>^2/<1/M>,
    C23 = <lam - lam^2/M> + <lam/M>^2/<1/M>, C44 = <mu>, C55 = C66 = 1/<1/mu>."""
    ep, ca = inputs.EPOXY, inputs.CARBON
    rve = inputs.bilayer(8, L, ep, ca)
    Ce = postproc.effective_stiffness(rve)
    M = np.array([ep["C"][0, 0], ca["C"][0, 0]])
    lam = np.array([ep["C"][0, 1], ca["C"][0, 1]])
    mu = np.array([ep["C"][3, 3], ca["C"][3, 3]])
    a = lambda v: float(np.mean(v))
    ref = {(0, 0): 1 / a(1 / M), (0, 1): a(lam / M) / a(1 / M), (0, 2): a(lam / M) / a(1 / M),
           (1, 1): a(M - lam ** 2 / M) + a(lam / M) ** 2 / a(1 / M),
           (2, 2): a(M - lam ** 2 / M) + a(lam / M) ** 2 / a(1 / M),
           (1, 2): a(lam - lam ** 2 / M) + a(lam / M) ** 2 / a(1 / M),
           (3, 3): a(mu), (4, 4): 1 / a(1 / mu), (5, 5): 1 / a(1 / mu)}
    for (i, j), v in ref.items():
        assert abs(Ce[i, j] - v) <= 1e-9 * v, (i, j, Ce[i, j], v)


def test_effective_stiffness_within_voigt_reuss_and_matches_long_wave_speeds():
    """The long-wave limit of the Bloch problem is the static homogenization of the same
    discretization: rho_bar c^2 are the Christoffel eigenvalues of C_eff.  On an odd grid
    (a symmetric frequency set, real fields) the two agree to the extrapolation error."""
    rve = inputs.polycrystal((5, 5, 5), (L, L, L), 6, 94, 2)
    Ce = postproc.effective_stiffness(rve)
    ops = Operators(rve, np.zeros(3))
    C = ops.C_field.reshape(-1, 6, 6)
    CV, CR = C.mean(axis=0), np.linalg.inv(np.linalg.inv(C).mean(axis=0))
    assert np.linalg.eigvalsh(CV - Ce).min() > -1e-9 * np.abs(CV).max()
    assert np.linalg.eigvalsh(Ce - CR).min() > -1e-9 * np.abs(CV).max()
    rho = float(np.mean(rve.rho[rve.grain_map]))
    for d in ([1, 0, 0], [1, 1, 0], [0.3, -0.5, 0.8]):
        dn = np.array(d, dtype=float) / np.linalg.norm(d)
        c = postproc.long_wave_speeds(rve, d, method="dense")
        ref = np.sqrt(np.sort(np.linalg.eigvalsh(_christoffel(Ce, dn))) / rho)
        np.testing.assert_allclose(c, ref, rtol=3e-8)
