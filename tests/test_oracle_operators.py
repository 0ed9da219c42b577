"""Pins of the oracle's K, M, M^-1 and preconditioner (Sec. 3.2 eqs. hatA, hatM;
Sec. 3.3 eqs. def_invM, matrixP, precond; Sec. 4.1 eq. anal_eigen_3D)."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2106_12487_amd import inputs
from oracle.operators import Operators
from oracle.solvers import dense_modes

L = 1e-3


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _poly(n, grains=5, idx=0):
    return inputs.polycrystal((n, n, n), (L, L, L), grains, 99, idx)


def test_homogeneous_isotropic_closed_form():
    """Sec. 4.1: a homogeneous isotropic cell has omega = c_{L,T} |xi + k| (one L, two T)."""
    E, nu, rho = 70e9, 0.33, 2700.0
    lam_, mu = inputs.lame(E, nu)
    rve = inputs.homogeneous((4, 4, 4), (L, L, L), inputs.isotropic_voigt(E, nu), rho)
    k = np.array([0.37, -0.21, 0.11]) * np.pi / L
    ops = Operators(rve, k)
    w, _ = dense_modes(ops, 3 * 64)
    # closed form over the label window, written directly from the integer labels
    m = [np.fft.fftfreq(4) * 4] * 3
    qq = np.array([(2 * np.pi * a / L + k[0]) ** 2 + (2 * np.pi * b / L + k[1]) ** 2
                   + (2 * np.pi * c / L + k[2]) ** 2 for a in m[0] for b in m[1] for c in m[2]])
    ref = np.sort(np.concatenate([(lam_ + 2 * mu) / rho * qq, mu / rho * qq, mu / rho * qq]))
    assert np.allclose(w, ref, rtol=1e-12, atol=0)


def test_homogeneous_cubic_along_x_closed_form():
    """Cubic crystal, propagation along [100]: rho w^2 = C11 q^2 (L) and C44 q^2 (T, twice).

    A wrong engineering-shear factor in the Voigt contraction would change the
    transverse branch (C44 vs 2 C44 or C44 / 2)."""
    C = inputs.CU["C"]
    rho = inputs.CU["rho"]
    rve = inputs.homogeneous((12, 1, 1), (L, L, L), C, rho)
    k = 0.43 * np.pi / L
    w, _ = dense_modes(Operators(rve, [k, 0, 0]), 36)
    q2 = (2 * np.pi * (np.fft.fftfreq(12) * 12) / L + k) ** 2
    ref = np.sort(np.concatenate([C[0, 0] * q2, C[3, 3] * q2, C[3, 3] * q2]) / rho)
    assert np.allclose(w, ref, rtol=1e-12)


def test_plane_wave_probe_matches_numpy_fft_of_stiffness():
    """K applied to one Fourier basis vector equals q_j(xi) C^_ijbl(xi - xi0) q_l(xi0) / N^3,
    with C^ the DFT of the tensor field C(x) computed by numpy."""
    rve = inputs.polycrystal((4, 6, 5), (L, 1.3 * L, 0.9 * L), 6, 98, 0)
    k = np.array([0.3, -0.45, 0.2]) * np.pi / L
    ops = Operators(rve, k)
    T = np.stack([inputs.voigt_to_tensor(inputs.c21_to_voigt(c)) for c in rve.C21])
    Tx = T[rve.grain_map.astype(int)]                           # (n0,n1,n2,3,3,3,3)
    Th = np.fft.fftn(Tx, axes=(0, 1, 2))
    n = rve.n
    ntot = np.prod(n)
    for (j0, b) in [((1, 2, 3), 0), ((0, 0, 0), 2), ((3, 5, 1), 1)]:
        U = np.zeros((3,) + n, dtype=complex)
        U[(b,) + j0] = 1.0
        got = ops.apply_K(U)
        q0 = ops.qvec[j0]
        shift = tuple(np.mod(np.arange(n[a]) - j0[a], n[a]) for a in range(3))
        Cs = Th[shift[0][:, None, None], shift[1][None, :, None], shift[2][None, None, :]]
        ref = np.einsum("xyzj,xyzijl,l->ixyz", ops.qvec, Cs[..., :, :, b, :], q0) / ntot
        assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("k", [[0.3, 0.1, -0.2], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
def test_hermitian_psd(k):
    ops = Operators(_poly(6, 7), np.array(k) * np.pi / L)
    u, v = _rand((3, 6, 6, 6), 1), _rand((3, 6, 6, 6), 2)
    Ku, Kv = ops.apply_K(u), ops.apply_K(v)
    scale = np.abs(np.vdot(u, Ku))
    assert abs(np.vdot(v, Ku) - np.conj(np.vdot(u, Kv))) <= 1e-13 * scale
    assert np.vdot(u, Ku).real > 0 and abs(np.vdot(u, Ku).imag) <= 1e-13 * scale
    Mu, Mv = ops.apply_M(u), ops.apply_M(v)
    assert abs(np.vdot(v, Mu) - np.conj(np.vdot(u, Mv))) <= 1e-13 * abs(np.vdot(u, Mu))


def test_exactly_three_rigid_zero_modes_at_gamma():
    ops = Operators(_poly(4, 5), [0.0, 0.0, 0.0])
    K, M = ops.dense("K"), ops.dense("M")
    w, X = sla.eigh(K, M)
    small = w < 1e-12 * w.max()
    assert small.sum() == 3
    # their eigenvectors live only on the xi = 0 coefficient (constant displacement)
    Z = X[:, small].reshape(3, 64, 3)
    assert np.allclose(np.delete(Z, 0, axis=1), 0.0, atol=1e-9 * np.abs(Z).max())


def test_k_plus_G_unitarily_equivalent():
    """K(k + G) = S K(k) S^H with S the cyclic relabelling of the DFT index; equal spectra."""
    rve = _poly(4, 5)
    k = np.array([0.31, -0.12, 0.4]) * np.pi / L
    nG = (1, 0, -2)
    G = 2 * np.pi * np.array(nG) / L
    a, b = Operators(rve, k), Operators(rve, k + G)
    shifted = np.roll(a.qvec, shift=tuple(-s for s in nG), axis=(0, 1, 2))
    assert np.allclose(b.qvec, shifted, rtol=0, atol=1e-9 * np.abs(a.qvec).max())
    u = _rand((3, 4, 4, 4), 5)
    roll = lambda v, sgn: np.roll(v, shift=tuple(sgn * s for s in nG), axis=(1, 2, 3))
    ref = roll(a.apply_K(roll(u, +1)), -1)
    assert np.allclose(b.apply_K(u), ref, atol=1e-12 * np.abs(ref).max())
    wa = sla.eigh(a.dense("K"), a.dense("M"), eigvals_only=True)
    wb = sla.eigh(b.dense("K"), b.dense("M"), eigvals_only=True)
    assert np.allclose(wa, wb, rtol=1e-12)


def test_inverse_mass_is_exact():
    ops = Operators(_poly(5, 4), [0.1, 0.2, 0.3])
    u = _rand((2, 3, 5, 5, 5), 3)
    assert np.allclose(ops.apply_Minv(ops.apply_M(u)), u, atol=1e-12 * np.abs(u).max())


def test_preconditioner_inverts_homogeneous_K():
    """For a homogeneous medium P^ = K^-1 on the range of K (eqs. matrixP, precond)."""
    rve = inputs.homogeneous((4, 5, 3), (L, L, L), inputs.TI["C"], inputs.TI["rho"])
    for k in ([0.2, 0.1, -0.3], [0.0, 0.0, 0.0]):
        ops = Operators(rve, np.array(k) * np.pi / L)
        u = _rand((3, 4, 5, 3), 4)
        u[:, ops.null_mask] = 0.0
        assert np.allclose(ops.precond(ops.apply_K(u)), u, atol=1e-12 * np.abs(u).max())


def test_voigt_upper_bound_on_acoustic_branches():
    """Courant-Fischer on the constant trial space: lambda_j(K, M) <= eig_j(P(C0, k)) / rho_bar."""
    rve = _poly(4, 6, 2)
    k = np.array([0.25, 0.1, 0.0]) * np.pi / L
    ops = Operators(rve, k)
    w, _ = dense_modes(ops, 3)
    P0 = inputs.voigt_to_tensor(ops.C0)
    Pk = np.einsum("ijkl,j,l->ik", P0, k, k) / ops.rho_bar
    assert np.all(w <= np.linalg.eigvalsh(Pk) * (1 + 1e-12))


def test_near_reciprocal_lattice_wave_vector_is_snapped():
    """A wave vector within rounding of a reciprocal lattice vector (e.g. the
    arc-length interpolated end of a closed path) is that vector: one voxel has
    xi + k = 0 exactly and K has the three rigid zero modes."""
    from oracle.fourier import snap_wavevector
    L = (1e-3, 1e-3, 1e-3)
    k = np.array([-6.98e-13, 2.0 * np.pi / 1e-3 + 4e-13, 0.0])
    ks = snap_wavevector(L, k)
    assert ks[0] == 0.0 and ks[1] == 2.0 * np.pi / 1e-3 and ks[2] == 0.0
    assert np.array_equal(snap_wavevector(L, [1e-3, 0.0, 0.0]), [1e-3, 0.0, 0.0])   # 1.6e-7 of 2 pi / L: kept
    rve = inputs.polycrystal((4, 4, 4), L, 3, 96, 3, phases=("cu", "al"))
    ops = Operators(rve, k)
    assert int(ops.null_mask.sum()) == 1
    w = np.linalg.eigvalsh(ops.dense("K"))
    assert np.sum(np.abs(w) <= 1e-9 * w.max()) == 3


def test_oracle_voigt_maps():
    """The oracle's own Voigt <-> tensor maps: the isotropic tensor from its Lame
    constants, the minor and major symmetries, and the 21 <-> 6x6 round trip."""
    from oracle import voigt
    lam_, mu = 51.0e9, 26.0e9
    d = np.eye(3)
    iso = (lam_ * np.einsum("ij,kl->ijkl", d, d)
           + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    C6 = np.zeros((6, 6))
    C6[:3, :3] = lam_
    C6[[0, 1, 2], [0, 1, 2]] = lam_ + 2 * mu
    C6[[3, 4, 5], [3, 4, 5]] = mu
    assert np.array_equal(voigt.voigt_to_tensor(C6), iso)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 6))
    S = A + A.T
    T = voigt.voigt_to_tensor(S)
    assert np.array_equal(T, T.transpose(1, 0, 2, 3)) and np.array_equal(T, T.transpose(0, 1, 3, 2))
    assert np.array_equal(T, T.transpose(2, 3, 0, 1))
    assert T[1, 2, 0, 1] == S[3, 5] and T[0, 2, 2, 2] == S[4, 2]
    c21 = S[np.triu_indices(6)]
    assert np.array_equal(voigt.c21_to_voigt(c21), S)
    # the row-major upper-triangle order: entry 6 is (1, 1), entry 11 is (2, 2)
    assert voigt.c21_to_voigt(np.arange(21.0))[1, 1] == 6 and voigt.c21_to_voigt(np.arange(21.0))[2, 2] == 11
