"""Seeded synthetic inputs: periodic Voronoi polycrystals, crystal stiffness
tensors, orientations, textures and wave-vector paths.

This module holds the microstructure generation that comes before the Bloch
method (the voxelized unit cell with its stiffness C(x) and density rho(x) is
the method's input, Sec. 3.2 and Algorithm "Full algorithm", step (a)).  It
contains none of the method's arithmetic (no Fourier operators, no solvers) and
is the only code shared by the HIP path and the CPU oracle.

Conventions
-----------
* Voigt 6x6 stiffness with engineering shear strain
  [e11, e22, e33, 2e23, 2e13, 2e12]; the 21 independent entries are stored as
  the upper triangle, row-major: (0,0),(0,1),...,(0,5),(1,1),...,(5,5).
* A rotation matrix R has the crystal axes as its columns, expressed in the
  sample frame; C'_ijkl = R_ia R_jb R_kc R_ld C_abcd.
* Grids are C-ordered [n0][n1][n2] with n2 fastest; voxel centres sit at
  (i + 1/2) L / n along each axis (Sec. 3.2, voxel-centre formula).
* Every random draw comes from numpy PCG64 seeded with
  SeedSequence([2106, 12487, config, index]); the draw order is fixed:
  seed points, then orientations, then the phase choice.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GPa = 1.0e9

# Voigt index pairs (engineering order 11,22,33,23,13,12).
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
TRIU_6 = [(a, b) for a in range(6) for b in range(a, 6)]


# --------------------------------------------------------------------------
# crystal stiffness in the crystal frame
# --------------------------------------------------------------------------
def cubic_voigt(c11: float, c12: float, c44: float) -> np.ndarray:
    """Cubic single-crystal Voigt matrix (Pa)."""
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    np.fill_diagonal(C[:3, :3], c11)
    C[3, 3] = C[4, 4] = C[5, 5] = c44
    return C


def isotropic_voigt(E: float, nu: float) -> np.ndarray:
    """Isotropic Voigt matrix from Young's modulus and Poisson's ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return cubic_voigt(lam + 2.0 * mu, lam, mu)


def lame(E: float, nu: float) -> tuple[float, float]:
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def hexagonal_voigt(c11, c12, c13, c33, c44) -> np.ndarray:
    """Transversely isotropic (hexagonal) Voigt matrix, c-axis = crystal x3."""
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = c11
    C[0, 1] = C[1, 0] = c12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = c13
    C[2, 2] = c33
    C[3, 3] = C[4, 4] = c44
    C[5, 5] = 0.5 * (c11 - c12)
    return C


# Material library (SI units).
CU = dict(C=cubic_voigt(168.4 * GPa, 121.4 * GPa, 75.4 * GPa), rho=8960.0)
AL = dict(C=isotropic_voigt(70.0 * GPa, 0.33), rho=2700.0)
TI = dict(C=hexagonal_voigt(162.4 * GPa, 92.0 * GPa, 69.0 * GPa, 180.7 * GPa, 46.7 * GPa),
          rho=4506.0)
# Table 1 of the paper (composite 1) and the Ni constants of Sec. 5.
EPOXY = dict(C=isotropic_voigt(4.507 * GPa, 0.4), rho=1200.0, E=4.507 * GPa, nu=0.4)
CARBON = dict(C=isotropic_voigt(230.0 * GPa, 0.3), rho=1750.0, E=230.0 * GPa, nu=0.3)
NI = dict(C=cubic_voigt(253.0 * GPa, 152.0 * GPa, 124.0 * GPa), rho=8908.0)


# --------------------------------------------------------------------------
# Voigt <-> tensor, rotation
# --------------------------------------------------------------------------
def voigt_to_tensor(C6: np.ndarray) -> np.ndarray:
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            v = C6[I, J]
            for a, b in ((i, j), (j, i)):
                for c, d in ((k, l), (l, k)):
                    T[a, b, c, d] = v
    return T


def tensor_to_voigt(T: np.ndarray) -> np.ndarray:
    C6 = np.empty((6, 6))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            C6[I, J] = T[i, j, k, l]
    return C6


def rotate_voigt(C6: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Stiffness of a crystal whose axes are the columns of R, in the sample frame."""
    T = voigt_to_tensor(C6)
    Tr = np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, T, optimize=True)
    return tensor_to_voigt(Tr)


def voigt_to_c21(C6: np.ndarray) -> np.ndarray:
    return np.array([C6[a, b] for a, b in TRIU_6])


def c21_to_voigt(c21: np.ndarray) -> np.ndarray:
    C6 = np.zeros((6, 6))
    for v, (a, b) in zip(c21, TRIU_6):
        C6[a, b] = C6[b, a] = v
    return C6


# --------------------------------------------------------------------------
# orientations
# --------------------------------------------------------------------------
def quat_to_matrix(w, x, y, z) -> np.ndarray:
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def haar_rotations(u: np.ndarray) -> np.ndarray:
    """Uniform (Haar) rotations from G x 3 uniforms (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = u[:, 0], u[:, 1], u[:, 2]
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    x, y = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    z, w = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    return np.stack([quat_to_matrix(*q) for q in zip(w, x, y, z)])


def rotvec_matrix(v: np.ndarray) -> np.ndarray:
    """Rodrigues: exp of the skew matrix of rotation vector v."""
    th = float(np.linalg.norm(v))
    if th == 0.0:
        return np.eye(3)
    k = v / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * (Kx @ Kx)


def rot_z(psi: float) -> np.ndarray:
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def fibre_rotations(axis, psi: np.ndarray) -> np.ndarray:
    """Fibre texture (Sec. 5.2, effect of texture): the crystal direction `axis` along
    sample z, spin psi about z.  R = Rz(psi) R0 with R0 the smallest rotation taking
    axis / |axis| to z (columns of R: crystal axes in the sample frame)."""
    a = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(a, z)
    s, c = np.linalg.norm(v), float(a @ z)
    R0 = np.eye(3) if s == 0.0 else rotvec_matrix(v / s * math.atan2(s, c))
    return np.stack([rot_z(p) @ R0 for p in psi])


def c_axis_texture(tilt: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """R = Exp([tx, ty, 0]) Rz(psi): c-axes spread about sample z, free spin about c."""
    return np.stack([rotvec_matrix(np.array([t[0], t[1], 0.0])) @ rot_z(p)
                     for t, p in zip(tilt, psi)])


# --------------------------------------------------------------------------
# periodic Voronoi
# --------------------------------------------------------------------------
def voronoi_grain_map(n, L, seeds: np.ndarray, chunk: int = 1 << 16, candidates: int = 8) -> np.ndarray:
    """Nearest seed (minimum-image Euclidean distance) of each voxel centre.

    Ties go to the lowest seed index.  Returns uint16 [n0, n1, n2].  A periodic
    k-d tree proposes the `candidates` nearest seeds of each voxel; the minimum-image
    distances to those are then compared exactly as for the full set (the true
    nearest seed, and any seed within rounding of it, is always among them).
    """
    from scipy.spatial import cKDTree
    n = tuple(int(v) for v in n)
    L = np.asarray(L, dtype=np.float64)
    axes = [(np.arange(n[a]) + 0.5) * (L[a] / n[a]) for a in range(3)]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    kc = min(candidates, seeds.shape[0])
    tree = cKDTree(np.mod(seeds, L), boxsize=L)
    out = np.empty(X.shape[0], dtype=np.uint16)
    for s in range(0, X.shape[0], chunk):
        _, cand = tree.query(X[s:s + chunk], k=kc)
        cand = np.sort(np.asarray(cand).reshape(-1, kc), axis=1)      # ascending seed index
        d = X[s:s + chunk, None, :] - seeds[cand]
        d -= L * np.round(d / L)
        best = np.argmin(np.einsum("vgk,vgk->vg", d, d), axis=1)
        out[s:s + chunk] = cand[np.arange(cand.shape[0]), best]
    return out.reshape(n)


# --------------------------------------------------------------------------
# RVE container and configurations
# --------------------------------------------------------------------------
@dataclass
class RVE:
    n: tuple
    L: tuple
    grain_map: np.ndarray          # uint16 [n0, n1, n2]
    C21: np.ndarray                # float64 [G, 21], sample frame, Pa
    rho: np.ndarray                # float64 [G], kg/m^3
    meta: dict = field(default_factory=dict)

    @property
    def n_grains(self) -> int:
        return int(self.C21.shape[0])

    def voigt(self) -> np.ndarray:
        return np.stack([c21_to_voigt(c) for c in self.C21])


def rng_for(config: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2106, 12487, config, index])))


def polycrystal(n, L, n_grains: int, config: int, index: int, texture: str = "haar",
                phases=("cu",)) -> RVE:
    """Periodic Voronoi polycrystal.

    texture: "haar" (uniform random), "ti_c_axis" (c-axes N(0, 15 deg) about z),
             "fibre100" / "fibre111" (crystal [100] / [111] along z, uniform spin about z).
    phases:  ("cu",), ("ti",), ("ni",) or ("cu", "al") (each grain Cu or Al with p = 1/2).
    """
    rng = rng_for(config, index)
    L = tuple(float(v) for v in L)
    seeds = rng.random((n_grains, 3)) * np.asarray(L)
    if texture == "haar":
        R = haar_rotations(rng.random((n_grains, 3)))
    elif texture in ("fibre100", "fibre111"):
        psi = rng.random((n_grains, 3))[:, 0] * 2.0 * np.pi
        R = fibre_rotations([1, 0, 0] if texture == "fibre100" else [1, 1, 1], psi)
    elif texture == "ti_c_axis":
        tilt = rng.normal(0.0, math.radians(15.0), size=(n_grains, 2))
        psi = rng.random(n_grains) * 2.0 * np.pi
        R = c_axis_texture(tilt, psi)
    else:
        raise ValueError(texture)
    lib = {"cu": CU, "al": AL, "ti": TI, "ni": NI}
    if len(phases) == 1:
        choice = [phases[0]] * n_grains
    else:
        u = rng.random(n_grains)
        choice = [phases[0] if x < 0.5 else phases[1] for x in u]
    C21 = np.stack([voigt_to_c21(rotate_voigt(lib[p]["C"], R[g])) for g, p in enumerate(choice)])
    rho = np.array([lib[p]["rho"] for p in choice])
    gmap = voronoi_grain_map(n, L, seeds)
    return RVE(tuple(int(v) for v in n), L, gmap, C21, rho,
               dict(config=config, index=index, texture=texture, phases=choice, R=R))


def homogeneous(n, L, C6: np.ndarray, rho: float) -> RVE:
    n = tuple(int(v) for v in n)
    return RVE(n, tuple(float(v) for v in L), np.zeros(n, dtype=np.uint16),
               voigt_to_c21(C6)[None, :], np.array([float(rho)]))


def bilayer(N: int, L: float, mat1: dict, mat2: dict) -> RVE:
    """1D two-phase laminate on an N x 1 x 1 grid: phase 1 in x < L/2, phase 2 beyond."""
    g = np.zeros((N, 1, 1), dtype=np.uint16)
    x = (np.arange(N) + 0.5) * (L / N)
    g[x > 0.5 * L, 0, 0] = 1
    C21 = np.stack([voigt_to_c21(mat1["C"]), voigt_to_c21(mat2["C"])])
    return RVE((N, 1, 1), (L, L, L), g, C21, np.array([mat1["rho"], mat2["rho"]]))


def ni_bar(n: int, n_grains: int, Dbar: float, sd: float, A: float, index: int, config: int = 51) -> RVE:
    """1D polycrystal (Sec. 5.1) on an n x 1 x 1 grid: n_grains layers along x with
    lengths drawn from N(Dbar, sd) (draws below Dbar / 5 are redrawn), rescaled to sum to
    L = n_grains Dbar; Ni constants with C44 = A (C11 - C12) / 2 (Zener ratio A);
    Haar-random orientations.  Draw order: lengths, then orientations."""
    rng = rng_for(config, index)
    lengths = np.empty(n_grains)
    for g in range(n_grains):
        x = rng.normal(Dbar, sd) if sd > 0 else Dbar
        while x < 0.2 * Dbar:
            x = rng.normal(Dbar, sd)
        lengths[g] = x
    L = n_grains * Dbar
    edges = np.concatenate([[0.0], np.cumsum(lengths)]) * (L / lengths.sum())
    R = haar_rotations(rng.random((n_grains, 3)))
    c11, c12 = NI["C"][0, 0], NI["C"][0, 1]
    C = cubic_voigt(c11, c12, A * (c11 - c12) / 2)
    x = (np.arange(n) + 0.5) * (L / n)
    g = np.clip(np.searchsorted(edges, x, side="right") - 1, 0, n_grains - 1).astype(np.uint16)
    C21 = np.stack([voigt_to_c21(rotate_voigt(C, R[i])) for i in range(n_grains)])
    return RVE((n, 1, 1), (L, L, L), g[:, None, None], C21, np.full(n_grains, NI["rho"]),
               dict(config=config, index=index, A=A, Dbar=Dbar, sd=sd, R=R))


def fibre_composite(n: int, L: float, section: str, vf: float, matrix: dict = None, fibre: dict = None) -> RVE:
    """Long-fibre composite (Sec. 4.3): one fibre along z per n x n x 1 cell, centred,
    square arrangement.  section "circle" (radius L sqrt(vf / pi)) or "square" (side
    L sqrt(vf), edges along x and y); a voxel is fibre when its centre lies inside.
    Phase 0 is the matrix (epoxy by default), phase 1 the fibre (carbon)."""
    matrix = matrix or EPOXY
    fibre = fibre or CARBON
    c = (np.arange(n) + 0.5) * (L / n) - 0.5 * L
    X, Y = np.meshgrid(c, c, indexing="ij")
    if section == "circle":
        inside = X ** 2 + Y ** 2 < vf * L * L / np.pi
    elif section == "square":
        h = 0.5 * L * math.sqrt(vf)
        inside = (np.abs(X) < h) & (np.abs(Y) < h)
    else:
        raise ValueError(section)
    g = inside.astype(np.uint16)[:, :, None]
    C21 = np.stack([voigt_to_c21(matrix["C"]), voigt_to_c21(fibre["C"])])
    return RVE((n, n, 1), (L, L, L), g, C21, np.array([matrix["rho"], fibre["rho"]]),
               dict(section=section, vf=vf, vf_voxels=float(inside.mean())))


# --------------------------------------------------------------------------
# wave-vector paths (simple cubic Brillouin zone)
# --------------------------------------------------------------------------
def sc_points(L: float) -> dict:
    p = np.pi / L
    return {"G": np.array([0.0, 0.0, 0.0]), "X": np.array([p, 0.0, 0.0]),
            "M": np.array([p, p, 0.0]), "R": np.array([p, p, p])}


def kpath(labels: str, n: int, L: float) -> np.ndarray:
    """n points equally spaced in arc length along the polyline, both ends included."""
    P = sc_points(L)
    verts = np.stack([P[c] for c in labels])
    seg = np.linalg.norm(np.diff(verts, axis=0), axis=1)
    s_v = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.linspace(0.0, s_v[-1], n)
    out = np.empty((n, 3))
    for i, si in enumerate(s):
        j = min(int(np.searchsorted(s_v, si, side="right")) - 1, len(seg) - 1)
        t = (si - s_v[j]) / seg[j]
        out[i] = (1 - t) * verts[j] + t * verts[j + 1]
        # samples on a vertex (up to rounding of the arc length) are the vertex itself
        near = np.nonzero(np.abs(s_v - si) <= 1e-12 * s_v[-1])[0]
        if near.size:
            out[i] = verts[near[0]]
    return out


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
L_MM = 1.0e-3

WORKLOADS = {
    1: dict(name="cu16_8g_gx", n=16, grains=8, kpath=None, nk=11, nmodes=6, block=12,
            tol_lin=1e-10, tol_eig=1e-11),
    2: dict(name="cu64_64g_gxmgr", n=64, grains=64, kpath="GXMGR", nk=40, nmodes=12, block=16,
            tol_lin=1e-8, tol_eig=1e-10),
    3: dict(name="cual_uneven8", grids=[32, 32, 40, 40, 48, 48, 64, 64],
            grains=[8, 12, 18, 26, 39, 58, 86, 128], kpath="GXMG", nk=24, nmodes=8, block=16,
            tol_lin=1e-8, tol_eig=1e-8),
    4: dict(name="ti128_512g_gxmgr", n=128, grains=512, kpath="GXMGR", nk=60, nmodes=12,
            block=16, tol_lin=1e-8, tol_eig=1e-8),
    5: dict(name="cu64_learned", n=64, n_train=200),
}


def workload_rve(config: int, index: int = 0) -> RVE:
    w = WORKLOADS[config]
    L = (L_MM, L_MM, L_MM)
    if config in (1, 2):
        return polycrystal((w["n"],) * 3, L, w["grains"], config, index)
    if config == 3:
        n = w["grids"][index]
        return polycrystal((n,) * 3, L, w["grains"][index], config, index, phases=("cu", "al"))
    if config == 4:
        return polycrystal((128,) * 3, L, 512, config, index, texture="ti_c_axis", phases=("ti",))
    if config == 5:
        rng = rng_for(5, 100000 + index)
        g = int(round(16 * 16 ** rng.random()))
        return polycrystal((64,) * 3, L, g, config, index)
    raise ValueError(config)


def workload_kpoints(config: int) -> np.ndarray:
    w = WORKLOADS[config]
    if config == 1:
        return np.array([[t * np.pi / L_MM, 0.0, 0.0] for t in np.linspace(0.0, 1.0, 11)])
    return kpath(w["kpath"], w["nk"], L_MM)
