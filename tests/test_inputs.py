"""Seeded input generators: determinism, Voronoi assignment, orientation statistics,
stiffness rotation invariants and k-path sampling."""
import numpy as np

from paper_2106_12487_amd import inputs

L = 1e-3


def test_polycrystal_is_deterministic_and_uses_all_grains():
    a = inputs.polycrystal((16, 16, 16), (L, L, L), 8, 1, 0)
    b = inputs.polycrystal((16, 16, 16), (L, L, L), 8, 1, 0)
    assert np.array_equal(a.grain_map, b.grain_map) and np.array_equal(a.C21, b.C21)
    assert a.grain_map.dtype == np.uint16 and set(np.unique(a.grain_map)) <= set(range(8))
    c = inputs.polycrystal((16, 16, 16), (L, L, L), 8, 1, 1)
    assert not np.array_equal(a.grain_map, c.grain_map)


def test_voronoi_brute_force_small():
    rng = np.random.default_rng(3)
    seeds = rng.random((5, 3)) * L
    g = inputs.voronoi_grain_map((5, 4, 3), (L, L, L), seeds)
    for idx in np.ndindex(5, 4, 3):
        x = (np.array(idx) + 0.5) * L / np.array([5, 4, 3])
        best, bd = None, np.inf
        for s in range(5):
            for sh in np.ndindex(3, 3, 3):
                d = np.sum((x - seeds[s] + (np.array(sh) - 1) * L) ** 2)
                if d < bd:
                    bd, best = d, s
        assert g[idx] == best


def _voronoi_all_seeds(n, Lv, seeds):
    """Every voxel against every seed (minimum image), lowest index on ties."""
    axes = [(np.arange(n[a]) + 0.5) * (Lv[a] / n[a]) for a in range(3)]
    X = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    d = X[:, None, :] - seeds[None, :, :]
    d -= np.asarray(Lv) * np.round(d / np.asarray(Lv))
    return np.argmin(np.einsum("vgk,vgk->vg", d, d), axis=1).reshape(n)


def test_voronoi_candidates_match_all_seeds():
    # the k-d tree only proposes candidates; the assignment equals the comparison with
    # every seed, on an uneven grid with many grains and on exact ties (lowest index wins)
    rng = np.random.default_rng(7)
    seeds = rng.random((300, 3)) * np.array([L, 2 * L, L])
    n = (24, 40, 17)
    assert np.array_equal(inputs.voronoi_grain_map(n, (L, 2 * L, L), seeds),
                          _voronoi_all_seeds(n, (L, 2 * L, L), seeds))
    # unit cell, seeds at x = 1/4 and 3/4: the voxel plane x = 1/2 of a 3-voxel grid is
    # exactly equidistant (and so is x = 1/6 vs 5/6 through the periodic image)
    tie = np.array([[0.75, 0.5, 0.5], [0.25, 0.5, 0.5]])
    g = inputs.voronoi_grain_map((3, 2, 2), (1.0, 1.0, 1.0), tie)
    assert np.array_equal(g, _voronoi_all_seeds((3, 2, 2), (1.0, 1.0, 1.0), tie))
    assert np.all(g[1] == 0)


def test_haar_rotations_are_rotations_and_unbiased():
    R = inputs.haar_rotations(np.random.default_rng(0).random((4000, 3)))
    assert np.allclose(np.einsum("nij,nkj->nik", R, R), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)
    assert np.abs(R.mean(axis=0)).max() < 0.05           # E[R] = 0 under Haar measure


def test_rotation_preserves_invariants_and_isotropy():
    R = inputs.haar_rotations(np.random.default_rng(1).random((3, 3)))
    C = inputs.CU["C"]
    M = np.diag([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])   # Mandel scaling
    ev0 = np.linalg.eigvalsh(M @ C @ M)
    for r in R:
        Cr = inputs.rotate_voigt(C, r)
        assert np.allclose(np.linalg.eigvalsh(M @ Cr @ M), ev0, rtol=1e-12)
        Ci = inputs.AL["C"]
        assert np.allclose(inputs.rotate_voigt(Ci, r), Ci, atol=1e-3)
    # 90 degrees about z swaps the x and y axes of a hexagonal crystal lying on its side
    Ch = inputs.TI["C"]
    Ry = inputs.rotvec_matrix(np.array([0.0, np.pi / 2, 0.0]))
    Cs = inputs.rotate_voigt(Ch, Ry)                      # c-axis now along x
    assert np.isclose(Cs[0, 0], Ch[2, 2]) and np.isclose(Cs[2, 2], Ch[0, 0])


def test_c21_roundtrip():
    C = inputs.rotate_voigt(inputs.TI["C"], inputs.haar_rotations(np.array([[0.2, 0.4, 0.7]]))[0])
    assert np.allclose(inputs.c21_to_voigt(inputs.voigt_to_c21(C)), C)


def test_ti_texture_spread():
    tilt = np.random.default_rng(2).normal(0, np.radians(15), (3000, 2))
    R = inputs.c_axis_texture(tilt, np.zeros(3000))
    ang = np.degrees(np.arccos(np.clip(R[:, 2, 2], -1, 1)))   # c-axis angle to z
    # tilt magnitude of an isotropic 2D normal with sigma 15 deg: Rayleigh, mean 15 sqrt(pi/2)
    assert abs(ang.mean() - 15 * np.sqrt(np.pi / 2)) < 1.0


def test_kpath_sampling():
    ks = inputs.kpath("GXMGR", 40, L)
    assert ks.shape == (40, 3)
    assert np.allclose(ks[0], 0) and np.allclose(ks[-1], np.pi / L)
    d = np.linalg.norm(np.diff(ks, axis=0), axis=1)
    # equal arc-length spacing except where a segment corner cuts a step
    assert np.isclose(np.median(d), d.max())
    ks1 = inputs.workload_kpoints(1)
    assert ks1.shape == (11, 3) and np.isclose(ks1[-1, 0], np.pi / L)
