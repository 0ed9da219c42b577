"""Several cells in one bw_lowest_modes_batched call: a cell of a grid no other cell
shares gets the results of its own bw_lowest_modes call bit for bit (same kernels,
deterministic reductions); cells of one grid form a group that shares every batched
launch; a failing cell is reported by index."""
import json
import os

import numpy as np
import pytest

from paper_2106_12487_amd import inputs

pytestmark = pytest.mark.gpu
L = inputs.L_MM


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _cells(lib, prec):
    shapes = [((16, 16, 16), 6), ((12, 12, 12), 4), ((8, 16, 8), 5), ((32, 16, 16), 9)]
    out = []
    for i, (n, g) in enumerate(shapes):
        rve = inputs.polycrystal(n, (L, L, L), g, 3, 50 + i, phases=("cu", "al"))
        out.append(lib.Rve.from_inputs(rve, prec))
    return out


@pytest.mark.parametrize("prec,method", [(0, 1), (1, 1), (0, 0)])
def test_batched_equals_separate_calls(lib, prec, method):
    _torch()
    print(f"\n[case] batched cells prec={prec} method={method}", flush=True)
    cells = _cells(lib, prec)
    ks = [inputs.kpath("GXMG", n, L)[1:] for n in (6, 4, 5, 3)]
    kw = dict(method=method, tol_omega=1e-6 if prec == 1 else 1e-9, tol_lin=1e-6 if prec == 1 else 1e-10)
    oms, ers, code, st = lib.bw_lowest_modes_batched(cells, ks, 6, **kw)
    assert code == 0, lib.bw_last_error()
    assert st["pcg_iterations"] > 0
    for c, k, om, er in zip(cells, ks, oms, ers):
        o1, e1, c1, _ = lib.bw_lowest_modes(c, k, 6, **kw)
        assert c1 == 0
        assert np.array_equal(om, o1) and np.array_equal(er, e1)
    for c in cells:
        c.close()


def test_batched_reports_failing_cell(lib):
    _torch()
    cells = _cells(lib, 1)
    tiny = inputs.polycrystal((2, 2, 1), (L, L, L), 2, 3, 60)
    cells.insert(1, lib.Rve.from_inputs(tiny, 1))
    ks = [inputs.kpath("GX", 3, L)[1:]] * len(cells)
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_lowest_modes_batched(cells, ks, 14, method=1, tol_omega=1e-5)    # 14 > 3 * 4 unknowns of cell 1
    assert e.value.code == lib.BW_EINVAL and "cell 1" in str(e.value)
    for c in cells:
        c.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cual32.json")
BAR = {0: 1e-9, 1: 1e-5}


def _omega_ref(rve):
    from oracle.operators import Operators
    C0 = Operators(rve, (0.0, 0.0, 0.0)).C0
    return 2 * np.pi / L * np.sqrt(C0[3, 3] / float(np.mean(rve.rho)))


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle values not generated")
@pytest.mark.parametrize("prec", [0, 1])
def test_equal_grid_cells_share_launches_against_stored_oracle(lib, prec):
    """The two 32^3 Cu/Al cells of the uneven workload with a 40^3 one between them:
    the 32^3 pair forms a group (one handle, every batched launch carries the wave
    vectors of both, each with its own grain map and reference stiffness), the 40^3
    cell runs alone.  The first cell's frequencies against the stored oracle values
    (Gamma and three wave vectors of the path) within the bar and the bounds; both
    grouped cells against their separate solves within the two bounds; the lone cell
    bit for bit; the group takes fewer batched PCG sweeps than the cells one by one."""
    _torch()
    g = json.load(open(GOLDEN))
    ks = np.array(g["k"])
    nm = g["nmodes"]
    rves = [inputs.workload_rve(3, 0), inputs.workload_rve(3, 2), inputs.workload_rve(3, 1)]
    assert rves[0].n == rves[2].n != rves[1].n
    print(f"\n[case] grouped 32^3 pair + 40^3 cell, prec={prec}", flush=True)
    cells = [lib.Rve.from_inputs(r, prec) for r in rves]
    kw = dict(method=lib.BW_LANCZOS, tol_omega=5e-6 if prec == 1 else 1e-10, tol_lin=1e-6 if prec == 1 else 1e-10)
    klists = [ks, ks[1:3], ks]
    oms, ers, code, st = lib.bw_lowest_modes_batched(cells, klists, nm, group_cells=True, **kw)
    assert code == 0, lib.bw_last_error()
    oms_s, ers_s, code_s, st_s = lib.bw_lowest_modes_batched(cells, klists, nm, **kw)
    assert code_s == 0, lib.bw_last_error()
    scale = _omega_ref(rves[0])
    e = np.abs(oms[0] - np.array(g["omega"])) / np.maximum(np.array(g["omega"]), scale)
    print(f"[case] cell 0 vs stored oracle: max rel err {e.max():.2e}, max bound {ers[0].max():.2e}", flush=True)
    assert e.max() <= BAR[prec]
    assert np.all(e <= ers[0] * 1.5 + 1e-12)
    for i in (0, 2):
        d = np.abs(oms[i] - oms_s[i]) / np.maximum(oms_s[i], scale)
        print(f"[case] cell {i} grouped vs alone: max rel diff {d.max():.2e}", flush=True)
        assert d.max() <= BAR[prec]
        assert np.all(d <= ers[i] + ers_s[i] + 1e-12)
    assert np.array_equal(oms[1], oms_s[1]) and np.array_equal(ers[1], ers_s[1])
    print(f"[case] batched PCG sweeps grouped {st['block_iterations']} vs separate {st_s['block_iterations']}",
          flush=True)
    assert st["block_iterations"] < 0.8 * st_s["block_iterations"]
    for c in cells:
        c.close()
