"""Several cells of uneven size in one bw_lowest_modes_batched call: each cell's
results equal those of its own bw_lowest_modes call bit for bit (same kernels,
deterministic reductions), and a failing cell is reported by index."""
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
