"""bw_apply_K_noalloc (the allocation-free K apply) against bw_apply_K through the
C ABI: bit-for-bit equal outputs (same kernels, identical wave-number tables) on
consecutive calls, the second with a smaller input, in both precisions and on the
paths the grid selects (register kernels, the 64^3 plane pass, the 128 x 128 slab
path); requests beyond the scratch area are refused."""
import numpy as np
import pytest

from paper_2106_12487_amd import inputs

pytestmark = pytest.mark.gpu
L = inputs.L_MM


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _rand(shape, seed, dt):
    torch = _torch()
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return torch.from_numpy(a).to("cuda").to(dt).contiguous()


CELLS = [((16, 16, 16), 8, 0), ((16, 16, 16), 8, 1), ((64, 64, 64), 16, 1), ((4, 128, 128), 5, 1),
         ((12, 8, 24), 5, 0)]


@pytest.mark.parametrize("n,grains,prec", CELLS)
def test_noalloc_matches_apply_K_on_consecutive_calls(lib, n, grains, prec):
    torch = _torch()
    rve = inputs.polycrystal(n, (L, 1.1 * L, 0.9 * L), grains, 93, 0)
    R = lib.Rve.from_inputs(rve, prec)
    dt = R.complex_dtype
    word = 16 if prec == 0 else 8
    nvox = int(np.prod(n))
    cap = (64 << 20) // (6 * nvox * word + 1024)
    calls = [(min(3, cap), [0.31, -0.12, 0.4], 1), (1, [1.0, 0.0, 0.0], 2), (1, [0.0, 0.0, 0.0], 3)]
    for nv, kk, seed in calls:
        k = np.array(kk) * np.pi / np.array(rve.L)
        print(f"\n[case] noalloc n={n} prec={prec} nvec={nv} k={kk}", flush=True)
        u = _rand((nv, 3) + n, seed, dt)
        y_ref = torch.empty_like(u)
        y = torch.full_like(u, float("nan"))
        lib.bw_apply_K(R, k, u, y_ref)
        lib.bw_apply_K_noalloc(R, k, u, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
    R.close()


def test_noalloc_refuses_requests_beyond_the_scratch_area(lib):
    torch = _torch()
    rve = inputs.polycrystal((64, 64, 64), (L, L, L), 8, 93, 1)
    R = lib.Rve.from_inputs(rve, 0)
    u = _rand((4, 3, 64, 64, 64), 5, R.complex_dtype)     # 4 x 6 x 64^3 x 16 B = 96 MiB > 64 MiB
    y = torch.empty_like(u)
    print("\n[case] noalloc beyond the scratch area", flush=True)
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_apply_K_noalloc(R, [0.1 * np.pi / L, 0.0, 0.0], u, y)
    assert e.value.code == lib.BW_EINVAL and "scratch" in str(e.value)
    # one vector fits (24 MiB) and matches
    y1 = torch.empty_like(u[:1])
    y0 = torch.empty_like(u[:1])
    lib.bw_apply_K_noalloc(R, [0.1 * np.pi / L, 0.0, 0.0], u[:1].contiguous(), y1)
    lib.bw_apply_K(R, [0.1 * np.pi / L, 0.0, 0.0], u[:1].contiguous(), y0)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    R.close()
