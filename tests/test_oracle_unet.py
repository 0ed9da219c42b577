"""Pins of the learned-preconditioner oracle (oracle/unet.py): convolution against
scipy's periodic correlation, adjoint identities of pooling / upsampling, the
backward pass against central finite differences, invariances of the feature
map, and the round trip target -> correction."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet
from oracle.operators import Operators
from paper_2106_12487_amd import inputs
from unet_cases import random_weights


def test_layout_count():
    _, n = unet.layout()
    assert n == sum(t * ci * co + co for ci, co, t in unet.LAYERS) == 332320


def test_conv_matches_scipy_periodic_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    y = unet.conv(x, W, b)
    for s in range(2):
        for co in range(2):
            ref = np.full(x.shape[1:4], b[co])
            for ci in range(3):
                K = np.zeros((3, 3, 3))
                for t in range(27):
                    d = unet.tap_offset(t, 27)
                    K[d[0] + 1, d[1] + 1, d[2] + 1] = W[t, co, ci]
                ref += ndimage.correlate(x[s, ..., ci], K, mode="wrap")
            assert np.allclose(y[s, ..., co], ref, rtol=1e-12, atol=1e-12)


def test_pool_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 6, 8, 3))
    yc = rng.standard_normal((2, 2, 3, 4, 3))
    assert np.isclose(np.vdot(unet.pool(x), yc), np.vdot(x, unet.pool_backward(yc)))
    assert np.isclose(np.vdot(unet.upsample(yc), x), np.vdot(yc, unet.upsample_backward(x)))
    assert np.allclose(unet.pool(unet.upsample(yc)), yc)
    assert np.allclose(unet.pool(np.ones_like(x)), 1.0)


@pytest.mark.parametrize("layer", list(range(9)))
def test_backward_matches_finite_differences(layer):
    # 8^3 so that the coarsest level is 2^3 (a 1^3 level puts every tap on one
    # voxel and makes ReLU kinks within the difference step likely)
    n = (8, 8, 8)
    rng = np.random.default_rng(10 + layer)
    w = random_weights(3)
    x = rng.standard_normal((1, 512, 32))
    x[..., unet.NIN:] = 0.0
    dy = rng.standard_normal((1, 512, 16))
    g = unet.backward(w, x, dy, n)
    d = np.zeros_like(w)
    (wo, bo) = unet.layout()[0][layer]
    cout = unet.LAYERS[layer][1]
    d[wo:bo + cout] = rng.standard_normal(bo + cout - wo)
    d = unet.mask_padding(d)
    eps = 1e-8       # small enough that no ReLU of the ~3e4 units is likely to switch
    L = lambda ww: float(np.sum(dy * unet.forward(ww, x, n)))   # noqa: E731
    fd = (L(w + eps * d) - L(w - eps * d)) / (2 * eps)
    an = float(g @ d)
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (layer, fd, an)


def _ops(k):
    rve = inputs.polycrystal((8, 8, 8), (inputs.L_MM,) * 3, 6, 5, 0)
    return Operators(rve, k)


def _residuals(ops, nb, seed):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((nb, 3) + ops.n) + 1j * rng.standard_normal((nb, 3) + ops.n)
    R[..., ops.null_mask] = 0.0
    return R


def test_feature_invariances():
    ops = _ops((700.0, -300.0, 1200.0))
    R = _residuals(ops, 2, 4)
    x, _, _, _ = unet.features(ops, R)
    xs, _, _, _ = unet.features(ops, 3.7 * R)
    assert np.allclose(xs, x, atol=1e-12)
    xr, _, _, _ = unet.features(ops, np.exp(0.9j) * R)
    for b in range(2):       # phase canonicalized up to the sign ambiguity of arg/2
        same = np.allclose(xr[b, :, :6], x[b, :, :6], atol=1e-10)
        flip = np.allclose(xr[b, :, :6], -x[b, :, :6], atol=1e-10)
        assert same or flip
    assert np.allclose(np.mean(x[:, :, :6] ** 2, axis=(1, 2)) * 2, 1.0)   # unit RMS of the complex field
    ev = x[:, :, 0:6:2] + 1j * x[:, :, 1:6:2]
    assert np.all(np.abs(np.angle(np.sum(ev * ev, axis=(1, 2))) % np.pi) < 1e-9)
    # material channels: C / C0_11 and rho / rho_bar of the voxel's grain
    assert np.allclose(x[0, :, 6], ops.C_field.reshape(-1, 6, 6)[:, 0, 0] / ops.C0[0, 0])
    assert np.allclose(x[0, :, 27], ops.rho_field.ravel() / ops.rho_bar)
    assert np.all(x[:, :, 28:] == 0.0)


def test_zero_head_is_plain_preconditioner():
    ops = _ops((0.0, 0.0, 0.0))          # Gamma: also checks the null voxel
    R = _residuals(ops, 2, 5)
    w = random_weights(6)
    wo, bo = unet.layout()[0][8]
    w[wo:bo + 16] = 0.0
    z = unet.apply(ops, w, R)
    assert np.allclose(z, ops.precond(R), rtol=0, atol=1e-14 * np.abs(z).max())


def test_target_correction_round_trip():
    ops = _ops((1500.0, 0.0, -400.0))
    R = _residuals(ops, 2, 7)
    rng = np.random.default_rng(8)
    Xs = rng.standard_normal(R.shape) + 1j * rng.standard_normal(R.shape)
    t = unet.target(ops, R, Xs, pscale=0.5)
    out = np.zeros(t.shape[:2] + (16,))
    out[:, :, :6] = t
    _, Z0, phi, s = unet.features(ops, R, pscale=0.5)
    assert np.allclose(Z0 + unet.correction(ops, out, phi, s), Xs, atol=1e-10)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(20)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8)]])
    a32 = a.astype(np.float32)
    ref = torch.from_numpy(a32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(unet.bf16(a32), ref)
    assert unet.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0              # tie to even
    assert unet.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_bf16_operands_change_little():
    n = (8, 8, 8)
    rng = np.random.default_rng(21)
    w = random_weights(22)
    x = rng.standard_normal((1, 512, 32))
    x[..., unet.NIN:] = 0.0
    y = unet.forward(w, x, n)
    yb = unet.forward(w, x, n, bf16_operands=True)
    assert 1e-4 < np.linalg.norm(yb - y) / np.linalg.norm(y) < 2e-2


@pytest.mark.parametrize("k", [(700.0, -300.0, 1200.0), (0.0, 0.0, 0.0)])
def test_residual_loss_gradient_matches_finite_differences(k):
    """The chain K (K z - r) / ||r||^2 -> F^H -> output map -> backward pass against central
    differences of the residual loss along random directions in the head and in the first
    layer (a wrong conjugate, factor N or phase fails by O(1)); at Gamma the null voxel."""
    ops = _ops(k)
    R = _residuals(ops, 2, 21)
    w = random_weights(22)
    loss, g = unet.residual_loss_grad(ops, w, R, pscale=2.0)
    assert np.isclose(loss, unet.residual_loss(ops, w, R, pscale=2.0), rtol=1e-12)
    rng = np.random.default_rng(23)
    offs, _ = unet.layout()
    for layer in (8, 0):
        wo, bo = offs[layer]
        cout = unet.LAYERS[layer][1]
        d = np.zeros_like(w)
        d[wo:bo + cout] = rng.standard_normal(bo + cout - wo)
        d = unet.mask_padding(d)
        eps = 1e-7
        fd = (unet.residual_loss(ops, w + eps * d, R, 2.0) - unet.residual_loss(ops, w - eps * d, R, 2.0)) / (2 * eps)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-4 * max(abs(an), 1e-12), (layer, fd, an)
