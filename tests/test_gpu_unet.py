"""GPU parity of the learned preconditioner (BF16 matrix-core U-Net, FP32
accumulation) against the FP64 oracle (oracle/unet.py), and of flexible PCG.

Bars: network outputs agree with the plain FP64 oracle to cosine > 0.999 and
relative 2-norm error < 1e-2 (BF16 operands carry 8 significant bits, so each
product is exact to ~4e-3 and errors average over the 27 * c_in terms of a
convolution).  Gradients and preconditioned vectors are compared with the
oracle evaluated on BF16-rounded convolution operands (oracle.unet.bf16), so
that both sides take the same ReLU decisions (against the plain FP64 oracle,
the ~0.5% of units whose pre-activation lies within the BF16 error of zero
switch and move gradient sums by ~10%).  The emulation is exact up to FP32
against FP64 accumulation, which still rounds ~6e-4 of the activations to a
neighbouring BF16 value; on the 8^3 case no such element reaches the output
(bar 1e-5 on outputs and gradients); on larger grids one such element at the
4x coarser level spreads over the whole field (outputs: bar 1e-2), and the
shifted activations again switch a few ReLUs in the backward pass (gradients:
1e-2 on 8x12x16, 1e-1 with cosine > 0.995 on 16^3; a wrong tap, transpose or
channel offset gives errors of order 1).
Padded channels are exactly zero; flexible PCG with a zero network follows
plain PCG.
"""
import numpy as np
import pytest

from oracle import unet
from oracle.operators import Operators
from paper_2106_12487_amd import inputs
from unet_cases import random_weights

pytestmark = pytest.mark.gpu
L = inputs.L_MM


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _f32(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").contiguous()


def _c64(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(torch.complex64).contiguous()


def _cmp(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    return rel, cos


def _ccmp(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cell(lib, n, grains=8, index=0):
    rve = inputs.polycrystal(n, (L,) * 3, grains, 5, index)
    return rve, lib.Rve.from_inputs(rve, lib.BW_MIXED)


def test_param_count_and_weights_roundtrip(lib):
    _torch()
    _, n = unet.layout()
    assert lib.bw_unet_param_count() == n
    net = lib.UNet(seed=3)
    w0 = net.get_weights()
    wo, bo = unet.layout()[0][8]
    assert np.all(w0[wo:bo + 16] == 0.0)                  # zero head: untrained net adds nothing
    assert np.all(w0[unet.layout()[0][0][1]:unet.layout()[0][1][0]] == 0.0)   # zero biases
    w = random_weights(4)
    wp = w.copy()
    wp[unet.layout()[0][0][0]] += 0.0
    net.set_weights(w)
    assert np.array_equal(net.get_weights(), w.astype(np.float32))
    with pytest.raises(lib.BlochwaveError):
        net.set_weights(w[:-1])
    bad = w.copy()
    bad[7] = np.nan
    with pytest.raises(lib.BlochwaveError):
        net.set_weights(bad)
    net.close()


@pytest.mark.parametrize("n,nb,tol,gtol", [((8, 8, 8), 2, 1e-5, 1e-5), ((8, 12, 16), 1, 1e-2, 1e-2),
                                           ((16, 16, 16), 1, 1e-2, 1e-1)])
def test_net_forward_backward_parity(lib, n, nb, tol, gtol):
    torch = _torch()
    V = int(np.prod(n))
    w = random_weights(5)
    net = lib.UNet()
    net.set_weights(w)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((nb, V, 32))
    x[..., unet.NIN:] = 0.0
    y = torch.zeros((nb, V, 16), dtype=torch.float32, device="cuda")
    lib.bw_unet_net_forward(net, n, _f32(x), y)
    torch.cuda.synchronize()
    yg = y.cpu().numpy()
    yo = unet.forward(w, x, n)
    assert np.all(yg[..., unet.NOUT:] == 0.0)
    rel, cos = _cmp(yg[..., :6], yo[..., :6])
    assert rel < 1e-2 and cos > 0.999, (rel, cos)
    dy = rng.standard_normal((nb, V, 16))
    dy[..., unet.NOUT:] = 0.0
    gg = lib.bw_unet_net_backward(net, n, _f32(x), _f32(dy))
    go = unet.backward(w, x, dy, n, bf16_operands=True)
    yb = unet.forward(w, x, n, bf16_operands=True)
    rel, cos = _cmp(yg[..., :6], yb[..., :6])
    assert rel < tol, rel
    per_layer = []
    for li, ((wo, bo), (cin, cout, taps)) in enumerate(zip(unet.layout()[0], unet.LAYERS)):
        per_layer.append(_cmp(gg[wo:bo], go[wo:bo]) + _cmp(gg[bo:bo + cout], go[bo:bo + cout]))
        print(f"layer {li}: W rel {per_layer[-1][0]:.2e} cos {per_layer[-1][1]:.6f}  "
              f"b rel {per_layer[-1][2]:.2e} cos {per_layer[-1][3]:.6f}")
    rel, cos = _cmp(gg, go)
    assert rel < gtol and cos > 0.995, (rel, cos)
    for li, (rw, cw, rb, cb) in enumerate(per_layer):
        assert rw < 2 * gtol and rb < 2 * gtol and cw > 0.995 and cb > 0.995, (li, rw, rb, cw, cb)
    net.close()


@pytest.mark.parametrize("k", [(700.0, -300.0, 1200.0), (0.0, 0.0, 0.0)])
def test_learned_apply_parity(lib, k):
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16))
    ops = Operators(rve, k)
    w = random_weights(7)
    net = lib.UNet()
    net.set_weights(w)
    rng = np.random.default_rng(8)
    r = rng.standard_normal((2, 3) + rve.n) + 1j * rng.standard_normal((2, 3) + rve.n)
    r[..., ops.null_mask] = 0.0
    z = torch.zeros((2, 3) + rve.n, dtype=torch.complex64, device="cuda")
    lib.bw_unet_apply(net, R, k, _c64(r), z)
    zg = z.cpu().numpy()
    zo = unet.apply(ops, w, r)
    corr = zo - ops.precond(r)
    assert np.linalg.norm(corr) > 0.05 * np.linalg.norm(zo)      # the network contributes
    assert _ccmp(zg, zo) < 2e-2 * np.linalg.norm(corr) / np.linalg.norm(zo) + 1e-5
    zb = unet.apply(ops, w, r, bf16_operands=True)
    assert _ccmp(zg, zb) < 1e-2 * np.linalg.norm(corr) / np.linalg.norm(zo) + 1e-5
    assert np.all(zg[..., ops.null_mask] == 0)
    net.close()
    R.close()


def test_train_step_parity(lib):
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=1)
    ks = np.array([[500.0, 0.0, 0.0], [900.0, 900.0, -300.0]])
    w = random_weights(9)
    net = lib.UNet()
    net.set_weights(w)
    rng = np.random.default_rng(10)
    r = rng.standard_normal((2, 3) + rve.n) + 1j * rng.standard_normal((2, 3) + rve.n)
    xs = 1e-12 * (rng.standard_normal((2, 3) + rve.n) + 1j * rng.standard_normal((2, 3) + rve.n))
    lr = 1e-3
    loss_g = lib.bw_unet_train_step(net, R, ks, _c64(r), _c64(xs), lr)
    # oracle loss and gradient, sample by sample (each sample has its own k)
    losses, grads = [], []
    for b in range(2):
        ops = Operators(rve, ks[b])
        x, _, _, _ = unet.features(ops, r[b:b + 1])
        out = unet.forward(w, x, ops.n)
        t = unet.target(ops, r[b:b + 1], xs[b:b + 1])
        losses.append(np.mean((out[..., :6] - t) ** 2))
        dy = np.zeros_like(out)
        dy[..., :6] = 2.0 * (out[..., :6] - t) / (2 * out.shape[1] * 6)
        grads.append(unet.backward(w, x, dy, ops.n))
    loss_o = float(np.mean(losses))
    assert abs(loss_g - loss_o) < 2e-2 * loss_o, (loss_g, loss_o)
    g = grads[0] + grads[1]
    step = net.get_weights().astype(np.float64) - w
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    # Adam's first step moves each weight by lr against the sign of its gradient
    agree = np.mean(np.sign(step[big]) == -np.sign(g[big]))
    assert agree > 0.98, agree
    assert np.allclose(np.abs(step[big]), lr, rtol=1e-2)
    net.close()
    R.close()


def test_train_step_residual_parity(lib):
    """The residual-loss step against the oracle's loss and gradient (BF16-rounded
    convolution operands on both sides): loss to 1e-2, and Adam's first step moves every
    weight with a sizeable gradient by lr against the oracle gradient's sign."""
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=6)
    ks = np.array([[500.0, 0.0, 0.0], [900.0, 900.0, -300.0]])
    w = random_weights(19)
    net = lib.UNet()
    net.set_weights(w)
    rng = np.random.default_rng(20)
    r = rng.standard_normal((2, 3) + rve.n) + 1j * rng.standard_normal((2, 3) + rve.n)
    lr = 1e-3
    loss_g = lib.bw_unet_train_step_residual(net, R, ks, _c64(r), lr)
    losses, grads = [], []
    for b in range(2):
        ops = Operators(rve, ks[b])
        lb, gb = unet.residual_loss_grad(ops, w, r[b:b + 1], bf16_operands=True)
        losses.append(lb)
        grads.append(gb / 2.0)                 # the batch mean over the two samples
    loss_o = float(np.mean(losses))
    print(f"\n[case] residual loss GPU {loss_g:.6e} oracle {loss_o:.6e}", flush=True)
    assert abs(loss_g - loss_o) < 1e-2 * loss_o, (loss_g, loss_o)
    g = grads[0] + grads[1]
    step = net.get_weights().astype(np.float64) - w
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    agree = np.mean(np.sign(step[big]) == -np.sign(g[big]))
    assert agree > 0.98, agree
    assert np.allclose(np.abs(step[big]), lr, rtol=1e-2)
    net.close()
    R.close()


def test_training_reduces_loss(lib):
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=2)
    k = (800.0, 200.0, 0.0)
    rng = np.random.default_rng(11)
    b = _c64(rng.standard_normal((4, 3) + rve.n) + 1j * rng.standard_normal((4, 3) + rve.n))
    x = torch.zeros_like(b)
    code, it, rr = lib.bw_pcg_solve(R, k, b, x, 1e-6)
    assert code == 0
    net = lib.UNet(seed=1)
    losses = [lib.bw_unet_train_step(net, R, k, b, x, 2e-3) for _ in range(40)]
    assert losses[-1] < 0.7 * losses[0], (losses[0], losses[-1])
    net.close()
    R.close()


def _rhs(rve, ops, nb, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((nb, 3) + rve.n) + 1j * rng.standard_normal((nb, 3) + rve.n)
    b[..., ops.null_mask] = 0.0
    return b


@pytest.mark.parametrize("k", [(1200.0, -400.0, 300.0), (0.0, 0.0, 0.0)])
def test_fpcg_zero_network_follows_pcg(lib, k):
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=3)
    ops = Operators(rve, k)
    b = _c64(_rhs(rve, ops, 3, 12))
    x1 = torch.zeros_like(b)
    code, it1, rr1 = lib.bw_pcg_solve(R, k, b, x1, 1e-6)
    assert code == 0
    net = lib.UNet()
    net.set_weights(np.zeros(lib.bw_unet_param_count()))
    for nn in (None, net):
        x2 = torch.zeros_like(b)
        code, it2, rr2, fb = lib.bw_pcg_solve_learned(R, nn, k, b, x2, 1e-6)
        assert code == 0 and np.all(rr2 <= 1e-6) and np.all(fb == 0)
        assert np.all(np.abs(it2 - it1) <= 2), (it1, it2)
        d = (x2 - x1).cpu().numpy()
        assert np.linalg.norm(d) <= 1e-4 * np.linalg.norm(x1.cpu().numpy())
    net.close()
    R.close()


def test_fpcg_falls_back_on_a_bad_network(lib):
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=4)
    k = (600.0, 600.0, 600.0)
    ops = Operators(rve, k)
    b = _c64(_rhs(rve, ops, 2, 13))
    net = lib.UNet()
    net.set_weights(random_weights(14, head_scale=300.0, bias_scale=30.0))
    x = torch.zeros_like(b)
    code, it, rr, fb = lib.bw_pcg_solve_learned(R, net, k, b, x, 1e-6, maxit=2000)
    assert code == lib.BW_ESTALL and np.all(rr <= 1e-6)      # valid results, stall reported
    assert np.all(fb >= 1), fb
    net.close()
    R.close()


def test_learned_argument_errors(lib):
    torch = _torch()
    net = lib.UNet()
    rve = inputs.polycrystal((8, 8, 6), (L,) * 3, 4, 5, 0)
    R = lib.Rve.from_inputs(rve, lib.BW_MIXED)
    r = torch.zeros((1, 3) + rve.n, dtype=torch.complex64, device="cuda")
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_unet_apply(net, R, (1.0, 0, 0), r, torch.zeros_like(r))
    assert e.value.code == lib.BW_EUNSUPPORTED
    R.close()
    rve = inputs.polycrystal((8, 8, 8), (L,) * 3, 4, 5, 0)
    R64 = lib.Rve.from_inputs(rve, lib.BW_FP64)
    r = torch.zeros((1, 3) + rve.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_unet_apply(net, R64, (1.0, 0, 0), r, torch.zeros_like(r))
    assert e.value.code == lib.BW_EINVAL
    R64.close()
    # Gamma: b must vanish on the null voxel
    R = lib.Rve.from_inputs(rve, lib.BW_MIXED)
    b = torch.ones((1, 3) + rve.n, dtype=torch.complex64, device="cuda")
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_pcg_solve_learned(R, net, (0.0, 0.0, 0.0), b, torch.zeros_like(b), 1e-6)
    assert e.value.code == lib.BW_EINVAL
    R.close()
    net.close()


def test_trained_network_gain_is_measured(lib, capsys):
    """Train on PCG trajectories of 4 cells (16^3) and compare flexible PCG with the
    network against the plain preconditioner on 2 unseen cells.  Reports the
    iteration and wall-time ratios; requires convergence to rtol with the network
    and no more than 2 extra iterations on average (the plain preconditioner
    already needs ~12 iterations at 1e-6 on these Cu cells, and the trained
    network has not been seen to reduce that)."""
    _torch()
    from paper_2106_12487_amd import train_precond as tp
    cells = [tp._cell(16, 8, i) for i in range(4)]
    pairs = tp.make_pairs(cells, 2, 4)
    net = lib.UNet(seed=2)
    losses = tp.train(net, cells, pairs, 300, 1e-3)
    assert np.all(np.isfinite(losses))
    ev = tp.evaluate(net, [tp._cell(16, 8, 1000 + i) for i in range(2)], 2, 4, rtol=1e-6)
    with capsys.disabled():
        print(f"\n[gain] plain {ev['plain_iters']:.2f} it, learned {ev['learned_iters']:.2f} it "
              f"(ratio {ev['iter_ratio']:.3f}), time ratio {ev['time_ratio']:.2f}, fallbacks {ev['fallbacks']}")
    for row in ev["rows"]:
        assert row["learned"]["code"] in (lib.BW_OK, lib.BW_ESTALL) and row["learned"]["relres"] <= 1e-6
    assert ev["learned_iters"] <= ev["plain_iters"] + 2
    net.close()


def test_lanczos_with_learned_preconditioner(lib):
    """BW_LEARNED in bw_lowest_modes: with a zero network (z = P^ r) the flexible inner
    solves follow plain PCG and the frequencies equal the plain mixed path's to 1e-5 with
    bounds below the target, at Gamma too; a trained-looking random network still gives
    valid results (BW_OK or BW_ESTALL); wrong uses are refused."""
    torch = _torch()
    rve, R = _cell(lib, (16, 16, 16), index=7)
    ks = np.array([[0.0, 0.0, 0.0], [0.31, -0.12, 0.4]]) * np.pi / L
    kw = dict(method=lib.BW_LANCZOS, tol_omega=5e-6, tol_lin=1e-6)
    w0, e0, c0, _ = lib.bw_lowest_modes(R, ks, 8, **kw)
    assert c0 == 0
    net = lib.UNet()
    net.set_weights(np.zeros(lib.bw_unet_param_count()))
    print("\n[case] Lanczos, learned preconditioner (zero network)", flush=True)
    w1, e1, c1, st = lib.bw_lowest_modes(R, ks, 8, net=net, **kw)
    assert c1 == 0, lib.bw_last_error()
    scale = 2 * np.pi / L * np.sqrt(inputs.c21_to_voigt(rve.C21[0])[3, 3] / rve.rho[0])
    assert np.abs(w1 - w0).max() <= 1e-5 * max(scale, w0.max()) and e1.max() <= 5e-6
    net.set_weights(random_weights(31))
    w2, e2, c2, _ = lib.bw_lowest_modes(R, ks, 8, net=net, **kw)
    assert c2 in (lib.BW_OK, lib.BW_ESTALL) and e2.max() <= 5e-6
    assert np.abs(w2 - w0).max() <= 2e-5 * max(scale, w0.max())
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_lowest_modes(R, ks, 8, method=lib.BW_SUBSPACE, block=12, net=net)
    assert e.value.code == lib.BW_EUNSUPPORTED
    R64 = lib.Rve.from_inputs(rve, lib.BW_FP64)
    with pytest.raises(lib.BlochwaveError) as e:
        lib.bw_lowest_modes(R64, ks, 8, net=net, **kw)
    assert e.value.code == lib.BW_EINVAL
    R64.close()
    net.close()
    R.close()
