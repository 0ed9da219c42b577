"""Learned preconditioner: U-Net, features and targets (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not part of the paper: the learned preconditioner extends the homogeneous-
reference preconditioner of Sec. 3.3 (eqs. matrixP, precond) with a network
correction,

    z = P^ r + F[ s e^{i phi} N(x) ],
    x = [ e^{-i phi} F^-1(P^ r) / s  (Re, Im of 3 components: 6 channels),
          21 scaled Voigt stiffness entries C / C0_11, scaled density rho / rho_bar,
          4 zero channels ]                               (32 channels per voxel)

with s the RMS of F^-1(P^ r) over voxels and components and phi = arg(sum of
(F^-1 P^ r)^2) / 2.  N is a 3-level U-Net of 3x3x3 periodic convolutions
(16 / 32 / 64 channels), ReLU, 2x2x2 average pooling, nearest upsampling with
skip concatenation (upsampled channels first) and a 1x1x1 head (16 outputs,
the first 6 used).  The supervised training loss is the mean squared error
between the first 6 outputs and e^{-i phi} F^-1(x* - P^ r) / s for x* = K^-1 r;
the residual loss is the batch mean of ||K z - r||^2 / ||r||^2 (Euclidean norms
of the Fourier coefficients), whose gradient with respect to conj z is
K (K z - r) / ||r||^2 since K is Hermitian.

Everything is FP64 and written for clarity (np.roll per tap).  With
bf16_operands=True every convolution first rounds its input and its weights to
bfloat16 (round to nearest even), as the matrix-core path does, while sums
stay FP64: the ReLU decisions of a network then follow those of a BF16
evaluation, so gradients can be compared element by element (otherwise units
whose pre-activation lies within the BF16 error of zero switch and move
gradient sums by O(1) per switched unit).  Parameter
layout: per layer W[tap][c_out][c_in] then b[c_out]; tap
t = 9 (d0 + 1) + 3 (d1 + 1) + (d2 + 1) reads the neighbour at offset d.

Pins (tests/test_oracle_unet.py): each convolution against
scipy.ndimage.correlate with periodic ("wrap") boundaries; pooling and
upsampling against their adjoint identities; the hand-written backward pass
against central finite differences of the forward pass; the feature map
against its scale and phase invariances; a zero head reproduces P^ r; the
bfloat16 rounding against torch's CPU conversion; the residual loss's gradient
against central finite differences of the loss.
"""
from __future__ import annotations

import numpy as np

from .fourier import fft3, ifft3

LAYERS = [(32, 16, 27), (16, 16, 27), (16, 32, 27), (32, 32, 27), (32, 64, 27), (64, 64, 27),
          (96, 32, 27), (48, 16, 27), (16, 16, 1)]          # (c_in, c_out, taps)
NIN, NOUT = 28, 6


def layout():
    """[(weight offset, bias offset)] per layer and the parameter count."""
    offs, o = [], 0
    for cin, cout, taps in LAYERS:
        offs.append((o, o + taps * cout * cin))
        o += taps * cout * cin + cout
    return offs, o


def unpack(w: np.ndarray):
    offs, _ = layout()
    out = []
    for (wo, bo), (cin, cout, taps) in zip(offs, LAYERS):
        out.append((w[wo:bo].reshape(taps, cout, cin), w[bo:bo + cout]))
    return out


def mask_padding(w: np.ndarray) -> np.ndarray:
    """Zero the weights of the padding channels (inputs 28..31 of layer 0, outputs 6..15 of the head)."""
    w = np.array(w, dtype=np.float64)
    (W0, _), (W8, b8) = unpack(w)[0], unpack(w)[8]
    W0[:, :, NIN:] = 0.0
    W8[:, NOUT:, :] = 0.0
    b8[NOUT:] = 0.0
    return w


def tap_offset(t: int, taps: int):
    if taps == 1:
        return (0, 0, 0)
    return (t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1)


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via float32; returns float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, rnd=None) -> np.ndarray:
    """Periodic correlation: y[i] = b + sum_t W[t] x[i + d_t]; x (nb, n0, n1, n2, c_in).
    `rnd` (optional) rounds the input and weights first."""
    if rnd is not None:
        x, W = rnd(x), rnd(W)
    y = np.zeros(x.shape[:-1] + (W.shape[1],))
    for t in range(W.shape[0]):
        d = tap_offset(t, W.shape[0])
        xs = np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))
        y += xs @ W[t].T
    return y + b


def conv_backward(x, W, dz, rnd=None):
    """Gradients of sum(dz * conv(x, W, b)) with respect to x, W and b (`rnd`
    rounds dz and W for the input gradient, as the matrix-core path does)."""
    dx = np.zeros_like(x)
    Wx, dzx = (rnd(W), rnd(dz)) if rnd is not None else (W, dz)
    dW = np.zeros_like(W)
    cin, cout = W.shape[2], W.shape[1]
    for t in range(W.shape[0]):
        d = tap_offset(t, W.shape[0])
        xs = np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))
        dW[t] = dz.reshape(-1, cout).T @ xs.reshape(-1, cin)
        dx += np.roll(dzx @ Wx[t], shift=d, axis=(1, 2, 3))
    return dx, dW, dz.reshape(-1, cout).sum(axis=0)


def pool(x):
    nb, n0, n1, n2, c = x.shape
    return x.reshape(nb, n0 // 2, 2, n1 // 2, 2, n2 // 2, 2, c).mean(axis=(2, 4, 6))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def upsample(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample_backward(dy):
    nb, n0, n1, n2, c = dy.shape
    return dy.reshape(nb, n0 // 2, 2, n1 // 2, 2, n2 // 2, 2, c).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def forward(w: np.ndarray, x: np.ndarray, n, cache: bool = False, bf16_operands: bool = False):
    """Network output (nb, V, 16) for inputs x (nb, V, 32)."""
    P = unpack(np.asarray(w, dtype=np.float64))
    r = bf16 if bf16_operands else None
    nb = x.shape[0]
    X0 = np.asarray(x, dtype=np.float64).reshape((nb,) + tuple(n) + (32,))
    A1 = relu(conv(X0, *P[0], r))
    S1 = relu(conv(A1, *P[1], r))
    P1 = pool(S1)
    A2 = relu(conv(P1, *P[2], r))
    S2 = relu(conv(A2, *P[3], r))
    P2 = pool(S2)
    A3 = relu(conv(P2, *P[4], r))
    B3 = relu(conv(A3, *P[5], r))
    C2 = np.concatenate([upsample(B3), S2], axis=-1)
    A4 = relu(conv(C2, *P[6], r))
    C1 = np.concatenate([upsample(A4), S1], axis=-1)
    A5 = relu(conv(C1, *P[7], r))
    O = conv(A5, *P[8], r)
    out = O.reshape(nb, -1, 16)
    if cache:
        return out, dict(X0=X0, A1=A1, S1=S1, P1=P1, A2=A2, S2=S2, P2=P2, A3=A3, B3=B3, C2=C2, A4=A4, C1=C1, A5=A5)
    return out


def backward(w: np.ndarray, x: np.ndarray, dy: np.ndarray, n, bf16_operands: bool = False) -> np.ndarray:
    """Gradient of sum(dy * forward(w, x)) with respect to the flat parameters."""
    w = np.asarray(w, dtype=np.float64)
    P = unpack(w)
    r = bf16 if bf16_operands else None
    _, c = forward(w, x, n, cache=True, bf16_operands=bf16_operands)
    nb = x.shape[0]
    g = [None] * len(LAYERS)
    dO = np.asarray(dy, dtype=np.float64).reshape((nb,) + tuple(n) + (16,))
    dA5, *g[8] = conv_backward(c["A5"], P[8][0], dO, r)
    dA5 = dA5 * (c["A5"] > 0)
    dC1, *g[7] = conv_backward(c["C1"], P[7][0], dA5, r)
    dA4 = upsample_backward(dC1[..., :32]) * (c["A4"] > 0)
    dC2, *g[6] = conv_backward(c["C2"], P[6][0], dA4, r)
    dB3 = upsample_backward(dC2[..., :64]) * (c["B3"] > 0)
    dA3, *g[5] = conv_backward(c["A3"], P[5][0], dB3, r)
    dA3 = dA3 * (c["A3"] > 0)
    dP2, *g[4] = conv_backward(c["P2"], P[4][0], dA3, r)
    dS2 = (dC2[..., 64:] + pool_backward(dP2)) * (c["S2"] > 0)
    dA2, *g[3] = conv_backward(c["A2"], P[3][0], dS2, r)
    dA2 = dA2 * (c["A2"] > 0)
    dP1, *g[2] = conv_backward(c["P1"], P[2][0], dA2, r)
    dS1 = (dC1[..., 32:] + pool_backward(dP1)) * (c["S1"] > 0)
    dA1, *g[1] = conv_backward(c["A1"], P[1][0], dS1, r)
    dA1 = dA1 * (c["A1"] > 0)
    _, *g[0] = conv_backward(c["X0"], P[0][0], dA1, r)
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in g])


# ---------------------------------------------------------------------------
# Bloch residuals <-> channels
# ---------------------------------------------------------------------------
def material_channels(ops) -> np.ndarray:
    """(V, 22): the 21 upper-triangle Voigt entries / C0_11 and rho / rho_bar of each voxel."""
    iu = np.triu_indices(6)
    C = ops.C_field.reshape(-1, 6, 6)[:, iu[0], iu[1]] / ops.C0[0, 0]
    rho = ops.rho_field.reshape(-1, 1) / ops.rho_bar
    return np.concatenate([C, rho], axis=1)


def features(ops, R: np.ndarray, pscale: float = 1.0):
    """Network inputs (nb, V, 32), P^ R, phases phi and scales s for residuals R (nb, 3, n0, n1, n2)."""
    nb = R.shape[0]
    Z0 = pscale * ops.precond(R)
    E = ifft3(Z0).reshape(nb, 3, -1)
    phi = 0.5 * np.angle(np.sum(E * E, axis=(1, 2)))
    s = np.sqrt(np.mean(np.abs(E) ** 2, axis=(1, 2)))
    En = E * (np.exp(-1j * phi) / s)[:, None, None]
    V = E.shape[2]
    x = np.zeros((nb, V, 32))
    x[:, :, 0:6:2] = En.real.transpose(0, 2, 1)
    x[:, :, 1:6:2] = En.imag.transpose(0, 2, 1)
    x[:, :, 6:28] = material_channels(ops)[None]
    return x, Z0, phi, s


def correction(ops, out: np.ndarray, phi, s) -> np.ndarray:
    """F[ s e^{i phi} (o_{2c} + i o_{2c+1}) ] for network outputs (nb, V, 16)."""
    nb = out.shape[0]
    D = (out[:, :, 0:6:2] + 1j * out[:, :, 1:6:2]).transpose(0, 2, 1)
    D = D * (s * np.exp(1j * phi))[:, None, None]
    return fft3(D.reshape((nb, 3) + ops.n))


def apply(ops, w: np.ndarray, R: np.ndarray, pscale: float = 1.0, bf16_operands: bool = False) -> np.ndarray:
    """Learned preconditioner z for residuals R; zero on the xi + k = 0 voxel."""
    x, Z0, phi, s = features(ops, R, pscale)
    z = Z0 + correction(ops, forward(w, x, ops.n, bf16_operands=bf16_operands), phi, s)
    z[..., ops.null_mask] = 0.0
    return z


def target(ops, R: np.ndarray, Xs: np.ndarray, pscale: float = 1.0) -> np.ndarray:
    """Normalized real-space training target (nb, V, 6) for pairs (R, X* = K^-1 R)."""
    _, Z0, phi, s = features(ops, R, pscale)
    nb = R.shape[0]
    D = ifft3(Xs - Z0).reshape(nb, 3, -1) * (np.exp(-1j * phi) / s)[:, None, None]
    t = np.zeros((nb, D.shape[2], 6))
    t[:, :, 0::2] = D.real.transpose(0, 2, 1)
    t[:, :, 1::2] = D.imag.transpose(0, 2, 1)
    return t


def loss(ops, w, R, Xs, pscale: float = 1.0) -> float:
    """Mean squared error of the network on pairs (R, X*)."""
    x, _, _, _ = features(ops, R, pscale)
    out = forward(w, x, ops.n)
    return float(np.mean((out[:, :, :6] - target(ops, R, Xs, pscale)) ** 2))


def residual_loss(ops, w, R, pscale: float = 1.0, bf16_operands: bool = False) -> float:
    """Mean over the batch of ||K z - R||^2 / ||R||^2 with z = apply(ops, w, R)."""
    nb = R.shape[0]
    E = ops.apply_K(apply(ops, w, R, pscale, bf16_operands)) - R
    return float(np.mean(np.sum(np.abs(E.reshape(nb, -1)) ** 2, axis=1) /
                         np.sum(np.abs(R.reshape(nb, -1)) ** 2, axis=1)))


def residual_loss_grad(ops, w, R, pscale: float = 1.0, bf16_operands: bool = False):
    """The residual loss and its gradient with respect to the parameters: g = K (K z - R) /
    ||R||^2 (the derivative with respect to conj z; zero on the xi + k = 0 voxel, where K
    vanishes), h = F^H g (the adjoint of the unnormalized forward DFT, N times the
    normalized inverse), and for the output o_{2c} + i o_{2c+1} that enters z as
    F[s e^{i phi} (.)], dL/do_{2c} = (2 / nb) s Re(e^{-i phi} h_c), dL/do_{2c+1} = (2 / nb) s
    Im(e^{-i phi} h_c); then the network's backward pass."""
    nb = R.shape[0]
    x, Z0, phi, s = features(ops, R, pscale)
    out = forward(w, x, ops.n, bf16_operands=bf16_operands)
    z = Z0 + correction(ops, out, phi, s)
    z[..., ops.null_mask] = 0.0
    E = ops.apply_K(z) - R
    rr = np.sum(np.abs(R.reshape(nb, -1)) ** 2, axis=1)
    loss = float(np.mean(np.sum(np.abs(E.reshape(nb, -1)) ** 2, axis=1) / rr))
    G = ops.apply_K(E) / rr[:, None, None, None, None]
    N = int(np.prod(ops.n))
    H = (N * ifft3(G)).reshape(nb, 3, -1) * (np.exp(-1j * phi) * s)[:, None, None]
    dy = np.zeros_like(out)
    dy[:, :, 0:6:2] = (2.0 / nb) * H.real.transpose(0, 2, 1)
    dy[:, :, 1:6:2] = (2.0 / nb) * H.imag.transpose(0, 2, 1)
    return loss, backward(w, x, dy, ops.n, bf16_operands=bf16_operands)
