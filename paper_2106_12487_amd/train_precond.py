"""Train the learned preconditioner on the GPU with the library's own kernels.

Training data come from the method's plain PCG (Sec. 3.3, Algorithm "InvA"):
for a right-hand side b and its solution x* (solved to `tol`), the iterates x_j
of the same solve give residuals r_j = b - K x_j whose exact correction is
K^-1 r_j = x* - x_j.  The default loss is the residual loss ||K z - r|| / ||r||
of the preconditioned residual (bw_unet_train_step_residual, which needs the r_j
alone); --loss mse trains on (r_j, x* - x_j) with the mean squared error of the
normalized real-space correction (bw_unet_train_step).  The network is evaluated
by flexible PCG on unseen cells against the plain preconditioner.

Usage (the learned-preconditioner workload: 64^3 Cu cells of 16-256 grains,
unseen 96^3 / 216-grain and 128^3 / 512-grain evaluation cells):
    python -m paper_2106_12487_amd.train_precond --cells 16 --steps 600 --eval-n 128 --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import blochwave as bw
from . import inputs

SNAPSHOTS = (0, 1, 2, 4, 7, 11, 16)


def _cell(n, grains, index, config=5):
    rve = inputs.polycrystal((n, n, n), (inputs.L_MM,) * 3, grains, config, index)
    return rve, bw.Rve.from_inputs(rve, bw.BW_MIXED)


def training_cell(index):
    """Cell `index` of the learned-preconditioner workload (64^3 Cu, 16-256 grains)."""
    rve = inputs.workload_rve(5, index)
    return rve, bw.Rve.from_inputs(rve, bw.BW_MIXED)


def eval_cell(n, index):
    """An unseen Cu cell with the training cells' mean grain volume (4096 voxels)."""
    return _cell(n, max(2, round(n ** 3 / 4096)), 1000 + index)


def _rhs(rve, nb, seed):
    import torch
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((nb, 3) + rve.n) + 1j * rng.standard_normal((nb, 3) + rve.n)
    return torch.from_numpy(b).to("cuda").to(torch.complex64).contiguous()


def _kpoints(rng, count):
    ks = np.asarray(inputs.workload_kpoints(2))
    return ks[rng.integers(1, len(ks), count)]          # skip Gamma (singular K)


def make_pairs(cells, kpc: int, nrhs: int, tol: float = 1e-7, seed: int = 0):
    """(cell index, k, r_j, x* - x_j) for every cell, kpc wave vectors per cell
    and the PCG iterates listed in SNAPSHOTS."""
    import torch
    rng = np.random.default_rng(seed)
    pairs = []
    for ci, (rve, R) in enumerate(cells):
        for k in _kpoints(rng, kpc):
            b = _rhs(rve, nrhs, int(rng.integers(1 << 30)))
            xs = torch.zeros_like(b)
            bw.bw_pcg_solve(R, k, b, xs, tol)
            for j in SNAPSHOTS:
                xj = torch.zeros_like(b)
                if j > 0:
                    bw.bw_pcg_solve(R, k, b, xj, 1e-30, maxit=j)
                Kx = torch.empty_like(b)
                bw.bw_apply_K(R, k, xj, Kx)
                pairs.append((ci, k, (b - Kx).contiguous(), (xs - xj).contiguous()))
    return pairs


def train(net, cells, pairs, steps: int, lr: float = 1e-3, seed: int = 0, log_every: int = 0,
          loss: str = "residual"):
    """Adam steps on randomly drawn pairs; the learning rate decays by 10x over the run."""
    rng = np.random.default_rng(seed)
    losses = []
    for it in range(steps):
        ci, k, r, e = pairs[int(rng.integers(len(pairs)))]
        rate = lr * (0.1 ** (it / max(steps - 1, 1)))
        if loss == "residual":
            losses.append(bw.bw_unet_train_step_residual(net, cells[ci][1], k, r, rate))
        else:
            losses.append(bw.bw_unet_train_step(net, cells[ci][1], k, r, e, rate))
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(f"[train] step {it} loss {np.mean(losses[-log_every:]):.4e}", flush=True)
    return losses


def evaluate(net, cells, kpc: int, nrhs: int, rtol: float = 1e-6, seed: int = 1):
    """Flexible-PCG iterations / wall time with the network against the plain preconditioner."""
    import torch
    rng = np.random.default_rng(seed)
    rows = []
    for ci, (rve, R) in enumerate(cells):
        for k in _kpoints(rng, kpc):
            b = _rhs(rve, nrhs, int(rng.integers(1 << 30)))
            res = {}
            for name, nn in (("plain", None), ("learned", net)):
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                code, it, rr, fb = bw.bw_pcg_solve_learned(R, nn, k, b, x, rtol)
                torch.cuda.synchronize()
                res[name] = dict(iters=it.tolist(), seconds=time.perf_counter() - t0, fallbacks=fb.tolist(),
                                 relres=float(rr.max()), code=code)
            rows.append(dict(cell=ci, k=k.tolist(), **res))
    pi = np.mean([np.mean(r["plain"]["iters"]) for r in rows])
    li = np.mean([np.mean(r["learned"]["iters"]) for r in rows])
    pt = np.sum([r["plain"]["seconds"] for r in rows])
    lt = np.sum([r["learned"]["seconds"] for r in rows])
    return dict(rows=rows, plain_iters=pi, learned_iters=li, iter_ratio=li / pi, plain_seconds=pt,
                learned_seconds=lt, time_ratio=lt / pt,
                fallbacks=int(sum(sum(r["learned"]["fallbacks"]) for r in rows)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64, help="training grid (64: the workload's cells)")
    ap.add_argument("--grains", type=int, default=0, help="grains per training cell (0: the workload's 16-256)")
    ap.add_argument("--cells", type=int, default=8)
    ap.add_argument("--loss", default="residual", choices=("residual", "mse"))
    ap.add_argument("--kpc", type=int, default=4, help="wave vectors per training cell")
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-cells", type=int, default=2)
    ap.add_argument("--eval-n", type=int, default=0, help="grid of the unseen evaluation cells (default --n)")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    t0 = time.perf_counter()
    if a.grains == 0 and a.n == 64:
        cells = [training_cell(i) for i in range(a.cells)]
    else:
        cells = [_cell(a.n, a.grains or max(2, round(a.n ** 3 / 4096)), i) for i in range(a.cells)]
    pairs = make_pairs(cells, a.kpc, a.nrhs)
    print(f"[train] {len(pairs)} batches of {a.nrhs} pairs in {time.perf_counter() - t0:.1f} s", flush=True)
    net = bw.UNet(seed=1)
    t1 = time.perf_counter()
    train(net, cells, pairs, a.steps, a.lr, log_every=max(a.steps // 10, 1), loss=a.loss)
    print(f"[train] {a.steps} steps in {time.perf_counter() - t1:.1f} s", flush=True)
    en = a.eval_n or a.n
    ev_cells = [eval_cell(en, i) for i in range(a.eval_cells)]
    ev = evaluate(net, ev_cells, 3, a.nrhs)
    print(json.dumps({k: v for k, v in ev.items() if k != "rows"}), flush=True)
    if a.out:
        np.save(a.out, net.get_weights())


if __name__ == "__main__":
    main()
