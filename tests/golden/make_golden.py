"""Writes the stored oracle eigenfrequencies that the GPU parity tests compare to.

Calls only the CPU oracle (oracle/) and the seeded input generators; nothing
here touches the HIP path.  Usage:

    python tests/golden/make_golden.py cu16      # 16^3, 8 grains, all 11 k on Gamma-X
    python tests/golden/make_golden.py cu64      # 64^3, 64 grains, sampled k of the path (Lanczos)
    python tests/golden/make_golden.py cual32    # 32^3 Cu/Al cell of the uneven workload, 4 k (Lanczos)
    python tests/golden/make_golden.py fibre128  # 128 x 128 x 1 epoxy / 55% circular carbon fibres, 4 k (Lanczos)

Output: tests/golden/<name>.json with the wave vectors (rad/m), omega (rad/s)
and the oracle settings.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2106_12487_amd import inputs  # noqa: E402
from oracle import solvers  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def nearest_path_indices(config, labels):
    ks = inputs.workload_kpoints(config)
    P = inputs.sc_points(inputs.L_MM)
    return [int(np.argmin(np.linalg.norm(ks - P[c], axis=1))) for c in labels]


def run(name):
    method = "subspace"
    if name == "cu16":
        cfg, nmodes, block = 1, 6, 12
        idx = list(range(11))
    elif name == "cu64":
        cfg, nmodes, block = 2, 12, 16
        ks = inputs.workload_kpoints(2)
        idx = nearest_path_indices(2, "GXMR")
        mid = [int(np.argmin(np.linalg.norm(ks - 0.5 * inputs.sc_points(inputs.L_MM)["X"], axis=1)))]
        idx = sorted(set(idx + mid))
        method = "lanczos"
    elif name == "cual32":
        cfg, nmodes, block = 3, 8, 16
        idx = [0, 5, 11, 17]
        method = "lanczos"
    elif name == "fibre128":
        # Sec. 4.3 workload: 90 k on M-Gamma-X-M; wave vectors off the symmetry points
        # (no symmetry-forced degeneracy, which a single-vector Lanczos would find once)
        cfg, nmodes, block = None, 10, 16
        idx = [18, 50, 60, 75]
        method = "lanczos"
    else:
        raise SystemExit(f"unknown golden set {name}")
    if cfg is None:
        rve = inputs.fibre_composite(128, inputs.L_MM, "circle", 0.55)
        ks = inputs.kpath("MGXM", 90, inputs.L_MM)[idx]
    else:
        rve = inputs.workload_rve(cfg, 0)
        ks = inputs.workload_kpoints(cfg)[idx]
    out = dict(name=name, config=cfg, nmodes=nmodes, block=block, method=method, tol_eig=1e-12, tol_lin=1e-12,
               k_index=idx, k=ks.tolist(), omega=[], seconds=[], pcg_iters=[], outer=[])
    path = os.path.join(HERE, f"{name}.json")
    for i, k in enumerate(ks):
        t = time.time()
        st = []
        w = solvers.lowest_modes(rve, k[None], nmodes, method=method, block=block,
                                 tol_eig=1e-12, tol_lin=1e-12, dense_max=0, warm_start=False, stats=st)
        out["omega"].append(w[0].tolist())
        out["pcg_iters"].append(int(st[0]["pcg_iters"]))
        out["outer"].append(int(st[0].get("outer", st[0].get("restarts", 0))))
        out["seconds"].append(time.time() - t)
        print(f"{name} k[{idx[i]}] {time.time() - t:.1f}s omega[:3]={w[0][:3]}", flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    for n in sys.argv[1:]:
        run(n)
