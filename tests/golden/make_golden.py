"""Writes the stored oracle eigenfrequencies that the GPU parity tests compare to.

Calls only the CPU oracle (oracle/) and the seeded input generators; nothing
here touches the HIP path.  Usage:

    python tests/golden/make_golden.py cu16      # 16^3, 8 grains, all 11 k on Gamma-X
    python tests/golden/make_golden.py cu64      # 64^3, 64 grains, sampled k of the path (Lanczos)
    python tests/golden/make_golden.py cual32    # 32^3 Cu/Al cell of the uneven workload, 4 k (Lanczos)
    python tests/golden/make_golden.py fibre128  # 128 x 128 x 1 epoxy / 55% circular carbon fibres, 4 k (Lanczos)
    python tests/golden/make_golden.py ti128:11  # 128^3 / 512-grain textured Ti, one path index per process
    python tests/golden/make_golden.py ti128-merge  # joins the ti128 parts into ti128.json

The 128^3 Ti set takes one to three hours per wave vector on a few host cores, so each
wave vector runs in a process of its own (tests/golden/ti128_k<index>.json) and the
parts are joined afterwards.

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


TI128_INDICES = [11, 22, 58]   # next to X on Gamma-X, next to M on X-M, next to R on Gamma-R


def merge_ti128():
    """Joins the per-wave-vector parts of the 128^3 Ti set (same settings) into ti128.json."""
    parts = []
    for i in TI128_INDICES:
        with open(os.path.join(HERE, f"ti128_k{i}.json")) as f:
            parts.append(json.load(f))
    out = {key: parts[0][key] for key in ("config", "nmodes", "block", "method", "tol_eig", "tol_lin")}
    out["name"] = "ti128"
    for key in ("k_index", "k", "omega", "seconds", "pcg_iters", "outer"):
        out[key] = [v for p in parts for v in p[key]]
    with open(os.path.join(HERE, "ti128.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


def run(name):
    method = "subspace"
    tol = 1e-12
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
    elif name.startswith("ti128:"):
        # the large textured workload: 128^3, 512 grains, hexagonal Ti with a c-axis
        # texture; 12 modes at one wave vector next to a symmetry point of the path
        cfg, nmodes, block = 4, 12, 16
        idx = [int(name.split(":")[1])]
        name = f"ti128_k{idx[0]}"
        method = "lanczos"
        tol = 1e-11
    else:
        raise SystemExit(f"unknown golden set {name}")
    if cfg is None:
        rve = inputs.fibre_composite(128, inputs.L_MM, "circle", 0.55)
        ks = inputs.kpath("MGXM", 90, inputs.L_MM)[idx]
    else:
        rve = inputs.workload_rve(cfg, 0)
        ks = inputs.workload_kpoints(cfg)[idx]
    out = dict(name=name, config=cfg, nmodes=nmodes, block=block, method=method, tol_eig=tol, tol_lin=tol,
               k_index=idx, k=ks.tolist(), omega=[], seconds=[], pcg_iters=[], outer=[])
    path = os.path.join(HERE, f"{name}.json")
    for i, k in enumerate(ks):
        t = time.time()
        st = []
        w = solvers.lowest_modes(rve, k[None], nmodes, method=method, block=block,
                                 tol_eig=tol, tol_lin=tol, dense_max=0, warm_start=False, stats=st)
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
        if n == "ti128-merge":
            merge_ti128()
        else:
            run(n)
