"""Benchmark: Bloch-wave dispersion throughput on one MI355X.

Workload: the lowest 12 branches at the 60 wave vectors of the simple-cubic path
Gamma-X-M-Gamma-R for a 128^3 periodic Voronoi polycrystal (512 grains,
hexagonal Ti constants, c-axes spread N(0, 15 deg) about z, L = 1 mm), every
result carrying an FP64 a-posteriori bound on its relative omega error of at
most 5e-6 (metric: 1e-5).  One "step" solves one of two consecutive 30-point
halves of the path, the halves in turn (20 steps = the whole path ten times); the
value is wave vectors solved per second over the timed steps.  The
cell and the wave vectors are on the GPU / host before the timed region.

Arms: "mixed" (FP32 FFTs / contraction / PCG vectors, FP64 reductions,
Rayleigh-Ritz and eigen-residuals, the wave vectors of a segment batched in three
concurrent groups; the reported value) and "fp64_plain_one_k" (the plain method in FP64, one wave vector
and one PCG right-hand side at a time, the whole path once), on the same GPU.  Both
arms solve the shift-invert systems to the same relative residual TOL_lin = 1e-3
(an input of the method, Algorithm "InvA"): the accuracy of every omega is
certified by its FP64 bound, not by the inner tolerance (tighter inner solves
give the same omega to 1e-10 in more PCG iterations); plus context arms (the 64^3 Cu polycrystal, operator
throughput, uneven cells, fibre composites, textures, dispersion post-processing).

Prints ONE JSON line (rank 0).  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X dense FP64 matrix

# Algorithmic HBM bytes per voxel and per vector of each kernel, in words of one
# complex number (8 B FP32 / 16 B FP64) plus the uint16 grain index where read.
KERNEL_WORDS = {
    "k_strain_row_pcg": (15, 0),     # read r, p; write p and 6 strain components
    "k_strain_row": (9, 0),
    "k_axis1_inv_pcg": (12, 0), "k_axis1_fwd_pcg": (12, 0),
    "k_axis1_inv": (12, 0), "k_axis1_fwd": (12, 0),
    "k_axis0_contract_pcg": (12, 2), "k_axis0_contract": (12, 2),
    "k_plane_contract_pcg": (12, 2), "k_plane_contract": (12, 2),   # 2D FFTs + contraction, one (i0, i1) plane
    "k_row_div_pcg": (12, 0),        # read 6 stress components and p; write K p
    "k_row_div": (9, 0),
    "k_pcg_update": (18, 0),         # read x, r, p, Kp; write x, r
    "k_pcg_update_z": (21, 0),       # the same, and z = P^ r over Kp (slab path)
    # three-pass slab path (n1 = n2 = 128): 2D transforms of (vector, i0) slabs
    "k_slab_strain_pcg": (15, 0),    # read z, p; write p and 6 strain components
    "k_slab_strain": (9, 0),
    "k_slab_div_pcg": (12, 0),       # read 6 stress components and p; write K p
    "k_slab_div": (9, 0),
    "k_axis1_inv_mass": (6, 0), "k_axis1_fwd_mass": (6, 0), "k_axis0_mass": (6, 2),
    "k_row_inv_mass": (6, 0), "k_row_fwd_mass": (6, 0),
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6,
                    help="timed steps (even: both path halves equally often)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--segments", type=int, default=SEGMENTS,
                    help="the 60-point path is solved in this many consecutive segments, one per step")
    ap.add_argument("--skip-fp64", action="store_true", help="do not run the plain FP64 arm")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--method", type=int, default=1, help="0 = subspace iteration, 1 = batched Lanczos")
    ap.add_argument("--skip-cu64", action="store_true", help="do not run the 64^3 Cu polycrystal arm")
    ap.add_argument("--skip-learned", action="store_true", help="do not train / run the learned preconditioner arm")
    ap.add_argument("--skip-operator-arm", action="store_true", help="do not time bw_apply_K at 64^3 and 128^3")
    ap.add_argument("--skip-uneven", action="store_true", help="do not run the batched uneven-cells arm")
    ap.add_argument("--skip-fibre", action="store_true", help="do not run the long-fibre composite arm")
    ap.add_argument("--skip-post", action="store_true",
                    help="do not run the group-velocity / long-wave-speed arm")
    ap.add_argument("--kgroups", type=int, default=KGROUPS,
                    help="concurrent wave-vector groups of the mixed arm's batched Lanczos (1: one batch)")
    ap.add_argument("--tol-lin", type=float, default=TOL_LIN,
                    help="relative residual of the inner PCG solves (both arms)")
    ap.add_argument("--operator-only", action="store_true",
                    help="only time bw_apply_K on the 128^3 Ti cell (8 vectors) and the 64^3 Cu cell (32 vectors); for counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with plain 1 GiB device copies (reference kernel for memory-counter runs)")
    return ap.parse_args()


TOL_OMEGA = 5e-6   # a-posteriori bound target on the relative omega error (metric: 1e-5)
TOL_LIN = 1e-3     # relative residual of the inner PCG solves (both arms of the dispersion benches)
KGROUPS = 3        # concurrent wave-vector groups of the mixed batched Lanczos
SEGMENTS = 2       # consecutive path segments, one solved per step


def run_arm(bw, rve_in, segs, precision, steps, warmup, tol_lin, tol_eig, timing=False, method=1, kbatch=0,
            tune=True, kgroups=1):
    """Solves the wave-vector segments `segs` (a list of k arrays) in rotation, one
    segment per step; returns the timed seconds, the wave vectors solved and the
    per-step statistics."""
    import torch
    R = bw.Rve.from_inputs(rve_in, precision)
    nk_max = max(len(k) for k in segs)
    if tune:   # FFT schedule for this cell at the arm's PCG batch (setup, outside the timed region)
        sp = bw.bw_autotune(R, min(nk_max, 64) if (method == 1 and kbatch == 0) else (kbatch or 16))
        print(f"[bench] precision {precision} autotune: schedule {bw.bw_fft_schedule(R)}, speedup {sp:.3f}",
              file=sys.stderr, flush=True)
    kw = dict(block=16, tol_eig=tol_eig, tol_lin=tol_lin, tol_omega=TOL_OMEGA, method=method, kbatch=kbatch,
              kgroups=kgroups)
    breakdown = None
    for i in range(warmup):
        if timing and i == warmup - 1:       # the last warmup step finds the dominant kernel
            bw.bw_timing_filter(None)
            bw.bw_timing_enable(True)
        _, _, _, st = bw.bw_lowest_modes(R, segs[i % len(segs)], 12, **kw)
        print(f"[bench] precision {precision} warmup {i}: {st['seconds']:.2f} s, outer {st['outer_iterations']}, "
              f"pcg {st['pcg_iterations']}", file=sys.stderr, flush=True)
    if timing and warmup > 0:
        breakdown = bw.bw_timing_report()
        bw.bw_timing_enable(False)
    torch.cuda.synchronize()
    if timing:
        # live HIP-event timing of the dominant kernel only, over the timed region
        dom = dominant(breakdown) if breakdown else None
        bw.bw_timing_filter(dom)
        bw.bw_timing_enable(True)
    t0 = time.perf_counter()
    stats = []
    maxb = 0.0
    nk_done = 0
    omegas = []
    for i in range(steps):
        ks = segs[i % len(segs)]
        w, err, code, st = bw.bw_lowest_modes(R, ks, 12, **kw)
        stats.append(st)
        omegas.append(w)
        nk_done += len(ks)
        maxb = max(maxb, float(err.max()))
        print(f"[bench] precision {precision} step {i}: {len(ks)} k in {st['seconds']:.2f} s, "
              f"outer {st['outer_iterations']}, pcg {st['pcg_iterations']}, max bound {float(err.max()):.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rep = None
    solo = None
    if timing:
        rep = bw.bw_timing_report()
        bw.bw_timing_enable(False)
        if kgroups > 1:
            # after the timed region: one segment as a single group, so that the
            # dominant kernel's launches run without the other groups' kernels
            # beside them (context for the roofline, not part of the value)
            bw.bw_timing_filter(dominant(rep))
            bw.bw_timing_enable(True)
            bw.bw_lowest_modes(R, segs[0], 12, **dict(kw, kgroups=1))
            solo = bw.bw_timing_report()
            bw.bw_timing_enable(False)
    R.close()
    torch.cuda.empty_cache()
    return dict(seconds=dt, nk=nk_done, stats=stats, max_bound=maxb, omega=omegas, code=code, timing=rep,
                breakdown=breakdown, solo=solo)


def gram_mfma(breakdown, nvox):
    """MFMA use of the Gram products X^H Y (FP64 complex, the Rayleigh-Ritz blocks) over the
    last warmup step: achieved FLOP/s (8 real flops per complex multiply-add, n = 3 nvox
    rows, sum of qx qy over the launches) against min(FP64 MFMA peak, intensity x 8 TB/s),
    the intensity of a q x q block being 8 q^2 n / (2 q n 16 B) = q / 4 flop/B."""
    g = (breakdown or {}).get("k_gram_mfma")
    if not g or not g["launches"] or not g["ms"]:
        return None
    flops = 8.0 * 3 * nvox * g["units"]
    q = (g["units"] / g["launches"]) ** 0.5
    achieved = flops / (g["ms"] * 1e-3) / 1e12
    bound = min(PEAK_FP64_MFMA_TFLOPS, q / 4.0 * PEAK_HBM_GBS / 1e3)
    return {"kernel": "k_gram_mfma", "dtype": "f64", "launches": g["launches"], "mean_block": round(q, 2),
            "achieved_TFLOPs": round(achieved, 3), "bound_TFLOPs": round(bound, 3),
            "frac_of_bound": round(achieved / bound, 4), "peak_TFLOPs": PEAK_FP64_MFMA_TFLOPS}


def dominant(rep):
    return max(((k, v) for k, v in rep.items() if k in KERNEL_WORDS), key=lambda kv: kv[1]["ms"])[0]


def roofline(rep, nvox, word_bytes, workload):
    best = max(((k, v) for k, v in rep.items() if k in KERNEL_WORDS), key=lambda kv: kv[1]["ms"])
    name, v = best
    words, extra = KERNEL_WORDS[name]
    bytes_total = v["units"] * nvox * (words * word_bytes + extra)
    per_launch = bytes_total / max(v["launches"], 1)
    avg_s = v["ms"] / max(v["launches"], 1) / 1e3
    # launches on concurrent streams (wave-vector groups) overlap: the kernel's
    # bytes over the time during which it ran (per-launch bytes / mean duration
    # when launches do not overlap)
    busy_s = v.get("union_ms", v["ms"]) / 1e3
    achieved = bytes_total / busy_s / 1e9
    traffic = measured_traffic(name, workload)
    if traffic is not None:   # counter bytes per voxel and active vector, at this run's launches
        traffic = int(traffic * per_launch / (words * word_bytes + extra))
    return dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic,
                bytes_per_launch=int(per_launch), avg_launch_us=round(avg_s * 1e6, 2),
                launches=v["launches"], bytes_per_voxel_vector=words * word_bytes + extra,
                busy_ms=round(busy_s * 1e3, 2), launch_overlap=round(v["ms"] / max(busy_s * 1e3, 1e-9), 3))


KERNEL_SOURCES = ("paper_2106_12487_amd/csrc/bw_ops_impl.h", "paper_2106_12487_amd/csrc/bw_fftreg.h",
                  "paper_2106_12487_amd/csrc/bw_slab.h", "paper_2106_12487_amd/csrc/bw_fft.h",
                  "paper_2106_12487_amd/csrc/bw_internal.h")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per voxel and active vector of `kernel` on `workload` from the
    committed counter runs (profiles/traffic_<kernel>_<workload>.json: FETCH_SIZE and
    WRITE_SIZE scaled by what they read for a 1 GiB copy), or None when there is none
    or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("sources_sha256_16") != kernel_sources_hash():
        return None
    return t.get("traffic_bytes_per_voxel_vector")


# Algorithmic bytes of one K apply per voxel and vector (3-pass model: strain + axis-2
# transforms 3 in / 6 out, axes 0-1 transforms + contraction 6 + grain id in / 6 out,
# axis-2 transforms + divergence 6 in / 3 out): 30 complex words + 2 B = 242 B in FP32.
APPLY_K_BYTES_FP32 = 30 * 8 + 2


def operator_arm(bw, rve_in, nvec=8, reps=10):
    """bw_apply_K throughput on a mixed cell in the streaming regime (working set above
    the 256 MB last-level cache): vector applies/s and GB/s of the 3-pass model."""
    import numpy as np
    import torch
    R = bw.Rve.from_inputs(rve_in, bw.BW_MIXED)
    bw.bw_autotune(R, nvec)
    rng = np.random.default_rng(3)
    u = torch.from_numpy(rng.standard_normal((nvec, 3) + tuple(rve_in.n)).astype(np.complex64)).to("cuda")
    y = torch.empty_like(u)
    k = (0.3 * np.pi / rve_in.L[0], 0.1 * np.pi / rve_in.L[1], 0.0)
    for _ in range(2):
        bw.bw_apply_K(R, k, u, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bw.bw_apply_K(R, k, u, y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    nvox = int(np.prod(rve_in.n))
    R.close()
    gbs = nvec * nvox * APPLY_K_BYTES_FP32 / dt / 1e9
    return {"grid": list(rve_in.n), "vectors": nvec, "ms_per_apply": round(dt * 1e3, 3),
            "vector_applies_per_s": round(nvec / dt, 1), "pass_model_bytes_per_voxel": APPLY_K_BYTES_FP32,
            "algorithmic_GBps": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}


def uneven_arm(bw, tol_omega=5e-6):
    """Batched uneven workload: 8 cells (32^3, 40^3, 48^3, 64^3, two each; Cu or Al
    grains), 24 wave vectors on Gamma-X-M-Gamma each, 8 modes, mixed, batched
    Lanczos; the cells one after the other, all cells in one batched call with each
    cell on a stream of its own (the default), and the same call with the cells of one
    grid grouped (their wave vectors share every batched launch)."""
    import numpy as np
    from paper_2106_12487_amd import inputs
    w = inputs.WORKLOADS[3]
    cells = [bw.Rve.from_inputs(inputs.workload_rve(3, i), bw.BW_MIXED) for i in range(len(w["grids"]))]
    ks = [inputs.workload_kpoints(3)] * len(cells)
    for c in cells:
        bw.bw_autotune(c, len(ks[0]))
    kw = dict(method=1, tol_omega=tol_omega, tol_lin=1e-6)
    nkt = sum(len(k) for k in ks)
    bw.bw_lowest_modes_batched(cells, ks, w["nmodes"], **kw)           # warm-up (workspaces, groups)
    bw.bw_lowest_modes_batched(cells, ks, w["nmodes"], group_cells=True, **kw)
    t0 = time.perf_counter()
    maxb = 0.0
    for c, k in zip(cells, ks):
        _, er, _, _ = bw.bw_lowest_modes(c, k, w["nmodes"], **kw)
        maxb = max(maxb, float(er.max()))
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, ers, _, st_s = bw.bw_lowest_modes_batched(cells, ks, w["nmodes"], **kw)
    t_str = time.perf_counter() - t0
    maxb = max(maxb, max(float(e.max()) for e in ers))
    t0 = time.perf_counter()
    _, ers, _, st_g = bw.bw_lowest_modes_batched(cells, ks, w["nmodes"], group_cells=True, **kw)
    t_grp = time.perf_counter() - t0
    maxb = max(maxb, max(float(e.max()) for e in ers))
    for c in cells:
        c.close()
    return {"workload": w["name"], "grids": w["grids"], "k_points": nkt, "modes": w["nmodes"],
            "sequential_kpoints_per_s": round(nkt / t_seq, 2),
            "batched_kpoints_per_s": round(nkt / t_str, 2),
            "grouped_kpoints_per_s": round(nkt / t_grp, 2),
            "batched_speedup": round(t_seq / t_str, 3), "grouped_speedup": round(t_seq / t_grp, 3),
            "pcg_sweeps_grouped": st_g["block_iterations"], "pcg_sweeps_streams": st_s["block_iterations"],
            "max_error_bound": maxb}


def dispersion_post_arm(bw, rve_in, ks, tol_omega=5e-6):
    """Group velocity (d omega / ds along the path) of the 12 branches at every wave
    vector of the workload from the mixed path's modes, and the long-wave speeds
    along [100], [110], [111]."""
    import numpy as np
    import torch
    R = bw.Rve.from_inputs(rve_in, bw.BW_MIXED)
    bw.bw_autotune(R, min(len(ks), 64))
    nm = 12
    modes = torch.zeros((len(ks), nm, 3) + tuple(rve_in.n), dtype=torch.complex64, device="cuda")
    w, _, code, _ = bw.bw_lowest_modes(R, ks, nm, method=1, tol_omega=tol_omega, tol_lin=1e-6, block=16,
                                       modes=modes)
    tang = np.gradient(ks, axis=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slopes = np.stack([bw.bw_group_velocity(R, ks[i], tang[i] if np.linalg.norm(tang[i]) > 0 else [1, 0, 0],
                                            modes[i], w[i], cluster_tol=1e-4) for i in range(len(ks))])
    t_gv = time.perf_counter() - t0
    # real-space displacement + strain maps of the 12 modes at every wave vector
    u = torch.empty_like(modes[0])
    eps = torch.empty((nm, 6) + tuple(rve_in.n), dtype=modes.dtype, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(ks)):
        bw.bw_mode_fields(R, ks[i], modes[i], u, eps)
    torch.cuda.synchronize()
    t_mf = time.perf_counter() - t0
    del modes, u, eps
    lw = {}
    t0 = time.perf_counter()
    for name, d in (("100", [1, 0, 0]), ("110", [1, 1, 0]), ("111", [1, 1, 1])):
        c, _ = bw.bw_long_wave_speeds(R, d)
        lw[name] = [round(float(v), 2) for v in c]
    t_lw = time.perf_counter() - t0
    # static homogenization (six cell problems at k = 0): rho_bar c^2 along [100] against
    # the long-wave speeds (the even grid's offset is ~1e-6)
    bw.bw_effective_stiffness(R)                                        # warm-up (workspaces)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ce, it_h, code_h = bw.bw_effective_stiffness(R)
    t_h = time.perf_counter() - t0
    rho = float(np.mean(rve_in.rho[rve_in.grain_map]))
    from paper_2106_12487_amd import inputs
    T = inputs.voigt_to_tensor(Ce)
    c_static = np.sqrt(np.sort(np.linalg.eigvalsh(T[:, 0, :, 0])) / rho)
    R.close()
    torch.cuda.empty_cache()
    return {"group_velocity_k_points_per_s": round(len(ks) / t_gv, 2), "modes": nm,
            "mode_fields_k_points_per_s": round(len(ks) / t_mf, 2),
            "acoustic_slopes_at_k1_m_per_s": [round(float(v), 2) for v in slopes[1, :3]],
            "long_wave_seconds_per_direction": round(t_lw / 3, 3), "long_wave_speeds_m_per_s": lw,
            "homogenization_seconds": round(t_h, 3), "homogenization_pcg_iterations": [int(v) for v in it_h],
            "static_speeds_100_m_per_s": [round(float(v), 2) for v in c_static],
            "status": int(code), "homogenization_status": int(code_h)}



def fibre_arm(bw, tol_omega=5e-6):
    """Sec. 4.3 workload: epoxy with long carbon fibres (55% circular, 65% square
    sections) on 128 x 128 x 1, 90 wave vectors on M-Gamma-X-M, 10 modes, mixed path,
    subspace iteration (block 16; the square cell's symmetry points carry exactly
    degenerate branches)."""
    import numpy as np
    from paper_2106_12487_amd import inputs
    ks = inputs.kpath("MGXM", 90, inputs.L_MM)
    out = {}
    for section, vf in (("circle", 0.55), ("square", 0.65)):
        R = bw.Rve.from_inputs(inputs.fibre_composite(128, inputs.L_MM, section, vf), bw.BW_MIXED)
        bw.bw_autotune(R, 16)
        kw = dict(method=0, block=16, tol_omega=tol_omega, tol_lin=1e-6)
        bw.bw_lowest_modes(R, ks[:2], 10, **kw)                      # warm-up (workspaces)
        t0 = time.perf_counter()
        w, er, code, st = bw.bw_lowest_modes(R, ks, 10, **kw)
        dt = time.perf_counter() - t0
        R.close()
        out[f"{section}_{int(round(vf * 100))}"] = {
            "k_points_per_s": round(len(ks) / dt, 2), "max_error_bound": float(er.max()), "status": int(code),
            "gap_5_6": [float(w[:, 4].max()), float(w[:, 5].min())], "pcg_iterations": st["pcg_iterations"]}
    return {"grid": [128, 128, 1], "k_points": len(ks), "modes": 10, "path": "M-G-X-M", **out}


def texture_arm(bw):
    """Sec. 5.2 effect of texture: long-wave speeds along x and z of 64^3 / 64-grain Ni
    polycrystals with random, [111]-fibre and [100]-fibre textures (mixed path), and of the
    Sec. 5.1 1D Ni bar (256 voxels, 64 grains, Zener 2.45) along the bar."""
    from paper_2106_12487_amd import inputs
    L = inputs.L_MM
    out = {}
    t0 = time.perf_counter()
    for tex in ("haar", "fibre111", "fibre100"):
        R = bw.Rve.from_inputs(inputs.polycrystal((64, 64, 64), (L, L, L), 64, 52, 0, texture=tex, phases=("ni",)),
                               bw.BW_MIXED)
        out[tex] = {d: [round(float(v), 2) for v in bw.bw_long_wave_speeds(R, vec)[0]]
                    for d, vec in (("x", [1, 0, 0]), ("z", [0, 0, 1]))}
        R.close()
    R = bw.Rve.from_inputs(inputs.ni_bar(256, 64, 50e-6, 50e-6, 2.45, 0), bw.BW_FP64)
    out["ni_bar_A2.45"] = [round(float(v), 2) for v in bw.bw_long_wave_speeds(R, [1, 0, 0])[0]]
    R.close()
    out["seconds"] = round(time.perf_counter() - t0, 2)
    return out


def copy_calibration(bw):
    import torch
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        bw.bw_diag_copy(src, dst)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x {n} bytes", file=sys.stderr, flush=True)


def copy_bandwidth(bw, reps=20):
    """Measured device-copy bandwidth (GB/s, read + write) of the library's plain
    streaming copy on 1 GiB: the practical ceiling of a streaming kernel."""
    import torch
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        bw.bw_diag_copy(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bw.bw_diag_copy(src, dst)
    e1.record()
    e1.synchronize()
    gbs = 2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(rve_in, k, budget_s, golden):
    """Oracle PCG on the workload (one right-hand side at wave vector k) for about
    budget_s seconds, scaled by the oracle's own PCG-iteration count per k-point
    from its shift-invert Lanczos runs on the same cell (tests/golden/<golden>.json)."""
    import numpy as np
    from oracle.operators import Operators
    from oracle import solvers
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ops = Operators(rve_in, k)
    rng = np.random.default_rng(0)
    b = rng.standard_normal((3,) + rve_in.n) + 1j * rng.standard_normal((3,) + rve_in.n)
    ops.precond(b)                                        # the preconditioner's setup
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    ops.apply_K(b)
    t_apply = time.perf_counter() - t0
    n_it = max(3, int(budget_s / max(1.3 * t_apply, 1e-3)))
    t0 = time.perf_counter()
    _, its, _ = solvers.pcg(ops, b, 1e-30, maxit=n_it)     # tolerance never met: exactly n_it iterations
    dt = time.perf_counter() - t0
    sec_per_it = dt / max(its, 1)
    grid = "x".join(str(v) for v in rve_in.n)
    gpath = os.path.join(ROOT, "tests", "golden", f"{golden}.json")
    its_per_k = None
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        if g.get("pcg_iters"):
            its_per_k = float(np.mean(g["pcg_iters"]))
    if its_per_k is None:
        return dict(value=None, unit="k-points/s", cores=cores, kind="oracle",
                    sample=f"{its} oracle PCG iterations at {grid} in {dt:.1f} s; no stored iteration count")
    return dict(value=1.0 / (sec_per_it * its_per_k), unit="k-points/s", cores=cores, kind="oracle",
                sample=(f"{its} oracle PCG iterations (1 RHS, {grid}, setup {t_setup:.1f} s) in {dt:.1f} s = "
                        f"{sec_per_it:.3f} s/iteration, times {its_per_k:.0f} PCG iterations per k-point of the "
                        f"oracle's shift-invert Lanczos in its full runs on this cell (tests/golden/{golden}.json, "
                        f"{len(g['pcg_iters'])} wave vectors); extrapolated"))


def learned_arm(bw, ti_rve, ti_ks, cells=8, steps=400, lr=2e-4):
    """The learned preconditioner on the workload it is meant for: a network trained (residual
    loss, on the GPU) on plain-PCG residuals of `cells` 64^3 Cu cells of 16-256 grains, then
    (a) flexible PCG on an unseen 128^3 / 512-grain Cu cell against the plain preconditioner,
    (b) the 12 lowest modes at one wave vector of the 128^3 Ti path with the learned inner
    solves against the plain mixed path (k-points/s, status)."""
    import numpy as np
    import torch
    from paper_2106_12487_amd import train_precond as tp
    t0 = time.perf_counter()
    tc = [tp.training_cell(i) for i in range(cells)]
    pairs = tp.make_pairs(tc, 2, 4)
    net = bw.UNet(seed=1)
    t1 = time.perf_counter()
    losses = tp.train(net, tc, pairs, steps, lr)
    t_train = time.perf_counter() - t1
    del pairs
    for _, R in tc:
        R.close()
    torch.cuda.empty_cache()
    ev_cell = tp.eval_cell(128, 0)
    ev = tp.evaluate(net, [ev_cell], 1, 4)
    ev_cell[1].close()
    R = bw.Rve.from_inputs(ti_rve, bw.BW_MIXED)
    bw.bw_autotune(R, 1)
    k = ti_ks[[17]]
    kw = dict(method=bw.BW_LANCZOS, tol_omega=TOL_OMEGA, tol_lin=1e-6)
    bw.bw_lowest_modes(R, k, 12, **kw)                                  # warm-up (workspaces)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    w0, e0, c0, st0 = bw.bw_lowest_modes(R, k, 12, **kw)
    t_plain = time.perf_counter() - t2
    t2 = time.perf_counter()
    w1, e1, c1, st1 = bw.bw_lowest_modes(R, k, 12, net=net, **kw)
    t_learned = time.perf_counter() - t2
    R.close()
    net.close()
    torch.cuda.empty_cache()
    scale = float(np.max(w0))
    return {"training": {"cells": cells, "grid": 64, "grains": "16-256", "pairs_batches": steps,
                         "loss": "residual ||K z - r||^2 / ||r||^2", "loss_first_50": float(np.mean(losses[:50])),
                         "loss_last_50": float(np.mean(losses[-50:])), "seconds": round(t_train, 1),
                         "setup_seconds": round(t1 - t0, 1)},
            "fpcg_cu128_512g": {"plain_iters": ev["plain_iters"], "learned_iters": ev["learned_iters"],
                                "iter_ratio": round(ev["iter_ratio"], 3), "time_ratio": round(ev["time_ratio"], 2),
                                "fallbacks": ev["fallbacks"]},
            "lanczos_ti128_one_k": {"plain_k_points_per_s": round(1 / t_plain, 3),
                                    "learned_k_points_per_s": round(1 / t_learned, 3),
                                    "ratio": round(t_plain / t_learned, 3), "status": int(c1),
                                    "pcg_iterations": [st0["pcg_iterations"], st1["pcg_iterations"]],
                                    "max_error_bound": float(e1.max()),
                                    "max_rel_diff_vs_plain": float(np.abs(w1 - w0).max() / scale)}}


def segments(ks, nseg):
    """The path split into nseg consecutive segments of (nearly) equal length."""
    import numpy as np
    return [s for s in np.array_split(ks, nseg) if len(s)]


def cu64_arm(bw, steps=2, warmup=1, fp64=True):
    """The 64^3 / 64-grain Cu polycrystal, 40 wave vectors of Gamma-X-M-Gamma-R, 12 modes:
    mixed batched Lanczos against the plain FP64 method one wave vector at a time."""
    import numpy as np
    from paper_2106_12487_amd import inputs
    rve = inputs.workload_rve(2, 0)
    ks = inputs.workload_kpoints(2)
    mixed = run_arm(bw, rve, [ks], bw.BW_MIXED, steps, warmup, TOL_LIN, 1e-6, kgroups=KGROUPS)
    out = {"workload": inputs.WORKLOADS[2]["name"], "grid": list(rve.n), "k_points": len(ks),
           "value": round(mixed["nk"] / mixed["seconds"], 3), "unit": "k-points/s",
           "max_error_bound": mixed["max_bound"]}
    if fp64:
        fp = run_arm(bw, rve, [ks], bw.BW_FP64, 1, 0, TOL_LIN, 1e-6, kbatch=1)
        out["fp64_plain_one_k"] = round(fp["nk"] / fp["seconds"], 3)
        out["speedup_over_fp64_plain"] = round(out["value"] / out["fp64_plain_one_k"], 3)
        out["max_rel_diff_vs_fp64"] = float((np.abs(mixed["omega"][-1] - fp["omega"][0]) /
                                             np.maximum(fp["omega"][0], 1.0)).max())
    return out


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding across GPUs is described, not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2106_12487_amd import blochwave as bw
    from paper_2106_12487_amd import inputs
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    w4 = inputs.WORKLOADS[4]
    rve_in = inputs.workload_rve(4, 0)
    ks = inputs.workload_kpoints(4)
    if a.operator_only:
        print(json.dumps({"apply_K_mixed": [operator_arm(bw, rve_in, nvec=8),
                                            operator_arm(bw, inputs.workload_rve(2, 0), nvec=32)]}), flush=True)
        return
    segs = segments(ks, a.segments)
    nvox = int(np.prod(rve_in.n))
    print(f"[bench] {w4['name']}: {len(ks)} wave vectors in {len(segs)} segments of {len(segs[0])}",
          file=sys.stderr, flush=True)
    mixed = run_arm(bw, rve_in, segs, bw.BW_MIXED, a.steps, a.warmup, a.tol_lin, 1e-6, timing=True,
                    method=a.method, kgroups=a.kgroups)
    out = {
        "metric": "k-points/s (12 modes, omega rel err 1e-5)",
        "value": round(mixed["nk"] / mixed["seconds"], 4),
        "unit": "k-points/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * mixed["seconds"] / a.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w4["name"], "grid": list(rve_in.n), "grains": rve_in.n_grains,
                   "material": "Ti hexagonal 162.4/92.0/69.0/180.7/46.7 GPa, c-axes N(0, 15 deg) about z",
                   "k_points": len(ks), "path": "G-X-M-G-R",
                   "step": f"one of {len(segs)} consecutive path segments ({len(segs[0])} wave vectors), in turn",
                   "modes": 12, "block": 16,
                   "method": "subspace" if a.method == 0 else "batched Lanczos",
                   "precision": "FP32 FFT/contraction/PCG vectors, FP64 reductions and Rayleigh-Ritz",
                   "tol_lin": a.tol_lin, "tol_omega_bound": TOL_OMEGA, "kgroups": a.kgroups},
        "max_error_bound": mixed["max_bound"],
        "k_points_solved": mixed["nk"],
        "solver_stats": mixed["stats"][-1],
    }
    out["roofline"] = roofline(mixed["timing"], nvox, 8, "ti128")
    if mixed.get("solo"):
        solo = roofline(mixed["solo"], nvox, 8, "ti128")
        out["roofline"]["single_group"] = {k: solo[k] for k in ("kernel", "achieved", "frac", "avg_launch_us",
                                                               "launches", "traffic")}
    cbw = copy_bandwidth(bw)
    out["roofline"]["copy_GBps"] = round(cbw, 1)
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / cbw, 4)
    if "single_group" in out["roofline"]:
        sg = out["roofline"]["single_group"]
        sg["frac_of_copy"] = round(sg["achieved"] / cbw, 4)
    out["mfma"] = gram_mfma(mixed["breakdown"], nvox)
    for kname, v in sorted((mixed["breakdown"] or {}).items(), key=lambda kv: -kv[1]["ms"]):
        print(f"[bench] kernel {kname:24s} launches {v['launches']:6d} total {v['ms']:9.1f} ms units {v['units']}",
              file=sys.stderr, flush=True)
    out["arms"] = {}
    if not a.skip_fp64:
        # baseline: the plain method in FP64, one wave vector (one PCG right-hand side) at a
        # time, over the whole path once
        fp = run_arm(bw, rve_in, [ks], bw.BW_FP64, 1, 0, a.tol_lin, 1e-6, method=1, kbatch=1)
        v64 = fp["nk"] / fp["seconds"]
        # the mixed arm's last pass over the path against the FP64 path
        last = np.concatenate(mixed["omega"][-len(segs):]) if a.steps >= len(segs) else None
        ref = fp["omega"][0]
        scale = 2 * np.pi / inputs.L_MM * 2000.0
        out["arms"]["fp64_plain_one_k"] = {"value": round(v64, 4), "unit": "k-points/s",
                                           "method": "Lanczos, FP64, one k and one RHS at a time, whole path",
                                           "max_error_bound": fp["max_bound"], "solver_stats": fp["stats"][-1]}
        out["arms"]["speedup_over_fp64_plain"] = round(out["value"] / v64, 3)
        if last is not None and last.shape == ref.shape:
            out["arms"]["max_rel_diff_vs_fp64"] = float((np.abs(last - ref) / np.maximum(ref, scale)).max())
        print(f"[bench] fp64 arm: {out['arms']['fp64_plain_one_k']['value']} k-points/s, speedup "
              f"{out['arms']['speedup_over_fp64_plain']}", file=sys.stderr, flush=True)
    if not a.skip_learned:
        out["arms"]["learned_preconditioner"] = learned_arm(bw, rve_in, ks)
        print(f"[bench] learned arm: {out['arms']['learned_preconditioner']}", file=sys.stderr, flush=True)
    if not a.skip_cu64:
        out["arms"]["cu64_64g_gxmgr"] = cu64_arm(bw, fp64=not a.skip_fp64)
        print(f"[bench] cu64 arm: {out['arms']['cu64_64g_gxmgr']}", file=sys.stderr, flush=True)
    if not a.skip_operator_arm:
        out["arms"]["apply_K_mixed"] = [operator_arm(bw, inputs.workload_rve(2, 0), nvec=32),
                                        operator_arm(bw, rve_in, nvec=8)]
        print(f"[bench] apply_K arm: {out['arms']['apply_K_mixed']}", file=sys.stderr, flush=True)
    if not a.skip_uneven:
        out["arms"]["uneven_batched"] = uneven_arm(bw)
        print(f"[bench] uneven arm: {out['arms']['uneven_batched']}", file=sys.stderr, flush=True)
    if not a.skip_fibre:
        out["arms"]["fibre_composite"] = fibre_arm(bw)
        print(f"[bench] fibre arm: {out['arms']['fibre_composite']}", file=sys.stderr, flush=True)
    if not a.skip_post:
        out["arms"]["textures_long_wave_m_per_s"] = texture_arm(bw)
        print(f"[bench] texture arm: {out['arms']['textures_long_wave_m_per_s']}", file=sys.stderr, flush=True)
        out["arms"]["dispersion_post"] = dispersion_post_arm(bw, inputs.workload_rve(2, 0),
                                                             inputs.workload_kpoints(2))
        print(f"[bench] dispersion post arm: {out['arms']['dispersion_post']}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(rve_in, ks[1], a.cpu_seconds, "ti128")
    if a.copy_calibration:
        copy_calibration(bw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
