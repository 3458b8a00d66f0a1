"""Throughput of the generalized shifted Krylov solver on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config c5] [--batch 1280]

Default workload (c5): the one-GPU share of a 10^6-atom amorphous hydrocarbon
box (M = 2.0e6, FP32-stored A and B beside the FP64 values).  65536 columns
are sampled uniformly; each is solved as a region problem on the atoms within
a radius drawn from U[6, 14] A of the column's atom (Sec. III-B, III-C), for
128 shifts z_k = eps_k + 0.01i on [-1, 1] Ha, to a relative residual of 1e-8.
The regions are cut into batches of about `--batch` columns (consecutive
regions); one step = one elses_regions_solve over one batch: the compact
per-region layout in one persistent launch per column-width group (Lanczos
outer process in the B inner product, FP32 Chebyshev-Richardson overlap
solves with FP64-accumulated refinement, fused multi-shift update), with the
density-matrix elements on the column patterns and e_j^T rho B e_j,
e_j^T rho A e_j per column.  The region sets are built before the timed
region; steps cycle through them.  Inputs are resident in HBM before the
timed region; a short untimed solve loads the kernels first.

Prints one JSON line with the metric (column x shift solves per second), the
roofline of the dominant kernel (the persistent compact solve: algorithmic
bytes per solve over the span from its first group launch's start to its last
group launch's end, measured with HIP events on the launch streams), the HBM
traffic of that solve from the committed rocprofv3 counter summary when it
was taken on the current kernel source at this batch size, an FP64 true
residual recomputed in the kernel for a subsample of columns, the plain FP64
tile method timed on a small sample for comparison, and the CPU oracle timed
on a bounded sample on the host's cores.

Other configurations: c1/c2 (global solves of every column of a 128/4096-atom
box), c3 (2048 regions of a 50000-atom box), c4 (16384 sampled columns of a
100000-atom box with the learned preconditioner and the plain overlap
iteration compared); --method arnoldi / balance / pass for the multiple
Arnoldi method, idle-lane measurements and the global pass alone.

    python bench.py --copy-calib 1073741824

runs only a plain device copy of the given size (the calibration of the HBM
byte counters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "column×shift solves/sec at 1e-8 rel. residual; SpMV HBM GB/s vs peak"

PASS_SOURCE = os.path.join(ROOT, "paper_1609_08377_amd", "csrc", "passes.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pass_group_step_c2_traffic.md")
C3_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pass_group_step32_c3_traffic.md")
MA_SOURCE = os.path.join(ROOT, "paper_1609_08377_amd", "csrc", "arnoldi.hip")
MA_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "ma_update_regions4096_traffic.md")

WORKLOADS = {
    # name: (n_atoms, n_shifts, description)
    "c1": (128, 32, "128-atom amorphous hydrocarbon box (C:H=1:2, 1.0 g/cm^3), M=257, all columns x 32 shifts "
                    "z=eps_k+0.01i on [-1,1] Ha, FP64, tol 1e-8, global"),
    "c2": (4096, 64, "4096-atom amorphous hydrocarbon box (C:H=1:2, 1.0 g/cm^3), M=8191 (4x4/4x1/1x1 atom "
                     "blocks, ~71 nnz/row), all 8191 columns x 64 shifts z=eps_k+0.01i on [-1,1] Ha, FP64, "
                     "tol 1e-8, global"),
    "c5": (1000000, 128, "one-GPU share of a 10^6-atom amorphous hydrocarbon box (C:H=1:2, 1.0 g/cm^3, "
                         "M=2.0e6, FP32-stored A and B): 65536 columns sampled uniformly, solved as region "
                         "problems (atoms within a radius U[6,14] A of the column's atom; columns on one atom "
                         "share its region) x 128 shifts z=eps_k+0.01i on [-1,1] Ha, tol 1e-8, compact "
                         "per-region layout in one persistent launch per column-width group, FP32 overlap "
                         "solves with FP64 refinement; rho on the patterns and tr(rho B) per column"),
    "c4": (100000, 64, "100000-atom amorphous hydrocarbon box (M=2.0e5): 16384 columns sampled uniformly, "
                       "solved as region problems (radius U[6,14] A) x 64 shifts, tol 1e-8, compact layout"),
    "c3": (50000, 64, "2048 local regions (centre atoms sampled without replacement, radius U[6,14] A, "
                      "187-3079 orbitals) carved from a 50000-atom amorphous hydrocarbon box (M=100001), all "
                      "orbitals of each centre x 64 shifts, packed into tiles and advanced by one launch "
                      "sequence, tol 1e-8"),
}
N_REGIONS = 2048
# sampled-column workloads: columns sampled from the whole box, solved as region problems
N_SAMPLED = {"c4": 16384, "c5": 65536}
REGION_SOURCE = os.path.join(ROOT, "paper_1609_08377_amd", "csrc", "region.hip")
C5_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "compact_kernel_c5_traffic.md")


def cpu_baseline(sysm, shifts, gpu_iters_mean: float, budget_s: float = 20.0):
    """Time the CPU oracle (plain C, OpenMP over columns) on a bounded sample."""
    import oracle
    A, B = oracle.to_csr(sysm, "A"), oracle.to_csr(sysm, "B")
    nthreads = oracle.max_threads()
    rng = np.random.default_rng(7)
    cols = np.sort(rng.choice(A.n, size=nthreads, replace=False)).astype(np.int32)
    # calibrate: a few iterations, then size the sample to the budget
    probe_it = 20
    t0 = time.perf_counter()
    oracle.shifted_solve(A, B, cols, shifts, tol=1e-8, max_it=probe_it, full=False, true_residual=False)
    t_probe = time.perf_counter() - t0
    per_it = t_probe / probe_it
    n_it = int(max(probe_it, min(gpu_iters_mean, budget_s / max(per_it, 1e-9))))
    t0 = time.perf_counter()
    r = oracle.shifted_solve(A, B, cols, shifts, tol=1e-8, max_it=n_it, full=False, true_residual=False)
    t = time.perf_counter() - t0
    done_it = float(np.mean(r.iters))
    # columns advance in parallel (one per thread): full-convergence time per column batch
    t_full = t / done_it * gpu_iters_mean
    value = len(cols) * len(shifts) / t_full
    sample = (f"{len(cols)} columns (one per thread) x {len(shifts)} shifts, oracle shifted COCG run for "
              f"{done_it:.0f} iterations in {t:.1f} s and scaled to the {gpu_iters_mean:.0f} outer iterations "
              f"the GPU needed for convergence")
    return {"value": value, "unit": "column-shift solves/s", "cores": nthreads, "kind": "oracle", "sample": sample}


def source_digest(path: str = PASS_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_traffic(kernel_tag: str, summary: str = TRAFFIC_SUMMARY, source: str = PASS_SOURCE):
    """HBM bytes per launch of the timed kernel from the committed counter summary.

    The summary holds lines `traffic <tag> <source digest> <bytes per launch>`;
    the figure counts only if it was taken on the current kernel source."""
    if not os.path.exists(summary):
        return None
    digest = source_digest(source)
    with open(summary) as f:
        for line in f:
            m = re.match(r"^traffic\s+(\S+)\s+(\S+)\s+([0-9.eE+]+)\s*$", line.strip().strip("`"))
            if m and m.group(1) == kernel_tag and m.group(2) == digest:
                return float(m.group(3))
    return None


def copy_calibration(nbytes: int):
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


def cpu_baseline_arnoldi(sysm, centres, radii, nu, budget_s: float = 15.0):
    """Time the multiple Arnoldi oracle (region carving + numpy/LAPACK) on a
    bounded sample of the benchmark's columns."""
    import oracle
    from oracle import arnoldi as oma
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        cores = 1
    rng = np.random.default_rng(11)
    order = rng.permutation(centres.size)
    n_cols = 0
    t0 = time.perf_counter()
    for i in order:
        atoms = oracle.region_atoms(sysm, int(centres[i]), float(radii[i]))
        for q in range(int(sysm.n_orb[centres[i]])):
            oma.region_column(sysm, atoms, int(sysm.orb_off[centres[i]]) + q, nu)
            n_cols += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t = time.perf_counter() - t0
    return {"value": n_cols / t, "unit": "columns/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_cols} columns of randomly chosen regions of the timed set, one after another "
                      f"(region carving, block Krylov basis, dense Rayleigh-Ritz) in {t:.1f} s; numpy/LAPACK "
                      f"with {cores} BLAS threads"}


def run_arnoldi(args):
    """One step = the multiple Arnoldi method (Eqs. 15-18) for every column of a
    set of kappa-atom regions: the subspace basis, the reduced pencils, the
    Eq. 18 weights, and rho on the column patterns plus e_j^T rho X e_j."""
    import ctypes

    import torch

    import synth
    import paper_1609_08377_amd as el

    n_atoms = WORKLOADS["c3"][0]
    sysm = synth.make_system(n_atoms, synth.config_seed(3))
    centres = np.arange(min(args.centres, n_atoms), dtype=np.int32)
    t_plan = time.perf_counter()
    radii = synth.kappa_radii(sysm, centres, args.kappa)
    ctx = el.Context(0)
    mat = el.Matrix.from_system(ctx, sysm)
    reg = el.Regions(ctx, mat, centres, radii, args.tile)
    t_plan = time.perf_counter() - t_plan
    lib = el.lib()
    lib.elses_ctx_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.elses_ctx_pass_stats.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6
    mu, kT = 0.0, 0.01
    small = el.Regions(ctx, mat, centres[:8], radii[:8], args.tile)
    el.region_arnoldi(ctx, small, nu=args.nu, mu=mu, kT=kT, want_rho=True)
    for w in range(args.warmup):
        print(f"warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
        el.region_arnoldi(ctx, reg, nu=args.nu, mu=mu, kT=kT, want_rho=True)
    lib.elses_ctx_set_profiling(ctx._h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for st in range(args.steps):
        out = el.region_arnoldi(ctx, reg, nu=args.nu, mu=mu, kT=kT, want_rho=True)
        print(f"step {st + 1}/{args.steps} done ({reg.n_cols} columns)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, avg_us, nbytes, flops = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    total, slots = ctypes.c_int64(), ctypes.c_int32()
    lib.elses_ctx_pass_stats(ctx._h, ctypes.byref(launches), ctypes.byref(avg_us), ctypes.byref(nbytes),
                             ctypes.byref(flops), ctypes.byref(total), ctypes.byref(slots))
    achieved = nbytes.value / (avg_us.value * 1e-6) / 1e9 if avg_us.value > 0 else 0.0
    value = reg.n_cols * args.steps / dt
    ma_tag = f"ma_update_regions{centres.size}"
    traffic = (committed_traffic(ma_tag, MA_TRAFFIC_SUMMARY, MA_SOURCE)
               if args.kappa == 100 and args.nu == 30 and args.tile == 64 else None)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_tag": ma_tag,
            "kernel": "ma_update_kernel<2> (Gram-Schmidt update: 2 candidates minus their projections on the 2b "
                      "basis vectors)",
            "bytes_per_launch": nbytes.value, "avg_launch_us": round(avg_us.value, 2),
            "timed_launches": launches.value}
    res = {
        "metric": "multiple-Arnoldi columns/sec (nu=%d, Eq. 18 sums and rho on the column patterns)" % args.nu,
        "value": round(value, 2), "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * dt / args.steps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"multiple Arnoldi on {centres.size} regions of {args.kappa} atoms (the centre "
                               f"atoms are {centres.size} consecutive atoms of the 50000-atom box's Morton order, "
                               f"a compact sub-volume) of the 50000-atom amorphous hydrocarbon box, all orbitals "
                               f"of each centre, nu={args.nu}, FP64",
                   "n_atoms": n_atoms, "regions": int(centres.size), "kappa": args.kappa, "nu": args.nu,
                   "columns": reg.n_cols, "region_tiles": reg.n_tiles, "tile_width": args.tile,
                   "tile_rows_total": reg.rows_total,
                   "useful_lane_fraction": round(reg.useful_rows / (reg.rows_total * args.tile), 4),
                   "region_orbitals_min_mean_max": [int(reg.region_orbitals.min()),
                                                    round(float(reg.region_orbitals.mean()), 1),
                                                    int(reg.region_orbitals.max())],
                   "subspace_dim_mean": round(float(out["dim"].mean()), 2),
                   "trace_rhoB_sum": round(float(out["col_traces"][:, 0].sum()), 6),
                   "region_set_build_s": round(t_plan, 2)},
        "roofline": roof,
    }
    if not args.no_cpu:
        print("timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline_arnoldi(sysm, centres, radii, args.nu, args.cpu_budget)
    print(json.dumps(res), flush=True)


def tile_idle(sysm, centres, iters, L):
    """Idle share of the lane-iterations of region tiles: consecutive regions fill
    tiles of L column slots, a tile runs until its slowest column converges, and a
    lane whose column has converged waits (region tiles have no refill)."""
    it = np.asarray(iters, dtype=np.float64)
    busy = lanes = 0.0
    c = used = 0
    tile = []
    for cen in centres:
        nc = int(sysm.n_orb[cen])
        if used + nc > L:
            t = it[tile]
            busy += t.sum()
            lanes += t.size * t.max()
            tile, used = [], 0
        tile.extend(range(c, c + nc))
        c += nc
        used += nc
    if tile:
        t = it[tile]
        busy += t.sum()
        lanes += t.size * t.max()
    return 1.0 - busy / lanes


def run_balance(args):
    """Ordered against disordered input (the paper's ideal diamond crystal against
    its amorphous polymers, Table II): the same region-mode shifted solve on
    kappa-atom regions of each, and the share of idle lane-iterations in the
    region tiles, the analogue of the barrier time the paper attributes to load
    imbalance (0.014 of the elapsed time for the crystal, 0.19 for the polymer)."""
    import torch

    import synth
    import paper_1609_08377_amd as el

    z = synth.shift_grid(64)
    cw = (-(1.0 / np.pi) * (2.0 / 64) * 0.5 * (1.0 - np.tanh(0.5 * (z.real - 0.0) / 0.01))).astype(np.complex128)
    ctx = el.Context(0)
    cases = {}
    for name, make in (("amorphous", lambda: synth.make_system(WORKLOADS["c3"][0], synth.config_seed(3))),
                       ("diamond", lambda: synth.make_diamond(18, synth.config_seed(6)))):
        sysm = make()
        n_cen = args.centres if name == "amorphous" else max(1, args.centres // 2)
        centres = np.arange(min(n_cen, sysm.n_atoms), dtype=np.int32)
        radii = synth.kappa_radii(sysm, centres, args.kappa)
        mat = el.Matrix.from_system(ctx, sysm)
        reg = el.Regions(ctx, mat, centres, radii, args.tile)
        small = el.Regions(ctx, mat, centres[:4], radii[:4], args.tile)
        el.region_solve(ctx, small, z, cw, want_x=False, max_outer=16, allow_not_converged=True)
        torch.cuda.synchronize()
        print(f"{name}: solving {reg.n_cols} columns", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        out = el.region_solve(ctx, reg, z, cw, want_x=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        iters = out["iters"].cpu().numpy()
        idle = tile_idle(sysm, centres, iters, args.tile)
        cases[name] = {"atoms": int(sysm.n_atoms), "regions": int(centres.size), "columns": int(reg.n_cols),
                       "region_orbitals_min_max": [int(reg.region_orbitals.min()), int(reg.region_orbitals.max())],
                       "outer_iters_min_mean_max": [int(iters.min()), round(float(iters.mean()), 1),
                                                    int(iters.max())],
                       "idle_lane_fraction": round(idle, 4), "solve_s": round(dt, 3),
                       "column_shift_solves_per_s": round(reg.n_cols * 64 / dt, 1)}
        del reg, small, mat
    res = {"metric": "idle share of region-tile lane-iterations (load imbalance), amorphous vs diamond",
           "value": cases["amorphous"]["idle_lane_fraction"], "unit": "fraction", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": round(1000.0 * cases["amorphous"]["solve_s"], 1),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"region-mode shifted solves (64 shifts, tol 1e-8, FP64) on {args.kappa}-atom "
                                  f"regions around consecutive (Morton-order) atoms of the 50000-atom amorphous box "
                                  f"and of a 46656-atom ideal diamond crystal, {args.tile}-lane tiles",
                      "kappa": args.kappa, "tile_width": args.tile, "disordered": cases["amorphous"],
                      "ordered": cases["diamond"],
                      "idle_ratio_disordered_over_ordered": round(
                          cases["amorphous"]["idle_lane_fraction"] /
                          max(cases["diamond"]["idle_lane_fraction"], 1e-12), 2)}}
    print(json.dumps(res), flush=True)


def popcount8(m):
    m = np.asarray(m, dtype=np.uint8)
    return np.unpackbits(m[:, None], axis=1).sum(1)


def cpu_baseline_regions(sysm, centres, masks, radii, z, gpu_iters_mean: float, budget_s: float = 20.0):
    """The CPU oracle on a bounded sample of the benchmark's region columns: each
    thread carves one column's region and runs the oracle's shifted COCG on it."""
    import concurrent.futures as cf

    import oracle
    nthreads = oracle.max_threads()
    rng = np.random.default_rng(13)
    pick = rng.choice(centres.size, size=nthreads, replace=False)
    jobs = []
    for r in pick:
        atoms = oracle.region_atoms(sysm, int(centres[r]), float(radii[r]))
        Ar, Br, omap = oracle.carve_region(sysm, atoms)
        q = int(np.nonzero([(int(masks[r]) >> b) & 1 for b in range(8)])[0][0])
        j = int(sysm.orb_off[centres[r]]) + q
        jobs.append((Ar, Br, int(np.nonzero(omap == j)[0][0])))

    def run(job, n_it):
        Ar, Br, jl = job
        r = oracle.shifted_solve(Ar, Br, np.array([jl], np.int32), z, tol=1e-8, max_it=n_it, full=False,
                                 true_residual=False, nthreads=1)
        return float(r.iters[0])

    with cf.ThreadPoolExecutor(max_workers=nthreads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda jb: run(jb, 20), jobs))
        per_it = (time.perf_counter() - t0) / 20
        n_it = int(max(20, min(gpu_iters_mean, budget_s / max(per_it, 1e-9))))
        t0 = time.perf_counter()
        done = list(ex.map(lambda jb: run(jb, n_it), jobs))
        t = time.perf_counter() - t0
    done_it = float(np.mean(done))
    t_full = t / done_it * gpu_iters_mean
    value = len(jobs) * len(z) / t_full
    sample = (f"{len(jobs)} region columns (one per thread, regions carved by the oracle) x {len(z)} shifts, "
              f"oracle shifted COCG (CSR, CG overlap solves) run for {done_it:.0f} iterations in {t:.1f} s and "
              f"scaled to the {gpu_iters_mean:.0f} outer iterations the GPU needed; COCG needs about 6 % more "
              f"iterations than the GPU's Lanczos recurrences, so the scaled rate slightly flatters the oracle")
    return {"value": value, "unit": "column-shift solves/s", "cores": nthreads, "kind": "oracle", "sample": sample}


def train_spai(ctx, el, seed: int):
    """The learned preconditioner's network, trained by the library's kernels on the exact
    inverses of three 500-atom boxes of the same generator (FP32, Adam)."""
    import torch

    feats, targs, masks = [], [], []
    for s_ in (11, 12, 13):
        m = el.Matrix.from_system(ctx, __import__("synth").make_system(500, s_))
        feats.append(el.spai_features(ctx, m))
        T, W = el.spai_targets(ctx, m)
        targs.append(T)
        masks.append(W)
    theta = torch.as_tensor(el.mlp_init(seed + 5), dtype=torch.float32).cuda()
    el.spai_train(ctx, theta, torch.cat(feats), torch.cat(targs), torch.cat(masks), steps=1500, batch=4096,
                  lr=2e-3, seed=1)
    return theta


def region_iters(sets, iters_all, args, n_sets):
    """Sum over the timed steps of each region's outer iterations (its slowest column)."""
    tot = 0
    for st, it in enumerate(iters_all):
        reg = sets[(args.warmup + st) % n_sets]
        it = it.cpu().numpy()
        per = np.zeros(int(reg.col_region.max()) + 1, dtype=np.int64)
        np.maximum.at(per, reg.col_region, it)
        tot += int(per.sum())
    return tot


def run_sampled(args):
    """One step = one compact region-set solve (elses_regions_solve) over a batch of
    consecutive sampled-column regions of the box: every region's shifted solve to
    tol 1e-8 (Lanczos outer steps, FP32 Richardson overlap solves with FP64
    refinement, fused multi-shift update), rho on the column patterns and
    e_j^T rho B e_j, e_j^T rho A e_j per column.  The region sets are built before
    the timed region; steps cycle through them."""
    import ctypes

    import torch

    import synth
    import paper_1609_08377_amd as el

    cfg = args.config
    n_atoms, K, desc = WORKLOADS[cfg]
    seed = synth.config_seed(int(cfg[1:]))
    t0 = time.perf_counter()
    sysm = synth.make_system(n_atoms, seed)
    t_gen = time.perf_counter() - t0
    print(f"{cfg}: system generated in {t_gen:.1f} s (M={sysm.M})", file=sys.stderr, flush=True)
    z = synth.shift_grid(K)
    cw = (-(1.0 / np.pi) * (2.0 / K) * 0.5 * (1.0 - np.tanh(0.5 * (z.real - 0.0) / 0.01))).astype(np.complex128)
    mixed = (args.precision or "mixed") == "mixed"
    ctx = el.Context(0)
    t0 = time.perf_counter()
    mat = el.Matrix.from_system(ctx, sysm, precision="mixed")
    t_mat = time.perf_counter() - t0
    print(f"{cfg}: matrix uploaded in {t_mat:.1f} s", file=sys.stderr, flush=True)
    precond = cfg == "c4" and not args.no_precond
    t_train = 0.0
    if precond:
        t0 = time.perf_counter()
        theta = train_spai(ctx, el, seed)
        el.set_preconditioner(ctx, mat, theta, bf16=True)
        t_train = time.perf_counter() - t0
        print(f"{cfg}: network trained on 500-atom boxes and M assembled in {t_train:.1f} s", file=sys.stderr,
              flush=True)
    cols = synth.sample_columns(sysm, N_SAMPLED[cfg], seed)
    centres, masks, radii = synth.column_regions(sysm, cols, seed)
    ncol = popcount8(masks)
    # batches of consecutive regions holding about args.batch columns each
    cut = np.searchsorted(np.cumsum(ncol), np.arange(args.batch, ncol.sum(), args.batch), side="left") + 1
    bounds = np.concatenate([[0], cut, [centres.size]])
    batches = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    n_sets = max(1, min(len(batches), args.steps + args.warmup, args.max_sets))
    t0 = time.perf_counter()
    sets = []
    for a, b in batches[:n_sets]:
        sets.append(el.Regions(ctx, mat, centres[a:b], radii[a:b], orb_mask=masks[a:b]))
    t_sets = time.perf_counter() - t0
    print(f"{cfg}: {n_sets} region sets of ~{args.batch} columns built in {t_sets:.1f} s", file=sys.stderr,
          flush=True)
    lib = el.lib()
    lib.elses_ctx_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.elses_ctx_pass_stats.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6

    def step(reg, **kw):
        kw.setdefault("precond", precond)
        return el.region_solve(ctx, reg, z, cw, want_x=True, mixed=mixed, **kw)

    # load the kernels outside the timed region
    small = el.Regions(ctx, mat, centres[:4], radii[:4], orb_mask=masks[:4])
    step(small, max_outer=16, allow_not_converged=True)
    for w in range(args.warmup):
        step(sets[w % n_sets])
        print(f"warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
    lib.elses_ctx_set_profiling(ctx._h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_solves = 0
    iters_all, resid_max, trace_b = [], 0.0, 0.0
    products = fallbacks = 0
    for st in range(args.steps):
        reg = sets[(args.warmup + st) % n_sets]
        out = step(reg)
        n_solves += reg.n_cols * K
        pr, fb = el.solve_counts(ctx)
        products += pr
        fallbacks += fb
        iters_all.append(out["iters"])
        resid_max = max(resid_max, float(out["resid"].max()))
        trace_b += float(out["traces"][0])
        print(f"step {st + 1}/{args.steps} done ({reg.n_cols} columns)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, avg_us, nbytes, flops = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    total, width = ctypes.c_int64(), ctypes.c_int32()
    lib.elses_ctx_pass_stats(ctx._h, ctypes.byref(launches), ctypes.byref(avg_us), ctypes.byref(nbytes),
                             ctypes.byref(flops), ctypes.byref(total), ctypes.byref(width))
    idle_share, _ = el.region_idle(ctx)
    lib.elses_ctx_set_profiling(ctx._h, 0)
    iters = torch.cat(iters_all).cpu().numpy()
    value = n_solves / dt
    achieved = nbytes.value / (avg_us.value * 1e-6) / 1e9 if avg_us.value > 0 else 0.0
    tag = f"compact_{cfg}_{'mixed' if mixed else 'fp64'}_w{width.value}_b{args.batch}"
    traffic = committed_traffic(tag, C5_TRAFFIC_SUMMARY, REGION_SOURCE)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"compact_kernel<{'float' if mixed else 'double'}, {width.value}> (persistent: every outer step "
                      f"of every region, regions from a device queue; the launches of the other column widths "
                      f"overlap it and are counted with it)",
            "traffic_tag": tag, "bytes_per_launch": nbytes.value, "avg_launch_us": round(avg_us.value, 1),
            "timed_launches": launches.value}
    # audit subsample (untimed): the first regions of the first set, every column carried
    # on its whole region and its FP64 true residual recomputed in the kernel
    n_aud = min(48, centres.size)
    areg = el.Regions(ctx, mat, centres[:n_aud], radii[:n_aud], orb_mask=masks[:n_aud])
    aout = el.region_solve(ctx, areg, z, cw, want_x=False, mixed=mixed, audit_every=1, precond=precond)
    audit_max = float(aout["resid"].max())
    reg_orbs = np.concatenate([s_.region_orbitals for s_ in sets])
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "column-shift solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000.0 * dt / args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64 mixed" if mixed else "f64", "data": "synthetic",
        "config": {"workload": cfg + ": " + desc, "n_atoms": n_atoms, "M": int(sysm.M), "nnz": int(sysm.nnz),
                   "sampled_columns": int(cols.size), "regions": int(centres.size),
                   "columns_per_step_target": args.batch, "batches_in_job": len(batches),
                   "region_sets_built": n_sets, "columns_timed": int(n_solves // K), "shifts": K, "tol": 1e-8,
                   "region_orbitals_min_mean_max": [int(reg_orbs.min()), round(float(reg_orbs.mean()), 1),
                                                    int(reg_orbs.max())],
                   "outer_iters_mean": round(float(iters.mean()), 1), "outer_iters_max": int(iters.max()),
                   "max_resid_estimate": resid_max,
                   "max_true_resid_audited": audit_max,
                   "audited_columns": int(areg.n_cols),
                   "trace_rhoB_timed_columns": trace_b,
                   "sparse_products_per_region_iteration": round(products / max(1, region_iters(sets, iters_all, args,
                                                                                                  n_sets)), 2),
                   "idle_workgroup_share": round(idle_share, 4),
                   "learned_preconditioner": precond, "preconditioner_fallbacks": fallbacks,
                   "system_generation_s": round(t_gen, 1), "matrix_upload_s": round(t_mat, 1),
                   "network_training_s": round(t_train, 1), "region_set_build_s": round(t_sets, 1)},
        "roofline": roof,
    }
    if precond:
        # the same region sets with the plain overlap iteration (Chebyshev-Richardson), for the
        # comparison the learned preconditioner is built for: outer iterations, products, time
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its_p, prods_p, nc_p = [], 0, 0
        for st in range(min(args.steps, n_sets)):
            reg = sets[(args.warmup + st) % n_sets]
            o2 = step(reg, precond=False)
            prods_p += el.solve_counts(ctx)[0]
            its_p.append(o2["iters"])
            nc_p += reg.n_cols
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t1
        its_p = torch.cat(its_p).cpu().numpy()
        its_q = torch.cat(iters_all[:min(args.steps, n_sets)]).cpu().numpy()
        res["precond_comparison"] = {
            "columns": int(nc_p),
            "with_M": {"col_shift_per_s": round(value, 1), "outer_iters_mean": round(float(iters.mean()), 1),
                       "sparse_products": int(products)},
            "plain": {"col_shift_per_s": round(nc_p * K / t_p, 1), "outer_iters_mean": round(float(its_p.mean()), 1),
                      "sparse_products": int(prods_p)},
            "note": "with_M: overlap solves by CG preconditioned with the learned M (BF16 inference, FP32/FP64 "
                    "values); plain: the Chebyshev-Richardson polynomial; products count A, B and M products "
                    "per region (one product serves the region's columns)"}
    if args.plain_sample > 0:
        # the plain FP64 GPU method (tile layout, one launch sequence per outer step) against the
        # compact mixed solve on the same columns
        nb = int(np.searchsorted(np.cumsum(ncol), args.plain_sample)) + 1
        print(f"timing the plain FP64 method on {int(ncol[:nb].sum())} columns", file=sys.stderr, flush=True)
        preg = el.Regions(ctx, mat, centres[:nb], radii[:nb], 64, orb_mask=masks[:nb])
        creg = el.Regions(ctx, mat, centres[:nb], radii[:nb], orb_mask=masks[:nb])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        el.region_solve(ctx, preg, z, cw, want_x=True, mixed=False)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        t1 = time.perf_counter()
        el.region_solve(ctx, creg, z, cw, want_x=True, mixed=mixed)
        torch.cuda.synchronize()
        t_comp = time.perf_counter() - t1
        nsel = int(creg.n_cols)
        plain_rate = nsel * K / t_plain
        res["plain_fp64_comparison"] = {
            "columns": nsel, "regions": nb,
            "plain_fp64_tiles_col_shift_per_s": round(plain_rate, 1),
            "this_path_same_sample_col_shift_per_s": round(nsel * K / t_comp, 1),
            "value_over_plain": round(value / plain_rate, 2),
            "note": "plain FP64 GPU method = the same shifted solves in FP64 with region tiles of 64 column "
                    "slots advanced by one launch sequence per outer step (no persistent queue), timed on the "
                    "first sampled regions; value_over_plain compares the timed steps' rate with it (the "
                    "compact launch needs many more regions than this sample to fill the GPU)"}
    if not args.no_cpu:
        print("timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline_regions(sysm, centres, masks, radii, z, float(iters.mean()),
                                                   args.cpu_budget)
    print(json.dumps(res), flush=True)


def run_infer(args):
    """The learned preconditioner's BF16 inference (matrix-core kernel) on every
    atom pair of the c4 box (100000 atoms): pairs per second and dense BF16
    TFLOP/s against the BF16 MFMA peak.  The network is a seeded random
    initialisation (the time does not depend on the weights); the features are
    computed once before the timed region; each timed call converts the
    weights to BF16 and runs the inference kernel."""
    import torch

    import synth
    import paper_1609_08377_amd as el

    n_atoms = WORKLOADS["c4"][0]
    sysm = synth.make_system(n_atoms, synth.config_seed(4))
    ctx = el.Context(0)
    mat = el.Matrix.from_system(ctx, sysm)
    feat = el.spai_features(ctx, mat)
    theta = torch.as_tensor(el.mlp_init(synth.config_seed(4) + 5), dtype=torch.float32).cuda()
    n = int(feat.shape[0])
    for _ in range(max(1, args.warmup)):
        el.spai_predict(ctx, theta, feat, bf16=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        el.spai_predict(ctx, theta, feat, bf16=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    flop = 2.0 * sum(a * b for a, b in ((40, 128), (128, 128), (128, 128), (128, 16))) * n
    print(json.dumps({"method": "infer", "pairs": n, "ms_per_call": round(dt * 1e3, 3),
                      "pairs_per_s": round(n / dt, 1), "tflops_per_call": round(flop / dt / 1e12, 2),
                      "flop_per_call": flop, "peak_tflops_bf16": 2500.0,
                      "note": "per call: weight conversion to BF16, the inference kernel, allocation of "
                              "its weight buffer and a stream synchronisation; the kernel's own time is "
                              "in the rocprofv3 trace"}), flush=True)


def run_pass(args):
    """The sparse pass alone at a workload's full matrix size: the Richardson step
    of the overlap solve (FP32-stored B with FP32 vectors for c5, FP64
    otherwise) on `--slots` right-hand sides, timed with HIP events over
    back-to-back launches, against the HBM roofline."""
    import ctypes

    import synth
    import paper_1609_08377_amd as el

    n_atoms, _, desc = WORKLOADS[args.config]
    precision = args.precision or ("mixed" if args.config == "c5" else "fp64")
    slots = args.slots or 256
    t0 = time.perf_counter()
    sysm = synth.make_system(n_atoms, synth.config_seed(int(args.config[1:])))
    ctx = el.Context(0)
    mat = el.Matrix.from_system(ctx, sysm, precision=precision)
    t_build = time.perf_counter() - t0
    lib = el.lib()
    lib.elses_time_pass.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    kind, w = (5, 4.0) if precision == "mixed" else (1, 8.0)
    us = ctypes.c_double()
    ctx.check(lib.elses_time_pass(ctx._h, mat._h, kind, el._variant(args.variant), slots, max(args.steps, 1) * 25,
                                  ctypes.byref(us)))
    nnzb = int(sysm.blk_row_ptr[-1])
    nbytes = sysm.nnz * w + nnzb * 4.0 + n_atoms * 20.0 + 3.0 * sysm.M * slots * w
    achieved = nbytes / (us.value * 1e-6) / 1e9
    res = {"metric": "SpMV HBM GB/s vs peak (Richardson pass of the overlap solve at full matrix size)",
           "value": round(achieved, 1), "unit": "GB/s", "n_gpus": 1, "steps": max(args.steps, 1) * 25,
           "warmup": 1, "ms_per_step": round(us.value / 1000.0, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": args.config + ": " + desc, "n_atoms": n_atoms, "M": int(sysm.M),
                      "nnz": int(sysm.nnz), "atom_blocks": nnzb, "slots": slots, "variant": args.variant,
                      "matrix_build_s": round(t_build, 1)},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "pass_group_kernel<PASS_STEP32>" if precision == "mixed" else
                                  "pass_group_kernel<PASS_STEP>",
                        "bytes_per_launch": nbytes, "avg_launch_us": round(us.value, 2)}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=0, help="columns per step (0: 1024 for c2, 1280 for c4/c5)")
    ap.add_argument("--max-sets", type=int, default=8, help="c4/c5: region sets built (steps cycle through them)")
    ap.add_argument("--plain-sample", type=int, default=192,
                    help="c4/c5: columns on which the plain FP64 tile method is timed against this path (0: skip)")
    ap.add_argument("--cols", type=int, default=0, help="limit the column count (0 = all)")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: fp64 for c1/c2, mixed (FP32-stored A, B) for c3")
    ap.add_argument("--tile", type=int, default=-1,
                    help="region layout: 0 compact, 64 / 128 tile width (default: compact for c3 solves, 64 for "
                         "the arnoldi and balance methods, which need tiles)")
    ap.add_argument("--regions", type=int, default=N_REGIONS, help="c3: number of regions")
    ap.add_argument("--region-order", default="index", choices=["index", "size"],
                    help="c3: pack regions in atom order, or largest radius first")
    ap.add_argument("--copy-calib", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--variant", default="auto", choices=["auto", "direct", "staged8", "staged4", "grouped", "grouped2", "grouped1"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-precond", action="store_true", help="c4: skip the learned preconditioner")
    ap.add_argument("--max-outer", type=int, default=20000,
                    help="cap on outer iterations (profiling runs only: capped runs do not converge)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--method", default="shifted", choices=["shifted", "arnoldi", "balance", "pass", "infer"],
                    help="arnoldi: the multiple Arnoldi method on kappa-atom regions of the 50000-atom box; "
                         "balance: idle lanes of region tiles, amorphous box against a diamond crystal")
    ap.add_argument("--centres", type=int, default=4096, help="arnoldi: region centres (consecutive atoms)")
    ap.add_argument("--nu", type=int, default=30, help="arnoldi: subspace dimension")
    ap.add_argument("--kappa", type=int, default=100, help="arnoldi: atoms per region")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU: sharding the columns over several GPUs "
                                   "is not implemented", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.method == "arnoldi":
        run_arnoldi(args)
        return
    if args.method == "balance":
        run_balance(args)
        return
    if args.method == "infer":
        run_infer(args)
        return
    if args.batch == 0:
        args.batch = 1280 if args.config in N_SAMPLED else 1024
    if args.tile < 0:
        args.tile = 0 if args.method == "shifted" else 64
    if args.method == "pass":
        run_pass(args)
        return
    if args.config in N_SAMPLED:
        run_sampled(args)
        return

    import torch

    import synth
    import paper_1609_08377_amd as el

    n_atoms, K, desc = WORKLOADS[args.config]
    seed = synth.config_seed(int(args.config[1:]))
    sysm = synth.make_system(n_atoms, seed)
    z = synth.shift_grid(K)
    cw = (-(1.0 / np.pi) * (2.0 / K) * 0.5 * (1.0 - np.tanh(0.5 * (z.real - 0.0) / 0.01))).astype(np.complex128)
    all_cols = np.arange(sysm.M, dtype=np.int32)
    if args.cols:
        all_cols = all_cols[:args.cols]
    batches = [all_cols[i:i + args.batch] for i in range(0, len(all_cols), args.batch)]
    region_mode = args.config == "c3"
    precision = args.precision or ("mixed" if region_mode else "fp64")
    mixed = precision == "mixed"

    ctx = el.Context(0)
    mat = el.Matrix.from_system(ctx, sysm, precision=precision)
    lib = el.lib()
    import ctypes
    lib.elses_ctx_set_profiling.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.elses_ctx_pass_stats.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 6

    extra = {}
    if region_mode:
        centres, radii = synth.sample_regions(sysm, args.regions, seed)
        if args.region_order == "size":
            o = np.argsort(-radii, kind="stable")
            centres, radii = centres[o], radii[o]
        t_plan = time.perf_counter()
        reg = el.Regions(ctx, mat, centres, radii, args.tile)
        extra = {"regions": int(centres.size), "region_tiles": reg.n_tiles,
                 "layout": "compact" if args.tile == 0 else f"tiles of {args.tile}",
                 "lane_rows_total": reg.rows_total,
                 "useful_lane_fraction": round(reg.useful_rows / (reg.rows_total * max(args.tile, 1)), 4),
                 "region_orbitals_min_mean_max": [int(reg.region_orbitals.min()),
                                                  round(float(reg.region_orbitals.mean()), 1),
                                                  int(reg.region_orbitals.max())],
                 "region_set_build_s": round(time.perf_counter() - t_plan, 2),
                 "region_order": args.region_order}
        small = el.Regions(ctx, mat, centres[:8], radii[:8], args.tile)
        batches = [reg.cols]

        def step(cols, max_outer=args.max_outer, r=reg):
            return el.region_solve(ctx, r, z, cw, want_x=True, max_outer=max_outer,
                                   allow_not_converged=max_outer < 20000, variant=args.variant, mixed=mixed)

        step(None, max_outer=16, r=small)
    else:
        def step(cols, max_outer=args.max_outer):
            return el.density_matrix(ctx, mat, cols, z, cw, slots=args.slots, want_x=True, max_outer=max_outer,
                                     allow_not_converged=max_outer < 20000, variant=args.variant, mixed=mixed)

        # load the kernels and touch the allocator outside the timed region
        step(batches[0][:64], max_outer=16)
    for w in range(args.warmup):
        print(f"warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
        step(batches[w % len(batches)])
    lib.elses_ctx_set_profiling(ctx._h, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    n_solves = 0
    iters_all, resid_max, trace_b = [], 0.0, 0.0
    for s in range(args.steps):
        cols = batches[s % len(batches)]
        out = step(cols)
        n_solves += len(cols) * K
        print(f"step {s + 1}/{args.steps} done ({len(cols)} columns)", file=sys.stderr, flush=True)
        iters_all.append(out["iters"])
        resid_max = max(resid_max, float(out["resid"].max()))
        trace_b += float(out["traces"][0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches = ctypes.c_int64()
    avg_us = ctypes.c_double()
    nbytes = ctypes.c_double()
    flops = ctypes.c_double()
    total = ctypes.c_int64()
    slots = ctypes.c_int32()
    lib.elses_ctx_pass_stats(ctx._h, ctypes.byref(launches), ctypes.byref(avg_us), ctypes.byref(nbytes),
                             ctypes.byref(flops), ctypes.byref(total), ctypes.byref(slots))
    ms_per_step = 1000.0 * dt / args.steps
    value = n_solves / dt
    iters = torch.cat(iters_all).cpu().numpy()
    achieved = nbytes.value / (avg_us.value * 1e-6) / 1e9 if avg_us.value > 0 else 0.0
    tag = ("step32" if mixed else "step64") + f"_{args.config}_{args.tile if region_mode else slots.value}"
    if region_mode and (args.regions != N_REGIONS or args.region_order != "index"):
        tag += f"_{args.regions}_{args.region_order}"  # counters were taken on the default region set
    summary = C3_TRAFFIC_SUMMARY if region_mode else TRAFFIC_SUMMARY
    traffic = committed_traffic(tag, summary) if args.variant == "auto" else None
    kernel = ("pass_group_kernel<PASS_STEP32> (FP32 B SpMM + Richardson step)" if mixed else
              "pass_group_kernel<PASS_STEP> (FP64 B SpMM + Richardson step)")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel, "traffic_tag": tag,
            "bytes_per_launch": nbytes.value, "avg_launch_us": round(avg_us.value, 2),
            "timed_launches": launches.value}
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "column-shift solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64 mixed" if mixed else "f64", "data": "synthetic",
        "config": {"workload": args.config + ": " + desc + (" [mixed precision: FP32-stored A, B]" if mixed else
                                                             " [FP64]"),
                   "n_atoms": n_atoms, "M": int(sysm.M), "columns_per_step": args.batch,
                   "batches_in_job": len(batches), "columns_timed": int(n_solves // K), "shifts": K, "tol": 1e-8,
                   "slots": slots.value, "outer_iters_mean": float(iters.mean()),
                   "outer_iters_max": int(iters.max()), "max_resid_estimate": resid_max,
                   "trace_rhoB_timed_columns": trace_b, "passes_per_step": int(total.value // max(args.steps, 1)),
                   "gflops_timed_pass": round(flops.value / (avg_us.value * 1e-6) / 1e9, 1) if avg_us.value else 0,
                   **extra},
        "roofline": roof,
    }
    if region_mode:
        res["config"].pop("columns_per_step", None)
        res["config"]["batches_in_job"] = 1
        if args.tile > 0:
            res["config"]["idle_lane_fraction"] = round(tile_idle(sysm, centres, iters, args.tile), 4)
        else:
            res["roofline"]["kernel"] = (f"compact_kernel<{'float' if mixed else 'double'}, {slots.value}> (one "
                                         f"persistent launch per column-width group)")
            res["roofline"]["traffic"] = None
    if not args.no_cpu and not region_mode:
        print("timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(sysm, z, float(iters.mean()), args.cpu_budget)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
