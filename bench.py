#!/usr/bin/env python3
"""Benchmark: mixed-precision H-matrix-vector product and BiCGSTAB
time-to-1e-8 residual on one MI355X, mixed (Method 2-Mixed) vs FP64.

Workload (default): the precision-stress scene at N = 330,240 -- a unit
icosphere of level 7 (327,680 flat triangles) plus 8 randomly placed
icospheres of level 2 (radius U[0.05, 0.2], seed 0), BEM collocation at the
centroids, cluster leaf 64, eta = 2, ACA tolerance 1e-6, right-hand side 1
on every sphere.  Inputs are synthetic and seeded (the paper's 6-sphere
geometry is not available).

One step = one BiCGSTAB solve from x0 = 0 to relative residual 1e-8 with the
mixed operator, confirmed with the FP64 true residual: every stage of the
path (stage-1 z partials, stage-1 reduction with D_m, stage-2 dense + V'
streaming, the device-side Krylov vector work and the FP64 residual check).
`value` = algorithmic bytes of all products executed in the timed solves
divided by their wall time (whole-job GB/s).  The timed solves run without
per-kernel events; per-kernel durations come from separate, untimed passes
with HIP events on the product's stream: a replica of the timed solves
(per executed product) and back-to-back products (every launch executes),
the latter giving the roofline entry of the dominant kernel (stage 2).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM traffic of the dominant kernel per launch, from the rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE runs recorded in profiles/ (scaled by the
# plain-copy calibration): stage-2 bytes per launch per (workload, variant)
# and operand tile.  Valid only for the kernel and layout sources they were
# measured with (their hash).
PROFILED_TRAFFIC = {
    ("sphere-L7+8", "M2-Mixed"): {"sources_sha256_16": "c8af5550e1f96ba1",
                                  "k_stage2_bytes": {1024: 3009.0e6, 2048: 3001.0e6, 4096: 3004.0e6}},
    ("sphere-L7+8", "BF16-scaled"): {"sources_sha256_16": "c8af5550e1f96ba1",
                                     "k_stage2_bytes": {1024: 1876.2e6, 2048: 1883.1e6, 4096: 1879.8e6}},
}
PROFILED_SOURCES = ["paper_1911_00093_amd/csrc/matvec.hip", "paper_1911_00093_amd/csrc/hmat_impl.h",
                    "paper_1911_00093_amd/csrc/pack.cpp"]


def sources_hash():
    import hashlib

    h = hashlib.sha256()
    for f in PROFILED_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
WORKLOADS = {
    "plates-128": dict(leaf=64, eta=2.0, eps=1e-5, refine=1e-4,
                       desc="two 1x1 plates, gap 0.1, 128x128 squares x 4 right triangles each, N=131072; "
                            "leaf 64, eta 2, ACA 1e-5; b = +1/-1"),
    "sphere-L7+8": dict(leaf=64, eta=2.0, eps=1e-6,
                        desc="unit icosphere L7 + 8 random icosphere-L2 spheres r~U[0.05,0.2] (seed 0), "
                             "N=330240; leaf 64, eta 2, ACA 1e-6; b = 1"),
    "sphere-L4": dict(leaf=32, eta=2.0, eps=1e-6,
                      desc="unit icosphere L4, N=5120; leaf 32, eta 2, ACA 1e-6; b = 1 (cache-resident)"),
    "sphere-L6+plates": dict(leaf=64, eta=2.0, eps=1e-5, learned=True,
                             desc="unit icosphere L6 (81,920) + two 1x1 plates at gap 0.1 (240x256 squares x 2 "
                                  "triangles each, offset 3 along x), N=327,680; leaf 64, eta 2, ACA 1e-5; "
                                  "b = 1 / +1 / -1; preconditioners none, block-Jacobi, learned leaf map "
                                  "(trained on 20,000 leaves of random ellipsoids and plate pairs, seed 1)"),
    "ellipsoids-64x16": dict(leaf=32, eta=2.0, eps=1e-6, nsys=64, nrhs=16, refine=1e-4,
                             desc="64 independent geodesic ellipsoids (frequency U{10..44}, N = 20 f^2 in "
                                  "[2000, 38720], semi-axes U[0.5, 2], seed 0), N = 1,089,460 in total; leaf 32, "
                                  "eta 2, ACA 1e-6 per mesh; 16 N(0,1) right-hand sides per mesh (seed 1)"),
}


# Early-check thresholds the FP64 baseline is timed with (besides the mixed
# solve's own): a restarted BiCGSTAB can converge in fewer iterations
# whatever the precision, so every speedup is taken against the fastest.
FP64_REFINES = (0.0, 1e-2, 1e-4)


def default_refine(variant, workload):
    """Threshold of the early FP64 true-residual checks when --refine is not
    given: 1e-2 for scaled BF16 (its operator error needs them), else the
    workload's measured best (none on the sphere scene, where every restart
    costs iterations; 1e-4 on plates-128 and the 64-mesh batch, where a
    restarted recurrence converges in fewer iterations)."""
    from paper_1911_00093_amd import hmat

    return 1e-2 if variant == hmat.BF16_SCALED else WORKLOADS[workload].get("refine", 0.0)


def _r4(v):
    return None if v is None else round(v, 4)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def assemble(args, mesh, W):
    """FP64 H-matrix of one mesh with the chosen setup builder (untimed)."""
    from paper_1911_00093_amd import hmat

    if args.assembly == "gpu":
        try:
            return hmat.hmat_assemble_bem_gpu(mesh.centroids, mesh.areas, leaf=W["leaf"], eta=W["eta"],
                                              eps=W["eps"])
        except hmat.HmatError as e:  # setup only (the same matrix either way): say so and go on
            log(f"[setup] GPU assembly failed ({e}); using the host builder")
    return hmat.hmat_assemble_bem(mesh.centroids, mesh.areas, leaf=W["leaf"], eta=W["eta"], eps=W["eps"])


def assembly_note(bs):
    st = bs.stats
    return (f"{'GPU' if st['rank_cap'] else 'host'} assembly: partition {st['ms_partition']:.0f} ms, "
            f"entries + ACA {st['ms_fill']:.0f} ms" +
            (f" (k_aca {st['ms_aca']:.1f} ms, k_emit {st['ms_emit']:.1f} ms, copy-back {st['ms_copy']:.0f} ms, "
             f"host-filled blocks {st['host_blocks']})" if st["rank_cap"] else ""))


def profiled_traffic(args, variant_name, tile):
    """Stage-2 HBM bytes per launch from the committed rocprofv3 counters, if
    they were taken for this workload, variant, operand tile and these
    sources."""
    P = PROFILED_TRAFFIC.get((args.workload, variant_name))
    if (P is not None and sources_hash() == P["sources_sha256_16"] and args.drop == 0 and not args.dense_split
            and args.eps is None):
        return P["k_stage2_bytes"].get(int(tile))
    return None


def storage_label(variant, c=-1, dense_split=False, drop=0):
    """What the product streams for a precision variant (Table 1 and the
    BF16 addition); x, y, D_m and the Krylov vectors are FP64 throughout."""
    from paper_1911_00093_amd import hmat

    lab = {
        hmat.M1_DOUBLE: "fp64 dense and low-rank factors",
        hmat.M1_SINGLE: "fp32 dense and low-rank factors, x rounded to fp32, z fp32",
        hmat.M1_MIXED: "fp32 dense and low-rank factors, x fp64, z fp32",
        hmat.M2_DOUBLE: "fp64 dense and scaled factors V', W', fp64 D_m",
        hmat.M2_SINGLE: "fp32 dense and scaled factors V', W', x rounded to fp32, fp64 D_m and z",
        hmat.M2_MIXED: "fp32 dense and scaled factors V', W', fp64 D_m, x and z",
        hmat.M3: f"terms split by c = {c}: fp64 above d_max 10^-c, fp32 below; fp64 D_m; dense "
                 + ("split by column with the same c" if dense_split else "fp64"),
        hmat.BF16_SCALED: "bf16 low-rank factors with power-of-two fp32 scales per block, fp32 dense, fp64 z",
    }[variant]
    return lab + (f"; terms below d_max 10^-{drop} deleted" if drop else "")


def host_cpu():
    """CPU model, logical CPUs usable by this process and the clock the kernel reports."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count(),
            "cpu_mhz": mhz}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere-L7+8", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="M2-Mixed")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--poll-every", type=int, default=4)
    ap.add_argument("--matvec-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-matvecs", type=int, default=3)
    ap.add_argument("--cpu-solve-iters", type=int, default=3,
                    help="oracle BiCGSTAB iterations timed for the CPU solve estimate")
    ap.add_argument("--eps", type=float, default=None, help="ACA tolerance (default: the workload's)")
    ap.add_argument("--refine", type=float, default=None,
                    help="early FP64 true-residual check ratio (default 1e-2 for BF16-scaled, else the "
                         "workload's: 1e-4 for plates-128 and ellipsoids-64x16, 0 otherwise); the FP64 "
                         "baseline is timed with 0, 1e-2, 1e-4 and this ratio, the fastest kept")
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "gmres"],
                    help="Krylov solver of the single-system workloads (GMRES: restarted, --restart steps)")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--drop", type=int, default=0,
                    help="Methods 2/3: delete low-rank terms with d_i < d_max 10^-drop (Sec. 4.5; 0 = off)")
    ap.add_argument("--c", type=int, default=-1, help="Method 3 split constant (Eqs. 19-20)")
    ap.add_argument("--dense-split", action="store_true",
                    help="Method 3: split the dense leaves by column with the same c (Sec. 4.5)")
    ap.add_argument("--assembly", default="gpu", choices=["gpu", "host"],
                    help="setup builder: entries and ACA on the GPU (default) or on the host threads")
    ap.add_argument("--no-bf16", action="store_true",
                    help="sphere-L7+8: skip the scaled-BF16 solves reported beside the headline variant")
    ap.add_argument("--no-autotune", action="store_true",
                    help="single-system workloads: keep the untuned launch configuration")
    ap.add_argument("--accuracy-tol", type=float, default=1e-10,
                    help="also time mixed and FP64 solves to this tolerance (0: skip), the mixed one with early "
                         "FP64 true-residual checks, and report both solutions' error against the FP64 1e-12 one")
    ap.add_argument("--sweep-variants", action="store_true",
                    help="every Table 1 variant, Method 3 for c = -1..7 and BF16 on the workload's blocks")
    ap.add_argument("--train-leaves", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=100)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}): the library has no multi-GPU path "
              "(independent systems would shard with no exchange; one system by row chunks with an all-gather "
              "of x per product).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1911_00093_amd import hmat, meshes, tuning

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    variant = hmat.PRECISION_NAMES.index(args.variant)
    W = dict(WORKLOADS[args.workload])
    if args.refine is None:
        args.refine = default_refine(variant, args.workload)
    if args.eps is not None:
        W["eps"] = args.eps
        W["desc"] = W["desc"].replace("ACA 1e-6", f"ACA {args.eps:g}").replace("ACA 1e-5", f"ACA {args.eps:g}")
    if "nsys" in W:
        return bench_batched(args, W, variant, dev, stream)
    if W.get("learned"):
        return bench_learned(args, W, variant, dev, stream)

    # ---------------- setup (untimed): mesh, FP64 H-matrix, conversions
    t0 = time.time()
    mesh = meshes.workload(args.workload)
    bs = assemble(args, mesh, W)
    log(f"[setup] {args.workload}: n={bs.n} blocks={bs.nblocks} assembly {time.time() - t0:.1f}s; "
        f"{assembly_note(bs)}")
    if args.sweep_variants:
        return bench_variant_sweep(args, W, mesh, bs, dev, stream)
    t0 = time.time()
    H64 = hmat.HMatrix(bs, hmat.M1_DOUBLE)
    Hm = hmat.HMatrix(bs, variant, c=args.c, drop=args.drop, dense_split=args.dense_split)
    log(f"[setup] builds {time.time() - t0:.1f}s")
    tune = {}
    if not args.no_autotune:  # launch configuration per handle, timed on its own blocks (results unchanged)
        t0 = time.time()
        for name, H in (("M1-Double", H64), (args.variant, Hm)):
            info = tuning.autotune(H, reps=10)
            tune[name] = {k: info[k] for k in ("stage1_grid", "stage2_grid", "stage2_tile")}
            tune[name].update(ms_fixed=_r4(info.get("ms_fixed")), ms_tuned=_r4(info.get("ms_tuned")),
                              cached=info["cached"])
        log(f"[setup] autotune {time.time() - t0:.1f}s: {tune}")
    st64, stm = H64.stats(), Hm.stats()
    B64, Bm = st64.algorithmic_bytes, stm.algorithmic_bytes
    b = torch.as_tensor(mesh.rhs()[bs.perm], device=dev)
    n = bs.n
    gm = args.solver == "gmres"
    wbytes = (hmat.lib().hmat_gmres_workspace_bytes(n, args.restart) if gm else hmat.hmat_solver_workspace_bytes(n))
    work = torch.empty(int(wbytes), dtype=torch.uint8, device=dev)

    def run(H, tol, x, use_graph=False, refine=None):
        if refine is None:
            refine = args.refine if H is Hm else 0.0
        if gm:
            return hmat.hmat_gmres(H, b, x=x, h_fp64=H64, tol=tol, maxiter=2000, restart=args.restart,
                                   poll_every=args.poll_every, work=work, use_graph=use_graph)
        return hmat.hmat_bicgstab(H, b, x=x, h_fp64=H64, tol=tol, maxiter=2000, poll_every=args.poll_every,
                                  work=work, refine=refine, use_graph=use_graph)

    def solve(H, tol, x=None):
        x = torch.zeros(n, dtype=torch.float64, device=dev) if x is None else x.zero_()
        return run(H, tol, x)

    # reference solution: FP64 to 1e-12
    xref, iref = solve(H64, 1e-12)
    xref = xref.clone()
    log(f"[setup] FP64 reference solve: {iref['iterations']} it, true res {iref['true_rel_res']:.2e}")

    # ---------------- warmup
    xw = torch.zeros(n, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        solve(Hm, args.tol, xw)
        solve(H64, args.tol, xw)
    torch.cuda.synchronize()

    # ---------------- timed region: K mixed solves (no per-kernel events)
    infos = []
    xs = torch.zeros(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        xs, info = solve(Hm, args.tol, xs)
        infos.append(info)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t_start
    assert all(i["status"] == 0 for i in infos), infos
    mv_bytes = sum(i["matvecs"] * Bm + i["matvecs_fp64"] * B64 for i in infos)
    value = mv_bytes / t_mixed / 1e9
    ms_per_step = 1e3 * t_mixed / args.steps
    err_mixed = float(torch.linalg.norm(xs - xref) / torch.linalg.norm(xref))

    # the same mixed solves with one iteration replayed from a HIP graph (no
    # per-kernel events can be recorded inside a graph, so this is timed apart)
    xg = torch.zeros(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        xg.zero_()
        run(Hm, args.tol, xg, use_graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t_start

    # FP64 solves, same protocol, with each threshold of FP64_REFINES and
    # the mixed solve's own; the fastest is the baseline.
    fp64_runs = {}

    def fp64_time(refine):
        if refine not in fp64_runs:
            x_ = torch.zeros(n, dtype=torch.float64, device=dev)
            run(H64, args.tol, x_, refine=refine)  # warm-up at this threshold
            torch.cuda.synchronize()
            t0_ = time.perf_counter()
            inf_ = []
            for _ in range(args.steps):
                x_.zero_()
                x_, i_ = run(H64, args.tol, x_, refine=refine)
                inf_.append(i_)
            torch.cuda.synchronize()
            fp64_runs[refine] = (time.perf_counter() - t0_, inf_, x_)
        return fp64_runs[refine][0]

    for r_ in sorted(set(FP64_REFINES) | {args.refine}) if not gm else (0.0,):
        fp64_time(r_)
    refine64 = min(fp64_runs, key=lambda r_: fp64_runs[r_][0])
    t_fp64, infos64, x64 = fp64_runs[refine64]
    err_fp64 = float(torch.linalg.norm(x64 - xref) / torch.linalg.norm(xref))
    err_same_tol = float(torch.linalg.norm(xs - x64) / torch.linalg.norm(x64))

    # a tighter tolerance: what the solution error against the FP64 1e-12
    # solve becomes when both solvers go further (untimed for the metric)
    accuracy = None
    if args.accuracy_tol > 0 and not gm:
        accuracy = {"tol": args.accuracy_tol, "mixed_refine": 1e-2}
        reps = max(1, min(args.steps, 3))
        # FP64: with each threshold of FP64_REFINES, the fastest kept
        for key, H, refine in [("mixed", Hm, 1e-2)] + [(f"fp64 {r_:g}", H64, r_) for r_ in FP64_REFINES]:
            xa = torch.zeros(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for _ in range(reps):
                xa, ia = hmat.hmat_bicgstab(H, b, x=xa.zero_(), h_fp64=H64, tol=args.accuracy_tol, maxiter=4000,
                                            poll_every=args.poll_every, work=work, refine=refine)
            torch.cuda.synchronize()
            assert ia["status"] == 0, (key, ia)
            accuracy[key] = {"ms": round(1e3 * (time.perf_counter() - t_start) / reps, 3),
                             "iterations": ia["iterations"], "restarts": ia["restarts"],
                             "true_rel_res": ia["true_rel_res"],
                             "solution_rel_err_vs_fp64_1e-12":
                                 float(torch.linalg.norm(xa - xref) / torch.linalg.norm(xref))}
        best = min((k for k in accuracy if k.startswith("fp64 ")), key=lambda k: accuracy[k]["ms"])
        accuracy["fp64"] = dict(accuracy[best], refine=float(best.split()[1]))
        for r_ in FP64_REFINES:
            del accuracy[f"fp64 {r_:g}"]
        accuracy["speedup_vs_fp64"] = round(accuracy["fp64"]["ms"] / accuracy["mixed"]["ms"], 3)
        log(f"[accuracy] {accuracy}")

    # ---------------- untimed: per-kernel durations with HIP events
    # (a) a replica of the timed mixed solves.  Products queued past the
    # recurrence's stop return at once; the device counts the products that
    # ran, so the time per executed product is the events' total over that
    # count (an upper bound: the returned launches add their few microseconds).
    Hm.set_profiling(True)
    Hm.kernel_times()  # reset
    xp = torch.zeros(n, dtype=torch.float64, device=dev)
    executed = 0
    for _ in range(args.steps):
        xp, ip = solve(Hm, args.tol, xp)
        executed += ip["matvecs"]
    ktp, kcount_p = Hm.kernel_times()
    Hm.set_profiling(False)
    solve_kernel_ms = [round(t * kcount_p / max(executed, 1), 4) for t in ktp]

    # (b) back-to-back products (the paper's matvec-only protocol): every
    # launch executes.  Whole-product time from events around all of them
    # (no per-kernel events in between), then the per-kernel durations from
    # a second pass with the per-kernel events on.
    matvec_gbs = {}
    kt_b2b = {}
    xv = torch.randn(n, dtype=torch.float64, device=dev)
    yv = torch.empty_like(xv)
    for name, H in (("M1-Double", H64), (args.variant, Hm)):
        ms, ms_best = product_sets(H, xv, yv, args.matvec_reps, stream)
        H.set_profiling(True)
        H.kernel_times()
        for _ in range(args.matvec_reps):
            H.matvec(xv, yv, stream=stream)
        kt_b2b[name], _ = H.kernel_times()
        H.set_profiling(False)
        matvec_gbs[name] = dict(ms=round(ms, 4), ms_best_set=round(ms_best, 4),
                                gbs=round(H.stats().algorithmic_bytes / ms / 1e6, 1),
                                frac=round(H.stats().algorithmic_bytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                                kernel_ms={"stage1": round(kt_b2b[name][0], 4),
                                           "stage1_reduce": round(kt_b2b[name][1], 4),
                                           "stage2": round(kt_b2b[name][2], 4)})
    kt = kt_b2b[args.variant]

    # STREAM-read ceiling over a buffer larger than the MALL
    buf = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    hmat.hmat_stream_read(buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        hmat.hmat_stream_read(buf)
    e1.record(stream)
    torch.cuda.synchronize()
    stream_gbs = buf.numel() * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    for m_ in matvec_gbs.values():
        m_["frac_of_stream_read"] = round(m_["gbs"] / stream_gbs, 4)
    # plain copy of a known size (1 GiB read + 1 GiB written): the reference
    # for scaling hardware byte counters of the product kernels
    dst = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    hmat.hmat_stream_copy(dst, buf[: 1 << 30])
    e0.record(stream)
    hmat.hmat_stream_copy(dst, buf[: 1 << 30])
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del buf, dst

    traffic = profiled_traffic(args, args.variant, tune.get(args.variant, {}).get("stage2_tile", 2048))

    # roofline of the dominant kernel (stage 2): algorithmic bytes of one
    # launch over its average duration in the back-to-back pass
    k2_bytes = stm.stage2_algorithmic_bytes
    k1_bytes = stm.stage1_algorithmic_bytes
    k2_gbs = k2_bytes / (kt[2] / 1e3) / 1e9 if kt[2] > 0 else 0.0
    k1_gbs = k1_bytes / (kt[0] / 1e3) / 1e9 if kt[0] > 0 else 0.0
    k2_solve_gbs = k2_bytes / (solve_kernel_ms[2] / 1e3) / 1e9 if solve_kernel_ms[2] > 0 else 0.0

    out = {
        "metric": "H-matvec GB/s and BiCG-STAB time-to-1e-8 residual, mixed vs FP64, 1 GPU",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {W['desc']}",
            "precision": args.variant,
            "storage": storage_label(variant, args.c, args.dense_split, args.drop),
            "arithmetic": "fp64 (stored values widened exactly; every product and sum in fp64)",
            "n": n,
            "step": (f"one restarted GMRES({args.restart}) solve" if gm else "one BiCGSTAB solve")
                    + f" x0=0 -> |r|/|b|<{args.tol:g} confirmed by the FP64 true residual",
            "solver": f"GMRES({args.restart})" if gm else "BiCGSTAB",
            "refine": args.refine,
            "drop": args.drop,
            "c": args.c,
            "dense_split": args.dense_split,
            "parallelism": "1 GPU",
        },
        "time_to_tol_ms": {"mixed": round(ms_per_step, 3), "fp64": round(1e3 * t_fp64 / args.steps, 3),
                           "mixed_graph_replay": round(1e3 * t_graph / args.steps, 3),
                           "fp64_by_refine": {f"{r_:g}": round(1e3 * v_[0] / args.steps, 3)
                                              for r_, v_ in sorted(fp64_runs.items())}},
        "speedup_vs_fp64": round(t_fp64 / t_mixed, 3),
        "iterations": {"mixed": infos[-1]["iterations"], "fp64": infos64[-1]["iterations"],
                       "mixed_restarts": infos[-1]["restarts"], "fp64_refine": refine64},
        "solution_rel_err": {"mixed_vs_fp64_1e-12": err_mixed, "fp64_1e-8_vs_fp64_1e-12": err_fp64,
                             "mixed_vs_fp64_same_tol": err_same_tol},
        "true_rel_res": {"mixed": infos[-1]["true_rel_res"], "fp64": infos64[-1]["true_rel_res"]},
        "accuracy_tighter_tol": accuracy,
        "bytes_per_matvec": {"mixed": int(Bm), "fp64": int(B64),
                             "mixed_stage1": int(k1_bytes), "mixed_stage2": int(k2_bytes)},
        "matvec_only": matvec_gbs,
        "autotune": tune or None,
        "row_chunks": int(stm.row_chunks),
        "kernel_ms_in_solves": {"stage1": solve_kernel_ms[0], "stage1_reduce": solve_kernel_ms[1],
                                "stage2": solve_kernel_ms[2], "launched": kcount_p, "executed": executed,
                                "note": "event time of the replica solves over the products that executed"},
        "stream_read_gbs": round(stream_gbs, 1),
        "copy_gbs": round(copy_gbs, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage2",
            "achieved": round(k2_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(k2_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(k2_bytes),
            "avg_launch_ms": round(kt[2], 4),
            "timing": f"HIP events around each of {args.matvec_reps} back-to-back products on the product's stream",
            "in_solves_achieved": round(k2_solve_gbs, 1),
            "stage1_achieved": round(k1_gbs, 1),
            "whole_product_frac": matvec_gbs[args.variant]["frac"],
            "frac_of_stream_read": round(k2_gbs / stream_gbs, 4),
        },
    }

    # the precision-stress configuration's own variant beside the headline:
    # scaled-BF16 low-rank factors, FP32 dense leaves (same protocol, its own
    # early true-residual checks)
    if args.workload == "sphere-L7+8" and variant != hmat.BF16_SCALED and not gm and not args.no_bf16:
        out["bf16_scaled"] = bench_extra_variant(args, bs, hmat.BF16_SCALED, H64, b, work, x64.new_zeros(n),
                                                 xref, fp64_time, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, W, variant, args.cpu_matvecs, Bm, args.drop, args.c,
                                           args.dense_split, b.cpu().numpy(), infos[-1], args.cpu_solve_iters,
                                           args.tol)
    print(json.dumps(out), flush=True)


def product_sets(H, xv, yv, reps, stream, sets=10):
    """Back-to-back products timed in `sets` sets of `reps` (HIP events around
    each set, nothing between the products): (mean ms, best set's ms)."""
    import torch

    for _ in range(3):
        H.matvec(xv, yv)
    per = []
    for _ in range(sets):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            H.matvec(xv, yv, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / reps)
    return float(np.mean(per)), float(min(per))


def bench_extra_variant(args, bs, variant, H64, b, work, x, xref, fp64_time, stream):
    """One more precision variant on the same blocks: K solves to tol (timed,
    no per-kernel events; early FP64 checks 1e-2 as for the variant's own
    runs), back-to-back products with per-kernel events (untimed pass)."""
    import torch

    from paper_1911_00093_amd import hmat, tuning

    H = hmat.HMatrix(bs, variant)
    tune = None
    if not args.no_autotune:
        info = tuning.autotune(H, reps=10)
        tune = {k: info[k] for k in ("stage1_grid", "stage2_grid", "stage2_tile")}
    refine = 1e-2 if variant == hmat.BF16_SCALED else 0.0
    t_fp64 = min(fp64_time(r_) for r_ in set(FP64_REFINES) | {refine})  # FP64's fastest threshold
    B = H.stats().algorithmic_bytes

    def solve():
        x.zero_()
        return hmat.hmat_bicgstab(H, b, x=x, h_fp64=H64, tol=args.tol, maxiter=2000, poll_every=args.poll_every,
                                  work=work, refine=refine)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [solve()[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(i["status"] == 0 for i in infos), infos
    accuracy = None
    if args.accuracy_tol > 0:  # reported whatever the outcome (status included), never asserted
        xa = torch.zeros_like(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xa, ia = hmat.hmat_bicgstab(H, b, x=xa, h_fp64=H64, tol=args.accuracy_tol, maxiter=4000,
                                    poll_every=args.poll_every, work=work, refine=1e-2)
        torch.cuda.synchronize()
        accuracy = {"tol": args.accuracy_tol, "status": ia["status"], "ms": round(1e3 * (time.perf_counter() - t0), 3),
                    "iterations": ia["iterations"], "restarts": ia["restarts"], "true_rel_res": ia["true_rel_res"],
                    "solution_rel_err_vs_fp64_1e-12": float(torch.linalg.norm(xa - xref) / torch.linalg.norm(xref))}
    xv = torch.randn(b.numel(), dtype=torch.float64, device=b.device)
    yv = torch.empty_like(xv)
    ms, ms_best = product_sets(H, xv, yv, args.matvec_reps, stream)
    H.set_profiling(True)
    H.kernel_times()
    for _ in range(args.matvec_reps):
        H.matvec(xv, yv, stream=stream)
    kt, _ = H.kernel_times()
    H.set_profiling(False)
    st = H.stats()
    return {"storage": storage_label(variant), "bytes_per_matvec": int(B), "refine": refine,
            "time_to_tol_ms": round(1e3 * dt / args.steps, 3), "speedup_vs_fp64": round(t_fp64 / dt, 3),
            "iterations": infos[-1]["iterations"], "restarts": infos[-1]["restarts"],
            "true_rel_res": infos[-1]["true_rel_res"],
            "solution_rel_err_vs_fp64_1e-12": float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref)),
            "matvec_ms": round(ms, 4), "matvec_ms_best_set": round(ms_best, 4), "matvec_gbs": round(B / ms / 1e6, 1),
            "matvec_frac": round(B / ms / 1e6 / HBM_PEAK_GBS, 4),
            "kernel_ms": {"stage1": round(kt[0], 4), "stage1_reduce": round(kt[1], 4), "stage2": round(kt[2], 4)},
            "stage2_frac": round(st.stage2_algorithmic_bytes / (kt[2] / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if kt[2] else None,
            "stage2_traffic": profiled_traffic(args, hmat.PRECISION_NAMES[variant],
                                               (tune or {}).get("stage2_tile", 2048)),
            "accuracy_tighter_tol": accuracy,
            "autotune": tune}


def bench_variant_sweep(args, W, mesh, bs, dev, stream):
    """Every precision variant on one workload's blocks (Table 1's six, Method 3
    for c = -1..7, Method 3 with the dense leaves split for c = -1, 0, 1,
    scaled BF16), each handle tuned: product time (10 sets of
    --matvec-reps back-to-back products, mean and best set), the product's
    difference from the FP64 product on x = 1 and on the FP64 solution, and
    the best of --steps BiCGSTAB solves to --tol confirmed by the FP64 true
    residual, with its error against an FP64 solve to 1e-12."""
    import torch

    from paper_1911_00093_amd import hmat, tuning

    n = bs.n
    H64 = hmat.HMatrix(bs, hmat.M1_DOUBLE)
    tuning.autotune(H64, reps=10)
    b = torch.as_tensor(mesh.rhs()[bs.perm], device=dev)
    work = torch.empty(hmat.hmat_solver_workspace_bytes(n), dtype=torch.uint8, device=dev)
    xref, _ = hmat.hmat_bicgstab(H64, b, tol=1e-12, maxiter=4000, work=work)
    xref = xref.clone()
    probes = {"x=1": torch.ones(n, dtype=torch.float64, device=dev), "x=sigma": xref}
    y64 = {k: H64.matvec(v).clone() for k, v in probes.items()}
    specs = ([(v, -1, False) for v in range(6)] + [(hmat.M3, c, False) for c in range(-1, 8)] +
             [(hmat.M3, c, True) for c in (-1, 0, 1)] + [(hmat.BF16_SCALED, -1, False)])
    rows, fp64_ms = [], None
    xv = torch.randn(n, dtype=torch.float64, device=dev)
    yv = torch.empty_like(xv)
    for v, c, split in specs:
        name = hmat.PRECISION_NAMES[v] + (f" c={c}" if v == hmat.M3 else "") + (", dense split" if split else "")
        H = H64 if v == hmat.M1_DOUBLE else hmat.HMatrix(bs, v, c=c, dense_split=split)
        if H is not H64:
            tuning.autotune(H, reps=10)
        ms_mean, ms_best = product_sets(H, xv, yv, args.matvec_reps, stream)
        err = {k: float(torch.linalg.norm(H.matvec(p) - y64[k]) / torch.linalg.norm(y64[k]))
               for k, p in probes.items()}
        # BF16: early checks 1e-2; the FP64 reference: its fastest threshold of FP64_REFINES
        refines = [1e-2] if v == hmat.BF16_SCALED else list(FP64_REFINES) if v == hmat.M1_DOUBLE else [0.0]
        best, x = None, torch.zeros(n, dtype=torch.float64, device=dev)
        for refine in refines:
            for _ in range(max(args.steps, 1)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = hmat.hmat_bicgstab(H, b, x=x.zero_(), h_fp64=H64, tol=args.tol, maxiter=4000,
                                             poll_every=args.poll_every, work=work, refine=refine)
                torch.cuda.synchronize()
                dt = 1e3 * (time.perf_counter() - t0)
                assert info["status"] == 0, (name, info)
                if best is None or dt < best[0]:
                    best = (dt, dict(info, refine=refine), float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref)))
        if v == hmat.M1_DOUBLE:
            fp64_ms = best[0]
        st = H.stats()
        B = st.algorithmic_bytes
        row = dict(variant=name, bytes_per_product=int(B), dense_bytes=int(st.bytes_dense), product_us_mean=round(1e3 * ms_mean, 2),
                   product_us_best=round(1e3 * ms_best, 2), gbs=round(B / ms_best / 1e6, 1),
                   err_vs_fp64_x1=err["x=1"], err_vs_fp64_sigma=err["x=sigma"],
                   iterations=best[1]["iterations"], restarts=best[1]["restarts"], refine=best[1]["refine"],
                   solve_ms=round(best[0], 3),
                   vs_fp64=round(fp64_ms / best[0], 3),
                   solution_err=best[2])
        rows.append(row)
        log(f"[sweep] {row}")
        if H is not H64:
            del H
            torch.cuda.empty_cache()
    out = {"metric": "H-matvec GB/s and BiCG-STAB time-to-1e-8 residual, every precision variant, 1 GPU",
           "workload": f"{args.workload}: {W['desc']}", "n": n, "tol": args.tol,
           "protocol": f"10 sets of {args.matvec_reps} back-to-back products (HIP events); best of "
                       f"{max(args.steps, 1)} solves x0=0 -> tol confirmed by the FP64 true residual; every handle "
                       "tuned", "variants": rows}
    print(json.dumps(out), flush=True)


def mr_product_bytes(st, nr, precision):
    """Algorithmic bytes of one product over nr right-hand sides: the stored
    matrix once, the FP64 D_m scales once, x and y (FP64) once per column."""
    from paper_1911_00093_amd import hmat

    mat = st.bytes_dense + st.bytes_v + st.bytes_w
    xs = 4 if precision in (hmat.M1_SINGLE, hmat.M2_SINGLE) else 8
    zd = st.algorithmic_bytes - mat - xs * st.n - 8 * st.n
    return mat + zd + nr * 16 * st.n, st.bytes_dense + st.bytes_v + nr * 8 * st.n


def bench_batched(args, W, variant, dev, stream):
    """Many independent systems x many right-hand sides: one step = the
    batched BiCGSTAB of every (mesh, right-hand side) pair to 1e-8, each
    confirmed by the FP64 true residual, with the iteration replayed from a
    HIP graph; the products run over all meshes and right-hand sides in one
    persistent launch per stage on the FP64 matrix cores."""
    import torch

    from paper_1911_00093_amd import hmat, meshes, tuning

    nsys, nrhs = W["nsys"], W["nrhs"]
    t0 = time.time()
    ms = meshes.random_ellipsoids(nsys, seed=0)
    if args.assembly == "gpu":
        try:
            bss = hmat.hmat_assemble_bem_gpu_batched(ms, leaf=W["leaf"], eta=W["eta"], eps=W["eps"])
        except hmat.HmatError as e:  # setup only (the same matrices either way): say so and go on
            log(f"[setup] GPU assembly failed ({e}); using the host builder")
            args.assembly = "host"
    if args.assembly != "gpu":
        bss = [assemble(args, m, W) for m in ms]
    n = sum(b.n for b in bss)
    log(f"[setup] {args.workload}: {nsys} meshes, n={n}, blocks={sum(b.nblocks for b in bss)}, "
        f"meshes + assembly {time.time() - t0:.1f}s; {assembly_note(bss[0])} (batch)")
    t0 = time.time()
    Hm = hmat.HMatrix(bss, variant, c=-1, nrhs_max=nrhs)
    H64 = hmat.HMatrix(bss, hmat.M1_DOUBLE, nrhs_max=nrhs)
    log(f"[setup] batched builds {time.time() - t0:.1f}s")
    t0 = time.time()
    tune = {"fixed_ms": {}, "tuned_ms": {}, "choice": {}}
    for name, H in (("M1-Double", H64), (args.variant, Hm)):
        info = tuning.autotune(H, reps=5)
        tune["fixed_ms"][name] = _r4(info.get("ms_fixed"))
        tune["tuned_ms"][name] = _r4(info.get("ms_tuned"))
        tune["choice"][name] = {k: info[k] for k in ("stage1_batch", "stage1_grid", "stage2_batch", "stage2_grid")}
    log(f"[setup] autotune {time.time() - t0:.1f}s: {tune}")
    stm, st64 = Hm.stats(), H64.stats()
    Bm, Bm2 = mr_product_bytes(stm, nrhs, variant)
    B64, _ = mr_product_bytes(st64, nrhs, hmat.M1_DOUBLE)
    # per-system bytes of a 16-column product (the products skip the systems
    # whose recurrences have all stopped, so work is counted per system)
    def system_bytes(precision, c):
        xs = 4 if precision in (hmat.M1_SINGLE, hmat.M2_SINGLE) else 8
        out = []
        for bs_ in bss:
            pl = hmat.hmat_plan(bs_, precision, c, nrhs)
            zd = pl.algorithmic_bytes - pl.matrix_bytes - xs * bs_.n - 8 * bs_.n
            out.append(pl.matrix_bytes + zd + nrhs * 16 * bs_.n)
        return np.array(out, dtype=np.float64)

    Bsys, Bsys64 = system_bytes(variant, -1), system_bytes(hmat.M1_DOUBLE, 0)
    for nm, tot, ref in (("mixed", Bsys.sum(), Bm), ("fp64", Bsys64.sum(), B64)):
        if abs(tot - ref) > 1e-9 * ref:
            log(f"[warn] {nm}: per-system bytes {tot:.0f} != handle bytes {ref:.0f}")
    rng = np.random.default_rng(1)
    b = torch.as_tensor(rng.standard_normal((nrhs, n))).to(dev).T  # (n, nrhs), column-major
    work = torch.empty(hmat.hmat_bicgstab_batched_workspace_bytes(Hm, nrhs), dtype=torch.uint8, device=dev)
    maxiter = 3000

    def solve(H, x, refine=None):
        x.zero_()
        return hmat.hmat_bicgstab_batched(H, b, x=x, h_fp64=H64, tol=args.tol, maxiter=maxiter,
                                          poll_every=args.poll_every, use_graph=True, work=work,
                                          refine=args.refine if refine is None else refine)

    xm = torch.zeros((nrhs, n), dtype=torch.float64, device=dev).T
    x64 = torch.zeros_like(xm)
    for _ in range(args.warmup):
        solve(Hm, xm)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(solve(Hm, xm))
        log(f"[step] mixed solve: {runs[-1][1]}")
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t_start
    for _, summ, per in runs:
        assert summ["status"] == 0, summ
    # executed work: each system's products (results[].products) and the
    # FP64 true-residual products over all systems
    mv_bytes = sum(float(Bsys @ p["products"][:, 0]) + s["matvecs_fp64"] * B64 for _, s, p in runs)
    value = mv_bytes / t_mixed / 1e9
    per = runs[-1][2]
    # FP64 solves with each threshold of FP64_REFINES and the mixed solve's
    # own: the fastest is the baseline
    fp64_runs = {}
    for refine in sorted(set(FP64_REFINES) | {args.refine}):
        solve(H64, x64, refine)  # warm-up at this threshold
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        runs64 = []
        for _ in range(args.steps):
            runs64.append(solve(H64, x64, refine))
            log(f"[step] FP64 solve (early checks {refine:g}): {runs64[-1][1]}")
        torch.cuda.synchronize()
        fp64_runs[refine] = (time.perf_counter() - t_start, runs64, x64.clone())
    refine64 = min(fp64_runs, key=lambda r_: fp64_runs[r_][0])
    t_fp64, runs64, x64 = fp64_runs[refine64]
    per64 = runs64[-1][2]
    err = float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))

    # back-to-back products with live kernel timing (HIP events on the stream)
    matvec = {}
    xv = torch.randn((nrhs, n), dtype=torch.float64, device=dev).T
    yv = torch.empty_like(xv)
    kt = {}
    for name, H, BB in (("M1-Double", H64, B64), (args.variant, Hm, Bm)):
        for _ in range(2):
            H.matvec(xv, yv)
        H.set_profiling(True)
        H.kernel_times()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(5, args.matvec_reps // 10)
        e0.record(stream)
        for _ in range(reps):
            H.matvec(xv, yv, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        kt[name], _ = H.kernel_times()
        H.set_profiling(False)
        ms_ = e0.elapsed_time(e1) / reps
        matvec[name] = dict(ms=round(ms_, 4), gbs=round(BB / ms_ / 1e6, 1))
    k = kt[args.variant]
    k2_gbs = Bm2 / (k[2] / 1e3) / 1e9 if k[2] > 0 else 0.0
    its = per["iterations"]
    out = {
        "metric": "H-matvec GB/s and BiCG-STAB time-to-1e-8 residual, mixed vs FP64, 1 GPU",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_mixed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {W['desc']}",
            "precision": args.variant,
            "storage": storage_label(variant) + "; widened exactly on the fp64 matrix cores",
            "n": n, "systems": nsys, "rhs_per_system": nrhs,
            "step": f"batched BiCGSTAB of all {nsys * nrhs} (mesh, rhs) pairs, x0=0 -> |r|/|b|<{args.tol:g} each, "
                    "confirmed by the FP64 true residual; iteration replayed from a HIP graph",
            "refine": args.refine,
            "parallelism": "1 GPU",
        },
        "time_all_solves_ms": {"mixed": round(1e3 * t_mixed / args.steps, 3),
                               "fp64": round(1e3 * t_fp64 / args.steps, 3),
                               "fp64_by_refine": {f"{r_:g}": round(1e3 * v_[0] / args.steps, 3)
                                                  for r_, v_ in sorted(fp64_runs.items())}},
        "speedup_vs_fp64": round(t_fp64 / t_mixed, 3),
        "iterations": {"mixed_max": int(its.max()), "mixed_median": float(np.median(its)),
                       "fp64_max": int(per64["iterations"].max()),
                       "fp64_median": float(np.median(per64["iterations"])),
                       "mixed_max_restarts": int(per["restarts"].max()),
                       "mixed_median_restarts": float(np.median(per["restarts"])), "fp64_refine": refine64},
        "products": {"mixed_launched": runs[-1][1]["matvecs"], "fp64_checks": runs[-1][1]["matvecs_fp64"],
                     "mixed_work_fraction": round(float(Bsys @ per["products"][:, 0]) / (runs[-1][1]["matvecs"] * Bm), 4),
                     "fp64_work_fraction": round(float(Bsys64 @ per64["products"][:, 0]) / (runs64[-1][1]["matvecs"] * B64), 4)},
        "solution_rel_err_mixed_vs_fp64": err,
        "max_true_rel_res": {"mixed": float(per["true_rel_res"].max()), "fp64": float(per64["true_rel_res"].max())},
        "bytes_per_product": {"mixed": int(Bm), "fp64": int(B64)},
        "matvec_only": matvec,
        "autotune": tune,
        "kernel_ms": {"stage1": round(k[0], 4), "stage1_reduce": round(k[1], 4), "stage2": round(k[2], 4)},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_mr_stage2",
            "achieved": round(k2_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(k2_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(ms, W, variant, nrhs)
    print(json.dumps(out), flush=True)


def bench_learned(args, W, variant, dev, stream):
    """Preconditioned solves: the learned leaf map is trained on the GPU by
    the library's own kernels (setup, timed separately), then one step = one
    mixed BiCGSTAB solve to 1e-8 (FP64 true residual) with each of no
    preconditioner, block-Jacobi and the learned map."""
    import torch

    from paper_1911_00093_amd import hmat, learned, meshes

    t0 = time.time()
    data = learned.training_set(target=args.train_leaves, seed=1, log=log)
    t_set = time.time() - t0
    log(f"[setup] training set: {data['m'].size} leaves from {data['meshes']} meshes, {t_set:.1f}s")
    dd = learned.to_device(data)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net, hist = learned.train(dd, epochs=args.epochs, batch=256, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[train] {args.epochs} epochs in {t_train:.2f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")

    t0 = time.time()
    mesh = meshes.workload(args.workload)
    bs = assemble(args, mesh, W)
    log(f"[setup] {args.workload}: n={bs.n} blocks={bs.nblocks} assembly {time.time() - t0:.1f}s; "
        f"{assembly_note(bs)}")
    H64 = hmat.HMatrix(bs, hmat.M1_DOUBLE)
    Hm = hmat.HMatrix(bs, variant, c=-1)
    Bm, B64 = Hm.stats().algorithmic_bytes, H64.stats().algorithmic_bytes
    b = torch.as_tensor(mesh.rhs()[bs.perm], device=dev)
    n = bs.n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uv = learned.factors(net, mesh, bs)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    eval_loss = learned.mean_loss(net, learned.to_device(learned.leaf_inputs(mesh, bs, with_inverse=True)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    jac = hmat.Precond(bs, hmat.PRECOND_JACOBI)  # leaf inverses on the GPU (hmat_batched_inverse)
    t_jac = time.perf_counter() - t0
    pre = {"none": None, "block-jacobi": jac, "learned": hmat.Precond(bs, hmat.PRECOND_LEARNED, uv=uv)}
    # the best map of the learned form in the training loss's own measure:
    # per leaf, U V^T = s_tau x (rank-16 truncated SVD of A^-1 - diag(A)^-1),
    # which bounds what any network of this output form can reach
    pre["form-optimum"] = hmat.Precond(bs, hmat.PRECOND_LEARNED, uv=form_optimum_factors(bs).to(dev))
    work = torch.empty(hmat.hmat_solver_workspace_bytes(n), dtype=torch.uint8, device=dev)
    xref, _ = hmat.hmat_bicgstab(H64, b, tol=1e-12, maxiter=4000, work=work)
    xref = xref.clone()
    res = {}
    for name, P in pre.items():
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            hmat.hmat_bicgstab(Hm, b, x=x.zero_(), h_fp64=H64, tol=args.tol, maxiter=4000, precond=P,
                               poll_every=args.poll_every, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            x, info = hmat.hmat_bicgstab(Hm, b, x=x.zero_(), h_fp64=H64, tol=args.tol, maxiter=4000, precond=P,
                                         poll_every=args.poll_every, work=work)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(i["status"] == 0 for i in infos), (name, infos)
        res[name] = dict(ms=round(1e3 * dt / args.steps, 3), iterations=infos[-1]["iterations"],
                         restarts=infos[-1]["restarts"],
                         gbs=round(sum(i["matvecs"] * Bm + i["matvecs_fp64"] * B64 for i in infos) / dt / 1e9, 1),
                         x_err_vs_fp64_1e12=float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref)))
        log(f"[solve] {name}: {res[name]}")
    L = res["learned"]
    out = {
        "metric": "H-matvec GB/s and BiCG-STAB time-to-1e-8 residual, mixed vs FP64, 1 GPU",
        "value": L["gbs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": L["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {W['desc']}",
            "precision": args.variant,
            "n": n,
            "step": "one mixed BiCGSTAB solve x0=0 -> |r|/|b|<1e-8 (FP64 true residual) with the learned "
                    "leaf-map preconditioner",
            "parallelism": "1 GPU",
        },
        "preconditioners": res,
        "training": {"leaves": int(data["m"].size), "meshes": int(data["meshes"]), "epochs": args.epochs,
                     "batch": 256, "lr": "cosine 2e-3 -> 2e-4", "set_build_s": round(t_set, 2), "train_s": round(t_train, 3),
                     "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1], "inference_s": round(t_infer, 4),
                     "loss_on_evaluation_leaves": eval_loss},
        "setup_s": {"block_jacobi": round(t_jac, 4), "learned_inference": round(t_infer, 4)},
        "speedup_learned_vs_none": round(res["none"]["ms"] / L["ms"], 3),
        "speedup_learned_vs_jacobi": round(res["block-jacobi"]["ms"] / L["ms"], 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_training(data)
    print(json.dumps(out), flush=True)


def form_optimum_factors(bs):
    """Float32 (leaves, 2048) factors U, V (row-major 64 x 16 each) of the
    map diag(A)^-1 + (1/s) U V^T closest to each leaf's exact inverse in the
    Frobenius norm: U V^T = s (rank-16 truncated SVD of A^-1 - diag(A)^-1)."""
    import torch

    from paper_1911_00093_amd import hmat

    blk, r0, rows = hmat.precond_leaves(bs, hmat.PRECOND_LEARNED)
    R = hmat.MLP_RANK
    out = np.zeros((blk.size, hmat.MLP_OUT), np.float32)
    for q in range(blk.size):
        m, off = int(rows[q]), int(bs.offset[blk[q]])
        A = bs.data[off:off + m * m].reshape(m, m, order="F")
        d = np.diag(A)
        E = np.linalg.inv(A) - np.diag(1.0 / d)
        u, sv, vt = np.linalg.svd(E)
        k = min(R, m)
        U = np.zeros((hmat.MLP_LEAF, R))
        V = np.zeros((hmat.MLP_LEAF, R))
        U[:m, :k] = u[:, :k] * sv[:k] * (d.sum() / m)
        V[:m, :k] = vt[:k].T
        out[q, :hmat.MLP_LEAF * R] = U.ravel()
        out[q, hmat.MLP_LEAF * R:] = V.ravel()
    return torch.as_tensor(out)


def cpu_baseline_training(data, steps=200, batch=256):
    """The oracle (FP64 numpy) taking `steps` Adam steps of the same batch
    size on the same training set."""
    import oracle.learned as OL
    from paper_1911_00093_amd import seeded

    from threadpoolctl import threadpool_limits

    p = seeded.init_params(0).astype(np.float64)
    m1, m2 = np.zeros_like(p), np.zeros_like(p)
    order = seeded.batch_order(data["m"].size, batch, steps * batch // data["m"].size + 1, seed=0)
    with threadpool_limits(limits=1):  # one core, like the other oracle baselines
        t0 = time.perf_counter()
        for t in range(1, steps + 1):
            idx = next(order)
            f = lambda a: np.asarray(a[idx], dtype=np.float64)
            _, g = OL.loss_and_grad(p, f(data["x"]), f(data["ainv"]), f(data["dinv"]), f(data["sinv"]),
                                    data["m"][idx])
            OL.adam_step(p, m1, m2, g, t)
        dt = time.perf_counter() - t0
    return {"value": round(steps * batch / dt, 1), "unit": "training samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} oracle Adam steps of batch {batch} (FP64 numpy) on the same training set",
            "host": host_cpu()}


def cpu_baseline_batched(ms, W, variant, nrhs, sample=4):
    """The oracle on a sample of the meshes: its own assembly (untimed), then
    one product per right-hand side (the oracle has no multi-column
    product), timed; bytes counted as for the device's 16-column product of
    the same meshes."""
    import oracle
    from paper_1911_00093_amd import hmat

    pick = ms[:sample]
    convs, B = [], 0
    for m in pick:
        h = oracle.HMatrix(m.centroids, m.areas, leaf=W["leaf"], eta=W["eta"], eps=W["eps"])
        convs.append(oracle.Converted(h, variant, -1))
        bs = hmat.BlockSet.from_arrays(h.n, h.row0, h.nrows, h.col0, h.ncols, h.kind, h.rank, h.offset, h.data)
        B += mr_product_bytes(_plan_stats(bs, variant), nrhs, variant)[0]
    rng = np.random.default_rng(0)
    X = [rng.standard_normal((nrhs, c.h.n)) for c in convs]
    t0 = time.perf_counter()
    for c, x in zip(convs, X):
        for k in range(nrhs):
            c.matvec(x[k])
    dt = time.perf_counter() - t0
    return {"value": round(B / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{nrhs} single-column oracle products on each of the first {sample} "
                      f"meshes (N = {sum(c.h.n for c in convs)}), {dt * 1e3:.0f} ms in total, after an untimed "
                      f"oracle assembly",
            "host": host_cpu()}


def _plan_stats(bs, precision):
    """Byte counts of a plan, in the fields mr_product_bytes reads."""
    from types import SimpleNamespace

    from paper_1911_00093_amd import hmat

    info = hmat.hmat_plan(bs, precision, c=-1)
    return SimpleNamespace(n=bs.n, bytes_dense=0, bytes_v=0, bytes_w=info.matrix_bytes,
                           algorithmic_bytes=info.algorithmic_bytes)


def cpu_baseline(mesh, W, variant, reps, B, drop, c, dense_split, b, gpu_info, solve_iters, tol):
    """The oracle as it stands (plain single-threaded C, FP64 arithmetic) on
    the same workload: its own assembly (untimed; it reproduces the library's
    blocks bit for bit, so the product moves the same B bytes), then `reps`
    products with the same precision variant, timed, and `solve_iters`
    iterations of its BiCGSTAB (Algorithm 1, FP64 true residual with its own
    FP64 conversion), timed; the whole solve is estimated from that as the
    time per iteration times the iterations the GPU solve took, plus one
    FP64 true-residual product per FP64 check the GPU solve made."""
    import oracle

    t0 = time.time()
    h = oracle.HMatrix(mesh.centroids, mesh.areas, leaf=W["leaf"], eta=W["eta"], eps=W["eps"])
    t1 = time.time()
    conv = oracle.Converted(h, variant, c, drop=drop, dense_split=dense_split)
    conv64 = conv if variant == oracle.M1_DOUBLE and not drop else oracle.Converted(h, oracle.M1_DOUBLE, 0)
    log(f"[cpu] oracle assembly {t1 - t0:.2f}s (1 thread), conversions {time.time() - t1:.2f}s")
    x = np.random.default_rng(0).standard_normal(h.n)
    conv.matvec(x)
    t0 = time.perf_counter()
    for _ in range(reps):
        conv.matvec(x)
    dt = (time.perf_counter() - t0) / reps
    t64 = time.perf_counter()
    conv64.matvec(x)
    dt64 = time.perf_counter() - t64
    # a few BiCGSTAB iterations (tol unreachable in that many): the initial
    # residual product, two products per iteration, and the FP64 true
    # residual the oracle takes when it stops without converging
    t0 = time.perf_counter()
    _, inf = oracle.bicgstab(conv, b, op64=conv64, tol=1e-300, maxiter=solve_iters)
    dts = time.perf_counter() - t0
    per_it = max(dts - dt - dt64, 0.0) / max(inf["iterations"], 1)
    est = dt + per_it * gpu_info["iterations"] + dt64 * gpu_info["matvecs_fp64"]
    from paper_1911_00093_amd import hmat

    return {"value": round(B / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} oracle products ({hmat.PRECISION_NAMES[variant]}, build arithmetic) on the full "
                      f"workload ({dt * 1e3:.0f} ms each) and {inf['iterations']} oracle BiCGSTAB iterations "
                      f"({dts:.1f} s), after an untimed oracle assembly",
            "ms_per_matvec": round(dt * 1e3, 1),
            "solve_ms_estimate": round(est * 1e3, 1),
            "solve_estimate": f"{per_it * 1e3:.0f} ms per oracle iteration x {gpu_info['iterations']} iterations "
                              f"+ initial residual + {gpu_info['matvecs_fp64']} FP64 true-residual products "
                              f"({dt64 * 1e3:.0f} ms each), at tol {tol:g}; not a measured oracle solve",
            "host": host_cpu()}


if __name__ == "__main__":
    main()
