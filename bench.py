#!/usr/bin/env python3
"""Benchmark of the VMAT column-generation hot path on one MI355X.

A step is one full plan (column generation until every beam has an aperture:
pricing, master solves with their dose products, adjoints and line searches)
on the prostate-shaped case: 180 beams at 2 deg, 40x40 beamlets at 5 mm
(288,000 beamlets), 128x128x64 voxels at 2.5 mm, about 1.09e8 non-zeros of D.
The timed step uses the master that streams D in every iteration (one forward
and one adjoint per master iteration), the configuration whose products the
metric counts; the plan time of the master over stored aperture doses is
reported beside it (`aperture_master`).

value = the bytes all D.x (forward) and D^T.r (adjoint) products run during
the timed plans move with the handle's layout (vmat_layout fwd_bytes and
adj_bytes: stored entries with their 16-bit local indices, row and slot
pointers, the gathered vector and the output) / wall time of those plans
(GB/s).  The roofline
object reports the dominant product kernel alone, timed with HIP events on the
stream it runs on, against the 8 TB/s HBM peak.  Its algorithmic bytes per
launch are those of a plain CSR product with int32 indices: nnz (v + 4) +
8 (rows + 1) + 4 (gathered vector) + 4 (output) (v = value bytes, +4 per
beamlet for FP8 scales); the fractions on the layout's own bytes (16-bit
local indices) and on the rocprofv3 HBM counters are reported beside it.  The
CPU baseline is the FP64 reference running the first column-generation
iterations of the same plan, with per-call reference times on the three cases
and an all-cores row-parallel product beside it.

Prints one JSON line.
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

PEAK_HBM_GBS = 8000.0

PEAK_FP64_TFLOPS = 78.6
VALUE_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}

# HBM bytes per launch from rocprofv3 FETCH_SIZE (x 2.0, calibrated on a
# 512 MiB copy) + WRITE_SIZE, for the product kernels as they stand
# (k_fwd_sell, k_adj_sell + k_adj_reduce).  Used only when the layout matches
# the one measured (same workload, storage and byte counts).
TRAFFIC_SOURCE = "profiles/fwd_adj_sell_prostate180_hbm_counters.md"
MEASURED_TRAFFIC = {
    ("prostate180", "f32", 676890628, 676191240): {
        "forward": (344731.94 * 2 + 8308.53) * 1024,
        "adjoint": (347202.12 * 2 + 3601.91 + 3750.31 * 2 + 2250.0) * 1024,
    },
}
METRIC = "D·x + Dᵀr HBM GB/s vs peak; plan s; bf16/fp8-D vs fp32 at stated dose error"


def time_kernel(fn, reps, torch, warm=1, warm_s=0.0):
    """Average ms of fn over reps launches, after warm launches and then
    more until warm_s seconds have passed."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps  # ms


def algorithmic_bytes(case, d_store, B=1):
    """Bytes one product has to move with a plain CSR layout (int32 indices,
    int64 row pointers, FP32 vectors): D once, the gathered vector read once
    and the output written once, each B times for B right-hand sides (FP64
    outputs of the batched products).  FP8 adds the per-beamlet scales."""
    v = VALUE_BYTES[d_store]
    nnz, nb, nv = case.nnz, case.n_beamlets, case.n_voxels
    sc = 4 * nb if d_store == "fp8" else 0
    out_b = 4 if B == 1 else 8
    fwd = nnz * (v + 4) + 8 * (nv + 1) + B * (4 * nb + out_b * nv) + sc
    adj = nnz * (v + 4) + 8 * (nb + 1) + B * (4 * nv + out_b * nb) + sc
    return fwd, adj


def host_info():
    """Host cores and CPU model (os.cpu_count, the affinity mask, lscpu)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return {"nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": model}


def median_time(fn, n=3):
    ts = []
    for _ in range(n):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_per_call(workloads, log, hn_iters=1):
    """The FP64 reference, one host core, per call on each case: forward and
    adjoint products, one pricing of the empty plan, the first
    column-generation iterations (pricing + master), and the full plan on the
    tiny case; plus the two products row-parallel on all host cores
    (oracle/rowpar.c).  Medians of 3 for the single calls."""
    import casegen
    import oracle as O
    from oracle import rowpar
    from threadpoolctl import threadpool_limits
    res = {}
    for wl in workloads:
        c = casegen.make_case(casegen.preset(wl))
        D = O.dose_matrix(c.row_ptr, c.col, c.val, c.n_voxels)
        Dt = D.T.tocsr()
        rng = np.random.default_rng(0)
        x = rng.random(c.n_beamlets)
        w = rng.standard_normal(c.n_voxels)
        N, R, C = c.n_beams, c.n_rows, c.n_cols
        l0 = np.zeros(N * R, np.int32)
        occ0 = np.zeros(N, np.uint8)
        r_ = {"nnz": c.nnz}
        with threadpool_limits(limits=1):
            r_["forward_s"] = round(median_time(lambda: O.dose(D, x)), 4)
            r_["adjoint_s"] = round(median_time(lambda: D @ w), 4)
            g = D @ w
            r_["pricing_s"] = round(median_time(lambda: O.price(g, np.zeros(N), l0, l0, occ0, c.theta_deg, c.gamma,
                                                                  R, C, c.max_leaf_step, c.circular)), 4)
            iters = N if wl == "tiny36" else (hn_iters if wl == "headneck180" else 1)
            t0 = time.perf_counter()
            sol = O.solve(D, c.alpha, c.beta, c.T, c.theta_deg, c.gamma, c.circular, R, C, c.max_leaf_step,
                          max_cg_iter=iters, with_margins=False)
            key = "full_plan_s" if iters == N else f"first_{iters}_cg_iterations_s"
            r_[key] = round(time.perf_counter() - t0, 3)
            r_["master_iters"] = int(sum(sol.master_iters))
        r_["rowpar_forward_s"] = round(median_time(lambda: rowpar.spmv(Dt, x)), 4)
        r_["rowpar_adjoint_s"] = round(median_time(lambda: rowpar.spmv(D, w)), 4)
        r_["rowpar_threads"] = rowpar.threads()
        res[wl] = r_
        log(f"[bench] cpu reference {wl}: {r_}")
        del D, Dt, c
    return res


def cpu_baseline(case, n_iter, log=None):
    """The FP64 reference, unmodified, on the first column-generation iterations
    of the same plan.  Returns (bytes-weighted product counts, seconds, result)."""
    import oracle as O
    from threadpoolctl import threadpool_limits
    D = O.dose_matrix(case.row_ptr, case.col, case.val, case.n_voxels)
    # one host core: scipy's sparse products are single-threaded, and numpy's
    # BLAS pool is held to one thread
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        res = O.solve(D, case.alpha, case.beta, case.T, case.theta_deg, case.gamma, case.circular,
                      case.n_rows, case.n_cols, case.max_leaf_step, max_cg_iter=n_iter, with_margins=False,
                      on_iter=(lambda t, k, c: log(f"[bench] reference iteration {t}: beam {k}, cost {c:.6g}"))
                      if log and n_iter is None else None)
        dt = time.perf_counter() - t0
    n_it = len(res.order)
    # one adjoint for the empty plan, then one forward + one adjoint per master iteration
    nf = sum(res.master_iters)
    na = 1 + sum(res.master_iters)
    return nf, na, n_it, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="prostate180")
    ap.add_argument("--d-store", default="f32", choices=["f32", "bf16", "f16", "fp8"])
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cpu-iters", type=int, default=16)
    ap.add_argument("--cpu-hn-iters", type=int, default=1,
                    help="column-generation iterations of the reference on the head-and-neck case")
    ap.add_argument("--no-cpu-per-call", action="store_true")
    ap.add_argument("--cpu-full-plan", action="store_true",
                    help="also run the reference's whole plan on the timed case (minutes on one core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--precision-workload", default="headneck180")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--variants", type=int, default=64)
    ap.add_argument("--no-batched-solve", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the variant plans run K at a time on K handles")
    ap.add_argument("--no-aperture-master", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autograd", action="store_true")
    ap.add_argument("--products-only", action="store_true",
                    help="no plans and no side studies: only the per-kernel product timing (for profiling)")
    ap.add_argument("--sequential-variants", type=int, default=4,
                    help="variants solved one at a time (master streaming D) for the batched-solve comparison")
    ap.add_argument("--sequential-apdose-variants", type=int, default=8,
                    help="variants solved one at a time with the aperture-dose master")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the tuned batched products at --variants right-hand sides (for profiling)")
    ap.add_argument("--apmaster-only", action="store_true",
                    help="only plans with the aperture-dose master (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured at one GPU's share; "
              "the multi-GPU sharding is a design (voxel-slab split) without a runnable path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import casegen
    import paper_1005_4396_amd as P

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    case = casegen.make_case(casegen.preset(args.workload))
    log(f"[bench] case {args.workload}: nb={case.n_beamlets} nv={case.n_voxels} nnz={case.nnz} "
        f"gen {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    prob = P.Problem.from_case(case, d_store=args.d_store)
    log(f"[bench] handle built in {time.perf_counter() - t0:.1f}s, device bytes {prob.device_bytes() / 1e9:.2f} GB")

    def one_plan():
        l, r, occ, y = prob.empty_plan()
        rep, tr = prob.solve(l, r, occ, y, want_trace=True)
        return rep, tr

    if args.batched_only:
        res = batched_study(case, prob, torch, args.variants, max(3, args.kernel_reps // 10), log, args.d_store)
        log(f"[bench] batched only: {res}")
        prob.close()
        return
    if args.apmaster_only:
        o = P.vmat.SolveOpts()
        o.max_cg_iter = 0
        o.master_mode = 1
        o.master = P.master_opts()
        for i in range(max(1, args.steps)):
            l, r, occ, y = prob.empty_plan()
            t0 = time.perf_counter()
            rep, _ = prob.solve(l, r, occ, y, o, want_trace=False)
            torch.cuda.synchronize()
            log(f"[bench] aperture-dose plan {i}: {time.perf_counter() - t0:.3f} s, cost {rep.F + rep.gG:.9g}")
        prob.close()
        return
    if args.products_only:
        args.steps = args.warmup = 0
        args.no_precision = args.no_batched = args.no_batched_solve = args.no_cpu_baseline = True
        args.no_concurrent = True
    for w in range(args.warmup):
        rep, tr = one_plan()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: cg={rep.cg_iters} master_iters={rep.master_iters} fwd={rep.n_forward} "
            f"adj={rep.n_adjoint} cost={rep.F + rep.gG:.6g}")

    torch.cuda.synchronize()
    reps = []
    t_start = time.perf_counter()
    for s in range(args.steps):
        rep, tr = one_plan()
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps if args.steps else None

    # the layout's bytes of the products run during the timed plans
    lay = prob.layout()
    fwd_b, adj_b = lay["fwd_bytes"], lay["adj_bytes"]
    n_fwd = sum(r.n_forward for r in reps)
    n_adj = sum(r.n_adjoint for r in reps)
    total_bytes = n_fwd * fwd_b + n_adj * adj_b
    value = total_bytes / wall / 1e9 if args.steps else None
    if args.steps:
        log(f"[bench] {args.steps} plans in {wall:.2f}s: {ms_per_step:.1f} ms/plan, fwd={n_fwd} adj={n_adj}")

    # per-kernel timing of the two products (HIP events on torch's current stream)
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.random(case.n_beamlets)).cuda()
    w = torch.from_numpy(rng.standard_normal(case.n_voxels).astype(np.float32)).cuda()
    zbuf = torch.empty(case.n_voxels, dtype=torch.float64, device="cuda")
    gbuf = torch.empty(case.n_beamlets, dtype=torch.float64, device="cuda")
    # 0.2 s of launches first: right after a handle's creation the device
    # runs the products about 3% slower for a while
    fwd_ms = time_kernel(lambda: prob.forward(x, zbuf), args.kernel_reps, torch, warm_s=0.2)
    adj_ms = time_kernel(lambda: prob.adjoint(w, gbuf), args.kernel_reps, torch, warm_s=0.2)
    fwd_gbs = fwd_b / fwd_ms / 1e6
    adj_gbs = adj_b / adj_ms / 1e6
    fwd_alg, adj_alg = algorithmic_bytes(case, args.d_store)
    dom = "forward" if fwd_ms * n_fwd >= adj_ms * n_adj else "adjoint"
    dom_ms = fwd_ms if dom == "forward" else adj_ms
    dom_alg, dom_lay = (fwd_alg, fwd_b) if dom == "forward" else (adj_alg, adj_b)
    dom_gbs = dom_alg / dom_ms / 1e6
    log(f"[bench] forward {fwd_ms:.4f} ms ({fwd_alg / fwd_ms / 1e6:.0f} GB/s algorithmic, {fwd_gbs:.0f} layout), "
        f"adjoint {adj_ms:.4f} ms ({adj_alg / adj_ms / 1e6:.0f} GB/s algorithmic, {adj_gbs:.0f} layout)")

    meas = MEASURED_TRAFFIC.get((args.workload, args.d_store, fwd_b, adj_b))
    traffic = round(meas[dom]) if meas else None

    # device copy ceiling (context)
    big = torch.empty(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    big2 = torch.empty_like(big)
    cp_ms = time_kernel(lambda: big2.copy_(big), 20, torch)
    copy_gbs = 2 * big.numel() * 4 / cp_ms / 1e6
    # streaming-read ceiling (context): 1 GiB read by the library's read
    # kernel, the best over a few grid sizes (the rate depends on the grid:
    # one workgroup per compute unit reads fastest on MI355X)
    del big2
    big = torch.empty(1024 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    big.zero_()
    rs_part = torch.empty(65536, dtype=torch.float32, device="cuda")
    read_by_grid = {}
    for grid in (256, 512, 1024, 8192, 65536):
        rd_ms = time_kernel(lambda: P.vmat.read_stream(big, rs_part, grid), 20, torch)
        read_by_grid[grid] = big.numel() * 4 / rd_ms / 1e6
    read_grid = max(read_by_grid, key=read_by_grid.get)
    read_gbs = read_by_grid[read_grid]
    # the same read with each product's share of writes mixed in (the
    # products write their outputs while they stream D): bytes read and
    # written over the time, as the layout byte counts are
    nv, nb = case.n_voxels, case.n_beamlets
    write_share = {"forward": 8 * nv / fwd_b, "adjoint": (8 * lay["slots"] + 8 * nb) / adj_b} if lay["tiled"] \
        else {"forward": 8 * nv / fwd_b, "adjoint": 8 * nb / adj_b}
    rw_gbs = {}
    for prod, f in write_share.items():
        wb = int(round(big.numel() * 4 * f / (1 - f) / 512)) * 512
        wbuf = torch.empty(wb // 8, dtype=torch.float64, device="cuda")
        rw_ms = time_kernel(lambda: P.vmat.read_write_stream(big, wbuf, rs_part, read_grid), 20, torch)
        rw_gbs[prod] = (big.numel() * 4 + wb) / rw_ms / 1e6
        del wbuf
    del big, rs_part
    log(f"[bench] device copy {copy_gbs:.0f} GB/s, streaming read {read_gbs:.0f} GB/s (grid {read_grid}; "
        + ", ".join(f"{g}: {v:.0f}" for g, v in read_by_grid.items()) + "); with the products' write shares "
        + ", ".join(f"{k} {100 * write_share[k]:.2f}%: {v:.0f} GB/s" for k, v in rw_gbs.items()))

    out = {
        "metric": METRIC,
        "value": round(value, 2) if value is not None else None,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3) if ms_per_step else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_beams": case.n_beams, "beamlets": case.n_beamlets,
                   "voxels": case.n_voxels, "nnz": case.nnz, "d_store": args.d_store,
                   "layout": "tiled" if lay["tiled"] else "plain",
                   "step": "one full column-generation plan"},
        "plan_s": round(ms_per_step / 1e3, 4) if ms_per_step else None,
        # the paper's own plan times (clinical cases of 1.8e7-5.5e7 non-zeros,
        # other hardware): context only, not the same workload
        "context": {"paper_plan_s_matlab_xeon_2_27ghz": [265, 512], "paper_plan_s_cuda_tesla_c1060": [18, 31]},
        "plan": {"cg_iters": reps[-1].cg_iters, "master_iters": reps[-1].master_iters,
                 "n_forward": reps[-1].n_forward, "n_adjoint": reps[-1].n_adjoint,
                 "n_ls_evals": reps[-1].n_ls_evals, "cost": reps[-1].F + reps[-1].gG} if reps else None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "frac_basis": "algorithmic bytes of a plain CSR product: nnz*(v+4) + 8*(rows+1) + "
                                   "4*(gathered vector) + 4*(output)",
                     "bytes_per_launch": dom_alg, "duration_ms": round(dom_ms, 5),
                     "layout_bytes_per_launch": dom_lay,
                     "frac_layout_bytes": round(dom_lay / dom_ms / 1e6 / PEAK_HBM_GBS, 4),
                     "frac_counter_bytes": round(traffic / dom_ms / 1e6 / PEAK_HBM_GBS, 4) if traffic else None,
                     "traffic_source": TRAFFIC_SOURCE if traffic else None},
        "products": {"forward_ms": round(fwd_ms, 5), "forward_GBs": round(fwd_gbs, 1), "forward_bytes": fwd_b,
                     "forward_alg_bytes": fwd_alg, "forward_alg_GBs": round(fwd_alg / fwd_ms / 1e6, 1),
                     "adjoint_alg_bytes": adj_alg, "adjoint_alg_GBs": round(adj_alg / adj_ms / 1e6, 1),
                     "adjoint_ms": round(adj_ms, 5), "adjoint_GBs": round(adj_gbs, 1), "adjoint_bytes": adj_b,
                     "nnz_per_s_fwd": round(case.nnz / fwd_ms / 1e6, 1), "nnz_per_s_adj": round(case.nnz / adj_ms / 1e6, 1),
                     "csr_fp32_equiv_GBs_fwd": round(8 * case.nnz / fwd_ms / 1e6, 1),
                     "device_copy_GBs": round(copy_gbs, 1), "read_stream_GBs": round(read_gbs, 1),
                     "read_stream_grid": read_grid,
                     "fwd_frac_of_read_stream": round(fwd_gbs / read_gbs, 3),
                     "adj_frac_of_read_stream": round(adj_gbs / read_gbs, 3),
                     "write_share": {k: round(v, 5) for k, v in write_share.items()},
                     "read_write_stream_GBs": {k: round(v, 1) for k, v in rw_gbs.items()},
                     "fwd_frac_of_read_write_stream": round(fwd_gbs / rw_gbs["forward"], 3),
                     "adj_frac_of_read_write_stream": round(adj_gbs / rw_gbs["adjoint"], 3), "layout": lay},
    }

    if not args.no_precision and args.d_store == "f32":
        out["precision"] = precision_study(args.precision_workload, torch, P, args.kernel_reps, log)

    if not args.no_aperture_master and args.steps:
        out["aperture_master"] = aperture_master_study(prob, P, torch, args.steps, ms_per_step, reps[-1], log)

    if not args.no_mixed and args.steps:
        out["mixed_resolution"] = mixed_resolution_study(case, prob, P, torch, log)

    if not args.no_autograd and args.steps:
        out["autograd"] = autograd_study(case, prob, P, torch, args.kernel_reps, log)

    if not args.no_batched:
        out["batched"] = batched_study(case, prob, torch, args.variants, max(3, args.kernel_reps // 10), log,
                                       args.d_store)
    if not args.no_batched_solve:
        out["batched_solve"] = batched_solve_study(case, prob, torch, P, args.variants, args.sequential_variants,
                                                   args.sequential_apdose_variants, log)

    if not args.no_concurrent:
        out["concurrent_variants"] = concurrent_study(case, torch, P, args.variants, (4, 8), log)

    if not args.no_cpu_baseline:
        nf, na, n_it, dt = cpu_baseline(case, args.cpu_iters)
        cpu_bytes = nf * fwd_b + na * adj_b
        out["cpu_baseline"] = {"value": round(cpu_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {n_it} column-generation iterations of the same plan "
                                         f"({nf} forward + {na} adjoint products, {dt:.1f} s)",
                               "host": host_info()}
        if reps:
            # the reference makes the same iterations as the GPU plan: scale
            # its time by master iterations (labelled as an extrapolation)
            gpu_mi = [int(v) for v in tr["master_iters"]]
            part = sum(gpu_mi[:n_it])
            if part > 0:
                out["cpu_baseline"]["full_plan_s_extrapolated"] = round(dt * sum(gpu_mi) / part, 1)
        if args.cpu_full_plan:
            nf2, na2, n_it2, dt2 = cpu_baseline(case, None, log)
            out["cpu_baseline"]["full_plan_s"] = round(dt2, 1)
            out["cpu_baseline"]["full_plan_value"] = round((nf2 * fwd_b + na2 * adj_b) / dt2 / 1e9, 4)
            log(f"[bench] reference full plan: {n_it2} iterations, {dt2:.1f} s")
        if not args.no_cpu_per_call:
            out["cpu_baseline"]["per_call"] = cpu_per_call(("tiny36", args.workload, args.precision_workload), log,
                                                           args.cpu_hn_iters)
        log(f"[bench] cpu baseline {out['cpu_baseline']}")

    prob.close()
    print(json.dumps(out), flush=True)


def batched_study(case, prob, torch, B, reps, log, d_store="f32"):
    """B objective variants (alpha, beta ~ U[0.5, 2] x base per structure,
    target T ~ U[0.95, 1.05] x base) sharing D: the tuned forward and adjoint
    SpMM timed alone against their HBM and FP64-VALU rooflines, and one
    batched cost + gradient (forward SpMM, eq. 1 per variant, adjoint SpMM)
    against B sequential single-variant evaluations (forward SpMV, eq. 1,
    adjoint SpMV)."""
    import casegen
    tab = casegen.variant_table(case, B, seed=1)
    rng = np.random.default_rng(5)
    X = rng.random((case.n_beamlets, B)).astype(np.float32)
    prob.reserve_batched(B)            # the tiled adjoint's slot sums
    t0 = time.perf_counter()
    fw, aw, times = prob.tune_batched(B, reps=3)
    log(f"[bench] tuned B={B}: forward {fw}, adjoint {aw} ({time.perf_counter() - t0:.1f}s) {times}")
    lab = torch.as_tensor(case.label, device="cuda")
    tabt = torch.as_tensor(tab, device="cuda")
    Xt = torch.as_tensor(X, device="cuda")
    Wt = torch.as_tensor(rng.standard_normal((case.n_voxels, B)).astype(np.float32), device="cuda")
    Zb = torch.empty(case.n_voxels, B, dtype=torch.float64, device="cuda")
    Gb = torch.empty(case.n_beamlets, B, dtype=torch.float64, device="cuda")
    f_ms = time_kernel(lambda: prob.forward_batched(Xt, Zb), reps, torch)
    a_ms = time_kernel(lambda: prob.adjoint_batched(Wt, Gb), reps, torch)
    fb, ab = algorithmic_bytes(case, d_store, B)
    flops = 2.0 * case.nnz * B
    b_ms = time_kernel(lambda: prob.grad_batched(lab, tabt, Xt), reps, torch)
    # sequential: the same work one variant at a time through the single-RHS path
    xs = [Xt[:, b].double().contiguous() for b in range(B)]
    Pb = [None] * B

    def seq():
        for b in range(B):
            Pb[b] = prob.grad_fluence(xs[b], want=("dF", "g"))
    s_ms = time_kernel(seq, max(1, reps // 3), torch)
    lay = prob.layout()
    seq_bytes = B * (lay["fwd_bytes"] + lay["adj_bytes"])

    def roof(ms, nbytes):
        return {"ms": round(ms, 4), "alg_bytes": nbytes, "GBs": round(nbytes / ms / 1e6, 1),
                "hbm_frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4),
                "fp64_TFLOPs": round(flops / ms / 1e9, 2),
                "valu_fp64_frac": round(flops / ms / 1e9 / PEAK_FP64_TFLOPS, 4)}
    res = {"variants": B, "forward_variant": list(fw), "adjoint_variant": list(aw),
           "forward": roof(f_ms, fb), "adjoint": roof(a_ms, ab),
           "tune_ms": {k: {f"{v[0]}x{v[1]}": (round(t, 4) if t != float("inf") else None) for v, t in d.items()}
                       for k, d in times.items()},
           "batched_ms": round(b_ms, 3), "sequential_ms": round(s_ms, 3), "speedup": round(s_ms / b_ms, 2),
           "spmv_equiv_GBs": round(seq_bytes / b_ms / 1e6, 1)}
    log(f"[bench] batched {B} variants: forward {f_ms:.3f} ms, adjoint {a_ms:.3f} ms; cost + gradient "
        f"{b_ms:.2f} ms vs sequential {s_ms:.2f} ms ({s_ms / b_ms:.1f}x)")
    return res


def aperture_master_study(prob, P, torch, steps, ms_stream, rep_stream, log):
    """The same plans with the master over stored aperture doses (master_mode
    1): D is streamed once per opened aperture (forward) and once per pricing
    (adjoint); the master iterations work on the aperture doses."""
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = 1
    o.master = P.master_opts()
    l, r, occ, y = prob.empty_plan()
    prob.solve(l, r, occ, y, o, want_trace=False)  # warm-up (reserves the aperture-dose store)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        l, r, occ, y = prob.empty_plan()
        rep, _ = prob.solve(l, r, occ, y, o, want_trace=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    log(f"[bench] aperture-dose master: {ms:.1f} ms/plan (streaming master {ms_stream:.1f}), "
        f"cost {rep.F + rep.gG:.9g} vs {rep_stream.F + rep_stream.gG:.9g}")
    return {"plan_s": round(ms / 1e3, 4), "streaming_master_plan_s": round(ms_stream / 1e3, 4),
            "speedup": round(ms_stream / ms, 2), "cost": rep.F + rep.gG,
            "cost_rel_diff_vs_streaming": abs(rep.F + rep.gG - (rep_stream.F + rep_stream.gG)) /
            (rep_stream.F + rep_stream.gG),
            "master_iters": rep.master_iters, "d_products": [rep.n_forward, rep.n_adjoint]}


def autograd_study(case, prob, P, torch, reps, log):
    """Differentiable dose + cost: one forward + backward of the fluence form
    (d cost / d x, 288,000 beamlets) and of the aperture form (d cost / d y,
    180 apertures, every aperture fully open), FP32 D."""
    rng = np.random.default_rng(9)
    N, R, C = case.n_beams, case.n_rows, case.n_cols
    x = torch.tensor(rng.random(case.n_beamlets) + 0.5, dtype=torch.float64, device="cuda", requires_grad=True)
    y = torch.tensor(rng.random(N) + 0.5, dtype=torch.float64, device="cuda", requires_grad=True)
    l = torch.zeros(N * R, dtype=torch.int32, device="cuda")
    r = torch.full((N * R,), C, dtype=torch.int32, device="cuda")
    occ = torch.ones(N, dtype=torch.uint8, device="cuda")

    def fx():
        x.grad = None
        P.fluence_cost(prob, x).backward()

    def fy():
        y.grad = None
        P.aperture_cost(prob, y, l, r, occ).backward()
    n = max(5, reps // 5)
    tx = time_kernel(fx, n, torch)
    ty = time_kernel(fy, n, torch)
    log(f"[bench] autograd: fluence form {tx:.3f} ms, aperture form {ty:.3f} ms (forward + backward)")
    return {"fluence_fwd_bwd_ms": round(tx, 4), "aperture_fwd_bwd_ms": round(ty, 4)}


def mixed_resolution_study(case, prob_full, P, torch, log):
    """Unspecified tissue at twice the voxel size (Sec. 3): plan on the mixed
    problem (aperture-dose master), then one full-resolution dose and cost of
    that plan, against the plan optimised at full resolution."""
    import casegen
    t0 = time.perf_counter()
    m, _ = casegen.mixed_resolution(case)
    t_build = time.perf_counter() - t0
    pm = P.Problem.from_case(m)
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = 1
    o.master = P.master_opts()
    l, r, occ, y = pm.empty_plan()
    pm.solve(l, r, occ, y, o, want_trace=False)       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l, r, occ, y = pm.empty_plan()
    rep, _ = pm.solve(l, r, occ, y, o, want_trace=False)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    cm = prob_full.grad(y, l, r, occ, want=())["cost"].cpu().numpy()
    t_eval = time.perf_counter() - t0
    pm.close()
    l2, r2, occ2, y2 = prob_full.empty_plan()
    rep_f, _ = prob_full.solve(l2, r2, occ2, y2, o, want_trace=False)
    full = rep_f.F + rep_f.gG
    log(f"[bench] mixed resolution: nv {case.n_voxels} -> {m.n_voxels}, nnz {case.nnz} -> {m.nnz}, plan "
        f"{t_plan * 1e3:.1f} ms, full-resolution cost {cm[0] + cm[1]:.6g} vs full plan {full:.6g}")
    return {"voxels": m.n_voxels, "nnz": m.nnz, "plan_s": round(t_plan, 4), "full_eval_s": round(t_eval, 4),
            "build_s": round(t_build, 2), "full_res_cost": float(cm[0] + cm[1]), "full_plan_cost": full,
            "cost_ratio": float((cm[0] + cm[1]) / full)}


def batched_solve_study(case, prob, torch, P, B, n_seq, n_seq_ap, log):
    """B plan variants solved by one lockstep column-generation run (every
    product an SpMM over the variants) against some of them solved one after
    another by the single-plan solver, with the master streaming D (n_seq
    variants) and with the aperture-dose master (n_seq_ap variants), each
    scaled to B."""
    import dataclasses

    import casegen
    tab = casegen.variant_table(case, B, seed=1)
    lab = torch.as_tensor(case.label, device="cuda")
    tabt = torch.as_tensor(tab, device="cuda")
    prob.reserve_batched(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans, reps, _, cnt = prob.solve_batched(lab, tabt, want_trace=False)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    log(f"[bench] batched solve of {B} variants: {t_b:.2f}s, {cnt[0]} forward + {cnt[1]} adjoint SpMM")

    def sequential(n, mode):
        o = P.vmat.SolveOpts()
        o.max_cg_iter = 0
        o.master_mode = mode
        o.master = P.master_opts()
        t = 0.0
        for b in range(n):
            w = tab[b][np.minimum(case.label, tab.shape[1] - 1)]
            cb = dataclasses.replace(case, alpha=w[:, 0].copy(), beta=w[:, 1].copy(), T=w[:, 2].copy())
            pb = P.Problem.from_case(cb)
            if mode == 1:
                pb.reserve_solve()
            l, r, occ, y = pb.empty_plan()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb.solve(l, r, occ, y, o, want_trace=False)
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            pb.close()
        return t * B / max(n, 1)
    n_seq, n_seq_ap = min(n_seq, B), min(n_seq_ap, B)
    t_seq_B = sequential(n_seq, 0)
    t_ap_B = sequential(n_seq_ap, 1)
    log(f"[bench] sequential single-variant plans scaled to {B}: streaming master {t_seq_B:.2f}s "
        f"({n_seq} measured), aperture-dose master {t_ap_B:.2f}s ({n_seq_ap} measured)")
    return {"variants": B, "batched_s": round(t_b, 3), "sequential_s": round(t_seq_B, 3),
            "sequential_measured": n_seq, "speedup": round(t_seq_B / t_b, 2),
            "sequential_apdose_s": round(t_ap_B, 3), "sequential_apdose_measured": n_seq_ap,
            "speedup_vs_apdose": round(t_ap_B / t_b, 2),
            "plans_per_s": round(B / t_b, 2), "spmm_forward": int(cnt[0]), "spmm_adjoint": int(cnt[1]),
            "master_iters_mean": round(float(np.mean([r.master_iters for r in reps])), 1),
            "costs_first": [round(r.F + r.gG, 3) for r in reps[:4]]}


def concurrent_study(case, torch, P, B, ks, log):
    """The same B plan variants with the aperture-dose master, K at a time:
    vmat_solve_variants, which makes K plan contexts over one handle's D, one
    host thread and stream each (each context takes its next variant with
    vmat_set_weights).  A plan with that master is bound by launch latency,
    so plans on K streams overlap.  The time includes making the contexts and
    their aperture-dose stores."""
    import casegen
    tab = torch.as_tensor(casegen.variant_table(case, B, seed=1), device="cuda")
    label = torch.as_tensor(case.label, device="cuda")
    o = P.vmat.SolveOpts()
    o.max_cg_iter = 0
    o.master_mode = 1
    o.master = P.master_opts()
    res = {"variants": B}
    owner = P.Problem.from_case(case)
    try:
        res["owner_device_bytes"] = owner.device_bytes()
        for K in ks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps, l, r, occ, y = owner.solve_variants(label, tab, K=K, opts=o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[f"k{K}_s"] = round(dt, 3)
            res[f"k{K}_plans_per_s"] = round(B / dt, 2)
            log(f"[bench] {B} variant plans, aperture-dose master, {K} at a time on one D "
                f"(vmat_solve_variants): {dt:.2f}s")
            res["costs_first"] = [round(rp.F + rp.gG, 3) for rp in reps[:4]]
            del l, r, occ, y
    finally:
        owner.close()
    return res


def precision_study(workload, torch, P, reps, log):
    """Forward/adjoint speed of BF16 and FP8 storage against FP32 on this GPU,
    on the head-and-neck-shaped case, at the dose error each gives for one
    full-open plan (every aperture fully open, random intensities) against an
    FP64 CPU product of the FP32 D (scipy, computed here)."""
    import scipy.sparse as sp

    import casegen
    t0 = time.perf_counter()
    case = casegen.make_case(casegen.preset(workload))
    log(f"[bench] precision case {workload}: nnz={case.nnz} gen {time.perf_counter() - t0:.1f}s")
    rng = np.random.default_rng(7)
    N, R, C = case.n_beams, case.n_rows, case.n_cols
    occ = np.ones(N, np.uint8)
    l = np.zeros(N * R, np.int32)
    r = np.full(N * R, C, np.int32)
    y = rng.random(N) + 0.5
    # FP64 reference dose: all beamlets open, so x_i = y_k of beamlet i's beam
    x_open = np.repeat(y, R * C)
    D = sp.csr_matrix((case.val.astype(np.float64), case.col, case.row_ptr),
                      shape=(case.n_beamlets, case.n_voxels))
    zo = D.T @ x_open
    del D
    T = lambda a, dt: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    yt, lt, rt, ot = T(y, torch.float64), T(l, torch.int32), T(r, torch.int32), T(occ, torch.uint8)
    x = torch.from_numpy(rng.random(case.n_beamlets)).cuda()
    w = torch.from_numpy(rng.standard_normal(case.n_voxels).astype(np.float32)).cuda()
    zb = torch.empty(case.n_voxels, dtype=torch.float64, device="cuda")
    gb = torch.empty(case.n_beamlets, dtype=torch.float64, device="cuda")
    res = {"workload": workload, "nnz": case.nnz}
    for fmt in ("f32", "bf16", "fp8"):
        prob = P.Problem.from_case(case, d_store=fmt)
        zg = prob.dose(yt, lt, rt, ot).cpu().numpy().astype(np.float64)
        err_l2 = float(np.linalg.norm(zg - zo) / np.linalg.norm(zo))
        err_inf = float(np.abs(zg - zo).max() / np.abs(zo).max())
        f_ms = time_kernel(lambda: prob.forward(x, zb), reps, torch, warm_s=0.2)
        a_ms = time_kernel(lambda: prob.adjoint(w, gb), reps, torch, warm_s=0.2)
        lay = prob.layout()
        res[fmt] = {"forward_ms": round(f_ms, 5), "adjoint_ms": round(a_ms, 5),
                    "forward_GBs": round(lay["fwd_bytes"] / f_ms / 1e6, 1),
                    "adjoint_GBs": round(lay["adj_bytes"] / a_ms / 1e6, 1),
                    "dose_rel_l2": err_l2, "dose_rel_inf": err_inf}
        # one full plan on this case (aperture-dose master)
        o = P.vmat.SolveOpts()
        o.max_cg_iter = 0
        o.master_mode = 1
        o.master = P.master_opts()
        lp, rp, op, yp = prob.empty_plan()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, _ = prob.solve(lp, rp, op, yp, o, want_trace=False)
        torch.cuda.synchronize()
        res[fmt]["plan_s"] = round(time.perf_counter() - t0, 4)
        res[fmt]["plan_cost"] = rep.F + rep.gG
        log(f"[bench] {fmt}: fwd {f_ms:.4f} ms adj {a_ms:.4f} ms dose err l2 {err_l2:.2e} inf {err_inf:.2e} "
            f"plan {res[fmt]['plan_s']:.3f} s cost {rep.F + rep.gG:.6g}")
        prob.close()
    for fmt in ("bf16", "fp8"):
        res[fmt]["speedup_vs_f32"] = round((res["f32"]["forward_ms"] + res["f32"]["adjoint_ms"]) /
                                           (res[fmt]["forward_ms"] + res[fmt]["adjoint_ms"]), 3)
    return res


if __name__ == "__main__":
    main()
