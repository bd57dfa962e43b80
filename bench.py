#!/usr/bin/env python3
"""Benchmark of the Krylov CBCT hot path on one MI355X.

Workload "medical256": 256^3 volume at 0.5 mm (40 seeded ellipsoids),
512 x 512 detector at 0.4 mm, 360 angles over 360 deg, DSO 1000 mm,
DSD 1500 mm, Poisson noise at I0 = 1e5 (synthetic stand-in for the medical
scan of the paper's Sec. 3.2).  All inputs are resident in HBM before any
timed region starts.

A step is one CGLS iteration: forward projection, matched back projection,
the fused vector updates and reductions, and the FP64 scalar recurrences.
`value` is CGLS iterations per second.  The same JSON line also reports the
forward projector in GRays/s, the back projector in GVoxel-views/s, LSQR
and LSMR iterations per second, 30-iteration solve times, a roofline entry
for the dominant kernel and the CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GRays/s fwd proj, GVoxel-views/s backproj; CGLS it/s; p50/p99 recon latency"
WORKLOAD = "medical256"
DTYPES = {"f32": "float32", "bf16": "bfloat16", "f16": "float16"}
HBM_PEAK_GBS = 8000.0
VALU_PEAK_GINSTS = 256 * 2.4  # 256 CUs x 2.4 GHz x one wave64 VALU instruction per CU-clock


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2211_14212_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def timed(fn, reps, torch):
    """Average ms per call, HIP events on the current stream (where the kernels run)."""
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def iter_rate(plan, b, solver, warmup, steps, torch, vec_dtype=None):
    """Iterations/s of `solver` over `steps` iterations after `warmup` ones,
    on a stream of its own (which lets CGLS replay a captured iteration)."""
    import numpy as np

    st = plan.state(b, solver, warmup + steps, vec_dtype=vec_dtype or torch.float32,
                    stream=torch.cuda.Stream(device=b.device))
    st.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st.stream)
    for _ in range(steps):
        st.step(1)
    e1.record(st.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    hist = st.history.cpu().numpy()
    st.close()
    # A run that ended early (breakdown, a non-finite value, the stop rule)
    # skips the rest of its kernels: its rate would not be an iteration rate.
    done = np.flatnonzero(hist[:, 3])
    if done.size:
        raise RuntimeError(f"{solver} stopped at iteration {done[0] + 1} of {warmup + steps} (done code "
                           f"{int(hist[done[0], 3])}); no iteration rate")
    return steps / (ms / 1000.0), ms, hist


def cpu_baseline_full_cgls(gd, b, n_iter):
    """The whole FP64 oracle CGLS run of a small workload, on all host
    threads and on one: iterations per second."""
    import numpy as np

    import oracle
    from oracle import solvers

    g = oracle.Geometry.from_dict(gd)
    b64 = np.asarray(b, dtype=np.float64)
    A, AT = (lambda v: oracle.forward(g, v)), (lambda y: oracle.adjoint(g, y))
    cores = oracle.num_threads()
    rates = {}
    for nth in (cores, 1):
        oracle.set_num_threads(nth)
        t0 = time.perf_counter()
        solvers.cgls(A, AT, b64, n_iter)
        rates[nth] = n_iter / (time.perf_counter() - t0)
    oracle.set_num_threads(cores)
    return {"value": rates[cores], "unit": "CGLS it/s", "cores": cores, "kind": "oracle",
            "sample": f"the full FP64 CGLS-{n_iter} of the workload (from the same noisy b)",
            "single_thread_it_per_s": rates[1]}


def cpu_baseline(gd, x, n_angles_sample=24):
    """The FP64 oracle on the host: forward and scatter adjoint over a subset
    of the angles, scaled to one CGLS iteration of the full workload."""
    import numpy as np

    import oracle

    g = oracle.Geometry.from_dict(gd)
    na = len(g.angles)
    sel = np.linspace(0, na, n_angles_sample, endpoint=False).astype(int)
    gs = g.with_angles([g.angles[a] for a in sel])
    t0 = time.perf_counter()
    y = oracle.forward(gs, x)
    t1 = time.perf_counter()
    oracle.adjoint(gs, y)
    t2 = time.perf_counter()
    scale = na / n_angles_sample
    t_iter = (t2 - t0) * scale
    return {
        "value": 1.0 / t_iter, "unit": "CGLS it/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"FP64 Siddon forward + scatter adjoint of the {WORKLOAD} phantom over {n_angles_sample} of "
                   f"{na} angles ({t2 - t0:.1f} s), scaled x{scale:.0f} to one CGLS iteration; vector updates "
                   "(<1% of an iteration) not included"),
        "fwd_grays_per_s": (len(gs.angles) * g.nu * g.nv) / (t1 - t0) / 1e9,
        "bwd_gvoxel_views_per_s": (g.nx * g.ny * g.nz * len(gs.angles)) / (t2 - t1) / 1e9,
        "cpu_model": _cpu_model(),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def counter_entry(kernel_key, digest):
    """The committed rocprofv3 counter summary of one projector kernel, if it
    was taken on the current kernel source; else None.  It holds the HBM bytes
    per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), the L2
    hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)) and the VALU instructions per
    unit of work (SQ_INSTS_VALU over nonzeros or voxel-views)."""
    path = os.path.join(ROOT, "profiles", f"{WORKLOAD}_counters.json")
    if not os.path.exists(path):
        return None
    k = json.load(open(path)).get("kernels", {}).get(kernel_key)
    if not k or k.get("src_digest") != digest:
        return None
    return k


def _phantom_slab(job):
    name, gd, k0, nz = job
    import synth

    g = dict(gd)
    g["nz"] = nz
    return k0, synth.phantom(name, g, full_n=gd["nx"], crop_origin=(k0, 0, 0))


def phantom_in_slabs(name, gd, slab=100, workers=8):
    """The workload's phantom, built in z-slabs by worker processes (each slab
    equals the same block of the full phantom).  Call before the GPU is used."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    out = np.empty((gd["nz"], gd["ny"], gd["nx"]), dtype=np.float32)
    jobs = [(name, gd, k0, min(slab, gd["nz"] - k0)) for k0 in range(0, gd["nz"], slab)]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        for k0, arr in ex.map(_phantom_slab, jobs):
            out[k0:k0 + arr.shape[0]] = arr
    return out


def precision_report(plan, b, xt, torch, wl):
    """c3: LSQR (lambda 10) and hybrid LSQR (lambda 10), 50 iterations, with
    the vectors stored in FP32, BF16 and FP16; each result against the FP32
    path and the phantom."""
    spec = {"lsqr": dict(lam=10.0), "hybrid_lsqr": dict(lam=10.0)}
    out = {}
    for solver, kw in spec.items():
        ref = None
        for name in ("f32", "bf16", "f16"):
            vdt = getattr(torch, DTYPES[name])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, h = plan.solve(b, solver, 50, kw["lam"], vec_dtype=vdt)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r = {"solve_s": round(dt, 3), "it_per_s": round(50 / dt, 3),
                 "rel_err_vs_phantom": round(float(torch.linalg.vector_norm(x - xt) / torch.linalg.vector_norm(xt)), 5)}
            if ref is None:
                ref = x.clone()
            else:
                r["rel_diff_vs_f32_path"] = float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))
            out[f"{solver}_{name}"] = r
            log(f"[precision] {solver} {name}: {r}")
            del x, h
    return out


# Every solver of the library on the same data, 30 iterations each (IRN-TV:
# 3 outer x 10 inner): wall time per iteration and error against the phantom.
SOLVER_RUNS = [
    ("cgls", "cgls", 30, 0.0, {}),
    ("lsqr", "lsqr", 30, 0.0, {}),
    ("lsmr", "lsmr", 30, 0.0, {}),
    ("hybrid_lsqr_gcv", "hybrid_lsqr", 30, 0.0, {"lam_rule": "gcv"}),
    ("ab_gmres_interp", "ab_gmres", 30, 0.0, {"backprojector": "interp"}),
    ("ba_gmres_interp", "ba_gmres", 30, 0.0, {"backprojector": "interp"}),
    ("sirt", "sirt", 30, 1.0, {}),
    ("os_sart_10_subsets", "os_sart", 30, 1.0, {"n_subsets": 10}),
    ("irn_tv_cgls_3x10", "irn_tv_cgls", 0, 1.0, {"tv_outer": 3, "tv_inner": 10, "tv_eps": 1e-3}),
    ("hybrid_flsqr_tv", "hybrid_flsqr_tv", 30, 0.1, {"tv_inner": 10, "tv_eps": 1e-3}),
]


def solver_report(plan, b, xt, torch, scale=1.0):
    """``scale`` shrinks every iteration count (profiling runs)."""
    out = {}
    nx = torch.linalg.vector_norm(xt)
    for label, solver, n, lam, kw in SOLVER_RUNS:
        kw = dict(kw)
        n = max(1, int(round(n * scale))) if n else 0
        if solver == "irn_tv_cgls":
            kw["tv_outer"] = max(1, int(round(kw["tv_outer"] * scale)))
        iters = kw["tv_outer"] * kw["tv_inner"] if solver == "irn_tv_cgls" else n
        log(f"[bench] solver {label}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, h = plan.solve(b, solver, n, lam, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        h = h.cpu().numpy()
        out[label] = {"iterations": iters, "lambda": lam, "s": round(dt, 3), "ms_per_iter": round(1e3 * dt / iters, 2),
                      "rel_err_vs_phantom": round(float(torch.linalg.vector_norm(x - xt) / nx), 4),
                      "last_hist_res": float(h[-1, 0]), "last_lambda": float(h[-1, 4])}
        log(f"[bench]   {out[label]}")
        del x, h
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5, help="calls per projector timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true", help="skip the solves (with --operators-only: the IRN-TV run)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD, help="synthetic workload (default: the benchmark's)")
    ap.add_argument("--vec-dtype", default="f32", choices=sorted(DTYPES),
                    help="storage of the projector-facing Krylov vectors")
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--serve-scale", type=float, default=0.25)
    ap.add_argument("--precision", action="store_true",
                    help="the 16-bit storage report instead of the step benchmark: LSQR and hybrid LSQR "
                         "(lambda 10, 50 iterations) with FP32, BF16 and FP16 vectors, each compared with the "
                         "FP32 path; prints its own JSON line")
    ap.add_argument("--operators-only", action="store_true",
                    help="projector timings and a short IRN-TV run only (for the largest workloads); prints its "
                         "own JSON line")
    ap.add_argument("--solvers", action="store_true",
                    help="report every solver's time per iteration and error vs the phantom instead of the "
                         "benchmark line")
    ap.add_argument("--solver-scale", type=float, default=1.0,
                    help="with --solvers: multiply every iteration count (e.g. 0.34 for a profiling run)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run the projectors (and a plain 1 GiB copy for counter calibration) "
                         "a few times, for rocprofv3; prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU angle-sharded "
              "path is a documented design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2211_14212_amd as kct
    import synth

    big_phantom = None
    if args.operators_only and synth.WORKLOADS[args.workload]["phantom"]["kind"] == "porous":
        log("[bench] phantom in slabs (worker processes, before the GPU is used)")
        big_phantom = phantom_in_slabs(args.workload, synth.geometry(args.workload))
    kct.require_gpu()
    dev = torch.device("cuda", 0)
    wl = args.workload
    vdt = getattr(torch, DTYPES[args.vec_dtype])
    gd = synth.geometry(wl)
    kg = kct.Geometry.from_dict(gd)
    stats = json.load(open(os.path.join(ROOT, "tests", "golden", "workload_stats.json"))).get(wl)
    if stats is None:  # no exact count stored: sizes only, nnz unknown
        stats = {"rays": kg.n_rays, "voxels": kg.n_voxels, "voxel_views": kg.n_voxels * len(kg.angles),
                 "nnz": None, "hit_rays": None}

    plan = kct.Plan(kg)
    if args.profile_kernels and synth.WORKLOADS[wl]["phantom"]["kind"] == "porous":
        # The projectors' memory traffic does not depend on the values: a
        # seeded uniform volume stands in for the slow porous phantom.
        log(f"[bench] uniform random volume ({wl})")
        xt = torch.rand(kg.vol_shape, device=dev, generator=torch.Generator(device=dev).manual_seed(4))
    else:
        log(f"[bench] phantom ({wl})")
        x_true = big_phantom if big_phantom is not None else synth.phantom(wl)
        xt = torch.from_numpy(x_true).to(dev)
    if args.profile_kernels:
        # Projector inputs and outputs in the --vec-dtype storage.
        xt = xt.to(vdt)
        y = torch.empty(kg.proj_shape, device=dev, dtype=vdt)
        xb = torch.empty(kg.vol_shape, device=dev, dtype=vdt)
        src = torch.ones(1 << 28, device=dev)  # 1 GiB of FP32
        dst = torch.empty_like(src)
        for _ in range(args.reps):
            plan.forward(xt, out=y)
            plan.backproject(y, out=xb)
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] profile-kernels done")
        return
    log("[bench] clean projections (GPU forward) + noise")
    if wl == WORKLOAD:
        b_clean = plan.forward(xt).cpu().numpy()
        b_np, noise_info = synth.add_noise(b_clean, synth.WORKLOADS[wl]["noise"], synth.WORKLOADS[wl]["seed"])
        del b_clean
        b = torch.from_numpy(b_np).to(dev)
        del b_np
    else:
        b, noise_info = synth.add_noise_torch(plan.forward(xt), synth.WORKLOADS[wl]["noise"],
                                              synth.WORKLOADS[wl]["seed"])
    torch.cuda.synchronize()

    if args.solvers:
        rep = solver_report(plan, b, xt, torch, args.solver_scale)
        print(json.dumps({"report": "solvers", "workload": wl, "data": "synthetic", "results": rep}), flush=True)
        return
    if args.precision:
        rep = precision_report(plan, b, xt, torch, wl)
        print(json.dumps({"report": "16-bit vector storage vs the FP32 path", "workload": wl, "data": "synthetic",
                          "results": rep}), flush=True)
        return
    if args.operators_only:
        # Projector timings in the workload's solver storage, one short IRN-TV
        # run, and the full IRN-TV time extrapolated from its per-iteration cost.
        # Cached blocks are returned between phases: at 1500^3 the phases
        # together would not fit the HBM.
        torch.cuda.empty_cache()
        sol = synth.WORKLOADS[wl]["solve"]
        x_in, b_in = xt.to(vdt), b.to(vdt)
        y_out = torch.empty(kg.proj_shape, device=dev, dtype=vdt)
        x_out = torch.empty(kg.vol_shape, device=dev, dtype=vdt)
        fwd_ms = timed(lambda: plan.forward(x_in, out=y_out), args.reps, torch)
        bwd_ms = timed(lambda: plan.backproject(b_in, out=x_out), args.reps, torch)
        del x_in, b_in, y_out, x_out
        torch.cuda.empty_cache()
        log(f"[bench] fwd {fwd_ms:.1f} ms  bwd {bwd_ms:.1f} ms")
        rep = {"fwd_ms": round(fwd_ms, 2), "bwd_ms": round(bwd_ms, 2),
               "fwd_grays_per_s": round(kg.n_rays / (fwd_ms / 1000.0) / 1e9, 3),
               "bwd_gvoxel_views_per_s": round(kg.n_voxels * len(kg.angles) / (bwd_ms / 1000.0) / 1e9, 3)}
        if stats.get("nnz"):
            rep["gsegments_per_s"] = round(stats["nnz"] / (fwd_ms / 1000.0) / 1e9, 2)
        if "n_outer" in sol and not args.no_solves:
            inner = 2
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, h = plan.solve(b, "irn_tv_cgls", 0, sol["lam"], vec_dtype=vdt, tv_outer=1, tv_inner=inner,
                              tv_eps=sol["eps"])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            done = np.flatnonzero(h.cpu().numpy()[:, 3])
            if done.size:
                raise RuntimeError(f"IRN-TV stopped at inner iteration {done[0] + 1} (done code "
                                   f"{int(h[done[0], 3])}); no timing")
            rep["irn_tv_1x2_s"] = round(dt, 3)
            rep["irn_tv_full_extrapolated_s"] = round(dt / inner * sol["n_outer"] * sol["n_inner"], 1)
            rep["irn_tv_full"] = f"{sol['n_outer']} outer x {sol['n_inner']} inner, lambda {sol['lam']}"
            del x, h
        print(json.dumps({"report": "operators", "workload": wl, "vec_storage": args.vec_dtype, "data": "synthetic",
                          "results": rep}), flush=True)
        return

    # ---- the step: one CGLS iteration ------------------------------------
    log("[bench] CGLS iterations")
    cgls_rate, cgls_ms, _ = iter_rate(plan, b, "cgls", args.warmup, args.steps, torch, vdt)
    log(f"[bench] CGLS {cgls_rate:.2f} it/s")

    # ---- operators ---------------------------------------------------------
    log("[bench] projector timings")
    y_out = torch.empty(kg.proj_shape, device=dev, dtype=vdt)
    x_out = torch.empty(kg.vol_shape, device=dev, dtype=vdt)
    x_in, b_in = xt.to(vdt), b.to(vdt)
    fwd_ms = timed(lambda: plan.forward(x_in, out=y_out), args.reps, torch)
    bwd_ms = timed(lambda: plan.backproject(b_in, out=x_out), args.reps, torch)
    del x_in, b_in
    n_rays, n_vv, nnz = stats["rays"], stats["voxel_views"], stats["nnz"]
    M, N = stats["voxels"], stats["rays"]
    log(f"[bench] fwd {fwd_ms:.2f} ms  bwd {bwd_ms:.2f} ms")

    lsqr_rate, _, _ = iter_rate(plan, b, "lsqr", args.warmup, args.steps, torch, vdt)
    lsmr_rate, _, _ = iter_rate(plan, b, "lsmr", args.warmup, args.steps, torch, vdt)
    log(f"[bench] LSQR {lsqr_rate:.2f} it/s  LSMR {lsmr_rate:.2f} it/s")

    solves = {}
    if not args.no_solves:
        for solver in ("cgls", "lsqr", "lsmr"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, hs = plan.solve(b, solver, 30, vec_dtype=vdt)
            torch.cuda.synchronize()
            solves[f"{solver}30_s"] = round(time.perf_counter() - t0, 4)
            h = hs.cpu().numpy()
            solves[f"{solver}30_last_res"] = float(h[-1, 0])
            err = float(torch.linalg.vector_norm(xs - xt) / torch.linalg.vector_norm(xt))
            solves[f"{solver}30_rel_err_vs_phantom"] = round(err, 4)
        log(f"[bench] solves {solves}")

    # ---- roofline of the dominant kernel ----------------------------------
    # Algorithmic bytes of a matrix-free sparse matvec: every nonzero a_ij
    # reads one input value, every output is written once.
    es = torch.tensor([], dtype=vdt).element_size()
    roofline = None
    if nnz is not None:
        if fwd_ms >= bwd_ms:
            kname, ms, alg = "forward", fwd_ms, nnz * es + N * es
            digest = src_digest("proj_fwd.hip")
        else:
            kname, ms, alg = "backward", bwd_ms, nnz * es + M * es
            digest = src_digest("proj_bwd.hip")
        achieved = alg / (ms / 1000.0) / 1e9
        ce = counter_entry(kname, digest) if wl == WORKLOAD and es == 4 else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": ce.get("hbm_bytes_per_launch") if ce else None, "kernel": kname,
                    "launch_ms": round(ms, 3), "algorithmic_bytes_per_launch": alg}
        if ce and "valu_insts_per_unit" in ce:
            # The issue ceiling the gathers really meet: one wave64 VALU
            # instruction per CU per clock (4 SIMDs, 4 cycles each).
            units = nnz if kname == "forward" else M * len(kg.angles)
            rate = ce["valu_insts_per_unit"] * units / (ms / 1000.0)
            roofline["l2_hit"] = round(ce["l2_hit"], 4) if "l2_hit" in ce else None
            roofline["valu"] = {"insts_per_unit": round(ce["valu_insts_per_unit"], 4), "unit": ce["unit"],
                                "achieved": round(rate / 1e9, 1), "peak": VALU_PEAK_GINSTS,
                                "unit_rate": "G wave-instructions/s", "frac": round(rate / 1e9 / VALU_PEAK_GINSTS, 4)}

    serving = None
    if not args.no_serve and wl == WORKLOAD:
        # Latency of the request mix (seeded stream, 2 req/s, shrunk by
        # --serve-scale in volume side, detector side and angle count):
        # continuous batching against serial per-request solves.
        from paper_2211_14212_amd import serve

        log("[bench] serving stream")
        del y_out, x_out
        torch.cuda.empty_cache()
        reqs = serve.make_requests(args.serve_requests, 2.0, seed=5, size_scale=args.serve_scale)
        batched = serve.summarize(serve.Server(200e9, keep_results=False).run(reqs))
        serial = serve.summarize(serve.serve_serial(reqs, keep_results=False))
        serving = {"requests": args.serve_requests, "rate_per_s": 2.0, "size_scale": args.serve_scale,
                   "batched": {k: round(v, 4) for k, v in batched.items()},
                   "serial": {k: round(v, 4) for k, v in serial.items()}}
        log(f"[bench] serving {serving}")

    cpu = None
    if not args.no_cpu_baseline and wl == WORKLOAD:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(gd, x_true)
        log(f"[bench] cpu {cpu['value']:.4f} it/s on {cpu['cores']} threads")
    elif not args.no_cpu_baseline and wl == "cgls32":
        log("[bench] cpu baseline (oracle, full CGLS-20)")
        cpu = cpu_baseline_full_cgls(gd, b.cpu().numpy(), 20)
        log(f"[bench] cpu {cpu['value']:.1f} it/s on {cpu['cores']} threads, {cpu['single_thread_it_per_s']:.1f} on 1")

    out = {
        "metric": METRIC, "value": round(cgls_rate, 3), "unit": "CGLS it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(cgls_ms / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl, "vec_storage": args.vec_dtype, "volume": [gd["nx"], gd["ny"], gd["nz"]], "voxel_mm": gd["vx"],
                   "detector": [gd["nu"], gd["nv"]], "pixel_mm": gd["du"], "angles": len(gd["angles"]),
                   "dso_mm": gd["dso"], "dsd_mm": gd["dsd"], "solver": "cgls",
                   "phantom": synth.WORKLOADS[wl]["phantom"]["kind"], "noise": synth.WORKLOADS[wl]["noise"],
                   "poisson_clamped_fraction": round(noise_info.get("clamped_fraction", 0.0), 5)},
        "fwd_grays_per_s": round(n_rays / (fwd_ms / 1000.0) / 1e9, 3),
        "fwd_hit_grays_per_s": (round(stats["hit_rays"] / (fwd_ms / 1000.0) / 1e9, 3)
                                if stats["hit_rays"] else None),
        "bwd_gvoxel_views_per_s": round(n_vv / (bwd_ms / 1000.0) / 1e9, 3),
        "fwd_ms": round(fwd_ms, 3), "bwd_ms": round(bwd_ms, 3),
        "gsegments_per_s": round(nnz / (fwd_ms / 1000.0) / 1e9, 2) if nnz else None,
        "lsqr_it_per_s": round(lsqr_rate, 3), "lsmr_it_per_s": round(lsmr_rate, 3),
        "solves": solves, "serving": serving, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
