#!/usr/bin/env python3
"""Benchmark of the Krylov CBCT hot path on one MI355X.

Headline workload "muct1500" (the largest configuration, a stand-in for the
micro-CT scan of the paper's Sec. 3.3): a 1500^3 volume at 10 um (seeded
porous cylinder, 2000 spherical pores, Gaussian blur sigma = 1 voxel, built
on the GPU), a 2000 x 2000 detector at 0.1 mm, 1571 angles over 360 deg,
DSO 150 mm, DSD 800 mm, Poisson noise at I0 = 1e5.  The solver is IRN-TV
(reweighted-norm TV, 10 outer x 20 inner CGLS iterations, lambda = 10,
eps = 1e-3) with the projector-facing vectors stored in FP16 (FP32 sums,
FP64 Krylov scalars).  All inputs are resident in HBM before any timed
region starts.

A step is one inner CGLS iteration of that IRN-TV run at full size: forward
projection of the search direction and its TV rows, matched back projection,
the fused vector updates and reductions, and the FP64 scalar recurrences.
`value` is inner iterations per second.  The same JSON line reports the
forward projector in GRays/s and the back projector in GVoxel-views/s (FP16
storage), a roofline entry for the dominant kernel, the FP64 oracle's rate
(timed on a 256^3 crop with all 1571 angles, extrapolated to the full size
by the nonzero count), the 256^3 medical workload's figures (CGLS it/s,
projector rates) and the serving stream's p50/p99 latency.

Other workloads and reports: --workload medical256 prints the same kind of
line for the 256^3 workload (a step is one CGLS iteration there);
--precision, --solvers, --operators-only and --profile-kernels print their
own reports.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

T_START = time.time()  # the bench's whole run, reported as wall_s

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GRays/s fwd proj, GVoxel-views/s backproj; CGLS it/s; p50/p99 recon latency"
WORKLOAD = "muct1500"      # the headline workload
MEDICAL = "medical256"     # the 256^3 workload reported beside it
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


def cpu_baseline(gd, x, n_angles_sample=24, name=MEDICAL):
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
        "sample": (f"FP64 Siddon forward + scatter adjoint of the {name} phantom over {n_angles_sample} of "
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


def counter_entry(workload, kernel_key, digest):
    """The committed rocprofv3 counter summary of one projector kernel, if it
    was taken on the current kernel source and the current launch-shape
    choices (`api.hip`, where the plan picks them); else None.  It holds the
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a plain
    copy), the L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)) and the VALU
    instructions per unit of work (SQ_INSTS_VALU over nonzeros or
    voxel-views)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.json")
    if not os.path.exists(path):
        return None
    k = json.load(open(path)).get("kernels", {}).get(kernel_key)
    if not k or k.get("src_digest") != digest or k.get("api_digest") != src_digest("api.hip"):
        return None
    return k


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


def cpu_baseline_extrapolated(stats, n_crop=256, det_crop=192):
    """The FP64 oracle on the micro-CT workload, which it cannot hold whole
    (the FP64 volume alone is 27 GB, and the adjoint keeps one per thread):
    forward and scatter adjoint of the porous phantom on the central
    ``n_crop``^3 block with the full 1571 angles and the central detector
    block, timed and turned into nonzeros per second, then extrapolated by
    the full problem's exact nonzero count to one inner CGLS iteration (one
    forward plus one adjoint; the TV stencils and vector updates are left
    out).  Labelled as an extrapolation."""
    import oracle
    import synth

    gd = synth.crop_geometry("muct1500", n_crop, det_crop, len(synth.geometry("muct1500")["angles"]))
    g = oracle.Geometry.from_dict(gd)
    o = (1500 - n_crop) // 2
    x = synth.phantom("muct1500", gd, full_n=1500, crop_origin=(o, o, o))
    t0 = time.perf_counter()
    nnz, _ = oracle.count_nnz(g)
    t1 = time.perf_counter()
    y = oracle.forward(g, x)
    t2 = time.perf_counter()
    oracle.adjoint(g, y)
    t3 = time.perf_counter()
    fwd_rate, adj_rate = nnz / (t2 - t1), nnz / (t3 - t2)
    t_iter = stats["nnz"] / fwd_rate + stats["nnz"] / adj_rate
    return {
        "value": 1.0 / t_iter, "unit": "IRN-TV inner CGLS it/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"FP64 Siddon forward + scatter adjoint of the central {n_crop}^3 block of the muct1500 phantom, "
                   f"all {len(g.angles)} angles, central {det_crop}^2 detector block ({nnz:.3e} nonzeros, "
                   f"{t3 - t1:.1f} s); EXTRAPOLATED by the full problem's {stats['nnz']:.3e} nonzeros to one inner "
                   "iteration (one forward + one adjoint; TV stencils and vector updates not included)"),
        "extrapolated": True,
        "fwd_gnnz_per_s": fwd_rate / 1e9, "bwd_gnnz_per_s": adj_rate / 1e9,
        "fwd_s_full_extrapolated": stats["nnz"] / fwd_rate, "bwd_s_full_extrapolated": stats["nnz"] / adj_rate,
        "count_s": round(t1 - t0, 2), "cpu_model": _cpu_model(),
    }


def roofline_entry(workload, kname, ms, nnz, n_out, es, n_units):
    """Roofline of one projector launch: algorithmic bytes of a matrix-free
    sparse matvec (every nonzero reads one input value, every output is
    written once) over the launch time, against the HBM peak.  The committed
    rocprofv3 counter summary of the workload adds the measured HBM traffic,
    the L2 hit rate and the VALU issue rate when it was taken on the current
    kernel source."""
    digest = src_digest("proj_fwd.hip" if kname == "forward" else "proj_bwd.hip")
    alg = nnz * es + n_out * es
    achieved = alg / (ms / 1000.0) / 1e9
    ce = counter_entry(workload, kname, digest)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": ce.get("hbm_bytes_per_launch") if ce else None,
           "kernel": kname, "launch_ms": round(ms, 3), "algorithmic_bytes_per_launch": alg,
           "achieved_is": "algorithmic bytes / launch time (an effective rate; caches serve most gathers)"}
    if ce:
        out["hbm_gbs_measured"] = round(ce["hbm_bytes_per_launch"] / (ms / 1000.0) / 1e9, 1)
        if "l2_hit" in ce:
            out["l2_hit"] = round(ce["l2_hit"], 4)
        if "valu_insts_per_unit" in ce:
            # The issue ceiling the gathers really meet: one wave64 VALU
            # instruction per CU per clock (4 SIMDs, 4 cycles each).
            rate = ce["valu_insts_per_unit"] * n_units / (ms / 1000.0)
            out["valu"] = {"insts_per_unit": round(ce["valu_insts_per_unit"], 4), "unit": ce["unit"],
                           "achieved": round(rate / 1e9, 1), "peak": VALU_PEAK_GINSTS,
                           "unit_rate": "G wave-instructions/s", "frac": round(rate / 1e9 / VALU_PEAK_GINSTS, 4)}
        pipe = ce.get("pipe")
        if pipe:
            # The vector memory pipe: texture address (TA) and data (TD) paths
            # busy as a fraction of active cycles, and L1 tag lookups per
            # 64-lane gather (rocprofv3 TA/TD/TCP counters).
            out["gather_pipe"] = {k: pipe[k] for k in ("ta_busy", "td_busy", "l1_tag_lookups_per_gather", "l1_hit")}
        # What limits the launch: the busiest of HBM (measured bytes against
        # the peak), VALU issue and the texture data path.
        cands = {"hbm": out.get("hbm_gbs_measured", 0.0) / HBM_PEAK_GBS}
        if "valu" in out:
            cands["valu_issue"] = out["valu"]["frac"]
        if pipe:
            cands["vector_memory_pipe"] = pipe["td_busy"]
        top = max(cands, key=cands.get)
        out["limiter"] = {"name": top, "busy": round(cands[top], 4)}
    return out


def muct_phantom(synth, gd, dev):
    """The micro-CT workload's porous phantom, built on the GPU."""
    ph = synth.WORKLOADS[WORKLOAD]["phantom"]
    return synth.porous_phantom_torch(gd, ph["n"], ph["radius_vox"], ph["cyl_frac"], ph["blur_sigma"],
                                      synth.WORKLOADS[WORKLOAD]["seed"], dev)


def load_stats(wl, kg):
    stats = json.load(open(os.path.join(ROOT, "tests", "golden", "workload_stats.json"))).get(wl)
    if stats is None:  # no exact count stored: sizes only, nnz unknown
        stats = {"rays": kg.n_rays, "voxels": kg.n_voxels, "voxel_views": kg.n_voxels * len(kg.angles),
                 "nnz": None, "hit_rays": None}
    return stats


def headline(args, torch, kct, synth):
    """The micro-CT step: inner CGLS iterations of IRN-TV at full size."""
    import numpy as np

    wl = WORKLOAD
    dev = torch.device("cuda", 0)
    vdt = getattr(torch, DTYPES[args.vec_dtype or "f16"])
    gd = synth.geometry(wl)
    kg = kct.Geometry.from_dict(gd)
    stats = load_stats(wl, kg)
    sol = synth.WORKLOADS[wl]["solve"]
    n_outer, n_inner, lam, eps = sol["n_outer"], sol["n_inner"], sol["lam"], sol["eps"]
    if args.warmup + args.steps > n_outer * n_inner:
        raise SystemExit(f"--warmup + --steps must be at most {n_outer * n_inner} (the run's inner iterations)")
    log(f"[bench] phantom ({wl}, on the GPU)")
    xt = muct_phantom(synth, gd, dev)
    log("[bench] clean projections (GPU forward) + noise")
    # A plan of its own for the data: its padded FP32 volume copies (27 GB)
    # are freed before the solver's workspace is allocated.
    plan = kct.Plan(kg)
    b, noise_info = synth.add_noise_torch(plan.forward(xt), synth.WORKLOADS[wl]["noise"], synth.WORKLOADS[wl]["seed"])
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    plan = kct.Plan(kg)

    log(f"[bench] IRN-TV inner iterations ({args.warmup} warm-up, {args.steps} timed)")
    st = plan.state(b, "irn_tv_cgls", 0, lam, vec_dtype=vdt, stream=torch.cuda.Stream(device=dev),
                    tv_outer=n_outer, tv_inner=n_inner, tv_eps=eps)
    st.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warm-up done; timing {args.steps} iterations")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event() for _ in range(args.steps)]
    e0.record(st.stream)
    for k in range(args.steps):
        st.step(1)
        marks[k].record(st.stream)
    e1.record(st.stream)
    # Every iteration is enqueued before the host waits: the waits below only
    # report progress (one line per finished iteration), the device never idles.
    for k, m in enumerate(marks):
        m.synchronize()
        log(f"[bench]   iteration {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / args.steps
    hist = st.history.cpu().numpy()[:args.warmup + args.steps]
    done = np.flatnonzero(hist[:, 3])
    if done.size:
        raise RuntimeError(f"IRN-TV stopped at inner iteration {done[0] + 1} (done code {int(hist[done[0], 3])}); "
                           "no iteration rate")
    st.close()
    del st, b
    torch.cuda.empty_cache()
    rate = 1000.0 / step_ms
    log(f"[bench] IRN-TV inner CGLS {rate:.4f} it/s ({step_ms:.0f} ms per iteration)")

    log(f"[bench] projector timings ({args.vec_dtype or 'f16'} storage)")
    x_in = xt.to(vdt)
    del xt
    y_out = torch.empty(kg.proj_shape, device=dev, dtype=vdt)
    x_out = torch.empty(kg.vol_shape, device=dev, dtype=vdt)
    fwd_ms = timed(lambda: plan.forward(x_in, out=y_out), args.reps, torch)
    bwd_ms = timed(lambda: plan.backproject(y_out, out=x_out), args.reps, torch)
    plan.check()
    del x_in, y_out, x_out
    plan.close()
    torch.cuda.empty_cache()
    log(f"[bench] fwd {fwd_ms:.0f} ms  bwd {bwd_ms:.0f} ms")
    n_vv = stats["voxel_views"]
    es = torch.tensor([], dtype=vdt).element_size()
    roofline = None
    if stats["nnz"]:
        if fwd_ms >= bwd_ms:
            roofline = roofline_entry(wl, "forward", fwd_ms, stats["nnz"], stats["rays"], es, stats["nnz"])
        else:
            roofline = roofline_entry(wl, "backward", bwd_ms, stats["nnz"], stats["voxels"], es, n_vv)

    medical = None
    if not args.no_medical:
        medical = medical_step(args, torch, kct, synth, extras=True)

    serving = serving_leg(args, torch) if not args.no_serve else None

    cpu = None
    if not args.no_cpu_baseline and stats["nnz"]:
        log("[bench] cpu baseline (oracle on a 256^3 crop, all angles, extrapolated by nonzeros)")
        cpu = cpu_baseline_extrapolated(stats)
        log(f"[bench] cpu {cpu['value']:.3e} it/s on {cpu['cores']} threads (extrapolated)")

    out = {
        "metric": METRIC, "value": round(rate, 5), "unit": "IRN-TV inner CGLS it/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl, "vec_storage": args.vec_dtype or "f16", "accumulation": "f32",
                   "krylov_scalars": "f64", "volume": [gd["nx"], gd["ny"], gd["nz"]], "voxel_mm": gd["vx"],
                   "detector": [gd["nu"], gd["nv"]], "pixel_mm": gd["du"], "angles": len(gd["angles"]),
                   "dso_mm": gd["dso"], "dsd_mm": gd["dsd"],
                   "solver": f"irn_tv_cgls {n_outer}x{n_inner}, lambda {lam}, eps {eps}",
                   "step": "one inner CGLS iteration", "phantom": "porous", "noise": synth.WORKLOADS[wl]["noise"],
                   "poisson_clamped_fraction": round(noise_info.get("clamped_fraction", 0.0), 5)},
        "fwd_grays_per_s": round(stats["rays"] / (fwd_ms / 1000.0) / 1e9, 3),
        "fwd_hit_grays_per_s": (round(stats["hit_rays"] / (fwd_ms / 1000.0) / 1e9, 3) if stats["hit_rays"] else None),
        "bwd_gvoxel_views_per_s": round(n_vv / (bwd_ms / 1000.0) / 1e9, 3),
        "fwd_ms": round(fwd_ms, 1), "bwd_ms": round(bwd_ms, 1),
        "gsegments_per_s": round(stats["nnz"] / (fwd_ms / 1000.0) / 1e9, 2) if stats["nnz"] else None,
        "irn_tv_full_extrapolated_s": round(step_ms / 1000.0 * n_outer * n_inner, 1),
        "medical256": medical, "serving": serving, "roofline": roofline, "cpu_baseline": cpu,
        "wall_s": round(time.time() - T_START, 1),
    }
    print(json.dumps(out), flush=True)


def serving_leg(args, torch):
    """Latency of the request mix (seeded stream, 2 req/s, shrunk by
    --serve-scale in volume side, detector side and angle count): continuous
    batching against serial per-request solves."""
    from paper_2211_14212_amd import serve

    log("[bench] serving stream")
    torch.cuda.empty_cache()
    reqs = serve.make_requests(args.serve_requests, 2.0, seed=5, size_scale=args.serve_scale)
    srv = serve.Server(200e9, keep_results=False, verbose=True)
    batched = serve.summarize(srv.run(reqs))
    serial = serve.summarize(serve.serve_serial(reqs, keep_results=False, verbose=True), rate=2.0)
    # The offered load: arrival rate x mean service time of a request alone
    # on the GPU (the serial path's solve times).
    rho = serial.pop("offered_load_rho")
    out = {"requests": args.serve_requests, "rate_per_s": 2.0, "size_scale": args.serve_scale,
           "offered_load_rho": round(rho, 3),
           "admission": f"{srv.policy}, {srv.max_active} active, fillers up to {srv.filler_frac} of the "
                        "first-come request's work, 2 iterations in flight each",
           "batched": {k: round(v, 4) for k, v in batched.items()},
           "serial": {k: round(v, 4) for k, v in serial.items()}}
    log(f"[bench] serving {out}")
    del reqs
    torch.cuda.empty_cache()
    return out


def medical_step(args, torch, kct, synth, extras=False):
    """The 256^3 workload: CGLS iterations per second (the step there),
    projector rates and a roofline entry.  ``extras``: the shorter set
    reported beside the headline (no LSQR/LSMR rates, solves or serving)."""
    wl = MEDICAL
    dev = torch.device("cuda", 0)
    vdt = getattr(torch, DTYPES[args.vec_dtype or "f32"]) if not extras else torch.float32
    gd = synth.geometry(wl)
    kg = kct.Geometry.from_dict(gd)
    stats = load_stats(wl, kg)
    plan = kct.Plan(kg)
    log(f"[bench] phantom ({wl})")
    x_true = synth.phantom(wl)
    xt = torch.from_numpy(x_true).to(dev)
    b_clean = plan.forward(xt).cpu().numpy()
    b_np, noise_info = synth.add_noise(b_clean, synth.WORKLOADS[wl]["noise"], synth.WORKLOADS[wl]["seed"])
    del b_clean
    b = torch.from_numpy(b_np).to(dev)
    del b_np
    torch.cuda.synchronize()
    steps, warmup = (10, 3) if extras else (args.steps, args.warmup)
    log(f"[bench] {wl} CGLS iterations")
    cgls_rate, cgls_ms, _ = iter_rate(plan, b, "cgls", warmup, steps, torch, vdt)
    log(f"[bench] {wl} CGLS {cgls_rate:.2f} it/s")
    y_out = torch.empty(kg.proj_shape, device=dev, dtype=vdt)
    x_out = torch.empty(kg.vol_shape, device=dev, dtype=vdt)
    x_in, b_in = xt.to(vdt), b.to(vdt)
    fwd_ms = timed(lambda: plan.forward(x_in, out=y_out), args.reps, torch)
    bwd_ms = timed(lambda: plan.backproject(b_in, out=x_out), args.reps, torch)
    plan.check()
    del x_in, b_in, y_out, x_out
    log(f"[bench] {wl} fwd {fwd_ms:.2f} ms  bwd {bwd_ms:.2f} ms")
    nnz, N, M, n_vv = stats["nnz"], stats["rays"], stats["voxels"], stats["voxel_views"]
    es = torch.tensor([], dtype=vdt).element_size()
    if fwd_ms >= bwd_ms:
        roofline = roofline_entry(wl, "forward", fwd_ms, nnz, N, es, nnz)
    else:
        roofline = roofline_entry(wl, "backward", bwd_ms, nnz, M, es, n_vv)
    out = {
        "workload": wl, "cgls_it_per_s": round(cgls_rate, 3), "ms_per_cgls_iteration": round(cgls_ms / steps, 3),
        "fwd_grays_per_s": round(N / (fwd_ms / 1000.0) / 1e9, 3),
        "fwd_hit_grays_per_s": round(stats["hit_rays"] / (fwd_ms / 1000.0) / 1e9, 3),
        "bwd_gvoxel_views_per_s": round(n_vv / (bwd_ms / 1000.0) / 1e9, 3),
        "fwd_ms": round(fwd_ms, 3), "bwd_ms": round(bwd_ms, 3),
        "gsegments_per_s": round(nnz / (fwd_ms / 1000.0) / 1e9, 2), "roofline": roofline,
    }
    if not extras:
        out["lsqr_it_per_s"] = round(iter_rate(plan, b, "lsqr", warmup, steps, torch, vdt)[0], 3)
        out["lsmr_it_per_s"] = round(iter_rate(plan, b, "lsmr", warmup, steps, torch, vdt)[0], 3)
        if not args.no_solves:
            solves = {}
            for solver in ("cgls", "lsqr", "lsmr"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xs, hs = plan.solve(b, solver, 30, vec_dtype=vdt)
                torch.cuda.synchronize()
                solves[f"{solver}30_s"] = round(time.perf_counter() - t0, 4)
                solves[f"{solver}30_last_res"] = float(hs.cpu().numpy()[-1, 0])
                solves[f"{solver}30_rel_err_vs_phantom"] = round(
                    float(torch.linalg.vector_norm(xs - xt) / torch.linalg.vector_norm(xt)), 4)
            out["solves"] = solves
    if not args.no_cpu_baseline:
        log(f"[bench] {wl} cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(gd, x_true)
        log(f"[bench] {wl} cpu {out['cpu_baseline']['value']:.4f} it/s on {out['cpu_baseline']['cores']} threads")
    out["_noise_info"] = noise_info
    out["_cgls_ms"] = cgls_ms
    plan.close()
    del xt, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 10; the headline: 6)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 3; the headline: 1)")
    ap.add_argument("--reps", type=int, default=None, help="calls per projector timing (default 5; the headline: 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true", help="skip the solves (with --operators-only: the IRN-TV run)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-medical", action="store_true", help="headline: leave out the 256^3 workload's figures")
    ap.add_argument("--workload", default=WORKLOAD, help="synthetic workload (default: the benchmark's)")
    ap.add_argument("--vec-dtype", default=None, choices=sorted(DTYPES),
                    help="storage of the projector-facing Krylov vectors (default: f16 for the micro-CT "
                         "workload, else f32)")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-scale", type=float, default=0.75,
                    help="volume side, detector side and angle count of the request stream, relative to the "
                         "workload's (0.75: offered load above one at 2 requests/s)")
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
    report = args.precision or args.operators_only or args.solvers or args.profile_kernels
    head = args.workload == WORKLOAD and not report
    if args.steps is None:
        args.steps = 6 if head else 10
    if args.warmup is None:
        args.warmup = 1 if head else 3
    if args.reps is None:
        args.reps = 2 if head else 5

    import numpy as np
    import torch

    import paper_2211_14212_amd as kct
    import synth

    if head:
        kct.require_gpu()
        headline(args, torch, kct, synth)
        return
    if args.workload == MEDICAL and not report:
        kct.require_gpu()
        m = medical_step(args, torch, kct, synth)
        gd = synth.geometry(MEDICAL)
        noise_info, cgls_ms = m.pop("_noise_info"), m.pop("_cgls_ms")
        out = {
            "metric": METRIC, "value": m["cgls_it_per_s"], "unit": "CGLS it/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(cgls_ms / args.steps, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": MEDICAL, "vec_storage": args.vec_dtype or "f32",
                       "volume": [gd["nx"], gd["ny"], gd["nz"]], "voxel_mm": gd["vx"],
                       "detector": [gd["nu"], gd["nv"]], "pixel_mm": gd["du"], "angles": len(gd["angles"]),
                       "dso_mm": gd["dso"], "dsd_mm": gd["dsd"], "solver": "cgls", "phantom": "ellipsoids",
                       "noise": synth.WORKLOADS[MEDICAL]["noise"],
                       "poisson_clamped_fraction": round(noise_info.get("clamped_fraction", 0.0), 5)},
            "roofline": m.pop("roofline"), "cpu_baseline": m.pop("cpu_baseline", None),
        }
        out.update({k: v for k, v in m.items() if k != "workload"})
        if not args.no_serve:
            out["serving"] = serving_leg(args, torch)
        out["wall_s"] = round(time.time() - T_START, 1)
        print(json.dumps(out), flush=True)
        return
    report_modes(args, np, torch, kct, synth)


def report_modes(args, np, torch, kct, synth):
    """--precision, --solvers, --operators-only and --profile-kernels."""
    vdt = getattr(torch, DTYPES[args.vec_dtype or ("f16" if args.workload == WORKLOAD else "f32")])
    kct.require_gpu()
    dev = torch.device("cuda", 0)
    wl = args.workload
    gd = synth.geometry(wl)
    kg = kct.Geometry.from_dict(gd)
    stats = load_stats(wl, kg)
    plan = kct.Plan(kg)
    if args.profile_kernels and synth.WORKLOADS[wl]["phantom"]["kind"] == "porous":
        # The projectors' memory traffic does not depend on the values: a
        # seeded uniform volume stands in for the slow porous phantom.
        log(f"[bench] uniform random volume ({wl})")
        xt = torch.rand(kg.vol_shape, device=dev, generator=torch.Generator(device=dev).manual_seed(4))
    elif synth.WORKLOADS[wl]["phantom"]["kind"] == "porous":
        log(f"[bench] phantom ({wl}, on the GPU)")
        xt = muct_phantom(synth, gd, dev)
    else:
        log(f"[bench] phantom ({wl})")
        xt = torch.from_numpy(synth.phantom(wl)).to(dev)
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
    if wl == MEDICAL:
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
    raise SystemExit("no report selected")


if __name__ == "__main__":
    main()
