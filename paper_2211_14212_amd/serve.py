"""Continuous-batching reconstruction server.

Requests (a geometry, measured projections b, a solver and an iteration
count) arrive over time.  The server admits them in arrival order while the
HBM they need (plan tables, workspace, b, x, history) fits a byte budget,
gives each admitted request its own HIP stream and device-resident Krylov
state (kct_state), and advances all active requests one iteration at a time,
so kernels of different requests overlap on the GPU.  Each request keeps up
to ``depth`` iterations enqueued ahead of the device (2 by default), so its
stream never waits for the host between iterations.  Plans (the per-angle
tables, whose build waits for the device) are made by a worker thread as
requests arrive, off the serving loop.  A request leaves when its last
iteration has run on the device; its memory is freed and queued requests are
admitted in its place.  A request that needs more memory than the whole
budget is rejected when its plan is ready, and so is one whose plan cannot
be made (an invalid geometry; the result carries the library's message).  Each request's result is bitwise the
same as a solo kct_solve of it (deterministic kernels, private buffers).
Admission is first-come first-served by default; ``policy="sjf"`` admits the
queued request with the least work first (ray-iterations, the cost of its
projector calls), which shortens typical latency when the stream outruns
the GPU, at the expense of the largest requests; ``policy="mixed"`` keeps one
slot first-come first-served (the oldest queued request is always the next
to run in it, so no request waits behind an endless supply of smaller ones)
and fills the other slots shortest-job-first with requests whose work is at
most ``filler_frac`` of the first-come request's, which then run beside it
without slowing it much (their kernels are small).
A request can be cancelled (``Server.cancel``): no further iteration of it is
enqueued, and once its last enqueued one has run its memory is freed and it
returns a result marked ``cancelled`` with no image.  The other requests are
unaffected, bit for bit.

Latency = completion time - arrival time.  The serial baseline runs the same
stream through the plain per-request path (one kct_solve at a time, FIFO).

CLI:  python -m paper_2211_14212_amd.serve [--requests 64] [--rate 2.0]
          [--size-scale 1.0] [--budget-gb 200] [--no-serial] [--sjf]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time
from collections import deque

import numpy as np
import torch

from . import Geometry, Plan
from ._lib import KCT_HIST_COLS


@dataclasses.dataclass
class Request:
    id: int
    arrival: float          # seconds after the stream starts
    geom: Geometry
    b: torch.Tensor         # FP32 projections on the server's device
    solver: str = "cgls"
    n_iter: int = 20
    lam: float = 0.0
    vec_dtype: torch.dtype = torch.float32


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    x: torch.Tensor | None
    history: torch.Tensor | None
    cancelled: bool = False
    rejected: bool = False   # needs more memory than the whole budget, or its plan failed
    error: str | None = None  # why the plan failed (a rejected request only)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req: Request, plan: Plan, state, stream, nbytes: int, admitted: float):
        self.req, self.plan, self.state, self.stream = req, plan, state, stream
        self.nbytes, self.admitted = nbytes, admitted
        self.events: deque = deque()  # one per enqueued step not yet seen complete
        self.enqueued = 0
        self.fifo_slot = False  # admitted to the first-come first-served slot ("mixed")

    def drain(self) -> None:
        """Forget the steps the device has finished."""
        while self.events and self.events[0].query():
            self.events.popleft()


def request_work(req: Request) -> int:
    """Ray-iterations of a request: the size of its projector calls."""
    return req.n_iter * req.geom.n_rays


def request_bytes(plan: Plan, req: Request) -> int:
    """Device bytes a request holds while active."""
    ws = plan.workspace_bytes(req.solver, req.n_iter, req.lam, req.vec_dtype)
    x = req.geom.n_voxels * 4
    hist = max(req.n_iter, 1) * KCT_HIST_COLS * 8
    return ws + x + hist + plan.device_bytes()


class Server:
    def __init__(self, budget_bytes: float = 200e9, device: int = 0, max_active: int = 3,
                 keep_results: bool = True, verbose: bool = False, policy: str = "mixed", depth: int = 2,
                 filler_frac: float = 0.5):
        if policy not in ("fifo", "sjf", "mixed"):
            raise ValueError(policy)
        if depth < 1:
            raise ValueError("depth must be at least 1")
        self.policy = policy
        self.depth = depth
        self.filler_frac = filler_frac
        self.budget = int(budget_bytes)
        self.device = torch.device("cuda", device)
        self.max_active = max_active
        self.keep_results = keep_results
        self.verbose = verbose
        self.log = []
        self.fifo_log: list[int] = []  # ids admitted to the first-come slot ("mixed"), in order
        self._cancel: set[int] = set()

    def cancel(self, req_id: int) -> None:
        """Cancel a request (queued or active); safe to call while ``run`` serves."""
        self._cancel.add(req_id)

    def run(self, requests: list[Request], cancel_after: dict[int, int] | None = None) -> list[Result]:
        """Serve `requests` (sorted by arrival) in real time; returns results by id.

        ``cancel_after`` maps a request id to an iteration count: the request
        is cancelled once that many of its iterations are enqueued (a
        deterministic trigger for ``cancel``)."""
        from concurrent.futures import ThreadPoolExecutor

        cancel_after = dict(cancel_after or {})
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque[Request] = deque()
        plans: dict = {}  # request id -> Future of its Plan, made by the worker thread
        active: list[_Active] = []
        used = 0
        results: dict[int, Result] = {}
        dev = self.device.index

        def make_plan(geom):
            with torch.cuda.device(dev):
                return Plan(geom, dev)

        t0 = time.perf_counter()
        with torch.cuda.device(self.device), ThreadPoolExecutor(max_workers=1) as worker:
            while pending or queue or active:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    req = pending.popleft()
                    queue.append(req)
                    plans[req.id] = worker.submit(make_plan, req.geom)
                # Cancelled requests still waiting leave at once.
                if any(q.id in self._cancel for q in queue):
                    keep: deque[Request] = deque()
                    for req in queue:
                        if req.id in self._cancel:
                            results[req.id] = Result(req.id, req.arrival, now, now, None, None, cancelled=True)
                            fut = plans.pop(req.id)
                            if fut.exception() is None:
                                fut.result().close()
                            self.log.append(("cancel", req.id, now, used))
                        else:
                            keep.append(req)
                    queue = keep
                # Admission while the next request fits the budget: the head
                # of the queue (FIFO) or the least work (SJF, ties by arrival),
                # once its plan is ready.
                while queue and len(active) < self.max_active:
                    head = next((a for a in active if a.fifo_slot), None)
                    fifo_turn = self.policy == "fifo" or (self.policy == "mixed" and head is None)
                    i = 0 if fifo_turn else min(range(len(queue)), key=lambda k: request_work(queue[k]))
                    if (self.policy == "mixed" and not fifo_turn and
                            request_work(queue[i]) > self.filler_frac * request_work(head.req)):
                        break
                    req = queue[i]
                    if not plans[req.id].done():
                        break
                    exc = plans[req.id].exception()
                    if exc is not None:  # e.g. an invalid geometry: the request alone fails
                        del queue[i]
                        plans.pop(req.id)
                        t = time.perf_counter() - t0
                        results[req.id] = Result(req.id, req.arrival, t, t, None, None, rejected=True, error=str(exc))
                        self.log.append(("error", req.id, t, used))
                        continue
                    plan = plans[req.id].result()
                    need = request_bytes(plan, req)
                    if need > self.budget:
                        del queue[i]
                        plans.pop(req.id)
                        plan.close()
                        t = time.perf_counter() - t0
                        results[req.id] = Result(req.id, req.arrival, t, t, None, None, rejected=True)
                        self.log.append(("reject", req.id, t, used))
                        continue
                    if used + need > self.budget:
                        break
                    del queue[i]
                    plans.pop(req.id)
                    stream = torch.cuda.Stream(device=self.device)
                    state = plan.state(req.b, req.solver, req.n_iter, req.lam, req.vec_dtype, stream=stream)
                    used += need
                    a = _Active(req, plan, state, stream, need, time.perf_counter() - t0)
                    a.fifo_slot = self.policy == "mixed" and fifo_turn
                    if a.fifo_slot:
                        self.fifo_log.append(req.id)
                    active.append(a)
                    self.log.append(("admit", req.id, a.admitted, used))
                # Keep up to `depth` iterations of every active request enqueued.
                progressed = False
                for a in active:
                    a.drain()
                    if cancel_after.get(a.req.id, -1) == a.enqueued:
                        self._cancel.add(a.req.id)
                    if a.req.id in self._cancel:
                        continue
                    while 0 <= a.enqueued < a.req.n_iter and len(a.events) < self.depth:
                        a.state.step(1)
                        a.enqueued += 1
                        ev = torch.cuda.Event()
                        ev.record(a.stream)
                        a.events.append(ev)
                        progressed = True
                        if cancel_after.get(a.req.id, -1) == a.enqueued:
                            self._cancel.add(a.req.id)
                            break
                    if a.enqueued == 0 and a.req.n_iter == 0:
                        a.state.step(0)
                        ev = torch.cuda.Event()
                        ev.record(a.stream)
                        a.events.append(ev)
                        a.enqueued = -1
                        progressed = True
                # Retire requests whose last iteration has completed.
                still = []
                for a in active:
                    cancelled = a.req.id in self._cancel
                    done_enq = a.enqueued == a.req.n_iter or a.enqueued == -1 or cancelled
                    if done_enq and not a.events:
                        fin = time.perf_counter() - t0
                        keep = self.keep_results and not cancelled
                        x = a.state.x if keep else None
                        h = a.state.history if keep else None
                        results[a.req.id] = Result(a.req.id, a.req.arrival, a.admitted, fin, x, h, cancelled)
                        a.stream.synchronize()  # the workspace is returned only once idle
                        a.state.close()
                        a.plan.close()
                        used -= a.nbytes
                        self.log.append(("cancel" if cancelled else "finish", a.req.id, fin, used))
                        if self.verbose and (len(results) % 8 == 0 or len(results) == len(requests)):
                            print(f"[serve] batched: {len(results)}/{len(requests)} done at {fin:.1f} s",
                                  file=sys.stderr, flush=True)
                    else:
                        still.append(a)
                active = still
                if not progressed:
                    if not active and not queue and pending:
                        time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                    else:
                        time.sleep(0.0001)
            for f in plans.values():  # plans of requests that never ran (cancelled while queued)
                f.result().close()
        return [results[r.id] for r in sorted(requests, key=lambda r: r.id)]


def serve_serial(requests: list[Request], device: int = 0, keep_results: bool = True,
                 verbose: bool = False) -> list[Result]:
    """Plain per-request path: each request solved alone with kct_solve in
    arrival order; latency includes waiting behind earlier requests."""
    dev = torch.device("cuda", device)
    out = {}
    t0 = time.perf_counter()
    with torch.cuda.device(dev):
        for req in sorted(requests, key=lambda r: r.arrival):
            now = time.perf_counter() - t0
            if req.arrival > now:
                time.sleep(req.arrival - now)
            start = time.perf_counter() - t0
            plan = Plan(req.geom, device)
            x, h = plan.solve(req.b, req.solver, req.n_iter, req.lam, req.vec_dtype)
            torch.cuda.synchronize()
            fin = time.perf_counter() - t0
            out[req.id] = Result(req.id, req.arrival, start, fin, x if keep_results else None,
                                 h if keep_results else None)
            plan.close()
            if verbose and (len(out) % 8 == 0 or len(out) == len(requests)):
                print(f"[serve] serial: {len(out)}/{len(requests)} done at {fin:.1f} s", file=sys.stderr, flush=True)
    return [out[r.id] for r in sorted(requests, key=lambda r: r.id)]


def percentile(values, q):
    """Nearest-rank percentile."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, int(math.ceil(q / 100.0 * len(v))))
    return v[k - 1]


def summarize(results: list[Result], rate: float | None = None) -> dict:
    """Latency percentiles and throughput of the served requests.  With the
    arrival ``rate``, also the offered load rho = rate x mean service time,
    the service time being admission to completion (for the serial path, a
    request's solve alone on the GPU)."""
    results = [r for r in results if not r.cancelled and not r.rejected]
    lat = [r.latency for r in results]
    makespan = max(r.finished for r in results) - min(r.arrival for r in results)
    out = {"n": len(results), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
           "mean_s": float(np.mean(lat)), "throughput_req_per_s": len(results) / makespan,
           "makespan_s": makespan}
    if rate is not None:
        out["offered_load_rho"] = rate * float(np.mean([r.finished - r.admitted for r in results]))
    return out


def stream_specs(n=64, rate=2.0, seed=5, size_scale=1.0, det_scale=None, angle_scale=None):
    """The seeded request stream of synth.serve_stream, shrunk by the scales:
    per request a dict with its id, arrival, geometry dict, solver, iteration
    count and the seed and ellipsoid count of its phantom."""
    import synth

    det_scale = size_scale if det_scale is None else det_scale
    angle_scale = size_scale if angle_scale is None else angle_scale
    out = []
    for r in synth.serve_stream(n, rate, seed):
        g = dict(r["geom"])
        n_vox = max(8, int(round(g["nx"] * size_scale)))
        side = max(8, 2 * int(round(g["nu"] * det_scale / 2)))
        na = max(4, int(round(g["n_angles"] * angle_scale)))
        pitch = 1.1 * n_vox * 0.5 * (g["dsd"] / g["dso"]) / side
        g.update(nx=n_vox, ny=n_vox, nz=n_vox, nu=side, nv=side, du=pitch, dv=pitch, n_angles=na)
        out.append(dict(r, geom=synth.geometry(g)))
    return out


def request_phantom(spec) -> np.ndarray:
    """The random ellipsoid phantom of one request (attenuation 0.01-0.05 per
    mm, i.e. 0.1-0.5 per cm)."""
    import synth

    gd = spec["geom"]
    return synth.ellipsoid_phantom(gd, spec["n_ellipsoids"], (2.0, 12.0 * gd["nx"] / 128), (0.01, 0.05),
                                   spec["seed"])


def make_requests(n=64, rate=2.0, seed=5, size_scale=1.0, device=0, det_scale=None, angle_scale=None):
    """The seeded request stream (``stream_specs``), with projections of each
    request's phantom made on the GPU (forward projection, Poisson noise at
    I0 = 1e5)."""
    import synth

    dev = torch.device("cuda", device)
    reqs = []
    for r in stream_specs(n, rate, seed, size_scale, det_scale, angle_scale):
        geom = Geometry.from_dict(r["geom"])
        plan = Plan(geom, device)
        b, _ = synth.add_noise_torch(plan.forward(torch.from_numpy(request_phantom(r)).to(dev)),
                                     dict(kind="poisson", i0=1.0e5), r["seed"])
        plan.close()
        reqs.append(Request(r["id"], r["arrival"], geom, b, r["solver"], r["n_iter"]))
        if len(reqs) % 8 == 0:
            print(f"[serve] generated {len(reqs)}/{n} requests", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return reqs


def main(argv=None):
    ap = argparse.ArgumentParser(description="continuous-batching server vs serial per-request path")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--size-scale", type=float, default=1.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-active", type=int, default=3)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--sjf", action="store_true", help="also serve the stream with shortest-job-first admission")
    ap.add_argument("--policy", default="mixed", choices=("fifo", "sjf", "mixed"), help="admission of the batched run")
    args = ap.parse_args(argv)
    print("[serve] generating requests", file=sys.stderr, flush=True)
    reqs = make_requests(args.requests, args.rate, size_scale=args.size_scale)
    work = sum(r.n_iter * r.geom.n_rays for r in reqs)
    print(f"[serve] {len(reqs)} requests, {work / 1e9:.1f} G ray-iterations", file=sys.stderr, flush=True)
    srv = Server(args.budget_gb * 1e9, max_active=args.max_active, keep_results=False, verbose=True,
                 policy=args.policy)
    res = srv.run(reqs)
    out = {"batched": summarize(res)}
    print(f"[serve] batched {out['batched']}", file=sys.stderr, flush=True)
    if args.sjf:
        sjf = Server(args.budget_gb * 1e9, max_active=16, keep_results=False, verbose=True,
                     policy="sjf").run(reqs)
        out["batched_sjf"] = summarize(sjf)
        print(f"[serve] batched, shortest job first {out['batched_sjf']}", file=sys.stderr, flush=True)
    if not args.no_serial:
        ser = serve_serial(reqs, keep_results=False, verbose=True)
        out["serial"] = summarize(ser)
        print(f"[serve] serial {out['serial']}", file=sys.stderr, flush=True)
    out["config"] = {"requests": args.requests, "rate_per_s": args.rate, "size_scale": args.size_scale,
                     "budget_gb": args.budget_gb, "max_active": args.max_active}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
