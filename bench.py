"""Benchmark of the EBIT interface step on one MI355X.

Default workload (the headline line): 8192 x 8192 FP64 grid, 2000 seeded
non-overlapping circles (radii uniform in [4, 32] cells), single-vortex face
velocity with period T = 4 at CFL 0.5 (dt = h/2, time factor cos(pi t / T)
folded into dt). One step is the whole hot path: ebit_advect (x and y sweeps
with circle fit, Color Vertex update and topology change) followed by
ebit_fraction_curvature.

Prints one JSON line: throughput in cell-steps/s over the timed steps (state
and velocities already resident in HBM), the roofline of the dominant kernel
(fraction + curvature, timed live with events on its stream), the whole-step
algorithmic-bytes roofline, and the CPU oracle timed on a bounded sample.

--workload batched: 256 independent grids (N log-uniform in [64, 1024], 1-20
circles or ellipses, own vortex period each) advanced by the batched entry
points, against a loop of per-grid handles on one stream.
--workload served: a pool serving a Poisson stream of requests (200/s, N
log-uniform in [128, 2048], steady random fields, 16-256 steps each); reports
cell-steps/s and the arrival-to-result latency percentiles.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "EBIT cell-steps/s + % HBM roofline; batched/served vs plain; p50/p99 latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_from_profile(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{n}.json")
    if not os.path.exists(path):
        return None
    try:
        import hashlib

        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2309_00338_amd", "csrc", "ebit_kernels.hip"), "rb").read()
        if rec.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(w, nsteps=1):
    """The oracle (single-threaded C) on the same grid: nsteps full steps."""
    import oracle

    st = w.state.copy()
    t0 = time.perf_counter()
    for k in range(nsteps):
        rc, _ = oracle.step(st, w.u, w.v, w.dts[k])
        assert rc == oracle.OK
        C = oracle.fraction(st)
        oracle.curvature(st, C)
    el = time.perf_counter() - t0
    return {"value": st.nx * st.ny * nsteps / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} full step(s) (advect + fraction + curvature) of the same {st.nx}x{st.ny} "
                      f"workload from its initial state, single-threaded C, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--circles", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("single", "batched", "served"), default="single")
    ap.add_argument("--grids", type=int, default=256, help="batched: number of grids")
    ap.add_argument("--served-seconds", type=float, default=4.0, help="served: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--pool-tiles", type=int, default=1 << 18, help="served: tile capacity of the pool")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (a plain copy kernel of known size, "
                         "the reference for scaling hardware byte counters), then exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)

    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I

    t0 = time.perf_counter()
    period, cfl = 4.0, 0.5
    w = I.many_circles(n=args.n, count=args.circles, rmin=4.0, rmax=32.0, period=period, cfl=cfl,
                       nsteps=args.warmup + args.steps)
    n = w.state.nx
    log(f"[bench] generated {w.meta['circles']} circles on {n}^2, {w.state.n_markers()} markers "
        f"in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    g = ebit.EbitGrid(w.state, device=dev)
    u = torch.from_numpy(w.u).to(dev)
    v = torch.from_numpy(w.v).to(dev)
    C = g.new_field()
    K = g.new_field()
    stream = g.stream
    torch.cuda.synchronize()
    log(f"[bench] uploaded; workspace {g.ws.numel() / 2**30:.2f} GiB")

    for k in range(args.warmup):
        g.advect(u, v, w.dts[k])
        g.fraction_curvature(C, K)
    torch.cuda.synchronize()
    g.sync()
    g.stats_reset()
    torch.cuda.synchronize()
    log("[bench] warmup done")

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    fc = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        g.advect(u, v, w.dts[args.warmup + k])
        fc[k][0].record(stream)
        g.fraction_curvature(C, K)
        fc[k][1].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    g.sync()
    el_ms = start.elapsed_time(end)
    fc_ms = sum(a.elapsed_time(b) for a, b in fc) / args.steps
    st = g.stats()
    log(f"[bench] timed {args.steps} steps: {el_ms:.3f} ms; fraction+curvature {fc_ms * 1e3:.1f} us/launch")

    ncell = n * n
    ms_step = el_ms / args.steps
    value = ncell * args.steps / (el_ms * 1e-3)
    I_step = st["interfacial"] / args.steps
    M_sweeps = st["markers"] / args.steps  # markers at the start of both sweeps, per step
    # algorithmic bytes: dense C and kappa writes, band offsets read for the
    # polygons, node-colour bit per cell, 32 B per marker-sweep (offset read +
    # write, two face velocities)
    fc_bytes = 16.0 * ncell + 8.0 * I_step
    step_bytes = ncell * (16.0 + 1.0 / 8.0) + 32.0 * M_sweeps + 8.0 * I_step
    achieved = fc_bytes / (fc_ms * 1e-3) / 1e9
    traffic = traffic_from_profile("frac_curv", n)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large single grid: {n}x{n} FP64, {w.meta['circles']} circles R~U[4,32] cells, "
                               f"single vortex T={period:g}, CFL {cfl}",
                   "grid": [n, n], "circles": w.meta["circles"], "seed": w.meta["seed"],
                   "markers_per_step": M_sweeps / 2.0, "interfacial_per_step": I_step},
        # one ebit_fraction_curvature call: k_frac_curv<3> then k_ghf (the
        # parabola fits of the cells it left), timed together with events
        "roofline": {"bound": "hbm", "kernel": "k_frac_curv<3> + k_ghf (one ebit_fraction_curvature call)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "us_per_launch": fc_ms * 1e3, "alg_bytes_per_launch": fc_bytes},
        "step_roofline": {"alg_bytes_per_step": step_bytes, "achieved_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
                          "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "counters": st,
    }
    # consumers of C and kappa (not part of the step): rho, mu and the face forces
    rho, mu = g.new_field(), g.new_field()
    fx = torch.empty((n, n + 1), dtype=torch.float64, device=dev)
    fy = torch.empty((n + 1, n), dtype=torch.float64, device=dev)
    fl = (1000.0, 1.2, 1e-3, 1.8e-5, 0.07)
    g.ns_fields(C, K, *fl, rho=rho, mu=mu, fx=fx, fy=fy)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(8):
        g.ns_fields(C, K, *fl, rho=rho, mu=mu, fx=fx, fy=fy)
    e1.record(stream)
    torch.cuda.synchronize()
    ns_us = e0.elapsed_time(e1) / 8 * 1e3
    # algorithmic bytes: four dense outputs (2 cell fields, 2 face fields) + C and kappa of the band
    ns_bytes = 8.0 * (2 * ncell + 2 * n * (n + 1)) + 16.0 * I_step
    out["ns_fields"] = {"us_per_launch": ns_us, "alg_bytes_per_launch": ns_bytes,
                        "achieved_GBs": ns_bytes / (ns_us * 1e-6) / 1e9,
                        "frac": ns_bytes / (ns_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] ns_fields: {ns_us:.1f} us/launch")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on two steps of the same grid")
        out["cpu_baseline"] = cpu_baseline(w, 2)
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """Batched form against a loop of per-grid handles, same grids and steps."""
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I

    t0 = time.perf_counter()
    nsteps = args.warmup + args.steps
    inst = I.batched_instances(count=args.grids, steps=nsteps)
    cells = sum(st.nx * st.ny for st, _, _, _ in inst)
    log(f"[bench] generated {len(inst)} grids, {cells:.3e} cells in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    b = ebit.EbitBatch([st for st, _, _, _ in inst], device=dev)
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    dts = torch.tensor([[d[k] for _, _, _, d in inst] for k in range(nsteps)], dtype=torch.float64, device=dev)
    C, K = b.new_fields()
    stream = b.stream

    def timed(step_fn):
        for k in range(args.warmup):
            step_fn(k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.warmup, nsteps):
            step_fn(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    def batched_step(k):
        b.advect(U, V, dts[k])
        b.fraction_curvature(C, K)

    ms_b = timed(batched_step)
    st_b = b.sync()
    if any(st_b):
        raise RuntimeError(f"batched run reported device errors: {sorted(set(st_b))}")
    log(f"[bench] batched: {ms_b * 1e3:.1f} us/step")
    del b, U, V, C, K
    torch.cuda.empty_cache()

    grids = [ebit.EbitGrid(st, device=dev) for st, _, _, _ in inst]
    vel = [(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)) for _, u, v, _ in inst]
    fields = [g.new_field() for g in grids]
    kfields = [g.new_field() for g in grids]

    def plain_step(k):
        for g, (u, v), (_, _, _, d), c, kk in zip(grids, vel, inst, fields, kfields):
            g.advect(u, v, d[k])
            g.fraction_curvature(c, kk)

    ms_p = timed(plain_step)
    for g in grids:
        g.sync()
    log(f"[bench] plain loop: {ms_p * 1e3:.1f} us/step")
    out = {
        "metric": METRIC, "value": cells / (ms_b * 1e-3), "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched: {len(inst)} grids, N log-uniform in [64,1024], 1-20 circles/ellipses, "
                               f"single vortex T~U[1,8], CFL 0.5", "grids": len(inst), "cells": cells, "seed": 1004},
        "plain": {"value": cells / (ms_p * 1e-3), "ms_per_step": ms_p,
                  "what": "one ebit_advect + ebit_fraction_curvature per grid per step, one stream"},
        "batched_vs_plain": ms_p / ms_b,
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Pool serving a Poisson request stream. The clock is wall time minus the
    client's time spent building requests; a request's latency runs from its
    arrival to the end of the GPU step that completes it."""
    import collections

    import numpy as np
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I

    count = max(1, int(round(args.served_seconds * args.rate)))
    reqs = I.served_requests(count, rate=args.rate)
    dev = torch.device("cuda:0")
    free, total = torch.cuda.mem_get_info(dev)
    arena = int(min(free * 0.6, 96 << 30))
    pool = ebit.EbitPool(max_grids=256, max_tiles=args.pool_tiles, arena_bytes=arena, device=dev)
    stream = pool.stream
    gen_time = 0.0
    wall0 = time.perf_counter()

    def clock():
        return time.perf_counter() - wall0 - gen_time

    pending = collections.deque()
    nxt = None
    exhausted = False
    live = {}  # slot -> (request, cells)
    lat, cell_steps, steps_run = [], 0, 0
    offered, last_arrival = 0, 0.0
    skip = 0.0  # idle time skipped when nothing is live and the next arrival is in the future
    done_all = False
    while not done_all:
        # bring in every request that has arrived
        while True:
            if nxt is None and not exhausted:
                try:
                    t = time.perf_counter()
                    req = next(reqs)
                    req["inst"] = I.served_instance(req)
                    gen_time += time.perf_counter() - t
                    nxt = req
                except StopIteration:
                    exhausted = True
            if nxt is not None and nxt["arrival"] <= clock() + skip:
                pending.append(nxt)
                nxt = None
                continue
            break
        # admit in arrival order while the pool has room
        while pending:
            req = pending[0]
            st, u, v, dt = req["inst"]
            slot = pool.admit(st, u, v, dt)
            if slot is None:
                break
            pending.popleft()
            live[slot] = (req, st.nx * st.ny)
            offered += st.nx * st.ny * req["steps"]
            last_arrival = req["arrival"]
            req.pop("inst")
        if not live:
            if exhausted and not pending and nxt is None:
                done_all = True
                continue
            if nxt is not None:
                skip = max(skip, nxt["arrival"] - clock())
            continue
        pool.step()
        torch.cuda.synchronize()
        steps_run += 1
        now = clock() + skip
        for slot in list(live):
            req, cells = live[slot]
            cell_steps += cells
            req["done"] = req.get("done", 0) + 1
            if req["done"] >= req["steps"]:
                _, _, _, status = pool.read(slot, fields=False)
                if status:
                    raise RuntimeError(f"request {req['id']} failed with status {status}")
                lat.append(now - req["arrival"])
                pool.retire(slot)
                del live[slot]
    elapsed = clock() + skip
    busy = clock()
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC, "value": cell_steps / elapsed, "unit": "cell-steps/s", "n_gpus": 1, "steps": steps_run,
        "warmup": 0, "ms_per_step": busy / max(steps_run, 1) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"served: Poisson {args.rate:g}/s for {args.served_seconds:g} s, N log-uniform in "
                               f"[128,2048], 1-50 circles, steady 4-mode fields, 16-256 steps", "requests": count,
                   "seed": 1005},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "served": {"requests": len(lat), "cell_steps": cell_steps, "pool_steps": steps_run,
                   "offered_cell_steps_per_s": offered / max(last_arrival, 1e-9),
                   "busy_cell_steps_per_s": cell_steps / busy, "span_s": elapsed, "busy_s": busy,
                   "client_generation_s": gen_time,
                   "what": "value = cell-steps delivered / span (arrival clock); busy rate excludes idle gaps; "
                           "latency = arrival to the end of the step completing the request, fields in HBM"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
