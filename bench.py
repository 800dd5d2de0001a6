"""Benchmark of the EBIT interface step on one MI355X.

Headline (the `value` of the JSON line): 8192 x 8192 FP64 grid, 2000 seeded
non-overlapping circles (radii uniform in [4, 32] cells), single-vortex face
velocity with period T = 4 at CFL 0.5 (dt = h/2, time factor cos(pi t / T)
folded into dt). One step is the whole hot path: ebit_advect (x and y sweeps
with circle fit, Color Vertex update and topology change) followed by
ebit_fraction_curvature. The sweep and fit workgroups per CU of its launch
schedule are tuned first on the same grid (paper_2309_00338_amd/tune.py),
outside the timed region; the fraction pass keeps its default split.

The same line carries the rest of the metric:
  roofline / step_roofline: the dominant kernel (fraction + curvature, timed
      live with events on its stream) and the whole step against HBM peak;
  batched: 256 independent grids (N log-uniform in [64, 1024], 1-20 circles or
      ellipses, own vortex period each) as one HIP graph of K steps, as eager
      batched launches, and as a loop of plain per-grid calls;
  served: a Poisson stream of requests (200/s, N log-uniform in [128, 2048],
      steady random fields, 16-256 steps each) through the pool, with
      arrival-to-result latency percentiles, against a plain per-request loop;
  film: the two-markers-per-edge step on the topology-change workload (500
      merging circle pairs on 4096^2, rupture gap 0.05 cells) against the
      one-marker step on the same grid and flow;
  cpu_baseline: the CPU oracle timed on a bounded sample of the headline grid.

--workload single|batched|served|film runs one part alone (its own JSON line).
"""
import argparse
import collections
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


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


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
    model, avail = host_cpu()
    return {"value": st.nx * st.ny * nsteps / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cores_available": avail,
            "sample": f"{nsteps} full step(s) (advect + fraction + curvature) of the same {st.nx}x{st.ny} "
                      f"workload from its initial state, single-threaded C on one core, {el:.1f} s"}


# ---------------------------------------------------------------------------
# headline: one large grid
# ---------------------------------------------------------------------------
def run_single(args):
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I
    from paper_2309_00338_amd import tune

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

    # launch schedule: tuned on this grid, then the grid is reset to its start
    tuned = None
    if not args.no_tune:
        k = [0]

        def tstep():
            g.advect(u, v, w.dts[k[0] % len(w.dts)])
            g.fraction_curvature(C, K)
            k[0] += 1

        # the fraction pass's split stays at its default, so that the profile of
        # the dominant kernel (taken without tuning) times the same schedule
        best, info = tune.tune(g, tstep, stream, fields=("sweep_per_cu", "fit_per_cu"), steps=4, reps=2)
        tuned = {"schedule": best, "us_per_step": info["us_per_step"],
                 "candidates_us": info["table"], "method": "coordinate descent, best of 2 x 4 steps each"}
        g.sync()
        g.set_state(w.state)
        log(f"[bench] tuned schedule {best}")

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
        "schedule": g.get_schedule(),
        "tuning": tuned,
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
    g.close()
    del g, u, v, C, K, rho, mu, fx, fy
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on two steps of the same grid")
        out["cpu_baseline"] = cpu_baseline(w, 2)
    return out


# ---------------------------------------------------------------------------
# two markers per edge
# ---------------------------------------------------------------------------
def film_state_bytes(nx, ny):
    """Bytes of one dense copy of the two-marker state: node and centre colours
    (1 B each), and per H and V edge a count (1 B) and an offset pair (16 B)."""
    nodes, cells, edges = (nx + 1) * (ny + 1), nx * ny, (ny + 1) * nx + ny * (nx + 1)
    return {"write": nodes + cells + 17 * edges, "read_dense": nodes + cells + edges, "cells": cells}


def run_film(args):
    """The two-markers-per-edge step (include/ebit_film.h) on the topology-change
    workload: 500 circle pairs driven into each other on 4096^2, rupture gap
    delta = 0.05 cells, so the meeting walls form films that thin and rupture.
    Timed with events on the handle's stream (advect + fraction per step),
    beside the one-marker step (advect + fraction) on the same grid and flow."""
    import torch

    from paper_2309_00338_amd import ebit, film
    from paper_2309_00338_amd import inputs as I

    n, steps, warmup = args.film_n, args.film_steps, 2
    t0 = time.perf_counter()
    w = I.merging_pairs(n=n, pairs=args.film_pairs, nsteps=warmup + steps)
    fs = film.FilmState.of(w.state)
    log(f"[bench] film: {w.meta['pairs']} pairs on {n}^2 generated in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    u = torch.from_numpy(w.u).to(dev)
    v = torch.from_numpy(w.v).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)

    def timed(stream, adv, frac):
        for k in range(warmup):
            adv(w.dts[k])
            frac()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(steps):
            adv(w.dts[warmup + k])
            frac()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / steps

    f = film.EbitFilm(fs, delta=args.film_delta, device=dev)
    film_us = timed(f.stream, lambda dt: f.advect(u, v, dt), lambda: f.fraction(C))
    assert f.sync() == 0
    fst = f.stats()
    f.close()
    del f
    torch.cuda.empty_cache()
    g = ebit.EbitGrid(w.state, device=dev)
    one_us = timed(g.stream, lambda dt: g.advect(u, v, dt), lambda: g.fraction(C))
    g.sync()
    g.close()
    del g
    torch.cuda.empty_cache()
    sb = film_state_bytes(n, n)
    # per sweep: the new copy written in full, the old colours and counts read in
    # full (offsets and velocities only at markers: not counted); the fraction
    # reads the colours and counts and writes C
    step_bytes = 2 * (sb["write"] + sb["read_dense"]) + sb["read_dense"] + 8 * sb["cells"]
    cells = sb["cells"]
    log(f"[bench] film: {film_us:.1f} us/step (one marker per edge: {one_us:.1f})")
    return {
        "workload": f"two markers per edge: merging pairs {n}x{n} FP64, {w.meta['pairs']} pairs R~U[8,24] cells, "
                    f"gap U[0.5,2], u=+-0.5 per pair plus shear, CFL 0.5, rupture gap {args.film_delta:g} cells",
        "grid": [n, n], "steps": steps, "warmup": warmup, "delta": args.film_delta,
        "us_per_step": film_us, "cell_steps_per_s": cells / (film_us * 1e-6),
        "roofline": {"bound": "hbm", "kernel": "whole film step (10 sweep passes + fraction), dense state",
                     "achieved": step_bytes / (film_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": step_bytes / (film_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "alg_bytes_per_step": step_bytes},
        "one_marker": {"us_per_step": one_us, "cell_steps_per_s": cells / (one_us * 1e-6),
                       "what": "ebit_advect + ebit_fraction on the same grid and flow (tiled one-marker step)"},
        "counters": fst,
    }


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
def run_batched(args, steps, warmup):
    """The batched form (graph of K steps and eager launches) against a loop of
    plain per-grid calls, same grids and steps."""
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I
    from paper_2309_00338_amd import tune

    steps += steps & 1  # the graph needs an even count
    t0 = time.perf_counter()
    nsteps = warmup + steps
    inst = I.batched_instances(count=args.grids, steps=nsteps)
    cells = sum(st.nx * st.ny for st, _, _, _ in inst)
    log(f"[bench] batched: {len(inst)} grids, {cells:.3e} cells, generated in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    states = [st for st, _, _, _ in inst]
    dts = torch.tensor([[d[k] for _, _, _, d in inst] for k in range(nsteps)], dtype=torch.float64, device=dev)

    def timed(stream, fn, n):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / n  # us per step

    # tune the batch's schedule on a scratch batch
    tb = ebit.EbitBatch(states, device=dev)
    U, V = tb.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    C, K = tb.new_fields()
    kk = [0]

    def tstep():
        tb.advect(U, V, dts[kk[0] % nsteps])
        tb.fraction_curvature(C, K)
        kk[0] += 1

    sched = None
    if not args.no_tune:
        sched, _ = tune.tune(tb, tstep, tb.stream, fields=tune.SEVERAL, steps=2, reps=1)
    tb.close()
    del tb

    # eager batched launches
    b = ebit.EbitBatch(states, device=dev)
    if sched:
        b.set_schedule(sched)
    for k in range(warmup):
        b.advect(U, V, dts[k])
        b.fraction_curvature(C, K)

    def eager():
        for k in range(warmup, nsteps):
            b.advect(U, V, dts[k])
            b.fraction_curvature(C, K)

    us_eager = timed(b.stream, eager, steps)
    if any(b.sync()):
        raise RuntimeError("batched run reported device errors")
    b.close()
    del b

    # the same steps as one captured graph (on a stream of its own)
    gs = torch.cuda.Stream(device=dev)
    b = ebit.EbitBatch(states, device=dev, stream=gs)
    if sched:
        b.set_schedule(sched)
    for k in range(warmup):
        b.advect(U, V, dts[k])
        b.fraction_curvature(C, K)
    graph = b.capture(steps, U, V, dts[warmup:].contiguous(), C, K)
    us_graph = timed(gs, graph.launch, steps)
    if any(b.sync()):
        raise RuntimeError("graph replay reported device errors")
    graph.close()
    b.close()
    del b, U, V, C, K
    torch.cuda.empty_cache()
    log(f"[bench] batched: graph {us_graph:.1f} us/step, eager {us_eager:.1f} us/step")

    # plain loop of per-grid handles on one stream
    grids = [ebit.EbitGrid(st, device=dev) for st in states]
    vel = [(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)) for _, u, v, _ in inst]
    fields = [(g.new_field(), g.new_field()) for g in grids]
    hd = [d for _, _, _, d in inst]
    for k in range(warmup):
        for g, (u, v), d, (c, kf) in zip(grids, vel, hd, fields):
            g.advect(u, v, d[k])
            g.fraction_curvature(c, kf)

    def plain():
        for k in range(warmup, nsteps):
            for g, (u, v), d, (c, kf) in zip(grids, vel, hd, fields):
                g.advect(u, v, d[k])
                g.fraction_curvature(c, kf)

    us_plain = timed(grids[0].stream, plain, steps)
    for g in grids:
        g.sync()
        g.close()
    del grids, vel, fields
    torch.cuda.empty_cache()
    log(f"[bench] batched: plain per-grid loop {us_plain:.1f} us/step")
    return {
        "workload": f"batched: {len(inst)} grids, N log-uniform in [64,1024], 1-20 circles/ellipses, "
                    f"single vortex T~U[1,8], CFL 0.5, seed 1004",
        "grids": len(inst), "cells": cells, "steps": steps, "warmup": warmup,
        "graph": {"us_per_step": us_graph, "cell_steps_per_s": cells / (us_graph * 1e-6),
                  "what": f"ebit_batch_capture of {steps} steps, one ebit_graph_launch"},
        "eager": {"us_per_step": us_eager, "cell_steps_per_s": cells / (us_eager * 1e-6),
                  "what": "ebit_batch_advect + ebit_batch_fraction_curvature per step"},
        "plain": {"us_per_step": us_plain, "cell_steps_per_s": cells / (us_plain * 1e-6),
                  "what": "one ebit_advect + ebit_fraction_curvature per grid per step, one stream"},
        "graph_vs_plain": us_plain / us_graph, "eager_vs_plain": us_plain / us_eager,
        "schedule": sched,
    }


# ---------------------------------------------------------------------------
# served form
# ---------------------------------------------------------------------------
def _make_request(req):
    """Worker: one request's instance as plain arrays (generation is the
    client's work, done before the clock starts)."""
    from paper_2309_00338_amd import inputs as I

    st, u, v, dt = I.served_instance(req)
    return {"id": req["id"], "arrival": req["arrival"], "steps": req["steps"], "nx": st.nx, "ny": st.ny,
            "h": st.h, "c": st.c, "cc": st.cc, "hoff": st.hoff, "voff": st.voff, "u": u, "v": v, "dt": dt}


def generate_requests(args, seconds):
    """The request stream, generated by worker processes before anything
    touches the GPU (they run numpy only)."""
    from concurrent.futures import ProcessPoolExecutor

    from paper_2309_00338_amd import inputs as I

    count = max(1, int(round(seconds * args.rate)))
    t0 = time.perf_counter()
    reqs = list(I.served_requests(count, rate=args.rate))
    workers = max(1, min(16, len(os.sched_getaffinity(0))) - 1)
    if workers <= 1:
        out = [_make_request(r) for r in reqs]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            out = list(ex.map(_make_request, reqs, chunksize=4))
    log(f"[bench] served: {count} requests generated in {time.perf_counter() - t0:.1f}s ({workers} workers)")
    return out


def run_served(args, seconds, plain_count, reqs):
    """The pool serving a Poisson request stream, clock = wall time from the
    first arrival's origin (requests were generated beforehand). Admission,
    stepping, retirement and status polling are all asynchronous: the host
    enqueues, and a request's completion time is the GPU timestamp of the
    event after the step that finished it (its fields are then in HBM), on the
    same origin as the arrival times. The same requests (a prefix of them)
    then run through a plain per-request loop for comparison."""
    import numpy as np
    import torch

    from paper_2309_00338_amd import ebit

    count = len(reqs)
    t0 = time.perf_counter()
    for r in reqs:  # pinned host memory: the admission uploads overlap the GPU's work
        for k in ("c", "cc", "hoff", "voff", "u", "v"):
            r[k] = torch.from_numpy(np.ascontiguousarray(r[k])).pin_memory()
    offered = sum(r["nx"] * r["ny"] * r["steps"] for r in reqs)
    log(f"[bench] served: {count} requests pinned in {time.perf_counter() - t0:.1f}s")

    dev = torch.device("cuda:0")
    free, _ = torch.cuda.mem_get_info(dev)
    arena = int(min(free * 0.5, 96 << 30))
    max_grids = 256
    pool = ebit.EbitPool(max_grids=max_grids, max_tiles=args.pool_tiles, arena_bytes=arena, device=dev)
    stream = pool.stream
    status_dev = torch.empty(max_grids, dtype=torch.int32, device=dev)
    ring = [torch.empty(max_grids, dtype=torch.int32).pin_memory() for _ in range(64)]
    ref = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ref.record(stream)
    live = {}  # slot -> [request, steps left]
    inflight = collections.deque()  # (event, finished [(request, slot)], status buffer or None)
    lat, cell_steps, pool_steps, nxt, depth_waits = [], 0, 0, 0, 0
    gpu_end = 0.0
    ring_i = 0

    def reap(block):
        nonlocal gpu_end
        while inflight and (block or inflight[0][0].query()):
            ev, done, sbuf = inflight.popleft()
            ev.synchronize()
            t_done = ref.elapsed_time(ev) * 1e-3
            gpu_end = max(gpu_end, t_done)
            for req, slot in done:
                if int(sbuf[slot]) != 0:
                    raise RuntimeError(f"request {req['id']} failed with status {int(sbuf[slot])}")
                lat.append(t_done - req["arrival"])
            block = False

    while nxt < count or live or inflight:
        now = time.perf_counter() - wall0
        while nxt < count and reqs[nxt]["arrival"] <= now:
            r = reqs[nxt]
            slot = pool.admit(r, r["u"], r["v"], r["dt"])
            if slot is None:
                break
            live[slot] = [r, r["steps"]]
            nxt += 1
        if live:
            pool.step()
            pool_steps += 1
            done = []
            for slot, ent in list(live.items()):
                cell_steps += ent[0]["nx"] * ent[0]["ny"]
                ent[1] -= 1
                if ent[1] == 0:
                    done.append((ent[0], slot))
                    del live[slot]
            sbuf = None
            if done:
                pool.status(status_dev)
                sbuf = ring[ring_i % len(ring)]
                ring_i += 1
                sbuf.copy_(status_dev, non_blocking=True)
                for _, slot in done:
                    pool.retire(slot)  # enqueued after the status copy: the slot is free for later admissions
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            inflight.append((ev, done, sbuf))
            # keep the host a few steps ahead of the GPU, no more (the status ring is finite)
            if len(inflight) > 8:
                depth_waits += 1
                reap(True)
        elif nxt < count:
            time.sleep(max(0.0, min(reqs[nxt]["arrival"] - (time.perf_counter() - wall0), 0.01)))
        reap(False)
    torch.cuda.synchronize()
    span = max(gpu_end, time.perf_counter() - wall0)
    pool.close()
    lat_ms = np.array(lat) * 1e3
    log(f"[bench] served: {len(lat)} requests, {pool_steps} pool steps, {span:.2f} s, "
        f"p50 {np.percentile(lat_ms, 50):.1f} ms p99 {np.percentile(lat_ms, 99):.1f} ms")

    # plain per-request loop over the first requests, one after the other
    sub = reqs[:plain_count]
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    plain_cells = 0
    from paper_2309_00338_amd.inputs import State

    for r in sub:
        st = State(r["nx"], r["ny"], r["h"], r["c"].numpy(), r["cc"].numpy(), r["hoff"].numpy(), r["voff"].numpy())
        g = ebit.EbitGrid(st, device=dev)
        u, v = r["u"].to(dev), r["v"].to(dev)
        Cp, Kp = g.new_field(), g.new_field()
        for _ in range(r["steps"]):
            g.advect(u, v, r["dt"])
            g.fraction_curvature(Cp, Kp)
        g.sync()
        g.close()
        plain_cells += r["nx"] * r["ny"] * r["steps"]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - p0
    sub_served = sum(r["nx"] * r["ny"] * r["steps"] for r in sub)
    assert sub_served == plain_cells
    log(f"[bench] served: plain loop over {len(sub)} requests {plain_s:.2f} s")
    return {
        "workload": f"served: Poisson {args.rate:g}/s for {seconds:g} s of arrivals, N log-uniform in [128,2048], "
                    f"1-50 circles, steady 4-mode fields, 16-256 steps, seed 1005",
        "requests": len(lat), "pool_steps": pool_steps, "span_s": span,
        "cell_steps_per_s": cell_steps / span,
        "offered_cell_steps_per_s": offered / max(reqs[-1]["arrival"], 1e-9),
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "host_waits_on_gpu": depth_waits,
        "plain": {"requests": len(sub), "cell_steps_per_s": plain_cells / plain_s, "seconds": plain_s,
                  "what": "per request: ebit_create, then its steps of ebit_advect + ebit_fraction_curvature, "
                          "one request after the other, no arrival waits"},
        "served_vs_plain": (cell_steps / span) / (plain_cells / plain_s),
        "what": "cell-steps delivered / span from the first arrival's origin to the last result; latency = "
                "arrival to the GPU end of the step completing the request (fields in HBM)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--circles", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the device-default launch schedule")
    ap.add_argument("--workload", choices=("all", "single", "batched", "served", "film"), default="all")
    ap.add_argument("--grids", type=int, default=256, help="batched: number of grids")
    ap.add_argument("--batched-steps", type=int, default=8, help="batched: timed steps inside the full line")
    ap.add_argument("--served-seconds", type=float, default=1.5, help="served: seconds of arrivals")
    ap.add_argument("--plain-requests", type=int, default=60, help="served: requests of the plain loop")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--pool-tiles", type=int, default=1 << 18, help="served: tile capacity of the pool")
    ap.add_argument("--film-n", type=int, default=4096, help="film: grid size")
    ap.add_argument("--film-pairs", type=int, default=500, help="film: circle pairs")
    ap.add_argument("--film-steps", type=int, default=8, help="film: timed steps")
    ap.add_argument("--film-delta", type=float, default=0.05, help="film: rupture gap in cells")
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
        print(json.dumps({"error": "the benchmark drives one GPU (one process per GPU); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    def line(part, d, steps, warmup, ms, value):
        return {"metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": steps,
                "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                "config": {"workload": d["workload"]}, part: d}

    if args.workload == "batched":
        d = run_batched(args, args.steps, args.warmup)
        print(json.dumps(line("batched", d, d["steps"], args.warmup, d["graph"]["us_per_step"] * 1e-3,
                              d["graph"]["cell_steps_per_s"])), flush=True)
        return
    if args.workload == "film":
        d = run_film(args)
        print(json.dumps(line("film", d, d["steps"], d["warmup"], d["us_per_step"] * 1e-3, d["cell_steps_per_s"])),
              flush=True)
        return
    reqs = generate_requests(args, args.served_seconds) if args.workload in ("all", "served") else None
    if args.workload == "served":
        d = run_served(args, args.served_seconds, args.plain_requests, reqs)
        print(json.dumps(line("served", d, d["pool_steps"], 0, d["span_s"] / max(d["pool_steps"], 1) * 1e3,
                              d["cell_steps_per_s"])), flush=True)
        return
    out = run_single(args)
    if args.workload == "all":
        out["batched"] = run_batched(args, args.batched_steps, 2)
        out["served"] = run_served(args, args.served_seconds, args.plain_requests, reqs)
        out["film"] = run_film(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
