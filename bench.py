"""Benchmark of the EBIT interface step on one MI355X.

Workload: 8192 x 8192 FP64 grid, 2000 seeded non-overlapping circles (radii
uniform in [4, 32] cells), single-vortex face velocity with period T = 4 at
CFL 0.5 (dt = h/2, time factor cos(pi t / T) folded into dt). One step is the
whole hot path: ebit_advect (x and y sweeps with circle fit, Color Vertex
update and topology change) followed by ebit_fraction_curvature.

Prints one JSON line: throughput in cell-steps/s over the timed steps (state
and velocities already resident in HBM), the roofline of the dominant kernel
(fraction + curvature, timed live with events on its stream), the whole-step
algorithmic-bytes roofline, and the CPU oracle timed on a bounded sample.
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
        "roofline": {"bound": "hbm", "kernel": "k_frac_curv<3> (ebit_fraction_curvature)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "us_per_launch": fc_ms * 1e3, "alg_bytes_per_launch": fc_bytes},
        "step_roofline": {"alg_bytes_per_step": step_bytes, "achieved_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
                          "frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "counters": st,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on one step of the same grid")
        out["cpu_baseline"] = cpu_baseline(w, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
