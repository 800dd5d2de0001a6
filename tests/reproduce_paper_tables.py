"""Reproduce the paper's kinematic tables with the GPU library.

Translation (Sec. 3.2, Table 1), single vortex T = 2 and T = 8 (Sec. 3.3,
Tables 3 and 4) and Zalesak's disk (Sec. 3.4, Table 5), circle fit (EBIT) and
straight line (EBIT-SL), at the paper's resolutions, through the C-ABI. Prints
one row per case with our E_area, E_shape and E_sym next to the published
values, and writes them as JSON when --out is given.

E_sym is estimated as sum |C(T) - C(0)| h^2, a lower bound of the area of the
symmetric difference of the two reconstructions. E_shape is not defined for
Zalesak's disk in the paper.

    python tests/reproduce_paper_tables.py [--nmax 512] [--out results.json]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))


def _markers_xy(st):
    hp = st.h_present()
    jj, ii = np.nonzero(hp)
    vp = st.v_present()
    jj2, ii2 = np.nonzero(vp)
    return (np.concatenate([ii + st.hoff[jj, ii], ii2.astype(np.float64)]),
            np.concatenate([jj.astype(np.float64), jj2 + st.voff[jj2, ii2]]))


def run_case(test, n, line, device):
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd import inputs as I

    if test == "translation":
        w = I.translation(n)
        centre = (0.25, 0.75)
    elif test == "zalesak":
        w = I.zalesak(n)
        centre = (0.5, 0.75)
    else:
        w = I.single_vortex(n, period=2.0 if test == "vortex_T2" else 8.0, cfl=0.125)
        centre = (0.5, 0.75)
    g = ebit.EbitGrid(w.state, flags=ebit.EBIT_FIT_LINE if line else 0, device=device)
    u = torch.from_numpy(w.u).to(device)
    v = torch.from_numpy(w.v).to(device)
    C0 = g.fraction().cpu().numpy()
    rev = w.meta.get("reverse_at")
    nu, nv = (-u, -v) if rev is not None else (u, v)
    t0 = time.perf_counter()
    for k, dt in enumerate(w.dts):
        if rev is not None and k >= rev:
            g.advect(nu, nv, dt)
        else:
            g.advect(u, v, dt)
    st = g.get_state()
    C1 = g.fraction().cpu().numpy()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if C1.sum() == 0.0:
        return {"NA": True, "steps": len(w.dts), "seconds": el}
    X, Y = _markers_xy(st)
    r = 0.15 * n
    out = {"E_area": abs(C1.sum() - C0.sum()) / C0.sum(),
           "E_sym": float(np.abs(C1 - C0).sum()) / (n * n), "steps": len(w.dts), "seconds": el}
    if test != "zalesak":
        out["E_shape"] = float(np.max(np.abs(np.hypot(X - centre[0] * n, Y - centre[1] * n) - r))) / n
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nmax", type=int, default=512)
    ap.add_argument("--tests", default="translation,vortex_T2,vortex_T8,zalesak")
    ap.add_argument("--out", default="")
    ap.add_argument("--device", default="cuda:0")
    args = ap.parse_args()
    rows = []
    for test in args.tests.split(","):
        for line in (False, True):
            key = test + ("_SL" if line else "")
            tab = GOLD[key]
            for k, n in enumerate(tab["N"]):
                if n > args.nmax:
                    continue
                res = run_case(test, n, line, args.device)
                paper = {m: tab[m][k] for m in ("E_area", "E_shape", "E_sym") if m in tab}
                rows.append({"test": test, "method": "EBIT-SL" if line else "EBIT", "N": n, "ours": res,
                             "paper": paper})
                def fmt(m):
                    o = res.get(m)
                    p = paper.get(m)
                    os_ = "NA" if res.get("NA") else ("-" if o is None else f"{o:.3e}")
                    ps = "-" if m not in paper else ("NA" if p is None else f"{p:.3e}")
                    return f"{m} {os_} (paper {ps})"
                print(f"{test:12s} {'SL' if line else 'CF'} N={n:5d}  " + "  ".join(fmt(m) for m in
                      ("E_area", "E_shape", "E_sym")) + f"  [{res['steps']} steps, {res['seconds']:.1f}s]",
                      flush=True)
    if args.out:
        json.dump(rows, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
