"""The AMR experiments of Section 3 on the GPU path.

For the D2 disk and the D2,2 pair, under independent (ILR) and variable (VLR)
level refinement at L levels and base N_k x N_k, this solves the force at
every leaf centre through the library (FP64 by default) and reports:
- the area-weighted L1, L2 and max errors of F_x, F_y and the radial force
  against the analytic force (the quantities of Tables 3-6), and their orders
  under halving;
- the zone and leaf counts and the solve time (the columns of Tables 8-9).

The analytic forces come from the test oracle's closed forms, so this is test
infrastructure, not part of the library.

    python tests/amr_study.py [--kinds ilr,vlr] [--disks d2,d22] [--levels 2,3]
                              [--sizes 128,256,512,1024] [--prec f64|f32]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import diskgen  # noqa: E402
from oracle import analytic as an  # noqa: E402


def layout(kind, disk, nlevels, n0):
    if nlevels == 1:
        return diskgen.Layout(n0, 1, [])
    gen = diskgen.ilr_layout if kind == "ilr" else diskgen.vlr_layout
    return gen(n0, nlevels, disk)


def run_case(gl, torch, kind, disk, nlevels, n0, prec="f64", reps=5):
    """One experiment: errors against the analytic force over all leaves,
    counts and the mean solve time (ms, events around back-to-back solves)."""
    lay = layout(kind, disk, nlevels, n0)
    prof = diskgen.d2 if disk == "d2" else diskgen.d22
    s, dx, dy = lay.sample(prof)
    dt = torch.float64 if prec == "f64" else torch.float32
    p = gl.Plan(lay.n0, gl.F64 if prec == "f64" else gl.F32, nlevels=lay.nlevels,
                patches=lay.patches)
    t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
    fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
    fy = torch.empty_like(fx)
    ws = p.workspace()
    p.solve(*t, fx=fx, fy=fy, workspace=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        p.solve(*t, fx=fx, fy=fy, workspace=ws)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    leaf = lay.leaf_mask()
    X, Y = lay.centres()
    X, Y = X[leaf], Y[leaf]
    gx = fx.double().cpu().numpy()[leaf]
    gy = fy.double().cpu().numpy()[leaf]
    ax, ay = (an.d2_force if disk == "d2" else an.d22_force)(X, Y)
    R = np.hypot(X, Y)
    A = lay.areas()[leaf]
    norms = {"x": an.norms(gx - ax, A), "y": an.norms(gy - ay, A),
             "R": an.norms((gx * X + gy * Y) / R - (ax * X + ay * Y) / R, A)}
    return {"kind": kind, "disk": disk, "levels": nlevels, "n_k": n0, "prec": prec,
            "zones": lay.total(), "leaves": int(leaf.sum()), "patches": len(lay.patches),
            "ms": ms, "norms": norms}


def orders(rows):
    """log2 ratios of successive errors (each norm of each component)."""
    out = []
    for a, b in zip(rows, rows[1:]):
        o = {}
        for c in ("x", "y", "R"):
            o[c] = [math.log2(u / v) if u > 0 and v > 0 else float("nan")
                    for u, v in zip(a["norms"][c], b["norms"][c])]
        out.append({"n_k": "%d/%d" % (a["n_k"], b["n_k"]), **o})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kinds", default="ilr,vlr")
    ap.add_argument("--disks", default="d2,d22")
    ap.add_argument("--levels", default="2,3")
    ap.add_argument("--sizes", default="128,256,512,1024")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    args = ap.parse_args()
    import torch

    import paper_2001_02765_amd as gl
    for kind in args.kinds.split(","):
        for disk in args.disks.split(","):
            for L in map(int, args.levels.split(",")):
                rows = []
                for n in map(int, args.sizes.split(",")):
                    if n << (L - 1) > 4096:
                        continue
                    t0 = time.perf_counter()
                    r = run_case(gl, torch, kind, disk, L, n, args.prec)
                    r["wall_s"] = time.perf_counter() - t0
                    rows.append(r)
                    print(json.dumps(r), flush=True)
                for o in orders(rows):
                    print(json.dumps({"kind": kind, "disk": disk, "levels": L, "orders": o}), flush=True)


if __name__ == "__main__":
    main()
