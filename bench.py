"""Benchmark: leaf forces per second of the thin-disk midplane force on one MI355X.

Workload (one step = one complete solve of the hot path): a uniform
1024 x 1024 grid on [-1,1]^2 (zero-padded 2048^2 FFT) of the noisy exponential
spiral disk exp(-r/0.25)(1 + 0.1 cos(2 theta - ln r / tan 20deg)) with 1%
seeded Gaussian noise and central-difference slopes, inputs resident in HBM.
The FP32 path is the headline value; the FP64 path, p50/p99 per-solve
latency, the per-stage roofline of the dominant kernel, the whole-solve
roofline under the compulsory and two-pass byte models, the spread over the
disks of seeds 0-4, the 2048^2-cell reading of the headline size, the exact
and nested-correction AMR workloads, the off-plane, batched and served
workloads (each beside the plain FP64 path), the headline solve's rate
with several independent solves in flight (batched calls, several streams),
the same convolution through
the vendor FFT library (torch.fft, a timing comparator outside the product
path), the achieved error of every result against the FP64 oracle (relative
L2 and max|dF|/max|F| on seeded target samples) and the CPU oracle's rate on
bounded samples are reported on the same JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def col_bytes(n, prec_bytes, nfields=3, nfam=1):
    """Algorithmic bytes of one column-kernel launch (uniform or AMR solve):
    read the n-row spectra of every input field at the M/2 odd x frequencies
    (M = 2n), read every kernel spectrum (M/2 x (M/2 + 1) reals per kind)
    once, write the column-inverted force spectra."""
    m = 2 * n
    cols = m // 2
    cplx = 2 * prec_bytes
    a = nfields * cols * n * cplx
    q = nfam * 6 * cols * (m // 2 + 1) * prec_bytes
    b = 2 * nfam * cols * n * cplx
    return a + q + b


def accuracy(got, ref, area=None, what=""):
    """Achieved error of GPU results against FP64 oracle values at the same
    targets: area-weighted relative L2 over all components, and
    max |dF| / max |F|."""
    a = 1.0 if area is None else np.asarray(area, dtype=np.float64)
    num = den = 0.0
    mx = mref = 0.0
    for g, r in zip(got, ref):
        g = np.asarray(g, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        num += float(np.sum((g - r) ** 2 * a))
        den += float(np.sum(r * r * a))
        mx = max(mx, float(np.max(np.abs(g - r))))
        mref = max(mref, float(np.max(np.abs(r))))
    return {"rel_l2": float(np.sqrt(num / den)), "max_rel": mx / mref, "targets": int(np.size(ref[0])),
            "against": what}


def _rects_uniform(n, h):
    e = -1.0 + h * np.arange(n)
    X, Y = np.meshgrid(e, e)
    rect = np.stack([X.ravel(), X.ravel() + h, Y.ravel(), Y.ravel() + h], 1)
    cent = np.stack([X.ravel() + 0.5 * h, Y.ravel() + 0.5 * h], 1)
    return rect, cent


def uniform_accuracy(fields, n, fx, fy, k, seed):
    """GPU uniform-grid result against the oracle's direct sum over every
    source cell at k seeded target cells (plus the four corner cells)."""
    import oracle
    s, dx, dy, h = fields
    rng = np.random.default_rng(seed)
    tg = np.unique(np.concatenate([rng.choice(n * n, k, replace=False), [0, n - 1, n * (n - 1), n * n - 1]]))
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, targets=tg, threads=len(os.sched_getaffinity(0)))
    got = (fx.double().cpu().numpy()[tg], fy.double().cpu().numpy()[tg])
    return accuracy(got, (ox, oy), what="oracle direct sum over every cell (FP64), %d seeded cells" % len(tg))


def leaf_targets(lay, per_level, seed):
    """Seeded leaf sample, per_level leaves of every leaf size."""
    import oracle
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(seed)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(per_level, len(cand)), replace=False))
    return rect, cent, idx, np.array(sorted(sel))


def amr_accuracy(lay, vals, fx, fy, per_level, seed, what="oracle leaf direct sum (FP64)"):
    """GPU AMR result against the exact leaf-by-leaf direct sum at sampled
    leaves of every level (area weighted)."""
    import oracle
    s, dx, dy = vals
    rect, cent, idx, sel = leaf_targets(lay, per_level, seed)
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent[sel], threads=len(os.sched_getaffinity(0)))
    area = (rect[sel, 1] - rect[sel, 0]) ** 2
    got = (fx.double().cpu().numpy()[idx[sel]], fy.double().cpu().numpy()[idx[sel]])
    return accuracy(got, (ox, oy), area, what="%s, %d leaves over every level" % (what, len(sel)))


# HBM traffic of the column kernel, measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the same counter
# reads for a plain copy of known size) and stored with a digest of the
# kernel's sources; it is reported only while those sources are unchanged.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_col_uniform1024.md")
KERNEL_SOURCES = ("fft_core.hpp", "kernels.hpp", "kernels_impl.hpp", "kernels_f32_col.hip")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2001_02765_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(kernel, n):
    """Bytes per launch from the counter record, or None if the record is
    missing, for another kernel or size, or older than the kernel sources."""
    try:
        with open(TRAFFIC_RECORD) as f:
            lines = [l for l in f if l.startswith("traffic-record: ")]
    except OSError:
        return None
    for l in lines:
        rec = json.loads(l[len("traffic-record: "):])
        if rec.get("kernel") == kernel and rec.get("n") == n and \
                rec.get("sources_sha256") == kernel_digest():
            return rec["fetch_bytes"] + rec["write_bytes"]
    return None


def sweep_variants(gl, torch, n, fields, steps, stages=("row_fwd", "col", "row_inv")):
    """Mean launch time of every valid variant of each solve kernel in
    stages of the FP32 solve at size n, one kernel at a time
    (GRAVITY_VARIANTS forces it; the other two at the tuned choice):
    {"tuned": ids, "row_fwd_ms": {id: ms}, "col_ms": {...}, "row_inv_ms": {...}}."""
    s, dx, dy, h = fields
    t = [torch.from_numpy(a.ravel()).to("cuda", torch.float32) for a in (s, dx, dy)]
    os.environ.pop("GRAVITY_VARIANTS", None)
    base = gl.Plan(n, gl.F32, h0=h).variants
    out = {"tuned": list(base)}
    for pos, stage in ((0, "row_fwd"), (1, "col"), (2, "row_inv")):
        if stage not in stages:
            continue
        res = {}
        for v in range(17):
            ids = list(base)
            ids[pos] = v
            os.environ["GRAVITY_VARIANTS"] = "%d,%d,%d" % tuple(ids)
            try:
                p = gl.Plan(n, gl.F32, h0=h)
            except gl.GravityError:
                continue
            fx, fy = torch.empty_like(t[0]), torch.empty_like(t[0])
            ws = p.workspace()
            for _ in range(3):  # the first launch of a code object loads it
                p.solve(*t, fx=fx, fy=fy, workspace=ws)
            res[v] = p.profile(*t, fx, fy, ws, reps=steps)[stage]
        out[stage + "_ms"] = res
    os.environ.pop("GRAVITY_VARIANTS", None)
    torch.cuda.synchronize()
    return out


def progress(msg, _t0=[None]):
    """One line per finished leg on stderr (the JSON result stays the only
    line on stdout)."""
    now = time.perf_counter()
    if _t0[0] is None:
        _t0[0] = now
    print("bench: %s (%.1f s)" % (msg, now - _t0[0]), file=sys.stderr, flush=True)


def run_precision(gl, torch, prec, n, steps, warmup, fields, latency=True, acc=True):
    dt = torch.float64 if prec == gl.F64 else torch.float32
    s, dx, dy, h = fields
    plan = gl.Plan(n, prec, h0=h)
    t = [torch.from_numpy(a.ravel()).to("cuda", dt) for a in (s, dx, dy)]
    fx = torch.empty(n * n, dtype=dt, device="cuda")
    fy = torch.empty(n * n, dtype=dt, device="cuda")
    ws = plan.workspace()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.solve(*t, fx=fx, fy=fy, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(*t, fx=fx, fy=fy, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    if not latency:
        return {"value": n * n / (ms * 1e-3), "ms_per_step": ms}
    # per-solve latency (one solve in flight), device events on the solve stream
    lat = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.solve(*t, fx=fx, fy=fy, workspace=ws, stream=stream)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    stages = plan.profile(*t, fx, fy, ws, reps=steps, stream=stream)
    torch.cuda.synchronize()
    return {
        "value": n * n / (ms * 1e-3),
        "ms_per_step": ms,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "stages_ms": stages,
        "variants": list(plan.variants),
        **({"accuracy": uniform_accuracy(fields, n, fx, fy, 256, 2024 + prec)} if acc else {}),
    }


def _timeit(torch, fn, reps):
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def _col_frac(n, prec_bytes, ms, nfam=1):
    """Column-kernel HBM fraction from the col_bytes model and a measured
    mean launch time."""
    gbs = col_bytes(n, prec_bytes, 3, nfam) / (ms * 1e-3) / 1e9
    return {"achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": col_bytes(n, prec_bytes, 3, nfam),
            "launch_ms": ms}


def amr_leg(gl, torch, reps):
    """3-level AMR workload (base 256^2, finest 1024^2): leaf forces/s of the
    exact path (FP32, FP64) and of the nested-correction path, each with its
    error against the exact leaf sum and the column kernel's HBM fraction."""
    import diskgen
    lay, s, dx, dy = diskgen.amr_config(0)
    out = {"workload": "AMR 3 levels, base 256^2, %d patches of 32^2, finest lattice 1024^2 "
                       "(2048^2 FFT), Kuzmin a=0.02 + clumps" % len(lay.patches),
           "leaves": lay.nleaves()}
    for name, prec, dt, amr in (("f32", gl.F32, torch.float32, "exact"), ("f64", gl.F64, torch.float64, "exact"),
                                ("nested_f32", gl.F32, torch.float32, "nested"),
                                ("nested_f64", gl.F64, torch.float64, "nested")):
        p = gl.Plan(lay.n0, prec, nlevels=lay.nlevels, patches=lay.patches, amr=amr)
        t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
        fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
        fy = torch.empty_like(fx)
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve(*t, fx=fx, fy=fy, workspace=ws), reps)
        r = {"ms": ms, "leaf_forces_per_s": p.n_leaves / (ms * 1e-3)}
        if amr == "exact":
            r["stages_ms"] = p.profile(*t, fx, fy, ws, reps=max(5, reps // 4))
            r["variants"] = list(p.variants)
            r["col_roofline"] = _col_frac(p.n_finest, 4 if prec == gl.F32 else 8, r["stages_ms"]["col"], 2)
        torch.cuda.synchronize()
        r["accuracy"] = amr_accuracy(lay, (s, dx, dy), fx, fy, 24, 5,
                                     what="exact leaf direct sum (FP64)" + (": the nested scheme's deviation"
                                                                           if amr == "nested" else ""))
        out[name] = r
    return out


def paper_amr_leg(gl, torch, reps):
    """The largest AMR experiment of the paper's Section 3: AMR(3, D2) under
    independent level refinement at N_k = 1024 (1.42M leaves, finest lattice
    4096^2), by the exact path (8192^2 FFT) and the nested-correction path,
    FP32 and FP64.  Table 8 times the same case with the direct sum on a
    P100 at 1.05e3 s (context: another algorithm on other hardware)."""
    import diskgen
    lay = diskgen.ilr_layout(1024, 3, "d2")
    s, dx, dy = lay.sample(diskgen.d2)
    out = {"workload": "AMR(3, D2) ILR, N_k = 1024: %d leaves in %d patches, finest lattice %d^2"
                       % (lay.nleaves(), len(lay.patches), lay.n_finest),
           "leaves": lay.nleaves(), "paper_p100_direct_s": 1.05e3}
    for name, prec, dt, amr in (("f32", gl.F32, torch.float32, "exact"), ("f64", gl.F64, torch.float64, "exact"),
                                ("nested_f32", gl.F32, torch.float32, "nested"),
                                ("nested_f64", gl.F64, torch.float64, "nested")):
        p = gl.Plan(lay.n0, prec, nlevels=lay.nlevels, patches=lay.patches, amr=amr)
        t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
        fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
        fy = torch.empty_like(fx)
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve(*t, fx=fx, fy=fy, workspace=ws), reps)
        r = {"ms": ms, "leaf_forces_per_s": p.n_leaves / (ms * 1e-3)}
        if amr == "exact":
            st = p.profile(*t, fx, fy, ws, reps=3)
            r["stages_ms"] = st
            r["variants"] = list(p.variants)
            r["col_roofline"] = _col_frac(p.n_finest, 4 if prec == gl.F32 else 8, st["col"], 2)
        torch.cuda.synchronize()
        r["accuracy"] = amr_accuracy(lay, (s, dx, dy), fx, fy, 16, 6,
                                     what="exact leaf direct sum (FP64)" + (": the nested scheme's deviation"
                                                                           if amr == "nested" else ""))
        out[name] = r
        del p, t, fx, fy, ws
    return out


def nested_leg(gl, torch, reps):
    """The served stream's largest requests, which only the nested-correction
    path solves: base 2048^2 with 4 levels (finest lattice 16384^2) and base
    1024^2 with 4 levels (8192^2), FP32 and FP64: leaf forces/s and the
    deviation from the exact leaf sum."""
    import diskgen
    out = {}
    for n0 in (2048, 1024):
        lay, prof = diskgen.request_pool_full(0, bases=(n0,), levels=(4,))[0]
        s, dx, dy = lay.sample(prof)
        leg = {"workload": "base %d^2, 4 levels, %d patches of 32^2 (%d leaves), finest lattice %d^2, Kuzmin "
                           "+ clumps" % (n0, len(lay.patches), lay.nleaves(), lay.n_finest),
               "leaves": lay.nleaves()}
        for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
            p = gl.Plan(lay.n0, prec, nlevels=lay.nlevels, patches=lay.patches, amr="nested")
            t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
            fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
            fy = torch.empty_like(fx)
            ws = p.workspace()
            ms = _timeit(torch, lambda: p.solve(*t, fx=fx, fy=fy, workspace=ws), reps)
            torch.cuda.synchronize()
            leg[name] = {"ms": ms, "leaf_forces_per_s": p.n_leaves / (ms * 1e-3),
                         "workspace_bytes": p.workspace_bytes,
                         "accuracy": amr_accuracy(lay, (s, dx, dy), fx, fy, 12, 7,
                                                  what="exact leaf direct sum (FP64): the nested scheme's "
                                                       "deviation")}
            del p, t, fx, fy, ws
        out["base%d_4levels" % n0] = leg
    return out


def n2048_leg(gl, torch, steps, warmup):
    """The other reading of "at 2048^2": 2048^2 cells (4096^2 zero-padded
    FFT), the same disk recipe, FP32 and FP64."""
    import diskgen
    n = 2048
    fields = diskgen.noisy_spiral(n, 0)
    out = {"workload": "uniform %dx%d cells on [-1,1]^2, zero-padded %d^2 FFT, noisy exponential spiral "
                       "disk with slopes" % (n, n, 2 * n)}
    for name, prec, pb in (("f32", gl.F32, 4), ("f64", gl.F64, 8)):
        r = run_precision(gl, torch, prec, n, steps, warmup, fields)
        r["col_roofline"] = _col_frac(n, pb, r["stages_ms"]["col"])
        out[name] = r
    return out


def offplane_leg(gl, torch, reps, fields, n):
    """The headline disk with targets at height z = 0.05 above every cell
    centre (25.6 cells at 1024^2): (Fx, Fy, Fz) per cell."""
    import oracle
    s, dx, dy, h = fields
    z = 0.05
    out = {"workload": "uniform %dx%d cells, zero-padded %d^2 FFT, targets at height z = %g "
                       "above the cell centres, (Fx, Fy, Fz)" % (n, n, 2 * n, z)}
    rect, cent = _rects_uniform(n, h)
    tg = np.random.default_rng(55).choice(n * n, 24, replace=False)
    ref = oracle.direct_z(rect, s.ravel(), dx.ravel(), dy.ravel(), cent[tg], z,
                          threads=len(os.sched_getaffinity(0)))
    for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
        p = gl.Plan(n, prec, h0=h, z=z)
        t = [torch.from_numpy(a.ravel()).to("cuda", dt) for a in (s, dx, dy)]
        fo = [torch.empty(n * n, dtype=dt, device="cuda") for _ in range(3)]
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve_xyz(*t, *fo, workspace=ws), reps)
        torch.cuda.synchronize()
        out[name] = {"ms": ms, "forces_per_s": n * n / (ms * 1e-3), "variants": list(p.variants),
                     "accuracy": accuracy([f.double().cpu().numpy()[tg] for f in fo], ref,
                                          what="oracle off-plane direct sum (FP64), 24 seeded cells")}
    return out


def batch_leg(gl, torch, reps):
    """64 independent disks of mixed sizes in one gravity_solve_batch (FP32)
    against the same 64 solves issued one by one."""
    import diskgen
    import oracle
    disks = diskgen.batch_disks(0)
    plans = [gl.Plan(n, gl.F32) for (n, _, _, _) in disks]
    ins = [[torch.from_numpy(a.ravel()).to("cuda", torch.float32) for a in d[1:]] for d in disks]
    outs = [(torch.empty_like(i[0]), torch.empty_like(i[0])) for i in ins]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    args = ([i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins],
            [o[0] for o in outs], [o[1] for o in outs])
    ms_p = _timeit(torch, lambda: gl.solve_batch(plans, *args, ws, persistent=True), reps)
    torch.cuda.synchronize()
    ms_b = _timeit(torch, lambda: gl.solve_batch(plans, *args, ws), reps)
    torch.cuda.synchronize()
    # achieved error of every disk of the batch at seeded targets
    rng = np.random.default_rng(64)
    got, ref = [[], []], [[], []]
    for (n, s, dx, dy), (fx, fy) in zip(disks, outs):
        tg = rng.choice(n * n, 3, replace=False)
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n, targets=tg, threads=len(os.sched_getaffinity(0)))
        scale = 1.0 / max(np.max(np.abs(ox)), np.max(np.abs(oy)))   # each disk weighted alike
        got[0].append(fx.double().cpu().numpy()[tg] * scale)
        got[1].append(fy.double().cpu().numpy()[tg] * scale)
        ref[0].append(ox * scale)
        ref[1].append(oy * scale)
    acc = accuracy([np.concatenate(g) for g in got], [np.concatenate(r) for r in ref],
                   what="oracle direct sum (FP64), 3 seeded cells of each of the 64 disks, each disk scaled to "
                        "its largest sampled force")
    ws1 = torch.empty(max(p.workspace_bytes for p in plans), dtype=torch.uint8, device="cuda")

    def seq():
        for p, i, o in zip(plans, ins, outs):
            p.solve(*i, fx=o[0], fy=o[1], workspace=ws1)
    ms_s = _timeit(torch, seq, reps)
    # the plain FP64 path, one solve at a time, on the same disks
    plans64 = [gl.Plan(n, gl.F64) for (n, _, _, _) in disks]
    ins64 = [[a.double() for a in i] for i in ins]
    outs64 = [(torch.empty_like(i[0]), torch.empty_like(i[0])) for i in ins64]
    ws64 = torch.empty(max(p.workspace_bytes for p in plans64), dtype=torch.uint8, device="cuda")

    def seq64():
        for p, i, o in zip(plans64, ins64, outs64):
            p.solve(*i, fx=o[0], fy=o[1], workspace=ws64)
    ms_64 = _timeit(torch, seq64, reps)
    cells = int(sum(d[0] ** 2 for d in disks))
    two_pass = 124 * cells   # FP32 two-pass byte model, per leaf
    return {"workload": "64 disks, n in {64..1024}, exponential/Kuzmin spirals, FP32",
            "cells": cells, "ms_batch": ms_b, "ms_batch_persistent": ms_p,
            "forces_per_s_batch_persistent": cells / (ms_p * 1e-3),
            "ms_sequential": ms_s, "ms_sequential_f64": ms_64,
            "forces_per_s_batch": cells / (ms_b * 1e-3), "forces_per_s_sequential": cells / (ms_s * 1e-3),
            "forces_per_s_sequential_f64": cells / (ms_64 * 1e-3),
            "roofline_two_pass": {"bytes": two_pass, "frac": two_pass / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "accuracy": acc}


def small_batch_leg(gl, torch, reps):
    """Many small disks (256 disks, n in {64, 128, 256}, FP32), where launch
    gaps dominate: grouped launches, one persistent launch, one by one."""
    import diskgen
    disks = diskgen.batch_disks(1, count=256, sizes=(64, 128, 256))
    plans = [gl.Plan(n, gl.F32) for (n, _, _, _) in disks]
    ins = [[torch.from_numpy(a.ravel()).to("cuda", torch.float32) for a in d[1:]] for d in disks]
    outs = [(torch.empty_like(i[0]), torch.empty_like(i[0])) for i in ins]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    args = ([i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins],
            [o[0] for o in outs], [o[1] for o in outs])
    ms_p = _timeit(torch, lambda: gl.solve_batch(plans, *args, ws, persistent=True), reps)
    ms_b = _timeit(torch, lambda: gl.solve_batch(plans, *args, ws), reps)
    ws1 = torch.empty(max(p.workspace_bytes for p in plans), dtype=torch.uint8, device="cuda")

    def seq():
        for p, i, o in zip(plans, ins, outs):
            p.solve(*i, fx=o[0], fy=o[1], workspace=ws1)
    ms_s = _timeit(torch, seq, reps)
    cells = int(sum(d[0] ** 2 for d in disks))
    return {"workload": "256 disks, n in {64, 128, 256}, exponential/Kuzmin spirals, FP32", "cells": cells,
            "ms_batch": ms_b, "ms_batch_persistent": ms_p, "ms_sequential": ms_s,
            "forces_per_s_batch": cells / (ms_b * 1e-3),
            "forces_per_s_batch_persistent": cells / (ms_p * 1e-3),
            "forces_per_s_sequential": cells / (ms_s * 1e-3)}


def serve_leg(gl, torch, nreq=2000, warm=200, rhos=(0.5, 0.8), budget=8 << 30):
    """Poisson stream of AMR solves through the continuous-batching server,
    over the full request mix (bases 128^2-2048^2, 1-4 levels, 4-256 patches
    of 32^2): the exact path where the finest lattice is at most 4096^2, the
    nested-correction path beyond.  Closed-loop capacity first, then
    arrivals at rho times it for each rho; every in-flight request writes
    its own outputs.  Beside it, the plain FP64 path solving the same
    layouts one at a time, and spot checks of served results against the
    exact leaf sum."""
    import diskgen
    pool = diskgen.request_pool_full(0)
    entries = []
    nslot = 16
    for lay, prof in pool:
        amr = "exact" if lay.n_finest <= 4096 else "nested"
        p = gl.Plan(lay.n0, gl.F32, nlevels=lay.nlevels, patches=lay.patches, amr=amr)
        s, dx, dy = lay.sample(prof)
        t = [torch.from_numpy(a).to("cuda", torch.float32) for a in (s, dx, dy)]
        outs = [(torch.empty_like(t[0]), torch.empty_like(t[0])) for _ in range(nslot)]
        entries.append({"plan": p, "in": t, "outs": outs, "lay": lay, "vals": (s, dx, dy), "amr": amr,
                        "last": [None] * nslot, "next": 0})
    torch.cuda.synchronize()
    srv = gl.Server(budget, nstreams=4, max_batch=8)
    rng = np.random.default_rng(1)
    picks = rng.integers(len(entries), size=nreq + warm)

    def submit(k):
        e = entries[picks[k]]
        slot = e["next"]
        e["next"] = (slot + 1) % nslot
        prev = e["last"][slot]
        if prev is not None and not srv.poll(prev):
            srv.wait(prev)   # the slot's previous request must be done with its outputs
        o = e["outs"][slot]
        tk = srv.submit(e["plan"], *e["in"], o[0], o[1])
        e["last"][slot] = tk
        return tk

    for k in range(warm):
        submit(k)
    srv.drain()
    srv.reset_stats()
    t0 = time.perf_counter()
    for k in range(warm, warm + nreq):
        submit(k)
    srv.drain()
    cap = nreq / (time.perf_counter() - t0)
    closed = srv.stats()
    runs = []
    for rho in rhos:
        srv.reset_stats()
        lam = rho * cap
        gaps = rng.exponential(1.0 / lam, size=nreq)
        t_arr = time.perf_counter() + np.cumsum(gaps)
        t0 = time.perf_counter()
        for k in range(nreq):
            while time.perf_counter() < t_arr[k]:
                pass
            submit(warm + k)
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        runs.append({"rho": rho, "rate_req_per_s": lam, "p50_ms": st["latency_p50_ms"],
                     "p99_ms": st["latency_p99_ms"], "max_ms": st["latency_max_ms"],
                     "leaf_forces_per_s": st["leaves_completed"] / wall,
                     "peak_bytes_in_use": st["peak_bytes_in_use"], "batches": st["batches"],
                     "completed": st["completed"]})
    budget_bytes = srv.stats()["budget_bytes"]
    srv.close()
    torch.cuda.synchronize()
    # spot checks: the last served result of a few layouts of each method
    checks = []
    for k, e in enumerate(entries):
        if k % 5 != 2 or e["last"][(e["next"] - 1) % nslot] is None:
            continue
        o = e["outs"][(e["next"] - 1) % nslot]
        a = amr_accuracy(e["lay"], e["vals"], o[0], o[1], 6, 100 + k,
                         what="exact leaf direct sum (FP64)" + (": nested deviation" if e["amr"] == "nested" else ""))
        a.update({"base": e["lay"].n0, "levels": e["lay"].nlevels, "method": e["amr"]})
        checks.append(a)
    # plain FP64 single solves of the same request mix (one stream, one at a
    # time): each layout timed alone, weighted by how often the stream asked for it
    weights = np.bincount(picks[warm:], minlength=len(entries))
    leaves = ms = 0.0
    for e, w in zip(entries, weights):
        lay = e["lay"]
        p = gl.Plan(lay.n0, gl.F64, nlevels=lay.nlevels, patches=lay.patches, amr=e["amr"])
        t64 = [a.double() for a in e["in"]]
        f = (torch.empty_like(t64[0]), torch.empty_like(t64[0]))
        ws = p.workspace()
        m = _timeit(torch, lambda: p.solve(*t64, fx=f[0], fy=f[1], workspace=ws), 3)
        leaves += p.n_leaves * float(w)
        ms += m * float(w)
        del p, t64, f, ws
    npat = [len(e["lay"].patches) for e in entries if e["lay"].nlevels > 1]
    return {"workload": "Poisson arrivals of AMR solves over %d seeded layouts (bases 128^2-2048^2, levels 1-4, "
                        "%d-%d patches of 32^2 per refined layout, finest lattice up to %d^2; exact path for "
                        "%d layouts with finest <= 4096^2, nested-correction path for %d beyond), FP32"
                        % (len(entries), min(npat), max(npat), max(e["lay"].n_finest for e in entries),
                           sum(e["amr"] == "exact" for e in entries), sum(e["amr"] == "nested" for e in entries)),
            "requests": nreq, "warmup_requests": warm, "unsupported_requests": 0,
            "capacity_req_per_s": cap,
            "closed_loop_p50_ms": closed["latency_p50_ms"], "closed_loop_p99_ms": closed["latency_p99_ms"],
            "budget_bytes": budget_bytes, "open_loop": runs,
            "plain_f64_leaf_forces_per_s": leaves / (ms * 1e-3), "accuracy_spot_checks": checks}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, fields, budget_s=25.0, with_amr=True):
    """The oracle's direct leaf sum (exact kernels per source cell, FP64,
    compensated) on a seeded sample of target cells of the same workload,
    every source included.  Returns forces/s and the thread count."""
    import oracle

    s, dx, dy, h = fields
    lay_rect, cent = _rects_uniform(n, h)
    rng = np.random.default_rng(7)
    threads = len(os.sched_getaffinity(0))

    def timed(k):
        tg = rng.choice(n * n, k, replace=False)
        t0 = time.perf_counter()
        oracle.direct(lay_rect, s.ravel(), dx.ravel(), dy.ravel(), cent[tg], threads=threads)
        return time.perf_counter() - t0

    k0 = max(threads, 8)
    t0 = timed(k0)
    k = int(max(k0, min(4096, k0 * budget_s / max(t0, 1e-3))))
    el = timed(k)
    # one core, as the paper's Fortran baseline ran: a few targets
    tg1 = rng.choice(n * n, 4, replace=False)
    t1 = time.perf_counter()
    oracle.direct(lay_rect, s.ravel(), dx.ravel(), dy.ravel(), cent[tg1], threads=1)
    el1 = time.perf_counter() - t1
    amr = cpu_baseline_amr(threads, budget_s / 3) if with_amr else None
    # the 64^2 Kuzmin disk (M = 1, a = 0.2), every cell against every cell
    import diskgen
    X, Y = diskgen.grid_centres(64)
    ks, kdx, kdy = diskgen.kuzmin(X, Y, 1.0, 0.2)
    t64 = time.perf_counter()
    oracle.uniform(ks, kdx, kdy, -1.0, -1.0, 2.0 / 64, threads=threads)
    el64 = time.perf_counter() - t64
    return {"value": k / el, "unit": "forces/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d seeded target cells of the %dx%d disk, each summed over all %d source "
                      "cells with the exact kernels (direct method), %.1f s" % (k, n, n, n * n, el),
            "value_1core": 4 / el1, "sample_1core": "4 target cells on one thread, %.1f s" % el1,
            "kuzmin64_full": {"value": 64 * 64 / el64, "unit": "forces/s",
                              "sample": "all 4096 cells of the 64x64 Kuzmin disk: the uniform-grid "
                                        "oracle (closed form per cell offset, then the O(N^4) "
                                        "compensated sum), %.3f s" % el64},
            **({"amr": amr} if amr else {})}


def cpu_baseline_amr(threads, budget_s):
    """The oracle's direct leaf sum on the 3-level AMR workload: seeded
    targets drawn equally from the leaves of each level, every leaf a
    source.  Returns leaf forces/s."""
    import diskgen
    import oracle

    lay, s, dx, dy = diskgen.amr_config(0)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    width = rect[:, 1] - rect[:, 0]
    levels = np.unique(width)
    rng = np.random.default_rng(11)

    def timed(per_level):
        tg = np.concatenate([rng.choice(np.nonzero(width == w)[0], min(per_level, int(np.sum(width == w))),
                                        replace=False) for w in levels])
        t0 = time.perf_counter()
        oracle.direct(rect, s[idx], dx[idx], dy[idx], cent[tg], threads=threads)
        return len(tg), time.perf_counter() - t0

    k0, e0 = timed(max(1, threads // len(levels)))
    per = int(max(1, min(2048 // len(levels), k0 / len(levels) * budget_s / max(e0, 1e-3))))
    k, el = timed(per)
    return {"value": k / el, "unit": "leaf forces/s",
            "sample": "%d seeded leaf targets (%d per level, %d levels) of the 3-level AMR workload, "
                      "each summed over all %d leaves, %.1f s" % (k, per, len(levels), len(idx), el)}


def throughput_leg(gl, torch, n, fields, reps):
    """Independent solves of the headline disk in flight together: 8 solves
    per gravity_solve_batch call (one launch per kernel over the 8), and
    solves spread round-robin over 2 and 3 streams (each with its own
    workspace and outputs).  The headline value times one solve at a time
    on one stream; these are the rates a stream of independent solves
    reaches when the kernels of neighbouring solves overlap."""
    s, dx, dy, h = fields
    out = {"workload": "uniform %dx%d cells, zero-padded %d^2 FFT, independent solves in flight together"
                       % (n, n, 2 * n)}
    for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
        plan = gl.Plan(n, prec, h0=h)
        t = [torch.from_numpy(a.ravel()).to("cuda", dt) for a in (s, dx, dy)]
        r = {}
        nb = 8
        outs = [(torch.empty(n * n, dtype=dt, device="cuda"), torch.empty(n * n, dtype=dt, device="cuda"))
                for _ in range(nb)]
        ws = torch.empty(gl.batch_workspace_bytes([plan] * nb), dtype=torch.uint8, device="cuda")
        ms = _timeit(torch, lambda: gl.solve_batch([plan] * nb, [t[0]] * nb, [t[1]] * nb, [t[2]] * nb,
                                                    [o[0] for o in outs], [o[1] for o in outs], ws), reps)
        r["batch8"] = {"ms_per_solve": ms / nb, "forces_per_s": nb * n * n / (ms * 1e-3)}
        for ns in (2, 3):
            streams = [torch.cuda.Stream() for _ in range(ns)]
            wss = [plan.workspace() for _ in range(ns)]
            k_per = 16

            def run():
                for k in range(ns * k_per):
                    i = k % ns
                    plan.solve(*t, fx=outs[i][0], fy=outs[i][1], workspace=wss[i], stream=streams[i])
            ms = _timeit(torch, run, max(10, reps))
            r["streams%d" % ns] = {"ms_per_solve": ms / (ns * k_per),
                                   "forces_per_s": ns * k_per * n * n / (ms * 1e-3)}
            del wss
        out[name] = r
        del outs, ws
    torch.cuda.synchronize()
    return out


def library_fft_leg(gl, torch, n, reps, ours):
    """Timing comparator outside the product path: the same zero-padded
    convolution written with the vendor FFT library through torch.fft
    (rocFFT): the three fields padded to (2n)^2, real-to-complex 2D
    transforms, the six spectral products, complex-to-real inverses of the
    two components, the n x n corner kept.  The spectra are random tensors
    of the right shape (only the time is compared; the library path is not
    part of the solve).  ours: {"f32": ms, "f64": ms} of the library's own
    solve at the same size."""
    m = 2 * n
    out = {"workload": "uniform %dx%d cells, zero-padded %d^2 FFT, torch.fft (rocFFT) rfft2 of 3 fields, "
                       "6 spectral products, irfft2 of 2 components" % (n, n, m)}
    g = torch.Generator(device="cuda").manual_seed(0)
    for name, dt, cdt in (("f32", torch.float32, torch.complex64), ("f64", torch.float64, torch.complex128)):
        src = torch.rand((3, n, n), dtype=dt, device="cuda", generator=g)
        kr = torch.rand((6, m, m // 2 + 1), dtype=dt, device="cuda", generator=g)
        ki = torch.rand((6, m, m // 2 + 1), dtype=dt, device="cuda", generator=g)
        kern = torch.complex(kr, ki).to(cdt)
        pad = torch.zeros((3, m, m), dtype=dt, device="cuda")
        res = torch.empty((2, n, n), dtype=dt, device="cuda")

        def solve():
            pad[:, :n, :n] = src
            X = torch.fft.rfft2(pad)
            fx = X[0] * kern[0] + X[1] * kern[1] + X[2] * kern[2]
            fy = X[0] * kern[3] + X[1] * kern[4] + X[2] * kern[5]
            res[0] = torch.fft.irfft2(fx, s=(m, m))[:n, :n]
            res[1] = torch.fft.irfft2(fy, s=(m, m))[:n, :n]
        ms = _timeit(torch, solve, reps)
        X = torch.fft.rfft2(pad)

        def transforms():  # the library's transforms alone (no padding, no products)
            torch.fft.rfft2(pad)
            torch.fft.irfft2(X[0], s=(m, m))
            torch.fft.irfft2(X[1], s=(m, m))
        ms_fft = _timeit(torch, transforms, reps)
        out[name] = {"ms": ms, "forces_per_s": n * n / (ms * 1e-3), "transforms_only_ms": ms_fft,
                     "ours_ms": ours[name], "speedup_of_ours": ms / ours[name]}
        del X
        del src, kr, ki, kern, pad, res
    torch.cuda.synchronize()
    return out


def seed_spread(gl, torch, n, steps, warmup, first):
    """FP32 forces/s of the headline solve on the disks of seeds 0-4 (seed 0
    is the main run): median and spread."""
    import diskgen
    vals = [first]
    for seed in range(1, 5):
        r = run_precision(gl, torch, gl.F32, n, steps, warmup, diskgen.noisy_spiral(n, seed),
                          latency=False)
        vals.append(r["value"])
    return {"seeds": list(range(5)), "forces_per_s": vals, "median": float(np.median(vals)),
            "min": float(min(vals)), "max": float(max(vals))}


def solve_roofline(n, ms32, ms64):
    """Whole-solve HBM roofline under two byte models per leaf (slopes on):
    compulsory (three fields in, two forces out, six real-quadrant kernel
    spectra read once: 44 B in FP32) and two passes out of cache (row
    forward, fused column pass, row inverse, each streaming its spectra
    through HBM once: 124 B in FP32); FP64 doubles both."""
    out = {}
    for name, ms, k in (("f32", ms32, 1), ("f64", ms64, 2)):
        bmin, b2 = 44 * k * n * n, 124 * k * n * n
        out[name] = {"ms": ms, "bytes_compulsory": bmin, "bytes_two_pass": b2,
                     "frac_compulsory": bmin / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "frac_two_pass": b2 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def copy_gbs(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes / s) of a 1 GiB buffer:
    the bandwidth a plain streaming kernel reaches on this GPU."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the AMR, batch and serving legs")
    ap.add_argument("--only", choices=["f32", "f64"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--legs", default="",
                    help="comma-separated subset of the extra legs to run (default: all)")
    ap.add_argument("--sweep-col", action="store_true",
                    help="as --sweep, the column kernel only")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark, time every valid variant of each kernel of the FP32 "
                         "headline solve (forced one kernel at a time, the others at the tuned choice); "
                         "profiling runs")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="instead of the solver, run --steps device copies of BYTES bytes "
                         "(reference kernel for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X "
              "(multi-GPU sharding is not part of this build); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import diskgen
    import paper_2001_02765_amd as gl

    if args.copy_calib:
        src = torch.ones(args.copy_calib // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": args.copy_calib, "copies": args.steps}), flush=True)
        return

    n = args.n
    fields = diskgen.noisy_spiral(n, 0)
    if args.sweep:
        print(json.dumps({"sweep": sweep_variants(gl, torch, n, fields, args.steps)}), flush=True)
        return
    if args.sweep_col:
        print(json.dumps({"sweep_col": sweep_variants(gl, torch, n, fields, args.steps, ("col",))}), flush=True)
        return
    if args.only:
        prec = gl.F32 if args.only == "f32" else gl.F64
        r = run_precision(gl, torch, prec, n, args.steps, args.warmup, fields, acc=False)
        print(json.dumps({"only": args.only, "n": n, **r}), flush=True)
        return
    progress("start")
    r32 = run_precision(gl, torch, gl.F32, n, args.steps, args.warmup, fields)
    progress("headline FP32")
    r64 = run_precision(gl, torch, gl.F64, n, args.steps, args.warmup, fields)
    progress("headline FP64")

    col_ms = r32["stages_ms"]["col"]
    achieved = col_bytes(n, 4) / (col_ms * 1e-3) / 1e9
    kname = "grav::k_col<float, %d, %d, 3, 1, 2>" % (2 * n, r32["variants"][1])
    traffic = stored_traffic(kname, n)
    roof = {"bound": "hbm", "kernel": kname + " (fused column transform, FP32)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            # counter-measured bytes over the same measured launch time
            "traffic_gbs": None if traffic is None else traffic / (col_ms * 1e-3) / 1e9,
            "bytes_per_launch": col_bytes(n, 4), "launch_ms": col_ms,
            "copy_gbs": copy_gbs(torch)}
    out = {
        "metric": "finest-cell forces/sec at 2048^2 (FP32 vs FP64 path); p50/p99 solve latency",
        "value": r32["value"],
        "unit": "forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uniform %dx%d cells on [-1,1]^2, zero-padded %d^2 FFT, noisy "
                               "exponential spiral disk with slopes" % (n, n, 2 * n),
                   "n": n, "fft": 2 * n, "slopes": True},
        "latency_ms": r32["latency_ms"],
        "accuracy": r32["accuracy"],
        "stages_ms": r32["stages_ms"],
        "variants": r32["variants"],
        "fp64": r64,
        "roofline": roof,
        "solve_roofline": solve_roofline(n, r32["ms_per_step"], r64["ms_per_step"]),
    }
    if not args.no_extra:
        legs = (("seed_spread", lambda: seed_spread(gl, torch, n, max(20, args.steps // 2), args.warmup,
                                                    r32["value"])),
                ("throughput", lambda: throughput_leg(gl, torch, n, fields, max(10, args.steps // 10))),
                ("library_fft", lambda: library_fft_leg(gl, torch, n, max(20, args.steps // 4),
                                                        {"f32": r32["ms_per_step"], "f64": r64["ms_per_step"]})),
                ("n2048", lambda: n2048_leg(gl, torch, max(10, args.steps // 4), 5)),
                ("amr", lambda: amr_leg(gl, torch, max(10, args.steps // 4))),
                ("paper_amr", lambda: paper_amr_leg(gl, torch, max(5, args.steps // 20))),
                ("nested", lambda: nested_leg(gl, torch, max(5, args.steps // 20))),
                ("offplane", lambda: offplane_leg(gl, torch, max(10, args.steps // 4), fields, n)),
                ("batch", lambda: batch_leg(gl, torch, max(5, args.steps // 20))),
                ("batch_small", lambda: small_batch_leg(gl, torch, max(5, args.steps // 20))),
                ("serve", lambda: serve_leg(gl, torch)))
        for name, fn in legs:
            if args.legs and name not in args.legs.split(","):
                continue
            out[name] = fn()
            progress(name)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, fields, with_amr=not args.no_extra)
        progress("cpu baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
