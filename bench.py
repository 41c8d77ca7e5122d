"""Benchmark: leaf forces per second of the thin-disk midplane force on one MI355X.

Workload (one step = one complete solve of the hot path): a uniform
1024 x 1024 grid on [-1,1]^2 (zero-padded 2048^2 FFT) of the noisy exponential
spiral disk exp(-r/0.25)(1 + 0.1 cos(2 theta - ln r / tan 20deg)) with 1%
seeded Gaussian noise and central-difference slopes, inputs resident in HBM.
The FP32 path is the headline value; the FP64 path, p50/p99 per-solve
latency, the per-stage roofline of the dominant kernel, the whole-solve
roofline under the compulsory and two-pass byte models, the spread over the
disks of seeds 0-4, the AMR, off-plane, batched and served workloads (each
beside the plain FP64 path) and the CPU oracle's rate on bounded samples are
reported on the same JSON line.

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


def run_precision(gl, torch, prec, n, steps, warmup, fields, latency=True):
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
    return {
        "value": n * n / (ms * 1e-3),
        "ms_per_step": ms,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "stages_ms": stages,
        "variants": list(plan.variants),
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


def amr_leg(gl, torch, reps):
    """3-level AMR workload (base 256^2, finest 1024^2): leaf forces/s."""
    import diskgen
    lay, s, dx, dy = diskgen.amr_config(0)
    out = {"workload": "AMR 3 levels, base 256^2, %d patches of 32^2, finest lattice 1024^2 "
                       "(2048^2 FFT), Kuzmin a=0.02 + clumps" % len(lay.patches),
           "leaves": lay.nleaves()}
    for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
        p = gl.Plan(lay.n0, prec, nlevels=lay.nlevels, patches=lay.patches)
        t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
        fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
        fy = torch.empty_like(fx)
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve(*t, fx=fx, fy=fy, workspace=ws), reps)
        out[name] = {"ms": ms, "leaf_forces_per_s": p.n_leaves / (ms * 1e-3),
                     "stages_ms": p.profile(*t, fx, fy, ws, reps=max(5, reps // 4))}
    return out


def paper_amr_leg(gl, torch, reps):
    """The largest AMR experiment of the paper's Section 3 that this path
    runs: AMR(3, D2) under independent level refinement at N_k = 1024 (1.42M
    leaves, finest lattice 4096^2, 8192^2 FFT), FP32 and FP64.  Table 8
    times the same case with the direct sum on a P100 at 1.05e3 s (context:
    another algorithm on other hardware)."""
    import diskgen
    lay = diskgen.ilr_layout(1024, 3, "d2")
    s, dx, dy = lay.sample(diskgen.d2)
    out = {"workload": "AMR(3, D2) ILR, N_k = 1024: %d leaves in %d patches, finest lattice %d^2"
                       % (lay.nleaves(), len(lay.patches), lay.n_finest),
           "leaves": lay.nleaves(), "paper_p100_direct_s": 1.05e3}
    for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
        p = gl.Plan(lay.n0, prec, nlevels=lay.nlevels, patches=lay.patches)
        t = [torch.from_numpy(a).to("cuda", dt) for a in (s, dx, dy)]
        fx = torch.empty(p.n_cells, dtype=dt, device="cuda")
        fy = torch.empty_like(fx)
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve(*t, fx=fx, fy=fy, workspace=ws), reps)
        out[name] = {"ms": ms, "leaf_forces_per_s": p.n_leaves / (ms * 1e-3)}
        del p, t, fx, fy, ws
    return out


def offplane_leg(gl, torch, reps, fields, n):
    """The headline disk with targets at height z = 0.05 above every cell
    centre (25.6 cells at 1024^2): (Fx, Fy, Fz) per cell."""
    s, dx, dy, h = fields
    z = 0.05
    out = {"workload": "uniform %dx%d cells, zero-padded %d^2 FFT, targets at height z = %g "
                       "above the cell centres, (Fx, Fy, Fz)" % (n, n, 2 * n, z)}
    for name, prec, dt in (("f32", gl.F32, torch.float32), ("f64", gl.F64, torch.float64)):
        p = gl.Plan(n, prec, h0=h, z=z)
        t = [torch.from_numpy(a.ravel()).to("cuda", dt) for a in (s, dx, dy)]
        fo = [torch.empty(n * n, dtype=dt, device="cuda") for _ in range(3)]
        ws = p.workspace()
        ms = _timeit(torch, lambda: p.solve_xyz(*t, *fo, workspace=ws), reps)
        out[name] = {"ms": ms, "forces_per_s": n * n / (ms * 1e-3), "variants": list(p.variants)}
    return out


def batch_leg(gl, torch, reps):
    """64 independent disks of mixed sizes in one gravity_solve_batch (FP32)
    against the same 64 solves issued one by one."""
    import diskgen
    disks = diskgen.batch_disks(0)
    plans = [gl.Plan(n, gl.F32) for (n, _, _, _) in disks]
    ins = [[torch.from_numpy(a.ravel()).to("cuda", torch.float32) for a in d[1:]] for d in disks]
    outs = [(torch.empty_like(i[0]), torch.empty_like(i[0])) for i in ins]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    args = ([i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins],
            [o[0] for o in outs], [o[1] for o in outs])
    ms_b = _timeit(torch, lambda: gl.solve_batch(plans, *args, ws), reps)
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
    return {"workload": "64 disks, n in {64..1024}, exponential/Kuzmin spirals, FP32",
            "cells": cells, "ms_batch": ms_b, "ms_sequential": ms_s, "ms_sequential_f64": ms_64,
            "forces_per_s_batch": cells / (ms_b * 1e-3), "forces_per_s_sequential": cells / (ms_s * 1e-3),
            "forces_per_s_sequential_f64": cells / (ms_64 * 1e-3)}


def serve_leg(gl, torch, nreq, rhos=(0.5, 0.8), budget=8 << 30):
    """Poisson stream of AMR solves of mixed sizes through the continuous-
    batching server: closed-loop capacity first, then arrivals at rho times it
    for each rho; beside it, the plain FP64 path solving the same layouts one
    at a time."""
    import diskgen
    pool = diskgen.request_pool(0, count=16)
    entries = []
    for lay, prof in pool:
        p = gl.Plan(lay.n0, gl.F32, nlevels=lay.nlevels, patches=lay.patches)
        s, dx, dy = lay.sample(prof)
        t = [torch.from_numpy(a).to("cuda", torch.float32) for a in (s, dx, dy)]
        outs = [(torch.empty_like(t[0]), torch.empty_like(t[0])) for _ in range(4)]
        entries.append((p, t, outs, lay))
    srv = gl.Server(budget, nstreams=4, max_batch=8)
    rng = np.random.default_rng(1)
    picks = rng.integers(len(entries), size=nreq)

    def submit(k):
        p, t, outs, _ = entries[picks[k]]
        o = outs[k % len(outs)]
        return srv.submit(p, *t, o[0], o[1])

    for k in range(min(200, nreq)):  # warm-up
        submit(k)
    srv.drain()
    srv.reset_stats()
    t0 = time.perf_counter()
    for k in range(nreq):
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
            submit(k)
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        runs.append({"rho": rho, "rate_req_per_s": lam, "p50_ms": st["latency_p50_ms"],
                     "p99_ms": st["latency_p99_ms"], "max_ms": st["latency_max_ms"],
                     "leaf_forces_per_s": st["leaves_completed"] / wall,
                     "peak_bytes_in_use": st["peak_bytes_in_use"], "batches": st["batches"]})
    budget_bytes = srv.stats()["budget_bytes"]
    srv.close()
    # plain FP64 single solves of the same request mix (one stream, one at a
    # time): each layout timed alone, weighted by how often the stream asked for it
    weights = np.bincount(picks, minlength=len(entries))
    leaves = ms = 0.0
    for (_, t, _, lay), w in zip(entries, weights):
        p = gl.Plan(lay.n0, gl.F64, nlevels=lay.nlevels, patches=lay.patches)
        t64 = [a.double() for a in t]
        f = (torch.empty_like(t64[0]), torch.empty_like(t64[0]))
        ws = p.workspace()
        m = _timeit(torch, lambda: p.solve(*t64, fx=f[0], fy=f[1], workspace=ws), 5)
        leaves += p.n_leaves * float(w)
        ms += m * float(w)
        del p, t64, f, ws
    levels = sorted({lay.nlevels for *_, lay in entries})
    bases = sorted({lay.n0 for *_, lay in entries})
    npat = [len(lay.patches) for *_, lay in entries if lay.nlevels > 1]
    finest = max(lay.n0 << (lay.nlevels - 1) for *_, lay in entries)
    return {"workload": "Poisson arrivals of AMR solves over %d seeded layouts (bases %s, levels %s, "
                        "%s patches of 32^2 per refined layout, finest lattice up to %d^2), FP32"
                        % (len(entries), "/".join(map(str, bases)), "/".join(map(str, levels)),
                           ("%d-%d" % (min(npat), max(npat))) if npat else "no", finest),
            "requests": nreq, "warmup_requests": min(200, nreq), "capacity_req_per_s": cap,
            "closed_loop_p50_ms": closed["latency_p50_ms"], "closed_loop_p99_ms": closed["latency_p99_ms"],
            "budget_bytes": budget_bytes, "open_loop": runs,
            "plain_f64_leaf_forces_per_s": leaves / (ms * 1e-3)}


def cpu_baseline(n, fields, budget_s=25.0, with_amr=True):
    """The oracle's direct leaf sum (exact kernels per source cell, FP64,
    compensated) on a seeded sample of target cells of the same workload,
    every source included.  Returns forces/s and the thread count."""
    import oracle

    s, dx, dy, h = fields
    lay_rect, cent = _uniform_rects(n, h)
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
    return {"value": k / el, "unit": "forces/s", "cores": threads, "kind": "oracle",
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


def _uniform_rects(n, h):
    e = -1.0 + h * np.arange(n)
    X, Y = np.meshgrid(e, e)
    rect = np.stack([X.ravel(), X.ravel() + h, Y.ravel(), Y.ravel() + h], 1)
    cent = np.stack([X.ravel() + 0.5 * h, Y.ravel() + 0.5 * h], 1)
    return rect, cent


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
    if args.only:
        prec = gl.F32 if args.only == "f32" else gl.F64
        r = run_precision(gl, torch, prec, n, args.steps, args.warmup, fields)
        print(json.dumps({"only": args.only, "n": n, **r}), flush=True)
        return
    r32 = run_precision(gl, torch, gl.F32, n, args.steps, args.warmup, fields)
    r64 = run_precision(gl, torch, gl.F64, n, args.steps, args.warmup, fields)

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
        "stages_ms": r32["stages_ms"],
        "variants": r32["variants"],
        "fp64": r64,
        "roofline": roof,
        "solve_roofline": solve_roofline(n, r32["ms_per_step"], r64["ms_per_step"]),
    }
    if not args.no_extra:
        out["seed_spread"] = seed_spread(gl, torch, n, max(20, args.steps // 2), args.warmup, r32["value"])
        out["amr"] = amr_leg(gl, torch, max(10, args.steps // 4))
        out["paper_amr"] = paper_amr_leg(gl, torch, max(5, args.steps // 20))
        out["offplane"] = offplane_leg(gl, torch, max(10, args.steps // 4), fields, n)
        out["batch"] = batch_leg(gl, torch, max(5, args.steps // 20))
        out["serve"] = serve_leg(gl, torch, nreq=max(200, 10 * args.steps))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, fields, with_amr=not args.no_extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
