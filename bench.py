#!/usr/bin/env python3
"""Benchmark of the reference-map band extrapolation on one MI355X.

One step = one full call of the hot path (classify, label, normals, L layer fits) over
one synthetic workload already resident in HBM.  Default workload: the 256^3 cavity
sphere (L = 4, FP64).  Prints ONE JSON line with throughput (band cells/s), the roofline
of the dominant kernel (timed live with HIP events on the launch stream), the whole-call
roofline, the CPU oracle timed on this host's cores, and the extra forms (FP32
accumulate, batched vs per-solid suspension) under "variants".
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
METRIC = "band cells extrapolated/s & % HBM roofline; p50/p99 latency, batched vs plain"
PRECISIONS = {"fp64": 0, "fp32acc": 1}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def band_and_box(stats, w):
    nb = sum(sum(s["n_band"][1:17]) for s in stats)
    return nb, w.box_cells


def time_calls(ctx, dw, opt, steps, warmup):
    """Average ms per call over `steps` back-to-back calls, timed with HIP events on the
    stream the library launches on, bracketed by device synchronisation."""
    import torch
    from paper_2104_00095_amd import rmx
    arr = dw.array()
    stream = torch.cuda.current_stream()
    h = rmx._stream_handle(stream)
    n = len(dw.solids)
    for _ in range(warmup):
        st = ctx.extrapolate_raw(dw.grid, arr, n, opt, h)
        if st < 0:
            raise rmx.RmxError(st, "warmup")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.extrapolate_raw(dw.grid, arr, n, opt, h)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def profile_phases(ctx, dw, opt, steps):
    """Per-phase (total ms, launches) over `steps` profiled calls, from HIP events placed
    around every launch on the launch stream."""
    import torch
    from paper_2104_00095_amd import rmx
    popt = rmx.options(opt.r_s, opt.r_max, opt.normal_layers, opt.precision,
                       (opt.flags & ~rmx.FLAG_GRAPH) | rmx.FLAG_PROFILE)
    ctx.profile_read()
    arr = dw.array()
    h = rmx._stream_handle(torch.cuda.current_stream())
    for _ in range(steps):
        ctx.extrapolate_raw(dw.grid, arr, len(dw.solids), popt, h)
    torch.cuda.synchronize()
    return ctx.profile_read()


# Phases of the profiler -> the kernel that runs them (each layer's fit is one launch of
# the same fit kernel).
KERNEL_NAMES = {"classify": "k_classify", "label": "k_label", "normal": "k_normal",
                "extrap": "k_extrap", "band": "k_band"}


def kernel_of(phase):
    return "extrap" if phase.startswith("extrap") else phase


def classify_bytes(w):
    """Bytes the classification must read under its exact early-out rule: xi_x of every
    cell, xi_y where dx^2 < T, xi_z where dx^2 + dy^2 < T (T = R^2 for a sphere,
    e_max^2 (1 + 1e-6) for an ellipsoid; the same operation order as the kernel), plus
    the 1-bit mask written."""
    import numpy as np
    total = 0.0
    for s in w.solids:
        c = s.shape.centre
        T = float(s.shape.semi[0]) ** 2 if s.shape.kind == 1 else \
            float(np.max(s.shape.semi)) ** 2 * (1.0 + 1e-6)
        with np.errstate(invalid="ignore"):
            dx = s.xi[0] - c[0]
            p = dx * dx
            ny = p < T
            dy = s.xi[1] - c[1]
            p2 = p + dy * dy
            nz = ny & (p2 < T)
        cells = s.xi[0].size
        total += 8.0 * cells + 8.0 * float(ny.sum()) + 8.0 * float(nz.sum()) + cells / 8.0
    return total


KERNEL_SOURCES = ("paper_2104_00095_amd/csrc/rmx_kernels.hip",
                  "paper_2104_00095_amd/csrc/rmx_device.h",
                  "paper_2104_00095_amd/csrc/rmx_internal.h")


def _code_only(text):
    """Source text without comments and whitespace (string and character literals kept):
    what changes the compiled kernels."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def kernel_source_hash():
    """SHA-256 of the kernel sources' code (comments and whitespace ignored)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def committed_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE counters, each scaled
    by the same counter on a plain device copy of known size) from the committed summary
    profiles/<kernel>_<workload>_counters.md, if it was taken on the current kernel
    code; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def model_bytes(kernel, w, stats):
    """The call's algorithmic HBM bytes attributed to a kernel by the byte model
    B = 24 |D| + 1 |D| + 24 N_band: classification reads xi of every box cell once (24 B),
    labelling writes one int8 label per box cell, and the fits write 24 B per band cell.
    The normal kernel moves nothing the model counts (None)."""
    cells = w.box_cells
    nb = sum(sum(s["n_band"][1:17]) for s in stats)
    return {"classify": 24.0 * cells, "label": 1.0 * cells, "normal": None,
            "extrap": 24.0 * nb, "band": 24.0 * nb}[kernel]


def kernel_table(phases, calls, w, stats, cls_bytes):
    """Per kernel: time per call, launches per call, average launch duration, the byte
    model's bytes per call and per launch, and the achieved fraction of the HBM peak."""
    agg = {}
    for ph, (ms, n) in phases.items():
        k = kernel_of(ph)
        a = agg.setdefault(k, [0.0, 0])
        a[0] += ms
        a[1] += n
    out = {}
    for k, (ms, n) in agg.items():
        b = model_bytes(k, w, stats)
        lpc = n / calls
        e = {"kernel": KERNEL_NAMES[k], "ms_per_call": ms / calls, "launches_per_call": lpc,
             "avg_launch_ms": ms / n, "model_bytes_per_call": b}
        if b is not None:
            e["model_bytes_per_launch"] = b / lpc
            e["hbm_frac"] = b / (ms / calls * 1e-3) / (HBM_PEAK_GBS * 1e9)
        out[k] = e
    if "classify" in out:
        # the exact early-out reads only what the predicate needs (fewer bytes than the
        # model's 24 B per cell on a sphere)
        e = out["classify"]
        e["early_out_bytes"] = cls_bytes
        e["early_out_hbm_frac"] = cls_bytes / (e["avg_launch_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, seconds, gpu=None, r_s=2, r_max=4, normal_layers=2):
    """The oracle as it stands, on this host's cores, on whole calls of the same workload
    until `seconds` of CPU work have run (at least one call); then the same on one thread
    for half as long.  `gpu`: {precision: per-solid (xi, labels) of one GPU call on the same
    input}; the oracle's output of its first call is compared with them (labels equal;
    relative max-norm error of xi over the band)."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    probs = [oracle.make_problem(w.grid_n, s.lo, s.ext,
                                 oracle.make_shape(s.shape.kind, s.shape.centre, s.shape.semi,
                                                   s.shape.rot),
                                 s.n_layers, r_s=r_s, r_max=r_max, normal_layers=normal_layers)
             for s in w.solids]

    def run(threads, secs, keep):
        calls, band, t0 = 0, 0, time.perf_counter()
        first = None
        while True:
            outs = []
            for p, s in zip(probs, w.solids):
                st, xo, lab, dec, stats = oracle.extrapolate(p, s.xi, nthreads=threads)
                band += int(stats[1:17].sum())
                if keep and first is None:
                    outs.append((xo, lab))
            if keep and first is None:
                first = outs
            calls += 1
            el = time.perf_counter() - t0
            if el >= secs:
                return band / el, calls, el, first

    rate, calls, el, first = run(cores, seconds, True)
    rate1, calls1, el1, _ = run(1, seconds / 2, False)
    res = {"value": rate, "unit": "band cells/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{calls} whole calls of {w.name} ({len(w.solids)} solid(s)), "
                     f"{el:.1f} s wall, OpenMP threads = {cores}",
           "one_thread": {"value": rate1, "unit": "band cells/s",
                          "sample": f"{calls1} whole calls, {el1:.1f} s wall, 1 thread"}}
    for prec, g in (gpu or {}).items():
        worst, same = 0.0, True
        for (xo, lo), (xg, lg) in zip(first, g):
            same &= bool(np.array_equal(lo, lg))
            worst = max(worst, rel_err(xg, xo, lo > 0))
        name = "fp64" if prec == 0 else "fp32acc"
        res[f"gpu_{name}_labels_equal"] = same
        res[f"gpu_{name}_rel_max_err"] = worst
    return res


def copy_calibration(n_bytes=1 << 30, reps=5):
    """A plain device-to-device copy of n_bytes (read n_bytes, write n_bytes), `reps`
    times: under a counter profiler, its FETCH_SIZE and WRITE_SIZE per dispatch against
    n_bytes give the scale of those counters."""
    import torch
    src = torch.ones(n_bytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": n_bytes, "copy_bytes_written": n_bytes,
                      "ms": ms, "GB_per_s": 2 * n_bytes / (ms * 1e-3) / 1e9}), flush=True)


def rel_err(a, b, band):
    import numpy as np
    if not band.any():
        return 0.0
    return float(np.max(np.abs(a[:, band] - b[:, band])) / np.max(np.abs(b[:, band])))


def gpu_outputs(ctx, w, precision):
    """One call on a fresh copy of the workload; host copies of xi and labels per solid."""
    import torch
    from paper_2104_00095_amd import fields, rmx
    dw = fields.upload(w)
    ctx.extrapolate(dw.grid, dw.solids, rmx.options(precision=precision), check=False)
    torch.cuda.synchronize()
    out = [(dw.xi[i].cpu().numpy(), dw.labels[i].cpu().numpy()) for i in range(len(w.solids))]
    del dw
    torch.cuda.empty_cache()
    return out


def serving_variants(ctx, n_requests=2000, rate=200.0, n_streams=4, log=print):
    """The serving trace (simulations of grids 32..192^3 with 1-64 ellipsoids, Poisson
    arrivals) through the request loop, against the plain form (requests in arrival order,
    one solid at a time).  Latency = completion - arrival.  Fields live on the device:
    generated there (same formula as the host generator), then resident."""
    import queue
    import threading
    import numpy as np
    import torch
    from paper_2104_00095_amd import rmx, synth, synth_device
    sims, reqs = synth.serving_trace(rate=rate)
    reqs = reqs[:n_requests]
    layouts = [synth.sim_layout(sp)[0] for sp in sims]
    opts = [rmx.options(precision=sp.precision) for sp in sims]
    resident = sum(25 * int(np.prod(sp.ext)) for lay in layouts for sp in lay)

    def fill(srv, ids):
        for sp, sid, lay in zip(sims, ids, layouts):
            for j, spec in enumerate(lay):
                srv.upload(sid, j, synth_device.affine_sine_field(spec, 1.0 / sp.n))
        torch.cuda.synchronize()

    def serve(budget, saturated):
        srv = rmx.Server(0, budget, n_streams)
        try:
            ids = []
            for sp, lay in zip(sims, layouts):
                templ = [rmx.solid_template(q.lo, q.ext, rmx.shape(q.shape.kind, q.shape.centre,
                                                                    q.shape.semi, q.shape.rot),
                                            q.n_layers) for q in lay]
                ids.append(srv.register(rmx.grid((sp.n,) * 3, 1.0 / sp.n), templ))
            fill(srv, ids)
            done = queue.Queue()
            band, comp, errors = [0] * len(reqs), [0.0] * len(reqs), []

            def waiter():
                while True:
                    item = done.get()
                    if item is None:
                        return
                    t, i, t_sub = item
                    st, l, stats = srv.wait(t, len(layouts[reqs[i].sim_id]))
                    if st < 0:
                        errors.append((i, st))
                    comp[i] = t_sub + l
                    band[i] = sum(sum(x["n_band"][1:17]) for x in stats)

            th = threading.Thread(target=waiter)
            th.start()
            t0 = time.perf_counter()
            for i, r in enumerate(reqs):
                if not saturated:
                    dt = t0 + r.arrival_s - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                t_sub = time.perf_counter()
                t = srv.submit(ids[r.sim_id], opts[r.sim_id])
                done.put((t, i, t_sub))
            done.put(None)
            th.join()
            if errors:
                raise RuntimeError(f"served requests failed: {errors[:5]}")
            arr = [t0 + (0.0 if saturated else r.arrival_s) for r in reqs]
            lat = np.array([c - a for c, a in zip(comp, arr)])
            span = max(comp) - t0
            used, peak = srv.usage()
        finally:
            srv.close()
        return {"p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "mean_ms": 1e3 * float(lat.mean()), "span_s": span,
                "band_cells_per_s": float(sum(band)) / span,
                "requests_per_s": len(reqs) / span, "hbm_budget_bytes": budget,
                "peak_admitted_bytes": peak}

    def plain(saturated):
        # the same fields, owned by a server (admission out of play), driven one solid at a
        # time in arrival order through a context
        srv = rmx.Server(0, 1 << 40, 1)
        try:
            ids, solids = [], []
            for sp, lay in zip(sims, layouts):
                templ = [rmx.solid_template(q.lo, q.ext, rmx.shape(q.shape.kind, q.shape.centre,
                                                                    q.shape.semi, q.shape.rot),
                                            q.n_layers) for q in lay]
                sid = srv.register(rmx.grid((sp.n,) * 3, 1.0 / sp.n), templ)
                ids.append(sid)
                row = []
                for j, t in enumerate(templ):
                    xp, lp = srv.field(sid, j)
                    t.xi = ctypes.c_void_p(xp)
                    t.labels = ctypes.c_void_p(lp)
                    row.append((rmx.Solid * 1)(t))
                solids.append(row)
            fill(srv, ids)
            grids = [rmx.grid((sp.n,) * 3, 1.0 / sp.n) for sp in sims]
            stats = (rmx.SolidStats * 1)()
            lat, band = [], 0
            t0 = time.perf_counter()
            for r in reqs:
                arrive = t0 + (0.0 if saturated else r.arrival_s)
                dt = arrive - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                for arr in solids[r.sim_id]:
                    st = rmx.lib().rmx_extrapolate(ctx.h, ctypes.byref(grids[r.sim_id]), arr, 1,
                                                   ctypes.byref(opts[r.sim_id]), None, stats)
                    if st < 0:
                        raise RuntimeError(f"plain call failed: {st}")
                    band += sum(stats[0].n_band[1:17])
                lat.append(time.perf_counter() - arrive)
            span = time.perf_counter() - t0
        finally:
            srv.close()
        lat = np.array(lat)
        return {"p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "mean_ms": 1e3 * float(lat.mean()), "span_s": span,
                "band_cells_per_s": band / span, "requests_per_s": len(reqs) / span}

    out = {"requests": len(reqs), "simulations": len(sims), "rate_per_s": rate,
           "streams": n_streams, "resident_field_bytes": resident}
    log("serving: trace replay, tight budget")
    out["served_4GiB"] = serve(4 << 30, False)
    log("serving: trace replay, plain")
    out["plain"] = plain(False)
    log("serving: saturated")
    out["served_saturated_64GiB"] = serve(64 << 30, True)
    out["plain_saturated"] = plain(True)
    return out


def step_variant(ctx, steps=100, warmup=10, n_layers=6, precision=0):
    """One time step (rmx_step: predictor, extrapolation from the predicted interior,
    corrector) on cavity256 with L = 6, advected by the cavity's own flow (plus a drift
    along z) at CFL 0.4.  Set-up, not timed: the band of step n by one extrapolation call.
    Timed: `steps` steps from the same state (xi^n is an input, so every step does the same
    work), HIP events on the launch stream; per-kernel times from RMX_FLAG_PROFILE.
    Byte model of the step's own kernels (transverse faces, faces, predictor, corrector;
    the extrapolation chain keeps its own): per predicted cell 96 B (xi^n, u^n and the face
    velocities read, xi^{n+1} written), per box cell 1 B of labels read and 1/8 B of mask
    written, per cell labelled at n + 1 74 B (two labels, xi^n and xi^{n+1} read, xi^{n+1/2}
    written).  The face-state scratch the kernels pass between them is not counted."""
    import numpy as np
    import torch
    from paper_2104_00095_amd import fields, rmx, synth
    w = synth.cavity256(n_layers=n_layers)
    dw = fields.upload(w)
    st, stats = ctx.extrapolate(dw.grid, dw.solids, rmx.options())
    assert st == 0
    # launch shapes (label tile width, fit blocks) tuned on this machine's extrapolation; the
    # step's chain plans the same boxes and layers, so it takes them too
    tuned = ctx.autotune(dw.grid, dw.solids, rmx.options(precision=precision), reps=5)
    vel = synth.step_velocity(w)
    dt = synth.step_dt(w, 0.4)
    s = w.solids[0]
    dev = "cuda"
    xi_n = dw.xi[0]
    lab_n = dw.labels[0]
    u = torch.from_numpy(vel[0].u).to(dev)
    uf = tuple(torch.from_numpy(f).to(dev) for f in vel[0].uf)
    xi_next = torch.zeros_like(xi_n)
    lab_next = torch.zeros_like(lab_n)
    xi_half = torch.zeros_like(xi_n)
    shp = rmx.shape(s.shape.kind, s.shape.centre, s.shape.semi, s.shape.rot)
    sol = rmx.step_solid(s.lo, s.ext, shp, s.n_layers, xi_n, lab_n, u, uf, xi_next, lab_next,
                         xi_half)
    arr = (rmx.StepSolid * 1)(sol)
    opt = rmx.options(precision=precision)
    stream = torch.cuda.current_stream()
    h = rmx._stream_handle(stream)
    st, sstats = ctx.step(dw.grid, [sol], dt, opt)
    assert st == 0, st
    for _ in range(warmup):
        ctx.step_raw(dw.grid, arr, 1, opt, dt, h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.step_raw(dw.grid, arr, 1, opt, dt, h)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # per-kernel times
    ctx.profile_read()
    popt = rmx.options(precision=precision, flags=rmx.FLAG_PROFILE)
    reps = max(10, steps // 5)
    for _ in range(reps):
        ctx.step_raw(dw.grid, arr, 1, popt, dt, h)
    torch.cuda.synchronize()
    ph = ctx.profile_read()
    # cell counts for the byte models (host, from the labels of both steps)
    ln = lab_n.cpu().numpy()
    lx = lab_next.cpu().numpy()
    L = n_layers
    e2, e1_, e0_ = ln.shape
    k, j, i = np.meshgrid(np.arange(e2), np.arange(e1_), np.arange(e0_), indexing="ij")
    inside = (i >= 3) & (i <= e0_ - 4) & (j >= 3) & (j <= e1_ - 4) & (k >= 3) & (k <= e2 - 4)
    n_pred = int(((ln >= 0) & (ln <= L - 4) & inside).sum())
    n_trans = int(((ln >= 0) & (ln <= L - 2)).sum())
    n_corr = int(((lx >= 0) & (lx <= L)).sum())
    box = ln.size
    nb = int(((lx >= 1) & (lx <= L)).sum())
    kern = {name: {"avg_launch_ms": tms / n, "launches_per_step": n / reps}
            for name, (tms, n) in ph.items()}
    own = ("step_trans", "step_faces", "step_predict", "step_correct")
    own_ms = sum(kern[k]["avg_launch_ms"] * kern[k]["launches_per_step"] for k in own)
    own_bytes = 96.0 * n_pred + 1.125 * box + 74.0 * n_corr
    dom = max(own, key=lambda k: kern[k]["avg_launch_ms"])
    out = {"workload": f"step_cavity256_L{L}", "ms_per_step": ms,
           "predicted_cells": n_pred, "transverse_cells": n_trans, "band_cells": nb,
           "box_cells": box,
           "predicted_cells_per_s": n_pred / (ms * 1e-3), "band_cells_per_s": nb / (ms * 1e-3),
           "dt": dt, "precision": precision, "launch_shapes": tuned, "kernels": kern,
           "step_roofline": {"bound": "hbm", "kernels": list(own), "dominant": f"k_{dom}",
                             "algorithmic_bytes": own_bytes, "ms": own_ms,
                             "achieved": own_bytes / (own_ms * 1e-3) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": own_bytes / (own_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}}
    del dw, u, uf, xi_next, lab_next, xi_half
    torch.cuda.empty_cache()
    return out


def blur_variant(ctx, name, steps=50, warmup=5, eps_cells=2.0):
    """The blur-zone consumers on a workload after its extrapolation (set-up, not timed):
    rmx_blur (phi of every solid and the multi-body modified Heaviside on the grid) and
    rmx_solid_stress (the blended neo-Hookean stress on the faces), each timed over `steps`
    calls with HIP events on the launch stream.  Byte models: rmx_blur writes 8 B of H per
    grid cell inside some box and reads 1 B of labels per box cell, plus 24 B of xi read and
    8 B of phi written per covered cell; rmx_solid_stress writes 48 B per face with a cell
    inside some box, plus 1 B of labels per box cell and 24 B of xi per covered cell read
    once.  (Covered: labelled 0..L.)"""
    import numpy as np
    import torch
    from paper_2104_00095_amd import fields, rmx
    w = make_workload(name)
    dw = fields.upload(w)
    st, stats = ctx.extrapolate(dw.grid, dw.solids, rmx.options())
    assert st == 0, st
    n0, n1, n2 = w.grid_n
    H = torch.ones((n2, n1, n0), dtype=torch.float64, device="cuda")
    phis = [torch.zeros(tuple(x.shape[1:]), dtype=torch.float64, device="cuda") for x in dw.xi]
    taus = [torch.zeros((6, n2 + (a == 2), n1 + (a == 1), n0 + (a == 0)), dtype=torch.float64,
                        device="cuda") for a in range(3)]
    eps = eps_cells * w.h
    G = [1.0] * len(w.solids)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the checked calls once (sizes, statuses), then timing through prebuilt arrays, as a
    # stepping loop that keeps its descriptors would call
    ctx.blur(dw.grid, dw.solids, eps, H, phis, stream)
    ctx.solid_stress(dw.grid, dw.solids, eps, G, taus, stream)
    import ctypes
    arr = dw.array()
    n = len(dw.solids)
    pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in phis])
    tp = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in taus])
    Ga = (ctypes.c_double * n)(*G)
    sh = ctypes.c_void_p(stream.cuda_stream)
    hp = ctypes.c_void_p(H.data_ptr())

    def call_h():
        assert ctx.blur_raw(dw.grid, arr, n, eps, hp, pp, sh) == 0

    def call_t():
        assert ctx.solid_stress_raw(dw.grid, arr, n, eps, Ga, tp, sh) == 0

    ms_h = timed(call_h)
    ms_t = timed(call_t)
    # byte models
    inbox = np.zeros((n2, n1, n0), bool)
    box_cells = covered = 0
    for s, lab in zip(w.solids, dw.labels):
        lo, e = s.lo, s.ext
        inbox[lo[2]:lo[2] + e[2], lo[1]:lo[1] + e[1], lo[0]:lo[0] + e[0]] = True
        box_cells += int(np.prod(e))
        lh = lab.cpu().numpy()
        covered += int(((lh >= 0) & (lh <= s.n_layers)).sum())
    n_cells = int(inbox.sum())
    faces = 0
    for a in range(3):
        f = np.zeros((n2 + (a == 2), n1 + (a == 1), n0 + (a == 0)), bool)
        sl_lo = [slice(0, n2), slice(0, n1), slice(0, n0)]
        sl_hi = list(sl_lo)
        sl_hi[2 - a] = slice(1, [n2, n1, n0][2 - a] + 1)
        f[tuple(sl_lo)] |= inbox
        f[tuple(sl_hi)] |= inbox
        faces += int(f.sum())
    b_h = 8.0 * n_cells + box_cells + 32.0 * covered
    b_t = 48.0 * faces + box_cells + 24.0 * covered
    pk = HBM_PEAK_GBS * 1e9
    out = {"workload": f"blur_{name}", "solids": len(w.solids), "eps_cells": eps_cells,
           "grid_cells_in_boxes": n_cells, "faces_written": faces, "covered_cells": covered,
           "blur": {"ms": ms_h, "model_bytes": b_h, "hbm_frac": b_h / (ms_h * 1e-3) / pk},
           "solid_stress": {"ms": ms_t, "model_bytes": b_t,
                            "hbm_frac": b_t / (ms_t * 1e-3) / pk}}
    del dw, H, phis, taus
    torch.cuda.empty_cache()
    return out


def make_workload(name):
    from paper_2104_00095_amd import synth
    if name == "cavity256":
        return synth.cavity256()
    if name == "ellipsoid128":
        return synth.ellipsoid128()
    if name == "suspension":
        return synth.suspension()
    if name == "sphere32":
        return synth.sphere32()
    if name == "periodic_box":
        # the suspension's size, with unequal spacings and periodic x and z
        return synth.periodic_box(seed=9, grid_n=(128, 128, 256),
                                  spacing=(1.0 / 128, 1.0 / 96, 1.0 / 192), n_solids=40,
                                  n_layers=4, semi_lo=0.04, semi_hi=0.1)
    raise SystemExit(f"unknown workload {name}")


def run_form(ctx, w, dw, opt, steps, warmup):
    st, stats = ctx.extrapolate(dw.grid, dw.solids, opt)
    nb, cells = band_and_box(stats, w)
    ms, wall = time_calls(ctx, dw, opt, steps, warmup)
    B = 25 * cells + 24 * nb
    return {"ms_per_call": ms, "host_ms_per_call": wall, "band_cells": nb,
            "band_cells_per_s": nb / (ms * 1e-3),
            "call_hbm_frac": B / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}, stats


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cavity256")
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--graph", action="store_true", help="replay the launch chain as a hipGraph")
    ap.add_argument("--step-only", action="store_true",
                    help="only time the time-step variant (predictor + extrapolation + "
                         "corrector on cavity256, L = 6) and print it")
    ap.add_argument("--blur-only", action="store_true",
                    help="only time the blur-zone consumers (suspension and cavity256)")
    ap.add_argument("--persistent", action="store_true",
                    help="the band work (normals and every layer's fits) in one persistent launch")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--shapes", default=None,
                    help="TILE_W,EXTRAP_BLOCKS: use these launch shapes instead of autotuning "
                         "(for profiles: only the timed shapes are launched)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (the reference for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters) and print its rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (solids are "
              "independent, so a batch would split by solid across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_00095_amd import fields, rmx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.blur_only:
        ctx = rmx.Context(0)
        for wl in ("suspension", "cavity256"):
            log(f"blur-zone consumers ({wl})")
            print(json.dumps(blur_variant(ctx, wl, max(10, args.steps // 4))), flush=True)
        ctx.close()
        return
    if args.step_only:
        ctx = rmx.Context(0)
        log("time step (cavity256, L = 6)")
        print(json.dumps(step_variant(ctx, args.steps, args.warmup,
                                      precision=PRECISIONS[args.precision])), flush=True)
        ctx.close()
        return

    log(f"generating {args.workload}")
    w = make_workload(args.workload)
    dw = fields.upload(w)
    ctx = rmx.Context(0)
    prec = PRECISIONS[args.precision]
    flags = (rmx.FLAG_GRAPH if args.graph else 0) | (rmx.FLAG_PERSISTENT if args.persistent else 0)
    opt = rmx.options(precision=prec, flags=flags)
    tuned = None
    if args.shapes:
        tw, eb = (int(v) for v in args.shapes.split(","))
        ctx.set_tuning(dw.grid, dw.solids, tw, eb, rmx.options(precision=prec))
        tuned = {"tile_w": tw, "extrap_blocks": eb, "ms": None}
    elif not args.no_autotune:
        log("autotune (label tile width, blocks per layer fit)")
        tuned = ctx.autotune(dw.grid, dw.solids, rmx.options(precision=prec), reps=5)
    log("timing")
    main_form, stats = run_form(ctx, w, dw, opt, args.steps, args.warmup)
    nb, cells = band_and_box(stats, w)
    ms = main_form["ms_per_call"]

    log("profiling kernels")
    prof_calls = max(10, min(args.steps, 50))
    phases = profile_phases(ctx, dw, opt, prof_calls)
    cb = classify_bytes(w)
    kt = kernel_table(phases, prof_calls, w, stats, cb)
    # the dominant kernel: the most time per call (summed over its launches)
    dom = max(kt, key=lambda k: kt[k]["ms_per_call"])
    d = kt[dom]
    if d["model_bytes_per_call"] is None:
        roof = {"bound": "latency", "kernel": d["kernel"], "achieved": None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}
    else:
        per_launch = d["model_bytes_per_launch"]
        roof = {"bound": "hbm", "kernel": d["kernel"],
                "achieved": per_launch / (d["avg_launch_ms"] * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "traffic": committed_traffic(d["kernel"], args.workload),
                "bytes_per_launch": per_launch, "avg_launch_ms": d["avg_launch_ms"],
                "launches_per_call": d["launches_per_call"],
                "byte_model": {"classify": "24 B read per box cell",
                               "label": "1 B written per box cell",
                               "extrap": "24 B written per band cell of the layer",
                               "band": "24 B written per band cell"}[dom]}
        roof["frac"] = roof["achieved"] / roof["peak"]
    B = 25 * cells + 24 * nb

    variants = {}
    if not args.no_variants:
        log("variants")
        other = 1 - prec
        o2 = rmx.options(precision=other, flags=flags)
        f2, _ = run_form(ctx, w, dw, o2, args.steps, args.warmup)
        variants[[k for k, v in PRECISIONS.items() if v == other][0]] = f2
        # layers by the 26-neighbour adjacency on the same fields (more band cells)
        fa, _ = run_form(ctx, w, dw, rmx.options(precision=prec, flags=flags | rmx.FLAG_ADJ26),
                         args.steps, args.warmup)
        variants["adj26"] = fa
        del dw
        torch.cuda.empty_cache()
        ws = make_workload("suspension")
        dws = fields.upload(ws)
        for name, fl in (("suspension_batched_graph", rmx.FLAG_GRAPH),
                         ("suspension_batched", 0),
                         ("suspension_per_solid", rmx.FLAG_PER_SOLID)):
            f, _ = run_form(ctx, ws, dws, rmx.options(flags=fl), max(20, args.steps // 4), 5)
            f["solids"] = len(ws.solids)
            variants[name] = f
        del dws
        ws = make_workload("sphere32")
        dws = fields.upload(ws)
        for name, fl in (("sphere32_graph", rmx.FLAG_GRAPH), ("sphere32", 0)):
            f, _ = run_form(ctx, ws, dws, rmx.options(flags=fl), args.steps, args.warmup)
            variants[name] = f
        del dws
        ws = make_workload("ellipsoid128")
        dws = fields.upload(ws)
        for name, pr in (("ellipsoid128_fp64", 0), ("ellipsoid128_fp32acc", 1)):
            f, _ = run_form(ctx, ws, dws, rmx.options(precision=pr), args.steps, args.warmup)
            variants[name] = f
        del dws
        # method variants: periodic x and z with unequal spacings, then the same boxes and
        # fields with equal spacings (the cost of the spacing-aware normal factor)
        ws = make_workload("periodic_box")
        for name, sp in (("periodic_box_unequal", ws.spacing), ("periodic_box_equal", None)):
            ws.spacing = sp if sp is not None else (0.0, 0.0, 0.0)
            dws = fields.upload(ws)
            f, _ = run_form(ctx, ws, dws, rmx.options(), max(20, args.steps // 4), 5)
            f["solids"] = len(ws.solids)
            variants[name] = f
            del dws
        torch.cuda.empty_cache()
        log("variants: time step")
        variants["step_cavity256"] = step_variant(ctx, args.steps, args.warmup)
        log("variants: blur-zone consumers")
        for wl in ("suspension", "cavity256"):
            variants[f"blur_{wl}"] = blur_variant(ctx, wl, max(10, args.steps // 4))
        if not args.no_serving:
            variants["serving"] = serving_variants(ctx, args.serving_requests, log=log)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        gpu = {p: gpu_outputs(ctx, w, p) for p in (0, 1)}
        cpu = cpu_baseline(w, args.cpu_seconds, gpu)

    out = {
        "metric": METRIC,
        "value": nb / (ms * 1e-3),
        "unit": "band cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(w.grid_n), "solids": len(w.solids),
                   "n_layers": max(s.n_layers for s in w.solids), "band_cells": nb,
                   "box_cells": cells, "precision": args.precision, "graph": args.graph,
                   "persistent": args.persistent,
                   "launch_shapes": tuned},
        "roofline": roof,
        "call_roofline": {"bound": "hbm", "algorithmic_bytes": B,
                          "achieved": B / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": B / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)},
        "kernels": kt,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
