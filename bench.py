#!/usr/bin/env python3
"""Benchmark: visibilities/s for one grid + one degrid call on one MI355X.

A step is one pass of the whole hot path over the wide-field workload
(2048^2 image, L = 0.4, W = 7, x0 = 0.25, 9,999,360 visibilities from 64
antennas in a 5 km disc, +-1 h, declination -30 deg, 1.4 GHz scaled so the
image is Nyquist-sampled; complex N(0, 1) visibility values, N(0, 1) image):
grid_visibilities followed by degrid_visibilities, FP32 arithmetic with FP64
coordinates, phases and tables.  Inputs are resident in HBM before timing.

Printed: one JSON line with the metric, the FP64 path's figures, per-stage
HIP-event times, the roofline of the dominant kernel and the CPU oracle's
throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_stats(uvw, N: int, L: float, W: int, x0: float, wmax: float, Np: int, nl: int, t_lo: int,
                   n_scale: float) -> dict:
    """Counts that fix the algorithmic bytes of the sparse stack (host numpy, no oracle).

    A visibility's first support index per axis is floor(xi + W/2) - W + 1 with
    xi = (l_max / x0) u, (l_max / x0) v, n_scale w after the Hermitian fold;
    bins are 16^3 tiles of the stack.  A tile is occupied when some visibility
    reaches it (what the library writes and reads); a visibility visits
    1 + [first index in tile >= 17 - W] tiles per axis.
    """
    import numpy as np

    u, v, w = (uvw[:, i].astype(np.float64) for i in range(3))
    neg = w < 0
    u, v, w = np.where(neg, -u, u), np.where(neg, -v, v), np.abs(w)
    umul = (L / 2) / x0
    fu = (np.floor(umul * u + W / 2).astype(np.int64) - W + 1) % Np
    fv = (np.floor(umul * v + W / 2).astype(np.int64) - W + 1) % Np
    ft = np.floor(n_scale * w + W / 2).astype(np.int64) - W + 1 - t_lo
    T = 16
    nb, nbt = Np // T, (nl + T - 1) // T
    B = 17 - W
    ct, cv, cu = ft % T >= B, fv % T >= B, fu % T >= B
    visits = int(np.sum((1 + ct) * (1 + cu) * (1 + cv)))
    occ = np.zeros((nbt, nb, nb), dtype=bool)          # tiles some visibility reaches
    for it in (0, 1):
        for iv in (0, 1):
            for iu in (0, 1):
                m = np.ones(ft.size, dtype=bool)
                if it:
                    m &= ct
                if iv:
                    m &= cv
                if iu:
                    m &= cu
                occ[ft[m] // T + it, (fv[m] // T + iv) % nb, (fu[m] // T + iu) % nb] = True
    cells_per_t = np.array([min(T, nl - T * i) for i in range(nbt)]) * T * T
    occ_cells = int(np.sum(occ.sum(axis=(1, 2)) * cells_per_t))
    rows = occ.any(axis=1)                              # [t tile][u tile]: any tile along v
    row_lines = int(np.sum(rows.sum(axis=1) * np.array([min(T, nl - T * i) for i in range(nbt)]) * T))
    return {"tiles_occupied": int(occ.sum()), "tiles": int(occ.size), "occupied_cells": occ_cells,
            "tile_visits": visits, "nonempty_lines": row_lines, "lines": nl * Np}


def stage_bytes(st: str, M: int, N: int, Np: int, nl: int, f64: bool, ws: dict, prepared: bool = False) -> float:
    """Algorithmic HBM bytes of one launch of a stage (what the stage must move)."""
    b = 16 if f64 else 8            # complex
    r = 8 if f64 else 4             # real
    rec = 56 if f64 else 32         # binned record
    tiles = ws["occupied_cells"] * b                    # occupied tiles of the stack
    inter_rows = ws["nonempty_lines"] * N * b           # intermediate lines that meet an occupied tile
    sort = 2 * M * rec                                  # per-bin sort: records in and out
    return {
        "grid_bin": M * (2 * 24 + b + rec) + sort,      # uvw read twice, vis, records written, sorted
        # records in (once per tile reached), tiles out; on a shared binning each visit also
        # reads the visibility the record names
        "grid_tiles": ws["tile_visits"] * (rec + (b if prepared else 0)) + tiles,
        "grid_fft_v": tiles + inter_rows,               # occupied tiles in, lines of occupied rows out
        "grid_transpose": inter_rows + inter_rows,      # live lines in and out (the others are zero)
        "degrid_transpose": inter_rows + inter_rows,    # lines the transform along q needs, in and out
        "grid_fft_u": inter_rows + 2 * N * N * r,       # live intermediate, correction in, map out
        "degrid_bin": M * (2 * 24 + rec) + sort,
        "degrid_fft_p": 2 * N * N * r + inter_rows,     # image, correction in, live intermediate out
        "degrid_fft_q": inter_rows + tiles,             # intermediate rows in, occupied tiles out
        # tiles and records in, one part out per visit; then per record its parts in, the visibility out
        "degrid_tiles": tiles + ws["tile_visits"] * (rec + b) + M * rec + ws["tile_visits"] * b + M * b,
    }[st]


def source_digest() -> str:
    """Digest of the device sources with comments and blank space removed, so
    that a comment edit does not disown the counters taken on them."""
    import re

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_11172_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith((".hpp", ".hip", ".inl")):
            continue
        text = open(os.path.join(csrc, f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def workload_key(name: str, N: int, W: int, x0: float, M: int, n_layers: int, pass_layers: int) -> str:
    """Names the workload and layer-pass size a counter run was taken on (counters hold for that one only)."""
    return f"{name} N={N} W={W} x0={x0:.6g} M={M} layers={n_layers} pass={pass_layers}"


def counters(key: str):
    """The committed rocprofv3 counter summary, if it was taken on the current
    sources and on this workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("source_digest") != source_digest() or t.get("workload") != key:
        return None
    return t


def traffic_for(kernel: str, prec: str, key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on the current sources."""
    t = counters(key)
    return None if t is None else t.get("per_launch_bytes", {}).get(f"{kernel}:{prec}")


def issue_for(kernel: str, prec: str, key: str):
    """VALU wave instructions per launch and their issue time from committed
    rocprofv3 counter runs, if taken on the current sources (a wave64 VALU
    instruction holds a SIMD for 4 cycles: 1024 SIMDs at 2.4 GHz)."""
    t = counters(key)
    if t is None:
        return None
    n = t.get("valu_per_launch", {}).get(f"{kernel}:{prec}")
    if n is None:
        return None
    return {"valu_instr_per_launch": n, "valu_issue_ms": 4.0 * n / (1024 * 2.4e9) * 1e3}


def cpu_baseline(w: dict, n_sample: int) -> dict:
    """The FP64 oracle, as written, timed on a bounded sample and scaled to the full call.

    Per-visibility steps are timed at two sample sizes (n and 2n) so that their
    fixed per-layer part (the oracle grids each layer through a full N'^2
    bincount) and their per-visibility slope are separated; the degrid
    correlation reads a stack whose every page holds data (each layer the
    transform of a random image, not untouched zero pages).  Two layers' transforms
    (IFFT, crop, w-screen; w-screen, pad, FFT) and a slice of the correction
    map are timed and scaled to all layers and pixels.  The 2-D transforms use
    every host core (scipy.fft workers); every other step runs on one.
    """
    import numpy as np

    from oracle import wstack
    from oracle.kernel_design import least_misfit
    from oracle.plan import make_plan

    plan = make_plan(w["N"], w["L"], w["W"], w["x0"], w["wmax"])
    lm = least_misfit(w["W"], w["x0"])
    M, nl = w["uvw"].shape[0], plan.n_layers
    z = plan.z()
    measured = 0.0

    def grid_vis(n):
        t0 = time.perf_counter()
        gi = wstack.grid_prepare(plan, lm, w["uvw"][:n], w["vis"][:n].astype(np.complex128))
        G = None
        for t in range(plan.t_lo, plan.t_hi + 1):
            G = wstack.grid_layer(plan, gi, t)
        return time.perf_counter() - t0, G

    # a stack with data in every layer: each layer the transform of a random image
    t0 = time.perf_counter()
    g = np.random.default_rng(3).standard_normal((plan.N, plan.N))
    stack = np.empty((nl, plan.Nprime, plan.Nprime), dtype=np.complex128)
    layer = wstack.degrid_layer(plan, g, plan.t_hi, z)
    t_degrid_layer = time.perf_counter() - t0
    for i in range(nl):
        stack[i] = layer
    measured += time.perf_counter() - t0

    def degrid_vis(n):
        t0 = time.perf_counter()
        wstack.degrid_correlate(plan, lm, w["uvw"][:n], stack)
        return time.perf_counter() - t0

    n1, n2 = n_sample, 2 * n_sample
    tg1, _ = grid_vis(n1)
    tg2, G = grid_vis(n2)
    td1, td2 = degrid_vis(n1), degrid_vis(n2)
    measured += tg1 + tg2 + td1 + td2
    g_slope, d_slope = max(tg2 - tg1, 0.0) / (n2 - n1), max(td2 - td1, 0.0) / (n2 - n1)
    g_fixed, d_fixed = max(tg1 - g_slope * n1, 0.0), max(td1 - d_slope * n1, 0.0)
    t0 = time.perf_counter()
    wstack.layer_image(plan, G, plan.t_hi, z)
    t_grid_layer = time.perf_counter() - t0
    n_pix = 8192 * 4
    t0 = time.perf_counter()
    lm.h(z.ravel()[:n_pix])
    t_pix = time.perf_counter() - t0
    t_corr = t_pix * (plan.N * plan.N / n_pix)
    del stack
    measured += t_grid_layer + t_pix
    t_grid = g_fixed + g_slope * M + nl * t_grid_layer + t_corr
    t_degrid = d_fixed + d_slope * M + nl * t_degrid_layer + t_corr
    cpus = os.cpu_count() or 1
    return {
        "value": M / (t_grid + t_degrid),
        "unit": "visibilities/s",
        "cores": cpus,
        "kind": "oracle",
        "sample": (f"oracle per-visibility steps (fold, phase, weights, w-spreading and uv-gridding into all "
                   f"{nl} layers; 3-D correlation from a filled {nl}-layer stack) on the first {n1} and {n2} "
                   f"visibilities (fixed + per-visibility fit), one layer's {plan.Nprime}^2 IFFT/crop/w-screen "
                   f"and one layer's pad/FFT, h_z on {n_pix} pixels; scaled to {M} visibilities, {nl} layers, "
                   f"{plan.N}^2 pixels; {measured:.1f} s measured; 2-D transforms on {cpus} threads (scipy.fft "
                   f"workers), all other steps numpy on one"),
        "host_cpus": cpus,
        "est_s_per_call": {"grid": t_grid, "degrid": t_degrid},
    }


def bandwidth_probe(dev, gb: float = 4.0, repeats: int = 5) -> dict:
    """Achievable HBM read + write rate: the library's streaming copy kernel
    over gb GB (src -> dst), timed with events on the launch stream."""
    import torch

    from paper_2101_11172_amd import wsgrid

    n = int(gb * 1e9) // 16 * 16
    src = torch.ones(n // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream(dev)
    wsgrid.wsg_bandwidth_probe(src.data_ptr(), dst.data_ptr(), n, stream.cuda_stream)   # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(repeats):
        wsgrid.wsg_bandwidth_probe(src.data_ptr(), dst.data_ptr(), n, stream.cuda_stream)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / repeats
    ok = bool(torch.equal(src[-1024:], dst[-1024:]))
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_read": n, "bytes_written": n, "ms": ms, "GBps": 2 * n / (ms * 1e-3) / 1e9, "copy_ok": ok}


def dft_errors(plan, w: dict, uvw, dev, n_pix: int = 10000, n_vis: int = 10000) -> dict:
    """Relative RMS error against the direct transform at sampled outputs, per
    result and precision: the dirty map of the workload's visibilities at
    n_pix random pixels, and the model visibilities of a 500-source sky at
    n_vis random baselines (direct transform on the device, float64)."""
    import numpy as np
    import torch

    from paper_2101_11172_amd import direct, inputs

    N, L = w["N"], w["L"]
    rng = np.random.default_rng(17)
    rows, cols = rng.integers(0, N, n_pix), rng.integers(0, N, n_pix)
    V = torch.from_numpy(w["vis"]).to(dev).to(torch.complex128)
    exact_g = direct.dft_grid(uvw, V, N, L, rows, cols)
    sky = torch.from_numpy(inputs.random_sky(N, 500, 9)).to(dev)
    idx = torch.from_numpy(np.random.default_rng(8).choice(uvw.shape[0], n_vis, replace=False)).to(dev)
    exact_d = direct.dft_degrid(uvw[idx].contiguous(), sky, N, L)
    rows_t, cols_t = torch.from_numpy(rows).to(dev), torch.from_numpy(cols).to(dev)

    def rel(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    out = {"grid_pixels": n_pix, "degrid_visibilities": n_vis}
    for name, cdt, rdt in (("fp32", torch.complex64, torch.float32), ("fp64", torch.complex128, torch.float64)):
        g = plan.grid(uvw, V.to(cdt))
        out[f"grid_{name}"] = rel(g[rows_t, cols_t].double(), exact_g)
        d = plan.degrid(uvw, sky.to(rdt))
        out[f"degrid_{name}"] = rel(d[idx].to(torch.complex128), exact_d)
    return out


def stage_table(stages: dict, f64: bool, M: int, N: int, Np: int, nl: int, ws: dict, calls: int,
                prepared: bool = False) -> dict:
    """Per call of grid or degrid: stage time (HIP events on the launch stream,
    summed over the stage's launches) and algorithmic bytes."""
    tab = {}
    for name, (ms, n) in stages.items():
        if n == 0:
            continue
        per = ms / calls
        nbytes = stage_bytes(name, M, N, Np, nl, f64, ws, prepared)
        tab[name] = {"ms": per, "launches_per_call": n / calls, "alg_bytes": nbytes,
                     "alg_GBps": nbytes / (per * 1e-3) / 1e9}
    return tab


def timed_plain(step, steps: int) -> float:
    """Milliseconds per step over `steps` steps, without stage events."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def timed(step, steps: int):
    """Run `steps` steps with per-stage event timing; returns (ms per step, stage times)."""
    import torch

    from paper_2101_11172_amd import wsgrid

    torch.cuda.synchronize()
    wsgrid.wsg_stage_times()            # clear
    wsgrid.wsg_stage_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wsgrid.wsg_stage_timing(False)
    return (t1 - t0) * 1e3 / steps, wsgrid.wsg_stage_times()


def channels_multi_main(args) -> int:
    """One grid_visibilities_multi plus one degrid_visibilities_multi of 32
    channels (1.0-1.8 GHz on the wide-field array, 4-10M visibilities each
    after random flagging, 224M in all) with image sizes per channel: the
    smallest of 1024^2, 1536^2, 2048^2 that Nyquist-samples the channel (1536^2
    up to 1.35 GHz, N' = 3072; 2048^2 above, N' = 4096), each size group on one
    plan with the group's largest |w|; FP32."""
    import numpy as np
    import torch

    from paper_2101_11172_amd import inputs, wsgrid

    dev = torch.device("cuda", 0)
    log("generating the batched-channel workload")
    w = inputs.channels_workload()
    L, W, x0, counts, freqs = w["L"], w["W"], w["x0"], w["counts"], w["freqs"]
    sizes = inputs.channel_image_sizes(freqs)
    M, C = int(sum(counts)), len(counts)
    off = np.concatenate([[0], np.cumsum(counts)])
    group_wmax = {}
    for c, n in enumerate(sizes):
        wc = float(np.max(np.abs(w["uvw"][off[c]:off[c + 1], 2]))) if counts[c] else 0.0
        group_wmax[n] = max(group_wmax.get(n, 0.0), wc)
    plans = {n: wsgrid.Plan(n, L, W, x0, group_wmax[n], device=dev) for n in sorted(group_wmax)}
    cap = int(args.max_workspace_gb * (1 << 30))
    ps = wsgrid.PlanSet([plans[n] for n in sizes], max_workspace_bytes=cap)
    uvw = torch.from_numpy(w["uvw"]).to(dev)
    vis = torch.from_numpy(w["vis"]).to(dev)
    del w
    img = torch.cat([torch.from_numpy(inputs.random_image(n, 200 + c).astype(np.float32)).reshape(-1)
                     for c, n in enumerate(sizes)]).to(dev)
    out_img = torch.empty(ps.map_elements(), dtype=torch.float32, device=dev)
    out_vis = torch.empty(M, dtype=torch.complex64, device=dev)
    groups = {n: {"channels": sizes.count(n), "N'": plans[n].info["Nprime"], "w_layers": plans[n].info["n_layers"],
                  "wmax": group_wmax[n]} for n in plans}
    log(f"channels={C} M={M} groups={groups}")
    tuned = None
    if args.autotune:
        from paper_2101_11172_amd.autotune import tune_multi
        tuned = tune_multi(ps, uvw, counts, vis, img, cap)
        ps.max_workspace_bytes = tuned["workspace_bytes"]
        log(f"autotune: workspace {tuned['workspace_bytes']} bytes, ms by workspace {tuned['ms']}")

    # The step: the channels' uvw binned once (one grid_prepare per size group),
    # then one gridding and one degridding of all channels on that binning.
    def step():
        ps.prepare(uvw, counts, torch.float32)
        ps.grid_prepared(vis, out=out_img)
        ps.degrid_prepared(img, out=out_vis)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ms, stages = timed(step, args.steps)
    log(f"channels (per-channel sizes, one binning per step): {ms:.3f} ms/step, {M / (ms * 1e-3):.4e} vis/s")
    prep_ws = sum(w.numel() for w in ps._prep_ws)
    ps._prep_ws, ps._prep = [], None
    torch.cuda.empty_cache()

    # The same work as two independent multi-plan calls, each binning uvw itself.
    sep_img, sep_vis = torch.empty_like(out_img), torch.empty_like(out_vis)

    def step_separate():
        ps.grid(uvw, counts, vis, out=sep_img)
        ps.degrid(uvw, counts, img, out=sep_vis)

    step_separate()
    ms_sep, stages_sep = timed(step_separate, args.steps)
    log(f"channels, separate multi-plan calls: {ms_sep:.3f} ms/step, {M / (ms_sep * 1e-3):.4e} vis/s")
    grid_rel = float(torch.linalg.vector_norm(out_img.double() - sep_img.double())
                     / torch.linalg.vector_norm(sep_img.double()))
    result = {
        "metric": "batched channels: visibilities/s grid+degrid, 32 channels, image size per channel",
        "value": M / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"batched channels: {C} channels 1.0-1.8 GHz of the wide-field array, 0-60% random "
                                f"flagging per channel, {M} visibilities, image size per channel "
                                f"({sizes.count(1536)} x 1536^2, {sizes.count(2048)} x 2048^2), L={L}, W={W}, "
                                f"x0={x0}, one plan per size group"),
                   "channels": C, "visibilities": M, "groups": {str(k): v for k, v in groups.items()},
                   "workspace_bytes": prep_ws,
                   "step": "uvw binned once per size group (grid_prepare), then one grid and one degrid of all "
                           "channels on that binning; separate_calls: grid/degrid_visibilities_multi"},
        "autotune": tuned,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items() if v[1]},
        "separate_calls": {"value": M / (ms_sep * 1e-3), "ms_per_step": ms_sep,
                           "workspace_bytes": ps.workspace(wsgrid.WSG_F32, counts).numel(),
                           "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages_sep.items() if v[1]},
                           "prepared_vs_separate": {"grid_rel_rms": grid_rel,
                                                    "degrid_equal": bool(torch.equal(out_vis, sep_vis))}},
    }
    print(json.dumps(result), flush=True)
    for p in plans.values():
        p.close()
    return 0


def channels_main(args) -> int:
    """One grid_visibilities_batch plus one degrid_visibilities_batch of 32
    channels (1.0-1.8 GHz on the wide-field array, 4-10M visibilities each
    after random flagging, 224M in all) on one 2048^2 plan, FP32."""
    import numpy as np
    import torch

    from paper_2101_11172_amd import inputs, wsgrid

    dev = torch.device("cuda", 0)
    log("generating the batched-channel workload")
    w = inputs.channels_workload()
    N, L, W, x0, wmax, counts = w["N"], w["L"], w["W"], w["x0"], w["wmax"], w["counts"]
    M, C = int(sum(counts)), len(counts)
    uvw = torch.from_numpy(w["uvw"]).to(dev)
    vis = torch.from_numpy(w["vis"]).to(dev)
    del w
    plan = wsgrid.Plan(N, L, W, x0, wmax, device=dev, max_workspace_bytes=int(args.max_workspace_gb * (1 << 30)))
    info = plan.info
    img = torch.from_numpy(np.stack([inputs.random_image(N, 200 + c).astype(np.float32) for c in range(C)])).to(dev)
    out_img = torch.empty((C, N, N), dtype=torch.float32, device=dev)
    out_vis = torch.empty(M, dtype=torch.complex64, device=dev)
    log(f"channels={C} M={M} (per channel {min(counts)}..{max(counts)}) N={N} N'={info['Nprime']} "
        f"layers={info['n_layers']}")
    tuned = None
    if args.autotune:
        from paper_2101_11172_amd.autotune import tune_pass_layers
        tuned = tune_pass_layers(plan, uvw, counts, vis, img, plan.max_workspace_bytes)
        plan.max_workspace_bytes = tuned["workspace_bytes"]
        log(f"autotune: {tuned['pass_layers']} layers per pass, ms by pass size {tuned['ms']}")

    def step():
        plan.grid_batch(uvw, counts, vis, out=out_img)
        plan.degrid_batch(uvw, counts, img, out=out_vis)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ws_bytes = plan.workspace(wsgrid.WSG_F32, M, C).numel()
    last_layer = (C - 1) * 16 * ((info["n_layers"] + 15) // 16) + info["n_layers"]
    per_pass = wsgrid.grid_layers_per_pass(plan._p, wsgrid.WSG_F32, C, M, ws_bytes)
    passes = -(-last_layer // per_pass)
    ms, stages = timed(step, args.steps)
    log(f"channels: {ms:.3f} ms/step, {M / (ms * 1e-3):.4e} vis/s, {passes} layer passes")
    result = {
        "metric": "batched channels: visibilities/s grid+degrid, 32 channels in one call per direction",
        "value": M / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"batched channels: {C} channels 1.0-1.8 GHz of the wide-field array (64 antennas, "
                                f"+-1 h), 0-60% random flagging per channel, {M} visibilities ({min(counts)}-"
                                f"{max(counts)} per channel), one {N}x{N} plan, L={L}, W={W}, x0={x0}, "
                                f"{info['n_layers']} w-layers per channel, {passes} layer passes"),
                   "channels": C, "visibilities": M, "N": N, "w_layers": info["n_layers"],
                   "workspace_bytes": ws_bytes, "layer_passes": passes},
        "autotune": tuned,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items() if v[1]},
    }
    print(json.dumps(result), flush=True)
    plan.close()
    return 0


def imaging_main(args) -> int:
    """One gradient step of ||degrid(I) - V||^2 per step: DegridFn forward
    (degrid_visibilities) and backward (grid_visibilities) on a 4096^2 FP32
    image with 50,003,456 visibilities (128 antennas in a 10 km-radius disc,
    +-2 h tracks of 6,152 dumps, declination -30 deg, uvw scaled to a
    Nyquist-sampled image, L = 0.5), W = 7, x0 = 0.25: N' = 8192, 223 w-layers
    taken in passes within the workspace cap."""
    import numpy as np
    import torch

    from paper_2101_11172_amd import inputs, wsgrid

    dev = torch.device("cuda", 0)
    N, L, W, x0 = 4096, 0.5, 7, 0.25
    log("generating the imaging workload")
    uvw = inputs.scale_to_image(inputs.array_uvw(128, 10000.0, -30.0, -30.0, 2.0, 6152, 1.4e9, 4), N, L)
    wmax = float(np.max(np.abs(uvw[:, 2])))
    M = uvw.shape[0]
    t_uvw = torch.from_numpy(uvw).to(dev)
    del uvw
    V = torch.from_numpy(inputs.random_vis(M, 5, np.complex64)).to(dev)
    cap = int(args.max_workspace_gb * (1 << 30))
    plan = wsgrid.Plan(N, L, W, x0, wmax, device=dev, max_workspace_bytes=cap)
    info = plan.info
    img = torch.nn.Parameter(torch.from_numpy(inputs.random_image(N, 6).astype(np.float32)).to(dev))
    log(f"M={M} N={N} N'={info['Nprime']} layers={info['n_layers']}")

    def step():
        loss = torch.sum(torch.abs(wsgrid.degrid_fn(plan, t_uvw, img) - V) ** 2)
        img.grad = None
        loss.backward()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    per_pass = wsgrid.grid_layers_per_pass(plan._p, wsgrid.WSG_F32, 1, M, plan.workspace(wsgrid.WSG_F32, M).numel())
    passes = -(-info["n_layers"] // per_pass)
    ms, _ = timed(step, args.steps)
    log(f"imaging: {ms:.3f} ms/step, {M / (ms * 1e-3):.4e} vis/s, {passes} layer passes")
    # stage breakdown from the same two calls made on this thread (autograd runs
    # the backward on a thread of its own, where stage timing is not enabled)
    vis = torch.empty(M, dtype=torch.complex64, device=dev)
    grad = torch.empty((N, N), dtype=torch.float32, device=dev)

    def direct():
        plan.degrid(t_uvw, img.detach(), out=vis)
        plan.grid(t_uvw, vis, out=grad)

    ms_direct, stages = timed(direct, args.steps)
    result = {
        "metric": "differentiable imaging: visibilities/s per gradient step (degrid forward + grid backward)",
        "value": M / (ms * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"differentiable imaging: {N}x{N} FP32 image parameter, L={L}, W={W}, x0={x0}, "
                                f"{M} visibilities (128 antennas in a 10 km disc, +-2 h tracks, dec -30, uvw "
                                f"scaled to a Nyquist-sampled image), {info['n_layers']} w-layers, "
                                f"N'={info['Nprime']}, {passes} layer passes"),
                   "N": N, "L": L, "visibilities": M, "w_layers": info["n_layers"], "fft_size": info["Nprime"],
                   "workspace_bytes": plan.workspace(wsgrid.WSG_F32, M).numel(), "layer_passes": passes},
        "direct_calls_ms_per_step": ms_direct,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items() if v[1]},
    }
    print(json.dumps(result), flush=True)
    plan.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dumps", type=int, default=4960, help="time samples (M = 2016 x dumps)")
    ap.add_argument("--fp64-steps", type=int, default=3, help="0 skips the FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=60000)
    ap.add_argument("--probe-gb", type=float, default=4.0,
                    help="bytes (GB) of the streaming copy that measures achievable HBM bandwidth (0: skip)")
    ap.add_argument("--no-dft", action="store_true", help="skip the errors against the direct transform")
    ap.add_argument("--copy-gb", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GB (counter calibration)")
    ap.add_argument("--no-z-offset", action="store_true",
                    help="widefield: the planner variant without z offset (Sec. 5.3; about twice the layers)")
    ap.add_argument("--workload", choices=("widefield", "lowcost", "widefield3", "imaging", "channels"),
                    default="widefield",
                    help="lowcost: the wide-field geometry at W=4, x0=0.5; widefield3: at x0=1/3 (N'=3072); "
                         "imaging: one differentiable-imaging gradient step per step (4096^2, 50M visibilities); "
                         "channels: one batched grid + degrid of 32 channels per step")
    ap.add_argument("--max-workspace-gb", type=float, default=None,
                    help="imaging and channels: workspace cap (layer passes); default 64 for imaging "
                         "(5 passes measured fastest: 40-64 GB 159.7-160.0 ms, 96 GB 161.4, 160 GB 165.7, "
                         "one pass 179.2), 96 for channels")
    ap.add_argument("--one-plan", action="store_true",
                    help="channels: one 2048^2 plan for every channel (instead of an image size per channel)")
    ap.add_argument("--pass-layers", type=int, default=None,
                    help="widefield, lowcost, widefield3: layers per pass (0: all in one pass); default: the "
                         "autotuner times every pass size and takes the fastest")
    ap.add_argument("--autotune", action="store_true",
                    help="channels: choose the layers per pass within the cap by timing (autotune.py) first")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path is built and measured on a single MI355X "
              "(multi-GPU sharding over w-layers is a design, not a measured run)", file=sys.stderr)
        return 2
    if args.max_workspace_gb is None:
        args.max_workspace_gb = 64.0 if args.workload == "imaging" else 96.0
    if args.workload == "imaging":
        return imaging_main(args)
    if args.workload == "channels":
        return channels_main(args) if args.one_plan else channels_multi_main(args)

    import numpy as np
    import torch

    from paper_2101_11172_amd import inputs, wsgrid

    dev = torch.device("cuda", 0)
    probe = bandwidth_probe(dev) if args.probe_gb > 0 else None
    if probe:
        log(f"bandwidth probe: {probe['GBps']:.0f} GB/s read + write ({probe['ms']:.3f} ms for 2 x "
            f"{probe['bytes_read'] / 1e9:.1f} GB)")
    if args.copy_gb > 0:
        n = int(args.copy_gb * 1e9) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)            # one elementwise kernel: reads and writes 4n bytes
        torch.cuda.synchronize()
        log(f"calibration kernel: {4 * n} bytes read, {4 * n} bytes written")
        del src, dst
    log(f"generating the {args.workload} workload")
    w = inputs.workload(args.workload, n_dumps=args.dumps, vis_dtype=np.complex64)
    N, L, W, x0, wmax = w["N"], w["L"], w["W"], w["x0"], w["wmax"]
    M = w["uvw"].shape[0]
    plan = wsgrid.Plan(N, L, W, x0, wmax, device=dev, z_offset=not args.no_z_offset)
    info = plan.info
    Np, nl = info["Nprime"], info["n_layers"]
    log(f"M={M} N={N} N'={Np} layers={nl} E={info['E']:.3e}")
    ws = workload_stats(w["uvw"], N, L, W, x0, wmax, Np, nl, info["t_lo"], info["n_scale"])
    log(f"occupied tiles {ws['tiles_occupied']}/{ws['tiles']}, tile visits {ws['tile_visits']}")
    uvw = torch.from_numpy(w["uvw"]).to(dev)
    vis32 = torch.from_numpy(w["vis"]).to(dev)
    img32 = torch.from_numpy(inputs.random_image(N, 5).astype(np.float32)).to(dev)

    # layer-pass size: timed by the autotuner over every pass size (one plain
    # grid + degrid each), or as given; the workspace is the smallest that holds it
    from paper_2101_11172_amd.autotune import tune_pass_layers, workspace_for_pass_layers
    tuned = None
    if args.pass_layers is None:
        tuned = tune_pass_layers(plan, uvw, [M], vis32, img32.reshape(1, N, N), 1 << 62, repeats=3,
                                 every_pass_size=True)
        pass_layers = tuned["pass_layers"]
        log(f"autotune: {pass_layers} layers per pass, ms by pass size {tuned['ms']}")
    else:
        pass_layers = min(nl, args.pass_layers) if args.pass_layers > 0 else nl
    plan.max_workspace_bytes = ws32_bytes = workspace_for_pass_layers(plan, wsgrid.WSG_F32, 1, M, pass_layers)
    out_img32 = torch.empty((N, N), dtype=torch.float32, device=dev)
    out_vis32 = torch.empty(M, dtype=torch.complex64, device=dev)

    def relrms(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    # The step: uvw binned once (grid_prepare), then one gridding and one
    # degridding of all visibilities on that binning.
    def step32():
        plan.prepare(uvw, torch.float32)
        plan.grid_prepared(vis32, out=out_img32)
        plan.degrid_prepared(img32, out=out_vis32)

    # The same work as two independent calls, each binning uvw itself.
    sep_img32, sep_vis32 = torch.empty_like(out_img32), torch.empty_like(out_vis32)

    def step32_separate():
        plan.grid(uvw, vis32, out=sep_img32)
        plan.degrid(uvw, img32, out=sep_vis32)

    for i in range(args.warmup):
        step32()
        step32_separate()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ms32 = timed_plain(step32, args.steps)
    _, stages32 = timed(step32, args.steps)
    log(f"fp32: {ms32:.3f} ms/step, {M / (ms32 * 1e-3):.4e} vis/s (one binning per step)")
    tab32 = stage_table(stages32, False, M, N, Np, nl, ws, args.steps, prepared=True)
    skipped = plan.skipped(wsgrid.WSG_F32)
    ms_sep = timed_plain(step32_separate, args.steps)
    _, stages_sep = timed(step32_separate, args.steps)
    log(f"fp32 separate calls: {ms_sep:.3f} ms/step, {M / (ms_sep * 1e-3):.4e} vis/s")
    separate = {"value": M / (ms_sep * 1e-3), "ms_per_step": ms_sep,
                "stages": stage_table(stages_sep, False, M, N, Np, nl, ws, args.steps),
                "prepared_vs_separate": {"grid_rel_rms": relrms(out_img32.double(), sep_img32.double()),
                                         "degrid_equal": bool(torch.equal(out_vis32, sep_vis32))}}

    fp64, acc = None, None
    if args.fp64_steps > 0:
        vis64, img64 = vis32.to(torch.complex128), img32.double()
        out_img64 = torch.empty((N, N), dtype=torch.float64, device=dev)
        out_vis64 = torch.empty(M, dtype=torch.complex128, device=dev)

        def step64():
            plan.prepare(uvw, torch.float64)
            plan.grid_prepared(vis64, out=out_img64)
            plan.degrid_prepared(img64, out=out_vis64)

        plan.max_workspace_bytes = workspace_for_pass_layers(plan, wsgrid.WSG_F64, 1, M, pass_layers)
        step64()
        ms64 = timed_plain(step64, args.fp64_steps)
        _, stages64 = timed(step64, args.fp64_steps)
        log(f"fp64: {ms64:.3f} ms/step, {M / (ms64 * 1e-3):.4e} vis/s")
        fp64 = {"value": M / (ms64 * 1e-3), "ms_per_step": ms64,
                "stages": stage_table(stages64, True, M, N, Np, nl, ws, args.fp64_steps, prepared=True)}
        acc = {"grid": relrms(out_img32.double(), out_img64),
               "degrid": relrms(out_vis32.to(torch.complex128), out_vis64)}

    dft_err = None
    if not args.no_dft:
        log("errors against the direct transform at sampled outputs")
        dft_err = dft_errors(plan, w, uvw, dev)
        log(f"dft errors: {dft_err}")

    dom = max(tab32, key=lambda k: tab32[k]["ms"])
    d = tab32[dom]
    achievable = probe["GBps"] if probe else None
    key = workload_key(args.workload + ("-no-z-offset" if args.no_z_offset else ""), N, W, x0, M, nl, pass_layers)
    per_launch = traffic_for(dom, "f32", key)          # counters: average HBM bytes per launch
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["alg_GBps"] / HBM_PEAK_GBS,
                "traffic": per_launch * d["launches_per_call"] if per_launch is not None else None,
                "achievable": achievable, "frac_of_achievable": d["alg_GBps"] / achievable if achievable else None,
                "alg_bytes_per_call": d["alg_bytes"], "ms_per_call": d["ms"],
                "launches_per_call": d["launches_per_call"]}
    issue = issue_for(dom, "f32", key)
    if issue:
        n = d["launches_per_call"]
        roofline["issue"] = {"valu_instr_per_call": issue["valu_instr_per_launch"] * n,
                             "valu_issue_ms": issue["valu_issue_ms"] * n,
                             "valu_issue_frac": issue["valu_issue_ms"] * n / d["ms"]}
    total_alg = sum(stage_bytes(s, M, N, Np, nl, False, ws, prepared=True) for s in tab32)
    result = {
        "metric": (f"visibilities/s grid+degrid at W={W},x0={x0:g}, FP32 vs FP64"
                   + (", at <=1e-6 DFT error" if (W, x0) == (7, 0.25) else "")),
        "value": M / (ms32 * 1e-3),
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ({"widefield": "wide-field single channel",
                                  "lowcost": "low-cost setting on the wide-field geometry",
                                  "widefield3": "wide-field geometry at x0=1/3 (radix-3 transforms)"}[args.workload]
                                + f": {N}x{N} image, L={L}, W={W}, x0={x0}, {M} "
                                f"visibilities (64 antennas in a 5 km disc, +-1 h tracks, dec -30, 1.4 GHz, "
                                f"uvw scaled to a Nyquist-sampled image), {nl} w-layers, N'={Np}"
                                + (", planner without z offset" if args.no_z_offset else "")),
                   "N": N, "L": L, "W": W, "x0": x0, "visibilities": M, "w_layers": nl, "fft_size": Np,
                   "z_offset": not args.no_z_offset, "pass_layers": pass_layers,
                   "workspace_bytes": ws32_bytes,
                   "step": "uvw binned once (grid_prepare), then one grid and one degrid of all visibilities on "
                           "that binning; separate_calls: the same two calls each binning uvw itself"},
        "roofline": roofline,
        "whole_step_alg_GBps": total_alg / (ms32 * 1e-3) / 1e9,
        "whole_step_frac_of_peak": total_alg / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "whole_step_frac_of_achievable": (total_alg / (ms32 * 1e-3) / 1e9 / achievable) if achievable else None,
        "hbm_probe": probe,
        "dft_error": dft_err,
        "fp64": fp64,
        "fp32_vs_fp64_rel_rms": acc,
        "stages": tab32,
        "separate_calls": separate,
        "autotune": tuned,
        # each call separately: the sum of its stage times (HIP events, FP32)
        "stage_sum_ms_per_call": {c: sum(v["ms"] for k, v in separate["stages"].items() if k.startswith(c + "_"))
                                  for c in ("grid", "degrid")},
        "stack_occupancy": ws,
        "skipped": skipped,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
        log(f"cpu oracle: {result['cpu_baseline']['value']:.4e} vis/s")
    print(json.dumps(result), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
