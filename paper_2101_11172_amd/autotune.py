"""Plane-batch autotuner for (batched) gridding and degridding.

The library takes the w-layers of all channels in passes whose size is set by
the workspace it is given (grid_layers_per_pass).  More layers per pass means
fewer, larger launches and more memory; fewer means more passes over the
binned records.  ``tune_pass_layers`` times one batched grid plus one batched
degrid for a few workspace sizes between the smallest the call accepts and a
memory cap (or for every pass size), and returns the fastest.  Which is
fastest depends on the workload: the 2048^2 wide-field call runs fastest in
passes of 32 of its 49 layers, the 4096^2 imaging call in five passes, the
batched channels in as few as the memory allows.  The 16 x 16 x 16 tile of the scatter and
gather kernels is fixed at compile time by their LDS budget and is not tuned.

Host logic and timing only: every call runs the library's own kernels.
"""
from __future__ import annotations

import torch

from . import wsgrid as wg


def workspace_for_pass_layers(plan: "wg.Plan", prec: int, nch: int, M: int, layers: int) -> int:
    """Smallest workspace whose layer passes hold at least `layers` layers
    (all of them if fewer), found by bisection over grid_layers_per_pass."""
    lo = wg.grid_workspace_bytes_batch(plan._p, prec, nch, M, True)
    hi = wg.grid_workspace_bytes_batch(plan._p, prec, nch, M)
    if wg.grid_layers_per_pass(plan._p, prec, nch, M, lo) >= layers:
        return lo
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if wg.grid_layers_per_pass(plan._p, prec, nch, M, mid) >= layers:
            hi = mid
        else:
            lo = mid
    return hi


def pass_sizes(plan: "wg.Plan", prec: int, nch: int, M: int) -> list:
    """Every distinct layer-pass size of a call (whole tile layers, up to all)."""
    full = wg.grid_workspace_bytes_batch(plan._p, prec, nch, M)
    top = wg.grid_layers_per_pass(plan._p, prec, nch, M, full)
    return sorted({min(top, 16 * k) for k in range(1, (top + 15) // 16 + 1)})


def tune_pass_layers(plan: "wg.Plan", uvw: torch.Tensor, counts, vis: torch.Tensor, image: torch.Tensor,
                     max_workspace_bytes: int, n_candidates: int = 4, repeats: int = 2,
                     every_pass_size: bool = False) -> dict:
    """Fastest workspace size (and its layers per pass) for these inputs.

    uvw, vis: concatenated channels (counts[c] visibilities each); image:
    [len(counts), N, N] of the matching real precision.  Returns
    {"workspace_bytes", "pass_layers", "ms": {pass_layers: ms per grid + degrid}}.
    """
    counts = [int(c) for c in counts]
    nch, M = len(counts), int(sum(counts))
    # the same checks as Plan.grid_batch / Plan.degrid_batch, before any launch
    plan.check_batch(uvw, counts, vis=vis)
    plan.check_batch(uvw, counts, image=image)
    prec = wg.WSG_F32 if vis.dtype == torch.complex64 else wg.WSG_F64
    rdt = torch.float32 if prec == wg.WSG_F32 else torch.float64
    if image.dtype != rdt:
        raise ValueError("image precision must match the visibilities' (float32 with complex64)")
    least = wg.grid_workspace_bytes_batch(plan._p, prec, nch, M, True)
    top = min(wg.grid_workspace_bytes_batch(plan._p, prec, nch, M), int(max_workspace_bytes))
    if top < least:
        raise ValueError(f"the cap is below the smallest workspace ({least} bytes)")
    if every_pass_size:      # each pass size within the cap, at its smallest workspace
        sizes = [workspace_for_pass_layers(plan, prec, nch, M, n) for n in pass_sizes(plan, prec, nch, M)]
        sizes = [b for b in sizes if b <= top] or [least]
    else:
        sizes = sorted({least + (top - least) * i // max(1, n_candidates - 1) for i in range(n_candidates)})
    by_layers = {}
    for b in sorted(sizes):      # keep the smallest workspace that gives each pass size
        by_layers.setdefault(wg.grid_layers_per_pass(plan._p, prec, nch, M, b), b)
    stream = torch.cuda.current_stream(plan.device)
    dirty = torch.empty((nch, plan.N, plan.N), dtype=rdt, device=plan.device)
    out = torch.empty(M, dtype=vis.dtype, device=plan.device)
    timings = {}
    for layers, nbytes in sorted(by_layers.items()):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=plan.device)

        def step():
            wg.grid_visibilities_batch(plan._p, prec, counts, uvw.data_ptr(), vis.data_ptr(), dirty.data_ptr(),
                                       ws.data_ptr(), nbytes, stream.cuda_stream)
            wg.degrid_visibilities_batch(plan._p, prec, counts, uvw.data_ptr(), image.data_ptr(), out.data_ptr(),
                                         ws.data_ptr(), nbytes, stream.cuda_stream)

        step()                                              # warm-up
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(repeats):
            step()
        end.record(stream)
        end.synchronize()
        timings[layers] = start.elapsed_time(end) / repeats
        del ws
        torch.cuda.empty_cache()      # the next candidate may need the memory back
    best = min(timings, key=timings.get)
    return {"workspace_bytes": by_layers[best], "pass_layers": best, "ms": timings}


def tune_multi(planset: "wg.PlanSet", uvw: torch.Tensor, counts, vis: torch.Tensor, image: torch.Tensor,
               max_workspace_bytes: int, n_candidates: int = 4, repeats: int = 2) -> dict:
    """As tune_pass_layers for channels with plans of their own (a PlanSet):
    times one grid_visibilities_multi plus one degrid_visibilities_multi for a
    few workspace sizes between the smallest the calls accept and the cap (the
    workspace sets every run's layers per pass) and returns the fastest.
    image: the packed maps of the matching real precision."""
    counts = [int(c) for c in counts]
    planset._check(uvw, counts)
    prec = wg.WSG_F32 if vis.dtype == torch.complex64 else wg.WSG_F64
    rdt = torch.float32 if prec == wg.WSG_F32 else torch.float64
    if vis.dtype not in (torch.complex64, torch.complex128) or image.dtype != rdt \
            or image.shape != (planset.map_elements(),) or vis.shape != (uvw.shape[0],):
        raise ValueError("vis [M] complex and packed image maps of the matching real precision are required")
    ptrs = planset._ptrs()
    least = wg.grid_workspace_bytes_multi(ptrs, prec, counts, True)
    top = min(wg.grid_workspace_bytes_multi(ptrs, prec, counts), int(max_workspace_bytes))
    if top < least:
        raise ValueError(f"the cap is below the smallest workspace ({least} bytes)")
    sizes = sorted({least + (top - least) * i // max(1, n_candidates - 1) for i in range(n_candidates)})
    stream = torch.cuda.current_stream(planset.device)
    dirty = torch.empty(planset.map_elements(), dtype=rdt, device=planset.device)
    out = torch.empty(uvw.shape[0], dtype=vis.dtype, device=planset.device)
    timings = {}
    for nbytes in sizes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=planset.device)

        def step():
            wg.grid_visibilities_multi(ptrs, prec, counts, uvw.data_ptr(), vis.data_ptr(), dirty.data_ptr(),
                                       ws.data_ptr(), nbytes, stream.cuda_stream)
            wg.degrid_visibilities_multi(ptrs, prec, counts, uvw.data_ptr(), image.data_ptr(), out.data_ptr(),
                                         ws.data_ptr(), nbytes, stream.cuda_stream)

        step()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(repeats):
            step()
        end.record(stream)
        end.synchronize()
        timings[nbytes] = start.elapsed_time(end) / repeats
        del ws
        torch.cuda.empty_cache()
    best = min(timings, key=timings.get)
    return {"workspace_bytes": best, "ms": timings}
