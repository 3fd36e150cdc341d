"""The shared-binning step captured into a HIP graph and replayed.

Every launch of grid_prepare, grid_visibilities_prepared and
degrid_visibilities_prepared goes to the caller's stream and none allocates,
synchronizes or clears memory with a memset (the workspace is the caller's,
zeroing is done by fill kernels), so the step can be captured.  The graph is
replayed several times with eager calls and synchronizations between the
replays; every replay must reproduce the eager result: degrid bit for bit, grid
within rounding (the LDS accumulation order of a tile is not fixed).
"""
import numpy as np
import pytest
import torch

from paper_2101_11172_amd import inputs
from paper_2101_11172_amd import wsgrid as wg

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def rel(a, b):
    return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))


@pytest.mark.parametrize("prec", [32, 64])
def test_prepared_step_replays_from_a_graph(prec):
    cdt, rdt, tol = (torch.complex64, torch.float32, 1e-6) if prec == 32 else (torch.complex128, torch.float64, 1e-12)
    w = inputs.workload("tiny")
    plan = wg.Plan(w["N"], w["L"], w["W"], w["x0"], w["wmax"], device=DEV, max_workspace_bytes=1)   # layer passes
    uvw = torch.from_numpy(w["uvw"]).to(DEV)
    vis = torch.from_numpy(w["vis"]).to(DEV, cdt)
    img = torch.from_numpy(inputs.random_image(w["N"], 181)).to(DEV, rdt)
    dirty = torch.empty((w["N"], w["N"]), dtype=rdt, device=DEV)
    out = torch.empty(uvw.shape[0], dtype=cdt, device=DEV)

    def step():
        plan.prepare(uvw, rdt)
        plan.grid_prepared(vis, out=dirty)
        plan.degrid_prepared(img, out=out)

    step()
    torch.cuda.synchronize()
    ref_g, ref_d = dirty.clone(), out.clone()
    side = torch.cuda.Stream()                       # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                       # warm the side stream before capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        step()
    torch.cuda.synchronize()
    for r in range(4):
        dirty.zero_()
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        eg = rel(dirty, ref_g)
        print(f"fp{prec} replay {r}: grid {eg:.2e}, degrid equal {bool(torch.equal(out, ref_d))}")
        assert torch.equal(out, ref_d) and eg <= tol, (r, eg)
        plan.degrid(uvw, img)                        # eager work between replays (its own binning)
        plan.prepare(uvw, rdt)
        torch.cuda.synchronize()
    plan.close()
