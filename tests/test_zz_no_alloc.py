"""grid_visibilities_noalloc (workspace in the library's static device buffer)
against grid_visibilities (caller's workspace), through the C-ABI.

Two calls in a row, the second with fewer visibilities than the first (the
buffer keeps the first call's contents, which the second must not see), in
both precisions, within the parity bar (FP64 1e-10, FP32 1e-6; the two calls
run the same kernels and differ only in the order of the scatter's LDS
atomics).  A plan too large for the buffer is rejected before any launch.
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


def test_noalloc_matches_grid_visibilities():
    w = inputs.workload("tiny")                       # N' = 512, 13 layers, 5,000 visibilities
    N, L, W, x0, wmax = w["N"], w["L"], w["W"], w["x0"], w["wmax"]
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    stream = torch.cuda.current_stream(DEV).cuda_stream
    bad = w["uvw"].copy()
    bad[::50, 2] = 2 * wmax                           # skipped: beyond wmax
    uvw_all = torch.from_numpy(bad).to(DEV)
    for prec, cdt, rdt, tol in ((wg.WSG_F64, torch.complex128, torch.float64, 1e-10),
                                (wg.WSG_F32, torch.complex64, torch.float32, 1e-6)):
        vis_all = torch.from_numpy(w["vis"]).to(DEV, cdt)
        for M in (5000, 1700):                         # the second call is smaller
            uvw, vis = uvw_all[:M].contiguous(), vis_all[:M].contiguous()
            ref = torch.empty((N, N), dtype=rdt, device=DEV)
            ws = torch.empty(wg.grid_workspace_bytes(plan._p, prec, M), dtype=torch.uint8, device=DEV)
            wg.grid_visibilities(plan._p, prec, M, uvw.data_ptr(), vis.data_ptr(), ref.data_ptr(),
                                 ws.data_ptr(), ws.numel(), stream)
            out = torch.full((N, N), float("nan"), dtype=rdt, device=DEV)
            wg.grid_visibilities_noalloc(plan._p, prec, M, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(), stream)
            torch.cuda.synchronize()
            e = rel(out, ref)
            print(f"prec {prec} M {M}: noalloc vs grid_visibilities rel {e:.3e}")
            assert torch.isfinite(out).all() and e <= tol, (prec, M, e)
            assert wg.grid_last_skipped(plan._p) == len(range(0, M, 50))
    plan.close()


def test_noalloc_rejects_a_plan_beyond_the_buffer():
    plan = wg.Plan(2048, 0.4, 7, 0.25, 500.0, device=DEV)   # one tile layer alone is 2 GB
    M = 10
    uvw = torch.zeros((M, 3), dtype=torch.float64, device=DEV)
    vis = torch.zeros(M, dtype=torch.complex64, device=DEV)
    out = torch.empty((2048, 2048), dtype=torch.float32, device=DEV)
    rc = wg.lib().grid_visibilities_noalloc(plan._p, wg.WSG_F32, M, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(),
                                            torch.cuda.current_stream(DEV).cuda_stream)
    assert rc == wg.WSG_EWORKSPACE and "scratch holds" in wg.grid_last_error()
    plan.close()
