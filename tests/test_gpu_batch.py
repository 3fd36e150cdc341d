"""Batched channels: grid_visibilities_batch / degrid_visibilities_batch.

Channels share one plan and differ in their visibilities (uvw scaled as for
channels at different frequencies, uneven counts including an empty channel).
Each channel's result must equal the single-channel call on that channel
(degrid bit for bit: the same parts summed in the same order; grid within
rounding: the LDS accumulation order of a tile is not fixed) and the FP64
oracle (1e-10 FP64, 1e-6 FP32, as in the parity tests).  With the smallest
workspace the layer passes cross channel boundaries.  13 layers per channel
at N = 64 leave 3 padding layers in each channel's last tile layer; 112 layers
at N = 128 give 7 tile layers per channel.
"""
import numpy as np
import pytest
import torch

from oracle import wstack
from oracle.kernel_design import least_misfit
from oracle.plan import make_plan
from paper_2101_11172_amd import inputs
from paper_2101_11172_amd import wsgrid as wg

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def channels(N, L, wmax, counts, seed):
    """Per channel: uvw of a common uniform draw scaled by its frequency ratio."""
    out = []
    for c, m in enumerate(counts):
        f = 1.0 - 0.3 * c / max(1, len(counts) - 1)          # frequency / highest frequency
        uvw = inputs.uniform_uvw(m, 0.9 * N / (2 * L), wmax, seed + c)
        out.append(uvw * np.array([f, f, f]))
    return out


CASES = [
    # N, L, W, x0, wmax, counts
    (64, 0.3, 7, 0.25, 100.0, [700, 0, 1300, 250]),
    (128, 0.8, 7, 0.25, 300.0, [2000, 3500, 900]),
]


@pytest.mark.parametrize("case", CASES, ids=["N64x4", "N128x3"])
def test_batch_matches_single_and_oracle(case):
    N, L, W, x0, wmax, counts = case
    uvws = channels(N, L, wmax, counts, 81)
    vis = [inputs.random_vis(m, 90 + c) for c, m in enumerate(counts)]
    imgs = np.stack([inputs.random_image(N, 95 + c) for c in range(len(counts))])
    op, lm = make_plan(N, L, W, x0, wmax), least_misfit(W, x0)
    uvw_all = torch.from_numpy(np.concatenate(uvws)).to(DEV)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    off = np.concatenate([[0], np.cumsum(counts)])
    for prec, tol in ((64, 1e-10), (32, 1e-6)):
        cdt = torch.complex128 if prec == 64 else torch.complex64
        rdt = torch.float64 if prec == 64 else torch.float32
        vis_all = torch.from_numpy(np.concatenate(vis)).to(DEV, cdt)
        img_all = torch.from_numpy(imgs).to(DEV, rdt)
        g = plan.grid_batch(uvw_all, counts, vis_all).cpu().double().numpy()
        d = plan.degrid_batch(uvw_all, counts, img_all).cpu().to(torch.complex128).numpy()
        for c, m in enumerate(counts):
            t_uvw = torch.from_numpy(uvws[c]).to(DEV)
            g1 = plan.grid(t_uvw, vis_all[off[c]:off[c + 1]].contiguous()).cpu().double().numpy()
            d1 = plan.degrid(t_uvw, img_all[c].contiguous()).cpu().to(torch.complex128).numpy()
            if m == 0:
                assert not np.any(g[c]) and d1.size == 0
                continue
            assert rel(g[c], g1) <= (1e-13 if prec == 64 else 1e-6), (prec, c, rel(g[c], g1))
            assert np.array_equal(d[off[c]:off[c + 1]], d1), (prec, c)
            ref_g = wstack.grid(op, lm, uvws[c], vis[c])
            ref_d = wstack.degrid(op, lm, uvws[c], imgs[c])
            assert rel(g[c], ref_g) <= tol, (prec, c, "grid", rel(g[c], ref_g))
            assert rel(d[off[c]:off[c + 1]], ref_d) <= tol, (prec, c, "degrid", rel(d[off[c]:off[c + 1]], ref_d))
    plan.close()


@pytest.mark.parametrize("case", CASES, ids=["N64x4", "N128x3"])
def test_batch_layer_passes_cross_channels(case):
    N, L, W, x0, wmax, counts = case
    uvws = channels(N, L, wmax, counts, 61)
    vis = np.concatenate([inputs.random_vis(m, 70 + c) for c, m in enumerate(counts)])
    imgs = np.stack([inputs.random_image(N, 75 + c) for c in range(len(counts))])
    uvw_all = torch.from_numpy(np.concatenate(uvws)).to(DEV)
    full = wg.Plan(N, L, W, x0, wmax, device=DEV)
    M = int(sum(counts))
    least = wg.grid_workspace_bytes_batch(full._p, wg.WSG_F64, len(counts), M, True)
    assert least < wg.grid_workspace_bytes_batch(full._p, wg.WSG_F64, len(counts), M)
    assert wg.grid_layers_per_pass(full._p, wg.WSG_F64, len(counts), M, least) == 16
    small = wg.Plan(N, L, W, x0, wmax, device=DEV, max_workspace_bytes=least)
    v = torch.from_numpy(vis).to(DEV)
    im = torch.from_numpy(imgs).to(DEV)
    g_full, g_small = full.grid_batch(uvw_all, counts, v), small.grid_batch(uvw_all, counts, v)
    d_full, d_small = full.degrid_batch(uvw_all, counts, im), small.degrid_batch(uvw_all, counts, im)
    assert small.workspace(wg.WSG_F64, M, len(counts)).numel() == least
    assert torch.equal(d_full, d_small)
    for c in range(len(counts)):
        if counts[c]:
            e = float(torch.linalg.vector_norm(g_full[c] - g_small[c]) / torch.linalg.vector_norm(g_full[c]))
            assert e <= 1e-13, (c, e)
    full.close()
    small.close()


def test_batch_rejects_bad_arguments():
    plan = wg.Plan(64, 0.3, 7, 0.25, 100.0, device=DEV)
    uvw = torch.zeros((10, 3), dtype=torch.float64, device=DEV)
    vis = torch.zeros(10, dtype=torch.complex64, device=DEV)
    with pytest.raises(ValueError):
        plan.grid_batch(uvw, [4, 5], vis)                      # counts do not add up
    ws = plan.workspace(wg.WSG_F32, 10, 1)
    out = torch.empty((65, 64, 64), dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError, match="channels"):
        wg.grid_visibilities_batch(plan._p, wg.WSG_F32, [0] * 65, uvw.data_ptr(), vis.data_ptr(), out.data_ptr(),
                                   ws.data_ptr(), ws.numel(), torch.cuda.current_stream(DEV).cuda_stream)
    plan.close()


def test_autotuner_picks_a_working_pass_size():
    from paper_2101_11172_amd.autotune import tune_pass_layers

    N, L, W, x0, wmax, counts = CASES[1]
    uvws = channels(N, L, wmax, counts, 41)
    M = int(sum(counts))
    uvw = torch.from_numpy(np.concatenate(uvws)).to(DEV)
    vis = torch.from_numpy(inputs.random_vis(M, 42)).to(DEV, torch.complex64)
    img = torch.from_numpy(np.stack([inputs.random_image(N, 43 + c) for c in range(len(counts))])).to(DEV,
                                                                                                      torch.float32)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    cap = wg.grid_workspace_bytes_batch(plan._p, wg.WSG_F32, len(counts), M)
    res = tune_pass_layers(plan, uvw, counts, vis, img, cap)
    assert len(res["ms"]) >= 2 and res["pass_layers"] in res["ms"]
    assert wg.grid_layers_per_pass(plan._p, wg.WSG_F32, len(counts), M, res["workspace_bytes"]) == res["pass_layers"]
    ref = plan.degrid_batch(uvw, counts, img)
    tuned = wg.Plan(N, L, W, x0, wmax, device=DEV, max_workspace_bytes=res["workspace_bytes"])
    assert torch.equal(tuned.degrid_batch(uvw, counts, img), ref)
    tuned.close()
    plan.close()


def test_multi_plan_channels_match_single_and_oracle():
    """grid/degrid_visibilities_multi: channels with plans of their own (image
    sizes 64^2 and 96^2, N' = 128 and 192, and their own wmax), consecutive
    channels sharing a plan batched together; each channel against the
    single-channel call with its plan (degrid bit for bit) and the oracle."""
    L, W, x0 = 0.3, 7, 0.25
    spec = [(64, 80.0), (64, 80.0), (96, 120.0), (96, 120.0), (96, 120.0)]     # (N_c, wmax of its plan)
    counts = [600, 0, 900, 400, 1100]
    plans = {key: wg.Plan(key[0], L, W, x0, key[1], device=DEV) for key in sorted(set(spec))}
    ps = wg.PlanSet([plans[k] for k in spec])
    uvws = [inputs.uniform_uvw(m, 0.9 * n / (2 * L), wmax, 300 + c) for c, ((n, wmax), m) in enumerate(zip(spec, counts))]
    vis = [inputs.random_vis(m, 310 + c) for c, m in enumerate(counts)]
    imgs = [inputs.random_image(n, 320 + c) for c, (n, _) in enumerate(spec)]
    uvw_all = torch.from_numpy(np.concatenate(uvws)).to(DEV)
    off = np.concatenate([[0], np.cumsum(counts)])
    for prec, tol in ((64, 1e-10), (32, 1e-6)):
        cdt, rdt = (torch.complex128, torch.float64) if prec == 64 else (torch.complex64, torch.float32)
        v_all = torch.from_numpy(np.concatenate(vis)).to(DEV, cdt)
        img_all = torch.cat([torch.from_numpy(f).to(DEV, rdt).reshape(-1) for f in imgs])
        maps = ps.maps(ps.grid(uvw_all, counts, v_all))
        vout = ps.degrid(uvw_all, counts, img_all).cpu().to(torch.complex128).numpy()
        for c, (n, wmax) in enumerate(spec):
            p = plans[(n, wmax)]
            op, lm = make_plan(n, L, W, x0, wmax), least_misfit(W, x0)
            u = torch.from_numpy(uvws[c]).to(DEV)
            g1 = p.grid(u, torch.from_numpy(vis[c]).to(DEV, cdt)).cpu().double().numpy()
            gm = maps[c].cpu().double().numpy()
            d1 = p.degrid(u, torch.from_numpy(imgs[c]).to(DEV, rdt)).cpu().to(torch.complex128).numpy()
            dm = vout[off[c]:off[c + 1]]
            assert np.array_equal(dm, d1), (prec, c)
            if counts[c] == 0:
                assert not np.any(gm)
                continue
            assert rel(gm, g1) <= (1e-14 if prec == 64 else 1e-6), (prec, c)
            assert rel(gm, wstack.grid(op, lm, uvws[c], vis[c])) <= tol, (prec, c)
            assert rel(dm, wstack.degrid(op, lm, uvws[c], imgs[c])) <= tol, (prec, c)
    # a plan that recurs after another plan's run is rejected before any launch
    bad = wg.PlanSet([plans[(64, 80.0)], plans[(96, 120.0)], plans[(64, 80.0)]])
    with pytest.raises(RuntimeError, match="consecutive"):
        bad.grid(uvw_all[:30].contiguous(), [10, 10, 10], torch.zeros(30, dtype=torch.complex64, device=DEV))
    for p in plans.values():
        p.close()


@pytest.mark.parametrize("cap", [None, 1], ids=["full", "smallest"])
def test_multi_plan_shared_binning_matches_multi(cap):
    """PlanSet.prepare + grid_prepared / degrid_prepared (one grid_prepare per
    run of channels on one plan, each run in its own workspace) against the
    plain multi-plan calls: degrid bit for bit, grid within rounding; with the
    smallest workspaces the runs go in layer passes."""
    L, W, x0 = 0.3, 7, 0.25
    spec = [(64, 80.0), (64, 80.0), (96, 300.0), (96, 300.0)]
    counts = [700, 300, 0, 1200]
    plans = {key: wg.Plan(key[0], L, W, x0, key[1], device=DEV) for key in sorted(set(spec))}
    uvw = torch.from_numpy(np.concatenate([inputs.uniform_uvw(m, 0.9 * n / (2 * L), wmax, 330 + c)
                                           for c, ((n, wmax), m) in enumerate(zip(spec, counts))])).to(DEV)
    vis = torch.from_numpy(inputs.random_vis(sum(counts), 340)).to(DEV)
    img = torch.cat([torch.from_numpy(inputs.random_image(n, 350 + c)).reshape(-1) for c, (n, _) in enumerate(spec)]).to(DEV)
    ps = wg.PlanSet([plans[k] for k in spec], max_workspace_bytes=cap)
    g_m, d_m = ps.grid(uvw, counts, vis).cpu().numpy(), ps.degrid(uvw, counts, img).cpu()
    ps.prepare(uvw, counts, torch.float64)
    g_p, d_p = ps.grid_prepared(vis).cpu().numpy(), ps.degrid_prepared(img).cpu()
    assert torch.equal(d_p, d_m)
    assert rel(g_p, g_m) <= 1e-13
    if cap is not None:
        assert any(wg.grid_layers_per_pass(p._p, wg.WSG_F64, c1 - c0, sum(counts[c0:c1]), w.numel())
                   < p.info["n_layers"] * (c1 - c0) for (p, c0, c1), w in zip(ps._runs(), ps._prep_ws))
    with pytest.raises(RuntimeError, match="prepare"):
        ps.grid_prepared(vis.to(torch.complex64))          # binned in FP64 only
    for p in plans.values():
        p.close()
