"""One binning shared by gridding and degridding: grid_prepare and the prepared
calls, through the C-ABI.

The fold, coordinates, support boxes, tile binning and phase of Algorithm 5
step 2 and Algorithm 6 steps 4-5 depend on uvw alone, so the prepared calls
must give the plain calls' results: degrid bit for bit (the same records, the
same parts summed in the same order), grid within rounding (the gridding value
is formed from the stored degridding phase, and the LDS accumulation order of a
tile is not fixed).  Against the FP64 oracle the parity bars hold (1e-10 FP64,
1e-6 FP32).  A plain call on the workspace replaces the binning, and the
prepared calls then fail.
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


@pytest.mark.parametrize("cap", [None, 1], ids=["one-pass", "layer-passes"])
def test_prepared_matches_plain_and_oracle(cap):
    N, L, W, x0, wmax, M = 128, 0.5, 7, 0.25, 250.0, 4000
    uvw = inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 121)
    uvw[::97, 2] = 1.5 * wmax                          # beyond wmax: skipped by the binning
    vis, img = inputs.random_vis(M, 122), inputs.random_image(N, 123)
    op, lm = make_plan(N, L, W, x0, wmax), least_misfit(W, x0)
    ref_g, ref_d = wstack.grid(op, lm, uvw, vis), wstack.degrid(op, lm, uvw, img)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV, max_workspace_bytes=cap)
    t_uvw = torch.from_numpy(uvw).to(DEV)
    n_skip = int(np.count_nonzero(np.abs(uvw[:, 2]) > wmax))
    for prec, tol, same in ((64, 1e-10, 1e-13), (32, 1e-6, 1e-6)):
        cdt, rdt = (torch.complex128, torch.float64) if prec == 64 else (torch.complex64, torch.float32)
        t_vis, t_img = torch.from_numpy(vis).to(DEV, cdt), torch.from_numpy(img).to(DEV, rdt)
        g_plain = plan.grid(t_uvw, t_vis).cpu().double().numpy()
        d_plain = plan.degrid(t_uvw, t_img).cpu()
        plan.prepare(t_uvw, rdt)
        assert wg.grid_last_skipped(plan._p) == n_skip
        g1 = plan.grid_prepared(t_vis).cpu().double().numpy()
        d1 = plan.degrid_prepared(t_img).cpu()
        g2 = plan.grid_prepared(t_vis).cpu().double().numpy()      # the binning survives both directions
        print(f"fp{prec} cap={cap}: prepared vs plain grid {rel(g1, g_plain):.2e}; vs oracle grid "
              f"{rel(g1, ref_g):.2e} degrid {rel(d1.to(torch.complex128).numpy(), ref_d):.2e}")
        assert torch.equal(d1, d_plain)
        assert rel(g1, g_plain) <= same and rel(g2, g1) <= same
        assert rel(g1, ref_g) <= tol and rel(d1.to(torch.complex128).numpy(), ref_d) <= tol
        assert torch.all(d1[::97] == 0)
    if cap is not None:
        assert wg.grid_layers_per_pass(plan._p, wg.WSG_F32, 1, M, plan._ws[wg.WSG_F32].numel()) < plan.info["n_layers"]
    plan.close()


def test_plain_call_replaces_the_binning():
    N, L, W, x0, wmax, M = 64, 0.3, 7, 0.25, 100.0, 1500
    uvw = torch.from_numpy(inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 131)).to(DEV)
    vis = torch.from_numpy(inputs.random_vis(M, 132)).to(DEV, torch.complex64)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    plan.prepare(uvw, torch.float32)
    assert plan.prepared_for(torch.float32, uvw) and not plan.prepared_for(torch.float64)
    ws = plan._ws[wg.WSG_F32]
    dirty = plan.grid_prepared(vis)
    plan.grid(uvw, vis)                                  # a plain call on the same workspace
    assert not plan.prepared_for(torch.float32)
    with pytest.raises(RuntimeError, match="prepare"):
        plan.grid_prepared(vis)
    # the library itself refuses the stale workspace, and a wrong size or precision
    stream = torch.cuda.current_stream(DEV).cuda_stream
    with pytest.raises(RuntimeError, match="grid_prepare"):
        wg.grid_visibilities_prepared(plan._p, wg.WSG_F32, vis.data_ptr(), dirty.data_ptr(), ws.data_ptr(),
                                      ws.numel(), stream)
    plan.prepare(uvw, torch.float32)
    ws = plan._ws[wg.WSG_F32]
    for prec, nbytes in ((wg.WSG_F64, ws.numel()), (wg.WSG_F32, ws.numel() - 256)):
        with pytest.raises(RuntimeError, match="grid_prepare"):
            wg.grid_visibilities_prepared(plan._p, prec, vis.data_ptr(), dirty.data_ptr(), ws.data_ptr(), nbytes,
                                          stream)
    wg.grid_visibilities_prepared(plan._p, wg.WSG_F32, vis.data_ptr(), dirty.data_ptr(), ws.data_ptr(), ws.numel(),
                                  stream)
    # a change of uvw in place is seen by prepared_for
    uvw[0, 0] += 1.0
    assert not plan.prepared_for(torch.float32, uvw)
    plan.close()


def test_prepared_channels_match_batch():
    N, L, W, x0, wmax = 64, 0.3, 7, 0.25, 100.0
    counts = [700, 0, 1300]
    uvw = np.concatenate([inputs.uniform_uvw(m, 0.9 * N / (2 * L) * (1 - 0.2 * c), wmax, 141 + c)
                          for c, m in enumerate(counts)])
    vis = inputs.random_vis(uvw.shape[0], 145)
    imgs = np.stack([inputs.random_image(N, 146 + c) for c in range(len(counts))])
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    t_uvw = torch.from_numpy(uvw).to(DEV)
    t_vis, t_img = torch.from_numpy(vis).to(DEV), torch.from_numpy(imgs).to(DEV)
    g_b = plan.grid_batch(t_uvw, counts, t_vis).cpu().numpy()
    d_b = plan.degrid_batch(t_uvw, counts, t_img).cpu()
    plan.prepare(t_uvw, torch.float64, counts)
    g_p = plan.grid_prepared(t_vis).cpu().numpy()
    d_p = plan.degrid_prepared(t_img).cpu()
    assert g_p.shape == (3, N, N) and torch.equal(d_p, d_b)
    for c in (0, 2):
        assert rel(g_p[c], g_b[c]) <= 1e-13
    assert np.all(g_p[1] == 0)
    plan.close()


def test_autograd_uses_the_shared_binning():
    N, L, W, x0, wmax, M = 64, 0.3, 7, 0.25, 100.0, 1200
    uvw = torch.from_numpy(inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 151)).to(DEV)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    img = torch.from_numpy(inputs.random_image(N, 152)).to(DEV).requires_grad_(True)
    target = torch.from_numpy(inputs.random_vis(M, 153)).to(DEV)
    vis = wg.degrid_fn(plan, uvw, img)
    assert plan.prepared_for(torch.float64, uvw)
    loss = (vis - target).abs().pow(2).sum()
    loss.backward()
    ref = plan.grid(uvw, (2 * (vis.detach() - target)).contiguous())     # plain gridding of dL/dvis
    assert rel(img.grad.cpu().numpy(), ref.cpu().numpy()) <= 1e-13
    plan.close()


def test_widefield_prepared_step():
    """The benchmarked step at full size: 9,999,360 visibilities, 2048^2, 49
    layers.  Prepared FP32 results against the plain calls (degrid bit for
    bit; grid within 1e-6)."""
    w = inputs.workload("widefield")
    plan = wg.Plan(w["N"], w["L"], w["W"], w["x0"], w["wmax"], device=DEV)
    uvw = torch.from_numpy(w["uvw"]).to(DEV)
    vis = torch.from_numpy(w["vis"]).to(DEV)
    img = torch.from_numpy(inputs.random_image(w["N"], 161)).to(DEV, torch.float32)
    g_plain, d_plain = plan.grid(uvw, vis), plan.degrid(uvw, img)
    plan.prepare(uvw, torch.float32)
    g, d = plan.grid_prepared(vis), plan.degrid_prepared(img)
    e = float(torch.linalg.vector_norm(g.double() - g_plain.double()) / torch.linalg.vector_norm(g_plain.double()))
    print(f"widefield prepared vs plain: grid {e:.2e}")
    assert torch.equal(d, d_plain) and e <= 1e-6
    plan.close()


@pytest.mark.parametrize("variant", [dict(method="original", n_bins=12), dict(Wz=3, z0=0.2), dict(method="no_offset"),
                                     dict(x0=1 / 3)], ids=["original", "own-w-axis", "no-offset", "x0=1/3"])
def test_prepared_variants_match_plain(variant):
    """The shared binning under every planner variant: degrid bit for bit,
    grid within rounding of the plain calls, both directions against the oracle's
    adjoint identity."""
    v = dict(variant)
    N, L, W, wmax, M = 64, 0.4, 7, 120.0, 2000
    x0 = v.pop("x0", 0.25)
    uvw = torch.from_numpy(inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 171)).to(DEV)
    vis = torch.from_numpy(inputs.random_vis(M, 172)).to(DEV)
    img = torch.from_numpy(inputs.random_image(N, 173)).to(DEV)
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV, **v)
    g_plain, d_plain = plan.grid(uvw, vis).cpu().numpy(), plan.degrid(uvw, img).cpu()
    plan.prepare(uvw, torch.float64)
    g, d = plan.grid_prepared(vis).cpu().numpy(), plan.degrid_prepared(img).cpu()
    assert torch.equal(d, d_plain) and rel(g, g_plain) <= 1e-13
    lhs = float(torch.real(torch.vdot(vis.cpu(), d)))
    rhs = float(np.sum(img.cpu().numpy() * g))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    plan.close()


@pytest.mark.parametrize("W", [1, 3, 8, 12, 16])
def test_prepared_widths_match_plain(W):
    """Every scatter configuration on a shared binning: W <= 7 (16 records per
    round, coefficients in registers), W = 8 (32 records per round, registers),
    W >= 9 (32 per round, coefficients from memory), against the plain calls."""
    N, L, x0, wmax, M = 64, 0.4, 0.25, 120.0, 2500
    uvw = torch.from_numpy(inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 191 + W)).to(DEV)
    for cdt, rdt, same in ((torch.complex128, torch.float64, 1e-13), (torch.complex64, torch.float32, 1e-6)):
        vis = torch.from_numpy(inputs.random_vis(M, 192)).to(DEV, cdt)
        img = torch.from_numpy(inputs.random_image(N, 193)).to(DEV, rdt)
        plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
        g_plain, d_plain = plan.grid(uvw, vis).cpu().double().numpy(), plan.degrid(uvw, img).cpu()
        plan.prepare(uvw, rdt)
        g, d = plan.grid_prepared(vis).cpu().double().numpy(), plan.degrid_prepared(img).cpu()
        assert torch.equal(d, d_plain) and rel(g, g_plain) <= same, (W, rdt, rel(g, g_plain))
        plan.close()


@pytest.mark.parametrize("rdt", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_prepared_empty_and_all_skipped(rdt):
    """A binning of no visibilities, and one of visibilities all beyond wmax:
    the prepared grid gives a zero map, the prepared degrid an empty output or
    zeros, as the plain calls do."""
    cdt = torch.complex128 if rdt == torch.float64 else torch.complex64
    N, L, W, x0, wmax, M = 64, 0.3, 7, 0.25, 100.0, 500
    plan = wg.Plan(N, L, W, x0, wmax, device=DEV)
    img = torch.from_numpy(inputs.random_image(N, 201)).to(DEV, rdt)
    none = torch.zeros((0, 3), dtype=torch.float64, device=DEV)
    plan.prepare(none, rdt)
    assert torch.count_nonzero(plan.grid_prepared(torch.zeros(0, dtype=cdt, device=DEV))).item() == 0
    assert plan.degrid_prepared(img).numel() == 0
    far = inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 202)
    far[:, 2] = np.where(far[:, 2] >= 0, 1.5, -1.5) * wmax          # every |w| beyond wmax
    t_far = torch.from_numpy(far).to(DEV)
    vis = torch.from_numpy(inputs.random_vis(M, 203)).to(DEV, cdt)
    plan.prepare(t_far, rdt)
    assert wg.grid_last_skipped(plan._p) == M
    assert torch.count_nonzero(plan.grid_prepared(vis)).item() == 0
    d = plan.degrid_prepared(img)
    assert d.shape == (M,) and torch.count_nonzero(d).item() == 0
    plan.close()
