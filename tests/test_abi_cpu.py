"""Host-side checks of the C-ABI library (no GPU compute).

* the library loads and exports every function include/wsgrid.h declares;
* its planner gives the oracle planner's values;
* its own least-misfit design applies the same h(x) g(x, nu) as the oracle's
  (only this product enters the operators, see oracle.kernel_design);
* argument validation.
"""
import os

import numpy as np
import pytest
import torch

from oracle.kernel_design import least_misfit
from oracle.plan import make_plan
from paper_2101_11172_amd import wsgrid as wg


def test_exports_every_declared_function():
    names = wg.header_functions()
    assert "grid_create" in names and "degrid_visibilities" in names
    for n in names:
        assert hasattr(wg.lib(), n), n


@pytest.mark.parametrize("z_offset", [True, False])
@pytest.mark.parametrize("args", [(256, 0.2, 7, 0.25, 300.0), (2048, 0.4, 7, 0.25, 511.3),
                                  (2048, 0.4, 4, 0.5, 511.3), (64, 0.3, 5, 0.2, 10.0)])
def test_planner_matches_oracle(args, z_offset):
    got = wg.wsg_plan_params(*args, z_offset=z_offset)
    p = make_plan(*args, z_offset=z_offset)
    assert got["Nprime"] == p.Nprime and got["t_lo"] == p.t_lo and got["t_hi"] == p.t_hi
    assert got["n0"] == p.n0 and got["n_scale"] == p.n_scale


@pytest.mark.parametrize("W,x0,tol", [(7, 0.25, 1e-12), (4, 0.25, 1e-12), (5, 0.2, 1e-12), (9, 0.25, 1e-11),
                                      (10, 0.25, 1e-11), (4, 0.5, 1e-8)])
def test_design_applies_same_product_as_oracle(W, x0, tol):
    nu = np.linspace(-0.5, 0.5, 41)
    x = np.linspace(-x0, x0, 33)
    c, h, E = wg.wsg_design_eval(W, x0, nu, x)
    lm = least_misfit(W, x0)
    s = np.arange(W) - (W - 1) / 2
    g = np.einsum("js,jsi->ji", c, np.exp(2j * np.pi * (s[None, :, None] - nu[:, None, None]) * x[None, None, :]))
    assert np.max(np.abs(h[None, :] * g - lm.hg(x, nu))) <= tol
    assert abs(E - lm.E) <= 1e-6 * lm.E


def test_design_rejects_bad_arguments():
    with pytest.raises(RuntimeError):
        wg.wsg_design_eval(0, 0.25, [0.0], [0.0])
    with pytest.raises(RuntimeError):
        wg.wsg_design_eval(7, 0.25, [0.7], [0.0])
    with pytest.raises(RuntimeError):
        wg.wsg_plan_params(255, 0.2, 7, 0.25, 1.0)
    with pytest.raises(RuntimeError):
        wg.wsg_plan_params(256, 0.2, 7, 0.3, 1.0)


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device error path")
def test_create_without_device_fails_cleanly():
    assert not wg.lib().grid_create(256, 0.2, 7, 0.25, 300.0)
    assert "device" in wg.grid_last_error()


def test_probe_and_last_skipped_reject_bad_arguments():
    # argument checks happen before any device call
    assert wg.lib().wsg_bandwidth_probe(16, 4096, 15, None) == wg.WSG_EINVAL       # not a multiple of 16
    assert wg.lib().wsg_bandwidth_probe(8, 4096, 16, None) == wg.WSG_EINVAL        # misaligned
    assert wg.lib().wsg_bandwidth_probe(4096, 4104, 64, None) == wg.WSG_EINVAL     # overlapping (and misaligned)
    assert wg.lib().wsg_bandwidth_probe(4096, 4112, 64, None) == wg.WSG_EINVAL     # overlapping
    assert wg.lib().grid_last_skipped(None) == wg.WSG_EINVAL


def test_prepared_calls_reject_bad_arguments():
    # null plans are refused before any device call
    one = wg._counts([10])
    assert wg.lib().grid_prepare(None, wg.WSG_F32, 1, one, 4096, 8192, 1 << 20, None) == wg.WSG_EINVAL
    assert wg.lib().grid_visibilities_prepared(None, wg.WSG_F32, 4096, 8192, 16384, 1 << 20, None) == wg.WSG_EINVAL
    assert wg.lib().degrid_visibilities_prepared(None, wg.WSG_F64, 4096, 8192, 16384, 1 << 20, None) == wg.WSG_EINVAL
    assert "null plan" in wg.grid_last_error()


@pytest.mark.parametrize("args", [(64, 0.3, 7, 0.25, 3, 0.2, 100.0), (256, 0.4, 7, 0.25, 1, 0.05, 300.0),
                                  (96, 0.4, 5, 1 / 3, 5, 1 / 3, 50.0)])
@pytest.mark.parametrize("z_offset", [True, False])
def test_axes_planner_matches_oracle(args, z_offset):
    N, L, W, x0, Wz, z0, wmax = args
    method = wg.WSG_IMPROVED if z_offset else wg.WSG_IMPROVED_NO_OFFSET
    got = wg.wsg_plan_params_axes(N, L, W, x0, Wz, z0, wmax, method)
    p = make_plan(N, L, W, x0, wmax, z_offset=z_offset, Wz=Wz, z0=z0)
    assert (got["Nprime"], got["t_lo"], got["t_hi"]) == (p.Nprime, p.t_lo, p.t_hi)
    assert got["n0"] == p.n0 and got["n_scale"] == p.n_scale


@pytest.mark.parametrize("n_bins", [0, 1, 20, 470])
def test_original_planner_matches_oracle(n_bins):
    from oracle.wstack_original import make_original_plan
    got = wg.wsg_plan_params_axes(900, 0.1047, 7, 0.25, 1, 0.25, 2715.0, wg.WSG_ORIGINAL, n_bins)
    p = make_original_plan(900, 0.1047, 7, 0.25, 2715.0, n_bins or None)
    assert got["t_lo"] == 0 and got["t_hi"] == p.n_bins - 1 and got["n0"] == 1.0
    assert abs(got["n_scale"] - 1.0 / p.dw) <= 1e-15 * got["n_scale"]
    if n_bins == 0:
        assert p.n_bins == 47          # Table 2 row a, eq. N_w


def test_axes_planner_rejects_bad_arguments():
    with pytest.raises(RuntimeError):
        wg.wsg_plan_params_axes(64, 0.3, 7, 0.25, 3, 0.2, 100.0, wg.WSG_ORIGINAL)   # original needs W_z = 1
    with pytest.raises(RuntimeError):
        wg.wsg_plan_params_axes(64, 0.3, 7, 0.25, 8, 0.2, 100.0, wg.WSG_IMPROVED)   # W_z > W
    with pytest.raises(RuntimeError):
        wg.wsg_plan_params_axes(64, 0.3, 7, 0.25, 1, 0.2, 0.0, wg.WSG_ORIGINAL)     # no w range to bin


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as C99 and as C++ without warnings
    import shutil
    import subprocess
    hdr = os.path.abspath(wg.HEADER)
    src = tmp_path / "use.c"
    src.write_text(f'#include "{hdr}"\nint main(void) {{ return WSG_NSTAGES == 10 ? 0 : 1; }}\n')
    for cc, std in (("gcc", "-std=c99"), ("g++", "-std=c++17")):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        lang = ["-x", "c++"] if cc == "g++" else []
        r = subprocess.run([cc, std, "-Wall", "-Wextra", "-Werror", *lang, "-c", str(src), "-o", str(tmp_path / "o")],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
