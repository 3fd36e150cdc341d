"""Pins for the oracle's planner (CPU): Table 2 layer counts, z range, n0."""
import json
import math
import os

import numpy as np
import pytest

from oracle.plan import layers_no_offset, layers_original, layers_required, make_plan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_layers.json")


def test_table2_layer_counts():
    # Table 2: one (n_max - n_min)(w_max - w_min) product reproduces every printed count
    g = json.load(open(GOLDEN))
    lo, hi = g["dn_dw_range"]
    for dn_dw in np.linspace(lo, hi, 9):
        for row in g["rows"]:
            if row["formula"] == "offset":
                got = layers_required(dn_dw, row["x0"], row["W"])
            elif row["formula"] == "no_offset":
                got = layers_no_offset(dn_dw, row["x0"], row["W"])
            else:
                got = layers_original(dn_dw)
            assert got == row["layers"], (dn_dw, row, got)


def test_z_spans_minus_z0_to_z0():
    # Sec. 5.3: z_max = +z0 at the map centre, z_min = -z0 at the corners
    p = make_plan(256, 0.4, 7, 0.25, 100.0)
    z = p.z()
    assert abs(z[128, 128] - 0.25) < 1e-15
    assert abs(z[0, 0] + 0.25) < 1e-12
    assert z.max() <= 0.25 + 1e-15 and z.min() >= -0.25 - 1e-12


def test_n_params_alt_form():
    # eq. n_params_alt: n0 = (n_max + n_min) / 2, n_scale = (n_max - n_min) / (2 z0)
    p = make_plan(512, 0.5, 5, 0.25, 10.0)
    n_min = math.sqrt(1 - 2 * 0.25 ** 2)
    assert abs(p.n0 - 0.5 * (1 + n_min)) < 1e-15
    assert abs(p.n_scale - (1 - n_min) / 0.5) < 1e-15


def test_fft_size_and_pixel_coordinates():
    p = make_plan(256, 0.2, 7, 0.25, 300.0)
    assert p.Nprime == 512
    x = p.pixel_x()
    assert x[0] == -0.25 and x[128] == 0.0
    # x = x0 l / l_max (Sec. 5.1)
    assert np.allclose(x, 0.25 * p.pixel_lm() / p.l_max, rtol=0, atol=1e-16)


def test_tiny_workload_layers():
    # 256^2, L = 0.2, W = 7, x0 = 0.25, |w| <= 300: layers -3 ... 9
    p = make_plan(256, 0.2, 7, 0.25, 300.0)
    assert (p.t_lo, p.t_hi, p.n_layers) == (-3, 9, 13)
    dn = 1 - p.n_min
    assert layers_required(dn * 300.0, 0.25, 7) == 14     # eq. count, one above touched


@pytest.mark.parametrize("args", [(255, 0.2, 7, 0.25, 1.0), (256, 0.2, 0, 0.25, 1.0),
                                  (256, 0.2, 7, 0.3, 1.0), (256, 1.5, 7, 0.25, 1.0),
                                  (256, 0.2, 7, 0.25, -1.0), (256, 0.2, 17, 0.25, 1.0)])
def test_invalid_plans(args):
    with pytest.raises(ValueError):
        make_plan(*args)


def test_no_offset_variant():
    # Sec. 5.3, eq. n_params_no_offset: n0 = 1, n_scale = (1 - n_min) / z0, so
    # z = 0 at the map centre and -z0 at the corners, twice the layer spacing rate
    p = make_plan(256, 0.4, 7, 0.25, 100.0)
    q = make_plan(256, 0.4, 7, 0.25, 100.0, z_offset=False)
    assert q.n0 == 1.0 and q.n_scale == 2.0 * p.n_scale and q.z_shift == 0.0
    z = q.z()
    assert z[128, 128] == 0.0
    assert abs(z[0, 0] + 0.25) < 1e-12
    assert z.max() == 0.0 and z.min() >= -0.25 - 1e-12
    # layers: floor(n_scale w_max + W/2) at the doubled n_scale
    assert q.t_lo == p.t_lo and q.t_hi == int(math.floor(q.n_scale * 100.0 + 3.5))
    assert q.n_layers > p.n_layers
