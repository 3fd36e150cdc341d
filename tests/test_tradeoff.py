"""The accuracy trade-off of the w-kernel (Sec. 6.1) from the library's own
least-misfit design (host only): layer factors 1 / (2 z0) at E = 1e-7 relative
to W_z = 7 against the ratios the paper reads off its figure, and the error at
the bisected z0 against the oracle's independent design."""
import json
import os

import pytest

from oracle.kernel_design import least_misfit
from paper_2101_11172_amd import tradeoff

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "layer_factors.json")


def test_layer_factors_match_the_paper():
    g = json.load(open(GOLDEN))
    base = tradeoff.layer_factor(7, g["E"])
    assert 1.9 < base < 2.2      # z0 just below 1/4 at E = 1e-7 (E(7, 1/4) = 1.2e-7)
    for W, ratio in g["relative_to_W7"].items():
        got = tradeoff.layer_factor(int(W), g["E"]) / base
        assert abs(got / ratio - 1.0) <= 0.15, (W, got, ratio)


@pytest.mark.parametrize("W,E", [(4, 1e-7), (3, 1e-5)])
def test_bisected_z0_against_the_oracle_design(W, E):
    z0 = tradeoff.z0_for_error(W, E)
    assert abs(least_misfit(W, z0).E / E - 1.0) <= 1e-3


def test_wider_kernels_need_fewer_layers():
    t = tradeoff.tradeoff_table(widths=(2, 3, 4, 5, 6, 7), errors=(1e-5,))
    f = [t[(W, 1e-5)] for W in (2, 3, 4, 5, 6, 7)]
    assert all(b < a for a, b in zip(f, f[1:])), f
