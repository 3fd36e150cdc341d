"""Pins for the oracle's least-misfit kernel design (CPU).

Each check is fixed by the paper or by mathematics, not by re-running the
oracle's own formulas:
* Sec. 6.1 prints E = 1.3e-7 for W = 7, x0 = 0.25;
* Sec. 6.3 (Fig. rms_relative_error) and Sec. 8: E falls steeply with W; smaller
  x0 makes it fall faster; x0 = 1/3 costs about an order of magnitude at W = 7;
* Sec. 6.2 (original method): with a top hat C and h = 1/sinc,
  L = 1 - exp(-i 2 pi nu z) / sinc z, whose map error is 1/sinc^2 - 1 in closed
  form, and E/z0 -> pi/3 as z0 -> 0 (the printed constant sqrt(pi/3) is read as
  a typo);
* C is even (Algorithm 1 box), so c_{-s}(-nu) = c_s(nu); h is even;
* h is the pointwise optimum for the converged C (stationarity of eq. norm_bound).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.kernel_design import LeastMisfit, error_bound, least_misfit, map_error


def test_error_bound_printed_value():
    # Sec. 6.1: least-misfit, x0 = 0.25, W = 7 achieves E = 1.3e-7
    E = least_misfit(7, 0.25).E
    assert 1.2e-7 <= E <= 1.4e-7, E


def test_error_falls_with_width():
    Es = [least_misfit(W, 0.25).E for W in range(1, 13)]
    for a, b in zip(Es, Es[1:]):
        assert b < 0.2 * a, Es
    # W = 7 is at the single-precision level (Sec. 6.3, Sec. 8)
    assert 1e-8 < Es[6] < 1e-6
    assert Es[11] < 1e-11


def test_smaller_crop_falls_faster():
    for W in range(3, 10):
        assert least_misfit(W, 0.2).E < least_misfit(W, 0.25).E < least_misfit(W, 1 / 3).E
    # Sec. 6.3: x0 = 1/3 costs about an order of magnitude at W = 7
    ratio = least_misfit(7, 1 / 3).E / least_misfit(7, 0.25).E
    assert 5.0 < ratio < 50.0, ratio


def _tophat_c(nu):
    return np.ones((np.size(nu), 1))


def _inv_sinc(x):
    return 1.0 / np.sinc(x)


@pytest.mark.parametrize("z", [0.01, 0.1, 0.25, 0.4])
def test_tophat_map_error_closed_form(z):
    # Sec. 6.2: W_z = 1 top hat with h = 1/sinc gives l(z) = 1/sinc^2 z - 1
    got = map_error(_tophat_c, _inv_sinc, 1, [z])[0]
    want = 1.0 / np.sinc(z) ** 2 - 1.0
    assert abs(got - want) <= 1e-12 * max(1.0, want)


@pytest.mark.parametrize("z0", [0.05, 0.25, 0.5])
def test_tophat_error_bound_closed_form(z0):
    got = error_bound(_tophat_c, _inv_sinc, 1, z0)
    integral, _ = quad(lambda z: 1.0 / np.sinc(z) ** 2 - 1.0, 0.0, z0, epsabs=1e-15, epsrel=1e-13)
    assert abs(got - math.sqrt(integral / z0)) <= 1e-10 * got


def test_tophat_small_z0_limit():
    z0 = 1e-3
    got = error_bound(_tophat_c, _inv_sinc, 1, z0)
    assert abs(got / z0 - math.pi / 3.0) < 1e-5


def test_kernel_is_even():
    lm = least_misfit(7, 0.25)
    nu = np.linspace(-0.5, 0.5, 41)
    c = lm.c(nu)
    c_mirror = lm.c(-nu)[:, ::-1]        # s -> -s, nu -> -nu
    assert np.max(np.abs(c - c_mirror)) <= 1e-12 * np.max(np.abs(c))
    u = np.linspace(-3.49, 3.49, 301)
    assert np.allclose(lm.kernel(u), lm.kernel(-u), rtol=0, atol=1e-12)
    x = np.linspace(0, 0.25, 17)
    assert np.allclose(lm.h(x), lm.h(-x), rtol=1e-14, atol=0)


def test_h_is_pointwise_optimum():
    lm = least_misfit(7, 0.25)
    rel = np.abs(lm.h(lm.xn) / lm.h_nodes - 1.0)
    assert rel.max() < 1e-8, rel.max()
    assert abs(lm.h([0.0])[0] - 1.0) < 1e-8       # scale convention h(0) = 1


def test_applied_product_independent_of_discretisation():
    # only h(x) g(x, nu) enters the operators; it must not depend on the node counts
    a = LeastMisfit(7, 0.25, n_x=24, n_nu=24)
    b = LeastMisfit(7, 0.25, n_x=48, n_nu=48)
    x = np.linspace(0, 0.25, 29)
    nu = np.linspace(-0.5, 0.5, 23)
    assert np.max(np.abs(a.hg(x, nu) - b.hg(x, nu))) < 5e-12
    assert abs(a.E - b.E) < 1e-3 * b.E


def test_kernel_support_and_size():
    lm = least_misfit(4, 0.25)
    # nu in [-1/2, 1/2) puts the support at (-W/2, W/2]
    assert lm.kernel(np.array([2.01, 2.5, -2.0, 7.0])).tolist() == [0.0, 0.0, 0.0, 0.0]
    assert lm.kernel(np.array([2.0]))[0] != 0.0
    assert lm.c(np.array([0.0])).shape == (1, 4)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        LeastMisfit(0, 0.25)
    with pytest.raises(ValueError):
        LeastMisfit(7, 0.6)
