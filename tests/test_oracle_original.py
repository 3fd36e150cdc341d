"""Pins for the oracle's original W-stacking, Algorithms 3 and 4 (CPU).

The truth is the exact DFT pair.  For the original method the error is set by
the nearest-bin approximation in w: a visibility at w = w[t] + d, d uniform
in [-dw/2, dw/2), contributes with the factor exp{-i 2 pi d (n - 1)} - 1 at a
pixel, whose mean square over d is 2 (1 - sinc(dw (n - 1))), sinc(x) =
sin(pi x)/(pi x).  For independent random visibility values the expected
relative error power of the dirty map at a pixel is that factor, so the
relative RMS error over the central square |x|, |y| <= R (the diagnostic of
Sec. 6.3) is sqrt(mean over its pixels of 2 (1 - sinc(dw (n - 1)))): small at
the map centre and growing outwards, and falling as 1/N_w (Sec. 6.2: the
error of the top hat is proportional to z0, hence to 1/N_w).  The x and y
gridding adds the least-misfit error E(W, x0), negligible here.  Exact
identities: the adjoint relation, the Hermitian fold, and visibilities at bin
midpoints (where only the 2-D gridding error remains).
"""
import numpy as np
import pytest

from oracle import dft, wstack_original as wo
from oracle.kernel_design import least_misfit
from oracle.plan import layers_original, make_plan
from paper_2101_11172_amd.inputs import random_image, random_vis, uniform_uvw


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def predicted(plan, R):
    x = (np.arange(plan.N) - plan.N // 2) / plan.Nprime
    m = np.abs(x) <= R + 1e-15
    nm1 = plan.n_minus_1()[np.ix_(m, m)]
    return float(np.sqrt(np.mean(2.0 * (1.0 - np.sinc(plan.dw * nm1)))))


N, L, W, x0, WMAX = 64, 0.5, 7, 0.25, 400.0


@pytest.fixture(scope="module")
def case():
    M = 6000
    uvw = uniform_uvw(M, 0.9 * N / (2 * L), WMAX, 31)
    V = random_vis(M, 32)
    p = make_plan(N, L, W, x0, WMAX)
    return uvw, V, dft.dft_grid(p, uvw, V)


@pytest.mark.parametrize("n_bins", [40, 163])       # 163: eq. N_w for this field and w range
def test_binning_error_closed_form(case, n_bins):
    uvw, V, exact = case
    p = wo.make_original_plan(N, L, W, x0, WMAX, n_bins)
    lm = least_misfit(W, x0)
    d = wo.grid(p, lm, uvw, V)
    # the squares hold 4,096, 1,089 and 289 pixels: the sampling spread of the
    # error power grows as the square shrinks (measured over seeds: within 4 %,
    # 7 % and 20 %)
    for R, tol in ((x0, 0.08), (x0 / 2, 0.12), (x0 / 4, 0.3)):
        got, want = wo.rms_in_square(d, exact, p.Nprime, R), predicted(p, R)
        assert abs(got / want - 1) < tol, (n_bins, R, got, want)
    # the error grows from the centre outwards by more than an order of magnitude
    ratio = predicted(p, x0) / predicted(p, x0 / 8)
    assert ratio > 20
    assert wo.rms_in_square(d, exact, p.Nprime, x0) / wo.rms_in_square(d, exact, p.Nprime, x0 / 8) > ratio / 2


def test_error_halves_with_twice_the_bins(case):
    uvw, V, exact = case
    lm = least_misfit(W, x0)
    e = [rel(wo.grid(wo.make_original_plan(N, L, W, x0, WMAX, nb), lm, uvw, V), exact) for nb in (40, 80)]
    assert abs(e[0] / e[1] - 2.0) < 0.15, e


def test_planted_mistakes_are_caught(case, monkeypatch):
    uvw, V, exact = case
    lm = least_misfit(W, x0)
    p = wo.make_original_plan(N, L, W, x0, WMAX, 163)
    good = wo.rms_in_square(wo.grid(p, lm, uvw, V), exact, p.Nprime, x0)
    # (1) bin centres at t dw (Algorithm 4's printed t - 0.5 taken literally would shift them the other way)
    monkeypatch.setattr(wo.OriginalPlan, "w_centre", lambda self, t: np.asarray(t, dtype=np.float64) * self.dw)
    bad = wo.rms_in_square(wo.grid(p, lm, uvw, V), exact, p.Nprime, x0)
    assert bad > 1.5 * good
    monkeypatch.undo()
    # (2) the bin phase with the wrong sign
    orig = wo.OriginalPlan.n_minus_1
    monkeypatch.setattr(wo.OriginalPlan, "n_minus_1", lambda self: -orig(self))
    assert wo.rms_in_square(wo.grid(p, lm, uvw, V), exact, p.Nprime, x0) > 10 * good


def test_visibilities_at_bin_midpoints():
    M = 800
    p = wo.make_original_plan(N, L, W, x0, WMAX, 10)
    uvw = uniform_uvw(M, 0.9 * N / (2 * L), WMAX, 41)
    t = np.random.default_rng(42).integers(0, 10, M)
    uvw[:, 2] = p.w_centre(t) * np.where(np.arange(M) % 2, -1.0, 1.0)       # some folded
    V = random_vis(M, 43)
    lm = least_misfit(W, x0)
    q = make_plan(N, L, W, x0, WMAX)
    assert rel(wo.grid(p, lm, uvw, V), dft.dft_grid(q, uvw, V)) <= 2 * np.sqrt(2) * lm.E
    f = random_image(N, 44)
    assert rel(wo.degrid(p, lm, uvw, f), dft.dft_degrid(q, uvw, f)) <= 2 * np.sqrt(2) * lm.E


def test_adjoint_and_hermitian():
    M = 500
    uvw = uniform_uvw(M, 0.9 * N / (2 * L), WMAX, 51)
    V, f = random_vis(M, 52), random_image(N, 53)
    p = wo.make_original_plan(N, L, W, x0, WMAX, 6)
    lm = least_misfit(W, x0)
    d = wo.degrid(p, lm, uvw, f)
    lhs = np.real(np.vdot(V, d))
    rhs = float(np.sum(f * wo.grid(p, lm, uvw, V)))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    assert np.max(np.abs(wo.degrid(p, lm, -uvw, f) - np.conj(d))) <= 1e-13 * np.max(np.abs(d))
    uvw2 = uvw.copy()
    uvw2[::5, 2] = 2 * WMAX                       # beyond wmax: skipped
    assert np.all(wo.degrid(p, lm, uvw2, f)[::5] == 0)


def test_default_bin_count_is_eq_N_w():
    # Table 2 row a: 47 bins from eq. N_w for the 6-degree field
    p = wo.make_original_plan(900, 0.1047, 7, 0.25, 2715.0)
    assert p.n_bins == layers_original((1 - p.n_min) * 2715.0) == 47


def test_rms_in_square():
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((64, 64)), rng.standard_normal((64, 64))
    assert abs(wo.rms_in_square(a, b, 128, 0.25) - rel(a, b)) < 1e-14      # R = x0: the whole map
    # R = 0: the centre pixel alone
    assert abs(wo.rms_in_square(a, b, 128, 0.0, relative=False) - abs(a[32, 32] - b[32, 32])) < 1e-15
