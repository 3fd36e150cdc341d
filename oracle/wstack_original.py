"""Original W-stacking, Algorithms 3 and 4, step by step (oracle, FP64).

Test infrastructure: see ``oracle/__init__.py``.

The comparison method of Sec. 4: visibilities are binned in w by the
nearest-midpoint rule, each bin is gridded in two dimensions only (u, v, with
the least-misfit C of width W and cropping x0), transformed, cropped and
phase-rotated by exp{i 2 pi w[t] (n - 1)} with its bin centre w[t], and the
bins' images are summed and corrected by h_x h_y.  Degridding (Algorithm 4) is
the transpose: correct, phase-rotate by exp{-i 2 pi w[t] (n - 1)}, zero-pad,
FFT, and a visibility is computed from its bin's plane as if it were measured
at (u, v, w[t]).

Readings (listed in the design doc):

* the Hermitian fold of Sec. 5.4 is applied first, as in the improved method,
  so the bins cover [w_min, w_max] = [0, w_max] (the paper: w_min "can be
  taken as zero");
* N_w bins of width dw = w_max / N_w with midpoints w[t] = (t + 1/2) dw
  (Algorithm 3 step 3; Algorithm 4 prints t - 0.5, read as the same midpoints,
  since the bins are those of Algorithm 3);
* bin t holds t dw <= w < (t + 1) dw (the set S[t] of Sec. 4), the last bin
  closed at w_max;
* the default N_w is eq. N_w's smallest integer, ceil(2 pi (n_max - n_min) w_max);
* only h_x h_y corrects the sum (Algorithm 3 step 5: the two-dimensional
  gridding correction); no function of z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.fft

from .kernel_design import LeastMisfit
from .plan import layers_original
from .wstack import _WORKERS, _crop, _fold, support


@dataclass(frozen=True)
class OriginalPlan:
    N: int
    L: float
    W: int
    x0: float
    wmax: float
    n_bins: int
    Nprime: int
    l_max: float
    n_min: float

    @property
    def dw(self) -> float:
        return self.wmax / self.n_bins

    def w_centre(self, t) -> np.ndarray:
        """Bin midpoints w[t] = (t + 1/2) dw."""
        return (np.asarray(t, dtype=np.float64) + 0.5) * self.dw

    def pixel_lm(self):
        i = np.arange(self.N, dtype=np.float64) - self.N // 2
        return i * (self.L / self.N)

    def pixel_x(self):
        return (np.arange(self.N, dtype=np.float64) - self.N // 2) / self.Nprime

    def n_minus_1(self):
        """n - 1 on the [m, l] pixel grid, as -(l^2 + m^2) / (1 + n)."""
        l = self.pixel_lm()
        r2 = l[None, :] ** 2 + l[:, None] ** 2
        return -r2 / (1.0 + np.sqrt(1.0 - r2))


def make_original_plan(N: int, L: float, W: int, x0: float, wmax: float, n_bins: int | None = None) -> OriginalPlan:
    """Plan of Algorithm 3 step 1: N_w bins over [0, wmax] (default: eq. N_w)."""
    if N <= 0 or N % 2:
        raise ValueError("N must be positive and even")
    if not (0.0 < x0 <= 0.5) or not (1 <= W <= 16):
        raise ValueError("x0 must be in (0, 1/2] and W in [1, 16]")
    Np = N / (2.0 * x0)
    if abs(Np - round(Np)) > 1e-9:
        raise ValueError("N / (2 x0) must be an integer")
    if not (0.0 < L < math.sqrt(2.0)) or not (wmax > 0.0):
        raise ValueError("L must be in (0, sqrt 2) and wmax > 0")
    l_max = 0.5 * L
    n_min = math.sqrt(1.0 - 2.0 * l_max * l_max)
    if n_bins is None:
        n_bins = max(1, layers_original((1.0 - n_min) * wmax))
    if n_bins < 1:
        raise ValueError("n_bins must be >= 1")
    return OriginalPlan(N=N, L=L, W=W, x0=x0, wmax=wmax, n_bins=int(n_bins), Nprime=int(round(Np)),
                        l_max=l_max, n_min=n_min)


def assign_bins(plan: OriginalPlan, w: np.ndarray) -> np.ndarray:
    """Nearest-midpoint bin of each folded w (Algorithm 3 step 2)."""
    t = np.floor(w / plan.dw).astype(np.int64)
    return np.minimum(t, plan.n_bins - 1)


def correction_2d(plan: OriginalPlan, lm: LeastMisfit) -> np.ndarray:
    """h_x(x) h_y(y) on the [j, i] pixel grid (Algorithm 3 step 5)."""
    hx = lm.h(plan.pixel_x())
    return hx[None, :] * hx[:, None]


def _uv_weights(plan: OriginalPlan, lm: LeastMisfit, uvw_f: np.ndarray):
    up = (plan.l_max / plan.x0) * uvw_f[:, 0]
    vp = (plan.l_max / plan.x0) * uvw_f[:, 1]
    r_first, nu_r = support(up, plan.W)
    s_first, nu_s = support(vp, plan.W)
    return r_first, lm.c(nu_r), s_first, lm.c(nu_s)


def grid(plan: OriginalPlan, lm: LeastMisfit, uvw, vis) -> np.ndarray:
    """Dirty map by Algorithm 3.  Returns the real [N, N] map."""
    W, Np = plan.W, plan.Nprime
    uvw_f, neg = _fold(uvw)
    V = np.asarray(vis, dtype=np.complex128).reshape(-1)
    V = np.where(neg, np.conj(V), V)
    keep = uvw_f[:, 2] <= plan.wmax
    uvw_f, V = uvw_f[keep], V[keep]
    t_bin = assign_bins(plan, uvw_f[:, 2])                              # step 2
    r_first, cx, s_first, cy = _uv_weights(plan, lm, uvw_f)
    nm1 = plan.n_minus_1()
    crop = _crop(plan)
    acc = np.zeros((plan.N, plan.N), dtype=np.complex128)
    aW = np.arange(W)
    for t in np.unique(t_bin):                                          # step 3 (empty bins add zero)
        k = np.nonzero(t_bin == t)[0]
        rr = (r_first[k, None] + aW[None, :]) % Np
        ss = (s_first[k, None] + aW[None, :]) % Np
        contrib = V[k, None, None] * cy[k, :, None] * cx[k, None, :]    # step 3a: 2-D gridding
        flat = (ss[:, :, None] * Np + rr[:, None, :]).ravel()
        G = (np.bincount(flat, weights=contrib.real.ravel(), minlength=Np * Np)
             + 1j * np.bincount(flat, weights=contrib.imag.ravel(), minlength=Np * Np)).reshape(Np, Np)
        P = scipy.fft.ifft2(G, workers=_WORKERS) * (Np * Np)           # step 3b
        acc += P[np.ix_(crop, crop)] * np.exp(2j * np.pi * plan.w_centre(t) * nm1)   # step 3c; step 4
    return (acc * correction_2d(plan, lm)).real                        # step 5


def degrid(plan: OriginalPlan, lm: LeastMisfit, uvw, image) -> np.ndarray:
    """Model visibilities by Algorithm 4.  Returns complex [M]."""
    W, Np, N = plan.W, plan.Nprime, plan.N
    f = np.asarray(image, dtype=np.float64).reshape(N, N)
    g = f * correction_2d(plan, lm)                                     # step 2a: correct
    uvw_f, neg = _fold(uvw)
    out = np.zeros(uvw_f.shape[0], dtype=np.complex128)
    keep = np.nonzero(uvw_f[:, 2] <= plan.wmax)[0]
    t_bin = assign_bins(plan, uvw_f[keep, 2])
    r_first, cx, s_first, cy = _uv_weights(plan, lm, uvw_f[keep])
    nm1 = plan.n_minus_1()
    crop = _crop(plan)
    aW = np.arange(W)
    for t in np.unique(t_bin):
        pad = np.zeros((Np, Np), dtype=np.complex128)
        pad[np.ix_(crop, crop)] = g * np.exp(-2j * np.pi * plan.w_centre(t) * nm1)   # pad, phase
        Q = scipy.fft.fft2(pad, workers=_WORKERS)                       # step 2b
        j = np.nonzero(t_bin == t)[0]
        rr = (r_first[j, None] + aW[None, :]) % Np
        ss = (s_first[j, None] + aW[None, :]) % Np
        vals = Q[ss[:, :, None], rr[:, None, :]]                        # step 2c: 2-D correlation
        acc = np.sum(vals * cy[j, :, None] * cx[j, None, :], axis=(1, 2))
        k = keep[j]
        out[k] = np.where(neg[k], np.conj(acc), acc)
    return out


def rms_in_square(a: np.ndarray, b: np.ndarray, Nprime: int, R: float, relative: bool = True) -> float:
    """RMS of a - b over the pixels with |x_i| <= R and |y_j| <= R, x_i = (i - N/2) / N'
    (the central-square diagnostic of Sec. 6.3); relative: divided by the RMS of b
    over the same pixels."""
    N = a.shape[0]
    x = (np.arange(N) - N // 2) / Nprime
    m = np.abs(x) <= R + 1e-15
    d = (a - b)[np.ix_(m, m)]
    e = float(np.sqrt(np.mean(np.abs(d) ** 2)))
    if relative:
        e /= float(np.sqrt(np.mean(np.abs(b[np.ix_(m, m)]) ** 2)))
    return e
