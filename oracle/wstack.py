"""Improved W-stacking, Algorithms 5 and 6, step by step (oracle, FP64).

Test infrastructure: see ``oracle/__init__.py``.

Conventions (readings listed in the design doc):

* images are real arrays [N, N] indexed [j, i]: row j <-> m_j, column i <-> l_i;
* u' = (l_max / x0) u, v' = (m_max / y0) v, w' = n_scale w (Sec. 5.2);
* support of one coordinate xi (Sec. 3.3, definition of nu_k): F = floor(xi + W/2),
  nu = xi + W/2 - F - 1/2 in [-1/2, 1/2); the W grid points F - W + 1 + a
  (a = 0 ... W-1) carry the weights C(F - W + 1 + a - xi) = c_{s_a}(nu) with
  s_a = a - (W-1)/2;
* uv-grid points are indexed modulo N' (the FFT is periodic in r, s), w-layers by
  t - t_lo;
* all transforms are unnormalised (scipy.fft on every core); dirty map uses
  e^{+i}, visibilities e^{-i} (eq. fourier_visibility); no natural weights 1/M;
  the image is f = I/n;
* Hermitian fold (Sec. 5.4): a visibility with w < 0 is replaced by its conjugate
  at (-u, -v, -w); visibilities with |w| > w_max are skipped (degrid returns 0).

``grid`` and ``degrid`` are compositions of the step functions below, which
follow the algorithms' numbered steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import os

import numpy as np
import scipy.fft

from .kernel_design import LeastMisfit
from .plan import Plan


# threads for the library 2-D transforms (the only multi-threaded step)
_WORKERS = os.cpu_count() or 1


def support(xi: np.ndarray, W: int):
    """First grid index F - W + 1 and fractional offset nu for coordinates xi."""
    F = np.floor(xi + 0.5 * W)
    nu = xi + 0.5 * W - F - 0.5
    return F.astype(np.int64) - W + 1, nu


def _fold(uvw: np.ndarray):
    uvw = np.asarray(uvw, dtype=np.float64).reshape(-1, 3)
    neg = uvw[:, 2] < 0.0
    sgn = np.where(neg, -1.0, 1.0)
    return uvw * sgn[:, None], neg


def _normalised(plan: Plan, uvw_f: np.ndarray):
    up = (plan.l_max / plan.x0) * uvw_f[:, 0]
    vp = (plan.l_max / plan.x0) * uvw_f[:, 1]
    wp = plan.n_scale * uvw_f[:, 2]
    return up, vp, wp


def _weights(lm: LeastMisfit, xi: np.ndarray, W: int):
    first, nu = support(xi, W)
    return first, lm.c(nu)                      # [M], [M, W]


_CORRECTIONS: dict = {}


def correction(plan: Plan, lm: LeastMisfit, lmz: LeastMisfit | None = None) -> np.ndarray:
    """h_x(x) h_y(y) h_z(z(x, y)) on the [j, i] pixel grid (Algorithm 5 step 5);
    h_x = h_y from lm, h_z from lmz (by default lm).

    The map depends only on the plan and the designs, so the last few are kept
    (read-only) for the next grid or degrid call."""
    lmz = lm if lmz is None else lmz
    key = (plan, id(lm), id(lmz))
    if key not in _CORRECTIONS:
        hx = lm.h(plan.pixel_x())
        hz = lmz.h(plan.z().ravel()).reshape(plan.N, plan.N)
        c = hx[None, :] * hx[:, None] * hz
        c.setflags(write=False)
        if len(_CORRECTIONS) >= 4:
            _CORRECTIONS.pop(next(iter(_CORRECTIONS)))
        _CORRECTIONS[key] = (lm, lmz, c)
    return _CORRECTIONS[key][2]


def _crop(plan: Plan) -> np.ndarray:
    """FFT bins of image indices 0 ... N-1: (i - N/2) mod N' (Algorithm 5 step 3c)."""
    return (np.arange(plan.N) - plan.N // 2) % plan.Nprime


# ---------------------------------------------------------------- Algorithm 5

@dataclass
class GridInput:
    """Folded, normalised visibilities with their phase and kernel weights."""
    Vh: np.ndarray          # V exp[i 2 pi w (n0 - 1)]
    t_first: np.ndarray
    cz: np.ndarray
    r_first: np.ndarray
    cx: np.ndarray
    s_first: np.ndarray
    cy: np.ndarray


def grid_prepare(plan: Plan, lm: LeastMisfit, uvw, vis, lmz: LeastMisfit | None = None) -> GridInput:
    """Fold (Sec. 5.4), skip |w| > w_max, multiply by exp[i 2 pi w (n0 - 1)] (step 2),
    and evaluate the weights per axis (W on u and v with lm, W_z on w with lmz,
    by default lm)."""
    W, lmz = plan.W, lm if lmz is None else lmz
    uvw_f, neg = _fold(uvw)
    V = np.asarray(vis, dtype=np.complex128).reshape(-1)
    V = np.where(neg, np.conj(V), V)
    keep = uvw_f[:, 2] <= plan.wmax
    uvw_f, V = uvw_f[keep], V[keep]
    up, vp, wp = _normalised(plan, uvw_f)
    # n0 - 1 = -z_shift n_scale (eq. n_params; 0 without z offset)
    Vh = V * np.exp(2j * np.pi * uvw_f[:, 2] * (-plan.z_shift * plan.n_scale))
    t_first, cz = _weights(lmz, wp, plan.W_z)
    r_first, cx = _weights(lm, up, W)
    s_first, cy = _weights(lm, vp, W)
    return GridInput(Vh, t_first, cz, r_first, cx, s_first, cy)


def grid_layer(plan: Plan, gi: GridInput, t: int) -> np.ndarray:
    """Steps 2-3a for layer t: values assigned to the layer with weight C_z(t - w'),
    then 2-D convolutional gridding with C_x, C_y.  Returns G_t [s, r]."""
    W, Np = plan.W, plan.Nprime
    c_idx = t - gi.t_first
    k = np.nonzero((c_idx >= 0) & (c_idx < plan.W_z))[0]
    if k.size == 0:
        return np.zeros((Np, Np), dtype=np.complex128)
    val = gi.Vh[k] * gi.cz[k, c_idx[k]]
    rr = (gi.r_first[k, None] + np.arange(W)[None, :]) % Np          # [nk, W]
    ss = (gi.s_first[k, None] + np.arange(W)[None, :]) % Np
    contrib = val[:, None, None] * gi.cy[k, :, None] * gi.cx[k, None, :]   # [nk, Wy, Wx]
    flat = (ss[:, :, None] * Np + rr[:, None, :]).ravel()
    return (np.bincount(flat, weights=contrib.real.ravel(), minlength=Np * Np)
            + 1j * np.bincount(flat, weights=contrib.imag.ravel(), minlength=Np * Np)).reshape(Np, Np)


def layer_image(plan: Plan, G: np.ndarray, t: int, z: np.ndarray) -> np.ndarray:
    """Steps 3b-3d: unnormalised 2-D IFFT, crop, phase exp(i 2 pi t z)."""
    Np = plan.Nprime
    crop = _crop(plan)
    P = scipy.fft.ifft2(G, workers=_WORKERS) * (Np * Np)
    return P[np.ix_(crop, crop)] * np.exp(2j * np.pi * t * z)


def grid(plan: Plan, lm: LeastMisfit, uvw, vis, dump: dict | None = None,
         lmz: LeastMisfit | None = None) -> np.ndarray:
    """Dirty map by Algorithm 5.  Returns the real [N, N] map.  lmz: the w-axis
    design (width plan.W_z, cropping plan.z0), by default lm."""
    gi = grid_prepare(plan, lm, uvw, vis, lmz)
    z = plan.z()
    acc = np.zeros((plan.N, plan.N), dtype=np.complex128)
    stack = [] if dump is not None else None
    for t in range(plan.t_lo, plan.t_hi + 1):
        G = grid_layer(plan, gi, t)
        if stack is not None:
            stack.append(G)
        acc += layer_image(plan, G, t, z)              # step 4: accumulate
    corr = correction(plan, lm, lmz)                    # step 5
    if dump is not None:
        dump["stack"] = np.array(stack)
        dump["acc"] = acc
        dump["corr"] = corr
    return (acc * corr).real


# ---------------------------------------------------------------- Algorithm 6

def degrid_layer(plan: Plan, g: np.ndarray, t: int, z: np.ndarray) -> np.ndarray:
    """Steps 3a-3c for layer t: phase exp(-i 2 pi t z), zero pad, unnormalised 2-D FFT."""
    Np = plan.Nprime
    crop = _crop(plan)
    pad = np.zeros((Np, Np), dtype=np.complex128)
    pad[np.ix_(crop, crop)] = g * np.exp(-2j * np.pi * t * z)
    return scipy.fft.fft2(pad, workers=_WORKERS)


def degrid_correlate(plan: Plan, lm: LeastMisfit, uvw, stack: np.ndarray,
                     lmz: LeastMisfit | None = None) -> np.ndarray:
    """Steps 4-5: 3-D correlation with C_x C_y C_z, phase exp[-i 2 pi w (n0 - 1)],
    conjugate for folded visibilities (Sec. 5.4)."""
    W, Wz, Np = plan.W, plan.W_z, plan.Nprime
    lmz = lm if lmz is None else lmz
    uvw_f, neg = _fold(uvw)
    out = np.zeros(uvw_f.shape[0], dtype=np.complex128)
    keep = np.nonzero(uvw_f[:, 2] <= plan.wmax)[0]
    aW, aWz = np.arange(W), np.arange(Wz)
    for lo in range(0, keep.size, 4096):
        k = keep[lo:lo + 4096]
        up, vp, wp = _normalised(plan, uvw_f[k])
        t_first, cz = _weights(lmz, wp, Wz)
        r_first, cx = _weights(lm, up, W)
        s_first, cy = _weights(lm, vp, W)
        tt = (t_first[:, None] + aWz[None, :]) - plan.t_lo                # [nk, W_z]
        ss = (s_first[:, None] + aW[None, :]) % Np
        rr = (r_first[:, None] + aW[None, :]) % Np
        vals = stack[tt[:, :, None, None], ss[:, None, :, None], rr[:, None, None, :]]
        wgt = cz[:, :, None, None] * cy[:, None, :, None] * cx[:, None, None, :]
        acc = np.sum(vals * wgt, axis=(1, 2, 3))
        acc = acc * np.exp(-2j * np.pi * uvw_f[k, 2] * (-plan.z_shift * plan.n_scale))
        out[k] = np.where(neg[k], np.conj(acc), acc)
    return out


def degrid(plan: Plan, lm: LeastMisfit, uvw, image, dump: dict | None = None,
           lmz: LeastMisfit | None = None) -> np.ndarray:
    """Model visibilities by Algorithm 6.  Returns complex [M].  lmz as for grid."""
    N, Np = plan.N, plan.Nprime
    f = np.asarray(image, dtype=np.float64).reshape(N, N)
    g = f * correction(plan, lm, lmz)                    # step 2
    z = plan.z()
    stack = np.zeros((plan.n_layers, Np, Np), dtype=np.complex128)
    for t in range(plan.t_lo, plan.t_hi + 1):            # step 3
        stack[t - plan.t_lo] = degrid_layer(plan, g, t, z)
    if dump is not None:
        dump["stack"] = stack
    return degrid_correlate(plan, lm, uvw, stack, lmz)   # steps 4-5
