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
* all transforms are unnormalised; dirty map uses e^{+i}, visibilities e^{-i}
  (eq. fourier_visibility); no natural weights 1/M; the image is f = I/n;
* Hermitian fold (Sec. 5.4): a visibility with w < 0 is replaced by its conjugate
  at (-u, -v, -w); visibilities with |w| > w_max are skipped (degrid returns 0).
"""
from __future__ import annotations

import numpy as np

from .kernel_design import LeastMisfit
from .plan import Plan


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


def correction(plan: Plan, lm: LeastMisfit) -> np.ndarray:
    """h_x(x) h_y(y) h_z(z(x, y)) on the [j, i] pixel grid (Algorithm 5 step 5)."""
    hx = lm.h(plan.pixel_x())
    hz = lm.h(plan.z().ravel()).reshape(plan.N, plan.N)
    return hx[None, :] * hx[:, None] * hz


def _weights(lm: LeastMisfit, xi: np.ndarray, W: int):
    first, nu = support(xi, W)
    return first, lm.c(nu)                      # [M], [M, W]


def grid(plan: Plan, lm: LeastMisfit, uvw, vis, dump: dict | None = None) -> np.ndarray:
    """Dirty map by Algorithm 5.  Returns the real [N, N] map."""
    W, Np, N = plan.W, plan.Nprime, plan.N
    uvw_f, neg = _fold(uvw)
    V = np.asarray(vis, dtype=np.complex128).reshape(-1)
    V = np.where(neg, np.conj(V), V)
    keep = uvw_f[:, 2] <= plan.wmax
    uvw_f, V = uvw_f[keep], V[keep]
    up, vp, wp = _normalised(plan, uvw_f)

    # Step 2: multiply by exp[i 2 pi w (n0 - 1)], with n0 - 1 = -z0 n_scale (eq. n_params),
    # and spread over the W_z layers with weights C_z(t - w').
    Vh = V * np.exp(2j * np.pi * uvw_f[:, 2] * (-plan.z0 * plan.n_scale))
    t_first, cz = _weights(lm, wp, W)
    r_first, cx = _weights(lm, up, W)
    s_first, cy = _weights(lm, vp, W)

    z = plan.z()
    acc = np.zeros((N, N), dtype=np.complex128)
    crop = (np.arange(N) - N // 2) % Np
    stack = np.zeros((plan.n_layers, Np, Np), dtype=np.complex128) if dump is not None else None
    for t in range(plan.t_lo, plan.t_hi + 1):
        # visibilities assigned to layer t and their w-weights
        c_idx = t - t_first
        sel = (c_idx >= 0) & (c_idx < W)
        k = np.nonzero(sel)[0]
        G = np.zeros((Np, Np), dtype=np.complex128)
        if k.size:
            val = Vh[k] * cz[k, c_idx[k]]
            # Step 3a: 2-D convolutional gridding with C_x, C_y
            rr = (r_first[k, None] + np.arange(W)[None, :]) % Np        # [nk, W]
            ss = (s_first[k, None] + np.arange(W)[None, :]) % Np
            contrib = val[:, None, None] * cy[k, :, None] * cx[k, None, :]   # [nk, Wy, Wx]
            flat = (ss[:, :, None] * Np + rr[:, None, :]).ravel()
            G = (np.bincount(flat, weights=contrib.real.ravel(), minlength=Np * Np)
                 + 1j * np.bincount(flat, weights=contrib.imag.ravel(), minlength=Np * Np)
                 ).reshape(Np, Np)
        if stack is not None:
            stack[t - plan.t_lo] = G
        # Step 3b: unnormalised 2-D inverse FFT;  3c: crop;  3d: phase exp(i 2 pi t z)
        P = np.fft.ifft2(G) * (Np * Np)
        P = P[np.ix_(crop, crop)]
        # Step 4: accumulate
        acc += P * np.exp(2j * np.pi * t * z)
    # Step 5: 3-D gridding correction, real part
    corr = correction(plan, lm)
    if dump is not None:
        dump["stack"] = stack
        dump["acc"] = acc
        dump["corr"] = corr
    return (acc * corr).real


def degrid(plan: Plan, lm: LeastMisfit, uvw, image, dump: dict | None = None) -> np.ndarray:
    """Model visibilities by Algorithm 6.  Returns complex [M]."""
    W, Np, N = plan.W, plan.Nprime, plan.N
    f = np.asarray(image, dtype=np.float64).reshape(N, N)
    # Step 2: multiply by the 3-D correction
    corr = correction(plan, lm)
    g = f * corr
    z = plan.z()
    crop = (np.arange(N) - N // 2) % Np
    stack = np.zeros((plan.n_layers, Np, Np), dtype=np.complex128)
    for t in range(plan.t_lo, plan.t_hi + 1):
        # Step 3a: phase exp(-i 2 pi t z);  3b: zero pad;  3c: unnormalised 2-D FFT
        pad = np.zeros((Np, Np), dtype=np.complex128)
        pad[np.ix_(crop, crop)] = g * np.exp(-2j * np.pi * t * z)
        stack[t - plan.t_lo] = np.fft.fft2(pad)
    if dump is not None:
        dump["stack"] = stack

    uvw_f, neg = _fold(uvw)
    M = uvw_f.shape[0]
    out = np.zeros(M, dtype=np.complex128)
    keep = np.nonzero(uvw_f[:, 2] <= plan.wmax)[0]
    for lo in range(0, keep.size, 4096):
        k = keep[lo:lo + 4096]
        up, vp, wp = _normalised(plan, uvw_f[k])
        t_first, cz = _weights(lm, wp, W)
        r_first, cx = _weights(lm, up, W)
        s_first, cy = _weights(lm, vp, W)
        # Step 4: 3-D correlation with C_x C_y C_z
        aW = np.arange(W)
        tt = (t_first[:, None] + aW[None, :]) - plan.t_lo                 # [nk, W]
        ss = (s_first[:, None] + aW[None, :]) % Np
        rr = (r_first[:, None] + aW[None, :]) % Np
        vals = stack[tt[:, :, None, None], ss[:, None, :, None], rr[:, None, None, :]]
        wgt = cz[:, :, None, None] * cy[:, None, :, None] * cx[:, None, None, :]
        acc = np.sum(vals * wgt, axis=(1, 2, 3))
        # Step 5: phase exp[-i 2 pi w (n0 - 1)]
        acc = acc * np.exp(-2j * np.pi * uvw_f[k, 2] * (-plan.z0 * plan.n_scale))
        out[k] = np.where(neg[k], np.conj(acc), acc)
    return out
