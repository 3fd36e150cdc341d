"""Exact direct Fourier transforms that the method approximates (oracle, FP64).

Test infrastructure: see ``oracle/__init__.py``.

* degrid (eq. fourier_visibility with f = I/n, Sec. 5.2):
      V_k = sum_{j,i} f_{ji} exp[-i 2 pi (u_k l_i + v_k m_j + w_k (n_{ji} - 1))]
* grid (the dirty map, adjoint; Sec. 4 and 5.2, without the 1/M weights):
      D_{ji} = Re sum_k V_k exp[+i 2 pi (u_k l_i + v_k m_j + w_k (n_{ji} - 1))]
with n - 1 = -(l^2 + m^2) / (1 + n).  Both are evaluated in float64 by brute force,
optionally on a subset of pixels or visibilities.
"""
from __future__ import annotations

import numpy as np

from .plan import Plan


def _pixels(plan: Plan, rows=None, cols=None):
    l = plan.pixel_lm()
    if rows is None:
        jj, ii = np.meshgrid(np.arange(plan.N), np.arange(plan.N), indexing="ij")
        rows, cols = jj.ravel(), ii.ravel()
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    lp, mp = l[cols], l[rows]
    r2 = lp * lp + mp * mp
    return lp, mp, -r2 / (1.0 + np.sqrt(1.0 - r2)), rows, cols


def dft_grid(plan: Plan, uvw, vis, rows=None, cols=None, chunk: int = 2048) -> np.ndarray:
    """Exact dirty map.  With rows/cols given, returns the values at those pixels only."""
    uvw = np.asarray(uvw, dtype=np.float64).reshape(-1, 3)
    V = np.asarray(vis, dtype=np.complex128).reshape(-1)
    full = rows is None
    lp, mp, nm1, rows, cols = _pixels(plan, rows, cols)
    out = np.empty(lp.size)
    for lo in range(0, lp.size, chunk):
        sl = slice(lo, lo + chunk)
        ph = (uvw[:, 0:1] * lp[None, sl] + uvw[:, 1:2] * mp[None, sl]
              + uvw[:, 2:3] * nm1[None, sl])
        out[sl] = (V[:, None] * np.exp(2j * np.pi * ph)).sum(0).real
    return out.reshape(plan.N, plan.N) if full else out


def dft_degrid(plan: Plan, uvw, image, vis_index=None, chunk: int = 256) -> np.ndarray:
    """Exact model visibilities (all, or those listed in vis_index)."""
    uvw = np.asarray(uvw, dtype=np.float64).reshape(-1, 3)
    if vis_index is not None:
        uvw = uvw[np.asarray(vis_index)]
    f = np.asarray(image, dtype=np.float64).reshape(-1)
    lp, mp, nm1, _, _ = _pixels(plan)
    nz = np.nonzero(f)[0]
    lp, mp, nm1, f = lp[nz], mp[nz], nm1[nz], f[nz]
    out = np.empty(uvw.shape[0], dtype=np.complex128)
    for lo in range(0, uvw.shape[0], chunk):
        u = uvw[lo:lo + chunk]
        ph = u[:, 0:1] * lp[None, :] + u[:, 1:2] * mp[None, :] + u[:, 2:3] * nm1[None, :]
        out[lo:lo + chunk] = (np.exp(-2j * np.pi * ph) * f[None, :]).sum(1)
    return out
