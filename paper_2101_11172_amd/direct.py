"""Direct Fourier transform pair at sampled outputs, with plain torch float64
operations on the device.

A measurement aid, not part of the operators: bench.py and the full-size tests
use it to state the error of a gridding or degridding run against the exact
result the method approximates (Sec. 2, eq. fourier_visibility; the dirty map
of Sec. 5.2 without the 1/M weights):

    V_k  = sum_ji f_ji exp[-i 2 pi (u_k l_i + v_k m_j + w_k (n_ji - 1))]
    D_ji = Re sum_k V_k exp[+i 2 pi (u_k l_i + v_k m_j + w_k (n_ji - 1))]

with l_i = (i - N/2) L/N, m_j = (j - N/2) L/N and n - 1 = -(l^2 + m^2)/(1 + n).
The phase is reduced to [-1/2, 1/2] turns before the float64 sine and cosine.
The tests pin these values to the CPU oracle's transform at a few outputs.
"""
from __future__ import annotations

import math

import torch


def _lmn(idx_rows, idx_cols, N: int, L: float, device):
    dl = L / N
    l = (torch.as_tensor(idx_cols, dtype=torch.float64, device=device) - N // 2) * dl
    m = (torch.as_tensor(idx_rows, dtype=torch.float64, device=device) - N // 2) * dl
    r2 = l * l + m * m
    return l, m, -r2 / (1.0 + torch.sqrt(1.0 - r2))


def dft_grid(uvw: torch.Tensor, vis: torch.Tensor, N: int, L: float, rows, cols, chunk: int = 16,
             progress: bool = False) -> torch.Tensor:
    """D_ji at the pixels (rows[p], cols[p]); float64 [len(rows)] on uvw's device.

    Phases are laid out [pixel][visibility] so that each sum runs along
    contiguous memory."""
    u, v, w = (uvw[:, i].contiguous() for i in range(3))
    vr, vi = vis.real.double().contiguous(), vis.imag.double().contiguous()
    out = []
    for lo in range(0, len(rows), chunk):
        l, m, nm1 = _lmn(rows[lo:lo + chunk], cols[lo:lo + chunk], N, L, uvw.device)
        ph = l[:, None] * u[None, :] + m[:, None] * v[None, :] + nm1[:, None] * w[None, :]
        ph = 2.0 * math.pi * (ph - torch.round(ph))
        out.append(torch.sum(torch.cos(ph) * vr[None, :] - torch.sin(ph) * vi[None, :], dim=1))
        if progress and (lo // chunk) % 125 == 124:
            torch.cuda.synchronize()
            print(f"  direct transform: {lo + chunk} of {len(rows)} pixels", flush=True)
    return torch.cat(out)


def dft_degrid(uvw: torch.Tensor, image: torch.Tensor, N: int, L: float, chunk: int = 4096) -> torch.Tensor:
    """V_k for every row of uvw from the nonzero pixels of the real image;
    complex128 [len(uvw)] on uvw's device."""
    f = image.double().reshape(-1)
    nz = torch.nonzero(f).reshape(-1)
    rows, cols = nz // N, nz % N
    l, m, nm1 = _lmn(rows, cols, N, L, uvw.device)
    fv = f[nz]
    out = []
    for lo in range(0, uvw.shape[0], chunk):
        q = uvw[lo:lo + chunk]
        ph = q[:, 0:1] * l[None, :] + q[:, 1:2] * m[None, :] + q[:, 2:3] * nm1[None, :]
        ph = 2.0 * math.pi * (ph - torch.round(ph))
        out.append(torch.complex(torch.sum(torch.cos(ph) * fv[None, :], dim=1),
                                 -torch.sum(torch.sin(ph) * fv[None, :], dim=1)))
    return torch.cat(out)
