"""Planner for improved W-stacking (oracle, FP64).

Test infrastructure: see ``oracle/__init__.py``.

* Pixel grid (Sec. 3.3 Algorithm 1 box, Sec. 5.1): N x N pixels of size
  dl = L / N; pixel i has l_i = (i - N/2) dl (same for m), l_max = L / 2.
* Normalised map coordinate x = x0 l / l_max (Sec. 5.1), which gives
  x_i = (i - N/2) / N' with FFT length N' = N / (2 x0) (Algorithm 1: N = 2 x0 N').
* z = (n - n0) / n_scale on the sphere (eq. z-on-sphere), with
  n_scale = (1 - n_min) / (2 z0) and n0 = 1 - z0 n_scale (eq. n_params),
  n_min = sqrt(1 - l_max^2 - m_max^2), and z0 = x0 by default (Sec. 6.2
  recommendation; Sec. 5.2 allows a z-axis gridding function of its own width
  W_z and cropping z0, eq. gridded_vis with C_z, and Sec. 6.1 trades W_z
  against z0).
  Then z runs from -z0 (map corners) to +z0 (centre).  The variant without z
  offset (Sec. 5.3, eq. n_params_no_offset) takes n_scale = (1 - n_min) / z0
  and n0 = 1, so that z runs from -z0 to 0 and z = 0 at the map centre, at
  about twice the number of layers.  In both, z = (n - 1) / n_scale + z_shift
  with z_shift = (1 - n0) / n_scale (z0, or 0 without offset).
* w-layers at w[t] = t / n_scale (Algorithm 5 step 1).  After the Hermitian fold
  (Sec. 5.4) w >= 0, so w' = n_scale w lies in [0, n_scale w_max].  With the
  support convention of ``wstack.support`` a visibility at w' touches layers
  floor(w' + W/2) - W + 1 ... floor(w' + W/2); the planner allocates exactly the
  layers that can be touched, t_lo = floor(W/2) - W + 1 ... t_hi =
  floor(n_scale w_max + W/2).
* ``layers_required`` is the count of eq. (N_{w'}+W): the smallest integer
  strictly above (n_max - n_min)(w_max - w_min) / (2 z0) + W; ``layers_no_offset``
  is the variant without z offset (Sec. 5.3), and ``layers_original`` is the
  bin count of eq. N_w for the original method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Plan:
    N: int
    L: float
    W: int
    x0: float
    wmax: float
    Nprime: int
    l_max: float
    n_min: float
    n_scale: float
    n0: float
    t_lo: int
    t_hi: int
    z_offset: bool = True
    Wz: int = 0            # width of C_z (0: the same as W)
    z0v: float = 0.0       # z cropping z0 (0: the same as x0)

    @property
    def n_layers(self) -> int:
        return self.t_hi - self.t_lo + 1

    @property
    def W_z(self) -> int:
        return self.Wz or self.W

    @property
    def z0(self) -> float:
        return self.z0v or self.x0

    @property
    def z_shift(self) -> float:
        """(1 - n0) / n_scale: z0 with the z offset, 0 without."""
        return self.z0 if self.z_offset else 0.0

    def pixel_lm(self):
        """Direction cosines of pixel columns (l) / rows (m): (i - N/2) L / N."""
        i = np.arange(self.N, dtype=np.float64) - self.N // 2
        return i * (self.L / self.N)

    def pixel_x(self):
        """Normalised coordinate x_i = (i - N/2) / N' of each pixel column (or row)."""
        return (np.arange(self.N, dtype=np.float64) - self.N // 2) / self.Nprime

    def n_minus_1(self):
        """n - 1 on the [m, l] pixel grid, as -(l^2 + m^2) / (1 + n) (no cancellation)."""
        l = self.pixel_lm()
        r2 = l[None, :] ** 2 + l[:, None] ** 2
        n = np.sqrt(1.0 - r2)
        return -r2 / (1.0 + n)

    def z(self):
        """z = (n - n0) / n_scale on the [m, l] pixel grid (eq. z-on-sphere)."""
        # n - n0 = (n - 1) + (1 - n0) = (n - 1) + z_shift n_scale
        return self.n_minus_1() / self.n_scale + self.z_shift


def make_plan(N: int, L: float, W: int, x0: float, wmax: float, z_offset: bool = True,
              Wz: int | None = None, z0: float | None = None) -> Plan:
    """Plan of the improved method; Wz, z0 default to W, x0 (the same gridding
    function on all three axes)."""
    if N <= 0 or N % 2:
        raise ValueError("N must be positive and even")
    if not (0.0 < x0 <= 0.5):
        raise ValueError("x0 must be in (0, 1/2]")
    Np = N / (2.0 * x0)
    if abs(Np - round(Np)) > 1e-9:
        raise ValueError("N / (2 x0) must be an integer")
    Wz = W if Wz is None else int(Wz)
    z0 = x0 if z0 is None else float(z0)
    if not (1 <= W <= 16) or not (1 <= Wz <= 16):
        raise ValueError("W and W_z must be in [1, 16]")
    if not (0.0 < z0 <= 0.5):
        raise ValueError("z0 must be in (0, 1/2]")
    if not (0.0 < L < math.sqrt(2.0)):
        raise ValueError("L must be in (0, sqrt 2)")
    if not (wmax >= 0.0):
        raise ValueError("wmax must be >= 0")
    l_max = 0.5 * L
    n_min = math.sqrt(1.0 - 2.0 * l_max * l_max)
    if z_offset:
        n_scale = (1.0 - n_min) / (2.0 * z0)      # eq. n_params
        n0 = 1.0 - z0 * n_scale
    else:
        n_scale = (1.0 - n_min) / z0              # eq. n_params_no_offset
        n0 = 1.0
    t_lo = Wz // 2 - Wz + 1
    t_hi = int(math.floor(n_scale * wmax + 0.5 * Wz))
    return Plan(N=N, L=L, W=W, x0=x0, wmax=wmax, Nprime=int(round(Np)), l_max=l_max,
                n_min=n_min, n_scale=n_scale, n0=n0, t_lo=t_lo, t_hi=t_hi, z_offset=z_offset,
                Wz=Wz, z0v=z0)


def layers_required(dn_dw: float, z0: float, W: int) -> int:
    """Smallest integer N_w' > (n_max - n_min)(w_max - w_min)/(2 z0) + W_z  (eq. N_{w'}+W)."""
    return int(math.floor(dn_dw / (2.0 * z0) + W)) + 1


def layers_no_offset(dn_dw: float, z0: float, W: int) -> int:
    """Smallest integer N_w'' > (n_max - n_min)(w_max - w_min)/z0 + W_z (Sec. 5.3, no z offset)."""
    return int(math.floor(dn_dw / z0 + W)) + 1


def layers_original(dn_dw: float) -> int:
    """Smallest integer N_w >= 2 pi (n_max - n_min)(w_max - w_min)  (eq. N_w)."""
    return int(math.ceil(2.0 * math.pi * dn_dw))
