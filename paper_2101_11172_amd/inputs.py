"""Seeded synthetic inputs for the improved W-stacking workloads.

This module draws inputs only: baseline coordinates, visibility values and sky
images.  It holds none of the gridding method's arithmetic and is the one piece
of code shared by the HIP path's tests/benchmark and the CPU oracle's tests.

Workloads (all seeded with ``numpy.random.default_rng``):

* ``tiny``   -- 256 x 256 image, L = 0.2; 5,000 visibilities with u, v uniform in
  +-600 wavelengths and w uniform in +-300; complex N(0, 1) values; a sky of 20
  point sources at distinct random pixels with fluxes log-uniform in [0.01, 1];
  W = 7, x0 = 0.25.
* ``widefield`` -- 2048 x 2048 image, L = 0.4; 64 antennas uniform by area in a
  disc of 5 km radius at latitude -30 deg, observing declination -30 deg for
  hour angles -1 h ... +1 h in T equally spaced dumps (T = 4,960 gives
  2,016 x 4,960 = 9,999,360 visibilities); uvw from the textbook equatorial
  transform at 1.4 GHz, then scaled so that max(|u|, |v|) = 0.95 N / (2 L),
  i.e. the image is Nyquist-sampled; complex N(0, 1) values (complex64 or
  complex128); W = 7, x0 = 0.25.
* ``lowcost`` -- the ``widefield`` geometry with W = 4, x0 = 0.5.
* ``widefield3`` -- the ``widefield`` geometry with x0 = 1/3 (N' = 3072, radix-3
  transforms; Sec. 6.3's cropping discussion).
* ``table2`` (``table2_workload``) -- stand-in for the Table 2 simulation: a
  512 x 512 image of a 6 degree field, 34 point sources, 27 antennas, 11
  two-minute snapshots from -5 h to +5 h, w scaled to the field's product
  (n_max - n_min) w_max = 7.44 of the printed layer counts.
* ``channels`` (``channels_workload``) -- the ``widefield`` array observed in
  32 channels at f_c = 1.0 + 0.8 c / 31 GHz: uvw of the 1.4 GHz tracks scaled
  by f_c / 1.4 GHz, then all channels by one factor so that the 1.8 GHz
  channel has max(|u|, |v|) = 0.95 N / (2 L) (N = 2048, L = 0.4); each channel
  flags a fraction U(0, 0.6) of its visibilities (Bernoulli per visibility),
  so the channels hold 4-10M visibilities each; complex N(0, 1) values.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299_792_458.0


def random_vis(M: int, seed: int, dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return v.astype(dtype)


def random_sky(N: int, n_src: int, seed: int, lo: float = 0.01, hi: float = 1.0) -> np.ndarray:
    """Real [N, N] image with n_src point sources at distinct random pixels."""
    rng = np.random.default_rng(seed)
    img = np.zeros((N, N), dtype=np.float64)
    pix = rng.choice(N * N, size=n_src, replace=False)
    flux = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_src))
    img.ravel()[pix] = flux
    return img


def random_image(N: int, seed: int) -> np.ndarray:
    """Dense real [N, N] image with N(0, 1) pixels (for adjoint identities)."""
    return np.random.default_rng(seed).standard_normal((N, N))


def uniform_uvw(M: int, umax: float, wmax: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    uvw = np.empty((M, 3))
    uvw[:, 0] = rng.uniform(-umax, umax, M)
    uvw[:, 1] = rng.uniform(-umax, umax, M)
    uvw[:, 2] = rng.uniform(-wmax, wmax, M)
    return uvw


def array_uvw(n_ant: int, radius_m: float, lat_deg: float, dec_deg: float,
              ha_hours: float, n_dumps: int, freq_hz: float, seed: int, ha_offset_h: float = 0.0) -> np.ndarray:
    """Earth-rotation uvw tracks in wavelengths, time-major order [dump][baseline].

    Antennas uniform by area in a disc (r = R sqrt(U), theta = 2 pi U), at height
    zero; baselines i < j; local (E, N, 0) -> equatorial (X, Y, Z) and the
    standard (H, delta) rotation to (u, v, w) (Thompson, Moran & Swenson, ch. 4).
    """
    rng = np.random.default_rng(seed)
    r = radius_m * np.sqrt(rng.uniform(size=n_ant))
    th = 2.0 * np.pi * rng.uniform(size=n_ant)
    E, Nn = r * np.cos(th), r * np.sin(th)
    ii, jj = np.triu_indices(n_ant, k=1)
    dE, dN = E[jj] - E[ii], Nn[jj] - Nn[ii]
    lat, dec = np.radians(lat_deg), np.radians(dec_deg)
    X, Y, Z = -dN * np.sin(lat), dE, dN * np.cos(lat)
    H = np.radians(15.0 * (ha_offset_h + np.linspace(-ha_hours, ha_hours, n_dumps)))[:, None]
    sH, cH = np.sin(H), np.cos(H)
    sd, cd = np.sin(dec), np.cos(dec)
    lam = C_LIGHT / freq_hz
    uvw = np.empty((n_dumps, ii.size, 3))
    uvw[..., 0] = (sH * X + cH * Y) / lam
    uvw[..., 1] = (-sd * cH * X + sd * sH * Y + cd * Z) / lam
    uvw[..., 2] = (cd * cH * X - cd * sH * Y + sd * Z) / lam
    return uvw.reshape(-1, 3)


def snapshots_uvw(n_ant: int, radius_m: float, lat_deg: float, dec_deg: float, ha_centres_h,
                  snapshot_s: float, n_per_snapshot: int, freq_hz: float, seed: int) -> np.ndarray:
    """Snapshot tracks: for each hour angle centre, n_per_snapshot dumps over
    snapshot_s seconds (the same antennas and transform as array_uvw)."""
    out = []
    for hc in ha_centres_h:
        one = array_uvw(n_ant, radius_m, lat_deg, dec_deg, snapshot_s / 7200.0, n_per_snapshot, freq_hz, seed,
                        ha_offset_h=float(hc))
        out.append(one)
    return np.concatenate(out)


def table2_workload(N: int = 512, seed: int = 21) -> dict:
    """Synthetic stand-in for the paper's Table 2 simulation (a 6 degree field
    observed on a 27-antenna array at 74 MHz, 2 minutes every hour from -5 h to
    +5 h, 34 point sources): 27 antennas uniform in a 5.7 km-radius disc at
    latitude 34 deg, declination 30 deg, 11 snapshots of 12 dumps; u, v scaled
    so the N x N image of L = 2 sin(3 deg) is Nyquist-sampled, and w scaled so
    that (n_max - n_min) w_max = 7.44, the product that reproduces Table 2's
    printed layer counts; complex visibilities are not drawn here (the test
    forms them from the sky)."""
    L = 2.0 * np.sin(np.radians(3.0))
    uvw = snapshots_uvw(27, 5700.0, 34.0, 30.0, np.arange(-5, 6), 120.0, 12, 74e6, seed)
    uvw = uvw.copy()
    uv_scale = 0.95 * N / (2.0 * L) / np.max(np.abs(uvw[:, :2]))
    uvw[:, :2] *= uv_scale
    dn = 1.0 - np.sqrt(1.0 - 2.0 * (L / 2) ** 2)
    uvw[:, 2] *= (7.44 / dn) / np.max(np.abs(uvw[:, 2]))
    return dict(name="table2", N=N, L=L, uvw=uvw, wmax=float(np.max(np.abs(uvw[:, 2]))),
                sky=random_sky(N, 34, seed + 1))


def scale_to_image(uvw: np.ndarray, N: int, L: float, fill: float = 0.95) -> np.ndarray:
    """Scale all of uvw so that max(|u|, |v|) = fill * N / (2 L) (Nyquist-sampled image)."""
    umax = np.max(np.abs(uvw[:, :2]))
    return uvw * (fill * N / (2.0 * L) / umax)


def channels_workload(n_channels: int = 32, n_dumps: int = 4960, seed: int = 3, vis_dtype=np.complex64) -> dict:
    """Batched-channel workload (see module docstring): concatenated uvw and
    values in channel order, with the per-channel counts."""
    rng = np.random.default_rng(seed)
    N, L = 2048, 0.4
    base = array_uvw(64, 5000.0, -30.0, -30.0, 1.0, n_dumps, 1.4e9, 1)
    freqs = 1.0e9 + 0.8e9 * np.arange(n_channels) / max(1, n_channels - 1)
    top = np.max(np.abs(base[:, :2])) * freqs[-1] / 1.4e9
    scale = 0.95 * N / (2.0 * L) / top
    uvws, counts = [], []
    for f in freqs:
        keep = rng.uniform(size=base.shape[0]) >= rng.uniform(0.0, 0.6)
        uvws.append(base[keep] * (scale * f / 1.4e9))
        counts.append(int(np.count_nonzero(keep)))
    uvw = np.concatenate(uvws)
    wmax = float(np.max(np.abs(uvw[:, 2])))
    return dict(name="channels", N=N, L=L, W=7, x0=0.25, wmax=wmax, uvw=uvw, counts=counts, freqs=freqs,
                vis=random_vis(uvw.shape[0], seed + 100, vis_dtype))


def channel_image_sizes(freqs, n_top: int = 2048, sizes=(1024, 1536, 2048)) -> list:
    """Image size per channel for the batched-channel workload: the smallest
    2^a or 3 2^a size in [1024, 2048] that Nyquist-samples the channel's uv
    extent, which scales with frequency (the top channel needs n_top)."""
    top = max(freqs)
    return [next(n for n in sizes if n >= n_top * f / top - 1e-9) for f in freqs]


def workload(name: str, seed: int | None = None, n_dumps: int = 4960,
             vis_dtype=np.complex64) -> dict:
    """Parameters and inputs of a named workload (see module docstring)."""
    if name == "tiny":
        seed = 0 if seed is None else seed
        uvw = uniform_uvw(5000, 600.0, 300.0, seed)
        return dict(name=name, N=256, L=0.2, W=7, x0=0.25, wmax=300.0, uvw=uvw,
                    vis=random_vis(5000, seed + 100, np.complex128),
                    sky=random_sky(256, 20, seed + 200))
    if name in ("widefield", "lowcost", "widefield3"):
        seed = 1 if seed is None else seed
        N, L = 2048, 0.4
        uvw = array_uvw(64, 5000.0, -30.0, -30.0, 1.0, n_dumps, 1.4e9, seed)
        uvw = scale_to_image(uvw, N, L)
        W, x0 = {"widefield": (7, 0.25), "lowcost": (4, 0.5), "widefield3": (7, 1 / 3)}[name]
        return dict(name=name, N=N, L=L, W=W, x0=x0, wmax=float(np.max(np.abs(uvw[:, 2]))),
                    uvw=uvw, vis=random_vis(uvw.shape[0], seed + 100, vis_dtype),
                    sky=None)
    raise ValueError(f"unknown workload {name!r}")
