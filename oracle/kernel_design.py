"""Least-misfit gridding function C and gridding correction h  (oracle, FP64).

Test infrastructure: see ``oracle/__init__.py``.

What the paper fixes (Sec. 3.3, Algorithm 1 box):

* the map-error residual (eq. csum2)
      L(x, nu) = 1 - h(x) * sum_s C(s - nu) * exp(i 2 pi (s - nu) x),
  with s running over -(W-1)/2 ... (W-1)/2 in unit steps and nu in [-1/2, 1/2);
* the error bound (eq. norm_bound)
      E^2 = 1/(2 x0) * int_{-x0}^{x0} int_{-1/2}^{1/2} |L(x, nu)|^2 dnu dx,
  and the map error function l(x) = int |L(x, nu)|^2 dnu;
* the least-misfit pair (C, h): C even, support of width W, chosen with h to
  minimise E for the given W and image cropping parameter x0.

The paper defers the construction to the authors' earlier work, so this module
minimises E directly (the reading is listed in the design doc):

* write c_s(nu) = C(s - nu).  For fixed h, the best c(nu) at each nu solves the
  W x W normal equations  A c(nu) = b(nu)  with
      A_{ss'} = int_0^{x0} h^2 cos(2 pi (s - s') x) dx,
      b_s(nu) = int_0^{x0} h   cos(2 pi (s - nu) x) dx
  (the x-integrands are even, so [0, x0] suffices);
* for fixed C the best h is pointwise
      h(x) = int Re g(x, nu) dnu / int |g(x, nu)|^2 dnu,
      g(x, nu) = sum_s c_s(nu) exp(i 2 pi (s - nu) x);
* variable projection: c is eliminated through the normal equations and damped
  Gauss-Newton runs on h at Gauss-Legendre nodes in x, with the residuals L at
  the (x, nu) node pairs weighted by the quadrature weights.  The start is a
  Kaiser-Bessel kernel whose shape parameter is scanned for the lowest E.
* only the product h*C enters L, so the scale is fixed by h(0) = 1.

The product h(x) g(x, nu) -- the only thing the gridding operators apply -- is
determined to ~1e-13 even though the split between h and C is not (the optimum
is flat along h -> h(1+eps), C -> C(1-eps)).
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(n: int, a: float, b: float):
    """n-point Gauss-Legendre nodes and weights on [a, b]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * t + 0.5 * (b + a), 0.5 * (b - a) * w


def offsets(W: int) -> np.ndarray:
    """The W offsets s = -(W-1)/2, ..., (W-1)/2 of eq. csum2."""
    return np.arange(W, dtype=np.float64) - 0.5 * (W - 1)


def error_bound(c_of_nu, h_of_x, W: int, x0: float, n_x: int = 200, n_nu: int = 200) -> float:
    """E of eq. norm_bound for arbitrary callables, by Gauss-Legendre quadrature.

    ``c_of_nu(nu)`` returns the [len(nu), W] array c_s(nu) = C(s - nu);
    ``h_of_x(x)`` returns h at the points x.  L is formed as a complex
    difference and squared, never as 1 - 2 h Re g + h^2 |g|^2, which cancels
    catastrophically when E^2 ~ 1e-14.
    """
    x, wx = gauss_legendre(n_x, 0.0, x0)
    nu, wn = gauss_legendre(n_nu, -0.5, 0.5)
    s = offsets(W)
    c = np.asarray(c_of_nu(nu), dtype=np.float64).reshape(n_nu, W)
    h = np.asarray(h_of_x(x), dtype=np.float64)
    ph = np.exp(2j * np.pi * (s[None, :, None] - nu[:, None, None]) * x[None, None, :])
    g = np.einsum("js,jsi->ji", c, ph)
    L = 1.0 - h[None, :] * g
    # (1/(2 x0)) * 2 * int_0^{x0}: the integrand is even in x
    return float(np.sqrt(np.sum(wn[:, None] * np.abs(L) ** 2 * wx[None, :]) / x0))


def map_error(c_of_nu, h_of_x, W: int, x, n_nu: int = 200) -> np.ndarray:
    """l(x) = int |L(x, nu)|^2 dnu at the points x (Sec. 3.3)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nu, wn = gauss_legendre(n_nu, -0.5, 0.5)
    s = offsets(W)
    c = np.asarray(c_of_nu(nu), dtype=np.float64).reshape(n_nu, W)
    ph = np.exp(2j * np.pi * (s[None, :, None] - nu[:, None, None]) * x[None, None, :])
    g = np.einsum("js,jsi->ji", c, ph)
    L = 1.0 - np.asarray(h_of_x(x))[None, :] * g
    return np.sum(wn[:, None] * np.abs(L) ** 2, axis=0)


class LeastMisfit:
    """Least-misfit (C, h) for width W and cropping parameter x0."""

    def __init__(self, W: int, x0: float, n_x: int = 32, n_nu: int = 32,
                 max_iter: int = 200):
        if not (1 <= W <= 16):
            raise ValueError("W must be in [1, 16]")
        if not (0.0 < x0 <= 0.5):
            raise ValueError("x0 must be in (0, 1/2]")
        self.W, self.x0 = int(W), float(x0)
        self.s = offsets(self.W)
        self.xn, self.wx = gauss_legendre(n_x, 0.0, self.x0)
        self.nun, self.wn = gauss_legendre(n_nu, -0.5, 0.5)
        ang = 2.0 * np.pi * (self.s[None, :, None] - self.nun[:, None, None]) * self.xn[None, None, :]
        self._cos, self._sin = np.cos(ang), np.sin(ang)                          # [n_nu, W, n_x]
        self._K = np.cos(2.0 * np.pi * (self.s[:, None] - self.s[None, :])[:, :, None]
                         * self.xn[None, None, :])                               # [W, W, n_x]
        self._sw = np.sqrt(self.wn[:, None] * self.wx[None, :] / self.x0)       # residual weights
        self.iterations = 0
        self.h_nodes = self._solve(max_iter)
        self.A = self._normal_matrix(self.h_nodes)
        self._c_nodes = self.c(self.nun)
        # scale convention h(0) = 1 (c scales inversely, the product h*C is unchanged)
        self.h_nodes = self.h_nodes / self.h([0.0])[0]
        self.A = self._normal_matrix(self.h_nodes)
        self._c_nodes = self.c(self.nun)
        self.E = error_bound(self.c, self.h, self.W, self.x0)

    # -- the two half-steps ------------------------------------------------
    def _normal_matrix(self, h):
        return np.einsum("sti,i->st", self._K, h * h * self.wx)

    def _rhs(self, h, nu):
        nu = np.atleast_1d(np.asarray(nu, dtype=np.float64))
        k = np.cos(2.0 * np.pi * (self.s[None, :, None] - nu[:, None, None]) * self.xn[None, None, :])
        return np.einsum("jsi,i->js", k, h * self.wx)

    def _residuals(self, h):
        """L at the (nu, x) nodes with c eliminated; analytic in h (complex-step safe)."""
        A = np.einsum("sti,i->st", self._K, h * h * self.wx)
        b = np.einsum("jsi,i->js", self._cos, h * self.wx)
        c = np.linalg.solve(A, b.T).T                                             # [n_nu, W]
        gr = np.einsum("js,jsi->ji", c, self._cos)
        gi = np.einsum("js,jsi->ji", c, self._sin)
        return np.concatenate([((1.0 - h * gr) * self._sw).ravel(),
                               ((-h * gi) * self._sw).ravel()])

    def _kaiser_bessel_start(self):
        best = None
        for beta in np.linspace(0.5, 3.5 * self.W, 400):
            t = 1.0 - (2.0 * (self.s[None, :] - self.nun[:, None]) / self.W) ** 2
            c = np.i0(beta * np.sqrt(np.clip(t, 0.0, None)))
            gr = np.einsum("js,jsi->ji", c, self._cos)
            gi = np.einsum("js,jsi->ji", c, self._sin)
            h = (self.wn[:, None] * gr).sum(0) / (self.wn[:, None] * (gr ** 2 + gi ** 2)).sum(0)
            h = h / h[0]
            r = self._residuals(h)
            f = float(r @ r)
            if best is None or f < best[0]:
                best = (f, h)
        return best[1]

    def _solve(self, max_iter):
        h = self._kaiser_bessel_start()
        n = h.size
        r = self._residuals(h)
        f = float(r @ r)
        lam = 1e-6
        for it in range(max_iter):
            J = np.empty((r.size, n - 1))
            for i in range(1, n):                       # h[0] = 1 is held fixed
                hc = h.astype(np.complex128)
                hc[i] += 1e-40j
                J[:, i - 1] = self._residuals(hc).imag / 1e-40
            scale = np.linalg.norm(J, axis=0)
            Js = J / scale
            accepted = False
            for _ in range(80):
                M = np.vstack([Js, np.sqrt(lam) * np.eye(n - 1)])
                rhs = np.concatenate([-r, np.zeros(n - 1)])
                d = np.linalg.lstsq(M, rhs, rcond=None)[0] / scale
                h_try = h.copy()
                h_try[1:] += d
                r_try = self._residuals(h_try)
                f_try = float(r_try @ r_try)
                if f_try < f:
                    h, r, f = h_try, r_try, f_try
                    lam = max(lam / 10.0, 1e-24)
                    accepted = True
                    break
                lam *= 4.0
            self.iterations = it + 1
            if not accepted or np.max(np.abs(d)) <= 1e-15 * np.max(np.abs(h)):
                break
        return h

    # -- the converged functions -------------------------------------------
    def c(self, nu) -> np.ndarray:
        """c_s(nu) = C(s - nu) for each nu: array [len(nu), W] (normal equations)."""
        b = self._rhs(self.h_nodes, nu)
        return np.linalg.solve(self.A, b.T).T

    def h(self, x) -> np.ndarray:
        """h(x) by the pointwise optimality formula (even in x)."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        out = np.empty_like(x)
        for lo in range(0, x.size, 8192):
            xs = x[lo:lo + 8192]
            ph = np.exp(2j * np.pi * (self.s[None, :, None] - self.nun[:, None, None]) * xs[None, None, :])
            g = np.einsum("js,jsi->ji", self._c_nodes, ph)
            out[lo:lo + 8192] = ((self.wn[:, None] * g.real).sum(0)
                                 / (self.wn[:, None] * np.abs(g) ** 2).sum(0))
        return out

    def kernel(self, u) -> np.ndarray:
        """C(u) at arbitrary u; zero outside [-W/2, W/2)."""
        u = np.atleast_1d(np.asarray(u, dtype=np.float64))
        out = np.zeros_like(u)
        for a, s in enumerate(self.s):
            nu = s - u
            m = (nu >= -0.5) & (nu < 0.5)
            if np.any(m):
                out[m] = self.c(nu[m])[:, a]
        return out

    def hg(self, x, nu) -> np.ndarray:
        """h(x) g(x, nu) on the grid x (columns) by nu (rows): what the operators apply."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        nu = np.atleast_1d(np.asarray(nu, dtype=np.float64))
        ph = np.exp(2j * np.pi * (self.s[None, :, None] - nu[:, None, None]) * x[None, None, :])
        return self.h(x)[None, :] * np.einsum("js,jsi->ji", self.c(nu), ph)


_CACHE: dict = {}


def least_misfit(W: int, x0: float) -> LeastMisfit:
    """Cached LeastMisfit(W, x0)."""
    key = (int(W), float(x0))
    if key not in _CACHE:
        _CACHE[key] = LeastMisfit(W, x0)
    return _CACHE[key]
