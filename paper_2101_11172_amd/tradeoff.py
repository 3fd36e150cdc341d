"""Accuracy against layer count for the w-direction kernel (Sec. 6.1).

For a w-kernel of width W_z, the least-misfit design error E grows with the
cropping parameter z0, and the number of w-layers grows as 1 / (2 z0) (the
first term of eq. N_{w'}+W).  ``layer_factor(W, E)`` is the 1 / (2 z0) at which
the library's own least-misfit design (``wsg_design_eval``, host only) reaches
error E, found by bisection in log z0; ``tradeoff_table`` gives it for several
widths and accuracies (the data of the paper's accuracy trade-off figure).
"""
from __future__ import annotations

import math

import numpy as np

from . import wsgrid as wg


def design_error(W: int, z0: float) -> float:
    """E of the least-misfit design for width W and cropping parameter z0."""
    _, _, e = wg.wsg_design_eval(W, z0, np.zeros(0), np.zeros(0))
    return e


def z0_for_error(W: int, E: float, lo: float = 1e-6, hi: float = 0.5, rel_tol: float = 1e-6) -> float:
    """Largest z0 in [lo, hi] whose design error is at most E (E increases with z0)."""
    if design_error(W, lo) > E:
        raise ValueError(f"W = {W} cannot reach E = {E} above z0 = {lo}")
    if design_error(W, hi) <= E:
        return hi
    while hi / lo > 1.0 + rel_tol:
        mid = math.sqrt(lo * hi)
        if design_error(W, mid) > E:
            hi = mid
        else:
            lo = mid
    return lo


def layer_factor(W: int, E: float) -> float:
    """1 / (2 z0) at error E: w-layers per unit of (n_max - n_min)(w_max - w_min)."""
    return 1.0 / (2.0 * z0_for_error(W, E))


def tradeoff_table(widths=(1, 2, 3, 4, 5, 6, 7), errors=(1e-3, 1e-5, 1e-7)) -> dict:
    """{(W, E): 1 / (2 z0)}, None where W cannot reach E."""
    out = {}
    for W in widths:
        for E in errors:
            try:
                out[(W, E)] = layer_factor(W, E)
            except ValueError:
                out[(W, E)] = None
    return out
