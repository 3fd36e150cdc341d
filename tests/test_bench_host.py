"""Host logic of bench.py (CPU): the occupancy, tile-visit and live-line counts
that fix the algorithmic bytes, against brute force over every support cell of
every visibility (a tile is occupied when a support cell of some visibility
lies in it; a visibility visits each tile its W^3 cells meet; a stack line
(t, r) is live when its row of tiles holds an occupied tile)."""
import numpy as np
import pytest

import bench
from oracle.plan import make_plan
from paper_2101_11172_amd import inputs


def brute_force(uvw, p, W):
    umul = (p.L / 2) / p.x0
    Np, nl, T = p.Nprime, p.n_layers, 16
    occ, visits = set(), 0
    for u, v, w in uvw:
        if w < 0:
            u, v, w = -u, -v, -w
        fu = int(np.floor(umul * u + W / 2)) - W + 1
        fv = int(np.floor(umul * v + W / 2)) - W + 1
        ft = int(np.floor(p.n_scale * w + W / 2)) - W + 1 - p.t_lo
        tiles = {((ft + a) // T, ((fv + b) % Np) // T, ((fu + c) % Np) // T)
                 for a in range(W) for b in range(W) for c in range(W)}
        visits += len(tiles)
        occ |= tiles
    rows = {(t, r) for (t, _, r) in occ}
    lines = sum(min(T, nl - T * t) * T for (t, _) in rows)
    return len(occ), visits, lines


@pytest.mark.parametrize("N,L,wmax,M", [(64, 0.3, 100.0, 300), (128, 0.8, 300.0, 400)])
def test_workload_stats_match_brute_force(N, L, wmax, M):
    W, x0 = 7, 0.25
    p = make_plan(N, L, W, x0, wmax)
    uvw = inputs.uniform_uvw(M, 0.9 * N / (2 * L), wmax, 7)
    ws = bench.workload_stats(uvw, N, L, W, x0, wmax, p.Nprime, p.n_layers, p.t_lo, p.n_scale)
    tiles, visits, lines = brute_force(uvw, p, W)
    assert ws["tiles_occupied"] == tiles
    assert ws["tile_visits"] == visits
    assert ws["nonempty_lines"] == lines
