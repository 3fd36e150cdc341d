"""Host logic of bench.py (CPU): the occupancy, tile-visit and live-line counts
that fix the algorithmic bytes, against brute force over every support cell of
every visibility (a tile is occupied when a support cell of some visibility
lies in it; a visibility visits each tile its W^3 cells meet; a stack line
(t, r) is live when its row of tiles holds an occupied tile)."""
import json

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


def test_counters_hold_for_their_workload_only(tmp_path, monkeypatch):
    # a counter summary is used only on the sources and the workload it was taken on
    (tmp_path / "profiles").mkdir()
    key = bench.workload_key("widefield", 2048, 7, 0.25, 9999360, 49, 32)
    t = {"source_digest": bench.source_digest(), "workload": key,
         "per_launch_bytes": {"grid_tiles:f32": 2.0e9}, "valu_per_launch": {"grid_tiles:f32": 1024 * 2.4e6}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(t))
    digest = bench.source_digest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: digest)
    assert bench.traffic_for("grid_tiles", "f32", key) == 2.0e9
    assert abs(bench.issue_for("grid_tiles", "f32", key)["valu_issue_ms"] - 4.0) < 1e-12
    other = bench.workload_key("widefield3", 2048, 7, 1 / 3, 9999360, 39, 32)
    assert bench.traffic_for("grid_tiles", "f32", other) is None and bench.issue_for("grid_tiles", "f32", other) is None
    t["source_digest"] = "0" * 16
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(t))
    assert bench.traffic_for("grid_tiles", "f32", key) is None


def test_more_than_one_gpu_is_refused():
    # one GPU is measured; a request for more exits with a message, before any device work
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
