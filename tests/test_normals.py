"""Surface normals of the map (Table I, "normal calculation"): the GPU
kernel against the oracle on the same seeded heights, written into both maps
as binary32 values.

Tolerance: |dn| <= 1e-5 per component.  The normal is a unit vector; the
GPU computes the central-difference gradient, the norm and the quotients in
binary32 (one rounding per operation, about 8 roundings on the longest
chain, i.e. below 1e-6), the oracle in binary64 from the same binary32
heights.  Validity (NaN) must agree exactly.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from paper_2309_16818_amd import mem, synth

N_TOL = 1e-5

pytestmark = pytest.mark.gpu


def terrain_heights(rng, W, H, res, ox, oy, hole_frac=0.05):
    """Binary32 heights of a seeded terrain at the cell centres of the grid
    whose logical cell (0, 0) is lattice cell (ox, oy), with holes."""
    # boxes are placed away from the origin: give small grids a terrain of
    # a few metres all the same
    ter = synth.make_terrain(rng, extent=max(max(W, H) * res, 8.0))
    xs = (ox + np.arange(W) + 0.5) * res
    ys = (oy + np.arange(H) + 0.5) * res
    X, Y = np.meshgrid(xs, ys)
    h = ter.height(X, Y)
    h[rng.uniform(size=h.shape) < hole_frac] = np.nan
    return h.astype(np.float32)


def pair_with_heights(W, H, res, moves, rng, hole_frac=0.05):
    g = mem.Map(mem.MapParams(W, H, res))
    o = O.OracleMap(W, H, res)
    for mx, my in moves:
        g.move(mx, my)
        o.move(mx, my)
    cx, cy = g.center()
    assert (cx, cy) == o.center()
    h = terrain_heights(rng, W, H, float(np.float32(res)), cx - W // 2, cy - H // 2, hole_frac)
    g.set_layer(mem.MEM_LAYER_ELEVATION, 0, torch.from_numpy(h))
    o.set_layer(O.LAYER_ELEVATION, 0, h.astype(np.float64))
    return g, o


def check_normals(g, o):
    a = g.normals()
    torch.cuda.synchronize()
    a = a.double().cpu().numpy()
    b = o.normals()
    assert a.shape == b.shape == (g.H, g.W, 3)
    assert np.array_equal(np.isnan(a), np.isnan(b)), np.argwhere(np.isnan(a) != np.isnan(b))[:5]
    ok = ~np.isnan(b)
    err = np.abs(a[ok] - b[ok]).max(initial=0.0)
    assert err <= N_TOL, err
    return int(ok.all(axis=2).sum())


@pytest.mark.parametrize("W,H,res,moves", [
    (61, 47, 0.05, [(0.4, -0.3)]),                       # ragged in both tile directions
    (130, 9, 0.04, [(1.0, 0.2), (-0.37, 0.11)]),         # three tile columns, ring offsets
    (200, 200, 0.04, [(3.1, -2.7)]),                     # small workload's grid
    (500, 500, 0.04, [(7.3, 5.9), (-0.2, 0.4)]),         # full workload's grid
])
def test_normals_match_oracle(W, H, res, moves):
    rng = np.random.default_rng(W * 1000 + H)
    g, o = pair_with_heights(W, H, res, moves, rng)
    n_ok = check_normals(g, o)
    # holes of 5% leave most interior normals defined
    assert n_ok > 0.5 * (W - 2) * (H - 2)


@pytest.mark.parametrize("W,H", [(1, 1), (2, 2), (1, 7), (7, 1), (3, 3), (2, 64), (65, 3)])
def test_normals_on_degenerate_grids(W, H):
    """Grids without interior cells give only NaN; a 3 x k grid has one
    interior row."""
    rng = np.random.default_rng(W + 31 * H)
    g, o = pair_with_heights(W, H, 0.1, [(0.25, -0.35)], rng, hole_frac=0.0)
    n_ok = check_normals(g, o)
    assert n_ok == max(W - 2, 0) * max(H - 2, 0)


def test_normals_of_an_empty_map_are_nan():
    g = mem.Map(mem.MapParams(37, 29, 0.05))
    n = g.normals()
    torch.cuda.synchronize()
    assert torch.isnan(n).all()


def test_normals_reject_a_wrong_output():
    g = mem.Map(mem.MapParams(8, 8, 0.05))
    with pytest.raises(ValueError):
        g.normals(out=torch.empty((8, 8, 2), dtype=torch.float32, device="cuda"))


def test_normals_into_an_unaligned_output():
    """An output that starts 4 bytes into an allocation gives the same
    normals as an aligned one."""
    rng = np.random.default_rng(7)
    g, o = pair_with_heights(128, 36, 0.05, [(0.3, 0.2)], rng)
    a = g.normals()
    buf = torch.empty(128 * 36 * 3 + 1, dtype=torch.float32, device="cuda")
    b = g.normals(out=buf[1:].view(36, 128, 3))
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))
    check_normals(g, o)


def test_normals_on_a_large_grid_at_sampled_windows():
    """An 8192 x 8192 map (67M cells, moved so that its storage wraps):
    normals depend only on a cell's 4-neighbours, so the oracle run on a
    window of the heights with a one-cell margin gives the exact expected
    normals of the window's interior; eight windows, two on the border."""
    S, res = 8192, 0.04
    rng = np.random.default_rng(8192)
    g = mem.Map(mem.MapParams(S, S, res, clear_min_count=0))
    g.move(37.3, -21.9)
    gen = torch.Generator(device="cuda").manual_seed(3)
    h = torch.randn((S, S), device="cuda", generator=gen) * 0.2
    h[torch.rand((S, S), device="cuda", generator=gen) < 0.03] = float("nan")
    g.set_layer(mem.MEM_LAYER_ELEVATION, 0, h)
    n = g.normals()
    torch.cuda.synchronize()
    wins = [(0, 0), (S - 64, S - 64)] + [tuple(rng.integers(1, S - 65, 2)) for _ in range(6)]
    for y0, x0 in wins:
        # window [y0 - 1, y0 + 65) x [x0 - 1, x0 + 65), clipped to the grid
        ya, yb, xa, xb = max(y0 - 1, 0), min(y0 + 65, S), max(x0 - 1, 0), min(x0 + 65, S)
        hw = h[ya:yb, xa:xb].double().cpu().numpy()
        o = O.OracleMap(xb - xa, yb - ya, res)
        o.set_layer(O.LAYER_ELEVATION, 0, hw)
        want = o.normals()
        got = n[ya:yb, xa:xb].double().cpu().numpy()
        # interior of the window: cells whose 4-neighbours lie in the window,
        # and grid border cells where the window reaches the border
        iy = slice(1 if ya > 0 or y0 > 0 else 0, (yb - ya) - (1 if yb < S else 0))
        ix = slice(1 if xa > 0 or x0 > 0 else 0, (xb - xa) - (1 if xb < S else 0))
        a, b = got[iy, ix], want[iy, ix]
        assert np.array_equal(np.isnan(a), np.isnan(b)), (y0, x0)
        ok = ~np.isnan(b)
        assert np.abs(a[ok] - b[ok]).max(initial=0.0) <= N_TOL, (y0, x0)
