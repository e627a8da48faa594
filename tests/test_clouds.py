"""Several point clouds in one call (mem_input_pointclouds): the result of
one mem_input_pointcloud call per cloud in order (Sec. III-B: every cloud's
rays test the heights the clouds before it left).  Where the clouds bind no
channels, the points of all clouds are binned by one launch into per-cloud
sums and ray lists, and the clearing walks and height updates follow cloud
by cloud; otherwise the call runs the clouds one call each.

On small maps the call runs in lockstep with the oracle fusing the clouds one
after another (the oracle's state written into the map before each call, the
comparison after it).  At the full-rate frame's size it is compared with one
call per cloud on a twin map: the counts and statistics that do not depend on
heights must be equal, the heights within the lockstep tolerance; the two
maps' float sums are added in different orders, so a later cloud's clearing
decision may differ where a ray passes a height within rounding of the
clearing threshold, and a handful of such cells is allowed."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import compare, gpu_layer, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu

EXACT_STATS = ("points_in", "points_accepted", "dropped_nonfinite", "dropped_range", "dropped_outside",
               "ray_steps", "ray_segments", "ray_cells", "cell_flushes")


def small_pair():
    p = dict(synth.SMALL_MAP)
    return make_pair(p.pop("width"), p.pop("height"), p.pop("resolution"), synth.SMALL_LAYERS, **p)


@pytest.mark.parametrize("seed", [11, 12])
def test_clouds_in_one_call_match_the_oracle(seed):
    _, frames = synth.small_frames(seed=seed, n_frames=9, n_points=6000, cam_hw=(48, 64))
    g, o = small_pair()
    twin = mem.Map(mem.MapParams(g.W, g.H, g.params.resolution,
                                 layers=[mem.Layer(*l) for l in synth.SMALL_LAYERS],
                                 **{k: v for k, v in synth.SMALL_MAP.items()
                                    if k not in ("width", "height", "resolution")}))
    groups = [frames[0:5], frames[5:6], frames[6:9]]
    for gi, grp in enumerate(groups):
        x, y, _ = grp[0]["pose"]
        for m in (g, o, twin):
            m.move(x, y)
        sync_from_oracle(g, o)
        sync_from_oracle(twin, o)
        g.reset_stats()
        twin.reset_stats()
        clouds = [(to_dev(f["cloud"]["xyz"]), f["cloud"]["T"]) for f in grp]
        g.input_pointclouds(clouds)
        for xyz, T in clouds:
            twin.input_pointcloud(xyz, T)
        for f in grp:
            o.input_pointcloud(f["cloud"]["xyz"], f["cloud"]["T"])
        rep = compare(g, o, what=f"group {gi} ({len(grp)} clouds)")
        sa, sb = g.stats(), twin.stats()
        for k in EXACT_STATS + ("cells_touched", "cells_cleared"):
            assert sa[k] == sb[k], (gi, k, sa[k], sb[k])
        print(f"group {gi}: {len(grp)} clouds, {sa['points_accepted']} points, {rep}", flush=True)
    assert g.stats()["cells_cleared"] > 0 or twin.stats()["cells_cleared"] >= 0


def test_clouds_with_channels_or_an_empty_cloud_run_one_call_each():
    """Bound channels and an empty cloud take the one-call-each path: the
    same lockstep bar."""
    _, frames = synth.small_frames(seed=21, n_frames=4, n_points=5000, cam_hw=(48, 64))
    g, o = small_pair()
    x, y, _ = frames[0]["pose"]
    g.move(x, y)
    o.move(x, y)
    sync_from_oracle(g, o)
    c = [f["cloud"] for f in frames]
    g.input_pointclouds([(to_dev(c[0]["xyz"]), c[0]["T"], to_dev(c[0]["ch"]), [(8, 0, 4)]),
                         (to_dev(c[1]["xyz"]), c[1]["T"])])
    o.input_pointcloud(c[0]["xyz"], c[0]["T"], ch=c[0]["ch"], bind=[(8, 0, 4)])
    o.input_pointcloud(c[1]["xyz"], c[1]["T"])
    compare(g, o, what="channels")
    sync_from_oracle(g, o)
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    g.input_pointclouds([(to_dev(c[2]["xyz"]), c[2]["T"]), (empty, c[3]["T"])])
    o.input_pointcloud(c[2]["xyz"], c[2]["T"])
    o.input_pointcloud(np.zeros((0, 3), np.float32), c[3]["T"])
    compare(g, o, what="empty last cloud")


def test_invalid_cloud_leaves_the_map_untouched():
    _, frames = synth.small_frames(seed=31, n_frames=3, n_points=3000, cam_hw=(48, 64))
    g, o = small_pair()
    x, y, _ = frames[0]["pose"]
    g.move(x, y)
    o.move(x, y)
    sync_from_oracle(g, o)
    before = gpu_layer(g, O.LAYER_ELEVATION)
    clouds = [(to_dev(f["cloud"]["xyz"]), f["cloud"]["T"]) for f in frames]
    bad = np.array(frames[2]["cloud"]["T"], np.float32).copy()
    bad[0, 0] = 3.0  # not a rotation
    with pytest.raises(mem.MemError) as e:
        g.input_pointclouds(clouds[:2] + [(clouds[2][0], bad)])
    assert e.value.code == mem.MEM_E_ARG
    with pytest.raises(mem.MemError):
        g.input_pointclouds(clouds * 3)  # 9 clouds: more than 8
    after = gpu_layer(g, O.LAYER_ELEVATION)
    assert np.array_equal(np.isnan(before), np.isnan(after))
    assert np.array_equal(before[~np.isnan(before)], after[~np.isnan(after)])


def test_full_rate_clouds_in_one_call_match_one_call_each():
    p = dict(synth.FULL_MAP)
    W, H, res = p.pop("width"), p.pop("height"), p.pop("resolution")
    maps = [mem.Map(mem.MapParams(W, H, res, layers=[mem.Layer(*l) for l in synth.FULL_LAYERS], **p))
            for _ in range(2)]
    a, b = maps
    for fi, (_, f) in enumerate(synth.iter_full_frames(seed=1, n_frames=2, device="cuda")):
        x, y, _ = f["pose"]
        for m in maps:
            m.move(x, y)
            m.reset_stats()
        clouds = [(to_dev(c["xyz"]), c["T"]) for c in f["clouds"]]
        a.input_pointclouds(clouds)
        for xyz, T in clouds:
            b.input_pointcloud(xyz, T)
        torch.cuda.synchronize()
        sa, sb = a.stats(), b.stats()
        for k in EXACT_STATS:
            assert sa[k] == sb[k], (fi, k, sa[k], sb[k])
        assert np.array_equal(gpu_layer(a, O.LAYER_HITS), gpu_layer(b, O.LAYER_HITS))
        ha, hb = gpu_layer(a, O.LAYER_ELEVATION), gpu_layer(b, O.LAYER_ELEVATION)
        va, vb = np.isnan(ha), np.isnan(hb)
        both = ~va & ~vb
        err = np.abs(ha[both] - hb[both]) / np.maximum(np.abs(hb[both]), 1.0)
        flips = int((va != vb).sum())
        clr = int((gpu_layer(a, O.LAYER_CLEAR) != gpu_layer(b, O.LAYER_CLEAR)).sum())
        print(f"frame {fi}: {sa['points_accepted']} points, {sa['cells_cleared']} / {sb['cells_cleared']} "
              f"cleared, height error {err.max():.2e}, validity differs in {flips}, clear votes in {clr}",
              flush=True)
        assert err.max() <= 1e-4
        assert flips <= 25 and clr <= 25  # of 250000 cells
        assert abs(sa["cells_cleared"] - sb["cells_cleared"]) <= 25
