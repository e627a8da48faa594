"""z-error count and drift compensation (Table I rows 1-2): the GPU map
against the oracle in lockstep with the feature on.

The consistency test is a binary32 decision on both sides, so the number
of consistent points must agree exactly.  The offset is a binary64 sum
rounded to binary32; the two sides sum in different orders (about 1e-16
relative apart), so the offsets agree to the bit unless a sum lands that
close to a rounding boundary: the test allows one binary32 ulp.  Heights,
variances and clearing votes then follow the lockstep bars.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from lockstep import compare, gpu_layer, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu


def pose(t):
    T = np.zeros((3, 4), np.float32)
    T[:, :3] = np.eye(3)
    T[:, 3] = t
    return T


def terrain_pair(rng, W, res, hole=0.1, **kw):
    g, o = make_pair(W, W, res, **kw)
    ter = synth.make_terrain(rng, extent=max(W * res, 8.0), amplitude=0.2)
    c = (np.arange(W) - W // 2 + 0.5) * res
    X, Y = np.meshgrid(c, c)
    h = ter.height(X, Y)
    h[rng.uniform(size=h.shape) < hole] = np.nan
    o.set_layer(O.LAYER_ELEVATION, 0, h)
    o.set_layer(O.LAYER_VARIANCE, 0, rng.uniform(1e-4, 2e-3, (W, W)))
    sync_from_oracle(g, o)
    return g, o, ter


def shifted_cloud(rng, ter, n, half, sensor, dz, noise=0.01, outliers=0.05):
    """Points on the terrain raised by dz, with noise and outliers half a
    metre off, in the frame of a sensor at `sensor` (identity rotation)."""
    xy = rng.uniform(-half, half, (n, 2))
    z = ter.height(xy[:, 0], xy[:, 1]) + dz + rng.normal(0, noise, n)
    out = rng.uniform(size=n) < outliers
    z[out] += rng.choice([-0.5, 0.5], int(out.sum()))
    return (np.concatenate([xy, z[:, None]], 1) - np.asarray(sensor)).astype(np.float32)


def check_drift(g, o, what):
    go, gn = g.drift()
    oo, on = o.drift_last()
    assert gn == on, f"{what}: consistent points {gn} vs {on}"
    assert abs(go - oo) <= np.spacing(np.float32(abs(oo))), f"{what}: offset {go} vs {oo}"
    return oo, on


@pytest.mark.parametrize("clear_min", [0, 2])
def test_drift_lockstep_on_terrain(clear_min):
    rng = np.random.default_rng(60 + clear_min)
    g, o, ter = terrain_pair(rng, 64, 0.05, clear_min_count=clear_min, max_range=10.0)
    g.set_drift_compensation(True, kappa=3.0, min_points=50)
    o.set_drift(True, kappa=3.0, min_points=50)
    sensor = (0.0, 0.0, 1.0)
    offsets = []
    # raised 4 cm twice (the second cloud finds the map already moved), then
    # 2 cm: after the first fusions the map's variances are small, so a
    # larger step would leave few points within 3 sigma
    for it, dz in enumerate((0.04, 0.04, 0.02)):
        cl = shifted_cloud(rng, ter, 20000, 1.55, sensor, dz)
        sync_from_oracle(g, o)
        g.input_pointcloud(to_dev(cl), pose(sensor))
        o.input_pointcloud(cl, pose(sensor))
        off, n = check_drift(g, o, f"cloud {it}")
        compare(g, o, what=f"drift cloud {it}")
        offsets.append(off)
        assert n > 2000
    assert abs(offsets[0] - 0.04) < 0.01  # the map follows the raised cloud


def test_drift_with_too_few_points_or_disabled_changes_nothing():
    rng = np.random.default_rng(61)
    g, o, ter = terrain_pair(rng, 48, 0.05, clear_min_count=0)
    g.set_drift_compensation(True, kappa=3.0, min_points=10**6)
    o.set_drift(True, kappa=3.0, min_points=10**6)
    cl = shifted_cloud(rng, ter, 3000, 1.15, (0, 0, 1.0), 0.05)
    before = gpu_layer(g, 0)
    g.input_pointcloud(to_dev(cl), pose((0, 0, 1.0)))
    o.input_pointcloud(cl, pose((0, 0, 1.0)))
    off, n = check_drift(g, o, "too few")
    assert off == 0.0 and n > 0
    after = gpu_layer(g, 0)
    untouched = gpu_layer(g, mem.MEM_LAYER_HITS) == 0
    assert np.array_equal(before[untouched], after[untouched], equal_nan=True)
    compare(g, o, what="too few")
    g.set_drift_compensation(False)
    o.set_drift(False)
    sync_from_oracle(g, o)
    g.input_pointcloud(to_dev(cl), pose((0, 0, 1.0)))
    o.input_pointcloud(cl, pose((0, 0, 1.0)))
    assert g.drift() == (0.0, 0) and o.drift_last() == (0.0, 0)
    compare(g, o, what="disabled")
    # empty cloud, feature on
    g.set_drift_compensation(True, 3.0, 1)
    o.set_drift(True, 3.0, 1)
    g.input_pointcloud(to_dev(np.zeros((0, 3), np.float32)), pose((0, 0, 1.0)))
    o.input_pointcloud(np.zeros((0, 3), np.float32), pose((0, 0, 1.0)))
    assert g.drift() == (0.0, 0) and o.drift_last() == (0.0, 0)


def test_drift_on_full_rate_frames():
    """The full workload's grid and sensors: the first frame's clouds build
    the map (the first finds no held height), then every cloud of the
    second frame, one of them raised 2 cm by its pose, is compensated."""
    p = dict(synth.FULL_MAP)
    W, H, res = p.pop("width"), p.pop("height"), p.pop("resolution")
    g, o = make_pair(W, H, res, **p)
    g.set_drift_compensation(True, kappa=3.0, min_points=100)
    o.set_drift(True, kappa=3.0, min_points=100)
    _, frames = synth.full_frames(seed=2, n_frames=2)
    applied = 0
    for fi, f in enumerate(frames):
        x, y, _ = f["pose"]
        g.move(x, y)
        o.move(x, y)
        for ci, c in enumerate(f["clouds"]):
            T = c["T"].copy()
            if fi == 1 and ci == 2:
                T[2, 3] += 0.02
            sync_from_oracle(g, o)
            g.input_pointcloud(to_dev(c["xyz"]), T)
            o.input_pointcloud(c["xyz"], T)
            off, n = check_drift(g, o, f"frame {fi} cloud {ci}")
            applied += off != 0.0
            compare(g, o, what=f"full frame {fi} cloud {ci}")
    assert applied >= 4


def test_drift_arguments_are_checked():
    g = mem.Map(mem.MapParams(8, 8, 0.1))
    for kappa, mn in ((0.0, 10), (float("nan"), 10), (-1.0, 10), (3.0, 0)):
        with pytest.raises(mem.MemError) as e:
            g.set_drift_compensation(True, kappa, mn)
        assert e.value.code == mem.MEM_E_ARG
    g.set_drift_compensation(False, 0.0, 0)  # disabling takes no parameters
