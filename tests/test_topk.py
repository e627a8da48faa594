"""Top-k class input (Sec. III-C): k (class, probability) pairs per point or
pixel, fused by the Dirichlet rule as the K-vector with each listed
probability at its class.  GPU against the oracle in lockstep (tolerances of
tests/lockstep.py: alpha 1e-4 relative, theta 1e-4, argmax exact outside
near-ties), on points with invalid listed classes, u8 / f32 images in HWC and
CHW layouts, several images of one pose, and the full workload's grid.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import compare, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu

ID = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)


def pose(t, R=None):
    T = ID.copy()
    if R is not None:
        T[:, :3] = R
    T[:, 3] = t
    return T


def topk_of(probs, k):
    """Indices of the k largest probabilities (as values) and the
    probabilities, per row of [..., K]."""
    idx = np.argsort(-probs, -1, kind="stable")[..., :k]
    return idx.astype(np.float32), np.take_along_axis(probs, idx, -1).astype(np.float32)


def spoil(rng, idx, K, frac=0.1):
    """Replaces some listed classes by values that are not classes."""
    bad = rng.uniform(size=idx.shape) < frac
    idx = idx.copy()
    idx[bad] = rng.choice(np.array([-1.0, K, K + 7, 0.5, np.nan], np.float32), int(bad.sum()))
    return idx


def seeded_heights(g, o, rng, valid_frac=0.9, hscale=0.05):
    H, W = g.H, g.W
    o.set_layer(O.LAYER_ELEVATION, 0, np.where(rng.uniform(size=(H, W)) < valid_frac,
                                               rng.normal(0, hscale, (H, W)), np.nan))
    o.set_layer(O.LAYER_VARIANCE, 0, rng.uniform(1e-4, 1e-2, (H, W)))
    sync_from_oracle(g, o)


@pytest.mark.parametrize("K,k,n", [(20, 3, 30001), (7, 7, 4097), (5, 1, 1)])
def test_topk_points_match_oracle(K, k, n):
    rng = np.random.default_rng(K * 100 + k)
    g, o = make_pair(40, 40, 0.05, layers=[(K, mem.MEM_DIRICHLET, 1.0), (K, mem.MEM_DIRICHLET, 0.5)],
                     clear_min_count=0)
    for it in range(3):
        xyz = np.stack([rng.uniform(-1.1, 1.1, n), rng.uniform(-1.1, 1.1, n), rng.normal(0, 0.05, n)],
                       1).astype(np.float32)
        probs = rng.dirichlet(np.ones(K), n).astype(np.float32)
        idx, p = topk_of(probs, k)
        idx = spoil(rng, idx, K)
        # one unbound channel, the top-k pairs, then the dense probabilities
        ch = np.concatenate([rng.uniform(size=(n, 1)).astype(np.float32), idx, p, probs], 1)
        bind = [(8, 1, 2 * k, k), (9, 1 + 2 * k, K)]
        T = pose((0.05, -0.02, 0.4))
        sync_from_oracle(g, o)
        g.input_pointcloud(to_dev(xyz), T, ch=to_dev(ch), bind=bind)
        o.input_pointcloud(xyz, T, ch=ch, bind=bind)
        compare(g, o, what=f"top-{k} of {K} points it={it}")


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("layout", ["hwc", "chw"])
def test_topk_images_match_oracle(dtype, layout):
    rng = np.random.default_rng(3 if dtype == "u8" else 4)
    K, k = 12, 3
    g, o = make_pair(48, 40, 0.05, layers=[(K, mem.MEM_DIRICHLET, 1.0)])
    seeded_heights(g, o, rng)
    h, w = 72, 96
    Kc = (60.0, 60.0, 47.5, 35.5)
    for it in range(3):
        probs = synth.class_image(rng, h, w, K)
        idx, p = topk_of(probs, k)
        if dtype == "u8":
            idx = np.where(rng.uniform(size=idx.shape) < 0.1, K + 3, idx)  # bytes that are no class
            img = np.concatenate([idx, np.round(p * 255)], -1).astype(np.uint8)
        else:
            img = np.concatenate([spoil(rng, idx, K), p], -1).astype(np.float32)
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(40)).astype(np.float32)
        T = pose((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.8), R)
        bind = [(8, 0, 2 * k, k)]
        sync_from_oracle(g, o)
        if layout == "hwc":
            dimg = to_dev(img)
            o.input_image(img, Kc, T, bind=bind)
        else:
            chw = np.ascontiguousarray(img.transpose(2, 0, 1))
            dimg = to_dev(chw).permute(1, 2, 0)
            o.input_image(chw, Kc, T, bind=bind, strides=(w, 1, h * w, h, w, 2 * k))
        g.input_image(dimg, Kc, T, bind=bind)
        compare(g, o, counts=False, what=f"top-k image {dtype} {layout} it={it}")
    alpha = o.get_layer(8, 1)
    assert (alpha > 1.0).any()


def test_topk_and_dense_class_images_of_one_pose():
    """A dense class image and its top-4 reduction fused in one call into
    two layers, next to an RGB image; the top-k layer stays within the
    dropped probability mass of the dense one."""
    rng = np.random.default_rng(5)
    K, k = 10, 4
    g, o = make_pair(64, 48, 0.05, layers=[(3, mem.MEM_EXPAVG, 0.5), (K, mem.MEM_DIRICHLET, 1.0),
                                           (K, mem.MEM_DIRICHLET, 1.0)])
    seeded_heights(g, o, rng)
    Kc = (80.0, 80.0, 63.5, 47.5)
    for it in range(2):
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(35)).astype(np.float32)
        T = pose((rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 0.9), R)
        rgb = rng.integers(0, 256, (96, 128, 3), dtype=np.uint8)
        probs = synth.class_image(rng, 96, 128, K)
        idx, p = topk_of(probs, k)
        top = np.concatenate([idx, p], -1)
        ims = [(rgb, Kc, [(8, 0, 3)]), (probs, Kc, [(9, 0, K)]), (top, Kc, [(10, 0, 2 * k, k)])]
        sync_from_oracle(g, o)
        g.input_images([(to_dev(a), kk, b) for a, kk, b in ims], T)
        for a, kk, b in ims:
            o.input_image(a, kk, T, bind=b)
        compare(g, o, counts=False, what=f"dense + top-k images it={it}")
    dense, top = o.get_layer(9, 1), o.get_layer(10, 1)
    assert (top <= dense + 1e-12).all()


def test_topk_on_the_full_grid():
    """The full workload's class layer (20 classes, 500 x 500 cells at
    0.04 m) fed a top-3 class image of 640 x 480 from a camera 1.2 m up."""
    rng = np.random.default_rng(6)
    p = dict(synth.FULL_MAP)
    W, H, res = p.pop("width"), p.pop("height"), p.pop("resolution")
    g, o = make_pair(W, H, res, layers=[(20, mem.MEM_DIRICHLET, 1.0)], **p)
    seeded_heights(g, o, rng, valid_frac=0.95, hscale=0.03)
    probs = synth.class_image(rng, 480, 640, 20)
    idx, pr = topk_of(probs, 3)
    img = np.concatenate([idx, pr], -1)
    R = synth.camera_rotation(0.7, math.radians(30)).astype(np.float32)
    T = pose((0.3, -0.2, 1.2), R)
    Kc = (320.0, 320.0, 319.5, 239.5)
    g.input_image(to_dev(img), Kc, T, bind=[(8, 0, 6, 3)])
    o.input_image(img, Kc, T, bind=[(8, 0, 6, 3)])
    compare(g, o, counts=False, what="top-3 image on the full grid")
    assert (o.get_layer(8, 1) > 1.0).sum() > 2000


def test_topk_bindings_are_checked():
    g = mem.Map(mem.MapParams(16, 16, 0.1, layers=[mem.Layer(5, mem.MEM_DIRICHLET, 1.0),
                                                   mem.Layer(4, mem.MEM_EXPAVG, 0.5)]))
    xyz = torch.zeros((4, 3), device="cuda")
    ch = torch.zeros((4, 12), device="cuda")
    for bind in ([(8, 0, 6, 2)],      # 2k inputs expected
                 [(8, 0, 12, 6)],     # more classes listed than the layer has
                 [(9, 0, 4, 2)],      # not a Dirichlet layer
                 [(8, 0, 6, -1)],     # negative k
                 [(8, 8, 6, 3)]):     # beyond the inputs
        with pytest.raises(mem.MemError) as e:
            g.input_pointcloud(xyz, ID, ch=ch, bind=bind)
        assert e.value.code == mem.MEM_E_ARG, bind
    img = torch.zeros((8, 8, 6), device="cuda")
    with pytest.raises(mem.MemError):
        g.input_image(img, (8.0, 8.0, 3.5, 3.5), ID, bind=[(9, 0, 6, 3)])
    with pytest.raises(mem.MemError) as e:  # a batch checks its bindings the same way
        mem.Batch([16], [16], 0.1, layers=[mem.Layer(5, mem.MEM_DIRICHLET, 1.0)], max_points=16,
                  cam=(8, 8, 6, mem.MEM_F32), img_bind=[(8, 0, 6, 2)])
    assert e.value.code == mem.MEM_E_ARG


def test_topk_in_a_batch_matches_the_oracle():
    """A batch of maps of different sizes whose camera image carries top-3
    class pairs beside three dense feature channels: every map in lockstep
    with its oracle over moves, clouds and images."""
    from test_batch import MapView, step_inputs, walk
    rng = np.random.default_rng(140)
    sizes = [(24, 24), (40, 33), (17, 50), (64, 64)]
    K, k, res = 12, 3, 0.05
    H, W = 48, 64
    layers = [(K, mem.MEM_DIRICHLET, 1.0), (3, mem.MEM_EXPAVG, 0.5)]
    bind = [(8, 0, 2 * k, k), (9, 2 * k, 3)]
    B = mem.Batch([w for w, _ in sizes], [h for _, h in sizes], res, layers=layers, max_points=100000,
                  cam=(H, W, 2 * k + 3, mem.MEM_F32), img_bind=bind)
    orcs = [O.OracleMap(w, h, res, max_range=100.0, layers=[l[:3] for l in layers]) for w, h in sizes]
    views = [MapView(B, m) for m in range(len(sizes))]
    poses = [(rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 6)) for _ in sizes]
    for it in range(3):
        poses = walk(rng, poses)
        counts = [int(c) for c in rng.integers(500, 3000, len(sizes))]
        xyz, offs, Ts, Tc, Ks, _ = step_inputs(rng, sizes, poses, counts)
        imgs = []
        for _ in sizes:
            idx, p = topk_of(synth.class_image(rng, H, W, K), k)
            imgs.append(np.concatenate([spoil(rng, idx, K), p, rng.uniform(0, 1, (H, W, 3)).astype(np.float32)], -1))
        imgs = np.stack(imgs).astype(np.float32)
        for v, o in zip(views, orcs):
            sync_from_oracle(v, o)
        B.step(np.array([q[:2] for q in poses], np.float32), to_dev(xyz.reshape(-1, 3)), offs, Ts,
               images=to_dev(imgs), K=Ks, T_cam=Tc)
        for m, (v, o) in enumerate(zip(views, orcs)):
            o.move(*poses[m][:2])
            o.input_pointcloud(xyz[offs[m]:offs[m + 1]], Ts[m])
            o.input_image(imgs[m], Ks[m], Tc[m], bind=bind)
            compare(v, o, counts=True, what=f"batch top-k step {it} map {m}")
    assert B.stats()["pairs_visible"] > 0
