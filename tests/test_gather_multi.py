"""Fused image gathers: mem_input_image_poses runs the gathers of bindings
that write different layers as one launch (k_gather_multi), splitting where
a layer repeats or a launch holds eight jobs.  Every layer must equal, bit
for bit, the same bindings fused one at a time (one mem_input_image call per
image and binding, each a single k_gather_fuse launch) on a twin map, with
every image type, storage type, rule, top-k input and channel width."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from lockstep import to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu

W, H, RES = 96, 72, 0.05
FP8_SCALE = [0.6] * 8 + [1.7] * 8


def layers():
    return [
        mem.Layer(3, mem.MEM_EXPAVG, 0.5),                             # 8: RGB
        mem.Layer(8, mem.MEM_GAUSS, 1.0, mem.MEM_BF16),                # 9: features
        mem.Layer(5, mem.MEM_DIRICHLET, 1.0),                          # 10: classes
        mem.Layer(16, mem.MEM_GAUSS, 0.5, mem.MEM_FP8_E4M3, FP8_SCALE),  # 11: features
        mem.Layer(4, mem.MEM_LATEST, 0.0),                             # 12: RGBA
        mem.Layer(8, mem.MEM_EXPAVG, 0.3, mem.MEM_BF16),               # 13
        mem.Layer(1, mem.MEM_GAUSS, 2.0),                              # 14
        mem.Layer(2, mem.MEM_LATEST, 0.0, mem.MEM_FP8_E4M3, [1.0, 2.0]),  # 15
        mem.Layer(3, mem.MEM_EXPAVG, 0.7),                             # 16
        mem.Layer(24, mem.MEM_GAUSS, 1.0),                             # 17
    ]


def pose_images(rng, p, n_poses):
    R = synth.camera_rotation(p * 2 * np.pi / n_poses + rng.uniform(-0.3, 0.3), math.radians(35)).astype(np.float32)
    T = np.zeros((3, 4), np.float32)
    T[:, :3] = R
    T[:, 3] = (rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 0.9)
    K = (80.0, 80.0, 63.5, 47.5)
    rgba = rng.integers(0, 256, (96, 128, 4), dtype=np.uint8)
    feat = synth.feature_image(rng, 48, 64, 48)
    cls = synth.class_image(rng, 96, 128, 5)
    probs = torch.from_numpy(cls)
    pk, ik = torch.topk(probs, 2, dim=-1)
    top = torch.cat([ik.float(), pk], -1).contiguous().numpy()
    ims = [
        # two layers of one u8 image; the dense class image; its top-2 form
        # into the same layer (a repeat: the group splits there)
        (rgba, K, [(8, 0, 3), (12, 0, 4)]),
        (feat, synth.scaled_intrinsics(K, 0.5), [(9, 0, 8), (11, 8, 16), (13, 24, 8), (14, 32, 1), (15, 33, 2),
                                                 (16, 35, 3), (17, 24, 24)]),
        (cls, K, [(10, 0, 5)]),
        (top, K, [(10, 0, 4, 2)]),
    ]
    return ims, T


@pytest.mark.parametrize("one_channel", [False, True])
@pytest.mark.parametrize("n_poses", [1, 3])
def test_fused_gathers_equal_one_binding_per_call(n_poses, one_channel):
    rng = np.random.default_rng(300 + n_poses + 10 * one_channel)
    lay = layers()
    a = mem.Map(mem.MapParams(W, H, RES, layers=lay))
    b = mem.Map(mem.MapParams(W, H, RES, layers=lay))
    h = np.where(rng.uniform(size=(H, W)) < 0.9, rng.normal(0, 0.08, (H, W)), np.nan).astype(np.float32)
    v = rng.uniform(1e-4, 1e-2, (H, W)).astype(np.float32)
    for m in (a, b):
        m.set_layer(mem.MEM_LAYER_ELEVATION, 0, torch.from_numpy(h))
        m.set_layer(mem.MEM_LAYER_VARIANCE, 0, torch.from_numpy(v))
    if one_channel:
        a.debug_gather_width(1)
        b.debug_gather_width(1)
    for it in range(2):
        poses = [pose_images(rng, p, n_poses) for p in range(n_poses)]
        dev = [([(to_dev(x), k, bd) for x, k, bd in ims], T) for ims, T in poses]
        a.input_image_poses(dev)
        for ims, T in dev:
            for x, k, bd in ims:
                for one in bd:
                    b.input_image(x, k, T, bind=[one])
        torch.cuda.synchronize()
        for lid in range(8, 18):
            x, y = a.get_layer(lid), b.get_layer(lid)
            assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), (lid, it)
        for lid in (9, 11, 14, 17):  # the Gaussian layers' variances
            x, y = a.get_layer(lid, 1), b.get_layer(lid, 1)
            assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), (lid, it)
    assert torch.isfinite(a.get_layer(17)[..., 0]).sum().item() > 100  # cells that the images reached
