"""The full-rate single-robot frame in lockstep with the oracle at full size:
a 500x500 grid at 0.04 m; per frame a 128x2048 LiDAR cloud and four
640x480 depth-camera clouds (height update and clearing ray cast), then four
camera poses in one mem_input_image_poses call, each with an RGB u8 image
(exponential averaging), a 160x120x64 feature map at scaled intrinsics
(Gaussian rule) and a 640x480 20-class image (Dirichlet rule) - the data
association and fusion of Sec. III-B and III-C at the scale of Table I.
Two consecutive frames of the benchmark's own input (same generator, same
seed), compared after every cloud and after the image call."""
import time

import numpy as np
import pytest

from lockstep import compare, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import synth

pytestmark = pytest.mark.gpu

BIND = {"rgb": [(8, 0, 3)], "features": [(9, 0, 64)], "classes": [(10, 0, 20)]}


def test_two_full_rate_frames_in_lockstep():
    p = dict(synth.FULL_MAP)
    W, H, res = p.pop("width"), p.pop("height"), p.pop("resolution")
    g, o = make_pair(W, H, res, layers=synth.FULL_LAYERS, **p)
    t0 = time.time()
    frames = [f for _, f in synth.iter_full_frames(seed=1, n_frames=2, device="cuda")]
    print(f"generated 2 frames in {time.time() - t0:.1f}s", flush=True)
    pairs = 0
    for fi, f in enumerate(frames):
        x, y, _ = f["pose"]
        g.move(x, y)
        o.move(x, y)
        for ci, c in enumerate(f["clouds"]):
            sync_from_oracle(g, o)
            g.input_pointcloud(to_dev(c["xyz"]), c["T"])
            o.input_pointcloud(c["xyz"], c["T"])
            rep = compare(g, o, what=f"frame {fi} cloud {ci}")
            print(f"frame {fi} cloud {ci}: {len(c['xyz'])} points, {rep}", flush=True)
        sync_from_oracle(g, o)
        g.reset_stats()
        poses = []
        for c in f["cameras"]:
            ims = [(to_dev(c["rgb"]), c["K"], BIND["rgb"]), (to_dev(c["features"]), c["K_feat"], BIND["features"]),
                   (to_dev(c["classes"]), c["K"], BIND["classes"])]
            poses.append((ims, c["T"]))
        g.input_image_poses(poses)
        for c in f["cameras"]:
            o.input_image(c["rgb"], c["K"], c["T"], bind=BIND["rgb"])
            o.input_image(c["features"], c["K_feat"], c["T"], bind=BIND["features"])
            o.input_image(c["classes"], c["K"], c["T"], bind=BIND["classes"])
        rep = compare(g, o, what=f"frame {fi} images")
        st = g.stats()
        pairs += st["pairs_visible"]
        print(f"frame {fi} images: {st['pairs_visible']} visible pairs, {rep}", flush=True)
    # every one of the 24 image fusions sees thousands of cells (about 9.5k
    # on average for this seed)
    assert pairs > 2 * 12 * 5000
    g.close()
