"""Batches of independent maps (mem_batch_*): every map of a batch step is
checked against the oracle in lockstep, against independent single maps,
for isolation between maps, and for tuning-independent integer results."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import compare, gpu_layer, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu

RES = 0.05
SIZES = [(24, 24), (40, 33), (64, 64), (17, 50), (50, 17), (31, 31)]
LAYERS = [(16, mem.MEM_GAUSS, 1.0), (3, mem.MEM_EXPAVG, 0.5)]
CAM = (48, 64, 19, mem.MEM_F32)
IMG_BIND = [(8, 0, 16), (9, 16, 3)]
KCAM = (40.0, 40.0, 31.5, 23.5)


class MapView:
    """One map of a batch with the single-map read-out interface."""

    def __init__(self, B, m):
        self.B, self.m = B, m
        self.layers = B.layers
        self.W, self.H = B.W[m], B.H[m]

    def center(self):
        return self.B.center(self.m)

    def get_layer(self, layer, view=0):
        return self.B.get_layer(self.m, layer, view)

    def set_layer(self, layer, view, values):
        self.B.set_layer(self.m, layer, view, values)


def make_batch(sizes=SIZES, max_points=200000, cam=CAM):
    return mem.Batch([w for w, _ in sizes], [h for _, h in sizes], RES, layers=LAYERS,
                     max_points=max_points, cam=cam, img_bind=IMG_BIND if cam else ())


def make_oracles(sizes=SIZES):
    return [O.OracleMap(w, h, RES, max_range=100.0, layers=[l[:3] for l in LAYERS]) for w, h in sizes]


def step_inputs(rng, sizes, poses, counts):
    """Per-map points on a smooth synthetic surface around each robot, plus a
    camera per map.  Returns host arrays and the concatenated device points."""
    xyz, offs, Ts, Tc, Ks = [], [0], [], [], []
    for (w, h), (x, y, yaw), n in zip(sizes, poses, counts):
        r = 0.5 * min(w, h) * RES * np.sqrt(rng.uniform(size=n))
        a = rng.uniform(0, 2 * np.pi, n)
        px, py = x + r * np.cos(a), y + r * np.sin(a)
        pz = 0.1 * np.sin(3 * px) * np.cos(2 * py) + 0.3 * (np.abs(px - x - 0.3) < 0.1) + rng.normal(0, 0.01, n)
        T = synth.pose_matrix(synth.rot_z(yaw), (x, y, 0.6))
        xyz.append(synth.to_sensor(np.stack([px, py, pz], 1), T))
        offs.append(offs[-1] + n)
        Ts.append(T)
        Tc.append(synth.pose_matrix(synth.camera_rotation(yaw, math.radians(30)), (x, y, 0.7)))
        Ks.append(KCAM)
    imgs = np.concatenate([synth.feature_image(rng, CAM[0], CAM[1], CAM[2])[None] for _ in sizes])
    return (np.concatenate(xyz).astype(np.float32), np.array(offs, np.int64), np.array(Ts), np.array(Tc),
            np.array(Ks, np.float32), imgs)


def walk(rng, poses, jump=None):
    out = []
    for k, (x, y, yaw) in enumerate(poses):
        if jump == k:
            out.append((x + 10.0, y, yaw))
            continue
        out.append((x + rng.uniform(-0.12, 0.12), y + rng.uniform(-0.12, 0.12), yaw + rng.uniform(-0.1, 0.1)))
    return out


def run_batch_step(B, poses, xyz, offs, Ts, imgs, Ks, Tc):
    B.step(np.array([p[:2] for p in poses], np.float32), to_dev(xyz.reshape(-1, 3)), offs, Ts,
           images=to_dev(imgs), K=Ks, T_cam=Tc)


def test_every_map_of_a_batch_matches_the_oracle_in_lockstep():
    rng = np.random.default_rng(0)
    B = make_batch()
    orcs = make_oracles()
    views = [MapView(B, m) for m in range(len(SIZES))]
    poses = [(rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 6)) for _ in SIZES]
    for it in range(4):
        poses = walk(rng, poses, jump=3 if it == 2 else None)
        counts = [int(c) for c in rng.integers(0, 3000, len(SIZES))]
        counts[1] = 0 if it == 1 else counts[1]  # a map without points this step
        xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, counts)
        for v, o in zip(views, orcs):
            sync_from_oracle(v, o)
        run_batch_step(B, poses, xyz, offs, Ts, imgs, Ks, Tc)
        for m, (v, o) in enumerate(zip(views, orcs)):
            o.move(*poses[m][:2])
            o.input_pointcloud(xyz[offs[m]:offs[m + 1]], Ts[m])
            o.input_image(imgs[m], Ks[m], Tc[m], bind=IMG_BIND)
            compare(v, o, counts=True, what=f"step {it} map {m}")
    st = B.stats()
    assert st["points_accepted"] > 0 and st["pairs_visible"] > 0


def test_batch_equals_independent_single_maps_and_graph_equals_direct():
    rng = np.random.default_rng(1)
    B = make_batch()
    Bd = make_batch()
    Bd.set_tuning(512, 2, 8, graph=0)
    singles = [mem.Map(mem.MapParams(w, h, RES, max_range=100.0,
                                     layers=[mem.Layer(*l) for l in LAYERS])) for w, h in SIZES]
    poses = [(rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 6)) for _ in SIZES]
    for it in range(3):
        poses = walk(rng, poses)
        counts = [int(c) for c in rng.integers(100, 4000, len(SIZES))]
        xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, counts)
        run_batch_step(B, poses, xyz, offs, Ts, imgs, Ks, Tc)
        run_batch_step(Bd, poses, xyz, offs, Ts, imgs, Ks, Tc)
        for m, s in enumerate(singles):
            s.move(*poses[m][:2])
            s.input_pointcloud(to_dev(xyz[offs[m]:offs[m + 1]]), Ts[m])
            s.input_image(to_dev(imgs[m]), Ks[m], Tc[m], bind=IMG_BIND)
    for m, s in enumerate(singles):
        for other in (B, Bd):
            assert other.center(m) == s.center()
            for L in (2, 3, 4):  # valid, hits, clears: exact
                assert torch.equal(other.get_layer(m, L), s.get_layer(L)), (m, L)
            for L, v in ((0, 0), (1, 0), (8, 0), (8, 1), (9, 0)):
                a, b = other.get_layer(m, L, v), s.get_layer(L, v)
                assert torch.equal(torch.isnan(a), torch.isnan(b))
                ok = ~torch.isnan(b) & ~torch.isinf(b)
                assert torch.allclose(a[ok], b[ok], rtol=1e-5, atol=1e-6), (m, L, v)


def test_profiled_steps_equal_graph_steps_and_time_every_stage():
    """With per-stage events on, a step launches its stages directly; the
    maps end equal to the same steps replayed as the captured graph."""
    rng = np.random.default_rng(11)
    A, P = make_batch(), make_batch()
    P.profile_enable(True)
    poses = [(rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 6)) for _ in SIZES]
    for it in range(2):
        poses = walk(rng, poses)
        counts = [int(c) for c in rng.integers(100, 4000, len(SIZES))]
        xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, counts)
        run_batch_step(A, poses, xyz, offs, Ts, imgs, Ks, Tc)
        run_batch_step(P, poses, xyz, offs, Ts, imgs, Ks, Tc)
    kern = P.profile_read()
    for stage in ("b_prep", "b_reset", "b_bin", "b_tile_ingest", "b_logical", "b_march", "b_finalize",
                  "b_project", "b_gather"):
        # two steps; the gather runs once per image binding (two)
        assert kern[stage][0] == (2 * len(IMG_BIND) if stage == "b_gather" else 2), (stage, kern.get(stage))
        assert kern[stage][1] > 0.0
    P.profile_enable(False)
    # integers exact; floats to the batch's own run-to-run bar (its per-cell
    # sums are LDS atomics, so their order differs between runs)
    for m in range(len(SIZES)):
        for L in (2, 3, 4):
            assert torch.equal(A.get_layer(m, L), P.get_layer(m, L)), (m, L)
        for L, v in ((0, 0), (1, 0), (8, 0), (8, 1), (9, 0)):
            a, b = A.get_layer(m, L, v), P.get_layer(m, L, v)
            assert torch.equal(torch.isnan(a), torch.isnan(b))
            ok = ~torch.isnan(b) & ~torch.isinf(b)
            assert torch.allclose(a[ok], b[ok], rtol=1e-5, atol=1e-6), (m, L, v)


def test_maps_are_isolated():
    rng = np.random.default_rng(2)
    A, Bb = make_batch(), make_batch()
    poses = [(0.1 * k, -0.1 * k, 0.5 * k) for k in range(len(SIZES))]
    counts = [2000] * len(SIZES)
    xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, counts)
    xyz2 = xyz.copy()
    xyz2[offs[2]:offs[3], 2] += 0.2  # perturb map 2 only
    run_batch_step(A, poses, xyz, offs, Ts, imgs, Ks, Tc)
    run_batch_step(Bb, poses, xyz2, offs, Ts, imgs, Ks, Tc)
    for m in range(len(SIZES)):
        same = torch.allclose(A.get_layer(m, 0), Bb.get_layer(m, 0), rtol=1e-5, atol=1e-6, equal_nan=True)
        assert same == (m != 2), m
        if m != 2:
            for L in (2, 3, 4):
                assert torch.equal(A.get_layer(m, L), Bb.get_layer(m, L))


def test_autotuner_choice_keeps_integer_results():
    rng = np.random.default_rng(3)
    A, T = make_batch(), make_batch()
    poses = [(0.0, 0.0, 0.3 * k) for k in range(len(SIZES))]
    counts = [3000] * len(SIZES)
    xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, counts)
    args = (np.array([p[:2] for p in poses], np.float32), to_dev(xyz), offs, Ts)
    t = T.tune(*args, images=to_dev(imgs), K=Ks, T_cam=Tc)
    assert t["chunk"] in (512, 1024, 2048) and t["tile"] in (8, 16) and t["step_ms"] > 0
    # tuning restored the maps: both batches start from empty maps here
    for m in range(len(SIZES)):
        assert torch.isnan(T.get_layer(m, 0)).all()
    for bb in (A, T):
        run_batch_step(bb, poses, xyz, offs, Ts, imgs, Ks, Tc)
    for m in range(len(SIZES)):
        for L in (2, 3, 4):
            assert torch.equal(A.get_layer(m, L), T.get_layer(m, L))


def test_batch_rejects_bad_inputs_without_touching_maps():
    B = make_batch(cam=None)
    poses = [(0.0, 0.0, 0.0)] * len(SIZES)
    rng = np.random.default_rng(4)
    xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, SIZES, poses, [10] * len(SIZES))
    bad = offs.copy()
    bad[3] = bad[2] - 1
    with pytest.raises(mem.MemError):
        B.step(np.zeros((len(SIZES), 2), np.float32), to_dev(xyz), bad, Ts)
    with pytest.raises(mem.MemError):
        B.step(np.zeros((len(SIZES), 2), np.float32), to_dev(xyz), offs, Ts, images=to_dev(imgs), K=Ks, T_cam=Tc)
    Tbad = Ts.copy()
    Tbad[4, 0, 0] = 3.0
    with pytest.raises(mem.MemError):
        B.step(np.zeros((len(SIZES), 2), np.float32), to_dev(xyz), offs, Tbad)
    for m in range(len(SIZES)):
        assert torch.isnan(B.get_layer(m, 0)).all() and B.center(m) == (0, 0)
    B.step(np.zeros((len(SIZES), 2), np.float32), to_dev(xyz), offs, Ts)
    assert sum(int(B.get_layer(m, 3).sum()) for m in range(len(SIZES))) == 10 * len(SIZES)


# Maps of the batched workload's sizes (sides 64-256 cells): several 64x64
# ingest tiles per map, sides that are not multiples of 64, non-square maps,
# clouds of 10k-60k points and rays of up to ~128 cells.
LARGE = [(256, 256), (200, 131), (65, 250), (129, 97), (256, 70), (100, 100), (190, 190)]


def test_large_uneven_maps_match_the_oracle_in_lockstep():
    rng = np.random.default_rng(5)
    counts_max = 60000
    B = make_batch(LARGE, max_points=len(LARGE) * counts_max)
    orcs = make_oracles(LARGE)
    views = [MapView(B, m) for m in range(len(LARGE))]
    poses = [(rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 6)) for _ in LARGE]
    long_rays = 0
    for it in range(4):
        poses = walk(rng, poses, jump=1 if it == 2 else None)
        counts = [int(c) for c in rng.integers(10000, counts_max + 1, len(LARGE))]
        xyz, offs, Ts, Tc, Ks, imgs = step_inputs(rng, LARGE, poses, counts)
        for v, o in zip(views, orcs):
            sync_from_oracle(v, o)
        run_batch_step(B, poses, xyz, offs, Ts, imgs, Ks, Tc)
        for m, (v, o) in enumerate(zip(views, orcs)):
            o.move(*poses[m][:2])
            cells = o.input_pointcloud(xyz[offs[m]:offs[m + 1]], Ts[m])
            # rays longer than 64 cells (the march's segmented path)
            ok = cells >= 0
            cx, cy = cells[ok] % LARGE[m][0], cells[ok] // LARGE[m][0]
            sx, sy = LARGE[m][0] // 2, LARGE[m][1] // 2
            long_rays += int((np.maximum(np.abs(cx - sx), np.abs(cy - sy)) > 66).sum())
            o.input_image(imgs[m], Ks[m], Tc[m], bind=IMG_BIND)
            compare(v, o, counts=True, what=f"step {it} map {m} ({LARGE[m][0]}x{LARGE[m][1]})")
        print(f"step {it}: {sum(counts)} points", flush=True)
    assert long_rays > 10000
    st = B.stats()
    assert st["points_accepted"] > 0 and st["pairs_visible"] > 0
