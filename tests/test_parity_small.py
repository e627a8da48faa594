"""GPU parity against the oracle on small inputs: the small workload in
lockstep, integer decisions bit-exact, fusion rules on both input paths,
the robot-centric shift, and the edge cases (empty, ragged, all dropped,
nothing in view)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import compare, gpu_layer, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu

ID = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)


def pose(t=(0.0, 0.0, 0.0), R=None):
    T = ID.copy()
    if R is not None:
        T[:, :3] = R
    T[:, 3] = t
    return T


def run_frame(g, o, frame, check=True):
    """move -> cloud -> RGB image -> class image, each call in lockstep."""
    x, y, _ = frame["pose"]
    sync_from_oracle(g, o)
    g.move(x, y)
    o.move(x, y)
    if check:
        compare(g, o, what="move")
    cl = frame["cloud"]
    sync_from_oracle(g, o)
    g.input_pointcloud(to_dev(cl["xyz"]), cl["T"], ch=to_dev(cl["ch"]), bind=[(8, 0, 4)])
    o.input_pointcloud(cl["xyz"], cl["T"], ch=cl["ch"], bind=[(8, 0, 4)])
    rep = compare(g, o, what="cloud") if check else {}
    cam = frame["camera"]
    for img, b in ((cam["rgb"], [(9, 0, 3)]), (cam["classes"], [(10, 0, 8)])):
        sync_from_oracle(g, o)
        dimg = to_dev(img)
        pg = g.debug_cell_pixels(img.shape[0], img.shape[1], cam["K"], cam["T"])
        g.input_image(dimg, cam["K"], cam["T"], bind=b)
        po = o.input_image(img, cam["K"], cam["T"], bind=b)
        torch.cuda.synchronize()
        assert np.array_equal(pg.cpu().numpy(), po), "cell pixels differ"
        if check:
            compare(g, o, what="image")
    return rep


def test_small_workload_lockstep(small_workload):
    _, frames = small_workload
    p = dict(synth.SMALL_MAP)
    g, o = make_pair(p.pop("width"), p.pop("height"), p.pop("resolution"), synth.SMALL_LAYERS, **p)
    for f in frames:
        cl = f["cloud"]
        # bit-exact association before the call
        cg = g.debug_point_cells(to_dev(cl["xyz"]), cl["T"]).cpu().numpy()
        sync_from_oracle(g, o)
        assert np.array_equal(cg, o.point_cells(cl["xyz"], cl["T"]))
        run_frame(g, o, f)
    st = g.stats()
    assert st["points_in"] == 10 * 20000
    assert st["points_accepted"] + st["dropped_nonfinite"] + st["dropped_range"] + st["dropped_outside"] == st["points_in"]
    assert st["pairs_visible"] > 0 and st["cells_touched"] > 0


@pytest.mark.parametrize("n", [0, 1, 63, 1023, 1025, 4097, 30001])
def test_point_cells_bit_exact_with_ragged_sizes(n):
    rng = np.random.default_rng(n)
    g, o = make_pair(37, 23, 0.05, max_range=1.2)
    g.move(0.31, -0.17)
    o.move(0.31, -0.17)
    xyz = rng.uniform(-1.2, 1.2, (n, 3)).astype(np.float32)
    if n > 10:
        xyz[::7, 0] = np.nan
        xyz[3::11, 2] = np.inf
    yaw = 0.7
    T = pose((0.2, 0.1, 0.5), synth.rot_z(yaw).astype(np.float32))
    a = g.debug_point_cells(to_dev(xyz.reshape(-1, 3)), T).cpu().numpy()
    b = o.point_cells(xyz, T)
    assert np.array_equal(a, b)
    sync_from_oracle(g, o)
    g.input_pointcloud(to_dev(xyz.reshape(-1, 3)), T)
    o.input_pointcloud(xyz, T)
    compare(g, o, what=f"n={n}")


def test_points_on_cell_edges_decide_like_the_oracle():
    """Points exactly on lattice lines and one ulp either side."""
    g, o = make_pair(16, 16, 0.04)
    base = (np.arange(-8, 9) * np.float32(0.04)).astype(np.float32)
    xs = np.concatenate([base, np.nextafter(base, np.float32(-1)), np.nextafter(base, np.float32(1))])
    X, Y = np.meshgrid(xs, xs)
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1).astype(np.float32)
    T = pose((0.0, 0.0, 0.0))
    a = g.debug_point_cells(to_dev(xyz), T).cpu().numpy()
    assert np.array_equal(a, o.point_cells(xyz, T))


def rand_map_state(g, o, rng, valid_frac=0.8, hscale=0.3):
    """Seeded heights (with holes) and variances, given to the oracle and
    then written from it into the GPU map."""
    H, W = g.H, g.W
    h = np.where(rng.uniform(size=(H, W)) < valid_frac, rng.normal(0, hscale, (H, W)), np.nan)
    o.set_layer(O.LAYER_ELEVATION, 0, h)
    o.set_layer(O.LAYER_VARIANCE, 0, rng.uniform(1e-4, 1e-2, (H, W)))
    sync_from_oracle(g, o)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cell_pixels_bit_exact_on_random_terrain(seed):
    rng = np.random.default_rng(100 + seed)
    g, o = make_pair(61, 47, 0.05, min_depth=0.1)
    g.move(0.4, -0.3)
    o.move(0.4, -0.3)
    rand_map_state(g, o, rng)
    for k in range(4):
        yaw = rng.uniform(0, 2 * np.pi)
        R = synth.camera_rotation(yaw, math.radians(rng.uniform(10, 50))).astype(np.float32)
        T = pose((0.4 + rng.uniform(-0.5, 0.5), -0.3 + rng.uniform(-0.5, 0.5), rng.uniform(0.3, 1.5)), R)
        K = (80.0, 80.0, 63.5, 47.5)
        a = g.debug_cell_pixels(96, 128, K, T).cpu().numpy()
        b = o.cell_pixels(96, 128, K, T)
        assert np.array_equal(a, b)
        assert (b == -3).sum() > 0 and (b >= 0).sum() > 0


RULES = [(mem.MEM_LATEST, 0.0), (mem.MEM_EXPAVG, 0.3), (mem.MEM_GAUSS, 0.5), (mem.MEM_DIRICHLET, 1.0)]


@pytest.mark.parametrize("C", [1, 3, 13])
def test_point_channel_rules(C):
    rng = np.random.default_rng(C)
    layers = [(C, r, p) for r, p in RULES]
    g, o = make_pair(20, 20, 0.1, layers=layers, clear_min_count=0)
    for it in range(4):
        n = int(rng.integers(500, 3000))
        xyz = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.normal(0, 0.1, n)], 1).astype(np.float32)
        ch = rng.uniform(0, 1, (n, 4 * C + 2)).astype(np.float32)
        bind = [(8 + k, 2 + k * C, C) for k in range(4)]
        T = pose((0.05, -0.02, 0.4))
        sync_from_oracle(g, o)
        g.input_pointcloud(to_dev(xyz), T, ch=to_dev(ch), bind=bind)
        o.input_pointcloud(xyz, T, ch=ch, bind=bind)
        compare(g, o, what=f"points C={C} it={it}")


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("layout", ["hwc", "chw"])
def test_image_channel_rules(dtype, layout):
    rng = np.random.default_rng(7)
    C = 5
    layers = [(C, r, p) for r, p in RULES]
    g, o = make_pair(40, 40, 0.05, layers=layers)
    rand_map_state(g, o, rng, valid_frac=0.9, hscale=0.05)
    h, w = 72, 96
    K = (60.0, 60.0, 47.5, 35.5)
    for it in range(3):
        img = (rng.integers(0, 256, (h, w, 4 * C)).astype(np.uint8) if dtype == "u8"
               else rng.uniform(0, 1, (h, w, 4 * C)).astype(np.float32))
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(40)).astype(np.float32)
        T = pose((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.8), R)
        bind = [(8 + k, k * C, C) for k in range(4)]
        sync_from_oracle(g, o)
        if layout == "hwc":
            dimg = to_dev(img)
            o.input_image(img, K, T, bind=bind)
        else:
            chw = np.ascontiguousarray(img.transpose(2, 0, 1))
            dimg = to_dev(chw).permute(1, 2, 0)  # [h, w, c] view with CHW strides
            o.input_image(chw, K, T, bind=bind, strides=(w, 1, h * w, h, w, 4 * C))
        g.input_image(dimg, K, T, bind=bind)
        compare(g, o, counts=False, what=f"image {dtype} {layout} it={it}")


def test_images_of_one_pose_equal_sequential_single_images():
    """mem_input_images (shared occlusion walk) against the oracle fusing the
    images one after another; two images bind the same exp.-averaging layer
    so their order matters."""
    rng = np.random.default_rng(17)
    layers = [(3, mem.MEM_EXPAVG, 0.5), (8, mem.MEM_GAUSS, 1.0), (5, mem.MEM_DIRICHLET, 1.0)]
    g, o = make_pair(64, 48, 0.05, layers=layers)
    rand_map_state(g, o, rng, valid_frac=0.9, hscale=0.08)
    for it in range(3):
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(35)).astype(np.float32)
        T = pose((rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 0.9), R)
        K = (80.0, 80.0, 63.5, 47.5)
        Kq = synth.scaled_intrinsics(K, 0.25)
        rgb = rng.integers(0, 256, (96, 128, 3), dtype=np.uint8)
        rgb2 = rng.integers(0, 256, (96, 128, 3), dtype=np.uint8)
        feat = synth.feature_image(rng, 24, 32, 8)
        cls = synth.class_image(rng, 96, 128, 5)
        ims = [(rgb, K, [(8, 0, 3)]), (feat, Kq, [(9, 0, 8)]), (cls, K, [(10, 0, 5)]), (rgb2, K, [(8, 0, 3)])]
        sync_from_oracle(g, o)
        g.input_images([(to_dev(a), k, b) for a, k, b in ims], T)
        for a, k, b in ims:
            o.input_image(a, k, T, bind=b)
        compare(g, o, counts=False, what=f"images it={it}")


@pytest.mark.parametrize("moves",[[(0.13, 0.0), (0.5, 0.27), (-0.31, 0.9), (-0.31, 0.9), (5.0, -5.0), (0.0, 0.0)]])
def test_move_matches_oracle_bitwise(moves):
    rng = np.random.default_rng(3)
    layers = [(3, mem.MEM_EXPAVG, 0.5), (2, mem.MEM_GAUSS, 1.0), (4, mem.MEM_DIRICHLET, 1.0)]
    g, o = make_pair(23, 17, 0.1, layers=layers)
    n = 4000
    xyz = np.stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-0.9, 0.9, n), rng.normal(0, 0.1, n)], 1).astype(np.float32)
    ch = rng.uniform(0, 1, (n, 9)).astype(np.float32)
    bind = [(8, 0, 3), (9, 3, 2), (10, 5, 4)]
    T = pose((0.0, 0.0, 0.5))
    g.input_pointcloud(to_dev(xyz), T, ch=to_dev(ch), bind=bind)
    o.input_pointcloud(xyz, T, ch=ch, bind=bind)
    for (x, y) in moves:
        sync_from_oracle(g, o)
        g.move(x, y)
        o.move(x, y)
        assert g.center() == o.center()
        for L, v in [(0, 0), (1, 0), (2, 0), (3, 0), (8, 0), (9, 0), (9, 1), (10, 1)]:
            a = gpu_layer(g, L, v)
            b = o.get_layer(L, v)
            assert np.array_equal(a, b, equal_nan=True), (x, y, L, v)


def test_single_point_sets_empty_cell_bit_exactly():
    g, _ = make_pair(8, 8, 0.25, clear_min_count=0)
    xyz = np.array([[0.1, 0.2, -0.4375], [0.6, 0.6, 0.3]], np.float32)
    g.input_pointcloud(to_dev(xyz), ID)
    h = gpu_layer(g, 0)
    v = gpu_layer(g, 1)
    assert h[4, 4] == np.float32(-0.4375)
    r2 = np.float32(np.float32(xyz[0, 0] * xyz[0, 0]) + np.float32(xyz[0, 1] * xyz[0, 1])) + np.float32(xyz[0, 2] * xyz[0, 2])
    s = np.float32(np.float32(0.01) + np.float32(np.float32(0.001) * r2))
    assert v[4, 4] == np.float32(s * s)
    assert h[6, 6] == np.float32(0.3)


def test_cloud_larger_than_one_clearing_pass():
    """More than 2^20 points in one call: the clearing march runs in passes
    and walks long rays in segments; the votes, heights and every loaded
    cell still match the oracle's walk of each whole ray."""
    rng = np.random.default_rng(11)
    g, o = make_pair(160, 160, 0.05, max_range=20.0, clear_margin=0.05, clear_min_count=2)
    n0 = 200_000
    xy = rng.uniform(-3.95, 3.95, (n0, 2))
    z = 0.3 * np.sin(2 * xy[:, 0]) + 0.2 * np.cos(3 * xy[:, 1])
    ground = np.concatenate([xy, z[:, None]], 1).astype(np.float32)
    g.input_pointcloud(to_dev(ground), ID)
    o.input_pointcloud(ground, ID)
    compare(g, o, what="terrain")
    sync_from_oracle(g, o)
    before = g.stats()
    # sensor 0.4 m up; targets at every range, many below the terrain so
    # that rays cross raised cells and vote; in the half plane y > -0.2 no
    # target is nearer than 2 m, so the cells there are crossed but receive
    # no point and can be cleared
    n1 = (1 << 20) + 123_457
    r = np.concatenate([rng.uniform(0.05, 1.0, n1 // 2), rng.uniform(1.0, 3.9, n1 - n1 // 2)])
    a = rng.uniform(0, 2 * np.pi, n1)
    r = np.where(a < np.pi, np.maximum(r, 2.0 + (r % 0.1) * 19), r)
    t = np.array([0.1, -0.2, 0.4], np.float32)
    tgt = np.stack([r * np.cos(a) + 0.1, r * np.sin(a) - 0.2, rng.uniform(-0.6, 0.2, n1)], 1)
    cloud = (tgt - t).astype(np.float32)
    rng.shuffle(cloud)
    g.input_pointcloud(to_dev(cloud), pose(tuple(t)))
    o.input_pointcloud(cloud, pose(tuple(t)))
    compare(g, o, what="cloud of more than one pass")
    st = g.stats()
    steps = st["ray_steps"] - before["ray_steps"]
    assert steps > 20 * n1
    assert st["ray_cells"] - before["ray_cells"] == steps  # every cell of every ray loaded once
    assert st["cells_cleared"] > before["cells_cleared"]


def test_empty_cloud_and_all_dropped_and_nothing_in_view():
    rng = np.random.default_rng(4)
    g, o = make_pair(30, 30, 0.1, layers=[(3, mem.MEM_LATEST, 0.0)], max_range=2.0)
    xyz = np.stack([rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500), np.zeros(500)], 1).astype(np.float32)
    g.input_pointcloud(to_dev(xyz), pose((0, 0, 1.0)))
    o.input_pointcloud(xyz, pose((0, 0, 1.0)))
    sync_from_oracle(g, o)
    # n = 0: only clears the per-cloud layers
    g.input_pointcloud(torch.empty((0, 3), dtype=torch.float32, device="cuda"), ID)
    o.input_pointcloud(np.zeros((0, 3), np.float32), ID)
    compare(g, o, what="empty cloud")
    assert gpu_layer(g, 3).sum() == 0
    # every point beyond max_range
    far = np.full((100, 3), 5.0, np.float32)
    sync_from_oracle(g, o)
    g.input_pointcloud(to_dev(far), ID)
    o.input_pointcloud(far, ID)
    compare(g, o, what="all dropped")
    # camera looking away from the grid
    R = synth.camera_rotation(0.0, math.radians(-80)).astype(np.float32)  # pitched up
    img = np.zeros((20, 30, 3), np.uint8)
    before = gpu_layer(g, 8)
    g.input_image(to_dev(img), (20.0, 20.0, 14.5, 9.5), pose((0, 0, 1.0), R), bind=[(8, 0, 3)])
    assert np.array_equal(gpu_layer(g, 8), before, equal_nan=True)


def test_invalid_arguments_leave_the_map_untouched():
    g, _ = make_pair(10, 10, 0.1, layers=[(3, mem.MEM_LATEST, 0.0)])
    xyz = to_dev(np.zeros((10, 3), np.float32))
    bad_R = pose((0, 0, 0), np.array([[2, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32))
    with pytest.raises(mem.MemError):
        g.input_pointcloud(xyz, bad_R)
    with pytest.raises(mem.MemError):
        g.input_pointcloud(xyz, ID, ch=to_dev(np.zeros((10, 2), np.float32)), bind=[(8, 0, 3)])
    with pytest.raises(mem.MemError):
        g.input_image(to_dev(np.zeros((4, 4, 3), np.uint8)), (0.0, 1.0, 1.0, 1.0), ID, bind=[(8, 0, 3)])
    with pytest.raises(mem.MemError):
        g.get_layer(20)
    assert np.isnan(gpu_layer(g, 0)).all()
    g.input_pointcloud(xyz, ID)  # the map still works
    assert gpu_layer(g, 3)[5, 5] == 10


@pytest.mark.parametrize("planes", [13, 14, 16, 17])
def test_point_channels_around_the_lds_limit(planes):
    """Bound channel planes around the most the ingest reduces in LDS (the
    hash table, the block statistics and planes x 2048 sums must fit one
    workgroup's LDS; beyond that the sums go to global atomics)."""
    rng = np.random.default_rng(planes)
    layers = [(planes - 4, mem.MEM_LATEST, 0.0), (4, mem.MEM_DIRICHLET, 1.0)]
    g, o = make_pair(30, 30, 0.05, layers=layers, clear_min_count=0)
    n = 5000
    xyz = np.stack([rng.uniform(-0.8, 0.8, n), rng.uniform(-0.8, 0.8, n), rng.normal(0, 0.05, n)], 1).astype(np.float32)
    ch = rng.uniform(0, 1, (n, planes)).astype(np.float32)
    bind = [(8, 0, planes - 4), (9, planes - 4, 4)]
    sync_from_oracle(g, o)
    g.input_pointcloud(to_dev(xyz), ID, ch=to_dev(ch), bind=bind)
    o.input_pointcloud(xyz, ID, ch=ch, bind=bind)
    compare(g, o, what=f"{planes} planes")
