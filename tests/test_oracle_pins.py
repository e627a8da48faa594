"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle with something other than its own formula: a
worked example, a closed form, an invariant, an independent algebraic form
of the same posterior, exact rational arithmetic, or a textbook routine.
CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ID = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)


def pose(t=(0.0, 0.0, 0.0), R=None):
    T = ID.copy()
    if R is not None:
        T[:, :3] = R
    T[:, 3] = t
    return T


def f32(x):
    return float(np.float32(x))


# ---------------------------------------------------------------------------
# Bresenham (Sec. III-B cites Bresenham's algorithm)
# ---------------------------------------------------------------------------

def test_bresenham_worked_examples():
    n = 0
    for line in open(os.path.join(GOLDEN, "bresenham_worked.txt")):
        if line.startswith("#") or not line.strip():
            continue
        lhs, rhs = line.split(":")
        ax, ay, bx, by = map(int, lhs.split())
        want = [tuple(map(int, c.split(","))) for c in rhs.split()]
        assert O.bresenham(ax, ay, bx, by) == want, line
        n += 1
    assert n == 7


def bresenham_closed_form(ax, ay, bx, by):
    """The cells of the line as nearest lattice points to the ideal segment:
    one cell per major-axis step, the minor offset rounded to nearest with
    ties toward the start (exact rationals)."""
    dx, dy = bx - ax, by - ay
    sx, sy = (1 if dx >= 0 else -1), (1 if dy >= 0 else -1)
    adx, ady = abs(dx), abs(dy)
    out = []
    if adx >= ady:
        for k in range(adx + 1):
            m = 0 if adx == 0 else math.ceil(Fraction(2 * k * ady - adx, 2 * adx))
            out.append((ax + sx * k, ay + sy * m))
    else:
        for k in range(ady + 1):
            m = math.ceil(Fraction(2 * k * adx - ady, 2 * ady))
            out.append((ax + sx * m, ay + sy * k))
    return out


def test_bresenham_closed_form_and_invariants():
    rng = np.random.default_rng(1)
    for _ in range(400):
        ax, ay, bx, by = (int(v) for v in rng.integers(-40, 41, 4))
        cells = O.bresenham(ax, ay, bx, by)
        assert cells == bresenham_closed_form(ax, ay, bx, by)
        assert cells[0] == (ax, ay) and cells[-1] == (bx, by)
        assert len(cells) == max(abs(bx - ax), abs(by - ay)) + 1
        for (x0, y0), (x1, y1) in zip(cells, cells[1:]):
            assert max(abs(x1 - x0), abs(y1 - y0)) == 1


# ---------------------------------------------------------------------------
# Point association (Sec. III-B: by horizontal coordinates)
# ---------------------------------------------------------------------------

def exact_cell(x, y, res, W, H, cx=0, cy=0):
    """Cell by exact rational arithmetic on the binary32 inputs."""
    inv = Fraction(f32(1.0 / res))
    gx = math.floor(Fraction(x) * inv)
    gy = math.floor(Fraction(y) * inv)
    ox, oy = cx - W // 2, cy - H // 2
    if not (ox <= gx < ox + W and oy <= gy < oy + H):
        return -3
    return (gy - oy) * W + (gx - ox)


def test_point_cells_match_exact_rationals_off_edges():
    W = H = 40
    res = 0.04
    m = O.OracleMap(W, H, res)
    rng = np.random.default_rng(2)
    xyz = rng.uniform(-1.0, 1.0, (3000, 3)).astype(np.float32)
    got = m.point_cells(xyz, ID)
    inv = f32(1.0 / res)
    checked = 0
    for p, g in zip(xyz, got):
        fx, fy = float(p[0]) * inv, float(p[1]) * inv
        if min(abs(fx - round(fx)), abs(fy - round(fy))) < 1e-4:
            continue  # within rounding distance of a cell edge
        assert g == exact_cell(float(p[0]), float(p[1]), res, W, H)
        checked += 1
    assert checked > 2900


def test_lattice_centres_land_in_their_cell_and_drop_reasons():
    W, H, res = 10, 6, 0.04
    m = O.OracleMap(W, H, res, max_range=5.0)
    pts = []
    want = []
    for iy in range(H):
        for ix in range(W):
            pts.append([((ix - W // 2) + 0.5) * res, ((iy - H // 2) + 0.5) * res, 0.0])
            want.append(iy * W + ix)
    pts += [[np.nan, 0, 0], [0, np.inf, 0], [6.0, 0, 0], [0.3, 0, 0], [0, -0.2, 0]]
    want += [-1, -1, -2, -3, -3]
    got = m.point_cells(np.array(pts, np.float32), ID)
    assert list(got) == want


def test_pose_transform_applied_before_association():
    m = O.OracleMap(20, 20, 0.1)
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)  # yaw 90 deg
    T = pose((0.25, -0.35, 1.0), R)
    p = np.array([[0.5, 0.25, -1.0]], np.float32)   # -> map (0.0, 0.15, 0.0)
    # map x = -0.25 + 0.25 = 0.0 -> lattice 0 -> ix 10; map y = 0.5 - 0.35 = 0.15 -> lattice 1 -> iy 11
    assert m.point_cells(p, T)[0] == 11 * 20 + 10


# ---------------------------------------------------------------------------
# Height fusion (information form of the conjugate Gaussian update)
# ---------------------------------------------------------------------------

def sigma2(p, c0=0.01, c1=0.001):
    """Noise model with its binary32 parameters (the map takes c0, c1 as
    binary32)."""
    c0, c1 = f32(c0), f32(c1)
    r2 = float(p[0]) ** 2 + float(p[1]) ** 2 + float(p[2]) ** 2
    return (c0 + c1 * r2) ** 2


def test_single_point_sets_empty_cell_exactly():
    m = O.OracleMap(8, 8, 0.25, clear_min_count=0)
    p = np.array([[0.1, 0.2, -0.4375]], np.float32)
    m.input_pointcloud(p, ID)
    j = m.point_cells(p, ID)[0]
    h = m.get_layer(O.LAYER_ELEVATION).reshape(-1)
    v = m.get_layer(O.LAYER_VARIANCE).reshape(-1)
    assert h[j] == float(p[0, 2])
    assert v[j] == sigma2(p[0])
    assert m.get_layer(O.LAYER_HITS).reshape(-1)[j] == 1
    assert np.isnan(np.delete(h, j)).all()


def kalman_sequence(zs, vs, h=None, v=None):
    """Scalar Kalman filter, one measurement at a time."""
    for z, r in zip(zs, vs):
        if h is None:
            h, v = z, r
            continue
        K = v / (v + r)
        h = h + K * (z - h)
        v = (1 - K) * v
    return h, v


@pytest.mark.parametrize("prior", [False, True])
def test_information_form_equals_sequential_kalman(prior):
    rng = np.random.default_rng(3)
    m = O.OracleMap(8, 8, 0.25, clear_min_count=0)
    h0 = v0 = None
    if prior:
        m.input_pointcloud(np.array([[0.05, 0.05, 0.3]], np.float32), ID)
        h0 = f32(0.3)
        v0 = sigma2(np.array([0.05, 0.05, 0.3], np.float32))
    # 30 points in cell (4, 4) at various ranges -> various variances
    pts = np.stack([rng.uniform(0.01, 0.24, 30), rng.uniform(0.01, 0.24, 30),
                    rng.normal(0.2, 0.05, 30)], 1).astype(np.float32)
    T = pose((0.0, 0.0, 0.0))
    Tz = T.copy()
    m.input_pointcloud(pts, Tz)
    h = m.get_layer(O.LAYER_ELEVATION)[4, 4]
    v = m.get_layer(O.LAYER_VARIANCE)[4, 4]
    for perm in [np.arange(30), rng.permutation(30), rng.permutation(30)]:
        zs = [float(pts[i, 2]) for i in perm]
        vs = [sigma2(pts[i]) for i in perm]
        hk, vk = kalman_sequence(zs, vs, h0, v0)
        assert abs(h - hk) <= 1e-12 * max(1.0, abs(hk))
        assert abs(v - vk) <= 1e-12 * vk


def test_two_clouds_equal_their_union():
    rng = np.random.default_rng(4)
    pts = rng.uniform(-0.9, 0.9, (400, 3)).astype(np.float32)
    a = O.OracleMap(8, 8, 0.25, clear_min_count=0)
    b = O.OracleMap(8, 8, 0.25, clear_min_count=0)
    a.input_pointcloud(pts[:150], ID)
    a.input_pointcloud(pts[150:], ID)
    b.input_pointcloud(pts, ID)
    for L in (O.LAYER_ELEVATION, O.LAYER_VARIANCE):
        x, y = a.get_layer(L), b.get_layer(L)
        assert np.array_equal(np.isnan(x), np.isnan(y))
        ok = ~np.isnan(x)
        assert np.allclose(x[ok], y[ok], rtol=1e-12, atol=1e-15)


def test_posterior_between_observations_and_variance_shrinks():
    rng = np.random.default_rng(5)
    m = O.OracleMap(4, 4, 0.5, clear_min_count=0)
    m.input_pointcloud(np.array([[0.1, 0.1, 0.5]], np.float32), ID)
    h0 = m.get_layer(O.LAYER_ELEVATION)[2, 2]
    v0 = m.get_layer(O.LAYER_VARIANCE)[2, 2]
    pts = np.stack([rng.uniform(0.01, 0.49, 20), rng.uniform(0.01, 0.49, 20),
                    rng.normal(0.0, 0.3, 20)], 1).astype(np.float32)
    m.input_pointcloud(pts, ID)
    h = m.get_layer(O.LAYER_ELEVATION)[2, 2]
    v = m.get_layer(O.LAYER_VARIANCE)[2, 2]
    zs = [h0] + [float(z) for z in pts[:, 2]]
    assert min(zs) <= h <= max(zs)
    assert v <= min([v0] + [sigma2(p) for p in pts])


# ---------------------------------------------------------------------------
# Clearing ray cast ("height update & ray cast", Table I)
# ---------------------------------------------------------------------------

def test_flat_ground_sensor_above_casts_no_votes():
    W = H = 30
    m = O.OracleMap(W, H, 0.1)
    g = (np.arange(W) - W // 2 + 0.5) * 0.1
    X, Y = np.meshgrid(g, g)
    ground = np.stack([X.ravel(), Y.ravel(), np.zeros(W * H)], 1).astype(np.float32)
    T = pose((0.02, 0.03, 1.0))
    m.input_pointcloud(ground - np.array([0.02, 0.03, 1.0], np.float32), T)
    m.input_pointcloud(ground - np.array([0.02, 0.03, 1.0], np.float32), T)
    assert m.get_layer(O.LAYER_CLEAR).sum() == 0
    assert m.get_layer(O.LAYER_VALID).sum() == W * H


def test_wall_votes_match_brute_force_and_hits_win():
    """Ground at z = 0 everywhere except a wall of height 2 m; a sensor at
    1 m looks at ground points beyond the wall.  A wall cell gets one vote
    per ray whose Bresenham cells include it strictly between the ends (the
    ray is below 2 m - margin everywhere, so every crossing votes)."""
    W = H = 24
    res = 0.25
    m = O.OracleMap(W, H, res, clear_margin=0.05)
    wall = {(15, y) for y in range(4, 20)}
    hgt = np.zeros((H, W))
    for (x, y) in wall:
        hgt[y, x] = 2.0
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, hgt)
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.full((H, W), 1e-4))
    s = np.array([-0.375, 0.125, 1.0])  # lattice (-2, 0) -> logical (10, 12)
    rng = np.random.default_rng(6)
    ix = rng.integers(17, 24, 200)
    iy = rng.integers(0, 24, 200)
    pm = np.stack([(ix - 12 + rng.uniform(0.1, 0.9, 200)) * res,
                   (iy - 12 + rng.uniform(0.1, 0.9, 200)) * res, np.zeros(200)], 1)
    # one extra point that lands on a wall cell itself: hits win
    pm = np.vstack([pm, [[(15 - 12 + 0.5) * res, (12 - 12 + 0.5) * res, 2.0]]])
    m.input_pointcloud((pm - s).astype(np.float32), pose(tuple(s)))
    votes = np.zeros((H, W), int)
    for x, y in zip(ix, iy):
        for (cx_, cy_) in bresenham_closed_form(10, 12, int(x), int(y))[1:-1]:
            if (cx_, cy_) in wall:
                votes[cy_, cx_] += 1
    got = m.get_layer(O.LAYER_CLEAR)
    assert np.array_equal(got, votes)
    valid = m.get_layer(O.LAYER_VALID)
    for (x, y) in wall:
        if (x, y) == (15, 12):
            assert valid[y, x] == 1  # received a point: never cleared
        else:
            assert valid[y, x] == (0 if votes[y, x] > 0 else 1)


def test_removed_box_is_cleared_next_frame():
    W = H = 40
    res = 0.05
    m = O.OracleMap(W, H, res)
    g = (np.arange(W) - W // 2 + 0.5) * res
    X, Y = np.meshgrid(g, g)
    box = (np.abs(X - 0.5) < 0.15) & (np.abs(Y) < 0.15)
    Z = np.where(box, 0.4, 0.0)
    s = np.array([0.01, 0.02, 1.2])
    T = pose(tuple(s))
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    m.input_pointcloud((pts - s).astype(np.float32), T)
    assert m.get_layer(O.LAYER_VALID)[box].all()
    # the box is gone: the ground behind it is now visible; box cells get no
    # point when the sensor sees them only at grazing angles - drop them
    pts2 = np.stack([X.ravel(), Y.ravel(), np.zeros(W * H)], 1)[~box.ravel()]
    m.input_pointcloud((pts2 - s).astype(np.float32), T)
    cleared = m.get_layer(O.LAYER_VALID)[box] == 0
    assert cleared.mean() > 0.5


# ---------------------------------------------------------------------------
# Fusion rules (Sec. III-C)
# ---------------------------------------------------------------------------

def one_cell_map(rule, C, param):
    return O.OracleMap(4, 4, 1.0, clear_min_count=0, layers=[(C, rule, param)])


def feed(m, values, n_per=1):
    """One cloud with n_per points in cell (2, 2) carrying `values`."""
    values = np.asarray(values, np.float32).reshape(-1, m.layers[0][0])
    xyz = np.tile(np.array([[0.5, 0.5, 0.0]], np.float32), (values.shape[0], 1))
    m.input_pointcloud(xyz, ID, ch=values, bind=[(O.LAYER_USER0, 0, values.shape[1])])


def test_latest_is_the_mean_of_this_update():  # Eq. (1)
    m = one_cell_map(O.LATEST, 3, 0.0)
    feed(m, [[1, 2, 3], [3, 2, 1], [2, 5, 2]])
    assert np.allclose(m.get_layer(O.LAYER_USER0)[2, 2], [2, 3, 2], rtol=0, atol=1e-12)
    feed(m, [[7, 7, 7]])
    assert np.allclose(m.get_layer(O.LAYER_USER0)[2, 2], [7, 7, 7])
    assert np.isnan(m.get_layer(O.LAYER_USER0)[0, 0]).all()


def test_fig4_exponential_decay_vs_gradual_dirichlet_decay():
    """Fig. 4: prior mass on class 0, then repeated class-1 measurements.
    Exponential averaging: theta_0(t) = (1-w)^t theta_0(0) (Eq. (2)).
    Dirichlet: theta_0(t) = alpha_00 / (sum alpha_0 + t) (Eq. (11)-(12))."""
    w = 0.5
    e = one_cell_map(O.EXPAVG, 2, w)
    d = one_cell_map(O.DIRICHLET, 2, 1.0)
    feed(e, [[1, 0]])
    feed(d, [[1, 0]])  # alpha = (2, 1)
    for t in range(1, 12):
        feed(e, [[0, 1]])
        feed(d, [[0, 1]])
        te = e.get_layer(O.LAYER_USER0)[2, 2, 0]
        td = d.get_layer(O.LAYER_USER0)[2, 2, 0]
        assert abs(te - (1 - f32(w)) ** t) < 1e-12  # w is a binary32 parameter
        assert abs(td - 2.0 / (3.0 + t)) < 1e-12
        if t >= 2:
            assert td > te  # with w = 1/2 the Bayesian decay is the more gradual one


def test_expavg_weight_one_is_latest():
    rng = np.random.default_rng(8)
    a = one_cell_map(O.EXPAVG, 4, 1.0)
    b = one_cell_map(O.LATEST, 4, 0.0)
    for _ in range(5):
        v = rng.normal(size=(3, 4))
        feed(a, v)
        feed(b, v)
        assert np.allclose(a.get_layer(O.LAYER_USER0), b.get_layer(O.LAYER_USER0), equal_nan=True)


def gauss_precision_form(mu0, s0, fs, sf2):
    """Posterior of a Gaussian mean with known variance, written in
    precision form: 1/s = 1/s0 + N/sf2, mu = s (mu0/s0 + sum f / sf2)."""
    N = len(fs)
    if s0 is None:
        prec = N / sf2
        return np.sum(fs, 0) / sf2 / prec, 1 / prec
    prec = 1 / s0 + N / sf2
    return (mu0 / s0 + np.sum(fs, 0) / sf2) / prec, 1 / prec


def test_gauss_matches_precision_form_and_is_conjugate():
    rng = np.random.default_rng(9)
    sf2 = 0.7
    m = one_cell_map(O.GAUSS, 5, sf2)
    u = one_cell_map(O.GAUSS, 5, sf2)
    allf = []
    mu, s = None, None
    for k in range(6):
        fs = rng.normal(size=(int(rng.integers(1, 6)), 5))
        fs32 = fs.astype(np.float32).astype(np.float64)
        feed(m, fs)
        allf.append(fs32)
        mu, s = gauss_precision_form(mu, s, fs32, f32(sf2))
        got_mu = m.get_layer(O.LAYER_USER0)[2, 2]
        got_s = m.get_layer(O.LAYER_USER0, O.VIEW_AUX)[2, 2, 0]
        assert np.allclose(got_mu, mu, rtol=1e-12, atol=1e-12)
        assert abs(got_s - s) <= 1e-12 * s
    feed(u, np.concatenate(allf))  # one update with every observation
    assert np.allclose(u.get_layer(O.LAYER_USER0)[2, 2], mu, rtol=1e-12, atol=1e-12)


def test_gauss_single_observation_on_unobserved_cell_is_exact():
    m = one_cell_map(O.GAUSS, 3, 0.5)
    f = np.array([[0.125, -3.5, 7.0]], np.float32)
    feed(m, f)
    assert np.array_equal(m.get_layer(O.LAYER_USER0)[2, 2], f[0].astype(np.float64))
    assert m.get_layer(O.LAYER_USER0, O.VIEW_AUX)[2, 2, 0] == 0.5  # sigma_f^2 / 1


def test_dirichlet_counts_stay_integer_and_theta_normalised():
    rng = np.random.default_rng(10)
    K = 6
    m = O.OracleMap(6, 6, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 1.0)])
    for _ in range(8):
        n = 300
        xyz = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.5, 1.5, n), np.zeros(n)], 1)
        onehot = np.eye(K, dtype=np.float32)[rng.integers(0, K, n)]
        m.input_pointcloud(xyz.astype(np.float32), ID, ch=onehot, bind=[(O.LAYER_USER0, 0, K)])
    alpha = m.get_layer(O.LAYER_USER0, O.VIEW_AUX)
    assert np.array_equal(alpha, np.round(alpha))
    theta = m.get_layer(O.LAYER_USER0)
    assert np.all((theta >= 0) & (theta <= 1))
    assert np.allclose(theta.sum(-1), 1.0, atol=1e-12)
    am = m.get_layer(O.LAYER_USER0, O.VIEW_ARGMAX)[..., 0]
    assert np.array_equal(am, np.argmax(alpha, -1))  # numpy: first maximum


def test_dirichlet_probability_inputs_keep_normalisation():
    rng = np.random.default_rng(11)
    K = 4
    m = O.OracleMap(6, 6, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 1.0)])
    for _ in range(5):
        n = 200
        xyz = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.5, 1.5, n), np.zeros(n)], 1)
        p = rng.dirichlet(np.ones(K), n).astype(np.float32)
        m.input_pointcloud(xyz.astype(np.float32), ID, ch=p, bind=[(O.LAYER_USER0, 0, K)])
    theta = m.get_layer(O.LAYER_USER0)
    assert np.allclose(theta.sum(-1), 1.0, atol=1e-12)


# ---------------------------------------------------------------------------
# Camera association (Sec. III-B, Fig. 3)
# ---------------------------------------------------------------------------

def down_camera(t):
    """Camera looking straight down: x right = map x, y down = -map y,
    z forward = -map z."""
    R = np.array([[1, 0, 0], [0, -1, 0], [0, 0, -1]], np.float32)
    return pose(t, R)


def test_known_points_land_on_known_pixels():
    """Exact case: res 0.25, camera 4 m above flat ground at z = 0, fx = fy =
    64, principal point (31.5, 31.5): cell centre x = (k + 0.5)/4 projects to
    u = 64 x / 4 + 31.5 exactly, pixel floor(u + 0.5)."""
    W = H = 16
    res = 0.25
    m = O.OracleMap(W, H, res)
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.zeros((H, W)))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.ones((H, W)))
    K = (64.0, 64.0, 31.5, 31.5)
    T = down_camera((0.0, 0.0, 4.0))
    pix = m.cell_pixels(64, 64, K, T)
    for iy in range(H):
        for ix in range(W):
            x = Fraction((ix - W // 2) * 2 + 1, 8)
            y = Fraction((iy - H // 2) * 2 + 1, 8)
            u = Fraction(64) * x / 4 + Fraction(63, 2)
            v = Fraction(64) * (-y) / 4 + Fraction(63, 2)
            col, row = math.floor(u + Fraction(1, 2)), math.floor(v + Fraction(1, 2))
            assert pix[iy, ix] == row * 64 + col


def test_cells_behind_camera_are_never_visible_and_flat_map_all_visible():
    W = H = 40
    res = 0.1
    m = O.OracleMap(W, H, res, min_depth=0.1)
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.zeros((H, W)))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.ones((H, W)))
    from paper_2309_16818_amd import synth
    Rc = synth.camera_rotation(0.0, math.radians(30))  # facing +x, pitched down
    T = pose((0.03, 0.02, 1.0), Rc.astype(np.float32))
    K = (100.0, 100.0, 99.5, 79.5)
    pix = m.cell_pixels(160, 200, K, T)
    g = (np.arange(W) - W // 2 + 0.5) * res
    X, _ = np.meshgrid(g, g)
    assert (pix[X < 0.03] < 0).all()           # behind the camera
    assert (pix != -3).all()                     # flat ground never occludes itself
    assert (pix >= 0).sum() > 100


def test_wall_occlusion_matches_brute_force():
    """A wall row of height 1 m in front of a camera at 1.5 m: cells behind
    the wall are occluded exactly when their Bresenham cells include a wall
    cell whose height is at or above the ray (checked with rationals)."""
    W = H = 32
    res = 0.125
    m = O.OracleMap(W, H, res, min_depth=0.05)
    hgt = np.zeros((H, W))
    wall_x = 20
    hgt[8:24, wall_x] = 1.0
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, hgt)
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.ones((H, W)))
    from paper_2309_16818_amd import synth
    Rc = synth.camera_rotation(0.0, math.radians(35)).astype(np.float32)
    t = (0.0625, 0.0625, 1.5)  # lattice (0, 0) -> logical (16, 16)
    T = pose(t, Rc)
    K = (200.0, 200.0, 199.5, 149.5)
    pix = m.cell_pixels(300, 400, K, T)
    ox = -W // 2
    for iy in range(H):
        for ix in range(W):
            if pix[iy, ix] == -2 or pix[iy, ix] == -1:
                continue
            xc = Fraction(2 * (ox + ix) + 1, 16)
            yc = Fraction(2 * (ox + iy) + 1, 16)
            hj = Fraction(hgt[iy, ix])
            cells = bresenham_closed_form(16, 16, ix, iy)[1:-1]
            xmaj = abs(ix - 16) >= abs(iy - 16)
            occ = False
            for (kx, ky) in cells:
                if hgt[ky, kx] == 0 and hj == 0:
                    continue
                c = Fraction(2 * (ox + (kx if xmaj else ky)) + 1, 16)
                s = Fraction(t[0]) if xmaj else Fraction(t[1])
                p = xc if xmaj else yc
                zr = Fraction(t[2]) + (hj - Fraction(t[2])) * (c - s) / (p - s)
                if Fraction(hgt[ky, kx]) >= zr:
                    occ = True
                    break
            assert (pix[iy, ix] == -3) == occ, (ix, iy)
    assert (pix == -3).sum() > 20


def test_image_fusion_reads_pixels_through_strides():
    W = H = 16
    m1 = O.OracleMap(W, H, 0.25, layers=[(3, O.LATEST, 0.0)])
    m2 = O.OracleMap(W, H, 0.25, layers=[(3, O.LATEST, 0.0)])
    for m in (m1, m2):
        m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.zeros((H, W)))
        m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.ones((H, W)))
    rng = np.random.default_rng(12)
    img = rng.integers(0, 256, (64, 64, 3), dtype=np.uint8)
    K = (64.0, 64.0, 31.5, 31.5)
    T = down_camera((0.0, 0.0, 4.0))
    pix = m1.input_image(img, K, T, bind=[(O.LAYER_USER0, 0, 3)])
    chw = np.ascontiguousarray(img.transpose(2, 0, 1))
    m2.input_image(chw, K, T, bind=[(O.LAYER_USER0, 0, 3)], strides=(64, 1, 64 * 64, 64, 64, 3))
    a, b = m1.get_layer(O.LAYER_USER0), m2.get_layer(O.LAYER_USER0)
    assert np.array_equal(a, b)
    for iy in range(H):
        for ix in range(W):
            r, c = divmod(int(pix[iy, ix]), 64)
            assert np.array_equal(a[iy, ix], img[r, c] / 255.0)


# ---------------------------------------------------------------------------
# Robot-centric grid
# ---------------------------------------------------------------------------

def filled_map(W, H, res, seed):
    rng = np.random.default_rng(seed)
    m = O.OracleMap(W, H, res, layers=[(2, O.EXPAVG, 0.5), (3, O.DIRICHLET, 1.0)])
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.where(rng.uniform(size=(H, W)) < 0.8,
                                                          rng.normal(size=(H, W)), np.nan))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, rng.uniform(0.1, 1, (H, W)))
    m.set_layer(O.LAYER_USER0, O.VIEW_VALUE, rng.normal(size=(H, W, 2)))
    m.set_layer(O.LAYER_USER0 + 1, O.VIEW_AUX, rng.uniform(1, 5, (H, W, 3)))
    return m


def rolled(a, sx, sy, fill):
    """numpy.roll of a by (-sy, -sx) with the wrapped strips reset."""
    H, W = a.shape[:2]
    out = np.roll(a, (-sy, -sx), axis=(0, 1)).astype(np.float64)
    if sx > 0:
        out[:, W - sx:] = fill
    elif sx < 0:
        out[:, :-sx] = fill
    if sy > 0:
        out[H - sy:, :] = fill
    elif sy < 0:
        out[:-sy, :] = fill
    return out


@pytest.mark.parametrize("sx,sy", [(3, 0), (0, -2), (2, 5), (-4, -1), (0, 0)])
def test_move_equals_roll_with_reset(sx, sy):
    W, H, res = 12, 10, 0.5
    m = filled_map(W, H, res, 13)
    before = {L: m.get_layer(*L) for L in [(0, 0), (2, 0), (8, 0), (9, 1)]}
    m.move(sx * res + 0.25, sy * res + 0.25)
    assert m.center() == (sx, sy)
    fills = {(0, 0): np.nan, (2, 0): 0.0, (8, 0): np.nan, (9, 1): 1.0}
    for L, b in before.items():
        assert np.array_equal(m.get_layer(*L), rolled(b, sx, sy, fills[L]), equal_nan=True), L


def test_move_there_and_back_restores_the_overlap_and_far_move_resets():
    W, H, res = 12, 10, 0.5
    m = filled_map(W, H, res, 14)
    b = m.get_layer(0, 0)
    m.move(2 * res, -3 * res)
    m.move(0.0, 0.0)
    a = m.get_layer(0, 0)
    # cells that stayed inside the grid through both moves: x >= 2, y < H - 3
    assert np.array_equal(a[:H - 3, 2:], b[:H - 3, 2:], equal_nan=True)
    assert np.isnan(a[H - 3:, :]).all() and np.isnan(a[:, :2]).all()
    m.move(100.0, 0.0)
    assert np.isnan(m.get_layer(0, 0)).all()
    assert (m.get_layer(O.LAYER_USER0 + 1, O.VIEW_AUX) == 1.0).all()


# ---------------------------------------------------------------------------
# Surface normals (Table I "normal calculation"): central differences of the
# heights over the 4-neighbourhood, NaN without a full neighbourhood.
# ---------------------------------------------------------------------------

def _oracle_with_heights(h, res):
    H, W = h.shape
    o = O.OracleMap(W, H, res)
    o.set_layer(O.LAYER_ELEVATION, 0, h)
    return o


def test_normals_of_a_plane_are_its_normal_and_border_is_nan():
    """Central differences are exact on a plane: every interior normal is
    (-a, -b, 1) / sqrt(a^2 + b^2 + 1) for h = a x + b y + c."""
    H, W, res, a, b = 9, 12, 0.05, 0.3, -0.7
    r32 = float(np.float32(res))  # the map's cell spacing is the binary32 resolution
    iy, ix = np.mgrid[0:H, 0:W]
    h = a * ix * r32 + b * iy * r32 + 0.25
    n = _oracle_with_heights(h, res).normals()
    want = np.array([-a, -b, 1.0]) / math.sqrt(a * a + b * b + 1.0)
    inner = n[1:-1, 1:-1]
    assert np.allclose(inner, want, rtol=0, atol=1e-12)
    assert np.isnan(n[0]).all() and np.isnan(n[-1]).all() and np.isnan(n[:, 0]).all() and np.isnan(n[:, -1]).all()
    assert np.allclose(np.linalg.norm(inner, axis=-1), 1.0, atol=1e-12)


def test_normals_of_a_parabola_follow_its_exact_slope():
    """For h = x^2 the central difference (x+r)^2 - (x-r)^2 over 2r is 2x
    exactly, so n = (-2x, 0, 1) / sqrt(4x^2 + 1); the y slope is zero."""
    H, W, res = 5, 11, 0.1
    iy, ix = np.mgrid[0:H, 0:W]
    x = (ix - 5) * float(np.float32(res))  # binary32 cell spacing
    n = _oracle_with_heights(x ** 2, res).normals()
    xs = x[1:-1, 1:-1]
    want = np.stack([-2 * xs, np.zeros_like(xs), np.ones_like(xs)], -1) / np.sqrt(4 * xs ** 2 + 1)[..., None]
    assert np.allclose(n[1:-1, 1:-1], want, rtol=0, atol=1e-12)


def test_normals_axes_and_missing_heights():
    """A slope along y only tilts the normal in y (a swapped axis fails), and
    a missing height removes the normals of the cell and its 4 neighbours."""
    H, W, res = 7, 8, 0.04
    iy, ix = np.mgrid[0:H, 0:W]
    h = 0.5 * iy * float(np.float32(res))
    h[3, 4] = np.nan
    n = _oracle_with_heights(h, res).normals()
    nan = np.isnan(n[..., 0])
    expect_nan = np.zeros((H, W), bool)
    expect_nan[0, :] = expect_nan[-1, :] = expect_nan[:, 0] = expect_nan[:, -1] = True
    for dy, dx in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
        expect_nan[3 + dy, 4 + dx] = True
    assert np.array_equal(nan, expect_nan)
    ok = ~nan
    assert np.allclose(n[ok][:, 0], 0.0, atol=1e-12)
    assert np.allclose(n[ok][:, 1], -0.5 / math.sqrt(1.25), atol=1e-12)


# ---------------------------------------------------------------------------
# Top-k class input (Sec. III-C): k (class, probability) pairs per point or
# pixel instead of the K probabilities, fused by the Dirichlet rule as the
# K-vector with each listed probability at its class.
# ---------------------------------------------------------------------------

def topk_inputs(rng, n, K, k, invalid=True):
    """n measurements of k distinct classes with probabilities; some listed
    indices invalid (negative, >= K, fractional, NaN) when asked."""
    idx = np.stack([rng.permutation(K)[:k] for _ in range(n)]).astype(np.float32)
    p = rng.dirichlet(np.ones(K), n)[:, :k].astype(np.float32)
    if invalid:
        bad = rng.uniform(size=idx.shape) < 0.1
        idx[bad] = rng.choice(np.array([-1.0, K, K + 3, 2.5, np.nan], np.float32), bad.sum())
    return idx, p


def brute_alpha(alpha0, cells, idx, p, K):
    """alpha0 plus, per measurement with a cell >= 0, each probability at its
    listed class if that class is an integer in [0, K)."""
    a = alpha0.copy()
    for j, ids, ps in zip(cells, idx, p):
        if j < 0:
            continue
        for c, q in zip(ids, ps):
            if np.isfinite(c) and c == int(c) and 0 <= c < K:
                a[j, int(c)] += float(q)
    return a


def test_topk_points_add_each_listed_probability_to_its_class():
    rng = np.random.default_rng(40)
    K, k, W = 7, 3, 6
    m = O.OracleMap(W, W, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 1.0)])
    alpha = np.ones((W * W, K))
    for _ in range(4):
        n = 400
        xyz = np.stack([rng.uniform(-1.6, 1.6, n), rng.uniform(-1.6, 1.6, n), np.zeros(n)], 1).astype(np.float32)
        idx, p = topk_inputs(rng, n, K, k)
        extra = rng.uniform(size=(n, 2)).astype(np.float32)  # unbound channels around the binding
        ch = np.concatenate([extra[:, :1], idx, p, extra[:, 1:]], 1)
        cells = m.point_cells(xyz, ID)
        alpha = brute_alpha(alpha, cells, idx, p, K)
        m.input_pointcloud(xyz, ID, ch=ch, bind=[(O.LAYER_USER0, 1, 2 * k, k)])
    got = m.get_layer(O.LAYER_USER0, O.VIEW_AUX).reshape(-1, K)
    assert np.allclose(got, alpha, rtol=1e-12, atol=1e-12)
    assert (got > 1.0).any()


def test_topk_listing_every_class_equals_the_dense_input():
    rng = np.random.default_rng(41)
    K, W, n = 5, 6, 500
    dense = O.OracleMap(W, W, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 1.0)])
    sparse = O.OracleMap(W, W, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 1.0)])
    xyz = np.stack([rng.uniform(-1.6, 1.6, n), rng.uniform(-1.6, 1.6, n), np.zeros(n)], 1).astype(np.float32)
    p = rng.dirichlet(np.ones(K), n).astype(np.float32)
    perm = np.stack([rng.permutation(K) for _ in range(n)])
    ch = np.concatenate([perm.astype(np.float32), np.take_along_axis(p, perm, 1)], 1)
    dense.input_pointcloud(xyz, ID, ch=p, bind=[(O.LAYER_USER0, 0, K)])
    sparse.input_pointcloud(xyz, ID, ch=ch, bind=[(O.LAYER_USER0, 0, 2 * K, K)])
    a, b = dense.get_layer(O.LAYER_USER0, O.VIEW_AUX), sparse.get_layer(O.LAYER_USER0, O.VIEW_AUX)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_topk_one_hot_counts_observations_per_class():
    """Top-1 with probability 1: alpha - alpha0 counts each class's points
    per cell exactly (integers)."""
    rng = np.random.default_rng(42)
    K, W, n = 4, 6, 600
    m = O.OracleMap(W, W, 0.5, clear_min_count=0, layers=[(K, O.DIRICHLET, 0.5)])
    xyz = np.stack([rng.uniform(-1.6, 1.6, n), rng.uniform(-1.6, 1.6, n), np.zeros(n)], 1).astype(np.float32)
    cls = rng.integers(0, K, n)
    m.input_pointcloud(xyz, ID, ch=np.stack([cls, np.ones(n)], 1).astype(np.float32), bind=[(O.LAYER_USER0, 0, 2, 1)])
    cells = m.point_cells(xyz, ID)
    want = np.full((W * W, K), 0.5)
    np.add.at(want, (cells[cells >= 0], cls[cells >= 0]), 1.0)
    assert np.array_equal(m.get_layer(O.LAYER_USER0, O.VIEW_AUX).reshape(-1, K), want)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_topk_image_pixels_fuse_their_listed_classes(dtype):
    """A top-2 class image seen from above: every visible cell adds its
    pixel's probabilities at its pixel's classes; u8 images carry the class
    as the byte and the probability as byte / 255."""
    W = H = 16
    K, k = 6, 2
    m = O.OracleMap(W, H, 0.25, layers=[(K, O.DIRICHLET, 1.0)])
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.zeros((H, W)))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.ones((H, W)))
    rng = np.random.default_rng(43)
    idx = rng.integers(0, K + 2, (64, 64, k))  # classes K, K+1 are invalid
    if dtype == "u8":
        img = np.concatenate([idx, rng.integers(0, 256, (64, 64, k))], -1).astype(np.uint8)
        probs = img[..., k:] / 255.0
    else:
        img = np.concatenate([idx, rng.uniform(0, 0.5, (64, 64, k))], -1).astype(np.float32)
        img[5, 7, 0] = 1.5  # fractional class: ignored
        probs = img[..., k:].astype(np.float64)
    T = down_camera((0.0, 0.0, 4.0))
    pix = m.input_image(img, (64.0, 64.0, 31.5, 31.5), T, bind=[(O.LAYER_USER0, 0, 2 * k, k)])
    got = m.get_layer(O.LAYER_USER0, O.VIEW_AUX)
    for iy in range(H):
        for ix in range(W):
            r, c = divmod(int(pix[iy, ix]), 64)
            want = np.ones(K)
            for q in range(k):
                v = float(img[r, c, q])
                if v == int(v) and 0 <= v < K:
                    want[int(v)] += probs[r, c, q]
            assert np.allclose(got[iy, ix], want, rtol=0, atol=1e-15), (ix, iy)


# ---------------------------------------------------------------------------
# z-error count and drift compensation (Table I rows 1-2, reading R23)
# ---------------------------------------------------------------------------

def flat_map(W, res, h0=0.0, v0=1e-4, **kw):
    m = O.OracleMap(W, W, res, clear_min_count=0, **kw)
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.full((W, W), h0))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.full((W, W), v0))
    return m


def centres(W, res, z):
    g = (np.arange(W) - W // 2 + 0.5) * res
    X, Y = np.meshgrid(g, g)
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1).astype(np.float32)


def test_drift_of_a_uniformly_raised_cloud_is_its_offset():
    """Every point 2^-5 m above a flat map: the weighted mean of equal errors
    is that error exactly, every held height moves by it, and the fused
    heights stay there."""
    W, res, d = 8, 0.5, 2.0 ** -5
    m = flat_map(W, res)
    m.set_drift(True, kappa=3.0, min_points=10)
    xyz = centres(W, res, d)
    m.input_pointcloud(xyz, ID)
    off, n = m.drift_last()
    assert off == d and n == W * W
    assert np.allclose(m.get_layer(O.LAYER_ELEVATION), d, rtol=0, atol=1e-15)


def test_drift_needs_its_minimum_of_consistent_points():
    W, res, d = 8, 0.5, 2.0 ** -5
    m = flat_map(W, res)
    m.set_drift(True, kappa=3.0, min_points=W * W + 1)
    m.input_pointcloud(centres(W, res, d)[: W * W // 2], ID)  # half the cells observed
    off, n = m.drift_last()
    assert off == 0.0 and n == W * W // 2
    h = m.get_layer(O.LAYER_ELEVATION).ravel()
    assert (h == 0.0).sum() == W * W // 2  # unobserved cells keep their height


def test_drift_matches_a_brute_force_of_its_definition():
    """Random terrain with random variances, a cloud raised by 3 cm with
    noise and 10 % outliers: the consistent set (binary32 test), the
    binary64 weighted mean rounded to binary32, and the shifted heights of
    cells without points, recomputed point by point."""
    rng = np.random.default_rng(50)
    W, res = 12, 0.25
    m = O.OracleMap(W, W, res, clear_min_count=0)
    h = rng.normal(0, 0.2, (W, W))
    h[rng.uniform(size=(W, W)) < 0.15] = np.nan
    v = rng.uniform(1e-4, 4e-3, (W, W))
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, h.astype(np.float32))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, v.astype(np.float32))
    kappa = np.float32(2.5)
    m.set_drift(True, kappa=float(kappa), min_points=5)
    n = 300
    xy = rng.uniform(-W * res / 2, W * res / 2, (n, 2))
    xyz = np.concatenate([xy, np.zeros((n, 1))], 1).astype(np.float32)
    cells = m.point_cells(xyz, ID)
    hh = np.nan_to_num(h.ravel()[np.maximum(cells, 0)])
    z = hh + 0.03 + rng.normal(0, 0.01, n)
    out = rng.uniform(size=n) < 0.1  # outliers a metre off
    z[out] += rng.choice([-1.0, 1.0], int(out.sum()))
    xyz[:, 2] = z.astype(np.float32)
    f32 = np.float32
    c0, c1 = f32(0.01), f32(0.001)
    sw = swe = 0.0
    cnt = 0
    for (x, y, zz), j in zip(xyz, cells):
        if j < 0 or np.isnan(h.ravel()[j]):
            continue
        r2 = f32(f32(f32(x * x) + f32(y * y)) + f32(zz * zz))
        sig = f32(c0 + f32(c1 * r2))
        vi = f32(sig * sig)
        e = f32(zz - f32(h.ravel()[j]))
        tot = f32(f32(v.ravel()[j]) + vi)
        if not f32(e * e) <= f32(f32(kappa * kappa) * tot):
            continue
        sw += 1.0 / float(tot)
        swe += float(e) / float(tot)
        cnt += 1
    want = float(f32(swe / sw))
    m.input_pointcloud(xyz, ID)
    off, got_n = m.drift_last()
    assert got_n == cnt and 0.5 * n < cnt < n
    assert off == want and abs(off - 0.03) < 0.005
    after = m.get_layer(O.LAYER_ELEVATION).ravel()
    hit = np.zeros(W * W, bool)
    hit[cells[cells >= 0]] = True
    keep = ~hit & ~np.isnan(h.ravel())
    assert np.array_equal(after[keep], (h.ravel()[keep].astype(f32) + f32(want)).astype(np.float64))


# ---------------------------------------------------------------------------
# Overlap clearance (Table I, reading R24)
# ---------------------------------------------------------------------------

def test_overlap_clearance_removes_other_levels_near_the_sensor():
    """A floor at 0 with a slab at 2.5 m over part of it (a level above) and
    a pit at -1.5 m: with ranges 1.2 m horizontally and 1 m vertically, only
    the slab and pit cells within 1.2 m of the sensor lose their heights,
    decided by brute force in binary32; an empty cloud still clears."""
    W, res = 24, 0.25
    m = O.OracleMap(W, W, res, clear_min_count=0)
    h = np.zeros((W, W))
    h[:, 14:] = 2.5
    h[2:6, 2:6] = -1.5
    h[10, 10] = np.nan
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, h)
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.full((W, W), 1e-3))
    m.set_overlap(True, range_xy=1.2, range_z=1.0)
    s = np.array([0.3, -0.1, 0.6], np.float32)
    m.input_pointcloud(np.zeros((0, 3), np.float32), pose(tuple(s)))
    f32 = np.float32
    want = ~np.isnan(h)
    for iy in range(W):
        for ix in range(W):
            if not want[iy, ix]:
                continue
            dx = f32(f32(f32(ix - W // 2) + f32(0.5)) * f32(res)) - s[0]
            dy = f32(f32(f32(iy - W // 2) + f32(0.5)) * f32(res)) - s[1]
            if f32(f32(dx * dx) + f32(dy * dy)) <= f32(f32(1.2) * f32(1.2)) and abs(f32(f32(h[iy, ix]) - s[2])) > f32(1.0):
                want[iy, ix] = False
    got = ~np.isnan(m.get_layer(O.LAYER_ELEVATION))
    assert np.array_equal(got, want)
    removed = ~np.isnan(h) & ~want
    assert removed.sum() > 10 and (h[removed] != 0).all()  # only slab and pit cells


def test_overlap_clearance_is_off_by_default_and_keeps_its_own_level():
    W, res = 16, 0.25
    m = O.OracleMap(W, W, res, clear_min_count=0)
    m.set_layer(O.LAYER_ELEVATION, O.VIEW_VALUE, np.full((W, W), 3.0))
    m.set_layer(O.LAYER_VARIANCE, O.VIEW_VALUE, np.full((W, W), 1e-3))
    m.input_pointcloud(np.zeros((0, 3), np.float32), pose((0.0, 0.0, 0.5)))
    assert not np.isnan(m.get_layer(O.LAYER_ELEVATION)).any()
    m.set_overlap(True, range_xy=10.0, range_z=3.0)  # 2.5 m away: within range_z
    m.input_pointcloud(np.zeros((0, 3), np.float32), pose((0.0, 0.0, 0.5)))
    assert not np.isnan(m.get_layer(O.LAYER_ELEVATION)).any()
    m.set_overlap(True, range_xy=10.0, range_z=2.0)
    m.input_pointcloud(np.zeros((0, 3), np.float32), pose((0.0, 0.0, 0.5)))
    assert np.isnan(m.get_layer(O.LAYER_ELEVATION)).all()


# ---------------------------------------------------------------------------
# PCA layer of a feature layer (post-processing plugin, reading R25)
# ---------------------------------------------------------------------------

def test_pca_recovers_known_axes_of_a_symmetric_cloud():
    """Pairs m +- a_i q_i along an orthonormal basis Q: the mean is m
    exactly, the covariance (1/d) sum a_i^2 q_i q_i^T, so the components
    are q_1..q_3 (signed), the eigenvalues a_i^2 / d, and the projection of
    m + a_1 q_1 is (a_1, 0, 0) up to the component's sign."""
    rng = np.random.default_rng(80)
    d = 8
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    a = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.4, 0.3, 0.2])
    m = rng.normal(size=d)
    pts = np.concatenate([m + a[:, None] * Q.T, m - a[:, None] * Q.T])  # 2d points
    vals = np.full((4, 5, d), np.nan)
    vals.reshape(-1, d)[: 2 * d] = pts
    out, lam, comp = O.pca_layer(vals)
    assert np.allclose(lam, a[:3] ** 2 / d, rtol=1e-12)
    for r in range(3):
        assert abs(abs(comp[r] @ Q[:, r]) - 1.0) < 1e-12
        j = np.argmax(np.abs(comp[r]))
        assert comp[r][j] > 0
    flat = out.reshape(-1, 3)
    assert np.allclose(np.abs(flat[0]), [a[0], 0, 0], atol=1e-12)
    assert np.isnan(flat[2 * d:]).all()


def test_pca_projections_are_centred_and_decorrelated():
    """Invariants at any size: the projections have zero mean and their
    covariance is diag(lambda); a channel permutation permutes the
    components and leaves the projections."""
    rng = np.random.default_rng(81)
    H, W, C = 20, 30, 12
    base = rng.normal(size=(H * W, 4)) @ rng.normal(size=(4, C)) * np.array([3, 2, 1, 0.5, *[0.2] * (C - 4)])
    vals = (base + 0.01 * rng.normal(size=base.shape)).reshape(H, W, C)
    vals[rng.uniform(size=(H, W)) < 0.2] = np.nan
    out, lam, comp = O.pca_layer(vals)
    p = out.reshape(-1, 3)
    p = p[np.isfinite(p).all(1)]
    assert np.allclose(p.mean(0), 0, atol=1e-10)
    assert np.allclose(p.T @ p / len(p), np.diag(lam), atol=1e-9 * lam[0])
    perm = rng.permutation(C)
    out2, lam2, comp2 = O.pca_layer(vals[..., perm])
    assert np.allclose(lam2, lam, rtol=1e-10)
    assert np.allclose(out2, out, atol=1e-9, equal_nan=True)


def test_pca_with_fewer_channels_than_components():
    vals = np.stack([np.arange(6.0), 2 * np.arange(6.0)], 1).reshape(2, 3, 2)
    out, lam, comp = O.pca_layer(vals)
    assert np.allclose(comp[0], [1, 2] / np.sqrt(5)) and (comp[2] == 0).all()
    assert np.allclose(lam[0], np.var(np.arange(6.0)) * 5)
    assert (out[..., 2] == 0).all()
