"""PCA layer of a feature layer (post-processing plugin): the GPU against the
oracle on the same seeded feature values (written into the oracle, then
from it into the GPU map at the layer's storage type).

Inputs have well separated leading eigenvalues (a low-rank model with
decreasing scales plus small noise), so the three components are unique.
Tolerances: the unobserved-cell pattern exactly; projections within
1e-5 sqrt(lambda_1) per component (binary64 sums and rotations, one
binary32 rounding of the output); eigenvalues within 1e-5 relative.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import make_pair, sync_from_oracle
from paper_2309_16818_amd import mem

pytestmark = pytest.mark.gpu


def features(rng, H, W, C, holes=0.15, scale=1.0):
    """Rank-6 structure with scales 4, 2.5, 1.6, 1, 0.6, 0.4 plus noise;
    some cells unobserved (all channels NaN) and some with one NaN channel."""
    r = min(6, C)
    basis = np.linalg.qr(rng.normal(size=(C, C)))[0][:, :r]
    z = rng.normal(size=(H * W, r)) * np.array([4.0, 2.5, 1.6, 1.0, 0.6, 0.4])[:r]
    f = z @ basis.T + 0.02 * rng.normal(size=(H * W, C)) + rng.normal(size=C)
    f[rng.uniform(size=H * W) < holes] = np.nan
    one = rng.uniform(size=H * W) < 0.05
    f[one, rng.integers(0, C, int(one.sum()))] = np.nan
    return scale * f.reshape(H, W, C)


def check(g, o, lid):
    out, lam = g.pca(lid)
    torch.cuda.synchronize()
    a = out.double().cpu().numpy()
    b, lam_o, _ = O.pca_layer(o.get_layer(lid))
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    scale = np.sqrt(max(lam_o[0], 1e-30))
    err = np.abs(a[ok] - b[ok]).max(initial=0.0) / scale
    assert err <= 1e-5, err
    assert np.allclose(lam, lam_o, rtol=1e-5, atol=1e-30)
    return int(ok.all(-1).sum()), lam_o


@pytest.mark.parametrize("C,storage,moves,scale", [
    (8, mem.MEM_F32, [(0.31, -0.47)], 1.0),
    (16, mem.MEM_BF16, [(1.0, 0.5), (-0.2, 0.35)], 1.0),
    (63, mem.MEM_F32, [(0.05, 0.05)], 1.0),
    (64, mem.MEM_FP8_E4M3, [], 0.1),  # inside the default FP8 scale (amax 1)
])
def test_pca_matches_oracle(C, storage, moves, scale):
    rng = np.random.default_rng(90 + C)
    g, o = make_pair(70, 53, 0.05, layers=[(C, mem.MEM_EXPAVG, 0.5, storage)])
    for mx, my in moves:
        g.move(mx, my)
        o.move(mx, my)
    o.set_layer(8, 0, features(rng, 53, 70, C, scale=scale))
    sync_from_oracle(g, o)
    n, lam = check(g, o, 8)
    assert n > 0.7 * 70 * 53 and lam[0] > lam[1] > lam[2] > 0


@pytest.mark.parametrize("C,storage", [(65, mem.MEM_F32), (200, mem.MEM_BF16), (384, mem.MEM_F32)])
def test_pca_of_wide_layers_matches_oracle(C, storage):
    """More than 64 channels (the 384-channel feature layer of the precision
    workload among them): covariance in 64 x 64 tiles, eigenpairs by
    orthogonal iteration, the same bars."""
    rng = np.random.default_rng(300 + C)
    g, o = make_pair(70, 53, 0.05, layers=[(C, mem.MEM_GAUSS, 1.0, storage)])
    g.move(0.4, -0.3)
    o.move(0.4, -0.3)
    o.set_layer(8, 0, features(rng, 53, 70, C))
    sync_from_oracle(g, o)
    n, lam = check(g, o, 8)
    assert n > 0.7 * 70 * 53 and lam[0] > lam[1] > lam[2] > 0


@pytest.mark.parametrize("C", [1, 2, 3])
def test_pca_with_few_channels(C):
    rng = np.random.default_rng(95 + C)
    g, o = make_pair(40, 30, 0.05, layers=[(C, mem.MEM_GAUSS, 1.0)])
    o.set_layer(8, 0, features(rng, 30, 40, C))
    sync_from_oracle(g, o)
    check(g, o, 8)
    out, lam = g.pca(8)
    if C < 3:
        assert lam[2] == 0.0
        v = out[..., 2].cpu().numpy()
        assert (v[np.isfinite(v)] == 0).all()


def test_pca_on_the_full_grid():
    """The full workload's grid (500 x 500) with a 64-channel feature layer."""
    rng = np.random.default_rng(99)
    g, o = make_pair(500, 500, 0.04, layers=[(64, mem.MEM_GAUSS, 1.0)])
    o.set_layer(8, 0, features(rng, 500, 500, 64, holes=0.4))
    sync_from_oracle(g, o)
    n, _ = check(g, o, 8)
    assert n > 100000


def test_pca_of_an_unobserved_layer_and_bad_layers():
    g = mem.Map(mem.MapParams(20, 20, 0.1, layers=[mem.Layer(5, mem.MEM_EXPAVG, 0.5),
                                                   mem.Layer(4, mem.MEM_DIRICHLET, 1.0),
                                                   mem.Layer(513, mem.MEM_LATEST, 0.0)]))
    out, lam = g.pca(8)
    torch.cuda.synchronize()
    assert torch.isnan(out).all() and lam == [0.0, 0.0, 0.0]
    with pytest.raises(mem.MemError) as e:
        g.pca(9)
    assert e.value.code == mem.MEM_E_ARG
    with pytest.raises(mem.MemError) as e:
        g.pca(10)
    assert e.value.code == mem.MEM_E_UNSUPPORTED
