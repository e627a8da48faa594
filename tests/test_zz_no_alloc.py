"""mem_pca_noalloc, the PCA entry point for callers that cannot allocate,
against mem_pca on the same maps through the C ABI.

Both run the same kernels in the same order, mem_pca with the map's own
scratch and mem_pca_noalloc with the library's static device array, so the
projections and eigenvalues must agree bit for bit.  Two calls in a row on
the static array, the second on a smaller map with fewer channels and fewer
workgroups, show that the first call's leftovers do not leak into the
second; the oracle checks the first map's result as in the PCA tests."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import make_pair, sync_from_oracle
from paper_2309_16818_amd import mem

pytestmark = pytest.mark.gpu


def features(rng, H, W, Cn, holes=0.2):
    r = min(5, Cn)
    basis = np.linalg.qr(rng.normal(size=(Cn, Cn)))[0][:, :r]
    z = rng.normal(size=(H * W, r)) * np.array([3.0, 2.0, 1.3, 0.8, 0.5])[:r]
    f = z @ basis.T + 0.02 * rng.normal(size=(H * W, Cn)) + rng.normal(size=Cn)
    f[rng.uniform(size=H * W) < holes] = np.nan
    return f.reshape(H, W, Cn)


def noalloc(g: mem.Map, lid: int):
    """mem_pca_noalloc through the C ABI into caller-allocated tensors."""
    out = torch.full((g.H, g.W, 3), -7.0, dtype=torch.float32, device="cuda")
    lam = torch.full((3,), -7.0, dtype=torch.float32, device="cuda")
    st = mem.load().mem_pca_noalloc(g._h, lid, C.c_void_p(out.data_ptr()), C.c_void_p(lam.data_ptr()),
                                    mem._stream(None))
    assert st == mem.MEM_OK, mem.load().mem_last_error()
    return out, lam


def test_noalloc_pca_equals_pca_on_two_calls_in_a_row():
    rng = np.random.default_rng(2024)
    g1, o1 = make_pair(150, 110, 0.05, layers=[(48, mem.MEM_EXPAVG, 0.5)])
    o1.set_layer(8, 0, features(rng, 110, 150, 48))
    sync_from_oracle(g1, o1)
    g2, o2 = make_pair(37, 29, 0.05, layers=[(12, mem.MEM_GAUSS, 1.0, mem.MEM_BF16)])
    o2.set_layer(8, 0, features(rng, 29, 37, 12))
    sync_from_oracle(g2, o2)

    # two calls in a row on the static array: the larger map, then the smaller
    a1, l1 = noalloc(g1, 8)
    a2, l2 = noalloc(g2, 8)
    torch.cuda.synchronize()
    for g, a, l, o in ((g1, a1, l1, o1), (g2, a2, l2, o2)):
        ref, lam = g.pca(8)
        torch.cuda.synchronize()
        x, y = a.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(np.isnan(x), np.isnan(y))
        assert np.array_equal(x[~np.isnan(x)], y[~np.isnan(y)])
        assert l.cpu().tolist() == lam
        b, lam_o, _ = O.pca_layer(o.get_layer(8))
        ok = ~np.isnan(b)
        assert np.array_equal(np.isnan(x), np.isnan(b))
        assert np.abs(x[ok] - b[ok]).max() / np.sqrt(lam_o[0]) <= 1e-5
        assert np.allclose(l.cpu().numpy(), lam_o, rtol=1e-5)
    # and once more on the larger map after the smaller one, without eigenvalues
    out = torch.zeros((g1.H, g1.W, 3), dtype=torch.float32, device="cuda")
    g1.pca_noalloc(8, out)
    torch.cuda.synchronize()
    x = out.cpu().numpy()
    y = a1.cpu().numpy()
    assert np.array_equal(x[~np.isnan(x)], y[~np.isnan(y)])
    g1.close()
    g2.close()


def test_noalloc_pca_rejects_wide_layers_without_launching():
    g = mem.Map(mem.MapParams(16, 12, 0.1, layers=[mem.Layer(65, mem.MEM_LATEST, 0.0),
                                                   mem.Layer(4, mem.MEM_DIRICHLET, 1.0)]))
    out = torch.full((12, 16, 3), 5.0, dtype=torch.float32, device="cuda")
    lib = mem.load()
    assert lib.mem_pca_noalloc(g._h, 8, C.c_void_p(out.data_ptr()), None, mem._stream(None)) == mem.MEM_E_UNSUPPORTED
    assert lib.mem_pca_noalloc(g._h, 9, C.c_void_p(out.data_ptr()), None, mem._stream(None)) == mem.MEM_E_ARG
    assert lib.mem_pca_noalloc(g._h, 8, None, None, mem._stream(None)) == mem.MEM_E_ARG
    torch.cuda.synchronize()
    assert (out == 5.0).all()
    g.close()
