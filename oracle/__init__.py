"""CPU oracle of the multi-modal elevation map update - TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liborc.so`` (plain C,
binary64 values, binary32 decisions; see ``mem_oracle.c``) with numpy
marshalling and shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

LATEST, EXPAVG, GAUSS, DIRICHLET = 0, 1, 2, 3
IMG_F32, IMG_U8 = 0, 3
LAYER_ELEVATION, LAYER_VARIANCE, LAYER_VALID, LAYER_HITS, LAYER_CLEAR = 0, 1, 2, 3, 4
LAYER_USER0 = 8
VIEW_VALUE, VIEW_AUX, VIEW_ARGMAX = 0, 1, 2

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P, I, F, I64 = C.c_void_p, C.c_int, C.c_float, C.c_int64
        L.orc_create.restype = P
        L.orc_create.argtypes = [I, I, F, F, F, F, F, I, F, I, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_move.argtypes = [P, F, F]
        L.orc_get_center.argtypes = [P, P, P]
        L.orc_set_center.argtypes = [P, I, I]
        L.orc_input_pointcloud.argtypes = [P, P, I64, P, I, P, I, P, P]
        L.orc_input_image.argtypes = [P, P, I, I, I, I, P, P, P, P, I, P]
        L.orc_cell_pixels.argtypes = [P, I, I, P, P, P]
        L.orc_point_cells.argtypes = [P, P, I64, P, P]
        L.orc_get_layer.argtypes = [P, I, I, P]
        L.orc_get_layer.restype = I
        L.orc_set_layer.argtypes = [P, I, I, P]
        L.orc_set_layer.restype = I
        L.orc_layer_channels.argtypes = [P, I]
        L.orc_layer_channels.restype = I
        L.orc_normals.argtypes = [P, P]
        L.orc_set_drift.argtypes = [P, I, C.c_float, I]
        L.orc_set_overlap.argtypes = [P, I, C.c_float, C.c_float]
        L.orc_drift_last.argtypes = [P, C.POINTER(C.c_double), C.POINTER(I)]
        L.orc_bresenham.argtypes = [I, I, I, I, P, P, I]
        L.orc_bresenham.restype = I
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _pose(T) -> np.ndarray:
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float32).reshape(3, 4))
    return T.reshape(12)


def _bind(bind) -> tuple[np.ndarray, int]:
    """Bindings (layer, ch_first, ch_count[, topk]) as int32 quadruples."""
    rows = [tuple(x) + (0,) * (4 - len(x)) for x in bind] if bind else [(0, 0, 0, 0)]
    b = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, 4))
    return b, (len(bind) if bind else 0)


def bresenham(ax: int, ay: int, bx: int, by: int) -> list[tuple[int, int]]:
    cap = abs(bx - ax) + abs(by - ay) + 2
    xs = np.zeros(cap, np.int32)
    ys = np.zeros(cap, np.int32)
    n = lib().orc_bresenham(ax, ay, bx, by, _ptr(xs), _ptr(ys), cap)
    return [(int(xs[i]), int(ys[i])) for i in range(n)]


class OracleMap:
    """One map of the oracle.  Layers are (channels, rule, param) triples."""

    def __init__(self, width, height, resolution, noise_c0=0.01, noise_c1=0.001,
                 max_range=100.0, clear_margin=0.05, clear_min_count=1,
                 min_depth=0.1, layers=()):
        L = lib()
        self.W, self.H = int(width), int(height)
        self.layers = [tuple(l) for l in layers]
        n = len(self.layers)
        ch = np.array([l[0] for l in self.layers] or [0], np.int32)
        ru = np.array([l[1] for l in self.layers] or [0], np.int32)
        pa = np.array([l[2] for l in self.layers] or [0], np.float32)
        self._keep = (ch, ru, pa)
        self._m = L.orc_create(self.W, self.H, resolution, noise_c0, noise_c1, max_range,
                               clear_margin, clear_min_count, min_depth, n,
                               _ptr(ch), _ptr(ru), _ptr(pa))

    def close(self):
        if self._m:
            lib().orc_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def move(self, x, y):
        lib().orc_move(self._m, float(x), float(y))

    def center(self):
        cx, cy = C.c_int(), C.c_int()
        lib().orc_get_center(self._m, C.byref(cx), C.byref(cy))
        return cx.value, cy.value

    def set_center(self, cx, cy):
        lib().orc_set_center(self._m, int(cx), int(cy))

    def input_pointcloud(self, xyz, T, ch=None, bind=()):
        xyz = np.ascontiguousarray(np.asarray(xyz, np.float32).reshape(-1, 3))
        n = xyz.shape[0]
        c = 0
        if ch is not None:
            ch = np.ascontiguousarray(np.asarray(ch, np.float32).reshape(n, -1))
            c = ch.shape[1]
        b, nb = _bind(bind)
        cells = np.zeros(max(n, 1), np.int32)
        lib().orc_input_pointcloud(self._m, _ptr(xyz), n, _ptr(ch), c, _ptr(b), nb,
                                   _ptr(_pose(T)), _ptr(cells))
        return cells[:n]

    def point_cells(self, xyz, T):
        xyz = np.ascontiguousarray(np.asarray(xyz, np.float32).reshape(-1, 3))
        n = xyz.shape[0]
        cells = np.zeros(max(n, 1), np.int32)
        lib().orc_point_cells(self._m, _ptr(xyz), n, _ptr(_pose(T)), _ptr(cells))
        return cells[:n]

    def input_image(self, img, K, T, bind=(), strides=None):
        img = np.asarray(img)
        if img.dtype == np.uint8:
            dt = IMG_U8
        else:
            img = img.astype(np.float32, copy=False)
            dt = IMG_F32
        if strides is None:
            img = np.ascontiguousarray(img)
            h, w, c = img.shape
            st = np.array([w * c, c, 1], np.int64)
        else:
            h, w, c = strides[3], strides[4], strides[5]
            st = np.array(strides[:3], np.int64)
        b, nb = _bind(bind)
        Kf = np.asarray(K, np.float32)
        pix = np.zeros(self.W * self.H, np.int32)
        lib().orc_input_image(self._m, _ptr(img), dt, h, w, c, _ptr(st), _ptr(Kf),
                              _ptr(_pose(T)), _ptr(b), nb, _ptr(pix))
        return pix.reshape(self.H, self.W)

    def cell_pixels(self, h, w, K, T):
        Kf = np.asarray(K, np.float32)
        pix = np.zeros(self.W * self.H, np.int32)
        lib().orc_cell_pixels(self._m, h, w, _ptr(Kf), _ptr(_pose(T)), _ptr(pix))
        return pix.reshape(self.H, self.W)

    def channels(self, layer, view=VIEW_VALUE):
        if view == VIEW_ARGMAX or (view == VIEW_AUX and layer >= LAYER_USER0
                                   and self.layers[layer - LAYER_USER0][1] == GAUSS):
            return 1
        return lib().orc_layer_channels(self._m, layer)

    def get_layer(self, layer, view=VIEW_VALUE):
        C_ = self.channels(layer, view)
        out = np.zeros(self.H * self.W * max(C_, 1), np.float64)
        r = lib().orc_get_layer(self._m, layer, view, _ptr(out))
        if r != 0:
            raise ValueError(f"oracle: no view {view} of layer {layer}")
        return out.reshape(self.H, self.W, C_) if C_ > 1 or layer >= LAYER_USER0 else out.reshape(self.H, self.W)

    def set_drift(self, on=True, kappa=3.0, min_points=100):
        """Drift compensation of later point clouds (see orc_set_drift)."""
        lib().orc_set_drift(self._m, 1 if on else 0, float(kappa), int(min_points))

    def set_overlap(self, on=True, range_xy=4.0, range_z=2.0):
        """Overlap clearance after later point clouds (see orc_set_overlap)."""
        lib().orc_set_overlap(self._m, 1 if on else 0, float(range_xy), float(range_z))

    def drift_last(self):
        """(offset applied by the last cloud, its consistent points)."""
        d, n = C.c_double(), C.c_int()
        lib().orc_drift_last(self._m, C.byref(d), C.byref(n))
        return d.value, n.value

    def normals(self):
        """[H, W, 3] unit surface normals from the heights: central
        differences over the 4-neighbourhood (see orc_normals)."""
        out = np.zeros(self.H * self.W * 3, np.float64)
        lib().orc_normals(self._m, _ptr(out))
        return out.reshape(self.H, self.W, 3)

    def set_layer(self, layer, view, values):
        v = np.ascontiguousarray(np.asarray(values, np.float64).reshape(-1))
        r = lib().orc_set_layer(self._m, layer, view, _ptr(v))
        if r != 0:
            raise ValueError(f"oracle: view {view} of layer {layer} is not settable")


# ---------------------------------------------------------------------------
# Learned completion network (unet_oracle.c)
# ---------------------------------------------------------------------------

def _unet_sigs(L):
    if getattr(L, "_unet_ready", False):
        return
    P, I = C.c_void_p, C.c_int
    L.orc_unet_num_params.restype = C.c_int64
    L.orc_unet_num_params.argtypes = [I, I, I]
    L.orc_unet_layer_offsets.argtypes = [I, I, I, P]
    L.orc_unet_forward.argtypes = [I, I, I, P, P, I, I, P, I]
    L.orc_unet_loss_grad.restype = C.c_double
    L.orc_unet_loss_grad.argtypes = [I, I, P, P, P, P, I, I, P, I]
    L.orc_round_bf16.restype = C.c_double
    L.orc_round_bf16.argtypes = [C.c_double]
    L._unet_ready = True


def unet_num_params(base, in_ch=3, out_ch=2):
    L = lib()
    _unet_sigs(L)
    return int(L.orc_unet_num_params(base, in_ch, out_ch))


def unet_layer_offsets(base, in_ch=3, out_ch=2):
    L = lib()
    _unet_sigs(L)
    off = np.zeros(18, np.int64)
    L.orc_unet_layer_offsets(base, in_ch, out_ch, _ptr(off))
    return off


def unet_forward(params, x, base, out_ch=2, bf16=False):
    """x: [B, S, S, Cin] NHWC; returns [B, S, S, out_ch].  bf16: the
    network's BF16 storage format (see unet_oracle.c), else binary64."""
    L = lib()
    _unet_sigs(L)
    x = np.ascontiguousarray(x, np.float64)
    B, S, _, cin = x.shape
    p = np.ascontiguousarray(params, np.float64)
    out = np.zeros((B, S, S, out_ch))
    L.orc_unet_forward(base, cin, out_ch, _ptr(p), _ptr(x), B, S, _ptr(out), int(bool(bf16)))
    return out


def unet_loss_grad(params, x, target, mask, base, bf16=False):
    """Gaussian NLL (mean over mask > 0) and its gradient."""
    L = lib()
    _unet_sigs(L)
    x = np.ascontiguousarray(x, np.float64)
    B, S, _, cin = x.shape
    p = np.ascontiguousarray(params, np.float64)
    t = np.ascontiguousarray(target, np.float64)
    m = np.ascontiguousarray(mask, np.float64)
    g = np.zeros_like(p)
    loss = L.orc_unet_loss_grad(base, cin, _ptr(p), _ptr(x), _ptr(t), _ptr(m), B, S, _ptr(g), int(bool(bf16)))
    return loss, g


def round_bf16(v):
    """Nearest BF16 of each value (through binary32, ties to even)."""
    L = lib()
    _unet_sigs(L)
    f = np.vectorize(L.orc_round_bf16, otypes=[np.float64])
    return f(np.asarray(v, np.float64))


# ---------------------------------------------------------------------------
# PCA layer of a feature layer (the post-processing plugin of the paper's
# post-processing figure; reading R25)
# ---------------------------------------------------------------------------

def pca_layer(values: np.ndarray, k: int = 3):
    """[H, W, C] feature values -> ([H, W, k] projections, [k] eigenvalues,
    [k, C] components).  Over the cells whose C values are all finite: the
    mean m and the population covariance S = (1/N) sum (f - m)(f - m)^T;
    the components are S's eigenvectors of the k largest eigenvalues in
    descending order, each signed so that its largest-magnitude entry (the
    first of equal ones) is positive; a cell's projection is
    ((f - m) . e_1, ..., (f - m) . e_k), NaN for the other cells.  Fewer
    than k channels leave the missing components and projections 0."""
    H, W, C = values.shape
    f = values.reshape(-1, C).astype(np.float64)
    ok = np.isfinite(f).all(1)
    out = np.full((H * W, k), np.nan)
    lam = np.zeros(k)
    comp = np.zeros((k, C))
    n = int(ok.sum())
    if n == 0:
        return out.reshape(H, W, k), lam, comp
    x = f[ok]
    m = x.sum(0) / n
    d = x - m
    S = (d.T @ d) / n
    w, V = np.linalg.eigh(S)          # ascending
    order = np.argsort(-w, kind="stable")[: min(k, C)]
    for r, i in enumerate(order):
        e = V[:, i]
        j = int(np.argmax(np.abs(e)))  # first of the largest magnitudes
        comp[r] = e if e[j] > 0 else -e
        lam[r] = w[i]
    out[ok] = d @ comp.T
    return out.reshape(H, W, k), lam, comp
