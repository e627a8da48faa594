"""Python binding of libmem.so (include/mem.h): argument marshalling only.

Every computation runs in the HIP kernels of libmem.so.  torch supplies
device memory (tensor data pointers) and the stream
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch  # imported first so that libmem.so binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmem.so")

MEM_OK, MEM_E_ARG, MEM_E_NOMEM, MEM_E_HIP, MEM_E_STATE, MEM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
MEM_LATEST, MEM_EXPAVG, MEM_GAUSS, MEM_DIRICHLET = 0, 1, 2, 3
MEM_F32, MEM_BF16, MEM_FP8_E4M3, MEM_U8 = 0, 1, 2, 3
MEM_LAYER_ELEVATION, MEM_LAYER_VARIANCE, MEM_LAYER_VALID, MEM_LAYER_HITS, MEM_LAYER_CLEAR = 0, 1, 2, 3, 4
MEM_LAYER_USER0 = 8
MEM_VIEW_VALUE, MEM_VIEW_AUX, MEM_VIEW_ARGMAX = 0, 1, 2

STAT_FIELDS = ("points_in", "points_accepted", "dropped_nonfinite", "dropped_range", "dropped_outside",
               "cells_touched", "cells_cleared", "ray_cells", "cells_in_view", "pairs_visible",
               "occl_cells", "ray_steps", "occl_steps", "cell_flushes", "ray_segments")

# Exported symbols of include/mem.h.
SYMBOLS = ("mem_create", "mem_destroy", "mem_move", "mem_input_pointcloud", "mem_input_image",
           "mem_input_images", "mem_get_layer", "mem_set_layer", "mem_normals", "mem_set_drift_compensation", "mem_get_drift",
           "mem_set_overlap_clearance", "mem_pca", "mem_pca_noalloc", "mem_input_image_poses", "mem_input_pointclouds",
           "mem_get_center", "mem_debug_point_cells", "mem_debug_gather_width",
           "mem_debug_cell_pixels", "mem_get_stats", "mem_reset_stats", "mem_profile_enable",
           "mem_profile_read", "mem_last_error")


class mem_layer_desc(C.Structure):
    _fields_ = [("channels", C.c_int32), ("rule", C.c_int32), ("storage", C.c_int32),
                ("param", C.c_float), ("ch_scale", C.c_void_p)]


class mem_params(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("resolution", C.c_float),
                ("noise_c0", C.c_float), ("noise_c1", C.c_float), ("max_range", C.c_float),
                ("clear_margin", C.c_float), ("clear_min_count", C.c_int32),
                ("min_depth", C.c_float), ("n_layers", C.c_int32),
                ("layers", C.POINTER(mem_layer_desc))]


class mem_binding(C.Structure):
    _fields_ = [("layer", C.c_int32), ("ch_first", C.c_int32), ("ch_count", C.c_int32), ("topk", C.c_int32)]


class mem_image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("c", C.c_int32), ("strides", C.c_int64 * 3), ("K", C.c_float * 4),
                ("bind", C.POINTER(mem_binding)), ("n_bind", C.c_int32)]


class mem_cloud(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n", C.c_int64), ("ch", C.c_void_p), ("c", C.c_int32),
                ("bind", C.POINTER(mem_binding)), ("n_bind", C.c_int32), ("T_map_sensor", C.c_float * 12)]


class mem_stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STAT_FIELDS]


class mem_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class MemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mem error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads libmem.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2309_16818_amd.build`")
    L = C.CDLL(path)
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    sig = {
        "mem_create": [C.POINTER(mem_params), P, C.POINTER(P)],
        "mem_destroy": [P, P],
        "mem_move": [P, F, F, P],
        "mem_input_pointcloud": [P, P, I64, P, I32, C.POINTER(mem_binding), I32, P, P],
        "mem_input_image": [P, P, I32, I32, I32, I32, P, P, P, C.POINTER(mem_binding), I32, P],
        "mem_input_images": [P, C.POINTER(mem_image), I32, P, P],
        "mem_input_image_poses": [P, C.POINTER(mem_image), C.POINTER(I32), I32, P, P],
        "mem_input_pointclouds": [P, C.POINTER(mem_cloud), I32, P],
        "mem_get_layer": [P, I32, I32, P, P],
        "mem_set_layer": [P, I32, I32, P, P],
        "mem_normals": [P, P, P],
        "mem_set_drift_compensation": [P, I32, F, I32],
        "mem_get_drift": [P, C.POINTER(F), C.POINTER(I32), P],
        "mem_set_overlap_clearance": [P, I32, F, F],
        "mem_pca": [P, I32, P, C.POINTER(F), P],
        "mem_pca_noalloc": [P, I32, P, P, P],
        "mem_get_center": [P, C.POINTER(I32), C.POINTER(I32)],
        "mem_debug_point_cells": [P, P, I64, P, P, P],
        "mem_debug_cell_pixels": [P, I32, I32, P, P, P, P],
        "mem_debug_gather_width": [P, I32],
        "mem_get_stats": [P, C.POINTER(mem_stats), P],
        "mem_reset_stats": [P, P],
        "mem_profile_enable": [P, I32],
        "mem_profile_read": [P, C.POINTER(mem_kernel_time), I32, C.POINTER(I32)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    L.mem_last_error.restype = C.c_char_p
    L.mem_last_error.argtypes = []
    L.mem_calib_copy.argtypes = [P, P, I64, P]
    L.mem_calib_copy.restype = C.c_int
    L.mem_calib_atomic.argtypes = [P, I32, I32, I64, I64, P]
    L.mem_calib_atomic.restype = C.c_int
    L.mem_calib_gather.argtypes = [P, I64, P, I64, I32, I32, P]
    L.mem_calib_gather.restype = C.c_int
    L.mem_calib_last_error.argtypes = []
    L.mem_calib_last_error.restype = C.c_char_p
    _lib = L
    return L


# Calibration kernels of include/mem_calib.h (the measured peaks).
CALIB_SYMBOLS = ("mem_calib_copy", "mem_calib_atomic", "mem_calib_gather", "mem_calib_last_error")
MEM_CALIB_I32, MEM_CALIB_F32 = 0, 1
MEM_CALIB_UNIQUE, MEM_CALIB_SCATTER, MEM_CALIB_SHARED = 0, 1, 2


def calib_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """mem_calib_copy of src's bytes into dst (device tensors, same size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst must be contiguous and hold src's bytes")
    if load().mem_calib_copy(_dev_ptr(src, "src"), _dev_ptr(dst, "dst"), nb, _stream(stream)) != 0:
        raise MemError(MEM_E_ARG, load().mem_calib_last_error().decode())


def calib_atomic(buf: torch.Tensor, pattern: int, n_ops: int, n_addr: int | None = None, stream=None):
    """mem_calib_atomic: n_ops atomic adds of 1 into buf (int32 or float32)."""
    dt = {torch.int32: MEM_CALIB_I32, torch.float32: MEM_CALIB_F32}[buf.dtype]
    n_addr = buf.numel() if n_addr is None else n_addr
    if n_addr > buf.numel():
        raise ValueError("n_addr exceeds the buffer")
    if load().mem_calib_atomic(_dev_ptr(buf, "buf"), dt, pattern, n_ops, n_addr, _stream(stream)) != 0:
        raise MemError(MEM_E_ARG, load().mem_calib_last_error().decode())


def calib_gather(buf: torch.Tensor, out: torch.Tensor, per_lane: int, runs: bool = False, stream=None):
    """mem_calib_gather: out.numel() lanes of per_lane loads from buf
    (float32, a power-of-two number of words), scattered or in per-lane runs
    of consecutive words; out receives each lane's sum."""
    if buf.dtype != torch.float32 or out.dtype != torch.float32:
        raise ValueError("buf and out must be float32")
    if load().mem_calib_gather(_dev_ptr(buf, "buf"), buf.numel(), _dev_ptr(out, "out"), out.numel(), per_lane,
                               1 if runs else 0, _stream(stream)) != 0:
        raise MemError(MEM_E_ARG, load().mem_calib_last_error().decode())


def _check(code: int):
    if code != MEM_OK:
        raise MemError(code, load().mem_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _floats(vals, n):
    a = (C.c_float * n)(*[float(v) for v in vals])
    return a


def _pose(T):
    t = torch.as_tensor(T, dtype=torch.float32).reshape(-1).tolist()
    if len(t) != 12:
        raise ValueError("pose must be 3x4")
    return _floats(t, 12)


def _bindings(bind):
    """Bindings (layer, ch_first, ch_count[, topk]) as a mem_binding array."""
    bind = list(bind or [])
    arr = (mem_binding * max(1, len(bind)))()
    for i, b in enumerate(bind):
        layer, f, cnt = b[:3]
        arr[i] = mem_binding(int(layer), int(f), int(cnt), int(b[3]) if len(b) > 3 else 0)
    return arr, len(bind)


def _dev_ptr(t: torch.Tensor, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    return C.c_void_p(t.data_ptr())


@dataclass
class Layer:
    channels: int
    rule: int
    param: float
    storage: int = MEM_F32
    ch_scale: list | None = None


@dataclass
class MapParams:
    width: int
    height: int
    resolution: float
    noise_c0: float = 0.01
    noise_c1: float = 0.001
    max_range: float = 100.0
    clear_margin: float = 0.05
    clear_min_count: int = 1
    min_depth: float = 0.1
    layers: list = field(default_factory=list)


class Map:
    """A map on the current HIP device (wraps mem_create ... mem_destroy)."""

    def __init__(self, params: MapParams, stream=None):
        L = load()
        self.params = params
        self.W, self.H = params.width, params.height
        self.layers = [l if isinstance(l, Layer) else Layer(*l) for l in params.layers]
        descs = (mem_layer_desc * max(1, len(self.layers)))()
        self._scales = []
        for i, l in enumerate(self.layers):
            sc = None
            if l.ch_scale is not None:
                sc = _floats(l.ch_scale, l.channels)
                self._scales.append(sc)
            descs[i] = mem_layer_desc(l.channels, l.rule, l.storage, l.param,
                                      C.cast(sc, C.c_void_p) if sc is not None else None)
        p = mem_params(params.width, params.height, params.resolution, params.noise_c0,
                       params.noise_c1, params.max_range, params.clear_margin,
                       params.clear_min_count, params.min_depth, len(self.layers), descs)
        h = C.c_void_p()
        _check(L.mem_create(C.byref(p), _stream(stream), C.byref(h)))
        self._h = h

    def close(self, stream=None):
        if getattr(self, "_h", None):
            load().mem_destroy(self._h, _stream(stream))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- update ---------------------------------------------------------------
    def move(self, x, y, stream=None):
        _check(load().mem_move(self._h, float(x), float(y), _stream(stream)))

    def input_pointcloud(self, xyz: torch.Tensor, T, ch: torch.Tensor | None = None, bind=(),
                         stream=None):
        if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
            raise ValueError("xyz must be a contiguous float32 [n, 3] tensor")
        n = xyz.shape[0]
        c, chp = 0, None
        if ch is not None:
            if ch.dtype != torch.float32 or ch.dim() != 2 or ch.shape[0] != n or not ch.is_contiguous():
                raise ValueError("ch must be a contiguous float32 [n, c] tensor")
            c, chp = ch.shape[1], _dev_ptr(ch, "ch")
        b, nb = _bindings(bind)
        _check(load().mem_input_pointcloud(self._h, _dev_ptr(xyz, "xyz"), n, chp, c, b, nb,
                                           _pose(T), _stream(stream)))

    def input_pointclouds(self, clouds, stream=None):
        """clouds: sequence of (xyz, T) or (xyz, T, ch, bind), each as for
        input_pointcloud; equals input_pointcloud for each in order."""
        arr = (mem_cloud * max(1, len(clouds)))()
        keep = []
        for k, cl in enumerate(clouds):
            xyz, T = cl[0], cl[1]
            ch = cl[2] if len(cl) > 2 else None
            bind = cl[3] if len(cl) > 3 else ()
            if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
                raise ValueError("xyz must be a contiguous float32 [n, 3] tensor")
            c, chp = 0, None
            if ch is not None:
                if ch.dtype != torch.float32 or ch.dim() != 2 or ch.shape[0] != xyz.shape[0] or not ch.is_contiguous():
                    raise ValueError("ch must be a contiguous float32 [n, c] tensor")
                c, chp = ch.shape[1], _dev_ptr(ch, "ch")
            b, nb = _bindings(bind)
            keep.append(b)
            arr[k] = mem_cloud(_dev_ptr(xyz, "xyz"), xyz.shape[0], chp, c, b, nb, _pose(T))
        _check(load().mem_input_pointclouds(self._h, arr, len(clouds), _stream(stream)))

    def input_image(self, img: torch.Tensor, K, T, bind=(), stream=None):
        if img.dim() != 3:
            raise ValueError("img must be [h, w, c] (any strides)")
        if img.dtype == torch.uint8:
            dt = MEM_U8
        elif img.dtype == torch.float32:
            dt = MEM_F32
        else:
            raise ValueError("img must be uint8 or float32")
        h, w, c = img.shape
        st = (C.c_int64 * 3)(*img.stride())
        b, nb = _bindings(bind)
        _check(load().mem_input_image(self._h, _dev_ptr(img, "img"), dt, h, w, c, st,
                                      _floats(K, 4), _pose(T), b, nb, _stream(stream)))

    def input_images(self, images, T, stream=None):
        """images: sequence of (img [h, w, c] tensor, K, bind) taken from one
        camera pose T; equals input_image for each in order."""
        arr = (mem_image * max(1, len(images)))()
        keep = []
        for k, (img, K, bind) in enumerate(images):
            if img.dim() != 3 or img.dtype not in (torch.uint8, torch.float32):
                raise ValueError("images must be uint8 or float32 [h, w, c] tensors")
            b, nb = _bindings(bind)
            keep.append(b)
            h, w, c = img.shape
            arr[k] = mem_image(_dev_ptr(img, "img"), MEM_U8 if img.dtype == torch.uint8 else MEM_F32,
                               h, w, c, (C.c_int64 * 3)(*img.stride()), _floats(K, 4), b, nb)
        _check(load().mem_input_images(self._h, arr, len(images), _pose(T), _stream(stream)))

    def input_image_poses(self, poses, stream=None):
        """poses: sequence of (images, T), images as for input_images; equals
        input_images for each pose in order."""
        flat = [im for images, _ in poses for im in images]
        arr = (mem_image * max(1, len(flat)))()
        keep = []
        for k, (img, K, bind) in enumerate(flat):
            if img.dim() != 3 or img.dtype not in (torch.uint8, torch.float32):
                raise ValueError("images must be uint8 or float32 [h, w, c] tensors")
            b, nb = _bindings(bind)
            keep.append(b)
            h, w, c = img.shape
            arr[k] = mem_image(_dev_ptr(img, "img"), MEM_U8 if img.dtype == torch.uint8 else MEM_F32,
                               h, w, c, (C.c_int64 * 3)(*img.stride()), _floats(K, 4), b, nb)
        counts = (C.c_int32 * max(1, len(poses)))(*[len(images) for images, _ in poses])
        Ts = (C.c_float * (12 * max(1, len(poses))))()
        for p, (_, T) in enumerate(poses):
            for q, v in enumerate(_pose(T)):
                Ts[12 * p + q] = v
        _check(load().mem_input_image_poses(self._h, arr, counts, len(poses), Ts, _stream(stream)))

    # -- read-out -------------------------------------------------------------
    def channels(self, layer: int, view: int = MEM_VIEW_VALUE) -> int:
        if layer < MEM_LAYER_USER0 or layer - MEM_LAYER_USER0 >= len(self.layers):
            return 1  # the library rejects unknown layers
        l = self.layers[layer - MEM_LAYER_USER0]
        if view == MEM_VIEW_ARGMAX or (view == MEM_VIEW_AUX and l.rule == MEM_GAUSS):
            return 1
        return l.channels

    def get_layer(self, layer: int, view: int = MEM_VIEW_VALUE, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
        Cn = self.channels(layer, view)
        if out is None:
            out = torch.empty((self.H, self.W, Cn), dtype=torch.float32, device="cuda")
        _check(load().mem_get_layer(self._h, layer, view, _dev_ptr(out, "out"), _stream(stream)))
        return out if layer >= MEM_LAYER_USER0 else out.reshape(self.H, self.W)

    def set_layer(self, layer: int, view: int, values: torch.Tensor, stream=None):
        v = values.to(device="cuda", dtype=torch.float32).contiguous()
        if v.numel() != self.H * self.W * self.channels(layer, view):
            raise ValueError("values have the wrong size")
        _check(load().mem_set_layer(self._h, layer, view, _dev_ptr(v, "values"), _stream(stream)))
        # `v` may be a temporary copy: keep it alive until the kernel has read it
        (stream or torch.cuda.current_stream()).synchronize()

    def set_drift_compensation(self, enable: bool = True, kappa: float = 3.0, min_points: int = 100):
        _check(load().mem_set_drift_compensation(self._h, 1 if enable else 0, float(kappa), int(min_points)))

    def set_overlap_clearance(self, enable: bool = True, range_xy: float = 4.0, range_z: float = 2.0):
        _check(load().mem_set_overlap_clearance(self._h, 1 if enable else 0, float(range_xy), float(range_z)))

    def pca(self, layer: int, out: torch.Tensor | None = None, stream=None):
        """([H, W, 3] projections on the layer's three leading principal
        components, [3] eigenvalues)."""
        if out is None:
            out = torch.empty((self.H, self.W, 3), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.H * self.W * 3:
            raise ValueError("out must be a contiguous float32 tensor of H x W x 3 elements")
        lam = (C.c_float * 3)()
        _check(load().mem_pca(self._h, layer, _dev_ptr(out, "out"), lam, _stream(stream)))
        return out, list(lam)

    def pca_noalloc(self, layer: int, out: torch.Tensor, eigenvalues: torch.Tensor | None = None, stream=None):
        """mem_pca_noalloc into caller-allocated device tensors: out [H, W, 3]
        float32, eigenvalues [3] float32 or None; nothing waits for the stream."""
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.H * self.W * 3:
            raise ValueError("out must be a contiguous float32 tensor of H x W x 3 elements")
        if eigenvalues is not None and (eigenvalues.dtype != torch.float32 or eigenvalues.numel() != 3
                                        or not eigenvalues.is_contiguous()):
            raise ValueError("eigenvalues must be a contiguous float32 tensor of 3 elements")
        lp = _dev_ptr(eigenvalues, "eigenvalues") if eigenvalues is not None else None
        _check(load().mem_pca_noalloc(self._h, layer, _dev_ptr(out, "out"), lp, _stream(stream)))

    def drift(self, stream=None):
        """(offset applied by the last point cloud, its consistent points)."""
        d, n = C.c_float(), C.c_int32()
        _check(load().mem_get_drift(self._h, C.byref(d), C.byref(n), _stream(stream)))
        return d.value, n.value

    def normals(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """[H, W, 3] surface normals of the heights (NaN on the border and
        next to cells without a height)."""
        if out is None:
            out = torch.empty((self.H, self.W, 3), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.H * self.W * 3:
            raise ValueError("out must be a contiguous float32 tensor of H x W x 3 elements")
        _check(load().mem_normals(self._h, _dev_ptr(out, "out"), _stream(stream)))
        return out

    def center(self):
        cx, cy = C.c_int32(), C.c_int32()
        _check(load().mem_get_center(self._h, C.byref(cx), C.byref(cy)))
        return cx.value, cy.value

    def debug_point_cells(self, xyz: torch.Tensor, T, stream=None) -> torch.Tensor:
        out = torch.empty(xyz.shape[0], dtype=torch.int32, device="cuda")
        _check(load().mem_debug_point_cells(self._h, _dev_ptr(xyz.contiguous(), "xyz"), xyz.shape[0],
                                            _pose(T), _dev_ptr(out, "out"), _stream(stream)))
        return out

    def debug_cell_pixels(self, h: int, w: int, K, T, stream=None) -> torch.Tensor:
        out = torch.empty((self.H, self.W), dtype=torch.int32, device="cuda")
        _check(load().mem_debug_cell_pixels(self._h, h, w, _floats(K, 4), _pose(T),
                                            _dev_ptr(out, "out"), _stream(stream)))
        return out

    def stats(self, stream=None) -> dict:
        s = mem_stats()
        _check(load().mem_get_stats(self._h, C.byref(s), _stream(stream)))
        return {f: getattr(s, f) for f in STAT_FIELDS}

    def reset_stats(self, stream=None):
        _check(load().mem_reset_stats(self._h, _stream(stream)))

    def debug_gather_width(self, width: int):
        """Tests: 1 forces one channel per lane in this map's image gathers,
        0 restores the automatic width."""
        _check(load().mem_debug_gather_width(self._h, width))

    def profile_enable(self, on: bool = True):
        _check(load().mem_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        arr = (mem_kernel_time * 64)()
        n = C.c_int32()
        _check(load().mem_profile_read(self._h, arr, 64, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 64))}


# ---------------------------------------------------------------------------
# Batches of maps (mem_batch_*)
# ---------------------------------------------------------------------------

class mem_batch_params(C.Structure):
    _fields_ = [("n_maps", C.c_int32), ("width", C.POINTER(C.c_int32)), ("height", C.POINTER(C.c_int32)),
                ("resolution", C.c_float), ("noise_c0", C.c_float), ("noise_c1", C.c_float),
                ("max_range", C.c_float), ("clear_margin", C.c_float), ("clear_min_count", C.c_int32),
                ("min_depth", C.c_float), ("n_layers", C.c_int32), ("layers", C.POINTER(mem_layer_desc)),
                ("max_points", C.c_int64), ("cam_h", C.c_int32), ("cam_w", C.c_int32), ("cam_c", C.c_int32),
                ("cam_dtype", C.c_int32), ("n_img_bind", C.c_int32), ("img_bind", C.POINTER(mem_binding))]


class mem_batch_input(C.Structure):
    _fields_ = [("robot_xy", C.c_void_p), ("xyz", C.c_void_p), ("offsets", C.c_void_p),
                ("T_map_sensor", C.c_void_p), ("images", C.c_void_p), ("K", C.c_void_p),
                ("T_map_cam", C.c_void_p)]


class mem_batch_tuning(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("wg_per_cu", C.c_int32), ("tile", C.c_int32), ("graph", C.c_int32),
                ("step_ms", C.c_double)]


BATCH_SYMBOLS = ("mem_batch_create", "mem_batch_destroy", "mem_batch_step", "mem_batch_tune",
                 "mem_batch_set_tuning", "mem_batch_get_tuning", "mem_batch_get_layer",
                 "mem_batch_set_layer", "mem_batch_get_center", "mem_batch_get_stats",
                 "mem_batch_reset_stats", "mem_batch_profile_enable", "mem_batch_profile_read")


def _load_batch():
    L = load()
    if getattr(L, "_batch_ready", False):
        return L
    P, I32 = C.c_void_p, C.c_int32
    sig = {
        "mem_batch_create": [C.POINTER(mem_batch_params), P, C.POINTER(P)],
        "mem_batch_destroy": [P, P],
        "mem_batch_step": [P, C.POINTER(mem_batch_input), P],
        "mem_batch_tune": [P, C.POINTER(mem_batch_input), P],
        "mem_batch_set_tuning": [P, C.POINTER(mem_batch_tuning)],
        "mem_batch_get_tuning": [P, C.POINTER(mem_batch_tuning)],
        "mem_batch_get_layer": [P, I32, I32, I32, P, P],
        "mem_batch_set_layer": [P, I32, I32, I32, P, P],
        "mem_batch_get_center": [P, I32, C.POINTER(I32), C.POINTER(I32)],
        "mem_batch_get_stats": [P, C.POINTER(mem_stats), P],
        "mem_batch_reset_stats": [P, P],
        "mem_batch_profile_enable": [P, I32],
        "mem_batch_profile_read": [P, C.POINTER(mem_kernel_time), I32, C.POINTER(I32)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    L._batch_ready = True
    return L


def _host_f32(a, n):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
    if a.size != n:
        raise ValueError(f"expected {n} floats, got {a.size}")
    return a


class Batch:
    """Independent maps of different sizes updated together (mem_batch_*)."""

    def __init__(self, widths, heights, resolution, layers=(), max_points=0, cam=None, img_bind=(),
                 noise_c0=0.01, noise_c1=0.001, max_range=100.0, clear_margin=0.05, clear_min_count=1,
                 min_depth=0.1, stream=None):
        L = _load_batch()
        self.n = len(widths)
        self.W = [int(w) for w in widths]
        self.H = [int(h) for h in heights]
        self.layers = [l if isinstance(l, Layer) else Layer(*l) for l in layers]
        self._w = (C.c_int32 * self.n)(*self.W)
        self._h = (C.c_int32 * self.n)(*self.H)
        descs = (mem_layer_desc * max(1, len(self.layers)))()
        for i, l in enumerate(self.layers):
            descs[i] = mem_layer_desc(l.channels, l.rule, l.storage, l.param, None)
        ib, nib = _bindings(img_bind)
        ch, cw, cc, cd = cam if cam is not None else (0, 0, 0, MEM_F32)
        self.cam = cam
        p = mem_batch_params(self.n, self._w, self._h, resolution, noise_c0, noise_c1, max_range, clear_margin,
                             clear_min_count, min_depth, len(self.layers), descs, int(max_points), ch, cw, cc, cd,
                             nib, ib)
        self._keep = (descs, ib)
        h = C.c_void_p()
        _check(L.mem_batch_create(C.byref(p), _stream(stream), C.byref(h)))
        self._b = h

    def close(self, stream=None):
        if getattr(self, "_b", None):
            _load_batch().mem_batch_destroy(self._b, _stream(stream))
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _input(self, robot_xy, xyz, offsets, T, images=None, K=None, T_cam=None):
        import numpy as np
        n = self.n
        self._in_keep = [
            _host_f32(robot_xy, 2 * n),
            np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1)),
            _host_f32(T, 12 * n),
        ]
        if self._in_keep[1].size != n + 1:
            raise ValueError("offsets must have n_maps + 1 entries")
        if xyz.dtype != torch.float32 or not xyz.is_contiguous() or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must be a contiguous float32 [n, 3] device tensor")
        img_p = None
        if images is not None:
            if not images.is_contiguous():
                raise ValueError("images must be contiguous [n_maps, h, w, c]")
            img_p = _dev_ptr(images, "images").value
            self._in_keep += [_host_f32(K, 4 * n), _host_f32(T_cam, 12 * n)]
        k = self._in_keep
        ptr = lambda a: a.ctypes.data_as(C.c_void_p).value
        return mem_batch_input(ptr(k[0]), _dev_ptr(xyz, "xyz").value if xyz.numel() else None, ptr(k[1]),
                               ptr(k[2]), img_p, ptr(k[3]) if images is not None else None,
                               ptr(k[4]) if images is not None else None)

    def step(self, robot_xy, xyz, offsets, T, images=None, K=None, T_cam=None, stream=None):
        inp = self._input(robot_xy, xyz, offsets, T, images, K, T_cam)
        _check(_load_batch().mem_batch_step(self._b, C.byref(inp), _stream(stream)))

    def tune(self, robot_xy, xyz, offsets, T, images=None, K=None, T_cam=None, stream=None):
        inp = self._input(robot_xy, xyz, offsets, T, images, K, T_cam)
        _check(_load_batch().mem_batch_tune(self._b, C.byref(inp), _stream(stream)))
        return self.tuning()

    def tuning(self) -> dict:
        t = mem_batch_tuning()
        _check(_load_batch().mem_batch_get_tuning(self._b, C.byref(t)))
        return {f: getattr(t, f) for f, _ in mem_batch_tuning._fields_}

    def set_tuning(self, chunk, wg_per_cu, tile, graph=1):
        t = mem_batch_tuning(chunk, wg_per_cu, tile, graph, 0.0)
        _check(_load_batch().mem_batch_set_tuning(self._b, C.byref(t)))

    def channels(self, layer, view=MEM_VIEW_VALUE):
        if layer < MEM_LAYER_USER0 or layer - MEM_LAYER_USER0 >= len(self.layers):
            return 1
        l = self.layers[layer - MEM_LAYER_USER0]
        if view == MEM_VIEW_ARGMAX or (view == MEM_VIEW_AUX and l.rule == MEM_GAUSS):
            return 1
        return l.channels

    def get_layer(self, m, layer, view=MEM_VIEW_VALUE, stream=None):
        Cn = self.channels(layer, view)
        out = torch.empty((self.H[m], self.W[m], Cn), dtype=torch.float32, device="cuda")
        _check(_load_batch().mem_batch_get_layer(self._b, m, layer, view, _dev_ptr(out, "out"), _stream(stream)))
        return out if layer >= MEM_LAYER_USER0 else out.reshape(self.H[m], self.W[m])

    def set_layer(self, m, layer, view, values, stream=None):
        v = values.to(device="cuda", dtype=torch.float32).contiguous()
        _check(_load_batch().mem_batch_set_layer(self._b, m, layer, view, _dev_ptr(v, "values"), _stream(stream)))
        (stream or torch.cuda.current_stream()).synchronize()

    def center(self, m):
        cx, cy = C.c_int32(), C.c_int32()
        _check(_load_batch().mem_batch_get_center(self._b, m, C.byref(cx), C.byref(cy)))
        return cx.value, cy.value

    def stats(self, stream=None) -> dict:
        s = mem_stats()
        _check(_load_batch().mem_batch_get_stats(self._b, C.byref(s), _stream(stream)))
        return {f: getattr(s, f) for f in STAT_FIELDS}

    def reset_stats(self, stream=None):
        _check(_load_batch().mem_batch_reset_stats(self._b, _stream(stream)))

    def profile_enable(self, on: bool = True):
        """While on, steps launch their stages directly with events around each."""
        _check(_load_batch().mem_batch_profile_enable(self._b, 1 if on else 0))

    def profile_read(self) -> dict:
        """{stage: (launches, total_ms)} since the last read."""
        arr = (mem_kernel_time * 64)()
        n = C.c_int32()
        _check(_load_batch().mem_batch_profile_read(self._b, arr, 64, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 64))}


UNET_SYMBOLS = ("mem_unet_num_params", "mem_unet_create", "mem_unet_destroy", "mem_unet_set_params",
                "mem_unet_get_params", "mem_unet_save", "mem_unet_load", "mem_unet_forward",
                "mem_unet_loss_grad", "mem_unet_train_step", "mem_unet_input", "mem_unet_complete",
                "mem_unet_profile_enable", "mem_unet_profile_read", "mem_complete", "mem_unet_debug_tiles")


def _load_unet():
    L = load()
    if getattr(L, "_unet_ready", False):
        return L
    P, I32, F = C.c_void_p, C.c_int32, C.c_float
    sig = {
        "mem_unet_create": [I32, I32, I32, C.c_uint64, F, P, C.POINTER(P)],
        "mem_unet_destroy": [P, P],
        "mem_unet_set_params": [P, P, P],
        "mem_unet_get_params": [P, P, P],
        "mem_unet_save": [P, C.c_char_p, P],
        "mem_unet_load": [P, C.c_char_p, P],
        "mem_unet_forward": [P, P, I32, P, P],
        "mem_unet_loss_grad": [P, P, P, P, I32, P, P, P],
        "mem_unet_train_step": [P, P, P, P, I32, F, P, P],
        "mem_unet_input": [P, P, I32, I32, F, P, P],
        "mem_unet_complete": [P, P, I32, F, F, P, P, P],
        "mem_complete": [P, P, F, F, P, P, P],
        "mem_unet_profile_enable": [P, I32],
        "mem_unet_debug_tiles": [P, I32],
        "mem_unet_profile_read": [P, C.POINTER(mem_kernel_time), I32, C.POINTER(I32)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    L.mem_unet_num_params.argtypes = [I32]
    L.mem_unet_num_params.restype = C.c_int64
    L._unet_ready = True
    return L


def unet_num_params(base: int) -> int:
    return int(_load_unet().mem_unet_num_params(int(base)))


class UNet:
    """The completion network (mem_unet_*): NHWC FP32 device tensors in and out."""

    def __init__(self, base=32, max_batch=1, size=256, seed=0, sigma0=0.3, stream=None):
        L = _load_unet()
        self.base, self.max_batch, self.size = int(base), int(max_batch), int(size)
        self.n_params = unet_num_params(base)
        h = C.c_void_p()
        _check(L.mem_unet_create(self.base, self.max_batch, self.size, int(seed), float(sigma0), _stream(stream),
                                 C.byref(h)))
        self._u = h

    def close(self, stream=None):
        if getattr(self, "_u", None):
            _load_unet().mem_unet_destroy(self._u, _stream(stream))
            self._u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _x(self, x, ch, what):
        if (x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 4 or x.shape[1] != self.size
                or x.shape[2] != self.size or x.shape[3] != ch):
            raise ValueError(f"{what} must be a contiguous float32 [B, {self.size}, {self.size}, {ch}] tensor")
        return _dev_ptr(x, what)

    def _tm(self, t, B, what):
        if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (B, self.size, self.size):
            raise ValueError(f"{what} must be a contiguous float32 [B, size, size] tensor")
        return _dev_ptr(t, what)

    def params(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_load_unet().mem_unet_get_params(self._u, _dev_ptr(out, "params"), _stream(stream)))
        return out

    def set_params(self, p, stream=None):
        p = p.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1)
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(_load_unet().mem_unet_set_params(self._u, _dev_ptr(p, "params"), _stream(stream)))
        (stream or torch.cuda.current_stream()).synchronize()

    def profile_enable(self, on=True):
        _check(_load_unet().mem_unet_profile_enable(self._u, 1 if on else 0))

    def debug_tiles(self, shape: int):
        """Force the tile shape of every nt product (0-3; -1 automatic)."""
        _check(_load_unet().mem_unet_debug_tiles(self._u, int(shape)))

    def profile_read(self) -> dict:
        """{name: (launches, total_ms)} since the last read."""
        arr = (mem_kernel_time * 64)()
        n = C.c_int32()
        _check(_load_unet().mem_unet_profile_read(self._u, arr, 64, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 64))}

    def save(self, path, stream=None):
        _check(_load_unet().mem_unet_save(self._u, os.fsencode(path), _stream(stream)))

    def load(self, path, stream=None):
        _check(_load_unet().mem_unet_load(self._u, os.fsencode(path), _stream(stream)))

    def forward(self, x, stream=None) -> torch.Tensor:
        B = x.shape[0]
        out = torch.empty((B, self.size, self.size, 2), dtype=torch.float32, device="cuda")
        _check(_load_unet().mem_unet_forward(self._u, self._x(x, 3, "x"), B, _dev_ptr(out, "out"),
                                             _stream(stream)))
        return out

    def loss_grad(self, x, target, mask, stream=None):
        B = x.shape[0]
        grad = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(_load_unet().mem_unet_loss_grad(self._u, self._x(x, 3, "x"), self._tm(target, B, "target"),
                                               self._tm(mask, B, "mask"), B,
                                               _dev_ptr(grad, "grad"), _dev_ptr(loss, "loss"), _stream(stream)))
        return loss, grad

    def train_step(self, x, target, mask, lr, loss_out=None, stream=None):
        B = x.shape[0]
        lp = _dev_ptr(loss_out, "loss") if loss_out is not None else None
        _check(_load_unet().mem_unet_train_step(self._u, self._x(x, 3, "x"), self._tm(target, B, "target"),
                                                self._tm(mask, B, "mask"), B, float(lr),
                                                lp, _stream(stream)))

    def complete_windows(self, x, z_ref, sigma_max, stream=None):
        """(height, sigma) [B, size, size] of prepared windows x (mem_unet_complete)."""
        B = x.shape[0]
        out_h = torch.empty((B, self.size, self.size), dtype=torch.float32, device="cuda")
        out_s = torch.empty_like(out_h)
        _check(_load_unet().mem_unet_complete(self._u, self._x(x, 3, "x"), B, float(z_ref), float(sigma_max),
                                              _dev_ptr(out_h, "out_h"), _dev_ptr(out_s, "out_sigma"),
                                              _stream(stream)))
        return out_h, out_s

    def complete(self, m: "Map", z_ref, sigma_max, stream=None):
        """(height, sigma) [H, W] of the map completed by the network (mem_complete)."""
        out_h = torch.empty((m.H, m.W), dtype=torch.float32, device="cuda")
        out_s = torch.empty((m.H, m.W), dtype=torch.float32, device="cuda")
        _check(_load_unet().mem_complete(m._h, self._u, float(z_ref), float(sigma_max), _dev_ptr(out_h, "out_h"),
                                         _dev_ptr(out_s, "out_sigma"), _stream(stream)))
        return out_h, out_s


def unet_input(h: torch.Tensor, v: torch.Tensor, z_ref, out: torch.Tensor | None = None, stream=None):
    """Network input [H, W, 3] of one window from its height / variance layers
    (mem_unet_input)."""
    if h.shape != v.shape or h.dim() != 2 or h.dtype != torch.float32 or v.dtype != torch.float32:
        raise ValueError("h and v must be float32 [H, W] tensors of one shape")
    h, v = h.contiguous(), v.contiguous()
    H, W = h.shape
    if out is None:
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    if tuple(out.shape) != (H, W, 3) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [H, W, 3] tensor")
    _check(_load_unet().mem_unet_input(_dev_ptr(h, "h"), _dev_ptr(v, "v"), W, H, float(z_ref), _dev_ptr(out, "x"),
                                       _stream(stream)))
    return out
