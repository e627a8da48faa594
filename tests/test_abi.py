"""The C ABI library loads, exports every entry point include/mem.h declares,
and rejects invalid arguments on the host before touching the device.  The
oracle and the GPU path share no source.  CPU only (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header=None):
    inc = os.path.join(ROOT, "include")
    names = [header] if header else sorted(f for f in os.listdir(inc) if f.endswith(".h"))
    text = "".join(open(os.path.join(inc, f)).read() for f in names)
    return sorted(set(re.findall(r"^\s*(?:mem_status|const char\*|int64_t|int)\s+(mem_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mem_create", "mem_destroy", "mem_move", "mem_input_pointcloud",
              "mem_input_image", "mem_get_layer"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2309_16818_amd import mem
    lib = mem.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert sorted(mem.SYMBOLS + mem.BATCH_SYMBOLS + mem.UNET_SYMBOLS + mem.CALIB_SYMBOLS) == declared_symbols()
    assert sorted(mem.CALIB_SYMBOLS) == declared_symbols("mem_calib.h")


def test_calibration_kernels_reject_bad_arguments():
    from paper_2309_16818_amd import mem
    lib = mem.load()
    assert lib.mem_calib_copy(None, None, 16, None) == -1
    assert lib.mem_calib_copy(C.c_void_p(16), C.c_void_p(32), 15, None) == -1
    assert lib.mem_calib_copy(C.c_void_p(8), C.c_void_p(32), 16, None) == -1
    assert lib.mem_calib_atomic(C.c_void_p(64), mem.MEM_CALIB_F32, mem.MEM_CALIB_SCATTER, 10, 12, None) == -1
    assert lib.mem_calib_atomic(C.c_void_p(64), mem.MEM_CALIB_F32, mem.MEM_CALIB_SCATTER, 20, 16, None) == -1
    assert lib.mem_calib_atomic(C.c_void_p(64), mem.MEM_CALIB_I32, mem.MEM_CALIB_UNIQUE, 20, 16, None) == -1
    assert lib.mem_calib_atomic(C.c_void_p(64), 7, mem.MEM_CALIB_UNIQUE, 1, 1, None) == -1
    assert lib.mem_calib_atomic(C.c_void_p(64), mem.MEM_CALIB_I32, 9, 1, 1, None) == -1
    assert b"pattern" in lib.mem_calib_last_error()


def test_struct_layouts_match_the_header():
    from paper_2309_16818_amd import mem
    assert C.sizeof(mem.mem_layer_desc) == 24
    assert mem.mem_layer_desc.ch_scale.offset == 16
    assert C.sizeof(mem.mem_params) == 48
    assert mem.mem_params.layers.offset == 40
    assert C.sizeof(mem.mem_binding) == 16 and mem.mem_binding.topk.offset == 12
    assert C.sizeof(mem.mem_stats) == 8 * len(mem.STAT_FIELDS)
    assert C.sizeof(mem.mem_kernel_time) == 48
    assert C.sizeof(mem.mem_image) == 80
    assert C.sizeof(mem.mem_batch_params) == 104 and mem.mem_batch_params.max_points.offset == 64
    assert C.sizeof(mem.mem_batch_input) == 56 and C.sizeof(mem.mem_batch_tuning) == 24
    assert mem.mem_image.strides.offset == 24 and mem.mem_image.bind.offset == 64


def _params(**kw):
    from paper_2309_16818_amd import mem
    d = dict(width=10, height=10, resolution=0.1, noise_c0=0.01, noise_c1=0.001, max_range=10.0,
             clear_margin=0.05, clear_min_count=1, min_depth=0.1, n_layers=0, layers=None)
    d.update(kw)
    return mem.mem_params(**d)


@pytest.mark.parametrize("kw,msg", [
    (dict(width=0), "grid"), (dict(height=20000), "grid"), (dict(resolution=0.0), "resolution"),
    (dict(resolution=float("nan")), "resolution"), (dict(noise_c0=0.0, noise_c1=0.0), "noise"),
    (dict(max_range=-1.0), "max_range"), (dict(clear_min_count=-1), "clearing"),
    (dict(n_layers=3), "n_layers"),
])
def test_create_rejects_bad_parameters_on_the_host(kw, msg):
    from paper_2309_16818_amd import mem
    lib = mem.load()
    p = _params(**kw)
    h = C.c_void_p()
    assert lib.mem_create(C.byref(p), None, C.byref(h)) == mem.MEM_E_ARG
    assert msg in lib.mem_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("layer,msg", [
    ((0, 0, 0, 1.0), "channels"), ((4, 7, 0, 1.0), "rule"), ((4, 0, 9, 1.0), "storage"),
    ((4, 3, 1, 1.0), "Dirichlet"), ((4, 1, 0, 1.5), "weight"), ((4, 2, 0, -1.0), "positive"),
])
def test_create_rejects_bad_layers(layer, msg):
    from paper_2309_16818_amd import mem
    lib = mem.load()
    arr = (mem.mem_layer_desc * 1)(mem.mem_layer_desc(*layer, None))
    p = _params(n_layers=1, layers=arr)
    h = C.c_void_p()
    assert lib.mem_create(C.byref(p), None, C.byref(h)) == mem.MEM_E_ARG
    assert msg in lib.mem_last_error().decode()


def test_null_handles_are_rejected():
    from paper_2309_16818_amd import mem
    lib = mem.load()
    T = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    assert lib.mem_move(None, 0.0, 0.0, None) == mem.MEM_E_ARG
    assert lib.mem_input_pointcloud(None, None, 0, None, 0, None, 0, T, None) == mem.MEM_E_ARG
    assert lib.mem_get_layer(None, 0, 0, None, None) == mem.MEM_E_ARG
    assert lib.mem_normals(None, None, None) == mem.MEM_E_ARG
    assert lib.mem_set_drift_compensation(None, 1, 3.0, 10) == mem.MEM_E_ARG
    assert lib.mem_get_drift(None, None, None, None) == mem.MEM_E_ARG
    assert lib.mem_set_overlap_clearance(None, 1, 4.0, 2.0) == mem.MEM_E_ARG
    assert lib.mem_pca(None, 8, None, None, None) == mem.MEM_E_ARG
    assert lib.mem_pca_noalloc(None, 8, None, None, None) == mem.MEM_E_ARG
    assert lib.mem_input_image_poses(None, None, None, 2, None, None) == mem.MEM_E_ARG
    assert lib.mem_destroy(None, None) == mem.MEM_OK


def test_unet_host_checks():
    """Parameter count agrees with the oracle's layout; bad sizes and NULL
    handles are rejected before any device work."""
    import oracle as O
    from paper_2309_16818_amd import mem
    lib = mem._load_unet()
    for base in (1, 2, 4, 32):
        assert lib.mem_unet_num_params(base) == O.unet_num_params(base)
    assert lib.mem_unet_num_params(0) == -1
    h = C.c_void_p()
    for args in ((0, 1, 16, 0.3), (32, 0, 256, 0.3), (32, 1, 12, 0.3), (32, 1, 4, 0.3), (32, 1, 8192, 0.3),
                 (257, 1, 16, 0.3), (4, 1, 16, 0.0), (4, 1, 16, float("nan"))):
        assert lib.mem_unet_create(*args[:3], 0, args[3], None, C.byref(h)) == mem.MEM_E_ARG, args
        assert not h.value
    assert lib.mem_unet_forward(None, None, 1, None, None) == mem.MEM_E_ARG
    assert lib.mem_unet_train_step(None, None, None, None, 1, 1e-3, None, None) == mem.MEM_E_ARG
    assert lib.mem_unet_loss_grad(None, None, None, None, 1, None, None, None) == mem.MEM_E_ARG
    assert lib.mem_complete(None, None, 0.0, 0.05, None, None, None) == mem.MEM_E_ARG
    assert lib.mem_unet_destroy(None, None) == mem.MEM_OK


def test_oracle_and_gpu_path_share_no_source():
    """Neither side includes or imports the other."""
    gpu_dir = os.path.join(ROOT, "paper_2309_16818_amd")
    orc_dir = os.path.join(ROOT, "oracle")
    for d, other in ((gpu_dir, "oracle"), (orc_dir, "paper_2309_16818_amd")):
        for base, _, files in os.walk(d):
            for f in files:
                if f.endswith((".py", ".c", ".h", ".hip", ".cpp")):
                    text = open(os.path.join(base, f)).read()
                    assert not re.search(rf"(import|from|#include)\s+[\"<]?[./]*{other}", text), (f, other)
    # the oracle sources are plain C: no HIP
    src = open(os.path.join(orc_dir, "mem_oracle.c")).read()
    assert "hip" not in src.lower().replace("ship", "")


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2309_16818_amd")
    for base, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                assert "oracle" not in re.findall(r"^\s*(?:import|from)\s+(\w+)",
                                                  open(os.path.join(base, f)).read(), re.M)
