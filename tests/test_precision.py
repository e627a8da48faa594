"""Reduced-precision layer storage (BF16, FP8 E4M3 with per-channel scales):
codecs against torch's own conversions, every E4M3 code round-trips, and a
fused update stays within one storage rounding of the binary64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from lockstep import gpu_layer, make_pair, sync_from_oracle, to_dev
from paper_2309_16818_amd import mem, synth

pytestmark = pytest.mark.gpu


def roundtrip(storage, values, scale=None):
    C = values.shape[-1]
    g = mem.Map(mem.MapParams(values.shape[1], values.shape[0], 0.1,
                              layers=[mem.Layer(C, mem.MEM_LATEST, 0.0, storage, scale)]))
    g.set_layer(8, 0, torch.tensor(values, dtype=torch.float32))
    out = gpu_layer(g, 8, 0)
    g.close()
    return out


def test_bf16_storage_rounds_to_nearest_even_like_torch():
    rng = np.random.default_rng(0)
    v = (rng.standard_normal((16, 16, 8)) * np.exp(rng.uniform(-20, 20, (16, 16, 8)))).astype(np.float32)
    v[0, 0, :4] = [0.0, -0.0, np.inf, -np.inf]
    want = torch.tensor(v).to(torch.bfloat16).float().numpy()
    got = roundtrip(mem.MEM_BF16, v)
    assert np.array_equal(got, want)


def test_every_e4m3_code_round_trips():
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    v = codes.reshape(16, 16, 1).astype(np.float32)
    got = roundtrip(mem.MEM_FP8_E4M3, v, scale=[448.0])  # amax 448 -> scale 1
    assert np.array_equal(got, v, equal_nan=True)
    assert np.isnan(got).sum() == 2  # 0x7F and 0xFF


def test_fp8_storage_matches_torch_e4m3_with_saturation_and_scales():
    rng = np.random.default_rng(1)
    C = 6
    amax = np.array([1.0, 0.5, 4.0, 100.0, 1e-3, 448.0], np.float32)
    v = (rng.standard_normal((12, 10, C)) * amax * 0.6).astype(np.float32)
    v[0, 0] = amax * 3.0   # saturates
    v[0, 1] = -amax * 3.0
    s = (amax / 448.0).astype(np.float32)
    q = np.clip(v / s, -448, 448)
    want = (torch.tensor(q).to(torch.float8_e4m3fn).float().numpy() * s).astype(np.float32)
    got = roundtrip(mem.MEM_FP8_E4M3, v, scale=list(amax))
    assert np.array_equal(got, want)


def test_fp8_encoder_on_a_sweep_of_all_binary32_patterns():
    """Every 64th binary32 bit pattern (both signs, every binade, zeros,
    subnormals, infinities, NaNs and the rounding ties of every binade),
    stored with scale 1 (amax 448), reads back as torch's E4M3 conversion
    after saturation at +-448."""
    u = np.arange(0, 2 ** 32, 64, dtype=np.uint64).astype(np.uint32)
    v = u.view(np.float32).reshape(8192, 8192, 1)
    want = torch.from_numpy(np.clip(v, -448.0, 448.0)).to(torch.float8_e4m3fn).float().numpy()
    g = mem.Map(mem.MapParams(8192, 8192, 0.1, layers=[mem.Layer(1, mem.MEM_LATEST, 0.0, mem.MEM_FP8_E4M3, [448.0])]))
    g.set_layer(8, 0, torch.from_numpy(v))
    got = g.get_layer(8).cpu().numpy().reshape(8192, 8192, 1)
    g.close()
    assert np.array_equal(got, want, equal_nan=True)


@pytest.mark.parametrize("C", [48, 200, 384])
@pytest.mark.parametrize("storage,rel", [(mem.MEM_F32, 1e-4), (mem.MEM_BF16, 2.0 ** -8), (mem.MEM_FP8_E4M3, 2.0 ** -3)])
def test_feature_fusion_within_one_storage_rounding(storage, rel, C):
    """One image update from the same state on both sides: the GPU result
    differs from the binary64 oracle by at most the storage rounding (plus
    binary32 arithmetic), per channel, relative to the layer's scale.  The
    widths span one pass of a pair's lanes over the channels (48), a ragged
    last pass (200) and the 384-channel feature layer of the precision
    workload (six passes of 64 lanes)."""
    rng = np.random.default_rng(2 + C)
    layers = [(C, mem.MEM_GAUSS, 1.0, storage), (C, mem.MEM_EXPAVG, 0.5, storage)]
    g, o = make_pair(48, 48, 0.05, layers=layers)
    h = np.where(rng.uniform(size=(48, 48)) < 0.9, rng.normal(0, 0.05, (48, 48)), np.nan)
    o.set_layer(O.LAYER_ELEVATION, 0, h)
    o.set_layer(O.LAYER_VARIANCE, 0, np.full((48, 48), 1e-3))
    K = (60.0, 60.0, 47.5, 35.5)
    for it in range(4):
        img = synth.feature_image(rng, 72, 96, 2 * C)
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(40)).astype(np.float32)
        T = np.zeros((3, 4), np.float32)
        T[:, :3] = R
        T[:, 3] = (rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.8)
        sync_from_oracle(g, o)
        g.input_image(to_dev(img), K, T, bind=[(8, 0, C), (9, C, C)])
        o.input_image(img, K, T, bind=[(8, 0, C), (9, C, C)])
        for lid in (8, 9):
            a, b = gpu_layer(g, lid), o.get_layer(lid)
            ok = ~np.isnan(b)
            assert np.array_equal(np.isnan(a), np.isnan(b))
            # unit-norm features: channel values are O(1/sqrt(C)); bound the
            # error by the storage rounding of the value plus the FP8
            # subnormal quantum of the default scale (1/448 * 2^-9)
            err = np.abs(a[ok] - b[ok])
            bound = rel * np.abs(b[ok]) + (1e-6 if storage != mem.MEM_FP8_E4M3 else 2.0 ** -9 / 448 + 1e-6)
            assert (err <= bound).all(), (storage, lid, float((err - bound).max()))


@pytest.mark.parametrize("C", [20, 64, 200, 384])
@pytest.mark.parametrize("storage", [mem.MEM_F32, mem.MEM_BF16, mem.MEM_FP8_E4M3])
def test_vector_gather_writes_the_one_channel_bits(storage, C):
    """The image gather with 16 bytes of storage per lane (4 FP32, 8 BF16 or
    16 FP8 channels) and the gather with one channel per lane put every
    element through the same arithmetic, so two maps fed the same images,
    one of them forced to one channel, hold the same layer bits: Gaussian and
    averaging rules, float and u8 images, widths that take the vector path
    (multiples of its channels per lane) and widths that fall back to one
    channel (20 channels in BF16 / FP8, 200 in FP8)."""
    rng = np.random.default_rng(40 + C + 7 * storage)
    scales = list(rng.uniform(0.2, 3.0, C).astype(np.float32)) if storage == mem.MEM_FP8_E4M3 else None
    _gather_bits_equal(rng, storage, C, scales, 3.0)


@pytest.mark.parametrize("C", [64, 384])
@pytest.mark.parametrize("spread", ["wide", "outside"])
def test_fp8_vector_gather_bits_on_scales_of_every_range(C, spread):
    """The vector gather divides by an FP8 scale through its binary32
    reciprocal and one correction step, which gives the correctly rounded
    quotient for scales from 2^-60 to 2^60; the one-channel gather divides.
    Scales whose exponents spread over 2^-55 .. 2^55 (quotients that flush
    to zero, saturate, and everything between) give the same bits on both;
    so does a layer with one scale outside the range ("outside": 2^-70),
    which takes the one-channel gather."""
    rng = np.random.default_rng(70 + C + (spread == "outside"))
    amax = 448.0 * np.exp2(rng.uniform(-55, 55, C)) * rng.uniform(1.0, 2.0, C)
    if spread == "outside":
        amax[C // 2] = 448.0 * 2.0 ** -70
    _gather_bits_equal(rng, mem.MEM_FP8_E4M3, C, list(amax.astype(np.float32)), 3.0)


def _gather_bits_equal(rng, storage, C, scales, gain):
    """Two maps fed the same four images, one forced to one channel per lane,
    hold the same bits in both layers and views."""
    maps = []
    for width in (0, 1):
        m = mem.Map(mem.MapParams(48, 48, 0.05, layers=[mem.Layer(C, mem.MEM_GAUSS, 1.0, storage, scales),
                                                         mem.Layer(C, mem.MEM_EXPAVG, 0.5, storage, scales)]))
        m.debug_gather_width(width)
        maps.append(m)
    h = np.where(rng.uniform(size=(48, 48)) < 0.9, rng.normal(0, 0.05, (48, 48)), np.nan).astype(np.float32)
    for m in maps:
        m.set_layer(mem.MEM_LAYER_ELEVATION, 0, torch.tensor(h))
        m.set_layer(mem.MEM_LAYER_VARIANCE, 0, torch.full((48, 48), 1e-3))
    K = (60.0, 60.0, 47.5, 35.5)
    for it in range(4):
        if it % 2:
            img = torch.tensor(rng.integers(0, 256, (72, 96, 2 * C)), dtype=torch.uint8, device="cuda")
        else:
            img = to_dev(synth.feature_image(rng, 72, 96, 2 * C) * gain)
        R = synth.camera_rotation(rng.uniform(0, 2 * np.pi), math.radians(40)).astype(np.float32)
        T = np.zeros((3, 4), np.float32)
        T[:, :3] = R
        T[:, 3] = (rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.8)
        for m in maps:
            m.input_image(img, K, T, bind=[(8, 0, C), (9, C, C)])
    for lid, view in ((8, 0), (8, 1), (9, 0)):
        a, b = gpu_layer(maps[0], lid, view), gpu_layer(maps[1], lid, view)
        assert np.isfinite(a).any()
        assert np.array_equal(a, b, equal_nan=True), (lid, view)
    for m in maps:
        m.close()
