"""Pins of the U-Net oracle (learned completion): forward and gradient
against torch's own binary64 convolution / pooling / transposed convolution
with autograd (an independent implementation), and central finite
differences.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle as O

SPEC = None


def spec(base, cin=3, cout=2):
    c = [base, 2 * base, 4 * base, 8 * base]
    L, prev = [], cin
    for l in range(4):
        L += [(9, prev, c[l]), (9, c[l], c[l])]
        prev = c[l]
    for l in (2, 1, 0):
        L += [(4, c[l + 1], c[l]), (9, 2 * c[l], c[l]), (9, c[l], c[l])]
    L.append((1, base, cout))
    return L


def torch_unet(p, x, base):
    """The same network with torch.nn.functional (NCHW inside)."""
    L = spec(base)
    offs = O.unet_layer_offsets(base)
    assert len(offs) == len(L)

    def wb(i):
        taps, ci, co = L[i]
        o = int(offs[i])
        w = p[o:o + taps * ci * co].view(taps, ci, co)
        b = p[o + taps * ci * co:o + taps * ci * co + co]
        return w, b

    def conv3(i, a):
        w, b = wb(i)
        ci, co = w.shape[1], w.shape[2]
        return F.conv2d(a, w.view(3, 3, ci, co).permute(3, 2, 0, 1), b, padding=1)

    def up(i, a):
        w, b = wb(i)
        ci, co = w.shape[1], w.shape[2]
        return F.conv_transpose2d(a, w.view(2, 2, ci, co).permute(2, 3, 0, 1), b, stride=2)

    a = x.permute(0, 3, 1, 2)
    enc = []
    for l in range(4):
        a = F.relu(conv3(2 * l + 1, F.relu(conv3(2 * l, a))))
        enc.append(a)
        if l < 3:
            a = F.max_pool2d(a, 2)
    d = enc[3]
    for j, l in enumerate((2, 1, 0)):
        k = 8 + 3 * j
        d = torch.cat([up(k, d), enc[l]], 1)
        d = F.relu(conv3(k + 2, F.relu(conv3(k + 1, d))))
    w, b = wb(17)
    out = F.conv2d(d, w.view(w.shape[1], w.shape[2]).t()[:, :, None, None], b)
    return out.permute(0, 2, 3, 1)


def nll(out, t, m):
    h, s = out[..., 0], out[..., 1]
    msk = m > 0
    cnt = max(int(msk.sum()), 1)
    return (0.5 * (s + (t - h) ** 2 * torch.exp(-s)))[msk].sum() / cnt


def sample(base, B, S, seed):
    rng = np.random.default_rng(seed)
    n = O.unet_num_params(base)
    p = rng.normal(0, 0.3, n)
    offs = list(O.unet_layer_offsets(base)) + [n]
    for i, (taps, ci, co) in enumerate(spec(base)):  # fan-in scaling keeps activations O(1)
        p[offs[i]:offs[i + 1]] *= np.sqrt(2.0 / (taps * ci)) / 0.3
    x = rng.normal(0, 1, (B, S, S, 3))
    t = rng.normal(0, 1, (B, S, S))
    m = (rng.uniform(size=(B, S, S)) < 0.7).astype(np.float64)
    return p, x, t, m


def test_parameter_count_of_the_four_level_unet():
    # 3x3 convs, 2x2 transposed convs and the 1x1 head, base width 32
    assert O.unet_num_params(32) == 1925634
    assert O.unet_num_params(4) == sum(t * ci * co + co for t, ci, co in spec(4))


@pytest.mark.parametrize("base,B,S", [(2, 2, 16), (4, 1, 32)])
def test_forward_and_gradient_match_torch_autograd(base, B, S):
    p, x, t, m = sample(base, B, S, base + S)
    out = O.unet_forward(p, x, base)
    pt = torch.tensor(p, requires_grad=True)
    ot = torch_unet(pt, torch.tensor(x), base)
    assert np.allclose(out, ot.detach().numpy(), rtol=1e-11, atol=1e-11)
    loss, g = O.unet_loss_grad(p, x, t, m, base)
    lt = nll(ot, torch.tensor(t), torch.tensor(m))
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * max(1.0, abs(loss))
    gt = pt.grad.numpy()
    assert np.allclose(g, gt, rtol=1e-9, atol=1e-12 * np.abs(gt).max())


def test_gradient_matches_central_differences():
    base, B, S = 2, 2, 16
    p, x, t, m = sample(base, B, S, 5)
    _, g = O.unet_loss_grad(p, x, t, m, base)
    rng = np.random.default_rng(6)
    offs = list(O.unet_layer_offsets(base)) + [len(p)]
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 12) for i in range(18)])
    h = 1e-6
    ok = 0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.unet_loss_grad(pp, x, t, m, base)[0] - O.unet_loss_grad(pm, x, t, m, base)[0]) / (2 * h)
        ok += abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max())
    assert ok >= 0.98 * len(idx)  # ReLU / max-pool kinks may catch a few


def test_loss_special_cases():
    base, B, S = 2, 1, 16
    p, x, t, m = sample(base, B, S, 7)
    loss, g = O.unet_loss_grad(p, x, t, np.zeros_like(m), base)
    assert loss == 0.0 and not g.any()
    out = O.unet_forward(p, x, base)
    loss, _ = O.unet_loss_grad(p, x, out[..., 0], m, base)  # perfect mean: loss = mean(s / 2)
    assert abs(loss - 0.5 * out[..., 1][m > 0].mean()) < 1e-12


def test_bf16_rounding_matches_torch():
    """The oracle's BF16 rounding (through binary32, ties to even) against
    torch's float32 -> bfloat16 conversion, including exact ties, values
    just beside them, subnormals, overflow to infinity and signed zeros."""
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 2000) * 10.0 ** rng.integers(-40, 39, 2000),
                        [0.0, -0.0, 1.0, -1.0, 3.4e38, -3.4e38, 1e-45, np.inf, -np.inf]])
    f32 = v.astype(np.float32)
    bits = f32[np.isfinite(f32)].view(np.uint32)
    ties = ((bits & 0xFFFF0000) | 0x8000).view(np.float32)
    ties = ties[np.isfinite(ties)].astype(np.float64)  # exactly half-way
    v = np.concatenate([v, ties, np.nextafter(ties, np.inf), np.nextafter(ties, -np.inf)])
    want = torch.tensor(v).float().to(torch.bfloat16).double().numpy()
    got = O.round_bf16(v)
    assert np.array_equal(got, want, equal_nan=True)
    assert np.signbit(O.round_bf16(-0.0))


def torch_unet_bf16(p, x, base, dtype=torch.float64, chunks=1):
    """torch_unet with the BF16 storage format: BF16 input and convolution
    weights, binary32 biases and head; every convolution / transposed
    convolution output stored in BF16, and the gradient with respect to it
    (after the ReLU mask) rounded to BF16.  Arithmetic in `dtype`; with
    chunks > 1 every 3x3 convolution sums its input channels in that many
    groups (another summation order of the same products)."""
    L = spec(base)
    offs = O.unet_layer_offsets(base)

    class Rf(torch.autograd.Function):  # forward-only BF16 rounding
        @staticmethod
        def forward(ctx, a):
            return a.float().to(torch.bfloat16).to(dtype)

        @staticmethod
        def backward(ctx, g):
            return g

    class Rb(torch.autograd.Function):  # gradient-only BF16 rounding
        @staticmethod
        def forward(ctx, a):
            return a.clone()

        @staticmethod
        def backward(ctx, g):
            return g.float().to(torch.bfloat16).to(dtype)

    rf, rb = Rf.apply, Rb.apply

    def wb(i):
        taps, ci, co = L[i]
        o = int(offs[i])
        w = p[o:o + taps * ci * co].view(taps, ci, co)
        b = p[o + taps * ci * co:o + taps * ci * co + co]
        w = w.float().to(dtype) if i == 17 else rf(w)
        return w, b.float().to(dtype)

    def conv3(i, a):
        w, b = wb(i)
        ci, co = w.shape[1], w.shape[2]
        w4 = w.view(3, 3, ci, co).permute(3, 2, 0, 1)
        k = min(chunks, ci)
        if k == 1:
            return F.conv2d(a, w4, b, padding=1)
        cut = [ci * j // k for j in range(k + 1)]
        parts = [F.conv2d(a[:, cut[j]:cut[j + 1]], w4[:, cut[j]:cut[j + 1]], None, padding=1) for j in range(k)]
        y = parts[-1]
        for q in parts[-2::-1]:
            y = y + q
        return y + b[None, :, None, None]

    def up(i, a):
        w, b = wb(i)
        ci, co = w.shape[1], w.shape[2]
        return F.conv_transpose2d(a, w.view(2, 2, ci, co).permute(2, 3, 0, 1), b, stride=2)

    block = lambda i, a: rf(F.relu(rb(conv3(i, a))))
    a = rf(x.permute(0, 3, 1, 2))
    enc = []
    for l in range(4):
        a = block(2 * l + 1, block(2 * l, a))
        enc.append(a)
        if l < 3:
            a = F.max_pool2d(a, 2)
    d = enc[3]
    for j, l in enumerate((2, 1, 0)):
        k = 8 + 3 * j
        d = torch.cat([rf(rb(up(k, d))), enc[l]], 1)
        d = block(k + 2, block(k + 1, d))
    w, b = wb(17)
    out = F.conv2d(d, w.view(w.shape[1], w.shape[2]).t()[:, :, None, None], b)
    return out.permute(0, 2, 3, 1)


@pytest.mark.parametrize("base,B,S", [(2, 2, 16), (4, 1, 32)])
def test_bf16_format_matches_torch_autograd_with_the_same_roundings(base, B, S):
    p, x, t, m = sample(base, B, S, 3 * base + S)
    out = O.unet_forward(p, x, base, bf16=True)
    pt = torch.tensor(p, requires_grad=True)
    ot = torch_unet_bf16(pt, torch.tensor(x), base)
    # same stored values up to the order of binary64 sums
    assert np.allclose(out, ot.detach().numpy(), rtol=1e-9, atol=1e-9)
    loss, g = O.unet_loss_grad(p, x, t, m, base, bf16=True)
    lt = nll(ot, torch.tensor(t), torch.tensor(m))
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-9 * max(1.0, abs(loss))
    gt = pt.grad.numpy()
    assert np.linalg.norm(g - gt) <= 1e-7 * np.linalg.norm(gt)
    # and the format really differs from binary64
    assert not np.allclose(out, O.unet_forward(p, x, base), rtol=1e-6, atol=0)


def test_fp32_format_error_budget_at_full_width():
    """The per-layer gradient bar of the GPU's base-32 cases
    (tests/test_unet.py, LAYER_BAR_WIDE) is 1.5 times the largest per-layer
    error of torch's FP32 convolutions in the same format against the
    BF16-format oracle, over eight summation orders; re-measured here."""
    import test_unet as TU
    worst = 0.0
    for base, B, S in TU.WIDE_CASES:
        p, x, t, m = TU.sample(base, B, S, 13 * base + S)  # the GPU test's inputs
        _, rg = O.unet_loss_grad(p, x, t, m, base, bf16=True)
        offs = list(O.unet_layer_offsets(base)) + [len(p)]
        for chunks in (1, 2, 3, 5):
            for onednn in (True, False):
                with torch.backends.mkldnn.flags(enabled=onednn):
                    pt = torch.tensor(p, dtype=torch.float32, requires_grad=True)
                    ot = torch_unet_bf16(pt, torch.tensor(x, dtype=torch.float32), base, torch.float32, chunks)
                    nll(ot, torch.tensor(t, dtype=torch.float32), torch.tensor(m, dtype=torch.float32)).backward()
                g = pt.grad.double().numpy()
                per = [np.linalg.norm(g[offs[i]:offs[i + 1]] - rg[offs[i]:offs[i + 1]])
                       / np.linalg.norm(rg[offs[i]:offs[i + 1]]) for i in range(18)]
                worst = max(worst, max(per))
    print(f"largest per-layer gradient error of FP32 in the BF16 format: {worst:.4f}")
    assert 0.02 < worst <= TU.LAYER_BAR_WIDE / 1.5
