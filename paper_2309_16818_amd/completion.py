"""Training pairs, training loop and evaluation of the completion network.

Pairs come from the map update itself (mem_batch_*): for every window of a
CompletionWorld the dense target is the fusion of five 360-degree sweeps and
the sparse input the fusion of one forward sensor with occluders.  The
network input and target are read out with mem_unet_input; training steps
are mem_unet_train_step; evaluation runs mem_unet_complete (network plus the
sigma gate).  This module only marshals tensors between those calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import mem, synth


@dataclass
class Pairs:
    x: torch.Tensor       # [n, S, S, 3] network input from the sparse fusion
    target: torch.Tensor  # [n, S, S] dense-fusion height - z_ref
    mask: torch.Tensor    # [n, S, S] 1 where the dense fusion has a height
    z_ref: np.ndarray     # [n] ground height under the robot

    def __len__(self):
        return self.x.shape[0]

    def subset(self, idx):
        idx = torch.as_tensor(idx, device=self.x.device)
        return Pairs(self.x[idx].contiguous(), self.target[idx].contiguous(), self.mask[idx].contiguous(),
                     self.z_ref[idx.cpu().numpy()])


MAP_KW = dict(noise_c0=0.01, noise_c1=0.001, max_range=20.0, clear_margin=0.05, clear_min_count=1,
              min_depth=0.1)


def _fuse(world: synth.CompletionWorld, steps):
    """Runs the map update over the steps' clouds on a fresh batch of maps;
    returns the batch."""
    n, S = world.n, world.size
    mp = max(int(st["offsets"][-1]) for st in steps)
    b = mem.Batch([S] * n, [S] * n, world.res, max_points=max(mp, 1), **MAP_KW)
    for st in steps:
        b.step(st["robot_xy"], st["xyz"], st["offsets"], st["T"])
    return b


def make_pairs(n, size=256, res=0.04, seed=0, chunk=64) -> Pairs:
    """n (input, target) pairs on n seeded worlds, generated `chunk` windows
    at a time."""
    xs, ts, ms, zs = [], [], [], []
    for c0 in range(0, n, chunk):
        k = min(chunk, n - c0)
        w = synth.CompletionWorld(k, size=size, res=res, seed=seed * 1000003 + c0)
        dense = _fuse(w, [w.dense_step(v) for v in range(len(w.VIEW))])
        sparse = _fuse(w, [w.sparse_step()])
        x = torch.empty((k, size, size, 3), dtype=torch.float32, device="cuda")
        xt = torch.empty((size, size, 3), dtype=torch.float32, device="cuda")
        t = torch.empty((k, size, size), dtype=torch.float32, device="cuda")
        m = torch.empty((k, size, size), dtype=torch.float32, device="cuda")
        for i in range(k):
            z = float(w.ground[i])
            mem.unet_input(sparse.get_layer(i, mem.MEM_LAYER_ELEVATION), sparse.get_layer(i, mem.MEM_LAYER_VARIANCE),
                           z, out=x[i])
            mem.unet_input(dense.get_layer(i, mem.MEM_LAYER_ELEVATION), dense.get_layer(i, mem.MEM_LAYER_VARIANCE),
                           z, out=xt)
            t[i] = xt[..., 0]
            m[i] = xt[..., 2]
        dense.close()
        sparse.close()
        xs.append(x)
        ts.append(t)
        ms.append(m)
        zs.append(w.ground.copy())
    torch.cuda.synchronize()
    return Pairs(torch.cat(xs), torch.cat(ts), torch.cat(ms), np.concatenate(zs))


def _augment(x, t, m, k):
    """One of the 8 symmetries of the square (rotations and flips) applied to
    a batch; heights are unchanged by them."""
    if k & 4:
        x, t, m = x.flip(2), t.flip(2), m.flip(2)
    r = k & 3
    if r:
        x, t, m = torch.rot90(x, r, (1, 2)), torch.rot90(t, r, (1, 2)), torch.rot90(m, r, (1, 2))
    return x.contiguous(), t.contiguous(), m.contiguous()


def train(net: mem.UNet, pairs: Pairs, steps: int, batch: int, lr: float, seed: int = 0,
          lr_final: float | None = None, log=None):
    """Adam steps on random augmented batches; cosine decay from lr to
    lr_final (default lr / 10).  Returns the loss of every step (host)."""
    rng = np.random.default_rng(seed)
    lr_final = lr / 10 if lr_final is None else lr_final
    loss = torch.zeros(steps, dtype=torch.float32, device="cuda")
    n = len(pairs)
    for s in range(steps):
        idx = torch.as_tensor(rng.choice(n, size=batch, replace=n < batch), device="cuda")
        x, t, m = _augment(pairs.x[idx], pairs.target[idx], pairs.mask[idx], int(rng.integers(8)))
        a = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * s / max(steps - 1, 1)))
        net.train_step(x, t, m, a, loss_out=loss[s:s + 1])
        if log and (s % 100 == 0 or s == steps - 1):
            log(f"step {s}: loss {loss[s].item():.4f}")
    return loss.cpu().numpy()


def evaluate(net: mem.UNet, pairs: Pairs, sigma_max: float, batch: int = 8) -> dict:
    """Coverage and height error of the classical fusion alone and of the
    gated completion, over the cells the dense fusion observed."""
    tot = dict(valid=0, cls=0, comp=0, new=0, se_cls=0.0, se_comp=0.0, se_new=0.0, new_within=0)
    for b0 in range(0, len(pairs), batch):
        sl = slice(b0, b0 + batch)
        x = pairs.x[sl].contiguous()
        h, _ = net.complete_windows(x, 0.0, sigma_max)
        t = pairs.target[sl]
        valid = pairs.mask[sl] > 0
        obs = x[..., 2] > 0
        cov = torch.isfinite(h)
        new = cov & ~obs & valid
        tot["valid"] += int(valid.sum())
        tot["cls"] += int((obs & valid).sum())
        tot["comp"] += int((cov & valid).sum())
        tot["new"] += int(new.sum())
        d = (h - t)
        tot["se_cls"] += float((d[obs & valid] ** 2).sum())
        tot["se_comp"] += float((d[cov & valid] ** 2).sum())
        tot["se_new"] += float((d[new] ** 2).sum())
        tot["new_within"] += int((d[new].abs() <= 2 * sigma_max).sum())
    v = max(tot["valid"], 1)
    r = lambda se, k: math.sqrt(se / k) if k else float("nan")
    return dict(coverage_classical=tot["cls"] / v, coverage_completed=tot["comp"] / v,
                rmse_classical=r(tot["se_cls"], tot["cls"]), rmse_completed=r(tot["se_comp"], tot["comp"]),
                rmse_filled=r(tot["se_new"], tot["new"]), filled_cells=tot["new"],
                filled_within_2sigma=tot["new_within"] / max(tot["new"], 1), valid_cells=tot["valid"])
