"""Exact render of a map of flat-topped cells, for the render pin of the
camera association (Sec. III-B, Fig. 3): every cell is a column of the
cell's square footprint up to its height.  A pinhole camera's pixel shows the
first column its ray enters below the column's top; the image channel holds
that cell's index (exactly representable in binary32), so a cell that the
update finds visible must gather its own index.

The render is independent of the oracle and of the library: a ray-column
walk (Amanatides-Woo cell traversal) in binary64 from the camera through
every pixel centre.

`classify` states, per cell, what the method must decide wherever the
geometry leaves no doubt: the projected top face covers its pixel with at
least one pixel of margin on every side, and along the straight line from
the camera to the top's centre every intermediate column of the major axis
is either clearly below the line (by `margin`) or, in some column, every cell
the line touches there is clearly above it.  The camera must sit above a cell
centre, so that the line of cells the method walks is the line the camera
sees along.
"""
from __future__ import annotations

import numpy as np


def project(K, T, pts):
    """Pixel coordinates (u, v) and depth of map points [N, 3] (binary64)."""
    R = np.asarray(T, np.float64)[:, :3]
    t = np.asarray(T, np.float64)[:, 3]
    P = (pts - t) @ R
    fx, fy, cx, cy = (float(k) for k in K)
    Z = P[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        return fx * P[:, 0] / Z + cx, fy * P[:, 1] / Z + cy, Z


def render_ids(h, res, origin, K, T, hw):
    """[H_img, W_img] image of the index (iy * W + ix) of the cell each pixel
    shows, -1 where the ray leaves the map without entering a column.
    h: [H, W] column heights (every cell holds one); origin: (ox, oy) integer
    lattice coordinates of cell (0, 0)."""
    Hm, Wm = h.shape
    hi, wi = hw
    R = np.asarray(T, np.float64)[:, :3]
    t = np.asarray(T, np.float64)[:, 3]
    fx, fy, cx, cy = (float(k) for k in K)
    pu, pv = np.meshgrid(np.arange(wi, dtype=np.float64), np.arange(hi, dtype=np.float64))
    dc = np.stack([(pu - cx) / fx, (pv - cy) / fy, np.ones_like(pu)], -1).reshape(-1, 3)
    d = dc @ R.T  # map-frame directions
    n = d.shape[0]
    # lattice coordinates (cell units), origin at cell (0, 0)'s corner
    gx0 = t[0] / res - origin[0]
    gy0 = t[1] / res - origin[1]
    gdx, gdy = d[:, 0] / res, d[:, 1] / res
    out = np.full(n, -1, np.int64)
    ix = np.full(n, int(np.floor(gx0)))
    iy = np.full(n, int(np.floor(gy0)))
    stx = np.where(gdx > 0, 1, -1)
    sty = np.where(gdy > 0, 1, -1)
    with np.errstate(divide="ignore", invalid="ignore"):
        tdx = np.where(gdx != 0, np.abs(1.0 / gdx), np.inf)
        tdy = np.where(gdy != 0, np.abs(1.0 / gdy), np.inf)
        nbx = np.where(gdx > 0, np.floor(gx0) + 1 - gx0, gx0 - np.floor(gx0))
        nby = np.where(gdy > 0, np.floor(gy0) + 1 - gy0, gy0 - np.floor(gy0))
        tmx = np.where(gdx != 0, nbx * tdx, np.inf)
        tmy = np.where(gdy != 0, nby * tdy, np.inf)
    s_in = np.zeros(n)
    live = np.ones(n, bool)
    for _ in range(2 * (Hm + Wm) + 4):
        if not live.any():
            break
        s_out = np.minimum(tmx, tmy)
        inside = (ix >= 0) & (ix < Wm) & (iy >= 0) & (iy < Hm)
        hc = np.where(inside, h[np.clip(iy, 0, Hm - 1), np.clip(ix, 0, Wm - 1)], -np.inf)
        z_out = t[2] + s_out * d[:, 2]
        z_in = t[2] + s_in * d[:, 2]
        hit = live & inside & (np.minimum(z_in, z_out) <= hc)
        out[hit] = iy[hit] * Wm + ix[hit]
        live &= ~hit
        # rays that left the lattice on the far side of the map are done
        gone = ((stx > 0) & (ix >= Wm)) | ((stx < 0) & (ix < 0)) | ((sty > 0) & (iy >= Hm)) | ((sty < 0) & (iy < 0))
        live &= ~gone
        stepx = tmx <= tmy
        s_in = s_out
        ix = np.where(stepx, ix + stx, ix)
        tmx = np.where(stepx, tmx + tdx, tmx)
        iy = np.where(~stepx, iy + sty, iy)
        tmy = np.where(~stepx, tmy + tdy, tmy)
    return out.reshape(hi, wi)


def classify(h, res, origin, K, T, hw, margin=0.02):
    """Per cell: 1 = must be visible and gather its own index, 0 = must not
    be fused (occluded), -1 = no claim (small footprint, outside the view,
    or a column within `margin` of the line).  Also returns the pixel
    (row, col) of every cell's top centre (floor(x + 0.5) convention)."""
    Hm, Wm = h.shape
    hi, wi = hw
    T = np.asarray(T, np.float64)
    cam = T[:, 3]
    iy, ix = np.meshgrid(np.arange(Hm), np.arange(Wm), indexing="ij")
    x0 = (origin[0] + ix) * res
    y0 = (origin[1] + iy) * res
    ctr = np.stack([x0 + 0.5 * res, y0 + 0.5 * res, h], -1).reshape(-1, 3)
    u, v, Z = project(K, T, ctr)
    pu, pv = np.floor(u + 0.5), np.floor(v + 0.5)
    ok = (Z > 0.1) & (pu >= 0) & (pu < wi) & (pv >= 0) & (pv < hi)
    # the top face's corners in the image: the pixel centre must lie inside
    # the projected quadrilateral with >= 1 px to every edge
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]
    cu, cv = [], []
    for a, b in corners:
        pts = np.stack([x0 + a * res, y0 + b * res, h], -1).reshape(-1, 3)
        uu, vv, zz = project(K, T, pts)
        ok &= zz > 0.1
        cu.append(uu)
        cv.append(vv)
    # winding of the quadrilateral, so that "inside" is positive either way
    sign = np.sign((cu[1] - cu[0]) * (cv[2] - cv[0]) - (cv[1] - cv[0]) * (cu[2] - cu[0]))
    dist = np.full(ok.shape, np.inf)
    for k in range(4):
        ax_, ay_ = cu[k], cv[k]
        bx_, by_ = cu[(k + 1) % 4], cv[(k + 1) % 4]
        ex, ey = bx_ - ax_, by_ - ay_
        cross = (ex * (pv - ay_) - ey * (pu - ax_)) / np.maximum(np.hypot(ex, ey), 1e-30)
        dist = np.minimum(dist, sign * cross)
    big = ok & (dist >= 1.0)
    # the camera's cell (the method walks from it)
    acx = int(np.floor(cam[0] / res)) - origin[0]
    acy = int(np.floor(cam[1] / res)) - origin[1]
    claim = np.full(Hm * Wm, -1, np.int64)
    for j in np.flatnonzero(big):
        bx, by = j % Wm, j // Wm
        dx, dy = bx - acx, by - acy
        xmajor = abs(dx) >= abs(dy)
        steps = max(abs(dx), abs(dy))
        if steps <= 1:
            claim[j] = 1
            continue
        p = ctr[j]
        verdict = 1
        for s in range(1, steps + 1):
            # major-axis column s: the line spans the column's two edges (the
            # target's own column up to the target's centre)
            lo_t, hi_t = (s - 0.5) / steps, min(s + 0.5, steps) / steps
            z_a = cam[2] + (p[2] - cam[2]) * lo_t
            z_b = cam[2] + (p[2] - cam[2]) * hi_t
            zmin, zmax = min(z_a, z_b), max(z_a, z_b)
            # minor coordinates (in cells, lattice of cell centres) spanned
            if xmajor:
                m0 = acy + dy * lo_t
                m1 = acy + dy * hi_t
                col = acx + (s if dx > 0 else -s)
            else:
                m0 = acx + dx * lo_t
                m1 = acx + dx * hi_t
                col = acy + (s if dy > 0 else -s)
            # widened by 0.15 cells: the pixel's own ray runs within a
            # fraction of a cell of this line
            lo_c = int(np.floor(min(m0, m1) - 0.15 + 0.5))
            hi_c = int(np.floor(max(m0, m1) + 0.15 + 0.5))
            hs = []
            for c in range(lo_c, hi_c + 1):
                cxk, cyk = (col, c) if xmajor else (c, col)
                if (cxk, cyk) != (bx, by) and 0 <= cxk < Wm and 0 <= cyk < Hm:
                    hs.append(h[cyk, cxk])
            if not hs:
                continue
            # a cell no higher than the target never occludes it: the line
            # descends to the target's height only at the target
            if all(hk < zmin - margin or (hk <= p[2] < cam[2]) for hk in hs):
                continue
            if s < steps and all(hk > zmax + margin for hk in hs):
                verdict = 0  # the method walks one of these cells
                break
            verdict = -1
            break
        claim[j] = verdict
    return claim.reshape(Hm, Wm), pv.reshape(Hm, Wm).astype(np.int64), pu.reshape(Hm, Wm).astype(np.int64)


def block_city(rng, W, H, levels=(0.1, 0.3, 0.55, 0.8), n_blocks=14, keep_clear=None):
    """Flat ground at 0 with axis-aligned flat-topped blocks 2-5 cells wide
    (so that every line crossing a block touches it in two cells of a
    column); keep_clear: (ix, iy, radius) of cells left at ground level."""
    h = np.zeros((H, W))
    for _ in range(n_blocks):
        bw, bh = rng.integers(2, 6, 2)
        x0 = int(rng.integers(0, W - bw))
        y0 = int(rng.integers(0, H - bh))
        h[y0:y0 + bh, x0:x0 + bw] = rng.choice(levels)
    if keep_clear is not None:
        cx, cy, r = keep_clear
        yy, xx = np.mgrid[0:H, 0:W]
        h[(xx - cx) ** 2 + (yy - cy) ** 2 <= r * r] = 0.0
    return h
