"""Screen-space marching of reflection rays against the depth buffer.

Oracle code (test infrastructure only).

Sec. 3.3 marches a reflection ray r(t) from the pixel's un-projected position
in screen space and reports an intersection where the ray passes from in
front of the depth buffer to behind it; Appendix D (Algorithm 1) gives the
fixed-step version with a depth-match threshold.  Two marches are defined:

* ``march_linear``: the fixed-step march of Algorithm 1.  Readings taken:
  samples t_k = k * step for k = 1..K (the sample at the origin would hit its
  own pixel), depth compared in view space, nearest depth texel.  The hit
  test joins the two statements of the paper: Sec. 3.3 asks for dz to change
  from negative to positive, Algorithm 1 for |dz| below a threshold.  A
  sample hits when 0 <= dz <= thickness and an earlier sample had dz < 0
  (the ray was in front of the depth buffer before it went behind it).
  Samples inside the origin pixel are skipped and never count as in front.

* ``march_hiz``: the same criterion, made exact for the piecewise-constant
  depth heightfield and accelerated by a min-max depth pyramid.  The paper
  marches in fixed steps only (Sec. 3.3, citing a screen-space DDA tracer);
  this hierarchical traversal is the build's own design, not the paper's.
  Its result with the iteration cap lifted is pinned to the pyramid-free
  definition ``brute_force_first_hit``; which rays reach the cap, and after
  how many iterations, is defined by the traversal below (the same sequence
  the GPU kernel takes).  The view-space ray is clipped
  to [0, min(max_dist, near-plane crossing)], projected to a screen segment
  P(s) = P0 + s (P1 - P0), s in [0, 1], whose depth 1/((1-s)/d0 + s/d1) is
  monotone in s, and clipped to the screen.  Along the segment the pixels are
  visited in order; in pixel q the ray's depth runs from d_in to d_out.  The
  ray hits q when its depth range meets the slab [D[q], D[q] + thickness]
  and it has been in front of the depth buffer before reaching the slab:
  either in an earlier pixel (lo < D there) or on entering q (d_in < D[q]).
  The origin pixel never counts.

  The traversal holds a level L and the level-0 pixel that contains the
  current point of the segment.  A cell can be skipped when the ray's depth
  range over the part of the segment inside it lies wholly in front of the
  cell's minimum depth (the ray is in front of every pixel there) or wholly
  behind the cell's maximum depth plus the thickness (no slab there can be
  met).  Each iteration looks at the level-L cell and its parent (level
  L + 1, below the top):
    - parent skippable: move to the parent's far boundary, L = L + 1;
    - else the level-L cell skippable: move to its far boundary;
    - else, above level 0: L = max(L - 2, 0) (the parent's own parent was
      already known not to be skippable, so the next pair is two levels
      down);
    - else at level 0 test the pixel; on a miss move to the next pixel.
  ``brute_force_first_hit`` scans every pixel the segment crosses, in order,
  and is what the traversal must reproduce when the iteration cap is lifted.

Result codes: q >= 0 hit pixel (j*W + i); -1 left the screen or the ray
segment; -4 iteration cap reached.
"""

import numpy as np

from . import camera

HIT_OFFSCREEN = -1
HIT_CAP = -4


def _reduce_levels(depth, op, pad_value):
    lv = [np.asarray(depth, np.float64)]
    while lv[-1].shape != (1, 1):
        d = lv[-1]
        h, w = d.shape
        ph, pw = h + (h & 1), w + (w & 1)
        pad = np.full((ph, pw), pad_value)
        pad[:h, :w] = d
        lv.append(op(pad.reshape(ph // 2, 2, pw // 2, 2), axis=(1, 3)))
    return lv


def hiz_pyramid(depth):
    """Levels 0..top of the min-depth pyramid (level 0 is the depth itself).

    Level L has ceil(W_{L-1}/2) x ceil(H_{L-1}/2) texels, each the minimum of
    its (up to four) children; the last level is 1 x 1.
    """
    return _reduce_levels(depth, np.min, np.inf)


def hiz_max_pyramid(depth):
    """The same levels holding the maximum depth of each cell."""
    return _reduce_levels(depth, np.max, -np.inf)


def march_linear(cam, depth, org_pix, V0, Dv, step_len, max_steps, max_dist, thickness):
    """Fixed-step march (Algorithm 1 with the readings above), vectorised.

    ``org_pix`` [n][2] integer (i, j); ``V0`` [n][3] view-space origins;
    ``Dv`` [n][3] view-space unit directions.  Returns (codes, iterations).
    """
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    n = V0.shape[0]
    codes = np.full(n, HIT_CAP, np.int64)
    iters = np.zeros(n, np.int64)
    active = np.ones(n, bool)
    armed = np.zeros(n, bool)
    K = int(max_steps)
    if step_len > 0:
        K = min(K, int(np.floor(max_dist / step_len)))
    for k in range(1, K + 1):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        iters[idx] = k
        v = V0[idx] + (k * step_len) * Dv[idx]
        behind = v[:, 2] <= c["z_near"]
        with np.errstate(divide="ignore", invalid="ignore"):
            px, py = camera.project(c, v)
        off = behind | ~(px >= 0) | ~(px < W) | ~(py >= 0) | ~(py < H)
        codes[idx[off]] = HIT_OFFSCREEN
        active[idx[off]] = False
        keep = ~off
        idx, v, px, py = idx[keep], v[keep], px[keep], py[keep]
        ix = np.floor(px).astype(np.int64)
        iy = np.floor(py).astype(np.int64)
        own = (ix == org_pix[idx, 0]) & (iy == org_pix[idx, 1])
        dz = v[:, 2] - depth[iy, ix]
        hit = ~own & armed[idx] & (dz >= 0) & (dz <= thickness)
        codes[idx[hit]] = iy[hit] * W + ix[hit]
        active[idx[hit]] = False
        armed[idx[~own & (dz < 0)]] = True
    iters[active] = K
    return codes, iters


def screen_segment(cam, org_pix, V0, Dv, max_dist):
    """Clip the view-space ray and project it: returns P0, dP, d0, d1, s_max, valid.

    P0 is the origin pixel's centre (V0 is its un-projection); the far end is
    the point at min(max_dist, near-plane crossing).  s_max is where the
    segment leaves the screen rectangle [0, W] x [0, H] (at most 1).
    """
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    d0 = V0[:, 2]
    t_end = np.full(V0.shape[0], float(max_dist))
    with np.errstate(divide="ignore", invalid="ignore"):
        t_near = (c["z_near"] - d0) / Dv[:, 2]
    toward = Dv[:, 2] < 0
    t_end[toward] = np.minimum(t_end[toward], t_near[toward])
    valid = t_end > 0
    E = V0 + t_end[:, None] * Dv
    with np.errstate(divide="ignore", invalid="ignore"):
        p1x, p1y = camera.project(c, E)
    P0 = org_pix.astype(np.float64) + 0.5
    dP = np.stack([p1x, p1y], axis=1) - P0
    s_max = np.ones(V0.shape[0])
    with np.errstate(divide="ignore", invalid="ignore"):
        for ax, lim in ((0, W), (1, H)):
            sx = np.where(dP[:, ax] > 0, (lim - P0[:, ax]) / dP[:, ax],
                          np.where(dP[:, ax] < 0, (0.0 - P0[:, ax]) / dP[:, ax], np.inf))
            s_max = np.minimum(s_max, sx)
    return P0, dP, d0, E[:, 2], s_max, valid


def _ray_depth(d0, d1, s):
    """Perspective-correct depth along the segment; exactly d0 at s = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        d = 1.0 / ((1.0 - s) / d0 + s / d1)
    return np.where(s == 0, d0, d)


def march_hiz(cam, pyramid, org_pix, V0, Dv, max_steps, max_dist, thickness):
    """Hierarchical march over the min-max pyramid, vectorised in lock step.

    ``pyramid`` is the pair (hiz_pyramid, hiz_max_pyramid) of the depth.
    Returns (codes, iterations).  ``max_steps`` caps the iterations.
    """
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    pyr_min, pyr_max = pyramid
    top = len(pyr_min) - 1
    depth = pyr_min[0]
    n = V0.shape[0]
    P0, dP, d0, d1, s_max, valid = screen_segment(cam, org_pix, V0, Dv, max_dist)
    codes = np.full(n, HIT_CAP, np.int64)
    iters = np.zeros(n, np.int64)
    codes[~valid] = HIT_OFFSCREEN
    active = valid.copy()
    s = np.zeros(n)
    armed = np.zeros(n, bool)
    L = np.zeros(n, np.int64)
    ix = org_pix[:, 0].astype(np.int64).copy()
    iy = org_pix[:, 1].astype(np.int64).copy()

    def cell(a, lv):
        """Bounds, exit parameter and skip tests of the level-lv cells that
        contain the current pixels of rays a."""
        size = np.left_shift(1, lv)
        x0 = (ix[a] >> lv) * size
        y0 = (iy[a] >> lv) * size
        x1 = np.minimum(x0 + size, W)
        y1 = np.minimum(y0 + size, H)
        with np.errstate(divide="ignore", invalid="ignore"):
            sx = np.where(dP[a, 0] > 0, (x1 - P0[a, 0]) / dP[a, 0],
                          np.where(dP[a, 0] < 0, (x0 - P0[a, 0]) / dP[a, 0], np.inf))
            sy = np.where(dP[a, 1] > 0, (y1 - P0[a, 1]) / dP[a, 1],
                          np.where(dP[a, 1] < 0, (y0 - P0[a, 1]) / dP[a, 1], np.inf))
        s_exit = np.minimum(np.minimum(sx, sy), s_max[a])
        din = _ray_depth(d0[a], d1[a], s[a])
        dout = _ray_depth(d0[a], d1[a], s_exit)
        hi = np.maximum(din, dout)
        lo = np.minimum(din, dout)
        front = hi < _gather(pyr_min, lv, ix[a], iy[a])        # in front of every pixel
        behind = lo > _gather(pyr_max, lv, ix[a], iy[a]) + thickness  # behind every slab
        return dict(x0=x0, y0=y0, x1=x1, y1=y1, sx=sx, sy=sy, s_exit=s_exit, din=din, lo=lo,
                    front=front, skip=front | behind)

    step = 0
    while active.any() and step < max_steps:
        step += 1
        a = np.nonzero(active)[0]
        iters[a] += 1
        La = L[a]
        child = cell(a, La)
        parent = cell(a, np.minimum(La + 1, top))
        up = parent["skip"] & (La < top)
        # the cell the ray moves across if it moves: the parent when it can
        # be skipped, else the level-L cell
        k = {key: np.where(up, parent[key], child[key]) for key in child}
        skip = up | child["skip"]
        level0 = ~skip & (La == 0)
        descend = ~skip & (La > 0)
        own = level0 & (ix[a] == org_pix[a, 0]) & (iy[a] == org_pix[a, 1])
        test = level0 & ~own
        dq = depth[iy[a], ix[a]]
        hit = test & (child["lo"] <= dq + thickness) & (armed[a] | (child["din"] < dq))
        advance = skip | own | (test & ~hit)
        # the ray was in front of the depth buffer somewhere in a cell it
        # skipped for that reason, or in a tested pixel it passes
        armed[a[(skip & k["front"] & (k["s_exit"] > s[a])) | (test & (child["lo"] < dq))]] = True
        ah = a[hit]
        codes[ah] = iy[ah] * W + ix[ah]
        active[ah] = False
        ad = a[descend]
        L[ad] = np.maximum(L[ad] - 2, 0)
        # advances: leave at the segment end, else step into the next cell
        se = k["s_exit"]
        ends = advance & (se >= s_max[a])
        codes[a[ends]] = HIT_OFFSCREEN
        active[a[ends]] = False
        mv = advance & ~ends
        am = a[mv]
        sem = se[mv]
        crx = k["sx"][mv] == sem
        cry = k["sy"][mv] == sem
        px = P0[am, 0] + sem * dP[am, 0]
        py = P0[am, 1] + sem * dP[am, 1]
        x0, x1, y0, y1 = k["x0"][mv], k["x1"][mv], k["y0"][mv], k["y1"][mv]
        nx = np.where(crx, np.where(dP[am, 0] > 0, x1, x0 - 1),
                      np.clip(np.floor(px).astype(np.int64), x0, x1 - 1))
        ny = np.where(cry, np.where(dP[am, 1] > 0, y1, y0 - 1),
                      np.clip(np.floor(py).astype(np.int64), y0, y1 - 1))
        ix[am] = nx
        iy[am] = ny
        s[am] = sem
        L[am] = np.where(up[mv], np.minimum(L[am] + 1, top), L[am])
        # a step past the screen edge (boundary coinciding with it) leaves too
        gone = (nx < 0) | (nx >= W) | (ny < 0) | (ny >= H)
        codes[am[gone]] = HIT_OFFSCREEN
        active[am[gone]] = False
    return codes, iters


def _gather(pyramid, L, ix, iy):
    out = np.empty(L.shape[0])
    for lv in np.unique(L):
        sel = L == lv
        out[sel] = pyramid[lv][iy[sel] >> lv, ix[sel] >> lv]
    return out


def brute_force_first_hit(cam, depth, org_pix, V0, Dv, max_dist, thickness, bbox=False):
    """First hit by scanning every pixel the segment crosses (no pyramid).

    For each pixel box [i, i+1] x [j, j+1] the s-interval of the clipped
    screen segment inside it is found by slab clipping, without any pyramid.
    The crossed pixels (positive-length intervals, origin excluded) are then
    walked in order of entry; the ray's depth over a pixel's interval
    (monotone in s) is compared with the slab [D, D + thickness] under the
    in-front-first rule.  Returns codes.

    With ``bbox`` only the pixels meeting the bounding box of the clipped
    segment are scanned (a pixel outside it cannot hold a positive-length
    part of the segment), which makes large images affordable for a few
    thousand rays; the full scan is for tiny images.
    """
    c = camera.unpack(cam)
    W, H = c["W"], c["H"]
    P0, dP, d0, d1, s_max, valid = screen_segment(cam, org_pix, V0, Dv, max_dist)
    n = V0.shape[0]
    out = np.full(n, HIT_OFFSCREEN, np.int64)
    D2 = np.asarray(depth, np.float64)
    if not bbox:
        jj_all, ii_all = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ii_all = ii_all.reshape(-1)
        jj_all = jj_all.reshape(-1)
        D_all = D2.reshape(-1)
    for r in range(n):
        if not valid[r]:
            continue
        if bbox:
            ends = np.stack([P0[r], P0[r] + min(s_max[r], 1.0) * dP[r]])
            lo = np.clip(np.floor(ends.min(0)).astype(np.int64) - 1, 0, [W - 1, H - 1])
            hi = np.clip(np.floor(ends.max(0)).astype(np.int64) + 1, 0, [W - 1, H - 1])
            jj, ii = np.meshgrid(np.arange(lo[1], hi[1] + 1), np.arange(lo[0], hi[0] + 1),
                                 indexing="ij")
            ii = ii.reshape(-1)
            jj = jj.reshape(-1)
            D = D2[jj, ii]
        else:
            ii, jj, D = ii_all, jj_all, D_all
        lo_s = np.zeros(ii.shape)
        hi_s = np.full(ii.shape, s_max[r])
        for ax, cell in ((0, ii), (1, jj)):
            if dP[r, ax] == 0:
                inside = (cell <= P0[r, ax]) & (P0[r, ax] < cell + 1)
                hi_s = np.where(inside, hi_s, -np.inf)
                continue
            sa = (cell - P0[r, ax]) / dP[r, ax]
            sb = (cell + 1 - P0[r, ax]) / dP[r, ax]
            lo_s = np.maximum(lo_s, np.minimum(sa, sb))
            hi_s = np.minimum(hi_s, np.maximum(sa, sb))
        crossed = hi_s > lo_s
        crossed &= ~((ii == org_pix[r, 0]) & (jj == org_pix[r, 1]))
        order = np.nonzero(crossed)[0]
        order = order[np.argsort(lo_s[order], kind="stable")]
        if order.size == 0:
            continue
        # the ray's depth range over each crossed pixel, in order of entry
        din = _ray_depth(d0[r], d1[r], lo_s[order])
        dout = _ray_depth(d0[r], d1[r], hi_s[order])
        lo, hi = np.minimum(din, dout), np.maximum(din, dout)
        Dk = D[order]
        # armed before pixel k: the ray was in front in some earlier pixel
        front = lo < Dk
        armed = np.concatenate([[False], np.cumsum(front)[:-1] > 0])
        hit = (hi >= Dk) & (lo <= Dk + thickness) & (armed | (din < Dk))
        if hit.any():
            k = order[np.argmax(hit)]
            out[r] = jj[k] * W + ii[k]
    return out
