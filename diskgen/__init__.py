"""Seeded synthetic inputs for the thin-disk force: densities, slopes, AMR layouts.

This module is shared by the oracle tests and the GPU path's tests and
benchmark.  It produces inputs only (surface densities, their first-order
slopes, composite AMR layouts, batches and request streams); it holds none of
the force computation.  Every random draw comes from
``numpy.random.default_rng(seed)``.

Layout conventions: arrays are row-major [y, x] (row j = y index, x fastest).
A uniform grid of n x n cells covers [x0, x0 + n h] x [y0, y0 + n h]; the
default is [-1, 1]^2.  Slopes (dsx, dsy) are the first-order Taylor
coefficients of Section 2 of the paper: the exact gradient at the cell centre
for analytic profiles, second-order central differences (one-sided at the
domain edge) for sampled noisy ones.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

# ----------------------------------------------------------------------------
# uniform grids and analytic profiles
# ----------------------------------------------------------------------------


def grid_centres(n, x0=-1.0, y0=-1.0, h=None):
    """Cell-centre coordinates (X, Y), each (n, n), of an n x n grid."""
    if h is None:
        h = 2.0 / n
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x0 + c, y0 + c)
    return X, Y


def kuzmin(X, Y, M=1.0, a=0.2, centre=(0.0, 0.0)):
    """Kuzmin disk s = M a / (2 pi (r^2 + a^2)^{3/2}) and its exact gradient."""
    dx = X - centre[0]
    dy = Y - centre[1]
    q = dx * dx + dy * dy + a * a
    s = M * a / (2 * np.pi * q ** 1.5)
    g = -3.0 * s / q
    return s, g * dx, g * dy


def d2(X, Y, alpha=0.25, sigma0=1.0, centre=(0.0, 0.0)):
    """D2 disk s0 (1 - R^2/alpha^2)^{3/2} (zero outside) and its exact gradient."""
    dx = X - centre[0]
    dy = Y - centre[1]
    t = np.clip(1.0 - (dx * dx + dy * dy) / alpha ** 2, 0.0, None)
    s = sigma0 * t ** 1.5
    g = -3.0 * sigma0 * np.sqrt(t) / alpha ** 2
    return s, g * dx, g * dy


def d22(X, Y, alpha=0.25, sigma0=1.0):
    """Two D2 disks centred at (0, 0.5) and (0, -0.5)."""
    a = d2(X, Y, alpha, sigma0, (0.0, 0.5))
    b = d2(X, Y, alpha, sigma0, (0.0, -0.5))
    return a[0] + b[0], a[1] + b[1], a[2] + b[2]


def spiral(X, Y, base="exp", scale=0.25, amp=0.1, pitch_deg=20.0, phase=0.0):
    """base(r) (1 + amp cos(2 theta - ln r / tan(pitch) + phase)) and exact gradient.

    base = "exp": exp(-r/scale); base = "kuzmin": (1 + r^2/scale^2)^{-3/2}.
    """
    r = np.hypot(X, Y)
    th = np.arctan2(Y, X)
    tp = np.tan(np.deg2rad(pitch_deg))
    if base == "exp":
        b = np.exp(-r / scale)
        db = -b / scale
    elif base == "kuzmin":
        q = 1.0 + (r / scale) ** 2
        b = q ** -1.5
        db = -3.0 * r / scale ** 2 * q ** -2.5
    else:
        raise ValueError(base)
    ph = 2 * th - np.log(r) / tp + phase
    f = 1.0 + amp * np.cos(ph)
    s = b * f
    ds_dr = db * f + b * amp * np.sin(ph) / (r * tp)
    ds_dth = -2.0 * amp * b * np.sin(ph)
    dsx = ds_dr * X / r - ds_dth * Y / (r * r)
    dsy = ds_dr * Y / r + ds_dth * X / (r * r)
    return s, dsx, dsy


def central_slopes(s, h):
    """Second-order differences of sampled s: central inside, one-sided at edges."""
    s = np.asarray(s, dtype=np.float64)
    return np.gradient(s, h, axis=1, edge_order=2), np.gradient(s, h, axis=0, edge_order=2)


def noisy_spiral(n, seed, noise=0.01):
    """Exponential spiral disk exp(-r/0.25)(1 + 0.1 cos(2 theta - ln r / tan 20deg))
    times (1 + noise xi), xi ~ N(0,1) per cell, clamped at 0; slopes by
    central differences.  Returns (sigma, dsx, dsy, h)."""
    X, Y = grid_centres(n)
    h = 2.0 / n
    s, _, _ = spiral(X, Y, "exp", 0.25, 0.1, 20.0, 0.0)
    rng = np.random.default_rng(seed)
    s = np.clip(s * (1.0 + noise * rng.standard_normal(s.shape)), 0.0, None)
    dsx, dsy = central_slopes(s, h)
    return s, dsx, dsy, h


def random_fields(n, seed, slopes=True):
    """Seeded random (sigma, dsx, dsy) on n x n (for property tests)."""
    rng = np.random.default_rng(seed)
    s = rng.random((n, n))
    if not slopes:
        return s, None, None
    return s, rng.standard_normal((n, n)), rng.standard_normal((n, n))


# ----------------------------------------------------------------------------
# composite AMR layouts
# ----------------------------------------------------------------------------


@dataclass
class Patch:
    """A rectangle of cells at refinement level ``level`` >= 1 (base = 0),
    with lower-left cell (i0, j0) in that level's global cell index."""
    level: int
    i0: int
    j0: int
    nx: int
    ny: int


@dataclass
class Block:
    level: int
    i0: int
    j0: int
    nx: int
    ny: int
    x0: float      # lower-left corner of the block
    y0: float
    h: float
    offset: int    # start of this block in the composite-packed arrays
    leaf_mask: np.ndarray = field(repr=False)  # (ny, nx) bool


@dataclass
class Layout:
    """Base n0 x n0 grid on [x0, x0 + n0 h0]^2 plus properly nested patches.

    Composite-packed arrays hold the base block first, then each patch in
    list order, each row-major [y, x]; covered (non-leaf) cells are present
    but ignored on input and zero on output.
    """
    n0: int
    nlevels: int
    patches: List[Patch]
    x0: float = -1.0
    y0: float = -1.0
    h0: float = None

    def __post_init__(self):
        if self.h0 is None:
            self.h0 = 2.0 / self.n0

    def h(self, level):
        return self.h0 / 2 ** level

    @property
    def n_finest(self):
        return self.n0 * 2 ** (self.nlevels - 1)

    def total(self):
        return self.n0 * self.n0 + sum(p.nx * p.ny for p in self.patches)

    def blocks(self):
        """Blocks in composite-packed order with their leaf masks."""
        out = []
        rects = [Patch(0, 0, 0, self.n0, self.n0)] + list(self.patches)
        # child footprints per level, in the parent level's cell index (ratio 2)
        foot = {}
        for c in self.patches:
            foot.setdefault(c.level, []).append((c.i0 // 2, c.j0 // 2, (c.i0 + c.nx + 1) // 2,
                                                 (c.j0 + c.ny + 1) // 2))
        foot = {l: np.array(v, dtype=np.int64) for l, v in foot.items()}
        off = 0
        for b in rects:
            h = self.h(b.level)
            mask = np.ones((b.ny, b.nx), dtype=bool)
            f = foot.get(b.level + 1)
            if f is not None:
                a0 = np.maximum(f[:, 0], b.i0)
                a1 = np.minimum(f[:, 2], b.i0 + b.nx)
                c0 = np.maximum(f[:, 1], b.j0)
                c1 = np.minimum(f[:, 3], b.j0 + b.ny)
                for k in np.nonzero((a0 < a1) & (c0 < c1))[0]:
                    mask[c0[k] - b.j0:c1[k] - b.j0, a0[k] - b.i0:a1[k] - b.i0] = False
            out.append(Block(b.level, b.i0, b.j0, b.nx, b.ny, self.x0 + b.i0 * h,
                             self.y0 + b.j0 * h, h, off, mask))
            off += b.nx * b.ny
        return out

    def nleaves(self):
        return int(sum(b.leaf_mask.sum() for b in self.blocks()))

    def leaf_mask(self):
        """Composite-packed boolean mask of leaf cells."""
        return np.concatenate([b.leaf_mask.ravel() for b in self.blocks()])

    def centres(self):
        """Composite-packed cell-centre coordinates (x, y), all cells."""
        xs, ys = [], []
        for b in self.blocks():
            X = b.x0 + (np.arange(b.nx) + 0.5) * b.h
            Y = b.y0 + (np.arange(b.ny) + 0.5) * b.h
            XX, YY = np.meshgrid(X, Y)
            xs.append(XX.ravel())
            ys.append(YY.ravel())
        return np.concatenate(xs), np.concatenate(ys)

    def areas(self):
        return np.concatenate([np.full(b.nx * b.ny, b.h * b.h) for b in self.blocks()])

    def sample(self, profile):
        """Evaluate profile(X, Y) -> (s, dsx, dsy) at every cell centre; covered
        cells are zeroed.  Returns composite-packed float64 arrays."""
        X, Y = self.centres()
        s, dx, dy = profile(X, Y)
        m = self.leaf_mask()
        return (np.where(m, s, 0.0), np.where(m, dx, 0.0), np.where(m, dy, 0.0))

    def validate(self):
        """Proper nesting: each level-l patch lies inside the union of level-(l-1)
        blocks, and same-level patches are disjoint."""
        for p in self.patches:
            if not (1 <= p.level < self.nlevels):
                return False
            n = self.n0 * 2 ** p.level
            if p.i0 < 0 or p.j0 < 0 or p.i0 + p.nx > n or p.j0 + p.ny > n:
                return False
            if p.i0 % 2 or p.j0 % 2 or p.nx % 2 or p.ny % 2:
                return False
        for l in range(1, self.nlevels):
            n = self.n0 * 2 ** l
            occ = np.zeros((n, n), dtype=np.int32)
            for p in self.patches:
                if p.level == l:
                    occ[p.j0:p.j0 + p.ny, p.i0:p.i0 + p.nx] += 1
            if occ.max(initial=0) > 1:
                return False
            if l >= 2:
                par = np.zeros((n // 2, n // 2), dtype=bool)
                for p in self.patches:
                    if p.level == l - 1:
                        par[p.j0:p.j0 + p.ny, p.i0:p.i0 + p.nx] = True
                for p in self.patches:
                    if p.level == l and not par[p.j0 // 2:(p.j0 + p.ny) // 2,
                                                p.i0 // 2:(p.i0 + p.nx) // 2].all():
                        return False
        return True


def flag_layout(profile, n0, nlevels, tile=16, thresh=0.1, x0=-1.0, y0=-1.0, h0=None):
    """Refine tiles of tile x tile parent cells into (2 tile)^2 child patches
    wherever max over the tile of h_parent |grad s| / s exceeds ``thresh``;
    level l+1 tiles are only taken inside level-l patches (proper nesting).
    Tiles are visited parent by parent, row-major within each parent."""
    if h0 is None:
        h0 = 2.0 / n0
    patches = []
    parents = [Patch(0, 0, 0, n0, n0)]
    for lvl in range(1, nlevels):
        hp = h0 / 2 ** (lvl - 1)
        new = []
        for par in parents:
            xs = x0 + (par.i0 + np.arange(par.nx) + 0.5) * hp
            ys = y0 + (par.j0 + np.arange(par.ny) + 0.5) * hp
            X, Y = np.meshgrid(xs, ys)
            s, dx, dy = profile(X, Y)
            with np.errstate(divide="ignore", invalid="ignore"):
                score = np.where(s > 0, hp * np.hypot(dx, dy) / s, 0.0)
            sc = score.reshape(par.ny // tile, tile, par.nx // tile, tile).max(axis=(1, 3))
            for tj, ti in np.argwhere(sc > thresh):
                new.append(Patch(lvl, 2 * (par.i0 + ti * tile), 2 * (par.j0 + tj * tile),
                                 2 * tile, 2 * tile))
        patches.extend(new)
        parents = new
        if not new:
            break
    return Layout(n0, nlevels, patches, x0, y0, h0)


def band_layout(n0, nlevels, centres, alpha, widths, x0=-1.0, y0=-1.0, h0=None):
    """Refinement around the edges of disks of radius ``alpha`` about each of
    ``centres`` (the D2 and D2,2 experiments of Section 3): every cell of level
    l (0 = base; at l >= 1 only cells that exist, i.e. children of refined
    cells) whose centre lies closer than ``widths[l]`` to one of the circles
    is split into 2 x 2 children.  Each run of consecutive refined cells along
    a row becomes one patch of 2 x 2k children, so the patches of a level are
    disjoint and nested in the level below."""
    if h0 is None:
        h0 = 2.0 / n0
    patches = []
    exists = np.ones((n0, n0), dtype=bool)
    for lvl in range(nlevels - 1):
        n = n0 << lvl
        h = h0 / 2 ** lvl
        c = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(x0 + c, y0 + c)
        d = np.full((n, n), np.inf)
        for cx, cy in centres:
            d = np.minimum(d, np.abs(np.hypot(X - cx, Y - cy) - alpha))
        flag = exists & (d < widths[lvl])
        del X, Y, d
        if not flag.any():
            break
        # runs of flagged cells along each row
        pad = np.zeros((n, 1), dtype=np.int8)
        edges = np.diff(np.concatenate([pad, flag.astype(np.int8), pad], axis=1), axis=1)
        rs, cs = np.nonzero(edges == 1)
        re, ce = np.nonzero(edges == -1)
        for j, i0, i1 in zip(rs, cs, ce):
            patches.append(Patch(lvl + 1, 2 * int(i0), 2 * int(j), 2 * int(i1 - i0), 2))
        exists = np.repeat(np.repeat(flag, 2, axis=0), 2, axis=1)
    return Layout(n0, nlevels, patches, x0, y0, h0)


def disk_centres(disk):
    """Centres of the D2 components: one disk at the origin (D2) or two at
    (0, +-0.5) (D2,2)."""
    return [(0.0, 0.0)] if disk == "d2" else [(0.0, 0.5), (0.0, -0.5)]


def _band_scale(disk):
    # the zone counts of the D2,2 experiments fit bands 0.8 times as wide as
    # those of D2 (equivalently, the D2 bands about circles of radius 0.2)
    return 1.0 if disk == "d2" else 0.8


def ilr_layout(n0, nlevels, disk="d2", alpha=0.25):
    """Independent level refinement (Section 3; reading): cells within 0.05
    of the disk edge are refined at the base level, within 0.025 at the next,
    the same physical band for every base size."""
    k = _band_scale(disk)
    return band_layout(n0, nlevels, disk_centres(disk), alpha,
                       [k * 0.05 / 2 ** l for l in range(nlevels)])


def vlr_layout(n0, nlevels, disk="d2", alpha=0.25):
    """Variable level refinement (Section 3; reading): the band is 12.8 cells
    of the level being refined (0.2 at a 128^2 base), so it narrows with
    every doubling of the base and with every level."""
    k = _band_scale(disk)
    h0 = 2.0 / n0
    return band_layout(n0, nlevels, disk_centres(disk), alpha,
                       [k * 12.8 * h0 / 2 ** l for l in range(nlevels)])


def clumps(seed, n=8, rmax=0.7):
    """Seeded Gaussian clumps A exp(-|x - xk|^2 / (2 w^2)): A ~ U[1,10],
    w ~ U[0.01, 0.04], centres uniform in the disk r < rmax."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(1, 10, n)
    w = rng.uniform(0.01, 0.04, n)
    r = rmax * np.sqrt(rng.random(n))
    t = rng.uniform(0, 2 * np.pi, n)
    return A, w, r * np.cos(t), r * np.sin(t)


def kuzmin_clumps_profile(seed, a=0.02, nclumps=8):
    """Kuzmin disk (M = 1, scale a) plus seeded Gaussian clumps, exact gradient."""
    A, w, cx, cy = clumps(seed, nclumps)

    def prof(X, Y):
        s, dx, dy = kuzmin(X, Y, 1.0, a)
        for k in range(len(A)):
            e = A[k] * np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2) / (2 * w[k] ** 2))
            s = s + e
            dx = dx - e * (X - cx[k]) / w[k] ** 2
            dy = dy - e * (Y - cy[k]) / w[k] ** 2
        return s, dx, dy

    return prof


def amr_config(seed, n0=256, nlevels=3, thresh=0.1, a=0.02):
    """3-level AMR workload: base n0^2 on [-1,1]^2, 32x32 child patches flagged
    by h |grad s| / s > thresh, Kuzmin (a) plus clumps, exact slopes."""
    prof = kuzmin_clumps_profile(seed, a)
    lay = flag_layout(prof, n0, nlevels, 16, thresh)
    s, dx, dy = lay.sample(prof)
    return lay, s, dx, dy


def table10_layout():
    """The paper's Appendix A example: 4 x 4 base on [0,1]^2; base cells 6 and
    11 (1-based, row-major) refined to level 2; level-2 cells 17 and 19
    (x in [0.25,0.375] y in [0.375,0.5], and x in [0.375,0.5] y in [0.25,0.375])
    refined to level 3.  28 leaves (14 / 6 / 8)."""
    patches = [Patch(1, 2, 2, 2, 2), Patch(1, 4, 4, 2, 2),
               Patch(2, 4, 6, 2, 2), Patch(2, 6, 4, 2, 2)]
    return Layout(4, 3, patches, 0.0, 0.0, 0.25)


# ----------------------------------------------------------------------------
# batches and request streams
# ----------------------------------------------------------------------------


def batch_disks(seed, count=64, sizes=(64, 128, 256, 512, 1024)):
    """Independent uniform disks: n ~ U(sizes), profile exponential or
    Kuzmin-like (p = 1/2), scale ~ U[0.05, 0.5], m = 2 amplitude ~ U[0, 0.2],
    phase ~ U[0, 2 pi), exact slopes.  Returns a list of (n, s, dsx, dsy)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        base = "exp" if rng.random() < 0.5 else "kuzmin"
        scale = rng.uniform(0.05, 0.5)
        amp = rng.uniform(0.0, 0.2)
        ph = rng.uniform(0, 2 * np.pi)
        X, Y = grid_centres(n)
        s, dx, dy = spiral(X, Y, base, scale, amp, 20.0, ph)
        out.append((n, s, dx, dy))
    return out


def limit_layout(lay, max_patches, rng):
    """Keep at most max_patches patches, preserving nesting: patches are kept
    level by level, each only if its parent region survived."""
    kept = []
    for lvl in range(1, lay.nlevels):
        cand = [p for p in lay.patches if p.level == lvl]
        if lvl > 1:
            par = [p for p in kept if p.level == lvl - 1]

            def inside(c):
                return any(q.i0 <= c.i0 // 2 and c.i0 // 2 + c.nx // 2 <= q.i0 + q.nx and
                           q.j0 <= c.j0 // 2 and c.j0 // 2 + c.ny // 2 <= q.j0 + q.ny for q in par)
            cand = [c for c in cand if inside(c)]
        room = max_patches - len(kept)
        if room <= 0:
            break
        if len(cand) > room:
            idx = sorted(rng.choice(len(cand), room, replace=False))
            cand = [cand[i] for i in idx]
        kept.extend(cand)
    used = max([p.level for p in kept], default=0) + 1
    return Layout(lay.n0, max(used, 1) if kept else 1, kept, lay.x0, lay.y0, lay.h0)


def limit_layout_all_levels(lay, max_patches, rng):
    """Keep at most max_patches patches (at least one per level), preserving
    nesting and every level of ``lay``: one chain of patches from level 1 to
    the deepest level is kept first, then the remaining room is filled level
    by level with random patches nested in those already kept."""
    if not lay.patches:
        return lay
    deepest = max(p.level for p in lay.patches)

    def inside(c, par):
        return any(q.i0 <= c.i0 // 2 and c.i0 // 2 + c.nx // 2 <= q.i0 + q.nx and
                   q.j0 <= c.j0 // 2 and c.j0 // 2 + c.ny // 2 <= q.j0 + q.ny for q in par)
    chain = [next(p for p in lay.patches if p.level == deepest)]
    for lvl in range(deepest - 1, 0, -1):
        chain.append(next(p for p in lay.patches if p.level == lvl and inside(chain[-1], [p])))
    kept = list(reversed(chain))
    room = max(max_patches, deepest) - len(kept)
    for lvl in range(1, deepest + 1):
        par = [p for p in kept if p.level == lvl - 1]
        cand = [c for c in lay.patches if c.level == lvl and c not in kept and
                (lvl == 1 or inside(c, par))]
        take = min(room, len(cand), int(rng.integers(0, room + 1)) if lvl < deepest else room)
        if take > 0:
            idx = sorted(rng.choice(len(cand), take, replace=False))
            kept.extend(cand[i] for i in idx)
            room -= take
    kept.sort(key=lambda p: p.level)
    return Layout(lay.n0, deepest + 1, kept, lay.x0, lay.y0, lay.h0)


def request_pool_full(seed, bases=(128, 256, 512, 1024, 2048), levels=(1, 2, 3, 4)):
    """The served-stream mix over every base size and level count: one layout
    per (base, levels) pair, 32x32 child patches flagged on a Kuzmin (scale a
    ~ U[0.02, 0.2]) plus clumps profile, capped at 4..256 patches (log-
    uniform) with every level kept.  Returns a list of (layout, profile)."""
    rng = np.random.default_rng(seed)
    out = []
    for n0 in bases:
        for lv in levels:
            a = float(rng.uniform(0.02, 0.2))
            prof = kuzmin_clumps_profile(int(rng.integers(1 << 30)), a)
            if lv == 1:
                out.append((Layout(n0, 1, []), prof))
                continue
            thresh = 0.05
            full = flag_layout(prof, n0, lv, 16, thresh)
            while max((p.level for p in full.patches), default=0) < lv - 1 and thresh > 1e-4:
                thresh *= 0.5
                full = flag_layout(prof, n0, lv, 16, thresh)
            cap = int(np.exp(rng.uniform(np.log(4), np.log(256))))
            out.append((limit_layout_all_levels(full, cap, rng), prof))
    return out


def request_pool(seed, count=12, bases=(128, 256, 512, 1024, 2048), max_finest=4096):
    """Distinct AMR request layouts for a served stream: base n0 from `bases`,
    1-4 levels with n0 * 2^(levels-1) <= max_finest, 32x32 child patches
    flagged on a Kuzmin (scale a ~ U[0.02, 0.2]) plus clumps profile and
    capped at 4..256 patches.  Returns a list of (layout, profile)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n0 = int(rng.choice(bases))
        lv_max = 1
        while lv_max < 4 and n0 * 2 ** lv_max <= max_finest:
            lv_max += 1
        levels = int(rng.integers(1, lv_max + 1))
        a = float(rng.uniform(0.02, 0.2))
        prof = kuzmin_clumps_profile(int(rng.integers(1 << 30)), a)
        if levels == 1:
            lay = Layout(n0, 1, [])
        else:
            full = flag_layout(prof, n0, levels, 16, 0.05)
            cap = int(np.exp(rng.uniform(np.log(4), np.log(256))))
            lay = limit_layout(full, cap, rng)
        out.append((lay, prof))
    return out
