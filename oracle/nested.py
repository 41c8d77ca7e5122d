"""Step-by-step CPU oracle of the nested-correction AMR solve (test
infrastructure only: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the product library never does).

What is approximated: the force at every leaf centre of a Berger-Oliger
composite grid (Section 3: leaves of refinement ratio 2, each with the
first-order Taylor density of Section 2) from all leaves, whose exact value
is the leaf-by-leaf direct sum of Section 2 (``oracle.direct``).  The paper
computes that sum directly and states that FFTs do not apply to AMR grids
(Section 4).  This scheme evaluates it approximately with uniform-lattice
convolutions only, each of which is an exact free-space sum of Section 2
kernels, so its cost follows the refined area instead of the finest
lattice.  Every step below is FP64 and every convolution is a plain direct
sum (``oracle.uniform`` / ``oracle.direct``); there is no FFT here.

Definitions (levels l = 0 .. L-1, level-l cell size h_l = h0 / 2^l, level-l
cells = the base grid (l = 0) or the cells of level-l patches):

1. Restriction, from the finest level down: every covered level-(l-1) cell
   gets the linear density of least squares distance to its four children's
   linear pieces (children that are covered themselves already carry their
   restricted values).  With h the parent size, d = h/4 the children's
   centre offsets, s_c, dsx_c, dsy_c the children's data:
       s   = mean of s_c                                  (mass)
       dsx = 3/(4h) (sum of right s_c - sum of left s_c) + sum dsx_c / 16
       dsy = 3/(4h) (sum of upper s_c - sum of lower s_c) + sum dsy_c / 16
   which conserves the mass and both first moments of the four children and
   reproduces any linear density exactly.
2. The level-l truncated composite is the layout with every patch of level
   > l removed: its leaves are the level-l cells and the coarser leaves, with
   the restricted data on level-l cells that are covered.
3. Level 0: F^0 = the exact force of the level-0 truncated composite (the
   base grid with restricted data) at every base cell centre.
4. Level l >= 1, in boxes: the level-l lattice is tiled by T x T boxes
   (T = 64, aligned to multiples of T); every box holding a level-l cell is
   solved.  Its extended region is the box grown by W = 32 level-l cells on
   every side (clipped to the domain).  For each level-l cell c of the box:
       F^l(c) = Ffine(c) + sum_k w_k [F^{l-1}(p_k) - Fcoarse(p_k)]
   Ffine: exact force at c of the level-l truncated composite inside the
   extended region (cells crossing the region's edge clipped to it, their
   linear density kept);  Fcoarse: the same for the level-(l-1) truncated
   composite inside the same region, at the parent-level cells p_k;  the
   bracket is the force of everything outside the region, smooth across the
   box, interpolated to c with the stencil of ``stencil``.
5. Each leaf takes F^l of its own level; covered cells are 0.

The only approximations are the restriction (step 1: exact in mass and first
moments) and the interpolation of the far field (step 4).
"""
import numpy as np

from . import direct as _direct
from . import uniform as _uniform

T_BOX = 64   # box side, level-l cells
W_EXT = 32   # extension of each box on every side, level-l cells


def cell_maps(lay):
    """Per level l: an (n_l, n_l) array of composite indices of the level-l
    cells, -1 where level l has no cell."""
    maps = []
    for l in range(lay.nlevels):
        n = lay.n0 << l
        m = np.full((n, n), -1, dtype=np.int64)
        maps.append(m)
    maps[0][:, :] = np.arange(lay.n0 * lay.n0).reshape(lay.n0, lay.n0)
    off = lay.n0 * lay.n0
    for p in lay.patches:
        blk = off + np.arange(p.nx * p.ny).reshape(p.ny, p.nx)
        maps[p.level][p.j0:p.j0 + p.ny, p.i0:p.i0 + p.nx] = blk
        off += p.nx * p.ny
    return maps


def restrict(lay, s, dsx, dsy):
    """Step 1: composite arrays with every covered cell replaced by the
    restriction of its children, finest level first."""
    s, dsx, dsy = (np.array(a, dtype=np.float64, copy=True) for a in (s, dsx, dsy))
    maps = cell_maps(lay)
    for l in range(lay.nlevels - 1, 0, -1):
        h = lay.h0 / 2 ** (l - 1)          # parent cell size
        fine, par = maps[l], maps[l - 1]
        n = par.shape[0]
        for J in range(n):
            for I in range(n):
                c00 = fine[2 * J, 2 * I] if 2 * J < fine.shape[0] else -1
                if par[J, I] < 0 or c00 < 0:
                    continue
                # children (a, b): x offset a, y offset b; left a = 0, lower b = 0
                ch = [[fine[2 * J + b, 2 * I + a] for a in range(2)] for b in range(2)]
                sc = [[s[ch[b][a]] for a in range(2)] for b in range(2)]
                p = par[J, I]
                s[p] = (sc[0][0] + sc[0][1] + sc[1][0] + sc[1][1]) / 4.0
                right = sc[0][1] + sc[1][1]
                left = sc[0][0] + sc[1][0]
                upper = sc[1][0] + sc[1][1]
                lower = sc[0][0] + sc[0][1]
                sx = sum(dsx[ch[b][a]] for a in range(2) for b in range(2))
                sy = sum(dsy[ch[b][a]] for a in range(2) for b in range(2))
                dsx[p] = 3.0 / (4.0 * h) * (right - left) + sx / 16.0
                dsy[p] = 3.0 / (4.0 * h) * (upper - lower) + sy / 16.0
    return s, dsx, dsy


def truncated_sources(lay, maps, vals, l, X0, X1, Y0, Y1):
    """Step 2 and the clipping of step 4: the leaves of the level-l truncated
    composite inside the level-l index rectangle [X0, X1) x [Y0, Y1), as
    source rectangles (xl, xr, yd, yu) with their linear data re-expanded
    about the centre of the part inside the rectangle."""
    s, dsx, dsy = vals
    hl = lay.h0 / 2 ** l
    rx0, rx1 = lay.x0 + X0 * hl, lay.x0 + X1 * hl
    ry0, ry1 = lay.y0 + Y0 * hl, lay.y0 + Y1 * hl
    rects, ss, xs, ys = [], [], [], []
    for k in range(l + 1):
        hk = lay.h0 / 2 ** k
        m = maps[k]
        n = m.shape[0]
        sh = l - k
        i0, i1 = max(0, X0 >> sh), min(n, -((-X1) >> sh))
        j0, j1 = max(0, Y0 >> sh), min(n, -((-Y1) >> sh))
        if i0 >= i1 or j0 >= j1:
            continue
        sub = m[j0:j1, i0:i1]
        J, I = np.nonzero(sub >= 0)
        I, J = I + i0, J + j0
        if k < l:   # leaves of the truncated composite only: not covered at level k + 1
            fm = maps[k + 1]
            cov = fm[np.minimum(2 * J, fm.shape[0] - 1), np.minimum(2 * I, fm.shape[0] - 1)] >= 0
            I, J = I[~cov], J[~cov]
        c = m[J, I]
        xl, xr = lay.x0 + I * hk, lay.x0 + (I + 1) * hk
        yd, yu = lay.y0 + J * hk, lay.y0 + (J + 1) * hk
        xc, yc = 0.5 * (xl + xr), 0.5 * (yd + yu)
        cxl, cxr = np.maximum(xl, rx0), np.minimum(xr, rx1)
        cyd, cyu = np.maximum(yd, ry0), np.minimum(yu, ry1)
        keep = (cxl < cxr) & (cyd < cyu)
        cxl, cxr, cyd, cyu, c, xc, yc = (a[keep] for a in (cxl, cxr, cyd, cyu, c, xc, yc))
        s2 = s[c] + dsx[c] * (0.5 * (cxl + cxr) - xc) + dsy[c] * (0.5 * (cyd + cyu) - yc)
        rects.append(np.stack([cxl, cxr, cyd, cyu], 1))
        ss.append(s2)
        xs.append(dsx[c])
        ys.append(dsy[c])
    if not rects:
        return np.zeros((0, 4)), np.zeros(0), np.zeros(0), np.zeros(0)
    return np.concatenate(rects), np.concatenate(ss), np.concatenate(xs), np.concatenate(ys)


def stencil(avail, I, J, sx, sy):
    """Interpolation of a parent-level field to the child centre at offset
    (sx, sy) / 4 parent cells from parent (I, J) (sx, sy = +-1), from the
    parent-level cells for which avail(I', J') holds ((I, J) always does).
    Tried in order:
      biquadratic on the 3 x 3 cells about (I, J), if all are available:
      the tensor product of the 3-point Lagrange weights at t = s/4 on the
      nodes -1, 0, 1, i.e. (-3/32, 15/16, 5/32) for s = +1, mirrored for -1;
    then, each over the neighbour directions (ex, ey) = (sx, sy), (-sx, sy),
    (sx, -sy), (-sx, -sy), with a = sx ex / 4, b = sy ey / 4:
      bilinear on (I,J), (I+ex,J), (I,J+ey), (I+ex,J+ey);
      the plane through (I,J), (I+ex,J), (I,J+ey);
      linear in x on (I,J), (I+ex,J), then linear in y on (I,J), (I,J+ey);
      the value at (I, J).
    Returns [(I', J', weight)]."""
    if all(avail(I + a, J + b) for a in (-1, 0, 1) for b in (-1, 0, 1)):
        wx = {-sx: -3.0 / 32.0, 0: 15.0 / 16.0, sx: 5.0 / 32.0}
        wy = {-sy: -3.0 / 32.0, 0: 15.0 / 16.0, sy: 5.0 / 32.0}
        return [(I + a, J + b, wx[a] * wy[b]) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    dirs = [(sx, sy), (-sx, sy), (sx, -sy), (-sx, -sy)]
    for ex, ey in dirs:
        if avail(I + ex, J) and avail(I, J + ey) and avail(I + ex, J + ey):
            a, b = sx * ex / 4.0, sy * ey / 4.0
            return [(I, J, (1 - a) * (1 - b)), (I + ex, J, a * (1 - b)),
                    (I, J + ey, (1 - a) * b), (I + ex, J + ey, a * b)]
    for ex, ey in dirs:
        if avail(I + ex, J) and avail(I, J + ey):
            a, b = sx * ex / 4.0, sy * ey / 4.0
            return [(I, J, 1 - a - b), (I + ex, J, a), (I, J + ey, b)]
    for ex in (sx, -sx):
        if avail(I + ex, J):
            a = sx * ex / 4.0
            return [(I, J, 1 - a), (I + ex, J, a)]
    for ey in (sy, -sy):
        if avail(I, J + ey):
            b = sy * ey / 4.0
            return [(I, J, 1 - b), (I, J + ey, b)]
    return [(I, J, 1.0)]


def boxes(lay, maps, l):
    """Step 4: the (bx, by) indices of the T x T boxes holding level-l cells."""
    m = maps[l]
    J, I = np.nonzero(m >= 0)
    return sorted(set(zip((I // T_BOX).tolist(), (J // T_BOX).tolist())), key=lambda b: (b[1], b[0]))


def nested(lay, s, dsx, dsy, G=1.0, threads=0):
    """The nested-correction force at every composite cell (leaves; covered
    cells 0).  Returns (fx, fy) composite-packed."""
    maps = cell_maps(lay)
    vals = restrict(lay, s, dsx, dsy)
    ncell = lay.total()
    Fx = np.zeros(ncell)
    Fy = np.zeros(ncell)
    # level 0: exact force of the restricted base grid at every base cell
    n0 = lay.n0
    b = slice(0, n0 * n0)
    fx0, fy0 = _uniform(vals[0][b].reshape(n0, n0), vals[1][b].reshape(n0, n0),
                        vals[2][b].reshape(n0, n0), lay.x0, lay.y0, lay.h0, G=G, threads=threads)
    Fx[b] = fx0.ravel()
    Fy[b] = fy0.ravel()
    for l in range(1, lay.nlevels):
        hl = lay.h0 / 2 ** l
        nl = n0 << l
        fine, par = maps[l], maps[l - 1]

        def avail(I, J, par=par):
            return 0 <= I < par.shape[0] and 0 <= J < par.shape[0] and par[J, I] >= 0
        for bx, by in boxes(lay, maps, l):
            X0, Y0 = bx * T_BOX, by * T_BOX
            EX0, EX1 = max(0, X0 - W_EXT), min(nl, X0 + T_BOX + W_EXT)
            EY0, EY1 = max(0, Y0 - W_EXT), min(nl, Y0 + T_BOX + W_EXT)
            sub = fine[Y0:min(nl, Y0 + T_BOX), X0:min(nl, X0 + T_BOX)]
            jj, ii = np.nonzero(sub >= 0)
            ii, jj = ii + X0, jj + Y0
            cells = fine[jj, ii]
            tx = lay.x0 + (ii + 0.5) * hl
            ty = lay.y0 + (jj + 0.5) * hl
            src = truncated_sources(lay, maps, vals, l, EX0, EX1, EY0, EY1)
            ffx, ffy = _direct(src[0], src[1], src[2], src[3], np.stack([tx, ty], 1), G=G,
                               threads=threads)
            # interpolation stencils on the parent level
            sts = [stencil(avail, i >> 1, j >> 1, 1 if i & 1 else -1, 1 if j & 1 else -1)
                   for i, j in zip(ii.tolist(), jj.tolist())]
            pset = sorted({(I, J) for st in sts for (I, J, _) in st})
            pidx = {p: k for k, p in enumerate(pset)}
            hp = lay.h0 / 2 ** (l - 1)
            px = np.array([lay.x0 + (I + 0.5) * hp for I, _ in pset])
            py = np.array([lay.y0 + (J + 0.5) * hp for _, J in pset])
            csrc = truncated_sources(lay, maps, vals, l - 1, EX0 // 2, -((-EX1) // 2),
                                     EY0 // 2, -((-EY1) // 2))
            cfx, cfy = _direct(csrc[0], csrc[1], csrc[2], csrc[3], np.stack([px, py], 1), G=G,
                               threads=threads)
            pc = np.array([par[J, I] for I, J in pset])
            ex = Fx[pc] - cfx
            ey = Fy[pc] - cfy
            for k, (c, st) in enumerate(zip(cells.tolist(), sts)):
                Fx[c] = ffx[k] + sum(w * ex[pidx[(I, J)]] for I, J, w in st)
                Fy[c] = ffy[k] + sum(w * ey[pidx[(I, J)]] for I, J, w in st)
    leaf = lay.leaf_mask()
    return np.where(leaf, Fx, 0.0), np.where(leaf, Fy, 0.0)
