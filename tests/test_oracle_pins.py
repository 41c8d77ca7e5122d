"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what it pins.  Together they are chosen so that a plausible
mistake in the oracle (a flipped sign, a dropped slope term, a wrong offset, a
transposed family, a wrong edge convention) fails at least one of them:

* exact kernels vs numerical quadrature of their defining integrals (Section 2)
* the self-cell closed forms (symmetry and an elementary integral)
* the far-field limit and a 30-digit quadrature of far entries (precision)
* Table 1 of the paper (D2 disk, uniform grid): printed error norms
* Table 2 of the paper (D2,2): printed L1 norms
* Kuzmin disk of the bench config 1, after removing the exterior mass
* additivity over cells, symmetry, Newton's third law, linearity
* AMR layout invariance on the paper's Appendix A layout
"""
import math
import os

import numpy as np
import pytest

import diskgen
import oracle
from oracle import analytic as an

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graded(lo, hi, p, d0):
    p = min(max(p, lo), hi)
    pts = {lo, hi, p}
    s = d0
    while p + s < hi:
        pts.add(p + s)
        s *= 2
    s = d0
    while p - s > lo:
        pts.add(p - s)
        s *= 2
    return np.array(sorted(pts))


def quad_kernels(xt, yt, xl, xr, yd, yu, npts=20):
    """Composite Gauss-Legendre integration of the six defining integrands of
    Section 2 over the source rectangle, graded towards the target."""
    g, w = np.polynomial.legendre.leggauss(npts)
    d0 = 0.25 * max(min(abs(xl - xt), abs(xr - xt), abs(yd - yt), abs(yu - yt)),
                    1e-3 * (xr - xl))

    def nodes(lo, hi, p):
        b = _graded(lo, hi, p, d0)
        a = 0.5 * (b[1:] - b[:-1])
        c = 0.5 * (b[1:] + b[:-1])
        return (c[:, None] + a[:, None] * g).ravel(), (a[:, None] * w).ravel()

    xs, wx = nodes(xl, xr, xt)
    ys, wy = nodes(yd, yu, yt)
    XB, YB = np.meshgrid(xs, ys)
    W = wy[:, None] * wx[None, :]
    u = XB - xt
    v = YB - yt
    r3 = (u * u + v * v) ** 1.5
    xc, yc = 0.5 * (xl + xr), 0.5 * (yd + yu)
    return np.array([np.sum(W * u / r3), np.sum(W * (XB - xc) * u / r3),
                     np.sum(W * (YB - yc) * u / r3), np.sum(W * v / r3),
                     np.sum(W * (XB - xc) * v / r3), np.sum(W * (YB - yc) * v / r3)])


@pytest.mark.parametrize("case", [
    # (target, source rectangle): separated, adjacent, diagonal, on an edge line
    ((0.0, 0.0), (3.0, 4.0, -1.0, 0.5)),
    ((0.1, -0.2), (-2.5, -1.5, 1.0, 1.75)),
    ((0.0, 0.0), (0.5, 1.5, -0.5, 0.5)),       # right neighbour of a unit cell
    ((0.0, 0.0), (-0.5, 0.5, 0.5, 1.5)),       # upper neighbour
    ((0.0, 0.0), (0.5, 1.5, 0.5, 1.5)),        # diagonal neighbour
    ((0.0, 0.0), (0.0, 1.0, 2.0, 3.0)),        # x-bar = x on the left edge line
    ((0.0, 0.0), (0.5, 2.0, 0.0, 0.25)),       # y-bar = y on the lower edge line
    ((0.3, 0.7), (-7.0, -6.0, 11.0, 13.0)),
])
def test_kernels_match_quadrature(case):
    (xt, yt), (xl, xr, yd, yu) = case
    k = oracle.cell_kernels(xt, yt, xl, xr, yd, yu)
    q = quad_kernels(xt, yt, xl, xr, yd, yu)
    scale = np.max(np.abs(q[[0, 3]]))
    np.testing.assert_allclose(k, q, rtol=1e-9, atol=1e-11 * scale)


def test_self_cell_closed_form():
    # target at the centre of its own cell: odd integrands vanish, and
    # int u^2/r^3 over [-a,a]^2 = 4 a ln(1 + sqrt 2)
    h = 0.375
    k = oracle.cell_kernels(1.0, 2.0, 1.0 - h / 2, 1.0 + h / 2, 2.0 - h / 2, 2.0 + h / 2)
    iuu = 2.0 * h * math.log1p(math.sqrt(2.0))
    np.testing.assert_allclose(k, [0.0, iuu, 0.0, 0.0, 0.0, iuu], atol=1e-15)


def test_boundary_target_rejected():
    with pytest.raises(ValueError):
        oracle.cell_kernels(0.0, 0.0, 0.0, 1.0, -0.5, 0.5)   # on the left edge
    with pytest.raises(ValueError):
        oracle.cell_kernels(0.0, 0.0, 0.0, 1.0, 0.0, 1.0)    # on a corner


def test_far_field_limit():
    # the cell integral of u/r^3 tends to the point-mass value dx/|d|^3
    for dx, dy in [(40, 30), (-90, 17), (5, -120)]:
        k = oracle.cell_kernels(0, 0, dx - 0.5, dx + 0.5, dy - 0.5, dy + 0.5)
        d3 = (dx * dx + dy * dy) ** 1.5
        assert abs(k[0] - dx / d3) < 1e-3 * abs(dx / d3) + 1e-12
        assert abs(k[3] - dy / d3) < 1e-3 * abs(dy / d3) + 1e-12


def test_far_entries_precision_vs_30_digit_quadrature():
    # the double difference cancels ~2 log10(d) digits; the oracle must still
    # give far entries to a few 1e-15 absolute (plain double gives ~1e-12 on Kxx)
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    # the last two cases are nearly axis-aligned, where ln(a + R) with a < 0
    # cancels unless it is evaluated in its stable form
    for dx, dy in [(1000, -700), (-1500, 1300), (2, -1200), (-1300, 1)]:
        k = oracle.cell_kernels(0, 0, dx - 0.5, dx + 0.5, dy - 0.5, dy + 0.5)

        def integ(f):
            return mp.quad(lambda x: mp.quad(lambda y: f(x, y), [dy - 0.5, dy + 0.5]),
                           [dx - 0.5, dx + 0.5])
        r3 = lambda x, y: (x * x + y * y) ** mp.mpf(1.5)
        ref = [integ(lambda x, y: x / r3(x, y)),
               integ(lambda x, y: (x - dx) * x / r3(x, y)),
               integ(lambda x, y: (y - dy) * x / r3(x, y))]
        assert abs(k[0] - float(ref[0])) < 1e-18
        assert abs(k[1] - float(ref[1])) < 5e-15
        assert abs(k[2] - float(ref[2])) < 5e-15


def test_far_entry_error_bound():
    """The stated per-entry accuracy of the oracle's kernels far from the
    target (the double differences cancel and the first-moment kernels
    subtract two terms of the monopole's size; the x87 extended precision
    leaves, with d the offset in cells and S = |K^{x,0}| + |K^{y,0}|): each
    centre kernel within 1e-18 d^2 S and each first-moment kernel within
    1e-14 d^2 S h of the 40-digit quadrature of its integrand (measured up
    to 6000 cells: 4e-19 and 5.4e-15).  At 4096-cell offsets that is 1.7e-11
    and 1.7e-7 of S (h = 1); such entries are small next to the near-field
    ones, so the sums stay far inside the 1e-12 parity bar."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for D, k in [(1000, 7), (11, 4000), (-4095, 11), (6000, 100)]:
        xl, xr, yd, yu = D - 0.5, D + 0.5, k - 0.5, k + 0.5
        r3 = lambda x, y: (x * x + y * y) ** mp.mpf(1.5)
        fs = [lambda x, y: x / r3(x, y), lambda x, y: (x - D) * x / r3(x, y),
              lambda x, y: (y - k) * x / r3(x, y), lambda x, y: y / r3(x, y),
              lambda x, y: (x - D) * y / r3(x, y), lambda x, y: (y - k) * y / r3(x, y)]
        ref = [float(mp.quad(f, [xl, xr], [yd, yu])) for f in fs]
        got = oracle.cell_kernels(0.0, 0.0, xl, xr, yd, yu)
        d2 = float(D * D + k * k)
        S = abs(ref[0]) + abs(ref[3])
        for i in (0, 3):
            assert abs(got[i] - ref[i]) <= 1e-18 * d2 * S, (D, k, i)
        for i in (1, 2, 4, 5):
            assert abs(got[i] - ref[i]) <= 1e-14 * d2 * S, (D, k, i)


def _load_table(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return {int(r[0]): [float(x) for x in r[1:]] for r in rows}


def _d2_errors(n, disk):
    X, Y = diskgen.grid_centres(n)
    prof = diskgen.d2 if disk == "d2" else diskgen.d22
    s, dx, dy = prof(X, Y)
    fx, fy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    ax, ay = (an.d2_force if disk == "d2" else an.d22_force)(X, Y)
    R = np.hypot(X, Y)
    fr = (fx * X + fy * Y) / R
    ar = (ax * X + ay * Y) / R
    A = (2.0 / n) ** 2
    return an.norms(fx - ax, A), an.norms(fy - ay, A), an.norms(fr - ar, A)


def test_table1_d2_uniform():
    """Table 1, row N_k = 128 (a 256^2 grid): max norms and L2 to the three
    printed digits, L1 within 3% (the area-weight reading is in the fixture)."""
    paper = _load_table("table1_d2.txt")[128]
    (x1, x2, xi), _, (r1, r2, ri) = _d2_errors(256, "d2")
    assert abs(xi - paper[2]) <= 0.006e-3
    assert abs(ri - paper[5]) <= 0.006e-3
    assert abs(2 * x2 - paper[1]) <= 0.006e-4
    assert abs(2 * r2 - paper[4]) <= 0.006e-3
    assert abs(4 * x1 / paper[0] - 1) < 0.03
    assert abs(4 * r1 / paper[3] - 1) < 0.03


def test_d2_second_order():
    # orders of Table 1 are near 2 in L1 and L2; check 64 -> 128 cells per side
    (a1, a2, _), _, _ = _d2_errors(64, "d2")
    (b1, b2, _), _, _ = _d2_errors(128, "d2")
    assert math.log2(a1 / b1) > 1.8
    assert math.log2(a2 / b2) > 1.7


def test_table2_d22_l1():
    """Table 2, row N_k = 128: the L1 norms (x, y, R) within 5%.  L2 and max
    norms of Table 2 are not reproduced by this reading (parity unpinned)."""
    paper = _load_table("table2_d22.txt")[128]
    (x1, _, _), (y1, _, _), (r1, _, _) = _d2_errors(256, "d22")
    assert abs(4 * x1 / paper[0] - 1) < 0.05
    assert abs(4 * y1 / paper[3] - 1) < 0.05
    assert abs(4 * r1 / paper[6] - 1) < 0.05


def test_kuzmin_truncated():
    """Kuzmin disk M = 1, a = 0.2 on [-1,1]^2: against the analytic force minus
    the force of the mass outside the square, the error is discretisation
    error (second order); against the untruncated force it stalls near 1.4%."""
    errs = []
    for n in (32, 64):
        X, Y = diskgen.grid_centres(n)
        s, dx, dy = diskgen.kuzmin(X, Y, 1.0, 0.2)
        fx, fy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
        tx, ty = an.kuzmin_truncated_force(X, Y)
        kx, ky = an.kuzmin_force(X, Y)
        errs.append(an.rel_l2((fx, fy), (tx, ty)))
        assert 0.012 < an.rel_l2((fx, fy), (kx, ky)) < 0.02
    assert errs[1] < 4e-3
    assert errs[0] / errs[1] > 3.3


def test_additivity_constant_and_linear():
    """Integral additivity: a density linear on a block of cells (with its exact
    slopes) gives at every target the closed form of the whole block."""
    n, h = 16, 0.125
    i0, i1, j0, j1 = 3, 11, 5, 9
    X, Y = diskgen.grid_centres(n, -1.0, -1.0, h)
    a, b, c = 0.7, -1.3, 2.1
    s = np.zeros((n, n))
    s[j0:j1, i0:i1] = a + b * X[j0:j1, i0:i1] + c * Y[j0:j1, i0:i1]
    dx = np.zeros((n, n))
    dy = np.zeros((n, n))
    dx[j0:j1, i0:i1] = b
    dy[j0:j1, i0:i1] = c
    fx, fy = oracle.uniform(s, dx, dy, -1.0, -1.0, h)
    xl, xr, yd, yu = -1 + i0 * h, -1 + i1 * h, -1 + j0 * h, -1 + j1 * h
    sc = a + b * 0.5 * (xl + xr) + c * 0.5 * (yd + yu)
    ex = np.zeros((n, n))
    ey = np.zeros((n, n))
    for j in range(n):
        for i in range(n):
            k = oracle.cell_kernels(X[j, i], Y[j, i], xl, xr, yd, yu)
            ex[j, i] = sc * k[0] + b * k[1] + c * k[2]
            ey[j, i] = sc * k[3] + b * k[4] + c * k[5]
    scale = np.max(np.abs(ex)) + np.max(np.abs(ey))
    assert np.max(np.abs(fx - ex)) < 1e-13 * scale
    assert np.max(np.abs(fy - ey)) < 1e-13 * scale


def test_mirror_and_transpose_symmetry():
    n = 24
    rng = np.random.default_rng(5)
    half = rng.random((n, n // 2))
    s = np.concatenate([half, half[:, ::-1]], axis=1)          # even in x
    hx = rng.standard_normal((n, n // 2))
    dx = np.concatenate([hx, -hx[:, ::-1]], axis=1)            # odd in x
    hy = rng.standard_normal((n, n // 2))
    dy = np.concatenate([hy, hy[:, ::-1]], axis=1)             # even in x
    fx, fy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    sc = np.max(np.abs(fx))
    assert np.max(np.abs(fx + fx[:, ::-1])) < 1e-13 * sc
    assert np.max(np.abs(fy - fy[:, ::-1])) < 1e-13 * sc
    # transposing the density (and swapping slopes) transposes and swaps F
    s2, dx2, dy2 = diskgen.random_fields(n, 9)
    gx, gy = oracle.uniform(s2, dx2, dy2, -1.0, -1.0, 2.0 / n)
    tx, ty = oracle.uniform(s2.T, dy2.T, dx2.T, -1.0, -1.0, 2.0 / n)
    sc = np.max(np.abs(gx))
    assert np.max(np.abs(tx - gy.T)) < 1e-13 * sc
    assert np.max(np.abs(ty - gx.T)) < 1e-13 * sc


def test_newton_third_law_without_slopes():
    n = 20
    s, _, _ = diskgen.random_fields(n, 3, slopes=False)
    fx, fy = oracle.uniform(s, None, None, -1.0, -1.0, 2.0 / n)
    assert abs(np.sum(s * fx)) < 1e-13 * np.sum(np.abs(s * fx))
    assert abs(np.sum(s * fy)) < 1e-13 * np.sum(np.abs(s * fy))


def test_linearity():
    n = 16
    a = diskgen.random_fields(n, 1)
    b = diskgen.random_fields(n, 2)
    fa = oracle.uniform(*a, -1.0, -1.0, 2.0 / n)
    fb = oracle.uniform(*b, -1.0, -1.0, 2.0 / n)
    c = [2.0 * p - 3.0 * q for p, q in zip(a, b)]
    fc = oracle.uniform(*c, -1.0, -1.0, 2.0 / n)
    for k in range(2):
        ref = 2.0 * fa[k] - 3.0 * fb[k]
        assert np.max(np.abs(fc[k] - ref)) < 1e-13 * np.max(np.abs(ref))


def test_uniform_table_equals_pairwise_sum():
    # the per-offset evaluation of the uniform form gives the pairwise sum bit
    # for bit on dyadic grids (same kernel arguments, same source order)
    n = 16
    s, dx, dy = diskgen.random_fields(n, 4)
    fx, fy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    lay = diskgen.Layout(n, 1, [])
    rect, cent, idx = oracle.leaves_of_composite(lay)
    gx, gy = oracle.direct(rect, s.ravel()[idx], dx.ravel()[idx], dy.ravel()[idx], cent)
    assert np.array_equal(fx.ravel()[idx], gx)
    assert np.array_equal(fy.ravel()[idx], gy)


def test_amr_layout_invariance_table10():
    """Refining a zone whose children inherit the parent's linear density
    leaves every other leaf's force unchanged (integral additivity across
    levels).  The paper's Appendix A layout puts base-cell centres on level-2
    edge lines, so the modified kernel for x-bar = x is exercised."""
    lay = diskgen.table10_layout()
    assert lay.validate()
    assert lay.nleaves() == 28
    assert [int(b.leaf_mask.sum()) for b in lay.blocks()] == [14, 2, 4, 4, 4]
    rng = np.random.default_rng(11)
    n0 = lay.n0
    sb = rng.random((n0, n0)) + 0.5
    gx = rng.standard_normal((n0, n0))
    gy = rng.standard_normal((n0, n0))
    # composite values: each cell takes its base ancestor's linear function
    X, Y = lay.centres()
    bi = np.floor((X - lay.x0) / lay.h0).astype(int)
    bj = np.floor((Y - lay.y0) / lay.h0).astype(int)
    bx = lay.x0 + (bi + 0.5) * lay.h0
    by = lay.y0 + (bj + 0.5) * lay.h0
    s = sb[bj, bi] + gx[bj, bi] * (X - bx) + gy[bj, bi] * (Y - by)
    dxs = gx[bj, bi]
    dys = gy[bj, bi]
    rect, cent, idx = oracle.leaves_of_composite(lay)
    fx, fy = oracle.direct(rect, s[idx], dxs[idx], dys[idx], cent)
    base = diskgen.Layout(n0, 1, [], lay.x0, lay.y0, lay.h0)
    rb, cb, ib = oracle.leaves_of_composite(base)
    ux, uy = oracle.direct(rb, sb.ravel(), gx.ravel(), gy.ravel(), cb)
    # the 14 unrefined base leaves are the first 14 composite leaves
    keep = idx < n0 * n0
    assert keep.sum() == 14
    sc = np.max(np.abs(ux))
    np.testing.assert_allclose(fx[keep], ux[idx[keep]], rtol=0, atol=1e-13 * sc)
    np.testing.assert_allclose(fy[keep], uy[idx[keep]], rtol=0, atol=1e-13 * sc)


# ---------------------------------------------------------------------------
# off-plane targets (Section 2 at z != 0)
# ---------------------------------------------------------------------------

def quad_kernels_z(xt, yt, z, xl, xr, yd, yu, npts=24):
    """Composite Gauss-Legendre integration of the nine defining integrands at
    height z over the source rectangle, graded towards the target's foot."""
    g, w = np.polynomial.legendre.leggauss(npts)
    d0 = 0.25 * max(min(abs(xl - xt), abs(xr - xt), abs(yd - yt), abs(yu - yt)), abs(z))

    def nodes(lo, hi, p):
        b = _graded(lo, hi, p, d0)
        a = 0.5 * (b[1:] - b[:-1])
        c = 0.5 * (b[1:] + b[:-1])
        return (c[:, None] + a[:, None] * g).ravel(), (a[:, None] * w).ravel()

    xs, wx = nodes(xl, xr, xt)
    ys, wy = nodes(yd, yu, yt)
    XB, YB = np.meshgrid(xs, ys)
    W = wy[:, None] * wx[None, :]
    u, v = XB - xt, YB - yt
    r3 = (u * u + v * v + z * z) ** 1.5
    ex, ey = XB - 0.5 * (xl + xr), YB - 0.5 * (yd + yu)
    out = []
    for d in (u, v, -z * np.ones_like(u)):  # displacement source - target
        out += [np.sum(W * d / r3), np.sum(W * ex * d / r3), np.sum(W * ey * d / r3)]
    return np.array(out)


@pytest.mark.parametrize("case", [
    # (target, z, source rectangle)
    ((0.0, 0.0), 0.3, (-0.5, 0.5, -0.5, 0.5)),     # above the centre of its own cell
    ((0.2, -0.1), 0.05, (-0.5, 0.5, -0.5, 0.5)),   # low above an off-centre point
    ((0.0, 0.0), -0.2, (0.5, 1.5, -0.5, 0.5)),     # below, right neighbour
    ((0.0, 0.0), 0.7, (0.5, 1.5, 0.5, 1.5)),       # diagonal neighbour
    ((0.0, 0.0), 0.1, (0.0, 1.0, 2.0, 3.0)),       # foot on an edge line
    ((0.3, 0.7), 2.5, (-7.0, -6.0, 11.0, 13.0)),   # far, high
])
def test_offplane_kernels_match_quadrature(case):
    (xt, yt), z, (xl, xr, yd, yu) = case
    k = oracle.cell_kernels_z(xt, yt, z, xl, xr, yd, yu)
    q = quad_kernels_z(xt, yt, z, xl, xr, yd, yu)
    scale = np.max(np.abs(q))
    np.testing.assert_allclose(k, q, rtol=1e-9, atol=1e-11 * scale)


def test_offplane_limits_and_parity_in_z():
    rect = (0.5, 1.5, -0.25, 0.75)
    k0 = oracle.cell_kernels(0.0, 0.0, *rect)
    for z in (1e-6, -1e-6):
        kz = oracle.cell_kernels_z(0.0, 0.0, z, *rect)
        np.testing.assert_allclose(kz[:6], k0, rtol=1e-9, atol=1e-12)   # in-plane limit
        assert np.max(np.abs(kz[6:])) < 1e-5                              # no vertical pull
    # directly above a cell the vertical kernel tends to -2 pi sgn(z) (the
    # field of an infinite sheet)
    for z in (1e-7, -1e-7):
        kz = oracle.cell_kernels_z(0.1, -0.2, z, -0.5, 0.5, -0.5, 0.5)
        assert abs(kz[6] + 2 * math.pi * math.copysign(1.0, z)) < 1e-5
    # x and y families even in z, the z family odd
    a = oracle.cell_kernels_z(0.3, -0.4, 0.6, *rect)
    b = oracle.cell_kernels_z(0.3, -0.4, -0.6, *rect)
    np.testing.assert_allclose(b[:6], a[:6], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(b[6:], -a[6:], rtol=1e-14, atol=1e-16)
    with pytest.raises(ValueError):
        oracle.cell_kernels_z(0.0, 0.0, 0.0, *rect)


def test_offplane_kuzmin_truncated():
    """Kuzmin disk M = 1, a = 0.2 on [-1,1]^2, targets at height z above the
    cell centres: against the analytic off-plane force minus the force of the
    mass outside the square the error is second-order discretisation error;
    against the untruncated force it stalls near 1%."""
    for z in (0.05, 0.3):
        errs = []
        for n in (32, 64):
            rng = np.random.default_rng(n)
            X, Y = diskgen.grid_centres(n)
            s, dx, dy = diskgen.kuzmin(X, Y, 1.0, 0.2)
            h = 2.0 / n
            rect = np.stack([X.ravel() - h / 2, X.ravel() + h / 2, Y.ravel() - h / 2,
                             Y.ravel() + h / 2], 1)
            sel = rng.choice(n * n, 100, replace=False)
            tg = np.stack([X.ravel()[sel], Y.ravel()[sel]], 1)
            f = oracle.direct_z(rect, s.ravel(), dx.ravel(), dy.ravel(), tg, z)
            errs.append(an.rel_l2(f, an.kuzmin_truncated_force_z(tg[:, 0], tg[:, 1], z)))
            assert 0.005 < an.rel_l2(f, an.kuzmin_force_z(tg[:, 0], tg[:, 1], z)) < 0.02
        assert errs[1] < 3e-3
        assert errs[0] / errs[1] > 3.3


def test_offplane_additivity_linear_block():
    """A density linear on a block of cells, with its exact slopes, gives at a
    target above the plane the closed form of the whole block."""
    h = 0.25
    xs = -1.0 + h * np.arange(6)
    ys = 0.5 + h * np.arange(4)
    X, Y = np.meshgrid(xs + h / 2, ys + h / 2)
    a, b, c = 0.7, -1.3, 2.1
    s = a + b * X + c * Y
    rect = np.stack([X.ravel() - h / 2, X.ravel() + h / 2, Y.ravel() - h / 2, Y.ravel() + h / 2], 1)
    tg = np.array([[0.1, -0.3], [-0.6, 0.9], [2.0, 2.0]])
    for z in (0.15, -0.8):
        f = oracle.direct_z(rect, s.ravel(), np.full(s.size, b), np.full(s.size, c), tg, z)
        xl, xr, yd, yu = xs[0], xs[-1] + h, ys[0], ys[-1] + h
        sc = a + b * 0.5 * (xl + xr) + c * 0.5 * (yd + yu)
        for i, (xt, yt) in enumerate(tg):
            k = oracle.cell_kernels_z(xt, yt, z, xl, xr, yd, yu)
            e = [sc * k[3 * m] + b * k[3 * m + 1] + c * k[3 * m + 2] for m in range(3)]
            got = [f[0][i], f[1][i], f[2][i]]
            np.testing.assert_allclose(got, e, rtol=1e-12, atol=1e-13 * max(map(abs, e)))
