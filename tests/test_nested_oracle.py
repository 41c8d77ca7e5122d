"""Pins of the nested-correction oracle (oracle/nested.py), on the CPU.

The scheme approximates the leaf-by-leaf direct sum of Section 2 on a
Section 3 composite grid.  Its oracle is pinned by what fixes it exactly:
the restriction conserves the children's mass and first moments and keeps
linear densities (checked against moment integrals written out here), the
interpolation stencils reproduce linear fields (and bilinear or biquadratic
ones where they use 4 or 9 cells) under every availability pattern, a
single level is the uniform direct sum, mass inside one box gives the exact
leaf sum at that box's leaves, the whole map is linear in the density, and
its deviation from the exact leaf sum (``oracle.direct``) is bounded and
falls as the grid is refined.  A planted wrong restriction coefficient or a
mirrored interpolation offset each break a bound here.
"""
import itertools

import numpy as np
import pytest

import diskgen
import oracle
from oracle import analytic as an
from oracle import nested


def _central_layout(n0):
    """Level 1 over [-1/4, 1/4]^2 and level 2 over [-1/8, 1/8]^2 on [-1, 1]^2."""
    n1, n2 = 2 * n0, 4 * n0
    a1 = int(0.375 * n1)
    a2 = int(0.4375 * n2)
    return diskgen.Layout(n0, 3, [diskgen.Patch(1, a1, a1, n1 - 2 * a1, n1 - 2 * a1),
                                  diskgen.Patch(2, a2, a2, n2 - 2 * a2, n2 - 2 * a2)])


def _kuzmin(X, Y):
    return diskgen.kuzmin(X, Y, 1.0, 0.2)


def _deviation(lay, s, dx, dy):
    fx, fy = nested.nested(lay, s, dx, dy)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent)
    area = (rect[:, 1] - rect[:, 0]) ** 2
    d = np.hypot(fx[idx] - ox, fy[idx] - oy)
    return an.rel_l2((fx[idx], fy[idx]), (ox, oy), area), float(d.max() / np.hypot(ox, oy).max())


def test_restriction_conserves_mass_and_first_moments():
    lay = diskgen.Layout(8, 3, [diskgen.Patch(1, 4, 2, 6, 8), diskgen.Patch(2, 10, 6, 4, 4)])
    assert lay.validate()
    rng = np.random.default_rng(3)
    n = lay.total()
    s, dx, dy = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    rs, rdx, rdy = nested.restrict(lay, s, dx, dy)
    maps = nested.cell_maps(lay)
    checked = 0
    for l in range(lay.nlevels - 1, 0, -1):
        h = lay.h0 / 2 ** (l - 1)
        hc = h / 2
        par, fine = maps[l - 1], maps[l]
        for J, I in zip(*np.nonzero(par >= 0)):
            if fine[2 * J, 2 * I] < 0:
                continue
            xp, yp = (I + 0.5) * h, (J + 0.5) * h
            m0 = mx = my = 0.0
            for b, a in itertools.product(range(2), range(2)):
                c = fine[2 * J + b, 2 * I + a]
                xc, yc = (2 * I + a + 0.5) * hc, (2 * J + b + 0.5) * hc
                area = hc * hc
                # integrals over the child of rho = s + dx (x - xc) + dy (y - yc)
                m0 += rs[c] * area
                mx += rs[c] * (xc - xp) * area + rdx[c] * hc ** 4 / 12.0
                my += rs[c] * (yc - yp) * area + rdy[c] * hc ** 4 / 12.0
            p = par[J, I]
            assert abs(rs[p] * h * h - m0) <= 1e-14 * (abs(m0) + h * h)
            assert abs(rdx[p] * h ** 4 / 12.0 - mx) <= 1e-14 * h ** 3
            assert abs(rdy[p] * h ** 4 / 12.0 - my) <= 1e-14 * h ** 3
            checked += 1
    assert checked == 6 * 8 // 4 + 4 * 4 // 4
    # leaves are untouched
    m = lay.leaf_mask()
    assert np.array_equal(rs[m], s[m]) and np.array_equal(rdx[m], dx[m])


def test_restriction_keeps_a_linear_density():
    lay = _central_layout(16)
    X, Y = lay.centres()
    s, dx, dy = 2.0 + 0.3 * X - 1.7 * Y, np.full_like(X, 0.3), np.full_like(X, -1.7)
    m = lay.leaf_mask()
    rs, rdx, rdy = nested.restrict(lay, np.where(m, s, 0), np.where(m, dx, 0), np.where(m, dy, 0))
    assert np.allclose(rs, s, rtol=0, atol=1e-14)
    assert np.allclose(rdx, 0.3, rtol=0, atol=1e-13) and np.allclose(rdy, -1.7, rtol=0, atol=1e-13)


@pytest.mark.parametrize("sx,sy", [(1, 1), (-1, 1), (1, -1), (-1, -1)])
def test_stencils_reproduce_polynomials_for_every_availability(sx, sy):
    I, J = 5, 7
    ring = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
    tx, ty = I + sx / 4.0, J + sy / 4.0
    for bits in range(1 << 8):
        have = {(I + a, J + b) for k, (a, b) in enumerate(ring) if bits >> k & 1} | {(I, J)}
        st = nested.stencil(lambda i, j: (i, j) in have, I, J, sx, sy)
        assert all((i, j) in have for i, j, _ in st)
        w = np.array([x[2] for x in st])
        pi = np.array([x[0] for x in st], float)
        pj = np.array([x[1] for x in st], float)
        assert abs(w.sum() - 1) < 1e-15
        # linear in each direction the available cells allow
        span_x = any(i != I for i, _, _ in st)
        span_y = any(j != J for _, j, _ in st)
        assert span_x == ((I - 1, J) in have or (I + 1, J) in have)
        assert span_y == ((I, J - 1) in have or (I, J + 1) in have)
        assert abs(w @ pi - (tx if span_x else I)) < 1e-14
        assert abs(w @ pj - (ty if span_y else J)) < 1e-14
        if len(st) >= 4:          # bilinear or biquadratic: the xy term too
            assert abs(w @ (pi * pj) - tx * ty) < 1e-13
        if len(st) == 9:          # biquadratic: x^2 y^2 too
            assert abs(w @ (pi ** 2 * pj ** 2) - tx ** 2 * ty ** 2) < 1e-11
        if len(have) == 9:
            assert len(st) == 9
        near = {(I + sx, J), (I, J + sy), (I + sx, J + sy)}
        if len(st) != 9 and near <= have:   # interpolation, not extrapolation
            assert {(i, j) for i, j, _ in st} == near | {(I, J)}


def test_single_level_is_the_uniform_sum():
    n = 32
    s, dx, dy = diskgen.random_fields(n, 4)
    lay = diskgen.Layout(n, 1, [])
    fx, fy = nested.nested(lay, s.ravel(), dx.ravel(), dy.ravel())
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    assert np.array_equal(fx, ox.ravel()) and np.array_equal(fy, oy.ravel())


def test_mass_inside_one_box_gives_the_exact_leaf_sum():
    """All mass on a level-1 patch well inside one box: the far field is
    zero, so every level-1 leaf gets the exact leaf sum."""
    lay = diskgen.Layout(64, 2, [diskgen.Patch(1, 16, 20, 24, 16)])
    rng = np.random.default_rng(8)
    n = lay.total()
    s, dx, dy = rng.random(n) + 0.1, rng.standard_normal(n), rng.standard_normal(n)
    fine = np.zeros(n, bool)
    fine[64 * 64:] = True
    s, dx, dy = (np.where(fine, a, 0.0) for a in (s, dx, dy))
    fx, fy = nested.nested(lay, s, dx, dy)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent)
    k = fine[idx]
    assert an.rel_l2((fx[idx][k], fy[idx][k]), (ox[k], oy[k])) < 1e-13


def test_linear_in_the_density():
    lay = _central_layout(16)
    rng = np.random.default_rng(2)
    n = lay.total()
    a = [rng.standard_normal(n) for _ in range(3)]
    b = [rng.standard_normal(n) for _ in range(3)]
    fa = nested.nested(lay, *a)
    fb = nested.nested(lay, *b)
    fc = nested.nested(lay, *[2 * x - 3 * y for x, y in zip(a, b)])
    for c in range(2):
        ref = 2 * fa[c] - 3 * fb[c]
        assert np.max(np.abs(fc[c] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_deviation_from_leaf_sum_is_bounded_and_falls():
    """Kuzmin disk (a = 0.2) with two nested central patches: the deviation
    from the exact leaf sum (relative L2, area weighted; max |dF| / max |F|)
    at base 32^2 and 64^2 stays below the bounds measured for this scheme
    (1.0e-4 and 1.5e-5 relative L2) and falls by more than 4x."""
    dev = []
    for n0 in (32, 64):
        lay = _central_layout(n0)
        s, dx, dy = lay.sample(_kuzmin)
        dev.append(_deviation(lay, s, dx, dy))
    assert dev[0][0] < 1.3e-4 and dev[0][1] < 2.5e-4
    assert dev[1][0] < 2.0e-5 and dev[1][1] < 5.0e-5
    assert dev[1][0] < dev[0][0] / 4


def test_deviation_on_a_flagged_clump_layout():
    """A flagged 3-level layout of the Kuzmin-plus-clumps profile (32x32
    child patches): deviation from the exact leaf sum below 1e-4."""
    lay, s, dx, dy = diskgen.amr_config(5, n0=32, nlevels=3, thresh=0.15, a=0.05)
    rl, mx = _deviation(lay, s, dx, dy)
    assert rl < 1e-4 and mx < 1e-4, (rl, mx)


def test_planted_mistakes_break_the_bounds(monkeypatch):
    lay = _central_layout(64)
    s, dx, dy = lay.sample(_kuzmin)
    orig = nested.stencil
    # mirrored child offset in the interpolation
    monkeypatch.setattr(nested, "stencil", lambda av, I, J, sx, sy: orig(av, I, J, -sx, -sy))
    assert _deviation(lay, s, dx, dy)[0] > 2.0e-5
    monkeypatch.setattr(nested, "stencil", orig)
    # restriction slope coefficient 3/(8h) in place of 3/(4h)
    orig_r = nested.restrict

    def bad_restrict(lay_, s_, dx_, dy_):
        rs, rdx, rdy = orig_r(lay_, s_, dx_, dy_)
        m = lay_.leaf_mask()
        sx = np.zeros_like(rs)
        maps = nested.cell_maps(lay_)
        for l in range(lay_.nlevels - 1, 0, -1):
            h = lay_.h0 / 2 ** (l - 1)
            par, fine = maps[l - 1], maps[l]
            for J, I in zip(*np.nonzero(par >= 0)):
                if fine[2 * J, 2 * I] >= 0:
                    p = par[J, I]
                    ch = [fine[2 * J + b, 2 * I + a] for b in range(2) for a in range(2)]
                    diff = (rs[ch[1]] + rs[ch[3]]) - (rs[ch[0]] + rs[ch[2]])
                    rdx[p] -= 3.0 / (8.0 * h) * diff
        del m, sx
        return rs, rdx, rdy
    monkeypatch.setattr(nested, "restrict", bad_restrict)
    assert _deviation(lay, s, dx, dy)[0] > 2.0e-5
