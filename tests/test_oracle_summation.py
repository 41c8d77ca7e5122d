"""Pins of the oracle's compensated summation (Neumaier's improvement of
Kahan summation), the step that makes its force sums accurate to a few units
of the last place even where the terms cancel heavily.

Every force sum of the oracle goes through the same two routines that
``oracle.nsum`` exports.  Neumaier's bound for n terms is
|computed - exact| <= 2u|S| + O(n u^2) sum|x_i| (u = 2^-53); on the cases
below the second term is far below the first, so the computed sum must lie
within a few u of the exactly rounded sum (``math.fsum``), while plain
summation misses it by many orders of magnitude (checked too, so that each
case keeps its power to catch a dropped compensation term).
"""
import math

import numpy as np

import oracle

U = 2.0 ** -53


def _naive(x):
    s = 0.0
    for v in x:
        s += v
    return s


def test_cancelling_triples():
    # the compensation recovers what one large term swallowed
    assert oracle.nsum([1e16, 1.0, -1e16]) == 1.0
    assert _naive([1e16, 1.0, -1e16]) == 0.0
    # the branch on |s| >= |x| (Neumaier): plain Kahan summation returns 0 here
    assert oracle.nsum([1.0, 1e100, 1.0, -1e100]) == 2.0
    assert oracle.nsum([]) == 0.0
    assert oracle.nsum([3.5]) == 3.5


def test_million_terms_heavy_cancellation():
    """10^6 terms: 500 000 values of magnitudes 1e-3 .. 1e3, their exact
    negations and 1000 unit-size terms, shuffled.  The large parts cancel
    exactly, so the sum is that of the small terms (condition number ~1e7)."""
    rng = np.random.default_rng(2001)
    a = rng.standard_normal(499_500) * 10.0 ** rng.uniform(-3, 3, 499_500)
    small = rng.standard_normal(1000)
    x = np.concatenate([a, -a, small])
    rng.shuffle(x)
    exact = math.fsum(x)
    cond = np.sum(np.abs(x)) / abs(exact)
    assert cond > 1e5
    got = oracle.nsum(x)
    assert abs(got - exact) <= 4 * U * abs(exact)
    naive = float(np.cumsum(x)[-1])
    assert abs(naive - exact) > 1e3 * U * abs(exact)


def test_direct_sum_is_compensated():
    """The force sum of oracle.direct against the exactly rounded sum of its
    per-source terms, on sources chosen so that those terms cancel in pairs
    to a residual ~1e-9 of their magnitude: each term is s_i K^{x,0}_i (zero
    slopes) with K from oracle.cell_kernels, formed exactly as the oracle
    forms it, so the two sums add the same numbers."""
    n = 40
    h = 2.0 / n
    e = -1.0 + h * np.arange(n)
    X, Y = np.meshgrid(e, e)
    rect = np.stack([X.ravel(), X.ravel() + h, Y.ravel(), Y.ravel() + h], 1)
    xt, yt = 0.013, 0.027
    k = np.array([oracle.cell_kernels(xt, yt, *r) for r in rect])
    keep = np.abs(k[:, 0]) > 1e-9
    rect, k = rect[keep], k[keep]
    m = len(rect) // 2 * 2
    rect, k = rect[:m], k[:m]
    rng = np.random.default_rng(77)
    perm = rng.permutation(m)
    sig = np.zeros(m)
    amp = 10.0 ** rng.uniform(6, 8, m // 2)
    eps = rng.standard_normal(m // 2)
    sig[perm[0::2]] = amp / k[perm[0::2], 0]
    sig[perm[1::2]] = -(amp + eps) / k[perm[1::2], 0]
    zero = np.zeros(m)
    fx, fy = oracle.direct(rect, sig, zero, zero, np.array([[xt, yt]]))
    # the oracle's term: s K0 + dsx Kxx + dsy Kxy, each product rounded, added left to right
    tx = sig * k[:, 0] + zero * k[:, 1] + zero * k[:, 2]
    ty = sig * k[:, 3] + zero * k[:, 4] + zero * k[:, 5]
    ex, ey = math.fsum(tx), math.fsum(ty)
    assert np.sum(np.abs(tx)) / abs(ex) > 1e8     # heavy cancellation
    assert abs(fx[0] - ex) <= 3 * U * abs(ex)
    assert abs(fy[0] - ey) <= 3 * U * abs(ey)
    assert abs(_naive(tx) - ex) > 1e4 * U * abs(ex)
