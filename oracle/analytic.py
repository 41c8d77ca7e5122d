"""Closed-form disk forces used to pin the oracle (test infrastructure only).

* D2 disk (Schulz 2009, n = 2): surface density s0 (1 - R^2/a^2)^{3/2} and its
  midplane radial force, as printed in Section 3 of the paper.
* D2,2: two D2 disks centred at (0, +0.5) and (0, -0.5) (Section 3), force by
  superposition.
* Kuzmin disk: s = M a / (2 pi (r^2 + a^2)^{3/2}), radial force
  -G M r / (r^2 + a^2)^{3/2}; on a finite square the force of the mass outside
  the square is removed by quadrature (``kuzmin_exterior_force``).  Above the
  plane the disk's potential is that of a point mass at depth a below the
  target's side, -G M / sqrt(r^2 + (a + |z|)^2) (``kuzmin_force_z``).
* Area-weighted error norms of Section 3.
"""
import numpy as np


def d2_radial_force(R, alpha=0.25, sigma0=1.0, G=1.0):
    """Midplane radial force of the D2 disk (Section 3, after Schulz 2009)."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty_like(R)
    inside = R <= alpha
    Ri = R[inside]
    out[inside] = -(3 * np.pi ** 2 * sigma0 * G * Ri / (16 * alpha ** 3)) * (4 * alpha ** 2 - 3 * Ri ** 2)
    Ro = R[~inside]
    out[~inside] = -(3 * np.pi * sigma0 * G / (8 * alpha ** 3)) * (
        Ro * (4 * alpha ** 2 - 3 * Ro ** 2) * np.arcsin(alpha / Ro)
        - alpha * (2 * alpha ** 2 - 3 * Ro ** 2) * np.sqrt(1 - alpha ** 2 / Ro ** 2))
    return out


def d2_force(X, Y, alpha=0.25, sigma0=1.0, G=1.0, centre=(0.0, 0.0)):
    """(Fx, Fy) of a D2 disk centred at ``centre``; zero at the centre itself."""
    dx = np.asarray(X, dtype=np.float64) - centre[0]
    dy = np.asarray(Y, dtype=np.float64) - centre[1]
    R = np.hypot(dx, dy)
    FR = d2_radial_force(R, alpha, sigma0, G)
    with np.errstate(invalid="ignore", divide="ignore"):
        fx = np.where(R > 0, FR * dx / np.where(R > 0, R, 1), 0.0)
        fy = np.where(R > 0, FR * dy / np.where(R > 0, R, 1), 0.0)
    return fx, fy


def d22_force(X, Y, alpha=0.25, sigma0=1.0, G=1.0):
    """(Fx, Fy) of the D2,2 pair of disks at (0, +-0.5) (Section 3)."""
    ax, ay = d2_force(X, Y, alpha, sigma0, G, (0.0, 0.5))
    bx, by = d2_force(X, Y, alpha, sigma0, G, (0.0, -0.5))
    return ax + bx, ay + by


def kuzmin_sigma(x, y, M=1.0, a=0.2):
    return M * a / (2 * np.pi * (x * x + y * y + a * a) ** 1.5)


def kuzmin_force(X, Y, M=1.0, a=0.2, G=1.0):
    """Midplane force of the untruncated Kuzmin disk: -G M r / (r^2+a^2)^{3/2}."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    q = (X * X + Y * Y + a * a) ** 1.5
    return -G * M * X / q, -G * M * Y / q


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _graded_breaks(lo, hi, p, d0):
    """Panel breakpoints on [lo, hi], geometrically graded (ratio 2) away from p.

    p is the target's projection (clipped into [lo, hi]); d0 the smallest panel.
    """
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


def _rect_force(xt, yt, xa, xb, ya, yb, sig, G, npts=12):
    """Force at (xt, yt) of density sig over [xa,xb]x[ya,yb] (target outside),
    by tensor Gauss-Legendre on panels graded towards the target."""
    dist = max(xa - xt, xt - xb, ya - yt, yt - yb, 0.0)
    d0 = max(dist, 1e-6) * 0.5
    bx = _graded_breaks(xa, xb, xt, d0)
    by = _graded_breaks(ya, yb, yt, d0)
    g, w = _gl(npts)
    # nodes and weights of the composite rule in each direction
    ax = 0.5 * (bx[1:] - bx[:-1])
    cx = 0.5 * (bx[1:] + bx[:-1])
    xs = (cx[:, None] + ax[:, None] * g[None, :]).ravel()
    wx = (ax[:, None] * w[None, :]).ravel()
    ay = 0.5 * (by[1:] - by[:-1])
    cy = 0.5 * (by[1:] + by[:-1])
    ys = (cy[:, None] + ay[:, None] * g[None, :]).ravel()
    wy = (ay[:, None] * w[None, :]).ravel()
    U = xs[None, :] - xt
    V = ys[:, None] - yt
    r3 = (U * U + V * V) ** 1.5
    S = sig(xs[None, :], ys[:, None]) * wy[:, None] * wx[None, :]
    return G * np.sum(S * U / r3), G * np.sum(S * V / r3)


def kuzmin_exterior_force(X, Y, M=1.0, a=0.2, G=1.0, half=1.0, far=60.0):
    """Force at each (X, Y) inside [-half, half]^2 of the Kuzmin mass outside
    that square, out to |x|, |y| <= far (the rest is below 1e-6 of F)."""
    sig = lambda x, y: kuzmin_sigma(x, y, M, a)
    strips = [(-far, far, half, far), (-far, far, -far, -half),
              (-far, -half, -half, half), (half, far, -half, half)]
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    fx = np.zeros(X.shape)
    fy = np.zeros(X.shape)
    for idx in np.ndindex(X.shape):
        sx = sy = 0.0
        for (xa, xb, ya, yb) in strips:
            gx, gy = _rect_force(X[idx], Y[idx], xa, xb, ya, yb, sig, G)
            sx += gx
            sy += gy
        fx[idx] = sx
        fy[idx] = sy
    return fx, fy


def kuzmin_truncated_force(X, Y, M=1.0, a=0.2, G=1.0, half=1.0):
    """Force of the Kuzmin density restricted to [-half, half]^2.

    Uses the eight-fold symmetry of a centred disk on a centred square: only
    targets with 0 <= y <= x are integrated, the rest are mirrored."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    ax_, ay_ = np.abs(X), np.abs(Y)
    lo = np.minimum(ax_, ay_)
    hi = np.maximum(ax_, ay_)
    key = np.round(np.stack([hi, lo], -1) * 2 ** 30).astype(np.int64).reshape(-1, 2)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.ravel()
    px = uniq[:, 0] / 2.0 ** 30
    py = uniq[:, 1] / 2.0 ** 30
    ex, ey = kuzmin_exterior_force(px, py, M, a, G, half)
    kx, ky = kuzmin_force(px, py, M, a, G)
    tx, ty = kx - ex, ky - ey  # force at (hi, lo) with hi >= lo >= 0
    tx = tx[inv].reshape(X.shape)
    ty = ty[inv].reshape(X.shape)
    swap = ay_ > ax_
    fx = np.where(swap, ty, tx) * np.sign(X)
    fy = np.where(swap, tx, ty) * np.sign(Y)
    return fx, fy


def kuzmin_force_z(X, Y, z, M=1.0, a=0.2, G=1.0):
    """Force at height z of the untruncated Kuzmin disk, whose potential above
    the plane is -G M / sqrt(r^2 + (a + |z|)^2): returns (Fx, Fy, Fz)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    b = a + abs(z)
    q = (X * X + Y * Y + b * b) ** 1.5
    return -G * M * X / q, -G * M * Y / q, -G * M * np.sign(z) * b / q


def _rect_force_z(xt, yt, z, xa, xb, ya, yb, sig, G, npts=12):
    """(Fx, Fy, Fz) at (xt, yt, z) of density sig over [xa,xb]x[ya,yb] in the
    plane, by tensor Gauss-Legendre on panels graded towards the target's foot."""
    dist = max(xa - xt, xt - xb, ya - yt, yt - yb, 0.0)
    d0 = max(dist, abs(z), 1e-6) * 0.5
    bx = _graded_breaks(xa, xb, xt, d0)
    by = _graded_breaks(ya, yb, yt, d0)
    g, w = _gl(npts)
    ax = 0.5 * (bx[1:] - bx[:-1])
    cx = 0.5 * (bx[1:] + bx[:-1])
    xs = (cx[:, None] + ax[:, None] * g[None, :]).ravel()
    wx = (ax[:, None] * w[None, :]).ravel()
    ay = 0.5 * (by[1:] - by[:-1])
    cy = 0.5 * (by[1:] + by[:-1])
    ys = (cy[:, None] + ay[:, None] * g[None, :]).ravel()
    wy = (ay[:, None] * w[None, :]).ravel()
    U = xs[None, :] - xt
    V = ys[:, None] - yt
    r3 = (U * U + V * V + z * z) ** 1.5
    S = sig(xs[None, :], ys[:, None]) * wy[:, None] * wx[None, :]
    return G * np.sum(S * U / r3), G * np.sum(S * V / r3), G * np.sum(S * (-z) / r3)


def kuzmin_truncated_force_z(X, Y, z, M=1.0, a=0.2, G=1.0, half=1.0, far=60.0):
    """Force at height z of the Kuzmin density restricted to [-half, half]^2:
    the analytic force minus that of the mass outside the square (out to
    |x|, |y| <= far), at each target (X, Y) in the square."""
    sig = lambda x, y: kuzmin_sigma(x, y, M, a)
    strips = [(-far, far, half, far), (-far, far, -far, -half),
              (-far, -half, -half, half), (half, far, -half, half)]
    X = np.asarray(X, dtype=np.float64).ravel()
    Y = np.asarray(Y, dtype=np.float64).ravel()
    kx, ky, kz = kuzmin_force_z(X, Y, z, M, a, G)
    out = [kx.copy(), ky.copy(), kz.copy()]
    for i in range(X.size):
        for (xa, xb, ya, yb) in strips:
            g = _rect_force_z(X[i], Y[i], z, xa, xb, ya, yb, sig, G)
            for c in range(3):
                out[c][i] -= g[c]
    return tuple(out)


def norms(err, area):
    """Area-weighted L1, L2 and max norms of Section 3."""
    err = np.abs(np.asarray(err, dtype=np.float64))
    area = np.broadcast_to(np.asarray(area, dtype=np.float64), err.shape)
    return (float(np.sum(err * area)), float(np.sqrt(np.sum(err * err * area))),
            float(np.max(err)))


def rel_l2(a, b, area=1.0):
    """Area-weighted relative L2 of a against b, over all components given.

    a, b: sequences of arrays (e.g. (fx, fy)); the norm runs over all of them."""
    num = 0.0
    den = 0.0
    for x, y in zip(a, b):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        ar = np.broadcast_to(np.asarray(area, dtype=np.float64), x.shape)
        num += float(np.sum((x - y) ** 2 * ar))
        den += float(np.sum(y * y * ar))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))
