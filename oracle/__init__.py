"""CPU oracle for the thin-disk midplane force (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package never
imports the product library: the two share no code.

``oracle.c`` holds the arithmetic (exact cell-integrated kernels of Section 2
and the direct double sum); this module only marshals numpy arrays into it.
``analytic`` holds the closed-form disk forces used to pin the oracle.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_cell_kernels.argtypes = [ctypes.c_double] * 6 + [dp]
        lib.oracle_cell_kernels.restype = ctypes.c_int
        lib.oracle_direct.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, dp,
                                      ctypes.c_double, dp, dp, ctypes.c_int]
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_uniform.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, dp, dp, dp, ctypes.c_double,
                                       ctypes.c_int64, i64p, dp, dp, ctypes.c_int]
        lib.oracle_uniform.restype = ctypes.c_int
        lib.oracle_cell_kernels_z.argtypes = [ctypes.c_double] * 7 + [dp]
        lib.oracle_cell_kernels_z.restype = ctypes.c_int
        lib.oracle_direct_z.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, dp,
                                        ctypes.c_double, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        lib.oracle_direct_z.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_nsum.argtypes = [ctypes.c_int64, dp]
        lib.oracle_nsum.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def max_threads():
    return _load().oracle_max_threads()


def nsum(x):
    """Neumaier-compensated sum of a 1-D array in its order: the summation
    every force sum of the oracle uses."""
    x = _f64(x).ravel()
    return float(_load().oracle_nsum(x.size, _dp(x)))


def cell_kernels(xt, yt, xl, xr, yd, yu):
    """Six exact kernels of one source rectangle at one target (Section 2).

    Returns (Kx0, Kxx, Kxy, Ky0, Kyx, Kyy); raises ValueError when the target
    lies on the rectangle's boundary, where the kernels diverge.
    """
    out = np.zeros(6)
    rc = _load().oracle_cell_kernels(float(xt), float(yt), float(xl), float(xr),
                                     float(yd), float(yu), _dp(out))
    if rc != 0:
        raise ValueError("target on source boundary")
    return out


def direct(rect, sigma, dsx, dsy, targets, G=1.0, threads=0):
    """Leaf-by-leaf direct sum (Section 2): F at each target from all sources.

    rect: (n, 4) array of {xl, xr, yd, yu}; sigma, dsx, dsy: (n,) (slopes may be
    None); targets: (m, 2).  Returns (fx, fy) of shape (m,).
    """
    rect = _f64(rect).reshape(-1, 4)
    n = rect.shape[0]
    sigma = _f64(sigma).reshape(n)
    dsx = None if dsx is None else _f64(dsx).reshape(n)
    dsy = None if dsy is None else _f64(dsy).reshape(n)
    targets = _f64(targets).reshape(-1, 2)
    m = targets.shape[0]
    fx = np.zeros(m)
    fy = np.zeros(m)
    rc = _load().oracle_direct(n, _dp(rect), _dp(sigma), _dp(dsx), _dp(dsy), m,
                               _dp(targets), float(G), _dp(fx), _dp(fy), int(threads))
    if rc != 0:
        raise ValueError("a target lies on a source boundary")
    return fx, fy


def cell_kernels_z(xt, yt, z, xl, xr, yd, yu):
    """Nine exact kernels of one source rectangle at a target at height z != 0
    above the disk plane (Section 2 at general z).

    Returns (Kx0, Kxx, Kxy, Ky0, Kyx, Kyy, Kz0, Kzx, Kzy).
    """
    out = np.zeros(9)
    rc = _load().oracle_cell_kernels_z(float(xt), float(yt), float(z), float(xl), float(xr),
                                       float(yd), float(yu), _dp(out))
    if rc != 0:
        raise ValueError("z must be finite and non-zero")
    return out


def direct_z(rect, sigma, dsx, dsy, targets, z, G=1.0, threads=0):
    """Direct sum at targets at height z != 0 above the disk: (fx, fy, fz)."""
    rect = _f64(rect).reshape(-1, 4)
    n = rect.shape[0]
    sigma = _f64(sigma).reshape(n)
    dsx = None if dsx is None else _f64(dsx).reshape(n)
    dsy = None if dsy is None else _f64(dsy).reshape(n)
    targets = _f64(targets).reshape(-1, 2)
    m = targets.shape[0]
    fx, fy, fz = np.zeros(m), np.zeros(m), np.zeros(m)
    rc = _load().oracle_direct_z(n, _dp(rect), _dp(sigma), _dp(dsx), _dp(dsy), m,
                                 _dp(targets), float(z), float(G), _dp(fx), _dp(fy), _dp(fz),
                                 int(threads))
    if rc != 0:
        raise ValueError("z must be finite and non-zero")
    return fx, fy, fz


def uniform(sigma, dsx, dsy, x0, y0, h, G=1.0, targets=None, threads=0):
    """Direct O(N^4) sum on a uniform n x n grid (arrays row-major, [y, x]).

    targets: optional flat cell indices; returns (fx, fy) at those cells
    (shape (m,)), else full (n, n) arrays.
    """
    sigma = _f64(sigma)
    n = sigma.shape[0]
    assert sigma.shape == (n, n)
    dsx = None if dsx is None else _f64(dsx)
    dsy = None if dsy is None else _f64(dsy)
    if targets is None:
        m, tp, tarr = n * n, None, None
    else:
        tarr = np.ascontiguousarray(targets, dtype=np.int64).ravel()
        m = tarr.size
        tp = tarr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    fx = np.zeros(m)
    fy = np.zeros(m)
    rc = _load().oracle_uniform(n, float(x0), float(y0), float(h), _dp(sigma), _dp(dsx),
                                _dp(dsy), float(G), 0 if tarr is None else m, tp,
                                _dp(fx), _dp(fy), int(threads))
    if rc != 0:
        raise RuntimeError("oracle_uniform failed (%d)" % rc)
    if targets is None:
        return fx.reshape(n, n), fy.reshape(n, n)
    return fx, fy


def leaves_of_composite(layout):
    """Source rectangles and centres of every leaf of a composite layout.

    ``layout`` is a diskgen AMR layout; returns (rect (n,4), centres (n,2),
    packed indices (n,)) in composite-packed order, leaves only.
    """
    rects, cents, idx = [], [], []
    for blk in layout.blocks():
        xs = blk.x0 + blk.h * np.arange(blk.nx)
        ys = blk.y0 + blk.h * np.arange(blk.ny)
        X, Y = np.meshgrid(xs, ys)
        leaf = blk.leaf_mask.ravel()
        r = np.stack([X.ravel(), X.ravel() + blk.h, Y.ravel(), Y.ravel() + blk.h], 1)
        c = np.stack([X.ravel() + 0.5 * blk.h, Y.ravel() + 0.5 * blk.h], 1)
        rects.append(r[leaf])
        cents.append(c[leaf])
        idx.append(blk.offset + np.nonzero(leaf)[0])
    return np.concatenate(rects), np.concatenate(cents), np.concatenate(idx)
