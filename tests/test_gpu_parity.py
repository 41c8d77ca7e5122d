"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: relative L2 over both force components (area weighted on AMR
layouts) <= 1e-12 for FP64 plans and <= 1e-5 for FP32 plans.
"""
import numpy as np
import pytest

import diskgen
import oracle
from oracle import analytic as an

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def gl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_02765_amd as m
    return m


def _prec(gl, name):
    return gl.F64 if name == "f64" else gl.F32


def _dt(name):
    return torch.float64 if name == "f64" else torch.float32


def _dev(a, name):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda", _dt(name))


def _host(t):
    return t.double().cpu().numpy()


def _err(got, ref, area=None):
    """The larger of the (area-weighted) relative L2 error and
    max_i |got_i - ref_i| / max_i |ref_i| over all components: a parity
    bound on both the aggregate and every element."""
    num = max(float(np.max(np.abs(np.asarray(g) - np.asarray(r)))) for g, r in zip(got, ref))
    den = max(float(np.max(np.abs(np.asarray(r)))) for r in ref)
    return max(an.rel_l2(got, ref, area) if area is not None else an.rel_l2(got, ref), num / den)


def gpu_uniform(gl, prec, s, dx, dy, h=None, G=1.0, slopes=True):
    n = s.shape[0]
    p = gl.Plan(n, _prec(gl, prec), slopes=slopes, G=G, h0=h if h else 2.0 / n)
    fx, fy = p.solve(_dev(s, prec), _dev(dx, prec) if slopes else None,
                     _dev(dy, prec) if slopes else None)
    torch.cuda.synchronize()
    return _host(fx).reshape(n, n), _host(fy).reshape(n, n)


def test_library_loaded(gl):
    import ctypes
    import os
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(gl.LIB_PATH) in maps


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_cell_sources(gl, prec):
    """One unit source cell at several positions, including the far corners
    (largest offsets of the kernel tables): F is the oracle's direct sum."""
    n = 32
    for (i, j) in [(0, 0), (n - 1, n - 1), (5, 17), (n - 1, 0)]:
        s = np.zeros((n, n))
        s[j, i] = 1.0
        dx = np.zeros((n, n))
        dy = np.zeros((n, n))
        dx[j, i] = 0.7
        dy[j, i] = -1.3
        fx, fy = gpu_uniform(gl, prec, s, dx, dy)
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
        assert _err((fx, fy), (ox, oy)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [16, 64, 128])
def test_uniform_random(gl, prec, n):
    s, dx, dy = diskgen.random_fields(n, 100 + n)
    fx, fy = gpu_uniform(gl, prec, s, dx, dy)
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    assert _err((fx, fy), (ox, oy)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_uniform_no_slopes(gl, prec):
    n = 64
    s, _, _ = diskgen.random_fields(n, 7, slopes=False)
    fx, fy = gpu_uniform(gl, prec, s, None, None, slopes=False)
    ox, oy = oracle.uniform(s, None, None, -1.0, -1.0, 2.0 / n)
    assert _err((fx, fy), (ox, oy)) < TOL[prec]


def test_zero_density_gives_zero_force(gl):
    n = 64
    z = np.zeros((n, n))
    fx, fy = gpu_uniform(gl, "f64", z, z, z)
    assert np.all(fx == 0) and np.all(fy == 0)


def test_kuzmin_64_fp64(gl):
    """Bench config 1: 64^2 Kuzmin disk (M = 1, a = 0.2) in FP64, G = 1."""
    n = 64
    X, Y = diskgen.grid_centres(n)
    s, dx, dy = diskgen.kuzmin(X, Y, 1.0, 0.2)
    fx, fy = gpu_uniform(gl, "f64", s, dx, dy)
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n)
    assert _err((fx, fy), (ox, oy)) < 1e-12
    tx, ty = an.kuzmin_truncated_force(X, Y)
    assert an.rel_l2((fx, fy), (tx, ty)) < 4e-3


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noisy_spiral_256_full(gl, prec):
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 3)
    fx, fy = gpu_uniform(gl, prec, s, dx, dy, h=h, G=2.5)
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, G=2.5)
    assert _err((fx, fy), (ox, oy)) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_headline_1024_sampled(gl, prec):
    """The 1024^2 noisy spiral disk (2048^2 zero-padded FFT): sampled targets
    against the oracle's full direct sum at those targets."""
    n = 1024
    s, dx, dy, h = diskgen.noisy_spiral(n, 0)
    fx, fy = gpu_uniform(gl, prec, s, dx, dy, h=h)
    rng = np.random.default_rng(2024)
    tg = np.concatenate([rng.choice(n * n, 40, replace=False),
                         [0, n - 1, n * n - 1, n * (n - 1), n * (n // 2) + n // 2]])
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, targets=tg)
    assert _err((fx.ravel()[tg], fy.ravel()[tg]), (ox, oy)) < TOL[prec]


_LARGE = {}


def _large_case(n):
    """Kuzmin spiral on an n x n grid and the oracle at its targets: at
    2048^2 one full row, one full column, 64 random cells and the corners;
    at 4096^2 a run of 256 cells along a row, 64 random cells and the
    corners (the oracle's per-offset table form, pinned to the pairwise
    sum), shared by both precisions."""
    if n not in _LARGE:
        X, Y = diskgen.grid_centres(n)
        s, dx, dy = diskgen.spiral(X, Y, "kuzmin", 0.3, 0.15, 20.0, 1.0)
        rng = np.random.default_rng(n)
        parts = [rng.choice(n * n, 64, replace=False), [0, n - 1, n * n - 1, n * (n - 1)]]
        if n <= 2048:
            parts += [1000 * n + np.arange(n), np.arange(n) * n + 700]
        else:
            parts += [3000 * n + 1900 + np.arange(256)]
        tg = np.unique(np.concatenate(parts))
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n, targets=tg)
        _LARGE[n] = (s, dx, dy, tg, (ox, oy))
    return _LARGE[n]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [2048, 4096])
def test_largest_sizes_sampled(gl, prec, n):
    """The two largest supported lattices (FFT sizes 4096 and 8192): full
    rows and columns (2048^2) or a run along a row (4096^2), random cells
    and the four corners against the oracle, in relative L2 and element by
    element (|dF_i| <= tol max|F|)."""
    s, dx, dy, tg, ref = _large_case(n)
    fx, fy = gpu_uniform(gl, prec, s, dx, dy)
    got = (fx.ravel()[tg], fy.ravel()[tg])
    e2 = an.rel_l2(got, ref)
    em = max(float(np.max(np.abs(g - r))) for g, r in zip(got, ref)) / max(float(np.max(np.abs(r))) for r in ref)
    print("%d^2 %s: %d targets, rel_l2 %.3e max_rel %.3e" % (n, prec, len(tg), e2, em))
    assert e2 < TOL[prec] and em < TOL[prec]


def test_table1_row_512_on_gpu(gl):
    """Table 1 row N_k = 256 (512^2 grid) from the GPU path: printed max norms
    to three digits (a property of the exact discrete sum at this size)."""
    n = 512
    X, Y = diskgen.grid_centres(n)
    s, dx, dy = diskgen.d2(X, Y)
    fx, fy = gpu_uniform(gl, "f64", s, dx, dy)
    ax, ay = an.d2_force(X, Y)
    R = np.hypot(X, Y)
    _, x2, xi = an.norms(fx - ax, (2.0 / n) ** 2)
    _, _, ri = an.norms((fx * X + fy * Y) / R - (ax * X + ay * Y) / R, (2.0 / n) ** 2)
    assert abs(xi - 1.93e-3) <= 0.006e-3
    assert abs(ri - 1.99e-3) <= 0.006e-3
    assert abs(2 * x2 - 2.44e-4) <= 0.006e-4


def _amr_parity(gl, lay, s, dx, dy, prec, targets=None):
    p = gl.Plan(lay.n0, _prec(gl, prec), slopes=True, x0=lay.x0, y0=lay.y0, h0=lay.h0,
                nlevels=lay.nlevels, patches=lay.patches)
    assert p.n_cells == lay.total()
    assert p.n_leaves == lay.nleaves()
    fx, fy = p.solve(_dev(s, prec), _dev(dx, prec), _dev(dy, prec))
    torch.cuda.synchronize()
    fx, fy = _host(fx), _host(fy)
    mask = lay.leaf_mask()
    assert np.all(fx[~mask] == 0) and np.all(fy[~mask] == 0)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    if targets is not None:
        sel = targets
    else:
        sel = np.arange(len(idx))
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent[sel])
    area = (rect[sel, 1] - rect[sel, 0]) * (rect[sel, 3] - rect[sel, 2])
    return _err((fx[idx[sel]], fy[idx[sel]]), (ox, oy), area)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_amr_table10_layout(gl, prec):
    """The paper's Appendix A layout (28 leaves on 3 levels) against the leaf
    direct sum, with a random linear density per leaf."""
    lay = diskgen.table10_layout()
    rng = np.random.default_rng(1)
    n = lay.total()
    s, dx, dy = rng.random(n) + 0.2, rng.standard_normal(n), rng.standard_normal(n)
    m = lay.leaf_mask()
    s, dx, dy = np.where(m, s, 0), np.where(m, dx, 0), np.where(m, dy, 0)
    assert _amr_parity(gl, lay, s, dx, dy, prec) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_amr_small_flagged(gl, prec):
    """A flagged 3-level layout (base 32^2, 32x32 child patches) of the Kuzmin
    plus clumps profile: every leaf against the leaf direct sum."""
    lay, s, dx, dy = diskgen.amr_config(5, n0=32, nlevels=3, thresh=0.15, a=0.05)
    assert lay.validate() and len(lay.patches) > 0
    assert _amr_parity(gl, lay, s, dx, dy, prec) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_amr_config3_sampled(gl, prec):
    """The 3-level AMR workload (base 256^2, finest lattice 1024^2): leaf
    targets sampled on every level against the leaf direct sum."""
    lay, s, dx, dy = diskgen.amr_config(0)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(9)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(12, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    assert _amr_parity(gl, lay, s, dx, dy, prec, targets=sel) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,disk", [("ilr", "d2"), ("vlr", "d22")])
def test_band_layouts_sampled(gl, prec, kind, disk):
    """The refinement layouts of the Section 3 experiments (3 levels, base
    128^2, hundreds of 2-row patches): leaf targets sampled on every level,
    and in the band about the disk edge, against the leaf direct sum."""
    gen = diskgen.ilr_layout if kind == "ilr" else diskgen.vlr_layout
    lay = gen(128, 3, disk)
    assert len(lay.patches) > 150
    s, dx, dy = lay.sample(diskgen.d2 if disk == "d2" else diskgen.d22)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(13)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(16, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    assert _amr_parity(gl, lay, s, dx, dy, prec, targets=sel) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n0,levels", [(1024, 2), (1024, 3)])
def test_amr_large_lattices_sampled(gl, prec, n0, levels):
    """AMR at the largest transform sizes (finest lattice 2048^2 and 4096^2,
    FFTs of 4096 and 8192 points per side): ILR layouts of the D2 disk, leaf
    targets sampled on every level against the leaf direct sum."""
    lay = diskgen.ilr_layout(n0, levels, "d2")
    s, dx, dy = lay.sample(diskgen.d2)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(17)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(8, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    assert _amr_parity(gl, lay, s, dx, dy, prec, targets=sel) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_amr_six_levels(gl, prec):
    """Deep nesting: a 32^2 base refined five times along a circle (six
    levels, leaves up to 32 finest cells wide, finest lattice 1024^2), with a
    random linear density per leaf: every leaf against the leaf direct sum."""
    lay = diskgen.band_layout(32, 6, [(0.1, 0.05)], 0.3, [0.08 / 2 ** l for l in range(6)])
    assert lay.validate() and max(p.level for p in lay.patches) == 5
    rng = np.random.default_rng(23)
    n = lay.total()
    s, dx, dy = rng.random(n) + 0.2, rng.standard_normal(n), rng.standard_normal(n)
    m = lay.leaf_mask()
    s, dx, dy = np.where(m, s, 0), np.where(m, dx, 0), np.where(m, dy, 0)
    assert _amr_parity(gl, lay, s, dx, dy, prec) < TOL[prec]


def test_ilr_d2_accuracy_and_order(gl):
    """AMR(2, D2) under ILR (Section 3, Table 3): against the analytic force
    the errors fall at second order in L1 and L2 from N_k = 128 to 256, and
    at each size they are below those of the uniform base grid."""
    import amr_study
    rows = [amr_study.run_case(gl, torch, "ilr", "d2", 2, n) for n in (128, 256)]
    uni = [amr_study.run_case(gl, torch, "ilr", "d2", 1, n) for n in (128, 256)]
    for r, u in zip(rows, uni):
        for c in ("x", "R"):
            assert r["norms"][c][0] < u["norms"][c][0]
            assert r["norms"][c][1] < u["norms"][c][1]
    o = amr_study.orders(rows)[0]
    assert o["x"][0] > 1.8 and o["R"][0] > 1.8
    assert o["x"][1] > 1.7 and o["R"][1] > 1.7


# ---------------------------------------------------------------------------
# off-plane targets (Section 2 at z != 0): (Fx, Fy, Fz) at height z
# ---------------------------------------------------------------------------

def _rects_uniform(n, h, x0=-1.0, y0=-1.0):
    X, Y = diskgen.grid_centres(n, x0, y0, h)
    rect = np.stack([X.ravel() - h / 2, X.ravel() + h / 2, Y.ravel() - h / 2, Y.ravel() + h / 2], 1)
    return X, Y, rect


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("zcells", [0.5, -3.0])
def test_offplane_uniform_full(gl, prec, zcells):
    """Random linear density on a 64^2 grid, every cell centre at height z,
    against the oracle's off-plane direct sum."""
    n = 64
    h = 2.0 / n
    rng = np.random.default_rng(11)
    s, dx, dy = rng.random((n, n)) + 0.1, rng.standard_normal((n, n)), rng.standard_normal((n, n))
    z = zcells * h
    p = gl.Plan(n, _prec(gl, prec), h0=h, z=z)
    assert p.ncomp == 3
    f = p.solve_xyz(_dev(s, prec), _dev(dx, prec), _dev(dy, prec))
    torch.cuda.synchronize()
    X, Y, rect = _rects_uniform(n, h)
    ref = oracle.direct_z(rect, s.ravel(), dx.ravel(), dy.ravel(), np.stack([X.ravel(), Y.ravel()], 1), z)
    assert _err([_host(c) for c in f], ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_offplane_noisy_spiral_256_sampled(gl, prec):
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 4)
    z = 0.02
    p = gl.Plan(n, _prec(gl, prec), h0=h, z=z)
    f = p.solve_xyz(_dev(s, prec), _dev(dx, prec), _dev(dy, prec))
    torch.cuda.synchronize()
    X, Y, rect = _rects_uniform(n, h)
    sel = np.random.default_rng(5).choice(n * n, 200, replace=False)
    ref = oracle.direct_z(rect, s.ravel(), dx.ravel(), dy.ravel(),
                          np.stack([X.ravel()[sel], Y.ravel()[sel]], 1), z)
    assert _err([_host(c)[sel] for c in f], ref) < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_offplane_amr_table10(gl, prec):
    """The Appendix A layout at height z: every leaf against the leaf sum."""
    lay = diskgen.table10_layout()
    rng = np.random.default_rng(6)
    m = lay.leaf_mask()
    s, dx, dy = [np.where(m, a, 0) for a in (rng.random(lay.total()) + 0.2,
                                               rng.standard_normal(lay.total()),
                                               rng.standard_normal(lay.total()))]
    z = 0.07
    p = gl.Plan(lay.n0, _prec(gl, prec), x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels,
                patches=lay.patches, z=z)
    f = [_host(c) for c in p.solve_xyz(_dev(s, prec), _dev(dx, prec), _dev(dy, prec))]
    torch.cuda.synchronize()
    assert all(np.all(c[~m] == 0) for c in f)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    ref = oracle.direct_z(rect, s[idx], dx[idx], dy[idx], cent, z)
    area = (rect[:, 1] - rect[:, 0]) * (rect[:, 3] - rect[:, 2])
    assert _err([c[idx] for c in f], ref, area) < TOL[prec]


def test_offplane_small_height_tends_to_midplane(gl):
    """(Fx, Fy) just above the disk approach the midplane solve."""
    n = 128
    s, dx, dy, h = diskgen.noisy_spiral(n, 7)
    t = [_dev(a, "f64") for a in (s, dx, dy)]
    mx, my = gl.Plan(n, gl.F64, h0=h).solve(*t)
    fx, fy, fz = gl.Plan(n, gl.F64, h0=h, z=1e-6 * h).solve_xyz(*t)
    torch.cuda.synchronize()
    assert an.rel_l2((_host(fx), _host(fy)), (_host(mx), _host(my))) < 1e-5


def test_amr_and_offplane_without_slopes(gl):
    """Piecewise-constant leaves (one input field) on the AMR path, in the
    plane and above it."""
    lay = diskgen.table10_layout()
    rng = np.random.default_rng(8)
    m = lay.leaf_mask()
    s = np.where(m, rng.random(lay.total()) + 0.2, 0)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    area = (rect[:, 1] - rect[:, 0]) * (rect[:, 3] - rect[:, 2])
    kw = dict(x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels, patches=lay.patches, slopes=False)
    fx, fy = gl.Plan(lay.n0, gl.F64, **kw).solve(_dev(s, "f64"))
    torch.cuda.synchronize()
    ox, oy = oracle.direct(rect, s[idx], None, None, cent)
    assert _err((_host(fx)[idx], _host(fy)[idx]), (ox, oy), area) < TOL["f64"]
    f = gl.Plan(lay.n0, gl.F64, z=-0.04, **kw).solve_xyz(_dev(s, "f64"))
    torch.cuda.synchronize()
    ref = oracle.direct_z(rect, s[idx], None, None, cent, -0.04)
    assert _err([_host(c)[idx] for c in f], ref, area) < TOL["f64"]


def test_injected_allocation_failure_recovers(gl, monkeypatch):
    """With every device allocation failing, a plan that needs new kernel
    spectra reports ENOMEM; once allocations succeed again the same plan
    builds and solves correctly (no half-built spectra are cached)."""
    n = 32  # no earlier test built spectra for this size at this height
    monkeypatch.setenv("GRAVITY_FAIL_ALLOC_AFTER", "0")
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(n, gl.F64, z=0.123)
    assert e.value.status == gl.ENOMEM
    monkeypatch.delenv("GRAVITY_FAIL_ALLOC_AFTER")
    p = gl.Plan(n, gl.F64, z=0.123)
    rng = np.random.default_rng(12)
    s = rng.random((n, n))
    f = p.solve_xyz(_dev(s, "f64"), _dev(np.zeros((n, n)), "f64"), _dev(np.zeros((n, n)), "f64"))
    torch.cuda.synchronize()
    X, Y, rect = _rects_uniform(n, 2.0 / n)
    ref = oracle.direct_z(rect, s.ravel(), None, None, np.stack([X.ravel(), Y.ravel()], 1), 0.123)
    assert _err([_host(c) for c in f], ref) < TOL["f64"]


def test_offplane_entry_points(gl):
    n = 32
    p = gl.Plan(n, gl.F32, z=0.1)
    q = gl.Plan(n, gl.F32)
    a = torch.zeros(n * n, device="cuda")
    with pytest.raises(gl.GravityError) as e:
        p.solve(a, a, a)
    assert e.value.status == gl.EINVAL
    with pytest.raises(gl.GravityError) as e:
        q.solve_xyz(a, a, a)
    assert e.value.status == gl.EINVAL
    ws = torch.empty(gl.batch_workspace_bytes([p]), dtype=torch.uint8, device="cuda")
    with pytest.raises(gl.GravityError) as e:
        gl.solve_batch([p], [a], [a], [a], [a.clone()], [a.clone()], ws)
    assert e.value.status == gl.EUNSUPPORTED
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(n, gl.F32, z=float("nan"))
    assert e.value.status == gl.EINVAL


def test_batch_bitwise_equals_single(gl):
    """Mixed sizes, precisions and layouts; more same-size solves than one
    launch carries (grouping splits them), results bit-identical to singles."""
    sizes = [64, 128, 64, 32] + [64] * 10
    plans, ins, outs, singles = [], [], [], []
    for k, n in enumerate(sizes):
        prec = "f32" if (k % 2 or k >= 4) else "f64"
        p = gl.Plan(n, _prec(gl, prec))
        s, dx, dy = diskgen.random_fields(n, 40 + k)
        t = [_dev(a, prec) for a in (s, dx, dy)]
        plans.append(p)
        ins.append(t)
        singles.append(p.solve(*t))
        outs.append((torch.empty_like(t[0]), torch.empty_like(t[0])))
    lay = diskgen.table10_layout()
    pa = gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=3, patches=lay.patches)
    rng = np.random.default_rng(3)
    ta = [_dev(rng.random(lay.total()), "f64") for _ in range(3)]
    plans.append(pa)
    ins.append(ta)
    singles.append(pa.solve(*ta))
    outs.append((torch.empty_like(ta[0]), torch.empty_like(ta[0])))
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    gl.solve_batch(plans, [t[0] for t in ins], [t[1] for t in ins], [t[2] for t in ins],
                   [o[0] for o in outs], [o[1] for o in outs], ws)
    torch.cuda.synchronize()
    for (a, b), (c, d) in zip(outs, singles):
        assert torch.equal(a, c) and torch.equal(b, d)


def test_deterministic(gl):
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 1)
    a = gpu_uniform(gl, "f32", s, dx, dy, h=h)
    b = gpu_uniform(gl, "f32", s, dx, dy, h=h)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_profiled_solve_equals_solve(gl):
    """The profiling entry point repeats every stage back to back; its outputs
    equal a plain solve's, bit for bit (uniform FP32 and AMR FP64)."""
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 2)
    p = gl.Plan(n, gl.F32, h0=h)
    t = [_dev(a, "f32") for a in (s, dx, dy)]
    fx, fy = p.solve(*t)
    gx, gy = torch.empty_like(fx), torch.empty_like(fy)
    st = p.profile(*t, gx, gy, p.workspace(), reps=3)
    torch.cuda.synchronize()
    assert set(st) == {"row_fwd", "col", "row_inv"} and all(v > 0 for v in st.values())
    assert torch.equal(fx, gx) and torch.equal(fy, gy)
    lay = diskgen.table10_layout()
    rng = np.random.default_rng(4)
    m = lay.leaf_mask()
    fields = [np.where(m, rng.random(lay.total()) + 0.1, 0) for _ in range(3)]
    pa = gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels,
                 patches=lay.patches)
    ta = [_dev(a, "f64") for a in fields]
    ax, ay = pa.solve(*ta)
    bx, by = torch.empty_like(ax), torch.empty_like(ay)
    st = pa.profile(*ta, bx, by, pa.workspace(), reps=2)
    torch.cuda.synchronize()
    assert list(st) == ["row_fwd", "col", "row_inv", "gather"]
    assert torch.equal(ax, bx) and torch.equal(ay, by)


def test_invalid_requests(gl):
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(48, gl.F32)
    assert e.value.status == gl.EUNSUPPORTED
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(8192, gl.F32)
    assert e.value.status == gl.EUNSUPPORTED
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(32, gl.F32, nlevels=2, patches=[(1, 1, 0, 4, 4)])  # odd corner
    assert e.value.status == gl.EINVAL
    with pytest.raises(gl.GravityError) as e:
        gl.Plan(32, gl.F32, nlevels=3, patches=[(2, 0, 0, 8, 8)])  # not nested
    assert e.value.status == gl.EINVAL
    p = gl.Plan(32, gl.F32)
    s = torch.zeros(32 * 32, device="cuda")
    with pytest.raises(gl.GravityError) as e:
        p.solve(s, None, None)  # slopes missing
    assert e.value.status == gl.EINVAL
    # arrays the library cannot size-check are checked by the binding
    with pytest.raises(ValueError, match="fx"):
        p.solve(s, s, s, fx=torch.empty(32 * 31, device="cuda"))
    with pytest.raises(ValueError, match="workspace"):
        p.solve(s, s, s, workspace=torch.empty(max(1, p.workspace_bytes // 2), dtype=torch.uint8,
                                               device="cuda"))
    with pytest.raises(ValueError, match="sigma"):
        p.solve(s.double(), s, s)


def test_empty_batch_is_a_no_op(gl):
    """A batch of no solves queues nothing, in the grouped and the
    persistent form (its workspace is the persistent launch's table room)."""
    ws = torch.empty(max(1, gl.batch_workspace_bytes([])), dtype=torch.uint8, device="cuda")
    gl.solve_batch([], [], None, None, [], [], ws)
    gl.solve_batch([], [], None, None, [], [], ws, persistent=True)
    assert gl.batch_persistent_abandoned([], ws) == 0
    torch.cuda.synchronize()


def test_server_results_same_alone_and_in_mix(gl):
    """Continuous batching: a mixed stream (sizes, precisions, uniform and AMR)
    submitted to a server under a tight HBM budget gives every request the
    bit-identical result of its solo solve, never exceeds the budget, and
    reports latencies."""
    rng = np.random.default_rng(17)
    lay = diskgen.table10_layout()
    lay2, s2, dx2, dy2 = diskgen.amr_config(5, n0=32, nlevels=3, thresh=0.15, a=0.05)
    kinds = []
    for n in (32, 64, 128, 256):
        for prec in ("f32", "f64"):
            kinds.append(("u", n, prec, gl.Plan(n, _prec(gl, prec))))
    kinds.append(("a", lay, "f64", gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0,
                                            nlevels=lay.nlevels, patches=lay.patches)))
    kinds.append(("a", lay2, "f32", gl.Plan(lay2.n0, gl.F32, nlevels=lay2.nlevels,
                                             patches=lay2.patches)))
    budget = max(k[3].workspace_bytes for k in kinds) * 3
    srv = gl.Server(budget, nstreams=3, max_batch=8)
    reqs = []
    for i in range(60):
        kind = kinds[rng.integers(len(kinds))]
        p = kind[3]
        vals = [_dev(rng.random(p.n_cells), kind[2]) for _ in range(3)]
        fx = torch.empty_like(vals[0])
        fy = torch.empty_like(vals[0])
        tk = srv.submit(p, *vals, fx, fy)
        reqs.append((tk, p, vals, fx, fy))
    lat = [srv.wait(r[0]) for r in reqs]
    st = srv.stats()
    assert st["completed"] == 60 and st["pending"] == 0
    assert st["peak_bytes_in_use"] <= budget
    assert min(lat) > 0 and st["latency_p99_ms"] >= st["latency_p50_ms"] > 0
    torch.cuda.synchronize()
    for tk, p, vals, fx, fy in reqs:
        ax, ay = p.solve(*vals)
        torch.cuda.synchronize()
        assert torch.equal(ax, fx) and torch.equal(ay, fy)
    srv.close()


def test_offplane_batch_and_server_match_single_solves(gl):
    """Off-plane plans in a batch (mixed with midplane ones) and through the
    server give the bit-identical results of their single solves."""
    rng = np.random.default_rng(21)
    lay = diskgen.table10_layout()
    plans = [gl.Plan(64, gl.F32, z=0.1), gl.Plan(64, gl.F32, z=0.1), gl.Plan(64, gl.F32),
             gl.Plan(128, gl.F64, z=-0.05),
             gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels,
                     patches=lay.patches, z=0.03)]
    dts = ["f32", "f32", "f32", "f64", "f64"]
    ins = [[_dev(rng.random(p.n_cells), d) for _ in range(3)] for p, d in zip(plans, dts)]
    outs = [[torch.empty_like(v[0]) for _ in range(3)] for v in ins]
    fz = [o[2] if p.ncomp == 3 else None for p, o in zip(plans, outs)]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    gl.solve_batch(plans, [v[0] for v in ins], [v[1] for v in ins], [v[2] for v in ins],
                   [o[0] for o in outs], [o[1] for o in outs], ws, fz=fz)
    torch.cuda.synchronize()
    for p, v, o in zip(plans, ins, outs):
        ref = p.solve_xyz(*v) if p.ncomp == 3 else p.solve(*v)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, o))
    srv = gl.Server(max(p.workspace_bytes for p in plans) * 2, nstreams=2, max_batch=4)
    reqs = []
    for i in range(20):
        k = int(rng.integers(len(plans)))
        p = plans[k]
        vals = [_dev(rng.random(p.n_cells), dts[k]) for _ in range(3)]
        o = [torch.empty_like(vals[0]) for _ in range(3)]
        tk = srv.submit(p, *vals, o[0], o[1], o[2] if p.ncomp == 3 else None)
        reqs.append((tk, p, vals, o))
    for r in reqs:
        srv.wait(r[0])
    torch.cuda.synchronize()
    for tk, p, vals, o in reqs:
        ref = p.solve_xyz(*vals) if p.ncomp == 3 else p.solve(*vals)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, o))
    with pytest.raises(gl.GravityError) as e:
        srv.submit(plans[0], *ins[0], outs[0][0], outs[0][1])   # off-plane without fz
    assert e.value.status == gl.EUNSUPPORTED
    srv.close()


def test_server_rejects_oversized_request(gl):
    p = gl.Plan(128, gl.F32)
    srv = gl.Server(p.workspace_bytes // 2, nstreams=1)
    t = torch.zeros(p.n_cells, device="cuda")
    with pytest.raises(gl.GravityError) as e:
        srv.submit(p, t, t, t, torch.empty_like(t), torch.empty_like(t))
    assert e.value.status == gl.ENOMEM
    srv.close()


def test_solve_replays_from_a_hip_graph(gl):
    """A solve launches kernels only (no allocation, memset or host wait), so
    a caller can capture it in a HIP graph: every replay, with eager work and
    synchronisations between replays, equals the eager result bit for bit."""
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 3)
    lay, a_s, a_dx, a_dy = diskgen.amr_config(2, n0=64, nlevels=3, thresh=0.1, a=0.05)
    cases = []
    for plan, vals in ((gl.Plan(n, gl.F32, h0=h), (s, dx, dy)),
                       (gl.Plan(lay.n0, gl.F64, nlevels=lay.nlevels, patches=lay.patches),
                        (a_s, a_dx, a_dy))):
        dt = plan.torch_dtype
        t = [torch.from_numpy(np.ascontiguousarray(v).ravel()).to("cuda", dt) for v in vals]
        out = (torch.empty(plan.n_cells, dtype=dt, device="cuda"),
               torch.empty(plan.n_cells, dtype=dt, device="cuda"))
        cases.append((plan, t, out, plan.workspace()))
    st = torch.cuda.Stream()
    refs = []
    with torch.cuda.stream(st):
        for plan, t, out, ws in cases:
            plan.solve(*t, fx=out[0], fy=out[1], workspace=ws, stream=st)
    torch.cuda.synchronize()
    refs = [(o[0].clone(), o[1].clone()) for _, _, o, _ in cases]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        for plan, t, out, ws in cases:
            plan.solve(*t, fx=out[0], fy=out[1], workspace=ws, stream=st)
    torch.cuda.synchronize()
    for rep in range(4):
        for _, _, out, _ in cases:
            out[0].fill_(float(rep + 1))
            out[1].fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, out, _), ref in zip(cases, refs):
            assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep
        # eager work between replays
        cases[0][0].solve(*cases[0][1], fx=cases[0][2][0], fy=cases[0][2][1], workspace=cases[0][3])
        torch.cuda.synchronize()


def test_plan_released_during_a_capture(gl):
    """A plan released while the caller captures a graph (a garbage collector
    may drop one at any point) frees its device memory without invalidating
    the capture; the captured solve replays bit for bit."""
    n = 128
    s, dx, dy, h = diskgen.noisy_spiral(n, 4)
    plan = gl.Plan(n, gl.F32, h0=h)
    t = [torch.from_numpy(np.ascontiguousarray(v).ravel()).to("cuda", torch.float32) for v in (s, dx, dy)]
    out = (torch.empty(n * n, device="cuda"), torch.empty(n * n, device="cuda"))
    ws = plan.workspace()
    # a cell size no other plan uses: its kernel spectra are its own, freed
    # when it goes
    doomed = gl.Plan(64, gl.F64, h0=2.0 / 64 * 1.2345)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan.solve(*t, fx=out[0], fy=out[1], workspace=ws, stream=st)
    torch.cuda.synchronize()
    ref = (out[0].clone(), out[1].clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        plan.solve(*t, fx=out[0], fy=out[1], workspace=ws, stream=st)
        doomed.close()
    for rep in range(2):
        out[0].fill_(0.0)
        out[1].fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep


def test_server_waits_for_the_callers_stream(gl):
    """Inputs still being written on the caller's stream when the request is
    submitted: the server's work waits for that stream (an event recorded at
    submit), so the result is the solve of the final inputs."""
    n = 256
    p = gl.Plan(n, gl.F32)
    s, dx, dy, h = diskgen.noisy_spiral(n, 5)
    final = [_dev(a, "f32") for a in (s, dx, dy)]
    ref = p.solve(*final)
    torch.cuda.synchronize()
    srv = gl.Server(4 * p.workspace_bytes, nstreams=2)
    side = torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    outs = []
    for rep in range(3):
        ins = [torch.zeros_like(t) for t in final]
        o = (torch.full_like(final[0], float("nan")), torch.full_like(final[0], float("nan")))
        with torch.cuda.stream(side):
            for _ in range(4):               # keep the side stream busy first
                big = (big @ big).tanh_()
            for t, f in zip(ins, final):
                t.copy_(f)
            tk = srv.submit(p, *ins, *o, stream=side)
        outs.append((tk, ins, o))
    for tk, ins, o in outs:
        srv.wait(tk)
        assert torch.equal(o[0], ref[0]) and torch.equal(o[1], ref[1])
    srv.close()
