"""GPU parity of every reachable kernel variant, element by element.

The plan's autotuner picks one variant of each of the three FFT kernels by
timing; any valid id can also be forced (GRAVITY_VARIANTS="rf,col,ri").  Here
every valid id of each kernel is forced in turn (the other two kernels at the
autotuned choice) and the result is compared with the oracle:
  * the whole 256^2 grid (512-point transforms);
  * 1024^2 (2048-point transforms, the benchmark's size): one full row, one
    full column (every row group of every XCD's share), and 256 random cells;
  * 3-level AMR layouts on 2048^2 and 4096^2 finest lattices (4096- and
    8192-point transforms, both kernel families, so the family-split column
    variants too): leaves sampled on every level.
Both precisions; both the relative L2 over the targets and a per-element
bound |dF_i| <= tol * max|F| are asserted.  Single-source tests pin every
entry of both kernel families (closed form and all Gauss-Legendre orders).
"""
import numpy as np
import pytest

import diskgen
import oracle
from oracle import analytic as an

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
N_ROW_VARIANTS, COL_VARIANTS = 12, (0, 1, 2, 3, 4, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16)


@pytest.fixture(scope="module")
def gl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_02765_amd as m
    return m


def _prec(gl, name):
    return gl.F64 if name == "f64" else gl.F32


def _dev(a, name):
    dt = torch.float64 if name == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda", dt)


def max_rel(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i| over all components."""
    num = max(float(np.max(np.abs(np.asarray(g) - np.asarray(r)))) for g, r in zip(got, ref))
    den = max(float(np.max(np.abs(np.asarray(r)))) for r in ref)
    return num / den


def _variant_sets(base):
    """(rf, col, ri) triples: each kernel's ids in turn, the others at base."""
    out = []
    for v in range(N_ROW_VARIANTS):
        out.append((v, base[1], base[2]))
    for v in COL_VARIANTS:
        out.append((base[0], v, base[2]))
    for v in range(N_ROW_VARIANTS):
        out.append((base[0], base[1], v))
    return sorted(set(out))


def _forced_plans(gl, monkeypatch, make):
    """Yield (variants, plan) for every valid forced variant triple."""
    monkeypatch.delenv("GRAVITY_VARIANTS", raising=False)
    base = make().variants
    n_ok = 0
    for vs in _variant_sets(base):
        monkeypatch.setenv("GRAVITY_VARIANTS", "%d,%d,%d" % vs)
        try:
            p = make()
        except gl.GravityError as e:
            assert e.status == gl.EINVAL, e
            continue
        assert tuple(p.variants) == vs
        n_ok += 1
        yield vs, p
    monkeypatch.delenv("GRAVITY_VARIANTS")
    assert n_ok >= 3


@pytest.fixture(scope="module")
def spiral256():
    n = 256
    s, dx, dy, h = diskgen.noisy_spiral(n, 11)
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h)
    return n, (s, dx, dy), h, (ox.ravel(), oy.ravel())


@pytest.fixture(scope="module")
def spiral1024():
    n = 1024
    s, dx, dy, h = diskgen.noisy_spiral(n, 0)
    rng = np.random.default_rng(1024)
    row = 517 * n + np.arange(n)
    col = np.arange(n) * n + 300
    tg = np.unique(np.concatenate([row, col, rng.choice(n * n, 256, replace=False),
                                   [0, n - 1, n * (n - 1), n * n - 1]]))
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, targets=tg)
    return n, (s, dx, dy), h, tg, (ox, oy)


def _amr_case(n0):
    lay = diskgen.ilr_layout(n0, 3, "d2")
    s, dx, dy = lay.sample(diskgen.d2)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(4 * n0)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(40, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent[sel])
    area = (rect[sel, 1] - rect[sel, 0]) * (rect[sel, 3] - rect[sel, 2])
    return lay, (s, dx, dy), idx[sel], area, (ox, oy)


@pytest.fixture(scope="module")
def amr_cases():
    return {2048: _amr_case(512), 4096: _amr_case(1024)}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_variant_256_full(gl, monkeypatch, spiral256, prec):
    n, fields, h, ref = spiral256
    t = [_dev(a, prec) for a in fields]
    worst = (0.0, 0.0)
    for vs, p in _forced_plans(gl, monkeypatch, lambda: gl.Plan(n, _prec(gl, prec), h0=h)):
        fx, fy = p.solve(*t)
        torch.cuda.synchronize()
        got = (fx.double().cpu().numpy(), fy.double().cpu().numpy())
        e2, em = an.rel_l2(got, ref), max_rel(got, ref)
        assert e2 < TOL[prec] and em < TOL[prec], (vs, e2, em)
        worst = (max(worst[0], e2), max(worst[1], em))
    print("256^2 %s worst rel_l2 %.3e max_rel %.3e" % (prec, *worst))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_variant_1024_row_column_sampled(gl, monkeypatch, spiral1024, prec):
    n, fields, h, tg, ref = spiral1024
    t = [_dev(a, prec) for a in fields]
    worst = (0.0, 0.0)
    for vs, p in _forced_plans(gl, monkeypatch, lambda: gl.Plan(n, _prec(gl, prec), h0=h)):
        fx, fy = p.solve(*t)
        torch.cuda.synchronize()
        got = (fx.double().cpu().numpy()[tg], fy.double().cpu().numpy()[tg])
        e2, em = an.rel_l2(got, ref), max_rel(got, ref)
        assert e2 < TOL[prec] and em < TOL[prec], (vs, e2, em)
        worst = (max(worst[0], e2), max(worst[1], em))
    print("1024^2 %s worst rel_l2 %.3e max_rel %.3e" % (prec, *worst))


@pytest.mark.parametrize("nf", [2048, 4096])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_variant_amr_large_transforms(gl, monkeypatch, amr_cases, prec, nf):
    lay, fields, sel, area, ref = amr_cases[nf]
    t = [_dev(a, prec) for a in fields]
    worst = (0.0, 0.0)

    def make():
        return gl.Plan(lay.n0, _prec(gl, prec), nlevels=lay.nlevels, patches=lay.patches)
    for vs, p in _forced_plans(gl, monkeypatch, make):
        assert p.fft_size == 2 * nf
        fx, fy = p.solve(*t)
        torch.cuda.synchronize()
        got = (fx.double().cpu().numpy()[sel], fy.double().cpu().numpy()[sel])
        e2, em = an.rel_l2(got, ref, area), max_rel(got, ref)
        assert e2 < TOL[prec] and em < TOL[prec], (vs, e2, em)
        worst = (max(worst[0], e2), max(worst[1], em))
        del p, fx, fy
    print("AMR %d^2 finest %s worst rel_l2 %.3e max_rel %.3e" % (nf, prec, *worst))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_column_variant_offplane_amr(gl, monkeypatch, prec):
    """Targets at a height above a 3-level AMR layout on a 2048^2 finest
    lattice (4096-point transforms, both kernel families, three force
    components): every valid column variant, the family-split ones
    included, against the off-plane leaf sum on sampled leaves of every
    level."""
    lay = diskgen.ilr_layout(512, 3, "d2")
    s, dx, dy = lay.sample(diskgen.d2)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(2048)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(12, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    z = 0.05
    ref = oracle.direct_z(rect, s[idx], dx[idx], dy[idx], cent[sel], z)
    area = (rect[sel, 1] - rect[sel, 0]) ** 2
    t = [_dev(a, prec) for a in (s, dx, dy)]

    def make():
        return gl.Plan(lay.n0, _prec(gl, prec), nlevels=lay.nlevels, patches=lay.patches, z=z)
    monkeypatch.delenv("GRAVITY_VARIANTS", raising=False)
    base = make().variants
    n_ok, worst = 0, (0.0, 0.0)
    for v in COL_VARIANTS:
        monkeypatch.setenv("GRAVITY_VARIANTS", "%d,%d,%d" % (base[0], v, base[2]))
        try:
            p = make()
        except gl.GravityError as e:
            assert e.status == gl.EINVAL, e
            continue
        assert p.fft_size == 4096
        n_ok += 1
        f = p.solve_xyz(*t)
        torch.cuda.synchronize()
        got = [c.double().cpu().numpy()[idx[sel]] for c in f]
        e2, em = an.rel_l2(got, ref, area), max_rel(got, ref)
        assert e2 < TOL[prec] and em < TOL[prec], (v, e2, em)
        worst = (max(worst[0], e2), max(worst[1], em))
        del p, f
    monkeypatch.delenv("GRAVITY_VARIANTS")
    assert n_ok >= 3
    print("off-plane AMR 2048^2 finest %s: %d column variants, worst rel_l2 %.3e max_rel %.3e"
          % (prec, n_ok, *worst))


def _single_source_check(fx, fy, ox, oy, prec, what):
    e2 = an.rel_l2((fx, fy), (ox, oy))
    em = max_rel((fx, fy), (ox, oy))
    print("%s %s rel_l2 %.3e max_rel %.3e" % (what, prec, e2, em))
    assert e2 < TOL[prec] and em < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_source_centre_family_every_offset(gl, prec):
    """One source cell (value and both slopes) in the corner of a 256^2 grid:
    every target is one entry of each cell-centre kernel table (offsets 0 to
    255 cells: the closed form and all four Gauss-Legendre orders), against
    the oracle's exact kernels of that one source."""
    n = 256
    h = 2.0 / n
    s, dx, dy = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    s[0, 0], dx[0, 0], dy[0, 0] = 1.0, 0.7, -1.3
    p = gl.Plan(n, _prec(gl, prec), h0=h, G=1.5)
    fx, fy = p.solve(*[_dev(a, prec) for a in (s, dx, dy)])
    torch.cuda.synchronize()
    X, Y = diskgen.grid_centres(n)
    rect = np.array([[-1.0, -1.0 + h, -1.0, -1.0 + h]])
    ox, oy = oracle.direct(rect, [1.0], [0.7], [-1.3], np.stack([X.ravel(), Y.ravel()], 1), G=1.5)
    _single_source_check(fx.double().cpu().numpy(), fy.double().cpu().numpy(), ox, oy, prec,
                         "centre family")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_source_corner_family_every_offset(gl, prec):
    """Two levels: base 128^2 with one base cell refined.  The only source is
    one of its four fine cells; every coarse leaf is a target at a lattice
    corner of the 256^2 finest lattice, so the targets cover every entry of
    the lattice-corner kernel tables out to 255 cells."""
    n0 = 128
    lay = diskgen.Layout(n0, 2, [diskgen.Patch(1, 0, 0, 2, 2)])
    s, dx, dy = np.zeros(lay.total()), np.zeros(lay.total()), np.zeros(lay.total())
    src = n0 * n0 + 3   # the upper-right fine cell of the refined base cell
    s[src], dx[src], dy[src] = 1.0, -0.4, 0.9
    p = gl.Plan(n0, _prec(gl, prec), nlevels=2, patches=lay.patches, G=0.8)
    fx, fy = p.solve(*[_dev(a, prec) for a in (s, dx, dy)])
    torch.cuda.synchronize()
    rect, cent, idx = oracle.leaves_of_composite(lay)
    k = int(np.nonzero(idx == src)[0][0])
    ox, oy = oracle.direct(rect[k:k + 1], [1.0], [-0.4], [0.9], cent, G=0.8)
    fx, fy = fx.double().cpu().numpy()[idx], fy.double().cpu().numpy()[idx]
    coarse = (rect[:, 1] - rect[:, 0]) > 1.5 * (2.0 / 256)
    assert np.count_nonzero(coarse) == n0 * n0 - 1
    _single_source_check(fx, fy, ox, oy, prec, "corner family (all leaves)")
    _single_source_check(fx[coarse], fy[coarse], ox[coarse], oy[coarse], prec,
                         "corner family (coarse leaves)")


def test_batch_of_64_disks_against_oracle(gl):
    """The 64-disk FP32 batch (sizes 64^2..1024^2) in one gravity_solve_batch:
    sampled targets of every disk against the oracle."""
    disks = diskgen.batch_disks(0)
    plans = [gl.Plan(n, gl.F32) for (n, _, _, _) in disks]
    ins = [[_dev(a, "f32") for a in d[1:]] for d in disks]
    outs = [(torch.empty_like(i[0]), torch.empty_like(i[0])) for i in ins]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    gl.solve_batch(plans, [i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins],
                   [o[0] for o in outs], [o[1] for o in outs], ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(64)
    worst = (0.0, 0.0)
    for (n, s, dx, dy), (fx, fy) in zip(disks, outs):
        tg = np.concatenate([rng.choice(n * n, 12, replace=False), [0, n * n - 1]])
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n, targets=tg)
        got = (fx.double().cpu().numpy()[tg], fy.double().cpu().numpy()[tg])
        e2, em = an.rel_l2(got, (ox, oy)), max_rel(got, (ox, oy))
        assert e2 < TOL["f32"] and em < TOL["f32"], (n, e2, em)
        worst = (max(worst[0], e2), max(worst[1], em))
    print("64-disk batch worst rel_l2 %.3e max_rel %.3e" % worst)


def test_served_request_with_4096_finest_lattice_against_oracle(gl):
    """A served AMR request on a 4096^2 finest lattice (8192-point
    transforms), through the server in a mix with smaller requests: sampled
    leaves of every level against the leaf direct sum."""
    big = None
    for lay, prof in diskgen.request_pool_full(0, bases=(1024, 512), levels=(3, 4)):
        if lay.n_finest == 4096:
            big = (lay, prof)
            break
    assert big is not None
    lay, prof = big
    s, dx, dy = lay.sample(prof)
    p = gl.Plan(lay.n0, gl.F32, nlevels=lay.nlevels, patches=lay.patches)
    small = gl.Plan(128, gl.F32)
    t = [_dev(a, "f32") for a in (s, dx, dy)]
    fx, fy = torch.empty_like(t[0]), torch.empty_like(t[0])
    srv = gl.Server(p.workspace_bytes + 4 * small.workspace_bytes, nstreams=2)
    st = [_dev(a, "f32") for a in diskgen.random_fields(128, 5)]
    others = [(torch.empty_like(st[0]), torch.empty_like(st[0])) for _ in range(4)]
    torch.cuda.synchronize()   # inputs written on torch's stream before the server reads them
    tks = [srv.submit(small, *st, *o) for o in others[:2]]
    tks.append(srv.submit(p, *t, fx, fy))
    tks += [srv.submit(small, *st, *o) for o in others[2:]]
    for tk in tks:
        srv.wait(tk)
    srv.close()
    rect, cent, idx = oracle.leaves_of_composite(lay)
    size = rect[:, 1] - rect[:, 0]
    rng = np.random.default_rng(77)
    sel = []
    for hv in np.unique(size):
        cand = np.nonzero(size == hv)[0]
        sel.extend(rng.choice(cand, min(24, len(cand)), replace=False))
    sel = np.array(sorted(sel))
    ox, oy = oracle.direct(rect, s[idx], dx[idx], dy[idx], cent[sel])
    area = (rect[sel, 1] - rect[sel, 0]) * (rect[sel, 3] - rect[sel, 2])
    got = (fx.double().cpu().numpy()[idx[sel]], fy.double().cpu().numpy()[idx[sel]])
    e2, em = an.rel_l2(got, (ox, oy), area), max_rel(got, (ox, oy))
    print("served 4096^2-finest request (%d levels, %d patches) rel_l2 %.3e max_rel %.3e"
          % (lay.nlevels, len(lay.patches), e2, em))
    assert e2 < TOL["f32"] and em < TOL["f32"]
