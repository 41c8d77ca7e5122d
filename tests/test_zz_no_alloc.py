"""The allocation-free solve (gravity_solve_noalloc): its workspace is the
library's static per-device scratch array.  Two calls in a row, the second
on a smaller input, each bit-identical to gravity_solve with a caller
workspace and within the parity tolerance of the oracle; oversize plans are
rejected with EUNSUPPORTED."""
import numpy as np
import pytest

import diskgen
import oracle
from oracle import analytic as an

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_02765_amd as m
    return m


def _run(gl, plan, fields, dt):
    t = [torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda", dt) for a in fields]
    ref = plan.solve(*t)
    # outputs pre-filled with garbage: the call must write every element
    fx = torch.full((plan.n_cells,), float("nan"), dtype=dt, device="cuda")
    fy = torch.full((plan.n_cells,), 7.0, dtype=dt, device="cuda")
    out = plan.solve_noalloc(*t, fx=fx, fy=fy)
    torch.cuda.synchronize()
    assert out[0] is fx and out[1] is fy
    assert torch.equal(fx, ref[0]) and torch.equal(fy, ref[1])
    return fx.double().cpu().numpy(), fy.double().cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_noalloc_matches_solve_twice_second_smaller(gl, prec, tol):
    dt = torch.float32 if prec == "f32" else torch.float64
    P = gl.F32 if prec == "f32" else gl.F64
    for n, seed in ((256, 3), (64, 4)):   # second call smaller
        s, dx, dy, h = diskgen.noisy_spiral(n, seed)
        plan = gl.Plan(n, P, h0=h)
        assert plan.workspace_bytes <= gl.NOALLOC_SCRATCH_BYTES
        fx, fy = _run(gl, plan, (s, dx, dy), dt)
        rng = np.random.default_rng(seed)
        tg = rng.choice(n * n, 64, replace=False)
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, targets=tg)
        assert an.rel_l2((fx[tg], fy[tg]), (ox, oy)) < tol


def test_noalloc_amr_and_headline_size(gl):
    """An AMR plan (lattice-corner family, gather) and the 1024^2 FP32 plan,
    the largest uniform FP32 plan the scratch array holds."""
    lay = diskgen.table10_layout()
    rng = np.random.default_rng(5)
    m = lay.leaf_mask()
    vals = [np.where(m, rng.random(lay.total()) + 0.1, 0.0) for _ in range(3)]
    p = gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels,
                patches=lay.patches)
    fx, fy = _run(gl, p, vals, torch.float64)
    rect, cent, idx = oracle.leaves_of_composite(lay)
    ox, oy = oracle.direct(rect, vals[0][idx], vals[1][idx], vals[2][idx], cent)
    assert an.rel_l2((fx[idx], fy[idx]), (ox, oy)) < 1e-12
    n = 1024
    s, dx, dy, h = diskgen.noisy_spiral(n, 0)
    p = gl.Plan(n, gl.F32, h0=h)
    fx, fy = _run(gl, p, (s, dx, dy), torch.float32)
    tg = np.concatenate([np.random.default_rng(8).choice(n * n, 24, replace=False), [0, n * n - 1]])
    ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, h, targets=tg)
    assert an.rel_l2((fx[tg], fy[tg]), (ox, oy)) < 1e-5


def test_noalloc_rejects_oversize_plan(gl):
    p = gl.Plan(1024, gl.F64)   # 84 MB of workspace
    assert p.workspace_bytes > gl.NOALLOC_SCRATCH_BYTES
    t = torch.zeros(p.n_cells, dtype=torch.float64, device="cuda")
    with pytest.raises(gl.GravityError) as e:
        p.solve_noalloc(t, t, t)
    assert e.value.status == gl.EUNSUPPORTED
