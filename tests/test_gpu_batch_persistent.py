"""GPU parity of the persistent batch launch (gravity_solve_batch_persistent):
mixed-size uniform solves in one launch per precision, against the oracle and
against single solves; the solves it does not take (AMR, 32^2, no slopes)
run as grouped launches in the same call and keep their single solves' bits.

Tolerances: relative L2 and max|dF| / max|F| <= 1e-12 (FP64), <= 1e-5 (FP32)
against the oracle; against gravity_solve (tuned variants, other transform
shapes) the same bounds, as both are within them of the exact sum.
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


def _dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda", dt)


def max_rel(got, ref):
    num = max(float(np.max(np.abs(np.asarray(g) - np.asarray(r)))) for g, r in zip(got, ref))
    den = max(float(np.max(np.abs(np.asarray(r)))) for r in ref)
    return num / den


def _run(gl, plans, ins, persistent, reps=1):
    outs = [(torch.full_like(i[0], float("nan")), torch.full_like(i[0], float("nan"))) for i in ins]
    ws = torch.empty(gl.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    for _ in range(reps):
        gl.solve_batch(plans, [i[0] for i in ins], [i[1] for i in ins], [i[2] for i in ins],
                       [o[0] for o in outs], [o[1] for o in outs], ws, persistent=persistent)
        if persistent:  # no unit gave up waiting
            assert gl.batch_persistent_abandoned(plans, ws) == 0
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_persistent_64_disk_batch_against_oracle(gl, prec):
    """The 64-disk workload (sizes 64^2..1024^2) in one persistent launch:
    sampled cells of every disk against the oracle, and every cell against
    the disk's single solve."""
    disks = diskgen.batch_disks(0)
    P = gl.F64 if prec == "f64" else gl.F32
    plans = [gl.Plan(n, P) for (n, _, _, _) in disks]
    ins = [[_dev(a, prec) for a in d[1:]] for d in disks]
    outs = _run(gl, plans, ins, True, reps=2)
    rng = np.random.default_rng(77)
    worst = [0.0, 0.0, 0.0]
    for (n, s, dx, dy), p, i, (fx, fy) in zip(disks, plans, ins, outs):
        tg = np.concatenate([rng.choice(n * n, 6, replace=False), [0, n * n - 1]])
        ox, oy = oracle.uniform(s, dx, dy, -1.0, -1.0, 2.0 / n, targets=tg)
        got = (fx.double().cpu().numpy()[tg], fy.double().cpu().numpy()[tg])
        e2, em = an.rel_l2(got, (ox, oy)), max_rel(got, (ox, oy))
        rx, ry = p.solve(*i)
        torch.cuda.synchronize()
        es = an.rel_l2((fx.double().cpu().numpy(), fy.double().cpu().numpy()),
                       (rx.double().cpu().numpy(), ry.double().cpu().numpy()))
        assert e2 < TOL[prec] and em < TOL[prec] and es < TOL[prec], (n, e2, em, es)
        worst = [max(worst[0], e2), max(worst[1], em), max(worst[2], es)]
    print("persistent 64-disk %s: worst rel_l2 %.3e max_rel %.3e vs single solve %.3e" % (prec, *worst))


def test_persistent_many_small_disks_mixed_precision_and_leftovers(gl):
    """200 small disks (64^2..256^2) in FP32 and FP64 together, plus solves
    the persistent launch does not take (an AMR layout, a 32^2 grid, a grid
    without slopes): the persistent ones match their single solves to the
    parity bound, the others bit for bit."""
    rng = np.random.default_rng(5)
    plans, ins, kinds = [], [], []
    for k in range(200):
        n = int(rng.choice([64, 128, 256]))
        prec = "f64" if k % 3 == 0 else "f32"
        plans.append(gl.Plan(n, gl.F64 if prec == "f64" else gl.F32))
        s, dx, dy = diskgen.random_fields(n, 1000 + k)
        ins.append([_dev(a, prec) for a in (s, dx, dy)])
        kinds.append(("persistent", prec))
    lay = diskgen.table10_layout()
    plans.append(gl.Plan(lay.n0, gl.F64, x0=lay.x0, y0=lay.y0, h0=lay.h0, nlevels=lay.nlevels,
                         patches=lay.patches))
    ins.append([_dev(rng.random(lay.total()), "f64") for _ in range(3)])
    kinds.append(("grouped", "f64"))
    plans.append(gl.Plan(16, gl.F32))
    ins.append([_dev(rng.random(16 * 16), "f32") for _ in range(3)])
    kinds.append(("grouped", "f32"))
    outs = _run(gl, plans, ins, True)
    for p, i, o, (kind, prec) in zip(plans, ins, outs, kinds):
        rx, ry = p.solve(*i)
        torch.cuda.synchronize()
        if kind == "grouped":
            assert torch.equal(rx, o[0]) and torch.equal(ry, o[1])
        else:
            got = (o[0].double().cpu().numpy(), o[1].double().cpu().numpy())
            ref = (rx.double().cpu().numpy(), ry.double().cpu().numpy())
            assert an.rel_l2(got, ref) < TOL[prec] and max_rel(got, ref) < TOL[prec]
    # the same solves again, and a smaller batch right after: the tables and
    # counters of each call start fresh
    outs2 = _run(gl, plans, ins, True)
    for a, b in zip(outs, outs2):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    outs3 = _run(gl, plans[:7], ins[:7], True)
    for a, b in zip(outs[:7], outs3):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_persistent_without_slopes_falls_back(gl):
    n = 64
    p = gl.Plan(n, gl.F32, slopes=False)
    s, _, _ = diskgen.random_fields(n, 9, slopes=False)
    t = _dev(s, "f32")
    fx, fy = torch.empty_like(t), torch.empty_like(t)
    ws = torch.empty(gl.batch_workspace_bytes([p]), dtype=torch.uint8, device="cuda")
    gl.solve_batch([p], [t], None, None, [fx], [fy], ws, persistent=True)
    rx, ry = p.solve(t)
    torch.cuda.synchronize()
    assert torch.equal(rx, fx) and torch.equal(ry, fy)
