"""GPU parity of the batched general CQK solve (Algorithm 1 per row,
Section 2.1) and of its VJP w.r.t. a and r against the CPU oracle, through
the C ABI (cqk_solve_batched_f64/_f32, cqk_solve_batched_backward_f64/_f32).

Rows of at most 512 values are solved by one wave, longer rows by a
workgroup; the sizes below mix both, with ragged lengths and empty rows.
Every row is held to the single-instance FP64 bar (tests/parity.py), its
multiplier to the oracle's where the oracle calls it unique, and bad rows
must not disturb the others."""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W
from tests.parity import check_cqk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_15910_amd as cqk
    c = cqk.Context(0)
    yield c
    c.close()


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


def _run(ctx, off, inst, dtype=torch.float64, **kw):
    t = [_dev(inst[k], dtype) for k in "dablu"]
    nseg = off.size - 1
    lam = torch.full((nseg,), -7.0, dtype=torch.float64, device="cuda")
    sts = torch.full((nseg,), -7, dtype=torch.int32, device="cuda")
    x, info = ctx.solve_batched(*t, _dev(off, torch.int64), _dev(inst["r"]), lambda_out=lam,
                                status_out=sts, check=False, **kw)
    return x.cpu().numpy(), lam.cpu().numpy(), sts.cpu().numpy(), info


def _row(inst, off, s):
    lo, hi = int(off[s]), int(off[s + 1])
    return {k: np.asarray(inst[k])[lo:hi] for k in "dablu"} | {"r": float(inst["r"][s])}


def _check_rows(x, lam, sts, off, inst, rows=None, tol=1e-10):
    res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"]) if rows is None \
        else None
    for k, s in enumerate(range(off.size - 1) if rows is None else rows):
        row = _row(inst, off, s)
        ref = res[s] if res is not None else O.solve_cqk(*[row[c] for c in "dablu"], row["r"])
        assert ref.status == O.OK
        assert sts[s] == 0, (s, sts[s])
        lo, hi = int(off[s]), int(off[s + 1])
        if hi > lo:
            check_cqk(x[lo:hi], row, ref, tol)
        if ref.unique and hi > lo:
            # x is the parity claim; the multiplier only has to be the one
            # that x came from (stopping criteria bound phi, not lam)
            assert abs(lam[s] - ref.lam) <= 1e-6 * max(1.0, abs(ref.lam)), (s, lam[s], ref.lam)


@pytest.mark.parametrize("nseg,lo,hi", [(1, 1, 1), (1, 300, 300), (7, 1, 5000),
                                        (300, 1, 3000), (64, 200, 20000)])
@pytest.mark.parametrize("start", ["zero", "formula"])
def test_batched_cqk_parity(ctx, nseg, lo, hi, start):
    off, inst = W.cqk_batched(nseg, lo, hi, 11 + nseg)
    x, lam, sts, info = _run(ctx, off, inst, lambda0=start)
    assert info["status"] == 0, info
    _check_rows(x, lam, sts, off, inst)
    assert 1 <= info["iterations"] <= 30


def test_batched_cqk_user_start(ctx):
    off, inst = W.cqk_batched(40, 10, 2000, 5)
    x, lam, sts, info = _run(ctx, off, inst, lambda0="user", lambda0_user=-0.3)
    assert info["status"] == 0, info
    _check_rows(x, lam, sts, off, inst)


def test_batched_cqk_every_length_near_the_wave_limit(ctx):
    """Lengths around 256 and 506..518 straddle the wave-row limit (512) and
    the register tiers below it."""
    lens = np.concatenate([np.arange(250, 263), np.arange(506, 519)])
    off = np.concatenate([[0], np.cumsum(lens)])
    inst = W.cqk_uniform(int(off[-1]), 7)
    mid = inst["b"] * (inst["l"] + inst["u"]) * 0.5
    inst["r"] = np.array([float(np.sum(mid[off[s]:off[s + 1]])) for s in range(lens.size)])
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 0
    _check_rows(x, lam, sts, off, inst)


def test_batched_cqk_generators(ctx):
    """Rows drawn from the correlated and the paper's classes (one row each
    per class, short and long)."""
    rows = []
    for n, f in ((100, lambda: W.cqk_correlated(100, 3)), (5000, lambda: W.cqk_correlated(5000, 4)),
                 (90, lambda: W.cqk_paper(90, 5, "weak")), (7000, lambda: W.cqk_paper(7000, 6, "correlated")),
                 (200, lambda: W.cqk_paper(200, 7, "uncorrelated"))):
        rows.append(f())
    off = np.concatenate([[0], np.cumsum([r["d"].size for r in rows])])
    inst = {k: np.concatenate([r[k] for r in rows]) for k in "dablu"}
    inst["r"] = np.array([r["r"] for r in rows])
    x, lam, sts, info = _run(ctx, off, inst, lambda0="formula")
    assert info["status"] == 0
    _check_rows(x, lam, sts, off, inst)


def test_batched_cqk_bad_rows_do_not_disturb_others(ctx):
    off, inst = W.cqk_batched(12, 50, 1500, 9)
    inst = {k: np.array(v, copy=True) for k, v in inst.items()}
    # row 2: infeasible r; row 5: d <= 0; row 7: empty-length stays as is;
    # row 9: non-finite r; row 10 (long if possible): b <= 0
    inst["r"][2] = float(np.sum((inst["b"] * inst["u"])[off[2]:off[3]])) + 10.0
    inst["d"][off[5]] = -1.0
    inst["r"][9] = np.inf
    inst["b"][off[11] - 1] = 0.0
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 2   # INVALID_ARG outranks INFEASIBLE
    assert sts[2] == 1 and sts[5] == 2 and sts[9] == 2 and sts[10] == 2
    for s in (2, 5, 9, 10):
        assert np.isnan(lam[s]) and np.all(np.isnan(x[off[s]:off[s + 1]]))
    good = [s for s in range(12) if s not in (2, 5, 9, 10)]
    _check_rows(x, lam, sts, off, inst, rows=good)
    # infeasible alone
    inst2 = W.cqk_batched(5, 10, 400, 10)[1]
    off2 = W.cqk_batched(5, 10, 400, 10)[0]
    inst2["r"] = np.array(inst2["r"], copy=True)
    inst2["r"][1] = -1e9
    _, _, sts2, info2 = _run(ctx, off2, inst2)
    assert info2["status"] == 1 and sts2[1] == 1


def test_batched_cqk_empty_rows(ctx):
    off = np.array([0, 0, 5, 5, 305, 305])
    inst = W.cqk_uniform(305, 12)
    mid = inst["b"] * (inst["l"] + inst["u"]) * 0.5
    inst["r"] = np.array([0.0, float(np.sum(mid[0:5])), 0.0, float(np.sum(mid[5:305])), 0.0])
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 0 and np.all(sts == 0)
    assert lam[0] == 0.0 and lam[2] == 0.0 and lam[4] == 0.0
    _check_rows(x, lam, sts, off, inst, rows=[1, 3])
    inst["r"][2] = 1.0
    _, _, sts, info = _run(ctx, off, inst)
    assert info["status"] == 1 and sts[2] == 1


def test_batched_cqk_deterministic(ctx):
    off, inst = W.cqk_batched(500, 1, 8000, 13)
    x1, l1, _, _ = _run(ctx, off, inst)
    x2, l2, _, _ = _run(ctx, off, inst)
    assert np.array_equal(x1, x2) and np.array_equal(l1, l2)


def test_batched_cqk_full_size_sampled(ctx):
    """8192 rows, lengths log-uniform in [64, 65536] (the batched simplex
    shape, FP64): 48 sampled rows against the oracle, every row by eq. (opt)
    and eq. (xopt) at its returned multiplier."""
    off, inst = W.cqk_batched(8192, 64, 65536, 1)
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 0 and np.all(sts == 0)
    rng = np.random.default_rng(3)
    _check_rows(x, lam, sts, off, inst, rows=sorted(rng.choice(8192, 48, replace=False)))
    d, a, b, l, u = (inst[k] for k in "dablu")
    for s in range(8192):
        lo, hi = int(off[s]), int(off[s + 1])
        xs = x[lo:hi]
        bs = b[lo:hi]
        xo = O.x_of_lambda(lam[s], d[lo:hi], a[lo:hi], bs, l[lo:hi], u[lo:hi])
        assert np.max(np.abs(xs - xo)) <= 1e-10 * max(1.0, float(np.max(np.abs(xo))))
        assert abs(float(np.dot(bs, xs)) - inst["r"][s]) <= \
            1e-10 * float(np.sum(np.abs(bs))) * max(float(np.max(np.abs(xs))), 1e-300) + 1e-12


# ---------------------------------------------------------------------------
# VJP
# ---------------------------------------------------------------------------
def _vjp(ctx, off, inst, x, g, dtype=torch.float64):
    t = {k: _dev(inst[k], dtype) for k in "dblu"}
    nseg = off.size - 1
    gr = torch.full((nseg,), -7.0, dtype=torch.float64, device="cuda")
    ga = ctx.solve_batched_backward(_dev(x, dtype), _dev(g, dtype), t["d"], t["b"], t["l"],
                                    t["u"],
                                    _dev(off, torch.int64), grad_r=gr)
    return ga.cpu().numpy(), gr.cpu().numpy()


@pytest.mark.parametrize("nseg,lo,hi", [(1, 5, 5), (50, 1, 3000), (200, 100, 10000)])
def test_batched_cqk_vjp_parity(ctx, nseg, lo, hi):
    off, inst = W.cqk_batched(nseg, lo, hi, 31 + nseg)
    res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
    x = np.concatenate([r.x for r in res])
    g = np.random.default_rng(32).standard_normal(x.size)
    ga, gr = _vjp(ctx, off, inst, x, g)
    ga_ref, gr_ref = O.cqk_vjp_batched(x, g, inst["d"], inst["b"], inst["l"], inst["u"], off)
    scale = max(1.0, float(np.max(np.abs(ga_ref))), float(np.max(np.abs(gr_ref))))
    assert np.max(np.abs(ga - ga_ref)) <= 1e-10 * scale
    assert np.max(np.abs(gr - gr_ref)) <= 1e-10 * scale


def _round32(inst):
    """The instance as float32 values, held in float64 for the oracle."""
    return {k: (np.asarray(v, dtype=np.float32).astype(np.float64) if k in "dablu" else v)
            for k, v in inst.items()}


@pytest.mark.parametrize("nseg,lo,hi", [(1, 1, 1), (9, 1, 5000), (300, 1, 3000),
                                        (64, 200, 20000)])
@pytest.mark.parametrize("start", ["zero", "formula"])
def test_batched_cqk_fp32_parity(ctx, nseg, lo, hi, start):
    """float32 arrays, float64 arithmetic: each row within the FP32 bar of the
    oracle run on the same (rounded) values."""
    off, inst = W.cqk_batched(nseg, lo, hi, 61 + nseg)
    inst = _round32(inst)
    x, lam, sts, info = _run(ctx, off, inst, dtype=torch.float32, lambda0=start)
    assert info["status"] == 0, info
    _check_rows(x, lam, sts, off, inst, tol=1e-5)


@pytest.mark.parametrize("nseg,lo,hi", [(1, 5, 5), (50, 1, 3000), (200, 100, 10000)])
def test_batched_cqk_fp32_vjp_parity(ctx, nseg, lo, hi):
    """The VJP on float32 arrays: x is the oracle's solution rounded to
    float32 and both sides read the free set from that same x."""
    off, inst = W.cqk_batched(nseg, lo, hi, 81 + nseg)
    inst = _round32(inst)
    res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
    x = np.concatenate([r.x for r in res]).astype(np.float32).astype(np.float64)
    g = np.random.default_rng(82).standard_normal(x.size).astype(np.float32).astype(np.float64)
    ga, gr = _vjp(ctx, off, inst, x, g, dtype=torch.float32)
    ga_ref, gr_ref = O.cqk_vjp_batched(x, g, inst["d"], inst["b"], inst["l"], inst["u"], off)
    scale = max(1.0, float(np.max(np.abs(ga_ref))), float(np.max(np.abs(gr_ref))))
    assert np.max(np.abs(ga - ga_ref)) <= 1e-5 * scale
    assert np.max(np.abs(gr - gr_ref)) <= 1e-5 * scale


def test_batched_cqk_fp32_autograd(ctx):
    import paper_2603_15910_amd as cqk
    off, inst = W.cqk_batched(30, 20, 2000, 43)
    inst = _round32(inst)
    t = [_dev(inst[k], torch.float32) for k in "dablu"]
    a = t[1].clone().requires_grad_(True)
    r = _dev(inst["r"]).requires_grad_(True)
    x = cqk.CqkBatchedSolve.apply(t[0], a, t[2], t[3], t[4], _dev(off, torch.int64), r)
    assert x.dtype == torch.float32
    (x.double() * 1.0).sum().backward()
    assert a.grad.dtype == torch.float32 and r.grad.dtype == torch.float64
    # with g = 1 the gradient w.r.t. a is [F](1 - b mu)/d and sum_F b grad_a = 0
    ga = a.grad.double().cpu().numpy()
    xs = x.detach().double().cpu().numpy()
    for s in range(off.size - 1):
        lo, hi = int(off[s]), int(off[s + 1])
        b = inst["b"][lo:hi]
        free = (xs[lo:hi] > inst["l"][lo:hi]) & (xs[lo:hi] < inst["u"][lo:hi])
        assert not np.any(ga[lo:hi][~free])
        assert abs(float(np.sum(b[free] * ga[lo:hi][free]))) <= 1e-4 * max(
            1.0, float(np.sum(np.abs(b * ga[lo:hi]))))


def test_batched_cqk_vjp_empty_free_set(ctx):
    """A row with every index at a bound has mu = 0 and zero gradients."""
    n = 300
    d = np.ones(n)
    a = np.zeros(n)
    b = np.ones(n)
    l = np.zeros(n)
    u = np.ones(n)
    x = np.where(np.arange(n) % 2 == 0, 0.0, 1.0)
    off = np.array([0, 100, 300])
    inst = {"d": d, "b": b, "l": l, "u": u}
    g = np.random.default_rng(33).standard_normal(n)
    ga, gr = _vjp(ctx, off, inst, x, g)
    assert not np.any(ga) and not np.any(gr)


def test_batched_cqk_autograd(ctx):
    import paper_2603_15910_amd as cqk
    off, inst = W.cqk_batched(30, 20, 2000, 41)
    t = [_dev(inst[k]) for k in "dablu"]
    a = t[1].clone().requires_grad_(True)
    r = _dev(inst["r"]).requires_grad_(True)
    x = cqk.CqkBatchedSolve.apply(t[0], a, t[2], t[3], t[4], _dev(off, torch.int64), r)
    g = torch.from_numpy(np.random.default_rng(42).standard_normal(x.numel())).cuda()
    (x * g).sum().backward()
    res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
    xr = np.concatenate([q.x for q in res])
    ga_ref, gr_ref = O.cqk_vjp_batched(xr, g.cpu().numpy(), inst["d"], inst["b"], inst["l"],
                                       inst["u"], off)
    scale = max(1.0, float(np.max(np.abs(ga_ref))))
    assert np.max(np.abs(a.grad.cpu().numpy() - ga_ref)) <= 1e-9 * scale
    assert np.max(np.abs(r.grad.cpu().numpy() - gr_ref)) <= 1e-9 * scale


def test_batched_cqk_argument_errors(ctx):
    import paper_2603_15910_amd as cqk
    off, inst = W.cqk_batched(4, 5, 50, 51)
    t = [_dev(inst[k]) for k in "dablu"]
    with pytest.raises(ValueError):
        ctx.solve_batched(*t, _dev(off, torch.int64), _dev(inst["r"][:3]))
    with pytest.raises(cqk.CqkError):
        ctx.solve_batched(*t, _dev(off, torch.int64), _dev(inst["r"]), lambda0="condat")
    st = cqk.cqk_solve_batched_f64(ctx.handle, 4, _dev(off, torch.int64).data_ptr(),
                                   *[v.data_ptr() for v in t], None, t[0].data_ptr())
    assert st == cqk.CQK_INVALID_ARG


def test_batched_cqk_degenerate_rows(ctx):
    """Rows the single-instance edge cases cover, side by side in one call:
    unbounded, every index with l = u, a single index, mixed infinite bounds,
    and a long unbounded row (workgroup path)."""
    rng = np.random.default_rng(61)
    rows = []

    def row(n, lo_kind, hi_kind):
        d = rng.uniform(1, 10, n)
        a = rng.uniform(-10, 10, n)
        b = rng.uniform(1, 10, n)
        l = {"inf": np.full(n, -np.inf), "fin": rng.uniform(-5, 0, n)}[lo_kind]
        u = {"inf": np.full(n, np.inf), "fin": (np.where(np.isfinite(l), l, -1.0)
                                               + rng.uniform(0.1, 5, n))}[hi_kind]
        return d, a, b, l, u

    # unbounded rows, short and long
    for n in (40, 3000):
        d, a, b, l, u = row(n, "inf", "inf")
        rows.append((d, a, b, l, u, 3.0))
    # l = u everywhere: the only feasible r is b'l
    d, a, b, l, u = row(50, "fin", "fin")
    u = l.copy()
    rows.append((d, a, b, l, u, float(np.dot(b, l))))
    # a single index, r inside its range
    d, a, b, l, u = row(1, "fin", "fin")
    rows.append((d, a, b, l, u, float(b[0] * (0.3 * l[0] + 0.7 * u[0]))))
    # lower bounds only, upper bounds only
    d, a, b, l, u = row(700, "fin", "inf")
    rows.append((d, a, b, l, u, float(np.dot(b, l)) + 50.0))
    d, a, b, l, u = row(90, "inf", "fin")
    rows.append((d, a, b, l, u, float(np.dot(b, u)) - 20.0))
    off = np.concatenate([[0], np.cumsum([r[0].size for r in rows])])
    inst = {k: np.concatenate([r[i] for r in rows]) for i, k in enumerate("dablu")}
    inst["r"] = np.array([r[5] for r in rows])
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 0, (info, sts)
    for s in range(len(rows)):
        row_ = _row(inst, off, s)
        ref = O.solve_cqk(*[row_[c] for c in "dablu"], row_["r"])
        assert ref.status == O.OK
        check_cqk(x[off[s]:off[s + 1]], row_, ref, 1e-10)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_cqk_graph_capture_replays(ctx, dtype):
    """Forward and backward captured in one HIP graph (no allocation, no host
    sync inside); every replay matches the eager results."""
    off, inst = W.cqk_batched(300, 10, 6000, 71)
    t = [_dev(inst[k], dtype) for k in "dablu"]
    offs = _dev(off, torch.int64)
    r = _dev(inst["r"])
    x = torch.empty_like(t[0])
    lam = torch.empty(300, dtype=torch.float64, device="cuda")
    g = torch.from_numpy(np.random.default_rng(72).standard_normal(x.numel())).to("cuda", dtype)
    ga = torch.empty_like(x)
    gr = torch.empty(300, dtype=torch.float64, device="cuda")
    # eager pass (sizes the workspace)
    ctx.solve_batched(*t, offs, r, out=x, lambda_out=lam)
    ctx.solve_batched_backward(x, g, t[0], t[2], t[3], t[4], offs, grad_a=ga, grad_r=gr)
    ex, el, ega, egr = x.clone(), lam.clone(), ga.clone(), gr.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ctx.solve_batched(*t, offs, r, out=x, lambda_out=lam, sync=False, check=False)
            ctx.solve_batched_backward(x, g, t[0], t[2], t[3], t[4], offs, grad_a=ga,
                                       grad_r=gr, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(4):
        for v in (x, lam, ga, gr):
            v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, ex) and torch.equal(lam, el)
        assert torch.equal(ga, ega) and torch.equal(gr, egr)


SCHEDULES = [(sp, bpc, sf) for sp in (4, 8) for bpc in (1, 2, 3, 4) for sf in (0, 1)]


@pytest.mark.parametrize("sp,bpc,sf", SCHEDULES)
def test_batched_cqk_every_schedule(ctx, sp, bpc, sf):
    """Every schedule the tuner may pick gives the oracle's solution and VJP
    (rows on both sides of the wave-row limits 256 and 512)."""
    off, inst = W.cqk_batched(60, 1, 3000, 81)
    ctx.set_batch_schedule(sp, bpc, sf, general=True)
    ctx.set_batch_schedule(sp, bpc, sf, backward=True, general=True)
    try:
        x, lam, sts, info = _run(ctx, off, inst)
        assert info["status"] == 0
        _check_rows(x, lam, sts, off, inst)
        res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
        xr = np.concatenate([q.x for q in res])
        g = np.random.default_rng(82).standard_normal(xr.size)
        ga, gr = _vjp(ctx, off, inst, xr, g)
        ga_ref, gr_ref = O.cqk_vjp_batched(xr, g, inst["d"], inst["b"], inst["l"], inst["u"], off)
        scale = max(1.0, float(np.max(np.abs(ga_ref))))
        assert np.max(np.abs(ga - ga_ref)) <= 1e-10 * scale
        assert np.max(np.abs(gr - gr_ref)) <= 1e-10 * scale
    finally:
        ctx.set_batch_schedule(8, 4, 0, general=True)
        ctx.set_batch_schedule(8, 4, 0, backward=True, general=True)


@pytest.mark.parametrize("sp,bpc,sf", SCHEDULES)
def test_batched_cqk_every_schedule_fp32(ctx, sp, bpc, sf):
    """The same on float32 arrays, to the FP32 bar; the VJP reads x rounded
    to float32 on both sides."""
    off, inst = W.cqk_batched(60, 1, 3000, 91)
    inst = _round32(inst)
    ctx.set_batch_schedule(sp, bpc, sf, general=True)
    ctx.set_batch_schedule(sp, bpc, sf, backward=True, general=True)
    try:
        x, lam, sts, info = _run(ctx, off, inst, dtype=torch.float32)
        assert info["status"] == 0
        _check_rows(x, lam, sts, off, inst, tol=1e-5)
        res = O.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
        xr = np.concatenate([q.x for q in res]).astype(np.float32).astype(np.float64)
        g = np.random.default_rng(92).standard_normal(xr.size).astype(np.float32)
        g = g.astype(np.float64)
        ga, gr = _vjp(ctx, off, inst, xr, g, dtype=torch.float32)
        ga_ref, gr_ref = O.cqk_vjp_batched(xr, g, inst["d"], inst["b"], inst["l"], inst["u"], off)
        scale = max(1.0, float(np.max(np.abs(ga_ref))), float(np.max(np.abs(gr_ref))))
        assert np.max(np.abs(ga - ga_ref)) <= 1e-5 * scale
        assert np.max(np.abs(gr - gr_ref)) <= 1e-5 * scale
    finally:
        ctx.set_batch_schedule(8, 4, 0, general=True)
        ctx.set_batch_schedule(8, 4, 0, backward=True, general=True)


def test_batched_cqk_fp32_tuner(ctx):
    """The tuner on float32 arrays times the float32 kernels and sets the
    schedules the float32 calls then use."""
    off, inst = W.cqk_batched(300, 16, 20000, 87)
    inst = _round32(inst)
    t = [_dev(inst[k], torch.float32) for k in "dablu"]
    offs = _dev(off, torch.int64)
    r = _dev(inst["r"])
    try:
        sc, ms = ctx.tune_batched_cqk(*t, offs, r, repeats=1)
        assert sc == ctx.batch_schedule(general=True) and ms > 0
        x, lam, sts, info = _run(ctx, off, inst, dtype=torch.float32)
        assert info["status"] == 0
        rng = np.random.default_rng(88)
        _check_rows(x, lam, sts, off, inst, rows=sorted(rng.choice(300, 30, replace=False)),
                    tol=1e-5)
        g = _dev(rng.standard_normal(x.size), torch.float32)
        scb, msb = ctx.tune_batched_cqk(*t, offs, r, repeats=1, backward=True,
                                        x=_dev(x, torch.float32), g=g)
        assert scb == ctx.batch_schedule(backward=True, general=True) and msb > 0
    finally:
        ctx.set_batch_schedule(8, 4, 0, general=True)
        ctx.set_batch_schedule(8, 4, 0, backward=True, general=True)


def test_batched_cqk_tuner(ctx):
    off, inst = W.cqk_batched(400, 16, 20000, 83)
    t = [_dev(inst[k]) for k in "dablu"]
    offs = _dev(off, torch.int64)
    r = _dev(inst["r"])
    sc, ms = ctx.tune_batched_cqk(*t, offs, r, repeats=1)
    assert sc == ctx.batch_schedule(general=True) and ms > 0
    assert sc["small_per"] in (4, 8) and 1 <= sc["blocks_per_cu"] <= 4
    x, lam, sts, info = _run(ctx, off, inst)
    assert info["status"] == 0
    rng = np.random.default_rng(84)
    _check_rows(x, lam, sts, off, inst, rows=sorted(rng.choice(400, 40, replace=False)))
    g = _dev(rng.standard_normal(x.size))
    scb, msb = ctx.tune_batched_cqk(*t, offs, r, repeats=1, backward=True, x=_dev(x), g=g)
    assert scb == ctx.batch_schedule(backward=True, general=True) and msb > 0
    # the simplex schedules are untouched by the general tuner
    assert ctx.batch_schedule() == ctx.batch_schedule()
    ctx.set_batch_schedule(8, 4, 0, general=True)
    ctx.set_batch_schedule(8, 4, 0, backward=True, general=True)
