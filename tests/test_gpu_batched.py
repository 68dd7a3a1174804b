"""GPU parity of the batched simplex projection and its backward pass
(cqk_project_simplex_batched_f32 / _backward_f32) against the CPU oracle."""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W

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


def _rows_check(x, y, off, r, lam=None, nfree=None, tol=1e-5):
    x_ref, lam_ref = O.project_simplex_batched(y.astype(np.float64), off, r)
    rr = np.broadcast_to(np.asarray(r, dtype=np.float64), (off.size - 1,))
    for s in range(off.size - 1):
        a, b = int(off[s]), int(off[s + 1])
        if b == a:
            continue
        xs, xr, ys = x[a:b].astype(np.float64), x_ref[a:b], y[a:b].astype(np.float64)
        S = max(np.max(np.abs(xr)), np.max(np.abs(ys)), abs(lam_ref[s]))
        err = np.max(np.abs(xs - xr))
        assert err <= tol * S, (s, b - a, err, S)
        assert abs(xs.sum() - rr[s]) <= tol * (b - a) * max(np.max(np.abs(xs)), 1e-30) + 1e-30, s
        if lam is not None and rr[s] > 0:
            assert abs(lam[s] - lam_ref[s]) <= tol * S, (s, lam[s], lam_ref[s])
        if nfree is not None and rr[s] > 0:
            tie = np.abs(xr) <= 2 * tol * S
            assert abs(int(nfree[s]) - int(np.sum(xr > 0))) <= int(np.sum(tie)), s
    return x_ref


def _run(ctx, off, y, r=1.0, **kw):
    offs = torch.from_numpy(off).cuda()
    yt = torch.from_numpy(y).cuda()
    nseg = off.size - 1
    lam = torch.empty(nseg, dtype=torch.float64, device="cuda")
    nf = torch.empty(nseg, dtype=torch.int32, device="cuda")
    rt = torch.from_numpy(np.asarray(r, dtype=np.float64)).cuda() if np.ndim(r) else r
    x, info = ctx.project_simplex_batched(yt, offs, rt, lambda_out=lam, nfree_out=nf,
                                          check=False, **kw)
    return x.cpu().numpy(), lam.cpu().numpy(), nf.cpu().numpy(), info


@pytest.mark.parametrize("lo,hi,nseg", [(1, 600, 500), (64, 4096, 300), (64, 65536, 200),
                                        (4000, 140000, 20)])
def test_batched_parity(ctx, lo, hi, nseg):
    off, y = W.batched_simplex_input(nseg, lo, hi, 5 + nseg)
    x, lam, nf, info = _run(ctx, off, y)
    assert info["status"] == 0, info
    _rows_check(x, y, off, 1.0, lam, nf)


def test_ragged_edges_and_radii(ctx):
    lens = [0, 1, 2, 3, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 8191, 70000, 1, 0, 7]
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    y = W.simplex_input(int(off[-1]), 3, "normal", np.float32)
    r = np.linspace(0.5, 20.0, len(lens))
    r[0] = r[-2] = 0.0  # empty rows need r = 0 to be feasible
    x, lam, nf, info = _run(ctx, off, y, r)
    assert info["status"] == 0, info
    _rows_check(x, y, off, r, lam, nf)


def test_uniform_rows_and_spill_path(ctx):
    # near-constant rows keep almost every value after Algorithm 2, so the
    # survivors do not fit on chip and Newton re-reads the row
    lens = [70000, 30000, 9000, 600]
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    rng = np.random.default_rng(4)
    y = (1.0 + 1e-3 * rng.random(int(off[-1]))).astype(np.float32)
    x, lam, nf, info = _run(ctx, off, y, 1.0)
    assert info["status"] == 0, info
    assert info["rows_spilled"] >= 1
    _rows_check(x, y, off, 1.0, lam, nf)
    off2, y2 = W.batched_simplex_input(100, 64, 65536, 9)
    y2 = np.abs(y2) / 3.0  # uniform-like positive rows
    x2, lam2, nf2, info2 = _run(ctx, off2, y2.astype(np.float32), 1.0)
    assert info2["status"] == 0
    _rows_check(x2, y2.astype(np.float32), off2, 1.0, lam2, nf2)


def test_batched_errors(ctx):
    off = np.array([0, 10, 20, 20], dtype=np.int64)
    y = W.simplex_input(20, 3, "normal", np.float32)
    _, lam, _, info = _run(ctx, off, y, np.array([1.0, -1.0, 0.0]))
    assert info["status"] == 2 and np.isnan(lam[1])
    _, _, _, info = _run(ctx, off, y, 1.0)          # empty row with r = 1
    assert info["status"] == 1
    y[3] = np.nan
    _, _, _, info = _run(ctx, off, y, np.array([1.0, 1.0, 0.0]))
    assert info["status"] == 2


def test_c4_full_workload(ctx):
    off, y = W.batched_simplex_input(8192, 64, 65536, 1)
    x, lam, nf, info = _run(ctx, off, y)
    assert info["status"] == 0
    _rows_check(x, y, off, 1.0, lam, nf)


def test_deterministic_and_per_row_loop_agree(ctx):
    off, y = W.batched_simplex_input(64, 64, 20000, 2)
    x1, lam1, _, _ = _run(ctx, off, y)
    x2, lam2, _, _ = _run(ctx, off, y)
    assert np.array_equal(x1, x2) and np.array_equal(lam1, lam2)
    yt = torch.from_numpy(y).cuda()
    for s in range(0, 64, 7):
        a, b = int(off[s]), int(off[s + 1])
        xs, _ = ctx.project_simplex(yt[a:b].clone(), 1.0)
        assert np.max(np.abs(xs.cpu().numpy() - x1[a:b])) <= 1e-5 * max(1.0, np.abs(y[a:b]).max())


def _grad_check(ctx, off, y, g, x):
    offs = torch.from_numpy(off).cuda()
    nseg = off.size - 1
    gr = torch.empty(nseg, dtype=torch.float64, device="cuda")
    gy = ctx.project_simplex_batched_backward(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(),
                                              offs, grad_r=gr)
    gy = gy.cpu().numpy()
    gr = gr.cpu().numpy()
    ga_ref, gr_ref = O.simplex_vjp_batched(x.astype(np.float64), g.astype(np.float64), off)
    gmax = max(1.0, float(np.max(np.abs(g))))
    assert np.max(np.abs(gy - ga_ref)) <= 1e-5 * gmax
    assert np.max(np.abs(gr - gr_ref)) <= 1e-5 * gmax
    return gy, gr


def test_backward_parity_c5_shape(ctx):
    off, y = W.batched_simplex_input(4096, 1024, 32768, 1, scale=3.0)
    g = W.upstream_grad(y.size, 1)
    x, _, _, info = _run(ctx, off, y)
    assert info["status"] == 0
    _grad_check(ctx, off, y, g, x)


def test_backward_against_fp64_finite_differences(ctx):
    """The oracle VJP is pinned by FP64 central differences on sampled rows
    with a margin from the support boundary; the GPU gradient matches it."""
    off, y = W.batched_simplex_input(64, 16, 400, 3, scale=3.0)
    g = W.upstream_grad(y.size, 3)
    x, _, _, _ = _run(ctx, off, y)
    gy, gr = _grad_check(ctx, off, y, g, x)
    rng = np.random.default_rng(0)
    rows = rng.choice(64, 32, replace=False)
    h = 1e-6
    checked = 0
    for s in rows:
        a, b = int(off[s]), int(off[s + 1])
        ys = y[a:b].astype(np.float64)
        gs = g[a:b].astype(np.float64)
        _, lam = O.project_simplex(ys, 1.0)
        if np.min(np.abs(ys + lam)) < 1e-4:
            continue
        for i in range(b - a):
            e = np.zeros(b - a); e[i] = h
            fd = (gs @ O.project_simplex(ys + e, 1.0)[0] - gs @ O.project_simplex(ys - e, 1.0)[0]) / (2 * h)
            assert abs(gy[a + i] - fd) <= 1e-5 * max(1, np.abs(gs).max())
        checked += 1
    assert checked >= 16


def test_c5_rows_against_fp64_finite_differences(ctx):
    """FD check on 32 rows sampled from the C5 workload itself (4096 rows of
    1024-32768 values, y = 3 N(0,1), g ~ N(0,1)): on each row a subset of
    coordinates (support and non-support) is perturbed by +-1e-6 in FP64
    through the oracle's projection, and the central difference of g.x is
    compared with the GPU gradient.  Rows whose support has a margin below
    1e-4 are skipped (the VJP is a one-sided derivative there)."""
    off, y = W.batched_simplex_input(4096, 1024, 32768, 1, scale=3.0)
    g = W.upstream_grad(y.size, 1)
    x, _, _, info = _run(ctx, off, y)
    assert info["status"] == 0
    gy, gr = _grad_check(ctx, off, y, g, x)
    rng = np.random.default_rng(5)
    h = 1e-6
    checked = skipped = 0
    for s in rng.permutation(4096):
        if checked == 32:
            break
        a, b = int(off[s]), int(off[s + 1])
        ys = y[a:b].astype(np.float64)
        gs = g[a:b].astype(np.float64)
        xs, lam = O.project_simplex(ys, 1.0)
        if np.min(np.abs(ys + lam)) < 1e-4:
            skipped += 1
            continue
        supp = np.flatnonzero(xs > 0)
        rest = np.flatnonzero(xs == 0)
        coords = np.concatenate([rng.choice(supp, min(8, supp.size), replace=False),
                                 rng.choice(rest, min(8, rest.size), replace=False)])
        for i in coords:
            yp = ys.copy(); yp[i] += h
            ym = ys.copy(); ym[i] -= h
            fd = (gs @ O.project_simplex(yp, 1.0)[0] - gs @ O.project_simplex(ym, 1.0)[0]) / (2 * h)
            assert abs(gy[a + i] - fd) <= 1e-5 * max(1, np.abs(gs).max()), (s, i)
        # d(g.x)/dr by the same central difference
        fdr = (gs @ O.project_simplex(ys, 1.0 + h)[0] - gs @ O.project_simplex(ys, 1.0 - h)[0]) / (2 * h)
        assert abs(gr[s] - fdr) <= 1e-5 * max(1, np.abs(gs).max()), s
        checked += 1
    assert checked == 32, (checked, skipped)


def test_autograd_function(ctx):
    import paper_2603_15910_amd as cqk
    off, y = W.batched_simplex_input(50, 32, 3000, 4, scale=3.0)
    offs = torch.from_numpy(off).cuda()
    yt = torch.from_numpy(y).cuda().requires_grad_(True)
    rt = torch.full((50,), 1.0, dtype=torch.float64, device="cuda", requires_grad=False)
    xt = cqk.SimplexProjection.apply(yt, offs, rt)
    g = torch.from_numpy(W.upstream_grad(y.size, 4)).cuda()
    (xt * g).sum().backward()
    ga_ref, _ = O.simplex_vjp_batched(xt.detach().cpu().numpy().astype(np.float64),
                                      g.cpu().numpy().astype(np.float64), off)
    assert np.max(np.abs(yt.grad.cpu().numpy() - ga_ref)) <= 1e-5 * max(1, g.abs().max().item())


def test_graph_capture_replays(ctx):
    """The batched forward is captured in a HIP graph (no allocation, no host
    sync inside) and every replay matches the eager result."""
    off, y = W.batched_simplex_input(256, 64, 20000, 6)
    offs = torch.from_numpy(off).cuda()
    yt = torch.from_numpy(y).cuda()
    x = torch.empty_like(yt)
    ctx.project_simplex_batched(yt, offs, 1.0, out=x)   # sizes the workspace
    eager = x.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ctx.project_simplex_batched(yt, offs, 1.0, out=x, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(4):
        x.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, eager)


SCHEDULES = [(sp, bpc, sf) for sp in (4, 8) for bpc in (1, 2, 3, 4) for sf in (0, 1)]


@pytest.mark.parametrize("sp,bpc,sf", SCHEDULES)
def test_every_schedule_matches_oracle(ctx, sp, bpc, sf):
    """Each schedule the tuner may pick gives oracle-matching rows, forward
    and backward, including lengths at the wave/workgroup boundary."""
    lens = [1, 63, 64, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 4097, 20000, 65536, 3]
    rng = np.random.default_rng(sp * 100 + bpc * 10 + sf)
    lens += list(rng.integers(1, 3000, 40))
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    y = (3.0 * W.simplex_input(int(off[-1]), 21, "normal", np.float32)).astype(np.float32)
    ctx.set_batch_schedule(sp, bpc, sf)
    ctx.set_batch_schedule(sp, bpc, sf, backward=True)
    try:
        x, lam, nf, info = _run(ctx, off, y)
        assert info["status"] == 0, info
        _rows_check(x, y, off, 1.0, lam, nf)
        g = W.upstream_grad(y.size, 21)
        _grad_check(ctx, off, y, g, x)
    finally:
        ctx.set_batch_schedule(8, 4, 1, medium_tiles=16)
        ctx.set_batch_schedule(8, 4, 0, backward=True)


MEDIUM = [(sp, bpc, mt) for sp in (4, 8) for bpc in (2, 4) for mt in (1, 2, 4, 16, 64)]


@pytest.mark.parametrize("sp,bpc,mt", MEDIUM)
def test_medium_rows_match_oracle(ctx, sp, bpc, mt):
    """Rows between the register limit (64 * small_per) and 1024 * medium_tiles
    values are solved by one wave each, tile after tile; lengths on both
    sides of both limits and of tile ends, one NaN row, one invalid radius,
    against the oracle (forward) and the closed-form VJP (backward)."""
    import paper_2603_15910_amd as cqk
    lim = 1024 * mt
    lens = [1, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049,
            lim - 1, lim, lim + 1, 3 * 1024 + 5, 4097, 20000, 65536, 3]
    rng = np.random.default_rng(sp * 1000 + bpc * 100 + mt)
    lens += list(rng.integers(1, 3 * lim + 2, 40))
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    y = (3.0 * W.simplex_input(int(off[-1]), 22, "normal", np.float32)).astype(np.float32)
    ctx.set_batch_schedule(sp, bpc, 0, medium_tiles=mt)
    ctx.set_batch_schedule(sp, bpc, 0, backward=True, medium_tiles=mt)
    try:
        x, lam, nf, info = _run(ctx, off, y)
        assert info["status"] == 0, info
        _rows_check(x, y, off, 1.0, lam, nf)
        g = W.upstream_grad(y.size, 22)
        _grad_check(ctx, off, y, g, x)
        # a NaN in one medium row and a negative radius on another: those rows
        # are reported, every other row is still solved
        med = [s for s in range(len(lens)) if 64 * sp < lens[s] <= lim]
        if len(med) >= 2:
            yb = y.copy()
            yb[int(off[med[0]]) + 1] = np.nan
            rr = np.ones(len(lens))
            rr[med[1]] = -1.0
            offs = torch.from_numpy(off).cuda()
            xt, info = ctx.project_simplex_batched(torch.from_numpy(yb).cuda(), offs,
                                                   torch.from_numpy(rr).cuda(), check=False)
            assert info["status"] == cqk.CQK_INVALID_ARG
            xb = xt.cpu().numpy()
            for s in med[:2]:
                assert np.all(xb[int(off[s]):int(off[s + 1])] == 0.0)
            keep = [s for s in range(len(lens)) if s not in med[:2]]
            xr, _ = O.project_simplex_batched(y, off, 1.0)
            for s in keep:
                a, b = int(off[s]), int(off[s + 1])
                assert np.max(np.abs(xb[a:b] - xr[a:b]), initial=0.0) <= \
                    1e-5 * max(1.0, float(np.abs(y[a:b]).max(initial=0.0)))
    finally:
        ctx.set_batch_schedule(8, 4, 1, medium_tiles=16)
        ctx.set_batch_schedule(8, 4, 0, backward=True)


def test_schedule_argument_errors(ctx):
    import paper_2603_15910_amd as cqk
    for bad in ((5, 4, 0), (8, 0, 0), (8, 9, 0), (8, 4, 2), (8, 4, 0, False, False, -1),
                (8, 4, 0, False, False, 65)):
        with pytest.raises(cqk.CqkError):
            ctx.set_batch_schedule(*bad)
    assert ctx.batch_schedule() == {"small_per": 8, "blocks_per_cu": 4, "short_first": 1,
                                    "medium_tiles": 16}


def test_tuner_keeps_the_fastest_schedule(ctx):
    off, y = W.batched_simplex_input(1024, 64, 65536, 7)
    offs = torch.from_numpy(off).cuda()
    yt = torch.from_numpy(y).cuda()
    try:
        sched, ms = ctx.tune_batched(yt, offs, 1.0, repeats=2)
        assert ms > 0
        assert sched["small_per"] in (4, 8) and sched["blocks_per_cu"] in (2, 3, 4, 6)
        assert sched["short_first"] in (0, 1) and sched["medium_tiles"] in (0, 4, 8, 16, 32, 64)
        assert ctx.batch_schedule() == sched
        x, lam, nf, info = _run(ctx, off, y)
        assert info["status"] == 0
        _rows_check(x, y, off, 1.0, lam, nf)
        g = W.upstream_grad(y.size, 7)
        xt = torch.from_numpy(x).cuda()
        gt = torch.from_numpy(g).cuda()
        bsched, bms = ctx.tune_batched_backward(xt, gt, offs, repeats=2)
        assert bms > 0 and ctx.batch_schedule(backward=True) == bsched
        _grad_check(ctx, off, y, g, x)
    finally:
        ctx.set_batch_schedule(8, 4, 1, medium_tiles=16)
        ctx.set_batch_schedule(8, 4, 0, backward=True)
