"""cqk_project_simplex_batched_noalloc_f32 on the GPU, through the C ABI.

The no-allocation variant runs the kernels of cqk_project_simplex_batched_f32
on a fixed per-GPU array instead of the context's workspace, so on the same
rows it must give the same x, multipliers and free counts bit for bit, and
both must match the oracle (row-wise sort solution of the simplex
projection, Sec. 1; FP32 tolerance 1e-5 relative).  Checked on two calls in
a row, the second on fewer and shorter rows (the array keeps the first
call's contents), on a graph captured by a context that never reserved a
workspace, and on the row limit, which is refused before anything runs.
"""

import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cqk():
    import paper_2603_15910_amd as cqk
    return cqk


def _inputs(nseg, lo, hi, seed):
    off, y = W.batched_simplex_input(nseg, lo, hi, seed)
    return off, y, torch.from_numpy(off).cuda(), torch.from_numpy(y).cuda()


def _run(cqk, ctx, offs, yt, noalloc):
    nseg = offs.numel() - 1
    x = torch.full_like(yt, float("nan"))
    lam = torch.full((nseg,), float("nan"), dtype=torch.float64, device="cuda")
    nf = torch.full((nseg,), -1, dtype=torch.int32, device="cuda")
    rt = torch.ones(nseg, dtype=torch.float64, device="cuda")
    info = cqk.cqk_info()
    fn = (cqk.cqk_project_simplex_batched_noalloc_f32 if noalloc
          else cqk.cqk_project_simplex_batched_f32)
    ctx._bind_stream()
    st = fn(ctx.handle, nseg, offs.data_ptr(), yt.data_ptr(), rt.data_ptr(), 0.0, x.data_ptr(),
            lam.data_ptr(), nf.data_ptr(), None, info)
    torch.cuda.synchronize()
    assert st == cqk.CQK_OK and info.status == cqk.CQK_OK, (st, info.as_dict())
    return x.cpu().numpy(), lam.cpu().numpy(), nf.cpu().numpy()


def _check_oracle(x, lam, nf, off, y):
    xr, lr = O.project_simplex_batched(y, off, 1.0)
    scale = max(1.0, float(np.abs(y).max()))
    assert np.max(np.abs(x.astype(np.float64) - xr)) <= 1e-5 * scale
    assert np.max(np.abs(lam - lr)) <= 1e-5 * scale
    tie = np.abs(xr) <= 2e-5 * scale
    for s in range(off.size - 1):
        lo, hi = int(off[s]), int(off[s + 1])
        sup = xr[lo:hi] > 0
        t = tie[lo:hi]
        assert int(nf[s]) >= int(np.sum(sup & ~t)) and int(nf[s]) <= int(np.sum(sup | t)), s


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = _cqk().Context(0)
    yield c
    c.close()


def test_two_calls_match_the_allocating_call(ctx):
    cqk = _cqk()
    # first call: many rows, wave rows and workgroup rows; second: fewer and
    # shorter rows, so stale list entries and counts of the first call sit
    # past the second call's rows in the shared array
    for nseg, lo, hi, seed in ((3000, 16, 20000, 41), (700, 1, 3000, 42)):
        print(f"noalloc parity nseg={nseg} lengths [{lo},{hi}] seed={seed}", flush=True)
        off, y, offs, yt = _inputs(nseg, lo, hi, seed)
        xa, la, na = _run(cqk, ctx, offs, yt, noalloc=False)
        xn, ln, nn = _run(cqk, ctx, offs, yt, noalloc=True)
        assert np.array_equal(xn.view(np.uint32), xa.view(np.uint32))
        assert np.array_equal(ln.view(np.uint64), la.view(np.uint64))
        assert np.array_equal(nn, na)
        _check_oracle(xn, ln, nn, off, y)


def test_row_limit_refused_before_launch(ctx):
    cqk = _cqk()
    nseg = cqk.CQK_NOALLOC_MAX_SEG + 1
    offs = torch.arange(nseg + 1, dtype=torch.int64, device="cuda")
    yt = torch.ones(nseg, dtype=torch.float32, device="cuda")
    x = torch.full_like(yt, 7.0)
    info = cqk.cqk_info()
    ctx._bind_stream()
    st = cqk.cqk_project_simplex_batched_noalloc_f32(ctx.handle, nseg, offs.data_ptr(),
                                                     yt.data_ptr(), None, 1.0, x.data_ptr(),
                                                     None, None, None, info)
    torch.cuda.synchronize()
    assert st == cqk.CQK_BUFFER_TOO_SMALL and info.status == cqk.CQK_BUFFER_TOO_SMALL
    assert bool(torch.all(x == 7.0))
    # the limit itself is accepted: one value per row, each projected to 1
    offs = offs[: cqk.CQK_NOALLOC_MAX_SEG + 1].contiguous()
    yt2 = yt[: cqk.CQK_NOALLOC_MAX_SEG].contiguous()
    x2, info = ctx.project_simplex_batched(yt2, offs, 1.0, noalloc=True)
    assert info["status"] == cqk.CQK_OK
    assert bool(torch.all(x2 == 1.0))


def test_captured_without_reserve(ctx):
    """A fresh context (no workspace) captures the no-allocation call; every
    replay matches the eager allocating call, with eager work in between."""
    cqk = _cqk()
    off, y, offs, yt = _inputs(512, 16, 20000, 43)
    nseg = off.size - 1
    xa, la, _ = _run(cqk, ctx, offs, yt, noalloc=False)
    c = cqk.Context(0)
    try:
        x = torch.empty_like(yt)
        lam = torch.empty(nseg, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                _, info = c.project_simplex_batched(yt, offs, 1.0, out=x, lambda_out=lam,
                                                    check=False, sync=False, noalloc=True)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        assert info["status"] == cqk.CQK_OK
        for rep in range(3):
            x.fill_(float("nan"))
            lam.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            st, _ = c.ctx_last_info()
            assert st == cqk.CQK_OK
            assert np.array_equal(x.cpu().numpy().view(np.uint32), xa.view(np.uint32)), rep
            assert np.array_equal(lam.cpu().numpy().view(np.uint64), la.view(np.uint64)), rep
            # eager work on the same GPU between replays, allocating call included
            _run(cqk, ctx, offs, yt, noalloc=False)
        del graph
    finally:
        c.close()
