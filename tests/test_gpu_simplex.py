"""GPU parity of the simplex and l1-ball projections against the CPU oracle,
through the C ABI (cqk_project_simplex_*, cqk_project_l1_*)."""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W
from tests.parity import check_simplex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {np.float32: 1e-5, np.float64: 1e-10}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_15910_amd as cqk
    c = cqk.Context(0)
    yield c
    c.close()


def _run(ctx, y, r, l1=False, **kw):
    yt = torch.from_numpy(y).cuda()
    fn = ctx.project_l1 if l1 else ctx.project_simplex
    x, info = fn(yt, r, check=False, **kw)
    return x.cpu().numpy(), info


def _ref(y, r, l1=False):
    y64 = y.astype(np.float64)
    return O.project_l1(y64, r) if l1 else O.project_simplex(y64, r)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["normal", "uniform", "normal_small"])
@pytest.mark.parametrize("start", ["condat", "zero", "formula"])
@pytest.mark.parametrize("n", [1, 2, 17, 4099, 65537, 1_000_003])
def test_simplex_parity(ctx, dtype, dist, start, n):
    y = W.simplex_input(n, 7 + n % 13, dist, dtype)
    x_ref, lam_ref = _ref(y, 1.0)
    x, info = _run(ctx, y, 1.0, lambda0=start)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype])


@pytest.mark.parametrize("dist", ["normal", "uniform"])
@pytest.mark.parametrize("accum", ["f32", "f64"])
@pytest.mark.parametrize("start", ["condat", "zero"])
def test_fp32_accumulator_variants(ctx, dist, accum, start):
    y = W.simplex_input(2_000_000, 3, dist, np.float32)
    x_ref, lam_ref = _ref(y, 1.0)
    x, info = _run(ctx, y, 1.0, lambda0=start, accum=accum)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, 1.0, 1e-5)


@pytest.mark.parametrize("compaction", ["off", "auto"])
@pytest.mark.parametrize("start", ["condat", "zero", "formula"])
def test_compaction_modes(ctx, compaction, start):
    y = W.simplex_input(300_001, 5, "normal", np.float64)
    x_ref, lam_ref = _ref(y, 1.0)
    x, info = _run(ctx, y, 1.0, lambda0=start, compaction=compaction)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, 1.0, 1e-10)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("start", ["condat", "zero", "formula"])
@pytest.mark.parametrize("radius", [0.5, 1.0, 30.0])
def test_l1_parity(ctx, dtype, start, radius):
    y = W.simplex_input(200_003, 11, "normal", dtype)
    y[::17] = 0.0
    x_ref, lam_ref = _ref(y, radius, l1=True)
    x, info = _run(ctx, y, radius, l1=True, lambda0=start)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, radius, TOL[dtype], l1=True)
    assert np.all(x[::17] == 0)
    assert np.all(np.sign(x[x != 0]) == np.sign(y[x != 0]))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_l1_inside_ball_is_identity(ctx, dtype):
    y = (W.simplex_input(10_000, 2, "normal", dtype) * 1e-5).astype(dtype)
    x, info = _run(ctx, y, 1.0, l1=True)
    assert info["status"] == 0 and info["stop_reason"] == 5
    np.testing.assert_array_equal(x, y)


def test_r_zero_and_empty(ctx):
    y = W.simplex_input(1000, 2, "normal", np.float32)
    x, info = _run(ctx, y, 0.0)
    assert info["status"] == 0 and np.all(x == 0)
    x, info = _run(ctx, y, 0.0, l1=True)
    assert info["status"] == 0 and np.all(x == 0)
    import paper_2603_15910_amd as cqk
    st = cqk.cqk_project_simplex_f32(ctx.handle, 0, None, 1.0, None)
    assert st == cqk.CQK_INFEASIBLE
    st = cqk.cqk_project_simplex_f32(ctx.handle, 0, None, 0.0, None)
    assert st == cqk.CQK_OK


def test_invalid_inputs(ctx):
    y = W.simplex_input(5000, 2, "normal", np.float32)
    y[1234] = np.nan
    for start in ("condat", "zero", "formula"):
        _, info = _run(ctx, y, 1.0, lambda0=start)
        assert info["status"] == 2, (start, info)
    y[1234] = np.inf
    _, info = _run(ctx, y, 1.0)
    assert info["status"] == 2
    import paper_2603_15910_amd as cqk
    yt = torch.zeros(16, device="cuda")
    assert cqk.cqk_project_simplex_f32(ctx.handle, 16, yt.data_ptr(), -1.0, yt.data_ptr()) == 2
    assert cqk.cqk_project_l1_f32(ctx.handle, 16, yt.data_ptr(), float("nan"), yt.data_ptr()) == 2


@pytest.mark.parametrize("dist", ["normal", "uniform"])
def test_condat_start_invariants(ctx, dist):
    """lam_0 from the GPU Algorithm 2 is an upper bound of lam* and every
    index it drops is zero at the solution (Section 2.2, eq. (lambdaJ))."""
    y = W.simplex_input(1_000_000, 4, dist, np.float64)
    x_ref, lam_ref = _ref(y, 1.0)
    x, info = _run(ctx, y, 1.0, lambda0="condat", trace=True)
    assert info["status"] == 0
    assert info["lambda0"] >= lam_ref - 1e-12
    assert info["n_after_init"] >= int(np.sum(x_ref > 0))
    # every wave region keeps at least its own sub-problem's support, about
    # sqrt(2 * region) values for uniform data: a few percent at this size
    assert info["n_after_init"] < y.size // 10


@pytest.mark.parametrize("start", ["zero", "formula", "condat"])
def test_theorem1_on_device_trace(ctx, start):
    y = W.simplex_input(500_000, 6, "normal", np.float64)
    _, lam_ref = _ref(y, 1.0)
    _, info = _run(ctx, y, 1.0, lambda0=start, trace=True)
    assert info["status"] == 0
    ev = [t for t in ctx.trace() if t["kind"] == 1]
    lams = [t["lam"] for t in ev]
    for k in range(1, len(ev)):
        assert lams[k] >= lam_ref - 1e-12
        if k + 1 < len(ev):
            assert lams[k + 1] <= lams[k]
            assert ev[k]["phi"] > 1.0


def test_deterministic_repeats(ctx):
    y = W.simplex_input(3_000_000, 8, "normal", np.float32)
    yt = torch.from_numpy(y).cuda()
    outs = []
    for _ in range(5):
        x, info = ctx.project_simplex(yt, 1.0)
        outs.append((x.cpu().numpy().tobytes(), info["lambda"]))
    assert all(o == outs[0] for o in outs)


def test_other_radius(ctx):
    y = W.simplex_input(100_000, 9, "uniform", np.float64)
    for r in (1e-3, 7.5, 5e4):
        x_ref, lam_ref = _ref(y, r)
        x, info = _run(ctx, y, r)
        assert info["status"] == 0
        check_simplex(x, y, x_ref, lam_ref, r, 1e-10)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_views(ctx, shift):
    """Arrays that start at any element offset are accepted (the kernels fall
    back to element accesses where a 16-byte access would be unaligned)."""
    y = W.simplex_input(100_003, 12, "normal", np.float32)
    base = torch.from_numpy(y).cuda()
    yv = base[shift:]
    xbuf = torch.empty(y.size, device="cuda")
    xv = xbuf[shift:]
    x_ref, lam_ref = _ref(y[shift:], 1.0)
    for start in ("condat", "zero"):
        xv.fill_(-1.0)
        _, info = ctx.project_simplex(yv, 1.0, out=xv, lambda0=start)
        assert info["status"] == 0
        check_simplex(xv.cpu().numpy(), y[shift:], x_ref, lam_ref, 1.0, 1e-5)


@pytest.mark.parametrize("dtype,n", [(np.float32, 32768), (np.float32, 32769),
                                     (np.float64, 16384), (np.float64, 16385)])
@pytest.mark.parametrize("start", ["condat", "zero"])
def test_tail_loop_capacity_boundary(ctx, dtype, n, start):
    """Sets of exactly the one-block loop's LDS capacity and one more."""
    for dist in ("uniform", "normal_small"):
        y = W.simplex_input(n, 31, dist, dtype)
        x_ref, lam_ref = _ref(y, 1.0)
        x, info = _run(ctx, y, 1.0, lambda0=start)
        assert info["status"] == 0, info
        check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_condat_start_sample_cases(ctx, dtype):
    """The Algorithm 2 start bounds lam* from a sample of tiles (one per wave,
    tile floor(w * ntiles / 1024) of 1024 values) and then filters all of y
    with it: inputs where the sample sees nothing of the support, ordered
    inputs, ties, and invalid values inside and outside the sample."""
    rng = np.random.default_rng(77)
    n = 3 * 1024 * 1024 + 517          # 3073 tiles: tile 1 is not sampled
    base = rng.standard_normal(n).astype(dtype)
    cases = {}
    spike = base.copy()
    spike[1024 + 300] = dtype(50.0)      # the whole support in an unsampled tile
    cases["spike_unsampled"] = (spike, False)
    neg = base.copy()
    neg[1024 + 301] = dtype(-60.0)       # l1: the largest |y| is negative, unsampled
    cases["l1_negative_spike"] = (neg, True)
    cases["ascending"] = (np.sort(base), False)
    cases["descending"] = (np.sort(base)[::-1].copy(), False)
    cases["ties"] = (np.full(n, 0.25, dtype=dtype), False)
    small = rng.standard_normal(6 * 1024 + 7).astype(dtype)   # fewer tiles than sample waves
    cases["six_tiles"] = (small, False)
    for name, (y, l1) in cases.items():
        x_ref, lam_ref = _ref(y, 1.0, l1)
        x, info = _run(ctx, y, 1.0, l1=l1, lambda0="condat")
        assert info["status"] == 0, (name, info)
        check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype], l1=l1)
        if not l1:
            assert info["lambda0"] >= lam_ref - 1e-9 * max(1.0, abs(lam_ref)), (name, info)
    for pos in (5, 1024 + 5):            # inside tile 0 (sampled), inside tile 1 (not)
        y = base.copy()
        y[pos] = np.nan
        _, info = _run(ctx, y, 1.0, lambda0="condat")
        assert info["status"] == 2, (pos, info)
