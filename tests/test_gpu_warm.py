"""GPU parity of the warm starts from a primal estimate xbar (general CQK:
Section 2.1, eq. (CQKlambda0) over the estimate's free set; simplex and l1:
Section 3.1, Algorithm 2 over the estimate's support) against the CPU oracle,
through the C ABI (cqk_solve_warm_*, cqk_project_simplex_warm_*,
cqk_project_l1_warm_*).

Checked for every case: the solution to the parity bar of the cold calls, and
lambda_0 itself --
  * general: equal to the oracle's warm lambda_0 for the same xbar (both sum
    in FP64; the tolerance is 1e-10 of the magnitudes summed);
  * simplex / l1: an upper bound of lam* (what Algorithm 2 guarantees over any
    index set), equal to lam* when xbar is the solution itself, and equal to
    the oracle's fallback max{r/n, -max v} when no index of the support is
    used.
The estimates are oracle solutions (of the same or of a perturbed problem),
fixed patterns, or seeded noise: none comes from the GPU path."""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W
from tests.parity import check_cqk, check_simplex

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


def _dev(v, dtype):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


def _solve(ctx, inst, xbar, dtype=torch.float64, **kw):
    t = [_dev(inst[k], dtype) for k in "dablu"]
    xb = _dev(xbar, dtype) if xbar is not None else None
    x, info = ctx.solve(*t, inst["r"], check=False, xbar=xb, **kw)
    return x.cpu().numpy().astype(np.float64), info


def _lam0_scale(inst, xbar):
    """Magnitudes summed by the warm lambda_0, divided by its denominator."""
    d, a, b, l, u, xb = (np.asarray(v, dtype=np.float64)
                         for v in (inst["d"], inst["a"], inst["b"], inst["l"], inst["u"], xbar))
    free = (xb > l) & (xb < u)
    if not free.any():
        free = np.ones_like(free)
        fixed = 0.0
    else:
        fixed = float(np.sum(np.abs(b[~free & (xb <= l)] * l[~free & (xb <= l)]))
                      + np.sum(np.abs(b[~free & (xb >= u)] * u[~free & (xb >= u)])))
    num = abs(inst["r"]) + fixed + float(np.sum(np.abs(b[free] * a[free] / d[free])))
    return num / float(np.sum(b[free] ** 2 / d[free]))


def _ref(inst):
    return O.solve_cqk(*[np.asarray(inst[k], dtype=np.float64) for k in "dablu"], inst["r"])


def _check_general(ctx, inst, xbar, dtype=torch.float64, tol=1e-10):
    ref = _ref(inst)
    x, info = _solve(ctx, inst, xbar, dtype)
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, tol)
    lam0_ref = O.cqk_lambda0_warm(*[np.asarray(inst[k], dtype=np.float64) for k in "dablu"],
                                  inst["r"], np.asarray(xbar, dtype=np.float64))
    assert abs(info["lambda0"] - lam0_ref) <= 1e-10 * _lam0_scale(inst, xbar), \
        (info["lambda0"], lam0_ref)
    return ref, info


# ---------------------------------------------------------------------------
# general CQK
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gen", ["uniform", "correlated", "paper_weak"])
@pytest.mark.parametrize("n", [1, 7, 4099, 65537, 300_001])
def test_general_warm_from_solution(ctx, gen, n):
    """xbar = x*: the warm lambda_0 is lam* (its free set and bounds are the
    solution's), so Newton stops at once."""
    inst = {"uniform": W.cqk_uniform, "correlated": W.cqk_correlated,
            "paper_weak": lambda n_, s: W.cqk_paper(n_, s, "weak")}[gen](n, 11)
    ref0 = _ref(inst)
    ref, info = _check_general(ctx, inst, ref0.x)
    if np.isfinite(ref.lam) and np.any((ref.x > inst["l"]) & (ref.x < inst["u"])):
        S = _lam0_scale(inst, ref0.x)
        assert abs(info["lambda0"] - ref.lam) <= 1e-9 * S
        assert info["iterations"] <= 2, info


@pytest.mark.parametrize("n", [4099, 1_000_003])
@pytest.mark.parametrize("eps", [1e-4, 1e-2])
def test_general_warm_from_previous_problem(ctx, n, eps):
    """The outer-loop use: xbar = the solution of the previous point, the
    problem moved a little (a perturbed)."""
    prev = W.cqk_uniform(n, 5)
    xbar = _ref(prev).x
    inst = W.cqk_perturbed(prev, 6, eps)
    _, info_w = _check_general(ctx, inst, xbar)
    _, info_c = _solve(ctx, inst, None)
    assert info_c["status"] == 0
    assert info_w["iterations"] <= info_c["iterations"], (info_w, info_c)


def test_general_warm_empty_free_set_falls_back(ctx):
    """No index strictly inside its bounds in xbar: xbar is discarded and
    lambda_0 is eq. (CQKlambda0) over all indices."""
    inst = W.cqk_uniform(70_001, 8)
    for xbar in (inst["l"].copy(), inst["u"].copy(), inst["l"] - 1.0,
                 np.where(np.arange(70_001) % 2 == 0, inst["l"], inst["u"])):
        _, info = _check_general(ctx, inst, xbar)
        lam0 = O.cqk_lambda0(*[inst[k] for k in "dablu"], inst["r"])
        assert abs(info["lambda0"] - lam0) <= 1e-10 * _lam0_scale(inst, xbar)


def test_general_warm_mixed_and_nan_estimate(ctx):
    """Entries beyond their bounds count as fixed at the bound they pass; a
    NaN entry counts nowhere."""
    n = 50_001
    inst = W.cqk_correlated(n, 9)
    g = np.random.default_rng(12)
    l, u = inst["l"], inst["u"]
    xbar = l + g.uniform(-0.5, 1.5, n) * (u - l)   # below, inside and above
    xbar[g.choice(n, 100, replace=False)] = np.nan
    _check_general(ctx, inst, xbar)


def test_general_warm_fp32(ctx):
    n = 200_003
    inst = W.cqk_uniform(n, 13, dtype=np.float32)
    ref = _ref(inst)
    xbar = ref.x.astype(np.float32)
    _check_general(ctx, inst, xbar, dtype=torch.float32, tol=1e-5)


def test_general_warm_ignores_lambda0_option(ctx):
    inst = W.cqk_uniform(10_007, 14)
    xbar = np.clip(inst["a"] / inst["d"], inst["l"], inst["u"])
    _, a = _solve(ctx, inst, xbar, lambda0="formula")
    _, b = _solve(ctx, inst, xbar, lambda0="user", lambda0_user=123.0)
    assert a["lambda0"] == b["lambda0"]
    lam0_ref = O.cqk_lambda0_warm(*[inst[k] for k in "dablu"], inst["r"], xbar)
    assert abs(a["lambda0"] - lam0_ref) <= 1e-10 * _lam0_scale(inst, xbar)


def test_general_warm_argument_errors(ctx):
    import paper_2603_15910_amd as cqk
    inst = W.cqk_uniform(1000, 15)
    t = [_dev(inst[k], torch.float64) for k in "dablu"]
    x = torch.empty_like(t[0])
    with pytest.raises(cqk.CqkError):   # xbar is the output
        ctx.solve(*t, inst["r"], out=x, xbar=x)
    with pytest.raises(cqk.CqkError):   # overlapping by one element
        big = torch.zeros(1001, dtype=torch.float64, device="cuda")
        ctx.solve(*t, inst["r"], out=big[1:], xbar=big[:1000])
    with pytest.raises(ValueError):
        ctx.solve(*t, inst["r"], xbar=torch.zeros(999, dtype=torch.float64, device="cuda"))
    # a null estimate through the C entry point
    info = cqk.cqk_info()
    st = cqk.cqk_solve_warm_f64(ctx.handle, 1000, *[v.data_ptr() for v in t], None,
                                inst["r"], x.data_ptr(), None, info)
    assert st == cqk.CQK_INVALID_ARG


# ---------------------------------------------------------------------------
# simplex and l1
# ---------------------------------------------------------------------------
def _proj(ctx, y, xbar, r, l1=False, **kw):
    dt = torch.float64 if y.dtype == np.float64 else torch.float32
    yt = _dev(y, dt)
    xb = _dev(np.asarray(xbar, dtype=y.dtype), dt) if xbar is not None else None
    fn = ctx.project_l1 if l1 else ctx.project_simplex
    x, info = fn(yt, r, check=False, xbar=xb, **kw)
    return x.cpu().numpy(), info


def _sref(y, r, l1=False):
    y64 = y.astype(np.float64)
    return O.project_l1(y64, r) if l1 else O.project_simplex(y64, r)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["normal", "uniform", "normal_small"])
@pytest.mark.parametrize("n", [1, 2, 17, 4099, 65537, 1_000_003])
def test_simplex_warm_from_solution(ctx, dtype, dist, n):
    y = W.simplex_input(n, 21 + n % 7, dist, dtype)
    x_ref, lam_ref = _sref(y, 1.0)
    x, info = _proj(ctx, y, x_ref, 1.0)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype])
    S = max(float(np.max(np.abs(y))), abs(lam_ref), 1.0)
    # the support of x* read back in this dtype is still the support
    if np.all((x_ref > 0) == (x_ref.astype(dtype) > 0)):
        assert abs(info["lambda0"] - lam_ref) <= 1e-9 * S * (1 if dtype == np.float64 else 1e3)
    assert info["lambda0"] >= lam_ref - 1e-12 * S


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [4099, 1_000_003])
@pytest.mark.parametrize("eps", [1e-3, 1e-1])
def test_simplex_warm_from_previous_point(ctx, dtype, n, eps):
    y0 = W.simplex_input(n, 31, "normal", dtype)
    xbar, _ = _sref(y0, 1.0)
    y = W.perturbed(y0, 32, eps)
    x_ref, lam_ref = _sref(y, 1.0)
    x, info = _proj(ctx, y, xbar, 1.0)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype])
    assert info["lambda0"] >= lam_ref - 1e-12 * max(1.0, abs(lam_ref))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [3, 5000, 300_001])
def test_simplex_warm_random_support(ctx, dtype, n):
    """Any support gives an upper bound (Algorithm 2 over any index set); the
    values outside it stay in the problem unless the bound fixes them."""
    y = W.simplex_input(n, 41, "normal", dtype)
    g = np.random.default_rng(42)
    for frac in (0.001, 0.3, 1.0):
        xbar = (g.uniform(size=n) < frac).astype(dtype)
        x_ref, lam_ref = _sref(y, 1.0)
        x, info = _proj(ctx, y, xbar, 1.0)
        assert info["status"] == 0, info
        check_simplex(x, y, x_ref, lam_ref, 1.0, TOL[dtype])
        if xbar.any():
            assert info["lambda0"] >= lam_ref - 1e-12 * max(1.0, abs(lam_ref))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 17, 100_003])
def test_simplex_warm_fallback(ctx, dtype, n):
    """Empty support: lambda_0 = max{r/n, -max y}, then Newton as usual."""
    y = W.simplex_input(n, 51, "normal", dtype)
    for r in (1.0, 3.5):
        x_ref, lam_ref = _sref(y, r)
        x, info = _proj(ctx, y, np.zeros(n), r)
        assert info["status"] == 0, info
        check_simplex(x, y, x_ref, lam_ref, r, TOL[dtype])
        lam0, J = O.simplex_lambda0_warm(y.astype(np.float64), r, np.zeros(n))
        assert J == []
        assert info["lambda0"] == lam0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [17, 4099, 1_000_003])
def test_l1_warm(ctx, dtype, n):
    y = W.simplex_input(n, 61, "normal", dtype)
    radius = 0.05 * float(np.sum(np.abs(y.astype(np.float64))))
    x_ref, lam_ref = _sref(y, radius, l1=True)
    # the solution, a previous point's solution, and a random sign pattern
    y_prev = W.perturbed(y, 62, 1e-2)
    xp, _ = _sref(y_prev, radius, l1=True)
    g = np.random.default_rng(63)
    for xbar in (x_ref, xp, np.where(g.uniform(size=n) < 0.2, -1.0, 0.0)):
        x, info = _proj(ctx, y, xbar, radius, l1=True)
        assert info["status"] == 0, info
        check_simplex(x, y, x_ref, lam_ref, radius, TOL[dtype], l1=True)
        S = max(float(np.max(np.abs(y))), abs(lam_ref), 1.0)
        assert info["lambda0"] >= lam_ref - 1e-12 * S


def test_l1_warm_support_of_zero_values(ctx):
    """l1: a support that holds only y_i = 0.  Algorithm 2 starts from one of
    them (lam = r - 0) and no other joins (|y_j| = 0 fails the test), so
    lambda_0 = r: not the fallback, which is for an empty support."""
    n = 20_001
    y = W.simplex_input(n, 71, "normal", np.float64)
    zero = np.arange(0, n, 97)
    y[zero] = 0.0
    xbar = np.zeros(n)
    xbar[zero] = 1.0
    radius = 10.0
    x_ref, lam_ref = _sref(y, radius, l1=True)
    x, info = _proj(ctx, y, xbar, radius, l1=True)
    assert info["status"] == 0, info
    check_simplex(x, y, x_ref, lam_ref, radius, 1e-10, l1=True)
    lam0, J = O.simplex_lambda0_warm(y, radius, xbar, l1=True)
    assert len(J) == 1 and y[J[0]] == 0.0 and lam0 == radius
    # the estimate's bound (first trace record); lambda_0 is at most that,
    # and at least lam*
    _, info = _proj(ctx, y, xbar, radius, l1=True, trace=True)
    tr = [t for t in ctx.trace() if t["kind"] != 7]   # 7: one thread's Algorithm 2
    assert tr[0]["kind"] == 0 and tr[0]["phi"] == lam0   # the estimate's own bound
    assert lam_ref - 1e-12 * radius <= info["lambda0"] <= lam0


def test_l1_warm_inside_ball(ctx):
    y = W.simplex_input(5000, 81, "normal", np.float32)
    radius = 2.0 * float(np.sum(np.abs(y.astype(np.float64))))
    x, info = _proj(ctx, y, y, radius, l1=True)
    assert info["status"] == 0
    assert np.array_equal(x, y)


def test_simplex_warm_r_zero_and_errors(ctx):
    import paper_2603_15910_amd as cqk
    y = W.simplex_input(1000, 91, "normal", np.float64)
    x, info = _proj(ctx, y, np.ones(1000), 0.0)
    assert info["status"] == 0 and not np.any(x)
    yt = _dev(y, torch.float64)
    out = torch.empty_like(yt)
    with pytest.raises(cqk.CqkError):
        ctx.project_simplex(yt, 1.0, out=out, xbar=out)
    with pytest.raises(cqk.CqkError):
        ctx.project_l1(yt, 1.0, out=out, xbar=out)
    # a non-finite y is still found on the device
    y[5] = np.inf
    _, info = _proj(ctx, y, np.ones(1000), 1.0)
    assert info["status"] == cqk.CQK_INVALID_ARG


def test_simplex_warm_deterministic(ctx):
    y = W.simplex_input(2_000_003, 95, "normal", np.float32)
    xbar = W.perturbed(y, 96, 1.0) > 2.0
    a, ia = _proj(ctx, y, xbar, 1.0)
    b, ib = _proj(ctx, y, xbar, 1.0)
    assert np.array_equal(a, b) and ia["lambda"] == ib["lambda"]
