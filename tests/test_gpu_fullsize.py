"""Parity at the benchmark sizes (n = 1e8), in the launch configuration
bench.py times, through the C ABI.

General CQK (both generators, seed 1): the GPU x is compared with the
oracle's exact sort solution element by element (max |x - x*| <= 1e-10 S,
the free/fixed partition equal away from ties, |b^T x - r| within
1e-10 ||b||_1 ||x||_inf), and with the stricter 1e-10 ||x*||_inf figure; it
is also checked by what defines the solution (every sampled x_i equals
eq. (xopt) at the returned multiplier, l <= x <= u).  At this size each
wave of the pass kernel owns 48 tiles, so its compaction ring wraps many
times.

Simplex and l1 (both distributions): all sixteen runs the benchmark times
(2 problems x 2 accumulators x 2 starts per distribution) are compared
with the sort solution; the paths that carry the multiplier in FP64 also
meet 1e-5 ||x*||_inf (pure FP32 arithmetic can only meet the
S-relative bound, since x = fl(y + lam) inherits half an ulp of lam).
"""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W
from tests.parity import check_cqk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 100_000_000


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_15910_amd as cqk
    c = cqk.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("gen", ["uniform", "correlated"])
def test_cqk_1e8_fp64_against_oracle(ctx, gen):
    inst = W.cqk_uniform(N, 1) if gen == "uniform" else W.cqk_correlated(N, 1)
    t = [torch.from_numpy(inst[k]).cuda() for k in "dablu"]
    x_dev, info = ctx.solve(*t, inst["r"], check=False)
    del t
    assert info["status"] == 0, info
    lam = info["lambda"]
    x = x_dev.cpu().numpy()
    del x_dev
    torch.cuda.empty_cache()
    d, a, b, l, u = (inst[k] for k in "dablu")
    r = inst["r"]
    # sampled outputs, each from eq. (xopt) at the returned multiplier
    rng = np.random.default_rng(7)
    idx = rng.choice(N, 200_000, replace=False)
    xo = O.x_of_lambda(lam, d[idx], a[idx], b[idx], l[idx], u[idx])
    S = max(np.max(np.abs(xo)), np.max(np.abs(a[idx] / d[idx])),
            abs(lam) * np.max(b[idx] / d[idx]))
    assert np.max(np.abs(x[idx] - xo)) <= 1e-10 * S
    assert np.all(x >= l) and np.all(x <= u)
    # element by element against the exact solution
    ref = O.solve_cqk(d, a, b, l, u, r)
    assert ref.status == O.OK
    check_cqk(x, inst, ref, 1e-10)
    xinf = float(np.max(np.abs(ref.x)))
    assert float(np.max(np.abs(x - ref.x))) <= 1e-10 * xinf
    free_ref = int(np.count_nonzero((ref.x > l) & (ref.x < u)))
    assert abs(info["n_free"] - free_ref) <= max(10, free_ref // 10**6)


@pytest.mark.parametrize("l1", [False, True])
@pytest.mark.parametrize("dist", ["normal", "uniform"])
def test_simplex_l1_1e8_every_benchmark_leg(ctx, dist, l1):
    y = W.simplex_input(N, 1, dist, np.float32)
    yd = y.astype(np.float64)
    x_ref, lam_ref = O.project_l1(yd, 1.0) if l1 else O.project_simplex(yd, 1.0)
    S = max(float(np.max(np.abs(x_ref))), float(np.max(np.abs(yd))), abs(lam_ref))
    xinf = float(np.max(np.abs(x_ref)))
    support = x_ref != 0
    yt = torch.from_numpy(y).cuda()
    x_dev = torch.empty_like(yt)
    proj = ctx.project_l1 if l1 else ctx.project_simplex
    for accum in ("f64", "f32"):
        for start in ("condat", "zero"):
            _, info = proj(yt, 1.0, out=x_dev, check=False, accum=accum, lambda0=start)
            assert info["status"] == 0, (accum, start, info)
            x = x_dev.cpu().numpy().astype(np.float64)
            err = float(np.max(np.abs(x - x_ref)))
            assert err <= 1e-5 * S, (accum, start, err, S)
            if accum == "f64":
                # the multiplier in FP64: the stricter bound holds too
                assert err <= 1e-5 * xinf, (accum, start, err, xinf)
                assert abs(info["lambda"] - lam_ref) <= 1e-10 * S
            tie = np.abs(x_ref) <= 2e-5 * S
            assert not np.any(((x != 0) != support) & ~tie), (accum, start)
            total = float(np.sum(np.abs(x))) if l1 else float(np.sum(x))
            # FP64 multiplier: each x_i is y_i + lam rounded once; FP32: the
            # check_simplex bound (every x_i within 1e-5 of its own scale)
            bound = 1e-6 if accum == "f64" else 1e-5 * N * xinf
            assert abs(total - 1.0) <= bound, (accum, start, total)
    del yt, x_dev
    torch.cuda.empty_cache()


def test_cqk_1e8_warm_from_previous_solution(ctx):
    """The warm start at the benchmark size: the previous point's solution
    (oracle x(lam) at the previous problem's multiplier, from eq. (xopt))
    starts a solve of the problem with a perturbed; the result is held to the
    same properties as the cold solve, and lambda_0 to the oracle's warm
    formula over all n."""
    prev = W.cqk_uniform(N, 1)
    d, b, l, u = (prev[k] for k in "dblu")
    r = prev["r"]
    t = {k: torch.from_numpy(prev[k]).cuda() for k in "dablu"}
    _, info0 = ctx.solve(*[t[k] for k in "dablu"], r, check=False)
    assert info0["status"] == 0
    xbar = O.x_of_lambda(info0["lambda"], d, prev["a"], b, l, u)
    a = W.perturbed(prev["a"], 2, 1e-3)
    del prev
    t["a"] = torch.from_numpy(a).cuda()
    x_dev, info = ctx.solve(*[t[k] for k in "dablu"], r, xbar=torch.from_numpy(xbar).cuda(),
                            check=False)
    del t
    assert info["status"] == 0, info
    lam0_ref = O.cqk_lambda0_warm(d, a, b, l, u, r, xbar)
    assert abs(info["lambda0"] - lam0_ref) <= 1e-9 * max(1.0, abs(lam0_ref))
    lam = info["lambda"]
    x = x_dev.cpu().numpy()
    del x_dev
    torch.cuda.empty_cache()
    rng = np.random.default_rng(8)
    idx = rng.choice(N, 200_000, replace=False)
    xo = O.x_of_lambda(lam, d[idx], a[idx], b[idx], l[idx], u[idx])
    S = max(np.max(np.abs(xo)), np.max(np.abs(a[idx] / d[idx])), abs(lam) * np.max(b[idx] / d[idx]))
    assert np.max(np.abs(x[idx] - xo)) <= 1e-10 * S
    b1 = float(np.sum(np.abs(b)))
    xinf = float(np.max(np.abs(x)))
    assert abs(O.phi(lam, d, a, b, l, u) - r) <= 1e-10 * b1 * xinf


def test_simplex_1e8_fp32_warm_against_sort(ctx):
    y0 = W.simplex_input(N, 1, "normal", np.float32)
    x0, _ = O.project_simplex(y0.astype(np.float64), 1.0)
    y = W.perturbed(y0, 2, 1e-3)
    del y0
    yt = torch.from_numpy(y).cuda()
    x_dev, info = ctx.project_simplex(yt, 1.0, xbar=torch.from_numpy(x0.astype(np.float32)).cuda(),
                                      check=False)
    assert info["status"] == 0, info
    x = x_dev.cpu().numpy()
    del x_dev, yt
    torch.cuda.empty_cache()
    x_ref, lam_ref = O.project_simplex(y.astype(np.float64), 1.0)
    S = max(float(np.max(np.abs(x_ref))), float(np.max(np.abs(y))), abs(lam_ref))
    assert info["lambda0"] >= lam_ref - 1e-12 * S
    assert abs(info["lambda"] - lam_ref) <= 1e-5 * S
    assert float(np.max(np.abs(x.astype(np.float64) - x_ref))) <= 1e-5 * S
