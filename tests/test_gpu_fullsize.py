"""Parity at the benchmark sizes (n = 1e8), in the launch configuration
bench.py times, through the C ABI.

At this size the exact oracle solve of the general problem would take
minutes, so the GPU result is checked by what defines the solution:
  * every sampled x_i equals eq. (xopt) at the returned multiplier,
    x_i = clamp((a_i + lam b_i)/d_i, l_i, u_i), computed by the oracle one
    index at a time;
  * phi(lam) = b^T x(lam) equals r to the stated tolerance
    (|b^T x - r| <= 1e-10 ||b||_1 ||x||_inf), phi summed by the oracle in
    extended precision over all n indices;
  * the free set is the one the oracle's slopes see at lam (phi'_- <= Q <= phi'_+
    counts agree with the GPU's n_free).
The simplex at n = 1e8 is compared with the oracle's exact sort solution.
"""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W

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
def test_cqk_1e8_fp64_properties_and_samples(ctx, gen):
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
    # the multiplier is a root of phi(lam) = r at the stated tolerance
    b1 = float(np.sum(np.abs(b)))
    xinf = float(np.max(np.abs(x)))
    assert abs(O.phi(lam, d, a, b, l, u) - r) <= 1e-10 * b1 * xinf
    # and the returned x itself is feasible
    assert abs(float(np.sum(b * x, dtype=np.float64)) - r) <= 1e-10 * b1 * xinf
    assert np.all(x >= l) and np.all(x <= u)
    # free set size: between the counts of the two one-sided slopes' sets
    t_ = (b * lam + a) / d
    free_strict = int(np.count_nonzero((t_ > l) & (t_ < u)))
    assert abs(info["n_free"] - free_strict) <= max(10, free_strict // 10**6)


@pytest.mark.parametrize("dist", ["normal", "uniform"])
def test_simplex_1e8_fp32_against_sort(ctx, dist):
    y = W.simplex_input(N, 1, dist, np.float32)
    yt = torch.from_numpy(y).cuda()
    x_dev, info = ctx.project_simplex(yt, 1.0, check=False)
    assert info["status"] == 0, info
    x = x_dev.cpu().numpy()
    del x_dev, yt
    torch.cuda.empty_cache()
    x_ref, lam_ref = O.project_simplex(y.astype(np.float64), 1.0)
    S = max(float(np.max(np.abs(x_ref))), float(np.max(np.abs(y))), abs(lam_ref))
    assert abs(info["lambda"] - lam_ref) <= 1e-5 * S
    assert float(np.max(np.abs(x.astype(np.float64) - x_ref))) <= 1e-5 * S
    assert abs(float(np.sum(x, dtype=np.float64)) - 1.0) <= 1e-5


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
