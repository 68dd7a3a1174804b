"""GPU parity of the SPG driver on the l1-constrained least-squares problem
of Section 5.2 (cqk_spg_l1_lasso_f64) against the oracle's SPG
(oracle.spg_l1_lasso): the same method, with the objective and the spectral
quotient formed from their definitions on the CPU and from the identities
f(x + t d) = f + t g'd + t^2/2 ||Ad||^2, s'y = t^2 ||Ad||^2 on the GPU.

Where the problem has one solution (A of full column rank) the iterates are
compared to a tight tolerance; where it need not (more columns than rows) the
objective values are compared and the returned point must be feasible and
stationary to the tolerance, checked with the oracle's projection."""
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


def _gpu(ctx, A, b, radius, **kw):
    x, info = ctx.spg_l1_lasso(torch.from_numpy(np.ascontiguousarray(A)).cuda(),
                               torch.from_numpy(b).cuda(), radius, check=False, **kw)
    return x.cpu().numpy(), info


def _pg(A, b, x, radius):
    g = A.T @ (A @ x - b)
    return float(np.max(np.abs(O.project_l1(x - g, radius)[0] - x)))


@pytest.mark.parametrize("m,n", [(300, 120), (301, 127), (1000, 64)])
@pytest.mark.parametrize("frac", [0.3, 5.0])
def test_spg_unique_solution(ctx, m, n, frac):
    A, b, _ = W.lasso_instance(m, n, 10, 71 + m + n)
    radius = frac * float(np.sum(np.abs(np.linalg.lstsq(A, b, rcond=None)[0])))
    x_ref, ref = O.spg_l1_lasso(A, b, radius, tol=1e-11)
    x, info = _gpu(ctx, A, b, radius, tol=1e-11)
    assert info["status"] == 0 and ref["status"] == O.OK, info
    scale = max(1.0, float(np.max(np.abs(x_ref))))
    assert np.max(np.abs(x - x_ref)) <= 1e-8 * scale
    assert abs(info["objective"] - ref["f"]) <= 1e-10 * max(1.0, ref["f"])
    assert np.sum(np.abs(x)) <= radius * (1 + 1e-12)
    if frac > 1:  # the ball is inactive: least squares
        assert np.max(np.abs(x - np.linalg.lstsq(A, b, rcond=None)[0])) <= 1e-8 * scale


@pytest.mark.parametrize("m,n,k", [(128, 2048, 20), (96, 5001, 8)])
def test_spg_underdetermined(ctx, m, n, k):
    A, b, x_true = W.lasso_instance(m, n, k, 81 + n)
    radius = float(np.sum(np.abs(x_true)))
    x_ref, ref = O.spg_l1_lasso(A, b, radius, tol=1e-7)
    x, info = _gpu(ctx, A, b, radius, tol=1e-7)
    assert info["status"] == 0, info
    assert info["pg"] <= 1e-7
    assert _pg(A, b, x, radius) <= 1e-6
    assert np.sum(np.abs(x)) <= radius * (1 + 1e-12)
    f = 0.5 * float(np.sum((A @ x - b) ** 2))
    assert abs(f - info["objective"]) <= 1e-10 * max(1.0, f)
    assert abs(f - ref["f"]) <= 1e-5 * max(1e-3, ref["f"])


def test_spg_warm_and_cold_projections_agree(ctx):
    A, b, x_true = W.lasso_instance(256, 4096, 30, 91)
    radius = 0.8 * float(np.sum(np.abs(x_true)))
    xw, iw = _gpu(ctx, A, b, radius, tol=1e-8, warm=True)
    xc, ic = _gpu(ctx, A, b, radius, tol=1e-8, warm=False)
    assert iw["status"] == 0 and ic["status"] == 0
    assert abs(iw["objective"] - ic["objective"]) <= 1e-9 * max(1.0, ic["objective"])
    assert iw["projections"] == 2 * iw["iterations"] + 1
    assert iw["newton_iterations"] <= ic["newton_iterations"]


def test_spg_iteration_limit_and_errors(ctx):
    import paper_2603_15910_amd as cqk
    A, b, _ = W.lasso_instance(64, 500, 5, 95)
    radius = 5.0
    _, ref = O.spg_l1_lasso(A, b, radius, tol=1e-14, max_iter=3)
    assert ref["status"] == O.NOT_CONVERGED
    x, info = _gpu(ctx, A, b, radius, tol=1e-14, max_iter=3)
    assert info["status"] == cqk.CQK_NOT_CONVERGED and info["iterations"] == 3
    assert np.sum(np.abs(x)) <= radius * (1 + 1e-12)
    At = torch.from_numpy(A).cuda()
    bt = torch.from_numpy(b).cuda()
    with pytest.raises(cqk.CqkError):
        ctx.spg_l1_lasso(At, bt, -1.0)
    with pytest.raises(cqk.CqkError):   # x over A
        ctx.spg_l1_lasso(At, bt, 1.0, out=At.view(-1)[:500])
    with pytest.raises(cqk.CqkError):
        ctx.spg_l1_lasso(At, bt, 1.0, memory=0)
