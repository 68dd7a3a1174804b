"""GPU pins of the algorithm steps themselves, through the C ABI:

* Algorithm 1 (Sec. 2.1) on the hand-traced instances of
  tests/golden/hand_examples.json: the GPU's iterates (evaluated points and
  breakpoint steps) equal the hand-derived ones, and the trace names the step
  that produced each (3 Newton, 4 secant, 5 breakpoint);
* the secant instance tiled over 300 002 indices (many tiles, a ragged
  tail, compaction on), whose iterates are exact in binary and so equal;
* Algorithm 2 (Sec. 2.2) on one thread's chunk: the GPU start records what
  lane 0 of the first wave computed, which must equal the sequential
  Algorithm 2 of the oracle on those values in that order (Sec. 4: each
  chunk runs Algorithm 2 on its own), and every value that lane dropped must
  be zero at the solution.
"""
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


def _iterates(trace):
    """The multipliers the GPU moved through: evaluated points (kind 1) and
    breakpoint steps (kind 5, phi known without a pass)."""
    return [t["lam"] for t in trace if t["kind"] in (1, 5)]


@pytest.mark.parametrize("compaction", ["off", "auto", "always"])
def test_alg1_golden_iterates(ctx, golden, compaction):
    for ex in golden["alg1_traces"]:
        t = [torch.tensor([float(v) for v in ex[k]], dtype=torch.float64, device="cuda")
             for k in "dablu"]
        x, info = ctx.solve(*t, ex["r"], check=False, trace=True, compaction=compaction)
        assert info["status"] == 0, (ex["name"], info)
        tr = ctx.trace()
        assert _iterates(tr) == ex["lams"], (ex["name"], tr)
        assert info["lambda"] == ex["lam"]
        assert x.cpu().numpy().tolist() == [float(v) for v in ex["x"]], ex["name"]
        steps = [t_["kind"] for t_ in tr if t_["kind"] in (3, 4, 6)]
        want = {"newton": 3, "secant": 4}
        # the step taken from each iterate but the last, in the oracle's names
        # (a breakpoint step is kind 5, followed by the Newton step from it)
        expect = [want[k] for k in ex["kinds"] if k in want]
        assert steps == expect, (ex["name"], steps)


def test_secant_tiled_many_tiles(ctx, golden):
    ex = next(e for e in golden["alg1_traces"] if e["name"] == "secant_step")
    k = 150_001
    inst = {c: np.tile(np.array([float(v) for v in ex[c]]), k) for c in "dablu"}
    r = float(ex["r"]) * k
    ref = O.solve_cqk(*[inst[c] for c in "dablu"], r)
    for compaction in ("off", "auto"):
        t = [torch.from_numpy(inst[c]).cuda() for c in "dablu"]
        x, info = ctx.solve(*t, r, check=False, trace=True, compaction=compaction)
        assert info["status"] == 0, info
        tr = ctx.trace()
        assert _iterates(tr) == ex["lams"]
        assert 4 in [t_["kind"] for t_ in tr]
        np.testing.assert_array_equal(x.cpu().numpy(), ref.x)


def _lane0_positions(V):
    """Indices in y of the 16 values lane 0 holds in the tile at index 0
    (value e at (e // V) * 64 * V + e % V)."""
    return np.array([(e // V) * 64 * V + e % V for e in range(16)])


@pytest.mark.parametrize("l1", [False, True])
@pytest.mark.parametrize("dtype,accum", [("f64", "default"), ("f32", "f64")])
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_alg2_one_chunk_equals_sequential(ctx, l1, dtype, accum, seed):
    npdt = np.float64 if dtype == "f64" else np.float32
    V = 2 if dtype == "f64" else 4
    n = 300_000
    rng = np.random.default_rng(100 + seed)
    y = (0.5 * rng.standard_normal(n)).astype(npdt)
    pos = _lane0_positions(V)
    # lane 0's values: spread over [0, 3) with a few restarts of Algorithm 2
    # forced by large late values; the tile's largest value (3) sits in
    # another lane, so the wave's filter threshold is 3 - r = 0
    vals = rng.uniform(0.0, 3.0, 16)
    vals[rng.choice(16, 3, replace=False)] = rng.uniform(2.0, 2.9, 3)
    if l1:
        vals *= rng.choice([-1.0, 1.0], 16)
        vals[rng.integers(0, 16)] = 0.0
    y[pos] = vals.astype(npdt)
    y[5 * V] = npdt(3.0)
    r = 3.0
    yt = torch.from_numpy(y).cuda()
    proj = ctx.project_l1 if l1 else ctx.project_simplex
    x, info = proj(yt, r, check=False, trace=True, accum=accum)
    assert info["status"] == 0, info
    tr = ctx.trace()
    assert tr and tr[0]["kind"] == 7, tr[:2]
    rec = tr[0]
    yd = y.astype(np.float64)
    v = np.abs(yd) if l1 else yd
    active = [e for e in range(16) if (rec["n_in"] >> e) & 1]
    # the filter: exactly the values above the recorded threshold
    assert active == [e for e in range(16) if v[pos[e]] > rec["slope"]]
    assert len(active) >= 8
    lam_seq, J = O.condat_lambda0(yd, r, I=pos[active], l1=l1)
    J_gpu = sorted(int(pos[e]) for e in range(16) if (rec["n_out"] >> e) & 1)
    assert J_gpu == sorted(J)
    assert rec["compacted"] == len(J)
    assert abs(rec["phi"] - float(np.sum(v[J]))) <= 1e-13 * max(1.0, float(np.sum(v[J])))
    assert abs(rec["lam"] - lam_seq) <= 1e-12 * max(1.0, abs(lam_seq))
    # Sec. 2.2: every value the lane dropped is zero at the solution
    xs, lam_star = O.project_l1(yd, r) if l1 else O.project_simplex(yd, r)
    kept = [e for e in range(16) if (rec["source"] >> e) & 1]
    dropped = [e for e in range(16) if e not in kept]
    S = max(float(np.max(np.abs(xs))), float(np.max(np.abs(yd))), abs(lam_star))
    assert all(abs(xs[pos[e]]) <= 2e-10 * S for e in dropped), (dropped, xs[pos])
    # and the bounds are upper bounds of lam* (Sec. 2.2)
    if not l1:
        assert rec["lam"] >= lam_star - 1e-12 * S and rec["lo"] >= lam_star - 1e-12 * S
    # the whole projection still matches the oracle
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert float(np.max(np.abs(x.cpu().numpy().astype(np.float64) - xs))) <= tol * S


def test_start_keeps_the_whole_support(ctx):
    """Every index the Algorithm 2 start drops is written 0 and never written
    again, so the final support containing the oracle's support shows that
    the dropped set lies in {x* = 0} for every chunk (Sec. 2.2), here at
    n = 2e6 where the start drops most values."""
    for dist in ("normal", "uniform"):
        y = W.simplex_input(2_000_000, 9, dist, np.float32)
        x, info = ctx.project_simplex(torch.from_numpy(y).cuda(), 1.0, check=False)
        assert info["status"] == 0
        assert info["n_after_init"] < y.size // 4
        xs, lam = O.project_simplex(y.astype(np.float64), 1.0)
        S = max(float(np.max(np.abs(xs))), float(np.max(np.abs(y))), abs(lam))
        xg = x.cpu().numpy()
        must = xs > 2e-5 * S
        assert np.all(xg[must] > 0)
