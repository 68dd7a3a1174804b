"""GPU parity of the general CQK path when a bracket estimated from a sample
lets the first pass compact (n >= 2^22 with compaction on), through the C
ABI: the result against the CPU oracle, Algorithm 1's iterates against a run
without compaction, and the return to the caller's arrays when an iterate
leaves the sampled bracket."""
import numpy as np
import pytest

from oracle import cqk_oracle as O
from paper_2603_15910_amd import workloads as W
from tests.parity import check_cqk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# the two samples: 64 and 16384 tiles of 64 indices spread evenly
SAMPLE_TILES = (64, 16384)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_15910_amd as cqk
    c = cqk.Context(0)
    yield c
    c.close()


def _solve(ctx, inst, dtype=torch.float64, **kw):
    t = [torch.from_numpy(np.asarray(inst[k])).to("cuda", dtype) for k in "dablu"]
    x, info = ctx.solve(*t, inst["r"], check=False, trace=True, **kw)
    return x.cpu().numpy().astype(np.float64), info, ctx.trace()


def _evals(tr):
    return [t for t in tr if t["kind"] == 1]


def _sampled_positions(n, tiles):
    """Indices a sample of `tiles` tiles reads: tile j covers
    [j * (n // tiles), + 64)."""
    span = n // tiles
    return (np.arange(tiles)[:, None] * span + np.arange(64)[None, :]).ravel()


def _estimates(tr):
    """The two bracket estimates' records (kinds 8 and 9)."""
    e1 = [t for t in tr if t["kind"] == 8]
    e2 = [t for t in tr if t["kind"] == 9]
    assert len(e1) == 1 and len(e2) == 1, (e1, e2)
    assert e1[0]["n_in"] == 64 * SAMPLE_TILES[0] and e2[0]["n_in"] == 64 * SAMPLE_TILES[1]
    return e1[0], e2[0]


def _newton_from_zero(inst):
    """lam_1 of Algorithm 1 from lam_0 = 0 (one Newton step, eq. (phideriv))."""
    d, a, b, l, u = (inst[k] for k in "dablu")
    c, s = b * a / d, b * b / d
    f = c
    ph = np.sum(np.clip(f, b * l, b * u))
    res = ph - inst["r"]
    if res > 0:
        slope = np.sum(np.where((f > b * l) & (f <= b * u), s, 0.0))
    else:
        slope = np.sum(np.where((f >= b * l) & (f < b * u), s, 0.0))
    return -res / slope


@pytest.mark.parametrize("gen", ["uniform", "correlated"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sampled_bracket_compacts_the_first_pass(ctx, gen, dtype):
    n = 4_500_007
    inst = W.cqk_uniform(n, 41) if gen == "uniform" else W.cqk_correlated(n, 41)
    if dtype == torch.float32:
        inst = {k: (v.astype(np.float32).astype(np.float64) if k in "dablu" else v)
                for k, v in inst.items()}
        inst["r"] = float(np.dot(inst["b"], (inst["l"] + inst["u"]) / 2))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    x, info, tr = _solve(ctx, inst, dtype, compaction="auto")
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, tol)
    s1, s = _estimates(tr)
    # even samples of i.i.d. indices: both brackets (5 standard deviations)
    # hold lam*; the second, used, is the narrower
    assert s1["lo"] < ref.lam < s1["hi"], (s1, ref.lam)
    assert s["compacted"] == 1 and s["lo"] < ref.lam < s["hi"], (s, ref.lam)
    assert s["hi"] - s["lo"] < s1["hi"] - s1["lo"], (s1, s)
    assert 0.0 < s["slope"] < 0.1, s
    ev = _evals(tr)
    assert ev[0]["source"] == 0 and ev[0]["n_out"] > 0, ev[0]
    # the first iterate strictly inside the bracket is evaluated on the set
    # the first pass wrote (set 1), unless a smaller set was adopted first;
    # uniform: lam_1 already; correlated: Newton from 0 overshoots, lam_2
    k = next(k for k in range(1, len(ev)) if s["lo"] < ev[k]["lam"] < s["hi"])
    if gen == "uniform":
        assert k == 1 and ev[0]["compacted"] == 1, ev[:2]
    assert ev[k - 1]["compacted"] == 1, ev[:k + 1]
    assert (ev[k]["source"] == 3 and ev[k]["n_in"] == ev[0]["n_out"]) or \
        ev[k]["n_in"] < ev[0]["n_out"], ev[:k + 1]
    # the first pass kept at most the share the sample allows (per wave: that
    # share of the indices read, plus one piece of 64)
    assert ev[0]["n_out"] <= (1.5 * s["slope"] + 1.0 / 32) * n + 64 * 8192, (ev[0], s)
    # Algorithm 1 moved through the same multipliers as without compaction
    # (to rounding: the sums over a compacted set are added in another order)
    _, _, tr0 = _solve(ctx, inst, dtype, compaction="off")
    assert not any(t["kind"] in (8, 9) for t in tr0)
    _same_iterates(ev, _evals(tr0))


def _same_iterates(ev, ev0, exact_first=True):
    """exact_first: lam_0 is the same number on both runs (lam_0 = 0); a
    formula start sums its terms in another order on the two paths."""
    lam_on = [t["lam"] for t in ev]
    lam_off = [t["lam"] for t in ev0]
    assert abs(len(lam_on) - len(lam_off)) <= 1, (lam_on, lam_off)
    k = min(len(lam_on), len(lam_off))
    if exact_first:
        assert lam_on[0] == lam_off[0]
    np.testing.assert_allclose(lam_on[:k], lam_off[:k], rtol=1e-9, atol=1e-12)


def test_iterate_outside_the_sampled_bracket_reads_the_arrays_again(ctx):
    """The second sample's tiles are made unrepresentative: nearly equal
    entries that put its solution on lam_1 with a bracket far narrower than
    |lam_1 - lam*|.  The first pass compacts for it and the second reads the
    set (lam_1 is inside); the next iterate lies outside, so a later pass
    reads the caller's arrays, and the result is still the oracle's."""
    n = 4_500_007
    inst = W.cqk_uniform(n, 43)
    pos = _sampled_positions(n, SAMPLE_TILES[1])
    rng = np.random.default_rng(44)
    noise = rng.uniform(-1e-3, 1e-3, pos.size)
    # d = b = 1 and bounds far apart: g_i = a_i + lam on the sample
    inst["d"][pos] = 1.0
    inst["b"][pos] = 1.0
    inst["l"][pos] = -50.0
    inst["u"][pos] = 50.0
    target = 0.0
    for _ in range(12):
        # sampled equation: sum_S (a_i + lam) = r m / n at lam = lam_1
        inst["r"] = float(np.dot(inst["b"], (inst["l"] + inst["u"]) / 2))
        inst["a"][pos] = inst["r"] / n - target + noise
        target = _newton_from_zero(inst)
    inst["r"] = float(np.dot(inst["b"], (inst["l"] + inst["u"]) / 2))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    assert abs(ref.lam - target) > 1e-4      # lam* far outside the bracket (~3e-6)
    x, info, tr = _solve(ctx, inst, compaction="auto")
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)
    _, s = _estimates(tr)
    assert s["compacted"] == 1 and s["lo"] < target < s["hi"], (s, target)
    assert not (s["lo"] < ref.lam < s["hi"])
    ev = _evals(tr)
    assert ev[0]["compacted"] == 1 and ev[1]["source"] == 3, ev[:2]
    assert any(t["source"] == 0 for t in ev[2:]), ev
    # and the multipliers are those of the run without compaction
    _, _, tr0 = _solve(ctx, inst, compaction="off")
    _same_iterates(ev, _evals(tr0))


def test_sample_that_cannot_move_gives_no_bracket(ctx):
    """Every sampled index fixed (l = u): the sampled equation has no
    solution, no bracket is used and the first pass only evaluates."""
    n = 4_194_304
    inst = W.cqk_uniform(n, 45)
    for tiles in SAMPLE_TILES:
        pos = _sampled_positions(n, tiles)
        inst["l"][pos] = 0.0
        inst["u"][pos] = 0.0
    inst["r"] = float(np.dot(inst["b"], (inst["l"] + inst["u"]) / 2))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info, tr = _solve(ctx, inst, compaction="auto")
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)
    s1, s = _estimates(tr)
    assert np.isnan(s1["lo"]) and np.isnan(s1["hi"]), s1
    assert s["compacted"] == 0 and np.isnan(s["lo"]) and np.isnan(s["hi"]), s
    ev = _evals(tr)
    assert ev[0]["compacted"] == 0 and ev[0]["n_out"] == 0, ev[0]


def test_sampled_bracket_with_infinite_bounds(ctx):
    """A quarter of the lower bounds -inf and a quarter of the upper +inf
    (sampled entries included): parity with the oracle."""
    n = 4_300_001
    inst = W.cqk_uniform(n, 47)
    rng = np.random.default_rng(48)
    inst["l"][rng.random(n) < 0.25] = -np.inf
    inst["u"][rng.random(n) < 0.25] = np.inf
    lo = np.where(np.isfinite(inst["l"]), inst["l"], -5.0)
    hi = np.where(np.isfinite(inst["u"]), inst["u"], 5.0)
    inst["r"] = float(np.dot(inst["b"], (lo + hi) / 2))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    for compaction in ("auto", "always"):
        x, info, tr = _solve(ctx, inst, compaction=compaction)
        assert info["status"] == 0, (compaction, info)
        check_cqk(x, inst, ref, 1e-10)
        _estimates(tr)


def test_sampled_bracket_under_graph_capture(ctx):
    """The two sample estimates and the first pass's set inside a captured
    graph: every replay estimates again on the data then in the arrays (the
    estimate's ticket and state are set by the solve's own first kernel), and
    each replay's x is the oracle's."""
    import paper_2603_15910_amd as cqk
    n = 4_400_003
    inst = W.cqk_uniform(n, 49)
    inst2 = W.cqk_uniform(n, 50)
    t = [torch.from_numpy(inst[k]).cuda() for k in "dablu"]
    x = torch.empty_like(t[0])
    c = cqk.Context(0)
    try:
        c.reserve(n, 0)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                c.solve(*t, inst["r"], out=x, check=False, max_iter=12, trace=True)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
        for rep in range(3):
            x.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            st, info = c.ctx_last_info()
            assert st == cqk.CQK_OK, info
            check_cqk(x.cpu().numpy(), inst, ref, 1e-10)
            _, s2 = _estimates(c.trace())
            assert s2["compacted"] == 1 and s2["lo"] < ref.lam < s2["hi"], s2
        # other a with the same r (r depends on b, l, u only)
        t[1].copy_(torch.from_numpy(inst2["a"]))
        graph.replay()
        st, info = c.ctx_last_info()
        assert st == cqk.CQK_OK, info
        inst3 = dict(inst, a=inst2["a"])
        ref3 = O.solve_cqk(*[inst3[k] for k in "dablu"], inst["r"])
        check_cqk(x.cpu().numpy(), inst3, ref3, 1e-10)
        _, s3 = _estimates(c.trace())
        assert s3["lo"] < ref3.lam < s3["hi"], (s3, ref3.lam)
    finally:
        c.close()


@pytest.mark.parametrize("name", ["breakpoint_step_right", "breakpoint_step_left"])
def test_breakpoint_step_takes_the_waiting_set(ctx, golden, name):
    """The hand-traced breakpoint examples tiled past 2^22 indices: the
    sampled bracket around lam* holds no breakpoint (the set the first pass
    writes is empty), the breakpoint search runs on the caller's arrays while
    the set waits, and the Newton step after the breakpoint step lands in the
    bracket and takes the set.  Algorithm 1's iterates are the hand-traced
    ones, exactly."""
    ex = next(e for e in golden["alg1_traces"] if e["name"] == name)
    k = 1_400_003
    inst = {c: np.tile(np.array([float(v) for v in ex[c]]), k) for c in "dablu"}
    r = float(ex["r"]) * k
    inst["r"] = r
    ref = O.solve_cqk(*[inst[c] for c in "dablu"], r)
    x, info, tr = _solve(ctx, inst, compaction="auto")
    assert info["status"] == 0, info
    np.testing.assert_array_equal(x, ref.x)
    _, s = _estimates(tr)
    assert s["compacted"] == 1 and s["lo"] < ex["lam"] < s["hi"], s
    assert [t["lam"] for t in tr if t["kind"] in (1, 5)] == ex["lams"]
    ev = _evals(tr)
    assert ev[0]["n_out"] == 0, ev[0]
    assert ev[-1]["source"] == 3 and ev[-1]["n_in"] == 0, ev[-1]


@pytest.mark.parametrize("perturb", [0.0, 1e-3])
def test_warm_start_writes_the_sampled_set(ctx, perturb):
    """A warm start past 2^22 indices: the sample comes first, the warm
    start's own pass writes the sampled set beside eq. (CQKlambda0)'s sums
    over the estimate's free set, and the Newton pass at the warm lam_0 reads
    that set.  x against the oracle, lam_0 against the oracle's warm start."""
    import paper_2603_15910_amd as cqk  # noqa: F401
    n = 4_300_007
    inst = W.cqk_uniform(n, 51)
    xbar = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"]).x
    if perturb:
        inst = dict(inst, a=inst["a"] + np.random.default_rng(52).uniform(-perturb, perturb, n))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    t = [torch.from_numpy(np.asarray(inst[k])).cuda() for k in "dablu"]
    xb = torch.from_numpy(xbar).cuda()
    x, info = ctx.solve(*t, inst["r"], xbar=xb, check=False, trace=True)
    assert info["status"] == 0, info
    check_cqk(x.cpu().numpy(), inst, ref, 1e-10)
    lam0_ref = O.cqk_lambda0_warm(*[inst[k] for k in "dablu"], inst["r"], xbar)
    assert abs(info["lambda0"] - lam0_ref) <= 1e-10 * (1.0 + abs(lam0_ref)), \
        (info["lambda0"], lam0_ref)
    tr = ctx.trace()
    assert [t_["kind"] for t_ in tr[:3]] == [8, 9, 0], tr[:3]
    s = tr[1]
    assert s["compacted"] == 1 and s["lo"] < lam0_ref < s["hi"], (s, lam0_ref)
    assert tr[2]["compacted"] == 1, tr[2]
    ev = _evals(tr)
    assert ev[0]["source"] == 3 and 0 < ev[0]["n_in"] < 0.1 * n, ev[0]


@pytest.mark.parametrize("gen", ["uniform", "correlated"])
def test_formula_start_writes_the_sampled_set(ctx, gen):
    """The eq. (CQKlambda0) start past 2^22 indices: its pass over all indices
    also writes the sampled set; lam_0 is the formula's, x the oracle's, and
    the Newton pass at lam_0 reads the set when lam_0 lies in its bracket."""
    n = 4_300_007
    inst = W.cqk_uniform(n, 53) if gen == "uniform" else W.cqk_correlated(n, 53)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info, tr = _solve(ctx, inst, lambda0="formula")
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)
    lam0 = O.cqk_lambda0(*[inst[k] for k in "dablu"], inst["r"])
    assert abs(info["lambda0"] - lam0) <= 1e-12 * (1.0 + abs(lam0)), (info["lambda0"], lam0)
    assert [t["kind"] for t in tr[:3]] == [8, 9, 0], tr[:3]
    s, ev = tr[1], _evals(tr)
    if s["compacted"] == 1 and s["lo"] < info["lambda0"] < s["hi"]:
        assert tr[2]["compacted"] == 1 and ev[0]["source"] == 3, (tr[2], ev[0])
    else:
        assert ev[0]["source"] == 0 and ev[0]["n_out"] == 0, ev[0]
    # Algorithm 1's iterates are those of the same start without compaction
    _, _, tr0 = _solve(ctx, inst, lambda0="formula", compaction="off")
    _same_iterates(ev, _evals(tr0), exact_first=False)
