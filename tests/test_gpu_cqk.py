"""GPU parity of the general CQK path (cqk_solve_f64 / cqk_solve_f32) against
the CPU oracle, through the C ABI."""
import math

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


def _dev(inst, dtype=torch.float64):
    return [torch.from_numpy(np.asarray(inst[k])).to("cuda", dtype) for k in "dablu"]


def _solve(ctx, inst, dtype=torch.float64, **kw):
    t = _dev(inst, dtype)
    x, info = ctx.solve(*t, inst["r"], check=False, **kw)
    return x.cpu().numpy().astype(np.float64), info


@pytest.mark.parametrize("seed", range(1, 21))
def test_uniform_n1e5_all_seeds(ctx, seed):
    inst = W.cqk_uniform(100_000, seed)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst)
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)
    assert 2 <= info["iterations"] <= 12


@pytest.mark.parametrize("gen", ["correlated", "paper_unc", "paper_weak", "paper_cor"])
@pytest.mark.parametrize("n", [1, 7, 1000, 4099, 65537, 300_001])
def test_generators_and_ragged_sizes(ctx, gen, n):
    f = {"correlated": lambda: W.cqk_correlated(n, 3),
         "paper_unc": lambda: W.cqk_paper(n, 4, "uncorrelated"),
         "paper_weak": lambda: W.cqk_paper(n, 5, "weak"),
         "paper_cor": lambda: W.cqk_paper(n, 6, "correlated")}[gen]
    inst = f()
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst)
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)


@pytest.mark.parametrize("compaction", ["off", "auto", "always"])
@pytest.mark.parametrize("lambda0", ["zero", "formula"])
def test_compaction_modes_agree(ctx, compaction, lambda0):
    inst = W.cqk_uniform(200_003, 11)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst, compaction=compaction, lambda0=lambda0, trace=True)
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)
    tr = ctx.trace()
    if compaction == "always":
        assert any(t["compacted"] for t in tr)
    if compaction == "off":
        assert not any(t["compacted"] for t in tr)
    # the bracket always contains the exact multiplier
    for t in tr:
        if t["kind"] == 1:
            assert t["lo"] <= ref.lam + 1e-9 * (1 + abs(ref.lam))
            assert t["hi"] >= ref.lam - 1e-9 * (1 + abs(ref.lam))


def test_compaction_keeps_iteration_count(ctx):
    inst = W.cqk_correlated(150_000, 12)
    _, i_off = _solve(ctx, inst, compaction="off")
    _, i_on = _solve(ctx, inst, compaction="always")
    assert abs(i_off["iterations"] - i_on["iterations"]) <= 1


def _tiny(rng, n, kind):
    d = rng.uniform(0.5, 3.0, n); a = rng.uniform(-3.0, 3.0, n); b = rng.uniform(0.5, 3.0, n)
    l = rng.uniform(-2.0, 0.5, n); u = l + rng.uniform(0.0, 2.0, n)
    if kind == "int":
        d = rng.integers(1, 3, n).astype(float); a = rng.integers(-3, 4, n).astype(float)
        b = rng.integers(1, 3, n).astype(float); l = rng.integers(-2, 1, n).astype(float)
        u = l + rng.integers(0, 3, n).astype(float)
    if kind == "inf":
        l[rng.random(n) < 0.3] = -np.inf
        u[rng.random(n) < 0.3] = np.inf
    lo = float(np.dot(b, np.where(np.isfinite(l), l, -5)))
    hi = float(np.dot(b, np.where(np.isfinite(u), u, 5)))
    r = float(rng.uniform(lo, hi)) if kind != "int" else float(rng.integers(math.floor(lo), math.ceil(hi) + 1))
    return {"d": d, "a": a, "b": b, "l": l, "u": u, "r": r}


@pytest.mark.parametrize("kind", ["real", "int", "inf"])
def test_tiny_against_bruteforce(ctx, kind):
    rng = np.random.default_rng(100 + ["real", "int", "inf"].index(kind))
    for trial in range(60):
        n = int(rng.integers(1, 7))
        inst = _tiny(rng, n, kind)
        bf = O.solve_bruteforce(*[inst[k] for k in "dablu"], inst["r"])
        x, info = _solve(ctx, inst)
        if bf is None:
            assert info["status"] == 1, (trial, info)
            continue
        assert info["status"] == 0, (trial, inst, info)
        scale = max(1.0, np.max(np.abs(bf[0])))
        assert np.max(np.abs(x - bf[0])) <= 1e-9 * scale, (trial, x, bf[0])


def test_edge_cases(ctx):
    one = np.ones(4)
    base = {"d": one, "a": one, "b": one, "l": np.zeros(4), "u": one}
    # infeasible on both sides
    for r in (4.5, -0.1):
        _, info = _solve(ctx, dict(base, r=r))
        assert info["status"] == 1, (r, info)
    # r at the boundary: x = u
    x, info = _solve(ctx, dict(base, r=4.0))
    assert info["status"] == 0 and np.all(x == 1.0)
    # invalid data found on the device
    for k, v in (("d", 0.0), ("b", -1.0), ("a", np.nan), ("l", 2.0), ("d", np.inf)):
        bad = {kk: np.array(vv, dtype=float) for kk, vv in base.items()}
        bad[k][1] = v
        _, info = _solve(ctx, dict(bad, r=1.0))
        assert info["status"] == 2, (k, v, info)
    # breakpoint branch: every index clamped at lam = 0
    inst = {"d": np.ones(3), "a": np.array([-5.0, -6.0, -7.0]), "b": np.ones(3),
            "l": np.zeros(3), "u": np.ones(3), "r": 1.5}
    x, info = _solve(ctx, inst)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    assert info["status"] == 0
    np.testing.assert_allclose(x, ref.x, atol=1e-12)
    # max_iter = 1 cannot converge on a real instance
    inst = W.cqk_uniform(5000, 3)
    _, info = _solve(ctx, inst, max_iter=1)
    assert info["status"] == 3
    # user start at the exact multiplier stops at once
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst, lambda0="user", lambda0_user=ref.lam)
    assert info["status"] == 0 and info["iterations"] <= 2
    check_cqk(x, inst, ref, 1e-10)


def test_unbounded_and_mixed_infinite_bounds(ctx):
    rng = np.random.default_rng(5)
    n = 50_000
    inst = W.cqk_uniform(n, 5)
    inst["l"] = inst["l"].copy(); inst["u"] = inst["u"].copy()
    inst["l"][rng.random(n) < 0.2] = -np.inf
    inst["u"][rng.random(n) < 0.2] = np.inf
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst)
    assert info["status"] == 0, info
    check_cqk(x, inst, ref, 1e-10)


def test_fp32_inputs(ctx):
    inst = W.cqk_uniform(123_457, 9, dtype=np.float32)
    inst64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in inst.items()}
    ref = O.solve_cqk(*[inst64[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst, dtype=torch.float32)
    assert info["status"] == 0, info
    check_cqk(x, inst64, ref, 1e-5)


def test_deterministic_repeats(ctx):
    inst = W.cqk_correlated(400_000, 13)
    t = _dev(inst)
    outs = []
    for _ in range(5):
        x, info = ctx.solve(*t, inst["r"])
        outs.append((x.cpu().numpy().tobytes(), info["lambda"], info["iterations"]))
    assert all(o == outs[0] for o in outs)


def test_info_fields(ctx):
    inst = W.cqk_uniform(100_000, 2)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    x, info = _solve(ctx, inst, timing=True, trace=True)
    assert info["status"] == 0
    assert info["stop_reason"] in (1, 2, 3, 4)
    assert info["residual"] <= 1e-10 * np.sum(np.abs(inst["b"])) * np.max(np.abs(x))
    assert info["n_free"] == int(np.sum((ref.x > inst["l"]) & (ref.x < inst["u"])))
    assert info["pass_bytes"] >= 40 * 100_000 * info["iterations"] * 0.2
    assert info["pass_ms"] > 0 and info["finalize_ms"] > 0


@pytest.mark.parametrize("shift", [1, 3])
def test_unaligned_views(ctx, shift):
    inst = W.cqk_uniform(50_001, 14)
    t = [torch.from_numpy(inst[k]).cuda()[shift:] for k in "dablu"]
    sub = {k: inst[k][shift:] for k in "dablu"}
    sub["r"] = float(np.dot(sub["b"], (sub["l"] + sub["u"]) / 2))
    ref = O.solve_cqk(*[sub[k] for k in "dablu"], sub["r"])
    xbuf = torch.empty(50_001, dtype=torch.float64, device="cuda")
    x, info = ctx.solve(*t, sub["r"], out=xbuf[shift:], check=False)
    assert info["status"] == 0
    check_cqk(x.cpu().numpy(), sub, ref, 1e-10)


@pytest.mark.parametrize("gen", ["uniform", "correlated"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_several_tiles_per_wave(ctx, gen, dtype):
    """n = 8e6 + 5: every wave of the pass kernel streams four tiles (a
    ragged last one), so its compaction ring wraps and flushes across tiles
    as at the benchmark size; all three compaction modes against the exact
    solution."""
    n = 8_000_005
    inst = W.cqk_uniform(n, 21) if gen == "uniform" else W.cqk_correlated(n, 21)
    if dtype == torch.float32:
        inst = {k: (v.astype(np.float32).astype(np.float64) if k in "dablu" else v)
                for k, v in inst.items()}
        inst["r"] = float(np.dot(inst["b"], (inst["l"] + inst["u"]) / 2))
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    for compaction in ("auto", "always", "off"):
        x, info = _solve(ctx, inst, dtype, compaction=compaction, trace=True)
        assert info["status"] == 0, (compaction, info)
        check_cqk(x, inst, ref, tol)
        if compaction != "off":
            assert any(t["compacted"] for t in ctx.trace())


def test_theta_tuner_keeps_the_fastest_candidate(ctx):
    """The theta tuner solves the instance at every candidate, keeps the
    fastest in the context, and every candidate solves it exactly."""
    from paper_2603_15910_amd import _lib as L
    from paper_2603_15910_amd import CqkError
    inst = W.cqk_uniform(2_000_003, 31)
    ref = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    t = _dev(inst)
    assert ctx.compact_theta == 0.5
    try:
        theta, ms, times = ctx.tune_theta(*t, inst["r"], repeats=1)
        assert theta in L.THETA_CANDIDATES and ctx.compact_theta == theta
        assert sorted(times) == sorted(L.THETA_CANDIDATES)
        assert ms == times[theta] == min(times.values()) and ms > 0
        x, info = _solve(ctx, inst)
        assert info["status"] == 0
        check_cqk(x, inst, ref, 1e-10)
        for th in L.THETA_CANDIDATES:
            x, info = _solve(ctx, inst, theta=th, trace=True)
            assert info["status"] == 0, (th, info)
            check_cqk(x, inst, ref, 1e-10)
        with pytest.raises(CqkError):
            ctx.compact_theta = 0.0
        with pytest.raises(CqkError):
            ctx.compact_theta = 1.5
    finally:
        ctx.compact_theta = 0.5
