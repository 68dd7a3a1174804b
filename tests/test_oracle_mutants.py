"""Planted mistakes: every mutant of the oracle must fail at least one pin.

Each mutant is the oracle's source with one plausible slip (a dropped term,
a wrong sign, a transposed operand, an off-by-one index) compiled into a
throw-away module on the CPU.  The pins below are fast versions of the ones
in test_oracle_pins.py; a mutant that passes all of them would mean the pins
cannot see that kind of mistake.
"""
import json
import os
import sys
import types

import numpy as np
import pytest

from paper_2603_15910_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC_PATH = os.path.join(ROOT, "oracle", "cqk_oracle.py")


def _module(src, name):
    m = types.ModuleType(name)
    sys.modules[name] = m          # dataclasses look their module up here
    exec(compile(src, name, "exec"), m.__dict__)
    return m


def _mutant(old, new):
    src = open(SRC_PATH).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    return _module(src.replace(old, new, 1), "oracle_mutant")


def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "hand_examples.json")) as f:
        return json.load(f)


def _f(v):
    return np.array([float(t) for t in v])


def pin_golden(M):
    g = _golden()
    for ex in g["cqk"]:
        res = M.solve_cqk(*[_f(ex[k]) for k in "dablu"], ex["r"])
        if ex.get("status"):
            if res.status != "INFEASIBLE":
                return False
            continue
        if res.status != "OK" or np.max(np.abs(res.x - _f(ex["x"]))) > 1e-12:
            return False
        if ex["lam"] is not None and abs(res.lam - ex["lam"]) > 1e-12:
            return False
    for ex in g["simplex"]:
        x, lam = M.project_simplex(ex["y"], ex["r"])
        if np.max(np.abs(x - _f(ex["x"]))) > 1e-12 or abs(lam - ex["lam"]) > 1e-12:
            return False
    for ex in g["l1"]:
        x, lam = M.project_l1(ex["y"], ex["radius"])
        if np.max(np.abs(x - _f(ex["x"]))) > 1e-12:
            return False
    for ex in g["alg2"]:
        lam, J = M.condat_lambda0(ex["y"], ex["r"])
        if abs(lam - ex["lam"]) > 1e-12 or sorted(J) != ex["J"]:
            return False
    for ex in g["vjp"]:
        gy, gr = M.simplex_vjp(ex["x"], ex["g"])
        if np.max(np.abs(gy - _f(ex["grad_y"]))) > 1e-12 or abs(gr - ex["grad_r"]) > 1e-12:
            return False
    for ex in g["alg1_traces"]:
        st, lam, tr = M.newton_cqk(*[_f(ex[k]) for k in "dablu"], ex["r"], lam0=0.0)
        if st != "OK" or [t["lam"] for t in tr] != ex["lams"] or lam != ex["lam"]:
            return False
        if [t.get("kind") for t in tr] != ex["kinds"]:
            return False
    for ex in g["alg4_traces"]:
        lam, tr = M.newton_simplex(_f(ex["y"]), ex["r"], ex["lam0"])
        if [t["lam"] for t in tr] != ex["lams"] or lam != ex["lam"]:
            return False
    return True


def pin_bruteforce(M):
    rng = np.random.default_rng(1)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        d = rng.uniform(0.5, 3, n); a = rng.uniform(-3, 3, n); b = rng.uniform(0.5, 3, n)
        l = rng.uniform(-2, 0.5, n); u = l + rng.uniform(0, 2, n)
        r = float(rng.uniform(np.dot(b, l), np.dot(b, u)))
        res = M.solve_cqk(d, a, b, l, u, r)
        bf = M.solve_bruteforce(d, a, b, l, u, r)
        if bf is None or res.status != "OK" or np.max(np.abs(res.x - bf[0])) > 1e-9:
            return False
    return True


def pin_kkt(M):
    inst = W.cqk_uniform(3000, 1)
    args = [inst[k] for k in "dablu"]
    res = M.solve_cqk(*args, inst["r"])
    if res.status != "OK":
        return False
    k = M.kkt_residuals(res.x, res.lam, *args, inst["r"])
    return k["bound"] == 0 and k["feas_rel"] < 1e-13 and k["stat_rel"] < 1e-12


def pin_simplex_special_case(M):
    y = W.simplex_input(2000, 3, "normal", np.float64)
    n = y.size
    res = M.solve_cqk(np.ones(n), y, np.ones(n), np.zeros(n), np.full(n, np.inf), 1.0)
    x, _ = M.project_simplex(y, 1.0)
    if res.status != "OK" or np.max(np.abs(res.x - x)) > 1e-12:
        return False
    # variational inequality of a projection, from outside the module
    rng = np.random.default_rng(2)
    for _ in range(50):
        z = rng.dirichlet(np.full(n, 0.5))
        if np.dot(y - x, z - x) > 1e-10:
            return False
    return abs(x.sum() - 1.0) < 1e-12 and np.all(x >= 0)


def pin_condat(M):
    y = W.simplex_input(1500, 21, "normal", np.float64)
    # reference projection from outside the module: bisection on
    # sum max(0, y + lam) = 1
    lo, hi = -float(y.max()), -float(y.max()) + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.maximum(y + mid, 0).sum() > 1.0:
            hi = mid
        else:
            lo = mid
    lam_star = 0.5 * (lo + hi)
    for l1 in (False, True):
        lam0, J = M.condat_lambda0(y, 1.0, l1=l1)
        v = np.abs(y) if l1 else y
        lam_ref = lo if not l1 else None
        if not l1:
            if lam0 < lam_star - 1e-9:
                return False
            if abs(lam0 - (1.0 - v[J].sum()) / len(J)) > 1e-12:
                return False
        fixed = np.setdiff1d(np.arange(y.size), J)
        if not l1 and np.any(y[fixed] + lam_star > 1e-9):
            return False
    lam_n, tr = M.newton_simplex(y, 1.0, 0.0)
    if abs(lam_n - lam_star) > 1e-9:
        return False
    for k in range(1, len(tr) - 1):
        Jk = y + tr[k]["lam"] > 0
        if abs(tr[k + 1]["lam"] - (1.0 - y[Jk].sum()) / Jk.sum()) > 1e-10:
            return False
    S = np.nonzero(np.maximum(y + lam_star, 0) > 1e-9)[0]
    if abs(M.lambda_J(y, 1.0, S) - lam_star) > 1e-9:
        return False
    return True


def pin_slopes(M):
    inst = W.cqk_uniform(500, 17)
    args = [inst[k] for k in "dablu"]
    t = np.sort(np.concatenate([(inst["d"] * inst["l"] - inst["a"]) / inst["b"],
                                (inst["d"] * inst["u"] - inst["a"]) / inst["b"]]))
    for lam in (-2.0, 0.0, 1.5):
        h = 0.25 * np.min(np.abs(t - lam))
        sp, sm = M.phi_slopes(lam, *args)
        f = lambda z: float(np.dot(inst["b"], np.clip((inst["b"] * z + inst["a"]) / inst["d"], inst["l"], inst["u"])))
        if abs(sp - (f(lam + h) - f(lam)) / h) > 1e-6 * max(1, sp):
            return False
        if abs(sm - (f(lam) - f(lam - h)) / h) > 1e-6 * max(1, sm):
            return False
    return True


def pin_newton_cqk(M):
    inst = W.cqk_uniform(3000, 4)
    args = [inst[k] for k in "dablu"]
    st, lam, tr = M.newton_cqk(*args, inst["r"])
    if st != "OK":
        return False
    x = np.clip((inst["b"] * lam + inst["a"]) / inst["d"], inst["l"], inst["u"])
    return abs(float(np.dot(inst["b"], x)) - inst["r"]) < 1e-9 * float(np.sum(np.abs(inst["b"] * x)))


def pin_vjp_fd(M):
    rng = np.random.default_rng(13)
    y = 3.0 * rng.standard_normal(30)
    x, lam = M.project_simplex(y, 1.0)
    g = rng.standard_normal(30)
    gy, gr = M.simplex_vjp(x, g)
    h = 1e-6
    for i in range(30):
        e = np.zeros(30); e[i] = h
        fd = (np.dot(g, M.project_simplex(y + e, 1.0)[0]) - np.dot(g, M.project_simplex(y - e, 1.0)[0])) / (2 * h)
        if abs(gy[i] - fd) > 1e-7:
            return False
    inst = W.cqk_uniform(25, 15)
    d, a, b, l, u, r = (inst[k] for k in ("d", "a", "b", "l", "u", "r"))
    res = M.solve_cqk(d, a, b, l, u, r)
    ga, _ = M.cqk_vjp(res.x, g[:25], d, b, l, u)
    for i in range(25):
        e = np.zeros(25); e[i] = h
        fd = (np.dot(g[:25], M.solve_cqk(d, a + e, b, l, u, r).x)
              - np.dot(g[:25], M.solve_cqk(d, a - e, b, l, u, r).x)) / (2 * h)
        if abs(ga[i] - fd) > 1e-6:
            return False
    return True


def pin_warm(M):
    # warm starts from the exact solutions return lam*; the hand instance;
    # the fallbacks
    inst = W.cqk_uniform(400, 9)
    d, a, b, l, u, r = (inst[k] for k in ("d", "a", "b", "l", "u", "r"))
    res = M.solve_cqk(d, a, b, l, u, r)
    if abs(M.cqk_lambda0_warm(d, a, b, l, u, r, res.x) - res.lam) > 1e-11 * max(1, abs(res.lam)):
        return False
    dd = np.array([1.0, 2.0, 1.0]); aa = np.array([4.0, 2.0, -1.0]); bb = np.array([1.0, 1.0, 2.0])
    if M.cqk_lambda0_warm(dd, aa, bb, np.zeros(3), np.ones(3), 2.5, np.array([1.5, 0.5, -1.0])) != 1.0:
        return False
    if M.cqk_lambda0_warm(dd, aa, bb, np.zeros(3), np.ones(3), 2.5, np.array([1.0, 0.0, 1.0])) \
            != (2.5 - 3.0) / 5.5:
        return False
    y = W.simplex_input(1000, 9, "normal", np.float64)
    x, lam = M.project_simplex(y, 1.0)
    lam0, J = M.simplex_lambda0_warm(y, 1.0, x)
    if abs(lam0 - lam) > 1e-11 * max(1, abs(lam)) or sorted(J) != list(np.flatnonzero(x > 0)):
        return False
    yy = np.array([0.3, -0.2, 0.9, 0.1])
    lam0, J = M.simplex_lambda0_warm(yy, 1.0, np.array([0.0, -1.0, 0.0, 0.0]))
    if J or lam0 != 0.25:
        return False
    lam0, J = M.simplex_lambda0_warm(yy, 5.0, np.zeros(4))
    return lam0 == 1.25


def pin_spg(M):
    # A = I: the solution is the projection of b; an inactive ball: least
    # squares; the batched loops row by row
    rng = np.random.default_rng(65)
    bvec = rng.standard_normal(30)
    x, info = M.spg_l1_lasso(np.eye(30), bvec, 2.0, tol=1e-12)
    if np.max(np.abs(x - M.project_l1(bvec, 2.0)[0])) > 1e-10:
        return False
    A = rng.standard_normal((50, 12))
    bb = rng.standard_normal(50)
    x, info = M.spg_l1_lasso(A, bb, 1e3, tol=1e-11)
    if np.max(np.abs(x - np.linalg.lstsq(A, bb, rcond=None)[0])) > 1e-8:
        return False
    x, info = M.spg_l1_lasso(A, bb, 0.3, tol=1e-11)
    g = A.T @ (A @ x - bb)
    if np.max(np.abs(M.project_l1(x - g, 0.3)[0] - x)) > 1e-9 or np.sum(np.abs(x)) > 0.3 + 1e-12:
        return False
    off, inst = W.cqk_batched(5, 1, 40, 66)
    res = M.solve_cqk_batched(*[inst[k] for k in "dablu"], off, inst["r"])
    for s in range(5):
        lo, hi = off[s], off[s + 1]
        if abs(float(np.dot(inst["b"][lo:hi], res[s].x)) - inst["r"][s]) > 1e-10 * max(1, abs(inst["r"][s])):
            return False
    return True


PINS = [pin_golden, pin_bruteforce, pin_kkt, pin_simplex_special_case, pin_condat,
        pin_newton_cqk, pin_vjp_fd, pin_slopes, pin_warm, pin_spg]


def _survives(M):
    for p in PINS:
        try:
            if not p(M):
                return False
        except Exception:
            return False
    return True


def test_unmutated_oracle_passes_every_pin():
    M = _module(open(SRC_PATH).read(), "oracle_copy")
    for p in PINS:
        assert p(M), p.__name__


MUTANTS = [
    ("xopt sign", "t = (b * lam + a) / d", "t = (-b * lam + a) / d"),
    ("xopt transposed", "t = (b * lam + a) / d", "t = (d * lam + a) / b"),
    ("xopt clamp order", "np.maximum(l, np.minimum(u, t))", "np.minimum(l, np.maximum(u, t))"),
    ("breakpoint sign", "(d * l - a) / b", "(d * l + a) / b"),
    ("phi drops b", "return _lsum(b64 * x_of_lambda", "return _lsum(x_of_lambda"),
    ("slope weight", "w = b * b / d\n    plus", "w = b / d\n    plus"),
    ("solver drops U term", "- np.sum(b[U] * u[U], dtype=np.longdouble)", ""),
    ("solver F term sign", "- np.sum(b[F] * a[F] / d[F], dtype=np.longdouble))",
     "+ np.sum(b[F] * a[F] / d[F], dtype=np.longdouble))"),
    ("solver partition swapped", "L = lbar >= right\n    U = ubar <= left",
     "L = lbar >= left\n    U = ubar <= right"),
    ("simplex off by one", "k = int(np.nonzero(cond)[0][-1]) + 1", "k = int(np.nonzero(cond)[0][-1])"),
    ("simplex drops r", "tau = float((cs[k - 1] - np.longdouble(r))", "tau = float((cs[k - 1])"),
    ("simplex wrong cumsum index", "tau = float((cs[k - 1]", "tau = float((cs[k]"),
    ("l1 sign restore", "return np.sign(y) * xa, lam", "return xa, lam"),
    ("alg2 divisor", "lam_new = (r - S - vj) / (len(J) + 1)", "lam_new = (r - S - vj) / len(J)"),
    ("alg2 restart test", "if lam_new < r - vj:", "if lam_new > r - vj:"),
    ("alg2 second loop test", "for j in Jt:\n        vj = float(v[j])\n        if keep(vj, lam):",
     "for j in Jt:\n        vj = float(v[j])\n        if True:"),
    ("lambdaJ sign", "return float((np.longdouble(r) - np.sum(y[J]",
     "return float((np.longdouble(r) + np.sum(y[J]"),
    ("alg4 slope", "step = (ph - r) / cm\n", "step = (ph - r) / (cm + 1)\n"),
    ("alg1 farthest right breakpoint", "nxt = float(np.min(right))", "nxt = float(np.max(right))"),
    ("alg1 farthest left breakpoint", "nxt = float(np.max(left))", "nxt = float(np.min(left))"),
    ("alg1 right search over ubar", "right = lbar[lbar > lam]", "right = ubar[ubar > lam]"),
    ("alg1 left search over lbar", "left = ubar[ubar < lam]", "left = lbar[lbar < lam]"),
    ("alg1 secant through hi only", "nxt = lo - (phlo - r) * (hi - lo) / (phhi - phlo)",
     "nxt = hi - (phhi - r) * (hi - lo) / (phhi - phlo) * 0.5"),
    ("alg4 no safeguard", "lam = max(float(lam0), ylow)", "lam = float(lam0)"),
    ("alg1 newton sign", "cand = lam - step\n                nxt = cand if cand < hi", "cand = lam + step\n                nxt = cand if cand < hi"),
    ("vjp sign", "return np.where(S, g - gbar, 0.0), gbar", "return np.where(S, g + gbar, 0.0), gbar"),
    ("vjp mean", "gbar = _lsum(g[S]) / k", "gbar = _lsum(g[S]) / x.size"),
    ("cqk vjp drops d", "return np.where(F, (g - b * mu) / d, 0.0), mu", "return np.where(F, (g - b * mu), 0.0), mu"),
    ("kkt sign", "g = d * x - a - lam * b", "g = d * x - a + lam * b"),
    ("warm drops fixed term", "return (float(r) - fixed - s) / q", "return (float(r) - s) / q"),
    ("warm fixed at wrong bound", "fixed = _lsum(np.concatenate([b[at_l] * l[at_l], b[at_u] * u[at_u]]))",
     "fixed = _lsum(np.concatenate([b[at_l] * u[at_l], b[at_u] * l[at_u]]))"),
    ("warm free set closed", "free = (xb > l) & (xb < u)", "free = (xb >= l) & (xb <= u)"),
    ("warm support test", "I = np.flatnonzero(xb != 0.0) if l1 else np.flatnonzero(xb > 0.0)",
     "I = np.flatnonzero(xb != 0.0) if l1 else np.flatnonzero(xb >= 0.0)"),
    ("warm fallback", "return max(float(r) / y.size, -float(np.max(v))), []",
     "return max(float(r), -float(np.max(v))), []"),
    ("spg gradient sign", "return A.T @ (A @ x - b)", "return A.T @ (b - A @ x)"),
    ("spg direction", "d = proj(x - lam * g) - x", "d = proj(x + lam * g) - x"),
    ("spg stop test", "pg = float(np.max(np.abs(proj(x - g) - x)))\n        nproj",
     "pg = float(np.max(np.abs(proj(x) - x)))\n        nproj"),
    ("batched row slice", "out.append(solve_cqk(d[lo:hi], a[lo:hi], b[lo:hi], l[lo:hi], u[lo:hi], float(r[s])))",
     "out.append(solve_cqk(d[lo:hi], a[lo:hi], b[lo:hi], l[lo:hi], u[lo:hi], float(r[0])))"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    M = _mutant(old, new)
    assert not _survives(M), f"planted mistake '{name}' passes every pin"
