"""Seeded synthetic inputs for the CQK, simplex, l1 and batched workloads.

This module only draws random numbers (numpy's PCG64 via ``default_rng``).
It holds none of the method's arithmetic and is shared by the tests, the
benchmark and the smoke check so that the GPU path and the CPU oracle see
identical inputs.  Every generator is deterministic in (sizes, seed).

Recipes (the paper's own random classes are in Section 5.1.1 for CQK and
Section 5.2.1 for the simplex):

* ``cqk_uniform``     d ~ U[1,10], a ~ U[-10,10], b ~ U[1,10], l ~ U[-5,0],
                      u = l + U[0.1,5], r = b^T(l+u)/2 (always feasible).
* ``cqk_correlated``  b ~ U[1,10], a = b + U[-1,1], d = b * U[0.5,2],
                      l, u as above, r = b^T(l+u)/2.
* ``cqk_paper``       the paper's three classes on U[10,25]: uncorrelated,
                      weakly correlated, correlated; l/u are the min/max of
                      two U[10,25] draws and r ~ U[b^T l, b^T u].
* ``simplex_input``   y ~ N(0,1), U[0,1] or N(0, sigma=1e-3) (the paper does
                      not say whether 1e-3 is a variance or a deviation; it is
                      used as the deviation here); redrawn if any y_i == 0.
* ``segment_offsets`` row lengths round(exp(U[ln lo, ln hi])) (log-uniform).
* ``cqk_batched``     rows of log-uniform length (``segment_offsets``), the
                      values drawn as in ``cqk_uniform`` over all rows, and
                      r per row = b^T(l+u)/2 over the row (feasible).
* ``lasso_instance``  the l1-constrained least-squares problem of Section 5.2
                      with a random matrix in place of its test matrices:
                      A ~ N(0, 1/m) (m x n, row-major), a k-sparse x_true
                      with N(0,1) entries, b = A x_true + 0.01 N(0,1).
* ``perturbed``       v + eps * std(v) * N(0,1), the next point of an outer
                      loop whose previous projection serves as a warm start
                      (Section 3.1): for CQK only a is perturbed,
                      so r stays feasible.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def cqk_uniform(n: int, seed: int, dtype=np.float64):
    g = _rng(seed)
    d = g.uniform(1.0, 10.0, n).astype(dtype)
    a = g.uniform(-10.0, 10.0, n).astype(dtype)
    b = g.uniform(1.0, 10.0, n).astype(dtype)
    l = g.uniform(-5.0, 0.0, n).astype(dtype)
    u = (l.astype(np.float64) + g.uniform(0.1, 5.0, n)).astype(dtype)
    r = float(np.dot(b.astype(np.float64), (l.astype(np.float64) + u.astype(np.float64)) * 0.5))
    return {"d": d, "a": a, "b": b, "l": l, "u": u, "r": r}


def cqk_correlated(n: int, seed: int, dtype=np.float64):
    g = _rng(seed)
    b = g.uniform(1.0, 10.0, n)
    a = (b + g.uniform(-1.0, 1.0, n)).astype(dtype)
    d = (b * g.uniform(0.5, 2.0, n)).astype(dtype)
    l = g.uniform(-5.0, 0.0, n).astype(dtype)
    u = (l.astype(np.float64) + g.uniform(0.1, 5.0, n)).astype(dtype)
    b = b.astype(dtype)
    r = float(np.dot(b.astype(np.float64), (l.astype(np.float64) + u.astype(np.float64)) * 0.5))
    return {"d": d, "a": a, "b": b, "l": l, "u": u, "r": r}


def cqk_paper(n: int, seed: int, cls: str = "uncorrelated", dtype=np.float64):
    g = _rng(seed)
    b = g.uniform(10.0, 25.0, n)
    if cls == "uncorrelated":
        d = g.uniform(10.0, 25.0, n)
        a = g.uniform(10.0, 25.0, n)
    elif cls == "weak":
        d = b + g.uniform(-5.0, 5.0, n)
        a = b + g.uniform(-5.0, 5.0, n)
    elif cls == "correlated":
        d = b + 5.0
        a = b + 5.0
    else:
        raise ValueError(cls)
    p = g.uniform(10.0, 25.0, n)
    q = g.uniform(10.0, 25.0, n)
    l = np.minimum(p, q)
    u = np.maximum(p, q)
    lo = float(np.dot(b, l))
    hi = float(np.dot(b, u))
    r = float(g.uniform(lo, hi))
    out = {k: v.astype(dtype) for k, v in dict(d=d, a=a, b=b, l=l, u=u).items()}
    out["r"] = r
    return out


def simplex_input(n: int, seed: int, dist: str = "normal", dtype=np.float32):
    g = _rng(seed)
    while True:
        if dist == "normal":
            y = g.standard_normal(n)
        elif dist == "uniform":
            y = g.uniform(0.0, 1.0, n)
        elif dist == "normal_small":
            y = g.normal(0.0, 1e-3, n)
        else:
            raise ValueError(dist)
        y = y.astype(dtype)
        if not np.any(y == 0):
            return y


def segment_offsets(nseg: int, lo: int, hi: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    lens = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), nseg))).astype(np.int64)
    lens = np.clip(lens, lo, hi)
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def batched_simplex_input(nseg: int, lo: int, hi: int, seed: int, scale: float = 1.0,
                          dtype=np.float32):
    off = segment_offsets(nseg, lo, hi, seed)
    g = _rng(seed + 7919)
    y = (scale * g.standard_normal(int(off[-1]))).astype(dtype)
    return off, y


def upstream_grad(n: int, seed: int, dtype=np.float32):
    return _rng(seed + 104729).standard_normal(n).astype(dtype)


def cqk_batched(nseg: int, lo: int, hi: int, seed: int):
    """Returns (offsets, instance dict with r a float64 array per row)."""
    off = segment_offsets(nseg, lo, hi, seed)
    inst = cqk_uniform(int(off[-1]), seed + 31337)
    mid = inst["b"] * (inst["l"] + inst["u"]) * 0.5
    r = np.zeros(nseg)
    for s in range(nseg):
        r[s] = float(np.sum(mid[off[s]:off[s + 1]]))
    inst["r"] = r
    return off, inst


def perturbed(v, seed: int, eps: float = 1e-3):
    """v + eps * std(v) * N(0,1), in v's dtype."""
    v = np.asarray(v)
    g = _rng(seed + 15485863)
    sd = float(np.std(v.astype(np.float64))) if v.size else 0.0
    return (v.astype(np.float64) + eps * sd * g.standard_normal(v.size)).astype(v.dtype)


def cqk_perturbed(inst: dict, seed: int, eps: float = 1e-3) -> dict:
    """The instance with a replaced by perturbed(a, seed, eps)."""
    out = dict(inst)
    out["a"] = perturbed(inst["a"], seed, eps)
    return out


def lasso_instance(m: int, n: int, k: int, seed: int):
    """Returns (A, b, x_true); A float64 [m, n] row-major."""
    g = _rng(seed)
    A = g.standard_normal((m, n)) / np.sqrt(m)
    x_true = np.zeros(n)
    idx = g.choice(n, size=min(k, n), replace=False)
    x_true[idx] = g.standard_normal(idx.size)
    b = A @ x_true + 0.01 * g.standard_normal(m)
    return A, b, x_true
