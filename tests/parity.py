"""Comparison helpers for the GPU-vs-oracle parity tests.

Tolerances (FP64 1e-10, FP32 1e-5, relative) are applied as follows:
* S = max_i max(|x*_i|, |a_i|/d_i, |lam*| b_i/d_i)  (simplex: max(|x*|, |y|, |lam*|));
* max_i |x_i - x*_i| <= tol * S;
* |b^T x - r| <= tol * ||b||_1 ||x||_inf, summed in extended precision;
* the fixed/free partition equals the oracle's except at ties, an index
  being a tie when its oracle value is within 2 tol S of a bound.
"""
import numpy as np


def lsum(v):
    return float(np.sum(np.asarray(v, dtype=np.float64), dtype=np.longdouble))


def cqk_scale(inst, x_ref, lam_ref):
    d, a, b = (np.asarray(inst[k], dtype=np.float64) for k in "dab")
    lam = lam_ref if np.isfinite(lam_ref) else 0.0
    return float(max(np.max(np.abs(x_ref)), np.max(np.abs(a) / d), abs(lam) * np.max(b / d)))


def check_cqk(x, inst, ref, tol):
    """x: GPU result (numpy); inst: generator dict; ref: oracle CQKResult."""
    x = np.asarray(x, dtype=np.float64)
    d, a, b, l, u = (np.asarray(inst[k], dtype=np.float64) for k in "dablu")
    S = cqk_scale(inst, ref.x, ref.lam)
    err = float(np.max(np.abs(x - ref.x))) if x.size else 0.0
    assert err <= tol * S, f"max|x-x*| = {err:.3e} > {tol:.1e} * S (S = {S:.3e})"
    feas = abs(lsum(b * x) - inst["r"])
    bound = tol * lsum(np.abs(b)) * (float(np.max(np.abs(x))) if x.size else 0.0)
    assert feas <= max(bound, 1e-300), f"|b'x-r| = {feas:.3e} > {bound:.3e}"
    tie = np.minimum(np.abs(ref.x - l), np.abs(ref.x - u)) <= 2 * tol * S
    with np.errstate(invalid="ignore"):
        free_ref = (ref.x > l) & (ref.x < u)
        free_gpu = (x > l) & (x < u)
    mism = np.nonzero((free_ref != free_gpu) & ~tie)[0]
    assert mism.size == 0, f"partition differs at {mism[:10]} (of {mism.size})"
    return err / S if S > 0 else err


def simplex_scale(y, x_ref, lam_ref):
    y = np.asarray(y, dtype=np.float64)
    return float(max(np.max(np.abs(x_ref)), np.max(np.abs(y)), abs(lam_ref)))


def check_simplex(x, y, x_ref, lam_ref, r, tol, l1=False):
    x = np.asarray(x, dtype=np.float64)
    S = simplex_scale(y, x_ref, lam_ref)
    err = float(np.max(np.abs(x - x_ref))) if x.size else 0.0
    assert err <= tol * S, f"max|x-x*| = {err:.3e} > {tol:.1e} * {S:.3e}"
    if x.size:
        s = lsum(np.abs(x)) if l1 else lsum(x)
        target = min(r, lsum(np.abs(y))) if l1 else r
        assert abs(s - target) <= tol * x.size * float(np.max(np.abs(x))) + 1e-300, (s, target)
        tie = np.abs(np.asarray(x_ref)) <= 2 * tol * S
        mism = np.nonzero(((x_ref != 0) != (x != 0)) & ~tie)[0]
        assert mism.size == 0, f"support differs at {mism[:10]} (of {mism.size})"
    return err / S if S > 0 else err
