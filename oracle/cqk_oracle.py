"""Plain CPU FP64 oracle for the continuous quadratic knapsack problem (CQK).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The library's product
path never imports, links or calls anything here, and nothing here imports the
library.  Inputs come from the seeded generators in
``paper_2603_15910_amd.workloads`` (which hold none of the method's
arithmetic); every expected value is computed here, from the paper's
definitions, in FP64 (sums in extended precision).

Problem (paper, Section 1, eq. (CQK)):

    min_x  1/2 x^T D x - a^T x   s.t.  b^T x = r,  l <= x <= u,

with D = diag(d), d > 0, b > 0, l <= u (bounds may be infinite).

Functions and the passage each follows:

* ``breakpoints``       -- Section 2.1, breakpoint definitions.
* ``x_of_lambda``       -- Section 2.1, eq. (xopt).
* ``phi``               -- Section 2.1, eq. (opt).
* ``phi_slopes``        -- Section 2.1, eq. (phideriv).
* ``solve_cqk``         -- exact solution by the plain definition: phi is
                           piecewise linear and non-decreasing (eq. (opt)),
                           so sort the breakpoints, locate the piece on which
                           phi crosses r, and solve the linear equation there.
* ``project_simplex``   -- problem (proj_Delta), textbook sort-based solution
                           (the reference cited next to proj_Delta in Sec. 1).
* ``project_l1``        -- l1-ball projection, Section 3.2 and Lemma 1.
* ``solve_bruteforce``  -- enumeration of all active sets (tiny n only).
* ``kkt_residuals``     -- optimality conditions from the Lagrangian of the
                           dual in Section 2.1.
* ``condat_lambda0``    -- Algorithm 2 (Condat-style initial multiplier),
                           with the l1 test of Section 3.2.
* ``lambda_J``          -- eq. (lambdaJ).
* ``cqk_lambda0``       -- eq. (CQKlambda0), J = all indices.
* ``cqk_lambda0_warm``  -- the warm start of Section 2.1 from a primal
                           estimate: eq. (CQKlambda0) over the estimate's
                           free set, its bound-fixed indices on the right-hand
                           side.
* ``simplex_lambda0_warm`` -- the warm start of Section 3.1: Algorithm 2 over
                           the estimate's support, with the fallback given
                           there when no support index is used.
* ``newton_simplex``    -- Algorithm 4 (trace for invariant tests).
* ``newton_cqk``        -- Algorithm 1 with the stopping criteria of
                           Section 5 (trace for invariant tests).
* ``simplex_vjp``       -- vector-Jacobian product of the simplex projection
                           on its (fixed) support, from eq. (lambdaJ).
* ``cqk_vjp``           -- the same for general CQK, from eq. (xopt)/(opt).
* ``solve_cqk_batched``, ``cqk_vjp_batched`` -- plain loops over rows.
* ``spg_l1_lasso``      -- the l1-constrained least-squares problem of
                           Section 5.2 (basis pursuit) solved by the spectral
                           projected gradient method the paper uses there
                           (Birgin, Martinez and Raydan's SPG2: spectral step,
                           non-monotone line search), each projection by
                           ``project_l1``, started at the origin, stopped when
                           the infinity norm of the projected gradient falls
                           below the tolerance.

Readings of passages the paper leaves open are listed next to the code that
takes them.  Parity pins for every function live in ``tests/test_oracle_*``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

OK = "OK"
INFEASIBLE = "INFEASIBLE"
INVALID_ARG = "INVALID_ARG"
NOT_CONVERGED = "NOT_CONVERGED"

EPS64 = float(np.finfo(np.float64).eps)
EPS32 = float(np.finfo(np.float32).eps)


def _lsum(v) -> float:
    """Sum in x87 extended precision (64-bit mantissa), returned as float."""
    v = np.asarray(v, dtype=np.float64)
    if v.size == 0:
        return 0.0
    return float(np.sum(v, dtype=np.longdouble))


def _as64(*arrs):
    return [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in arrs]


# ---------------------------------------------------------------------------
# Input checks (Section 5: d > 0, b > 0, l <= u; Section 1: b > 0 assumed)
# ---------------------------------------------------------------------------
def validate(d, a, b, l, u, r) -> str:
    d, a, b, l, u = _as64(d, a, b, l, u)
    n = d.size
    if not all(x.size == n for x in (a, b, l, u)):
        return INVALID_ARG
    if not math.isfinite(float(r)):
        return INVALID_ARG
    if n == 0:
        return OK
    if not (np.all(np.isfinite(d)) and np.all(d > 0)):
        return INVALID_ARG
    if not (np.all(np.isfinite(b)) and np.all(b > 0)):
        return INVALID_ARG
    if not np.all(np.isfinite(a)):
        return INVALID_ARG
    if np.any(np.isnan(l)) or np.any(np.isnan(u)):
        return INVALID_ARG
    if np.any(l > u) or np.any(l == np.inf) or np.any(u == -np.inf):
        return INVALID_ARG
    return OK


# ---------------------------------------------------------------------------
# Section 2.1 definitions
# ---------------------------------------------------------------------------
def breakpoints(d, a, b, l, u):
    """lbar_i = (d_i l_i - a_i)/b_i and ubar_i = (d_i u_i - a_i)/b_i.

    An infinite bound gives an infinite breakpoint of the same sign."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    with np.errstate(invalid="ignore"):
        lbar = np.where(np.isfinite(l), (d * l - a) / b, -np.inf)
        ubar = np.where(np.isfinite(u), (d * u - a) / b, np.inf)
    return lbar, ubar


def x_of_lambda(lam, d, a, b, l, u):
    """eq. (xopt): x_i(lam) = max{l_i, min{u_i, (b_i lam + a_i)/d_i}}."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    t = (b * lam + a) / d
    return np.maximum(l, np.minimum(u, t))


def phi(lam, d, a, b, l, u) -> float:
    """eq. (opt): phi(lam) = b^T x(lam), summed in extended precision."""
    b64 = np.asarray(b, dtype=np.float64)
    return _lsum(b64 * x_of_lambda(lam, d, a, b, l, u))


def phi_slopes(lam, d, a, b, l, u):
    """eq. (phideriv): (phi'_+(lam), phi'_-(lam)).

    phi'_+ sums b_i^2/d_i over lbar_i <= lam < ubar_i,
    phi'_- sums it over lbar_i < lam <= ubar_i."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    lbar, ubar = breakpoints(d, a, b, l, u)
    w = b * b / d
    plus = _lsum(w[(lbar <= lam) & (lam < ubar)])
    minus = _lsum(w[(lbar < lam) & (lam <= ubar)])
    return plus, minus


def objective(x, d, a) -> float:
    x, d, a = _as64(x, d, a)
    return _lsum(0.5 * d * x * x - a * x)


# ---------------------------------------------------------------------------
# O1: exact breakpoint-sort CQK solver
# ---------------------------------------------------------------------------
@dataclass
class CQKResult:
    status: str
    x: np.ndarray | None = None
    lam: float = float("nan")
    unique: bool = True            # False when lam lies on a plateau of phi
    at_lower: np.ndarray | None = None
    at_upper: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def solve_cqk(d, a, b, l, u, r) -> CQKResult:
    """Exact solution of (CQK) from the plain definition.

    phi is piecewise linear and non-decreasing with kinks only at the
    breakpoints (Section 2.1), and x(lam) solves (CQK) exactly when
    phi(lam) = r (eq. (opt)).  So: sort the finite breakpoints, binary-search
    the piece [beta_j, beta_{j+1}] on which phi crosses r (phi evaluated from
    scratch at every probe, summed in extended precision), split the indices
    into L (at l), F (free) and U (at u) on the open piece, and solve the
    linear equation
        sum_L b_i l_i + sum_U b_i u_i + sum_F b_i (a_i + lam b_i)/d_i = r.
    If no index is free on that piece phi is flat there: every lam in it is
    optimal (the paper's Fig. 1(b) plateau) and the left end is returned with
    ``unique=False``; x is unique either way (strictly convex objective).
    """
    st = validate(d, a, b, l, u, r)
    if st != OK:
        return CQKResult(st)
    d, a, b, l, u = _as64(d, a, b, l, u)
    r = float(r)
    n = d.size
    if n == 0:
        if r == 0.0:
            return CQKResult(OK, np.zeros(0), 0.0, False, np.zeros(0, bool), np.zeros(0, bool))
        return CQKResult(INFEASIBLE)

    # Feasibility: b^T l <= r <= b^T u.
    smin = -math.inf if np.any(np.isinf(l)) else _lsum(b * l)
    smax = math.inf if np.any(np.isinf(u)) else _lsum(b * u)
    if r < smin or r > smax:
        return CQKResult(INFEASIBLE)

    lbar, ubar = breakpoints(d, a, b, l, u)
    bp = np.unique(np.concatenate([lbar[np.isfinite(lbar)], ubar[np.isfinite(ubar)]]))

    def phi_at(lam):
        return phi(lam, d, a, b, l, u)

    if bp.size == 0:
        left, right = -math.inf, math.inf
    elif phi_at(bp[0]) > r:
        left, right = -math.inf, float(bp[0])
    elif phi_at(bp[-1]) <= r:
        left, right = float(bp[-1]), math.inf
    else:
        lo, hi = 0, bp.size - 1           # phi(bp[lo]) <= r < phi(bp[hi])
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if phi_at(bp[mid]) <= r:
                lo = mid
            else:
                hi = mid
        left, right = float(bp[lo]), float(bp[hi])

    # Partition on the open piece (left, right): every breakpoint is <= left
    # or >= right, so these comparisons are exact.
    L = lbar >= right
    U = ubar <= left
    F = ~(L | U)
    w = b * b / d
    Q = _lsum(w[F])
    if math.isfinite(left) and phi_at(left) == r:
        lam = left
        x = x_of_lambda(lam, d, a, b, l, u)
        sp, sm = phi_slopes(lam, d, a, b, l, u)
        unique = (sp > 0) and (sm > 0)
        return CQKResult(OK, x, lam, unique, x <= l, x >= u)
    if Q > 0:
        num = (np.longdouble(r) - np.sum(b[L] * l[L], dtype=np.longdouble)
               - np.sum(b[U] * u[U], dtype=np.longdouble)
               - np.sum(b[F] * a[F] / d[F], dtype=np.longdouble))
        lam = float(num / np.longdouble(Q))
        unique = True
    else:
        lam = left if math.isfinite(left) else right
        unique = False
    x = np.empty(n)
    x[L] = l[L]
    x[U] = u[U]
    tF = (a[F] + lam * b[F]) / d[F]
    x[F] = np.minimum(u[F], np.maximum(l[F], tF))
    return CQKResult(OK, x, lam, unique, L.copy(), U.copy())


# ---------------------------------------------------------------------------
# O4: brute force over active sets (tiny n)
# ---------------------------------------------------------------------------
def solve_bruteforce(d, a, b, l, u, r, tol=1e-9):
    """Enumerate every assignment of each index to {at l, free, at u}.

    For an assignment with a free index, lam solves the linear equation
    b^T x = r; without one, the assignment must meet b^T x = r by itself and
    lam is any value consistent with it.  An assignment is kept when it is
    consistent with eq. (xopt): free => l <= t_i(lam) <= u, at l => t_i <= l,
    at u => t_i >= u.  Among kept assignments the one with the least objective
    is returned.  Plain Python floats, exponential in n: n <= 10 or so.
    Returns (x, lam) or None when nothing is feasible."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    n = d.size
    r = float(r)
    best = None
    choices = []
    for i in range(n):
        c = ["F"]
        if math.isfinite(l[i]):
            c.append("L")
        if math.isfinite(u[i]):
            c.append("U")
        choices.append(c)
    for assign in itertools.product(*choices):
        fixed = 0.0
        Q = 0.0
        s = 0.0
        for i, c in enumerate(assign):
            if c == "L":
                fixed += b[i] * l[i]
            elif c == "U":
                fixed += b[i] * u[i]
            else:
                Q += b[i] * b[i] / d[i]
                s += b[i] * a[i] / d[i]
        if Q > 0:
            lam_lo = lam_hi = (r - fixed - s) / Q
        else:
            if abs(fixed - r) > tol * (1.0 + abs(r)):
                continue
            # lam range on which every fixed index stays at its bound
            lam_lo, lam_hi = -math.inf, math.inf
            for i, c in enumerate(assign):
                if c == "L":
                    lam_hi = min(lam_hi, (d[i] * l[i] - a[i]) / b[i])
                else:
                    lam_lo = max(lam_lo, (d[i] * u[i] - a[i]) / b[i])
            if lam_lo > lam_hi + tol:
                continue
        lam = lam_lo if math.isfinite(lam_lo) else (lam_hi if math.isfinite(lam_hi) else 0.0)
        x = np.empty(n)
        ok = True
        for i, c in enumerate(assign):
            t = (a[i] + lam * b[i]) / d[i]
            scale = tol * (1.0 + abs(t) + abs(l[i] if math.isfinite(l[i]) else 0.0)
                           + abs(u[i] if math.isfinite(u[i]) else 0.0))
            if c == "L":
                ok &= t <= l[i] + scale
                x[i] = l[i]
            elif c == "U":
                ok &= t >= u[i] - scale
                x[i] = u[i]
            else:
                ok &= (l[i] - scale <= t <= u[i] + scale)
                x[i] = t
            if not ok:
                break
        if not ok:
            continue
        f = float(np.sum(0.5 * d * x * x - a * x))
        if best is None or f < best[0] - 1e-15 * (1 + abs(f)):
            best = (f, x, lam)
    if best is None:
        return None
    return best[1], best[2]


# ---------------------------------------------------------------------------
# O5: KKT residuals
# ---------------------------------------------------------------------------
def kkt_residuals(x, lam, d, a, b, l, u, r):
    """Optimality measures for (x, lam) from the Lagrangian in Section 2.1.

    The gradient of 1/2 x^T D x - a^T x - lam b^T x is g_i = d_i x_i - a_i -
    lam b_i.  At a minimiser over the box: g_i = 0 if l_i < x_i < u_i,
    g_i >= 0 if x_i = l_i, g_i <= 0 if x_i = u_i; and b^T x = r.
    Returns a dict with the feasibility residual |b^T x - r|, the largest bound
    violation and the largest sign/stationarity violation, each also scaled.
    """
    x, d, a, b, l, u = _as64(x, d, a, b, l, u)
    feas = abs(_lsum(b * x) - float(r))
    b1 = _lsum(np.abs(b))
    xinf = float(np.max(np.abs(x))) if x.size else 0.0
    with np.errstate(invalid="ignore"):
        bound = float(np.max(np.maximum(np.maximum(l - x, x - u), 0.0))) if x.size else 0.0
    g = d * x - a - lam * b
    gscale = d * np.abs(x) + np.abs(a) + abs(lam) * b
    at_l = x <= l
    at_u = x >= u
    free = ~(at_l | at_u)
    viol = np.zeros_like(g)
    viol[free] = np.abs(g[free])
    viol[at_l & ~at_u] = np.maximum(-g[at_l & ~at_u], 0.0)
    viol[at_u & ~at_l] = np.maximum(g[at_u & ~at_l], 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.where(gscale > 0, viol / gscale, viol)
    return {
        "feas_abs": feas,
        "feas_rel": feas / (b1 * xinf) if b1 * xinf > 0 else feas,
        "bound": bound,
        "stat_abs": float(np.max(viol)) if x.size else 0.0,
        "stat_rel": float(np.max(rel)) if x.size else 0.0,
    }


# ---------------------------------------------------------------------------
# O2, O3: simplex and l1-ball projections
# ---------------------------------------------------------------------------
def project_simplex(y, r=1.0):
    """Euclidean projection onto {x >= 0, sum x = r}, textbook sort method.

    Sort y decreasingly; k = max{j : y_(j) - (sum_{i<=j} y_(i) - r)/j > 0};
    tau = (sum_{i<=k} y_(i) - r)/k; x = max(0, y - tau).  In the CQK
    notation (D = I, a = y, b = 1, l = 0, u = inf) the multiplier is
    lam* = -tau.  Returns (x, lam*).  r = 0 gives x = 0."""
    y = np.asarray(y, dtype=np.float64)
    r = float(r)
    if not math.isfinite(r) or r < 0:
        raise ValueError("simplex radius must be finite and >= 0")
    n = y.size
    if n == 0:
        if r != 0:
            raise ValueError("empty simplex with r > 0 is infeasible")
        return np.zeros(0), 0.0
    s = np.sort(y)[::-1]
    cs = np.cumsum(s.astype(np.longdouble))
    j = np.arange(1, n + 1, dtype=np.longdouble)
    cond = s.astype(np.longdouble) - (cs - np.longdouble(r)) / j > 0
    if not np.any(cond):
        return np.zeros(n), -float(s[0])
    k = int(np.nonzero(cond)[0][-1]) + 1
    tau = float((cs[k - 1] - np.longdouble(r)) / np.longdouble(k))
    return np.maximum(y - tau, 0.0), -tau


def project_l1(y, radius=1.0):
    """Projection onto {x : sum |x_i| <= radius} (Section 3.2, Lemma 1).

    If y is in the ball it is its own projection (lam* = 0).  Otherwise
    x = sgn(y) * P_Delta(|y|), with sgn(0) = 0 as in the paper's notation,
    and lam* <= 0 is the simplex multiplier for |y|.  Returns (x, lam*)."""
    y = np.asarray(y, dtype=np.float64)
    radius = float(radius)
    if not math.isfinite(radius) or radius < 0:
        raise ValueError("l1 radius must be finite and >= 0")
    if _lsum(np.abs(y)) <= radius:
        return y.copy(), 0.0
    xa, lam = project_simplex(np.abs(y), radius)
    return np.sign(y) * xa, lam


# ---------------------------------------------------------------------------
# eq. (lambdaJ) and Algorithm 2
# ---------------------------------------------------------------------------
def lambda_J(y, r, J) -> float:
    """eq. (lambdaJ): lam_J = (r - sum_{i in J} y_i)/|J|."""
    J = np.asarray(list(J), dtype=np.int64)
    y = np.asarray(y, dtype=np.float64)
    return float((np.longdouble(r) - np.sum(y[J], dtype=np.longdouble)) / np.longdouble(J.size))


def condat_lambda0(y, r, I=None, l1=False):
    """Algorithm 2 run sequentially over the index list I (default 0..n-1).

    J starts as the first index with lam = r - y_{i1}; each later index j
    with y_j + lam > 0 gives the candidate lam' = (r - sum_J y - y_j)/(|J|+1);
    if lam' < r - y_j the index joins J (lam <- lam'), otherwise J is moved
    into the deferred set J~ and restarted as {j} with lam = r - y_j.  After
    the scan every deferred index with y_j + lam > 0 joins J.  The paper
    writes the sums over J with the index list notation; the reading used
    here is the plain sum over J.

    With ``l1=True`` the values are |y| and the membership test is
    min{|y_j|, |y_j| + lam} > 0 (Section 3.2); the scan starts at the first
    index with |y| > 0 (a reading: the paper does not say what to do when
    the first value is zero).

    Returns (lam, J as a list of indices).  lam equals lam_J for the
    returned J at every step, so lam >= lam* (Section 2.2)."""
    y = np.asarray(y, dtype=np.float64)
    v = np.abs(y) if l1 else y
    idx = list(range(y.size)) if I is None else [int(i) for i in I]
    if l1:
        idx = [i for i in idx if v[i] != 0.0] + [i for i in idx if v[i] == 0.0]

    def keep(val, lam):
        return min(val, val + lam) > 0 if l1 else val + lam > 0

    if not idx:
        return math.nan, []
    r = float(r)
    i1 = idx[0]
    J = [i1]
    S = float(v[i1])
    lam = r - S
    Jt = []
    for j in idx[1:]:
        vj = float(v[j])
        if keep(vj, lam):
            lam_new = (r - S - vj) / (len(J) + 1)
            if lam_new < r - vj:
                J.append(j)
                S += vj
                lam = lam_new
            else:
                Jt.extend(J)
                J = [j]
                S = vj
                lam = r - vj
    for j in Jt:
        vj = float(v[j])
        if keep(vj, lam):
            lam = (r - S - vj) / (len(J) + 1)
            J.append(j)
            S += vj
    return lam, J


def cqk_lambda0(d, a, b, l, u, r) -> float:
    """eq. (CQKlambda0) with J = all indices: the multiplier of the problem
    without bounds, (r - sum b a/d) / sum b^2/d."""
    d, a, b = _as64(d, a, b)
    return (float(r) - _lsum(b * a / d)) / _lsum(b * b / d)


def cqk_lambda0_warm(d, a, b, l, u, r, xbar) -> float:
    """Warm start of Section 2.1 from a primal estimate xbar.

    The indices strictly inside their bounds in xbar, J = {l < xbar < u}, are
    taken as free; an index at or beyond a bound in xbar is taken as fixed at
    that bound.  lam0 is then the multiplier of that guess:

        lam0 = (r - sum_{xbar <= l} b l - sum_{xbar >= u} b u - sum_J b a/d)
               / sum_J b^2/d.

    Reading: the paper applies eq. (CQKlambda0) with this J and calls the
    other indices "expected to have active bounds"; the printed formula has
    no term for them, and the reading here moves their b x (at the bound they
    reach) to the right-hand side, so that the estimate x* itself returns
    lam*.  With J empty xbar is discarded and J = all indices (plain
    eq. (CQKlambda0))."""
    d, a, b, l, u, xb = _as64(d, a, b, l, u, xbar)
    free = (xb > l) & (xb < u)
    if not free.any():
        return cqk_lambda0(d, a, b, l, u, r)
    at_l = (~free) & (xb <= l)
    at_u = (~free) & (xb >= u)
    fixed = _lsum(np.concatenate([b[at_l] * l[at_l], b[at_u] * u[at_u]]))
    s = _lsum(b[free] * a[free] / d[free])
    q = _lsum(b[free] * b[free] / d[free])
    return (float(r) - fixed - s) / q


def simplex_lambda0_warm(y, r, xbar, l1=False):
    """Warm start of Section 3.1: Algorithm 2 over I = {xbar > 0} (the
    support of the estimate; l1: {xbar != 0}), in index order.  When no
    index of I is used (I empty), lam0 = max{r/n, -max y}.

    Reading: the fallback is printed as max{r/n, -y_1}; -y_1 is read as
    -max_i y_i (l1: -max |y_i|), the lower bound of lam* that the section
    names, so lam0 >= that bound as stated there.

    Returns (lam0, J): J the indices Algorithm 2 used (empty on the
    fallback)."""
    y = np.asarray(y, dtype=np.float64)
    xb = np.asarray(xbar, dtype=np.float64)
    I = np.flatnonzero(xb != 0.0) if l1 else np.flatnonzero(xb > 0.0)
    lam, J = condat_lambda0(y, r, I=I, l1=l1) if I.size else (math.nan, [])
    if not J:
        v = np.abs(y) if l1 else y
        return max(float(r) / y.size, -float(np.max(v))), []
    return lam, J


# ---------------------------------------------------------------------------
# Algorithm 4 and Algorithm 1 traces (invariant tests only)
# ---------------------------------------------------------------------------
def newton_simplex(y, r, lam0, eps=EPS64, max_iter=200):
    """Algorithm 4 on (proj_Delta), with stopping criteria 2 and 3 of Sec. 5.

    Returns (lam_final, trace) where trace is a list of dicts with
    lam, phi, slope for each evaluated iterate (k = 0, 1, ...)."""
    y = np.asarray(y, dtype=np.float64)
    tol = eps ** 0.75
    ylow = -float(np.max(y))
    lam = max(float(lam0), ylow)

    def ev(lam):
        z = y + lam
        return _lsum(np.maximum(z, 0.0)), int(np.sum(z >= 0)), int(np.sum(z > 0))

    trace = []
    ph, cp, cm = ev(lam)
    trace.append({"lam": lam, "phi": ph, "cplus": cp, "cminus": cm})
    if ph == r:
        return lam, trace
    slope = cp if ph < r else cm
    step = (ph - r) / slope
    lam_prev, lam = lam, lam - step
    lo, hi = (lam_prev, math.inf) if ph < r else (-math.inf, lam_prev)
    for _ in range(max_iter):
        ph, cp, cm = ev(lam)
        trace.append({"lam": lam, "phi": ph, "cplus": cp, "cminus": cm})
        if ph <= r:
            break
        hi = lam
        step = (ph - r) / cm
        if abs(step) < tol:
            lam = lam - step
            break
        nxt = lam - step
        if nxt == lam:
            break
        if hi - lo < tol * max(abs(hi), abs(lo)):
            break
        lam = nxt
    return lam, trace


def newton_cqk(d, a, b, l, u, r, lam0=0.0, eps=EPS64, max_iter=200):
    """Algorithm 1 with the stopping criteria 1-3 of Section 5.

    Readings where the paper is silent:
    * criterion 2 uses the one-sided slope that the step uses, and is skipped
      when that slope is zero;
    * when criterion 2 fires the returned multiplier is lam_k - step (the step
      is already known), kept inside the bracket;
    * the closest breakpoint to the right of lam_lo is min{lbar_i > lam_lo}
      and to the left of lam_hi is max{ubar_i < lam_hi} (when the needed
      slope is zero no other breakpoint can be nearer).
    Returns (status, lam_final, trace)."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    r = float(r)
    tol = eps ** 0.75
    lbar, ubar = breakpoints(d, a, b, l, u)
    lo, hi = -math.inf, math.inf
    phlo = phhi = math.nan
    lam = float(lam0)
    lam_prev = math.nan
    trace = []
    for k in range(max_iter):
        x = x_of_lambda(lam, d, a, b, l, u)
        ph = _lsum(b * x)
        A = _lsum(np.abs(b * x))
        sp, sm = phi_slopes(lam, d, a, b, l, u)
        res = ph - r
        rec = {"lam": lam, "phi": ph, "splus": sp, "sminus": sm, "lo": lo, "hi": hi}
        trace.append(rec)
        if res == 0 or abs(res) < tol * (A + abs(r)):
            rec["stop"] = 1
            return OK, lam, trace
        if lam_prev == lam:
            rec["stop"] = 2
            return OK, lam, trace
        step = None
        if res < 0:
            lo, phlo = lam, ph
            if sp > 0:
                step = res / sp
                cand = lam - step
                nxt = cand if cand < hi else None
            else:
                right = lbar[lbar > lam]
                if right.size == 0:
                    return INFEASIBLE, lam, trace
                nxt = float(np.min(right))
                rec["kind"] = "breakpoint"
        else:
            hi, phhi = lam, ph
            if sm > 0:
                step = res / sm
                cand = lam - step
                nxt = cand if cand > lo else None
            else:
                left = ubar[ubar < lam]
                if left.size == 0:
                    return INFEASIBLE, lam, trace
                nxt = float(np.max(left))
                rec["kind"] = "breakpoint"
        if step is not None and abs(step) < tol:
            rec["stop"] = 2
            fin = min(max(lam - step, lo), hi)
            return OK, fin, trace
        if hi - lo < tol * max(abs(hi), abs(lo)):
            rec["stop"] = 3
            return OK, lam, trace
        if nxt is None:
            nxt = lo - (phlo - r) * (hi - lo) / (phhi - phlo)
            rec["kind"] = "secant"
        elif "kind" not in rec:
            rec["kind"] = "newton"
        lam_prev, lam = lam, nxt
    return NOT_CONVERGED, lam, trace


# ---------------------------------------------------------------------------
# O7: vector-Jacobian products
# ---------------------------------------------------------------------------
def simplex_vjp(x, g):
    """VJP of x = P_Delta(y; r) w.r.t. (y, r) at a point where the support
    S = {x_i > 0} is locally constant.

    On S, x_i = y_i + lam_J with J = S and lam_J = (r - sum_S y)/|S|
    (eq. (lambdaJ)), off S x_i = 0.  Hence dx_S/dy_S = I - 11^T/|S|,
    dx_S/dr = 1/|S|, and for an upstream gradient g:
        grad_y_i = [i in S](g_i - mean_S g),   grad_r = mean_S g.
    An empty support (only possible for r = 0) gives zeros."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    S = x > 0
    k = int(np.sum(S))
    if k == 0:
        return np.zeros_like(g), 0.0
    gbar = _lsum(g[S]) / k
    return np.where(S, g - gbar, 0.0), gbar


def cqk_vjp(x, g, d, b, l, u):
    """VJP of the CQK solution x*(a, r) w.r.t. (a, r) on a locally constant
    free set F = {l_i < x_i < u_i}.

    On F, x_i = (a_i + lam b_i)/d_i (eq. (xopt)); b^T x = r (eq. (opt)) gives
    lam = (r - sum_L b l - sum_U b u - sum_F b a/d) / sum_F b^2/d.  With
    q = sum_F b^2/d and mu = (sum_F g_i b_i/d_i)/q:
        grad_a_i = [i in F](g_i - b_i mu)/d_i,   grad_r = mu."""
    x, g, d, b, l, u = _as64(x, g, d, b, l, u)
    F = (x > l) & (x < u)
    q = _lsum((b * b / d)[F])
    if q == 0:
        return np.zeros_like(g), 0.0
    mu = _lsum((g * b / d)[F]) / q
    return np.where(F, (g - b * mu) / d, 0.0), mu


# ---------------------------------------------------------------------------
# Batched forms (a plain loop over rows)
# ---------------------------------------------------------------------------
def project_simplex_batched(values, offsets, r):
    """Row-by-row simplex projection; r is a scalar or one value per row."""
    values = np.asarray(values, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    nseg = offsets.size - 1
    rr = np.broadcast_to(np.asarray(r, dtype=np.float64), (nseg,))
    x = np.zeros_like(values)
    lam = np.zeros(nseg)
    for s in range(nseg):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            x[lo:hi], lam[s] = project_simplex(values[lo:hi], rr[s])
    return x, lam


def solve_cqk_batched(d, a, b, l, u, offsets, r):
    """Row-by-row solve_cqk; r has one value per row.  Returns the list of
    per-row CQKResult."""
    d, a, b, l, u = _as64(d, a, b, l, u)
    offsets = np.asarray(offsets, dtype=np.int64)
    r = np.asarray(r, dtype=np.float64)
    out = []
    for s in range(offsets.size - 1):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        out.append(solve_cqk(d[lo:hi], a[lo:hi], b[lo:hi], l[lo:hi], u[lo:hi], float(r[s])))
    return out


def cqk_vjp_batched(x, g, d, b, l, u, offsets):
    """Row-by-row cqk_vjp: (grad_a, grad_r per row)."""
    x, g, d, b, l, u = _as64(x, g, d, b, l, u)
    offsets = np.asarray(offsets, dtype=np.int64)
    nseg = offsets.size - 1
    ga = np.zeros_like(g)
    gr = np.zeros(nseg)
    for s in range(nseg):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            ga[lo:hi], gr[s] = cqk_vjp(x[lo:hi], g[lo:hi], d[lo:hi], b[lo:hi], l[lo:hi],
                                       u[lo:hi])
    return ga, gr


def simplex_vjp_batched(x, g, offsets):
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    nseg = offsets.size - 1
    ga = np.zeros_like(g)
    gr = np.zeros(nseg)
    for s in range(nseg):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            ga[lo:hi], gr[s] = simplex_vjp(x[lo:hi], g[lo:hi])
    return ga, gr


# ---------------------------------------------------------------------------
# SPG for the l1-constrained least-squares problem (Section 5.2, basis
# pursuit): min 1/2 ||A x - b||^2  s.t.  ||x||_1 <= radius
# ---------------------------------------------------------------------------
SPG_GAMMA = 1e-4     # sufficient decrease
SPG_SIGMA1 = 0.1     # safeguards of the quadratic interpolation
SPG_SIGMA2 = 0.9
SPG_LMIN = 1e-30     # spectral step bounds
SPG_LMAX = 1e30


def spg_l1_lasso(A, b, radius, tol=1e-4, max_iter=10000, memory=10):
    """The spectral projected gradient method (SPG2 of Birgin, Martinez and
    Raydan) on f(x) = 1/2 ||Ax - b||^2 over the l1 ball, as Section 5.2
    applies it: x_0 = 0; the step length of iteration k is the spectral
    (Barzilai-Borwein) quotient s's/s'y of the previous step, clipped to
    [1e-30, 1e30] (1e30 when s'y <= 0), the first one 1/||P(x_0 - g_0) -
    x_0||_inf; the direction d = P(x - lam g) - x; the non-monotone line
    search accepts t when f(x + t d) <= max of the last `memory` values of f
    + 1e-4 t g'd, else t becomes the minimiser of the quadratic through
    f(x), g'd and f(x + t d) if that lies in [0.1, 0.9 t], else t/2.  Stops
    when ||P(x - g) - x||_inf <= tol.

    f and g are formed from their definitions at every point (A x - b, then
    A^T of it).  Returns (x, info) with info: iterations, f, pg,
    projections, status ("OK" or "NOT_CONVERGED")."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[1]

    def f_of(x):
        res = A @ x - b
        return 0.5 * float(res @ res)

    def grad(x):
        return A.T @ (A @ x - b)

    def proj(v):
        return project_l1(v, radius)[0]

    x = proj(np.zeros(n))
    g = grad(x)
    fx = f_of(x)
    hist = [fx]
    pg = float(np.max(np.abs(proj(x - g) - x))) if n else 0.0
    lam = min(SPG_LMAX, max(SPG_LMIN, 1.0 / pg)) if pg > 0 else 1.0
    nproj = 2
    it = 0
    status = OK
    while pg > tol:
        if it >= max_iter:
            status = NOT_CONVERGED
            break
        d = proj(x - lam * g) - x
        nproj += 1
        gtd = float(g @ d)
        fmax = max(hist[-memory:])
        t = 1.0
        while True:
            fn = f_of(x + t * d)
            if fn <= fmax + SPG_GAMMA * t * gtd:
                break
            tq = -0.5 * t * t * gtd / (fn - fx - t * gtd)
            t = tq if (SPG_SIGMA1 <= tq <= SPG_SIGMA2 * t) else 0.5 * t
        s_ = t * d
        x = x + s_
        gn = grad(x)
        y_ = gn - g
        g = gn
        fx = fn
        hist.append(fx)
        sty = float(s_ @ y_)
        lam = SPG_LMAX if sty <= 0 else min(SPG_LMAX, max(SPG_LMIN, float(s_ @ s_) / sty))
        it += 1
        pg = float(np.max(np.abs(proj(x - g) - x)))
        nproj += 1
    return x, {"iterations": it, "f": fx, "pg": pg, "projections": nproj, "status": status}
