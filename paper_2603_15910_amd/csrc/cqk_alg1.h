// Algorithm 1 of the general CQK method in the per-index form
//     g_i(lam) = b_i x_i(lam) = min(max(c_i + lam s_i, b_i l_i), b_i u_i),
//     c_i = b_i a_i / d_i,  s_i = b_i^2 / d_i
// (eq. (xopt) times b_i > 0): the per-index terms of an evaluation and of the
// closest-breakpoint search, and the scalar update run after each, on a run
// state record.  Shared by the single-instance solver (one state in device
// memory, updated by one thread) and the batched solver (one state per row,
// updated redundantly by every lane of the wave or block that owns the row).
#pragma once

#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

// Partial record of an evaluation pass: NSUM sums.  A breakpoint pass writes
// two (key, weight) pairs instead.
//
// An evaluation at lam ends with one of two brackets: [lam, hi] when
// phi(lam) < r (side 0) or [lo, lam] when phi(lam) > r (side 1).  The pass
// does not know which until its sums are reduced, so it drops the indices
// each side's bracket resolves into that side's sums and writes each side's
// survivors to its own compacted set; the update keeps the side that
// happened.  Per side: D_* below, at P_SIDE + side * D_N.
enum {
  D_F = 0,   // bounds of the indices the side's bracket fixes
  D_AF,      // |bounds| of those
  D_C0,      // c of the indices free on the side's whole bracket
  D_C1,      // s of those
  D_A0,      // sgn * c of those
  D_A1,      // sgn * s of those
  D_NOUT,    // survivors written
  D_DROP,    // waves that gave the side up (more survivors than theta allows)
  D_N
};
enum {
  P_P = 0,     // sum g_i(lam)
  P_A,         // sum |g_i(lam)|
  P_QP,        // phi'_+ part
  P_QM,        // phi'_- part
  P_SIDE,      // side 0, then side 1 (2 * D_N values)
  P_NIN = P_SIDE + 2 * D_N,  // indices read
  P_BAD,       // indices failing the input checks
  NSUM
};
constexpr int NPART = NSUM;

// Compacted sets: the caller's arrays are source 0, the three compacted sets
// sources 1..3.  An evaluation reading source `src` writes side k's
// survivors to side_dst(src, k), the two sets other than src; passes over
// the caller's arrays leave set 3 alone, which is where the first pass
// writes the sampled-bracket set.
__device__ __host__ __forceinline__ int side_dst(int src, int side) {
  return (src + side) % 3 + 1;
}
constexpr int kSpecSet = 3;


struct Acc {
  double s[NSUM];
};

__device__ __forceinline__ void acc_init(Acc& a) {
#pragma unroll
  for (int i = 0; i < NSUM; ++i) a.s[i] = 0.0;
}

// Per-index form of the original data (eq. (xopt) times b), with the input
// checks of Section 5.
__device__ __forceinline__ void to_form(double d, double a, double b, double l, double u,
                                        double& c, double& s, double& bl, double& bu,
                                        double& bad) {
  const double inv = 1.0 / d;
  c = (b * a) * inv;
  s = (b * b) * inv;
  bl = b * l;
  bu = b * u;
  const bool ok = (d > 0.0) && (d < inf_d()) && (b > 0.0) && (b < inf_d()) &&
                  (fabs(a) < inf_d()) && (l <= u) && (l < inf_d()) && (u > -inf_d());
  bad += ok ? 0.0 : 1.0;
}

// Dropped-index sums of one side: fixed at l or at u on the side's whole
// bracket, or free on it with g keeping one sign (pos: g >= 0 there).
// Written as selects so the accumulators stay in registers.
__device__ __forceinline__ void side_sums(Acc& acc, int o, bool at_l, bool at_u, bool fr,
                                          double bl, double bu, double c, double s, bool pos) {
  const double fixv = at_l ? bl : (at_u ? bu : 0.0);
  acc.s[o + D_F] += fixv;
  acc.s[o + D_AF] += fabs(fixv);
  const double fc = fr ? c : 0.0, fs = fr ? s : 0.0;
  const double sg = pos ? 1.0 : -1.0;
  acc.s[o + D_C0] += fc;
  acc.s[o + D_C1] += fs;
  acc.s[o + D_A0] += sg * fc;
  acc.s[o + D_A1] += sg * fs;
}

// One index of an evaluation pass at lam with bracket [lo, hi].  With
// COMPACT, returns which sides keep the index (bit k: side k), after adding
// it to the sums of the sides that drop it; else returns 0.
template <bool COMPACT>
__device__ __forceinline__ int eval_index(Acc& acc, double c, double s, double bl, double bu,
                                          double lam, double lo, double hi) {
  const double f = fma(s, lam, c);
  const double g = fmin(fmax(f, bl), bu);
  acc.s[P_P] += g;
  acc.s[P_A] += fabs(g);
  const bool ge_l = f >= bl, gt_l = f > bl, lt_u = f < bu, le_u = f <= bu;
  acc.s[P_QP] += (ge_l && lt_u) ? s : 0.0;
  acc.s[P_QM] += (gt_l && le_u) ? s : 0.0;
  if (!COMPACT) return 0;
  const double fl = fma(s, lo, c);
  const double fh = fma(s, hi, c);
  int keep = 0;
  {  // side 0: [lam, hi]
    const bool at_l = fh <= bl, at_u = f >= bu;
    const bool fr = !at_l && !at_u && ge_l && (fh <= bu) && (f >= 0.0 || fh <= 0.0);
    side_sums(acc, P_SIDE, at_l, at_u, fr, bl, bu, c, s, f >= 0.0);
    keep |= (at_l || at_u || fr) ? 0 : 1;
  }
  {  // side 1: [lo, lam]
    const bool at_l = f <= bl, at_u = fl >= bu;
    const bool fr = !at_l && !at_u && (fl >= bl) && le_u && (fl >= 0.0 || f <= 0.0);
    side_sums(acc, P_SIDE + D_N, at_l, at_u, fr, bl, bu, c, s, fl >= 0.0);
    keep |= (at_l || at_u || fr) ? 0 : 2;
  }
  return keep;
}

// One index of the first evaluation pass classified on a bracket [p, q]
// estimated from a sample (not yet known to hold lam*): dropped into side 0's
// sums when its bound is active on all of [p, q] or it is free on all of it
// with g keeping one sign; returns 1 when kept.  The sums are exact for every
// lam strictly inside (p, q), wherever lam* is.
__device__ __forceinline__ int spec_index(Acc& acc, double c, double s, double bl, double bu,
                                          double p, double q) {
  const double fp = fma(s, p, c);
  const double fq = fma(s, q, c);
  const bool at_l = fq <= bl, at_u = fp >= bu;
  const bool fr = !at_l && !at_u && (fp >= bl) && (fq <= bu) && (fp >= 0.0 || fq <= 0.0);
  side_sums(acc, P_SIDE, at_l, at_u, fr, bl, bu, c, s, fp >= 0.0);
  return (at_l || at_u || fr) ? 0 : 1;
}

// Closest breakpoints around lam (Algorithm 1, breakpoint steps), with the
// slope that opens there.  The candidates are chosen with the same predicate
// the slopes use (an index below its lower bound at lam can only become free
// as lam grows), so an index that rounding left on the wrong side of a
// breakpoint equal to lam is still found (its key is then lam itself).
// Indices with l = u never become free and are skipped.
//   ks[0]: (min over candidates of max(lbar_i, lam), sum of s_i at that key)
//   ks[1]: (min of -min(ubar_i, lam), sum of s_i)  -- the left search
__device__ __forceinline__ void bkpt_index(KeySum* ks, double c, double s, double bl, double bu,
                                           double lam) {
  if (!(bl < bu)) return;
  const double f = fma(s, lam, c);
  if (f < bl) ks[0] = ks_min(ks[0], KeySum{fmax((bl - c) / s, lam), s});
  if (f > bu) ks[1] = ks_min(ks[1], KeySum{-fmin((bu - c) / s, lam), s});
}

__device__ __forceinline__ void trace_push(GenState* st, cqk_trace_rec* tr, int kind, int compacted, int source,
                           double lam, double phi, double slope, int64_t nin, int64_t nout) {
  if (st->ntrace < st->trace_cap) {
    cqk_trace_rec& t = tr[st->ntrace];
    t.iter = st->iter;
    t.kind = kind;
    t.compacted = compacted;
    t.source = source;
    t.lam = lam;
    t.phi = phi;
    t.slope = slope;
    t.lo = st->lo;
    t.hi = st->hi;
    t.n_in = nin;
    t.n_out = nout;
  }
  st->ntrace += 1;
}

__device__ __forceinline__ void finish(GenState* st, double lamf, int reason) {
  st->status = CQK_OK;
  st->lam_final = lamf;
  st->stop_reason = reason;
}

// A compacted set's dropped-index sums hold on a bracket [vlo, vhi]: for a
// set made from Algorithm 1's own bracket that bracket holds every later
// iterate; for the sampled-bracket set it need not.  The next evaluation at
// `next` keeps the current source only if next lies strictly inside, a
// breakpoint search only if Algorithm 1's whole bracket does (the breakpoint
// it looks for lies between the bracket end and lam*); otherwise the next
// pass reads the caller's arrays again.
__device__ __forceinline__ void to_caller_arrays(GenState* st) {
  st->src = 0;
  st->F = st->AF = st->C0 = st->C1 = st->A0 = st->A1 = 0.0;
  st->n_src = st->n_all;
  st->vlo = -inf_d();
  st->vhi = inf_d();
}
__device__ __forceinline__ void check_source_eval(GenState* st, double next) {
  if (st->src != 0 && !(next > st->vlo && next < st->vhi)) to_caller_arrays(st);
}
// Source of an evaluation at `next` once the sampled-bracket set exists: it
// replaces the caller's arrays, or a larger set just adopted, when next lies
// strictly inside its bracket.  It waits only while the passes read the
// caller's arrays (passes over a compacted set may overwrite it).  Returns
// whether it was taken.
__device__ __forceinline__ bool take_spec_set(GenState* st, double next) {
  if (!st->spend) return false;
  const bool inside = next > st->sp && next < st->sq;
  const bool take = inside && (st->src == 0 || st->sn < st->n_src);
  if (take) {
    st->F = st->sF;
    st->AF = st->sAF;
    st->C0 = st->sC0;
    st->C1 = st->sC1;
    st->A0 = st->sA0;
    st->A1 = st->sA1;
    st->src = kSpecSet;
    st->n_src = st->sn;
    st->vlo = st->sp;
    st->vhi = st->sq;
  }
  if (take || st->src != 0) st->spend = 0;
  return take;
}
__device__ __forceinline__ void check_source_bkpt(GenState* st) {
  if (st->src != 0 && !(st->vlo <= st->lo && st->hi <= st->vhi)) to_caller_arrays(st);
}

// Sides the next evaluation (at st->lam) need not write.  One the sample's
// estimate of lam* puts more than kSideSkip standard deviations on the far
// side of lam* will not happen but for a wrong estimate (which then only
// costs that pass's compaction).  One whose bracket covers more than
// kSkipShare * theta of the source's bracket would keep more than theta of
// a compacted source (its breakpoints taken as spread evenly over that
// bracket) and be given up, after some of its writes.
constexpr double kSideSkip = 4.0;
constexpr double kSkipShare = 1.25;
__device__ __forceinline__ void plan_sides(GenState* st) {
  const double lam = st->lam, slam = st->slam, ssd = st->ssd;
  int skip = ((lam > slam + kSideSkip * ssd) ? 1 : 0) | ((lam < slam - kSideSkip * ssd) ? 2 : 0);
  const double vw = st->vhi - st->vlo;
  if (st->src != 0 && vw > 0.0 && vw < inf_d()) {
    const double clo = fmax(st->lo, st->vlo), chi = fmin(st->hi, st->vhi);
    const double cap = kSkipShare * st->theta * vw;
    skip |= ((chi - lam) > cap) ? 1 : 0;
    skip |= ((lam - clo) > cap) ? 2 : 0;
  }
  st->skip = skip;
}

__device__ __forceinline__ void advance(GenState* st, double next) {
  st->lam_prev = st->lam;
  st->lam = next;
  st->mode = kModeEval;
  if (st->compaction != CQK_COMPACT_OFF) plan_sides(st);
  if (st->iter >= st->max_iter) {
    st->status = CQK_NOT_CONVERGED;
    st->lam_final = st->lam_prev;
  }
}

// The scalar part of Algorithm 1, run by one thread after an evaluation pass.
__device__ __forceinline__ void update_after_eval(GenState* st, const double* t, cqk_trace_rec* tr) {
  const double lam = st->lam;
  const int source = st->src;
  const double lo_in = st->lo, hi_in = st->hi;
  // the first pass wrote the sampled-bracket set in side 0's slot instead of
  // the two sides
  const bool spec = st->spec != 0;
  st->spec = 0;
  st->passes += 1;
  if (t[P_BAD] > 0.0) {
    st->status = CQK_INVALID_ARG;
    return;
  }
  if (spec && t[P_SIDE + D_DROP] == 0.0) {
    // every wave kept the sampled-bracket set: it waits in set 3
    st->sF = t[P_SIDE + D_F];
    st->sAF = t[P_SIDE + D_AF];
    st->sC0 = t[P_SIDE + D_C0];
    st->sC1 = t[P_SIDE + D_C1];
    st->sA0 = t[P_SIDE + D_A0];
    st->sA1 = t[P_SIDE + D_A1];
    st->sn = (int64_t)t[P_SIDE + D_NOUT];
    st->spend = 1;
  }
  // algorithmic bytes: the set read (caller's arrays or the 32-byte form) and
  // the survivors written for both sides
  const double nout = t[P_SIDE + D_NOUT] + t[P_SIDE + D_N + D_NOUT];
  st->bytes += ((source == 0) ? st->in_bytes : 32.0) * t[P_NIN] + 32.0 * nout;
  const double phi = (st->F + st->C0) + (lam * st->C1 + t[P_P]);
  const double A = (st->AF + st->A0) + (lam * st->A1 + t[P_A]);
  const double Qp = st->C1 + t[P_QP];
  const double Qm = st->C1 + t[P_QM];
  const double r0 = st->r;
  // the side the evaluation chose; its compacted set (if every wave kept it)
  // becomes the source of the next pass
  const int side = (phi - r0 < 0.0) ? 0 : 1;
  const int o = P_SIDE + side * D_N;
  const bool compacted =
      !spec && (st->compaction != CQK_COMPACT_OFF) && (phi != r0) && (t[o + D_DROP] == 0.0);
  if (compacted) {
    st->F += t[o + D_F];
    st->AF += t[o + D_AF];
    st->C0 += t[o + D_C0];
    st->C1 += t[o + D_C1];
    st->A0 += t[o + D_A0];
    st->A1 += t[o + D_A1];
    st->src = side_dst(source, side);
    st->n_src = (int64_t)t[o + D_NOUT];
    // the side's bracket, within the one the source's sums hold on
    st->vlo = (side == 0) ? lam : fmax(lo_in, st->vlo);
    st->vhi = (side == 0) ? fmin(hi_in, st->vhi) : lam;
  } else {
    st->n_src = (int64_t)t[P_NIN];
  }
  const double r = st->r, tol = st->tol;
  const double res = phi - r;
  // selects rather than branches, so the state stays in registers
  const double lo = (res < 0.0) ? lam : st->lo;
  const double hi = (res > 0.0) ? lam : st->hi;
  st->phi_lo = (res < 0.0) ? phi : st->phi_lo;
  st->phi_hi = (res > 0.0) ? phi : st->phi_hi;
  st->lo = lo;
  st->hi = hi;
  const double slope = (res < 0.0) ? Qp : Qm;
  const int ti = st->ntrace;
  trace_push(st, tr, 1, compacted ? 1 : 0, source, lam, phi, slope, (int64_t)t[P_NIN],
             (int64_t)nout);
  st->iter += 1;
  // Section 5 criterion 1 (and the exact stop of Algorithm 1)
  if (res == 0.0) return finish(st, lam, 4);
  if (fabs(res) < tol * (A + fabs(r))) return finish(st, lam, 1);
  // criterion 3
  if (hi - lo < tol * fmax(fabs(hi), fabs(lo))) return finish(st, lam, 3);
  double next;
  bool secant = false;
  if (slope > 0.0) {
    const double step = res / slope;
    if (fabs(step) < tol) return finish(st, fmin(fmax(lam - step, lo), hi), 2);  // criterion 2
    next = lam - step;
    secant = (res < 0.0) ? !(next < hi) : !(next > lo);
  } else {
    // slope zero: the closest breakpoint in the needed direction (the
    // sampled-bracket set is not used for it)
    st->mode = (res < 0.0) ? kModeBreakRight : kModeBreakLeft;
    if (st->src != 0) st->spend = 0;
    check_source_bkpt(st);
    return;
  }
  int kind = 3;  // the Newton step
  if (secant) {
    next = lo - (st->phi_lo - r) * (hi - lo) / (st->phi_hi - st->phi_lo);
    kind = 4;
    // rounding can put the secant point on an end of a bracket a few ulps
    // wide: bisect then
    if (!(next > lo && next < hi)) {
      next = 0.5 * (lo + hi);
      kind = 6;
    }
  }
  if (next == lam) return finish(st, lam, 2);  // criterion 2, lam_{k-1} = lam_k
  if (take_spec_set(st, next)) {
    if (tr != nullptr && ti < st->trace_cap) tr[ti].compacted = 1;
  } else {
    check_source_eval(st, next);
  }
  trace_push(st, tr, kind, 0, source, next, phi, slope, 0, 0);
  advance(st, next);
}

// Breakpoint step of Algorithm 1.  phi is constant between lam_k and the
// closest breakpoint bp (no index changes on that interval), so the next
// iterate lam_{k+1} = bp is evaluated without another pass: phi(bp) =
// phi(lam_k) and the one-sided slope at bp is the summed s of the indices
// whose breakpoint is bp.  The Newton step from bp follows as in Algorithm 1.
__device__ __forceinline__ void update_after_bkpt(GenState* st, const KeySum* ks, cqk_trace_rec* tr) {
  st->passes += 1;
  st->bytes += ((st->src == 0) ? st->in_bytes : 32.0) * (double)st->n_src;
  const bool right = st->mode == kModeBreakRight;
  const double bp = right ? ks[0].k : -ks[1].k;
  const double sw = right ? ks[0].w : ks[1].w;
  trace_push(st, tr, 2, 0, st->src, st->lam, bp, sw, (int64_t)st->n_src, 0);
  if (!(fabs(bp) < inf_d())) {
    st->status = CQK_INFEASIBLE;
    return;
  }
  const double phi = right ? st->phi_lo : st->phi_hi;
  const double r = st->r, tol = st->tol;
  const double res = phi - r;
  const double lo = right ? bp : st->lo, hi = right ? st->hi : bp;
  st->lo = lo;
  st->hi = hi;
  trace_push(st, tr, 5, 0, st->src, bp, phi, sw, 0, 0);
  st->iter += 1;
  st->lam_prev = st->lam;
  st->lam = bp;
  if (st->iter >= st->max_iter) {
    st->status = CQK_NOT_CONVERGED;
    st->lam_final = bp;
    return;
  }
  if (hi - lo < tol * fmax(fabs(hi), fabs(lo))) return finish(st, bp, 3);
  if (!(sw > 0.0)) {  // still flat past bp: search again from bp
    if (st->src != 0) st->spend = 0;
    check_source_bkpt(st);
    return;
  }
  const double step = res / sw;
  double next = bp - step;
  if (fabs(step) < tol) return finish(st, fmin(fmax(next, lo), hi), 2);
  int kind = 3;
  if (!(next > lo && next < hi)) {
    next = lo - (st->phi_lo - r) * (hi - lo) / (st->phi_hi - st->phi_lo);
    kind = 4;
    if (!(next > lo && next < hi)) {
      next = 0.5 * (lo + hi);
      kind = 6;
    }
  }
  if (next == bp) return finish(st, bp, 2);
  trace_push(st, tr, kind, 0, st->src, next, phi, sw, 0, 0);
  if (!take_spec_set(st, next)) check_source_eval(st, next);
  advance(st, next);
}

}  // namespace
}  // namespace cqk
