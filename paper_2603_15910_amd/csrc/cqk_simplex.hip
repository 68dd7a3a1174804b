// Simplex and l1-ball projections: Algorithm 4 (semismooth Newton for
// (proj_Delta)) started from a GPU mapping of Algorithm 2, with compaction of
// the indices already known to be zero at the solution.
//
// Paper: Section 2.2 (eq. (lambdaJ): any non-empty J gives lam_J >= lam*,
// Algorithm 2), Section 3 (Theorem 1, Algorithm 4, warm start and fixing),
// Section 3.2 (l1 ball, Lemma 1), Section 4 (Algorithm 2 per chunk, merged
// through the partial sums of each chunk), Section 5 (stopping criteria 2
// and 3).  In the notation of (CQK): D = I, a = y, b = 1, l = 0, u = +inf,
// x(lam) = max(0, y + lam), phi(lam) = sum max(0, y + lam),
// phi'_+(lam) = #{y + lam >= 0}, phi'_-(lam) = #{y + lam > 0}.
// For the l1 ball the same runs on |y| and x gets the signs of y back.
//
// Kernels:
//   spx_condat_kernel    one read of y: every thread runs Algorithm 2 on 16
//                        register-resident values; the block merges the
//                        thread sets (counts and sums) into lam_J bounds and
//                        keeps only values above every bound found; survivors
//                        (value, index) go to the block's region.  The last
//                        block merges all blocks: lam_0 and a prefix scan of
//                        the survivor counts.
//   spx_gather_kernel    packs the block regions into one dense array.
//   spx_formula_kernel   eq. (CQKlambda0) start: lam_0 = (r - sum y)/n, plus
//                        max y for the safeguard of Algorithm 4.
//   spx_iter_kernel      one evaluation of phi and the counts over the
//                        current set; drops y + lam_k <= 0 (valid because
//                        lam_k >= lam*, Theorem 1); Algorithm 4's update in
//                        the last block.
//   spx_finalize_kernel  dense x = max(0, y + lam*) (or 0, or a copy of y);
//   spx_scatter_kernel   x[idx] for the surviving indices when the rest of x
//                        is known to be zero.
#include <algorithm>
#include <cmath>

#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kRBlock = 1024;  // one-block reductions of partial records
constexpr int kWaves = kBlock / kWave;
constexpr int kCondatK = 16;  // values per thread per tile in Algorithm 2
constexpr int kRefine = 8;    // block refinement rounds per tile

struct SpxArgs {
  const void* y;
  void* x;
  int64_t n;
  int64_t chunk0;   // region size of the original layout
  void* val[2];     // compacted values (signed y), TIn
  uint32_t* idx[2]; // their indices in y
  int32_t* cnt[2];  // per-block counts of each buffer
  int64_t* offs;    // prefix of the Algorithm 2 survivor counts
  double* partials;
  SpxState* st;
  cqk_trace_rec* trace;
  int G0, G2;
};

template <typename T>
__device__ __forceinline__ T absval(T v) {
  return v < T(0) ? -v : v;
}

__device__ void spx_trace(SpxState* st, cqk_trace_rec* tr, int kind, int compacted, int source,
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

__device__ void spx_finish(SpxState* st, double lamf, int reason) {
  st->status = CQK_OK;
  st->lam_final = lamf;
  st->stop_reason = reason;
}

// ---------------------------------------------------------------------------
// Algorithm 2 on one thread's K values.  The paper's tests
//   y_j + lam > 0            with lam = (r - S)/|J|, and
//   lam' < r - y_j           with lam' = (r - S - y_j)/(|J| + 1)
// are used multiplied through by the positive counts, so the scan needs no
// division: c y_j + r - S > 0 and r - S - y_j < (c + 1)(r - y_j).
// l1: the value is |y| and the first test is min{|y|, |y| + lam} > 0
// (Section 3.2); the scan starts at the first non-zero value.
// Returns the membership mask of J and its count / sum.
// ---------------------------------------------------------------------------
template <int K, typename TA>
__device__ __forceinline__ uint32_t condat_thread(const TA* v, uint32_t active, TA r, bool l1,
                                                  int& c_out, TA& s_out) {
  uint32_t J = 0, Jt = 0;
  int c = 0;
  TA S = TA(0);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t bit = 1u << j;
    if (!(active & bit)) continue;
    const TA vj = v[j];
    if (c == 0) {
      if (l1 && !(vj > TA(0))) continue;
      J = bit;
      c = 1;
      S = vj;
      continue;
    }
    const bool keep = (!l1 || vj > TA(0)) && ((TA)c * vj + (r - S) > TA(0));
    if (keep) {
      if ((r - S - vj) < (TA)(c + 1) * (r - vj)) {
        J |= bit;
        S += vj;
        c += 1;
      } else {
        Jt |= J;
        J = bit;
        S = vj;
        c = 1;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t bit = 1u << j;
    if (Jt & bit) {
      const TA vj = v[j];
      const bool keep = (!l1 || vj > TA(0)) && ((TA)c * vj + (r - S) > TA(0));
      if (keep) {
        J |= bit;
        S += vj;
        c += 1;
      }
    }
  }
  c_out = c;
  s_out = S;
  return J;
}

// Loads V consecutive values of y starting at i (count-guarded).
template <typename TIn>
__device__ __forceinline__ void load_y(const TIn* y, int64_t i, int64_t n, TIn* o) {
  constexpr int V = VecWidth<TIn>::value;
  if (i + V <= n && aligned16(y + i)) {
    if constexpr (V == 4) {
      flt4 v = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(y + i));
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    } else {
      dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(y + i));
      o[0] = v.x;
      o[1] = v.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (i + k < n) ? y[i + k] : TIn(0);
  }
}

// Block-wide sum of one int and one double (thread 0 gets both, then
// broadcast through LDS).
__device__ __forceinline__ void block_sum_cs(int c, double s, double* lds, int* out_c,
                                             double* out_s) {
  double in[2] = {(double)c, s};
  double tot[2];
  __shared__ double bc[2];
  block_reduce<2, 0, 0, kBlock>(in, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    bc[0] = tot[0];
    bc[1] = tot[1];
  }
  __syncthreads();
  *out_c = (int)bc[0];
  *out_s = bc[1];
  __syncthreads();
}

// Partial record of the Algorithm 2 kernel.
enum { C_CNT = 0, C_SUM, C_ABS, C_BAD, C_NOUT, C_NSUM };  // + min lam, max v
constexpr int C_NPART = C_NSUM + 2;

template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_condat_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  constexpr int K = kCondatK;
  constexpr int NL = K / V;  // vector loads per thread per tile
  constexpr int64_t TILE = (int64_t)kBlock * K;
  const bool l1 = st->l1 != 0;
  const TA r = (TA)st->r;
  const double rd = st->r;
  const int64_t off = (int64_t)blockIdx.x * A.chunk0;
  const int64_t count = max((int64_t)0, min(A.chunk0, A.n - off));
  const TIn* y = (const TIn*)A.y + off;
  TIn* outv = (TIn*)A.val[1] + off;
  uint32_t* outi = A.idx[1] + off;

  __shared__ double lds[C_NPART * (kBlock / kWave)];
  __shared__ double tot[C_NPART];
  __shared__ int lds_i[kBlock / kWave + 1];

  double run_c = 0.0, run_s = 0.0;       // survivors kept so far by this block
  double lam_min = inf_d();              // smallest valid bound seen
  double acc[C_NSUM] = {0, 0, 0, 0, 0};
  double vmax = -inf_d();
  int64_t written = 0;
  for (int64_t base = 0; base < count; base += TILE) {
    TIn yv[K];
    TA v[K];
    uint32_t active = 0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t i = base + (int64_t)q * kBlock * V + (int64_t)threadIdx.x * V;
      load_y<TIn>(y, i, count, &yv[q * V]);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = q * V + k;
        const bool in = i + k < count;
        const TA t = (TA)yv[e];
        v[e] = l1 ? absval(t) : t;
        if (in) {
          active |= 1u << e;
          const double td = (double)yv[e];
          acc[C_ABS] += fabs(td);
          acc[C_BAD] += (fabs(td) < inf_d()) ? 0.0 : 1.0;
          vmax = fmax(vmax, (double)v[e]);
        }
      }
    }
    int c = 0;
    TA S = TA(0);
    const uint32_t J = condat_thread<K, TA>(v, active, r, l1, c, S);
    const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
    int ct;
    double skt;
    block_sum_cs(c, (double)S, lds, &ct, &skt);
    // Every lam below is lam_J of some non-empty J, hence >= lam*
    // (Section 2.2): the union of the thread sets, its union with the
    // block's earlier survivors, and the refinements
    //   lam <- lam_J'  with  J' = {j in J : y_j + lam > 0},
    // each of which can only lower lam (it is the Newton step of Algorithm 4
    // on the tile's own sub-problem).
    double lam_b = (ct > 0) ? (rd - skt) / (double)ct : inf_d();
    if (ct > 0 && run_c > 0.0) lam_b = fmin(lam_b, (rd - (skt + run_s)) / ((double)ct + run_c));
    if (run_c > 0.0) lam_b = fmin(lam_b, (rd - run_s) / run_c);
    uint32_t keep = 0;
    int nk = 0;
    double ks = 0.0;
    auto select = [&](double lam_blk) {
      const TA lt = (TA)fmin(lam_t, lam_blk);
      keep = 0;
      nk = 0;
      ks = 0.0;
#pragma unroll
      for (int e = 0; e < K; ++e) {
        if (((J >> e) & 1u) && (v[e] + lt > TA(0))) {
          keep |= 1u << e;
          ++nk;
          ks += (double)v[e];
        }
      }
    };
    for (int it = 0; it < kRefine; ++it) {
      select(lam_b);
      int kc;
      double kss;
      block_sum_cs(nk, ks, lds, &kc, &kss);
      if (kc == 0) break;
      double nl = (rd - kss) / (double)kc;
      if (run_c > 0.0) nl = fmin(nl, (rd - (kss + run_s)) / ((double)kc + run_c));
      if (!(nl < lam_b)) break;
      lam_b = nl;
    }
    select(lam_b);
    int total;
    const int pos0 = block_excl_scan<kBlock>(nk, lds_i, &total);
    int64_t pos = written + pos0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t i = base + (int64_t)q * kBlock * V + (int64_t)threadIdx.x * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = q * V + k;
        if ((keep >> e) & 1u) {
          outv[pos] = yv[e];
          outi[pos] = (uint32_t)(off + i + k);
          ++pos;
        }
      }
    }
    written += total;
    int kc;
    double kss;
    block_sum_cs(nk, ks, lds, &kc, &kss);
    run_c += (double)kc;
    run_s += kss;
    lam_min = fmin(lam_min, lam_b);
    if (run_c > 0.0) lam_min = fmin(lam_min, (rd - run_s) / run_c);
  }
  if (threadIdx.x == 0) {
    acc[C_CNT] = run_c;
    acc[C_SUM] = run_s;
    acc[C_NOUT] = (double)written;
    A.cnt[1][blockIdx.x] = (int32_t)written;
  } else {
    acc[C_CNT] = acc[C_SUM] = acc[C_NOUT] = 0.0;
  }
  double mn[1] = {lam_min};
  double mx[1] = {vmax};
  block_reduce<C_NSUM, 1, 1, kBlock>(acc, mn, mx, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, C_NPART);
  }
}

// Merges the blocks of spx_condat_kernel (one block): lam_0 from the union of
// the surviving sets, the smallest bound any block found, the l1 ball test,
// and the prefix of the survivor counts for the gather.
__global__ __launch_bounds__(kRBlock) void spx_condat_merge_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[C_NPART * (kRBlock / kWave)];
  __shared__ double tot[C_NPART];
  __shared__ int lds_i[kRBlock / kWave + 1];
  reduce_partials<C_NSUM, 1, 1, kRBlock>(A.partials, G, lds, tot);
  __shared__ int s_go;
  __shared__ int64_t s_m, s_ch;
  if (threadIdx.x == 0) {
    st->passes += 1;
    st->sum_abs = tot[C_ABS];
    st->vmax = tot[C_NSUM + 1];
    s_go = 0;
    if (tot[C_BAD] > 0.0) {
      st->status = CQK_INVALID_ARG;
    } else if (st->l1 && tot[C_ABS] <= st->r) {
      st->fin_mode = kFinCopy;
      spx_finish(st, 0.0, 5);
    } else {
      const double m = tot[C_CNT];
      double lam0 = (m > 0.0) ? (st->r - tot[C_SUM]) / m : 0.0;
      lam0 = fmin(lam0, tot[C_NSUM]);
      st->lam = lam0;
      st->lam0 = lam0;
      st->n_init = (int64_t)m;
      st->m = (int64_t)m;
      st->hi = lam0;
      int64_t ch = ((int64_t)m + (int64_t)A.G2 * kWaves - 1) / ((int64_t)A.G2 * kWaves);
      ch = (ch + 7) / 8 * 8;
      if (ch < 8) ch = 8;
      st->chunk_src = ch;
      st->src = 1;
      st->n_src = (int64_t)m;
      st->compact_next = (st->compaction != CQK_COMPACT_OFF) ? 1 : 0;
      s_m = (int64_t)m;
      s_ch = ch;
      s_go = 1;
    }
    spx_trace(st, A.trace, 0, 1, 0, st->lam, tot[C_SUM], tot[C_CNT], A.n, (int64_t)tot[C_NOUT]);
  }
  __syncthreads();
  if (!s_go) return;
  // exclusive scan of the per-block survivor counts, and the counts of the
  // dense layout the Newton passes read (G2 x 4 wave regions of chunk_src)
  int64_t base = 0;
  for (int g0 = 0; g0 < G; g0 += kRBlock) {
    const int g = g0 + threadIdx.x;
    const int cnt = (g < G) ? A.cnt[1][g] : 0;
    int totc;
    const int ex = block_excl_scan<kRBlock>(cnt, lds_i, &totc);
    if (g < G) A.offs[g] = base + ex;
    base += totc;
  }
  const int64_t m = s_m, ch = s_ch;
  for (int g = threadIdx.x; g < A.G2 * kWaves; g += kRBlock) {
    const int64_t s0 = (int64_t)g * ch;
    A.cnt[0][g] = (int32_t)max((int64_t)0, min(ch, m - s0));
  }
}

template <typename TIn>
__global__ __launch_bounds__(kBlock) void spx_gather_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  const int64_t off = (int64_t)blockIdx.x * A.chunk0;
  const int64_t cnt = A.cnt[1][blockIdx.x];
  const int64_t dst = A.offs[blockIdx.x];
  const TIn* sv = (const TIn*)A.val[1] + off;
  const uint32_t* si = A.idx[1] + off;
  TIn* dv = (TIn*)A.val[0] + dst;
  uint32_t* di = A.idx[0] + dst;
  for (int64_t i = threadIdx.x; i < cnt; i += kBlock) {
    dv[i] = sv[i];
    di[i] = si[i];
  }
}

// eq. (CQKlambda0) with J = all indices, D = I, b = 1: lam_0 = (r - sum y)/n,
// then lam_0 <- max(lam_0, -max y) (Algorithm 4, first line).
enum { F_SUM = 0, F_ABS, F_BAD, F_NSUM };
template <typename TIn>
__global__ __launch_bounds__(kBlock) void spx_formula_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  const bool l1 = st->l1 != 0;
  const int64_t off = (int64_t)blockIdx.x * A.chunk0;
  const int64_t count = max((int64_t)0, min(A.chunk0, A.n - off));
  const TIn* y = (const TIn*)A.y + off;
  double acc[F_NSUM] = {0, 0, 0};
  double vmax = -inf_d();
  for (int64_t i = (int64_t)threadIdx.x * V; i < count; i += (int64_t)kBlock * V) {
    TIn yv[V];
    load_y<TIn>(y, i, count, yv);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (i + k < count) {
        const double t = (double)yv[k];
        const double v = l1 ? fabs(t) : t;
        acc[F_SUM] += v;
        acc[F_ABS] += fabs(t);
        acc[F_BAD] += (fabs(t) < inf_d()) ? 0.0 : 1.0;
        vmax = fmax(vmax, v);
      }
    }
  }
  __shared__ double lds[(F_NSUM + 1) * (kBlock / kWave)];
  __shared__ double tot[F_NSUM + 1];
  block_reduce<F_NSUM, 0, 1, kBlock>(acc, nullptr, &vmax, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, F_NSUM + 1);
  }
}

__global__ __launch_bounds__(kRBlock) void spx_formula_update_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[(F_NSUM + 1) * (kRBlock / kWave)];
  __shared__ double tot[F_NSUM + 1];
  reduce_partials<F_NSUM, 0, 1, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->passes += 1;
    st->sum_abs = tot[F_ABS];
    st->vmax = tot[F_NSUM];
    if (tot[F_BAD] > 0.0) {
      st->status = CQK_INVALID_ARG;
    } else if (st->l1 && tot[F_ABS] <= st->r) {
      st->fin_mode = kFinCopy;
      spx_finish(st, 0.0, 5);
    } else {
      double lam0 = (st->r - tot[F_SUM]) / (double)A.n;
      lam0 = fmax(lam0, -tot[F_NSUM]);
      st->lam = lam0;
      st->lam0 = lam0;
      st->need_safeguard = 0;
    }
    spx_trace(st, A.trace, 0, 0, 0, st->lam, tot[F_SUM], (double)A.n, A.n, 0);
  }
}

// Partial record of an evaluation pass.
enum { S_PHI = 0, S_CM, S_CP, S_BAD, S_NIN, S_NOUT, S_ABS, S_NSUM };  // + max v

template <typename TA>
__device__ __forceinline__ void spx_eval(TA v, TA lam, TA& phi, double& cm, double& cp) {
  const TA z = v + lam;
  phi += z > TA(0) ? z : TA(0);
  cm += z > TA(0) ? 1.0 : 0.0;
  cp += z >= TA(0) ? 1.0 : 0.0;
}

// Algorithm 4's update, run by one thread after an evaluation pass.
__device__ void spx_update(SpxState* st, const double* t, double vmax, cqk_trace_rec* tr,
                           bool compacted, int source) {
  st->passes += 1;
  if (t[S_BAD] > 0.0) {
    st->status = CQK_INVALID_ARG;
    return;
  }
  const double lam = st->lam, r = st->r, tol = st->tol;
  const double phi = t[S_PHI], cm = t[S_CM], cp = t[S_CP];
  if (compacted) {
    st->src = (source == 1) ? 2 : 1;
    st->n_src = (int64_t)t[S_NOUT];
  } else {
    st->n_src = (int64_t)t[S_NIN];
  }
  if (!st->first_done) {
    st->first_done = 1;
    if (source == 0) {
      st->sum_abs = t[S_ABS];
      st->vmax = vmax;
      if (st->l1 && t[S_ABS] <= r) {
        st->fin_mode = kFinCopy;
        return spx_finish(st, 0.0, 5);
      }
    }
    // Algorithm 4, first line: lam_0 >= -max y, re-evaluated if it was not
    if (st->need_safeguard && lam < -st->vmax) {
      spx_trace(st, tr, 1, compacted, source, lam, phi, 0.0, (int64_t)t[S_NIN], 0);
      st->lam = -st->vmax;
      st->lam0 = st->lam;
      st->need_safeguard = 0;
      return;
    }
  }
  const int k = st->iter;
  st->iter += 1;
  double slope;
  if (k == 0 && phi < r) {
    slope = cp;
    st->lo = lam;
  } else {
    slope = cm;
    if (phi > r) st->hi = lam;
  }
  spx_trace(st, tr, 1, compacted, source, lam, phi, slope, (int64_t)t[S_NIN],
            compacted ? (int64_t)t[S_NOUT] : 0);
  if (phi == r) return spx_finish(st, lam, 4);
  if (k > 0 && phi <= r) return spx_finish(st, lam, 4);  // Algorithm 4 stop
  const double step = (phi - r) / slope;
  const double next = lam - step;
  if (fabs(step) < tol) return spx_finish(st, next, 2);
  if (k > 0 && cm == st->cm_prev) return spx_finish(st, next, 4);  // free set fixed
  if (next == lam) return spx_finish(st, lam, 2);
  if (st->hi - st->lo < tol * fmax(fabs(st->hi), fabs(st->lo))) return spx_finish(st, lam, 3);
  st->cm_prev = cm;
  st->lam_prev = lam;
  st->lam = next;
  // every later iterate is >= lam* (Theorem 1), so y + lam_k <= 0 fixes x at 0
  st->compact_next = (st->compaction != CQK_COMPACT_OFF) ? 1 : 0;
  if (st->iter >= st->max_iter) {
    st->status = CQK_NOT_CONVERGED;
    st->lam_final = lam;
  }
}

template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_pass_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  constexpr int E = 2 * V;
  constexpr int64_t TILE = (int64_t)kWave * E;
  const bool l1 = st->l1 != 0;
  const int src = st->src;
  const bool compact = st->compact_next != 0;
  const double lamd = st->lam;
  const TA lam = (TA)lamd;
  // every wave streams its own region rid (deterministic layout, no barriers)
  const int lane = threadIdx.x & (kWave - 1);
  const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
  const int64_t chunk = (src == 0) ? A.chunk0 / kWaves : st->chunk_src;
  const int64_t off = (int64_t)rid * chunk;
  int64_t count;
  const TIn* yv;
  const uint32_t* iv = nullptr;
  TIn* ov = nullptr;
  uint32_t* oi = nullptr;
  int32_t* ocnt = nullptr;
  if (src == 0) {
    count = max((int64_t)0, min(chunk, A.n - off));
    yv = (const TIn*)A.y + off;
  } else {
    const int si = src - 1;
    count = A.cnt[si][rid];
    yv = (const TIn*)A.val[si] + off;
    iv = A.idx[si] + off;
  }
  if (compact) {
    const int di = (src == 1) ? 1 : 0;
    ov = (TIn*)A.val[di] + off;
    oi = A.idx[di] + off;
    ocnt = A.cnt[di] + rid;
  }
  __shared__ double lds[(S_NSUM + 1) * (kBlock / kWave)];
  __shared__ double tot[S_NSUM + 1];
  TA phi = TA(0);
  double acc[S_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  double vmax = -inf_d();
  int64_t written = 0;
  for (int64_t base = 0; base < count; base += TILE) {
    TIn y[E];
    uint32_t id[E];
    bool keep[E];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
      load_y<TIn>(yv, i, count, &y[w * V]);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        keep[e] = false;
        if (i + k < count) {
          const TA t = (TA)y[e];
          const TA v = l1 ? absval(t) : t;
          spx_eval<TA>(v, lam, phi, acc[S_CM], acc[S_CP]);
          acc[S_NIN] += 1.0;
          if (src == 0) {
            const double td = (double)y[e];
            acc[S_ABS] += fabs(td);
            acc[S_BAD] += (fabs(td) < inf_d()) ? 0.0 : 1.0;
            vmax = fmax(vmax, (double)v);
          }
          keep[e] = compact && (v + lam > TA(0));
          if (compact) id[e] = (src == 0) ? (uint32_t)(off + i + k) : iv[i + k];
        }
      }
    }
    if (compact) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint64_t m = __ballot(keep[e]);
        if (keep[e]) {
          const int64_t pos = written + lane_prefix(m);
          ov[pos] = y[e];
          oi[pos] = id[e];
        }
        written += __popcll(m);
      }
    }
  }
  if (compact && lane == 0) {
    *ocnt = (int32_t)written;
    acc[S_NOUT] = (double)written;
  }
  // phi: reduced in the working precision TA (wave, then waves in order)
  TA phw = phi;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) phw += __shfl_xor(phw, o, kWave);
  __shared__ TA phl[kBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) phl[threadIdx.x / kWave] = phw;
  acc[S_PHI] = 0.0;
  block_reduce<S_NSUM, 0, 1, kBlock>(acc, nullptr, &vmax, lds, tot);
  if (threadIdx.x == 0) {
    TA pb = phl[0];
    for (int w = 1; w < kBlock / kWave; ++w) pb += phl[w];
    tot[S_PHI] = (double)pb;
    write_partial(A.partials, tot, S_NSUM + 1);
  }
}

// One block: phi summed in TA in block order, counts exactly in double, then
// Algorithm 4's update.
template <typename TA>
__global__ __launch_bounds__(kRBlock) void spx_update_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  const bool compact = st->compact_next != 0;
  const int src = st->src;
  __shared__ double lds[(S_NSUM + 1) * (kRBlock / kWave)];
  __shared__ double tot[S_NSUM + 1];
  __shared__ TA phl[kRBlock / kWave];
  TA pg = TA(0);
  for (int g = threadIdx.x; g < G; g += kRBlock)
    pg += (TA)A.partials[(size_t)S_PHI * G + g];
  reduce_partials<S_NSUM, 0, 1, kRBlock>(A.partials, G, lds, tot);
  TA pw = pg;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) pw += __shfl_xor(pw, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) phl[threadIdx.x / kWave] = pw;
  __syncthreads();
  if (threadIdx.x == 0) {
    TA pb = phl[0];
    for (int w = 1; w < kRBlock / kWave; ++w) pb += phl[w];
    tot[S_PHI] = (double)pb;
    SpxState sc = *st;  // register copy: one round trip to memory
    spx_update(&sc, tot, tot[S_NSUM], A.trace, compact, src);
    *st = sc;
  }
}

// Dense finalize over all n: x = max(0, y + lam) (l1: with the signs of y),
// or zeros (the scatter kernel then writes the survivors), or a copy of y.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_finalize_kernel(SpxArgs A) {
  SpxState* st = A.st;
  const int status = st->status;
  if (status != CQK_OK && status != CQK_NOT_CONVERGED) return;
  constexpr int V = VecWidth<TIn>::value;
  const int mode = st->fin_mode;
  const bool l1 = st->l1 != 0;
  const TA lam = (TA)st->lam_final;
  const int64_t off = (int64_t)blockIdx.x * A.chunk0;
  const int64_t count = max((int64_t)0, min(A.chunk0, A.n - off));
  const TIn* y = (const TIn*)A.y + off;
  TIn* x = (TIn*)A.x + off;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)threadIdx.x * V; i < count; i += (int64_t)kBlock * V) {
    TIn o[V];
    if (mode == kFinScatter || mode == kFinZero) {
#pragma unroll
      for (int k = 0; k < V; ++k) o[k] = TIn(0);
    } else {
      TIn yv[V];
      load_y<TIn>(y, i, count, yv);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        if (mode == kFinCopy) {
          o[k] = yv[k];
        } else {
          const TA t = (TA)yv[k];
          const TA v = l1 ? absval(t) : t;
          const TA z = v + lam;
          TA xv = z > TA(0) ? z : TA(0);
          if (l1 && t < TA(0)) xv = -xv;
          o[k] = (TIn)xv;
        }
        if (i + k < count) {
          acc[0] += fabs((double)o[k]);
          acc[1] += (o[k] != TIn(0)) ? 1.0 : 0.0;
        }
      }
    }
    if (i + V <= count && aligned16(x + i)) {
      if constexpr (V == 4) {
        flt4 w;
        w.x = o[0];
        w.y = o[1];
        w.z = o[2];
        w.w = o[3];
        __builtin_nontemporal_store(w, reinterpret_cast<flt4*>(x + i));
      } else {
        dbl2 w;
        w.x = o[0];
        w.y = o[1];
        __builtin_nontemporal_store(w, reinterpret_cast<dbl2*>(x + i));
      }
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (i + k < count) x[i + k] = o[k];
    }
  }
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, 2);
  }
}

// Totals of the finalize (dense modes) or of the scatter (scatter mode).
__global__ __launch_bounds__(kRBlock) void spx_fin_reduce_kernel(SpxArgs A, int G, int scatter) {
  SpxState* st = A.st;
  const int status = st->status;
  if (status != CQK_OK && status != CQK_NOT_CONVERGED) return;
  if ((st->fin_mode == kFinScatter) != (scatter != 0)) return;
  __shared__ double lds[2 * (kRBlock / kWave)];
  __shared__ double tot[2];
  reduce_partials<2, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->res_P = tot[0];
    st->n_free = (int64_t)tot[1];
  }
}

// x[idx] = max(0, v + lam) for the indices that survived every compaction;
// all other x are zero (written by the finalize kernel first).
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_scatter_kernel(SpxArgs A) {
  SpxState* st = A.st;
  const int status = st->status;
  if (status != CQK_OK && status != CQK_NOT_CONVERGED) return;
  if (st->fin_mode != kFinScatter) return;
  const bool l1 = st->l1 != 0;
  const TA lam = (TA)st->lam_final;
  const int si = st->src - 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
  const int64_t off = (int64_t)rid * st->chunk_src;
  const int64_t count = A.cnt[si][rid];
  const TIn* v = (const TIn*)A.val[si] + off;
  const uint32_t* iv = A.idx[si] + off;
  TIn* x = (TIn*)A.x;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = lane; i < count; i += kWave) {
    const TA t = (TA)v[i];
    const TA z = (l1 ? absval(t) : t) + lam;
    TA xv = z > TA(0) ? z : TA(0);
    if (l1 && t < TA(0)) xv = -xv;
    const TIn xo = (TIn)xv;
    x[iv[i]] = xo;
    acc[0] += fabs((double)xo);
    acc[1] += (xo != TIn(0)) ? 1.0 : 0.0;
  }
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, 2);
  }
}

// Marks the finalize mode once the Newton loop has stopped: the zero-fill +
// scatter form whenever the final set is a compacted one (every index left
// out of it is fixed at zero), the dense map otherwise.
__global__ void spx_pick_fin_kernel(SpxState* st) {
  if (st->fin_mode == kFinDense && st->src != 0) st->fin_mode = kFinScatter;
}

__global__ void spx_init_kernel(SpxState* st, SpxState init) { *st = init; }

int grid0(int64_t n, int num_cus) {
  const int64_t want = (n + 2047) / 2048;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cus * 8));
}

template <typename TIn, typename TA>
cqk_status run_simplex(cqk_ctx* ctx, int64_t n, const TIn* y, double r, TIn* x, bool l1,
                       const cqk_opts& o, cqk_info* info) {
  if (n > (int64_t)UINT32_MAX) return CQK_INVALID_ARG;
  const int G0i = grid0(n, ctx->num_cus);
  int64_t chunk0 = (n + G0i - 1) / G0i;
  chunk0 = (chunk0 + 31) / 32 * 32;  // wave regions of chunk0/4, multiples of 8
  const int G0 = (int)((n + chunk0 - 1) / chunk0);
  const int G2 = ctx->num_cus * 4;
  const int Gmax = std::max(G0, G2);
  const bool condat = o.lambda0_mode == CQK_LAMBDA0_CONDAT;
  const bool formula = o.lambda0_mode == CQK_LAMBDA0_FORMULA;

  const size_t part_bytes = ((size_t)Gmax * 8 * sizeof(double) + 255) / 256 * 256;
  const size_t cnt_bytes = ((size_t)2 * Gmax * kWaves * sizeof(int32_t) + 255) / 256 * 256;
  const size_t offs_bytes = ((size_t)(G0 + 1) * sizeof(int64_t) + 255) / 256 * 256;
  const size_t cap = (size_t)G0 * chunk0;
  const size_t val_bytes = (cap * sizeof(TIn) + 255) / 256 * 256;
  const size_t idx_bytes = (cap * sizeof(uint32_t) + 255) / 256 * 256;
  const bool need_bufs = (o.compaction != CQK_COMPACT_OFF) || condat;
  const size_t total = part_bytes + cnt_bytes + offs_bytes +
                       (need_bufs ? 2 * (val_bytes + idx_bytes) : 0);
  cqk_status stt = ensure_buffer(ctx->ws, total);
  if (stt != CQK_OK) return stt;
  stt = ensure_buffer(ctx->state, 1024 + sizeof(cqk_trace_rec) * kMaxTrace);
  if (stt != CQK_OK) return stt;

  char* ws = (char*)ctx->ws.ptr;
  SpxArgs A{};
  A.y = y;
  A.x = x;
  A.n = n;
  A.chunk0 = chunk0;
  A.partials = (double*)ws;
  A.cnt[0] = (int32_t*)(ws + part_bytes);
  A.cnt[1] = A.cnt[0] + Gmax * kWaves;
  A.offs = (int64_t*)(ws + part_bytes + cnt_bytes);
  if (need_bufs) {
    char* b = ws + part_bytes + cnt_bytes + offs_bytes;
    A.val[0] = b;
    A.idx[0] = (uint32_t*)(b + val_bytes);
    A.val[1] = b + val_bytes + idx_bytes;
    A.idx[1] = (uint32_t*)(b + 2 * val_bytes + idx_bytes);
  }
  A.st = (SpxState*)ctx->state.ptr;
  A.trace = (cqk_trace_rec*)((char*)ctx->state.ptr + 1024);
  A.G0 = G0;
  A.G2 = G2;

  const double eps = sizeof(TA) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  SpxState init{};
  init.lam = (o.lambda0_mode == CQK_LAMBDA0_USER) ? o.lambda0_user : 0.0;
  init.lam0 = init.lam;
  init.lam_prev = init.lam_final = __builtin_nan("");
  init.r = r;
  init.tol = (o.tol > 0.0) ? o.tol : std::pow(eps, 0.75);
  init.lo = -__builtin_huge_val();
  init.hi = __builtin_huge_val();
  init.cm_prev = -1.0;
  init.n_src = n;
  init.chunk_src = chunk0 / kWaves;
  init.status = kRunning;
  init.max_iter = o.max_iter;
  init.compaction = o.compaction;
  init.trace_cap = o.trace ? kMaxTrace : 0;
  init.l1 = l1 ? 1 : 0;
  init.fin_mode = kFinDense;
  init.need_safeguard = (!condat && !formula) ? 1 : 0;
  if (r == 0.0) {
    init.status = CQK_OK;
    init.fin_mode = kFinZero;
    init.lam_final = 0.0;
    init.stop_reason = 5;
  }

  hipStream_t s = ctx->stream;
  const size_t nev = (size_t)2 * (o.max_iter + 16);
  if (o.timing) {
    stt = ensure_events(ctx, nev);
    if (stt != CQK_OK) return stt;
  }
  hipLaunchKernelGGL(spx_init_kernel, dim3(1), dim3(1), 0, s, A.st, init);
  int ev = 0;
  auto launch = [&](auto kern, int grid) {
    const bool rec = o.timing && ev + 2 <= (int)nev;
    if (rec) hipEventRecord(ctx->events[ev], s);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, A);
    if (rec) {
      hipEventRecord(ctx->events[ev + 1], s);
      ev += 2;
    }
  };
  // one-block reduction of the partial records of a grid of `grid` blocks
  auto reduce = [&](auto kern, int grid) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(kRBlock), 0, s, A, grid);
  };
  int G = G0;
  if (r != 0.0) {
    if (condat) {
      launch(spx_condat_kernel<TIn, TA>, G0);
      reduce(spx_condat_merge_kernel, G0);
      launch(spx_gather_kernel<TIn>, G0);
      G = G2;
    } else if (formula) {
      launch(spx_formula_kernel<TIn>, G0);
      reduce(spx_formula_update_kernel, G0);
    }
    if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
    SpxState* hs = (SpxState*)ctx->host_pinned;
    int launched = 0;
    const int max_launch = o.max_iter + 2;
    int batch = 6;
    while (launched < max_launch) {
      const int k = std::min(batch, max_launch - launched);
      for (int i = 0; i < k; ++i) {
        launch(spx_pass_kernel<TIn, TA>, G);
        reduce(spx_update_kernel<TA>, G);
      }
      launched += k;
      if (hip_ok(hipMemcpyAsync(hs, A.st, sizeof(SpxState), hipMemcpyDeviceToHost, s)) != CQK_OK)
        return CQK_DEVICE_ERROR;
      if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
      if (hs->status != kRunning) break;
      batch = 4;
    }
  }
  const int work_events = ev;
  hipLaunchKernelGGL(spx_pick_fin_kernel, dim3(1), dim3(1), 0, s, A.st);
  launch(spx_finalize_kernel<TIn, TA>, G0);
  hipLaunchKernelGGL(spx_fin_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A, G0, 0);
  launch(spx_scatter_kernel<TIn, TA>, G);
  hipLaunchKernelGGL(spx_fin_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A, G, 1);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  SpxState* hs = (SpxState*)ctx->host_pinned;
  if (hip_ok(hipMemcpyAsync(hs, A.st, sizeof(SpxState), hipMemcpyDeviceToHost, s)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
  const int ntrace = std::min(hs->ntrace, init.trace_cap);
  ctx->last_trace.resize(ntrace);
  if (ntrace > 0 && hip_ok(hipMemcpy(ctx->last_trace.data(), A.trace,
                                     sizeof(cqk_trace_rec) * ntrace,
                                     hipMemcpyDeviceToHost)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  if (hs->status == kRunning) hs->status = CQK_NOT_CONVERGED;
  if (info) {
    info->status = hs->status;
    info->iterations = hs->iter;
    info->passes = hs->passes;
    info->stop_reason = hs->stop_reason;
    info->lambda = hs->lam_final;
    info->lambda0 = hs->lam0;
    const double target = (l1 && hs->fin_mode == kFinCopy) ? hs->sum_abs : r;
    info->residual = std::fabs(hs->res_P - target);
    info->abs_bx = hs->res_P;
    info->n_free = hs->n_free;
    info->n_after_init = hs->n_init;
    info->pass_bytes = 0.0;
    info->pass_ms = 0.0;
    info->finalize_ms = 0.0;
    const bool scatter = hs->fin_mode == kFinScatter;
    info->finalize_bytes = (double)n * sizeof(TIn) * ((scatter || hs->fin_mode == kFinZero) ? 1.0 : 2.0);
    for (int i = 0; i < ntrace; ++i) {
      const cqk_trace_rec& t = ctx->last_trace[i];
      const double per_in = (t.source == 0) ? (double)sizeof(TIn) : (double)sizeof(TIn) + 4.0;
      const double per_out = (double)sizeof(TIn) + 4.0;
      info->pass_bytes += per_in * (double)t.n_in + per_out * (double)t.n_out;
    }
    if (o.timing) {
      const int worked = std::min(hs->passes + (condat ? 1 : 0), work_events / 2);
      for (int i = 0; i < worked; ++i) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]);
        info->pass_ms += ms;
      }
      for (int j = 0; j < 2; ++j) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->events[work_events + 2 * j],
                            ctx->events[work_events + 2 * j + 1]);
        info->finalize_ms += ms;
      }
    }
  }
  return CQK_OK;
}

}  // namespace

cqk_status run_simplex_f32(cqk_ctx* ctx, int64_t n, const float* y, double r, float* x, bool l1,
                           const cqk_opts& o, cqk_info* info) {
  if (o.accum == CQK_ACCUM_F32) return run_simplex<float, float>(ctx, n, y, r, x, l1, o, info);
  return run_simplex<float, double>(ctx, n, y, r, x, l1, o, info);
}

cqk_status run_simplex_f64(cqk_ctx* ctx, int64_t n, const double* y, double r, double* x,
                           bool l1, const cqk_opts& o, cqk_info* info) {
  return run_simplex<double, double>(ctx, n, y, r, x, l1, o, info);
}

}  // namespace cqk
