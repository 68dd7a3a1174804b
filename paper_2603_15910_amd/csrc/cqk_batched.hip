// Batched simplex projections (many rows of uneven length in one launch) and
// the vector-Jacobian product of the projection.
//
// Per row the method is the one of the single-instance path: Algorithm 2 per
// thread chunk merged into lam_J bounds (Section 2.2 eq. (lambdaJ),
// Section 4), then Algorithm 4 from that start (Section 3, Theorem 1), then
// x = max(0, y + lam*).  The backward pass follows from eq. (lambdaJ) on a
// fixed support S = {x > 0}: lam* = (r - sum_S y)/|S|, so
//   dx_S/dy_S = I - 11^T/|S|,  dx_S/dr = 1/|S|,
//   grad_y = [x > 0](g - mean_S g),  grad_r = mean_S g.
//
// Schedule.  Rows are classified on the device by length: long rows (more
// than kSmallMax values) get a whole 256-thread workgroup, short rows one
// wave each (four per workgroup).  Long rows are listed by decreasing length
// bucket (longest first); one persistent kernel pulls work items from an
// atomic counter until the list is exhausted.  A long row is read once from
// HBM: each thread runs Algorithm 2 on 16 values per tile, the block refines
// the tile's bound and appends the surviving values to an LDS list; Newton
// runs on that list; x is then written densely (the row is re-read from
// cache; a row of one tile keeps its values in registers).  A short row
// stays in registers from load to store.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kK = 16;              // values per thread per tile (long rows)
constexpr int kTile = kBlock * kK;  // 4096
constexpr int kSmallPer = 8;        // values per lane (short rows)
constexpr int kSmallMax = kWave * kSmallPer;  // 512
constexpr int kLdsCap = 6144;       // survivor values kept in LDS per long row
constexpr int kNB = 24;             // length buckets (bucket 0: short rows)
constexpr int kRefine = 8;
constexpr int kMaxNewton = 100;

enum BatFlags : int32_t { kBadRadius = 1, kBadValue = 2, kInfeasible = 4 };

struct BatArgs {
  int32_t nseg;
  const int64_t* off;
  const float* y;
  const double* r;
  double r_scalar;
  float* x;
  double* lam_out;
  int32_t* nfree_out;
  const float* g;       // backward: upstream gradient
  float* gy;            // backward: grad_y
  double* gr;           // backward: grad_r
  int32_t* list;        // row ids: long rows by bucket, then short rows
  int32_t* counters;    // [0,kNB) counts, [kNB,2kNB) cursors, [2kNB,3kNB) bases,
                        // 3kNB: n_long, +1: n_short, +2: n_items, +3: queue, +4: flags,
                        // +5: ticket, +6: survivors total, +7: overflow rows
  double* partials;
};

constexpr int CTR_NLONG = 3 * kNB, CTR_NSHORT = 3 * kNB + 1, CTR_NITEMS = 3 * kNB + 2,
              CTR_QUEUE = 3 * kNB + 3, CTR_FLAGS = 3 * kNB + 4, CTR_TICKET = 3 * kNB + 5,
              CTR_SURV = 3 * kNB + 6, CTR_OVER = 3 * kNB + 7, CTR_TOTAL = 3 * kNB + 8;

__device__ __forceinline__ int bucket_of(int64_t L) {
  if (L <= kSmallMax) return 0;
  int b = 64 - __clzll((unsigned long long)L);  // bit length, >= 10 here
  b = b - 9;                                   // 1 .. for L > 512
  return b >= kNB ? kNB - 1 : b;
}

__global__ void bat_zero_kernel(int32_t* counters) {
  for (int i = threadIdx.x; i < CTR_TOTAL; i += blockDim.x) counters[i] = 0;
}

__global__ __launch_bounds__(kBlock) void bat_count_kernel(BatArgs A) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s < A.nseg) {
    const int64_t L = A.off[s + 1] - A.off[s];
    atomicAdd(&A.counters[bucket_of(L)], 1);
    __threadfence();
  }
  if (!last_block_arrives((uint32_t*)&A.counters[CTR_TICKET])) return;
  if (threadIdx.x == 0) {
    int base = 0;
    for (int b = kNB - 1; b >= 1; --b) {  // long rows, longest bucket first
      A.counters[2 * kNB + b] = base;
      base += A.counters[b];
    }
    A.counters[CTR_NLONG] = base;
    A.counters[2 * kNB + 0] = base;
    const int nshort = A.counters[0];
    A.counters[CTR_NSHORT] = nshort;
    A.counters[CTR_NITEMS] = base + (nshort + kWaves - 1) / kWaves;
    A.counters[CTR_TICKET] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void bat_place_kernel(BatArgs A) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= A.nseg) return;
  const int64_t L = A.off[s + 1] - A.off[s];
  const int b = bucket_of(L);
  const int pos = A.counters[2 * kNB + b] + atomicAdd(&A.counters[kNB + b], 1);
  A.list[pos] = s;
}

__device__ __forceinline__ double row_radius(const BatArgs& A, int s) {
  return A.r ? A.r[s] : A.r_scalar;
}

// Sum of an int and two doubles over the block; every thread gets the totals.
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* lds, double* o) {
  __shared__ double bc[3];
  double in[3] = {a, b, c};
  double tot[3];
  block_reduce<3, 0, 0, kBlock>(in, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    bc[0] = tot[0];
    bc[1] = tot[1];
    bc[2] = tot[2];
  }
  __syncthreads();
  o[0] = bc[0];
  o[1] = bc[1];
  o[2] = bc[2];
  __syncthreads();
}

__device__ __forceinline__ double wave_sum_d(double v) { return wave_sum(v); }

// Algorithm 2 over K values (division-free comparisons, see the simplex
// kernels): returns the J mask, its count and sum.
template <int K>
__device__ __forceinline__ uint32_t alg2(const float* v, uint32_t active, float r, int& c,
                                         float& S) {
  uint32_t J = 0, Jt = 0;
  c = 0;
  S = 0.f;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t bit = 1u << j;
    if (!(active & bit)) continue;
    const float vj = v[j];
    if (c == 0) {
      J = bit;
      c = 1;
      S = vj;
      continue;
    }
    if ((float)c * vj + (r - S) > 0.f) {
      if ((r - S - vj) < (float)(c + 1) * (r - vj)) {
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
    if ((Jt & bit) && ((float)c * v[j] + (r - S) > 0.f)) {
      J |= bit;
      S += v[j];
      c += 1;
    }
  }
  return J;
}

// ---------------------------------------------------------------------------
// One long row, whole workgroup.
// ---------------------------------------------------------------------------
__device__ void solve_long_row(const BatArgs& A, int s, double* lds, float* surv, int* lds_i) {
  const int64_t base = A.off[s];
  const int64_t L = A.off[s + 1] - base;
  const double rd = row_radius(A, s);
  const float* y = A.y + base;
  float* x = A.x + base;
  if (!(rd >= 0.0) || !(rd < inf_d())) {
    for (int64_t i = threadIdx.x; i < L; i += kBlock) x[i] = 0.f;
    if (threadIdx.x == 0) {
      atomicOr(&A.counters[CTR_FLAGS], kBadRadius);
      if (A.lam_out) A.lam_out[s] = __builtin_nan("");
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  const float r = (float)rd;
  const bool single = L <= kTile;
  double run_c = 0.0, run_s = 0.0, lam_min = inf_d(), bad = 0.0;
  int nsurv = 0;  // block-uniform
  bool overflow = false;
  float v[kK];
  for (int64_t t0 = 0; t0 < L; t0 += kTile) {
    uint32_t active = 0;
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) {
      const int64_t i = t0 + (int64_t)q * kBlock * 4 + (int64_t)threadIdx.x * 4;
      if (i + 4 <= L && aligned16(y + i)) {
        flt4 w = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(y + i));
        v[4 * q] = w.x;
        v[4 * q + 1] = w.y;
        v[4 * q + 2] = w.z;
        v[4 * q + 3] = w.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[4 * q + k] = (i + k < L) ? y[i + k] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i + k < L) {
          active |= 1u << (4 * q + k);
          bad += (fabsf(v[4 * q + k]) < __builtin_huge_valf()) ? 0.0 : 1.0;
        }
      }
    }
    int c;
    float S;
    const uint32_t J = alg2<kK>(v, active, r, c, S);
    const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
    double tt[3];
    block_sum3((double)c, (double)S, 0.0, lds, tt);
    double lam_b = (tt[0] > 0) ? (rd - tt[1]) / tt[0] : inf_d();
    if (tt[0] > 0 && run_c > 0) lam_b = fmin(lam_b, (rd - (tt[1] + run_s)) / (tt[0] + run_c));
    if (run_c > 0) lam_b = fmin(lam_b, (rd - run_s) / run_c);
    uint32_t keep = 0;
    int nk = 0;
    double ks = 0.0;
    auto select = [&](double lb) {
      const double lt = fmin(lam_t, lb);
      keep = 0;
      nk = 0;
      ks = 0.0;
#pragma unroll
      for (int e = 0; e < kK; ++e) {
        if (((J >> e) & 1u) && ((double)v[e] + lt > 0.0)) {
          keep |= 1u << e;
          ++nk;
          ks += (double)v[e];
        }
      }
    };
    for (int it = 0; it < kRefine; ++it) {
      select(lam_b);
      block_sum3((double)nk, ks, 0.0, lds, tt);
      if (tt[0] == 0.0) break;
      double nl = (rd - tt[1]) / tt[0];
      if (run_c > 0) nl = fmin(nl, (rd - (tt[1] + run_s)) / (tt[0] + run_c));
      if (!(nl < lam_b)) break;
      lam_b = nl;
    }
    select(lam_b);
    int total;
    const int p0 = block_excl_scan<kBlock>(nk, lds_i, &total);
    if (!overflow && nsurv + total <= kLdsCap) {
      int p = nsurv + p0;
#pragma unroll
      for (int e = 0; e < kK; ++e)
        if ((keep >> e) & 1u) surv[p++] = v[e];
      nsurv += total;
    } else {
      overflow = true;
    }
    block_sum3((double)nk, ks, 0.0, lds, tt);
    run_c += tt[0];
    run_s += tt[1];
    lam_min = fmin(lam_min, lam_b);
    if (run_c > 0) lam_min = fmin(lam_min, (rd - run_s) / run_c);
  }
  double tb[3];
  block_sum3(bad, 0.0, 0.0, lds, tb);
  if (tb[0] > 0.0 || L == 0 || rd == 0.0) {
    for (int64_t i = threadIdx.x; i < L; i += kBlock) x[i] = 0.f;
    if (threadIdx.x == 0) {
      if (tb[0] > 0.0) atomicOr(&A.counters[CTR_FLAGS], kBadValue);
      if (L == 0 && rd > 0.0) atomicOr(&A.counters[CTR_FLAGS], kInfeasible);
      if (A.lam_out) A.lam_out[s] = (tb[0] > 0.0 || L == 0) ? __builtin_nan("") : 0.0;
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  __syncthreads();  // survivors in LDS visible to every thread
  // Algorithm 4 from lam_0 >= lam*: lam_{k+1} = lam_J(J_k), J_k = {y + lam_k > 0}
  double lam = lam_min;
  double prev_c = -1.0;
  for (int it = 0; it < kMaxNewton; ++it) {
    double cc = 0.0, ss = 0.0, ph = 0.0;
    if (!overflow) {
      for (int i = threadIdx.x; i < nsurv; i += kBlock) {
        const double z = (double)surv[i] + lam;
        if (z > 0.0) {
          cc += 1.0;
          ss += (double)surv[i];
          ph += z;
        }
      }
    } else {
      for (int64_t i = threadIdx.x; i < L; i += kBlock) {
        const double yv = (double)y[i];
        const double z = yv + lam;
        if (z > 0.0) {
          cc += 1.0;
          ss += yv;
          ph += z;
        }
      }
    }
    double tt[3];
    block_sum3(cc, ss, ph, lds, tt);
    if (tt[0] == prev_c) break;
    if (it > 0 && tt[2] <= rd) break;
    if (tt[0] == 0.0) break;
    const double nl = (rd - tt[1]) / tt[0];
    if (!(nl < lam)) break;
    prev_c = tt[0];
    lam = nl;
  }
  // x = max(0, y + lam*), formed in FP64 and rounded once
  double nf = 0.0;
  if (single) {
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) {
      const int64_t i = (int64_t)q * kBlock * 4 + (int64_t)threadIdx.x * 4;
      float o[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        o[k] = (float)fmax((double)v[4 * q + k] + lam, 0.0);
        if (i + k < L) nf += (o[k] > 0.f) ? 1.0 : 0.0;
      }
      if (i + 4 <= L && aligned16(x + i)) {
        flt4 w;
        w.x = o[0];
        w.y = o[1];
        w.z = o[2];
        w.w = o[3];
        __builtin_nontemporal_store(w, reinterpret_cast<flt4*>(x + i));
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (i + k < L) x[i + k] = o[k];
      }
    }
  } else {
    for (int64_t i0 = (int64_t)threadIdx.x * 4; i0 < L; i0 += (int64_t)kBlock * 4) {
      if (i0 + 4 <= L && aligned16(y + i0) && aligned16(x + i0)) {
        flt4 w = *reinterpret_cast<const flt4*>(y + i0);
        w.x = (float)fmax((double)w.x + lam, 0.0);
        w.y = (float)fmax((double)w.y + lam, 0.0);
        w.z = (float)fmax((double)w.z + lam, 0.0);
        w.w = (float)fmax((double)w.w + lam, 0.0);
        nf += (w.x > 0.f) + (w.y > 0.f) + (w.z > 0.f) + (w.w > 0.f);
        __builtin_nontemporal_store(w, reinterpret_cast<flt4*>(x + i0));
      } else {
        for (int64_t i = i0; i < i0 + 4 && i < L; ++i) {
          const float o = (float)fmax((double)y[i] + lam, 0.0);
          nf += (o > 0.f) ? 1.0 : 0.0;
          x[i] = o;
        }
      }
    }
  }
  double tn[3];
  block_sum3(nf, 0.0, 0.0, lds, tn);
  if (threadIdx.x == 0) {
    if (A.lam_out) A.lam_out[s] = lam;
    if (A.nfree_out) A.nfree_out[s] = (int32_t)tn[0];
    atomicAdd(&A.counters[CTR_SURV], nsurv);
    if (overflow) atomicAdd(&A.counters[CTR_OVER], 1);
  }
}

// ---------------------------------------------------------------------------
// One short row (L <= 512), one wave, values in registers.
// ---------------------------------------------------------------------------
__device__ void solve_short_row(const BatArgs& A, int s) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t base = A.off[s];
  const int64_t L = A.off[s + 1] - base;
  const double rd = row_radius(A, s);
  const float* y = A.y + base;
  float* x = A.x + base;
  float v[kSmallPer];
  uint32_t active = 0;
  double bad = 0.0;
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int64_t i = (int64_t)k * kWave + lane;
    v[k] = (i < L) ? y[i] : 0.f;
    if (i < L) {
      active |= 1u << k;
      bad += (fabsf(v[k]) < __builtin_huge_valf()) ? 0.0 : 1.0;
    }
  }
  bad = wave_sum(bad);
  const bool bad_r = !(rd >= 0.0) || !(rd < inf_d());
  if (bad_r || bad > 0.0 || L == 0 || rd == 0.0) {
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int64_t i = (int64_t)k * kWave + lane;
      if (i < L) x[i] = 0.f;
    }
    if (lane == 0) {
      int f = 0;
      if (bad_r) f |= kBadRadius;
      if (bad > 0.0) f |= kBadValue;
      if (L == 0 && rd > 0.0) f |= kInfeasible;
      if (f) atomicOr(&A.counters[CTR_FLAGS], f);
      if (A.lam_out) A.lam_out[s] = (f) ? __builtin_nan("") : 0.0;
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  const float r = (float)rd;
  int c;
  float S;
  const uint32_t J = alg2<kSmallPer>(v, active, r, c, S);
  const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
  const double cw = wave_sum((double)c), sw = wave_sum((double)S);
  double lam_b = (cw > 0) ? (rd - sw) / cw : inf_d();
  // refinement on the wave's own sub-problem, then Algorithm 4 on the row
  uint32_t cand = J;
  for (int it = 0; it < kRefine; ++it) {
    const double lt = fmin(lam_t, lam_b);
    double nk = 0.0, ks = 0.0;
#pragma unroll
    for (int e = 0; e < kSmallPer; ++e)
      if (((cand >> e) & 1u) && (double)v[e] + lt > 0.0) {
        nk += 1.0;
        ks += (double)v[e];
      }
    nk = wave_sum(nk);
    ks = wave_sum(ks);
    if (nk == 0.0) break;
    const double nl = (rd - ks) / nk;
    if (!(nl < lam_b)) break;
    lam_b = nl;
  }
  // every value of the row is still in registers: run Algorithm 4 on all of it
  double lam = fmin(lam_b, wave_min(lam_t));
  double prev_c = -1.0;
  for (int it = 0; it < kMaxNewton; ++it) {
    double cc = 0.0, ss = 0.0, ph = 0.0;
#pragma unroll
    for (int e = 0; e < kSmallPer; ++e) {
      const double z = (double)v[e] + lam;
      if (((active >> e) & 1u) && z > 0.0) {
        cc += 1.0;
        ss += (double)v[e];
        ph += z;
      }
    }
    cc = wave_sum(cc);
    ss = wave_sum(ss);
    ph = wave_sum(ph);
    if (cc == prev_c) break;
    if (it > 0 && ph <= rd) break;
    if (cc == 0.0) break;
    const double nl = (rd - ss) / cc;
    if (!(nl < lam)) break;
    prev_c = cc;
    lam = nl;
  }
  double nf = 0.0;
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int64_t i = (int64_t)k * kWave + lane;
    if (i < L) {
      const float o = (float)fmax((double)v[k] + lam, 0.0);
      nf += (o > 0.f) ? 1.0 : 0.0;
      x[i] = o;
    }
  }
  nf = wave_sum(nf);
  if (lane == 0) {
    if (A.lam_out) A.lam_out[s] = lam;
    if (A.nfree_out) A.nfree_out[s] = (int32_t)nf;
  }
  (void)cand;
}

__global__ __launch_bounds__(kBlock) void bat_solve_kernel(BatArgs A) {
  __shared__ double lds[3 * kWaves];
  __shared__ float surv[kLdsCap];
  __shared__ int lds_i[kWaves + 1];
  __shared__ int s_item;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= nitems) break;
    if (item < nlong) {
      solve_long_row(A, A.list[item], lds, surv, lds_i);
    } else {
      const int k = (item - nlong) * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) solve_short_row(A, A.list[nlong + k]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Backward: grad_y = [x > 0](g - mean_S g), grad_r = mean_S g.
// ---------------------------------------------------------------------------
__device__ void vjp_long_row(const BatArgs& A, int s, double* lds) {
  const int64_t base = A.off[s];
  const int64_t L = A.off[s + 1] - base;
  const float* x = A.x + base;
  const float* g = A.g + base;
  float* gy = A.gy + base;
  const bool single = L <= kTile;
  float xs[kK], gs[kK];
  double cnt = 0.0, sum = 0.0;
  if (single) {
#pragma unroll
    for (int q = 0; q < kK; ++q) {
      const int64_t i = (int64_t)q * kBlock + threadIdx.x;
      xs[q] = (i < L) ? x[i] : 0.f;
      gs[q] = (i < L) ? g[i] : 0.f;
      if (xs[q] > 0.f) {
        cnt += 1.0;
        sum += (double)gs[q];
      }
    }
  } else {
    for (int64_t i0 = (int64_t)threadIdx.x * 4; i0 < L; i0 += (int64_t)kBlock * 4) {
      if (i0 + 4 <= L && aligned16(x + i0) && aligned16(g + i0)) {
        flt4 xv = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(x + i0));
        flt4 gv = *reinterpret_cast<const flt4*>(g + i0);
        if (xv.x > 0.f) { cnt += 1.0; sum += gv.x; }
        if (xv.y > 0.f) { cnt += 1.0; sum += gv.y; }
        if (xv.z > 0.f) { cnt += 1.0; sum += gv.z; }
        if (xv.w > 0.f) { cnt += 1.0; sum += gv.w; }
      } else {
        for (int64_t i = i0; i < i0 + 4 && i < L; ++i)
          if (x[i] > 0.f) { cnt += 1.0; sum += g[i]; }
      }
    }
  }
  double tt[3];
  block_sum3(cnt, sum, 0.0, lds, tt);
  const double gbar = (tt[0] > 0.0) ? tt[1] / tt[0] : 0.0;
  const float gb = (float)gbar;
  if (single) {
#pragma unroll
    for (int q = 0; q < kK; ++q) {
      const int64_t i = (int64_t)q * kBlock + threadIdx.x;
      if (i < L) gy[i] = (xs[q] > 0.f) ? gs[q] - gb : 0.f;
    }
  } else {
    for (int64_t i0 = (int64_t)threadIdx.x * 4; i0 < L; i0 += (int64_t)kBlock * 4) {
      if (i0 + 4 <= L && aligned16(x + i0) && aligned16(g + i0) && aligned16(gy + i0)) {
        flt4 xv = *reinterpret_cast<const flt4*>(x + i0);
        flt4 gv = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(g + i0));
        flt4 o;
        o.x = xv.x > 0.f ? gv.x - gb : 0.f;
        o.y = xv.y > 0.f ? gv.y - gb : 0.f;
        o.z = xv.z > 0.f ? gv.z - gb : 0.f;
        o.w = xv.w > 0.f ? gv.w - gb : 0.f;
        __builtin_nontemporal_store(o, reinterpret_cast<flt4*>(gy + i0));
      } else {
        for (int64_t i = i0; i < i0 + 4 && i < L; ++i) gy[i] = (x[i] > 0.f) ? g[i] - gb : 0.f;
      }
    }
  }
  if (threadIdx.x == 0 && A.gr) A.gr[s] = gbar;
}

__device__ void vjp_short_row(const BatArgs& A, int s) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t base = A.off[s];
  const int64_t L = A.off[s + 1] - base;
  float xs[kSmallPer], gs[kSmallPer];
  double cnt = 0.0, sum = 0.0;
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int64_t i = (int64_t)k * kWave + lane;
    xs[k] = (i < L) ? A.x[base + i] : 0.f;
    gs[k] = (i < L) ? A.g[base + i] : 0.f;
    if (xs[k] > 0.f) {
      cnt += 1.0;
      sum += (double)gs[k];
    }
  }
  cnt = wave_sum(cnt);
  sum = wave_sum(sum);
  const double gbar = (cnt > 0.0) ? sum / cnt : 0.0;
  const float gb = (float)gbar;
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int64_t i = (int64_t)k * kWave + lane;
    if (i < L) A.gy[base + i] = (xs[k] > 0.f) ? gs[k] - gb : 0.f;
  }
  if (lane == 0 && A.gr) A.gr[s] = gbar;
}

__global__ __launch_bounds__(kBlock) void bat_vjp_kernel(BatArgs A) {
  __shared__ double lds[3 * kWaves];
  __shared__ int s_item;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= nitems) break;
    if (item < nlong) {
      vjp_long_row(A, A.list[item], lds);
    } else {
      const int k = (item - nlong) * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) vjp_short_row(A, A.list[nlong + k]);
    }
    __syncthreads();
  }
}

struct BatWs {
  int32_t* list;
  int32_t* counters;
  double* partials;
};

cqk_status bat_workspace(cqk_ctx* ctx, int32_t nseg, BatWs* w) {
  const size_t list_bytes = ((size_t)nseg * sizeof(int32_t) + 255) / 256 * 256;
  const size_t ctr_bytes = 256 * sizeof(int32_t);
  cqk_status st = ensure_buffer(ctx->ws, list_bytes + ctr_bytes);
  if (st != CQK_OK) return st;
  char* p = (char*)ctx->ws.ptr;
  w->list = (int32_t*)p;
  w->counters = (int32_t*)(p + list_bytes);
  w->partials = nullptr;
  return CQK_OK;
}

int persistent_grid(cqk_ctx* ctx, int items) {
  const int g = ctx->num_cus * 4;
  return std::max(1, std::min(g, items));
}

void plan(cqk_ctx* ctx, const BatArgs& A) {
  hipStream_t s = ctx->stream;
  hipLaunchKernelGGL(bat_zero_kernel, dim3(1), dim3(256), 0, s, A.counters);
  const int gb = (A.nseg + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(bat_count_kernel, dim3(gb), dim3(kBlock), 0, s, A);
  hipLaunchKernelGGL(bat_place_kernel, dim3(gb), dim3(kBlock), 0, s, A);
}

}  // namespace

cqk_status run_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const float* y,
                           const double* r, double r_scalar, float* x, double* lambda_out,
                           int32_t* nfree_out, const cqk_opts& o, cqk_info* info) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  BatArgs A{};
  A.nseg = nseg;
  A.off = offsets;
  A.y = y;
  A.r = r;
  A.r_scalar = r_scalar;
  A.x = x;
  A.lam_out = lambda_out;
  A.nfree_out = nfree_out;
  A.list = w.list;
  A.counters = w.counters;
  hipStream_t s = ctx->stream;
  if (o.timing) {
    st = ensure_events(ctx, 2);
    if (st != CQK_OK) return st;
    hipEventRecord(ctx->events[0], s);
  }
  plan(ctx, A);
  // items <= nseg, so a grid of min(persistent size, nseg) covers them
  hipLaunchKernelGGL(bat_solve_kernel, dim3(persistent_grid(ctx, nseg)), dim3(kBlock), 0, s, A);
  if (o.timing) hipEventRecord(ctx->events[1], s);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  if (info) std::memset(info, 0, sizeof(*info));
  if (!o.sync) {
    if (info) info->status = CQK_OK;
    return CQK_OK;
  }
  int32_t* hc = (int32_t*)ctx->host_pinned;
  if (hip_ok(hipMemcpyAsync(hc, A.counters, CTR_TOTAL * sizeof(int32_t), hipMemcpyDeviceToHost,
                            s)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
  const int flags = hc[CTR_FLAGS];
  int status = CQK_OK;
  if (flags & (kBadRadius | kBadValue)) status = CQK_INVALID_ARG;
  else if (flags & kInfeasible) status = CQK_INFEASIBLE;
  if (info) {
    info->status = status;
    info->n_after_init = hc[CTR_SURV];
    info->iterations = 0;
    info->passes = 1;
    info->rows_spilled = hc[CTR_OVER];
    if (o.timing) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]);
      info->pass_ms = ms;
    }
  }
  return CQK_OK;
}

cqk_status run_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const float* x, const float* g, float* grad_y,
                                    double* grad_r, const cqk_opts& o) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  BatArgs A{};
  A.nseg = nseg;
  A.off = offsets;
  A.x = const_cast<float*>(x);
  A.g = g;
  A.gy = grad_y;
  A.gr = grad_r;
  A.list = w.list;
  A.counters = w.counters;
  hipStream_t s = ctx->stream;
  plan(ctx, A);
  hipLaunchKernelGGL(bat_vjp_kernel, dim3(persistent_grid(ctx, nseg)), dim3(kBlock), 0, s, A);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  if (o.sync && hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
  return CQK_OK;
}

}  // namespace cqk
