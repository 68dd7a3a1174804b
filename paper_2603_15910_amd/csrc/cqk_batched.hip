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
// Schedule.  Rows are classified on the device by length: rows of at most
// 64 * small_per values go to one wave each (four per workgroup), longer rows
// get a whole workgroup.  Workgroup rows are listed by decreasing length
// bucket; one persistent kernel pulls work items from an atomic counter
// (wave rows first or workgroup rows first) until the list is exhausted.
// small_per, the number of persistent workgroups per compute unit and that
// order form the schedule, which the tuner picks by timing every candidate
// on the caller's rows.
//
// A workgroup row is read once from HBM and x written once: each wave takes
// every fourth tile of 1024 values, writes zeros to that part of x, runs
// Algorithm 2 on 16 values per lane on its first tile with values above its
// running bound and keeps every such value of later tiles (wave reductions
// only), appending them with their indices to its LDS list.  After one barrier every wave combines the four lists'
// bounds, runs Algorithm 4 on the lists from the combined bound (all waves
// get the same multiplier) and writes x for its own list's entries; every
// other x is the zero already written.  The backward pass
// does the same with the support: zeros first, then g - mean_S g on S.
// A wave row keeps its values in registers from load to store.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "cqk_alg1.h"
#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kK = 16;               // values per lane per wave tile (workgroup rows)
constexpr int kWTile = kWave * kK;   // 1024
constexpr int kSurvW = 1024;         // LDS list slots per wave (value + index)
constexpr int kNBW = 24;             // length buckets (bit length) of each row class
constexpr int kNB = 2 * kNBW;        // wave rows 0 .. kNBW - 1, workgroup rows kNBW .. kNB - 1
constexpr int kRefine = 8;
constexpr int kMaxNewton = 100;

enum BatFlags : int32_t { kBadRadius = 1, kBadValue = 2, kInfeasible = 4, kNotConverged = 8 };

struct BatArgs {
  int32_t nseg;
  int32_t small_max;    // longest row solved from one wave's registers
  int32_t med_max;      // longest row solved by one wave (tile by tile above small_max)
  int32_t short_first;  // 1: wave rows are handed out first
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
  int32_t* list;        // row ids: workgroup rows by bucket, then wave rows
  int64_t* lrow;        // per list entry: the row's first element and its length
  int32_t* counters;    // CTR_* below
  int32_t* bhist;       // planning: rows per length bucket of each block of kPBlock rows
};

// The call's counters: rows of each class, work items, the work queue, the
// flags, the survivors total and the rows whose lists overflowed.
constexpr int CTR_NLONG = 0, CTR_NSHORT = 1, CTR_NITEMS = 2, CTR_QUEUE = 3, CTR_FLAGS = 4,
              CTR_SURV = 6, CTR_OVER = 7, CTR_TOTAL = 8;

// Length bucket of a row of L values: its bit length, in the wave-row range
// if L <= wave_max, else in the workgroup-row range.  (Finer buckets, with
// the two bits below the leading one, made the solve kernel slower.)
__device__ __forceinline__ int bucket_of(int64_t L, int wave_max) {
  int b = 64 - __clzll((unsigned long long)L);
  b = b >= kNBW ? kNBW - 1 : b;
  return (L <= wave_max) ? b : kNBW + b;
}

// Planning: the rows are listed by length bucket (workgroup rows longest
// bucket first, then the wave rows longest bucket first, so the four wave
// rows of one work item have about the same length), in row order inside a
// bucket, without atomics: each block of kPBlock rows counts its buckets
// with ballots, then each block places its rows after the rows of its bucket
// in earlier blocks.
constexpr int kPBlock = 1024;
constexpr int kPW = kPBlock / kWave;

// Longest row one wave solves: the simplex forward's medium limit, else the
// register limit.
template <typename Args>
__device__ __forceinline__ int wave_row_max(const Args& A) {
  return A.small_max;
}

template <>
__device__ __forceinline__ int wave_row_max<BatArgs>(const BatArgs& A) {
  return A.med_max;
}

// length bucket of row s, -1 past the last row.  Args: the simplex or the
// general form's argument record (both carry nseg, small_max, off and the
// planning buffers).
template <typename Args>
__device__ __forceinline__ int plan_bucket(const Args& A, int s) {
  return (s < A.nseg) ? bucket_of(A.off[s + 1] - A.off[s], wave_row_max(A)) : -1;
}

template <typename Args>
__global__ __launch_bounds__(kPBlock) void bat_count_kernel(Args A) {
  __shared__ int wh[kPW][kNB];
  const int s = blockIdx.x * kPBlock + (int)threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int b = plan_bucket(A, s);
  for (int k = 0; k < kNB; ++k) {
    const uint64_t m = __ballot(b == k);
    if (lane == 0) wh[w][k] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kNB) {
    int c = 0;
    for (int q = 0; q < kPW; ++q) c += wh[q][threadIdx.x];
    A.bhist[(size_t)blockIdx.x * kNB + threadIdx.x] = c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.counters[CTR_QUEUE] = 0;
    A.counters[CTR_FLAGS] = 0;
    A.counters[CTR_SURV] = 0;
    A.counters[CTR_OVER] = 0;
  }
}

template <typename Args>
__global__ __launch_bounds__(kPBlock) void bat_place_kernel(Args A) {
  __shared__ int part[2][kNB][32];
  __shared__ int base[kNB], pre[kNB];
  __shared__ int wh[kPW][kNB];
  const int nblk = gridDim.x;
  // bucket totals over all blocks and over the blocks before this one,
  // 32 threads per bucket
  for (int idx = threadIdx.x; idx < kNB * 32; idx += kPBlock) {
    const int k = idx / 32, sub = idx % 32;
    int t = 0, p = 0;
    for (int q = sub; q < nblk; q += 32) {
      const int v = A.bhist[(size_t)q * kNB + k];
      t += v;
      p += (q < (int)blockIdx.x) ? v : 0;
    }
    part[0][k][sub] = t;
    part[1][k][sub] = p;
  }
  const int s = blockIdx.x * kPBlock + (int)threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int b = plan_bucket(A, s);
  int rank = 0;
  for (int k = 0; k < kNB; ++k) {
    const uint64_t m = __ballot(b == k);
    if (b == k) rank = lane_prefix(m);
    if (lane == 0) wh[w][k] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kNB) {
    const int k = threadIdx.x;
    int t = 0, p = 0;
    for (int q = 0; q < 32; ++q) {
      t += part[0][k][q];
      p += part[1][k][q];
    }
    base[k] = t;  // totals for now
    pre[k] = p;
    // exclusive scan of the per-wave counts of this block
    int c = 0;
    for (int q = 0; q < kPW; ++q) {
      const int v = wh[q][k];
      wh[q][k] = c;
      c += v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // workgroup rows, longest bucket first, then the wave rows, longest first
    int acc = 0;
    for (int k = kNB - 1; k >= kNBW; --k) {
      const int t = base[k];
      base[k] = acc;
      acc += t;
    }
    const int nlong = acc;
    for (int k = kNBW - 1; k >= 0; --k) {
      const int t = base[k];
      base[k] = acc;
      acc += t;
    }
    const int nshort = acc - nlong;
    if (blockIdx.x == 0) {
      A.counters[CTR_NLONG] = nlong;
      A.counters[CTR_NSHORT] = nshort;
      A.counters[CTR_NITEMS] = nlong + (nshort + kWaves - 1) / kWaves;
    }
  }
  __syncthreads();
  if (b >= 0) {
    const int pos = base[b] + pre[b] + wh[w][b] + rank;
    A.list[pos] = s;
    // the solve kernels read the row's extent with its id, in one round trip
    A.lrow[2 * (size_t)pos] = A.off[s];
    A.lrow[2 * (size_t)pos + 1] = A.off[s + 1] - A.off[s];
  }
}

__device__ __forceinline__ double row_radius(const BatArgs& A, int s) {
  return A.r ? A.r[s] : A.r_scalar;
}

// Block sum of three doubles; every thread gets the totals.
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* lds, double* o) {
  __shared__ double bc[3];
  double in[3] = {a, b, c};
  block_reduce<3, 0, 0, kBlock>(in, nullptr, nullptr, lds, bc);
  o[0] = bc[0];
  o[1] = bc[1];
  o[2] = bc[2];
  __syncthreads();
}

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

// LDS of one workgroup: the four waves' lists and their bound records.
struct BatLds {
  float sv[kWaves][kSurvW];
  int32_t si[kWaves][kSurvW];
  double ws[kWaves][8];
  double red[3 * kWaves];
  int item;
};

enum { W_C = 0, W_S, W_LMIN, W_VMAX, W_BAD, W_N, W_NF };

// One wave's share of Algorithm 2 on a tile of kK values per lane already in
// registers (v, active): the lanes' sets, the wave's bound refined against
// its running survivors (run_c, run_s), the values kept.  Returns the keep
// mask; nk/ks are the lane's kept count and sum; lam_min takes the new bound.
__device__ __forceinline__ uint32_t wave_tile_alg2(const float* v, uint32_t active, double rd,
                                                   double run_c, double run_s, double& lam_min,
                                                   double& nk, double& ks) {
  const float r = (float)rd;
  int c = 0;
  float S = 0.f;
  uint32_t J;
  if (__ballot(__popc(active) > 1) != 0) {
    J = alg2<kK>(v, active, r, c, S);
  } else {
    // at most one value per lane: Algorithm 2 keeps it
    J = active;
    c = __popc(active);
#pragma unroll
    for (int e = 0; e < kK; ++e)
      if ((active >> e) & 1u) S = v[e];
  }
  const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
  // every bound below is lam_J of a non-empty J, hence >= lam* (eq. (lambdaJ))
  const double ct = wave_sum((double)c), skt = wave_sum((double)S);
  double lam_b = (ct > 0.0) ? (rd - skt) / ct : inf_d();
  if (ct > 0.0 && run_c > 0.0) lam_b = fmin(lam_b, (rd - (skt + run_s)) / (ct + run_c));
  if (run_c > 0.0) lam_b = fmin(lam_b, (rd - run_s) / run_c);
  uint32_t keep = 0;
  auto select = [&](double lb) {
    const double lt = fmin(lam_t, lb);
    keep = 0;
    nk = 0.0;
    ks = 0.0;
#pragma unroll
    for (int e = 0; e < kK; ++e) {
      if (((J >> e) & 1u) && ((double)v[e] + lt > 0.0)) {
        keep |= 1u << e;
        nk += 1.0;
        ks += (double)v[e];
      }
    }
  };
  for (int it = 0; it < kRefine; ++it) {
    select(lam_b);
    const double kc = wave_sum(nk), kss = wave_sum(ks);
    if (kc == 0.0) break;
    double nl = (rd - kss) / kc;
    if (run_c > 0.0) nl = fmin(nl, (rd - (kss + run_s)) / (kc + run_c));
    if (!(nl < lam_b)) break;
    lam_b = nl;
  }
  select(lam_b);
  lam_min = fmin(lam_min, lam_b);
  return keep;
}

// One wave tile of a row: kK values per lane, four 16-byte vectors at
// t0 + q*256 + lane*4 (q < 4); when the tile is in range every load is
// issued before the first use.  Rows start at any element, so the vectors
// are only element-aligned.
__device__ __forceinline__ void load_wtile(const float* p, int64_t t0, int lane, int64_t n,
                                           float* o) {
  if (t0 + kWTile <= n) {
    flt4u r[kK / 4];
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) r[q] = ld16(p + t0 + q * kWave * 4 + lane * 4);
#pragma unroll
    for (int q = 0; q < kK / 4; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) o[4 * q + k] = r[q][k];
  } else {
    // a part tile: whole vectors still move 16 bytes, the one that crosses
    // the end value by value
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) {
      const int64_t i = t0 + q * kWave * 4 + lane * 4;
      if (i + 4 <= n) {
        const flt4u r = ld16(p + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) o[4 * q + k] = r[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[4 * q + k] = (i + k < n) ? p[i + k] : 0.f;
      }
    }
  }
}

__device__ __forceinline__ void zero_wtile(float* p, int64_t t0, int lane, int64_t n) {
  const flt4u z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < kK / 4; ++q) {
    const int64_t i = t0 + q * kWave * 4 + lane * 4;
    if (i + 4 <= n) {
      st16(p + i, z);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i + k < n) p[i + k] = 0.f;
    }
  }
}

// The largest float not above x: v > result exactly when v + x' > 0 for
// x' = -x, so a bound filters FP32 values with one FP32 compare.
__device__ __forceinline__ float float_at_or_below(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -__builtin_huge_valf());
  return f;
}

// Algorithm 4 from lam (>= lam*) on the four LDS lists, run by one wave:
// lam_{k+1} = lam_J(J_k), J_k = {v + lam_k > 0}; stops as the paper's
// Algorithm 4 (phi(lam_k) <= r for k >= 1) or when J no longer changes.
__device__ __forceinline__ double wave_newton_lists(const BatLds& L, const int* nw, double rd,
                                                    double lam) {
  const int lane = threadIdx.x & (kWave - 1);
  double prev_c = -1.0;
  for (int it = 0; it < kMaxNewton; ++it) {
    double cc = 0.0, ss = 0.0, ph = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      for (int i = lane; i < nw[w]; i += kWave) {
        const double v = (double)L.sv[w][i];
        const double z = v + lam;
        if (z > 0.0) {
          cc += 1.0;
          ss += v;
          ph += z;
        }
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
  return lam;
}

// A wave's running state over its tiles of one row: the values kept so far
// (count, sum, list length), the smallest bound found (each bound lam_J of
// some set J, so >= lam*), the largest value and a NaN once a value is NaN
// or infinite.
struct WaveRun {
  double c = 0.0, s = 0.0, lam = inf_d();
  float vmx = -__builtin_huge_valf();
  float badf = 0.f;
  int nw = 0;
};

// One tile (values t0 .. t0 + 1023) of a row of n values for the calling
// wave: x = 0 over the tile; on the wave's first tile of the row Algorithm 2
// per lane with the wave's refinement, on a later one the running bound;
// the values kept are appended with their positions to the wave's list
// (sv, si; entries past kSurvW are counted, not stored).  A tile whose
// largest value is at or below the running bound costs one test.
__device__ __forceinline__ void wave_row_tile(const float* y, float* x, int64_t n, int64_t t0,
                                              double rd, WaveRun& R, float* sv, int32_t* si) {
  static_assert(kK < 32, "a lane's kept count must fit in five bits");
  const int lane = threadIdx.x & (kWave - 1);
  float v[kK];
  uint32_t active = 0;
  float tmax = -__builtin_huge_valf();
  load_wtile(y, t0, lane, n, v);
  if (t0 + kWTile <= n) {
    // a tile wholly in the row: no per-value range tests
    const flt4u z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) st16(x + t0 + q * kWave * 4 + lane * 4, z);
    active = (1u << kK) - 1u;
#pragma unroll
    for (int e = 0; e < kK; ++e) {
      R.badf += v[e] * 0.f;
      tmax = fmaxf(tmax, v[e]);
    }
  } else {
    // x is zero wherever the lists do not write it
    zero_wtile(x, t0, lane, n);
#pragma unroll
    for (int q = 0; q < kK / 4; ++q) {
      const int64_t i = t0 + (int64_t)q * kWave * 4 + (int64_t)lane * 4;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i + k < n) {
          active |= 1u << (4 * q + k);
          R.badf += v[4 * q + k] * 0.f;
          tmax = fmaxf(tmax, v[4 * q + k]);
        }
      }
    }
  }
  R.vmx = fmaxf(R.vmx, tmax);
  // the first bound of the row: lam_J of the tile's largest value alone
  // (Algorithm 2's first set), so that Algorithm 2 below only scans the
  // values above it
  if (R.lam == inf_d()) {
    const double m = wave_max((double)tmax);
    if (m > -inf_d()) R.lam = rd - m;
  }
  // values at or below the wave's best bound so far are zero at the
  // solution (v <= thr exactly when v + lam <= 0)
  if (R.lam < inf_d()) {
    const float thr = float_at_or_below(-R.lam);
    if (__ballot(tmax > thr) == 0) return;
#pragma unroll
    for (int e = 0; e < kK; ++e)
      if (!(v[e] > thr)) active &= ~(1u << e);
  }
  if (__ballot(active != 0u) == 0) return;
  uint32_t keep;
  if (R.c > 0.0) {
    // a later tile: the running bound has already filtered it and every
    // value left is kept; lam_J of everything kept so far becomes the
    // bound below (again >= lam*)
    keep = active;
  } else {
    double nk, ks;
    keep = wave_tile_alg2(v, active, rd, R.c, R.s, R.lam, nk, ks);
  }
  // this lane's place in the list: its kept count (five bits) summed over
  // the lanes below it, one bit at a time
  const int c = __popc(keep);
  int pre = 0, nt = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const uint64_t m = __ballot((c >> b) & 1);
    pre += lane_prefix(m) << b;
    nt += __popcll(m) << b;
  }
  if (nt == 0) return;
  int pos = R.nw + pre;
  double ks = 0.0;
#pragma unroll
  for (int q = 0; q < kK / 4; ++q) {
    if ((keep >> (4 * q)) & 0xFu) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = 4 * q + k;
        if ((keep >> e) & 1u) {
          if (pos < kSurvW) {
            sv[pos] = v[e];
            si[pos] = (int32_t)(t0 + q * kWave * 4 + lane * 4 + k);
          }
          ++pos;
          ks += (double)v[e];
        }
      }
    }
  }
  R.nw += nt;
  R.c += (double)nt;
  R.s += wave_sum(ks);
  R.lam = fmin(R.lam, (rd - R.s) / R.c);
}

// ---------------------------------------------------------------------------
// One workgroup row.
// ---------------------------------------------------------------------------
__device__ void solve_long_row(const BatArgs& A, int s, int64_t base, int64_t n, BatLds& L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const double rd = row_radius(A, s);
  const float* y = A.y + base;
  float* x = A.x + base;
  if (!(rd >= 0.0) || !(rd < inf_d())) {
    for (int64_t i = threadIdx.x; i < n; i += kBlock) x[i] = 0.f;
    if (threadIdx.x == 0) {
      atomicOr(&A.counters[CTR_FLAGS], kBadRadius);
      if (A.lam_out) A.lam_out[s] = __builtin_nan("");
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  WaveRun R;
  const int64_t ntiles = (n + kWTile - 1) / kWTile;
  for (int64_t t = wid; t < ntiles; t += kWaves)
    wave_row_tile(y, x, n, t * kWTile, rd, R, L.sv[wid], L.si[wid]);
  const double run_c = R.c, run_s = R.s, lam_min = R.lam;
  const float vmx = R.vmx, badf = R.badf;
  const int nw = R.nw;
  const double wbad = wave_sum((badf == 0.f) ? 0.0 : 1.0);
  const double wmax = wave_max((double)vmx);
  if (lane == 0) {
    L.ws[wid][W_C] = run_c;
    L.ws[wid][W_S] = run_s;
    L.ws[wid][W_LMIN] = lam_min;
    L.ws[wid][W_VMAX] = wmax;
    L.ws[wid][W_BAD] = wbad;
    L.ws[wid][W_N] = (double)nw;
  }
  __syncthreads();
  // every wave combines the four records in the same order
  double C = 0.0, S = 0.0, lmin = inf_d(), vmax = -inf_d(), bad = 0.0;
  bool over = false;
  int nws[kWaves];
  int ntot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    C += L.ws[w][W_C];
    S += L.ws[w][W_S];
    lmin = fmin(lmin, L.ws[w][W_LMIN]);
    vmax = fmax(vmax, L.ws[w][W_VMAX]);
    bad += L.ws[w][W_BAD];
    nws[w] = (int)L.ws[w][W_N];
    over = over || nws[w] > kSurvW;
    ntot += nws[w];
  }
  if (bad > 0.0 || n == 0 || rd == 0.0) {
    // x is already zero
    if (threadIdx.x == 0) {
      if (bad > 0.0) atomicOr(&A.counters[CTR_FLAGS], kBadValue);
      if (n == 0 && rd > 0.0) atomicOr(&A.counters[CTR_FLAGS], kInfeasible);
      if (A.lam_out) A.lam_out[s] = (bad > 0.0 || n == 0) ? __builtin_nan("") : 0.0;
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  const double lam0 = (C > 0.0) ? fmin((rd - S) / C, lmin) : lmin;
  if (over) {
    // a list overflowed: Algorithm 4 over the row itself (re-read from cache)
    double lam = lam0, prev_c = -1.0;
    for (int it = 0; it < kMaxNewton; ++it) {
      double cc = 0.0, ss = 0.0, ph = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const double yv = (double)y[i];
        const double z = yv + lam;
        if (z > 0.0) {
          cc += 1.0;
          ss += yv;
          ph += z;
        }
      }
      double tt[3];
      block_sum3(cc, ss, ph, L.red, tt);
      if (tt[0] == prev_c) break;
      if (it > 0 && tt[2] <= rd) break;
      if (tt[0] == 0.0) break;
      const double nl = (rd - tt[1]) / tt[0];
      if (!(nl < lam)) break;
      prev_c = tt[0];
      lam = nl;
    }
    double nf = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const float o = (float)fmax((double)y[i] + lam, 0.0);
      nf += (o > 0.f) ? 1.0 : 0.0;
      x[i] = o;
    }
    double tn[3];
    block_sum3(nf, 0.0, 0.0, L.red, tn);
    if (threadIdx.x == 0) {
      if (A.lam_out) A.lam_out[s] = lam;
      if (A.nfree_out) A.nfree_out[s] = (int32_t)tn[0];
      atomicAdd(&A.counters[CTR_SURV], ntot);
      atomicAdd(&A.counters[CTR_OVER], 1);
    }
    return;
  }
  // Algorithm 4 from lam_0 (>= lam*) on the lists.  (The start refinement of
  // the single-instance path, 12 candidate sets, is left out here: on lists
  // in LDS it cost more than the Newton steps it saves.)
  double lam = lam0;
  lam = wave_newton_lists(L, nws, rd, lam);
  // x for this wave's list; every other x of the row is already zero
  double nf = 0.0;
  for (int i = lane; i < nws[wid]; i += kWave) {
    const float o = (float)fmax((double)L.sv[wid][i] + lam, 0.0);
    x[L.si[wid][i]] = o;
    nf += (o > 0.f) ? 1.0 : 0.0;
  }
  nf = wave_sum(nf);
  if (lane == 0) L.ws[wid][W_NF] = nf;
  __syncthreads();
  if (threadIdx.x == 0) {
    double nft = 0.0;
    for (int w = 0; w < kWaves; ++w) nft += L.ws[w][W_NF];
    if (A.lam_out) A.lam_out[s] = lam;
    if (A.nfree_out) A.nfree_out[s] = (int32_t)nft;
    atomicAdd(&A.counters[CTR_SURV], ntot);
  }
}

// Algorithm 4 from lam (>= lam*) on one wave's LDS list of n values.
__device__ __forceinline__ double wave_newton_list(const float* lv, int n, double rd, double lam) {
  const int lane = threadIdx.x & (kWave - 1);
  double prev_c = -1.0;
  for (int it = 0; it < kMaxNewton; ++it) {
    double cc = 0.0, ss = 0.0, ph = 0.0;
    for (int i = lane; i < n; i += kWave) {
      const double v = (double)lv[i];
      const double z = v + lam;
      if (z > 0.0) {
        cc += 1.0;
        ss += v;
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
  return lam;
}

// ---------------------------------------------------------------------------
// One medium row (64 * SP < n <= med_max): one wave takes every tile of the
// row, as each wave of a workgroup row takes every fourth, then runs
// Algorithm 4 on its own list.  No workgroup barrier: the four waves of a
// work item solve four rows of about the same length at once.
// ---------------------------------------------------------------------------
__device__ void solve_medium_row(const BatArgs& A, int s, int64_t base, int64_t n, BatLds& L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const double rd = row_radius(A, s);
  const float* y = A.y + base;
  float* x = A.x + base;
  if (!(rd >= 0.0) || !(rd < inf_d())) {
    for (int64_t i = lane; i < n; i += kWave) x[i] = 0.f;
    if (lane == 0) {
      atomicOr(&A.counters[CTR_FLAGS], kBadRadius);
      if (A.lam_out) A.lam_out[s] = __builtin_nan("");
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  WaveRun R;
  const int64_t ntiles = (n + kWTile - 1) / kWTile;
  for (int64_t t = 0; t < ntiles; ++t)
    wave_row_tile(y, x, n, t * kWTile, rd, R, L.sv[wid], L.si[wid]);
  const bool bad = wave_sum((R.badf == 0.f) ? 0.0 : 1.0) > 0.0;
  if (bad || rd == 0.0) {
    // x is already zero
    if (lane == 0) {
      if (bad) atomicOr(&A.counters[CTR_FLAGS], kBadValue);
      if (A.lam_out) A.lam_out[s] = bad ? __builtin_nan("") : 0.0;
      if (A.nfree_out) A.nfree_out[s] = 0;
    }
    return;
  }
  double lam = (R.c > 0.0) ? fmin((rd - R.s) / R.c, R.lam) : R.lam;
  double nf = 0.0;
  const bool over = R.nw > kSurvW;
  if (over) {
    // the list overflowed: Algorithm 4 over the row itself (re-read)
    double prev_c = -1.0;
    for (int it = 0; it < kMaxNewton; ++it) {
      double cc = 0.0, ss = 0.0, ph = 0.0;
      for (int64_t i = lane; i < n; i += kWave) {
        const double yv = (double)y[i];
        const double z = yv + lam;
        if (z > 0.0) {
          cc += 1.0;
          ss += yv;
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
    for (int64_t i = lane; i < n; i += kWave) {
      const float o = (float)fmax((double)y[i] + lam, 0.0);
      nf += (o > 0.f) ? 1.0 : 0.0;
      x[i] = o;
    }
  } else {
    lam = wave_newton_list(L.sv[wid], R.nw, rd, lam);
    // x for the list; every other x of the row is already zero
    for (int i = lane; i < R.nw; i += kWave) {
      const float o = (float)fmax((double)L.sv[wid][i] + lam, 0.0);
      x[L.si[wid][i]] = o;
      nf += (o > 0.f) ? 1.0 : 0.0;
    }
  }
  nf = wave_sum(nf);
  if (lane == 0) {
    if (A.lam_out) A.lam_out[s] = lam;
    if (A.nfree_out) A.nfree_out[s] = (int32_t)nf;
    atomicAdd(&A.counters[CTR_SURV], R.nw);
    if (over) atomicAdd(&A.counters[CTR_OVER], 1);
  }
}

// ---------------------------------------------------------------------------
// One wave row (L <= 64 * SP), values in registers.
// ---------------------------------------------------------------------------
template <int SP>
__device__ void solve_short_row(const BatArgs& A, int s, int64_t base, int64_t L) {
  const int lane = threadIdx.x & (kWave - 1);
  const double rd = row_radius(A, s);
  const float* y = A.y + base;
  float* x = A.x + base;
  float v[SP];
  uint32_t active = 0;
  double bad = 0.0;
#pragma unroll
  for (int k = 0; k < SP; ++k) v[k] = 0.f;
  if (L > 0) {
    // every load issued before the first use (index clamped to the row)
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int64_t i = (int64_t)k * kWave + lane;
      v[k] = y[i < L ? i : L - 1];
    }
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int64_t i = (int64_t)k * kWave + lane;
      if (i < L) {
        active |= 1u << k;
        bad += (fabsf(v[k]) < __builtin_huge_valf()) ? 0.0 : 1.0;
      } else {
        v[k] = 0.f;
      }
    }
  }
  bad = wave_sum(bad);
  const bool bad_r = !(rd >= 0.0) || !(rd < inf_d());
  if (bad_r || bad > 0.0 || L == 0 || rd == 0.0) {
#pragma unroll
    for (int k = 0; k < SP; ++k) {
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
  // Algorithm 2 scans only the values above the first bound, lam_J of the
  // row's largest value alone
  float vm = -__builtin_huge_valf();
#pragma unroll
  for (int k = 0; k < SP; ++k)
    if ((active >> k) & 1u) vm = fmaxf(vm, v[k]);
  const double lam_first = rd - wave_max((double)vm);
  const float thr = float_at_or_below(-lam_first);
  uint32_t scan = 0;
#pragma unroll
  for (int k = 0; k < SP; ++k) scan |= (((active >> k) & 1u) && v[k] > thr) ? (1u << k) : 0u;
  int c;
  float S;
  const uint32_t J = alg2<SP>(v, scan, r, c, S);
  const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
  const double cw = wave_sum((double)c), sw = wave_sum((double)S);
  double lam_b = (cw > 0) ? fmin((rd - sw) / cw, lam_first) : lam_first;
  // refinement on the wave's own sub-problem, then Algorithm 4 on the row
  for (int it = 0; it < kRefine; ++it) {
    const double lt = fmin(lam_t, lam_b);
    double nk = 0.0, ks = 0.0;
#pragma unroll
    for (int e = 0; e < SP; ++e)
      if (((J >> e) & 1u) && (double)v[e] + lt > 0.0) {
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
    for (int e = 0; e < SP; ++e) {
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
  for (int k = 0; k < SP; ++k) {
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
}

// Work item -> workgroup row (true) or group of four wave rows (false), and
// its index in that class, under the schedule's order.
__device__ __forceinline__ bool item_is_long(const BatArgs& A, int item, int nlong, int nsg,
                                             int* idx) {
  if (A.short_first) {
    if (item < nsg) {
      *idx = item;
      return false;
    }
    *idx = item - nsg;
    return true;
  }
  if (item < nlong) {
    *idx = item;
    return true;
  }
  *idx = item - nlong;
  return false;
}

template <int SP>
__global__ __launch_bounds__(kBlock, 3) void bat_solve_kernel(BatArgs A) {
  __shared__ BatLds L;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  const int nsg = nitems - nlong;
  for (;;) {
    if (threadIdx.x == 0) L.item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = L.item;
    __syncthreads();
    if (item >= nitems) break;
    int idx;
    if (item_is_long(A, item, nlong, nsg, &idx)) {
      solve_long_row(A, A.list[idx], A.lrow[2 * (size_t)idx], A.lrow[2 * (size_t)idx + 1], L);
    } else {
      const int k = idx * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) {
        const size_t e = (size_t)nlong + k;
        const int64_t Lr = A.lrow[2 * e + 1];
        if (Lr <= A.small_max) solve_short_row<SP>(A, A.list[e], A.lrow[2 * e], Lr);
        else solve_medium_row(A, A.list[e], A.lrow[2 * e], Lr, L);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Backward: grad_y = [x > 0](g - mean_S g), grad_r = mean_S g.
// ---------------------------------------------------------------------------
// One tile (values t0 .. t0 + 1023) of a row of n values for the calling
// wave's VJP: grad_y = 0 over the tile, the support's count and sum of g
// added to (cnt, sum), its (g, position) pairs appended to the wave's list
// (sv, si; entries past kSurvW are counted, not stored).
__device__ __forceinline__ void vjp_row_tile(const float* x, const float* g, float* gy, int64_t n,
                                             int64_t t0, double& cnt, double& sum, int& nw,
                                             float* sv, int32_t* si) {
  const int lane = threadIdx.x & (kWave - 1);
  float xs[kK], gs[kK];
  uint32_t sup = 0;
  load_wtile(x, t0, lane, n, xs);
  load_wtile(g, t0, lane, n, gs);
  // grad_y is zero off the support
  zero_wtile(gy, t0, lane, n);
#pragma unroll
  for (int q = 0; q < kK / 4; ++q) {
    const int64_t i = t0 + (int64_t)q * kWave * 4 + (int64_t)lane * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = 4 * q + k;
      if (i + k < n && xs[e] > 0.f) {
        sup |= 1u << e;
        cnt += 1.0;
        sum += (double)gs[e];
      }
    }
  }
  if (__ballot(sup != 0u) == 0) return;
#pragma unroll
  for (int e = 0; e < kK; ++e) {
    const bool kb = (sup >> e) & 1u;
    const uint64_t m = __ballot(kb);
    if (kb) {
      const int pos = nw + lane_prefix(m);
      if (pos < kSurvW) {
        sv[pos] = gs[e];
        si[pos] = (int32_t)(t0 + (e / 4) * kWave * 4 + lane * 4 + (e % 4));
      }
    }
    nw += __popcll(m);
  }
}

__device__ void vjp_long_row(const BatArgs& A, int s, int64_t base, int64_t n, BatLds& L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const float* x = A.x + base;
  const float* g = A.g + base;
  float* gy = A.gy + base;
  double cnt = 0.0, sum = 0.0;
  int nw = 0;
  const int64_t ntiles = (n + kWTile - 1) / kWTile;
  for (int64_t t = wid; t < ntiles; t += kWaves)
    vjp_row_tile(x, g, gy, n, t * kWTile, cnt, sum, nw, L.sv[wid], L.si[wid]);
  cnt = wave_sum(cnt);
  sum = wave_sum(sum);
  if (lane == 0) {
    L.ws[wid][W_C] = cnt;
    L.ws[wid][W_S] = sum;
    L.ws[wid][W_N] = (double)nw;
  }
  __syncthreads();
  double C = 0.0, Sg = 0.0;
  bool over = false;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    C += L.ws[w][W_C];
    Sg += L.ws[w][W_S];
    over = over || L.ws[w][W_N] > (double)kSurvW;
  }
  const double gbar = (C > 0.0) ? Sg / C : 0.0;
  const float gb = (float)gbar;
  if (over) {
    // the support did not fit the lists: a second pass over the row
    for (int64_t i = threadIdx.x; i < n; i += kBlock)
      if (x[i] > 0.f) gy[i] = g[i] - gb;
  } else {
    for (int i = lane; i < nw; i += kWave) gy[L.si[wid][i]] = L.sv[wid][i] - gb;
  }
  if (threadIdx.x == 0 && A.gr) A.gr[s] = gbar;
}

// A medium row's VJP (64 * SP < n <= med_max) by one wave, tile after tile.
__device__ void vjp_medium_row(const BatArgs& A, int s, int64_t base, int64_t n, BatLds& L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const float* x = A.x + base;
  const float* g = A.g + base;
  float* gy = A.gy + base;
  double cnt = 0.0, sum = 0.0;
  int nw = 0;
  const int64_t ntiles = (n + kWTile - 1) / kWTile;
  for (int64_t t = 0; t < ntiles; ++t)
    vjp_row_tile(x, g, gy, n, t * kWTile, cnt, sum, nw, L.sv[wid], L.si[wid]);
  const double C = wave_sum(cnt), Sg = wave_sum(sum);
  const double gbar = (C > 0.0) ? Sg / C : 0.0;
  const float gb = (float)gbar;
  if (nw > kSurvW) {
    // the support did not fit the list: a second pass over the row
    for (int64_t i = lane; i < n; i += kWave)
      if (x[i] > 0.f) gy[i] = g[i] - gb;
  } else {
    for (int i = lane; i < nw; i += kWave) gy[L.si[wid][i]] = L.sv[wid][i] - gb;
  }
  if (lane == 0 && A.gr) A.gr[s] = gbar;
}

template <int SP>
__device__ void vjp_short_row(const BatArgs& A, int s, int64_t base, int64_t L) {
  const int lane = threadIdx.x & (kWave - 1);
  float xs[SP], gs[SP];
  double cnt = 0.0, sum = 0.0;
#pragma unroll
  for (int k = 0; k < SP; ++k) xs[k] = gs[k] = 0.f;
  if (L > 0) {
    // every load issued before the first use (index clamped to the row)
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int64_t i = (int64_t)k * kWave + lane;
      const int64_t e = base + (i < L ? i : L - 1);
      xs[k] = A.x[e];
      gs[k] = A.g[e];
    }
#pragma unroll
    for (int k = 0; k < SP; ++k)
      if ((int64_t)k * kWave + lane >= L) xs[k] = gs[k] = 0.f;
  }
#pragma unroll
  for (int k = 0; k < SP; ++k) {
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
  for (int k = 0; k < SP; ++k) {
    const int64_t i = (int64_t)k * kWave + lane;
    if (i < L) A.gy[base + i] = (xs[k] > 0.f) ? gs[k] - gb : 0.f;
  }
  if (lane == 0 && A.gr) A.gr[s] = gbar;
}

template <int SP>
__global__ __launch_bounds__(kBlock) void bat_vjp_kernel(BatArgs A) {
  __shared__ BatLds L;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  const int nsg = nitems - nlong;
  for (;;) {
    if (threadIdx.x == 0) L.item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = L.item;
    __syncthreads();
    if (item >= nitems) break;
    int idx;
    if (item_is_long(A, item, nlong, nsg, &idx)) {
      vjp_long_row(A, A.list[idx], A.lrow[2 * (size_t)idx], A.lrow[2 * (size_t)idx + 1], L);
    } else {
      const int k = idx * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) {
        const size_t e = (size_t)nlong + k;
        const int64_t Lr = A.lrow[2 * e + 1];
        if (Lr <= A.small_max) vjp_short_row<SP>(A, A.list[e], A.lrow[2 * e], Lr);
        else vjp_medium_row(A, A.list[e], A.lrow[2 * e], Lr, L);
      }
    }
    __syncthreads();
  }
}


// ===========================================================================
// Batched general CQK (Section 2.1, Algorithm 1 per row) and its VJP.
//
// Row s is (d, a, b, l, u)[off[s] .. off[s+1]) with its own r[s].  Every row
// runs Algorithm 1 from lam = 0 (or eq. (CQKlambda0) over the row) with its
// own bracket, breakpoint and secant state: the scalar update of the
// single-instance solver on a state record each wave or workgroup keeps in
// registers, every lane updating its own copy from the same reduced sums (so
// all copies stay identical and the control flow uniform).  A row of at most
// 64 * small_per values is one wave's, its per-index form (c, s, bl, bu) held in
// registers from load to store (4 or 8 values per lane, by the schedule); a
// longer row is a workgroup's, which re-reads the row from memory at every
// evaluation.  x = clamp((a + lam b)/d, l, u)
// (eq. (xopt)) is written once.
//
// Backward, on a locally constant free set F = {l < x < u} (eq. (xopt) on F
// and eq. (opt) differentiated): with q = sum_F b^2/d and
// mu = (sum_F g b/d)/q,
//   grad_a = [F](g - b mu)/d,   grad_r = mu   (both 0 when F is empty).
// ===========================================================================
constexpr int kCqkU = 4;    // values per thread in flight in a workgroup pass
constexpr int CTR_ITSUM = CTR_SURV, CTR_ITMAX = CTR_OVER;

struct BatCqkArgs {
  int32_t nseg;
  int32_t small_max;    // longest wave row
  int32_t short_first;  // 1: wave rows are handed out first
  int32_t lambda0_mode; // CQK_LAMBDA0_ZERO, _FORMULA or _USER
  int32_t max_iter;
  double tol;
  double lam0_user;     // the start of every row with CQK_LAMBDA0_USER
  const int64_t* off;
  const void *d, *a, *b, *l, *u;  // TIn (float or double)
  const double* r;
  void* x;              // forward output; backward input (TIn)
  double* lam_out;
  int32_t* status_out;
  const void* g;        // backward: upstream gradient (TIn)
  void* ga;             // backward: grad_a (TIn)
  double* gr;           // backward: grad_r
  int32_t* list;
  int64_t* lrow;
  int32_t* counters;
  int32_t* bhist;
};

__device__ __forceinline__ GenState cqk_row_state(const BatCqkArgs& A, double r) {
  GenState st{};
  st.lam = (A.lambda0_mode == CQK_LAMBDA0_USER) ? A.lam0_user : 0.0;
  st.lam0 = st.lam;
  st.lam_prev = __builtin_nan("");
  st.lam_final = __builtin_nan("");
  st.lo = -inf_d();
  st.hi = inf_d();
  st.phi_lo = st.phi_hi = __builtin_nan("");
  st.r = r;
  st.tol = A.tol;
  st.status = kRunning;
  st.max_iter = A.max_iter;
  st.compaction = CQK_COMPACT_OFF;
  st.mode = kModeEval;
  return st;
}

// Per-row outputs and the call's flags, by one thread of the row's owner.
__device__ __forceinline__ void cqk_row_report(const BatCqkArgs& A, int s, const GenState& st,
                                               double lam) {
  if (A.lam_out) A.lam_out[s] = lam;
  if (A.status_out) A.status_out[s] = st.status;
  int f = 0;
  if (st.status == CQK_INVALID_ARG) f = kBadValue;
  else if (st.status == CQK_INFEASIBLE) f = kInfeasible;
  else if (st.status == CQK_NOT_CONVERGED) f = kNotConverged;
  if (f) atomicOr(&A.counters[CTR_FLAGS], f);
  atomicAdd(&A.counters[CTR_ITSUM], st.iter);
  atomicMax(&A.counters[CTR_ITMAX], st.iter);
}

// The arrays of a call in their element type (FP64 values are used as
// they are, FP32 values are widened to FP64 for the arithmetic).
template <typename TIn>
struct CqkArrays {
  const TIn *d, *a, *b, *l, *u, *g;
  TIn *x, *ga;
  __device__ explicit CqkArrays(const BatCqkArgs& A)
      : d((const TIn*)A.d), a((const TIn*)A.a), b((const TIn*)A.b), l((const TIn*)A.l),
        u((const TIn*)A.u), g((const TIn*)A.g), x((TIn*)A.x), ga((TIn*)A.ga) {}
};

// x_i of eq. (xopt) at the row's multiplier.
template <typename TIn>
__device__ __forceinline__ double cqk_x_at(const CqkArrays<TIn>& V, int64_t i, double lam) {
  const double t = fma((double)V.b[i], lam, (double)V.a[i]) / (double)V.d[i];
  return fmin(fmax(t, (double)V.l[i]), (double)V.u[i]);
}

__device__ __forceinline__ bool cqk_has_lambda(const GenState& st) {
  return st.status == CQK_OK || st.status == CQK_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// One wave row (L <= 64 * SP), per-index form in registers.
// ---------------------------------------------------------------------------
template <int SP, typename TIn>
__device__ void cqk_short_row(const BatCqkArgs& A, int s, int64_t base, int64_t L) {
  const CqkArrays<TIn> V(A);
  const int lane = threadIdx.x & (kWave - 1);
  double c[SP], sv[SP], bl[SP], bu[SP];
  double bad = 0.0, sc = 0.0, ss = 0.0;
#pragma unroll
  for (int k = 0; k < SP; ++k) c[k] = sv[k] = bl[k] = bu[k] = 0.0;
  if (L > 0) {
    // every load issued before the first use (index clamped to the row), so
    // the row costs one memory round trip, not one per value of a lane
    TIn rd[SP], ra[SP], rb[SP], rl[SP], ru[SP];
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int64_t i = lane + (int64_t)k * kWave;
      const int64_t e = base + (i < L ? i : L - 1);
      rd[k] = V.d[e];
      ra[k] = V.a[e];
      rb[k] = V.b[e];
      rl[k] = V.l[e];
      ru[k] = V.u[e];
    }
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      if (lane + (int64_t)k * kWave < L) {
        to_form((double)rd[k], (double)ra[k], (double)rb[k], (double)rl[k], (double)ru[k], c[k],
                sv[k], bl[k], bu[k], bad);
        sc += c[k];
        ss += sv[k];
      }
    }
  }
  const double r = A.r[s];
  GenState st = cqk_row_state(A, r);
  if (wave_sum(bad) > 0.0 || !(fabs(r) < inf_d())) {
    st.status = CQK_INVALID_ARG;
  } else if (L == 0) {
    st.status = (r == 0.0) ? CQK_OK : CQK_INFEASIBLE;
    st.lam_final = 0.0;
  } else if (A.lambda0_mode == CQK_LAMBDA0_FORMULA) {
    const double tc = wave_sum(sc), ts = wave_sum(ss);
    st.lam = st.lam0 = (ts > 0.0) ? (r - tc) / ts : 0.0;
  }
  while (st.status == kRunning) {
    if (st.mode == kModeEval) {
      Acc acc;
      acc_init(acc);
#pragma unroll
      for (int k = 0; k < SP; ++k)
        if (lane + (int64_t)k * kWave < L) eval_index<false>(acc, c[k], sv[k], bl[k], bu[k], st.lam, st.lo, st.hi);
      double t[NSUM];
#pragma unroll
      for (int i = 0; i < NSUM; ++i) t[i] = 0.0;
      t[P_P] = wave_sum(acc.s[P_P]);
      t[P_A] = wave_sum(acc.s[P_A]);
      t[P_QP] = wave_sum(acc.s[P_QP]);
      t[P_QM] = wave_sum(acc.s[P_QM]);
      t[P_NIN] = (double)L;
      update_after_eval(&st, t, nullptr);
    } else {
      KeySum ks[2] = {KeySum{inf_d(), 0.0}, KeySum{inf_d(), 0.0}};
#pragma unroll
      for (int k = 0; k < SP; ++k)
        if (lane + (int64_t)k * kWave < L) bkpt_index(ks, c[k], sv[k], bl[k], bu[k], st.lam);
      ks[0] = wave_ks_min(ks[0]);
      ks[1] = wave_ks_min(ks[1]);
      update_after_bkpt(&st, ks, nullptr);
    }
  }
  const bool ok = cqk_has_lambda(st);
  const double lam = ok ? st.lam_final : __builtin_nan("");
#pragma unroll
  for (int k = 0; k < SP; ++k) {
    const int64_t i = lane + (int64_t)k * kWave;
    if (i < L) V.x[base + i] = (TIn)(ok ? cqk_x_at(V, base + i, lam) : __builtin_nan(""));
  }
  if (lane == 0) cqk_row_report(A, s, st, lam);
}

// ---------------------------------------------------------------------------
// One workgroup row: every evaluation streams the row.
// ---------------------------------------------------------------------------
struct CqkLds {
  double red[8 * kWaves];
  double tot[8];
  KeySum ks[2];
  int item;
};

template <typename TIn>
__device__ void cqk_long_row(const BatCqkArgs& A, int s, int64_t base, int64_t L, CqkLds& S) {
  const CqkArrays<TIn> V(A);
  const double r = A.r[s];
  GenState st = cqk_row_state(A, r);
  const TIn* d = V.d + base;
  const TIn* a = V.a + base;
  const TIn* b = V.b + base;
  const TIn* l = V.l + base;
  const TIn* u = V.u + base;
  constexpr int64_t STEP = (int64_t)kBlock * kCqkU;
  // kCqkU values per thread with every load issued before the first use:
  // the loads are unconditional (a lane past the end re-reads the last value,
  // L > i0 >= 0 inside the loop) and the neutral values are selected after,
  // so no load sits behind a branch and its own wait
  auto stream = [&](auto&& fn) {
    for (int64_t i0 = threadIdx.x; i0 < L; i0 += STEP) {
      TIn rd[kCqkU], ra[kCqkU], rb[kCqkU], rl[kCqkU], ru[kCqkU];
#pragma unroll
      for (int k = 0; k < kCqkU; ++k) {
        const int64_t i = i0 + (int64_t)k * kBlock;
        const int64_t ic = i < L ? i : L - 1;
        rd[k] = d[ic];
        ra[k] = a[ic];
        rb[k] = b[ic];
        rl[k] = l[ic];
        ru[k] = u[ic];
      }
      double vd[kCqkU], va[kCqkU], vb[kCqkU], vl[kCqkU], vu[kCqkU];
#pragma unroll
      for (int k = 0; k < kCqkU; ++k) {
        const bool in = i0 + (int64_t)k * kBlock < L;
        vd[k] = in ? (double)rd[k] : 1.0;
        va[k] = in ? (double)ra[k] : 0.0;
        vb[k] = in ? (double)rb[k] : 1.0;
        vl[k] = in ? (double)rl[k] : 0.0;
        vu[k] = in ? (double)ru[k] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kCqkU; ++k)
        if (i0 + (int64_t)k * kBlock < L) fn(i0 + (int64_t)k * kBlock, vd[k], va[k], vb[k], vl[k], vu[k]);
    }
  };
  if (!(fabs(r) < inf_d())) {
    st.status = CQK_INVALID_ARG;
  } else if (A.lambda0_mode == CQK_LAMBDA0_FORMULA) {
    double acc[3] = {0.0, 0.0, 0.0};
    stream([&](int64_t, double vd, double va, double vb, double vl, double vu) {
      double c, sv, bl, bu;
      to_form(vd, va, vb, vl, vu, c, sv, bl, bu, acc[2]);
      acc[0] += c;
      acc[1] += sv;
    });
    block_reduce<3, 0, 0, kBlock>(acc, nullptr, nullptr, S.red, S.tot);
    if (S.tot[2] > 0.0) st.status = CQK_INVALID_ARG;
    else st.lam = st.lam0 = (S.tot[1] > 0.0) ? (r - S.tot[0]) / S.tot[1] : 0.0;
  }
  while (st.status == kRunning) {
    if (st.mode == kModeEval) {
      Acc acc;
      acc_init(acc);
      double bad = 0.0;
      const double lam = st.lam, lo = st.lo, hi = st.hi;
      stream([&](int64_t, double vd, double va, double vb, double vl, double vu) {
        double c, sv, bl, bu;
        to_form(vd, va, vb, vl, vu, c, sv, bl, bu, bad);
        eval_index<false>(acc, c, sv, bl, bu, lam, lo, hi);
      });
      double v[5] = {acc.s[P_P], acc.s[P_A], acc.s[P_QP], acc.s[P_QM], bad};
      block_reduce<5, 0, 0, kBlock>(v, nullptr, nullptr, S.red, S.tot);
      double t[NSUM];
#pragma unroll
      for (int i = 0; i < NSUM; ++i) t[i] = 0.0;
      t[P_P] = S.tot[0];
      t[P_A] = S.tot[1];
      t[P_QP] = S.tot[2];
      t[P_QM] = S.tot[3];
      t[P_BAD] = S.tot[4];
      t[P_NIN] = (double)L;
      update_after_eval(&st, t, nullptr);
    } else {
      KeySum ks[2] = {KeySum{inf_d(), 0.0}, KeySum{inf_d(), 0.0}};
      const double lam = st.lam;
      double bad = 0.0;
      stream([&](int64_t, double vd, double va, double vb, double vl, double vu) {
        double c, sv, bl, bu;
        to_form(vd, va, vb, vl, vu, c, sv, bl, bu, bad);
        bkpt_index(ks, c, sv, bl, bu, lam);
      });
      block_ks_min<2, kBlock>(ks, S.red, S.ks);
      const KeySum kt[2] = {S.ks[0], S.ks[1]};
      __syncthreads();
      update_after_bkpt(&st, kt, nullptr);
    }
  }
  const bool ok = cqk_has_lambda(st);
  const double lam = ok ? st.lam_final : __builtin_nan("");
  TIn* x = V.x + base;
  stream([&](int64_t i, double vd, double va, double vb, double vl, double vu) {
    const double t = fma(vb, lam, va) / vd;
    x[i] = (TIn)(ok ? fmin(fmax(t, vl), vu) : __builtin_nan(""));
  });
  if (threadIdx.x == 0) cqk_row_report(A, s, st, lam);
}

template <int SP, typename TIn>
__global__ __launch_bounds__(kBlock) void bat_cqk_solve_kernel(BatCqkArgs A) {
  __shared__ CqkLds S;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  const int nsg = nitems - nlong;
  for (;;) {
    if (threadIdx.x == 0) S.item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = S.item;
    __syncthreads();
    if (item >= nitems) break;
    int idx;
    bool is_long;
    if (A.short_first) {
      is_long = item >= nsg;
      idx = is_long ? item - nsg : item;
    } else {
      is_long = item < nlong;
      idx = is_long ? item : item - nlong;
    }
    if (is_long) {
      cqk_long_row<TIn>(A, A.list[idx], A.lrow[2 * (size_t)idx], A.lrow[2 * (size_t)idx + 1], S);
    } else {
      const int k = idx * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) {
        const size_t e = (size_t)nlong + k;
        cqk_short_row<SP, TIn>(A, A.list[e], A.lrow[2 * e], A.lrow[2 * e + 1]);
      }
    }
    __syncthreads();
  }
}

// Backward of one wave row.
template <int SP, typename TIn>
__device__ void cqk_vjp_short_row(const BatCqkArgs& A, int s, int64_t base, int64_t L) {
  const CqkArrays<TIn> V(A);
  const int lane = threadIdx.x & (kWave - 1);
  double q = 0.0, m = 0.0;
  double gv[SP], bd[SP], dv[SP];
  bool fr[SP];
#pragma unroll
  for (int k = 0; k < SP; ++k) {
    fr[k] = false;
    gv[k] = bd[k] = 0.0;
    dv[k] = 1.0;
  }
  if (L > 0) {
    // every load issued before the first use (index clamped to the row)
    TIn rx[SP], rl[SP], ru[SP], rg[SP], rd[SP], rb[SP];
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      const int64_t i = lane + (int64_t)k * kWave;
      const int64_t e = base + (i < L ? i : L - 1);
      rx[k] = V.x[e];
      rl[k] = V.l[e];
      ru[k] = V.u[e];
      rg[k] = V.g[e];
      rd[k] = V.d[e];
      rb[k] = V.b[e];
    }
#pragma unroll
    for (int k = 0; k < SP; ++k) {
      if (lane + (int64_t)k * kWave < L) {
        const double xv = (double)rx[k];
        fr[k] = (xv > (double)rl[k]) && (xv < (double)ru[k]);
        gv[k] = (double)rg[k];
        dv[k] = (double)rd[k];
        bd[k] = (double)rb[k];
        if (fr[k]) {
          q += bd[k] * bd[k] / dv[k];
          m += gv[k] * bd[k] / dv[k];
        }
      }
    }
  }
  q = wave_sum(q);
  m = wave_sum(m);
  const double mu = (q > 0.0) ? m / q : 0.0;
#pragma unroll
  for (int k = 0; k < SP; ++k) {
    const int64_t i = lane + (int64_t)k * kWave;
    if (i < L) V.ga[base + i] = (TIn)(fr[k] ? (gv[k] - bd[k] * mu) / dv[k] : 0.0);
  }
  if (lane == 0 && A.gr) A.gr[s] = mu;
}

// Backward of one workgroup row: the two sums, then the map.
template <typename TIn>
__device__ void cqk_vjp_long_row(const BatCqkArgs& A, int s, int64_t base, int64_t L,
                                 CqkLds& S) {
  const CqkArrays<TIn> V(A);
  constexpr int64_t STEP = (int64_t)kBlock * kCqkU;
  // kCqkU values per thread, all six loads of each issued before the first
  // use (index clamped to the row, L > i0 >= 0 inside the loop); lanes past
  // the end count as not free
  auto stream = [&](int64_t i0, bool (&fr)[kCqkU], double (&xg)[kCqkU], double (&xb)[kCqkU],
                    double (&xd)[kCqkU]) {
    TIn rx[kCqkU], rl[kCqkU], ru[kCqkU], rb[kCqkU], rd[kCqkU], rg[kCqkU];
#pragma unroll
    for (int k = 0; k < kCqkU; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      const int64_t e = base + (i < L ? i : L - 1);
      rx[k] = V.x[e];
      rl[k] = V.l[e];
      ru[k] = V.u[e];
      rb[k] = V.b[e];
      rd[k] = V.d[e];
      rg[k] = V.g[e];
    }
#pragma unroll
    for (int k = 0; k < kCqkU; ++k) {
      const double xv = (double)rx[k];
      fr[k] = (i0 + (int64_t)k * kBlock < L) && (xv > (double)rl[k]) && (xv < (double)ru[k]);
      xg[k] = (double)rg[k];
      xb[k] = (double)rb[k];
      xd[k] = (double)rd[k];
    }
  };
  double acc[2] = {0.0, 0.0};
  for (int64_t i0 = threadIdx.x; i0 < L; i0 += STEP) {
    bool fr[kCqkU];
    double xg[kCqkU], xb[kCqkU], xd[kCqkU];
    stream(i0, fr, xg, xb, xd);
#pragma unroll
    for (int k = 0; k < kCqkU; ++k) {
      if (fr[k]) {
        acc[0] += xb[k] * xb[k] / xd[k];
        acc[1] += xg[k] * xb[k] / xd[k];
      }
    }
  }
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, S.red, S.tot);
  const double q = S.tot[0];
  const double mu = (q > 0.0) ? S.tot[1] / q : 0.0;
  for (int64_t i0 = threadIdx.x; i0 < L; i0 += STEP) {
    bool fr[kCqkU];
    double xg[kCqkU], xb[kCqkU], xd[kCqkU];
    stream(i0, fr, xg, xb, xd);
#pragma unroll
    for (int k = 0; k < kCqkU; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      if (i < L) V.ga[base + i] = (TIn)(fr[k] ? (xg[k] - xb[k] * mu) / xd[k] : 0.0);
    }
  }
  if (threadIdx.x == 0 && A.gr) A.gr[s] = mu;
}

template <int SP, typename TIn>
__global__ __launch_bounds__(kBlock) void bat_cqk_vjp_kernel(BatCqkArgs A) {
  __shared__ CqkLds S;
  const int nlong = A.counters[CTR_NLONG];
  const int nshort = A.counters[CTR_NSHORT];
  const int nitems = A.counters[CTR_NITEMS];
  const int nsg = nitems - nlong;
  for (;;) {
    if (threadIdx.x == 0) S.item = atomicAdd(&A.counters[CTR_QUEUE], 1);
    __syncthreads();
    const int item = S.item;
    __syncthreads();
    if (item >= nitems) break;
    int idx;
    bool is_long;
    if (A.short_first) {
      is_long = item >= nsg;
      idx = is_long ? item - nsg : item;
    } else {
      is_long = item < nlong;
      idx = is_long ? item : item - nlong;
    }
    if (is_long) {
      cqk_vjp_long_row<TIn>(A, A.list[idx], A.lrow[2 * (size_t)idx], A.lrow[2 * (size_t)idx + 1],
                            S);
    } else {
      const int k = idx * kWaves + (int)(threadIdx.x / kWave);
      if (k < nshort) {
        const size_t e = (size_t)nlong + k;
        cqk_vjp_short_row<SP, TIn>(A, A.list[e], A.lrow[2 * e], A.lrow[2 * e + 1]);
      }
    }
    __syncthreads();
  }
}

struct BatWs {
  int32_t* list;
  int32_t* counters;
  int32_t* bhist;
  int64_t* lrow;
};

constexpr size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Bytes of the planning buffers of a batched call on nseg rows: the row list,
// the counters, the bucket histogram of each planning block and the row
// extents, each on a 256-byte boundary.
constexpr size_t bat_ws_bytes(size_t nseg) {
  return round256(nseg * sizeof(int32_t)) + round256(CTR_TOTAL * sizeof(int32_t)) +
         round256((nseg > kPBlock ? (nseg + kPBlock - 1) / kPBlock : 1) * kNB * sizeof(int32_t)) +
         round256(nseg * 2 * sizeof(int64_t));
}

// Carves the planning buffers out of base (bat_ws_bytes(nseg) bytes).
void bat_layout(void* base, int32_t nseg, BatWs* w) {
  const size_t list_bytes = round256((size_t)nseg * sizeof(int32_t));
  const size_t ctr_bytes = round256(CTR_TOTAL * sizeof(int32_t));
  const size_t nblk = std::max<size_t>(1, ((size_t)nseg + kPBlock - 1) / kPBlock);
  const size_t hist_bytes = round256(nblk * kNB * sizeof(int32_t));
  char* p = (char*)base;
  w->list = (int32_t*)p;
  w->counters = (int32_t*)(p + list_bytes);
  w->bhist = (int32_t*)(p + list_bytes + ctr_bytes);
  w->lrow = (int64_t*)(p + list_bytes + ctr_bytes + hist_bytes);
}

cqk_status bat_workspace(cqk_ctx* ctx, int32_t nseg, BatWs* w) {
  cqk_status st = ensure_buffer(ctx, ctx->ws, bat_ws_bytes((size_t)nseg));
  if (st != CQK_OK) return st;
  bat_layout(ctx->ws.ptr, nseg, w);
  return CQK_OK;
}

// The planning buffers of cqk_project_simplex_batched_noalloc_f32: a fixed
// device array (one copy per GPU, alive until the process ends) for up to
// CQK_NOALLOC_MAX_SEG rows.  Host code never names it in a launch or a copy:
// its address on a device comes from hipGetSymbolAddress (noalloc_scratch).
static_assert(CQK_NOALLOC_MAX_SEG > 0, "row limit of the no-allocation call");
constexpr size_t kScratchBytes = bat_ws_bytes(CQK_NOALLOC_MAX_SEG);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int persistent_grid(cqk_ctx* ctx, const cqk_batch_schedule& sc, int nseg) {
  const int g = ctx->num_cus * sc.blocks_per_cu;
  return std::max(1, std::min(g, nseg));
}

template <typename Args>
void plan(cqk_ctx* ctx, const Args& A) {
  hipStream_t s = ctx->stream;
  const int gb = std::max(1, (A.nseg + kPBlock - 1) / kPBlock);
  hipLaunchKernelGGL(bat_count_kernel<Args>, dim3(gb), dim3(kPBlock), 0, s, A);
  hipLaunchKernelGGL(bat_place_kernel<Args>, dim3(gb), dim3(kPBlock), 0, s, A);
}

// Rows above the register limit and up to medium_tiles tiles are solved by
// one wave.
void apply_schedule(const cqk_batch_schedule& sc, BatArgs* A) {
  A->small_max = kWave * sc.small_per;
  A->med_max = std::max(A->small_max, sc.medium_tiles * kWTile);
  A->short_first = sc.short_first;
}

// Queues one forward call under schedule sc.
void launch_forward(cqk_ctx* ctx, const cqk_batch_schedule& sc, BatArgs A) {
  apply_schedule(sc, &A);
  plan(ctx, A);
  const dim3 grid(persistent_grid(ctx, sc, A.nseg));
  if (sc.small_per == 4)
    hipLaunchKernelGGL(bat_solve_kernel<4>, grid, dim3(kBlock), 0, ctx->stream, A);
  else
    hipLaunchKernelGGL(bat_solve_kernel<8>, grid, dim3(kBlock), 0, ctx->stream, A);
}

void launch_backward(cqk_ctx* ctx, const cqk_batch_schedule& sc, BatArgs A) {
  apply_schedule(sc, &A);
  plan(ctx, A);
  const dim3 grid(persistent_grid(ctx, sc, A.nseg));
  if (sc.small_per == 4)
    hipLaunchKernelGGL(bat_vjp_kernel<4>, grid, dim3(kBlock), 0, ctx->stream, A);
  else
    hipLaunchKernelGGL(bat_vjp_kernel<8>, grid, dim3(kBlock), 0, ctx->stream, A);
}

BatArgs forward_args(int32_t nseg, const int64_t* offsets, const float* y, const double* r,
                     double r_scalar, float* x, double* lambda_out, int32_t* nfree_out,
                     const BatWs& w) {
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
  A.bhist = w.bhist;
  A.lrow = w.lrow;
  return A;
}

BatArgs backward_args(int32_t nseg, const int64_t* offsets, const float* x, const float* g,
                      float* grad_y, double* grad_r, const BatWs& w) {
  BatArgs A{};
  A.nseg = nseg;
  A.off = offsets;
  A.x = const_cast<float*>(x);
  A.g = g;
  A.gy = grad_y;
  A.gr = grad_r;
  A.list = w.list;
  A.counters = w.counters;
  A.bhist = w.bhist;
  A.lrow = w.lrow;
  return A;
}

// The candidate schedules the tuner times.
// The batched simplex candidates: also the medium-row limit (medium_tiles,
// in tiles of 1024 values; 0: none).
int candidate_schedules_fwd(cqk_batch_schedule* out, int cap) {
  int k = 0;
  for (int sp : {4, 8})
    for (int bpc : {2, 3, 4, 6})
      for (int sf : {0, 1})
        for (int med : {0, 4, 8, 16, 32, 64})
          if (k < cap) out[k++] = cqk_batch_schedule{sp, bpc, sf, med};
  return k;
}

int candidate_schedules(cqk_batch_schedule* out, int cap) {
  int k = 0;
  for (int sp : {4, 8})
    for (int bpc : {1, 2, 3, 4})
      for (int sf : {0, 1})
        if (k < cap) out[k++] = cqk_batch_schedule{sp, bpc, sf, 0};
  return k;
}

// Times `launch` for each candidate (`repeats` runs each after one warm-up,
// the fastest counts) and returns the index of the best.
template <typename Launch>
cqk_status tune(cqk_ctx* ctx, const cqk_batch_schedule* cand, int ncand, int repeats,
                Launch launch, int* best, double* best_ms) {
  cqk_status st = ensure_events(ctx, 2);
  if (st != CQK_OK) return st;
  hipStream_t s = ctx->stream;
  *best = 0;
  *best_ms = 1e300;
  for (int c = 0; c < ncand; ++c) {
    launch(cand[c]);
    double t = 1e300;
    for (int k = 0; k < repeats; ++k) {
      hipEventRecord(ctx->events[0], s);
      launch(cand[c]);
      hipEventRecord(ctx->events[1], s);
      if (hip_ok(hipEventSynchronize(ctx->events[1])) != CQK_OK) return CQK_DEVICE_ERROR;
      float ms = 0.f;
      hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]);
      t = std::min(t, (double)ms);
    }
    if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
    if (t < *best_ms) {
      *best_ms = t;
      *best = c;
    }
  }
  return CQK_OK;
}


// Batched general CQK: the plan, then one persistent launch.
BatCqkArgs cqk_args(int32_t nseg, const int64_t* offsets, const void* d, const void* a,
                    const void* b, const void* l, const void* u, const BatWs& w) {
  BatCqkArgs A{};
  A.nseg = nseg;
  A.off = offsets;
  A.d = d;
  A.a = a;
  A.b = b;
  A.l = l;
  A.u = u;
  A.list = w.list;
  A.counters = w.counters;
  A.bhist = w.bhist;
  A.lrow = w.lrow;
  return A;
}

// The batched general CQK under schedule sc: rows of at most
// 64 * small_per values go to one wave (small_per 4 or 8 values per lane in
// registers), blocks_per_cu persistent workgroups per compute unit.
void cqk_apply_schedule(cqk_ctx* ctx, const cqk_batch_schedule& sc, BatCqkArgs* A, dim3* grid) {
  A->small_max = kWave * sc.small_per;
  A->short_first = sc.short_first;
  *grid = dim3(std::max(1, std::min(ctx->num_cus * sc.blocks_per_cu, A->nseg)));
}

template <typename TIn>
void launch_cqk_forward(cqk_ctx* ctx, const cqk_batch_schedule& sc, BatCqkArgs A) {
  dim3 grid;
  cqk_apply_schedule(ctx, sc, &A, &grid);
  plan(ctx, A);
  if (sc.small_per == 4)
    hipLaunchKernelGGL((bat_cqk_solve_kernel<4, TIn>), grid, dim3(kBlock), 0, ctx->stream, A);
  else
    hipLaunchKernelGGL((bat_cqk_solve_kernel<8, TIn>), grid, dim3(kBlock), 0, ctx->stream, A);
}

template <typename TIn>
void launch_cqk_backward(cqk_ctx* ctx, const cqk_batch_schedule& sc, BatCqkArgs A) {
  dim3 grid;
  cqk_apply_schedule(ctx, sc, &A, &grid);
  plan(ctx, A);
  if (sc.small_per == 4)
    hipLaunchKernelGGL((bat_cqk_vjp_kernel<4, TIn>), grid, dim3(kBlock), 0, ctx->stream, A);
  else
    hipLaunchKernelGGL((bat_cqk_vjp_kernel<8, TIn>), grid, dim3(kBlock), 0, ctx->stream, A);
}

}  // namespace

namespace {
template <typename TIn>
cqk_status run_batched_cqk(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const TIn* d,
                           const TIn* a, const TIn* b, const TIn* l, const TIn* u,
                           const double* r, TIn* x, double* lambda_out, int32_t* status_out,
                           const cqk_opts& o, cqk_info* info) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  BatCqkArgs A = cqk_args(nseg, offsets, d, a, b, l, u, w);
  A.r = r;
  A.x = x;
  A.lam_out = lambda_out;
  A.status_out = status_out;
  A.lambda0_mode = o.lambda0_mode;
  A.lam0_user = o.lambda0_user;
  A.max_iter = o.max_iter;
  A.tol = (o.tol > 0.0) ? o.tol : std::pow(2.220446049250313e-16, 0.75);
  hipStream_t s = ctx->stream;
  if (o.timing) {
    st = ensure_events(ctx, 2);
    if (st != CQK_OK) return st;
    hipEventRecord(ctx->events[0], s);
  }
  launch_cqk_forward<TIn>(ctx, ctx->sched_cqk_fwd, A);
  if (o.timing) hipEventRecord(ctx->events[1], s);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  // the call's result from the device counters (host copy in hc)
  int32_t* hc = (int32_t*)ctx->host_pinned;
  const bool timing = o.timing != 0;
  auto fill = [ctx, hc, timing](cqk_info* inf) {
    const int flags = hc[CTR_FLAGS];
    int status = CQK_OK;
    if (flags & kBadValue) status = CQK_INVALID_ARG;
    else if (flags & kInfeasible) status = CQK_INFEASIBLE;
    else if (flags & kNotConverged) status = CQK_NOT_CONVERGED;
    std::memset(inf, 0, sizeof(*inf));
    inf->status = status;
    inf->iterations = hc[CTR_ITMAX];
    inf->passes = hc[CTR_ITSUM];
    if (timing) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]);
      inf->pass_ms = ms;
    }
  };
  int32_t* dc = A.counters;
  ctx->last = [hc, dc, fill](cqk_info* inf) -> cqk_status {
    if (hip_ok(hipMemcpy(hc, dc, CTR_TOTAL * sizeof(int32_t), hipMemcpyDeviceToHost)) != CQK_OK)
      return CQK_DEVICE_ERROR;
    fill(inf);
    return CQK_OK;
  };
  if (info) std::memset(info, 0, sizeof(*info));
  if (!o.sync) return CQK_OK;
  if (hip_ok(hipMemcpyAsync(hc, A.counters, CTR_TOTAL * sizeof(int32_t), hipMemcpyDeviceToHost,
                            s)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
  if (info) fill(info);
  return CQK_OK;
}

template <typename TIn>
cqk_status run_batched_cqk_backward(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const TIn* x, const TIn* g, const TIn* d, const TIn* b,
                                    const TIn* l, const TIn* u, TIn* grad_a, double* grad_r,
                                    const cqk_opts& o) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  BatCqkArgs A = cqk_args(nseg, offsets, d, nullptr, b, l, u, w);
  A.x = const_cast<TIn*>(x);
  A.g = g;
  A.ga = grad_a;
  A.gr = grad_r;
  launch_cqk_backward<TIn>(ctx, ctx->sched_cqk_bwd, A);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  ctx->last = ok_info;
  if (o.sync && hip_ok(hipStreamSynchronize(ctx->stream)) != CQK_OK) return CQK_DEVICE_ERROR;
  return CQK_OK;
}
}  // namespace

cqk_status run_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                               const double* d, const double* a, const double* b,
                               const double* l, const double* u, const double* r, double* x,
                               double* lambda_out, int32_t* status_out, const cqk_opts& o,
                               cqk_info* info) {
  return run_batched_cqk<double>(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out,
                                 status_out, o, info);
}

cqk_status run_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                               const float* d, const float* a, const float* b, const float* l,
                               const float* u, const double* r, float* x, double* lambda_out,
                               int32_t* status_out, const cqk_opts& o, cqk_info* info) {
  return run_batched_cqk<float>(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out, status_out,
                                o, info);
}

cqk_status run_batched_cqk_backward_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                        const double* x, const double* g, const double* d,
                                        const double* b, const double* l, const double* u,
                                        double* grad_a, double* grad_r, const cqk_opts& o) {
  return run_batched_cqk_backward<double>(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r,
                                          o);
}

cqk_status run_batched_cqk_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                        const float* x, const float* g, const float* d,
                                        const float* b, const float* l, const float* u,
                                        float* grad_a, double* grad_r, const cqk_opts& o) {
  return run_batched_cqk_backward<float>(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r,
                                         o);
}

namespace {
template <typename TIn>
cqk_status tune_batched_cqk(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const TIn* d,
                            const TIn* a, const TIn* b, const TIn* l, const TIn* u,
                            const double* r, TIn* x, const TIn* g, TIn* grad_a,
                            int32_t backward, int32_t repeats, cqk_batch_schedule* best,
                            double* best_ms) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  BatCqkArgs A = cqk_args(nseg, offsets, d, a, b, l, u, w);
  A.r = r;
  A.x = x;
  A.g = g;
  A.ga = grad_a;
  A.lambda0_mode = CQK_LAMBDA0_ZERO;
  A.max_iter = 100;
  A.tol = std::pow(2.220446049250313e-16, 0.75);
  cqk_batch_schedule cand[32];
  const int nc = candidate_schedules(cand, 32);
  int bi = 0;
  double ms = 0.0;
  if (backward)
    st = tune(ctx, cand, nc, repeats,
              [&](const cqk_batch_schedule& sc) { launch_cqk_backward<TIn>(ctx, sc, A); }, &bi,
              &ms);
  else
    st = tune(ctx, cand, nc, repeats,
              [&](const cqk_batch_schedule& sc) { launch_cqk_forward<TIn>(ctx, sc, A); }, &bi,
              &ms);
  if (st != CQK_OK) return st;
  (backward ? ctx->sched_cqk_bwd : ctx->sched_cqk_fwd) = cand[bi];
  if (best) *best = cand[bi];
  if (best_ms) *best_ms = ms;
  return CQK_OK;
}
}  // namespace

cqk_status tune_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const double* d, const double* a, const double* b,
                                const double* l, const double* u, const double* r, double* x,
                                const double* g, double* grad_a, int32_t backward,
                                int32_t repeats, cqk_batch_schedule* best, double* best_ms) {
  return tune_batched_cqk<double>(ctx, nseg, offsets, d, a, b, l, u, r, x, g, grad_a, backward,
                                  repeats, best, best_ms);
}

cqk_status tune_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const float* d, const float* a, const float* b, const float* l,
                                const float* u, const double* r, float* x, const float* g,
                                float* grad_a, int32_t backward, int32_t repeats,
                                cqk_batch_schedule* best, double* best_ms) {
  return tune_batched_cqk<float>(ctx, nseg, offsets, d, a, b, l, u, r, x, g, grad_a, backward,
                                 repeats, best, best_ms);
}

bool valid_schedule(const cqk_batch_schedule& sc) {
  return (sc.small_per == 4 || sc.small_per == 8) && sc.blocks_per_cu >= 1 &&
         sc.blocks_per_cu <= 8 && (sc.short_first == 0 || sc.short_first == 1) &&
         sc.medium_tiles >= 0 && sc.medium_tiles <= 64;
}


// The info record of the last batched forward call from the host copy of its
// counters.
void bat_fill_info(cqk_ctx* ctx, cqk_info* inf) {
  const int32_t* hc = (const int32_t*)ctx->host_pinned;
  const int flags = hc[CTR_FLAGS];
  int status = CQK_OK;
  if (flags & (kBadRadius | kBadValue)) status = CQK_INVALID_ARG;
  else if (flags & kInfeasible) status = CQK_INFEASIBLE;
  std::memset(inf, 0, sizeof(*inf));
  inf->status = status;
  inf->n_after_init = hc[CTR_SURV];
  inf->iterations = 0;
  inf->passes = 1;
  inf->rows_spilled = hc[CTR_OVER];
  if (ctx->bat_timing) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]);
    inf->pass_ms = ms;
  }
}

// Reads the outcome of the last batched forward call from its device
// counters (ctx->bat_counters) once the stream has finished it.
cqk_status bat_read_last(cqk_ctx* ctx, cqk_info* inf) {
  int32_t* hc = (int32_t*)ctx->host_pinned;
  if (hip_ok(hipMemcpy(hc, ctx->bat_counters, CTR_TOTAL * sizeof(int32_t),
                       hipMemcpyDeviceToHost)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  bat_fill_info(ctx, inf);
  return CQK_OK;
}

// One batched forward call with its planning buffers in w.  Allocates
// nothing unless o.timing asks for events the context does not have yet.
cqk_status run_batched_f32_on(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                              const float* y, const double* r, double r_scalar, float* x,
                              double* lambda_out, int32_t* nfree_out, const BatWs& w,
                              const cqk_opts& o, cqk_info* info) {
  const BatArgs A = forward_args(nseg, offsets, y, r, r_scalar, x, lambda_out, nfree_out, w);
  hipStream_t s = ctx->stream;
  if (o.timing) {
    cqk_status st = ensure_events(ctx, 2);
    if (st != CQK_OK) return st;
    hipEventRecord(ctx->events[0], s);
  }
  launch_forward(ctx, ctx->sched_fwd, A);
  if (o.timing) hipEventRecord(ctx->events[1], s);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  ctx->bat_counters = A.counters;
  ctx->bat_timing = o.timing != 0;
  // one captured pointer: std::function keeps it without a heap allocation
  ctx->last = [ctx](cqk_info* inf) -> cqk_status { return bat_read_last(ctx, inf); };
  if (info) std::memset(info, 0, sizeof(*info));
  if (!o.sync) return CQK_OK;
  if (hip_ok(hipMemcpyAsync(ctx->host_pinned, A.counters, CTR_TOTAL * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s)) != CQK_OK)
    return CQK_DEVICE_ERROR;
  if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
  if (info) bat_fill_info(ctx, info);
  return CQK_OK;
}

cqk_status run_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const float* y,
                           const double* r, double r_scalar, float* x, double* lambda_out,
                           int32_t* nfree_out, const cqk_opts& o, cqk_info* info) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  return run_batched_f32_on(ctx, nseg, offsets, y, r, r_scalar, x, lambda_out, nfree_out, w, o,
                            info);
}

cqk_status noalloc_scratch(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return CQK_DEVICE_ERROR;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    // the caller made `device` current
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CQK_DEVICE_ERROR;
    }
    addr[device] = p;
  }
  *out = addr[device];
  return CQK_OK;
}

cqk_status run_batched_noalloc_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                   const float* y, const double* r, double r_scalar, float* x,
                                   double* lambda_out, int32_t* nfree_out, const cqk_opts& o,
                                   cqk_info* info) {
  if (nseg > CQK_NOALLOC_MAX_SEG) return CQK_BUFFER_TOO_SMALL;
  if (!ctx->scratch) return CQK_DEVICE_ERROR;
  BatWs w;
  bat_layout(ctx->scratch, nseg, &w);
  cqk_opts o2 = o;
  o2.timing = 0;  // events would be created on first use
  return run_batched_f32_on(ctx, nseg, offsets, y, r, r_scalar, x, lambda_out, nfree_out, w, o2,
                            info);
}

cqk_status run_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const float* x, const float* g, float* grad_y,
                                    double* grad_r, const cqk_opts& o) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  launch_backward(ctx, ctx->sched_bwd, backward_args(nseg, offsets, x, g, grad_y, grad_r, w));
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  ctx->last = ok_info;
  if (o.sync && hip_ok(hipStreamSynchronize(ctx->stream)) != CQK_OK) return CQK_DEVICE_ERROR;
  return CQK_OK;
}

cqk_status tune_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const float* y,
                            const double* r, double r_scalar, float* x, int32_t repeats,
                            cqk_batch_schedule* best, double* best_ms) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  const BatArgs A = forward_args(nseg, offsets, y, r, r_scalar, x, nullptr, nullptr, w);
  cqk_batch_schedule cand[128];
  const int nc = candidate_schedules_fwd(cand, 128);
  int bi = 0;
  double ms = 0.0;
  st = tune(ctx, cand, nc, repeats,
            [&](const cqk_batch_schedule& sc) { launch_forward(ctx, sc, A); }, &bi, &ms);
  if (st != CQK_OK) return st;
  ctx->sched_fwd = cand[bi];
  if (best) *best = cand[bi];
  if (best_ms) *best_ms = ms;
  return CQK_OK;
}

cqk_status tune_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                     const float* x, const float* g, float* grad_y,
                                     int32_t repeats, cqk_batch_schedule* best,
                                     double* best_ms) {
  BatWs w;
  cqk_status st = bat_workspace(ctx, nseg, &w);
  if (st != CQK_OK) return st;
  const BatArgs A = backward_args(nseg, offsets, x, g, grad_y, nullptr, w);
  cqk_batch_schedule cand[128];
  const int nc = candidate_schedules_fwd(cand, 128);
  int bi = 0;
  double ms = 0.0;
  st = tune(ctx, cand, nc, repeats,
            [&](const cqk_batch_schedule& sc) { launch_backward(ctx, sc, A); }, &bi, &ms);
  if (st != CQK_OK) return st;
  ctx->sched_bwd = cand[bi];
  if (best) *best = cand[bi];
  if (best_ms) *best_ms = ms;
  return CQK_OK;
}

}  // namespace cqk
