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
// Layout: the grid is G0 blocks of 4 waves.  Passes over y hand its tiles to
// the waves grid-stride (tile t to wave t mod NR); wave w writes the values
// it keeps, with their indices in y, to region w of a compacted set (ballot
// + lane prefix counts: deterministic, no block-wide synchronisation), and
// later passes stream those regions.
//
// Kernels:
//   spx_condat_sample_kernel  Algorithm 2 on a sample of up to 1024 tiles
//                           spread evenly over y: every thread runs it on 16
//                           register-resident values above the tile's first
//                           bound, the wave merges the lanes' sets into lam_J
//                           bounds and refines them; block records of the
//                           smallest bound and of the kept sets' counts and
//                           sums.
//   spx_condat_kernel       one read of y (and x = 0 written over it),
//                           starting from the sample's bound: each wave keeps
//                           every value above its running bound, which the
//                           kept values lower further (wave reductions only,
//                           no barriers); a tile with no value above it costs
//                           one test.
//   spx_condat_merge_kernel lam_0 = the smallest bound any wave found and the
//                           bound of the union of every surviving set.
//   spx_pass_kernel<MULTI>  right after the start: the survivors' counts and
//                           sums at 12 candidate points give 12 more bounds,
//                           the smallest becomes lam_0 (spx_start_update_kernel).
//   spx_formula_kernel      eq. (CQKlambda0) start, plus max y.
//   spx_pass_kernel         one evaluation of phi and the counts over the
//                           current set; drops y + lam_k <= 0 (valid because
//                           lam_k >= lam*, Theorem 1).
//   spx_update_kernel       Algorithm 4's update (one block); once the next set
//                           fits in LDS the grid pass before it packs the set
//                           densely and this kernel runs every remaining
//                           iteration inside its block.
//   spx_tail_kernel         the same loop for an input that fits from the
//                           start (read from y).
//   spx_finalize_kernel     dense x = max(0, y + lam*) (or 0, or a copy of y);
//   spx_scatter_kernel      x[idx] for the surviving indices when the rest of
//                           x is known to be zero.
// The finalize kernels do nothing while the loop is still running, so the
// host queues them behind every batch of iterations and waits once per batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kRBlock = 1024;  // one-block kernels (reductions, the tail loop)
constexpr int kWaves = kBlock / kWave;
constexpr int kCondatK = 16;   // values per lane per tile in Algorithm 2
constexpr int kRefine = 8;     // refinement rounds on a sample tile
constexpr int kTailBytes = 128 * 1024;  // LDS copy of the set the tail loop runs on
constexpr int kCand = 12;               // start refinement candidates

// Tail states (SpxState::tail): the set of the next evaluation fits the
// one-block loop.
//   kTailPack: it sits in compacted regions; the next grid pass copies them
//              densely to tval/tidx (at offsets this block writes to toff),
//              and the update kernel after it runs the loop on that copy;
//   kTailY:    the caller's y itself is that small (run from y at once).
enum : int32_t { kTailNone = 0, kTailPack = 1, kTailY = 2 };

struct SpxArgs {
  const void* y;
  const void* xw;    // primal estimate of a warm start (or null), TIn
  void* x;
  int64_t n;
  int64_t chunk0;    // block region of the original layout; wave region = chunk0/4
  void* val[2];      // compacted values (signed y), TIn
  uint32_t* idx[2];  // their indices in y
  int32_t* cnt[2];   // per-wave-region counts of each buffer
  void* tval;        // dense copy of the set the tail loop runs on (TIn)
  uint32_t* tidx;    // its indices in y
  int32_t* toff;     // per wave region: offset of its survivors in that copy
  double* partials;
  SpxState* st;
  cqk_trace_rec* trace;
  // Algorithm 2 sample: samp_waves waves over samp_ntiles tiles of y; its
  // block records (samp_blocks of them, value-major)
  double* samp;
  int64_t samp_ntiles;
  int32_t samp_waves;
  int32_t samp_blocks;
  // sparse output (x is null then)
  uint32_t* bm;      // one bit per index, ceil(n/32) words
  int64_t nwords;
  int64_t sp_wpb;    // bitmap words per block of the count and write kernels
  int32_t* sp_cnt;   // per block: set bits in its words
  int64_t* sp_idx;   // caller's output: indices, values
  void* sp_val;
  int64_t sp_cap;
};

template <typename T>
__device__ __forceinline__ T absval(T v) {
  return v < T(0) ? -v : v;
}

__device__ __forceinline__ void spx_trace(SpxState* st, cqk_trace_rec* tr, int kind, int compacted, int source,
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

__device__ __forceinline__ void spx_finish(SpxState* st, double lamf, int reason) {
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

// Loads V consecutive values of y starting at i (count-guarded; one 16-byte
// load when the vector is in range).
template <typename TIn>
__device__ __forceinline__ void load_y(const TIn* y, int64_t i, int64_t n, TIn* o) {
  constexpr int V = VecWidth<TIn>::value;
  if (i + V <= n) {
    const typename Raw16<TIn>::type v = ld16(y + i);
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (i + k < n) ? y[i + k] : TIn(0);
  }
}

// NL vectors per lane at base + q*64*V + lane*V, q < NL; when the whole tile
// is in range every load is issued before the first use.
template <typename TIn, int NL>
__device__ __forceinline__ void load_tile(const TIn* y, int64_t base, int lane, int64_t n,
                                          TIn* o) {
  constexpr int V = VecWidth<TIn>::value;
  if (base + (int64_t)NL * kWave * V <= n) {
    typename Raw16<TIn>::type r[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) r[q] = ld16(y + base + (int64_t)q * kWave * V + lane * V);
#pragma unroll
    for (int q = 0; q < NL; ++q)
#pragma unroll
      for (int k = 0; k < V; ++k) o[q * V + k] = r[q][k];
  } else {
#pragma unroll
    for (int q = 0; q < NL; ++q)
      load_y<TIn>(y, base + (int64_t)q * kWave * V + lane * V, n, &o[q * V]);
  }
}

// load_tile and zero_tile for a tile known to be in range: no checks.
template <typename TIn, int NL>
__device__ __forceinline__ void load_tile_full(const TIn* y, int64_t base, int lane, TIn* o) {
  constexpr int V = VecWidth<TIn>::value;
  typename Raw16<TIn>::type r[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) r[q] = ld16(y + base + (int64_t)q * kWave * V + lane * V);
#pragma unroll
  for (int q = 0; q < NL; ++q)
#pragma unroll
    for (int k = 0; k < V; ++k) o[q * V + k] = r[q][k];
}

template <typename TIn, int NL>
__device__ __forceinline__ void zero_tile_full(TIn* x, int64_t base, int lane) {
  constexpr int V = VecWidth<TIn>::value;
  typename Raw16<TIn>::type z;
#pragma unroll
  for (int k = 0; k < V; ++k) z[k] = TIn(0);
#pragma unroll
  for (int q = 0; q < NL; ++q) st16(x + base + (int64_t)q * kWave * V + lane * V, z);
}

// |v| when mask clears the sign bit (l1), v when it is all ones.
__device__ __forceinline__ float abs_if(float v, uint32_t mask) {
  return __int_as_float((int)((uint32_t)__float_as_int(v) & mask));
}
__device__ __forceinline__ double abs_if(double v, uint32_t mask) {
  return __hiloint2double((int)((uint32_t)__double2hiint(v) & mask), __double2loint(v));
}

// The largest T not above x (so that v > result never drops a v > x).
template <typename T>
__device__ __forceinline__ T round_down_to(double x);
template <>
__device__ __forceinline__ float round_down_to<float>(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -__builtin_huge_valf());
  return f;
}
template <>
__device__ __forceinline__ double round_down_to<double>(double x) {
  return x;
}

// Zeros at the NL vectors per lane load_tile reads.
template <typename TIn, int NL>
__device__ __forceinline__ void zero_tile(TIn* x, int64_t base, int lane, int64_t n) {
  constexpr int V = VecWidth<TIn>::value;
  typename Raw16<TIn>::type z;
#pragma unroll
  for (int k = 0; k < V; ++k) z[k] = TIn(0);
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int64_t i = base + (int64_t)q * kWave * V + lane * V;
    if (i + V <= n) {
      st16(x + i, z);
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (i + k < n) x[i + k] = TIn(0);
    }
  }
}

// Partial record of the streaming Algorithm 2 kernel.
// C_CNTI, C_SUMI: the kept values of a warm start's support I.
enum { C_CNT = 0, C_SUM, C_ABS, C_BAD, C_NOUT, C_CNTI, C_SUMI, C_NSUM };
constexpr int C_NPART = C_NSUM + 3;  // + min lam, max v, max v over I
// Block record of the sample kernel (value-major, like the partial records):
// the smallest bound its waves found, and the count and sum of the sets they
// kept.
enum { SM_LAM = 0, SM_CNT, SM_SUM, SM_N };
constexpr int kSampleWaves = 1024;  // tiles in the sample, at most

// Algorithm 2 on a sample of y (Section 2.2, Section 4).  Wave w of the ns
// sample waves takes tile floor(w * ntiles / ns), so the sample is spread
// evenly over y and holds distinct tiles when ntiles >= ns.  The wave's first
// bound is lam_J of the tile's largest value alone (Algorithm 2's first set);
// each thread runs Algorithm 2 on its K values above that bound, and the wave
// merges the lanes' sets into lam_J of their union and refines it with
//   lam <- lam_J'  with  J' = {j in J : y_j + lam > 0},
// each step of which can only lower lam (Algorithm 4's step on the tile's own
// sub-problem).  Every bound is lam_J of a non-empty J, hence >= lam*
// (eq. (lambdaJ)), and so is lam_J of the union of the waves' final sets,
// which the streaming kernel forms from the block records.
// The kernel also starts the solve: `init` is the solve's initial state,
// which block 0 stores (no kernel of the call runs before this one).
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_condat_sample_kernel(SpxArgs A, SpxState init) {
  SpxState* st = A.st;
  if (blockIdx.x == 0 && threadIdx.x == 0) *st = init;
  if (init.status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  constexpr int K = kCondatK;
  constexpr int NL = K / V;  // vector loads per lane per tile
  constexpr int64_t TILE = (int64_t)kWave * K;
  const bool l1 = init.l1 != 0;
  const TA r = (TA)init.r;
  const double rd = init.r;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = (int)(threadIdx.x / kWave);
  const int w = blockIdx.x * kWaves + wid;
  const int ns = A.samp_waves;
  const int64_t count = A.n;
  const uint32_t amask = l1 ? 0x7FFFFFFFu : 0xFFFFFFFFu;
  __shared__ double lds[SM_N * kWaves];

  double lam_b = inf_d(), nk = 0.0, ks = 0.0;
  if (w < ns) {
    const int64_t base = (int64_t)w * A.samp_ntiles / ns * TILE;
    TIn yv[K];
    const bool full = base + TILE <= count;
    if (full)
      load_tile_full<TIn, NL>((const TIn*)A.y, base, lane, yv);
    else
      load_tile<TIn, NL>((const TIn*)A.y, base, lane, count, yv);
    TIn av[K];  // the values Algorithm 2 sees: y, or |y| for l1
    uint32_t inm = 0;
    TIn tmax = -(TIn)__builtin_huge_val();
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t i = base + (int64_t)q * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = q * V + k;
        const bool in = full || (i + k < count);
        av[e] = abs_if(yv[e], amask);
        inm |= in ? (1u << e) : 0u;
        tmax = max(tmax, in ? av[e] : -(TIn)__builtin_huge_val());
      }
    }
    const double m = wave_max((double)tmax);
    if (m > -inf_d()) {
      const double lam_first = rd - m;
      // values at or below -lam_first are zero at the solution; the threshold
      // is rounded down into TIn so that the test keeps every value it must
      const TIn thr = round_down_to<TIn>(-lam_first);
      uint32_t active = 0;
#pragma unroll
      for (int e = 0; e < K; ++e) active |= (((inm >> e) & 1u) && av[e] > thr) ? (1u << e) : 0u;
      double lb = lam_first;
      if (__ballot(active != 0u) != 0) {
        TA v[K];
#pragma unroll
        for (int e = 0; e < K; ++e) v[e] = (TA)av[e];
        int c = 0;
        TA S = TA(0);
        uint32_t J;
        if (__ballot(__popc(active) > 1) != 0) {
          J = condat_thread<K, TA>(v, active, r, l1, c, S);
        } else {
          // at most one value per lane: it joins J (l1: if non-zero)
          J = 0;
#pragma unroll
          for (int e = 0; e < K; ++e) {
            if (((active >> e) & 1u) && (!l1 || v[e] > TA(0))) {
              J |= 1u << e;
              c += 1;
              S += v[e];
            }
          }
        }
        const double lam_t = (c > 0) ? (rd - (double)S) / (double)c : inf_d();
        const double ct = wave_sum((double)c);
        const double skt = wave_sum((double)S);
        if (ct > 0.0) lb = fmin(lb, (rd - skt) / ct);
        uint32_t keep = 0;
        auto select = [&](double bound) {
          const TA lt = (TA)fmin(lam_t, bound);
          keep = 0;
          nk = 0.0;
          ks = 0.0;
#pragma unroll
          for (int e = 0; e < K; ++e) {
            if (((J >> e) & 1u) && (v[e] + lt > TA(0))) {
              keep |= 1u << e;
              nk += 1.0;
              ks += (double)v[e];
            }
          }
        };
        for (int it = 0; it < kRefine; ++it) {
          select(lb);
          const double kc = wave_sum(nk), kss = wave_sum(ks);
          if (kc == 0.0) break;
          const double nl = (rd - kss) / kc;
          if (!(nl < lb)) break;
          lb = nl;
        }
        select(lb);
        // with tracing on, lane 0 of the wave on tile 0 records its own
        // Algorithm 2: the values it saw, J, the thread's bound and the values
        // the wave's refined bound kept
        if (w == 0 && lane == 0 && init.trace_cap > 0) {
          cqk_trace_rec& t = A.trace[0];
          t.iter = 0;
          t.kind = 7;
          t.compacted = c;
          t.source = (int32_t)keep;
          t.lam = lam_t;
          t.phi = (double)S;
          t.slope = (double)thr;
          t.lo = lb;
          t.hi = (double)base;
          t.n_in = (int64_t)active;
          t.n_out = (int64_t)J;
          st->ntrace = 1;
        }
      }
      lam_b = lb;
    }
  }
  const double wc = wave_sum(nk), wsum = wave_sum(ks);
  if (lane == 0) {
    lds[SM_LAM * kWaves + wid] = lam_b;
    lds[SM_CNT * kWaves + wid] = wc;
    lds[SM_SUM * kWaves + wid] = wsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = lds[SM_LAM * kWaves], b = lds[SM_CNT * kWaves], c = lds[SM_SUM * kWaves];
    for (int i = 1; i < kWaves; ++i) {
      a = fmin(a, lds[SM_LAM * kWaves + i]);
      b += lds[SM_CNT * kWaves + i];
      c += lds[SM_SUM * kWaves + i];
    }
    A.samp[SM_LAM * gridDim.x + blockIdx.x] = a;
    A.samp[SM_CNT * gridDim.x + blockIdx.x] = b;
    A.samp[SM_SUM * gridDim.x + blockIdx.x] = c;
  }
}

// The streaming pass of the Algorithm 2 start (Section 2.2, Section 4): one
// read of y, and x = 0 written over it.  Every wave starts from the bound the
// sample gives (the smallest bound of its waves and lam_J of the union of
// their sets) and takes tiles grid-stride.  In each tile it keeps every value
// above its running bound (l1: if non-zero); the kept values join its set J,
// and the bound becomes min(bound, lam_J): still >= lam*, so the values at or
// below -bound are zero at the solution.  Most tiles hold no value above the
// bound and cost one test on the lanes' maxima.
//
// WARM: also the warm start of Section 3.1 from a primal estimate xbar, with
// I = {xbar > 0} (l1: xbar != 0).  The kernel runs as without it: every bound
// it finds is lam_J of some non-empty J, so it fixes values at zero whatever
// J is.  It also sums the kept values of I and takes the largest value of I,
// from which the merge forms the estimate's lam_J.
template <typename TIn, bool WARM>
__global__ __launch_bounds__(kBlock) void spx_condat_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  constexpr int K = kCondatK;
  constexpr int NL = K / V;  // vector loads per lane per tile
  constexpr int64_t TILE = (int64_t)kWave * K;
  static_assert(K < 32, "a lane's kept count must fit in five bits");
  const bool l1 = st->l1 != 0;
  const double rd = st->r;
  const int lane = threadIdx.x & (kWave - 1);
  const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
  // tiles go to waves grid-stride (tile t to wave t mod NR); wave rid keeps
  // its survivors in region rid, which holds every value the wave reads
  const int64_t nr = (int64_t)gridDim.x * kWaves;
  const int64_t cw = A.chunk0 / kWaves;
  const int64_t count = A.n;
  const TIn* y = (const TIn*)A.y;
  TIn* x = (TIn*)A.x;
  TIn* outv = (TIn*)A.val[1] + (int64_t)rid * cw;
  uint32_t* outi = A.idx[1] + (int64_t)rid * cw;

  __shared__ double lds[C_NPART * (kBlock / kWave)];
  __shared__ double tot[C_NPART];

  // the sample's bound (every wave forms the same value)
  double lam_min;
  {
    const int g = A.samp_blocks;
    double sl = inf_d(), sc = 0.0, ss = 0.0;
    for (int i = lane; i < g; i += kWave) {
      sl = fmin(sl, A.samp[SM_LAM * g + i]);
      sc += A.samp[SM_CNT * g + i];
      ss += A.samp[SM_SUM * g + i];
    }
    sl = wave_min(sl);
    sc = wave_sum(sc);
    ss = wave_sum(ss);
    lam_min = (sc > 0.0) ? fmin(sl, (rd - ss) / sc) : sl;
    // NaN only from invalid data, which the merge reports
    if (!(lam_min <= inf_d())) lam_min = inf_d();
  }
  // wave-uniform: the values this wave kept so far
  double run_c = 0.0, run_s = 0.0;
  double acc[C_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  double abs_sum = 0.0;            // sum |y| (l1 only)
  double run_ci = 0.0, run_si = 0.0;  // kept values of I (WARM)
  TIn vmx = -(TIn)__builtin_huge_val();
  TIn vmxI = -(TIn)__builtin_huge_val();
  TIn badacc = TIn(0);             // NaN once any y is NaN or infinite
  int64_t written = 0;
  const uint32_t amask = l1 ? 0x7FFFFFFFu : 0xFFFFFFFFu;
  // -lam_min rounded down into TIn, recomputed only when lam_min moves
  TIn thr = -(TIn)__builtin_huge_val();
  double thr_of = 0.0;
  bool thr_set = false;
  // One tile; `full` (a tile wholly in range) is known at compile time, so
  // the in-range tests of the other tiles cost nothing here.
  // yv: the tile's values, loaded by the caller
  auto tile = [&](const int64_t base, auto full_tag, const TIn* yv) {
    constexpr bool full = decltype(full_tag)::value;
    TIn av[K];  // y, or |y| for l1
    uint32_t inI = 0xFFFFFFFFu;  // the values of I (WARM)
    if constexpr (WARM) {
      TIn xv[K];
      load_tile<TIn, NL>((const TIn*)A.xw, base, lane, count, xv);
      inI = 0;
#pragma unroll
      for (int e = 0; e < K; ++e) inI |= (l1 ? (xv[e] != TIn(0)) : (xv[e] > TIn(0))) ? (1u << e) : 0u;
    }
    // x_i = 0 for every index (survivors get their value from the scatter at
    // the end); a sparse output has no x
    if (x != nullptr) {
      if constexpr (full)
        zero_tile_full<TIn, NL>(x, base, lane);
      else
        zero_tile<TIn, NL>(x, base, lane, count);
    }
    TIn tmax = -(TIn)__builtin_huge_val();
    TIn tmaxI = -(TIn)__builtin_huge_val();
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t i = base + (int64_t)q * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = q * V + k;
        const bool in = full || (i + k < count);
        av[e] = abs_if(yv[e], amask);
        badacc += in ? yv[e] * TIn(0) : TIn(0);
        if (l1) abs_sum += in ? (double)av[e] : 0.0;
        tmax = max(tmax, in ? av[e] : -(TIn)__builtin_huge_val());
        if constexpr (WARM)
          tmaxI = max(tmaxI, (in && ((inI >> e) & 1u)) ? av[e] : -(TIn)__builtin_huge_val());
      }
    }
    vmx = max(vmx, tmax);
    if constexpr (WARM) vmxI = max(vmxI, tmaxI);
    // no bound yet (a sample that found none): lam_J of the tile's largest
    // value alone
    if (lam_min == inf_d()) {
      const double m = wave_max((double)tmax);
      if (m > -inf_d()) lam_min = rd - m;
    }
    if (!thr_set || lam_min != thr_of) {
      thr = round_down_to<TIn>(-lam_min);
      thr_of = lam_min;
      thr_set = true;
    }
    if (__ballot(tmax > thr) == 0) return;
    uint32_t keep = 0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int64_t i = base + (int64_t)q * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = q * V + k;
        const bool in = full || (i + k < count);
        keep |= (in && av[e] > thr && (!l1 || av[e] > TIn(0))) ? (1u << e) : 0u;
      }
    }
    // this lane's place among the wave's kept values: its count (five bits)
    // summed over the lanes below it, one bit at a time
    const int c = __popc(keep);
    int pre = 0, nt = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const uint64_t m = __ballot((c >> b) & 1);
      pre += lane_prefix(m) << b;
      nt += __popcll(m) << b;
    }
    if (nt == 0) return;
    int64_t pos = written + pre;
    double ks = 0.0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      if ((keep >> (q * V)) & ((1u << V) - 1u)) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int e = q * V + k;
          if ((keep >> e) & 1u) {
            outv[pos] = yv[e];
            outi[pos] = (uint32_t)(base + (int64_t)q * kWave * V + (int64_t)lane * V + k);
            ks += (double)av[e];
            ++pos;
          }
        }
      }
    }
    if constexpr (WARM) {
      double ci = 0.0, si = 0.0;
#pragma unroll
      for (int e = 0; e < K; ++e) {
        const bool kI = ((keep & inI) >> e) & 1u;
        ci += kI ? 1.0 : 0.0;
        si += kI ? (double)av[e] : 0.0;
      }
      run_ci += wave_sum(ci);
      run_si += wave_sum(si);
    }
    written += nt;
    run_c += (double)nt;
    run_s += wave_sum(ks);
    lam_min = fmin(lam_min, (rd - run_s) / run_c);
  };
  const int64_t stride = nr * TILE;
  for (int64_t base = (int64_t)rid * TILE; base < count; base += stride) {
    TIn ycur[K];
    if (base + TILE <= count) {
      load_tile_full<TIn, NL>(y, base, lane, ycur);
      tile(base, std::true_type{}, ycur);
    } else {
      load_tile<TIn, NL>(y, base, lane, count, ycur);
      tile(base, std::false_type{}, ycur);
    }
  }
  if (lane == 0) {
    acc[C_CNT] = run_c;
    acc[C_SUM] = run_s;
    acc[C_NOUT] = (double)written;
    acc[C_CNTI] = run_ci;
    acc[C_SUMI] = run_si;
    A.cnt[1][rid] = (int32_t)written;
  } else {
    acc[C_CNT] = acc[C_SUM] = acc[C_NOUT] = acc[C_CNTI] = acc[C_SUMI] = 0.0;
  }
  acc[C_BAD] = (badacc == TIn(0)) ? 0.0 : 1.0;
  acc[C_ABS] = abs_sum;
  const double vmax[2] = {(double)vmx, (double)vmxI};
  block_reduce<C_NSUM, 1, 2, kBlock>(acc, &lam_min, vmax, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, C_NPART);
}

// Partial record of an evaluation pass.
enum { S_PHI = 0, S_CM, S_CP, S_BAD, S_NIN, S_NOUT, S_ABS, S_NSUM };  // + max v
constexpr int kPassRec = S_NSUM + 1;
// a MULTI pass's record: the S_NSUM sums, then 2 * kCand candidate sums

// Algorithm 4's update, run by one thread after an evaluation (source: 0 the
// caller's y, 1/2 a compacted buffer, 3 the packed set of the tail loop).
__device__ __forceinline__ void spx_update(SpxState* st, const double* t, double vmax, cqk_trace_rec* tr,
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
  // selects rather than branches, so the state stays in registers
  const bool below = (k == 0 && phi < r);
  const double slope = below ? cp : cm;
  st->lo = below ? lam : st->lo;
  st->hi = (!below && phi > r) ? lam : st->hi;
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
  if (st->n_src <= st->tail_cap && st->src != 0) st->tail = kTailPack;
  if (st->iter >= st->max_iter) {
    st->status = CQK_NOT_CONVERGED;
    st->lam_final = lam;
  }
}

// Shared memory of the tail loop; a kernel that may run the loop declares one.
template <typename TIn, typename TA>
struct TailLds {
  static constexpr int CAP = kTailBytes / (int)sizeof(TIn);
  static constexpr int NW = kRBlock / kWave;
  TIn tv[CAP];
  int off[NW + 1];
  double lds[(S_NSUM + 1) * NW];
  double tot[S_NSUM + 1];
  TA phl[NW];
  int run;
  double lam;
};

// Exclusive prefix of the region counts of buffer si (one block of kRBlock
// threads): toff[r] = sum of counts of regions < r.
__device__ __forceinline__ void spx_tail_offsets(const SpxArgs& A, int NR, int si, int* lds_i) {
  constexpr int P = 8;  // regions per thread per round
  int base = 0;
  for (int r0 = 0; r0 < NR; r0 += kRBlock * P) {
    int c[P];
    int csum = 0;
    const int rb = r0 + threadIdx.x * P;
    if (rb + P <= NR) {
      // two 16-byte loads (the count arrays are 256-byte aligned, rb % 8 == 0)
      const int4v* cp = reinterpret_cast<const int4v*>(A.cnt[si] + rb);
      const int4v c0 = cp[0], c1 = cp[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = c0[j];
        c[4 + j] = c1[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < P; ++j) c[j] = (rb + j < NR) ? A.cnt[si][rb + j] : 0;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) csum += c[j];
    int totc;
    int ex = base + block_excl_scan<kRBlock>(csum, lds_i, &totc);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int r = r0 + threadIdx.x * P + j;
      if (r < NR) A.toff[r] = ex;
      ex += c[j];
    }
    base += totc;
  }
}

// The remaining Newton iterations inside one block of kRBlock threads, on a
// copy of the current set in LDS (the caller's y when it is small from the
// start, else the dense copy the last grid pass made, whose indices stay in
// tidx for the final scatter).  Each iteration is one sweep of LDS.
// `sc` is thread 0's copy of the state (status running, tail set); src and
// l1 are the block-uniform values of that state.  Thread 0 stores the state
// back when the loop has stopped.
template <typename TIn, typename TA>
__device__ __forceinline__ void spx_tail_run(const SpxArgs& A, int64_t total, SpxState& sc,
                                             int src, bool l1, TailLds<TIn, TA>& L) {
  constexpr int CAP = TailLds<TIn, TA>::CAP;
  constexpr int NW = TailLds<TIn, TA>::NW;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  if (total > CAP) {
    // the updates only hand over sets that fit
    if (threadIdx.x == 0) {
      sc.status = CQK_DEVICE_ERROR;
      *A.st = sc;
    }
    return;
  }
  const int m = (int)total;
  const TIn* from = (src == 0) ? (const TIn*)A.y : (const TIn*)A.tval;
#pragma unroll 4
  for (int i = threadIdx.x; i < m; i += kRBlock) L.tv[i] = from[i];
  if (threadIdx.x == 0) L.lam = sc.lam;
  __syncthreads();
  for (;;) {
    const TA lam = (TA)L.lam;
    TA phi = TA(0);
    double acc[S_NSUM] = {0, 0, 0, 0, 0, 0, 0};
    double vmax = -inf_d();
    int cm = 0, cp = 0;
#pragma unroll 4
    for (int i = threadIdx.x; i < m; i += kRBlock) {
      const TA t = (TA)L.tv[i];
      const TA vv = l1 ? absval(t) : t;
      const TA z = vv + lam;
      phi += z > TA(0) ? z : TA(0);
      cm += z > TA(0) ? 1 : 0;
      cp += z >= TA(0) ? 1 : 0;
      if (src == 0) {
        const double td = (double)t;
        acc[S_ABS] += fabs(td);
        acc[S_BAD] += (fabs(td) < inf_d()) ? 0.0 : 1.0;
        vmax = fmax(vmax, (double)vv);
      }
    }
    acc[S_CM] = (double)cm;
    acc[S_CP] = (double)cp;
    acc[S_NIN] = (threadIdx.x == 0) ? (double)m : 0.0;
    const TA phw = wave_sum(phi);
    if (lane == 0) L.phl[wid] = phw;
    block_reduce<S_NSUM, 0, 1, kRBlock>(acc, nullptr, &vmax, L.lds, L.tot);
    if (threadIdx.x == 0) {
      TA pb = L.phl[0];
      for (int w = 1; w < NW; ++w) pb += L.phl[w];
      double t[S_NSUM + 1];
      for (int i = 0; i < S_NSUM + 1; ++i) t[i] = L.tot[i];
      t[S_PHI] = (double)pb;
      spx_update(&sc, t, t[S_NSUM], A.trace, false, src == 0 ? 0 : 3);
      L.run = (sc.status == kRunning) ? 1 : 0;
      L.lam = sc.lam;
    }
    __syncthreads();
    if (!L.run) break;
  }
  if (threadIdx.x == 0) {
    sc.tail = kTailNone;
    if (src != 0) {
      sc.src = 3;  // the dense list: the scatter reads it
      sc.n_src = m;
    }
    *A.st = sc;
  }
}

// Shared flags handed from thread 0 to the block: enter the tail loop (or
// write the region offsets for the pack), and the state's src and l1.
struct TailGo {
  int go, offsets, src, l1;
  int64_t n;
};

__device__ __forceinline__ void tail_flags(TailGo* f, const SpxState& s, bool run_now) {
  const bool running = s.status == kRunning;
  f->go = (running && run_now) ? 1 : 0;
  f->offsets = (running && !run_now && s.tail == kTailPack) ? 1 : 0;
  f->src = s.src;
  f->l1 = s.l1;
  f->n = s.n_src;
}

// The loop over y itself when the instance is that small from the start.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kRBlock) void spx_tail_kernel(SpxArgs A) {
  __shared__ TailLds<TIn, TA> L;
  __shared__ TailGo f;
  SpxState sc;
  if (threadIdx.x == 0) {
    sc = *A.st;
    tail_flags(&f, sc, sc.tail == kTailY);
  }
  __syncthreads();
  if (f.go) spx_tail_run<TIn, TA>(A, A.n, sc, 0, f.l1 != 0, L);
}

// Merges the blocks of spx_condat_kernel (one block): lam_0 is the smallest
// of the bounds the waves found and the bound of the union of every
// surviving set (all of them >= lam*), the l1 ball test, and the survivor
// count; a set that fits goes straight into the tail loop.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kRBlock) void spx_condat_merge_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[C_NPART * (kRBlock / kWave)];
  __shared__ double tot[C_NPART];
  __shared__ int offl[kRBlock / kWave + 1];
  __shared__ TailGo f;
  reduce_partials<C_NSUM, 1, 2, kRBlock>(A.partials, G, lds, tot);
  SpxState s;
  if (threadIdx.x == 0) {
    double lam_w = __builtin_nan("");
    s = *st;
    s.passes += 1;
    s.sum_abs = tot[C_ABS];
    s.vmax = tot[C_NSUM + 1];
    s.x_zeroed = 1;
    if (tot[C_BAD] > 0.0) {
      s.status = CQK_INVALID_ARG;
    } else if (s.l1 && tot[C_ABS] <= s.r) {
      s.fin_mode = kFinCopy;
      spx_finish(&s, 0.0, 5);
    } else {
      const double m = tot[C_CNT];
      const double wb = tot[C_NSUM];  // the smallest bound a wave found
      const double vmaxI = tot[C_NSUM + 2];
      s.n_init = (int64_t)tot[C_NOUT];
      s.src = 2;  // the survivors sit in buffer 1, one region per wave
      s.n_src = (int64_t)tot[C_NOUT];
      // lam_J of the union of the kept sets, and the smallest wave bound
      double lam0 = fmin((m > 0.0) ? (s.r - tot[C_SUM]) / m : wb, wb);
      if (s.warm && !(vmaxI > -inf_d())) {
        // warm start with an empty support: the fallback of Section 3.1,
        // lam_0 = max{r/n, -max v}.  It is not known to be >= lam*, so
        // Algorithm 4 starts from it as from the formula start (its first
        // step decides the side, compaction follows).  The buffer lost only
        // values below a lam_J, zero at the solution: the reduced problem
        // has the same multiplier.
        lam_w = fmax(s.r / (double)A.n, -s.vmax);
        s.lam = lam_w;
        s.lam0 = lam_w;
        s.first_done = 1;
        s.need_safeguard = 0;
        s.compact_next = 0;
        s.multi = 0;
        s.tail = kTailNone;
      } else {
        if (s.warm) {
          // the estimate's lam_J: over the kept values of I (every value of
          // I above lam* is kept), or, if none was kept, over I's largest
          // value alone (Algorithm 2's first set).  Every candidate is an
          // upper bound of lam*; the smallest one starts Algorithm 4.
          lam_w = s.r - vmaxI;
          if (tot[C_CNTI] > 0.0) lam_w = fmin(lam_w, (s.r - tot[C_SUMI]) / tot[C_CNTI]);
          lam0 = fmin(lam0, lam_w);
        }
        s.lam = lam0;
        s.lam0 = lam0;
        s.hi = lam0;
        s.compact_next = (s.compaction != CQK_COMPACT_OFF) ? 1 : 0;
        s.tail = (s.n_src <= s.tail_cap) ? kTailPack : kTailNone;
        s.multi = s.tail ? 0 : 1;
      }
    }
    // a warm start records the estimate's own lam_J (NaN without one) and
    // the count of I's kept values in place of the union's sum and count
    spx_trace(&s, A.trace, 0, 1, 0, s.lam, s.warm ? lam_w : tot[C_SUM],
              s.warm ? tot[C_CNTI] : tot[C_CNT], A.n, (int64_t)tot[C_NOUT]);
    *st = s;
    tail_flags(&f, s, false);
  }
  __syncthreads();
  if (f.offsets) spx_tail_offsets(A, G * kWaves, f.src - 1, offl);
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
  if (threadIdx.x == 0) write_partial(A.partials, tot, F_NSUM + 1);
}

__global__ __launch_bounds__(kRBlock) void spx_formula_update_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[(F_NSUM + 1) * (kRBlock / kWave)];
  __shared__ double tot[F_NSUM + 1];
  reduce_partials<F_NSUM, 0, 1, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x != 0) return;
  SpxState s = *st;
  s.passes += 1;
  s.sum_abs = tot[F_ABS];
  s.vmax = tot[F_NSUM];
  if (tot[F_BAD] > 0.0) {
    s.status = CQK_INVALID_ARG;
  } else if (s.l1 && tot[F_ABS] <= s.r) {
    s.fin_mode = kFinCopy;
    spx_finish(&s, 0.0, 5);
  } else {
    double lam0 = (s.r - tot[F_SUM]) / (double)A.n;
    lam0 = fmax(lam0, -tot[F_NSUM]);
    s.lam = lam0;
    s.lam0 = lam0;
    s.need_safeguard = 0;
    s.first_done = 1;
  }
  spx_trace(&s, A.trace, 0, 0, 0, s.lam, tot[F_SUM], (double)A.n, A.n, 0);
  *st = s;
}

// Candidate j of the start refinement: between lam_0 and -max v (a lower
// bound of lam*), halving the distance to -max v at every step.
__device__ __forceinline__ double cand_lambda(double lam0, double vmax, int j) {
  return -vmax + (lam0 + vmax) / (double)(1u << j);
}

// A value every lane of the wave holds, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// One evaluation of phi and its one-sided slopes at lam_k over the current
// set (counts exactly in double, phi in TA), dropping y + lam_k <= 0 when
// compaction is on (lam_k >= lam*).  MULTI: the pass right after Algorithm 2
// also counts and sums, for every candidate lam_j, the set
// J_j = {v + lam_j > 0}; each lam_{J_j} = (r - S_j)/c_j is an upper bound of
// lam* (eq. (lambdaJ)), and j = 0 gives Algorithm 4's first step.
template <typename TIn, typename TA, bool MULTI>
__global__ __launch_bounds__(kBlock) void spx_pass_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (st->status != kRunning || (st->multi != 0) != MULTI) return;
  if (st->tail != kTailNone) {
    // the set fits the one-block loop: copy each wave region of it to its
    // place in the dense list (offsets from the update kernel)
    if (!MULTI && st->tail == kTailPack) {
      const int si = st->src - 1;
      const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
      const int64_t off = (int64_t)rid * (A.chunk0 / kWaves);
      const int c = A.cnt[si][rid];
      const int64_t o = A.toff[rid];
      const int64_t cap = st->tail_cap;
      const TIn* sv = (const TIn*)A.val[si] + off;
      const uint32_t* sx = A.idx[si] + off;
      for (int i = (int)(threadIdx.x & (kWave - 1)); i < c; i += kWave) {
        if (o + i < cap) {
          ((TIn*)A.tval)[o + i] = sv[i];
          A.tidx[o + i] = sx[i];
        }
      }
    }
    return;
  }
  constexpr int V = VecWidth<TIn>::value;
  constexpr int E = 4 * V;
  constexpr int64_t TILE = (int64_t)kWave * E;
  constexpr int NC = MULTI ? kCand : 1;
  const bool l1 = st->l1 != 0;
  const int src = st->src;
  const bool compact = st->compact_next != 0;
  const TA lam = (TA)st->lam;
  // every wave streams its own region rid (deterministic layout, no barriers)
  const int lane = threadIdx.x & (kWave - 1);
  const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
  const int64_t chunk = A.chunk0 / kWaves;
  const int64_t off = (int64_t)rid * chunk;
  int64_t count;
  const TIn* yv;
  const uint32_t* iv = nullptr;
  TIn* ov = nullptr;
  uint32_t* oi = nullptr;
  int32_t* ocnt = nullptr;
  // the caller's y: tiles grid-stride over all waves (as in the Algorithm 2
  // kernel); a compacted set: the wave's own region
  int64_t base0 = 0, step = TILE;
  if (src == 0) {
    count = A.n;
    yv = (const TIn*)A.y;
    base0 = (int64_t)rid * TILE;
    step = (int64_t)gridDim.x * kWaves * TILE;
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
  // candidate multipliers in scalar registers, counts in integers: the
  // MULTI pass then needs few enough vector registers to keep all of its
  // short waves resident at once
  TA lj[NC];
  int cc[NC];
  double cs[NC];
  if constexpr (MULTI) {
    const double lam0 = st->lam, vmx = st->vmax;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      lj[j] = wave_uniform((TA)cand_lambda(lam0, vmx, j));
      cc[j] = 0;
      cs[j] = 0.0;
    }
  }
  __shared__ double lds[(S_NSUM + 1) * (kBlock / kWave)];
  __shared__ double tot[S_NSUM + 1];
  TA phi = TA(0);
  double acc[S_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  // per-lane counts in integers; |y| sums only where the l1 test needs them
  int cm = 0, cp = 0, nin = 0;
  double abs_sum = 0.0;
  TIn vmx = -(TIn)__builtin_huge_val();
  TIn badacc = TIn(0);
  int64_t written = 0;
  for (int64_t base = base0; base < count; base += step) {
    const bool full = base + TILE <= count;
    TIn y[E];
    bool keep[E];
    load_tile<TIn, E / V>(yv, base, lane, count, y);
#pragma unroll
    for (int w = 0; w < E / V; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        keep[e] = false;
        if (full || i + k < count) {
          const TIn a = l1 ? absval(y[e]) : y[e];
          const TA v = (TA)a;
          const TA z = v + lam;
          phi += z > TA(0) ? z : TA(0);
          cm += z > TA(0) ? 1 : 0;
          cp += z >= TA(0) ? 1 : 0;
          nin += 1;
          if (src == 0) {
            badacc += y[e] * TIn(0);
            vmx = max(vmx, a);
            if (l1) abs_sum += (double)a;
          }
          if constexpr (MULTI) {
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              const bool in = v + lj[j] > TA(0);
              cc[j] += in ? 1 : 0;
              cs[j] += in ? (double)v : 0.0;
            }
          }
          keep[e] = compact && (z > TA(0));
        }
      }
    }
    if (compact) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint64_t m = __ballot(keep[e]);
        if (keep[e]) {
          const int64_t pos = written + lane_prefix(m);
          const int64_t i = base + (int64_t)(e / V) * kWave * V + (int64_t)lane * V + (e % V);
          ov[pos] = y[e];
          oi[pos] = (src == 0) ? (uint32_t)i : iv[i];
        }
        written += __popcll(m);
      }
    }
  }
  if (compact && lane == 0) {
    *ocnt = (int32_t)written;
    acc[S_NOUT] = (double)written;
  }
  acc[S_CM] = (double)cm;
  acc[S_CP] = (double)cp;
  acc[S_NIN] = (double)nin;
  acc[S_ABS] = abs_sum;
  acc[S_BAD] = (badacc == TIn(0)) ? 0.0 : 1.0;
  const double vmax = (double)vmx;
  // phi: reduced in the working precision TA (wave, then waves in order)
  const TA phw = wave_sum(phi);
  __shared__ TA phl[kBlock / kWave];
  if (lane == 0) phl[threadIdx.x / kWave] = phw;
  acc[S_PHI] = 0.0;
  if constexpr (MULTI) {
    // one record: the pass sums, then the candidate counts and sums (the
    // set is compacted, so there is no max to carry)
    constexpr int NV = S_NSUM + 2 * NC;
    __shared__ double lds2[NV * (kBlock / kWave)];
    __shared__ double tot2[NV];
    double all[NV];
#pragma unroll
    for (int i = 0; i < S_NSUM; ++i) all[i] = acc[i];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      all[S_NSUM + j] = (double)cc[j];
      all[S_NSUM + NC + j] = cs[j];
    }
    block_reduce<NV, 0, 0, kBlock>(all, nullptr, nullptr, lds2, tot2);
    if (threadIdx.x == 0) {
      TA pb = phl[0];
      for (int w = 1; w < kBlock / kWave; ++w) pb += phl[w];
      tot2[S_PHI] = (double)pb;
      write_partial(A.partials, tot2, NV);
    }
  } else {
    block_reduce<S_NSUM, 0, 1, kBlock>(acc, nullptr, &vmax, lds, tot);
    if (threadIdx.x == 0) {
      TA pb = phl[0];
      for (int w = 1; w < kBlock / kWave; ++w) pb += phl[w];
      tot[S_PHI] = (double)pb;
      write_partial(A.partials, tot, S_NSUM + 1);
    }
  }
}

// One block: phi summed in TA in block order, counts exactly in double, then
// Algorithm 4's update.  When the update finds that the next set fits the
// one-block loop it writes the region offsets for the pack; the update
// after that pack runs the loop.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kRBlock) void spx_update_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning || st->multi || st->tail == kTailY) return;
  __shared__ TailLds<TIn, TA> L;
  __shared__ TailGo f;
  SpxState sc;
  if (st->tail == kTailPack) {
    // the grid pass just before this one copied the set to tval
    if (threadIdx.x == 0) {
      sc = *st;
      tail_flags(&f, sc, true);
    }
    __syncthreads();
    if (f.go) spx_tail_run<TIn, TA>(A, f.n, sc, f.src, f.l1 != 0, L);
    return;
  }
  const bool compact = st->compact_next != 0;
  const int src = st->src;
  __shared__ double lds[(S_NSUM + 1) * (kRBlock / kWave)];
  __shared__ double tot[S_NSUM + 1];
  __shared__ TA phl[kRBlock / kWave];
  TA pg = TA(0);
  for (int g = threadIdx.x; g < G; g += kRBlock) pg += (TA)A.partials[(size_t)S_PHI * G + g];
  reduce_partials<S_NSUM, 0, 1, kRBlock>(A.partials, G, lds, tot);
  const TA pw = wave_sum(pg);
  if ((threadIdx.x & (kWave - 1)) == 0) phl[threadIdx.x / kWave] = pw;
  __syncthreads();
  if (threadIdx.x == 0) {
    TA pb = phl[0];
    for (int w = 1; w < kRBlock / kWave; ++w) pb += phl[w];
    tot[S_PHI] = (double)pb;
    sc = *st;  // register copy: one round trip to memory
    spx_update(&sc, tot, tot[S_NSUM], A.trace, compact, src);
    *st = sc;
    tail_flags(&f, sc, false);
  }
  __syncthreads();
  if (f.offsets) spx_tail_offsets(A, G * kWaves, f.src - 1, L.off);
}

// Closes the start after the MULTI pass: keeps that pass's compaction (done
// at lam_0 >= lam*) and moves lam_0 down to the smallest candidate bound; a
// set that now fits goes on into the tail loop.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kRBlock) void spx_start_update_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (st->status != kRunning || st->tail || !st->multi) return;
  constexpr int NV = S_NSUM + 2 * kCand;  // the MULTI pass's record
  __shared__ double lds[NV * (kRBlock / kWave)];
  __shared__ double tot[NV];
  __shared__ int offl[kRBlock / kWave + 1];
  __shared__ TailGo f;
  reduce_partials<NV, 0, 0, kRBlock>(A.partials, G, lds, tot);
  const double* tc = tot + S_NSUM;
  SpxState s;
  if (threadIdx.x == 0) {
    s = *st;
    s.passes += 1;
    s.multi = 0;
    const int src0 = s.src;
    const bool compacted = s.compact_next != 0;
    if (compacted) {
      s.src = (src0 == 1) ? 2 : 1;
      s.n_src = (int64_t)tot[S_NOUT];
    }
    double best = s.lam;
    for (int j = 0; j < kCand; ++j) {
      if (tc[j] > 0.0) best = fmin(best, (s.r - tc[kCand + j]) / tc[j]);
    }
    spx_trace(&s, A.trace, 0, compacted ? 1 : 0, src0, best, tot[S_PHI], tot[S_CM],
              (int64_t)tot[S_NIN], compacted ? (int64_t)tot[S_NOUT] : 0);
    s.lam = best;
    s.lam0 = best;
    s.hi = best;
    if (s.n_src <= s.tail_cap && s.src != 0) s.tail = kTailPack;
    *st = s;
    tail_flags(&f, s, false);
  }
  __syncthreads();
  if (f.offsets) spx_tail_offsets(A, G * kWaves, f.src - 1, offl);
}

// How x is written once the Newton loop has stopped: the zero fill + scatter
// form whenever the final set is a compacted one (every index left out of it
// is fixed at zero), the dense map otherwise.
__device__ __forceinline__ int spx_fin_mode(const SpxState* st) {
  const int mode = st->fin_mode;
  return (mode == kFinDense && st->src != 0) ? (int)kFinScatter : mode;
}

__device__ __forceinline__ bool spx_done(const SpxState* st) {
  return st->status == CQK_OK || st->status == CQK_NOT_CONVERGED;
}

// Dense finalize over all n: x = max(0, y + lam) (l1: with the signs of y),
// or zeros (the scatter kernel then writes the survivors), or a copy of y.
// For FP32 data with FP64 accumulation y + lam is formed in FP64 and x is
// rounded once.  Does nothing while the solve is still running.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_finalize_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (!spx_done(st)) return;
  constexpr int V = VecWidth<TIn>::value;
  const int mode = spx_fin_mode(st);
  const bool l1 = st->l1 != 0;
  const TA lam = (TA)st->lam_final;
  const int64_t off = (int64_t)blockIdx.x * A.chunk0;
  const int64_t count = max((int64_t)0, min(A.chunk0, A.n - off));
  const TIn* y = (const TIn*)A.y + off;
  TIn* x = (TIn*)A.x + off;
  double acc[2] = {0.0, 0.0};
  constexpr int U = 4;
  constexpr int64_t TILE = (int64_t)kBlock * V * U;
  const bool zero = (mode == kFinScatter || mode == kFinZero);
  if (mode == kFinScatter && st->x_zeroed) return;  // zeros already in place
  for (int64_t base = 0; base < count; base += TILE) {
    const bool full = base + TILE <= count;
    TIn yv[U * V];
    if (!zero) {
      if (full) {
        typename Raw16<TIn>::type r[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          r[u] = ld16(y + base + (int64_t)u * kBlock * V + (int64_t)threadIdx.x * V);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int k = 0; k < V; ++k) yv[u * V + k] = r[u][k];
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
          load_y<TIn>(y, base + (int64_t)u * kBlock * V + (int64_t)threadIdx.x * V, count,
                      &yv[u * V]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + (int64_t)u * kBlock * V + (int64_t)threadIdx.x * V;
      TIn o[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        if (zero) {
          o[k] = TIn(0);
        } else if (mode == kFinCopy) {
          o[k] = yv[u * V + k];
        } else {
          const TA t = (TA)yv[u * V + k];
          const TA vv = l1 ? absval(t) : t;
          const TA z = vv + lam;
          TA xv = z > TA(0) ? z : TA(0);
          if (l1 && t < TA(0)) xv = -xv;
          o[k] = (TIn)xv;
        }
        if (!zero && i + k < count) {
          acc[0] += fabs((double)o[k]);
          acc[1] += (o[k] != TIn(0)) ? 1.0 : 0.0;
        }
      }
      if (i + V <= count) {
        typename Raw16<TIn>::type w;
#pragma unroll
        for (int k = 0; k < V; ++k) w[k] = o[k];
        st16(x + i, w);
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k)
          if (i + k < count) x[i + k] = o[k];
      }
    }
  }
  if (mode == kFinScatter) return;  // the scatter kernel writes the totals
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, 2);
}

// x[idx] = max(0, v + lam) for the indices that survived every compaction;
// all other x are zero (written by the finalize kernel first).
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_scatter_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (!spx_done(st) || spx_fin_mode(st) != kFinScatter) return;
  const bool l1 = st->l1 != 0;
  const TA lam = (TA)st->lam_final;
  const int src = st->src;
  const int lane = threadIdx.x & (kWave - 1);
  TIn* x = (TIn*)A.x;
  double acc[2] = {0.0, 0.0};
  auto put = [&](TIn yv, uint32_t ix) {
    const TA t = (TA)yv;
    const TA z = (l1 ? absval(t) : t) + lam;
    TA xv = z > TA(0) ? z : TA(0);
    if (l1 && t < TA(0)) xv = -xv;
    const TIn xo = (TIn)xv;
    x[ix] = xo;
    acc[0] += fabs((double)xo);
    acc[1] += (xo != TIn(0)) ? 1.0 : 0.0;
  };
  if (src == 3) {
    // the tail loop's list: indices only, the values come from y
    const TIn* y = (const TIn*)A.y;
    const int64_t m = st->n_src;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
      const uint32_t ix = A.tidx[i];
      put(y[ix], ix);
    }
  } else {
    const int si = src - 1;
    const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
    const int64_t off = (int64_t)rid * (A.chunk0 / kWaves);
    const int64_t count = A.cnt[si][rid];
    const TIn* v = (const TIn*)A.val[si] + off;
    const uint32_t* iv = A.idx[si] + off;
    for (int64_t i = lane; i < count; i += kWave) put(v[i], iv[i]);
  }
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, 2);
}

// Totals of the finalize (dense modes) or of the scatter (scatter mode).
__global__ __launch_bounds__(kRBlock) void spx_fin_reduce_kernel(SpxArgs A, int G) {
  SpxState* st = A.st;
  if (!spx_done(st)) return;
  __shared__ double lds[2 * (kRBlock / kWave)];
  __shared__ double tot[2];
  reduce_partials<2, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->res_P = tot[0];
    st->n_free = (int64_t)tot[1];
  }
}

// x_i from y_i and lam* (Sec. 1 (proj_Delta); l1: Lemma 1), or y_i itself when
// y is inside the l1 ball.  FP32 data with FP64 accumulation forms y + lam in
// FP64 and rounds once, as the dense finalize does.
template <typename TIn, typename TA>
__device__ __forceinline__ TIn spx_x_of(TIn yv, TA lam, bool l1, bool copy) {
  if (copy) return yv;
  const TA t = (TA)yv;
  const TA z = (l1 ? absval(t) : t) + lam;
  TA xv = z > TA(0) ? z : TA(0);
  if (l1 && t < TA(0)) xv = -xv;
  return (TIn)xv;
}

// Sparse output, first kernel: sets one bit per index whose x is non-zero in
// a bitmap that is all zero on entry (the write kernel clears what it read).
// The final set is read as the scatter reads it; its indices of one 32-bit
// word may sit in the regions of different waves, hence an atomic OR.  When
// x is a dense map of y (nothing was compacted, or y is inside the l1 ball)
// y is read in wave tiles and each word is assembled from ballots and stored
// whole.  Also the partial record of sum |x| and the count.
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_sp_mark_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (!spx_done(st)) return;
  const int mode = spx_fin_mode(st);
  const bool l1 = st->l1 != 0;
  const TA lam = (TA)st->lam_final;
  const int lane = threadIdx.x & (kWave - 1);
  double acc[2] = {0.0, 0.0};
  if (mode == kFinScatter) {
    auto mark = [&](TIn yv, uint32_t ix) {
      const TIn xo = spx_x_of<TIn, TA>(yv, lam, l1, false);
      if (xo != TIn(0)) atomicOr(A.bm + (ix >> 5), 1u << (ix & 31u));
      acc[0] += fabs((double)xo);
      acc[1] += (xo != TIn(0)) ? 1.0 : 0.0;
    };
    if (st->src == 3) {
      const TIn* y = (const TIn*)A.y;
      const int64_t m = st->n_src;
      for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
           i += (int64_t)gridDim.x * kBlock) {
        const uint32_t ix = A.tidx[i];
        mark(y[ix], ix);
      }
    } else {
      const int si = st->src - 1;
      const int rid = blockIdx.x * kWaves + (int)(threadIdx.x / kWave);
      const int64_t off = (int64_t)rid * (A.chunk0 / kWaves);
      const int64_t count = A.cnt[si][rid];
      const TIn* v = (const TIn*)A.val[si] + off;
      const uint32_t* iv = A.idx[si] + off;
      for (int64_t i = lane; i < count; i += kWave) mark(v[i], iv[i]);
    }
  } else if (mode != kFinZero) {
    constexpr int V = VecWidth<TIn>::value;
    constexpr int64_t T = (int64_t)kWave * V;  // values per wave tile
    constexpr int LW = 32 / V;                 // lanes per bitmap word
    constexpr int WPT = kWave / LW;            // words per wave tile
    const bool copy = mode == kFinCopy;
    const TIn* y = (const TIn*)A.y;
    const int64_t n = A.n;
    const int64_t ntiles = (n + T - 1) / T;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave; t < ntiles; t += nw) {
      const int64_t i = t * T + (int64_t)lane * V;
      TIn yv[V];
      load_y<TIn>(y, i, n, yv);
      uint64_t m[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const TIn xo = spx_x_of<TIn, TA>(yv[k], lam, l1, copy);
        const bool nz = (i + k < n) && xo != TIn(0);
        acc[0] += nz ? fabs((double)xo) : 0.0;
        acc[1] += nz ? 1.0 : 0.0;
        m[k] = __ballot(nz);
      }
      // word j of the tile: lanes j*LW .. j*LW+LW-1, value k of lane
      // j*LW + q at bit q*V + k
      if (lane < WPT) {
        uint32_t w = 0;
#pragma unroll
        for (int q = 0; q < LW; ++q)
#pragma unroll
          for (int k = 0; k < V; ++k)
            w |= (uint32_t)((m[k] >> (lane * LW + q)) & 1u) << (q * V + k);
        const int64_t wi = t * WPT + lane;
        if (wi < A.nwords) A.bm[wi] = w;
      }
    }
  }
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, 2);
}

// The count and write kernels give each thread kSpWords consecutive bitmap
// words per step (four 16-byte loads); a block covers sp_wpb words, a
// multiple of kSpStep.
constexpr int kSpWords = 16;
constexpr int64_t kSpStep = (int64_t)kBlock * kSpWords;

// The thread's kSpWords words at w (zero beyond w1); w is a multiple of 16
// and the bitmap 256-byte aligned.
__device__ __forceinline__ void sp_load_words(const uint32_t* bm, int64_t w, int64_t w1,
                                              uint32_t* o) {
  if (w + kSpWords <= w1) {
#pragma unroll
    for (int q = 0; q < kSpWords / 4; ++q) {
      const int4v v = *reinterpret_cast<const int4v*>(bm + w + 4 * q);
#pragma unroll
      for (int j = 0; j < 4; ++j) o[4 * q + j] = (uint32_t)v[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kSpWords; ++j) o[j] = (w + j < w1) ? bm[w + j] : 0u;
  }
}

// Bits of word w that name indices below n (all of them except in the last
// word): the count and the write ignore anything beyond n.
__device__ __forceinline__ uint32_t sp_word_mask(int64_t w, int64_t n) {
  const int64_t rest = n - w * 32;
  return (rest >= 32) ? 0xFFFFFFFFu : ((rest <= 0) ? 0u : ((1u << rest) - 1u));
}

// Sparse output, second kernel: set bits per block of sp_wpb bitmap words.
__global__ __launch_bounds__(kBlock) void spx_sp_count_kernel(SpxArgs A) {
  SpxState* st = A.st;
  if (!spx_done(st) || spx_fin_mode(st) == kFinZero) return;
  const int64_t w0 = (int64_t)blockIdx.x * A.sp_wpb;
  const int64_t w1 = min(w0 + A.sp_wpb, A.nwords);
  int c = 0;
  for (int64_t w = w0 + (int64_t)threadIdx.x * kSpWords; w < w1; w += kSpStep) {
    uint32_t b[kSpWords];
    sp_load_words(A.bm, w, w1, b);
#pragma unroll
    for (int j = 0; j < kSpWords; ++j) c += __popc(b[j] & sp_word_mask(w + j, A.n));
  }
  __shared__ int lds_i[kBlock / kWave + 1];
  int total = 0;
  block_excl_scan<kBlock>(c, lds_i, &total);
  if (threadIdx.x == 0) A.sp_cnt[blockIdx.x] = total;
}

// Sparse output, last kernel: each block places the set bits of its words at
// its offset (the counts of the blocks before it) in ascending index order,
// with x_i recomputed from y_i, and clears the words it read.  If the support
// exceeds the caller's capacity nothing is written (the count is still
// returned).
template <typename TIn, typename TA>
__global__ __launch_bounds__(kBlock) void spx_sp_write_kernel(SpxArgs A, int GS) {
  SpxState* st = A.st;
  if (!spx_done(st)) return;
  const int mode = spx_fin_mode(st);
  if (mode == kFinZero) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->nnz = 0;
    return;
  }
  double acc[2] = {0.0, 0.0};  // entries before this block, all entries
  for (int b = threadIdx.x; b < GS; b += kBlock) {
    const double c = (double)A.sp_cnt[b];
    acc[0] += (b < (int)blockIdx.x) ? c : 0.0;
    acc[1] += c;
  }
  __shared__ double lds[2 * (kBlock / kWave)];
  __shared__ double tot[2];
  __shared__ int lds_i[kBlock / kWave + 1];
  block_reduce<2, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  const int64_t before = (int64_t)tot[0];
  const int64_t total = (int64_t)tot[1];
  const bool over = total > A.sp_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->nnz = total;
    st->sp_over = over ? 1 : 0;
  }
  const bool l1 = st->l1 != 0;
  const bool copy = mode == kFinCopy;
  const TA lam = (TA)st->lam_final;
  const TIn* y = (const TIn*)A.y;
  TIn* ov = (TIn*)A.sp_val;
  const int64_t w0 = (int64_t)blockIdx.x * A.sp_wpb;
  const int64_t w1 = min(w0 + A.sp_wpb, A.nwords);
  int64_t pos = before;
  for (int64_t ws = w0; ws < w1; ws += kSpStep) {
    const int64_t w = ws + (int64_t)threadIdx.x * kSpWords;
    uint32_t b[kSpWords];
    sp_load_words(A.bm, w, w1, b);
    int c = 0;
#pragma unroll
    for (int j = 0; j < kSpWords; ++j) c += __popc(b[j] & sp_word_mask(w + j, A.n));
    int step = 0;
    const int ex = block_excl_scan<kBlock>(c, lds_i, &step);
    if (c != 0) {
      int64_t p = pos + ex;
#pragma unroll
      for (int j = 0; j < kSpWords; ++j) {
        if (b[j] == 0u) continue;
        uint32_t rest = b[j] & sp_word_mask(w + j, A.n);
        if (!over) {
          while (rest != 0u) {
            const int k = __builtin_ctz(rest);
            rest &= rest - 1u;
            const int64_t ix = (w + j) * 32 + k;
            A.sp_idx[p] = ix;
            ov[p] = spx_x_of<TIn, TA>(y[ix], lam, l1, copy);
            ++p;
          }
        }
        A.bm[w + j] = 0u;  // leave the bitmap clear for the next call
      }
    }
    pos += step;
  }
}

__global__ void spx_init_kernel(SpxState* st, SpxState init) { *st = init; }

int grid0(int64_t n, int num_cus) {
  const int64_t want = (n + 2047) / 2048;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cus * 8));
}

template <typename TIn, typename TA>
cqk_status run_simplex(cqk_ctx* ctx, int64_t n, const TIn* y, const TIn* xw, SparseOut* sp,
                       double r, TIn* x, bool l1, const cqk_opts& o, cqk_info* info) {
  if (n > (int64_t)UINT32_MAX) return CQK_INVALID_ARG;
  constexpr int64_t CAP = kTailBytes / (int64_t)sizeof(TIn);
  // G0 blocks of kWaves waves.  Passes over y hand out tiles of at most
  // kWave * kCondatK values grid-stride, at most tpw each per wave, so a wave
  // region of chunk0/kWaves = tpw tiles holds every survivor a wave keeps
  // (the pass kernel's FP64 tiles are half as long, hence at most 2 tpw).
  const int G0i = grid0(n, ctx->num_cus);
  constexpr int64_t kT = (int64_t)kWave * kCondatK;
  const int64_t ntiles = (n + kT - 1) / kT;
  const int64_t tpw =
      std::max<int64_t>(1, (ntiles + (int64_t)G0i * kWaves - 1) / ((int64_t)G0i * kWaves));
  const int64_t chunk0 = tpw * kT * kWaves;
  const int G0 = (int)std::max<int64_t>(1, (n + chunk0 - 1) / chunk0);
  const int NR = G0 * kWaves;
  // a warm start runs Algorithm 2 over the estimate's support, whatever the
  // start option says
  const bool warm = xw != nullptr;
  const bool condat = warm || o.lambda0_mode == CQK_LAMBDA0_CONDAT;
  const bool formula = !warm && o.lambda0_mode == CQK_LAMBDA0_FORMULA;

  // the Algorithm 2 sample: one tile per wave, spread evenly over y; its
  // block records follow the partial records of the grid passes
  const int ns = (int)std::min<int64_t>(ntiles, kSampleWaves);
  const int GSm = (ns + kWaves - 1) / kWaves;
  const size_t prec = (size_t)G0 * (kPassRec + 2 * kCand);
  const size_t part_bytes = ((prec + (size_t)SM_N * GSm) * sizeof(double) + 255) / 256 * 256;
  const size_t cnt_bytes = ((size_t)2 * NR * sizeof(int32_t) + 255) / 256 * 256;
  const size_t cap = (size_t)G0 * chunk0;
  const size_t val_bytes = (cap * sizeof(TIn) + 255) / 256 * 256;
  const size_t idx_bytes = (cap * sizeof(uint32_t) + 255) / 256 * 256;
  const size_t tcap = (size_t)std::min<int64_t>(n, CAP);
  const size_t ti_bytes = (tcap * sizeof(uint32_t) + 255) / 256 * 256;
  const size_t tv_bytes = (tcap * sizeof(TIn) + 255) / 256 * 256;
  const size_t to_bytes = ((size_t)NR * sizeof(int32_t) + 255) / 256 * 256;
  const bool need_bufs = (o.compaction != CQK_COMPACT_OFF) || condat;
  // sparse output: GS blocks of sp_wpb bitmap words (a multiple of kSpStep) each
  const bool sparse = sp != nullptr;
  const int64_t nwords = (n + 31) / 32;
  const int GS =
      (int)std::min<int64_t>(1024, std::max<int64_t>(1, (nwords + kSpStep - 1) / kSpStep));
  const int64_t wpb = ((nwords + GS - 1) / GS + kSpStep - 1) / kSpStep * kSpStep;
  const size_t sc_bytes = sparse ? ((size_t)GS * sizeof(int32_t) + 255) / 256 * 256 : 0;
  const size_t total = part_bytes + cnt_bytes + ti_bytes + tv_bytes + to_bytes + sc_bytes +
                       (need_bufs ? 2 * (val_bytes + idx_bytes) : 0);
  cqk_status stt = ensure_buffer(ctx, ctx->ws, total);
  if (stt != CQK_OK) return stt;
  if (sparse) {
    const size_t bm_bytes = ((size_t)nwords * sizeof(uint32_t) + 255) / 256 * 256;
    const bool grows = ctx->bitmap.bytes < bm_bytes;
    stt = ensure_buffer(ctx, ctx->bitmap, bm_bytes);
    if (stt != CQK_OK) return stt;
    if (grows) ctx->bitmap_clean = false;
    // all zero from here, the whole allocation (a later, longer call reads
    // more of it); the write kernel clears what it reads
    if (!ctx->bitmap_clean &&
        hip_ok(hipMemsetAsync(ctx->bitmap.ptr, 0, ctx->bitmap.bytes, ctx->stream)) != CQK_OK)
      return CQK_DEVICE_ERROR;
    ctx->bitmap_clean = false;  // until this call has run to its end
  }
  stt = ensure_buffer(ctx, ctx->state, 1024 + sizeof(cqk_trace_rec) * kMaxTrace);
  if (stt != CQK_OK) return stt;

  char* ws = (char*)ctx->ws.ptr;
  SpxArgs A{};
  A.y = y;
  A.xw = xw;
  A.x = sparse ? nullptr : x;
  A.n = n;
  A.chunk0 = chunk0;
  A.partials = (double*)ws;
  A.samp = A.partials + prec;
  A.samp_ntiles = ntiles;
  A.samp_waves = ns;
  A.samp_blocks = GSm;
  A.cnt[0] = (int32_t*)(ws + part_bytes);
  A.cnt[1] = A.cnt[0] + NR;
  A.tidx = (uint32_t*)(ws + part_bytes + cnt_bytes);
  A.tval = ws + part_bytes + cnt_bytes + ti_bytes;
  A.toff = (int32_t*)(ws + part_bytes + cnt_bytes + ti_bytes + tv_bytes);
  if (need_bufs) {
    char* b = ws + part_bytes + cnt_bytes + ti_bytes + tv_bytes + to_bytes;
    A.val[0] = b;
    A.idx[0] = (uint32_t*)(b + val_bytes);
    A.val[1] = b + val_bytes + idx_bytes;
    A.idx[1] = (uint32_t*)(b + 2 * val_bytes + idx_bytes);
  }
  A.st = (SpxState*)ctx->state.ptr;
  A.trace = (cqk_trace_rec*)((char*)ctx->state.ptr + 1024);
  if (sparse) {
    A.bm = (uint32_t*)ctx->bitmap.ptr;
    A.nwords = nwords;
    A.sp_wpb = wpb;
    A.sp_cnt = (int32_t*)(ws + part_bytes + cnt_bytes + ti_bytes + tv_bytes + to_bytes +
                          (need_bufs ? 2 * (val_bytes + idx_bytes) : 0));
    A.sp_idx = sp->idx;
    A.sp_val = sp->val;
    A.sp_cap = sp->cap;
  }

  const double eps = sizeof(TA) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  SpxState init{};
  init.lam = (!warm && o.lambda0_mode == CQK_LAMBDA0_USER) ? o.lambda0_user : 0.0;
  init.warm = warm ? 1 : 0;
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
  // the tail loop takes sets of at most CAP values (its LDS copy); a small
  // instance whose start reads y anyway goes there at once
  init.tail_cap = CAP;
  init.tail = (!condat && n <= CAP) ? kTailY : kTailNone;
  if (r == 0.0) {
    init.status = CQK_OK;
    init.fin_mode = kFinZero;
    init.lam_final = 0.0;
    init.stop_reason = 5;
  }

  hipStream_t s = ctx->stream;
  // sync = 0 or graph capture (dense output only): every pass the iteration
  // cap allows is queued at once, nothing is read back; cqk_ctx_last_info
  // reads the result later.  No per-pass timing then.
  const bool deferred = !sparse && (!o.sync || stream_capturing(s));
  const bool timing = o.timing && !deferred;
  // events 0..3: the finalize and scatter of the last finalize chain;
  // then one pair per grid pass
  const size_t nev = (size_t)4 + 2 * (o.max_iter + 8);
  if (timing) {
    stt = ensure_events(ctx, nev);
    if (stt != CQK_OK) return stt;
  }
  // the Algorithm 2 sample kernel stores the initial state itself
  const bool init_in_sample = condat && r != 0.0;
  if (!init_in_sample) hipLaunchKernelGGL(spx_init_kernel, dim3(1), dim3(1), 0, s, A.st, init);
  int ev = 4;
  int npass = 0;  // grid passes queued
  auto launch = [&](auto kern, int grid) {
    const bool rec = timing && ev + 2 <= (int)nev;
    launch_timed(kern, dim3(grid), dim3(kBlock), s, rec ? ctx->events[ev] : nullptr,
                 rec ? ctx->events[ev + 1] : nullptr, A);
    if (rec) ev += 2;
    ++npass;
  };
  // one-block reduction of the partial records of a grid of `grid` blocks
  auto reduce = [&](auto kern, int grid) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(kRBlock), 0, s, A, grid);
  };
  auto tail = [&]() {
    hipLaunchKernelGGL((spx_tail_kernel<TIn, TA>), dim3(1), dim3(kRBlock), 0, s, A);
  };
  // Writes x once the state says the loop has stopped; a no-op before that,
  // so it can follow every batch and the host waits once per batch.
  auto fin_chain = [&]() {
    if (sparse) {
      launch_timed(spx_sp_mark_kernel<TIn, TA>, dim3(G0), dim3(kBlock), s,
                   timing ? ctx->events[0] : nullptr, timing ? ctx->events[1] : nullptr, A);
      hipLaunchKernelGGL(spx_fin_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A, G0);
      hipLaunchKernelGGL(spx_sp_count_kernel, dim3(GS), dim3(kBlock), 0, s, A);
      launch_timed(spx_sp_write_kernel<TIn, TA>, dim3(GS), dim3(kBlock), s,
                   timing ? ctx->events[2] : nullptr, timing ? ctx->events[3] : nullptr, A,
                   GS);
      return;
    }
    // after the Algorithm 2 start of a simplex projection x = 0 is written
    // and the final set is a compacted one: the finalize would return at
    // once (l1 may still copy y), so only the scatter runs
    if (condat && !l1 && r != 0.0) {
      if (timing) {
        (void)hipEventRecord(ctx->events[0], s);
        (void)hipEventRecord(ctx->events[1], s);
      }
    } else {
      launch_timed(spx_finalize_kernel<TIn, TA>, dim3(G0), dim3(kBlock), s,
                   timing ? ctx->events[0] : nullptr, timing ? ctx->events[1] : nullptr, A);
    }
    launch_timed(spx_scatter_kernel<TIn, TA>, dim3(G0), dim3(kBlock), s,
                 timing ? ctx->events[2] : nullptr, timing ? ctx->events[3] : nullptr, A);
    hipLaunchKernelGGL(spx_fin_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A, G0);
  };
  SpxState* hs = (SpxState*)ctx->host_pinned;
  auto wait_state = [&]() -> cqk_status {
    if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
    if (hip_ok(hipMemcpyAsync(hs, A.st, sizeof(SpxState), hipMemcpyDeviceToHost, s)) != CQK_OK)
      return CQK_DEVICE_ERROR;
    return hip_ok(hipStreamSynchronize(s));
  };
  if (r == 0.0) {
    fin_chain();
    if (!deferred && wait_state() != CQK_OK) return CQK_DEVICE_ERROR;
  } else {
    if (condat) {
      {
        const bool rec = timing && ev + 2 <= (int)nev;
        launch_timed(spx_condat_sample_kernel<TIn, TA>, dim3(GSm), dim3(kBlock), s,
                     rec ? ctx->events[ev] : nullptr, rec ? ctx->events[ev + 1] : nullptr, A,
                     init);
        if (rec) ev += 2;
        ++npass;
      }
      if (warm)
        launch(spx_condat_kernel<TIn, true>, G0);
      else
        launch(spx_condat_kernel<TIn, false>, G0);
      reduce(spx_condat_merge_kernel<TIn, TA>, G0);
    } else if (formula) {
      launch(spx_formula_kernel<TIn>, G0);
      reduce(spx_formula_update_kernel, G0);
    }
    // a small instance whose start reads y anyway runs in one block at once
    if (init.tail) tail();
    if (condat) {
      launch(spx_pass_kernel<TIn, TA, true>, G0);
      reduce(spx_start_update_kernel<TIn, TA>, G0);
    }
    int launched = 0;
    const int max_launch = o.max_iter + 2;
    // after the refined start of Algorithm 2 at most one more pass usually
    // leaves a set small enough for the one-block loop, which then takes a
    // pass (the pack) and an update (the loop)
    int batch = deferred ? max_launch : 2;
    for (;;) {
      const int k = std::min(batch, max_launch - launched);
      for (int i = 0; i < k; ++i) {
        launch(spx_pass_kernel<TIn, TA, false>, G0);
        reduce(spx_update_kernel<TIn, TA>, G0);
      }
      launched += k;
      fin_chain();
      if (deferred) {
        if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
        break;
      }
      if (wait_state() != CQK_OK) return CQK_DEVICE_ERROR;
      if (hs->status != kRunning || launched >= max_launch) break;
      batch = 4;
    }
  }
  const int pass_events = ev;
  const int trace_cap = init.trace_cap;
  // bytes of y the Algorithm 2 sample reads
  double samp_bytes = 0.0;
  for (int w = 0; w < ns; ++w) {
    const int64_t base = (int64_t)w * ntiles / ns * kT;
    samp_bytes += (double)sizeof(TIn) * (double)std::min<int64_t>(kT, n - base);
  }
  // Fills an info record from the state copy in hs (the stream synchronised),
  // reading the trace ring too.
  auto report = [ctx, hs, A, trace_cap, n, r, l1, sparse, warm, timing, pass_events, nwords,
                 npass, samp_bytes](cqk_info* info) -> cqk_status {
    const int ntrace = std::min(hs->ntrace, trace_cap);
    ctx->last_trace.resize(ntrace);
    if (ntrace > 0 && hip_ok(hipMemcpy(ctx->last_trace.data(), A.trace,
                                       sizeof(cqk_trace_rec) * ntrace,
                                       hipMemcpyDeviceToHost)) != CQK_OK)
      return CQK_DEVICE_ERROR;
    std::memset(info, 0, sizeof(*info));
    info->status = (hs->status == kRunning) ? CQK_NOT_CONVERGED : hs->status;
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
    info->pass_launches = npass;
    info->finalize_ms = 0.0;
    info->rows_spilled = 0;
    const bool scatter = hs->fin_mode == kFinDense && hs->src != 0;
    // dense map: read y, write x; zero fill: write x (nothing when the
    // Algorithm 2 kernel already wrote the zeros); scatter: per survivor
    // read value and index, write x
    double fin = (double)n * sizeof(TIn) * ((scatter || hs->fin_mode == kFinZero) ? 1.0 : 2.0);
    if (scatter && hs->x_zeroed) fin = 0.0;
    if (scatter) fin += (2.0 * sizeof(TIn) + 4.0) * (double)hs->n_src;
    if (sparse) {
      // mark: the final set (scatter form) or y and the bitmap (dense
      // form); count and write: the bitmap twice; per entry an index and a
      // value written and y read again
      const double bm = 4.0 * (double)nwords;
      fin = 0.0;
      if (hs->fin_mode != kFinZero) {
        fin = scatter ? (sizeof(TIn) + 4.0) * (double)hs->n_src : (double)n * sizeof(TIn) + bm;
        fin += 2.0 * bm + (8.0 + 2.0 * sizeof(TIn)) * (double)hs->nnz;
      }
    }
    info->finalize_bytes = fin;
    for (int i = 0; i < ntrace; ++i) {
      const cqk_trace_rec& t = ctx->last_trace[i];
      if (t.kind == 7) continue;  // one thread's Algorithm 2, not a pass
      const double per_in = (t.source == 0) ? (double)sizeof(TIn) : (double)sizeof(TIn) + 4.0;
      const double per_out = (double)sizeof(TIn) + 4.0;
      info->pass_bytes += per_in * (double)t.n_in + per_out * (double)t.n_out;
      // the Algorithm 2 start also reads its sample of y, writes x = 0
      // everywhere (not for a sparse output) and reads the estimate of a
      // warm start
      if (t.kind == 0 && t.source == 0 && t.compacted)
        info->pass_bytes += samp_bytes + sizeof(TIn) * (double)t.n_in *
                                             ((sparse ? 0.0 : 1.0) + (warm ? 1.0 : 0.0));
    }
    ctx->last_pass_ms.clear();
    if (timing) {
      // every grid pass launched (those after the loop stopped return at
      // once); the tail loop runs in one block between them and is not here
      for (int i = 4; i + 1 < pass_events; i += 2) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]);
        info->pass_ms += ms;
        ctx->last_pass_ms.push_back(ms);
      }
      for (int j = 0; j < 2; ++j) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->events[2 * j], ctx->events[2 * j + 1]);
        info->finalize_ms += ms;
      }
    }
    if (sparse && hs->sp_over && (info->status == CQK_OK || info->status == CQK_NOT_CONVERGED))
      info->status = CQK_BUFFER_TOO_SMALL;
    return CQK_OK;
  };
  ctx->last = [hs, A, report](cqk_info* inf) -> cqk_status {
    if (hip_ok(hipMemcpy(hs, A.st, sizeof(SpxState), hipMemcpyDeviceToHost)) != CQK_OK)
      return CQK_DEVICE_ERROR;
    return report(inf);
  };
  if (deferred) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = CQK_OK;
      info->pass_launches = npass;
    }
    return CQK_OK;
  }
  cqk_info tmp;
  const cqk_status rs = report(info ? info : &tmp);
  if (sparse) {
    ctx->bitmap_clean = true;  // cleared by the write kernel, or never set
    sp->nnz = hs->nnz;
  }
  return rs;
}

}  // namespace

cqk_status run_simplex_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xw, SparseOut* sp,
                           double r, float* x, bool l1, const cqk_opts& o, cqk_info* info) {
  if (o.accum == CQK_ACCUM_F32)
    return run_simplex<float, float>(ctx, n, y, xw, sp, r, x, l1, o, info);
  return run_simplex<float, double>(ctx, n, y, xw, sp, r, x, l1, o, info);
}

cqk_status run_simplex_f64(cqk_ctx* ctx, int64_t n, const double* y, const double* xw,
                           SparseOut* sp, double r, double* x, bool l1, const cqk_opts& o,
                           cqk_info* info) {
  return run_simplex<double, double>(ctx, n, y, xw, sp, r, x, l1, o, info);
}

}  // namespace cqk
