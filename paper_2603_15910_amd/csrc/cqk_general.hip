// General CQK: semismooth Newton on the dual equation phi(lam) = r.
//
// Paper: Section 2.1 (eq. (xopt), eq. (opt), eq. (phideriv), Algorithm 1,
// eq. (CQKlambda0)), Section 2.2 (variable fixing), Section 4 (the pass is a
// map over indices followed by a reduction), Section 5 (stopping criteria).
//
// Every pass works on the per-index form
//     g_i(lam) = b_i x_i(lam) = min(max(c_i + lam s_i, b_i l_i), b_i u_i),
//     c_i = b_i a_i / d_i,  s_i = b_i^2 / d_i,
// which is eq. (xopt) multiplied by b_i > 0.  phi(lam) = sum_i g_i(lam); the
// one-sided slopes of eq. (phideriv) sum s_i over b l <= c + lam s < b u and
// b l < c + lam s <= b u.
//
// Kernels:
//   gen_pass_kernel     one pass over the current index set (evaluation at
//                       lam, or the closest-breakpoint search), each block
//                       writing one partial record;
//   gen_update_kernel   one block: reduces the records and runs the scalar
//                       Algorithm 1 update on the device-resident state;
//   gen_lambda0_kernel  eq. (CQKlambda0) over all indices, with input checks;
//   gen_finalize_kernel x(lam*) over all n indices (eq. (xopt)), b^T x;
//   gen_sample_kernel, gen_sample2_kernel, gen_sample3_kernel (+ reduces),
//   gen_spec_pass_kernel,
//   gen_warm_spec_kernel: the sampled bracket (below).
// The host queues passes in batches and reads the state once per batch;
// a pass queued after the loop has stopped returns at once.
//
// Compaction.  Within a Newton bracket [lo, hi] an index whose bound is
// active on the whole bracket (c + hi s <= b l, or c + lo s >= b u) has the
// same value at every later iterate; so does an index that is free on the
// whole bracket, whose contribution is the line c + lam s.  Such indices are
// dropped from later passes (their contributions kept as a few scalars) and
// the survivors are written, in the per-index form above, to a compacted
// set: wave w always owns the same pieces of it, so no grid-wide scan is
// needed and the layout is deterministic.  In exact arithmetic the values of
// phi and its slopes are unchanged; this is the fixing of Section 2.2 applied
// through the bracket, plus the free-side analogue.
//
// The evaluation at lam_k itself narrows the bracket to [lam_k, hi] or
// [lo, lam_k], and that narrower bracket resolves far more indices than
// [lo, hi]; but which of the two it is only follows from the pass's reduced
// sums.  So an evaluation pass writes both candidate sets (one per side, each
// with its own dropped-index sums), and the update keeps the side that
// happened.  A side that would keep more than theta of the indices a wave
// reads is given up by that wave at once (before it writes), which makes the
// side unusable for the pass and costs nothing more; sides that resolve
// little are thus never written.  The first pass of a solve has a one-sided
// bracket at best, which resolves little: without more it does not compact
// (gen_first_pass_kernel).
//
// Sampled bracket (a GPU addition).  For large n two small kernels estimate
// lam* from a sample with a bracket of a few standard deviations, and the
// first pass (or the lam_0 pass of a warm or formula start) also writes the
// indices with a breakpoint in that bracket to set 3.  Every compacted set
// carries the bracket its dropped sums hold on (GenState vlo, vhi) and is
// read only at a multiplier strictly inside it, so Algorithm 1's iterates do
// not depend on the estimate; the sampled set waits in set 3 until an
// iterate falls inside (take_spec_set).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "cqk_alg1.h"
#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kRBlock = 1024;  // one-block reductions of partial records
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kUnroll = 2;
// values per lane in one tile of a pass: kUnroll 16-byte vectors of FP64,
// or half as many vectors of FP32, so both element types hold as many
// values in registers
constexpr int kTileE = kUnroll * 2;
constexpr int kPair = 2;  // adjacent tiles a wave reads per step of a pass over the caller's arrays
// the general pass kernel reads a step's tiles one after the other (its
// compaction state leaves no registers for both tiles' loads at once)
constexpr bool kPairUnrollGeneral = false;
constexpr int kStage = 128;  // LDS ring per wave, side and array for compaction
constexpr int kPieceLog = 6;
constexpr int kPiece = 1 << kPieceLog;  // compacted sets are stored in pieces of this many values
static_assert(kPiece == kWave, "a full flush writes one piece, one value per lane");
static_assert(kStage >= kPiece + kWave - 1, "the ring holds a piece plus one slot's survivors");
// The sampled-bracket pass keeps one side: a ring twice as long, written out
// kSpecFlush pieces at a time (fewer, larger bursts of stores between the
// loads of the pass)
constexpr int kStageSpec = 256;
constexpr int kSpecFlush = 2;
static_assert(kStageSpec >= kSpecFlush * kPiece + kWave - 1, "ring of the sampled-bracket pass");

struct GenArgs {
  const void* d;
  const void* a;
  const void* b;
  const void* l;
  const void* u;
  const void* xw;   // primal estimate for the warm start (or null)
  void* x;
  int64_t n;
  int64_t chunk;
  int64_t region;   // values one wave can keep in a compacted set
  double* buf[3];   // compacted sets 1..3: array j (c, s, bl, bu) of set k is
                    // the plane buf[k-1] + j NR region, in pieces of kPiece
                    // values (see Pieces)
  int32_t* cnt[3];  // survivors of each wave in each set
  double* partials;
  float* smp;       // the sample, 4 floats per index (compaction only)
  GenState* st;
  cqk_trace_rec* trace;
};

// Sources: the caller's arrays or a compacted region.
template <typename TIn>
struct SrcOrig {
  static constexpr int V = VecWidth<TIn>::value;
  const TIn *d, *a, *b, *l, *u;
  __device__ __forceinline__ void load(int64_t i, int64_t n, double* c, double* s, double* bl,
                                       double* bu, double& bad) const {
    double vd[V], va[V], vb[V], vl[V], vu[V];
    Vec<TIn, V>::load(d, i, n, 1.0, vd);
    Vec<TIn, V>::load(a, i, n, 0.0, va);
    Vec<TIn, V>::load(b, i, n, 1.0, vb);
    Vec<TIn, V>::load(l, i, n, 0.0, vl);
    Vec<TIn, V>::load(u, i, n, 0.0, vu);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      double tb = 0.0;
      to_form(vd[k], va[k], vb[k], vl[k], vu[k], c[k], s[k], bl[k], bu[k], tb);
      if (i + k < n) bad += tb;
    }
  }
  // U full vectors per lane, every load issued before the first use
  template <int U>
  __device__ __forceinline__ void load_fast(int64_t base, int lane, double* c, double* s,
                                            double* bl, double* bu, double& bad) const {
    typename Raw16<TIn>::type rd[U], ra[U], rb[U], rl[U], ru[U];
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
      rd[w] = ld16(d + i);
      ra[w] = ld16(a + i);
      rb[w] = ld16(b + i);
      rl[w] = ld16(l + i);
      ru[w] = ld16(u + i);
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        double tb = 0.0;
        to_form((double)rd[w][k], (double)ra[w][k], (double)rb[w][k], (double)rl[w][k],
                (double)ru[w][k], c[e], s[e], bl[e], bu[e], tb);
        bad += tb;
      }
    }
  }
};

// The caller's arrays and a primal estimate xbar (warm start, end of
// Section 2.1): loads like SrcOrig and adds each index to the warm start's
// sums as it goes (wm, WS_* below): free in xbar (l < xbar < u) into the
// free set J's sums, at or beyond a bound into the fixed sum; a NaN entry
// of xbar counts nowhere.  xbar is compared with l and u as given.
enum { WS_SJ = 0, WS_QJ, WS_FIX, WS_NJ, WS_SALL, WS_QALL, WS_N };
template <typename TIn>
struct SrcOrigWarm {
  static constexpr int V = VecWidth<TIn>::value;
  const TIn *d, *a, *b, *l, *u, *xw;
  double* wm;  // WS_N sums of the calling thread
  __device__ __forceinline__ void add(double vl, double vu, double vx, double c, double s,
                                      double bl, double bu) const {
    const bool fr = (vx > vl) && (vx < vu);
    const bool at_l = !fr && (vx <= vl);
    const bool at_u = !fr && (vx >= vu);
    wm[WS_SJ] += fr ? c : 0.0;
    wm[WS_QJ] += fr ? s : 0.0;
    wm[WS_NJ] += fr ? 1.0 : 0.0;
    wm[WS_FIX] += at_l ? bl : (at_u ? bu : 0.0);
    wm[WS_SALL] += c;
    wm[WS_QALL] += s;
  }
  __device__ __forceinline__ void load(int64_t i, int64_t n, double* c, double* s, double* bl,
                                       double* bu, double& bad) const {
    double vd[V], va[V], vb[V], vl[V], vu[V], vx[V];
    Vec<TIn, V>::load(d, i, n, 1.0, vd);
    Vec<TIn, V>::load(a, i, n, 0.0, va);
    Vec<TIn, V>::load(b, i, n, 1.0, vb);
    Vec<TIn, V>::load(l, i, n, 0.0, vl);
    Vec<TIn, V>::load(u, i, n, 0.0, vu);
    Vec<TIn, V>::load(xw, i, n, 0.0, vx);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      double tb = 0.0;
      to_form(vd[k], va[k], vb[k], vl[k], vu[k], c[k], s[k], bl[k], bu[k], tb);
      if (i + k < n) {
        bad += tb;
        add(vl[k], vu[k], vx[k], c[k], s[k], bl[k], bu[k]);
      }
    }
  }
  template <int U>
  __device__ __forceinline__ void load_fast(int64_t base, int lane, double* c, double* s,
                                            double* bl, double* bu, double& bad) const {
    typename Raw16<TIn>::type rd[U], ra[U], rb[U], rl[U], ru[U], rx[U];
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
      rd[w] = ld16(d + i);
      ra[w] = ld16(a + i);
      rb[w] = ld16(b + i);
      rl[w] = ld16(l + i);
      ru[w] = ld16(u + i);
      rx[w] = ld16(xw + i);
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        double tb = 0.0;
        to_form((double)rd[w][k], (double)ra[w][k], (double)rb[w][k], (double)rl[w][k],
                (double)ru[w][k], c[e], s[e], bl[e], bu[e], tb);
        bad += tb;
        add((double)rl[w][k], (double)ru[w][k], (double)rx[w][k], c[e], s[e], bl[e], bu[e]);
      }
    }
  }
};

// The caller's arrays, adding every index to the sums of eq. (CQKlambda0)
// over all indices as it loads them (wm[WS_SALL], wm[WS_QALL]).
template <typename TIn>
struct SrcOrigSum {
  static constexpr int V = VecWidth<TIn>::value;
  SrcOrig<TIn> o;
  double* wm;
  __device__ __forceinline__ void load(int64_t i, int64_t n, double* c, double* s, double* bl,
                                       double* bu, double& bad) const {
    o.load(i, n, c, s, bl, bu, bad);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (i + k < n) {
        wm[WS_SALL] += c[k];
        wm[WS_QALL] += s[k];
      }
    }
  }
  template <int U>
  __device__ __forceinline__ void load_fast(int64_t base, int lane, double* c, double* s,
                                            double* bl, double* bu, double& bad) const {
    o.template load_fast<U>(base, lane, c, s, bl, bu, bad);
#pragma unroll
    for (int e = 0; e < U * V; ++e) {
      wm[WS_SALL] += c[e];
      wm[WS_QALL] += s[e];
    }
  }
};

// A compacted set is stored in pieces of kPiece values: value j of wave rid
// lives at piece_pos(j) of each plane, so piece k of every wave sits next to
// piece k of the others.  Waves write and read their k-th pieces at about the
// same time, so the compacted stream moves through neighbouring addresses
// like the grid-stride passes over the caller's arrays.
struct Pieces {
  int64_t rid, nr;
  __device__ __forceinline__ int64_t pos(int64_t j) const {
    return ((j >> kPieceLog) * nr + rid) * kPiece + (j & (kPiece - 1));
  }
};

struct SrcForm {
  static constexpr int V = 2;
  const double *c, *s, *bl, *bu;  // planes
  Pieces P;
  __device__ __forceinline__ void load(int64_t i, int64_t n, double* oc, double* os, double* obl,
                                       double* obu, double&) const {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const bool in = i + k < n;
      const int64_t q = in ? P.pos(i + k) : 0;
      oc[k] = in ? c[q] : 0.0;
      os[k] = in ? s[q] : 1.0;
      obl[k] = in ? bl[q] : 0.0;
      obu[k] = in ? bu[q] : 0.0;
    }
  }
  // a lane's two values never straddle a piece (i is even, kPiece too)
  template <int U>
  __device__ __forceinline__ void load_fast(int64_t base, int lane, double* oc, double* os,
                                            double* obl, double* obu, double&) const {
    dbl2u rc[U], rs[U], rl[U], ru[U];
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t q = P.pos(base + (int64_t)w * kWave * V + (int64_t)lane * V);
      rc[w] = ld16(c + q);
      rs[w] = ld16(s + q);
      rl[w] = ld16(bl + q);
      ru[w] = ld16(bu + q);
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
#pragma unroll
      for (int k = 0; k < V; ++k) {
        oc[w * V + k] = rc[w][k];
        os[w * V + k] = rs[w][k];
        obl[w * V + k] = rl[w][k];
        obu[w * V + k] = ru[w][k];
      }
    }
  }
};

// Runs tile(base, full) over one wave's tiles of TILE values in [0, count):
// steps of P adjacent tiles starting at `first`, `stride` apart; full tiles
// take the unguarded path, the tiles of the step that reaches `count` the
// checked one.  Reading P adjacent tiles (4 KB of each array for P = 2 in
// FP64) per step streams HBM faster than one tile per step.
template <int P, bool UNROLL, typename F>
__device__ __forceinline__ void for_tiles(int64_t count, int64_t first, int64_t stride,
                                          int64_t TILE, F&& tile) {
  int64_t base = first;
  for (; base + P * TILE <= count; base += stride) {
    if constexpr (UNROLL) {
#pragma unroll
      for (int p = 0; p < P; ++p) tile(base + p * TILE, std::true_type{});
    } else {
#pragma unroll 1
      for (int p = 0; p < P; ++p) tile(base + p * TILE, std::true_type{});
    }
  }
  for (int64_t b = base; b < count && b < base + P * TILE; b += TILE) {
    if (b + TILE <= count) tile(b, std::true_type{});
    else tile(b, std::false_type{});
  }
}

// How a pass treats the indices it evaluates.
enum PassMode {
  kEvalOnly = 0,   // phi and its slopes only (both sides marked given up)
  kTwoSides = 1,   // also compact for both brackets the evaluation can end with
  kSampled = 2     // also compact for the sampled bracket [lo, hi] (side 0 only)
};

// One wave streams its tiles.  With kTwoSides each index is also classified
// for both sides of the evaluation (see eval_index): the survivors of slot e
// of every lane are staged per side in the wave's slice of LDS (ballot +
// lane prefix count, slot after slot, so the layout is deterministic and
// needs no block-wide synchronisation) and written out kPiece = 64 at a
// time: one 512-byte store per array.  A side is given up for the whole pass
// (D_DROP) as soon as a flush would leave the wave with more than theta
// times the indices it has read: such a set would not pay for its writes,
// and a side given up early writes nothing.  At most theta * read + kPiece
// survivors are ever written, which bounds the wave's region.  With
// kSampled only side 0 exists, classified on [lo, hi] (spec_index), theta is
// the share the sample allows, and the ring is written kSpecFlush pieces at
// a time (at most theta * read + kSpecFlush * kPiece survivors).
// The LDS operations of one wave complete in issue order, so a lane reads
// what another lane staged without a wait; the wave-scope fences only keep
// the compiler from reordering those accesses.
template <typename Src, int MODE>
__device__ void eval_pass(const Src& src, int64_t count, int64_t first, int64_t stride, double lam,
                          double lo, double hi, double theta, double* const* out, Pieces op,
                          int32_t* const* out_cnt, Acc& acc, double* stg, int skip = 0) {
  constexpr bool COMPACT = MODE != kEvalOnly;
  constexpr int NSIDE = (MODE == kSampled) ? 1 : 2;
  constexpr int STG = (MODE == kSampled) ? kStageSpec : kStage;  // ring length
  constexpr int FP = (MODE == kSampled) ? kSpecFlush : 1;        // pieces per flush
  constexpr int V = Src::V;
  constexpr int U = kTileE / V;  // 16-byte vectors per lane and array
  constexpr int E = kTileE;
  constexpr int64_t TILE = (int64_t)kWave * E;
  const int lane = threadIdx.x & (kWave - 1);
  // per side: values written, ring head, values staged, given up
  int64_t written[2] = {0, 0};
  int head[2] = {0, 0}, pend[2] = {0, 0};
  // sides given up from the start: skip (bit k: side k), and side 1 of the
  // sampled-bracket pass
  bool drop[2] = {(skip & 1) != 0, MODE == kSampled || (skip & 2) != 0};
  int64_t seen = 0;  // indices read so far
  // `written` and `head` are multiples of kPiece at every full flush, so a
  // flush fills (the start of) one piece: a full one with 8 bytes per lane
  // and array, the last one value by value; non-temporal, like the other
  // streams
  auto flush = [&](int k, int m) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const double* sg = stg + k * 4 * STG;
    double* const* o = out + 4 * k;
    const int64_t p0 = op.pos(written[k]);
    if (lane < m) {
      const int q = (head[k] + lane) & (STG - 1);
#pragma unroll
      for (int j = 0; j < 4; ++j) __builtin_nontemporal_store(sg[j * STG + q], &o[j][p0 + lane]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    head[k] = (head[k] + m) & (STG - 1);
    written[k] += m;
    pend[k] -= m;
  };
  // full tiles take the unguarded path; only the last tile of a region checks
  // its range
  auto tile = [&](int64_t base, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    double c[E], s[E], bl[E], bu[E];
    if (FULL) {
      src.template load_fast<U>(base, lane, c, s, bl, bu, acc.s[P_BAD]);
    } else {
#pragma unroll
      for (int w = 0; w < U; ++w) {
        const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
        src.load(i, count, &c[w * V], &s[w * V], &bl[w * V], &bu[w * V], acc.s[P_BAD]);
      }
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        const bool in = FULL || i + k < count;
        int keep = 0;
        if (MODE == kSampled) {
          if (in) {
            eval_index<false>(acc, c[e], s[e], bl[e], bu[e], lam, lo, hi);
            keep = spec_index(acc, c[e], s[e], bl[e], bu[e], lo, hi);
          }
        } else {
          keep = in ? eval_index<COMPACT>(acc, c[e], s[e], bl[e], bu[e], lam, lo, hi) : 0;
        }
        seen += FULL ? kWave : __popcll(__ballot(in));
        if (COMPACT) {
#pragma unroll
          for (int side = 0; side < NSIDE; ++side) {
            if (drop[side]) continue;
            const bool kp = (keep >> side) & 1;
            const uint64_t m = __ballot(kp);
            if (kp) {
              double* sg = stg + side * 4 * STG;
              const int q = (head[side] + pend[side] + lane_prefix(m)) & (STG - 1);
              sg[q] = c[e];
              sg[STG + q] = s[e];
              sg[2 * STG + q] = bl[e];
              sg[3 * STG + q] = bu[e];
            }
            pend[side] += __popcll(m);
            // pend < FP * kPiece before this slot, so the ring never holds
            // more than FP * kPiece + 63 <= STG values
            if (pend[side] >= FP * kPiece) {
              if ((double)(written[side] + FP * kPiece) <= theta * (double)seen) {
#pragma unroll
                for (int f = 0; f < FP; ++f) flush(side, kPiece);
              } else {
                drop[side] = true;
              }
            }
          }
        }
      }
    }
  };
  // one side's ring leaves registers for both tiles' loads at once
  for_tiles<kPair, (MODE == kSampled) || kPairUnrollGeneral>(count, first, stride, TILE, tile);
  if (lane == 0) acc.s[P_NIN] += (double)seen;
  if (COMPACT) {
#pragma unroll
    for (int side = 0; side < NSIDE; ++side) {
      if (!drop[side] && pend[side] > 0) {
        if ((double)(written[side] + pend[side]) <= theta * (double)seen + FP * kPiece) {
          if constexpr (FP > 1) {
            while (pend[side] >= kPiece) flush(side, kPiece);
          }
          if (pend[side] > 0) flush(side, pend[side]);
        } else {
          drop[side] = true;
        }
      }
      if (lane == 0) {
        *out_cnt[side] = (int32_t)written[side];
        acc.s[P_SIDE + side * D_N + D_NOUT] += (double)written[side];
        acc.s[P_SIDE + side * D_N + D_DROP] += drop[side] ? 1.0 : 0.0;
      }
    }
  }
  // sides that were not written count as given up by every wave
  if (lane == 0) {
    if (!COMPACT) acc.s[P_SIDE + D_DROP] += 1.0;
    if (!COMPACT || NSIDE < 2) acc.s[P_SIDE + D_N + D_DROP] += 1.0;
  }
}

template <typename Src>
__device__ void bkpt_pass(const Src& src, int64_t count, int64_t first, int64_t stride, double lam,
                          KeySum* ks) {
  constexpr int V = Src::V;
  constexpr int U = kTileE / V;  // 16-byte vectors per lane and array
  constexpr int E = kTileE;
  constexpr int64_t TILE = (int64_t)kWave * E;
  const int lane = threadIdx.x & (kWave - 1);
  auto tile = [&](int64_t base, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    double c[E], s[E], bl[E], bu[E];
    double dummy = 0.0;
    if (FULL) {
      src.template load_fast<U>(base, lane, c, s, bl, bu, dummy);
    } else {
#pragma unroll
      for (int w = 0; w < U; ++w) {
        const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
        src.load(i, count, &c[w * V], &s[w * V], &bl[w * V], &bu[w * V], dummy);
      }
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        if (FULL || i + k < count) bkpt_index(ks, c[e], s[e], bl[e], bu[e], lam);
      }
    }
  };
  for_tiles<kPair, kPairUnrollGeneral>(count, first, stride, TILE, tile);
}


// One pass over the current index set.  Every block writes one partial
// record; the scalar update runs in gen_update_kernel, so no block needs a
// device-scope fence (the kernel boundary publishes the partials once).
template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_pass_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const int mode = st->mode;
  const int src = st->src;
  const bool compact = (mode == kModeEval) && (st->compaction != CQK_COMPACT_OFF);
  const double lam = st->lam, lo = st->lo, hi = st->hi, theta = st->theta;
  // the sides' brackets stay within the one the source's sums hold on
  const double clo = fmax(lo, st->vlo), chi = fmin(hi, st->vhi);
  // sides not to write, chosen by the update before this pass (plan_sides)
  const int skip = st->skip;
  // Passes over the caller's arrays hand tiles to waves grid-stride (tile t
  // to wave t mod NR), so all waves stream through neighbouring addresses;
  // wave rid keeps its survivors (at most `region`) in its pieces of a
  // compacted set, and later passes stream those pieces.
  const int rid = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
  const int64_t nr = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t plane = nr * A.region;  // one array of a compacted set
  const Pieces pc{rid, nr};

  __shared__ double lds[NPART * (kBlock / kWave)];
  __shared__ double tot[NPART];
  __shared__ double stage[kWavesPerBlock * 2 * 4 * kStage];
  double* stg = stage + (threadIdx.x / kWave) * 2 * 4 * kStage;

  Acc acc;
  acc_init(acc);
  KeySum ks[2] = {KeySum{inf_d(), 0.0}, KeySum{inf_d(), 0.0}};
  // the two sides' output sets and counts
  double* out[8];
  int32_t* oc[2];
  if (compact) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int d = side_dst(src, k) - 1;
      double* rb = A.buf[d];
#pragma unroll
      for (int j = 0; j < 4; ++j) out[4 * k + j] = rb + j * plane;
      oc[k] = A.cnt[d] + rid;
    }
  }
  if (src == 0) {
    SrcOrig<TIn> s{(const TIn*)A.d, (const TIn*)A.a, (const TIn*)A.b, (const TIn*)A.l,
                   (const TIn*)A.u};
    constexpr int64_t T = (int64_t)kWave * kTileE;
    const int64_t first = (int64_t)rid * kPair * T, stride = nr * kPair * T;
    if (mode != kModeEval)
      bkpt_pass(s, A.n, first, stride, lam, ks);
    else if (compact)
      eval_pass<SrcOrig<TIn>, kTwoSides>(s, A.n, first, stride, lam, clo, chi, theta, out, pc,
                                         oc, acc, stg, skip);
    else
      eval_pass<SrcOrig<TIn>, kEvalOnly>(s, A.n, first, stride, lam, lo, hi, theta, nullptr, pc,
                                         nullptr, acc, stg);
  } else {
    const double* sb = A.buf[src - 1];
    SrcForm s{sb, sb + plane, sb + 2 * plane, sb + 3 * plane, pc};
    constexpr int64_t T = (int64_t)kWave * kTileE;
    const int64_t count = A.cnt[src - 1][rid];
    // the wave's own region, front to back
    constexpr int64_t S = kPair * T;
    if (mode != kModeEval)
      bkpt_pass(s, count, 0, S, lam, ks);
    else if (compact)
      eval_pass<SrcForm, kTwoSides>(s, count, 0, S, lam, clo, chi, theta, out, pc, oc, acc, stg,
                                    skip);
    else
      eval_pass<SrcForm, kEvalOnly>(s, count, 0, S, lam, lo, hi, theta, nullptr, pc, nullptr,
                                    acc, stg);
  }

  if (mode == kModeEval) {
    block_reduce<NSUM, 0, 0, kBlock>(acc.s, nullptr, nullptr, lds, tot);
    if (threadIdx.x == 0) {
      write_partial(A.partials, tot, NPART);
    }
  } else {
    __shared__ KeySum ktot[2];
    block_ks_min<2, kBlock>(ks, lds, ktot);
    if (threadIdx.x == 0) {
      const double v[4] = {ktot[0].k, ktot[0].w, ktot[1].k, ktot[1].w};
      write_partial(A.partials, v, 4);
    }
  }
}

// The first Newton pass of a solve: an evaluation over the caller's arrays.
// Its bracket is one-sided at best, so each side would keep most indices and
// nothing is compacted; without the compaction rings and sums the kernel
// needs far fewer registers and no LDS beyond the block reduction, so more
// waves stream at once.  Same tiles and partial record as gen_pass_kernel
// (both sides marked as given up).
template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_first_pass_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const double lam = st->lam;
  const int lane = threadIdx.x & (kWave - 1);
  const int rid = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
  const int64_t nr = (int64_t)gridDim.x * kWavesPerBlock;
  SrcOrig<TIn> src{(const TIn*)A.d, (const TIn*)A.a, (const TIn*)A.b, (const TIn*)A.l,
                   (const TIn*)A.u};
  constexpr int V = SrcOrig<TIn>::V;
  constexpr int U = kTileE / V;  // 16-byte vectors per lane and array
  constexpr int E = kTileE;
  constexpr int64_t T = (int64_t)kWave * E;
  const int64_t count = A.n;
  Acc acc;
  acc_init(acc);
  int64_t seen = 0;
  auto tile = [&](int64_t base, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    double c[E], s[E], bl[E], bu[E];
    if (FULL) {
      src.template load_fast<U>(base, lane, c, s, bl, bu, acc.s[P_BAD]);
    } else {
#pragma unroll
      for (int w = 0; w < U; ++w) {
        const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
        src.load(i, count, &c[w * V], &s[w * V], &bl[w * V], &bu[w * V], acc.s[P_BAD]);
      }
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int64_t i = base + (int64_t)w * kWave * V + (int64_t)lane * V;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int e = w * V + k;
        if (FULL || i + k < count) eval_index<false>(acc, c[e], s[e], bl[e], bu[e], lam, 0.0, 0.0);
      }
    }
    seen += FULL ? T : std::min<int64_t>(T, count - base);
  };
  for_tiles<kPair, true>(count, (int64_t)rid * kPair * T, nr * kPair * T, T, tile);
  double v[6] = {acc.s[P_P], acc.s[P_A], acc.s[P_QP], acc.s[P_QM], acc.s[P_BAD],
                 lane == 0 ? (double)seen : 0.0};
  __shared__ double lds[6 * (kBlock / kWave)];
  __shared__ double tot[6];
  block_reduce<6, 0, 0, kBlock>(v, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    double rec[NPART];
#pragma unroll
    for (int i = 0; i < NPART; ++i) rec[i] = 0.0;
    rec[P_P] = tot[0];
    rec[P_A] = tot[1];
    rec[P_QP] = tot[2];
    rec[P_QM] = tot[3];
    rec[P_BAD] = tot[4];
    rec[P_NIN] = tot[5];
    rec[P_SIDE + D_DROP] = 1.0;
    rec[P_SIDE + D_N + D_DROP] = 1.0;
    write_partial(A.partials, rec, NPART);
  }
}

// The first Newton pass with a sampled bracket: the evaluation at lam_0 of
// gen_first_pass_kernel, and the indices whose breakpoints fall in the
// bracket [sp, sq] that gen_sample_kernel estimated written to compacted set
// 3 (kSpecSet), with the others' contributions summed (spec_index).
// Only one side's LDS ring.  When the sample gave no bracket, the plain
// evaluation.
template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_spec_pass_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const int rid = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
  const int64_t nr = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t plane = nr * A.region;
  const Pieces pc{rid, nr};
  __shared__ double lds[NPART * (kBlock / kWave)];
  __shared__ double tot[NPART];
  __shared__ double stage[kWavesPerBlock * 4 * kStageSpec];
  double* stg = stage + (threadIdx.x / kWave) * 4 * kStageSpec;
  Acc acc;
  acc_init(acc);
  SrcOrig<TIn> s{(const TIn*)A.d, (const TIn*)A.a, (const TIn*)A.b, (const TIn*)A.l,
                 (const TIn*)A.u};
  constexpr int64_t T = (int64_t)kWave * kTileE;
  const int64_t first = (int64_t)rid * kPair * T, stride = nr * kPair * T;
  const double lam = st->lam;
  if (st->spec != 0) {
    double* out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = A.buf[kSpecSet - 1] + j * plane;
    int32_t* oc[1] = {A.cnt[kSpecSet - 1] + rid};
    eval_pass<SrcOrig<TIn>, kSampled>(s, A.n, first, stride, lam, st->sp, st->sq, st->scap, out,
                                      pc, oc, acc, stg);
  } else {
    eval_pass<SrcOrig<TIn>, kEvalOnly>(s, A.n, first, stride, lam, 0.0, 0.0, 0.0, nullptr, pc,
                                       nullptr, acc, stg);
  }
  block_reduce<NSUM, 0, 0, kBlock>(acc.s, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, NPART);
}

// The lam_0 pass with the sampled bracket: the sums of eq. (CQKlambda0) --
// over a warm start's free set (WARM, end of Section 2.1, SrcOrigWarm) or
// over all indices (SrcOrigSum) -- and the indices with a breakpoint in
// [sp, sq] written to set 3 as the first Newton pass does without a lam_0
// pass (gen_spec_pass_kernel), so that the Newton pass at lam_0 can already
// read that set.  The sums travel in side 1's slots of the partial record
// (side 1 is not used).
template <typename TIn, bool WARM>
__global__ __launch_bounds__(kBlock) void gen_warm_spec_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const int rid = blockIdx.x * kWavesPerBlock + (int)(threadIdx.x / kWave);
  const int64_t nr = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t plane = nr * A.region;
  const Pieces pc{rid, nr};
  __shared__ double lds[NPART * (kBlock / kWave)];
  __shared__ double tot[NPART];
  __shared__ double stage[kWavesPerBlock * 4 * kStageSpec];
  double* stg = stage + (threadIdx.x / kWave) * 4 * kStageSpec;
  Acc acc;
  acc_init(acc);
  double wm[WS_N] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  using Src = typename std::conditional<WARM, SrcOrigWarm<TIn>, SrcOrigSum<TIn>>::type;
  Src s;
  if constexpr (WARM) {
    s = Src{(const TIn*)A.d, (const TIn*)A.a, (const TIn*)A.b, (const TIn*)A.l, (const TIn*)A.u,
            (const TIn*)A.xw, wm};
  } else {
    s = Src{{(const TIn*)A.d, (const TIn*)A.a, (const TIn*)A.b, (const TIn*)A.l, (const TIn*)A.u},
            wm};
  }
  constexpr int64_t T = (int64_t)kWave * kTileE;
  const int64_t first = (int64_t)rid * kPair * T, stride = nr * kPair * T;
  if (st->spec != 0) {
    double* out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = A.buf[kSpecSet - 1] + j * plane;
    int32_t* oc[1] = {A.cnt[kSpecSet - 1] + rid};
    eval_pass<Src, kSampled>(s, A.n, first, stride, 0.0, st->sp, st->sq, st->scap, out, pc, oc,
                             acc, stg);
  } else {
    eval_pass<Src, kEvalOnly>(s, A.n, first, stride, 0.0, 0.0, 0.0, 0.0, nullptr, pc, nullptr,
                              acc, stg);
  }
#pragma unroll
  for (int j = 0; j < WS_N; ++j) acc.s[P_SIDE + D_N + j] = wm[j];
  block_reduce<NSUM, 0, 0, kBlock>(acc.s, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, NPART);
}
static_assert(WS_N < D_DROP, "the warm sums fit side 1's slots below its drop count");

// lam_0 from gen_warm_spec_kernel's sums (as gen_warm_update_kernel, or
// gen_lambda0_update_kernel without a warm start), the sampled-bracket set
// kept waiting in set 3, and taken at once when lam_0 lies inside its
// bracket.
__global__ __launch_bounds__(kRBlock) void gen_warm_spec_update_kernel(GenArgs A, int G) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[NPART * (kRBlock / kWave)];
  __shared__ double tot[NPART];
  reduce_partials<NSUM, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    GenState sv = *st;
    GenState* s = &sv;
    const double* w = tot + P_SIDE + D_N;
    const double nout = tot[P_SIDE + D_NOUT];
    const bool warm = s->warm != 0;
    s->passes += 1;
    s->bytes += (warm ? s->in_bytes * 6.0 / 5.0 : s->in_bytes) * (double)A.n + 32.0 * nout;
    if (tot[P_BAD] > 0.0) {
      s->status = CQK_INVALID_ARG;
    } else {
      const double lam0 =
          (warm && w[WS_NJ] > 0.0) ? (s->r - w[WS_FIX] - w[WS_SJ]) / w[WS_QJ]
          : (w[WS_QALL] > 0.0)     ? (s->r - w[WS_SALL]) / w[WS_QALL]
                                   : 0.0;
      s->lam = lam0;
      s->lam0 = lam0;
      if (s->spec != 0 && tot[P_SIDE + D_DROP] == 0.0) {
        s->sF = tot[P_SIDE + D_F];
        s->sAF = tot[P_SIDE + D_AF];
        s->sC0 = tot[P_SIDE + D_C0];
        s->sC1 = tot[P_SIDE + D_C1];
        s->sA0 = tot[P_SIDE + D_A0];
        s->sA1 = tot[P_SIDE + D_A1];
        s->sn = (int64_t)nout;
        s->spend = 1;
      }
      s->spec = 0;
      take_spec_set(s, lam0);
      plan_sides(s);
      // over the caller's arrays the first Newton pass has a one-sided
      // bracket at best: neither side is written (as gen_first_pass_kernel)
      if (s->src == 0) s->skip = 3;
    }
    if (warm)
      trace_push(s, A.trace, 0, s->src != 0 ? 1 : 0, 0, s->lam, w[WS_SJ], w[WS_QJ], A.n,
                 (int64_t)w[WS_NJ]);
    else
      trace_push(s, A.trace, 0, s->src != 0 ? 1 : 0, 0, s->lam, w[WS_SALL], w[WS_QALL], A.n, 0);
    *st = sv;
  }
}

// Bracket estimate from a sample (a GPU addition to the variable fixing of
// Section 2.2, which lets the first pass compact; Algorithm 1 itself is
// unchanged), in three kernels.
//
// gen_sample_kernel: kSmpBlocks blocks read kSmpTiles tiles of 64
// consecutive indices spread evenly over [0, n), one tile per wave, and
// store them in the per-index form rounded to float; the last block to
// finish solves the sampled equation
//     (n/m) sum_{i in sample} g_i(lam) = r
// by Newton steps safeguarded by bisection.  By the delta method the
// solution's standard deviation is sd(g) sqrt(m) / sum_{sample, free} s_i,
// and the bracket is the solution +- kSmpWidth of those; the share of the
// sample with a breakpoint in it is counted.
//
// gen_sample2_kernel and gen_sample2_reduce_kernel: a sample kS2M / kSmpM
// times larger (kS2Tiles tiles in FP64, summed per block, the block records
// combined in order by one block) takes one Newton step of the same
// equation from the first solution (within a few of the first standard
// deviations of its own, where the sampled phi is close to linear).  The
// bracket is set as above, widened to take in Algorithm 1's first iterate
// as the sample predicts it when that is near, and the share is scaled by
// the bracket's width.  The share, with a margin, caps what the first pass
// may keep; a bracket that would keep more than half of theta is not used,
// nor one from a sample with invalid values (the first pass then only
// evaluates).  Whether lam* lies in the bracket does not matter for
// correctness: a pass at a multiplier outside reads the caller's arrays.
constexpr int kSmpThreads = 512;
constexpr int kSmpWaves = kSmpThreads / kWave;
constexpr int kSmpPer = 8;     // sampled indices per thread of the solving block
constexpr int kSmpTiles = kSmpWaves * kSmpPer;
constexpr int kSmpBlocks = kSmpTiles / kSmpWaves;
constexpr int64_t kSmpM = (int64_t)kSmpTiles * kWave;  // first sample's size
constexpr double kSmpWidth = 5.0;
constexpr int kSmpIter = 48;
constexpr int kS2Threads = 256;
constexpr int kS2Waves = kS2Threads / kWave;
constexpr int kS2PerWave = 8;  // tiles per wave
constexpr int kS2Blocks = 512;
constexpr double kS2Lam1Width = 4.0;
enum { S2_G = 0, S2_G2, S2_SF, S2_BAD, S2_G0, S2_QP0, S2_QM0, S2_C, S2_S, S2_N };
constexpr int kS2Tiles = kS2Blocks * kS2Waves * kS2PerWave;
constexpr int64_t kS2M = (int64_t)kS2Tiles * kWave;    // second sample's size
constexpr int64_t kSmpMinN = (int64_t)1 << 22;
static_assert(kSmpMinN >= (int64_t)kS2Tiles * kWave, "every sampled tile lies inside the arrays");

template <typename TIn>
__global__ __launch_bounds__(kSmpThreads) void gen_sample_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  {
    // the host launches this for n >= kSmpMinN only, so span >= 64 and
    // every tile lies inside [0, n)
    const int64_t span = A.n / kSmpTiles;
    const int j = blockIdx.x * kSmpWaves + w;
    const int64_t i = (int64_t)j * span + lane;
    const TIn* d = (const TIn*)A.d;
    const TIn* a = (const TIn*)A.a;
    const TIn* b = (const TIn*)A.b;
    const TIn* l = (const TIn*)A.l;
    const TIn* u = (const TIn*)A.u;
    double fc, fs, fl, fu, bad = 0.0;
    to_form((double)d[i], (double)a[i], (double)b[i], (double)l[i], (double)u[i], fc, fs, fl, fu,
            bad);
    flt4u v;
    v.x = (float)fc;
    v.y = (float)fs;
    v.z = (float)fl;
    v.w = (float)fu;
    const bool fin = __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && v.y > 0.0f &&
                     !__builtin_isnan(v.z) && !__builtin_isnan(v.w);
    // an entry that cannot be used is marked by s = NaN
    if (!(bad == 0.0 && fin)) v.y = __builtin_nanf("");
    *reinterpret_cast<flt4u*>(A.smp + 4 * ((int64_t)j * kWave + lane)) = v;
  }
  // the last block to finish reads every block's stores and solves (the
  // block's stores reach its L2 before the barrier; one device-scope release
  // by thread 0 then publishes them with the ticket)
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = (atomicAdd(&st->ticket, 1u) == (unsigned)(kSmpBlocks - 1));
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  float c[kSmpPer], s[kSmpPer], bl[kSmpPer], bu[kSmpPer];
  double nbad = 0.0;
#pragma unroll
  for (int k = 0; k < kSmpPer; ++k) {
    const flt4u v = *reinterpret_cast<const flt4u*>(A.smp + 4 * ((int64_t)k * kSmpThreads + threadIdx.x));
    c[k] = v.x;
    s[k] = v.y;
    bl[k] = v.z;
    bu[k] = v.w;
    nbad += __builtin_isnan(v.y) ? 1.0 : 0.0;
  }
  __shared__ double red[2][kSmpWaves][4];
  int par = 0;
  // block sums of four values, the same in every thread (fixed order)
  auto bsum = [&](double (&v)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) red[par][w][q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double t = 0.0;
      for (int ww = 0; ww < kSmpWaves; ++ww) t += red[par][ww][q];
      v[q] = t;
    }
    par ^= 1;
  };
  const double m = (double)kSmpM;
  const double rs = st->r * (m / (double)A.n);
  double lam = (double)(float)st->lam, lo = -inf_d(), hi = inf_d();
  bool found = false;
  {
    double v[4] = {nbad, 0.0, 0.0, 0.0};
    bsum(v);
    nbad = v[0];
  }
  // per-thread sums in float (the sample is float), block sums in double
  for (int it = 0; it < kSmpIter && nbad == 0.0; ++it) {
    const float lf = (float)lam;
    float t4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kSmpPer; ++k) {
      const float f = fmaf(s[k], lf, c[k]);
      const float g = fminf(fmaxf(f, bl[k]), bu[k]);
      t4[0] += g;
      t4[1] += fabsf(g);
      t4[2] += (f >= bl[k] && f < bu[k]) ? s[k] : 0.0f;
      t4[3] += (f > bl[k] && f <= bu[k]) ? s[k] : 0.0f;
    }
    double v[4] = {t4[0], t4[1], t4[2], t4[3]};
    bsum(v);
    const double res = v[0] - rs;
    if (fabs(res) <= 1e-7 * (v[1] + fabs(rs))) {
      found = true;
      break;
    }
    if (res < 0.0) lo = lam;
    else hi = lam;
    const double slope = (res < 0.0) ? v[2] : v[3];
    double next = (slope > 0.0) ? lam - res / slope : lam;
    if (!(next > lo && next < hi)) {
      if (lo > -inf_d() && hi < inf_d()) next = 0.5 * (lo + hi);
      else next = (res < 0.0) ? lam + (1.0 + fabs(lam)) : lam - (1.0 + fabs(lam));
    }
    // the multiplier is kept in float: a step that float cannot resolve ends
    // the search at the root's float resolution
    const double nf = (double)(float)next;
    if (nf == lam) {
      found = true;
      break;
    }
    lam = nf;
  }
  double p = __builtin_nan(""), q = __builtin_nan(""), sdl = 0.0, share = 1.0;
  if (found) {
    const float lf = (float)lam;
    float t3[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kSmpPer; ++k) {
      const float f = fmaf(s[k], lf, c[k]);
      const float g = fminf(fmaxf(f, bl[k]), bu[k]);
      t3[0] += g;
      t3[1] += g * g;
      t3[2] += (f > bl[k] && f < bu[k]) ? s[k] : 0.0f;
    }
    double v[4] = {t3[0], t3[1], t3[2], 0.0};
    bsum(v);
    const double mean = v[0] / m;
    const double sdg = sqrt(fmax(v[1] / m - mean * mean, 0.0));
    sdl = (v[2] > 0.0) ? sdg * sqrt(m) / v[2] : 0.0;
    const double half = kSmpWidth * sdl;
    if (half > 0.0 && half < inf_d()) {
      p = lam - half;
      q = lam + half;
      const float pf = (float)p, qf = (float)q;
      float kept = 0.0f;
#pragma unroll
      for (int k = 0; k < kSmpPer; ++k) {
        const float fp = fmaf(s[k], pf, c[k]);
        const float fq = fmaf(s[k], qf, c[k]);
        const bool at_l = fq <= bl[k], at_u = fp >= bu[k];
        const bool fr = !at_l && !at_u && fp >= bl[k] && fq <= bu[k] && (fp >= 0.0f || fq <= 0.0f);
        kept += (at_l || at_u || fr) ? 0.0f : 1.0f;
      }
      double w4[4] = {kept, 0.0, 0.0, 0.0};
      bsum(w4);
      share = w4[0] / m;
    }
  }
  if (threadIdx.x == 0) {
    st->s1ok = (p < q) ? 1 : 0;
    st->s1lam = lam;
    st->s1half = (p < q) ? 0.5 * (q - p) : 0.0;
    st->s1share = share;
    st->ticket = 0;
    st->passes += 1;
    st->bytes += st->in_bytes * m;
    if (st->ntrace < st->trace_cap) {
      cqk_trace_rec& t = A.trace[st->ntrace];
      t.iter = st->iter;
      t.kind = 8;
      t.compacted = 0;
      t.source = 0;
      t.lam = lam;
      t.phi = sdl;
      t.slope = share;
      t.lo = p;
      t.hi = q;
      t.n_in = kSmpM;
      t.n_out = (int64_t)(share * (double)A.n);
    }
    st->ntrace += 1;
  }
}

template <typename TIn>
__global__ __launch_bounds__(kS2Threads) void gen_sample2_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const bool ok1 = st->s1ok != 0;
  // at the first solution: sum g, sum g^2, sum of s over the free indices;
  // invalid entries; at lam_0: sum g and the one-sided slope sums
  double v[S2_N] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (ok1) {
    const double lam = st->s1lam, lam0 = st->lam;
    // n >= kSmpMinN: span >= 64, every tile inside [0, n)
    const int64_t span = A.n / kS2Tiles;
    const TIn* d = (const TIn*)A.d;
    const TIn* a = (const TIn*)A.a;
    const TIn* b = (const TIn*)A.b;
    const TIn* l = (const TIn*)A.l;
    const TIn* u = (const TIn*)A.u;
    TIn vd[kS2PerWave], va[kS2PerWave], vb[kS2PerWave], vl[kS2PerWave], vu[kS2PerWave];
#pragma unroll
    for (int k = 0; k < kS2PerWave; ++k) {
      const int j = (k * kS2Blocks + (int)blockIdx.x) * kS2Waves + w;
      const int64_t i = (int64_t)j * span + lane;
      vd[k] = d[i];
      va[k] = a[i];
      vb[k] = b[i];
      vl[k] = l[i];
      vu[k] = u[i];
    }
#pragma unroll
    for (int k = 0; k < kS2PerWave; ++k) {
      double c, s, bl, bu, bad = 0.0;
      to_form((double)vd[k], (double)va[k], (double)vb[k], (double)vl[k], (double)vu[k], c, s,
              bl, bu, bad);
      const double f = fma(s, lam, c);
      const double g = fmin(fmax(f, bl), bu);
      const double f0 = fma(s, lam0, c);
      const double g0 = fmin(fmax(f0, bl), bu);
      const bool fin = __builtin_isfinite(g) && __builtin_isfinite(s) && __builtin_isfinite(g0);
      v[S2_G] += fin ? g : 0.0;
      v[S2_G2] += fin ? g * g : 0.0;
      v[S2_SF] += (fin && f > bl && f < bu) ? s : 0.0;
      v[S2_BAD] += (bad == 0.0 && fin) ? 0.0 : 1.0;
      v[S2_G0] += fin ? g0 : 0.0;
      v[S2_QP0] += (fin && f0 >= bl && f0 < bu) ? s : 0.0;
      v[S2_QM0] += (fin && f0 > bl && f0 <= bu) ? s : 0.0;
      v[S2_C] += fin ? c : 0.0;
      v[S2_S] += fin ? s : 0.0;
    }
  }
  __shared__ double lds[S2_N * kS2Waves];
  __shared__ double tot[S2_N];
  block_reduce<S2_N, 0, 0, kS2Threads>(v, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, S2_N);
}

// Combines gen_sample2_kernel's block records in block order and sets the
// bracket (one block).
__global__ __launch_bounds__(kRBlock) void gen_sample2_reduce_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const bool ok1 = st->s1ok != 0;
  __shared__ double rl[S2_N * (kRBlock / kWave)];
  __shared__ double all[S2_N];
  reduce_partials<S2_N, 0, 0, kRBlock>(A.partials, kS2Blocks, rl, all);
  if (threadIdx.x == 0) {
    const double m = (double)kS2M;
    const double theta = st->theta;
    const double rs = st->r * (m / (double)A.n);
    double lam = __builtin_nan(""), p = __builtin_nan(""), q = __builtin_nan("");
    double sdl = 0.0, share = 1.0, lam1_pred = __builtin_nan("");
    bool use = false;
    if (ok1 && all[S2_BAD] == 0.0 && all[S2_SF] > 0.0) {
      lam = st->s1lam - (all[S2_G] - rs) / all[S2_SF];
      const double mean = all[S2_G] / m;
      sdl = sqrt(fmax(all[S2_G2] / m - mean * mean, 0.0)) * sqrt(m) / all[S2_SF];
      const double half = kSmpWidth * sdl;
      // the step stays within the first bracket, where one step is accurate
      if (half > 0.0 && half < inf_d() && fabs(lam - st->s1lam) < st->s1half) {
        p = lam - half;
        q = lam + half;
        // Algorithm 1's first point outside the sample's reach, predicted
        // from the sample: the first iterate from a known lam_0, or the
        // formula start's lam_0 itself (eq. (CQKlambda0) over the sample; a
        // warm start's is not predicted).  The bracket also takes it in
        // (with kS2Lam1Width deviations of margin) when that at most doubles
        // its width, so that the pass at it already reads the set.
        double lam1 = __builtin_nan("");
        if (st->lam0_later == 0) {
          const double res0 = all[S2_G0] - rs;
          const double sl0 = (res0 < 0.0) ? all[S2_QP0] : all[S2_QM0];
          if (sl0 > 0.0) lam1 = st->lam - res0 / sl0;
        } else if (st->warm == 0 && all[S2_S] > 0.0) {
          lam1 = (rs - all[S2_C]) / all[S2_S];
        }
        lam1_pred = lam1;
        const double p1 = fmin(p, lam1 - kS2Lam1Width * sdl);
        const double q1 = fmax(q, lam1 + kS2Lam1Width * sdl);
        if (q1 - p1 <= 4.0 * half) {
          p = p1;
          q = q1;
        }
        share = st->s1share * ((q - p) / (2.0 * st->s1half));
      }
    }
    if (!(p < q) && ok1) {
      // the first estimate's bracket
      lam = st->s1lam;
      p = st->s1lam - st->s1half;
      q = st->s1lam + st->s1half;
      share = st->s1share;
    }
    use = (p < q) && (share < 0.5 * theta);
    st->slam = (p < q) ? lam : __builtin_nan("");
    st->ssd = (p < q) ? ((sdl > 0.0 && !(lam == st->s1lam)) ? sdl : st->s1half / kSmpWidth)
                      : __builtin_nan("");
    st->sp = use ? p : __builtin_nan("");
    st->sq = use ? q : __builtin_nan("");
    st->scap = use ? fmin(theta, 1.5 * share + 1.0 / 32.0) : 0.0;
    st->spec = use ? 1 : 0;
    // a predicted first iterate of a known lam_0 left outside: the third
    // estimate looks at the second
    st->s2lam1 = (use && st->lam0_later == 0 && __builtin_isfinite(lam1_pred) &&
                  !(lam1_pred > p && lam1_pred < q))
                     ? lam1_pred
                     : __builtin_nan("");
    st->passes += 1;
    st->bytes += st->in_bytes * m;
    if (st->ntrace < st->trace_cap) {
      cqk_trace_rec& t = A.trace[st->ntrace];
      t.iter = st->iter;
      t.kind = 9;
      t.compacted = use ? 1 : 0;
      t.source = 0;
      t.lam = lam;
      t.phi = sdl;
      t.slope = share;
      t.lo = p;
      t.hi = q;
      t.n_in = kS2M;
      t.n_out = (int64_t)(share * (double)A.n);
    }
    st->ntrace += 1;
  }
}

// Third estimate: when Newton's first step from lam_0 lands outside the
// bracket (the sample predicts lam_1 far from lam*), the pass at lam_1 reads
// the caller's arrays, and so would the pass at lam_2 if that too lay
// outside.  gen_sample3_kernel evaluates the sampled phi and its one-sided
// slopes at the predicted lam_1 (kS3Tiles tiles, FP64, per-block sums);
// gen_sample3_reduce_kernel takes the Newton step from it and widens the
// bracket to the predicted lam_2 (+- kS3Width deviations) when that keeps
// it within kS3MaxWiden times the width of the bracket around lam* and the
// share allowed.  Both return at once when there is nothing to predict.
constexpr int kS3Blocks = 256;
constexpr int kS3Threads = 256;
constexpr int kS3Waves = kS3Threads / kWave;
constexpr int kS3PerWave = 4;
constexpr int kS3Tiles = kS3Blocks * kS3Waves * kS3PerWave;
constexpr int64_t kS3M = (int64_t)kS3Tiles * kWave;
constexpr double kS3Width = 6.0;
constexpr double kS3MaxWiden = 6.0;
static_assert(kSmpMinN >= (int64_t)kS3Tiles * kWave, "every sampled tile lies inside the arrays");
enum { S3_G = 0, S3_QP, S3_QM, S3_BAD, S3_N };

template <typename TIn>
__global__ __launch_bounds__(kS3Threads) void gen_sample3_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const double mu = st->s2lam1;
  if (!__builtin_isfinite(mu)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t span = A.n / kS3Tiles;  // n >= kSmpMinN: span >= 64
  const TIn* d = (const TIn*)A.d;
  const TIn* a = (const TIn*)A.a;
  const TIn* b = (const TIn*)A.b;
  const TIn* l = (const TIn*)A.l;
  const TIn* u = (const TIn*)A.u;
  TIn vd[kS3PerWave], va[kS3PerWave], vb[kS3PerWave], vl[kS3PerWave], vu[kS3PerWave];
#pragma unroll
  for (int k = 0; k < kS3PerWave; ++k) {
    const int j = (k * kS3Blocks + (int)blockIdx.x) * kS3Waves + w;
    const int64_t i = (int64_t)j * span + lane;
    vd[k] = d[i];
    va[k] = a[i];
    vb[k] = b[i];
    vl[k] = l[i];
    vu[k] = u[i];
  }
  double v[S3_N] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kS3PerWave; ++k) {
    double c, s, bl, bu, bad = 0.0;
    to_form((double)vd[k], (double)va[k], (double)vb[k], (double)vl[k], (double)vu[k], c, s, bl,
            bu, bad);
    const double f = fma(s, mu, c);
    const double g = fmin(fmax(f, bl), bu);
    const bool fin = __builtin_isfinite(g) && __builtin_isfinite(s);
    v[S3_G] += fin ? g : 0.0;
    v[S3_QP] += (fin && f >= bl && f < bu) ? s : 0.0;
    v[S3_QM] += (fin && f > bl && f <= bu) ? s : 0.0;
    v[S3_BAD] += (bad == 0.0 && fin) ? 0.0 : 1.0;
  }
  __shared__ double lds[S3_N * kS3Waves];
  __shared__ double tot[S3_N];
  block_reduce<S3_N, 0, 0, kS3Threads>(v, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, S3_N);
}

__global__ __launch_bounds__(kRBlock) void gen_sample3_reduce_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  const double mu = st->s2lam1;
  if (!__builtin_isfinite(mu)) return;
  __shared__ double rl[S3_N * (kRBlock / kWave)];
  __shared__ double all[S3_N];
  reduce_partials<S3_N, 0, 0, kRBlock>(A.partials, kS3Blocks, rl, all);
  if (threadIdx.x == 0) {
    const double m = (double)kS3M;
    const double res = all[S3_G] - st->r * (m / (double)A.n);
    const double sl = (res < 0.0) ? all[S3_QP] : all[S3_QM];
    const double p = st->sp, q = st->sq, ssd = st->ssd;
    if (all[S3_BAD] == 0.0 && sl > 0.0 && p < q) {
      const double lam2 = mu - res / sl;
      const double p2 = fmin(p, lam2 - kS3Width * ssd);
      const double q2 = fmax(q, lam2 + kS3Width * ssd);
      const double base = 2.0 * kSmpWidth * ssd;
      const double share = st->s1share * ((q2 - p2) / (2.0 * st->s1half));
      if (q2 - p2 <= kS3MaxWiden * base && share < 0.5 * st->theta) {
        st->sp = p2;
        st->sq = q2;
        st->scap = fmin(st->theta, 1.5 * share + 1.0 / 32.0);
        // the second estimate's trace record shows the bracket used
        const int ti = st->ntrace - 1;
        if (ti >= 0 && ti < st->trace_cap && A.trace[ti].kind == 9) {
          A.trace[ti].lo = p2;
          A.trace[ti].hi = q2;
          A.trace[ti].slope = share;
          A.trace[ti].n_out = (int64_t)(share * (double)A.n);
        }
      }
    }
    st->bytes += st->in_bytes * m;
  }
}

// Combines the G partial records of the pass in block order and runs the
// scalar part of Algorithm 1 (one block).
__global__ __launch_bounds__(kRBlock) void gen_update_kernel(GenArgs A, int G) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[NPART * (kRBlock / kWave)];
  __shared__ double tot[NPART];
  // the scalar update works on a register copy of the state record (one
  // round trip to memory instead of one per field access)
  if (st->mode == kModeEval) {
    reduce_partials<NSUM, 0, 0, kRBlock>(A.partials, G, lds, tot);
    if (threadIdx.x == 0) {
      GenState s = *st;
      update_after_eval(&s, tot, A.trace);
      *st = s;
    }
  } else {
    __shared__ KeySum ktot[2];
    reduce_partials_ks<2, kRBlock>(A.partials, G, lds, ktot);
    if (threadIdx.x == 0) {
      GenState s = *st;
      update_after_bkpt(&s, ktot, A.trace);
      *st = s;
    }
  }
}

// eq. (CQKlambda0) with J = all indices: lam0 = (r - sum b a/d) / sum b^2/d,
// plus the input checks.
template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_lambda0_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  const int64_t bchunk = A.chunk * kWavesPerBlock;
  const int64_t off = (int64_t)blockIdx.x * bchunk;
  const int64_t count = max((int64_t)0, min(bchunk, A.n - off));
  SrcOrig<TIn> src{(const TIn*)A.d + off, (const TIn*)A.a + off, (const TIn*)A.b + off,
                   (const TIn*)A.l + off, (const TIn*)A.u + off};
  double sums[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)threadIdx.x * V; i < count; i += (int64_t)kBlock * V) {
    double c[V], s[V], bl[V], bu[V];
    src.load(i, count, c, s, bl, bu, sums[2]);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (i + k < count) {
        sums[0] += c[k];
        sums[1] += s[k];
      }
    }
  }
  __shared__ double lds[3 * (kBlock / kWave)];
  __shared__ double tot[3];
  block_reduce<3, 0, 0, kBlock>(sums, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, 3);
  }
}

__global__ __launch_bounds__(kRBlock) void gen_lambda0_update_kernel(GenArgs A, int G) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[3 * (kRBlock / kWave)];
  __shared__ double tot[3];
  reduce_partials<3, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->passes += 1;
    st->bytes += st->in_bytes * (double)A.n;
    if (tot[2] > 0.0) {
      st->status = CQK_INVALID_ARG;
    } else {
      const double lam0 = (tot[1] > 0.0) ? (st->r - tot[0]) / tot[1] : 0.0;
      st->lam = lam0;
      st->lam0 = lam0;
    }
    trace_push(st, A.trace, 0, 0, 0, st->lam, tot[0], tot[1], A.n, 0);
  }
}

// Warm start from a primal estimate xbar (end of Section 2.1): the indices
// strictly inside their bounds in xbar are taken as free, an index at or
// beyond a bound as fixed at that bound, and lam_0 is the multiplier of that
// guess, eq. (CQKlambda0) over the free set J with the fixed indices' b x on
// the right-hand side:
//   lam_0 = (r - sum_{xbar <= l} b l - sum_{xbar >= u} b u - sum_J b a/d)
//           / sum_J b^2/d.
// With J empty the estimate is discarded: eq. (CQKlambda0) over all indices.
// Also the input checks.  (An entry of xbar that is NaN counts nowhere.)
enum { WM_SJ = 0, WM_QJ, WM_FIX, WM_NJ, WM_SALL, WM_QALL, WM_BAD, WM_NSUM };

template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_warm_kernel(GenArgs A) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  constexpr int V = VecWidth<TIn>::value;
  const int64_t n = A.n;
  const TIn* d = (const TIn*)A.d;
  const TIn* a = (const TIn*)A.a;
  const TIn* b = (const TIn*)A.b;
  const TIn* l = (const TIn*)A.l;
  const TIn* u = (const TIn*)A.u;
  const TIn* xw = (const TIn*)A.xw;
  double acc[WM_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * V; i < n;
       i += (int64_t)gridDim.x * kBlock * V) {
    double vd[V], va[V], vb[V], vl[V], vu[V], vx[V];
    Vec<TIn, V>::load(d, i, n, 1.0, vd);
    Vec<TIn, V>::load(a, i, n, 0.0, va);
    Vec<TIn, V>::load(b, i, n, 1.0, vb);
    Vec<TIn, V>::load(l, i, n, 0.0, vl);
    Vec<TIn, V>::load(u, i, n, 0.0, vu);
    Vec<TIn, V>::load(xw, i, n, 0.0, vx);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (i + k < n) {
        double c, s, bl, bu, bad = 0.0;
        to_form(vd[k], va[k], vb[k], vl[k], vu[k], c, s, bl, bu, bad);
        const bool fr = (vx[k] > vl[k]) && (vx[k] < vu[k]);
        const bool at_l = !fr && (vx[k] <= vl[k]);
        const bool at_u = !fr && (vx[k] >= vu[k]);
        acc[WM_SJ] += fr ? c : 0.0;
        acc[WM_QJ] += fr ? s : 0.0;
        acc[WM_NJ] += fr ? 1.0 : 0.0;
        acc[WM_FIX] += at_l ? bl : (at_u ? bu : 0.0);
        acc[WM_SALL] += c;
        acc[WM_QALL] += s;
        acc[WM_BAD] += bad;
      }
    }
  }
  __shared__ double lds[WM_NSUM * (kBlock / kWave)];
  __shared__ double tot[WM_NSUM];
  block_reduce<WM_NSUM, 0, 0, kBlock>(acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) write_partial(A.partials, tot, WM_NSUM);
}

__global__ __launch_bounds__(kRBlock) void gen_warm_update_kernel(GenArgs A, int G) {
  GenState* st = A.st;
  if (st->status != kRunning) return;
  __shared__ double lds[WM_NSUM * (kRBlock / kWave)];
  __shared__ double tot[WM_NSUM];
  reduce_partials<WM_NSUM, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->passes += 1;
    st->bytes += (st->in_bytes * 6.0 / 5.0) * (double)A.n;  // the five arrays and xbar
    if (tot[WM_BAD] > 0.0) {
      st->status = CQK_INVALID_ARG;
    } else {
      const double lam0 = (tot[WM_NJ] > 0.0)
                              ? (st->r - tot[WM_FIX] - tot[WM_SJ]) / tot[WM_QJ]
                              : (st->r - tot[WM_SALL]) / tot[WM_QALL];
      st->lam = lam0;
      st->lam0 = lam0;
    }
    trace_push(st, A.trace, 0, 0, 0, st->lam, tot[WM_SJ], tot[WM_QJ], A.n, (int64_t)tot[WM_NJ]);
  }
}

// x_i = clamp((a_i + lam b_i)/d_i, l_i, u_i) over all n (eq. (xopt)), with
// b^T x, sum |b x| and the free count reduced for the caller's info.
template <typename TIn>
__global__ __launch_bounds__(kBlock) void gen_finalize_kernel(GenArgs A) {
  GenState* st = A.st;
  const int status = st->status;
  if (status != CQK_OK && status != CQK_NOT_CONVERGED) return;
  constexpr int V = VecWidth<TIn>::value;
  const double lam = st->lam_final;
  const int64_t count = A.n;
  const TIn* d = (const TIn*)A.d;
  const TIn* a = (const TIn*)A.a;
  const TIn* b = (const TIn*)A.b;
  const TIn* l = (const TIn*)A.l;
  const TIn* u = (const TIn*)A.u;
  TIn* x = (TIn*)A.x;
  double sums[3] = {0.0, 0.0, 0.0};
  // x_i from the loaded values; the residual sums use x as stored
  auto map = [&](const double* vd, const double* va, const double* vb, const double* vl,
                 const double* vu, int64_t i, TIn* xo) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const double t = fma(vb[k], lam, va[k]) / vd[k];
      const double xv = fmin(fmax(t, vl[k]), vu[k]);
      xo[k] = (TIn)xv;
      const double xr = (double)xo[k];
      if (i + k < count) {
        sums[0] += vb[k] * xr;
        sums[1] += fabs(vb[k] * xr);
        sums[2] += (xr > vl[k] && xr < vu[k]) ? 1.0 : 0.0;
      }
    }
  };
  // Tiles go to blocks grid-stride, four vectors per thread and array in
  // flight: with every block streaming its own contiguous part instead, this
  // read + write stream ran ~8 % slower.
  constexpr int U = 4;
  constexpr int64_t TILE = (int64_t)kBlock * V * U;
  for (int64_t base = (int64_t)blockIdx.x * TILE; base < count;
       base += (int64_t)gridDim.x * TILE) {
    if (base + TILE <= count) {
      // full tile: every load issued before the first use
      typename Raw16<TIn>::type rd[U], ra[U], rb[U], rl[U], ru[U];
#pragma unroll
      for (int w = 0; w < U; ++w) {
        const int64_t i = base + (int64_t)w * kBlock * V + (int64_t)threadIdx.x * V;
        rd[w] = ld16(d + i);
        ra[w] = ld16(a + i);
        rb[w] = ld16(b + i);
        rl[w] = ld16(l + i);
        ru[w] = ld16(u + i);
      }
#pragma unroll
      for (int w = 0; w < U; ++w) {
        const int64_t i = base + (int64_t)w * kBlock * V + (int64_t)threadIdx.x * V;
        double vd[V], va[V], vb[V], vl[V], vu[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
          vd[k] = rd[w][k];
          va[k] = ra[w][k];
          vb[k] = rb[w][k];
          vl[k] = rl[w][k];
          vu[k] = ru[w][k];
        }
        TIn xo[V];
        map(vd, va, vb, vl, vu, i, xo);
        typename Raw16<TIn>::type o;
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = xo[k];
        st16(x + i, o);
      }
    } else {
      for (int64_t i = base + (int64_t)threadIdx.x * V; i < min(count, base + TILE);
           i += (int64_t)kBlock * V) {
        double vd[V], va[V], vb[V], vl[V], vu[V];
        Vec<TIn, V>::load(d, i, count, 1.0, vd);
        Vec<TIn, V>::load(a, i, count, 0.0, va);
        Vec<TIn, V>::load(b, i, count, 0.0, vb);
        Vec<TIn, V>::load(l, i, count, 0.0, vl);
        Vec<TIn, V>::load(u, i, count, 0.0, vu);
        TIn xo[V];
        map(vd, va, vb, vl, vu, i, xo);
#pragma unroll
        for (int k = 0; k < V; ++k)
          if (i + k < count) x[i + k] = xo[k];
      }
    }
  }
  __shared__ double lds[3 * (kBlock / kWave)];
  __shared__ double tot[3];
  block_reduce<3, 0, 0, kBlock>(sums, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) {
    write_partial(A.partials, tot, 3);
  }
}

__global__ __launch_bounds__(kRBlock) void gen_finalize_reduce_kernel(GenArgs A, int G) {
  GenState* st = A.st;
  const int status = st->status;
  if (status != CQK_OK && status != CQK_NOT_CONVERGED) return;
  __shared__ double lds[3 * (kRBlock / kWave)];
  __shared__ double tot[3];
  reduce_partials<3, 0, 0, kRBlock>(A.partials, G, lds, tot);
  if (threadIdx.x == 0) {
    st->res_P = tot[0];
    st->res_A = tot[1];
    st->n_free = (int64_t)tot[2];
  }
}

__global__ void gen_init_kernel(GenState* st, GenState init) { *st = init; }

int choose_grid(int64_t n, int num_cus) {
  const int64_t want = (n + 1023) / 1024;
  const int64_t cap = (int64_t)num_cus * 8;
  return (int)std::max<int64_t>(1, std::min(want, cap));
}

}  // namespace

// G blocks of kWavesPerBlock waves.  A pass over the caller's arrays hands
// its steps (kPair adjacent tiles of 64 lanes x kTileE values) to the NR waves grid-stride, at most `tpw` steps each (chunk = tpw
// steps).  A wave keeps at most theta * chunk + kSpecFlush * kPiece survivors
// of a side (eval_pass), so its region in a compacted set holds that many values,
// rounded up to whole pieces.  The primal recovery runs grid-stride on its
// own grid GF of 4-vector tiles.  Workspace: partials | counts (3 x NR) |
// with compaction: the sample of gen_sample_kernel and three compacted sets
// (4 planes of NR x region doubles each).
GenLayout gen_layout(int64_t n, int num_cus, int vec, bool compaction, double theta) {
  GenLayout L{};
  const int64_t T = (int64_t)kWave * kTileE * kPair;
  const int G0 = choose_grid(n, num_cus);
  const int64_t ntiles = (n + T - 1) / T;
  const int64_t tpw = std::max<int64_t>(
      1, (ntiles + (int64_t)G0 * kWavesPerBlock - 1) / ((int64_t)G0 * kWavesPerBlock));
  L.chunk = tpw * T;
  const int64_t bchunk = L.chunk * kWavesPerBlock;
  L.G = (int)std::max<int64_t>(1, (n + bchunk - 1) / bchunk);
  L.NR = L.G * kWavesPerBlock;
  const double th = std::min(1.0, std::max(0.0, theta));
  const int64_t keep = (int64_t)std::ceil(th * (double)L.chunk) + kSpecFlush * kPiece;
  // a multiple of kPiece (so of 16): every plane starts a 128-byte line
  L.region = std::min<int64_t>((L.chunk + kPiece - 1) / kPiece * kPiece,
                               (keep + kPiece - 1) / kPiece * kPiece);
  const int64_t ftile = (int64_t)kBlock * vec * 4;
  L.GF = (int)std::max<int64_t>(1, std::min<int64_t>(4 * (int64_t)L.G, (n + ftile - 1) / ftile));
  L.part_bytes = ((size_t)L.G * NPART * sizeof(double) + 255) / 256 * 256;
  L.cnt_bytes = ((size_t)3 * L.NR * sizeof(int32_t) + 255) / 256 * 256;
  const size_t buf_bytes =
      compaction ? (size_t)3 * 4 * (size_t)L.NR * (size_t)L.region * sizeof(double) : 0;
  // the sampled-bracket estimate's sample (4 floats per index)
  L.smp_bytes = compaction ? (size_t)kSmpM * 4 * sizeof(float) : 0;
  L.bytes = L.part_bytes + L.cnt_bytes + L.smp_bytes + buf_bytes;
  return L;
}

// theta of a call: the options' if they give one, else the context's (0.5
// unless set or tuned); COMPACT_ALWAYS keeps every side whatever its size
double gen_theta(const cqk_ctx* ctx, const cqk_opts& o) {
  if (o.compaction == CQK_COMPACT_ALWAYS) return 1.0;
  return (o.compact_theta > 0.0) ? o.compact_theta : ctx->theta;
}

namespace {

template <typename TIn>
cqk_status run_general(cqk_ctx* ctx, int64_t n, const TIn* d, const TIn* a, const TIn* b,
                       const TIn* l, const TIn* u, const TIn* xw, double r, TIn* x,
                       const cqk_opts& o, cqk_info* info) {
  const bool compaction = o.compaction != CQK_COMPACT_OFF;
  const double theta = gen_theta(ctx, o);
  const GenLayout Lg = gen_layout(n, ctx->num_cus, VecWidth<TIn>::value, compaction, theta);
  const int G = Lg.G, NR = Lg.NR, GF = Lg.GF;
  const int64_t chunk = Lg.chunk;
  const size_t part_bytes = Lg.part_bytes, cnt_bytes = Lg.cnt_bytes;
  cqk_status stt = ensure_buffer(ctx, ctx->ws, Lg.bytes);
  if (stt != CQK_OK) return stt;
  const size_t st_bytes = 1024 + sizeof(cqk_trace_rec) * kMaxTrace;
  stt = ensure_buffer(ctx, ctx->state, st_bytes);
  if (stt != CQK_OK) return stt;

  char* ws = (char*)ctx->ws.ptr;
  GenArgs A{};
  A.d = d;
  A.a = a;
  A.b = b;
  A.l = l;
  A.u = u;
  A.xw = xw;
  A.x = x;
  A.n = n;
  A.chunk = chunk;
  A.region = Lg.region;
  A.partials = (double*)ws;
  A.cnt[0] = (int32_t*)(ws + part_bytes);
  A.cnt[1] = A.cnt[0] + NR;
  A.cnt[2] = A.cnt[1] + NR;
  if (compaction) {
    A.smp = (float*)(ws + part_bytes + cnt_bytes);
    double* bb = (double*)(ws + part_bytes + cnt_bytes + Lg.smp_bytes);
    for (int k = 0; k < 3; ++k) A.buf[k] = bb + (size_t)k * 4 * NR * Lg.region;
  }
  A.st = (GenState*)ctx->state.ptr;
  A.trace = (cqk_trace_rec*)((char*)ctx->state.ptr + 1024);

  const bool is_f32 = sizeof(TIn) == 4;
  const double eps = (is_f32 && o.accum == CQK_ACCUM_F32) ? 1.1920928955078125e-07
                                                          : 2.220446049250313e-16;
  // With compaction on large inputs, a bracket estimated from a sample lets
  // the first pass compact (gen_sample_kernel, gen_sample2_kernel); below
  // kSmpMinN the sample costs more than it saves.  A warm or formula start
  // then runs its lam_0 pass after the sample and writes the sampled set
  // itself (gen_warm_spec_kernel), and the first Newton pass is a general
  // one.
  // (the second estimate's block records use the partials buffer)
  const bool sampled = compaction && n >= kSmpMinN && (int64_t)G * NPART >= (int64_t)kS2Blocks * S2_N;
  const bool formula = xw == nullptr && o.lambda0_mode == CQK_LAMBDA0_FORMULA;
  const bool warm_spec = sampled && (xw != nullptr || formula);
  GenState init{};
  init.lam = (o.lambda0_mode == CQK_LAMBDA0_USER && xw == nullptr) ? o.lambda0_user : 0.0;
  init.lam0 = init.lam;
  init.lam_prev = __builtin_nan("");
  init.lo = -__builtin_huge_val();
  init.hi = __builtin_huge_val();
  init.phi_lo = init.phi_hi = __builtin_nan("");
  init.r = r;
  init.tol = (o.tol > 0.0) ? o.tol : std::pow(eps, 0.75);
  init.theta = theta;
  init.n_src = n;
  init.n_all = n;
  init.vlo = -__builtin_huge_val();
  init.vhi = __builtin_huge_val();
  init.sp = init.sq = __builtin_nan("");
  init.slam = init.ssd = init.s2lam1 = __builtin_nan("");
  init.warm = (xw != nullptr) ? 1 : 0;
  init.lam0_later = warm_spec ? 1 : 0;
  init.in_bytes = 5.0 * sizeof(TIn);
  init.status = kRunning;
  init.max_iter = o.max_iter;
  init.compaction = o.compaction;
  init.trace_cap = o.trace ? kMaxTrace : 0;
  init.nblocks = G;
  init.lam_final = __builtin_nan("");

  hipStream_t s = ctx->stream;
  // sync = 0 or graph capture: every pass the iteration cap allows is queued
  // at once (those after the loop stops return at once) and nothing is read
  // back; cqk_ctx_last_info reads the result later.  No per-pass timing then.
  const bool deferred = !o.sync || stream_capturing(s);
  const bool timing = o.timing && !deferred;
  // timing 2: only the first Newton pass and the recovery carry events (the
  // runtime leaves a few microseconds around every timed dispatch)
  const bool timing_all = timing && o.timing != 2;
  // events 0, 1: the finalize of the last batch; then one pair per grid pass
  const size_t nev = (size_t)2 + 2 * (o.max_iter * 2 + 8);
  if (timing) {
    stt = ensure_events(ctx, nev);
    if (stt != CQK_OK) return stt;
  }
  hipLaunchKernelGGL(gen_init_kernel, dim3(1), dim3(1), 0, s, A.st, init);
  if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  int ev = 2;
  int npass = 0;  // grid passes queued
  // a grid pass (timed when asked) followed by its one-block reduction
  auto launch = [&](auto kern, auto reduce, bool first_newton) {
    const bool rec = (timing_all || (timing && first_newton)) && ev + 2 <= (int)nev;
    launch_timed(kern, dim3(G), dim3(kBlock), s, rec ? ctx->events[ev] : nullptr,
                 rec ? ctx->events[ev + 1] : nullptr, A);
    if (rec) ev += 2;
    ++npass;
    hipLaunchKernelGGL(reduce, dim3(1), dim3(kRBlock), 0, s, A, G);
  };
  // The primal recovery does nothing while the loop still runs, so it is
  // queued behind every batch and the host waits once per batch.
  auto finalize = [&]() {
    launch_timed(gen_finalize_kernel<TIn>, dim3(GF), dim3(kBlock), s,
                 timing ? ctx->events[0] : nullptr, timing ? ctx->events[1] : nullptr, A);
    hipLaunchKernelGGL(gen_finalize_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A, GF);
  };
  if (xw != nullptr && !warm_spec)
    launch(gen_warm_kernel<TIn>, gen_warm_update_kernel, false);
  else if (formula && !warm_spec)
    launch(gen_lambda0_kernel<TIn>, gen_lambda0_update_kernel, false);
  if (sampled) {
    bool rec = timing_all && ev + 2 <= (int)nev;
    launch_timed(gen_sample_kernel<TIn>, dim3(kSmpBlocks), dim3(kSmpThreads), s,
                 rec ? ctx->events[ev] : nullptr, rec ? ctx->events[ev + 1] : nullptr, A);
    if (rec) ev += 2;
    rec = timing_all && ev + 2 <= (int)nev;
    launch_timed(gen_sample2_kernel<TIn>, dim3(kS2Blocks), dim3(kS2Threads), s,
                 rec ? ctx->events[ev] : nullptr, rec ? ctx->events[ev + 1] : nullptr, A);
    if (rec) ev += 2;
    hipLaunchKernelGGL(gen_sample2_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A);
    npass += 2;
    if (!warm_spec) {
      hipLaunchKernelGGL(gen_sample3_kernel<TIn>, dim3(kS3Blocks), dim3(kS3Threads), 0, s, A);
      hipLaunchKernelGGL(gen_sample3_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, A);
    }
  }
  if (warm_spec && xw != nullptr)
    launch(gen_warm_spec_kernel<TIn, true>, gen_warm_spec_update_kernel, false);
  else if (warm_spec)
    launch(gen_warm_spec_kernel<TIn, false>, gen_warm_spec_update_kernel, false);
  GenState* hs = (GenState*)ctx->host_pinned;
  int launched = 0;
  const int max_launch = 2 * o.max_iter + 4;
  // the first Newton pass evaluates the caller's arrays: with the sampled
  // bracket it also compacts for it, else the lean kernel runs; every later
  // pass the general one
  auto pass = [&]() {
    if (launched == 0 && warm_spec) launch(gen_pass_kernel<TIn>, gen_update_kernel, true);
    else if (launched == 0 && sampled) launch(gen_spec_pass_kernel<TIn>, gen_update_kernel, true);
    else if (launched == 0) launch(gen_first_pass_kernel<TIn>, gen_update_kernel, true);
    else launch(gen_pass_kernel<TIn>, gen_update_kernel, false);
    ++launched;
  };
  if (deferred) {
    while (launched < max_launch) pass();
    finalize();
    if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
  } else {
    // Algorithm 1 typically stops after five to seven evaluations here
    int batch = 6;
    while (launched < max_launch) {
      const int k = std::min(batch, max_launch - launched);
      for (int i = 0; i < k; ++i) pass();
      finalize();
      if (hip_ok(hipGetLastError()) != CQK_OK) return CQK_DEVICE_ERROR;
      if (hip_ok(hipMemcpyAsync(hs, A.st, sizeof(GenState), hipMemcpyDeviceToHost, s)) != CQK_OK)
        return CQK_DEVICE_ERROR;
      if (hip_ok(hipStreamSynchronize(s)) != CQK_OK) return CQK_DEVICE_ERROR;
      if (hs->status != kRunning) break;
      batch = 4;
    }
  }
  const int pass_events = ev;
  const int trace_cap = init.trace_cap;
  // Fills an info record from the state copy in hs (the stream synchronised),
  // reading the trace ring too.
  auto report = [ctx, hs, A, trace_cap, n, r, timing, pass_events, npass](cqk_info* inf) -> cqk_status {
    const int ntrace = std::min(hs->ntrace, trace_cap);
    ctx->last_trace.resize(ntrace);
    ctx->last_trace_count = hs->ntrace;
    if (ntrace > 0) {
      if (hip_ok(hipMemcpy(ctx->last_trace.data(), A.trace, sizeof(cqk_trace_rec) * ntrace,
                           hipMemcpyDeviceToHost)) != CQK_OK)
        return CQK_DEVICE_ERROR;
    }
    std::memset(inf, 0, sizeof(*inf));
    inf->status = (hs->status == kRunning) ? CQK_NOT_CONVERGED : hs->status;
    inf->iterations = hs->iter;
    inf->passes = hs->passes;
    inf->stop_reason = hs->stop_reason;
    inf->lambda = hs->lam_final;
    inf->lambda0 = hs->lam0;
    inf->residual = std::fabs(hs->res_P - r);
    inf->abs_bx = hs->res_A;
    inf->n_free = hs->n_free;
    inf->n_after_init = 0;
    inf->finalize_bytes = (double)n * (6.0 * sizeof(TIn));
    inf->pass_launches = npass;
    ctx->last_pass_ms.clear();
    if (timing) {
      // every grid pass queued; those after the loop stopped returned at once
      for (int i = 2; i + 1 < pass_events; i += 2) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]);
        inf->pass_ms += ms;
        ctx->last_pass_ms.push_back(ms);
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, ctx->events[0], ctx->events[1]);
      inf->finalize_ms = ms;
    }
    // algorithmic bytes of the grid passes, summed on the device
    inf->pass_bytes = hs->bytes;
    return CQK_OK;
  };
  ctx->last = [hs, A, report](cqk_info* inf) -> cqk_status {
    if (hip_ok(hipMemcpy(hs, A.st, sizeof(GenState), hipMemcpyDeviceToHost)) != CQK_OK)
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
  return report(info ? info : &tmp);
}

}  // namespace

cqk_status run_general_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                           const double* b, const double* l, const double* u, const double* xw,
                           double r, double* x, const cqk_opts& o, cqk_info* info) {
  return run_general<double>(ctx, n, d, a, b, l, u, xw, r, x, o, info);
}

cqk_status run_general_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                           const float* b, const float* l, const float* u, const float* xw,
                           double r, float* x, const cqk_opts& o, cqk_info* info) {
  return run_general<float>(ctx, n, d, a, b, l, u, xw, r, x, o, info);
}

}  // namespace cqk
