// Device building blocks shared by the libcqk kernels (gfx950, wave64).
//
// Reductions are deterministic: a fixed sequence of lane exchanges inside the
// wave, wave results combined in wave order through LDS, block partials
// combined in a fixed order by a one-block reduction kernel.  Repeated calls
// on the same input give bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cqk {

constexpr int kWave = 64;

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));
// 16-byte vectors at element alignment: global_load/store_dwordx4 needs only
// dword alignment, so rows and views that start anywhere still move 16 bytes
// per lane per access.
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float flt4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef int32_t int4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double inf_d() { return __builtin_huge_val(); }

// ---------------------------------------------------------------------------
// Wave reductions through DPP lane moves (no LDS round trip): pairs and quads
// (quad_perm), eight and sixteen lanes (half-row and row mirrors), then rows
// 0+1 and 2+3 (row_bcast15) and all four rows (row_bcast31) into lane 63,
// read back as a scalar.  Every lane gets the same bits, and the order of
// the operations is fixed, so repeated calls agree bit for bit.  Must be
// called with the whole wave active.
// ---------------------------------------------------------------------------
namespace dpp {
constexpr int kXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141;
constexpr int kMirror = 0x140;
constexpr int kBcast15 = 0x142;
constexpr int kBcast31 = 0x143;
}  // namespace dpp

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v, float identity) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                         __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v, double identity) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t o = __builtin_bit_cast(uint64_t, identity);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u,
                                                            CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      (int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float read_lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double read_lane63(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T identity, Op op) {
  v = op(v, dpp_move<dpp::kXor1, 0xF>(v, identity));
  v = op(v, dpp_move<dpp::kXor2, 0xF>(v, identity));
  v = op(v, dpp_move<dpp::kHalfMirror, 0xF>(v, identity));
  v = op(v, dpp_move<dpp::kMirror, 0xF>(v, identity));
  v = op(v, dpp_move<dpp::kBcast15, 0xA>(v, identity));
  v = op(v, dpp_move<dpp::kBcast31, 0xC>(v, identity));
  return read_lane63(v);
}

struct OpAdd {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMin {
  __device__ __forceinline__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
  __device__ __forceinline__ double operator()(double a, double b) const { return fmax(a, b); }
};

__device__ __forceinline__ double wave_sum(double v) { return wave_reduce(v, 0.0, OpAdd{}); }
__device__ __forceinline__ float wave_sum(float v) { return wave_reduce(v, 0.0f, OpAdd{}); }
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, __builtin_huge_val(), OpMin{});
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, -__builtin_huge_val(), OpMax{});
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Number of set bits of a wave mask below this lane.
__device__ __forceinline__ int lane_prefix(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum of a 32-bit count across the wave (Hillis-Steele).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Block reductions of NS sums and NM mins / NX maxes held per thread.
// `lds` needs (NS + NM + NX) * (blockDim/64) doubles; `out` is in LDS and
// holds the block totals (combined in wave order) for every thread on return.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Many sums over a wave by halving exchanges: at each of the six lane bits
// (5, 4 through cross-row swizzles; 3, 2, 1, 0 through DPP mirrors and quad
// permutes, each pairing lanes with opposite bit) a lane keeps half of the
// values it still holds, adds its partner's copy of that half, and hands the
// other half to the partner; once one value is left the remaining steps add
// the partner's value.  N sums then cost about N exchanges instead of the 6N
// of one butterfly per value.  Afterwards lane l holds in v[0] the total of
// value (l >> (6 - log2 N)) & (N - 1); lanes that share it hold the same
// bits.  Whole wave active.
// ---------------------------------------------------------------------------
namespace detail {
template <int BIT>
__device__ __forceinline__ double lane_swap(double v) {
  if constexpr (BIT == 5) return __shfl_xor(v, 32, kWave);
  else if constexpr (BIT == 4) return __shfl_xor(v, 16, kWave);
  else if constexpr (BIT == 3) return dpp_move<dpp::kMirror, 0xF>(v, 0.0);
  else if constexpr (BIT == 2) return dpp_move<dpp::kHalfMirror, 0xF>(v, 0.0);
  else if constexpr (BIT == 1) return dpp_move<dpp::kXor2, 0xF>(v, 0.0);
  else return dpp_move<dpp::kXor1, 0xF>(v, 0.0);
}

template <int BIT, int M>
__device__ __forceinline__ void halve(double* v, int lane) {
  if constexpr (M > 1) {
    const bool low = ((lane >> BIT) & 1) == 0;
#pragma unroll
    for (int k = 0; k < M / 2; ++k) {
      const double send = low ? v[M / 2 + k] : v[k];
      const double keep = low ? v[k] : v[M / 2 + k];
      v[k] = keep + lane_swap<BIT>(send);
    }
  } else {
    v[0] = v[0] + lane_swap<BIT>(v[0]);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int at_least_one(int n) { return n < 1 ? 1 : n; }
}  // namespace detail

template <int N>
__device__ __forceinline__ void wave_sum_many(double* v) {
  static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "N: a power of two up to 64");
  const int lane = threadIdx.x & (kWave - 1);
  detail::halve<5, N>(v, lane);
  detail::halve<4, detail::at_least_one(N / 2)>(v, lane);
  detail::halve<3, detail::at_least_one(N / 4)>(v, lane);
  detail::halve<2, detail::at_least_one(N / 8)>(v, lane);
  detail::halve<1, detail::at_least_one(N / 16)>(v, lane);
  detail::halve<0, detail::at_least_one(N / 32)>(v, lane);
}

template <int NS, int NM, int NX, int BLOCK>
__device__ __forceinline__ void block_reduce(const double* sums, const double* mins,
                                             const double* maxs, double* lds, double* out) {
  constexpr int NW = BLOCK / kWave;
  constexpr int NV = NS + NM + NX;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  if constexpr (NS >= 4) {
    static_assert(NS <= 32, "at most 32 sums");
    constexpr int N = (NS <= 4) ? 4 : (NS <= 8) ? 8 : (NS <= 16) ? 16 : 32;
    constexpr int SH = 6 - detail::ilog2(N);
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = (i < NS) ? sums[i] : 0.0;
    wave_sum_many<N>(v);
    const int idx = (lane >> SH) & (N - 1);
    if ((lane & ((1 << SH) - 1)) == 0 && idx < NS) lds[idx * NW + wid] = v[0];
  } else {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double v = wave_sum(sums[i]);
      if (lane == 0) lds[i * NW + wid] = v;
    }
  }
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    double v = wave_min(mins[i]);
    if (lane == 0) lds[(NS + i) * NW + wid] = v;
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    double v = wave_max(maxs[i]);
    if (lane == 0) lds[(NS + NM + i) * NW + wid] = v;
  }
  __syncthreads();
  // one thread per value combines the waves, in wave order
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    double acc = lds[i * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const double t = lds[i * NW + w];
      if (i < NS) acc += t;
      else if (i < NS + NM) acc = fmin(acc, t);
      else acc = fmax(acc, t);
    }
    out[i] = acc;
  }
  __syncthreads();
}

// Exclusive block scan of one count per thread; returns the thread's offset
// and writes the block total to *total (all threads).  `lds_i` needs
// BLOCK/64 + 1 ints.
template <int BLOCK>
__device__ __forceinline__ int block_excl_scan(int v, int* lds_i, int* total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  int incl = wave_incl_scan(v);
  if (lane == kWave - 1) lds_i[wid] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    int t = lds_i[w];
    base += (w < wid) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// Partial records are stored value-major: value i of block g at
// partials[i * G + g], so the reducing block reads them coalesced.
__device__ __forceinline__ void write_partial(double* partials, const double* v, int nv) {
  for (int i = 0; i < nv; ++i) partials[(size_t)i * gridDim.x + blockIdx.x] = v[i];
}

// Deterministic reduction of G partial records of NV doubles (first NS are
// sums, then NM mins, then NX maxes) by the whole block; out[] (shared) holds
// the results for every thread on return.  Records are value-major, so value
// i of all G records is one contiguous row.  Each row is cut into S segments
// (S = NW / NV when there are fewer rows than waves), and wave w takes the
// (row, segment) items w, w + NW, ...: each lane combines its strided share
// of the segment with all of a round's loads in flight, one butterfly
// combines the lanes, and the segments of a row are combined in order at the
// end.  lds must hold NV * (BLOCK / kWave) doubles.
template <int NS, int NM, int NX, int BLOCK>
__device__ __forceinline__ void reduce_partials(const double* partials, int G, double* lds,
                                                double* out) {
  constexpr int NV = NS + NM + NX;
  constexpr int NW = BLOCK / kWave;
  constexpr int S = (NV < NW) ? NW / NV : 1;
  constexpr int R = 32;  // loads per lane and round
  const int lane = threadIdx.x & (kWave - 1);
  const int seg = ((G + S - 1) / S + kWave - 1) / kWave * kWave;
  for (int j = (int)(threadIdx.x / kWave); j < NV * S; j += NW) {
    const int i = j / S;
    const int kind = (i < NS) ? 0 : ((i < NS + NM) ? 1 : 2);  // wave-uniform
    const double idv = (kind == 0) ? 0.0 : ((kind == 1) ? inf_d() : -inf_d());
    const double* row = partials + (size_t)i * G;
    const int g_end = min(G, (j % S + 1) * seg);
    double a = idv;
    for (int g0 = (j % S) * seg; g0 < g_end; g0 += kWave * R) {
      double v[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int g = g0 + k * kWave + lane;
        v[k] = (g < g_end) ? row[g] : idv;
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < R; ++k)
        a = (kind == 0) ? a + v[k] : ((kind == 1) ? fmin(a, v[k]) : fmax(a, v[k]));
    }
    a = (kind == 0) ? wave_sum(a) : ((kind == 1) ? wave_min(a) : wave_max(a));
    if (lane == 0) lds[j] = a;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    const int kind = (i < NS) ? 0 : ((i < NS + NM) ? 1 : 2);
    double a = lds[i * S];
    for (int q = 1; q < S; ++q) {
      const double v = lds[i * S + q];
      a = (kind == 0) ? a + v : ((kind == 1) ? fmin(a, v) : fmax(a, v));
    }
    out[i] = a;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// (key, weight) reduction: the smallest key with the summed weight of every
// entry holding that key.  Associative and commutative, so the butterfly and
// the ordered block/grid combination give the same bits everywhere.
// ---------------------------------------------------------------------------
struct KeySum {
  double k, w;
};

__device__ __forceinline__ KeySum ks_min(KeySum a, KeySum b) {
  if (a.k < b.k) return a;
  if (b.k < a.k) return b;
  return KeySum{a.k, a.w + b.w};
}

__device__ __forceinline__ KeySum wave_ks_min(KeySum v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    KeySum t{__shfl_xor(v.k, o, kWave), __shfl_xor(v.w, o, kWave)};
    v = ks_min(v, t);
  }
  return v;
}

// NK key-sum pairs per thread -> thread 0 gets the block result.
template <int NK, int BLOCK>
__device__ __forceinline__ void block_ks_min(const KeySum* v, double* lds, KeySum* out) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    KeySum r = wave_ks_min(v[i]);
    if (lane == 0) {
      lds[(2 * i) * NW + wid] = r.k;
      lds[(2 * i + 1) * NW + wid] = r.w;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      KeySum acc{lds[(2 * i) * NW], lds[(2 * i + 1) * NW]};
      for (int w = 1; w < NW; ++w) acc = ks_min(acc, KeySum{lds[(2 * i) * NW + w], lds[(2 * i + 1) * NW + w]});
      out[i] = acc;
    }
  }
  __syncthreads();
}

// Grid version over G partial records of NK pairs (k0, w0, k1, w1, ...).
template <int NK, int BLOCK>
__device__ __forceinline__ void reduce_partials_ks(const double* partials, int G, double* lds,
                                                   KeySum* out) {
  KeySum acc[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) acc[i] = KeySum{inf_d(), 0.0};
  for (int g = threadIdx.x; g < G; g += BLOCK) {
#pragma unroll
    for (int i = 0; i < NK; ++i)
      acc[i] = ks_min(acc[i], KeySum{partials[(size_t)(2 * i) * G + g],
                                     partials[(size_t)(2 * i + 1) * G + g]});
  }
  block_ks_min<NK, BLOCK>(acc, lds, out);
}

// ---------------------------------------------------------------------------
// Vector loads with a count guard: one 16-byte load where the whole vector is
// in range, element loads otherwise; out-of-range lanes get `fill`.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool aligned16(const void* p) {
  return ((uintptr_t)p & 15u) == 0;
}

// Unguarded 16-byte load / store at element alignment; the caller has
// checked the range.  Both are non-temporal: the data is streamed once.
// (Ordinary stores make an output kernel look faster on its own, but leave
// dirty lines that the next kernel then pays to write back: whole solves
// in a loop ran 2 % slower with them.)
template <typename T>
struct Raw16;
template <>
struct Raw16<double> {
  typedef dbl2u type;
};
template <>
struct Raw16<float> {
  typedef flt4u type;
};
template <typename T>
__device__ __forceinline__ typename Raw16<T>::type ld16(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename Raw16<T>::type*>(p));
}
template <typename T>
__device__ __forceinline__ void st16(T* p, typename Raw16<T>::type v) {
  __builtin_nontemporal_store(v, reinterpret_cast<typename Raw16<T>::type*>(p));
}

template <typename T, int V>
struct Vec;
template <>
struct Vec<double, 2> {
  static __device__ __forceinline__ void load(const double* p, int64_t i, int64_t n, double fill,
                                              double* o) {
    if (i + 2 <= n) {
      dbl2u v = ld16(p + i);
      o[0] = v.x;
      o[1] = v.y;
    } else {
      o[0] = (i < n) ? p[i] : fill;
      o[1] = (i + 1 < n) ? p[i + 1] : fill;
    }
  }
};
template <>
struct Vec<float, 4> {
  static __device__ __forceinline__ void load(const float* p, int64_t i, int64_t n, double fill,
                                              double* o) {
    if (i + 4 <= n) {
      flt4u v = ld16(p + i);
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k] = (i + k < n) ? (double)p[i + k] : fill;
    }
  }
};

template <typename T>
struct VecWidth;
template <>
struct VecWidth<double> {
  static constexpr int value = 2;
};
template <>
struct VecWidth<float> {
  static constexpr int value = 4;
};

}  // namespace cqk
