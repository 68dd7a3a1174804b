// Device building blocks shared by the libcqk kernels (gfx950, wave64).
//
// Reductions are deterministic: a fixed xor butterfly inside the wave, wave
// results combined in wave order through LDS, block partials combined in
// block order by the last block to finish (ticket counter).  Repeated calls
// on the same input give bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cqk {

constexpr int kWave = 64;

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef int32_t int4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double inf_d() { return __builtin_huge_val(); }

// ---------------------------------------------------------------------------
// Wave reductions: xor butterfly, every lane ends with the same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
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
// `lds` needs (NS + NM + NX) * (blockDim/64) doubles.  Thread 0 receives the
// block totals in out[] (combined in wave order).
// ---------------------------------------------------------------------------
template <int NS, int NM, int NX, int BLOCK>
__device__ __forceinline__ void block_reduce(const double* sums, const double* mins,
                                             const double* maxs, double* lds, double* out) {
  constexpr int NW = BLOCK / kWave;
  constexpr int NV = NS + NM + NX;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double v = wave_sum(sums[i]);
    if (lane == 0) lds[i * NW + wid] = v;
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
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double acc = lds[i * NW];
      for (int w = 1; w < NW; ++w) {
        double t = lds[i * NW + w];
        if (i < NS) acc += t;
        else if (i < NS + NM) acc = fmin(acc, t);
        else acc = fmax(acc, t);
      }
      out[i] = acc;
    }
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

// ---------------------------------------------------------------------------
// Grid completion ticket: returns true in exactly one block, the last one to
// arrive, after every other block's partial is visible to it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool last_block_arrives(uint32_t* ticket) {
  __shared__ bool s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    uint32_t t = atomicAdd(ticket, 1u);
    s_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last;
}

// Deterministic reduction of G partial records of NV doubles (first NS are
// sums, then NM mins, then NX maxes) by the whole block; thread 0 gets out[].
template <int NS, int NM, int NX, int BLOCK>
__device__ __forceinline__ void reduce_partials(const double* partials, int G, double* lds,
                                                double* out) {
  constexpr int NV = NS + NM + NX;
  double s[NS > 0 ? NS : 1], mn[NM > 0 ? NM : 1], mx[NX > 0 ? NX : 1];
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NM; ++i) mn[i] = inf_d();
#pragma unroll
  for (int i = 0; i < NX; ++i) mx[i] = -inf_d();
  for (int g = threadIdx.x; g < G; g += BLOCK) {
    const double* p = partials + (size_t)g * NV;
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] += __builtin_nontemporal_load(p + i);
#pragma unroll
    for (int i = 0; i < NM; ++i) mn[i] = fmin(mn[i], __builtin_nontemporal_load(p + NS + i));
#pragma unroll
    for (int i = 0; i < NX; ++i) mx[i] = fmax(mx[i], __builtin_nontemporal_load(p + NS + NM + i));
  }
  block_reduce<NS, NM, NX, BLOCK>(s, mn, mx, lds, out);
}

// ---------------------------------------------------------------------------
// Vector loads with a count guard (16-byte loads where the whole vector is in
// range, element loads otherwise; out-of-range lanes get `fill`).
// ---------------------------------------------------------------------------
template <typename T, int V>
struct Vec;
template <>
struct Vec<double, 2> {
  static __device__ __forceinline__ void load(const double* p, int64_t i, int64_t n, double fill,
                                              double* o) {
    if (i + 2 <= n) {
      dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(p + i));
      o[0] = v.x;
      o[1] = v.y;
    } else {
      o[0] = (i < n) ? p[i] : fill;
      o[1] = fill;
    }
  }
};
template <>
struct Vec<float, 4> {
  static __device__ __forceinline__ void load(const float* p, int64_t i, int64_t n, double fill,
                                              double* o) {
    if (i + 4 <= n) {
      flt4 v = __builtin_nontemporal_load(reinterpret_cast<const flt4*>(p + i));
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
