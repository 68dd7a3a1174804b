// Spectral projected gradient (SPG) on the l1-constrained least-squares
// problem of Section 5.2 (basis pursuit):
//     min 1/2 ||A x - b||^2   s.t.  ||x||_1 <= radius,
// with every projection onto the l1 ball done by the library's projection
// (Section 3.2, Algorithm 4 with Algorithm 2 as the start), warm-started from
// the current iterate as Section 3.1 suggests.  The SPG steps are those of
// Birgin, Martinez and Raydan's SPG2: x_0 = 0, the spectral step
// lam_{k+1} = s's / s'y clipped to [1e-30, 1e30] (the first one
// 1/||P(x_0 - g_0) - x_0||_inf), the direction d = P(x - lam g) - x, and a
// non-monotone line search over the last `memory` objective values with
// safeguarded quadratic interpolation; stop when ||P(x - g) - x||_inf <= tol.
//
// For this f the line search needs no extra product: with r = A x - b and
// Ad = A d,  f(x + t d) = f(x) + t g'd + t^2/2 ||Ad||^2  (g'd = r'Ad), and
// s'y = t^2 ||Ad||^2, s's = t^2 ||d||^2, so each iteration costs two
// products with A (A d, then A^T r at the new point) and two projections
// (the direction and the stopping test).
//
// A is dense, row-major m x n, FP64.  Kernels:
//   spg_gemv_n_kernel   y = A v (- b): one block per row, 16-byte loads;
//   spg_gemv_t_kernel   partial column sums of A^T v over row chunks,
//   spg_cols_kernel     the chunks summed in order (deterministic);
//   spg_vec_kernel      fused vector updates with their reductions;
//   spg_reduce_kernel   one block: the partial records to a result array.
// The host runs the scalar part and reads a few reduced values per step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "cqk_device.h"
#include "cqk_internal.h"

namespace cqk {
namespace {

constexpr int kBlock = 256;
constexpr int kRBlock = 1024;
constexpr int kRowsPerChunk = 128;  // rows per block of the transposed product
constexpr int kColsPerBlock = 2 * kBlock;
constexpr double kLMin = 1e-30, kLMax = 1e30, kGamma = 1e-4, kSigma1 = 0.1, kSigma2 = 0.9;

// y_i = sum_j A_ij v_j (minus b_i when b is given); one block per row.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void spg_gemv_n_kernel(const double* A, const double* v,
                                                           const double* b, int64_t n,
                                                           double* y) {
  const int64_t i = blockIdx.x;
  const double* row = A + i * n;
  double acc = 0.0;
  if (VEC) {
    // row and v 16-byte aligned (n even): pairs, four in flight per thread
    const int64_t np = n / 2;
    const double2* r2 = reinterpret_cast<const double2*>(row);
    const double2* v2 = reinterpret_cast<const double2*>(v);
    int64_t j = threadIdx.x;
    for (; j + 3 * kBlock < np; j += 4 * kBlock) {
      double2 a[4], w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a[k] = r2[j + k * kBlock];
        w[k] = v2[j + k * kBlock];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += a[k].x * w[k].x + a[k].y * w[k].y;
    }
    for (; j < np; j += kBlock) {
      const double2 a = r2[j], w = v2[j];
      acc += a.x * w.x + a.y * w.y;
    }
  } else {
    for (int64_t j = threadIdx.x; j < n; j += kBlock) acc += row[j] * v[j];
  }
  __shared__ double lds[kBlock / kWave];
  __shared__ double tot[1];
  block_reduce<1, 0, 0, kBlock>(&acc, nullptr, nullptr, lds, tot);
  if (threadIdx.x == 0) y[i] = b ? tot[0] - b[i] : tot[0];
}

// part[c][j] = sum over the rows of chunk c of v_i A_ij; block (x: column
// tile of kColsPerBlock, y: chunk c), two adjacent columns per thread.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void spg_gemv_t_kernel(const double* A, const double* v,
                                                           int64_t m, int64_t n, double* part) {
  const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + 2 * (int64_t)threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kRowsPerChunk;
  const int64_t i1 = min(i0 + (int64_t)kRowsPerChunk, m);
  double s0 = 0.0, s1 = 0.0;
  if (j < n) {
    if (VEC && j + 1 < n) {
      for (int64_t i = i0; i < i1; ++i) {
        const double2 a = *reinterpret_cast<const double2*>(A + i * n + j);
        const double w = v[i];
        s0 += w * a.x;
        s1 += w * a.y;
      }
    } else {
      const bool two = j + 1 < n;
      for (int64_t i = i0; i < i1; ++i) {
        const double w = v[i];
        s0 += w * A[i * n + j];
        if (two) s1 += w * A[i * n + j + 1];
      }
    }
    double* out = part + (int64_t)blockIdx.y * n;
    out[j] = s0;
    if (j + 1 < n) out[j + 1] = s1;
  }
}

// g_j = sum over chunks c (in order) of part[c][j].
__global__ __launch_bounds__(kBlock) void spg_cols_kernel(const double* part, int nchunk,
                                                          int64_t n, double* g) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n + j];
  g[j] = s;
}

// Fused vector steps over n (or m) values, each block writing one partial
// record of kVS sums (then one max):
//   OP_STEP:  out = x - lam g                                   (no sums)
//   OP_DIR:   d = p - x;  sums g'd, d'd;  max |d|
//   OP_AXPY:  x += t d  (n),                                    (no sums)
//   OP_DOT:   sums u'w, w'w, u'u  over m                        (no writes)
enum SpgOp { OP_STEP = 0, OP_DIR = 1, OP_AXPY = 2, OP_DOT = 3 };
constexpr int kVS = 3;

template <int OP>
__global__ __launch_bounds__(kBlock) void spg_vec_kernel(int64_t n, double c, const double* x,
                                                        const double* u, double* out,
                                                        double* partials) {
  double acc[kVS] = {0.0, 0.0, 0.0};
  double mx = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kBlock) {
    if (OP == OP_STEP) {
      out[j] = x[j] - c * u[j];
    } else if (OP == OP_DIR) {
      // x: the iterate, u: the gradient, out: in the projection p, out d
      const double dj = out[j] - x[j];
      out[j] = dj;
      acc[0] += u[j] * dj;
      acc[1] += dj * dj;
      mx = fmax(mx, fabs(dj));
    } else if (OP == OP_AXPY) {
      out[j] += c * u[j];
    } else {
      const double a = x[j], w = u[j];
      acc[0] += a * w;
      acc[1] += w * w;
      acc[2] += a * a;
    }
  }
  if (OP == OP_DIR || OP == OP_DOT) {
    __shared__ double lds[(kVS + 1) * (kBlock / kWave)];
    __shared__ double tot[kVS + 1];
    block_reduce<kVS, 0, 1, kBlock>(acc, nullptr, &mx, lds, tot);
    if (threadIdx.x == 0) write_partial(partials, tot, kVS + 1);
  }
}

// One block: G partial records of kVS sums and one max -> res[0..kVS].
__global__ __launch_bounds__(kRBlock) void spg_reduce_kernel(const double* partials, int G,
                                                             double* res) {
  __shared__ double lds[(kVS + 1) * (kRBlock / kWave)];
  __shared__ double tot[kVS + 1];
  reduce_partials<kVS, 0, 1, kRBlock>(partials, G, lds, tot);
  if (threadIdx.x <= kVS) res[threadIdx.x] = tot[threadIdx.x];
}

struct SpgWs {
  double *r, *Ad, *g, *z, *p, *d, *part, *partials, *res;
  int nchunk, gvec;
};

}  // namespace

void fill_default_spg_opts(cqk_spg_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-4;
  o->max_iter = 10000;
  o->memory = 10;
  o->warm = 1;
}

cqk_status run_spg_l1_lasso_f64(cqk_ctx* ctx, int64_t m, int64_t n, const double* A,
                                const double* b, double radius, double* x,
                                const cqk_spg_opts& so, cqk_spg_info* info) {
  using clock = std::chrono::steady_clock;
  const auto t_start = clock::now();
  double proj_ms = 0.0;
  hipStream_t s = ctx->stream;
  SpgWs W;
  W.nchunk = (int)((m + kRowsPerChunk - 1) / kRowsPerChunk);
  W.gvec = (int)std::max<int64_t>(1, std::min<int64_t>((std::max(m, n) + kBlock - 1) / kBlock,
                                                       (int64_t)ctx->num_cus * 4));
  auto al = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
  const size_t bm = al((size_t)m * 8), bn = al((size_t)n * 8);
  const size_t bpart = al((size_t)W.nchunk * n * 8);
  const size_t bpar = al((size_t)(kVS + 1) * W.gvec * 8);
  const size_t total = 2 * bm + 4 * bn + bpart + bpar + 256;
  cqk_status st = ensure_buffer(ctx, ctx->spg, total);
  if (st != CQK_OK) return st;
  char* w = (char*)ctx->spg.ptr;
  W.r = (double*)w;
  W.Ad = (double*)(w + bm);
  W.g = (double*)(w + 2 * bm);
  W.z = (double*)(w + 2 * bm + bn);
  W.p = (double*)(w + 2 * bm + 2 * bn);
  W.d = (double*)(w + 2 * bm + 3 * bn);
  W.part = (double*)(w + 2 * bm + 4 * bn);
  W.partials = (double*)(w + 2 * bm + 4 * bn + bpart);
  W.res = (double*)(w + 2 * bm + 4 * bn + bpart + bpar);
  // scalars come back through the upper half of the context's pinned buffer
  // (its start mirrors the projection's state)
  double* hres = (double*)((char*)ctx->host_pinned + ctx->host_pinned_bytes / 2);

  const bool vec = (n % 2 == 0) && ((uintptr_t)A % 16 == 0);
  auto gemv_n = [&](const double* v, const double* bb, double* y) {
    if (vec && ((uintptr_t)v % 16 == 0))
      hipLaunchKernelGGL(spg_gemv_n_kernel<true>, dim3((unsigned)m), dim3(kBlock), 0, s, A, v, bb, n, y);
    else
      hipLaunchKernelGGL(spg_gemv_n_kernel<false>, dim3((unsigned)m), dim3(kBlock), 0, s, A, v, bb, n, y);
  };
  auto gemv_t = [&](const double* v, double* out) {
    const dim3 grid((unsigned)((n + kColsPerBlock - 1) / kColsPerBlock), (unsigned)W.nchunk);
    if (vec)
      hipLaunchKernelGGL(spg_gemv_t_kernel<true>, grid, dim3(kBlock), 0, s, A, v, m, n, W.part);
    else
      hipLaunchKernelGGL(spg_gemv_t_kernel<false>, grid, dim3(kBlock), 0, s, A, v, m, n, W.part);
    hipLaunchKernelGGL(spg_cols_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, W.part, W.nchunk, n, out);
  };
  // queue a reduction and read its kVS + 1 results
  auto fetch = [&](double* dst) -> cqk_status {
    hipLaunchKernelGGL(spg_reduce_kernel, dim3(1), dim3(kRBlock), 0, s, W.partials, W.gvec, W.res);
    if (hip_ok(hipMemcpyAsync(dst, W.res, (kVS + 1) * sizeof(double), hipMemcpyDeviceToHost, s)) !=
        CQK_OK)
      return CQK_DEVICE_ERROR;
    return hip_ok(hipStreamSynchronize(s));
  };
  cqk_opts po;
  fill_default_opts(&po);
  po.lambda0_mode = CQK_LAMBDA0_CONDAT;
  int64_t nproj = 0, newton = 0;
  // p = P(z), warm-started from x when asked; returns the projection status
  auto project = [&](const double* z, double* p) -> cqk_status {
    const auto t0 = clock::now();
    cqk_info pi;
    cqk_status e = run_simplex_f64(ctx, n, z, so.warm ? x : nullptr, nullptr, radius, p, true,
                                   po, &pi);
    proj_ms += std::chrono::duration<double, std::milli>(clock::now() - t0).count();
    nproj += 1;
    newton += pi.iterations;
    if (e != CQK_OK) return e;
    return (pi.status == CQK_OK) ? CQK_OK : (cqk_status)pi.status;
  };

  // x_0 = 0 = P(0); r = A x_0 - b; g = A^T r
  if (hip_ok(hipMemsetAsync(x, 0, (size_t)n * 8, s)) != CQK_OK) return CQK_DEVICE_ERROR;
  gemv_n(x, b, W.r);
  double fx = 0.0;
  std::vector<double> hist;
  double lam = 1.0;
  int it = 0;
  int status = CQK_OK;
  double pg = 0.0;
  auto objective = [&]() -> cqk_status {
    hipLaunchKernelGGL(spg_vec_kernel<OP_DOT>, dim3(W.gvec), dim3(kBlock), 0, s, m, 0.0, W.r,
                       W.r, nullptr, W.partials);
    cqk_status e = fetch(hres);
    fx = 0.5 * hres[2];
    return e;
  };
  // the projected gradient at x: pg = ||P(x - g) - x||_inf
  auto proj_grad = [&]() -> cqk_status {
    hipLaunchKernelGGL(spg_vec_kernel<OP_STEP>, dim3(W.gvec), dim3(kBlock), 0, s, n, 1.0, x, W.g,
                       W.z, W.partials);
    cqk_status e = project(W.z, W.p);
    if (e != CQK_OK) return e;
    hipLaunchKernelGGL(spg_vec_kernel<OP_DIR>, dim3(W.gvec), dim3(kBlock), 0, s, n, 0.0, x, W.g,
                       W.p, W.partials);
    e = fetch(hres);
    pg = hres[kVS];
    return e;
  };
  gemv_t(W.r, W.g);
  cqk_status e = objective();
  if (e != CQK_OK) return e;
  hist.push_back(fx);
  e = proj_grad();
  if (e != CQK_OK) return e;
  lam = (pg > 0.0) ? std::min(kLMax, std::max(kLMin, 1.0 / pg)) : 1.0;
  const int M = std::max(1, so.memory);
  while (pg > so.tol) {
    if (it >= so.max_iter) {
      status = CQK_NOT_CONVERGED;
      break;
    }
    // d = P(x - lam g) - x, with g'd and d'd
    hipLaunchKernelGGL(spg_vec_kernel<OP_STEP>, dim3(W.gvec), dim3(kBlock), 0, s, n, lam, x, W.g,
                       W.z, W.partials);
    e = project(W.z, W.d);
    if (e != CQK_OK) return e;
    hipLaunchKernelGGL(spg_vec_kernel<OP_DIR>, dim3(W.gvec), dim3(kBlock), 0, s, n, 0.0, x, W.g,
                       W.d, W.partials);
    if ((e = fetch(hres)) != CQK_OK) return e;
    const double gtd = hres[0], dd = hres[1];
    // Ad and ||Ad||^2
    gemv_n(W.d, nullptr, W.Ad);
    hipLaunchKernelGGL(spg_vec_kernel<OP_DOT>, dim3(W.gvec), dim3(kBlock), 0, s, m, 0.0, W.Ad,
                       W.Ad, nullptr, W.partials);
    if ((e = fetch(hres)) != CQK_OK) return e;
    const double c2 = hres[1];
    // non-monotone line search on f(x + t d) = f + t gtd + t^2/2 c2
    const size_t h0 = (hist.size() > (size_t)M) ? hist.size() - M : 0;
    const double fmax = *std::max_element(hist.begin() + h0, hist.end());
    double t = 1.0, fn = 0.0;
    for (int ls = 0; ls < 200; ++ls) {
      fn = fx + t * gtd + 0.5 * t * t * c2;
      if (fn <= fmax + kGamma * t * gtd) break;
      const double tq = -0.5 * t * t * gtd / (fn - fx - t * gtd);
      t = (tq >= kSigma1 && tq <= kSigma2 * t) ? tq : 0.5 * t;
    }
    // x += t d, r += t Ad, g = A^T r, f = 1/2 ||r||^2
    hipLaunchKernelGGL(spg_vec_kernel<OP_AXPY>, dim3(W.gvec), dim3(kBlock), 0, s, n, t, nullptr,
                       W.d, x, W.partials);
    hipLaunchKernelGGL(spg_vec_kernel<OP_AXPY>, dim3(W.gvec), dim3(kBlock), 0, s, m, t, nullptr,
                       W.Ad, W.r, W.partials);
    gemv_t(W.r, W.g);
    if ((e = objective()) != CQK_OK) return e;
    hist.push_back(fx);
    // spectral step: s's / s'y = d'd / ||Ad||^2
    lam = (c2 <= 0.0) ? kLMax : std::min(kLMax, std::max(kLMin, dd / c2));
    it += 1;
    if ((e = proj_grad()) != CQK_OK) return e;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->iterations = it;
    info->projections = nproj;
    info->newton_iterations = newton;
    info->objective = fx;
    info->pg = pg;
    info->proj_ms = proj_ms;
    info->total_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
  }
  return CQK_OK;
}

}  // namespace cqk
