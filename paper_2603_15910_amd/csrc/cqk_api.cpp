// extern "C" entry points of libcqk: argument checks, context and workspace
// management, dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/cqk.h"
#include "cqk_internal.h"

namespace cqk {

cqk_status hip_ok(hipError_t e) { return e == hipSuccess ? CQK_OK : CQK_DEVICE_ERROR; }

// Every entry point that takes a cqk_info reports its return value in
// info->status too, also when it returns before reaching the solver.
cqk_status stamped(cqk_info* info, cqk_status st) {
  if (info && st != CQK_OK) info->status = st;
  return st;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e == hipErrorStreamCaptureImplicit) {
    // the legacy null stream while another stream captures
    (void)hipGetLastError();
    return true;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

cqk_status ensure_buffer(cqk_ctx* ctx, DeviceBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.ptr) return CQK_OK;
  // no allocation (or free) while a graph is being captured
  if (stream_capturing(ctx->stream)) return CQK_NO_MEMORY;
  if (b.ptr) {
    if (hipFree(b.ptr) != hipSuccess) return CQK_DEVICE_ERROR;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes < 4096 ? 4096 : bytes;
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return CQK_NO_MEMORY;
  }
  b.ptr = p;
  b.bytes = want;
  return CQK_OK;
}

cqk_status ensure_events(cqk_ctx* ctx, size_t count) {
  while (ctx->events.size() < count) {
    hipEvent_t e;
    // timing only (read after the stream is synchronised): no system-scope
    // fence, which would write back the L2 caches between the kernels timed
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
      return CQK_DEVICE_ERROR;
    ctx->events.push_back(e);
  }
  return CQK_OK;
}

void fill_default_opts(cqk_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->lambda0_mode = CQK_LAMBDA0_ZERO;
  o->lambda0_user = 0.0;
  o->max_iter = 100;
  o->tol = 0.0;
  o->compaction = CQK_COMPACT_AUTO;
  o->compact_theta = 0.0;
  o->accum = CQK_ACCUM_DEFAULT;
  o->sync = 1;
  o->trace = 0;
  o->timing = 0;
}

}  // namespace cqk

using namespace cqk;

namespace {

cqk_status check_opts(const cqk_opts* in, cqk_opts* out, bool simplex) {
  if (in) {
    *out = *in;
  } else {
    fill_default_opts(out);
    if (simplex) out->lambda0_mode = CQK_LAMBDA0_CONDAT;
  }
  if (out->max_iter <= 0 || out->max_iter > 200) return CQK_INVALID_ARG;
  if (out->lambda0_mode < 0 || out->lambda0_mode > 3) return CQK_INVALID_ARG;
  if (!simplex && out->lambda0_mode == CQK_LAMBDA0_CONDAT) return CQK_INVALID_ARG;
  if (out->lambda0_mode == CQK_LAMBDA0_USER && !std::isfinite(out->lambda0_user))
    return CQK_INVALID_ARG;
  if (out->compaction < 0 || out->compaction > 2) return CQK_INVALID_ARG;
  if (!(out->compact_theta <= 1.0) || std::isnan(out->tol)) return CQK_INVALID_ARG;
  if (out->accum < 0 || out->accum > 2) return CQK_INVALID_ARG;
  return CQK_OK;
}

// true if the n-element arrays at p and q share any byte
template <typename T>
bool overlaps(const T* p, const T* q, int64_t n) {
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q, len = (uintptr_t)n * sizeof(T);
  return a < b + len && b < a + len;
}

// true if [p, p + pb) and [q, q + qb) share any byte
bool overlaps_bytes(const void* p, size_t pb, const void* q, size_t qb) {
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
  return pb > 0 && qb > 0 && a < b + qb && b < a + pb;
}

void info_trivial(cqk_info* info, int status, double lam) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->status = status;
  info->lambda = lam;
  info->stop_reason = 5;
}

// A call answered on the host (empty input): its info is also what
// cqk_ctx_last_info reports for it.
void last_trivial(cqk_ctx* ctx, cqk_info* info, int status, double lam) {
  info_trivial(&ctx->trivial, status, lam);
  if (info) *info = ctx->trivial;
  // one captured pointer: std::function keeps it without a heap allocation
  ctx->last = [ctx](cqk_info* out) {
    *out = ctx->trivial;
    return CQK_OK;
  };
}

template <typename T>
cqk_status solve_common(cqk_ctx* ctx, int64_t n, const T* d, const T* a, const T* b, const T* l,
                        const T* u, const T* xw, bool warm, double r, T* x, const cqk_opts* opts,
                        cqk_info* info) {
  if (!ctx || n < 0 || !std::isfinite(r)) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, false);
  if (st != CQK_OK) return st;
  if (n == 0) {
    const int s = (r == 0.0) ? CQK_OK : CQK_INFEASIBLE;
    last_trivial(ctx, info, s, 0.0);
    return (cqk_status)s;
  }
  if (!d || !a || !b || !l || !u || !x) return CQK_INVALID_ARG;
  if (warm && (!xw || overlaps(xw, (const T*)x, n))) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  cqk_info tmp;
  cqk_info* inf = info ? info : &tmp;
  if constexpr (sizeof(T) == 8)
    st = run_general_f64(ctx, n, d, a, b, l, u, xw, r, x, o, inf);
  else
    st = run_general_f32(ctx, n, d, a, b, l, u, xw, r, x, o, inf);
  if (st != CQK_OK) return st;
  return (cqk_status)inf->status;
}

template <typename T>
cqk_status simplex_common(cqk_ctx* ctx, int64_t n, const T* y, const T* xw, bool warm, double r,
                          T* x, bool l1, const cqk_opts* opts, cqk_info* info,
                          SparseOut* sp = nullptr) {
  if (!ctx || n < 0 || !std::isfinite(r) || r < 0.0) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, true);
  if (st != CQK_OK) return st;
  if (n == 0) {
    const int s = (r == 0.0 || l1) ? CQK_OK : CQK_INFEASIBLE;
    last_trivial(ctx, info, s, 0.0);
    if (sp) sp->nnz = 0;
    return (cqk_status)s;
  }
  if (!y || (!x && !sp)) return CQK_INVALID_ARG;
  if (warm && (!xw || (x && overlaps(xw, (const T*)x, n)))) return CQK_INVALID_ARG;
  if (sp) {
    // the support's size is decided on the host: sparse calls always wait
    if (!o.sync || stream_capturing(ctx->stream)) return CQK_INVALID_ARG;
    if (sp->cap < 0 || (sp->cap > 0 && (!sp->idx || !sp->val))) return CQK_INVALID_ARG;
    const size_t yb = (size_t)n * sizeof(T), ib = (size_t)sp->cap * 8, vb = (size_t)sp->cap * sizeof(T);
    if (overlaps_bytes(sp->idx, ib, y, yb) || overlaps_bytes(sp->val, vb, y, yb) ||
        overlaps_bytes(sp->idx, ib, sp->val, vb))
      return CQK_INVALID_ARG;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  cqk_info tmp;
  cqk_info* inf = info ? info : &tmp;
  if constexpr (sizeof(T) == 8)
    st = run_simplex_f64(ctx, n, y, xw, sp, r, x, l1, o, inf);
  else
    st = run_simplex_f32(ctx, n, y, xw, sp, r, x, l1, o, inf);
  if (st != CQK_OK) return st;
  return (cqk_status)inf->status;
}

template <typename T>
cqk_status sparse_common(cqk_ctx* ctx, int64_t n, const T* y, const T* xbar, double r,
                         int64_t cap, int64_t* idx, T* val, int64_t* nnz, bool l1,
                         const cqk_opts* opts, cqk_info* info) {
  SparseOut sp{idx, val, cap, 0};
  const cqk_status st =
      simplex_common<T>(ctx, n, y, xbar, xbar != nullptr, r, nullptr, l1, opts, info, &sp);
  if (nnz) *nnz = sp.nnz;
  return st;
}

constexpr double kThetaCands[CQK_THETA_CANDIDATES] = {0.2, 0.3, 0.4, 0.5, 0.6, 0.75, 1.0};

// Times solve_common at every candidate theta (median of `repeats` after a
// warm-up, host clock around the synchronised call) and keeps the fastest.
template <typename T>
cqk_status tune_theta(cqk_ctx* ctx, int64_t n, const T* d, const T* a, const T* b, const T* l,
                      const T* u, double r, T* x, const cqk_opts* opts, int32_t repeats,
                      double* best_theta, double* best_ms, double* times_ms) {
  if (!ctx || n <= 0 || repeats < 1 || repeats > 100) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, false);
  if (st != CQK_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // the tuner synchronises
  o.compaction = CQK_COMPACT_AUTO;
  o.sync = 1;
  o.trace = 0;
  o.timing = 0;
  double times[CQK_THETA_CANDIDATES];
  std::vector<double> runs((size_t)repeats);
  for (int c = 0; c < CQK_THETA_CANDIDATES; ++c) {
    o.compact_theta = kThetaCands[c];
    for (int k = -1; k < repeats; ++k) {
      const auto t0 = std::chrono::steady_clock::now();
      st = solve_common<T>(ctx, n, d, a, b, l, u, nullptr, false, r, x, &o, nullptr);
      const auto t1 = std::chrono::steady_clock::now();
      if (st != CQK_OK) return st;
      if (k >= 0) runs[(size_t)k] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    std::sort(runs.begin(), runs.end());
    times[c] = runs[(size_t)repeats / 2];
  }
  int best = 0;
  for (int c = 1; c < CQK_THETA_CANDIDATES; ++c)
    if (times[c] < times[best]) best = c;
  ctx->theta = kThetaCands[best];
  if (best_theta) *best_theta = kThetaCands[best];
  if (best_ms) *best_ms = times[best];
  if (times_ms)
    for (int c = 0; c < CQK_THETA_CANDIDATES; ++c) times_ms[c] = times[c];
  return CQK_OK;
}
}  // namespace

extern "C" {

cqk_status cqk_create(cqk_ctx** out, void* hip_stream) {
  if (!out) return CQK_INVALID_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CQK_DEVICE_ERROR;
  cqk_ctx* ctx = new (std::nothrow) cqk_ctx();
  if (!ctx) return CQK_NO_MEMORY;
  ctx->device = dev;
  ctx->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cus = prop.multiProcessorCount;
  // the no-allocation batched call's buffers on this device (looked up now,
  // while dev is current); a failed lookup only disables that call
  if (noalloc_scratch(dev, &ctx->scratch) != CQK_OK) ctx->scratch = nullptr;
  ctx->host_pinned_bytes = 64 * 1024;
  if (hipHostMalloc(&ctx->host_pinned, ctx->host_pinned_bytes, hipHostMallocDefault) !=
      hipSuccess) {
    delete ctx;
    return CQK_NO_MEMORY;
  }
  *out = ctx;
  return CQK_OK;
}

void cqk_destroy(cqk_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  else hipDeviceSynchronize();
  if (ctx->ws.ptr) hipFree(ctx->ws.ptr);
  if (ctx->state.ptr) hipFree(ctx->state.ptr);
  if (ctx->bitmap.ptr) hipFree(ctx->bitmap.ptr);
  if (ctx->spg.ptr) hipFree(ctx->spg.ptr);
  if (ctx->host_pinned) hipHostFree(ctx->host_pinned);
  for (hipEvent_t e : ctx->events) hipEventDestroy(e);
  delete ctx;
}

cqk_status cqk_set_stream(cqk_ctx* ctx, void* hip_stream) {
  if (!ctx) return CQK_INVALID_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return CQK_OK;
}

cqk_status cqk_reserve(cqk_ctx* ctx, int64_t max_n, int32_t max_seg) {
  if (!ctx || max_n < 0 || max_seg < 0) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  // compaction buffers dominate: three sets of 4 doubles per index at the
  // largest theta (COMPACT_ALWAYS; the general solver's exact layout,
  // padding included), plus slack for the other paths' partial records
  const size_t gen = std::max(gen_layout(max_n, ctx->num_cus, 2, true, 1.0).bytes,
                              gen_layout(max_n, ctx->num_cus, 4, true, 1.0).bytes);
  const size_t want = std::max(gen, (size_t)max_n * 64) + (size_t)max_seg * 64 + (4u << 20);
  cqk_status st = ensure_buffer(ctx, ctx->ws, want);
  if (st != CQK_OK) return st;
  return ensure_buffer(ctx, ctx->state, 1024 + sizeof(cqk_trace_rec) * kMaxTrace);
}

const char* cqk_status_string(int32_t s) {
  switch (s) {
    case CQK_OK: return "CQK_OK";
    case CQK_INFEASIBLE: return "CQK_INFEASIBLE";
    case CQK_INVALID_ARG: return "CQK_INVALID_ARG";
    case CQK_NOT_CONVERGED: return "CQK_NOT_CONVERGED";
    case CQK_DEVICE_ERROR: return "CQK_DEVICE_ERROR";
    case CQK_NO_MEMORY: return "CQK_NO_MEMORY";
    case CQK_BUFFER_TOO_SMALL: return "CQK_BUFFER_TOO_SMALL";
    default: return "CQK_UNKNOWN_STATUS";
  }
}

void cqk_default_opts(cqk_opts* opts) {
  if (opts) fill_default_opts(opts);
}

cqk_status cqk_ctx_last_info(cqk_ctx* ctx, cqk_info* info) {
  if (!ctx || !info) return CQK_INVALID_ARG;
  if (!ctx->last) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  // waiting is not possible while the stream captures a graph
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;
  if (hip_ok(hipStreamSynchronize(ctx->stream)) != CQK_OK) return CQK_DEVICE_ERROR;
  const cqk_status st = ctx->last(info);
  if (st != CQK_OK) return st;
  return (cqk_status)info->status;
}

cqk_status cqk_last_trace(cqk_ctx* ctx, cqk_trace_rec* out, int32_t cap, int32_t* count) {
  if (!ctx || cap < 0 || (cap > 0 && !out)) return CQK_INVALID_ARG;
  const int32_t have = (int32_t)ctx->last_trace.size();
  const int32_t k = cap < have ? cap : have;
  for (int32_t i = 0; i < k; ++i) out[i] = ctx->last_trace[i];
  if (count) *count = have;
  return CQK_OK;
}

cqk_status cqk_last_pass_ms(cqk_ctx* ctx, float* ms, int32_t cap, int32_t* count) {
  if (!ctx || cap < 0 || (cap > 0 && !ms)) return CQK_INVALID_ARG;
  const int32_t have = (int32_t)ctx->last_pass_ms.size();
  const int32_t k = cap < have ? cap : have;
  for (int32_t i = 0; i < k; ++i) ms[i] = ctx->last_pass_ms[i];
  if (count) *count = have;
  return CQK_OK;
}

cqk_status cqk_solve_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                         const double* b, const double* l, const double* u, double r, double* x,
                         const cqk_opts* opts, cqk_info* info) {
  return stamped(info, solve_common<double>(ctx,
                         n, d, a, b, l, u, nullptr, false, r, x, opts, info));
}

cqk_status cqk_solve_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                         const float* b, const float* l, const float* u, double r, float* x,
                         const cqk_opts* opts, cqk_info* info) {
  return stamped(info, solve_common<float>(ctx,
                         n, d, a, b, l, u, nullptr, false, r, x, opts, info));
}

cqk_status cqk_project_simplex_f32(cqk_ctx* ctx, int64_t n, const float* y, double r, float* x,
                                   const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<float>(ctx, n, y, nullptr, false, r, x, false, opts, info));
}

cqk_status cqk_project_simplex_f64(cqk_ctx* ctx, int64_t n, const double* y, double r,
                                   double* x, const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<double>(ctx, n, y, nullptr, false, r, x, false, opts, info));
}

cqk_status cqk_project_l1_f32(cqk_ctx* ctx, int64_t n, const float* y, double radius, float* x,
                              const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<float>(ctx,
                         n, y, nullptr, false, radius, x, true, opts, info));
}

cqk_status cqk_project_l1_f64(cqk_ctx* ctx, int64_t n, const double* y, double radius,
                              double* x, const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<double>(ctx,
                         n, y, nullptr, false, radius, x, true, opts, info));
}

cqk_status cqk_solve_warm_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                              const double* b, const double* l, const double* u,
                              const double* xbar, double r, double* x, const cqk_opts* opts,
                              cqk_info* info) {
  return stamped(info, solve_common<double>(ctx, n, d, a, b, l, u, xbar, true, r, x, opts, info));
}

cqk_status cqk_solve_warm_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                              const float* b, const float* l, const float* u, const float* xbar,
                              double r, float* x, const cqk_opts* opts, cqk_info* info) {
  return stamped(info, solve_common<float>(ctx, n, d, a, b, l, u, xbar, true, r, x, opts, info));
}

cqk_status cqk_project_simplex_warm_f32(cqk_ctx* ctx, int64_t n, const float* y,
                                        const float* xbar, double r, float* x,
                                        const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<float>(ctx, n, y, xbar, true, r, x, false, opts, info));
}

cqk_status cqk_project_simplex_warm_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                        const double* xbar, double r, double* x,
                                        const cqk_opts* opts, cqk_info* info) {
  return stamped(info, simplex_common<double>(ctx, n, y, xbar, true, r, x, false, opts, info));
}

cqk_status cqk_project_l1_warm_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xbar,
                                   double radius, float* x, const cqk_opts* opts,
                                   cqk_info* info) {
  return stamped(info, simplex_common<float>(ctx, n, y, xbar, true, radius, x, true, opts, info));
}

cqk_status cqk_project_l1_warm_f64(cqk_ctx* ctx, int64_t n, const double* y, const double* xbar,
                                   double radius, double* x, const cqk_opts* opts,
                                   cqk_info* info) {
  return stamped(info, simplex_common<double>(ctx, n, y, xbar, true, radius, x, true, opts, info));
}

cqk_status cqk_project_simplex_sparse_f32(cqk_ctx* ctx, int64_t n, const float* y,
                                          const float* xbar, double r, int64_t cap,
                                          int64_t* idx, float* val, int64_t* nnz,
                                          const cqk_opts* opts, cqk_info* info) {
  return stamped(info, sparse_common<float>(ctx,
                         n, y, xbar, r, cap, idx, val, nnz, false, opts, info));
}

cqk_status cqk_project_simplex_sparse_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                          const double* xbar, double r, int64_t cap,
                                          int64_t* idx, double* val, int64_t* nnz,
                                          const cqk_opts* opts, cqk_info* info) {
  return stamped(info, sparse_common<double>(ctx,
                         n, y, xbar, r, cap, idx, val, nnz, false, opts, info));
}

cqk_status cqk_project_l1_sparse_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xbar,
                                     double radius, int64_t cap, int64_t* idx, float* val,
                                     int64_t* nnz, const cqk_opts* opts, cqk_info* info) {
  return stamped(info, sparse_common<float>(ctx,
                         n, y, xbar, radius, cap, idx, val, nnz, true, opts, info));
}

cqk_status cqk_project_l1_sparse_f64(cqk_ctx* ctx, int64_t n, const double* y,
                                     const double* xbar, double radius, int64_t cap,
                                     int64_t* idx, double* val, int64_t* nnz,
                                     const cqk_opts* opts, cqk_info* info) {
  return stamped(info, sparse_common<double>(ctx,
                         n, y, xbar, radius, cap, idx, val, nnz, true, opts, info));
}

}  // extern "C"

namespace {

template <typename T>
cqk_status batched_cqk_common(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const T* d,
                              const T* a, const T* b, const T* l, const T* u, const double* r,
                              T* x, double* lambda_out, int32_t* status_out,
                              const cqk_opts* opts, cqk_info* info) {
  if (!ctx || nseg < 0) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, false);
  if (st != CQK_OK) return st;
  if (nseg == 0) {
    last_trivial(ctx, info, CQK_OK, 0.0);
    return CQK_OK;
  }
  if (!offsets || !d || !a || !b || !l || !u || !r || !x) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  cqk_info tmp;
  cqk_info* inf = info ? info : &tmp;
  if constexpr (sizeof(T) == 8)
    st = run_batched_cqk_f64(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out, status_out, o,
                             inf);
  else
    st = run_batched_cqk_f32(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out, status_out, o,
                             inf);
  if (st != CQK_OK) return st;
  return (cqk_status)inf->status;
}

template <typename T>
cqk_status batched_cqk_backward_common(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                       const T* x, const T* g, const T* d, const T* b,
                                       const T* l, const T* u, T* grad_a, double* grad_r,
                                       const cqk_opts* opts) {
  if (!ctx || nseg < 0) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, false);
  if (st != CQK_OK) return st;
  if (nseg == 0) {
    ctx->last = ok_info;
    return CQK_OK;
  }
  if (!offsets || !x || !g || !d || !b || !l || !u || !grad_a) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if constexpr (sizeof(T) == 8)
    return run_batched_cqk_backward_f64(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r, o);
  else
    return run_batched_cqk_backward_f32(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r, o);
}

}  // namespace

extern "C" {

cqk_status cqk_solve_batched_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                 const double* d, const double* a, const double* b,
                                 const double* l, const double* u, const double* r, double* x,
                                 double* lambda_out, int32_t* status_out, const cqk_opts* opts,
                                 cqk_info* info) {
  return stamped(info, batched_cqk_common<double>(ctx, nseg, offsets, d, a, b, l, u, r, x,
                                               lambda_out, status_out, opts, info));
}

cqk_status cqk_solve_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                 const float* d, const float* a, const float* b, const float* l,
                                 const float* u, const double* r, float* x, double* lambda_out,
                                 int32_t* status_out, const cqk_opts* opts, cqk_info* info) {
  return stamped(info, batched_cqk_common<float>(ctx, nseg, offsets, d, a, b, l, u, r, x,
                                               lambda_out, status_out, opts, info));
}

cqk_status cqk_solve_batched_backward_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                          const double* x, const double* g, const double* d,
                                          const double* b, const double* l, const double* u,
                                          double* grad_a, double* grad_r, const cqk_opts* opts) {
  return batched_cqk_backward_common<double>(ctx, nseg, offsets, x, g, d, b, l, u, grad_a,
                                             grad_r, opts);
}

cqk_status cqk_solve_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                          const float* x, const float* g, const float* d,
                                          const float* b, const float* l, const float* u,
                                          float* grad_a, double* grad_r, const cqk_opts* opts) {
  return batched_cqk_backward_common<float>(ctx, nseg, offsets, x, g, d, b, l, u, grad_a,
                                            grad_r, opts);
}

void cqk_spg_default_opts(cqk_spg_opts* opts) {
  if (opts) fill_default_spg_opts(opts);
}

cqk_status cqk_spg_l1_lasso_f64(cqk_ctx* ctx, int64_t m, int64_t n, const double* A,
                                const double* b, double radius, double* x,
                                const cqk_spg_opts* opts, cqk_spg_info* info) {
  if (!ctx || m <= 0 || n <= 0 || !A || !b || !x) return CQK_INVALID_ARG;
  if (!std::isfinite(radius) || radius < 0.0 || n > (int64_t)UINT32_MAX) return CQK_INVALID_ARG;
  cqk_spg_opts o;
  if (opts) o = *opts;
  else fill_default_spg_opts(&o);
  if (!(o.tol >= 0.0) || o.max_iter < 0 || o.memory < 1 || (o.warm != 0 && o.warm != 1))
    return CQK_INVALID_ARG;
  // x is written while A, b are read: no overlap
  if (overlaps_bytes(x, (size_t)n * 8, A, (size_t)m * n * 8) ||
      overlaps_bytes(x, (size_t)n * 8, b, (size_t)m * 8))
    return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // SPG is driven by the host
  cqk_spg_info tmp;
  cqk_spg_info* inf = info ? info : &tmp;
  const cqk_status st = run_spg_l1_lasso_f64(ctx, m, n, A, b, radius, x, o, inf);
  ctx->last = nullptr;  // the SPG result is in *info only
  if (st != CQK_OK) return st;
  return (cqk_status)inf->status;
}

cqk_status cqk_project_simplex_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                           const float* y, const double* r, double r_scalar,
                                           float* x, double* lambda_out, int32_t* nfree_out,
                                           const cqk_opts* opts, cqk_info* info) {
  if (!ctx || nseg < 0) return stamped(info, CQK_INVALID_ARG);
  if (!r && (!std::isfinite(r_scalar) || r_scalar < 0.0)) return stamped(info, CQK_INVALID_ARG);
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, true);
  if (st != CQK_OK) return stamped(info, st);
  if (nseg == 0) {
    last_trivial(ctx, info, CQK_OK, 0.0);
    return CQK_OK;
  }
  if (!offsets || !y || !x) return stamped(info, CQK_INVALID_ARG);
  if (hipSetDevice(ctx->device) != hipSuccess) return stamped(info, CQK_DEVICE_ERROR);
  ctx->last = nullptr;
  cqk_info tmp;
  cqk_info* inf = info ? info : &tmp;
  st = run_batched_f32(ctx, nseg, offsets, y, r, r_scalar, x, lambda_out, nfree_out, o, inf);
  if (st != CQK_OK) return stamped(info, st);
  return stamped(info, (cqk_status)inf->status);
}

cqk_status cqk_project_simplex_batched_noalloc_f32(cqk_ctx* ctx, int32_t nseg,
                                                   const int64_t* offsets, const float* y,
                                                   const double* r, double r_scalar, float* x,
                                                   double* lambda_out, int32_t* nfree_out,
                                                   const cqk_opts* opts, cqk_info* info) {
  if (!ctx || nseg < 0) return stamped(info, CQK_INVALID_ARG);
  if (!r && (!std::isfinite(r_scalar) || r_scalar < 0.0)) return stamped(info, CQK_INVALID_ARG);
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, true);
  if (st != CQK_OK) return stamped(info, st);
  if (nseg > CQK_NOALLOC_MAX_SEG) return stamped(info, CQK_BUFFER_TOO_SMALL);
  if (nseg == 0) {
    last_trivial(ctx, info, CQK_OK, 0.0);
    return CQK_OK;
  }
  if (!offsets || !y || !x) return stamped(info, CQK_INVALID_ARG);
  if (hipSetDevice(ctx->device) != hipSuccess) return stamped(info, CQK_DEVICE_ERROR);
  ctx->last = nullptr;
  cqk_info tmp;
  cqk_info* inf = info ? info : &tmp;
  st = run_batched_noalloc_f32(ctx, nseg, offsets, y, r, r_scalar, x, lambda_out, nfree_out, o,
                               inf);
  if (st != CQK_OK) return stamped(info, st);
  return stamped(info, (cqk_status)inf->status);
}

cqk_status cqk_project_simplex_batched_backward_f32(cqk_ctx* ctx, int32_t nseg,
                                                    const int64_t* offsets, const float* x,
                                                    const float* g, float* grad_y,
                                                    double* grad_r, const cqk_opts* opts) {
  if (!ctx || nseg < 0) return CQK_INVALID_ARG;
  cqk_opts o;
  cqk_status st = check_opts(opts, &o, true);
  if (st != CQK_OK) return st;
  if (nseg == 0) {
    ctx->last = ok_info;
    return CQK_OK;
  }
  if (!offsets || !x || !g || !grad_y) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  return run_batched_backward_f32(ctx, nseg, offsets, x, g, grad_y, grad_r, o);
}

namespace {
// which: 0/1 batched simplex forward/backward, 2/3 batched general forward/backward
cqk_batch_schedule* schedule_slot(cqk_ctx* ctx, int32_t which) {
  switch (which) {
    case 0: return &ctx->sched_fwd;
    case 1: return &ctx->sched_bwd;
    case 2: return &ctx->sched_cqk_fwd;
    case 3: return &ctx->sched_cqk_bwd;
    default: return nullptr;
  }
}
}  // namespace

cqk_status cqk_get_batch_schedule(cqk_ctx* ctx, int32_t which, cqk_batch_schedule* out) {
  if (!ctx || !out) return CQK_INVALID_ARG;
  cqk_batch_schedule* slot = schedule_slot(ctx, which);
  if (!slot) return CQK_INVALID_ARG;
  *out = *slot;
  return CQK_OK;
}

cqk_status cqk_set_batch_schedule(cqk_ctx* ctx, int32_t which, const cqk_batch_schedule* sched) {
  if (!ctx || !sched) return CQK_INVALID_ARG;
  cqk_batch_schedule* slot = schedule_slot(ctx, which);
  if (!slot || !valid_schedule(*sched)) return CQK_INVALID_ARG;
  *slot = *sched;
  return CQK_OK;
}

cqk_status cqk_tune_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const double* d, const double* a, const double* b,
                                    const double* l, const double* u, const double* r,
                                    double* x, const double* g, double* grad_a,
                                    int32_t backward, int32_t repeats, cqk_batch_schedule* best,
                                    double* best_ms) {
  if (!ctx || nseg <= 0 || repeats < 1 || repeats > 100) return CQK_INVALID_ARG;
  if (backward != 0 && backward != 1) return CQK_INVALID_ARG;
  if (!offsets || !d || !b || !l || !u || !x) return CQK_INVALID_ARG;
  if (backward ? (!g || !grad_a) : (!a || !r)) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // the tuner synchronises
  return tune_batched_cqk_f64(ctx, nseg, offsets, d, a, b, l, u, r, x, g, grad_a, backward,
                              repeats, best, best_ms);
}

cqk_status cqk_tune_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const float* d, const float* a, const float* b,
                                    const float* l, const float* u, const double* r, float* x,
                                    const float* g, float* grad_a, int32_t backward,
                                    int32_t repeats, cqk_batch_schedule* best,
                                    double* best_ms) {
  if (!ctx || nseg <= 0 || repeats < 1 || repeats > 100) return CQK_INVALID_ARG;
  if (backward != 0 && backward != 1) return CQK_INVALID_ARG;
  if (!offsets || !d || !b || !l || !u || !x) return CQK_INVALID_ARG;
  if (backward ? (!g || !grad_a) : (!a || !r)) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // the tuner synchronises
  return tune_batched_cqk_f32(ctx, nseg, offsets, d, a, b, l, u, r, x, g, grad_a, backward,
                              repeats, best, best_ms);
}

cqk_status cqk_tune_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const float* y, const double* r, double r_scalar, float* x,
                                int32_t repeats, cqk_batch_schedule* best, double* best_ms) {
  if (!ctx || nseg <= 0 || repeats < 1 || repeats > 100) return CQK_INVALID_ARG;
  if (!offsets || !y || !x) return CQK_INVALID_ARG;
  if (!r && (!std::isfinite(r_scalar) || r_scalar < 0.0)) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // the tuner synchronises
  return tune_batched_f32(ctx, nseg, offsets, y, r, r_scalar, x, repeats, best, best_ms);
}

cqk_status cqk_tune_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                         const float* x, const float* g, float* grad_y,
                                         int32_t repeats, cqk_batch_schedule* best,
                                         double* best_ms) {
  if (!ctx || nseg <= 0 || repeats < 1 || repeats > 100) return CQK_INVALID_ARG;
  if (!offsets || !x || !g || !grad_y) return CQK_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return CQK_DEVICE_ERROR;
  ctx->last = nullptr;
  if (stream_capturing(ctx->stream)) return CQK_INVALID_ARG;  // the tuner synchronises
  return tune_batched_backward_f32(ctx, nseg, offsets, x, g, grad_y, repeats, best, best_ms);
}

cqk_status cqk_get_compact_theta(cqk_ctx* ctx, double* theta) {
  if (!ctx || !theta) return CQK_INVALID_ARG;
  *theta = ctx->theta;
  return CQK_OK;
}

cqk_status cqk_set_compact_theta(cqk_ctx* ctx, double theta) {
  if (!ctx || !(theta > 0.0 && theta <= 1.0)) return CQK_INVALID_ARG;
  ctx->theta = theta;
  return CQK_OK;
}

cqk_status cqk_tune_theta_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                              const double* b, const double* l, const double* u, double r,
                              double* x, const cqk_opts* opts, int32_t repeats,
                              double* best_theta, double* best_ms, double* times_ms) {
  return tune_theta<double>(ctx, n, d, a, b, l, u, r, x, opts, repeats, best_theta, best_ms,
                            times_ms);
}

cqk_status cqk_tune_theta_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                              const float* b, const float* l, const float* u, double r,
                              float* x, const cqk_opts* opts, int32_t repeats,
                              double* best_theta, double* best_ms, double* times_ms) {
  return tune_theta<float>(ctx, n, d, a, b, l, u, r, x, opts, repeats, best_theta, best_ms,
                           times_ms);
}

}  // extern "C"
