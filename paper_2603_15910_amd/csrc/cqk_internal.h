// Host-side internals of libcqk: the context, device state records and the
// kernel launchers each translation unit provides.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "../../include/cqk.h"

namespace cqk {

constexpr int kMaxTrace = 512;
constexpr int kMaxDevices = 64;

// Launches a kernel on stream s.  With a pair of events the dispatch itself
// stamps its start and end into them, so no marker packet sits between two
// kernels (an event recorded on the stream would add a few microseconds of
// idle time around every timed kernel).
template <typename F, typename... Args>
inline void launch_timed(F kern, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, Args... args) {
  if (e0 != nullptr) {
    hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, args...);
  } else {
    hipLaunchKernelGGL(kern, grid, block, 0, s, args...);
  }
}

// Run state of the general (Algorithm 1) solver, one record in device memory.
struct GenState {
  double lam, lam_prev, lo, hi, phi_lo, phi_hi;
  double F, AF, C0, C1, A0, A1;   // contributions of indices dropped from the pass
  double lam_final, lam0;
  double r, tol, theta;
  double res_P, res_A;            // finalize: b^T x and sum |b x|
  double bytes;                   // algorithmic bytes of the grid passes so far
  double in_bytes;                // bytes per index of the caller's arrays
  // The dropped-index sums of the current source hold for lam in [vlo, vhi]
  // (the caller's arrays: everywhere); a pass at a multiplier outside it
  // reads the caller's arrays again.
  double vlo, vhi;
  // Bracket [sp, sq] estimated from a sample of the indices, and the share of
  // indices the first pass may keep for it (sp < sq only when in use); the
  // dropped-index sums and size of the set the first pass wrote for it,
  // while that set waits in set 3 for an iterate inside (spend = 1)
  double sp, sq, scap;
  double sF, sAF, sC0, sC1, sA0, sA1;
  int64_t sn;
  // the first estimate (solution, bracket half-width, share of the sample
  // inside), refined by the second
  double s1lam, s1half, s1share;
  // the sample's estimate of lam* and its standard deviation (NaN: none)
  double slam, ssd;
  // Algorithm 1's first iterate as the sample predicts it, when it lies
  // outside the bracket (NaN otherwise): the third estimate predicts the
  // second iterate from it
  double s2lam1;
  int64_t n_src;                  // indices in the current source
  int64_t n_all;                  // indices of the caller's arrays
  int64_t n_free;                 // finalize: free indices
  int32_t status, iter, passes, mode, src, stop_reason, max_iter;
  int32_t compaction, trace_cap, ntrace, nblocks;
  uint32_t ticket;
  int32_t spec;                   // 1: the next evaluation writes the sampled-bracket set
  int32_t spend;                  // 1: that set waits in set 3
  int32_t s1ok;                   // 1: the first estimate found a bracket
  int32_t skip;                   // sides the next evaluation does not write (bit k: side k)
  int32_t warm;                   // 1: lam_0 comes from a primal estimate
  int32_t lam0_later;             // 1: lam_0 is computed after the sample (warm or formula start)
};

// Run state of the simplex / l1 solver (Algorithm 4 on a compacted set).
struct SpxState {
  double lam, lam_prev, lam0, lam_final, r, tol;
  double lo, hi, sum_abs, vmax;
  double res_P;                   // finalize: sum of x (l1: sum |x|)
  double cm_prev;
  int64_t n_src, n_init, n_free, tail_cap, chunk_src;
  int64_t nnz;                    // sparse output: entries of the support
  int32_t status, iter, passes, src, compact_next, stop_reason, max_iter;
  int32_t compaction, trace_cap, ntrace, l1, fin_mode, need_safeguard, first_done;
  int32_t tail;                   // 1: the remaining iterations run in one block
  int32_t multi;                  // 1: the next pass refines the start (candidates)
  int32_t x_zeroed;               // 1: the start already wrote x = 0 everywhere
  int32_t warm;                   // 1: a warm start (the start pass also reads xbar)
  int32_t sp_over;                // sparse output: the support exceeded the capacity
  int32_t pad_[1];
};

// Sparse output of a simplex / l1 projection: the support in ascending index
// order, as (index, value) pairs in caller memory of `cap` entries.
struct SparseOut {
  int64_t* idx;
  void* val;
  int64_t cap;
  int64_t nnz;   // set on return
};

// How the simplex finalize writes x.
enum FinMode : int32_t { kFinDense = 0, kFinScatter = 1, kFinCopy = 2, kFinZero = 3 };

enum RunStatus : int32_t { kRunning = -1 };

enum GenMode : int32_t { kModeEval = 0, kModeBreakRight = 1, kModeBreakLeft = 2 };

struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace cqk

struct cqk_ctx {
  int device = 0;
  int num_cus = 256;
  hipStream_t stream = nullptr;
  cqk::DeviceBuf ws;          // compaction buffers, partials, per-block counts
  cqk::DeviceBuf state;       // run-state records + trace ring
  cqk::DeviceBuf bitmap;      // sparse output: one bit per index, zero between calls
  cqk::DeviceBuf spg;         // the SPG driver's vectors
  bool bitmap_clean = false;  // the bitmap is known to be all zero
  void* host_pinned = nullptr;  // pinned mirror of the state + trace
  size_t host_pinned_bytes = 0;
  std::vector<hipEvent_t> events;
  int32_t last_trace_count = 0;
  std::vector<cqk_trace_rec> last_trace;
  std::vector<float> last_pass_ms;  // kernel time of each grid pass of the last timed call
  double theta = 0.5;  // compaction threshold of AUTO calls that give none
  cqk_batch_schedule sched_fwd{8, 4, 1, 16};  // batched forward / backward schedules
  cqk_batch_schedule sched_bwd{8, 4, 0, 0};
  cqk_batch_schedule sched_cqk_fwd{8, 4, 0, 0};  // batched general CQK forward / backward
  cqk_batch_schedule sched_cqk_bwd{8, 4, 0, 0};
  // Reads the device-side result of the last call into an info record (the
  // stream already synchronised); set by every call that got past its host
  // checks, so cqk_ctx_last_info can report a call queued with sync = 0 or
  // replayed from a captured graph.
  std::function<cqk_status(cqk_info*)> last;
  cqk_info trivial{};               // the last call answered on the host
  int32_t* bat_counters = nullptr;  // device counters of the last batched forward call
  bool bat_timing = false;          // that call recorded events[0..1]
  void* scratch = nullptr;  // this device's no-allocation planning buffers (noalloc_scratch)
};

namespace cqk {

// Grows b to at least `bytes`.  While ctx's stream is capturing a graph it
// allocates nothing: a buffer too small then gives CQK_NO_MEMORY.
cqk_status ensure_buffer(cqk_ctx* ctx, DeviceBuf& b, size_t bytes);
// true while stream s is capturing a graph
bool stream_capturing(hipStream_t s);
cqk_status hip_ok(hipError_t e);
// the device-side result of a call that always ends OK (the backward calls)
inline cqk_status ok_info(cqk_info* inf) {
  *inf = cqk_info{};
  inf->status = CQK_OK;
  return CQK_OK;
}
cqk_status ensure_events(cqk_ctx* ctx, size_t count);
void fill_default_opts(cqk_opts* o);

// Launchers (each returns CQK_OK or CQK_DEVICE_ERROR / CQK_NO_MEMORY).
// Grid and workspace of the general solver for n indices of `vec` values per
// 16-byte vector (2: FP64 inputs, 4: FP32 inputs).
struct GenLayout {
  int G, NR, GF;
  int64_t chunk, region;
  size_t part_bytes, cnt_bytes, smp_bytes, bytes;
};
// theta: the largest survivor fraction a compacted set may keep (1: any)
GenLayout gen_layout(int64_t n, int num_cus, int vec, bool compaction, double theta);

// xw: the primal estimate of a warm start, or null (opts.lambda0_mode then
// chooses the start)
cqk_status run_general_f64(cqk_ctx* ctx, int64_t n, const double* d, const double* a,
                           const double* b, const double* l, const double* u, const double* xw,
                           double r, double* x, const cqk_opts& o, cqk_info* info);
cqk_status run_general_f32(cqk_ctx* ctx, int64_t n, const float* d, const float* a,
                           const float* b, const float* l, const float* u, const float* xw,
                           double r, float* x, const cqk_opts& o, cqk_info* info);
// xw: warm-start estimate or null; sp: sparse output (x is then unused) or
// null
cqk_status run_simplex_f32(cqk_ctx* ctx, int64_t n, const float* y, const float* xw, SparseOut* sp,
                           double r, float* x, bool l1, const cqk_opts& o, cqk_info* info);
cqk_status run_simplex_f64(cqk_ctx* ctx, int64_t n, const double* y, const double* xw,
                           SparseOut* sp, double r, double* x, bool l1, const cqk_opts& o,
                           cqk_info* info);
// SPG on the l1-constrained least-squares problem (dense row-major A).
void fill_default_spg_opts(cqk_spg_opts* o);
cqk_status run_spg_l1_lasso_f64(cqk_ctx* ctx, int64_t m, int64_t n, const double* A,
                                const double* b, double radius, double* x,
                                const cqk_spg_opts& so, cqk_spg_info* info);
// Batched general CQK (FP64 rows) and its VJP w.r.t. a and r.
cqk_status run_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                               const double* d, const double* a, const double* b,
                               const double* l, const double* u, const double* r, double* x,
                               double* lambda_out, int32_t* status_out, const cqk_opts& o,
                               cqk_info* info);
cqk_status run_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                               const float* d, const float* a, const float* b, const float* l,
                               const float* u, const double* r, float* x, double* lambda_out,
                               int32_t* status_out, const cqk_opts& o, cqk_info* info);
cqk_status run_batched_cqk_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                        const float* x, const float* g, const float* d,
                                        const float* b, const float* l, const float* u,
                                        float* grad_a, double* grad_r, const cqk_opts& o);
cqk_status run_batched_cqk_backward_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                        const double* x, const double* g, const double* d,
                                        const double* b, const double* l, const double* u,
                                        double* grad_a, double* grad_r, const cqk_opts& o);
cqk_status tune_batched_cqk_f64(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const double* d, const double* a, const double* b,
                                const double* l, const double* u, const double* r, double* x,
                                const double* g, double* grad_a, int32_t backward,
                                int32_t repeats, cqk_batch_schedule* best, double* best_ms);
cqk_status tune_batched_cqk_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                const float* d, const float* a, const float* b, const float* l,
                                const float* u, const double* r, float* x, const float* g,
                                float* grad_a, int32_t backward, int32_t repeats,
                                cqk_batch_schedule* best, double* best_ms);
cqk_status run_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const float* y,
                           const double* r, double r_scalar, float* x, double* lambda_out,
                           int32_t* nfree_out, const cqk_opts& o, cqk_info* info);
cqk_status run_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                    const float* x, const float* g, float* grad_y,
                                    double* grad_r, const cqk_opts& o);
// The batched simplex projection on the fixed per-GPU planning buffers
// (no allocation): CQK_BUFFER_TOO_SMALL beyond CQK_NOALLOC_MAX_SEG rows.
cqk_status run_batched_noalloc_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                   const float* y, const double* r, double r_scalar, float* x,
                                   double* lambda_out, int32_t* nfree_out, const cqk_opts& o,
                                   cqk_info* info);
// Device address of those buffers on `device` (which must be current),
// looked up once per device.
cqk_status noalloc_scratch(int device, void** out);
bool valid_schedule(const cqk_batch_schedule& sc);
cqk_status tune_batched_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets, const float* y,
                            const double* r, double r_scalar, float* x, int32_t repeats,
                            cqk_batch_schedule* best, double* best_ms);
cqk_status tune_batched_backward_f32(cqk_ctx* ctx, int32_t nseg, const int64_t* offsets,
                                     const float* x, const float* g, float* grad_y,
                                     int32_t repeats, cqk_batch_schedule* best,
                                     double* best_ms);

}  // namespace cqk
