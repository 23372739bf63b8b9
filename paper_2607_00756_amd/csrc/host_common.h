// Host-side helpers shared by the C-ABI entry points (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "bip_internal.h"

namespace bip {

inline int64_t roundup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

inline int err(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

#define HIPCHK(expr, what)                         \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

inline hipEvent_t take_event(bip_plan* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` on stream `st`; when profiling, bracket it with events.
template <typename F>
hipError_t timed(bip_plan* p, int stage, hipStream_t st, F&& launch) {
  if (!p->profiling) return launch();
  hipEvent_t a = take_event(p), b = take_event(p);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  p->timed.push_back({stage, a, b});
  return e;
}

// One device block from the caller's allocator, or stream-ordered from the
// HIP pool when there is none.
inline void* raw_alloc(const bip_alloc* al, size_t bytes, hipStream_t s) {
  if (al && al->alloc) return al->alloc(bytes, (void*)s, al->ctx);
  void* ptr = nullptr;
  if (hipMallocAsync(&ptr, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ptr;
}
inline void raw_release(const bip_alloc* al, void* ptr, size_t bytes, hipStream_t s) {
  if (!ptr) return;
  if (al && al->release) al->release(ptr, bytes, (void*)s, al->ctx);
  else (void)hipFreeAsync(ptr, s);
}

inline const bip_alloc* plan_alloc(const bip_plan* p) { return p->has_alloc ? &p->alloc : nullptr; }

// A block owned by the plan until bip_plan_destroy.
inline int plan_block(bip_plan* p, void** out, size_t bytes, hipStream_t s) {
  *out = raw_alloc(plan_alloc(p), bytes, s);
  if (!*out) return err(BIP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  p->allocations.push_back({*out, bytes});
  p->bytes_now += (int64_t)bytes;
  p->bytes_peak = std::max(p->bytes_peak, p->bytes_now);
  return BIP_OK;
}
inline void plan_release(bip_plan* p, void* ptr, hipStream_t s) {
  for (size_t i = 0; i < p->allocations.size(); ++i)
    if (p->allocations[i].ptr == ptr) {
      raw_release(plan_alloc(p), ptr, p->allocations[i].bytes, s);
      p->bytes_now -= (int64_t)p->allocations[i].bytes;
      p->allocations.erase(p->allocations.begin() + i);
      return;
    }
}

template <typename T>
int dalloc(bip_plan* p, T** out, size_t count, hipStream_t s) {
  *out = nullptr;
  if (count == 0) return BIP_OK;
  void* ptr = nullptr;
  int rc = plan_block(p, &ptr, count * sizeof(T), s);
  *out = (T*)ptr;
  return rc;
}

// Copy a host table into a new plan block.  The source must stay alive until
// the stream has passed the copy.
template <typename T>
int upload(bip_plan* p, T** out, const std::vector<T>& v, hipStream_t s) {
  int rc = dalloc(p, out, v.size(), s);
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  return BIP_OK;
}

struct Workspace {
  char* base = nullptr;
  size_t used = 0;
  void* take(size_t bytes) {
    void* p = base + used;
    used += roundup((int64_t)bytes, 256);
    return p;
  }
};

// Grow the plan's workspace to `bytes`.  The old block is released in stream
// order, so no synchronization is needed.
inline int ensure_work(bip_plan* p, size_t bytes, hipStream_t s) {
  if (p->work_bytes >= bytes) return BIP_OK;
  if (p->d_work) {
    plan_release(p, p->d_work, s);
    p->d_work = nullptr;
    p->work_bytes = 0;
  }
  void* ptr = nullptr;
  int rc = plan_block(p, &ptr, bytes, s);
  if (rc) return rc;
  p->d_work = ptr;
  p->work_bytes = bytes;
  return BIP_OK;
}

// Largest parent-column batch of a sweep: BIP_COLUMN_BATCH if set (0 = all
// columns), else as many as fit in kColumnBatchBytes of state (224 MiB: a
// batch and what the passes read besides stay inside the 256 MB Infinity
// Cache; 192, 256 and 384 MiB batches measured slower).
constexpr int64_t kColumnBatchBytes = (int64_t)224 << 20;
inline int column_batch(int64_t G) {
  const char* env = std::getenv("BIP_COLUMN_BATCH");
  int64_t b = env ? std::atoll(env) : kColumnBatchBytes / (G * 8);
  if (b <= 0) b = INT32_MAX;
  return (int)std::min<int64_t>(b, INT32_MAX);
}
// Split precision runs the Gram matrix on single FP16 products when its sum
// runs over at least this many detector beams: the FP16 rounding of the
// operand (2^-11) then averages to well under the 1e-4 target (measured
// 5e-6 at 32,417 beams); smaller detectors keep the hi+lo BF16 products.
constexpr int kGramFp16MinBeams = 4096;
inline int gram_precision(int precision, int ndet) {
  return precision == BIP_PREC_SPLIT_BF16 && ndet >= kGramFp16MinBeams ? BIP_PREC_FP16 : precision;
}

// The batch actually used for a sweep over n columns: the fewest batches of
// at most cap columns, of equal size (the last one at most a column short).
inline int balanced_batch(int n, int cap) {
  if (n <= 0) return 1;
  const int64_t nb = ((int64_t)n + cap - 1) / cap;
  return (int)((n + nb - 1) / nb);
}

// Job groups of the quadratic form.  Its workgroups hold a CU each (LDS), so
// qt tiles x z groups run in ceil(qt z / n_cu) rounds of ceil(nat / z) jobs
// per workgroup: take the z with the fewest job-rounds, the smallest on ties
// (fewer partial rows to reduce).
inline int quad_groups(int qt, int nat, int n_cu) {
  int best = 1;
  int64_t cost = INT64_MAX;
  for (int z = 1; z <= std::min(GEMM_MAX_ZSPLIT, nat); ++z) {
    const int64_t c = ((int64_t)qt * z + n_cu - 1) / n_cu * ((nat + z - 1) / z);
    if (c < cost) {
      cost = c;
      best = z;
    }
  }
  return best;
}

inline GatherArgs gather_args(const bip_plan* p, int side) {
  GatherArgs g;
  g.rec = side == 1 ? p->d_grec1 : p->d_grec2;
  g.win = side == 1 ? p->d_win1 : p->d_win2;
  return g;
}

inline ReconArgs recon_args(const bip_plan* p, int a, int side) {
  ReconArgs r;
  r.win = (side == 1 ? p->d_win1 + p->off1[a] : p->d_win2 + p->off2[a]);
  r.rowptr = side == 1 ? p->d_rp1 : p->d_rp2;
  r.col = side == 1 ? p->d_col1 : p->d_col2;
  r.w = side == 1 ? p->d_w1 : p->d_w2;
  r.ellc = side == 1 ? p->d_ellc1 : p->d_ellc2;
  r.ellw = side == 1 ? p->d_ellw1 : p->d_ellw2;
  r.tstart = side == 1 ? p->d_tstart1 : p->d_tstart2;
  r.tpar = side == 1 ? p->d_tpar1 : p->d_tpar2;
  r.ell_loc = side == 1 ? p->d_eloc1 : p->d_eloc2;
  r.tile_np = side == 1 ? p->tile_np1 : p->tile_np2;
  r.scale = 1.f;
  r.beams = side == 1 ? p->d_beams : p->d_det;
  r.nb = side == 1 ? p->B : p->ndet;
  r.W = side == 1 ? p->W1[a] : p->W[a];  // S1: the enlarged window in focal mode
  r.oy = side == 1 ? p->oy1[a] : p->oy[a];
  r.ox = side == 1 ? p->ox1[a] : p->ox[a];
  r.ny = p->g.ny;
  r.nx = p->g.nx;
  r.tw = p->d_tw;
  r.L = p->L;
  r.retilt_sign = side == 1 ? +1 : -1;
  r.mode = p->o.recon_mode;
  return r;
}

}  // namespace bip
