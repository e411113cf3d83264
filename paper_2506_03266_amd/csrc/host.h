// host.h -- host-side helpers shared by the library's translation units:
// error reporting for the C ABI and optional per-kernel event timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "mpd.h"

namespace mpd {

// Message of the last failed call on this thread (returned by mpd_last_error).
extern thread_local std::string g_last_error;

// Records a printf-style message and returns `code`.
int fail_with(int code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail_with(MPD_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));       \
  } while (0)

// Optional per-kernel timing with HIP events on the launch stream.  Safe
// to use from several host threads (records are guarded by a mutex).
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::mutex mu;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    std::lock_guard<std::mutex> lk(mu);
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
extern Profiler g_prof;

// Records events around one launch when profiling is on.
struct ProfScope {
  ProfRec r{nullptr, nullptr, nullptr};
  hipStream_t st;
  ProfScope(const char *name, hipStream_t s) : st(s) {
    if (!g_prof.on) return;
    r.name = name;
    r.a = g_prof.get();
    r.b = g_prof.get();
    if (r.a) (void)hipEventRecord(r.a, st);
  }
  ~ProfScope() {
    if (!g_prof.on || !r.a || !r.b) return;
    (void)hipEventRecord(r.b, st);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.recs.push_back(r);
  }
};

// Compute units of the current device (cached per device).
int cu_count();

// floor(p 2^32) clamped to [0, 2^32]: the flip threshold of noise strength p.
uint64_t threshold_of(double p);

// Forward pass of the decode-time predictor (cnn.hip) on count maps
// [n][M][M]: pred [n], and optionally feat / argmax [n][16] and the stored
// activations of layers 1-3 (`store`, M <= 32 only).  `ws` holds
// cnn_forward_ws(M, n) bytes, 256-byte aligned.
size_t cnn_forward_ws(int M, int64_t n);
int cnn_forward_run(const uint8_t *counts, int M, int64_t n, const float *params, float *pred, float *feat,
                    int32_t *argmax, uint16_t *store, void *ws, hipStream_t stream);

}  // namespace mpd
