// Context object and error plumbing shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hh.h"

// A stream of work inside one call: its stream, its graph-capture stream,
// its timing events and the prefix of its workspace buffers.  The context's
// own lane has an empty prefix; a batch of several shapes runs its shape
// groups on extra lanes concurrently.
struct hh_lane {
  hipStream_t stream = nullptr, cap = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::string prefix;
};

struct hh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, std::pair<void*, size_t>> bufs;
  std::map<std::string, std::pair<void*, size_t>> host_bufs;  // pinned host staging (hipHostMalloc)
  std::vector<hipEvent_t> evpool;
  hipEvent_t t0 = nullptr, t1 = nullptr;  // call timing
  hipEvent_t e0 = nullptr, e1 = nullptr;  // autotuner timing
  hipStream_t cap = nullptr;              // stream used only to capture graphs
  int max_lds = 65536;                    // LDS bytes a workgroup may use
  // tuned tile variants (z, y, x) per (nx, ny, nz, precision, aniso, systems bucket)
  std::map<std::array<int, 6>, std::array<int, 3>> plans;
  std::string plan_file;  // tuned plans appended here and read by hh_plan_cache (empty: none)
  std::string arch;       // gcnArchName up to its feature list
  // instantiated graphs of iteration chunks, keyed by their launch arguments
  std::map<std::string, hipGraphExec_t> graphs;
  double setup_ms = 0.0;                  // tuning and graph construction of the current call
  // networks used by hh_hierarchical(use_surrogate = 1) (owned by the caller)
  struct hh_net* sur_a = nullptr;
  struct hh_net* sur_b = nullptr;
  double sur_spread = 0.0, sur_bound = 0.0;
  // While arena_base is set (the allocation-free entry point), ws() carves
  // its buffers from that preallocated region with a bump pointer reset per
  // call, and never allocates or frees device memory.
  char* arena_base = nullptr;
  size_t arena_size = 0, arena_used = 0;
  std::map<std::string, std::pair<void*, size_t>> arena_bufs;
  double call_bytes = 0.0;                // algorithmic bytes of the current call's solver passes
  long long call_retried = 0;             // images of the current call solved again in FP64
  std::array<int, 3> last_plan{{0, 0, 0}};
  // extra lanes of concurrent shape groups (created on first use, default priority)
  std::vector<hh_lane> aux;
  hipEvent_t fork = nullptr;
  // guards the maps, counters and message above when lanes run in threads
  std::recursive_mutex mu;
};

// Sets the context's error message (lanes may fail concurrently).
inline void set_err(hh_ctx* ctx, const std::string& msg) {
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  ctx->err = msg;
}

inline void clear_graphs(hh_ctx* ctx) {
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
  ctx->graphs.clear();
}


struct Fail {
  int code;
};

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_err(ctx, std::string(#expr) + ": " + hipGetErrorString(e_));                      \
      throw Fail{e_ == hipErrorOutOfMemory ? HH_ENOMEM : HH_EDEVICE};                      \
    }                                                                                      \
  } while (0)

[[noreturn]] inline void fail(hh_ctx* ctx, int code, const std::string& msg) {
  set_err(ctx, msg);
  throw Fail{code};
}

// Workspace buffer `name`, grown on demand; `st` is the stream whose work may
// still use the old buffer when it has to grow (default: the context's).
inline void* ws(hh_ctx* ctx, const std::string& name, size_t bytes, hipStream_t st) {
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  if (ctx->arena_base) {
    auto a = ctx->arena_bufs.find(name);
    if (a != ctx->arena_bufs.end() && a->second.second >= bytes) return a->second.first;
    const size_t sz = (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
    if (ctx->arena_used + sz > ctx->arena_size)
      fail(ctx, HH_ENOMEM, "the call needs more than the " + std::to_string(ctx->arena_size) +
                               " bytes of the library's static scratch (at buffer " + name + ")");
    void* p = ctx->arena_base + ctx->arena_used;
    ctx->arena_used += sz;
    ctx->arena_bufs[name] = {p, sz};
    return p;
  }
  auto it = ctx->bufs.find(name);
  if (it != ctx->bufs.end() && it->second.second >= bytes) return it->second.first;
  if (it != ctx->bufs.end()) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(it->second.first));
    ctx->bufs.erase(it);
  }
  void* p = nullptr;
  const size_t sz = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(ctx, HH_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes for " + name + " failed");
  }
  ctx->bufs[name] = {p, sz};
  return p;
}
inline void* ws(hh_ctx* ctx, const std::string& name, size_t bytes) { return ws(ctx, name, bytes, ctx->stream); }

// Pinned host buffer `name` for staging copies, grown on demand (after the
// context's stream has drained); freed with the context.
template <class T>
inline T* pinned(hh_ctx* ctx, const std::string& name, size_t count) {
  std::lock_guard<std::recursive_mutex> g(ctx->mu);
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  auto it = ctx->host_bufs.find(name);
  if (it != ctx->host_bufs.end() && it->second.second >= bytes) return static_cast<T*>(it->second.first);
  if (it != ctx->host_bufs.end()) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipHostFree(it->second.first));
    ctx->host_bufs.erase(it);
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    fail(ctx, HH_ENOMEM, "pinned host allocation of " + std::to_string(bytes) + " bytes for " + name + " failed");
  }
  ctx->host_bufs[name] = {p, bytes};
  return static_cast<T*>(p);
}


template <class F>
int guarded(hh_ctx* ctx, F&& f) {
  if (!ctx) return HH_EINVAL;
  ctx->err.clear();
  try {
    HIPCHK(hipSetDevice(ctx->device));
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return HH_EDEVICE;
  } catch (...) {
    ctx->err = "unknown error";
    return HH_EDEVICE;
  }
}
