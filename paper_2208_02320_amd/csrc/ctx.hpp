// Context object and error plumbing shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/hh.h"

struct hh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, std::pair<void*, size_t>> bufs;
  std::vector<hipEvent_t> evpool;
  hipEvent_t t0 = nullptr, t1 = nullptr;  // call timing
  hipEvent_t e0 = nullptr, e1 = nullptr;  // autotuner timing
  hipStream_t cap = nullptr;              // stream used only to capture graphs
  int max_lds = 65536;                    // LDS bytes a workgroup may use
  // tuned tile variants (z, y, x) per (nx, ny, nz, precision, aniso, systems bucket)
  std::map<std::array<int, 6>, std::array<int, 3>> plans;
  // instantiated graphs of iteration chunks, keyed by their launch arguments
  std::map<std::string, hipGraphExec_t> graphs;
  double setup_ms = 0.0;                  // tuning and graph construction of the current call
  std::array<int, 3> last_plan{{0, 0, 0}};
};

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
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                       \
      throw Fail{e_ == hipErrorOutOfMemory ? HH_ENOMEM : HH_EDEVICE};                      \
    }                                                                                      \
  } while (0)

[[noreturn]] inline void fail(hh_ctx* ctx, int code, const std::string& msg) {
  ctx->err = msg;
  throw Fail{code};
}

inline void* ws(hh_ctx* ctx, const std::string& name, size_t bytes) {
  auto it = ctx->bufs.find(name);
  if (it != ctx->bufs.end() && it->second.second >= bytes) return it->second.first;
  if (it != ctx->bufs.end()) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
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
