// Host side of the C ABI declared in include/hh.h: validation, workspace,
// the per-group solve loop, and the two-level scheme.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/hh.h"
#include "cnn.hpp"
#include "ctx.hpp"
#include "hh_internal.hpp"
#include "kernels.hpp"

using namespace hh;

namespace {

// reason of the calling thread's last failed hh_create
thread_local std::string g_create_error;

// Device scratch of the allocation-free entry point: one static array per
// GPU the library runs on, held until the process ends.  Host code uses it
// only through the address hipGetSymbolAddress returns for each device
// (taken once per device by hh_create, with that device current).
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The address of this device's scratch (the device is current); HH_OK or HH_EDEVICE.
int init_scratch(int device, std::string& why) {
  if (device < 0 || device >= kMaxDevices) {
    why = "hh_create: device index beyond the scratch table";
    return HH_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return HH_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    why = std::string("hh_create: hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e);
    return HH_EDEVICE;
  }
  g_scratch_ptr[device] = ptr;
  return HH_OK;
}

int status_code(int s) {
  switch (s) {
    case kConverged: return HH_OK;
    case kNoConv: return HH_ENOCONV;
    case kStagnated: return HH_ESTAGNATED;
    case kBreakdown: return HH_EBREAKDOWN;
    case kNonFinite: return HH_EBREAKDOWN;
    case kSingularStatus: return HH_ESINGULAR;
    case kRunning: return HH_ENOCONV;
    default: return HH_EDEVICE;
  }
}

// Severity order used to report the worst status of several results.
int worse(int a, int b) {
  auto rank = [](int c) {
    switch (c) {
      case HH_OK: return 0;
      case HH_ENOCONV: return 1;
      case HH_ESTAGNATED: return 2;
      case HH_ESINGULAR: return 3;
      case HH_EBREAKDOWN: return 4;
      default: return 5;
    }
  };
  return rank(b) > rank(a) ? b : a;
}

struct Profile {
  hh_ctx* ctx;
  bool on;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> marks;
  size_t used = 0;
  hh_report* rep;
  hipEvent_t ev() {
    if (used >= ctx->evpool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ctx->evpool.push_back(e);
    }
    return ctx->evpool[used++];
  }
  template <class F>
  void run(int cls, F&& f) {
    if (!on) {
      f();
      return;
    }
    hipEvent_t a = ev(), b = ev();
    HIPCHK(hipEventRecord(a, ctx->stream));
    f();
    HIPCHK(hipEventRecord(b, ctx->stream));
    marks.emplace_back(cls, a, b);
  }
  // Called after a stream synchronisation: accumulate and recycle events.
  void flush() {
    if (!on) return;
    for (auto& m : marks) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, std::get<1>(m), std::get<2>(m)));
      if (rep) {
        rep->kernel_ms[std::get<0>(m)] += ms;
        rep->kernel_launches[std::get<0>(m)] += 1;
      }
    }
    marks.clear();
    used = 0;
  }
};

struct Item {
  int nx, ny, nz;
  long long lab_off;  // iso: byte offset into the label pack
  long long cf_off;   // aniso: element offset into the stiffness pack
  int region[6];
  std::vector<hh_phase> phases;
};

// Iteration limits of a group: the options' values, or (0) derived from
// the phase contrast kappa = largest / smallest eigenvalue of the phase
// stiffnesses (3K once and 2G five times per isotropic phase).  Conjugate
// gradients reduce the error by 2 ((sqrt(kappa) - 1) / (sqrt(kappa) + 1))^k
// after k steps, so about sqrt(kappa) ln(2 / tol) / 2 steps reach tol in
// exact arithmetic; the cap allows twice that.
struct Limits {
  int max_iter, stall;
};
Limits solve_limits(const hh_opts& o, const std::vector<Item>& items, bool aniso) {
  double kappa = 1.0;
  if (!aniso) {
    double hi = 0.0, lo = 1e300;
    for (const Item& it : items)
      for (const hh_phase& p : it.phases) {
        hi = std::max(hi, std::max(3.0 * p.K, 2.0 * p.G));
        lo = std::min(lo, std::min(3.0 * p.K, 2.0 * p.G));
      }
    if (lo > 0.0 && hi > 0.0) kappa = hi / lo;
  }
  const double s = std::sqrt(kappa);
  Limits l;
  if (o.max_iter > 0) {
    l.max_iter = o.max_iter;
  } else if (aniso) {
    l.max_iter = 1000;
  } else {
    l.max_iter = int(std::min(1e6, std::max(1000.0, std::ceil(s * std::log(2.0 / o.tol)))));
  }
  if (o.stall_limit > 0) l.stall = o.stall_limit;
  else l.stall = aniso ? 100 : int(std::min(1e6, std::max(100.0, std::ceil(s))));
  return l;
}

struct GroupResult {
  std::vector<double> C72;  // per item: raw (36) then symmetrized (36)
  std::vector<int> status;  // per item HH code
  std::vector<int> iters;   // per item x 6
  std::vector<double> rel;  // per item x 6
  double voxel_iters = 0.0;
};

void unit_loads(double L[6][6]) {
  for (int a = 0; a < 6; ++a)
    for (int c = 0; c < 6; ++c) L[a][c] = (a == c) ? (c < 3 ? 1.0 : 0.5) : 0.0;
}

void loads_from_voigt(const double* v, double L[6][6]) {
  for (int a = 0; a < 6; ++a)
    for (int c = 0; c < 6; ++c) L[a][c] = v[6 * a + c] * (c < 3 ? 1.0 : 0.5);
}

bool loads_independent(const double L[6][6]) {
  double A[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = L[i][j];
  double scale = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) scale = std::max(scale, std::fabs(A[i][j]));
  if (scale == 0.0) return false;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    if (std::fabs(A[piv][c]) <= 1e-12 * scale) return false;
    for (int j = 0; j < 6; ++j) std::swap(A[c][j], A[piv][j]);
    for (int r = c + 1; r < 6; ++r) {
      const double f = A[r][c] / A[c][c];
      for (int j = 0; j < 6; ++j) A[r][j] -= f * A[c][j];
    }
  }
  return true;
}

void check_opts(hh_ctx* ctx, const hh_opts& o) {
  if (!(o.tol > 0.0) || !(o.tol < 1.0)) fail(ctx, HH_EINVAL, "tol must be in (0, 1)");
  if (o.max_iter < 0) fail(ctx, HH_EINVAL, "max_iter must be >= 0 (0: from the phase contrast)");
  if (o.scheme != 0 && o.scheme != 1) fail(ctx, HH_EINVAL, "scheme must be 0 (CG) or 1 (basic)");
  if (o.precision != 0 && o.precision != 1) fail(ctx, HH_EINVAL, "precision must be 0 or 1");
  if (o.nyquist != 0 && o.nyquist != 1) fail(ctx, HH_EINVAL, "nyquist must be 0 or 1");
  if (o.stall_limit < 0) fail(ctx, HH_EINVAL, "stall_limit must be >= 0 (0: from the phase contrast)");
  if (o.retry != 0 && o.retry != 1) fail(ctx, HH_EINVAL, "retry must be 0 or 1");
  if (o.verify != 0 && o.verify != 1) fail(ctx, HH_EINVAL, "verify must be 0 or 1");
  if (o.lanes < 0 || o.lanes > 4) fail(ctx, HH_EINVAL, "lanes must be in 0..4");
  if (o.chunk < 1) fail(ctx, HH_EINVAL, "chunk must be >= 1");
  if (o.tune != 0 && o.tune != 1) fail(ctx, HH_EINVAL, "tune must be 0 or 1");
  if (o.graph != 0 && o.graph != 1) fail(ctx, HH_EINVAL, "graph must be 0 or 1");
  for (int i = 0; i < 3; ++i)
    if (o.plan[i] < -1 || o.plan[i] >= kNVariant) fail(ctx, HH_EINVAL, "plan entries must be -1 or a variant index");
  if (o.loads_per_wave < 0 || o.loads_per_wave > 6) fail(ctx, HH_EINVAL, "loads_per_wave must be in 0..6");
}

void check_shape(hh_ctx* ctx, int nx, int ny, int nz, int precision) {
  if (nx < 1 || ny < 1 || nz < 1) fail(ctx, HH_EINVAL, "image dimensions must be positive");
  for (int n : {nx, ny, nz})
    if (!size_ops(n, precision))
      fail(ctx, HH_EUNSUPPORTED, "axis length " + std::to_string(n) + " has no compiled FFT passes at this precision");
}

void check_phases(hh_ctx* ctx, const hh_phase* ph, int nphase) {
  if (!ph || nphase < 1 || nphase > kMaxPhase)
    fail(ctx, HH_EINVAL, "need 1.." + std::to_string(kMaxPhase) + " phases");
  for (int i = 0; i < nphase; ++i)
    if (!(ph[i].K > 0.0) || !(ph[i].G > 0.0) || !std::isfinite(ph[i].K) || !std::isfinite(ph[i].G))
      fail(ctx, HH_EINVAL, "phase moduli must be positive and finite");
}

void check_region(hh_ctx* ctx, const int* r, int nx, int ny, int nz) {
  if (!(0 <= r[0] && r[0] < r[3] && r[3] <= nx && 0 <= r[1] && r[1] < r[4] && r[4] <= ny && 0 <= r[2] &&
        r[2] < r[5] && r[5] <= nz))
    fail(ctx, HH_EINVAL, "region must satisfy 0 <= lo < hi <= size on every axis");
}

// Solves all items (same shape) for six loads; results per item.
// Compiled tile variants of one axis pass that fit the device's LDS.
struct PassVariants {
  SizeOpsFn f[kNVariant] = {};
  int geom[kNVariant] = {};     // columns per tile (z, y) or rows per tile (x)
  int threads[kNVariant] = {};  // workgroup size
  bool ok[kNVariant] = {};
  // variant v is worth timing: available and unlike every earlier one
  bool distinct(int v) const {
    if (!ok[v]) return false;
    for (int u = 0; u < v; ++u)
      if (ok[u] && geom[u] == geom[v] && threads[u] == threads[v]) return false;
    return true;
  }
};

PassVariants pass_variants(hh_ctx* ctx, int n, int P, int info_geom, int info_lds, int info_threads) {
  PassVariants pv;
  for (int v = 0; v < kNVariant; ++v) {
    SizeOpsFn f = size_ops(n, P, v);
    if (!f) continue;
    int lds = 0, gm = 0, th = 0;
    f(info_lds, 0, nullptr, nullptr, &lds);
    f(info_geom, 0, nullptr, nullptr, &gm);
    f(info_threads, 0, nullptr, nullptr, &th);
    if (lds > ctx->max_lds) continue;
    pv.f[v] = f;
    pv.geom[v] = gm;
    pv.threads[v] = th;
    pv.ok[v] = true;
  }
  return pv;
}

constexpr int kMaxLanes = 4;  // concurrent shape groups of a batch (hardware queues per process)

// Creates the extra lanes of concurrent shape groups once per context.
void ensure_lanes(hh_ctx* ctx, int n) {
  if (!ctx->fork) HIPCHK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  while (int(ctx->aux.size()) < n) {
    hh_lane l;
    l.prefix = "lane" + std::to_string(ctx->aux.size()) + "/";
    // all streams keep the default priority
    HIPCHK(hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&l.cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&l.e0));
    HIPCHK(hipEventCreate(&l.e1));
    ctx->aux.push_back(l);
  }
}

// Tuned plans on disk (hh_plan_cache): one line per shape,
//   hh-plan <arch> <variants> <nx> <ny> <nz> <precision> <aniso> <bucket> <z> <y> <x>
// where <variants> names the compiled tile-variant set, so that a file
// written by another build or GPU is ignored.
const char* kPlanTag = "v5";
void save_plan(hh_ctx* ctx, const std::array<int, 6>& key, const std::array<int, 3>& plan) {
  if (ctx->plan_file.empty()) return;
  FILE* f = std::fopen(ctx->plan_file.c_str(), "a");
  if (!f) return;  // the cache is an optimisation: a read-only location only costs tuning time
  std::fprintf(f, "hh-plan %s %s %d %d %d %d %d %d %d %d %d\n", ctx->arch.c_str(), kPlanTag, key[0], key[1], key[2],
               key[3], key[4], key[5], plan[0], plan[1], plan[2]);
  std::fclose(f);
}

// The context's own lane: its stream, capture stream and timing events.
hh_lane main_lane(hh_ctx* ctx) {
  hh_lane l;
  l.stream = ctx->stream;
  l.cap = ctx->cap;
  l.e0 = ctx->e0;
  l.e1 = ctx->e1;
  return l;
}

double ms_since(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

GroupResult solve_group(hh_ctx* ctx, const std::vector<Item>& items, const unsigned char* labels,
                        const void* cfield, bool aniso, const hh_opts& o, const double loads[6][6],
                        Profile& prof, void* cfield_out, const hh_lane& lane, int nlanes) {
  const int nx = items[0].nx, ny = items[0].ny, nz = items[0].nz;
  const int P = o.precision;
  const Limits lim = solve_limits(o, items, aniso);
  const PassVariants vz = pass_variants(ctx, nz, P, kOpInfoZ, kOpInfoLdsZ, kOpInfoThreadsZ);
  const PassVariants vy = pass_variants(ctx, ny, P, kOpInfoZ, kOpInfoLdsZ, kOpInfoThreadsZ);
  const PassVariants vx = pass_variants(ctx, nx, P, kOpInfoX, kOpInfoLdsX, kOpInfoThreadsX);
  if (!vz.ok[0] || !vy.ok[0] || !vx.ok[0]) fail(ctx, HH_EUNSUPPORTED, "unsupported axis length");
  const PassVariants* pvs[3] = {&vz, &vy, &vx};
  const int hx = nx / 2 + 1;
  const int hxp = spectrum_pitch(hx);
  const long long nfreq = (long long)hxp * ny * nz;
  const size_t cb = P == 0 ? 8 : 16;
  // geometry of a z variant (M columns per tile): 3-vector fields are stored
  // per z-pass tile, [tile][z][M][3]
  auto nwgz_of = [&](int M) { return ny * ((hx + M - 1) / M); };
  auto nafreq_of = [&](int M) { return (long long)nwgz_of(M) * nz * M; };
  long long nafreq_max = 0;
  for (int v = 0; v < kNVariant; ++v)
    if (vz.ok[v]) nafreq_max = std::max(nafreq_max, nafreq_of(vz.geom[v]));
  // per-row and per-column partial sums (independent of the tile variant)
  const int nrow = ny * nz, ncol = ny * hx;
  const int nchunk_x = (nrow + kFinChunk - 1) / kFinChunk, nchunk_z = (ncol + kFinChunk - 1) / kFinChunk;
  // tmp + ar + ap + the row and column partial sums
  const size_t per_sys = size_t(nfreq) * 6 * cb + size_t(nafreq_max) * 6 * cb + sizeof(double) * (size_t(nrow) * kPartX + ncol);

  size_t freeb = 0, totalb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totalb));
  const size_t budget = std::min<size_t>(size_t(24) << 30, freeb / (2 * size_t(nlanes)));
  int wave = int(std::max<size_t>(1, budget / (6 * per_sys)));
  wave = std::min<int>(wave, int(items.size()));
  wave = std::min(wave, 65535 / 6);
  // Loads per wave: all six, unless the six systems of one image do not fit
  // in the device memory (what is free plus the field buffers this call
  // re-allocates).  Then each image runs alone, a few of its loads at a
  // time, and its stiffness is formed once the final states of all six loads
  // are in.
  size_t held = 0;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    for (const char* name : {"tmp", "ar", "ap"}) {
      auto it = ctx->bufs.find(lane.prefix + name);
      if (it != ctx->bufs.end()) held += it->second.second;
    }
  }
  const size_t avail = size_t(0.85 * double(freeb + held));
  const int fit = 6 * per_sys <= avail ? 6 : int(std::max<size_t>(1, avail / per_sys));
  const int loads_per_wave = std::min(fit, o.loads_per_wave > 0 ? o.loads_per_wave : 6);
  if (loads_per_wave < 6) wave = 1;

  // tile variants: forced, cached for this context, or tuned on the first wave
  std::array<int, 3> plan{{0, 0, 0}};
  for (int i = 0; i < 3; ++i) {
    if (o.plan[i] < 0) continue;
    if (o.plan[i] >= kNVariant || !pvs[i]->ok[o.plan[i]])
      fail(ctx, HH_EINVAL, "tile variant " + std::to_string(o.plan[i]) + " is not available for this pass");
    plan[i] = o.plan[i];
  }
  const bool forced_all = o.plan[0] >= 0 && o.plan[1] >= 0 && o.plan[2] >= 0;
  int bucket = 0;
  while ((6 << bucket) < wave * 6 && bucket < 20) ++bucket;
  const std::array<int, 6> key{{nx, ny, nz, P, aniso ? 1 : 0, bucket}};
  bool need_tune = false;
  if (!forced_all && o.tune && P == 0 && loads_per_wave == 6) {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
      for (int i = 0; i < 3; ++i)
        if (o.plan[i] < 0) plan[i] = it->second[i];
    } else {
      need_tune = true;
    }
  }

  GroupResult res;
  const int nitems = int(items.size());
  res.C72.assign(size_t(nitems) * 72, 0.0);
  res.status.assign(nitems, HH_OK);
  res.iters.assign(size_t(nitems) * 6, 0);
  res.rel.assign(size_t(nitems) * 6, 0.0);

  // reference medium of the basic scheme
  double ref_lam = o.ref_lambda, ref_mu = o.ref_mu;
  if (o.scheme == 1 && (ref_lam <= 0.0 || ref_mu <= 0.0)) {
    if (aniso) fail(ctx, HH_EINVAL, "the basic scheme on anisotropic voxels needs ref_lambda and ref_mu");
    double lmin = 1e300, lmax = -1e300, mmin = 1e300, mmax = -1e300;
    for (const Item& it : items)
      for (const hh_phase& p : it.phases) {
        const double l = p.K - 2.0 * p.G / 3.0;
        lmin = std::min(lmin, l);
        lmax = std::max(lmax, l);
        mmin = std::min(mmin, p.G);
        mmax = std::max(mmax, p.G);
      }
    ref_lam = 0.5 * (lmin + lmax);
    ref_mu = 0.5 * (mmin + mmax);
    if (ref_lam + 2.0 * ref_mu / 3.0 <= 0.0) ref_lam = 0.0;
  }

  std::vector<SysState> split_state(6);  // final states of an image solved a few loads at a time
  for (int w0 = 0; w0 < nitems; w0 += wave) {
    const int nw = std::min(wave, nitems - w0);
    for (int a0 = 0; a0 < 6; a0 += loads_per_wave) {
      const int la = std::min(loads_per_wave, 6 - a0);  // loads of this wave
      const int nsys = nw * la;
      std::vector<ItemDesc> idesc(nw);
      std::vector<SysDesc> sdesc(nsys);
      for (int i = 0; i < nw; ++i) {
        const Item& it = items[w0 + i];
        ItemDesc& d = idesc[i];
        std::memset(&d, 0, sizeof(d));
        d.lab_off = it.lab_off;
        d.cf_off = it.cf_off;
        for (int k = 0; k < 6; ++k) d.region[k] = it.region[k];
        d.nphase = int(it.phases.size());
        const double vol = double(it.region[3] - it.region[0]) * (it.region[4] - it.region[1]) *
                           (it.region[5] - it.region[2]);
        d.inv_region = 1.0 / vol;
        for (int k = 0; k < d.nphase; ++k) {
          d.lam[k] = it.phases[k].K - 2.0 * it.phases[k].G / 3.0;
          d.mu[k] = it.phases[k].G;
        }
        for (int a = 0; a < la; ++a) sdesc[i * la + a] = SysDesc{i, a0 + a};
      }
      auto* d_items = static_cast<ItemDesc*>(ws(ctx, lane.prefix + "items", sizeof(ItemDesc) * nw, lane.stream));
      auto* d_sys = static_cast<SysDesc*>(ws(ctx, lane.prefix + "sys", sizeof(SysDesc) * nsys, lane.stream));
      auto* d_state = static_cast<SysState*>(ws(ctx, lane.prefix + "state", sizeof(SysState) * nw * 6, lane.stream));
      auto* d_px = static_cast<double*>(ws(ctx, lane.prefix + "part_x", sizeof(double) * kPartX * size_t(nrow) * nsys, lane.stream));
      auto* d_pz = static_cast<double*>(ws(ctx, lane.prefix + "part_z", sizeof(double) * size_t(ncol) * nsys, lane.stream));
      auto* d_cx = static_cast<double*>(ws(ctx, lane.prefix + "chunk_x", sizeof(double) * kPartX * size_t(nchunk_x) * nsys, lane.stream));
      auto* d_cz = static_cast<double*>(ws(ctx, lane.prefix + "chunk_z", sizeof(double) * size_t(nchunk_z) * nsys, lane.stream));
      void* d_tmp = ws(ctx, lane.prefix + "tmp", size_t(nfreq) * 6 * cb * nsys, lane.stream);
      void* d_ar = ws(ctx, lane.prefix + "ar", size_t(nafreq_max) * 3 * cb * nsys, lane.stream);
      void* d_ap = ws(ctx, lane.prefix + "ap", size_t(nafreq_max) * 3 * cb * nsys, lane.stream);
      auto* d_out = static_cast<double*>(ws(ctx, lane.prefix + "cout", sizeof(double) * 72 * nw, lane.stream));
      auto* d_ist = static_cast<int*>(ws(ctx, lane.prefix + "istatus", sizeof(int) * nw, lane.stream));
      auto* d_cnt = static_cast<int*>(ws(ctx, lane.prefix + "count", sizeof(int), lane.stream));
      HIPCHK(hipMemcpyAsync(d_items, idesc.data(), sizeof(ItemDesc) * nw, hipMemcpyHostToDevice, lane.stream));
      HIPCHK(hipMemcpyAsync(d_sys, sdesc.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, lane.stream));

      // launch arguments for a choice of z and x variants over the first ns systems
      auto make_args = [&](int ns, int zv, int xv) {
        GroupArgs g;
        std::memset(&g, 0, sizeof(g));
        g.nx = nx;
        g.ny = ny;
        g.nz = nz;
        g.hx = hx;
        g.hxp = hxp;
        g.nsys = ns;
        g.nyq_zero = o.nyquist;
        g.max_iter = lim.max_iter;
        g.scheme = o.scheme;
        g.aniso = aniso ? 1 : 0;
        g.stall_limit = lim.stall;
        g.tol2 = o.tol * o.tol;
        const double u = P == 0 ? 5.96e-8 : 1.11e-16;
        g.zero_rhs2 = (64.0 * u) * (64.0 * u);
        g.ref_lam = o.scheme == 1 ? ref_lam : 0.0;
        g.ref_mu = o.scheme == 1 ? ref_mu : 0.5;
        for (int a = 0; a < 6; ++a)
          for (int c = 0; c < 6; ++c) g.loads[a][c] = loads[a][c];
        g.sys = d_sys;
        g.items = d_items;
        g.labels = labels;
        g.cfield = cfield;
        g.tmp = d_tmp;
        g.ar = d_ar;
        g.ap = d_ap;
        g.tmp_stride = nfreq * 6;
        g.a_stride = nafreq_of(vz.geom[zv]) * 3;
        g.state = d_state;
        g.part_x = d_px;
        g.part_z = d_pz;
        g.chunk_x = d_cx;
        g.chunk_z = d_cz;
        g.nrow_x = nrow;
        g.ncol_z = ncol;
        g.nchunk_x = nchunk_x;
        g.nchunk_z = nchunk_z;
        (void)xv;
        return g;
      };
      const hipStream_t st = lane.stream;

      if (need_tune && w0 == 0) {
        // Time each distinct variant of each pass on this group's buffers, over
        // enough systems to cover ~2^24 voxels, before the right-hand side
        // overwrites them.  Fields are cleared first; states read as running.
        const auto t_start = std::chrono::steady_clock::now();
        const double vox = double(nx) * ny * nz;
        const int items_t = int(std::min<double>(nw, std::max(1.0, std::ceil(16777216.0 / (6.0 * vox)))));
        const int ns = items_t * 6;
        HIPCHK(hipMemsetAsync(d_state, 0, sizeof(SysState) * ns, st));
        HIPCHK(hipMemsetAsync(d_tmp, 0, size_t(nfreq) * 6 * cb * ns, st));
        HIPCHK(hipMemsetAsync(d_ar, 0, size_t(nafreq_max) * 3 * cb * ns, st));
        HIPCHK(hipMemsetAsync(d_ap, 0, size_t(nafreq_max) * 3 * cb * ns, st));
        auto timeit = [&](auto&& launch) {
          launch();
          HIPCHK(hipEventRecord(lane.e0, st));
          for (int r = 0; r < 3; ++r) launch();
          HIPCHK(hipEventRecord(lane.e1, st));
          HIPCHK(hipEventSynchronize(lane.e1));
          HIPCHK(hipGetLastError());
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, lane.e0, lane.e1));
          return ms;
        };
        float best[3] = {1e30f, 1e30f, 1e30f};
        std::array<int, 3> pick = plan;
        for (int v = 0; v < kNVariant; ++v) {
          if (o.plan[0] < 0 && vz.distinct(v)) {
            const GroupArgs gt = make_args(ns, v, 0);
            const float t = timeit([&] {
              vz.f[v](kOpZ, kZInvCg, &gt, st, nullptr);
              vz.f[v](kOpZ, kZFwdCg, &gt, st, nullptr);
            });
            if (t < best[0]) best[0] = t, pick[0] = v;
          }
          if (o.plan[1] < 0 && vy.distinct(v)) {
            const GroupArgs gt = make_args(ns, 0, 0);
            const float t = timeit([&] {
              vy.f[v](kOpY, +1, &gt, st, nullptr);
              vy.f[v](kOpY, -1, &gt, st, nullptr);
            });
            if (t < best[1]) best[1] = t, pick[1] = v;
          }
          if (o.plan[2] < 0 && vx.distinct(v)) {
            const GroupArgs gt = make_args(ns, 0, v);
            const float t = timeit([&] { vx.f[v](kOpX, kXCg, &gt, st, nullptr); });
            if (t < best[2]) best[2] = t, pick[2] = v;
          }
        }
        plan = pick;
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        if (o.plan[0] < 0 && o.plan[1] < 0 && o.plan[2] < 0) {
          ctx->plans[key] = plan;
          save_plan(ctx, key, plan);
        }
        need_tune = false;
        ctx->setup_ms += ms_since(t_start);
      }
      {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        ctx->last_plan = plan;
      }
      const SizeOpsFn oz = vz.f[plan[0]], oy = vy.f[plan[1]], ox = vx.f[plan[2]];

      HIPCHK(hipMemsetAsync(d_state, 0, sizeof(SysState) * nsys, lane.stream));
      HIPCHK(hipMemsetAsync(d_ap, 0, size_t(nafreq_max) * 3 * cb * nsys, lane.stream));
      if (o.scheme == 1) HIPCHK(hipMemsetAsync(d_ar, 0, size_t(nafreq_max) * 3 * cb * nsys, lane.stream));
      const GroupArgs g = make_args(nsys, plan[0], plan[2]);

      // right-hand side b = -G * (C : E)
      prof.run(HH_K_SETUP, [&] { ox(kOpX, kXRhs, &g, st, nullptr); });
      prof.run(HH_K_FIN, [&] { launch_fin_x(kXRhs, g, st); });
      if (o.scheme == 0) {
        prof.run(HH_K_SETUP, [&] { oy(kOpY, -1, &g, st, nullptr); });
        prof.run(HH_K_SETUP, [&] { oz(kOpZ, kZFwdRhs, &g, st, nullptr); });
        prof.run(HH_K_FIN, [&] { launch_fin_z(kZFwdRhs, g, st); });
      }
      const bool cg = o.scheme == 0;
      // one CG (or fixed-point) iteration: five passes and two finalize kernels
      auto iteration = [&](hipStream_t s) {
        oz(kOpZ, cg ? kZInvCg : kZInvFp, &g, s, nullptr);
        oy(kOpY, +1, &g, s, nullptr);
        ox(kOpX, cg ? kXCg : kXFp, &g, s, nullptr);
        launch_fin_x(cg ? kXCg : kXFp, g, s);
        oy(kOpY, -1, &g, s, nullptr);
        oz(kOpZ, cg ? kZFwdCg : kZFwdFp, &g, s, nullptr);
        launch_fin_z(cg ? kZFwdCg : kZFwdFp, g, s);
      };
      const bool use_graph = o.graph && !o.profile && lane.cap;
      int launched = 0;
      const int limit = lim.max_iter + 1;
      while (launched < limit) {
        const int chunk = std::min(o.chunk, limit - launched);
        if (use_graph) {
          // the chunk's launches depend only on their arguments: capture once, replay
          std::string gk(reinterpret_cast<const char*>(&g), sizeof(g));
          const std::uintptr_t tag[5] = {std::uintptr_t(chunk), std::uintptr_t(cg ? 1 : 0),
                                         reinterpret_cast<std::uintptr_t>(oz), reinterpret_cast<std::uintptr_t>(oy),
                                         reinterpret_cast<std::uintptr_t>(ox)};
          gk.append(reinterpret_cast<const char*>(tag), sizeof(tag));
          std::lock_guard<std::recursive_mutex> lk(ctx->mu);  // the cache is shared by the lanes
          auto it = ctx->graphs.find(gk);
          hipGraphExec_t ex = nullptr;
          if (it != ctx->graphs.end()) {
            ex = it->second;
          } else {
            const auto t_start = std::chrono::steady_clock::now();
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(lane.cap, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < chunk; ++k) iteration(lane.cap);
            const hipError_t ec = hipStreamEndCapture(lane.cap, &graph);
            const hipError_t el = hipGetLastError();
            if (ec != hipSuccess || el != hipSuccess || !graph) {
              if (graph) (void)hipGraphDestroy(graph);
              fail(ctx, HH_EDEVICE, std::string("graph capture failed: ") +
                                        hipGetErrorString(ec != hipSuccess ? ec : el));
            }
            const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess)
              fail(ctx, HH_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
            if (nlanes == 1 && ctx->graphs.size() >= 64) clear_graphs(ctx);
            ctx->graphs[gk] = ex;
            ctx->setup_ms += ms_since(t_start);
          }
          HIPCHK(hipGraphLaunch(ex, st));
        } else {
          for (int k = 0; k < chunk; ++k) {
            prof.run(HH_K_ZINV, [&] { oz(kOpZ, cg ? kZInvCg : kZInvFp, &g, st, nullptr); });
            prof.run(HH_K_YINV, [&] { oy(kOpY, +1, &g, st, nullptr); });
            prof.run(HH_K_X, [&] { ox(kOpX, cg ? kXCg : kXFp, &g, st, nullptr); });
            prof.run(HH_K_FIN, [&] { launch_fin_x(cg ? kXCg : kXFp, g, st); });
            prof.run(HH_K_YFWD, [&] { oy(kOpY, -1, &g, st, nullptr); });
            prof.run(HH_K_ZFWD, [&] { oz(kOpZ, cg ? kZFwdCg : kZFwdFp, &g, st, nullptr); });
            prof.run(HH_K_FIN, [&] { launch_fin_z(cg ? kZFwdCg : kZFwdFp, g, st); });
          }
        }
        launched += chunk;
        HIPCHK(hipGetLastError());
        launch_count_running(d_state, nsys, d_cnt, st);
        int running = 0;
        HIPCHK(hipMemcpyAsync(&running, d_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        prof.flush();
        if (running == 0) break;
      }
      if (la < 6) {
        // keep this wave's final states; after the last load, all six go back
        // to the state array, in load order, for the stiffness of the image
        HIPCHK(hipMemcpyAsync(split_state.data() + a0, d_state, sizeof(SysState) * la, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (a0 + la < 6) continue;
        HIPCHK(hipMemcpyAsync(d_state, split_state.data(), sizeof(SysState) * 6, hipMemcpyHostToDevice, st));
      }
      void* cf_out = nullptr;
      if (cfield_out) cf_out = static_cast<char*>(cfield_out) + size_t(w0) * 21 * (P == 0 ? 4 : 8);
      prof.run(HH_K_OTHER, [&] { launch_stiffness(P, d_state, nw, d_out, cf_out, d_ist, st); });
      HIPCHK(hipGetLastError());
      std::vector<SysState> hst(size_t(nw) * 6);
      std::vector<int> ist(nw);
      HIPCHK(hipMemcpyAsync(res.C72.data() + size_t(w0) * 72, d_out, sizeof(double) * 72 * nw, hipMemcpyDeviceToHost,
                            st));
      HIPCHK(hipMemcpyAsync(hst.data(), d_state, sizeof(SysState) * nw * 6, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(ist.data(), d_ist, sizeof(int) * nw, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      prof.flush();
      const double vox = double(nx) * ny * nz;
      // algorithmic bytes: 63 complex words per frequency and iteration (zinv
      // 15, y 12 + 12, x 12, zfwd 12) plus the voxel data, 27 words for the RHS
      const double nfa = double(hx) * ny * nz;
      const double vdata = aniso ? vox * 21.0 * (P == 0 ? 4.0 : 8.0) : vox;
      const double it_bytes = nfa * double(cb) * 63.0 + vdata, rhs_bytes = nfa * double(cb) * 27.0 + vdata;
      double bytes = 0.0;
      for (int i = 0; i < nw; ++i) {
        int code = status_code(ist[i]);
        for (int a = 0; a < 6; ++a) {
          const SysState& s = hst[i * 6 + a];
          res.iters[size_t(w0 + i) * 6 + a] = s.iter;
          res.rel[size_t(w0 + i) * 6 + a] = s.bb > 0.0 ? std::sqrt(s.rr / s.bb) : 0.0;
          res.voxel_iters += vox * s.iter;
          bytes += it_bytes * s.iter + rhs_bytes;
          code = worse(code, status_code(s.status == kRunning ? kNoConv : s.status));
        }
        res.status[w0 + i] = code;
      }
      std::lock_guard<std::recursive_mutex> lk(ctx->mu);
      ctx->call_bytes += bytes;
    }
  }
  return res;
}

// solve_group, then (opts.retry, FP32 fields, isotropic phases) the images
// that stopped at the FP32 floor solved again with FP64 fields: a residual
// that stopped decreasing (HH_ESTAGNATED), or (p, Ap) rounded to <= 0 or a
// non-finite value (HH_EBREAKDOWN; in exact arithmetic (p, Ap) > 0).  Their
// stiffness replaces the FP32 one, also in the next level's field when the
// caller builds one.
GroupResult solve_group_retry(hh_ctx* ctx, const std::vector<Item>& items, const unsigned char* labels,
                              const void* cfield, bool aniso, const hh_opts& o, const double loads[6][6],
                              Profile& prof, void* cfield_out, const hh_lane& lane, int nlanes) {
  GroupResult r = solve_group(ctx, items, labels, cfield, aniso, o, loads, prof, cfield_out, lane, nlanes);
  if (!o.retry || o.precision != 0 || aniso) return r;
  std::vector<int> idx;
  for (size_t i = 0; i < items.size(); ++i)
    if ((r.status[i] == HH_ESTAGNATED || r.status[i] == HH_EBREAKDOWN) && size_ops(items[i].nx, 1) &&
        size_ops(items[i].ny, 1) &&
        size_ops(items[i].nz, 1))
      idx.push_back(int(i));
  if (idx.empty()) return r;
  std::vector<Item> sub;
  for (int i : idx) sub.push_back(items[i]);
  hh_opts o64 = o;
  o64.precision = 1;
  o64.tune = 0;
  o64.plan[0] = o64.plan[1] = o64.plan[2] = -1;
  // FP64 fields have no FP32 floor: at least the contrast-derived stall limit
  hh_opts oa = o;
  oa.stall_limit = 0;
  o64.stall_limit = std::max(o.stall_limit, solve_limits(oa, sub, false).stall);
  const std::array<int, 3> keep_plan = ctx->last_plan;
  GroupResult r64 = solve_group(ctx, sub, labels, nullptr, false, o64, loads, prof, nullptr, lane, nlanes);
  ctx->last_plan = keep_plan;
  std::vector<float> field(idx.size() * 21);
  for (size_t k = 0; k < idx.size(); ++k) {
    const int i = idx[k];
    std::copy(r64.C72.begin() + k * 72, r64.C72.begin() + (k + 1) * 72, r.C72.begin() + size_t(i) * 72);
    r.status[i] = r64.status[k];
    for (int a = 0; a < 6; ++a) {
      r.iters[size_t(i) * 6 + a] = r64.iters[k * 6 + a];
      r.rel[size_t(i) * 6 + a] = r64.rel[k * 6 + a];
    }
    const double* S = r64.C72.data() + k * 72 + 36;
    int q = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) field[k * 21 + q++] = float(S[a * 6 + b]);
  }
  r.voxel_iters += r64.voxel_iters;
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->call_retried += (long long)idx.size();
  }
  if (cfield_out) {
    for (size_t k = 0; k < idx.size(); ++k)
      HIPCHK(hipMemcpyAsync(static_cast<float*>(cfield_out) + size_t(idx[k]) * 21, field.data() + k * 21,
                            sizeof(float) * 21, hipMemcpyHostToDevice, lane.stream));
    HIPCHK(hipStreamSynchronize(lane.stream));
  }
  return r;
}

void begin_report(hh_ctx* ctx, hh_report* rep) {
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->err_vs_oracle = -1.0;
  }
  ctx->setup_ms = 0.0;
  ctx->call_bytes = 0.0;
  ctx->call_retried = 0;
  HIPCHK(hipEventRecord(ctx->t0, ctx->stream));
}

void end_report(hh_ctx* ctx, hh_report* rep) {
  HIPCHK(hipEventRecord(ctx->t1, ctx->stream));
  HIPCHK(hipEventSynchronize(ctx->t1));
  if (rep) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    rep->seconds = ms * 1e-3;
    rep->setup_ms = ctx->setup_ms;
    rep->bytes_moved = ctx->call_bytes;
    rep->retried = ctx->call_retried;
    for (int i = 0; i < 3; ++i) rep->plan[i] = ctx->last_plan[i];
  }
}

void fill_item_report(hh_report* rep, const GroupResult& r, int item) {
  if (!rep) return;
  for (int a = 0; a < 6; ++a) {
    rep->iters[a] = r.iters[size_t(item) * 6 + a];
    rep->rel_resid[a] = r.rel[size_t(item) * 6 + a];
  }
  const double* C = r.C72.data() + size_t(item) * 72;
  double mx = 0.0, md = 0.0;
  for (int i = 0; i < 36; ++i) mx = std::max(mx, std::fabs(C[i]));
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) md = std::max(md, std::fabs(C[i * 6 + j] - C[j * 6 + i]));
  rep->asym = mx > 0.0 ? md / mx : 0.0;
}

// Labels to the device (copy when on host) and check them against nphase.
// check_device = false leaves labels already on the device unchecked: the
// caller then checks them itself before anything indexes a phase table.
const unsigned char* device_labels(hh_ctx* ctx, const uint8_t* labels, long long bytes, bool on_device,
                                   const std::vector<long long>& off, const std::vector<long long>& cnt,
                                   const std::vector<int>& nphase, const char* bufname, bool check_device = true) {
  const unsigned char* d = nullptr;
  const int n = int(off.size());
  if (!on_device) {
    for (int i = 0; i < n; ++i) {
      const uint8_t* p = labels + off[i];
      uint8_t m = 0;
      for (long long k = 0; k < cnt[i]; ++k) m = std::max(m, p[k]);
      if (m >= nphase[i]) fail(ctx, HH_EINVAL, "label " + std::to_string(m) + " >= nphase in item " + std::to_string(i));
    }
    auto* buf = static_cast<unsigned char*>(ws(ctx, bufname, size_t(bytes)));
    HIPCHK(hipMemcpyAsync(buf, labels, size_t(bytes), hipMemcpyHostToDevice, ctx->stream));
    d = buf;
  } else if (!check_device) {
    d = labels;
  } else {
    d = labels;
    auto* d_off = static_cast<long long*>(ws(ctx, "lm_off", sizeof(long long) * n));
    auto* d_cnt = static_cast<long long*>(ws(ctx, "lm_cnt", sizeof(long long) * n));
    auto* d_max = static_cast<int*>(ws(ctx, "lm_max", sizeof(int) * n));
    HIPCHK(hipMemcpyAsync(d_off, off.data(), sizeof(long long) * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(d_cnt, cnt.data(), sizeof(long long) * n, hipMemcpyHostToDevice, ctx->stream));
    launch_label_max(d, d_off, d_cnt, n, *std::max_element(cnt.begin(), cnt.end()), d_max, ctx->stream);
    HIPCHK(hipGetLastError());
    std::vector<int> mx(n);
    HIPCHK(hipMemcpyAsync(mx.data(), d_max, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i)
      if (mx[i] >= nphase[i])
        fail(ctx, HH_EINVAL, "label " + std::to_string(mx[i]) + " >= nphase in item " + std::to_string(i));
  }
  return d;
}

// ||A - B||_F / ||B||_F of two 6x6 Voigt stiffnesses in Mandel scaling
// (shear rows and columns times sqrt 2)
double mandel_rel_error(const double* A, const double* B) {
  double num = 0.0, den = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const double w = (i < 3 ? 1.0 : std::sqrt(2.0)) * (j < 3 ? 1.0 : std::sqrt(2.0));
      const double d = (A[i * 6 + j] - B[i * 6 + j]) * w, b = B[i * 6 + j] * w;
      num += d * d;
      den += b * b;
    }
  return den > 0.0 ? std::sqrt(num / den) : -1.0;
}

void write_C(const GroupResult& r, int item, double* C_out, double* C_raw) {
  const double* C = r.C72.data() + size_t(item) * 72;
  if (C_out) std::memcpy(C_out, C + 36, sizeof(double) * 36);
  if (C_raw) std::memcpy(C_raw, C, sizeof(double) * 36);
}

// Device bytes one image's solve with all six loads together takes from the
// workspace: spectrum and both 3-vector fields of the six systems (the
// largest z-tile layout), the row and column sums and their chunk sums, and
// 64 KiB for the descriptors, states and label checks.
size_t noalloc_bytes(hh_ctx* ctx, int nx, int ny, int nz, int precision) {
  const PassVariants vz = pass_variants(ctx, nz, precision, kOpInfoZ, kOpInfoLdsZ, kOpInfoThreadsZ);
  const int hx = nx / 2 + 1;
  const size_t cb = precision == 0 ? 8 : 16;
  const size_t nfreq = size_t(spectrum_pitch(hx)) * ny * nz;
  size_t nafreq = 0;
  for (int v = 0; v < kNVariant; ++v)
    if (vz.ok[v]) nafreq = std::max(nafreq, size_t(ny) * ((hx + vz.geom[v] - 1) / vz.geom[v]) * nz * vz.geom[v]);
  const size_t nrow = size_t(ny) * nz, ncol = size_t(ny) * hx;
  const size_t nchunk = (nrow + kFinChunk - 1) / kFinChunk + (ncol + kFinChunk - 1) / kFinChunk;
  const size_t per_sys = nfreq * 6 * cb + nafreq * 6 * cb + 8 * (nrow * kPartX + ncol + nchunk * kPartX);
  return 6 * per_sys + (size_t(64) << 10);
}

// The two-level scheme with network subimage stiffnesses, the gate and the
// FFT fallback (body of hh_hierarchical_surrogate and of hh_hierarchical
// with use_surrogate = 1).
int hierarchical_surrogate_impl(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device,
                                const hh_phase* phases, int nphase, int n_sub, int pad, hh_net* net_a,
                                hh_net* net_b, double spread_tol, double bound_tol, const hh_opts& o,
                                double C_out[36], double* C_sub, int* fallback, hh_report* report) {
  if (!labels || !C_out || !net_a) fail(ctx, HH_EINVAL, "labels, net_a and C_out are required");
  if (nx < 1 || ny < 1 || nz < 1 || n_sub < 1) fail(ctx, HH_EINVAL, "sizes must be positive");
  if (nx % n_sub || ny % n_sub || nz % n_sub) fail(ctx, HH_EINVAL, "the subimage size must divide the image size");
  if (pad < 0 || 2 * pad >= std::min(nx, std::min(ny, nz)))
    fail(ctx, HH_EINVAL, "padding must satisfy 0 <= 2 pad < image size");
  // a network reads either the n_sub^3 core (offset pad) or the whole box
  const int in_a = hh_net_input_size(net_a), in_b = net_b ? hh_net_input_size(net_b) : in_a;
  auto window_ok = [&](int e) { return e == n_sub || e == n_sub + 2 * pad; };
  if (!window_ok(in_a) || !window_ok(in_b))
    fail(ctx, HH_EINVAL, "the network input edge must be the subimage size or the padded box size");
  if (!(spread_tol > 0.0) || !(bound_tol >= 0.0)) fail(ctx, HH_EINVAL, "bad gate tolerances");
  const int b = n_sub + 2 * pad;
  const int mx = nx / n_sub, my = ny / n_sub, mz = nz / n_sub;
  check_shape(ctx, b, b, b, o.precision);
  // one subimage: the intermediate image is a single voxel, whose solve is the identity
  const bool single = mx == 1 && my == 1 && mz == 1;
  if (!single) check_shape(ctx, mx, my, mz, o.precision);
  check_phases(ctx, phases, nphase);
  if (nphase > 8) fail(ctx, HH_EINVAL, "the surrogate takes at most 8 phases");
  const long long nvox = (long long)nx * ny * nz;
  const int nitems = mx * my * mz;
  begin_report(ctx, report);
  const hipStream_t st = ctx->stream;
  // device labels are checked from the cores' label counts below (the cores
  // tile the image), not by a pass of their own
  const unsigned char* d_img =
      device_labels(ctx, labels, nvox, labels_on_device != 0, {0}, {nvox}, {nphase}, "image", false);
  const long long box = (long long)b * b * b;
  Profile prof{ctx, o.profile != 0, {}, 0, report};
  // Networks that read the cores take them straight from the image (its
  // blocks are the cores); the padded boxes are then gathered only when the
  // gate sends items to the FFT solver.
  const bool image_in = in_a == n_sub && (!net_b || in_b == n_sub) && hh_net_image_input(net_a, d_img, nx, ny) &&
                        (!net_b || hh_net_image_input(net_b, d_img, nx, ny));
  unsigned char* d_pack = nullptr;
  auto gather = [&] {
    d_pack = static_cast<unsigned char*>(ws(ctx, "pack", size_t(box * nitems)));
    prof.run(HH_K_SETUP, [&] { launch_gather_pad(d_img, nx, ny, nz, n_sub, pad, d_pack, st); });
  };
  if (!image_in) gather();
  // label counts of the cores (bounds, core-input networks) and, for a
  // network that reads the whole box, of the boxes; the predictions
  auto* c21a = static_cast<double*>(ws(ctx, "sur_c21a", sizeof(double) * 21 * nitems));
  double* c21b = net_b ? static_cast<double*>(ws(ctx, "sur_c21b", sizeof(double) * 21 * nitems)) : nullptr;
  auto* d_counts = static_cast<int*>(ws(ctx, "sur_counts", sizeof(int) * 8 * size_t(nitems)));
  const bool box_in = in_a != n_sub || (net_b && in_b != n_sub);
  int* d_counts_box = box_in ? static_cast<int*>(ws(ctx, "sur_counts_box", sizeof(int) * 8 * size_t(nitems))) : nullptr;
  unsigned* d_if_core = nullptr;  // interface counts (core and box windows), where a network has their statistics
  unsigned* d_if_box = nullptr;
  prof.run(HH_K_OTHER, [&] {
    // a second network runs on a lane stream of its own, concurrently with the
    // first (each has its own buffers; one network given twice stays on st)
    const bool two = net_b && net_b != net_a;
    hipStream_t sb = st;
    if (two) {
      ensure_lanes(ctx, 1);
      sb = ctx->aux[0].stream;
      HIPCHK(hipEventRecord(ctx->fork, st));
      HIPCHK(hipStreamWaitEvent(sb, ctx->fork, 0));
    }
    // st waits for the lane's work however this scope ends
    struct Join {
      hh_ctx* c;
      hipStream_t st, sb;
      bool on;
      ~Join() {
        if (on) {
          (void)hipEventRecord(c->aux[0].e1, sb);
          (void)hipStreamWaitEvent(st, c->aux[0].e1, 0);
        }
      }
    } join{ctx, st, sb, two};
    // label counts of the cores (the heads' fraction features, the bounds):
    // with two networks on image windows, on the lane, and the first network
    // waits for them only before its first head
    const bool counts_on_lane = two && image_in;
    hipEvent_t counts_ready = nullptr;
    // with image windows and an interface test (then of the cores), one pass
    // gives the interface and the label counts
    const bool fused = image_in && (hh_net_has_interface_stats(net_a) || hh_net_has_interface_stats(net_b));
    if (fused) {
      d_if_core = static_cast<unsigned*>(ws(ctx, "sur_iface", sizeof(unsigned) * size_t(nitems)));
      hh_launch_interfaces_image(d_img, nx, ny, n_sub, nitems, d_if_core, counts_on_lane ? sb : st, d_counts);
    } else if (image_in) {
      hh_launch_counts_image(d_img, nx, ny, n_sub, nitems, d_counts, counts_on_lane ? sb : st);
    } else {
      hh_launch_counts(d_pack, nitems, b, pad, n_sub, d_counts, st);
    }
    if (box_in) hh_launch_counts(d_pack, nitems, b, 0, b, d_counts_box, st);
    if (counts_on_lane) {
      counts_ready = ctx->aux[0].e0;
      HIPCHK(hipEventRecord(counts_ready, sb));
    }
    // interface counts of the windows a network with texture statistics reads
    // (only the gate needs them): on the lane, ahead of the second network
    for (hh_net* net : {net_a, net_b}) {
      if (!hh_net_has_interface_stats(net)) continue;
      const bool core = hh_net_input_size(net) == n_sub;
      unsigned*& d = core ? d_if_core : d_if_box;
      if (d) continue;
      d = static_cast<unsigned*>(ws(ctx, core ? "sur_iface" : "sur_iface_box", sizeof(unsigned) * size_t(nitems)));
      if (image_in)
        hh_launch_interfaces_image(d_img, nx, ny, n_sub, nitems, d, sb, nullptr);
      else
        hh_launch_interfaces(d_pack, nitems, b, core ? pad : 0, core ? n_sub : b, d, sb);
    }
    if (image_in) {
      hh_net_predict_image(ctx, net_a, d_img, nx, ny, nitems, c21a, d_counts, st, counts_ready);
      if (net_b) hh_net_predict_image(ctx, net_b, d_img, nx, ny, nitems, c21b, d_counts, sb, nullptr);
    } else {
      hh_net_predict_device(ctx, net_a, d_pack, nitems, b, in_a == n_sub ? pad : 0, c21a,
                            in_a == n_sub ? d_counts : d_counts_box, st);
      if (net_b)
        hh_net_predict_device(ctx, net_b, d_pack, nitems, b, in_b == n_sub ? pad : 0, c21b,
                              in_b == n_sub ? d_counts : d_counts_box, sb);
    }
  });
  // Voigt and Reuss stiffness of each core's phase fractions
  std::vector<double> cp(21 * nphase), sp(21 * nphase);
  for (int q = 0; q < nphase; ++q) {
    const double K = phases[q].K, G = phases[q].G;
    double C[6][6] = {}, S[6][6] = {};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        C[i][j] = (i == j) ? K + 4.0 * G / 3.0 : K - 2.0 * G / 3.0;
        S[i][j] = (i == j) ? 1.0 / (9.0 * K) + 1.0 / (3.0 * G) : 1.0 / (9.0 * K) - 1.0 / (6.0 * G);
      }
    for (int i = 3; i < 6; ++i) {
      C[i][i] = G;
      S[i][i] = 1.0 / G;
    }
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) {
        cp[q * 21 + k] = C[i][j];
        sp[q * 21 + k] = S[i][j];
        ++k;
      }
  }
  auto* d_cp = static_cast<double*>(ws(ctx, "sur_cp", sizeof(double) * 21 * nphase));
  auto* d_sp = static_cast<double*>(ws(ctx, "sur_sp", sizeof(double) * 21 * nphase));
  auto* cv21 = static_cast<double*>(ws(ctx, "sur_cv", sizeof(double) * 21 * nitems));
  auto* cr21 = static_cast<double*>(ws(ctx, "sur_cr", sizeof(double) * 21 * nitems));
  auto* d_flag = static_cast<int*>(ws(ctx, "sur_flag", sizeof(int) * nitems));
  HIPCHK(hipMemcpyAsync(d_cp, cp.data(), sizeof(double) * 21 * nphase, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_sp, sp.data(), sizeof(double) * 21 * nphase, hipMemcpyHostToDevice, st));
  prof.run(HH_K_OTHER, [&] {
    hh_launch_bounds(d_counts, nitems, n_sub, nphase, d_cp, d_sp, cv21, cr21, st);
    const FracGate ga = hh_net_fraction_gate(net_a, in_a == n_sub ? d_counts : d_counts_box,
                                             in_a == n_sub ? d_if_core : d_if_box);
    const FracGate gb = hh_net_fraction_gate(net_b, in_b == n_sub ? d_counts : d_counts_box,
                                             in_b == n_sub ? d_if_core : d_if_box);
    hh_launch_gate(c21a, c21b, cv21, cr21, nitems, spread_tol, bound_tol, ga, gb, d_flag, st);
  });
  HIPCHK(hipGetLastError());
  // flags and predictions through pinned staging buffers (a pageable copy of
  // these 0.7 MB arrays costs several times the transfer)
  const size_t nf = 21 * size_t(nitems);
  int* flag = pinned<int>(ctx, "sur_flag_h", size_t(nitems));
  double* ha = pinned<double>(ctx, "sur_c21a_h", nf);
  double* hb = net_b ? pinned<double>(ctx, "sur_c21b_h", nf) : nullptr;
  double* field = pinned<double>(ctx, "sur_field_h", nf);
  int* hc = labels_on_device ? pinned<int>(ctx, "sur_counts_h", 8 * size_t(nitems)) : nullptr;
  HIPCHK(hipMemcpyAsync(flag, d_flag, sizeof(int) * nitems, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ha, c21a, sizeof(double) * nf, hipMemcpyDeviceToHost, st));
  if (net_b) HIPCHK(hipMemcpyAsync(hb, c21b, sizeof(double) * nf, hipMemcpyDeviceToHost, st));
  if (hc) HIPCHK(hipMemcpyAsync(hc, d_counts, sizeof(int) * 8 * nitems, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  prof.flush();
  // labels >= nphase (device input): every voxel lies in exactly one core; a
  // label below 8 shows in its count, and a core whose counts sum to less than
  // n_sub^3 holds a label of 8 or more
  if (hc) {
    const long long nc = (long long)n_sub * n_sub * n_sub;
    for (int i = 0; i < nitems; ++i) {
      long long sum = 0;
      for (int c = 0; c < 8; ++c) {
        sum += hc[8 * i + c];
        if (c >= nphase && hc[8 * i + c] > 0)
          fail(ctx, HH_EINVAL, "label " + std::to_string(c) + " >= nphase in subimage " + std::to_string(i));
      }
      if (sum != nc) fail(ctx, HH_EINVAL, "a label of 8 or more (>= nphase) in subimage " + std::to_string(i));
    }
  }
  // FFT solves of the gated items
  std::vector<int> fb;
  for (int i = 0; i < nitems; ++i)
    if (flag[i]) fb.push_back(i);
  for (size_t i = 0; i < nf; ++i) field[i] = net_b ? 0.5 * (ha[i] + hb[i]) : ha[i];
  double vi = 0.0;
  int rc = HH_OK;
  double L[6][6];
  unit_loads(L);
  if (!fb.empty()) {
    if (!d_pack) gather();
    std::vector<Item> items(fb.size());
    for (size_t k = 0; k < fb.size(); ++k) {
      Item& it = items[k];
      it.nx = it.ny = it.nz = b;
      it.lab_off = box * fb[k];
      it.cf_off = -1;
      const int r[6] = {pad, pad, pad, pad + n_sub, pad + n_sub, pad + n_sub};
      std::memcpy(it.region, r, sizeof(r));
      it.phases.assign(phases, phases + nphase);
    }
    GroupResult r1 = solve_group_retry(ctx, items, d_pack, nullptr, false, o, L, prof, nullptr, main_lane(ctx), 1);
    vi += r1.voxel_iters;
    for (size_t k = 0; k < fb.size(); ++k) {
      rc = worse(rc, r1.status[k]);
      const double* S = r1.C72.data() + k * 72 + 36;
      int q = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) field[size_t(fb[k]) * 21 + q++] = S[i * 6 + j];
    }
  }
  if (C_sub) std::memcpy(C_sub, field, sizeof(double) * nf);
  if (fallback) std::memcpy(fallback, flag, sizeof(int) * nitems);
  if (single) {
    end_report(ctx, report);
    int q = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j) C_out[i * 6 + j] = C_out[j * 6 + i] = field[q++];
    if (report) {
      report->voxel_iters = vi;
      report->items = nitems;
      report->status = rc;
    }
    return rc;
  }
  // level 2
  auto* d_field = static_cast<double*>(ws(ctx, "sur_field", sizeof(double) * nf));
  HIPCHK(hipMemcpyAsync(d_field, field, sizeof(double) * nf, hipMemcpyHostToDevice, st));
  void* cf = ws(ctx, "cfield", nf * (o.precision == 0 ? 4 : 8));
  launch_convert_field(o.precision, d_field, cf, (long long)nf, st);
  HIPCHK(hipGetLastError());
  Item l2;
  l2.nx = mx;
  l2.ny = my;
  l2.nz = mz;
  l2.lab_off = 0;
  l2.cf_off = 0;
  const int whole[6] = {0, 0, 0, mx, my, mz};
  std::memcpy(l2.region, whole, sizeof(l2.region));
  l2.phases.assign(1, hh_phase{1.0, 1.0});
  GroupResult r2 = solve_group(ctx, {l2}, nullptr, cf, true, o, L, prof, nullptr, main_lane(ctx), 1);
  end_report(ctx, report);
  write_C(r2, 0, C_out, nullptr);
  rc = worse(rc, r2.status[0]);
  if (report) {
    fill_item_report(report, r2, 0);
    report->voxel_iters = vi + r2.voxel_iters;
    report->items = nitems;
    report->status = rc;
  }
  return rc;
}

}  // namespace

extern "C" {

void hh_default_opts(hh_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->max_iter = 0;
  o->scheme = 0;
  o->precision = 0;
  o->nyquist = 0;
  o->profile = 0;
  o->stall_limit = 0;
  o->chunk = 8;
  o->ref_lambda = 0.0;
  o->ref_mu = 0.0;
  o->tune = 1;
  o->graph = 1;
  o->plan[0] = o->plan[1] = o->plan[2] = -1;
  o->loads_per_wave = 0;
  o->retry = 1;
  o->verify = 0;
  o->lanes = 0;
}

int hh_create(hh_ctx** out, int device, void* hip_stream) {
  // the reason of a failure stays readable without a context: hh_last_error(NULL)
  auto failed = [](int code, const std::string& why, hipError_t e) {
    g_create_error = why + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
    return code;
  };
  g_create_error.clear();
  if (!out) return failed(HH_EINVAL, "hh_create: ctx pointer is NULL", hipSuccess);
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return failed(HH_EDEVICE, "hh_create: hipGetDeviceCount failed", e);
  if (device < 0 || device >= ndev)
    return failed(HH_EDEVICE, "hh_create: device " + std::to_string(device) + " out of range (" +
                                  std::to_string(ndev) + " devices)", hipSuccess);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return failed(HH_EDEVICE, "hh_create: hipGetDeviceProperties failed", e);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return failed(HH_EDEVICE, std::string("hh_create: device is ") + prop.gcnArchName + ", not gfx950", hipSuccess);
  auto* ctx = new hh_ctx();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->max_lds = int(prop.sharedMemPerBlock);
  ctx->arch = prop.gcnArchName;
  ctx->arch = ctx->arch.substr(0, ctx->arch.find(':'));
  const char* step = "hipSetDevice";
  e = hipSetDevice(device);
  if (e == hipSuccess) step = "hipEventCreate", e = hipEventCreate(&ctx->t0);
  if (e == hipSuccess) e = hipEventCreate(&ctx->t1);
  if (e == hipSuccess) e = hipEventCreate(&ctx->e0);
  if (e == hipSuccess) e = hipEventCreate(&ctx->e1);
  // the capture stream keeps the default priority
  if (e == hipSuccess) step = "hipStreamCreateWithFlags", e = hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    hh_destroy(ctx);
    return failed(HH_EDEVICE, std::string("hh_create: ") + step + " failed", e);
  }
  std::string why;
  if (init_scratch(device, why) != HH_OK) {
    hh_destroy(ctx);
    return failed(HH_EDEVICE, why, hipSuccess);
  }
  *out = ctx;
  return HH_OK;
}

int hh_set_stream(hh_ctx* ctx, void* hip_stream) {
  if (!ctx) return HH_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return HH_OK;
}

void hh_release_workspace(hh_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  clear_graphs(ctx);  // they hold the addresses of the buffers freed here
  for (auto& b : ctx->bufs) (void)hipFree(b.second.first);
  ctx->bufs.clear();
  for (auto& b : ctx->host_bufs) (void)hipHostFree(b.second.first);
  ctx->host_bufs.clear();
}

void hh_destroy(hh_ctx* ctx) {
  if (!ctx) return;
  hh_release_workspace(ctx);
  for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
  if (ctx->t0) (void)hipEventDestroy(ctx->t0);
  if (ctx->t1) (void)hipEventDestroy(ctx->t1);
  if (ctx->e0) (void)hipEventDestroy(ctx->e0);
  if (ctx->e1) (void)hipEventDestroy(ctx->e1);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  for (hh_lane& l : ctx->aux) {
    (void)hipStreamSynchronize(l.stream);
    (void)hipStreamDestroy(l.stream);
    (void)hipStreamDestroy(l.cap);
    (void)hipEventDestroy(l.e0);
    (void)hipEventDestroy(l.e1);
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  delete ctx;
}

const char* hh_last_error(const hh_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

long long hh_workspace_bytes(const hh_ctx* ctx) {
  if (!ctx) return 0;
  long long s = 0;
  for (auto& b : ctx->bufs) s += (long long)b.second.second;
  return s;
}

int hh_size_supported(int n, int precision) {
  if (precision != 0 && precision != 1) return 0;
  return size_ops(n, precision) ? 1 : 0;
}

int hh_homogenize(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device,
                  const hh_phase* phases, int nphase, const double* loads, const int* region, const hh_opts* opts,
                  double C_out[36], double C_raw[36], hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    if (!labels || !C_out) fail(ctx, HH_EINVAL, "labels and C_out are required");
    check_shape(ctx, nx, ny, nz, o.precision);
    check_phases(ctx, phases, nphase);
    Item it;
    it.nx = nx;
    it.ny = ny;
    it.nz = nz;
    it.lab_off = 0;
    it.cf_off = -1;
    const int whole[6] = {0, 0, 0, nx, ny, nz};
    const int* r = region ? region : whole;
    check_region(ctx, r, nx, ny, nz);
    std::memcpy(it.region, r, sizeof(it.region));
    it.phases.assign(phases, phases + nphase);
    double L[6][6];
    if (loads) {
      loads_from_voigt(loads, L);
      if (!loads_independent(L)) fail(ctx, HH_EINVAL, "the six loads are not independent");
    } else {
      unit_loads(L);
    }
    const long long nvox = (long long)nx * ny * nz;
    begin_report(ctx, report);
    const unsigned char* d_lab =
        device_labels(ctx, labels, nvox, labels_on_device != 0, {0}, {nvox}, {nphase}, "labels");
    Profile prof{ctx, o.profile != 0, {}, 0, report};
    GroupResult res = solve_group_retry(ctx, {it}, d_lab, nullptr, false, o, L, prof, nullptr, main_lane(ctx), 1);
    end_report(ctx, report);
    write_C(res, 0, C_out, C_raw);
    if (report) {
      fill_item_report(report, res, 0);
      report->voxel_iters = res.voxel_iters;
      report->items = 1;
      report->status = res.status[0];
    }
    if (o.verify && report && size_ops(nx, 1) && size_ops(ny, 1) && size_ops(nz, 1)) {
      // the same solve with FP64 fields at tol 1e-10, outside the timed call
      hh_opts o64 = o;
      o64.precision = 1;
      o64.tol = 1e-10;
      o64.tune = 0;
      o64.profile = 0;
      o64.plan[0] = o64.plan[1] = o64.plan[2] = -1;
      Profile quiet{ctx, false, {}, 0, nullptr};
      const std::array<int, 3> keep_plan = ctx->last_plan;
      GroupResult r64 = solve_group(ctx, {it}, d_lab, nullptr, false, o64, L, quiet, nullptr, main_lane(ctx), 1);
      ctx->last_plan = keep_plan;
      report->err_vs_oracle = mandel_rel_error(res.C72.data() + 36, r64.C72.data() + 36);
    }
    if (res.status[0] != HH_OK) ctx->err = "solve did not converge cleanly (see report.status)";
    return res.status[0];
  });
}

int hh_homogenize_noalloc(hh_ctx* ctx, const uint8_t* labels_device, int nx, int ny, int nz, const hh_phase* phases,
                          int nphase, const hh_opts* opts, double C_out[36], hh_report* report) {
  if (!ctx) return HH_EINVAL;
  hh_opts o;
  hh_default_opts(&o);
  if (opts) o = *opts;
  // plain launches only (no graph instantiation), no profiling events, no
  // FP64 retry or check (they would need more scratch)
  o.graph = 0;
  o.profile = 0;
  o.retry = 0;
  o.verify = 0;
  o.lanes = 1;
  int rc = guarded(ctx, [&]() -> int {
    if (!labels_device || !C_out) fail(ctx, HH_EINVAL, "labels_device and C_out are required");
    check_opts(ctx, o);
    check_shape(ctx, nx, ny, nz, o.precision);
    const size_t need = noalloc_bytes(ctx, nx, ny, nz, o.precision);
    if (need > kScratchBytes)
      fail(ctx, HH_EINVAL, "a " + std::to_string(nx) + "x" + std::to_string(ny) + "x" + std::to_string(nz) +
                               " image needs about " + std::to_string(need) + " bytes of scratch; the allocation-free "
                               "entry point holds " + std::to_string(kScratchBytes) + " (FP32 images up to about 64^3)");
    void* base = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      base = g_scratch_ptr[ctx->device];
    }
    if (!base) fail(ctx, HH_EDEVICE, "the static scratch of this device was not set up");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->arena_base = static_cast<char*>(base);
    ctx->arena_size = kScratchBytes;
    ctx->arena_used = 0;
    ctx->arena_bufs.clear();
    return HH_OK;
  });
  if (rc != HH_OK) return rc;
  rc = hh_homogenize(ctx, labels_device, nx, ny, nz, 1, phases, nphase, nullptr, nullptr, &o, C_out, nullptr, report);
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  ctx->arena_base = nullptr;
  ctx->arena_size = ctx->arena_used = 0;
  ctx->arena_bufs.clear();
  return rc;
}

int hh_homogenize_aniso(hh_ctx* ctx, const double* C21, int nx, int ny, int nz, int c21_on_device,
                        const hh_opts* opts, double C_out[36], double C_raw[36], hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    if (!C21 || !C_out) fail(ctx, HH_EINVAL, "C21 and C_out are required");
    check_shape(ctx, nx, ny, nz, o.precision);
    const long long nvox = (long long)nx * ny * nz;
    const long long nval = nvox * 21;
    if (!c21_on_device) {
      for (long long i = 0; i < nval; ++i)
        if (!std::isfinite(C21[i])) fail(ctx, HH_EINVAL, "non-finite stiffness component");
    }
    begin_report(ctx, report);
    const double* src = C21;
    if (!c21_on_device) {
      auto* d = static_cast<double*>(ws(ctx, "c21_in", sizeof(double) * nval));
      HIPCHK(hipMemcpyAsync(d, C21, sizeof(double) * nval, hipMemcpyHostToDevice, ctx->stream));
      src = d;
    }
    void* cf = ws(ctx, "cfield", size_t(nval) * (o.precision == 0 ? 4 : 8));
    launch_convert_field(o.precision, src, cf, nval, ctx->stream);
    HIPCHK(hipGetLastError());
    Item it;
    it.nx = nx;
    it.ny = ny;
    it.nz = nz;
    it.lab_off = 0;
    it.cf_off = 0;
    const int whole[6] = {0, 0, 0, nx, ny, nz};
    std::memcpy(it.region, whole, sizeof(it.region));
    it.phases.assign(1, hh_phase{1.0, 1.0});
    double L[6][6];
    unit_loads(L);
    Profile prof{ctx, o.profile != 0, {}, 0, report};
    GroupResult res = solve_group(ctx, {it}, nullptr, cf, true, o, L, prof, nullptr, main_lane(ctx), 1);
    end_report(ctx, report);
    write_C(res, 0, C_out, C_raw);
    if (report) {
      fill_item_report(report, res, 0);
      report->voxel_iters = res.voxel_iters;
      report->items = 1;
      report->status = res.status[0];
    }
    return res.status[0];
  });
}

int hh_homogenize_batch(hh_ctx* ctx, int nitems, const int* dims, const uint8_t* labels, long long labels_bytes,
                        int labels_on_device, const long long* label_off, const hh_phase* phases,
                        const int* phase_off, const int* nphase, const int* regions, const hh_opts* opts,
                        double* C_out, double* C_raw, int* item_status, int* item_iters, hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    if (nitems < 1 || !dims || !labels || !label_off || !phases || !phase_off || !nphase || !C_out)
      fail(ctx, HH_EINVAL, "missing batch arguments");
    std::vector<Item> items(nitems);
    std::vector<long long> off(nitems), cnt(nitems);
    std::vector<int> nph(nitems);
    for (int i = 0; i < nitems; ++i) {
      Item& it = items[i];
      it.nx = dims[3 * i];
      it.ny = dims[3 * i + 1];
      it.nz = dims[3 * i + 2];
      check_shape(ctx, it.nx, it.ny, it.nz, o.precision);
      check_phases(ctx, phases + phase_off[i], nphase[i]);
      it.phases.assign(phases + phase_off[i], phases + phase_off[i] + nphase[i]);
      it.lab_off = label_off[i];
      it.cf_off = -1;
      const long long nv = (long long)it.nx * it.ny * it.nz;
      if (it.lab_off < 0 || it.lab_off + nv > labels_bytes) fail(ctx, HH_EINVAL, "item labels outside the pack");
      off[i] = it.lab_off;
      cnt[i] = nv;
      nph[i] = nphase[i];
      const int whole[6] = {0, 0, 0, it.nx, it.ny, it.nz};
      const int* r = regions ? regions + 6 * i : whole;
      check_region(ctx, r, it.nx, it.ny, it.nz);
      std::memcpy(it.region, r, sizeof(it.region));
    }
    double L[6][6];
    unit_loads(L);
    begin_report(ctx, report);
    const unsigned char* d_lab =
        device_labels(ctx, labels, labels_bytes, labels_on_device != 0, off, cnt, nph, "labels");
    // group by shape
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < nitems; ++i) groups[{items[i].nx, items[i].ny, items[i].nz}].push_back(i);
    std::vector<std::vector<int>> members;
    for (auto& kv : groups) members.push_back(kv.second);
    const int ngroup = int(members.size());
    std::vector<GroupResult> results(ngroup);
    auto group_items = [&](int q) {
      std::vector<Item> gi;
      for (int i : members[q]) gi.push_back(items[i]);
      return gi;
    };
    // Shape groups run concurrently on up to kMaxLanes lanes (threads with
    // their own streams and buffers), largest work first, so the tail
    // iterations of one group overlap the work of the others; each system
    // computes the same bits on any lane.
    int nl = o.lanes > 0 ? o.lanes : 1;
    nl = std::min(nl, ngroup);
    if (o.profile) nl = 1;
    if (nl <= 1) {
      Profile prof{ctx, o.profile != 0, {}, 0, report};
      for (int q = 0; q < ngroup; ++q)
        results[q] = solve_group_retry(ctx, group_items(q), d_lab, nullptr, false, o, L, prof, nullptr,
                                       main_lane(ctx), 1);
    } else {
      ensure_lanes(ctx, nl);
      std::vector<int> order(ngroup);
      for (int q = 0; q < ngroup; ++q) order[q] = q;
      auto work = [&](int q) {
        const double v = double(items[members[q][0]].nx) * items[members[q][0]].ny * items[members[q][0]].nz;
        return v * double(members[q].size());
      };
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
      // the lanes start after the labels are on the device
      HIPCHK(hipEventRecord(ctx->fork, ctx->stream));
      for (int l = 0; l < nl; ++l) HIPCHK(hipStreamWaitEvent(ctx->aux[l].stream, ctx->fork, 0));
      std::atomic<int> next{0};
      std::vector<int> lane_rc(nl, HH_OK);
      std::vector<std::string> lane_err(nl);
      std::vector<std::thread> th;
      for (int l = 0; l < nl; ++l)
        th.emplace_back([&, l]() {
          try {
            if (hipSetDevice(ctx->device) != hipSuccess) throw Fail{HH_EDEVICE};
            Profile quiet{ctx, false, {}, 0, nullptr};
            for (int k = next++; k < ngroup; k = next++)
              results[order[k]] = solve_group_retry(ctx, group_items(order[k]), d_lab, nullptr, false, o, L, quiet,
                                                    nullptr, ctx->aux[l], nl);
          } catch (const Fail& e) {
            lane_rc[l] = e.code;
            std::lock_guard<std::recursive_mutex> lk(ctx->mu);
            lane_err[l] = ctx->err;
          } catch (...) {
            lane_rc[l] = HH_EDEVICE;
            lane_err[l] = "unknown error in a lane";
          }
        });
      for (auto& t : th) t.join();
      for (int l = 0; l < nl; ++l)
        if (lane_rc[l] != HH_OK) fail(ctx, lane_rc[l], lane_err[l]);
    }
    int rc = HH_OK;
    double vi = 0.0;
    for (int q = 0; q < ngroup; ++q) {
      const GroupResult& res = results[q];
      vi += res.voxel_iters;
      for (size_t k = 0; k < members[q].size(); ++k) {
        const int i = members[q][k];
        write_C(res, int(k), C_out + size_t(i) * 36, C_raw ? C_raw + size_t(i) * 36 : nullptr);
        if (item_status) item_status[i] = res.status[k];
        if (item_iters)
          for (int a = 0; a < 6; ++a) item_iters[size_t(i) * 6 + a] = res.iters[k * 6 + a];
        rc = worse(rc, res.status[k]);
        if (report && i == 0) fill_item_report(report, res, int(k));
      }
    }
    end_report(ctx, report);
    if (report) {
      report->voxel_iters = vi;
      report->items = nitems;
      report->status = rc;
    }
    return rc;
  });
}

int hh_hierarchical(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device,
                    const hh_phase* phases, int nphase, int n_sub, int pad, int use_surrogate, const hh_opts* opts,
                    double C_out[36], double* C_sub, hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    if (use_surrogate != 0 && use_surrogate != 1) fail(ctx, HH_EINVAL, "use_surrogate must be 0 or 1");
    if (use_surrogate) {
      if (!ctx->sur_a) fail(ctx, HH_EINVAL, "use_surrogate = 1 needs networks attached with hh_set_surrogate");
      return hierarchical_surrogate_impl(ctx, labels, nx, ny, nz, labels_on_device, phases, nphase, n_sub, pad,
                                         ctx->sur_a, ctx->sur_b, ctx->sur_spread, ctx->sur_bound, o, C_out, C_sub,
                                         nullptr, report);
    }
    if (!labels || !C_out) fail(ctx, HH_EINVAL, "labels and C_out are required");
    if (nx < 1 || ny < 1 || nz < 1 || n_sub < 1) fail(ctx, HH_EINVAL, "sizes must be positive");
    if (nx % n_sub || ny % n_sub || nz % n_sub) fail(ctx, HH_EINVAL, "the subimage size must divide the image size");
    if (pad < 0 || 2 * pad >= std::min(nx, std::min(ny, nz)))
      fail(ctx, HH_EINVAL, "padding must satisfy 0 <= 2 pad < image size");
    const int b = n_sub + 2 * pad;
    const int mx = nx / n_sub, my = ny / n_sub, mz = nz / n_sub;
    check_shape(ctx, b, b, b, o.precision);
    // one subimage: the intermediate image is a single voxel, whose solve is the identity
    const bool single = mx == 1 && my == 1 && mz == 1;
    if (!single) check_shape(ctx, mx, my, mz, o.precision);
    check_phases(ctx, phases, nphase);
    const long long nvox = (long long)nx * ny * nz;
    const int nitems = mx * my * mz;
    begin_report(ctx, report);
    const unsigned char* d_img =
        device_labels(ctx, labels, nvox, labels_on_device != 0, {0}, {nvox}, {nphase}, "image");
    const long long box = (long long)b * b * b;
    auto* d_pack = static_cast<unsigned char*>(ws(ctx, "pack", size_t(box * nitems)));
    Profile prof{ctx, o.profile != 0, {}, 0, report};
    prof.run(HH_K_SETUP, [&] { launch_gather_pad(d_img, nx, ny, nz, n_sub, pad, d_pack, ctx->stream); });
    HIPCHK(hipGetLastError());
    std::vector<Item> items(nitems);
    for (int i = 0; i < nitems; ++i) {
      Item& it = items[i];
      it.nx = it.ny = it.nz = b;
      it.lab_off = box * i;
      it.cf_off = -1;
      const int r[6] = {pad, pad, pad, pad + n_sub, pad + n_sub, pad + n_sub};
      std::memcpy(it.region, r, sizeof(r));
      it.phases.assign(phases, phases + nphase);
    }
    double L[6][6];
    unit_loads(L);
    void* cf = ws(ctx, "cfield", size_t(nitems) * 21 * (o.precision == 0 ? 4 : 8));
    GroupResult r1 = solve_group_retry(ctx, items, d_pack, nullptr, false, o, L, prof, cf, main_lane(ctx), 1);
    int rc = HH_OK;
    for (int i = 0; i < nitems; ++i) rc = worse(rc, r1.status[i]);
    if (C_sub) {
      for (int i = 0; i < nitems; ++i) {
        const double* S = r1.C72.data() + size_t(i) * 72 + 36;
        int k = 0;
        for (int p = 0; p < 6; ++p)
          for (int q = p; q < 6; ++q) C_sub[size_t(i) * 21 + k++] = S[p * 6 + q];
      }
    }
    if (single) {
      end_report(ctx, report);
      const double* S = r1.C72.data() + 36;
      for (int i = 0; i < 36; ++i) C_out[i] = S[i];
      if (report) {
        report->voxel_iters = r1.voxel_iters;
        report->items = nitems;
        report->status = rc;
      }
      return rc;
    }
    Item l2;
    l2.nx = mx;
    l2.ny = my;
    l2.nz = mz;
    l2.lab_off = 0;
    l2.cf_off = 0;
    const int whole[6] = {0, 0, 0, mx, my, mz};
    std::memcpy(l2.region, whole, sizeof(l2.region));
    l2.phases.assign(1, hh_phase{1.0, 1.0});
    GroupResult r2 = solve_group(ctx, {l2}, nullptr, cf, true, o, L, prof, nullptr, main_lane(ctx), 1);
    end_report(ctx, report);
    write_C(r2, 0, C_out, nullptr);
    rc = worse(rc, r2.status[0]);
    if (report) {
      fill_item_report(report, r2, 0);
      report->voxel_iters = r1.voxel_iters + r2.voxel_iters;
      report->items = nitems;
      report->status = rc;
    }
    return rc;
  });
}

int hh_hierarchical_levels(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device,
                           const hh_phase* phases, int nphase, const int* n_sub, const int* pad, int nlevels,
                           const hh_opts* opts, double C_out[36], hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    if (!labels || !C_out || !n_sub || !pad) fail(ctx, HH_EINVAL, "labels, n_sub, pad and C_out are required");
    if (nlevels < 1 || nlevels > 8) fail(ctx, HH_EINVAL, "nlevels must be in 1..8");
    if (nx < 1 || ny < 1 || nz < 1) fail(ctx, HH_EINVAL, "sizes must be positive");
    // the chain of images: level l cuts (dx, dy, dz) into n_sub[l]^3 blocks
    int d[3] = {nx, ny, nz};
    for (int l = 0; l < nlevels; ++l) {
      const int n = n_sub[l], p = pad[l];
      if (n < 1) fail(ctx, HH_EINVAL, "block sizes must be positive");
      if (d[0] % n || d[1] % n || d[2] % n)
        fail(ctx, HH_EINVAL, "block size " + std::to_string(n) + " of level " + std::to_string(l + 1) +
                                 " does not divide its image");
      if (p < 0 || 2 * p >= std::min(d[0], std::min(d[1], d[2])))
        fail(ctx, HH_EINVAL, "padding must satisfy 0 <= 2 pad < image size at every level");
      check_shape(ctx, n + 2 * p, n + 2 * p, n + 2 * p, o.precision);
      for (int& e : d) e /= n;
    }
    const bool single = d[0] == 1 && d[1] == 1 && d[2] == 1;
    if (!single) check_shape(ctx, d[0], d[1], d[2], o.precision);
    check_phases(ctx, phases, nphase);
    const size_t tb = o.precision == 0 ? 4 : 8;
    begin_report(ctx, report);
    Profile prof{ctx, o.profile != 0, {}, 0, report};
    double L[6][6];
    unit_loads(L);
    // level 1: the label image
    const int n1 = n_sub[0], p1 = pad[0], b1 = n1 + 2 * p1;
    int mx = nx / n1, my = ny / n1, mz = nz / n1;
    const int items1 = mx * my * mz;
    const long long nvox = (long long)nx * ny * nz;
    const unsigned char* d_img =
        device_labels(ctx, labels, nvox, labels_on_device != 0, {0}, {nvox}, {nphase}, "image");
    const long long box1 = (long long)b1 * b1 * b1;
    auto* d_pack = static_cast<unsigned char*>(ws(ctx, "pack", size_t(box1 * items1)));
    prof.run(HH_K_SETUP, [&] { launch_gather_pad(d_img, nx, ny, nz, n1, p1, d_pack, ctx->stream); });
    HIPCHK(hipGetLastError());
    std::vector<Item> items(items1);
    for (int i = 0; i < items1; ++i) {
      Item& it = items[i];
      it.nx = it.ny = it.nz = b1;
      it.lab_off = box1 * i;
      it.cf_off = -1;
      const int r[6] = {p1, p1, p1, p1 + n1, p1 + n1, p1 + n1};
      std::memcpy(it.region, r, sizeof(r));
      it.phases.assign(phases, phases + nphase);
    }
    const char* names[2] = {"levels_cf0", "levels_cf1"};
    void* cf = ws(ctx, names[0], size_t(items1) * 21 * tb);
    GroupResult last = solve_group_retry(ctx, items, d_pack, nullptr, false, o, L, prof, cf, main_lane(ctx), 1);
    int rc = HH_OK;
    for (int st : last.status) rc = worse(rc, st);
    double vi = last.voxel_iters;
    // further levels: blocks of the intermediate image with anisotropic voxels
    for (int l = 1; l < nlevels; ++l) {
      const int n = n_sub[l], p = pad[l], b = n + 2 * p;
      const int nit = (mx / n) * (my / n) * (mz / n);
      const long long box = (long long)b * b * b;
      void* pack = ws(ctx, "levels_pack", size_t(nit) * size_t(box) * 21 * tb);
      prof.run(HH_K_SETUP, [&] { launch_gather_field(o.precision, cf, mx, my, mz, n, p, pack, ctx->stream); });
      HIPCHK(hipGetLastError());
      std::vector<Item> lv(nit);
      for (int i = 0; i < nit; ++i) {
        Item& it = lv[i];
        it.nx = it.ny = it.nz = b;
        it.lab_off = 0;
        it.cf_off = box * 21 * i;
        const int r[6] = {p, p, p, p + n, p + n, p + n};
        std::memcpy(it.region, r, sizeof(r));
        it.phases.assign(1, hh_phase{1.0, 1.0});
      }
      void* next = ws(ctx, names[l % 2], size_t(nit) * 21 * tb);
      last = solve_group(ctx, lv, nullptr, pack, true, o, L, prof, next, main_lane(ctx), 1);
      for (int st : last.status) rc = worse(rc, st);
      vi += last.voxel_iters;
      cf = next;
      mx /= n;
      my /= n;
      mz /= n;
    }
    if (single) {
      end_report(ctx, report);
      write_C(last, 0, C_out, nullptr);
    } else {
      Item fin;
      fin.nx = mx;
      fin.ny = my;
      fin.nz = mz;
      fin.lab_off = 0;
      fin.cf_off = 0;
      const int whole[6] = {0, 0, 0, mx, my, mz};
      std::memcpy(fin.region, whole, sizeof(fin.region));
      fin.phases.assign(1, hh_phase{1.0, 1.0});
      last = solve_group(ctx, {fin}, nullptr, cf, true, o, L, prof, nullptr, main_lane(ctx), 1);
      end_report(ctx, report);
      write_C(last, 0, C_out, nullptr);
      rc = worse(rc, last.status[0]);
      vi += last.voxel_iters;
    }
    if (report) {
      fill_item_report(report, last, 0);
      report->voxel_iters = vi;
      report->items = items1;
      report->status = rc;
    }
    return rc;
  });
}

int hh_gather_subimages(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device, int n_sub,
                        int pad, uint8_t* pack_device) {
  return guarded(ctx, [&]() -> int {
    if (!labels || !pack_device) fail(ctx, HH_EINVAL, "labels and pack_device are required");
    if (nx < 1 || ny < 1 || nz < 1 || n_sub < 1) fail(ctx, HH_EINVAL, "sizes must be positive");
    if (nx % n_sub || ny % n_sub || nz % n_sub) fail(ctx, HH_EINVAL, "the subimage size must divide the image size");
    if (pad < 0 || 2 * pad >= std::min(nx, std::min(ny, nz)))
      fail(ctx, HH_EINVAL, "padding must satisfy 0 <= 2 pad < image size");
    const long long nvox = (long long)nx * ny * nz;
    const unsigned char* d = labels;
    if (!labels_on_device) {
      auto* buf = static_cast<unsigned char*>(ws(ctx, "image", size_t(nvox)));
      HIPCHK(hipMemcpyAsync(buf, labels, size_t(nvox), hipMemcpyHostToDevice, ctx->stream));
      d = buf;
    }
    launch_gather_pad(d, nx, ny, nz, n_sub, pad, pack_device, ctx->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HH_OK;
  });
}

int hh_hierarchical_surrogate(hh_ctx* ctx, const uint8_t* labels, int nx, int ny, int nz, int labels_on_device,
                              const hh_phase* phases, int nphase, int n_sub, int pad, hh_net* net_a, hh_net* net_b,
                              double spread_tol, double bound_tol, const hh_opts* opts, double C_out[36],
                              double* C_sub, int* fallback, hh_report* report) {
  return guarded(ctx, [&]() -> int {
    hh_opts o;
    hh_default_opts(&o);
    if (opts) o = *opts;
    check_opts(ctx, o);
    return hierarchical_surrogate_impl(ctx, labels, nx, ny, nz, labels_on_device, phases, nphase, n_sub, pad, net_a,
                                       net_b, spread_tol, bound_tol, o, C_out, C_sub, fallback, report);
  });
}

int hh_plan_cache(hh_ctx* ctx, const char* path) {
  return guarded(ctx, [&]() -> int {
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->plan_file = path ? path : "";
    if (!path) return HH_OK;
    FILE* f = std::fopen(path, "r");
    if (!f) return HH_OK;  // created by the first tuned shape
    char tag[64], arch[64], ver[16];
    int v[11];
    int loaded = 0;
    while (std::fscanf(f, "%63s %63s %15s %d %d %d %d %d %d %d %d %d", tag, arch, ver, &v[0], &v[1], &v[2], &v[3],
                       &v[4], &v[5], &v[6], &v[7], &v[8]) == 12) {
      if (std::strcmp(tag, "hh-plan") != 0 || ctx->arch != arch || std::strcmp(ver, kPlanTag) != 0) continue;
      bool ok = true;
      for (int i = 6; i < 9; ++i) ok = ok && v[i] >= 0 && v[i] < kNVariant;
      if (!ok) continue;
      ctx->plans[std::array<int, 6>{{v[0], v[1], v[2], v[3], v[4], v[5]}}] = {{v[6], v[7], v[8]}};
      ++loaded;
    }
    std::fclose(f);
    (void)loaded;
    return HH_OK;
  });
}

int hh_set_surrogate(hh_ctx* ctx, hh_net* net_a, hh_net* net_b, double spread_tol, double bound_tol) {
  return guarded(ctx, [&]() -> int {
    if (!net_a && net_b) fail(ctx, HH_EINVAL, "net_b needs net_a");
    if (net_a && (!(spread_tol > 0.0) || !(bound_tol >= 0.0))) fail(ctx, HH_EINVAL, "bad gate tolerances");
    ctx->sur_a = net_a;
    ctx->sur_b = net_b;
    ctx->sur_spread = spread_tol;
    ctx->sur_bound = bound_tol;
    return HH_OK;
  });
}

int hh_richardson(const int* n, const double* C, int m, double C_inf[36], double slope[36]) {
  if (!n || !C || !C_inf || m < 2) return HH_EINVAL;
  // least squares of v = a + b / n over the m sizes, per entry
  double s1 = 0, sx = 0, sxx = 0;
  for (int i = 0; i < m; ++i) {
    if (n[i] <= 0) return HH_EINVAL;
    const double x = 1.0 / n[i];
    s1 += 1;
    sx += x;
    sxx += x * x;
  }
  const double det = s1 * sxx - sx * sx;
  if (!(std::fabs(det) > 1e-300 * std::max(1.0, sxx))) return HH_EINVAL;
  for (int k = 0; k < 36; ++k) {
    double sy = 0, sxy = 0;
    for (int i = 0; i < m; ++i) {
      const double x = 1.0 / n[i], y = C[size_t(i) * 36 + k];
      sy += y;
      sxy += x * y;
    }
    const double a = (sxx * sy - sx * sxy) / det;
    const double b = (s1 * sxy - sx * sy) / det;
    C_inf[k] = a;
    if (slope) slope[k] = b;
  }
  return HH_OK;
}

int hh_moduli(const double C[36], double* K, double* G) {
  if (!C || !K || !G) return HH_EINVAL;
  const double d = C[0] + C[7] + C[14];
  const double o = C[1] + C[2] + C[8];
  const double s = C[21] + C[28] + C[35];
  *K = (d + 2.0 * o) / 9.0;
  *G = (d - o + 3.0 * s) / 15.0;
  return HH_OK;
}

int hh_mean_moduli(const double* C_sub, long long m, double* K, double* G) {
  if (!C_sub || !K || !G || m < 1) return HH_EINVAL;
  // upper-triangle index of (i, j), i <= j, row-major
  auto at = [](int i, int j) { return i * 6 - i * (i - 1) / 2 + (j - i); };
  double sk = 0.0, sg = 0.0;
  for (long long q = 0; q < m; ++q) {
    const double* c = C_sub + q * 21;
    const double d = c[at(0, 0)] + c[at(1, 1)] + c[at(2, 2)];
    const double o = c[at(0, 1)] + c[at(0, 2)] + c[at(1, 2)];
    const double s = c[at(3, 3)] + c[at(4, 4)] + c[at(5, 5)];
    sk += (d + 2.0 * o) / 9.0;
    sg += (d - o + 3.0 * s) / 15.0;
  }
  *K = sk / double(m);
  *G = sg / double(m);
  return HH_OK;
}

}  // extern "C"
