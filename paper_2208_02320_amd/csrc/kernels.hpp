// Launch interface between the host orchestration and the pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "hh_internal.hpp"

namespace hh {

enum : int { kZInvCg = 0, kZFwdCg = 1, kZFwdRhs = 2, kZInvFp = 3, kZFwdFp = 4 };
enum : int { kXCg = 0, kXRhs = 1, kXFp = 2 };
enum : int {
  kOpZ = 0,
  kOpY = 1,
  kOpX = 2,
  kOpInfoZ = 3,
  kOpInfoX = 4,
  kOpInfoLdsZ = 5,
  kOpInfoLdsX = 6,
  kOpInfoThreadsZ = 7,
  kOpInfoThreadsX = 8
};
// Number of compiled tile variants per FP32 size (see variant_budget).
constexpr int kNVariant = 5;

using SizeOpsFn = void (*)(int what, int mode, const GroupArgs* g, hipStream_t st, int* info);

SizeOpsFn size_ops(int n, int precision, int variant = 0);
// per-file size tables (sizes_f32_*.hip, sizes_f64_*.hip)
SizeOpsFn size_ops_f32_0(int n, int v);
SizeOpsFn size_ops_f32_1(int n, int v);
SizeOpsFn size_ops_f32_2(int n, int v);
SizeOpsFn size_ops_f32_3(int n, int v);
SizeOpsFn size_ops_f32_4(int n, int v);
SizeOpsFn size_ops_f32_5(int n, int v);
SizeOpsFn size_ops_f32_6(int n, int v);
SizeOpsFn size_ops_f32_7(int n, int v);
SizeOpsFn size_ops_f32_8(int n, int v);
SizeOpsFn size_ops_f32_9(int n, int v);
SizeOpsFn size_ops_f32_10(int n, int v);
SizeOpsFn size_ops_f32_11(int n, int v);
SizeOpsFn size_ops_f32_12(int n, int v);
SizeOpsFn size_ops_f32_13(int n, int v);
SizeOpsFn size_ops_f32_14(int n, int v);
SizeOpsFn size_ops_f32_15(int n, int v);
SizeOpsFn size_ops_f32_16(int n, int v);
SizeOpsFn size_ops_f32_17(int n, int v);
SizeOpsFn size_ops_f32_18(int n, int v);
SizeOpsFn size_ops_f32_19(int n, int v);
SizeOpsFn size_ops_f32_20(int n, int v);
SizeOpsFn size_ops_f32_21(int n, int v);
SizeOpsFn size_ops_f32_22(int n, int v);
SizeOpsFn size_ops_f32_23(int n, int v);
SizeOpsFn size_ops_f32_24(int n, int v);
SizeOpsFn size_ops_f32_25(int n, int v);
SizeOpsFn size_ops_f32_26(int n, int v);
SizeOpsFn size_ops_f32_27(int n, int v);
SizeOpsFn size_ops_f32_28(int n, int v);
SizeOpsFn size_ops_f64_0(int n, int v);
SizeOpsFn size_ops_f64_1(int n, int v);
SizeOpsFn size_ops_f64_2(int n, int v);
SizeOpsFn size_ops_f64_3(int n, int v);
SizeOpsFn size_ops_f64_4(int n, int v);
SizeOpsFn size_ops_f64_5(int n, int v);
SizeOpsFn size_ops_f64_6(int n, int v);
void launch_fin_x(int mode, const GroupArgs& g, hipStream_t st);
void launch_fin_z(int mode, const GroupArgs& g, hipStream_t st);
void launch_stiffness(int precision, const SysState* state, int nitems, double* out, void* cfield_out,
                      int* status_out, hipStream_t st);

void launch_gather_pad(const unsigned char* img, int nx, int ny, int nz, int n, int p, unsigned char* out,
                       hipStream_t st);
// Boxes (n + 2p)^3 of the (mz, my, mx) image of 21-component stiffnesses
// (FP32 or FP64) around each n^3 block, wrapped: out[item][box voxel][21].
void launch_gather_field(int precision, const void* src, int mx, int my, int mz, int n, int p, void* out,
                         hipStream_t st);
void launch_label_max(const unsigned char* labels, const long long* off, const long long* count, int nitems,
                      long long max_count, int* out, hipStream_t st);
void launch_count_running(const SysState* st, int n, int* count, hipStream_t s);
void launch_convert_field(int precision, const double* src, void* dst, long long n, hipStream_t st);

}  // namespace hh
