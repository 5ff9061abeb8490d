// 3-D CNN surrogate of the subimage stiffness: one-hot phase labels of a
// subimage -> its 21 stiffness components.  Inference and training kernels
// on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32 accumulation.
//
// Network (all convolutions 3x3x3, stride 2, zero padding 1, bias, ReLU):
//   one-hot [P <= 8 channels, padded to 8] n^3 -> 32 ch (n/2)^3 -> 32 ch (n/4)^3
//   -> 64 ch (n/8)^3 -> 64 ch (n/16)^3 -> global mean (64 features), plus the
//   window's 8 standardized phase fractions (a skip path from the input) ->
//   linear 72 -> 21.
// Activations are channels-last BF16 [b][z][y][x][c]; activation gradients
// FP32; parameters FP32 master copies with BF16 working copies [tap][cout][cin]
// (forward) and [tap][cin][cout] (data gradient).
//
// A convolution is an implicit GEMM (M = output voxels, N = output channels,
// K = 27 taps x input channels).  MFMA operand layout for 16x16x32 BF16:
// lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16],
// j = 0..7, and D[4 (l / 16) + i][l % 16], i = 0..3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <string>
#include <vector>

#include "cnn.hpp"
#include "intdiv.hpp"

#pragma once

namespace hh {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
  return z;
}

// 16-byte load of 8 consecutive bf16
__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// ---------------------------------------------------------------------------
// The network input, one n^3 window of uint8 labels per item, in one of two
// layouts:
//   box mode: the window at (o, o, o) of each of the label boxes of edge
//     `box`, `stride` bytes apart (rows box bytes apart, planes box^2);
//   image mode (mx > 0): item item0 + b is the n^3 block (bz, by, bx) of one
//     image with rows `row` and planes `plane` bytes apart, where
//     item0 + b = (bz my + by) mx + bx.
// The first layer reads the labels and forms their one-hot code in registers.
// Only the label and interface counts and the LDS-staged first layer
// (k_conv_fwd_rows4s) take image windows; every reader uses row and plane.
// ---------------------------------------------------------------------------
struct LabelWindow {
  const unsigned char* labels;
  long long stride;      // box mode: bytes from one box to the next
  int box, o;            // box mode: box edge and the window's offset in it
  long long row, plane;  // bytes between window rows and between window planes
  int mx, my, n, item0;  // image mode: blocks per row and column, block edge, first item
};
__host__ inline LabelWindow box_window(const unsigned char* labels, long long stride, int box, int o) {
  return LabelWindow{labels, stride, box, o, box, (long long)box * box, 0, 0, 0, 0};
}
__host__ inline LabelWindow image_window(const unsigned char* img, int nx, int ny, int n, int item0) {
  return LabelWindow{img, 0, 0, 0, nx, (long long)nx * ny, nx / n, ny / n, n, item0};
}


// Output voxel v (< Do^3) of one item -> (oz, oy, ox).
struct Grid3 {
  int D, D2;         // edge and edge^2
  float inv, inv2;   // their reciprocals
};
__host__ inline Grid3 make_grid3(int D) { return Grid3{D, D * D, 1.0f / float(D), 1.0f / float(D * D)}; }
__device__ __forceinline__ void split3(const Grid3& g, int v, int& z, int& y, int& x) {
  z = fdiv(v, g.D2, g.inv2);
  const int r = v - z * g.D2;
  y = fdiv(r, g.D, g.inv);
  x = r - y * g.D;
}

// labels of item b as a base pointer at its window's origin
__host__ __device__ __forceinline__ const unsigned char* window_base(const LabelWindow& w, int b) {
  if (w.mx > 0) {
    const int i = w.item0 + b, bx = i % w.mx, by = (i / w.mx) % w.my, bz = i / (w.mx * w.my);
    return w.labels + (long long)bz * w.n * w.plane + (long long)by * w.n * w.row + (long long)bx * w.n;
  }
  return w.labels + (long long)b * w.stride + w.o * w.plane + w.o * w.row + w.o;
}

typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
// one-hot code of a label over 4 channels (the zero code for 4 and above)
__device__ __forceinline__ bf16x4v onehot4(int lab) {
  bf16x4v h;
#pragma unroll
  for (int c = 0; c < 4; ++c) h[c] = (__bf16)(c == lab ? 1.0f : 0.0f);
  return h;
}

__device__ __forceinline__ bf16x8 onehot8(int lab) {
  bf16x8 h;
#pragma unroll
  for (int c = 0; c < 8; ++c) h[c] = (__bf16)(c == lab ? 1.0f : 0.0f);
  return h;
}

// Label counts of each window: cnt[b][c] += number of voxels with label c
// (c < 8).  Grid (row blocks, batch).  The block's window rows are cut into
// W-byte chunks (cw per row; the launcher picks W so that every chunk is an
// aligned word).  Per chunk, each label adds 1 to its 4-bit field of a word
// (label 8 and above shift out of it); the fields then go to two words of
// byte counters (even and odd labels).  The launcher bounds the bytes per
// thread by count_rows_per_block, so no byte counter overflows.  Wave sums
// in 16-bit fields, then one atomic per block and label.
inline int count_rows_per_block(int n) {
  const int r = 61440 / n;  // at most 240 + W bytes per thread
  return r < 1 ? 1 : (r > n * n ? n * n : r);
}

// Per chunk, each label adds 1 to its 4-bit field (labels 8 and above shift
// out); the fields go to byte counters of the even and odd labels.
template <int W, class CT>
__device__ __forceinline__ void count_chunk(const CT& v, unsigned& ev, unsigned& od) {
  unsigned nib = 0u;
#pragma unroll
  for (int j = 0; j < W; ++j) nib += unsigned(1ull << (4u * min(chunk_byte(v, j), 8u)));
  ev += nib & 0x0F0F0F0Fu;
  od += (nib >> 4) & 0x0F0F0F0Fu;
}

// The block's byte counters summed into cnt8[0..8): wave sums in 16-bit
// fields, then one atomic per block and label.  Every thread of the block
// takes part.
__device__ __forceinline__ void flush_counts(unsigned ev, unsigned od, int* __restrict__ cnt8) {
  const int lane = threadIdx.x & 63;
  // 16-bit fields: (0, 1), (2, 3), (4, 5), (6, 7)
  unsigned pr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) pr[i] = ((ev >> (8 * i)) & 0xFFu) | (((od >> (8 * i)) & 0xFFu) << 16);
  __shared__ int s[8];
  if (threadIdx.x < 8) s[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    unsigned v = pr[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) {
      if (v & 0xFFFFu) atomicAdd(&s[2 * i], int(v & 0xFFFFu));
      if (v >> 16) atomicAdd(&s[2 * i + 1], int(v >> 16));
    }
  }
  __syncthreads();
  if (threadIdx.x < 8 && s[threadIdx.x]) atomicAdd(&cnt8[threadIdx.x], s[threadIdx.x]);
}

template <int W>
__global__ void __launch_bounds__(256) k_count_labels(LabelWindow w, int n, float inv_n, int cw, float inv_cw,
                                                      int rows, int item0, int* __restrict__ cnt) {
  using CT = typename Chunk<W>::type;
  const int b = item0 + blockIdx.y;
  const int r0 = blockIdx.x * rows, nr = min(rows, n * n - r0);
  const unsigned char* base = window_base(w, b);
  const int tasks = nr * cw;
  unsigned ev = 0u, od = 0u;  // byte counters of labels 0 2 4 6 and 1 3 5 7
  for (int t = threadIdx.x; t < tasks; t += 256) {
    const int rl = fdiv(t, cw, inv_cw), k = t - rl * cw;
    const int r = r0 + rl, z = fdiv(r, n, inv_n), y = r - z * n;
    count_chunk<W>(*reinterpret_cast<const CT*>(base + z * w.plane + y * w.row + k * W), ev, od);
  }
  flush_counts(ev, od, cnt + b * 8);
}

// cnt[item0 .. item0 + nitems) += label counts of the n^3 windows of lw
// (items item0 ...); the caller zeroes cnt.
inline void launch_count_labels(const LabelWindow& lw, int n, int item0, int nitems, int* cnt, hipStream_t st) {
  const unsigned char* first = window_base(lw, 0);
  const int W = chunk_width({lw.mx > 0 ? (long long)n : lw.stride, lw.row, lw.plane, (long long)n}, first, first);
  const int cw = n / W, rows = count_rows_per_block(n);
  const unsigned gx = unsigned((n * n + rows - 1) / rows);
  const float inv_n = 1.0f / float(n), inv_cw = 1.0f / float(cw);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    const int ni = nitems - i0 < 65535 ? nitems - i0 : 65535;
    const dim3 g(gx, unsigned(ni));
    if (W == 8)
      k_count_labels<8><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt);
    else if (W == 4)
      k_count_labels<4><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt);
    else
      k_count_labels<1><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt);
  }
}

// Number of nonzero bytes of a 64-bit word.
__device__ __forceinline__ unsigned nonzero_bytes(unsigned long long d) {
  d |= d >> 4;
  d |= d >> 2;
  d |= d >> 1;
  return unsigned(__popcll(d & 0x0101010101010101ull));
}

// Interface counts of each window: cnt[b] += number of face-adjacent voxel
// pairs inside the n^3 window (along x, y and z) whose labels differ.  Same
// grid and W-byte chunks as k_count_labels; a chunk is compared byte by
// byte with itself shifted by one voxel in x (and the first voxel of the
// next chunk), with the chunk one row up in y and one plane up in z.  Wave
// sums, then one atomic per block.
// LABELS: the same pass also adds the windows' label counts to lcnt[b][8]
// (as k_count_labels, whose grid and chunks it shares).
template <int W, bool LABELS = false>
__global__ void __launch_bounds__(256) k_count_interfaces(LabelWindow w, int n, float inv_n, int cw, float inv_cw,
                                                          int rows, int item0, unsigned* __restrict__ cnt,
                                                          int* __restrict__ lcnt) {
  using CT = typename Chunk<W>::type;
  const int b = item0 + blockIdx.y;
  const int r0 = blockIdx.x * rows, nr = min(rows, n * n - r0);
  const unsigned char* base = window_base(w, b);
  const int tasks = nr * cw;
  const long long plane = w.plane;
  unsigned c = 0u;
  unsigned ev = 0u, od = 0u;  // label byte counters (LABELS)
  for (int t = threadIdx.x; t < tasks; t += 256) {
    const int rl = fdiv(t, cw, inv_cw), k = t - rl * cw;
    const int r = r0 + rl, z = fdiv(r, n, inv_n), y = r - z * n;
    const unsigned char* p = base + z * w.plane + y * w.row + k * W;
    const CT v = *reinterpret_cast<const CT*>(p);
    if constexpr (LABELS) count_chunk<W>(v, ev, od);
    if constexpr (W == 8) {
      // whole words: bytes that differ are the nonzero bytes of an XOR
      const unsigned long long a = (unsigned long long)v.x | ((unsigned long long)v.y << 32);
      const unsigned long long nxt = k + 1 < cw ? (unsigned long long)p[W] : (a >> 56);  // no pair past the row end
      c += nonzero_bytes(a ^ ((a >> 8) | (nxt << 56)));
      if (y + 1 < n) {
        const uint2 u = *reinterpret_cast<const uint2*>(p + w.row);
        c += nonzero_bytes(a ^ ((unsigned long long)u.x | ((unsigned long long)u.y << 32)));
      }
      if (z + 1 < n) {
        const uint2 u = *reinterpret_cast<const uint2*>(p + plane);
        c += nonzero_bytes(a ^ ((unsigned long long)u.x | ((unsigned long long)u.y << 32)));
      }
    } else {
#pragma unroll
      for (int j = 0; j + 1 < W; ++j) c += chunk_byte(v, j) != chunk_byte(v, j + 1);
      if (k + 1 < cw) c += chunk_byte(v, W - 1) != unsigned(p[W]);
      if (y + 1 < n) {
        const CT u = *reinterpret_cast<const CT*>(p + w.row);
#pragma unroll
        for (int j = 0; j < W; ++j) c += chunk_byte(v, j) != chunk_byte(u, j);
      }
      if (z + 1 < n) {
        const CT u = *reinterpret_cast<const CT*>(p + plane);
#pragma unroll
        for (int j = 0; j < W; ++j) c += chunk_byte(v, j) != chunk_byte(u, j);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  __shared__ unsigned s;
  if (threadIdx.x == 0) s = 0u;
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0 && s) atomicAdd(&cnt[b], s);
  if constexpr (LABELS) flush_counts(ev, od, lcnt + b * 8);
}

// cnt[item0 .. item0 + nitems) += interface counts of the n^3 windows of lw
// (items item0 ...), and with lcnt the label counts as well ([item][8]); the
// caller zeroes both.
inline void launch_count_interfaces(const LabelWindow& lw, int n, int item0, int nitems, unsigned* cnt,
                                    hipStream_t st, int* lcnt = nullptr) {
  const unsigned char* first = window_base(lw, 0);
  const int W = chunk_width({lw.mx > 0 ? (long long)n : lw.stride, lw.row, lw.plane, (long long)n}, first, first);
  const int cw = n / W, rows = count_rows_per_block(n);
  const unsigned gx = unsigned((n * n + rows - 1) / rows);
  const float inv_n = 1.0f / float(n), inv_cw = 1.0f / float(cw);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    const int ni = nitems - i0 < 65535 ? nitems - i0 : 65535;
    const dim3 g(gx, unsigned(ni));
    if (lcnt) {
      if (W == 8)
        k_count_interfaces<8, true><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, lcnt);
      else if (W == 4)
        k_count_interfaces<4, true><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, lcnt);
      else
        k_count_interfaces<1, true><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, lcnt);
    } else if (W == 8) {
      k_count_interfaces<8><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, nullptr);
    } else if (W == 4) {
      k_count_interfaces<4><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, nullptr);
    } else {
      k_count_interfaces<1><<<g, 256, 0, st>>>(lw, n, inv_n, cw, inv_cw, rows, item0 + i0, cnt, nullptr);
    }
  }
}

__global__ void k_zero_int(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// forward convolution + bias + ReLU.  256 threads = 4 waves; each wave
// computes RB row blocks of 16 output voxels x COUT channels, so that every
// B fragment (weights) it loads serves RB MFMAs.  X: [b][D^3][CIN] (or, with
// LAB, the label window, CIN = 8), Y: [b][Do^3][COUT].
// ---------------------------------------------------------------------------
// v of lane l - 1 within each row of 16 lanes (DPP row shift right by one);
// the first lane of a row gets zero
__device__ __forceinline__ bf16x8 from_left_lane(bf16x8 v) {
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x4 u = __builtin_bit_cast(i32x4, v);
  i32x4 o;
#pragma unroll
  for (int j = 0; j < 4; ++j) o[j] = __builtin_amdgcn_update_dpp(0, u[j], 0x111, 0xF, 0xF, false);
  return __builtin_bit_cast(bf16x8, o);
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
// BF16 and ReLU of four output channels.  The ReLU acts on the BF16 bit
// patterns: a value with its sign bit set is a negative 16-bit integer, so a
// packed integer max with 0 clears it (rounding keeps the sign, so this
// equals rounding after the ReLU)
__device__ __forceinline__ bf16x4 relu4(const f32x4& a) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef short i16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 lo = __builtin_convertvector(f32x2{a[0], a[1]}, bf16x2);
  const bf16x2 hi = __builtin_convertvector(f32x2{a[2], a[3]}, bf16x2);
  const i16x2 l = __builtin_elementwise_max(__builtin_bit_cast(i16x2, lo), i16x2{0, 0});
  const i16x2 h = __builtin_elementwise_max(__builtin_bit_cast(i16x2, hi), i16x2{0, 0});
  const bf16x2 lr = __builtin_bit_cast(bf16x2, l), hr = __builtin_bit_cast(bf16x2, h);
  return bf16x4{lr[0], lr[1], hr[0], hr[1]};
}
// bias, BF16 and ReLU
__device__ __forceinline__ bf16x4 bias_relu4(const f32x4& a, const float4& bb) {
  return relu4(f32x4{a[0] + bb.x, a[1] + bb.y, a[2] + bb.z, a[3] + bb.w});
}

// A wave's RB x NT accumulator tiles (D = W x X^T, so lane l holds channels
// t 16 + 4 (l / 16) + i of voxel v0 + 16 r + l % 16) with bias and ReLU,
// written to Yb ([nvo][COUT], one item) through the wave's LDS tile so ([VW][COUT])
// as whole 16-byte chunks: the wave's VW = 16 RB voxels are consecutive.
// In the tile, 16-byte chunk j of voxel v sits at chunk j ^ ((v / 4) % CV)
// of its row (CV chunks per voxel): the 16 lanes of a row block, whose
// voxels' rows lie 64 bytes apart, then write 16 different banks.
// ADD_BIAS false: the accumulators already hold the bias (bias unused).
template <int RB, int NT, int COUT, bool ADD_BIAS = true>
__device__ __forceinline__ void store_staged(const f32x4 (&acc)[RB][NT], const float* __restrict__ bias, __bf16* so,
                                             __bf16* __restrict__ Yb, int nvo, int v0, int lane) {
  constexpr int VW = 16 * RB, CV = COUT / 8;  // chunks per voxel
  static_assert((CV & (CV - 1)) == 0, "chunks per voxel: a power of two");
  const int q = lane >> 4, l = lane & 15;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + 4 * q;  // four channels: half (co / 4) % 2 of chunk co / 8
    float4 bb = float4{0.f, 0.f, 0.f, 0.f};
    if constexpr (ADD_BIAS) bb = *reinterpret_cast<const float4*>(bias + co);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int v = r * 16 + l;
      const int sw = ((co / 8) ^ ((v >> 2) & (CV - 1))) * 8 + (co & 7);
      *reinterpret_cast<bf16x4*>(so + v * COUT + sw) = ADD_BIAS ? bias_relu4(acc[r][t], bb) : relu4(acc[r][t]);
    }
  }
  __syncthreads();
  constexpr int CH = VW * CV;         // chunks per wave
  const int nv = min(VW, nvo - v0);  // valid voxels of this wave (may be <= 0)
  uint4* dst = reinterpret_cast<uint4*>(Yb + (long long)v0 * COUT);
  const uint4* src = reinterpret_cast<const uint4*>(so);
#pragma unroll
  for (int c = lane; c < CH; c += 64) {
    const int v = c / CV, j = c % CV;
    if (c * 16 < nv * COUT * 2) dst[c] = src[v * CV + (j ^ ((v >> 2) & (CV - 1)))];
  }
}

// XS (x shift; CIN = 32, output rows of at most 16 voxels that tile the 16
// lanes of a row block): the taps come in (tz, ty) groups of three.  A lane
// loads its voxel's inputs at x = 2 ox (tx = 1) and 2 ox + 1 (tx = 2); the
// input at x = 2 ox - 1 (tx = 0) is the tx = 2 input of the lane on its left,
// taken across the row with a DPP shift (zero padding at ox = 0).  Two loads
// per three taps instead of three.
// YR (with XS; output rows of 16 voxels, RB = 4): a wave's four row blocks
// are four consecutive output rows of one slice, so the ty = 0 inputs of row
// block r are the ty = 2 inputs of row block r - 1, already in registers: 18
// loads per tz instead of 24.
// WPB (with XS): waves per workgroup; above 4, the layer's weights
// (27 x COUT x 32 BF16: 55 KB at COUT = 32, 110 KB at 64) are staged once
// per workgroup in LDS as MFMA fragments instead of every wave streaming them
// from L2 (8 waves for the second layer, two workgroups per CU; 16 for the
// third, one).
// LAB with CIN = 4 (networks of at most four phases): a lane's eight K values
// are the four channels of two consecutive taps, so K = 27 x 4 takes 4 k-steps
// instead of 7; W is then laid out [tap pair][COUT][8] (k_cast_pairs4).
// The 32-channel-input layers are asked to fit four waves per SIMD: the
// compiler then keeps the accumulators in VGPRs (the second layer: 119
// registers against 136 with AGPRs, three waves per SIMD), with no spills.
template <int CIN, int COUT, bool LAB, int RB, bool XS = false, bool YR = false, int WPB = 4>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu((CIN == 32 && !LAB) ? 4 : 1))) k_conv_fwd(const __bf16* __restrict__ X, LabelWindow lw,
                                                  const __bf16* __restrict__ W, const float* __restrict__ bias,
                                                  __bf16* __restrict__ Y, int D, Grid3 go) {
  static_assert((LAB ? (CIN == 8 || CIN == 4) : CIN % 8 == 0) && COUT % 16 == 0, "channel counts");
  constexpr bool L4 = LAB && CIN == 4;
  static_assert(!XS || (CIN == 32 && !LAB), "the x-shift path takes one tap per K step");
  static_assert(!YR || (XS && RB == 4), "row reuse: x-shift path, four row blocks");
  constexpr int KT = 27 * CIN, KS = (KT + 31) / 32, NT = COUT / 16;
  constexpr int VW = 16 * RB;  // output voxels of one wave
  // one-hot codes of labels 0..7 and a zero row (index 8) for padding and labels >= 8
  __shared__ bf16x8 sOne[9];
  __shared__ bf16x4v sOne4[5];  // four-channel codes of labels 0..3 and a zero row (index 4)
  // first layer (large output): each wave's output tile goes out through LDS
  // as whole 16-byte chunks; deeper layers store 8-byte words directly
  constexpr bool STAGE = LAB;
  __shared__ __align__(16) __bf16 sOut[STAGE ? 4 : 1][STAGE ? VW * COUT : 8];
  const int nvo = go.D2 * go.D;  // output voxels per item
  const int b = blockIdx.y;      // item
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr bool WL = WPB > 4;
  constexpr int TH = 64 * WPB;  // threads per workgroup
  const int v0 = blockIdx.x * (WPB * VW) + wave * VW;
  // WL: the weights in LDS as MFMA fragments [tap][t][q][l] (16 bytes each),
  // so that a wave's fragment read is contiguous
  constexpr int NWF = WL ? 27 * (COUT / 16) * 4 * 16 : 1;
  __shared__ bf16x8 sWf[NWF];
  if constexpr (WL) {
    static_assert(XS && CIN == 32, "weights in LDS: the x-shift path");
    constexpr int KF = (NWF + TH - 1) / TH;
    bf16x8 wv[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int e = threadIdx.x + k * TH;
      const int l = e % 16, qq = (e / 16) % 4, tt = (e / 64) % (COUT / 16), tap = e / (64 * (COUT / 16));
      if (NWF % TH == 0 || e < NWF) wv[k] = ld8(W + ((tap * COUT + tt * 16 + l) * CIN + 8 * qq));
    }
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int e = threadIdx.x + k * TH;
      if (NWF % TH == 0 || e < NWF) sWf[e] = wv[k];
    }
    __syncthreads();
  }
  if constexpr (LAB) {
    if (threadIdx.x < 9) sOne[threadIdx.x] = threadIdx.x < 8 ? onehot8(threadIdx.x) : zero8();
    if (threadIdx.x < 5) sOne4[threadIdx.x] = onehot4(threadIdx.x);
    __syncthreads();
  }
  const __bf16* Xb = LAB ? nullptr : X + (long long)b * D * D * D * CIN;
  const unsigned char* Lb = LAB ? window_base(lw, b) : nullptr;
  const int rs = LAB ? lw.box : D;  // row stride of the input, in voxels
  // per row block: offset of input corner (2o - 1) and which axes sit at o = 0
  // (their tap 0 falls in the zero padding; 2o + t - 1 never reaches D)
  int base[RB];
  unsigned lowm[RB];  // bit 0: z, 1: y, 2: x at the low edge; bit 3: voxel past the end
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int va = v0 + r * 16 + (lane & 15);
    int oz, oy, ox;
    split3(go, va < nvo ? va : 0, oz, oy, ox);
    base[r] = ((2 * oz - 1) * rs + 2 * oy - 1) * rs + 2 * ox - 1;
    lowm[r] = (oz == 0 ? 1u : 0u) | (oy == 0 ? 2u : 0u) | (ox == 0 ? 4u : 0u) | (va < nvo ? 0u : 8u);
  }
  // input of k-step ks for row block r: a zero fragment where the tap falls
  // in the padding; loads are issued without branches from a safe address
  auto tap_of = [&](int ks) { return (ks * 32 + (lane >> 4) * 8) / CIN; };
  auto tap_mask = [&](int tap) {
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
    return (tz == 0 ? 1u : 0u) | (ty == 0 ? 2u : 0u) | (tx == 0 ? 4u : 0u);
  };
  auto tap_off = [&](int tap) { return ((tap / 9) * rs + (tap / 3) % 3) * rs + tap % 3; };
  using Raw = typename std::conditional<LAB, int, bf16x8>::type;
  auto load_a = [&](int ks, int r, bool& ok) -> Raw {
    const int tap = tap_of(ks);
    if constexpr (L4) {
      // taps tap and tap + 1: both labels, each mapped to row 4 (zero) where padded
      const bool ok0 = tap < 27 && (lowm[r] & (tap_mask(tap) | 8u)) == 0u;
      const bool ok1 = tap + 1 < 27 && (lowm[r] & (tap_mask(tap + 1) | 8u)) == 0u;
      const int l0 = int(Lb[ok0 ? base[r] + tap_off(tap) : 0]);
      const int l1 = int(Lb[ok1 ? base[r] + tap_off(tap + 1) : 0]);
      ok = true;
      return (ok0 ? min(l0, 4) : 4) | ((ok1 ? min(l1, 4) : 4) << 8);
    }
    ok = tap < 27 && (lowm[r] & (tap_mask(tap) | 8u)) == 0u;
    const int off = ok ? base[r] + tap_off(tap) : 0;
    if constexpr (LAB) {
      return int(Lb[off]);
    } else {
      const int c0 = (ks * 32 + (lane >> 4) * 8) % CIN;
      return ld8(Xb + off * CIN + c0);
    }
  };
  auto load_b = [&](int ks, int t) {
    const int k = ks * 32 + (lane >> 4) * 8;
    if constexpr (L4) {
      const int j = k / 8;  // tap pair
      return ld8(W + ((j < 14 ? j : 0) * COUT + t * 16 + (lane & 15)) * 8);
    }
    const int tap = k / CIN, c0 = k % CIN;
    return ld8(W + ((tap < 27 ? tap : 0) * COUT + t * 16 + (lane & 15)) * CIN + c0);
  };
  f32x4 acc[RB][NT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (XS) {
    const int c0 = (lane >> 4) * 8;
    bool xlo[RB];  // ox = 0: the tx = 0 input is padding
#pragma unroll
    for (int r = 0; r < RB; ++r) xlo[r] = (lowm[r] & 4u) != 0u;
    // inputs at tx = 1, 2 of group g = 3 tz + ty, from a safe address where padded
    auto load_pair = [&](int g, int r, bf16x8& a1, bf16x8& a2) {
      const int tz = g / 3, ty = g % 3;
      const unsigned m = (tz == 0 ? 1u : 0u) | (ty == 0 ? 2u : 0u) | 8u;
      const bool ok = (lowm[r] & m) == 0u;
      const int off = ok ? base[r] + (tz * rs + ty) * rs + 1 : 0;
      const bf16x8 u1 = ld8(Xb + off * CIN + c0), u2 = ld8(Xb + (off + 1) * CIN + c0);
      a1 = ok ? u1 : zero8();
      a2 = ok ? u2 : zero8();
    };
    // the three taps of group gz from the tx = 1, 2 inputs of every row block
    auto group = [&](int gz, const bf16x8 (&c1)[RB], const bf16x8 (&c2)[RB]) {
      bf16x8 a0[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const bf16x8 sh = from_left_lane(c2[r]);
        a0[r] = xlo[r] ? zero8() : sh;
      }
#pragma unroll
      for (int tx = 0; tx < 3; ++tx) {
        const int tap = gz * 3 + tx;
        bf16x8 bw[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          bw[t] = WL ? sWf[((tap * NT + t) * 4 + (lane >> 4)) * 16 + (lane & 15)]
                     : ld8(W + (tap * COUT + t * 16 + (lane & 15)) * CIN + c0);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const bf16x8 a = tx == 0 ? a0[r] : (tx == 1 ? c1[r] : c2[r]);
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[r][t] = mfma(bw[t], a, acc[r][t]);
        }
      }
    };
    if constexpr (YR) {
      // the row blocks are consecutive output rows of one slice: row block r's
      // ty = 0 inputs (row 2 oy - 1) are row block r - 1's ty = 2 inputs
#pragma unroll
      for (int tz = 0; tz < 3; ++tz) {
        bf16x8 p1[RB], p2[RB];
        {
          bf16x8 c1[RB], c2[RB];
#pragma unroll
          for (int r = 0; r < RB; ++r) load_pair(3 * tz + 1, r, c1[r], c2[r]);
          group(3 * tz + 1, c1, c2);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) load_pair(3 * tz + 2, r, p1[r], p2[r]);
        group(3 * tz + 2, p1, p2);
        bf16x8 e1[RB], e2[RB];
        load_pair(3 * tz, 0, e1[0], e2[0]);
#pragma unroll
        for (int r = 1; r < RB; ++r) {
          e1[r] = p1[r - 1];
          e2[r] = p2[r - 1];
        }
        group(3 * tz, e1, e2);
      }
    } else {
#pragma unroll
      for (int gz = 0; gz < 9; ++gz) {
        bf16x8 c1[RB], c2[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) load_pair(gz, r, c1[r], c2[r]);
        group(gz, c1, c2);
      }
    }
  } else {
  // software pipeline: the loads of k-step ks + 1 are in flight during the MFMAs of ks
  Raw ra[RB];
  bool rok[RB];
  bf16x8 rb_[NT];
#pragma unroll
  for (int r = 0; r < RB; ++r) ra[r] = load_a(0, r, rok[r]);
#pragma unroll
  for (int t = 0; t < NT; ++t) rb_[t] = load_b(0, t);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 a[RB], bw[NT];
    const bool btap = tap_of(ks) < 27;
#pragma unroll
    for (int t = 0; t < NT; ++t) bw[t] = btap ? rb_[t] : zero8();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if constexpr (L4) {
        const bf16x4v lo = sOne4[ra[r] & 0xff], hi = sOne4[ra[r] >> 8];
        a[r] = bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      } else if constexpr (LAB) {
        a[r] = sOne[rok[r] ? min(ra[r], 8) : 8];
      } else {
        a[r] = rok[r] ? ra[r] : zero8();
      }
    }
    if (ks + 1 < KS) {
#pragma unroll
      for (int r = 0; r < RB; ++r) ra[r] = load_a(ks + 1, r, rok[r]);
#pragma unroll
      for (int t = 0; t < NT; ++t) rb_[t] = load_b(ks + 1, t);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = mfma(bw[t], a[r], acc[r][t]);
  }
  }
  // D = W x X^T: lane l holds, for row block r and tile t, output channels
  // t 16 + 4 (l / 16) + i (i = 0..3) of voxel v0 + 16 r + l % 16: bias, ReLU,
  // and the four channels as one 8-byte word
  if constexpr (STAGE) {
    store_staged<RB, NT, COUT>(acc, bias, sOut[wave], Y + (long long)b * nvo * COUT, nvo, v0, lane);
  } else {
    const int q = lane >> 4;
    __bf16* Yb = Y + (long long)b * nvo * COUT;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + 4 * q;
      const float4 bb = *reinterpret_cast<const float4*>(bias + co);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int v = v0 + r * 16 + (lane & 15);
        if (v < nvo) *reinterpret_cast<bf16x4*>(Yb + (long long)v * COUT + co) = bias_relu4(acc[r][t], bb);
      }
    }
  }
}

// One-hot codes of two labels a, c in 0..4 (4: the zero code) as one 16-byte
// LDS entry 5 a + c, a in channels 0-3 and c in channels 4-7 (25 entries),
// and entry 25, ones in channels 0 and 1: the input of the bias slot.
constexpr int kPairs = 26;
__device__ __forceinline__ void fill_pairs(bf16x8* t) {
  if (threadIdx.x < kPairs) {
    const bf16x4v lo = onehot4(threadIdx.x / 5), hi = onehot4(threadIdx.x % 5);
    const __bf16 one = (__bf16)1.0f, z = (__bf16)0.0f;
    t[threadIdx.x] = threadIdx.x < 25 ? bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]}
                                      : bf16x8{one, one, z, z, z, z, z, z};
  }
}
// the entry of labels a | c << 16 (each clamped to 4 first), plus `skip`
// bytes (16: from the zero pair (4, 4) to the bias entry)
__device__ __forceinline__ bf16x8 pair_code(const bf16x8* t, unsigned ac, unsigned skip = 0u) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  const u16x2 p = __builtin_elementwise_min(__builtin_bit_cast(u16x2, ac), u16x2{4, 4});
  const unsigned e = __builtin_amdgcn_udot2(p, u16x2{80, 16}, skip, false);  // 16 (5 a + c) + skip
  return *reinterpret_cast<const bf16x8*>(reinterpret_cast<const unsigned char*>(t) + e);
}

// First layer of networks of at most four phases, for label windows whose
// rows start on even addresses: the 27 taps go by rows (tz, ty) of three.
// K slot s = 4 ks + q of a voxel (q = lane / 16) is half s & 1 of row
// j = s / 2 (tz = j / 3, ty = j % 3):
//   half 0: taps tx = 1, 2, the labels at x = 2 ox and 2 ox + 1 (one aligned
//           2-byte load);
//   half 1: tap tx = 0, the label at 2 ox - 1 (high byte of the 2-byte word at
//           2 ox - 2; zero padding at ox = 0), and an empty tap.
// Nine rows take 5 k-steps (rows 9, slots 18 and 19, are empty).  Per k-step
// and row block a lane issues one load, and the two labels' four-channel
// one-hot codes are one 16-byte entry of an LDS table (labels 4 and above:
// the zero code).  W is laid out [slot][COUT][8] (k_cast_rows4).
template <int COUT, int RB>
__global__ void __launch_bounds__(256) k_conv_fwd_rows4(LabelWindow lw, const __bf16* __restrict__ W,
                                                        const float* __restrict__ bias, __bf16* __restrict__ Y,
                                                        Grid3 go) {
  static_assert(COUT % 16 == 0, "channel count");
  constexpr int KS = 5, NT = COUT / 16, VW = 16 * RB;
  constexpr unsigned kPad = 0x00040004u;  // both labels of a slot in the padding
  __shared__ bf16x8 sPair[kPairs];
  __shared__ __align__(16) __bf16 sOut[4][VW * COUT];
  const int nvo = go.D2 * go.D;  // output voxels per item
  const int b = blockIdx.y;      // item
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
  const int v0 = blockIdx.x * (64 * RB) + wave * VW;
  fill_pairs(sPair);
  __syncthreads();
  const unsigned char* Lb = window_base(lw, b);
  const unsigned rs = unsigned(lw.box), rs2 = rs * rs;
  const bool h1 = (q & 1) != 0;  // this lane's slots are halves 1
  // per row block: offset of (2 oz - 1, 2 oy - 1, x0), x0 = 2 ox (half 0) or
  // 2 ox - 2 (half 1), modulo 2^32; edge bits: 1 oz = 0, 2 oy = 0, 4 the
  // tx = 0 tap at ox = 0 (half 1), 8 always (rows 9).  Voxels past the end
  // take voxel 0's loads (their outputs are not stored).
  unsigned base[RB], edge[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int va = v0 + r * 16 + (lane & 15);
    int oz, oy, ox;
    split3(go, va < nvo ? va : 0, oz, oy, ox);
    base[r] = (unsigned(2 * oz - 1) * rs + unsigned(2 * oy - 1)) * rs + unsigned(2 * ox) - (h1 ? 2u : 0u);
    edge[r] = (oz == 0 ? 1u : 0u) | (oy == 0 ? 2u : 0u) | (h1 && ox == 0 ? 4u : 0u) | 8u;
  }
  // row of k-step ks: j = 2 ks + q / 2; its offset and the edge bits that
  // put it in the padding
  auto row_off = [&](int j) { return unsigned(j / 3) * rs2 + unsigned(j % 3) * rs; };
  auto row_mask = [](int j) { return j >= 9 ? 8u : (j / 3 == 0 ? 1u : 0u) | (j % 3 == 0 ? 2u : 0u) | 4u; };
  const bool qhi = q >= 2;
  unsigned roff[KS], rmask[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    roff[ks] = qhi ? row_off(2 * ks + 1) : row_off(2 * ks);
    rmask[ks] = qhi ? row_mask(2 * ks + 1) : row_mask(2 * ks);
  }
  // byte selectors of v_perm over {4, word}: half 0 (label x0, label x0 + 1),
  // half 1 (label x0 + 1, 4), as two 16-bit fields
  const unsigned psel = h1 ? 0x0C040C01u : 0x0C010C00u;
  auto load_a = [&](int ks, int r, bool& ok) -> unsigned {
    ok = (edge[r] & rmask[ks]) == 0u;
    const unsigned off = ok ? base[r] + roff[ks] : 0u;
    return *reinterpret_cast<const unsigned short*>(Lb + off);
  };
  auto onehot_pair = [&](unsigned w, bool ok) -> bf16x8 {
    return pair_code(sPair, ok ? __builtin_amdgcn_perm(4u, w, psel) : kPad);
  };
  auto load_b = [&](int ks, int t) { return ld8(W + ((4 * ks + q) * COUT + t * 16 + (lane & 15)) * 8); };
  f32x4 acc[RB][NT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // software pipeline: the loads of k-step ks + 1 are in flight during the MFMAs of ks
  unsigned ra[RB];
  bool rok[RB];
  bf16x8 rb_[NT];
#pragma unroll
  for (int r = 0; r < RB; ++r) ra[r] = load_a(0, r, rok[r]);
#pragma unroll
  for (int t = 0; t < NT; ++t) rb_[t] = load_b(0, t);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 a[RB], bw[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bw[t] = rb_[t];
#pragma unroll
    for (int r = 0; r < RB; ++r) a[r] = onehot_pair(ra[r], rok[r]);
    if (ks + 1 < KS) {
#pragma unroll
      for (int r = 0; r < RB; ++r) ra[r] = load_a(ks + 1, r, rok[r]);
#pragma unroll
      for (int t = 0; t < NT; ++t) rb_[t] = load_b(ks + 1, t);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = mfma(bw[t], a[r], acc[r][t]);
  }
  store_staged<RB, NT, COUT>(acc, bias, sOut[wave], Y + (long long)b * nvo * COUT, nvo, v0, lane);
}

// The same first layer with the workgroup's label footprint and the weights
// staged in LDS, for output edges DO that divide 256 (a workgroup's 256
// voxels are R = 256 / DO whole output rows of one slice) and label windows
// whose rows start on W-aligned addresses (W = 2 or 8).  K slots as in
// k_conv_fwd_rows4.  The footprint holds planes z = 2 oz - 1 .. 2 oz + 1 and
// rows y = 2 oy0 - 1 .. 2 oy0 + 2 R - 1 of the labels at x = -8 .. 2 DO - 1,
// with everything outside the window (the zero padding) stored as label 4,
// the zero code, so no tap needs an edge test; a fourth plane of 4s serves
// the empty row 9.
template <int DO, int W, int COUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_conv_fwd_rows4s(LabelWindow lw, const __bf16* __restrict__ Wr,
                                                         const float* __restrict__ bias, __bf16* __restrict__ Y) {
  static_assert(256 % DO == 0 && DO % 16 == 0 && (W == 2 || W == 8) && COUT % 16 == 0, "shapes");
  constexpr int RB = 4, KS = 5, NT = COUT / 16, VW = 16 * RB;
  constexpr int R = 256 / DO;     // output rows per workgroup
  constexpr int NY = 2 * R + 1;   // footprint rows per plane
  constexpr int RW = 2 * DO + 8;  // bytes per footprint row; label x at byte 8 + x
  constexpr int U = 2 * DO / W, NU = 3 * NY * U, KU = (NU + 255) / 256;  // label units of W bytes
  constexpr int NWU = 20 * COUT, KW = (NWU + 255) / 256;                // weight units of 16 bytes
  using Unit = typename std::conditional<W == 8, unsigned long long, unsigned short>::type;
  constexpr Unit kFour = W == 8 ? Unit(0x0404040404040404ull) : Unit(0x0404u);
  // the staged weights and labels, and after the last k-step the waves'
  // output tiles in the same bytes (more resident workgroups per CU)
  constexpr int IN_BYTES = NWU * 16 + 4 * NY * RW, OUT_BYTES = 4 * VW * COUT * 2;
  __shared__ __align__(16) unsigned char smem[IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES];
  __shared__ bf16x8 sPair[kPairs];
  bf16x8* sW = reinterpret_cast<bf16x8*>(smem);
  unsigned char* sLab = smem + NWU * 16;
  constexpr int nvo = DO * DO * DO;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4;
  const int oz = blockIdx.x / (DO / R), oy0 = (blockIdx.x % (DO / R)) * R;
  const unsigned char* Lb = window_base(lw, b);
  // every global load first, then the LDS writes
  Unit lv[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int u = threadIdx.x + k * 256;
    const int row = u / U, c = u % U, zz = row / NY, yy = row % NY;
    const int z = 2 * oz - 1 + zz, y = 2 * oy0 - 1 + yy;
    lv[k] = kFour;
    if ((NU % 256 == 0 || u < NU) && z >= 0 && y >= 0)
      lv[k] = *reinterpret_cast<const Unit*>(Lb + z * lw.plane + y * lw.row + c * W);
  }
  bf16x8 wv[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int i = threadIdx.x + k * 256;
    if (NWU % 256 == 0 || i < NWU) wv[k] = ld8(Wr + i * 8);
  }
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int u = threadIdx.x + k * 256;
    const int row = u / U, c = u % U;
    if (NU % 256 == 0 || u < NU) *reinterpret_cast<Unit*>(sLab + row * RW + 8 + c * W) = lv[k];
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int i = threadIdx.x + k * 256;
    if (NWU % 256 == 0 || i < NWU) sW[i] = wv[k];
  }
  // x = -8 .. -1 of the three planes, and the whole fourth plane: 4s
  for (int i = threadIdx.x; i < 3 * NY + NY * RW / 8; i += 256) {
    const int off = i < 3 * NY ? i * RW : 3 * NY * RW + (i - 3 * NY) * 8;
    *reinterpret_cast<unsigned long long*>(sLab + off) = 0x0404040404040404ull;
  }
  fill_pairs(sPair);
  __syncthreads();
  const bool h1 = (q & 1) != 0, qhi = q >= 2;
  // row block r: output row rho (of the workgroup's R) and ox; footprint
  // offset of its tap row (tz, ty) = (0, 0) at x0 = 2 ox (half 0) or 2 ox - 2
  unsigned lb[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int u = wave * VW + r * 16 + (lane & 15);
    const int rho = u / DO, ox = u % DO;
    lb[r] = unsigned(2 * rho * RW + 8 + 2 * ox - (h1 ? 2 : 0));
  }
  // tap row j = 2 ks + q / 2 (tz = j / 3, ty = j % 3; j = 9 is the plane of 4s)
  auto row_off = [](int j) { return unsigned(((j / 3) * NY + j % 3) * RW); };
  unsigned roff[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) roff[ks] = qhi ? row_off(2 * ks + 1) : row_off(2 * ks);
  const unsigned psel = h1 ? 0x0C040C01u : 0x0C010C00u;
  // slot 19 (k-step 4, q = 3) reads the zero pair of the plane of 4s and
  // takes the bias entry instead: WR's slot 19 holds the bias (high and low
  // BF16 parts), so the MFMAs add it
  const unsigned bias_skip = q == 3 ? 16u : 0u;
  auto onehot_pair = [&](int ks, int r) -> bf16x8 {
    const unsigned w = *reinterpret_cast<const unsigned short*>(sLab + lb[r] + roff[ks]);
    return pair_code(sPair, __builtin_amdgcn_perm(4u, w, psel), ks == KS - 1 ? bias_skip : 0u);
  };
  f32x4 acc[RB][NT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 a[RB], bw[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bw[t] = sW[(4 * ks + q) * COUT + t * 16 + (lane & 15)];
#pragma unroll
    for (int r = 0; r < RB; ++r) a[r] = onehot_pair(ks, r);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = mfma(bw[t], a[r], acc[r][t]);
  }
  __syncthreads();  // every wave is done with the staged inputs
  store_staged<RB, NT, COUT, false>(acc, bias, reinterpret_cast<__bf16*>(smem) + wave * VW * COUT,
                                    Y + (long long)b * nvo * COUT, nvo, blockIdx.x * 256 + wave * VW, lane);
}

// Forward convolution with the K steps of RB 16-voxel row blocks split over
// the 4 waves of a workgroup (for the deep layers with few voxels and long
// K): wave w takes k-steps w, w + 4, ... of every row block, so each weight
// fragment it loads serves RB MFMAs.  The four partials of a row block are
// summed through LDS in wave order, the same sums for every RB.
template <int CIN, int COUT, int RB = 1>
__global__ void __launch_bounds__(256) k_conv_fwd_splitk(const __bf16* __restrict__ X, const __bf16* __restrict__ W,
                                                         const float* __restrict__ bias, __bf16* __restrict__ Y, int D,
                                                         Grid3 go) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0, "channel counts");
  constexpr int KT = 27 * CIN, KS = (KT + 31) / 32, NT = COUT / 16;
  __shared__ f32x4 red[4][RB][NT][64];
  const int nvo = go.D2 * go.D;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v0 = blockIdx.x * 16 * RB;
  bool valid[RB];
  int oz[RB], oy[RB], ox[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int va = v0 + r * 16 + (lane & 15);
    valid[r] = va < nvo;
    split3(go, valid[r] ? va : 0, oz[r], oy[r], ox[r]);
  }
  const __bf16* Xb = X + (long long)b * D * D * D * CIN;
  f32x4 acc[RB][NT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = wave; ks < KS; ks += 4) {
    const int k = ks * 32 + (lane >> 4) * 8;
    const int tap = k / CIN, c0 = k % CIN;
    bf16x8 a[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      a[r] = zero8();
      const int iz = 2 * oz[r] + tap / 9 - 1, iy = 2 * oy[r] + (tap / 3) % 3 - 1, ix = 2 * ox[r] + tap % 3 - 1;
      if (valid[r] && tap < 27 && iz >= 0 && iy >= 0 && ix >= 0) a[r] = ld8(Xb + ((iz * D + iy) * D + ix) * CIN + c0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 bw = zero8();
      if (tap < 27) bw = ld8(W + (tap * COUT + t * 16 + (lane & 15)) * CIN + c0);
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r][t] = mfma(a[r], bw, acc[r][t]);
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) red[wave][r][t][lane] = acc[r][t];
  __syncthreads();
  __bf16* Yb = Y + (long long)b * nvo * COUT;
  for (int r = wave; r < RB; r += 4) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + (lane & 15);
      const float bb = bias[co];
      const f32x4 s0 = red[0][r][t][lane], s1 = red[1][r][t][lane], s2 = red[2][r][t][lane], s3 = red[3][r][t][lane];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float sum = s0[i] + s1[i] + s2[i] + s3[i];
        const int v = v0 + r * 16 + (lane >> 4) * 4 + i;
        if (v < nvo) Yb[v * COUT + co] = (__bf16)fmaxf(sum + bb, 0.0f);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// data gradient: dX[i][cin] = sum_{tap, cout} dZ[o(i, tap)][cout] W[tap][cout][cin]
// with dZ = dY * (Y > 0).  Input voxels are processed by parity class
// (pz, py, px) so that each 16-voxel MFMA row block visits only valid taps:
// along an axis an even input index is reached by tap 1 only, an odd one by
// taps 0 and 2.  Wt: [tap][cin][cout].  dX FP32 [b][D^3][CIN].
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv_dgrad(const float* __restrict__ dY, const __bf16* __restrict__ Y,
                                                    const __bf16* __restrict__ Wt, float* __restrict__ dX, int D,
                                                    Grid3 gh, int cls) {
  static_assert(CIN % 16 == 0 && COUT % 32 == 0, "channel counts");
  constexpr int NT = CIN / 16, KC = COUT / 32;
  const int Do = D / 2;
  const int pz = (cls >> 2) & 1, py = (cls >> 1) & 1, px = cls & 1;
  const int ncls = gh.D2 * gh.D;  // voxels of one parity class in one item (h = D / 2 per axis)
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v0 = blockIdx.x * 64 + wave * 16;
  const int va = v0 + (lane & 15);
  const bool valid_a = va < ncls;
  int jz, jy, jx;
  split3(gh, valid_a ? va : 0, jz, jy, jx);
  const int nvo = Do * Do * Do;
  const float* dYb = dY + (long long)b * nvo * COUT;
  const __bf16* Yb = Y + (long long)b * nvo * COUT;
  // taps along each axis for this parity: even -> {1}, odd -> {0, 2}
  const int nz_t = pz ? 2 : 1, ny_t = py ? 2 : 1, nx_t = px ? 2 : 1;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int a_ = 0; a_ < nz_t; ++a_)
    for (int b_ = 0; b_ < ny_t; ++b_)
      for (int c_ = 0; c_ < nx_t; ++c_) {
        const int tz = pz ? 2 * a_ : 1, ty = py ? 2 * b_ : 1, tx = px ? 2 * c_ : 1;
        const int tap = (tz * 3 + ty) * 3 + tx;
        // i = 2 j + p = 2 o + t - 1  ->  o = j + (p + 1 - t) / 2
        const int oz = jz + (pz + 1 - tz) / 2, oy = jy + (py + 1 - ty) / 2, ox = jx + (px + 1 - tx) / 2;
        const bool in = valid_a && oz < Do && oy < Do && ox < Do;
        const int ov = (oz * Do + oy) * Do + ox;
        for (int kc = 0; kc < KC; ++kc) {
          const int co0 = kc * 32 + (lane >> 4) * 8;
          bf16x8 a = zero8();
          if (in) {
            const float* gp = dYb + ov * COUT + co0;
            const bf16x8 yv = ld8(Yb + ov * COUT + co0);
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)((float)yv[j] > 0.0f ? gp[j] : 0.0f);
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 bw = ld8(Wt + (tap * CIN + t * 16 + (lane & 15)) * COUT + co0);
            acc[t] = mfma(a, bw, acc[t]);
          }
        }
      }
  float* dXb = dX + (long long)b * D * D * D * CIN;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = v0 + (lane >> 4) * 4 + i;
    if (v < ncls) {
      int z, y, x;
      split3(gh, v, z, y, x);
      const int base = (((2 * z + pz) * D + 2 * y + py) * D + 2 * x + px) * CIN;
#pragma unroll
      for (int t = 0; t < NT; ++t) dXb[base + t * 16 + (lane & 15)] = acc[t][i];
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient of a layer with bf16 input activations, one tap per block:
// partial dW[tap][cout][cin] over a chunk of output voxels, dZ = dY * (Y > 0).
// The chunk of dZ and of the gathered input is staged in LDS transposed
// (channel-major) so that MFMA fragments (K = voxels) are 16-byte LDS reads.
// The bias gradient rides on tap 13.
// Partials: part[chunk][tap][COUT][CIN], bias partials pb[chunk][COUT].
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv_wgrad(const float* __restrict__ dY, const __bf16* __restrict__ Y,
                                                    const __bf16* __restrict__ X, float* __restrict__ part,
                                                    float* __restrict__ pb, int D, Grid3 go, int batch, int chunk) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0 && 256 % COUT == 0, "channel counts");
  constexpr int MT = COUT / 16, NTN = (CIN + 15) / 16;  // output tiles (cout x cin)
  constexpr int VS = 32;                                 // voxels per staged step (= MFMA K)
  __shared__ __bf16 sZ[COUT][VS + 8];
  __shared__ __bf16 sX[NTN * 16][VS + 8];
  __shared__ int sPos[VS][4];  // item, iz0, iy0, ix0 (input corner 2o - 1) of each staged voxel; item -1 if none
  const int tap = blockIdx.y;
  const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
  const int nvo = go.D2 * go.D;
  const float inv_nvo = 1.0f / float(nvo);
  const long long total = (long long)nvo * batch;
  const long long vbeg = (long long)blockIdx.x * chunk;
  const long long vend = vbeg + chunk < total ? vbeg + chunk : total;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave w owns output tiles w, w+4, ... of the MT x NTN grid
  constexpr int TILES = MT * NTN, TPW = (TILES + 3) / 4;
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;  // bias partial for cout = threadIdx.x % COUT (tap 13 blocks)
  __shared__ float sB[256];
  // (item, voxel) of the first staged voxel, carried from step to step
  int b0 = int(vbeg / nvo), r0 = int(vbeg - (long long)b0 * nvo);
  for (long long vs = vbeg; vs < vend; vs += VS) {
    __syncthreads();
    if (threadIdx.x < VS) {
      const int vl = threadIdx.x;
      int bi = -1, z = 0, y = 0, x = 0;
      if (vs + vl < vend) {
        const int q = fdiv(r0 + vl, nvo, inv_nvo);
        bi = b0 + q;
        split3(go, r0 + vl - q * nvo, z, y, x);
      }
      sPos[vl][0] = bi;
      sPos[vl][1] = 2 * z - 1;
      sPos[vl][2] = 2 * y - 1;
      sPos[vl][3] = 2 * x - 1;
    }
    __syncthreads();
    // stage dZ^T: COUT x VS
    for (int e = threadIdx.x; e < COUT * VS; e += 256) {
      const int co = e % COUT, vl = e / COUT;
      float zv = 0.0f;
      if (vs + vl < vend) {
        const long long v = vs + vl;
        const float gv = dY[v * COUT + co];
        zv = (float)Y[v * COUT + co] > 0.0f ? gv : 0.0f;
      }
      sZ[co][vl] = (__bf16)zv;
      if (tap == 13) bsum += zv;  // co == threadIdx.x % COUT since 256 % COUT == 0
    }
    // stage X^T for this tap: CIN x VS (zero rows beyond CIN)
    for (int e = threadIdx.x; e < NTN * 16 * VS; e += 256) {
      const int ci = e % (NTN * 16), vl = e / (NTN * 16);
      float xv = 0.0f;
      const int bi = sPos[vl][0];
      if (bi >= 0 && ci < CIN) {
        const int iz = sPos[vl][1] + tz, iy = sPos[vl][2] + ty, ix = sPos[vl][3] + tx;
        if (iz >= 0 && iy >= 0 && ix >= 0)  // 2 o + t - 1 < D always
          xv = (float)X[((long long)bi * D * D * D + (iz * D + iy) * D + ix) * CIN + ci];
      }
      sX[ci][vl] = (__bf16)xv;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tile = wave + 4 * q;
      if (tile < TILES) {
        const int mt = tile / NTN, nt = tile % NTN;
        bf16x8 a, bw;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[j] = sZ[mt * 16 + (lane & 15)][(lane >> 4) * 8 + j];
          bw[j] = sX[nt * 16 + (lane & 15)][(lane >> 4) * 8 + j];
        }
        acc[q] = mfma(a, bw, acc[q]);
      }
    }
    // advance the carried (item, voxel) by one step
    r0 += VS;
    const int q = fdiv(r0, nvo, inv_nvo);
    b0 += q;
    r0 -= q * nvo;
  }
  // D tile rows = cout (A rows), cols = cin (B cols)
  float* out = part + ((long long)blockIdx.x * 27 + tap) * COUT * CIN;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int tile = wave + 4 * q;
    if (tile < TILES) {
      const int mt = tile / NTN, nt = tile % NTN;
      const int ci = nt * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = mt * 16 + (lane >> 4) * 4 + i;
        if (ci < CIN) out[co * CIN + ci] = acc[q][i];
      }
    }
  }
  if (tap == 13) {
    sB[threadIdx.x] = bsum;
    __syncthreads();
    if (threadIdx.x < COUT) {
      float t = 0.0f;
      for (int r = threadIdx.x; r < 256; r += COUT) t += sB[r];
      pb[(long long)blockIdx.x * COUT + threadIdx.x] = t;
    }
  }
}

// Weight gradient of the first layer (8 one-hot input channels): each block
// takes one chunk of voxels for all 27 taps.  Per 32-voxel step, dZ^T is
// staged once, and so are the 27 tap labels of every staged voxel (8 where
// the tap falls in the padding); the one-hot B fragments are formed in
// registers from those labels.  Wave w owns taps w, w + 4, ...  Output and
// bias partials are laid out as k_conv_wgrad's.
template <int COUT>
__global__ void __launch_bounds__(256) k_conv_wgrad_lab(const float* __restrict__ dY, const __bf16* __restrict__ Y,
                                                        LabelWindow lw, float* __restrict__ part,
                                                        float* __restrict__ pb, Grid3 go, int batch, int chunk) {
  static_assert(COUT % 16 == 0 && 256 % COUT == 0, "channel counts");
  constexpr int CIN = 8, MT = COUT / 16, VS = 32, TPW = 7;  // taps per wave: ceil(27 / 4)
  __shared__ __bf16 sZ[COUT][VS + 8];
  __shared__ unsigned char sL[VS][28];
  __shared__ int sPos[VS][4];  // item, iz0, iy0, ix0 (input corner 2 o - 1) of each staged voxel; item -1 if none
  __shared__ float sB[256];
  const int nvo = go.D2 * go.D;
  const float inv_nvo = 1.0f / float(nvo);
  const long long total = (long long)nvo * batch;
  const long long vbeg = (long long)blockIdx.x * chunk;
  const long long vend = vbeg + chunk < total ? vbeg + chunk : total;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x4 acc[TPW][MT];
#pragma unroll
  for (int q = 0; q < TPW; ++q)
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[q][m] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;  // bias partial for cout = threadIdx.x % COUT
  int b0 = int(vbeg / nvo), r0 = int(vbeg - (long long)b0 * nvo);
  for (long long vs = vbeg; vs < vend; vs += VS) {
    __syncthreads();
    if (threadIdx.x < VS) {
      const int vl = threadIdx.x;
      int bi = -1, z = 0, y = 0, x = 0;
      if (vs + vl < vend) {
        const int q = fdiv(r0 + vl, nvo, inv_nvo);
        bi = b0 + q;
        split3(go, r0 + vl - q * nvo, z, y, x);
      }
      sPos[vl][0] = bi;
      sPos[vl][1] = 2 * z - 1;
      sPos[vl][2] = 2 * y - 1;
      sPos[vl][3] = 2 * x - 1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < COUT * VS; e += 256) {
      const int co = e % COUT, vl = e / COUT;
      float zv = 0.0f;
      if (vs + vl < vend) {
        const long long v = vs + vl;
        const float gv = dY[v * COUT + co];
        zv = (float)Y[v * COUT + co] > 0.0f ? gv : 0.0f;
      }
      sZ[co][vl] = (__bf16)zv;
      bsum += zv;  // co == threadIdx.x % COUT since 256 % COUT == 0
    }
    for (int e = threadIdx.x; e < VS * 27; e += 256) {
      const int vl = e / 27, t = e - vl * 27;
      unsigned lab = 8u;
      const int bi = sPos[vl][0];
      if (bi >= 0) {
        const int iz = sPos[vl][1] + t / 9, iy = sPos[vl][2] + (t / 3) % 3, ix = sPos[vl][3] + t % 3;
        if (iz >= 0 && iy >= 0 && ix >= 0)  // 2 o + t - 1 < D always
          lab = min(unsigned(window_base(lw, bi)[(iz * lw.box + iy) * lw.box + ix]), 8u);
      }
      sL[vl][t] = (unsigned char)lab;
    }
    __syncthreads();
    bf16x8 a[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int j = 0; j < 8; ++j) a[m][j] = sZ[m * 16 + (lane & 15)][(lane >> 4) * 8 + j];
    const unsigned ci = unsigned(lane & 15);  // B column: input channel (8..15 stay zero)
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wave + 4 * q;
      if (t < 27) {
        bf16x8 bw;
#pragma unroll
        for (int j = 0; j < 8; ++j) bw[j] = (__bf16)(ci < 8u && sL[(lane >> 4) * 8 + j][t] == ci ? 1.0f : 0.0f);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[q][m] = mfma(a[m], bw, acc[q][m]);
      }
    }
    r0 += VS;
    const int q = fdiv(r0, nvo, inv_nvo);
    b0 += q;
    r0 -= q * nvo;
  }
  // D tile rows = cout (A rows), cols = cin (B cols)
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + 4 * q;
    if (t < 27) {
      float* out = part + ((long long)blockIdx.x * 27 + t) * COUT * CIN;
      const int cin = lane & 15;
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = m * 16 + (lane >> 4) * 4 + i;
          if (cin < CIN) out[co * CIN + cin] = acc[q][m][i];
        }
    }
  }
  sB[threadIdx.x] = bsum;
  __syncthreads();
  if (threadIdx.x < COUT) {
    float t = 0.0f;
    for (int r = threadIdx.x; r < 256; r += COUT) t += sB[r];
    pb[(long long)blockIdx.x * COUT + threadIdx.x] = t;
  }
}

// Sum of weight-gradient partials over chunks, out[i] = sum_c part[c * n + i],
// for many chunks: a block of 16 waves takes 64 consecutive outputs (one per
// lane); wave w sums chunks w, w + 16, ... and the 16 wave sums are added in
// wave order.  The order is fixed, so results do not depend on timing.
__global__ void __launch_bounds__(1024) k_reduce_parts_wide(const float* __restrict__ part, int nchunk, long long n,
                                                            float* __restrict__ out) {
  __shared__ float sS[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long i = (long long)blockIdx.x * 64 + lane;
  float s = 0.0f;
  if (i < n) {
    int c = wave;
    for (; c + 48 < nchunk; c += 64) {
      const float a0 = part[(long long)c * n + i], a1 = part[(long long)(c + 16) * n + i];
      const float a2 = part[(long long)(c + 32) * n + i], a3 = part[(long long)(c + 48) * n + i];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; c < nchunk; c += 16) s += part[(long long)c * n + i];
  }
  sS[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && i < n) {
    float t = 0.0f;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += sS[w][lane];
    out[i] = t;
  }
}

// sum partials over chunks in fixed order: out[i] = sum_c part[c * n + i]
__global__ void k_reduce_parts(const float* __restrict__ part, int nchunk, long long n, float* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * n + i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------------------
// head: global mean over V voxels of the last activation (64 channels), the
// 8 standardized phase fractions (f_c - mu_c) sc_c appended, f_c from the
// label counts (72 features), linear 72 -> 21,
// and (training) squared loss against targets with its gradients.  Only the
// 64 pooled features pass a gradient back.  One block of 64 threads per item.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_head(const __bf16* __restrict__ A, int V, const int* __restrict__ cnt,
                                             double inv_nv, const float* __restrict__ fmu,
                                             const float* __restrict__ fsc, const float* __restrict__ Wfc,
                                             const float* __restrict__ bfc,
                                             float* __restrict__ out, const float* __restrict__ target,
                                             float* __restrict__ dA, float* __restrict__ dW_item,
                                             float* __restrict__ loss_item, float inv_count,
                                             const double* __restrict__ dmean, const double* __restrict__ dscale,
                                             double* __restrict__ c21) {
  constexpr int C = 64, F = 72, O = 21;
  __shared__ float feat[F];
  __shared__ float dout[O];
  __shared__ float part[C][9];  // [thread][channel of its group of 8] (padded row)
  const int b = blockIdx.x, c = threadIdx.x;
  const __bf16* Ab = A + (long long)b * V * C;
  // mean pool: 16-byte chunk k holds channels 8 (k % 8) .. + 7 of voxel k / 8;
  // thread c takes chunks c, c + 64, ... (always channel group c % 8), then
  // the 8 threads of a group are summed in a fixed order
  float p8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
  for (int k = c; k < V * 8; k += C) {
    const bf16x8 x = ld8(Ab + (long long)k * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) p8[j] += (float)x[j];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) part[c][j] = p8[j];
  __syncthreads();
  {
    float s = 0.0f;
    for (int t = c / 8; t < C; t += 8) s += part[t][c % 8];
    feat[c] = s / float(V);
  }
  if (c < F - C) feat[C + c] = (float(double(cnt[b * (F - C) + c]) * inv_nv) - fmu[c]) * fsc[c];
  __syncthreads();
  if (c < O) {
    float y = bfc[c];
    for (int k = 0; k < F; ++k) y += Wfc[c * F + k] * feat[k];
    out[b * O + c] = y;
    // the denormalized stiffness y scale + mean (FP64) when asked for
    if (c21) c21[b * O + c] = double(y) * dscale[c] + dmean[c];
    if (target) dout[c] = 2.0f * (y - target[b * O + c]) * inv_count;
  }
  __syncthreads();
  if (!target) return;
  if (c == 0) {
    float l = 0.0f;
    for (int o = 0; o < O; ++o) {
      const float d = out[b * O + o] - target[b * O + o];
      l += d * d;
    }
    loss_item[b] = l * inv_count;
  }
  // parameter gradients of this item: dW[o][k] = dout[o] feat[k], db[o] = dout[o]
  for (int e = c; e < O * F; e += C) dW_item[(long long)b * (O * F + O) + e] = dout[e / F] * feat[e % F];
  if (c < O) dW_item[(long long)b * (O * F + O) + O * F + c] = dout[c];
  // dfeat[k] = sum_o dout[o] W[o][k]; the mean spreads it evenly over V voxels
  float g = 0.0f;
  for (int o = 0; o < O; ++o) g += dout[o] * Wfc[o * F + c];
  g /= float(V);
  for (int v = 0; v < V; ++v) dA[((long long)b * V + v) * C + c] = g;
}

// Adam on FP32 masters, then BF16 working copies of the convolution weights:
// W [tap][cout][cin] and Wt [tap][cin][cout].
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// First-layer weights for the four-channel path: W4[j][co][c] is tap 2 j
// (c < 4) or tap 2 j + 1 (c >= 4), channel c % 4, zero past tap 26; j < 14.
__global__ void k_cast_pairs4(const float* __restrict__ w, int cout, __bf16* __restrict__ W4) {
  const int n = 14 * cout * 8;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = i % 8, co = (i / 8) % cout, j = i / (8 * cout);
    const int tap = 2 * j + c / 4;
    W4[i] = (__bf16)(tap < 27 ? w[((long long)tap * cout + co) * 8 + c % 4] : 0.0f);
  }
}

// First-layer weights for the row paths (k_conv_fwd_rows4, _rows4s): slot
// s < 18 is half s & 1 of row j = s / 2 (taps 3 j .. 3 j + 2); half 0 holds
// tap 3 j + 1 (c < 4) and tap 3 j + 2 (c >= 4), half 1 tap 3 j (c < 4) and
// zeros.  Slot 18 is zero; slot 19 holds the bias as a high and a low BF16
// part (c = 0, 1; their sum is the bias to 2^-16 relative), which
// k_conv_fwd_rows4s multiplies by ones and k_conv_fwd_rows4 by zeros.
// WR[s][co][c], channel c % 4.
__global__ void k_cast_rows4(const float* __restrict__ w, const float* __restrict__ bias, int cout,
                             __bf16* __restrict__ WR) {
  const int n = 20 * cout * 8;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = i % 8, co = (i / 8) % cout, s = i / (8 * cout), j = s / 2;
    if (s == 19) {
      const __bf16 hi = (__bf16)bias[co];
      WR[i] = c == 0 ? hi : (c == 1 ? (__bf16)(bias[co] - (float)hi) : (__bf16)0.0f);
      continue;
    }
    const int tap = (s & 1) ? (c < 4 ? 3 * j : -1) : 3 * j + 1 + c / 4;
    WR[i] = (__bf16)(j < 9 && tap >= 0 ? w[((long long)tap * cout + co) * 8 + c % 4] : 0.0f);
  }
}

__global__ void k_cast_weights(const float* __restrict__ w, int cin, int cout, __bf16* __restrict__ W,
                               __bf16* __restrict__ Wt) {
  const long long n = 27LL * cout * cin;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ci = int(i % cin), co = int((i / cin) % cout), t = int(i / ((long long)cin * cout));
    const float x = w[i];
    W[i] = (__bf16)x;
    if (Wt) Wt[((long long)t * cin + ci) * cout + co] = (__bf16)x;
  }
}

// ---------------------------------------------------------------------------
// gate: SPD (FP64 Cholesky) and the Voigt-Reuss bracket of the item's phase
// fractions (quadratic-form sense, Mandel scaling), plus the spread between
// two predictions.  flag = 1 sends the item to the FFT solver.
// ---------------------------------------------------------------------------
__device__ bool chol_pd(double A[6][6]) {
  for (int j = 0; j < 6; ++j) {
    double s = A[j][j];
    for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
    if (!(s > 0.0)) return false;
    const double d = sqrt(s);
    A[j][j] = d;
    for (int i = j + 1; i < 6; ++i) {
      double t = A[i][j];
      for (int k = 0; k < j; ++k) t -= A[i][k] * A[j][k];
      A[i][j] = t / d;
    }
  }
  return true;
}

__global__ void k_gate(const double* __restrict__ c21a, const double* __restrict__ c21b,
                       const double* __restrict__ cv21, const double* __restrict__ cr21, int nitems, double spread_tol,
                       double bound_tol, FracGate ga, FracGate gb, int* __restrict__ flag) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  const double s[6] = {1.0, 1.0, 1.0, 1.4142135623730951, 1.4142135623730951, 1.4142135623730951};
  double C[6][6], CV[6][6], CR[6][6], B[6][6];
  int k = 0;
  double nrm = 0.0, dif = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      const double a = c21a[(long long)it * 21 + k], b = c21b ? c21b[(long long)it * 21 + k] : a;
      C[i][j] = C[j][i] = 0.5 * (a + b) * s[i] * s[j];
      CV[i][j] = CV[j][i] = cv21[(long long)it * 21 + k] * s[i] * s[j];
      CR[i][j] = CR[j][i] = cr21[(long long)it * 21 + k] * s[i] * s[j];
      const double w = (i == j ? 1.0 : 2.0) * s[i] * s[i] * s[j] * s[j];
      nrm += w * a * a;
      dif += w * (a - b) * (a - b);
      ++k;
    }
  int bad = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) B[i][j] = C[i][j];
  if (!chol_pd(B)) bad = 1;
  // C_V - C >= -tol |C| and C - C_R >= -tol |C|, checked as shifted PD tests
  const double shift = bound_tol * sqrt(nrm);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) B[i][j] = CV[i][j] - C[i][j] + (i == j ? shift : 0.0);
  if (!chol_pd(B)) bad = 1;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) B[i][j] = C[i][j] - CR[i][j] + (i == j ? shift : 0.0);
  if (!chol_pd(B)) bad = 1;
  if (c21b && dif > spread_tol * spread_tol * nrm) bad = 1;
  // phase fractions of each network's input window against its training range
  auto outside = [&](const FracGate& q) {
    if (!q.counts || !(q.zmax > 0.0)) return false;
    bool out = false;
    for (int c = 0; c < 8; ++c) {
      const double d = fabs(double(q.counts[(long long)it * 8 + c]) * q.inv_nv - q.mu[c]);
      out = out || (q.sc[c] > 0.0 ? d * q.sc[c] > q.zmax : d > 0.5 * q.inv_nv);
    }
    // interface density of the window (its texture), where the network has
    // training statistics of it
    if (q.iface && q.isc > 0.0)
      out = out || fabs(double(q.iface[it]) * q.inv_pairs - q.imu) * q.isc > q.zmax;
    return out;
  };
  if (outside(ga) || outside(gb)) bad = 1;
  flag[it] = bad;
}

// Voigt (arithmetic mean of stiffness) and Reuss (inverse of the mean
// compliance) stiffnesses of each item's phase mixture, 21 components each,
// from its label counts (k_count_labels over the n^3 core).  One thread per item.
__global__ void k_bounds_from_counts(const int* __restrict__ cnt, int nitems, double inv_nv, int nphase,
                                     const double* __restrict__ Cp21, const double* __restrict__ Sp21,
                                     double* __restrict__ cv21, double* __restrict__ cr21) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  double f[8];
  for (int p = 0; p < 8; ++p) f[p] = p < nphase ? double(cnt[it * 8 + p]) * inv_nv : 0.0;
  double S[6][6], Ci[6][6];
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      double cv = 0.0, sv = 0.0;
      for (int p = 0; p < nphase; ++p) {
        cv += f[p] * Cp21[p * 21 + k];
        sv += f[p] * Sp21[p * 21 + k];
      }
      cv21[(long long)it * 21 + k] = cv;
      S[i][j] = S[j][i] = sv;
      ++k;
    }
  // Reuss stiffness = S^-1 (Gauss-Jordan, S is SPD)
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Ci[i][j] = (i == j) ? 1.0 : 0.0;
  for (int c = 0; c < 6; ++c) {
    const double d = 1.0 / S[c][c];
    for (int j = 0; j < 6; ++j) {
      S[c][j] *= d;
      Ci[c][j] *= d;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const double fct = S[r][c];
      for (int j = 0; j < 6; ++j) {
        S[r][j] -= fct * S[c][j];
        Ci[r][j] -= fct * Ci[c][j];
      }
    }
  }
  k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) cr21[(long long)it * 21 + k++] = Ci[i][j];
}

}  // namespace cnn
}  // namespace hh
