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
#include <string>
#include <vector>

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
// The network input: the n^3 window at (o, o, o) of each of `batch` label
// boxes of edge `box` (uint8, `stride` bytes apart).  The first layer reads
// the labels and forms their one-hot code (8 channels) in registers.
// ---------------------------------------------------------------------------
struct LabelWindow {
  const unsigned char* labels;
  long long stride;
  int box, o;
};

__device__ __forceinline__ int label_at(const LabelWindow& w, long long b, int z, int y, int x) {
  return w.labels[b * w.stride + ((long long)(z + w.o) * w.box + (y + w.o)) * w.box + (x + w.o)];
}

__device__ __forceinline__ bf16x8 onehot8(int lab) {
  bf16x8 h;
#pragma unroll
  for (int c = 0; c < 8; ++c) h[c] = (__bf16)(c == lab ? 1.0f : 0.0f);
  return h;
}

// Label counts of each window: cnt[b][c] += number of voxels with label c
// (c < 8).  Grid (row blocks, batch); each wave takes whole x-rows (lanes
// along x), counts in registers, then one atomic per block and label.
constexpr int kCountRows = 64;

__global__ void __launch_bounds__(256) k_count_labels(LabelWindow w, int n, int* __restrict__ cnt) {
  const int b = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.x * kCountRows, r1 = min(n * n, r0 + kCountRows);
  int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = r0 + wave; r < r1; r += 4) {
    const int z = r / n, y = r - z * n;
    for (int x = lane; x < n; x += 64) {
      const int lab = label_at(w, b, z, y, x);
#pragma unroll
      for (int k = 0; k < 8; ++k) c[k] += (lab == k) ? 1 : 0;
    }
  }
  __shared__ int s[8];
  if (threadIdx.x < 8) s[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int v = c[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0 && v) atomicAdd(&s[k], v);
  }
  __syncthreads();
  if (threadIdx.x < 8 && s[threadIdx.x]) atomicAdd(&cnt[b * 8 + threadIdx.x], s[threadIdx.x]);
}

__global__ void k_zero_int(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Input voxel of output voxel (oz, oy, ox) under tap t (stride 2, pad 1);
// returns -1 when it falls in the zero padding.
__device__ __forceinline__ long long in_voxel(int oz, int oy, int ox, int t, int D) {
  const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
  const int iz = 2 * oz + tz - 1, iy = 2 * oy + ty - 1, ix = 2 * ox + tx - 1;
  if (iz < 0 || iy < 0 || ix < 0 || iz >= D || iy >= D || ix >= D) return -1;
  return ((long long)iz * D + iy) * D + ix;
}

// ---------------------------------------------------------------------------
// forward convolution + bias + ReLU.  256 threads = 4 waves; each wave
// computes RB row blocks of 16 output voxels x COUT channels, so that every
// B fragment (weights) it loads serves RB MFMAs.  X: [b][D^3][CIN] (or, with
// LAB, the label window, CIN = 8), Y: [b][Do^3][COUT].
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool LAB, int RB>
__global__ void __launch_bounds__(256) k_conv_fwd(const __bf16* __restrict__ X, LabelWindow lw,
                                                  const __bf16* __restrict__ W, const float* __restrict__ bias,
                                                  __bf16* __restrict__ Y, int D, int batch) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0, "channel counts");
  static_assert(!LAB || CIN == 8, "label input has 8 channels");
  constexpr int KT = 27 * CIN, KS = (KT + 31) / 32, NT = COUT / 16;
  const int Do = D / 2;
  const long long nvo = (long long)Do * Do * Do, total = nvo * batch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long v0 = (long long)blockIdx.x * (64 * RB) + wave * (16 * RB);
  // the voxel whose A row this lane loads, per row block
  bool valid[RB];
  long long bidx[RB];
  int oz[RB], oy[RB], ox[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const long long va = v0 + r * 16 + (lane & 15);
    valid[r] = va < total;
    const long long ba = valid[r] ? va / nvo : 0, ra = valid[r] ? va - ba * nvo : 0;
    bidx[r] = ba;
    oz[r] = int(ra / ((long long)Do * Do));
    oy[r] = int((ra / Do) % Do);
    ox[r] = int(ra % Do);
  }
  f32x4 acc[RB][NT];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 32 + (lane >> 4) * 8;
    const int tap = k / CIN, c0 = k % CIN;
    bf16x8 b[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      b[t] = zero8();
      if (tap < 27) b[t] = ld8(W + ((long long)tap * COUT + t * 16 + (lane & 15)) * CIN + c0);
    }
    const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      bf16x8 a = zero8();
      if (valid[r] && tap < 27) {
        const int iz = 2 * oz[r] + tz - 1, iy = 2 * oy[r] + ty - 1, ix = 2 * ox[r] + tx - 1;
        if (iz >= 0 && iy >= 0 && ix >= 0 && iz < D && iy < D && ix < D) {
          if constexpr (LAB)
            a = onehot8(label_at(lw, bidx[r], iz, iy, ix));
          else
            a = ld8(X + (bidx[r] * (long long)D * D * D + ((long long)iz * D + iy) * D + ix) * CIN + c0);
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = mfma(a, b[t], acc[r][t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + (lane & 15);
    const float bb = bias[co];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long v = v0 + r * 16 + (lane >> 4) * 4 + i;
        if (v < total) Y[v * COUT + co] = (__bf16)fmaxf(acc[r][t][i] + bb, 0.0f);
      }
  }
}

// Forward convolution with the K steps of one 16-voxel row block split over
// the 4 waves of a workgroup (for the deep layers with few voxels and long
// K), partial sums reduced through LDS.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_conv_fwd_splitk(const __bf16* __restrict__ X, const __bf16* __restrict__ W,
                                                         const float* __restrict__ bias, __bf16* __restrict__ Y, int D,
                                                         int batch) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0, "channel counts");
  constexpr int KT = 27 * CIN, KS = (KT + 31) / 32, NT = COUT / 16;
  __shared__ float red[3][NT][64][4];
  const int Do = D / 2;
  const long long nvo = (long long)Do * Do * Do, total = nvo * batch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long v0 = (long long)blockIdx.x * 16;
  const long long va = v0 + (lane & 15);
  const bool valid = va < total;
  const long long ba = valid ? va / nvo : 0, ra = valid ? va - ba * nvo : 0;
  const int oz = int(ra / ((long long)Do * Do)), oy = int((ra / Do) % Do), ox = int(ra % Do);
  const __bf16* Xb = X + ba * (long long)D * D * D * CIN;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = wave; ks < KS; ks += 4) {
    const int k = ks * 32 + (lane >> 4) * 8;
    const int tap = k / CIN, c0 = k % CIN;
    bf16x8 a = zero8();
    if (valid && tap < 27) {
      const int iz = 2 * oz + tap / 9 - 1, iy = 2 * oy + (tap / 3) % 3 - 1, ix = 2 * ox + tap % 3 - 1;
      if (iz >= 0 && iy >= 0 && ix >= 0 && iz < D && iy < D && ix < D)
        a = ld8(Xb + (((long long)iz * D + iy) * D + ix) * CIN + c0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 b = zero8();
      if (tap < 27) b = ld8(W + ((long long)tap * COUT + t * 16 + (lane & 15)) * CIN + c0);
      acc[t] = mfma(a, b, acc[t]);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave - 1][t][lane][i] = acc[t][i];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + (lane & 15);
      const float bb = bias[co];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float sum = acc[t][i] + red[0][t][lane][i] + red[1][t][lane][i] + red[2][t][lane][i];
        const long long v = v0 + (lane >> 4) * 4 + i;
        if (v < total) Y[v * COUT + co] = (__bf16)fmaxf(sum + bb, 0.0f);
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
                                                    int batch, int cls) {
  static_assert(CIN % 16 == 0 && COUT % 32 == 0, "channel counts");
  constexpr int NT = CIN / 16, KC = COUT / 32;
  const int Do = D / 2;
  const int pz = (cls >> 2) & 1, py = (cls >> 1) & 1, px = cls & 1;
  const int h = D / 2;  // voxels per axis in a parity class
  const long long ncls = (long long)h * h * h;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long v0 = (long long)blockIdx.x * 64 + wave * 16;
  const long long va = v0 + (lane & 15);
  const bool valid_a = va < ncls * batch;
  const long long ba = valid_a ? va / ncls : 0, ra = valid_a ? va - ba * ncls : 0;
  const int jz = int(ra / ((long long)h * h)), jy = int((ra / h) % h), jx = int(ra % h);
  const long long nvo = (long long)Do * Do * Do;
  const float* dYb = dY + ba * nvo * COUT;
  const __bf16* Yb = Y + ba * nvo * COUT;
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
        const bool in = valid_a && oz >= 0 && oy >= 0 && ox >= 0 && oz < Do && oy < Do && ox < Do;
        const long long ov = ((long long)oz * Do + oy) * Do + ox;
        for (int kc = 0; kc < KC; ++kc) {
          const int co0 = kc * 32 + (lane >> 4) * 8;
          bf16x8 a = zero8();
          if (in) {
            const float* g = dYb + ov * COUT + co0;
            const bf16x8 yv = ld8(Yb + ov * COUT + co0);
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)((float)yv[j] > 0.0f ? g[j] : 0.0f);
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 b = ld8(Wt + ((long long)tap * CIN + t * 16 + (lane & 15)) * COUT + co0);
            acc[t] = mfma(a, b, acc[t]);
          }
        }
      }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int ci = t * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long v = v0 + (lane >> 4) * 4 + i;
      if (v < ncls * batch) {
        const long long b = v / ncls, r = v - b * ncls;
        const int z = 2 * int(r / ((long long)h * h)) + pz, y = 2 * int((r / h) % h) + py, x = 2 * int(r % h) + px;
        dX[(b * (long long)D * D * D + ((long long)z * D + y) * D + x) * CIN + ci] = acc[t][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient, one tap per block: partial dW[tap][cout][cin] over a chunk
// of output voxels, dZ = dY * (Y > 0).  The chunk of dZ and of the gathered
// input is staged in LDS transposed (channel-major) so that MFMA fragments
// (K = voxels) are 16-byte LDS reads.  The bias gradient rides on tap 13.
// Partials: part[chunk][tap][COUT][CIN], bias partials pb[chunk][COUT].
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool LAB>
__global__ void __launch_bounds__(256) k_conv_wgrad(const float* __restrict__ dY, const __bf16* __restrict__ Y,
                                                    const __bf16* __restrict__ X, LabelWindow lw,
                                                    float* __restrict__ part, float* __restrict__ pb, int D,
                                                    int batch, int chunk) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0 && 256 % COUT == 0, "channel counts");
  static_assert(!LAB || CIN == 8, "label input has 8 channels");
  constexpr int MT = COUT / 16, NTN = (CIN + 15) / 16;  // output tiles (cout x cin)
  constexpr int VS = 32;                                 // voxels per staged step (= MFMA K)
  __shared__ __bf16 sZ[COUT][VS + 8];
  __shared__ __bf16 sX[NTN * 16][VS + 8];
  const int tap = blockIdx.y;
  const int Do = D / 2;
  const long long nvo = (long long)Do * Do * Do, total = nvo * batch;
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
  for (long long vs = vbeg; vs < vend; vs += VS) {
    __syncthreads();
    // stage dZ^T: COUT x VS
    for (int e = threadIdx.x; e < COUT * VS; e += 256) {
      const int co = e % COUT, vl = e / COUT;
      const long long v = vs + vl;
      float z = 0.0f;
      if (v < vend) {
        const float g = dY[v * COUT + co];
        z = (float)Y[v * COUT + co] > 0.0f ? g : 0.0f;
      }
      sZ[co][vl] = (__bf16)z;
      if (tap == 13) bsum += z;  // co == threadIdx.x % COUT since 256 % COUT == 0
    }
    // stage X^T for this tap: CIN x VS (zero rows beyond CIN)
    for (int e = threadIdx.x; e < NTN * 16 * VS; e += 256) {
      const int ci = e % (NTN * 16), vl = e / (NTN * 16);
      const long long v = vs + vl;
      float xv = 0.0f;
      if (v < vend && ci < CIN) {
        const long long b = v / nvo, r = v - b * nvo;
        const int oz = int(r / ((long long)Do * Do)), oy = int((r / Do) % Do), ox = int(r % Do);
        const long long iv = in_voxel(oz, oy, ox, tap, D);
        if (iv >= 0) {
          if constexpr (LAB) {
            const int iz = int(iv / ((long long)D * D)), iy = int((iv / D) % D), ix = int(iv % D);
            xv = label_at(lw, b, iz, iy, ix) == ci ? 1.0f : 0.0f;
          } else {
            xv = (float)X[(b * (long long)D * D * D + iv) * CIN + ci];
          }
        }
      }
      sX[ci][vl] = (__bf16)xv;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tile = wave + 4 * q;
      if (tile < TILES) {
        const int mt = tile / NTN, nt = tile % NTN;
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[j] = sZ[mt * 16 + (lane & 15)][(lane >> 4) * 8 + j];
          b[j] = sX[nt * 16 + (lane & 15)][(lane >> 4) * 8 + j];
        }
        acc[q] = mfma(a, b, acc[q]);
      }
    }
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
                                             float* __restrict__ loss_item, float inv_count) {
  constexpr int C = 64, F = 72, O = 21;
  __shared__ float feat[F];
  __shared__ float dout[O];
  const int b = blockIdx.x, c = threadIdx.x;
  const __bf16* Ab = A + (long long)b * V * C;
  float s = 0.0f;
  for (int v = 0; v < V; ++v) s += (float)Ab[(long long)v * C + c];
  feat[c] = s / float(V);
  if (c < F - C) feat[C + c] = (float(double(cnt[b * (F - C) + c]) * inv_nv) - fmu[c]) * fsc[c];
  __syncthreads();
  if (c < O) {
    float y = bfc[c];
    for (int k = 0; k < F; ++k) y += Wfc[c * F + k] * feat[k];
    out[b * O + c] = y;
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
                       double bound_tol, int* __restrict__ flag) {
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
  flag[it] = bad;
}

// Phase fractions of the n^3 core of each box (one block per item) and the
// Voigt (arithmetic mean of stiffness) and Reuss (inverse of the mean
// compliance) stiffnesses of that mixture, 21 components each.
__global__ void __launch_bounds__(256) k_phase_bounds(const unsigned char* __restrict__ labels, int box, int o, int n,
                                                      int nphase, const double* __restrict__ Cp21,
                                                      const double* __restrict__ Sp21, double* __restrict__ cv21,
                                                      double* __restrict__ cr21) {
  __shared__ int cnt[16];
  const int it = blockIdx.x;
  if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
  __syncthreads();
  const unsigned char* L = labels + (long long)it * box * box * box;
  const long long nv = (long long)n * n * n;
  int local[16];
  for (int p = 0; p < 16; ++p) local[p] = 0;
  for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
    const int z = int(v / (n * n)) + o, y = int((v / n) % n) + o, x = int(v % n) + o;
    const int lab = L[((long long)z * box + y) * box + x];
    if (lab < 16) local[lab] += 1;
  }
  for (int p = 0; p < nphase; ++p)
    if (local[p]) atomicAdd(&cnt[p], local[p]);
  __syncthreads();
  if (threadIdx.x != 0) return;
  double f[16];
  for (int p = 0; p < nphase; ++p) f[p] = double(cnt[p]) / double(nv);
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

// y = x * scale + mean per component (denormalize FP32 network outputs)
__global__ void k_denorm(const float* __restrict__ x, const double* __restrict__ mean,
                         const double* __restrict__ scale, int n, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * 21) y[i] = double(x[i]) * scale[i % 21] + mean[i % 21];
}

}  // namespace cnn
}  // namespace hh
