// Pass kernels of the periodic Fourier-Galerkin elasticity solve on gfx950.
//
// The discrete problem (paper, Appendix A): find the compatible zero-mean
// strain eps* with  G * (C : eps*) = - G * (C : E),  G the projection onto
// compatible fields, solved by conjugate gradients; then average stress and
// strain over Omega_R (Sec. 4).
//
// Data layout (per system = one image and one load case):
//   tmp : 6 strain/stress components of the half spectrum, complex,
//         [z][y][kx][c] with kx in [0, nx/2] and c = 11 22 33 23 13 12
//   ar, ap : residual and search direction, kept in frequency space in their
//         3-vector form: a compatible symmetric field is n (x) a + a (x) n at
//         each frequency (n the unit wave vector), so 3 complex values per
//         frequency describe it exactly and keep it compatible by construction.
//
// One CG iteration is five passes over the spectrum, each a kernel:
//   zinv : p = r + beta p (3-vector), expand to 6 components, inverse z-FFT
//   yinv : inverse y-FFT
//   x    : inverse x-FFT (two real lines per complex line), sigma = C : p,
//          (p, sigma) and region sums in FP64, forward x-FFT
//   yfwd : forward y-FFT
//   zfwd : forward z-FFT, projection to 3-vector form q, r -= alpha q, (r, r)
// with small FP64 finalize kernels for alpha and beta in between.
//
// Numerics: fields and FFTs in T (float or double); every reduction, the CG
// scalars and the averages in double.  (p, A p) equals (p, C:p) because p is
// compatible, so it is formed in real space where C:p is at hand.  x is never
// stored: the averages of eps and sigma are linear in it and are accumulated
// as sum_k alpha_k <p_k>_R and sum_k alpha_k <C:p_k>_R.
#pragma once

#include "fft.hpp"
#include "hh_internal.hpp"
#include "kernels.hpp"

namespace hh {

// LDS budget of one tile.  y/z passes: at least 4 kx columns per tile so
// that every tile row is a whole number of 64-byte sectors (no partial
// writes), except in FP32 above 512 points, where 4 columns would not fit in
// LDS and tiles take 2; x pass: full spectrum rows.
#ifndef HH_LDS_TILE_X
#define HH_LDS_TILE_X (24 * 1024)
#endif
#ifndef HH_LDS_TILE_YZ
#define HH_LDS_TILE_YZ (48 * 1024)
#endif
inline constexpr int kLdsTile = HH_LDS_TILE_X;
inline constexpr int kLdsTileYZ = HH_LDS_TILE_YZ;

// Tile variants: the same kernels compiled for several LDS budgets and
// workgroup sizes.  Variants 0, 1, 2: the default, half and double budget
// (narrower or wider tiles, more or fewer resident workgroups per CU);
// 3 and 4: the default and half budget with at least 256 threads per
// workgroup in the x pass (fewer loads in flight per thread).  The y and z
// passes run variants 3 and 4 as 0 and 1.  The context times the distinct
// ones per shape and keeps the fastest.
constexpr int variant_budget(int base, int v) {
  return (v == 1 || v == 4) ? base / 2 : (v == 2 ? base * 2 : base);
}
constexpr int variant_min_threads(int v) { return v >= 3 ? 256 : 64; }
constexpr int yz_variant(int v) { return v >= 3 ? v - 3 : v; }

constexpr int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
constexpr int round64(int v) { return (v + 63) / 64 * 64; }
constexpr int maxi(int a, int b) { return a > b ? a : b; }
// LDS padding (complex words per block of N1 tile rows): when successive
// blocks would start on the same bank (64 banks of 4 bytes), shift each by
// one row so that the second DFT step of a wave spreads over the banks.
constexpr int lds_pad(int n1, int n2, int L, int cb) {
  return (n2 > 1 && (n1 * L * (cb / 4)) % 64 == 0) ? L : 0;
}

template <int N, class T, int V = 0>
struct AxisCfg {
  static constexpr int N1 = split_n1(N), N2 = N / N1;
  static constexpr int CB = int(sizeof(cx<T>));
  static constexpr int M = clampi(variant_budget(kLdsTileYZ, V) / (N * 6 * CB), CB == 8 && N <= 512 ? 4 : 2, 16);
  static constexpr int L = 6 * M;
  static constexpr int P = lds_pad(N1, N2, L, CB);
  static constexpr int THREADS = clampi(round64(L * maxi(N1, N2)), 64, 512);
  static constexpr int LDS = (N * L + N2 * P + N) * CB;
};

template <int N, class T, int V = 0>
struct XCfg {
  static constexpr int N1 = split_n1(N), N2 = N / N1;
  static constexpr int CB = int(sizeof(cx<T>));
  static constexpr int R = clampi(variant_budget(kLdsTile, V) / (N * 3 * CB), 1, 32);
  static constexpr int L = 3 * R;
  static constexpr int P = lds_pad(N1, N2, L, CB);
  static constexpr int THREADS = clampi(round64(L * maxi(N1, N2)), variant_min_threads(V), 512);
  static constexpr int LDS = (N * L + N2 * P + N) * CB;
  // waves per SIMD that the LDS budget admits (160 KB per CU); in FP32 with
  // register DFTs of at most 16 points the compiler is asked to fit them (at
  // most 6, 80 registers), so that registers do not cut that occupancy
  static constexpr int OCC = clampi((163840 / LDS * (THREADS / 64) + 3) / 4, 1, 8);
  static constexpr int WAVES_HINT = (CB == 8 && N1 <= 16 && N2 <= 16) ? (OCC < 6 ? OCC : 6) : 1;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Signed wave number of FFT index i on an n-point axis; 0 at the Nyquist
// index (nyq set there).
__device__ __forceinline__ int kint(int i, int n, bool& nyq) {
  nyq = (2 * i == n);
  return nyq ? 0 : ((2 * i <= n) ? i : i - n);
}

__device__ __forceinline__ float inv_sqrt(float x) { return __frsqrt_rn(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// Unit wave vector of frequency (kx, ky, kz) in the field precision T, from
// k_d = m_d / N_d; false where the operator is zero.
template <class T>
__device__ __forceinline__ bool unit_k(const GroupArgs& g, int kx, int ky, int kz, T n[3]) {
  bool qx, qy, qz;
  const int mx = kint(kx, g.nx, qx), my = kint(ky, g.ny, qy), mz = kint(kz, g.nz, qz);
  if ((mx == 0 && my == 0 && mz == 0) || (g.nyq_zero && (qx || qy || qz))) {
    n[0] = n[1] = n[2] = T(0);
    return false;
  }
  // reciprocals of the axis lengths are loop invariants of every caller
  const T a = T(mx) * (T(1) / T(g.nx)), b = T(my) * (T(1) / T(g.ny)), c = T(mz) * (T(1) / T(g.nz));
  const T inv = inv_sqrt(a * a + b * b + c * c);
  n[0] = a * inv;
  n[1] = b * inv;
  n[2] = c * inv;
  return true;
}

// Symmetric field n (x) a + a (x) n in components 11 22 33 23 13 12.
template <class T>
__device__ __forceinline__ void expand_sym(const T n[3], const cx<T> a[3], cx<T> e[6]) {
  e[0] = T(2) * n[0] * a[0];
  e[1] = T(2) * n[1] * a[1];
  e[2] = T(2) * n[2] * a[2];
  e[3] = n[1] * a[2] + n[2] * a[1];
  e[4] = n[0] * a[2] + n[2] * a[0];
  e[5] = n[0] * a[1] + n[1] * a[0];
}

// t = S n for the symmetric S given by its 6 components; returns n.S.n.
template <class T>
__device__ __forceinline__ cx<T> sym_dot_n(const cx<T> s[6], const T n[3], cx<T> t[3]) {
  t[0] = n[0] * s[0] + n[1] * s[5] + n[2] * s[4];
  t[1] = n[0] * s[5] + n[1] * s[1] + n[2] * s[3];
  t[2] = n[0] * s[4] + n[1] * s[3] + n[2] * s[2];
  return n[0] * t[0] + n[1] * t[1] + n[2] * t[2];
}

// ||n (x) a + a (x) n||_F^2 = 2 |a|^2 + 2 |n.a|^2
template <class T>
__device__ __forceinline__ double sym_norm2(const T n[3], const cx<T> a[3]) {
  double aa = 0.0;
  for (int i = 0; i < 3; ++i) aa += double(a[i].re) * a[i].re + double(a[i].im) * a[i].im;
  const double nr = double(n[0]) * a[0].re + double(n[1]) * a[1].re + double(n[2]) * a[2].re;
  const double ni = double(n[0]) * a[0].im + double(n[1]) * a[1].im + double(n[2]) * a[2].im;
  return 2.0 * aa + 2.0 * (nr * nr + ni * ni);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// v of another lane of the same row of 16 lanes, by a DPP move (no LDS
// traffic): CTRL 0xB1 and 0x4E are the quad permutations [1 0 3 2] and
// [2 3 0 1]; 0x141 mirrors each half row (lane i <-> 7 - i), 0x140 the row
// (i <-> 15 - i).  Every lane reads a lane of its own row.
template <int CTRL>
__device__ __forceinline__ double dpp_pair(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(u)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(u >> 32)), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (unsigned long long)unsigned(lo) | ((unsigned long long)unsigned(hi) << 32));
}

// Sum of one value over the kLineGroups consecutive lanes of a group (one row
// of 16 lanes): pairs, quads, half rows, rows, each step adding a partner
// lane's partial.  Addition commutes, so every lane of the group ends with
// the same bits, and the tree is the same whatever wave or task the group
// sits in; every lane of the wave must take part.
// Sum over the 64 lanes of a wave in a fixed tree: the butterfly within
// each row of 16 lanes, then the four row sums as (r0 + r1) + (r2 + r3);
// every lane gets the result.
__device__ __forceinline__ double group_sum(double v);
__device__ __forceinline__ double wave_sum_fixed(double v) {
  v = group_sum(v);
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  double r[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(u)), 16 * w));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(u >> 32)), 16 * w));
    r[w] = __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
  }
  return (r[0] + r[1]) + (r[2] + r[3]);
}

__device__ __forceinline__ double group_sum(double v) {
  static_assert(kLineGroups == 16, "butterfly over one row of 16 lanes");
  v += dpp_pair<0xB1>(v);
  v += dpp_pair<0x4E>(v);
  v += dpp_pair<0x141>(v);
  v += dpp_pair<0x140>(v);
  return v;
}

// Sum NV doubles over the block; result valid in thread 0.  scratch holds
// at least (blockDim.x / 64) * NV doubles and is not otherwise in use.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[wid * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += scratch[w * NV + i];
      v[i] = s;
    }
  }
}

template <class T>
__device__ __forceinline__ cx<T>* cptr(void* p, long long off) {
  return reinterpret_cast<cx<T>*>(p) + off;
}

// ---------------------------------------------------------------------------
// Batched tile movement.  Every thread first issues all of its 16-byte
// global loads into registers and only then writes LDS, so a wave keeps
// many requests in flight; LDS row r holds `rowU` 16-byte units.
// ---------------------------------------------------------------------------
template <int ROWS, int ROWU, int THREADS, int N1, int PU, class RowMap>
__device__ __forceinline__ void tile_load(uint4* __restrict__ lds, const uint4* __restrict__ src, int validU,
                                          long long gstride, RowMap map) {
  constexpr int TOTAL = ROWS * ROWU, KMAX = (TOTAL + THREADS - 1) / THREADS;
  uint4 v[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int idx = threadIdx.x + k * THREADS;
    const int r = idx / ROWU, j = idx - r * ROWU;
    v[k] = make_uint4(0u, 0u, 0u, 0u);
    if ((TOTAL % THREADS == 0 || idx < TOTAL) && j < validU) v[k] = src[(long long)map(r) * gstride + j];
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int idx = threadIdx.x + k * THREADS;
    const int r = idx / ROWU;
    if (TOTAL % THREADS == 0 || idx < TOTAL) lds[idx + (PU ? (r / N1) * PU : 0)] = v[k];
  }
}

template <int ROWS, int ROWU, int THREADS, int N1, int PU, class RowMap>
__device__ __forceinline__ void tile_store(const uint4* __restrict__ lds, uint4* __restrict__ dst, int validU,
                                           long long gstride, RowMap map) {
  constexpr int TOTAL = ROWS * ROWU, KMAX = (TOTAL + THREADS - 1) / THREADS;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int idx = threadIdx.x + k * THREADS;
    const int r = idx / ROWU, j = idx - r * ROWU;
    if ((TOTAL % THREADS == 0 || idx < TOTAL) && j < validU)
      dst[(long long)map(r) * gstride + j] = lds[idx + (PU ? (r / N1) * PU : 0)];
  }
}

template <class T>
struct alignas(2 * sizeof(cx<T>)) cpair {
  cx<T> a, b;
};

// ---------------------------------------------------------------------------
// z pass
// ---------------------------------------------------------------------------
template <int N, class T, int MODE, int V>
__global__ void __launch_bounds__((AxisCfg<N, T, V>::THREADS)) k_zpass(GroupArgs g) {
  using Cf = AxisCfg<N, T, V>;
  constexpr int N1 = Cf::N1, N2 = Cf::N2, TH = Cf::THREADS;
  constexpr int CB = Cf::CB;
  constexpr int M = Cf::M, L = 6 * M, ROWU = L * CB / 16, P = Cf::P, PU = P * CB / 16;
  constexpr int KT = (N * M + TH - 1) / TH;  // (z, kx) tasks per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;

  const int s = blockIdx.y;
  SysState* st = g.state + s;
  if (MODE != kZFwdRhs && st->status != kRunning) return;
  const int ntx = (g.hx + Cf::M - 1) / Cf::M;
  const int y = blockIdx.x / ntx;
  const int kx0 = (blockIdx.x % ntx) * Cf::M;
  const int mk = min(M, g.hx - kx0);  // valid columns of this tile
  const int validU = 6 * mk * CB / 16;
  cx<T>* tmp = cptr<T>(g.tmp, s * g.tmp_stride);
  cx<T>* ar = cptr<T>(g.ar, s * g.a_stride);
  cx<T>* ap = cptr<T>(g.ap, s * g.a_stride);
  const long long plane = (long long)g.ny * g.hxp;  // frequencies per z plane (padded rows)
  uint4* tile_g = reinterpret_cast<uint4*>(tmp + ((long long)y * g.hxp + kx0) * 6);
  const long long gstride = plane * 6 * CB / 16;
  constexpr int ntask = N * M;
  // 3-vector fields are stored tile-major: [tile = blockIdx.x][z][kxl][3]
  const long long atile = (long long)blockIdx.x * N * M * 3;

  fill_twiddles<N, T>(tw);

  if constexpr (MODE == kZInvCg || MODE == kZInvFp) {
    const T beta = T(st->beta);
    cx<T> ra[KT][3], pa[KT][3];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int task = threadIdx.x + k * TH;
      const int kxl = task % M, z = task / M;
      if (task < ntask && kxl < mk) {
        const long long off = atile + (z * M + kxl) * 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) ra[k][i] = ar[off + i];
        if constexpr (MODE == kZInvCg) {
#pragma unroll
          for (int i = 0; i < 3; ++i) pa[k][i] = ap[off + i];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int task = threadIdx.x + k * TH;
      const int kxl = task % M, z = task / M, kx = kx0 + kxl;
      if (task < ntask && kxl >= mk) {
#pragma unroll
        for (int c = 0; c < 6; ++c) buf[lds_at<N1, P>(z, L) + kxl * 6 + c] = cx<T>{T(0), T(0)};
      } else if (task < ntask) {
        cx<T> a[3];
        if constexpr (MODE == kZInvCg) {
          const long long off = atile + (z * M + kxl) * 3;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            a[i] = ra[k][i] + beta * pa[k][i];
            ap[off + i] = a[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i) a[i] = ra[k][i];
        }
        T n[3];
        unit_k<T>(g, kx, y, z, n);
        cx<T> e[6];
        expand_sym(n, a, e);
#pragma unroll
        for (int c = 0; c < 6; ++c) buf[lds_at<N1, P>(z, L) + kxl * 6 + c] = e[c];
      }
    }
    __syncthreads();
    fft_nat2perm<N1, N2, +1, T, P>(buf, L, tw);
    tile_store<N, ROWU, TH, N1, PU>(reinterpret_cast<const uint4*>(buf), tile_g, validU, gstride,
                            [](int pos) { return perm_idx<N1, N2>(pos); });
  } else {
    // prefetch the residual for the epilogue together with the tile
    cx<T> ra[KT][3];
    if constexpr (MODE != kZFwdRhs) {
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int task = threadIdx.x + k * TH;
        const int kxl = task % M, kz = perm_idx<N1, N2>(task / M);
        if (task < ntask && kxl < mk) {
          const long long off = atile + (kz * M + kxl) * 3;
#pragma unroll
          for (int i = 0; i < 3; ++i) ra[k][i] = ar[off + i];
        }
      }
    }
    tile_load<N, ROWU, TH, N1, PU>(reinterpret_cast<uint4*>(buf), tile_g, validU, gstride,
                                   [](int r) { return r; });
    __syncthreads();
    fft_nat2perm<N1, N2, -1, T, P>(buf, L, tw);
    const T alpha = T(st->alpha);
    const T g1 = T(0.5 / g.ref_mu);
    const T g2 = T((g.ref_lam + g.ref_mu) / (g.ref_lam + 2.0 * g.ref_mu));
    double val[KT];  // per-frequency terms of the column sums
#pragma unroll
    for (int k = 0; k < KT; ++k) val[k] = 0.0;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int task = threadIdx.x + k * TH;
      const int kxl = task % M, pos = task / M, kx = kx0 + kxl;
      if (task < ntask && kxl < mk) {
        const int kz = perm_idx<N1, N2>(pos);
        cx<T> sg[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = buf[lds_at<N1, P>(pos, L) + kxl * 6 + c];
        T n[3];
        const bool live = unit_k<T>(g, kx, y, kz, n);
        cx<T> t[3];
        const cx<T> ntn = sym_dot_n(sg, n, t);
        cx<T> q[3];  // 3-vector form of the projection of sigma
#pragma unroll
        for (int i = 0; i < 3; ++i) q[i] = live ? t[i] - (T(0.5) * n[i]) * ntn : cx<T>{T(0), T(0)};
        const long long off = atile + (kz * M + kxl) * 3;
        const double w = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
        cx<T> r[3];
        if constexpr (MODE == kZFwdCg) {
#pragma unroll
          for (int i = 0; i < 3; ++i) r[i] = ra[k][i] - alpha * q[i];
          val[k] = w * sym_norm2(n, r);
        } else if constexpr (MODE == kZFwdRhs) {
#pragma unroll
          for (int i = 0; i < 3; ++i) r[i] = cx<T>{-q[i].re, -q[i].im};
          val[k] = w * sym_norm2(n, r);
        } else {  // basic fixed point: eps* <- eps* - Gamma0 sigma
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const cx<T> gi = live ? g1 * (t[i] - (g2 * n[i]) * ntn) : cx<T>{T(0), T(0)};
            r[i] = ra[k][i] - gi;
          }
          val[k] = w * sym_norm2(n, q);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) ar[off + i] = r[i];
      }
    }
    // column sums over z: staged by (column, position); one wave per
    // column, lane g summing positions g, g + 64, ... in order, then the
    // butterfly over each row of 16 lanes and the four row sums in a fixed
    // order (every wave of every tile variant forms the same tree)
    __syncthreads();
    double* vd = reinterpret_cast<double*>(buf);  // [M][N]
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int task = threadIdx.x + k * TH;
      if (task < ntask) vd[(task % M) * N + task / M] = val[k];
    }
    __syncthreads();
    static_assert(TH % 64 == 0, "whole waves");
    constexpr int NC = M * kColGroups, KC = (NC + TH - 1) / TH;
    double* pcol = g.part_z + (long long)s * g.ncol_z + (long long)y * g.hx + kx0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int q = threadIdx.x + k * TH;
      const int kxl = q / kColGroups, gq = q % kColGroups;
      const bool task = (NC % TH == 0 || q < NC) && kxl < mk;
      double a = 0.0;
      if (task)
        for (int pos = gq; pos < N; pos += kColGroups) a += vd[kxl * N + pos];
      a = wave_sum_fixed(a);
      if (task && gq == 0) pcol[kxl] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// y pass (plain FFT along y of the 6-component spectrum, in place)
// ---------------------------------------------------------------------------
template <int N, class T, int S, int V>
__global__ void __launch_bounds__((AxisCfg<N, T, V>::THREADS)) k_ypass(GroupArgs g) {
  using Cf = AxisCfg<N, T, V>;
  constexpr int N1 = Cf::N1, N2 = Cf::N2, TH = Cf::THREADS, CB = Cf::CB;
  constexpr int M = Cf::M, L = 6 * M, ROWU = L * CB / 16, P = Cf::P, PU = P * CB / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;
  const int s = blockIdx.y;
  if (g.state[s].status != kRunning) return;
  const int ntx = (g.hx + Cf::M - 1) / Cf::M;
  const int z = blockIdx.x / ntx;
  const int kx0 = (blockIdx.x % ntx) * Cf::M;
  const int mk = min(M, g.hx - kx0);
  const int validU = 6 * mk * CB / 16;
  uint4* tile_g = reinterpret_cast<uint4*>(cptr<T>(g.tmp, s * g.tmp_stride) +
                                           ((long long)z * g.ny * g.hxp + kx0) * 6);
  const long long gstride = (long long)g.hxp * 6 * CB / 16;
  fill_twiddles<N, T>(tw);
  tile_load<N, ROWU, TH, N1, PU>(reinterpret_cast<uint4*>(buf), tile_g, validU, gstride,
                                 [](int r) { return r; });
  __syncthreads();
  fft_nat2perm<N1, N2, S, T, P>(buf, L, tw);
  tile_store<N, ROWU, TH, N1, PU>(reinterpret_cast<const uint4*>(buf), tile_g, validU, gstride,
                          [](int pos) { return perm_idx<N1, N2>(pos); });
}

// ---------------------------------------------------------------------------
// x pass: C2R, constitutive law, reductions, R2C
// ---------------------------------------------------------------------------
template <int N, class T, int MODE, int V>
__global__ void __launch_bounds__((XCfg<N, T, V>::THREADS))
__attribute__((amdgpu_waves_per_eu(XCfg<N, T, V>::WAVES_HINT))) k_xpass(GroupArgs g) {
  using Cf = XCfg<N, T, V>;
  constexpr int N1 = Cf::N1, N2 = Cf::N2, TH = Cf::THREADS;
  constexpr int R = Cf::R, L = 3 * R, P = Cf::P;
  constexpr int HX = N / 2 + 1, HXP = spectrum_pitch(HX);  // spectrum row length and pitch
  constexpr int NU = R * HX * 3;                          // (row, kx, pair) units per tile
  constexpr int KX = (NU + TH - 1) / TH;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;
  __shared__ T s_lam[kMaxPhase], s_mu[kMaxPhase];
  __shared__ unsigned char s_rin[R];  // tile row inside the averaging region (y and z)
  __shared__ cx<T> s_dc[L];           // kx = 0 input of each line (its sum over x is N times this)

  const int s = blockIdx.y;
  SysState* st = g.state + s;
  if (MODE != kXRhs && st->status != kRunning) return;
  const SysDesc sd = g.sys[s];
  const ItemDesc& it = g.items[sd.item];
  const int rows = g.ny * g.nz;
  const int r0 = blockIdx.x * R;
  const int nr = min(R, rows - r0);  // rows of this tile; the rest are zero lines
  cx<T>* tmp = cptr<T>(g.tmp, s * g.tmp_stride) + (long long)r0 * HXP * 6;
  cpair<T>* tmpp = reinterpret_cast<cpair<T>*>(tmp);  // 3 pairs per frequency

  // Units (row, kx, pair) of the spectrum tile.  LM (line mapping; the
  // workgroup has at least N1 threads per LDS line): thread j of line l = 3 row + pair
  // takes kx = j + N1 k, so the LDS positions of kx and N - kx step by a
  // compile-time stride and no index is divided; the 3 N1 threads of a row
  // still read 3 N1 consecutive pairs.  Otherwise unit f = thread + k TH.
  constexpr bool LM = TH >= N1 * L && N % 2 == 0;  // threads past N1 L idle in the unit loops
  constexpr int KXL = (HX + N1 - 1) / N1;  // kx per thread with LM
  constexpr int KU = LM ? KXL : KX;
  const int lj = threadIdx.x % N1, lln = threadIdx.x / N1;  // LM: kx offset, line
  const int lrl = lln / 3, lpr = lln - 3 * (lln / 3);       // LM: row, pair
  // issue this tile's global loads first: nothing they need waits on memory
  cpair<T> v[KU];
  if constexpr (MODE != kXRhs) {
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      if constexpr (LM) {
        const int kx = lj + N1 * k;
        if ((KXL * N1 == HX || kx < HX) && lrl < nr) v[k] = tmpp[(lrl * HXP + kx) * 3 + lpr];
      } else {
        const int f = threadIdx.x + k * TH;
        const int pr = f % 3, q = f / 3, kx = q % HX, rl = q / HX;
        if ((NU % TH == 0 || f < NU) && rl < nr) v[k] = tmpp[(rl * HXP + kx) * 3 + pr];
      }
    }
  }
  fill_twiddles<N, T>(tw);
  if (threadIdx.x < kMaxPhase) {
    const int i = threadIdx.x < it.nphase ? threadIdx.x : 0;
    s_lam[threadIdx.x] = T(it.lam[i]);
    s_mu[threadIdx.x] = T(it.mu[i]);
  }
  if (threadIdx.x < R) {
    const int row = r0 + threadIdx.x, zr = row / g.ny, yr = row - zr * g.ny;
    s_rin[threadIdx.x] = threadIdx.x < nr && yr >= it.region[1] && yr < it.region[4] && zr >= it.region[2] &&
                         zr < it.region[5];
  }

  // labels of this thread's voxels, fetched before anything waits on memory
  constexpr int KE = (R * N + TH - 1) / TH;
  int lab_pre[KE];
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int task = threadIdx.x + k * TH;
    const int rl = task % R, pos = task / R;
    lab_pre[k] = 0;
    if (!g.aniso && (R * N % TH == 0 || task < R * N) && rl < nr)
      lab_pre[k] = g.labels[it.lab_off + (long long)(r0 + rl) * N + perm_idx<N1, N2>(pos)];
  }

  if constexpr (MODE != kXRhs) {
    // unpack: complex line (pair) = A + i B with A, B the spectra of two real lines
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      int kx, rl, l;
      bool in;
      if constexpr (LM) {
        kx = lj + N1 * k;
        rl = lrl;
        l = lln;
        in = (KXL * N1 == HX || kx < HX) && (TH == N1 * L || lln < L);
      } else {
        const int f = threadIdx.x + k * TH;
        const int pr = f % 3, q = f / 3;
        kx = q % HX;
        rl = q / HX;
        l = rl * 3 + pr;
        in = NU % TH == 0 || f < NU;
      }
      if (in) {
        cx<T> A = v[k].a, B = v[k].b;
        if (rl >= nr) A = B = cx<T>{T(0), T(0)};
        if (kx == 0 || 2 * kx == N) {
          buf[lds_at<N1, P>(kx, L) + l] = cx<T>{A.re, B.re};
          if (kx == 0) s_dc[l] = cx<T>{A.re, B.re};
        } else {
          buf[lds_at<N1, P>(kx, L) + l] = cx<T>{A.re - B.im, A.im + B.re};
          buf[lds_at<N1, P>(N - kx, L) + l] = cx<T>{A.re + B.im, B.re - A.im};
        }
      }
    }
    __syncthreads();
    fft_nat2perm<N1, N2, +1, T, P>(buf, L, tw);
  } else {
    __syncthreads();
  }

  // constitutive law on the voxels of this tile (positions are permuted)
  const T invV = T(1.0 / (double(N) * g.ny * g.nz));
  T E[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) E[c] = T(g.loads[sd.load][c]);
  const int x0 = it.region[0], y0 = it.region[1], z0 = it.region[2];
  const int x1 = it.region[3], y1 = it.region[4], z1 = it.region[5];
  // Whole-box region: sum p = 0 (p is zero-mean) and the row sums of sigma
  // are the kx = 0 outputs of the forward transform, so no per-voxel sums.
  const bool whole = x0 == 0 && x1 == N && y0 == 0 && y1 == g.ny && z0 == 0 && z1 == g.nz;
  double* prow = g.part_x + ((long long)s * g.nrow_x + r0) * kPartX;  // row sums of this tile
  // Region sums of one field held in buf (p before the law, sigma after it),
  // per line l = 3 row + pair.  The region's x range [x0, x1) holds K
  // points; the summed set S is that range when K <= N - K and its
  // complement otherwise, the region's sum then being the line's total
  // minus the complement's (the total comes from the transform: N times
  // the kx = 0 input for p, the kx = 0 output for sigma).  The elements of
  // S in increasing x are summed in kLineGroups groups, group g taking
  // elements g, g + kLineGroups, ... in order, and the groups are added in
  // a butterfly; the result sits in the group-0 lane of each line's task.
  constexpr int NQ = 3 * R * kLineGroups;
  constexpr int KQ = (NQ + TH - 1) / TH;
  // Every task of a thread has the same group (the thread count is a
  // multiple of kLineGroups); the LDS offsets of its elements of S are
  // found once (kept in registers for lines up to 256 points).
  constexpr int NJS = (N / 2 + kLineGroups - 1) / kLineGroups;  // |S| <= N / 2
  constexpr bool kOffRegs = NJS <= 8;
  const int gq = threadIdx.x % kLineGroups;
  const int K = x1 - x0;
  const bool comp = N - K < K;
  const int KS = comp ? N - K : K;
  auto s_off = [&](int j) -> int {  // LDS offset of element gq + kLineGroups j of S, -1 past its end
    const int i = gq + kLineGroups * j;
    if (i >= KS) return -1;
    const int x = comp ? (i < x0 ? i : x1 + (i - x0)) : x0 + i;
    return lds_at<N1, P>((x % N2) * N1 + x / N2, L);  // position of x (inverse of perm_idx)
  };
  int soff[kOffRegs ? NJS : 1];
  if constexpr (kOffRegs) {
    if (!whole) {
#pragma unroll
      for (int j = 0; j < NJS; ++j) soff[j] = s_off(j);
    }
  }
  auto region_sums = [&](double (&sr)[KQ], double (&si)[KQ]) {
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      const int q = threadIdx.x + k * TH;
      const int l = q / kLineGroups;
      const int rl = l / 3;
      const bool rin = (NQ % TH == 0 || q < NQ) && rl < nr && s_rin[rl];
      double a = 0.0, b = 0.0;
      if (rin) {
#pragma unroll
        for (int j = 0; j < NJS; ++j) {
          int o;
          if constexpr (kOffRegs) o = soff[j];
          else o = s_off(j);
          if (o >= 0) {
            const cx<T> v = buf[o + l];
            a += double(v.re);
            b += double(v.im);
          }
        }
      }
      if (__ballot(rin) != 0ull) {  // a wave without region rows has only zeros to add
        a = group_sum(a);
        b = group_sum(b);
      }
      sr[k] = a;
      si[k] = b;
    }
  };
  // the sums' entries base + 2 pair, + 1 of each row, from S's sums and the
  // lines' totals; zero outside the region
  auto region_write = [&](int base, const double (&sr)[KQ], const double (&si)[KQ], const cx<T>* tot,
                          double tscale, double scale, bool add_e) {
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      const int q = threadIdx.x + k * TH;
      const int l = q / kLineGroups;
      const int rl = l / 3, pr = l - 3 * (l / 3);
      if ((NQ % TH == 0 || q < NQ) && rl < nr && gq == 0) {
        double a = 0.0, b = 0.0;
        if (s_rin[rl]) {
          a = sr[k];
          b = si[k];
          if (comp) {
            const cx<T> t = tot[l];
            a = tscale * double(t.re) - a;
            b = tscale * double(t.im) - b;
          }
          a *= scale;
          b *= scale;
          if (add_e) {
            a += double(K) * double(E[2 * pr]);
            b += double(K) * double(E[2 * pr + 1]);
          }
        }
        prow[(long long)rl * kPartX + base + 2 * pr] = a;
        prow[(long long)rl * kPartX + base + 2 * pr + 1] = b;
      }
    }
  };
  if (MODE != kXRhs && !whole) {
    double sr[KQ], si[KQ];
    region_sums(sr, si);
    region_write(1, sr, si, s_dc, double(N), 1.0 / (double(N) * g.ny * g.nz), MODE == kXFp);
  }
  if (MODE == kXRhs && !whole) {
    // the right-hand side's p is the constant E
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      const int q = threadIdx.x + k * TH;
      const int l = q / kLineGroups;
      const int rl = l / 3, pr = l - 3 * (l / 3);
      if ((NQ % TH == 0 || q < NQ) && rl < nr && gq == 0) {
        const bool rin = s_rin[rl];
        prow[(long long)rl * kPartX + 1 + 2 * pr] = rin ? double(K) * double(E[2 * pr]) : 0.0;
        prow[(long long)rl * kPartX + 2 + 2 * pr] = rin ? double(K) * double(E[2 * pr + 1]) : 0.0;
      }
    }
  }
  // per-voxel values of the row sums of (p, C:p) (CG) or (C:E, C:E) (RHS)
  double pv[KE];
#pragma unroll
  for (int k = 0; k < KE; ++k) pv[k] = 0.0;
  if (!whole) __syncthreads();  // the region sums of p have read buf
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int task = threadIdx.x + k * TH;
    if (R * N % TH != 0 && task >= R * N) break;
    const int rl = task % R, pos = task / R;
    const int x = perm_idx<N1, N2>(pos);
    const int row = r0 + rl;
    const bool valid = rl < nr;
    T p[6];
    if constexpr (MODE == kXRhs) {
#pragma unroll
      for (int c = 0; c < 6; ++c) p[c] = valid ? E[c] : T(0);
    } else {
#pragma unroll
      for (int pr = 0; pr < 3; ++pr) {
        const cx<T> v = buf[lds_at<N1, P>(pos, L) + rl * 3 + pr];
        p[2 * pr] = v.re * invV;
        p[2 * pr + 1] = v.im * invV;
      }
      if constexpr (MODE == kXFp) {
#pragma unroll
        for (int c = 0; c < 6; ++c) p[c] += valid ? E[c] : T(0);
      }
    }
    const long long vox = (long long)row * N + x;
    T sg[6];
    if (!valid) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = T(0);
    } else if (g.aniso) {
      const T* Cv = reinterpret_cast<const T*>(g.cfield) + it.cf_off + vox * 21;
      // sigma_V = C_V eps_eng with eps_eng = (e11 e22 e33 2e23 2e13 2e12)
      const T ee[6] = {p[0], p[1], p[2], T(2) * p[3], T(2) * p[4], T(2) * p[5]};
      T Cm[6][6];
      int kk = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
          Cm[i][j] = Cv[kk];
          Cm[j][i] = Cv[kk];
          ++kk;
        }
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        T a = T(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) a += Cm[i][j] * ee[j];
        sg[i] = a;
      }
    } else {
      const int lab = lab_pre[k];
      const T lam = s_lam[lab], mu2 = T(2) * s_mu[lab];
      const T tr = lam * (p[0] + p[1] + p[2]);
#pragma unroll
      for (int c = 0; c < 6; ++c) sg[c] = mu2 * p[c] + (c < 3 ? tr : T(0));
    }
    if (valid) {
      if constexpr (MODE == kXRhs) {
        double ss = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) ss += (c < 3 ? 1.0 : 2.0) * double(sg[c]) * sg[c];
        pv[k] = ss;
      } else if constexpr (MODE == kXCg) {
        // p : C : p >= 0 per voxel, formed in T and summed in double
        T ps = T(0);
#pragma unroll
        for (int c = 0; c < 6; ++c) ps += (c < 3 ? T(1) : T(2)) * p[c] * sg[c];
        pv[k] = double(ps);
      }
    }
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) buf[lds_at<N1, P>(pos, L) + rl * 3 + pr] = cx<T>{sg[2 * pr], sg[2 * pr + 1]};
  }
  __syncthreads();
  double ssr[KQ], ssi[KQ];  // sigma's sums over S, completed after the transform
  if (!whole) {
    region_sums(ssr, ssi);
    __syncthreads();  // buf is read above and transformed below
  }
  fft_perm2nat<N1, N2, -1, T, P>(buf, L, tw);
  if (!whole) {
    // the kx = 0 output of line l is the line's total of sigma
    const cx<T>* tot = buf + lds_at<N1, P>(0, L);
    region_write(7, ssr, ssi, tot, 1.0, 1.0, false);
  }
  // whole box: the kx = 0 output of line row * 3 + pair is the row sum of
  // sigma components 2 pair (re) and 2 pair + 1 (im); the row sums of p are
  // 0, or N E in FP mode (p carries E there)
  if (whole) {
    for (int l = threadIdx.x; l < 3 * nr; l += TH) {
      const int rl = l / 3, pr = l - 3 * (l / 3);
      const cx<T> z0v = buf[lds_at<N1, P>(0, L) + l];
      double* o = prow + (long long)rl * kPartX;
      o[7 + 2 * pr] = double(z0v.re);
      o[8 + 2 * pr] = double(z0v.im);
      o[1 + 2 * pr] = MODE == kXFp ? double(N) * double(E[2 * pr]) : 0.0;
      o[2 + 2 * pr] = MODE == kXFp ? double(N) * double(E[2 * pr + 1]) : 0.0;
    }
  }
  auto pack = [&](int kx, int rl, int pr) {
    const int l = rl * 3 + pr;
    const cx<T> zk = buf[lds_at<N1, P>(kx, L) + l];
    const cx<T> zm = buf[lds_at<N1, P>((N - kx) % N, L) + l];
    cpair<T> o;
    o.a = cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
    o.b = cx<T>{T(0.5) * (zk.im + zm.im), T(0.5) * (zm.re - zk.re)};
    tmpp[(rl * HXP + kx) * 3 + pr] = o;
  };
  if constexpr (LM) {
#pragma unroll
    for (int k = 0; k < KXL; ++k) {
      const int kx = lj + N1 * k;
      if ((KXL * N1 == HX || kx < HX) && lrl < nr) pack(kx, lrl, lpr);
    }
  } else {
    for (int f = threadIdx.x; f < NU; f += TH) {
      const int pr = f % 3, q = f / 3, kx = q % HX, rl = q / HX;
      if (rl < nr) pack(kx, rl, pr);
    }
  }
  __syncthreads();
  // row sums of the per-voxel values: staged by position, then each row in
  // kLineGroups groups and a butterfly
  double* vs = reinterpret_cast<double*>(buf);  // [R][N]
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int task = threadIdx.x + k * TH;
    if (R * N % TH == 0 || task < R * N) vs[(task % R) * N + task / R] = pv[k];
  }
  __syncthreads();
  if constexpr (MODE != kXFp) {
    constexpr int NR = R * kLineGroups, KR = (NR + TH - 1) / TH;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int q = threadIdx.x + k * TH;
      const int rl = q / kLineGroups, gq = q % kLineGroups;
      double a = 0.0;
      if ((NR % TH == 0 || q < NR) && rl < nr)
        for (int pos = gq; pos < N; pos += kLineGroups) a += vs[rl * N + pos];
      a = group_sum(a);
      if ((NR % TH == 0 || q < NR) && rl < nr && gq == 0) prow[(long long)rl * kPartX] = a;
    }
  } else {
    for (int rl = threadIdx.x; rl < nr; rl += TH) prow[(long long)rl * kPartX] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int N, class T, int V>
struct Ops {
  static void z(int mode, const GroupArgs& g, hipStream_t st) {
    using Cf = AxisCfg<N, T, V>;
    const dim3 grid(g.ny * ((g.hx + Cf::M - 1) / Cf::M), g.nsys);
    switch (mode) {
      case kZInvCg: k_zpass<N, T, kZInvCg, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kZFwdCg: k_zpass<N, T, kZFwdCg, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kZFwdRhs: k_zpass<N, T, kZFwdRhs, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kZInvFp: k_zpass<N, T, kZInvFp, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kZFwdFp: k_zpass<N, T, kZFwdFp, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
    }
  }
  static void y(int dir, const GroupArgs& g, hipStream_t st) {
    using Cf = AxisCfg<N, T, V>;
    const dim3 grid(g.nz * ((g.hx + Cf::M - 1) / Cf::M), g.nsys);
    if (dir < 0) k_ypass<N, T, -1, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g);
    else k_ypass<N, T, +1, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g);
  }
  static void x(int mode, const GroupArgs& g, hipStream_t st) {
    using Cf = XCfg<N, T, V>;
    const dim3 grid((g.ny * g.nz + Cf::R - 1) / Cf::R, g.nsys);
    switch (mode) {
      case kXCg: k_xpass<N, T, kXCg, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kXRhs: k_xpass<N, T, kXRhs, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
      case kXFp: k_xpass<N, T, kXFp, V><<<grid, Cf::THREADS, Cf::LDS, st>>>(g); break;
    }
  }
};

// The lowest-numbered variant with the same tile configuration as V, so
// that variants which coincide at a size share one set of kernels.
template <int N, class T, int V, int U = 0>
constexpr int canon_x() {
  if constexpr (U >= V) {
    return V;
  } else if constexpr (XCfg<N, T, U>::R == XCfg<N, T, V>::R && XCfg<N, T, U>::THREADS == XCfg<N, T, V>::THREADS) {
    return U;
  } else {
    return canon_x<N, T, V, U + 1>();
  }
}
template <int N, class T, int V, int U = 0>
constexpr int canon_yz() {
  if constexpr (U >= V) {
    return V;
  } else if constexpr (AxisCfg<N, T, U>::M == AxisCfg<N, T, V>::M &&
                       AxisCfg<N, T, U>::THREADS == AxisCfg<N, T, V>::THREADS) {
    return U;
  } else {
    return canon_yz<N, T, V, U + 1>();
  }
}

template <int N, class T, int V>
void size_ops_impl(int what, int mode, const GroupArgs* g, hipStream_t st, int* info) {
  constexpr int VZ = canon_yz<N, T, yz_variant(V)>();
  constexpr int VX = canon_x<N, T, V>();
  switch (what) {
    case kOpZ: Ops<N, T, VZ>::z(mode, *g, st); break;
    case kOpY: Ops<N, T, VZ>::y(mode, *g, st); break;
    case kOpX: Ops<N, T, VX>::x(mode, *g, st); break;
    case kOpInfoZ: *info = AxisCfg<N, T, VZ>::M; break;
    case kOpInfoX: *info = XCfg<N, T, VX>::R; break;
    case kOpInfoLdsZ: *info = AxisCfg<N, T, VZ>::LDS; break;
    case kOpInfoLdsX: *info = XCfg<N, T, VX>::LDS; break;
    case kOpInfoThreadsZ: *info = AxisCfg<N, T, VZ>::THREADS; break;
    case kOpInfoThreadsX: *info = XCfg<N, T, VX>::THREADS; break;
  }
}

// FP32 sizes have all tile variants, FP64 sizes the default one.
#define HH_CASE_F(N)                              \
  case N:                                         \
    return v == 1   ? &size_ops_impl<N, float, 1> \
           : v == 2 ? &size_ops_impl<N, float, 2> \
           : v == 3 ? &size_ops_impl<N, float, 3> \
           : v == 4 ? &size_ops_impl<N, float, 4> \
                    : &size_ops_impl<N, float, 0>;
#define HH_CASE_D(N) \
  case N:            \
    return v == 0 ? &size_ops_impl<N, double, 0> : nullptr;

}  // namespace hh
