// Hierarchical-scheme data movement and small utility kernels.
//
// Partition + padding (paper, Sec. 3 and Sec. 4 / Fig. 4): every n^3 block
// of the image is copied with p voxels of surrounding material on each side
// into a contiguous pack of (n + 2p)^3 boxes; indices wrap periodically at
// the image edge.
#include <hip/hip_runtime.h>

#include "hh_internal.hpp"
#include "intdiv.hpp"
#include "kernels.hpp"

namespace hh {

// Copy of the boxes: grid (row blocks of kGatherRows box rows, items).  The
// block's rows are cut into W-byte chunks (cw per row); W is chosen by the
// launcher so that every chunk maps to W aligned, contiguous source bytes
// (no wrap inside a chunk).  The source row (z, y) wraps once per row and x
// once per chunk (p < nx, so one step suffices).  Each thread issues kGatherU
// chunk loads before their stores.
constexpr int kGatherRows = 256, kGatherU = 4;

template <int W>
__global__ void __launch_bounds__(256) k_gather_pad(const unsigned char* __restrict__ img, int nx, int ny, int nz,
                                                    int n, int p, int mx, int my, int item0, int cw, float inv_cw,
                                                    float inv_b, unsigned char* __restrict__ out) {
  using CT = typename Chunk<W>::type;
  const int b = n + 2 * p;
  const int item = item0 + blockIdx.y;
  const int bx = item % mx, by = (item / mx) % my, bz = item / (mx * my);
  const int r0 = blockIdx.x * kGatherRows, nr = min(kGatherRows, b * b - r0);
  const int tasks = nr * cw;
  const int x0 = bx * n - p;
  unsigned char* dst_item = out + (long long)item * b * b * b;
  for (int t0 = threadIdx.x; t0 < tasks; t0 += 256 * kGatherU) {
    CT v[kGatherU];
    long long d[kGatherU];
#pragma unroll
    for (int u = 0; u < kGatherU; ++u) {
      const int t = t0 + u * 256;
      d[u] = -1;
      if (t < tasks) {
        const int rl = fdiv(t, cw, inv_cw), k = t - rl * cw;
        const int r = r0 + rl, zz = fdiv(r, b, inv_b), yy = r - zz * b;
        int z = bz * n - p + zz, y = by * n - p + yy, x = x0 + k * W;
        z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
        y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
        v[u] = *reinterpret_cast<const CT*>(img + ((long long)z * ny + y) * nx + x);
        d[u] = (long long)r * b + k * W;
      }
    }
#pragma unroll
    for (int u = 0; u < kGatherU; ++u)
      if (d[u] >= 0) *reinterpret_cast<CT*>(dst_item + d[u]) = v[u];
  }
}

// Boxes of an intermediate image of 21-component stiffnesses (the next
// level of repeated coarse-graining): grid (box voxel blocks of 256, items);
// one thread copies the 21 values of one box voxel from its wrapped source.
template <class T>
__global__ void __launch_bounds__(256) k_gather_field(const T* __restrict__ src, int mx, int my, int mz, int n,
                                                      int p, int item0, T* __restrict__ out) {
  const int b = n + 2 * p, nb3 = b * b * b;
  const int item = item0 + blockIdx.y;
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= nb3) return;
  const int bx = mx / n, by = my / n;  // blocks per axis
  const int ix = item % bx, iy = (item / bx) % by, iz = item / (bx * by);
  const int zz = v / (b * b), yy = (v / b) % b, xx = v % b;
  int z = iz * n - p + zz, y = iy * n - p + yy, x = ix * n - p + xx;
  z = z < 0 ? z + mz : (z >= mz ? z - mz : z);
  y = y < 0 ? y + my : (y >= my ? y - my : y);
  x = x < 0 ? x + mx : (x >= mx ? x - mx : x);
  const T* s = src + (((long long)z * my + y) * mx + x) * 21;
  T* d = out + ((long long)item * nb3 + v) * 21;
#pragma unroll
  for (int c = 0; c < 21; ++c) d[c] = s[c];
}

// Largest label of each item: blockIdx.y = item, blocks along x split it.
// The item's 16-byte-aligned body goes in 16-byte loads, its even and odd
// bytes kept as packed 16-bit maxima; the few bytes before and after it
// one at a time.
__global__ void k_label_max(const unsigned char* __restrict__ labels, const long long* __restrict__ off,
                            const long long* __restrict__ count, int* __restrict__ out) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  __shared__ int smax[256];
  const int item = blockIdx.y;
  const unsigned char* p = labels + off[item];
  const long long n = count[item];
  const long long head = min(n, (long long)((16u - unsigned(reinterpret_cast<uintptr_t>(p) & 15u)) & 15u));
  const long long nv = (n - head) / 16;  // aligned 16-byte words
  const uint4* pv = reinterpret_cast<const uint4*>(p + head);
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x, nt = (long long)gridDim.x * blockDim.x;
  u16x2 me = {0, 0}, mo = {0, 0};
  auto take = [&](unsigned w) {
    me = __builtin_elementwise_max(me, __builtin_bit_cast(u16x2, w & 0x00FF00FFu));
    mo = __builtin_elementwise_max(mo, __builtin_bit_cast(u16x2, (w >> 8) & 0x00FF00FFu));
  };
  for (long long i = tid; i < nv; i += nt) {
    const uint4 v = pv[i];
    take(v.x);
    take(v.y);
    take(v.z);
    take(v.w);
  }
  int m = max(max(int(me[0]), int(me[1])), max(int(mo[0]), int(mo[1])));
  for (long long i = tid; i < head; i += nt) m = max(m, int(p[i]));
  for (long long i = head + nv * 16 + tid; i < n; i += nt) m = max(m, int(p[i]));
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out + item, smax[0]);
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Number of systems still iterating.
__global__ void k_count_running(const SysState* __restrict__ st, int n, int* __restrict__ count) {
  __shared__ int sc[256];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += (st[i].status == kRunning) ? 1 : 0;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sc[threadIdx.x] += sc[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = sc[0];
}

template <class T>
__global__ void k_convert_field(const double* __restrict__ src, T* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = T(src[i]);
}

void launch_gather_pad(const unsigned char* img, int nx, int ny, int nz, int n, int p, unsigned char* out,
                       hipStream_t st) {
  const int mx = nx / n, my = ny / n, mz = nz / n;
  const int nitems = mx * my * mz;
  const int b = n + 2 * p;
  const int W = chunk_width({(long long)n, (long long)p, (long long)nx}, img, out);
  const int cw = b / W;
  const float inv_cw = 1.0f / float(cw), inv_b = 1.0f / float(b);
  const unsigned rb = unsigned((b * b + kGatherRows - 1) / kGatherRows);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    const int ni = nitems - i0 < 65535 ? nitems - i0 : 65535;
    const dim3 grid(rb, unsigned(ni));
    if (W == 8)
      k_gather_pad<8><<<grid, 256, 0, st>>>(img, nx, ny, nz, n, p, mx, my, i0, cw, inv_cw, inv_b, out);
    else if (W == 4)
      k_gather_pad<4><<<grid, 256, 0, st>>>(img, nx, ny, nz, n, p, mx, my, i0, cw, inv_cw, inv_b, out);
    else
      k_gather_pad<1><<<grid, 256, 0, st>>>(img, nx, ny, nz, n, p, mx, my, i0, cw, inv_cw, inv_b, out);
  }
}

void launch_gather_field(int precision, const void* src, int mx, int my, int mz, int n, int p, void* out,
                         hipStream_t st) {
  const int nitems = (mx / n) * (my / n) * (mz / n);
  const int b = n + 2 * p;
  const unsigned gx = unsigned((b * b * b + 255) / 256);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    const int ni = nitems - i0 < 65535 ? nitems - i0 : 65535;
    const dim3 grid(gx, unsigned(ni));
    if (precision == 0)
      k_gather_field<float><<<grid, 256, 0, st>>>(static_cast<const float*>(src), mx, my, mz, n, p, i0,
                                                  static_cast<float*>(out));
    else
      k_gather_field<double><<<grid, 256, 0, st>>>(static_cast<const double*>(src), mx, my, mz, n, p, i0,
                                                   static_cast<double*>(out));
  }
}

void launch_label_max(const unsigned char* labels, const long long* off, const long long* count, int nitems,
                      long long max_count, int* out, hipStream_t st) {
  k_fill_int<<<(nitems + 255) / 256, 256, 0, st>>>(out, nitems, 0);
  long long bx = (max_count + 256 * 64 - 1) / (256 * 64);  // at least 64 bytes per thread
  bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
  for (int i0 = 0; i0 < nitems; i0 += 65535) {
    const int ni = nitems - i0 < 65535 ? nitems - i0 : 65535;
    k_label_max<<<dim3(unsigned(bx), unsigned(ni)), 256, 0, st>>>(labels, off + i0, count + i0, out + i0);
  }
}

void launch_count_running(const SysState* st, int n, int* count, hipStream_t s) {
  k_count_running<<<1, 256, 0, s>>>(st, n, count);
}

void launch_convert_field(int precision, const double* src, void* dst, long long n, hipStream_t st) {
  const long long blocks = (n + 255) / 256;
  const int nb = int(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  if (precision == 0) k_convert_field<float><<<nb, 256, 0, st>>>(src, reinterpret_cast<float*>(dst), n);
  else k_convert_field<double><<<nb, 256, 0, st>>>(src, reinterpret_cast<double*>(dst), n);
}

}  // namespace hh
