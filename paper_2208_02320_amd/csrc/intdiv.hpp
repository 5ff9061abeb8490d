// Integer quotient by a runtime divisor through a float reciprocal, for the
// index splitting of the data-movement kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>

namespace hh {

// floor(a / d) for 0 <= a < 2^23 and d >= 1, given inv = 1.0f / d: the
// float quotient is within one of the true one, and one integer step fixes it.
__device__ __forceinline__ int fdiv(int a, int d, float inv) {
  int q = int(float(a) * inv);
  const int r = a - q * d;
  q += (r >= d ? 1 : 0) - (r < 0 ? 1 : 0);
  return q;
}

// Widest chunk (8, 4 or 1 bytes) that divides every value in `vals` and
// the two addresses: byte rows cut into such chunks move as aligned words.
inline int chunk_width(std::initializer_list<long long> vals, const void* a, const void* b) {
  for (int w : {8, 4}) {
    bool ok = reinterpret_cast<unsigned long long>(a) % w == 0 && reinterpret_cast<unsigned long long>(b) % w == 0;
    for (long long v : vals) ok = ok && v % w == 0;
    if (ok) return w;
  }
  return 1;
}

// W-byte word type
template <int W>
struct Chunk;
template <>
struct Chunk<8> {
  using type = uint2;
};
template <>
struct Chunk<4> {
  using type = unsigned;
};
template <>
struct Chunk<1> {
  using type = unsigned char;
};

// byte j of a chunk
__device__ __forceinline__ unsigned chunk_byte(uint2 v, int j) { return ((j < 4 ? v.x : v.y) >> (8 * (j & 3))) & 0xFFu; }
__device__ __forceinline__ unsigned chunk_byte(unsigned v, int j) { return (v >> (8 * j)) & 0xFFu; }
__device__ __forceinline__ unsigned chunk_byte(unsigned char v, int) { return v; }

}  // namespace hh
