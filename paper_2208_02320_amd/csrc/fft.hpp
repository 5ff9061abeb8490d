// Device FFT building blocks for gfx950: complex arithmetic, compile-time
// twiddles, fully unrolled register DFTs of small mixed-radix length
// (radices 2, 3, 4, 5) and a two-step (four-step) DFT of a batch of lines
// held in LDS.
//
// These carry out the FFT convolution of Appendix A of the paper (forward
// transform, multiplication in frequency space, inverse transform); the
// paper leaves the FFT itself to a library, so the factorisation and data
// movement here are this implementation's own.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace hh {

template <class T>
struct cx {
  T re, im;
};

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
// (S i) * a for S = +1 / -1
template <int S, class T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  if constexpr (S > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Compile-time trigonometry: cos / sin of 2*pi*num/den, by exact octant
// reduction of the rational angle and Taylor series on [0, pi/4].
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double sin_series(double x) {
  double x2 = x * x, t = x, s = x;
  for (int n = 1; n <= 12; ++n) {
    t *= -x2 / double((2 * n) * (2 * n + 1));
    s += t;
  }
  return s;
}
constexpr double cos_series(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int n = 1; n <= 12; ++n) {
    t *= -x2 / double((2 * n - 1) * (2 * n));
    s += t;
  }
  return s;
}
constexpr double cos2pi(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  if (2 * num > den) num = den - num;  // cos(2pi(1-t)) = cos(2pi t)
  double sgn = 1.0;
  if (4 * num > den) {  // cos(2pi t) = -cos(2pi(1/2 - t))
    num = den - 2 * num;
    den *= 2;
    sgn = -1.0;
  }
  const double th = 2.0 * kPi * double(num) / double(den);  // in [0, pi/2]
  return sgn * (th <= kPi / 4 ? cos_series(th) : sin_series(kPi / 2 - th));
}
constexpr double sin2pi(long num, long den) { return cos2pi(4 * num - den, 4 * den); }

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int smallest_factor(int r) {
  for (int p = 2; p * p <= r; ++p)
    if (r % p == 0) return p;
  return r;
}
constexpr bool is_prime(int r) { return r > 1 && smallest_factor(r) == r; }
constexpr int first_radix(int r) { return (r % 4 == 0 && r != 8) ? 4 : smallest_factor(r); }

// Lengths whose register DFT is built here: every prime factor at most kMaxPrime.
constexpr int kMaxPrime = 53;
constexpr bool dft_length_ok(int n) {
  if (n < 1) return false;
  while (n > 1) {
    const int p = smallest_factor(n);
    if (p > kMaxPrime) return false;
    n /= p;
  }
  return true;
}

// ---------------------------------------------------------------------------
// In-register DFT of length R, natural order in and out:
//   X[k] = sum_j v[j] exp(S 2 pi i j k / R),  S = -1 forward, +1 inverse.
// ---------------------------------------------------------------------------
template <int R, int S, class T>
__device__ __forceinline__ void dft(cx<T>* v) {
  static_assert(dft_length_ok(R), "register DFT length has a prime factor above kMaxPrime");
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    constexpr T s3 = T(0.866025403784438646763723170752936183);
    const cx<T> t1 = v[1] + v[2];
    const cx<T> t2 = v[0] - T(0.5) * t1;
    const cx<T> t3 = mul_si<S>(s3 * (v[1] - v[2]));
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  } else if constexpr (R == 4) {
    const cx<T> a = v[0] + v[2], b = v[0] - v[2];
    const cx<T> c = v[1] + v[3], d = mul_si<S>(v[1] - v[3]);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  } else if constexpr (R == 5) {
    constexpr T c1 = T(cos2pi(1, 5)), c2 = T(cos2pi(2, 5));
    constexpr T s1 = T(sin2pi(1, 5)), s2 = T(sin2pi(2, 5));
    const cx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
    const cx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
    const cx<T> r1 = v[0] + c1 * a1 + c2 * a2;
    const cx<T> r2 = v[0] + c2 * a1 + c1 * a2;
    const cx<T> i1 = mul_si<S>(s1 * b1 + s2 * b2);
    const cx<T> i2 = mul_si<S>(s2 * b1 - s1 * b2);
    v[0] = v[0] + a1 + a2;
    v[1] = r1 + i1;
    v[4] = r1 - i1;
    v[2] = r2 + i2;
    v[3] = r2 - i2;
  } else if constexpr (is_prime(R)) {
    // odd prime R: pair j with R - j; with a_j = v_j + v_{R-j} and
    // b_j = v_j - v_{R-j} (j = 1 .. H),
    //   X_k     = v_0 + sum_j cos(2 pi jk/R) a_j + S i sum_j sin(2 pi jk/R) b_j
    //   X_{R-k} = the same with the sine sum subtracted
    constexpr int H = (R - 1) / 2;
    cx<T> a[H], b[H];
    cx<T> x0 = v[0];
    static_for<1, H + 1>([&](auto J) {
      constexpr int j = decltype(J)::value;
      a[j - 1] = v[j] + v[R - j];
      b[j - 1] = v[j] - v[R - j];
      x0 = x0 + a[j - 1];
    });
    static_for<1, H + 1>([&](auto K) {
      constexpr int k = decltype(K)::value;
      cx<T> re = v[0], im = {T(0), T(0)};
      static_for<1, H + 1>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr T c = T(cos2pi(j * k, R)), sn = T(sin2pi(j * k, R));
        re = re + c * a[j - 1];
        im = im + sn * b[j - 1];
      });
      const cx<T> t = mul_si<S>(im);
      v[k] = re + t;
      v[R - k] = re - t;
    });
    v[0] = x0;
  } else {
    // R = A * B:  j = j1 + A j2,  k = k2 + B k1
    constexpr int A = first_radix(R), B = R / A;
    cx<T> w[R];
    static_for<0, A>([&](auto J1) {
      constexpr int j1 = decltype(J1)::value;
      cx<T> t[B];
      static_for<0, B>([&](auto J2) {
        constexpr int j2 = decltype(J2)::value;
        t[j2] = v[j1 + A * j2];
      });
      dft<B, S, T>(t);
      static_for<0, B>([&](auto K2) {
        constexpr int k2 = decltype(K2)::value;
        if constexpr ((j1 * k2) % R == 0) {
          w[j1 * B + k2] = t[k2];
        } else {
          constexpr T c = T(cos2pi(j1 * k2, R));
          constexpr T s = T(S * sin2pi(j1 * k2, R));
          w[j1 * B + k2] = cmul(t[k2], cx<T>{c, s});
        }
      });
    });
    static_for<0, B>([&](auto K2) {
      constexpr int k2 = decltype(K2)::value;
      cx<T> t[A];
      static_for<0, A>([&](auto J1) {
        constexpr int j1 = decltype(J1)::value;
        t[j1] = w[j1 * B + k2];
      });
      dft<A, S, T>(t);
      static_for<0, A>([&](auto K1) {
        constexpr int k1 = decltype(K1)::value;
        v[k2 + B * k1] = t[k1];
      });
    });
  }
}

// ---------------------------------------------------------------------------
// Block-level two-step DFT of length N = N1 * N2 over L lines in LDS.
//
// Layout: element e of line l lives at buf[e * L + l] (lines fastest, so a
// wave touching consecutive lines touches consecutive LDS words).
// tw[m] = (cos 2 pi m / N, sin 2 pi m / N) for m in [0, N).
//
// fft_nat2perm: natural input; output element m = k2 + N2 k1 is left at
//               position k1 + N1 k2.
// fft_perm2nat: input in that permuted order; output in natural order.
// Used with opposite signs back to back, the pair needs no reordering pass.
// Both end with a barrier.
// ---------------------------------------------------------------------------
template <int N1, int N2>
__device__ __forceinline__ int perm_pos(int m) {
  return (m / N2) + N1 * (m % N2);
}
template <int N1, int N2>
__device__ __forceinline__ int perm_idx(int pos) {
  return (pos / N1) + N2 * (pos % N1);
}

template <int N, int S, class T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* tw, int m) {
  const cx<T> w = tw[m];
  return {w.re, T(S) * w.im};
}

// Element e of line l sits at buf[e * L + (e / N1) * P + l]: P extra
// complex words after every block of N1 elements shift the blocks across
// LDS banks (P = 0 is the plain layout).
template <int N1, int P>
__device__ __forceinline__ int lds_at(int e, int L) {
  return e * L + (P ? (e / N1) * P : 0);
}

template <int N1, int N2, int S, class T, int P = 0>
__device__ __forceinline__ void fft_nat2perm(cx<T>* buf, int L, const cx<T>* tw) {
  constexpr int N = N1 * N2;
  if constexpr (N2 > 1) {
    for (int task = threadIdx.x; task < L * N1; task += blockDim.x) {
      const int l = task % L, j1 = task / L;
      cx<T> v[N2];
#pragma unroll
      for (int j2 = 0; j2 < N2; ++j2) v[j2] = buf[(j1 + N1 * j2) * L + j2 * P + l];
      dft<N2, S, T>(v);
#pragma unroll
      for (int k2 = 1; k2 < N2; ++k2) v[k2] = cmul(v[k2], twiddle<N, S>(tw, (j1 * k2) % N));
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) buf[(j1 + N1 * k2) * L + k2 * P + l] = v[k2];
    }
    __syncthreads();
  }
  for (int task = threadIdx.x; task < L * N2; task += blockDim.x) {
    const int l = task % L, k2 = task / L;
    cx<T> v[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) v[j1] = buf[(j1 + N1 * k2) * L + k2 * P + l];
    dft<N1, S, T>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) buf[(k1 + N1 * k2) * L + k2 * P + l] = v[k1];
  }
  __syncthreads();
}

template <int N1, int N2, int S, class T, int P = 0>
__device__ __forceinline__ void fft_perm2nat(cx<T>* buf, int L, const cx<T>* tw) {
  constexpr int N = N1 * N2;
  // factors (A, B) = (N2, N1): step one runs DFT_N1 over contiguous runs
  for (int task = threadIdx.x; task < L * N2; task += blockDim.x) {
    const int l = task % L, j1 = task / L;  // j1 in [0, N2)
    cx<T> v[N1];
#pragma unroll
    for (int j2 = 0; j2 < N1; ++j2) v[j2] = buf[(N1 * j1 + j2) * L + j1 * P + l];
    dft<N1, S, T>(v);
    if constexpr (N2 > 1) {
#pragma unroll
      for (int k2 = 1; k2 < N1; ++k2) v[k2] = cmul(v[k2], twiddle<N, S>(tw, (j1 * k2) % N));
    }
#pragma unroll
    for (int k2 = 0; k2 < N1; ++k2) buf[(N1 * j1 + k2) * L + j1 * P + l] = v[k2];
  }
  __syncthreads();
  if constexpr (N2 > 1) {
    for (int task = threadIdx.x; task < L * N1; task += blockDim.x) {
      const int l = task % L, k2 = task / L;  // k2 in [0, N1)
      cx<T> v[N2];
#pragma unroll
      for (int j1 = 0; j1 < N2; ++j1) v[j1] = buf[(N1 * j1 + k2) * L + j1 * P + l];
      dft<N2, S, T>(v);
#pragma unroll
      for (int k1 = 0; k1 < N2; ++k1) buf[(N1 * k1 + k2) * L + k1 * P + l] = v[k1];
    }
    __syncthreads();
  }
}

// Twiddle table exp(2 pi i m / N), m in [0, N), evaluated at compile time
// (the series above in double, then rounded to T) and placed in read-only
// device memory, one per (N, T).
template <class T, int N>
struct TwTable {
  cx<T> v[N];
};
template <class T, int N, int... I>
constexpr TwTable<T, N> make_twiddles(std::integer_sequence<int, I...>) {
  return TwTable<T, N>{{cx<T>{T(cos2pi(I, N)), T(sin2pi(I, N))}...}};
}
template <int N, class T>
__device__ const TwTable<T, N> kTwiddles = make_twiddles<T, N>(std::make_integer_sequence<int, N>{});

// Copy the table into tw[0..N) (LDS); the caller's next barrier publishes it.
template <int N, class T>
__device__ __forceinline__ void fill_twiddles(cx<T>* tw) {
  for (int m = threadIdx.x; m < N; m += blockDim.x) tw[m] = kTwiddles<N, T>.v[m];
}

// Split of N for the two-step DFT: N <= 16 in one register step, otherwise
// the divisor pair closest to sqrt(N), larger factor first.
constexpr int split_n1(int n) {
  if (n <= 16) return n;
  int best = n;
  for (int d = 1; d <= n; ++d) {
    if (n % d == 0 && d * d >= n && d < best) best = d;
  }
  return best;
}

}  // namespace hh
