// In-register DFT building blocks for the gfx950 Poisson kernels.
//
// The exchange operator needs one periodic Poisson solve per orbital pair
// (arXiv 2110.07670, Eq. (3), evaluated in reciprocal space as the text after
// Eq. (4) states).  Every 1-D transform of length N used here is split as
// N = N1 * N2 (four-step form): a length-N1 DFT over the N1 elements
// t2 + N2*j1 of each of N2 residues t2, a twiddle w_N^(t2*k1), and a length-N2
// DFT over t2.  The small DFTs below run entirely in registers with twiddles
// fixed at compile time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace acex {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// a * b
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// a * (-i) for the forward sign, a * (+i) for the inverse sign
template <bool INV, typename T>
__device__ __forceinline__ cx<T> rot_i(cx<T> a) {
  if constexpr (INV) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ------------------------------------------------------------------ constants
// cos and sin of 2*pi*k/n at compile time: exact integer quadrant reduction,
// then Horner-form Taylor series on [0, pi/4] (|x|^27/27! < 1e-26 there).

constexpr double kPi = 3.14159265358979323846;

constexpr double hsin(double x) {
  double x2 = x * x, r = 1.0;
  for (int k = 13; k >= 1; --k) r = 1.0 - x2 / double((2 * k) * (2 * k + 1)) * r;
  return x * r;
}
constexpr double hcos(double x) {
  double x2 = x * x, r = 1.0;
  for (int k = 13; k >= 1; --k) r = 1.0 - x2 / double((2 * k - 1) * (2 * k)) * r;
  return r;
}
// returns {cos, sin} of 2 pi k / n
struct cs_pair {
  double c, s;
};
constexpr cs_pair turn_cs(long k, long n) {
  long kk = ((k % n) + n) % n;
  long q = (4 * kk) / n;
  long r = 4 * kk - q * n;  // angle within the quadrant = r * (pi/2) / n
  double c = 0, s = 0;
  if (2 * r <= n) {
    double th = double(r) * (kPi / 2.0) / double(n);
    c = hcos(th);
    s = hsin(th);
  } else {
    double ph = double(n - r) * (kPi / 2.0) / double(n);
    c = hsin(ph);
    s = hcos(ph);
  }
  switch (q) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}

template <long K, long N>
struct TW {
  static constexpr cs_pair v = turn_cs(K, N);
};

// x * w_N^E with w_N = exp(-2 pi i / N) (forward) or exp(+2 pi i / N) (inverse)
template <long E, long N, bool INV, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> x) {
  constexpr long e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return x;
  } else if constexpr (4 * e == N) {
    return rot_i<INV>(x);
  } else if constexpr (2 * e == N) {
    return {-x.re, -x.im};
  } else if constexpr (4 * e == 3 * N) {
    return rot_i<!INV>(x);
  } else {
    constexpr T c = T(TW<e, N>::v.c);
    constexpr T s = INV ? T(TW<e, N>::v.s) : T(-TW<e, N>::v.s);
    return {x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// ------------------------------------------------------------------ static loop
template <int I, int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    sfor<I + 1, N>(f);
  }
}

// first factor of a composite in-register DFT size
template <int R>
struct split_of {
  static constexpr int value = (R % 4 == 0) ? 4 : (R % 3 == 0) ? 3 : (R % 5 == 0) ? 5 : 2;
};

// ------------------------------------------------------------------ DFT_R in registers
// Natural order in and out: a[k] <- sum_n a[n] w_R^(n k); no scaling.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T>* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  } else if constexpr (R == 3) {
    // w = exp(-+2 pi i/3) = -1/2 -+ i sqrt(3)/2
    constexpr T h = T(0.86602540378443864676);
    cx<T> s = a[1] + a[2];
    cx<T> d = a[1] - a[2];
    cx<T> m = {a[0].re - T(0.5) * s.re, a[0].im - T(0.5) * s.im};
    cx<T> r = rot_i<INV>(d);  // -i d (fwd)
    r = {r.re * h, r.im * h};
    a[0] = a[0] + s;
    a[1] = m + r;
    a[2] = m - r;
  } else if constexpr (R == 4) {
    cx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
    cx<T> s13 = a[1] + a[3], d13 = rot_i<INV>(a[1] - a[3]);
    a[0] = s02 + s13;
    a[2] = s02 - s13;
    a[1] = d02 + d13;
    a[3] = d02 - d13;
  } else if constexpr (R == 5) {
    constexpr T c1 = T(TW<1, 5>::v.c), c2 = T(TW<2, 5>::v.c);
    constexpr T s1 = T(TW<1, 5>::v.s), s2 = T(TW<2, 5>::v.s);
    cx<T> b1 = a[1] + a[4], b2 = a[2] + a[3];
    cx<T> d1 = a[1] - a[4], d2 = a[2] - a[3];
    cx<T> t1 = {a[0].re + c1 * b1.re + c2 * b2.re, a[0].im + c1 * b1.im + c2 * b2.im};
    cx<T> t2 = {a[0].re + c2 * b1.re + c1 * b2.re, a[0].im + c2 * b1.im + c1 * b2.im};
    cx<T> u1 = {s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im};
    cx<T> u2 = {s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im};
    u1 = rot_i<INV>(u1);  // -i u1 (fwd)
    u2 = rot_i<INV>(u2);
    a[0] = a[0] + b1 + b2;
    a[1] = t1 + u1;
    a[4] = t1 - u1;
    a[2] = t2 + u2;
    a[3] = t2 - u2;
  } else {
    constexpr int R1 = split_of<R>::value;
    constexpr int R2 = R / R1;
    static_assert(R1 * R2 == R, "bad split");
    cx<T> y[R];
    sfor<0, R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      cx<T> t[R1];
      sfor<0, R1>([&](auto n1c) { t[decltype(n1c)::value] = a[n2 + R2 * decltype(n1c)::value]; });
      dft<R1, INV>(t);
      sfor<0, R1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        y[n2 * R1 + k1] = twc<long(n2) * k1, R, INV>(t[k1]);
      });
    });
    sfor<0, R1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      cx<T> t[R2];
      sfor<0, R2>([&](auto n2c) { t[decltype(n2c)::value] = y[decltype(n2c)::value * R1 + k1]; });
      dft<R2, INV>(t);
      sfor<0, R2>([&](auto k2c) { a[k1 + R1 * decltype(k2c)::value] = t[decltype(k2c)::value]; });
    });
  }
}

// ------------------------------------------------------------------ length splits
// N = N1 * N2 for the grid lengths the library instantiates.  N1 is the
// first-step DFT size (over stride-N2 elements), N2 the second.
template <int N>
struct fft_split;
template <> struct fft_split<16> { static constexpr int N1 = 4, N2 = 4; };
template <> struct fft_split<24> { static constexpr int N1 = 6, N2 = 4; };
template <> struct fft_split<32> { static constexpr int N1 = 8, N2 = 4; };
template <> struct fft_split<40> { static constexpr int N1 = 10, N2 = 4; };
template <> struct fft_split<48> { static constexpr int N1 = 8, N2 = 6; };
template <> struct fft_split<64> { static constexpr int N1 = 8, N2 = 8; };
template <> struct fft_split<80> { static constexpr int N1 = 10, N2 = 8; };
template <> struct fft_split<96> { static constexpr int N1 = 12, N2 = 8; };
template <> struct fft_split<120> { static constexpr int N1 = 12, N2 = 10; };
template <> struct fft_split<128> { static constexpr int N1 = 16, N2 = 8; };
template <> struct fft_split<144> { static constexpr int N1 = 12, N2 = 12; };
template <> struct fft_split<160> { static constexpr int N1 = 16, N2 = 10; };
template <> struct fft_split<192> { static constexpr int N1 = 16, N2 = 12; };

// Frequency index held at position p after the forward four-step transform:
// position a + N2*b holds X[b + N1*a].
template <int N>
__device__ __forceinline__ int freq_of_pos(int p) {
  constexpr int N1 = fft_split<N>::N1, N2 = fft_split<N>::N2;
  return p / N2 + N1 * (p % N2);
}

}  // namespace acex
