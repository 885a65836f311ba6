// Compile-time FFT codelets held entirely in registers.
//
// dft<N, S>(x) replaces x[0..N) by sum_n x[n] exp(S 2 pi i n k / N) (S = -1
// forward, +1 inverse, unnormalised) for N a product of 2, 3, 4, 5.  Mixed
// radix decimation in time: N = P Q, Q-point transforms of the P decimated
// subsequences, twiddles exp(S 2 pi i p k2 / N), then P-point transforms
// across p.  Every index is a compile-time constant after unrolling, so the
// whole transform lives in registers.  Twiddle constants come from a
// constexpr Taylor evaluation of sin and cos after reduction to [0, pi/4],
// accurate to about one unit in the last place.
#pragma once

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define RTE_HD __host__ __device__ __forceinline__
#else
#define RTE_HD inline
#endif

namespace rte {
namespace ct {

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double sin_series(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// cos / sin of 2 pi r / n for integers r, n > 0
constexpr double cis_re(long r, long n, bool want_sin) {
  r %= n;
  if (r < 0) r += n;
  const long q = (4 * r) / n;       // quadrant
  const long r4 = 4 * r - q * n;    // in [0, n)
  double c0 = 0, s0 = 0;
  if (2 * r4 <= n) {
    const double x = (kPi / 2) * (double)r4 / (double)n;
    c0 = cos_series(x);
    s0 = sin_series(x);
  } else {
    const double x = (kPi / 2) * (double)(n - r4) / (double)n;
    c0 = sin_series(x);
    s0 = cos_series(x);
  }
  double c = c0, s = s0;
  if (q == 1) { c = -s0; s = c0; }
  else if (q == 2) { c = -c0; s = -s0; }
  else if (q == 3) { c = s0; s = -c0; }
  return want_sin ? s : c;
}

template <int N>
struct Roots {
  double c[N > 0 ? N : 1];
  double s[N > 0 ? N : 1];
  constexpr Roots() : c(), s() {
    for (int k = 0; k < N; ++k) {
      c[k] = cis_re(k, N, false);
      s[k] = cis_re(k, N, true);
    }
  }
};

template <int N>
constexpr Roots<N> roots{};

constexpr int first_radix(int N) {
  return (N % 4 == 0 && N != 4) ? 4 : (N % 2 == 0 && N != 2) ? 2 : (N % 3 == 0 && N != 3) ? 3 : (N % 5 == 0 && N != 5) ? 5 : N;
}

}  // namespace ct

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
RTE_HD cx<T> cx_add(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
RTE_HD cx<T> cx_sub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
// multiply by S*i (S = +-1)
template <int S, typename T>
RTE_HD cx<T> cx_si(cx<T> a) { return S > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re}; }
template <typename T>
RTE_HD cx<T> cx_rot(cx<T> a, double c, double s) {
  return {a.re * T(c) - a.im * T(s), a.re * T(s) + a.im * T(c)};
}

template <int N, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<1, S, T> {
  static RTE_HD void run(cx<T>*) {}
};

template <int S, typename T>
struct Dft<2, S, T> {
  static RTE_HD void run(cx<T>* x) {
    const cx<T> a = x[0], b = x[1];
    x[0] = cx_add(a, b);
    x[1] = cx_sub(a, b);
  }
};

template <int S, typename T>
struct Dft<3, S, T> {
  static RTE_HD void run(cx<T>* x) {
    const T h = T(0.86602540378443864676);
    const cx<T> s = cx_add(x[1], x[2]);
    const cx<T> d = cx_sub(x[1], x[2]);
    const cx<T> t = {x[0].re - T(0.5) * s.re, x[0].im - T(0.5) * s.im};
    cx<T> r = cx_si<S>(d);
    r.re *= h;
    r.im *= h;
    x[0] = cx_add(x[0], s);
    x[1] = cx_add(t, r);
    x[2] = cx_sub(t, r);
  }
};

template <int S, typename T>
struct Dft<4, S, T> {
  static RTE_HD void run(cx<T>* x) {
    const cx<T> a = cx_add(x[0], x[2]), b = cx_sub(x[0], x[2]);
    const cx<T> c = cx_add(x[1], x[3]), d = cx_si<S>(cx_sub(x[1], x[3]));
    x[0] = cx_add(a, c);
    x[2] = cx_sub(a, c);
    x[1] = cx_add(b, d);
    x[3] = cx_sub(b, d);
  }
};

template <int S, typename T>
struct Dft<5, S, T> {
  static RTE_HD void run(cx<T>* x) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    const cx<T> a1 = cx_add(x[1], x[4]), a2 = cx_add(x[2], x[3]);
    const cx<T> b1 = cx_sub(x[1], x[4]), b2 = cx_sub(x[2], x[3]);
    const cx<T> t1 = {x[0].re + c1 * a1.re + c2 * a2.re, x[0].im + c1 * a1.im + c2 * a2.im};
    const cx<T> t2 = {x[0].re + c2 * a1.re + c1 * a2.re, x[0].im + c2 * a1.im + c1 * a2.im};
    const cx<T> u1 = cx_si<S>(cx<T>{s1 * b1.re + s2 * b2.re, s1 * b1.im + s2 * b2.im});
    const cx<T> u2 = cx_si<S>(cx<T>{s2 * b1.re - s1 * b2.re, s2 * b1.im - s1 * b2.im});
    x[0] = cx_add(x[0], cx_add(a1, a2));
    x[1] = cx_add(t1, u1);
    x[4] = cx_sub(t1, u1);
    x[2] = cx_add(t2, u2);
    x[3] = cx_sub(t2, u2);
  }
};

template <int N, int S, typename T>
struct Dft {
  static constexpr int P = ct::first_radix(N);
  static constexpr int Q = N / P;
  static RTE_HD void run(cx<T>* x) {
    cx<T> y[N];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      cx<T> t[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) t[q] = x[p + P * q];
      Dft<Q, S, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) {
        const int e = (p * k2) % N;
        y[p * Q + k2] = (e == 0) ? t[k2] : cx_rot(t[k2], ct::roots<N>.c[e], S * ct::roots<N>.s[e]);
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) {
      cx<T> t[P];
#pragma unroll
      for (int p = 0; p < P; ++p) t[p] = y[p * Q + k2];
      Dft<P, S, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) x[k2 + Q * k1] = t[k1];
    }
  }
};

}  // namespace rte
