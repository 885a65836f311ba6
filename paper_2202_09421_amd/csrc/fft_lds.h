// Mixed-radix (2, 3, 4, 5) Stockham FFT on complex lines held in LDS.
//
// The FC derivative (Sec. 4.3, eqs. RTEFCSum and RTEFCSumder) needs a DFT of
// the continued line of length N_p, a product of primes <= 5 by construction.
// Each pass reads R points at stride N/R, applies the twiddles of the current
// sub-transform length Ns, does an R-point DFT in registers and writes the
// results to their self-sorted positions (Stockham autosort), ping-ponging
// between two LDS buffers.  Twiddles exp(-2 pi i t k / (Ns R)) come from a
// table precomputed on the host in FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace rte {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, T wr, T wi) {
  return {a.re * wr - a.im * wi, a.re * wi + a.im * wr};
}
// -i * a and +i * a
template <typename T>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> a) { return {a.im, -a.re}; }
template <typename T>
__device__ __forceinline__ cplx<T> mul_pi(cplx<T> a) { return {-a.im, a.re}; }

template <typename T>
__device__ __forceinline__ void dft2(cplx<T>* x) {
  cplx<T> a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft3(cplx<T>* x) {
  const T h = T(0.86602540378443864676);  // sin(pi/3)
  cplx<T> s = cadd(x[1], x[2]);
  cplx<T> d = csub(x[1], x[2]);
  cplx<T> t = {x[0].re - T(0.5) * s.re, x[0].im - T(0.5) * s.im};
  x[0] = cadd(x[0], s);
  cplx<T> r = mul_mi(d);
  r.re *= h;
  r.im *= h;
  x[1] = cadd(t, r);
  x[2] = csub(t, r);
}

template <typename T>
__device__ __forceinline__ void dft4(cplx<T>* x) {
  cplx<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
  cplx<T> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
  x[0] = cadd(a, c);
  x[2] = csub(a, c);
  x[1] = cadd(b, mul_mi(d));
  x[3] = csub(b, mul_mi(d));
}

template <typename T>
__device__ __forceinline__ void dft5(cplx<T>* x) {
  const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
  const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
  cplx<T> a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
  cplx<T> b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
  cplx<T> y0 = cadd(x[0], cadd(a1, a2));
  cplx<T> t1 = {x[0].re + c1 * a1.re + c2 * a2.re, x[0].im + c1 * a1.im + c2 * a2.im};
  cplx<T> t2 = {x[0].re + c2 * a1.re + c1 * a2.re, x[0].im + c2 * a1.im + c1 * a2.im};
  cplx<T> u1 = {s1 * b1.re + s2 * b2.re, s1 * b1.im + s2 * b2.im};
  cplx<T> u2 = {s2 * b1.re - s1 * b2.re, s2 * b1.im - s1 * b2.im};
  x[0] = y0;
  x[1] = cadd(t1, mul_mi(u1));
  x[4] = csub(t1, mul_mi(u1));
  x[2] = cadd(t2, mul_mi(u2));
  x[3] = csub(t2, mul_mi(u2));
}

// One Stockham pass of radix R over `nlines` lines of length N (line stride
// `ls` complex entries) from src to dst.  All threads of the block take part.
template <typename T>
__device__ __forceinline__ void fft_pass(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                         int N, int R, int Ns, const double* __restrict__ tw,
                                         int nlines, int ls, int tid, int nthr) {
  const int nbf = N / R;
  const int total = nlines * nbf;
  for (int idx = tid; idx < total; idx += nthr) {
    const int line = idx / nbf;
    const int j = idx - line * nbf;
    const int k = j % Ns;
    const cplx<T>* s = src + line * ls + j;
    cplx<T> x[5];
#pragma unroll
    for (int t = 0; t < 5; ++t)
      if (t < R) x[t] = s[t * nbf];
    if (Ns > 1) {
      const double* w = tw + 2 * (k * (R - 1));
#pragma unroll
      for (int t = 1; t < 5; ++t)
        if (t < R) x[t] = cmul(x[t], T(w[2 * (t - 1)]), T(w[2 * (t - 1) + 1]));
    }
    switch (R) {
      case 2: dft2(x); break;
      case 3: dft3(x); break;
      case 4: dft4(x); break;
      default: dft5(x); break;
    }
    cplx<T>* d = dst + line * ls + (j / Ns) * Ns * R + k;
#pragma unroll
    for (int t = 0; t < 5; ++t)
      if (t < R) d[t * Ns] = x[t];
  }
}

}  // namespace rte
