// CPU check of the library's FFT building blocks against a brute-force
// O(N^2) DFT in long double:
//   * every register codelet Dft<N, S, T> used by the four-step line kernels
//     (forward and inverse, FP64 and FP32 data);
//   * the four-step composition of the line kernels for every instantiated
//     split N_p = N1 x N2 (length-N1 transforms over the stride-N2 index,
//     twiddles, length-N2 transforms, derivative factor, inverse transforms),
//     i.e. y = IDFT(i mu_k DFT(x)) for a random multiplier mu;
//   * the Stockham passes of the generic kernel (radix 4 first, then 2, 3, 5)
//     for the lengths listed in the generated include file.
// Built with g++ and AddressSanitizer / UndefinedBehaviorSanitizer, so every
// index of the transforms is bounds-checked on the host.  The lists of
// lengths come from generated files (fft_cases.inc) written by the Python
// test from the kernel sources.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fft_codelets.h"
#include "fft_lds.h"

using namespace rte;
typedef std::complex<long double> cld;

static int g_fail = 0;
static double g_worst = 0.0;

static std::vector<cld> dft_ref(const std::vector<cld>& x, int S) {
  const int N = (int)x.size();
  std::vector<cld> y(N);
  for (int k = 0; k < N; ++k) {
    cld acc = 0;
    for (int n = 0; n < N; ++n) {
      const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)(((long)n * k) % N) / N;
      acc += x[n] * cld(std::cos(a), S * std::sin(a));
    }
    y[k] = acc;
  }
  return y;
}

static double rel_err(const std::vector<cld>& a, const std::vector<cld>& b) {
  long double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += std::norm(a[i] - b[i]);
    den += std::norm(b[i]);
  }
  return (double)std::sqrt(num / den);
}

static void report(const char* what, int N1, int N2, int S, double err, double tol) {
  if (err > g_worst && tol < 1e-10) g_worst = err;
  if (!(err <= tol)) {
    std::printf("FAIL %s N=%d,%d S=%d err=%.3e tol=%.1e\n", what, N1, N2, S, err, tol);
    ++g_fail;
  }
}

static std::vector<cld> random_line(int N, unsigned seed) {
  std::mt19937_64 r(seed);
  std::uniform_real_distribution<double> u(-1, 1);
  std::vector<cld> x(N);
  for (auto& v : x) v = cld(u(r), u(r));
  return x;
}

template <int N, int S, typename T>
static void check_codelet(double tol) {
  const std::vector<cld> x = random_line(N, 17 * N + (S > 0));
  cx<T> v[N];
  for (int i = 0; i < N; ++i) v[i] = {T(x[i].real()), T(x[i].imag())};
  std::vector<cld> xr(N);
  for (int i = 0; i < N; ++i) xr[i] = cld(v[i].re, v[i].im);  // the rounded input
  Dft<N, S, T>::run(v);
  std::vector<cld> y(N);
  for (int i = 0; i < N; ++i) y[i] = cld(v[i].re, v[i].im);
  report(sizeof(T) == 8 ? "codelet f64" : "codelet f32", N, 1, S, rel_err(y, dft_ref(xr, S)), tol);
}

template <int N>
static void check_codelet_all() {
  check_codelet<N, -1, double>(4e-16 * (1 + std::log2((double)N)));
  check_codelet<N, 1, double>(4e-16 * (1 + std::log2((double)N)));
  check_codelet<N, -1, float>(2e-7 * (1 + std::log2((double)N)));
  check_codelet<N, 1, float>(2e-7 * (1 + std::log2((double)N)));
}

// Four-step y = IDFT(i mu DFT(x)), in the order of the line kernels.
template <int N1, int N2>
static void check_split() {
  constexpr int N = N1 * N2;
  const std::vector<cld> x = random_line(N, 1000 + N);
  std::mt19937_64 r(7 * N);
  std::uniform_real_distribution<double> u(-1, 1);
  std::vector<double> mu(N);
  for (auto& m : mu) m = u(r);
  std::vector<double> wr(N), wi(N);  // exp(-2 pi i e / N)
  for (int e = 0; e < N; ++e) {
    const long double a = -2.0L * 3.141592653589793238462643383279502884L * e / N;
    wr[e] = (double)std::cos(a);
    wi[e] = (double)std::sin(a);
  }
  std::vector<cx<double>> buf(N);  // element i = n1 N2 + n2 at [n1][n2]
  for (int i = 0; i < N; ++i) buf.at(i) = {(double)x[i].real(), (double)x[i].imag()};
  for (int n2 = 0; n2 < N2; ++n2) {  // step A
    cx<double> v[N1];
    for (int i = 0; i < N1; ++i) v[i] = buf.at(i * N2 + n2);
    Dft<N1, -1, double>::run(v);
    for (int k1 = 1; k1 < N1; ++k1) {
      const int e = (n2 * k1) % N;
      v[k1] = cx_rot(v[k1], wr[e], wi[e]);
    }
    for (int i = 0; i < N1; ++i) buf.at(i * N2 + n2) = v[i];
  }
  for (int k1 = 0; k1 < N1; ++k1) {  // step B
    cx<double> v[N2];
    for (int i = 0; i < N2; ++i) v[i] = buf.at(k1 * N2 + i);
    Dft<N2, -1, double>::run(v);
    for (int k2 = 0; k2 < N2; ++k2) {
      const double m = mu.at(k1 + N1 * k2);
      v[k2] = {-m * v[k2].im, m * v[k2].re};
    }
    Dft<N2, 1, double>::run(v);
    for (int n2 = 1; n2 < N2; ++n2) {
      const int e = (n2 * k1) % N;
      v[n2] = cx_rot(v[n2], wr[e], -wi[e]);
    }
    for (int i = 0; i < N2; ++i) buf.at(k1 * N2 + i) = v[i];
  }
  for (int n2 = 0; n2 < N2; ++n2) {  // step A'
    cx<double> v[N1];
    for (int i = 0; i < N1; ++i) v[i] = buf.at(i * N2 + n2);
    Dft<N1, 1, double>::run(v);
    for (int i = 0; i < N1; ++i) buf.at(i * N2 + n2) = v[i];
  }
  std::vector<cld> X = dft_ref(x, -1);
  for (int k = 0; k < N; ++k) X[k] *= cld(0, mu[k]);
  const std::vector<cld> want = dft_ref(X, 1);
  std::vector<cld> got(N);
  for (int i = 0; i < N; ++i) got[i] = cld(buf[i].re, buf[i].im);
  report("four-step", N1, N2, 0, rel_err(got, want), 2e-15 * (1 + std::log2((double)N)));
}

// Forward DFT by the generic kernel's Stockham passes.
static void check_stockham(int N) {
  std::vector<int> rad;
  int m = N;
  while (m % 4 == 0) { rad.push_back(4); m /= 4; }
  while (m % 2 == 0) { rad.push_back(2); m /= 2; }
  while (m % 3 == 0) { rad.push_back(3); m /= 3; }
  while (m % 5 == 0) { rad.push_back(5); m /= 5; }
  if (m != 1) { std::printf("FAIL stockham N=%d not 5-smooth\n", N); ++g_fail; return; }
  std::vector<double> tw;
  std::vector<int> off;
  int Ns = 1;
  for (int R : rad) {
    off.push_back((int)tw.size() / 2);
    for (int k = 0; k < Ns; ++k)
      for (int t = 1; t < R; ++t) {
        const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)(((long)t * k) % (Ns * R)) / (Ns * R);
        tw.push_back((double)std::cos(a));
        tw.push_back((double)std::sin(a));
      }
    Ns *= R;
  }
  const int nlines = 2, ls = N;
  const std::vector<cld> x0 = random_line(N, 5 * N), x1 = random_line(N, 5 * N + 1);
  std::vector<cplx<double>> A((size_t)nlines * ls), B((size_t)nlines * ls);
  for (int i = 0; i < N; ++i) {
    A[i] = {(double)x0[i].real(), (double)x0[i].imag()};
    A[ls + i] = {(double)x1[i].real(), (double)x1[i].imag()};
  }
  cplx<double>* src = A.data();
  cplx<double>* dst = B.data();
  Ns = 1;
  for (size_t p = 0; p < rad.size(); ++p) {
    fft_pass<double>(src, dst, N, rad[p], Ns, tw.data() + 2 * off[p], nlines, ls, 0, 1);
    std::swap(src, dst);
    Ns *= rad[p];
  }
  for (int l = 0; l < nlines; ++l) {
    std::vector<cld> got(N);
    for (int i = 0; i < N; ++i) got[i] = cld(src[l * ls + i].re, src[l * ls + i].im);
    report("stockham", N, l, -1, rel_err(got, dft_ref(l ? x1 : x0, -1)), 2e-15 * (1 + std::log2((double)N)));
  }
}

int main() {
  int ncase = 0;
#define CODELET(N) check_codelet_all<N>(), ++ncase;
#define SPLIT(N1, N2) check_split<N1, N2>(), ++ncase;
#define STOCKHAM(N) check_stockham(N), ++ncase;
#include "fft_cases.inc"
  std::printf("cases %d failures %d worst %.3e\n", ncase, g_fail, g_worst);
  return g_fail ? 1 : 0;
}
