// Four-step line kernel templates (included by the translation units that
// instantiate them for the supported extended lengths).
#pragma once
// Four-step line passes for the common extended lengths N_p = N1 * N2.
//
// FC-Gram continuation + filtered spectral derivative along x lines (rows)
// and y lines (columns) of one state, or the exact transpose (Sec. 4.3).
// The DFT of length N_p is split as in the four-step algorithm:
//   A : N2 transforms of length N1 over the stride-N2 index, twiddle w^{n2 k1}
//   B : N1 transforms of length N2 over each contiguous block, multiply by
//       the derivative factor i mu_k at k = k1 + N1 k2, inverse length-N2
//       transform, twiddle w^{-n2 k1}
//   A': N2 inverse transforms of length N1
// Each transform is a compile-time codelet held in registers, so a line makes
// three LDS round trips.
//
// Work unit: two neighbouring lines of one ordinate group, four complex
// lines: complex line r holds slot r of the first line in its real part and
// slot r of the second in its imaginary part (the operator is real-linear, so
// both are differentiated by one complex transform).  Pairing one ordinate of
// two neighbouring lines keeps the rounding of each relative to values of
// similar size; pairing two ordinates of one line (a bright and a dim one,
// near a beam) makes the dim one's derivative inherit the bright one's
// rounding, which grew the gradient maps' error 4x at 513 x 513 x 64.
// Loads and stores keep one lane per (point, line): the two lanes of a pair
// hold the same point of the two lines and swap two values each (DPP, no
// LDS) to form or split full complex entries.  A workgroup is one wave and handles
// two consecutive units; every global load of both units, and of the FC
// tables, is issued before the first one is transformed, so the memory
// latency is paid once per wave.  x units come first, then y units; unit
// pairs are even-aligned so a wave's two y units cover four adjacent
// columns, i.e. whole 128-byte segments of the row-aligned state.

#include "fft_codelets.h"
#include "rte_internal.h"

namespace rte {

template <typename T>
struct Lines4Args {
  const T* in;
  T* out[2];
  const double* coef[2];   // xi, eta in slot order
  FcPlanDev fc;            // identical for every direction of the launch
  int nlines[2];
  int npe[2];              // line pairs per (source, group), rounded up to even
  int64_t line_stride[2], pt_stride[2];
  int64_t grp_stride, inst_stride;
  int G;
  int dir_first;           // direction of units [0, units_first)
  int units_first;
  int nunits;
  int nt_out;              // plan streams its state arrays (non-temporal stores where they pay)
};

// Store of one (point, line) lane's 4 slots (lengths up to kLongLine).  NT:
// with the non-temporal hint (the outputs are not read again by the pass),
// for plans that stream their state arrays.  Measured at N_p = 540: 11 %
// faster FP32 passes, 1 % faster FP64 transposes, but a 5 % slower FP64
// forward pass, which keeps ordinary stores.
typedef double d2v_st __attribute__((ext_vector_type(2)));
typedef float f4v_st __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ void store_slots(double* q, const double* v) {
  if constexpr (NT) {
    const d2v_st a = {v[0], v[1]}, b = {v[2], v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<d2v_st*>(q));
    __builtin_nontemporal_store(b, reinterpret_cast<d2v_st*>(q) + 1);
  } else {
    reinterpret_cast<double2*>(q)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(q)[1] = make_double2(v[2], v[3]);
  }
}
template <bool NT>
__device__ __forceinline__ void store_slots(float* q, const double* v) {
  if constexpr (NT) {
    const f4v_st a = {float(v[0]), float(v[1]), float(v[2]), float(v[3])};
    __builtin_nontemporal_store(a, reinterpret_cast<f4v_st*>(q));
  } else {
    *reinterpret_cast<float4*>(q) = make_float4(float(v[0]), float(v[1]), float(v[2]), float(v[3]));
  }
}

constexpr int kLP = 4;  // complex lines per unit (slot r of both lines, r = 0..3)

// One unit per workgroup: workgroup b runs on XCD b % 8, so units 2x and
// 2x + 1 of each chunk of 16 (the two column pairs of one 128-byte row
// segment) go to workgroups b and b + 8 of that chunk, i.e. to one XCD and
// its L2.
__device__ __forceinline__ int remap_unit16(int b) {
  const int chunk = b >> 4, x = b & 7, h = (b >> 3) & 1;
  return chunk * 16 + 2 * x + h;
}
constexpr size_t kLines4MaxLds = 64 * 1024;
// Extended lengths above kLongLine (up to 40 x 40): the line buffer alone
// takes up to 80 KB, so the continuation matrix is read from global memory
// (L1 / L2) instead of LDS, and the LDS cap is raised (gfx950: 160 KB per CU).
constexpr size_t kLines4MaxLdsLong = 96 * 1024;

// thread-owned loads of one unit: point i of line it (0/1) for
// e = tid + NTH t, i = e / 2, it = e % 2; 4 slots each
template <typename T, int TMAX>
struct UnitRegs {
  T v[TMAX][4];
};

struct UnitDesc {
  int dir;
  bool live, has1;
  int64_t base;
  int s0;
};

template <typename T>
__device__ __forceinline__ UnitDesc decode_unit(const Lines4Args<T>& a, int u) {
  UnitDesc d;
  int r = u;
  d.dir = a.dir_first;
  if (u >= a.units_first) {
    d.dir = 1 - a.dir_first;
    r = u - a.units_first;
  }
  const int npe = a.npe[d.dir];
  const int pair = r % npe;
  const int g = (r / npe) % a.G;
  const int q = r / (npe * a.G);
  const int line0 = 2 * pair;
  d.live = (u < a.nunits) && (line0 < a.nlines[d.dir]);
  d.has1 = line0 + 1 < a.nlines[d.dir];
  d.base = (int64_t)q * a.inst_stride + (int64_t)g * a.grp_stride + (int64_t)line0 * a.line_stride[d.dir];
  d.s0 = g * kGroup;
  return d;
}

template <typename T, int TMAX, int NTH>
__device__ __forceinline__ void load_unit(const Lines4Args<T>& a, const UnitDesc& d, int n, int tid,
                                          UnitRegs<T, TMAX>& R) {
  const T* in = a.in + d.base;
  const int64_t ls = a.line_stride[d.dir], ps = a.pt_stride[d.dir];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int e = tid + NTH * t, it = e & 1, i = e >> 1;
    if (d.live && i < n && (it == 0 || d.has1)) {
      const T* p = in + it * ls + (int64_t)i * ps;
      if constexpr (sizeof(T) == 8) {
        const double2 x = reinterpret_cast<const double2*>(p)[0];
        const double2 y = reinterpret_cast<const double2*>(p)[1];
        R.v[t][0] = x.x; R.v[t][1] = x.y; R.v[t][2] = y.x; R.v[t][3] = y.y;
      } else {
        const float4 x = *reinterpret_cast<const float4*>(p);
        R.v[t][0] = x.x; R.v[t][1] = x.y; R.v[t][2] = x.z; R.v[t][3] = x.w;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) R.v[t][r] = T(0);
    }
  }
}

// LDS layout (doubles): buf [kLP][LSZ] complex (rows of PS entries, PS the
// smallest odd count >= N2: step B's lanes read rows PS apart, and an odd
// stride of 16-byte entries spreads 16 consecutive lanes over distinct
// banks; line stride LSZ = 2 mod 4 entries so that the two complex lines
// stored by neighbouring lanes fall in different bank halves) | roots,
// complex, entry e at e + e / 16
// (spreads the strided twiddle reads over the banks) | mu [N] | continuation
// matrix [(C+E) x 2d].  The transpose keeps its 2d fold values per line in
// the line's own extension region (positions n .. n + 2d - 1, free once the
// fold sums are formed; C + E >= 2d is checked by the plan).
template <int N1, int N2>
struct L4Smem {
  static constexpr int N = N1 * N2;
  static constexpr int PS = N2 | 1;
  static constexpr int LSZ0 = N1 * PS;
  static constexpr int LSZ = LSZ0 + (6 - LSZ0 % 4) % 4;
  static constexpr int NR = N + N / 16 + 1;
  static constexpr int BUF = 2 * kLP * LSZ;
  static constexpr int ROOTS = 2 * NR;
  static constexpr int MU = N;
  // nmx = (C + E) * 2d continuation entries staged (0 when read from global
  // memory).  TG: the twiddles are read from global memory (L1 / L2) instead
  // of being staged; mus: the multipliers are staged.
  static constexpr int mu_off(bool tg) { return BUF + (tg ? 0 : ROOTS); }
  static constexpr int mx_off(bool tg, bool mus) { return mu_off(tg) + (mus ? MU : 0); }
  static constexpr size_t bytes(int nmx, bool tg, bool mus) {
    return sizeof(double) * (size_t)(mx_off(tg, mus) + nmx);
  }
};

// Derivative multipliers staged in LDS: with staged tables, and with global
// twiddles in the FP32 forward pass up to kLongLine (its N2 multiplier reads
// per step-B transform then stay off the vector memory pipe: 4 % faster at
// N_p = 540).  With global twiddles the FP64 forward pass (1.5 % faster with
// the smaller LDS footprint), the transpose (5 % slower with them staged)
// and the long lines read them from global memory.
template <typename T, bool TG, int N, bool ADJ>
constexpr bool kMuStaged = !TG || (sizeof(T) == 4 && N <= kLongLine && !ADJ);

// The forward pass with staged tables stages the continuation matrix
// ((C + E) x 2d entries) in LDS when it has at most kFcTab entries.  The
// forward pass with global twiddles (whose LDS holds the multipliers
// instead) loads each continuation lane's row into registers at the start;
// the transpose and the long lines read it from global memory (staged, the
// transpose is 9 % slower at N_p = 540).  Reads go through the staged copy
// or the table, chosen by a uniform flag, so that each is an LDS or a global
// load (a pointer that may be either compiles to flat loads).
template <bool ADJ, int N, bool TG>
constexpr bool kMxGlobal = ADJ || N > kLongLine || TG;

// Forward pass with global twiddles up to kLongLine: continuation rows in
// registers, loaded with the unit.
template <bool ADJ, int N, bool TG>
constexpr bool kMxPrefetch = !ADJ && TG && N <= kLongLine;

// Continuation-matrix reads through address-space-qualified pointers: the
// staged copy (LDS) or the table (global memory), selected by a uniform flag.
typedef __attribute__((address_space(3))) const double* lds_cdptr;
typedef __attribute__((address_space(1))) const double* glb_cdptr;
// Mx: the staged copy when staged, else the table (the long lines read
// through it unqualified: never staged).
template <int N>
__device__ __forceinline__ double mx_at(bool staged, const double* MxS, const double* Mx, int i) {
  if constexpr (N > kLongLine) {
    return Mx[i];
  } else {
    if (staged) return ((lds_cdptr)MxS)[i];
    return ((glb_cdptr)Mx)[i];
  }
}

struct MxRows {
  double mr[kMaxFcD], ml[kMaxFcD];
  // row `lane` (< C + E) of the continuation matrix: its d right and d left
  // matching-value coefficients
  __device__ __forceinline__ void load(const FcPlanDev& fc, int lane) {
    const int dd = fc.d;
    const bool on = lane < fc.C + fc.E;
#pragma unroll
    for (int k = 0; k < kMaxFcD; ++k) {
      mr[k] = (on && k < dd) ? fc.Mx[lane * 2 * dd + k] : 0.0;
      ml[k] = (on && k < dd) ? fc.Mx[lane * 2 * dd + dd + k] : 0.0;
    }
  }
};

__host__ __device__ inline int l4_staged_mx(const FcPlanDev& fc, bool mx_global) {
  const int nmx = 2 * fc.d * (fc.C + fc.E);
  return (mx_global || nmx > kFcTab) ? 0 : nmx;
}

template <typename T, bool ADJ, int N1, int N2, bool TG>
inline size_t l4_lds_bytes(const FcPlanDev& fc) {
  return L4Smem<N1, N2>::bytes(l4_staged_mx(fc, kMxGlobal<ADJ, N1 * N2, TG>), TG, kMuStaged<T, TG, N1 * N2, ADJ>);
}

__device__ __forceinline__ int rix(int e) { return e + (e >> 4); }

// Value of the neighbouring lane (lane ^ 1) of a lane pair: DPP quad
// permutation [1, 0, 3, 2] on the two 32-bit halves.  Both lanes of every
// pair must be active.
__device__ __forceinline__ double pair_swap(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Staging of one (point, line) lane: x = its 4 slots (scaled), it = its line.
// Writes complex lines 2 it and 2 it + 1 at LDS position ph: line r holds
// {first line's slot r, second line's slot r}.
__device__ __forceinline__ void stage_pair(cx<double>* buf, int LSZ, int ph, int it, const double* x) {
  const bool odd = it != 0;
  const double r0 = pair_swap(odd ? x[0] : x[2]);
  const double r1 = pair_swap(odd ? x[1] : x[3]);
  // it = 0: lines 0, 1 = {x0, r0}, {x1, r1}; it = 1: lines 2, 3 = {r0, x2}, {r1, x3}
  const cx<double> a = {odd ? r0 : x[0], odd ? x[2] : r0};
  const cx<double> b = {odd ? r1 : x[1], odd ? x[3] : r1};
  buf[(2 * it) * LSZ + ph] = a;
  buf[(2 * it + 1) * LSZ + ph] = b;
}

template <typename T, int TMAX, int N1, int N2, int NTH>
__device__ __forceinline__ void stage_unit(const UnitRegs<T, TMAX>& R, const UnitDesc& d, const double* coef,
                                           bool adj, int n, int tid, cx<double>* buf) {
  typedef L4Smem<N1, N2> SM;
  double cf[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cf[r] = adj ? coef[d.s0 + r] : 1.0;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int e = tid + NTH * t, it = e & 1, i = e >> 1;
    if (i < n) {   // both lanes of a pair have the same point i
      const int ph = (i / N2) * SM::PS + i % N2;
      double x[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = cf[r] * (double)R.v[t][r];
      stage_pair(buf, SM::LSZ, ph, it, x);
    }
  }
  if (adj) {
    const int ext = SM::N - n;
    for (int e = tid; e < kLP * ext; e += NTH) {
      const int l = e / ext, i = n + e % ext;
      buf[l * SM::LSZ + (i / N2) * SM::PS + i % N2] = {0.0, 0.0};
    }
  }
}

// Twiddles w^(b k), k = 1 .. K - 1, of the length-N roots table: only the
// table values w^(b 2^j) are loaded, and every other power is one complex
// product of an earlier power and one of them, at most log2 K products deep
// (relative error a few units in the last place).  Loading 5 values instead
// of K - 1 leaves the vector memory pipe to the state streams.  Used up to
// kLongLine; the long lines load every twiddle.
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <int N, int K>
struct TwPow {
  static constexpr int NB = ilog2c(K - 1) + 1;   // powers 2^0 .. 2^(NB-1) <= K - 1
  cx<double> P[NB];
  cx<double> w[K];
  // TG: from the global table; otherwise from the staged copy in LDS (both
  // paths then do identical arithmetic)
  template <bool TG>
  __device__ __forceinline__ void init(const double* groots, const cx<double>* roots, int b) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = (b << j) % N;
      P[j] = TG ? cx<double>{groots[2 * e], groots[2 * e + 1]} : roots[rix(e)];
    }
  }
  template <int k>
  __device__ __forceinline__ cx<double> get() {
    constexpr int lb = k & -k;
    constexpr int j = ilog2c(lb);
    static_assert(j < NB, "power table too short");
    if constexpr (k == lb) {
      w[k] = P[j];
    } else {
      const cx<double> a = w[k - lb], p = P[j];
      w[k] = {a.re * p.re - a.im * p.im, a.re * p.im + a.im * p.re};
    }
    return w[k];
  }
};

// x[k] *= w^(S b k) for k = k0 .. K - 1 (S = +-1 conjugates)
template <int N, int K, int k, int S>
struct TwApply {
  static __device__ __forceinline__ void run(TwPow<N, K>& tp, cx<double>* x) {
    const cx<double> w = tp.template get<k>();
    x[k] = cx_rot(x[k], w.re, S * w.im);
    TwApply<N, K, k + 1, S>::run(tp, x);
  }
};
template <int N, int K, int S>
struct TwApply<N, K, K, S> {
  static __device__ __forceinline__ void run(TwPow<N, K>&, cx<double>*) {}
};

// Continuation, derivative (or its transpose) and store of one staged unit.
template <typename T, bool ADJ, int N1, int N2, int NTH, bool TG>
__device__ __forceinline__ void transform_unit(const Lines4Args<T>& a, const UnitDesc& d, int n, int dd, int CE,
                                               int tid, cx<double>* buf, const cx<double>* roots,
                                               const double* mu, const double* Mx, const double* MxS, bool mx_st,
                                               const MxRows& mxr) {
  const double* __restrict__ groots = a.fc.roots;
  const double* __restrict__ gmu = a.fc.mu;
  typedef L4Smem<N1, N2> SM;
  constexpr int N = SM::N, PS = SM::PS, LSZ = SM::LSZ;
  auto ph = [](int i) { return (i / N2) * PS + i % N2; };

  if (!ADJ) {
    // extension values (Sec. 4.3 steps 1-4 as one linear map of the 2d
    // matching values); lane p < C + E computes position n + p of each line
    if (tid < CE) {
      const int lane = tid;
      double sr[kLP], si[kLP];
#pragma unroll
      for (int l = 0; l < kLP; ++l) sr[l] = si[l] = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxFcD; ++k) {
        if (k < dd) {
          constexpr bool PF = kMxPrefetch<ADJ, N1 * N2, TG>;
          const double mr = PF ? mxr.mr[k] : mx_at<N>(mx_st, MxS, Mx, lane * 2 * dd + k);
          const double ml = PF ? mxr.ml[k] : mx_at<N>(mx_st, MxS, Mx, lane * 2 * dd + dd + k);
#pragma unroll
          for (int l = 0; l < kLP; ++l) {
            const cx<double> gr = buf[l * LSZ + ph(n - dd + k)];
            const cx<double> gl = buf[l * LSZ + ph(dd - 1 - k)];
            sr[l] += mr * gr.re + ml * gl.re;
            si[l] += mr * gr.im + ml * gl.im;
          }
        }
      }
#pragma unroll
      for (int l = 0; l < kLP; ++l) buf[l * LSZ + ph(n + lane)] = {sr[l], si[l]};
    }
    __syncthreads();
  }

  // step A: length-N1 transforms along the stride-N2 index
  for (int job = tid; job < kLP * N2; job += NTH) {
    const int l = job / N2, n2 = job % N2;
    cx<double> x[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = buf[l * LSZ + i * PS + n2];
    Dft<N1, -1, double>::run(x);
    if constexpr (N <= kLongLine) {
      TwPow<N, N1> tp;
      tp.template init<TG>(groots, roots, n2);
      TwApply<N, N1, 1, 1>::run(tp, x);
    } else {
#pragma unroll
      for (int k1 = 1; k1 < N1; ++k1) {
        const int e = (n2 * k1) % N;
        const cx<double> w = TG ? cx<double>{groots[2 * e], groots[2 * e + 1]} : roots[rix(e)];
        x[k1] = cx_rot(x[k1], w.re, w.im);
      }
    }
#pragma unroll
    for (int i = 0; i < N1; ++i) buf[l * LSZ + i * PS + n2] = x[i];
  }
  __syncthreads();
  // step B: length-N2 transforms, derivative factor, inverse transforms
  for (int job = tid; job < kLP * N1; job += NTH) {
    const int l = job / N1, k1 = job % N1;
    cx<double> x[N2];
#pragma unroll
    for (int i = 0; i < N2; ++i) x[i] = buf[l * LSZ + k1 * PS + i];
    Dft<N2, -1, double>::run(x);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const double m = kMuStaged<T, TG, N, ADJ> ? mu[k1 + N1 * k2] : gmu[k1 + N1 * k2];
      const cx<double> X = x[k2];
      x[k2] = ADJ ? cx<double>{m * X.im, -m * X.re} : cx<double>{-m * X.im, m * X.re};
    }
    Dft<N2, 1, double>::run(x);
    if constexpr (N <= kLongLine) {
      TwPow<N, N2> tp;
      tp.template init<TG>(groots, roots, k1);
      TwApply<N, N2, 1, -1>::run(tp, x);
    } else {
#pragma unroll
      for (int n2 = 1; n2 < N2; ++n2) {
        const int e = (n2 * k1) % N;
        const cx<double> w = TG ? cx<double>{groots[2 * e], groots[2 * e + 1]} : roots[rix(e)];
        x[n2] = cx_rot(x[n2], w.re, -w.im);
      }
    }
#pragma unroll
    for (int i = 0; i < N2; ++i) buf[l * LSZ + k1 * PS + i] = x[i];
  }
  __syncthreads();

  // step A': inverse length-N1 transforms
  for (int job = tid; job < kLP * N2; job += NTH) {
    const int l = job / N2, n2 = job % N2;
    cx<double> x[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = buf[l * LSZ + i * PS + n2];
    Dft<N1, 1, double>::run(x);
#pragma unroll
    for (int i = 0; i < N1; ++i) buf[l * LSZ + i * PS + n2] = x[i];
  }
  __syncthreads();

  if (ADJ) {
    // fold the extension region back onto the 2d matching points (transpose
    // of the continuation): thread t < kLP 2d forms column c of line l, and
    // after every thread has read the region stores it at position n + c
    static_assert(kLP * 2 * kMaxFcD <= NTH, "one fold column per thread");
    const bool act = tid < kLP * 2 * dd;
    const int l = tid / (2 * dd), c = tid % (2 * dd);
    double sr = 0.0, si = 0.0;
    if (act) {
#pragma unroll 4
      for (int p = 0; p < CE; ++p) {
        const double mv = mx_at<N>(mx_st, MxS, Mx, p * 2 * dd + c);
        const cx<double> y = buf[l * LSZ + ph(n + p)];
        sr += mv * y.re;
        si += mv * y.im;
      }
    }
    __syncthreads();
    if (act) buf[l * LSZ + ph(n + c)] = {sr, si};
    __syncthreads();
  }

  // epilogue: scale (forward) or add the fold (transpose) and store
  double c4[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) c4[r] = ADJ ? 1.0 : -a.coef[d.dir][d.s0 + r];
  T* out = a.out[d.dir] + d.base;
  const int64_t ls = a.line_stride[d.dir], ps = a.pt_stride[d.dir];
  constexpr int TMAX = (2 * N + NTH - 1) / NTH;
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    const int e = tid + NTH * t, it = e & 1, i = e >> 1;
    if (i < n) {   // both lanes of a pair have the same point i
      // complex lines 2 it, 2 it + 1 of this point (plus the fold), then the
      // lane's own line: two slots from its entries, two from its partner's
      cx<double> z0 = buf[(2 * it) * LSZ + ph(i)], z1 = buf[(2 * it + 1) * LSZ + ph(i)];
      if (ADJ) {
        if (i >= n - dd) {
          const int fp = ph(n + (i - (n - dd)));
          z0 = cx_add(z0, buf[(2 * it) * LSZ + fp]);
          z1 = cx_add(z1, buf[(2 * it + 1) * LSZ + fp]);
        }
        if (i < dd) {
          const int fp = ph(n + dd + (dd - 1 - i));
          z0 = cx_add(z0, buf[(2 * it) * LSZ + fp]);
          z1 = cx_add(z1, buf[(2 * it + 1) * LSZ + fp]);
        }
      }
      const bool odd = it != 0;
      const double r0 = pair_swap(odd ? z0.re : z0.im);
      const double r1 = pair_swap(odd ? z1.re : z1.im);
      // it = 0: {z0.re, z1.re, r0, r1}; it = 1: {r0, r1, z0.im, z1.im}
      const double dv[4] = {odd ? r0 : z0.re, odd ? r1 : z1.re, odd ? z0.im : r0, odd ? z1.im : r1};
      if (it == 1 && !d.has1) continue;
      T* q = out + it * ls + (int64_t)i * ps;
      if constexpr (N <= kLongLine) {
        const double sv[4] = {c4[0] * dv[0], c4[1] * dv[1], c4[2] * dv[2], c4[3] * dv[3]};
        if constexpr (sizeof(T) == 4 || ADJ) {
          if (a.nt_out) store_slots<true>(q, sv);
          else store_slots<false>(q, sv);
        } else {
          store_slots<false>(q, sv);
        }
      } else if constexpr (sizeof(T) == 8) {
        reinterpret_cast<double2*>(q)[0] = make_double2(c4[0] * dv[0], c4[1] * dv[1]);
        reinterpret_cast<double2*>(q)[1] = make_double2(c4[2] * dv[2], c4[3] * dv[3]);
      } else {
        *reinterpret_cast<float4*>(q) =
            make_float4(float(c4[0] * dv[0]), float(c4[1] * dv[1]), float(c4[2] * dv[2]), float(c4[3] * dv[3]));
      }
    }
  }
}

// Issue the loads of the FC tables into registers (kept until staged).
// MXG: the continuation matrix stays in global memory (long lines).
template <int N, int NTH, bool TG, bool MXG, bool MUS>
struct TabRegs {
  static constexpr int RT = TG ? 1 : (N + NTH - 1) / NTH, MT = MUS ? (N + NTH - 1) / NTH : 1,
                       XT = MXG ? 1 : (kFcTab + NTH - 1) / NTH;
  double rr[RT][2], mm[MT], xx[XT];
  __device__ __forceinline__ void load(const FcPlanDev& fc, int lane) {
    const int nmx = l4_staged_mx(fc, MXG);
    if (!TG) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int k = lane + NTH * t;
        rr[t][0] = (k < N) ? fc.roots[2 * k] : 0.0;
        rr[t][1] = (k < N) ? fc.roots[2 * k + 1] : 0.0;
      }
    }
    if (MUS) {
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int k = lane + NTH * t;
        mm[t] = (k < N) ? fc.mu[k] : 0.0;
      }
    }
    if (!MXG) {
#pragma unroll
      for (int t = 0; t < XT; ++t) {
        const int k = lane + NTH * t;
        xx[t] = (k < nmx) ? fc.Mx[k] : 0.0;
      }
    }
  }
  __device__ __forceinline__ void stage(cx<double>* roots, double* mu, double* Mx, int nmx, int lane) const {
    if (!TG) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int k = lane + NTH * t;
        if (k < N) roots[rix(k)] = {rr[t][0], rr[t][1]};
      }
    }
    if (MUS) {
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int k = lane + NTH * t;
        if (k < N) mu[k] = mm[t];
      }
    }
    if (!MXG) {
#pragma unroll
      for (int t = 0; t < XT; ++t) {
        const int k = lane + NTH * t;
        if (k < nmx) Mx[k] = xx[t];
      }
    }
  }
};

// A workgroup of NW waves (NTH = 64 NW threads) transforms one unit at a
// time.  UPW = 2: the workgroup's two units and the tables are all loaded
// before the first transform.  UPW = 1 (also for long lines, whose loads alone
// would fill the register file): tables first, then the unit in chunks of
// 8 load slots per thread.
template <typename T, bool ADJ, int N1, int N2, int UPW, int NW, bool TG>
__global__ __launch_bounds__(64 * NW) void lines4_kernel(Lines4Args<T> a) {
  constexpr int N = N1 * N2;
  constexpr int NTH = 64 * NW;
  constexpr int TMAX = (2 * N + NTH - 1) / NTH;
  constexpr bool MXG = kMxGlobal<ADJ, N, TG>;
  constexpr bool MUS = kMuStaged<T, TG, N, ADJ>;
  typedef L4Smem<N1, N2> SM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  cx<double>* buf = reinterpret_cast<cx<double>*>(sm);
  cx<double>* roots = reinterpret_cast<cx<double>*>(sm + SM::BUF);
  double* mu = sm + SM::mu_off(TG);
  double* MxS = sm + SM::mx_off(TG, MUS);       // staged copy (unused when nmx_st == 0)
  const int nmx_st = l4_staged_mx(a.fc, MXG);
  const double* Mx = nmx_st ? MxS : a.fc.Mx;
  const bool mx_st = nmx_st != 0;

  const FcPlanDev& fc = a.fc;
  const int n = fc.n, dd = fc.d, CE = fc.C + fc.E;
  const int tid = threadIdx.x;
  MxRows mxr;
  if constexpr (kMxPrefetch<ADJ, N, TG>) mxr.load(fc, tid);

  if constexpr (UPW == 2) {
    const UnitDesc d0 = decode_unit(a, 2 * (int)blockIdx.x);
    const UnitDesc d1 = decode_unit(a, 2 * (int)blockIdx.x + 1);
    UnitRegs<T, TMAX> R0, R1;
    load_unit<T, TMAX, NTH>(a, d0, n, tid, R0);
    load_unit<T, TMAX, NTH>(a, d1, n, tid, R1);
    TabRegs<N, NTH, TG, MXG, MUS> tab;
    tab.load(fc, tid);
    tab.stage(roots, mu, MxS, nmx_st, tid);
    if (d0.live) {
      stage_unit<T, TMAX, N1, N2, NTH>(R0, d0, a.coef[d0.dir], ADJ, n, tid, buf);
      __syncthreads();
      transform_unit<T, ADJ, N1, N2, NTH, TG>(a, d0, n, dd, CE, tid, buf, roots, mu, Mx, MxS, mx_st, mxr);
    }
    if (d1.live) {
      __syncthreads();
      stage_unit<T, TMAX, N1, N2, NTH>(R1, d1, a.coef[d1.dir], ADJ, n, tid, buf);
      __syncthreads();
      transform_unit<T, ADJ, N1, N2, NTH, TG>(a, d1, n, dd, CE, tid, buf, roots, mu, Mx, MxS, mx_st, mxr);
    }
  } else {
    const UnitDesc d0 = decode_unit(a, remap_unit16((int)blockIdx.x));
    if (!d0.live) return;
    {
      TabRegs<N, NTH, TG, MXG, MUS> tab;
      tab.load(fc, tid);
      tab.stage(roots, mu, MxS, nmx_st, tid);
    }
    constexpr int CH = 8;
    for (int c0 = 0; c0 < TMAX; c0 += CH) {
      UnitRegs<T, CH> R;
      const T* in = a.in + d0.base;
      const int64_t ls = a.line_stride[d0.dir], ps = a.pt_stride[d0.dir];
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int e = tid + NTH * (c0 + t), it = e & 1, i = e >> 1;
        if (c0 + t < TMAX && i < n && (it == 0 || d0.has1)) {
          const T* p = in + it * ls + (int64_t)i * ps;
          if constexpr (sizeof(T) == 8) {
            const double2 x = reinterpret_cast<const double2*>(p)[0];
            const double2 y = reinterpret_cast<const double2*>(p)[1];
            R.v[t][0] = x.x; R.v[t][1] = x.y; R.v[t][2] = y.x; R.v[t][3] = y.y;
          } else {
            const float4 x = *reinterpret_cast<const float4*>(p);
            R.v[t][0] = x.x; R.v[t][1] = x.y; R.v[t][2] = x.z; R.v[t][3] = x.w;
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) R.v[t][r] = T(0);
        }
      }
      const double* cf = a.coef[d0.dir];
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        const int e = tid + NTH * (c0 + t), it = e & 1, i = e >> 1;
        if (c0 + t < TMAX && i < n) {
          const int ph = (i / N2) * SM::PS + i % N2;
          double x[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) x[r] = (ADJ ? cf[d0.s0 + r] : 1.0) * (double)R.v[t][r];
          stage_pair(buf, SM::LSZ, ph, it, x);
        }
      }
    }
    if (ADJ) {
      const int ext = N - n;
      for (int e = tid; e < kLP * ext; e += NTH) {
        const int l = e / ext, i = n + e % ext;
        buf[l * SM::LSZ + (i / N2) * SM::PS + i % N2] = {0.0, 0.0};
      }
    }
    __syncthreads();
    transform_unit<T, ADJ, N1, N2, NTH, TG>(a, d0, n, dd, CE, tid, buf, roots, mu, Mx, MxS, mx_st, mxr);
  }
}

// Two units per workgroup only where both units' loads fit in registers.
template <int N1, int N2, int NW>
constexpr bool kPairOk = (2 * N1 * N2 + 64 * NW - 1) / (64 * NW) <= 9;

template <typename T, bool ADJ, int N1, int N2, int NW, bool TG>
inline hipError_t go_nw(const Lines4Args<T>& a, int upw, hipStream_t s) {
  const size_t sh = l4_lds_bytes<T, ADJ, N1, N2, TG>(a.fc);
  if (sh > kLines4MaxLds) return hipErrorNotSupported;
  if constexpr (kPairOk<N1, N2, NW>) {
    if (upw == 2) {
      const int groups = (a.nunits + 1) / 2;
      if (groups == 0) return hipSuccess;
      hipLaunchKernelGGL((lines4_kernel<T, ADJ, N1, N2, 2, NW, TG>), dim3((unsigned)groups), dim3(64 * NW), sh, s, a);
      return hipGetLastError();
    }
  }
  if (a.nunits == 0) return hipSuccess;
  const int groups = ((a.nunits + 15) / 16) * 16;
  hipLaunchKernelGGL((lines4_kernel<T, ADJ, N1, N2, 1, NW, TG>), dim3((unsigned)groups), dim3(64 * NW), sh, s, a);
  return hipGetLastError();
}

// One unit per two-wave workgroup, tables from global memory: the only
// variant instantiated for the lengths outside the fully tuned set.
template <typename T, bool ADJ, int N1, int N2>
inline hipError_t go_one(const Lines4Args<T>& a, hipStream_t s) {
  const size_t sh = l4_lds_bytes<T, ADJ, N1, N2, true>(a.fc);
  if (sh > kLines4MaxLds) return hipErrorNotSupported;
  if (a.nunits == 0) return hipSuccess;
  const int groups = ((a.nunits + 15) / 16) * 16;
  hipLaunchKernelGGL((lines4_kernel<T, ADJ, N1, N2, 1, 2, true>), dim3((unsigned)groups), dim3(128), sh, s, a);
  return hipGetLastError();
}

// Lengths outside the fully tuned set are instantiated once (one unit per
// two-wave workgroup, tables read from global memory) in the files
// line4_extra*.hip; each returns hipErrorNotSupported for lengths it lacks.
hipError_t lines4_extra0(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_extra0(const Lines4Args<float>& a, bool adj, hipStream_t s);
hipError_t lines4_extra1(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_extra1(const Lines4Args<float>& a, bool adj, hipStream_t s);
hipError_t lines4_extra2(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_extra2(const Lines4Args<float>& a, bool adj, hipStream_t s);
hipError_t lines4_extra3(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_extra3(const Lines4Args<float>& a, bool adj, hipStream_t s);

// Extended lengths above kLongLine: one unit per two-wave workgroup, twiddles,
// multipliers and continuation matrix from global memory (line4_long*.hip).
template <typename T, bool ADJ, int N1, int N2>
inline hipError_t go_long(const Lines4Args<T>& a, hipStream_t s) {
  static_assert(N1 * N2 > kLongLine, "long-line variant");
  const size_t sh = l4_lds_bytes<T, ADJ, N1, N2, true>(a.fc);
  if (sh > kLines4MaxLdsLong) return hipErrorNotSupported;
  if (a.nunits == 0) return hipSuccess;
  const int groups = ((a.nunits + 15) / 16) * 16;
  hipLaunchKernelGGL((lines4_kernel<T, ADJ, N1, N2, 1, 2, true>), dim3((unsigned)groups), dim3(128), sh, s, a);
  return hipGetLastError();
}

hipError_t lines4_long0(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_long0(const Lines4Args<float>& a, bool adj, hipStream_t s);
hipError_t lines4_long1(const Lines4Args<double>& a, bool adj, hipStream_t s);
hipError_t lines4_long1(const Lines4Args<float>& a, bool adj, hipStream_t s);

}  // namespace rte
