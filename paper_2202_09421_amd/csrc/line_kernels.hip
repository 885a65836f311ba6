// Line passes of the FC-DOM step: FC-Gram continuation + filtered spectral
// derivative along x lines (rows) or y lines (columns), and its exact
// transpose for the adjoint (Sec. 4.3; Algorithm 1, loops over y_j and x_i).
//
// Storage: a state is [q][g][j][i][r] with g = ordinate group (4 slots),
// r = slot within the group and rows padded to nxp nodes, so a row of one
// group is contiguous and a column of one group is a run of 32-byte (FP64)
// chunks.  This generic kernel (any 5-smooth N_p, runtime Stockham passes)
// serves the lengths without a four-step split.  One workgroup handles one
// (line, group, source): the 4 slots form two complex lines (slots r0 + i r1
// and r2 + i r3), differentiated together since the FC operator is
// real-linear.
//
// Forward derivative of a complex line z (n points):
//   c_R = Q^T z[n-d..n-1], c_L = Q^T rev(z[0..d-1])          (Gram projection)
//   z[n+p] = (A c_R)[p] (p < C) + (A c_L)[C+E-1-p] (p >= E)  (blends + E zeros)
//   Z = FFT(z); Y = i mu_k Z  (mu = 2 pi kappa / (Np h) * filter / Np, 0 at Nyquist)
//   Dz = IFFT(Y * Np) = conj(FFT(conj(Y)))
// Transpose: zero-extend, multiply by -i mu, inverse, then fold the extension
// region back through A and Q onto the first and last d points.
#include "fft_lds.h"
#include "rte_internal.h"

namespace rte {

template <typename T>
struct LineArgs {
  const T* in;
  T* out;
  const double* coef;  // xi or eta per slot
  FcPlanDev fc;
  int nlines;
  int64_t line_stride, pt_stride, grp_stride, inst_stride;
};

// XCD-aware line index: the 8 XCDs receive blocks round-robin, so block b
// runs on XCD b % 8.  Lines 4x..4x+3 of every chunk of 32 go to XCD x, which
// keeps neighbouring columns (sharing 128-byte lines of the y pass) in one L2.
__device__ __forceinline__ int remap_line(int b) {
  const int chunk = b >> 5;
  const int x = b & 7;
  const int k = (b >> 3) & 3;
  return chunk * 32 + 4 * x + k;
}

template <typename T, bool adj>
__global__ __launch_bounds__(kLineThreads) void line_kernel(LineArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const FcPlanDev& fc = a.fc;
  const int n = fc.n, Np = fc.Np, d = fc.d, C = fc.C, E = fc.E;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int line = remap_line(blockIdx.x);
  if (line >= a.nlines) return;
  const int g = blockIdx.y, q = blockIdx.z;

  // Lines are transformed in FP64 for both storage precisions: in FP32 the
  // FFT rounding noise, multiplied by the derivative factor (up to pi/h),
  // would dominate the detector traces (~1e-4 relative).
  typedef double CT;
  cplx<CT>* bufA = reinterpret_cast<cplx<CT>*>(smem_raw);
  cplx<CT>* bufB = bufA + 2 * Np;
  // 2 lines x 2 ends x kMaxFcD coefficients (x2 for the fold), always FP64:
  // the Gram projection of the matching values cancels heavily and the blends
  // reach |A| ~ 5e3, so in FP32 it would lose ~4 digits
  cplx<double>* cs = reinterpret_cast<cplx<double>*>(bufB + 2 * Np);

  const int64_t base = (int64_t)q * a.inst_stride + (int64_t)g * a.grp_stride + (int64_t)line * a.line_stride;
  const T* in = a.in + base;
  const int s0 = g * kGroup;

  CT cf[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cf[r] = adj ? CT(a.coef[s0 + r]) : CT(1);

  // ---- load the line (4 slots per point) into two complex lines
  for (int i = tid; i < n; i += nthr) {
    const T* p = in + (int64_t)i * a.pt_stride;
    const CT v0 = p[0], v1 = p[1], v2 = p[2], v3 = p[3];
    bufA[i] = {v0 * cf[0], v1 * cf[1]};
    bufA[Np + i] = {v2 * cf[2], v3 * cf[3]};
  }
  if (adj) {
    for (int i = n + tid; i < Np; i += nthr) {
      bufA[i] = {CT(0), CT(0)};
      bufA[Np + i] = {CT(0), CT(0)};
    }
  }
  __syncthreads();

  if (!adj) {
    // ---- Gram projections of the matching values (Sec. 4.3 step 1)
    for (int t = tid; t < 4 * d; t += nthr) {
      const int ln = t / (2 * d), rem = t % (2 * d), end = rem / d, j = rem % d;
      const cplx<CT>* z = bufA + ln * Np;
      double sr = 0, si = 0;
      for (int k = 0; k < d; ++k) {
        const double qv = fc.Q[k * d + j];
        const cplx<CT> v = end ? z[n - d + k] : z[d - 1 - k];
        sr += qv * (double)v.re;
        si += qv * (double)v.im;
      }
      cs[(ln * 2 + end) * kMaxFcD + j] = {sr, si};
    }
    __syncthreads();
    // ---- blends to zero, zero padding, sum (steps 2-4)
    const int CE = C + E;
    for (int t = tid; t < 2 * CE; t += nthr) {
      const int ln = t / CE, p = t % CE;
      const cplx<double>* cL = cs + (ln * 2 + 0) * kMaxFcD;
      const cplx<double>* cR = cs + (ln * 2 + 1) * kMaxFcD;
      double sr = 0, si = 0;
      if (p < C) {
        for (int j = 0; j < d; ++j) {
          const double av = fc.A[p * d + j];
          sr += av * cR[j].re;
          si += av * cR[j].im;
        }
      }
      if (p >= E) {
        const int pp = CE - 1 - p;
        for (int j = 0; j < d; ++j) {
          const double av = fc.A[pp * d + j];
          sr += av * cL[j].re;
          si += av * cL[j].im;
        }
      }
      bufA[ln * Np + n + p] = {CT(sr), CT(si)};
    }
    __syncthreads();
  }

  // ---- forward FFT
  cplx<CT>* src = bufA;
  cplx<CT>* dst = bufB;
  for (int p = 0; p < fc.npass; ++p) {
    fft_pass<CT>(src, dst, Np, fc.radix[p], fc.ns[p], fc.tw + 2 * fc.twoff[p], 2, Np, tid, nthr);
    __syncthreads();
    cplx<CT>* t = src;
    src = dst;
    dst = t;
  }
  // ---- multiply by +-i mu and conjugate (inverse via a forward transform)
  for (int t = tid; t < 2 * Np; t += nthr) {
    const int k = t % Np;
    const CT m = CT(fc.mu[k]);
    const cplx<CT> X = src[t];
    src[t] = adj ? cplx<CT>{m * X.im, m * X.re} : cplx<CT>{-m * X.im, -m * X.re};
  }
  __syncthreads();
  for (int p = 0; p < fc.npass; ++p) {
    fft_pass<CT>(src, dst, Np, fc.radix[p], fc.ns[p], fc.tw + 2 * fc.twoff[p], 2, Np, tid, nthr);
    __syncthreads();
    cplx<CT>* t = src;
    src = dst;
    dst = t;
  }
  // src now holds conj(derivative) at all Np positions

  if (adj) {
    // ---- fold the extension region back (transpose of steps 1-4)
    cplx<double>* ys = cs;                // [ln][end][j]: A^T z_ext
    cplx<double>* gs = cs + 4 * kMaxFcD;  // [ln][end][k]: Q (A^T z_ext)
    for (int t = tid; t < 4 * d; t += nthr) {
      const int ln = t / (2 * d), rem = t % (2 * d), end = rem / d, j = rem % d;
      const cplx<CT>* z = src + ln * Np;
      double sr = 0, si = 0;
      for (int p = 0; p < C; ++p) {
        const double av = fc.A[p * d + j];
        const cplx<CT> v = end ? z[n + p] : z[Np - 1 - p];
        sr += av * (double)v.re;
        si -= av * (double)v.im;  // conjugate on the fly
      }
      ys[(ln * 2 + end) * kMaxFcD + j] = {sr, si};
    }
    __syncthreads();
    for (int t = tid; t < 4 * d; t += nthr) {
      const int ln = t / (2 * d), rem = t % (2 * d), end = rem / d, k = rem % d;
      const cplx<double>* y = ys + (ln * 2 + end) * kMaxFcD;
      double sr = 0, si = 0;
      for (int j = 0; j < d; ++j) {
        const double qv = fc.Q[k * d + j];
        sr += qv * y[j].re;
        si += qv * y[j].im;
      }
      gs[(ln * 2 + end) * kMaxFcD + k] = {sr, si};
    }
    __syncthreads();
  }

  // ---- epilogue: scale (forward) or add the fold (transpose) and store
  CT c4[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) c4[r] = adj ? CT(1) : -CT(a.coef[s0 + r]);
  T* out = a.out + base;
  const cplx<double>* gs = cs + 4 * kMaxFcD;
  for (int i = tid; i < n; i += nthr) {
    const cplx<CT> z0 = src[i], z1 = src[Np + i];
    CT dv[4] = {z0.re, -z0.im, z1.re, -z1.im};
    if (adj) {
      if (i >= n - d) {
        const int k = i - (n - d);
        dv[0] += gs[(0 * 2 + 1) * kMaxFcD + k].re;
        dv[1] += gs[(0 * 2 + 1) * kMaxFcD + k].im;
        dv[2] += gs[(1 * 2 + 1) * kMaxFcD + k].re;
        dv[3] += gs[(1 * 2 + 1) * kMaxFcD + k].im;
      }
      if (i < d) {
        const int k = d - 1 - i;
        dv[0] += gs[(0 * 2 + 0) * kMaxFcD + k].re;
        dv[1] += gs[(0 * 2 + 0) * kMaxFcD + k].im;
        dv[2] += gs[(1 * 2 + 0) * kMaxFcD + k].re;
        dv[3] += gs[(1 * 2 + 0) * kMaxFcD + k].im;
      }
    }
    const int64_t off = (int64_t)i * a.pt_stride;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[off + r] = T(c4[r] * dv[r]);
  }
}

template <typename T, bool adj>
static hipError_t launch_mode(const Plan& p, const void* in, void* out, int dir, hipStream_t s) {
  LineArgs<T> a;
  a.in = static_cast<const T*>(in);
  a.out = static_cast<T*>(out);
  a.coef = (dir == 0) ? p.dev.xi : p.dev.eta;
  a.fc = (dir == 0) ? p.fcx : p.fcy;
  a.grp_stride = p.grp_stride;
  a.inst_stride = p.inst_stride;
  if (dir == 0) {
    a.nlines = (int)p.ny;
    a.line_stride = p.nxp * kGroup;
    a.pt_stride = kGroup;
  } else {
    a.nlines = (int)p.nx;
    a.line_stride = kGroup;
    a.pt_stride = p.nxp * kGroup;
  }
  const int Np = a.fc.Np;
  const size_t shmem = line_shmem_bytes(Np, p.dtype);
  dim3 grid((unsigned)(((a.nlines + 31) / 32) * 32), (unsigned)p.G, (unsigned)p.cnq);
  hipLaunchKernelGGL((line_kernel<T, adj>), grid, dim3(kLineThreads), shmem, s, a);
  return hipGetLastError();
}

hipError_t launch_line_generic(const Plan& p, const void* in, void* out, int mode, int dir, hipStream_t s) {
  if (p.dtype == RTE_F64)
    return mode == LINE_ADJ ? launch_mode<double, true>(p, in, out, dir, s) : launch_mode<double, false>(p, in, out, dir, s);
  return mode == LINE_ADJ ? launch_mode<float, true>(p, in, out, dir, s) : launch_mode<float, false>(p, in, out, dir, s);
}

// Both line sets: one four-step launch when the x and y plans coincide,
// otherwise one launch per direction (four-step where N_p has a split).
hipError_t launch_lines(const Plan& p, const LineLaunch& L, hipStream_t s) {
  const bool four_x = p.fcx.n1 > 0 && !p.sched.line_generic, four_y = p.fcy.n1 > 0 && !p.sched.line_generic;
  if (L.dirs == 3 && p.fc_same && four_x) {
    const hipError_t e = launch_lines4(p, L, s);
    if (e != hipErrorNotSupported) return e;
  }
  for (int dir = 0; dir < 2; ++dir) {
    if (!(L.dirs & (1 << dir))) continue;
    void* out = dir == 0 ? L.out_x : L.out_y;
    hipError_t e = hipErrorNotSupported;
    if (dir == 0 ? four_x : four_y) {
      LineLaunch one = L;
      one.dirs = 1 << dir;
      e = launch_lines4(p, one, s);
    }
    if (e == hipErrorNotSupported) e = launch_line_generic(p, L.in, out, L.mode, dir, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Static LDS limit check used by the plan (bytes of dynamic shared memory).
size_t line_shmem_bytes(int Np, int /*dtype*/) {
  return sizeof(cplx<double>) * (size_t)(4 * Np + 8 * kMaxFcD);
}

}  // namespace rte
