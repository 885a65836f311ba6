// Four-step line passes for the common extended lengths N_p = N1 * N2.
//
// Same operation as line_kernels.hip (FC-Gram continuation + filtered
// spectral derivative along x or y lines, or its transpose; Sec. 4.3), but
// the DFT of length N_p is split as in the four-step algorithm:
//   A : N2 transforms of length N1 over the stride-N2 index, twiddle w^{n2 k1}
//   B : N1 transforms of length N2 over each contiguous block, multiply by
//       the derivative factor i mu_k at k = k1 + N1 k2, inverse length-N2
//       transform, twiddle w^{-n2 k1}
//   A': N2 inverse transforms of length N1
// Each transform is a compile-time codelet held in registers, so a line makes
// three LDS round trips instead of one per radix pass.  A workgroup is one
// wave and handles four complex lines: two neighbouring lines (rows or
// columns) of one ordinate group, each giving two complex lines.  LDS rows of
// N2 entries are padded by one entry to spread the block reads of step B
// over the banks.
#include "fft_codelets.h"
#include "rte_internal.h"

namespace rte {

template <typename T>
struct Line4Args {
  const T* in;
  const T* aux;
  const T* aux2;
  T* out;
  const double* coef;
  double cdt;
  FcPlanDev fc;
  int nlines;
  int64_t line_stride, pt_stride, grp_stride, inst_stride;
};

// Block b runs on XCD b % 8; pairs 2x, 2x+1 of every chunk of 16 pairs go to
// XCD x, so four neighbouring columns share one L2.
__device__ __forceinline__ int remap_pair(int b) {
  const int chunk = b >> 4, x = b & 7, k = (b >> 3) & 1;
  return chunk * 16 + 2 * x + k;
}

constexpr int kLP = 4;  // complex lines per workgroup

template <typename T, int MODE, int N1, int N2>
__global__ __launch_bounds__(64) void line4_kernel(Line4Args<T> a) {
  constexpr int N = N1 * N2;
  constexpr int PS = N2 + 1;
  constexpr int LSZ = N1 * PS;
  constexpr bool adj = (MODE == LINE_ADJ_X || MODE == LINE_ADJ_Y);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<double>* buf = reinterpret_cast<cx<double>*>(smem_raw);
  cx<double>* cs = buf + kLP * LSZ;  // [l][end][kMaxFcD] and a second copy for the fold

  const FcPlanDev& fc = a.fc;
  const int n = fc.n, d = fc.d, C = fc.C, E = fc.E;
  const int lane = threadIdx.x;
  const int line0 = 2 * remap_pair(blockIdx.x);
  if (line0 >= a.nlines) return;
  const bool has1 = line0 + 1 < a.nlines;
  const int g = blockIdx.y, q = blockIdx.z;
  const int64_t base0 = (int64_t)q * a.inst_stride + (int64_t)g * a.grp_stride + (int64_t)line0 * a.line_stride;
  const int s0 = g * kGroup;
  auto ph = [](int i) { return (i / N2) * PS + i % N2; };

  double cf[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cf[r] = adj ? a.coef[s0 + r] : 1.0;

  // ---- load two lines x four slots as four complex lines
  for (int e = lane; e < 2 * n; e += 64) {
    const int it = e & 1, i = e >> 1;
    cx<double> z0 = {0.0, 0.0}, z1 = {0.0, 0.0};
    if (it == 0 || has1) {
      const T* p = a.in + base0 + it * a.line_stride + (int64_t)i * a.pt_stride;
      z0 = {cf[0] * (double)p[0], cf[1] * (double)p[1]};
      z1 = {cf[2] * (double)p[2], cf[3] * (double)p[3]};
    }
    buf[(2 * it) * LSZ + ph(i)] = z0;
    buf[(2 * it + 1) * LSZ + ph(i)] = z1;
  }
  if (adj) {
    const int ext = N - n;
    for (int e = lane; e < kLP * ext; e += 64) {
      const int l = e / ext, i = n + e % ext;
      buf[l * LSZ + ph(i)] = {0.0, 0.0};
    }
  }
  __syncthreads();

  if (!adj) {
    // Gram projections (Sec. 4.3 step 1)
    for (int t = lane; t < kLP * 2 * d; t += 64) {
      const int l = t / (2 * d), rem = t % (2 * d), end = rem / d, j = rem % d;
      double sr = 0, si = 0;
      for (int k = 0; k < d; ++k) {
        const double qv = fc.Q[k * d + j];
        const cx<double> v = buf[l * LSZ + ph(end ? n - d + k : d - 1 - k)];
        sr += qv * v.re;
        si += qv * v.im;
      }
      cs[(l * 2 + end) * kMaxFcD + j] = {sr, si};
    }
    __syncthreads();
    // blends to zero, E zeros, sum (steps 2-4)
    const int CE = C + E;
    for (int t = lane; t < kLP * CE; t += 64) {
      const int l = t / CE, p = t % CE;
      double sr = 0, si = 0;
      if (p < C)
        for (int j = 0; j < d; ++j) {
          const double av = fc.A[p * d + j];
          sr += av * cs[(l * 2 + 1) * kMaxFcD + j].re;
          si += av * cs[(l * 2 + 1) * kMaxFcD + j].im;
        }
      if (p >= E) {
        const int pp = CE - 1 - p;
        for (int j = 0; j < d; ++j) {
          const double av = fc.A[pp * d + j];
          sr += av * cs[(l * 2 + 0) * kMaxFcD + j].re;
          si += av * cs[(l * 2 + 0) * kMaxFcD + j].im;
        }
      }
      buf[l * LSZ + ph(n + p)] = {sr, si};
    }
    __syncthreads();
  }

  const double* __restrict__ roots = fc.roots;
  const double* __restrict__ mu = fc.mu;
  // ---- step A: length-N1 transforms along the stride-N2 index
  for (int job = lane; job < kLP * N2; job += 64) {
    const int l = job / N2, n2 = job % N2;
    cx<double> x[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = buf[l * LSZ + i * PS + n2];
    Dft<N1, -1, double>::run(x);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      const int e = (n2 * k1) % N;
      x[k1] = cx_rot(x[k1], roots[2 * e], roots[2 * e + 1]);
    }
#pragma unroll
    for (int i = 0; i < N1; ++i) buf[l * LSZ + i * PS + n2] = x[i];
  }
  __syncthreads();
  // ---- step B: length-N2 transforms, derivative factor, inverse transforms
  for (int job = lane; job < kLP * N1; job += 64) {
    const int l = job / N1, k1 = job % N1;
    cx<double> x[N2];
#pragma unroll
    for (int i = 0; i < N2; ++i) x[i] = buf[l * LSZ + k1 * PS + i];
    Dft<N2, -1, double>::run(x);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const double m = mu[k1 + N1 * k2];
      const cx<double> X = x[k2];
      x[k2] = adj ? cx<double>{m * X.im, -m * X.re} : cx<double>{-m * X.im, m * X.re};
    }
    Dft<N2, 1, double>::run(x);
#pragma unroll
    for (int n2 = 1; n2 < N2; ++n2) {
      const int e = (n2 * k1) % N;
      x[n2] = cx_rot(x[n2], roots[2 * e], -roots[2 * e + 1]);
    }
#pragma unroll
    for (int i = 0; i < N2; ++i) buf[l * LSZ + k1 * PS + i] = x[i];
  }
  __syncthreads();
  // ---- step A': inverse length-N1 transforms
  for (int job = lane; job < kLP * N2; job += 64) {
    const int l = job / N2, n2 = job % N2;
    cx<double> x[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) x[i] = buf[l * LSZ + i * PS + n2];
    Dft<N1, 1, double>::run(x);
#pragma unroll
    for (int i = 0; i < N1; ++i) buf[l * LSZ + i * PS + n2] = x[i];
  }
  __syncthreads();

  cx<double>* gs = cs + kLP * 2 * kMaxFcD;
  if (adj) {
    // fold the extension region back onto the first and last d points
    for (int t = lane; t < kLP * 2 * d; t += 64) {
      const int l = t / (2 * d), rem = t % (2 * d), end = rem / d, j = rem % d;
      double sr = 0, si = 0;
      for (int p = 0; p < C; ++p) {
        const double av = fc.A[p * d + j];
        const cx<double> v = buf[l * LSZ + ph(end ? n + p : N - 1 - p)];
        sr += av * v.re;
        si += av * v.im;
      }
      cs[(l * 2 + end) * kMaxFcD + j] = {sr, si};
    }
    __syncthreads();
    for (int t = lane; t < kLP * 2 * d; t += 64) {
      const int l = t / (2 * d), rem = t % (2 * d), end = rem / d, k = rem % d;
      double sr = 0, si = 0;
      for (int j = 0; j < d; ++j) {
        const double qv = fc.Q[k * d + j];
        sr += qv * cs[(l * 2 + end) * kMaxFcD + j].re;
        si += qv * cs[(l * 2 + end) * kMaxFcD + j].im;
      }
      gs[(l * 2 + end) * kMaxFcD + k] = {sr, si};
    }
    __syncthreads();
  }

  // ---- epilogue
  double c4[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) c4[r] = a.coef[s0 + r];
  for (int e = lane; e < 2 * n; e += 64) {
    const int it = e & 1, i = e >> 1;
    if (it == 1 && !has1) continue;
    const cx<double> z0 = buf[(2 * it) * LSZ + ph(i)], z1 = buf[(2 * it + 1) * LSZ + ph(i)];
    double dv[4] = {z0.re, z0.im, z1.re, z1.im};
    if (adj) {
      if (i >= n - d) {
        const int k = i - (n - d);
        const cx<double> ga = gs[((2 * it) * 2 + 1) * kMaxFcD + k], gb = gs[((2 * it + 1) * 2 + 1) * kMaxFcD + k];
        dv[0] += ga.re; dv[1] += ga.im; dv[2] += gb.re; dv[3] += gb.im;
      }
      if (i < d) {
        const int k = d - 1 - i;
        const cx<double> ga = gs[((2 * it) * 2 + 0) * kMaxFcD + k], gb = gs[((2 * it + 1) * 2 + 0) * kMaxFcD + k];
        dv[0] += ga.re; dv[1] += ga.im; dv[2] += gb.re; dv[3] += gb.im;
      }
    }
    const int64_t off = base0 + it * a.line_stride + (int64_t)i * a.pt_stride;
    T o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (MODE == LINE_FWD_X) o[r] = T(-c4[r] * dv[r]);
      else if (MODE == LINE_FWD_Y) o[r] = T((double)a.aux[off + r] - c4[r] * dv[r]);
      else if (MODE == LINE_ADJ_X) o[r] = T(dv[r]);
      else o[r] = T((double)a.aux2[off + r] - a.cdt * ((double)a.aux[off + r] + dv[r]));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) a.out[off + r] = o[r];
  }
}

bool fourstep_split(int Np, int* n1, int* n2) {
  switch (Np) {
    case 90: *n1 = 9; *n2 = 10; return true;
    case 160: *n1 = 16; *n2 = 10; return true;
    case 288: *n1 = 16; *n2 = 18; return true;
    case 540: *n1 = 20; *n2 = 27; return true;
    case 1080: *n1 = 30; *n2 = 36; return true;
    default: return false;
  }
}

template <typename T, int MODE, int N1, int N2>
static hipError_t go(const Line4Args<T>& a, dim3 grid, hipStream_t s) {
  const size_t sh = sizeof(cx<double>) * (size_t)(kLP * N1 * (N2 + 1) + 4 * kLP * kMaxFcD);
  hipLaunchKernelGGL((line4_kernel<T, MODE, N1, N2>), grid, dim3(64), sh, s, a);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t by_size(const Line4Args<T>& a, dim3 grid, hipStream_t s) {
  switch (a.fc.Np) {
    case 90: return go<T, MODE, 9, 10>(a, grid, s);
    case 160: return go<T, MODE, 16, 10>(a, grid, s);
    case 288: return go<T, MODE, 16, 18>(a, grid, s);
    case 540: return go<T, MODE, 20, 27>(a, grid, s);
    case 1080: return go<T, MODE, 30, 36>(a, grid, s);
    default: return hipErrorNotSupported;
  }
}

template <typename T>
static hipError_t launch4_t(const Plan& p, const LineLaunch& L, hipStream_t s) {
  Line4Args<T> a;
  a.in = static_cast<const T*>(L.in);
  a.aux = static_cast<const T*>(L.aux);
  a.aux2 = static_cast<const T*>(L.aux2);
  a.out = static_cast<T*>(L.out);
  a.coef = (L.dir == 0) ? p.dev.xi : p.dev.eta;
  a.cdt = L.cdt;
  a.fc = (L.dir == 0) ? p.fcx : p.fcy;
  a.grp_stride = p.ny * p.nx * kGroup;
  a.inst_stride = p.G * a.grp_stride;
  if (L.dir == 0) {
    a.nlines = (int)p.ny;
    a.line_stride = p.nx * kGroup;
    a.pt_stride = kGroup;
  } else {
    a.nlines = (int)p.nx;
    a.line_stride = kGroup;
    a.pt_stride = p.nx * kGroup;
  }
  const int npairs = (a.nlines + 1) / 2;
  dim3 grid((unsigned)(((npairs + 15) / 16) * 16), (unsigned)p.G, (unsigned)p.Nq);
  switch (L.mode) {
    case LINE_FWD_X: return by_size<T, LINE_FWD_X>(a, grid, s);
    case LINE_FWD_Y: return by_size<T, LINE_FWD_Y>(a, grid, s);
    case LINE_ADJ_X: return by_size<T, LINE_ADJ_X>(a, grid, s);
    default: return by_size<T, LINE_ADJ_Y>(a, grid, s);
  }
}

hipError_t launch_line4(const Plan& p, const LineLaunch& L, hipStream_t s) {
  if (p.dtype == RTE_F64) return launch4_t<double>(p, L, s);
  return launch4_t<float>(p, L, s);
}

}  // namespace rte
