// Node passes of the FC-DOM step and its adjoint, plus the small detector,
// misfit and gradient kernels.
//
// Forward node pass (Sec. 4.1-4.2, eq. RTEAB4; Algorithm 1 "right hand side"
// and "impose boundary conditions"): for a tile of nodes with all M ordinates,
//   S    = W u                       HG scattering, a dense M x M contraction
//                                    per node, on FP64/FP32 MFMA 16x16x4
//   L^n  = b S - (a + b) u + X + Y   X = -xi Dx u, Y = -eta Dy u from the line passes
//   u~   = u + c dt (chi0 L^n + chi1 L^{n-1} + chi2 L^{n-2} + chi3 L^{n-3})
//   u^{n+1} = f u~(reflected slot) + q(x_b, t_{n+1}) on incoming boundary
//             entries (eq. RTE, last line), u~ elsewhere
//   flux[w][pos] = sum_m kappa_w(m) u^{n+1}_m on boundary nodes (eq. OpMed)
//
// Adjoint node pass (exact transpose, reverse time): with v^k = P^T ubar^k,
//   ubar^{n+1} = P1^{n+1} - c dt (Dx^T(xi w^{n+1}) + Dy^T(eta w^{n+1}))
//   v^{n+1} = P^T ubar^{n+1}
//   w^n  = sum_l chi_l v^{n+1+l}
//   P1^n = v^{n+1} + c dt (b W w - (a + b) w) + D_e^T Gbar^n
//   dJ/da += -c dt sum_m u^n_m w_m,   dJ/db += c dt sum_m u^n_m ((W w)_m - w_m)
// The line passes of the same step then form the transposed derivatives of w^n.
#include <algorithm>
#include <type_traits>

#include "rte_internal.h"

namespace rte {

constexpr double kChi0 = 55.0 / 24.0, kChi1 = -59.0 / 24.0, kChi2 = 37.0 / 24.0, kChi3 = -9.0 / 24.0;

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Operands of both 16x16x4 variants: lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Result element v of lane l is D[row][l%16] with
// row = l/16 + 4v for FP64 and row = 4(l/16) + v for FP32 (gfx950, measured).
template <>
struct Mfma<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Tiling.  A wave owns a 16-node tile (16 consecutive positions of the
// row-padded layout) and one row tile of 16 output slots (4 ordinate groups);
// lane l holds 4 values of node l % 16 (which 4: see the lane maps below).
// The scattering D[s][node] = sum_s' Wt[s'][s] X[s'][node] is a 16 x 16 x Mpad
// MFMA product per wave: the A operand is the wave's slice of the HG matrix
// (kept in registers), the B operand (X at all slots of the tile) is
// exchanged through LDS among the RT waves that share the tile, and the
// result lands in exactly the (node, slot) registers of the lane that owns
// it.  Boundary coupling only mixes slots of one group (the groups are
// reflection orbits).
// Lane maps.  FP64: lane (node, r) holds slot r of the 4 groups of its row
// tile (the FP64 MFMA returns rows r, r + 4, r + 8, r + 12 to lane r), so
// every access is a 512-byte run of 8-byte lanes and the boundary coupling
// uses wave shuffles among the 4 lanes of a node.  FP32 ("vector lanes"):
// lane (node, r) holds the 4 slots of group r of its row tile (the FP32 MFMA
// returns rows 4r .. 4r + 3 to lane r), so each array is one 16-byte load
// per lane and the boundary coupling stays in the lane's registers.
// NT tiles x RT row tiles per block; RTC = RT at compile time (1..4) or 0
// for RT >= 5 (NT = 1).
struct NodeGeom {
  int nx, ny, nxp, M, Mpad, G, nb, npos, K1, RT, NT, npos_total;
  int q0;                   // first source of the chunk (blockIdx.y is the source within it)
  int ntiles, tile_shift;   // tiles are visited from the one holding the last row's start
  int64_t grp_stride, inst_stride;
};

__device__ __forceinline__ int node_type(int j, int i, int nx, int ny) {
  const int tx = (i == 0) ? 1 : ((i == nx - 1) ? 2 : 0);
  const int ty = (j == 0) ? 1 : ((j == ny - 1) ? 2 : 0);
  return tx + 3 * ty;
}

__device__ __forceinline__ int boundary_pos(int j, int i, int nx, int ny) {
  if (j == 0) return i;
  if (j == ny - 1) return nx + i;
  if (i == 0) return 2 * nx + j - 1;
  return 2 * nx + (ny - 2) + j - 1;
}

template <typename T>
constexpr bool kVecLane = sizeof(T) == 4;

// slot (ordinate storage index) of value v of the lane
template <typename T, typename TL>
__device__ __forceinline__ int lane_slot(const TL& t, int v) {
  return kVecLane<T> ? 4 * (4 * t.rt + t.r) + v : 4 * (4 * t.rt + v) + t.r;
}

struct TileLane {
  int node, r, rt, nt, P, j, i;
  bool valid, bnd;
};

__device__ __forceinline__ TileLane tile_lane(const NodeGeom& G) {
  TileLane t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  t.node = lane & 15;
  t.r = lane >> 4;
  t.rt = wave % G.RT;
  t.nt = wave / G.RT;
  // the first and last rows are all boundary nodes, whose waves take longer:
  // visit the last row first so that it does not trail the grid
  int tile = (int)blockIdx.x * G.NT + t.nt;
  tile = (tile < G.ntiles) ? (tile + G.tile_shift) % G.ntiles : G.ntiles;
  t.P = tile * 16 + t.node;
  t.j = t.P / G.nxp;
  t.i = t.P - t.j * G.nxp;
  t.valid = (t.P < G.npos_total) && (t.i < G.nx);
  t.bnd = t.valid && (t.i == 0 || t.i == G.nx - 1 || t.j == 0 || t.j == G.ny - 1);
  return t;
}

// MFMA product for the wave's row tile: B operand from the LDS tile Bs
// ([Mpad][16] of this tile), A fragments af (preloaded) or read from Wt.
template <typename T, int RTC>
__device__ __forceinline__ typename Mfma<T>::acc_t scatter_tile(const T* Bs, const T* af, const double* __restrict__ Wt,
                                                               const NodeGeom& G, const TileLane& t) {
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc = {0, 0, 0, 0};
  if constexpr (RTC > 0) {
#pragma unroll
    for (int ks = 0; ks < 4 * RTC; ++ks) acc = Mfma<T>::step(af[ks], Bs[(4 * ks + t.r) * 16 + t.node], acc);
  } else {
    const int col = 16 * t.rt + t.node;
    for (int ks = 0; ks < 4 * G.RT; ++ks)
      acc = Mfma<T>::step(T(Wt[(4 * ks + t.r) * G.Mpad + col]), Bs[(4 * ks + t.r) * 16 + t.node], acc);
  }
  return acc;
}

// Element access at a 32-bit byte offset from a per-block base pointer: the
// base stays in scalar registers and one offset register serves every array
// (one instance of a state is below 4 GiB; checked by the plan).  Every
// element is read or written once per launch.  NT (plans whose state arrays
// are far larger than the 256 MiB memory-side cache): the accesses carry the
// non-temporal hint, 5-7 % faster node passes at 513 x 513 x 64; on arrays
// the cache holds between launches (257 x 257 x 32) the hint costs 3-8 %.
template <bool NT, typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t boff) {
  const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
  if constexpr (!NT) {
    return *p;
  } else if constexpr (std::is_same<T, float4>::value) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return __builtin_nontemporal_load(p);
  }
}
template <bool NT, typename T>
__device__ __forceinline__ void sto(T* base, uint32_t boff, T v) {
  T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff);
  if constexpr (!NT) {
    *p = v;
  } else if constexpr (std::is_same<T, float4>::value) {
    const f4v w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f4v*>(p));
  } else {
    __builtin_nontemporal_store(v, p);
  }
}

// The lane's 4 values of one array: per-value offsets off[v] (FP64) or one
// 16-byte vector at off[0] (FP32); ok[v] masks the values.
template <bool NT, typename T>
__device__ __forceinline__ void ld4(const T* base, const uint32_t* off, const bool* ok, T* x) {
  if constexpr (kVecLane<T>) {
    float4 q = {0.f, 0.f, 0.f, 0.f};
    if (ok[0]) q = ldo<NT>(reinterpret_cast<const float4*>(base), off[0]);
    x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = ok[v] ? ldo<NT>(base, off[v]) : T(0);
  }
}
template <bool NT, typename T>
__device__ __forceinline__ void st4(T* base, const uint32_t* off, const bool* ok, const T* x) {
  if constexpr (kVecLane<T>) {
    if (ok[0]) sto<NT>(reinterpret_cast<float4*>(base), off[0], make_float4(x[0], x[1], x[2], x[3]));
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (ok[v]) sto<NT>(base, off[v], x[v]);
  }
}
// Lane offsets and masks of the 4 values.
template <typename T>
__device__ __forceinline__ void lane_offsets(const NodeGeom& G, const TileLane& t, uint32_t* off, bool* ok) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int s = lane_slot<T>(t, v);
    ok[v] = t.valid && (s >> 2) < G.G;
    off[v] = (uint32_t)(((uint32_t)(s >> 2) * (uint32_t)G.grp_stride + (uint32_t)t.P * kGroup + (s & 3)) * sizeof(T));
  }
}
// Byte offset of the value at the reversed ordinate of the lane's value v
// (same node): the paired forward state of the continuous adjoint.
template <typename T>
__device__ __forceinline__ uint32_t pair_offset(const NodeGeom& G, const TileLane& t, const int32_t* slot_rev, int v) {
  const int sr = slot_rev[lane_slot<T>(t, v)];
  return (uint32_t)(((uint32_t)(sr >> 2) * (uint32_t)G.grp_stride + (uint32_t)t.P * kGroup + (sr & 3)) * sizeof(T));
}
// Value of slot c (0..3) of the group that holds the lane's value v, for the
// same node: another lane's register (FP64) or one of the lane's own (FP32).
template <typename T>
__device__ __forceinline__ T group_peer(const T* x, int v, int c, const TileLane& t) {
  if constexpr (kVecLane<T>) {
    return c == 0 ? x[0] : (c == 1 ? x[1] : (c == 2 ? x[2] : x[3]));
  } else {
    return __shfl(x[v], t.node + 16 * c);
  }
}

template <typename T, int RTC>
__device__ __forceinline__ void load_afrag(T* af, const double* __restrict__ Wt, const NodeGeom& G, const TileLane& t) {
  if constexpr (RTC > 0) {
    const int col = 16 * t.rt + t.node;
#pragma unroll
    for (int ks = 0; ks < 4 * RTC; ++ks) af[ks] = T(Wt[(4 * ks + t.r) * G.Mpad + col]);
  }
}

// ---------------------------------------------------------------- forward
template <typename T>
struct NodeFwdArgs {
  const T* u; const T* X; const T* Y; const T* L1; const T* L2; const T* L3;
  const T* mu_a; const T* mu_s;
  T* u_out; T* L_out; double* flux;
  const double* Wt; const BcRule* bc; const double* kappa;
  const double* beam_sp; const double* beam_an; const double* beam_tt; const int32_t* beam_off;
  // continuous adjoint (CADJ): inflow source table, paired forward state,
  // reversed-ordinate slots, gradient maps, quadrature dtheta dx dy dt
  const double* csrc; const T* upair; const int32_t* slot_rev; double* ga; double* gb;
  double quad;
  // extended forward (EXT): separable source and inflow tables, ordinate of each slot
  rte_separable vsrc, inflow;
  const int32_t* slot_m;
  NodeGeom geo;
  int step;
  double cdt;
};

// L_out may alias L3: each element is read and then written by one lane.
// CADJ: the same step applied to psi (the adjoint of eq. AdjointProblem in
// reversed time and ordinates, which satisfies the forward equation): the
// inflow source is (1 - f) csrc instead of the beams, and the lane adds the
// eq. (FDwin22) terms of its input psi paired with upair (u at the same
// physical time, ordinate theta + pi) to the gradient maps:
//   ga -= quad sum psi u~,  gb += quad sum ((W psi) - psi) u~.
// MODE 0: the beam problem; MODE 1: CADJ (above); MODE 2: EXT, the
// extended forward: q = sum_k X_k Y_k Th_k is added to L^n, and on inflow
// entries the separable data replace the beams (when inflow.rank > 0).
// Time level n of the tables is row n + 3 (the start-up passes use n < 0).
__device__ __forceinline__ double sep_value(const rte_separable& f, int row, int K4, int i, int j, int nx, int ny,
                                            int M, int m) {
  double acc = 0.0;
  for (int k = 0; k < f.rank; ++k)
    acc += f.X[((int64_t)k * K4 + row) * nx + i] * f.Y[((int64_t)k * K4 + row) * ny + j] * f.Th[(int64_t)k * M + m];
  return acc;
}

template <typename T, int RTC, int MODE, bool NT>
__global__ __launch_bounds__(RTC == 0 ? 1024 : 512) void node_fwd_kernel(NodeFwdArgs<T> a) {
  constexpr bool CADJ = MODE == 1;
  constexpr bool EXT = MODE == 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const NodeGeom& G = a.geo;
  const TileLane t = tile_lane(G);
  T* Bs = reinterpret_cast<T*>(smem_raw) + (size_t)t.nt * G.Mpad * 16;
  double* Fx = reinterpret_cast<double*>(smem_raw + ((sizeof(T) * (size_t)G.NT * G.Mpad * 16 + 15) & ~size_t(15)));
  const int q = G.q0 + (int)blockIdx.y;   // source (beams, detector flux)
  const int64_t ib = (int64_t)blockIdx.y * G.inst_stride;

  const T* uq = a.u + ib;
  const T* Xq = a.X + ib;
  const T* Yq = a.Y + ib;
  const T* L1q = a.L1 + ib;
  const T* L2q = a.L2 + ib;
  const T* L3q = a.L3 + ib;
  T* uoq = a.u_out + ib;
  T* Loq = a.L_out + ib;
  T u[4], X[4], Y[4], L1[4], L2[4], L3[4], up[4];
  uint32_t off[4];
  bool gv[4];
  lane_offsets<T>(G, t, off, gv);
  if constexpr (kVecLane<T>) {
    ld4<NT>(uq, off, gv, u);
    ld4<NT>(Xq, off, gv, X);
    ld4<NT>(Yq, off, gv, Y);
    ld4<NT>(L1q, off, gv, L1);
    ld4<NT>(L2q, off, gv, L2);
    ld4<NT>(L3q, off, gv, L3);
  } else {
    // value by value, all arrays of one value together (this issue order
    // streams measurably faster than array by array)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      u[v] = X[v] = Y[v] = L1[v] = L2[v] = L3[v] = up[v] = T(0);
      if (gv[v]) {
        u[v] = ldo<NT>(uq, off[v]); X[v] = ldo<NT>(Xq, off[v]); Y[v] = ldo<NT>(Yq, off[v]);
        L1[v] = ldo<NT>(L1q, off[v]); L2[v] = ldo<NT>(L2q, off[v]); L3[v] = ldo<NT>(L3q, off[v]);
        if constexpr (CADJ) up[v] = ldo<NT>(a.upair + ib, pair_offset<T>(G, t, a.slot_rev, v));
      }
    }
  }
  if constexpr (kVecLane<T>) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      up[v] = T(0);
      if constexpr (CADJ) {
        if (gv[v]) up[v] = ldo<NT>(a.upair + ib, pair_offset<T>(G, t, a.slot_rev, v));
      }
    }
  }
  const int gn = t.j * G.nx + t.i;
  const T A = t.valid ? a.mu_a[gn] : T(0), B = t.valid ? a.mu_s[gn] : T(0);
  T af[RTC > 0 ? 4 * RTC : 1];
  load_afrag<T, RTC>(af, a.Wt, G, t);

#pragma unroll
  for (int v = 0; v < 4; ++v) Bs[lane_slot<T>(t, v) * 16 + t.node] = u[v];
  __syncthreads();
  const typename Mfma<T>::acc_t S = scatter_tile<T, RTC>(Bs, af, a.Wt, G, t);

  // L^n (plus the volumetric source) and the AB4 combination
  const T cdt = T(a.cdt);
  T qv[4] = {T(0), T(0), T(0), T(0)};
  if constexpr (EXT) {
    if (a.vsrc.rank > 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (gv[v])
          qv[v] = T(sep_value(a.vsrc, a.step + 3, G.K1 + 3, t.i, t.j, G.nx, G.ny, G.M, a.slot_m[lane_slot<T>(t, v)]));
    }
  }
  T un[4], Ln[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Ln[v] = B * S[v] - (A + B) * u[v] + X[v] + Y[v];
    if constexpr (EXT) Ln[v] += qv[v];
    un[v] = u[v] + cdt * (T(kChi0) * Ln[v] + T(kChi1) * L1[v] + T(kChi2) * L2[v] + T(kChi3) * L3[v]);
    if constexpr (!kVecLane<T>) {
      if (gv[v]) sto<NT>(Loq, off[v], Ln[v]);
    }
  }
  if constexpr (kVecLane<T>) st4<NT>(Loq, off, gv, Ln);

  // inflow condition with Fresnel reflection and the beams at t_{n+1}.  The
  // boundary tables (reflection rules, beam factors, detector weights) of the
  // lane's 4 slots are all requested at once: one memory round trip.
  const bool wave_bnd = __ballot(t.bnd) != 0;
  const int wl0 = !t.bnd ? -1 : ((t.i == 0) ? 0 : ((t.i == G.nx - 1) ? 1 : -1));
  const int wl1 = !t.bnd ? -1 : ((t.j == 0) ? 2 : ((t.j == G.ny - 1) ? 3 : -1));
  double pw0 = 0.0, pw1 = 0.0;
  if (wave_bnd) {
    const int ty = t.bnd ? node_type(t.j, t.i, G.nx, G.ny) : 0;
    const int bp = t.bnd ? boundary_pos(t.j, t.i, G.nx, G.ny) : 0;
    BcRule br[4];
    T src[4];
    double k0[4], k1[4];
    const int b0 = a.beam_off[q], b1 = a.beam_off[q + 1];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = lane_slot<T>(t, v);
      const bool on = t.bnd && gv[v];
      br[v].flag = 0; br[v].src_a = s; br[v].src_b = s; br[v].pad = 0; br[v].coef_a = 0.0; br[v].coef_b = 0.0;
      if (on) br[v] = a.bc[ty * G.M + s];
      src[v] = T(0);
      if constexpr (CADJ) {
        if (on)
          src[v] = T((1.0 - br[v].coef_a - br[v].coef_b) *
                     a.csrc[((int64_t)q * G.K1 + a.step + 1) * 4 * G.npos + bp]);
      } else if (EXT && a.inflow.rank > 0) {
        if (on && br[v].flag)
          src[v] = T(sep_value(a.inflow, a.step + 4, G.K1 + 3, t.i, t.j, G.nx, G.ny, G.M, a.slot_m[s]));
      } else {
        if (on && a.step >= 0)
          for (int b = b0; b < b1; ++b)
            src[v] += T(a.beam_sp[(int64_t)b * G.nb + bp] * a.beam_an[b * G.M + s]) * T(a.beam_tt[(int64_t)b * G.K1 + a.step + 1]);
      }
      k0[v] = (on && a.flux && wl0 >= 0) ? a.kappa[wl0 * G.M + s] : 0.0;
      k1[v] = (on && a.flux && wl1 >= 0) ? a.kappa[wl1 * G.M + s] : 0.0;
    }
    const T uc[4] = {un[0], un[1], un[2], un[3]};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T ta = group_peer(uc, v, br[v].src_a & 3, t);
      const T tb = group_peer(uc, v, br[v].src_b & 3, t);
      if (br[v].flag) un[v] = T(br[v].coef_a) * ta + T(br[v].coef_b) * tb + src[v];
    }
    // detector flux on boundary nodes (FP64): lane partial over its 4
    // groups, then over the 4 slot lanes of the node, then over the row tiles
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      pw0 += k0[v] * (double)un[v];
      pw1 += k1[v] * (double)un[v];
    }
    pw0 += __shfl_xor(pw0, 16);
    pw1 += __shfl_xor(pw1, 16);
    pw0 += __shfl_xor(pw0, 32);
    pw1 += __shfl_xor(pw1, 32);
  }
  st4<NT>(uoq, off, gv, un);

  if constexpr (CADJ) {
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      pa += (double)u[v] * (double)up[v];
      pb += ((double)S[v] - (double)u[v]) * (double)up[v];
    }
    pa += __shfl_xor(pa, 16);
    pb += __shfl_xor(pb, 16);
    pa += __shfl_xor(pa, 32);
    pb += __shfl_xor(pb, 32);
    if (G.RT > 1) {
      if (t.r == 0) {
        Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 0] = pa;
        Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 1] = pb;
      }
      __syncthreads();
      if (t.rt != 0 || t.r != 0 || !t.valid) return;
      pa = pb = 0.0;
      for (int k = 0; k < G.RT; ++k) {
        pa += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 0];
        pb += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 1];
      }
    } else if (t.r != 0 || !t.valid) {
      return;
    }
    const int64_t Nn = (int64_t)G.nx * G.ny;
    a.ga[(int64_t)q * Nn + gn] -= a.quad * pa;
    a.gb[(int64_t)q * Nn + gn] += a.quad * pb;
    return;
  }
  if (a.flux == nullptr) return;

  if (G.RT > 1) {
    if (t.r == 0) {
      Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 0] = pw0;
      Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 1] = pw1;
    }
    __syncthreads();
    if (t.rt != 0 || !t.bnd || t.r != 0) return;
    pw0 = pw1 = 0.0;
    for (int k = 0; k < G.RT; ++k) {
      pw0 += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 0];
      pw1 += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 1];
    }
  } else if (!t.bnd || t.r != 0) {
    return;
  }
  const int64_t fb = ((int64_t)q * G.K1 + a.step + 1) * 4;
  if (wl0 >= 0) a.flux[(fb + wl0) * G.npos + t.j] = pw0;
  if (wl1 >= 0) a.flux[(fb + wl1) * G.npos + t.i] = pw1;
}

// ---------------------------------------------------------------- adjoint
template <typename T>
struct NodeAdjArgs {
  const T* atx; const T* aty; T* ap1; T* v1_out;
  const T* v2; const T* v3; const T* v4; const T* u;
  const T* mu_a; const T* mu_s; const double* inj;
  T* w_out; double* ga; double* gb;
  const double* Wt; const BcRuleT* bct; const double* kappa;
  NodeGeom geo;
  int step;
  double cdt;
};

// ap1 is read (P1^{n+1}) and overwritten (P1^n) element by element by one lane.
template <typename T, int RTC, bool NT>
__global__ __launch_bounds__(RTC == 0 ? 1024 : 512) void node_adj_kernel(NodeAdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const NodeGeom& G = a.geo;
  const TileLane t = tile_lane(G);
  T* Bs = reinterpret_cast<T*>(smem_raw) + (size_t)t.nt * G.Mpad * 16;
  double* Fx = reinterpret_cast<double*>(smem_raw + ((sizeof(T) * (size_t)G.NT * G.Mpad * 16 + 15) & ~size_t(15)));
  const int q = G.q0 + (int)blockIdx.y;   // source (injection, gradient maps)
  const int64_t ib = (int64_t)blockIdx.y * G.inst_stride;
  const int Nn = G.nx * G.ny;

  const T* txq = a.atx + ib;
  const T* tyq = a.aty + ib;
  T* p1q = a.ap1 + ib;
  const T* v2q = a.v2 + ib;
  const T* v3q = a.v3 + ib;
  const T* v4q = a.v4 + ib;
  const T* uq = a.u + ib;
  T* wq = a.w_out + ib;
  T* v1q = a.v1_out + ib;
  T tx[4], ty[4], p1[4], v2[4], v3[4], v4[4], uu[4];
  uint32_t off[4];
  bool gv[4];
  lane_offsets<T>(G, t, off, gv);
  if constexpr (kVecLane<T>) {
    ld4<NT>(txq, off, gv, tx);
    ld4<NT>(tyq, off, gv, ty);
    ld4<NT>(static_cast<const T*>(p1q), off, gv, p1);
    ld4<NT>(v2q, off, gv, v2);
    ld4<NT>(v3q, off, gv, v3);
    ld4<NT>(v4q, off, gv, v4);
    ld4<NT>(uq, off, gv, uu);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      tx[v] = ty[v] = p1[v] = v2[v] = v3[v] = v4[v] = uu[v] = T(0);
      if (gv[v]) {
        tx[v] = ldo<NT>(txq, off[v]); ty[v] = ldo<NT>(tyq, off[v]); p1[v] = ldo<NT>(p1q, off[v]);
        v2[v] = ldo<NT>(v2q, off[v]); v3[v] = ldo<NT>(v3q, off[v]); v4[v] = ldo<NT>(v4q, off[v]);
        uu[v] = ldo<NT>(uq, off[v]);
      }
    }
  }
  const int gn = t.j * G.nx + t.i;
  const T A = t.valid ? a.mu_a[gn] : T(0), B = t.valid ? a.mu_s[gn] : T(0);
  T af[RTC > 0 ? 4 * RTC : 1];
  load_afrag<T, RTC>(af, a.Wt, G, t);
  // the node's gradient-map entries, read with the state by the one lane
  // per node that updates them at the end (no load round trip after the
  // reduction); each (source, node) belongs to one block of the launch
  const bool gw = t.rt == 0 && t.r == 0 && t.valid;
  double ga0 = 0.0, gb0 = 0.0;
  if (gw) {
    ga0 = a.ga[(int64_t)q * Nn + gn];
    gb0 = a.gb[(int64_t)q * Nn + gn];
  }

  // ubar^{n+1}, then v^{n+1} = P^T ubar^{n+1} on boundary nodes
  const double cdt = a.cdt;
  T v1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) v1[v] = T((double)p1[v] - cdt * ((double)tx[v] + (double)ty[v]));
  // boundary tables of the lane's 4 slots (transposed rules, detector
  // injection) requested at once
  const bool wave_bnd = __ballot(t.bnd) != 0;
  T injv[4] = {T(0), T(0), T(0), T(0)};
  if (wave_bnd) {
    const int tyn = t.bnd ? node_type(t.j, t.i, G.nx, G.ny) : 0;
    const int64_t ib4 = ((int64_t)q * G.K1 + a.step) * 4;
    const double g0 = (t.bnd && t.i == 0) ? a.inj[(ib4 + 0) * G.npos + t.j] : 0.0;
    const double g1 = (t.bnd && t.i == G.nx - 1) ? a.inj[(ib4 + 1) * G.npos + t.j] : 0.0;
    const double g2 = (t.bnd && t.j == 0) ? a.inj[(ib4 + 2) * G.npos + t.i] : 0.0;
    const double g3 = (t.bnd && t.j == G.ny - 1) ? a.inj[(ib4 + 3) * G.npos + t.i] : 0.0;
    BcRuleT rt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = lane_slot<T>(t, v);
      const bool on = t.bnd && gv[v];
      rt[v].is_target = 0; rt[v].ntgt = 0; rt[v].tgt[0] = s; rt[v].tgt[1] = s; rt[v].coef[0] = 0.0; rt[v].coef[1] = 0.0;
      if (on) rt[v] = a.bct[tyn * G.M + s];
      // detector misfit enters through the outgoing boundary entries
      if (on) {
        T p = T(0);
        if (t.i == 0) p += T(a.kappa[0 * G.M + s] * g0);
        if (t.i == G.nx - 1) p += T(a.kappa[1 * G.M + s] * g1);
        if (t.j == 0) p += T(a.kappa[2 * G.M + s] * g2);
        if (t.j == G.ny - 1) p += T(a.kappa[3 * G.M + s] * g3);
        injv[v] = p;
      }
    }
    const T vc[4] = {v1[0], v1[1], v1[2], v1[3]};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T t0 = group_peer(vc, v, rt[v].tgt[0] & 3, t);
      const T t1 = group_peer(vc, v, rt[v].tgt[1] & 3, t);
      if (t.bnd && gv[v]) {
        T val = rt[v].is_target ? T(0) : v1[v];
        if (rt[v].ntgt > 0) val += T(rt[v].coef[0]) * t0;
        if (rt[v].ntgt > 1) val += T(rt[v].coef[1]) * t1;
        v1[v] = val;
      }
    }
  }

  // w^n, and W w on the MFMA
  T w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    w[v] = T(kChi0) * v1[v] + T(kChi1) * v2[v] + T(kChi2) * v3[v] + T(kChi3) * v4[v];
    Bs[lane_slot<T>(t, v) * 16 + t.node] = w[v];
  }
  __syncthreads();
  const typename Mfma<T>::acc_t S = scatter_tile<T, RTC>(Bs, af, a.Wt, G, t);

  // P1^n, stores and the gradient products
  const T cdtT = T(cdt);
  double pa = 0.0, pb = 0.0;
  T pn[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    pn[v] = v1[v] + cdtT * (B * S[v] - (A + B) * w[v]) + injv[v];
    if constexpr (!kVecLane<T>) {
      if (gv[v]) {
        sto<NT>(p1q, off[v], pn[v]);
        sto<NT>(wq, off[v], w[v]);
        sto<NT>(v1q, off[v], v1[v]);
      }
    }
    pa += (double)uu[v] * (double)w[v];
    pb += (double)uu[v] * ((double)S[v] - (double)w[v]);
  }
  if constexpr (kVecLane<T>) {
    st4<NT>(p1q, off, gv, pn);
    st4<NT>(wq, off, gv, w);
    st4<NT>(v1q, off, gv, v1);
  }
  pa += __shfl_xor(pa, 16);
  pb += __shfl_xor(pb, 16);
  pa += __shfl_xor(pa, 32);
  pb += __shfl_xor(pb, 32);
  if (G.RT > 1) {
    if (t.r == 0) {
      Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 0] = pa;
      Fx[((t.nt * G.RT + t.rt) * 16 + t.node) * 2 + 1] = pb;
    }
    __syncthreads();
    if (t.rt != 0 || t.r != 0 || !t.valid) return;
    pa = pb = 0.0;
    for (int k = 0; k < G.RT; ++k) {
      pa += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 0];
      pb += Fx[((t.nt * G.RT + k) * 16 + t.node) * 2 + 1];
    }
  } else if (t.r != 0 || !t.valid) {
    return;
  }
  a.ga[(int64_t)q * Nn + gn] = ga0 - cdt * pa;
  a.gb[(int64_t)q * Nn + gn] = gb0 + cdt * pb;
}

// ---------------------------------------------------------------- launchers
static NodeGeom make_geom(const Plan& p) {
  NodeGeom g;
  g.nx = (int)p.nx; g.ny = (int)p.ny; g.nxp = (int)p.nxp;
  g.M = (int)p.M; g.Mpad = (int)p.Mpad; g.G = (int)p.G;
  g.nb = (int)p.nb; g.npos = (int)p.npos; g.K1 = (int)(p.K + 1);
  g.RT = (int)(p.Mpad / 16);
  g.NT = p.sched.node_tiles_per_block;
  g.npos_total = (int)(p.ny * p.nxp);
  g.q0 = (int)p.cq0;
  g.ntiles = (g.npos_total + 15) / 16;
  g.tile_shift = (int)((p.ny - 1) * p.nxp / 16);
  g.grp_stride = p.grp_stride;
  g.inst_stride = p.inst_stride;
  return g;
}

bool node_tiles_ok(const Plan& p, int nt) {
  const int rt = (int)(p.Mpad / 16);
  if (rt > 4) return nt == 1;
  return (nt == 1 || nt == 2 || nt == 4) && nt * rt <= 8;
}

int node_tiles_default(const Plan& p) {
  const int rt = (int)(p.Mpad / 16);
  return (rt <= 4 && 4 % rt == 0) ? 4 / rt : 1;
}

static size_t node_shmem(const NodeGeom& g, size_t es) {
  return ((es * (size_t)g.NT * g.Mpad * 16 + 15) & ~size_t(15)) + sizeof(double) * 2 * (size_t)g.NT * g.RT * 16;
}

static dim3 node_grid(const Plan& p, const NodeGeom& g) {
  const int tiles = (g.npos_total + 15) / 16;
  return dim3((unsigned)((tiles + g.NT - 1) / g.NT), (unsigned)p.cnq);
}

template <typename T, int MODE, bool NT>
static void launch_node_fwd_rt(const NodeFwdArgs<T>& a, dim3 grid, dim3 block, size_t sh, hipStream_t s) {
  switch (a.geo.RT) {
    case 1: hipLaunchKernelGGL((node_fwd_kernel<T, 1, MODE, NT>), grid, block, sh, s, a); break;
    case 2: hipLaunchKernelGGL((node_fwd_kernel<T, 2, MODE, NT>), grid, block, sh, s, a); break;
    case 3: hipLaunchKernelGGL((node_fwd_kernel<T, 3, MODE, NT>), grid, block, sh, s, a); break;
    case 4: hipLaunchKernelGGL((node_fwd_kernel<T, 4, MODE, NT>), grid, block, sh, s, a); break;
    default: hipLaunchKernelGGL((node_fwd_kernel<T, 0, MODE, NT>), grid, block, sh, s, a); break;
  }
}

template <typename T, bool NT>
static void launch_node_fwd_nt(int mode, const NodeFwdArgs<T>& a, dim3 grid, dim3 block, size_t sh, hipStream_t s) {
  if (mode == 1) launch_node_fwd_rt<T, 1, NT>(a, grid, block, sh, s);
  else if (mode == 2) launch_node_fwd_rt<T, 2, NT>(a, grid, block, sh, s);
  else launch_node_fwd_rt<T, 0, NT>(a, grid, block, sh, s);
}

template <typename T>
static hipError_t launch_node_fwd_mode(int mode, bool nt, const NodeFwdArgs<T>& a, dim3 grid, dim3 block, size_t sh,
                                       hipStream_t s) {
  if (nt) launch_node_fwd_nt<T, true>(mode, a, grid, block, sh, s);
  else launch_node_fwd_nt<T, false>(mode, a, grid, block, sh, s);
  return hipGetLastError();
}

template <typename T>
static hipError_t node_fwd_t(const Plan& p, const NodeFwdLaunch& L, hipStream_t s) {
  NodeFwdArgs<T> a;
  a.u = (const T*)L.u; a.X = (const T*)L.X; a.Y = (const T*)L.Y;
  a.L1 = (const T*)L.L1; a.L2 = (const T*)L.L2; a.L3 = (const T*)L.L3;
  a.mu_a = (const T*)L.mu_a; a.mu_s = (const T*)L.mu_s;
  a.u_out = (T*)L.u_out; a.L_out = (T*)L.L_out; a.flux = L.flux;
  a.Wt = p.dev.Wt; a.bc = p.dev.bc; a.kappa = p.dev.kappa;
  a.beam_sp = p.dev.beam_sp; a.beam_an = p.dev.beam_an; a.beam_tt = p.dev.beam_tt; a.beam_off = p.dev.beam_off;
  a.csrc = L.csrc; a.upair = (const T*)L.upair; a.slot_rev = p.dev.slot_rev; a.ga = L.ga; a.gb = L.gb;
  a.vsrc = L.vsrc ? *L.vsrc : rte_separable{0, 0, nullptr, nullptr, nullptr};
  a.inflow = L.inflow ? *L.inflow : rte_separable{0, 0, nullptr, nullptr, nullptr};
  a.slot_m = p.dev.slot_m;
  a.geo = make_geom(p);
  a.step = L.step;
  a.cdt = p.prob.c * p.prob.dt;
  a.quad = (2.0 * 3.14159265358979323846 / (double)p.M) * ((p.prob.xmax - p.prob.xmin) / (double)p.prob.Nx) *
           ((p.prob.ymax - p.prob.ymin) / (double)p.prob.Ny) * p.prob.dt;
  const dim3 grid = node_grid(p, a.geo), block((unsigned)(64 * a.geo.NT * a.geo.RT));
  const size_t sh = node_shmem(a.geo, sizeof(T));
  if (L.csrc && (!L.upair || !L.ga || !L.gb || L.flux || L.vsrc || L.inflow)) return hipErrorInvalidValue;
  const int mode = L.csrc ? 1 : ((L.vsrc || L.inflow) ? 2 : 0);
  if (mode == 2 && (L.step < -3 || L.step >= p.K)) return hipErrorInvalidValue;
  return launch_node_fwd_mode<T>(mode, p.stream_nt, a, grid, block, sh, s);
}

hipError_t launch_node_fwd(const Plan& p, const NodeFwdLaunch& L, hipStream_t s) {
  return p.dtype == RTE_F64 ? node_fwd_t<double>(p, L, s) : node_fwd_t<float>(p, L, s);
}

template <typename T, bool NT>
static void launch_node_adj_rt(const NodeAdjArgs<T>& a, dim3 grid, dim3 block, size_t sh, hipStream_t s) {
  switch (a.geo.RT) {
    case 1: hipLaunchKernelGGL((node_adj_kernel<T, 1, NT>), grid, block, sh, s, a); break;
    case 2: hipLaunchKernelGGL((node_adj_kernel<T, 2, NT>), grid, block, sh, s, a); break;
    case 3: hipLaunchKernelGGL((node_adj_kernel<T, 3, NT>), grid, block, sh, s, a); break;
    case 4: hipLaunchKernelGGL((node_adj_kernel<T, 4, NT>), grid, block, sh, s, a); break;
    default: hipLaunchKernelGGL((node_adj_kernel<T, 0, NT>), grid, block, sh, s, a); break;
  }
}

template <typename T>
static hipError_t node_adj_t(const Plan& p, const NodeAdjLaunch& L, hipStream_t s) {
  NodeAdjArgs<T> a;
  a.atx = (const T*)L.atx; a.aty = (const T*)L.aty; a.ap1 = (T*)L.ap1; a.v1_out = (T*)L.v1_out;
  a.v2 = (const T*)L.v2; a.v3 = (const T*)L.v3; a.v4 = (const T*)L.v4; a.u = (const T*)L.u;
  a.mu_a = (const T*)L.mu_a; a.mu_s = (const T*)L.mu_s; a.inj = L.inj;
  a.w_out = (T*)L.w_out; a.ga = L.ga; a.gb = L.gb;
  a.Wt = p.dev.Wt; a.bct = p.dev.bct; a.kappa = p.dev.kappa;
  a.geo = make_geom(p);
  a.step = L.step;
  a.cdt = p.prob.c * p.prob.dt;
  const dim3 grid = node_grid(p, a.geo), block((unsigned)(64 * a.geo.NT * a.geo.RT));
  const size_t sh = node_shmem(a.geo, sizeof(T));
  if (p.stream_nt) launch_node_adj_rt<T, true>(a, grid, block, sh, s);
  else launch_node_adj_rt<T, false>(a, grid, block, sh, s);
  return hipGetLastError();
}

hipError_t launch_node_adj(const Plan& p, const NodeAdjLaunch& L, hipStream_t s) {
  return p.dtype == RTE_F64 ? node_adj_t<double>(p, L, s) : node_adj_t<float>(p, L, s);
}

// G[q][jd][k] = sum_{w,pos} det_w[jd][w][pos] flux[q][k+1][w][pos]
__global__ void detect_kernel(const double* __restrict__ flux, const double* __restrict__ dw, double* __restrict__ G,
                              int q0, int Nq, int Nd, int K, int npos) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Nq * Nd * K;
  if (t0 >= total) return;
  const int64_t t = t0 + (int64_t)q0 * Nd * K;
  const int k = (int)(t % K);
  const int jd = (int)((t / K) % Nd);
  const int q = (int)(t / ((int64_t)K * Nd));
  const double* f = flux + ((int64_t)q * (K + 1) + k + 1) * 4 * npos;
  const double* w = dw + (int64_t)jd * 4 * npos;
  double acc = 0.0;
  for (int x = 0; x < 4 * npos; ++x) acc += w[x] * f[x];
  G[t] = acc;
}

// inj[q][n][w][pos] = sum_jd det_w[jd][w][pos] Gbar[q][jd][n-1], n = 1..K
__global__ void inject_kernel(const double* __restrict__ Gbar, const double* __restrict__ dw, double* __restrict__ inj,
                              int q0, int Nq, int Nd, int K, int npos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)K * 4 * npos;
  if (t >= (int64_t)Nq * per) return;
  const int q = q0 + (int)(t / per);
  const int64_t r = t % per;
  const int n = 1 + (int)(r / (4 * npos));
  const int x = (int)(r % (4 * npos));
  double acc = 0.0;
  for (int jd = 0; jd < Nd; ++jd) acc += dw[(int64_t)jd * 4 * npos + x] * Gbar[((int64_t)q * Nd + jd) * K + n - 1];
  inj[((int64_t)q * (K + 1) + n) * 4 * npos + x] = acc;
}

// Gbar = dt (G - Gm); J (+)= 1/2 dt sum (G - Gm)^2 over n entries (one block,
// fixed reduction order; accumulate adds to J, for the chunks after the first)
__global__ __launch_bounds__(1024) void misfit_kernel(const double* __restrict__ G, const double* __restrict__ Gm,
                                                      double* __restrict__ Gbar, double* __restrict__ J, int64_t n,
                                                      double dt, int accumulate) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 1024) {
    const double r = G[t] - Gm[t];
    Gbar[t] = dt * r;
    acc += r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = (accumulate ? *J : 0.0) + 0.5 * dt * red[0];
}

// src[q][k][bp] = sum_jd det_sp[jd][bp] r(q, jd, K - k), k = 0..K, with
// r(q, jd, n) = G[q][jd][n-1] - Gm[q][jd][n-1] for n >= 1 and r(., ., 0) = 0
__global__ void cadj_source_kernel(const double* __restrict__ G, const double* __restrict__ Gm,
                                   const double* __restrict__ sp, double* __restrict__ src, int q0, int Nq, int Nd,
                                   int K, int nb, int rowlen) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)(K + 1) * nb;
  if (t >= (int64_t)Nq * per) return;
  const int q = q0 + (int)(t / per);
  const int64_t r = t % per;
  const int k = (int)(r / nb);
  const int bp = (int)(r % nb);
  const int n = K - k;
  double acc = 0.0;
  if (n >= 1)
    for (int jd = 0; jd < Nd; ++jd) {
      const int64_t gi = ((int64_t)q * Nd + jd) * K + n - 1;
      acc += sp[(int64_t)jd * nb + bp] * (G[gi] - Gm[gi]);
    }
  src[((int64_t)q * (K + 1) + k) * rowlen + bp] = acc;
}

__global__ void grad_reduce_kernel(const double* __restrict__ ga, const double* __restrict__ gb, double* __restrict__ da,
                                   double* __restrict__ db, int Nq, int64_t Nn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Nn) return;
  double sa = 0.0, sb = 0.0;
  for (int q = 0; q < Nq; ++q) {
    sa += ga[(int64_t)q * Nn + t];
    sb += gb[(int64_t)q * Nn + t];
  }
  da[t] = sa;
  db[t] = sb;
}

template <typename T>
__global__ void unpermute_kernel(const T* __restrict__ st, T* __restrict__ out, const int32_t* __restrict__ slot_m,
                                 int M, int nx, int nxp, int64_t Nn, int Nq, int64_t grp_stride, int64_t inst_stride) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Nq * Nn * M;
  if (t >= total) return;
  const int s = (int)(t % M);
  const int64_t gn = (t / M) % Nn;
  const int q = (int)(t / (M * Nn));
  const int g = s / kGroup, r = s % kGroup;
  const int64_t j = gn / nx, i = gn - j * nx;
  const T v = st[(int64_t)q * inst_stride + (int64_t)g * grp_stride + (j * nxp + i) * kGroup + r];
  out[((int64_t)q * Nn + gn) * M + slot_m[s]] = v;
}

template <typename T>
__global__ void permute_kernel(const T* __restrict__ in, T* __restrict__ st, const int32_t* __restrict__ slot_m, int M,
                               int nx, int nxp, int64_t Nn, int Nq, int64_t grp_stride, int64_t inst_stride) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Nq * Nn * M;
  if (t >= total) return;
  const int s = (int)(t % M);
  const int64_t gn = (t / M) % Nn;
  const int q = (int)(t / (M * Nn));
  const int g = s / kGroup, r = s % kGroup;
  const int64_t j = gn / nx, i = gn - j * nx;
  st[(int64_t)q * inst_stride + (int64_t)g * grp_stride + (j * nxp + i) * kGroup + r] = in[((int64_t)q * Nn + gn) * M + slot_m[s]];
}

// Scalar flux of a state, eq. (photondensity) with the trapezoid rule on the
// uniform ordinates: phi[q][j][i] = dtheta sum_s u[q][s][j][i] over the M
// live slots (the sum does not depend on the slot order), accumulated in
// FP64 in slot order.  Grid: x over nodes of a row, y over rows, z over the
// chunk's sources.
template <typename T>
__global__ void flux_map_kernel(const T* __restrict__ st, double* __restrict__ out, int M, int nx, int nxp,
                                int64_t grp_stride, int64_t inst_stride, int64_t out_q_stride, double dth) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= nx) return;
  const int j = (int)blockIdx.y, q = (int)blockIdx.z;
  const T* p = st + (int64_t)q * inst_stride + ((int64_t)j * nxp + i) * kGroup;
  double acc = 0.0;
  for (int s = 0; s < M; ++s) acc += (double)p[(int64_t)(s / kGroup) * grp_stride + s % kGroup];
  out[(int64_t)q * out_q_stride + (int64_t)j * nx + i] = dth * acc;
}

// Non-finite scan: every lane that meets a NaN or an infinity stores 1 (all
// writers store the same value, so no atomics are needed).
__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n, unsigned long long* __restrict__ flag) {
  bool bad = false;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[t]);
  if (bad) flag[0] = 1ull;
}

hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(nonfinite_kernel, dim3(blocks), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

// Zero fill and device copy as kernels (8-byte words): graph captures of the
// step sequence then hold only kernel nodes.
__global__ void fill_zero_kernel(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) p[t] = 0ull;
}
__global__ void copy_words_kernel(unsigned long long* __restrict__ d, const unsigned long long* __restrict__ s, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) d[t] = s[t];
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 8;
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (unsigned long long*)p, n);
  return hipGetLastError();
}

hipError_t launch_copy(void* d, const void* src, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 8;
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(copy_words_kernel, dim3(blocks), dim3(256), 0, s, (unsigned long long*)d,
                     (const unsigned long long*)src, n);
  return hipGetLastError();
}

// detect, inject and misfit work on the sources of the current chunk
hipError_t launch_detect(const Plan& p, const double* flux, double* G, int K, hipStream_t s) {
  const int64_t total = p.cnq * p.Nd * K;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(detect_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, flux, p.dev.det_w, G,
                     (int)p.cq0, (int)p.cnq, (int)p.Nd, K, (int)p.npos);
  return hipGetLastError();
}

hipError_t launch_inject(const Plan& p, const double* Gbar, double* inj, int K, hipStream_t s) {
  const int64_t total = p.cnq * (int64_t)K * 4 * p.npos;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(inject_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Gbar, p.dev.det_w, inj,
                     (int)p.cq0, (int)p.cnq, (int)p.Nd, K, (int)p.npos);
  return hipGetLastError();
}

hipError_t launch_misfit(const Plan& p, const double* G, const double* Gm, double* Gbar, double* J, int K,
                         hipStream_t s) {
  const int64_t off = p.cq0 * p.Nd * (int64_t)K;
  hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(1024), 0, s, G + off, Gm + off, Gbar + off, J,
                     p.cnq * p.Nd * (int64_t)K, p.prob.dt, p.cq0 > 0 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cadj_source(const Plan& p, const double* G, const double* Gm, double* src, int K, hipStream_t s) {
  const int64_t total = p.cnq * (int64_t)(K + 1) * p.nb;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(cadj_source_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G, Gm, p.dev.det_sp,
                     src, (int)p.cq0, (int)p.cnq, (int)p.Nd, K, (int)p.nb, (int)(4 * p.npos));
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const Plan& p, const double* ga, const double* gb, double* da, double* db,
                              hipStream_t s) {
  const int64_t Nn = p.nx * p.ny;
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)((Nn + 255) / 256)), dim3(256), 0, s, ga, gb, da, db,
                     (int)p.Nq, Nn);
  return hipGetLastError();
}

hipError_t launch_permute(const Plan& p, const void* in, void* state, hipStream_t s) {
  const int64_t Nn = p.nx * p.ny;
  const int64_t total = p.cnq * Nn * p.M;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (p.dtype == RTE_F64)
    hipLaunchKernelGGL(permute_kernel<double>, grid, dim3(256), 0, s, (const double*)in, (double*)state, p.dev.slot_m,
                       (int)p.M, (int)p.nx, (int)p.nxp, Nn, (int)p.cnq, p.grp_stride, p.inst_stride);
  else
    hipLaunchKernelGGL(permute_kernel<float>, grid, dim3(256), 0, s, (const float*)in, (float*)state, p.dev.slot_m,
                       (int)p.M, (int)p.nx, (int)p.nxp, Nn, (int)p.cnq, p.grp_stride, p.inst_stride);
  return hipGetLastError();
}

hipError_t launch_flux_map(const Plan& p, const void* state, double* out, int64_t out_q_stride, hipStream_t s) {
  if (p.nx > 65535 * 256 || p.ny > 65535 || p.cnq > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((p.nx + 255) / 256), (unsigned)p.ny, (unsigned)p.cnq);
  const double dth = 6.283185307179586476925 / (double)p.M;  // 2 pi / M
  if (p.dtype == RTE_F64)
    hipLaunchKernelGGL(flux_map_kernel<double>, grid, dim3(256), 0, s, (const double*)state, out, (int)p.M,
                       (int)p.nx, (int)p.nxp, p.grp_stride, p.inst_stride, out_q_stride, dth);
  else
    hipLaunchKernelGGL(flux_map_kernel<float>, grid, dim3(256), 0, s, (const float*)state, out, (int)p.M,
                       (int)p.nx, (int)p.nxp, p.grp_stride, p.inst_stride, out_q_stride, dth);
  return hipGetLastError();
}

// the chunk's sources into out[cq0 .. cq0 + cnq)
hipError_t launch_unpermute(const Plan& p, const void* state, void* out, hipStream_t s) {
  const int64_t Nn = p.nx * p.ny;
  const int64_t total = p.cnq * Nn * p.M;
  const dim3 grid((unsigned)((total + 255) / 256));
  const int64_t off = p.cq0 * Nn * p.M;
  if (p.dtype == RTE_F64)
    hipLaunchKernelGGL(unpermute_kernel<double>, grid, dim3(256), 0, s, (const double*)state, (double*)out + off,
                       p.dev.slot_m, (int)p.M, (int)p.nx, (int)p.nxp, Nn, (int)p.cnq, p.grp_stride, p.inst_stride);
  else
    hipLaunchKernelGGL(unpermute_kernel<float>, grid, dim3(256), 0, s, (const float*)state, (float*)out + off,
                       p.dev.slot_m, (int)p.M, (int)p.nx, (int)p.nxp, Nn, (int)p.cnq, p.grp_stride, p.inst_stride);
  return hipGetLastError();
}

}  // namespace rte
