// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rte.h"

namespace rte {

constexpr int kGroup = 4;        // ordinate slots per storage group (one reflection orbit)
constexpr int kMaxPasses = 12;   // FFT passes (radices 2,3,4,5)
constexpr int kMaxFcD = 8;       // matching points supported
// state arrays (one chunk) above this size are streamed with the
// non-temporal hint: a node pass then moves 8-10 such arrays, well beyond
// the 256 MiB memory-side cache that holds smaller plans' arrays between
// launches
constexpr int64_t kStreamNtBytes = int64_t(64) << 20;
constexpr int kLineThreads = 128; // generic (Stockham) line kernel
constexpr int kFcTab = 384;      // continuation matrix entries ((C+E) * 2d) staged by the four-step kernel
constexpr int kLongLine = 600;   // four-step lengths above this read the continuation matrix from global memory

void set_error(const std::string& msg);
const char* last_error();
int plan_create(const rte_problem*, const rte_beam*, int64_t, const rte_detector*, int64_t, rte_plan**);
int plan_destroy(rte_plan*);
size_t line_shmem_bytes(int Np, int dtype);

// FC-Gram derivative plan for one line direction (device pointers inside).
struct FcPlanDev {
  int n;        // nodes per line
  int Np;       // extended length n + C + E
  int E, d, C;
  int npass;
  int radix[kMaxPasses];
  int ns[kMaxPasses];       // Stockham sub-transform length before the pass
  int twoff[kMaxPasses];    // offset (complex entries) into the twiddle table
  const double* tw;         // complex twiddles, interleaved (re, im), FP64
  const double* mu;         // Np real multipliers: derivative factor * filter / Np
  const double* Q;          // d*d
  const double* A;          // C*d
  int n1, n2;               // four-step split Np = n1 * n2 (0: generic Stockham kernel)
  const double* roots;      // Np complex roots exp(-2 pi i e / Np), interleaved
  const double* Mx;         // (C+E) x 2d continuation matrix [MR | ML] (four-step kernel)
};

// Four-step splits with register codelets (Np -> n1 x n2); 0 if none.
bool fourstep_split(int Np, int* n1, int* n2);

// Per-slot boundary rule for one node type (9 types: interior, 4 edges, 4 corners).
struct BcRule {
  int32_t flag;     // 1 if (node type, slot) is overwritten by the inflow condition
  int32_t src_a, src_b;
  int32_t pad;
  double coef_a, coef_b;
};

// Transpose of the boundary map: for source slot s', the targets it feeds.
struct BcRuleT {
  int32_t is_target;   // slot is overwritten (its own value does not pass through)
  int32_t ntgt;
  int32_t tgt[2];
  double coef[2];
};

struct DeviceTables {
  // ordinates in storage order (slot s = 4*g + r)
  double* xi = nullptr;     // [M]
  double* eta = nullptr;    // [M]
  double* Wt = nullptr;     // [Mpad16][Mpad16] HG matrix in slot order (zero padded)
  BcRule* bc = nullptr;     // [9][M]
  BcRuleT* bct = nullptr;   // [9][M]
  double* kappa = nullptr;  // [4][M] detector factor per wall and slot
  double* det_w = nullptr;  // [Nd][4][npos] detector weights
  // beams: per beam spatial (boundary position) and angular (slot) factors, temporal samples
  double* beam_sp = nullptr;   // [nbeams][nb]
  double* beam_an = nullptr;   // [nbeams][M]
  double* beam_tt = nullptr;   // [nbeams][K+1]
  int32_t* beam_off = nullptr; // [Nq+1] CSR offsets of beams per source
  int32_t* slot_m = nullptr;   // [M] slot -> ordinate index
  double* fc_buf = nullptr;    // FC tables of both directions
  // continuous adjoint: detector footprint w(|x_b - x_j| / sigma_d) at the
  // boundary positions, and the slot of the reversed ordinate theta + pi
  double* det_sp = nullptr;    // [Nd][nb]
  int32_t* slot_rev = nullptr; // [Mpad] (padding slots map to themselves)
  // non-finite guard flag (one 8-byte word, the only mutable plan memory)
  unsigned long long* guard_flag = nullptr;
};

struct Plan {
  rte_problem prob{};
  int dtype = RTE_F64;
  int64_t nx = 0, ny = 0, M = 0, G = 0, Mpad = 0, K = 0, Nq = 0, Nd = 0, nbeams = 0;
  // state layout [q][g][j][i][r]: rows padded to nxp nodes so that every row
  // starts on a 128-byte boundary (4 FP64 or 8 FP32 nodes of one group)
  int64_t nxp = 0;
  int64_t grp_stride = 0;   // ny * nxp * kGroup elements
  int64_t inst_stride = 0;  // G * grp_stride
  bool fc_same = false;     // x and y FC plans identical: both line sets in one launch
  rte_schedule sched{1, 0, 0, 2, 1, 0};  // launch schedule (node_tiles_per_block resolved at create)
  int64_t sched_version = 0;       // bumped by every schedule change (graph keys)
  int64_t nb = 0;     // boundary nodes 2(nx+ny)-4
  int64_t npos = 0;   // max(nx, ny)
  std::vector<int> slot_m;  // slot -> ordinate index
  FcPlanDev fcx{}, fcy{};
  DeviceTables dev;
  int64_t ckpt_every = 0;
  // combination chunks: the workspace holds `chunk` sources; kernels work on
  // sources [cq0, cq0 + cnq) of the current chunk (set by the orchestration)
  int64_t chunk = 1;
  mutable int64_t cq0 = 0, cnq = 1;
  // one state array of a chunk exceeds kStreamNtBytes: the per-step kernels
  // stream their state arrays with the non-temporal hint (set at create)
  bool stream_nt = false;
  int64_t saved_chunk = -1;    // chunk whose forward states are in the workspace
  bool have_forward = false;   // a saved forward lives in the workspace
  int64_t saved_K = 0;
  const void* saved_ws = nullptr;  // workspace base of the saved forward
  // staged gradient (rte_gradient_range): next op expected and the
  // argument pointers of the sequence in progress
  int64_t range_next = -1;
  const void* range_key[9] = {nullptr};
  // graph mode: rte_gradient recorded once per argument set, then replayed
  bool use_graph = false;
  bool guard = false;          // scan outputs for NaN / Inf after each call
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gkey[9] = {nullptr};
  int64_t gkey_bytes = 0;
  int64_t gkey_sched = -1;
  // instrumentation: event pairs per kernel class
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec[RTE_K_COUNT];
};

// Bracket a launch with profiling events when enabled.
hipError_t prof_begin(Plan& p, int cls, hipStream_t s, hipEvent_t* stop);
hipError_t prof_end(hipEvent_t stop, hipStream_t s);

// ---------------------------------------------------------------- workspace map
struct Workspace {
  char* base = nullptr;
  int64_t bytes = 0;
  // state-sized arrays (plan dtype), each Nq*M*ny*nx elements
  void* states = nullptr;    // store-all: (K+1) states; checkpoint: segment store (s+1)
  void* ckpts = nullptr;     // checkpoint mode: n_ckpt * 4 states (u, L1, L2, L3)
  void* work_u[2] = {nullptr, nullptr};  // checkpoint mode: ping-pong current state
  void* lring[3] = {nullptr, nullptr, nullptr};
  void* tx = nullptr;        // forward: -xi Dx u^n
  void* ty = nullptr;        // forward: -eta Dy u^n
  void* vring[4] = {nullptr, nullptr, nullptr, nullptr};  // adjoint ring v^k
  void* wbuf = nullptr;      // adjoint w^n (aliases tx: live only inside one adjoint step)
  // adjoint carries from step n+1 to step n: ubar^{n+1} = ap1 - c dt (atx + aty)
  void* atx = nullptr;       // Dx^T(xi w^{n+1})
  void* aty = nullptr;       // Dy^T(eta w^{n+1})
  void* ap1 = nullptr;       // v^{n+2} + c dt (b W w - (a+b) w)^{n+1} + D_e^T Gbar
  double* flux = nullptr;    // [Nq][K+1][4][npos] detector flux / adjoint injection
  double* ga = nullptr;      // [Nq][ny*nx]
  double* gb = nullptr;
  double* gbar = nullptr;    // [Nq][Nd][K] misfit cotangent (rte_gradient)
  double* scratch = nullptr; // small reductions
};

// rte_forward without kept states into the device buffer [buf, buf + bytes)
// (256-byte aligned); a forward saved in another workspace stays valid
int forward_into(Plan& p, const void* mu_a, const void* mu_s, double* G, void* u_final, void* buf, int64_t bytes,
                 hipStream_t st);

int64_t state_elems(const Plan& p);
// bytes between consecutive state arrays of the workspace
int64_t state_stride_bytes(const Plan& p);
int64_t workspace_bytes(const Plan& p, bool with_adjoint);
bool map_workspace(const Plan& p, void* base, int64_t bytes, bool with_adjoint, Workspace* ws);

// ---------------------------------------------------------------- kernel launchers
enum LineMode {
  LINE_FWD = 0,  // out_x = -xi Dx(in), out_y = -eta Dy(in)
  LINE_ADJ = 1   // out_x = Dx^T(xi in), out_y = Dy^T(eta in)
};

// Both line sets of one state (dirs bit 0: x lines / rows, bit 1: y lines /
// columns).  Launched as one kernel when the two FC plans coincide.
struct LineLaunch {
  const void* in;
  void* out_x;
  void* out_y;
  int mode;
  int dirs;
};

hipError_t launch_lines(const Plan& p, const LineLaunch& L, hipStream_t s);
// four-step kernel for one direction set; hipErrorNotSupported if Np has no split
hipError_t launch_lines4(const Plan& p, const LineLaunch& L, hipStream_t s);
// generic Stockham kernel for one direction
hipError_t launch_line_generic(const Plan& p, const void* in, void* out, int mode, int dir, hipStream_t s);

struct NodeFwdLaunch {
  const void* u;       // u^n
  const void* X;       // -xi Dx u^n
  const void* Y;       // -eta Dy u^n
  const void* L1;      // L^{n-1}
  const void* L2;
  const void* L3;
  const void* mu_a;
  const void* mu_s;
  void* u_out;         // u^{n+1}
  void* L_out;         // L^n
  double* flux;        // [Nq][K+1][4][npos] or nullptr (replay)
  int step;            // n (time level of u)
  // continuous adjoint (the same step applied to psi, the time- and
  // ordinate-reversed adjoint): inflow source from csrc instead of the beams,
  // and the gradient terms of the input psi paired with the forward state
  // upair (u at the same physical time); csrc == nullptr: ordinary forward
  const double* csrc = nullptr;  // [Nq][K+1][4 npos] (first nb entries used)
  const void* upair = nullptr;
  double* ga = nullptr;          // [Nq][ny*nx]
  double* gb = nullptr;
  // extended forward (rte_forward_ex): separable volumetric source and
  // inflow data; step may be -3..-1 for the start-up history passes
  const rte_separable* vsrc = nullptr;
  const rte_separable* inflow = nullptr;
};
hipError_t launch_node_fwd(const Plan& p, const NodeFwdLaunch& L, hipStream_t s);

struct NodeAdjLaunch {
  const void* atx;     // pieces of ubar^{n+1}: ap1 - c dt (atx + aty)
  const void* aty;
  void* ap1;           // read as P1^{n+1}, overwritten with P1^n
  void* v1_out;        // ring slot for v^{n+1} = P^T ubar^{n+1}
  const void* v2;      // v^{n+2}
  const void* v3;
  const void* v4;
  const void* u;       // u^n
  const void* mu_a;
  const void* mu_s;
  const double* inj;   // [Nq][K+1][4][npos] detector injection
  void* w_out;         // w^n
  double* ga;          // [Nq][ny*nx]
  double* gb;
  int step;            // n
};
hipError_t launch_node_adj(const Plan& p, const NodeAdjLaunch& L, hipStream_t s);
// admissible node tiles per block for this plan (RT = Mpad / 16 row tiles)
bool node_tiles_ok(const Plan& p, int nt);
int node_tiles_default(const Plan& p);

hipError_t launch_detect(const Plan& p, const double* flux, double* G, int K, hipStream_t s);
hipError_t launch_inject(const Plan& p, const double* Gbar, double* inj, int K, hipStream_t s);
hipError_t launch_misfit(const Plan& p, const double* G, const double* Gm, double* Gbar, double* J,
                         int K, hipStream_t s);
// continuous adjoint inflow source of the current chunk's sources:
// src[q][k][bp] = sum_j det_sp[j][bp] r_j(t_{K-k}), r(t_n) = G^n - G~^n (n >= 1), r(t_0) = 0
hipError_t launch_cadj_source(const Plan& p, const double* G, const double* Gm, double* src, int K, hipStream_t s);
hipError_t launch_grad_reduce(const Plan& p, const double* ga, const double* gb, double* da, double* db,
                              hipStream_t s);
hipError_t launch_unpermute(const Plan& p, const void* state, void* out, hipStream_t s);
// natural [cnq][ny][nx][M] (the chunk's sources) into the state layout (padding untouched)
hipError_t launch_permute(const Plan& p, const void* in, void* state, hipStream_t s);
// scalar flux of the chunk's sources: out[q'][j][i] for q' = 0 .. cnq - 1 at
// out + q' out_q_stride (the caller offsets out to the chunk's first source)
hipError_t launch_flux_map(const Plan& p, const void* state, double* out, int64_t out_q_stride, hipStream_t s);
// flag[0] = 1 if any of x[0 .. n) is NaN or infinite (flag left alone otherwise)
hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long* flag, hipStream_t s);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);
hipError_t launch_copy(void* d, const void* src, int64_t bytes, hipStream_t s);

}  // namespace rte
