// C ABI entry points: orchestration of the per-step kernels (Algorithm 1 for
// the forward; the exact discrete adjoint in reverse time; checkpointed
// segment replay when the states do not all fit).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <sstream>
#include <string>
#include <vector>

#include "rte_internal.h"

using namespace rte;

namespace {

#define RTE_CHECK(expr)                                                  \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) {                                              \
      std::ostringstream o_;                                             \
      o_ << #expr << ": " << hipGetErrorString(e_);                      \
      set_error(o_.str());                                               \
      return RTE_EDEVICE;                                                \
    }                                                                    \
  } while (0)

struct Ctx {
  Plan& p;
  Workspace& ws;
  hipStream_t st;
  const void* mu_a;
  const void* mu_s;
  int64_t S;  // state stride in bytes
  const rte_forward_extra* ext = nullptr;  // rte_forward_ex: source, inflow data
};

inline void* at(void* base, int64_t k, int64_t S) { return static_cast<char*>(base) + k * S; }

// Non-finite guard: scan the FP64 outputs of a call on the stream, wait, and
// report RTE_EUNSTABLE if any value is NaN or infinite.
struct Out {
  const double* x;
  int64_t n;
};
int guard_check(Plan& p, hipStream_t st, const std::vector<Out>& outs) {
  if (!p.guard) return RTE_OK;
  RTE_CHECK(launch_zero(p.dev.guard_flag, 8, st));
  for (const Out& o : outs)
    if (o.x) RTE_CHECK(launch_nonfinite(o.x, o.n, p.dev.guard_flag, st));
  unsigned long long h = 0;
  RTE_CHECK(hipMemcpyAsync(&h, p.dev.guard_flag, 8, hipMemcpyDeviceToHost, st));
  RTE_CHECK(hipStreamSynchronize(st));
  if (h) {
    set_error("non-finite values in the outputs: dt beyond the stiff stability limit or non-finite medium maps");
    return RTE_EUNSTABLE;
  }
  return RTE_OK;
}

#define TIMED(cls, expr)                          \
  do {                                            \
    hipEvent_t stop_;                             \
    RTE_CHECK(prof_begin(c.p, (cls), c.st, &stop_)); \
    RTE_CHECK(expr);                              \
    RTE_CHECK(prof_end(stop_, c.st));             \
  } while (0)

// One forward step u^n -> u^{n+1}: x and y lines (one launch), node update.
int fwd_step(Ctx& c, int n, const void* un, void* unp1, double* flux) {
  LineLaunch ll{un, c.ws.tx, c.ws.ty, LINE_FWD, 3};
  TIMED(RTE_K_LINES_FWD, launch_lines(c.p, ll, c.st));
  NodeFwdLaunch nf;
  nf.u = un;
  nf.X = c.ws.tx;
  nf.Y = c.ws.ty;
  nf.L1 = c.ws.lring[(n + 2) % 3];
  nf.L2 = c.ws.lring[(n + 1) % 3];
  nf.L3 = c.ws.lring[n % 3];
  nf.mu_a = c.mu_a;
  nf.mu_s = c.mu_s;
  nf.u_out = unp1;
  nf.L_out = c.ws.lring[n % 3];
  nf.flux = flux;
  nf.step = n;
  if (c.ext) {
    nf.vsrc = &c.ext->source;
    nf.inflow = &c.ext->inflow;
  }
  TIMED(RTE_K_NODE_FWD, launch_node_fwd(c.p, nf, c.st));
  return RTE_OK;
}

// One adjoint step n (K..1) given u^n: node pass (forms v^{n+1} from the
// carried pieces of ubar^{n+1}, then w^n, P1^n and the gradient terms), then
// the transposed line derivatives of w^n, carried to step n-1.
int adj_step(Ctx& c, int n, const void* un) {
  NodeAdjLaunch na;
  na.atx = c.ws.atx;
  na.aty = c.ws.aty;
  na.ap1 = c.ws.ap1;
  na.v1_out = c.ws.vring[(n + 1) % 4];
  na.v2 = c.ws.vring[(n + 2) % 4];
  na.v3 = c.ws.vring[(n + 3) % 4];
  na.v4 = c.ws.vring[n % 4];
  na.u = un;
  na.mu_a = c.mu_a;
  na.mu_s = c.mu_s;
  na.inj = c.ws.flux;
  na.w_out = c.ws.wbuf;
  na.ga = c.ws.ga;
  na.gb = c.ws.gb;
  na.step = n;
  TIMED(RTE_K_NODE_ADJ, launch_node_adj(c.p, na, c.st));
  LineLaunch ll{c.ws.wbuf, c.ws.atx, c.ws.aty, LINE_ADJ, 3};
  TIMED(RTE_K_LINES_ADJ, launch_lines(c.p, ll, c.st));
  return RTE_OK;
}

// Sources are solved in chunks of p.chunk (one chunk when the workspace holds
// them all).  Chunk k covers sources [k chunk, min((k + 1) chunk, Nq)).
int64_t n_chunks(const Plan& p) { return (p.Nq + p.chunk - 1) / p.chunk; }

void set_chunk(const Plan& p, int64_t k) {
  p.cq0 = k * p.chunk;
  p.cnq = std::min(p.chunk, p.Nq - p.cq0);
}

void reset_chunk(const Plan& p) {
  p.cq0 = 0;
  p.cnq = p.chunk;
}

// The workspace now holds the saved forward of every source; the states of
// the last chunk are resident.
void mark_saved(Plan& p, const void* wsp) {
  p.have_forward = true;
  p.saved_chunk = n_chunks(p) - 1;
  p.saved_K = p.K;
  p.saved_ws = wsp;
}

// Maps the workspace; RTE_EINVAL for a base that is not 256-byte aligned
// (the kernels issue 16-byte vector accesses at offsets that are multiples
// of 256 from it), RTE_ENOMEM for a buffer that is too small.
int map_or_fail(const Plan& p, void* wsp, int64_t wsb, bool adj, Workspace* ws) {
  if (reinterpret_cast<uintptr_t>(wsp) % 256 != 0) {
    set_error("workspace must be 256-byte aligned");
    return RTE_EINVAL;
  }
  if (map_workspace(p, wsp, wsb, adj, ws)) return RTE_OK;
  std::ostringstream o;
  o << "workspace too small: need " << workspace_bytes(p, adj) << " bytes";
  set_error(o.str());
  return RTE_ENOMEM;
}

// Forward of the current chunk, in pieces: start (zero history, u^0 = 0) and
// step n (with its checkpoint copy when due).  State u^n lives in the state
// store when every state is kept, else in the ping-pong pair.
void* fwd_state(const Ctx& c, bool store_all, int n) {
  return store_all ? at(c.ws.states, n, c.S) : c.ws.work_u[n & 1];
}

int forward_start(Ctx& c, bool save) {
  const bool store_all = save && c.p.ckpt_every == 0;
  for (int k = 0; k < 3; ++k) RTE_CHECK(launch_zero(c.ws.lring[k], c.S, c.st));
  RTE_CHECK(launch_zero(fwd_state(c, store_all, 0), c.S, c.st));
  return RTE_OK;
}

int forward_op(Ctx& c, bool save, int n) {
  const bool store_all = save && c.p.ckpt_every == 0;
  const int64_t s = c.p.ckpt_every, S = c.S;
  void* un = fwd_state(c, store_all, n);
  if (save && s > 0 && n % s == 0) {
    void* ck = at(c.ws.ckpts, (n / s) * 4, S);
    RTE_CHECK(launch_copy(ck, un, S, c.st));
    RTE_CHECK(launch_copy(at(ck, 1, S), c.ws.lring[(n + 2) % 3], S, c.st));
    RTE_CHECK(launch_copy(at(ck, 2, S), c.ws.lring[(n + 1) % 3], S, c.st));
    RTE_CHECK(launch_copy(at(ck, 3, S), c.ws.lring[n % 3], S, c.st));
  }
  return fwd_step(c, n, un, fwd_state(c, store_all, n + 1), c.ws.flux);
}

// Time loop of the forward for the current chunk (u^0 = 0, zero history);
// writes the chunk's detector flux; keeps states or checkpoints when save.
int forward_chunk(Ctx& c, bool save, void* u_final) {
  if (int rc = forward_start(c, save)) return rc;
  for (int n = 0; n < c.p.K; ++n)
    if (int rc = forward_op(c, save, n)) return rc;
  if (u_final) RTE_CHECK(launch_unpermute(c.p, fwd_state(c, save && c.p.ckpt_every == 0, (int)c.p.K), u_final, c.st));
  return RTE_OK;
}

// Adjoint of the current chunk in pieces: start (zero ring and carries:
// ubar^{K+1} = 0, v^{K+2..K+4} = 0), the restore of checkpoint j at the start
// of segment j (checkpoint mode), and step n given u^n.
int adjoint_start(Ctx& c) {
  for (int k = 0; k < 4; ++k) RTE_CHECK(launch_zero(c.ws.vring[k], c.S, c.st));
  RTE_CHECK(launch_zero(c.ws.atx, c.S, c.st));
  RTE_CHECK(launch_zero(c.ws.aty, c.S, c.st));
  RTE_CHECK(launch_zero(c.ws.ap1, c.S, c.st));
  return RTE_OK;
}

int segment_restore(Ctx& c, int j) {
  const int64_t S = c.S;
  const int k0 = j * (int)c.p.ckpt_every;
  void* ck = at(c.ws.ckpts, (int64_t)j * 4, S);
  RTE_CHECK(launch_copy(c.ws.states, ck, S, c.st));
  RTE_CHECK(launch_copy(c.ws.lring[(k0 + 2) % 3], at(ck, 1, S), S, c.st));
  RTE_CHECK(launch_copy(c.ws.lring[(k0 + 1) % 3], at(ck, 2, S), S, c.st));
  RTE_CHECK(launch_copy(c.ws.lring[k0 % 3], at(ck, 3, S), S, c.st));
  return RTE_OK;
}

// Operation cursor: the gradient is a fixed sequence of operations and a
// call enqueues those with index in [first, last).
struct OpCursor {
  int64_t first, last, idx;
  bool take() {
    const bool t = idx >= first && idx < last;
    ++idx;
    return t;
  }
};

// Reverse time loop of the adjoint for the current chunk, whose forward
// states (or checkpoints) are in the workspace and whose detector injection
// is in ws.flux; accumulates the chunk's gradient partials into ga, gb.
// Operations: start, then K adjoint steps (every state kept) or, per
// segment from the last, the restore, the replay steps and the adjoint steps.
int adjoint_ops(Ctx& c, OpCursor& r) {
  Plan& p = c.p;
  const int64_t S = c.S;
  const int K = (int)p.K;
  if (r.take())
    if (int rc = adjoint_start(c)) return rc;
  if (p.ckpt_every == 0) {
    for (int n = K; n >= 1; --n)
      if (r.take())
        if (int rc = adj_step(c, n, at(c.ws.states, n, S))) return rc;
    return RTE_OK;
  }
  const int s = (int)p.ckpt_every;
  const int nseg = (K + s - 1) / s;
  for (int j = nseg - 1; j >= 0; --j) {
    const int k0 = j * s, k1 = std::min(k0 + s, K);
    if (r.take())
      if (int rc = segment_restore(c, j)) return rc;
    for (int k = k0; k < k1; ++k)
      if (r.take())
        if (int rc = fwd_step(c, k, at(c.ws.states, k - k0, S), at(c.ws.states, k + 1 - k0, S), nullptr)) return rc;
    for (int n = k1; n > k0; --n)
      if (r.take())
        if (int rc = adj_step(c, n, at(c.ws.states, n - k0, S))) return rc;
  }
  return RTE_OK;
}

int adjoint_chunk(Ctx& c) {
  OpCursor r{0, INT64_MAX, 0};
  return adjoint_ops(c, r);
}

int run_forward(Plan& p, const void* mu_a, const void* mu_s, double* G, void* u_final, int save, void* wsp,
                int64_t wsb, hipStream_t st) {
  Workspace ws;
  if (int rc = map_or_fail(p, wsp, wsb, save != 0, &ws)) return rc;
  const int64_t S = state_stride_bytes(p);
  Ctx c{p, ws, st, mu_a, mu_s, S};
  p.have_forward = false;
  RTE_CHECK(launch_zero(ws.flux, p.Nq * (p.K + 1) * 4 * p.npos * 8, st));
  const int64_t nc = n_chunks(p);
  for (int64_t k = 0; k < nc; ++k) {
    set_chunk(p, k);
    int rc = forward_chunk(c, save != 0, u_final);
    if (rc == RTE_OK && G) rc = launch_detect(p, ws.flux, G, (int)p.K, st) == hipSuccess ? RTE_OK : RTE_EDEVICE;
    if (rc != RTE_OK) {
      reset_chunk(p);
      if (rc == RTE_EDEVICE && last_error()[0] == '\0') set_error("detector kernel launch failed");
      return rc;
    }
  }
  reset_chunk(p);
  if (save) mark_saved(p, wsp);
  return RTE_OK;
}

// Adjoint of the last saved forward.  The chunk whose states are in the
// workspace goes first; every other chunk's forward is recomputed.
int run_adjoint(Plan& p, const void* mu_a, const void* mu_s, const double* Gbar, double* da, double* db, void* wsp,
                int64_t wsb, hipStream_t st) {
  if (!p.have_forward) {
    set_error("rte_adjoint needs a preceding rte_forward with save_states=1 on this plan");
    return RTE_ESTATE;
  }
  if (wsp != p.saved_ws) {
    set_error("rte_adjoint needs the workspace of the saving forward (another buffer was passed)");
    return RTE_ESTATE;
  }
  Workspace ws;
  if (int rc = map_or_fail(p, wsp, wsb, true, &ws)) return rc;
  const int64_t S = state_stride_bytes(p);
  Ctx c{p, ws, st, mu_a, mu_s, S};
  const int64_t gbytes = p.Nq * p.nx * p.ny * 8;
  RTE_CHECK(launch_zero(ws.ga, gbytes, st));
  RTE_CHECK(launch_zero(ws.gb, gbytes, st));
  const int64_t nc = n_chunks(p);
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t k = (p.saved_chunk + nc - i) % nc;  // saved chunk first
    set_chunk(p, k);
    int rc = (i == 0) ? RTE_OK : forward_chunk(c, true, nullptr);
    if (rc == RTE_OK && launch_inject(p, Gbar, ws.flux, (int)p.K, st) != hipSuccess) rc = RTE_EDEVICE;
    if (rc == RTE_OK) rc = adjoint_chunk(c);
    if (rc != RTE_OK) {
      reset_chunk(p);
      if (rc == RTE_EDEVICE && last_error()[0] == '\0') set_error("injection kernel launch failed");
      return rc;
    }
  }
  p.saved_chunk = (p.saved_chunk + 1) % nc;  // the last chunk processed
  reset_chunk(p);
  RTE_CHECK(launch_grad_reduce(p, ws.ga, ws.gb, da, db, st));
  return RTE_OK;
}

// ---------------------------------------------------------------- continuous adjoint
// psi(x, theta, s) = lambda(x, theta + pi, T - s) solves the forward equation
// (eq. AdjointProblem in reversed time and ordinates), so each of its steps is
// a forward step whose node pass takes the detector residual as inflow source
// and adds the eq. (FDwin22) terms.  Its arrays: without checkpoints no
// forward step runs meanwhile and the forward work arrays are free; with
// checkpoints the segment replays use them and psi takes the adjoint arrays.
struct PsiArrays {
  void* psi[2];
  void* lr[3];
  void* X;
  void* Y;
};

PsiArrays psi_arrays(const Plan& p, const Workspace& ws) {
  if (p.ckpt_every == 0) return {{ws.vring[3], ws.ap1}, {ws.lring[0], ws.lring[1], ws.lring[2]}, ws.tx, ws.ty};
  return {{ws.vring[0], ws.vring[1]}, {ws.vring[2], ws.vring[3], ws.ap1}, ws.atx, ws.aty};
}

// psi^k -> psi^{k+1}; upair = u^{K-k} (the forward state at the physical time of psi^k)
int psi_step(Ctx& c, const PsiArrays& A, int k, const void* upair) {
  const void* in = A.psi[k & 1];
  LineLaunch ll{in, A.X, A.Y, LINE_FWD, 3};
  TIMED(RTE_K_LINES_FWD, launch_lines(c.p, ll, c.st));
  NodeFwdLaunch nf;
  nf.u = in;
  nf.X = A.X;
  nf.Y = A.Y;
  nf.L1 = A.lr[(k + 2) % 3];
  nf.L2 = A.lr[(k + 1) % 3];
  nf.L3 = A.lr[k % 3];
  nf.mu_a = c.mu_a;
  nf.mu_s = c.mu_s;
  nf.u_out = A.psi[(k + 1) & 1];
  nf.L_out = A.lr[k % 3];
  nf.flux = nullptr;
  nf.step = k;
  nf.csrc = c.ws.flux;
  nf.upair = upair;
  nf.ga = c.ws.ga;
  nf.gb = c.ws.gb;
  TIMED(RTE_K_NODE_FWD, launch_node_fwd(c.p, nf, c.st));
  return RTE_OK;
}

// The psi time loop of the current chunk (forward states or checkpoints in
// the workspace, residual source table in ws.flux): psi^0 = 0, zero history.
int cadj_chunk(Ctx& c) {
  Plan& p = c.p;
  Workspace& ws = c.ws;
  hipStream_t st = c.st;
  const int64_t S = c.S;
  const int K = (int)p.K;
  const PsiArrays A = psi_arrays(p, ws);
  RTE_CHECK(launch_zero(A.psi[0], S, st));
  for (int k = 0; k < 3; ++k) RTE_CHECK(launch_zero(A.lr[k], S, st));
  if (p.ckpt_every == 0) {
    for (int k = 0; k < K; ++k) {
      int rc = psi_step(c, A, k, at(ws.states, K - k, S));
      if (rc != RTE_OK) return rc;
    }
    return RTE_OK;
  }
  const int s = (int)p.ckpt_every;
  const int nseg = (K + s - 1) / s;
  for (int j = nseg - 1; j >= 0; --j) {
    const int k0 = j * s, k1 = std::min(k0 + s, K);
    void* ck = at(ws.ckpts, (int64_t)j * 4, S);
    RTE_CHECK(launch_copy(ws.states, ck, S, st));
    RTE_CHECK(launch_copy(ws.lring[(k0 + 2) % 3], at(ck, 1, S), S, st));
    RTE_CHECK(launch_copy(ws.lring[(k0 + 1) % 3], at(ck, 2, S), S, st));
    RTE_CHECK(launch_copy(ws.lring[k0 % 3], at(ck, 3, S), S, st));
    for (int k = k0; k < k1; ++k) {
      int rc = fwd_step(c, k, at(ws.states, k - k0, S), at(ws.states, k + 1 - k0, S), nullptr);
      if (rc != RTE_OK) return rc;
    }
    for (int n = k1; n > k0; --n) {
      int rc = psi_step(c, A, K - n, at(ws.states, n - k0, S));
      if (rc != RTE_OK) return rc;
    }
  }
  return RTE_OK;
}

// ---------------------------------------------------------------- extended forward
// rte_forward_ex for the current chunk: start-up history L^{-k} from the given
// states (lines and node pass at time level -k, the state update discarded),
// initial state, then the time loop with the separable source and inflow.
int forward_ex_chunk(Ctx& c, void* u_final) {
  Plan& p = c.p;
  Workspace& ws = c.ws;
  hipStream_t st = c.st;
  const int64_t S = c.S;
  const rte_forward_extra* ex = c.ext;
  const int64_t es = (p.dtype == RTE_F64) ? 8 : 4;
  const int64_t nat = p.nx * p.ny * p.M * es;  // one source, natural layout
  for (int k = 0; k < 3; ++k) RTE_CHECK(launch_zero(ws.lring[k], S, st));
  RTE_CHECK(launch_zero(ws.work_u[0], S, st));
  if (ex->u_hist) {
    for (int k = 3; k >= 1; --k) {
      const char* h = static_cast<const char*>(ex->u_hist) + ((int64_t)(k - 1) * p.Nq + p.cq0) * nat;
      RTE_CHECK(launch_permute(p, h, ws.work_u[0], st));
      LineLaunch ll{ws.work_u[0], ws.tx, ws.ty, LINE_FWD, 3};
      TIMED(RTE_K_LINES_FWD, launch_lines(p, ll, st));
      void* Lk = ws.lring[(3 - k) % 3];  // L^{-k}: ring slot (-k) mod 3
      NodeFwdLaunch nf;
      nf.u = ws.work_u[0];
      nf.X = ws.tx;
      nf.Y = ws.ty;
      nf.L1 = nf.L2 = nf.L3 = Lk;        // read and overwritten by the same lane; update discarded
      nf.mu_a = c.mu_a;
      nf.mu_s = c.mu_s;
      nf.u_out = ws.work_u[1];
      nf.L_out = Lk;
      nf.flux = nullptr;
      nf.step = -k;
      nf.vsrc = &ex->source;
      nf.inflow = &ex->inflow;
      TIMED(RTE_K_NODE_FWD, launch_node_fwd(p, nf, st));
    }
  }
  if (ex->u0) {
    RTE_CHECK(launch_zero(ws.work_u[0], S, st));
    RTE_CHECK(launch_permute(p, static_cast<const char*>(ex->u0) + p.cq0 * nat, ws.work_u[0], st));
  } else if (ex->u_hist) {
    RTE_CHECK(launch_zero(ws.work_u[0], S, st));
  }
  // scalar-flux snapshots of u^n: out[q][k] for every k with snap_steps[k] == n
  const int64_t Nn = p.nx * p.ny;
  auto snap = [&](int n, const void* un) -> int {
    for (int k = 0; k < ex->n_snap; ++k)
      if (ex->snap_steps[k] == n)
        RTE_CHECK(launch_flux_map(p, un, ex->snap_flux + (p.cq0 * ex->n_snap + k) * Nn, ex->n_snap * Nn, st));
    return RTE_OK;
  };
  if (int rc = snap(0, ws.work_u[0])) return rc;
  for (int n = 0; n < p.K; ++n) {
    int rc = fwd_step(c, n, ws.work_u[n & 1], ws.work_u[(n + 1) & 1], ws.flux);
    if (rc == RTE_OK) rc = snap(n + 1, ws.work_u[(n + 1) & 1]);
    if (rc != RTE_OK) return rc;
  }
  if (u_final) RTE_CHECK(launch_unpermute(p, ws.work_u[p.K & 1], u_final, st));
  return RTE_OK;
}

int run_forward_ex(Plan& p, const void* mu_a, const void* mu_s, const rte_forward_extra* ex, double* G,
                   void* u_final, void* wsp, int64_t wsb, hipStream_t st) {
  Workspace ws;
  if (int rc = map_or_fail(p, wsp, wsb, false, &ws)) return rc;
  const int64_t S = state_stride_bytes(p);
  Ctx c{p, ws, st, mu_a, mu_s, S};
  c.ext = ex;
  p.have_forward = false;
  RTE_CHECK(launch_zero(ws.flux, p.Nq * (p.K + 1) * 4 * p.npos * 8, st));
  const int64_t nc = n_chunks(p);
  for (int64_t k = 0; k < nc; ++k) {
    set_chunk(p, k);
    int rc = forward_ex_chunk(c, u_final);
    if (rc == RTE_OK && G) rc = launch_detect(p, ws.flux, G, (int)p.K, st) == hipSuccess ? RTE_OK : RTE_EDEVICE;
    if (rc != RTE_OK) {
      reset_chunk(p);
      if (rc == RTE_EDEVICE && last_error()[0] == '\0') set_error("detector kernel launch failed");
      return rc;
    }
  }
  reset_chunk(p);
  return RTE_OK;
}

struct GradArgs {
  const void* mu_a;
  const void* mu_s;
  const double* G_meas;
  double* J;
  double* dmu_a;
  double* dmu_s;
  double* G;
  void* ws;
  int64_t wsb;
};

std::vector<Out> grad_outputs(const Plan& p, const GradArgs& a) {
  return {{a.J, 1}, {a.dmu_a, p.nx * p.ny}, {a.dmu_s, p.nx * p.ny}, {a.G, p.Nq * p.Nd * p.K}};
}

// The gradient as a fixed sequence of operations, chunk by chunk: op 0 zeroes
// the detector flux and the gradient partials; per chunk, the forward start,
// K forward steps (states or checkpoints kept), the misfit (detector
// traces, J, cotangent, injection), then the adjoint operations of
// adjoint_ops; the last op reduces the partials over the sources.  A call
// enqueues the ops with index in [first, last) on st and returns the total
// count in *n_ops; every op is a function of the plan, the arguments and
// its index only, so consecutive ranges compose to the whole gradient bit
// for bit.
int enqueue_gradient_ops(Plan& p, const GradArgs& a, hipStream_t st, int64_t first, int64_t last, int64_t* n_ops) {
  Workspace ws;
  if (int rc = map_or_fail(p, a.ws, a.wsb, true, &ws)) return rc;
  const int64_t S = state_stride_bytes(p);
  Ctx c{p, ws, st, a.mu_a, a.mu_s, S};
  OpCursor r{first, last, 0};
  const int64_t nc = n_chunks(p);
  const int K = (int)p.K;
  auto body = [&]() -> int {
    if (r.take()) {
      p.have_forward = false;
      RTE_CHECK(launch_zero(ws.flux, p.Nq * (p.K + 1) * 4 * p.npos * 8, st));
      const int64_t gbytes = p.Nq * p.nx * p.ny * 8;
      RTE_CHECK(launch_zero(ws.ga, gbytes, st));
      RTE_CHECK(launch_zero(ws.gb, gbytes, st));
    }
    for (int64_t k = 0; k < nc; ++k) {
      set_chunk(p, k);
      if (r.take())
        if (int rc = forward_start(c, true)) return rc;
      for (int n = 0; n < K; ++n)
        if (r.take())
          if (int rc = forward_op(c, true, n)) return rc;
      if (r.take()) {
        hipError_t e = launch_detect(p, ws.flux, a.G, K, st);
        if (e == hipSuccess) e = launch_misfit(p, a.G, a.G_meas, ws.gbar, a.J, K, st);
        if (e == hipSuccess) e = launch_inject(p, ws.gbar, ws.flux, K, st);
        if (e != hipSuccess) {
          set_error(std::string("detector/misfit kernel launch failed: ") + hipGetErrorString(e));
          return RTE_EDEVICE;
        }
      }
      if (int rc = adjoint_ops(c, r)) return rc;
    }
    reset_chunk(p);
    if (r.take()) {
      RTE_CHECK(launch_grad_reduce(p, ws.ga, ws.gb, a.dmu_a, a.dmu_s, st));
      mark_saved(p, a.ws);
    }
    return RTE_OK;
  };
  const int rc = body();
  reset_chunk(p);
  if (n_ops) *n_ops = r.idx;
  return rc;
}

// Number of operations of one gradient (see enqueue_gradient_ops).
int64_t gradient_op_count(const Plan& p) {
  const int64_t K = p.K, s = p.ckpt_every;
  const int64_t adj = s > 0 ? 1 + ((K + s - 1) / s) + 2 * K : 1 + K;
  return 2 + n_chunks(p) * (1 + K + 1 + adj);
}

int enqueue_gradient(Plan& p, const GradArgs& a, hipStream_t st) {
  return enqueue_gradient_ops(p, a, st, 0, gradient_op_count(p), nullptr);
}

// Graph mode: record the whole sequence once per argument set, then replay.
// Forward with kept states, misfit, residual source, psi loop with the
// gradient terms, chunk by chunk: all enqueued on st.
int enqueue_gradient_continuous(Plan& p, const GradArgs& a, hipStream_t st) {
  Workspace ws;
  if (int rc = map_or_fail(p, a.ws, a.wsb, true, &ws)) return rc;
  const int64_t S = state_stride_bytes(p);
  Ctx c{p, ws, st, a.mu_a, a.mu_s, S};
  p.have_forward = false;
  RTE_CHECK(launch_zero(ws.flux, p.Nq * (p.K + 1) * 4 * p.npos * 8, st));
  const int64_t gbytes = p.Nq * p.nx * p.ny * 8;
  RTE_CHECK(launch_zero(ws.ga, gbytes, st));
  RTE_CHECK(launch_zero(ws.gb, gbytes, st));
  const int64_t nc = n_chunks(p);
  const int K = (int)p.K;
  for (int64_t k = 0; k < nc; ++k) {
    set_chunk(p, k);
    int rc = forward_chunk(c, true, nullptr);
    hipError_t e = hipSuccess;
    if (rc == RTE_OK) e = launch_detect(p, ws.flux, a.G, K, st);
    if (rc == RTE_OK && e == hipSuccess) e = launch_misfit(p, a.G, a.G_meas, ws.gbar, a.J, K, st);
    if (rc == RTE_OK && e == hipSuccess) e = launch_cadj_source(p, a.G, a.G_meas, ws.flux, K, st);
    if (rc == RTE_OK && e != hipSuccess) {
      set_error(std::string("detector/misfit/source kernel launch failed: ") + hipGetErrorString(e));
      rc = RTE_EDEVICE;
    }
    if (rc == RTE_OK) rc = cadj_chunk(c);
    if (rc != RTE_OK) {
      reset_chunk(p);
      return rc;
    }
  }
  reset_chunk(p);
  RTE_CHECK(launch_grad_reduce(p, ws.ga, ws.gb, a.dmu_a, a.dmu_s, st));
  mark_saved(p, a.ws);
  return RTE_OK;
}

int graph_gradient(Plan& p, const GradArgs& a, hipStream_t st) {
  const void* key[9] = {a.mu_a, a.mu_s, a.G_meas, a.J, a.dmu_a, a.dmu_s, a.G, a.ws, nullptr};
  bool same = p.gexec != nullptr && p.gkey_bytes == a.wsb && p.gkey_sched == p.sched_version;
  for (int k = 0; k < 8 && same; ++k) same = (p.gkey[k] == key[k]);
  if (!same) {
    if (p.gexec) {
      RTE_CHECK(hipGraphExecDestroy(p.gexec));
      p.gexec = nullptr;
    }
    if (!p.cap_stream) RTE_CHECK(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
    const bool prof = p.prof;
    p.prof = false;  // no event nodes in the recorded graph
    RTE_CHECK(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_gradient(p, a, p.cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(p.cap_stream, &graph);
    p.prof = prof;
    if (rc != RTE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    RTE_CHECK(ec);
    const hipError_t ei = hipGraphInstantiate(&p.gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    RTE_CHECK(ei);
    for (int k = 0; k < 8; ++k) p.gkey[k] = key[k];
    p.gkey_bytes = a.wsb;
    p.gkey_sched = p.sched_version;
  }
  RTE_CHECK(hipGraphLaunch(p.gexec, st));
  mark_saved(p, a.ws);
  return RTE_OK;
}

// ---- autotuner
bool sched_ok(const Plan& p, const rte_schedule& s) {
  return (s.line_units_per_wave == 1 || s.line_units_per_wave == 2) && (s.line_generic == 0 || s.line_generic == 1) &&
         node_tiles_ok(p, s.node_tiles_per_block) && (s.line_waves_per_unit == 1 || s.line_waves_per_unit == 2) &&
         (s.line_global_tables == 0 || s.line_global_tables == 1) && s.reserved == 0;
}

// Zeroed state-sized arrays of the gradient workspace and the launch records
// of the four per-step kernel classes on them (timing only: the values do not
// matter, every access stays inside the workspace).
struct TuneSet {
  Workspace ws;
  LineLaunch lf, lb;
  NodeFwdLaunch nf;
  NodeAdjLaunch na;
  int64_t S = 0;   // bytes per state
  int nst = 2;     // zeroed states at the start of the state store
  void* state(int k) const { return static_cast<char*>(ws.states) + (int64_t)(k % nst) * S; }
  // launch r of a timed run reads and writes distinct stored states, as the
  // time loop does: the forward walks up the store, the adjoint down
  NodeFwdLaunch fwd_at(int r) const {
    NodeFwdLaunch L = nf;
    L.u = state(r);
    L.u_out = state(r + 1);
    return L;
  }
  NodeAdjLaunch adj_at(int r) const {
    NodeAdjLaunch L = na;
    L.u = state(nst - 1 - r % nst);
    return L;
  }
};

int tune_setup(Plan& p, const void* mu_a, const void* mu_s, void* wsp, int64_t wsb, hipStream_t st, int nstates,
               TuneSet* t) {
  Workspace& ws = t->ws;
  if (int rc = map_or_fail(p, wsp, wsb, true, &ws)) return rc;
  p.have_forward = false;
  const int64_t S = state_stride_bytes(p);
  const int64_t cap = p.ckpt_every > 0 ? p.ckpt_every + 1 : p.K + 1;
  t->S = S;
  t->nst = (int)std::max<int64_t>(2, std::min<int64_t>(nstates, cap));
  for (int k = 0; k < t->nst; ++k) RTE_CHECK(launch_zero(static_cast<char*>(ws.states) + k * S, S, st));
  void* u0 = ws.states;
  void* u1 = static_cast<char*>(ws.states) + S;
  void* arrays[] = {ws.lring[0], ws.lring[1], ws.lring[2], ws.tx, ws.ty, ws.vring[0], ws.vring[1],
                    ws.vring[2], ws.vring[3], ws.atx, ws.aty, ws.ap1};
  for (void* a : arrays) RTE_CHECK(launch_zero(a, S, st));
  RTE_CHECK(launch_zero(ws.flux, p.Nq * (p.K + 1) * 4 * p.npos * 8, st));
  RTE_CHECK(launch_zero(ws.ga, p.Nq * p.nx * p.ny * 8, st));
  RTE_CHECK(launch_zero(ws.gb, p.Nq * p.nx * p.ny * 8, st));
  t->lf = LineLaunch{u0, ws.tx, ws.ty, LINE_FWD, 3};
  t->lb = LineLaunch{ws.wbuf, ws.atx, ws.aty, LINE_ADJ, 3};
  t->nf = NodeFwdLaunch{u0, ws.tx, ws.ty, ws.lring[1], ws.lring[2], ws.lring[0], mu_a, mu_s, u1, ws.lring[0], ws.flux, 0};
  t->na = NodeAdjLaunch{ws.atx, ws.aty, ws.ap1, ws.vring[1], ws.vring[2], ws.vring[3], ws.vring[0], u0,
                        mu_a, mu_s, ws.flux, ws.wbuf, ws.ga, ws.gb, (int)p.K};
  return RTE_OK;
}

// Mean microseconds per launch of `launch` over `reps` back-to-back launches
// recorded as one graph and replayed between two events on st.
template <typename F>
int time_graph(Plan& p, hipStream_t st, int reps, F&& launch, double* us) {
  if (!p.cap_stream) RTE_CHECK(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  RTE_CHECK(launch(st, 0));  // warm-up, eager
  RTE_CHECK(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch(p.cap_stream, r);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p.cap_stream, &graph);
  if (err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    RTE_CHECK(err);
  }
  RTE_CHECK(ec);
  hipGraphExec_t gx = nullptr;
  err = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  RTE_CHECK(err);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err == hipSuccess) err = hipGraphLaunch(gx, st);  // warm-up replay
  if (err == hipSuccess) err = hipEventRecord(e0, st);
  if (err == hipSuccess) err = hipGraphLaunch(gx, st);
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(gx);
  RTE_CHECK(err);
  *us = 1000.0 * ms / reps;
  return RTE_OK;
}

int time_kernels(Plan& p, const void* mu_a, const void* mu_s, void* wsp, int64_t wsb, hipStream_t st, int reps,
                 double* us) {
  TuneSet t;
  int rc = tune_setup(p, mu_a, mu_s, wsp, wsb, st, reps + 1, &t);
  if (rc != RTE_OK) return rc;
  const bool prof = p.prof;
  p.prof = false;
  rc = time_graph(p, st, reps, [&](hipStream_t s, int) { return launch_lines(p, t.lf, s); }, &us[RTE_K_LINES_FWD]);
  if (rc == RTE_OK)
    rc = time_graph(p, st, reps, [&](hipStream_t s, int r) { return launch_node_fwd(p, t.fwd_at(r), s); },
                    &us[RTE_K_NODE_FWD]);
  if (rc == RTE_OK)
    rc = time_graph(p, st, reps, [&](hipStream_t s, int r) { return launch_node_adj(p, t.adj_at(r), s); },
                    &us[RTE_K_NODE_ADJ]);
  if (rc == RTE_OK)
    rc = time_graph(p, st, reps, [&](hipStream_t s, int) { return launch_lines(p, t.lb, s); }, &us[RTE_K_LINES_ADJ]);
  p.prof = prof;
  return rc;
}

int autotune(Plan& p, const void* mu_a, const void* mu_s, void* wsp, int64_t wsb, hipStream_t st, rte_schedule* out) {
  TuneSet tset;
  int rc0 = tune_setup(p, mu_a, mu_s, wsp, wsb, st, 8, &tset);
  if (rc0 != RTE_OK) return rc0;
  const bool prof = p.prof;
  p.prof = false;
  const int reps = 5;
  const rte_schedule start = p.sched;
  rte_schedule best = p.sched;

  // line passes: forward and transpose launches of each admissible variant
  struct LineCand {
    int upw, nw, generic, tg;
  };
  std::vector<LineCand> line_cands;
  const bool four = p.fcx.n1 > 0 || p.fcy.n1 > 0;
  if (four)
    for (int upw : {2, 1})
      for (int nw : {1, 2})
        for (int tg : {0, 1}) line_cands.push_back({upw, nw, 0, tg});
  // the generic kernel transforms two ordinates of one line as one complex
  // line (less accurate near beams): a candidate only without a split
  if (!four) line_cands.push_back({1, 1, 1, 0});
  double best_ms = 1e30;
  for (const auto& c : line_cands) {
    p.sched.line_units_per_wave = c.upw;
    p.sched.line_waves_per_unit = c.nw;
    p.sched.line_generic = c.generic;
    p.sched.line_global_tables = c.tg;
    double f = 0.0, b = 0.0;
    const LineLaunch lf = tset.lf, lb = tset.lb;
    int rc = time_graph(p, st, reps, [&](hipStream_t s, int) { return launch_lines(p, lf, s); }, &f);
    if (rc == RTE_OK) rc = time_graph(p, st, reps, [&](hipStream_t s, int) { return launch_lines(p, lb, s); }, &b);
    if (rc != RTE_OK) {
      p.sched = start;
      p.prof = prof;
      return rc;
    }
    if (f + b < best_ms) {
      best_ms = f + b;
      best.line_units_per_wave = c.upw;
      best.line_waves_per_unit = c.nw;
      best.line_generic = c.generic;
      best.line_global_tables = c.tg;
    }
  }
  p.sched.line_units_per_wave = best.line_units_per_wave;
  p.sched.line_waves_per_unit = best.line_waves_per_unit;
  p.sched.line_generic = best.line_generic;
  p.sched.line_global_tables = best.line_global_tables;

  // node passes: tiles per block
  best_ms = 1e30;
  for (int nt : {1, 2, 4}) {
    if (!node_tiles_ok(p, nt)) continue;
    p.sched.node_tiles_per_block = nt;
    double f = 0.0, b = 0.0;
    int rc = time_graph(p, st, reps, [&](hipStream_t s, int r) { return launch_node_fwd(p, tset.fwd_at(r), s); }, &f);
    if (rc == RTE_OK)
      rc = time_graph(p, st, reps, [&](hipStream_t s, int r) { return launch_node_adj(p, tset.adj_at(r), s); }, &b);
    if (rc != RTE_OK) {
      p.sched = start;
      p.prof = prof;
      return rc;
    }
    if (f + b < best_ms) {
      best_ms = f + b;
      best.node_tiles_per_block = nt;
    }
  }
  p.sched = best;
  ++p.sched_version;
  p.prof = prof;
  if (out) *out = best;
  return RTE_OK;
}

struct Batch {
  std::vector<Plan*> plans;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipStream_t s0 = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> key;
};

bool nonnull(const void* p, const char* what) {
  if (!p) {
    set_error(std::string(what) + " is NULL");
    return false;
  }
  return true;
}

}  // namespace

namespace rte {

// rte_forward without kept states into a caller-chosen device buffer; leaves
// a forward saved in another workspace valid and records no profiling
// events.
int forward_into(Plan& p, const void* mu_a, const void* mu_s, double* G, void* u_final, void* buf, int64_t bytes,
                 hipStream_t st) {
  const bool had = p.have_forward, prof = p.prof;
  const int64_t chunk = p.saved_chunk;
  const void* sws = p.saved_ws;
  p.prof = false;
  const int rc = run_forward(p, mu_a, mu_s, G, u_final, 0, buf, bytes, st);
  p.prof = prof;
  p.have_forward = had;
  p.saved_chunk = chunk;
  p.saved_ws = sws;
  return rc != RTE_OK ? rc : guard_check(p, st, {{G, p.Nq * p.Nd * p.K}});
}

}  // namespace rte

extern "C" {

int rte_plan_create(const rte_problem* prob, const rte_beam* beams, int64_t n_beams, const rte_detector* dets,
                    int64_t n_det, rte_plan** out) {
  try {
    set_error("");
    return plan_create(prob, beams, n_beams, dets, n_det, out);
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_plan_destroy(rte_plan* plan) { return plan_destroy(plan); }

int rte_plan_info(const rte_plan* h, int64_t* Nq, int64_t* Nd, int64_t* Npx, int64_t* Npy) {
  if (!nonnull(h, "plan")) return RTE_EINVAL;
  const Plan& p = *reinterpret_cast<const Plan*>(h);
  if (Nq) *Nq = p.Nq;
  if (Nd) *Nd = p.Nd;
  if (Npx) *Npx = p.fcx.Np;
  if (Npy) *Npy = p.fcy.Np;
  return RTE_OK;
}

int rte_workspace_bytes(const rte_plan* h, int with_adjoint, int64_t* bytes) {
  if (!nonnull(h, "plan") || !nonnull(bytes, "bytes")) return RTE_EINVAL;
  *bytes = workspace_bytes(*reinterpret_cast<const Plan*>(h), with_adjoint != 0);
  return RTE_OK;
}

int rte_forward(rte_plan* h, const void* mu_a, const void* mu_s, double* G, void* u_final, int save_states,
                void* workspace, int64_t workspace_bytes, void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = run_forward(p, mu_a, mu_s, G, u_final, save_states, workspace, workspace_bytes, st);
    return rc != RTE_OK ? rc : guard_check(p, st, {{G, p.Nq * p.Nd * p.K}});
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_adjoint(rte_plan* h, const void* mu_a, const void* mu_s, const double* G_bar, double* dmu_a, double* dmu_s,
                void* workspace, int64_t workspace_bytes, void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(G_bar, "G_bar") ||
      !nonnull(dmu_a, "dmu_a") || !nonnull(dmu_s, "dmu_s") || !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = run_adjoint(p, mu_a, mu_s, G_bar, dmu_a, dmu_s, workspace, workspace_bytes, st);
    return rc != RTE_OK ? rc : guard_check(p, st, {{dmu_a, p.nx * p.ny}, {dmu_s, p.nx * p.ny}});
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_gradient(rte_plan* h, const void* mu_a, const void* mu_s, const double* G_meas, double* J, double* dmu_a,
                 double* dmu_s, double* G, void* workspace, int64_t workspace_bytes, void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(G_meas, "G_meas") ||
      !nonnull(J, "J") || !nonnull(dmu_a, "dmu_a") || !nonnull(dmu_s, "dmu_s") || !nonnull(G, "G") ||
      !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    GradArgs a{mu_a, mu_s, G_meas, J, dmu_a, dmu_s, G, workspace, workspace_bytes};
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = p.use_graph ? graph_gradient(p, a, st) : enqueue_gradient(p, a, st);
    return rc != RTE_OK ? rc : guard_check(p, st, grad_outputs(p, a));
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_gradient_ops(const rte_plan* h, int64_t* n_ops) {
  if (!nonnull(h, "plan") || !nonnull(n_ops, "n_ops")) return RTE_EINVAL;
  *n_ops = gradient_op_count(*reinterpret_cast<const Plan*>(h));
  return RTE_OK;
}

int rte_gradient_range(rte_plan* h, const void* mu_a, const void* mu_s, const double* G_meas, double* J,
                       double* dmu_a, double* dmu_s, double* G, void* workspace, int64_t workspace_bytes,
                       int64_t first, int64_t last, void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(G_meas, "G_meas") ||
      !nonnull(J, "J") || !nonnull(dmu_a, "dmu_a") || !nonnull(dmu_s, "dmu_s") || !nonnull(G, "G") ||
      !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    const int64_t total = gradient_op_count(p);
    if (first < 0 || last < first || last > total) {
      std::ostringstream o;
      o << "op range [" << first << ", " << last << ") outside [0, " << total << "]";
      set_error(o.str());
      return RTE_EINVAL;
    }
    const void* key[9] = {mu_a, mu_s, G_meas, J, dmu_a, dmu_s, G, workspace,
                          reinterpret_cast<const void*>(workspace_bytes)};
    if (first == 0) {
      for (int k = 0; k < 9; ++k) p.range_key[k] = key[k];
      p.range_next = 0;
    } else {
      if (first != p.range_next) {
        set_error("op ranges of one gradient must be enqueued in order, starting at 0");
        return RTE_ESTATE;
      }
      for (int k = 0; k < 9; ++k)
        if (p.range_key[k] != key[k]) {
          set_error("op ranges of one gradient must pass the same arguments");
          return RTE_ESTATE;
        }
    }
    GradArgs a{mu_a, mu_s, G_meas, J, dmu_a, dmu_s, G, workspace, workspace_bytes};
    hipStream_t st = static_cast<hipStream_t>(stream);
    p.range_next = -1;
    int rc = enqueue_gradient_ops(p, a, st, first, last, nullptr);
    if (rc != RTE_OK) return rc;
    p.range_next = last < total ? last : -1;
    return last == total ? guard_check(p, st, grad_outputs(p, a)) : RTE_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

static bool separable_ok(const rte_separable& f, const char* what) {
  if (f.rank < 0) {
    set_error(std::string(what) + ".rank must be >= 0");
    return false;
  }
  if (f.rank > 0 && (!f.X || !f.Y || !f.Th)) {
    set_error(std::string(what) + ": X, Y and Th are required when rank > 0");
    return false;
  }
  return true;
}

int rte_forward_ex(rte_plan* h, const void* mu_a, const void* mu_s, const rte_forward_extra* extra, double* G,
                   void* u_final, void* workspace, int64_t workspace_bytes, void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(extra, "extra") ||
      !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  if (!separable_ok(extra->source, "source") || !separable_ok(extra->inflow, "inflow")) return RTE_EINVAL;
  if (extra->n_snap < 0 || (extra->n_snap > 0 && (!extra->snap_steps || !extra->snap_flux))) {
    set_error("n_snap must be >= 0, with snap_steps and snap_flux when positive");
    return RTE_EINVAL;
  }
  const int64_t K = reinterpret_cast<Plan*>(h)->K;
  for (int k = 0; k < extra->n_snap; ++k)
    if (extra->snap_steps[k] < 0 || extra->snap_steps[k] > K) {
      set_error("snap_steps entries must lie in [0, K]");
      return RTE_EINVAL;
    }
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = run_forward_ex(p, mu_a, mu_s, extra, G, u_final, workspace, workspace_bytes, st);
    return rc != RTE_OK ? rc
                        : guard_check(p, st, {{G, p.Nq * p.Nd * p.K},
                                              {extra->snap_flux, p.Nq * extra->n_snap * p.nx * p.ny}});
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_gradient_continuous(rte_plan* h, const void* mu_a, const void* mu_s, const double* G_meas, double* J,
                            double* dmu_a, double* dmu_s, double* G, void* workspace, int64_t workspace_bytes,
                            void* stream) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(G_meas, "G_meas") ||
      !nonnull(J, "J") || !nonnull(dmu_a, "dmu_a") || !nonnull(dmu_s, "dmu_s") || !nonnull(G, "G") ||
      !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    Plan& p = *reinterpret_cast<Plan*>(h);
    GradArgs a{mu_a, mu_s, G_meas, J, dmu_a, dmu_s, G, workspace, workspace_bytes};
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = enqueue_gradient_continuous(p, a, st);
    return rc != RTE_OK ? rc : guard_check(p, st, grad_outputs(p, a));
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_plan_set_graph(rte_plan* h, int enable) {
  if (!nonnull(h, "plan")) return RTE_EINVAL;
  Plan& p = *reinterpret_cast<Plan*>(h);
  p.use_graph = enable != 0;
  if (!p.use_graph && p.gexec) {
    RTE_CHECK(hipGraphExecDestroy(p.gexec));
    p.gexec = nullptr;
  }
  return RTE_OK;
}

int rte_plan_get_schedule(const rte_plan* h, rte_schedule* out) {
  if (!nonnull(h, "plan") || !nonnull(out, "out")) return RTE_EINVAL;
  *out = reinterpret_cast<const Plan*>(h)->sched;
  return RTE_OK;
}

int rte_plan_set_schedule(rte_plan* h, const rte_schedule* sched) {
  if (!nonnull(h, "plan") || !nonnull(sched, "sched")) return RTE_EINVAL;
  Plan& p = *reinterpret_cast<Plan*>(h);
  rte_schedule s = *sched;
  if (s.line_units_per_wave == 0) s.line_units_per_wave = 1;
  if (s.line_waves_per_unit == 0) s.line_waves_per_unit = 2;
  if (s.node_tiles_per_block == 0) s.node_tiles_per_block = node_tiles_default(p);
  if (!sched_ok(p, s)) {
    std::ostringstream o;
    o << "schedule out of range: line_units_per_wave " << s.line_units_per_wave << ", line_waves_per_unit "
      << s.line_waves_per_unit << ", line_generic " << s.line_generic << ", line_global_tables "
      << s.line_global_tables << ", node_tiles_per_block " << s.node_tiles_per_block << " (M = " << p.M << ")";
    set_error(o.str());
    return RTE_EINVAL;
  }
  p.sched = s;
  ++p.sched_version;
  return RTE_OK;
}

int rte_plan_time_kernels(rte_plan* h, const void* mu_a, const void* mu_s, void* workspace, int64_t workspace_bytes,
                          void* stream, int reps, double* us) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(workspace, "workspace") ||
      !nonnull(us, "us"))
    return RTE_EINVAL;
  if (reps < 1 || reps > 10000) {
    set_error("reps must be in [1, 10000]");
    return RTE_EINVAL;
  }
  try {
    set_error("");
    return time_kernels(*reinterpret_cast<Plan*>(h), mu_a, mu_s, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream), reps, us);
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_plan_autotune(rte_plan* h, const void* mu_a, const void* mu_s, void* workspace, int64_t workspace_bytes,
                      void* stream, rte_schedule* chosen) {
  if (!nonnull(h, "plan") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(workspace, "workspace"))
    return RTE_EINVAL;
  try {
    set_error("");
    return autotune(*reinterpret_cast<Plan*>(h), mu_a, mu_s, workspace, workspace_bytes,
                    static_cast<hipStream_t>(stream), chosen);
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_batch_create(rte_plan* const* plans, int64_t n, rte_batch** out) {
  if (!nonnull(plans, "plans") || !nonnull(out, "out")) return RTE_EINVAL;
  *out = nullptr;
  if (n < 1 || n > 1024) {
    set_error("batch size must be in [1, 1024]");
    return RTE_EINVAL;
  }
  Batch* b = new Batch();
  for (int64_t i = 0; i < n; ++i) {
    if (!plans[i]) {
      delete b;
      set_error("plan entry is NULL");
      return RTE_EINVAL;
    }
    b->plans.push_back(reinterpret_cast<Plan*>(plans[i]));
  }
  *out = reinterpret_cast<rte_batch*>(b);
  return RTE_OK;
}

int rte_batch_destroy(rte_batch* h) {
  if (!h) return RTE_OK;
  Batch* b = reinterpret_cast<Batch*>(h);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->s0) (void)hipStreamDestroy(b->s0);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  delete b;
  return RTE_OK;
}

int rte_batch_gradient(rte_batch* h, const void* const* mu_a, const void* const* mu_s, const double* const* G_meas,
                       double* const* J, double* const* dmu_a, double* const* dmu_s, double* const* G,
                       void* const* workspaces, const int64_t* ws_bytes, void* stream) {
  if (!nonnull(h, "batch") || !nonnull(mu_a, "mu_a") || !nonnull(mu_s, "mu_s") || !nonnull(G_meas, "G_meas") ||
      !nonnull(J, "J") || !nonnull(dmu_a, "dmu_a") || !nonnull(dmu_s, "dmu_s") || !nonnull(G, "G") ||
      !nonnull(workspaces, "workspaces") || !nonnull(ws_bytes, "ws_bytes"))
    return RTE_EINVAL;
  try {
    set_error("");
    Batch& b = *reinterpret_cast<Batch*>(h);
    const size_t n = b.plans.size();
    std::vector<GradArgs> args(n);
    std::vector<const void*> key;
    for (size_t i = 0; i < n; ++i) {
      args[i] = GradArgs{mu_a[i], mu_s[i], G_meas[i], J[i], dmu_a[i], dmu_s[i], G[i], workspaces[i], ws_bytes[i]};
      if (!args[i].mu_a || !args[i].mu_s || !args[i].G_meas || !args[i].J || !args[i].dmu_a || !args[i].dmu_s ||
          !args[i].G || !args[i].ws) {
        set_error("a pointer of batch entry " + std::to_string(i) + " is NULL");
        return RTE_EINVAL;
      }
      const void* k[10] = {args[i].mu_a, args[i].mu_s, args[i].G_meas, args[i].J, args[i].dmu_a, args[i].dmu_s,
                           args[i].G, args[i].ws, reinterpret_cast<const void*>(args[i].wsb),
                           reinterpret_cast<const void*>(b.plans[i]->sched_version)};
      key.insert(key.end(), k, k + 10);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!b.gexec || key != b.key) {
      if (b.gexec) {
        RTE_CHECK(hipGraphExecDestroy(b.gexec));
        b.gexec = nullptr;
      }
      if (!b.s0) RTE_CHECK(hipStreamCreateWithFlags(&b.s0, hipStreamNonBlocking));
      while (b.streams.size() < n) {
        hipStream_t s;
        RTE_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b.streams.push_back(s);
      }
      while (b.events.size() < n + 1) {
        hipEvent_t e;
        RTE_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b.events.push_back(e);
      }
      // one captured graph: fork one branch per instance, join at the end
      RTE_CHECK(hipStreamBeginCapture(b.s0, hipStreamCaptureModeThreadLocal));
      int rc = RTE_OK;
      hipError_t e = hipEventRecord(b.events[n], b.s0);
      for (size_t i = 0; i < n && rc == RTE_OK && e == hipSuccess; ++i) {
        e = hipStreamWaitEvent(b.streams[i], b.events[n], 0);
        if (e != hipSuccess) break;
        const bool prof = b.plans[i]->prof;
        b.plans[i]->prof = false;
        rc = enqueue_gradient(*b.plans[i], args[i], b.streams[i]);
        b.plans[i]->prof = prof;
        if (rc != RTE_OK) break;
        e = hipEventRecord(b.events[i], b.streams[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b.s0, b.events[i], 0);
      }
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(b.s0, &graph);
      if (rc != RTE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      RTE_CHECK(e);
      RTE_CHECK(ec);
      const hipError_t ei = hipGraphInstantiate(&b.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      RTE_CHECK(ei);
      b.key = key;
    }
    RTE_CHECK(hipGraphLaunch(b.gexec, st));
    for (size_t i = 0; i < n; ++i) mark_saved(*b.plans[i], args[i].ws);
    for (size_t i = 0; i < n; ++i)
      if (int rc = guard_check(*b.plans[i], st, grad_outputs(*b.plans[i], args[i]))) return rc;
    return RTE_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RTE_EINVAL;
  }
}

int rte_plan_set_guard(rte_plan* h, int enable) {
  if (!nonnull(h, "plan")) return RTE_EINVAL;
  reinterpret_cast<Plan*>(h)->guard = enable != 0;
  return RTE_OK;
}

int rte_profile_enable(rte_plan* h, int enable) {
  if (!nonnull(h, "plan")) return RTE_EINVAL;
  Plan& p = *reinterpret_cast<Plan*>(h);
  p.prof = enable != 0;
  if (!p.prof)
    for (int c = 0; c < RTE_K_COUNT; ++c) {
      for (auto& e : p.ev_rec[c]) {
        p.ev_pool.push_back(e.first);
        p.ev_pool.push_back(e.second);
      }
      p.ev_rec[c].clear();
    }
  return RTE_OK;
}

int rte_profile_read(rte_plan* h, double* total_ms, int64_t* launches) {
  if (!nonnull(h, "plan") || !nonnull(total_ms, "total_ms") || !nonnull(launches, "launches")) return RTE_EINVAL;
  Plan& p = *reinterpret_cast<Plan*>(h);
  for (int c = 0; c < RTE_K_COUNT; ++c) {
    double tot = 0.0;
    for (auto& e : p.ev_rec[c]) {
      RTE_CHECK(hipEventSynchronize(e.second));
      float ms = 0.f;
      RTE_CHECK(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
    }
    total_ms[c] = tot;
    launches[c] = (int64_t)p.ev_rec[c].size();
    for (auto& e : p.ev_rec[c]) {
      p.ev_pool.push_back(e.first);
      p.ev_pool.push_back(e.second);
    }
    p.ev_rec[c].clear();
  }
  return RTE_OK;
}

const char* rte_last_error(void) { return last_error(); }

}  // extern "C"
