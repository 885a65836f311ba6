// Host-side plan: every table the kernels read, computed once in FP64.
//
//   ordinates ........ Sec. 4.1 eq. (RTETrapz): theta_m = 2 pi m / M, stored in
//                      reflection-orbit order (slots 4g..4g+3 = m, M/2-m, -m, M/2+m)
//   HG matrix ........ Sec. 2 eq. (Henyey-Greeinstein) normalised as in Sec. 4.1
//   Fresnel / BC ..... Sec. 2 eq. (RTE): reflection theta_r = 2 theta_nu - theta + pi,
//                      unpolarised Fresnel reflectance from Snell's law, corner rule
//   beams ............ Sec. 3.1 eq. (RTEsources2) with the window eq. (sourcelabwind)
//   detectors ........ Sec. 3.1 eq. (OpMed): trapezoid along walls, outgoing ordinates
//   FC derivative .... Sec. 4.3: E rule (N_p 5-smooth), filtered multiplier
//                      eqs. (FFilter)/(RTEFCSumder) with period N_p h, FFT radix plan
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "fc_table_d5_C25.h"
#include "rte_internal.h"

namespace rte {

static const double kPi = 3.14159265358979323846;

thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------- small math
static double window_fn(double v) {
  v = std::fabs(v);
  if (v == 0.0) return 1.0;
  if (v >= 1.0) return 0.0;
  return std::exp(2.0 * std::exp(-1.0 / v) / (v - 1.0));
}

static double fresnel_r(double cos_i, double n1, double n2) {
  if (n1 == n2) return 0.0;
  cos_i = std::min(std::max(cos_i, 0.0), 1.0);
  const double sin_i = std::sqrt(std::max(0.0, 1.0 - cos_i * cos_i));
  const double sin_t = n1 / n2 * sin_i;
  if (sin_t >= 1.0) return 1.0;
  const double cos_t = std::sqrt(1.0 - sin_t * sin_t);
  const double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
  const double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

// exact signs of cos / sin of 2 pi m / M
static int sgn_cos(int m, int M) {
  const long r = (4L * m) % (4L * M);
  if (r == M || r == 3L * M) return 0;
  return (r < M || r > 3L * M) ? 1 : -1;
}
static int sgn_sin(int m, int M) {
  const long r = (2L * m) % (2L * M);
  if (r == 0 || r == M) return 0;
  return r < M ? 1 : -1;
}
// +1: |cos| > |sin|, -1: smaller, 0: equal
static int x_dominant(int m, int M) {
  const int h = m % (M / 2);
  if (8L * h == M || 8L * h == 3L * M) return 0;
  return (8L * h < M || 8L * h > 3L * M) ? 1 : -1;
}

struct WallDesc {
  bool xwall;
  double nx, ny;
};
static const WallDesc kWalls[4] = {{true, -1, 0}, {true, 1, 0}, {false, 0, -1}, {false, 0, 1}};

static int wall_sign(int w, int m, int M) {
  return kWalls[w].xwall ? sgn_cos(m, M) * (int)kWalls[w].nx : sgn_sin(m, M) * (int)kWalls[w].ny;
}
static double wall_dot(int w, int m, int M) {
  const double th = 2.0 * kPi * m / M;
  return std::cos(th) * kWalls[w].nx + std::sin(th) * kWalls[w].ny;
}
static int wall_reflect(int w, int m, int M) {
  return kWalls[w].xwall ? ((M / 2 - m) % M + M) % M : ((M - m) % M);
}

static bool smooth5(int64_t n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// ---------------------------------------------------------------- device upload helper
template <typename V>
static bool upload(const std::vector<V>& h, V** d) {
  if (h.empty()) {
    *d = nullptr;
    return true;
  }
  if (hipMalloc((void**)d, h.size() * sizeof(V)) != hipSuccess) return false;
  return hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice) == hipSuccess;
}

// ---------------------------------------------------------------- FC plan for one direction
static bool build_fc(const rte_problem& pb, int n, double h, std::vector<double>& buf, FcPlanDev& fc,
                     std::vector<size_t>& offs) {
  const int d = (int)pb.fc_d, C = (int)pb.fc_C;
  int E = 0;
  while (!smooth5(n + C + E)) ++E;
  const int Np = n + C + E;
  fc.n = n;
  fc.Np = Np;
  fc.E = E;
  fc.d = d;
  fc.C = C;
  // radix plan: 4s first, then 2, 3, 5
  int m = Np, np = 0;
  std::vector<int> rad;
  while (m % 4 == 0) { rad.push_back(4); m /= 4; }
  while (m % 2 == 0) { rad.push_back(2); m /= 2; }
  while (m % 3 == 0) { rad.push_back(3); m /= 3; }
  while (m % 5 == 0) { rad.push_back(5); m /= 5; }
  if ((int)rad.size() > kMaxPasses) return false;
  // twiddles
  size_t off0 = buf.size();
  offs.push_back(off0);
  int Ns = 1, tw_count = 0;
  std::vector<double> tw;
  for (int R : rad) {
    fc.radix[np] = R;
    fc.ns[np] = Ns;
    fc.twoff[np] = tw_count;
    for (int k = 0; k < Ns; ++k)
      for (int t = 1; t < R; ++t) {
        const long a = ((long)t * k) % ((long)Ns * R);
        const double ang = -2.0 * kPi * (double)a / (double)(Ns * R);
        tw.push_back(std::cos(ang));
        tw.push_back(std::sin(ang));
        ++tw_count;
      }
    Ns *= R;
    ++np;
  }
  fc.npass = np;
  buf.insert(buf.end(), tw.begin(), tw.end());
  // multipliers: derivative factor 2 pi kappa / (Np h), filter, 1/Np, zero Nyquist
  offs.push_back(buf.size());
  for (int k = 0; k < Np; ++k) {
    const double kap = (k <= Np / 2) ? (double)k : (double)(k - Np);
    double mu = 2.0 * kPi * kap / (Np * h) * std::exp(-pb.filt_alpha * std::pow(std::fabs(2.0 * kap / Np), 2.0 * pb.filt_beta));
    if (Np % 2 == 0 && k == Np / 2) mu = 0.0;
    buf.push_back(mu / Np);
  }
  offs.push_back(buf.size());
  for (int i = 0; i < d * d; ++i) buf.push_back(pb.fc_Q[i]);
  offs.push_back(buf.size());
  for (int i = 0; i < C * d; ++i) buf.push_back(pb.fc_A[i]);
  // roots of unity for the four-step kernel
  offs.push_back(buf.size());
  for (int e = 0; e < Np; ++e) {
    const double ang = -2.0 * kPi * (double)e / (double)Np;
    buf.push_back(std::cos(ang));
    buf.push_back(std::sin(ang));
  }
  // continuation matrix (Sec. 4.3 steps 1-4 as one linear map): extension
  // value p (0 <= p < C + E) = sum_k MR[p][k] g[n-d+k] + sum_k ML[p][k] g[d-1-k]
  // with MR[p][k] = sum_j A[p][j] Q[k][j] (p < C) and
  //      ML[p][k] = sum_j A[C+E-1-p][j] Q[k][j] (p >= E); row p = [MR | ML]
  offs.push_back(buf.size());
  const int CE = C + E;
  for (int p = 0; p < CE; ++p) {
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < d; ++k) {
        long double acc = 0.0L;
        const int row = side == 0 ? p : CE - 1 - p;
        const bool on = side == 0 ? (p < C) : (p >= E);
        if (on)
          for (int j = 0; j < d; ++j) acc += (long double)pb.fc_A[row * d + j] * (long double)pb.fc_Q[k * d + j];
        buf.push_back((double)acc);
      }
  }
  // the extension values are formed by one thread each (CE <= 64); the
  // transpose keeps its 2d fold values in the C+E extension positions
  if (!fourstep_split(Np, &fc.n1, &fc.n2) || CE > 64 || CE < 2 * d) fc.n1 = fc.n2 = 0;
  return true;
}

// ---------------------------------------------------------------- validation
static bool validate(const rte_problem* p, const rte_beam* beams, int64_t nbm, const rte_detector* dets,
                     int64_t nd) {
  std::ostringstream e;
  if (!p) e << "problem is NULL";
  else if (p->dtype != RTE_F64 && p->dtype != RTE_F32) e << "dtype must be RTE_F64 or RTE_F32";
  else if (p->M < 4 || p->M % 4) e << "M must be a positive multiple of 4 (got " << p->M << ")";
  else if (p->M > 256) e << "M > 256 is not supported";
  else if (p->fc_d < 2 || p->fc_d > kMaxFcD) e << "fc_d must be in [2, " << kMaxFcD << "]";
  else if (p->fc_C < 1) e << "fc_C must be positive";
  else if (p->Nx + 1 < 2 * p->fc_d || p->Ny + 1 < 2 * p->fc_d) e << "each side needs at least 2*fc_d nodes";
  else if (p->Nx > 8192 || p->Ny > 8192) e << "Nx, Ny must be <= 8192";
  else if (p->K < 1) e << "K must be >= 1";
  else if (!(p->xmax > p->xmin) || !(p->ymax > p->ymin)) e << "empty domain";
  else if (!(p->dt > 0) || !(p->c > 0)) e << "dt and c must be positive";
  else if (!(std::fabs(p->g) < 1.0)) e << "|g| must be < 1";
  else if (!(p->n_in > 0) || !(p->n_out > 0)) e << "refractive indices must be positive";
  else if (!p->fc_Q != !p->fc_A) e << "fc_Q and fc_A must be given together (or both NULL)";
  else if (p->ckpt_every < 0) e << "ckpt_every must be >= 0";
  else if (p->combo_chunk < 0) e << "combo_chunk must be >= 0";
  else if (nbm < 0 || (nbm > 0 && !beams)) e << "bad beam array";
  else if (nd < 0 || (nd > 0 && !dets)) e << "bad detector array";
  if (e.str().empty()) {
    // AB4 is stable on the imaginary axis up to |lambda| = 0.43; the spectral
    // advection -c (xi D_x + eta D_y) has eigenvalues up to
    // c pi sqrt(1/dx^2 + 1/dy^2) in magnitude (the stiff part c (a + b)
    // depends on the maps passed to each call and is left to the caller)
    const double dx = (p->xmax - p->xmin) / (double)p->Nx, dy = (p->ymax - p->ymin) / (double)p->Ny;
    const double lam = p->c * p->dt * kPi * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy));
    if (lam > 0.43)
      e << "dt beyond the AB4 stability limit of the advection: c dt pi sqrt(1/dx^2 + 1/dy^2) = " << lam
        << " > 0.43";
  }
  // beams and detectors sit on the boundary (Sec. 2.1): within 1e-9 of the
  // domain size of one side, and inside the side's extent
  auto on_boundary = [&](double x, double y) {
    const double tol = 1e-9 * std::max(p->xmax - p->xmin, p->ymax - p->ymin);
    const bool in_x = x >= p->xmin - tol && x <= p->xmax + tol, in_y = y >= p->ymin - tol && y <= p->ymax + tol;
    return in_x && in_y &&
           (std::fabs(x - p->xmin) <= tol || std::fabs(x - p->xmax) <= tol || std::fabs(y - p->ymin) <= tol ||
            std::fabs(y - p->ymax) <= tol);
  };
  if (e.str().empty()) {
    for (int64_t k = 0; k < nbm; ++k)
      if (!on_boundary(beams[k].x, beams[k].y)) {
        e << "beam " << k << " is not on the boundary";
        break;
      }
    for (int64_t k = 0; k < nd && e.str().empty(); ++k)
      if (!on_boundary(dets[k].x, dets[k].y)) {
        e << "detector " << k << " is not on the boundary";
        break;
      }
  }
  if (e.str().empty()) {
    for (int64_t k = 0; k < nbm; ++k)
      if (beams[k].group < 0 || beams[k].group > 4096 || !(beams[k].sigma_x > 0) || !(beams[k].sigma_theta > 0) ||
          !(beams[k].sigma_t > 0)) {
        e << "beam " << k << " has a bad group or width";
        break;
      } else if (beams[k].profile != RTE_PROFILE_GAUSSIAN && beams[k].profile != RTE_PROFILE_WINDOW) {
        e << "beam " << k << " has an unknown temporal profile " << beams[k].profile;
        break;
      }
    for (int64_t k = 0; k < nd; ++k)
      if (!(dets[k].sigma_d > 0)) {
        e << "detector " << k << " has a non-positive width";
        break;
      }
  }
  if (!e.str().empty()) {
    set_error(e.str());
    return false;
  }
  return true;
}

static void free_tables(DeviceTables& t) {
  void* ps[] = {t.xi, t.eta, t.Wt, t.bc, t.bct, t.kappa, t.det_w, t.beam_sp, t.beam_an, t.beam_tt, t.beam_off,
                t.slot_m, t.fc_buf, t.det_sp, t.slot_rev, t.guard_flag};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  t = DeviceTables();
}

int plan_create(const rte_problem* prob, const rte_beam* beams, int64_t n_beams, const rte_detector* dets,
                int64_t n_det, rte_plan** out) {
  if (!out) {
    set_error("out is NULL");
    return RTE_EINVAL;
  }
  *out = nullptr;
  if (!validate(prob, beams, n_beams, dets, n_det)) return RTE_EINVAL;
  // FC table: the caller's, or the built-in one for (d, C) = (5, 25)
  rte_problem pbt = *prob;
  if (!prob->fc_Q) {
    if (prob->fc_d != kBuiltinFcD || prob->fc_C != kBuiltinFcC) {
      std::ostringstream o;
      o << "no built-in FC table for fc_d = " << prob->fc_d << ", fc_C = " << prob->fc_C
        << " (built in: " << kBuiltinFcD << ", " << kBuiltinFcC << "): pass fc_Q and fc_A";
      set_error(o.str());
      return RTE_EUNSUPPORTED;
    }
    pbt.fc_Q = kBuiltinFcQ;
    pbt.fc_A = kBuiltinFcA;
  }
  Plan* P = new Plan();
  Plan& p = *P;
  p.prob = *prob;
  p.prob.fc_Q = nullptr;
  p.prob.fc_A = nullptr;
  p.dtype = prob->dtype;
  p.nx = prob->Nx + 1;
  p.ny = prob->Ny + 1;
  p.M = prob->M;
  p.G = p.M / kGroup;
  p.Mpad = ((p.M + 15) / 16) * 16;
  {
    const int64_t align = (prob->dtype == RTE_F64) ? 4 : 8;  // nodes per 128 bytes of one group
    p.nxp = ((p.nx + align - 1) / align) * align;
    // a row pitch that is a multiple of 2 KB puts the rows of a node tile's
    // neighbourhood on few memory channels: pad such rows by 128 bytes
    const int64_t pitch = p.nxp * kGroup * (prob->dtype == RTE_F64 ? 8 : 4);
    if (pitch % 2048 == 0) p.nxp += align;
  }
  p.grp_stride = p.ny * p.nxp * kGroup;
  p.inst_stride = p.G * p.grp_stride;
  if (p.inst_stride * (prob->dtype == RTE_F64 ? 8 : 4) >= (int64_t(1) << 32)) {
    set_error("one source's state exceeds 4 GiB (ordinates x nodes too large)");
    delete P;
    return RTE_EUNSUPPORTED;
  }
  p.K = prob->K;
  p.Nd = n_det;
  p.nbeams = n_beams;
  p.nb = 2 * (p.nx + p.ny) - 4;
  p.npos = std::max(p.nx, p.ny);
  p.ckpt_every = prob->ckpt_every;
  int maxg = 0;
  for (int64_t k = 0; k < n_beams; ++k) maxg = std::max(maxg, beams[k].group);
  p.Nq = maxg + 1;
  p.chunk = (prob->combo_chunk > 0) ? std::min<int64_t>(prob->combo_chunk, p.Nq) : p.Nq;
  p.cq0 = 0;
  p.cnq = p.chunk;
  p.stream_nt = p.chunk * p.inst_stride * (prob->dtype == RTE_F64 ? 8 : 4) > kStreamNtBytes;
  const int M = (int)p.M;
  const double dx = (prob->xmax - prob->xmin) / prob->Nx;
  const double dy = (prob->ymax - prob->ymin) / prob->Ny;

  // ---- ordinate slots: orbit {m, M/2-m, -m, M/2+m}; last group {0, M/2, M/4, 3M/4}
  p.slot_m.resize(M);
  for (int g = 0; g + 1 < (int)p.G; ++g) {
    const int m = g + 1;
    p.slot_m[4 * g + 0] = m;
    p.slot_m[4 * g + 1] = M / 2 - m;
    p.slot_m[4 * g + 2] = M - m;
    p.slot_m[4 * g + 3] = M / 2 + m;
  }
  {
    const int g = (int)p.G - 1;
    p.slot_m[4 * g + 0] = 0;
    p.slot_m[4 * g + 1] = M / 2;
    p.slot_m[4 * g + 2] = M / 4;
    p.slot_m[4 * g + 3] = 3 * M / 4;
  }
  std::vector<int> slot_of(M);
  for (int s = 0; s < M; ++s) slot_of[p.slot_m[s]] = s;
  std::vector<double> xi(M), eta(M);
  for (int s = 0; s < M; ++s) {
    const double th = 2.0 * kPi * p.slot_m[s] / M;
    xi[s] = std::cos(th);
    eta[s] = std::sin(th);
  }

  // ---- HG matrix, normalised so each row sums to one, in slot order
  std::vector<double> pk(M);
  {
    const double g = prob->g;
    for (int k = 0; k <= M / 2; ++k) {
      const double mu = std::cos(2.0 * kPi * k / M);
      pk[k] = (1.0 - g * g) / std::pow(1.0 + g * g - 2.0 * g * mu, prob->hg_exponent);
    }
    for (int k = M / 2 + 1; k < M; ++k) pk[k] = pk[M - k];
    double sum = 0.0;
    for (int k = 0; k < M; ++k) sum += pk[k];
    for (int k = 0; k < M; ++k) pk[k] /= sum;
  }
  std::vector<double> Wt((size_t)p.Mpad * p.Mpad, 0.0);
  for (int s = 0; s < M; ++s)
    for (int t = 0; t < M; ++t) Wt[(size_t)s * p.Mpad + t] = pk[((p.slot_m[s] - p.slot_m[t]) % M + M) % M];

  // ---- boundary rules per node type (tx: 0 none, 1 xmin, 2 xmax; ty likewise)
  std::vector<BcRule> bc(9 * M);
  std::vector<BcRuleT> bct(9 * M);
  for (int ty = 0; ty < 3; ++ty)
    for (int tx = 0; tx < 3; ++tx) {
      const int type = tx + 3 * ty;
      int walls[2], nw = 0;
      if (tx) walls[nw++] = tx - 1;      // 0: xmin, 1: xmax
      if (ty) walls[nw++] = 2 + ty - 1;  // 2: ymin, 3: ymax
      for (int s = 0; s < M; ++s) {
        const int m = p.slot_m[s];
        BcRule r{};
        r.src_a = r.src_b = s;
        int inc[2], ni = 0;
        for (int t = 0; t < nw; ++t)
          if (wall_sign(walls[t], m, M) < 0) inc[ni++] = walls[t];
        if (ni == 2) {
          const int dom = x_dominant(m, M);
          const int xw = kWalls[inc[0]].xwall ? inc[0] : inc[1];
          const int yw = kWalls[inc[0]].xwall ? inc[1] : inc[0];
          if (dom > 0) { inc[0] = xw; ni = 1; }
          else if (dom < 0) { inc[0] = yw; ni = 1; }
        }
        if (ni >= 1) {
          r.flag = 1;
          const double f0 = fresnel_r(std::fabs(wall_dot(inc[0], m, M)), prob->n_in, prob->n_out);
          r.src_a = slot_of[wall_reflect(inc[0], m, M)];
          r.coef_a = f0 / ni;
          if (ni == 2) {
            const double f1 = fresnel_r(std::fabs(wall_dot(inc[1], m, M)), prob->n_in, prob->n_out);
            r.src_b = slot_of[wall_reflect(inc[1], m, M)];
            r.coef_b = f1 / 2;
          }
        }
        bc[type * M + s] = r;
      }
      for (int s = 0; s < M; ++s) {
        BcRuleT rt{};
        rt.is_target = bc[type * M + s].flag;
        for (int t = 0; t < M; ++t) {
          const BcRule& r = bc[type * M + t];
          if (!r.flag) continue;
          if (r.src_a == s && rt.ntgt < 2) { rt.tgt[rt.ntgt] = t; rt.coef[rt.ntgt] = r.coef_a; ++rt.ntgt; }
          if (r.coef_b != 0.0 && r.src_b == s && rt.ntgt < 2) { rt.tgt[rt.ntgt] = t; rt.coef[rt.ntgt] = r.coef_b; ++rt.ntgt; }
        }
        bct[type * M + s] = rt;
      }
    }

  // ---- node coordinates (same formula as the grid: xmin + i dx)
  auto xcoord = [&](int i) { return prob->xmin + dx * i; };
  auto ycoord = [&](int j) { return prob->ymin + dy * j; };

  // ---- detectors
  std::vector<double> kappa(4 * M, 0.0);
  for (int w = 0; w < 4; ++w)
    for (int s = 0; s < M; ++s) {
      const int m = p.slot_m[s];
      if (wall_sign(w, m, M) > 0) {
        const double dot = wall_dot(w, m, M);
        kappa[w * M + s] = (2.0 * kPi / M) * (1.0 - fresnel_r(std::fabs(dot), prob->n_in, prob->n_out)) * dot;
      }
    }
  std::vector<double> detw((size_t)n_det * 4 * p.npos, 0.0);
  for (int64_t jd = 0; jd < n_det; ++jd)
    for (int w = 0; w < 4; ++w) {
      const int len = kWalls[w].xwall ? (int)p.ny : (int)p.nx;
      const double ds = kWalls[w].xwall ? dy : dx;
      for (int pos = 0; pos < len; ++pos) {
        double xb, yb;
        if (w == 0) { xb = xcoord(0); yb = ycoord(pos); }
        else if (w == 1) { xb = xcoord((int)p.nx - 1); yb = ycoord(pos); }
        else if (w == 2) { xb = xcoord(pos); yb = ycoord(0); }
        else { xb = xcoord(pos); yb = ycoord((int)p.ny - 1); }
        const double om = (pos == 0 || pos == len - 1) ? 0.5 : 1.0;
        const double dist = std::hypot(xb - dets[jd].x, yb - dets[jd].y);
        detw[((size_t)jd * 4 + w) * p.npos + pos] = om * ds * window_fn(dist / dets[jd].sigma_d);
      }
    }

  // ---- continuous adjoint (eq. AdjointProblem): detector footprints at the
  // boundary positions (inflow source of the reversed problem) and the slot
  // of the reversed ordinate m + M/2 (pairs psi with u in the gradient)
  std::vector<double> detsp((size_t)std::max<int64_t>(n_det, 1) * p.nb, 0.0);
  for (int64_t jd = 0; jd < n_det; ++jd)
    for (int64_t bp = 0; bp < p.nb; ++bp) {
      int j, i;
      if (bp < p.nx) { j = 0; i = (int)bp; }
      else if (bp < 2 * p.nx) { j = (int)p.ny - 1; i = (int)(bp - p.nx); }
      else if (bp < 2 * p.nx + p.ny - 2) { i = 0; j = (int)(bp - 2 * p.nx + 1); }
      else { i = (int)p.nx - 1; j = (int)(bp - 2 * p.nx - (p.ny - 2) + 1); }
      const double dist = std::hypot(xcoord(i) - dets[jd].x, ycoord(j) - dets[jd].y);
      detsp[(size_t)jd * p.nb + bp] = window_fn(dist / dets[jd].sigma_d);
    }
  std::vector<int32_t> srev((size_t)p.Mpad);
  for (int s = 0; s < (int)p.Mpad; ++s) srev[s] = s < M ? slot_of[(p.slot_m[s] + M / 2) % M] : s;

  // ---- beams grouped per generalised source (CSR)
  std::vector<int> order(n_beams);
  for (int64_t k = 0; k < n_beams; ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return beams[a].group < beams[b].group; });
  std::vector<int32_t> boff(p.Nq + 1, 0);
  for (int64_t k = 0; k < n_beams; ++k) boff[beams[k].group + 1]++;
  for (int64_t q = 0; q < p.Nq; ++q) boff[q + 1] += boff[q];
  std::vector<double> bsp((size_t)n_beams * p.nb), ban((size_t)n_beams * M), btt((size_t)n_beams * (p.K + 1));
  for (int64_t kk = 0; kk < n_beams; ++kk) {
    const rte_beam& b = beams[order[kk]];
    for (int64_t bp = 0; bp < p.nb; ++bp) {
      int j, i;
      if (bp < p.nx) { j = 0; i = (int)bp; }
      else if (bp < 2 * p.nx) { j = (int)p.ny - 1; i = (int)(bp - p.nx); }
      else if (bp < 2 * p.nx + p.ny - 2) { i = 0; j = (int)(bp - 2 * p.nx + 1); }
      else { i = (int)p.nx - 1; j = (int)(bp - 2 * p.nx - (p.ny - 2) + 1); }
      const double r2 = (xcoord(i) - b.x) * (xcoord(i) - b.x) + (ycoord(j) - b.y) * (ycoord(j) - b.y);
      bsp[(size_t)kk * p.nb + bp] = std::exp(-r2 / (2.0 * b.sigma_x * b.sigma_x));
    }
    for (int s = 0; s < M; ++s) {
      const double th = 2.0 * kPi * p.slot_m[s] / M;
      double dd = std::fabs(std::fmod(th - b.theta, 2.0 * kPi));
      dd = std::min(dd, 2.0 * kPi - dd);
      ban[(size_t)kk * M + s] = window_fn(dd / b.sigma_theta);
    }
    // temporal profile T(t - tau) of eq. (RTEsources2): Gaussian, or the
    // window of eq. (sourcelabwind) in |t - t_s| / sigma_t as in eq. (sourcelab)
    for (int64_t n = 0; n <= p.K; ++n) {
      const double dtt = n * prob->dt - b.tau - b.t0;
      btt[(size_t)kk * (p.K + 1) + n] = b.profile == RTE_PROFILE_WINDOW
                                            ? window_fn(dtt / b.sigma_t)
                                            : std::exp(-(dtt * dtt) / (2.0 * b.sigma_t * b.sigma_t));
    }
  }

  // ---- FC plans
  std::vector<double> fcbuf;
  std::vector<size_t> ox, oy;
  if (!build_fc(pbt, (int)p.nx, dx, fcbuf, p.fcx, ox) || !build_fc(pbt, (int)p.ny, dy, fcbuf, p.fcy, oy)) {
    set_error("FC extended length needs too many FFT passes");
    delete P;
    return RTE_EUNSUPPORTED;
  }
  if (line_shmem_bytes(std::max(p.fcx.Np, p.fcy.Np), p.dtype) > 160 * 1024) {
    set_error("lines too long for the LDS line pass");
    delete P;
    return RTE_EUNSUPPORTED;
  }

  p.sched.node_tiles_per_block = node_tiles_default(p);
  p.fc_same = p.fcx.n == p.fcy.n && p.fcx.Np == p.fcy.Np && p.fcx.E == p.fcy.E &&
              std::equal(fcbuf.begin() + ox[1], fcbuf.begin() + ox[2], fcbuf.begin() + oy[1]);

  // ---- upload
  std::vector<int32_t> slotm(p.slot_m.begin(), p.slot_m.end());
  bool ok = upload(xi, &p.dev.xi) && upload(eta, &p.dev.eta) && upload(Wt, &p.dev.Wt) && upload(bc, &p.dev.bc) &&
            upload(bct, &p.dev.bct) && upload(kappa, &p.dev.kappa) && upload(detw, &p.dev.det_w) &&
            upload(bsp, &p.dev.beam_sp) && upload(ban, &p.dev.beam_an) && upload(btt, &p.dev.beam_tt) &&
            upload(boff, &p.dev.beam_off) && upload(slotm, &p.dev.slot_m) && upload(fcbuf, &p.dev.fc_buf) &&
            upload(detsp, &p.dev.det_sp) && upload(srev, &p.dev.slot_rev) &&
            upload(std::vector<unsigned long long>(1, 0ull), &p.dev.guard_flag);
  if (!ok) {
    set_error("device allocation or upload of the plan tables failed");
    free_tables(p.dev);
    delete P;
    return RTE_EDEVICE;
  }
  const double* fb = p.dev.fc_buf;
  p.fcx.tw = fb + ox[0]; p.fcx.mu = fb + ox[1]; p.fcx.Q = fb + ox[2]; p.fcx.A = fb + ox[3]; p.fcx.roots = fb + ox[4];
  p.fcy.tw = fb + oy[0]; p.fcy.mu = fb + oy[1]; p.fcy.Q = fb + oy[2]; p.fcy.A = fb + oy[3]; p.fcy.roots = fb + oy[4];
  p.fcx.Mx = fb + ox[5];
  p.fcy.Mx = fb + oy[5];
  *out = reinterpret_cast<rte_plan*>(P);
  return RTE_OK;
}

int plan_destroy(rte_plan* h) {
  if (!h) return RTE_OK;
  Plan* p = reinterpret_cast<Plan*>(h);
  free_tables(p->dev);
  for (int c = 0; c < RTE_K_COUNT; ++c)
    for (auto& e : p->ev_rec[c]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
  return RTE_OK;
}

static hipError_t take_event(Plan& p, hipEvent_t* e) {
  if (!p.ev_pool.empty()) {
    *e = p.ev_pool.back();
    p.ev_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

hipError_t prof_begin(Plan& p, int cls, hipStream_t s, hipEvent_t* stop) {
  *stop = nullptr;
  if (!p.prof) return hipSuccess;
  hipEvent_t a, b;
  hipError_t e = take_event(p, &a);
  if (e != hipSuccess) return e;
  e = take_event(p, &b);
  if (e != hipSuccess) return e;
  p.ev_rec[cls].push_back({a, b});
  *stop = b;
  return hipEventRecord(a, s);
}

hipError_t prof_end(hipEvent_t stop, hipStream_t s) { return stop ? hipEventRecord(stop, s) : hipSuccess; }

// ---------------------------------------------------------------- workspace
int64_t state_elems(const Plan& p) { return p.chunk * p.inst_stride; }

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

int64_t state_stride_bytes(const Plan& p) {
  const int64_t es = (p.dtype == RTE_F64) ? 8 : 4;
  return align256(state_elems(p) * es);
}

struct Layout {
  int64_t states, ckpts, work_u, lring, tx, ty, vring, atx, aty, ap1, flux, ga, gb, gbar, scratch, total;
};

// Forward: lring[3], tx, ty.  Adjoint: vring[4], w (aliases tx), the carries
// atx, aty, ap1.  With every state kept no forward step runs during the
// adjoint, so vring[0..2] alias the L ring and atx aliases ty; with
// checkpoints the segment replays need the forward arrays while the adjoint
// ring and carries are live, so those are separate.
static Layout layout(const Plan& p, bool adj) {
  const int64_t S = state_stride_bytes(p);
  const bool ck = p.ckpt_every > 0;
  const int64_t s = p.ckpt_every;
  Layout L{};
  int64_t o = 0;
  L.states = o;
  if (adj) o += ck ? (s + 1) * S : (p.K + 1) * S;
  L.ckpts = o;
  if (adj && ck) o += ((p.K + s - 1) / s) * 4 * S;
  L.work_u = o;
  if (!adj || ck) o += 2 * S;
  L.lring = o;
  o += 3 * S;
  L.tx = o;
  o += S;
  L.ty = o;
  o += S;
  L.vring = o;
  if (adj) o += ck ? 4 * S : S;
  L.atx = o;
  if (adj && ck) o += S;
  L.aty = o;
  if (adj) o += S;
  L.ap1 = o;
  if (adj) o += S;
  L.flux = o;
  o += align256(p.Nq * (p.K + 1) * 4 * p.npos * 8);
  L.ga = o;
  o += adj ? align256(p.Nq * p.nx * p.ny * 8) : 0;
  L.gb = o;
  o += adj ? align256(p.Nq * p.nx * p.ny * 8) : 0;
  L.gbar = o;
  o += adj ? align256(p.Nq * p.Nd * p.K * 8) : 0;
  L.scratch = o;
  o += 256;
  L.total = o;
  return L;
}

int64_t workspace_bytes(const Plan& p, bool adj) { return layout(p, adj).total; }

bool map_workspace(const Plan& p, void* base, int64_t bytes, bool adj, Workspace* ws) {
  const Layout L = layout(p, adj);
  if (!base || bytes < L.total) return false;
  const int64_t S = state_stride_bytes(p);
  char* b = static_cast<char*>(base);
  ws->base = b;
  ws->bytes = bytes;
  ws->states = adj ? b + L.states : nullptr;
  ws->ckpts = (adj && p.ckpt_every > 0) ? b + L.ckpts : nullptr;
  if (!adj || p.ckpt_every > 0) {
    ws->work_u[0] = b + L.work_u;
    ws->work_u[1] = b + L.work_u + S;
  }
  for (int k = 0; k < 3; ++k) ws->lring[k] = b + L.lring + k * S;
  ws->tx = b + L.tx;
  ws->ty = b + L.ty;
  if (adj) {
    const bool ck = p.ckpt_every > 0;
    if (ck) {
      for (int k = 0; k < 4; ++k) ws->vring[k] = b + L.vring + k * S;
      ws->atx = b + L.atx;
    } else {
      for (int k = 0; k < 3; ++k) ws->vring[k] = ws->lring[k];
      ws->vring[3] = b + L.vring;
      ws->atx = ws->ty;
    }
    ws->wbuf = ws->tx;
    ws->aty = b + L.aty;
    ws->ap1 = b + L.ap1;
    ws->ga = reinterpret_cast<double*>(b + L.ga);
    ws->gb = reinterpret_cast<double*>(b + L.gb);
    ws->gbar = reinterpret_cast<double*>(b + L.gbar);
  }
  ws->flux = reinterpret_cast<double*>(b + L.flux);
  ws->scratch = reinterpret_cast<double*>(b + L.scratch);
  return true;
}

}  // namespace rte
