// vs_host.cpp -- host side of the C ABI (include/vinesim.h): validation, the
// create-time sPAM force-law table (Sec. 3.1, Eq. 1 solved for G = F_t / P_act),
// the wrinkling-energy table (Sec. 3.2), device allocation and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vinesim.h"
#include "vs_device.h"

namespace vs {
hipError_t launch_rollout(const KParams& P, const KData& D, int n_steps, int record_traj,
                          int nmax_class, hipStream_t stream);
hipError_t launch_grad(const KParams& P, const KData& D, const double* goal,
                       const double* weights, int T, double* dP, double* ds0, double* ds1,
                       double* loss, int* status, int nmax_class, hipStream_t stream);
}

using vs::SpamTable;
using vs::WrTable;

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Gauss-Legendre rules (nodes by Newton's method on the Legendre recurrence)

struct GaussRule {
  int n;
  std::vector<double> x, w;
  explicit GaussRule(int n_) : n(n_), x(n_), w(n_) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        double step = p1 / dp;
        z -= step;
        if (std::fabs(step) < 1e-17) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussRule& gauss48() {
  static const GaussRule g(48);
  return g;
}

// F(phi|m) and E(phi|m) (parameter convention) by composite Gauss-Legendre
// quadrature of (1 - m sin^2 t)^(-+1/2) over [0, phi]; both integrands are analytic
// for m <= 1/2, so two 48-point panels reach round-off.
void ellint_FE(double phi, double m, double* F, double* E) {
  const GaussRule& g = gauss48();
  double sF = 0.0, sE = 0.0;
  for (int panel = 0; panel < 2; ++panel) {
    double a = 0.5 * phi * panel, b = 0.5 * phi * (panel + 1);
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    for (int i = 0; i < g.n; ++i) {
      double s = std::sin(c + h * g.x[i]);
      double d = std::sqrt(1.0 - m * s * s);
      sF += g.w[i] * h / d;
      sE += g.w[i] * h * d;
    }
  }
  *F = sF;
  *E = sE;
}

struct SpamGeom {
  double Rc, Ract, a, l0;
};

// Eq. 1b with l_a = l0, multiplied by cos^2(phi): its smallest root in (0, phi_Rc]
// is the unsaturated state; its derivative is used by the Newton steps.
double eq1b(const SpamGeom& g, double m, double phi, double* dres) {
  double F, E;
  ellint_FE(phi, m, &F, &E);
  double c = std::cos(phi), s = std::sin(phi), sm = std::sqrt(m);
  double res = F * c / sm - (g.l0 / g.Rc) * (c * c + g.a / (2.0 * m));
  if (dres) {
    double dF = 1.0 / std::sqrt(1.0 - m * s * s);
    *dres = (dF * c - F * s) / sm + (g.l0 / g.Rc) * 2.0 * c * s;
  }
  return res;
}

// strain and force per unit pressure for contraction parameter m (Eq. 1a-d)
void spam_point(const SpamGeom& g, double m, double* eps, double* G) {
  const double phiRc = std::acos(g.Rc / g.Ract);
  const int kScan = 64;
  double lo = 1e-12, flo = eq1b(g, m, lo, nullptr), phi = -1.0;
  for (int k = 1; k <= kScan && phi < 0.0; ++k) {
    double hi = phiRc * k / kScan, fhi = eq1b(g, m, hi, nullptr);
    if (flo < 0.0 && fhi >= 0.0) {
      // safeguarded Newton inside [lo, hi]
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 100; ++it) {
        double d, f = eq1b(g, m, x, &d);
        if (f < 0.0) lo = x; else hi = x;
        double xn = x - f / d;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-16 * x) {
          x = xn;
          break;
        }
        x = xn;
      }
      phi = x;
    } else {
      lo = hi;
      flo = fhi;
    }
  }
  double la = g.l0;
  if (phi < 0.0) {  // saturated: phi = phi_Rc, Eq. 1b gives the active length
    phi = phiRc;
    double F, E, c = std::cos(phi);
    ellint_FE(phi, m, &F, &E);
    la = g.Rc * F / (std::sqrt(m) * c * (1.0 + g.a / (2.0 * m * c * c)));
  }
  double F, E, c = std::cos(phi);
  ellint_FE(phi, m, &F, &E);
  *eps = (la - 2.0 * g.Rc * (E - 0.5 * F) / (std::sqrt(m) * c)) / g.l0;
  *G = kPi * g.Rc * g.Rc * (1.0 - 2.0 * m) / (2.0 * m * c * c);
}

// m in [m_lo, m_hi] with eps(m) = target (eps increases with m): regula falsi
// (Illinois variant) on a bracket.
double spam_invert(const SpamGeom& g, double target, double m_lo, double e_lo, double m_hi,
                   double e_hi) {
  double fa = e_lo - target, fb = e_hi - target, a = m_lo, b = m_hi;
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    double m = (a * fb - b * fa) / (fb - fa);
    if (!(m > a && m < b)) m = 0.5 * (a + b);
    double e, G;
    spam_point(g, m, &e, &G);
    double fm = e - target;
    if (fm == 0.0) return m;
    if ((fm < 0.0) == (fa < 0.0)) {
      a = m;
      fa = fm;
      if (side == -1) fb *= 0.5;
      side = -1;
    } else {
      b = m;
      fb = fm;
      if (side == 1) fa *= 0.5;
      side = 1;
    }
    if (b - a <= 4e-16 * b) break;
  }
  return 0.5 * (a + b);
}

// Chebyshev series of f on [-1, 1] from values at the first-kind nodes
void cheb_coeffs(const std::vector<double>& f, int deg, double* c) {
  int N = deg + 1;
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += f[k] * std::cos(kPi * j * (k + 0.5) / N);
    c[j] = 2.0 * s / N;
  }
  c[0] *= 0.5;
}

double cheb_eval_host(const double* c, int deg, double x) {
  double b1 = 0.0, b2 = 0.0;
  for (int j = deg; j >= 1; --j) {
    double t = 2.0 * x * b1 - b2 + c[j];
    b2 = b1;
    b1 = t;
  }
  return x * b1 - b2 + c[0];
}

void build_spam_table(SpamTable* T, double l0, double Rc, double Ract, double a) {
  SpamGeom g{Rc, Ract, a, l0};
  constexpr int P = vs::kSpamPieces, D = vs::kSpamDeg;
  std::memset(T, 0, sizeof(*T));
  T->l0 = l0;
  // coarse map m -> eps to bracket the inversions
  const int NM = 400;
  std::vector<double> mg(NM + 1), eg(NM + 1);
  for (int i = 0; i <= NM; ++i) {
    double s = (double)i / NM;
    mg[i] = 0.002 + (0.5 - 0.002) * s;
    double G;
    spam_point(g, mg[i], &eg[i], &G);
  }
  double Gdummy;
  spam_point(g, 0.5, &T->emax, &Gdummy);
  auto m_of_eps = [&](double eps) {
    int i = 0;
    while (i < NM && eg[i + 1] < eps) ++i;
    return spam_invert(g, eps, mg[i], eg[i], mg[i + 1], eg[i + 1]);
  };
  for (int k = 0; k <= P; ++k) {
    double s = (double)k / P;
    T->bnd[k] = T->emax * s * s;
  }
  std::vector<double> f(D + 1);
  for (int k = 0; k < P; ++k) {
    double lo = T->bnd[k], hi = T->bnd[k + 1];
    for (int q = 0; q <= D; ++q) {
      double x = std::cos(kPi * (q + 0.5) / (D + 1));
      double eps = 0.5 * (lo + hi) + 0.5 * (hi - lo) * x;
      double e, G;
      spam_point(g, m_of_eps(eps), &e, &G);
      f[q] = G;
    }
    cheb_coeffs(f, D, T->c[k]);
    // derivative series (in x) and integral series (in x, zero at x = -1)
    double av[D + 3] = {0}, dv[D + 3] = {0};
    for (int j = 0; j <= D; ++j) av[j] = T->c[k][j];
    av[0] *= 2.0;
    for (int j = D; j >= 1; --j) dv[j - 1] = dv[j + 1] + 2.0 * j * av[j];
    for (int j = 0; j <= D; ++j) T->dc[k][j] = dv[j];
    T->dc[k][0] *= 0.5;
    for (int j = 1; j <= D + 1; ++j) T->ic[k][j] = (av[j - 1] - av[j + 1]) / (2.0 * j);
    T->ic[k][0] = 0.0;
    T->ic[k][0] = -cheb_eval_host(T->ic[k], D + 1, -1.0);
    T->cum[k + 1] = T->cum[k] + 0.5 * (hi - lo) * cheb_eval_host(T->ic[k], D + 1, 1.0);
  }
  T->G0 = cheb_eval_host(T->c[0], D, -1.0);
}

// wrinkling fraction h(x) of Eq. 2 on the host (same law as the kernel)
double wr_h_host(double x, double epsc) {
  double th_on = 2.0 * std::asin(epsc);
  if (x <= th_on) return x / (2.0 * th_on);
  if (x > kPi) x = kPi;
  double c = std::fmin(1.0, std::fmax(-1.0, 2.0 * epsc / std::sin(0.5 * x) - 1.0));
  double gm = std::acos(c);
  return (std::sin(2.0 * gm) + 2.0 * kPi - 2.0 * gm) /
         (4.0 * (std::sin(gm) + (kPi - gm) * std::cos(gm)));
}

void build_wr_table(WrTable* T, double epsc) {
  std::memset(T, 0, sizeof(*T));
  constexpr int P = vs::kIhPieces, D = vs::kIhDeg;
  T->th_on = 2.0 * std::asin(epsc);
  T->umax = std::sqrt(kPi - T->th_on);
  T->du = T->umax / P;
  T->cum[0] = T->th_on / 4.0;
  std::vector<double> f(D + 1);
  double c[D + 1], av[D + 3];
  for (int k = 0; k < P; ++k) {
    const double a = k * T->du, b = a + T->du;
    for (int q = 0; q <= D; ++q) {
      const double t = std::cos(kPi * (q + 0.5) / (D + 1));
      const double u = 0.5 * (a + b) + 0.5 * (b - a) * t;
      f[q] = 2.0 * u * wr_h_host(T->th_on + u * u, epsc);
    }
    cheb_coeffs(f, D, c);
    for (int j = 0; j <= D + 2; ++j) av[j] = j <= D ? c[j] : 0.0;
    av[0] *= 2.0;
    for (int j = 1; j <= D + 1; ++j) T->ic[k][j] = (av[j - 1] - av[j + 1]) / (2.0 * j);
    T->ic[k][0] = 0.0;
    T->ic[k][0] = -cheb_eval_host(T->ic[k], D + 1, -1.0);
    T->cum[k + 1] = T->cum[k] + 0.5 * T->du * cheb_eval_host(T->ic[k], D + 1, 1.0);
  }
  T->h_pi = wr_h_host(kPi, epsc);
  T->ih_pi = T->cum[P];
}

thread_local std::string g_create_error;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

struct vine_sim {
  vine_params prm;
  int B = 0, N = 0, T = 0, S = 0;
  std::vector<double> link_lens;      // distinct link lengths (table ids)
  std::vector<SpamTable> tables_h;
  // device arrays
  int* ii = nullptr;
  double* dd = nullptr;
  double* cover = nullptr;
  double* spam = nullptr;
  int* okind = nullptr;
  double* obs = nullptr;
  SpamTable* tables = nullptr;
  WrTable* wr = nullptr;
  double* theta = nullptr;
  int* ncur = nullptr;
  int* tcur = nullptr;
  double* tip = nullptr;
  double* rho = nullptr;
  int* iters = nullptr;
  int* status = nullptr;
  int* ncont = nullptr;
  unsigned long long* chash = nullptr;
  double* maxpen = nullptr;
  double* traj = nullptr;
  double* jevals = nullptr;
  double* nsolves = nullptr;
  int trace_robot = -1, trace_cap = 0;
  double* trace = nullptr;
  int* trace_n = nullptr;
  bool traj_valid = false;  // some step since the reset recorded its joint angles
  bool traj_all = true;     // every step since the reset did
  std::string err;
};

namespace {

int fail(vine_sim* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

void free_all(vine_sim* h) {
  void* ptrs[] = {h->ii, h->dd, h->cover, h->spam, h->okind, h->obs, h->tables, h->wr, h->theta,
                  h->ncur, h->tcur, h->tip, h->rho, h->iters, h->status, h->ncont, h->chash,
                  h->maxpen, h->traj, h->jevals, h->nsolves, h->trace, h->trace_n};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1));
}

vs::KParams kparams(const vine_params& p) {
  vs::KParams k;
  k.epsc = p.eps_crit;
  k.kc = p.k_c;
  k.tol = p.tol;
  k.c_mu = p.c_mu;
  k.step_max = p.step_max;
  k.c1 = p.armijo_c1;
  k.Ract = p.R_act;
  k.max_iter = p.max_iter;
  k.substeps = p.growth_substeps;
  k.dense_solver = p.solver == 1;
  return k;
}

vs::KData kdata(vine_sim* h) {
  vs::KData D;
  D.n_inst = h->B;
  D.n_max = h->N;
  D.t_max = h->T;
  D.ii = h->ii;
  D.dd = h->dd;
  D.cover = h->cover;
  D.spam = h->spam;
  D.n_spam = h->S;
  D.okind = h->okind;
  D.obs = h->obs;
  D.tables = h->tables;
  D.wr = h->wr;
  D.theta = h->theta;
  D.ncur = h->ncur;
  D.tcur = h->tcur;
  D.tip = h->tip;
  D.rho = h->rho;
  D.iters = h->iters;
  D.status = h->status;
  D.ncont = h->ncont;
  D.chash = h->chash;
  D.maxpen = h->maxpen;
  D.traj = h->traj;
  D.jevals = h->jevals;
  D.nsolves = h->nsolves;
  D.trace_robot = h->trace ? h->trace_robot : -1;
  D.trace_cap = h->trace_cap;
  D.trace = h->trace;
  D.trace_n = h->trace_n;
  return D;
}

}  // namespace

extern "C" {

void vine_params_default(vine_params* p) {
  if (!p) return;
  p->R_c = 0.005;
  p->R_act = 0.01718;
  p->a_corr = 1e-4;
  p->eps_crit = 0.01;
  p->k_c = 1e4;
  p->tol = 1e-10;
  p->c_mu = 1.0;
  p->step_max = 0.05;
  p->armijo_c1 = 1e-4;
  p->max_iter = 500;
  p->growth_substeps = 2;
  p->solver = 0;
  p->reserved = 0;
}

int32_t vine_sim_create(const vine_params* params, const vine_instance* inst, int32_t n_inst,
                        const vine_spam* spams, int32_t n_spams, const vine_obstacle* obstacles,
                        int32_t n_obstacles, vine_sim** out) {
  if (!params || !inst || !out || n_inst < 1 || n_spams < 0 || n_obstacles < 0 ||
      (n_spams > 0 && !spams) || (n_obstacles > 0 && !obstacles))
    return fail(nullptr, VINE_EINVAL, "null pointer or negative count");
  const vine_params& p = *params;
  if (!finite_pos(p.R_c) || !finite_pos(p.R_act) || !(p.R_act > p.R_c) || !(p.a_corr >= 0.0) ||
      !std::isfinite(p.a_corr) || !(p.eps_crit > 0.0 && p.eps_crit < 1.0) || !finite_pos(p.k_c) ||
      !finite_pos(p.tol) || !(p.c_mu >= 0.0) || !std::isfinite(p.c_mu) ||
      !finite_pos(p.step_max) || !(p.armijo_c1 > 0.0 && p.armijo_c1 < 1.0) || p.max_iter < 0 ||
      p.growth_substeps < 1 || !(p.solver == 0 || p.solver == 1))
    return fail(nullptr, VINE_EINVAL, "invalid vine_params");
  int N = 0;
  for (int b = 0; b < n_inst; ++b) {
    const vine_instance& I = inst[b];
    char msg[160];
    std::snprintf(msg, sizeof msg, "instance %d: ", b);
    if (I.n_links < 1) return fail(nullptr, VINE_EINVAL, std::string(msg) + "n_links < 1");
    if (I.n_links > VINE_MAX_LINKS)
      return fail(nullptr, VINE_ECAPACITY, std::string(msg) + "n_links above VINE_MAX_LINKS");
    if (!finite_pos(I.link_len) || !finite_pos(I.tube_radius) || !finite_pos(I.body_pressure) ||
        !std::isfinite(I.base_x) || !std::isfinite(I.base_y) || !std::isfinite(I.base_heading))
      return fail(nullptr, VINE_EINVAL, std::string(msg) + "non-positive or non-finite geometry");
    if (I.spam_count < 0 || I.spam_offset < 0 || (int64_t)I.spam_offset + I.spam_count > n_spams ||
        I.obs_count < 0 || I.obs_offset < 0 ||
        (int64_t)I.obs_offset + I.obs_count > n_obstacles)
      return fail(nullptr, VINE_EINVAL, std::string(msg) + "sPAM/obstacle range out of bounds");
    if (I.obs_count > VINE_MAX_OBSTACLES || I.spam_count > VINE_MAX_SPAMS)
      return fail(nullptr, VINE_ECAPACITY, std::string(msg) + "too many obstacles or sPAMs");
    for (int s = 0; s < I.spam_count; ++s) {
      const vine_spam& S = spams[I.spam_offset + s];
      if (!std::isfinite(S.s_start) || !std::isfinite(S.s_end) || S.s_start < 0.0 ||
          S.s_end < S.s_start || !(S.side == 1.0 || S.side == -1.0) ||
          !std::isfinite(S.pressure) || S.pressure < 0.0)
        return fail(nullptr, VINE_EINVAL, std::string(msg) + "invalid sPAM");
    }
    for (int k = 0; k < I.obs_count; ++k) {
      const vine_obstacle& O = obstacles[I.obs_offset + k];
      if (!(O.kind == 0 || O.kind == 1) || !std::isfinite(O.cx) || !std::isfinite(O.cy) ||
          !finite_pos(O.a) || (O.kind == 1 && !finite_pos(O.b)))
        return fail(nullptr, VINE_EINVAL, std::string(msg) + "invalid obstacle");
    }
    if (I.n_links > N) N = I.n_links;
  }
  if (p.solver == 1 && N > 64)
    return fail(nullptr, VINE_ECAPACITY, "the dense cross-check solver holds at most 64 links");
  vine_sim* h = new (std::nothrow) vine_sim();
  if (!h) return fail(nullptr, VINE_ENOMEM, "host allocation failed");
  h->prm = p;
  h->B = n_inst;
  h->N = N;
  h->T = N;
  h->S = n_spams;
  // host-side derived inputs
  std::vector<int> ii(8 * (size_t)n_inst);
  std::vector<double> dd(6 * (size_t)n_inst);
  std::vector<int> okind;
  std::vector<double> obs;
  std::vector<double> cover;
  for (int b = 0; b < n_inst; ++b) {
    const vine_instance& I = inst[b];
    int tid = -1;
    for (size_t t = 0; t < h->link_lens.size(); ++t)
      if (h->link_lens[t] == I.link_len) tid = (int)t;
    if (tid < 0) {
      tid = (int)h->link_lens.size();
      h->link_lens.push_back(I.link_len);
    }
    ii[8 * b + 0] = I.n_links;
    ii[8 * b + 1] = (int)okind.size();
    ii[8 * b + 2] = I.obs_count;
    ii[8 * b + 3] = tid;
    ii[8 * b + 4] = (int)(cover.size() / 2);
    ii[8 * b + 5] = I.spam_offset;
    ii[8 * b + 6] = I.spam_count;
    ii[8 * b + 7] = 0;
    dd[6 * b + 0] = I.link_len;
    dd[6 * b + 1] = I.tube_radius;
    dd[6 * b + 2] = I.body_pressure;
    dd[6 * b + 3] = I.base_x;
    dd[6 * b + 4] = I.base_y;
    dd[6 * b + 5] = I.base_heading;
    for (int k = 0; k < I.obs_count; ++k) {
      const vine_obstacle& O = obstacles[I.obs_offset + k];
      okind.push_back(O.kind);
      obs.push_back(O.cx);
      obs.push_back(O.cy);
      obs.push_back(O.a);
      obs.push_back(O.kind == 1 ? O.b : 0.0);
    }
    // joint j takes the pressure-weighted fraction of link [j l, (j+1) l] each sPAM covers
    const double l = I.link_len;
    for (int j = 0; j < I.n_links; ++j) {
      double pp = 0.0, pm = 0.0;
      for (int s = 0; s < I.spam_count; ++s) {
        const vine_spam& S = spams[I.spam_offset + s];
        double lo = std::fmax(S.s_start, j * l), hi = std::fmin(S.s_end, (j + 1) * l);
        if (hi > lo) {
          double w = (hi - lo) / l;
          if (S.side > 0.0) pp += w * S.pressure; else pm += w * S.pressure;
        }
      }
      cover.push_back(pp);
      cover.push_back(pm);
    }
  }
  h->tables_h.resize(h->link_lens.size());
  for (size_t t = 0; t < h->link_lens.size(); ++t)
    build_spam_table(&h->tables_h[t], h->link_lens[t], p.R_c, p.R_act, p.a_corr);
  WrTable wr;
  build_wr_table(&wr, p.eps_crit);
  const size_t B = n_inst, NN = N, TT = N;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&h->ii, ii.size()));
  A(dalloc(&h->dd, dd.size()));
  A(dalloc(&h->cover, cover.size()));
  A(dalloc(&h->spam, 4 * (size_t)n_spams));
  A(dalloc(&h->okind, okind.size()));
  A(dalloc(&h->obs, obs.size()));
  A(dalloc(&h->tables, h->tables_h.size()));
  A(dalloc(&h->wr, 1));
  A(dalloc(&h->theta, B * NN));
  A(dalloc(&h->ncur, B));
  A(dalloc(&h->tcur, B));
  A(dalloc(&h->tip, B * TT * 3));
  A(dalloc(&h->rho, B * TT));
  A(dalloc(&h->iters, B * TT));
  A(dalloc(&h->status, B * TT));
  A(dalloc(&h->ncont, B * TT));
  A(dalloc(&h->chash, B * TT));
  A(dalloc(&h->maxpen, B * TT));
  A(dalloc(&h->traj, B * TT * NN));
  A(dalloc(&h->jevals, B));
  A(dalloc(&h->nsolves, B));
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("device allocation: ") + hipGetErrorString(e));
  }
  A(hipMemcpy(h->ii, ii.data(), sizeof(int) * ii.size(), hipMemcpyHostToDevice));
  A(hipMemcpy(h->dd, dd.data(), sizeof(double) * dd.size(), hipMemcpyHostToDevice));
  if (!cover.empty())
    A(hipMemcpy(h->cover, cover.data(), sizeof(double) * cover.size(), hipMemcpyHostToDevice));
  if (n_spams > 0) {
    std::vector<double> sp(4 * (size_t)n_spams);
    for (int i = 0; i < n_spams; ++i) {
      sp[4 * i + 0] = spams[i].s_start;
      sp[4 * i + 1] = spams[i].s_end;
      sp[4 * i + 2] = spams[i].side;
      sp[4 * i + 3] = spams[i].pressure;
    }
    A(hipMemcpy(h->spam, sp.data(), sizeof(double) * sp.size(), hipMemcpyHostToDevice));
  }
  if (!okind.empty()) {
    A(hipMemcpy(h->okind, okind.data(), sizeof(int) * okind.size(), hipMemcpyHostToDevice));
    A(hipMemcpy(h->obs, obs.data(), sizeof(double) * obs.size(), hipMemcpyHostToDevice));
  }
  A(hipMemcpy(h->tables, h->tables_h.data(), sizeof(SpamTable) * h->tables_h.size(),
              hipMemcpyHostToDevice));
  A(hipMemcpy(h->wr, &wr, sizeof(WrTable), hipMemcpyHostToDevice));
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, VINE_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
  }
  if (vine_sim_reset(h, nullptr) != VINE_OK) {
    std::string m = h->err;
    free_all(h);
    delete h;
    return fail(nullptr, VINE_EDEVICE, m);
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, VINE_EDEVICE, "synchronise after reset");
  }
  *out = h;
  return VINE_OK;
}

int32_t vine_sim_reset(vine_sim* h, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  hipStream_t s = (hipStream_t)stream;
  const size_t B = h->B, NN = h->N, TT = h->T;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(hipMemsetAsync(h->theta, 0, sizeof(double) * B * NN, s));
  A(hipMemsetAsync(h->ncur, 0, sizeof(int) * B, s));
  A(hipMemsetAsync(h->tcur, 0, sizeof(int) * B, s));
  A(hipMemsetAsync(h->tip, 0, sizeof(double) * B * TT * 3, s));
  A(hipMemsetAsync(h->rho, 0, sizeof(double) * B * TT, s));
  A(hipMemsetAsync(h->iters, 0, sizeof(int) * B * TT, s));
  A(hipMemsetAsync(h->status, 0, sizeof(int) * B * TT, s));
  A(hipMemsetAsync(h->ncont, 0, sizeof(int) * B * TT, s));
  A(hipMemsetAsync(h->chash, 0, sizeof(unsigned long long) * B * TT, s));
  A(hipMemsetAsync(h->maxpen, 0, sizeof(double) * B * TT, s));
  A(hipMemsetAsync(h->jevals, 0, sizeof(double) * B, s));
  A(hipMemsetAsync(h->nsolves, 0, sizeof(double) * B, s));
  h->traj_valid = false;
  h->traj_all = true;
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("reset: ") + hipGetErrorString(e));
  return VINE_OK;
}

static int32_t advance(vine_sim* h, int32_t n_steps, int32_t record_traj, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (n_steps < 0) n_steps = h->T;
  if (n_steps == 0) return VINE_OK;
  hipError_t e = vs::launch_rollout(kparams(h->prm), kdata(h), n_steps, record_traj, h->N,
                                    (hipStream_t)stream);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  if (record_traj) h->traj_valid = true; else h->traj_all = false;
  return VINE_OK;
}

int32_t vine_sim_step(vine_sim* h, int32_t n_steps, int32_t record_traj, void* stream) {
  if (n_steps < 0) return fail(h, VINE_EINVAL, "n_steps < 0");
  return advance(h, n_steps, record_traj, stream);
}

int32_t vine_sim_rollout(vine_sim* h, int32_t n_steps, int32_t record_traj, void* stream) {
  return advance(h, n_steps < 0 ? -1 : n_steps, record_traj, stream);
}

int32_t vine_sim_grad(vine_sim* h, const double* goal, const double* step_weights,
                      double* dL_dP, double* dL_ds_start, double* dL_ds_end, double* loss,
                      int32_t* adj_status, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (!goal || !loss || (h->S > 0 && (!dL_dP || !dL_ds_start || !dL_ds_end)))
    return fail(h, VINE_EINVAL, "null goal, loss or gradient pointer");
  if (step_weights && !(h->traj_valid && h->traj_all))
    return fail(h, VINE_ESTATE,
                "step weights need the joint angles of every step since the reset "
                "(record_traj on every step/rollout call)");
  hipError_t e = vs::launch_grad(kparams(h->prm), kdata(h), goal, step_weights, h->T, dL_dP,
                                 dL_ds_start, dL_ds_end, loss, adj_status, h->N,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return VINE_OK;
}

int64_t vine_sim_field_bytes(const vine_sim* h, int32_t field) {
  if (!h) return 0;
  const int64_t B = h->B, N = h->N, T = h->T;
  switch (field) {
    case VINE_F_THETA: return 8 * B * N;
    case VINE_F_NLINKS: return 4 * B;
    case VINE_F_TIP: return 8 * B * T * 3;
    case VINE_F_RHO: return 8 * B * T;
    case VINE_F_ITERS: return 4 * B * T;
    case VINE_F_STATUS: return 4 * B * T;
    case VINE_F_NCONTACT: return 4 * B * T;
    case VINE_F_CHASH: return 8 * B * T;
    case VINE_F_MAXPEN: return 8 * B * T;
    case VINE_F_TRAJ: return 8 * B * T * N;
    case VINE_F_JEVALS: return 8 * B;
    case VINE_F_NSOLVES: return 8 * B;
    default: return 0;
  }
}

int32_t vine_sim_read(const vine_sim* hc, int32_t field, void* dst, int32_t dst_on_device,
                      void* stream) {
  vine_sim* h = const_cast<vine_sim*>(hc);
  if (!h || !dst) return fail(h, VINE_EINVAL, "null handle or destination");
  const void* src = nullptr;
  switch (field) {
    case VINE_F_THETA: src = h->theta; break;
    case VINE_F_NLINKS: src = h->ncur; break;
    case VINE_F_TIP: src = h->tip; break;
    case VINE_F_RHO: src = h->rho; break;
    case VINE_F_ITERS: src = h->iters; break;
    case VINE_F_STATUS: src = h->status; break;
    case VINE_F_NCONTACT: src = h->ncont; break;
    case VINE_F_CHASH: src = h->chash; break;
    case VINE_F_MAXPEN: src = h->maxpen; break;
    case VINE_F_TRAJ:
      if (!h->traj_valid) return fail(h, VINE_ESTATE, "no trajectory was recorded");
      src = h->traj;
      break;
    case VINE_F_JEVALS: src = h->jevals; break;
    case VINE_F_NSOLVES: src = h->nsolves; break;
    default: return fail(h, VINE_EINVAL, "unknown field");
  }
  size_t bytes = (size_t)vine_sim_field_bytes(h, field);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(dst, src, bytes,
                                dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && !dst_on_device) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("read: ") + hipGetErrorString(e));
  return VINE_OK;
}

void vine_sim_dims(const vine_sim* h, int32_t dims[3]) {
  if (!dims) return;
  dims[0] = h ? h->B : 0;
  dims[1] = h ? h->T : 0;
  dims[2] = h ? h->N : 0;
}

void vine_sim_destroy(vine_sim* h) {
  if (!h) return;
  free_all(h);
  delete h;
}

const char* vine_sim_last_error(const vine_sim* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int32_t vine_sim_trace(vine_sim* h, int32_t robot, int32_t capacity) {
  if (!h || robot < -1 || robot >= h->B || capacity < 0) return fail(h, VINE_EINVAL, "bad arguments");
  if (h->trace) (void)hipFree(h->trace);
  if (h->trace_n) (void)hipFree(h->trace_n);
  h->trace = nullptr;
  h->trace_n = nullptr;
  h->trace_robot = -1;
  h->trace_cap = 0;
  if (robot < 0 || capacity == 0) return VINE_OK;
  hipError_t e = dalloc(&h->trace, (size_t)capacity * vs::kTraceCols);
  if (e == hipSuccess) e = dalloc(&h->trace_n, 1);
  if (e == hipSuccess) e = hipMemset(h->trace_n, 0, sizeof(int));
  if (e != hipSuccess) return fail(h, VINE_ENOMEM, "trace buffer");
  h->trace_robot = robot;
  h->trace_cap = capacity;
  return VINE_OK;
}

int32_t vine_sim_trace_read(const vine_sim* hc, double* dst, int32_t capacity) {
  vine_sim* h = const_cast<vine_sim*>(hc);
  if (!h || !dst || !h->trace) return fail(h, VINE_ESTATE, "no trace buffer");
  int n = 0;
  hipError_t e = hipMemcpy(&n, h->trace_n, sizeof(int), hipMemcpyDeviceToHost);
  if (n > capacity) n = capacity;
  if (n > h->trace_cap) n = h->trace_cap;
  if (e == hipSuccess && n > 0)
    e = hipMemcpy(dst, h->trace, sizeof(double) * vs::kTraceCols * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, "trace read");
  return n;
}

int32_t vine_sim_spam_law(const vine_sim* hc, double l, int32_t n, const double* eps, double* G,
                          double* dG, double* IG) {
  vine_sim* h = const_cast<vine_sim*>(hc);
  if (!h || n < 0 || (n > 0 && !eps)) return fail(h, VINE_EINVAL, "bad arguments");
  int tid = -1;
  for (size_t t = 0; t < h->link_lens.size(); ++t)
    if (h->link_lens[t] == l) tid = (int)t;
  if (tid < 0) return fail(h, VINE_EINVAL, "not a link length of this simulation");
  const SpamTable& T = h->tables_h[tid];
  constexpr int P = vs::kSpamPieces, D = vs::kSpamDeg;
  for (int i = 0; i < n; ++i) {
    double e = eps[i];
    if (e >= T.emax) {
      if (G) G[i] = 0.0;
      if (dG) dG[i] = 0.0;
      if (IG) IG[i] = T.cum[P];
      continue;
    }
    int k = (int)(P * std::sqrt(std::fmax(e, 0.0) / T.emax));
    k = k < 0 ? 0 : (k > P - 1 ? P - 1 : k);
    double a = T.bnd[k], b = T.bnd[k + 1], x = (2.0 * e - a - b) / (b - a);
    if (G) G[i] = cheb_eval_host(T.c[k], D, x);
    if (dG) dG[i] = cheb_eval_host(T.dc[k], D - 1, x) * 2.0 / (b - a);
    if (IG) IG[i] = T.cum[k] + 0.5 * (b - a) * cheb_eval_host(T.ic[k], D + 1, x);
  }
  return VINE_OK;
}

}  // extern "C"
