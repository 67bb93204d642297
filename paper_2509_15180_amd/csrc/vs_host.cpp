// vs_host.cpp -- host side of the C ABI (include/vinesim.h): validation, the
// create-time sPAM force-law table (Sec. 3.1, Eq. 1 solved for G = F_t / P_act),
// the wrinkling-energy table (Sec. 3.2), device allocation and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <array>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <type_traits>
#include <vector>

#include "../../include/vinesim.h"
#include "vs_device.h"
#include "vs_server.h"
#include "vs_synth.h"

static_assert(vs::kMaxObs == VINE_MAX_OBSTACLES, "obstacle capacity of the kernels");
static_assert(vs::kScratchBytes == VINE_GRAD_SCRATCH_BYTES, "scratch size of the kernels");

namespace vs {
hipError_t launch_rollout(const KParams& P, const KData& D, int n_steps, int nmax_class,
                          int waves, hipStream_t stream);
hipError_t launch_grad(const KParams& P, const KData& D, const double* goal,
                       const double* weights, int T, int t0, const double* traj, int traj_rows,
                       const GradPart& part, double* dP, double* ds0, double* ds1, double* loss,
                       int* status, int nmax_class, hipStream_t stream);
hipError_t launch_zero3(double* a, double* b, double* c, int n, hipStream_t stream);
hipError_t launch_reset(const KData& D, hipStream_t stream);
hipError_t launch_seg_load(const KData& Dseg, const int* ii_handle, const double* ckpt,
                           const int* tcur, int n_ckpt, int q, int ce, hipStream_t stream);
hipError_t scratch_address(void** out);
hipError_t rollout_occupancy(int nmax_class, int waves, int* per_cu);
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

// the same law in long double: near pi the numerator and denominator of Eq. 2a both
// cancel, which costs the double formula ~1e-13; the h series is fitted to these values
double wr_h_host_ld(double x, double epsc) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double th_on = 2.0L * asinl((long double)epsc);
  long double xl = x;
  if (xl <= th_on) return (double)(xl / (2.0L * th_on));
  if (xl > pi) xl = pi;
  long double c = 2.0L * epsc / sinl(0.5L * xl) - 1.0L;
  c = c > 1.0L ? 1.0L : (c < -1.0L ? -1.0L : c);
  const long double gm = acosl(c);
  return (double)((sinl(2.0L * gm) + 2.0L * pi - 2.0L * gm) /
                  (4.0L * (sinl(gm) + (pi - gm) * cosl(gm))));
}

// its slope above the onset, in long double.  With s = sin(x/2), cos(g) = 2 eps_c / s - 1
// for the wrinkle angle g = gamma0, and N, D the numerator and denominator of Eq. 2a,
//   dh/dx = 4 eps_c cos(x/2) (N (pi - g) - sin(g) D) / (s^2 D^2)
// (the 1/sin(gamma0) of dgamma0/dx cancels); acos near 1 loses half the digits in double
double wr_dh_host_ld(double x, double epsc) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double xl = x, s = sinl(0.5L * xl), co = cosl(0.5L * xl);
  long double c = 2.0L * epsc / s - 1.0L;
  c = c > 1.0L ? 1.0L : c;
  const long double g = acosl(c), sg = sqrtl((1.0L - c) * (1.0L + c));
  const long double N = 2.0L * sg * c + 2.0L * pi - 2.0L * g;
  const long double D = 4.0L * (sg + (pi - g) * c);
  return (double)(4.0L * epsc * co * (N * (pi - g) - sg * D) / (s * s * D * D));
}

void build_wr_table(WrTable* T, double epsc) {
  std::memset(T, 0, sizeof(*T));
  constexpr int P = vs::kIhPieces, D = vs::kIhDeg;
  T->th_on = 2.0 * std::asin(epsc);
  T->umax = std::sqrt(kPi - T->th_on);
  T->du = T->umax / P;
  T->cum[0] = T->th_on / 4.0;
  std::vector<double> f(D + 1), hv(D + 1), dv(D + 1);
  double c[D + 1], av[D + 3];
  for (int k = 0; k < P; ++k) {
    const double a = k * T->du, b = a + T->du;
    for (int q = 0; q <= D; ++q) {
      const double t = std::cos(kPi * (q + 0.5) / (D + 1));
      const double u = 0.5 * (a + b) + 0.5 * (b - a) * t;
      hv[q] = wr_h_host_ld(T->th_on + u * u, epsc);
      dv[q] = wr_dh_host_ld(T->th_on + u * u, epsc);
      f[q] = 2.0 * u * wr_h_host(T->th_on + u * u, epsc);
    }
    cheb_coeffs(hv, D, T->hc[k]);
    cheb_coeffs(dv, D, T->dhc[k]);
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

bool spam_ok(const vine_spam& S) {
  return std::isfinite(S.s_start) && std::isfinite(S.s_end) && S.s_start >= 0.0 &&
         S.s_end >= S.s_start && (S.side == 1.0 || S.side == -1.0) && std::isfinite(S.pressure) &&
         S.pressure >= 0.0;
}

// Joint j of a robot takes the pressure-weighted fraction of link [j l, (j+1) l] that
// each of its sPAMs covers, on the sPAM's side (appends 2 doubles per joint).
void append_cover(const vine_instance& I, const vine_spam* spams, std::vector<double>& cover) {
  const double l = I.link_len;
  for (int j = 0; j < I.n_links; ++j) {
    double pp = 0.0, pm = 0.0;
    for (int s = 0; s < I.spam_count; ++s) {
      const vine_spam& S = spams[I.spam_offset + s];
      const double lo = std::fmax(S.s_start, j * l), hi = std::fmin(S.s_end, (j + 1) * l);
      if (hi > lo) {
        const double w = (hi - lo) / l;
        if (S.side > 0.0) pp += w * S.pressure; else pm += w * S.pressure;
      }
    }
    cover.push_back(pp);
    cover.push_back(pm);
  }
}

}  // namespace

struct vine_sim {
  vine_params prm;
  int B = 0, N = 0, T = 0, S = 0;
  long long theta_len = 0, rec_len = 0;  // elements of theta and of each record array
  int skip_done = 0;                     // serving slabs: robots at full length do nothing
  std::vector<double> link_lens;      // distinct link lengths (table ids)
  std::vector<SpamTable> tables_h;
  std::vector<vine_instance> inst_h;  // as given at create (sPAM ranges, lengths)
  uint64_t config_hash = 0;  // of the parameters and every input at create (autotune cache)
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
  double* tiplen = nullptr;  // per step: the tip link's length
  double* ulast = nullptr;   // [B] soft growth: the tip link's length in link lengths
  double* traj = nullptr;    // [B][n_rec][N], allocated for rec_every on first use
  int rec_every = 0, n_rec = 0;
  double* ckpt = nullptr;    // [B][n_ckpt][N], allocated for ckpt_every on first use
  int ckpt_every = 0, n_ckpt = 0;
  double* jevals = nullptr;
  double* nsolves = nullptr;
  double* negsteps = nullptr;
  double* cycles = nullptr;
  double* wtime = nullptr;
  double wall_period = 0.0;  // seconds per device wall-clock tick
  // recomputation of a checkpoint segment for the adjoint (allocated on first use):
  // state, records and trajectory of ckpt_every steps
  struct Seg {
    double *theta = nullptr, *tip = nullptr, *rho = nullptr, *maxpen = nullptr,
           *traj = nullptr, *jevals = nullptr, *nsolves = nullptr, *negsteps = nullptr,
           *cycles = nullptr, *wtime = nullptr, *gsums = nullptr, *gloss = nullptr,
           *tiplen = nullptr, *ulast = nullptr;
    int *ncur = nullptr, *tcur = nullptr, *iters = nullptr, *status = nullptr, *ncont = nullptr,
        *gstat = nullptr, *ii = nullptr;
    unsigned long long* chash = nullptr;
    int steps = 0;  // ckpt_every the buffers were sized for
  } seg;
  // robots grouped by chain-length class (64/128/256/512 links), longest expected work
  // first within a class; each class runs as its own launch on its own stream
  static constexpr int kClasses = 4;
  int* order = nullptr;
  std::vector<int> order_h;  // host copy of the launch order
  int cls_first[kClasses] = {0, 0, 0, 0}, cls_count[kClasses] = {0, 0, 0, 0};
  int waves[kClasses] = {2, 2, 2, 2};  // per robot in the class's rollout launches
  // the order in which the class launches are issued: a launch lasts as long as its
  // slowest robot, so the class holding the slowest robot goes first and its first
  // workgroups (that robot) find the compute units free; longest chains first until
  // measured
  int cls_order[kClasses] = {3, 2, 1, 0};
  std::vector<int> cls_h;     // each robot's class
  std::vector<double> cyc_h;  // each robot's cycles, as vine_sim_tune_order last read them
  // The head: the robots whose measured cycles are at least head_frac of the slowest's,
  // of any class, placed first in the launch order and run as one launch of their own
  // (sized for the longest of them) with head_waves per robot, beside the classes'
  // launches of the rest.  Empty until measured, or with head_frac = 0.
  double head_frac = 0.0;
  int head_waves = 4, head_count = 0, head_links = 0;
  double head_ms[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // the autotuner's whole-batch times
  hipStream_t cls_stream[kClasses] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[kClasses] = {nullptr, nullptr, nullptr, nullptr};
  // vine_sim_rollout_graph: reset + full rollout captured once per (rec_every, ckpt_every)
  hipStream_t cap_stream = nullptr;
  static constexpr int kGraphs = 4;
  hipGraphExec_t graph[kGraphs] = {nullptr, nullptr, nullptr, nullptr};
  int graph_key[kGraphs][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}};
  int trace_robot = -1, trace_cap = 0;
  double* trace = nullptr;
  int* trace_n = nullptr;
  bool traj_valid = false;  // some step since the reset recorded its joint angles
  bool traj_all = true;     // every step since the reset did, with the same rec_every
  bool ckpt_all = true;     // every step since the reset wrote checkpoints (same ckpt_every)
  bool ckpt_any = false;
  void* scratch = nullptr;  // this device's static scratch (vine_sim_grad_noalloc)
  std::string err;
};

namespace {

int fail(vine_sim* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

void drop_graphs(vine_sim* h) {
  for (int k = 0; k < vine_sim::kGraphs; ++k) {
    if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
    h->graph[k] = nullptr;
    h->graph_key[k][0] = h->graph_key[k][1] = -1;
  }
}

void free_seg(vine_sim* h) {
  vine_sim::Seg& g = h->seg;
  void* ptrs[] = {g.theta, g.tip, g.rho, g.maxpen, g.traj, g.jevals, g.nsolves, g.negsteps,
                  g.cycles, g.wtime, g.gsums, g.gloss, g.ncur, g.tcur, g.iters, g.status, g.ncont,
                  g.gstat, g.ii, g.chash, g.tiplen, g.ulast};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  g = vine_sim::Seg();
}

void free_all(vine_sim* h) {
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (int c = 0; c < vine_sim::kClasses; ++c) {
    if (h->cls_stream[c]) (void)hipStreamDestroy(h->cls_stream[c]);
    if (h->ev_join[c]) (void)hipEventDestroy(h->ev_join[c]);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  free_seg(h);
  void* ptrs[] = {h->order, h->ii, h->dd, h->cover, h->spam, h->okind, h->obs, h->tables, h->wr, h->theta,
                  h->ncur, h->tcur, h->tip, h->rho, h->iters, h->status, h->ncont, h->chash,
                  h->maxpen, h->traj, h->ckpt, h->jevals, h->nsolves, h->negsteps, h->cycles,
                  h->wtime, h->tiplen, h->ulast,
                  h->trace, h->trace_n};
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
  k.pd_shift = p.pd_shift;
  k.wg = p.growth_stiffness;
  k.max_iter = p.max_iter;
  k.substeps = p.growth_substeps;
  return k;
}

vs::KData kdata(vine_sim* h) {
  vs::KData D;
  D.n_inst = h->B;
  D.n_max = h->N;
  D.t_max = h->T;
  D.theta_len = h->theta_len;
  D.rec_len = h->rec_len;
  D.skip_done = h->skip_done;
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
  D.tiplen = h->tiplen;
  D.ulast = h->ulast;
  D.traj = nullptr;  // set by the calls that record (advance)
  D.rec_every = h->rec_every;
  D.n_rec = h->n_rec;
  D.ckpt = nullptr;
  D.ckpt_every = h->ckpt_every;
  D.n_ckpt = h->n_ckpt;
  D.jevals = h->jevals;
  D.nsolves = h->nsolves;
  D.negsteps = h->negsteps;
  D.cycles = h->cycles;
  D.wtime = h->wtime;
  D.wall_period = h->wall_period;
  D.trace_robot = h->trace ? h->trace_robot : -1;
  D.order = h->order;
  D.launch_first = 0;
  D.launch_count = 0;
  D.trace_cap = h->trace_cap;
  D.trace = h->trace;
  D.trace_n = h->trace_n;
  return D;
}

constexpr int kClassLinks[vine_sim::kClasses] = {64, 128, 256, 512};

int link_class(int n) {
  int c = 0;
  while (c + 1 < vine_sim::kClasses && n > kClassLinks[c]) ++c;
  return c;
}

// Run launch(links, waves, D) for the head and every non-empty class (links: the class's
// longest chain, waves: per robot in its rollout launches).  A single launch goes on the
// caller's stream; several fork onto the handle's streams, the head first, one stream per
// launch in issue order, and join back, so that short and long chains share the device.
// The caller's stream waits for the joins only once every launch is issued: a stream can
// share a hardware queue with another, and a wait enqueued there earlier would hold back
// the launches issued behind it.
template <typename F>
hipError_t for_each_class(vine_sim* h, hipStream_t stream, vs::KData D, F launch) {
  int used = h->head_count > 0 ? 1 : 0, only = -1;
  for (int c = 0; c < vine_sim::kClasses; ++c)
    if (h->cls_count[c] > 0) {
      ++used;
      only = c;
    }
  if (used <= 1) {
    if (h->head_count > 0) {
      D.launch_first = 0;
      D.launch_count = h->head_count;
      return launch(h->head_links, h->head_waves, D, stream);
    }
    if (only < 0) return hipSuccess;
    D.launch_first = h->cls_first[only];
    D.launch_count = h->cls_count[only];
    return launch(kClassLinks[only], h->waves[only], D, stream);
  }
  hipError_t e = hipEventRecord(h->ev_fork, stream);
  int slot = 0;
  auto fork = [&](int first, int count, int links, int waves) {
    const int k = slot++ % vine_sim::kClasses;  // five launches: the last shares the first's
    hipStream_t cs = h->cls_stream[k];
    e = hipStreamWaitEvent(cs, h->ev_fork, 0);
    D.launch_first = first;
    D.launch_count = count;
    if (e == hipSuccess) e = launch(links, waves, D, cs);
    if (e == hipSuccess) e = hipEventRecord(h->ev_join[k], cs);
  };
  if (e == hipSuccess && h->head_count > 0) fork(0, h->head_count, h->head_links, h->head_waves);
  for (int i = 0; i < vine_sim::kClasses && e == hipSuccess; ++i) {
    const int c = h->cls_order[i];
    if (h->cls_count[c] > 0) fork(h->cls_first[c], h->cls_count[c], kClassLinks[c], h->waves[c]);
  }
  for (int k = 0; k < std::min(slot, vine_sim::kClasses) && e == hipSuccess; ++k)
    e = hipStreamWaitEvent(stream, h->ev_join[k], 0);
  return e;
}

// The launch order from the robots' measured cycles (none measured: the current order):
// the head (robots at or above head_frac of the slowest's cycles, slowest first), then
// each class's other robots, slowest first; the class launches are issued with the class
// of the slowest remaining robot first (ties: longer chains first).  Drops the captured
// rollouts if the order changed, and copies it to the device on stream s.
hipError_t arrange(vine_sim* h, hipStream_t s) {
  const std::vector<double>& cyc = h->cyc_h;
  const bool measured = cyc.size() == (size_t)h->B;
  double top = 0.0;
  if (measured)
    for (double x : cyc) top = std::max(top, x);
  const bool use_head = measured && h->head_frac > 0.0 && top > 0.0;
  std::vector<int> head, cls[vine_sim::kClasses];
  for (int b : h->order_h) {
    if (use_head && cyc[b] >= h->head_frac * top) head.push_back(b);
    else cls[h->cls_h[b]].push_back(b);
  }
  auto slower = [&](int a, int b) { return cyc[a] > cyc[b]; };
  double slowest[vine_sim::kClasses] = {0.0, 0.0, 0.0, 0.0};
  if (measured) {
    std::stable_sort(head.begin(), head.end(), slower);
    for (int c = 0; c < vine_sim::kClasses; ++c) {
      std::stable_sort(cls[c].begin(), cls[c].end(), slower);
      if (!cls[c].empty()) slowest[c] = cyc[cls[c].front()];
    }
  }
  std::vector<int> order(head);
  int links = 0;
  for (int b : head) links = std::max(links, kClassLinks[h->cls_h[b]]);
  for (int c = 0; c < vine_sim::kClasses; ++c) {
    h->cls_first[c] = (int)order.size();
    h->cls_count[c] = (int)cls[c].size();
    order.insert(order.end(), cls[c].begin(), cls[c].end());
  }
  int ord[vine_sim::kClasses] = {3, 2, 1, 0};
  std::stable_sort(ord, ord + vine_sim::kClasses,
                   [&](int a, int b) { return slowest[a] > slowest[b]; });
  bool changed = order != h->order_h || (int)head.size() != h->head_count ||
                 links != h->head_links ||
                 !std::equal(ord, ord + vine_sim::kClasses, h->cls_order);
  h->order_h = order;
  h->head_count = (int)head.size();
  h->head_links = links;
  std::copy(ord, ord + vine_sim::kClasses, h->cls_order);
  if (changed) drop_graphs(h);  // the captures hold the launches
  hipError_t e = hipMemcpyAsync(h->order, h->order_h.data(), sizeof(int) * h->order_h.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

template <typename F>
hipError_t for_each_class(vine_sim* h, hipStream_t stream, F launch) {
  return for_each_class(h, stream, kdata(h), launch);
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
  p->pd_shift = 1e-8;
  p->growth_stiffness = 0.0;
  p->max_iter = 500;
  p->growth_substeps = 2;
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
      !finite_pos(p.step_max) || !(p.armijo_c1 > 0.0 && p.armijo_c1 < 1.0) ||
      !finite_pos(p.pd_shift) || p.max_iter < 0 || p.growth_substeps < 1 ||
      !(p.growth_stiffness >= 0.0) || !std::isfinite(p.growth_stiffness))
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
    for (int s = 0; s < I.spam_count; ++s)
      if (!spam_ok(spams[I.spam_offset + s]))
        return fail(nullptr, VINE_EINVAL, std::string(msg) + "invalid sPAM");
    for (int k = 0; k < I.obs_count; ++k) {
      const vine_obstacle& O = obstacles[I.obs_offset + k];
      if (!(O.kind == 0 || O.kind == 1) || !std::isfinite(O.cx) || !std::isfinite(O.cy) ||
          !finite_pos(O.a) || (O.kind == 1 && !finite_pos(O.b)))
        return fail(nullptr, VINE_EINVAL, std::string(msg) + "invalid obstacle");
    }
    if (I.n_links > N) N = I.n_links;
  }
  vine_sim* h = new (std::nothrow) vine_sim();
  if (!h) return fail(nullptr, VINE_ENOMEM, "host allocation failed");
  h->prm = p;
  h->B = n_inst;
  h->N = N;
  h->T = N;
  h->S = n_spams;
  h->theta_len = (long long)n_inst * N;
  h->rec_len = (long long)n_inst * N;
  // host-side derived inputs
  std::vector<int> ii(vs::kII * (size_t)n_inst);
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
    int* row = ii.data() + vs::kII * (size_t)b;
    row[vs::kNTarget] = I.n_links;
    row[vs::kObsOff] = (int)okind.size();
    row[vs::kObsCnt] = I.obs_count;
    row[vs::kTableId] = tid;
    row[vs::kCoverOff] = (int)(cover.size() / 2);
    row[vs::kSpamOff] = I.spam_offset;
    row[vs::kSpamCnt] = I.spam_count;
    row[vs::kThetaOff] = b * N;  // N = T: every robot gets a row of each
    row[vs::kRecOff] = b * N;
    row[vs::kRecCap] = N;
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
    append_cover(I, spams, cover);
  }
  h->inst_h.assign(inst, inst + n_inst);
  {
    // FNV-1a over the parameters and the inputs: the key of the autotuner's cache
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void* data, size_t bytes) {
      const unsigned char* q = (const unsigned char*)data;
      for (size_t i = 0; i < bytes; ++i) x = (x ^ q[i]) * 1099511628211ull;
    };
    mix(&p, sizeof(p));
    mix(inst, sizeof(vine_instance) * (size_t)n_inst);
    if (n_spams > 0) mix(spams, sizeof(vine_spam) * (size_t)n_spams);
    if (n_obstacles > 0) mix(obstacles, sizeof(vine_obstacle) * (size_t)n_obstacles);
    h->config_hash = x;
  }
  // launch order: by class, then by decreasing n^2 (4 + K), a proxy of the work
  std::vector<int> order(n_inst);
  for (int b = 0; b < n_inst; ++b) order[b] = b;
  auto cost = [&](int b) {
    return (double)inst[b].n_links * inst[b].n_links * (4.0 + inst[b].obs_count);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ca = link_class(inst[a].n_links), cb = link_class(inst[b].n_links);
    if (ca != cb) return ca < cb;
    return cost(a) > cost(b);
  });
  h->cls_h.resize(n_inst);
  for (int b = 0; b < n_inst; ++b) {
    h->cls_h[b] = link_class(inst[b].n_links);
    h->cls_count[h->cls_h[b]]++;
  }
  for (int c = 1; c < vine_sim::kClasses; ++c)
    h->cls_first[c] = h->cls_first[c - 1] + h->cls_count[c - 1];
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
  A(dalloc(&h->order, order.size()));
  for (int c = 0; c < vine_sim::kClasses; ++c) {
    A(hipStreamCreateWithFlags(&h->cls_stream[c], hipStreamNonBlocking));
    A(hipEventCreateWithFlags(&h->ev_join[c], hipEventDisableTiming));
  }
  A(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
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
  A(dalloc(&h->tiplen, B * TT));
  A(dalloc(&h->ulast, B));
  A(dalloc(&h->jevals, B));
  A(dalloc(&h->nsolves, B));
  A(dalloc(&h->negsteps, B));
  A(dalloc(&h->cycles, B));
  A(dalloc(&h->wtime, B));
  {
    int dev = 0, khz = 0;
    A(hipGetDevice(&dev));
    A(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    h->wall_period = khz > 0 ? 1e-3 / khz : 0.0;
  }
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("device allocation: ") + hipGetErrorString(e));
  }
  A(hipMemcpy(h->order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
  h->order_h = order;
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
  // this device's static scratch for vine_sim_grad_noalloc (looked up once per device)
  if (vs::scratch_address(&h->scratch) != hipSuccess) {
    free_all(h);
    delete h;
    return fail(nullptr, VINE_EDEVICE, "device scratch address");
  }
  *out = h;
  return VINE_OK;
}

int32_t vine_sim_reset(vine_sim* h, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  const hipError_t e = vs::launch_reset(kdata(h), (hipStream_t)stream);
  h->traj_valid = false;
  h->traj_all = true;
  h->ckpt_any = false;
  h->ckpt_all = true;
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("reset: ") + hipGetErrorString(e));
  return VINE_OK;
}

// The trajectory buffer for rec_every (B x ceil(T / rec_every) x N doubles), allocated
// on first use and again when rec_every changes (the recorded rows are then invalid).
static int32_t ensure_traj(vine_sim* h, int rec_every) {
  if (h->traj && h->rec_every == rec_every) return VINE_OK;
  if (h->traj) (void)hipFree(h->traj);
  h->traj = nullptr;
  h->traj_valid = false;
  drop_graphs(h);  // captured launches hold the buffer's address
  const int rows = (h->T + rec_every - 1) / rec_every;
  hipError_t e = dalloc(&h->traj, (size_t)h->B * rows * h->N);
  if (e != hipSuccess) {
    h->traj = nullptr;
    h->rec_every = h->n_rec = 0;
    return fail(h, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("trajectory allocation: ") + hipGetErrorString(e));
  }
  h->rec_every = rec_every;
  h->n_rec = rows;
  return VINE_OK;
}

// The checkpoint buffer for ckpt_every (B x ceil(T / ckpt_every) x N doubles).
static int32_t ensure_ckpt(vine_sim* h, int ckpt_every) {
  if (h->ckpt && h->ckpt_every == ckpt_every) return VINE_OK;
  if (h->ckpt) (void)hipFree(h->ckpt);
  h->ckpt = nullptr;
  h->ckpt_any = false;
  drop_graphs(h);
  const int rows = (h->T + ckpt_every - 1) / ckpt_every;
  hipError_t e = dalloc(&h->ckpt, (size_t)h->B * rows * h->N);
  if (e != hipSuccess) {
    h->ckpt = nullptr;
    h->ckpt_every = h->n_ckpt = 0;
    return fail(h, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("checkpoint allocation: ") + hipGetErrorString(e));
  }
  h->ckpt_every = ckpt_every;
  h->n_ckpt = rows;
  return VINE_OK;
}

// KData of a launch that records every rec_every-th step (0: none) and checkpoints
// every ckpt_every-th (0: none); the buffers must exist.
static vs::KData kdata_rec(vine_sim* h, int rec_every, int ckpt_every) {
  vs::KData D = kdata(h);
  if (rec_every > 0) D.traj = h->traj;
  if (ckpt_every > 0) D.ckpt = h->ckpt;
  return D;
}

static int32_t check_rec(vine_sim* h, int32_t record_every, int32_t ckpt_every) {
  if (record_every < 0 || ckpt_every < 0)
    return fail(h, VINE_EINVAL, "record_every and ckpt_every must be >= 0");
  if (record_every > 0) {
    const int32_t r = ensure_traj(h, record_every);
    if (r != VINE_OK) return r;
  }
  if (ckpt_every > 0) {
    const int32_t r = ensure_ckpt(h, ckpt_every);
    if (r != VINE_OK) return r;
  }
  return VINE_OK;
}

static void note_rec(vine_sim* h, int32_t record_every, int32_t ckpt_every) {
  if (record_every > 0) h->traj_valid = true; else h->traj_all = false;
  if (ckpt_every > 0) h->ckpt_any = true; else h->ckpt_all = false;
}

static int32_t advance(vine_sim* h, int32_t n_steps, int32_t record_every, int32_t ckpt_every,
                       void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (n_steps < 0) n_steps = h->T;
  int32_t r = check_rec(h, record_every, ckpt_every);
  if (r != VINE_OK) return r;
  if (n_steps == 0) return VINE_OK;
  const vs::KParams kp = kparams(h->prm);
  hipError_t e = for_each_class(h, (hipStream_t)stream, kdata_rec(h, record_every, ckpt_every),
                                [&](int links, int waves, const vs::KData& D, hipStream_t s) {
                                  return vs::launch_rollout(kp, D, n_steps, links,
                                                            waves, s);
                                });
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  note_rec(h, record_every, ckpt_every);
  return VINE_OK;
}

int32_t vine_sim_step(vine_sim* h, int32_t n_steps, int32_t record_every, int32_t ckpt_every,
                      void* stream) {
  if (n_steps < 0) return fail(h, VINE_EINVAL, "n_steps < 0");
  return advance(h, n_steps, record_every, ckpt_every, stream);
}

int32_t vine_sim_rollout(vine_sim* h, int32_t n_steps, int32_t record_every, int32_t ckpt_every,
                         void* stream) {
  return advance(h, n_steps < 0 ? -1 : n_steps, record_every, ckpt_every, stream);
}

int32_t vine_sim_tune_order(vine_sim* h, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> cyc(h->B);
  hipError_t e = hipMemcpyAsync(cyc.data(), h->cycles, sizeof(double) * h->B,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("read cycles: ") + hipGetErrorString(e));
  h->cyc_h = cyc;
  e = arrange(h, s);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("write order: ") + hipGetErrorString(e));
  return VINE_OK;
}

int32_t vine_sim_set_head(vine_sim* h, double fraction, int32_t waves, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (!(fraction >= 0.0 && fraction <= 1.0))
    return fail(h, VINE_EINVAL, "head fraction must be in [0, 1]");
  if (waves != 1 && waves != 2 && waves != 4)
    return fail(h, VINE_EINVAL, "waves per robot must be 1, 2 or 4");
  h->head_frac = fraction;
  if (h->head_waves != waves) drop_graphs(h);
  h->head_waves = waves;
  hipError_t e = arrange(h, (hipStream_t)stream);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("write order: ") + hipGetErrorString(e));
  return VINE_OK;
}

int32_t vine_sim_head(const vine_sim* h, double* fraction, int32_t* waves, int32_t* count,
                      double ms[6]) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (fraction) *fraction = h->head_frac;
  if (waves) *waves = h->head_waves;
  if (count) *count = h->head_count;
  if (ms)
    for (int k = 0; k < 6; ++k) ms[k] = h->head_ms[k];
  return VINE_OK;
}

int32_t vine_sim_set_waves(vine_sim* h, const int32_t waves[4]) {
  if (!h || !waves) return fail(h, VINE_EINVAL, "null handle or waves");
  for (int c = 0; c < vine_sim::kClasses; ++c)
    if (waves[c] != 1 && waves[c] != 2 && waves[c] != 4)
      return fail(h, VINE_EINVAL, "waves per robot must be 1, 2 or 4");
  bool changed = false;
  for (int c = 0; c < vine_sim::kClasses; ++c) {
    changed = changed || h->waves[c] != waves[c];
    h->waves[c] = waves[c];
  }
  if (changed) drop_graphs(h);  // the captures hold the launches' block sizes
  return VINE_OK;
}

namespace {
// the autotuner's choices, per configuration (hash of the parameters and inputs)
struct Tuned {
  std::array<int32_t, vine_sim::kClasses> waves;
  double head_frac;
  bool head_tuned;  // the head was measured (needs the robots' measured cycles)
};
std::mutex g_tune_mu;
std::map<uint64_t, Tuned> g_tune;
}  // namespace

int32_t vine_sim_autotune(vine_sim* h, int32_t waves[4], double ms[12], int32_t* cached,
                          void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  hipStream_t s = (hipStream_t)stream;
  Tuned best{{2, 2, 2, 2}, 0.0, false};
  double t[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double th[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  bool hit = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(h->config_hash);
    if (it != g_tune.end()) {
      best = it->second;
      hit = true;
    }
  }
  const bool measured = h->cyc_h.size() == (size_t)h->B;
  const bool tune_head = measured && !(hit && best.head_tuned);
  hipError_t e = hipSuccess;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!hit || tune_head) {
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
  }
  const vs::KParams kp = kparams(h->prm);
  if (!hit) {
    // each class alone (the head dissolved), from zero length to full, with 1, 2 and 4
    // waves per robot
    h->head_frac = 0.0;
    if (e == hipSuccess) e = arrange(h, s);
    for (int c = 0; c < vine_sim::kClasses && e == hipSuccess; ++c) {
      if (h->cls_count[c] == 0) continue;
      vs::KData D = kdata(h);
      D.launch_first = h->cls_first[c];
      D.launch_count = h->cls_count[c];
      const int ws[3] = {1, 2, 4};
      for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        e = vs::launch_reset(kdata(h), s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = vs::launch_rollout(kp, D, h->T, kClassLinks[c], ws[k], s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        t[3 * c + k] = f;
      }
      // the fastest; two waves (the default) unless another measured faster
      best.waves[c] = 2;
      double tb = t[3 * c + 1];
      if (t[3 * c] < tb) {
        best.waves[c] = 1;
        tb = t[3 * c];
      }
      if (t[3 * c + 2] < tb) best.waves[c] = 4;
    }
  }
  auto set_waves = [&](const std::array<int32_t, vine_sim::kClasses>& w) {
    for (int c = 0; c < vine_sim::kClasses; ++c) {
      if (h->waves[c] != w[c]) drop_graphs(h);
      h->waves[c] = w[c];
    }
  };
  if (h->head_waves != 4) drop_graphs(h);
  h->head_waves = 4;
  if (tune_head) {
    // The whole batch as it is launched: the classes with their fastest wave counts alone,
    // or with two waves each, and with no head or with the robots at or above 1/2 or 1/4
    // of the slowest's measured cycles in a head of four waves per robot.  The batch lasts
    // at least as long as its slowest robot, which more waves shorten, while fewer waves
    // per robot keep more robots on the device; which balance wins depends on the batch.
    const std::array<int32_t, vine_sim::kClasses> cand[2] = {best.waves, {2, 2, 2, 2}};
    const double fr[3] = {0.0, 0.5, 0.25};
    int kb = 0;  // the fastest (ties: the earlier candidate)
    for (int k = 0; k < 6 && e == hipSuccess; ++k) {
      if (k >= 3 && cand[1] == cand[0]) break;
      set_waves(cand[k / 3]);
      h->head_frac = fr[k % 3];
      e = arrange(h, s);
      if (e == hipSuccess) e = vs::launch_reset(kdata(h), s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = for_each_class(h, s, [&](int links, int w, const vs::KData& D, hipStream_t cs) {
          return vs::launch_rollout(kp, D, h->T, links, w, cs);
        });
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float f = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
      th[k] = f;
      if (th[k] < th[kb]) kb = k;
    }
    best.waves = cand[kb / 3];
    best.head_frac = fr[kb % 3];
    best.head_tuned = true;
  }
  set_waves(best.waves);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!hit || tune_head) {  // the measurements ran rollouts: end reset
    if (e == hipSuccess) e = vs::launch_reset(kdata(h), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    h->traj_valid = false;
    h->traj_all = h->ckpt_all = true;
    h->ckpt_any = false;
  }
  h->head_frac = best.head_frac;
  if (e == hipSuccess) e = arrange(h, s);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  if (!hit || tune_head) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[h->config_hash] = best;
  }
  for (int k = 0; k < 6; ++k) h->head_ms[k] = th[k];
  if (waves) {
    bool present[vine_sim::kClasses] = {false, false, false, false};
    for (int c : h->cls_h) present[c] = true;
    for (int c = 0; c < vine_sim::kClasses; ++c) waves[c] = present[c] ? best.waves[c] : 0;
  }
  if (ms)
    for (int k = 0; k < 12; ++k) ms[k] = t[k];
  if (cached) *cached = hit ? 1 : 0;
  return VINE_OK;
}

int32_t vine_sim_rollout_graph(vine_sim* h, int32_t record_every, int32_t ckpt_every,
                               void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  int32_t r = check_rec(h, record_every, ckpt_every);
  if (r != VINE_OK) return r;
  int g = -1;
  for (int k = 0; k < vine_sim::kGraphs; ++k)
    if (h->graph[k] && h->graph_key[k][0] == record_every && h->graph_key[k][1] == ckpt_every)
      g = k;
  if (g < 0) {
    for (int k = 0; k < vine_sim::kGraphs && g < 0; ++k)
      if (!h->graph[k]) g = k;
    if (g < 0) {  // all slots taken: drop the oldest capture
      (void)hipGraphExecDestroy(h->graph[0]);
      for (int k = 1; k < vine_sim::kGraphs; ++k) {
        h->graph[k - 1] = h->graph[k];
        h->graph_key[k - 1][0] = h->graph_key[k][0];
        h->graph_key[k - 1][1] = h->graph_key[k][1];
      }
      g = vine_sim::kGraphs - 1;
      h->graph[g] = nullptr;
    }
    // capture on a stream of the handle's own (the caller's may be the null stream);
    // the class streams join the capture through the fork/join events
    hipError_t e = hipSuccess;
    if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const vs::KParams kp = kparams(h->prm);
      hipError_t le = vs::launch_reset(kdata(h), h->cap_stream);
      if (le == hipSuccess)
        le = for_each_class(h, h->cap_stream, kdata_rec(h, record_every, ckpt_every),
                            [&](int links, int waves, const vs::KData& D, hipStream_t s) {
                              return vs::launch_rollout(kp, D, h->T, links,
                                                        waves, s);
                            });
      e = hipStreamEndCapture(h->cap_stream, &graph);  // ends the capture in every case
      if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&h->graph[g], graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      h->graph[g] = nullptr;
      return fail(h, VINE_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    h->graph_key[g][0] = record_every;
    h->graph_key[g][1] = ckpt_every;
  }
  const hipError_t e = hipGraphLaunch(h->graph[g], (hipStream_t)stream);
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  // as after vine_sim_reset + vine_sim_rollout
  h->traj_valid = record_every > 0;
  h->traj_all = record_every > 0;
  h->ckpt_any = ckpt_every > 0;
  h->ckpt_all = ckpt_every > 0;
  return VINE_OK;
}

// Segment buffers for recomputing ckpt_every steps from a checkpoint.
static hipError_t ensure_seg(vine_sim* h) {
  vine_sim::Seg& g = h->seg;
  if (g.theta && g.steps == h->ckpt_every) return hipSuccess;
  free_seg(h);
  const size_t B = h->B, N = h->N, C = h->ckpt_every;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&g.theta, B * N));
  A(dalloc(&g.ncur, B));
  A(dalloc(&g.tcur, B));
  A(dalloc(&g.tip, B * C * 3));
  A(dalloc(&g.rho, B * C));
  A(dalloc(&g.iters, B * C));
  A(dalloc(&g.status, B * C));
  A(dalloc(&g.ncont, B * C));
  A(dalloc(&g.chash, B * C));
  A(dalloc(&g.maxpen, B * C));
  A(dalloc(&g.tiplen, B * C));
  A(dalloc(&g.ulast, B));
  A(dalloc(&g.traj, B * C * N));
  A(dalloc(&g.jevals, B));
  A(dalloc(&g.nsolves, B));
  A(dalloc(&g.negsteps, B));
  A(dalloc(&g.cycles, B));
  A(dalloc(&g.wtime, B));
  A(dalloc(&g.gsums, B * vs::kWave * 3));
  A(dalloc(&g.gloss, B));
  A(dalloc(&g.gstat, B));
  A(dalloc(&g.ii, B * vs::kII));
  if (e != hipSuccess) {
    free_seg(h);
    return e;
  }
  g.steps = h->ckpt_every;
  return hipSuccess;
}

// Views of the segment buffers inside one block of device memory of `bytes` bytes (each
// array 256-byte aligned); false when they do not fit.
static bool seg_view(void* base, size_t bytes, size_t B, size_t N, size_t C, vine_sim::Seg* g) {
  size_t off = 0;
  auto take = [&](auto** p, size_t count) {
    off = (off + 255) & ~(size_t)255;
    *p = reinterpret_cast<std::remove_reference_t<decltype(**p)>*>((char*)base + off);
    off += sizeof(**p) * (count > 0 ? count : 1);
  };
  take(&g->theta, B * N);
  take(&g->ncur, B);
  take(&g->tcur, B);
  take(&g->tip, B * C * 3);
  take(&g->rho, B * C);
  take(&g->iters, B * C);
  take(&g->status, B * C);
  take(&g->ncont, B * C);
  take(&g->chash, B * C);
  take(&g->maxpen, B * C);
  take(&g->tiplen, B * C);
  take(&g->ulast, B);
  take(&g->traj, B * C * N);
  take(&g->jevals, B);
  take(&g->nsolves, B);
  take(&g->negsteps, B);
  take(&g->cycles, B);
  take(&g->wtime, B);
  take(&g->gsums, B * vs::kWave * 3);
  take(&g->gloss, B);
  take(&g->gstat, B);
  take(&g->ii, B * vs::kII);
  g->steps = (int)C;
  return off <= bytes;
}

// vine_sim_grad with the segment buffers of the checkpoint path in g (null: allocated in
// the handle on first use).
static int32_t grad_impl(vine_sim* h, const double* goal, const double* step_weights,
                         double* dL_dP, double* dL_ds_start, double* dL_ds_end, double* loss,
                         int32_t* adj_status, void* stream, const vine_sim::Seg* g) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (!goal || !loss || (h->S > 0 && (!dL_dP || !dL_ds_start || !dL_ds_end)))
    return fail(h, VINE_EINVAL, "null goal, loss or gradient pointer");
  if (h->prm.growth_stiffness > 0.0)
    return fail(h, VINE_ESTATE, "the adjoint covers hard growth only (growth_stiffness = 0)");
  const bool full_traj = h->traj_valid && h->traj_all && h->rec_every == 1;
  const bool from_ckpt = h->ckpt && h->ckpt_any && h->ckpt_all;
  if (step_weights && !full_traj && !from_ckpt)
    return fail(h, VINE_ESTATE,
                "step weights need the joint angles of every step since the reset: record "
                "every step (record_every = 1) or checkpoints (ckpt_every > 0) on every "
                "step/rollout call");
  hipStream_t s = (hipStream_t)stream;
  const vs::KParams kp = kparams(h->prm);
  hipError_t e = hipSuccess;
  if (step_weights && !full_traj && !g) {
    e = ensure_seg(h);
    if (e != hipSuccess)
      return fail(h, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                  std::string("segment allocation: ") + hipGetErrorString(e));
    g = &h->seg;
  }
  e = vs::launch_zero3(dL_dP, dL_ds_start, dL_ds_end, h->S, s);
  if (e == hipSuccess && (!step_weights || full_traj)) {
    const vs::GradPart one{nullptr, nullptr, nullptr, 1, 1};
    e = for_each_class(h, s, [&](int links, int, const vs::KData& D, hipStream_t cs) {
      return vs::launch_grad(kp, D, goal, step_weights, h->T, 0, h->traj, h->n_rec, one, dL_dP,
                             dL_ds_start, dL_ds_end, loss, adj_status, links, cs);
    });
  } else if (e == hipSuccess) {
    // recompute the states of each checkpoint segment (the same kernel from the same
    // state, so bitwise the states of the rollout), then its terms of the adjoint
    vs::KData Dseg = kdata(h);
    Dseg.t_max = h->ckpt_every;
    Dseg.ii = g->ii;  // the handle's robot rows with the segment's record fields
    Dseg.theta = g->theta;
    Dseg.ncur = g->ncur;
    Dseg.tcur = g->tcur;
    Dseg.tip = g->tip;
    Dseg.rho = g->rho;
    Dseg.iters = g->iters;
    Dseg.status = g->status;
    Dseg.ncont = g->ncont;
    Dseg.chash = g->chash;
    Dseg.maxpen = g->maxpen;
    Dseg.tiplen = g->tiplen;
    Dseg.ulast = g->ulast;
    Dseg.traj = g->traj;
    Dseg.rec_every = 1;
    Dseg.n_rec = h->ckpt_every;
    Dseg.ckpt = nullptr;
    Dseg.jevals = g->jevals;
    Dseg.nsolves = g->nsolves;
    Dseg.negsteps = g->negsteps;
    Dseg.cycles = g->cycles;
    Dseg.wtime = g->wtime;
    Dseg.trace_robot = -1;
    const int ce = h->ckpt_every;
    for (int q = 0; q < h->n_ckpt && e == hipSuccess; ++q) {
      const int t0 = q * ce, len = std::min(ce, h->T - t0);
      e = vs::launch_seg_load(Dseg, h->ii, h->ckpt, h->tcur, h->n_ckpt, q, ce, s);
      if (e == hipSuccess)
        e = for_each_class(h, s, Dseg, [&](int links, int waves, const vs::KData& D, hipStream_t cs) {
          return vs::launch_rollout(kp, D, len, links, waves, cs);
        });
      const vs::GradPart part{g->gsums, g->gloss, g->gstat, q == 0, q == h->n_ckpt - 1};
      if (e == hipSuccess)
        e = for_each_class(h, s, [&](int links, int, const vs::KData& D, hipStream_t cs) {
          return vs::launch_grad(kp, D, goal, step_weights + t0, len, t0, g->traj, ce, part,
                                 dL_dP, dL_ds_start, dL_ds_end, loss, adj_status, links, cs);
        });
    }
  }
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return VINE_OK;
}

int32_t vine_sim_grad(vine_sim* h, const double* goal, const double* step_weights,
                      double* dL_dP, double* dL_ds_start, double* dL_ds_end, double* loss,
                      int32_t* adj_status, void* stream) {
  return grad_impl(h, goal, step_weights, dL_dP, dL_ds_start, dL_ds_end, loss, adj_status,
                   stream, nullptr);
}

int32_t vine_sim_grad_noalloc(vine_sim* h, const double* goal, const double* step_weights,
                              double* dL_dP, double* dL_ds_start, double* dL_ds_end,
                              double* loss, int32_t* adj_status, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  const bool full_traj = h->traj_valid && h->traj_all && h->rec_every == 1;
  if (!step_weights || full_traj || !(h->ckpt && h->ckpt_any && h->ckpt_all))
    return grad_impl(h, goal, step_weights, dL_dP, dL_ds_start, dL_ds_end, loss, adj_status,
                     stream, nullptr);  // no segment buffers needed (or the state error)
  if (!h->scratch) return fail(h, VINE_EDEVICE, "no device scratch for this handle's device");
  vine_sim::Seg view;
  if (!seg_view(h->scratch, VINE_GRAD_SCRATCH_BYTES, h->B, h->N, h->ckpt_every, &view)) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "the segment buffers of %d robots x %d links x %d steps per checkpoint exceed "
                  "the %llu-byte device scratch (use vine_sim_grad)",
                  h->B, h->N, h->ckpt_every, (unsigned long long)VINE_GRAD_SCRATCH_BYTES);
    return fail(h, VINE_ECAPACITY, msg);
  }
  return grad_impl(h, goal, step_weights, dL_dP, dL_ds_start, dL_ds_end, loss, adj_status,
                   stream, &view);
}

int32_t vine_sim_set_spams(vine_sim* h, const vine_spam* spams, int32_t n_spams, void* stream) {
  if (!h) return fail(nullptr, VINE_EINVAL, "null handle");
  if (n_spams != h->S || (n_spams > 0 && !spams))
    return fail(h, VINE_EINVAL, "n_spams differs from the count given at create");
  for (int i = 0; i < n_spams; ++i)
    if (!spam_ok(spams[i])) return fail(h, VINE_EINVAL, "invalid sPAM");
  std::vector<double> cover, sp(4 * (size_t)n_spams);
  for (const vine_instance& I : h->inst_h) append_cover(I, spams, cover);
  for (int i = 0; i < n_spams; ++i) {
    sp[4 * i + 0] = spams[i].s_start;
    sp[4 * i + 1] = spams[i].s_end;
    sp[4 * i + 2] = spams[i].side;
    sp[4 * i + 3] = spams[i].pressure;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  // ordered after the work already queued on the stream; the host buffers are
  // released only once the copies are done
  if (!cover.empty())
    A(hipMemcpyAsync(h->cover, cover.data(), sizeof(double) * cover.size(),
                     hipMemcpyHostToDevice, s));
  if (n_spams > 0)
    A(hipMemcpyAsync(h->spam, sp.data(), sizeof(double) * sp.size(), hipMemcpyHostToDevice, s));
  A(hipStreamSynchronize(s));
  if (e != hipSuccess) return fail(h, VINE_EDEVICE, std::string("set_spams: ") + hipGetErrorString(e));
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
    case VINE_F_TRAJ: return 8 * B * h->n_rec * N;
    case VINE_F_JEVALS: return 8 * B;
    case VINE_F_NSOLVES: return 8 * B;
    case VINE_F_CYCLES: return 8 * B;
    case VINE_F_NEGSTEPS: return 8 * B;
    case VINE_F_TIME: return 8 * B;
    case VINE_F_CKPT: return 8 * B * h->n_ckpt * N;
    case VINE_F_TIPLEN: return 8 * B * T;
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
    case VINE_F_CYCLES: src = h->cycles; break;
    case VINE_F_TIME: src = h->wtime; break;
    case VINE_F_NEGSTEPS: src = h->negsteps; break;
    case VINE_F_CKPT:
      if (!h->ckpt_any) return fail(h, VINE_ESTATE, "no checkpoints were written");
      src = h->ckpt;
      break;
    case VINE_F_TIPLEN: src = h->tiplen; break;
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
  drop_graphs(h);  // captured launches hold the trace buffer's address
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

int32_t vine_sim_occupancy(int32_t waves, int32_t per_cu[4], int32_t* compute_units) {
  if (waves != 1 && waves != 2 && waves != 4)
    return fail(nullptr, VINE_EINVAL, "waves per robot must be 1, 2 or 4");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (int c = 0; c < vine_sim::kClasses && e == hipSuccess; ++c) {
    int k = 0;
    e = vs::rollout_occupancy(kClassLinks[c], waves, &k);
    if (per_cu) per_cu[c] = k;
  }
  if (e != hipSuccess) return fail(nullptr, VINE_EDEVICE, std::string("occupancy: ") + hipGetErrorString(e));
  if (compute_units) *compute_units = cus;
  return VINE_OK;
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

int32_t vine_spam_synth(const vine_params* params, double link_len, double tube_radius,
                        double body_pressure, const double* pressures, int32_t n_pressures,
                        const double* unit_lengths, int32_t n_lengths, const double* targets,
                        int32_t n_targets, double tol, double* designs, double* angles,
                        void* stream) {
  if (!params || !pressures || !unit_lengths || n_pressures < 1 || n_lengths < 1 ||
      n_targets < 0 || (n_targets > 0 && (!targets || !designs)))
    return fail(nullptr, VINE_EINVAL, "null pointer or non-positive count");
  if (n_pressures > VINE_SYNTH_MAX || n_lengths > VINE_SYNTH_MAX)
    return fail(nullptr, VINE_ECAPACITY, "more pressures or unit lengths than VINE_SYNTH_MAX");
  const vine_params& p = *params;
  if (!finite_pos(p.R_c) || !finite_pos(p.R_act) || !(p.R_act > p.R_c) || !(p.a_corr >= 0.0) ||
      !std::isfinite(p.a_corr) || !(p.eps_crit > 0.0 && p.eps_crit < 1.0))
    return fail(nullptr, VINE_EINVAL, "invalid vine_params");
  if (!finite_pos(link_len) || !finite_pos(tube_radius) || !finite_pos(body_pressure) ||
      !(tol >= 0.0) || !std::isfinite(tol))
    return fail(nullptr, VINE_EINVAL, "invalid link length, tube radius, body pressure or tolerance");
  for (int k = 0; k < n_pressures; ++k)
    if (!finite_pos(pressures[k]) || (k > 0 && !(pressures[k] > pressures[k - 1])))
      return fail(nullptr, VINE_EINVAL, "pressures must be positive, finite and rising");
  for (int j = 0; j < n_lengths; ++j)
    if (!finite_pos(unit_lengths[j]) || (j > 0 && !(unit_lengths[j] > unit_lengths[j - 1])))
      return fail(nullptr, VINE_EINVAL, "unit lengths must be positive, finite and rising");
  for (int i = 0; i < n_targets; ++i)
    if (!std::isfinite(targets[i])) return fail(nullptr, VINE_EINVAL, "non-finite target angle");
  // the quadrature rule of the elliptic integrals (Eq. 1), nodes then weights
  const GaussRule& g48 = gauss48();
  std::vector<double> gl(g48.x);
  gl.insert(gl.end(), g48.w.begin(), g48.w.end());
  hipStream_t st = (hipStream_t)stream;
  double *d_gl = nullptr, *d_p = nullptr, *d_l = nullptr, *d_ang = nullptr, *d_t = nullptr,
         *d_des = nullptr;
  const size_t na = (size_t)n_pressures * n_lengths;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&d_gl, gl.size()));
  A(dalloc(&d_p, (size_t)n_pressures));
  A(dalloc(&d_l, (size_t)n_lengths));
  A(dalloc(&d_ang, na));
  if (n_targets > 0) {
    A(dalloc(&d_t, (size_t)n_targets));
    A(dalloc(&d_des, 3 * (size_t)n_targets));
  }
  if (e == hipSuccess) {
    A(hipMemcpyAsync(d_gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(d_p, pressures, sizeof(double) * n_pressures, hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(d_l, unit_lengths, sizeof(double) * n_lengths, hipMemcpyHostToDevice, st));
    if (n_targets > 0)
      A(hipMemcpyAsync(d_t, targets, sizeof(double) * n_targets, hipMemcpyHostToDevice, st));
    vs::SynthArgs a{d_gl, d_gl + 48, d_p, d_l, d_ang, n_pressures, n_lengths, p.R_c, p.R_act,
                    p.a_corr, link_len, 2.0 * tube_radius + p.R_act,
                    kPi * body_pressure * tube_radius * tube_radius * tube_radius, p.eps_crit};
    A(vs::launch_synth_angles(a, st));
    A(vs::launch_synth_select(a, d_t, n_targets, tol, d_des, st));
    if (angles) A(hipMemcpyAsync(angles, d_ang, sizeof(double) * na, hipMemcpyDeviceToHost, st));
    if (n_targets > 0)
      A(hipMemcpyAsync(designs, d_des, sizeof(double) * 3 * n_targets, hipMemcpyDeviceToHost, st));
    A(hipStreamSynchronize(st));
  }
  const bool oom = e == hipErrorOutOfMemory;
  void* bufs[] = {d_gl, d_p, d_l, d_ang, d_t, d_des};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (e != hipSuccess)
    return fail(nullptr, oom ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("synthesis: ") + hipGetErrorString(e));
  return VINE_OK;
}

int32_t vine_spam_solve(const vine_params* params, int32_t n, const double* eps,
                        const double* unit_lengths, double* out, void* stream) {
  if (!params || n < 0 || (n > 0 && (!eps || !unit_lengths || !out)))
    return fail(nullptr, VINE_EINVAL, "null pointer or negative count");
  const vine_params& p = *params;
  if (!finite_pos(p.R_c) || !finite_pos(p.R_act) || !(p.R_act > p.R_c) || !(p.a_corr >= 0.0) ||
      !std::isfinite(p.a_corr))
    return fail(nullptr, VINE_EINVAL, "invalid vine_params");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(eps[i]) || !finite_pos(unit_lengths[i]))
      return fail(nullptr, VINE_EINVAL, "non-finite strain or non-positive unit length");
  if (n == 0) return VINE_OK;
  const GaussRule& g48 = gauss48();
  std::vector<double> gl(g48.x);
  gl.insert(gl.end(), g48.w.begin(), g48.w.end());
  hipStream_t st = (hipStream_t)stream;
  double *d_gl = nullptr, *d_e = nullptr, *d_l = nullptr, *d_o = nullptr;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&d_gl, gl.size()));
  A(dalloc(&d_e, (size_t)n));
  A(dalloc(&d_l, (size_t)n));
  A(dalloc(&d_o, 4 * (size_t)n));
  if (e == hipSuccess) {
    A(hipMemcpyAsync(d_gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(d_e, eps, sizeof(double) * n, hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(d_l, unit_lengths, sizeof(double) * n, hipMemcpyHostToDevice, st));
    vs::SynthArgs a{d_gl, d_gl + 48, nullptr, nullptr, nullptr, 0, 0, p.R_c, p.R_act, p.a_corr,
                    0.0, 0.0, 0.0, 0.0};
    A(vs::launch_spam_solve(a, d_e, d_l, n, d_o, st));
    A(hipMemcpyAsync(out, d_o, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st));
    A(hipStreamSynchronize(st));
  }
  const bool oom = e == hipErrorOutOfMemory;
  void* bufs[] = {d_gl, d_e, d_l, d_o};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (e != hipSuccess)
    return fail(nullptr, oom ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("sPAM solve: ") + hipGetErrorString(e));
  return VINE_OK;
}

int32_t vine_mlp_forward(const double* weights, int32_t n, const double* x, double* y,
                         void* stream) {
  if (!weights || n < 0 || (n > 0 && (!x || !y)))
    return fail(nullptr, VINE_EINVAL, "null pointer or negative count");
  for (int k = 0; k < VINE_MLP_WEIGHTS; ++k)
    if (!std::isfinite(weights[k])) return fail(nullptr, VINE_EINVAL, "non-finite weight");
  if (n == 0) return VINE_OK;
  hipStream_t st = (hipStream_t)stream;
  double *d_w = nullptr, *d_x = nullptr, *d_y = nullptr;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  A(dalloc(&d_w, (size_t)VINE_MLP_WEIGHTS));
  A(dalloc(&d_x, 2 * (size_t)n));
  A(dalloc(&d_y, 2 * (size_t)n));
  if (e == hipSuccess) {
    A(hipMemcpyAsync(d_w, weights, sizeof(double) * VINE_MLP_WEIGHTS, hipMemcpyHostToDevice, st));
    A(hipMemcpyAsync(d_x, x, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
    A(vs::launch_mlp_forward(d_w, d_x, n, d_y, st));
    A(hipMemcpyAsync(y, d_y, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
    A(hipStreamSynchronize(st));
  }
  const bool oom = e == hipErrorOutOfMemory;
  void* bufs[] = {d_w, d_x, d_y};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (e != hipSuccess)
    return fail(nullptr, oom ? VINE_ENOMEM : VINE_EDEVICE,
                std::string("surrogate: ") + hipGetErrorString(e));
  return VINE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching over a slab of resident robots.  The slab's per-robot
// arrays live in pools: a row pool (one row per link: joint angle, sPAM coverage and
// one step's records; a robot of n links holds n consecutive rows) and an obstacle
// pool, each with a first-fit free list, so the device memory a robot takes follows its
// size and admission is by a byte budget.  Each call admits the queued robots that fit
// as one group and launches the group to full length at once, one launch per
// chain-length class, each on a stream of the server's own pool, so a group runs
// alongside the groups before it and never waits for them; the host only polls events.

namespace vs {
hipError_t launch_slot_reset(const KData& D, const int* slots, int count, hipStream_t stream);
}

namespace {

// first-fit free list over [0, cap)
struct FreeList {
  std::map<int64_t, int64_t> free;  // offset -> length
  int64_t cap = 0, used = 0;
  void init(int64_t c) {
    cap = c;
    used = 0;
    free.clear();
    if (c > 0) free[0] = c;
  }
  int64_t take(int64_t len) {
    if (len <= 0) return 0;
    for (auto it = free.begin(); it != free.end(); ++it)
      if (it->second >= len) {
        const int64_t off = it->first, rest = it->second - len;
        free.erase(it);
        if (rest > 0) free[off + len] = rest;
        used += len;
        return off;
      }
    return -1;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (const auto& f : free) m = std::max(m, f.second);
    return m;
  }
  void give(int64_t off, int64_t len) {
    if (len <= 0) return;
    used -= len;
    auto it = free.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

template <typename T>
hipError_t halloc(T** p, size_t count) {  // pinned host staging
  return hipHostMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1), hipHostMallocDefault);
}

constexpr int64_t kRowBytes = 8 + 24 + 8 + 4 + 4 + 4 + 8 + 8 + 8 + 16;  // theta, records, coverage
constexpr int64_t kObsBytes = 4 + 32;
constexpr int64_t kSlotBytes = 4 * vs::kII + 48 + 8 + 8 + 40 + 4;  // ii, dd, counts, tip length, counters, order

}  // namespace

struct vine_server {
  vine_sim* h = nullptr;  // the slab
  int slots = 0, max_links = 0, max_obs = 0, max_spams = 0;
  int64_t hbm_bytes = 0;
  static constexpr int kMaxTables = 8;
  // Lanes: streams that each carry at most one group at a time, one per hardware queue of
  // the process (HIP gives four by default, GPU_MAX_HW_QUEUES sets it).  Streams share the
  // queues in turn, so a stream beyond them would wait behind another stream's group.
  static constexpr int kMaxLanes = 32;
  int lanes = 4;
  struct Robot {
    int64_t req = 0;
    int index = 0;  // within the request
    vine_instance inst{};
    std::vector<vine_spam> spams;
    std::vector<vine_obstacle> obs;
    int64_t row = -1, obs_off = -1;
    int start = 0;               // links it starts with (vine_server_submit_from)
    std::vector<double> theta0;  // their joint angles
  };
  struct Request {
    int n_robots = 0, n_done = 0, worst = 0;
    std::vector<double> tips;                 // 3 per robot
    std::vector<std::vector<double>> theta;   // per robot
  };
  struct Group {
    int64_t order_off = -1;            // its robots' slots at order[order_off, + count)
    int count = 0;
    std::vector<hipEvent_t> ev_run;    // one per class launch
    hipEvent_t ev_out = nullptr;       // results copied out
    int stream = 0;                    // its lane: copies in, launch, copies out
    int state = 0;                     // 1 running, 2 being read back
    int waves = 2;                     // per robot
  };
  std::deque<Robot> queue;
  std::vector<Robot> live;  // by slot
  std::vector<int> busy;    // by slot
  FreeList rows, obst, order_ranges;
  std::list<Group> groups;
  std::unordered_map<int64_t, Request> reqs;
  std::deque<int64_t> completed;
  int64_t joint_updates = 0, n_completed = 0, resident = 0, reading = 0;
  // waves of the resident robots, and the waves the device holds at two per SIMD (what
  // the two- and four-wave kernels of the classes up to 256 links fit in registers)
  int64_t resident_waves = 0, wave_slots = 0;
  hipStream_t pool[kMaxLanes] = {};
  bool lane_busy[kMaxLanes] = {};
  // pinned staging at the pools' offsets: inputs, launch orders, results
  int* st_ii = nullptr;
  double* st_dd = nullptr;
  double* st_cover = nullptr;
  int* st_okind = nullptr;
  double* st_obs = nullptr;
  int* st_order = nullptr;
  int* st_start = nullptr;  // links each robot of a group starts with, at the order offsets
  double* st_theta = nullptr;
  double* st_tip = nullptr;
  int* st_status = nullptr;
  vs::SlotStage stage{};  // the staging at its device-visible addresses (the group kernels')
  std::string err;
};

namespace {

int sfail(vine_server* s, int code, const std::string& msg) {
  if (s) s->err = msg; else g_create_error = msg;
  return code;
}

int table_for(vine_server* sv, double l) {
  vine_sim* h = sv->h;
  for (size_t t = 0; t < h->link_lens.size(); ++t)
    if (h->link_lens[t] == l) return (int)t;
  if ((int)h->link_lens.size() >= vine_server::kMaxTables) return -1;
  SpamTable T;
  build_spam_table(&T, l, h->prm.R_c, h->prm.R_act, h->prm.a_corr);
  const int t = (int)h->link_lens.size();
  if (hipMemcpy(h->tables + t, &T, sizeof(SpamTable), hipMemcpyHostToDevice) != hipSuccess)
    return -2;
  h->link_lens.push_back(l);
  h->tables_h.push_back(T);
  return t;
}

void drop_group_events(vine_server::Group& g) {
  for (hipEvent_t e : g.ev_run)
    if (e) (void)hipEventDestroy(e);
  g.ev_run.clear();
  if (g.ev_out) (void)hipEventDestroy(g.ev_out);
  g.ev_out = nullptr;
}

void free_server(vine_server* s) {
  for (hipStream_t st : s->pool)
    if (st) (void)hipStreamSynchronize(st);
  for (auto& g : s->groups) drop_group_events(g);
  s->groups.clear();
  for (hipStream_t st : s->pool)
    if (st) (void)hipStreamDestroy(st);
  void* pinned[] = {s->st_ii, s->st_dd, s->st_cover, s->st_okind, s->st_obs, s->st_order,
                    s->st_start, s->st_theta, s->st_tip, s->st_status};
  for (void* p : pinned)
    if (p) (void)hipHostFree(p);
  if (s->h) vine_sim_destroy(s->h);
}

// hipSuccess when every event has completed, hipErrorNotReady while one has not
hipError_t events_done(const std::vector<hipEvent_t>& evs) {
  for (hipEvent_t e : evs) {
    const hipError_t q = hipEventQuery(e);
    if (q != hipSuccess) return q;
  }
  return hipSuccess;
}

// Launch the admitted robots `adm` (slots, all of one chain-length class) as a group on
// lane `lane`: inputs staged in pinned memory and copied asynchronously, the slots'
// state cleared, one rollout launch to full length, all on the lane's stream.
int launch_group(vine_server* s, int lane, std::vector<int>& adm) {
  vine_sim* h = s->h;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  vine_server::Group g;
  g.count = (int)adm.size();
  g.order_off = s->order_ranges.take(g.count);  // fits: count <= the longest free run
  g.stream = lane;
  hipStream_t sa = s->pool[lane];
  // launch order: longest expected work first
  auto cost = [&](int b) {
    const vine_server::Robot& r = s->live[b];
    const double n = r.inst.n_links, s0 = r.start;
    return (n * n - s0 * s0) * (4.0 + r.inst.obs_count);
  };
  std::stable_sort(adm.begin(), adm.end(), [&](int a, int b) { return cost(a) > cost(b); });
  int nmax = 0;
  for (int slot : adm) {
    const vine_server::Robot& r = s->live[slot];
    const int n = r.inst.n_links, K = (int)r.obs.size();
    nmax = std::max(nmax, n);
    const int64_t row = r.row, oo = r.obs_off;
    const vine_instance& I = r.inst;
    int* ii = s->st_ii + vs::kII * (size_t)slot;
    ii[vs::kNTarget] = n;
    ii[vs::kObsOff] = (int)oo;
    ii[vs::kObsCnt] = K;
    ii[vs::kTableId] = table_for(s, I.link_len);  // a lookup: built at submit
    ii[vs::kCoverOff] = (int)row;
    ii[vs::kSpamOff] = 0;
    ii[vs::kSpamCnt] = 0;
    ii[vs::kThetaOff] = (int)row;
    ii[vs::kRecOff] = (int)row;
    ii[vs::kRecCap] = n;
    double* dd = s->st_dd + 6 * (size_t)slot;
    dd[0] = I.link_len;
    dd[1] = I.tube_radius;
    dd[2] = I.body_pressure;
    dd[3] = I.base_x;
    dd[4] = I.base_y;
    dd[5] = I.base_heading;
    std::vector<double> cover;
    append_cover(I, r.spams.data(), cover);
    std::copy(cover.begin(), cover.end(), s->st_cover + 2 * row);
    if (r.start > 0) std::copy(r.theta0.begin(), r.theta0.end(), s->st_theta + row);
    for (int k = 0; k < K; ++k) {
      const vine_obstacle& O = r.obs[k];
      s->st_okind[oo + k] = O.kind;
      double* o = s->st_obs + 4 * (oo + k);
      o[0] = O.cx;
      o[1] = O.cy;
      o[2] = O.a;
      o[3] = O.kind == 1 ? O.b : 0.0;
    }
  }
  // the group's inputs go from the staging to the slab in one launch, on the lane's stream
  // (a staging region is rewritten only after its robot has been read back, long after)
  std::copy(adm.begin(), adm.end(), s->st_order + g.order_off);
  bool resumed = false;
  for (int i = 0; i < g.count; ++i) {
    s->st_start[g.order_off + i] = s->live[adm[i]].start;
    resumed = resumed || s->live[adm[i]].start > 0;
  }
  const vs::SlotInputs in{h->ii, h->dd, h->cover, h->okind, h->obs, h->order};
  A(vs::launch_slot_load(in, s->stage, (int)g.order_off, g.count, sa));
  vs::KData D = kdata(h);
  A(vs::launch_slot_reset(D, h->order + g.order_off, g.count, sa));
  if (resumed) A(vs::launch_slot_start(D, s->stage, (int)g.order_off, g.count, sa));
  D.launch_first = (int)g.order_off;
  D.launch_count = g.count;
  // four waves per robot (the same results, each robot's steps faster) while every
  // resident robot keeps a wave slot; two once the device fills up
  g.waves = link_class(nmax) < 3 && s->resident_waves + 4LL * g.count <= s->wave_slots ? 4 : 2;
  A(vs::launch_rollout(kparams(h->prm), D, nmax, kClassLinks[link_class(nmax)], g.waves, sa));
  hipEvent_t ev = nullptr;
  A(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  A(hipEventRecord(ev, sa));
  g.ev_run.push_back(ev);
  g.state = 1;
  s->resident += g.count;
  s->resident_waves += (int64_t)g.waves * g.count;
  s->lane_busy[lane] = true;
  s->groups.push_back(std::move(g));
  if (e != hipSuccess) return sfail(s, VINE_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return VINE_OK;
}

}  // namespace

extern "C" {

int32_t vine_server_create(const vine_params* params, int32_t slots, int64_t hbm_bytes,
                           int32_t max_links, int32_t max_obstacles, int32_t max_spams,
                           vine_server** out) {
  if (!params || !out || slots < 1 || max_links < 1 || max_obstacles < 0 || max_spams < 0)
    return sfail(nullptr, VINE_EINVAL, "null pointer or non-positive size");
  if (max_links > VINE_MAX_LINKS || max_obstacles > VINE_MAX_OBSTACLES ||
      max_spams > VINE_MAX_SPAMS)
    return sfail(nullptr, VINE_ECAPACITY, "bounds above the library's limits");
  // the budget buys whole robots at the bounds: max_links rows + max_obstacles obstacles
  const int64_t per_robot = kRowBytes * max_links + kObsBytes * max_obstacles;
  const int64_t units = (hbm_bytes - kSlotBytes * (int64_t)slots) / per_robot;
  if (units < 1)
    return sfail(nullptr, VINE_EINVAL, "the byte budget does not hold one robot at the bounds");
  // a slab of `slots` robots at zero size, pools sized from the budget
  vine_instance ph{};
  ph.n_links = max_links;
  ph.link_len = 0.02;
  ph.tube_radius = 0.025;
  ph.body_pressure = 1000.0;
  vine_sim* h = nullptr;
  int rc = vine_sim_create(params, &ph, 1, nullptr, 0, nullptr, 0, &h);
  if (rc != VINE_OK) return rc;
  vine_server* s = new (std::nothrow) vine_server();
  if (!s) {
    vine_sim_destroy(h);
    return sfail(nullptr, VINE_ENOMEM, "host allocation failed");
  }
  s->h = h;
  s->slots = slots;
  s->max_links = max_links;
  s->max_obs = max_obstacles;
  s->max_spams = max_spams;
  const int64_t R = units * max_links, Ko = std::max<int64_t>(1, units * max_obstacles);
  s->rows.init(R);
  s->obst.init(units * max_obstacles);
  s->order_ranges.init(slots);
  s->live.resize(slots);
  s->busy.assign(slots, 0);
  // replace the slab's per-robot arrays by pools of the budget's size
  void* old[] = {h->ii, h->dd, h->cover, h->spam, h->okind, h->obs, h->theta, h->ncur, h->tcur,
                 h->tip, h->rho, h->iters, h->status, h->ncont, h->chash, h->maxpen, h->tiplen,
                 h->ulast, h->jevals, h->nsolves, h->negsteps, h->cycles, h->wtime, h->order};
  for (void* p : old) (void)hipFree(p);
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  const size_t B = slots;
  A(dalloc(&h->ii, B * vs::kII));
  A(dalloc(&h->dd, B * 6));
  A(dalloc(&h->cover, (size_t)R * 2));
  A(dalloc(&h->spam, 1));
  A(dalloc(&h->okind, (size_t)Ko));
  A(dalloc(&h->obs, (size_t)Ko * 4));
  A(dalloc(&h->theta, (size_t)R));
  A(dalloc(&h->ncur, B));
  A(dalloc(&h->tcur, B));
  A(dalloc(&h->tip, (size_t)R * 3));
  A(dalloc(&h->rho, (size_t)R));
  A(dalloc(&h->iters, (size_t)R));
  A(dalloc(&h->status, (size_t)R));
  A(dalloc(&h->ncont, (size_t)R));
  A(dalloc(&h->chash, (size_t)R));
  A(dalloc(&h->maxpen, (size_t)R));
  A(dalloc(&h->tiplen, (size_t)R));
  A(dalloc(&h->ulast, B));
  A(dalloc(&h->jevals, B));
  A(dalloc(&h->nsolves, B));
  A(dalloc(&h->negsteps, B));
  A(dalloc(&h->cycles, B));
  A(dalloc(&h->wtime, B));
  A(dalloc(&h->order, B));
  SpamTable* t8 = nullptr;
  A(dalloc(&t8, vine_server::kMaxTables));
  if (e == hipSuccess)
    e = hipMemcpy(t8, h->tables_h.data(), sizeof(SpamTable) * h->tables_h.size(),
                  hipMemcpyHostToDevice);
  (void)hipFree(h->tables);
  h->tables = t8;
  {
    // one lane per hardware queue of the process (HIP's GPU_MAX_HW_QUEUES, default 4): a
    // stream beyond them would share a queue, and its launches wait behind another lane's
    const char* q = std::getenv("GPU_MAX_HW_QUEUES");
    const int hwq = q ? std::atoi(q) : 0;
    s->lanes = hwq >= 1 ? std::min(hwq, (int)vine_server::kMaxLanes) : 4;
  }
  for (int k = 0; k < s->lanes; ++k)
    A(hipStreamCreateWithFlags(&s->pool[k], hipStreamNonBlocking));
  A(halloc(&s->st_ii, B * vs::kII));
  A(halloc(&s->st_dd, B * 6));
  A(halloc(&s->st_cover, (size_t)R * 2));
  A(halloc(&s->st_okind, (size_t)Ko));
  A(halloc(&s->st_obs, (size_t)Ko * 4));
  A(halloc(&s->st_order, B));
  A(halloc(&s->st_start, B));
  A(halloc(&s->st_theta, (size_t)R));
  A(halloc(&s->st_tip, (size_t)R * 3));
  A(halloc(&s->st_status, (size_t)R));
  if (e == hipSuccess) {
    // the staging's device-visible addresses, for the group load and store kernels
    auto dev = [&](void* host) {
      void* d = nullptr;
      A(hipHostGetDevicePointer(&d, host, 0));
      return d;
    };
    vs::SlotStage& g = s->stage;
    g.ii = (const int*)dev(s->st_ii);
    g.dd = (const double*)dev(s->st_dd);
    g.cover = (const double*)dev(s->st_cover);
    g.okind = (const int*)dev(s->st_okind);
    g.obs = (const double*)dev(s->st_obs);
    g.order = (const int*)dev(s->st_order);
    g.start = (const int*)dev(s->st_start);
    g.theta = (double*)dev(s->st_theta);
    g.tip = (double*)dev(s->st_tip);
    g.status = (int*)dev(s->st_status);
  }
  h->B = slots;
  h->N = max_links;
  h->T = max_links;
  h->S = 0;
  h->theta_len = R;
  h->rec_len = R;
  h->skip_done = 1;
  h->inst_h.clear();
  h->order_h.assign(B, 0);
  for (int c = 0; c < vine_sim::kClasses; ++c) h->cls_first[c] = h->cls_count[c] = 0;
  if (e == hipSuccess) {
    // every slot empty: zero rows (target 0 links), zero state
    std::vector<int> ii(B * vs::kII, 0);
    e = hipMemcpy(h->ii, ii.data(), sizeof(int) * ii.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = vs::launch_reset(kdata(h), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    vine_server_destroy(s);
    return sfail(nullptr, e == hipErrorOutOfMemory ? VINE_ENOMEM : VINE_EDEVICE,
                 std::string("server allocation: ") + hipGetErrorString(e));
  }
  s->hbm_bytes = kRowBytes * R + kObsBytes * Ko + kSlotBytes * (int64_t)slots;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      s->wave_slots = 8LL * cus;  // four SIMDs per compute unit, two waves each
  }
  *out = s;
  return VINE_OK;
}

int32_t vine_server_submit(vine_server* s, int64_t request_id, const vine_instance* inst,
                           int32_t n_inst, const vine_spam* spams, int32_t n_spams,
                           const vine_obstacle* obstacles, int32_t n_obstacles) {
  return vine_server_submit_from(s, request_id, inst, n_inst, spams, n_spams, obstacles,
                                 n_obstacles, nullptr, nullptr);
}

int32_t vine_server_submit_from(vine_server* s, int64_t request_id, const vine_instance* inst,
                                int32_t n_inst, const vine_spam* spams, int32_t n_spams,
                                const vine_obstacle* obstacles, int32_t n_obstacles,
                                const int32_t* start_links, const double* start_theta) {
  if (!s || !inst || n_inst < 1 || n_spams < 0 || n_obstacles < 0 || (n_spams > 0 && !spams) ||
      (n_obstacles > 0 && !obstacles))
    return sfail(s, VINE_EINVAL, "null pointer or negative count");
  if (s->reqs.count(request_id)) return sfail(s, VINE_EINVAL, "request id already in use");
  for (int b = 0; b < n_inst; ++b) {
    const vine_instance& I = inst[b];
    if (I.n_links < 1 || !finite_pos(I.link_len) || !finite_pos(I.tube_radius) ||
        !finite_pos(I.body_pressure) || !std::isfinite(I.base_x) || !std::isfinite(I.base_y) ||
        !std::isfinite(I.base_heading) || I.spam_count < 0 || I.spam_offset < 0 ||
        (int64_t)I.spam_offset + I.spam_count > n_spams || I.obs_count < 0 ||
        I.obs_offset < 0 || (int64_t)I.obs_offset + I.obs_count > n_obstacles)
      return sfail(s, VINE_EINVAL, "invalid instance");
    if (I.n_links > s->max_links || I.obs_count > s->max_obs || I.spam_count > s->max_spams)
      return sfail(s, VINE_ECAPACITY, "robot above the server's bounds");
    for (int k = 0; k < I.spam_count; ++k)
      if (!spam_ok(spams[I.spam_offset + k])) return sfail(s, VINE_EINVAL, "invalid sPAM");
    for (int k = 0; k < I.obs_count; ++k) {
      const vine_obstacle& O = obstacles[I.obs_offset + k];
      if (!(O.kind == 0 || O.kind == 1) || !std::isfinite(O.cx) || !std::isfinite(O.cy) ||
          !finite_pos(O.a) || (O.kind == 1 && !finite_pos(O.b)))
        return sfail(s, VINE_EINVAL, "invalid obstacle");
    }
  }
  // starting states: 0 <= s < n_links, finite angles, hard growth only
  int64_t n_theta = 0;
  if (start_links) {
    for (int b = 0; b < n_inst; ++b) {
      if (start_links[b] < 0 || start_links[b] >= inst[b].n_links)
        return sfail(s, VINE_EINVAL, "starting link count outside [0, n_links)");
      n_theta += start_links[b];
    }
    if (n_theta > 0 && !start_theta) return sfail(s, VINE_EINVAL, "null starting joint angles");
    for (int64_t k = 0; k < n_theta; ++k)
      if (!std::isfinite(start_theta[k])) return sfail(s, VINE_EINVAL, "non-finite joint angle");
    if (n_theta > 0 && s->h->prm.growth_stiffness != 0.0)
      return sfail(s, VINE_ESTATE, "a starting state needs hard growth (growth_stiffness 0)");
  }
  // the sPAM table of each link length (built and uploaded on its first use)
  for (int b = 0; b < n_inst; ++b) {
    const int tid = table_for(s, inst[b].link_len);
    if (tid < 0)
      return sfail(s, tid == -1 ? VINE_ECAPACITY : VINE_EDEVICE,
                   tid == -1 ? "more than 8 distinct link lengths" : "table upload failed");
  }
  vine_server::Request R;
  R.n_robots = n_inst;
  R.tips.assign(3 * (size_t)n_inst, 0.0);
  R.theta.resize(n_inst);
  s->reqs.emplace(request_id, std::move(R));
  int64_t at = 0;  // this robot's first starting angle
  for (int b = 0; b < n_inst; ++b) {
    vine_server::Robot r;
    r.req = request_id;
    r.index = b;
    if (start_links && start_links[b] > 0) {
      r.start = start_links[b];
      r.theta0.assign(start_theta + at, start_theta + at + r.start);
      at += r.start;
    }
    r.inst = inst[b];
    r.spams.assign(spams + inst[b].spam_offset, spams + inst[b].spam_offset + inst[b].spam_count);
    r.obs.assign(obstacles + inst[b].obs_offset,
                 obstacles + inst[b].obs_offset + inst[b].obs_count);
    r.inst.spam_offset = 0;
    r.inst.obs_offset = 0;
    s->queue.push_back(std::move(r));
  }
  return VINE_OK;
}

int32_t vine_server_tick(vine_server* s) {
  if (!s) return sfail(s, VINE_EINVAL, "null server");
  vine_sim* h = s->h;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
  };
  int done_now = 0;
  // 1. groups that finished: copy their results out; groups read back: hand them over
  for (auto it = s->groups.begin(); it != s->groups.end() && e == hipSuccess;) {
    vine_server::Group& g = *it;
    if (g.state == 1) {
      const hipError_t q = events_done(g.ev_run);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      A(q);
      hipStream_t st = s->pool[g.stream];
      A(vs::launch_slot_store(kdata(h), s->stage, (int)g.order_off, g.count, st));
      A(hipEventCreateWithFlags(&g.ev_out, hipEventDisableTiming));
      A(hipEventRecord(g.ev_out, st));
      g.state = 2;
      s->reading += g.count;
      ++it;
      continue;
    }
    const hipError_t q = hipEventQuery(g.ev_out);
    if (q == hipErrorNotReady) {
      ++it;
      continue;
    }
    A(q);
    for (int i = 0; i < g.count && e == hipSuccess; ++i) {
      const int slot = s->st_order[g.order_off + i];
      vine_server::Robot& r = s->live[slot];
      vine_server::Request& R = s->reqs[r.req];
      const int n = r.inst.n_links;
      const int64_t row = r.row;
      R.theta[r.index].assign(s->st_theta + row, s->st_theta + row + n);
      std::copy(s->st_tip + 3 * (row + n - 1), s->st_tip + 3 * (row + n),
                R.tips.begin() + 3 * (size_t)r.index);
      for (int t = 0; t < n; ++t) R.worst = std::max(R.worst, s->st_status[row + t]);
      s->joint_updates += (int64_t)n * (n + 1) / 2 - (int64_t)r.start * (r.start + 1) / 2;
      if (++R.n_done == R.n_robots) {
        s->completed.push_back(r.req);
        ++s->n_completed;
        ++done_now;
      }
      s->rows.give(r.row, n);
      s->obst.give(r.obs_off, (int64_t)r.obs.size());
      s->busy[slot] = 0;
      r = vine_server::Robot();
    }
    s->order_ranges.give(g.order_off, g.count);
    s->resident -= g.count;
    s->resident_waves -= (int64_t)g.waves * g.count;
    s->reading -= g.count;
    s->lane_busy[g.stream] = false;
    drop_group_events(g);
    it = s->groups.erase(it);
  }
  if (e != hipSuccess) return sfail(s, VINE_EDEVICE, std::string("read-back: ") + hipGetErrorString(e));
  // 2. admission, one group per idle lane: the queue's oldest robot fixes the group's
  // chain-length class, and the queued robots of that class join it in arrival order
  // while free slots, rows, obstacle space and a contiguous run of the order array (a
  // group's launch order is contiguous there) hold them.  Robots of other classes keep
  // their places.  A lightly loaded server runs each request as soon as it arrives; under
  // load the queue builds up while the lanes are busy and the groups grow.
  for (int lane = 0; lane < s->lanes && e == hipSuccess; ++lane) {
    if (s->lane_busy[lane] || s->queue.empty()) continue;
    const int cls = link_class(s->queue.front().inst.n_links);
    const int64_t room = s->order_ranges.largest();
    std::vector<int> adm;
    int slot = 0;
    for (auto it = s->queue.begin(); it != s->queue.end() && (int64_t)adm.size() < room;) {
      if (link_class(it->inst.n_links) != cls) {
        ++it;
        continue;
      }
      while (slot < s->slots && s->busy[slot]) ++slot;
      if (slot == s->slots) break;
      const int n = it->inst.n_links, K = (int)it->obs.size();
      const int64_t row = s->rows.take(n);
      if (row < 0) break;
      const int64_t oo = s->obst.take(K);
      if (oo < 0) {
        s->rows.give(row, n);
        break;
      }
      vine_server::Robot r = std::move(*it);
      it = s->queue.erase(it);
      r.row = row;
      r.obs_off = oo;
      s->live[slot] = std::move(r);
      s->busy[slot] = 1;
      adm.push_back(slot);
    }
    if (adm.empty()) break;  // the oldest robot does not fit yet: keep the arrival order
    if (launch_group(s, lane, adm) != VINE_OK) return VINE_EDEVICE;
  }
  return done_now;
}

int32_t vine_server_poll(vine_server* s, int64_t* ids, int32_t* worst_status, int32_t cap) {
  if (!s || (cap > 0 && !ids)) return sfail(s, VINE_EINVAL, "null server or buffer");
  int k = 0;
  while (k < cap && !s->completed.empty()) {
    const int64_t id = s->completed.front();
    s->completed.pop_front();
    ids[k] = id;
    if (worst_status) worst_status[k] = s->reqs[id].worst;
    ++k;
  }
  return k;
}

int32_t vine_server_result(const vine_server* sc, int64_t request_id, int32_t robot, double* tip,
                           double* theta) {
  vine_server* s = const_cast<vine_server*>(sc);
  if (!s || !tip) return sfail(s, VINE_EINVAL, "null server or buffer");
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end() || it->second.n_done < it->second.n_robots || robot < 0 ||
      robot >= it->second.n_robots)
    return sfail(s, VINE_EINVAL, "unknown or unfinished request, or robot out of range");
  std::copy(it->second.tips.begin() + 3 * (size_t)robot,
            it->second.tips.begin() + 3 * (size_t)robot + 3, tip);
  if (theta) std::copy(it->second.theta[robot].begin(), it->second.theta[robot].end(), theta);
  return VINE_OK;
}

int32_t vine_server_release(vine_server* s, int64_t request_id) {
  if (!s) return sfail(s, VINE_EINVAL, "null server");
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end() || it->second.n_done < it->second.n_robots)
    return sfail(s, VINE_EINVAL, "unknown or unfinished request");
  s->reqs.erase(it);
  return VINE_OK;
}

void vine_server_stats(const vine_server* s, int64_t out[8]) {
  if (!s || !out) return;
  out[0] = (int64_t)s->queue.size();
  out[1] = s->resident;
  out[2] = s->n_completed;
  out[3] = s->joint_updates;
  out[4] = s->rows.used;
  out[5] = s->rows.cap;
  out[6] = s->hbm_bytes;
  out[7] = (int64_t)s->groups.size();
}

void vine_server_destroy(vine_server* s) {
  if (!s) return;
  free_server(s);
  delete s;
}

const char* vine_server_last_error(const vine_server* s) {
  return s ? s->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
