/*
 * vine_oracle.c -- plain FP64 CPU oracle for the quasi-static growth step of a
 * soft growing ("vine") robot (arXiv 2509.15180).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  It shares no code, header, table or
 * helper with the HIP path, and it is written for clarity, not speed: dense
 * analytic Hessians solved by Gaussian elimination, all link/obstacle pairs,
 * adaptive quadrature.
 *
 * What it computes, in the paper's order (section / equation):
 *   Sec. 3.1, Eq. 1a-d   sPAM force-strain law; G(eps) = F_t / P_act for an actuator
 *                        unit of length l0 equal to the link length.
 *   Sec. 3.2, Eq. 2a-b   wrinkling-based restoring moment M(theta).
 *   Sec. 3.3, Eq. 3a-b   strain eps = (2R + R_act) theta / l and the net joint moment.
 *   Sec. 4.1, Eq. 4      the next state minimises a cost of bending, growth and contact;
 *                        read as the potential energy
 *                          Pi(theta) = sum_j E_j(theta_j) + k_c/2 sum_{links,obstacles} pen^2,
 *                        E_j the integral of the joint moment, so dPi/dtheta = 0 is the
 *                        joint moment balance under penalty contact.
 *   Sec. 4.1, Alg. 1     one growth step: append a link and descend to that equilibrium.
 *                        The fixed 50 gradient steps are replaced by a converged damped
 *                        Newton descent (scaled residual <= tol).
 *   Sec. 5               the design search over sPAM placement and pressure; here the
 *                        derivative of a tip-to-goal loss with respect to those
 *                        parameters, by the adjoint of each step's equilibrium
 *                        (vo_gradient), pinned against finite differences of rollouts.
 * Readings of points the paper leaves open are listed in the design notes
 * (parameter choices, contact geometry, growth sub-steps, solver rules).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define VO_PI 3.14159265358979323846

#include <stdio.h>
int vo_verbose = 0; /* per-iteration trace of chain_solve on stderr (debugging aid) */

/* ------------------------------------------------------------------------- */
/* parameters                                                                */

typedef struct {
  double Rc, Ract, acorr;   /* sPAM constriction radius, actuator radius, correction a (Sec. 3.1) */
  double epsc;              /* critical wrinkling strain (Sec. 3.2) */
  double kc;                /* penalty stiffness, N/m (contact term of Eq. 4) */
  double tol;               /* convergence: max_j |r_j| / M_max <= tol */
  int max_iter;             /* Newton iterations per solve */
  int substeps;             /* growth sub-steps per appended link */
  double fd_h;              /* finite-difference step for the Hessian */
  double c1;                /* Armijo constant */
  double c_mu;              /* damping per unit residual: mu = c_mu max_j |r_j| (1/rad) */
  double step_max;          /* cap on max_j |step_j| (rad) */
  double mu_up;             /* factor by which mu is raised when a step does not descend */
  int cheb_n;               /* Chebyshev degree of the G fit */
  double pd_shift;          /* delta / M_max: a state is a minimum when H + delta I is
                               positive definite (1/rad) */
  double wg;                /* growth stiffness, N/m: 0 = hard growth (each step appends a
                               link of prescribed length); > 0 = soft growth (the tip link's
                               length is free under the growth term of Eq. 4) */
} vo_prm;

static void prm_from(const double* p, vo_prm* P) {
  P->Rc = p[0];
  P->Ract = p[1];
  P->acorr = p[2];
  P->epsc = p[3];
  P->kc = p[4];
  P->tol = p[5];
  P->max_iter = (int)p[6];
  P->substeps = (int)p[7];
  P->fd_h = p[8];
  P->c1 = p[9];
  P->c_mu = p[10];
  P->cheb_n = (int)p[11];
  P->step_max = p[12];
  P->mu_up = p[13];
  P->pd_shift = p[14];
  P->wg = p[15];
}

/* ------------------------------------------------------------------------- */
/* Carlson's symmetric elliptic integrals (B. C. Carlson, "Numerical computation
 * of real or complex elliptic integrals", Numer. Algorithms 10, 1995):
 * duplication until the arguments agree to 1e-3, then the truncated series. */

double vo_rf(double x, double y, double z) {
  for (int k = 0; k < 200; ++k) {
    double mu = (x + y + z) / 3.0;
    double X = 1.0 - x / mu, Y = 1.0 - y / mu, Z = 1.0 - z / mu;
    double e = fmax(fabs(X), fmax(fabs(Y), fabs(Z)));
    if (e < 1e-3) {
      double E2 = X * Y - Z * Z, E3 = X * Y * Z;
      return (1.0 - E2 / 10.0 + E3 / 14.0 + E2 * E2 / 24.0 - 3.0 * E2 * E3 / 44.0) / sqrt(mu);
    }
    double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
    double lam = sx * sy + sy * sz + sz * sx;
    x = 0.25 * (x + lam);
    y = 0.25 * (y + lam);
    z = 0.25 * (z + lam);
  }
  return NAN;
}

double vo_rd(double x, double y, double z) {
  double sum = 0.0, fac = 1.0;
  for (int k = 0; k < 200; ++k) {
    double mu = (x + y + 3.0 * z) / 5.0;
    double X = 1.0 - x / mu, Y = 1.0 - y / mu, Z = 1.0 - z / mu;
    double e = fmax(fabs(X), fmax(fabs(Y), fabs(Z)));
    if (e < 1e-3) {
      double ea = X * Y, eb = Z * Z;
      double E2 = ea - 6.0 * eb;
      double E3 = (3.0 * ea - 8.0 * eb) * Z;
      double E4 = 3.0 * (ea - eb) * eb;
      double E5 = ea * Z * eb;
      double s = 1.0 - 3.0 * E2 / 14.0 + E3 / 6.0 + 9.0 * E2 * E2 / 88.0 - 3.0 * E4 / 22.0 -
                 9.0 * E2 * E3 / 52.0 + 3.0 * E5 / 26.0;
      return 3.0 * sum + fac * s / (mu * sqrt(mu));
    }
    double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
    double lam = sx * sy + sy * sz + sz * sx;
    sum += fac / (sz * (z + lam));
    fac *= 0.25;
    x = 0.25 * (x + lam);
    y = 0.25 * (y + lam);
    z = 0.25 * (z + lam);
  }
  return NAN;
}

/* Incomplete elliptic integrals in the parameter convention (m = k^2),
 * 0 <= phi <= pi/2: F(phi|m) = sin(phi) R_F(c^2, 1 - m s^2, 1),
 * E(phi|m) = F - (m/3) s^3 R_D(c^2, 1 - m s^2, 1). */
double vo_ellf(double phi, double m) {
  double s = sin(phi), c = cos(phi);
  return s * vo_rf(c * c, 1.0 - m * s * s, 1.0);
}

double vo_elle(double phi, double m) {
  double s = sin(phi), c = cos(phi);
  double d = 1.0 - m * s * s;
  return s * vo_rf(c * c, d, 1.0) - (m / 3.0) * s * s * s * vo_rd(c * c, d, 1.0);
}

/* ------------------------------------------------------------------------- */
/* sPAM model, Sec. 3.1 (Eq. 1a-d).  For a contraction parameter m in (0, 1/2]:
 *  unsaturated: l_a = l0 and phi in (0, phi_Rc] is the smallest root of Eq. 1b,
 *      F(phi|m)/(sqrt(m) cos phi) = (l_a/R_c)(1 + a/(2 m cos^2 phi));
 *  saturated (no such root): phi = phi_Rc (Eq. 1c) and Eq. 1b gives l_a;
 *  then Eq. 1a gives the strain, eps = (l_a - 2 R_c (E - F/2)/(sqrt(m) cos phi)) / l0,
 *  and Eq. 1d the force per unit pressure, G = pi R_c^2 (1 - 2m) / (2 m cos^2 phi). */

static double eq1b_resid(double phi, double m, double l0, const vo_prm* P) {
  /* Eq. 1b multiplied by cos^2(phi) so that both sides stay finite. */
  double c = cos(phi);
  return vo_ellf(phi, m) * c / sqrt(m) - (l0 / P->Rc) * (c * c + P->acorr / (2.0 * m));
}

int vo_spam_state(double m, double l0, const double* prm, double* eps, double* G, double* phi_out) {
  vo_prm P;
  prm_from(prm, &P);
  double phiRc = acos(P.Rc / P.Ract);
  const int NS = 512;
  double phi = -1.0, la = l0;
  int sat = 0;
  double a = 0.0, ga = eq1b_resid(1e-12, m, l0, &P);
  for (int k = 1; k <= NS; ++k) {
    double b = phiRc * (double)k / NS;
    double gb = eq1b_resid(b, m, l0, &P);
    if (ga < 0.0 && gb >= 0.0) {
      for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
        double c = 0.5 * (a + b);
        if (eq1b_resid(c, m, l0, &P) < 0.0) a = c; else b = c;
      }
      phi = 0.5 * (a + b);
      break;
    }
    a = b;
    ga = gb;
  }
  if (phi < 0.0) {
    sat = 1;
    phi = phiRc;
    double c = cos(phi);
    la = P.Rc * vo_ellf(phi, m) / (sqrt(m) * c * (1.0 + P.acorr / (2.0 * m * c * c)));
  }
  double c = cos(phi);
  double F = vo_ellf(phi, m), E = vo_elle(phi, m);
  *eps = (la - 2.0 * P.Rc * (E - 0.5 * F) / (sqrt(m) * c)) / l0;
  *G = VO_PI * P.Rc * P.Rc * (1.0 - 2.0 * m) / (2.0 * m * c * c);
  if (phi_out) *phi_out = phi;
  return sat;
}

static double spam_eps(double m, double l0, const double* prm) {
  double e, G;
  vo_spam_state(m, l0, prm, &e, &G, NULL);
  return e;
}

/* m0: contraction parameter of zero strain; eps(m) increases on [m0, 1/2]. */
static double spam_m0(double l0, const double* prm) {
  double a = 1e-6, b = 0.5;
  for (int it = 0; it < 200 && b - a > 1e-17; ++it) {
    double c = 0.5 * (a + b);
    if (spam_eps(c, l0, prm) < 0.0) a = c; else b = c;
  }
  return 0.5 * (a + b);
}

/* Exact G(eps) for 0 <= eps <= eps_max by bisection on m; 0 beyond eps_max (slack). */
static double spam_G_exact_mm(double eps, double l0, const double* prm, double m0, double emax) {
  if (eps >= emax) return 0.0;
  double a = m0, b = 0.5;
  if (eps > 0.0) {
    for (int it = 0; it < 200 && b - a > 1e-17; ++it) {
      double c = 0.5 * (a + b);
      if (spam_eps(c, l0, prm) < eps) a = c; else b = c;
    }
  } else {
    b = m0;
  }
  double e, G;
  vo_spam_state(eps > 0.0 ? 0.5 * (a + b) : m0, l0, prm, &e, &G, NULL);
  return G;
}

double vo_spam_G_exact(double eps, double l0, const double* prm) {
  return spam_G_exact_mm(eps, l0, prm, spam_m0(l0, prm), spam_eps(0.5, l0, prm));
}

/* ------------------------------------------------------------------------- */
/* Chebyshev representation of G on [0, eps_max] (bulk evaluation).  G(eps) has a
 * pole a little below eps = 0, so the degree is high (default 128). */

#define VO_CHEB_MAX 256
typedef struct {
  double l0, emax, G0;
  int N;
  double c[VO_CHEB_MAX + 2];  /* G  = sum' c_j T_j(x), x = 2 eps/emax - 1 (c_0 halved) */
  double d[VO_CHEB_MAX + 2];  /* dG/dx */
  double q[VO_CHEB_MAX + 3];  /* integral in x from -1 */
} vo_gfit;

static double cheb_eval(const double* c, int N, double x) {
  /* Clenshaw, c[0] already halved */
  double b1 = 0.0, b2 = 0.0;
  for (int j = N; j >= 1; --j) {
    double t = 2.0 * x * b1 - b2 + c[j];
    b2 = b1;
    b1 = t;
  }
  return x * b1 - b2 + c[0];
}

static void gfit_build(vo_gfit* g, double l0, const double* prm, int N) {
  if (N > VO_CHEB_MAX) N = VO_CHEB_MAX;
  g->l0 = l0;
  g->N = N;
  g->emax = spam_eps(0.5, l0, prm);
  double m0 = spam_m0(l0, prm);
  double f[VO_CHEB_MAX + 1];
  for (int k = 0; k <= N; ++k) {
    double x = cos(VO_PI * (k + 0.5) / (N + 1));
    f[k] = spam_G_exact_mm(0.5 * (x + 1.0) * g->emax, l0, prm, m0, g->emax);
  }
  for (int j = 0; j <= N; ++j) {
    double s = 0.0;
    for (int k = 0; k <= N; ++k) s += f[k] * cos(VO_PI * j * (k + 0.5) / (N + 1));
    g->c[j] = 2.0 * s / (N + 1);
  }
  g->c[0] *= 0.5;
  g->c[N + 1] = 0.0;
  /* derivative series: a'_{j-1} = a'_{j+1} + 2 j a_j (full a_0 convention) */
  double a[VO_CHEB_MAX + 3] = {0}, da[VO_CHEB_MAX + 3] = {0};
  for (int j = 0; j <= N + 2; ++j) a[j] = (j <= N) ? g->c[j] : 0.0;
  a[0] *= 2.0;
  da[N + 1] = da[N + 2] = 0.0;
  da[N] = 0.0;
  for (int j = N; j >= 1; --j) da[j - 1] = da[j + 1] + 2.0 * j * a[j];
  for (int j = 0; j <= N + 1; ++j) g->d[j] = da[j];
  g->d[0] *= 0.5;
  /* integral series: A_j = (a_{j-1} - a_{j+1}) / (2 j), constant fixed so that Q(-1) = 0 */
  for (int j = 1; j <= N + 1; ++j) g->q[j] = (a[j - 1] - a[j + 1]) / (2.0 * j);
  g->q[0] = 0.0;
  g->q[N + 2] = 0.0;
  double at_m1 = cheb_eval(g->q, N + 1, -1.0);
  g->q[0] = -at_m1;
  g->G0 = cheb_eval(g->c, N, -1.0);
}

/* process-wide cache of fits, keyed by l0 and the sPAM constants */
#define VO_GCACHE 64
static vo_gfit* gcache[VO_GCACHE];
static double gkey[VO_GCACHE][5];
static int gcount = 0;

static const vo_gfit* gfit_get(double l0, const double* prm) {
  const vo_gfit* out = NULL;
#ifdef _OPENMP
#pragma omp critical(vo_gfit_cache)
#endif
  {
    for (int k = 0; k < gcount && !out; ++k)
      if (gkey[k][0] == l0 && gkey[k][1] == prm[0] && gkey[k][2] == prm[1] &&
          gkey[k][3] == prm[2] && gkey[k][4] == prm[11])
        out = gcache[k];
    if (!out) {
      vo_gfit* g = (vo_gfit*)malloc(sizeof(vo_gfit));
      gfit_build(g, l0, prm, (int)prm[11]);
      if (gcount < VO_GCACHE) {
        gcache[gcount] = g;
        gkey[gcount][0] = l0;
        gkey[gcount][1] = prm[0];
        gkey[gcount][2] = prm[1];
        gkey[gcount][3] = prm[2];
        gkey[gcount][4] = prm[11];
        ++gcount;
      }
      out = g;
    }
  }
  return out;
}

/* G, dG/deps and int_0^eps G for 0 <= eps; slack (0, 0, const) beyond eps_max */
static void gfit_eval(const vo_gfit* g, double eps, double* G, double* dG, double* IG) {
  if (eps >= g->emax) {
    if (G) *G = 0.0;
    if (dG) *dG = 0.0;
    if (IG) *IG = 0.5 * g->emax * cheb_eval(g->q, g->N + 1, 1.0);
    return;
  }
  double x = 2.0 * eps / g->emax - 1.0;
  if (G) *G = cheb_eval(g->c, g->N, x);
  if (dG) *dG = cheb_eval(g->d, g->N - 1, x) * 2.0 / g->emax;
  if (IG) *IG = 0.5 * g->emax * cheb_eval(g->q, g->N + 1, x);
}

/* ------------------------------------------------------------------------- */
/* Wrinkling-based restoring moment, Sec. 3.2 (Eq. 2a-b), as a fraction of
 * M_max = pi P_vine R^3:  M = M_max f(gamma0),
 *   f(g) = (sin 2g + 2 pi - 2 g) / (4 (sin g + (pi - g) cos g)),
 *   gamma0 = acos(2 eps_c / sin(theta/2) - 1).
 * Below wrinkling onset (theta < theta_on = 2 asin(eps_c)) Eq. 2b is undefined;
 * the moment rises linearly from 0 to f(0) = 1/2 there.  |theta| is clamped at pi. */

static double wr_f(double g) {
  return (sin(2.0 * g) + 2.0 * VO_PI - 2.0 * g) / (4.0 * (sin(g) + (VO_PI - g) * cos(g)));
}

double vo_wr_h(double x, double epsc) {
  double th_on = 2.0 * asin(epsc);
  if (x <= th_on) return x / (2.0 * th_on);
  if (x > VO_PI) x = VO_PI;
  double arg = 2.0 * epsc / sin(0.5 * x) - 1.0;
  if (arg > 1.0) arg = 1.0;
  if (arg < -1.0) arg = -1.0;
  return wr_f(acos(arg));
}

/* Gauss-Legendre nodes by Newton iteration on P_n (textbook construction). */
#define VO_GL 20
static double gl_x[VO_GL], gl_w[VO_GL];
static int gl_ready = 0;

static void gl_init(void) {
  if (gl_ready) return;
  int n = VO_GL;
  for (int i = 0; i < n; ++i) {
    double z = cos(VO_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double dz = p1 / pp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    gl_x[i] = z;
    gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
  gl_ready = 1;
}

static double gl_rule(double (*f)(double, double), double par, double a, double b) {
  double h = 0.5 * (b - a), c = 0.5 * (a + b), s = 0.0;
  for (int i = 0; i < VO_GL; ++i) s += gl_w[i] * f(c + h * gl_x[i], par);
  return s * h;
}

static double adapt(double (*f)(double, double), double par, double a, double b, double whole,
                    double tol, int depth) {
  double m = 0.5 * (a + b);
  double l = gl_rule(f, par, a, m), r = gl_rule(f, par, m, b);
  /* stop at the tolerance or at the round-off level of the pieces */
  if (depth > 30 || fabs(l + r - whole) <= fmax(tol, 1e-13 * (fabs(l) + fabs(r)))) return l + r;
  return adapt(f, par, a, m, l, 0.5 * tol, depth + 1) + adapt(f, par, m, b, r, 0.5 * tol, depth + 1);
}

/* dh/dx for x >= 0 (one-sided from below at the onset, 0 beyond pi) */
double vo_wr_dh(double x, double epsc) {
  double th_on = 2.0 * asin(epsc);
  if (x <= th_on) return 1.0 / (2.0 * th_on);
  if (x >= VO_PI) return 0.0;
  double s = sin(0.5 * x);
  double u = 2.0 * epsc / s - 1.0;
  if (u > 1.0) u = 1.0;
  double g = acos(u);
  double du = -epsc * cos(0.5 * x) / (s * s);
  double one_m_u2 = 4.0 * epsc * (s - epsc) / (s * s); /* 1 - u^2 without cancellation */
  double dg = -du / sqrt(one_m_u2);
  double N = sin(2.0 * g) + 2.0 * VO_PI - 2.0 * g, dN = 2.0 * cos(2.0 * g) - 2.0;
  double D = 4.0 * (sin(g) + (VO_PI - g) * cos(g)), dD = -4.0 * (VO_PI - g) * sin(g);
  return (dN * D - N * dD) / (D * D) * dg;
}

static double wr_h_cb(double x, double epsc) { return vo_wr_h(x, epsc); }

/* int_0^x h(t) dt for x >= 0 (energy of the body moment per M_max) */
double vo_wr_int(double x, double epsc) {
  gl_init();
  double th_on = 2.0 * asin(epsc);
  if (x <= th_on) return x * x / (4.0 * th_on);
  double s = th_on / 4.0;
  double hi = x < VO_PI ? x : VO_PI;
  s += adapt(wr_h_cb, epsc, th_on, hi, gl_rule(wr_h_cb, epsc, th_on, hi), 1e-16, 0);
  if (x > VO_PI) s += vo_wr_h(VO_PI, epsc) * (x - VO_PI);
  return s;
}

/* ------------------------------------------------------------------------- */
/* Contact geometry.  The body of link i (Sec. 4.1: rigid segments in contact with
 * obstacles, Eq. 4's penetration term) is sampled by two disks of radius R, the
 * tube radius, centred on the link axis at its midpoint and at its distal end.
 * Each (disk, obstacle) pair contributes k_c/2 pen^2 with pen = max(0, -g) and
 *   g = dist(centre, obstacle) - R,
 * dist = |x - c| - rho for a circle and the signed distance to the rectangle
 * (negative inside).  n = d(dist)/dx is the outward unit normal at the centre. */

/* kappa: curvature of the distance field at x (its Hessian is kappa tau tau^T, tau the
 * unit tangent); 1/|x - c| for a circle, 1/(distance to the corner) in a rectangle's
 * corner region, 0 on its side regions and inside it. */
double vo_dist_circle(double x, double y, const double* o, double* nx, double* ny, double* kappa) {
  double vx = x - o[0], vy = y - o[1];
  double d = sqrt(vx * vx + vy * vy);
  if (d > 0.0) {
    *nx = vx / d;
    *ny = vy / d;
    *kappa = 1.0 / d;
  } else {
    *nx = 1.0;
    *ny = 0.0;
    *kappa = 0.0;
  }
  return d - o[2];
}

/* rectangle centre o[0..1], half-extents o[2..3] */
double vo_dist_box(double x, double y, const double* o, double* nx, double* ny, double* kappa) {
  double sx = x >= o[0] ? 1.0 : -1.0, sy = y >= o[1] ? 1.0 : -1.0;
  double dx = fabs(x - o[0]) - o[2], dy = fabs(y - o[1]) - o[3];
  *kappa = 0.0;
  if (dx > 0.0 || dy > 0.0) {
    double ox = dx > 0.0 ? dx : 0.0, oy = dy > 0.0 ? dy : 0.0;
    double d = sqrt(ox * ox + oy * oy);
    *nx = sx * ox / d;
    *ny = sy * oy / d;
    if (dx > 0.0 && dy > 0.0) *kappa = 1.0 / d;
    return d;
  }
  /* inside: distance to the nearest side, negative */
  if (dx >= dy) {
    *nx = sx;
    *ny = 0.0;
    return dx;
  }
  *nx = 0.0;
  *ny = sy;
  return dy;
}

/* ------------------------------------------------------------------------- */
/* one chain */

typedef struct {
  const vo_prm* P;
  const vo_gfit* G;
  int n;                 /* links present */
  double l, R, Pv, bx, by, bpsi;
  double last_len;       /* length of the tip link (hard growth: growth sub-steps) */
  int soft;              /* soft growth: the variables are (theta_0..theta_{n-1}, u), the
                            tip link's length u l, with the growth term (wg/2)(l (tgt - u))^2 */
  double tgt;            /* soft growth: the tip link's target length in link lengths */
  int frozen;            /* soft growth: u sits on its bound u = 0 with dPi/du > 0 and is
                            held there (the system is the joints' alone) */
  double arm, Mmax;
  const double *Pp, *Pm; /* pressure-weighted sPAM coverage per joint, +/- side */
  int K;
  const int* kind;
  const double* obs;
} vo_chain;

/* joint moment q_j(theta) (Eq. 3b with Eq. 2) and its energy E_j(theta) = int_0^theta q_j */
static void joint_law(const vo_chain* c, int j, double th, double* q, double* E) {
  const vo_prm* P = c->P;
  double ath = fabs(th);
  double Mb = (th >= 0.0 ? 1.0 : -1.0) * c->Mmax * vo_wr_h(ath, P->epsc);
  double ep = th > 0.0 ? c->arm * th / c->l : 0.0;
  double em = th < 0.0 ? -c->arm * th / c->l : 0.0;
  double Gp, Gm, IGp, IGm;
  gfit_eval(c->G, ep, &Gp, NULL, &IGp);
  gfit_eval(c->G, em, &Gm, NULL, &IGm);
  double pp = c->Pp[j], pm = c->Pm[j];
  if (q) *q = Mb - c->arm * (pp * Gp - pm * Gm);
  if (E) {
    double Eb = c->Mmax * vo_wr_int(ath, P->epsc);
    double G0 = c->G->G0;
    double Ea = (th >= 0.0) ? (-c->l * pp * IGp + c->arm * pm * G0 * th)
                            : (-c->arm * pp * G0 * th - c->l * pm * IGm);
    *E = Eb + Ea;
  }
}

typedef struct {
  int i, k;
  double lam, xx, xy, nx, ny, pen, kappa;
  double f; /* the disk's place on its link as a fraction of the link's length */
} vo_contact;

/* scratch for one chain: poses and unit link directions */
typedef struct {
  double *px, *py, *tx, *ty;
} vo_pose;

static void pose_alloc(vo_pose* w, int n) {
  w->px = (double*)malloc(sizeof(double) * (size_t)(4 * n + 8));
  w->py = w->px + n + 2;
  w->tx = w->py + n + 2;
  w->ty = w->tx + n + 2;
}

/* Poses (Sec. 4.1, minimal coordinates: heading of link i = base heading + sum_{j<=i}
 * theta_j), residual r = dPi/dtheta (nullable), energy Pi (when want_E), and the
 * contacts (nullable list, capacity cap; count in *ncl). */
static double chain_eval(const vo_chain* c, const double* th, double* r, int want_E,
                         vo_contact* cl, int cap, int* ncl, vo_pose* w) {
  const vo_prm* P = c->P;
  int n = c->n;
  double *px = w->px, *py = w->py, *tx = w->tx, *ty = w->ty;
  /* soft growth: th[n] = u, the tip link's length in link lengths (a link of negative
   * length has no energy: the line search never accepts one) */
  if (c->soft && !(th[n] >= 0.0)) return INFINITY;
  const double last = c->soft ? th[n] * c->l : c->last_len;
  double phi = c->bpsi;
  px[0] = c->bx;
  py[0] = c->by;
  double Pi = 0.0;
  for (int i = 0; i < n; ++i) {
    phi += th[i];
    tx[i] = cos(phi);
    ty[i] = sin(phi);
    double L = (i == n - 1) ? last : c->l;
    px[i + 1] = px[i] + L * tx[i];
    py[i + 1] = py[i] + L * ty[i];
  }
  for (int j = 0; j < n; ++j) {
    double q, E;
    joint_law(c, j, th[j], r ? &q : NULL, want_E ? &E : NULL);
    if (want_E) Pi += E;
    if (r) r[j] = q;
  }
  double ru = 0.0; /* soft growth: dPi/du */
  if (c->soft) {
    const double gap = c->l * (c->tgt - th[n]);
    if (want_E) Pi += 0.5 * P->wg * gap * gap;
    ru = -P->wg * c->l * gap;
  }
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    double L = (i == n - 1) ? last : c->l;
    for (int h = 1; h <= 2; ++h) {        /* disks at s = L/2 and s = L */
      double s = 0.5 * h * L;
      double xx = px[i] + s * tx[i], xy = py[i] + s * ty[i];
      for (int k = 0; k < c->K; ++k) {
        double nx, ny, kap;
        const double* o = c->obs + 4 * k;
        double g = (c->kind[k] == 0 ? vo_dist_circle(xx, xy, o, &nx, &ny, &kap)
                                     : vo_dist_box(xx, xy, o, &nx, &ny, &kap)) - c->R;
        if (g < 0.0) {
          double pen = -g, lam = P->kc * pen;
          Pi += 0.5 * P->kc * pen * pen;
          if (r) {
            /* dPi/dtheta_j for every joint j <= i: -lam times the moment arm (x - p_j) x n */
            for (int j = 0; j <= i; ++j) r[j] -= lam * ((xx - px[j]) * ny - (xy - py[j]) * nx);
            /* soft growth: the disk moves by f l t per unit of u */
            if (c->soft && i == n - 1) ru -= lam * 0.5 * h * c->l * (nx * tx[i] + ny * ty[i]);
          }
          if (cl && cnt < cap) {
            vo_contact* e = &cl[cnt];
            e->i = i;
            e->k = k;
            e->lam = lam;
            e->xx = xx;
            e->xy = xy;
            e->nx = nx;
            e->ny = ny;
            e->pen = pen;
            e->kappa = kap;
            e->f = 0.5 * h;
          }
          ++cnt;
        }
      }
    }
  }
  if (ncl) *ncl = cnt;
  if (r && c->soft) r[n] = ru;
  return Pi;
}

/* dq_j/dtheta (one-sided conventions: below onset at |theta| = theta_on; at theta = 0 the
 * mean of the two one-sided actuator slopes) */
static double joint_dq(const vo_chain* c, int j, double th) {
  const vo_prm* P = c->P;
  double d = c->Mmax * vo_wr_dh(fabs(th), P->epsc);
  double k = c->arm * c->arm / c->l;
  double pp = c->Pp[j], pm = c->Pm[j];
  if (th > 0.0) {
    double dG;
    gfit_eval(c->G, c->arm * th / c->l, NULL, &dG, NULL);
    d -= k * pp * dG;
  } else if (th < 0.0) {
    double dG;
    gfit_eval(c->G, -c->arm * th / c->l, NULL, &dG, NULL);
    d -= k * pm * dG;
  } else {
    double dG;
    gfit_eval(c->G, 0.0, NULL, &dG, NULL);
    d -= 0.5 * k * (pp + pm) * dG;
  }
  return d;
}

/* Exact Hessian of Pi (dense, row-major n x n) at the state whose poses are in w and
 * whose penetrating contacts are cl[0..ncl).  For a disk centre x on link i with
 * distance-field normal n, curvature kappa and force lam = k_c pen, with
 * v_j = z x (x - p_j) the velocity of x under joint j (j <= i):
 *   dg/dtheta_j = n.v_j = a_j,
 *   d2g/dtheta_j dtheta_m = kappa (tau.v_j)(tau.v_m) - n.(x - p_max(j,m)),
 * so the pair adds k_c a a^T - lam d2g. */
static void chain_hessian(const vo_chain* c, const double* th, const vo_contact* cl, int ncl,
                          const vo_pose* w, double* H, double* a, double* b, double* u) {
  int n = c->n;
  const int uvar = c->soft && !c->frozen;
  const int m = n + uvar; /* soft growth: row and column n belong to u */
  memset(H, 0, sizeof(double) * (size_t)m * m);
  for (int j = 0; j < n; ++j) H[j * m + j] = joint_dq(c, j, th[j]);
  if (uvar) H[n * m + n] = c->P->wg * c->l * c->l;
  for (int e = 0; e < ncl; ++e) {
    const vo_contact* q = &cl[e];
    int i = q->i;
    double tx = -q->ny, ty = q->nx; /* tangent */
    for (int j = 0; j <= i; ++j) {
      double vx = -(q->xy - w->py[j]), vy = q->xx - w->px[j];
      a[j] = q->nx * vx + q->ny * vy;
      b[j] = tx * vx + ty * vy;
      u[j] = q->nx * w->px[j] + q->ny * w->py[j];
    }
    double nxx = q->nx * q->xx + q->ny * q->xy;
    double kc = c->P->kc, lk = q->lam * q->kappa;
    for (int j = 0; j <= i; ++j)
      for (int k = 0; k <= i; ++k) {
        int mx = j > k ? j : k;
        H[j * m + k] += kc * a[j] * a[k] - lk * b[j] * b[k] + q->lam * (nxx - u[mx]);
      }
    if (uvar && i == n - 1) {
      /* soft growth: x moves by f l t per unit of u, t the tip link's direction, and t
       * turns with every joint (dt/dtheta_j = z x t); with n_t = n.t, tau_t = tau.t and
       * nz = n.(z x t):
       *   d2Pi/du2          = (f l)^2 (k_c n_t^2 - lam kappa tau_t^2),
       *   d2Pi/du dtheta_j  = f l (k_c a_j n_t - lam kappa b_j tau_t - lam nz) */
      const double ltx = w->tx[i], lty = w->ty[i], fl = q->f * c->l;
      const double nt = q->nx * ltx + q->ny * lty, taut = tx * ltx + ty * lty;
      const double nz = -q->nx * lty + q->ny * ltx;
      H[n * m + n] += fl * fl * (kc * nt * nt - lk * taut * taut);
      for (int j = 0; j <= i; ++j) {
        const double x = fl * (kc * a[j] * nt - lk * b[j] * taut - q->lam * nz);
        H[j * m + n] += x;
        H[n * m + j] += x;
      }
    }
  }
}

/* dense (H + mu I) x = b by Gaussian elimination with partial pivoting; 0 on success */
static int dense_solve(int n, const double* H, double mu, const double* b, double* x, double* W) {
  int w = n + 1;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) W[i * w + j] = H[i * n + j] + (i == j ? mu : 0.0);
    W[i * w + n] = b[i];
  }
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(W[k * w + k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(W[i * w + k]) > best) {
        best = fabs(W[i * w + k]);
        p = i;
      }
    if (!(best > 0.0)) return -1;
    if (p != k)
      for (int j = k; j <= n; ++j) {
        double t = W[k * w + j];
        W[k * w + j] = W[p * w + j];
        W[p * w + j] = t;
      }
    for (int i = k + 1; i < n; ++i) {
      double f = W[i * w + k] / W[k * w + k];
      if (f != 0.0)
        for (int j = k; j <= n; ++j) W[i * w + j] -= f * W[k * w + j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = W[i * w + n];
    for (int j = i + 1; j < n; ++j) s -= W[i * w + j] * x[j];
    x[i] = s / W[i * w + i];
  }
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return -1;
  return 0;
}

/* LDL^T factorisation of the symmetric matrix H + mu I (dense, row-major n x n),
 * eliminating the joints from the tip (index n-1) down to the base:
 *   H + mu I = U diag(D) U^T,  U unit upper triangular.
 * A (n x n) receives U above its diagonal; D the pivots.  By Sylvester's law of
 * inertia the number of negative pivots is the number of negative eigenvalues, so
 * H + mu I is positive definite exactly when every pivot is.  Returns the number of
 * negative pivots, or -1 on a zero or non-finite pivot. */
static int ldlt_tip(int n, const double* H, double mu, double* A, double* D) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[i * n + j] = H[i * n + j] + (i == j ? mu : 0.0);
  int neg = 0;
  for (int k = n - 1; k >= 0; --k) {
    double dk = A[k * n + k];
    if (!isfinite(dk) || dk == 0.0) return -1;
    D[k] = dk;
    if (dk < 0.0) ++neg;
    for (int i = 0; i < k; ++i) A[i * n + k] /= dk; /* U_ik */
    for (int i = 0; i < k; ++i)
      for (int j = 0; j <= i; ++j) {
        A[i * n + j] -= A[i * n + k] * dk * A[j * n + k];
        A[j * n + i] = A[i * n + j];
      }
  }
  return neg;
}

/* Direction of negative curvature from the factorisation above: v with U^T v = e_k, so
 * that v^T (H + mu I) v = D_k.  v vanishes below joint k and v_k = 1. */
static void neg_curv_dir(int n, const double* A, int k, double* v) {
  for (int m = 0; m < n; ++m) v[m] = 0.0;
  v[k] = 1.0;
  for (int m = k + 1; m < n; ++m) {
    double s = 0.0;
    for (int i = k; i < m; ++i) s += A[i * n + m] * v[i];
    v[m] = -s;
  }
}

typedef struct {
  int iters, backtracks, mu_raises, status, neg_steps, tie_steps;
  double rho;
} vo_solve_stats;

/* Descent of Pi from th (in place) to a local minimum (Eq. 4 is an argmin).
 * At each iterate, with the exact Hessian H (analytic; by central differences of r when
 * fd_h > 0) and delta = pd_shift M_max:
 *  - factorise H + mu I by LDL^T from the tip to the base (ldlt_tip), mu starting at
 *    max(c_mu max_j |r_j|, delta) and raised tenfold only when a pivot vanishes;
 *  - converged (status 0) when rho = max_j |r_j| / M_max <= tol and H + delta I is
 *    positive definite: a stationary point that is not a saddle;
 *  - H + mu I positive definite: the step (H + mu I) d = -r (Gaussian elimination), an
 *    implicit Euler step of the overdamped motion (gradient flow) that the quasi-static
 *    model stands for, which becomes Newton's step as the residual vanishes;
 *  - otherwise a step along negative curvature: d = s v with v from neg_curv_dir at the
 *    most negative pivot (ties: the joint nearest the base), its sign chosen so that
 *    r.d <= 0, and d_k > 0 when |r.v| <= tol M_max |v|_1 (a slope that a residual within
 *    the convergence tolerance could produce: at a converged saddle the sign of r.v is
 *    noise, and a symmetric saddle has r.v = 0);
 *  - cap max_j |d_j| at step_max (curvature steps are scaled to it);
 *  - Armijo backtracking on Pi (halving, constant c1) against the predicted change
 *    alpha r.d (+ alpha^2 d.H d / 2 for a curvature step), skipped once the predicted
 *    decrease of the full step is below 1e-12 M_max (round-off level of Pi).
 * status: 0 converged, 1 iteration limit, 2 no descent / line search failure,
 * 4 non-finite state. */
static void chain_solve(const vo_chain* c0, double* th, vo_solve_stats* st, vo_pose* w) {
  vo_chain cc = *c0;
  vo_chain* c = &cc;
  const vo_prm* P = c->P;
  const int nj = c->n;        /* joints; the step cap applies to them */
  const int nv = nj + c->soft; /* values: soft growth adds u = th[nj] (the buffers' size) */
  size_t nn = (size_t)nv;
  double* buf = (double*)malloc(sizeof(double) * (2 * nn * nn + nn * (nn + 1) + 11 * nn + 16));
  double* H = buf;
  double* A = H + nn * nn;
  double* W = A + nn * nn;
  double* r = W + nn * (nn + 1);
  double* rp = r + nn;
  double* rm = rp + nn;
  double* d = rm + nn;
  double* tt = d + nn;
  double* ha = tt + nn;
  double* hb = ha + nn;
  double* hu = hb + nn;
  double* piv = hu + nn;
  double* Hd = piv + nn;
  int capc = 2 * nv * (c->K > 0 ? c->K : 1) + 1, ncl = 0;
  vo_contact* cl = (vo_contact*)malloc(sizeof(vo_contact) * (size_t)capc);
  const double delta = P->pd_shift * c->Mmax;
  memset(st, 0, sizeof(*st));
  st->status = 1;
  double Pi = chain_eval(c, th, r, 1, cl, capc, &ncl, w);
  for (int it = 0; it <= P->max_iter; ++it) {
    /* soft growth: u >= 0; on the bound with dPi/du > 0 it is held there and the
     * iteration works on the joints alone */
    c->frozen = c->soft && th[nj] <= 0.0 && r[nj] > 0.0;
    const int n = nj + (c->soft && !c->frozen); /* this iteration's variables */
    double rmax = 0.0;
    for (int j = 0; j < n; ++j) rmax = fmax(rmax, fabs(r[j]));
    st->rho = rmax / c->Mmax;
    if (!isfinite(st->rho) || !isfinite(Pi)) {
      st->status = 4;
      break;
    }
    const int small = st->rho <= P->tol;
    if (P->fd_h > 0.0) {
      /* Hessian by central differences of r (cross-check mode) */
      double h = P->fd_h;
      for (int j = 0; j < n; ++j) {
        memcpy(tt, th, sizeof(double) * nn); /* (u, when held, stays) */
        tt[j] = th[j] + h;
        chain_eval(c, tt, rp, 0, NULL, 0, NULL, w);
        tt[j] = th[j] - h;
        chain_eval(c, tt, rm, 0, NULL, 0, NULL, w);
        for (int i = 0; i < n; ++i) H[i * n + j] = (rp[i] - rm[i]) / (2.0 * h);
      }
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
          double a = 0.5 * (H[i * n + j] + H[j * n + i]);
          H[i * n + j] = H[j * n + i] = a;
        }
      chain_eval(c, th, NULL, 0, NULL, 0, NULL, w); /* restore poses */
    } else {
      chain_hessian(c, th, cl, ncl < capc ? ncl : capc, w, H, ha, hb, hu);
    }
    /* mu: the implicit-Euler damping 1/h = c_mu |r|_inf, at least delta; raised tenfold
     * while a pivot vanishes or the step does not descend */
    double mu = fmax(P->c_mu * rmax, delta);
    int mode = 0; /* 1: Newton step in d, 2: curvature step in d, 3: converged */
    double slope = 0.0, curv = 0.0;
    for (int tries = 0; tries < 24; ++tries) {
      if (tries > 0) {
        mu = fmax(P->mu_up * mu, delta);
        st->mu_raises++;
      }
      int neg = ldlt_tip(n, H, mu, A, piv);
      if (neg < 0) continue;
      if (neg == 0) {
        if (small) {
          mode = 3;
          break;
        }
        for (int i = 0; i < n; ++i) rp[i] = -r[i];
        if (dense_solve(n, H, mu, rp, d, W) != 0) continue;
        slope = 0.0;
        for (int i = 0; i < n; ++i) slope += r[i] * d[i];
        if (slope < 0.0) {
          mode = 1;
          break;
        }
        continue;
      }
      int k = 0;
      for (int j = 1; j < n; ++j)
        if (piv[j] < piv[k]) k = j;
      neg_curv_dir(n, A, k, d);
      double vmax = 0.0, rv = 0.0, v1 = 0.0;
      for (int i = 0; i < n; ++i) {
        if (i < nj) vmax = fmax(vmax, fabs(d[i]));
        rv += r[i] * d[i];
        v1 += fabs(d[i]);
      }
      if (vmax == 0.0) vmax = fabs(d[nj]); /* soft growth: curvature along u alone */
      /* the slope along v counts as zero when a residual within the tolerance could
       * produce it (always so at a converged saddle): then the tie rule, d_k > 0 */
      const int tie = fabs(rv) <= P->tol * c->Mmax * v1;
      double s = (tie ? 1.0 : (rv > 0.0 ? -1.0 : 1.0)) * P->step_max / vmax;
      for (int i = 0; i < n; ++i) d[i] *= s;
      slope = s * rv;
      curv = 0.0;
      for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int j = 0; j < n; ++j) a += H[i * n + j] * d[j];
        Hd[i] = a;
        curv += d[i] * a;
      }
      mode = 2;
      st->neg_steps++;
      if (tie) st->tie_steps++; /* the sign came from the tie rule */
      break;
    }
    if (mode == 3) {
      st->status = 0;
      break;
    }
    if (it == P->max_iter) break;
    st->iters++;
    if (mode == 0) {
      st->status = 2;
      break;
    }
    if (mode == 1) {
      /* cap the joint-space step length so that the iterates follow the flow */
      double dmax = 0.0;
      for (int i = 0; i < nj; ++i) dmax = fmax(dmax, fabs(d[i]));
      if (dmax > P->step_max) {
        double f = P->step_max / dmax;
        for (int i = 0; i < n; ++i) d[i] *= f;
        slope *= f;
      }
    }
    double alpha = 1.0, Pn = 0.0;
    int accepted = 0;
    int skip = (-(slope + 0.5 * curv) < 1e-12 * c->Mmax);
    for (int ls = 0; ls < 40; ++ls) {
      for (int i = 0; i < nj; ++i) tt[i] = th[i] + alpha * d[i];
      /* soft growth: a trial tip length below zero is projected onto u = 0, and the
       * predicted change then takes the tip length's actual move */
      double lin = alpha * slope;
      if (c->soft) {
        tt[nj] = th[nj];
        if (!c->frozen) {
          const double ut = th[nj] + alpha * d[nj];
          tt[nj] = ut;
          if (ut < 0.0) {
            tt[nj] = 0.0;
            lin += r[nj] * (-th[nj] - alpha * d[nj]);
          }
        }
      }
      Pn = chain_eval(c, tt, rm, 1, cl, capc, &ncl, w);
      if (skip || Pn <= Pi + P->c1 * (lin + 0.5 * alpha * alpha * curv)) {
        accepted = 1;
        break;
      }
      alpha *= 0.5;
      st->backtracks++;
    }
    if (!accepted) {
      st->status = 2;
      break;
    }
    if (vo_verbose)
      fprintf(stderr, "it %d rho %.3e mu %.3e mode %d slope %.3e curv %.3e alpha %.3e Pi %.12e\n",
              it, st->rho, mu, mode, slope, curv, alpha, Pn);
    memcpy(th, tt, sizeof(double) * nn);
    memcpy(r, rm, sizeof(double) * nn);
    Pi = Pn;
  }
  c->frozen = 0;
  free(cl);
  free(buf);
}

/* ------------------------------------------------------------------------- */
/* rollout driver */

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

/* per-joint pressure-weighted sPAM coverage: w = |[s0,s1] ∩ [j l,(j+1) l]| / l */
static void spam_coverage(int n, double l, const double* spam, int ns, double* Pp, double* Pm) {
  for (int j = 0; j < n; ++j) Pp[j] = Pm[j] = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double* e = spam + 4 * s;
    for (int j = 0; j < n; ++j) {
      double lo = fmax(e[0], j * l), hi = fmin(e[1], (j + 1) * l);
      if (hi > lo) {
        double w = (hi - lo) / l;
        if (e[2] > 0.0) Pp[j] += w * e[3]; else Pm[j] += w * e[3];
      }
    }
  }
}

static void chain_init(vo_chain* c, const vo_prm* P, const double* prm, const double* d, int K,
                       const int* kind, const double* obs) {
  memset(c, 0, sizeof(*c));
  c->P = P;
  c->l = d[0];
  c->R = d[1];
  c->Pv = d[2];
  c->bx = d[3];
  c->by = d[4];
  c->bpsi = d[5];
  c->arm = 2.0 * c->R + P->Ract;
  c->Mmax = VO_PI * c->Pv * c->R * c->R * c->R;
  c->K = K;
  c->kind = kind;
  c->obs = obs;
  c->last_len = c->l;
  c->G = gfit_get(c->l, prm);
}

/* Roll out every instance for n_steps growth steps (Alg. 1 repeated).  Arrays as in
 * the workload module.  Outputs (all nullable except theta):
 *  theta  [B][n_max]        final joint angles
 *  tip    [B][T][3]         tip x, y, heading after each step
 *  rho    [B][T], iters [B][T], status [B][T] (-1 once the instance is full grown),
 *  ncont  [B][T], chash [B][T] (order-free hash of the contact set), maxpen [B][T]
 *  traj   [B][T][n_max]     joint angles after each step
 *  stats  [B][6]            total iterations, backtracks, damping raises, max contacts,
 *                           steps along negative curvature, those of them whose sign
 *                           the tie rule chose
 *  tiplen [B][T]            length of the tip link after each step
 *
 * Hard growth (wg = 0): each step appends a link at zero angle whose length reaches l
 * in `substeps` sub-steps (Sec. 4.1's growth at a rate, with the growth term of Eq. 4
 * satisfied exactly).  Soft growth (wg > 0): the tip link's length u l is a variable
 * of the minimisation, under the growth term (wg/2) (l (tgt - u))^2 of Eq. 4, whose
 * target grows at the prescribed rate of one link length per step: at sub-step s of
 * step t, tgt = t + s/substeps - (n - 1) (capped at 1 once the robot has its target
 * link count).  A step appends a link only when the tip link has reached full length
 * (u >= 1; the excess u - 1 starts the new link), so a blocked tip stops growing while
 * its target, and with it the growth force, keeps rising; a tip link that has grown
 * longer than a link within a sub-step (the growth released when a block gives way) is
 * split into a full link and a new tip link at zero angle, and the sub-step solved
 * again.  The robot is done when it has its target link count with a full tip link. */
int vo_rollout(int B, const int* inst_i, const double* inst_d, const double* spam,
               const int* obs_kind, const double* obs_d, const double* prm, int n_steps,
               int n_threads, int n_max, double* theta, double* tip, double* rho, int* iters,
               int* status, int* ncont, uint64_t* chash, double* maxpen, double* traj,
               double* stats, double* tiplen) {
  vo_prm P;
  prm_from(prm, &P);
  gl_init();
  for (int b = 0; b < B; ++b) gfit_get(inst_d[6 * b], prm); /* build fits up front */
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int b = 0; b < B; ++b) {
    const int* ii = inst_i + 5 * b;
    int ntar = ii[0];
    int nalloc = ntar > 0 ? ntar : 1;
    vo_chain c;
    chain_init(&c, &P, prm, inst_d + 6 * b, ii[4], obs_kind + ii[3], obs_d + 4 * (size_t)ii[3]);
    double* Pp = (double*)calloc((size_t)nalloc * 2, sizeof(double));
    double* Pm = Pp + nalloc;
    spam_coverage(ntar, c.l, spam + 4 * (size_t)ii[1], ii[2], Pp, Pm);
    c.Pp = Pp;
    c.Pm = Pm;
    double* th = (double*)calloc((size_t)nalloc + 1, sizeof(double)); /* + u (soft) */
    vo_pose w;
    pose_alloc(&w, nalloc);
    int capc = 2 * nalloc * (c.K > 0 ? c.K : 1) + 1;
    vo_contact* cl = (vo_contact*)malloc(sizeof(vo_contact) * (size_t)capc);
    double tot_it = 0, tot_bt = 0, tot_mu = 0, max_c = 0, tot_neg = 0, tot_tie = 0;
    c.n = 0;
    c.soft = P.wg > 0.0;
    const double full = 1.0 - 1e-12; /* a tip link at full length */
    for (int t = 0; t < n_steps; ++t) {
      int st_worst = 0, it_sum = 0;
      double rho_last = 0.0;
      int grow;
      if (c.soft) {
        if (c.n == 0 || (th[c.n] >= full && c.n < ntar)) {
          const double u = c.n == 0 ? 0.0 : fmax(th[c.n] - 1.0, 0.0);
          c.n += 1;
          th[c.n - 1] = 0.0;
          th[c.n] = u;
        }
        grow = !(c.n == ntar && th[c.n] >= full);
      } else {
        grow = c.n < ntar;
        if (grow) {
          c.n += 1;
          th[c.n - 1] = 0.0;
        }
      }
      if (grow) {
        for (int s = 1; s <= P.substeps; ++s) {
          for (;;) {
            if (c.soft) {
              c.tgt = (double)t + (double)s / P.substeps - (double)(c.n - 1);
              if (c.n == ntar && c.tgt > 1.0) c.tgt = 1.0;
            } else {
              c.last_len = c.l * (double)s / P.substeps;
            }
            vo_solve_stats st;
            chain_solve(&c, th, &st, &w);
            it_sum += st.iters;
            tot_bt += st.backtracks;
            tot_mu += st.mu_raises;
            tot_neg += st.neg_steps;
            tot_tie += st.tie_steps;
            if (st.status > st_worst) st_worst = st.status;
            rho_last = st.rho;
            /* soft growth: a tip link longer than a link (growth released after a block)
             * is split, its first l staying as link n - 1 and the rest starting a new link
             * at zero angle, and the sub-step is solved again */
            if (!(c.soft && c.n < ntar && th[c.n] > 1.0 + 1e-12)) break;
            const double u = th[c.n] - 1.0;
            th[c.n] = 0.0;
            c.n += 1;
            th[c.n] = u;
          }
        }
      } else {
        if (!c.soft) c.last_len = c.l;
        st_worst = -1;
      }
      tot_it += it_sum;
      int ncl = 0;
      if (c.n > 0) chain_eval(&c, th, NULL, 0, cl, capc, &ncl, &w);
      if (ncl > max_c) max_c = ncl;
      size_t bt = (size_t)b * n_steps + t;
      if (tip) {
        double hd = c.bpsi;
        for (int i = 0; i < c.n; ++i) hd += th[i];
        tip[3 * bt + 0] = c.n > 0 ? w.px[c.n] : c.bx;
        tip[3 * bt + 1] = c.n > 0 ? w.py[c.n] : c.by;
        tip[3 * bt + 2] = hd;
      }
      if (rho) rho[bt] = rho_last;
      if (tiplen) tiplen[bt] = c.n == 0 ? 0.0 : (c.soft ? th[c.n] * c.l : c.last_len);
      if (iters) iters[bt] = it_sum;
      if (status) status[bt] = st_worst;
      {
        /* contact set: (link, obstacle) pairs in which either disk of the link penetrates */
        uint64_t hsh = 0;
        double mp = 0.0;
        int npair = 0;
        for (int e = 0; e < ncl && e < capc; ++e) {
          int dup = 0;
          for (int f = 0; f < e; ++f)
            if (cl[f].i == cl[e].i && cl[f].k == cl[e].k) dup = 1;
          if (!dup) {
            hsh += splitmix64((uint64_t)cl[e].i * 1024u + (uint64_t)cl[e].k);
            ++npair;
          }
          if (cl[e].pen > mp) mp = cl[e].pen;
        }
        if (ncont) ncont[bt] = npair;
        if (chash) chash[bt] = hsh;
        if (maxpen) maxpen[bt] = mp;
      }
      if (traj)
        for (int i = 0; i < n_max; ++i) traj[bt * n_max + i] = (i < c.n) ? th[i] : 0.0;
    }
    for (int i = 0; i < n_max; ++i) theta[(size_t)b * n_max + i] = (i < c.n) ? th[i] : 0.0;
    if (stats) {
      stats[6 * b + 0] = tot_it;
      stats[6 * b + 1] = tot_bt;
      stats[6 * b + 2] = tot_mu;
      stats[6 * b + 3] = max_c;
      stats[6 * b + 4] = tot_neg;
      stats[6 * b + 5] = tot_tie;
    }
    free(Pp);
    free(th);
    free(w.px);
    free(cl);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* single-chain hooks for the tests */

/* Residual r [n], energy Pi (returned), contacts for one chain of n links.
 * contacts (nullable) receives up to cap rows (i, k, lam, x, y, nx, ny, pen). */
/* soft = 1: th and r hold n + 1 entries, the last being u (the tip link's length in
 * link lengths), and tgt is its target (soft growth, see vo_rollout) */
static double chain_eval_hook(int n, const double* d, const double* spam, int ns, int K,
                              const int* kind, const double* obs, const double* prm,
                              double last_len, int soft, double tgt, const double* th, double* r,
                              int* ncontact, double* contacts, int cap) {
  vo_prm P;
  prm_from(prm, &P);
  gl_init();
  vo_chain c;
  chain_init(&c, &P, prm, d, K, kind, obs);
  double* Pp = (double*)calloc((size_t)n * 2 + 2, sizeof(double));
  spam_coverage(n, c.l, spam, ns, Pp, Pp + n + 1);
  c.Pp = Pp;
  c.Pm = Pp + n + 1;
  c.n = n;
  c.last_len = last_len > 0.0 ? last_len : c.l;
  c.soft = soft;
  c.tgt = tgt;
  vo_pose w;
  pose_alloc(&w, n + 1);
  int capc = 2 * n * (K > 0 ? K : 1) + 1;
  vo_contact* cl = (vo_contact*)malloc(sizeof(vo_contact) * (size_t)capc);
  int ncl = 0;
  double Pi = chain_eval(&c, th, r, 1, cl, capc, &ncl, &w);
  if (ncontact) *ncontact = ncl;
  if (contacts)
    for (int e = 0; e < ncl && e < cap && e < capc; ++e) {
      double* o = contacts + 8 * e;
      o[0] = cl[e].i;
      o[1] = cl[e].k;
      o[2] = cl[e].lam;
      o[3] = cl[e].xx;
      o[4] = cl[e].xy;
      o[5] = cl[e].nx;
      o[6] = cl[e].ny;
      o[7] = cl[e].pen;
    }
  free(cl);
  free(w.px);
  free(Pp);
  return Pi;
}

double vo_chain_eval(int n, const double* d, const double* spam, int ns, int K, const int* kind,
                     const double* obs, const double* prm, double last_len, const double* th,
                     double* r, int* ncontact, double* contacts, int cap) {
  return chain_eval_hook(n, d, spam, ns, K, kind, obs, prm, last_len, 0, 0.0, th, r, ncontact,
                         contacts, cap);
}

double vo_chain_eval_soft(int n, const double* d, const double* spam, int ns, int K,
                          const int* kind, const double* obs, const double* prm, double tgt,
                          const double* x, double* r, int* ncontact, double* contacts, int cap) {
  return chain_eval_hook(n, d, spam, ns, K, kind, obs, prm, 0.0, 1, tgt, x, r, ncontact,
                         contacts, cap);
}

/* Solve one equilibrium from th (in place); returns status; info = iters, backtracks,
 * damping raises, rho, steps along negative curvature */
static int chain_solve_hook(int n, const double* d, const double* spam, int ns, int K,
                            const int* kind, const double* obs, const double* prm,
                            double last_len, int soft, double tgt, double* th, double* info) {
  vo_prm P;
  prm_from(prm, &P);
  gl_init();
  vo_chain c;
  chain_init(&c, &P, prm, d, K, kind, obs);
  double* Pp = (double*)calloc((size_t)n * 2 + 2, sizeof(double));
  spam_coverage(n, c.l, spam, ns, Pp, Pp + n + 1);
  c.Pp = Pp;
  c.Pm = Pp + n + 1;
  c.n = n;
  c.last_len = last_len > 0.0 ? last_len : c.l;
  c.soft = soft;
  c.tgt = tgt;
  vo_pose w;
  pose_alloc(&w, n + 1);
  vo_solve_stats st;
  chain_solve(&c, th, &st, &w);
  if (info) {
    info[0] = st.iters;
    info[1] = st.backtracks;
    info[2] = st.mu_raises;
    info[3] = st.rho;
    info[4] = st.neg_steps;
  }
  free(w.px);
  free(Pp);
  return st.status;
}

int vo_chain_solve(int n, const double* d, const double* spam, int ns, int K, const int* kind,
                   const double* obs, const double* prm, double last_len, double* th,
                   double* info) {
  return chain_solve_hook(n, d, spam, ns, K, kind, obs, prm, last_len, 0, 0.0, th, info);
}

int vo_chain_solve_soft(int n, const double* d, const double* spam, int ns, int K,
                        const int* kind, const double* obs, const double* prm, double tgt,
                        double* x, double* info) {
  return chain_solve_hook(n, d, spam, ns, K, kind, obs, prm, 0.0, 1, tgt, x, info);
}

/* G, dG/deps, int_0^eps G from the Chebyshev fit; info = G(0), eps_max, tail size */
void vo_gfit_eval(double l0, const double* prm, int n, const double* eps, double* G, double* dG,
                  double* IG, double* info) {
  const vo_gfit* g = gfit_get(l0, prm);
  for (int i = 0; i < n; ++i)
    gfit_eval(g, eps[i], G ? &G[i] : NULL, dG ? &dG[i] : NULL, IG ? &IG[i] : NULL);
  if (info) {
    info[0] = g->G0;
    info[1] = g->emax;
    info[2] = fabs(g->c[g->N]) + fabs(g->c[g->N - 1]);
  }
}

void vo_spam_coverage(int n, double l, const double* spam, int ns, double* Pp, double* Pm) {
  spam_coverage(n, l, spam, ns, Pp, Pm);
}

/* joint moment and energy for explicit per-joint pressures (for tests) */
void vo_joint_law(const double* d, double pp, double pm, const double* prm, int n,
                  const double* th, double* q, double* E) {
  vo_prm P;
  prm_from(prm, &P);
  gl_init();
  vo_chain c;
  chain_init(&c, &P, prm, d, 0, NULL, NULL);
  double Pp = pp, Pm = pm;
  c.Pp = &Pp;
  c.Pm = &Pm;
  for (int i = 0; i < n; ++i) joint_law(&c, 0, th[i], q ? &q[i] : NULL, E ? &E[i] : NULL);
}

/* analytic Hessian H [m][m] of Pi for one chain (m = n, or n + 1 for soft growth) */
static void chain_hessian_hook(int n, const double* d, const double* spam, int ns, int K,
                               const int* kind, const double* obs, const double* prm,
                               double last_len, int soft, double tgt, const double* th,
                               double* H) {
  vo_prm P;
  prm_from(prm, &P);
  gl_init();
  vo_chain c;
  chain_init(&c, &P, prm, d, K, kind, obs);
  double* Pp = (double*)calloc((size_t)n * 2 + 2, sizeof(double));
  spam_coverage(n, c.l, spam, ns, Pp, Pp + n + 1);
  c.Pp = Pp;
  c.Pm = Pp + n + 1;
  c.n = n;
  c.last_len = last_len > 0.0 ? last_len : c.l;
  c.soft = soft;
  c.tgt = tgt;
  vo_pose w;
  pose_alloc(&w, n + 1);
  int capc = 2 * n * (K > 0 ? K : 1) + 1, ncl = 0;
  vo_contact* cl = (vo_contact*)malloc(sizeof(vo_contact) * (size_t)capc);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(3 * n + 3));
  chain_eval(&c, th, NULL, 0, cl, capc, &ncl, &w);
  chain_hessian(&c, th, cl, ncl, &w, H, tmp, tmp + n + 1, tmp + 2 * n + 2);
  free(tmp);
  free(cl);
  free(w.px);
  free(Pp);
}

void vo_chain_hessian(int n, const double* d, const double* spam, int ns, int K, const int* kind,
                      const double* obs, const double* prm, double last_len, const double* th,
                      double* H) {
  chain_hessian_hook(n, d, spam, ns, K, kind, obs, prm, last_len, 0, 0.0, th, H);
}

void vo_chain_hessian_soft(int n, const double* d, const double* spam, int ns, int K,
                           const int* kind, const double* obs, const double* prm, double tgt,
                           const double* x, double* H) {
  chain_hessian_hook(n, d, spam, ns, K, kind, obs, prm, 0.0, 1, tgt, x, H);
}

/* ------------------------------------------------------------------------- */
/* Gradient of L = sum_t w_t |tip_t - goal|^2 with respect to each sPAM's pressure,
 * start and end (arc length).  Every weighted step's state is a converged equilibrium,
 * r_t(theta_t; p) = 0, and r_t does not depend on the previous step's state, so
 *   dL/dp = - sum_t lam_t . dr_t/dp,   H_t lam_t = w_t dL_t/dtheta,
 * with H_t the exact Hessian at theta_t (dense solve here).  p enters r only through
 * the joint coverage: dq_j/dP+_j = -arm G(eps+_j), dq_j/dP-_j = +arm G(eps-_j), and
 * P+-_j = sum_s w_sj P_s with w_sj = |[s0, s1] ^ [j l, (j+1) l]| / l.
 * traj: [B][T][n_max] joint angles after each step (as vo_rollout writes them);
 * weights: [T] (NULL: the last step only); goal: [B][2]; outputs indexed like spam. */
int vo_gradient(int B, const int* inst_i, const double* inst_d, const double* spam,
                const int* obs_kind, const double* obs_d, const double* prm, int T, int n_max,
                const double* traj, const double* weights, const double* goal, int n_threads,
                double* dP, double* ds0, double* ds1, double* loss) {
  vo_prm P;
  prm_from(prm, &P);
  if (P.wg > 0.0) return -1; /* soft growth: the states also hold the tip length; not here */
  gl_init();
  for (int b = 0; b < B; ++b) gfit_get(inst_d[6 * b], prm);
  /* per-robot partial sums (robots may share sPAM records), added in robot order */
  size_t* slot = (size_t*)malloc(sizeof(size_t) * ((size_t)B + 1));
  slot[0] = 0;
  for (int b = 0; b < B; ++b) slot[b + 1] = slot[b] + (size_t)inst_i[5 * b + 2];
  double* part = (double*)calloc(3 * slot[B] + 1, sizeof(double));
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int b = 0; b < B; ++b) {
    const int* ii = inst_i + 5 * b;
    const int ntar = ii[0], ns = ii[2];
    double* pb = part + 3 * slot[b];
    const double* sp = spam + 4 * (size_t)ii[1];
    vo_chain c;
    chain_init(&c, &P, prm, inst_d + 6 * b, ii[4], obs_kind + ii[3], obs_d + 4 * (size_t)ii[3]);
    double* Pp = (double*)calloc((size_t)ntar * 2 + 2, sizeof(double));
    spam_coverage(ntar, c.l, sp, ns, Pp, Pp + ntar + 1);
    c.Pp = Pp;
    c.Pm = Pp + ntar + 1;
    size_t nn = (size_t)ntar;
    double* H = (double*)malloc(sizeof(double) * (nn * nn + nn * (nn + 1) + 8 * nn + 8));
    double* Wm = H + nn * nn;
    double* g = Wm + nn * (nn + 1);
    double* lam = g + nn;
    double* ha = lam + nn;
    double* hb = ha + nn;
    double* hu = hb + nn;
    vo_pose w;
    pose_alloc(&w, ntar + 1);
    int capc = 2 * ntar * (c.K > 0 ? c.K : 1) + 1, ncl = 0;
    vo_contact* cl = (vo_contact*)malloc(sizeof(vo_contact) * (size_t)capc);
    double Lsum = 0.0;
    for (int t = 0; t < T; ++t) {
      double wt = weights ? weights[t] : (t == T - 1 ? 1.0 : 0.0);
      if (wt == 0.0) continue;
      int n = t + 1 < ntar ? t + 1 : ntar;
      c.n = n;
      c.last_len = c.l;
      const double* th = traj + ((size_t)b * T + t) * n_max;
      chain_eval(&c, th, NULL, 0, cl, capc, &ncl, &w);
      double ex = w.px[n] - goal[2 * b], ey = w.py[n] - goal[2 * b + 1];
      Lsum += wt * (ex * ex + ey * ey);
      /* dL/dtheta_j = 2 w (tip - goal) . (z x (tip - p_j)) */
      for (int j = 0; j < n; ++j) {
        double vx = -(w.py[n] - w.py[j]), vy = w.px[n] - w.px[j];
        g[j] = 2.0 * wt * (ex * vx + ey * vy);
      }
      chain_hessian(&c, th, cl, ncl < capc ? ncl : capc, &w, H, ha, hb, hu);
      if (dense_solve(n, H, 0.0, g, lam, Wm) != 0) continue;
      for (int s = 0; s < ns; ++s) {
        const double* e = sp + 4 * s;
        double gP = 0.0, g0 = 0.0, g1 = 0.0;
        for (int j = 0; j < n; ++j) {
          double lo = fmax(e[0], j * c.l), hi = fmin(e[1], (j + 1) * c.l);
          if (!(hi > lo)) continue;
          double th_j = th[j];
          double eps = e[2] > 0.0 ? (th_j > 0.0 ? c.arm * th_j / c.l : 0.0)
                                  : (th_j < 0.0 ? -c.arm * th_j / c.l : 0.0);
          double G;
          gfit_eval(c.G, eps, &G, NULL, NULL);
          double dq = e[2] > 0.0 ? -c.arm * G : c.arm * G; /* dq_j / dP^side_j */
          double wsj = (hi - lo) / c.l;
          gP += -lam[j] * dq * wsj;
          if (e[0] > j * c.l) g0 += -lam[j] * dq * (-e[3] / c.l);
          if (e[1] < (j + 1) * c.l) g1 += -lam[j] * dq * (e[3] / c.l);
        }
        pb[3 * s + 0] += gP;
        pb[3 * s + 1] += g0;
        pb[3 * s + 2] += g1;
      }
    }
    if (loss) loss[b] = Lsum;
    free(cl);
    free(w.px);
    free(H);
    free(Pp);
  }
  for (int b = 0; b < B; ++b)
    for (int s = 0; s < inst_i[5 * b + 2]; ++s) {
      const int k = inst_i[5 * b + 1] + s;
      dP[k] = ds0[k] = ds1[k] = 0.0;
    }
  for (int b = 0; b < B; ++b)
    for (int s = 0; s < inst_i[5 * b + 2]; ++s) {
      const int k = inst_i[5 * b + 1] + s;
      const double* pb = part + 3 * (slot[b] + (size_t)s);
      dP[k] += pb[0];
      ds0[k] += pb[1];
      ds1[k] += pb[2];
    }
  free(part);
  free(slot);
  return 0;
}
