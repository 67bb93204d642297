// vs_synth.hip -- gfx950 kernels of actuator synthesis (Sec. 4.2).
//
// A joint whose link is covered by one sPAM of unit length l0 at pressure P rests in free
// space (Sec. 3.3, Eq. 3b = 0) at the angle theta where the wrinkling moment (Eq. 2)
// balances the actuator's moment at the strain of Eq. 3a:
//   q = pi P_vine R^3 h(theta) - arm P G,   theta = eps l / arm.
// Along the sPAM's states m in [m0, 1/2] (m0: zero strain) the strain eps(m) of Eq. 1a
// rises to its slack value and the force per unit pressure G(m) of Eq. 1d falls to zero,
// so q rises from negative to positive and bisection on m finds the one root (below m0
// the strain is negative and so is q).  Each state
// is solved exactly from Eq. 1 (no fitted table: for unit lengths above about 35 mm the
// actuator saturates inside the strain range, and G(eps) has a kink there).
//
// One 64-lane wave solves one (pressure, unit length): the 96 Gauss-Legendre nodes of the
// elliptic integrals F and E are spread over the lanes and summed by a wave reduction;
// all other control flow is uniform across the wave.  One thread per target then takes
// the highest pressure with a unit length whose angle is within the tolerance, and of its
// unit lengths the one whose angle is nearest.

#include "vs_synth.h"

namespace vs {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kLanes = 64;

__device__ double wave_sum(double v) {
#pragma unroll
  for (int o = kLanes / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kLanes);
  return v;
}

// F(phi|m) and E(phi|m) (parameter convention): two 48-point Gauss-Legendre panels over
// [0, phi] of (1 - m sin^2 t)^(-1/2) and (1 - m sin^2 t)^(1/2), analytic for m <= 1/2.
__device__ void ellint_FE(const SynthArgs& A, double phi, double m, double* F, double* E) {
  double sF = 0.0, sE = 0.0;
  for (int q = threadIdx.x; q < 96; q += kLanes) {
    const int panel = q >= 48, i = q - 48 * panel;
    const double h = 0.25 * phi, c = h * (2 * panel + 1);
    const double s = sin(c + h * A.gl_x[i]), d = sqrt(1.0 - m * s * s);
    sF += A.gl_w[i] * h / d;
    sE += A.gl_w[i] * h * d;
  }
  *F = wave_sum(sF);
  *E = wave_sum(sE);
}

// Eq. 1b with l_a = l0, times cos^2(phi); its smallest root in (0, phi_Rc] is the
// unsaturated state.  dres: its derivative in phi.
__device__ double eq1b(const SynthArgs& A, double l0, double m, double phi, double* dres) {
  double F, E;
  ellint_FE(A, phi, m, &F, &E);
  const double c = cos(phi), s = sin(phi), sm = sqrt(m);
  if (dres) *dres = (c / sqrt(1.0 - m * s * s) - F * s) / sm + (l0 / A.R_c) * 2.0 * c * s;
  return F * c / sm - (l0 / A.R_c) * (c * c + A.a_corr / (2.0 * m));
}

// Strain and force per unit pressure of the state m (Eq. 1a-d): unsaturated when Eq. 1b
// has a root up to phi_Rc (a scan of 64 brackets, then safeguarded Newton), else
// saturated at phi = phi_Rc with the active length from Eq. 1b.
__device__ void spam_point(const SynthArgs& A, double l0, double m, double* eps, double* G,
                           double* phi_out = nullptr) {
  const double phi_rc = acos(A.R_c / A.R_act);
  double lo = 1e-12, flo = eq1b(A, l0, m, lo, nullptr), phi = -1.0;
  for (int k = 1; k <= 64 && phi < 0.0; ++k) {
    double hi = phi_rc * k / 64, fhi = eq1b(A, l0, m, hi, nullptr);
    if (flo < 0.0 && fhi >= 0.0) {
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 100; ++it) {
        double d, f = eq1b(A, l0, m, x, &d);
        if (f < 0.0) lo = x; else hi = x;
        double xn = x - f / d;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const bool done = fabs(xn - x) <= 1e-16 * x;
        x = xn;
        if (done) break;
      }
      phi = x;
    } else {
      lo = hi;
      flo = fhi;
    }
  }
  double F, E, la = l0;
  if (phi < 0.0) {
    phi = phi_rc;
    ellint_FE(A, phi, m, &F, &E);
    const double c = cos(phi);
    la = A.R_c * F / (sqrt(m) * c * (1.0 + A.a_corr / (2.0 * m * c * c)));
  } else {
    ellint_FE(A, phi, m, &F, &E);
  }
  const double c = cos(phi);
  *eps = (la - 2.0 * A.R_c * (E - 0.5 * F) / (sqrt(m) * c)) / l0;
  *G = kPi * A.R_c * A.R_c * (1.0 - 2.0 * m) / (2.0 * m * c * c);
  if (phi_out) *phi_out = phi;
}

// m0: the state of zero strain (the strain of Eq. 1a rises with m on [m0, 1/2])
__device__ double zero_strain_m(const SynthArgs& A, double l0) {
  double lo = 1e-6, hi = 0.5, e, G;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    spam_point(A, l0, mid, &e, &G);
    if (e < 0.0) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// h = M / (pi P_vine R^3) of Eq. 2 above the wrinkling onset theta_on = 2 asin(eps_c),
// linear from 0 to its onset value 1/2 below it.
__device__ double wrinkle_h(double x, double eps_c) {
  const double th_on = 2.0 * asin(eps_c);
  if (x <= th_on) return x / (2.0 * th_on);
  x = fmin(x, kPi);
  const double arg = fmin(fmax(2.0 * eps_c / sin(0.5 * x) - 1.0, -1.0), 1.0);
  const double g = acos(arg);
  return (sin(2.0 * g) + 2.0 * kPi - 2.0 * g) / (4.0 * (sin(g) + (kPi - g) * cos(g)));
}

}  // namespace

__global__ void __launch_bounds__(kLanes) synth_angle_kernel(SynthArgs a) {
  const int pair = blockIdx.x;
  if (pair >= a.n_p * a.n_l) return;
  const int k = pair / a.n_l, j = pair - k * a.n_l;
  const double P = a.pressures[k], l0 = a.lengths[j];
  double e, G;
  // the rest state: the first m where the balance q turns non-negative.  Below the
  // zero-strain state m0 the strain and the angle are negative and q < 0 too, so the
  // bracket can start below m0 without finding it first.
  double lo = 1e-6, hi = 0.5;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    spam_point(a, l0, mid, &e, &G);
    const double q = a.m_max * wrinkle_h(e * a.link_len / a.arm, a.eps_c) - a.arm * P * G;
    if (q < 0.0) lo = mid; else hi = mid;
  }
  spam_point(a, l0, 0.5 * (lo + hi), &e, &G);
  if (threadIdx.x == 0) a.angles[pair] = e * a.link_len / a.arm;
}

// The sPAM state of a given strain (the inverse of Eq. 1a): m in [m0, 1/2] with
// eps(m) = eps by bisection, then phi and G there; strains at or beyond slack give the
// slack state (m = 1/2, G = 0), strains at or below zero the state m0.
__global__ void __launch_bounds__(kLanes) spam_solve_kernel(SynthArgs a, const double* eps,
                                                            const double* l0s, int n,
                                                            double* out) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const double target = eps[i], l0 = l0s[i];
  double e, G, phi;
  spam_point(a, l0, 0.5, &e, &G);
  const bool slack = target >= e;
  double lo = 0.5, hi = 0.5;
  if (!slack && target <= 0.0) {
    lo = zero_strain_m(a, l0);
  } else if (!slack) {
    // below m0 the strain is negative, below the target too: no need to find m0 first
    lo = 1e-6;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      spam_point(a, l0, mid, &e, &G);
      if (e < target) lo = mid; else hi = mid;
    }
  }
  const double m = (slack || target <= 0.0) ? lo : 0.5 * (lo + hi);
  spam_point(a, l0, m, &e, &G, &phi);
  if (threadIdx.x == 0) {
    out[4 * (size_t)i] = m;
    out[4 * (size_t)i + 1] = phi;
    out[4 * (size_t)i + 2] = G;
    out[4 * (size_t)i + 3] = e;
  }
}

// The surrogate of Sec. 4.3: a 2-32-2 perceptron with ReLU, y = W2 relu(W1 x + b1) + b2,
// weights packed as W1 [32][2], b1 [32], W2 [2][32], b2 [2]; one thread per sample.
__global__ void mlp_forward_kernel(const double* w, const double* x, int n, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x0 = x[2 * (size_t)i], x1 = x[2 * (size_t)i + 1];
  const double *W1 = w, *b1 = w + 64, *W2 = w + 96, *b2 = w + 160;
  double y0 = b2[0], y1 = b2[1];
#pragma unroll 8
  for (int k = 0; k < 32; ++k) {
    const double h = fmax(W1[2 * k] * x0 + W1[2 * k + 1] * x1 + b1[k], 0.0);
    y0 += W2[k] * h;
    y1 += W2[32 + k] * h;
  }
  y[2 * (size_t)i] = y0;
  y[2 * (size_t)i + 1] = y1;
}

__global__ void synth_select_kernel(SynthArgs a, const double* targets, int n_t, double tol,
                                    double* designs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_t) return;
  const double t = targets[i];
  double P = 0.0, l0 = 0.0, th = 0.0;
  for (int k = a.n_p - 1; k >= 0; --k) {
    const double* row = a.angles + (size_t)k * a.n_l;
    int best = 0;
    double err = fabs(row[0] - t);
    for (int j = 1; j < a.n_l; ++j) {
      const double e = fabs(row[j] - t);
      if (e < err) {
        err = e;
        best = j;
      }
    }
    if (err <= tol) {
      P = a.pressures[k];
      l0 = a.lengths[best];
      th = row[best];
      break;
    }
  }
  designs[3 * (size_t)i] = P;
  designs[3 * (size_t)i + 1] = l0;
  designs[3 * (size_t)i + 2] = th;
}

hipError_t launch_synth_angles(const SynthArgs& a, hipStream_t stream) {
  const int n = a.n_p * a.n_l;
  if (n <= 0) return hipSuccess;
  if (!a.gl_x || !a.gl_w || !a.pressures || !a.lengths || !a.angles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(synth_angle_kernel, dim3(n), dim3(kLanes), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_synth_select(const SynthArgs& a, const double* targets, int n_t, double tol,
                               double* designs, hipStream_t stream) {
  if (n_t <= 0) return hipSuccess;
  if (!a.angles || !a.pressures || !a.lengths || !targets || !designs || a.n_p <= 0 || a.n_l <= 0)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(synth_select_kernel, dim3((n_t + 255) / 256), dim3(256), 0, stream, a,
                     targets, n_t, tol, designs);
  return hipGetLastError();
}

hipError_t launch_spam_solve(const SynthArgs& a, const double* eps, const double* l0s, int n,
                             double* out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (!a.gl_x || !a.gl_w || !eps || !l0s || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(spam_solve_kernel, dim3(n), dim3(kLanes), 0, stream, a, eps, l0s, n, out);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const double* w, const double* x, int n, double* y,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (!w || !x || !y) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, w, x, n, y);
  return hipGetLastError();
}

}  // namespace vs
