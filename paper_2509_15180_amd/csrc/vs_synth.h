// vs_synth.h -- actuator synthesis (Sec. 4.2): launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace vs {

// One synthesis problem on the device.  Angles are per joint (rad), pressures in Pa,
// lengths in m.
struct SynthArgs {
  const double* gl_x;       // [48] Gauss-Legendre nodes on [-1, 1]
  const double* gl_w;       // [48] and weights (the elliptic integrals of Eq. 1)
  const double* pressures;  // [n_p], rising
  const double* lengths;    // [n_l], rising
  double* angles;           // [n_p][n_l]: rest angle of each (pressure, unit length)
  int n_p, n_l;
  double R_c, R_act, a_corr;           // sPAM constants (Eq. 1)
  double link_len, arm, m_max, eps_c;  // l, 2 R + R_act, pi P_vine R^3, eps_critical
};

// One 64-lane wave per (pressure, unit length).
hipError_t launch_synth_angles(const SynthArgs& a, hipStream_t stream);
// designs[i] = (P, l0, theta) for targets[i], or (0, 0, 0) when no pressure fits
hipError_t launch_synth_select(const SynthArgs& a, const double* targets, int n_t, double tol,
                               double* designs, hipStream_t stream);

// The sPAM state of each strain: out[4 i ..] = (m, phi, G, eps reached); a wave per sample.
hipError_t launch_spam_solve(const SynthArgs& a, const double* eps, const double* l0s, int n,
                             double* out, hipStream_t stream);
// The 2-32-2 ReLU surrogate (weights: W1 [32][2], b1 [32], W2 [2][32], b2 [2]).
hipError_t launch_mlp_forward(const double* w, const double* x, int n, double* y,
                              hipStream_t stream);

}  // namespace vs
