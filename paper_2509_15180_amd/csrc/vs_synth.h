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

}  // namespace vs
