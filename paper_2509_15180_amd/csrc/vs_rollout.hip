// vs_rollout.hip -- gfx950 kernel for the batched quasi-static growth step of the
// vine robot (arXiv 2509.15180, Sec. 3-4).
//
// One wavefront (64 lanes) owns one robot; lanes stride over its links.  All model
// arithmetic is FP64: on gfx950 an FP64 FMA issues at the rate of an unpacked FP32
// FMA, and the equilibrium must be resolved to 1e-10 of the body's moment scale.
//
// A growth step (Alg. 1, read as a converged solve of the energy of Eq. 4):
//   append a link at zero angle; for each growth sub-step (tip length l s/S):
//     repeat
//       poses by wave prefix scans of theta and of the link vectors (Sec. 4.1);
//       joint moments q_j (Eq. 2, Eq. 3) and penetrating disk/obstacle pairs,
//       compacted deterministically with ballots into an LDS contact list;
//       residual r_j = q_j - sum_{contacts on links >= j} lam (x - p_j) x n
//       (suffix scans of per-link force and moment sums);
//       stop when max_j |r_j| / M_max <= tol;
//       (H + mu I) d = -r with the exact Hessian: by default a sequential O(n)
//       Riccati sweep along the chain (a structured solve and a dense LU are
//       cross-checks), mu = c_mu |r|_inf raised tenfold until d descends;
//       cap |d|_inf; Armijo backtracking on the energy.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "vs_device.h"

namespace vs {

constexpr int kMaxC = 128;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// wave primitives (blockDim == 64: one wave per block)

// DPP moves of a double (both halves with the same pattern; lanes whose source is
// out of the row, or whose row is masked off, read 0)
template <int CTRL, int ROWMASK = 0xf, int BANKMASK = 0xf, bool BOUND = true>
__device__ __forceinline__ double dpp(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, BANKMASK, BOUND);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, BANKMASK, BOUND);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_bcast(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// inclusive prefix sum over the 64 lanes: shifts within 16-lane rows, then the row
// broadcasts of lanes 15 and 31 (all lanes must be active)
__device__ __forceinline__ double wscan_incl(double v, int /*lane*/) {
  v += dpp<0x111>(v);                   // row_shr:1
  v += dpp<0x112>(v);                   // row_shr:2
  v += dpp<0x114>(v);                   // row_shr:4
  v += dpp<0x118>(v);                   // row_shr:8
  v += dpp<0x142, 0xa, 0xf, false>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc, 0xf, false>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ double wsum(double v) { return lane_bcast(wscan_incl(v, 0), kWave - 1); }

// inclusive suffix sum: total minus the exclusive prefix
__device__ __forceinline__ double wscan_suffix(double v, int lane) {
  double incl = wscan_incl(v, lane);
  return lane_bcast(incl, kWave - 1) - incl + v;
}

__device__ __forceinline__ double wmax(double v) {  // arguments are >= 0
  v = fmax(v, dpp<0x111>(v));
  v = fmax(v, dpp<0x112>(v));
  v = fmax(v, dpp<0x114>(v));
  v = fmax(v, dpp<0x118>(v));
  v = fmax(v, dpp<0x142, 0xa, 0xf, false>(v));
  v = fmax(v, dpp<0x143, 0xc, 0xf, false>(v));
  return lane_bcast(v, kWave - 1);
}

// argmax of |value| over lanes; ties -> smallest index (value < 0 marks "no row")
__device__ __forceinline__ void wargmax(double& v, int& idx) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    double ov = __shfl_xor(v, o, kWave);
    int oi = __shfl_xor(idx, o, kWave);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// DPP move of a double whose lanes without a source (or in masked-off rows) keep idv
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_or(double v, double idv) {
  int lo = __builtin_amdgcn_update_dpp(__double2loint(idv), __double2loint(v), CTRL, ROWMASK, 0xf,
                                       false);
  int hi = __builtin_amdgcn_update_dpp(__double2hiint(idv), __double2hiint(v), CTRL, ROWMASK, 0xf,
                                       false);
  return __hiloint2double(hi, lo);
}

// Minimum and maximum over each 16-lane row (lanes 16r + 15 hold row r's result; lanes
// outside the chain pass +/-1e300, which never wins)
__device__ __forceinline__ double row_min(double v) {
  v = fmin(v, dpp_or<0x111>(v, 1e300));  // row_shr:1
  v = fmin(v, dpp_or<0x112>(v, 1e300));  // row_shr:2
  v = fmin(v, dpp_or<0x114>(v, 1e300));  // row_shr:4
  v = fmin(v, dpp_or<0x118>(v, 1e300));  // row_shr:8
  return v;
}

__device__ __forceinline__ double row_max(double v) {
  v = fmax(v, dpp_or<0x111>(v, -1e300));
  v = fmax(v, dpp_or<0x112>(v, -1e300));
  v = fmax(v, dpp_or<0x114>(v, -1e300));
  v = fmax(v, dpp_or<0x118>(v, -1e300));
  return v;
}

// Scans of affine maps y -> A y + B over the 64 lanes.  compose(later, earlier) =
// (A_l A_e, A_l B_e + B_l); identity (1, 0).
__device__ __forceinline__ void aff_compose(double& A, double& B, double Ae, double Be) {
  B = fma(A, Be, B);
  A *= Ae;
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ void aff_level(double& A, double& B) {
  const double Ae = dpp_or<CTRL, ROWMASK>(A, 1.0), Be = dpp_or<CTRL, ROWMASK>(B, 0.0);
  aff_compose(A, B, Ae, Be);
}

// lane i: f_i o f_{i-1} o ... o f_0
__device__ __forceinline__ void aff_scan_prefix(double& A, double& B) {
  aff_level<0x111>(A, B);        // row_shr:1
  aff_level<0x112>(A, B);        // row_shr:2
  aff_level<0x114>(A, B);        // row_shr:4
  aff_level<0x118>(A, B);        // row_shr:8
  aff_level<0x142, 0xa>(A, B);   // row_bcast:15 into rows 1 and 3
  aff_level<0x143, 0xc>(A, B);   // row_bcast:31 into rows 2 and 3
}

// lane i: f_i o f_{i+1} o ... o f_63
__device__ __forceinline__ void aff_scan_suffix(double& A, double& B, int lane) {
  aff_level<0x101>(A, B);        // row_shl:1
  aff_level<0x102>(A, B);        // row_shl:2
  aff_level<0x104>(A, B);        // row_shl:4
  aff_level<0x108>(A, B);        // row_shl:8
  {  // rows 0 and 2 take the aggregates of rows 1 and 3 (held by lanes 16 and 48)
    const double A16 = lane_bcast(A, 16), B16 = lane_bcast(B, 16);
    const double A48 = lane_bcast(A, 48), B48 = lane_bcast(B, 48);
    const int row = lane >> 4;
    if (row == 0) aff_compose(A, B, A16, B16);
    if (row == 2) aff_compose(A, B, A48, B48);
  }
  {  // rows 0 and 1 take the aggregate of rows 2-3 (lane 32)
    const double A32 = lane_bcast(A, 32), B32 = lane_bcast(B, 32);
    if (lane < 32) aff_compose(A, B, A32, B32);
  }
}

// 2x2 matrices [a b; c d]; x <- x * e (x is the later factor)
struct M2 {
  double a, b, c, d;
};

__device__ __forceinline__ void m2_mul(M2& x, const M2& e) {
  const double a = fma(x.a, e.a, x.b * e.c), b = fma(x.a, e.b, x.b * e.d);
  const double c = fma(x.c, e.a, x.d * e.c), d = fma(x.c, e.b, x.d * e.d);
  x.a = a;
  x.b = b;
  x.c = c;
  x.d = d;
}

// scale by a power of two so that the largest entry lies in [0.5, 1): only ratios of
// entries are used, and the exponent would otherwise drift over long products
__device__ __forceinline__ void m2_norm(M2& x) {
  const double m = fmax(fmax(fabs(x.a), fabs(x.b)), fmax(fabs(x.c), fabs(x.d)));
  int e = 0;
  if (m > 0.0 && m <= 1.7e308) (void)frexp(m, &e);
  x.a = ldexp(x.a, -e);
  x.b = ldexp(x.b, -e);
  x.c = ldexp(x.c, -e);
  x.d = ldexp(x.d, -e);
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ void m2_level(M2& x) {
  M2 e;
  e.a = dpp_or<CTRL, ROWMASK>(x.a, 1.0);
  e.b = dpp_or<CTRL, ROWMASK>(x.b, 0.0);
  e.c = dpp_or<CTRL, ROWMASK>(x.c, 0.0);
  e.d = dpp_or<CTRL, ROWMASK>(x.d, 1.0);
  m2_mul(x, e);
  m2_norm(x);
}

// lane i: M_i M_{i-1} ... M_0 (up to a positive scale)
__device__ __forceinline__ void m2_scan_prefix(M2& x) {
  m2_level<0x111>(x);
  m2_level<0x112>(x);
  m2_level<0x114>(x);
  m2_level<0x118>(x);
  m2_level<0x142, 0xa>(x);
  m2_level<0x143, 0xc>(x);
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  // splitmix64 finaliser (Steele, Lea, Flood 2014)
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// ---------------------------------------------------------------------------
// model laws


__device__ __forceinline__ double clenshaw(const double* c, int deg, double x) {
  double b1 = 0.0, b2 = 0.0;
  for (int j = deg; j >= 1; --j) {
    double t = fma(2.0 * x, b1, c[j] - b2);
    b2 = b1;
    b1 = t;
  }
  return fma(x, b1, c[0] - b2);
}

// LDS copies of the series that every evaluation sums: G and its integral (not the
// slope, which only the Newton set-up needs) and the integral of the body moment.
// Same member names as SpamTable / WrTable, so the laws below take either.
struct SpamLds {
  static constexpr bool kHasSlope = false;
  double emax, G0;
  double bnd[kSpamPieces + 1], cum[kSpamPieces + 1];
  double c[kSpamPieces][kSpamDeg + 1];
  double ic[kSpamPieces][kSpamDeg + 2];
};

struct WrLds {
  double th_on, du, h_pi, ih_pi;
  double cum[kIhPieces + 1];
  double ic[kIhPieces][kIhDeg + 2];
};

// The wrinkling moment fraction h (Eq. 2a) and its integral from 0 (the energy of the
// body moment per pi P R^3).  Below the onset both are exact (h is linear); above it they
// are piecewise Chebyshev series in u = sqrt(x - theta_on): h itself, and the exact
// antiderivative of a fit of 2 u h(theta_on + u^2), so that the integral's slope in x
// equals h to the fits' accuracy.  Beyond pi, h stays at h(pi).
template <class Tab>
__device__ void wr_law(double x, const Tab& T, const WrTable& Th, bool want_h, bool want_ih,
                       double& h, double& ih) {
  if (x <= T.th_on) {
    h = x / (2.0 * T.th_on);
    ih = x * x / (4.0 * T.th_on);
    return;
  }
  if (x >= kPi) {
    h = T.h_pi;
    ih = T.ih_pi + T.h_pi * (x - kPi);
    return;
  }
  const double u = sqrt(x - T.th_on);
  int k = (int)(u / T.du);
  k = k > kIhPieces - 1 ? kIhPieces - 1 : k;
  const double a = k * T.du;
  const double t = 2.0 * (u - a) / T.du - 1.0;
  if (want_h) h = clenshaw(Th.hc[k], kIhDeg, t);
  if (want_ih) ih = T.cum[k] + 0.5 * T.du * clenshaw(T.ic[k], kIhDeg + 1, t);
}

// Slope dh/dx: 1/(2 theta_on) on the linear branch (also at the onset itself), a series in
// the same u above it (the series was fitted to a long-double closed form, which in double
// loses digits to the arccosine near the onset and to cancellation near pi), 0 from pi on.
__device__ double wr_slope(double x, const WrTable& T) {
  if (x <= T.th_on) return 0.5 / T.th_on;
  if (x >= kPi) return 0.0;
  const double u = sqrt(x - T.th_on);
  int k = (int)(u / T.du);
  k = k > kIhPieces - 1 ? kIhPieces - 1 : k;
  const double a = k * T.du;
  const double t = 2.0 * (u - a) / T.du - 1.0;
  return clenshaw(T.dhc[k], kIhDeg, t);
}

// sPAM force per unit pressure G(eps) (Eq. 1d / P_act), its slope and integral.  A
// table without the slope series gives a NaN slope (never asked for).
template <class Tab>
__device__ void spam_law(const Tab& T, double eps, double* G, double* dG, double* IG) {
  if (eps >= T.emax) {
    if (G) *G = 0.0;
    if (dG) *dG = 0.0;
    if (IG) *IG = T.cum[kSpamPieces];
    return;
  }
  int k = (int)(kSpamPieces * sqrt(eps / T.emax));
  k = k < 0 ? 0 : (k > kSpamPieces - 1 ? kSpamPieces - 1 : k);
  double a = T.bnd[k], b = T.bnd[k + 1];
  double x = (2.0 * eps - a - b) / (b - a);
  if (G) *G = clenshaw(T.c[k], kSpamDeg, x);
  if constexpr (Tab::kHasSlope) {
    if (dG) *dG = clenshaw(T.dc[k], kSpamDeg - 1, x) * 2.0 / (b - a);
  } else {
    if (dG) *dG = __builtin_nan("");
  }
  if (IG) *IG = T.cum[k] + 0.5 * (b - a) * clenshaw(T.ic[k], kSpamDeg + 1, x);
}

struct Ctx {
  int n, K;
  int step, sub;           // for the solver trace
  double* trace;           // non-null only for the traced robot
  int* trace_n;
  int trace_cap;
  double l, R, Mmax, arm, bx, by, bpsi, last_len;
  const SpamTable* tab;
  const WrTable* wr;
  // this robot's obstacles in global memory (copied into LDS, see stage_resident)
  const double* obs;  // [K][4]: cx, cy, a, b
  const int* okind;   // [K]
  KParams P;
};

// joint moment (Eq. 3b with Eq. 2), slope and energy for angle th and coverage pp/pm.
// Only the actuator side the bend stretches needs the force law; the other side sits
// at zero strain, G(0) = G0.
template <class TS, class TW>
__device__ void joint_law(const Ctx& c, const TS& ts, const TW& tw, double th, double pp,
                          double pm, double* q, double* dq, double* E) {
  const double ath = fabs(th);
  const double G0 = ts.G0;
  const double eps = c.arm * ath / c.l;
  double G = G0, dG = 0.0, IG = 0.0;
  if (th != 0.0)
    spam_law(ts, eps, q ? &G : nullptr, dq ? &dG : nullptr, E ? &IG : nullptr);
  else if (dq)
    spam_law(ts, 0.0, nullptr, &dG, nullptr);
  const double pstr = th >= 0.0 ? pp : pm;  // stretched side
  double h = 0.0, ih = 0.0;
  if (q || E) wr_law(ath, tw, *c.wr, q != nullptr, E != nullptr, h, ih);
  if (q) {
    const double Mb = (th >= 0.0 ? 1.0 : -1.0) * c.Mmax * h;
    *q = th >= 0.0 ? Mb - c.arm * (pp * G - pm * G0) : Mb - c.arm * (pp * G0 - pm * G);
  }
  if (dq) {
    const double k = c.arm * c.arm / c.l;
    double d = c.Mmax * wr_slope(ath, *c.wr);
    d -= th != 0.0 ? k * pstr * dG : 0.5 * k * (pp + pm) * dG;
    *dq = d;
  }
  if (E) {
    const double Eb = c.Mmax * ih;
    const double Ea = th >= 0.0 ? (-c.l * pp * IG + c.arm * pm * G0 * th)
                                : (-c.arm * pp * G0 * th - c.l * pm * IG);
    *E = Eb + Ea;
  }
}

// Gap g = dist(x, obstacle) - R of a body disk at (x, y), with outward normal and the
// curvature of the distance field.  Returns false (no contact, outputs unset) when
// the disk is clearly clear of the obstacle; the squared-distance pre-test keeps a
// relative margin so that every pair it rejects also has g >= 0 when evaluated.
__device__ __forceinline__ bool obs_gap(int kind, double ox, double oy, double oa, double ob,
                                        double R, double x, double y, double& g, double& nx,
                                        double& ny, double& kap) {
  if (kind == 0) {
    const double vx = x - ox, vy = y - oy;
    const double d2 = vx * vx + vy * vy, rr = oa + R;
    if (!(d2 < rr * rr * (1.0 + 1e-12))) return false;
    const double d = sqrt(d2);
    if (d > 0.0) {
      const double id = 1.0 / d;
      nx = vx * id;
      ny = vy * id;
      kap = id;
    } else {
      nx = 1.0;
      ny = 0.0;
      kap = 0.0;
    }
    g = (d - oa) - R;
    return g < 0.0;
  }
  const double sx = x >= ox ? 1.0 : -1.0, sy = y >= oy ? 1.0 : -1.0;
  const double dx = fabs(x - ox) - oa, dy = fabs(y - oy) - ob;
  if (dx >= R || dy >= R) return false;
  kap = 0.0;
  if (dx > 0.0 || dy > 0.0) {
    const double ox = fmax(dx, 0.0), oy = fmax(dy, 0.0);
    const double d2 = ox * ox + oy * oy;
    if (!(d2 < R * R * (1.0 + 1e-12))) return false;
    const double d = sqrt(d2), id = 1.0 / d;
    nx = sx * ox * id;
    ny = sy * oy * id;
    if (dx > 0.0 && dy > 0.0) kap = id;
    g = d - R;
    return g < 0.0;
  }
  if (dx >= dy) {
    nx = sx;
    ny = 0.0;
    g = dx - R;
  } else {
    nx = 0.0;
    ny = sy;
    g = dy - R;
  }
  return true;
}

// The pre-tests of obs_gap alone: false only for pairs obs_gap rejects.  Both tests
// are computed and one is selected, so that the wave does not branch on the kind.
__device__ __forceinline__ bool obs_near(int kind, double ox, double oy, double oa, double ob,
                                         double R, double x, double y) {
  const double vx = x - ox, vy = y - oy, rr = oa + R;
  const bool circ = vx * vx + vy * vy < rr * rr * (1.0 + 1e-12);
  const bool box = (int)(fabs(vx) - oa < R) & (int)(fabs(vy) - ob < R);
  return kind == 0 ? circ : box;
}

// ---------------------------------------------------------------------------
// LDS working set of one robot

constexpr int kMaxCL = 16;             // contact links the structured solve holds
constexpr int kMaxCols = 3 * kMaxCL;   // columns of its low-rank term

// FULL_ = false is the layout of the chain-sweep launches (every class when the sweep
// solves the Newton systems): no space for the structured and dense solves, the law
// tables read from global memory, and the trial angles of the line search kept in b
// (free once the step is solved).  That cuts the 256-link robot from 71 to 53 KB (three
// robots per compute unit instead of two) and lets the kernel compile without spills.
template <int NMAX, int WN_ = 1, bool FULL_ = true, bool HELP_ = false>
struct Smem {
  static constexpr int WN = WN_;  // order of the dense cross-check system (64, else unused)
  static constexpr bool kFull = FULL_;
  static constexpr bool kHelper = HELP_;  // a second wave takes each evaluation's obstacle phase
  static constexpr int NS = FULL_ ? kMaxCL : 1, NSC = FULL_ ? kMaxCols : 1;
  struct ResObs {
    double ox[kMaxObs], oy[kMaxObs], oa[kMaxObs], ob[kMaxObs];
    int okind[kMaxObs];
  };
  struct ResFull : ResObs {
    SpamLds sp;
    WrLds wr;
  };
  union {
    double W[WN][WN + 1];                           // (H + mu I | -r), LU in place
    struct {
      double G[NSC][kMaxCols + 1];  // U^T T^-1 U, then (I + S G | S c) and its LU in place
    } sm;
    double F[FULL_ ? kWave : 1][17];  // one chunk of forward-substituted columns (Gram by MFMA)
    std::conditional_t<FULL_, ResFull, ResObs> res;  // the robot's obstacles (and law tables)
                                                     // while no solve holds this space
  };
  int res_ok;  // res holds this robot's data
  double th[NMAX], tt[FULL_ ? NMAX : 1], d[NMAX], r[NMAX];
  double px[NMAX + 1], py[NMAX + 1], tx[NMAX], ty[NMAX];
  double pp[NMAX], pm[NMAX];
  // Newton set-up and solves
  double dq[NMAX];     // joint stiffness q'_j
  double cg[NMAX];     // geometric stiffness, diagonal in absolute angles
  double dinv[NMAX];   // 1 / pivots of the tridiagonal part
  double ell[NMAX];    // its unit lower multipliers
  double z[NMAX], v[NMAX], aux[NMAX], b[NMAX];
  double ps1[NMAX], ps2[NMAX];
  int lidx[NMAX];      // link -> contact-link slot (or -1)
  int clink[NS];       // contact-link slot -> link
  double cM[NS][6];    // 3x3 contact block per contact link (symmetric: 00 01 02 11 12 22)
  double cvec[NSC], wvec[NSC];
  double gcarry[FULL_ ? 16 : 1];  // forward-substitution carries between row chunks (Gram pass)
  int ncl_links;
  int ci[kMaxC], ck[kMaxC];
  double cl[kMaxC], cxx[kMaxC], cxy[kMaxC], cnx[kMaxC], cny[kMaxC], ckap[kMaxC], cpen[kMaxC];
  int ncl;
  int overflow;
  double jevals, nsolves;  // work counters (lane 0 updates)
  int cmd, cmd_seq, eval_n;  // solver wave -> helper wave: 1 = obstacle phase, 2 = end
  double eval_last;
};

// Barrier of the solver's own wave.  A wave's LDS operations complete in the order it
// issues them, so ordering the accesses of its lanes needs only a compiler fence.  In the
// two-wave launches the solver wave meets its helper wave only at the barriers of
// evaluate() and at its end, so every other barrier must be this one.
template <class SM>
__device__ __forceinline__ void bsync() {
  if constexpr (SM::kHelper) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Copy the robot's obstacles (structure of arrays) and the series of its law tables
// into LDS.  The space is shared with the structured and dense solves, which clear
// res_ok; evaluate() copies again then.
template <class SM>
__device__ void stage_resident(SM& S, const Ctx& c) {
  const int lane = threadIdx.x;
  for (int k = lane; k < c.K; k += kWave) {
    S.res.ox[k] = c.obs[4 * (size_t)k];
    S.res.oy[k] = c.obs[4 * (size_t)k + 1];
    S.res.oa[k] = c.obs[4 * (size_t)k + 2];
    S.res.ob[k] = c.obs[4 * (size_t)k + 3];
    S.res.okind[k] = c.okind[k];
  }
  if constexpr (SM::kFull) {
  static_assert(sizeof(S.res) <= sizeof(S.sm), "resident data must fit the solve space");
  const SpamTable& T = *c.tab;
  for (int i = lane; i < kSpamPieces * (kSpamDeg + 1); i += kWave)
    (&S.res.sp.c[0][0])[i] = (&T.c[0][0])[i];
  for (int i = lane; i < kSpamPieces * (kSpamDeg + 2); i += kWave)
    (&S.res.sp.ic[0][0])[i] = (&T.ic[0][0])[i];
  for (int i = lane; i <= kSpamPieces; i += kWave) {
    S.res.sp.bnd[i] = T.bnd[i];
    S.res.sp.cum[i] = T.cum[i];
  }
  const WrTable& W = *c.wr;
  for (int i = lane; i < kIhPieces * (kIhDeg + 2); i += kWave)
    (&S.res.wr.ic[0][0])[i] = (&W.ic[0][0])[i];
  for (int i = lane; i <= kIhPieces; i += kWave) S.res.wr.cum[i] = W.cum[i];
  if (lane == 0) {
    S.res.sp.emax = T.emax;
    S.res.sp.G0 = T.G0;
    S.res.wr.th_on = W.th_on;
    S.res.wr.du = W.du;
    S.res.wr.h_pi = W.h_pi;
    S.res.wr.ih_pi = W.ih_pi;
  }
  }
  if (lane == 0) S.res_ok = 1;
  bsync<SM>();
}

// The contact part of an evaluation at the poses in S (n links, the last of length
// last_len), on one wave whose lane index is lane: penetrating (disk, obstacle) pairs
// into the contact list, each link's contact sums into ps1, ps2, aux and v, and ncl and
// overflow.
template <class SM>
__device__ void obstacle_phase(SM& S, const Ctx& c, int n, double last_len, int lane) {
  // penetrating (disk, obstacle) pairs, compacted in (obstacle, disk, link) order per
  // chunk.  The exact gap (square root, divisions) is taken only for pairs whose
  // cheap pre-test some lane of the wave passes.
  int cnt = 0;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int base = 0; base < n; base += kWave) {
    const int j = base + lane;
    const bool on = j < n;
    const double L = (j == n - 1) ? last_len : c.l;
    const double pxj = on ? S.px[j] : 0.0, pyj = on ? S.py[j] : 0.0;
    const double txj = on ? S.tx[j] : 0.0, tyj = on ? S.ty[j] : 0.0;
    double xs[2], ys[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const double s = 0.5 * (hh + 1) * L;
      xs[hh] = pxj + s * txj;
      ys[hh] = pyj + s * tyj;
    }
    // this link's contact sums, in the order the contacts are listed: moment and force
    // (residual), and the force's moment along the link (geometric stiffness)
    double a_s1 = 0.0, a_fx = 0.0, a_fy = 0.0, a_q = 0.0;
    // Broad phase: the bounding box of each 16-lane row's disk centres, and per obstacle
    // whether its box widened by the tube radius (and a relative 1e-9) meets any row's
    // box.  An obstacle that meets none fails the pair pre-test for every disk of the
    // chunk, so the rounds below visit only the others, in index order (the contact list
    // keeps the order of a full sweep).
    unsigned long long cand0 = 0ull, cand1 = 0ull;
    {
      const double bx0 = row_min(on ? fmin(xs[0], xs[1]) : 1e300);
      const double bx1 = row_max(on ? fmax(xs[0], xs[1]) : -1e300);
      const double by0 = row_min(on ? fmin(ys[0], ys[1]) : 1e300);
      const double by1 = row_max(on ? fmax(ys[0], ys[1]) : -1e300);
      double rx0[4], rx1[4], ry0[4], ry1[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rx0[r] = lane_bcast(bx0, 16 * r + 15);
        rx1[r] = lane_bcast(bx1, 16 * r + 15);
        ry0[r] = lane_bcast(by0, 16 * r + 15);
        ry1[r] = lane_bcast(by1, 16 * r + 15);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = lane + kWave * q;
        bool meets = false;
        if (k < c.K) {
          const double cx = S.res.ox[k], cy = S.res.oy[k], oa = S.res.oa[k];
          const double ob = S.res.okind[k] == 0 ? oa : S.res.ob[k];
          const double ex = (oa + c.R) * (1.0 + 1e-9), ey = (ob + c.R) * (1.0 + 1e-9);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            meets = meets || ((cx + ex >= rx0[r]) && (cx - ex <= rx1[r]) &&
                              (cy + ey >= ry0[r]) && (cy - ey <= ry1[r]));
        }
        const unsigned long long m = __ballot(meets);
        if (q == 0) cand0 = m; else cand1 = m;
      }
    }
    while (cand0 | cand1) {
      // the next four candidates (repeating the last one when fewer are left)
      int ks[4], nk = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (cand0) {
          ks[u] = __builtin_ctzll(cand0);
          cand0 &= cand0 - 1ull;
          ++nk;
        } else if (cand1) {
          ks[u] = kWave + __builtin_ctzll(cand1);
          cand1 &= cand1 - 1ull;
          ++nk;
        } else {
          ks[u] = ks[u > 0 ? u - 1 : 0];
        }
      }
      // four obstacles per round, read from LDS at addresses the whole wave shares
      // (broadcast reads), issued together
      double ox[4], oy[4], oa[4], ob[4];
      int kd[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = ks[u];
        ox[u] = S.res.ox[k];
        oy[u] = S.res.oy[k];
        oa[u] = S.res.oa[k];
        ob[u] = S.res.ob[k];
        kd[u] = S.res.okind[k];
      }
      unsigned near = 0u;  // bit 2u + hh: disk hh may touch obstacle ks[u]
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
          near |= (unsigned)obs_near(kd[u], ox[u], oy[u], oa[u], ob[u], c.R, xs[hh], ys[hh])
                  << (2 * u + hh);
      near &= on ? (1u << (2 * nk)) - 1u : 0u;
      if (__ballot(near != 0u) == 0ull) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const bool nr = (near >> (2 * u + hh)) & 1u;
          if (__ballot(nr) == 0ull) continue;
          double g = 0.0, nx = 0.0, ny = 0.0, kap = 0.0;
          const bool hit =
              nr && obs_gap(kd[u], ox[u], oy[u], oa[u], ob[u], c.R, xs[hh], ys[hh], g, nx, ny, kap);
          const unsigned long long m = __ballot(hit);
          if (m) {
            const int pos = cnt + __popcll(m & lt);
            if (hit && pos < kMaxC) {
              const double pen = -g, lam = c.P.kc * pen;
              S.ci[pos] = j;
              S.ck[pos] = ks[u];
              S.cl[pos] = lam;
              S.cxx[pos] = xs[hh];
              S.cxy[pos] = ys[hh];
              S.cnx[pos] = nx;
              S.cny[pos] = ny;
              S.ckap[pos] = kap;
              S.cpen[pos] = pen;
              a_s1 += lam * (xs[hh] * ny - ys[hh] * nx);
              a_fx += lam * nx;
              a_fy += lam * ny;
              const double sd = (xs[hh] - pxj) * txj + (ys[hh] - pyj) * tyj;
              a_q += lam * sd * (nx * txj + ny * tyj);
            }
            cnt += __popcll(m);
          }
        }
      }
    }
    if (on) {  // read by the suffix sums below and by structured_setup
      S.ps1[j] = a_s1;
      S.ps2[j] = a_fx;
      S.aux[j] = a_fy;
      S.v[j] = a_q;
    }
  }
  const int nc = cnt < kMaxC ? cnt : kMaxC;
  if (lane == 0) {
    S.ncl = nc;
    S.overflow = cnt > kMaxC;
  }
}

// Poses, joint moments, contacts, residual (into S.r) and energy at angles th.
template <class SM>
__device__ double evaluate(SM& S, const Ctx& c, const double* th, bool want_E) {
  const int lane = threadIdx.x;
  const int n = c.n;
  if (__builtin_amdgcn_readfirstlane(S.res_ok) == 0) stage_resident(S, c);
  if (lane == 0) S.jevals += n;
  double cphi = c.bpsi, cx = c.bx, cy = c.by;
  for (int base = 0; base < n; base += kWave) {
    int j = base + lane;
    bool on = j < n;
    double phi = wscan_incl(on ? th[j] : 0.0, lane) + cphi;
    double sj, cj;
    sincos(phi, &sj, &cj);
    double L = (j == n - 1) ? c.last_len : c.l;
    double ex = on ? L * cj : 0.0, ey = on ? L * sj : 0.0;
    double sx = wscan_incl(ex, lane) + cx, sy = wscan_incl(ey, lane) + cy;
    if (on) {
      S.tx[j] = cj;
      S.ty[j] = sj;
      S.px[j + 1] = sx;
      S.py[j + 1] = sy;
    }
    cphi = __shfl(phi, kWave - 1, kWave);
    cx = __shfl(sx, kWave - 1, kWave);
    cy = __shfl(sy, kWave - 1, kWave);
  }
  if (lane == 0) {
    S.px[0] = c.bx;
    S.py[0] = c.by;
  }
  if constexpr (SM::kHelper) {
    if (lane == 0) {
      S.eval_n = n;
      S.eval_last = c.last_len;
      S.cmd = 1;
      S.cmd_seq += 1;
    }
    __syncthreads();  // the poses are in LDS: the helper wave starts the obstacle phase
  } else {
    bsync<SM>();
  }
  double Esum = 0.0;
  for (int j = lane; j < n; j += kWave) {
    double q, E = 0.0;
    if constexpr (SM::kFull) {
      joint_law(c, S.res.sp, S.res.wr, th[j], S.pp[j], S.pm[j], &q, nullptr, want_E ? &E : nullptr);
    } else if constexpr (SM::kHelper) {
      // the joint slopes too, while the helper wave is busy with the contacts: the Newton
      // set-up that follows an evaluation is always at the angles last evaluated
      double dqj;
      joint_law(c, *c.tab, *c.wr, th[j], S.pp[j], S.pm[j], &q, &dqj, want_E ? &E : nullptr);
      S.dq[j] = dqj;
    } else {
      joint_law(c, *c.tab, *c.wr, th[j], S.pp[j], S.pm[j], &q, nullptr, want_E ? &E : nullptr);
    }
    S.r[j] = q;
    Esum += E;
  }
  if constexpr (SM::kHelper) {
    __syncthreads();  // the helper wave's contacts and contact sums are in LDS
  } else {
    obstacle_phase(S, c, n, c.last_len, lane);
    bsync<SM>();
  }
  const int nc = S.ncl;
  // per-link force and moment sums, then suffix sums from the tip toward the base
  double c1 = 0.0, c2x = 0.0, c2y = 0.0;
  int nchunk = (n + kWave - 1) / kWave;
  for (int ch = nchunk - 1; ch >= 0; --ch) {
    int j = ch * kWave + lane;
    double s1 = j < n ? S.ps1[j] : 0.0, s2x = j < n ? S.ps2[j] : 0.0;
    double s2y = j < n ? S.aux[j] : 0.0;
    s1 = wscan_suffix(s1, lane) + c1;
    s2x = wscan_suffix(s2x, lane) + c2x;
    s2y = wscan_suffix(s2y, lane) + c2y;
    if (j < n) S.r[j] -= s1 - (S.px[j] * s2y - S.py[j] * s2x);
    c1 = __shfl(s1, 0, kWave);
    c2x = __shfl(s2x, 0, kWave);
    c2y = __shfl(s2y, 0, kWave);
  }
  double pen2 = 0.0;
  for (int e = lane; e < nc; e += kWave) pen2 += 0.5 * c.P.kc * S.cpen[e] * S.cpen[e];
  bsync<SM>();
  return wsum(Esum) + wsum(pen2);
}

// W = (H + mu I | -r) at the state last evaluated (poses, contacts and r in S)
template <class SM>
__device__ void assemble(SM& S, const Ctx& c, const double* th, double mu,
                         const double* rhs) {
  const int lane = threadIdx.x, n = c.n;
  if (lane == 0) S.res_ok = 0;  // W overwrites the resident data
  for (int j = lane; j < n; j += kWave) {
    for (int m = 0; m < n; ++m) S.W[j][m] = 0.0;
    double dq;
    joint_law(c, *c.tab, *c.wr, th[j], S.pp[j], S.pm[j], nullptr, &dq, nullptr);
    S.W[j][j] = dq + mu;
    S.W[j][n] = rhs[j];
  }
  __syncthreads();
  const int nc = S.ncl;
  for (int e = 0; e < nc; ++e) {
    const int i = S.ci[e];
    const double lam = S.cl[e], xx = S.cxx[e], xy = S.cxy[e], nx = S.cnx[e], ny = S.cny[e];
    const double lk = lam * S.ckap[e], kc = c.P.kc;
    const double nxx = nx * xx + ny * xy;
    for (int j = lane; j <= i; j += kWave) {
      double vx = -(xy - S.py[j]), vy = xx - S.px[j];
      double aj = nx * vx + ny * vy, bj = -ny * vx + nx * vy, uj = nx * S.px[j] + ny * S.py[j];
      for (int m = 0; m <= i; ++m) {
        double wx = -(xy - S.py[m]), wy = xx - S.px[m];
        double am = nx * wx + ny * wy, bm = -ny * wx + nx * wy;
        double umax = (j > m) ? uj : (nx * S.px[m] + ny * S.py[m]);
        S.W[j][m] += kc * aj * am - lk * bj * bm + lam * (nxx - umax);
      }
    }
    __syncthreads();
  }
}

// LU with partial pivoting of the n x n system stored row-major in A (row stride ld,
// right-hand side in column n); solution into x.  false on a zero pivot or a
// non-finite solution.
__device__ bool lu_solve(double* A, int ld, int n, double* x) {
  const int lane = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + lane; i < n; i += kWave) {
      double v = fabs(A[i * ld + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    wargmax(best, bi);
    if (!(best > 0.0)) return false;
    if (bi != k) {
      for (int j = k + lane; j <= n; j += kWave) {
        double t = A[k * ld + j];
        A[k * ld + j] = A[bi * ld + j];
        A[bi * ld + j] = t;
      }
      __syncthreads();
    }
    const double piv = A[k * ld + k];
    for (int i = k + 1 + lane; i < n; i += kWave) {
      double f = A[i * ld + k] / piv;
      if (f != 0.0)
        for (int j = k; j <= n; ++j) A[i * ld + j] -= f * A[k * ld + j];
    }
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    double xi = A[i * ld + n] / A[i * ld + i];
    for (int j = lane; j < i; j += kWave) A[j * ld + n] -= A[j * ld + i] * xi;
    if (lane == 0) x[i] = xi;
    __syncthreads();
  }
  bool ok = true;
  for (int j = lane; j < n; j += kWave) ok = ok && isfinite(x[j]);
  return __all(ok);
}

template <class SM>
__device__ bool lu_solve_dense(SM& S, int n) {
  return lu_solve(&S.W[0][0], SM::WN + 1, n, S.d);
}

// Per-iteration set-up of the structured solve (independent of mu): joint slopes,
// the contact links, their 3x3 blocks, and the geometric diagonal.
//
// In absolute angles phi = L theta (L: lower-triangular ones), the exact Hessian is
//   H_phi = L^-T diag(q') L^-1 + diag(C) + sum_{contact links i} U_i M_i U_i^T,
// with U_i = [X_i, Y_i, e_i], X_i = (l cos phi_m)_{m<i}, Y_i = (l sin phi_m)_{m<i},
//   C_m = l t_m . (sum of contact forces on links beyond m) + sum_{disks on m} lam s n.t_m,
//   M_i = sum_{disks on i} k_c alpha alpha^T - lam kappa beta beta^T,
//   alpha = (n_y, -n_x, s t_i x n), beta = (n_x, n_y, s t_i . n),
// s the disk's distance from the link's proximal joint.  C takes the per-link contact
// sums that evaluate() leaves in S.ps2, S.aux and S.v, so this must follow the
// evaluation of the same state.  Returns false when more than kMaxCL links are in
// contact, and (after the slopes, the contact-link flags in lidx and C, all that the
// chain sweep needs) when blocks is false.
template <class SM>
__device__ bool structured_setup(SM& S, const Ctx& c, bool blocks = true) {
  const int lane = threadIdx.x, n = c.n, nc = S.ncl;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int j = lane; j < n; j += kWave) {
    if constexpr (!SM::kHelper) {  // two-wave launches: evaluate() left them in dq
      double d;
      joint_law(c, *c.tab, *c.wr, S.th[j], S.pp[j], S.pm[j], nullptr, &d, nullptr);
      S.dq[j] = d;
    }
    S.lidx[j] = -1;
  }
  bsync<SM>();
  for (int e = lane; e < nc; e += kWave) S.lidx[S.ci[e]] = 0;
  bsync<SM>();
  int L = 0;
  for (int base = 0; base < n && blocks && SM::kFull; base += kWave) {
    int j = base + lane;
    bool f = j < n && S.lidx[j] == 0;
    unsigned long long m = __ballot(f);
    if (f) {
      int pos = L + __popcll(m & lt);
      S.lidx[j] = pos < kMaxCL ? pos : kMaxCL;
      if (pos < kMaxCL) S.clink[pos] = j;
    }
    L += __popcll(m);
  }
  if (lane == 0) S.ncl_links = L;
  bsync<SM>();
  // geometric diagonal: suffix sums of per-link forces, chunks from the tip down
  double cfx = 0.0, cfy = 0.0;
  const int nchunk = (n + kWave - 1) / kWave;
  for (int ch = nchunk - 1; ch >= 0; --ch) {
    const int j = ch * kWave + lane;
    // per-link contact force and its moment along the link, summed by evaluate()
    const double fx = j < n ? S.ps2[j] : 0.0, fy = j < n ? S.aux[j] : 0.0;
    const double q = j < n ? S.v[j] : 0.0;
    double sx = wscan_suffix(fx, lane) + cfx, sy = wscan_suffix(fy, lane) + cfy;
    if (j < n) S.cg[j] = c.l * (S.tx[j] * (sx - fx) + S.ty[j] * (sy - fy)) + q;
    cfx = __shfl(sx, 0, kWave);
    cfy = __shfl(sy, 0, kWave);
  }
  bsync<SM>();
  if (!SM::kFull || !blocks || L > kMaxCL) return false;
  // 3x3 blocks, one lane per contact link (contacts visited in list order)
  for (int a = lane; a < L; a += kWave) {
    const int i = S.clink[a];
    const double ti_x = S.tx[i], ti_y = S.ty[i];
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0;
    for (int e = 0; e < nc; ++e) {
      if (S.ci[e] != i) continue;
      const double nx = S.cnx[e], ny = S.cny[e], lam = S.cl[e], lk = lam * S.ckap[e];
      const double s = (S.cxx[e] - S.px[i]) * ti_x + (S.cxy[e] - S.py[i]) * ti_y;
      const double a0 = ny, a1 = -nx, a2 = s * (ti_x * ny - ti_y * nx);
      const double b0 = nx, b1 = ny, b2 = s * (ti_x * nx + ti_y * ny);
      const double kc = c.P.kc;
      m0 += kc * a0 * a0 - lk * b0 * b0;
      m1 += kc * a0 * a1 - lk * b0 * b1;
      m2 += kc * a0 * a2 - lk * b0 * b2;
      m3 += kc * a1 * a1 - lk * b1 * b1;
      m4 += kc * a1 * a2 - lk * b1 * b2;
      m5 += kc * a2 * a2 - lk * b2 * b2;
    }
    S.cM[a][0] = m0;
    S.cM[a][1] = m1;
    S.cM[a][2] = m2;
    S.cM[a][3] = m3;
    S.cM[a][4] = m4;
    S.cM[a][5] = m5;
  }
  bsync<SM>();
  return true;
}

// ---------------------------------------------------------------------------
// Tridiagonal part by wave scans.  T_mm = t_m = k_m + k_{m+1} + C_m and
// T_{m-1,m} = e_m = -k_m, k_j = q'_j + mu (k_n = 0).  The LDL^T pivots
// D_m = t_m - e_m^2 / D_{m-1} are ratios p_m / p_{m-1} of leading principal minors,
// which obey p_m = t_m p_{m-1} - e_m^2 p_{m-2}: a prefix product of the 2x2 matrices
// [t_m, -e_m^2; 1, 0] (first column of the product = (p_m, p_{m-1})).  The
// substitutions y_m = b_m - l_{m-1} y_{m-1} and x_m = y_m / D_m - l_m x_{m+1},
// l_m = T_{m,m+1} / D_m, are affine recurrences: prefix and suffix scans of affine
// maps.  Rows go 64 to a chunk; chunks are chained through the scan carries.
// Returns false on a vanishing or non-finite pivot (the caller raises mu).
template <class SM>
__device__ bool tri_factor(SM& S, int n, double mu) {
  const int lane = threadIdx.x;
  M2 carry{1.0, 0.0, 0.0, 1.0};
  bool ok = true;
  for (int base = 0; base < n; base += kWave) {
    const int m = base + lane;
    const bool on = m < n;
    double km = 0.0, kn = 0.0, cm = 0.0;
    if (on) {
      km = S.dq[m] + mu;
      kn = m + 1 < n ? S.dq[m + 1] + mu : 0.0;
      cm = S.cg[m];
    }
    const double t = km + kn + cm;
    const double e = m >= 1 ? -km : 0.0;
    M2 x = on ? M2{t, -e * e, 1.0, 0.0} : M2{1.0, 0.0, 0.0, 1.0};
    m2_scan_prefix(x);
    if (base > 0) {
      m2_mul(x, carry);
      m2_norm(x);
    }
    if (on) {
      const double D = x.a / x.c;
      ok = ok && isfinite(D) && fabs(D) > 1e-14 * (fabs(t) + fabs(e));
      const double di = 1.0 / D;
      S.dinv[m] = di;
      S.ell[m] = m + 1 < n ? -kn * di : 0.0;
    }
    carry = M2{lane_bcast(x.a, kWave - 1), lane_bcast(x.b, kWave - 1), lane_bcast(x.c, kWave - 1),
               lane_bcast(x.d, kWave - 1)};
  }
  __syncthreads();
  return __all(ok);
}

// Forward substitution y = L^-1 b into dst (b and dst in LDS; dst may be b)
template <class SM>
__device__ void tri_fwd(SM& S, int n, const double* b, double* dst) {
  const int lane = threadIdx.x;
  double carry = 0.0;
  for (int base = 0; base < n; base += kWave) {
    const int m = base + lane;
    double A = 1.0, B = 0.0;
    if (m < n) {
      A = m > 0 ? -S.ell[m - 1] : 0.0;
      B = b[m];
    }
    aff_scan_prefix(A, B);
    const double y = fma(A, carry, B);
    if (m < n) dst[m] = y;
    carry = lane_bcast(y, kWave - 1);
  }
}

// Back substitution x = D^-1 y - L^T-part, in place on y
template <class SM>
__device__ void tri_bwd(SM& S, int n, double* y) {
  const int lane = threadIdx.x;
  double carry = 0.0;
  for (int base = (n - 1) / kWave * kWave; base >= 0; base -= kWave) {
    const int m = base + lane;
    double A = 1.0, B = 0.0;
    if (m < n) {
      A = -S.ell[m];
      B = y[m] * S.dinv[m];
    }
    aff_scan_suffix(A, B, lane);
    const double x = fma(A, carry, B);
    if (m < n) y[m] = x;
    carry = lane_bcast(x, 0);
  }
  __syncthreads();
}

// T x = b with the factors in S.dinv / S.ell (b and dst in LDS; dst may be b)
template <class SM>
__device__ void tri_solve(SM& S, int n, const double* b, double* dst) {
  tri_fwd(S, n, b, dst);
  tri_bwd(S, n, dst);
}

// value of low-rank column b (contact-link slot b/3; kinds X, Y, e) at row m
template <class SM>
__device__ __forceinline__ double ucol(const SM& S, double l, int b, int m) {
  const int i = S.clink[b / 3], k = b % 3;
  if (k == 2) return m == i ? 1.0 : 0.0;
  if (m >= i) return 0.0;
  return l * (k == 0 ? S.tx[m] : S.ty[m]);
}

// one level of a prefix scan of the affine maps (A, B_b), the same A for every column
template <int CTRL, int ROWMASK, int NB>
__device__ __forceinline__ void aff_level_multi(double& A, double (&B)[NB], unsigned act) {
  const double Ae = dpp_or<CTRL, ROWMASK>(A, 1.0);
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (act & (1u << i)) B[i] = fma(A, dpp_or<CTRL, ROWMASK>(B[i], 0.0), B[i]);
  A *= Ae;
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Gram matrix of the contact columns by FP64 MFMA (ncol <= 15).  With T = L D L^T,
//   G = U^T T^-1 U = F^T D^-1 F and c = U^T T^-1 v = F^T D^-1 y,
// F = L^-1 U and y = L^-1 v: forward substitutions only, eight columns per pass of
// scans (the recurrence coefficients are shared).  Per chunk of 64 rows the columns
// [F | y] (16 wide, y last) go through LDS into 16 v_mfma_f64_16x16x4 steps that
// accumulate [F | y]^T D^-1 [F | y].  y is also left in S.z for the back substitution.
template <class SM>
__device__ void gram_mfma(SM& S, const Ctx& c, int ncol) {
  constexpr int NC = 16, NB = 8;  // columns 0..ncol-1: U; column NC-1: v
  const int lane = threadIdx.x, n = c.n;
  if (lane < NC) S.gcarry[lane] = 0.0;
  __syncthreads();
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int base = 0; base < n; base += kWave) {
    const int m = base + lane;
    const bool on = m < n;
    const double A0 = on ? (m > 0 ? -S.ell[m - 1] : 0.0) : 1.0;
    for (int half = 0; half < NC / NB; ++half) {
      unsigned act = 0u;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int b = NB * half + i;
        if (b < ncol || b == NC - 1) act |= 1u << i;
      }
      if (act == 0u) continue;
      double A = A0, B[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int b = NB * half + i;
        B[i] = (on && (act & (1u << i))) ? (b == NC - 1 ? S.v[m] : ucol(S, c.l, b, m)) : 0.0;
      }
      aff_level_multi<0x111, 0xf>(A, B, act);  // row_shr:1
      aff_level_multi<0x112, 0xf>(A, B, act);  // row_shr:2
      aff_level_multi<0x114, 0xf>(A, B, act);  // row_shr:4
      aff_level_multi<0x118, 0xf>(A, B, act);  // row_shr:8
      aff_level_multi<0x142, 0xa>(A, B, act);  // row_bcast:15
      aff_level_multi<0x143, 0xc>(A, B, act);  // row_bcast:31
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (!(act & (1u << i))) continue;
        const int b = NB * half + i;
        const double y = on ? fma(A, S.gcarry[b], B[i]) : 0.0;
        S.F[lane][b] = y;
        if (b == NC - 1 && on) S.z[m] = y;
        if (lane == kWave - 1) S.gcarry[b] = y;
      }
    }
    __syncthreads();
    // lane l carries row 4 kb + l / 16, column l % 16 of both operands
    const int rsub = lane >> 4, col = lane & 15;
#pragma unroll 4
    for (int kb = 0; kb < kWave / 4; ++kb) {
      const int r = 4 * kb + rsub;
      const double a = S.F[r][col];
      const double di = base + r < n ? S.dinv[base + r] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a * di, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // lane l, register v holds entry (l / 16 + 4 v, l % 16)
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = (lane >> 4) + 4 * v, col = lane & 15;
    if (row < ncol) {
      if (col < ncol) S.sm.G[row][col] = acc[v];
      else if (col == NC - 1) S.cvec[row] = acc[v];
    }
  }
  __syncthreads();
}

// out[(3a + k) * stride] = (U^T y)_{3a+k}: exclusive prefix sums of l cos(phi) y and
// l sin(phi) y at contact link i_a, and y_{i_a}
template <class SM>
__device__ void ut_times(SM& S, const Ctx& c, const double* y, double* out, int stride) {
  const int lane = threadIdx.x, n = c.n, L = S.ncl_links;
  double c1 = 0.0, c2 = 0.0;
  for (int base = 0; base < n; base += kWave) {
    const int m = base + lane;
    const double a = m < n ? c.l * S.tx[m] * y[m] : 0.0;
    const double b = m < n ? c.l * S.ty[m] * y[m] : 0.0;
    const double ia = wscan_incl(a, lane) + c1, ib = wscan_incl(b, lane) + c2;
    if (m < n) {
      S.ps1[m] = ia - a;
      S.ps2[m] = ib - b;
    }
    c1 = lane_bcast(ia, kWave - 1);
    c2 = lane_bcast(ib, kWave - 1);
  }
  __syncthreads();
  for (int a = lane; a < L; a += kWave) {
    const int i = S.clink[a];
    out[(3 * a + 0) * stride] = S.ps1[i];
    out[(3 * a + 1) * stride] = S.ps2[i];
    out[(3 * a + 2) * stride] = y[i];
  }
  __syncthreads();
}

// K = I + S G with S = blockdiag(M_a), in place in S.sm.G: the three rows of a block
// depend on the same three rows of G only; the right-hand side S c goes to column ncol.
template <class SM>
__device__ void capacitance_matrix(SM& S, int L) {
  const int ncol = 3 * L;
  for (int blk = threadIdx.x; blk < L; blk += kWave) {
    const double* M = S.cM[blk];
    double* g0 = S.sm.G[3 * blk];
    double* g1 = S.sm.G[3 * blk + 1];
    double* g2 = S.sm.G[3 * blk + 2];
    const int r0 = 3 * blk;
    for (int col = 0; col <= ncol; ++col) {
      const double a0 = col < ncol ? g0[col] : S.cvec[r0];
      const double a1 = col < ncol ? g1[col] : S.cvec[r0 + 1];
      const double a2 = col < ncol ? g2[col] : S.cvec[r0 + 2];
      g0[col] = (col == r0 ? 1.0 : 0.0) + M[0] * a0 + M[1] * a1 + M[2] * a2;
      g1[col] = (col == r0 + 1 ? 1.0 : 0.0) + M[1] * a0 + M[3] * a1 + M[4] * a2;
      g2[col] = (col == r0 + 2 ? 1.0 : 0.0) + M[2] * a0 + M[4] * a1 + M[5] * a2;
    }
  }
  __syncthreads();
}

// (I + S G) w = S c for one or two contact links (order NC = 3 or 6), the common case:
// every lane assembles and eliminates the whole system in registers (Gaussian
// elimination with partial pivoting, fully unrolled), so no lane waits on another.
template <int NC, class SM>
__device__ bool tiny_solve(SM& S) {
  double K[NC][NC + 1];
#pragma unroll
  for (int b = 0; b < NC / 3; ++b) {
    const double* M = S.cM[b];
    const double m[3][3] = {{M[0], M[1], M[2]}, {M[1], M[3], M[4]}, {M[2], M[4], M[5]}};
#pragma unroll
    for (int r3 = 0; r3 < 3; ++r3) {
      const int r = 3 * b + r3;
#pragma unroll
      for (int col = 0; col <= NC; ++col) {
        double v = col == r ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          v += m[r3][k] * (col < NC ? S.sm.G[3 * b + k][col] : S.cvec[3 * b + k]);
        K[r][col] = col < NC ? v : v - (col == r ? 1.0 : 0.0);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    int p = k;
    double best = fabs(K[k][k]);
#pragma unroll
    for (int i = k + 1; i < NC; ++i) {
      const double v = fabs(K[i][k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!(best > 0.0)) return false;
#pragma unroll
    for (int i = k + 1; i < NC; ++i) {
      if (p != i) continue;
#pragma unroll
      for (int j = k; j <= NC; ++j) {
        const double t = K[k][j];
        K[k][j] = K[i][j];
        K[i][j] = t;
      }
    }
    const double inv = 1.0 / K[k][k];
#pragma unroll
    for (int i = k + 1; i < NC; ++i) {
      const double f = K[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j <= NC; ++j) K[i][j] = fma(-f, K[k][j], K[i][j]);
    }
  }
  double x[NC];
  bool fin = true;
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    double sum = K[i][NC];
#pragma unroll
    for (int j = i + 1; j < NC; ++j) sum = fma(-K[i][j], x[j], sum);
    x[i] = sum / K[i][i];
    fin = fin && isfinite(x[i]);
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NC; ++i) S.wvec[i] = x[i];
  __syncthreads();
  return fin;
}

// (K | S c) w for ncol <= 15, one row per lane: Gauss-Jordan with partial pivoting
// over the rows not yet used as pivots.  Rows stay in LDS between pivot steps; a step
// loads the lane's row and the pivot row whole, so its loads issue together.
template <class SM>
__device__ bool small_solve(SM& S, int ncol) {
  constexpr int NC = 16;  // row length bound (ncol + 1 <= NC)
  const int lane = threadIdx.x;
  const bool row = lane < ncol;
  double* Kr = S.sm.G[row ? lane : 0];
  bool used = !row, ok = true;
  int mycol = -1;
  for (int k = 0; k < ncol; ++k) {
    double v = used ? -1.0 : fabs(Kr[k]);
    int idx = lane;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) {  // rows live in lanes 0..15
      const double ov = __shfl_xor(v, o, kWave);
      const int oi = __shfl_xor(idx, o, kWave);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = __builtin_amdgcn_readlane(idx, 0);
    if (!(lane_bcast(v, 0) > 0.0)) {
      ok = false;
      break;
    }
    const double* Kp = S.sm.G[p];
    double pr[NC], my[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      pr[j] = j <= ncol ? Kp[j] : 0.0;
      my[j] = j <= ncol ? Kr[j] : 0.0;
    }
    const double inv = 1.0 / Kp[k], f = Kr[k] * inv;
    __syncthreads();
    if (row) {
      if (lane == p) {
#pragma unroll
        for (int j = 0; j < NC; ++j)
          if (j > k && j <= ncol) Kr[j] = my[j] * inv;
        Kr[k] = 1.0;
        used = true;
        mycol = k;
      } else {
#pragma unroll
        for (int j = 0; j < NC; ++j)
          if (j > k && j <= ncol) Kr[j] = fma(-f, pr[j], my[j]);
        Kr[k] = 0.0;
      }
    }
    __syncthreads();
  }
  if (ok && mycol >= 0) S.wvec[mycol] = Kr[ncol];
  __syncthreads();
  if (!ok) return false;
  bool fin = true;
  for (int j = lane; j < ncol; j += kWave) fin = fin && isfinite(S.wvec[j]);
  return __all(fin);
}

// (H + mu I) d = rhs (theta space) through the structure above: factor the
// tridiagonal part, then Woodbury for the contact blocks,
//   (T + U S U^T)^-1 v = z - T^-1 U w,  z = T^-1 v,  (I + S G) w = S U^T z,
//   G = U^T T^-1 U (one column per tridiagonal solve).
// Result into S.d.  false on a vanishing pivot or a failed small solve.
template <class SM>
__device__ bool structured_solve(SM& S, const Ctx& c, double mu, const double* rhs) {
  const int lane = threadIdx.x, n = c.n, L = S.ncl_links;
  if (lane == 0) S.res_ok = 0;  // G and F overwrite the resident data
  if (!tri_factor(S, n, mu)) return false;
  // right-hand side in absolute angles: b_m - b_{m+1}
  for (int m = lane; m < n; m += kWave) S.v[m] = rhs[m] - (m + 1 < n ? rhs[m + 1] : 0.0);
  __syncthreads();
  const int ncol = 3 * L;
  if (L == 0) {
    tri_solve(S, n, S.v, S.z);
  } else if (ncol <= 15) {
    gram_mfma(S, c, ncol);  // G, c and the forward half of z
    tri_bwd(S, n, S.z);
    bool ok;
    if (L == 1) {
      ok = tiny_solve<3>(S);
    } else if (L == 2) {
      ok = tiny_solve<6>(S);
    } else {
      capacitance_matrix(S, L);
      ok = small_solve(S, ncol);
    }
    if (!ok) return false;
  } else {
    tri_solve(S, n, S.v, S.z);
    ut_times(S, c, S.z, S.cvec, 1);
    for (int col = 0; col < ncol; ++col) {
      const int i = S.clink[col / 3], k = col % 3;
      for (int m = lane; m < n; m += kWave)
        S.v[m] = k == 2 ? (m == i ? 1.0 : 0.0) : (m < i ? c.l * (k == 0 ? S.tx[m] : S.ty[m]) : 0.0);
      __syncthreads();
      tri_solve(S, n, S.v, S.aux);
      ut_times(S, c, S.aux, &S.sm.G[0][col], kMaxCols + 1);
    }
    {
      capacitance_matrix(S, L);
      if (!lu_solve(&S.sm.G[0][0], kMaxCols + 1, ncol, S.wvec)) return false;
    }
  }
  if (L > 0) {
    // correction: T v = U w, d_phi = z - v
    for (int m = lane; m < n; m += kWave) {
      double u = 0.0;
      for (int a = 0; a < L; ++a) {
        const int i = S.clink[a];
        if (m < i) u += c.l * (S.tx[m] * S.wvec[3 * a] + S.ty[m] * S.wvec[3 * a + 1]);
        else if (m == i) u += S.wvec[3 * a + 2];
      }
      S.v[m] = u;
    }
    __syncthreads();
    tri_solve(S, n, S.v, S.v);
    for (int m = lane; m < n; m += kWave) S.z[m] -= S.v[m];
    __syncthreads();
  }
  // back to relative angles
  bool fin = true;
  for (int j = lane; j < n; j += kWave) {
    const double dj = S.z[j] - (j > 0 ? S.z[j - 1] : 0.0);
    S.d[j] = dj;
    fin = fin && isfinite(dj);
  }
  __syncthreads();
  return __all(fin);
}

// 1/x from the hardware reciprocal and two Newton steps (each doubles the correct
// bits; the result is within an ulp or two, and non-finite for a zero or non-finite x)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// (H + mu I) d = rhs directly in relative angles, for any number of contact links
// (the default Newton solve; the structured solve hands over to it beyond its
// capacity of contact links).
// With B_j = (1, px_j, py_j) the exact Hessian has the chain form
//   H_jm = q'_j [j = m] + B_j^T (sum_{k >= max(j,m)} S_k) B_m,
//   S_k = sum_{contacts on link k} (k_c a a^T - lam kappa b b^T) + e0 e0^T C_k,
// a = (n_y x_x - n_x x_y, -n_y, n_x), b = (n . x, -n_x, -n_y) (so that the contact
// gradient is B_j . a), C_k the geometric diagonal.  Writing F_j = sum_{k >= j} S_k V_k
// with V_k = sum_{m <= k} B_m d_m, the rows read (q'_j + mu) d_j + B_j . F_j = rhs_j;
// the affine map F_{j+1} = A_{j+1} V_j + z_{j+1} is carried from the tip to the base
// (a Riccati sweep of 3x3 matrices), then d follows from the base out.  One lane,
// O(n).  false on a vanishing pivot.
template <class SM>
__device__ bool chain_solve_seq(SM& S, const Ctx& c, double mu, const double* rhs) {
  const int lane = threadIdx.x, n = c.n, nc = S.ncl;
  double* s00 = S.dinv;
  double* s01 = S.ell;
  double* s02 = S.z;
  double* s11 = S.v;
  double* s12 = S.aux;
  double* s22 = S.ps1;
  for (int k = lane; k < n; k += kWave) {
    double m0 = S.cg[k], m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, m5 = 0.0;
    if (S.lidx[k] >= 0) {
      for (int e = 0; e < nc; ++e) {
        if (S.ci[e] != k) continue;
        const double nx = S.cnx[e], ny = S.cny[e], x = S.cxx[e], y = S.cxy[e];
        const double kc = c.P.kc, lk = S.cl[e] * S.ckap[e];
        const double a0 = ny * x - nx * y, a1 = -ny, a2 = nx;
        const double b0 = nx * x + ny * y, b1 = -nx, b2 = -ny;
        m0 += kc * a0 * a0 - lk * b0 * b0;
        m1 += kc * a0 * a1 - lk * b0 * b1;
        m2 += kc * a0 * a2 - lk * b0 * b2;
        m3 += kc * a1 * a1 - lk * b1 * b1;
        m4 += kc * a1 * a2 - lk * b1 * b2;
        m5 += kc * a2 * a2 - lk * b2 * b2;
      }
    }
    s00[k] = m0;
    s01[k] = m1;
    s02[k] = m2;
    s11[k] = m3;
    s12[k] = m4;
    s22[k] = m5;
  }
  bsync<SM>();
  if (lane == 0) {
    // One lane walks the chain, two links per pass: while one link computes, the
    // inputs of the link after the next are loading (indices are clamped, so the last
    // loads repeat valid ones).  Each link's B^T A B is stored, and all lanes test the
    // pivots after the walk (a failed pivot makes the remaining values non-finite).
    double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0, A5 = 0;  // symmetric 00 01 02 11 12 22
    double z0 = 0, z1 = 0, z2 = 0;
    struct In {
      double s0, s1, s2, s3, s4, s5, B1, B2, d, r;
    };
    auto load_in = [&](int k) {
      k = k > 0 ? k : 0;
      return In{s00[k], s01[k], s02[k], s11[k], s12[k], s22[k], S.px[k], S.py[k], S.dq[k], rhs[k]};
    };
    auto inward = [&](const In& q, int k) {
      A0 += q.s0;
      A1 += q.s1;
      A2 += q.s2;
      A3 += q.s3;
      A4 += q.s4;
      A5 += q.s5;
      const double B1 = q.B1, B2 = q.B2, dk = q.d + mu;
      const double h0 = fma(A2, B2, fma(A1, B1, A0));
      const double h1 = fma(A4, B2, fma(A3, B1, A1));
      const double h2 = fma(A5, B2, fma(A4, B1, A2));
      const double bh = fma(B2, h2, fma(B1, h1, h0));
      const double D = dk + bh;
      const double iD = rcp_nr(D);
      const double u = q.r - fma(B2, z2, fma(B1, z1, z0));
      const double g0 = h0 * iD, g1 = h1 * iD, g2 = h2 * iD, w = u * iD;
      A0 = fma(-h0, g0, A0);
      A1 = fma(-h0, g1, A1);
      A2 = fma(-h0, g2, A2);
      A3 = fma(-h1, g1, A3);
      A4 = fma(-h1, g2, A4);
      A5 = fma(-h2, g2, A5);
      z0 = fma(h0, w, z0);
      z1 = fma(h1, w, z1);
      z2 = fma(h2, w, z2);
      s00[k] = g0;  // the slots of S_k now hold what the outward pass needs
      s01[k] = g1;
      s02[k] = g2;
      s11[k] = w;
      s12[k] = bh;
    };
    In qa = load_in(n - 1), qb = load_in(n - 2);
    int k;
    for (k = n - 1; k >= 1; k -= 2) {
      inward(qa, k);
      qa = load_in(k - 2);
      inward(qb, k - 1);
      qb = load_in(k - 3);
    }
    if (k == 0) inward(qa, 0);
    // outward: d_k = w_k - g_k . V_{k-1}, V_k = V_{k-1} + B_k d_k
    struct Out {
      double g0, g1, g2, w, B1, B2;
    };
    auto load_out = [&](int k) {
      k = k < n ? k : 0;
      return Out{s00[k], s01[k], s02[k], s11[k], S.px[k], S.py[k]};
    };
    double V0 = 0, V1 = 0, V2 = 0;
    auto outward = [&](const Out& o, int k) {
      const double x = o.w - fma(o.g2, V2, fma(o.g1, V1, o.g0 * V0));
      V0 += x;
      V1 = fma(o.B1, x, V1);
      V2 = fma(o.B2, x, V2);
      S.d[k] = x;
    };
    Out oa = load_out(0), ob = load_out(1);
    for (k = 0; k + 1 < n; k += 2) {
      outward(oa, k);
      oa = load_out(k + 2);
      outward(ob, k + 1);
      ob = load_out(k + 3);
    }
    if (k < n) outward(oa, k);
  }
  bsync<SM>();
  // the pivots D = (q' + mu) + B^T A B, rounded as in the walk
  bool fin = true;
  for (int j = lane; j < n; j += kWave) {
    const double dk = S.dq[j] + mu, bh = s12[j], D = dk + bh;
    fin = fin && isfinite(D) && fabs(D) > 1e-14 * (fabs(dk) + fabs(bh)) && isfinite(S.d[j]);
  }
  return __all(fin);
}

// One equilibrium solve from S.th (in place).  Returns the status code.
template <class SM, bool DENSE>
__device__ int solve(SM& S, const Ctx& c, int& iters, double& rho) {
  const int lane = threadIdx.x, n = c.n;
  const KParams& P = c.P;
  int status = 1;
  double Pi = evaluate(S, c, S.th, true);
  for (int it = 0; it <= P.max_iter; ++it) {
    if (S.overflow) {
      status = 3;
      break;
    }
    double rm = 0.0;
    bool fin = true;
    for (int j = lane; j < n; j += kWave) {
      rm = fmax(rm, fabs(S.r[j]));
      fin = fin && isfinite(S.r[j]);
    }
    rm = wmax(rm);
    rho = rm / c.Mmax;
    if (!__all(fin) || !isfinite(Pi)) {
      status = 4;
      break;
    }
    if (rho <= P.tol) {
      status = 0;
      break;
    }
    if (it == P.max_iter) break;
    ++iters;
    bool ok = false;
    double slope = 0.0, mu = P.c_mu * rm;
    const bool structured = structured_setup(S, c, SM::kFull && !P.seq_solver);
    for (int j = lane; j < n; j += kWave) S.b[j] = -S.r[j];
    bsync<SM>();
    for (int tries = 0; tries < 24; ++tries) {
      if (tries > 0) mu = fmax(10.0 * mu, 1e-8 * c.Mmax);
      if (lane == 0) S.nsolves += 1.0;
      if constexpr (DENSE) {
        assemble(S, c, S.th, mu, S.b);
        if (!lu_solve_dense(S, n)) continue;
      } else if constexpr (SM::kFull) {
        if (structured ? !structured_solve(S, c, mu, S.b) : !chain_solve_seq(S, c, mu, S.b))
          continue;
      } else {
        if (!chain_solve_seq(S, c, mu, S.b)) continue;
      }
      double s = 0.0;
      for (int j = lane; j < n; j += kWave) s += S.r[j] * S.d[j];
      slope = wsum(s);
      if (slope < 0.0) {
        ok = true;
        break;
      }
    }
    if (!ok) {
      status = 2;
      break;
    }
    double dm = 0.0;
    for (int j = lane; j < n; j += kWave) dm = fmax(dm, fabs(S.d[j]));
    dm = wmax(dm);
    if (dm > P.step_max) {
      double f = P.step_max / dm;
      for (int j = lane; j < n; j += kWave) S.d[j] *= f;
      slope *= f;
    }
    bsync<SM>();
    const bool skip = -slope < 1e-12 * c.Mmax;
    double* tt = SM::kFull ? S.tt : S.b;  // trial angles (b is free once the step is solved)
    double alpha = 1.0, Pn = 0.0;
    bool acc = false;
    for (int ls = 0; ls < 40; ++ls) {
      for (int j = lane; j < n; j += kWave) tt[j] = S.th[j] + alpha * S.d[j];
      bsync<SM>();
      Pn = evaluate(S, c, tt, true);
      if (skip || Pn <= Pi + P.c1 * alpha * slope) {
        acc = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!acc) {
      status = 2;
      break;
    }
    if (c.trace && lane == 0) {
      int row = c.trace_n[0];
      if (row < c.trace_cap) {
        double* t = c.trace + (size_t)row * kTraceCols;
        t[0] = c.step; t[1] = c.sub; t[2] = it; t[3] = rho; t[4] = mu; t[5] = slope;
        t[6] = alpha; t[7] = Pn; t[8] = 0; t[9] = S.ncl;
        c.trace_n[0] = row + 1;
      }
    }
    for (int j = lane; j < n; j += kWave) S.th[j] = tt[j];
    Pi = Pn;
    bsync<SM>();
  }
  if (status != 0) evaluate(S, c, S.th, false);  // poses/contacts of the kept state
  return status;
}

// ---------------------------------------------------------------------------

// The helper wave of a two-wave launch: the obstacle phase of each evaluation the solver
// wave posts (between the two barriers of evaluate()), until the solver wave posts its
// end.  A barrier with no new command also ends the loop: a barrier completes without
// waves that have ended, so the helper never waits on a solver wave that is gone.
template <class SM>
__device__ void obstacle_helper(SM& S, const Ctx& c) {
  const int lane = threadIdx.x & (kWave - 1);
  int seen = 0;
  for (;;) {
    __syncthreads();
    const int seq = S.cmd_seq, cmd = S.cmd;
    if (seq == seen || cmd != 1) break;
    seen = seq;
    obstacle_phase(S, c, S.eval_n, S.eval_last, lane);
    __syncthreads();
  }
}

// One robot per workgroup: one wave (HELP = false) or two, the second taking the
// obstacle phase of every evaluation while the first sums the joint law.
template <int NMAX, bool DENSE, bool FULL = true, bool HELP = false>
__global__ __launch_bounds__(HELP ? 2 * kWave : kWave) __attribute__((amdgpu_waves_per_eu(1, 1))) void rollout_kernel(KParams P, KData D, int n_steps,
                                                        int record_traj) {
  using SMT = Smem<NMAX, DENSE ? 64 : 1, FULL, HELP>;
  __shared__ SMT S;
  if ((int)blockIdx.x >= D.launch_count) return;
  const int b = D.order[D.launch_first + blockIdx.x];
  const int lane = threadIdx.x;
  const int* ii = D.ii + 8 * b;
  const double* dd = D.dd + 6 * b;
  Ctx c;
  const int ntar = ii[0];
  c.K = ii[2] < kMaxObs ? ii[2] : kMaxObs;  // the boundary rejects more
  c.l = dd[0];
  c.R = dd[1];
  c.Mmax = kPi * dd[2] * c.R * c.R * c.R;
  c.arm = 2.0 * c.R + P.Ract;
  c.bx = dd[3];
  c.by = dd[4];
  c.bpsi = dd[5];
  c.tab = D.tables + ii[3];
  c.wr = D.wr;
  c.P = P;
  c.trace = (b == D.trace_robot) ? D.trace : nullptr;
  c.trace_n = D.trace_n;
  c.trace_cap = D.trace_cap;
  c.obs = D.obs + 4 * (size_t)ii[1];
  c.okind = D.okind + ii[1];
  if constexpr (HELP) {
    if (threadIdx.x >= kWave) {
      obstacle_helper(S, c);
      return;
    }
  }
  if (lane == 0) {
    S.res_ok = 0;  // staged by the first evaluation
    S.cmd = 0;
    S.cmd_seq = 0;
  }
  for (int j = lane; j < ntar; j += kWave) {
    S.pp[j] = D.cover[2 * (size_t)(ii[4] + j)];
    S.pm[j] = D.cover[2 * (size_t)(ii[4] + j) + 1];
  }
  const long long t_begin = clock64();  // this robot's time in the launch (for scheduling)
  int n = D.ncur[b];
  int t = D.tcur[b];
  if (lane == 0) {
    S.jevals = 0.0;
    S.nsolves = 0.0;
  }
  for (int j = lane; j < n; j += kWave) S.th[j] = D.theta[(size_t)b * D.n_max + j];
  bsync<SMT>();
  for (int step = 0; step < n_steps && t < D.t_max; ++step, ++t) {
    int st_worst = 0, its = 0;
    double rho = 0.0;
    if (n < ntar) {
      ++n;
      if (lane == 0) S.th[n - 1] = 0.0;
      bsync<SMT>();
      c.n = n;
      for (int s = 1; s <= P.substeps; ++s) {
        c.last_len = c.l * (double)s / (double)P.substeps;
        c.step = t;
        c.sub = s;
        int st = solve<SMT, DENSE>(S, c, its, rho);
        st_worst = st > st_worst ? st : st_worst;
      }
    } else {
      c.n = n;
      c.last_len = c.l;
      st_worst = -1;
      if (n > 0) evaluate(S, c, S.th, false);
    }
    // record the state after this step
    const size_t bt = (size_t)b * D.t_max + t;
    double hsum = 0.0;
    for (int j = lane; j < n; j += kWave) hsum += S.th[j];
    hsum = wsum(hsum);
    int nc = n > 0 ? S.ncl : 0;
    unsigned long long hv = 0ull;
    int npair = 0;
    double mp = 0.0;
    for (int e = lane; e < nc; e += kWave) {
      bool dup = false;
      for (int f = 0; f < e; ++f) dup = dup || (S.ci[f] == S.ci[e] && S.ck[f] == S.ck[e]);
      if (!dup) {
        hv += mix64((unsigned long long)S.ci[e] * 1024ull + (unsigned long long)S.ck[e]);
        ++npair;
      }
      mp = fmax(mp, S.cpen[e]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      hv += __shfl_xor(hv, o, kWave);
      npair += __shfl_xor(npair, o, kWave);
    }
    mp = wmax(mp);
    if (lane == 0) {
      D.tip[3 * bt + 0] = n > 0 ? S.px[n] : c.bx;
      D.tip[3 * bt + 1] = n > 0 ? S.py[n] : c.by;
      D.tip[3 * bt + 2] = c.bpsi + hsum;
      D.rho[bt] = rho;
      D.iters[bt] = its;
      D.status[bt] = st_worst;
      D.ncont[bt] = npair;
      D.chash[bt] = hv;
      D.maxpen[bt] = mp;
    }
    if (record_traj && D.traj)
      for (int j = lane; j < D.n_max; j += kWave)
        D.traj[bt * D.n_max + j] = j < n ? S.th[j] : 0.0;
    bsync<SMT>();
  }
  for (int j = lane; j < n; j += kWave) D.theta[(size_t)b * D.n_max + j] = S.th[j];
  if (lane == 0) {
    D.ncur[b] = n;
    D.tcur[b] = t;
    D.jevals[b] += S.jevals;
    D.nsolves[b] += S.nsolves;
    D.cycles[b] += (double)(clock64() - t_begin);
  }
  if constexpr (HELP) {
    if (lane == 0) {
      S.cmd = 2;
      S.cmd_seq += 1;
    }
    __syncthreads();  // releases the helper wave, which then ends
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the growth step.  For L = sum_t w_t |tip_t - goal|^2 over converged
// states (r_t(theta_t; p) = 0, independent of the previous state):
//   dL/dp = - sum_t lam_t . dr_t/dp,  H_t lam_t = w_t dL_t/dtheta,
// H_t the exact Hessian (same structured solve, mu = 0).  An sPAM's pressure P_s and
// its ends s0, s1 enter r only through the coverage of the joints it spans:
//   dq_j/dP+-_j = -+arm G(eps+-_j),  w_sj = |[s0, s1] ^ [j l, (j+1) l]| / l.
template <int NMAX>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 1))) void grad_kernel(KParams P, KData D, const double* goal,
                                                     const double* weights, int T,
                                                     double* dP, double* ds0, double* ds1,
                                                     double* loss, int* status) {
  __shared__ Smem<NMAX, 1> S;
  if ((int)blockIdx.x >= D.launch_count) return;
  const int b = D.order[D.launch_first + blockIdx.x], lane = threadIdx.x;
  const int* ii = D.ii + 8 * b;
  const double* dd = D.dd + 6 * b;
  Ctx c;
  const int ntar = ii[0];
  c.K = ii[2] < kMaxObs ? ii[2] : kMaxObs;  // the boundary rejects more
  c.l = dd[0];
  c.R = dd[1];
  c.Mmax = kPi * dd[2] * c.R * c.R * c.R;
  c.arm = 2.0 * c.R + P.Ract;
  c.bx = dd[3];
  c.by = dd[4];
  c.bpsi = dd[5];
  c.tab = D.tables + ii[3];
  c.wr = D.wr;
  c.P = P;
  c.trace = nullptr;
  c.last_len = c.l;
  c.obs = D.obs + 4 * (size_t)ii[1];
  c.okind = D.okind + ii[1];
  if (lane == 0) S.res_ok = 0;  // staged by the first evaluation
  for (int j = lane; j < ntar; j += kWave) {
    S.pp[j] = D.cover[2 * (size_t)(ii[4] + j)];
    S.pm[j] = D.cover[2 * (size_t)(ii[4] + j) + 1];
  }
  const int soff = ii[5], ns = ii[6];
  const double gx = goal[2 * b], gy = goal[2 * b + 1];
  double aP = 0.0, a0 = 0.0, a1 = 0.0, Lsum = 0.0;  // this lane's sPAM (lane < ns)
  int st = 0;
  const int taken = D.tcur[b];
  for (int t = 0; t < (weights ? (T < taken ? T : taken) : 1); ++t) {
    const double wt = weights ? weights[t] : 1.0;
    if (wt == 0.0) continue;
    int n;
    if (weights) {
      n = t + 1 < ntar ? t + 1 : ntar;
      for (int j = lane; j < n; j += kWave) S.th[j] = D.traj[((size_t)b * D.t_max + t) * D.n_max + j];
    } else {
      n = D.ncur[b];
      for (int j = lane; j < n; j += kWave) S.th[j] = D.theta[(size_t)b * D.n_max + j];
    }
    if (n == 0) continue;
    c.n = n;
    __syncthreads();
    evaluate(S, c, S.th, false);
    const double ex = S.px[n] - gx, ey = S.py[n] - gy;
    Lsum += wt * (ex * ex + ey * ey);
    if (S.overflow) {  // contact list truncated: the Hessian would be wrong
      st = 1;
      continue;
    }
    for (int j = lane; j < n; j += kWave) {
      const double vx = -(S.py[n] - S.py[j]), vy = S.px[n] - S.px[j];
      S.b[j] = 2.0 * wt * (ex * vx + ey * vy);
    }
    __syncthreads();
    const bool ok = structured_setup(S, c) ? structured_solve(S, c, 0.0, S.b)
                                           : chain_solve_seq(S, c, 0.0, S.b);
    if (!ok) {
      st = 1;
      continue;
    }
    // one lane per sPAM of this robot (at most kWave of them)
    if (lane < ns) {
      const double* e = D.spam + 4 * (size_t)(soff + lane);
      const int j0 = (int)floor(e[0] / c.l);
      for (int j = j0 < 0 ? 0 : j0; j < n && j * c.l < e[1]; ++j) {
        const double lo = fmax(e[0], j * c.l), hi = fmin(e[1], (j + 1) * c.l);
        if (!(hi > lo)) continue;
        const double th = S.th[j];
        const double eps = e[2] > 0.0 ? (th > 0.0 ? c.arm * th / c.l : 0.0)
                                      : (th < 0.0 ? -c.arm * th / c.l : 0.0);
        double G;
        spam_law(*c.tab, eps, &G, nullptr, nullptr);
        const double lq = S.d[j] * (e[2] > 0.0 ? -c.arm * G : c.arm * G);  // lam_j dq_j/dP
        aP -= lq * (hi - lo) / c.l;
        if (e[0] > j * c.l) a0 += lq * e[3] / c.l;
        if (e[1] < (j + 1) * c.l) a1 -= lq * e[3] / c.l;
      }
    }
    __syncthreads();
  }
  // robots may share sPAM records: their contributions add up
  if (lane < ns) {
    atomicAdd(&dP[soff + lane], aP);
    atomicAdd(&ds0[soff + lane], a0);
    atomicAdd(&ds1[soff + lane], a1);
  }
  if (lane == 0) {
    loss[b] = Lsum;
    if (status) status[b] = st;
  }
}

__global__ void zero3_kernel(double* a, double* b, double* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = 0.0;
    b[i] = 0.0;
    c[i] = 0.0;
  }
}

hipError_t launch_zero3(double* a, double* b, double* c, int n, hipStream_t stream) {
  if (n > 0)
    hipLaunchKernelGGL(zero3_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, a, b, c, n);
  return hipGetLastError();
}

// One launch per chain-length class: D.order[D.launch_first ...] lists the robots of
// the class (longest expected work first), D.launch_count of them.
hipError_t launch_grad(const KParams& P, const KData& D, const double* goal,
                       const double* weights, int T, double* dP, double* ds0, double* ds1,
                       double* loss, int* status, int nmax_class, hipStream_t stream) {
  if (D.launch_count <= 0) return hipSuccess;
  dim3 grid(D.launch_count), block(kWave);
  if (nmax_class == 64)
    hipLaunchKernelGGL((grad_kernel<64>), grid, block, 0, stream, P, D, goal, weights, T, dP, ds0,
                       ds1, loss, status);
  else if (nmax_class == 128)
    hipLaunchKernelGGL((grad_kernel<128>), grid, block, 0, stream, P, D, goal, weights, T, dP,
                       ds0, ds1, loss, status);
  else if (nmax_class == 256)
    hipLaunchKernelGGL((grad_kernel<256>), grid, block, 0, stream, P, D, goal, weights, T, dP,
                       ds0, ds1, loss, status);
  else if (nmax_class == 512)
    hipLaunchKernelGGL((grad_kernel<512>), grid, block, 0, stream, P, D, goal, weights, T, dP,
                       ds0, ds1, loss, status);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Zero the state and records of every robot (a kernel rather than memsets, so that
// a captured graph holds no memset nodes).
__global__ void reset_kernel(KData D) {
  const size_t B = D.n_inst, stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = i0; i < B * D.n_max; i += stride) D.theta[i] = 0.0;
  for (size_t i = i0; i < B * D.t_max * 3; i += stride) D.tip[i] = 0.0;
  for (size_t i = i0; i < B * D.t_max; i += stride) {
    D.rho[i] = 0.0;
    D.iters[i] = 0;
    D.status[i] = 0;
    D.ncont[i] = 0;
    D.chash[i] = 0ull;
    D.maxpen[i] = 0.0;
  }
  for (size_t i = i0; i < B; i += stride) {
    D.ncur[i] = 0;
    D.tcur[i] = 0;
    D.jevals[i] = 0.0;
    D.nsolves[i] = 0.0;
    D.cycles[i] = 0.0;
  }
}

// Zero the state and records of the robots in slots[0..count) (one block per robot).
__global__ void slot_reset_kernel(KData D, const int* slots, int count) {
  if ((int)blockIdx.x >= count) return;
  const size_t b = (size_t)slots[blockIdx.x];
  for (int j = threadIdx.x; j < D.n_max; j += blockDim.x) D.theta[b * D.n_max + j] = 0.0;
  for (int t = threadIdx.x; t < D.t_max; t += blockDim.x) {
    const size_t bt = b * D.t_max + t;
    D.tip[3 * bt] = 0.0;
    D.tip[3 * bt + 1] = 0.0;
    D.tip[3 * bt + 2] = 0.0;
    D.rho[bt] = 0.0;
    D.iters[bt] = 0;
    D.status[bt] = 0;
    D.ncont[bt] = 0;
    D.chash[bt] = 0ull;
    D.maxpen[bt] = 0.0;
  }
  if (threadIdx.x == 0) {
    D.ncur[b] = 0;
    D.tcur[b] = 0;
    D.jevals[b] = 0.0;
    D.nsolves[b] = 0.0;
    D.cycles[b] = 0.0;
  }
}

hipError_t launch_slot_reset(const KData& D, const int* slots, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(slot_reset_kernel, dim3(count), dim3(256), 0, stream, D, slots, count);
  return hipGetLastError();
}

hipError_t launch_reset(const KData& D, hipStream_t stream) {
  const size_t work = (size_t)D.n_inst * (D.t_max * 3 > D.n_max ? D.t_max * 3 : D.n_max);
  const size_t blocks = (work + 255) / 256 < 4096 ? (work + 255) / 256 : 4096;
  hipLaunchKernelGGL(reset_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     stream, D);
  return hipGetLastError();
}

// host-side launcher (instantiated for the supported chain lengths)
hipError_t launch_rollout(const KParams& P, const KData& D, int n_steps, int record_traj,
                          int nmax_class, hipStream_t stream) {
  if (D.launch_count <= 0) return hipSuccess;
  dim3 grid(D.launch_count), block(kWave);
  if (P.dense_solver) {
    if (nmax_class != 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((rollout_kernel<64, true>), grid, block, 0, stream, P, D, n_steps,
                       record_traj);
  } else if (nmax_class == 64) {
    if (P.seq_solver)
      hipLaunchKernelGGL((rollout_kernel<64, false, false, true>), grid, dim3(2 * kWave), 0,
                         stream, P, D, n_steps, record_traj);
    else
      hipLaunchKernelGGL((rollout_kernel<64, false>), grid, block, 0, stream, P, D, n_steps,
                         record_traj);
  } else if (nmax_class == 128) {
    if (P.seq_solver)
      hipLaunchKernelGGL((rollout_kernel<128, false, false, true>), grid, dim3(2 * kWave), 0,
                         stream, P, D, n_steps, record_traj);
    else
      hipLaunchKernelGGL((rollout_kernel<128, false>), grid, block, 0, stream, P, D, n_steps,
                         record_traj);
  } else if (nmax_class == 256) {
    if (P.seq_solver)
      hipLaunchKernelGGL((rollout_kernel<256, false, false, true>), grid, dim3(2 * kWave), 0,
                         stream, P, D, n_steps, record_traj);
    else
      hipLaunchKernelGGL((rollout_kernel<256, false>), grid, block, 0, stream, P, D, n_steps,
                         record_traj);
  } else if (nmax_class == 512) {
    if (P.seq_solver)
      hipLaunchKernelGGL((rollout_kernel<512, false, false, true>), grid, dim3(2 * kWave), 0,
                         stream, P, D, n_steps, record_traj);
    else
      hipLaunchKernelGGL((rollout_kernel<512, false>), grid, block, 0, stream, P, D, n_steps,
                         record_traj);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vs
