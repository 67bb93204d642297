// vs_rollout.hip -- gfx950 kernels of the batched quasi-static growth step of the vine
// robot (arXiv 2509.15180, Sec. 3-4) and of its adjoint.
//
// One workgroup owns one robot.  In the rollout launches a solver wave (64 lanes
// striding over the links) runs the descent and a helper wave takes the obstacle phase
// of every evaluation; the adjoint runs on one wave.  All model arithmetic is FP64: on
// gfx950 an FP64 FMA issues at the rate of an unpacked FP32 FMA, and the equilibrium
// must be resolved to 1e-10 of the body's moment scale.
//
// A growth step (Alg. 1, read as a converged descent to a local minimum of the energy
// of Eq. 4, which the paper states as an argmin):
//   append a link at zero angle; for each growth sub-step (tip length l s/S):
//     repeat
//       poses by wave prefix scans of theta and of the link vectors (Sec. 4.1);
//       joint moments q_j (Eq. 2, Eq. 3) and penetrating disk/obstacle pairs,
//       compacted deterministically with ballots into an LDS contact list;
//       residual r_j = q_j - sum_{contacts on links >= j} lam (x - p_j) x n
//       (suffix scans of per-link force and moment sums);
//       factorise H + mu I (H the exact Hessian) by a sequential O(n) Riccati sweep
//       from the tip; its pivots give the inertia (Sylvester's law);
//       stop when max_j |r_j| / M_max <= tol and H + delta I is positive definite;
//       positive definite: the damped Newton step (H + mu I) d = -r, |d|_inf capped;
//       indefinite: a step along the negative curvature of the most negative pivot;
//       Armijo backtracking on the energy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vs_device.h"

namespace vs {

constexpr int kMaxC = 128;
constexpr double kFull = 1.0 - 1e-12;  // soft growth: a tip link at full length
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
  // soft growth: the tip link's length u l is a variable (S.u), under the growth term
  // (wg/2) (l (tgt - u))^2 of Eq. 4 with this sub-step's target tgt (link lengths)
  bool soft;
  double tgt;
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
// LDS working set of one robot.  HELP_: helper waves beside the solver wave take the
// obstacle phase of each evaluation (the rollout launches); without them one wave does
// everything (the adjoint, and one-wave rollouts).  FOUR_: three helper waves, which split
// the joint law and the obstacle phase by chunks of 64 links (the second half of the
// chunks' contacts goes to a second region of the contact list, appended after the first).
template <int NMAX, bool HELP_, bool FOUR_ = false>
struct Smem {
  static constexpr bool kHelper = HELP_;
  static constexpr bool kFour = FOUR_;
  static constexpr int kRegions = FOUR_ ? 2 : 1;
  struct {
    double ox[kMaxObs], oy[kMaxObs], oa[kMaxObs], ob[kMaxObs];
    int okind[kMaxObs];
  } res;       // the robot's obstacles (structure of arrays), staged by the first evaluation
  int res_ok;  // res holds this robot's obstacles
  double th[NMAX], d[NMAX], r[NMAX];
  double b[NMAX];  // right-hand side of the Newton system, then the line search's trial angles
  double px[NMAX + 1], py[NMAX + 1], tx[NMAX], ty[NMAX];
  double pp[NMAX], pm[NMAX];
  double dq[NMAX];  // joint stiffness q'_j
  double cg[NMAX];  // geometric stiffness of the contact forces, diagonal in absolute angles
  // per-link contact sums of an evaluation (moment, force x, force y, the force's moment
  // along the link); the sweep reuses them, with sw0..sw2, for its blocks and factors
  double ps1[NMAX], ps2[NMAX], aux[NMAX], v[NMAX];
  double sw0[NMAX], sw1[NMAX], sw2[NMAX];
  int lidx[NMAX];  // 1 when link j carries a contact
  int ci[kRegions * kMaxC], ck[kRegions * kMaxC];
  double cl[kRegions * kMaxC], cxx[kRegions * kMaxC], cxy[kRegions * kMaxC],
      cnx[kRegions * kMaxC], cny[kRegions * kMaxC], ckap[kRegions * kMaxC],
      cpen[kRegions * kMaxC];
  int ncl;
  int overflow;
  int cnt0, cnt1;                 // pairs found in each region's chunks (may exceed kMaxC)
  double ech[NMAX / kWave];       // joint energy of each chunk of 64 joints
  int eval_trial, eval_E;         // solver -> helpers: angles in b (trial) or th; energy wanted
  double jevals, nsolves, negsteps;  // work counters (lane 0 updates)
  int cmd, cmd_seq, eval_n;  // solver wave -> helper wave: 1 = obstacle phase, 2 = end
  double eval_last;
  // soft growth (the variable u after the joints): the accepted u, the u an evaluation
  // uses, dPi/du there, its coupling to the joints (H_ju = cu . B_j) and diagonal H_uu, the
  // right-hand side, step and pivot of the last sweep
  double u, ue, ru, cu0, cu1, cu2, huu, bu, du, Du;
  int uvar;  // the tip length is a variable of this iteration (not held on u = 0)
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

// Copy the robot's obstacles into LDS (structure of arrays).
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
  if (lane == 0) S.res_ok = 1;
  bsync<SM>();
}

// The contact part of an evaluation at the poses in S (n links, the last of length
// last_len) for the chunks of 64 links [ch0, ch1), on one wave whose lane index is lane:
// penetrating (disk, obstacle) pairs into the contact list from position base (at most
// kMaxC of them), each link's contact sums into ps1, ps2, aux and v.  Returns the number
// of pairs found (uniform; more than kMaxC when the list is too short).
template <class SM>
__device__ int obstacle_phase(SM& S, const Ctx& c, int n, double last_len, int lane, int ch0,
                              int ch1, int base_pos) {
  // penetrating (disk, obstacle) pairs, compacted in (obstacle, disk, link) order per
  // chunk.  The exact gap (square root, divisions) is taken only for pairs whose
  // cheap pre-test some lane of the wave passes.
  int cnt = 0;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int base = ch0 * kWave; base < n && base < ch1 * kWave; base += kWave) {
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
              const int at = base_pos + pos;
              S.ci[at] = j;
              S.ck[at] = ks[u];
              S.cl[at] = lam;
              S.cxx[at] = xs[hh];
              S.cxy[at] = ys[hh];
              S.cnx[at] = nx;
              S.cny[at] = ny;
              S.ckap[at] = kap;
              S.cpen[at] = pen;
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
    if (on) {  // read by evaluate()'s suffix sums and by newton_setup
      S.ps1[j] = a_s1;
      S.ps2[j] = a_fx;
      S.aux[j] = a_fy;
      S.v[j] = a_q;
    }
  }
  return cnt;
}

// The joint law of chunks [ch0, ch1) of 64 joints at angles th, on one wave: moments into
// r, slopes into dq (when a helper wave shares the evaluation: the Newton set-up that
// follows an evaluation is always at the angles last evaluated), and each chunk's energy,
// summed over its lanes, into ech.
template <class SM>
__device__ void joint_law_chunks(SM& S, const Ctx& c, const double* th, bool want_E, int ch0,
                                 int ch1, int lane) {
  const int n = c.n;
  for (int k = ch0; k < ch1; ++k) {
    const int j = k * kWave + lane;
    double E = 0.0;
    if (j < n) {
      double q;
      if constexpr (SM::kHelper) {
        double dqj;
        joint_law(c, *c.tab, *c.wr, th[j], S.pp[j], S.pm[j], &q, &dqj, want_E ? &E : nullptr);
        S.dq[j] = dqj;
      } else {
        joint_law(c, *c.tab, *c.wr, th[j], S.pp[j], S.pm[j], &q, nullptr, want_E ? &E : nullptr);
      }
      S.r[j] = q;
    }
    E = wsum(E);
    if (lane == 0) S.ech[k] = E;
  }
}

// Poses, joint moments, contacts, residual (into S.r) and energy at angles th.  In the
// two-wave launches the joint slopes q'_j are computed here as well (into S.dq), while
// the helper wave is busy with the contacts: the Newton set-up that follows an
// evaluation is always at the angles last evaluated.
template <class SM>
__device__ double evaluate(SM& S, const Ctx& c, const double* th, bool want_E) {
  const int lane = threadIdx.x;
  const int n = c.n;
  if (__builtin_amdgcn_readfirstlane(S.res_ok) == 0) stage_resident(S, c);
  if (lane == 0) S.jevals += n;
  // the tip link's length: prescribed (hard growth) or u l (soft growth, u = S.ue)
  const double ue = c.soft ? S.ue : 0.0;
  const double last = c.soft ? ue * c.l : c.last_len;
  double cphi = c.bpsi, cx = c.bx, cy = c.by;
  for (int base = 0; base < n; base += kWave) {
    int j = base + lane;
    bool on = j < n;
    double phi = wscan_incl(on ? th[j] : 0.0, lane) + cphi;
    double sj, cj;
    sincos(phi, &sj, &cj);
    double L = (j == n - 1) ? last : c.l;
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
  const int nch = (n + kWave - 1) / kWave;
  if constexpr (SM::kHelper) {
    if (lane == 0) {
      S.eval_n = n;
      S.eval_last = last;
      S.eval_trial = th != S.th;
      S.eval_E = want_E;
      S.cmd = 1;
      S.cmd_seq += 1;
    }
    __syncthreads();  // the poses are in LDS: the helper waves start
  } else {
    bsync<SM>();
  }
  // the joint law of the solver's chunks (with four waves the first half of them; a
  // helper takes the rest): moments into r, slopes into dq (with helpers), and each
  // chunk's energy into ech
  joint_law_chunks<SM>(S, c, th, want_E, 0, SM::kFour ? (nch + 1) / 2 : nch, lane);
  if constexpr (SM::kHelper) {
    __syncthreads();  // the helpers' contacts, contact sums and joint laws are in LDS
  } else {
    const int cnt = obstacle_phase(S, c, n, last, lane, 0, nch, 0);
    if (lane == 0) {
      S.cnt0 = cnt;
      S.cnt1 = 0;
    }
    bsync<SM>();
  }
  {
    // the contact list: the first region's pairs, then (four waves) the second's
    const int c0 = S.cnt0, c1 = SM::kFour ? S.cnt1 : 0;
    const int n0 = c0 < kMaxC ? c0 : kMaxC;
    if constexpr (SM::kFour) {
      const int n1 = c1 < kMaxC - n0 ? c1 : kMaxC - n0;
      for (int e = lane; e < n1; e += kWave) {
        const int from = kMaxC + e, to = n0 + e;
        S.ci[to] = S.ci[from];
        S.ck[to] = S.ck[from];
        S.cl[to] = S.cl[from];
        S.cxx[to] = S.cxx[from];
        S.cxy[to] = S.cxy[from];
        S.cnx[to] = S.cnx[from];
        S.cny[to] = S.cny[from];
        S.ckap[to] = S.ckap[from];
        S.cpen[to] = S.cpen[from];
      }
    }
    if (lane == 0) {
      const int tot = c0 + c1;
      S.ncl = tot < kMaxC ? tot : kMaxC;
      S.overflow = tot > kMaxC;
    }
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
  double Esum = 0.0;  // the chunks' joint energies in chunk order (the same in every mode)
  for (int k = 0; k < nch; ++k) Esum += S.ech[k];
  double pen2 = 0.0;
  for (int e = lane; e < nc; e += kWave) pen2 += 0.5 * c.P.kc * S.cpen[e] * S.cpen[e];
  double grow = 0.0;
  if (c.soft) {
    // dPi/du: the growth term, and each contact on the tip link, whose disk at fraction f
    // of the link moves by f l t per unit of u
    const double gap = c.l * (c.tgt - ue);
    grow = 0.5 * c.P.wg * gap * gap;
    const double tx = S.tx[n - 1], ty = S.ty[n - 1], px = S.px[n - 1], py = S.py[n - 1];
    double acc = 0.0;
    for (int e = lane; e < nc; e += kWave) {
      if (S.ci[e] != n - 1) continue;
      const double sd = (S.cxx[e] - px) * tx + (S.cxy[e] - py) * ty;
      const double f = sd > 0.75 * last ? 1.0 : 0.5;
      acc += S.cl[e] * f * (S.cnx[e] * tx + S.cny[e] * ty);
    }
    acc = wsum(acc);
    if (lane == 0) S.ru = -c.P.wg * c.l * gap - c.l * acc;
  }
  bsync<SM>();
  return Esum + wsum(pen2) + grow;
}

// Per-iteration set-up of the Newton system at the state last evaluated: the joint
// slopes (one-wave launches; the two-wave evaluation left them in dq), which links carry
// contacts, and the geometric stiffness of the contact forces in absolute angles,
//   C_m = l t_m . (sum of contact forces on links beyond m) + sum_{disks on m} lam s n.t_m,
// s the disk's distance from the link's proximal joint, from the per-link sums that
// evaluate() leaves in ps2, aux and v.
template <class SM>
__device__ void newton_setup(SM& S, const Ctx& c) {
  const int lane = threadIdx.x, n = c.n, nc = S.ncl;
  for (int j = lane; j < n; j += kWave) {
    if constexpr (!SM::kHelper) {
      double d;
      joint_law(c, *c.tab, *c.wr, S.th[j], S.pp[j], S.pm[j], nullptr, &d, nullptr);
      S.dq[j] = d;
    }
    S.lidx[j] = 0;
  }
  bsync<SM>();
  for (int e = lane; e < nc; e += kWave) S.lidx[S.ci[e]] = 1;
  double cfx = 0.0, cfy = 0.0;
  const int nchunk = (n + kWave - 1) / kWave;
  for (int ch = nchunk - 1; ch >= 0; --ch) {
    const int j = ch * kWave + lane;
    const double fx = j < n ? S.ps2[j] : 0.0, fy = j < n ? S.aux[j] : 0.0;
    const double q = j < n ? S.v[j] : 0.0;
    double sx = wscan_suffix(fx, lane) + cfx, sy = wscan_suffix(fy, lane) + cfy;
    if (j < n) S.cg[j] = c.l * (S.tx[j] * (sx - fx) + S.ty[j] * (sy - fy)) + q;
    cfx = __shfl(sx, 0, kWave);
    cfy = __shfl(sy, 0, kWave);
  }
  if (c.soft && __builtin_amdgcn_readfirstlane(S.uvar)) {
    // soft growth: the tip length's row of the Hessian.  A contact on the tip link at
    // fraction f, with n_t = n.t, tau_t = tau.t and nz = n.(z x t) for the link direction
    // t (which turns with every joint), adds (f l)^2 (k_c n_t^2 - lam kappa tau_t^2) to
    // H_uu and f l (k_c n_t a - lam kappa tau_t b - lam nz e_0) to the coupling vector cu
    // (H_ju = cu . B_j, a and b the contact's vectors of the chain form).
    const double tx = S.tx[n - 1], ty = S.ty[n - 1], px = S.px[n - 1], py = S.py[n - 1];
    const double last = S.ue * c.l;
    double h = 0.0, k0 = 0.0, k1 = 0.0, k2 = 0.0;
    for (int e = lane; e < nc; e += kWave) {
      if (S.ci[e] != n - 1) continue;
      const double x = S.cxx[e], y = S.cxy[e], nx = S.cnx[e], ny = S.cny[e];
      const double sd = (x - px) * tx + (y - py) * ty;
      const double fl = (sd > 0.75 * last ? 1.0 : 0.5) * c.l;
      const double lam = S.cl[e], lk = lam * S.ckap[e], kc = c.P.kc;
      const double nt = nx * tx + ny * ty, taut = -ny * tx + nx * ty, nz = -nx * ty + ny * tx;
      h += fl * fl * (kc * nt * nt - lk * taut * taut);
      const double wa = kc * nt, wb = lk * taut;
      k0 += fl * (wa * (ny * x - nx * y) - wb * (nx * x + ny * y) - lam * nz);
      k1 += fl * (wa * -ny - wb * -nx);
      k2 += fl * (wa * nx - wb * -ny);
    }
    h = wsum(h);
    k0 = wsum(k0);
    k1 = wsum(k1);
    k2 = wsum(k2);
    if (lane == 0) {
      S.huu = c.P.wg * c.l * c.l + h;
      S.cu0 = k0;
      S.cu1 = k1;
      S.cu2 = k2;
    }
  }
  bsync<SM>();
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

constexpr int kSweepFail = 0;   // a vanishing or non-finite pivot, or a non-finite step
constexpr int kSweepPD = 1;     // H + mu I positive definite; the step is in S.d
constexpr int kSweepIndef = 2;  // a negative pivot: H + mu I is indefinite

// (H + mu I) d = rhs directly in relative angles, for any number of contacts.
// With B_j = (1, px_j, py_j) the exact Hessian has the chain form
//   H_jm = q'_j [j = m] + B_j^T (sum_{k >= max(j,m)} S_k) B_m,
//   S_k = sum_{contacts on link k} (k_c a a^T - lam kappa b b^T) + e0 e0^T C_k,
// a = (n_y x_x - n_x x_y, -n_y, n_x), b = (n . x, -n_x, -n_y) (so that the contact
// gradient is B_j . a), C_k the geometric diagonal.  Writing F_j = sum_{k >= j} S_k V_k
// with V_k = sum_{m <= k} B_m d_m, the rows read (q'_j + mu) d_j + B_j . F_j = rhs_j;
// the affine map F_{j+1} = A_{j+1} V_j + z_{j+1} is carried from the tip to the base
// (a Riccati sweep of 3x3 matrices), then d follows from the base out.  The sweep is
// the LDL^T factorisation of H + mu I that eliminates the joints from the tip,
//   H + mu I = U diag(D) U^T,  D_j = q'_j + mu + B_j^T A_j B_j,
// so by Sylvester's law of inertia H + mu I is positive definite exactly when every
// pivot D_j is.  One lane, O(n).  Leaves the factors for neg_curv_dir: g_j (U's column
// j is g_j . B_m for m < j) in sw0..sw2 and B_j^T A_j B_j in aux.
template <class SM>
__device__ int chain_solve_seq(SM& S, const Ctx& c, double mu, const double* rhs) {
  const int lane = threadIdx.x, n = c.n, nc = S.ncl;
  const bool uv = c.soft && __builtin_amdgcn_readfirstlane(S.uvar);
  double* s00 = S.sw0;
  double* s01 = S.sw1;
  double* s02 = S.sw2;
  double* s11 = S.v;
  double* s12 = S.aux;
  double* s22 = S.ps1;
  for (int k = lane; k < n; k += kWave) {
    double m0 = S.cg[k], m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, m5 = 0.0;
    if (S.lidx[k]) {
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
    // pivots after the walk (a vanishing pivot makes the remaining values non-finite).
    double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0, A5 = 0;  // symmetric 00 01 02 11 12 22
    double z0 = 0, z1 = 0, z2 = 0;
    double iDu = 0.0;
    if (uv) {
      // soft growth: the tip length is eliminated first (pivot H_uu + mu); its coupling
      // H_ju = cu . B_j to every joint leaves A = -cu cu^T / D_u and z = cu b_u / D_u
      const double Du = S.huu + mu;
      iDu = rcp_nr(Du);
      const double k0 = S.cu0, k1 = S.cu1, k2 = S.cu2;
      const double g0 = k0 * iDu, g1 = k1 * iDu, g2 = k2 * iDu, wu = S.bu * iDu;
      A0 = -k0 * g0;
      A1 = -k0 * g1;
      A2 = -k0 * g2;
      A3 = -k1 * g1;
      A4 = -k1 * g2;
      A5 = -k2 * g2;
      z0 = k0 * wu;
      z1 = k1 * wu;
      z2 = k2 * wu;
      S.Du = Du;
    }
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
    // soft growth: d_u = (b_u - cu . V_{n-1}) / D_u
    if (uv) S.du = (S.bu - fma(S.cu2, V2, fma(S.cu1, V1, S.cu0 * V0))) * iDu;
  }
  bsync<SM>();
  // the pivots D = (q' + mu) + B^T A B, rounded as in the walk
  bool fin = true, pos = true, dfin = true;
  for (int j = lane; j < n; j += kWave) {
    const double dk = S.dq[j] + mu, bh = s12[j], D = dk + bh;
    fin = fin && isfinite(D) && fabs(D) > 1e-14 * (fabs(dk) + fabs(bh));
    pos = pos && D > 0.0;
    dfin = dfin && isfinite(S.d[j]);
  }
  if (uv) {
    const double Du = S.Du;
    fin = fin && isfinite(Du) && Du != 0.0;
    pos = pos && Du > 0.0;
    dfin = dfin && isfinite(S.du);
  }
  if (!__all(fin)) return kSweepFail;
  if (!__all(pos)) return kSweepIndef;
  return __all(dfin) ? kSweepPD : kSweepFail;
}

// Direction of negative curvature from the factors the last (indefinite) sweep left:
// at the most negative pivot D_k (ties: the joint nearest the base), v with U^T v = e_k,
// i.e. the outward pass with w = e_k: v_j = 0 below k, v_k = 1 and v_j = -g_j . V_{j-1}
// beyond.  Then v^T (H + mu I) v = D_k < 0.  v into S.d; returns D_k.
template <class SM>
__device__ double neg_curv_dir(SM& S, const Ctx& c, double mu) {
  const int lane = threadIdx.x, n = c.n;
  double best = __builtin_huge_val();
  int bk = n;
  for (int j = lane; j < n; j += kWave) {
    const double D = (S.dq[j] + mu) + S.aux[j];
    if (D < best) {
      best = D;
      bk = j;
    }
    S.d[j] = 0.0;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ob = __shfl_xor(best, o, kWave);
    const int oi = __shfl_xor(bk, o, kWave);
    if (ob < best || (ob == best && oi < bk)) {
      best = ob;
      bk = oi;
    }
  }
  // soft growth: the tip length's pivot, eliminated first, comes after every joint
  const bool uv = c.soft && __builtin_amdgcn_readfirstlane(S.uvar);
  if (uv && S.Du < best) {
    best = S.Du;
    bk = n;
  }
  bsync<SM>();
  if (lane == 0) {
    if (bk == n) {  // along the tip length alone
      S.du = 1.0;
    } else {
      double V0 = 1.0, V1 = S.px[bk], V2 = S.py[bk];
      S.d[bk] = 1.0;
      for (int j = bk + 1; j < n; ++j) {
        const double x = -fma(S.sw2[j], V2, fma(S.sw1[j], V1, S.sw0[j] * V0));
        V0 += x;
        V1 = fma(S.px[j], x, V1);
        V2 = fma(S.py[j], x, V2);
        S.d[j] = x;
      }
      if (uv) S.du = -fma(S.cu2, V2, fma(S.cu1, V1, S.cu0 * V0)) / S.Du;
    }
  }
  bsync<SM>();
  return best;
}

// One equilibrium solve from S.th (in place): descent to a local minimum of the energy.
// Returns the status code.  With delta = pd_shift M_max, each iterate:
//  - factorises H + mu I, mu from max(c_mu |r|_inf, delta), raised tenfold only while the
//    sweep fails (a vanishing pivot) or a positive-definite step does not descend;
//  - converged when rho <= tol and H + delta I is positive definite;
//  - positive definite: the damped Newton step, capped at step_max;
//  - indefinite: d = s v (neg_curv_dir), |d|_inf = step_max, sign so that r.d <= 0, and
//    d_k > 0 when |r.v| <= tol M_max |v|_1 (a slope that a residual within the tolerance
//    could produce: at a converged saddle the sign of r.v is noise);
//  - Armijo backtracking on the energy against alpha r.d (+ alpha^2 d.H d / 2 for a
//    curvature step), skipped once the full step's predicted decrease is below
//    1e-12 M_max, the round-off level of the energy.
template <class SM>
__device__ int solve(SM& S, const Ctx& c, int& iters, double& rho) {
  const int lane = threadIdx.x, n = c.n;
  const KParams& P = c.P;
  const double delta = P.pd_shift * c.Mmax;
  int status = 1;
  if (c.soft && lane == 0) S.ue = S.u;
  bsync<SM>();
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
    // soft growth: u >= 0; on the bound with dPi/du > 0 it is held there and the
    // iteration works on the joints alone
    const bool uv = c.soft && !(S.u <= 0.0 && S.ru > 0.0);
    if (uv) {  // the tip length's residual (N m per link length, like the moments)
      rm = fmax(rm, fabs(S.ru));
      fin = fin && isfinite(S.ru);
    }
    if (c.soft && lane == 0) S.uvar = uv;
    rho = rm / c.Mmax;
    if (!__all(fin) || !isfinite(Pi)) {
      status = 4;
      break;
    }
    const bool small = rho <= P.tol;
    newton_setup(S, c);
    for (int j = lane; j < n; j += kWave) S.b[j] = -S.r[j];
    if (c.soft && lane == 0) S.bu = -S.ru;
    bsync<SM>();
    double mu = fmax(P.c_mu * rm, delta), slope = 0.0, curv = 0.0;
    int mode = 0;  // 1 Newton step, 2 curvature step, 3 converged
    for (int tries = 0; tries < 24; ++tries) {
      if (tries > 0) mu = fmax(10.0 * mu, delta);
      if (lane == 0) S.nsolves += 1.0;
      const int f = chain_solve_seq(S, c, mu, S.b);
      if (f == kSweepFail) continue;
      if (f == kSweepPD) {
        if (small) {
          mode = 3;
          break;
        }
        double s = 0.0;
        for (int j = lane; j < n; j += kWave) s += S.r[j] * S.d[j];
        slope = wsum(s);
        if (uv) slope += S.ru * S.du;
        if (slope < 0.0) {
          mode = 1;
          break;
        }
        continue;
      }
      const double Dk = neg_curv_dir(S, c, mu);
      double vm = 0.0, rv = 0.0, vv = 0.0, v1 = 0.0;
      for (int j = lane; j < n; j += kWave) {
        vm = fmax(vm, fabs(S.d[j]));
        rv += S.r[j] * S.d[j];
        vv += S.d[j] * S.d[j];
        v1 += fabs(S.d[j]);
      }
      vm = wmax(vm);
      rv = wsum(rv);
      vv = wsum(vv);
      v1 = wsum(v1);
      if (uv) {
        const double du = S.du;
        rv += S.ru * du;
        vv += du * du;
        v1 += fabs(du);
        if (vm == 0.0) vm = fabs(du);  // curvature along the tip length alone
      }
      const bool tie = fabs(rv) <= P.tol * c.Mmax * v1;
      const double s = (tie ? 1.0 : (rv > 0.0 ? -1.0 : 1.0)) * P.step_max / vm;
      for (int j = lane; j < n; j += kWave) S.d[j] *= s;
      if (uv) {
        bsync<SM>();
        if (lane == 0) S.du *= s;
      }
      slope = s * rv;
      curv = (Dk - mu * vv) * (s * s);
      if (lane == 0) S.negsteps += 1.0;
      mode = 2;
      break;
    }
    if (mode == 3) {
      status = 0;
      break;
    }
    if (it == P.max_iter) break;
    ++iters;
    if (mode == 0) {
      status = 2;
      break;
    }
    if (mode == 1) {
      double dm = 0.0;
      for (int j = lane; j < n; j += kWave) dm = fmax(dm, fabs(S.d[j]));
      dm = wmax(dm);
      if (dm > P.step_max) {  // the joints' step; the tip length's scales with it
        double f = P.step_max / dm;
        for (int j = lane; j < n; j += kWave) S.d[j] *= f;
        if (uv) {
          bsync<SM>();
          if (lane == 0) S.du *= f;
        }
        slope *= f;
      }
    }
    bsync<SM>();
    const bool skip = -(slope + 0.5 * curv) < 1e-12 * c.Mmax;
    double* tt = S.b;  // trial angles (b is free once the step is known)
    double alpha = 1.0, Pn = 0.0;
    bool acc = false;
    for (int ls = 0; ls < 40; ++ls) {
      for (int j = lane; j < n; j += kWave) tt[j] = S.th[j] + alpha * S.d[j];
      // soft growth: a trial tip length below zero is projected onto u = 0, and the
      // predicted change then takes the tip length's actual move
      double lin = alpha * slope;
      if (c.soft) {
        double ut = S.u;
        if (uv) {
          ut = S.u + alpha * S.du;
          if (ut < 0.0) {
            lin += S.ru * (-S.u - alpha * S.du);
            ut = 0.0;
          }
        }
        if (lane == 0) S.ue = ut;
      }
      bsync<SM>();
      Pn = evaluate(S, c, tt, true);
      if (skip || Pn <= Pi + P.c1 * (lin + 0.5 * alpha * alpha * curv)) {
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
        t[6] = alpha; t[7] = Pn; t[8] = mode; t[9] = S.ncl;
        c.trace_n[0] = row + 1;
      }
    }
    for (int j = lane; j < n; j += kWave) S.th[j] = tt[j];
    if (c.soft && lane == 0) S.u = S.ue;
    Pi = Pn;
    bsync<SM>();
  }
  if (status != 0) {  // poses/contacts of the kept state
    if (c.soft && lane == 0) S.ue = S.u;
    bsync<SM>();
    evaluate(S, c, S.th, false);
  }
  return status;
}

// ---------------------------------------------------------------------------

// The helper wave of a two-wave launch: the obstacle phase of each evaluation the solver
// wave posts (between the two barriers of evaluate()), until the solver wave posts its
// end.  A barrier with no new command also ends the loop: a barrier completes without
// waves that have ended, so the helper never waits on a solver wave that is gone.
// With four waves the helpers split the work by chunks of 64 links: wave 1 the joint law
// of the second half of the chunks, wave 2 the obstacle phase of the first half (first
// region of the contact list), wave 3 that of the second half (second region).
template <class SM>
__device__ void obstacle_helper(SM& S, const Ctx& c0) {
  const int lane = threadIdx.x & (kWave - 1);
  const int role = (int)(threadIdx.x / kWave);
  Ctx c = c0;
  int seen = 0;
  for (;;) {
    __syncthreads();
    const int seq = S.cmd_seq, cmd = S.cmd;
    if (seq == seen || cmd != 1) break;
    seen = seq;
    const int n = S.eval_n, nch = (n + kWave - 1) / kWave, half = (nch + 1) / 2;
    if constexpr (SM::kFour) {
      if (role == 1) {
        c.n = n;
        joint_law_chunks<SM>(S, c, S.eval_trial ? S.b : S.th, S.eval_E != 0, half, nch, lane);
      } else if (role == 2) {
        const int cnt = obstacle_phase(S, c, n, S.eval_last, lane, 0, half, 0);
        if (lane == 0) S.cnt0 = cnt;
      } else {
        const int cnt = obstacle_phase(S, c, n, S.eval_last, lane, half, nch, kMaxC);
        if (lane == 0) S.cnt1 = cnt;
      }
    } else {
      const int cnt = obstacle_phase(S, c, n, S.eval_last, lane, 0, nch, 0);
      if (lane == 0) S.cnt0 = cnt;
    }
    __syncthreads();
  }
}

// Robot b's constants into c.
__device__ __forceinline__ void robot_ctx(Ctx& c, const KParams& P, const KData& D, int b) {
  const int* ii = D.ii + kII * b;
  const double* dd = D.dd + 6 * b;
  c.K = ii[kObsCnt] < kMaxObs ? ii[kObsCnt] : kMaxObs;  // the boundary rejects more
  c.l = dd[0];
  c.R = dd[1];
  c.Mmax = kPi * dd[2] * c.R * c.R * c.R;
  c.arm = 2.0 * c.R + P.Ract;
  c.bx = dd[3];
  c.by = dd[4];
  c.bpsi = dd[5];
  c.tab = D.tables + ii[kTableId];
  c.wr = D.wr;
  c.P = P;
  c.trace = nullptr;
  c.trace_n = D.trace_n;
  c.trace_cap = D.trace_cap;
  c.last_len = c.l;
  c.soft = P.wg > 0.0;
  c.tgt = 1.0;
  c.obs = D.obs + 4 * (size_t)ii[kObsOff];
  c.okind = D.okind + ii[kObsOff];
}

// One robot per workgroup of WAVES waves: the solver wave runs the growth steps, the
// helper waves take the obstacle phase (and with four waves half the joint law) of every
// evaluation.  Per step it records the tip, residual, iterations, status and contact set;
// with D.traj the joint angles after every rec_every-th step (and the last); with D.ckpt
// the state before every ckpt_every-th step (the checkpoints from which the adjoint
// recomputes the states).
// Registers: one wave per robot needs all of a SIMD's (the whole evaluation on one wave);
// with helper waves each wave fits in half, so two waves share a SIMD and a compute unit
// holds twice the robots (told that one wave per SIMD is the target, the compiler pads
// the allocation past half).  The 512-link class holds one robot per compute unit by its
// LDS alone.
template <int NMAX, bool SOFT, int WAVES>
constexpr int kWavesPerEu = (WAVES == 1 || NMAX > 256) ? 1 : 2;

template <int NMAX, bool SOFT, int WAVES>
__global__ __launch_bounds__(4 * kWave) __attribute__((amdgpu_waves_per_eu(
    kWavesPerEu<NMAX, SOFT, WAVES>, kWavesPerEu<NMAX, SOFT, WAVES>))) void rollout_kernel(
    KParams P, KData D, int n_steps) {
  using SMT = Smem<NMAX, (WAVES > 1), (WAVES == 4)>;
  __shared__ SMT S;
  if ((int)blockIdx.x >= D.launch_count) return;
  const int b = D.order[D.launch_first + blockIdx.x];
  const int lane = threadIdx.x;
  const int* ii = D.ii + kII * b;
  const int ntar = ii[kNTarget];
  // a robot at its target length (soft growth: with a full tip link) has nothing to grow
  if (D.skip_done && D.ncur[b] >= ntar && (!SOFT || D.ulast[b] >= kFull)) return;
  Ctx c;
  robot_ctx(c, P, D, b);
  c.soft = SOFT;  // a constant of the launch, so hard growth carries none of the soft code
  c.trace = (b == D.trace_robot) ? D.trace : nullptr;
  double* theta = D.theta + ii[kThetaOff];
  const size_t rec0 = (size_t)ii[kRecOff];
  const int rec_cap = ii[kRecCap];
  if constexpr (WAVES > 1) {
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
    S.pp[j] = D.cover[2 * (size_t)(ii[kCoverOff] + j)];
    S.pm[j] = D.cover[2 * (size_t)(ii[kCoverOff] + j) + 1];
  }
  const long long t_begin = clock64();  // this robot's time in the launch (for scheduling)
  const long long w_begin = wall_clock64();  // and in seconds (constant-rate counter)
  int n = D.ncur[b];
  int t = D.tcur[b];
  if (lane == 0) {
    S.jevals = 0.0;
    S.nsolves = 0.0;
    S.negsteps = 0.0;
    S.u = c.soft ? D.ulast[b] : 1.0;
    S.ue = S.u;
  }
  for (int j = lane; j < n; j += kWave) S.th[j] = theta[j];
  bsync<SMT>();
  for (int step = 0; step < n_steps && t < rec_cap; ++step, ++t) {
    if (D.ckpt && t % D.ckpt_every == 0) {
      double* row = D.ckpt + ((size_t)b * D.n_ckpt + t / D.ckpt_every) * D.n_max;
      for (int j = lane; j < D.n_max; j += kWave) row[j] = j < n ? S.th[j] : 0.0;
    }
    int st_worst = 0, its = 0;
    double rho = 0.0;
    // hard growth: append a link when short of the target.  Soft growth: append only
    // when the tip link is full (its excess starts the new link); done with the target
    // link count and a full tip link.
    bool grow;
    if (c.soft) {
      const double u = S.u;  // uniform: every lane reads the value lane 0 wrote
      if (n == 0 || (u >= kFull && n < ntar)) {
        ++n;
        if (lane == 0) {
          S.th[n - 1] = 0.0;
          S.u = n == 1 ? 0.0 : fmax(u - 1.0, 0.0);
        }
      }
      bsync<SMT>();
      grow = !(n == ntar && S.u >= kFull);
    } else {
      grow = n < ntar;
      if (grow) {
        ++n;
        if (lane == 0) S.th[n - 1] = 0.0;
        bsync<SMT>();
      }
    }
    if (grow) {
      c.n = n;
      for (int s = 1; s <= P.substeps; ++s) {
        for (;;) {
          if (c.soft) {
            double tg = (double)t + (double)s / (double)P.substeps - (double)(n - 1);
            c.tgt = (n == ntar && tg > 1.0) ? 1.0 : tg;
          } else {
            c.last_len = c.l * (double)s / (double)P.substeps;
          }
          c.step = t;
          c.sub = s;
          int st = solve(S, c, its, rho);
          st_worst = st > st_worst ? st : st_worst;
          // soft growth: a tip link grown longer than a link is split, its first l
          // staying as link n - 1 and the rest starting a new link at zero angle; the
          // sub-step is solved again
          if (!(c.soft && n < ntar && S.u > 1.0 + 1e-12)) break;
          bsync<SMT>();
          if (lane == 0) {
            S.th[n] = 0.0;
            S.u = S.u - 1.0;
          }
          ++n;
          c.n = n;
          bsync<SMT>();
        }
      }
    } else {
      c.n = n;
      if (!c.soft) c.last_len = c.l;
      st_worst = -1;
      if (n > 0) {
        if (c.soft && lane == 0) S.ue = S.u;
        bsync<SMT>();
        evaluate(S, c, S.th, false);
      }
    }
    // record the state after this step
    const size_t bt = rec0 + t;
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
      D.tiplen[bt] = n == 0 ? 0.0 : (c.soft ? S.u * c.l : c.last_len);
    }
    if (D.traj && ((t + 1) % D.rec_every == 0 || t == rec_cap - 1)) {
      double* row = D.traj + ((size_t)b * D.n_rec + t / D.rec_every) * D.n_max;
      for (int j = lane; j < D.n_max; j += kWave) row[j] = j < n ? S.th[j] : 0.0;
    }
    bsync<SMT>();
  }
  for (int j = lane; j < n; j += kWave) theta[j] = S.th[j];
  if (lane == 0) {
    D.ncur[b] = n;
    D.tcur[b] = t;
    if (c.soft) D.ulast[b] = S.u;
    D.jevals[b] += S.jevals;
    D.nsolves[b] += S.nsolves;
    D.negsteps[b] += S.negsteps;
    D.cycles[b] += (double)(clock64() - t_begin);
    D.wtime[b] += (double)(wall_clock64() - w_begin) * D.wall_period;
  }
  if constexpr (WAVES > 1) {
    if (lane == 0) {
      S.cmd = 2;
      S.cmd_seq += 1;
    }
    __syncthreads();  // releases the helper waves, which then end
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the growth step.  For L = sum_t w_t |tip_t - goal|^2 over converged
// states (r_t(theta_t; p) = 0, independent of the previous state):
//   dL/dp = - sum_t lam_t . dr_t/dp,  H_t lam_t = w_t dL_t/dtheta,
// H_t the exact Hessian, solved by the same sweep with mu = 0.  An sPAM's pressure P_s
// and its ends s0, s1 enter r only through the coverage of the joints it spans:
//   dq_j/dP+-_j = -+arm G(eps+-_j),  w_sj = |[s0, s1] ^ [j l, (j+1) l]| / l.
// The launch covers the steps [t0, t0 + T): weights[t] weighs step t0 + t, whose
// joint angles are row t of traj ([B][traj_rows][n_max]); weights == null takes the
// current state (D.theta) with weight 1.  A rollout recomputed from checkpoints runs one
// launch per segment: each lane's running sums (its sPAM's three derivatives, the loss,
// the status) continue from where the previous segment left them in part (unless
// part.first) and are stored there again (unless part.last, which commits them), so the
// sums are added in the same order as in a single launch and agree bit for bit.
// status[b]: bit 0 an adjoint system was singular or its contact list overflowed (that
// step's term is left out), bit 1 a weighted step had not converged in the rollout (its
// term is the derivative of the branch it sits on).
template <int NMAX>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 1))) void grad_kernel(
    KParams P, KData D, const double* goal, const double* weights, int T, int t0,
    const double* traj, int traj_rows, GradPart part, double* dP, double* ds0, double* ds1,
    double* loss, int* status) {
  __shared__ Smem<NMAX, false> S;
  if ((int)blockIdx.x >= D.launch_count) return;
  const int b = D.order[D.launch_first + blockIdx.x], lane = threadIdx.x;
  const int* ii = D.ii + kII * b;
  Ctx c;
  robot_ctx(c, P, D, b);
  const int ntar = ii[kNTarget];
  if (lane == 0) S.res_ok = 0;  // staged by the first evaluation
  for (int j = lane; j < ntar; j += kWave) {
    S.pp[j] = D.cover[2 * (size_t)(ii[kCoverOff] + j)];
    S.pm[j] = D.cover[2 * (size_t)(ii[kCoverOff] + j) + 1];
  }
  const int soff = ii[kSpamOff], ns = ii[kSpamCnt];
  const double gx = goal[2 * b], gy = goal[2 * b + 1];
  double aP = 0.0, a0 = 0.0, a1 = 0.0, Lsum = 0.0;  // this lane's sPAM (lane < ns)
  int st = 0;
  double* mine = part.sums ? part.sums + 3 * ((size_t)b * kWave + lane) : nullptr;
  if (!part.first) {
    aP = mine[0];
    a0 = mine[1];
    a1 = mine[2];
    Lsum = part.loss[b];
    st = part.status[b];
  }
  int taken = D.tcur[b] - t0;  // steps of this range the robot has taken
  taken = taken < 0 ? 0 : (taken < T ? taken : T);
  for (int t = 0; t < (weights ? taken : 1); ++t) {
    const double wt = weights ? weights[t] : 1.0;
    if (wt == 0.0) continue;
    int n, tg;  // links, and the global step whose state this is
    if (weights) {
      tg = t0 + t;
      n = tg + 1 < ntar ? tg + 1 : ntar;
      for (int j = lane; j < n; j += kWave)
        S.th[j] = traj[((size_t)b * traj_rows + t) * D.n_max + j];
    } else {
      tg = D.tcur[b] - 1;
      n = D.ncur[b];
      for (int j = lane; j < n; j += kWave) S.th[j] = D.theta[ii[kThetaOff] + j];
    }
    if (n == 0) continue;
    if (tg >= 0) {
      const int fs = D.status[(size_t)ii[kRecOff] + tg];
      if (fs > 0) st |= 2;
    }
    c.n = n;
    __syncthreads();
    evaluate(S, c, S.th, false);
    const double ex = S.px[n] - gx, ey = S.py[n] - gy;
    Lsum += wt * (ex * ex + ey * ey);
    if (S.overflow) {  // contact list truncated: the Hessian would be wrong
      st |= 1;
      continue;
    }
    for (int j = lane; j < n; j += kWave) {
      const double vx = -(S.py[n] - S.py[j]), vy = S.px[n] - S.px[j];
      S.b[j] = 2.0 * wt * (ex * vx + ey * vy);
    }
    newton_setup(S, c);
    if (chain_solve_seq(S, c, 0.0, S.b) == kSweepFail) {
      st |= 1;
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
  if (!part.last) {
    mine[0] = aP;
    mine[1] = a0;
    mine[2] = a1;
    if (lane == 0) {
      part.loss[b] = Lsum;
      part.status[b] = st;
    }
    return;
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

// Host-side check before a launch: every array the kernels write or read per robot is
// present (a missing buffer is reported as an error instead of reaching the device).
static bool state_complete(const KData& D) {
  return D.ii && D.dd && D.cover && D.okind && D.obs && D.tables && D.wr && D.order && D.theta &&
         D.ncur && D.tcur && D.tip && D.rho && D.iters && D.status && D.ncont && D.chash &&
         D.maxpen && D.tiplen && D.ulast && D.jevals && D.nsolves && D.negsteps &&
         D.cycles && D.wtime;
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
                       const double* weights, int T, int t0, const double* traj, int traj_rows,
                       const GradPart& part, double* dP, double* ds0, double* ds1, double* loss,
                       int* status, int nmax_class, hipStream_t stream) {
  if (D.launch_count <= 0) return hipSuccess;
  if ((!part.first || !part.last) && !(part.sums && part.loss && part.status))
    return hipErrorInvalidValue;
  if (!state_complete(D) || !goal || !loss || (D.n_spam > 0 && !(dP && ds0 && ds1)) ||
      (weights && !traj))
    return hipErrorInvalidValue;
  dim3 grid(D.launch_count), block(kWave);
#define VS_GRAD(NM)                                                                          \
  hipLaunchKernelGGL((grad_kernel<NM>), grid, block, 0, stream, P, D, goal, weights, T, t0, \
                     traj, traj_rows, part, dP, ds0, ds1, loss, status)
  if (nmax_class == 64)
    VS_GRAD(64);
  else if (nmax_class == 128)
    VS_GRAD(128);
  else if (nmax_class == 256)
    VS_GRAD(256);
  else if (nmax_class == 512)
    VS_GRAD(512);
  else
    return hipErrorInvalidValue;
#undef VS_GRAD
  return hipGetLastError();
}

// Zero the state and records of every robot (a kernel rather than memsets, so that
// a captured graph holds no memset nodes).
__global__ void reset_kernel(KData D) {
  const size_t B = D.n_inst, stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = i0; i < (size_t)D.theta_len; i += stride) D.theta[i] = 0.0;
  for (size_t i = i0; i < (size_t)D.rec_len * 3; i += stride) D.tip[i] = 0.0;
  for (size_t i = i0; i < (size_t)D.rec_len; i += stride) {
    D.rho[i] = 0.0;
    D.iters[i] = 0;
    D.status[i] = 0;
    D.ncont[i] = 0;
    D.chash[i] = 0ull;
    D.maxpen[i] = 0.0;
    D.tiplen[i] = 0.0;
  }
  for (size_t i = i0; i < B; i += stride) {
    D.ncur[i] = 0;
    D.tcur[i] = 0;
    D.ulast[i] = 0.0;
    D.jevals[i] = 0.0;
    D.nsolves[i] = 0.0;
    D.negsteps[i] = 0.0;
    D.cycles[i] = 0.0;
    D.wtime[i] = 0.0;
  }
}

// Zero the state and records of the robots in slots[0..count) (one block per robot).
__global__ void slot_reset_kernel(KData D, const int* slots, int count) {
  if ((int)blockIdx.x >= count) return;
  const size_t b = (size_t)slots[blockIdx.x];
  const int* ii = D.ii + kII * b;
  for (int j = threadIdx.x; j < ii[kNTarget]; j += blockDim.x) D.theta[ii[kThetaOff] + j] = 0.0;
  for (int t = threadIdx.x; t < ii[kRecCap]; t += blockDim.x) {
    const size_t bt = (size_t)ii[kRecOff] + t;
    D.tip[3 * bt] = 0.0;
    D.tip[3 * bt + 1] = 0.0;
    D.tip[3 * bt + 2] = 0.0;
    D.rho[bt] = 0.0;
    D.iters[bt] = 0;
    D.status[bt] = 0;
    D.ncont[bt] = 0;
    D.chash[bt] = 0ull;
    D.maxpen[bt] = 0.0;
    D.tiplen[bt] = 0.0;
  }
  if (threadIdx.x == 0) {
    D.ncur[b] = 0;
    D.tcur[b] = 0;
    D.ulast[b] = 0.0;
    D.jevals[b] = 0.0;
    D.nsolves[b] = 0.0;
    D.negsteps[b] = 0.0;
    D.cycles[b] = 0.0;
    D.wtime[b] = 0.0;
  }
}

// Start of a recomputed segment: every robot's state from checkpoint q (the state before
// step q ce) into the segment state of Dseg (one block per robot); the segment's records
// start at 0.  A robot whose rollout had not reached step q ce (tcur) has no such
// checkpoint and is marked as having taken the whole segment, so that it does nothing.
// Dseg.ii is the handle's robot rows with the record fields of the segment buffers.
__global__ void seg_load_kernel(KData Dseg, const int* ii_handle, const double* ckpt,
                                const int* tcur, int n_ckpt, int q, int ce) {
  const int b = blockIdx.x;
  if (b >= Dseg.n_inst) return;
  int* iis = const_cast<int*>(Dseg.ii) + kII * (size_t)b;
  const int* iih = ii_handle + kII * (size_t)b;
  const int ntar = iih[kNTarget];
  const bool have = tcur[b] > q * ce;
  const int n = !have ? 0 : (q * ce < ntar ? q * ce : ntar);
  const double* src = ckpt + ((size_t)b * n_ckpt + q) * Dseg.n_max;
  double* th = Dseg.theta + (size_t)b * Dseg.n_max;
  for (int j = threadIdx.x; j < Dseg.n_max; j += blockDim.x) th[j] = j < n ? src[j] : 0.0;
  if (threadIdx.x < kII) {
    const int f = threadIdx.x;
    iis[f] = f == kThetaOff ? b * Dseg.n_max
           : f == kRecOff   ? b * ce
           : f == kRecCap   ? ce
                            : iih[f];
  }
  if (threadIdx.x == 0) {
    Dseg.ncur[b] = n;
    Dseg.tcur[b] = have ? 0 : ce;
    Dseg.jevals[b] = 0.0;
    Dseg.nsolves[b] = 0.0;
    Dseg.negsteps[b] = 0.0;
    Dseg.cycles[b] = 0.0;
    Dseg.wtime[b] = 0.0;
  }
}

hipError_t launch_seg_load(const KData& Dseg, const int* ii_handle, const double* ckpt,
                           const int* tcur, int n_ckpt, int q, int ce, hipStream_t stream) {
  if (!state_complete(Dseg) || !ii_handle || !ckpt || !tcur) return hipErrorInvalidValue;
  hipLaunchKernelGGL(seg_load_kernel, dim3(Dseg.n_inst), dim3(64), 0, stream, Dseg, ii_handle,
                     ckpt, tcur, n_ckpt, q, ce);
  return hipGetLastError();
}

hipError_t launch_slot_reset(const KData& D, const int* slots, int count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (!state_complete(D) || !slots) return hipErrorInvalidValue;
  hipLaunchKernelGGL(slot_reset_kernel, dim3(count), dim3(256), 0, stream, D, slots, count);
  return hipGetLastError();
}

hipError_t launch_reset(const KData& D, hipStream_t stream) {
  if (!state_complete(D)) return hipErrorInvalidValue;
  const size_t work = (size_t)(D.rec_len * 3 > D.theta_len ? D.rec_len * 3 : D.theta_len);
  const size_t blocks = (work + 255) / 256 < 4096 ? (work + 255) / 256 : 4096;
  hipLaunchKernelGGL(reset_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     stream, D);
  return hipGetLastError();
}

// Robots (workgroups) of one chain-length class resident per compute unit, with 1, 2 or 4
// waves per robot.
hipError_t rollout_occupancy(int nmax_class, int waves, int* per_cu) {
  const int block = waves * kWave;
#define VS_OCC(NM)                                                                            \
  return waves == 4   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                          \
                          per_cu, rollout_kernel<NM, false, 4>, block, 0)                     \
         : waves == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                          \
                          per_cu, rollout_kernel<NM, false, 2>, block, 0)                     \
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(                          \
                          per_cu, rollout_kernel<NM, false, 1>, block, 0);
  if (waves != 1 && waves != 2 && waves != 4) return hipErrorInvalidValue;
  if (nmax_class == 64) VS_OCC(64)
  if (nmax_class == 128) VS_OCC(128)
  if (nmax_class == 256) VS_OCC(256)
  if (nmax_class == 512) VS_OCC(512)
#undef VS_OCC
  return hipErrorInvalidValue;
}

// host-side launcher (instantiated for the supported chain lengths)
hipError_t launch_rollout(const KParams& P, const KData& D, int n_steps, int nmax_class,
                          int waves, hipStream_t stream) {
  if (D.launch_count <= 0) return hipSuccess;
  if (!state_complete(D)) return hipErrorInvalidValue;
  if (D.traj && D.rec_every < 1) return hipErrorInvalidValue;
  if (D.ckpt && D.ckpt_every < 1) return hipErrorInvalidValue;
  if (waves != 1 && waves != 2 && waves != 4) return hipErrorInvalidValue;
  dim3 grid(D.launch_count), block(waves * kWave);
  const bool soft = P.wg > 0.0;
#define VS_ROLL1(NM, SO, W) \
  hipLaunchKernelGGL((rollout_kernel<NM, SO, W>), grid, block, 0, stream, P, D, n_steps);
#define VS_ROLL(NM)                                          \
  if (soft) {                                                \
    if (waves == 4) { VS_ROLL1(NM, true, 4) }                \
    else if (waves == 2) { VS_ROLL1(NM, true, 2) }           \
    else { VS_ROLL1(NM, true, 1) }                           \
  } else {                                                   \
    if (waves == 4) { VS_ROLL1(NM, false, 4) }               \
    else if (waves == 2) { VS_ROLL1(NM, false, 2) }          \
    else { VS_ROLL1(NM, false, 1) }                          \
  }
  if (nmax_class == 64) {
    VS_ROLL(64)
  } else if (nmax_class == 128) {
    VS_ROLL(128)
  } else if (nmax_class == 256) {
    VS_ROLL(256)
  } else if (nmax_class == 512) {
    VS_ROLL(512)
  } else {
    return hipErrorInvalidValue;
  }
#undef VS_ROLL
#undef VS_ROLL1
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free adjoint (vine_sim_grad_noalloc): one static
// array per device, held until the process ends.  In host code the array's name is a
// host-side stand-in, not a device address, so its address on each device is looked up
// once (with that device current) and kept; launches and copies use that address only.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Address of the current device's scratch (looked up on the first call for a device).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace vs
