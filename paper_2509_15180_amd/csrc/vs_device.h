// vs_device.h -- device-side data layout shared by the host launcher and the
// gfx950 kernels of the vine-robot simulator.
#pragma once
#include <stdint.h>

namespace vs {

constexpr int kWave = 64;
constexpr int kMaxObs = 128;  // obstacles per robot (the boundary's VINE_MAX_OBSTACLES)
// bytes of the static device scratch of the allocation-free adjoint (per device)
constexpr unsigned long long kScratchBytes = 128ull << 20;

// sPAM force law G(eps) = F_t / P_act (Sec. 3.1, Eq. 1d) on [0, eps_max] as a
// piecewise Chebyshev series: pieces [b_k, b_{k+1}] with b_k = eps_max (k/P)^2
// (graded toward eps = 0, where G changes fastest), degree D per piece.
constexpr int kSpamPieces = 24;
constexpr int kSpamDeg = 20;

struct SpamTable {
  static constexpr bool kHasSlope = true;
  double l0;                                 // actuator unit length (= link length)
  double emax;                               // slack strain eps(m = 1/2)
  double G0;                                 // G(0)
  double bnd[kSpamPieces + 1];               // piece boundaries in eps
  double cum[kSpamPieces + 1];               // int_0^{b_k} G
  double c[kSpamPieces][kSpamDeg + 1];       // G      = sum' c_j T_j(x)   (c_0 halved)
  double dc[kSpamPieces][kSpamDeg + 1];      // dG/dx  = sum' dc_j T_j(x)  (dc_0 halved)
  double ic[kSpamPieces][kSpamDeg + 2];      // int_{b_k}^{eps} G dx' = sum' ic_j T_j(x), 0 at x=-1
};

// The wrinkling moment fraction h (Eq. 2) above the onset and its integral: in
// u = sqrt(x - theta_on) on [0, sqrt(pi - theta_on)], pieces of equal width du; on piece
// k the integrand 2 u h(theta_on + u^2) is a Chebyshev series whose antiderivative (zero
// at the piece's left end, variable t in [-1, 1]) is stored, and h(theta_on + u^2) and
// its slope dh/dx are two more series.  Both are analytic in u: the bend angle gamma_0
// grows like u at the onset, and h - h(theta_on) starts at u^2.
constexpr int kIhPieces = 32;
constexpr int kIhDeg = 16;

struct WrTable {
  double th_on;       // 2 asin(eps_crit)
  double umax;        // sqrt(pi - th_on)
  double du;          // piece width in u
  double h_pi;        // h(pi)
  double ih_pi;       // int_0^pi h
  double cum[kIhPieces + 1];          // int_0^{x(u_k)} h at piece boundaries
  double ic[kIhPieces][kIhDeg + 2];   // per piece: antiderivative series in t
  double hc[kIhPieces][kIhDeg + 1];   // per piece: h(th_on + u^2) itself, series in t
  double dhc[kIhPieces][kIhDeg + 1];  // per piece: dh/dx at th_on + u^2, series in t
};

// Solver and model constants passed by value to the kernels.
struct KParams {
  double epsc, kc, tol, c_mu, step_max, c1, Ract;
  double pd_shift;    // delta / M_max: converged states have H + delta I positive definite
  double wg;          // growth stiffness (N/m): 0 hard growth, > 0 soft growth
  int max_iter, substeps;
};

// Fields of the per-robot integer row ii[b][kII].
constexpr int kII = 10;
enum : int {
  kNTarget = 0,   // target link count
  kObsOff = 1,    // first obstacle (rows of obs, okind)
  kObsCnt = 2,
  kTableId = 3,   // sPAM force-law table
  kCoverOff = 4,  // first joint row of cover
  kSpamOff = 5,   // first sPAM record
  kSpamCnt = 6,
  kThetaOff = 7,  // first element of the robot's joint angles in theta
  kRecOff = 8,    // first element of its per-step records (tip row = 3 x that)
  kRecCap = 9     // per-step records it holds (steps it can take)
};

// Per-robot and per-simulation device arrays (structure of arrays).
struct KData {
  int n_inst;
  int n_max;          // largest target link count (row length of traj, ckpt)
  int t_max;          // recorded steps per robot (rows of traj)
  long long theta_len, rec_len;  // elements of theta and of each per-step record array
  int skip_done;      // robots at their target length do nothing (serving)
  // inputs
  const int* ii;      // [B][kII], fields above
  const double* dd;   // [B][6]: l, R, P_vine, base_x, base_y, base_heading
  const double* cover;// [sum n][2]: P+_j, P-_j
  const int* okind;   // [O]
  const double* obs;  // [O][4]: cx, cy, a, b
  const double* spam; // [S][4]: s_start, s_end, side, pressure (as given at create)
  int n_spam;
  const SpamTable* tables;
  const WrTable* wr;
  // robots of the current launch: order[launch_first + blockIdx.x], launch_count blocks
  const int* order;
  int launch_first, launch_count;
  // state
  double* theta;      // robot b: [ii[b][kThetaOff], + n_target)
  int* ncur;          // [B]
  int* tcur;          // [B] steps recorded so far
  double* ulast;      // [B] soft growth: the tip link's length in link lengths
  // per-step records, robot b at [ii[b][kRecOff], + ii[b][kRecCap])...
  double* tip;        // ...times 3 (x, y, heading)
  double* rho;
  int* iters;
  int* status;
  int* ncont;
  unsigned long long* chash;
  double* maxpen;
  double* tiplen;     // the tip link's length
  double* traj;       // [B][n_rec][N] or null: joint angles after every rec_every-th step
  int rec_every, n_rec;  // (row t / rec_every after step t; the last step always)
  double* ckpt;       // [B][n_ckpt][N] or null: the state before every ckpt_every-th step
  int ckpt_every, n_ckpt;
  // work counters per robot (accumulated over calls)
  double* jevals;     // [B] sum over residual/energy evaluations of the link count
  double* nsolves;    // [B] factorisations of H + mu I
  double* negsteps;   // [B] steps along negative curvature
  double* cycles;     // [B] shader-clock cycles spent in rollout launches since the reset
  double* wtime;      // [B] seconds spent in rollout launches since the reset
  double wall_period; // seconds per tick of the device's constant-rate wall clock
  // solver trace of one robot (diagnostics): rows of kTraceCols doubles
  int trace_robot;    // -1: off
  int trace_cap;      // rows
  double* trace;      // [cap][kTraceCols]; trace_n[0] counts rows written
  int* trace_n;
};
// Running sums of the adjoint between the launches of a segmented (checkpointed)
// gradient: per robot and lane its sPAM's three derivatives, and the loss and status.
struct GradPart {
  double* sums;   // [B][kWave][3] or null (single launch)
  double* loss;   // [B]
  int* status;    // [B]
  int first, last;  // start from zero; commit to the outputs
};

constexpr int kTraceCols = 10;  // step, substep, iter, rho, mu, slope, alpha, Pi, mode, ncontacts

}  // namespace vs
