/*
 * vinesim.h -- C ABI of the MI355X (gfx950) vine-robot simulator: the batched
 * quasi-static growth step of a soft growing robot (arXiv 2509.15180).
 *
 * Model (paper section / equation):
 *   - a robot is a chain of rigid links of length l in minimal coordinates, the
 *     relative joint angles theta (Sec. 4.1);
 *   - each joint carries the wrinkling-based restoring moment of the inflated body
 *     (Sec. 3.2, Eq. 2) and the moment of the sPAM actuators that cover it
 *     (Sec. 3.1, Eq. 1; Sec. 3.3, Eq. 3: strain eps = (2R + R_act) theta / l);
 *   - one growth step appends a link and brings the chain to a minimum-energy state
 *     of Eq. 4 (an argmin) read as a potential energy: joint energies plus a penalty
 *     k_c/2 pen^2 on every penetration of the body into an obstacle (Alg. 1).  The
 *     state reached is the local minimum that a damped descent from the previous
 *     state (new link straight) finds; stationary points that are not minima
 *     (saddles, such as a straight body pushed head-on into an obstacle) are left
 *     along their negative curvature.
 *
 * Units are SI throughout: metres, pascals, radians, newtons.
 *
 * Conventions
 *   - Every entry point returns 0 on success or a negative VINE_E* code.  A call
 *     that fails leaves the simulation state unchanged; vine_sim_last_error()
 *     then describes the failure.
 *   - Numerical non-convergence is NOT a call error: it is reported per instance
 *     and per step in the STATUS field.
 *   - Pointers marked "host" are read during the call only and may be freed
 *     on return.  The library owns all device memory it allocates; the handle
 *     frees it in vine_sim_destroy().
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     asynchronously on it; synchronise the stream before reading results on the
 *     host through a caller-owned buffer.
 *   - One handle must not be used from two threads at once.  Several handles may
 *     share a device.
 */
#ifndef VINESIM_H
#define VINESIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define VINE_OK 0
#define VINE_EINVAL (-1)    /* a size, pressure or geometry is NaN, negative or out of range */
#define VINE_ENOMEM (-2)    /* device or host allocation failed */
#define VINE_EDEVICE (-3)   /* a HIP runtime call failed */
#define VINE_ESTATE (-4)    /* call not valid in the handle's current state */
#define VINE_ECAPACITY (-5) /* more links, obstacles or sPAMs per robot than supported */

/* per-step status codes in the STATUS field */
#define VINE_ST_CONVERGED 0   /* max_j |r_j| / M_max <= tol and H + pd_shift M_max I positive definite */
#define VINE_ST_MAXITER 1     /* iteration limit reached */
#define VINE_ST_NODESCENT 2   /* no descent direction / line search failed */
#define VINE_ST_CAPACITY 3    /* more simultaneous disk/obstacle contacts than the contact list holds */
#define VINE_ST_NONFINITE 4   /* a non-finite residual or energy appeared */
#define VINE_ST_DONE (-1)     /* the robot had already reached its target length */

/* Simulation-wide constants.  Defaults (vine_params_default): R_c = 5 mm,
 * R_act = 17.18 mm, a = 1e-4 (Sec. 3.1); eps_crit = 0.01 (Sec. 3.2: fitted in the
 * paper, value not printed); k_c = 1e4 N/m; tol = 1e-10; pd_shift = 1e-8 /rad;
 * max_iter = 500; growth_substeps = 2; c_mu = 1 /rad; step_max = 0.05 rad;
 * armijo_c1 = 1e-4; growth_stiffness = 0 (hard growth).
 *
 * The descent (one growth sub-step): at each iterate the exact Hessian H of the energy
 * is factorised as H + mu I = U D U^T by a Riccati sweep that eliminates the joints from
 * the tip (O(n) for any number of contacts; its pivots D give the inertia), with
 * mu = max(c_mu max_j |r_j|, pd_shift M_max) raised tenfold while a pivot vanishes.
 * Converged: max_j |r_j| / M_max <= tol and every pivot at mu = pd_shift M_max positive.
 * Positive definite: the step (H + mu I) d = -r, |d|_inf capped at step_max.  Otherwise a
 * step of length step_max along v with U^T v = e_k, k the most negative pivot.  Armijo
 * backtracking on the energy. */
typedef struct vine_params {
  double R_c;            /* sPAM constriction radius (m), Eq. 1 */
  double R_act;          /* sPAM tube radius (m), Eq. 1c */
  double a_corr;         /* sPAM correction factor a (dimensionless), Eq. 1b */
  double eps_crit;       /* critical wrinkling strain, Eq. 2b */
  double k_c;            /* contact penalty stiffness (N/m), Eq. 4 contact term */
  double tol;            /* convergence: max_j |r_j| / (pi P R^3) <= tol */
  double c_mu;           /* damping per unit residual, mu = c_mu max_j |r_j| (1/rad) */
  double step_max;       /* cap on the joint-space step per iteration (rad) */
  double armijo_c1;      /* sufficient-decrease constant of the line search */
  double pd_shift;       /* delta / M_max (1/rad): a stationary state is accepted when
                            H + delta I is positive definite */
  double growth_stiffness; /* w_g (N/m), Eq. 4's growth term.  0: hard growth, each step
                            appends a link whose length is prescribed (l s / S at sub-step
                            s).  > 0: soft growth, the tip link's length u l is a variable
                            of the minimisation under the term (w_g/2) (l (tgt - u))^2,
                            whose target tgt rises by one link length per step
                            (tgt = t + s/S - (n - 1) at sub-step s of step t, at most 1
                            once the robot has its target link count); a link is appended
                            only when the tip link is full (u >= 1, its excess starting the
                            new one), a tip link grown longer than a link within a sub-step
                            is split and the sub-step solved again, and the robot is done
                            with its target link count and a full tip link.  A blocked
                            tip thus stops while the growth force builds (Sec. 4.1).  The
                            tip length's residual is in N m per link length, like the
                            joints' moments, and the step cap applies to the joints */
  int32_t max_iter;      /* iterations per equilibrium solve */
  int32_t growth_substeps; /* sub-steps in which an appended link reaches full length */
  int32_t reserved;
} vine_params;

/* One robot.  n_links: target link count (1..VINE_MAX_LINKS).  Its sPAMs are
 * spams[spam_offset .. spam_offset + spam_count) and its obstacles
 * obstacles[obs_offset .. obs_offset + obs_count). */
typedef struct vine_instance {
  int32_t n_links;
  int32_t spam_offset, spam_count;
  int32_t obs_offset, obs_count;
  int32_t reserved;
  double link_len;       /* l (m), also the sPAM unit length l0 */
  double tube_radius;    /* R_vine (m) */
  double body_pressure;  /* P_vine (Pa) */
  double base_x, base_y; /* base position (m) */
  double base_heading;   /* heading of the first link at zero joint angle (rad) */
} vine_instance;

/* An sPAM actuator along the body (Sec. 3.1).  It covers arc length
 * [s_start, s_end] from the base; joint j takes the pressure-weighted fraction of
 * link j = [j l, (j+1) l] it covers.  side = +1 pulls theta positive, -1 negative. */
typedef struct vine_spam {
  double s_start, s_end; /* m, 0 <= s_start <= s_end */
  double side;           /* +1 or -1 */
  double pressure;       /* P_act (Pa), >= 0 */
} vine_spam;

/* An obstacle.  kind 0: circle, centre (cx, cy), radius a (b unused).
 * kind 1: axis-aligned rectangle, centre (cx, cy), half-width a, half-height b. */
typedef struct vine_obstacle {
  int32_t kind;
  int32_t reserved;
  double cx, cy, a, b;
} vine_obstacle;

#define VINE_MAX_LINKS 512   /* links per robot */
#define VINE_MAX_OBSTACLES 128
#define VINE_MAX_SPAMS 64

/* Fields for vine_sim_read.  T = the longest target length (steps recorded per
 * robot), N = the largest n_links, B = the number of robots.  Row-major. */
typedef enum vine_field {
  VINE_F_THETA = 0,    /* double [B][N]    joint angles (0 beyond the current length) */
  VINE_F_NLINKS = 1,   /* int32  [B]       current link count */
  VINE_F_TIP = 2,      /* double [B][T][3] tip x, y, heading after each step */
  VINE_F_RHO = 3,      /* double [B][T]    scaled residual at the end of each step */
  VINE_F_ITERS = 4,    /* int32  [B][T]    Newton iterations spent in each step */
  VINE_F_STATUS = 5,   /* int32  [B][T]    VINE_ST_* of each step */
  VINE_F_NCONTACT = 6, /* int32  [B][T]    (link, obstacle) pairs in contact after each step */
  VINE_F_CHASH = 7,    /* uint64 [B][T]    order-free hash of that contact set */
  VINE_F_MAXPEN = 8,   /* double [B][T]    deepest penetration after each step (m) */
  VINE_F_TRAJ = 9,     /* double [B][R][N] joint angles after every record_every-th step (row
                          t / record_every after step t) and after the last step T - 1,
                          R = ceil(T / record_every), as last recorded */
  VINE_F_JEVALS = 10,  /* double [B]       work counter: sum over residual evaluations of the
                          link count (since create or the last reset) */
  VINE_F_NSOLVES = 11, /* double [B]       work counter: linear solves of the Newton system */
  VINE_F_CYCLES = 12,  /* double [B]       shader-clock cycles each robot's wave spent in rollout
                          launches since the reset (what vine_sim_tune_order sorts by) */
  VINE_F_NEGSTEPS = 13, /* double [B]      work counter: steps along negative curvature */
  VINE_F_CKPT = 14,    /* double [B][C][N] checkpoints: row q is the state before step
                          q ckpt_every (joint angles, 0 beyond the link count then),
                          C = ceil(T / ckpt_every) */
  VINE_F_TIME = 15,    /* double [B]       seconds each robot's workgroup spent in rollout
                          launches since the reset (device wall clock): its rollout latency
                          once it runs */
  VINE_F_TIPLEN = 16   /* double [B][T]    length of the tip link after each step (m): l
                          in hard growth; the variable u l in soft growth */
} vine_field;

typedef struct vine_sim vine_sim;

/* Fill p with the defaults listed above. */
void vine_params_default(vine_params* p);

/* Create a simulation of n_inst robots at zero length on the current HIP device.
 * params, inst, spams and obstacles are host arrays (copied).  Builds the sPAM
 * force-law table (Sec. 3.1, Eq. 1 solved for every distinct link length) and each
 * joint's sPAM coverage.  Errors: VINE_EINVAL (NaN or non-positive sizes or
 * pressures, side not +-1, s_start > s_end, unknown obstacle kind, n_inst < 1,
 * offsets out of range), VINE_ECAPACITY (n_links > VINE_MAX_LINKS, more than
 * VINE_MAX_OBSTACLES obstacles or VINE_MAX_SPAMS sPAMs on one robot), VINE_ENOMEM,
 * VINE_EDEVICE.  *out is set only on success. */
int32_t vine_sim_create(const vine_params* params, const vine_instance* inst, int32_t n_inst,
                        const vine_spam* spams, int32_t n_spams, const vine_obstacle* obstacles,
                        int32_t n_obstacles, vine_sim** out);

/* Advance every robot that is shorter than its target by n_steps growth steps
 * (Alg. 1 repeated): append a link at zero angle, then, for each growth sub-step,
 * solve the equilibrium.  Robots at their target length are left unchanged and
 * record VINE_ST_DONE.  n_steps = 0 is a no-op (n_steps < 0: VINE_EINVAL).
 *   record_every  0: no trajectory; r >= 1: the joint angles after every r-th step
 *                 (and after step T - 1) go to VINE_F_TRAJ.  The buffer
 *                 (B x ceil(T / r) x N doubles) is allocated on the first call that
 *                 records with this r; a call with another r reallocates it.
 *   ckpt_every    0: no checkpoints; c >= 1: the state before every c-th step goes to
 *                 VINE_F_CKPT (B x ceil(T / c) x N doubles, allocated likewise).  With
 *                 checkpoints on every call since the reset, vine_sim_grad recomputes
 *                 the weighted steps from them instead of needing the trajectory
 *                 (32 keeps 1/32 of the states).
 * Asynchronous on stream.  Errors: VINE_EINVAL, VINE_ENOMEM, VINE_EDEVICE. */
int32_t vine_sim_step(vine_sim* h, int32_t n_steps, int32_t record_every, int32_t ckpt_every,
                      void* stream);

/* Grow every robot to its target length in one launch (n_steps = -1) or by
 * n_steps steps.  Same semantics as vine_sim_step. */
int32_t vine_sim_rollout(vine_sim* h, int32_t n_steps, int32_t record_every, int32_t ckpt_every,
                         void* stream);

/* Launch-order autotuning.  A batched launch lasts as long as its last robot, and the
 * robots of a chain-length class start in the handle's launch order as compute units
 * free up, so a long robot that starts late lengthens the launch.  At create the order
 * is a work estimate (links^2 x (4 + obstacles), longest first); this call replaces it,
 * inside each class, by the cycles each robot measured in the rollouts since the last
 * reset (VINE_F_CYCLES), longest first, for the launches that follow (repeated rollouts
 * of the same batch, as in a design search).  The class launches, which run
 * concurrently, are issued longest chains first at create; this call reorders them by
 * their slowest robot, slowest first, so that robot's workgroup finds the compute units
 * free (captured rollouts are recaptured if the order changes).  Robots never interact,
 * so results do not depend on either order.  Synchronises the stream.  Errors:
 * VINE_EINVAL, VINE_EDEVICE. */
int32_t vine_sim_tune_order(vine_sim* h, void* stream);

/* vine_sim_reset followed by vine_sim_rollout(h, -1, record_every, ckpt_every, stream)
 * (every robot regrown from zero length to its target, Sec. 4 growth steps), as one HIP
 * graph: the reset and the per-class launches (with their fork/join across the
 * handle's streams) are captured on the first call for each (record_every, ckpt_every)
 * (up to four kept) and replayed by later calls, so a repeated rollout costs one graph
 * launch.  The graph holds no memset nodes.  Results are bitwise those of the two eager
 * calls.  Captures are dropped by vine_sim_trace and when a trajectory or checkpoint
 * buffer is reallocated (they hold the buffers' addresses).  Errors: VINE_EINVAL,
 * VINE_ENOMEM (trajectory, checkpoints), VINE_EDEVICE (capture, launch). */
int32_t vine_sim_rollout_graph(vine_sim* h, int32_t record_every, int32_t ckpt_every,
                               void* stream);

/* Gradient of a tip-reaching loss with respect to the actuation design, by the
 * adjoint of the equilibrium conditions (Sec. 5 searches sPAM placement and
 * pressure with the simulator in the loop; the adjoint differentiates each step's
 * fixed point r(theta; p) = 0 of the Eq. 4 energy).  For robot b
 *     L_b = sum_t w_t |tip_b(t) - goal_b|^2
 * over the equilibria theta_b(t) after step t, and for every sPAM record s given
 * at create:  dL/dP_s, dL/ds_start_s, dL/ds_end_s of L = sum_b L_b (records shared
 * by several robots collect the sum).  Each equilibrium contributes
 *     -lam^T dr/dp with H lam = w_t dL_t/dtheta,
 * H the exact Hessian of the energy at theta_b(t) (factorised by the sweep the growth
 * solver uses, undamped).  Equilibria are taken as they were computed: the derivative
 * of a step whose status is not VINE_ST_CONVERGED, or across a change of the contact
 * set, is that of the smooth branch the state sits on (flagged in adj_status).
 *   goal          device, double [B][2]
 *   step_weights  device, double [T] (T from vine_sim_dims), or NULL: the loss
 *                 is then w = 1 on the current state alone.  With weights, steps
 *                 not yet taken by a robot are skipped, and every step/rollout call
 *                 since the last reset must have recorded every step
 *                 (record_every = 1) or written checkpoints (ckpt_every > 0, the
 *                 same on every call), else VINE_ESTATE.  Without the full
 *                 trajectory the states are recomputed segment by segment from the
 *                 checkpoints (bitwise the states of the rollout; one more rollout's
 *                 work, and B x ckpt_every x N doubles of segment buffers allocated
 *                 on first use).
 *   dL_dP, dL_ds_start, dL_ds_end   device, double [n_spams] (overwritten)
 *   loss          device, double [B] (overwritten with L_b)
 *   adj_status    device, int32 [B] or NULL: bit 0 set when an adjoint system was
 *                 singular or had more contacts than the contact list holds (that
 *                 step's term is then left out); bit 1 set when a weighted step had
 *                 not converged in the rollout (VINE_ST_* > 0).
 * Soft growth (growth_stiffness > 0) gives VINE_ESTATE: its states include the tip
 * length, which this adjoint does not differentiate.
 * Asynchronous on stream.  Errors: VINE_EINVAL (null pointers), VINE_ESTATE,
 * VINE_ENOMEM, VINE_EDEVICE. */
int32_t vine_sim_grad(vine_sim* h, const double* goal, const double* step_weights,
                      double* dL_dP, double* dL_ds_start, double* dL_ds_end, double* loss,
                      int32_t* adj_status, void* stream);

/* Bytes of the per-device scratch of vine_sim_grad_noalloc (128 MiB). */
#define VINE_GRAD_SCRATCH_BYTES (128ull << 20)

/* vine_sim_grad for callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as vine_sim_grad (bitwise the same outputs), but it allocates nothing:
 * the segment buffers of the checkpoint path (the recomputed states, records and
 * trajectory of ckpt_every steps, the robot rows and the adjoint's running sums; about
 * 8 B x (N + ckpt_every (N + 10) + 210) per robot) live in a static device array of
 * VINE_GRAD_SCRATCH_BYTES per device, held until the process ends.  Paths that need no
 * segment buffers (the final-state loss, a recorded trajectory) behave exactly as
 * vine_sim_grad.  Needs beyond the array give VINE_ECAPACITY (use vine_sim_grad).
 * Every call on a device shares that device's array and overwrites what the last call
 * left (every value is written before it is read); calls that overlap on one device
 * race, so serialise them (e.g. issue them on one stream). */
int32_t vine_sim_grad_noalloc(vine_sim* h, const double* goal, const double* step_weights,
                              double* dL_dP, double* dL_ds_start, double* dL_ds_end,
                              double* loss, int32_t* adj_status, void* stream);

/* Replace the sPAM records (placement and pressure; Sec. 3.1 and Sec. 5: the design
 * variables of the search) without rebuilding the handle.  spams: host, n_spams
 * records laid out as at create (each robot keeps its offset and count), which must
 * equal the count given at create, else VINE_EINVAL; invalid records as at create
 * give VINE_EINVAL and change nothing.  The robots' state is kept: call
 * vine_sim_reset before a fresh rollout.  The update is ordered after the work
 * already queued on `stream`; the call returns once it is done. */
int32_t vine_sim_set_spams(vine_sim* h, const vine_spam* spams, int32_t n_spams, void* stream);

/* Reset every robot to zero length (the records are cleared). */
int32_t vine_sim_reset(vine_sim* h, void* stream);

/* Copy a field into a caller-owned buffer of at least vine_sim_field_bytes() bytes:
 * device memory when dst_on_device != 0 (asynchronous on stream), else host memory
 * (the call synchronises the stream).  VINE_ESTATE for VINE_F_TRAJ when no
 * trajectory was recorded. */
int32_t vine_sim_read(const vine_sim* h, int32_t field, void* dst, int32_t dst_on_device,
                      void* stream);

/* Bytes needed by vine_sim_read for a field; 0 for an unknown field. */
int64_t vine_sim_field_bytes(const vine_sim* h, int32_t field);

/* Sizes: dims[0] = B robots, dims[1] = T recorded steps, dims[2] = N links. */
void vine_sim_dims(const vine_sim* h, int32_t dims[3]);

/* Destroy the handle and free its device memory.  NULL is allowed. */
void vine_sim_destroy(vine_sim* h);

/* Text of the last failure on this handle (owned by the handle, valid until the
 * next call on it).  With h == NULL: the last failure of the calling thread in a call
 * without a handle (vine_sim_create, vine_spam_synth, vine_spam_solve, vine_mlp_forward). */
const char* vine_sim_last_error(const vine_sim* h);

/* Evaluate the sPAM force law table the library built for link length l at
 * n host points eps[]: G = F_t / P_act (m^2), dG/deps, and int_0^eps G.  For
 * tests of the create-time table.  Returns VINE_EINVAL if l is not a link length
 * of this simulation. */
int32_t vine_sim_spam_law(const vine_sim* h, double l, int32_t n, const double* eps, double* G,
                          double* dG, double* IG);

/* ------------------------------------------------------------------------- */
/* Actuator synthesis (Sec. 4.2): the sPAM to build for a wanted bend.
 *
 * A joint whose link is covered by one sPAM of unit length l0 at pressure P rests in
 * free space where Eq. 3b's net moment vanishes: the wrinkling moment of Eq. 2,
 * pi P_vine R^3 h(theta), equals arm P G(eps; l0), the force of Eq. 1d at the strain
 * eps = arm theta / l of Eq. 3a (arm = 2 R + R_act, l the link length).  Fabrication
 * allows only a discrete set of pressures and unit lengths (a 1 mm grid in the paper).
 * For each target joint angle this returns the highest pressure of the set for which
 * some unit length of the grid rests within tol of the target, and of those unit lengths
 * the one whose rest angle is nearest (the first, i.e. shortest, of equal ones):
 * designs[3 i .. 3 i + 2] = (P, l0, rest angle), or (0, 0, 0) when no pressure fits.
 * The paper prefers the highest feasible pressure because it gave the most repeatable
 * bends; where it solves Eq. 1 by Levenberg-Marquardt from many starts, here every
 * (pressure, unit length) pair of the grid is solved exactly (one device wave each:
 * bisection on the sPAM's contraction parameter, each state solved from Eq. 1 with the
 * elliptic integrals spread over the lanes), and one device thread per target applies
 * the rule.
 *   pressures     [n_pressures] Pa, positive, strictly rising (<= VINE_SYNTH_MAX)
 *   unit_lengths  [n_lengths] m, positive, strictly rising (<= VINE_SYNTH_MAX)
 *   targets       [n_targets] joint angles (rad); designs [3 n_targets] out
 *   angles        NULL, or [n_pressures][n_lengths] out: every pair's rest angle
 *   link_len, tube_radius, body_pressure: l, R_vine, P_vine of the body
 * Host arrays; device memory is allocated and freed inside the call, which runs on
 * `stream` and returns when the results are copied back.  Errors: VINE_EINVAL (also
 * pressures or lengths not rising, a non-finite target or a negative tolerance),
 * VINE_ECAPACITY, VINE_ENOMEM, VINE_EDEVICE; vine_sim_last_error(NULL) describes
 * the failure. */
#define VINE_SYNTH_MAX 4096
int32_t vine_spam_synth(const vine_params* params, double link_len, double tube_radius,
                        double body_pressure, const double* pressures, int32_t n_pressures,
                        const double* unit_lengths, int32_t n_lengths, const double* targets,
                        int32_t n_targets, double tol, double* designs, double* angles,
                        void* stream);

/* The sPAM state of a given strain, solved exactly from Eq. 1 (Sec. 3.1): for each
 * sample i, the contraction parameter m in [m0, 1/2] whose strain (Eq. 1a) is eps[i]
 * for unit length unit_lengths[i] (bisection; the strain rises with m), with phi the
 * smallest root of Eq. 1b up to phi_Rc (unsaturated) or phi_Rc (saturated) and
 * G = F_t / P_act of Eq. 1d: out[4 i .. 4 i + 3] = (m, phi, G, strain reached).  A strain
 * at or above the slack strain gives the slack state (m = 1/2, G = 0); one at or below
 * zero gives m0.  This is the map the paper's surrogate (Sec. 4.3) approximates; here
 * it runs as one device wave per sample.  Host arrays of n doubles (out: 4 n); device
 * memory is allocated inside; returns when the results are copied back.  Errors:
 * VINE_EINVAL (non-finite strain, non-positive unit length), VINE_ENOMEM, VINE_EDEVICE. */
int32_t vine_spam_solve(const vine_params* params, int32_t n, const double* eps,
                        const double* unit_lengths, double* out, void* stream);

/* The neural surrogate of Sec. 4.3, a 2-32-2 perceptron with ReLU:
 * y = W2 relu(W1 x + b1) + b2 for each sample x[2 i .. 2 i + 1] into y[2 i .. 2 i + 1].
 * weights: VINE_MLP_WEIGHTS doubles packed as W1 [32][2], b1 [32], W2 [2][32], b2 [2]
 * (any input and output scaling is the caller's).  One device thread per sample; host
 * arrays; device memory is allocated inside.  Errors: VINE_EINVAL, VINE_ENOMEM,
 * VINE_EDEVICE. */
#define VINE_MLP_WEIGHTS 162
int32_t vine_mlp_forward(const double* weights, int32_t n, const double* x, double* y,
                         void* stream);

/* Occupancy of the current device: robots of each chain-length class (up to 64, 128,
 * 256 and 512 links) resident per compute unit in a rollout launch with `waves` (1, 2 or
 * 4) 64-lane waves per robot, and the number of compute units.  For reports of how busy a
 * launch keeps the device.  Errors: VINE_EINVAL (waves), VINE_EDEVICE. */
int32_t vine_sim_occupancy(int32_t waves, int32_t per_cu[4], int32_t* compute_units);

/* Waves per robot of each class's rollout launches (classes of up to 64, 128, 256 and
 * 512 links).  1: one wave does every evaluation's joint law and obstacle phase; 2
 * (default): the obstacle phase runs on a helper wave beside the joint law; 4: three
 * helpers, one taking the joint law of the second half of the chunks of 64 links and two
 * the obstacle phase of each half (a second contact-list region, appended after the
 * first), which shortens each evaluation of a long robot at the price of more LDS and
 * fewer robots per compute unit.  Results are bitwise the same in every case.  Drops the
 * captured rollouts when a value changes.  Errors: VINE_EINVAL. */
int32_t vine_sim_set_waves(vine_sim* h, const int32_t waves[4]);

/* The head: the robots whose cycles, as vine_sim_tune_order last measured them, are at
 * least `fraction` of the slowest robot's, of any class, taken out of their classes and
 * run as one launch of their own (sized for the longest of them) with `waves` per robot,
 * issued before the classes' launches and concurrent with them.  A batch lasts at least
 * as long as its slowest robot, which more waves per robot shorten, while fewer waves per
 * robot keep more robots on the device; the head gives the few slowest robots the first
 * and the rest the second.  fraction 0 (the default) or no measured cycles: no head.
 * Results are bitwise the same with or without a head.  Drops the captured rollouts when
 * the launches change; writes the launch order on the stream and synchronises it.
 * Errors: VINE_EINVAL (fraction outside [0, 1], waves not 1, 2 or 4), VINE_EDEVICE. */
int32_t vine_sim_set_head(vine_sim* h, double fraction, int32_t waves, void* stream);

/* The head as set (fraction, waves per robot, robots in it; each argument host or NULL)
 * and ms (host, 6, or NULL): the autotuner's times of the whole batch, [3 k + j] with the
 * classes' wave counts of candidate k (0: each class's fastest alone, 1: two waves in
 * every class) and head fraction j (0, 1/2, 1/4); 0 when not measured.
 * Errors: VINE_EINVAL. */
int32_t vine_sim_head(const vine_sim* h, double* fraction, int32_t* waves, int32_t* count,
                      double ms[6]);

/* Autotuner: for each chain-length class present, time the class's rollout from zero
 * length to full with 1, 2 and 4 waves per robot (without a head), in the handle's
 * current launch order, and keep the fastest (vine_sim_set_waves; 2 unless another
 * measured faster); then, if vine_sim_tune_order has measured the robots, time the whole
 * batch as it is launched with those wave counts and with two waves in every class, each
 * with no head and with heads of four waves per robot at fractions 1/2 and 1/4
 * (vine_sim_set_head), and keep the fastest (ties: the earlier).  The
 * choice is remembered for this configuration (a hash of the parameters and every input
 * given at create) in a cache of the process, so that later handles of the same
 * configuration take it without measuring (the head part is measured, once, by the first
 * call on a handle whose robots are measured; a head needs the handle's own cycles).
 * waves (host, 4, or NULL): the choice, 0 for classes with no robot; ms (host, 12, or
 * NULL): [3 c + k] the time of class c with 1, 2, 4 waves for k = 0, 1, 2 (0 when not
 * measured); cached (host or NULL): 1 when the wave counts were taken from the cache.
 * Measuring runs the rollouts, so the robots end reset to zero length.  Synchronises the
 * stream.  Errors: VINE_EINVAL, VINE_EDEVICE. */
int32_t vine_sim_autotune(vine_sim* h, int32_t waves[4], double ms[12], int32_t* cached,
                          void* stream);

/* Diagnostics: record one row per accepted Newton iteration of robot `robot`
 * (step, sub-step, iteration, rho, mu, slope, step factor alpha, energy, step kind:
 * 1 damped Newton, 2 negative curvature; contacts) into a device buffer of `capacity` rows on later step/rollout calls.
 * robot = -1 switches tracing off. */
int32_t vine_sim_trace(vine_sim* h, int32_t robot, int32_t capacity);

/* Copy up to `capacity` trace rows (10 doubles each) to host memory; returns the
 * number of rows copied, or a negative VINE_E* code. */
int32_t vine_sim_trace_read(const vine_sim* h, double* dst, int32_t capacity);

/* ------------------------------------------------------------------------- */
/* Serving: continuous batching of rollout requests on one device.
 *
 * The paper's planner (Sec. 5) issues many short simulation jobs whose sizes vary
 * (designs of different length, several environment samples each).  A server keeps the
 * robots it has admitted resident on the device; queued robots are admitted as soon as
 * a lane, a slot and device memory are free and start at once, next to the robots
 * already running, so long and short jobs share the device.
 *
 * Device memory is a budget, not a worst case: a robot of n links and K obstacles takes
 * n rows of a row pool (joint angle, sPAM coverage and one growth step's records per
 * row, 92 bytes) and K entries of an obstacle pool (36 bytes), allocated first-fit on
 * admission and freed when it is read back.
 *
 * vine_server_tick never waits for the device.  It reads back the groups whose launch
 * has finished (their results are copied out asynchronously and handed over on a later
 * call, their memory freed then) and starts a group on each idle lane.  A lane is one of
 * the server's streams, one per hardware queue of the process (GPU_MAX_HW_QUEUES when it
 * is set at create, at most 32; HIP's default is 4), and carries one group at a time.  A group takes the chain-length class (up to 64, 128, 256
 * or 512 links) of the oldest queued robot and every queued robot of that class that
 * fits (a free slot and room in both pools), in arrival order; robots of other classes
 * keep their places, and when the oldest robot does not fit nothing overtakes it.  Its
 * rows are copied in from pinned host staging (asynchronously) and it grows to full
 * length in one launch, longest expected work first.  A lightly loaded server so starts
 * each request on arrival; under load the queue builds up while the lanes are busy and
 * the groups grow.  A request is a set of robots (e.g. one design on S environment
 * samples) and completes when all of its robots are read back.  Results are bitwise
 * those of the same robots run through vine_sim_create / vine_sim_rollout (robots never
 * interact, and the kernels are the same). */
typedef struct vine_server vine_server;

/* slots: robots resident at once; hbm_bytes: device memory for the pools and per-slot
 * rows, split so that the pools hold floor((hbm_bytes - 148 slots) / (92 max_links +
 * 36 max_obstacles)) robots at the bounds (more of smaller ones); max_links /
 * max_obstacles / max_spams bound each robot (<= VINE_MAX_LINKS / VINE_MAX_OBSTACLES /
 * VINE_MAX_SPAMS).  Device and pinned host memory are allocated here, once.  Up to 8
 * distinct link lengths are supported over the server's life (the force-law table is
 * built on first use of a length).  Errors: VINE_EINVAL (also a budget below one robot
 * at the bounds), VINE_ECAPACITY, VINE_ENOMEM, VINE_EDEVICE. */
int32_t vine_server_create(const vine_params* params, int32_t slots, int64_t hbm_bytes,
                           int32_t max_links, int32_t max_obstacles, int32_t max_spams,
                           vine_server** out);

/* Queue one request (FIFO).  Host arrays as for vine_sim_create (offsets relative to
 * these arrays); copied.  request_id is the caller's and must not be queued twice at
 * once.  Robots above the server's bounds, or a ninth distinct link length, give
 * VINE_ECAPACITY, invalid input VINE_EINVAL; nothing is queued then.  The force-law
 * table of a new link length is built and uploaded here (a blocking copy). */
int32_t vine_server_submit(vine_server* s, int64_t request_id, const vine_instance* inst,
                           int32_t n_inst, const vine_spam* spams, int32_t n_spams,
                           const vine_obstacle* obstacles, int32_t n_obstacles);

/* vine_server_submit with a starting state per robot: robot b starts grown to
 * start_links[b] links (0 <= start_links[b] < n_links; 0 = from zero) with the joint
 * angles start_theta[o_b .. o_b + start_links[b]), o_b the sum of the counts before it
 * (host array, copied), and takes growth steps start_links[b] .. n_links - 1.  A growth
 * step depends on the state only through the joint angles and the link count (Alg. 1),
 * so a robot started from the first s links of an earlier rollout of a design with the
 * same sPAMs over those links ends bitwise where a rollout of its design from zero
 * ends: the planner (Alg. 2) propagates a child T steps from its parent this way.  Its
 * records (status, tip) exist for steps start_links[b] on; the request's worst status
 * covers those steps.  Hard growth only: with growth_stiffness > 0 a nonzero start is
 * VINE_ESTATE.  start_links NULL: as vine_server_submit.  Errors as vine_server_submit,
 * and VINE_EINVAL for a count outside the range, a NULL start_theta with a nonzero
 * count or a non-finite angle; nothing is queued then. */
int32_t vine_server_submit_from(vine_server* s, int64_t request_id, const vine_instance* inst,
                                int32_t n_inst, const vine_spam* spams, int32_t n_spams,
                                const vine_obstacle* obstacles, int32_t n_obstacles,
                                const int32_t* start_links, const double* start_theta);

/* One scheduling round (see above): hand over the groups read back, start reading back
 * the groups that finished, admit and launch the queued robots that fit.  Returns the
 * number of requests completed by this call, or a negative VINE_E* code.  It does not
 * block: call it repeatedly while requests are queued or resident (vine_server_stats). */
int32_t vine_server_tick(vine_server* s);

/* Completed requests not yet polled, oldest first: their ids into ids[] (host, up to
 * cap entries) and, if worst_status is non-NULL, the largest per-step status over the
 * request's robots (0 = every step converged).  Returns the number written. */
int32_t vine_server_poll(vine_server* s, int64_t* ids, int32_t* worst_status, int32_t cap);

/* Final state of robot `robot` (its index in the request) of a completed request:
 * tip (x, y, heading) into tip[3] and, if theta is non-NULL, its joint angles into
 * theta[0 .. n_links).  Results are kept until vine_server_release.  VINE_EINVAL for
 * an unknown or unfinished request or robot. */
int32_t vine_server_result(const vine_server* s, int64_t request_id, int32_t robot, double* tip,
                           double* theta);

/* Forget a completed request's results. */
int32_t vine_server_release(vine_server* s, int64_t request_id);

/* Counters: [0] robots queued, [1] robots resident (running or being read back),
 * [2] requests completed, [3] joint-updates of the robots read back (sum over growth
 * steps of the link count), [4] rows in use, [5] row capacity, [6] device bytes of the
 * pools and slot rows, [7] groups in flight. */
void vine_server_stats(const vine_server* s, int64_t out[8]);

void vine_server_destroy(vine_server* s);
const char* vine_server_last_error(const vine_server* s);

#ifdef __cplusplus
}
#endif

#endif /* VINESIM_H */
