/*
 * rbfib.h -- C ABI of the MI355X hot path of the Rigid-Body Fluctuating
 * Immersed Boundary (RB-FIB) method (Sprinkle, Donev, Bhalla & Patankar,
 * "Brownian dynamics of fully confined suspensions of rigid particles without
 * Green's functions").
 *
 * What the library computes
 * -------------------------
 * For rigid bodies p with tracking points q_p and unit-quaternion orientations
 * theta_p, made of markers r_i = q_p + R(theta_p) r_i^ref, suspended in a
 * Stokes fluid on a staggered grid of Nx x Ny x Nz cells with a periodic or
 * no-slip (possibly sliding) or free-slip wall boundary per axis, the library applies and
 * solves the constrained saddle-point system of eqs. (LangevinD1-D4):
 *
 *     [ -eta Lm   G   -S   0 ] [ v      ]   [ f_v                          ]
 *     [   -D      0    0   0 ] [ pi     ] = [ 0                            ]
 *     [   -J      0    0   K ] [ lambda ]   [ -slip + J_bc                 ]
 *     [    0      0   K^T  0 ] [ U      ]   [ F                            ]
 *
 * (Sec. III: MAC operators Lm = DT GT, G = -D^*; interpolation J and spreading
 * S through a 4- or 6-point delta kernel, J = dV S^*; (K U)_i = u_p + omega_p x
 * (r_i - q_p), (K^T lambda)_p = [sum lambda_i; sum (r_i - q_p) x lambda_i]),
 * and advances the bodies by the Split-Euler-Maruyama scheme of Algorithm 1
 * with the random-finite-difference drift (Sec. IV).  Walls enter S and J by
 * reflection of the kernel support (odd for the normal component and for
 * tangential components at no-slip walls, even for tangential components at
 * free-slip walls); a wall sliding with tangential velocity U_w adds
 * 2 eta U_w / h^2 to the momentum rows next to it and J_bc to the constraint
 * rows.
 *
 * Conventions
 * -----------
 *  * All array arguments are DEVICE pointers owned by the caller, FP64,
 *    contiguous, row-major, unless a comment says "host".  The library never
 *    frees caller memory.  A context owns all workspace it allocates.
 *  * Work is enqueued on the HIP stream given at creation.  Every entry point
 *    that takes orientations checks them on the device and reads the result
 *    back, and those that return convergence or rejection information wait
 *    for their results, so all of these synchronise that stream before
 *    returning; rbfib_fluctuating_stress is asynchronous.
 *  * Quaternions are scalar first (w, x, y, z).  Body arrays are [nb, 3]
 *    (q), [nb, 4] (theta), [nb, 6] (forces/torques or velocities [u, omega]).
 *    Marker arrays are [nm, 3].
 *  * State vector (x, y of rbfib_apply_saddle; optional full solution of a
 *    solve), per replica and concatenated over replicas in order:
 *        [ u_x | u_y | u_z | pi | lambda (nm x 3) | U (nb x 6) ]
 *    where each of u_x, u_y, u_z, pi has Nx*Ny*Nz entries, x fastest.  Entry
 *    (i, j, k) of u_c is the c-face at coordinate i*h along c (cell centred
 *    along the other axes).  Along a wall axis c the slot i_c = 0 is the wall
 *    face: it is not an unknown, is ignored on input and is written as 0.
 *    rbfib_layout returns the offsets.
 *  * Batched contexts hold independent replicas (each its own grid and
 *    bodies); bodies and markers of all replicas are concatenated in replica
 *    order and rbfib_info arrays have one entry per replica.
 *
 * Errors
 * ------
 * Every int-returning call returns RBFIB_OK (0) or a negative code:
 *   RBFIB_EINVAL   bad argument (sizes, fewer than 4 cells on an axis, a
 *                  periodic axis with no no-slip wall axis, NULL pointer, bad options,
 *                  an orientation theta_p with | |theta_p| - 1 | > 1e-12 or
 *                  not finite -- Sec. II requires unit quaternions);
 *   RBFIB_EREJECT  unphysical configuration: a marker outside the open domain
 *                  along a wall axis, or body centres closer than
 *                  opts.min_body_dist (the paper rejects and repeats such
 *                  steps); state left unchanged;
 *   RBFIB_ENOCONV  max_iter reached before tol; outputs hold the last iterate,
 *                  info holds the residual reached;
 *   RBFIB_ENUMERIC a NaN or Inf appeared in the Krylov recurrences;
 *   RBFIB_EDEVICE  a HIP runtime call failed;
 *   RBFIB_ENOMEM   device allocation failed.
 * For batched calls the return value is the first non-OK replica status in
 * replica order (EREJECT and ENOCONV) or a global failure; per-replica status
 * is in info[r].status.
 */
#ifndef RBFIB_H
#define RBFIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBFIB_OK        0
#define RBFIB_EINVAL   -1
#define RBFIB_EREJECT  -2
#define RBFIB_ENOCONV  -3
#define RBFIB_ENUMERIC -4
#define RBFIB_EDEVICE  -5
#define RBFIB_ENOMEM   -6

#define RBFIB_PERIODIC 0
#define RBFIB_WALL     1   /* no-slip wall, possibly sliding (wall_vel)                 */
#define RBFIB_SLIP     2   /* free-slip wall: no normal flow, no tangential stress       */

typedef struct rbfib_ctx rbfib_ctx;

/* Grid and boundary conditions (Sec. III.A; Sec. VI for the sliding wall; free-slip
 * walls are one of the combinations of boundary conditions the formulation admits,
 * Introduction and Conclusion).  At least one axis must be RBFIB_WALL, or none
 * periodic: otherwise a uniform flow along the periodic axes is free and the
 * mobility problem is singular. */
typedef struct {
    int n[3];                  /* cells per axis, x y z                              */
    int bc[3];                 /* RBFIB_PERIODIC, RBFIB_WALL or RBFIB_SLIP per axis   */
    double h;                  /* cell width; dV = h^3                               */
    double eta;                /* viscosity                                          */
    double wall_vel[3][2][3];  /* [axis][0 low, 1 high][component]; tangential only, */
                               /*    no-slip walls only                              */
} rbfib_grid;

/* Rigid bodies as marker agglomerates (Sec. III.B).  Host memory, copied. */
typedef struct {
    int nb;                    /* number of bodies                                   */
    int nm;                    /* number of markers (sum over bodies)                */
    const int *marker_offset;  /* host [nb + 1], CSR body -> markers, offset[0] = 0  */
    const double *r_ref;       /* host [nm, 3], body-frame marker offsets            */
} rbfib_bodies;

/* Solver options; rbfib_default_opts fills every field. */
typedef struct {
    double tol;                /* relative residual ||b - A x|| / ||b||  (1e-6)      */
    int restart;               /* FGMRES restart length (100)                        */
    int max_iter;              /* total iteration cap (600)                          */
    int precond_fp32;          /* 1: multigrid preconditioner in FP32, and FGMRES    */
                               /*    keeps the preconditioned vectors in FP32 (A is  */
                               /*    applied to the stored values) (0)               */
    int mg_sweeps;             /* damped-Jacobi sweeps before and after, 1..16 (2)   */
    int mg_sweeps_p;           /* the same for the pressure cycle; 0: mg_sweeps (3)  */
    double mg_omega;           /* Jacobi damping (0.9)                               */
    double blob_radius;        /* blob radius of the body block, units of h (1.2)    */
    double rfd_delta;          /* random-finite-difference delta (1e-5)              */
    double min_body_dist;      /* rejection distance between body centres (0 = off)  */
    int check_every;           /* iterations between host convergence checks (5)    */
    int use_graphs;            /* 1: replay each FGMRES iteration as a captured HIP  */
                               /*    graph on the library's stream (1)               */
    int mg_fused;              /* multigrid levels as two fused kernels (sweeps +    */
                               /*    residual + restriction; prolongation + sweeps)  */
                               /*    with the same values as the separate kernels;   */
                               /*    needs mg_sweeps == 2.  0 never, 1 on levels     */
                               /*    with enough workgroups to fill the device,      */
                               /*    2 on every level (0)                            */
    int mg_bottom;             /* > 0: each replica's coarse levels, from the first  */
                               /*    whose grids fit mg_bottom KB (at most 64), run  */
                               /*    in one workgroup per (replica, component) with  */
                               /*    every grid in LDS and the same values as the    */
                               /*    separate kernels; 0: separate kernels on every  */
                               /*    level; fixed at creation (32)                   */
    double mg_cheby;           /* > 0: sweep k of nu has weight 1 / lambda_k, the    */
                               /*    roots of the degree-nu Chebyshev polynomial on  */
                               /*    [mg_cheby, 2]; 0: every sweep mg_omega (0.27)   */
    int krylov_s;              /* Arnoldi steps per block, 1..4: the block's new     */
                               /*    vectors are orthogonalised in one pass over the */
                               /*    basis (tol >= 1e-9; a shorter last block runs   */
                               /*    single steps) (2)                               */
    int mg_first2;             /* 1: the first two sweeps of each down pass as one   */
                               /*    kernel on every level (b read once, the first   */
                               /*    iterate never stored; same values as two        */
                               /*    sweeps); 0: two launches (1)                    */
    int kernel;                /* width of the delta kernel of S and J (Sec. III.B), */
                               /*    fixed at creation: 4 = Peskin's 4-point         */
                               /*    function, 6 = the 6-point function of Bao,      */
                               /*    Kaiser & Peskin the paper uses (blob radius     */
                               /*    1.47 h; set blob_radius to match) (4)           */
    int no_drift;              /* 1: rbfib_sem_step drops the random finite          */
                               /*    differences of Algorithm 1 (no RFD solves, no   */
                               /*    stochastic drift): the naive Euler-Maruyama     */
                               /*    scheme, whose equilibrium is biased (Appendix   */
                               /*    A); for demonstrating that bias only (0)        */
} rbfib_opts;

typedef struct {
    int iters;                 /* FGMRES iterations (constrained solves summed)      */
    double rel_residual;       /* true relative residual of the last solve           */
    int status;                /* RBFIB_OK, RBFIB_ENOCONV, RBFIB_EREJECT, ...        */
} rbfib_info;

void rbfib_default_opts(rbfib_opts *opts);
const char *rbfib_strerror(int code);
/* Text of the last failure seen on this thread (HIP error string, allocation size). */
const char *rbfib_last_error(void);

/* One replica.  hip_stream: a hipStream_t (NULL = default stream). */
int rbfib_create(const rbfib_grid *grid, const rbfib_bodies *bodies, const rbfib_opts *opts,
                 void *hip_stream, rbfib_ctx **out);

/* nrep independent replicas solved together (one launch per kernel step). */
int rbfib_create_batch(int nrep, const rbfib_grid *grids, const rbfib_bodies *bodies,
                       const rbfib_opts *opts, void *hip_stream, rbfib_ctx **out);

void rbfib_destroy(rbfib_ctx *ctx);

/* Update the solver options of an existing context (same fields as creation). */
int rbfib_set_opts(rbfib_ctx *ctx, const rbfib_opts *opts);

/* Length of one packed state vector (all replicas). */
long long rbfib_state_size(const rbfib_ctx *ctx);

/* Host out[nrep * 4]: offsets of u_x, pi, lambda and U of each replica. */
int rbfib_layout(const rbfib_ctx *ctx, long long *out);

/* Marker geometry at (q, theta) (Sec. II, III.B): r [nm, 3] = q_p + R(theta_p) r_ref,
 * tile [nm] = linear index (x fastest, per replica) of the 4x4x4-cell tile holding
 * floor(r / h) (wrapped on periodic axes), perm [nm] = markers stably sorted by tile
 * (replica-local indices).  Any output may be NULL. */
int rbfib_markers(rbfib_ctx *ctx, const double *q, const double *theta,
                  double *r, int *tile, int *perm);

/* y = A x for the homogeneous operator above at configuration (q, theta)
 * (Algorithm 1 block matrix with the signs of eqs. D1-D4).  x and y are state
 * vectors and must not alias.  Markers must lie inside the domain along wall
 * axes (indices are clamped, never out of bounds, but the result is then
 * meaningless). */
int rbfib_apply_saddle(rbfib_ctx *ctx, const double *q, const double *theta,
                       const double *x, double *y);

/* Allocation-free y = A x for ONE replica, for callers that cannot allocate device
 * memory: code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same operator and the same kernels as rbfib_apply_saddle on a
 * context created from (grid, bodies), but no context: every table the kernels
 * need lives in one fixed device array of the library (about 10 MiB per device,
 * held until the process ends), so the call neither allocates nor frees device
 * memory.  grid and bodies: host, as for rbfib_create (marker_offset and r_ref are
 * copied to the device on every call); q [nb, 3], theta [nb, 4], x and y (state
 * vectors of the replica, must not alias): device; hip_stream: the stream all work
 * is enqueued on (NULL = default stream).  Limits: at most 8192 markers, 2048
 * bodies, 1024 markers per body, 2^23 cells and 2^17 tiles of 4x4x4 cells; larger
 * inputs return RBFIB_EINVAL before any work is enqueued.  Asynchronous: the
 * orientations are not checked (they must be unit quaternions), and markers must
 * lie inside the domain along wall axes, as for rbfib_apply_saddle.  Every call on a
 * device uses that device's array and leaves its contents there: calls that overlap
 * on one device (different streams, or host threads without ordering) race. */
int rbfib_apply_saddle_noalloc(const rbfib_grid *grid, const rbfib_bodies *bodies, const double *q,
                               const double *theta, const double *x, double *y, void *hip_stream);

/* Preconditioner z = P^-1 r (for inspection; the solver applies it internally). */
int rbfib_precondition(rbfib_ctx *ctx, const double *q, const double *theta,
                       const double *r, double *z);

/* Deterministic mobility solve (eqs. D1-D4 with no noise): given forces and
 * torques FT [nb, 6] and optional marker slip [nm, 3] (NULL = 0), returns the
 * rigid velocities U [nb, 6] = N F - N K^T M^-1 slip (+ the response to sliding
 * walls).  x_out (optional, state vector) receives the full solution (v, pi,
 * lambda, U).  include_bc = 0 drops the wall-velocity terms.  info: host,
 * one entry per replica (may be NULL). */
int rbfib_solve_mobility(rbfib_ctx *ctx, const double *q, const double *theta,
                         const double *FT, const double *slip, int include_bc,
                         double *U, double *x_out, rbfib_info *info);

/* Fluctuating-stress forcing sqrt(2 kT eta / (dV dt)) DT W (eq. DFHD) written
 * into the velocity slots of the state vector f (other slots zeroed), with W
 * i.i.d. N(0,1) from Philox4x32-10 (seed, stream 1, step) over the nine
 * stress families xx, yy, zz, xy, xz, yx, yz, zx, zy: family (c, c) on cells,
 * family (c, b) on edges with (N_b + 1 if wall else N_b) nodes along b, each
 * x fastest; per replica, replica r uses step counter step and seed
 * seed + r. */
int rbfib_fluctuating_stress(rbfib_ctx *ctx, double kT, double dt, uint64_t seed,
                             uint64_t step, double *f);

/* One Split-Euler-Maruyama step (Algorithm 1): random forces and torques,
 * RFD solve, unconstrained Stokes solve, random finite differences of K^T, K,
 * J and S, the noisy constrained solve with force FT - D^KT and slip
 * slip + D^K - D^J - D^S, then q += dt u, theta = Rotate(theta, dt omega).
 * q and theta are updated in place only when the step is accepted.  FT are
 * the deterministic forces at the current configuration (caller evaluated).
 * U [nb, 6] receives U^n.  Replica r draws from seed + r. */
int rbfib_sem_step(rbfib_ctx *ctx, double *q, double *theta, const double *FT,
                   const double *slip, double kT, double dt, uint64_t seed, uint64_t step,
                   double *U, rbfib_info *info);

/* Caller-side conservative forces of the paper's confined test problems.
 * Every marker i of body p, at r_i = q_p + d_i with d_i = R(theta_p) r_i^ref,
 * feels the soft wall repulsion of eq. Usoft (Sec. V.A),
 *     Phi(r) = phi0 (1 + (d - r)/b)  for r < d,   phi0 exp((d - r)/b)  for r >= d,
 * from both faces of every non-periodic axis (r = its distance to the face,
 * the faces at 0 and n h), plus the constant force fconst (App. A: the
 * buoyant weight -m_e g z-hat of each blob).  Energies in the caller's units. */
typedef struct {
    double phi0;               /* strength of the repulsion                         */
    double d;                  /* range where the profile turns exponential         */
    double b;                  /* decay length (> 0)                                */
    double fconst[3];          /* constant force on every marker                    */
} rbfib_potential;

/* FT [nb, 6] (device, FP64, overwritten) = per body [sum_i f_i ; sum_i d_i x f_i],
 * f_i = -grad of marker i's energy; the torque is about the tracking point q_p.
 * q [nb, 3], theta [nb, 4] device, theta unit quaternions (not checked here;
 * rbfib_sem_step checks them).  Asynchronous on the context's stream.
 * RBFIB_EINVAL: a null pointer, b <= 0 or a non-finite parameter. */
int rbfib_body_forces(rbfib_ctx *ctx, const double *q, const double *theta,
                      const rbfib_potential *pot, double *FT);

/* Deterministically second-order variants of the SEM step (the Conclusion names
 * trapezoidal, midpoint and Adams-Bashforth extensions without writing one out;
 * this is the reading implemented): a two-stage Runge-Kutta rule on the
 * deterministic velocity with predictor fraction alpha in (0, 1] -- alpha = 1 the
 * trapezoidal (Heun) form, alpha = 1/2 the explicit midpoint form -- around the
 * unchanged random part of Algorithm 1.  Two calls, because the caller evaluates
 * the forces at the predicted configuration:
 *
 * rbfib_sem_rk2_predict: Algorithm 1 at Q^n = (q, theta) with forces FT = F(Q^n)
 *   and the same random numbers as rbfib_sem_step (seed + r, step), giving U^n;
 *   the deterministic velocity U_det^n = N(Q^n) F(Q^n) with the slip and boundary
 *   data (one more constrained solve); and the predictor Q* = (q + alpha dt u^n,
 *   Rotate(theta, alpha dt omega^n)) written to q_pred [nb, 3] and theta_pred
 *   [nb, 4] (Q^n there for replicas whose step was rejected).  q and theta are not
 *   modified.  The context keeps Q^n, Q*, alpha and both velocities.
 * rbfib_sem_rk2_correct: U_det* = N(Q*) F(Q*) with FT_pred = F(Q*) and slip_pred
 *   (NULL: none) at Q*, then U_c = U^n + (U_det* - U_det^n) / (2 alpha) and
 *   Q^{n+1} = (q^n + dt u_c, Rotate(theta^n, dt omega_c)) from the stored Q^n,
 *   written to q and theta; U (may be NULL) receives U_c [nb, 6].
 * At kT = 0 these are Heun's method and the midpoint rule for dQ/dt = N(Q) F(Q).
 * Rejection as in rbfib_sem_step: a replica whose Algorithm 1 step is rejected,
 * whose Q* or Q^{n+1} leaves the domain, or whose solves fail keeps Q^n (q and
 * theta are not written for it; RBFIB_EREJECT or the failure in info).  Five
 * constrained solves and one unconstrained solve per step.  The corrector without
 * a preceding predictor on the context, or alpha outside (0, 1], returns
 * RBFIB_EINVAL; info as for rbfib_sem_step. */
int rbfib_sem_rk2_predict(rbfib_ctx *ctx, const double *q, const double *theta, const double *FT,
                          const double *slip, double kT, double dt, double alpha, uint64_t seed,
                          uint64_t step, double *q_pred, double *theta_pred, rbfib_info *info);
int rbfib_sem_rk2_correct(rbfib_ctx *ctx, double *q, double *theta, const double *FT_pred,
                          const double *slip_pred, double *U, rbfib_info *info);

/* Adams-Bashforth variant of the SEM step, deterministically second order (the
 * Conclusion's third named extension; reading implemented): Algorithm 1 at Q^n
 * with the same random numbers as rbfib_sem_step gives U^n, the deterministic
 * velocity U_det^n = N(Q^n) F(Q^n) (slip and boundary data; one more constrained
 * solve) is extrapolated with the previous step's,
 *     U_c = U^n + (U_det^n - U_det^{n-1}) / 2,
 * and Q^{n+1} = (q + dt u_c, Rotate(theta, dt omega_c)) is written to q and theta.
 * U_det_prev [nb, 6] (device, caller owned) holds U_det^{n-1} on entry when
 * have_prev = 1 (have_prev = 0: none, the step is Algorithm 1's) and receives
 * U_det^n on return for every replica.  U (may be NULL) receives U_c.  At kT = 0
 * this is the two-step Adams-Bashforth rule.  Rejection as in rbfib_sem_step, plus
 * Q^{n+1} outside the domain.  Four constrained solves and one unconstrained
 * solve per step; one call, since the forces are needed at Q^n only. */
int rbfib_sem_ab2_step(rbfib_ctx *ctx, double *q, double *theta, const double *FT, const double *slip,
                       double kT, double dt, uint64_t seed, uint64_t step, double *U_det_prev,
                       int have_prev, double *U, rbfib_info *info);

/* Vector-Jacobian product of U = N(q, theta) F (no slip, no wall motion;
 * eqs. D1-D4 differentiated): given Ubar = dL/dU [nb, 6], returns
 * dFT = dL/dF [nb, 6], dq = dL/dq [nb, 3], dphi [nb, 3] (gradient with respect
 * to a lab-frame rotation vector applied to each body) and dtheta [nb, 4]
 * (gradient with respect to the unit quaternion, tangent to the unit sphere).
 * Any output may be NULL.  Re-solves the forward problem (the Krylov basis is
 * recomputed, not stored) and solves the adjoint system, which has the same
 * operator; the body-position gradient enters through the derivative of the
 * kernel in J (and S = J^T / dV).  info: iterations of both solves, the larger
 * of the two residuals. */
int rbfib_mobility_vjp(rbfib_ctx *ctx, const double *q, const double *theta, const double *FT,
                       const double *Ubar, double *dFT, double *dq, double *dphi, double *dtheta,
                       rbfib_info *info);

/* Average duration (ms) of the dominant kernel class over the last solve,
 * measured with HIP events on the context stream, and its average algorithmic
 * bytes per launch.  which: 0 = fused MAC saddle apply, 1 = level-0 smoother
 * sweep (separate kernels), 2 = level-0 fused down kernel (two sweeps, residual,
 * restriction), 3 = level-0 fused up kernel (prolongation, two sweeps),
 * 4 = FGMRES dot products of the basis with w (the dot kernel and its reduction),
 * 5 = FGMRES basis update of w with its norm, 6 = spreading -S lambda of the
 * apply (bytes: read-modify-write of the three FP64 velocity components on every
 * cell of every target tile, plus each marker's position and lambda).  Only solves
 * run with timing enabled (rbfib_enable_timing) are counted; a timing run reads
 * the active-tile count back before each timed spreading launch. */
int rbfib_kernel_stats(rbfib_ctx *ctx, int which, double *avg_ms, double *bytes_per_launch,
                       long long *launches);
int rbfib_enable_timing(rbfib_ctx *ctx, int on);

/* Launch geometry of a context (host out[5]): Krylov vector elements per workgroup
 * (512, 1024 or 2048), workgroups of the spreading pass, (tile, marker) pairs staged
 * per LDS round of spreading (16, 32 or 64), grid points per thread of the
 * multigrid and cell kernels (1 or 4), and z planes per workgroup of the z-marching
 * fluid apply (0: the two-cells-per-thread apply).  Chosen at creation from the
 * table the autotuner writes (the file named by the environment variable
 * RBFIB_TUNING, else tuning.txt beside the library; built-in defaults without one):
 * the first line
 *     cells_lo cells_hi reps_lo reps_hi krylov_chunk spread_grid spread_p mg_npt [apply_kc]
 * whose inclusive ranges hold the context's total cell count and replica count
 * (mg_npt 0: four points per thread on batches of at least 2^22 cells, else one;
 * apply_kc absent or 0: the two-cell apply).
 * The geometry changes only how work is split; results differ at most by the order
 * of floating-point sums. */
int rbfib_launch_geometry(const rbfib_ctx *ctx, int *out);

#ifdef __cplusplus
}
#endif

#endif /* RBFIB_H */
