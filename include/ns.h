/* ns.h - C ABI of the MI355X (gfx950) library for one time step of the
 * level-set, Brinkman-penalised, two-phase (water/air) incompressible
 * Navier-Stokes solver of arXiv 2206.07732 on a uniform staggered grid.
 *
 * The step (Sec. "Solution methodology", one fixed-point cycle per step as in
 * Sec. "Time stepping scheme") is
 *   1. levelset_advect_reinit: sigma^n -> sigma^{n+1}           (Sec. "Level set
 *      advection"; reinitialisation of Sec. "Interface tracking")
 *   2. momentum_step: rho, mu, chi at t^{n+1} from sigma^{n+1} and the body
 *      level set psi (eqn_ls_flow, eqn_ls_solid, eqn_Hflow, eqn_Hbody), then
 *      the predictor u* of eqn_c_discrete_momentum with the Brinkman force
 *      eqn_bp_discrete implicit and gravity on rho^flow
 *   3. projection_solve: -div(beta grad p) = -div(u*)/dt so that the
 *      corrected velocity meets eqn_c_discrete_continuity, solved by flexible
 *      CG preconditioned with a geometric multigrid V(2,2) cycle (red-black
 *      Gauss-Seidel smoother), in FP64 or with the V-cycle in FP32.
 *
 * Grid (Sec. "Spatial discretization"): nx*ny*nz cells of size h, cell
 * (i,j,k) centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h); gravity along -z; a 2-D
 * tank in the (x,z) plane is ny == 1.  Arrays are x-fastest, FP64:
 *   cell  a[i + nx*(j + ny*k)]                    nx*ny*nz
 *   u     u[i + (nx+1)*(j + ny*k)]  x = i h       (nx+1)*ny*nz
 *   v     v[i + nx*(j + (ny+1)*k)]  y = j h       nx*(ny+1)*nz
 *   w     w[i + nx*(j + ny*k)]      z = k h       nx*ny*(nz+1)
 * Boundaries: x, y and bottom are free-slip walls (their normal faces stay
 * 0); the top (z = nz h) is open with p = 0 on the boundary face.
 *
 * Memory and streams.  Every array pointer is a DEVICE pointer owned by the
 * caller.  ns_init borrows the field arrays and the workspace for the life of
 * the context; the library never calls hipMalloc.  It allocates a host
 * context, pinned host memory for the values the host tests (the CG scalars,
 * the per-block partials of grids of at most 8192 blocks, up to 128 KB, and
 * free bodies' force partials), one event and one capture-only stream, and
 * the recorded V-cycle graphs; ns_destroy releases them.  All device work is enqueued on the stream given to ns_init;
 * calls that return solver statistics or diagnostics synchronise that stream.
 * A context must not be used from two host threads at once.
 *
 * Errors.  Every call returns an ns_status and never aborts the process.
 * ns_last_error gives a message for the last failing call on a context.
 */
#ifndef NS_H
#define NS_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NS_OK = 0,
  NS_EINVAL = -1,   /* bad argument: sizes, null or misaligned pointer, too small workspace */
  NS_ENOCONV = -2,  /* projection hit max_iters before rtol; u and p hold the last iterate */
  NS_ENAN = -3,     /* a non-finite value appeared in the solve */
  NS_EHIP = -4,     /* a HIP runtime call failed */
  NS_ESTATE = -5,   /* call out of order (e.g. projection before momentum) */
  NS_EUNSTABLE = -6 /* the step left the scheme's stability bound: with consistent
                       transport a carried face density came out <= 0, which
                       happens once the outflow Courant number passes 1/2 (take
                       dt from ns_cfl_dt); u and p are not updated */
} ns_status;

typedef enum { NS_PREC_FP64 = 0, NS_PREC_MIXED = 1 } ns_prec;   /* V-cycle precision   */
/* Projection guess.  NS_X0_AUTO: the learned guess only where it pays.  A
 * step runs the network (a trial) on the first projection, whenever the
 * iterations the learned guess saved on its trials, at the last solve's time
 * per CG iteration, outweigh the inference's device time, and otherwise on
 * every 8th step; the other steps start from p_prev without inference.  On a
 * trial the residual of p_prev is measured beside the learned guess's, and
 * the iterations saved are their log ratio over the last solve's log
 * contraction per iteration (averaged over trials, the latest weighted 1/2). */
typedef enum { NS_X0_ZERO = 0, NS_X0_PREV = 1, NS_X0_LEARNED = 2, NS_X0_AUTO = 3 } ns_x0;

/* A rigid body given by an analytic level set psi (negative inside), built
 * from primitive distance functions with min/max (Sec. "Interface tracking":
 * psi is reset directly from the geometry each step).  A heave offset zeta
 * shifts it along z; its velocity is u_b = dzeta/dt e_z (eq_ub_velocity
 * restricted to heave).
 *   Prescribed heave (free_heave = 0): zeta(t) = A sin(omega t + phase).
 *   Free heave (free_heave = 1, Sec. "Fluid-structure coupling"): zeta and
 *   zdot start at zeta0, zdot0 and follow eqn_newton_u,
 *     m (zdot^{n+1} - zdot^n) / dt = F_hydro,z - m g + F_PTO,
 *   with a linear-damper power take-off F_PTO = -c zdot^{n+1} and
 *   zeta^{n+1} = zeta^n + dt zdot^{n+1}.  F_hydro is eqn_int_fh summed over
 *   the body's stair-step surface (faces across which its psi changes sign)
 *   from the pressure, velocity and viscosity that the previous step left;
 *   on the first ns_step, from the fields it starts from (a caller driving
 *   the three stages alone gets, on its first momentum_step, the force with
 *   the viscosity of the level set as that call finds it).  momentum_step
 *   advances the heave once per call; projection_solve computes the next
 *   force.  mass is per metre of depth in a 2-D tank. */
typedef struct {
  int kind;           /* 0: box in the (x,z) plane, psi = max(|x-xc|-a, |z-zc|-b)
                         1: vertical cylinder, psi = max(r - R, z_bot - z, z - z_top) */
  double c[3];        /* kind 0: (xc, unused, zc); kind 1: (xc, yc, unused)            */
  double half[3];     /* kind 0: (a, unused, b);  kind 1: (R, z_bot, z_top)            */
  double heave_amp, heave_omega, heave_phase;   /* prescribed heave                    */
  int free_heave;     /* 0: prescribed heave; 1: free heave                           */
  double mass;        /* m (kg), > 0 for a free body                                  */
  double pto_damping; /* c (N s/m), >= 0                                              */
  double zeta0, zdot0;/* initial heave offset (m) and velocity (m/s) of a free body   */
} ns_body;

typedef struct {
  int nx, ny, nz;              /* cells; ny == 1 for a 2-D (x,z) tank; nx >= 2,      */
                               /* ny >= 1, nz >= 2, and no face array (nx+1) ny nz,  */
                               /* nx (ny+1) nz, nx ny (nz+1) above 2e9 entries       */
  double h;                    /* uniform spacing (m), > 0                           */
  double rho_w, mu_w;          /* water (liquid) density and viscosity              */
  double rho_a, mu_a;          /* air (gas)                                         */
  double rho_s, mu_s;          /* solid                                             */
  double g;                    /* gravity magnitude, acting along -z                */
  double n_cells;              /* Heaviside half-width in cells (eqn_Hflow)         */
  double inv_kappa_p;          /* 1/kappa_p of eqn_brinkman_force                   */
  double proj_penalty_weight;  /* w in beta = 1/(rho_f + w dt chi_f/kappa_p)        */
  int n_bodies;                /* 0..4                                              */
  ns_body body[4];
  int reinit_iters;            /* pseudo-time steps of the reinitialisation         */
  double reinit_dtau_over_h;   /* pseudo-time step / h (<= 1/3 in 3-D)              */
  int nu_pre, nu_post;         /* red-black sweep pairs before / after coarse grid  */
  int coarse_sweeps;           /* sweep pairs each way on the coarsest level        */
  int max_iters;               /* CG iteration cap                                  */
  double rtol;                 /* stop when ||b - A p||_2 <= rtol ||b||_2           */
  int prec;                    /* ns_prec                                           */
  int x0;                      /* ns_x0                                             */
  double p_scale;              /* P0 of the learned guess p0 = p_prev + P0 delta,
                                  e.g. rho_w g depth; > 0 when x0 = NS_X0_LEARNED
                                  or NS_X0_AUTO                                    */
  /* Numerical wave tank (Sec. "Numerical wave tank"); all zero: a closed
   * tank.  The tank generates the linear waves listed in waves[]:
   * eta = sum a cos(kappa x - omega t + phase), with potential-flow velocity
   * u = sum a omega cosh(kappa z)/sinh(kappa d) cos(.), w = sum a omega
   * sinh(kappa z)/sinh(kappa d) sin(.) under the surface (z from the bed),
   * none above it, v = 0.
   *   gen_len > 0: the inlet face x = 0 carries that u (in place of a wall),
   *     and after each step a generation zone x in [0, gen_len] relaxes u, v,
   *     w and sigma toward the wave at t^{n+1}: phi <- a phi + (1 - a) phi_t,
   *     a = 1 - (exp(chi^3.5) - 1)/(e - 1), chi = 1 - x / gen_len.
   *   damp_len > 0: a damping zone x in [L - damp_len, L] relaxes them toward
   *     still water (u = v = w = 0, sigma = z - depth), chi = (x - L +
   *     damp_len) / damp_len.
   *   vort_width > 0: the predictor adds the damping force -g u, g = rho_a
   *     (cos(pi z~) + 1)/(4 dt), z~ = (z - z_top)/vort_width >= -1, implicitly. */
  double depth;                /* still-water depth d (m), > 0 with zones       */
  double gen_len, damp_len;    /* relaxation zone lengths (m), >= 0             */
  double vort_width;           /* vorticity damping zone width (m), >= 0        */
  int n_waves;                 /* 0..64                                         */
  struct { double a, kappa, omega, phase; } waves[64];
  /* 1: the predictor takes the conservative form of eqn_c_discrete_momentum
   * with consistent mass/momentum transport (Sec. "Multiphase incompressible
   * Navier-Stokes solution"): the face density starts from the density of
   * the level set the step starts from and is carried over the step by the
   * same limited upwind mass fluxes that carry momentum, rb = rho^n_f -
   * dt/h sum m, (rb u* - rho^n_f u^n)/dt + sum(m v)/h = forces, and beta
   * uses rb.  ns_step takes rho^n from the fields it starts from; a caller
   * driving the stages alone gets, on its first momentum_step, the density
   * of the level set as that call finds it.  0: the advective form. */
  int consistent;
  /* > 0: the viscous term is Crank-Nicolson (Sec. "Time stepping scheme"):
   * half of it at t^n, half at the predicted velocity, each face solving
   *   D_f u*_f - 1/2 L(u*)_f = rhs_f
   * with D_f the implicit diagonal of the predictor and L the viscous
   * operator.  The system is solved by point-Jacobi sweeps from the explicit
   * predictor, u_f <- (rhs_f + 1/2 (L(u)_f + a_f u_f))/(D_f + 1/2 a_f), a_f
   * the magnitude of L's diagonal; walls and the inlet keep their values.
   * cn_sweeps sweeps run between convergence checks: after each batch the
   * largest change of the batch's last sweep over all faces is compared with
   * cn_tol times the largest |u*|, and batches continue until it is below,
   * at most 64 sweeps in all (then momentum_step returns NS_ENOCONV).  Each
   * sweep contracts the error by a factor of order nu dt/h^2.  A check
   * synchronises the stream once.  0: explicit viscous term.  At most 64. */
  int cn_sweeps;
  double cn_tol;               /* > 0 when cn_sweeps > 0, e.g. 1e-10            */
} ns_params;

/* The caller's state arrays (device, FP64, layouts above); read and written
 * in place.  p holds the full pressure p^{n+1/2}; on entry to a step it is the
 * previous step's pressure, used as the initial guess when x0 = NS_X0_PREV. */
typedef struct {
  double* sigma;
  double* u;
  double* v;
  double* w;
  double* p;
} ns_fields;

typedef struct {
  int iters;               /* CG iterations of the last projection                    */
  int converged;           /* 1 if the true residual met rtol                         */
  double rel_resid0;       /* ||b - A x0|| / ||b||                                    */
  double rel_resid;        /* last recursive residual / ||b||                         */
  double true_rel_resid;   /* ||b - A p|| / ||b|| recomputed at exit                  */
  double ms;               /* wall time of the call, stream-synchronised (ms)         */
  int x0_fallback;         /* 1 if the learned guess was non-finite and p_prev was used */
  int cn_sweeps;           /* Crank-Nicolson sweeps of the step's predictor (0: explicit) */
  /* Device time per phase (ms) while ns_phase_timing is on, else zeros:
   * [0] level set (advection + reinitialisation), [1] properties and
   * predictor, [2] projection set-up (right-hand side, initial guess with
   * any network inference), [3] the CG solve, [4] velocity correction (with
   * the wave tank's zones and free bodies' forces), [5] the whole step;
   * [0], [1] and [5] are filled by ns_step only; [6], [7] are 0. */
  double t_ms[8];
  int x0_used;             /* the guess the solve started from: NS_X0_ZERO, _PREV or
                              _LEARNED (a non-finite learned guess counts as _PREV) */
  double x0_gain;          /* NS_X0_AUTO: CG iterations the learned guess is estimated
                              to save over p_prev after this step's update; else 0 */
} ns_stats;

/* Internal arrays a caller may inspect or fill through ns_buffer (device
 * pointers into the workspace; element counts as listed). */
typedef enum {
  NS_BUF_US = 0,    /* u* (predictor), u-face count, FP64      */
  NS_BUF_VS = 1,    /* v*                                      */
  NS_BUF_WS = 2,    /* w*                                      */
  NS_BUF_BX = 3,    /* beta on x faces (level 0), FP64        */
  NS_BUF_BY = 4,
  NS_BUF_BZ = 5,
  NS_BUF_RHS = 6,   /* b = -div(u*)/dt, cells, FP64            */
  NS_BUF_RHO = 7,   /* rho at cell centres (t^{n+1}), FP64     */
  NS_BUF_MU = 8,
  NS_BUF_CHI = 9,
  NS_BUF_RHOFLOW = 10,
  NS_BUF_BXF = 11,  /* FP32 copies of the level-0 beta (written by momentum_step) */
  NS_BUF_BYF = 12,
  NS_BUF_BZF = 13,
  NS_BUF_COUNT = 14
} ns_buffer_id;

typedef struct ns_ctx ns_ctx;

/* Bytes of device workspace ns_init needs for these parameters (0 if the
 * parameters are invalid). */
size_t ns_workspace_bytes(const ns_params* params);

/* Validate params, carve the workspace (device, >= ns_workspace_bytes,
 * 256-byte aligned) and bind the fields.  hip_stream is a hipStream_t (NULL:
 * the default stream).  On success *out owns a new context. */
ns_status ns_init(const ns_params* params, ns_fields fields, void* workspace, size_t ws_bytes,
                  void* hip_stream, ns_ctx** out);

/* Step 1: sigma^n -> sigma^{n+1} in place (advection by u^n over dt, then
 * reinit_iters relaxation steps). */
ns_status levelset_advect_reinit(ns_ctx* ctx, double dt);

/* Step 2: properties at t_np1 from the current sigma and the bodies, then
 * the predictor u* (internal buffer NS_BUF_US/VS/WS) and the projection
 * coefficients beta (NS_BUF_BX/BY/BZ) from u^n. */
ns_status momentum_step(ns_ctx* ctx, double dt, double t_np1);

/* Step 3: b = -div(u*)/dt, solve A p = b (guess from params.x0), then
 * u^{n+1} = u* - dt beta grad p into the fields.  stats may be NULL.
 * Returns NS_ENOCONV if max_iters was reached before rtol. */
ns_status projection_solve(ns_ctx* ctx, double dt, ns_stats* stats);

/* Steps 1-3 in order for t^n -> t^n + dt. */
ns_status ns_step(ns_ctx* ctx, double dt, double t_n, ns_stats* stats);

/* Solve A p = b with the beta and b currently in NS_BUF_BX/BY/BZ and
 * NS_BUF_RHS (caller-filled or from momentum_step/projection), p = fields.p
 * holding the initial guess; no velocity correction. */
ns_status ns_pcg_solve(ns_ctx* ctx, ns_stats* stats);

/* y = A x with the current level-0 beta (x, y: device, cells). */
ns_status ns_apply_A(ns_ctx* ctx, const double* x, double* y);

/* z = M r: one V-cycle of the current hierarchy (rebuilt from the level-0
 * beta) in the precision of params.prec (r, z: device, cells). */
ns_status ns_vcycle(ns_ctx* ctx, const double* r, double* z);

/* Device pointer and element count of an internal array. */
ns_status ns_buffer(ns_ctx* ctx, int which, void** dev_ptr, size_t* count);

/* State of body m (host memory, no device work): out[0] zeta, out[1] zdot,
 * out[2..4] the last hydrodynamic force (Fx, Fy, Fz) of eqn_int_fh, out[5]
 * the last F_PTO.  For a prescribed body zeta and zdot are those of the last
 * momentum_step and the force entries are 0.  NS_EINVAL for a bad m. */
ns_status ns_body_state(ns_ctx* ctx, int body, double out[6]);

/* out[0] max|div_h u|, out[1] water volume sum (1 - H(sigma)) h^d,
 * out[2] kinetic energy 1/2 sum rho^flow |u_c|^2 h^d, out[3] max|u_face|.
 * out is host memory; synchronises the stream. */
ns_status ns_diagnostics(ns_ctx* ctx, double out[4]);

/* How the CG loop issues its preconditioner.  Each V-cycle, with the dot
 * product that follows it, is a segment of some thirty kernels.
 * NS_LAUNCH_GRAPH (the default): each segment is recorded once per context
 * into a HIP graph for each set of vectors the loop uses it with (at most
 * 16 graphs; recording runs nothing, and the graphs live until ns_destroy),
 * and every later use is one graph launch on the context's stream.
 * NS_LAUNCH_STREAM: the same kernels with the same arguments launched one by
 * one, so results are bitwise the same in both modes.  A graph launch saves
 * the host some thirty kernel launches for a fixed device-side cost of a few
 * microseconds, which keeps the device fed on slow hosts.  While kernel
 * timing is enabled the loop launches kernel by kernel.  If recording a
 * graph fails, the context falls back to NS_LAUNCH_STREAM for the rest of
 * its life and the solve continues.  NS_EINVAL for another value. */
typedef enum {
  NS_LAUNCH_STREAM = 0,
  NS_LAUNCH_GRAPH = 1
} ns_launch_mode;
ns_status ns_set_launch_mode(ns_ctx* ctx, int mode);

/* How the finest level runs the red-black sweeps that follow the first pass
 * of each smoothing (the red pass of one sweep and the black pass after it):
 * fused = 1 as one launch that reads each face coefficient once, the black
 * values taking theirs from the red values' loads; fused = 0 as two colour
 * passes.  The fused launch applies to 3-D levels with ny, nz >= 4 and at
 * least 32 cell pairs per row.  ns_create picks the two passes: the fused
 * launch, whose planes are a chain of dependent steps, pays only for an FP64
 * cycle on levels of at least 2^24 cells whose passes load every face, and
 * there the line tables (ns_set_face_tables) are on, a colour pass loads few
 * faces, and two passes take less time.
 * Results are bitwise the same either way.  Recorded V-cycle graphs are released and recorded again on their
 * next use (synchronises the stream).  NS_EINVAL for another value, or
 * fused = 1 on a grid it does not apply to. */
ns_status ns_set_fine_sweep(ns_ctx* ctx, int fused);
/* *fused = 1 if the finest level's sweeps run as one launch, else 0.
 * NS_EINVAL for a null argument. */
ns_status ns_get_fine_sweep(const ns_ctx* ctx, int* fused);

/* Line tables of the finest level's face coefficients (on = 1; ns_create
 * turns them on for a finest level of at least 2^21 cells, where they pay:
 * a kernel reading them waits one cache round trip for its lines' entries,
 * which a smaller, latency-bound level cannot hide).  Each solve first
 * records, for every x-line of each face array
 * (the faces along x at one j, k), whether all its faces hold one value (for
 * x-faces: every interior face, the two wall faces being zero), and that
 * value.  In a two-phase tank most lines lie wholly in water or wholly in
 * air, where 1/rho is one constant; the finest level's kernels then read one
 * table entry for such a line instead of its faces, about a third of the
 * bytes a CG iteration moves.  The face arrays themselves are unchanged and
 * results are bitwise the same either way.  Recorded V-cycle graphs are
 * released and recorded again on their next use (synchronises the stream).
 * NS_EINVAL for another value. */
ns_status ns_set_face_tables(ns_ctx* ctx, int on);
/* *on = 1 if the line tables are used, else 0.  NS_EINVAL for a null argument. */
ns_status ns_get_face_tables(const ns_ctx* ctx, int* on);

/* Kernel timing, a profiling aid.  While enabled for a kernel, each of its
 * next max_launches dispatches on the context's stream carries a start and
 * stop HIP event recorded by the dispatch itself (hipExtLaunchKernelGGL),
 * so the elapsed time is the kernel's own execution.  max_launches <= 0
 * disables.  Events are host-API objects; no device memory is allocated. */
typedef enum {
  NS_TIME_SMOOTH0 = 0,   /* the finest-level smoother: the fused red-black sweep where it
                            is used (ns_set_fine_sweep), else one colour pass      */
  NS_TIME_SPMV = 1       /* the CG operator application with its dot product       */
} ns_timed_kernel;
ns_status ns_timing_enable(ns_ctx* ctx, int kernel, int max_launches);

/* Sum of the recorded kernel durations (ms) and their count since the last
 * read; synchronises the stream and restarts the count. */
ns_status ns_timing_read(ns_ctx* ctx, double* total_ms, int* launches);

/* Average duration (ms) of `reps` back-to-back dispatches of one kernel on
 * the context's stream, bracketed by one pair of HIP events: the finest-level
 * smoother pass (one colour, params.prec precision) or the CG operator
 * application.  Runs on the current coefficients, read as a solve reads
 * them (the line tables built first when they are on), with vectors that
 * are dead between steps, so it may be called between time steps without
 * changing the state; synchronises the stream.  Needs momentum_step (or filled
 * coefficients) first, else NS_ESTATE. */
ns_status ns_time_kernel(ns_ctx* ctx, int kernel, int reps, double* avg_ms);

/* ---------------------------------------------------------------------
 * Learned initial guess (a small 3-level convolutional encoder-decoder,
 * 16/32/64 channels, 3x3x3 kernels, bfloat16 on the matrix cores with FP32
 * accumulation) mapping four features of the projection to a correction
 * delta: p0 = p_prev + P0 delta.  The features are the right-hand side
 * b h^2 rho_w / P0, the density as ln(rho/rho_w)/ln(rho_a/rho_w), p_prev / P0
 * and the residual (b - A p_prev) h^2 rho_w / P0.  The CG solve that follows
 * is unchanged and meets the same rtol whatever the guess.
 * Parameters are exchanged as FP32 in a canonical flat order: for each of the
 * six layers (4->16, 16->32, 32->64, 96->32, 48->16 3x3x3, 16->1 1x1x1) the
 * weights w[co][ci][kz][ky][kx] then the biases b[co].
 * ------------------------------------------------------------------- */
typedef struct ns_net ns_net;

/* Number of FP32 parameters in the canonical order. */
size_t ns_net_param_count(void);

/* Device workspace for a network on an nx*ny*nz grid (each a multiple of 4,
 * >= 4); training != 0 adds gradients, optimiser state and backward
 * buffers.  0 when the sizes are invalid. */
size_t ns_net_workspace_bytes(int nx, int ny, int nz, int training);

/* Bind a workspace (device, 256-byte aligned, caller-owned) and a stream.
 * Parameters start at zero until ns_net_set_params. */
ns_status ns_net_create(int nx, int ny, int nz, int training, void* workspace, size_t ws_bytes,
                        void* hip_stream, ns_net** out);
void ns_net_destroy(ns_net* net);
const char* ns_net_last_error(ns_net* net);

/* Upload / download the FP32 parameters (HOST arrays of
 * ns_net_param_count() floats); set_params also resets the optimiser. */
ns_status ns_net_set_params(ns_net* net, const float* host_params, size_t n);
ns_status ns_net_get_params(ns_net* net, float* host_params, size_t n);

/* Gradients of the last ns_net_train_step (host array, canonical order). */
ns_status ns_net_get_grads(ns_net* net, float* host_grads, size_t n);

/* Load four feature channels (device FP32, channel-first, 4*nx*ny*nz). */
ns_status ns_net_set_input(ns_net* net, const float* feat4);

/* Run the network on the loaded input; delta_out (device FP32, nx*ny*nz)
 * receives delta when not NULL. */
ns_status ns_net_forward(ns_net* net, float* delta_out);

/* One training step on one sample (device FP32 features, target delta* =
 * (p* - p_prev)/P0 and the sample's face coefficients beta on x, y, z faces,
 * layouts as the velocity faces): forward, the energy-norm loss
 *   L = e'Ae / t'At,  e = t - delta,
 * i.e. ||p* - p0||_A^2 / ||p* - p_prev||_A^2 (below 1 when the guess beats
 * p_prev in the norm CG minimises), backward, and when update != 0 an Adam
 * step (betas 0.9/0.999, eps 1e-8) of rate lr.  *loss gets L (synchronises). */
ns_status ns_net_train_step(ns_net* net, const float* feat4, const float* target, const float* beta_x,
                            const float* beta_y, const float* beta_z, float lr, int update, double* loss);

/* Use `net` (same grid) for x0 = NS_X0_LEARNED or NS_X0_AUTO in this context. */
ns_status ns_attach_net(ns_ctx* ctx, ns_net* net);

/* The four features of the projection about to be solved (after
 * momentum_step), with p_prev (device FP64 cells) as the previous pressure,
 * into feat4 (device FP32, 4 * cells, channel-first). */
ns_status ns_features(ns_ctx* ctx, double dt, const double* p_prev, float* feat4);

/* Training target t = (p - p_prev) / P0 of the solved pressure fields.p
 * (device FP64 p_prev, device FP32 t). */
ns_status ns_target(ns_ctx* ctx, const double* p_prev, float* t);

/* Time step of the CFL rule (Sec. "Time stepping scheme": the paper's runs
 * keep the Courant number at or below 0.5) on the current fields:
 *   *dt_out = min(cfl h / m, dt_max),  m = max over cells of |u_c| + |v_c| + |w_c|,
 * each cell velocity the mean of its two faces (dt_max when m = 0).  The
 * maximum is taken on the device by an order-independent reduction, so the
 * result does not depend on the launch.  dt_out is host memory; synchronises
 * the stream.  NS_EINVAL unless cfl > 0 and dt_max > 0; NS_ENAN if a
 * velocity is not finite. */
ns_status ns_cfl_dt(ns_ctx* ctx, double cfl, double dt_max, double* dt_out);

/* The CFL rule of ns_cfl_dt for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It needs no context and allocates nothing: u, v, w are the
 * face velocities of an nx*ny*nz grid of spacing h (device, FP64, the
 * layouts above, same limits on the sizes as ns_params), and the time step
 * min(cfl h / m, dt_max) (dt_max when m = 0; NaN when a velocity is not
 * finite) is stored to dt_dev, one caller-owned device double, in stream
 * order on hip_stream; the call does not wait for it.  Its scratch (the
 * per-block maxima, 16 KiB, every grid size fits) is a device array of the
 * library's own, one per GPU, held until the process ends: calls that
 * overlap on one GPU (other streams or threads) race on it.  The result is
 * bit for bit that of ns_cfl_dt.  NS_EINVAL for bad sizes, a non-positive h,
 * cfl or dt_max, or a null or misaligned pointer; NS_EHIP if the current
 * device cannot be queried or the launch fails. */
ns_status ns_cfl_dt_noalloc(int nx, int ny, int nz, double h, const double* u, const double* v, const double* w,
                            double cfl, double dt_max, double* dt_dev, void* hip_stream);

/* Per-phase device timing of the steps (ns_stats.t_ms): on != 0 records HIP
 * events between the phases of every later call (host-API objects, created
 * on the first use; no device memory); 0 stops it. */
ns_status ns_phase_timing(ns_ctx* ctx, int on);

/* Number of multigrid levels for these sizes. */
int ns_num_levels(int nx, int ny, int nz);

const char* ns_last_error(ns_ctx* ctx);

/* Release the context (host memory only; the caller's device memory is
 * untouched).  NULL is accepted. */
void ns_destroy(ns_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
