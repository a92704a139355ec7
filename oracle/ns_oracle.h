/* Oracle for the two-phase Brinkman-penalised level-set Navier-Stokes step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation used by the tests and by the CPU-baseline timing to check
 * the GPU library.  It shares no code, header or constant with the GPU
 * library, and nothing on the product path may call it.
 *
 * Grid (Sec. "Spatial discretization"): nx x ny x nz cells of size h, cell
 * (i,j,k) centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h); x-faces at x = i h,
 * y-faces at y = j h, z-faces at z = k h.  Arrays are x-fastest:
 *   cell  c[i + nx*(j + ny*k)]
 *   u     u[i + (nx+1)*(j + ny*k)]      (nx+1)*ny*nz
 *   v     v[i + nx*(j + (ny+1)*k)]      nx*(ny+1)*nz
 *   w     w[i + nx*(j + ny*k)]          nx*ny*(nz+1)
 * A 2-D tank in the (x, z) plane is ny == 1.  Gravity acts along -z.
 */
#ifndef NS_ORACLE_H
#define NS_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int kind;            /* 0: box in the (x,z) plane, 1: vertical cylinder          */
  double c[3];         /* box: (xc, -, zc); cylinder: (xc, yc, -)                  */
  double half[3];      /* box: (a, -, b) half-widths; cylinder: (R, z_bot, z_top)  */
  double heave_amp, heave_omega, heave_phase;  /* zeta(t) = A sin(w t + phi)     */
  int free_heave;      /* 1: heave follows eqn_newton_u; zeta, zdot are its state  */
  double mass;         /* m of eqn_newton_u (per unit depth in 2-D)                */
  double pto_damping;  /* c of the linear-damper PTO force F_PTO = -c zdot         */
  double zeta, zdot;   /* heave offset and velocity of a free body                 */
} orc_body;

typedef struct {
  int nx, ny, nz;
  double h;
  double rho_w, mu_w, rho_a, mu_a, rho_s, mu_s, g;
  double n_cells;              /* Heaviside half-width in cells                  */
  double inv_kappa_p;          /* Brinkman 1/kappa_p                             */
  double proj_penalty_weight;  /* beta = 1/(rho + w dt chi/kappa_p)              */
  int n_bodies;
  orc_body body[4];
  int reinit_iters;
  double reinit_dtau_over_h;
  int nu_pre, nu_post, coarse_sweeps, max_iters;
  double rtol;
  int prec;                    /* 0: FP64 V-cycle, 1: FP32 V-cycle               */
  /* numerical wave tank (Sec. "Numerical wave tank"); zeros: a closed tank */
  double depth;                /* still-water depth d                            */
  double gen_len;              /* wave generation zone x in [0, gen_len]         */
  double damp_len;             /* wave damping zone x in [L - damp_len, L]       */
  double vort_width;           /* vorticity damping zone width below the top     */
  int n_waves;                 /* generated linear components (<= 64)            */
  double wave_a[64], wave_k[64], wave_om[64], wave_ph[64];
  int consistent;              /* 1: conservative predictor with consistent       */
                               /*    mass/momentum transport                     */
  int crank_nicolson;          /* 1: Crank-Nicolson viscous term, its system      */
                               /*    solved to convergence; 0: explicit           */
} orc_params;

typedef struct {
  int iters;
  double rel_resid0, rel_resid, true_rel_resid;
} orc_stats;

/* individual steps (each documented in ns_oracle.c) */
void orc_levelset_advect(const orc_params* P, const double* sigma, const double* u, const double* v,
                         const double* w, double dt, double* sigma_out);
void orc_reinit(const orc_params* P, const double* sigma0, double* sigma_out);
void orc_properties(const orc_params* P, const double* sigma, double t, double* rho, double* rho_flow,
                    double* mu, double* chi);
void orc_momentum(const orc_params* P, const double* u, const double* v, const double* w,
                  const double* sigma, double t_np1, double dt, double* us, double* vs, double* ws);
void orc_face_beta(const orc_params* P, const double* sigma, double t_np1, double dt, double* bx,
                   double* by, double* bz);
/* the conservative predictor with consistent transport: u* and the face
 * density rb carried over the step (rho_n: cell density at t^n) */
void orc_momentum_cons(const orc_params* P, const double* u, const double* v, const double* w,
                       const double* sigma, double t_np1, double dt, const double* rho_n, double* us, double* vs,
                       double* ws, double* rbx, double* rby, double* rbz);
void orc_face_beta_rho(const orc_params* P, const double* rbx, const double* rby, const double* rbz,
                       const double* sigma, double t_np1, double dt, double* bx, double* by, double* bz);
void orc_rhs(const orc_params* P, const double* us, const double* vs, const double* ws, double dt,
             double* b);
void orc_apply_A(int nx, int ny, int nz, double h, const double* bx, const double* by,
                 const double* bz, const double* x, double* y);
int  orc_num_levels(int nx, int ny, int nz);
void orc_vcycle(const orc_params* P, const double* bx, const double* by, const double* bz,
                const double* r, double* z);
int  orc_pcg(const orc_params* P, const double* bx, const double* by, const double* bz,
             const double* b, double* x, orc_stats* st);
void orc_correct(const orc_params* P, const double* us, const double* vs, const double* ws,
                 const double* p, const double* bx, const double* by, const double* bz, double dt,
                 double* u, double* v, double* w);
/* time step of the CFL rule on the current face velocities */
double orc_cfl_dt(const orc_params* P, const double* u, const double* v, const double* w, double cfl,
                  double dt_max);
/* status of the last predictor: bit 0 a non-positive transported density,
 * bit 1 a Crank-Nicolson solve that did not converge */
int  orc_last_flags(void);
/* orc_step / orc_step_from return 0, 1 when CG did not converge, 2 when the
 * consistent transport's face density came out non-positive (the step stops
 * after the predictor), 3 when the Crank-Nicolson solve did not converge */
int  orc_step(const orc_params* P, double* sigma, double* u, double* v, double* w, double* p,
              double dt, double t_n, int x0_prev, orc_stats* st);
int  orc_step_from(const orc_params* P, double* sigma, double* u, double* v, double* w, double* p,
                   double dt, double t_n, int x0_prev, const double* rho_n, orc_stats* st);
void orc_diagnostics(const orc_params* P, const double* sigma, const double* u, const double* v,
                     const double* w, double* out4);
/* hydrodynamic force on body m (eqn_int_fh); mu: cell viscosity; F: (Fx, Fy, Fz) */
void orc_hydro_force(const orc_params* P, int m, const double* p, const double* u, const double* v,
                     const double* w, const double* mu, double t, double* F);
/* relaxation zones of the numerical wave tank at time t, in place */
void orc_relax(const orc_params* P, double t, double* sigma, double* u, double* v, double* w);
/* heave update of a free body (eqn_newton_u, linear-damper PTO, implicit) */
void orc_heave_update(double mass, double pto_damping, double g, double dt, double fz, double* zeta,
                      double* zdot);

#ifdef __cplusplus
}
#endif
#endif
