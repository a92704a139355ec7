/* Oracle for one time step of the level-set, Brinkman-penalised, two-phase
 * incompressible Navier-Stokes solver (arXiv 2206.07732, Sec. "Continuous
 * equations of motion" through "Fluid-structure coupling").
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded FP64 reference that
 * the tests and the CPU-baseline timing use to check the GPU library.  It
 * shares no code with the GPU library.  Loops are written straight from the
 * equations; there is no tiling, fusion or reordering.
 *
 * Where the paper is silent the oracle takes these readings (all listed with
 * their reasons in the design notes of the repository):
 *   - boundary ghosts are the nearest interior value (index clamp): zero
 *     normal gradient for the level set and viscosity, free slip for
 *     tangential velocity; wall-normal faces carry zero velocity;
 *   - the top of the tank is open with p = 0 on the boundary face;
 *   - advection uses a Koren-limited (kappa = 1/3) upwind face value in
 *     place of the xsPPM7 scheme the paper cites;
 *   - the momentum predictor is explicit in advection and viscosity and
 *     implicit in the Brinkman term; the pressure follows from a
 *     non-incremental projection with beta = 1/(rho_f + w dt chi_f/kappa_p);
 *   - the projection is solved by flexible preconditioned CG with a V(2,2)
 *     red-black Gauss-Seidel multigrid cycle as preconditioner.
 */
#include "ns_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Built with -fopenmp (the CPU-baseline timing build only) the outer loops of
 * the grid passes are split over the host's cores, each thread a contiguous
 * block of planes; the dot products then sum per thread.  The build the tests
 * use has no OpenMP and runs every loop in order on one thread. */
#ifdef _OPENMP
#define ORC_PAR _Pragma("omp parallel for schedule(static)")
#else
#define ORC_PAR
#endif

/* --------------------------------------------------------------------------
 * indexing with clamped (nearest-interior) ghosts
 * ------------------------------------------------------------------------ */
static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* number of entries of a face array normal to direction c */
static size_t face_count(const orc_params* P, int c) {
  return (size_t)(P->nx + (c == 0)) * (size_t)(P->ny + (c == 1)) * (size_t)(P->nz + (c == 2));
}
static size_t ncell(const orc_params* P) { return (size_t)P->nx * P->ny * P->nz; }

/* cell value at (i,j,k), clamped to the grid */
static double cellv(const orc_params* P, const double* a, int i, int j, int k) {
  i = clampi(i, 0, P->nx - 1);
  j = clampi(j, 0, P->ny - 1);
  k = clampi(k, 0, P->nz - 1);
  return a[i + (size_t)P->nx * (j + (size_t)P->ny * k)];
}

/* face value of component c (array f) at face index (i,j,k), clamped */
static double facev(const orc_params* P, int c, const double* f, int i, int j, int k) {
  int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
  i = clampi(i, 0, mx - 1);
  j = clampi(j, 0, my - 1);
  k = clampi(k, 0, mz - 1);
  return f[i + (size_t)mx * (j + (size_t)my * k)];
}

/* --------------------------------------------------------------------------
 * smoothed Heaviside, eqn_Hflow / eqn_Hbody (Sec. "Density and viscosity
 * specification"): 0 below -eps, 1 above eps, smooth in between.
 * ------------------------------------------------------------------------ */
static double heaviside(double phi, double eps) {
  if (phi < -eps) return 0.0;
  if (phi > eps) return 1.0;
  return 0.5 * (1.0 + phi / eps + sin(M_PI * phi / eps) / M_PI);
}

/* --------------------------------------------------------------------------
 * body level set psi (Sec. "Interface tracking": reinitialised directly by
 * CSG min/max of primitive distance functions; negative inside) and the
 * rigid heave velocity u_b = zdot e_z (eq_ub_velocity reduced to heave).
 * ------------------------------------------------------------------------ */
static double body_psi_one(const orc_body* b, double x, double y, double z, double t, double* zdot) {
  double zeta = b->heave_amp * sin(b->heave_omega * t + b->heave_phase);
  *zdot = b->heave_amp * b->heave_omega * cos(b->heave_omega * t + b->heave_phase);
  if (b->free_heave) {  /* heave from the body's own state (eqn_newton_u) */
    zeta = b->zeta;
    *zdot = b->zdot;
  }
  if (b->kind == 0) {
    double dx = fabs(x - b->c[0]) - b->half[0];
    double dz = fabs(z - (b->c[2] + zeta)) - b->half[2];
    return fmax(dx, dz);
  }
  double r = sqrt((x - b->c[0]) * (x - b->c[0]) + (y - b->c[1]) * (y - b->c[1]));
  double below = (b->half[1] + zeta) - z;
  double above = z - (b->half[2] + zeta);
  return fmax(r - b->half[0], fmax(below, above));
}

/* union of bodies: psi = min over bodies; zdot of the body attaining it */
static double body_psi(const orc_params* P, double x, double y, double z, double t, double* zdot) {
  double best = INFINITY;
  *zdot = 0.0;
  for (int m = 0; m < P->n_bodies; ++m) {
    double zd;
    double s = body_psi_one(&P->body[m], x, y, z, t, &zd);
    if (s < best) {
      best = s;
      *zdot = zd;
    }
  }
  return best;
}

/* --------------------------------------------------------------------------
 * Limited upwind face value (Koren, kappa = 1/3 in smooth regions).
 * sU is the upwind cell, sUU the one behind it, sD the downwind cell.
 * ------------------------------------------------------------------------ */
static double koren(double sUU, double sU, double sD) {
  double dup = sU - sUU;
  double ddn = sD - sU;
  if (dup * ddn <= 0.0) return sU;
  double a = 2.0 * fabs(dup);
  double b = (2.0 * fabs(ddn) + fabs(dup)) / 3.0;
  double c = 2.0 * fabs(ddn);
  double m = fmin(a, fmin(b, c));
  return sU + 0.5 * (ddn > 0.0 ? m : -m);
}

/* --------------------------------------------------------------------------
 * Level-set advection (Sec. "Level set advection").  With one fixed-point
 * cycle per step (Sec. "Time stepping scheme": u^{n+1,0} = u^n,
 * sigma^{n+1,0} = sigma^n) the update is forward Euler:
 *   sigma* = sigma^n - dt Q(u^n, sigma^n),
 *   Q = div_h(u sigma_f) - sigma div_h(u)   (advective form u . grad sigma),
 * with sigma_f the limited upwind value on each face.
 * ------------------------------------------------------------------------ */
void orc_levelset_advect(const orc_params* P, const double* sigma, const double* u, const double* v,
                         const double* w, double dt, double* sigma_out) {
  const double* vel[3] = {u, v, w};
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  ORC_PAR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double sc = cellv(P, sigma, i, j, k);
        double flux = 0.0, divu = 0.0;
        for (int d = 0; d < 3; ++d) {
          int e[3] = {d == 0, d == 1, d == 2};
          /* face on the + side of the cell has index (i,j,k)+e_d, the - side (i,j,k) */
          double ap = facev(P, d, vel[d], i + e[0], j + e[1], k + e[2]);
          double am = facev(P, d, vel[d], i, j, k);
#define S(o) cellv(P, sigma, i + (o) * e[0], j + (o) * e[1], k + (o) * e[2])
          double sp = ap >= 0.0 ? koren(S(-1), S(0), S(1)) : koren(S(2), S(1), S(0));
          double sm = am >= 0.0 ? koren(S(-2), S(-1), S(0)) : koren(S(1), S(0), S(-1));
#undef S
          flux += ap * sp - am * sm;
          divu += ap - am;
        }
        double q = (flux - sc * divu) / P->h;
        sigma_out[i + (size_t)nx * (j + (size_t)ny * k)] = sc - dt * q;
      }
}

/* --------------------------------------------------------------------------
 * Reinitialisation (Sec. "Interface tracking": relaxation of Sussman et al.
 * to the steady state of d sigma/d tau + S(sigma0)(|grad sigma| - 1) = 0).
 * Jacobi pseudo-time steps of size dtau with the first-order Godunov upwind
 * gradient and the smoothed sign S = sigma0 / sqrt(sigma0^2 + h^2).
 * ------------------------------------------------------------------------ */
void orc_reinit(const orc_params* P, const double* sigma0, double* sigma_out) {
  const size_t n = ncell(P);
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h, dtau = P->reinit_dtau_over_h * h;
  double* cur = (double*)malloc(n * sizeof(double));
  double* nxt = (double*)malloc(n * sizeof(double));
  memcpy(cur, sigma0, n * sizeof(double));
  for (int it = 0; it < P->reinit_iters; ++it) {
    ORC_PAR
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t c = i + (size_t)nx * (j + (size_t)ny * k);
          double s0 = sigma0[c];
          double sgn = s0 / sqrt(s0 * s0 + h * h);
          double sc = cur[c];
          double g2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            int e[3] = {d == 0, d == 1, d == 2};
            double a = (sc - cellv(P, cur, i - e[0], j - e[1], k - e[2])) / h;  /* backward */
            double b = (cellv(P, cur, i + e[0], j + e[1], k + e[2]) - sc) / h;  /* forward  */
            double t1, t2;
            if (sgn > 0.0) {
              t1 = fmax(a, 0.0);
              t2 = fmin(b, 0.0);
            } else {
              t1 = fmin(a, 0.0);
              t2 = fmax(b, 0.0);
            }
            g2 += fmax(t1 * t1, t2 * t2);
          }
          nxt[c] = (sgn == 0.0) ? sc : sc - dtau * sgn * (sqrt(g2) - 1.0);
        }
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  memcpy(sigma_out, cur, n * sizeof(double));
  free(cur);
  free(nxt);
}

/* --------------------------------------------------------------------------
 * Material properties (eqn_ls_flow, eqn_ls_solid): flowing-phase property
 * from sigma, then the solid correction from psi; chi = 1 - H_body
 * (Sec. "Fluid-structure coupling").  Evaluated at cell centres at time t.
 * ------------------------------------------------------------------------ */
void orc_properties(const orc_params* P, const double* sigma, double t, double* rho, double* rho_flow,
                    double* mu, double* chi) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h, eps = P->n_cells * h;
  ORC_PAR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = i + (size_t)nx * (j + (size_t)ny * k);
        double zd;
        double psi = body_psi(P, (i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h, t, &zd);
        double hf = heaviside(sigma[c], eps);
        double hb = heaviside(psi, eps);
        double rf = P->rho_w + (P->rho_a - P->rho_w) * hf;
        double mf = P->mu_w + (P->mu_a - P->mu_w) * hf;
        if (rho_flow) rho_flow[c] = rf;
        if (rho) rho[c] = P->rho_s + (rf - P->rho_s) * hb;
        if (mu) mu[c] = P->mu_s + (mf - P->mu_s) * hb;
        if (chi) chi[c] = 1.0 - hb;
      }
}

/* is face (i,j,k) of component c a wall face (zero normal velocity)? The
 * top z-face (k == nz) is open, every other boundary face is a wall. */
static int is_wall_face(const orc_params* P, int c, int i, int j, int k) {
  if (c == 0) return i == 0 || i == P->nx;
  if (c == 1) return j == 0 || j == P->ny;
  return k == 0;
}

/* --------------------------------------------------------------------------
 * Numerical wave tank (Sec. "Numerical wave tank").
 * Target wave: the superposition of linear components (Sec. "Regular waves"
 * and "Irregular waves") a_i cos(k_i x - om_i t + ph_i), with potential-flow
 * velocity under the surface (z from the bed) and none above it.
 * ------------------------------------------------------------------------ */
static double wave_eta(const orc_params* P, double x, double t) {
  double eta = 0.0;
  for (int q = 0; q < P->n_waves; ++q) eta += P->wave_a[q] * cos(P->wave_k[q] * x - P->wave_om[q] * t + P->wave_ph[q]);
  return eta;
}

/* horizontal (c = 0) or vertical (c = 2) target velocity at (x, z, t); v = 0 */
static double wave_vel(const orc_params* P, int c, double x, double z, double t) {
  if (c == 1 || z >= P->depth + wave_eta(P, x, t)) return 0.0;
  double s = 0.0;
  for (int q = 0; q < P->n_waves; ++q) {
    double k = P->wave_k[q], th = k * x - P->wave_om[q] * t + P->wave_ph[q];
    double amp = P->wave_a[q] * P->wave_om[q] / sinh(k * P->depth);
    s += (c == 0) ? amp * cosh(k * z) * cos(th) : amp * sinh(k * z) * sin(th);
  }
  return s;
}

/* relaxation weight of the relaxation-zone method the tank uses (Jacobsen et
 * al.): 1 at the zone's inner edge (chi = 0), 0 at the tank end (chi = 1) */
static double relax_alpha(double chi) { return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / (exp(1.0) - 1.0); }

/* vorticity damping coefficient g(z~) = rho_a (cos(pi z~) + 1) / (4 dt),
 * z~ = (z - z_top) / width over the top `width` of the tank, 0 below it */
static double vort_damp(const orc_params* P, double z, double dt) {
  if (P->vort_width <= 0.0) return 0.0;
  double zt = (z - P->nz * P->h) / P->vort_width;
  if (zt < -1.0) return 0.0;
  return P->rho_a * (cos(M_PI * zt) + 1.0) / (4.0 * dt);
}

/* The zones after each step: every field phi in them becomes
 * alpha phi + (1 - alpha) phi_target, with the target wave in the
 * generation zone [0, gen_len] (chi = 1 - x / gen_len) and still water in
 * the damping zone [L - damp_len, L] (chi = (x - L + damp_len) / damp_len). */
static int relax_weight(const orc_params* P, double x, int* gen, double* alpha) {
  double L = P->nx * P->h;
  if (P->gen_len > 0.0 && x <= P->gen_len) {
    *gen = 1;
    *alpha = relax_alpha(1.0 - x / P->gen_len);
    return 1;
  }
  if (P->damp_len > 0.0 && x >= L - P->damp_len) {
    *gen = 0;
    *alpha = relax_alpha((x - (L - P->damp_len)) / P->damp_len);
    return 1;
  }
  return 0;
}

void orc_relax(const orc_params* P, double t, double* sigma, double* u, double* v, double* w) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h;
  double* vel[3] = {u, v, w};
  int gen;
  double al;
  for (int c = 0; c < 3; ++c) {
    int mx = nx + (c == 0), my = ny + (c == 1), mz = nz + (c == 2);
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          double x = (c == 0) ? i * h : (i + 0.5) * h;
          double z = (c == 2) ? k * h : (k + 0.5) * h;
          if (!relax_weight(P, x, &gen, &al)) continue;
          size_t f = i + (size_t)mx * (j + (size_t)my * k);
          double target = gen ? wave_vel(P, c, x, z, t) : 0.0;
          vel[c][f] = al * vel[c][f] + (1.0 - al) * target;
        }
  }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double x = (i + 0.5) * h, z = (k + 0.5) * h;
        if (!relax_weight(P, x, &gen, &al)) continue;
        size_t c = i + (size_t)nx * (j + (size_t)ny * k);
        double target = z - (P->depth + (gen ? wave_eta(P, x, t) : 0.0));
        sigma[c] = al * sigma[c] + (1.0 - al) * target;
      }
}

/* --------------------------------------------------------------------------
 * Momentum predictor (eqn_c_discrete_momentum with the Brinkman term
 * eqn_bp_discrete taken implicitly, gravity on the flowing density; the
 * pressure gradient is left to the projection):
 *   (rho_f/dt + chi_f/kp) u*_f = rho_f (u^n_f/dt - (u.grad u)_f)
 *                                + (div mu (grad u + grad u^T))_f
 *                                + rho^flow_f g_f + chi_f/kp u_b,f
 * Properties are those at t^{n+1} (from sigma^{n+1}); advection and
 * viscous stress use u^n.  Face values of rho, rho^flow and chi are the
 * mean of the two adjacent cells; edge viscosities the mean of four.
 * ------------------------------------------------------------------------ */
/* Viscous stress of component c along direction d at face (i, j, k),
 * ((tau_+) - (tau_-))/h with tau = mu (du_c/dx_d + du_d/dx_c) on the edges
 * (mean of four cell viscosities) or 2 mu du_c/dx_c at the cell centres
 * (d = c).  diag (may be NULL) receives the magnitude of the coefficient of
 * the face's own value in the interior stencil. */
static double visc_dir(const orc_params* P, const double* mu, const double* const F[3], int c, int d, int i, int j,
                       int k, double* diag) {
  const double h = P->h;
  int ec[3] = {c == 0, c == 1, c == 2};
  int ed[3] = {d == 0, d == 1, d == 2};
#define FV(o) facev(P, c, F[c], i + (o) * ed[0], j + (o) * ed[1], k + (o) * ed[2])
  double tp, tm;
  if (d == c) {
    /* normal stress 2 mu du_c/dx_c at the cell centres either side */
    double mup = cellv(P, mu, i, j, k);
    double mum = cellv(P, mu, i - ec[0], j - ec[1], k - ec[2]);
    tp = 2.0 * mup * (FV(1) - FV(0)) / h;
    tm = 2.0 * mum * (FV(0) - FV(-1)) / h;
    if (diag) *diag = 2.0 * (mup + mum) / (h * h);
  } else {
    /* shear stress mu (du_c/dx_d + du_d/dx_c) on the edges either side */
    double mep = 0.25 * (cellv(P, mu, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, mu, i, j, k) +
                         cellv(P, mu, i - ec[0] + ed[0], j - ec[1] + ed[1], k - ec[2] + ed[2]) +
                         cellv(P, mu, i + ed[0], j + ed[1], k + ed[2]));
    double mem = 0.25 * (cellv(P, mu, i - ec[0] - ed[0], j - ec[1] - ed[1], k - ec[2] - ed[2]) +
                         cellv(P, mu, i - ed[0], j - ed[1], k - ed[2]) +
                         cellv(P, mu, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, mu, i, j, k));
    double dudp = (FV(1) - FV(0)) / h;
    double dudm = (FV(0) - FV(-1)) / h;
    double dvp = (facev(P, d, F[d], i + ed[0], j + ed[1], k + ed[2]) -
                  facev(P, d, F[d], i + ed[0] - ec[0], j + ed[1] - ec[1], k + ed[2] - ec[2])) / h;
    double dvm = (facev(P, d, F[d], i, j, k) - facev(P, d, F[d], i - ec[0], j - ec[1], k - ec[2])) / h;
    tp = mep * (dudp + dvp);
    tm = mem * (dudm + dvm);
    if (diag) *diag = (mep + mem) / (h * h);
  }
#undef FV
  return (tp - tm) / h;
}

/* Status of the last predictor call: bit 0 set when a transported face
 * density came out non-positive, bit 1 when the Crank-Nicolson system did
 * not converge. */
static int g_flags = 0;
int orc_last_flags(void) { return g_flags; }

/* Crank-Nicolson viscous term (Sec. "Time stepping scheme"): each face that
 * is not a wall or the inlet solves
 *   D_f u*_f - 1/2 L(u*)_f = rhs_f,
 * rhs_f holding the explicit terms and 1/2 L(u^n)_f, D_f the implicit
 * diagonal (D_f = 0 marks a fixed face).  The system is solved to
 * convergence by Gauss-Seidel sweeps in place over u, then v, then w, each
 * face from the latest values of every component:
 *   u_f <- (rhs_f + 1/2 (L(u)_f + a_f u_f)) / (D_f + 1/2 a_f),
 * a_f the magnitude of the interior diagonal of L; any fixed point of this
 * update solves the system above.  Sweeps stop once a sweep changes no face
 * by more than 1e-15 of the largest |u*|; 500 sweeps without that set bit 1
 * of the status. */
static void cn_solve(const orc_params* P, const double* mu, double* const rhs[3], double* const D[3],
                     double* const out[3]) {
  for (int s = 0; s < 500; ++s) {
    const double* F[3] = {out[0], out[1], out[2]};
    double dmax = 0.0, umax = 0.0;
    for (int c = 0; c < 3; ++c) {
      int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
      for (int k = 0; k < mz; ++k)
        for (int j = 0; j < my; ++j)
          for (int i = 0; i < mx; ++i) {
            size_t f = i + (size_t)mx * (j + (size_t)my * k);
            if (D[c][f] == 0.0) continue;
            double L = 0.0, a = 0.0;
            for (int d = 0; d < 3; ++d) {
              double ad;
              L += visc_dir(P, mu, F, c, d, i, j, k, &ad);
              a += ad;
            }
            double nv = (rhs[c][f] + 0.5 * (L + a * out[c][f])) / (D[c][f] + 0.5 * a);
            dmax = fmax(dmax, fabs(nv - out[c][f]));
            umax = fmax(umax, fabs(nv));
            out[c][f] = nv;
          }
    }
    if (dmax <= 1e-15 * umax) return;
  }
  g_flags |= 2;
}

/* With rho_n (cell density at t^n) the predictor takes the conservative form
 * of eqn_c_discrete_momentum with consistent mass/momentum transport (Sec.
 * "Multiphase incompressible Navier-Stokes solution"): the face density is
 * carried over the step by the same mass fluxes that carry momentum,
 *   rb_f = rho^n_f - dt/h sum (m_+ - m_-),  m = a rho_upwind(rho^n_f),
 *   (rb_f u*_f - rho^n_f u^n_f)/dt + 1/h sum (m_+ v_+ - m_- v_-) = forces,
 * with the Koren-limited upwind face density and velocity of the advective
 * form; rb (face arrays, may be NULL) receives rb_f.  Without rho_n it is
 * the advective form above. */
static void momentum_impl(const orc_params* P, const double* u, const double* v, const double* w,
                          const double* sigma, double t_np1, double dt, const double* rho_n, double* us,
                          double* vs, double* ws, double* const rb[3]);

void orc_momentum(const orc_params* P, const double* u, const double* v, const double* w,
                  const double* sigma, double t_np1, double dt, double* us, double* vs, double* ws) {
  double* const none[3] = {NULL, NULL, NULL};
  momentum_impl(P, u, v, w, sigma, t_np1, dt, NULL, us, vs, ws, none);
}

void orc_momentum_cons(const orc_params* P, const double* u, const double* v, const double* w,
                       const double* sigma, double t_np1, double dt, const double* rho_n, double* us, double* vs,
                       double* ws, double* rbx, double* rby, double* rbz) {
  double* const rb[3] = {rbx, rby, rbz};
  momentum_impl(P, u, v, w, sigma, t_np1, dt, rho_n, us, vs, ws, rb);
}

static void momentum_impl(const orc_params* P, const double* u, const double* v, const double* w,
                          const double* sigma, double t_np1, double dt, const double* rho_n, double* us,
                          double* vs, double* ws, double* const rb[3]) {
  const size_t n = ncell(P);
  const double h = P->h;
  double* rho = (double*)malloc(n * sizeof(double));
  double* rfl = (double*)malloc(n * sizeof(double));
  double* mu = (double*)malloc(n * sizeof(double));
  double* chi = (double*)malloc(n * sizeof(double));
  orc_properties(P, sigma, t_np1, rho, rfl, mu, chi);
  const double* F[3] = {u, v, w};
  double* out[3] = {us, vs, ws};
  /* Crank-Nicolson: half the viscous term at t^n goes to the right-hand side */
  const int cn = P->crank_nicolson != 0;
  int flags = 0;
  const double wv = cn ? 0.5 : 1.0;
  double* rhsA[3] = {NULL, NULL, NULL};
  double* DA[3] = {NULL, NULL, NULL};
  if (cn)
    for (int c = 0; c < 3; ++c) {
      rhsA[c] = (double*)calloc(face_count(P, c), sizeof(double));
      DA[c] = (double*)calloc(face_count(P, c), sizeof(double));
    }

  for (int c = 0; c < 3; ++c) {
    int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
    int ec[3] = {c == 0, c == 1, c == 2};
    #ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : flags)
#endif
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          size_t f = i + (size_t)mx * (j + (size_t)my * k);
          if (c == 0 && i == 0 && P->gen_len > 0.0) {
            /* the inlet of the wave tank: the target wave's velocity */
            out[c][f] = wave_vel(P, 0, 0.0, (k + 0.5) * h, t_np1);
            if (rho_n && rb[c]) rb[c][f] = 0.0;
            continue;
          }
          if (is_wall_face(P, c, i, j, k)) {
            out[c][f] = 0.0;
            if (rho_n && rb[c]) rb[c][f] = 0.0;
            continue;
          }
          double uf = F[c][f];
          double adv = 0.0, visc = 0.0, conv = 0.0, mflux = 0.0;
          for (int d = 0; d < 3; ++d) {
            int ed[3] = {d == 0, d == 1, d == 2};
#define FC(o) facev(P, c, F[c], i + (o) * ed[0], j + (o) * ed[1], k + (o) * ed[2])
/* face density at t^n of the face o steps along d: mean of its two cells */
#define RF(o)                                                                                        \
  (0.5 * (cellv(P, rho_n, i - ec[0] + (o) * ed[0], j - ec[1] + (o) * ed[1], k - ec[2] + (o) * ed[2]) + \
          cellv(P, rho_n, i + (o) * ed[0], j + (o) * ed[1], k + (o) * ed[2])))
            /* advecting velocities on the + and - sides of the control volume */
            double ap, am;
            if (d == c) {
              ap = 0.5 * (FC(0) + FC(1));
              am = 0.5 * (FC(-1) + FC(0));
            } else {
              ap = 0.5 * (facev(P, d, F[d], i + ed[0] - ec[0], j + ed[1] - ec[1], k + ed[2] - ec[2]) +
                          facev(P, d, F[d], i + ed[0], j + ed[1], k + ed[2]));
              am = 0.5 * (facev(P, d, F[d], i - ec[0], j - ec[1], k - ec[2]) +
                          facev(P, d, F[d], i, j, k));
            }
            double vp = ap >= 0.0 ? koren(FC(-1), FC(0), FC(1)) : koren(FC(2), FC(1), FC(0));
            double vm = am >= 0.0 ? koren(FC(-2), FC(-1), FC(0)) : koren(FC(1), FC(0), FC(-1));
            adv += ap * (vp - uf) - am * (vm - uf);
            if (rho_n) {
              /* mass fluxes with the same upwinding, and the momentum they carry */
              double rp = ap >= 0.0 ? koren(RF(-1), RF(0), RF(1)) : koren(RF(2), RF(1), RF(0));
              double rm = am >= 0.0 ? koren(RF(-2), RF(-1), RF(0)) : koren(RF(1), RF(0), RF(-1));
              double mp = ap * rp, mm = am * rm;
              conv += mp * vp - mm * vm;
              mflux += mp - mm;
            }

            visc += visc_dir(P, mu, F, c, d, i, j, k, NULL);
#undef FC
          }
          adv /= h;
          /* face properties: mean of the two cells sharing the face */
          double rhof = 0.5 * (cellv(P, rho, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, rho, i, j, k));
          double rflf = 0.5 * (cellv(P, rfl, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, rfl, i, j, k));
          double chif = 0.5 * (cellv(P, chi, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, chi, i, j, k));
          double grav = (c == 2) ? -P->g * rflf : 0.0;
          double ub = 0.0;
          if (c == 2 && P->n_bodies > 0) {
            body_psi(P, (i + 0.5) * h, (j + 0.5) * h, k * h, t_np1, &ub);
          }
          double pen = chif * P->inv_kappa_p;
          /* vorticity damping force -g(z~) u, taken implicitly like the penalty */
          double damp = vort_damp(P, (c == 2) ? k * h : (k + 0.5) * h, dt);
          if (rho_n) {
            double r0 = 0.5 * (cellv(P, rho_n, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, rho_n, i, j, k));
            double rbf = r0 - dt * mflux / h;
            /* a transported density at or below zero leaves the projection
             * operator indefinite: the step is outside the scheme's bound */
            if (!(rbf > 0.0)) flags |= 1;
            double num = r0 * uf / dt - conv / h + wv * visc + grav + pen * ub;
            double den = rbf / dt + pen + damp;
            out[c][f] = cn ? (num + 0.5 * visc) / den : num / den;
            if (rb[c]) rb[c][f] = rbf;
            if (cn) rhsA[c][f] = num, DA[c][f] = den;
            continue;
          }
          double num = rhof * (uf / dt - adv) + wv * visc + grav + pen * ub;
          double den = rhof / dt + pen + damp;
          out[c][f] = cn ? (num + 0.5 * visc) / den : num / den;
          if (cn) rhsA[c][f] = num, DA[c][f] = den;
        }
  }
  g_flags = flags;
  if (cn) {
    cn_solve(P, mu, rhsA, DA, out);
    for (int c = 0; c < 3; ++c) {
      free(rhsA[c]);
      free(DA[c]);
    }
  }
  free(rho);
  free(rfl);
  free(mu);
  free(chi);
}
#undef RF

/* --------------------------------------------------------------------------
 * Projection coefficient on faces: beta_f = 1/(rho_f + w dt chi_f/kappa_p),
 * the inverse of the implicit momentum diagonal times dt (w = 1), or the
 * plain 1/rho_f (w = 0).  Wall faces get beta = 0.
 * ------------------------------------------------------------------------ */
void orc_face_beta(const orc_params* P, const double* sigma, double t_np1, double dt, double* bx,
                   double* by, double* bz) {
  const size_t n = ncell(P);
  double* rho = (double*)malloc(n * sizeof(double));
  double* chi = (double*)malloc(n * sizeof(double));
  orc_properties(P, sigma, t_np1, rho, NULL, NULL, chi);
  double* out[3] = {bx, by, bz};
  for (int c = 0; c < 3; ++c) {
    int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
    int ec[3] = {c == 0, c == 1, c == 2};
    ORC_PAR
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          size_t f = i + (size_t)mx * (j + (size_t)my * k);
          if (is_wall_face(P, c, i, j, k)) {
            out[c][f] = 0.0;
            continue;
          }
          double rhof = 0.5 * (cellv(P, rho, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, rho, i, j, k));
          double chif = 0.5 * (cellv(P, chi, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, chi, i, j, k));
          out[c][f] = 1.0 / (rhof + P->proj_penalty_weight * dt * chif * P->inv_kappa_p);
        }
  }
  free(rho);
  free(chi);
}

/* beta_f = 1/(rb_f + w dt chi_f/kappa_p) with the transported face density
 * rb_f of the consistent form (walls 0) */
void orc_face_beta_rho(const orc_params* P, const double* rbx, const double* rby, const double* rbz,
                       const double* sigma, double t_np1, double dt, double* bx, double* by, double* bz) {
  const size_t n = ncell(P);
  double* rho = (double*)malloc(n * sizeof(double));
  double* chi = (double*)malloc(n * sizeof(double));
  orc_properties(P, sigma, t_np1, rho, NULL, NULL, chi);
  const double* rb[3] = {rbx, rby, rbz};
  double* out[3] = {bx, by, bz};
  for (int c = 0; c < 3; ++c) {
    int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
    int ec[3] = {c == 0, c == 1, c == 2};
    ORC_PAR
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          size_t f = i + (size_t)mx * (j + (size_t)my * k);
          if (is_wall_face(P, c, i, j, k)) {
            out[c][f] = 0.0;
            continue;
          }
          double chif = 0.5 * (cellv(P, chi, i - ec[0], j - ec[1], k - ec[2]) + cellv(P, chi, i, j, k));
          out[c][f] = 1.0 / (rb[c][f] + P->proj_penalty_weight * dt * chif * P->inv_kappa_p);
        }
  }
  free(rho);
  free(chi);
}

/* b = -div_h(u*) / dt  (eqn_c_discrete_continuity applied to u^{n+1}) */
void orc_rhs(const orc_params* P, const double* us, const double* vs, const double* ws, double dt,
             double* b) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  ORC_PAR
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double div = (facev(P, 0, us, i + 1, j, k) - facev(P, 0, us, i, j, k)) +
                     (facev(P, 1, vs, i, j + 1, k) - facev(P, 1, vs, i, j, k)) +
                     (facev(P, 2, ws, i, j, k + 1) - facev(P, 2, ws, i, j, k));
        b[i + (size_t)nx * (j + (size_t)ny * k)] = -div / (P->h * dt);
      }
}

/* --------------------------------------------------------------------------
 * Multigrid hierarchy and V-cycle, in FP64 and in FP32 from one template.
 * ------------------------------------------------------------------------ */
/* active directions coarsen by 2 while every active size is even */
int orc_num_levels(int nx, int ny, int nz) {
  int n[3] = {nx, ny, nz};
  int act[3] = {nx > 1, ny > 1, nz > 1};
  int L = 1;
  for (;;) {
    int ok = 1;
    for (int d = 0; d < 3; ++d)
      if (act[d] && (n[d] < 2 || n[d] % 2 != 0)) ok = 0;
    if (!ok || L >= 30) break;
    for (int d = 0; d < 3; ++d)
      if (act[d]) n[d] /= 2;
    ++L;
  }
  return L;
}

#define MG_REAL double
#define MG_SFX _d
#include "ns_oracle_mg.inc"
#undef MG_REAL
#undef MG_SFX
#define MG_REAL float
#define MG_SFX _f
#include "ns_oracle_mg.inc"
#undef MG_REAL
#undef MG_SFX

/* y = A x on the finest level: (A x)_c = (1/h^2) [ sum over non-wall faces
 * beta_f (x_c - x_nb) + 2 beta_top x_c on the top row ] */
void orc_apply_A(int nx, int ny, int nz, double h, const double* bx, const double* by,
                 const double* bz, const double* x, double* y) {
  mglev_d L;
  L.n[0] = nx;
  L.n[1] = ny;
  L.n[2] = nz;
  L.h = h;
  L.beta[0] = (double*)bx;
  L.beta[1] = (double*)by;
  L.beta[2] = (double*)bz;
  apply_A_d(&L, x, y);
}

typedef struct {
  int L;
  mglev_d dl[30];
  mglev_f fl[30];
  int prec;
} orc_mg;

static void mg_build(const orc_params* P, const double* bx, const double* by, const double* bz,
                     orc_mg* M) {
  M->L = orc_num_levels(P->nx, P->ny, P->nz);
  M->prec = P->prec;
  build_levels_d(P, bx, by, bz, M->L, M->dl);
  if (M->prec) build_levels_f(P, bx, by, bz, M->L, M->fl);
}

static void mg_free(orc_mg* M) {
  free_levels_d(M->L, M->dl);
  if (M->prec) free_levels_f(M->L, M->fl);
}

/* z = M r: one V-cycle from a zero guess.  In mixed mode the V-cycle runs in
 * FP32 on (float) r and its result is widened back to FP64. */
static void mg_apply(const orc_params* P, orc_mg* M, const double* r, double* z) {
  size_t n = (size_t)P->nx * P->ny * P->nz;
  if (!M->prec) {
    memcpy(M->dl[0].b, r, n * sizeof(double));
    vcycle_d(P, M->dl, M->L, 0);
    memcpy(z, M->dl[0].e, n * sizeof(double));
  } else {
    for (size_t c = 0; c < n; ++c) M->fl[0].b[c] = (float)r[c];
    vcycle_f(P, M->fl, M->L, 0);
    for (size_t c = 0; c < n; ++c) z[c] = (double)M->fl[0].e[c];
  }
}

void orc_vcycle(const orc_params* P, const double* bx, const double* by, const double* bz,
                const double* r, double* z) {
  orc_mg M;
  mg_build(P, bx, by, bz, &M);
  mg_apply(P, &M, r, z);
  mg_free(&M);
}

static double dot(const double* a, const double* b, size_t n) {
  double s = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : s)
#endif
  for (size_t c = 0; c < n; ++c) s += a[c] * b[c];
  return s;
}

/* --------------------------------------------------------------------------
 * Flexible (Polak-Ribiere) preconditioned CG for A x = b, x holding the
 * initial guess on entry.  Stops when ||b - A x||_2 <= rtol ||b||_2 on the
 * recursive residual, confirmed on the true residual (a failed confirmation
 * restarts from the true residual).  Returns 0 when converged, 1 otherwise.
 * ------------------------------------------------------------------------ */
int orc_pcg(const orc_params* P, const double* bx, const double* by, const double* bz,
            const double* b, double* x, orc_stats* st) {
  const size_t n = ncell(P);
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h;
  double* r = (double*)calloc(n, sizeof(double));
  double* z = (double*)calloc(n, sizeof(double));
  double* zn = (double*)calloc(n, sizeof(double));
  double* d = (double*)calloc(n, sizeof(double));
  double* q = (double*)calloc(n, sizeof(double));
  orc_mg M;
  mg_build(P, bx, by, bz, &M);
  int converged = 0, it = 0;

  double bnorm = sqrt(dot(b, b, n));
  if (bnorm == 0.0) {
    memset(x, 0, n * sizeof(double));
    st->iters = 0;
    st->rel_resid0 = st->rel_resid = st->true_rel_resid = 0.0;
    converged = 1;
    goto done;
  }
  orc_apply_A(nx, ny, nz, h, bx, by, bz, x, q);
  for (size_t c = 0; c < n; ++c) r[c] = b[c] - q[c];
  double rnorm = sqrt(dot(r, r, n));
  st->rel_resid0 = rnorm / bnorm;
  st->rel_resid = rnorm / bnorm;
  if (rnorm <= P->rtol * bnorm) {
    converged = 1;
  } else {
    mg_apply(P, &M, r, z);
    memcpy(d, z, n * sizeof(double));
    double rho = dot(r, z, n);
    while (it < P->max_iters) {
      orc_apply_A(nx, ny, nz, h, bx, by, bz, d, q);
      double alpha = rho / dot(d, q, n);
      ORC_PAR
      for (size_t c = 0; c < n; ++c) {
        x[c] += alpha * d[c];
        r[c] -= alpha * q[c];
      }
      ++it;
      rnorm = sqrt(dot(r, r, n));
      st->rel_resid = rnorm / bnorm;
      if (rnorm <= P->rtol * bnorm) {
        /* confirm on the true residual; restart from it if it fails */
        orc_apply_A(nx, ny, nz, h, bx, by, bz, x, q);
        for (size_t c = 0; c < n; ++c) r[c] = b[c] - q[c];
        rnorm = sqrt(dot(r, r, n));
        st->rel_resid = rnorm / bnorm;
        if (rnorm <= P->rtol * bnorm) {
          converged = 1;
          break;
        }
        mg_apply(P, &M, r, z);
        memcpy(d, z, n * sizeof(double));
        rho = dot(r, z, n);
        continue;
      }
      mg_apply(P, &M, r, zn);
      double rzn = dot(r, zn, n);
      double rzo = dot(r, z, n);
      double beta = (rzn - rzo) / rho;
      ORC_PAR
      for (size_t c = 0; c < n; ++c) d[c] = zn[c] + beta * d[c];
      rho = rzn;
      double* t = z;
      z = zn;
      zn = t;
    }
  }
  st->iters = it;
  orc_apply_A(nx, ny, nz, h, bx, by, bz, x, q);
  for (size_t c = 0; c < n; ++c) q[c] = b[c] - q[c];
  st->true_rel_resid = sqrt(dot(q, q, n)) / bnorm;
done:
  mg_free(&M);
  free(r);
  free(z);
  free(zn);
  free(d);
  free(q);
  return converged ? 0 : 1;
}

/* --------------------------------------------------------------------------
 * Velocity correction u^{n+1} = u* - dt beta_f grad_h p on every non-wall
 * face; on the open top the boundary value p = 0 sits half a cell above the
 * last cell centre.
 * ------------------------------------------------------------------------ */
void orc_correct(const orc_params* P, const double* us, const double* vs, const double* ws,
                 const double* p, const double* bx, const double* by, const double* bz, double dt,
                 double* u, double* v, double* w) {
  const double* S[3] = {us, vs, ws};
  const double* B[3] = {bx, by, bz};
  double* out[3] = {u, v, w};
  const double h = P->h;
  for (int c = 0; c < 3; ++c) {
    int mx = P->nx + (c == 0), my = P->ny + (c == 1), mz = P->nz + (c == 2);
    int ec[3] = {c == 0, c == 1, c == 2};
    ORC_PAR
    for (int k = 0; k < mz; ++k)
      for (int j = 0; j < my; ++j)
        for (int i = 0; i < mx; ++i) {
          size_t f = i + (size_t)mx * (j + (size_t)my * k);
          if (c == 0 && i == 0 && P->gen_len > 0.0) {
            out[c][f] = S[c][f];   /* the inlet keeps its prescribed velocity */
            continue;
          }
          if (is_wall_face(P, c, i, j, k)) {
            out[c][f] = 0.0;
            continue;
          }
          double grad;
          if (c == 2 && k == P->nz) {
            grad = (0.0 - cellv(P, p, i, j, k - 1)) / (0.5 * h);
          } else {
            grad = (cellv(P, p, i, j, k) - cellv(P, p, i - ec[0], j - ec[1], k - ec[2])) / h;
          }
          out[c][f] = S[c][f] - dt * B[c][f] * grad;
        }
  }
}

/* --------------------------------------------------------------------------
 * One time step (Sec. "Solution methodology" order, one fixed-point cycle):
 * level set to n+1, properties at n+1, momentum predictor, projection.
 * p holds p^{n-1/2} on entry (used as the initial guess when x0_prev) and
 * p^{n+1/2} on exit.  Returns the CG status.
 * ------------------------------------------------------------------------ */
int orc_step(const orc_params* P, double* sigma, double* u, double* v, double* w, double* p,
             double dt, double t_n, int x0_prev, orc_stats* st) {
  return orc_step_from(P, sigma, u, v, w, p, dt, t_n, x0_prev, NULL, st);
}

/* As orc_step; with consistent transport rho_n_in (may be NULL: the
 * properties of sigma and the bodies as P holds them, at t_n) is the density
 * the step starts from. */
int orc_step_from(const orc_params* P, double* sigma, double* u, double* v, double* w, double* p,
                  double dt, double t_n, int x0_prev, const double* rho_n_in, orc_stats* st) {
  const size_t n = ncell(P);
  double* rho_n = NULL;
  if (P->consistent) {  /* the density the step starts from */
    rho_n = (double*)malloc(n * sizeof(double));
    if (rho_n_in)
      memcpy(rho_n, rho_n_in, n * sizeof(double));
    else
      orc_properties(P, sigma, t_n, rho_n, NULL, NULL, NULL);
  }
  double* s1 = (double*)malloc(n * sizeof(double));
  orc_levelset_advect(P, sigma, u, v, w, dt, s1);
  orc_reinit(P, s1, sigma);
  free(s1);
  const double t1 = t_n + dt;
  size_t nu = face_count(P, 0), nv = face_count(P, 1), nw = face_count(P, 2);
  double* us = (double*)malloc(nu * sizeof(double));
  double* vs = (double*)malloc(nv * sizeof(double));
  double* ws = (double*)malloc(nw * sizeof(double));
  double* bx = (double*)malloc(nu * sizeof(double));
  double* by = (double*)malloc(nv * sizeof(double));
  double* bz = (double*)malloc(nw * sizeof(double));
  double* b = (double*)malloc(n * sizeof(double));
  if (P->consistent) {
    double* rbx = (double*)malloc(nu * sizeof(double));
    double* rby = (double*)malloc(nv * sizeof(double));
    double* rbz = (double*)malloc(nw * sizeof(double));
    orc_momentum_cons(P, u, v, w, sigma, t1, dt, rho_n, us, vs, ws, rbx, rby, rbz);
    orc_face_beta_rho(P, rbx, rby, rbz, sigma, t1, dt, bx, by, bz);
    free(rbx);
    free(rby);
    free(rbz);
    free(rho_n);
  } else {
    orc_momentum(P, u, v, w, sigma, t1, dt, us, vs, ws);
    orc_face_beta(P, sigma, t1, dt, bx, by, bz);
  }
  int rc = (g_flags & 1) ? 2 : (g_flags & 2) ? 3 : 0;
  if (rc == 0) {
    orc_rhs(P, us, vs, ws, dt, b);
    if (!x0_prev) memset(p, 0, n * sizeof(double));
    rc = orc_pcg(P, bx, by, bz, b, p, st);
    orc_correct(P, us, vs, ws, p, bx, by, bz, dt, u, v, w);
    if (P->gen_len > 0.0 || P->damp_len > 0.0) orc_relax(P, t1, sigma, u, v, w);
  }
  free(us);
  free(vs);
  free(ws);
  free(bx);
  free(by);
  free(bz);
  free(b);
  return rc;
}

/* Time step of the CFL rule (Sec. "Time stepping scheme"; the paper keeps
 * the Courant number at or below 0.5): dt = cfl h / m with m the largest
 * cell value of |u_c| + |v_c| + |w_c|, each cell velocity the mean of its two
 * faces, capped at dt_max (dt_max for a fluid at rest). */
double orc_cfl_dt(const orc_params* P, const double* u, const double* v, const double* w, double cfl,
                  double dt_max) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  double m = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(max : m)
#endif
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double uc = 0.5 * fabs(facev(P, 0, u, i, j, k) + facev(P, 0, u, i + 1, j, k));
        double vc = 0.5 * fabs(facev(P, 1, v, i, j, k) + facev(P, 1, v, i, j + 1, k));
        double wc = 0.5 * fabs(facev(P, 2, w, i, j, k) + facev(P, 2, w, i, j, k + 1));
        double s = uc + vc + wc;
        if (s > m) m = s;   /* a maximum: the same in any order */
      }
  if (!(m > 0.0)) return dt_max;
  double dt = cfl * P->h / m;
  return dt < dt_max ? dt : dt_max;
}

/* max |div_h u|, water volume sum (1 - H(sigma)) h^d, kinetic energy
 * 1/2 sum rho_flow |u_c|^2 h^d (cell-averaged velocity), max |u_face| */
void orc_diagnostics(const orc_params* P, const double* sigma, const double* u, const double* v,
                     const double* w, double* out4) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h, eps = P->n_cells * h;
  const double vol = (ny == 1) ? h * h : h * h * h;
  double mdiv = 0.0, wv = 0.0, ke = 0.0, mu = 0.0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = i + (size_t)nx * (j + (size_t)ny * k);
        double up = facev(P, 0, u, i + 1, j, k), um = facev(P, 0, u, i, j, k);
        double vp = facev(P, 1, v, i, j + 1, k), vm = facev(P, 1, v, i, j, k);
        double wp = facev(P, 2, w, i, j, k + 1), wm = facev(P, 2, w, i, j, k);
        double div = ((up - um) + (vp - vm) + (wp - wm)) / h;
        if (fabs(div) > mdiv) mdiv = fabs(div);
        double hf = heaviside(sigma[c], eps);
        wv += (1.0 - hf) * vol;
        double rf = P->rho_w + (P->rho_a - P->rho_w) * hf;
        double uc = 0.5 * (up + um), vc = 0.5 * (vp + vm), wc = 0.5 * (wp + wm);
        ke += 0.5 * rf * (uc * uc + vc * vc + wc * wc) * vol;
      }
  const double* F[3] = {u, v, w};
  for (int c = 0; c < 3; ++c) {
    size_t m = face_count(P, c);
    for (size_t f = 0; f < m; ++f)
      if (fabs(F[c][f]) > mu) mu = fabs(F[c][f]);
  }
  out4[0] = mdiv;
  out4[1] = wv;
  out4[2] = ke;
  out4[3] = mu;
}

/* --------------------------------------------------------------------------
 * Hydrodynamic force on body m, eqn_int_fh (Sec. "Fluid-structure coupling"):
 *   F = sum over f of ( -p_f n_f + mu_f (grad u + grad u^T)_f . n_f ) dA_f
 * over the faces of the stair-step body surface (Sec. "NLFK calculation",
 * eqn_NLFK_p): a face belongs to it when the body's level set psi has
 * opposite signs in the two cells the face separates.
 *   n_f   unit normal out of the body: from the cell with psi < 0 to the other
 *   p_f   the two cell pressures interpolated linearly to psi = 0, i.e.
 *         weighted by the other cell's |psi|
 *   mu_f  mean of the two cells' viscosity
 *   grad  central differences at the face centre (MAC grid): a velocity
 *         component's derivative across the face from the cell-centred means
 *         of the two cells, a derivative of the face's own normal velocity
 *         along the face from its two neighbours; indices clamp to the grid
 *   dA_f  h^2 in 3-D, h in 2-D (per unit depth)
 * In 2-D (ny == 1) the y-direction carries no faces and no derivatives.
 * ------------------------------------------------------------------------ */

/* cell-centred mean of velocity component c at cell (i,j,k) */
static double vel_cell(const orc_params* P, int c, const double* vel, int i, int j, int k) {
  int di = (c == 0), dj = (c == 1), dk = (c == 2);
  return 0.5 * (facev(P, c, vel, i, j, k) + facev(P, c, vel, i + di, j + dj, k + dk));
}

void orc_hydro_force(const orc_params* P, int m, const double* p, const double* u, const double* v,
                     const double* w, const double* mu, double t, double* F) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const double h = P->h;
  const double dA = (ny == 1) ? h : h * h;
  const double* vel[3] = {u, v, w};
  const orc_body* B = &P->body[m];
  F[0] = F[1] = F[2] = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (d == 1 && ny == 1) continue;
    const int di = (d == 0), dj = (d == 1), dk = (d == 2);
    /* interior faces normal to d: between cell a = (i,j,k) - e_d and b = (i,j,k) */
    for (int k = dk; k < nz; ++k)
      for (int j = dj; j < ny; ++j)
        for (int i = di; i < nx; ++i) {
          const int ia = i - di, ja = j - dj, ka = k - dk;
          double zd;
          const double psa = body_psi_one(B, (ia + 0.5) * h, (ja + 0.5) * h, (ka + 0.5) * h, t, &zd);
          const double psb = body_psi_one(B, (i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h, t, &zd);
          if ((psa < 0.0) == (psb < 0.0)) continue;
          const double nd = (psa < 0.0) ? 1.0 : -1.0;   /* out of the body along d */
          const double pa = cellv(P, p, ia, ja, ka), pb = cellv(P, p, i, j, k);
          const double pf = (fabs(psb) * pa + fabs(psa) * pb) / (fabs(psa) + fabs(psb));
          const double muf = 0.5 * (cellv(P, mu, ia, ja, ka) + cellv(P, mu, i, j, k));
          F[d] += -pf * nd * dA;
          for (int c = 0; c < 3; ++c) {
            if (c == 1 && ny == 1) continue;
            double G;
            if (c == d) {
              /* 2 d(u_d)/dx_d at the face: neighbours of the face along d */
              G = 2.0 * (facev(P, d, vel[d], i + di, j + dj, k + dk) - facev(P, d, vel[d], i - di, j - dj, k - dk)) /
                  (2.0 * h);
            } else {
              const int ci = (c == 0), cj = (c == 1), ck = (c == 2);
              /* d(u_c)/dx_d across the face, from the cell-centred means */
              const double dcd = (vel_cell(P, c, vel[c], i, j, k) - vel_cell(P, c, vel[c], ia, ja, ka)) / h;
              /* d(u_d)/dx_c along the face, from the face's neighbours along c */
              const double ddc = (facev(P, d, vel[d], i + ci, j + cj, k + ck) -
                                  facev(P, d, vel[d], i - ci, j - cj, k - ck)) / (2.0 * h);
              G = dcd + ddc;
            }
            F[c] += muf * G * nd * dA;
          }
        }
  }
}

/* Heave of a free body, eqn_newton_u with the linear-damper PTO force
 * F_PTO = -c zdot^{n+1} taken at the new time level:
 *   m (zdot^{n+1} - zdot^n) / dt = Fz - m g - c zdot^{n+1},
 * then zeta^{n+1} = zeta^n + dt zdot^{n+1}. */
void orc_heave_update(double mass, double pto_damping, double g, double dt, double fz, double* zeta,
                      double* zdot) {
  const double zn = (*zdot + dt * (fz - mass * g) / mass) / (1.0 + dt * pto_damping / mass);
  *zdot = zn;
  *zeta += dt * zn;
}
