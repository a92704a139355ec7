// Grid kernels of the time step on gfx950: level-set advection and
// reinitialisation, material properties, the momentum predictor, the
// projection right-hand side, the velocity correction and diagnostics.
//
// Threads are laid out 64 along x (one wavefront per x-row segment, so every
// load of a row is one contiguous 512-byte FP64 segment) by 4 along y (or
// along z for a 2-D tank).  Out-of-grid neighbours are the nearest interior
// value: zero normal gradient for scalars, free slip for tangential
// velocity, zero for wall-normal velocity (whose faces hold 0).
#include <algorithm>
#include <cmath>

#include "ns_internal.h"

namespace nsk {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Geo {
  dim3 grid, block;
};

inline Geo geo3(int mx, int my, int mz) {
  dim3 b = (my >= 4) ? dim3(64, 4, 1) : dim3(64, 1, 4);
  return {dim3((mx + 63) / 64, (my + b.y - 1) / b.y, (mz + b.z - 1) / b.z), b};
}

constexpr double kE = 2.718281828459045235360287471352662;   // e

__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

// cell value with clamped indices
__device__ __forceinline__ double cv(const double* __restrict__ a, const Dims& n, int i, int j, int k) {
  i = clampi(i, 0, n.nx - 1);
  j = clampi(j, 0, n.ny - 1);
  k = clampi(k, 0, n.nz - 1);
  // 32-bit index arithmetic: every array has fewer than 2^31 entries (the
  // context refuses grids with more than 2e9 faces), and the predictor's
  // ~35 clamped loads per face made 64-bit products a large share of its
  // instructions
  return a[i + n.nx * (j + n.ny * k)];
}

// face value of component C with clamped indices
template <int C>
__device__ __forceinline__ double fv(const double* __restrict__ a, const Dims& n, int i, int j, int k) {
  const int mx = n.nx + (C == 0), my = n.ny + (C == 1), mz = n.nz + (C == 2);
  i = clampi(i, 0, mx - 1);
  j = clampi(j, 0, my - 1);
  k = clampi(k, 0, mz - 1);
  return a[i + mx * (j + my * k)];
}

// Koren-limited upwind face value; up2 is the cell behind the upwind cell up,
// dn the downwind cell.  Third order (kappa = 1/3) where smooth, first order
// at extrema, total-variation diminishing.
__device__ __forceinline__ double koren(double up2, double up, double dn) {
  const double a = up - up2;
  const double b = dn - up;
  if (a * b <= 0.0) return up;
  const double fa = fabs(a), fb = fabs(b);
  const double lim = fmin(fmin(2.0 * fa, (2.0 * fb + fa) * (1.0 / 3.0)), 2.0 * fb);
  return up + copysign(0.5 * lim, b);
}

// The Koren value at a face between m (its negative side) and p, with mm
// behind m and pp beyond p, upwind of the advecting velocity a.  The upwind
// side's three values are selected first, so one limiter is evaluated
// instead of both sides' and a select of the two.
__device__ __forceinline__ double koren_face(double a, double mm, double m, double p, double pp) {
  const bool pos = a >= 0.0;
  return koren(pos ? mm : pp, pos ? m : p, pos ? p : m);
}

__device__ __forceinline__ double heaviside(double phi, double eps) {
  if (phi < -eps) return 0.0;
  if (phi > eps) return 1.0;
  return 0.5 * (1.0 + phi / eps + sin(kPi * phi / eps) * (1.0 / kPi));
}

// level set of one body at (x,y,z,t) and its heave velocity: prescribed
// heave A sin(w t + phi), or the free body's own state
__device__ double body_psi_one(const BodyK& B, double x, double y, double z, double t, double* zdot) {
  double zeta, zd;
  if (B.fh) {
    zeta = B.zeta;
    zd = B.zdot;
  } else {
    const double arg = B.om * t + B.ph;
    zeta = B.amp * sin(arg);
    zd = B.amp * B.om * cos(arg);
  }
  *zdot = zd;
  if (B.kind == 0) return fmax(fabs(x - B.c0) - B.h0, fabs(z - (B.c2 + zeta)) - B.h2);
  const double dx = x - B.c0, dy = y - B.c1;
  const double r = sqrt(dx * dx + dy * dy);
  return fmax(r - B.h0, fmax((B.h1 + zeta) - z, z - (B.h2 + zeta)));
}

// union of the analytic bodies at (x,y,z,t); zdot of the nearest one
__device__ double body_psi(const Phys& P, double x, double y, double z, double t, double* zdot) {
  double best = INFINITY;
  double zd_best = 0.0;
  for (int m = 0; m < P.nb; ++m) {
    double zd;
    const double s = body_psi_one(P.body[m], x, y, z, t, &zd);
    if (s < best) {
      best = s;
      zd_best = zd;
    }
  }
  *zdot = zd_best;
  return best;
}

// --------------------------------------------------------------------------
// numerical wave tank (Sec. "Numerical wave tank")
// --------------------------------------------------------------------------
// the generated wave: elevation, and horizontal (c = 0) or vertical (c = 2)
// potential-flow velocity under the surface at (x, z from the bed, t)
__device__ double tank_eta(const Phys& P, double x, double t) {
  double eta = 0.0;
  for (int q = 0; q < P.nwave; ++q) {
    const double* W = P.waves + 4 * q;
    eta += W[0] * cos(W[1] * x - W[2] * t + W[3]);
  }
  return eta;
}

__device__ double tank_vel(const Phys& P, int c, double x, double z, double t) {
  if (c == 1 || z >= P.depth + tank_eta(P, x, t)) return 0.0;
  double s = 0.0;
  for (int q = 0; q < P.nwave; ++q) {
    const double* W = P.waves + 4 * q;
    const double th = W[1] * x - W[2] * t + W[3];
    const double amp = W[0] * W[2] / sinh(W[1] * P.depth);
    s += (c == 0) ? amp * cosh(W[1] * z) * cos(th) : amp * sinh(W[1] * z) * sin(th);
  }
  return s;
}

// relaxation weight (the relaxation-zone method): 1 at the inner edge, 0 at the end
__device__ __forceinline__ double relax_weight(double chi) {
  return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / (kE - 1.0);
}

// vorticity damping coefficient over the top vort_w of the tank
__device__ __forceinline__ double vort_coeff(const Phys& P, double z, double dt) {
  if (P.vort_w <= 0.0) return 0.0;
  const double zt = (z - P.n.nz * P.h) / P.vort_w;
  return zt < -1.0 ? 0.0 : P.rho_a * (cos(kPi * zt) + 1.0) / (4.0 * dt);
}

// --------------------------------------------------------------------------
// level-set advection: sigma* = sigma - dt/h sum_d [a+ (s+ - s) - a- (s- - s)]
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_advect(Phys P, const double* __restrict__ s,
                                                const double* __restrict__ u,
                                                const double* __restrict__ v,
                                                const double* __restrict__ w, double dt,
                                                double* __restrict__ out) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t c = i + (size_t)n.nx * j + sxy * k;
  const double sc = s[c];
  double acc = 0.0;
  // each direction's four neighbours are loaded before the upwind side is
  // chosen, so no load waits on the velocity's sign
  {  // x
    const size_t fm = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
    const double am = u[fm], ap = u[fm + 1];
    auto S = [&](int o) { return s[c + (clampi(i + o, 0, n.nx - 1) - i)]; };
    const double m2 = S(-2), m1 = S(-1), p1 = S(1), p2 = S(2);
    const double sp = koren_face(ap, m1, sc, p1, p2);
    const double sm = koren_face(am, m2, m1, sc, p1);
    acc += ap * (sp - sc) - am * (sm - sc);
  }
  {  // y
    const size_t fm = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
    const double am = v[fm], ap = v[fm + n.nx];
    auto S = [&](int o) { return s[c + (ptrdiff_t)(clampi(j + o, 0, n.ny - 1) - j) * n.nx]; };
    const double m2 = S(-2), m1 = S(-1), p1 = S(1), p2 = S(2);
    const double sp = koren_face(ap, m1, sc, p1, p2);
    const double sm = koren_face(am, m2, m1, sc, p1);
    acc += ap * (sp - sc) - am * (sm - sc);
  }
  {  // z
    const double am = w[c], ap = w[c + sxy];
    auto S = [&](int o) { return s[c + (ptrdiff_t)(clampi(k + o, 0, n.nz - 1) - k) * (ptrdiff_t)sxy]; };
    const double m2 = S(-2), m1 = S(-1), p1 = S(1), p2 = S(2);
    const double sp = koren_face(ap, m1, sc, p1, p2);
    const double sm = koren_face(am, m2, m1, sc, p1);
    acc += ap * (sp - sc) - am * (sm - sc);
  }
  out[c] = sc - (dt / P.h) * acc;
}

// --------------------------------------------------------------------------
// reinitialisation pseudo-step: Godunov upwind |grad sigma|, smoothed sign of
// the pre-reinitialisation field sigma0.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_reinit(Phys P, const double* __restrict__ s0,
                                                const double* __restrict__ cur,
                                                double* __restrict__ nxt, double dtau) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t c = i + (size_t)n.nx * j + sxy * k;
  // every load is issued before the sign test, so none waits on it
  const double a0 = s0[c];
  const double sc = cur[c];
  const double nb[6] = {cur[i > 0 ? c - 1 : c],
                        cur[i < n.nx - 1 ? c + 1 : c],
                        cur[j > 0 ? c - n.nx : c],
                        cur[j < n.ny - 1 ? c + n.nx : c],
                        cur[k > 0 ? c - sxy : c],
                        cur[k < n.nz - 1 ? c + sxy : c]};
  const double h = P.h;
  const double sg = a0 / sqrt(a0 * a0 + h * h);
  // (a cell on the interface, sg = 0, keeps its value: selected at the end
  // rather than returned early, so the neighbour loads are not sunk behind
  // the wait for a0)
  const double ih = 1.0 / h;
  double g2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double a = (sc - nb[2 * d]) * ih;      // backward difference
    const double b = (nb[2 * d + 1] - sc) * ih;  // forward difference
    double t1, t2;
    if (sg > 0.0) {
      t1 = fmax(a, 0.0);
      t2 = fmin(b, 0.0);
    } else {
      t1 = fmin(a, 0.0);
      t2 = fmax(b, 0.0);
    }
    g2 += fmax(t1 * t1, t2 * t2);
  }
  const double upd = sc - dtau * sg * (sqrt(g2) - 1.0);
  nxt[c] = sg == 0.0 ? sc : upd;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) b[q] = a[q];
}

// --------------------------------------------------------------------------
// properties at cell centres: two-stage Heaviside blend (flowing phases by
// sigma, then the solid by psi); chi = 1 - H_body.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_props(Phys P, const double* __restrict__ sigma, double t,
                                               double* __restrict__ rho, double* __restrict__ rfl,
                                               double* __restrict__ mu, double* __restrict__ chi) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const size_t c = i + (size_t)n.nx * (j + (size_t)n.ny * k);
  double zd;
  const double psi = body_psi(P, (i + 0.5) * P.h, (j + 0.5) * P.h, (k + 0.5) * P.h, t, &zd);
  const double hf = heaviside(sigma[c], P.eps);
  const double hb = heaviside(psi, P.eps);
  const double rf = P.rho_w + (P.rho_a - P.rho_w) * hf;
  const double mf = P.mu_w + (P.mu_a - P.mu_w) * hf;
  rfl[c] = rf;
  rho[c] = P.rho_s + (rf - P.rho_s) * hb;
  mu[c] = P.mu_s + (mf - P.mu_s) * hb;
  chi[c] = 1.0 - hb;
}

// --------------------------------------------------------------------------
// momentum predictor for velocity component C (faces normal to C)
// --------------------------------------------------------------------------
// Viscous stress of component C along direction D at a face,
// ((tau_+) - (tau_-))/h: tau = 2 mu du_C/dx_C at the cell centres either side
// (D = C), else mu (du_C/dx_D + du_D/dx_C) on the edges either side with the
// mean of their four cell viscosities.  m1, p1: the face's neighbours along D;
// dvp, dvm: du_D/dx_C on the two edges.  *a (if not null) receives the
// magnitude of the coefficient of the face's own value.
template <int C, int D>
__device__ __forceinline__ double visc_stress(const double* __restrict__ mu, const Dims& n, int i, int j, int k,
                                              double uf, double m1, double p1, double dvp, double dvm, double ih,
                                              double* a) {
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  constexpr int di = (D == 0), dj = (D == 1), dk = (D == 2);
  double tp, tm;
  if constexpr (C == D) {
    const double mup = cv(mu, n, i, j, k), mum = cv(mu, n, i - ci, j - cj, k - ck);
    tp = 2.0 * mup * (p1 - uf) * ih;
    tm = 2.0 * mum * (uf - m1) * ih;
    if (a) *a = 2.0 * (mup + mum) * ih * ih;
  } else {
    const double mep = 0.25 * (cv(mu, n, i - ci, j - cj, k - ck) + cv(mu, n, i, j, k) +
                               cv(mu, n, i - ci + di, j - cj + dj, k - ck + dk) +
                               cv(mu, n, i + di, j + dj, k + dk));
    const double mem = 0.25 * (cv(mu, n, i - ci - di, j - cj - dj, k - ck - dk) +
                               cv(mu, n, i - di, j - dj, k - dk) + cv(mu, n, i - ci, j - cj, k - ck) +
                               cv(mu, n, i, j, k));
    tp = mep * ((p1 - uf) * ih + dvp);
    tm = mem * ((uf - m1) * ih + dvm);
    if (a) *a = (mep + mem) * ih * ih;
  }
  return (tp - tm) * ih;
}

// One direction D of the predictor of component C: advection (advective
// form), viscous stress, and with CONS the consistent transport's mass flux
// (Koren-limited upwind face density at t^n times the advecting velocity)
// and the momentum it carries (times the same upwind velocity).
template <int C, int D, bool CONS>
__device__ __forceinline__ void mom_dir(const double* __restrict__ uc, const double* __restrict__ ud,
                                        const double* __restrict__ mu, const double* __restrict__ rho_n,
                                        const Dims& n, int i, int j, int k, double uf, double ih, double& adv,
                                        double& visc, double& conv, double& mflux) {
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  constexpr int di = (D == 0), dj = (D == 1), dk = (D == 2);
  const double m2 = fv<C>(uc, n, i - 2 * di, j - 2 * dj, k - 2 * dk);
  const double m1 = fv<C>(uc, n, i - di, j - dj, k - dk);
  const double p1 = fv<C>(uc, n, i + di, j + dj, k + dk);
  const double p2 = fv<C>(uc, n, i + 2 * di, j + 2 * dj, k + 2 * dk);
  double ap, am, dvp = 0.0, dvm = 0.0;
  if constexpr (C == D) {
    ap = 0.5 * (uf + p1);
    am = 0.5 * (m1 + uf);
  } else {
    // transverse velocity on the two faces meeting the edge above / below
    const double vpp = fv<D>(ud, n, i + di, j + dj, k + dk);
    const double vpm = fv<D>(ud, n, i + di - ci, j + dj - cj, k + dk - ck);
    const double vmp = fv<D>(ud, n, i, j, k);
    const double vmm = fv<D>(ud, n, i - ci, j - cj, k - ck);
    ap = 0.5 * (vpm + vpp);
    am = 0.5 * (vmm + vmp);
    dvp = (vpp - vpm) * ih;
    dvm = (vmp - vmm) * ih;
  }
  const double vp = koren_face(ap, m1, uf, p1, p2);
  const double vm = koren_face(am, m2, m1, uf, p1);
  adv += ap * (vp - uf) - am * (vm - uf);
  if constexpr (CONS) {
    // face density at t^n of the face o steps along D: mean of its two cells
    auto rf = [&](int o) {
      return 0.5 * (cv(rho_n, n, i - ci + o * di, j - cj + o * dj, k - ck + o * dk) +
                    cv(rho_n, n, i + o * di, j + o * dj, k + o * dk));
    };
    const double rm2 = rf(-2), rm1 = rf(-1), r0 = rf(0), rp1 = rf(1), rp2 = rf(2);
    const double mp = ap * koren_face(ap, rm1, r0, rp1, rp2);
    const double mm = am * koren_face(am, rm2, rm1, r0, rp1);
    conv += mp * vp - mm * vm;
    mflux += mp - mm;
  }
  visc += visc_stress<C, D>(mu, n, i, j, k, uf, m1, p1, dvp, dvm, ih, nullptr);
}

// The predictor of component C.  CONS: the conservative form with
// consistent mass/momentum transport, from the cell density rho_n at t^n:
// (rb u* - rho^n_f u^n)/dt + conv/h = forces, rb = rho^n_f - dt mflux/h, and
// beta from rb; otherwise the advective form with rho_f at t^{n+1}.
template <int C, bool CONS>
__global__ void __launch_bounds__(256) k_momentum(Phys P, const double* __restrict__ u,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ rho,
                                                  const double* __restrict__ rfl,
                                                  const double* __restrict__ mu,
                                                  const double* __restrict__ chi,
                                                  const double* __restrict__ rho_n, double dt, double t1,
                                                  double* __restrict__ out, double* __restrict__ beta,
                                                  float* __restrict__ betaf, double* __restrict__ cn_rhs,
                                                  double* __restrict__ cn_diag, double* __restrict__ flag) {
  const Dims n = P.n;
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  const int mx = n.nx + ci, my = n.ny + cj, mz = n.nz + ck;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= mx || j >= my || k >= mz) return;
  const size_t f = i + (size_t)mx * (j + (size_t)my * k);
  const bool wall = (C == 0) ? (i == 0 || i == n.nx) : (C == 1) ? (j == 0 || j == n.ny) : (k == 0);
  if (wall) {
    // the inlet of a wave tank carries the generated wave's velocity
    out[f] = (C == 0 && i == 0 && P.gen_len > 0.0) ? tank_vel(P, 0, 0.0, (k + 0.5) * P.h, t1) : 0.0;
    beta[f] = 0.0;
    betaf[f] = 0.0f;
    if (cn_rhs) {
      cn_rhs[f] = 0.0;
      cn_diag[f] = 0.0;   // marks a face the Crank-Nicolson sweeps keep
    }
    return;
  }
  const double* uc = (C == 0) ? u : (C == 1) ? v : w;
  const double uf = uc[f];
  const double ih = 1.0 / P.h;
  double adv = 0.0, visc = 0.0, conv = 0.0, mflux = 0.0;
  mom_dir<C, 0, CONS>(uc, u, mu, rho_n, n, i, j, k, uf, ih, adv, visc, conv, mflux);
  mom_dir<C, 1, CONS>(uc, v, mu, rho_n, n, i, j, k, uf, ih, adv, visc, conv, mflux);
  mom_dir<C, 2, CONS>(uc, w, mu, rho_n, n, i, j, k, uf, ih, adv, visc, conv, mflux);
  adv *= ih;
  const double rf = 0.5 * (cv(rho, n, i - ci, j - cj, k - ck) + cv(rho, n, i, j, k));
  const double rff = 0.5 * (cv(rfl, n, i - ci, j - cj, k - ck) + cv(rfl, n, i, j, k));
  const double xf = 0.5 * (cv(chi, n, i - ci, j - cj, k - ck) + cv(chi, n, i, j, k));
  double ub = 0.0;
  if (C == 2 && P.nb > 0) body_psi(P, (i + 0.5) * P.h, (j + 0.5) * P.h, k * P.h, t1, &ub);
  const double grav = (C == 2) ? -P.g * rff : 0.0;
  const double pen = xf * P.inv_kp;
  const double damp = vort_coeff(P, (C == 2) ? k * P.h : (k + 0.5) * P.h, dt);   // -g u, implicit
  // Crank-Nicolson keeps half the viscous term at t^n on the right-hand side
  // and writes the first iterate of its sweeps (the explicit value)
  const double wv = cn_rhs ? 0.5 : 1.0;
  if constexpr (CONS) {
    const double r0 = 0.5 * (cv(rho_n, n, i - ci, j - cj, k - ck) + cv(rho_n, n, i, j, k));
    const double rb = r0 - dt * mflux * ih;
    // a carried density at or below zero makes the projection operator
    // indefinite: the step is past the transport's Courant bound
    if (!(rb > 0.0)) *flag = 1.0;
    const double num = r0 * uf / dt - conv * ih + wv * visc + grav + pen * ub;
    const double den = rb / dt + pen + damp;
    out[f] = cn_rhs ? (num + 0.5 * visc) / den : num / den;
    if (cn_rhs) {
      cn_rhs[f] = num;
      cn_diag[f] = den;
    }
    const double bt = 1.0 / (rb + P.pen_w * dt * pen);
    beta[f] = bt;
    betaf[f] = (float)bt;
    return;
  }
  const double num = rf * (uf / dt - adv) + wv * visc + grav + pen * ub;
  const double den = rf / dt + pen + damp;
  out[f] = cn_rhs ? (num + 0.5 * visc) / den : num / den;
  if (cn_rhs) {
    cn_rhs[f] = num;
    cn_diag[f] = den;
  }
  const double bt = 1.0 / (rf + P.pen_w * dt * pen);
  beta[f] = bt;
  betaf[f] = (float)bt;
}

// Viscous stress of component C along D from the iterate, with its diagonal.
template <int C, int D>
__device__ __forceinline__ void sweep_dir(const double* __restrict__ uc, const double* __restrict__ ud,
                                          const double* __restrict__ mu, const Dims& n, int i, int j, int k,
                                          double uf, double ih, double& L, double& a) {
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  constexpr int di = (D == 0), dj = (D == 1), dk = (D == 2);
  const double m1 = fv<C>(uc, n, i - di, j - dj, k - dk);
  const double p1 = fv<C>(uc, n, i + di, j + dj, k + dk);
  double dvp = 0.0, dvm = 0.0;
  if constexpr (C != D) {
    dvp = (fv<D>(ud, n, i + di, j + dj, k + dk) - fv<D>(ud, n, i + di - ci, j + dj - cj, k + dk - ck)) * ih;
    dvm = (fv<D>(ud, n, i, j, k) - fv<D>(ud, n, i - ci, j - cj, k - ck)) * ih;
  }
  double ad;
  L += visc_stress<C, D>(mu, n, i, j, k, uf, m1, p1, dvp, dvm, ih, &ad);
  a += ad;
}

// Largest value over a 256-thread block (64 x 4 or 64 x 1 x 4), two
// quantities at once; thread 0 returns them.
__device__ __forceinline__ void block_max2(double& a, double& b) {
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_down(a, off, 64));
    b = fmax(b, __shfl_down(b, off, 64));
  }
  __shared__ double sm[4][2];
  const int tid = threadIdx.x + 64 * (threadIdx.y + blockDim.y * threadIdx.z);
  if ((tid & 63) == 0) {
    sm[tid >> 6][0] = a;
    sm[tid >> 6][1] = b;
  }
  __syncthreads();
  if (tid == 0) {
    a = fmax(fmax(sm[0][0], sm[1][0]), fmax(sm[2][0], sm[3][0]));
    b = fmax(fmax(sm[0][1], sm[1][1]), fmax(sm[2][1], sm[3][1]));
  }
}

// One point-Jacobi sweep of the Crank-Nicolson viscous system of component C,
//   D_f u_f - 1/2 L(u)_f = rhs_f,
// from the iterate (u, v, w): u_f <- (rhs_f + 1/2 (L(u)_f + a_f u_f)) / (D_f + 1/2 a_f),
// a_f the magnitude of L's diagonal; a face with D_f = 0 (a wall or the
// inlet) keeps its value.  With part, the block's largest |u_new - u| and
// largest |u_new| over the faces it updates go to part[2 lin], part[2 lin + 1].
template <int C>
__global__ void __launch_bounds__(256) k_cn_sweep(Phys P, const double* __restrict__ u,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ mu,
                                                  const double* __restrict__ rhs,
                                                  const double* __restrict__ diag, double* __restrict__ out,
                                                  double* __restrict__ part) {
  const Dims n = P.n;
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  const int mx = n.nx + ci, my = n.ny + cj, mz = n.nz + ck;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  double du = 0.0, um = 0.0;
  if (i < mx && j < my && k < mz) {
    const size_t f = i + (size_t)mx * (j + (size_t)my * k);
    const double* uc = (C == 0) ? u : (C == 1) ? v : w;
    const double uf = uc[f];
    const double dg = diag[f];
    double nv = uf;
    if (dg != 0.0) {
      const double ih = 1.0 / P.h;
      double L = 0.0, a = 0.0;
      sweep_dir<C, 0>(uc, u, mu, n, i, j, k, uf, ih, L, a);
      sweep_dir<C, 1>(uc, v, mu, n, i, j, k, uf, ih, L, a);
      sweep_dir<C, 2>(uc, w, mu, n, i, j, k, uf, ih, L, a);
      nv = (rhs[f] + 0.5 * (L + a * uf)) / (dg + 0.5 * a);
      du = fabs(nv - uf);
      um = fabs(nv);
    }
    out[f] = nv;
  }
  if (part) {   // uniform over the grid
    block_max2(du, um);
    if (threadIdx.x + threadIdx.y + threadIdx.z == 0) {
      part[2 * (size_t)tl.lin] = du;
      part[2 * (size_t)tl.lin + 1] = um;
    }
  }
}

// The CFL rule's per-block maximum of |u_c| + |v_c| + |w_c|, each cell
// velocity the mean of its two faces; a value that is not finite counts as
// infinite (a maximum would otherwise drop a NaN).
__global__ void __launch_bounds__(256) k_cfl(Phys P, const double* __restrict__ u, const double* __restrict__ v,
                                             const double* __restrict__ w, double* __restrict__ partials) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  double m = 0.0, unused = 0.0;
  if (i < n.nx && j < n.ny && k < n.nz) {
    const size_t sxy = (size_t)n.nx * n.ny;
    const size_t c = i + (size_t)n.nx * j + sxy * k;
    const size_t fu = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
    const size_t fvv = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
    const double uc = 0.5 * fabs(u[fu] + u[fu + 1]);
    const double vc = 0.5 * fabs(v[fvv] + v[fvv + n.nx]);
    const double wc = 0.5 * fabs(w[c] + w[c + sxy]);
    const double sum = (uc + vc) + wc;
    m = isfinite(sum) ? sum : INFINITY;
  }
  block_max2(m, unused);
  if (threadIdx.x + threadIdx.y + threadIdx.z == 0) partials[tl.lin] = m;
}

// out[q] = max over p of partials[K p + q], q < K (one 1024-thread block)
template <int K>
__global__ void __launch_bounds__(1024) k_max_finalize(const double* __restrict__ partials, int nparts,
                                                       double* __restrict__ out) {
  double m[2] = {0.0, 0.0};
  for (int p = threadIdx.x; p < nparts; p += 1024)
#pragma unroll
    for (int q = 0; q < K; ++q) m[q] = fmax(m[q], partials[(size_t)K * p + q]);
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < K; ++q) m[q] = fmax(m[q], __shfl_down(m[q], off, 64));
  __shared__ double sm[16][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < K; ++q) sm[wid][q] = m[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[2] = {0.0, 0.0};
    for (int w = 0; w < 16; ++w)
#pragma unroll
      for (int q = 0; q < K; ++q) r[q] = fmax(r[q], sm[w][q]);
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] = r[q];
  }
}

// b = -div_h(u*) / dt
__global__ void __launch_bounds__(256) k_rhs(Phys P, const double* __restrict__ us,
                                             const double* __restrict__ vs,
                                             const double* __restrict__ ws, double scale,
                                             double* __restrict__ b) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t c = i + (size_t)n.nx * j + sxy * k;
  const size_t fu = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fv_ = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  const double div = (us[fu + 1] - us[fu]) + (vs[fv_ + n.nx] - vs[fv_]) + (ws[c + sxy] - ws[c]);
  b[c] = div * scale;
}

// u^{n+1} = u* - dt beta grad_h p on non-wall faces of component C
template <int C>
__global__ void __launch_bounds__(256) k_correct(Phys P, const double* __restrict__ us,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ beta, double dt,
                                                 double* __restrict__ u) {
  const Dims n = P.n;
  constexpr int ci = (C == 0), cj = (C == 1), ck = (C == 2);
  const int mx = n.nx + ci, my = n.ny + cj, mz = n.nz + ck;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= mx || j >= my || k >= mz) return;
  const size_t f = i + (size_t)mx * (j + (size_t)my * k);
  const bool wall = (C == 0) ? (i == 0 || i == n.nx) : (C == 1) ? (j == 0 || j == n.ny) : (k == 0);
  if (wall) {
    u[f] = (C == 0 && i == 0 && P.gen_len > 0.0) ? us[f] : 0.0;   // a tank's inlet keeps its wave
    return;
  }
  const double ih = 1.0 / P.h;
  double grad;
  if (C == 2 && k == n.nz) {
    grad = -cv(p, n, i, j, k - 1) * (2.0 * ih);   // p = 0 half a cell above
  } else {
    grad = (cv(p, n, i, j, k) - cv(p, n, i - ci, j - cj, k - ck)) * ih;
  }
  u[f] = us[f] - dt * beta[f] * grad;
}

// The wave tank's relaxation zones after a step: phi <- a phi + (1 - a) target
// over the columns of the generation zone [0, gen_len] (target: the wave at
// t) and of the damping zone [L - damp_len, L] (still water).  The launch
// covers only those columns: column q < ng is x-index q, the others
// x-index i_damp + (q - ng).  C = 0, 1, 2: the velocity faces; C = 3: sigma.
template <int C>
__global__ void __launch_bounds__(256) k_relax(Phys P, double t, int ng, int i_damp, int ncol,
                                               double* __restrict__ a) {
  const Dims n = P.n;
  const int my = n.ny + (C == 1), mz = n.nz + (C == 2), mx = n.nx + (C == 0);
  const Tile tl = xcd_tile();
  const int q = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (q >= ncol || j >= my || k >= mz) return;
  const int i = q < ng ? q : i_damp + (q - ng);
  if (i >= mx) return;
  const double h = P.h;
  const double x = (C == 0) ? i * h : (i + 0.5) * h;
  const double z = (C == 2) ? k * h : (k + 0.5) * h;
  const double L = n.nx * h;
  bool gen;
  double al;
  if (P.gen_len > 0.0 && x <= P.gen_len) {
    gen = true;
    al = relax_weight(1.0 - x / P.gen_len);
  } else if (P.damp_len > 0.0 && x >= L - P.damp_len) {
    gen = false;
    al = relax_weight((x - (L - P.damp_len)) / P.damp_len);
  } else {
    return;
  }
  double target;
  if constexpr (C == 3)
    target = z - (P.depth + (gen ? tank_eta(P, x, t) : 0.0));
  else
    target = gen ? tank_vel(P, C, x, z, t) : 0.0;
  const size_t f = i + (size_t)mx * (j + (size_t)my * k);
  a[f] = al * a[f] + (1.0 - al) * target;
}

// Hydrodynamic force on body m, eqn_int_fh (Sec. "Fluid-structure
// coupling"): the sum over its stair-step surface (the faces across which the
// body's level set changes sign, Sec. "NLFK calculation") of
// (-p_f n_f + mu_f (grad u + grad u^T) . n_f) dA_f, with n_f out of the body,
// p_f the two cell pressures interpolated linearly to psi = 0, mu_f their
// mean viscosity, central differences at the face centre, dA_f = h^2 (h in
// 2-D).  One thread per cell of the box [lo, lo + ext), for the three faces
// below it; the box holds every cell within two of the body, so no face of
// the surface lies on its edge.  Per-block partials (Fx, Fy, Fz) in tile
// order.
__global__ void __launch_bounds__(256) k_hydro_force(Phys P, int m, int i0, int j0, int k0, int ex, int ey,
                                                     int ez, double t, const double* __restrict__ p,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ mu,
                                                     double* __restrict__ partials) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int li = tl.x * blockDim.x + threadIdx.x;
  const int lj = tl.y * blockDim.y + threadIdx.y;
  const int lk = tl.z * blockDim.z + threadIdx.z;
  double F[3] = {0.0, 0.0, 0.0};
  if (li < ex && lj < ey && lk < ez) {
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const BodyK B = P.body[m];
    const double h = P.h, ih = 1.0 / h;
    const bool two_d = (n.ny == 1);
    const double dA = two_d ? h : h * h;
    double zd;
    const double psb = body_psi_one(B, (i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h, t, &zd);
    // cell-centred mean of component c at a cell
    auto cmean = [&](int c, int a, int b2, int c2) {
      switch (c) {
        case 0: return 0.5 * (fv<0>(u, n, a, b2, c2) + fv<0>(u, n, a + 1, b2, c2));
        case 1: return 0.5 * (fv<1>(v, n, a, b2, c2) + fv<1>(v, n, a, b2 + 1, c2));
        default: return 0.5 * (fv<2>(w, n, a, b2, c2) + fv<2>(w, n, a, b2, c2 + 1));
      }
    };
    // face value of component d at face index (a, b2, c2)
    auto face = [&](int d, int a, int b2, int c2) {
      return d == 0 ? fv<0>(u, n, a, b2, c2) : (d == 1 ? fv<1>(v, n, a, b2, c2) : fv<2>(w, n, a, b2, c2));
    };
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d == 1 && two_d) continue;
      const int di = (d == 0), dj = (d == 1), dk = (d == 2);
      if ((d == 0 && i < 1) || (d == 1 && j < 1) || (d == 2 && k < 1)) continue;
      const int ia = i - di, ja = j - dj, ka = k - dk;
      const double psa = body_psi_one(B, (ia + 0.5) * h, (ja + 0.5) * h, (ka + 0.5) * h, t, &zd);
      if ((psa < 0.0) == (psb < 0.0)) continue;
      const double nd = (psa < 0.0) ? 1.0 : -1.0;
      const double pa = cv(p, n, ia, ja, ka), pb = cv(p, n, i, j, k);
      const double wa = fabs(psa), wb = fabs(psb);
      const double pf = (wb * pa + wa * pb) / (wa + wb);
      const double muf = 0.5 * (cv(mu, n, ia, ja, ka) + cv(mu, n, i, j, k));
      F[d] -= pf * nd * dA;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c == 1 && two_d) continue;
        double G;
        if (c == d) {
          G = (face(d, i + di, j + dj, k + dk) - face(d, i - di, j - dj, k - dk)) * ih;
        } else {
          const int ci = (c == 0), cj = (c == 1), ck = (c == 2);
          G = (cmean(c, i, j, k) - cmean(c, ia, ja, ka)) * ih +
              (face(d, i + ci, j + cj, k + ck) - face(d, i - ci, j - cj, k - ck)) * (0.5 * ih);
        }
        F[c] += muf * G * nd * dA;
      }
    }
  }
  // fixed-order block sum
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < 3; ++q) F[q] += __shfl_down(F[q], off, 64);
  __shared__ double sm[4][3];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  if ((tid & 63) == 0)
#pragma unroll
    for (int q = 0; q < 3; ++q) sm[tid >> 6][q] = F[q];
  __syncthreads();
  if (tid == 0)
#pragma unroll
    for (int q = 0; q < 3; ++q) partials[3 * (size_t)tl.lin + q] = (sm[0][q] + sm[1][q]) + (sm[2][q] + sm[3][q]);
}

// per-block partial diagnostics: max|div|, water volume, kinetic energy, max|u_c|
__global__ void __launch_bounds__(256) k_diag(Phys P, const double* __restrict__ sigma,
                                              const double* __restrict__ u,
                                              const double* __restrict__ v,
                                              const double* __restrict__ w,
                                              double* __restrict__ partials) {
  const Dims n = P.n;
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  double vals[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n.nx && j < n.ny && k < n.nz) {
    const size_t sxy = (size_t)n.nx * n.ny;
    const size_t c = i + (size_t)n.nx * j + sxy * k;
    const size_t fu = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
    const size_t fvv = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
    const double um = u[fu], up = u[fu + 1], vm = v[fvv], vp = v[fvv + n.nx], wm = w[c],
                 wp = w[c + sxy];
    const double h = P.h;
    const double vol = (n.ny == 1) ? h * h : h * h * h;
    const double div = ((up - um) + (vp - vm) + (wp - wm)) / h;
    const double hf = heaviside(sigma[c], P.eps);
    const double rf = P.rho_w + (P.rho_a - P.rho_w) * hf;
    const double uc = 0.5 * (up + um), vc = 0.5 * (vp + vm), wc = 0.5 * (wp + wm);
    vals[0] = fabs(div);
    vals[1] = (1.0 - hf) * vol;
    vals[2] = 0.5 * rf * (uc * uc + vc * vc + wc * wc) * vol;
    vals[3] = fmax(fmax(fmax(fabs(um), fabs(up)), fmax(fabs(vm), fabs(vp))), fmax(fabs(wm), fabs(wp)));
  }
  for (int off = 32; off > 0; off >>= 1) {
    vals[0] = fmax(vals[0], __shfl_down(vals[0], off, 64));
    vals[1] += __shfl_down(vals[1], off, 64);
    vals[2] += __shfl_down(vals[2], off, 64);
    vals[3] = fmax(vals[3], __shfl_down(vals[3], off, 64));
  }
  __shared__ double sm[4][4];
  const int tid = threadIdx.x + 64 * (threadIdx.y + blockDim.y * threadIdx.z);
  const int lane = tid & 63, wid = tid >> 6;
  if (lane == 0)
    for (int q = 0; q < 4; ++q) sm[wid][q] = vals[q];
  __syncthreads();
  if (tid == 0) {
    const size_t blk = tl.lin;
    partials[4 * blk + 0] = fmax(fmax(sm[0][0], sm[1][0]), fmax(sm[2][0], sm[3][0]));
    partials[4 * blk + 1] = (sm[0][1] + sm[1][1]) + (sm[2][1] + sm[3][1]);
    partials[4 * blk + 2] = (sm[0][2] + sm[1][2]) + (sm[2][2] + sm[3][2]);
    partials[4 * blk + 3] = fmax(fmax(sm[0][3], sm[1][3]), fmax(sm[2][3], sm[3][3]));
  }
}

__global__ void __launch_bounds__(1024) k_diag_finalize(const double* __restrict__ partials, int nparts,
                                                        double* __restrict__ scal) {
  double vals[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nparts; q += 1024) {
    vals[0] = fmax(vals[0], partials[4 * q + 0]);
    vals[1] += partials[4 * q + 1];
    vals[2] += partials[4 * q + 2];
    vals[3] = fmax(vals[3], partials[4 * q + 3]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    vals[0] = fmax(vals[0], __shfl_down(vals[0], off, 64));
    vals[1] += __shfl_down(vals[1], off, 64);
    vals[2] += __shfl_down(vals[2], off, 64);
    vals[3] = fmax(vals[3], __shfl_down(vals[3], off, 64));
  }
  __shared__ double sm[16][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int q = 0; q < 4; ++q) sm[wid][q] = vals[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < 16; ++q) {
      r[0] = fmax(r[0], sm[q][0]);
      r[1] += sm[q][1];
      r[2] += sm[q][2];
      r[3] = fmax(r[3], sm[q][3]);
    }
    for (int q = 0; q < 4; ++q) scal[S_DIAG + q] = r[q];
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_advect(const Phys& P, const double* s, const double* u, const double* v, const double* w,
                   double dt, double* out, hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_advect, g.grid, g.block, 0, st, P, s, u, v, w, dt, out);
}

void launch_reinit(const Phys& P, const double* s0, const double* cur, double* nxt, double dtau,
                   hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_reinit, g.grid, g.block, 0, st, P, s0, cur, nxt, dtau);
}

void launch_copy(const double* src, double* dst, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
}

// A launch evaluates the bodies at one time: a prescribed heave's sine and
// cosine are taken here, once, and the kernels receive those bodies with
// zeta, zdot set and fh = 1, as for a free body's state (fh is read on the
// device only to choose between the stored heave and the formula).  The
// kernels had evaluated both per cell or face.
static Phys heave_at(const Phys& P, double t) {
  Phys Q = P;
  for (int m = 0; m < Q.nb; ++m) {
    BodyK& B = Q.body[m];
    if (B.fh) continue;
    const double arg = B.om * t + B.ph;
    B.zeta = B.amp * std::sin(arg);
    B.zdot = B.amp * B.om * std::cos(arg);
    B.fh = 1;
  }
  return Q;
}

void launch_props(const Phys& P, const double* sigma, double t, double* rho, double* rfl, double* mu,
                  double* chi, hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_props, g.grid, g.block, 0, st, heave_at(P, t), sigma, t, rho, rfl, mu, chi);
}

void launch_momentum(const Phys& P, const double* u, const double* v, const double* w,
                     const double* rho, const double* rfl, const double* mu, const double* chi,
                     const double* rho_n, double dt, double t1, double* us, double* vs, double* ws, double* bx,
                     double* by, double* bz, float* bxf, float* byf, float* bzf, double* const* cn_rhs,
                     double* const* cn_diag, double* flag, hipStream_t st) {
  const Dims n = P.n;
  const Phys Pt = heave_at(P, t1);
  Geo gx = geo3(n.nx + 1, n.ny, n.nz);
  Geo gy = geo3(n.nx, n.ny + 1, n.nz);
  Geo gz = geo3(n.nx, n.ny, n.nz + 1);
  double* r[3] = {nullptr, nullptr, nullptr};
  double* dg[3] = {nullptr, nullptr, nullptr};
  if (cn_rhs)
    for (int c = 0; c < 3; ++c) r[c] = cn_rhs[c], dg[c] = cn_diag[c];
  if (rho_n) {
    hipLaunchKernelGGL((k_momentum<0, true>), gx.grid, gx.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                       t1, us, bx, bxf, r[0], dg[0], flag);
    hipLaunchKernelGGL((k_momentum<1, true>), gy.grid, gy.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                       t1, vs, by, byf, r[1], dg[1], flag);
    hipLaunchKernelGGL((k_momentum<2, true>), gz.grid, gz.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                       t1, ws, bz, bzf, r[2], dg[2], flag);
    return;
  }
  hipLaunchKernelGGL((k_momentum<0, false>), gx.grid, gx.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                     t1, us, bx, bxf, r[0], dg[0], flag);
  hipLaunchKernelGGL((k_momentum<1, false>), gy.grid, gy.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                     t1, vs, by, byf, r[1], dg[1], flag);
  hipLaunchKernelGGL((k_momentum<2, false>), gz.grid, gz.block, 0, st, Pt, u, v, w, rho, rfl, mu, chi, rho_n, dt,
                     t1, ws, bz, bzf, r[2], dg[2], flag);
}

void launch_cn_sweep(const Phys& P, const double* u, const double* v, const double* w, const double* mu,
                     double* const* rhs, double* const* diag, double* uo, double* vo, double* wo, double* part,
                     double* out2, hipStream_t st) {
  const Dims n = P.n;
  Geo gx = geo3(n.nx + 1, n.ny, n.nz);
  Geo gy = geo3(n.nx, n.ny + 1, n.nz);
  Geo gz = geo3(n.nx, n.ny, n.nz + 1);
  const size_t bx = (size_t)gx.grid.x * gx.grid.y * gx.grid.z, by = (size_t)gy.grid.x * gy.grid.y * gy.grid.z;
  const size_t bz = (size_t)gz.grid.x * gz.grid.y * gz.grid.z;
  hipLaunchKernelGGL(k_cn_sweep<0>, gx.grid, gx.block, 0, st, P, u, v, w, mu, rhs[0], diag[0], uo, part);
  hipLaunchKernelGGL(k_cn_sweep<1>, gy.grid, gy.block, 0, st, P, u, v, w, mu, rhs[1], diag[1], vo,
                     part ? part + 2 * bx : nullptr);
  hipLaunchKernelGGL(k_cn_sweep<2>, gz.grid, gz.block, 0, st, P, u, v, w, mu, rhs[2], diag[2], wo,
                     part ? part + 2 * (bx + by) : nullptr);
  if (part)
    hipLaunchKernelGGL(k_max_finalize<2>, dim3(1), dim3(1024), 0, st, part, (int)(bx + by + bz), out2);
}

int cn_part_blocks(const Dims& n) {
  Geo gx = geo3(n.nx + 1, n.ny, n.nz);
  Geo gy = geo3(n.nx, n.ny + 1, n.nz);
  Geo gz = geo3(n.nx, n.ny, n.nz + 1);
  return (int)((size_t)gx.grid.x * gx.grid.y * gx.grid.z + (size_t)gy.grid.x * gy.grid.y * gy.grid.z +
               (size_t)gz.grid.x * gz.grid.y * gz.grid.z);
}

void launch_cfl_max(const Phys& P, const double* u, const double* v, const double* w, double* partials,
                    double* out, hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  const int nb = (int)(g.grid.x * g.grid.y * g.grid.z);
  hipLaunchKernelGGL(k_cfl, g.grid, g.block, 0, st, P, u, v, w, partials);
  hipLaunchKernelGGL(k_max_finalize<1>, dim3(1), dim3(1024), 0, st, partials, nb, out);
}

void launch_rhs(const Phys& P, const double* us, const double* vs, const double* ws, double dt,
                double* b, hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_rhs, g.grid, g.block, 0, st, P, us, vs, ws, -1.0 / (P.h * dt), b);
}

void launch_correct(const Phys& P, const double* us, const double* vs, const double* ws,
                    const double* p, const double* bx, const double* by, const double* bz, double dt,
                    double* u, double* v, double* w, hipStream_t st) {
  const Dims n = P.n;
  Geo gx = geo3(n.nx + 1, n.ny, n.nz);
  hipLaunchKernelGGL(k_correct<0>, gx.grid, gx.block, 0, st, P, us, p, bx, dt, u);
  Geo gy = geo3(n.nx, n.ny + 1, n.nz);
  hipLaunchKernelGGL(k_correct<1>, gy.grid, gy.block, 0, st, P, vs, p, by, dt, v);
  Geo gz = geo3(n.nx, n.ny, n.nz + 1);
  hipLaunchKernelGGL(k_correct<2>, gz.grid, gz.block, 0, st, P, ws, p, bz, dt, w);
}

int diag_blocks(const Phys& P) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  return (int)(g.grid.x * g.grid.y * g.grid.z);
}

int launch_diag_partials(const Phys& P, const double* sigma, const double* u, const double* v,
                         const double* w, double* partials, hipStream_t st) {
  Geo g = geo3(P.n.nx, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_diag, g.grid, g.block, 0, st, P, sigma, u, v, w, partials);
  return (int)(g.grid.x * g.grid.y * g.grid.z);
}

void launch_diag_finalize(const double* partials, int nparts, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_finalize, dim3(1), dim3(1024), 0, st, partials, nparts, scal);
}

int launch_hydro_force(const Phys& P, int m, double t, const double* p, const double* u, const double* v,
                       const double* w, const double* mu, double* partials, int max_blocks, hipStream_t st) {
  const BodyK& B = P.body[m];
  const double zeta = B.fh ? B.zeta : B.amp * sin(B.om * t + B.ph);
  // the body's extent, then every cell within two of it
  double lo[3], hi[3];
  if (B.kind == 0) {
    lo[0] = B.c0 - B.h0, hi[0] = B.c0 + B.h0;
    lo[1] = 0.0, hi[1] = P.n.ny * P.h;
    lo[2] = B.c2 + zeta - B.h2, hi[2] = B.c2 + zeta + B.h2;
  } else {
    lo[0] = B.c0 - B.h0, hi[0] = B.c0 + B.h0;
    lo[1] = B.c1 - B.h0, hi[1] = B.c1 + B.h0;
    lo[2] = B.h1 + zeta, hi[2] = B.h2 + zeta;
  }
  const int nn[3] = {P.n.nx, P.n.ny, P.n.nz};
  int a[3], e[3];
  for (int d = 0; d < 3; ++d) {
    const double L = std::floor(lo[d] / P.h) - 2.0, H = std::ceil(hi[d] / P.h) + 2.0;
    const int a0 = (int)std::max(0.0, std::min(L, (double)nn[d]));
    const int a1 = (int)std::max(0.0, std::min(H, (double)nn[d]));
    a[d] = a0;
    e[d] = a1 - a0;
  }
  if (e[0] <= 0 || e[1] <= 0 || e[2] <= 0) return 0;
  Geo g = geo3(e[0], e[1], e[2]);
  const long long blocks = (long long)g.grid.x * g.grid.y * g.grid.z;
  if (blocks > max_blocks) return -1;
  hipLaunchKernelGGL(k_hydro_force, g.grid, g.block, 0, st, heave_at(P, t), m, a[0], a[1], a[2], e[0], e[1], e[2], t, p, u, v,
                     w, mu, partials);
  return (int)blocks;
}

void launch_relax(const Phys& P, double t, double* sigma, double* u, double* v, double* w, hipStream_t st) {
  if (!(P.gen_len > 0.0) && !(P.damp_len > 0.0)) return;
  // columns that can lie in a zone: x-index 0..ng-1 (generation) and
  // i_damp..nx (damping), one spare column each way for the face arrays
  const double h = P.h;
  const int nx = P.n.nx;
  const int ng = P.gen_len > 0.0 ? std::min(nx + 1, (int)std::floor(P.gen_len / h) + 2) : 0;
  const int i_damp = P.damp_len > 0.0 ? std::max(ng, (int)std::floor((nx * h - P.damp_len) / h) - 1) : nx + 1;
  const int ncol = ng + std::max(0, nx + 1 - i_damp);
  if (ncol <= 0) return;
  Geo gu = geo3(ncol, P.n.ny, P.n.nz);
  hipLaunchKernelGGL(k_relax<0>, gu.grid, gu.block, 0, st, P, t, ng, i_damp, ncol, u);
  if (P.n.ny > 1) {
    Geo gv = geo3(ncol, P.n.ny + 1, P.n.nz);
    hipLaunchKernelGGL(k_relax<1>, gv.grid, gv.block, 0, st, P, t, ng, i_damp, ncol, v);
  }
  Geo gw = geo3(ncol, P.n.ny, P.n.nz + 1);
  hipLaunchKernelGGL(k_relax<2>, gw.grid, gw.block, 0, st, P, t, ng, i_damp, ncol, w);
  hipLaunchKernelGGL(k_relax<3>, gu.grid, gu.block, 0, st, P, t, ng, i_damp, ncol, sigma);
}

}  // namespace nsk
