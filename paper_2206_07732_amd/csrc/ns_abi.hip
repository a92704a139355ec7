// C ABI of the gfx950 library (declared in include/ns.h): context and
// workspace management, the V-cycle schedule and the flexible
// preconditioned CG driver.  Every arithmetic step runs in the kernels of
// ns_grid.hip and ns_mg.hip; this file only sequences launches on the
// caller's stream and reads back the one residual scalar per CG iteration
// that the stopping test needs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ns_internal.h"

using namespace nsk;

struct ns_ctx {
  ns_params P;
  ns_fields F;
  Phys phys;
  hipStream_t st;
  size_t nc, nu, nv, nw;
  // workspace views
  double *us, *vs, *ws;
  double *sig_a, *sig_b;
  double *rho, *rfl, *mu, *chi;
  double* rho_prev;   // consistent transport: the density of the level set the step starts from
  bool have_rho_n;    // rho holds the density at the start of the next momentum_step
  double* cn_rhs[3];  // Crank-Nicolson viscous term: right-hand side per face,
  double* cn_diag[3]; // implicit diagonal (0 on walls and the inlet),
  double* cn_tmp[3];  // and the second iterate of the Jacobi sweeps
  double* cnpart;     // per-block (largest change, largest |u*|) of a checked sweep
  int last_cn;        // sweeps the last predictor ran
  bool phase_on;      // ns_phase_timing
  bool ph_step;       // ns_step recorded the events of its first two phases
  hipEvent_t ph_ev[6];
  double *b, *r, *z, *zn, *d, *d2, *q;
  double *partials;
  double *scal;
  int nparts;
  int L;
  Level lev[32];
  double* host;       // pinned, coherent host mirror of the scalars
  double* host_dev;   // its device address
  double* hpart;      // pinned, coherent host partials (nparts <= kHostPartsMax), or null
  double* hpart_dev;  // their device address
  bool have_beta;
  int timed_kernel;   // -1 or an ns_timed_kernel id
  KTimer kt;
  hipEvent_t ev_rr;   // marks the residual read-back of a CG iteration
  int launch_mode;    // ns_launch_mode
  bool fine_rb;       // the finest level's red-black sweeps as one launch each
  bool face_tabs;     // the finest level's kernels read uniform face lines through their tables
  struct {
    double F[3];      // last hydrodynamic force (eqn_int_fh)
    double fpto;      // last power take-off force
  } bs[4];            // free-body state beside the heave kept in phys.body
  int nfree;          // number of free bodies
  bool force_ready;   // bs[].F belongs to the current fields
  double t_props;     // time of the last property evaluation
  double* fpart;      // pinned host copy of the force partials (3 per block per free body)
  int fcap;           // its capacity in blocks per body
  hipStream_t cap_st; // capture-only stream: the V-cycle graphs are recorded on it
  struct {
    int kind;
    const void* a;
    const void* b;
    const void* c;
    int flag;
    hipGraphExec_t exec;
  } gs[16];           // recorded CG segments, keyed by kind and vectors
  int ngs;
  ns_net* net;        // learned guess (not owned)
  struct {
    double gain;      // CG iterations the learned guess saves over p_prev (trial average)
    double t_inf;     // device time of the last inference (ms)
    double t_it;      // wall time per CG iteration of the last solve (ms)
    int trials;       // steps that ran the network so far
    int since;        // steps since the last trial
    hipEvent_t ev[2]; // around the last inference
  } ax;               // x0 = NS_X0_AUTO
  int tail64, tail32; // first level of the LDS tail per precision (L: none)
  size_t lds64, lds32;
  double* pack64;     // the tail levels' bx, by, bz, 1/D (tail kernel's LDS image)
  float* pack32;
  size_t npack64, npack32;
  char err[512];
};

namespace {

constexpr size_t kAlign = 256;

struct Carve {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

ns_status fail(ns_ctx* X, ns_status s, const char* fmt, ...) {
  if (X) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(X->err, sizeof(X->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

#define HIPCHK(X, call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail((X), NS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int count_levels(int nx, int ny, int nz) {
  int n[3] = {nx, ny, nz};
  bool act[3] = {nx > 1, ny > 1, nz > 1};
  int L = 1;
  while (L < 30) {
    bool ok = true;
    for (int d = 0; d < 3; ++d)
      if (act[d] && (n[d] < 2 || (n[d] & 1))) ok = false;
    if (!ok) break;
    for (int d = 0; d < 3; ++d)
      if (act[d]) n[d] /= 2;
    ++L;
  }
  return L;
}

bool valid_params(const ns_params* P, char* why, size_t nwhy) {
  if (!P) return snprintf(why, nwhy, "params is NULL"), false;
  if (P->nx < 2 || P->ny < 1 || P->nz < 2)
    return snprintf(why, nwhy, "grid %dx%dx%d: need nx >= 2, ny >= 1, nz >= 2", P->nx, P->ny, P->nz), false;
  {
    // cells and faces are indexed in 32-bit arithmetic: the largest face
    // array, (nx+1) ny nz or one of its two siblings, must stay below 2^31
    const double x = P->nx, y = P->ny, z = P->nz;
    const double faces = std::max(std::max((x + 1) * y * z, x * (y + 1) * z), x * y * (z + 1));
    if (faces > 2.0e9) return snprintf(why, nwhy, "grid %dx%dx%d too large: more than 2e9 faces", P->nx, P->ny, P->nz), false;
  }
  if (!(P->h > 0.0)) return snprintf(why, nwhy, "h must be > 0"), false;
  if (P->n_bodies < 0 || P->n_bodies > 4) return snprintf(why, nwhy, "n_bodies must be 0..4"), false;
  if (!(P->rho_w > 0 && P->rho_a > 0 && P->rho_s > 0))
    return snprintf(why, nwhy, "densities must be > 0"), false;
  if (!(P->n_cells > 0.0)) return snprintf(why, nwhy, "n_cells must be > 0"), false;
  if (P->reinit_iters < 0 || P->nu_pre < 0 || P->nu_post < 0 || P->coarse_sweeps < 0 || P->max_iters < 0)
    return snprintf(why, nwhy, "iteration counts must be >= 0"), false;
  if (P->prec != NS_PREC_FP64 && P->prec != NS_PREC_MIXED) return snprintf(why, nwhy, "bad prec"), false;
  if (P->x0 != NS_X0_ZERO && P->x0 != NS_X0_PREV && P->x0 != NS_X0_LEARNED && P->x0 != NS_X0_AUTO)
    return snprintf(why, nwhy, "bad x0"), false;
  if ((P->x0 == NS_X0_LEARNED || P->x0 == NS_X0_AUTO) && !(P->p_scale > 0.0))
    return snprintf(why, nwhy, "p_scale must be > 0 for the learned guess"), false;
  if (!(P->gen_len >= 0.0 && P->damp_len >= 0.0 && P->vort_width >= 0.0) || !std::isfinite(P->gen_len) ||
      !std::isfinite(P->damp_len) || !std::isfinite(P->vort_width))
    return snprintf(why, nwhy, "wave tank zone sizes must be finite and >= 0"), false;
  if (P->n_waves < 0 || P->n_waves > 64) return snprintf(why, nwhy, "n_waves must be 0..64"), false;
  if (P->consistent != 0 && P->consistent != 1) return snprintf(why, nwhy, "consistent must be 0 or 1"), false;
  if (P->cn_sweeps < 0 || P->cn_sweeps > 64) return snprintf(why, nwhy, "cn_sweeps must be 0..64"), false;
  if (P->cn_sweeps > 0 && !(P->cn_tol > 0.0 && std::isfinite(P->cn_tol)))
    return snprintf(why, nwhy, "cn_tol must be finite and > 0 with cn_sweeps > 0"), false;
  if ((P->gen_len > 0.0 || P->damp_len > 0.0) && !(P->depth > 0.0 && std::isfinite(P->depth)))
    return snprintf(why, nwhy, "a wave tank with relaxation zones needs depth > 0"), false;
  for (int q = 0; q < P->n_waves; ++q) {
    const auto& W = P->waves[q];
    if (!(std::isfinite(W.a) && std::isfinite(W.omega) && std::isfinite(W.phase) && W.kappa > 0.0 &&
          std::isfinite(W.kappa)))
      return snprintf(why, nwhy, "wave component %d: finite a, omega, phase and kappa > 0 needed", q), false;
  }
  for (int m = 0; m < P->n_bodies; ++m) {
    const ns_body& B = P->body[m];
    if (B.kind != 0 && B.kind != 1) return snprintf(why, nwhy, "bad body kind"), false;
    if (B.free_heave != 0 && B.free_heave != 1) return snprintf(why, nwhy, "free_heave must be 0 or 1"), false;
    if (B.free_heave && !(B.mass > 0.0 && std::isfinite(B.mass)))
      return snprintf(why, nwhy, "body %d: a free body needs mass > 0", m), false;
    if (B.free_heave && !(B.pto_damping >= 0.0 && std::isfinite(B.pto_damping) && std::isfinite(B.zeta0) &&
                          std::isfinite(B.zdot0)))
      return snprintf(why, nwhy, "body %d: pto_damping must be >= 0 and zeta0, zdot0 finite", m), false;
  }
  return true;
}

size_t pad4(size_t n) { return (n + 3) / 4 * 4; }

// elements of the tail pack from level l down: bx, by, bz and 1/D per level
size_t tail_pack_elems(const Level* lev, int L, int l) {
  size_t tot = 0;
  for (int q = l; q < L; ++q) {
    const Dims n = lev[q].n;
    const size_t c = (size_t)n.nx * n.ny * n.nz;
    tot += pad4((size_t)(n.nx + 1) * n.ny * n.nz) + pad4((size_t)n.nx * (n.ny + 1) * n.nz) +
           pad4((size_t)n.nx * n.ny * (n.nz + 1)) + pad4(c);
  }
  return tot;
}

// LDS elements of the tail from level l down: the pack, then b and e per
// level, then (when the tail restricts, i.e. has more than one level) a
// residual scratch of level l's size
size_t tail_elems(const Level* lev, int L, int l) {
  size_t tot = tail_pack_elems(lev, L, l);
  for (int q = l; q < L; ++q) {
    const Dims n = lev[q].n;
    tot += 2 * pad4((size_t)n.nx * n.ny * n.nz);
  }
  return tot + (l < L - 1 ? pad4((size_t)lev[l].n.nx * lev[l].n.ny * lev[l].n.nz) : 0);
}

// first level whose tail fits the LDS budget and the workgroup (L: none)
int plan_tail(const Level* lev, int L, size_t w, size_t* bytes) {
  for (int l = 0; l < L; ++l) {
    const Dims n = lev[l].n;
    const size_t pairs = (size_t)((n.nx + 1) / 2) * n.ny * n.nz;
    if (pairs > 2 * (size_t)kTailThreads) continue;
    if (L - l > kTailMaxLevels) continue;
    const size_t b = tail_elems(lev, L, l) * w;
    if (b <= kTailLdsBytes) {
      *bytes = b;
      return l;
    }
  }
  *bytes = 0;
  return L;
}

// lay out every internal array; with ctx == nullptr only the size is computed
size_t carve(const ns_params* P, ns_ctx* X, char* base) {
  Carve cv{base, 0};
  const size_t nc = (size_t)P->nx * P->ny * P->nz;
  const size_t nu = (size_t)(P->nx + 1) * P->ny * P->nz;
  const size_t nv = (size_t)P->nx * (P->ny + 1) * P->nz;
  const size_t nw = (size_t)P->nx * P->ny * (P->nz + 1);
  Dims n0{P->nx, P->ny, P->nz};
  const int nparts = std::max(cg_blocks(n0), 1);
  double* us = cv.take<double>(nu);
  double* vs = cv.take<double>(nv);
  double* ws = cv.take<double>(nw);
  double* sa = cv.take<double>(nc);
  double* sb = cv.take<double>(nc);
  double* rho = cv.take<double>(nc);
  double* rfl = cv.take<double>(nc);
  double* mu = cv.take<double>(nc);
  double* rho_prev = P->consistent ? cv.take<double>(nc) : nullptr;   // rho at t^n
  double* cn[9] = {};   // Crank-Nicolson: rhs, diagonal and second iterate of u, v, w
  if (P->cn_sweeps > 0)
    for (int q = 0; q < 9; ++q) cn[q] = cv.take<double>(q % 3 == 0 ? nu : q % 3 == 1 ? nv : nw);
  double* cnpart = P->cn_sweeps > 0 ? cv.take<double>(2 * (size_t)cn_part_blocks(n0)) : nullptr;
  double* chi = cv.take<double>(nc);
  double* b = cv.take<double>(nc);
  double* r = cv.take<double>(nc);
  double* z = cv.take<double>(nc);
  double* zn = cv.take<double>(nc);
  double* d = cv.take<double>(nc);
  double* d2 = cv.take<double>(nc);
  double* q = cv.take<double>(nc);
  double* part = cv.take<double>((size_t)4 * nparts);
  double* scal = cv.take<double>(S_COUNT);
  double* waves = cv.take<double>(4 * 64);   // the wave tank's components
  const int L = count_levels(P->nx, P->ny, P->nz);
  Level lev[32];
  bool act[3] = {P->nx > 1, P->ny > 1, P->nz > 1};
  for (int l = 0; l < L; ++l) {
    Level& V = lev[l];
    if (l == 0) {
      V.n = n0;
      V.h = P->h;
    } else {
      const Level& F = lev[l - 1];
      V.n = Dims{F.n.nx / F.f[0], F.n.ny / F.f[1], F.n.nz / F.f[2]};
      V.h = 2.0 * F.h;
    }
    V.h0 = P->h;
    for (int dd = 0; dd < 3; ++dd) V.f[dd] = act[dd] ? 2 : 1;
  }
  // The levels of the single-workgroup tail keep their face coefficients and
  // 1/D in one contiguous pack per precision, laid out as the tail kernel's
  // LDS image (bx, by, bz, 1/D per level, each padded to 4 elements), so the
  // kernel stages them with one flat copy.
  size_t lds64 = 0, lds32 = 0;
  const int t64 = plan_tail(lev, L, sizeof(double), &lds64);
  const int t32 = plan_tail(lev, L, sizeof(float), &lds32);
  const size_t np64 = tail_pack_elems(lev, L, t64), np32 = tail_pack_elems(lev, L, t32);
  double* pk64 = cv.take<double>(np64);
  float* pk32 = cv.take<float>(np32);
  size_t o64 = 0, o32 = 0;
  auto from64 = [&](size_t n) {
    double* p = pk64 ? pk64 + o64 : nullptr;
    o64 += pad4(n);
    return p;
  };
  auto from32 = [&](size_t n) {
    float* p = pk32 ? pk32 + o32 : nullptr;
    o32 += pad4(n);
    return p;
  };
  for (int l = 0; l < L; ++l) {
    Level& V = lev[l];
    const size_t c = (size_t)V.n.nx * V.n.ny * V.n.nz;
    const size_t fu = (size_t)(V.n.nx + 1) * V.n.ny * V.n.nz;
    const size_t fv = (size_t)V.n.nx * (V.n.ny + 1) * V.n.nz;
    const size_t fw = (size_t)V.n.nx * V.n.ny * (V.n.nz + 1);
    const size_t c2 = 2 * (size_t)((V.n.nx + 1) / 2) * V.n.ny * V.n.nz;   // colour-split size
    if (l >= t32) {
      V.bxf = from32(fu);
      V.byf = from32(fv);
      V.bzf = from32(fw);
      V.invdf = from32(c);
    } else {
      V.bxf = cv.take<float>(fu);
      V.byf = cv.take<float>(fv);
      V.bzf = cv.take<float>(fw);
      V.invdf = cv.take<float>(c2);
    }
    if (l >= t64) {
      V.bx = from64(fu);
      V.by = from64(fv);
      V.bz = from64(fw);
      V.invd = from64(c);
    } else {
      V.bx = cv.take<double>(fu);
      V.by = cv.take<double>(fv);
      V.bz = cv.take<double>(fw);
      V.invd = cv.take<double>(c2);
    }
    // the line tables of the finest and the first coarse level's face
    // arrays (one entry per x-line)
    V.tx = V.ty = V.tz = nullptr;
    V.txf = V.tyf = V.tzf = nullptr;
    V.tab_ok = V.tabf_ok = false;
    if (l <= 1) {
      const size_t lx = (size_t)V.n.ny * V.n.nz, ly = (size_t)(V.n.ny + 1) * V.n.nz;
      const size_t lz = (size_t)V.n.ny * (V.n.nz + 1);
      V.tx = cv.take<double>(lx);
      V.ty = cv.take<double>(ly);
      V.tz = cv.take<double>(lz);
      V.txf = cv.take<float>(lx);
      V.tyf = cv.take<float>(ly);
      V.tzf = cv.take<float>(lz);
    }
    // b and e: colour-split (2 ceil(nx/2) ny nz entries) above the tail,
    // natural on tail levels; level 0 keeps its own split pair (its natural
    // b and e are the CG vectors, and for FP32 the bfn/efn interface).  A
    // coarse split level's e has a third plane, the black plane's copy that
    // its fused red-black passes read.
    const size_t cs = 2 * (size_t)((V.n.nx + 1) / 2) * V.n.ny * V.n.nz;
    // a third plane for the black plane's copy that a fused red-black pass
    // reads: on the coarse levels, and on the finest where its fused sweep applies
    const size_t ces = (l >= 1 || gs_rb_fine_fits(V.n)) ? cs + cs / 2 : cs;
    V.bf = cv.take<float>(l < t32 ? cs : c);
    V.ef = cv.take<float>(l < t32 ? ces : c);
    V.bfn = V.efn = nullptr;
    if (l == 0) {
      V.bfn = t32 > 0 ? cv.take<float>(c) : V.bf;
      V.efn = t32 > 0 ? cv.take<float>(c) : V.ef;
    }
    if (l == 0 && t64 == 0) {
      V.b = V.e = nullptr;   // a tail-only hierarchy works on the CG vectors directly
    } else {
      V.b = cv.take<double>(l < t64 ? cs : c);
      V.e = cv.take<double>(l < t64 ? ces : c);
    }
  }
  if (X) {
    X->nc = nc;
    X->nu = nu;
    X->nv = nv;
    X->nw = nw;
    X->us = us;
    X->vs = vs;
    X->ws = ws;
    X->sig_a = sa;
    X->sig_b = sb;
    X->rho = rho;
    X->rfl = rfl;
    X->mu = mu;
    X->rho_prev = rho_prev;
    for (int c = 0; c < 3; ++c) {
      X->cn_rhs[c] = cn[c];
      X->cn_diag[c] = cn[3 + c];
      X->cn_tmp[c] = cn[6 + c];
    }
    X->cnpart = cnpart;
    X->chi = chi;
    X->b = b;
    X->r = r;
    X->z = z;
    X->zn = zn;
    X->d = d;
    X->d2 = d2;
    X->q = q;
    X->partials = part;
    X->scal = scal;
    X->phys.waves = waves;
    X->nparts = nparts;
    X->L = L;
    for (int l = 0; l < L; ++l) X->lev[l] = lev[l];
    X->tail64 = t64;
    X->tail32 = t32;
    X->lds64 = lds64;
    X->lds32 = lds32;
    X->pack64 = pk64;
    X->pack32 = pk32;
    X->npack64 = np64;
    X->npack32 = np32;
  }
  return cv.off + kAlign;
}

Phys make_phys(const ns_params& P) {
  Phys ph{};
  ph.n = Dims{P.nx, P.ny, P.nz};
  ph.h = P.h;
  ph.rho_w = P.rho_w;
  ph.mu_w = P.mu_w;
  ph.rho_a = P.rho_a;
  ph.mu_a = P.mu_a;
  ph.rho_s = P.rho_s;
  ph.mu_s = P.mu_s;
  ph.g = P.g;
  ph.eps = P.n_cells * P.h;
  ph.inv_kp = P.inv_kappa_p;
  ph.pen_w = P.proj_penalty_weight;
  ph.nb = P.n_bodies;
  ph.depth = P.depth;
  ph.gen_len = P.gen_len;
  ph.damp_len = P.damp_len;
  ph.vort_w = P.vort_width;
  ph.nwave = P.n_waves;
  ph.waves = nullptr;   // set when the workspace is carved
  for (int m = 0; m < P.n_bodies; ++m) {
    const ns_body& B = P.body[m];
    ph.body[m] = BodyK{B.kind,          B.c[0],          B.c[1],      B.c[2],  B.half[0],
                       B.half[1],       B.half[2],       B.heave_amp, B.heave_omega,
                       B.heave_phase,   B.free_heave,    B.zeta0,     B.zdot0};
  }
  return ph;
}

// ------------------------------------------------------------------ V-cycle
template <typename T>
struct LV;
template <>
struct LV<double> {
  static double* bx(const Level& L) { return L.bx; }
  static double* by(const Level& L) { return L.by; }
  static double* bz(const Level& L) { return L.bz; }
  static double* b(const Level& L) { return L.b; }
  static double* e(const Level& L) { return L.e; }
  static double* invd(const Level& L) { return L.invd; }
};
template <>
struct LV<float> {
  static float* bx(const Level& L) { return L.bxf; }
  static float* by(const Level& L) { return L.byf; }
  static float* bz(const Level& L) { return L.bzf; }
  static float* b(const Level& L) { return L.bf; }
  static float* e(const Level& L) { return L.ef; }
  static float* invd(const Level& L) { return L.invdf; }
};

template <typename T>
int tail_start(const ns_ctx* X) {
  return sizeof(T) == 8 ? X->tail64 : X->tail32;
}
template <typename T>
size_t tail_bytes(const ns_ctx* X) {
  return sizeof(T) == 8 ? X->lds64 : X->lds32;
}

// coarse coefficients of every level from level 0, and 1/D of every level
// (the tail stages it), in precision T: one launch per level
template <typename T>
void build_hierarchy(ns_ctx* X) {
  const Level& V0 = X->lev[0];
  launch_invdiag<T>(V0, LV<T>::bx(V0), LV<T>::by(V0), LV<T>::bz(V0), LV<T>::invd(V0), 0 < tail_start<T>(X), X->st);
  for (int l = 1; l < X->L; ++l) {
    const Level& F = X->lev[l - 1];
    const Level& C = X->lev[l];
    launch_coarsen_level<T>(F, LV<T>::bx(F), LV<T>::by(F), LV<T>::bz(F), C, LV<T>::bx(C), LV<T>::by(C),
                            LV<T>::bz(C), LV<T>::invd(C), l < tail_start<T>(X), X->st);
  }
  // the first coarse level's line tables, in the cycle's precision, where
  // its passes run outside the tail and it is large enough for them to pay
  if (X->face_tabs && X->L > 1 && 1 < tail_start<T>(X) && face_tables_pay(X->lev[1].n)) {
    Level& V1 = X->lev[1];
    if constexpr (sizeof(T) == 8) {
      launch_face_tables<double>(V1.n, V1.bx, V1.by, V1.bz, V1.tx, V1.ty, V1.tz, X->st);
      V1.tab_ok = true;
    } else {
      launch_face_tables<float>(V1.n, V1.bxf, V1.byf, V1.bzf, V1.txf, V1.tyf, V1.tzf, X->st);
      V1.tabf_ok = true;
    }
  }
}

template <typename T>
void launch_tail(ns_ctx* X, int l0, const T* b, T* e, size_t bytes) {
  TailDesc<T> D{};
  D.nl = X->L - l0;
  D.nu_pre = X->P.nu_pre;
  D.nu_post = X->P.nu_post;
  D.coarse_sweeps = X->P.coarse_sweeps;
  // LDS image: the pack (bx, by, bz, 1/D per level) then b, e per level
  int off = 0;
  auto take = [&](size_t n) {
    const int o = off;
    off += (int)pad4(n);
    return o;
  };
  for (int q = 0; q < D.nl; ++q) {
    const Level& V = X->lev[l0 + q];
    const Dims n = V.n;
    D.n[q] = n;
    for (int d = 0; d < 3; ++d) D.f[q][d] = V.f[d];
    D.h2[q] = (T)(V.h * V.h);
    D.obx[q] = take((size_t)(n.nx + 1) * n.ny * n.nz);
    D.oby[q] = take((size_t)n.nx * (n.ny + 1) * n.nz);
    D.obz[q] = take((size_t)n.nx * n.ny * (n.nz + 1));
    D.oid[q] = take((size_t)n.nx * n.ny * n.nz);
  }
  D.npack = off;
  for (int q = 0; q < D.nl; ++q) {
    const size_t mc = (size_t)D.n[q].nx * D.n[q].ny * D.n[q].nz;
    D.ob[q] = take(mc);
    D.oe[q] = take(mc);
  }
  D.ors = D.nl > 1 ? take((size_t)D.n[0].nx * D.n[0].ny * D.n[0].nz) : 0;
  D.pack = LV<T>::bx(X->lev[l0]);   // the pack starts with the first tail level's bx
  D.b0 = b;
  D.ge = e;
  launch_vcycle_tail<T>(D, bytes, X->st);
}

// e_l = V(l, b_l); level 0 takes b0 and returns e0 in natural order.  Levels
// above the tail work on colour-split b and e; the first sweep of level 0
// reads b0 in natural order and writes its split copy, and the last red pass
// of level 0 writes e0 in natural order.
// The flexible CG's next two products (r z, r z_old) requested of an FP64
// V-cycle: its last kernel computes them when it is the finest level's last
// red pass (nparts: the partials it left; 0 when the cycle had no such pass).
struct DotsReq {
  const double* r;
  const double* zold;
  double* z;     // the cycle's FP64 result, natural order
  int nparts;
};

// b0d: an FP32 cycle's finest-level right-hand side in FP64 (natural), read
// by its first kernel in place of b0 (the levels below the finest, the
// tail, and a cycle without pre-smoothing read b0)
template <typename T>
void vcycle(ns_ctx* X, int l, const T* b0, T* e0, DotsReq* dq = nullptr, const double* b0d = nullptr) {
  const ns_params& P = X->P;
  const Level& L = X->lev[l];
  hipStream_t st = X->st;
  if (l == tail_start<T>(X)) {
    launch_tail<T>(X, l, l == 0 ? b0 : LV<T>::b(L), l == 0 ? e0 : LV<T>::e(L), tail_bytes<T>(X));
    return;
  }
  T* b = LV<T>::b(L);   // split
  T* e = LV<T>::e(L);   // split
  const T *bx = LV<T>::bx(L), *by = LV<T>::by(L), *bz = LV<T>::bz(L);
  KTimer* kt = (l == 0 && X->timed_kernel == NS_TIME_SMOOTH0) ? &X->kt : nullptr;
  const size_t nsplit = 2 * (size_t)((L.n.nx + 1) / 2) * L.n.ny * L.n.nz;
  // the red pass that writes the cycle's result (level 0): with the
  // products fused, into the FP64 z, when they are requested (no kernel
  // timer on it), else into e0
  auto last_red = [&]() {
    if (dq && !kt) {
      dq->nparts = launch_gs_last_dots<T>(L, bx, by, bz, b, e, dq->z, dq->r, dq->zold, X->partials, st);
      return;
    }
    launch_gs<T>(L, bx, by, bz, b, e, 0, st, kt, e0);
  };
  // the first pre-smoothing kernel (red from zero + black); red_out false
  // where a red pass follows it, which overwrites the red values unread
  auto first = [&](T* bcopy, bool red_out) {
    if constexpr (sizeof(T) == 4) {
      if (l == 0 && b0d) {
        launch_gs_first_nat64(L, bx, by, bz, b0d, LV<T>::invd(L), e, b, st, bcopy, red_out);
        return;
      }
    }
    launch_gs_first<T>(L, bx, by, bz, l == 0 ? b0 : b, l == 0, LV<T>::invd(L), e, b, st, bcopy, red_out);
  };
  if (l == X->L - 1) {
    // a coarsest level too large for the tail: its sweeps with the
    // multi-block kernels, forward (red, black) then backward (black, red)
    // from zero; at level 0 the last red pass writes e0
    const int S = P.coarse_sweeps;
    if (S == 0) {
      if (l == 0)
        launch_fill<T>(e0, (size_t)L.n.nx * L.n.ny * L.n.nz, st);
      else
        launch_fill<T>(e, nsplit, st);
      return;
    }
    first(nullptr, S < 2);   // a second forward sweep starts with a red pass
    for (int s = 1; s < S; ++s) {
      launch_gs<T>(L, bx, by, bz, b, e, 0, st, kt);
      launch_gs<T>(L, bx, by, bz, b, e, 1, st, kt);
    }
    for (int s = 0; s < S; ++s) {
      launch_gs<T>(L, bx, by, bz, b, e, 1, st, kt);
      if (l == 0 && s == S - 1)
        last_red();
      else
        launch_gs<T>(L, bx, by, bz, b, e, 0, st, kt);
    }
    return;
  }
  // On a coarse level whose rows fit one tile, the first (red, black) pair
  // after a kernel that leaves the black plane's copy is one fused launch;
  // on the finest level the same pair is the fused sweep that reads each
  // face coefficient once.
  const bool fine = l == 0 && X->fine_rb;
  const bool rb = (l >= 1 && gs_rb_fits(L.n)) || fine;
  T* ecopy = rb ? e + nsplit : nullptr;
  auto fused = [&]() {
    if (fine)
      launch_gs_rb_fine<T>(L, bx, by, bz, b, e, ecopy, st, kt);
    else
      launch_gs_rb<T>(L, bx, by, bz, b, e, ecopy, st);
  };
  // with the fused sweep on the finest level, the timer follows it
  KTimer* kgs = fine ? nullptr : kt;
  // pre-smoothing: (red from zero + black) fused, then red, black pairs
  if (P.nu_pre > 0) {
    const bool rb_pre = rb && P.nu_pre >= 2;
    first(rb_pre ? ecopy : nullptr, P.nu_pre < 2);   // a second sweep starts with a red pass
    int s = 1;
    if (rb_pre) {
      fused();
      s = 2;
    }
    for (; s < P.nu_pre; ++s) {
      launch_gs<T>(L, bx, by, bz, b, e, 0, st, kgs);
      launch_gs<T>(L, bx, by, bz, b, e, 1, st, kgs);
    }
  } else {
    if (l == 0) launch_split_copy<T>(L, b0, b, true, st);
    launch_fill<T>(e, nsplit, st);
  }
  const Level& C = X->lev[l + 1];
  const bool csplit = (l + 1) < tail_start<T>(X);
  launch_resid_restrict<T>(L, bx, by, bz, b, e, C, LV<T>::b(C), csplit, st);
  vcycle<T>(X, l + 1, nullptr, nullptr);
  // post-smoothing: (prolongation + black) fused, then red, then black, red
  // pairs; at level 0 the last red pass writes e0
  if (P.nu_post > 0 && rb && P.nu_post >= 2) {
    // (prolongation + black), then (red, black) fused, then red, black
    // pairs and the last red (at level 0 writing e0)
    launch_gs_prolong<T>(L, bx, by, bz, b, e, C, LV<T>::e(C), csplit, st, ecopy);
    fused();
    for (int s = 2; s < P.nu_post; ++s) {
      launch_gs<T>(L, bx, by, bz, b, e, 0, st, kgs);
      launch_gs<T>(L, bx, by, bz, b, e, 1, st, kgs);
    }
    if (l == 0)
      last_red();
    else
      launch_gs<T>(L, bx, by, bz, b, e, 0, st, kgs);
  } else if (P.nu_post > 0) {
    launch_gs_prolong<T>(L, bx, by, bz, b, e, C, LV<T>::e(C), csplit, st);
    if (l == 0 && P.nu_post == 1)
      last_red();
    else
      launch_gs<T>(L, bx, by, bz, b, e, 0, st, kgs);
    for (int s = 1; s < P.nu_post; ++s) {
      launch_gs<T>(L, bx, by, bz, b, e, 1, st, kgs);
      if (l == 0 && s == P.nu_post - 1)
        last_red();
      else
        launch_gs<T>(L, bx, by, bz, b, e, 0, st, kgs);
    }
  } else {
    launch_prolong<T>(L, e, C, LV<T>::e(C), csplit, st);
    if (l == 0) launch_split_copy<T>(L, e, e0, false, st);
  }
}

// z = M r, one kernel launch at a time on the context's stream.  With zold
// the cycle's last kernel also leaves the partials of r z and r z_old in
// X->partials when it can; returns how many (0: not fused, or not asked).
int precond_launch(ns_ctx* X, const double* r, double* z, const double* zold = nullptr) {
  DotsReq dq{r, zold, z, 0};
  if (X->P.prec == NS_PREC_FP64) {
    vcycle<double>(X, 0, r, z, zold ? &dq : nullptr);
    return dq.nparts;
  }
  // FP32 cycle: its first kernel reads r itself, rounding it to FP32, where
  // the finest level is above the tail and pre-smooths; its last kernel
  // writes z in FP64 with the products when it can
  Level& L0 = X->lev[0];
  const bool direct = tail_start<float>(X) > 0 && X->P.nu_pre > 0;
  if (!direct) launch_d2f(r, L0.bfn, X->nc, X->st);
  vcycle<float>(X, 0, L0.bfn, L0.efn, zold ? &dq : nullptr, direct ? r : nullptr);
  if (dq.nparts > 0) return dq.nparts;
  if (zold) return launch_f2d_dots(L0.efn, z, X->nc, r, zold, X->partials, X->st);
  launch_f2d(L0.efn, z, X->nc, X->st);
  return 0;
}

// The CG loop's V-cycles, each with the dot product that follows it, are
// issued as segments. In graph mode a segment is recorded once per context
// and key (kind, the vectors it works on, a flag) and replayed with one
// hipGraphLaunch: one host call instead of some thirty kernel launches, for
// a fixed device-side cost per graph launch of a few microseconds. Recording
// runs nothing, on the context's capture-only stream, and every other
// argument is fixed for the context's life. In stream mode, or while a kernel
// is being timed, the segment's kernels are launched one by one. `launch`
// issues them on X->st.
enum SegKind { SEG_PRECOND_RHO = 1, SEG_PRECOND_BETA = 2 };

template <class F>
ns_status issue(ns_ctx* X, int kind, const void* a, const void* b, const void* c, int flag, F&& launch) {
  if (X->launch_mode == NS_LAUNCH_GRAPH && X->timed_kernel < 0) {
    for (int q = 0; q < X->ngs; ++q) {
      const auto& g = X->gs[q];
      if (g.kind == kind && g.a == a && g.b == b && g.c == c && g.flag == flag) {
        HIPCHK(X, hipGraphLaunch(g.exec, X->st));
        return NS_OK;
      }
    }
    if (X->ngs < (int)(sizeof(X->gs) / sizeof(X->gs[0]))) {
      hipStream_t run = X->st;
      X->st = X->cap_st;
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipStreamBeginCapture(X->cap_st, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        launch();
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(X->cap_st, &g);
        if (e == hipSuccess) {
          e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
        }
      }
      X->st = run;
      if (e == hipSuccess) {
        X->gs[X->ngs++] = {kind, a, b, c, flag, exec};
        HIPCHK(X, hipGraphLaunch(exec, X->st));
        return NS_OK;
      }
      // Recording failed (nothing recorded ran): this context launches one
      // by one from now on, with bitwise the same results.
      (void)hipGetLastError();
      X->launch_mode = NS_LAUNCH_STREAM;
    }
  }
  launch();
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

// The finest level's line tables, built from its face arrays as they are now
// (a solve's kernels then take uniform lines from them), or left invalid
// when switched off.  Whatever writes the face arrays marks them invalid.
void build_face_tables(ns_ctx* X) {
  Level& L0 = X->lev[0];
  L0.tab_ok = L0.tabf_ok = false;
  if (X->L > 1) X->lev[1].tab_ok = X->lev[1].tabf_ok = false;   // built again after coarsening
  if (!X->face_tabs) return;
  launch_face_tables<double>(L0.n, L0.bx, L0.by, L0.bz, L0.tx, L0.ty, L0.tz, X->st);
  L0.tab_ok = true;
  if (X->P.prec != NS_PREC_FP64) {
    launch_face_tables<float>(L0.n, L0.bxf, L0.byf, L0.bzf, L0.txf, L0.tyf, L0.tzf, X->st);
    L0.tabf_ok = true;
  }
}

void prepare_hierarchy(ns_ctx* X) {
  build_face_tables(X);
  if (X->P.prec == NS_PREC_FP64)
    build_hierarchy<double>(X);
  else
    build_hierarchy<float>(X);
}

// Totals of a reduction the host reads: summed here, in block order, from the
// host partials when the grid is small enough to have them, else as the
// finalize kernel stored them to the mirror. q selects the value (0 or 1) of
// an nv-valued reduction; mirror_slot is its S_* index.
double host_total(const ns_ctx* X, int nv, int q, int mirror_slot) {
  if (!X->hpart) return X->host[mirror_slot];
  double s = 0.0;
  for (int b = 0; b < X->nparts; ++b) s += X->hpart[(size_t)nv * b + q];
  return s;
}

// wait until the work queued so far has stored its scalars to the host mirror
ns_status wait_host(ns_ctx* X) {
  HIPCHK(X, hipEventRecord(X->ev_rr, X->st));
  HIPCHK(X, hipEventSynchronize(X->ev_rr));
  return NS_OK;
}

ns_status read_scal(ns_ctx* X) {
  HIPCHK(X, hipMemcpyAsync(X->host, X->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, X->st));
  HIPCHK(X, hipStreamSynchronize(X->st));
  return NS_OK;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// flexible PCG on A p = b with x = fields.p as the initial guess.
//
// The host reads ||r||^2 once per iteration. While it waits, the device is
// kept busy with the next preconditioner application, which is unused when
// the test passes. It is not queued when the last two residuals predict
// that this iteration comes within a factor ten of the tolerance: skipping
// it wrongly costs the device one host round trip (tens of microseconds),
// queueing it wrongly a whole V-cycle, which a prediction at the tolerance
// itself did in most solves. A residual that meets the tolerance is
// confirmed on the true residual b - A x, which is then also the reported
// one.
ns_status pcg(ns_ctx* X, ns_stats* stats) {
  const ns_params& P = X->P;
  const Dims n = X->lev[0].n;
  const double h = P.h;
  const Level& L0 = X->lev[0];
  hipStream_t st = X->st;
  double* x = X->F.p;
  const CgScratch cs{X->partials, X->scal, X->host_dev, X->hpart_dev};
  ns_stats S{};
  double* z = X->z;
  double* zn = X->zn;
  double* d = X->d;
  double* dn = X->d2;
  // segments: z = M r then rho = <r, z>; zn = M r then beta and rho;
  // then d = z + beta d, q = A d, alpha, x += alpha d, r -= alpha q, ||r||^2
  auto precond_rho = [&](double* zz) {
    return issue(X, SEG_PRECOND_RHO, zz, nullptr, nullptr, 0, [&] {
      precond_launch(X, X->r, zz);
      launch_dot_rho(n, X->r, zz, cs, X->st);
    });
  };
  auto precond_beta = [&](double* znew, const double* zold) {
    return issue(X, SEG_PRECOND_BETA, znew, zold, nullptr, 0, [&] {
      // the products come with the cycle's last kernel when it can give them
      const int np = precond_launch(X, X->r, znew, zold);
      if (np > 0)
        launch_finalize_beta(cs, np, X->st);
      else
        launch_dots_beta(n, X->r, znew, zold, cs, X->st);
    });
  };
  // (four kernels: launched directly, a graph launch would cost the device
  // more than it saves the host).  x += alpha d is applied one iteration
  // late, by the next direction update, which reads d anyway: the vector
  // update then reads and writes only r (8 bytes per cell less per
  // iteration, the same arithmetic).  xpend: x lacks the latest alpha d;
  // sync_x applies it before anything reads x.
  bool xpend = false;
  auto dir_update = [&](const double* zz, const double* dold, double* dnew, int first) {
    launch_dir_spmv(n, h, L0.bx, L0.by, L0.bz, zz, dold, dnew, X->q, first, cs, X->st,
                    X->timed_kernel == NS_TIME_SPMV ? &X->kt : nullptr, xpend ? x : nullptr, face_tab(L0, L0.bx));
    launch_cg_update(n, X->q, X->r, cs, X->st);
    xpend = true;
    HIPCHK(X, hipGetLastError());
    return NS_OK;
  };
  auto sync_x = [&](const double* dcur) {
    if (xpend) launch_x_update(n, dcur, x, cs, X->st);
    xpend = false;
  };
  prepare_hierarchy(X);
  launch_resid_norm(n, h, L0.bx, L0.by, L0.bz, X->b, x, X->r, cs, FIN_RESID0, st, face_tab(L0, L0.bx));
  HIPCHK(X, hipEventRecord(X->ev_rr, st));
  // first direction d = z = M r, rho = <r, z>, queued before the host has
  // seen ||b|| and ||r||; unused if b = 0 or the guess already converges
  ns_status s = precond_rho(z);
  if (s != NS_OK) return s;
  HIPCHK(X, hipEventSynchronize(X->ev_rr));
  if (X->host[S_FLAGS] != 0.0)
    return fail(X, NS_EUNSTABLE, "a carried face density came out <= 0: the step's outflow Courant number is "
                "above the limited transport's bound of 1/2 (take dt from the CFL rule)");
  const double bb = host_total(X, 2, 1, S_BB);
  double rr = host_total(X, 2, 0, S_RR);
  if (!std::isfinite(bb) || !std::isfinite(rr)) return fail(X, NS_ENAN, "non-finite right-hand side or guess");
  if (bb == 0.0) {
    launch_fill<double>(x, X->nc, st);
    S.converged = 1;
    if (stats) *stats = S;
    return NS_OK;
  }
  const double bnorm = std::sqrt(bb);
  const double tol2 = P.rtol * P.rtol * bb;
  S.rel_resid0 = S.rel_resid = std::sqrt(rr) / bnorm;
  bool conv = rr <= tol2;
  double true_rr = rr;   // ||b - A x||^2 of the latest confirmed test
  double rr_prev = 0.0;  // ||r||^2 one iteration back (0: none since the last (re)start)
  int it = 0;
  bool first = true;
  while (!conv && it < P.max_iters) {
    // d = z + beta d (or z), q = A d, alpha = rho / <d, q>, then x and r
    if ((s = dir_update(z, d, dn, first ? 1 : 0)) != NS_OK) return s;
    std::swap(d, dn);
    first = false;
    ++it;
    HIPCHK(X, hipEventRecord(X->ev_rr, st));
    // the residual this iteration is expected to reach, at the rate of the
    // last one, against 10x the tolerance (100x in the squares)
    const bool likely_done = rr_prev > 0.0 && rr * (rr / rr_prev) <= 100.0 * tol2;
    const bool ahead = it < P.max_iters && !likely_done;
    if (ahead && (s = precond_beta(zn, z)) != NS_OK) return s;
    HIPCHK(X, hipEventSynchronize(X->ev_rr));
    rr_prev = rr;
    rr = host_total(X, 1, 0, S_RR);
    if (!std::isfinite(rr)) {
      S.iters = it;
      if (stats) *stats = S;
      return fail(X, NS_ENAN, "non-finite residual at CG iteration %d", it);
    }
    S.rel_resid = std::sqrt(rr) / bnorm;
    if (rr <= tol2) {
      // confirm on the true residual; restart from it when it fails
      sync_x(d);
      launch_resid_norm(n, h, L0.bx, L0.by, L0.bz, X->b, x, X->r, cs, FIN_RESID0, st, face_tab(L0, L0.bx));
      if ((s = wait_host(X)) != NS_OK) return s;
      rr = true_rr = host_total(X, 2, 0, S_RR);
      S.rel_resid = std::sqrt(rr) / bnorm;
      if (rr <= tol2) {
        conv = true;
        break;
      }
      if (it >= P.max_iters) break;
      if ((s = precond_rho(z)) != NS_OK) return s;
      first = true;
      rr_prev = 0.0;
      continue;
    }
    if (it >= P.max_iters) break;
    if (!ahead && (s = precond_beta(zn, z)) != NS_OK) return s;
    std::swap(z, zn);
  }
  sync_x(d);
  if (!conv) {
    // true residual at exit (into q, leaving r as the recursion left it)
    launch_resid_norm(n, h, L0.bx, L0.by, L0.bz, X->b, x, X->q, cs, FIN_TRR, st, face_tab(L0, L0.bx));
    if ((s = wait_host(X)) != NS_OK) return s;
    true_rr = host_total(X, 2, 0, S_TRR);
  }
  S.iters = it;
  S.true_rel_resid = std::sqrt(true_rr) / bnorm;
  S.converged = S.true_rel_resid <= P.rtol ? 1 : 0;
  if (stats) *stats = S;
  if (!std::isfinite(S.true_rel_resid)) return fail(X, NS_ENAN, "non-finite final residual");
  if (!conv) return fail(X, NS_ENOCONV, "CG reached max_iters=%d at rel resid %.3e", P.max_iters, S.rel_resid);
  return NS_OK;
}


bool aligned8(const void* p) { return p && ((uintptr_t)p & 7) == 0; }

}  // namespace

extern "C" {

int ns_num_levels(int nx, int ny, int nz) { return count_levels(nx, ny, nz); }

ns_status ns_attach_net(ns_ctx* X, ns_net* N) {
  if (!X) return NS_EINVAL;
  if (N && !net_matches(N, X->lev[0].n)) return fail(X, NS_EINVAL, "network grid differs from the solver grid");
  X->net = N;
  return NS_OK;
}

ns_status ns_features(ns_ctx* X, double dt, const double* p_prev, float* feat4) {
  if (!X) return NS_EINVAL;
  if (!aligned8(p_prev) || !feat4) return fail(X, NS_EINVAL, "p_prev and feat4 must be device pointers");
  if (!(dt > 0.0)) return fail(X, NS_EINVAL, "dt must be > 0");
  if (!X->have_beta) return fail(X, NS_ESTATE, "ns_features before momentum_step");
  if (!(X->P.p_scale > 0.0)) return fail(X, NS_EINVAL, "p_scale must be > 0");
  const Level& L0 = X->lev[0];
  launch_rhs(X->phys, X->us, X->vs, X->ws, dt, X->b, X->st);
  launch_apply_A(L0.n, X->P.h, L0.bx, L0.by, L0.bz, p_prev, X->q, X->st);
  net_features(nullptr, L0.n, X->P.h, X->P.rho_w, X->P.rho_a, X->P.p_scale, X->b, X->rho, p_prev, X->q, feat4,
               X->st);
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

ns_status ns_target(ns_ctx* X, const double* p_prev, float* t) {
  if (!X) return NS_EINVAL;
  if (!aligned8(p_prev) || !t) return fail(X, NS_EINVAL, "p_prev and t must be device pointers");
  if (!(X->P.p_scale > 0.0)) return fail(X, NS_EINVAL, "p_scale must be > 0");
  net_target((long)X->nc, X->F.p, p_prev, X->P.p_scale, t, X->st);
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

size_t ns_workspace_bytes(const ns_params* params) {
  char why[256];
  if (!valid_params(params, why, sizeof(why))) return 0;
  return carve(params, nullptr, nullptr);
}

ns_status ns_init(const ns_params* params, ns_fields fields, void* workspace, size_t ws_bytes,
                  void* hip_stream, ns_ctx** out) {
  if (!out) return NS_EINVAL;
  *out = nullptr;
  ns_ctx* X = new (std::nothrow) ns_ctx();
  if (!X) return NS_EINVAL;
  char why[256];
  if (!valid_params(params, why, sizeof(why))) {
    delete X;
    return NS_EINVAL;
  }
  if (!aligned8(fields.sigma) || !aligned8(fields.u) || !aligned8(fields.v) || !aligned8(fields.w) ||
      !aligned8(fields.p) || !workspace || ((uintptr_t)workspace % kAlign) != 0) {
    delete X;
    return NS_EINVAL;
  }
  const size_t need = carve(params, nullptr, nullptr);
  if (ws_bytes < need) {
    delete X;
    return NS_EINVAL;
  }
  X->P = *params;
  X->F = fields;
  X->st = (hipStream_t)hip_stream;
  X->phys = make_phys(*params);
  carve(params, X, (char*)workspace);
  if (params->n_waves > 0 &&
      (hipMemcpyAsync(const_cast<double*>(X->phys.waves), params->waves, sizeof(double) * 4 * params->n_waves,
                      hipMemcpyHostToDevice, X->st) != hipSuccess ||
       hipStreamSynchronize(X->st) != hipSuccess)) {
    delete X;
    return NS_EHIP;
  }
  // From here on a failure releases what was acquired through ns_destroy,
  // which accepts a partly built context (its fields start null).
  // Coherent and mapped: the reduction kernels store the values the host
  // tests straight into it, so reading them needs no copy
  if (hipHostMalloc((void**)&X->host, S_COUNT * sizeof(double), hipHostMallocCoherent | hipHostMallocMapped) !=
      hipSuccess) {
    delete X;
    return NS_EHIP;
  }
  if (hipHostGetDevicePointer((void**)&X->host_dev, X->host, 0) != hipSuccess) {
    ns_destroy(X);
    return NS_EHIP;
  }
  for (int q = 0; q < S_COUNT; ++q) X->host[q] = 0.0;
  // small grids: the reductions the host alone reads leave their per-block
  // partials in host memory, and the host sums them (no finalize launch)
  X->fpart = nullptr;
  X->hpart = X->hpart_dev = nullptr;
  if (X->nparts <= kHostPartsMax) {
    if (hipHostMalloc((void**)&X->hpart, (size_t)2 * X->nparts * sizeof(double),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&X->hpart_dev, X->hpart, 0) != hipSuccess) {
      ns_destroy(X);
      return NS_EHIP;
    }
  }
  // free bodies: heave state, and pinned host room for the force partials;
  // a force launch writes three partials per block into the device partials
  // (4 nparts doubles), so it may use at most 4 nparts / 3 blocks, which a
  // body's box within the grid does not exceed (a bigger one is refused)
  X->have_rho_n = false;
  X->nfree = 0;
  for (int m = 0; m < params->n_bodies; ++m) X->nfree += params->body[m].free_heave ? 1 : 0;
  for (int m = 0; m < 4; ++m) X->bs[m] = {{0.0, 0.0, 0.0}, 0.0};
  X->force_ready = false;
  X->t_props = 0.0;
  X->fcap = (4 * X->nparts) / 3;
  if (X->nfree > 0 &&
      hipHostMalloc((void**)&X->fpart, (size_t)3 * 4 * X->fcap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    ns_destroy(X);
    return NS_EHIP;
  }
  if (hipEventCreateWithFlags(&X->ev_rr, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&X->ax.ev[0]) != hipSuccess || hipEventCreate(&X->ax.ev[1]) != hipSuccess) {
    ns_destroy(X);
    return NS_EHIP;
  }
  if (hipStreamCreateWithFlags(&X->cap_st, hipStreamNonBlocking) != hipSuccess) {
    ns_destroy(X);
    return NS_EHIP;
  }
  X->launch_mode = NS_LAUNCH_GRAPH;
  X->face_tabs = face_tables_pay(X->lev[0].n);
  X->fine_rb = gs_rb_fine_pays(X->lev[0].n, X->P.prec == NS_PREC_FP64, X->face_tabs);
  X->ngs = 0;
  X->have_beta = false;
  X->timed_kernel = -1;
  X->kt = KTimer{nullptr, 0, 0};
  launch_fill<double>(X->scal, S_COUNT, X->st);
  *out = X;
  return NS_OK;
}

static void free_timer(ns_ctx* X) {
  if (X->kt.ev) {
    for (int q = 0; q < 2 * X->kt.cap; ++q) (void)hipEventDestroy(X->kt.ev[q]);
    delete[] X->kt.ev;
  }
  X->kt = KTimer{nullptr, 0, 0};
  X->timed_kernel = -1;
}

void ns_destroy(ns_ctx* X) {
  if (!X) return;
  free_timer(X);
  for (int q = 0; q < X->ngs; ++q) (void)hipGraphExecDestroy(X->gs[q].exec);
  if (X->cap_st) (void)hipStreamDestroy(X->cap_st);
  if (X->ev_rr) (void)hipEventDestroy(X->ev_rr);
  for (int q = 0; q < 2; ++q)
    if (X->ax.ev[q]) (void)hipEventDestroy(X->ax.ev[q]);
  for (int q = 0; q < 6; ++q)
    if (X->ph_ev[q]) (void)hipEventDestroy(X->ph_ev[q]);
  if (X->host) (void)hipHostFree(X->host);
  if (X->hpart) (void)hipHostFree(X->hpart);
  if (X->fpart) (void)hipHostFree(X->fpart);
  delete X;
}

ns_status ns_phase_timing(ns_ctx* X, int on) {
  if (!X) return NS_EINVAL;
  if (on && !X->ph_ev[0])
    for (int q = 0; q < 6; ++q) HIPCHK(X, hipEventCreate(&X->ph_ev[q]));
  X->phase_on = on != 0;
  return NS_OK;
}

ns_status ns_cfl_dt(ns_ctx* X, double cfl, double dt_max, double* dt_out) {
  if (!X || !dt_out) return NS_EINVAL;
  if (!(cfl > 0.0) || !(dt_max > 0.0)) return fail(X, NS_EINVAL, "cfl and dt_max must be > 0");
  launch_cfl_max(X->phys, X->F.u, X->F.v, X->F.w, X->partials, X->host_dev + S_CFL, X->st);
  HIPCHK(X, hipGetLastError());
  ns_status s = wait_host(X);
  if (s != NS_OK) return s;
  const double m = X->host[S_CFL];
  if (!std::isfinite(m)) return fail(X, NS_ENAN, "non-finite velocity in the CFL rule");
  if (!(m > 0.0)) {
    *dt_out = dt_max;
    return NS_OK;
  }
  const double dt = cfl * X->P.h / m;
  *dt_out = dt < dt_max ? dt : dt_max;
  return NS_OK;
}

ns_status ns_set_fine_sweep(ns_ctx* X, int fused) {
  if (!X) return NS_EINVAL;
  if (fused != 0 && fused != 1) return fail(X, NS_EINVAL, "fused must be 0 or 1");
  if (fused && !gs_rb_fine_fits(X->lev[0].n)) return fail(X, NS_EINVAL, "the fused sweep does not apply to this grid");
  X->fine_rb = fused != 0;
  // the recorded V-cycle graphs hold the old schedule: record them again
  HIPCHK(X, hipStreamSynchronize(X->st));
  for (int q = 0; q < X->ngs; ++q) (void)hipGraphExecDestroy(X->gs[q].exec);
  X->ngs = 0;
  return NS_OK;
}

ns_status ns_get_fine_sweep(const ns_ctx* X, int* fused) {
  if (!X || !fused) return NS_EINVAL;
  *fused = X->fine_rb ? 1 : 0;
  return NS_OK;
}

ns_status ns_set_face_tables(ns_ctx* X, int on) {
  if (!X) return NS_EINVAL;
  if (on != 0 && on != 1) return fail(X, NS_EINVAL, "on must be 0 or 1");
  X->face_tabs = on != 0;
  for (int l = 0; l < X->L && l <= 1; ++l)
    X->lev[l].tab_ok = X->lev[l].tabf_ok = false;   // built again by the next solve when on
  // the recorded V-cycle graphs hold the tables' addresses or none: record them again
  HIPCHK(X, hipStreamSynchronize(X->st));
  for (int q = 0; q < X->ngs; ++q) (void)hipGraphExecDestroy(X->gs[q].exec);
  X->ngs = 0;
  return NS_OK;
}

ns_status ns_get_face_tables(const ns_ctx* X, int* on) {
  if (!X || !on) return NS_EINVAL;
  *on = X->face_tabs ? 1 : 0;
  return NS_OK;
}

ns_status ns_set_launch_mode(ns_ctx* X, int mode) {
  if (!X) return NS_EINVAL;
  if (mode != NS_LAUNCH_STREAM && mode != NS_LAUNCH_GRAPH) return fail(X, NS_EINVAL, "unknown launch mode %d", mode);
  X->launch_mode = mode;
  return NS_OK;
}

ns_status ns_timing_enable(ns_ctx* X, int kernel, int max_launches) {
  if (!X) return NS_EINVAL;
  HIPCHK(X, hipStreamSynchronize(X->st));
  free_timer(X);
  if (max_launches <= 0) return NS_OK;
  if (kernel != NS_TIME_SMOOTH0 && kernel != NS_TIME_SPMV)
    return fail(X, NS_EINVAL, "unknown timed kernel %d", kernel);
  X->kt.ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches];
  if (!X->kt.ev) return fail(X, NS_EINVAL, "cannot hold %d event pairs", max_launches);
  for (int q = 0; q < 2 * max_launches; ++q) {
    if (hipEventCreate(&X->kt.ev[q]) != hipSuccess) {
      X->kt.cap = q / 2;
      for (int r = 0; r < q; ++r) (void)hipEventDestroy(X->kt.ev[r]);
      delete[] X->kt.ev;
      X->kt = KTimer{nullptr, 0, 0};
      return fail(X, NS_EHIP, "hipEventCreate failed");
    }
  }
  X->kt.cap = max_launches;
  X->kt.n = 0;
  X->timed_kernel = kernel;
  return NS_OK;
}

ns_status ns_time_kernel(ns_ctx* X, int kernel, int reps, double* avg_ms) {
  if (!X || !avg_ms || reps <= 0) return NS_EINVAL;
  if (kernel != NS_TIME_SMOOTH0 && kernel != NS_TIME_SPMV)
    return fail(X, NS_EINVAL, "unknown timed kernel %d", kernel);
  if (!X->have_beta) return fail(X, NS_ESTATE, "no coefficients yet: call momentum_step first");
  if (kernel == NS_TIME_SMOOTH0 && (X->P.prec == NS_PREC_FP64 ? X->tail64 : X->tail32) == 0)
    return fail(X, NS_EINVAL, "the whole hierarchy runs in the coarse-level tail: no finest smoother pass");
  hipEvent_t a, b;
  HIPCHK(X, hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(X, NS_EHIP, "hipEventCreate failed");
  }
  Level& L0 = X->lev[0];
  const Dims n = L0.n;
  const CgScratch cs{X->partials, X->scal, X->host_dev, nullptr};
  build_face_tables(X);   // as a solve reads the coefficients
  (void)hipStreamSynchronize(X->st);
  (void)hipEventRecord(a, X->st);
  for (int q = 0; q < reps; ++q) {
    if (kernel == NS_TIME_SMOOTH0) {
      // the finest smoother pass of the configured precision (the fused
      // red-black sweep where it is used, else one colour pass), on the
      // level's colour-split b and e, which are dead between V-cycles
      const size_t ns = 2 * (size_t)((n.nx + 1) / 2) * n.ny * n.nz;
      if (X->P.prec == NS_PREC_FP64) {
        if (X->fine_rb)
          launch_gs_rb_fine<double>(L0, L0.bx, L0.by, L0.bz, L0.b, L0.e, L0.e + ns, X->st);
        else
          launch_gs<double>(L0, L0.bx, L0.by, L0.bz, L0.b, L0.e, q & 1, X->st);
      } else {
        if (X->fine_rb)
          launch_gs_rb_fine<float>(L0, L0.bxf, L0.byf, L0.bzf, L0.bf, L0.ef, L0.ef + ns, X->st);
        else
          launch_gs<float>(L0, L0.bxf, L0.byf, L0.bzf, L0.bf, L0.ef, q & 1, X->st);
      }
    } else {
      launch_dir_spmv(n, X->P.h, L0.bx, L0.by, L0.bz, X->zn, X->d, X->d2, X->q, 1, cs, X->st, nullptr, nullptr,
                      face_tab(L0, L0.bx));
    }
  }
  (void)hipEventRecord(b, X->st);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(X, NS_EHIP, "event timing: %s", hipGetErrorString(e));
  *avg_ms = (double)ms / reps;
  return NS_OK;
}

ns_status ns_timing_read(ns_ctx* X, double* total_ms, int* launches) {
  if (!X || !total_ms || !launches) return NS_EINVAL;
  HIPCHK(X, hipStreamSynchronize(X->st));
  double tot = 0.0;
  for (int q = 0; q < X->kt.n; ++q) {
    float ms = 0.0f;
    HIPCHK(X, hipEventElapsedTime(&ms, X->kt.ev[2 * q], X->kt.ev[2 * q + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = X->kt.n;
  X->kt.n = 0;
  return NS_OK;
}

const char* ns_last_error(ns_ctx* X) { return X ? X->err : "null context"; }

// Force on every free body from the current pressure, velocity and the
// viscosity in the workspace: the kernels and the copies of their partials
// into pinned host memory are queued; free_forces_sum, after the stream has
// been synchronised, sums each body's partials in block order.
int free_forces_queue(ns_ctx* X, int nb[4]) {
  for (int m = 0; m < X->phys.nb; ++m) {
    nb[m] = 0;
    if (!X->phys.body[m].fh) continue;
    nb[m] = launch_hydro_force(X->phys, m, X->t_props, X->F.p, X->F.u, X->F.v, X->F.w, X->mu, X->partials,
                               X->fcap, X->st);
    if (nb[m] < 0) return -1;
    if (nb[m] > 0 &&
        hipMemcpyAsync(X->fpart + (size_t)3 * X->fcap * m, X->partials, (size_t)3 * nb[m] * sizeof(double),
                       hipMemcpyDeviceToHost, X->st) != hipSuccess)
      return -1;
  }
  return 0;
}

void free_forces_sum(ns_ctx* X, const int nb[4]) {
  for (int m = 0; m < X->phys.nb; ++m) {
    if (!X->phys.body[m].fh) continue;
    const double* q = X->fpart + (size_t)3 * X->fcap * m;
    double F[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nb[m]; ++b)
      for (int c = 0; c < 3; ++c) F[c] += q[3 * b + c];
    for (int c = 0; c < 3; ++c) X->bs[m].F[c] = F[c];
  }
  X->force_ready = true;
}

// The force of the current fields when none is at hand (the first step):
// the viscosity of the current level set and heave at time t, then the force.
ns_status ensure_free_forces(ns_ctx* X, double t) {
  if (X->nfree == 0 || X->force_ready) return NS_OK;
  X->t_props = t;
  launch_props(X->phys, X->F.sigma, t, X->rho, X->rfl, X->mu, X->chi, X->st);
  int nb[4];
  if (free_forces_queue(X, nb) != 0) return fail(X, NS_EHIP, "hydrodynamic force: launch or copy failed");
  HIPCHK(X, hipStreamSynchronize(X->st));
  free_forces_sum(X, nb);
  return NS_OK;
}

// eqn_newton_u for every free body with the force of the current fields:
// m (zdot' - zdot) / dt = Fz - m g - c zdot', zeta' = zeta + dt zdot'
void free_heave_update(ns_ctx* X, double dt) {
  for (int m = 0; m < X->phys.nb; ++m) {
    BodyK& B = X->phys.body[m];
    if (!B.fh) continue;
    const ns_body& Q = X->P.body[m];
    const double zd = (B.zdot + dt * (X->bs[m].F[2] - Q.mass * X->P.g) / Q.mass) / (1.0 + dt * Q.pto_damping / Q.mass);
    B.zdot = zd;
    B.zeta += dt * zd;
    X->bs[m].fpto = -Q.pto_damping * zd;
  }
  X->force_ready = false;
}

ns_status levelset_advect_reinit(ns_ctx* X, double dt) {
  if (!X) return NS_EINVAL;
  if (!(dt > 0.0)) return fail(X, NS_EINVAL, "dt must be > 0");
  const Phys& ph = X->phys;
  hipStream_t st = X->st;
  launch_advect(ph, X->F.sigma, X->F.u, X->F.v, X->F.w, dt, X->sig_a, st);
  const int nr = X->P.reinit_iters;
  const double dtau = X->P.reinit_dtau_over_h * X->P.h;
  if (nr == 0) {
    launch_copy(X->sig_a, X->F.sigma, X->nc, st);
  } else {
    // sig_a keeps sigma0 (for the sign); ping-pong between the field and
    // sig_b so that the last pseudo-step lands in the field
    const double* cur = X->sig_a;
    for (int it = 0; it < nr; ++it) {
      double* dst = ((nr - 1 - it) % 2 == 0) ? X->F.sigma : X->sig_b;
      launch_reinit(ph, X->sig_a, cur, dst, dtau, st);
      cur = dst;
    }
  }
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

ns_status momentum_step(ns_ctx* X, double dt, double t_np1) {
  if (!X) return NS_EINVAL;
  if (!(dt > 0.0)) return fail(X, NS_EINVAL, "dt must be > 0");
  hipStream_t st = X->st;
  if (X->nfree > 0) {
    // ns_step has already taken the force of the state the step starts from;
    // a caller driving the stages alone gets that of the current fields
    ns_status s = ensure_free_forces(X, t_np1 - dt);
    if (s != NS_OK) return s;
    free_heave_update(X, dt);
  }
  const Phys& ph = X->phys;
  if (X->P.consistent) {
    // the density at t^n: the last properties (ns_step fills them on its
    // first step; a caller driving the stages alone gets the current level set's)
    if (!X->have_rho_n) launch_props(ph, X->F.sigma, t_np1 - dt, X->rho, X->rfl, X->mu, X->chi, st);
    std::swap(X->rho, X->rho_prev);
  }
  X->t_props = t_np1;
  launch_props(ph, X->F.sigma, t_np1, X->rho, X->rfl, X->mu, X->chi, st);
  Level& L0 = X->lev[0];
  // Crank-Nicolson: the predictor writes the first iterate and the sweeps
  // alternate between u* and a second set, starting in the one that leaves
  // the first batch's last iterate in u*
  const int S = X->P.cn_sweeps;
  double* us3[3] = {X->us, X->vs, X->ws};
  double** cur = (S % 2) ? X->cn_tmp : us3;
  double** nxt = (S % 2) ? us3 : X->cn_tmp;
  X->host[S_FLAGS] = 0.0;   // the consistent predictor stores 1 here on a density <= 0
  launch_momentum(ph, X->F.u, X->F.v, X->F.w, X->rho, X->rfl, X->mu, X->chi, X->P.consistent ? X->rho_prev : nullptr,
                  dt, t_np1, cur[0], cur[1], cur[2], L0.bx, L0.by, L0.bz, L0.bxf, L0.byf, L0.bzf,
                  S > 0 ? X->cn_rhs : nullptr, S > 0 ? X->cn_diag : nullptr, X->host_dev + S_FLAGS, st);
  X->last_cn = 0;
  X->have_beta = false;
  L0.tab_ok = L0.tabf_ok = false;   // new face coefficients
  if (S > 0) {
    // batches of S sweeps, the last of each measuring its largest change,
    // until that change is below cn_tol of the largest |u*|
    constexpr int kCnMaxSweeps = 64;
    for (;;) {
      for (int q = 0; q < S; ++q) {
        const bool last = q == S - 1;
        launch_cn_sweep(ph, cur[0], cur[1], cur[2], X->mu, X->cn_rhs, X->cn_diag, nxt[0], nxt[1], nxt[2],
                        last ? X->cnpart : nullptr, last ? X->host_dev + S_CNDU : nullptr, st);
        std::swap(cur, nxt);
      }
      X->last_cn += S;
      HIPCHK(X, hipGetLastError());
      ns_status s = wait_host(X);
      if (s != NS_OK) return s;
      const double du = X->host[S_CNDU], um = X->host[S_CNU];
      if (!std::isfinite(du) || !std::isfinite(um)) return fail(X, NS_ENAN, "non-finite Crank-Nicolson iterate");
      if (du <= X->P.cn_tol * um) break;
      if (X->last_cn + S > kCnMaxSweeps)
        return fail(X, NS_ENOCONV, "Crank-Nicolson sweeps did not converge: last change %.3e of max |u*| %.3e "
                    "after %d sweeps", du, um, X->last_cn);
    }
    if (cur != us3) {   // an odd number of extra batches left the iterate in the second set
      launch_copy(cur[0], X->us, X->nu, st);
      launch_copy(cur[1], X->vs, X->nv, st);
      launch_copy(cur[2], X->ws, X->nw, st);
    }
  }
  X->have_rho_n = X->P.consistent != 0;
  HIPCHK(X, hipGetLastError());
  X->have_beta = true;
  return NS_OK;
}

ns_status projection_solve(ns_ctx* X, double dt, ns_stats* stats) {
  if (!X) return NS_EINVAL;
  if (!(dt > 0.0)) return fail(X, NS_EINVAL, "dt must be > 0");
  if (!X->have_beta) return fail(X, NS_ESTATE, "projection_solve before momentum_step");
  const double t0 = now_ms();
  const Phys& ph = X->phys;
  hipStream_t st = X->st;
  const bool timed = X->phase_on;
  const bool whole = timed && X->ph_step;
  X->ph_step = false;
  if (timed) HIPCHK(X, hipEventRecord(X->ph_ev[2], st));
  launch_rhs(ph, X->us, X->vs, X->ws, dt, X->b, st);
  int fallback = 0, used = X->P.x0;
  bool trial = false;
  double rel_prev = 0.0;
  if (X->P.x0 == NS_X0_AUTO) {
    if (!X->net) return fail(X, NS_ESTATE, "x0 = NS_X0_AUTO needs ns_attach_net");
    constexpr int kAutoRetry = 8;
    trial = X->ax.trials == 0 || X->ax.since + 1 >= kAutoRetry || X->ax.gain * X->ax.t_it > X->ax.t_inf;
    used = trial ? NS_X0_LEARNED : NS_X0_PREV;
  }
  if (used == NS_X0_ZERO) {
    launch_fill<double>(X->F.p, X->nc, st);
  } else if (used == NS_X0_LEARNED) {
    // p0 = p_prev + P0 delta(features of b, rho, p_prev); p_prev if not finite
    ns_net* N = X->net;
    if (!N) return fail(X, NS_ESTATE, "x0 = NS_X0_LEARNED needs ns_attach_net");
    const Level& L0 = X->lev[0];
    double* pprev = net_pprev(N);
    launch_copy(X->F.p, pprev, X->nc, st);
    if (trial) {
      // ||b - A p_prev||: the residual the step would start from without the network
      const CgScratch cs{X->partials, X->scal, X->host_dev, X->hpart_dev};
      launch_resid_norm(L0.n, X->P.h, L0.bx, L0.by, L0.bz, X->b, pprev, X->r, cs, FIN_RESID0, st);
      HIPCHK(X, hipEventRecord(X->ax.ev[0], st));
    }
    launch_apply_A(L0.n, X->P.h, L0.bx, L0.by, L0.bz, pprev, net_Ap(N), st);
    net_features(N, L0.n, X->P.h, X->P.rho_w, X->P.rho_a, X->P.p_scale, X->b, X->rho, pprev, net_Ap(N),
                 net_feat(N), st);
    if (net_guess(N, X->P.p_scale, X->F.p, st, trial ? X->ax.ev[1] : nullptr) != 0) {
      launch_copy(pprev, X->F.p, X->nc, st);
      fallback = 1;
      used = NS_X0_PREV;
    }
    if (trial) {   // net_guess synchronised the stream
      const double bb = host_total(X, 2, 1, S_BB), rr = host_total(X, 2, 0, S_RR);
      // formed as the solve forms its starting relative residual, so that a
      // guess equal to p_prev compares equal
      rel_prev = bb > 0.0 ? std::sqrt(rr) / std::sqrt(bb) : 0.0;
      float ms = 0.f;
      HIPCHK(X, hipEventElapsedTime(&ms, X->ax.ev[0], X->ax.ev[1]));
      X->ax.t_inf = ms;
    }
  }
  ns_stats S{};
  if (timed) HIPCHK(X, hipEventRecord(X->ph_ev[3], st));
  const double tc = now_ms();
  ns_status s = pcg(X, &S);
  S.x0_fallback = fallback;
  S.x0_used = used;
  S.cn_sweeps = X->last_cn;
  if (X->P.x0 == NS_X0_AUTO && (s == NS_OK || s == NS_ENOCONV)) {
    X->ax.t_it = (now_ms() - tc) / (S.iters > 0 ? S.iters : 1);
    if (trial) {
      // iterations saved: log(r_prev / r_learned) over the solve's log contraction per iteration
      double saved = 0.0;
      const double q = S.iters > 0 && S.rel_resid0 > 0.0 ? std::pow(S.rel_resid / S.rel_resid0, 1.0 / S.iters) : 0.0;
      if (!fallback && q > 0.0 && q < 1.0 && rel_prev > 0.0 && S.rel_resid0 > 0.0)
        saved = std::log(rel_prev / S.rel_resid0) / -std::log(q);
      if (std::isfinite(saved)) X->ax.gain = X->ax.trials == 0 ? saved : 0.5 * (X->ax.gain + saved);
      ++X->ax.trials;
      X->ax.since = 0;
    } else {
      ++X->ax.since;
    }
    S.x0_gain = X->ax.gain;
  }
  if (s != NS_OK && s != NS_ENOCONV) {
    if (stats) *stats = S;
    return s;
  }
  const Level& L0 = X->lev[0];
  if (timed) HIPCHK(X, hipEventRecord(X->ph_ev[4], st));
  launch_correct(ph, X->us, X->vs, X->ws, X->F.p, L0.bx, L0.by, L0.bz, dt, X->F.u, X->F.v, X->F.w, st);
  // the wave tank's relaxation zones, at the time of the step's properties
  launch_relax(ph, X->t_props, X->F.sigma, X->F.u, X->F.v, X->F.w, st);
  // the zones changed sigma: the density consistent transport starts the next
  // step from, and the viscosity of the force below, are those of the
  // relaxed level set
  if ((ph.gen_len > 0.0 || ph.damp_len > 0.0) && (X->nfree > 0 || X->P.consistent))
    launch_props(ph, X->F.sigma, X->t_props, X->rho, X->rfl, X->mu, X->chi, st);
  // the hydrodynamic force of the new fields, for the next heave update
  int nb[4];
  if (X->nfree > 0 && free_forces_queue(X, nb) != 0)
    return fail(X, NS_EHIP, "hydrodynamic force: launch or copy failed");
  HIPCHK(X, hipGetLastError());
  if (timed) HIPCHK(X, hipEventRecord(X->ph_ev[5], st));
  HIPCHK(X, hipStreamSynchronize(st));
  if (X->nfree > 0) free_forces_sum(X, nb);
  if (timed) {
    // [2] set-up, [3] CG, [4] correction; from ns_step also [0], [1] and the whole step
    float ms;
    for (int q = whole ? 0 : 2; q < 5; ++q) {
      HIPCHK(X, hipEventElapsedTime(&ms, X->ph_ev[q], X->ph_ev[q + 1]));
      S.t_ms[q] = ms;
    }
    if (whole) {
      HIPCHK(X, hipEventElapsedTime(&ms, X->ph_ev[0], X->ph_ev[5]));
      S.t_ms[5] = ms;
    }
  }
  S.ms = now_ms() - t0;
  if (stats) *stats = S;
  return s;
}

ns_status ns_step(ns_ctx* X, double dt, double t_n, ns_stats* stats) {
  if (!X) return NS_EINVAL;
  const double t0 = now_ms();
  // free bodies: on the first step, the force of the state the step starts from
  ns_status s = ensure_free_forces(X, t_n);
  if (s != NS_OK) return s;
  // consistent transport: on the first step, the density the step starts from
  if (X->P.consistent && !X->have_rho_n) {
    launch_props(X->phys, X->F.sigma, t_n, X->rho, X->rfl, X->mu, X->chi, X->st);
    X->have_rho_n = true;
  }
  if (X->phase_on) HIPCHK(X, hipEventRecord(X->ph_ev[0], X->st));
  s = levelset_advect_reinit(X, dt);
  if (s != NS_OK) return s;
  if (X->phase_on) HIPCHK(X, hipEventRecord(X->ph_ev[1], X->st));
  if ((s = momentum_step(X, dt, t_n + dt)) != NS_OK) return s;
  X->ph_step = X->phase_on;
  ns_stats S{};
  s = projection_solve(X, dt, &S);
  S.ms = now_ms() - t0;
  if (stats) *stats = S;
  return s;
}

ns_status ns_pcg_solve(ns_ctx* X, ns_stats* stats) {
  if (!X) return NS_EINVAL;
  const double t0 = now_ms();
  // the FP32 level-0 copy follows the (possibly caller-written) FP64 beta
  Level& L0 = X->lev[0];
  launch_d2f(L0.bx, L0.bxf, X->nu, X->st);
  launch_d2f(L0.by, L0.byf, X->nv, X->st);
  launch_d2f(L0.bz, L0.bzf, X->nw, X->st);
  ns_stats S{};
  ns_status s = pcg(X, &S);
  HIPCHK(X, hipStreamSynchronize(X->st));
  S.ms = now_ms() - t0;
  if (stats) *stats = S;
  return s;
}

ns_status ns_apply_A(ns_ctx* X, const double* x, double* y) {
  if (!X) return NS_EINVAL;
  if (!aligned8(x) || !aligned8(y)) return fail(X, NS_EINVAL, "x and y must be 8-byte aligned device pointers");
  const Level& L0 = X->lev[0];
  launch_apply_A(L0.n, X->P.h, L0.bx, L0.by, L0.bz, x, y, X->st);
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

ns_status ns_vcycle(ns_ctx* X, const double* r, double* z) {
  if (!X) return NS_EINVAL;
  if (!aligned8(r) || !aligned8(z)) return fail(X, NS_EINVAL, "r and z must be 8-byte aligned device pointers");
  Level& L0 = X->lev[0];
  launch_d2f(L0.bx, L0.bxf, X->nu, X->st);
  launch_d2f(L0.by, L0.byf, X->nv, X->st);
  launch_d2f(L0.bz, L0.bzf, X->nw, X->st);
  prepare_hierarchy(X);
  precond_launch(X, r, z);   // caller pointers: launched, never recorded
  HIPCHK(X, hipGetLastError());
  return NS_OK;
}

ns_status ns_buffer(ns_ctx* X, int which, void** dev_ptr, size_t* count) {
  if (!X || !dev_ptr) return NS_EINVAL;
  const Level& L0 = X->lev[0];
  void* p = nullptr;
  size_t c = 0;
  switch (which) {
    case NS_BUF_US: p = X->us; c = X->nu; break;
    case NS_BUF_VS: p = X->vs; c = X->nv; break;
    case NS_BUF_WS: p = X->ws; c = X->nw; break;
    case NS_BUF_BX: p = L0.bx; c = X->nu; break;
    case NS_BUF_BY: p = L0.by; c = X->nv; break;
    case NS_BUF_BZ: p = L0.bz; c = X->nw; break;
    case NS_BUF_RHS: p = X->b; c = X->nc; break;
    case NS_BUF_RHO: p = X->rho; c = X->nc; break;
    case NS_BUF_MU: p = X->mu; c = X->nc; break;
    case NS_BUF_CHI: p = X->chi; c = X->nc; break;
    case NS_BUF_RHOFLOW: p = X->rfl; c = X->nc; break;
    case NS_BUF_BXF: p = L0.bxf; c = X->nu; break;
    case NS_BUF_BYF: p = L0.byf; c = X->nv; break;
    case NS_BUF_BZF: p = L0.bzf; c = X->nw; break;
    default: return fail(X, NS_EINVAL, "unknown buffer id %d", which);
  }
  *dev_ptr = p;
  if (count) *count = c;
  if (which == NS_BUF_BX || which == NS_BUF_BY || which == NS_BUF_BZ || which == NS_BUF_RHS)
    X->have_beta = true;   // the caller may fill the projection inputs directly
  if (which == NS_BUF_BX || which == NS_BUF_BY || which == NS_BUF_BZ || which == NS_BUF_BXF || which == NS_BUF_BYF ||
      which == NS_BUF_BZF)
    X->lev[0].tab_ok = X->lev[0].tabf_ok = false;   // the caller may write them
  return NS_OK;
}

ns_status ns_body_state(ns_ctx* X, int body, double out[6]) {
  if (!X || !out) return NS_EINVAL;
  if (body < 0 || body >= X->phys.nb) return fail(X, NS_EINVAL, "no body %d", body);
  const BodyK& B = X->phys.body[body];
  out[0] = B.fh ? B.zeta : B.amp * std::sin(B.om * X->t_props + B.ph);
  out[1] = B.fh ? B.zdot : B.amp * B.om * std::cos(B.om * X->t_props + B.ph);
  for (int c = 0; c < 3; ++c) out[2 + c] = B.fh ? X->bs[body].F[c] : 0.0;
  out[5] = B.fh ? X->bs[body].fpto : 0.0;
  return NS_OK;
}

ns_status ns_diagnostics(ns_ctx* X, double out[4]) {
  if (!X || !out) return NS_EINVAL;
  const int np = launch_diag_partials(X->phys, X->F.sigma, X->F.u, X->F.v, X->F.w, X->partials, X->st);
  launch_diag_finalize(X->partials, np, X->scal, X->st);
  ns_status s = read_scal(X);
  if (s != NS_OK) return s;
  for (int q = 0; q < 4; ++q) out[q] = X->host[S_DIAG + q];
  return NS_OK;
}

}  // extern "C"
