// Internal declarations shared by the kernel and ABI translation units of
// the gfx950 library.  Not part of the public ABI (see include/ns.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ns.h"

namespace nsk {

// The tile (block coordinates in the launch grid) a workgroup works on.
// Workgroups are handed to the eight XCDs round-robin by linear id, and each
// XCD has its own L2; this gives XCD x the contiguous run of tiles
// [start(x), start(x + 1)) of the tile order, so that tiles sharing halo
// rows and planes mostly share an L2.  The order takes the tile rows in
// bands of four to kTileBand (x fastest, then y within the band, then z,
// then the next band), the widest such band that divides the grid's tile
// rows, else all of them in one band (plain x, y, z order).  A tile's
// z-neighbours then run a band's width of tiles after it rather than a
// whole plane's, and the planes a stencil reads three times are still in
// the L2: on 512x256x256 the finest-level stencils' L2 misses fell from
// 1.3-1.6x to 1.02-1.04x their algorithmic bytes, and their time by 2-7%.
// xcd_tile_flat keeps plain order for kernels that march along z
// themselves.  Both are bijections for any grid, so no result depends on
// the dispatch order.  lin is the tile's position in the order, which also
// numbers its reduction partial.
struct Tile {
  int x, y, z, lin;
};
constexpr int kTileBand = 8;
__device__ __forceinline__ Tile xcd_tile_order(int band) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int nb = gx * gy * (int)gridDim.z;
  const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  Tile t;
  t.lin = x * q + (x < r ? x : r) + (b >> 3);
  const int per = gx * band * (int)gridDim.z;   // tiles per band
  const int bi = t.lin / per, rem = t.lin - bi * per;
  t.x = rem % gx;
  const int yz = rem / gx;
  t.y = bi * band + yz % band;
  t.z = yz / band;
  return t;
}
__device__ __forceinline__ Tile xcd_tile_flat() { return xcd_tile_order(gridDim.y); }
__device__ __forceinline__ Tile xcd_tile() {
  const int gy = gridDim.y;
  int band = gy;
  for (int d = kTileBand; d >= kTileBand / 2; --d)
    if (gy % d == 0) {
      band = d;
      break;
    }
  return xcd_tile_order(band);
}

struct Dims {
  int nx, ny, nz;
};

struct BodyK {
  int kind;
  double c0, c1, c2;
  double h0, h1, h2;
  double amp, om, ph;
  int fh;              // free heave: zeta, zdot below are the body's state
  double zeta, zdot;
};

// Physical constants and geometry passed by value to the grid kernels.
struct Phys {
  Dims n;
  double h;
  double rho_w, mu_w, rho_a, mu_a, rho_s, mu_s, g;
  double eps;      // Heaviside half-width n_cells * h
  double inv_kp;   // 1 / kappa_p
  double pen_w;    // projection penalty weight
  int nb;
  BodyK body[4];
  // numerical wave tank: zones (0: none), still-water depth, the generated
  // wave's components (device array: a, kappa, omega, phase per component)
  double depth, gen_len, damp_len, vort_w;
  int nwave;
  const double* waves;
};

// One multigrid level.  Level 0 of the FP64 hierarchy aliases the CG
// vectors (b = r, e = z); level 0 of the FP32 hierarchy has its own b, e.
// Line tables of a level's face coefficients.  A line is the faces along x
// of one (j, k): (nx + 1) x-faces (ny nz lines), nx y-faces ((ny + 1) nz
// lines), nx z-faces (ny (nz + 1) lines).  Entry (line) holds the value
// every face of the line takes (for an x-line: every interior face, its two
// wall faces being zero), or the all-ones marker where they differ.  In a
// two-phase tank most lines lie wholly in water or wholly in air, so a
// kernel whose wavefront covers one line reads one entry instead of the
// line's faces.  The face arrays stay complete; a table only spares loads.
template <typename T>
struct FaceTab {
  const T* x = nullptr;
  const T* y = nullptr;
  const T* z = nullptr;
};

struct Level {
  Dims n;
  double h;
  double h0;                    // finest-level spacing (h == h0 on level 0)
  int f[3];                     // coarsening factor towards level + 1
  double *bx, *by, *bz;         // FP64 face coefficients (walls = 0)
  float *bxf, *byf, *bzf;       // FP32 copies
  double *b, *e;                // FP64 right-hand side and correction (split above the tail)
  float *bf, *ef;               // FP32
  float *bfn, *efn;             // level 0, FP32: natural-order b and e of the mixed V-cycle
  double* invd;                 // 1 / diagonal (h^2 scaled), FP64
  float* invdf;                 // FP32
  // level 0: line tables of bx, by, bz (FP64) and of their FP32 copies;
  // valid while tab_ok / tabf_ok (the arrays unchanged since they were built)
  double *tx, *ty, *tz;
  float *txf, *tyf, *tzf;
  bool tab_ok, tabf_ok;
};

// the line tables of L's face arrays of type T when they are current and
// bx is that array, else none
template <typename T>
inline FaceTab<T> face_tab(const Level& L, const T* bx) {
  FaceTab<T> t;
  if constexpr (sizeof(T) == 8) {
    if (L.tab_ok && bx == L.bx) t = FaceTab<T>{L.tx, L.ty, L.tz};
  } else {
    if (L.tabf_ok && bx == L.bxf) t = FaceTab<T>{L.txf, L.tyf, L.tzf};
  }
  return t;
}

// Device scalars of the CG iteration (one cache line each group).
enum ScalIdx {
  S_BB = 0,     // ||b||^2
  S_RR = 1,     // ||r||^2 (latest)
  S_RHO = 2,    // <r, z>
  S_ALPHA = 3,
  S_BETA = 4,
  S_DQ = 5,     // <d, A d>
  S_TRR = 6,    // ||b - A x||^2 recomputed
  S_CFL = 7,    // max over cells of |u_c| + |v_c| + |w_c| (the CFL rule)
  S_DIAG = 8,   // 4 diagnostics
  S_FLAGS = 12, // set to 1 by the predictor when a carried face density is <= 0
  S_CNDU = 13,  // Crank-Nicolson: largest change of the last sweep
  S_CNU = 14,   //   and the largest |u*| it produced
  S_COUNT = 16
};

// Event pairs recorded with selected dispatches (profiling aid).
struct KTimer {
  hipEvent_t* ev;   // 2 * cap events: start, stop per launch
  int cap;
  int n;
};

// Coarse-level tail of the V-cycle run by one workgroup from LDS.
constexpr int kTailMaxLevels = 12;
constexpr int kTailThreads = 512;
constexpr size_t kTailLdsBytes = 160 * 1024;   // gfx950: 160 KB of LDS per workgroup

template <typename T>
struct TailDesc {
  int nl;                                   // levels in the tail (>= 1)
  int nu_pre, nu_post, coarse_sweeps;
  Dims n[kTailMaxLevels];
  int f[kTailMaxLevels][3];                 // coarsening factor of level l towards l + 1
  T h2[kTailMaxLevels];
  int obx[kTailMaxLevels], oby[kTailMaxLevels], obz[kTailMaxLevels];  // LDS offsets (elements)
  int ob[kTailMaxLevels], oe[kTailMaxLevels], oid[kTailMaxLevels];
  int ors;                                  // LDS scratch: one value per cell of the first level
  // staging: the first npack LDS elements are a flat copy of pack (the tail
  // levels' bx, by, bz, 1/D), then the first level's b goes to ob[0]
  const T* pack;
  int npack;
  const T* b0;
  T* ge;                                    // correction of the first tail level (output)
};

enum FinMode { FIN_RESID0 = 0, FIN_RHO = 1, FIN_ALPHA = 2, FIN_RR = 3, FIN_BETA = 4, FIN_TRR = 5 };

// Per-block partial sums and the CG scalars.
struct CgScratch {
  double* partials;
  double* scal;
  double* hscal;   // device address of the pinned host mirror of scal (the
                   // values the host tests: S_BB, S_RR, S_TRR)
  double* hpart;   // device address of pinned host partials, or null: when
                   // set, the reductions only the host reads (||r||^2,
                   // ||b||^2, the true residual) leave their per-block
                   // partials there for the host to sum, with no finalize
};

// the host sums the partials of its own reductions up to this many blocks
constexpr int kHostPartsMax = 8192;

// ---------------------------------------------------------------- launchers
// grid step kernels (ns_grid.hip)
void launch_advect(const Phys& P, const double* s, const double* u, const double* v, const double* w,
                   double dt, double* out, hipStream_t st);
void launch_reinit(const Phys& P, const double* s0, const double* cur, double* nxt, double dtau,
                   hipStream_t st);
void launch_copy(const double* src, double* dst, size_t n, hipStream_t st);
void launch_props(const Phys& P, const double* sigma, double t, double* rho, double* rfl, double* mu,
                  double* chi, hipStream_t st);
// rho_n set: the consistent form, which stores 1.0 to *flag (device address of
// host-mapped memory) when a carried face density comes out <= 0
void launch_momentum(const Phys& P, const double* u, const double* v, const double* w,
                     const double* rho, const double* rfl, const double* mu, const double* chi,
                     const double* rho_n, double dt, double t1, double* us, double* vs, double* ws, double* bx,
                     double* by, double* bz, float* bxf, float* byf, float* bzf, double* const* cn_rhs,
                     double* const* cn_diag, double* flag, hipStream_t st);
// one Jacobi sweep of the Crank-Nicolson viscous system: (u, v, w) -> (uo, vo, wo);
// with part (2 cn_part_blocks values), also each block's largest change and
// largest |new value| over the faces it updates, then their maxima to out2
// (two doubles, e.g. the host mirror)
void launch_cn_sweep(const Phys& P, const double* u, const double* v, const double* w, const double* mu,
                     double* const* rhs, double* const* diag, double* uo, double* vo, double* wo, double* part,
                     double* out2, hipStream_t st);
int cn_part_blocks(const Dims& n);
// the CFL rule's maximum over cells of |u_c| + |v_c| + |w_c| (infinite if any
// is not finite) into *out; partials holds one value per diag_blocks block
void launch_cfl_max(const Phys& P, const double* u, const double* v, const double* w, double* partials,
                    double* out, hipStream_t st);
void launch_rhs(const Phys& P, const double* us, const double* vs, const double* ws, double dt,
                double* b, hipStream_t st);
void launch_correct(const Phys& P, const double* us, const double* vs, const double* ws,
                    const double* p, const double* bx, const double* by, const double* bz, double dt,
                    double* u, double* v, double* w, hipStream_t st);
int launch_diag_partials(const Phys& P, const double* sigma, const double* u, const double* v,
                         const double* w, double* partials, hipStream_t st);
void launch_diag_finalize(const double* partials, int nparts, double* scal, hipStream_t st);
// relaxation zones of the wave tank at time t, in place (no-op without zones)
void launch_relax(const Phys& P, double t, double* sigma, double* u, double* v, double* w, hipStream_t st);
// hydrodynamic force on body m over the cells of its bounding box: three
// per-block partials (Fx, Fy, Fz) in tile order; returns the block count, or
// -1 without launching when it would exceed max_blocks
int launch_hydro_force(const Phys& P, int m, double t, const double* p, const double* u, const double* v,
                       const double* w, const double* mu, double* partials, int max_blocks, hipStream_t st);
int diag_blocks(const Phys& P);

// multigrid and CG kernels (ns_mg.hip)
// Multigrid kernels.  On levels above the tail b, e and 1/D are colour-split
// (cell (i,j,k) at ((i+j+k)&1) P + (i>>1) + ceil(nx/2) (j + ny k)); tail
// levels keep the natural layout.
// one colour pass (nat: also write the pair, both colours, to nat in natural order)
template <typename T>
void launch_gs(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, int colour,
               hipStream_t st, KTimer* kt = nullptr, T* nat = nullptr);
// red from zero + black; b natural (b_natural, its split copy written to bs) or split
// (bcopy, when set: a copy of the black plane, for a fused pass to read);
// red_out false: the red values are not stored (the next pass is a red one)
template <typename T>
void launch_gs_first(const Level& L, const T* bx, const T* by, const T* bz, const T* b, bool b_natural,
                     const T* invd, T* e, T* bs, hipStream_t st, T* bcopy = nullptr, bool red_out = true);
// prolongation of the next level's correction ec (split or natural) + black
template <typename T>
void launch_gs_prolong(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e,
                       const Level& C, const T* ec, bool ec_split, hipStream_t st, T* bcopy = nullptr);
// a red then a black pass in one launch, reading the black plane's copy
// bold; only where gs_rb_fits (rows of at most 32 pairs)
bool gs_rb_fits(const Dims& n);
template <typename T>
void launch_gs_rb(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, const T* bold,
                  hipStream_t st);
// the finest level's red then black pass in one launch, each face coefficient
// read once (3-D levels where gs_rb_fine_fits; the default where
// gs_rb_fine_pays for the cycle's precision and the line tables' use); bold:
// the black plane's copy
bool gs_rb_fine_fits(const Dims& n);
bool gs_rb_fine_pays(const Dims& n, bool fp64, bool tables);
template <typename T>
void launch_gs_rb_fine(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, const T* bold,
                       hipStream_t st, KTimer* kt = nullptr);
// coarse b = restricted residual (coarse layout split or natural)
template <typename T>
void launch_resid_restrict(const Level& F, const T* bx, const T* by, const T* bz, const T* b,
                           const T* e, const Level& C, T* bc, bool c_split, hipStream_t st);
template <typename T>
void launch_prolong(const Level& F, T* e, const Level& C, const T* ec, bool ec_split, hipStream_t st);
template <typename T>
void launch_split_copy(const Level& L, const T* src, T* dst, bool to_split, hipStream_t st);
template <typename T>
void launch_invdiag(const Level& L, const T* bx, const T* by, const T* bz, T* invd, bool split, hipStream_t st);
template <typename T>
void launch_coarsen_level(const Level& F, const T* fbx, const T* fby, const T* fbz, const Level& C, T* cbx,
                          T* cby, T* cbz, T* invd, bool split, hipStream_t st);
template <typename T>
void launch_fill(T* a, size_t n, hipStream_t st);
// the line tables tx, ty, tz of the face arrays bx, by, bz of a level with extents n
template <typename T>
void launch_face_tables(const Dims& n, const T* bx, const T* by, const T* bz, T* tx, T* ty, T* tz, hipStream_t st);
// whether the library turns the line tables on for a finest level of extents n
bool face_tables_pay(const Dims& n);
template <typename T>
void launch_vcycle_tail(const TailDesc<T>& D, size_t lds_bytes, hipStream_t st);
void launch_d2f(const double* a, float* b, size_t n, hipStream_t st);
void launch_f2d(const float* a, double* b, size_t n, hipStream_t st);
// the V-cycle's last kernel (its FP64 result z in natural order) fused with
// the flexible CG's two products (r z, r z_old): per-block partials, two per
// block; each returns the block count
template <typename T>
int launch_gs_last_dots(const Level& L, const T* bx, const T* by, const T* bz, const T* b, const T* e,
                        double* nat, const double* r, const double* zold, double* partials, hipStream_t st);
// the finest level's first kernel of an FP32 cycle reading its natural b in
// FP64 (the CG residual), rounded as it is read
void launch_gs_first_nat64(const Level& L, const float* bx, const float* by, const float* bz, const double* b,
                           const float* invd, float* e, float* bs, hipStream_t st, float* bcopy = nullptr,
                           bool red_out = true);
int launch_f2d_dots(const float* a, double* z, size_t n, const double* r, const double* zold, double* partials,
                    hipStream_t st);

int cg_blocks(const Dims& n);
void launch_resid_norm(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                       const double* b, const double* x, double* r, const CgScratch& cs, int mode,
                       hipStream_t st, const FaceTab<double>& ft = FaceTab<double>{});
void launch_dot_rho(const Dims& n, const double* r, const double* z, const CgScratch& cs, hipStream_t st);
// beta and rho from two-valued partials already in cs.partials
void launch_finalize_beta(const CgScratch& cs, int nparts, hipStream_t st);
void launch_dots_beta(const Dims& n, const double* r, const double* zn, const double* z,
                      const CgScratch& cs, hipStream_t st);
// d = z + beta d_old and q = A d; with x, also the previous iteration's
// pending x += alpha d_old
void launch_dir_spmv(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                     const double* zn, const double* dold, double* dnew, double* q, int first,
                     const CgScratch& cs, hipStream_t st, KTimer* kt = nullptr, double* x = nullptr,
                     const FaceTab<double>& ft = FaceTab<double>{});
// r -= alpha q and ||r||^2; x += alpha d is left pending
void launch_cg_update(const Dims& n, const double* q, double* r, const CgScratch& cs, hipStream_t st);
// the pending x += alpha d
void launch_x_update(const Dims& n, const double* d, double* x, const CgScratch& cs, hipStream_t st);
void launch_apply_A(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                    const double* x, double* y, hipStream_t st);

// learned guess (ns_net.hip)
void net_features(ns_net* N, const Dims& n, double h, double rho_w, double rho_a, double P0, const double* b,
                  const double* rho, const double* pprev, const double* Ap, float* feat, hipStream_t st);
int net_matches(const ns_net* N, const Dims& n);
double* net_pprev(ns_net* N);
double* net_Ap(ns_net* N);
float* net_feat(ns_net* N);
int net_guess(ns_net* N, double P0, double* p, hipStream_t st, hipEvent_t done = nullptr);
void net_target(long nv, const double* p, const double* pprev, double P0, float* t, hipStream_t st);

}  // namespace nsk
