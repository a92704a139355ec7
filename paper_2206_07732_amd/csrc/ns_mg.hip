// Multigrid (red-black Gauss-Seidel V-cycle) and conjugate-gradient kernels
// for the pressure projection on gfx950.
//
// Operator on a level with spacing h (walls carry beta = 0, so every cell
// sums all six faces; the open top face couples to the ghost -x_c):
//   (A x)_c = (1/h^2) [ sum_f beta_f (x_c - x_nb) + 2 beta_top x_c (top row) ]
// V-cycle kernels are templated on the arithmetic type (double or float);
// the CG vectors and their reductions are always FP64.
//
// Launch count, not bandwidth, limits the small levels, so the schedule fuses
// what the algorithm allows:
//   * the first pre-smoothing pass (red from a zero guess) and the black pass
//     after it are one kernel: the red values h^2 b / D are recomputed by
//     the black cells from b and 1/D;
//   * prolongation and the first post-smoothing (black) pass are one kernel:
//     the black cells read their red neighbours plus the parent correction,
//     and the red cells are left for the red pass that follows, which
//     overwrites them without reading them;
//   * all levels from about a thousand cells down run in one workgroup out of
//     LDS;
//   * the direction update d = z + beta d is folded into the operator
//     application, which carries q = A d by its recurrence A z + beta q;
//     every CG reduction ends in one fixed-order pass over the per-block
//     partials, so results are bitwise reproducible.
#include <hip/hip_ext.h>

#include "ns_internal.h"

namespace nsk {

namespace {

struct Geo {
  dim3 grid, block;
};

inline Geo geo3(int mx, int my, int mz) {
  dim3 b = (my >= 4) ? dim3(64, 4, 1) : dim3(64, 1, 4);
  return {dim3((mx + 63) / 64, (my + b.y - 1) / b.y, (mz + b.z - 1) / b.z), b};
}

// sum_f beta_f (x_c - x_nb) + top term, without the 1/h^2 factor
template <typename T>
__device__ __forceinline__ T stencil(const Dims& n, const T* __restrict__ bx, const T* __restrict__ by,
                                     const T* __restrict__ bz, const T* __restrict__ x, int i, int j,
                                     int k, size_t c) {
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t fx = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fy = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  const T xc = x[c];
  const T xw = x[i > 0 ? c - 1 : c];
  const T xe = x[i < n.nx - 1 ? c + 1 : c];
  const T xs = x[j > 0 ? c - n.nx : c];
  const T xn = x[j < n.ny - 1 ? c + n.nx : c];
  const T xd = x[k > 0 ? c - sxy : c];
  const T xu = x[k < n.nz - 1 ? c + sxy : c];
  const T bu = bz[c + sxy];
  T acc = bx[fx] * (xc - xw) + bx[fx + 1] * (xc - xe) + by[fy] * (xc - xs) +
          by[fy + n.nx] * (xc - xn) + bz[c] * (xc - xd);
  acc += (k < n.nz - 1) ? bu * (xc - xu) : (T)2 * bu * xc;
  return acc;
}

// ------------------------------------------------------------ line tables
template <typename T>
struct TabBits;
template <>
struct TabBits<double> {
  using U = unsigned long long;
};
template <>
struct TabBits<float> {
  using U = unsigned;
};

// true with v the value every face of the line holds, where the table says
// so; else false (v = 0), also without a table.  With a line that is the
// same on every lane the entry is a scalar load, and a branch on the result
// a scalar branch.
template <typename T>
__device__ __forceinline__ bool line_val(const T* __restrict__ tab, int line, T& v) {
  using U = typename TabBits<T>::U;
  v = (T)0;
  if (tab == nullptr) return false;
  const T t = tab[line];
  if (__builtin_bit_cast(U, t) == ~U(0)) return false;
  v = t;
  return true;
}

// The six faces of one cell per lane, for a wavefront whose lanes share the
// cell's j and k (ju, ku: those values, the same on every lane; blockDim.x is
// 64): the x-line (j, k), the y-lines j and j + 1 and the z-lines k and k + 1
// of plane k, each taken from its table where the line is one value, else
// loaded.  load() issues the loads, under scalar branches, so that a
// wavefront on lines of one value issues none; get(), called after the
// caller's loads are all in flight (past its sched_barrier), picks the
// values, so no wait is placed between the loads.  TAB false: plain loads,
// no table code (the coarse levels' first-pass instance; their colour and
// prolongation passes keep the table code with null tables, see k_gs).
template <typename T, bool TAB = true>
struct FaceLd {
  T t[5];
  bool u[5];
  T l[6];
  // fx, fy: the x- and y-face index of the cell's west and south faces; fz:
  // its down face (the cell's natural index)
  __device__ __forceinline__ void load(const Dims& n, const FaceTab<T>& ft, const T* __restrict__ bx,
                                       const T* __restrict__ by, const T* __restrict__ bz, int ju, int ku,
                                       size_t fx, size_t fy, size_t fz) {
    if constexpr (!TAB) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        u[q] = false;
        t[q] = (T)0;
      }
      l[0] = bx[fx];
      l[1] = bx[fx + 1];
      l[2] = by[fy];
      l[3] = by[fy + n.nx];
      l[4] = bz[fz];
      l[5] = bz[fz + (size_t)n.nx * n.ny];
      return;
    }
    u[0] = line_val(ft.x, ju + n.ny * ku, t[0]);
    u[1] = line_val(ft.y, ju + (n.ny + 1) * ku, t[1]);
    u[2] = line_val(ft.y, ju + 1 + (n.ny + 1) * ku, t[2]);
    u[3] = line_val(ft.z, ju + n.ny * ku, t[3]);
    u[4] = line_val(ft.z, ju + n.ny * (ku + 1), t[4]);
    // a face of a one-value line is left unset (get() never reads it):
    // zeroing it on that side of the branch made the compiler wait there,
    // in some instances, for every load in flight
    if (!u[0]) {
      l[0] = bx[fx];
      l[1] = bx[fx + 1];
    }
    if (!u[1]) l[2] = by[fy];
    if (!u[2]) l[3] = by[fy + n.nx];
    if (!u[3]) l[4] = bz[fz];
    if (!u[4]) l[5] = bz[fz + (size_t)n.nx * n.ny];
  }
  // the faces of the lane's cell, in column i (a line of one value has zero
  // wall faces)
  __device__ __forceinline__ void get(const Dims& n, int i, T& bw, T& be, T& bs, T& bn, T& bd, T& bu) const {
    bw = u[0] ? (i > 0 ? t[0] : (T)0) : l[0];
    be = u[0] ? (i < n.nx - 1 ? t[0] : (T)0) : l[1];
    bs = u[1] ? t[1] : l[2];
    bn = u[2] ? t[2] : l[3];
    bd = u[3] ? t[3] : l[4];
    bu = u[4] ? t[4] : l[5];
  }
};

// the line tables of a level's three face arrays in one launch, a
// wavefront per line: lines [0, lx) of bx ((nx + 1) faces each, walls first
// and last, which must be zero), then [lx, lx + ly) of by and the rest of bz
// (nx faces each); the comparison is of bit patterns, so a line of equal
// values is exactly one value
template <typename T>
__global__ void __launch_bounds__(256) k_face_table(Dims n, const T* __restrict__ bx, const T* __restrict__ by,
                                                    const T* __restrict__ bz, T* __restrict__ tx,
                                                    T* __restrict__ ty, T* __restrict__ tz) {
  using U = typename TabBits<T>::U;
  const int lx = n.ny * n.nz, ly = (n.ny + 1) * n.nz, lz = n.ny * (n.nz + 1);
  int line = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (line >= lx + ly + lz) return;
  const bool xw = line < lx;
  const T* a = bx;
  T* tab = tx;
  if (!xw) {
    line -= lx;
    a = by;
    tab = ty;
    if (line >= ly) {
      line -= ly;
      a = bz;
      tab = tz;
    }
  }
  const int len = xw ? n.nx + 1 : n.nx;
  const T* p = a + (size_t)line * len;
  const int lo = xw ? 1 : 0, hi = xw ? len - 1 : len;
  const U v = lo < hi ? __builtin_bit_cast(U, p[lo]) : U(0);
  bool same = true;
  for (int i = lo + lane; i < hi; i += 64) same &= __builtin_bit_cast(U, p[i]) == v;
  if (xw && lane == 0) same &= __builtin_bit_cast(U, p[0]) == U(0) && __builtin_bit_cast(U, p[len - 1]) == U(0);
  const bool all = __all(same);
  if (lane == 0) tab[line] = __builtin_bit_cast(T, all ? v : ~U(0));
}

// --------------------------------------------------------------- reductions
__device__ __forceinline__ int block_tid() {
  return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}

// sum NV values over the block; the totals end in thread 0 (fixed tree)
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_down(v[q], off, 64);
  __shared__ double sm[16][NV];
  const int tid = block_tid();
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) >> 6;
  if ((tid & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sm[tid >> 6][q] = v[q];
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sm[w][q];
      v[q] = s;
    }
  }
  __syncthreads();
}

// write the block's NV sums to partials[NV * slot + q] (thread 0); slot is
// the block's tile index, so the partials lie in tile order
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ partials, int slot) {
  block_sum<NV>(v);
  if (block_tid() == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[NV * (size_t)slot + q] = v[q];
  }
}

// --------------------------------------------------------------- smoothers
// Levels above the coarse-level tail keep b, e and 1/D colour-split: cell
// (i, j, k) of colour c = (i + j + k) & 1 lives at c P + p with the pair index
// p = (i >> 1) + hx (j + ny k), hx = ceil(nx / 2), P = hx ny nz.  A colour pass
// then reads and writes only its own colour's entries (and the other
// colour's as neighbours), instead of whole lines of both.  The face
// coefficients stay in their natural layout.
struct SplitGeo {
  int hx;
  size_t P;
};
__host__ __device__ inline SplitGeo split_geo(const Dims& n) {
  const int hx = (n.nx + 1) >> 1;
  return SplitGeo{hx, (size_t)hx * n.ny * n.nz};
}
__device__ __forceinline__ size_t sidx(const Dims& n, const SplitGeo& g, int i, int j, int k) {
  return (size_t)((i + j + k) & 1) * g.P + (size_t)(i >> 1) + (size_t)g.hx * (j + (size_t)n.ny * k);
}
// index of cell (i, j, k) of a level's correction, split or natural
__device__ __forceinline__ size_t lidx(const Dims& n, const SplitGeo& g, bool split, int i, int j, int k) {
  return split ? sidx(n, g, i, j, k) : (size_t)i + (size_t)n.nx * (j + (size_t)n.ny * k);
}

// Threads own cell pairs (2ti, 2ti+1) of a row; the red cell of the pair is
// 2ti + ((j+k) & 1), the black one the other; pos is the pair index.
// (a 64 x bdy x bdz = 256-thread block of geo3; bdz is derived, since
// reading blockDim.y and .z together made the compiler fetch both in one
// misaligned vector load, waited on before any other load)
#define PAIR_INDEX                                                        \
  const Tile tl = xcd_tile();                                             \
  const int bdy = blockDim.y, bdz = 4 / bdy;                              \
  const int ti = tl.x * 64 + threadIdx.x;                                 \
  const int j = tl.y * bdy + threadIdx.y;                                 \
  const int k = tl.z * bdz + threadIdx.z;                                 \
  if (j >= n.ny || k >= n.nz) return;                                     \
  const SplitGeo sg = split_geo(n);                                       \
  if (ti >= sg.hx) return;                                                \
  const size_t sxy = (size_t)n.nx * n.ny;                                 \
  const size_t row = (size_t)n.nx * j + sxy * k;                          \
  const size_t pos = (size_t)ti + (size_t)sg.hx * (j + (size_t)n.ny * k)

// Gauss-Seidel value of cell (i, j, k) with pair index pos: (h^2 b + sum over
// non-wall faces of beta_f x_nb) / D, the neighbour values o(q) taken from the
// other colour at the neighbours' pair indices.  Wall terms are dropped by
// selects and every load goes through an in-range index (a wall neighbour
// through the cell's own pair index), so all of a thread's loads are in
// flight together and a 0 * garbage product never enters a sum.
// The loads of that value (faces; y and z neighbours), gathered apart from
// its arithmetic so that a kernel can issue them with its other loads,
// before anything waits on one.
template <typename T>
struct GsIn {
  T bw, be, bs, bn, bd, bu;   // faces: west, east, south, north, down, up
  T vs, vn, vd, vu;           // neighbour values: south, north, down, up
};
template <typename T, typename O>
__device__ __forceinline__ GsIn<T> gs_gather(const Dims& n, const SplitGeo& sg, const T* __restrict__ bx,
                                             const T* __restrict__ by, const T* __restrict__ bz, int i, int j,
                                             int k, size_t pos, O o) {
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t c = i + (size_t)n.nx * j + sxy * k;
  const size_t fx = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fy = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  const bool top = (k == n.nz - 1);
  const bool S = j > 0, N = j < n.ny - 1, D = k > 0;
  const size_t sz = (size_t)sg.hx * n.ny;
  const size_t ps = S ? pos - sg.hx : pos, pn = N ? pos + sg.hx : pos;
  const size_t pd = D ? pos - sz : pos, pu = top ? pos : pos + sz;
  return GsIn<T>{bx[fx], bx[fx + 1], by[fy], by[fy + n.nx], bz[c], bz[c + sxy], o(ps), o(pn), o(pd), o(pu)};
}
// the neighbour values of gs_gather alone (the faces left zero, for a
// FaceLd to fill)
template <typename T, typename O>
__device__ __forceinline__ GsIn<T> gs_gather_nb(const Dims& n, const SplitGeo& sg, int j, int k, size_t pos, O o) {
  const bool top = (k == n.nz - 1);
  const bool S = j > 0, N = j < n.ny - 1, D = k > 0;
  const size_t sz = (size_t)sg.hx * n.ny;
  const size_t ps = S ? pos - sg.hx : pos, pn = N ? pos + sg.hx : pos;
  const size_t pd = D ? pos - sz : pos, pu = top ? pos : pos + sz;
  return GsIn<T>{(T)0, (T)0, (T)0, (T)0, (T)0, (T)0, o(ps), o(pn), o(pd), o(pu)};
}
template <typename T>
__device__ __forceinline__ T gs_combine(const Dims& n, const GsIn<T>& g, T h2, T bc, int i, int j, int k, T vw,
                                        T ve) {
  const bool top = (k == n.nz - 1);
  const bool W = i > 0, E = i < n.nx - 1, S = j > 0, N = j < n.ny - 1, D = k > 0;
  const T diag = g.bw + g.be + g.bs + g.bn + g.bd + (top ? (T)2 * g.bu : g.bu);
  const T num = h2 * bc + (W ? g.bw * vw : (T)0) + (E ? g.be * ve : (T)0) + (S ? g.bs * g.vs : (T)0) +
                (N ? g.bn * g.vn : (T)0) + (D ? g.bd * g.vd : (T)0) + (top ? (T)0 : g.bu * g.vu);
  return num / diag;
}
template <typename T, typename O>
__device__ __forceinline__ T gs_split_value_x(const Dims& n, const SplitGeo& sg, T h2, const T* __restrict__ bx,
                                             const T* __restrict__ by, const T* __restrict__ bz, T bc, int i,
                                             int j, int k, size_t pos, T vw, T ve, O o) {
  return gs_combine<T>(n, gs_gather<T>(n, sg, bx, by, bz, i, j, k, pos, o), h2, bc, i, j, k, vw, ve);
}

// the same with the x neighbours loaded: cell i - 1 is in pair (i - 1) >> 1,
// cell i + 1 in pair (i + 1) >> 1
template <typename T, typename O>
__device__ __forceinline__ T gs_split_value(const Dims& n, const SplitGeo& sg, T h2, const T* __restrict__ bx,
                                           const T* __restrict__ by, const T* __restrict__ bz, T bc, int i, int j,
                                           int k, size_t pos, O o) {
  const bool W = i > 0, E = i < n.nx - 1;
  const size_t pw = W ? pos - (size_t)((i & 1) ? 0 : 1) : pos;
  const size_t pe = E ? pos + (size_t)((i & 1) ? 1 : 0) : pos;
  return gs_split_value_x<T>(n, sg, h2, bx, by, bz, bc, i, j, k, pos, o(pw), o(pe), o);
}

// one colour of Gauss-Seidel on colour-split b, e (FINE: finest-level
// instance, own symbol).  With nat set (the last pass of the finest level's
// V-cycle) the pair is written, both colours, to nat in natural order
// instead of back into e.
// NZ (gs_planes: two on the finest level in FP32, else one): planes per
// thread.  A pass over a level whose line tables spare most face loads is
// bound by its loads' latency, a block living about one memory round trip: a
// thread taking two planes k, k + 1 (its loads all issued before it waits on
// one) halves the rounds of blocks.  On 512x256x256 that took the FP32
// colour pass from 108 to 84 us and the prolongation pass from 128 to 123;
// the FP64 ones, which move twice the bytes, stayed at 154 us and went from
// 198 to 206, and keep one plane.
template <typename T>
constexpr int gs_planes(bool fine) { return fine && sizeof(T) == 4 ? 2 : 1; }
// The pass's body: TAB, the instance with line-table code (the finest
// level's, and the first coarse level's where it has tables); NZ planes per
// thread.
template <typename T, bool TAB, int NZ>
__device__ __forceinline__ void gs_body(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                        const T* __restrict__ bz, const T* __restrict__ b, T* __restrict__ e,
                                        int colour, T* __restrict__ nat, FaceTab<T> ft) {
  // the block is 64 x by x bz = 256 threads (geo3); blockDim.z is derived,
  // since reading blockDim.y and .z together made the compiler fetch both in
  // one misaligned vector load, waited on before any other load
  const Tile tl = xcd_tile();
  const int bdy = blockDim.y, bdz = 4 / bdy;
  const int tix = tl.x * 64 + threadIdx.x;
  const int j = tl.y * bdy + threadIdx.y;
  const int k0 = (tl.z * bdz + threadIdx.z) * NZ;
  if (j >= n.ny || k0 >= n.nz) return;
  const SplitGeo sg = split_geo(n);
  // a lane past the row's end works on its last pair and stores nothing:
  // returning it early made the compiler put the other lanes' loads under
  // that branch, past the barrier
  const bool tlive = tix < sg.hx;
  const int ti = tlive ? tix : sg.hx - 1;
  const T* eo = e + (size_t)(1 - colour) * sg.P;
  const auto o = [&](size_t q) { return eo[q]; };
  if constexpr (NZ == 1) {
    // One plane: written out.  In the per-plane form below the compiler
    // moved this case's loads past the barrier, a second memory round trip
    // per wavefront (the FP64 pass 153 -> 158 us on 512x256x256).
    if (!tlive) return;
    const int k = k0;
    const int par = (j + k + colour) & 1;
    const int i = 2 * ti + par, io = 2 * ti + 1 - par;
    const size_t pos = (size_t)ti + (size_t)sg.hx * (j + (size_t)n.ny * k);
    const size_t row = (size_t)n.nx * j + (size_t)n.nx * n.ny * k;
    // a cell past the row's end gathers through the row's last cell and stores nothing
    const int ic = i < n.nx ? i : n.nx - 1;
    const bool W = ic > 0, E = ic < n.nx - 1;
    const size_t pw = W ? pos - (size_t)((ic & 1) ? 0 : 1) : pos;
    const size_t pe = E ? pos + (size_t)((ic & 1) ? 1 : 0) : pos;
    GsIn<T> g = gs_gather_nb<T>(n, sg, j, k, pos, o);
    const T vw = o(pw), ve = o(pe), bc = b[(size_t)colour * sg.P + pos];
    FaceLd<T, TAB> F;
    F.load(n, ft, bx, by, bz, __builtin_amdgcn_readfirstlane(j), __builtin_amdgcn_readfirstlane(k),
           ic + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k), ic + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k),
           row + ic);
    __builtin_amdgcn_sched_barrier(0);
    F.get(n, ic, g.bw, g.be, g.bs, g.bn, g.bd, g.bu);
    if (i < n.nx) {
      const T v = gs_combine<T>(n, g, h2, bc, i, j, k, vw, ve);
      if (nat)
        nat[row + i] = v;
      else
        e[(size_t)colour * sg.P + pos] = v;
    }
    if (nat && io < n.nx) nat[row + io] = eo[pos];
    return;
  }
  // per plane: a plane past the grid's top repeats the last one and stores
  // nothing; a cell past the row's end gathers through the row's last cell
  // and stores nothing
  int kq[NZ], iq[NZ], icq[NZ];
  size_t posq[NZ], rowq[NZ];
  GsIn<T> g[NZ];
  T vw[NZ], ve[NZ], bc[NZ];
  FaceLd<T, TAB> F[NZ];
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    const int k = min(k0 + q, n.nz - 1);
    const int par = (j + k + colour) & 1;
    const int i = 2 * ti + par, ic = i < n.nx ? i : n.nx - 1;
    const size_t pos = (size_t)ti + (size_t)sg.hx * (j + (size_t)n.ny * k);
    const size_t row = (size_t)n.nx * j + (size_t)n.nx * n.ny * k;
    const bool W = ic > 0, E = ic < n.nx - 1;
    const size_t pw = W ? pos - (size_t)((ic & 1) ? 0 : 1) : pos;
    const size_t pe = E ? pos + (size_t)((ic & 1) ? 1 : 0) : pos;
    // the faces' branches first, then the plain loads: issued before the
    // branches, these were moved past the barrier (to their uses) by the
    // compiler, a second memory round trip per wavefront
    F[q].load(n, ft, bx, by, bz, __builtin_amdgcn_readfirstlane(j), __builtin_amdgcn_readfirstlane(k),
              ic + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k), ic + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k),
              row + ic);
    g[q] = gs_gather_nb<T>(n, sg, j, k, pos, o);
    vw[q] = o(pw);
    ve[q] = o(pe);
    bc[q] = b[(size_t)colour * sg.P + pos];
    kq[q] = k;
    iq[q] = i;
    icq[q] = ic;
    posq[q] = pos;
    rowq[q] = row;
  }
  __builtin_amdgcn_sched_barrier(0);
  // every value is formed (a repeated plane's or a clamped cell's too) and
  // only the stores are guarded: a value formed under the guard let the
  // compiler sink its loads past the barrier, into the guarded block
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    F[q].get(n, icq[q], g[q].bw, g[q].be, g[q].bs, g[q].bn, g[q].bd, g[q].bu);
    const int i = iq[q], io = 2 * ti + 1 - (i & 1);
    const T v = gs_combine<T>(n, g[q], h2, bc[q], icq[q], j, kq[q], vw[q], ve[q]);
    const bool live = tlive && k0 + q < n.nz;
    if (live && i < n.nx) {
      if (nat)
        nat[rowq[q] + i] = v;
      else
        e[(size_t)colour * sg.P + posq[q]] = v;
    }
    if (live && nat && io < n.nx) nat[rowq[q] + io] = eo[posq[q]];
  }
}

// one colour pass (FINE: the finest level's instance, its own symbol).  The
// coarse instance keeps the table code's shape with no tables: with plain
// face loads the compiler moved all its loads past the barrier.
template <typename T, bool FINE>
__global__ void __launch_bounds__(256) k_gs(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                            const T* __restrict__ bz, const T* __restrict__ b, T* __restrict__ e,
                                            int colour, T* __restrict__ nat, FaceTab<T> ft) {
  gs_body<T, true, gs_planes<T>(FINE)>(n, h2, bx, by, bz, b, e, colour, nat, ft);
}

// the same on the first coarse level where it has line tables (own symbol)
template <typename T>
__global__ void __launch_bounds__(256) k_gs_c1(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                               const T* __restrict__ bz, const T* __restrict__ b, T* __restrict__ e,
                                               int colour, T* __restrict__ nat, FaceTab<T> ft) {
  gs_body<T, true, gs_planes<T>(true)>(n, h2, bx, by, bz, b, e, colour, nat, ft);
}

// The last red pass of the finest level, writing the V-cycle's result z in
// natural order and in FP64 (as k_gs with nat; an FP32 cycle's values are
// widened exactly), fused with the two products the flexible CG needs next:
// per block, sum over its cells of r z and r z_old, red cell then black cell
// of each pair, in tile order.  Every thread reaches the block reduction (no
// early return).
template <typename T>
__global__ void __launch_bounds__(256) k_gs_last_dots(Dims n, T h2, const T* __restrict__ bx,
                                                      const T* __restrict__ by, const T* __restrict__ bz,
                                                      const T* __restrict__ b, const T* __restrict__ e,
                                                      double* __restrict__ nat, const double* __restrict__ r,
                                                      const double* __restrict__ zold,
                                                      double* __restrict__ partials, FaceTab<T> ft) {
  const Tile tl = xcd_tile();
  const int ti = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  const SplitGeo sg = split_geo(n);
  double v[2] = {0.0, 0.0};
  const bool live = j < n.ny && k < n.nz && ti < sg.hx;
  const size_t pos = live ? (size_t)ti + (size_t)sg.hx * (j + (size_t)n.ny * k) : 0;
  const T* eo = e + sg.P;   // the black plane
  // This pair's black value.  The red cell's x neighbours are this pair's
  // black cell and the adjacent pair's, which the adjacent lane holds (a
  // wavefront is 64 consecutive pairs of one row); every lane takes part in
  // the shuffles, and only a row's end lanes load their neighbour.  Every
  // load is issued before the shuffles wait for eb, through in-range indices
  // (a lane outside the grid, or a red cell past the row's end, reads cells
  // of the grid and stores nothing).
  const int par = (j + k) & 1;
  const int i = 2 * ti + par, io = 2 * ti + 1 - par;
  const int jj = live ? j : 0, kk = live ? k : 0;
  const int ir = live ? min(i, n.nx - 1) : 0, iq = live ? min(io, n.nx - 1) : 0;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t row = (size_t)n.nx * jj + sxy * kk;
  const int lane = threadIdx.x;
  const T eb = eo[pos];
  GsIn<T> g = gs_gather_nb<T>(n, sg, jj, kk, pos, [&](size_t q) { return eo[q]; });
  FaceLd<T> F;   // the wavefront's lines (j, k), clamped into the grid for a wavefront outside it
  F.load(n, ft, bx, by, bz, __builtin_amdgcn_readfirstlane(min(j, n.ny - 1)),
         __builtin_amdgcn_readfirstlane(min(k, n.nz - 1)), ir + (size_t)(n.nx + 1) * (jj + (size_t)n.ny * kk),
         ir + (size_t)n.nx * (jj + (size_t)(n.ny + 1) * kk), row + ir);
  const T bc = b[pos];
  T ex = 0;   // the row-end lanes' x neighbour from outside the wavefront
  if (live && lane == 0 && par == 0 && ir > 0) ex = eo[pos - 1];
  if (live && lane == 63 && par == 1 && ir < n.nx - 1) ex = eo[pos + 1];
  const double rr = r[row + ir], zr = zold[row + ir], rq = r[row + iq], zq = zold[row + iq];
  __builtin_amdgcn_sched_barrier(0);
  F.get(n, ir, g.bw, g.be, g.bs, g.bn, g.bd, g.bu);
  const T ebl = __shfl_up(eb, 1, 64), ebr = __shfl_down(eb, 1, 64);
  // formed on every lane from in-grid values, then kept by selects: a use
  // under a branch would let the compiler sink r's and z_old's loads past
  // the shuffles
  T vw = eb, ve = eb;   // par 1: west is this pair's black; par 0: east is
  if (par == 0 && ir > 0) vw = lane > 0 ? ebl : ex;
  if (par == 1 && ir < n.nx - 1) ve = lane < 63 ? ebr : ex;
  const double z = (double)gs_combine<T>(n, g, h2, bc, ir, jj, kk, vw, ve), zb = (double)eb;
  const bool red_ok = live && i < n.nx, black_ok = live && io < n.nx;
  if (red_ok) nat[row + i] = z;
  if (black_ok) nat[row + io] = zb;
  v[0] = (red_ok ? rr * z : 0.0) + (black_ok ? rq * zb : 0.0);
  v[1] = (red_ok ? rr * zr : 0.0) + (black_ok ? rq * zq : 0.0);
  block_partials<2>(v, partials, tl.lin);
}

// red pass from a zero guess followed by the black pass, in one launch: the
// red values the black cells need are recomputed from b and 1/D.  NAT: b is
// read in natural order (the finest level, whose b is a CG vector) and its
// colour-split copy is written to bs for the later passes; a natural b may
// be FP64 under an FP32 cycle (TB = double), rounded to T as it is read.
template <typename T, bool TAB, bool NAT, typename TB>
__device__ __forceinline__ void gs_first_body(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                              const T* __restrict__ bz, const TB* __restrict__ b,
                                              const T* __restrict__ invd, T* __restrict__ e, T* __restrict__ bs,
                                              T* __restrict__ bcopy, FaceTab<T> ft, int red_out) {
  static_assert(NAT || sizeof(TB) == sizeof(T), "a colour-split b has the cycle's type");
  PAIR_INDEX;
  const int par = (j + k) & 1;
  const int ir = 2 * ti + par, ib = 2 * ti + 1 - par;
  const size_t sz = (size_t)sg.hx * n.ny;
  // b of the cell (ii, jj, kk) of colour c with pair index q, as stored (an
  // FP64 b is rounded to T after the loads: rounded as it arrived, each
  // conversion waited for its load)
  auto bval = [&](int c, size_t q, int ii, int jj, int kk) -> TB {
    if constexpr (NAT)
      return b[(size_t)ii + (size_t)n.nx * jj + sxy * kk];
    else
      return b[(size_t)c * sg.P + q];
  };
  // This pair's red value h2 b / D, formed also where the red cell lies past
  // the row's end (b clamped into the row, an unused 1/D entry), since the
  // adjacent lane reads it: the black cell's x neighbours are this pair's red
  // cell and the adjacent pair's (a wavefront is 64 consecutive pairs of one
  // row), and only a row's end lanes load theirs.  Every load is issued
  // before the shuffles wait for that value; a black cell past the row's end
  // gathers through the row's last cell and stores nothing.
  const int lane = threadIdx.x;
  const int irc = ir < n.nx ? ir : n.nx - 1, ibc = ib < n.nx ? ib : n.nx - 1;
  const TB br0 = bval(0, pos, irc, j, k);
  const T idr = invd[pos];
  const TB bb0 = bval(1, pos, ibc, j, k);
  // the red neighbours' b and 1/D through in-range indices (walls: own pair)
  const bool W = ibc > 0, E = ibc < n.nx - 1, S = j > 0, N = j < n.ny - 1, D = k > 0, U = k < n.nz - 1;
  const size_t ps = S ? pos - sg.hx : pos, pn = N ? pos + sg.hx : pos, pd = D ? pos - sz : pos, pu = U ? pos + sz : pos;
  const int js = S ? j - 1 : j, jn = N ? j + 1 : j;
  const int kd = D ? k - 1 : k, ku = U ? k + 1 : k;
  const TB bS0 = bval(0, ps, ibc, js, k), bN0 = bval(0, pn, ibc, jn, k);
  const T iS = invd[ps], iN = invd[pn];
  const TB bD0 = bval(0, pd, ibc, j, kd), bU0 = bval(0, pu, ibc, j, ku);
  const T iD = invd[pd], iU = invd[pu];
  TB bX0 = 0;   // lane 63's east or lane 0's west red neighbour, outside the wavefront
  T iX = 0;
  const bool xe = lane == 63 && par == 0 && E, xw = lane == 0 && par == 1 && W;
  if (xe || xw) {   // one block of loads: two made the second wait for the first's
    const int dx = xe ? 1 : -1;
    bX0 = bval(0, pos + dx, ibc + dx, j, k);
    iX = invd[pos + dx];
  }
  const size_t c = row + ibc;
  const size_t fx = ibc + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fy = ibc + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  FaceLd<T, TAB> F;
  F.load(n, ft, bx, by, bz, __builtin_amdgcn_readfirstlane(j), __builtin_amdgcn_readfirstlane(k), fx, fy, c);
  __builtin_amdgcn_sched_barrier(0);
  T bw, be, bsy, bn, bd, bu;
  F.get(n, ibc, bw, be, bsy, bn, bd, bu);
  const T br = (T)br0, bb = (T)bb0, bS = (T)bS0, bN = (T)bN0, bD = (T)bD0, bU = (T)bU0, bX = (T)bX0;
  const T rv = h2 * br * idr;
  if (ir < n.nx) {
    // the red values are not stored where the next pass is a red one, which
    // overwrites them without reading them
    if (red_out) e[pos] = rv;
    if constexpr (NAT) bs[pos] = br;
  }
  const T rl = __shfl_up(rv, 1, 64), rr = __shfl_down(rv, 1, 64);
  if (ib >= n.nx) return;
  if constexpr (NAT) bs[sg.P + pos] = bb;
  T vw = rv, ve = rv;   // par 0: west is this pair's red cell; par 1: east is
  if (par == 0 && E) ve = lane < 63 ? rr : h2 * bX * iX;
  if (par == 1 && W) vw = lane > 0 ? rl : h2 * bX * iX;
  const T vs = h2 * bS * iS, vn = h2 * bN * iN, vd = h2 * bD * iD, vu = h2 * bU * iU;
  const bool top = !U;
  const T diag = bw + be + bsy + bn + bd + (top ? (T)2 * bu : bu);
  const T num = h2 * bb + (W ? bw * vw : (T)0) + (E ? be * ve : (T)0) + (S ? bsy * vs : (T)0) +
                (N ? bn * vn : (T)0) + (D ? bd * vd : (T)0) + (top ? (T)0 : bu * vu);
  const T vb = num / diag;
  e[sg.P + pos] = vb;
  if (bcopy) bcopy[pos] = vb;   // the black plane as a fused red-black pass will read it
}

// (FINE: the finest level's instance, its own symbol)
template <typename T, bool FINE, bool NAT, typename TB = T>
__global__ void __launch_bounds__(256) k_gs_first(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                                  const T* __restrict__ bz, const TB* __restrict__ b,
                                                  const T* __restrict__ invd, T* __restrict__ e, T* __restrict__ bs,
                                                  T* __restrict__ bcopy, FaceTab<T> ft, int red_out) {
  gs_first_body<T, FINE, NAT, TB>(n, h2, bx, by, bz, b, invd, e, bs, bcopy, ft, red_out);
}

// the same on the first coarse level where it has line tables (own symbol)
template <typename T>
__global__ void __launch_bounds__(256) k_gs_first_c1(Dims n, T h2, const T* __restrict__ bx,
                                                     const T* __restrict__ by, const T* __restrict__ bz,
                                                     const T* __restrict__ b, const T* __restrict__ invd,
                                                     T* __restrict__ e, T* __restrict__ bs, T* __restrict__ bcopy,
                                                     FaceTab<T> ft, int red_out) {
  gs_first_body<T, true, false, T>(n, h2, bx, by, bz, b, invd, e, bs, bcopy, ft, red_out);
}

// prolongation e += P ec followed by the black pass, in one launch; only the
// black cells are written (the red pass that follows overwrites the red ones
// without reading them).  ec is the next level's correction, colour-split
// (csplit) or natural (a tail level).
template <typename T, bool TAB, int NZ>
__device__ __forceinline__ void gs_prolong_body(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                                const T* __restrict__ bz, const T* __restrict__ b,
                                                T* __restrict__ e, Dims nc, int sxc, int syc, int szc, int csplit,
                                                const T* __restrict__ ec, T* __restrict__ bcopy, FaceTab<T> ft) {
  // NZ planes per thread, as in k_gs
  // the block is 64 x by x bz = 256 threads (geo3); blockDim.z is derived,
  // since reading blockDim.y and .z together made the compiler fetch both in
  // one misaligned vector load, waited on before any other load
  const Tile tl = xcd_tile();
  const int bdy = blockDim.y, bdz = 4 / bdy;
  const int tix = tl.x * 64 + threadIdx.x;
  const int j = tl.y * bdy + threadIdx.y;
  const int k0 = (tl.z * bdz + threadIdx.z) * NZ;
  if (j >= n.ny || k0 >= n.nz) return;
  const SplitGeo sg = split_geo(n);
  // a lane past the row's end works on its last pair and stores nothing:
  // returning it early made the compiler put the other lanes' loads under
  // that branch, past the barrier
  const bool tlive = tix < sg.hx;
  const int ti = tlive ? tix : sg.hx - 1;
  // the parent's entry in 32-bit arithmetic (a level's arrays have fewer
  // than 2^31 entries; six of these per thread dominated its instruction count)
  const int chx = (nc.nx + 1) >> 1, cP = chx * nc.ny * nc.nz;
  auto cidx = [&](int ii, int jj, int kk) {
    const int I = ii >> sxc, J = jj >> syc, K = kk >> szc;
    return csplit ? ((I + J + K) & 1) * cP + (I >> 1) + chx * (J + nc.ny * K) : I + nc.nx * (J + nc.ny * K);
  };
  const size_t sz = (size_t)sg.hx * n.ny, sxy = (size_t)n.nx * n.ny;
  // per plane (a plane past the grid's top repeats the last one, and a black
  // cell past the row's end its row's last cell; neither is stored): the red
  // neighbours' values and their parents' corrections, the faces and b,
  // every load before the first wait.  The indices are all formed first:
  // interleaved with the loads, the compiler's 32-bit multiply-adds read a
  // register pair whose upper half was a load's destination, and waited.
  T ev[NZ][6], qv[NZ][6], bcell[NZ];
  int iq[NZ], kq[NZ], qi[NZ][6];
  size_t posq[NZ], en[NZ][6], fxq[NZ], fyq[NZ], cq[NZ];
  FaceLd<T, TAB> F[NZ];
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    const int k = min(k0 + q, n.nz - 1);
    const int ib = 2 * ti + 1 - ((j + k) & 1);   // the black cell
    const int i = ib < n.nx ? ib : n.nx - 1;
    const size_t pos = (size_t)ti + (size_t)sg.hx * (j + (size_t)n.ny * k);
    const bool W = i > 0, E = i < n.nx - 1, S = j > 0, N = j < n.ny - 1, D = k > 0, U = k < n.nz - 1;
    en[q][0] = W ? pos - (size_t)((i & 1) ? 0 : 1) : pos;
    en[q][1] = E ? pos + (size_t)((i & 1) ? 1 : 0) : pos;
    en[q][2] = S ? pos - sg.hx : pos;
    en[q][3] = N ? pos + sg.hx : pos;
    en[q][4] = D ? pos - sz : pos;
    en[q][5] = U ? pos + sz : pos;
    qi[q][0] = cidx(W ? i - 1 : i, j, k);
    qi[q][1] = cidx(E ? i + 1 : i, j, k);
    qi[q][2] = cidx(i, S ? j - 1 : j, k);
    qi[q][3] = cidx(i, N ? j + 1 : j, k);
    qi[q][4] = cidx(i, j, D ? k - 1 : k);
    qi[q][5] = cidx(i, j, U ? k + 1 : k);
    cq[q] = (size_t)n.nx * j + sxy * k + i;
    fxq[q] = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
    fyq[q] = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
    iq[q] = ib;
    kq[q] = k;
    posq[q] = pos;
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
#pragma unroll
    for (int d = 0; d < 6; ++d) ev[q][d] = e[en[q][d]];
#pragma unroll
    for (int d = 0; d < 6; ++d) qv[q][d] = ec[qi[q][d]];
    F[q].load(n, ft, bx, by, bz, __builtin_amdgcn_readfirstlane(j), __builtin_amdgcn_readfirstlane(kq[q]), fxq[q],
              fyq[q], cq[q]);
    bcell[q] = b[sg.P + posq[q]];
  }
  __builtin_amdgcn_sched_barrier(0);
  // every value formed, only the stores guarded (as in gs_body)
#pragma unroll
  for (int q = 0; q < NZ; ++q) {
    const int k = kq[q], i = min(iq[q], n.nx - 1);
    const bool W = i > 0, E = i < n.nx - 1, S = j > 0, N = j < n.ny - 1, D = k > 0, U = k < n.nz - 1;
    T bw, be, bs, bn, bd, bu;
    F[q].get(n, i, bw, be, bs, bn, bd, bu);
    const T vw = ev[q][0] + qv[q][0], ve = ev[q][1] + qv[q][1], vs = ev[q][2] + qv[q][2];
    const T vn = ev[q][3] + qv[q][3], vd = ev[q][4] + qv[q][4], vu = ev[q][5] + qv[q][5];
    const bool top = !U;
    const T diag = bw + be + bs + bn + bd + (top ? (T)2 * bu : bu);
    const T num = h2 * bcell[q] + (W ? bw * vw : (T)0) + (E ? be * ve : (T)0) + (S ? bs * vs : (T)0) +
                  (N ? bn * vn : (T)0) + (D ? bd * vd : (T)0) + (top ? (T)0 : bu * vu);
    const T vb = num / diag;
    if (tlive && k0 + q < n.nz && iq[q] < n.nx) {
      e[sg.P + posq[q]] = vb;
      if (bcopy) bcopy[posq[q]] = vb;   // the black plane as a fused red-black pass will read it
    }
  }
}

// (FINE: the finest level's instance, its own symbol; the coarse one keeps
// the table code's shape, as k_gs)
template <typename T, bool FINE>
__global__ void __launch_bounds__(256) k_gs_prolong(Dims n, T h2, const T* __restrict__ bx, const T* __restrict__ by,
                                                    const T* __restrict__ bz, const T* __restrict__ b,
                                                    T* __restrict__ e, Dims nc, int sxc, int syc, int szc, int csplit,
                                                    const T* __restrict__ ec, T* __restrict__ bcopy, FaceTab<T> ft) {
  gs_prolong_body<T, true, gs_planes<T>(FINE)>(n, h2, bx, by, bz, b, e, nc, sxc, syc, szc, csplit, ec, bcopy, ft);
}

// the same on the first coarse level where it has line tables (own symbol)
template <typename T>
__global__ void __launch_bounds__(256) k_gs_prolong_c1(Dims n, T h2, const T* __restrict__ bx,
                                                       const T* __restrict__ by, const T* __restrict__ bz,
                                                       const T* __restrict__ b, T* __restrict__ e, Dims nc, int sxc,
                                                       int syc, int szc, int csplit, const T* __restrict__ ec,
                                                       T* __restrict__ bcopy, FaceTab<T> ft) {
  gs_prolong_body<T, true, gs_planes<T>(true)>(n, h2, bx, by, bz, b, e, nc, sxc, syc, szc, csplit, ec, bcopy, ft);
}

// A red pass then a black pass of Gauss-Seidel in one launch, on a level
// whose rows are at most 32 pairs (ceil(nx/2) <= 32), where launch latency,
// not bytes, bounds a pass.  A block takes whole rows: TY rows by TZ planes
// of pairs (TX >= ceil(nx/2) lanes per row).  It forms the red values of its
// tile and of a ring one row wide in y and z around it (the red cells its
// black cells read) from the black plane as it stood before the launch,
// which the previous kernel copied to bold (this launch overwrites the
// black plane while other blocks still read it).  It then forms its black
// values from those red values, held in LDS.  Each value comes from the same
// arithmetic, on the same inputs, as in the two separate passes, so the
// results are theirs bit for bit.  Every global load of a thread is issued
// before it waits on any.
constexpr int kRbThreads = 256;
constexpr int kRbMaxIter = 3;   // ring-extended tile entries per thread
constexpr int kRbMaxExt = kRbThreads * kRbMaxIter;

template <typename T>
__global__ void __launch_bounds__(kRbThreads) k_gs_rb(Dims n, T h2, const T* __restrict__ bx,
                                                      const T* __restrict__ by, const T* __restrict__ bz,
                                                      const T* __restrict__ b, T* __restrict__ e,
                                                      const T* __restrict__ bold, int TX, int TY, int TZ) {
  __shared__ T R[kRbMaxExt];
  const SplitGeo sg = split_geo(n);
  const Tile tl = xcd_tile_flat();
  const int ty0 = tl.y * TY, tz0 = tl.z * TZ;
  const int ry = n.ny > 1 ? 1 : 0;   // ring width in y (none in a 2-D tank)
  const int EY = TY + 2 * ry, NE = TX * EY * (TZ + 2);
  const int t = threadIdx.x;
  const size_t sxy = (size_t)n.nx * n.ny;
  auto ob = [&](size_t q) { return bold[q]; };
  // red entries of the ring-extended tile: entry q is pair q % TX of row
  // (ty0 + ey - ry, tz0 + ez - 1); an entry outside the grid gathers through
  // red cell (parity, 0, 0) and is stored as 0
  GsIn<T> gr[kRbMaxIter];
  T br[kRbMaxIter], rw[kRbMaxIter], re[kRbMaxIter];
  int ri[kRbMaxIter], rj[kRbMaxIter], rk[kRbMaxIter];
  size_t rp[kRbMaxIter];
  bool rok[kRbMaxIter];
#pragma unroll
  for (int u = 0; u < kRbMaxIter; ++u) {
    const int q = t + u * kRbThreads;
    const int ex = q % TX, ey = (q / TX) % EY, ez = q / (TX * EY);
    const int j = ty0 + ey - ry, k = tz0 + ez - 1;
    const int i = 2 * ex + ((j + k) & 1);
    rok[u] = q < NE && j >= 0 && j < n.ny && k >= 0 && k < n.nz && i < n.nx;
    rj[u] = rok[u] ? j : 0;
    rk[u] = rok[u] ? k : 0;
    ri[u] = rok[u] ? i : 0;
    rp[u] = (size_t)(ri[u] >> 1) + (size_t)sg.hx * (rj[u] + (size_t)n.ny * rk[u]);
    gr[u] = gs_gather<T>(n, sg, bx, by, bz, ri[u], rj[u], rk[u], rp[u], ob);
    br[u] = b[rp[u]];
    const bool W = ri[u] > 0, E = ri[u] < n.nx - 1;
    rw[u] = bold[W ? rp[u] - (size_t)((ri[u] & 1) ? 0 : 1) : rp[u]];
    re[u] = bold[E ? rp[u] + (size_t)((ri[u] & 1) ? 1 : 0) : rp[u]];
  }
  // this thread's black cell: pair px of row (ty0 + py, tz0 + pz); the tile
  // has exactly kRbThreads cells (TX TY TZ = kRbThreads), so pz < TZ
  const int px = t % TX, py = (t / TX) % TY, pz = t / (TX * TY);
  const int jb = ty0 + py, kb = tz0 + pz;
  const int ib = 2 * px + 1 - ((jb + kb) & 1);
  const bool bok = jb < n.ny && kb < n.nz && ib < n.nx;
  const int jc = bok ? jb : 0, kc = bok ? kb : 0, ic = bok ? ib : 1;
  const size_t pb = (size_t)(ic >> 1) + (size_t)sg.hx * (jc + (size_t)n.ny * kc);
  const size_t cb = ic + (size_t)n.nx * jc + sxy * kc;
  const size_t fxb = ic + (size_t)(n.nx + 1) * (jc + (size_t)n.ny * kc);
  const size_t fyb = ic + (size_t)n.nx * (jc + (size_t)(n.ny + 1) * kc);
  const T bw = bx[fxb], be = bx[fxb + 1], bs = by[fyb], bn = by[fyb + n.nx], bd = bz[cb], bu = bz[cb + sxy];
  const T bb = b[sg.P + pb];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kRbMaxIter; ++u) {
    const int q = t + u * kRbThreads;
    if (q < NE) {
      T v = (T)0;
      if (rok[u]) {
        v = gs_combine<T>(n, gr[u], h2, br[u], ri[u], rj[u], rk[u], rw[u], re[u]);
        const int ey = (q / TX) % EY, ez = q / (TX * EY);
        if (ey >= ry && ey < ry + TY && ez >= 1 && ez <= TZ) e[rp[u]] = v;
      }
      R[q] = v;
    }
  }
  __syncthreads();
  if (bok) {
    const int ey = py + ry, ez = pz + 1;
    const int row = TX * (ey + EY * ez);
    const int L = px + row;
    const bool W = ib > 0, E = ib < n.nx - 1, S = jb > 0, N = jb < n.ny - 1, D = kb > 0, U = kb < n.nz - 1;
    const T vw = R[W ? ((ib - 1) >> 1) + row : L], ve = R[E ? ((ib + 1) >> 1) + row : L];
    const GsIn<T> g{bw, be, bs, bn, bd, bu, R[S ? L - TX : L], R[N ? L + TX : L], R[D ? L - TX * EY : L],
                    R[U ? L + TX * EY : L]};
    e[sg.P + pb] = gs_combine<T>(n, g, h2, bb, ib, jb, kb, vw, ve);
  }
}

// A red pass then a black pass of Gauss-Seidel in one launch on the finest
// level, reading each face coefficient once.  Every face borders one red and
// one black cell, so the black update takes its six coefficients from the
// red updates beside it instead of loading them again:
//   * its z-faces are the down face of the red cell above it and the up face
//     of the red cell below it, both in the same pair column, which the same
//     thread computes on the planes above and below;
//   * its x-faces are the faces of the red cell of its own pair and of the
//     adjacent pair (the adjacent lane: a row of the block is one wave of 64
//     consecutive pairs; the end lanes load their outer face);
//   * its y-faces are those of the red cells of the rows beside it (LDS).
// A block marches up a chunk of KZ planes: at plane m it forms the red
// values of plane m, then the black values of plane m - 1, whose red
// neighbours are then all known.  Its 64 lanes by TY + 2 rows of pairs store
// every lane of the TY inner rows; the first and last rows form a ring whose
// red values the block's own black cells read.  One more wave, the halo,
// forms for each inner row the red values of the two pairs just beyond the
// row's ends (lanes 0 .. TY - 1 the west pair, 32 .. 31 + TY the east one),
// which the end lanes' black cells read from LDS.  Ring and halo values are
// recomputed (the neighbouring block forms and stores them too).  Red values
// are formed from the black plane as it stood before the launch, which the
// previous kernel copied to bold (this launch overwrites the black plane
// while other blocks still read it).  Each value comes from the same
// arithmetic on the same inputs as in the two separate passes, so the
// results are theirs bit for bit.
//
// The march is bound by memory latency, not bandwidth: a plane's work is a
// few dozen instructions per thread against one trip to HBM.  So every load
// of a plane is issued, unconditionally from clamped addresses, before the
// planes below it are computed, and waits only at its first use: one plane
// ahead in FP64, two in FP32, whose planes carry half the bytes each (with
// one plane in flight the FP32 march moved 3.2 TB/s, the FP64 one 4.3; a
// second FP64 plane would not fit the 128 registers a 1024-thread block
// allows).  The loop is unrolled by the depth so that the planes' registers
// rotate without copies.
constexpr int kRbfLanes = 64;
template <typename T>
constexpr int rbf_depth() { return sizeof(T) == 4 ? 3 : 2; }

template <typename T>
struct RbfLoads {
  T fw, fe, fs, fn, fd, fu;  // the faces of the red cell of plane m
  T bc;                      // its right-hand side
  T bo_u;                    // this pair's black value (before the launch) on plane m + 1
  T xo, yo;                  // black values beside the row ends and the ring rows on plane m
  T bb;                      // the right-hand side of this pair's black cell on plane m - 1
  T xf;                      // that cell's outer x-face, for a row's end lanes
};

// what a halo lane loads for the red cell of its pair on plane m
template <typename T>
struct RbfHaloLoads {
  T fw, fe, fs, fn, fd, fu, bc;
  T own, xo;   // black values (before the launch) of its pair and of the x-adjacent pair
  T ys, yn;    // of the rows beside it
  T zd, zu;    // of the planes below and above
};

template <typename T, int TY>
__global__ void __launch_bounds__(kRbfLanes * (TY + 3)) k_gs_rb_fine(Dims n, T h2, const T* __restrict__ bx,
                                                                     const T* __restrict__ by,
                                                                     const T* __restrict__ bz,
                                                                     const T* __restrict__ b, T* __restrict__ e,
                                                                     const T* __restrict__ bold, int KZ) {
  constexpr int R = TY + 2;
  static_assert(TY <= 32, "a halo lane per inner row and side");
  // One barrier per plane, between its red and black phases.  A wave may
  // then form the red values of plane m + 1 while another still reads those
  // of plane m - 1 in its black phase, so the red values, their y-faces and
  // the halo's values take three slots (plane mod 3); the black values
  // before the launch need two, since their readers (the red phase) all
  // finish before the barrier.
  __shared__ T BO[2][R][kRbfLanes];    // black values (as before the launch) of a plane
  __shared__ T RN[3][R][kRbfLanes];    // red values of a plane
  __shared__ T RYS[3][R][kRbfLanes];   // their south and north faces
  __shared__ T RYN[3][R][kRbfLanes];
  __shared__ T HH[3][2][R];            // the halo's red values: [plane mod 3][west, east][row]
  const SplitGeo sg = split_geo(n);
  const Tile tl = xcd_tile_flat();
  const int lane = threadIdx.x, r = threadIdx.y;
  const bool halo = r == R;            // the halo wave (wave-uniform)
  const int tx0 = tl.x * kRbfLanes;    // this block's first pair of a row
  const int k0 = tl.z * KZ, kz1 = min(k0 + KZ, n.nz);
  const size_t sz = (size_t)sg.hx * n.ny;   // pairs per plane
  const size_t fxs = (size_t)(n.nx + 1) * n.ny, fys = (size_t)n.nx * (n.ny + 1), fzs = (size_t)n.nx * n.ny;
  const auto clampz = [&](int m) { return (size_t)min(max(m, 0), n.nz - 1); };
  // ---- a main lane: pair ti of row j
  const int ti = tx0 + lane, j = tl.y * TY - 1 + r;
  const bool ok = !halo && ti < sg.hx && j >= 0 && j < n.ny;
  const bool inner = ok && r >= 1 && r <= TY;
  const int tic = min(ti, sg.hx - 1), jc = min(max(j, 0), n.ny - 1);
  const size_t prow = (size_t)tic + (size_t)sg.hx * jc;   // this pair in plane 0
  // the pairs whose black values the row ends and the ring rows read
  const size_t xrow = (size_t)(lane == 0 ? max(tic - 1, 0) : lane == kRbfLanes - 1 ? min(tic + 1, sg.hx - 1) : tic) +
                      (size_t)sg.hx * jc;
  const size_t yrow = (size_t)tic + (size_t)sg.hx * (r == 0 ? max(jc - 1, 0) : r == R - 1 ? min(jc + 1, n.ny - 1) : jc);
  // the outer x-face of a black cell on a row's end lane: the west face of
  // an even column on lane 0, the east face of an odd one on lane 63 (a
  // shuffle there would return the lane's own face)
  const int xfi = lane == 0 ? 2 * ti : 2 * ti + 2;
  // ---- a halo lane: the pair beyond the west (side 0) or east (side 1) row end, inner row hr
  const int side = lane >> 5, hr = (lane & 31) + 1;
  const int hp = side ? tx0 + kRbfLanes : tx0 - 1, hj = tl.y * TY - 1 + hr;
  const bool hok = halo && hr <= TY && hp >= 0 && hp < sg.hx && hj < n.ny;
  const int hpc = min(max(hp, 0), sg.hx - 1), hjc = min(hj, n.ny - 1);
  // face indices from the unclamped cell, kept in the face range: a ring
  // cell outside the grid holds the wall face it shares with the grid; at
  // m = -1 the up face is the bed, at m = nz the down face is the open top
  const auto load = [&](int m, RbfLoads<T>& L) {
    const size_t mc = clampz(m);
    const int iru = 2 * ti + ((j + m) & 1);
    const int irc = min(max(iru, 0), n.nx - 1);
    const size_t xf = (size_t)(n.nx + 1) * jc + fxs * mc;
    L.fw = bx[(size_t)min(max(iru, 0), n.nx) + xf];
    L.fe = bx[(size_t)min(max(iru + 1, 0), n.nx) + xf];
    L.fs = by[(size_t)irc + (size_t)n.nx * min(max(j, 0), n.ny) + fys * mc];
    L.fn = by[(size_t)irc + (size_t)n.nx * min(max(j + 1, 0), n.ny) + fys * mc];
    L.fd = bz[(size_t)irc + (size_t)n.nx * jc + fzs * (size_t)min(max(m, 0), n.nz)];
    L.fu = bz[(size_t)irc + (size_t)n.nx * jc + fzs * (size_t)min(max(m + 1, 0), n.nz)];
    L.bc = b[prow + sz * mc];
    L.bo_u = bold[prow + sz * clampz(m + 1)];
    L.xo = bold[xrow + sz * mc];
    L.yo = bold[yrow + sz * mc];
    L.bb = b[sg.P + prow + sz * clampz(m - 1)];
    L.xf = bx[(size_t)min(max(xfi, 0), n.nx) + (size_t)(n.nx + 1) * jc + fxs * clampz(m - 1)];
  };
  const auto load_h = [&](int m, RbfHaloLoads<T>& H) {
    const size_t mc = clampz(m);
    const int par = (hj + m) & 1;
    const int iru = 2 * hp + par;
    const int irc = min(max(iru, 0), n.nx - 1);
    const size_t xf = (size_t)(n.nx + 1) * hjc + fxs * mc;
    const size_t pr = (size_t)hpc + (size_t)sg.hx * hjc;
    H.fw = bx[(size_t)min(max(iru, 0), n.nx) + xf];
    H.fe = bx[(size_t)min(max(iru + 1, 0), n.nx) + xf];
    H.fs = by[(size_t)irc + (size_t)n.nx * hjc + fys * mc];
    H.fn = by[(size_t)irc + (size_t)n.nx * (hjc + 1) + fys * mc];
    H.fd = bz[(size_t)irc + (size_t)n.nx * hjc + fzs * mc];
    H.fu = bz[(size_t)irc + (size_t)n.nx * hjc + fzs * (mc + 1)];
    H.bc = b[pr + sz * mc];
    H.own = bold[pr + sz * mc];
    H.xo = bold[(size_t)min(max(par ? hpc + 1 : hpc - 1, 0), sg.hx - 1) + (size_t)sg.hx * hjc + sz * mc];
    H.ys = bold[(size_t)hpc + (size_t)sg.hx * max(hjc - 1, 0) + sz * mc];
    H.yn = bold[(size_t)hpc + (size_t)sg.hx * min(hjc + 1, n.ny - 1) + sz * mc];
    H.zd = bold[pr + sz * clampz(m - 1)];
    H.zu = bold[pr + sz * clampz(m + 1)];
  };
  T bo_d = bold[prow + sz * clampz(k0 - 2)], bo_c = bold[prow + sz * clampz(k0 - 1)];
  if (!(ok && k0 - 2 >= 0)) bo_d = (T)0;
  if (!(ok && k0 - 1 >= 0)) bo_c = (T)0;
  T rv1 = 0, rv2 = 0, fu1 = 0, fu2 = 0, fw1 = 0, fe1 = 0;
  // the halo wave's plane: the red value of its pair on plane m, to LDS
  const auto plane_h = [&](int m, const RbfHaloLoads<T>& H) {
    const int par = (hj + m) & 1;
    const int iru = 2 * hp + par;
    T rv = (T)0;
    if (hok && m >= 0 && m < n.nz && iru < n.nx) {
      const int mc = m;
      const T vw = par == 0 ? H.xo : H.own, ve = par == 0 ? H.own : H.xo;
      const T vd = m > 0 ? H.zd : (T)0, vu = m + 1 < n.nz ? H.zu : (T)0;
      const GsIn<T> g{H.fw, H.fe, H.fs, H.fn, H.fd, H.fu, H.ys, H.yn, vd, vu};
      rv = gs_combine<T>(n, g, h2, H.bc, iru, hj, mc, vw, ve);
    }
    if (hr <= TY) HH[(m + 3) % 3][side][hr] = rv;
    __syncthreads();
  };
  const auto plane = [&](int m, const RbfLoads<T>& L) {
    // ---- the red cell of this pair on plane m (ring rows included)
    const int mc = (int)clampz(m);
    const int par = (j + m) & 1;
    const int iru = 2 * ti + par;                     // possibly outside the grid
    const int irc = min(max(iru, 0), n.nx - 1);
    const bool live = ok && m >= 0 && m < n.nz;
    const T bo_u = (ok && m + 1 >= 0 && m + 1 < n.nz) ? L.bo_u : (T)0;
    // x neighbours: this pair's black cell and the adjacent pair's (the
    // adjacent lane; the row's end lanes loaded theirs)
    const T bl = __shfl_up(bo_c, 1, kRbfLanes), br = __shfl_down(bo_c, 1, kRbfLanes);
    const T xo = live ? L.xo : (T)0, yo = live ? L.yo : (T)0;
    const T vw = par == 0 ? (lane > 0 ? bl : xo) : bo_c;
    const T ve = par == 1 ? (lane < kRbfLanes - 1 ? br : xo) : bo_c;
    const T vs = r > 0 ? BO[m & 1][r - 1][lane] : yo;
    const T vn = r < R - 1 ? BO[m & 1][r + 1][lane] : yo;
    T rv = (T)0;
    if (live && iru < n.nx) {
      const GsIn<T> g{L.fw, L.fe, L.fs, L.fn, L.fd, L.fu, vs, vn, bo_d, bo_u};
      rv = gs_combine<T>(n, g, h2, L.bc, irc, jc, mc, vw, ve);
      if (inner && m >= k0 && m < kz1) e[prow + sz * mc] = rv;
    }
    const int sm = (m + 3) % 3, sb = (m + 2) % 3;   // the slots of planes m and m - 1
    RN[sm][r][lane] = rv;
    RYS[sm][r][lane] = L.fs;
    RYN[sm][r][lane] = L.fn;
    BO[(m + 1) & 1][r][lane] = bo_u;
    // the adjacent lanes' red values and x-faces of plane m - 1 (every lane
    // takes part in the shuffles)
    const T xfe = __shfl_up(fe1, 1, kRbfLanes), xrl = __shfl_up(rv1, 1, kRbfLanes);
    const T xfw = __shfl_down(fw1, 1, kRbfLanes), xrr = __shfl_down(rv1, 1, kRbfLanes);
    __syncthreads();
    // ---- the black cell of this pair on plane m - 1 (inner threads)
    const int mb = m - 1;
    if (inner && mb >= k0 && mb < kz1) {
      const int ib = iru;      // the black cell of plane m - 1 shares the column of plane m's red cell
      if (ib < n.nx) {
        const bool even = (ib & 1) == 0;
        const T bw = lane > 0 ? xfe : L.xf, be = lane < kRbfLanes - 1 ? xfw : L.xf;
        const T vwb = lane > 0 ? xrl : HH[sb][0][r], veb = lane < kRbfLanes - 1 ? xrr : HH[sb][1][r];
        const GsIn<T> g{even ? bw : fe1, even ? fw1 : be, RYN[sb][r - 1][lane], RYS[sb][r + 1][lane],
                        fu2, L.fd, RN[sb][r - 1][lane], RN[sb][r + 1][lane], rv2, rv};
        const T bb = L.bb;
        e[sg.P + prow + sz * (size_t)mb] = gs_combine<T>(n, g, h2, bb, ib, j, mb, even ? vwb : rv1, even ? rv1 : veb);
      }
    }
    rv2 = rv1;
    rv1 = rv;
    fu2 = fu1;
    fu1 = L.fu;
    fw1 = L.fw;
    fe1 = L.fe;
    bo_d = bo_c;
    bo_c = bo_u;
  };
  // plane p's loads sit in buffer (p - k0 + 1) % D; the halo wave and the
  // main waves pass the same planes, so they meet the same barriers (the
  // two-deep form is written out: as the general loop it spilled in FP64)
  constexpr int D = rbf_depth<T>();
  if (halo) {
    if constexpr (D == 2) {
      RbfHaloLoads<T> A, B;
      load_h(k0 - 1, A);
      __syncthreads();
      for (int m = k0 - 1; m <= kz1; m += 2) {
        load_h(m + 1, B);
        __builtin_amdgcn_sched_barrier(0);
        plane_h(m, A);
        if (m + 1 > kz1) break;
        load_h(m + 2, A);
        __builtin_amdgcn_sched_barrier(0);
        plane_h(m + 1, B);
      }
    } else {
      RbfHaloLoads<T> H[D];
#pragma unroll
      for (int q = 0; q < D - 1; ++q) load_h(k0 - 1 + q, H[q]);
      __syncthreads();
      for (int m = k0 - 1; m <= kz1; m += D) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
          if (q > 0 && m + q > kz1) return;
          load_h(m + q + D - 1, H[(q + D - 1) % D]);
          __builtin_amdgcn_sched_barrier(0);
          plane_h(m + q, H[q]);
        }
      }
    }
    return;
  }
  if constexpr (D == 2) {
    RbfLoads<T> A, B;
    load(k0 - 1, A);
    BO[(k0 - 1) & 1][r][lane] = bo_c;
    __syncthreads();
    for (int m = k0 - 1; m <= kz1; m += 2) {
      load(m + 1, B);
      __builtin_amdgcn_sched_barrier(0);
      plane(m, A);
      if (m + 1 > kz1) break;
      load(m + 2, A);
      __builtin_amdgcn_sched_barrier(0);
      plane(m + 1, B);
    }
  } else {
    RbfLoads<T> A[D];
#pragma unroll
    for (int q = 0; q < D - 1; ++q) load(k0 - 1 + q, A[q]);
    BO[(k0 - 1) & 1][r][lane] = bo_c;
    __syncthreads();
    for (int m = k0 - 1; m <= kz1; m += D) {
#pragma unroll
      for (int q = 0; q < D; ++q) {
        if (q > 0 && m + q > kz1) return;
        load(m + q + D - 1, A[(q + D - 1) % D]);
        __builtin_amdgcn_sched_barrier(0);
        plane(m + q, A[q]);
      }
    }
  }
}

// the residual b - A x of one cell from its value, its neighbours' (a wall
// neighbour given as the cell's own value) and its six faces; up: the cell
// is below the top row (else the open top's ghost term 2 beta_top x_c)
template <typename T>
__device__ __forceinline__ T cell_resid(T bcell, T ih2, T xc, T xw, T xe, T xs, T xn, T xd, T xu, T cw, T ce, T cs,
                                        T cn, T cd, T bu, bool up) {
  T acc = cw * (xc - xw) + ce * (xc - xe) + cs * (xc - xs) + cn * (xc - xn) + cd * (xc - xd);
  acc += up ? bu * (xc - xu) : (T)2 * bu * xc;
  return bcell - ih2 * acc;
}

// coarse rhs = mean over the children of the fine residual b - A e (fine b,
// e colour-split; the coarse b colour-split when csplit, else natural).  A
// block takes a tile of fine cells (32 x 4 x 2; 64 x 1 x 4 in 2-D), one
// thread per cell: each computes its cell's residual into LDS, then one
// thread per coarse cell of the tile sums its children from LDS in the
// order (dk, dj, di).  Tile extents are even, so a coarse cell's children
// never straddle two tiles.
template <typename T>
__global__ void __launch_bounds__(256) k_resid_restrict(Dims nf, int fx, int fy, int fz, T ih2,
                                                        const T* __restrict__ bx, const T* __restrict__ by,
                                                        const T* __restrict__ bz, const T* __restrict__ b,
                                                        const T* __restrict__ e, Dims nc, int csplit, T inv,
                                                        T* __restrict__ bc) {
  __shared__ T sr[256];
  const int TX = blockDim.x, TY = blockDim.y;
  const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
  const Tile tl = xcd_tile();
  const int i = tl.x * TX + tx, j = tl.y * TY + ty, k = tl.z * blockDim.z + tz;
  // Index arithmetic in 32 bits (every array of a level has fewer than 2^31
  // entries): the kernel issues more integer instructions than loads, and
  // 64-bit products cost several each.
  const int hx = (nf.nx + 1) >> 1, P = hx * nf.ny * nf.nz;
  const int sxy = nf.nx * nf.ny, sz = hx * nf.ny;
  T r = 0;
  if (i < nf.nx && j < nf.ny && k < nf.nz) {
    const int c = i + nf.nx * j + sxy * k;
    const int fxi = i + (nf.nx + 1) * (j + nf.ny * k);
    const int fyi = i + nf.nx * (j + (nf.ny + 1) * k);
    const int par = (i + j + k) & 1;
    const int rowp = hx * (j + nf.ny * k);          // first pair of the cell's row
    const int own = par * P + (i >> 1) + rowp;      // the cell's own entry
    const int oth = (1 - par) * P + rowp;           // the other colour's row (all six neighbours)
    const int pc = oth + (i >> 1);
    // walls read the cell's own entry, so their (x_c - x_nb) is zero
    const T xc = e[own];
    const T xw = e[i > 0 ? oth + ((i - 1) >> 1) : own];
    const T xe = e[i < nf.nx - 1 ? oth + ((i + 1) >> 1) : own];
    const T xs = e[j > 0 ? pc - hx : own];
    const T xn = e[j < nf.ny - 1 ? pc + hx : own];
    const T xd = e[k > 0 ? pc - sz : own];
    const T xu = e[k < nf.nz - 1 ? pc + sz : own];
    const T cw = bx[fxi], ce = bx[fxi + 1], cs = by[fyi], cn = by[fyi + nf.nx], cd = bz[c], bu = bz[c + sxy];
    const T bcell = b[own];
    // all loads above are in flight together: the compiler may not sink the
    // up neighbour's load into the branch that uses it
    __builtin_amdgcn_sched_barrier(0);
    r = cell_resid<T>(bcell, ih2, xc, xw, xe, xs, xn, xd, xu, cw, ce, cs, cn, cd, bu, k < nf.nz - 1);
  }
  const int t = (tz * TY + ty) * TX + tx;
  sr[t] = r;
  __syncthreads();
  // each coarse cell of the tile is summed by the thread of its corner child
  // (the factors are 1 or 2 and the tile's extents even, so shifts replace
  // divisions)
  const int sx = fx - 1, sy = fy - 1, sz2 = fz - 1;
  if ((tx & sx) | (ty & sy) | (tz & sz2)) return;
  const int CX = TX >> sx, CY = TY >> sy, CZ = (int)blockDim.z >> sz2;
  const int I = tl.x * CX + (tx >> sx), J = tl.y * CY + (ty >> sy), K = tl.z * CZ + (tz >> sz2);
  if (I >= nc.nx || J >= nc.ny || K >= nc.nz) return;
  T sum = 0;
  for (int dk = 0; dk < fz; ++dk)
    for (int dj = 0; dj < fy; ++dj)
      for (int di = 0; di < fx; ++di) sum += sr[((tz + dk) * TY + ty + dj) * TX + tx + di];
  const int chx = (nc.nx + 1) >> 1, cP = chx * nc.ny * nc.nz;
  const int ci = csplit ? ((I + J + K) & 1) * cP + (I >> 1) + chx * (J + nc.ny * K) : I + nc.nx * (J + nc.ny * K);
  bc[ci] = sum * inv;
}

// The same on a level whose extents are all even and which is halved in
// every direction, so that coarse cell (I, J, K) holds fine pair I of rows
// 2J, 2J + 1 and planes 2K, 2K + 1.  One thread per pair of cells: every
// load of a wave is 64 consecutive pairs of one colour, or the faces of one
// row (y and z faces as two-element vector loads), and a pair's x
// neighbours come from the adjacent lanes; a cell-per-thread tile issues
// half as many loads again, at stride two.  A block takes 64 pairs x 2 rows
// x 2 planes, the children of 64 coarse cells, and its first wave sums each
// coarse cell's eight residuals in k_resid_restrict's order (dk, dj, di), so
// the result is the same.
template <typename T>
__global__ void __launch_bounds__(256) k_resid_restrict_pairs(Dims nf, T ih2, const T* __restrict__ bx,
                                                              const T* __restrict__ by, const T* __restrict__ bz,
                                                              const T* __restrict__ b, const T* __restrict__ e,
                                                              Dims nc, int csplit, T inv, T* __restrict__ bc,
                                                              FaceTab<T> ft) {
  using T2 = T __attribute__((ext_vector_type(2)));
  __shared__ T sr[2][2][2][64];   // [dk][dj][di][lane]
  const Tile tl = xcd_tile();
  const int lane = threadIdx.x, dj = threadIdx.y, dk = threadIdx.z;
  const int hx = nf.nx >> 1;
  const int ti = tl.x * 64 + lane, j = 2 * tl.y + dj, k = 2 * tl.z + dk;
  const bool live = ti < hx;
  const int tc = live ? ti : hx - 1;   // lanes past the row's end work on its last pair and store nothing
  // 32-bit index arithmetic: every array of a level has fewer than 2^31 entries
  const int P = hx * nf.ny * nf.nz, sz = hx * nf.ny, sxy = nf.nx * nf.ny;
  const int pos = tc + hx * (j + nf.ny * k);
  const int par = (j + k) & 1;   // colour of the pair's first cell A (i = 2 tc); B is i = 2 tc + 1
  const int pa = par * P + pos, pb = (1 - par) * P + pos;
  const bool W = tc > 0, E = tc < hx - 1, S = j > 0, N = j < nf.ny - 1, D = k > 0, U = k < nf.nz - 1;
  // A's y and z neighbours have B's colour, and B's have A's; a wall
  // neighbour reads the cell's own entry
  const T xa = e[pa], xb = e[pb];
  const T xas = e[S ? pb - hx : pa], xan = e[N ? pb + hx : pa], xad = e[D ? pb - sz : pa], xau = e[U ? pb + sz : pa];
  const T xbs = e[S ? pa - hx : pb], xbn = e[N ? pa + hx : pb], xbd = e[D ? pa - sz : pb], xbu = e[U ? pa + sz : pb];
  // outside the wavefront: lane 0 loads A's west neighbour (B of the pair
  // before), lane 63 B's east one (A of the pair after)
  const T xo = e[lane == 0 ? (W ? pb - 1 : pa) : lane == 63 ? (E ? pa + 1 : pb) : pa];
  const int fx = 2 * tc + (nf.nx + 1) * (j + nf.ny * k);
  const int fy = 2 * tc + nf.nx * (j + (nf.ny + 1) * k);
  const int c = 2 * tc + nf.nx * j + sxy * k;
  // the faces: each line (the x-line j, k; y-lines j, j + 1; z-lines k, k + 1)
  // through its table where it is one value (the wavefront is one row), else
  // loaded under a scalar branch; picked after every load is in flight
  const int ju = __builtin_amdgcn_readfirstlane(j), ku = __builtin_amdgcn_readfirstlane(k);
  T tx, ts, tn, td, tu;
  const bool ux = line_val(ft.x, ju + nf.ny * ku, tx), us = line_val(ft.y, ju + (nf.ny + 1) * ku, ts);
  const bool un = line_val(ft.y, ju + 1 + (nf.ny + 1) * ku, tn), ud = line_val(ft.z, ju + nf.ny * ku, td);
  const bool uu = line_val(ft.z, ju + nf.ny * (ku + 1), tu);
  // A's west face; the face between A and B; B's east face, for lane 63.  A
  // face of a one-value line is left unset until it is taken from the
  // table below: zeroing it on that side of the branch made the FP32
  // instance wait there for every load in flight.
  T fwa, fab, feo;
  T2 fs, fn, fd, fu;
  if (!ux) {
    fwa = bx[fx];
    fab = bx[fx + 1];
    feo = bx[lane == 63 ? fx + 2 : fx];
  }
  if (!us) fs = *reinterpret_cast<const T2*>(by + fy);
  if (!un) fn = *reinterpret_cast<const T2*>(by + fy + nf.nx);
  if (!ud) fd = *reinterpret_cast<const T2*>(bz + c);
  if (!uu) fu = *reinterpret_cast<const T2*>(bz + c + sxy);
  const T ba = b[pa], bb = b[pb];
  __builtin_amdgcn_sched_barrier(0);
  if (ux) {   // walls: face 0 and face nx (nx is even, so 2 tc + 1 is inside)
    fwa = tc > 0 ? tx : (T)0;
    fab = tx;
    feo = 2 * tc + 2 < nf.nx ? tx : (T)0;
  }
  if (us) fs = T2{ts, ts};
  if (un) fn = T2{tn, tn};
  if (ud) fd = T2{td, td};
  if (uu) fu = T2{tu, tu};
  const T xbl = __shfl_up(xb, 1, 64), xar = __shfl_down(xa, 1, 64), fwr = __shfl_down(fwa, 1, 64);
  const T xaw = W ? (lane > 0 ? xbl : xo) : xa;
  const T xbe = E ? (lane < 63 ? xar : xo) : xb;
  const T feb = lane < 63 ? fwr : feo;
  sr[dk][dj][0][lane] = cell_resid<T>(ba, ih2, xa, xaw, xb, xas, xan, xad, xau, fwa, fab, fs.x, fn.x, fd.x, fu.x, U);
  sr[dk][dj][1][lane] = cell_resid<T>(bb, ih2, xb, xa, xbe, xbs, xbn, xbd, xbu, fab, feb, fs.y, fn.y, fd.y, fu.y, U);
  __syncthreads();
  if (dj | dk) return;
  T sum = 0;
#pragma unroll
  for (int qk = 0; qk < 2; ++qk)
#pragma unroll
    for (int qj = 0; qj < 2; ++qj)
#pragma unroll
      for (int qi = 0; qi < 2; ++qi) sum += sr[qk][qj][qi][lane];
  if (!live) return;
  const int I = ti, J = tl.y, K = tl.z;
  const int chx = (nc.nx + 1) >> 1, cP = chx * nc.ny * nc.nz;
  const int ci = csplit ? ((I + J + K) & 1) * cP + (I >> 1) + chx * (J + nc.ny * K) : I + nc.nx * (J + nc.ny * K);
  bc[ci] = sum * inv;
}

// colour-split fine correction += parent's coarse correction (nu_post == 0)
template <typename T>
__global__ void __launch_bounds__(256) k_prolong(Dims nf, int sx, int sy, int sz, T* __restrict__ e, Dims nc,
                                                 int csplit, const T* __restrict__ ec) {
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= nf.nx || j >= nf.ny || k >= nf.nz) return;
  const SplitGeo sg = split_geo(nf), cg = split_geo(nc);
  e[sidx(nf, sg, i, j, k)] += ec[lidx(nc, cg, csplit != 0, i >> sx, j >> sy, k >> sz)];
}

// natural <-> colour-split copies (the finest level's edge cases)
template <typename T>
__global__ void __launch_bounds__(256) k_split_copy(Dims n, const T* __restrict__ src, T* __restrict__ dst,
                                                    int to_split) {
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const SplitGeo sg = split_geo(n);
  const size_t c = i + (size_t)n.nx * (j + (size_t)n.ny * k), s = sidx(n, sg, i, j, k);
  if (to_split)
    dst[s] = src[c];
  else
    dst[c] = src[s];
}

// 1 / (sum of the cell's face coefficients, top face counted twice), stored
// colour-split (levels above the tail) or natural (tail levels)
template <typename T>
__global__ void __launch_bounds__(256) k_invdiag(Dims n, const T* __restrict__ bx, const T* __restrict__ by,
                                                 const T* __restrict__ bz, int split, T* __restrict__ invd) {
  const Tile tl = xcd_tile();
  const int i = tl.x * blockDim.x + threadIdx.x;
  const int j = tl.y * blockDim.y + threadIdx.y;
  const int k = tl.z * blockDim.z + threadIdx.z;
  if (i >= n.nx || j >= n.ny || k >= n.nz) return;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t c = i + (size_t)n.nx * j + sxy * k;
  const size_t fx = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fy = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  const T bu = bz[c + sxy];
  const T diag = bx[fx] + bx[fx + 1] + by[fy] + by[fy + n.nx] + bz[c] + (k == n.nz - 1 ? (T)2 * bu : bu);
  invd[lidx(n, split_geo(n), split != 0, i, j, k)] = (T)1 / diag;
}

// Coarse face coefficient of component C at coarse face (I, J, K): the mean
// of the fine faces covering it, summed in the order (dk, dj, di).
// (the coarsening factors fx, fy, fz are 1 or 2).  The candidate fine faces
// are loaded through indices clamped into the array (coarse_face_load), and
// those within the factors summed in the order (dk, dj, di)
// (coarse_face_sum); a kernel loads all six faces before it sums any, so
// that every load is in flight before the first wait.
template <typename T>
struct FaceIn {
  T v[2][2][2];   // [dk][dj][di]
};
template <typename T, int C>
__device__ __forceinline__ FaceIn<T> coarse_face_load(const Dims& nf, int fx, int fy, int fz,
                                                      const T* __restrict__ fb, int I, int J, int K) {
  const int fmx = nf.nx + (C == 0), fmy = nf.ny + (C == 1), fmz = nf.nz + (C == 2);
  FaceIn<T> f;
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const int i = min(I * fx + di, fmx - 1), j = min(J * fy + dj, fmy - 1), k = min(K * fz + dk, fmz - 1);
        f.v[dk][dj][di] = fb[i + (size_t)fmx * (j + (size_t)fmy * k)];
      }
  return f;
}
template <typename T, int C>
__device__ __forceinline__ T coarse_face_sum(int fx, int fy, int fz, const FaceIn<T>& f) {
  const int ni = (C == 0) ? 1 : fx, nj = (C == 1) ? 1 : fy, nk = (C == 2) ? 1 : fz;
  T sum = 0;
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di)
        if (dk < nk && dj < nj && di < ni) sum += f.v[dk][dj][di];
  return sum / (T)(ni * nj * nk);
}

// One coarse level of the hierarchy in one launch: each coarse cell forms its
// six face coefficients from the fine level, writes the faces it owns (its
// lower faces, and its upper ones on the grid's upper edges) and its 1/D
// (the sum of its faces, the top face twice, as in k_invdiag), colour-split
// (split) or natural.  A face shared by two cells is formed by both with the
// same arithmetic, and written once.
template <typename T>
__global__ void __launch_bounds__(256) k_coarsen_level(Dims nf, int fx, int fy, int fz, const T* __restrict__ fbx,
                                                       const T* __restrict__ fby, const T* __restrict__ fbz,
                                                       Dims nc, T* __restrict__ cbx, T* __restrict__ cby,
                                                       T* __restrict__ cbz, int split, T* __restrict__ invd) {
  const Tile tl = xcd_tile();
  const int I = tl.x * blockDim.x + threadIdx.x;
  const int J = tl.y * blockDim.y + threadIdx.y;
  const int K = tl.z * blockDim.z + threadIdx.z;
  if (I >= nc.nx || J >= nc.ny || K >= nc.nz) return;
  const FaceIn<T> fw = coarse_face_load<T, 0>(nf, fx, fy, fz, fbx, I, J, K);
  const FaceIn<T> fe = coarse_face_load<T, 0>(nf, fx, fy, fz, fbx, I + 1, J, K);
  const FaceIn<T> fs = coarse_face_load<T, 1>(nf, fx, fy, fz, fby, I, J, K);
  const FaceIn<T> fn = coarse_face_load<T, 1>(nf, fx, fy, fz, fby, I, J + 1, K);
  const FaceIn<T> fd = coarse_face_load<T, 2>(nf, fx, fy, fz, fbz, I, J, K);
  const FaceIn<T> fu = coarse_face_load<T, 2>(nf, fx, fy, fz, fbz, I, J, K + 1);
  // (the barrier keeps the compiler from sinking a load into the branch of
  // the sum that uses it)
  __builtin_amdgcn_sched_barrier(0);
  const T bw = coarse_face_sum<T, 0>(fx, fy, fz, fw), be = coarse_face_sum<T, 0>(fx, fy, fz, fe);
  const T bs = coarse_face_sum<T, 1>(fx, fy, fz, fs), bn = coarse_face_sum<T, 1>(fx, fy, fz, fn);
  const T bd = coarse_face_sum<T, 2>(fx, fy, fz, fd), bu = coarse_face_sum<T, 2>(fx, fy, fz, fu);
  const size_t fxi = I + (size_t)(nc.nx + 1) * (J + (size_t)nc.ny * K);
  const size_t fyi = I + (size_t)nc.nx * (J + (size_t)(nc.ny + 1) * K);
  const size_t c = I + (size_t)nc.nx * (J + (size_t)nc.ny * K);
  const size_t sxy = (size_t)nc.nx * nc.ny;
  cbx[fxi] = bw;
  if (I == nc.nx - 1) cbx[fxi + 1] = be;
  cby[fyi] = bs;
  if (J == nc.ny - 1) cby[fyi + nc.nx] = bn;
  cbz[c] = bd;
  if (K == nc.nz - 1) cbz[c + sxy] = bu;
  const T diag = bw + be + bs + bn + bd + (K == nc.nz - 1 ? (T)2 * bu : bu);
  invd[lidx(nc, split_geo(nc), split != 0, I, J, K)] = (T)1 / diag;
}

// ------------------------------------------------------- coarse-level tail
// Every level from the first tail level down to the coarsest runs in one
// workgroup with coefficients, 1/D, right-hand sides and corrections held in
// LDS, so a smoothing pass costs a barrier instead of a launch.  Levels whose
// cell pairs fit one wavefront run in wavefront 0 alone, ordered by
// wavefront-level fences instead of workgroup barriers.  Each thread decodes
// its cell pairs once per level visit, with every LDS index a pass of either
// colour needs, so that a pass is its loads and its arithmetic.
//
// Walls carry beta = 0 and every correction in LDS is finite (the tail zeroes
// them all before its first level), so a wall term beta_f e_nb is an exact
// zero and the passes add it unconditionally; only the open top face, whose
// coefficient is not zero, is dropped by a select.
struct TailCell {
  int c;          // cell index (b, e, 1/D, bz of the lower face)
  int fx, fy;     // west x-face and south y-face
  int w, e, s, n, d, u;   // neighbour cells; the cell itself through a wall or the top
  bool ok, top;   // the cell exists (i < nx); it lies in the top row
};
struct TailPairs {
  int ti[2], j[2], k[2];
  int np;
  TailCell cell[2][2];   // [pair][colour]: the pair's red cell, then its black one
};

// lanes 0..nthr-1 take pairs t and t + nthr
__device__ __forceinline__ void tail_decode(const Dims& n, int tid, int nthr, TailPairs& tp) {
  const int hx = (n.nx + 1) >> 1;
  const int NP = hx * n.ny * n.nz;
  const int sxy = n.nx * n.ny;
  tp.np = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int t = tid + q * nthr;
    if (t < NP) {
      tp.ti[q] = t % hx;
      const int r = t / hx;
      tp.j[q] = r % n.ny;
      tp.k[q] = r / n.ny;
      tp.np = q + 1;
      const int j = tp.j[q], k = tp.k[q];
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int i = 2 * tp.ti[q] + ((j + k + col) & 1);
        TailCell& x = tp.cell[q][col];
        x.ok = i < n.nx;
        x.top = k == n.nz - 1;
        x.c = i + n.nx * j + sxy * k;
        x.fx = i + (n.nx + 1) * (j + n.ny * k);
        x.fy = i + n.nx * (j + (n.ny + 1) * k);
        x.w = i > 0 ? x.c - 1 : x.c;
        x.e = i < n.nx - 1 ? x.c + 1 : x.c;
        x.s = j > 0 ? x.c - n.nx : x.c;
        x.n = j < n.ny - 1 ? x.c + n.nx : x.c;
        x.d = k > 0 ? x.c - sxy : x.c;
        x.u = x.top ? x.c : x.c + sxy;
      }
    }
  }
}

// ordering point between two phases: a workgroup barrier, or (WAVE) a
// wavefront-level fence for phases run by wavefront 0 alone
template <bool WAVE>
__device__ __forceinline__ void tail_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T, bool WAVE, int COLOUR>
__device__ __forceinline__ void tail_pass(const Dims& n, const TailPairs& tp, T h2, const T* bx, const T* by,
                                          const T* bz, const T* invd, const T* b, T* e, bool from_zero) {
  const int sxy = n.nx * n.ny;
#pragma unroll
  for (int q = 0; q < 2; ++q) {   // compile-time indices: the cells stay in registers
    if (q >= tp.np) break;
    const TailCell& x = tp.cell[q][COLOUR];
    if (x.ok) {
      const T id = invd[x.c], bc = b[x.c];
      if (from_zero) {
        e[x.c] = (h2 * bc) * id;
      } else {
        // every load is issued before the arithmetic starts (the scheduling
        // barrier keeps the compiler from interleaving them with the sums,
        // which would wait on each pair in turn); the up term is formed and
        // then selected, so that its loads do not sit behind a branch
        const T cw = bx[x.fx], ce = bx[x.fx + 1], cs = by[x.fy], cn = by[x.fy + n.nx];
        const T cd = bz[x.c], cu = bz[x.c + sxy];
        const T ew = e[x.w], ee = e[x.e], es = e[x.s], en = e[x.n], ed = e[x.d], eu = e[x.u];
        __builtin_amdgcn_sched_barrier(0);
        T num = h2 * bc;
        num += cw * ew;   // west, east, south, north, down, up
        num += ce * ee;
        num += cs * es;
        num += cn * en;
        num += cd * ed;
        const T with_up = num + cu * eu;
        num = x.top ? num : with_up;
        e[x.c] = num * id;
      }
    }
  }
  tail_sync<WAVE>();
}

// One level's share of the tail, run either by the whole workgroup or (WAVE)
// by wavefront 0 alone.
template <typename T, bool WAVE>
struct TailLevel {
  const TailDesc<T>& D;
  T* sm;
  int tid, nthr;

  template <int C0>
  __device__ void smooth_from(int l, const TailPairs& tp, int pairs, bool from_zero) const {
    const Dims n = D.n[l];
    const T *bx = sm + D.obx[l], *by = sm + D.oby[l], *bz = sm + D.obz[l], *b = sm + D.ob[l];
    const T* invd = sm + D.oid[l];
    T* e = sm + D.oe[l];
    const T h2 = D.h2[l];
    for (int s = 0; s < pairs; ++s) {
      tail_pass<T, WAVE, C0>(n, tp, h2, bx, by, bz, invd, b, e, from_zero && s == 0);
      tail_pass<T, WAVE, 1 - C0>(n, tp, h2, bx, by, bz, invd, b, e, false);
    }
  }

  // `pairs` (red, black) or (black, red) sweeps
  __device__ void smooth(int l, const TailPairs& tp, int first_colour, int pairs, bool from_zero) const {
    if (first_colour == 0)
      smooth_from<0>(l, tp, pairs, from_zero);
    else
      smooth_from<1>(l, tp, pairs, from_zero);
  }

  __device__ void zero(int l) const {
    const int N = D.n[l].nx * D.n[l].ny * D.n[l].nz;
    T* e = sm + D.oe[l];
    for (int c = tid; c < N; c += nthr) e[c] = (T)0;
    tail_sync<WAVE>();
  }

  // pre-smoothing, then the restricted residual into the next level's b
  __device__ void down(int l) const {
    TailPairs tp;
    tail_decode(D.n[l], tid, nthr, tp);
    if (D.nu_pre > 0) {
      // the red pass from zero writes the red cells without reading e; the
      // black pass after it reads them (and its own zeroed entries at walls)
      smooth(l, tp, 0, D.nu_pre, true);
    } else {
      zero(l);
    }
    const Dims nf = D.n[l], nc = D.n[l + 1];
    const int fx = D.f[l][0], fy = D.f[l][1], fz = D.f[l][2];
    const T *bx = sm + D.obx[l], *by = sm + D.oby[l], *bz = sm + D.obz[l], *b = sm + D.ob[l];
    const T* e = sm + D.oe[l];
    T* bc = sm + D.ob[l + 1];
    T* rs = sm + D.ors;   // scratch: the fine residual
    const T ih2 = (T)1 / D.h2[l];
    const T inv = (T)1 / (T)(fx * fy * fz);
    const int sxy = nf.nx * nf.ny;
    // every fine cell's residual b - A e, each thread for both cells of its
    // pairs (a wall term is an exact zero) ...
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= tp.np) break;
      // both cells' loads first (a cell past the row's end reads the
      // pair's other cell, and is not stored), then their sums
      T v[2][14];
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const TailCell& x = tp.cell[q][col];
        const int c = x.ok ? x.c : tp.cell[q][1 - col].c;
        const int w = x.ok ? x.w : c, ea = x.ok ? x.e : c, so = x.ok ? x.s : c, no = x.ok ? x.n : c;
        const int d = x.ok ? x.d : c, u = x.ok ? x.u : c;
        const int ix = x.ok ? x.fx : tp.cell[q][1 - col].fx, iy = x.ok ? x.fy : tp.cell[q][1 - col].fy;
        v[col][0] = e[c];
        v[col][1] = bx[ix];
        v[col][2] = bx[ix + 1];
        v[col][3] = by[iy];
        v[col][4] = by[iy + nf.nx];
        v[col][5] = bz[c];
        v[col][6] = bz[c + sxy];
        v[col][7] = e[w];
        v[col][8] = e[ea];
        v[col][9] = e[so];
        v[col][10] = e[no];
        v[col][11] = e[d];
        v[col][12] = e[u];
        v[col][13] = b[c];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const TailCell& x = tp.cell[q][col];
        const T* a = v[col];
        const T xc = a[0];
        T acc = 0;
        acc += a[1] * (xc - a[7]);    // west, east, south, north, down, up
        acc += a[2] * (xc - a[8]);
        acc += a[3] * (xc - a[9]);
        acc += a[4] * (xc - a[10]);
        acc += a[5] * (xc - a[11]);
        acc += x.top ? (T)2 * a[6] * xc : a[6] * (xc - a[12]);
        if (x.ok) rs[x.c] = a[13] - ih2 * acc;
      }
    }
    tail_sync<WAVE>();
    // ... then each coarse cell's mean of its children, summed in the order
    // (dk, dj, di) by the thread whose pair is the cell's (dj, dk) = (0, 0)
    // corner: a level that is restricted has an even nx, so a pair (ti, j, k)
    // is exactly the two x-children of coarse column ti (fx = 2; fy, fz are
    // 1 along a dimension of one cell, else 2)
    const int sy = fy - 1, sz = fz - 1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= tp.np) break;
      const int ti = tp.ti[q], j = tp.j[q], k = tp.k[q];
      if ((j & sy) == 0 && (k & sz) == 0) {
        T sum = 0;
        for (int dk = 0; dk < fz; ++dk)
          for (int dj = 0; dj < fy; ++dj) {
            const int f = 2 * ti + nf.nx * (j + dj) + sxy * (k + dk);
            sum += rs[f];
            sum += rs[f + 1];
          }
        bc[ti + nc.nx * ((j >> sy) + nc.ny * (k >> sz))] = sum * inv;
      }
    }
    tail_sync<WAVE>();
  }

  // coarsest level: sweeps forward (red, black) then backward (black, red) from zero
  __device__ void coarsest(int l) const {
    const Dims n = D.n[l];
    if (n.nx <= 2 && n.ny == 1 && n.nz == 1) {
      coarsest_row(l);
      return;
    }
    if (D.coarse_sweeps > 0) {
      TailPairs tp;
      tail_decode(D.n[l], tid, nthr, tp);
      smooth(l, tp, 0, D.coarse_sweeps, true);
      smooth(l, tp, 1, D.coarse_sweeps, false);
    } else {
      zero(l);
    }
  }

  // A coarsest level of one or two cells in a row: the same sweeps, with the
  // same arithmetic, done by one thread in registers.  Cell 0 is red, cell 1
  // black; the face between them is bx[1]; there is no other neighbour.
  __device__ void coarsest_row(int l) const {
    if (tid == 0) {
      const bool two = D.n[l].nx == 2;
      const T h2 = D.h2[l];
      const T *b = sm + D.ob[l], *invd = sm + D.oid[l], *bx = sm + D.obx[l];
      T* e = sm + D.oe[l];
      const T r0 = h2 * b[0], i0 = invd[0];
      const T r1 = two ? h2 * b[1] : (T)0, i1 = two ? invd[1] : (T)0, w = two ? bx[1] : (T)0;
      T e0 = 0, e1 = 0;
      const int S = D.coarse_sweeps;
      for (int s = 0; s < S; ++s) {   // forward: red (from zero first), black
        T num = r0;
        if (two && s > 0) num += w * e1;
        e0 = num * i0;
        num = r1;
        num += w * e0;
        e1 = num * i1;
      }
      for (int s = 0; s < S; ++s) {   // backward: black, red
        T num = r1;
        num += w * e0;
        e1 = num * i1;
        num = r0;
        if (two) num += w * e1;
        e0 = num * i0;
      }
      e[0] = e0;
      if (two) e[1] = e1;
    }
    tail_sync<WAVE>();
  }

  // prolongation of the next level's correction (both cells of a pair share
  // one coarse cell: fx = 2), then post-smoothing
  __device__ void up(int l) const {
    const Dims nf = D.n[l], nc = D.n[l + 1];
    const int sy = D.f[l][1] - 1, sz = D.f[l][2] - 1;
    T* e = sm + D.oe[l];
    const T* ec = sm + D.oe[l + 1];
    TailPairs tp;
    tail_decode(nf, tid, nthr, tp);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= tp.np) break;
      const int ti = tp.ti[q], j = tp.j[q], k = tp.k[q];
      const T add = ec[ti + nc.nx * ((j >> sy) + nc.ny * (k >> sz))];
      const int c = 2 * ti + nf.nx * (j + nf.ny * k);
      e[c] += add;
      if (2 * ti + 1 < nf.nx) e[c + 1] += add;
    }
    tail_sync<WAVE>();
    smooth(l, tp, 1, D.nu_post, false);
  }
};

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail(TailDesc<T> D) {
  extern __shared__ double tail_smem[];
  T* sm = reinterpret_cast<T*>(tail_smem);
  const int nl = D.nl;
  const int tid = threadIdx.x;
  // stage the pack (every coefficient array and 1/D) and the first
  // right-hand side: one flat loop, sixteen independent loads in flight per
  // thread
  {
    // each load from one address chosen by a select (past the end: the last
    // entry of b0, not stored), so no load waits behind a branch
    const int np = D.npack, n0 = D.n[0].nx * D.n[0].ny * D.n[0].nz, total = np + n0;
    for (int base = tid; base < total; base += 16 * kTailThreads) {
      T v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = base + u * kTailThreads;
        const T* src = q < np ? D.pack + q : D.b0 + min(max(q - np, 0), n0 - 1);
        v[u] = *src;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = base + u * kTailThreads;
        if (q < total) sm[q < np ? q : D.ob[0] + (q - np)] = v[u];
      }
    }
    // every level's correction starts at zero: the passes read a cell's own
    // entry through a wall before it is first written
    for (int l = 0; l < nl; ++l) {
      const int N = D.n[l].nx * D.n[l].ny * D.n[l].nz;
      for (int c = tid; c < N; c += kTailThreads) sm[D.oe[l] + c] = (T)0;
    }
  }
  __syncthreads();
  // first level (ls) from which every level fits one wavefront
  int ls = nl;
  while (ls > 0 && ((D.n[ls - 1].nx + 1) / 2) * D.n[ls - 1].ny * D.n[ls - 1].nz <= 64) --ls;
  const TailLevel<T, false> big{D, sm, tid, kTailThreads};
  for (int l = 0; l < ls && l < nl - 1; ++l) big.down(l);
  if (ls >= nl) big.coarsest(nl - 1);
  if (ls < nl) {
    if (tid < 64) {
      const TailLevel<T, true> small{D, sm, tid, 64};
      for (int l = ls; l < nl - 1; ++l) small.down(l);
      small.coarsest(nl - 1);
      for (int l = nl - 2; l >= ls; --l) small.up(l);
    }
    __syncthreads();
  }
  for (int l = (ls < nl ? ls : nl - 1) - 1; l >= 0; --l) big.up(l);
  {
    const int N0 = D.n[0].nx * D.n[0].ny * D.n[0].nz;
    for (int q = tid; q < N0; q += kTailThreads) D.ge[q] = sm[D.oe[0] + q];
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ a, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) a[q] = (T)0;
}

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) b[q] = (float)a[q];
}

__global__ void k_f2d(const float* __restrict__ a, double* __restrict__ b, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) b[q] = (double)a[q];
}

// the FP32 V-cycle's result to FP64 z, fused with the per-block sums of r z
// and r z_old (block order); every thread reaches the reduction
__global__ void __launch_bounds__(256) k_f2d_dots(const float* __restrict__ a, double* __restrict__ z, size_t n,
                                                  const double* __restrict__ r, const double* __restrict__ zold,
                                                  double* __restrict__ partials) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (q < n) {
    const double zq = (double)a[q];
    z[q] = zq;
    const double rv = r[q];
    v[0] = rv * zq;
    v[1] = rv * zold[q];
  }
  block_partials<2>(v, partials, (int)blockIdx.x);
}

// ------------------------------------------------------------------ CG (FP64)
#define CELL_INDEX                                                         \
  const Tile tl = xcd_tile();                                              \
  const int i = tl.x * blockDim.x + threadIdx.x;                           \
  const int j = tl.y * blockDim.y + threadIdx.y;                           \
  const int k = tl.z * blockDim.z + threadIdx.z;                           \
  const bool inside = (i < n.nx && j < n.ny && k < n.nz);                  \
  const size_t c = inside ? i + (size_t)n.nx * (j + (size_t)n.ny * k) : 0

// r = b - A x; totals (r.r, b.b) -> scal (RESID0: S_RR, S_BB; TRR: S_TRR)
__global__ void __launch_bounds__(256) k_resid_norm(Dims n, double ih2, const double* __restrict__ bx,
                                                    const double* __restrict__ by,
                                                    const double* __restrict__ bz,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    double* __restrict__ partials, FaceTab<double> ft) {
  CELL_INDEX;
  double v[2] = {0.0, 0.0};
  // As k_dir_spmv: a wavefront is one x-row of 64 cells (blockDim.x == 64);
  // every load is issued before the first wait, through in-range indices (a
  // lane outside the grid reads around cell 0), the x neighbours come from
  // the adjacent lanes (a row's end lanes load theirs), and the faces of the
  // wavefront's lines through their tables where a line is one value.
  const int lane = threadIdx.x;
  const int ii = inside ? i : 0, jj = inside ? j : 0, kk = inside ? k : 0;
  const size_t sxy = (size_t)n.nx * n.ny;
  const double xc = x[c];
  const double xs = x[jj > 0 ? c - n.nx : c], xn = x[jj < n.ny - 1 ? c + n.nx : c];
  const double xd = x[kk > 0 ? c - sxy : c], xu = x[kk < n.nz - 1 ? c + sxy : c];
  const bool xlo = lane == 0 && ii > 0, xhi = lane == 63 && ii < n.nx - 1;
  double xx = 0.0;
  if (xlo || xhi) xx = x[xhi ? c + 1 : c - 1];
  const double bc = b[c];
  const int ju = __builtin_amdgcn_readfirstlane(min(j, n.ny - 1)), ku = __builtin_amdgcn_readfirstlane(min(k, n.nz - 1));
  FaceLd<double> F;
  F.load(n, ft, bx, by, bz, ju, ku, ii + (size_t)(n.nx + 1) * (jj + (size_t)n.ny * kk),
         ii + (size_t)n.nx * (jj + (size_t)(n.ny + 1) * kk), c);
  __builtin_amdgcn_sched_barrier(0);
  double cw, ce, cs, cn, cd, cu;
  F.get(n, ii, cw, ce, cs, cn, cd, cu);
  const double xl = __shfl_up(xc, 1, 64), xr = __shfl_down(xc, 1, 64);
  if (inside) {
    double xw = xc, xe = xc;
    if (i > 0) xw = lane > 0 ? xl : xx;
    if (i < n.nx - 1) xe = lane < 63 ? xr : xx;
    double acc = cw * (xc - xw) + ce * (xc - xe) + cs * (xc - xs) + cn * (xc - xn) + cd * (xc - xd);
    acc += (k < n.nz - 1) ? cu * (xc - xu) : 2.0 * cu * xc;
    const double rc = bc - ih2 * acc;
    r[c] = rc;
    v[0] = rc * rc;
    v[1] = bc * bc;
  }
  block_partials<2>(v, partials, tl.lin);
}

// rho = <r, z>
__global__ void __launch_bounds__(256) k_dot_rho(Dims n, const double* __restrict__ r,
                                                 const double* __restrict__ z, double* __restrict__ partials) {
  CELL_INDEX;
  double v[1] = {inside ? r[c] * z[c] : 0.0};
  block_partials<1>(v, partials, tl.lin);
}

// flexible (Polak-Ribiere) beta = (<r, zn> - <r, z>) / rho, then rho = <r, zn>
__global__ void __launch_bounds__(256) k_dots_beta(Dims n, const double* __restrict__ r,
                                                   const double* __restrict__ zn,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ partials) {
  CELL_INDEX;
  double v[2] = {0.0, 0.0};
  if (inside) {
    const double rc = r[c];
    v[0] = rc * zn[c];
    v[1] = rc * z[c];
  }
  block_partials<2>(v, partials, tl.lin);
}

// d = zn + beta d_old, q = A d = A zn + beta q_old (first: d = zn, q = A zn);
// alpha = rho / <d, q>.  Carrying q = A d by its recurrence keeps the
// stencil on zn alone, and d_old and q_old are read pointwise: the stencil's
// load count, not its bytes, limits this kernel.  With xupd it also applies
// the previous iteration's x += alpha d_old (alpha still in scal, d_old
// already loaded here), which the vector update then leaves out.  A wavefront is one x-row of
// 64 cells (blockDim.x == 64), so the x neighbours of zn come from the
// adjacent lanes and only a row's end lanes load them; every lane takes part
// in the shuffles (c is 0 outside the grid).
__global__ void __launch_bounds__(256) k_dir_spmv(Dims n, double ih2, const double* __restrict__ bx,
                                                  const double* __restrict__ by,
                                                  const double* __restrict__ bz,
                                                  const double* __restrict__ zn,
                                                  const double* __restrict__ dold,
                                                  double* __restrict__ dnew, double* __restrict__ q,
                                                  int first, const double* __restrict__ scal,
                                                  double* __restrict__ partials, double* __restrict__ x,
                                                  int xupd, FaceTab<double> ft) {
  CELL_INDEX;
  double v[1] = {0.0};
  // Every load is issued before the shuffles wait for zc: the faces and the
  // y and z neighbours through in-range indices (a lane outside the grid
  // reads around cell 0), the row-end lanes' x neighbour, and d_old, q_old
  // (also on a first iteration, which does not use them).
  const int lane = threadIdx.x;
  const int ii = inside ? i : 0, jj = inside ? j : 0, kk = inside ? k : 0;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t fx = ii + (size_t)(n.nx + 1) * (jj + (size_t)n.ny * kk);
  const size_t fy = ii + (size_t)n.nx * (jj + (size_t)(n.ny + 1) * kk);
  const double zc = zn[c];
  const double zs = zn[jj > 0 ? c - n.nx : c], zno = zn[jj < n.ny - 1 ? c + n.nx : c];
  const double zd = zn[kk > 0 ? c - sxy : c], zu = zn[kk < n.nz - 1 ? c + sxy : c];
  double zx = 0.0;   // lane 0's west and lane 63's east neighbour lie outside the wavefront
  if (lane == 0 && ii > 0) zx = zn[c - 1];
  if (lane == 63 && ii < n.nx - 1) zx = zn[c + 1];
  const double dol = dold[c], qol = q[c];
  const double xo = xupd ? x[c] : 0.0;
  // the faces: of the wavefront's x-line (j, k), the y-lines j, j + 1 and the
  // z-lines k, k + 1, each through its table where the line is one value
  const int ju = __builtin_amdgcn_readfirstlane(min(j, n.ny - 1)), ku = __builtin_amdgcn_readfirstlane(min(k, n.nz - 1));
  FaceLd<double> F;
  F.load(n, ft, bx, by, bz, ju, ku, fx, fy, c);
  __builtin_amdgcn_sched_barrier(0);
  double cw, ce, cs, cn, cd, cu;
  F.get(n, ii, cw, ce, cs, cn, cd, cu);
  const double zl = __shfl_up(zc, 1, 64), zr = __shfl_down(zc, 1, 64);
  if (inside) {
    if (xupd) x[c] = xo + scal[S_ALPHA] * dol;
    double zw = zc, ze = zc;
    if (i > 0) zw = lane > 0 ? zl : zx;
    if (i < n.nx - 1) ze = lane < 63 ? zr : zx;
    double acc = cw * (zc - zw) + ce * (zc - ze) + cs * (zc - zs) + cn * (zc - zno) + cd * (zc - zd);
    acc += (k < n.nz - 1) ? cu * (zc - zu) : 2.0 * cu * zc;
    const double qz = ih2 * acc;
    double dc = zc, qc = qz;
    if (!first) {
      const double beta = scal[S_BETA];
      dc = zc + beta * dol;
      qc = qz + beta * qol;
    }
    dnew[c] = dc;
    q[c] = qc;
    v[0] = dc * qc;
  }
  block_partials<1>(v, partials, tl.lin);
}

// r -= alpha q; ||r||^2 (the matching x += alpha d is applied by the next
// direction update, or by k_x_update before x is read)
__global__ void __launch_bounds__(256) k_cg_update(Dims n, const double* __restrict__ q, double* __restrict__ r,
                                                   const double* __restrict__ scal,
                                                   double* __restrict__ partials) {
  CELL_INDEX;
  double v[1] = {0.0};
  if (inside) {
    const double rc = r[c] - scal[S_ALPHA] * q[c];
    r[c] = rc;
    v[0] = rc * rc;
  }
  block_partials<1>(v, partials, tl.lin);
}

// x += alpha d: the update the CG vector update leaves pending
__global__ void __launch_bounds__(256) k_x_update(Dims n, const double* __restrict__ d, double* __restrict__ x,
                                                  const double* __restrict__ scal) {
  CELL_INDEX;
  if (inside) x[c] = x[c] + scal[S_ALPHA] * d[c];
}

__global__ void __launch_bounds__(256) k_apply_A(Dims n, double ih2, const double* __restrict__ bx,
                                                 const double* __restrict__ by,
                                                 const double* __restrict__ bz,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y) {
  CELL_INDEX;
  if (inside) y[c] = ih2 * stencil<double>(n, bx, by, bz, x, i, j, k, c);
}


// first stage of a large reduction: block g sums partials [g W, (g + 1) W),
// W = 4 x 1024, thread t the four consecutive ones from g W + 4 t in order,
// then the block's fixed tree; out[nv g + q] gets the block's sums
constexpr int kFinChunk = 4 * 1024;
__global__ void __launch_bounds__(1024) k_finalize_chunks(const double* __restrict__ partials, int nparts, int nv,
                                                          double* __restrict__ out) {
  const int q0 = (int)blockIdx.x * kFinChunk + 4 * (int)threadIdx.x;
  double a[4], c[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = min(q0 + u, nparts - 1);
    a[u] = partials[nv * q];
    c[u] = nv > 1 ? partials[nv * q + 1] : 0.0;
  }
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (q0 + u < nparts) {
      v[0] += a[u];
      v[1] += c[u];
    }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    out[nv * (size_t)blockIdx.x] = v[0];
    if (nv > 1) out[nv * (size_t)blockIdx.x + 1] = v[1];
  }
}

// fixed-order sum of the per-block partials and the CG scalar recurrences;
// the values the host tests are also stored to its pinned mirror
template <int B>
__global__ void __launch_bounds__(1024) k_finalize(const double* __restrict__ partials, int nparts,
                                                   int nv, int mode, double* __restrict__ scal,
                                                   double* __restrict__ hscal) {
  // thread t sums partials t, t + 1024, t + 2048, ... in that order; each
  // batch of B is loaded (clamped, unconditional) before it is added, so the
  // loads are in flight together.  B only sets how many loads one batch
  // issues, never the order of the additions.
  double v[2] = {0.0, 0.0};
  for (int base = threadIdx.x; base < nparts; base += 1024 * B) {
    double a[B], c[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int q = min(base + 1024 * u, nparts - 1);
      a[u] = partials[nv * q];
      c[u] = nv > 1 ? partials[nv * q + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (base + 1024 * u < nparts) {
        v[0] += a[u];
        if (nv > 1) v[1] += c[u];
      }
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    const double a = v[0], b = v[1];
    switch (mode) {
      case FIN_RESID0:
        scal[S_RR] = a;
        scal[S_BB] = b;
        hscal[S_RR] = a;
        hscal[S_BB] = b;
        break;
      case FIN_TRR:
        scal[S_TRR] = a;
        hscal[S_TRR] = a;
        break;
      case FIN_RHO: scal[S_RHO] = a; break;
      case FIN_BETA: scal[S_BETA] = (a - b) / scal[S_RHO]; scal[S_RHO] = a; break;
      case FIN_ALPHA: scal[S_DQ] = a; scal[S_ALPHA] = scal[S_RHO] / a; break;
      case FIN_RR:
        scal[S_RR] = a;
        hscal[S_RR] = a;
        break;
    }
  }
}


}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_gs(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, int colour,
               hipStream_t st, KTimer* kt, T* nat) {
  const bool fine = (L.h == L.h0);
  const FaceTab<T> ft = face_tab(L, bx);
  const bool tab1 = !fine && ft.x != nullptr;   // a coarse level with line tables
  const int pl = gs_planes<T>(fine || tab1);   // planes per thread
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, (L.n.nz + pl - 1) / pl);
  auto kern = fine ? k_gs<T, true> : tab1 ? k_gs_c1<T> : k_gs<T, false>;
  if (kt && kt->n < kt->cap) {
    hipExtLaunchKernelGGL(kern, g.grid, g.block, 0, st, kt->ev[2 * kt->n], kt->ev[2 * kt->n + 1], 0, L.n,
                          (T)(L.h * L.h), bx, by, bz, b, e, colour, nat, ft);
    ++kt->n;
    return;
  }
  hipLaunchKernelGGL(kern, g.grid, g.block, 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, e, colour, nat, ft);
}

template <typename T>
void launch_gs_first(const Level& L, const T* bx, const T* by, const T* bz, const T* b, bool b_natural,
                     const T* invd, T* e, T* bs, hipStream_t st, T* bcopy, bool red_out) {
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, L.n.nz);
  const bool fine = (L.h == L.h0);
  const FaceTab<T> ft = face_tab(L, bx);
  const bool tab1 = !fine && ft.x != nullptr && !b_natural;   // a coarse level with line tables
  void (*kern)(Dims, T, const T*, const T*, const T*, const T*, const T*, T*, T*, T*, FaceTab<T>, int);
  if (b_natural)
    kern = fine ? k_gs_first<T, true, true> : k_gs_first<T, false, true>;
  else
    kern = fine ? k_gs_first<T, true, false> : tab1 ? k_gs_first_c1<T> : k_gs_first<T, false, false>;
  hipLaunchKernelGGL(kern, g.grid, g.block, 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, invd, e, bs, bcopy, ft,
                     red_out ? 1 : 0);
}

template <typename T>
void launch_gs_prolong(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e,
                       const Level& C, const T* ec, bool ec_split, hipStream_t st, T* bcopy) {
  const bool fine = (L.h == L.h0);
  const FaceTab<T> ft = face_tab(L, bx);
  const bool tab1 = !fine && ft.x != nullptr;   // a coarse level with line tables
  const int pl = gs_planes<T>(fine || tab1);   // planes per thread
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, (L.n.nz + pl - 1) / pl);
  auto kern = fine ? k_gs_prolong<T, true> : tab1 ? k_gs_prolong_c1<T> : k_gs_prolong<T, false>;
  hipLaunchKernelGGL(kern, g.grid, g.block, 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, e, C.n, L.f[0] >> 1,
                     L.f[1] >> 1, L.f[2] >> 1, ec_split ? 1 : 0, ec, bcopy, ft);
}

// the fused red-black pass's tile (TX lanes per row, TY rows, TZ planes), or
// false where a row does not fit one tile
static bool gs_rb_tile(const Dims& n, int& TX, int& TY, int& TZ) {
  const int hx = (n.nx + 1) / 2;
  if (hx > 32) return false;
  TX = hx > 16 ? 32 : hx > 8 ? 16 : 8;
  TY = n.ny > 1 ? 4 : 1;
  // TX TY is 8 to 128, a divisor of kRbThreads: the tile has one black cell
  // per thread
  static_assert(kRbThreads % (32 * 4) == 0, "every TX TY divides the block");
  TZ = kRbThreads / (TX * TY);
  // the ring-extended tile within the kernel's LDS and its unrolled loads
  return TX * (TY + (n.ny > 1 ? 2 : 0)) * (TZ + 2) <= kRbMaxExt;
}

bool gs_rb_fits(const Dims& n) {
  int TX, TY, TZ;
  return gs_rb_tile(n, TX, TY, TZ);
}

template <typename T>
void launch_gs_rb(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, const T* bold,
                  hipStream_t st) {
  int TX, TY, TZ;
  if (!gs_rb_tile(L.n, TX, TY, TZ)) return;   // callers check gs_rb_fits first
  const dim3 grid(1, (L.n.ny + TY - 1) / TY, (L.n.nz + TZ - 1) / TZ);
  hipLaunchKernelGGL(k_gs_rb<T>, grid, dim3(kRbThreads), 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, e, bold, TX,
                     TY, TZ);
}

// the finest level's fused red-black sweep: where it applies (a 3-D level
// whose rows fill at least half a wave), where it pays, and its launch.  A
// block runs 64 lanes by kRbfRows + 2 rows of pairs and the halo wave (1024
// threads) up a chunk of planes.
constexpr int kRbfRows = 13;    // inner rows of a block (TY)

bool gs_rb_fine_fits(const Dims& n) {
  return n.ny >= 4 && n.nz >= 4 && (n.nx + 1) / 2 >= 32;
}

// A block's march is a chain of dependent planes: the launch wins over two
// colour passes on large grids only, in FP64 only, and only where the
// passes load every face (on 512 x 256 x 256 378 us against 2 x 223 in FP64,
// but 249 against 2 x 116 in FP32, whose planes carry half the bytes for the
// same instructions; slower in both on 256 x 128 x 128 and 128 x 64 x 64).
// With the line tables a colour pass loads few faces and takes 153 us there,
// and the two passes win (the march's loads stay as many).
bool gs_rb_fine_pays(const Dims& n, bool fp64, bool tables) {
  return fp64 && !tables && gs_rb_fine_fits(n) && (long)n.nx * n.ny * n.nz >= (1L << 24);
}

// compute units of the current device (one block of the sweep per unit)
static int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] > 0) return cache[dev];
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  cache[dev] = v;
  return v;
}

// The chunk of planes a block marches.  A block holds its compute unit for
// its whole march (KZ + 2 planes), so the sweep takes about (rounds of
// blocks) x (KZ + 2) plane times: the chunk is chosen to minimise that
// product, ties going to fewer chunks.  512 x 256 x 256 gets 3 chunks of 86
// planes, 240 blocks, one round.
static int rbf_planes(int tiles, int nz, int cus) {
  long best = -1;
  int best_kz = nz;
  for (int nzc = 1; nzc <= nz; ++nzc) {
    const int kz = (nz + nzc - 1) / nzc;
    const int chunks = (nz + kz - 1) / kz;
    const long rounds = ((long)tiles * chunks + cus - 1) / cus;
    const long cost = rounds * (kz + 2);
    if (best < 0 || cost < best) {
      best = cost;
      best_kz = kz;
    }
  }
  return best_kz;
}

template <typename T>
void launch_gs_rb_fine(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, const T* bold,
                       hipStream_t st, KTimer* kt) {
  constexpr int TY = kRbfRows;
  static_assert(kRbfLanes * (TY + 3) == 1024, "a block of 1024 threads");
  const int hx = (L.n.nx + 1) / 2;
  const int gx = (hx + kRbfLanes - 1) / kRbfLanes, gy = (L.n.ny + TY - 1) / TY;
  const int KZ = rbf_planes(gx * gy, L.n.nz, device_cus());
  const dim3 grid(gx, gy, (L.n.nz + KZ - 1) / KZ);
  const dim3 blk(kRbfLanes, TY + 3);
  const T h2 = (T)(L.h * L.h);
  if (kt && kt->n < kt->cap) {
    hipExtLaunchKernelGGL((k_gs_rb_fine<T, TY>), grid, blk, 0, st, kt->ev[2 * kt->n], kt->ev[2 * kt->n + 1], 0, L.n,
                          h2, bx, by, bz, b, e, bold, KZ);
    ++kt->n;
    return;
  }
  hipLaunchKernelGGL((k_gs_rb_fine<T, TY>), grid, blk, 0, st, L.n, h2, bx, by, bz, b, e, bold, KZ);
}

// the pair form of the residual-restriction: even extents, halved in every
// direction (the fine level is colour-split wherever it is called)
static bool resid_pairs_fit(const Level& F) {
  return F.f[0] == 2 && F.f[1] == 2 && F.f[2] == 2 && F.n.nx % 2 == 0 && F.n.ny % 2 == 0 && F.n.nz % 2 == 0;
}

template <typename T>
void launch_resid_restrict(const Level& F, const T* bx, const T* by, const T* bz, const T* b,
                           const T* e, const Level& C, T* bc, bool c_split, hipStream_t st) {
  const T ih2 = (T)(1.0 / (F.h * F.h));
  if (resid_pairs_fit(F)) {
    const dim3 grid((F.n.nx / 2 + 63) / 64, F.n.ny / 2, F.n.nz / 2);
    hipLaunchKernelGGL(k_resid_restrict_pairs<T>, grid, dim3(64, 2, 2), 0, st, F.n, ih2, bx, by, bz, b, e, C.n,
                       c_split ? 1 : 0, (T)0.125, bc, face_tab(F, bx));
    return;
  }
  // fine-cell tiles with even extents (a coarse cell's children in one tile)
  const dim3 blk = (F.n.ny > 1) ? dim3(32, 4, 2) : dim3(64, 1, 4);
  const Geo g{dim3((F.n.nx + blk.x - 1) / blk.x, (F.n.ny + blk.y - 1) / blk.y, (F.n.nz + blk.z - 1) / blk.z), blk};
  const T inv = (T)(1.0 / (F.f[0] * F.f[1] * F.f[2]));
  hipLaunchKernelGGL(k_resid_restrict<T>, g.grid, g.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], ih2, bx,
                     by, bz, b, e, C.n, c_split ? 1 : 0, inv, bc);
}

template <typename T>
void launch_prolong(const Level& F, T* e, const Level& C, const T* ec, bool ec_split, hipStream_t st) {
  Geo g = geo3(F.n.nx, F.n.ny, F.n.nz);
  hipLaunchKernelGGL(k_prolong<T>, g.grid, g.block, 0, st, F.n, F.f[0] >> 1, F.f[1] >> 1, F.f[2] >> 1, e, C.n,
                     ec_split ? 1 : 0, ec);
}

template <typename T>
void launch_split_copy(const Level& L, const T* src, T* dst, bool to_split, hipStream_t st) {
  Geo g = geo3(L.n.nx, L.n.ny, L.n.nz);
  hipLaunchKernelGGL(k_split_copy<T>, g.grid, g.block, 0, st, L.n, src, dst, to_split ? 1 : 0);
}

template <typename T>
void launch_invdiag(const Level& L, const T* bx, const T* by, const T* bz, T* invd, bool split, hipStream_t st) {
  Geo g = geo3(L.n.nx, L.n.ny, L.n.nz);
  hipLaunchKernelGGL(k_invdiag<T>, g.grid, g.block, 0, st, L.n, bx, by, bz, split ? 1 : 0, invd);
}

template <typename T>
void launch_coarsen_level(const Level& F, const T* fbx, const T* fby, const T* fbz, const Level& C, T* cbx,
                          T* cby, T* cbz, T* invd, bool split, hipStream_t st) {
  Geo g = geo3(C.n.nx, C.n.ny, C.n.nz);
  hipLaunchKernelGGL(k_coarsen_level<T>, g.grid, g.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], fbx, fby, fbz, C.n,
                     cbx, cby, cbz, split ? 1 : 0, invd);
}

template <typename T>
void launch_vcycle_tail(const TailDesc<T>& D, size_t lds_bytes, hipStream_t st) {
  // dynamic LDS above 64 KB needs the kernel's limit raised (once per process)
  static bool raised = false;
  if (lds_bytes > 64 * 1024 && !raised) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_vcycle_tail<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTailLdsBytes);
    raised = true;
  }
  hipLaunchKernelGGL(k_vcycle_tail<T>, dim3(1), dim3(kTailThreads), lds_bytes, st, D);
}

template <typename T>
void launch_fill(T* a, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
}

template <typename T>
void launch_face_tables(const Dims& n, const T* bx, const T* by, const T* bz, T* tx, T* ty, T* tz, hipStream_t st) {
  const int lines = n.ny * n.nz + (n.ny + 1) * n.nz + n.ny * (n.nz + 1);
  hipLaunchKernelGGL(k_face_table<T>, dim3((lines + 3) / 4), dim3(256), 0, st, n, bx, by, bz, tx, ty, tz);
}

// Where the line tables pay: each kernel that reads them waits one cache
// round trip for its lines' entries before it issues their faces' loads, which
// a latency-bound level cannot hide (128 x 64 x 64: the FP64 step 2.5% slower
// with them); from 2^21 cells on the bytes they spare win (256 x 128 x 128:
// 7.00 -> 6.27 ms, 512 x 256 x 256: 51.1 -> 41.5 ms).
bool face_tables_pay(const Dims& n) { return (long)n.nx * n.ny * n.nz >= (1L << 21); }


void launch_d2f(const double* a, float* b, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

template <typename T>
int launch_gs_last_dots(const Level& L, const T* bx, const T* by, const T* bz, const T* b, const T* e,
                        double* nat, const double* r, const double* zold, double* partials, hipStream_t st) {
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, L.n.nz);
  hipLaunchKernelGGL(k_gs_last_dots<T>, g.grid, g.block, 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, e, nat, r,
                     zold, partials, face_tab(L, bx));
  return (int)(g.grid.x * g.grid.y * g.grid.z);
}

void launch_gs_first_nat64(const Level& L, const float* bx, const float* by, const float* bz, const double* b,
                           const float* invd, float* e, float* bs, hipStream_t st, float* bcopy, bool red_out) {
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, L.n.nz);
  hipLaunchKernelGGL((k_gs_first<float, true, true, double>), g.grid, g.block, 0, st, L.n, (float)(L.h * L.h), bx,
                     by, bz, b, invd, e, bs, bcopy, face_tab(L, bx), red_out ? 1 : 0);
}

int launch_f2d_dots(const float* a, double* z, size_t n, const double* r, const double* zold, double* partials,
                    hipStream_t st) {
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_f2d_dots, dim3(nb), dim3(256), 0, st, a, z, n, r, zold, partials);
  return nb;
}

void launch_f2d(const float* a, double* b, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

int cg_blocks(const Dims& n) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  return (int)(g.grid.x * g.grid.y * g.grid.z);
}

static void finalize(const CgScratch& cs, int nparts, int mode, hipStream_t st) {
  const int nv = (mode == FIN_RESID0 || mode == FIN_TRR || mode == FIN_BETA) ? 2 : 1;
  const double* src = cs.partials;
  // Beyond one batch of 16 loads per thread, one workgroup walking every
  // partial waits on a chain of batches (27 us for the 131072 blocks of a
  // 512 x 256 x 256 level): the chunks are summed first, one workgroup
  // each, into the partials buffer's free room after the nv * nparts values
  // (the buffer holds 4 per block of the finest level; nv <= 2), and their
  // sums finalized.  Up to one batch a single launch is cheaper.
  if (nparts > 16 * 1024) {
    const int G = (nparts + kFinChunk - 1) / kFinChunk;
    double* mid = cs.partials + (size_t)nv * nparts;
    hipLaunchKernelGGL(k_finalize_chunks, dim3(G), dim3(1024), 0, st, cs.partials, nparts, nv, mid);
    src = mid;
    nparts = G;
  }
  // loads per thread per batch: as many as the partials need, at most 16
  const int per = (nparts + 1023) / 1024;
  const dim3 g(1), b(1024);
  if (per <= 1)
    hipLaunchKernelGGL(k_finalize<1>, g, b, 0, st, src, nparts, nv, mode, cs.scal, cs.hscal);
  else if (per <= 2)
    hipLaunchKernelGGL(k_finalize<2>, g, b, 0, st, src, nparts, nv, mode, cs.scal, cs.hscal);
  else if (per <= 4)
    hipLaunchKernelGGL(k_finalize<4>, g, b, 0, st, src, nparts, nv, mode, cs.scal, cs.hscal);
  else
    hipLaunchKernelGGL(k_finalize<16>, g, b, 0, st, src, nparts, nv, mode, cs.scal, cs.hscal);
}

void launch_finalize_beta(const CgScratch& cs, int nparts, hipStream_t st) { finalize(cs, nparts, FIN_BETA, st); }

void launch_resid_norm(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                       const double* b, const double* x, double* r, const CgScratch& cs, int mode,
                       hipStream_t st, const FaceTab<double>& ft) {
  Geo g = geo3(n.nx, n.ny, n.nz);   // blockDim.x == 64: a wavefront per x-line
  hipLaunchKernelGGL(k_resid_norm, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, b, x, r,
                     cs.hpart ? cs.hpart : cs.partials, ft);
  if (!cs.hpart) finalize(cs, (int)(g.grid.x * g.grid.y * g.grid.z), mode, st);
}

void launch_dot_rho(const Dims& n, const double* r, const double* z, const CgScratch& cs, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_dot_rho, g.grid, g.block, 0, st, n, r, z, cs.partials);
  finalize(cs, (int)(g.grid.x * g.grid.y * g.grid.z), FIN_RHO, st);
}

void launch_dots_beta(const Dims& n, const double* r, const double* zn, const double* z,
                      const CgScratch& cs, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_dots_beta, g.grid, g.block, 0, st, n, r, zn, z, cs.partials);
  finalize(cs, (int)(g.grid.x * g.grid.y * g.grid.z), FIN_BETA, st);
}

void launch_dir_spmv(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                     const double* zn, const double* dold, double* dnew, double* q, int first,
                     const CgScratch& cs, hipStream_t st, KTimer* kt, double* x, const FaceTab<double>& ft) {
  Geo g = geo3(n.nx, n.ny, n.nz);   // blockDim.x == 64: a wavefront per x-line
  const int xupd = x ? 1 : 0;
  if (kt && kt->n < kt->cap) {
    (void)hipStreamSynchronize(st);
    hipExtLaunchKernelGGL(k_dir_spmv, g.grid, g.block, 0, st, kt->ev[2 * kt->n], kt->ev[2 * kt->n + 1], 0,
                          n, 1.0 / (h * h), bx, by, bz, zn, dold, dnew, q, first, (const double*)cs.scal,
                          cs.partials, x, xupd, ft);
    ++kt->n;
  } else {
    hipLaunchKernelGGL(k_dir_spmv, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, zn, dold, dnew, q,
                       first, (const double*)cs.scal, cs.partials, x, xupd, ft);
  }
  finalize(cs, (int)(g.grid.x * g.grid.y * g.grid.z), FIN_ALPHA, st);
}

void launch_cg_update(const Dims& n, const double* q, double* r, const CgScratch& cs, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_cg_update, g.grid, g.block, 0, st, n, q, r, (const double*)cs.scal,
                     cs.hpart ? cs.hpart : cs.partials);
  if (!cs.hpart) finalize(cs, (int)(g.grid.x * g.grid.y * g.grid.z), FIN_RR, st);
}

void launch_x_update(const Dims& n, const double* d, double* x, const CgScratch& cs, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_x_update, g.grid, g.block, 0, st, n, d, x, (const double*)cs.scal);
}

void launch_apply_A(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                    const double* x, double* y, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_apply_A, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, x, y);
}

#define NSK_INST(T)                                                                                   \
  template void launch_gs<T>(const Level&, const T*, const T*, const T*, const T*, T*, int, hipStream_t,   \
                             KTimer*, T*);                                                                \
  template int launch_gs_last_dots<T>(const Level&, const T*, const T*, const T*, const T*, const T*,     \
                                      double*, const double*, const double*, double*, hipStream_t);       \
  template void launch_gs_first<T>(const Level&, const T*, const T*, const T*, const T*, bool, const T*,  \
                                   T*, T*, hipStream_t, T*, bool);                                        \
  template void launch_gs_prolong<T>(const Level&, const T*, const T*, const T*, const T*, T*,           \
                                     const Level&, const T*, bool, hipStream_t, T*);                      \
  template void launch_gs_rb<T>(const Level&, const T*, const T*, const T*, const T*, T*, const T*,     \
                                hipStream_t);                                                             \
  template void launch_gs_rb_fine<T>(const Level&, const T*, const T*, const T*, const T*, T*, const T*,  \
                                     hipStream_t, KTimer*);                                               \
  template void launch_resid_restrict<T>(const Level&, const T*, const T*, const T*, const T*, const T*,  \
                                         const Level&, T*, bool, hipStream_t);                            \
  template void launch_prolong<T>(const Level&, T*, const Level&, const T*, bool, hipStream_t);           \
  template void launch_split_copy<T>(const Level&, const T*, T*, bool, hipStream_t);                     \
  template void launch_invdiag<T>(const Level&, const T*, const T*, const T*, T*, bool, hipStream_t);    \
  template void launch_coarsen_level<T>(const Level&, const T*, const T*, const T*, const Level&, T*, \
                                        T*, T*, T*, bool, hipStream_t);                               \
  template void launch_fill<T>(T*, size_t, hipStream_t);                                              \
  template void launch_face_tables<T>(const Dims&, const T*, const T*, const T*, T*, T*, T*, hipStream_t); \
  template void launch_vcycle_tail<T>(const TailDesc<T>&, size_t, hipStream_t);
NSK_INST(double)
NSK_INST(float)
#undef NSK_INST

}  // namespace nsk
