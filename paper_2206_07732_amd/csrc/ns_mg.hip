// Multigrid (red-black Gauss-Seidel V-cycle) and conjugate-gradient kernels
// for the pressure projection on gfx950.
//
// Operator on a level with spacing h (walls carry beta = 0, so every cell
// sums all six faces; the open top face couples to the ghost -x_c):
//   (A x)_c = (1/h^2) [ sum_f beta_f (x_c - x_nb) + 2 beta_top x_c (top row) ]
// V-cycle kernels are templated on the arithmetic type (double or float);
// the CG vectors and their reductions are always FP64.  Reductions are
// deterministic: wavefront shuffle, then LDS across the block's four
// wavefronts, then one fixed-order pass over the per-block partials.
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
  const T bu = bz[c + sxy];
  T acc = bx[fx] * (xc - xw) + bx[fx + 1] * (xc - xe) + by[fy] * (xc - xs) +
          by[fy + n.nx] * (xc - xn) + bz[c] * (xc - xd);
  if (k < n.nz - 1)
    acc += bu * (xc - x[c + sxy]);
  else
    acc += (T)2 * bu * xc;
  return acc;
}

// reduce NV doubles over a 256-thread block (4 wavefronts), thread 0 writes
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ partials) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_down(v[q], off, 64);
  __shared__ double sm[4][NV];
  const int tid = threadIdx.x + 64 * (threadIdx.y + blockDim.y * threadIdx.z);
  const int lane = tid & 63, wid = tid >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sm[wid][q] = v[q];
  __syncthreads();
  if (tid == 0) {
    const size_t blk = blockIdx.x + gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[NV * blk + q] = (sm[0][q] + sm[1][q]) + (sm[2][q] + sm[3][q]);
  }
}

// --------------------------------------------------------------- smoother
// One colour of Gauss-Seidel.  Thread ti owns the cell pair (2ti, 2ti+1) of
// its row and updates the one of the requested colour.  With first != 0 the
// correction is taken as zero before the pass: the colour cell gets
// h^2 b / D and the other cell of the pair is cleared.
// FINE marks the finest-level instance (a separate symbol for profiling).
template <typename T, bool FINE>
__global__ void __launch_bounds__(256) k_gs(Dims n, T h2, const T* __restrict__ bx,
                                            const T* __restrict__ by, const T* __restrict__ bz,
                                            const T* __restrict__ b, T* __restrict__ e, int colour,
                                            int first) {
  const int ti = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z * blockDim.z + threadIdx.z;
  if (j >= n.ny || k >= n.nz) return;
  const int par = (j + k + colour) & 1;
  const int i = 2 * ti + par;
  const size_t sxy = (size_t)n.nx * n.ny;
  const size_t row = (size_t)n.nx * j + sxy * k;
  if (first) {
    const int io = 2 * ti + 1 - par;
    if (io < n.nx) e[row + io] = (T)0;
  }
  if (i >= n.nx) return;
  const size_t c = row + i;
  const size_t fx = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
  const size_t fy = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
  const T bw = bx[fx], be = bx[fx + 1], bs = by[fy], bn = by[fy + n.nx], bd = bz[c],
          bu = bz[c + sxy];
  const bool top = (k == n.nz - 1);
  const T diag = bw + be + bs + bn + bd + (top ? (T)2 * bu : bu);
  T num = h2 * b[c];
  if (!first) {
    num += bw * e[i > 0 ? c - 1 : c] + be * e[i < n.nx - 1 ? c + 1 : c] +
           bs * e[j > 0 ? c - n.nx : c] + bn * e[j < n.ny - 1 ? c + n.nx : c] +
           bd * e[k > 0 ? c - sxy : c] + (top ? (T)0 : bu * e[c + sxy]);
  }
  e[c] = num / diag;
}

// coarse rhs = mean over the children of the fine residual b - A e
template <typename T>
__global__ void __launch_bounds__(256) k_resid_restrict(Dims nf, int fx, int fy, int fz, T ih2,
                                                        const T* __restrict__ bx,
                                                        const T* __restrict__ by,
                                                        const T* __restrict__ bz,
                                                        const T* __restrict__ b,
                                                        const T* __restrict__ e, Dims nc, T inv,
                                                        T* __restrict__ bc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int K = blockIdx.z * blockDim.z + threadIdx.z;
  if (I >= nc.nx || J >= nc.ny || K >= nc.nz) return;
  T sum = 0;
  for (int dk = 0; dk < fz; ++dk)
    for (int dj = 0; dj < fy; ++dj)
      for (int di = 0; di < fx; ++di) {
        const int i = fx * I + di, j = fy * J + dj, k = fz * K + dk;
        const size_t c = i + (size_t)nf.nx * (j + (size_t)nf.ny * k);
        sum += b[c] - ih2 * stencil<T>(nf, bx, by, bz, e, i, j, k, c);
      }
  bc[I + (size_t)nc.nx * (J + (size_t)nc.ny * K)] = sum * inv;
}

// fine correction += parent's coarse correction
template <typename T>
__global__ void __launch_bounds__(256) k_prolong(Dims nf, int fx, int fy, int fz, T* __restrict__ e,
                                                 Dims nc, const T* __restrict__ ec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z * blockDim.z + threadIdx.z;
  if (i >= nf.nx || j >= nf.ny || k >= nf.nz) return;
  e[i + (size_t)nf.nx * (j + (size_t)nf.ny * k)] +=
      ec[(i / fx) + (size_t)nc.nx * ((j / fy) + (size_t)nc.ny * (k / fz))];
}

// coarsest level: `sweeps` red-black pairs forward then backward, from zero,
// in one workgroup
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_solve(Dims n, T h2, const T* __restrict__ bx,
                                                      const T* __restrict__ by,
                                                      const T* __restrict__ bz,
                                                      const T* __restrict__ b, T* __restrict__ e,
                                                      int sweeps) {
  const int N = n.nx * n.ny * n.nz;
  const size_t sxy = (size_t)n.nx * n.ny;
  for (int c = threadIdx.x; c < N; c += blockDim.x) e[c] = (T)0;
  __syncthreads();
  auto pass = [&](int colour) {
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      const int i = c % n.nx;
      const int j = (c / n.nx) % n.ny;
      const int k = c / (int)sxy;
      if (((i + j + k) & 1) != colour) continue;
      const size_t fx = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
      const size_t fy = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
      const T bw = bx[fx], be = bx[fx + 1], bs = by[fy], bn = by[fy + n.nx], bd = bz[c],
              bu = bz[c + sxy];
      const bool top = (k == n.nz - 1);
      const T diag = bw + be + bs + bn + bd + (top ? (T)2 * bu : bu);
      const T num = h2 * b[c] + bw * e[i > 0 ? c - 1 : c] + be * e[i < n.nx - 1 ? c + 1 : c] +
                    bs * e[j > 0 ? c - n.nx : c] + bn * e[j < n.ny - 1 ? c + n.nx : c] +
                    bd * e[k > 0 ? c - sxy : c] + (top ? (T)0 : bu * e[c + sxy]);
      e[c] = num / diag;
    }
    __syncthreads();
  };
  for (int s = 0; s < sweeps; ++s) {
    pass(0);
    pass(1);
  }
  for (int s = 0; s < sweeps; ++s) {
    pass(1);
    pass(0);
  }
}

// coarse face coefficient = mean of the fine faces covering it
template <typename T, int C>
__global__ void __launch_bounds__(256) k_coarsen_beta(Dims nf, int fx, int fy, int fz,
                                                      const T* __restrict__ fb, Dims nc,
                                                      T* __restrict__ cb) {
  const int mx = nc.nx + (C == 0), my = nc.ny + (C == 1), mz = nc.nz + (C == 2);
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int K = blockIdx.z * blockDim.z + threadIdx.z;
  if (I >= mx || J >= my || K >= mz) return;
  const int fmx = nf.nx + (C == 0), fmy = nf.ny + (C == 1);
  const int ni = (C == 0) ? 1 : fx, nj = (C == 1) ? 1 : fy, nk = (C == 2) ? 1 : fz;
  T sum = 0;
  for (int dk = 0; dk < nk; ++dk)
    for (int dj = 0; dj < nj; ++dj)
      for (int di = 0; di < ni; ++di) {
        const int i = I * fx + di, j = J * fy + dj, k = K * fz + dk;
        sum += fb[i + (size_t)fmx * (j + (size_t)fmy * k)];
      }
  cb[I + (size_t)mx * (J + (size_t)my * K)] = sum / (T)(ni * nj * nk);
}


// ------------------------------------------------------- coarse-level tail
// All levels from `first` down to the coarsest run in one workgroup of 1024
// threads with coefficients, right-hand sides and corrections held in LDS,
// so that each smoothing pass costs a barrier instead of a kernel launch.
template <typename T>
__device__ __forceinline__ void tail_gs(const Dims& n, T h2, const T* bx, const T* by, const T* bz,
                                        const T* b, T* e, int colour, bool first) {
  const int N = n.nx * n.ny * n.nz;
  const int sxy = n.nx * n.ny;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const int i = c % n.nx;
    const int j = (c / n.nx) % n.ny;
    const int k = c / sxy;
    const bool mine = ((i + j + k) & 1) == colour;
    if (!mine) {
      if (first) e[c] = (T)0;
      continue;
    }
    const int fx = i + (n.nx + 1) * (j + n.ny * k);
    const int fy = i + n.nx * (j + (n.ny + 1) * k);
    const T bw = bx[fx], be = bx[fx + 1], bs = by[fy], bn = by[fy + n.nx], bd = bz[c], bu = bz[c + sxy];
    const bool top = (k == n.nz - 1);
    const T diag = bw + be + bs + bn + bd + (top ? (T)2 * bu : bu);
    T num = h2 * b[c];
    if (!first) {
      num += bw * e[i > 0 ? c - 1 : c] + be * e[i < n.nx - 1 ? c + 1 : c] +
             bs * e[j > 0 ? c - n.nx : c] + bn * e[j < n.ny - 1 ? c + n.nx : c] +
             bd * e[k > 0 ? c - sxy : c] + (top ? (T)0 : bu * e[c + sxy]);
    }
    e[c] = num / diag;
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(1024) k_vcycle_tail(TailDesc<T> D) {
  extern __shared__ double tail_smem[];
  T* sm = reinterpret_cast<T*>(tail_smem);
  const int nl = D.nl;
  // stage coefficients of every tail level and the first right-hand side
  for (int l = 0; l < nl; ++l) {
    const Dims n = D.n[l];
    const int mu = (n.nx + 1) * n.ny * n.nz, mv = n.nx * (n.ny + 1) * n.nz, mw = n.nx * n.ny * (n.nz + 1);
    for (int q = threadIdx.x; q < mu; q += blockDim.x) sm[D.obx[l] + q] = D.gbx[l][q];
    for (int q = threadIdx.x; q < mv; q += blockDim.x) sm[D.oby[l] + q] = D.gby[l][q];
    for (int q = threadIdx.x; q < mw; q += blockDim.x) sm[D.obz[l] + q] = D.gbz[l][q];
  }
  {
    const int N0 = D.n[0].nx * D.n[0].ny * D.n[0].nz;
    for (int q = threadIdx.x; q < N0; q += blockDim.x) sm[D.ob[0] + q] = D.gb[q];
  }
  __syncthreads();
  auto smooth = [&](int l, int first_colour, int pairs, bool from_zero) {
    const Dims n = D.n[l];
    const T *bx = sm + D.obx[l], *by = sm + D.oby[l], *bz = sm + D.obz[l], *b = sm + D.ob[l];
    T* e = sm + D.oe[l];
    for (int s = 0; s < pairs; ++s) {
      tail_gs<T>(n, D.h2[l], bx, by, bz, b, e, first_colour, from_zero && s == 0);
      tail_gs<T>(n, D.h2[l], bx, by, bz, b, e, 1 - first_colour, false);
    }
  };
  auto zero = [&](int l) {
    const int N = D.n[l].nx * D.n[l].ny * D.n[l].nz;
    T* e = sm + D.oe[l];
    for (int c = threadIdx.x; c < N; c += blockDim.x) e[c] = (T)0;
    __syncthreads();
  };
  // down-leg
  for (int l = 0; l < nl - 1; ++l) {
    if (D.nu_pre > 0)
      smooth(l, 0, D.nu_pre, true);
    else
      zero(l);
    const Dims nf = D.n[l], nc = D.n[l + 1];
    const int fx = D.f[l][0], fy = D.f[l][1], fz = D.f[l][2];
    const T *bx = sm + D.obx[l], *by = sm + D.oby[l], *bz = sm + D.obz[l], *b = sm + D.ob[l];
    const T* e = sm + D.oe[l];
    T* bc = sm + D.ob[l + 1];
    const T ih2 = (T)1 / D.h2[l];
    const T inv = (T)1 / (T)(fx * fy * fz);
    const int Nc = nc.nx * nc.ny * nc.nz;
    const int sxy = nf.nx * nf.ny;
    for (int C = threadIdx.x; C < Nc; C += blockDim.x) {
      const int I = C % nc.nx, J = (C / nc.nx) % nc.ny, K = C / (nc.nx * nc.ny);
      T sum = 0;
      for (int dk = 0; dk < fz; ++dk)
        for (int dj = 0; dj < fy; ++dj)
          for (int di = 0; di < fx; ++di) {
            const int i = fx * I + di, j = fy * J + dj, k = fz * K + dk;
            const int c = i + nf.nx * (j + nf.ny * k);
            const int ix = i + (nf.nx + 1) * (j + nf.ny * k);
            const int iy = i + nf.nx * (j + (nf.ny + 1) * k);
            const T xc = e[c];
            T acc = bx[ix] * (xc - e[i > 0 ? c - 1 : c]) + bx[ix + 1] * (xc - e[i < nf.nx - 1 ? c + 1 : c]) +
                    by[iy] * (xc - e[j > 0 ? c - nf.nx : c]) +
                    by[iy + nf.nx] * (xc - e[j < nf.ny - 1 ? c + nf.nx : c]) +
                    bz[c] * (xc - e[k > 0 ? c - sxy : c]);
            acc += (k < nf.nz - 1) ? bz[c + sxy] * (xc - e[c + sxy]) : (T)2 * bz[c + sxy] * xc;
            sum += b[c] - ih2 * acc;
          }
      bc[C] = sum * inv;
    }
    __syncthreads();
  }
  // coarsest level: sweeps forward (red, black) then backward (black, red) from zero
  {
    const int l = nl - 1;
    if (D.coarse_sweeps > 0) {
      smooth(l, 0, D.coarse_sweeps, true);
      smooth(l, 1, D.coarse_sweeps, false);
    } else {
      zero(l);
    }
  }
  // up-leg
  for (int l = nl - 2; l >= 0; --l) {
    const Dims nf = D.n[l], nc = D.n[l + 1];
    const int fx = D.f[l][0], fy = D.f[l][1], fz = D.f[l][2];
    T* e = sm + D.oe[l];
    const T* ec = sm + D.oe[l + 1];
    const int N = nf.nx * nf.ny * nf.nz;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      const int i = c % nf.nx, j = (c / nf.nx) % nf.ny, k = c / (nf.nx * nf.ny);
      e[c] += ec[(i / fx) + nc.nx * ((j / fy) + nc.ny * (k / fz))];
    }
    __syncthreads();
    smooth(l, 1, D.nu_post, false);
  }
  {
    const int N0 = D.n[0].nx * D.n[0].ny * D.n[0].nz;
    for (int q = threadIdx.x; q < N0; q += blockDim.x) D.ge[q] = sm[D.oe[0] + q];
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

// ------------------------------------------------------------------ CG (FP64)
#define CELL_INDEX                                              \
  const int i = blockIdx.x * blockDim.x + threadIdx.x;          \
  const int j = blockIdx.y * blockDim.y + threadIdx.y;          \
  const int k = blockIdx.z * blockDim.z + threadIdx.z;          \
  const bool inside = (i < n.nx && j < n.ny && k < n.nz);       \
  const size_t c = inside ? i + (size_t)n.nx * (j + (size_t)n.ny * k) : 0

// r = b - A x; partials (r.r, b.b)
__global__ void __launch_bounds__(256) k_resid_norm(Dims n, double ih2, const double* __restrict__ bx,
                                                    const double* __restrict__ by,
                                                    const double* __restrict__ bz,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r,
                                                    double* __restrict__ partials) {
  CELL_INDEX;
  double v[2] = {0.0, 0.0};
  if (inside) {
    const double bc = b[c];
    const double rc = bc - ih2 * stencil<double>(n, bx, by, bz, x, i, j, k, c);
    r[c] = rc;
    v[0] = rc * rc;
    v[1] = bc * bc;
  }
  block_partials<2>(v, partials);
}

// q = A d; partial d.q
__global__ void __launch_bounds__(256) k_spmv_dot(Dims n, double ih2, const double* __restrict__ bx,
                                                  const double* __restrict__ by,
                                                  const double* __restrict__ bz,
                                                  const double* __restrict__ d,
                                                  double* __restrict__ q,
                                                  double* __restrict__ partials) {
  CELL_INDEX;
  double v[1] = {0.0};
  if (inside) {
    const double qc = ih2 * stencil<double>(n, bx, by, bz, d, i, j, k, c);
    q[c] = qc;
    v[0] = d[c] * qc;
  }
  block_partials<1>(v, partials);
}

__global__ void __launch_bounds__(256) k_apply_A(Dims n, double ih2, const double* __restrict__ bx,
                                                 const double* __restrict__ by,
                                                 const double* __restrict__ bz,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y) {
  CELL_INDEX;
  if (inside) y[c] = ih2 * stencil<double>(n, bx, by, bz, x, i, j, k, c);
}

// x += alpha d; r -= alpha q; partial r.r
__global__ void __launch_bounds__(256) k_cg_update(Dims n, const double* __restrict__ scal,
                                                   const double* __restrict__ d,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ partials) {
  CELL_INDEX;
  double v[1] = {0.0};
  if (inside) {
    const double alpha = scal[S_ALPHA];
    x[c] += alpha * d[c];
    const double rc = r[c] - alpha * q[c];
    r[c] = rc;
    v[0] = rc * rc;
  }
  block_partials<1>(v, partials);
}

// partials (r.zn, r.z)
__global__ void __launch_bounds__(256) k_dots2(Dims n, const double* __restrict__ r,
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
  block_partials<2>(v, partials);
}

__global__ void __launch_bounds__(256) k_dot1(Dims n, const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              double* __restrict__ partials) {
  CELL_INDEX;
  double v[1] = {0.0};
  if (inside) v[0] = a[c] * b[c];
  block_partials<1>(v, partials);
}

// d = zn + beta d   (first: d = zn)
__global__ void __launch_bounds__(256) k_cg_dir(Dims n, const double* __restrict__ scal,
                                                const double* __restrict__ zn,
                                                double* __restrict__ d, int first) {
  CELL_INDEX;
  if (!inside) return;
  d[c] = first ? zn[c] : zn[c] + scal[S_BETA] * d[c];
}

// fixed-order sum of the per-block partials and the scalar recurrences
__global__ void __launch_bounds__(1024) k_finalize(const double* __restrict__ partials, int nparts,
                                                   int nv, int mode, double* __restrict__ scal) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nparts; q += 1024) {
    a += partials[nv * q];
    if (nv > 1) b += partials[nv * q + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  __shared__ double sa[16], sb[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sa[wid] = a;
    sb[wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int q = 0; q < 16; ++q) {
      a += sa[q];
      b += sb[q];
    }
    switch (mode) {
      case FIN_RESID0:
        scal[S_RR] = a;
        scal[S_BB] = b;
        break;
      case FIN_RHO:
        scal[S_RHO] = a;
        break;
      case FIN_ALPHA:
        scal[S_DQ] = a;
        scal[S_ALPHA] = scal[S_RHO] / a;
        break;
      case FIN_RR:
        scal[S_RR] = a;
        break;
      case FIN_BETA:
        scal[S_BETA] = (a - b) / scal[S_RHO];
        scal[S_RHO] = a;
        break;
      case FIN_TRR:
        scal[S_TRR] = a;
        break;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_gs(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e, int colour,
               int first, hipStream_t st, KTimer* kt) {
  Geo g = geo3((L.n.nx + 1) / 2, L.n.ny, L.n.nz);
  const bool fine = (L.h == L.h0);
  auto kern = fine ? k_gs<T, true> : k_gs<T, false>;
  if (kt && kt->n < kt->cap) {
    (void)hipStreamSynchronize(st);   // time the kernel alone, not its wait for the previous one
    hipExtLaunchKernelGGL(kern, g.grid, g.block, 0, st, kt->ev[2 * kt->n], kt->ev[2 * kt->n + 1], 0, L.n,
                          (T)(L.h * L.h), bx, by, bz, b, e, colour, first);
    ++kt->n;
    return;
  }
  hipLaunchKernelGGL(kern, g.grid, g.block, 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b, e, colour, first);
}

template <typename T>
void launch_resid_restrict(const Level& F, const T* bx, const T* by, const T* bz, const T* b,
                           const T* e, const Level& C, T* bc, hipStream_t st) {
  Geo g = geo3(C.n.nx, C.n.ny, C.n.nz);
  const T ih2 = (T)(1.0 / (F.h * F.h));
  const T inv = (T)(1.0 / (F.f[0] * F.f[1] * F.f[2]));
  hipLaunchKernelGGL(k_resid_restrict<T>, g.grid, g.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], ih2, bx,
                     by, bz, b, e, C.n, inv, bc);
}

template <typename T>
void launch_prolong(const Level& F, T* e, const Level& C, const T* ec, hipStream_t st) {
  Geo g = geo3(F.n.nx, F.n.ny, F.n.nz);
  hipLaunchKernelGGL(k_prolong<T>, g.grid, g.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], e, C.n, ec);
}

template <typename T>
void launch_coarse_solve(const Level& L, const T* bx, const T* by, const T* bz, const T* b, T* e,
                         int sweeps, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(256), 0, st, L.n, (T)(L.h * L.h), bx, by, bz, b,
                     e, sweeps);
}

template <typename T>
void launch_coarsen_beta(const Level& F, const T* fbx, const T* fby, const T* fbz, const Level& C,
                         T* cbx, T* cby, T* cbz, hipStream_t st) {
  Geo gx = geo3(C.n.nx + 1, C.n.ny, C.n.nz);
  hipLaunchKernelGGL((k_coarsen_beta<T, 0>), gx.grid, gx.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], fbx,
                     C.n, cbx);
  Geo gy = geo3(C.n.nx, C.n.ny + 1, C.n.nz);
  hipLaunchKernelGGL((k_coarsen_beta<T, 1>), gy.grid, gy.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], fby,
                     C.n, cby);
  Geo gz = geo3(C.n.nx, C.n.ny, C.n.nz + 1);
  hipLaunchKernelGGL((k_coarsen_beta<T, 2>), gz.grid, gz.block, 0, st, F.n, F.f[0], F.f[1], F.f[2], fbz,
                     C.n, cbz);
}

template <typename T>
void launch_vcycle_tail(const TailDesc<T>& D, size_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(k_vcycle_tail<T>, dim3(1), dim3(kTailThreads), lds_bytes, st, D);
}

template <typename T>
void launch_fill(T* a, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
}

void launch_d2f(const double* a, float* b, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

void launch_f2d(const float* a, double* b, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}

int cg_blocks(const Dims& n) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  return (int)(g.grid.x * g.grid.y * g.grid.z);
}

void launch_resid_norm(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                       const double* b, const double* x, double* r, double* partials, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_resid_norm, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, b, x, r,
                     partials);
}

void launch_spmv_dot(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                     const double* d, double* q, double* partials, hipStream_t st, KTimer* kt) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  if (kt && kt->n < kt->cap) {
    (void)hipStreamSynchronize(st);
    hipExtLaunchKernelGGL(k_spmv_dot, g.grid, g.block, 0, st, kt->ev[2 * kt->n], kt->ev[2 * kt->n + 1],
                          0, n, 1.0 / (h * h), bx, by, bz, d, q, partials);
    ++kt->n;
    return;
  }
  hipLaunchKernelGGL(k_spmv_dot, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, d, q, partials);
}

void launch_apply_A(const Dims& n, double h, const double* bx, const double* by, const double* bz,
                    const double* x, double* y, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_apply_A, g.grid, g.block, 0, st, n, 1.0 / (h * h), bx, by, bz, x, y);
}

void launch_cg_update(const Dims& n, const double* scal, const double* d, const double* q, double* x,
                      double* r, double* partials, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_cg_update, g.grid, g.block, 0, st, n, scal, d, q, x, r, partials);
}

void launch_dots2(const Dims& n, const double* r, const double* zn, const double* z, double* partials,
                  hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_dots2, g.grid, g.block, 0, st, n, r, zn, z, partials);
}

void launch_dot1(const Dims& n, const double* a, const double* b, double* partials, hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_dot1, g.grid, g.block, 0, st, n, a, b, partials);
}

void launch_cg_dir(const Dims& n, const double* scal, const double* zn, double* d, int first,
                   hipStream_t st) {
  Geo g = geo3(n.nx, n.ny, n.nz);
  hipLaunchKernelGGL(k_cg_dir, g.grid, g.block, 0, st, n, scal, zn, d, first);
}

void launch_finalize(const double* partials, int nparts, int mode, double* scal, hipStream_t st) {
  const int nv = (mode == FIN_RESID0 || mode == FIN_BETA || mode == FIN_TRR) ? 2 : 1;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, partials, nparts, nv, mode, scal);
}

#define NSK_INST(T)                                                                                 \
  template void launch_gs<T>(const Level&, const T*, const T*, const T*, const T*, T*, int, int,    \
                             hipStream_t, KTimer*);                                                 \
  template void launch_resid_restrict<T>(const Level&, const T*, const T*, const T*, const T*,      \
                                         const T*, const Level&, T*, hipStream_t);                  \
  template void launch_prolong<T>(const Level&, T*, const Level&, const T*, hipStream_t);           \
  template void launch_coarse_solve<T>(const Level&, const T*, const T*, const T*, const T*, T*, int, \
                                       hipStream_t);                                                \
  template void launch_coarsen_beta<T>(const Level&, const T*, const T*, const T*, const Level&, T*, \
                                       T*, T*, hipStream_t);                                        \
  template void launch_fill<T>(T*, size_t, hipStream_t);                                            \
  template void launch_vcycle_tail<T>(const TailDesc<T>&, size_t, hipStream_t);
NSK_INST(double)
NSK_INST(float)
#undef NSK_INST

}  // namespace nsk
