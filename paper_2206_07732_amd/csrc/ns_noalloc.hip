// The CFL rule (ns_cfl_dt) for callers that cannot allocate: no context, no
// workspace argument, no allocation of any kind.  Its only scratch is a
// file-scope device array of per-block maxima; the kernel walks the cells
// with a fixed number of blocks, so the array's size does not depend on the
// grid.  The time step is formed on the device and stored to a caller-owned
// device double, so the call is stream-ordered and never waits.
#include <algorithm>
#include <mutex>

#include "ns_internal.h"

namespace nsk {
namespace {

constexpr int kNoAllocBlocks = 2048;   // blocks of the walk = partials in the scratch
constexpr int kMaxDevices = 64;

// per-block maxima of the last call on this device (16 KiB; every GPU the
// library runs on holds its own copy until the process ends)
static __device__ __align__(256) double scratch[kNoAllocBlocks];

std::mutex g_mu;
double* g_scratch[kMaxDevices];        // the array's device address, per device

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// Each block walks cells blockIdx.x * 256 + tid, then a grid's worth
// further on, keeping the largest |u_c| + |v_c| + |w_c| (each cell velocity
// the mean of its two faces, a value that is not finite counting as
// infinite); part[blockIdx.x] gets the block's maximum.
__global__ void __launch_bounds__(256) k_cfl_walk(Dims n, const double* __restrict__ u, const double* __restrict__ v,
                                                  const double* __restrict__ w, double* __restrict__ part) {
  const long nc = (long)n.nx * n.ny * n.nz;
  const size_t sxy = (size_t)n.nx * n.ny;
  double m = 0.0;
  for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < nc; c += (long)gridDim.x * 256) {
    const int i = (int)(c % n.nx);
    const long r = c / n.nx;
    const int j = (int)(r % n.ny), k = (int)(r / n.ny);
    const size_t fu = i + (size_t)(n.nx + 1) * (j + (size_t)n.ny * k);
    const size_t fv = i + (size_t)n.nx * (j + (size_t)(n.ny + 1) * k);
    const double uc = 0.5 * fabs(u[fu] + u[fu + 1]);
    const double vc = 0.5 * fabs(v[fv] + v[fv + n.nx]);
    const double wc = 0.5 * fabs(w[c] + w[c + sxy]);
    const double s = (uc + vc) + wc;
    m = fmax(m, isfinite(s) ? s : INFINITY);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
}

// *dt = min(cfl h / m, dt_max) with m the maximum of the nb partials (dt_max
// for m = 0, NaN for a velocity that is not finite)
__global__ void __launch_bounds__(256) k_cfl_dt_from(const double* __restrict__ part, int nb, double h, double cfl,
                                                     double dt_max, double* __restrict__ dt) {
  double m = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256) m = fmax(m, part[q]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
    double r;
    if (!isfinite(m))
      r = NAN;
    else if (!(m > 0.0))
      r = dt_max;
    else {
      const double t = cfl * h / m;
      r = t < dt_max ? t : dt_max;
    }
    *dt = r;
  }
}

}  // namespace
}  // namespace nsk

using namespace nsk;

extern "C" ns_status ns_cfl_dt_noalloc(int nx, int ny, int nz, double h, const double* u, const double* v,
                                       const double* w, double cfl, double dt_max, double* dt_dev,
                                       void* hip_stream) {
  if (nx < 2 || ny < 1 || nz < 2) return NS_EINVAL;
  const double x = nx, y = ny, z = nz;
  if (std::max(std::max((x + 1) * y * z, x * (y + 1) * z), x * y * (z + 1)) > 2.0e9) return NS_EINVAL;
  if (!(h > 0.0) || !(cfl > 0.0) || !(dt_max > 0.0)) return NS_EINVAL;
  for (const void* p : {(const void*)u, (const void*)v, (const void*)w, (const void*)dt_dev})
    if (!p || ((uintptr_t)p & 7) != 0) return NS_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NS_EHIP;
  double* part = nullptr;
  if (scratch_ptr(dev, &part) != hipSuccess) return NS_EHIP;
  const long nc = (long)nx * ny * nz;
  const int nb = (int)std::min<long>(kNoAllocBlocks, (nc + 255) / 256);
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_cfl_walk, dim3(nb), dim3(256), 0, st, Dims{nx, ny, nz}, u, v, w, part);
  hipLaunchKernelGGL(k_cfl_dt_from, dim3(1), dim3(256), 0, st, part, nb, h, cfl, dt_max, dt_dev);
  return hipGetLastError() == hipSuccess ? NS_OK : NS_EHIP;
}
