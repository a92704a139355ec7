// Learned initial guess for the pressure projection on gfx950: a 3-level
// convolutional encoder-decoder (16/32/64 channels, 3x3x3 kernels, ReLU,
// 2x2x2 average pooling, nearest upsampling, skip connections by channel
// concatenation, 1x1x1 head) in bfloat16 with FP32 accumulation on the
// matrix cores, with its hand-written backward pass and Adam optimiser.
//
// Layout: activations are channels-last bfloat16, a[v * C + c] with the voxel
// index v = x + nx (y + ny z) of their resolution.  The first layer's four
// input channels are padded to 16 (zeros), so every convolution has C_in and
// C_out in multiples of 16.  A convolution is an implicit GEMM,
//   Y[v][co] = sum_{tap, ci} X[v + tap][ci] W[co][tap][ci],
// M = voxels, N = C_out, K = 27 C_in, computed 16 voxels x 16 channels x 16
// inputs at a time by v_mfma_f32_16x16x16_bf16:
//   A (16 voxels x 16 inputs):  lane l holds row l%16, inputs 4(l/16)..+3
//   B (16 inputs x 16 outputs): lane l holds column l%16, inputs 4(l/16)..+3
//   D (16 voxels x 16 outputs): lane l holds column l%16, rows 4(l/16)..+3
// The backward pass w.r.t. the input is the same convolution with the
// kernel flipped in space and its channel roles swapped; the weight gradient
// is a GEMM over voxels per tap, summed over voxel chunks in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "ns_internal.h"

namespace nsk {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct VDims {
  int nx, ny, nz;
};

__device__ __forceinline__ long vox_count(const VDims& d) { return (long)d.nx * d.ny * d.nz; }

// ------------------------------------------------------------ convolution
// 3x3x3 convolution with zero padding as an implicit GEMM on the matrix
// cores.  A block computes a 16 x 4 x 4 tile of output voxels for every
// output channel; wave w owns the four x-rows of z-plane w of the tile.  The
// input is staged in LDS 16 channels at a time with its one-voxel halo
// (18 x 6 x 6 voxels, 20.7 KB), and each v_mfma_f32_16x16x32_bf16 takes two
// taps x 16 input channels as its K = 32 (a 28th, zero tap pads the last
// pair).  With k = 16 (tap - 2p) + ci for tap pair p:
//   A (16 voxels x 32 k): lane l holds voxel row l%16, k = 8(l/16)..+7
//   B (32 k x 16 out):    lane l holds output column l%16, k = 8(l/16)..+7
//   D (16 x 16):          lane l holds column l%16, rows 4(l/16)..+3
// Each weight fragment read from the cache feeds the wave's four rows.
// The input is the channel concatenation of a tensor at this resolution
// (channels [0, ca), channel stride sa) and, for channels [ca, CIN), a tensor
// at half resolution read through nearest upsampling (channel stride sb), so
// the decoder never materialises its upsampled inputs.
// EPI 0: + bias, ReLU; 1: plain (gradient w.r.t. the input); 2: + bias,
// ReLU, then the 1x1x1 head 16 -> 1 into delta (FP32), storing the
// activation only when Y is given.
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2, kHV = kHX * kHY * kHZ;
// The two 8-channel halves of a staged chunk live in separate planes
// (16-byte entries).  Adjacent 16-lane groups of an A-fragment read take the
// two halves of the same voxels; the LDS serves half of one group with half
// of the next, which is free of bank conflicts only when their entries are a
// multiple of 16 apart, so the plane stride is a multiple of 16 entries.
constexpr int kPlane = (kHV + 15) / 16 * 16;

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }

// offset of tap (dz, dy, dx) = (tap / 9, tap / 3 % 3, tap % 3) in the halo tile (0 for the pad tap)
__host__ __device__ constexpr int tap_off(int tap) {
  return tap >= 27 ? 0 : ((tap / 9) * kHY + (tap / 3) % 3) * kHX + tap % 3;
}

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(256) k_conv(VDims d, const uint16_t* __restrict__ XA, int sa, int ca,
                                              const uint16_t* __restrict__ XB, int sb,
                                              const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                              uint16_t* __restrict__ Y, int ys, int yo,
                                              const float* __restrict__ hw, const float* __restrict__ hb,
                                              float* __restrict__ delta) {
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels in multiples of 16");
  static_assert(EPI != 2 || COUT == 16, "the fused head takes 16 channels");
  constexpr int NT = COUT / 16, NC = CIN / 16;
  constexpr int NE = (2 * kHV + 255) / 256;   // 16-byte tile pieces per thread
  // Weight fragments are loaded per tap pair (they stay in the caches):
  // holding a chunk's fourteen ahead in registers cost two of the wide
  // layers a wave per SIMD of occupancy, and the forward 9%.
  __shared__ u32x4 tile[2][2 * kPlane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
  const int cnx = d.nx >> 1, cny = d.ny >> 1;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  // this thread's tile pieces: fine and coarse voxel of each, in-grid mask
  int vf[NE], vc[NE];
  unsigned ok = 0;
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = tid + 256 * i, hv = e >> 1;
    const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    vf[i] = vc[i] = 0;
    if (e < 2 * kHV && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz) {
      ok |= 1u << i;
      vf[i] = gx + d.nx * (gy + d.ny * gz);
      vc[i] = (gx >> 1) + cnx * ((gy >> 1) + cny * (gz >> 1));
    }
  }
  const int half8 = 8 * (tid & 1);   // every piece of a thread has the same half (256 is even)
  u32x4 pre[NE];
  auto fetch = [&](int c) {
    const bool fromA = 16 * c < ca;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      pre[i] = zero;
      if (ok >> i & 1u) {
        const uint16_t* src = fromA ? XA + (long)vf[i] * sa + 16 * c + half8
                                    : XB + (long)vc[i] * sb + (16 * c - ca) + half8;
        pre[i] = *reinterpret_cast<const u32x4*>(src);
      }
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = tid + 256 * i;
      if (e < 2 * kHV) tile[buf][(e & 1) * kPlane + (e >> 1)] = pre[i];
    }
  };
  // weight fragment of tap pair p, output tile t, chunk c
  const uint16_t* wl = W + (long)r * 27 * CIN + (long)(kg >> 1) * CIN + 8 * (kg & 1);
  auto wfrag = [&](int p, int t, int c) -> bf16x8 {
    const int tap = 2 * p + (kg >> 1);
    return as_bf16x8(tap < 27 ? *reinterpret_cast<const u32x4*>(wl + (long)t * 16 * 27 * CIN + 2 * p * CIN + 16 * c)
                              : zero);
  };
  const int lbase = (kg & 1) * kPlane + wave * kHY * kHX + r;   // this lane's A piece for tap 0, row 0
  f32x4 acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  put(0);
  __syncthreads();
  // The tap pairs are software-pipelined: the four activation fragments of
  // pair p + 1 are read from LDS, and the weight fragments of pair p + WD
  // requested, before pair p's MFMAs issue, so that an MFMA never waits on
  // the read just before it (with the reads one fragment ahead, each MFMA
  // waited out an LDS round trip and the layer ran at a quarter of the MFMA
  // peak).  The first pairs' weights are requested before the next chunk's
  // tile pieces, which the in-order load counter would otherwise make them
  // wait behind.
  constexpr int WD = NT == 1 ? 3 : 1;   // weight prefetch distance in tap pairs
  bf16x8 aq[2][4], bq[WD + 1][NT];
#pragma unroll 1
  for (int c = 0; c < NC; ++c) {
    const u32x4* T = tile[c & 1] + lbase;
    auto lda = [&](int p, bf16x8 (&a)[4]) {
      const bool tv = 2 * p + (kg >> 1) < 27;
      const int o = (kg >> 1) ? tap_off(2 * p + 1) : tap_off(2 * p);
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = as_bf16x8(tv ? T[o + m * kHX] : zero);
    };
#pragma unroll
    for (int q = 0; q < WD; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t) bq[q][t] = wfrag(q, t, c);
    if (c + 1 < NC) fetch(c + 1);
    lda(0, aq[0]);
#pragma unroll
    for (int p = 0; p < 14; ++p) {
      if (p + WD < 14) {
#pragma unroll
        for (int t = 0; t < NT; ++t) bq[(p + WD) % (WD + 1)][t] = wfrag(p + WD, t, c);
      }
      if (p + 1 < 14) lda(p + 1, aq[(p + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[p & 1][m], bq[p % (WD + 1)][t], acc[m][t], 0, 0, 0);
    }
    if (c + 1 < NC) put((c + 1) & 1);
    __syncthreads();
  }
  // Epilogue.  Up to 64 output channels the wave's 64 voxels x COUT results
  // are transposed through its own slice of the (now idle) tile memory and
  // stored as 16-byte pieces of 8 channels; wider layers store directly.
  constexpr bool STAGE = COUT <= 64;
  static_assert(!STAGE || 4 * 64 * COUT * 2 <= (int)sizeof(tile), "staging fits in the tile");
  const bool store = (EPI != 2) || (Y != nullptr);
  uint16_t* stg = reinterpret_cast<uint16_t*>(&tile[0][0]) + wave * 64 * COUT;
  const int z = z0 + wave;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int y = y0 + m;
    const long row = (long)d.nx * (y + (long)d.ny * z);
    float hs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + r;
      const float bb = (EPI == 1) ? 0.f : bias[co];
      const float wh = (EPI == 2) ? hw[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * kg + i;
        float val = acc[m][t][i] + bb;
        if (EPI != 1) val = fmaxf(val, 0.f);
        const uint16_t q = f2bf(val);
        if (STAGE)
          stg[(m * 16 + 4 * kg + i) * COUT + co] = q;
        else if (store && x < d.nx && y < d.ny && z < d.nz)
          Y[(row + x) * ys + yo + co] = q;
        if (EPI == 2) hs[i] = wh * bf2f(q);
      }
    }
    if (EPI == 2) {
      // sum the 16 channels: the 16 lanes of one row group
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) hs[i] += __shfl_xor(hs[i], o, 16);
      if (r == 0 && y < d.ny && z < d.nz) {
        const float b0 = hb[0];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + 4 * kg + i;
          if (x < d.nx) delta[row + x] = hs[i] + b0;
        }
      }
    }
  }
  if (STAGE && store) {
    __syncthreads();
    constexpr int G = COUT / 8;   // 16-byte pieces per voxel
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int q = lane + 64 * j, vl = q / G, cg = q % G;
      const int x = x0 + (vl & 15), y = y0 + (vl >> 4);
      if (x < d.nx && y < d.ny && z < d.nz)
        *reinterpret_cast<u32x4*>(Y + ((long)x + (long)d.nx * (y + (long)d.ny * z)) * ys + yo + 8 * cg) =
            *reinterpret_cast<const u32x4*>(stg + vl * COUT + 8 * cg);
    }
  }
}

// The same convolution with K running over 32 input channels of one tap
// (channel-major), for the half-resolution decoder layer at inference (96
// input channels).  With the K of an MFMA inside one tap, the activation
// fragment of halo row y serves the output rows y - dy for all three dy taps
// of a (dz, dx) pair: a wave reads its ten halo rows once per (dz, dx) and
// issues 24 NT MFMAs from them, where the tap-pair form reads one fragment
// per MFMA row group.  A block computes a 16 x 8 x 4 tile of output voxels;
// wave w owns the eight x-rows of z-plane w, so each weight fragment feeds
// eight MFMAs.  Input channels are staged 32 at a time into LDS as four
// planes of 8 channels (16-byte entries; the plane stride a multiple of 16
// entries, so a 16-lane group's reads stay free of bank conflicts).
// Epilogues as k_conv.  At 256 x 128 x 128 it runs the 96 -> 32 layer in
// 108 us against k_conv's 155; for the 48 -> 16 layer (a 16-channel
// remainder chunk, run half empty or as tap pairs) it measured 348 and
// 328 us against k_conv's 321, and for 32 -> 64 (an eighth of the voxels)
// 23.5 against 21 us, so those stay on k_conv.  Its single-buffered 68 KB
// tile leaves two blocks per compute unit; a chunk's staging is hidden only
// by the other block.
constexpr int kCX = 16, kCY = 8, kCZ = 4;
constexpr int kCHX = kCX + 2, kCHY = kCY + 2, kCHZ = kCZ + 2, kCHV = kCHX * kCHY * kCHZ;
constexpr int kCPlane = (kCHV + 15) / 16 * 16;

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(256) k_conv_cm(VDims d, const uint16_t* __restrict__ XA, int sa, int ca,
                                                 const uint16_t* __restrict__ XB, int sb,
                                                 const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                                 uint16_t* __restrict__ Y, int ys, int yo,
                                                 const float* __restrict__ hw, const float* __restrict__ hb,
                                                 float* __restrict__ delta) {
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels in multiples of 16");
  static_assert(EPI != 1, "the gradient w.r.t. the input runs on k_conv");
  static_assert(EPI != 2 || COUT == 16, "the fused head takes 16 channels");
  static_assert(CIN % 32 == 0, "whole chunks of 32 input channels");
  constexpr int NT = COUT / 16, NC = CIN / 32;
  __shared__ u32x4 tile[4 * kCPlane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int x0 = blockIdx.x * kCX, y0 = blockIdx.y * kCY, z0 = blockIdx.z * kCZ;
  const int cnx = d.nx >> 1, cny = d.ny >> 1;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  f32x4 acc[kCY][NT];
#pragma unroll
  for (int m = 0; m < kCY; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // weight fragment: output column r of tile t, channels 32 c + 8 kg .. + 7 of tap
  const uint16_t* wl = W + (long)r * 27 * CIN + 8 * kg;
  auto wfrag = [&](int tap, int t, int c) -> bf16x8 {
    return as_bf16x8(*reinterpret_cast<const u32x4*>(wl + (long)t * 16 * 27 * CIN + (long)tap * CIN + 32 * c));
  };
#pragma unroll 1
  for (int c = 0; c < NC; ++c) {
    if (c > 0) __syncthreads();   // every wave is done with the previous chunk
    // stage channels [32 c, 32 c + 32): lanes 16 g .. 16 g + 15 take group g
    // (8 channels) of 16 consecutive halo voxels, so a wave reads 16 whole
    // 64-byte voxel slices and writes 16 consecutive entries of each plane.
    // Every load is issued (from a clamped address) before the first write.
    constexpr int NS = (kCHV + 63) / 64;
    const int ch = 32 * c + 8 * kg;
    u32x4 v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int hv = 64 * s + 16 * wave + r;
      const int hx = hv % kCHX, hy = (hv / kCHX) % kCHY, hz = hv / (kCHX * kCHY);
      const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
      const bool in = hv < kCHV && gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz;
      const int cx = in ? gx : 0, cy = in ? gy : 0, cz = in ? gz : 0;
      const uint16_t* src = ch < ca ? XA + (long)(cx + d.nx * (cy + d.ny * cz)) * sa + ch
                                    : XB + (long)((cx >> 1) + cnx * ((cy >> 1) + cny * (cz >> 1))) * sb + (ch - ca);
      const u32x4 w = *reinterpret_cast<const u32x4*>(src);
      v[s] = in ? w : zero;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int hv = 64 * s + 16 * wave + r;
      if (hv < kCHV) tile[kg * kCPlane + hv] = v[s];
    }
    __syncthreads();
    const u32x4* T = tile + kg * kCPlane + r;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        bf16x8 b[3][NT];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int t = 0; t < NT; ++t) b[dy][t] = wfrag(9 * dz + 3 * dy + dx, t, c);
        bf16x8 a[kCHY];
#pragma unroll
        for (int hy = 0; hy < kCHY; ++hy) a[hy] = as_bf16x8(T[((wave + dz) * kCHY + hy) * kCHX + dx]);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int m = 0; m < kCY; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
              acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m + dy], b[dy][t], acc[m][t], 0, 0, 0);
      }
    }
  }
  // Epilogue: + bias, ReLU, BF16; the wave's 128 voxels x COUT results are
  // transposed through its own slice of the tile memory and stored as
  // 16-byte pieces of 8 channels.
  static_assert(kCY * 16 * COUT * 2 * 4 <= (int)sizeof(tile), "staging fits in the tile");
  const bool store = (EPI != 2) || (Y != nullptr);
  __syncthreads();
  uint16_t* stg = reinterpret_cast<uint16_t*>(&tile[0]) + wave * kCY * 16 * COUT;
  const int z = z0 + wave;
#pragma unroll
  for (int m = 0; m < kCY; ++m) {
    const int y = y0 + m;
    const long row = (long)d.nx * (y + (long)d.ny * z);
    float hs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + r;
      const float bb = bias[co];
      const float wh = (EPI == 2) ? hw[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float val = fmaxf(acc[m][t][i] + bb, 0.f);
        const uint16_t q = f2bf(val);
        stg[(m * 16 + 4 * kg + i) * COUT + co] = q;
        if (EPI == 2) hs[i] = wh * bf2f(q);
      }
    }
    if (EPI == 2) {
      // sum the 16 channels: the 16 lanes of one row group
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) hs[i] += __shfl_xor(hs[i], o, 16);
      if (r == 0 && y < d.ny && z < d.nz) {
        const float b0 = hb[0];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + 4 * kg + i;
          if (x < d.nx) delta[row + x] = hs[i] + b0;
        }
      }
    }
  }
  if (store) {
    __syncthreads();
    constexpr int G = COUT / 8;   // 16-byte pieces per voxel
#pragma unroll
    for (int j = 0; j < 2 * G; ++j) {
      const int q = lane + 64 * j, vl = q / G, cg = q % G;
      const int x = x0 + (vl & 15), y = y0 + (vl >> 4);
      if (x < d.nx && y < d.ny && z < d.nz)
        *reinterpret_cast<u32x4*>(Y + ((long)x + (long)d.nx * (y + (long)d.ny * z)) * ys + yo + 8 * cg) =
            *reinterpret_cast<const u32x4*>(stg + vl * COUT + 8 * cg);
    }
  }
}

// First layer at inference: the four FP32 feature channels (channel-first,
// feat[c nv + v]) are converted to bfloat16 while staged in LDS (8 bytes per
// halo voxel), and K runs over (tap, channel) compactly, k = 4 tap + ci with
// 108 real entries padded to 128: four K = 32 steps instead of fourteen.
// Wc is [16 outputs][128 k].  Output: + bias, ReLU, bfloat16, channel stride ys.
__global__ void __launch_bounds__(256) k_conv_in(VDims d, const float* __restrict__ feat,
                                                 const uint16_t* __restrict__ Wc, const float* __restrict__ bias,
                                                 uint16_t* __restrict__ Y, int ys) {
  __shared__ u32x2 tile[kHV + 8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kg = lane >> 4;
  const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
  const long nv = vox_count(d);
  for (int e = threadIdx.x; e < kHV; e += 256) {
    const int hx = e % kHX, hy = (e / kHX) % kHY, hz = e / (kHX * kHY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    u32x2 val = {0u, 0u};
    if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz) {
      const long v = (long)gx + (long)d.nx * (gy + (long)d.ny * gz);
      val[0] = (uint32_t)f2bf(feat[v]) | ((uint32_t)f2bf(feat[nv + v]) << 16);
      val[1] = (uint32_t)f2bf(feat[2 * nv + v]) | ((uint32_t)f2bf(feat[3 * nv + v]) << 16);
    }
    tile[e] = val;
  }
  __syncthreads();
  f32x4 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int t0 = 8 * st + 2 * kg, t1 = t0 + 1;   // this lane's two taps
    const bf16x8 b = as_bf16x8(*reinterpret_cast<const u32x4*>(Wc + r * 128 + 32 * st + 8 * kg));
    const int o0 = ((t0 / 9) * kHY + (t0 / 3) % 3) * kHX + t0 % 3;
    const int o1 = ((t1 / 9) * kHY + (t1 / 3) % 3) * kHX + t1 % 3;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int base = (wave * kHY + m) * kHX + r;
      const u32x2 p0 = t0 < 27 ? tile[base + o0] : u32x2{0u, 0u};
      const u32x2 p1 = t1 < 27 ? tile[base + o1] : u32x2{0u, 0u};
      const u32x4 a = {p0[0], p0[1], p1[0], p1[1]};
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), b, acc[m], 0, 0, 0);
    }
  }
  // transpose through LDS and store 16-byte pieces (as in k_conv)
  __shared__ uint16_t stg_all[4 * 64 * 16];
  uint16_t* stg = stg_all + wave * 64 * 16;
  const float bb = bias[r];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) stg[(m * 16 + 4 * kg + i) * 16 + r] = f2bf(fmaxf(acc[m][i] + bb, 0.f));
  __syncthreads();
  const int z = z0 + wave;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = lane + 64 * j, vl = q >> 1, cg = q & 1;
    const int x = x0 + (vl & 15), y = y0 + (vl >> 4);
    if (x < d.nx && y < d.ny && z < d.nz)
      *reinterpret_cast<u32x4*>(Y + ((long)x + (long)d.nx * (y + (long)d.ny * z)) * ys + 8 * cg) =
          *reinterpret_cast<const u32x4*>(stg + vl * 16 + 8 * cg);
  }
}

// compact first-layer weights: Wc[co][4 tap + ci] from the padded FP32 master W[co][tap][16]
__global__ void k_compact_w0(const float* __restrict__ w, uint16_t* __restrict__ wc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 16 * 128) return;
  const int co = q / 128, k = q % 128, tap = k / 4, ci = k % 4;
  wc[q] = tap < 27 ? f2bf(w[(co * 27 + tap) * 16 + ci]) : (uint16_t)0;
}

// weight gradient of one tap: part[blk][tap][co][ci] = sum over this block's
// voxels of dY[v][co] X[v + tap][ci]
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_wgrad(VDims d, const uint16_t* __restrict__ X,
                                               const uint16_t* __restrict__ dY, int vox_per_block,
                                               float* __restrict__ part) {
  constexpr int NO = COUT / 16, NI = CIN / 16;
  __shared__ float red[4][COUT * CIN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int tap = blockIdx.y;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const long nv = vox_count(d);
  const long v_begin = (long)blockIdx.x * vox_per_block;
  const long v_end = v_begin + vox_per_block < nv ? v_begin + vox_per_block : nv;
  f32x4 acc[NO][NI];
#pragma unroll
  for (int a = 0; a < NO; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long vb = v_begin + 16 * wave; vb < v_end; vb += 64) {
    // voxels vb + 4 kq + i, i = 0..3, are this lane's k entries
    long nbv[4];
    bool live[4], in[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long v = vb + 4 * kq + i;
      live[i] = v < v_end;
      const int x = (int)(v % d.nx), y = (int)((v / d.nx) % d.ny), z = (int)(v / ((long)d.nx * d.ny));
      const int xx = x + dx, yy = y + dy, zz = z + dz;
      in[i] = live[i] && xx >= 0 && xx < d.nx && yy >= 0 && yy < d.ny && zz >= 0 && zz < d.nz;
      nbv[i] = in[i] ? (long)xx + (long)d.nx * (yy + (long)d.ny * zz) : 0;
    }
    bf16x4 A[NO], B[NI];
#pragma unroll
    for (int a = 0; a < NO; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) A[a][i] = live[i] ? (short)dY[(vb + 4 * kq + i) * COUT + a * 16 + row] : (short)0;
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) B[b][i] = in[i] ? (short)X[nbv[i] * CIN + b * 16 + row] : (short)0;
#pragma unroll
    for (int a = 0; a < NO; ++a)
#pragma unroll
      for (int b = 0; b < NI; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[a], B[b], acc[a][b], 0, 0, 0);
  }
  // D lane layout: column ci = b*16 + row, rows co = a*16 + 4 kq + i
#pragma unroll
  for (int a = 0; a < NO; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave][(a * 16 + 4 * kq + i) * CIN + b * 16 + row] = acc[a][b][i];
  __syncthreads();
  float* out = part + ((size_t)blockIdx.x * 27 + tap) * (COUT * CIN);
  for (int q = threadIdx.x; q < COUT * CIN; q += 256) out[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// g[(co * 27 + tap) * CIN + ci] = sum over blocks of part[blk][tap][co][ci]
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nblk, int cin, int cout,
                               float* __restrict__ g) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = 27 * cout * cin;
  if (q >= per) return;
  const int tap = q / (cout * cin), r = q % (cout * cin), co = r / cin, ci = r % cin;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * per + q];
  g[((size_t)co * 27 + tap) * cin + ci] = s;
}

// per-block channel sums of dY (bias gradient), then their fixed-order total:
// thread t handles channel t % C of voxels v0 + t / C, v0 + t / C + 256 / C, ...
__global__ void __launch_bounds__(256) k_bias_part(long nv, int C, const uint16_t* __restrict__ dY,
                                                   int vox_per_block, float* __restrict__ part) {
  __shared__ float sm[256];
  const long v0 = (long)blockIdx.x * vox_per_block;
  const long v1 = v0 + vox_per_block < nv ? v0 + vox_per_block : nv;
  const int c = threadIdx.x % C, lanes = 256 / C, r = threadIdx.x / C;
  float s = 0.f;
  if (r < lanes)
    for (long v = v0 + r; v < v1; v += lanes) s += bf2f(dY[v * C + c]);
  sm[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < C) {
    float t = 0.f;
    for (int q = 0; q < lanes; ++q) t += sm[q * C + threadIdx.x];
    part[(size_t)blockIdx.x * C + threadIdx.x] = t;
  }
}

__global__ void k_bias_reduce(const float* __restrict__ part, int nblk, int C, float* __restrict__ g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * C + c];
  g[c] = s;
}

// ------------------------------------------------------- resampling, head
// 2x2x2 average of a fine tensor (channel stride is, offset io) into a dense
// coarse one; a thread takes 8 channels of one coarse voxel
__global__ void k_pool(VDims fine, const uint16_t* __restrict__ in, int is, int io, int C,
                       uint16_t* __restrict__ out) {
  const VDims c{fine.nx / 2, fine.ny / 2, fine.nz / 2};
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = C / 8;
  if (q >= vox_count(c) * groups) return;
  const int g = (int)(q % groups);
  const long v = q / groups;
  const int X = (int)(v % c.nx), Y = (int)((v / c.nx) % c.ny), Z = (int)(v / ((long)c.nx * c.ny));
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        const long f = (2L * X + i) + (long)fine.nx * ((2L * Y + j) + (long)fine.ny * (2L * Z + k));
        const u32x4 w = *reinterpret_cast<const u32x4*>(in + f * is + io + 8 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          s[2 * e] += __uint_as_float(w[e] << 16);
          s[2 * e + 1] += __uint_as_float(w[e] & 0xFFFF0000u);
        }
      }
  u32x4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = (uint32_t)f2bf(s[2 * e] * 0.125f) | ((uint32_t)f2bf(s[2 * e + 1] * 0.125f) << 16);
  *reinterpret_cast<u32x4*>(out + v * C + 8 * g) = o;
}

// nearest x2 upsampling of a dense coarse tensor into a fine one (stride os, offset oo)
__global__ void k_up(VDims coarse, const uint16_t* __restrict__ in, int C, uint16_t* __restrict__ out,
                     int os, int oo) {
  const VDims f{coarse.nx * 2, coarse.ny * 2, coarse.nz * 2};
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= vox_count(f) * C) return;
  const int ch = (int)(q % C);
  const long v = q / C;
  const int x = (int)(v % f.nx), y = (int)((v / f.nx) % f.ny), z = (int)(v / ((long)f.nx * f.ny));
  const long p = (x / 2) + (long)coarse.nx * ((y / 2) + (long)coarse.ny * (z / 2));
  out[v * os + oo + ch] = in[p * C + ch];
}

// delta = b + sum_c w_c a_c (1x1x1 head, FP32 out)
__global__ void k_head(long nv, const uint16_t* __restrict__ a, const float* __restrict__ w,
                       const float* __restrict__ b, float* __restrict__ delta) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  float s = b[0];
#pragma unroll
  for (int c = 0; c < 16; ++c) s += w[c] * bf2f(a[v * 16 + c]);
  delta[v] = s;
}

// ------------------------------------------------------------- backward
// d5 = ddelta w_c (a_c > 0)
__global__ void k_head_bwd(long nv, const float* __restrict__ dd, const uint16_t* __restrict__ a,
                           const float* __restrict__ w, uint16_t* __restrict__ d5) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nv * 16) return;
  const long v = q / 16;
  const int c = (int)(q % 16);
  d5[q] = f2bf(a[q] != 0 && bf2f(a[q]) > 0.f ? dd[v] * w[c] : 0.f);
}

// per-block partials of (sum ddelta a_c for c < 16, sum ddelta)
__global__ void __launch_bounds__(256) k_head_wgrad_part(long nv, const float* __restrict__ dd,
                                                         const uint16_t* __restrict__ a, int vox_per_block,
                                                         float* __restrict__ part) {
  __shared__ float sm[256][17];
  const long v0 = (long)blockIdx.x * vox_per_block;
  const long v1 = v0 + vox_per_block < nv ? v0 + vox_per_block : nv;
  float s[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) s[c] = 0.f;
  for (long v = v0 + threadIdx.x; v < v1; v += 256) {
    const float g = dd[v];
#pragma unroll
    for (int c = 0; c < 16; ++c) s[c] += g * bf2f(a[v * 16 + c]);
    s[16] += g;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) sm[threadIdx.x][c] = s[c];
  __syncthreads();
  if (threadIdx.x < 17) {
    float t = 0.f;
    for (int q = 0; q < 256; ++q) t += sm[q][threadIdx.x];
    part[(size_t)blockIdx.x * 17 + threadIdx.x] = t;
  }
}

// d (coarse, dense C) = (sum over the 8 children of dC[child][oo + c]) (a > 0)
__global__ void k_up_bwd_mask(VDims coarse, const uint16_t* __restrict__ dC, int os, int oo, int C,
                              const uint16_t* __restrict__ a, uint16_t* __restrict__ d) {
  const VDims f{coarse.nx * 2, coarse.ny * 2, coarse.nz * 2};
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= vox_count(coarse) * C) return;
  const int ch = (int)(q % C);
  const long v = q / C;
  if (!(bf2f(a[q]) > 0.f)) {
    d[q] = 0;
    return;
  }
  const int X = (int)(v % coarse.nx), Y = (int)((v / coarse.nx) % coarse.ny),
            Z = (int)(v / ((long)coarse.nx * coarse.ny));
  float s = 0.f;
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        const long fv = (2L * X + i) + (long)f.nx * ((2L * Y + j) + (long)f.ny * (2L * Z + k));
        s += bf2f(dC[fv * os + oo + ch]);
      }
  d[q] = f2bf(s);
}

// d (fine, dense C) = (dC[v][c] (stride os) + dp[parent][c] / 8) (a[v][c] > 0, stride as)
__global__ void k_skip_mask(VDims fine, const uint16_t* __restrict__ dC, int os, const uint16_t* __restrict__ dp,
                            const uint16_t* __restrict__ a, int as, int C, uint16_t* __restrict__ d) {
  const VDims c{fine.nx / 2, fine.ny / 2, fine.nz / 2};
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= vox_count(fine) * C) return;
  const int ch = (int)(q % C);
  const long v = q / C;
  if (!(bf2f(a[v * as + ch]) > 0.f)) {
    d[q] = 0;
    return;
  }
  const int x = (int)(v % fine.nx), y = (int)((v / fine.nx) % fine.ny), z = (int)(v / ((long)fine.nx * fine.ny));
  const long p = (x / 2) + (long)c.nx * ((y / 2) + (long)c.ny * (z / 2));
  d[q] = f2bf(bf2f(dC[v * os + ch]) + 0.125f * bf2f(dp[p * C + ch]));
}

// W' [ci][26 - tap][co] = W[co][tap][ci]  (bfloat16, for the input gradient)
__global__ void k_flip_transpose(const float* __restrict__ w, int cin, int cout, uint16_t* __restrict__ wt) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cout * 27 * cin) return;
  const int co = q / (27 * cin), r = q % (27 * cin), tap = r / cin, ci = r % cin;
  wt[((size_t)ci * 27 + (26 - tap)) * cout + co] = f2bf(w[q]);
}

__global__ void k_to_bf16(const float* __restrict__ a, long n, uint16_t* __restrict__ b) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) b[q] = f2bf(a[q]);
}

// Adam with bias correction; padded (always-zero-gradient) entries stay put
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float c1, float c2) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = 0.9f * m[q] + 0.1f * gq;
  const float vq = 0.999f * v[q] + 0.001f * gq * gq;
  m[q] = mq;
  v[q] = vq;
  th[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + 1e-8f);
}

// ------------------------------------------------ features, loss, guess
// four input channels (channel-first FP32): rhs h^2 rho_w / P0, the
// log-density fraction, p_prev / P0 and the residual (b - A p_prev) h^2 rho_w / P0
__global__ void k_features(long nv, double s, double lr_w, double inv_lr, double inv_P0,
                           const double* __restrict__ b, const double* __restrict__ rho,
                           const double* __restrict__ pprev, const double* __restrict__ Ap,
                           float* __restrict__ feat) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double bb = b[v];
  feat[v] = (float)(bb * s);
  feat[nv + v] = (float)((log(rho[v]) - lr_w) * inv_lr);
  feat[2 * nv + v] = (float)(pprev[v] * inv_P0);
  feat[3 * nv + v] = (float)((bb - Ap[v]) * s);
}

// channel-first FP32 features -> channels-last bfloat16 input, padded to 16
__global__ void k_set_input(long nv, const float* __restrict__ feat, uint16_t* __restrict__ x0) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  u32x4 lo = {0u, 0u, 0u, 0u};
  lo[0] = (uint32_t)f2bf(feat[v]) | ((uint32_t)f2bf(feat[nv + v]) << 16);
  lo[1] = (uint32_t)f2bf(feat[2 * nv + v]) | ((uint32_t)f2bf(feat[3 * nv + v]) << 16);
  u32x4* o = reinterpret_cast<u32x4*>(x0 + v * 16);
  o[0] = lo;
  o[1] = u32x4{0u, 0u, 0u, 0u};
}

// p = p_prev + P0 delta
__global__ void k_apply_delta(long nv, const double* __restrict__ pprev, const float* __restrict__ delta,
                              double P0, double* __restrict__ p) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) p[v] = pprev[v] + P0 * (double)delta[v];
}

// target delta = (p* - p_prev) / P0
__global__ void k_target(long nv, const double* __restrict__ p, const double* __restrict__ pprev, double inv_P0,
                         float* __restrict__ t) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) t[v] = (float)((p[v] - pprev[v]) * inv_P0);
}

// y = A x in FP32 on the finest grid (sum_f beta_f (x_c - x_nb), open top
// face coupling to -x_c; the 1/h^2 factor cancels in the loss ratio)
__global__ void __launch_bounds__(256) k_spmv_f32(VDims d, const float* __restrict__ bx,
                                                  const float* __restrict__ by, const float* __restrict__ bz,
                                                  const float* __restrict__ x, float* __restrict__ y) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= vox_count(d)) return;
  const int i = (int)(c % d.nx), j = (int)((c / d.nx) % d.ny), k = (int)(c / ((long)d.nx * d.ny));
  const long sxy = (long)d.nx * d.ny;
  const long fx = i + (long)(d.nx + 1) * (j + (long)d.ny * k);
  const long fy = i + (long)d.nx * (j + (long)(d.ny + 1) * k);
  const float xc = x[c];
  float a = 0.f;
  if (i > 0) a += bx[fx] * (xc - x[c - 1]);
  if (i < d.nx - 1) a += bx[fx + 1] * (xc - x[c + 1]);
  if (j > 0) a += by[fy] * (xc - x[c - d.nx]);
  if (j < d.ny - 1) a += by[fy + d.nx] * (xc - x[c + d.nx]);
  if (k > 0) a += bz[c] * (xc - x[c - sxy]);
  a += (k < d.nz - 1) ? bz[c + sxy] * (xc - x[c + sxy]) : 2.f * bz[c + sxy] * xc;
  y[c] = a;
}

// e = t - delta (the guess's error in units of P0)
__global__ void k_err(long nv, const float* __restrict__ delta, const float* __restrict__ t, float* __restrict__ e) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) e[v] = t[v] - delta[v];
}

// per-block (sum e Ae, sum t At)
__global__ void __launch_bounds__(256) k_loss_part(long nv, const float* __restrict__ e, const float* __restrict__ Ae,
                                                   const float* __restrict__ t, const float* __restrict__ At,
                                                   double* __restrict__ part) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long)gridDim.x * 256) {
    a += (double)e[v] * (double)Ae[v];
    b += (double)t[v] * (double)At[v];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa[0];
    part[2 * blockIdx.x + 1] = sb[0];
  }
}

// out[0] = loss = e'Ae / t'At, out[1] = -2 / t'At
__global__ void k_loss_fin(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nblk; ++q) {
    a += part[2 * q];
    b += part[2 * q + 1];
  }
  out[0] = b > 0.0 ? a / b : 0.0;
  out[1] = b > 0.0 ? -2.0 / b : 0.0;
}

// dL/ddelta = -2 A e / t'At  (A symmetric)
__global__ void k_dloss(long nv, const float* __restrict__ Ae, const double* __restrict__ out, float* __restrict__ dd) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) dd[v] = (float)(out[1] * (double)Ae[v]);
}

__global__ void k_finite_count(long n, const float* __restrict__ a, int* __restrict__ bad) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n && !isfinite(a[q])) atomicAdd(bad, 1);
}

inline dim3 g1(long n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

// ==================================================================== the net
// conv layers 1..5 (index 0..4): padded C_in, C_out, and the head (16 -> 1)
static const int kCin[5] = {16, 16, 32, 96, 48};
static const int kCinTrue[5] = {4, 16, 32, 96, 48};
static const int kCout[5] = {16, 32, 64, 32, 16};

}  // namespace nsk

using namespace nsk;

struct ns_net {
  VDims res0, res1, res2;
  long v0, v1, v2;
  int training;
  hipStream_t st;
  // internal parameter layout: per conv layer W[co][tap][ci_pad] then b[co];
  // then the head w[16], b[1]
  size_t np;
  size_t ow[5], ob[5], ohw, ohb;
  float *theta, *m, *v, *g;
  uint16_t *wf[5], *wt[5];
  uint16_t* wc0;   // first layer, compact K (inference)
  uint16_t *x0, *C1, *p1, *C2, *p2, *a3, *a4, *a5;
  float* delta;
  // backward
  float* dd;
  uint16_t *d5, *dC1, *d4, *dC2, *d3, *dp2, *d2, *dp1, *d1;
  float* wpart;
  size_t wpart_elems;
  double* red;
  int* bad;
  double* host;
  // learned-guess staging
  float* feat;
  float* target;
  float* eb;
  double* pprev;
  double* Ap;
  int step;
  char err[256];
};

namespace {

constexpr size_t kAlignN = 256;

struct NetCarve {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlignN - 1) / kAlignN * kAlignN;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int kWgradVox = 4096;   // voxels per weight-gradient block

size_t net_layout(ns_net* N, int nx, int ny, int nz, int training, char* base) {
  NetCarve cv{base, 0};
  VDims d0{nx, ny, nz}, d1{nx / 2, ny / 2, nz / 2}, d2{nx / 4, ny / 4, nz / 4};
  const long v0 = (long)nx * ny * nz, v1 = v0 / 8, v2 = v0 / 64;
  size_t np = 0, ow[5], ob[5];
  for (int l = 0; l < 5; ++l) {
    ow[l] = np;
    np += (size_t)kCout[l] * 27 * kCin[l];
    ob[l] = np;
    np += kCout[l];
  }
  const size_t ohw = np;
  np += 16;
  const size_t ohb = np;
  np += 1;
  float* theta = cv.take<float>(np);
  float *m = nullptr, *v = nullptr, *g = nullptr;
  if (training) {
    m = cv.take<float>(np);
    v = cv.take<float>(np);
    g = cv.take<float>(np);
  }
  uint16_t *wf[5], *wt[5];
  for (int l = 0; l < 5; ++l) {
    wf[l] = cv.take<uint16_t>((size_t)kCout[l] * 27 * kCin[l]);
    wt[l] = cv.take<uint16_t>((size_t)kCout[l] * 27 * kCin[l]);
  }
  uint16_t* wc0 = cv.take<uint16_t>(16 * 128);
  uint16_t* x0 = cv.take<uint16_t>(v0 * 16);
  uint16_t* C1 = cv.take<uint16_t>(v0 * 48);
  uint16_t* p1 = cv.take<uint16_t>(v1 * 16);
  uint16_t* C2 = cv.take<uint16_t>(v1 * 96);
  uint16_t* p2 = cv.take<uint16_t>(v2 * 32);
  uint16_t* a3 = cv.take<uint16_t>(v2 * 64);
  uint16_t* a4 = cv.take<uint16_t>(v1 * 32);
  uint16_t* a5 = cv.take<uint16_t>(v0 * 16);
  float* delta = cv.take<float>(v0);
  float* feat = cv.take<float>(4 * v0);
  float* target = cv.take<float>(v0);
  float* eb = cv.take<float>(3 * v0);   // e, A e, A t of the loss
  double* pprev = cv.take<double>(v0);
  double* Ap = cv.take<double>(v0);
  double* red = cv.take<double>(4096);
  int* bad = cv.take<int>(64);
  float* dd = nullptr;
  uint16_t *d5 = nullptr, *dC1 = nullptr, *d4 = nullptr, *dC2 = nullptr, *d3 = nullptr, *dp2 = nullptr,
           *d2p = nullptr, *dp1 = nullptr, *d1p = nullptr;
  float* wpart = nullptr;
  size_t wpart_elems = 0;
  if (training) {
    dd = cv.take<float>(v0);
    d5 = cv.take<uint16_t>(v0 * 16);
    dC1 = cv.take<uint16_t>(v0 * 48);
    d4 = cv.take<uint16_t>(v1 * 32);
    dC2 = cv.take<uint16_t>(v1 * 96);
    d3 = cv.take<uint16_t>(v2 * 64);
    dp2 = cv.take<uint16_t>(v2 * 32);
    d2p = cv.take<uint16_t>(v1 * 32);
    dp1 = cv.take<uint16_t>(v1 * 16);
    d1p = cv.take<uint16_t>(v0 * 16);
    // the largest (blocks x 27 x C_out x C_in) over the layers
    for (int l = 0; l < 5; ++l) {
      const long vl = (l == 0 || l == 4) ? v0 : (l == 1 || l == 3) ? v1 : v2;
      const size_t nb = (size_t)((vl + kWgradVox - 1) / kWgradVox);
      const size_t e = nb * 27 * (size_t)kCout[l] * kCin[l];
      if (e > wpart_elems) wpart_elems = e;
    }
    // bias and head partials share the buffer
    const size_t eb = (size_t)((v0 + kWgradVox - 1) / kWgradVox) * 96;
    if (eb > wpart_elems) wpart_elems = eb;
    wpart = cv.take<float>(wpart_elems);
  }
  if (N) {
    N->res0 = d0;
    N->res1 = d1;
    N->res2 = d2;
    N->v0 = v0;
    N->v1 = v1;
    N->v2 = v2;
    N->training = training;
    N->np = np;
    for (int l = 0; l < 5; ++l) {
      N->ow[l] = ow[l];
      N->ob[l] = ob[l];
      N->wf[l] = wf[l];
      N->wt[l] = wt[l];
    }
    N->ohw = ohw;
    N->ohb = ohb;
    N->theta = theta;
    N->m = m;
    N->v = v;
    N->g = g;
    N->wc0 = wc0;
    N->x0 = x0;
    N->C1 = C1;
    N->p1 = p1;
    N->C2 = C2;
    N->p2 = p2;
    N->a3 = a3;
    N->a4 = a4;
    N->a5 = a5;
    N->delta = delta;
    N->feat = feat;
    N->target = target;
    N->eb = eb;
    N->pprev = pprev;
    N->Ap = Ap;
    N->red = red;
    N->bad = bad;
    N->dd = dd;
    N->d5 = d5;
    N->dC1 = dC1;
    N->d4 = d4;
    N->dC2 = dC2;
    N->d3 = d3;
    N->dp2 = dp2;
    N->d2 = d2p;
    N->dp1 = dp1;
    N->d1 = d1p;
    N->wpart = wpart;
    N->wpart_elems = wpart_elems;
  }
  return cv.off + kAlignN;
}

ns_status nfail(ns_net* N, ns_status s, const char* msg) {
  if (N) snprintf(N->err, sizeof(N->err), "%s", msg);
  return s;
}

template <int CIN, int COUT, int EPI>
void conv(const ns_net* N, VDims d, const uint16_t* XA, int sa, int ca, const uint16_t* XB, int sb,
          const uint16_t* W, const float* bias, uint16_t* Y, int ys, int yo, const float* hw = nullptr,
          const float* hb = nullptr, float* delta = nullptr) {
  const dim3 grid((d.nx + kTX - 1) / kTX, (d.ny + kTY - 1) / kTY, (d.nz + kTZ - 1) / kTZ);
  hipLaunchKernelGGL((k_conv<CIN, COUT, EPI>), grid, dim3(256), 0, N->st, d, XA, sa, ca, XB, sb, W, bias, Y, ys,
                     yo, hw, hb, delta);
}

template <int CIN, int COUT, int EPI>
void conv_cm(const ns_net* N, VDims d, const uint16_t* XA, int sa, int ca, const uint16_t* XB, int sb,
             const uint16_t* W, const float* bias, uint16_t* Y, int ys, int yo, const float* hw = nullptr,
             const float* hb = nullptr, float* delta = nullptr) {
  const dim3 grid((d.nx + kCX - 1) / kCX, (d.ny + kCY - 1) / kCY, (d.nz + kCZ - 1) / kCZ);
  hipLaunchKernelGGL((k_conv_cm<CIN, COUT, EPI>), grid, dim3(256), 0, N->st, d, XA, sa, ca, XB, sb, W, bias, Y,
                     ys, yo, hw, hb, delta);
}

// bf16 copies (forward and flipped-transposed) of the FP32 master weights
void refresh_weights(ns_net* N) {
  hipLaunchKernelGGL(k_compact_w0, dim3(8), dim3(256), 0, N->st, N->theta + N->ow[0], N->wc0);
  for (int l = 0; l < 5; ++l) {
    const long n = (long)kCout[l] * 27 * kCin[l];
    hipLaunchKernelGGL(k_to_bf16, g1(n), dim3(256), 0, N->st, N->theta + N->ow[l], n, N->wf[l]);
    hipLaunchKernelGGL(k_flip_transpose, g1(n), dim3(256), 0, N->st, N->theta + N->ow[l], kCin[l], kCout[l],
                       N->wt[l]);
  }
}

// Training forward: every activation the backward pass reads is stored,
// including the concatenated decoder inputs C2 = [a2, up(a3)] and
// C1 = [a1, up(a4)] and the last activation a5.
void forward_train(ns_net* N) {
  const float* th = N->theta;
  conv<16, 16, 0>(N, N->res0, N->x0, 16, 16, nullptr, 0, N->wf[0], th + N->ob[0], N->C1, 48, 0);
  hipLaunchKernelGGL(k_pool, g1(N->v1 * 2), dim3(256), 0, N->st, N->res0, N->C1, 48, 0, 16, N->p1);
  conv<16, 32, 0>(N, N->res1, N->p1, 16, 16, nullptr, 0, N->wf[1], th + N->ob[1], N->C2, 96, 0);
  hipLaunchKernelGGL(k_pool, g1(N->v2 * 4), dim3(256), 0, N->st, N->res1, N->C2, 96, 0, 32, N->p2);
  conv<32, 64, 0>(N, N->res2, N->p2, 32, 32, nullptr, 0, N->wf[2], th + N->ob[2], N->a3, 64, 0);
  hipLaunchKernelGGL(k_up, g1(N->v1 * 64), dim3(256), 0, N->st, N->res2, N->a3, 64, N->C2, 96, 32);
  conv<96, 32, 0>(N, N->res1, N->C2, 96, 96, nullptr, 0, N->wf[3], th + N->ob[3], N->a4, 32, 0);
  hipLaunchKernelGGL(k_up, g1(N->v0 * 32), dim3(256), 0, N->st, N->res1, N->a4, 32, N->C1, 48, 16);
  conv<48, 16, 0>(N, N->res0, N->C1, 48, 48, nullptr, 0, N->wf[4], th + N->ob[4], N->a5, 16, 0);
  hipLaunchKernelGGL(k_head, g1(N->v0), dim3(256), 0, N->st, N->v0, N->a5, th + N->ohw, th + N->ohb, N->delta);
}

// Inference forward: the decoder convolutions read the skip tensor and the
// coarse tensor directly (no upsampled copies), and the head is fused into
// the last convolution, so a5 is never stored.
// The input is the FP32 feature tensor in N->feat.
void forward_infer(ns_net* N) {
  const float* th = N->theta;
  uint16_t* a1 = N->C1;   // dense [v0][16] in the concatenation buffer's memory
  uint16_t* a2 = N->C2;   // dense [v1][32]
  {
    const VDims d = N->res0;
    const dim3 grid((d.nx + kTX - 1) / kTX, (d.ny + kTY - 1) / kTY, (d.nz + kTZ - 1) / kTZ);
    hipLaunchKernelGGL(k_conv_in, grid, dim3(256), 0, N->st, d, N->feat, N->wc0, th + N->ob[0], a1, 16);
  }
  hipLaunchKernelGGL(k_pool, g1(N->v1 * 2), dim3(256), 0, N->st, N->res0, a1, 16, 0, 16, N->p1);
  conv<16, 32, 0>(N, N->res1, N->p1, 16, 16, nullptr, 0, N->wf[1], th + N->ob[1], a2, 32, 0);
  hipLaunchKernelGGL(k_pool, g1(N->v2 * 4), dim3(256), 0, N->st, N->res1, a2, 32, 0, 32, N->p2);
  conv<32, 64, 0>(N, N->res2, N->p2, 32, 32, nullptr, 0, N->wf[2], th + N->ob[2], N->a3, 64, 0);
  conv_cm<96, 32, 0>(N, N->res1, a2, 32, 32, N->a3, 64, N->wf[3], th + N->ob[3], N->a4, 32, 0);
  conv<48, 16, 2>(N, N->res0, a1, 16, 16, N->a4, 32, N->wf[4], th + N->ob[4], nullptr, 16, 0, th + N->ohw,
                  th + N->ohb, N->delta);
}

void forward(ns_net* N) {
  if (N->training)
    forward_train(N);
  else
    forward_infer(N);
}

template <int CIN, int COUT>
void wgrad(ns_net* N, VDims d, long nv, const uint16_t* X, const uint16_t* dY, int layer) {
  const int nb = (int)((nv + kWgradVox - 1) / kWgradVox);
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(nb, 27), dim3(256), 0, N->st, d, X, dY, kWgradVox, N->wpart);
  const int per = 27 * COUT * CIN;
  hipLaunchKernelGGL(k_wgrad_reduce, g1(per), dim3(256), 0, N->st, N->wpart, nb, CIN, COUT, N->g + N->ow[layer]);
  hipLaunchKernelGGL(k_bias_part, dim3(nb), dim3(256), 0, N->st, nv, COUT, dY, kWgradVox, N->wpart);
  hipLaunchKernelGGL(k_bias_reduce, dim3(1), dim3(128), 0, N->st, N->wpart, nb, COUT, N->g + N->ob[layer]);
}

void backward(ns_net* N) {
  const float* th = N->theta;
  hipStream_t st = N->st;
  // head
  {
    const int nb = (int)((N->v0 + kWgradVox - 1) / kWgradVox);
    hipLaunchKernelGGL(k_head_wgrad_part, dim3(nb), dim3(256), 0, st, N->v0, N->dd, N->a5, kWgradVox, N->wpart);
    hipLaunchKernelGGL(k_bias_reduce, dim3(1), dim3(32), 0, st, N->wpart, nb, 17, N->g + N->ohw);
    hipLaunchKernelGGL(k_head_bwd, g1(N->v0 * 16), dim3(256), 0, st, N->v0, N->dd, N->a5, th + N->ohw, N->d5);
  }
  // layer 5: input C1 (48), output 16
  wgrad<48, 16>(N, N->res0, N->v0, N->C1, N->d5, 4);
  conv<16, 48, 1>(N, N->res0, N->d5, 16, 16, nullptr, 0, N->wt[4], nullptr, N->dC1, 48, 0);
  hipLaunchKernelGGL(k_up_bwd_mask, g1(N->v1 * 32), dim3(256), 0, st, N->res1, N->dC1, 48, 16, 32, N->a4, N->d4);
  // layer 4: input C2 (96), output 32
  wgrad<96, 32>(N, N->res1, N->v1, N->C2, N->d4, 3);
  conv<32, 96, 1>(N, N->res1, N->d4, 32, 32, nullptr, 0, N->wt[3], nullptr, N->dC2, 96, 0);
  hipLaunchKernelGGL(k_up_bwd_mask, g1(N->v2 * 64), dim3(256), 0, st, N->res2, N->dC2, 96, 32, 64, N->a3, N->d3);
  // layer 3: input p2 (32), output 64
  wgrad<32, 64>(N, N->res2, N->v2, N->p2, N->d3, 2);
  conv<64, 32, 1>(N, N->res2, N->d3, 64, 64, nullptr, 0, N->wt[2], nullptr, N->dp2, 32, 0);
  hipLaunchKernelGGL(k_skip_mask, g1(N->v1 * 32), dim3(256), 0, st, N->res1, N->dC2, 96, N->dp2, N->C2, 96, 32, N->d2);
  // layer 2: input p1 (16), output 32
  wgrad<16, 32>(N, N->res1, N->v1, N->p1, N->d2, 1);
  conv<32, 16, 1>(N, N->res1, N->d2, 32, 32, nullptr, 0, N->wt[1], nullptr, N->dp1, 16, 0);
  hipLaunchKernelGGL(k_skip_mask, g1(N->v0 * 16), dim3(256), 0, st, N->res0, N->dC1, 48, N->dp1, N->C1, 48, 16, N->d1);
  // layer 1: input x0 (16), output 16
  wgrad<16, 16>(N, N->res0, N->v0, N->x0, N->d1, 0);
}

// canonical parameter index (the flat order of ns_net_set_params and
// ns_net_get_params) <-> internal index
// conv layer l: canonical w[co][ci][kz][ky][kx] (ci < true C_in) then b[co];
// internal W[co][tap][ci_pad], tap = (kz * 3 + ky) * 3 + kx
template <typename F>
void for_each_param(const ns_net* N, F f) {
  size_t c = 0;
  for (int l = 0; l < 5; ++l) {
    const int cin = kCinTrue[l], cinp = kCin[l], cout = kCout[l];
    for (int co = 0; co < cout; ++co)
      for (int ci = 0; ci < cin; ++ci)
        for (int tap = 0; tap < 27; ++tap) f(c++, N->ow[l] + ((size_t)co * 27 + tap) * cinp + ci);
    for (int co = 0; co < cout; ++co) f(c++, N->ob[l] + co);
  }
  for (int q = 0; q < 16; ++q) f(c++, N->ohw + q);
  f(c++, N->ohb);
}

size_t canonical_count() {
  size_t n = 0;
  for (int l = 0; l < 5; ++l) n += (size_t)kCout[l] * kCinTrue[l] * 27 + kCout[l];
  return n + 17;
}

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

size_t ns_net_param_count(void) { return canonical_count(); }

size_t ns_net_workspace_bytes(int nx, int ny, int nz, int training) {
  if (nx < 4 || ny < 4 || nz < 4 || nx % 4 || ny % 4 || nz % 4) return 0;
  return net_layout(nullptr, nx, ny, nz, training ? 1 : 0, nullptr);
}

ns_status ns_net_create(int nx, int ny, int nz, int training, void* ws, size_t bytes, void* stream,
                        ns_net** out) {
  if (!out) return NS_EINVAL;
  *out = nullptr;
  if (nx < 4 || ny < 4 || nz < 4 || nx % 4 || ny % 4 || nz % 4) return NS_EINVAL;
  if (!ws || ((uintptr_t)ws % kAlignN) != 0) return NS_EINVAL;
  const size_t need = net_layout(nullptr, nx, ny, nz, training ? 1 : 0, nullptr);
  if (bytes < need) return NS_EINVAL;
  ns_net* N = new (std::nothrow) ns_net();
  if (!N) return NS_EINVAL;
  net_layout(N, nx, ny, nz, training ? 1 : 0, (char*)ws);
  N->st = (hipStream_t)stream;
  N->step = 0;
  if (hipHostMalloc((void**)&N->host, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete N;
    return NS_EHIP;
  }
  if (hipMemsetAsync(N->theta, 0, N->np * sizeof(float), N->st) != hipSuccess) {
    (void)hipHostFree(N->host);
    delete N;
    return NS_EHIP;
  }
  if (training && (hipMemsetAsync(N->m, 0, N->np * sizeof(float), N->st) != hipSuccess ||
                   hipMemsetAsync(N->v, 0, N->np * sizeof(float), N->st) != hipSuccess ||
                   hipMemsetAsync(N->g, 0, N->np * sizeof(float), N->st) != hipSuccess)) {
    ns_net_destroy(N);
    return NS_EHIP;
  }
  *out = N;
  return NS_OK;
}

void ns_net_destroy(ns_net* N) {
  if (!N) return;
  if (N->host) (void)hipHostFree(N->host);
  delete N;
}

const char* ns_net_last_error(ns_net* N) { return N ? N->err : "null net"; }

ns_status ns_net_set_params(ns_net* N, const float* host_params, size_t n) {
  if (!N || !host_params) return NS_EINVAL;
  if (n != canonical_count()) return nfail(N, NS_EINVAL, "parameter count mismatch");
  std::vector<float> internal(N->np, 0.0f);
  for_each_param(N, [&](size_t c, size_t i) { internal[i] = host_params[c]; });
  if (hipMemcpyAsync(N->theta, internal.data(), N->np * sizeof(float), hipMemcpyHostToDevice, N->st) != hipSuccess)
    return nfail(N, NS_EHIP, "upload failed");
  if (N->training) {
    (void)hipMemsetAsync(N->m, 0, N->np * sizeof(float), N->st);
    (void)hipMemsetAsync(N->v, 0, N->np * sizeof(float), N->st);
    N->step = 0;
  }
  refresh_weights(N);
  if (hipStreamSynchronize(N->st) != hipSuccess) return nfail(N, NS_EHIP, "synchronise failed");
  return NS_OK;
}

static ns_status download(ns_net* N, const float* dev, float* host, size_t n) {
  if (n != canonical_count()) return nfail(N, NS_EINVAL, "parameter count mismatch");
  std::vector<float> internal(N->np);
  if (hipMemcpyAsync(internal.data(), dev, N->np * sizeof(float), hipMemcpyDeviceToHost, N->st) != hipSuccess ||
      hipStreamSynchronize(N->st) != hipSuccess)
    return nfail(N, NS_EHIP, "download failed");
  for_each_param(N, [&](size_t c, size_t i) { host[c] = internal[i]; });
  return NS_OK;
}

ns_status ns_net_get_params(ns_net* N, float* host_params, size_t n) {
  if (!N || !host_params) return NS_EINVAL;
  return download(N, N->theta, host_params, n);
}

ns_status ns_net_get_grads(ns_net* N, float* host_grads, size_t n) {
  if (!N || !host_grads) return NS_EINVAL;
  if (!N->training) return nfail(N, NS_ESTATE, "not a training net");
  return download(N, N->g, host_grads, n);
}

ns_status ns_net_set_input(ns_net* N, const float* feat4) {
  if (!N || !feat4) return NS_EINVAL;
  if (N->training)
    hipLaunchKernelGGL(k_set_input, g1(N->v0), dim3(256), 0, N->st, N->v0, feat4, N->x0);
  else if (hipMemcpyAsync(N->feat, feat4, 4 * N->v0 * sizeof(float), hipMemcpyDeviceToDevice, N->st) != hipSuccess)
    return nfail(N, NS_EHIP, "copy failed");
  return hipGetLastError() == hipSuccess ? NS_OK : nfail(N, NS_EHIP, "launch failed");
}

ns_status ns_net_forward(ns_net* N, float* delta_out) {
  if (!N) return NS_EINVAL;
  forward(N);
  if (delta_out)
    if (hipMemcpyAsync(delta_out, N->delta, N->v0 * sizeof(float), hipMemcpyDeviceToDevice, N->st) != hipSuccess)
      return nfail(N, NS_EHIP, "copy failed");
  return hipGetLastError() == hipSuccess ? NS_OK : nfail(N, NS_EHIP, "launch failed");
}

ns_status ns_net_train_step(ns_net* N, const float* feat4, const float* target, const float* bx, const float* by,
                            const float* bz, float lr, int update, double* loss) {
  if (!N || !feat4 || !target || !bx || !by || !bz) return NS_EINVAL;
  if (!N->training) return nfail(N, NS_ESTATE, "not a training net");
  hipStream_t st = N->st;
  hipLaunchKernelGGL(k_set_input, g1(N->v0), dim3(256), 0, st, N->v0, feat4, N->x0);
  forward(N);
  // energy-norm loss L = e'Ae / t'At with e = t - delta
  float *e = N->eb, *Ae = N->eb + N->v0, *At = N->eb + 2 * N->v0;
  const int nb = 256;
  hipLaunchKernelGGL(k_err, g1(N->v0), dim3(256), 0, st, N->v0, N->delta, target, e);
  hipLaunchKernelGGL(k_spmv_f32, g1(N->v0), dim3(256), 0, st, N->res0, bx, by, bz, e, Ae);
  hipLaunchKernelGGL(k_spmv_f32, g1(N->v0), dim3(256), 0, st, N->res0, bx, by, bz, target, At);
  hipLaunchKernelGGL(k_loss_part, dim3(nb), dim3(256), 0, st, N->v0, e, Ae, target, At, N->red);
  hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(64), 0, st, N->red, nb, N->red + 2 * nb);
  hipLaunchKernelGGL(k_dloss, g1(N->v0), dim3(256), 0, st, N->v0, Ae, N->red + 2 * nb, N->dd);
  backward(N);
  if (update) {
    ++N->step;
    const float c1 = 1.0f - powf(0.9f, (float)N->step), c2 = 1.0f - powf(0.999f, (float)N->step);
    hipLaunchKernelGGL(k_adam, g1((long)N->np), dim3(256), 0, st, N->theta, N->g, N->m, N->v, (long)N->np, lr, c1, c2);
    refresh_weights(N);
  }
  if (hipMemcpyAsync(N->host, N->red + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return nfail(N, NS_EHIP, "train step failed");
  if (loss) *loss = N->host[0];
  return std::isfinite(N->host[0]) ? NS_OK : nfail(N, NS_ENAN, "non-finite loss");
}

}  // extern "C"

// --------------------------------------------- hooks used by the projection
namespace nsk {

void net_features(ns_net* N, const Dims& n, double h, double rho_w, double rho_a, double P0, const double* b,
                  const double* rho, const double* pprev, const double* Ap, float* feat, hipStream_t st) {
  const long nv = (long)n.nx * n.ny * n.nz;
  (void)N;
  hipLaunchKernelGGL(k_features, g1(nv), dim3(256), 0, st, nv, h * h * rho_w / P0, log(rho_w),
                     1.0 / (log(rho_a) - log(rho_w)), 1.0 / P0, b, rho, pprev, Ap, feat);
}

int net_matches(const ns_net* N, const Dims& n) {
  return N && N->res0.nx == n.nx && N->res0.ny == n.ny && N->res0.nz == n.nz;
}

double* net_pprev(ns_net* N) { return N->pprev; }
double* net_Ap(ns_net* N) { return N->Ap; }
float* net_feat(ns_net* N) { return N->feat; }

// p = p_prev + P0 delta from the current features; returns the number of
// non-finite outputs (device counter read back synchronously); done, if
// given, is recorded once p is written
int net_guess(ns_net* N, double P0, double* p, hipStream_t st, hipEvent_t done) {
  hipStream_t keep = N->st;
  N->st = st;
  if (N->training) hipLaunchKernelGGL(k_set_input, g1(N->v0), dim3(256), 0, st, N->v0, N->feat, N->x0);
  forward(N);
  (void)hipMemsetAsync(N->bad, 0, sizeof(int), st);
  hipLaunchKernelGGL(k_finite_count, g1(N->v0), dim3(256), 0, st, N->v0, N->delta, N->bad);
  hipLaunchKernelGGL(k_apply_delta, g1(N->v0), dim3(256), 0, st, N->v0, N->pprev, N->delta, P0, p);
  if (done) (void)hipEventRecord(done, st);
  int bad = 0;
  (void)hipMemcpyAsync(N->host, N->bad, sizeof(int), hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  memcpy(&bad, N->host, sizeof(int));
  N->st = keep;
  return bad;
}

void net_target(long nv, const double* p, const double* pprev, double P0, float* t, hipStream_t st) {
  hipLaunchKernelGGL(k_target, g1(nv), dim3(256), 0, st, nv, p, pprev, 1.0 / P0, t);
}

}  // namespace nsk
