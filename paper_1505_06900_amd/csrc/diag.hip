// Lattice-independent diagnostic kernels: enstrophy of a velocity field and
// the plain copy used as bandwidth probe / hardware-counter calibration.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ops.hpp"

namespace lbrr {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void block_sum_store1(double v, double* __restrict__ out) {
  __shared__ double lds[kReduceBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double s = wave_sum(v);
  if (lane == 0) lds[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kReduceBlock / 64; ++w) t += lds[w];
    out[blockIdx.x] = t;
  }
}

// Per-block partial sums of |omega|^2 / 2, omega by second-order central
// differences on the periodic lattice (2D: the scalar w_z).
__global__ void __launch_bounds__(kReduceBlock) k_enstrophy(const double* __restrict__ u, int d, int nx, int ny,
                                                            int nz, int64_t per_block, double* __restrict__ partials) {
  const int64_t nodes = int64_t(nx) * ny * nz;
  const int64_t begin = int64_t(blockIdx.x) * per_block;
  const int64_t end = begin + per_block < nodes ? begin + per_block : nodes;
  const double* ux = u;
  const double* uy = u + nodes;
  const double* uz = u + 2 * nodes;
  double acc = 0.0;
  for (int64_t n = begin + threadIdx.x; n < end; n += kReduceBlock) {
    const int x = int(n % nx);
    const int y = int((n / nx) % ny);
    const int z = int(n / (int64_t(nx) * ny));
    const int64_t row = n - x;
    const int64_t xp = row + (x + 1 == nx ? 0 : x + 1), xm = row + (x == 0 ? nx - 1 : x - 1);
    const int64_t plane = n - int64_t(y) * nx;
    const int64_t yp = plane + int64_t(y + 1 == ny ? 0 : y + 1) * nx;
    const int64_t ym = plane + int64_t(y == 0 ? ny - 1 : y - 1) * nx;
    const int64_t sxy = int64_t(nx) * ny;
    const int64_t vol = n - int64_t(z) * sxy;
    const int64_t zp = vol + int64_t(z + 1 == nz ? 0 : z + 1) * sxy;
    const int64_t zm = vol + int64_t(z == 0 ? nz - 1 : z - 1) * sxy;
    const double duy_dx = 0.5 * (uy[xp] - uy[xm]);
    const double dux_dy = 0.5 * (ux[yp] - ux[ym]);
    if (d == 2) {
      const double w = duy_dx - dux_dy;
      acc += 0.5 * w * w;
    } else {
      const double duz_dy = 0.5 * (uz[yp] - uz[ym]);
      const double duy_dz = 0.5 * (uy[zp] - uy[zm]);
      const double dux_dz = 0.5 * (ux[zp] - ux[zm]);
      const double duz_dx = 0.5 * (uz[xp] - uz[xm]);
      const double wx = duz_dy - duy_dz, wy = dux_dz - duz_dx, wz = duy_dx - dux_dy;
      acc += 0.5 * (wx * wx + wy * wy + wz * wz);
    }
  }
  block_sum_store1(acc, partials);
}

__global__ void __launch_bounds__(kReduceBlock) k_final1(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kReduceBlock) acc += partials[b];
  block_sum_store1(acc, out);
}

// One 16-byte element per thread, non-temporal store: the best plain-copy
// form measured on MI355X (about 6.4 TB/s for read + write).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n16) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(src[i], &dst[i]);
}

}  // namespace

hipError_t launch_enstrophy(const double* u, int d, int nx, int ny, int nz, double* partials, int nblocks,
                            double* out, hipStream_t s) {
  const int64_t nodes = int64_t(nx) * ny * nz;
  const int64_t per_block = (nodes + nblocks - 1) / nblocks;
  hipLaunchKernelGGL(k_enstrophy, dim3(nblocks), dim3(kReduceBlock), 0, s, u, d, nx, ny, nz, per_block, partials);
  hipLaunchKernelGGL(k_final1, dim3(1), dim3(kReduceBlock), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t n, hipStream_t s) {
  const size_t n16 = n / 16;
  const size_t blocks = (n16 + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0xffffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const u32x4*>(src),
                     static_cast<u32x4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace lbrr
