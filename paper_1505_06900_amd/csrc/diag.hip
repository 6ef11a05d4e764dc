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

// Derivative along one axis of a field at node n (index stride st, position i
// of n >= 0 along an axis of n_ nodes): second-order central differences,
// periodic; on a walled axis the first and last node use the second-order
// one-sided formulas (-3 a0 + 4 a1 - a2)/2 and (3 a_n-1 - 4 a_n-2 + a_n-3)/2.
__device__ __forceinline__ double axis_derivative(const double* __restrict__ a, int64_t n, int64_t st, int i, int n_,
                                                  bool walled) {
  if (walled && i == 0) return 0.5 * (-3.0 * a[n] + 4.0 * a[n + st] - a[n + 2 * st]);
  if (walled && i == n_ - 1) return 0.5 * (3.0 * a[n] - 4.0 * a[n - st] + a[n - 2 * st]);
  const int64_t p = (i + 1 == n_) ? n - int64_t(i) * st : n + st;
  const int64_t m = (i == 0) ? n + int64_t(n_ - 1) * st : n - st;
  return 0.5 * (a[p] - a[m]);
}

// Per-block partial sums of |omega|^2 / 2, omega by second-order differences
// (periodic, one-sided on the walls of `walls`: bit 0 x, 1 y, 2 z); 2D: w_z.
// On a walled axis the first and last node carry weight 1/2: the sum is the
// trapezoid rule of the integral over the box whose faces are the wall nodes.
__global__ void __launch_bounds__(kReduceBlock) k_enstrophy(const double* __restrict__ u, int d, int nx, int ny,
                                                            int nz, int walls, int64_t per_block,
                                                            double* __restrict__ partials) {
  const int64_t nodes = int64_t(nx) * ny * nz;
  const int64_t begin = int64_t(blockIdx.x) * per_block;
  const int64_t end = begin + per_block < nodes ? begin + per_block : nodes;
  const double* ux = u;
  const double* uy = u + nodes;
  const double* uz = u + 2 * nodes;
  const bool wx = walls & 1, wy = walls & 2, wz = walls & 4;
  const int64_t sxy = int64_t(nx) * ny;
  double acc = 0.0;
  for (int64_t n = begin + threadIdx.x; n < end; n += kReduceBlock) {
    const int x = int(n % nx);
    const int y = int((n / nx) % ny);
    const int z = int(n / sxy);
    const double duy_dx = axis_derivative(uy, n, 1, x, nx, wx);
    const double dux_dy = axis_derivative(ux, n, nx, y, ny, wy);
    const double wt = ((wx && (x == 0 || x == nx - 1)) ? 0.5 : 1.0) * ((wy && (y == 0 || y == ny - 1)) ? 0.5 : 1.0) *
                      ((wz && (z == 0 || z == nz - 1)) ? 0.5 : 1.0);
    if (d == 2) {
      const double w = duy_dx - dux_dy;
      acc += wt * (0.5 * w * w);
    } else {
      const double duz_dy = axis_derivative(uz, n, nx, y, ny, wy);
      const double duy_dz = axis_derivative(uy, n, sxy, z, nz, wz);
      const double dux_dz = axis_derivative(ux, n, sxy, z, nz, wz);
      const double duz_dx = axis_derivative(uz, n, 1, x, nx, wx);
      const double wxv = duz_dy - duy_dz, wyv = dux_dz - duz_dx, wzv = duy_dx - dux_dy;
      acc += wt * (0.5 * (wxv * wxv + wyv * wyv + wzv * wzv));
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

hipError_t launch_enstrophy(const double* u, int d, int nx, int ny, int nz, int walls, double* partials, int nblocks,
                            double* out, hipStream_t s) {
  const int64_t nodes = int64_t(nx) * ny * nz;
  const int64_t per_block = (nodes + nblocks - 1) / nblocks;
  hipLaunchKernelGGL(k_enstrophy, dim3(nblocks), dim3(kReduceBlock), 0, s, u, d, nx, ny, nz, walls, per_block,
                     partials);
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
