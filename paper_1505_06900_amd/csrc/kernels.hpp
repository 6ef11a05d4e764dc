// Device kernels of the library and their host-side launchers, templated on
// lattice L, Hermite order N and population storage type S.  Each lattice's
// translation unit instantiates them (kernels_d2q9.hip, kernels_d3q19.hip,
// kernels_d3q27.hip) and exposes a LatticeOps table used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>

#include "collide.hpp"
#include "ops.hpp"

namespace lbrr {

// storage element -> collision precision
template <class S>
struct Prec;
template <>
struct Prec<double> {
  using R = double;
};
template <>
struct Prec<float> {
  using R = float;
};
template <>
struct Prec<_Float16> {
  using R = float;  // v_cvt_f16_f32 rounds to nearest even; f16 subnormals are kept
};

template <class S, class R>
__device__ __forceinline__ S to_store(R v) {
  return static_cast<S>(v);
}

// Element offset of node n (linear index (z*ny + y)*nx + x) in a population array.
__device__ __forceinline__ int64_t node_offset(const StepArgs& a, uint32_t n) {
  const uint32_t x = n % uint32_t(a.nx), r = n / uint32_t(a.nx);
  const uint32_t y = r % uint32_t(a.ny), z = r / uint32_t(a.ny);
  return int64_t(z) * a.sz + int64_t(y) * a.sy + x;
}

// Block barrier for an LDS exchange: waits for the LDS accesses of every wave
// but leaves global loads and stores in flight (for kernels whose threads
// share nothing through global memory within a launch), so a prefetch
// survives the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Fused pull-streaming + regularised collision, one thread per node.
//
// The thread at node x gathers f_i from x - xi_i (periodic), i.e. the
// streaming half of Eq. discr_bgk_reg, collides in registers and writes the
// q post-collision values at its own address.  Block = runs of nodes along x
// in 256 / blockDim.x rows (blockDim.x a multiple of 64, step_block), so
// every wave lies in one (y, z) row: the y/z wrap and every row base are
// wave-uniform scalars; the x +-1 neighbours are per-lane loads one element off the
// aligned row segment, served by the same cache lines.  All q loads are in
// flight before the first use.  Stores are non-temporal: the output is not
// read again before the next step has streamed the whole lattice.
template <class L, int N, class S>
__global__ void __launch_bounds__(256) k_step(const S* __restrict__ src, S* __restrict__ dst, StepArgs a) {
  using R = typename Prec<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + __builtin_amdgcn_readfirstlane(threadIdx.y), z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const int xm = (x == 0) ? a.nx - 1 : x - 1;
  const int xp = (x == a.nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? a.ny - 1 : y - 1;
  const int yp = (y == a.ny - 1) ? 0 : y + 1;
  const int zm = (z == 0) ? a.nz - 1 : z - 1;
  const int zp = (z == a.nz - 1) ? 0 : z + 1;
  // Up to 19 populations: the row bases are wave-uniform (scalar registers)
  // and each lane adds one of three 32-bit byte offsets, so an access needs no
  // per-lane 64-bit address (launch_step checks that nx * sizeof(S) fits in
  // 32 bits): 432 -> 391 VALU instructions per node for D3Q19 order 4 FP16,
  // +5% for FP16 D3Q19 and D2Q9.  D3Q27 keeps per-lane addresses: its 27 scalar
  // bases made the FP16 step 2.5% slower and FP32 no faster.
  constexpr bool kScalarRows = L::Q <= 19;
  const uint32_t ox = uint32_t(x) * uint32_t(sizeof(S)), om = uint32_t(xm) * uint32_t(sizeof(S)),
                 op = uint32_t(xp) * uint32_t(sizeof(S));
  R f[L::Q];
  sfor<0, L::Q>([&](auto I) {
    constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
    const int ys = (cy == 1) ? ym : ((cy == -1) ? yp : y);
    const int zs = (cz == 1) ? zm : ((cz == -1) ? zp : z);
    const S* row = src + int64_t(I) * a.si + int64_t(zs) * a.sz + int64_t(ys) * a.sy;
    if constexpr (kScalarRows) {
      const uint32_t off = (cx == 1) ? om : ((cx == -1) ? op : ox);
      f[I] = R(*reinterpret_cast<const S*>(reinterpret_cast<const char*>(row) + off));
    } else {
      f[I] = R(row[(cx == 1) ? xm : ((cx == -1) ? xp : x)]);
    }
  });
  collide<L, N, R>(f, R(a.rho0), R(a.omega1));
  S* out = dst + int64_t(z) * a.sz + int64_t(y) * a.sy;
  S* outx = out + x;
  sfor<0, L::Q>([&](auto I) {
    S* p = kScalarRows ? reinterpret_cast<S*>(reinterpret_cast<char*>(out + int64_t(I) * a.si) + ox)
                       : outx + int64_t(I) * a.si;
    __builtin_nontemporal_store(to_store<S, R>(f[I]), p);
  });
}

// ---------------------------------------------------------------------------
// The same step with resting no-slip walls on the first and last node of the
// axes flagged in `walls` (bit 0 x, bit 1 y, bit 2 z): the regularised
// Dirichlet boundary of Sec. 3.7 with u_bc = 0.  At a wall node a population
// whose source lies outside the box is unknown: it takes the off-equilibrium
// part of its opposite (for u = 0 and w_i = w_opp: d_i = d_opp) if that one is
// known, else the equilibrium value (d_i = w_i (rho - rho0)); rho - rho0 then
// follows from the zeroth moment of the completed set,
//   (rho - rho0) (1 - sum_buried w_i) = sum_known d_i + sum_bounced d_opp,
// a1^(2) is its second moment minus (rho - rho0) c_s^2 I (u = 0), and the node
// collides with (rho, u = 0, a1^(2)), i.e. its populations are replaced by the
// regularised f0 + f1 before the collision.  Other nodes are unchanged.
// Population Q-1-i moves along -xi_i (canonical order of every lattice here).
template <class L>
constexpr bool opposite_is_reversed() {
  for (int i = 0; i < L::Q; ++i)
    if (L::cx(L::Q - 1 - i) != -L::cx(i) || L::cy(L::Q - 1 - i) != -L::cy(i) || L::cz(L::Q - 1 - i) != -L::cz(i))
      return false;
  return true;
}

template <class L, int N, class S>
__global__ void __launch_bounds__(256) k_step_walls(const S* __restrict__ src, S* __restrict__ dst, StepArgs a,
                                                    int walls) {
  static_assert(opposite_is_reversed<L>(), "population order");
  using R = typename Prec<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + __builtin_amdgcn_readfirstlane(threadIdx.y), z = blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  const int xm = (x == 0) ? a.nx - 1 : x - 1;
  const int xp = (x == a.nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? a.ny - 1 : y - 1;
  const int yp = (y == a.ny - 1) ? 0 : y + 1;
  const int zm = (z == 0) ? a.nz - 1 : z - 1;
  const int zp = (z == a.nz - 1) ? 0 : z + 1;
  R f[L::Q];  // sources outside a walled box wrap around here and are replaced below
  sfor<0, L::Q>([&](auto I) {
    constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
    const int xs = (cx == 1) ? xm : ((cx == -1) ? xp : x);
    const int ys = (cy == 1) ? ym : ((cy == -1) ? yp : y);
    const int zs = (cz == 1) ? zm : ((cz == -1) ? zp : z);
    const S* row = src + int64_t(I) * a.si + int64_t(zs) * a.sz + int64_t(ys) * a.sy;
    f[I] = R(row[xs]);
  });
  // sides of the box this node lies on: -1 (first node), +1 (last node), 0
  const int sx = (walls & 1) ? (x == 0 ? -1 : (x == a.nx - 1 ? 1 : 0)) : 0;
  const int sy = (walls & 2) ? (y == 0 ? -1 : (y == a.ny - 1 ? 1 : 0)) : 0;
  const int sz = (L::D == 3 && (walls & 4)) ? (z == 0 ? -1 : (z == a.nz - 1 ? 1 : 0)) : 0;
  if (sx == 0 && sy == 0 && sz == 0) {
    collide<L, N, R>(f, R(a.rho0), R(a.omega1));
  } else {
    // population with velocity c comes from outside iff some side s != 0 has c = -s
    auto from_outside = [&](int cx, int cy, int cz) {
      return (sx != 0 && cx == -sx) || (sy != 0 && cy == -sy) || (sz != 0 && cz == -sz);
    };
    R sd = R(0), wb = R(0);
    sfor<0, L::Q>([&](auto I) {
      constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
      constexpr int O = L::Q - 1 - int(I);  // opposite velocity
      if (!from_outside(cx, cy, cz)) sd = sd + f[I];
      else if (!from_outside(-cx, -cy, -cz)) sd = sd + f[O];
      else wb = wb + R(L::w(I));
    });
    const R drho = sd / (R(1) - wb);
    R g[L::Q];
    sfor<0, L::Q>([&](auto I) {
      constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
      constexpr int O = L::Q - 1 - int(I);
      if (!from_outside(cx, cy, cz)) g[I] = f[I];
      else if (!from_outside(-cx, -cy, -cz)) g[I] = f[O];
      else g[I] = R(L::w(I)) * drho;
    });
    const Moments<R> m = raw_moments<L, R>(g);
    constexpr R cs2 = R(kCs2);
    Hydro<R> h;
    h.drho = drho;
    h.rho = R(a.rho0) + drho;
    h.ux = h.uy = h.uz = h.jx = h.jy = h.jz = R(0);
    h.axx = m.pxx - drho * cs2;
    h.ayy = m.pyy - drho * cs2;
    h.axy = m.pxy;
    if constexpr (L::D == 3) {
      h.azz = m.pzz - drho * cs2;
      h.axz = m.pxz;
      h.ayz = m.pyz;
    } else {
      h.azz = h.axz = h.ayz = R(0);
    }
    R C[3][3][3];
    coefficients<L, N, R>(h, R(a.omega1), C);
    reconstruct<L, N, R>(C, f);
  }
  S* out = dst + int64_t(z) * a.sz + int64_t(y) * a.sy + x;
  sfor<0, L::Q>([&](auto I) { __builtin_nontemporal_store(to_store<S, R>(f[I]), out + int64_t(I) * a.si); });
}

// Copy between the internal layout and compact SoA [q][node].
template <class L, class S>
__global__ void __launch_bounds__(256) k_repack(const S* __restrict__ src, S* __restrict__ dst, StepArgs a,
                                                bool to_compact) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = node_offset(a, uint32_t(n));
  for (int i = 0; i < L::Q; ++i) {
    if (to_compact) dst[i * nodes + n] = src[i * a.si + off];
    else dst[i * a.si + off] = src[i * nodes + n];
  }
}

// ---------------------------------------------------------------------------
// Initial state: post-collision populations of f0(rho, u) + f1(u, pi1).
template <class L, int N, class S, class T>
__global__ void __launch_bounds__(256) k_init(const T* __restrict__ rho, const T* __restrict__ u,
                                              const T* __restrict__ pi1, S* __restrict__ dst, StepArgs a) {
  using R = typename Prec<S>::R;
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  Hydro<R> h;
  h.rho = R(rho[n]);
  h.drho = R(double(rho[n]) - a.rho0);
  h.ux = R(u[n]);
  h.uy = R(u[nodes + n]);
  h.uz = (L::D == 3) ? R(u[2 * nodes + n]) : R(0);
  h.jx = h.rho * h.ux;
  h.jy = h.rho * h.uy;
  h.jz = h.rho * h.uz;
  h.axx = h.ayy = h.azz = h.axy = h.axz = h.ayz = R(0);
  if (pi1 != nullptr) {
    if constexpr (L::D == 2) {
      h.axx = R(pi1[n]);
      h.axy = R(pi1[nodes + n]);
      h.ayy = R(pi1[2 * nodes + n]);
    } else {
      h.axx = R(pi1[n]);
      h.axy = R(pi1[nodes + n]);
      h.axz = R(pi1[2 * nodes + n]);
      h.ayy = R(pi1[3 * nodes + n]);
      h.ayz = R(pi1[4 * nodes + n]);
      h.azz = R(pi1[5 * nodes + n]);
    }
  }
  R C[3][3][3];
  coefficients<L, N, R>(h, R(a.omega1), C);
  R f[L::Q];
  reconstruct<L, N, R>(C, f);
  const int64_t off = node_offset(a, uint32_t(n));
  sfor<0, L::Q>([&](auto I) { dst[int64_t(I) * a.si + off] = to_store<S, R>(f[I]); });
}

// ---------------------------------------------------------------------------
// Macroscopic fields of the stored (post-collision) state.
template <class L, class S, class T>
__global__ void __launch_bounds__(256) k_moments(const S* __restrict__ src, T* __restrict__ rho, T* __restrict__ u,
                                                 T* __restrict__ pi1, StepArgs a, double inv_omega1) {
  using R = typename Prec<S>::R;
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  R f[L::Q];
  const int64_t off = node_offset(a, uint32_t(n));
  sfor<0, L::Q>([&](auto I) { f[I] = R(src[int64_t(I) * a.si + off]); });
  const Moments<R> m = raw_moments<L, R>(f);
  const Hydro<R> h = hydro<L, R>(m, R(a.rho0));
  if (rho) rho[n] = T(double(a.rho0) + double(h.drho));
  if (u) {
    u[n] = T(h.ux);
    u[nodes + n] = T(h.uy);
    if constexpr (L::D == 3) u[2 * nodes + n] = T(h.uz);
  }
  if (pi1) {
    const R s = R(inv_omega1);
    if constexpr (L::D == 2) {
      pi1[n] = T(h.axx * s);
      pi1[nodes + n] = T(h.axy * s);
      pi1[2 * nodes + n] = T(h.ayy * s);
    } else {
      pi1[n] = T(h.axx * s);
      pi1[nodes + n] = T(h.axy * s);
      pi1[2 * nodes + n] = T(h.axz * s);
      pi1[3 * nodes + n] = T(h.ayy * s);
      pi1[4 * nodes + n] = T(h.ayz * s);
      pi1[5 * nodes + n] = T(h.azz * s);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions: wave butterfly (64 lanes) -> LDS across waves -> one
// partial per block; the final sum over blocks runs in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* __restrict__ out) {
  __shared__ double lds[NV][kReduceBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double s = wave_sum(v[c]);
    if (lane == 0) lds[c][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < kReduceBlock / 64; ++w) s += lds[threadIdx.x][w];
    out[int64_t(blockIdx.x) * NV + threadIdx.x] = s;
  }
}

// Per-block partial totals {rho, rho u_x, rho u_y, rho u_z, rho |u|^2 / 2}.
template <class L, class S>
__global__ void __launch_bounds__(kReduceBlock) k_totals(const S* __restrict__ src, double* __restrict__ partials,
                                                         StepArgs a, int64_t per_block) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t begin = int64_t(blockIdx.x) * per_block;
  const int64_t end = begin + per_block < nodes ? begin + per_block : nodes;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t n = begin + threadIdx.x; n < end; n += kReduceBlock) {
    double f[L::Q];
    const int64_t off = node_offset(a, uint32_t(n));
    sfor<0, L::Q>([&](auto I) { f[I] = double(src[int64_t(I) * a.si + off]); });
    const Moments<double> m = raw_moments<L, double>(f);
    const double rho = a.rho0 + m.d0;
    acc[0] += rho;
    acc[1] += m.jx;
    acc[2] += m.jy;
    acc[3] += m.jz;
    acc[4] += 0.5 * (m.jx * m.jx + m.jy * m.jy + m.jz * m.jz) / rho;
  }
  block_sum_store<5>(acc, partials);
}

// Sum of per-block partials in a fixed order: thread t adds blocks t, t+B, ...
// then a fixed tree over the threads.
template <int NV>
__global__ void __launch_bounds__(kReduceBlock) k_final(const double* __restrict__ partials, int nblocks,
                                                        double* __restrict__ out) {
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kReduceBlock) {
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] += partials[int64_t(b) * NV + c];
  }
  block_sum_store<NV>(acc, out);
}

// Velocity field (FP64) of the stored state, for the vorticity diagnostic.
template <class L, class S>
__global__ void __launch_bounds__(256) k_velocity(const S* __restrict__ src, double* __restrict__ u, StepArgs a) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  double f[L::Q];
  const int64_t off = node_offset(a, uint32_t(n));
  sfor<0, L::Q>([&](auto I) { f[I] = double(src[int64_t(I) * a.si + off]); });
  const Moments<double> m = raw_moments<L, double>(f);
  const double inv = 1.0 / (a.rho0 + m.d0);
  u[n] = m.jx * inv;
  u[nodes + n] = m.jy * inv;
  if constexpr (L::D == 3) u[2 * nodes + n] = m.jz * inv;
}

// ---------------------------------------------------------------------------
// Block of the population step: 256 threads as bx x (256 / bx) with bx in
// {256, 128, 64}, the width leaving the fewest idle lanes at the end of a row
// (ties: the wider).  With 256-wide blocks only, nx = 320 / 384 / 448 left
// 37% / 25% / 12% of the lanes idle and ran at 21.2 / 22.0 / 23.4 GLUPS
// (D3Q27 FP32) against 27.5 at 256 and 26.4 at 512.
inline dim3 step_block(int nx) {
  int best = 256, idle = (nx + 255) / 256 * 256 - nx;
  for (int bx : {128, 64}) {
    const int w = (nx + bx - 1) / bx * bx - nx;
    if (w < idle) {
      best = bx;
      idle = w;
    }
  }
  return dim3(unsigned(best), unsigned(256 / best));
}

inline hipError_t step_grid(const StepArgs& a, dim3& grid, dim3& block) {
  block = step_block(a.nx);
  grid = dim3(unsigned((a.nx + block.x - 1) / block.x), unsigned((a.ny + block.y - 1) / block.y), unsigned(a.nz));
  return (grid.y > 65535u || grid.z > 65535u) ? hipErrorInvalidValue : hipSuccess;
}

// Blocks of the population step per compute unit, limited by reserving LDS
// that the kernel does not use (0: no limit, eight 256-thread blocks, eight
// waves per SIMD).  Measured on MI355X, one run, interleaved (GLUPS, default
// -> six blocks): D3Q27 FP16 512^3 50.2 -> 54.0, 256^3 54.4 -> 55.8; FP64
// 512^3 11.8 -> 12.1, 256^3 unchanged.  D3Q27 FP32 gains nothing, and D3Q19
// FP16 (71.1 -> 69.3) and D2Q9 FP16 (151 -> 138) lose, so they keep every
// block.  With 27 streams of 2- or 8-byte lanes, fewer waves in flight keep
// fewer DRAM pages open at once.  LBRR_STEP_BLOCKS_PER_CU=0..8 overrides.
template <class L, class S>
int step_blocks_per_cu() {
  int blocks = (L::Q == 27 && sizeof(S) != 4) ? 6 : 0;
  if (const char* e = std::getenv("LBRR_STEP_BLOCKS_PER_CU")) {
    const int v = std::atoi(e);
    if (v >= 0 && v <= 8) blocks = v;
  }
  return blocks;
}

// Dynamic LDS bytes per block that leave room for at most `blocks` blocks per
// compute unit (a multiple of 2 KiB, so the count does not depend on the
// allocation granularity); 0 when there is no limit or the device is unknown.
inline unsigned lds_reserve(int blocks) {
  if (blocks <= 0) return 0u;
  int dev = 0, per_cu = 0, per_block = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 0u;
  const int r = per_cu / blocks / 2048 * 2048;
  return unsigned(r < per_block ? r : per_block);
}

template <class L, int N, class S>
hipError_t launch_step(const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  dim3 grid, block;
  if (step_grid(a, grid, block) != hipSuccess) return hipErrorInvalidValue;
  if (uint64_t(a.nx) * sizeof(S) > 0xffffffffull) return hipErrorInvalidValue;  // 32-bit lane byte offsets
  const unsigned lds = lds_reserve(step_blocks_per_cu<L, S>());
  hipLaunchKernelGGL((k_step<L, N, S>), grid, block, lds, s, static_cast<const S*>(src), static_cast<S*>(dst), a);
  return hipGetLastError();
}

template <class L, int N, class S>
hipError_t launch_step_walls(const void* src, void* dst, const StepArgs& a, int walls, hipStream_t s) {
  dim3 grid, block;
  if (step_grid(a, grid, block) != hipSuccess) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_step_walls<L, N, S>), grid, block, 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                     a, walls);
  return hipGetLastError();
}

template <class L, int N, class S>
hipError_t launch_init(int dtype, const void* rho, const void* u, const void* pi1, void* dst, const StepArgs& a,
                       hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  dim3 grid(unsigned((nodes + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL((k_init<L, N, S, double>), grid, dim3(256), 0, s, static_cast<const double*>(rho),
                       static_cast<const double*>(u), static_cast<const double*>(pi1), static_cast<S*>(dst), a);
  else
    hipLaunchKernelGGL((k_init<L, N, S, float>), grid, dim3(256), 0, s, static_cast<const float*>(rho),
                       static_cast<const float*>(u), static_cast<const float*>(pi1), static_cast<S*>(dst), a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_moments(int dtype, const void* src, void* rho, void* u, void* pi1, const StepArgs& a,
                          double inv_omega1, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  dim3 grid(unsigned((nodes + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL((k_moments<L, S, double>), grid, dim3(256), 0, s, static_cast<const S*>(src),
                       static_cast<double*>(rho), static_cast<double*>(u), static_cast<double*>(pi1), a, inv_omega1);
  else
    hipLaunchKernelGGL((k_moments<L, S, float>), grid, dim3(256), 0, s, static_cast<const S*>(src),
                       static_cast<float*>(rho), static_cast<float*>(u), static_cast<float*>(pi1), a, inv_omega1);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_totals(const void* src, double* partials, int nblocks, double* out, const StepArgs& a,
                         hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t per_block = (nodes + nblocks - 1) / nblocks;
  hipLaunchKernelGGL((k_totals<L, S>), dim3(nblocks), dim3(kReduceBlock), 0, s, static_cast<const S*>(src), partials,
                     a, per_block);
  hipLaunchKernelGGL((k_final<5>), dim3(1), dim3(kReduceBlock), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_velocity(const void* src, double* u, const StepArgs& a, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  hipLaunchKernelGGL((k_velocity<L, S>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                     static_cast<const S*>(src), u, a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_repack(const void* src, void* dst, bool to_compact, const StepArgs& a, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  hipLaunchKernelGGL((k_repack<L, S>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                     static_cast<const S*>(src), static_cast<S*>(dst), a, to_compact);
  return hipGetLastError();
}

// order dispatch: N in [2, L::NMAX]
template <class L, class S>
hipError_t step_by_order(int order, const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_step<L, 2, S>(src, dst, a, s);
    case 3: return launch_step<L, 3, S>(src, dst, a, s);
    case 4: return launch_step<L, 4, S>(src, dst, a, s);
    case 5: if constexpr (L::NMAX >= 5) return launch_step<L, 5, S>(src, dst, a, s); break;
    case 6: if constexpr (L::NMAX >= 6) return launch_step<L, 6, S>(src, dst, a, s); break;
  }
  return hipErrorInvalidValue;
}

template <class L, class S>
hipError_t init_by_order(int order, int dtype, const void* rho, const void* u, const void* pi1, void* dst,
                         const StepArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_init<L, 2, S>(dtype, rho, u, pi1, dst, a, s);
    case 3: return launch_init<L, 3, S>(dtype, rho, u, pi1, dst, a, s);
    case 4: return launch_init<L, 4, S>(dtype, rho, u, pi1, dst, a, s);
    case 5: if constexpr (L::NMAX >= 5) return launch_init<L, 5, S>(dtype, rho, u, pi1, dst, a, s); break;
    case 6: if constexpr (L::NMAX >= 6) return launch_init<L, 6, S>(dtype, rho, u, pi1, dst, a, s); break;
  }
  return hipErrorInvalidValue;
}

}  // namespace lbrr
