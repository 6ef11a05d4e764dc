// Bandwidth probes: plain streams of known size over device buffers.  They
// measure what HBM delivers to simple access patterns on this GPU, the
// achievable ceiling beside the 8 TB/s peak against which the step kernels'
// rooflines are quoted.  Nothing of the lattice Boltzmann update runs here.
//
// kind 0  copy          dst[i] = src[i]
// kind 1  read          every element of src is loaded and folded into a
//                       per-thread value that is written only if it equals
//                       a value a zero-filled buffer cannot produce
// kind 2  write         dst[i] = a constant
// kind 3  stream copy   the buffer is split into `streams` equal planes and
//                       each thread copies its element of every plane (as a
//                       step kernel reads q planes and writes q planes)
// Elements are 4, 8 or 16 bytes per lane.  blocks_per_cu = 0 launches one
// thread per element (kinds 0-2) or per plane element (kind 3); > 0 launches
// that many 256-thread blocks per compute unit, each striding over the buffer
// (kinds 0-2).  Loads and stores are plain or non-temporal.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ops.hpp"

namespace lbrr {

namespace {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class V>
__device__ __forceinline__ unsigned fold(V v) {
  if constexpr (sizeof(V) == 4) return v;
  else if constexpr (sizeof(V) == 8) return v.x ^ v.y;
  else return v.x ^ v.y ^ v.z ^ v.w;
}

template <class V>
__device__ __forceinline__ V splat(unsigned c) {
  if constexpr (sizeof(V) == 4) return c;
  else if constexpr (sizeof(V) == 8) return V{c, c};
  else return V{c, c, c, c};
}

template <class V, bool NT>
__device__ __forceinline__ V load(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <class V, bool NT>
__device__ __forceinline__ void store(V v, V* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// kinds 0-2, one element per thread (Stride = false) or grid-stride (Stride = true)
template <class V, int Kind, bool NT, bool Stride>
__global__ void __launch_bounds__(256) k_probe(const V* __restrict__ src, V* __restrict__ dst, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t step = Stride ? size_t(gridDim.x) * blockDim.x : n;
  unsigned acc = 0;
  for (; i < n; i += step) {
    if constexpr (Kind == 0) store<V, NT>(load<V, NT>(src + i), dst + i);
    if constexpr (Kind == 1) acc ^= fold(load<V, NT>(src + i)) + unsigned(i);
    if constexpr (Kind == 2) store<V, NT>(splat<V>(0x3c003c00u), dst + i);
  }
  if constexpr (Kind == 1) {
    // the fold of a zero-filled buffer is the xor of the indices, never ~0 over a whole grid
    if (acc == 0xffffffffu && threadIdx.x == 0) dst[blockIdx.x] = splat<V>(acc);
  }
}

// kind 3: `streams` planes of `plane` elements each, one plane element per thread
template <class V, bool NT>
__global__ void __launch_bounds__(256) k_probe_streams(const V* __restrict__ src, V* __restrict__ dst, size_t plane,
                                                       int streams) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  V v[32];
#pragma unroll
  for (int s = 0; s < 32; ++s)
    if (s < streams) v[s] = load<V, NT>(src + size_t(s) * plane + i);
#pragma unroll
  for (int s = 0; s < 32; ++s)
    if (s < streams) store<V, NT>(v[s], dst + size_t(s) * plane + i);
}

template <class V, int Kind, bool NT>
hipError_t launch_kind(const void* src, void* dst, size_t nbytes, int blocks_per_cu, int streams, int cus,
                       hipStream_t s) {
  const size_t n = nbytes / sizeof(V);
  const V* sp = static_cast<const V*>(src);
  V* dp = static_cast<V*>(dst);
  if (Kind == 3) {
    const size_t plane = n / size_t(streams);
    const size_t blocks = (plane + 255) / 256;
    if (blocks == 0 || blocks > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_probe_streams<V, NT>), dim3(unsigned(blocks)), dim3(256), 0, s, sp, dp, plane, streams);
  } else if (blocks_per_cu == 0) {
    const size_t blocks = (n + 255) / 256;
    if (blocks == 0 || blocks > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_probe<V, Kind, NT, false>), dim3(unsigned(blocks)), dim3(256), 0, s, sp, dp, n);
  } else {
    const unsigned blocks = unsigned(blocks_per_cu) * unsigned(cus);
    hipLaunchKernelGGL((k_probe<V, Kind, NT, true>), dim3(blocks), dim3(256), 0, s, sp, dp, n);
  }
  return hipGetLastError();
}

template <class V, bool NT>
hipError_t launch_vec(int kind, const void* src, void* dst, size_t nbytes, int blocks_per_cu, int streams, int cus,
                      hipStream_t s) {
  switch (kind) {
    case 0: return launch_kind<V, 0, NT>(src, dst, nbytes, blocks_per_cu, streams, cus, s);
    case 1: return launch_kind<V, 1, NT>(src, dst, nbytes, blocks_per_cu, streams, cus, s);
    case 2: return launch_kind<V, 2, NT>(src, dst, nbytes, blocks_per_cu, streams, cus, s);
    default: return launch_kind<V, 3, NT>(src, dst, nbytes, blocks_per_cu, streams, cus, s);
  }
}

}  // namespace

hipError_t launch_probe(int kind, int vec_bytes, int blocks_per_cu, int nontemporal, int streams, const void* src,
                        void* dst, size_t nbytes, int cus, hipStream_t s) {
  if (nontemporal) {
    if (vec_bytes == 4) return launch_vec<unsigned, true>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
    if (vec_bytes == 8) return launch_vec<u32x2, true>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
    return launch_vec<u32x4, true>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
  }
  if (vec_bytes == 4) return launch_vec<unsigned, false>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
  if (vec_bytes == 8) return launch_vec<u32x2, false>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
  return launch_vec<u32x4, false>(kind, src, dst, nbytes, blocks_per_cu, streams, cus, s);
}

}  // namespace lbrr
