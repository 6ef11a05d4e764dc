// Host-side interface between the C ABI (api.hip) and the per-lattice kernel
// translation units.  Plain function pointers; no torch types.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbrr {

constexpr int kReduceBlock = 256;
// Inner rows of a row-aligned tile of the 3D FP32 moment step (k_mstep_t):
// TY + 3 waves per block.  9 rows, 12 waves: no spills (D3Q27 order 4: 123
// VGPRs, one block per CU); 13 rows, 16 waves (1024 threads, 128 VGPRs per
// lane) spilled 11-18 VGPRs.
constexpr int kTileRows = 9;

// Launch parameters shared by the kernels.  Population (or moment field) i of node (x, y, z)
// lives at element i*si + z*sz + y*sy + x of a buffer; the host picks the
// strides (layout) and checks that every index stays inside the allocation.
struct StepArgs {
  int nx, ny, nz;
  int64_t si, sy, sz;  // element strides of population, row and plane
  double rho0;         // reference density of the deviation storage
  double omega1;       // 1 - 1/tau
  int lz;              // z-planes per block of the moment-state step (3D)
  int walls;           // moment-state step: resting walls on the axes of this mask (bit 0 x, 1 y, 2 z)
};

struct LatticeOps {
  int q, d, nmax;
  hipError_t (*step)(int order, int storage, const void* src, void* dst, const StepArgs& a, hipStream_t s);
  hipError_t (*init)(int order, int storage, int dtype, const void* rho, const void* u, const void* pi1, void* dst,
                     const StepArgs& a, hipStream_t s);
  hipError_t (*moments)(int storage, int dtype, const void* src, void* rho, void* u, void* pi1, const StepArgs& a,
                        double inv_omega1, hipStream_t s);
  hipError_t (*totals)(int storage, const void* src, double* partials, int nblocks, double* out, const StepArgs& a,
                       hipStream_t s);
  hipError_t (*velocity)(int storage, const void* src, double* u, const StepArgs& a, hipStream_t s);
  // copy between the internal layout and compact SoA [q][nz][ny][nx] (to_compact: internal -> compact)
  hipError_t (*repack)(int storage, const void* src, void* dst, bool to_compact, const StepArgs& a, hipStream_t s);
  // moment storage: post-collision deviations of the state, compact SoA [q][nz][ny][nx]
  hipError_t (*mpopulations)(int order, int storage, const void* src, void* dst, const StepArgs& a, hipStream_t s);
  // population storage with resting walls on the axes of `walls` (bit 0 x, 1 y, 2 z)
  hipError_t (*step_walls)(int order, int storage, const void* src, void* dst, const StepArgs& a, int walls,
                           hipStream_t s);
};

// Storage kinds (values of lb_storage): populations 0 FP64, 1 FP32, 2 FP16;
// moments 3 FP64, 4 FP32.
constexpr bool is_moment_storage(int storage) { return storage == 3 || storage == 4; }

const LatticeOps& ops_d2q9();
const LatticeOps& ops_d3q19();
const LatticeOps& ops_d3q27();

// diagnostics kernels (diag.hip)
hipError_t launch_probe(int kind, int vec_bytes, int blocks_per_cu, int nontemporal, int streams, const void* src,
                        void* dst, size_t nbytes, int cus, hipStream_t s);
hipError_t launch_enstrophy(const double* u, int d, int nx, int ny, int nz, int walls, double* partials, int nblocks,
                            double* out, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t n, hipStream_t s);

}  // namespace lbrr
