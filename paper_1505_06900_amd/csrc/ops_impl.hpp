// Per-lattice dispatch tables (LatticeOps) over order and storage, used by
// the C ABI.  Population storage: 0 FP64, 1 FP32, 2 FP16 (kernels.hpp);
// moment storage: 3 FP64, 4 FP32 (mkernels.hpp).
#pragma once

#include "kernels.hpp"
#include "mkernels.hpp"

namespace lbrr {

template <class L, class S>
hipError_t mstep_by_order(int order, const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_mstep<L, 2, S>(src, dst, a, s);
    case 3: return launch_mstep<L, 3, S>(src, dst, a, s);
    case 4: return launch_mstep<L, 4, S>(src, dst, a, s);
    case 5: if constexpr (L::NMAX >= 5) return launch_mstep<L, 5, S>(src, dst, a, s); break;
    case 6: if constexpr (L::NMAX >= 6) return launch_mstep<L, 6, S>(src, dst, a, s); break;
  }
  return hipErrorInvalidValue;
}

template <class L, class S>
hipError_t mpop_by_order(int order, const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return launch_mpopulations<L, 2, S>(src, dst, a, s);
    case 3: return launch_mpopulations<L, 3, S>(src, dst, a, s);
    case 4: return launch_mpopulations<L, 4, S>(src, dst, a, s);
    case 5: if constexpr (L::NMAX >= 5) return launch_mpopulations<L, 5, S>(src, dst, a, s); break;
    case 6: if constexpr (L::NMAX >= 6) return launch_mpopulations<L, 6, S>(src, dst, a, s); break;
  }
  return hipErrorInvalidValue;
}

template <class L, class S>
hipError_t step_walls_by_order(int order, const void* src, void* dst, const StepArgs& a, int walls, hipStream_t s) {
  switch (order) {
    case 2: return launch_step_walls<L, 2, S>(src, dst, a, walls, s);
    case 3: return launch_step_walls<L, 3, S>(src, dst, a, walls, s);
    case 4: return launch_step_walls<L, 4, S>(src, dst, a, walls, s);
    case 5: if constexpr (L::NMAX >= 5) return launch_step_walls<L, 5, S>(src, dst, a, walls, s); break;
    case 6: if constexpr (L::NMAX >= 6) return launch_step_walls<L, 6, S>(src, dst, a, walls, s); break;
  }
  return hipErrorInvalidValue;
}

template <class L>
struct OpsImpl {
  static hipError_t step(int order, int storage, const void* src, void* dst, const StepArgs& a, hipStream_t s) {
    switch (storage) {
      case 0: return step_by_order<L, double>(order, src, dst, a, s);
      case 1: return step_by_order<L, float>(order, src, dst, a, s);
      case 2: return step_by_order<L, _Float16>(order, src, dst, a, s);
      case 3: return mstep_by_order<L, double>(order, src, dst, a, s);
      case 4: return mstep_by_order<L, float>(order, src, dst, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t init(int order, int storage, int dtype, const void* rho, const void* u, const void* pi1,
                         void* dst, const StepArgs& a, hipStream_t s) {
    switch (storage) {
      case 0: return init_by_order<L, double>(order, dtype, rho, u, pi1, dst, a, s);
      case 1: return init_by_order<L, float>(order, dtype, rho, u, pi1, dst, a, s);
      case 2: return init_by_order<L, _Float16>(order, dtype, rho, u, pi1, dst, a, s);
      case 3: return launch_minit<L, double>(dtype, rho, u, pi1, dst, a, s);
      case 4: return launch_minit<L, float>(dtype, rho, u, pi1, dst, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t moments(int storage, int dtype, const void* src, void* rho, void* u, void* pi1,
                            const StepArgs& a, double inv_omega1, hipStream_t s) {
    switch (storage) {
      case 0: return launch_moments<L, double>(dtype, src, rho, u, pi1, a, inv_omega1, s);
      case 1: return launch_moments<L, float>(dtype, src, rho, u, pi1, a, inv_omega1, s);
      case 2: return launch_moments<L, _Float16>(dtype, src, rho, u, pi1, a, inv_omega1, s);
      case 3: return launch_mmoments<L, double>(dtype, src, rho, u, pi1, a, s);
      case 4: return launch_mmoments<L, float>(dtype, src, rho, u, pi1, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t totals(int storage, const void* src, double* partials, int nblocks, double* out,
                           const StepArgs& a, hipStream_t s) {
    switch (storage) {
      case 0: return launch_totals<L, double>(src, partials, nblocks, out, a, s);
      case 1: return launch_totals<L, float>(src, partials, nblocks, out, a, s);
      case 2: return launch_totals<L, _Float16>(src, partials, nblocks, out, a, s);
      case 3: return launch_mtotals<L, double>(src, partials, nblocks, out, a, s);
      case 4: return launch_mtotals<L, float>(src, partials, nblocks, out, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t velocity(int storage, const void* src, double* u, const StepArgs& a, hipStream_t s) {
    switch (storage) {
      case 0: return launch_velocity<L, double>(src, u, a, s);
      case 1: return launch_velocity<L, float>(src, u, a, s);
      case 2: return launch_velocity<L, _Float16>(src, u, a, s);
      case 3: return launch_mvelocity<L, double>(src, u, a, s);
      case 4: return launch_mvelocity<L, float>(src, u, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t repack(int storage, const void* src, void* dst, bool to_compact, const StepArgs& a,
                           hipStream_t s) {
    switch (storage) {
      case 0: return launch_repack<L, double>(src, dst, to_compact, a, s);
      case 1: return launch_repack<L, float>(src, dst, to_compact, a, s);
      case 2: return launch_repack<L, _Float16>(src, dst, to_compact, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t mpopulations(int order, int storage, const void* src, void* dst, const StepArgs& a,
                                 hipStream_t s) {
    switch (storage) {
      case 3: return mpop_by_order<L, double>(order, src, dst, a, s);
      case 4: return mpop_by_order<L, float>(order, src, dst, a, s);
    }
    return hipErrorInvalidValue;
  }
  static hipError_t step_walls(int order, int storage, const void* src, void* dst, const StepArgs& a, int walls,
                               hipStream_t s) {
    switch (storage) {
      case 0: return step_walls_by_order<L, double>(order, src, dst, a, walls, s);
      case 1: return step_walls_by_order<L, float>(order, src, dst, a, walls, s);
      case 2: return step_walls_by_order<L, _Float16>(order, src, dst, a, walls, s);
    }
    return hipErrorInvalidValue;
  }
  static const LatticeOps& table() {
    static const LatticeOps t = {L::Q, L::D, L::NMAX, &step, &init, &moments, &totals, &velocity, &repack,
                                 &mpopulations, &step_walls};
    return t;
  }
};

}  // namespace lbrr
