// Kernel instantiations for the D3Q19 lattice.
#include "kernels.hpp"

namespace lbrr {
const LatticeOps& ops_d3q19() { return OpsImpl<D3Q19>::table(); }
}  // namespace lbrr
