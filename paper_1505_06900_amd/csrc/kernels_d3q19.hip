// Kernel instantiations for the D3Q19 lattice.
#include "ops_impl.hpp"

namespace lbrr {
const LatticeOps& ops_d3q19() { return OpsImpl<D3Q19>::table(); }
}  // namespace lbrr
