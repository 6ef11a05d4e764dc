// Kernel instantiations for the D3Q27 lattice.
#include "ops_impl.hpp"

namespace lbrr {
const LatticeOps& ops_d3q27() { return OpsImpl<D3Q27>::table(); }
}  // namespace lbrr
