// Kernel instantiations for the D2Q9 lattice.
#include "ops_impl.hpp"

namespace lbrr {
const LatticeOps& ops_d2q9() { return OpsImpl<D2Q9>::table(); }
}  // namespace lbrr
