// Explicit instantiations of the gate kernels for d in {8}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(8)
}  // namespace fock
