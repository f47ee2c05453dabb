// Explicit instantiations of the gate kernels for d in {6, 7}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(6)
FOCK_GATE_INSTANTIATE(7)
}  // namespace fock
