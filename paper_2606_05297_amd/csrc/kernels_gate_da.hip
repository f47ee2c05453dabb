// Explicit instantiations of the gate kernels for d in {2, 3, 4, 5}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(2)
FOCK_GATE_INSTANTIATE(3)
FOCK_GATE_INSTANTIATE(4)
FOCK_GATE_INSTANTIATE(5)
}  // namespace fock
