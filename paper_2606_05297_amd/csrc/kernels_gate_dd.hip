// Explicit instantiations of the gate kernels for d in {9, 10, 11, 12}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(9)
FOCK_GATE_INSTANTIATE(10)
FOCK_GATE_INSTANTIATE(11)
FOCK_GATE_INSTANTIATE(12)
}  // namespace fock
