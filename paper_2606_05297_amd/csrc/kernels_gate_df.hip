// Explicit instantiations of the gate kernels for d in {15, 16}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(15)
FOCK_GATE_INSTANTIATE(16)
}  // namespace fock
