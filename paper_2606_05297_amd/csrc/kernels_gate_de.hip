// Explicit instantiations of the gate kernels for d in {13, 14}.
#include "gate_kernels.h"

namespace fock {
FOCK_GATE_INSTANTIATE(13)
FOCK_GATE_INSTANTIATE(14)
}  // namespace fock
