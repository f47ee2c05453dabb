// Dense (matrix-core) two-mode gate variant.
#pragma once

#include "fock_internal.h"

namespace fock {

bool dense_supported(int d);
size_t dense_w_bytes(int d);  // scratch for the real 2d^2 x 2d^2 matrix (0 if unsupported)
// psi <- U psi (dag: U^+) on the pair (i, j) by the dense GEMM; W: dense_w_bytes(d) of device scratch.
int launch_gate_dense(const Geometry &geo, int i, int j, int kind, bool dag, const float2 *U, const float2 *src,
                      float2 *psi, float *W, hipStream_t s);
int gate_variant();

}  // namespace fock
