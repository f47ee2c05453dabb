// FP64-state path: parameters and launchers (f64_kernels.hip).
#pragma once

#include "device_common.h"

namespace fock {

// Hamiltonian in double precision (same terms and signs as HamArgs).
struct H64 {
  int L, d, wrap;  // wrap: the ring bond (0, L-1) exists
  uint32_t n_amp;
  double J, Delta, c2, mu;  // c2 = U/2 + K
};

// Fibres of one op: M local amplitudes (d^2 over modes i < j, or d over mode i
// when j = -1), nfib fibres, fpw fibres per 256-thread workgroup.
struct Fib64 {
  int L, d, i, j, M, fpw;
  uint32_t si, sj, nfib;
};

Fib64 make_fib64(int L, int d, const fock_op_t &op);
int fib64_blocks(const Fib64 &a);
int launch64_apply_h(const H64 &h, const double2 *psi, double2 *hpsi, double *partial, int *nblocks, hipStream_t s);
int launch64_fib_apply(const Fib64 &a, const double2 *src, double2 *dst, const double2 *U, bool dag, hipStream_t s);
int launch64_fib_adj(const Fib64 &a, double2 *phi, double2 *lam, const double2 *U, const double2 *A,
                     double *partial, hipStream_t s);
int launch64_fib_pool(const Fib64 &a, const double2 *psi, const double2 *hpsi, const double2 *A, double *partial,
                      hipStream_t s);
// Dense M x M tables of n gates at utab + recs[k].u_off (Mmax = largest M).
int launch64_build(const double *theta, const GateRec *recs, int n, const EigTables &T, int Mmax, double2 *utab,
                   hipStream_t s);

}  // namespace fock
