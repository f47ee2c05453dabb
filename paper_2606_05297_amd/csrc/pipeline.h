// Host pipeline shared by the C ABI entry points and the ADAPT driver.
#pragma once

#include "fock_internal.h"

namespace fock {

struct Layout {
  size_t theta = 0, recs = 0, utab = 0, partial = 0, result = 0, pairs = 0, diags = 0, wdense = 0, total = 0;
  int G = 0;     // blocks of the row-parallel kernels
  int rs = 0;    // row stride of the per-gate reverse-step partials
  int nmax = 0;  // gates
  int pmax = 0;  // pool chunk
};

struct Ctx {
  Geometry g;
  HamArgs h;
  EigTables T;
  hipStream_t s;
  char *ws;
  Layout L;
  // Optional store of forward states: nstore device buffers of one state each
  // (stride `sstride` amplitudes).  With a store, a gradient evaluation keeps
  // phi_k = O_k..O_1 psi0 in buffer k - 1 and the reverse sweep reads it
  // instead of undoing each gate on phi.
  float2 *store = nullptr;
  int nstore = 0;
  size_t sstride = 0;
  // Real states (d = 8, ADAPT driver): float32 copies of psi0 and the forward
  // and adjoint states, used by evaluations whose gates are all HR or PR.
  float *psi0_r = nullptr, *phi_r = nullptr, *lam_r = nullptr;
};

int check_geometry(int L, int d, uint32_t *namp);
// check_ham takes full d^L states only; check_ham_layout also the parity-halved
// layout (namp = d^L / 2 then) and, with allow_real, FOCK_LAYOUT_REAL.
int check_ham(const fock_ham_t *h, uint32_t *namp);
int check_ham_layout(const fock_ham_t *h, uint32_t *namp, bool allow_real = false);
bool half_layout_op_ok(const fock_op_t &op, int L);
// Switch of the ADAPT driver's real states (FOCK_REAL_*).
int real_states_mode();
// Switch of the ADAPT driver's automatic parity-halved layout (FOCK_SECTOR_*),
// and whether it applies to this chain, pool and warm-up layer.
int sector_layout_mode();
bool half_layout_wanted(const fock_ham_t &h, const fock_op_t *pool, int P, const fock_op_t *ops, int n);
int check_op(const fock_op_t &op, int L);
int check_ptr(const void *p, const char *name);
HamArgs make_ham_args(const fock_ham_t &h);
Layout make_layout(uint32_t namp, int L, int d, int P, int n, int half = 0);
int make_ctx(const fock_ham_t &ham, uint32_t namp, int P, int n, void *ws, size_t ws_bytes, hipStream_t s, Ctx *c);
// Attach a store of nmax forward states to c if switched on and the device has
// room; *owner receives the allocation to free (nullptr: no store).
int attach_state_store(Ctx &c, int nmax, void **owner);
int stage_gates(Ctx &c, const fock_op_t *ops, const double *theta, int n, const int *nblk);
// psi <- O_k src (src == psi: in place)
int forward_gate(Ctx &c, const fock_op_t &op, int k, bool dag, const float2 *src, float2 *psi);
int apply_h_dev(Ctx &c, const float2 *psi, float2 *hpsi, double *res2);
int fetch_results(Ctx &c, int count, double *host);
// Energy (Rayleigh quotient) and optionally all dE/dtheta of ops/theta applied to psi0.
int run_circuit(Ctx &c, const fock_op_t *ops, const double *theta, int n, const void *psi0, float2 *phi,
                float2 *lam, bool grad, double *E, double *norm2, double *dE);
// All dE/dtheta from phi = psi_n, lam = H psi_n (overwritten) by the reverse sweep alone.
int run_reverse(Ctx &c, const fock_op_t *ops, const double *theta, int n, float2 *phi, float2 *lam, double norm2,
                double *dE);
// psi = circuit(psi0) into phi, its Rayleigh energy, norm and the raw pool
// gradients 2 Re <H psi|A_k psi> (g, host, P), with H psi left in lam.
int run_score(Ctx &c, const fock_op_t *ops, const double *theta, int n, const void *psi0, float2 *phi,
              float2 *lam, const fock_op_t *pool, int P, double *E, double *norm2, double *g);
// H psi, (<psi|H psi>, <psi|psi>) into res[0..1] and the pool gradients into
// res[2..2+P) (device); fused slab scoring where the pool allows it.
int score_dev(Ctx &c, const fock_op_t *pool, int P, const float2 *psi, float2 *hpsi, double *res);
// 2 Re <hpsi|A_k psi> for the pool into res[0..P) (device).
int pool_dev(Ctx &c, const fock_op_t *pool, int P, const float2 *psi, const float2 *hpsi, double *res);

}  // namespace fock
