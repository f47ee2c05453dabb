// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fock.h"

namespace fock {

constexpr int kMaxD = 16;
constexpr int kMaxL = 24;
constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxPairs = 160;       // distinct mode pairs per pool-gradient launch
constexpr int kMaxSlots = 256;       // pool entries per pool-gradient launch
constexpr int kMaxDiagOps = 48;      // single-mode pool entries per launch

// ---------------------------------------------------------------- errors
int set_error(int code, const char *fmt, ...);
#define FOCK_HIP(call)                                                             \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::fock::set_error(FOCK_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- exact unsigned division by an invariant
// Granlund & Montgomery (1994), Thm 4.2 with N = 32: for 0 <= n < 2^31,
// floor(n / v) = (n * m) >> (32 + l) with l = ceil(log2 v), m = floor(2^(32+l)/v) + 1.
struct FastDiv {
  uint64_t m;
  uint32_t sh;
  uint32_t v;
};
FastDiv make_fastdiv(uint32_t v);
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.sh);
}

// ---------------------------------------------------------------- Hamiltonian on the device
struct HamArgs {
  int L, d;
  int nrows;          // d^(L-1): rows of d amplitudes along mode 0
  int periodic_wrap;  // 1 if the bond (0, L-1) exists and L >= 3
  float J, Delta, c2, mu;  // c2 = U/2 + K
  int srow[kMaxL];    // d^(r-1) for r >= 1: stride of mode r in rows
  float sq[kMaxD + 1];  // sqrt(0..d)
  const int *order;   // tile processed by workgroup b (device table), or null: contiguous runs per XCD
  int hi_m;           // two-pass stencil: bonds among the top hi_m modes (and the ring bond) are applied
                      // by a first pass that stages those modes in LDS; 0 = single pass
  int lanes;          // 1: lane-split stencil (d = 8, 4 <= L <= 10, open chain, single pass)
  int slab;           // 1: two-pass slab stencil (L = 8, d = 8; stencil2.hip)
  int half;           // 1: parity-halved layout (the top mode stores m with n_top = 2 m + parity)
  int sector;         // total parity of the states in the halved layout (0 even, 1 odd)
};

// ---------------------------------------------------------------- pool gradients
struct PoolPair {
  int16_t i, j;
  int16_t slot[5];  // output slot for HR, HI, DH, PR, PI (-1 = absent)
  int16_t pad;
};
struct PoolDiag {
  int16_t r, type, slot, r2;  // KERR / ROT on mode r (r2 = -1), CK on modes (r, r2)
};
// Pool entries scored by the slab kernels (L = 8, d = 8): slot[p][type] for
// the pairs p = 0..6 ~ (p, p + 1) and p = 7 ~ the ring pair (0, 7), types
// HR..PI (-1 = absent); up to kSlabDiag diagonal entries (KERR, ROT, CK).
constexpr int kSlabDiag = 16;
struct SlabPool {
  int16_t slot[8][5];
  PoolDiag diag[kSlabDiag];
  int ndiag, nslots;
};

struct PoolArgs {
  int L, d, nrows, npairs, ndiag, nslots;
  int srow[kMaxL];
  float sq[kMaxD + 1];
  const int *order;  // as HamArgs::order
};

// ---------------------------------------------------------------- gates
// A two-mode gate on (i, j) with d levels acts blockwise.  Kind SUM groups
// (n_i, n_j) by n_i + n_j (number-conserving generators), kind DIFF by
// n_i - n_j (two-mode squeezers).  Blocks are indexed by s = 0..2d-2; within
// block s the members are ordered by increasing n_i:
//   SUM : n_i = a, n_j = s - a,       a in [max(0, s-d+1), min(s, d-1)]
//   DIFF: t = s - (d-1), n_i = a, n_j = a - t,  a in [max(0, t), min(d-1, d-1+t)]
// A packed table stores the blocks in order of s, each b x b row-major
// (entry [p][q] maps member q to member p).
enum GateKind { KIND_SUM = 0, KIND_DIFF = 1 };

// One gate of a circuit as seen by the device-side gate build.
struct GateRec {
  int type, u_off;  // generator type, complex offset of its table in the U buffer
  int nblk, pad;    // workgroups of its reverse-step kernel (partials to reduce)
};

// Per-(d) gate eigendata on the device: for each two-mode type t < 5, the
// packed blocks of V (complex double, b x b row-major per block, column m is
// eigenvector m) and the eigenvalues lambda (b per block) of G = -i A, and the
// packed blocks of A itself (complex float).
// Two-mode generator types with eigendata tables: HR, HI, DH, PR, PI and CK.
constexpr int kTwoModeTypes = 6;
// Table slot of a two-mode type (FOCK_HR..FOCK_PI -> 0..4, FOCK_CK -> 5).
__host__ __device__ inline int table_slot(int type) { return type == FOCK_CK ? 5 : type; }

struct EigTables {
  const double *V[kTwoModeTypes];
  const double *lam[kTwoModeTypes];
  const float2 *A[kTwoModeTypes];
  // single-mode squeezers SR (0), SI (1): d x d eigenvectors of G = -i A, its
  // eigenvalues, and A itself (dense d x d, row-major)
  const double *V1[2];
  const double *lam1[2];
  const float2 *A1[2];
  int d, psize;
};

// Angles and gate records of a short circuit, passed to the table build as
// kernel arguments instead of through a staging copy.
constexpr int kArgGates = 64;
struct GateArgs {
  int n, pad;
  double theta[kArgGates];
  GateRec rec[kArgGates];
};

// Parity-halved layout (d = 8, open chain, states of one total parity sigma):
// the top mode L-1 stores m = 0..d/2-1 and n_{L-1} = 2 m + ((n_0 + .. + n_{L-2}
// + sigma) mod 2), so a state holds d^L / 2 amplitudes at index
// sum_{r < L-1} n_r d^r + m d^(L-1).  Every generator that keeps the total
// parity and leaves mode L-1 alone acts on it as on a tensor whose top mode has
// d/2 levels; the pair (L-2, L-1) and the bonds that touch mode L-1 have
// kernels of their own.
struct Geometry {
  int L, d;
  uint32_t n_amp;
  int half = 0;    // 1: parity-halved layout (n_amp = d^L / 2)
  int sector = 0;  // its total parity
};
// Parity of the base-8 digit sum of x (digits are 3-bit fields; x < 2^30).
__host__ __device__ inline int octal_digit_parity(uint32_t x) { return __builtin_popcount(x & 0x09249249u) & 1; }

inline int block_lo(int kind, int d, int s) {
  if (kind == KIND_SUM) return s - (d - 1) > 0 ? s - (d - 1) : 0;
  int t = s - (d - 1);
  return t > 0 ? t : 0;
}
inline int block_hi(int kind, int d, int s) {
  if (kind == KIND_SUM) return s < d - 1 ? s : d - 1;
  int t = s - (d - 1);
  return (d - 1 + t) < d - 1 ? d - 1 + t : d - 1;
}
inline int packed_size(int d) {  // sum of b^2 over blocks (same for SUM and DIFF)
  int tot = 0;
  for (int s = 0; s <= 2 * d - 2; ++s) {
    int b = block_hi(KIND_SUM, d, s) - block_lo(KIND_SUM, d, s) + 1;
    tot += b * b;
  }
  return tot;
}

// Host: dense local generator (d^2 x d^2 with local index n_i*d + n_j for
// two-mode types, d x d for single-mode types), complex double interleaved.
void generator_dense(int type, int d, std::vector<double> &m);
int gate_kind(int type);
bool is_single_mode(int type);
// Generators diagonal in the Fock basis (KERR, ROT, CK): pool scoring takes
// them as -2 f(n) Im(conj(H psi) psi) terms instead of pair terms.
bool is_pool_diagonal(int type);
// Single-mode squeezers (SR, SI): dense d x d gate on each fibre of one mode.
bool is_squeeze(int type);
// Library-owned device eigendata for cutoff d (built on first use, per device).
int get_tables(int d, EigTables *out);
// Size of one gate's slot in a U buffer (complex entries).
inline int gate_stride(int d) { return packed_size(d); }

// ---------------------------------------------------------------- launchers (kernels_*.hip)
int launch_apply_h(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int *nblocks,
                   hipStream_t s);
int apply_h_blocks(const HamArgs &h);
// Rows per workgroup tile of the stencil-type kernels (apply-H, pool gradients).
int apply_h_tile_rows(int L, int d);
int apply_h_hi_modes(int L, int d, int periodic_wrap);
int launch_pool(const PoolArgs &a, const PoolPair *pairs, const PoolDiag *diags, const float2 *psi,
                const float2 *hpsi, double *partial, int *nblocks, hipStream_t s);
int pool_blocks(const PoolArgs &a);
int launch_gate_build(const double *theta, const GateRec *recs, int n, const EigTables &T, float2 *utab,
                      hipStream_t s);
int launch_gate_build_args(const GateArgs &ga, const EigTables &T, float2 *utab, double *theta_out,
                           GateRec *recs_out, hipStream_t s);
// psi <- U src (dag = false) or U^+ src (dag = true) for a two-mode gate on
// (i, j); src == psi applies it in place.
int launch_gate(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float2 *src, float2 *psi,
                hipStream_t s);
// Fused reverse step: partial[blk] = per-block sum of Re<lam|A phi>, then
// phi <- U^+ phi (unless write_phi is false: phi is then only read) and
// lam <- U^+ lam.
int launch_gate_adj(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float2 *phi,
                    float2 *lam, double *partial, hipStream_t s, bool write_phi = true);
int gate_blocks_count(const Geometry &g, int i);  // workgroups of a gate on (i, j)
// Top pair (L-2, L-1) of the parity-halved layout (gate_half.hip); the general
// launchers above route to these.
int launch_gate_half(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float2 *src,
                     float2 *psi, hipStream_t s);
int launch_gate_adj_half(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float2 *phi,
                         float2 *lam, double *partial, hipStream_t s, bool write_phi);
int half_top_blocks(const Geometry &g);
int gate_blocks_max(const Geometry &g);
// Single-mode diagonal gate with device phase table ph[d].
int launch_diag(const Geometry &g, int r, int type, bool dag, const float2 *ph, const float2 *src, float2 *psi,
                hipStream_t s);
int launch_diag_adj(const Geometry &g, int r, int type, const float2 *ph, float2 *phi, float2 *lam,
                    double *partial, hipStream_t s, bool write_phi = true);
int diag_blocks_count(const Geometry &g);
// A run of consecutive single-mode phase gates ops[k0..k1) (KERR / ROT, at
// most kMaxDiagRun) applied as one diagonal pass; U = table of gate k0 (the
// run's tables follow at the gate stride).  The reverse step writes gate g's
// workgroup sums to partial[g * rs + block] (diag_blocks_count(g) blocks).
constexpr int kMaxDiagRun = 32;
struct DiagRun {
  int nrows, ng, stride;  // rows of d amplitudes; gates; float2 between gate tables
  int8_t r[kMaxDiagRun];
  int8_t kerr[kMaxDiagRun];
  FastDiv dsr[kMaxDiagRun];  // divide a row index by d^(r-1) (r >= 1)
};
DiagRun diag_run_params(const Geometry &g, const fock_op_t *ops, int k0, int k1);
// End (exclusive) of the run of single-mode phase gates (KERR, ROT) that starts
// at ops[k] when at least two start there (at most kMaxDiagRun), else k.  The
// single-point drivers and the batched sweep group gates with this one rule.
int diag_run_end(const fock_op_t *ops, int n, int k);
int launch_diag_run(const Geometry &g, const DiagRun &a, bool dag, const float2 *U, const float2 *src, float2 *psi,
                    hipStream_t s);
int launch_diag_run_adj(const Geometry &g, const DiagRun &a, const float2 *U, float2 *phi, float2 *lam,
                        double *partial, int rs, hipStream_t s, bool write_phi = true);
// Squeezer gates (gate1_kernels.hip): U, A are d x d row-major; the reverse
// step and the pool scoring write one partial per workgroup
// (diag_blocks_count(g) of them).
int launch_gate1(const Geometry &g, int r, bool dag, const float2 *U, const float2 *src, float2 *psi,
                 hipStream_t s);
int launch_gate1_adj(const Geometry &g, int r, const float2 *U, const float2 *A, float2 *phi, float2 *lam,
                     double *partial, hipStream_t s);
int launch_pool1(const Geometry &g, int r, const float2 *A, const float2 *psi, const float2 *hpsi, double *partial,
                 int *nblocks, hipStream_t s);
// out[c] = sum_b partial[b * ncols + c] for c < ncols, in a fixed order.
int launch_reduce(const double *partial, int nblocks, int ncols, double *out, hipStream_t s);
// out[k] = sum_{b < recs[k].nblk} partial[k * row_stride + b] for k < n, in a fixed order.
int launch_reduce_rows(const double *partial, int row_stride, const GateRec *recs, int n, double *out,
                       hipStream_t s);
// The gate rows (into out[2 + k]) and the energy / norm partials epart (two
// columns of ne rows, into out[0], out[1]) of a gradient evaluation, one launch.
int launch_reduce_rows_energy(const double *partial, int row_stride, const GateRec *recs, int n,
                              const double *epart, int ne, double *out, hipStream_t s);

// ---------------------------------------------------------------- profiling
// Tile schedule of the stencil kernels (H psi, pool scoring): which tile each
// workgroup processes.  Scheme 0 = contiguous runs of tiles per XCD (no
// table); others are host-built permutations (see build_tile_order).  The
// result of a kernel does not depend on the schedule (partials are indexed by
// tile).  *order receives a device table of ntiles entries or nullptr.
int stencil_order_table(int L, int d, int ntiles, const int **order);
// The same for an explicit scheme (tables are built once per device and kept).
int stencil_order_table_for(int L, int d, int ntiles, int scheme, const int **order);
int stencil_schedule();
// Work split of the H psi kernel (FOCK_STENCIL_*), and whether the lane
// split covers (L, d, ring bond).
int stencil_variant();
bool lanes_stencil_ok(int L, int d, int periodic_wrap);
bool slab_stencil_ok(int L, int d);
// Two-pass slab H psi (stencil2.hip): column pass writes the bonds among modes
// 4..7 into hpsi, row pass adds the rest in place; *nblocks pencils of
// (<psi|H psi>, <psi|psi>) partials.
int launch_apply_h2(const HamArgs &h, const float2 *psi, float2 *hpsi, double *partial, int *nblocks,
                    hipStream_t s);
// The same on real states (float32 amplitudes, open chains; H has real
// matrix elements): 4 bytes per amplitude in each pass.
bool apply_h2_real_supported(const HamArgs &h);
int launch_apply_h2_real(const HamArgs &h, const float *psi, float *hpsi, double *partial, int *nblocks,
                         hipStream_t s);
// Slab pool scoring (stencil2.hip): one FP64 partial per (workgroup, slot),
// pool_slab_blocks(h) workgroups, slot values already doubled.
int launch_pool_slab(const SlabPool &sp, const HamArgs &h, const float2 *psi, const float2 *hpsi, double *partial,
                     int *nblocks, hipStream_t s);
int pool_slab_blocks(const HamArgs &h);
// Pencil partials of launch_apply_h2 / launch_score_slab (2 doubles each).
int apply_h2_blocks(const HamArgs &h);
// Fused scoring (stencil2.hip): H psi into hpsi with (<psi|H psi>, <psi|psi>)
// partials per pencil in hpart (apply_h2 layout), and the pool partials of
// every slot in ppart (launch_pool_slab layout), from one column pass, one row
// pass that scores the row-shape entries as it completes H psi, and the
// column-shape pool pass.
int launch_score_slab(const SlabPool &sp, const HamArgs &h, const float2 *psi, float2 *hpsi, double *hpart,
                      double *ppart, hipStream_t s);

// Real states (gate_real.hip, d = 8): gates and reverse steps of the real
// generators HR and PR on float32 amplitudes (tables: the complex ones, real
// parts), in the full or the parity-halved geometry; the gate on (i, j) is
// available when real_gate_supported.  launch_real_convert widens n real
// amplitudes to complex64 (imaginary parts zero) or keeps the real parts;
// launch_imag_any raises *flag (atomic max of the bit pattern of |Im|) when
// any imaginary part of c is non-zero.
bool real_gate_supported(const Geometry &g, int i, int j);
int real_gate_blocks(const Geometry &g, int i, int j);
int launch_rgate(const Geometry &g, int i, int j, int kind, bool dag, const float2 *U, const float *src, float *psi,
                 hipStream_t s);
int launch_rgate_adj(const Geometry &g, int i, int j, int kind, const float2 *U, const float2 *A, float *phi,
                     float *lam, double *partial, hipStream_t s, bool write_phi);
int launch_real_convert(uint32_t n, bool to_complex, const void *src, void *dst, hipStream_t s);

// Fused runs of real gates (gate_real_fuse.hip): ng <= kRFuseMax gates whose
// pairs are tile modes (o, o+1) of modes a..a+2 (a + 2 <= real_fuse_top), in
// circuit order; reverse: their reverse steps in reverse order, gate k's tile
// partials into ops[k].part[0 .. real_fuse_blocks(g, true)).
constexpr int kRFuseMax = 8;
struct RFuseOp {
  int kind, o;
  const float2 *U, *A;
  double *part;
};
bool real_fuse_supported(const Geometry &g);
int real_fuse_top(const Geometry &g);
int real_fuse_blocks(const Geometry &g, bool reverse);
int launch_rfuse(const Geometry &g, int a, int ng, const RFuseOp *ops, const float *src, float *dst, hipStream_t s);
int launch_rfuse_adj(const Geometry &g, int a, int ng, const RFuseOp *ops, float *phi, float *lam, hipStream_t s);
int launch_imag_any(const float2 *c, uint32_t n, unsigned int *flag, hipStream_t s);

// Parity sectors (sector.hip, d = 8): partial (even, odd) sums of |Re| + |Im|
// of a full state, sector_norms_blocks(n) pairs; full <-> parity-halved conversion.
int sector_norms_blocks(uint32_t n);
int launch_sector_norms(const float2 *psi, uint32_t n, double *partial, hipStream_t s);
int launch_sector_convert(int L, int sector, bool to_half, const float2 *src, float2 *dst, hipStream_t s);

struct ProfScope {
  int id;
  hipStream_t s;
  double bytes;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(int id, hipStream_t s, double bytes);
  ~ProfScope();
};
void prof_harvest();

}  // namespace fock
