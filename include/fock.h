/*
 * fock.h - C ABI of libfock, the MI355X (gfx950) statevector engine for
 * CV-ADAPT-VQE on truncated-Fock bosonic chains.
 *
 * Problem statement followed (arXiv 2606.05297):
 *   - Fock basis and truncated ladder operators: Sec. II.A.
 *   - Gates O = exp(theta A), single-parameter form: Sec. II.B, Sec. IV.B.
 *   - Bose-Hubbard, bosonic Kitaev chain, Kitaev + Kerr Hamiltonians:
 *     Sec. III, Eqs. (BoseHubbard), (BosonicKitaevChain), (BosonicKitaevChain_Kerr).
 *   - Energy E = <psi|H|psi>, pool gradient g = <psi|[H,A]|psi>: Sec. IV.B, Eq. (grad).
 *   - ADAPT loop (score, select, append, re-optimise with BFGS): Sec. IV.B, Sec. V.A.
 *
 * Conventions shared by every entry point
 *   - State: complex64 (interleaved float re, im), d^L amplitudes, basis state
 *     |n_0 .. n_{L-1}> at flat index sum_r n_r d^r (mode 0 has stride 1).
 *     State pointers are DEVICE pointers, at least 16-byte aligned.
 *   - Limits: 2 <= d <= 16, 1 <= L <= 24, d^L <= 2^31.
 *   - Host scalars are double.  Reductions (energies, norms, gradients) are
 *     accumulated in double in a fixed order, so repeated calls on the same
 *     inputs return bit-identical results.
 *   - Ownership: the caller owns every buffer it passes (inputs, outputs,
 *     workspace) and the stream.  Entry points other than adapt_* never
 *     allocate device memory; the library keeps only small internal pinned
 *     staging buffers and per-(type, d) gate eigendata.
 *   - Streams: work is enqueued on `stream` (a hipStream_t; NULL means the
 *     null stream).  Calls that return host scalars synchronise that stream
 *     before returning.
 *   - Errors: every function returns FOCK_OK (0) or a negative FOCK_ERR_*
 *     code; arguments are validated before any device work is enqueued, and
 *     fock_last_error() describes the most recent failure on the calling
 *     thread.  No C++ exception crosses the ABI.
 */
#ifndef FOCK_H
#define FOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *fock_stream_t; /* hipStream_t */

enum {
  FOCK_OK = 0,
  FOCK_ERR_ARG = -1,         /* invalid argument (null pointer, bad mode, ...) */
  FOCK_ERR_SIZE = -2,        /* d^L too large or workspace too small */
  FOCK_ERR_UNSUPPORTED = -3, /* d or L outside the supported range */
  FOCK_ERR_NONFINITE = -4,   /* NaN/Inf angle or energy */
  FOCK_ERR_HIP = -5,         /* HIP runtime error */
  FOCK_ERR_LINESEARCH = -6,  /* BFGS line search failed (last good point kept) */
  FOCK_ERR_STATE = -7        /* call not valid in the object's current state */
};

/* Lattice Hamiltonian (Sec. III, build sign convention):
 *   H = sum_bonds [ -J (a_i^+ a_j + a_j^+ a_i) + Delta (a_i a_j + a_i^+ a_j^+) ]
 *     + sum_r [ (U/2 + K) n_r (n_r - 1) - mu n_r ]
 * Bonds: (r, r+1) for r = 0..L-2, plus (0, L-1) when periodic and L >= 3.
 * Bose-Hubbard: Delta = K = 0.  Kitaev + Kerr: U = 0.
 * layout: how the state buffers of the call hold psi.
 *   FOCK_LAYOUT_FULL (0): the d^L tensor, index sum_r n_r d^r.
 *   FOCK_LAYOUT_EVEN (1), FOCK_LAYOUT_ODD (2): a state of total parity
 *     sigma = 0 resp. 1 (sum_r n_r = sigma mod 2) in the parity-halved layout:
 *     the top mode stores m = 0..d/2-1 with n_{L-1} = 2 m + ((n_0 + .. + n_{L-2}
 *     + sigma) mod 2), at index sum_{r < L-1} n_r d^r + m d^(L-1), so a state
 *     holds d^L / 2 amplitudes (the other half of the tensor is zero).  H and
 *     every two-mode generator keep the total parity (Sec. II.B, III), so the
 *     sector is closed under them.  Open chains of L = 8, d = 8 under the slab
 *     stencil only; taken by fock_workspace_bytes, fock_apply_H, fock_pool_grads
 *     and fock_score (pools of HR..PI on nearest-neighbour pairs),
 *     fock_energy_grad_adjoint and fock_adjoint_sweep (HR..PI gates on pairs
 *     (i, j) with j < L-1, or (L-2, L-1)); FOCK_ERR_UNSUPPORTED elsewhere and
 *     for other ops.  Every other call takes layout 0 only.
 * FOCK_LAYOUT_REAL (4), added to any of the three: the state buffers hold
 *     float32 amplitudes (4 bytes each, same count and order).  H has real
 *     matrix elements (Sec. III) and HR, PR are real antisymmetric (Sec. II.B),
 *     so a real state stays real under H and their gates.  Open chains of
 *     L = 8, d = 8 under the slab stencil; taken by fock_workspace_bytes,
 *     fock_apply_H and fock_energy_grad_adjoint (HR and PR gates only; psi0,
 *     psi_work and lam_work are float32); FOCK_ERR_UNSUPPORTED elsewhere. */
enum { FOCK_LAYOUT_FULL = 0, FOCK_LAYOUT_EVEN = 1, FOCK_LAYOUT_ODD = 2, FOCK_LAYOUT_REAL = 4 };
typedef struct {
  int32_t L, d, periodic, layout;
  double J, U, mu, Delta, K;
} fock_ham_t;

/* Conversions between a full d^L state of one total parity and its
 * parity-halved layout (FOCK_LAYOUT_EVEN / _ODD, see fock_ham_t), d = 8,
 * 2 <= L <= 10.  pack: half[c] = full[index of c] for the d^L / 2 stored
 * amplitudes (the other parity part of full is not read); unpack writes every
 * amplitude of full (zero outside the sector).  Device buffers of d^L resp.
 * d^L / 2 complex64, 16-byte aligned, not overlapping; stream-ordered on
 * `stream`, no allocation.  FOCK_ERR_ARG / FOCK_ERR_UNSUPPORTED on bad
 * arguments. */
int fock_sector_pack(int L, int d, int layout, const void *full, void *half, fock_stream_t stream);
int fock_sector_unpack(int L, int d, int layout, const void *half, void *full, fock_stream_t stream);

/* Anti-Hermitian generators A (gate = exp(theta A)), Sec. II.B and Table I:
 *   FOCK_HR   a_i^+ a_j - a_j^+ a_i              (beam splitter, phi = pi)
 *   FOCK_HI   i (a_i^+ a_j + a_j^+ a_i)          (beam splitter, phi = pi/2)
 *   FOCK_DH   i (N_i a_i^+ a_j + a_j^+ a_i N_i)  (density-assisted hop)
 *   FOCK_PR   a_i a_j - a_i^+ a_j^+              (two-mode squeezer, phi = 0)
 *   FOCK_PI   i (a_i a_j + a_i^+ a_j^+)          (two-mode squeezer, phi = pi/2)
 *   FOCK_KERR i N_i^2   (single mode, j = -1)    (Kerr gate)
 *   FOCK_ROT  i N_i     (single mode, j = -1)    (phase rotation)
 *   FOCK_CK   i N_i N_j                          (cross-Kerr gate)
 *   FOCK_SR   (a_i^2 - a_i^+2) / 2   (single mode, j = -1)  (squeezer, phi = 0)
 *   FOCK_SI   i (a_i^2 + a_i^+2) / 2 (single mode, j = -1)  (squeezer, phi = -pi/2)
 * Two-mode ops need 0 <= i < j < L.  The batched sweep (fock_sweep_*) and
 * fused gate runs do not take SR / SI (FOCK_ERR_UNSUPPORTED, resp. the
 * per-gate kernels run). */
enum {
  FOCK_HR = 0, FOCK_HI = 1, FOCK_DH = 2, FOCK_PR = 3, FOCK_PI = 4, FOCK_KERR = 5, FOCK_ROT = 6, FOCK_CK = 7,
  FOCK_SR = 8, FOCK_SI = 9
};
/* Two-parameter gates exp(theta A(phi)) of Sec. II.B, pool entries of the
 * complex128 driver (adapt64_*) only:
 *   FOCK_BS   beam splitter, A = e^{i phi} a_i a_j^+ - e^{-i phi} a_i^+ a_j
 *   FOCK_TMS  two-mode squeezer, A = e^{i phi} a_i a_j - e^{-i phi} a_i^+ a_j^+
 *   FOCK_SQ   single-mode squeezer (j = -1), A = (e^{-i phi} a_i^2 - e^{i phi} a_i^+2) / 2
 * Each is R(c phi) exp(theta A(0)) R(-c phi) with phase rotations R on mode j
 * (BS: c = 1, TMS: c = -1) or i (SQ: c = 1/2), and is expanded to those three
 * gates (adapt64_get_ansatz returns the expanded circuit). */
enum { FOCK_BS = 10, FOCK_TMS = 11, FOCK_SQ = 12 };

typedef struct {
  int32_t type, i, j;
} fock_op_t;

/* Message for the last failure on this thread ("" if none). */
const char *fock_last_error(void);

/* ABI version (incremented on incompatible changes). */
int fock_version(void);

/* Workspace bytes large enough for every low-level call below on this
 * Hamiltonian's state size with a pool of n_pool ops and circuits of up to
 * n_ops gates.  Returns FOCK_ERR_UNSUPPORTED / FOCK_ERR_SIZE for bad sizes. */
int fock_workspace_bytes(const fock_ham_t *ham, int n_pool, int n_ops, size_t *bytes);

/* hpsi = H psi (Sec. III).  If E / norm2 are non-NULL they receive
 * <psi|H|psi> and <psi|psi> (double; the stream is synchronised).
 * psi and hpsi: device, d^L complex64 each, must not overlap.
 * ws: device workspace of ws_bytes (see fock_workspace_bytes). */
int fock_apply_H(const fock_ham_t *ham, const void *psi, void *hpsi, double *E, double *norm2,
                 void *ws, size_t ws_bytes, fock_stream_t stream);

/* psi <- exp(theta A_op) psi in place (or its adjoint exp(-theta A_op) when
 * adjoint != 0), Sec. II.B.  The gate is exp of the truncated generator, hence
 * exactly unitary; its conserved blocks (n_i + n_j for HR/HI/DH/CK, n_i - n_j
 * for PR/PI, single levels for KERR/ROT, the parity of n_i for SR/SI) keep
 * boson number or parity leakage at 0. */
int fock_apply_gate2(int L, int d, fock_op_t op, double theta, int adjoint, void *psi,
                     void *ws, size_t ws_bytes, fock_stream_t stream);

/* Pool scoring, Eq. (grad): grads[k] = 2 Re <hpsi| A_k psi> = <psi|[H, A_k]|psi>
 * for k < P, where hpsi = H psi (from fock_apply_H).  grads: host array of P
 * doubles (stream synchronised).  P <= 4096. */
int fock_pool_grads(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi,
                    const void *hpsi, double *grads, void *ws, size_t ws_bytes, fock_stream_t stream);

/* Pool scoring with H psi in one call (Eq. (grad) on the Hamiltonian of
 * Sec. III): hpsi = H psi, E = <psi|H|psi>, norm2 = <psi|psi> (both nullable)
 * and grads[k] = 2 Re <H psi| A_k psi> for k < P (host, P doubles), the stream
 * synchronised once.  Where L = 8, d = 8 (the slab stencil variant) and every
 * entry is a two-mode generator on a nearest-neighbour pair (or the ring pair
 * (0, 7) of a ring) or a diagonal generator (at most 16), with no duplicates
 * and P <= 256, the scoring is fused: the row pass that completes H psi also
 * scores the entries of modes 0..4 against it from the same LDS slices, and
 * one column-shape pass scores the rest; otherwise fock_apply_H then
 * fock_pool_grads run.  Same results as those two calls to FP32 rounding. */
int fock_score(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi, void *hpsi, double *E,
               double *norm2, double *grads, void *ws, size_t ws_bytes, fock_stream_t stream);

/* Energy of the ansatz psi = O_n(theta_n) ... O_1(theta_1) psi0 (newest gate
 * acts last, Sec. IV.B) and, when dEdtheta is non-NULL, all dE/dtheta_k by one
 * reverse sweep: dE/dtheta_k = 2 Re <lambda_k| A_k phi_k> / <psi|psi> with
 * phi_k = O_k..O_1 psi0 and lambda_k = O_{k+1}^+ .. O_n^+ H psi.
 * E receives the Rayleigh quotient <psi|H|psi>/<psi|psi>; norm2 (nullable)
 * receives <psi|psi>.  psi0: device input (unchanged).  psi_work, lam_work:
 * device d^L complex64 scratch; on return without gradient they hold psi and
 * H psi.  ops/theta: host arrays of n entries (n <= 4096). */
int fock_energy_grad_adjoint(const fock_ham_t *ham, const fock_op_t *ops, const double *theta, int n,
                             const void *psi0, void *psi_work, void *lam_work, double *E,
                             double *norm2, double *dEdtheta, void *ws, size_t ws_bytes,
                             fock_stream_t stream);

/* The reverse sweep of fock_energy_grad_adjoint on its own (the adjoint
 * gradient identity of Sec. IV.B applied to every parameter): given
 * psi_work = psi_n and lam_work = H psi_n as left by an energy-only call
 * (dEdtheta == NULL) of the same ops/theta, and that call's norm2, writes all
 * dE/dtheta_k = 2 Re <lambda_k| A_k phi_k> / norm2 into dEdtheta (host, n).
 * psi_work and lam_work are overwritten (they end as psi0 and
 * O_1^+..O_n^+ H psi_n up to rounding).  Lets a caller run the forward pass
 * and the gradient pass separately (e.g. an autograd backward).  Same
 * workspace as fock_energy_grad_adjoint for n gates. */
int fock_adjoint_sweep(const fock_ham_t *ham, const fock_op_t *ops, const double *theta, int n, void *psi_work,
                       void *lam_work, double norm2, double *dEdtheta, void *ws, size_t ws_bytes,
                       fock_stream_t stream);

/* Build ahead of time, on the current device, what the calls on (L, d) would
 * otherwise create on their first use: the gate eigendata of cutoff d (device
 * memory and a synchronous upload, Sec. II.B), the tile-order tables of the
 * stencil schedules 1-3 for open and ring chains, and this thread's pinned
 * staging buffers at their base size (64 kB each) with its pinned results
 * buffer for real-state gradient evaluations (32 kB).  Afterwards fock_apply_H,
 * fock_apply_gate2 and fock_energy_grad_adjoint on (L, d) from this thread
 * allocate nothing and add no synchronisation of their own beyond their
 * documented result fetch, for circuits of up to ~2,700 gates.  (Pool scoring
 * outside the slab kernels stages its pair tables through the pinned buffer,
 * which grows on its first such call.)  Idempotent; FOCK_ERR_UNSUPPORTED /
 * FOCK_ERR_SIZE as fock_workspace_bytes; the tables are kept until the process
 * ends. */
int fock_prepare(int L, int d);

/* fock_apply_H without any allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): hpsi = H psi as fock_apply_H, with the per-workgroup energy and
 * norm partials in a fixed 1 MiB device array owned by the library (one per
 * GPU, kept until the process ends) instead of a caller workspace, and the
 * reduced pair written to DEVICE memory: res_dev[0] = <psi|H|psi>,
 * res_dev[1] = <psi|psi> (double; res_dev nullable, 8-byte aligned).  No host
 * synchronisation and no pinned staging; the work is only enqueued on stream.
 * Same kernels and reduction order as fock_apply_H (bit-identical results).
 * Limit: at most 65,536 workgroup partials (every L=8 lattice with d <= 8 and
 * any d^L <= 2^28 fits); larger lattices return FOCK_ERR_SIZE.  Calls that
 * overlap on one GPU (concurrent streams or threads) share the array and race;
 * serialise them.  Tile schedules 1-3 (fock_set_stencil_schedule) are taken
 * as schedule 0 here, since their order tables are allocated on first use. */
int fock_apply_H_noalloc(const fock_ham_t *ham, const void *psi, void *hpsi, double *res_dev, fock_stream_t stream);

/* ------------------------------------------------------------------ ADAPT */

typedef struct {
  int32_t max_iters;      /* iteration cap (ADAPT steps) */
  int32_t bfgs_maxiter;   /* BFGS iteration cap per step (1000 in Sec. V.A) */
  double grad_tol;        /* stop when ||g||_2 over the pool < grad_tol */
  double tie_tau;         /* candidates |g_k| >= (1 - tie_tau) max|g|; lowest index wins */
  double gtol_floor_rel;  /* BFGS L-inf tolerance max(min(1e-6, 1e-5|g_sel|), floor*max(1,|E|)) */
  double warm_gtol;       /* BFGS tolerance for the warm-up layer alone */
  int32_t n_warm;         /* warm-up layer length (0 = none) */
  int32_t grad_mode;      /* 0 = adjoint sweep, 1 = central finite differences (plain) */
  const fock_op_t *warm_ops;    /* host, n_warm entries, copied at create */
  const double *warm_theta0;    /* host, n_warm initial angles, copied at create */
  double fd_step;         /* finite-difference step for grad_mode 1 */
  int32_t recycle_hessian;/* 1: seed each BFGS with the previous inverse Hessian (Appendix D) */
  int32_t warm_fixed;     /* 1: the warm-up angles stay at warm_theta0 (never optimised; Appendix D's
                             fixed warm-up); complex128 driver only, 0 elsewhere */
  double noise_rel;       /* BFGS also stops once the predicted decrease < noise_rel*max(1,|E|) (FP32 noise),
                             from its second iteration on */
} fock_adapt_opts_t;

typedef struct {
  int32_t iter;        /* ADAPT step index (0 = warm-up layer) */
  int32_t k_sel;       /* selected pool index, -1 if none */
  int32_t converged;   /* 1 when ||g||_2 < grad_tol (no op appended) */
  int32_t status;      /* FOCK_OK or FOCK_ERR_LINESEARCH */
  int32_t bfgs_iters, bfgs_evals, n_params, capped;
  double g_sel;        /* |g_k*| at selection */
  double g_norm2, g_inf;
  double E;            /* energy after re-optimisation (Rayleigh quotient) */
  double norm2;        /* <psi|psi> at that point */
  double E_init;       /* energy at the start of BFGS */
} fock_adapt_report_t;

typedef struct fock_adapt fock_adapt_t;

/* Default options: max_iters 60, bfgs_maxiter 1000, grad_tol 1e-3,
 * tie_tau 1e-4, gtol_floor_rel 1e-5, warm_gtol 1e-6, fd_step 1e-3, noise_rel 1e-7. */
void adapt_default_opts(fock_adapt_opts_t *opts);

/* Create an ADAPT run on `ham` (layout 0) with `pool` (P ops, host, copied)
 * from the device state psi0 (d^L complex64, copied).  The object owns its
 * device buffers (three states, in the layout adapt_layout reports, plus
 * workspace) and uses `stream`.  With a warm-up layer, its angles are
 * BFGS-optimised here (report via adapt_warm_report). */
int adapt_create(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi0,
                 const fock_adapt_opts_t *opts, fock_stream_t stream, fock_adapt_t **out);

/* One ADAPT iteration (Sec. IV.B): score the pool on the current state,
 * test convergence, select (tie band, lowest index), append exp(theta A_k)
 * with theta = 0 (or the pending proposal, see adapt_propose), re-optimise all
 * angles by BFGS.  Returns FOCK_ERR_STATE once the run has converged/capped. */
int adapt_step(fock_adapt_t *st, fock_adapt_report_t *rep);

/* adapt_step in two halves, so that a caller can propose starting angles for
 * the circuit the step has actually chosen (Sec. IV.B: the initial point of
 * each re-optimisation is {theta_prev, 0}).  adapt_step_select scores the
 * pool, tests convergence and, unless converged or capped, selects and appends
 * exp(theta A_k) with theta = 0 (rep: iter, k_sel, g_sel, g_norm2, g_inf, E,
 * norm2, n_params including the new angle).  adapt_step_finish then starts
 * BFGS from {theta_prev, 0} or from a pending proposal whose energy is not
 * higher, and fills the whole report as adapt_step.  FOCK_ERR_STATE for a
 * select while a step is pending and for a finish without one. */
int adapt_step_select(fock_adapt_t *st, fock_adapt_report_t *rep);
int adapt_step_finish(fock_adapt_t *st, fock_adapt_report_t *rep);

/* Report of the warm-up optimisation done in adapt_create. */
int adapt_warm_report(fock_adapt_t *st, fock_adapt_report_t *rep);

/* Current ansatz: ops and angles (warm-up layer first).  cap = array size;
 * *n receives the full length. */
int adapt_get_ansatz(fock_adapt_t *st, fock_op_t *ops, double *theta, int cap, int *n);

/* Proposal for the angles used as the BFGS start of the next step: the full
 * vector of length n_params + 1 before adapt_step / adapt_step_select, or of
 * length n_params (the new angle already appended) between adapt_step_select
 * and adapt_step_finish.  It is used only if its energy is not above the
 * plain start {theta_prev, 0}; otherwise the plain start is kept.  *accepted
 * (after the step) via adapt_last_proposal. */
int adapt_propose(fock_adapt_t *st, const double *theta, int n);
int adapt_last_proposal(fock_adapt_t *st, int *accepted, double *E_prop, double *E_plain);

/* Number of forward states the run keeps for its gradient evaluations (0: none;
 * see fock_set_state_store). */
int adapt_state_store(fock_adapt_t *st, int *nstates);

/* Whether the run keeps float32 copies of its states (*real = 1): with the
 * switch on (fock_set_real_states), d = 8 and psi0 with every imaginary part
 * exactly zero.  An evaluation whose gates are all HR or PR then runs its
 * gates and reverse steps on real amplitudes (4 bytes each): H (Sec. III) is
 * real and these generators are real antisymmetric (Sec. II.B), so psi,
 * H psi and the reverse sweep's states stay real; H psi and the pool scoring
 * run on a complex64 copy.  Evaluations with any other gate run in complex64.
 * Energies, gradients and selections agree with the complex path to FP32
 * rounding (the gate tables' imaginary parts are rounding noise). */
int adapt_real(fock_adapt_t *st, int *real);

/* Layout the run keeps its states in (FOCK_LAYOUT_*): with the sector switch
 * on (fock_set_sector_layout), adapt_create picks FOCK_LAYOUT_EVEN / _ODD when
 * psi0 has exactly zero amplitude outside one total-parity sector, the chain
 * is an open L = 8, d = 8 chain under the slab stencil, the pool holds only
 * HR..PI generators on nearest-neighbour pairs (each at most once) and the
 * warm-up layer only HR..PI gates on pairs (i, j) with j < L-1 or (L-2, L-1);
 * otherwise FOCK_LAYOUT_FULL.  Both layouts give the same energies, gradients
 * and selections to FP32 rounding. */
int adapt_layout(fock_adapt_t *st, int *layout);

int adapt_destroy(fock_adapt_t *st);

/* ------------------------------------------------------------------ HVA-CV-VQE */

/* The paper's fixed-structure baseline (Sec. IV.A, Eq. (HVA_ansatz)): the
 * ansatz repeats one layer of gates exp(theta A_k), the generators being the
 * Hamiltonian's own terms (hopping HI, pairing PI, Kerr, rotation; layer ops
 * given by the caller, host, copied), and grows one layer at a time (Sec. V.A):
 * hva_add_layer appends a layer whose angles start at theta_new (host, layer
 * size; the paper draws them uniformly in [-0.05, 0.05]), keeps the earlier
 * angles at their previous optimum and BFGS-re-optimises all of them (opts:
 * bfgs_maxiter, gtol_floor_rel, noise_rel as for adapt_create; L-infinity
 * tolerance max(gtol, gtol_floor_rel max(1, |E|)), the paper's gtol being
 * 1e-9).  The report carries the layer count (iter), E, BFGS iterations and
 * evaluations, the parameter count and the final ||g||_inf.  Same evaluation
 * pipeline as adapt_step.  psi0: device complex64 (copied once `stream` is
 * synchronised); the handle owns its buffers.  max_layers * layer size <= 4096. */
typedef struct fock_hva fock_hva_t;
int hva_create(const fock_ham_t *ham, const fock_op_t *layer, int n_layer, int max_layers, const void *psi0,
               const fock_adapt_opts_t *opts, double gtol, fock_stream_t stream, fock_hva_t **out);
int hva_add_layer(fock_hva_t *st, const double *theta_new, fock_adapt_report_t *rep);
/* Energy of psi0 (no layer). */
int hva_initial_report(fock_hva_t *st, fock_adapt_report_t *rep);
/* Current ansatz (all layers' gates and angles), as adapt_get_ansatz. */
int hva_get_ansatz(fock_hva_t *st, fock_op_t *ops, double *theta, int cap, int *n);
int hva_destroy(fock_hva_t *st);

/* ------------------------------------------------------------------ batched sweep */

/* One point of a parameter sweep: its Hamiltonian, pool (P <= 256 ops, host,
 * copied), optional warm-up layer and initial state (device, copied). */
typedef struct {
  fock_ham_t ham;
  const fock_op_t *pool;
  int32_t P;
  int32_t n_warm;
  const fock_op_t *warm_ops;
  const double *warm_theta0;
  const void *psi0;
} fock_sweep_point_t;

typedef struct fock_sweep fock_sweep_t;

/* CV-ADAPT-VQE (Sec. IV.B) on npts points of uneven (L, d), d in {4, 6, 8},
 * run in lockstep: every phase of all points is one batched launch per d,
 * and each energy + adjoint-gradient round of the BFGS re-optimisations is a
 * replay of one captured HIP graph.  Results per point are identical to
 * adapt_step on that point alone (same kernels, same reduction order).
 * opts: iteration caps, tolerances and BFGS settings shared by all points
 * (its warm-up fields are ignored; each point brings its own).  The sweep owns
 * its device buffers and a private stream; `stream` is synchronised once at
 * creation (psi0 buffers must be ready on it). */
int fock_sweep_create(const fock_sweep_point_t *pts, int npts, const fock_adapt_opts_t *opts,
                      fock_stream_t stream, fock_sweep_t **out);
/* One ADAPT iteration on every unfinished point; reps: host array of npts
 * reports (unfinished points only are updated).  *n_active (nullable)
 * receives the number of points that took part.  FOCK_ERR_STATE when every
 * point has finished. */
int fock_sweep_step(fock_sweep_t *sw, fock_adapt_report_t *reps, int *n_active);
/* Reports of the warm-up optimisations done at creation (npts entries). */
int fock_sweep_warm_reports(fock_sweep_t *sw, fock_adapt_report_t *reps);
/* Ansatz of one point (warm-up layer first); see adapt_get_ansatz. */
int fock_sweep_get_ansatz(fock_sweep_t *sw, int point, fock_op_t *ops, double *theta, int cap, int *n);
/* Warm-start proposal for point's next step (n = its current parameter
 * count + 1), as adapt_propose: used only when its energy is not above the
 * plain start.  Outcome of the last step's proposal: fock_sweep_last_proposal. */
int fock_sweep_propose(fock_sweep_t *sw, int point, const double *theta, int n);
int fock_sweep_last_proposal(fock_sweep_t *sw, int point, int *accepted, double *E_prop, double *E_plain);
/* Workgroups of the persistent batched launches (autotuner knob). */
int fock_sweep_set_grid(fock_sweep_t *sw, int grid);
/* Choose that grid by timing one forward + H psi round of the unfinished
 * points for 256..4096 workgroups (HIP events).  cache_path (nullable): JSON
 * lines keyed by architecture and sweep size, read first, appended after
 * tuning.  *best_grid (nullable) receives the choice. */
int fock_sweep_autotune(fock_sweep_t *sw, const char *cache_path, int *best_grid);
int fock_sweep_destroy(fock_sweep_t *sw);

/* ------------------------------------------------------------------ BFGS */

/* Objective for fock_bfgs_minimize: f(x) and its gradient g (both host);
 * return 0, or a negative code to abort the minimisation. */
typedef int (*fock_objective_fn)(void *ctx, int n, const double *x, double *f, double *g);

/* BFGS with a strong-Wolfe line search (the minimiser used by adapt_step,
 * Sec. V.A): stops when ||g||_inf < gtol or after maxiter iterations.  x
 * (host, n) is the start on entry and the result on return.  Hinv (nullable,
 * host n x n row-major) seeds the inverse Hessian when non-zero and receives
 * the final one.  *status = FOCK_OK or FOCK_ERR_LINESEARCH (last accepted point
 * kept). */
int fock_bfgs_minimize(int n, double *x, fock_objective_fn fn, void *ctx, double gtol, int maxiter, double *Hinv,
                       int *iters, int *evals, double *fmin, int *status);

/* ------------------------------------------------------------------ dense gate variant */

/* Forward two-mode gates (fock_apply_gate2 and the forward circuit of the
 * adjoint evaluation) as a dense d^2 x d^2 contraction on FP32 matrix cores
 * (v_mfma_f32_16x16x4_f32): each fibre's 2d^2 real components times the real
 * form of U, ignoring its conserved-block structure (Sec. II.B).  d in
 * {4, 6, 8}; other cutoffs and single-mode gates keep the block kernels.
 * Same results to FP32 rounding.  Process-wide; FOCK_GATE_BLOCK by default. */
enum { FOCK_GATE_BLOCK = 0, FOCK_GATE_DENSE_MFMA = 1 };
int fock_set_gate_variant(int variant);
int fock_get_gate_variant(void);

/* ------------------------------------------------------------------ gate fusion */

/* Circuits evaluated by fock_energy_grad_adjoint and adapt_step run runs of
 * consecutive gates whose modes (with mode 0) fit one tile of d^s <= 4096
 * amplitudes as one pass: the tile is staged in LDS and the gates are applied
 * there one after another (forward), or the tiles of phi and lambda are staged
 * and the reverse steps of the run are taken there (adjoint sweep).  Same
 * operations as the per-gate kernels (same block arithmetic); gradient partials
 * are summed over other tiles, so results agree to FP32/FP64 rounding, not
 * bitwise.  d in {2, 4, 6, 8}; process-wide mode: FOCK_FUSE_OFF (the
 * default), FOCK_FUSE_FORWARD (forward circuit only) or FOCK_FUSE_ALL (forward
 * and adjoint sweep).  The batched sweep does not fuse. */
enum { FOCK_FUSE_OFF = 0, FOCK_FUSE_FORWARD = 1, FOCK_FUSE_ALL = 2 };
int fock_set_gate_fusion(int mode);
int fock_get_gate_fusion(void);

/* ------------------------------------------------------------------ stencil schedules */

/* Order in which the workgroups of fock_apply_H and fock_pool_grads visit the
 * LDS tiles (d^K consecutive rows; tile t has base-d digits c_0..c_{m-1}, the
 * occupations of the modes above the tile).  Workgroup b runs on XCD b % 8.
 *   0: each XCD takes a contiguous run of tiles, natural order (default);
 *   1: contiguous runs, the highest free digit fastest;
 *   2: each XCD takes an octant of the three top digits, natural order;
 *   3: octants, the three top digits fastest;
 *   4: two passes for fock_apply_H: the first stages the rows of the top m
 *      modes (d^m <= 512 rows) in LDS and applies the bonds among them and the
 *      ring bond, writing H psi; the second runs the contiguous tiles of
 *      scheme 0 for the remaining bonds and the diagonal and adds in place.
 *      Fewer neighbour rows cross XCDs at the price of one more state
 *      read + write.  Pool scoring runs as scheme 0.
 * Schemes 0-3 give bit-identical results (partials are indexed by tile);
 * scheme 4 sums the bond terms of a row in another order (FP32 rounding
 * level).  Process-wide; schemes 1-3 that do not divide the tiles over the 8
 * XCDs evenly run as scheme 0. */
enum { FOCK_SCHED_TWO_PASS = 4, FOCK_SCHED_NUM = 5 };
int fock_set_stencil_schedule(int scheme);
int fock_get_stencil_schedule(void);
/* Host-side copy of scheme's permutation for n tiles (order[b] = tile of
 * workgroup b); the identity-per-XCD map for scheme 0 or a fallback. */
int fock_stencil_schedule_table(int L, int d, int scheme, int *order, int n);
/* Autotuner: times fock_apply_H on (psi -> hpsi) under every schedule (HIP
 * events on stream, median of 5 after a warm-up), selects the fastest and
 * returns it in *best_scheme (nullable).  cache_path (nullable): JSON lines
 * keyed by architecture and (L, d, boundary, model), read first, appended after
 * tuning.  hpsi is overwritten. */
int fock_autotune_stencil(const fock_ham_t *ham, const void *psi, void *hpsi, void *ws, size_t ws_bytes,
                          fock_stream_t stream, const char *cache_path, int *best_scheme);

/* Work split of the H psi kernel (same operator, Sec. III):
 *   FOCK_STENCIL_ROWS  - one thread per row of d amplitudes (every d, L, boundary);
 *   FOCK_STENCIL_LANES - four lanes per row, two amplitudes each, with the bonds
 *      beyond the LDS tile read as 1 kB blocks at wavefront-uniform offsets.
 *      Used where d = 8, 4 <= L <= 10, the chain is open and the schedule is
 *      single-pass; elsewhere the row split runs.
 *   FOCK_STENCIL_SLAB  - (the default) two LDS-resident passes for L = 8, d = 8,
 *      open or ring: a column pass applies the bonds among modes 4..7 (and the
 *      ring bond) streaming mode 7 over 128-byte segments of the low modes and
 *      writes them to hpsi; a row pass applies the bonds among modes 0..4
 *      streaming mode 4 over contiguous 32 kB slices and adds them in place.
 *      Every neighbour comes from LDS or registers; 40 B/amplitude of traffic
 *      in long contiguous runs.  Elsewhere (and with schedule 4) the row split runs.
 * The variants sum an amplitude's terms in different orders (FP32 rounding
 * level).  Takes effect for handles (ADAPT runs, sweeps) created after the
 * call and for the direct fock_apply_H calls; process-wide. */
enum { FOCK_STENCIL_ROWS = 0, FOCK_STENCIL_LANES = 1, FOCK_STENCIL_SLAB = 2 };
int fock_set_stencil_variant(int variant);
int fock_get_stencil_variant(void);

/* Forward-state store of the ADAPT and HVA drivers (Sec. IV.B's gradients by
 * one reverse sweep).  With a store, a gradient evaluation writes
 * phi_k = O_k phi_{k-1} into slot k - 1 of a buffer holding one state per gate
 * slot (instead of updating phi in place), and the reverse sweep reads phi_k
 * from the store.  Each reverse step then reads phi_k and updates lam (24 B per
 * amplitude, against 32 B for undoing the gate on phi as well), while the
 * forward gates write each state to fresh memory.
 *   FOCK_STORE_OFF  (0) never keep states;
 *   FOCK_STORE_ON   (1) keep them whenever the store fits;
 *   FOCK_STORE_AUTO (2, the default) keep them when one state exceeds the
 *                   256 MiB Infinity Cache.  Smaller states are rewritten in
 *                   place inside the cache, which is as fast (measured at
 *                   L = 8, d = 8: 134 MB states, equal step rates; at L = 9,
 *                   1.07 GB states, the store gives 10 % more steps/s).
 * A store is allocated only when it takes at most half of the free device
 * memory (d^L * 8 B per slot).  Circuits with squeezer gates or fused gate
 * runs, and the caller-buffer calls (fock_energy_grad_adjoint,
 * fock_adjoint_sweep), always use the in-place sweep.  The two orders give the
 * same gradients to FP32 rounding.  Applies to drivers created after the
 * call; FOCK_ERR_ARG for other values; process-wide. */
enum { FOCK_STORE_OFF = 0, FOCK_STORE_ON = 1, FOCK_STORE_AUTO = 2 };
int fock_set_state_store(int mode);
int fock_get_state_store(void);

/* Parity-halved states in the ADAPT driver (see adapt_layout):
 *   FOCK_SECTOR_OFF  (0) always the full d^L layout;
 *   FOCK_SECTOR_AUTO (1) the parity-halved layout where adapt_layout says
 *                    (default): half the state bytes of every kernel.
 * Applies to drivers created after the call; FOCK_ERR_ARG for other values;
 * process-wide. */
enum { FOCK_SECTOR_OFF = 0, FOCK_SECTOR_AUTO = 1 };
int fock_set_sector_layout(int mode);
int fock_get_sector_layout(void);

/* Real states in the ADAPT driver (see adapt_real): FOCK_REAL_OFF (0) never,
 * FOCK_REAL_AUTO (1) where adapt_real says (default).  Applies to drivers
 * created after the call; FOCK_ERR_ARG for other values; process-wide. */
enum { FOCK_REAL_OFF = 0, FOCK_REAL_AUTO = 1 };
int fock_set_real_states(int mode);
int fock_get_real_states(void);

/* Fused runs of real gates.  An evaluation on real states (see adapt_real and
 * FOCK_LAYOUT_REAL) at d = 8 with >= 2^21 stored amplitudes takes each run of
 * >= 2 consecutive HR / PR gates whose pairs lie inside three consecutive modes
 * (a, a+1, a+2; below the top mode in the parity-halved layout) as one pass:
 * tiles of 32 (forward) or 16 (reverse) sets of the 512 amplitudes over those
 * modes are staged in LDS, and the run's gates (Sec. II.B), or its reverse steps
 * with their gradient terms (Sec. IV.B), are applied there in order.  States
 * are the same bit for bit as gate by gate; gradient partials are summed per
 * tile, so gradients agree to FP32/FP64 rounding.  At most 8 gates per run.
 * Process-wide: FOCK_RFUSE_ON (default) or FOCK_RFUSE_OFF (gate by gate). */
enum { FOCK_RFUSE_OFF = 0, FOCK_RFUSE_ON = 1 };
int fock_set_real_fusion(int mode);
int fock_get_real_fusion(void);

/* The runs that an evaluation of ops[0..n) on real states would launch under
 * the current fusion mode (host only: no device work).  run_k0[r] is the first
 * gate of run r (runs are consecutive and cover the circuit in order), run_a[r]
 * the lowest of its three tile modes, or -1 for a gate taken by the per-gate
 * kernels; *nruns receives the count.  ham->layout selects the geometry (full
 * or parity-halved; FOCK_LAYOUT_REAL optional).  run_k0 and run_a hold n
 * entries (caller owned).  Errors: FOCK_ERR_ARG (layout, pairs, NULL arrays),
 * FOCK_ERR_UNSUPPORTED (a gate other than HR or PR). */
int fock_real_fusion_plan(const fock_ham_t *ham, const fock_op_t *ops, int n, int *run_k0, int *run_a, int *nruns);

/* ------------------------------------------------------------------ FP64 states */

/* CV-ADAPT-VQE (Sec. IV.B) on complex128 states, for runs that resolve energy
 * differences far below the complex64 state's ~1e-7 relative rounding (the
 * paper runs to |E - E0| ~ 1e-10, Sec. V).  Same loop as adapt_step: pool
 * scoring, tie band, append at theta = 0, BFGS with the L-inf tolerance and
 * optional Hessian recycling (no noise-floor stop).  Plain kernels (one thread
 * per amplitude for H psi; one workgroup per group of fibres with a dense
 * local gate matrix of d^2 x d^2 or d x d), meant for lattices of up to ~1e6
 * amplitudes.  psi0: device, d^L complex128 (copied); opts: as adapt_create
 * (a warm-up layer of one-parameter ops leads the ansatz, is BFGS-optimised
 * here with tolerance max(warm_gtol, gtol_floor_rel max(1,|E|)) and re-optimised
 * with every step, Appendix C; with warm_fixed its angles stay at warm_theta0
 * and BFGS runs over the other angles only, Appendix D), except that finite-difference gradients are
 * refused (FOCK_ERR_UNSUPPORTED); gtol_floor_rel is taken as given, and its default
 * (1e-5, the complex64 resolution) stops BFGS once ||g||_inf < 1e-5 |E|, which
 * caps the energy error near 1e-6 |E|: complex128 runs pass ~1e-11.  The handle owns its buffers and a private stream;
 * `stream` is synchronised once at creation. */
typedef struct fock_adapt64 fock_adapt64_t;
int adapt64_create(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi0,
                   const fock_adapt_opts_t *opts, fock_stream_t stream, fock_adapt64_t **out);
/* One ADAPT iteration; FOCK_ERR_STATE once converged or capped. */
int adapt64_step(fock_adapt64_t *st, fock_adapt_report_t *rep);
/* Report of the warm-up optimisation done in adapt64_create (iter 0; without
 * a warm-up layer: the energy of psi0, no BFGS iterations). */
int adapt64_warm_report(fock_adapt64_t *st, fock_adapt_report_t *rep);
/* Current ansatz as gates and gate angles (see adapt_get_ansatz); a
 * two-parameter op appears as its three gates.  The report's n_params counts
 * the logical parameters (two per two-parameter op). */
int adapt64_get_ansatz(fock_adapt64_t *st, fock_op_t *ops, double *theta, int cap, int *n);
/* E (Rayleigh quotient) and, if dEdtheta is non-NULL, all dE/dtheta_k of the
 * ansatz ops/theta (ops no wider than the pool's) on the
 * handle's psi0, by the FP64 forward pass and reverse sweep.  ops are gates
 * (no two-parameter types), n <= n_warm + 3 (max_iters + 1). */
int adapt64_energy_grad(fock_adapt64_t *st, const fock_op_t *ops, const double *theta, int n, double *E,
                        double *dEdtheta);
int adapt64_destroy(fock_adapt64_t *st);

/* ------------------------------------------------------------------ warm-start network */

/* A small network proposes the initial angles of an ADAPT step from the
 * point's features (J, Delta, K, n / 64): an addition on top of the plain
 * {theta_prev, 0} initialisation of Sec. IV.B (the paper notes that initial
 * parameters matter, Sec. V.B, and re-uses optimiser information across steps,
 * Appendix D).  Architecture 4 -> 128 -> 128 -> 64, SiLU hidden activations,
 * linear output; bf16 inputs, weights and hidden activations (round to nearest
 * even), FP32 biases, FP32 MFMA accumulation, FP32 output.  Loss: masked mean
 * squared error over the first nvalid[b] outputs of row b.  Training: Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master parameters; the backward
 * pass rounds its error signals to bf16 before the products.  Parameter vector
 * (FP32, this order): W1 [128 x 4], b1 [128], W2 [128 x 128], b2 [128],
 * W3 [64 x 128], b3 [64]; W is [out x in] row-major.
 * X [B x 4], T [B x 64], Y [B x 64] (FP32, row-major) and nvalid [B] (int32) are
 * DEVICE pointers; parameters and gradients cross as host arrays.  All calls
 * are ordered on `stream`; those returning host values synchronise it.  The
 * object owns its device buffers (about 101.6 kB x ceil(max_batch / 64)). */
typedef struct fock_mlp fock_mlp_t;
enum { FOCK_MLP_IN = 4, FOCK_MLP_HIDDEN = 128, FOCK_MLP_OUT = 64, FOCK_MLP_NPARAMS = 25408 };

int fock_mlp_create(int max_batch, fock_mlp_t **out);
/* Load FP32 master parameters (host, FOCK_MLP_NPARAMS); resets Adam state. */
int fock_mlp_set_params(fock_mlp_t *net, const float *params, int n, fock_stream_t stream);
int fock_mlp_get_params(fock_mlp_t *net, float *params, int n, fock_stream_t stream);
/* Y = net(X) for B <= max_batch rows. */
int fock_mlp_forward(fock_mlp_t *net, const float *X, int B, float *Y, fock_stream_t stream);
/* Masked-MSE loss (nullable) and its gradient (host, nullable) at the current
 * parameters; no update. */
int fock_mlp_loss_grad(fock_mlp_t *net, const float *X, const float *T, const int *nvalid, int B, double *loss,
                       float *grad, fock_stream_t stream);
/* One Adam step on the batch; *loss (nullable; non-null synchronises) is the
 * loss before the step. */
int fock_mlp_adam_step(fock_mlp_t *net, const float *X, const float *T, const int *nvalid, int B, float lr,
                       double *loss, fock_stream_t stream);
int fock_mlp_destroy(fock_mlp_t *net);

/* ------------------------------------------------------------------ profiling */

/* Streaming-bandwidth probe: the measured HBM ceiling the kernel rooflines are
 * read against.  kind 0 copies `bytes` from a to b, kind 1 reads a (one float
 * per workgroup is written to b), kind 2 updates b in place (multiplies every
 * complex64 value by i).  grid workgroups of 256 threads, grid-stride, 16-byte
 * accesses; one untimed warm-up launch, then *ms = mean duration (ms) of
 * `iters` launches from HIP events on `stream` (synchronised on return).
 * Buffers are the caller's (device, 16-byte aligned, `bytes` each; a unused
 * for kind 2).  FOCK_ERR_ARG on a bad kind, size, grid, count or pointer. */
int fock_stream_probe(int kind, const void *a, void *b, size_t bytes, int grid, int iters, double *ms,
                      fock_stream_t stream);


/* Kernel ids for per-kernel timing by HIP events recorded on the launch stream. */
enum { FOCK_K_APPLY_H = 0, FOCK_K_POOL = 1, FOCK_K_GATE = 2, FOCK_K_ADJ = 3, FOCK_K_DIAG = 4,
       FOCK_K_REDUCE = 5, FOCK_K_MLP_FWD = 6, FOCK_K_MLP_TRAIN = 7, FOCK_K_GATE_DENSE = 8,
       FOCK_K_SCORE = 9 /* fused scoring: H psi and pool partials, fock_score / adapt_step */,
       FOCK_K_RGATE = 10, FOCK_K_RADJ = 11 /* gates and reverse steps on real states (adapt_real) */,
       FOCK_K_CONVERT = 12 /* real <-> complex64 state conversion around H psi */,
       FOCK_K_APPLY_H_REAL = 13 /* two-pass H psi on real states */,
       FOCK_K_RFUSE = 14, FOCK_K_RFUSE_ADJ = 15 /* fused runs of real gates / reverse steps */,
       FOCK_K_NUM = 16 };

/* Enable/disable event timing of launches (off by default). */
int fock_prof_enable(int on);
/* Time only every `every`-th launch of each kernel id (1, the default: every
 * launch).  Each timed launch is bracketed by two event records on its
 * stream, which lengthen the gaps between dependent kernels; sampling keeps
 * that cost off the untimed launches.  Counting restarts at fock_prof_reset.
 * FOCK_ERR_ARG for every < 1; process-wide. */
int fock_prof_set_sample(int every);
/* Launch count, summed duration (ms) and summed algorithmic bytes (FLOPs for
 * the two network kernels) of kernel id
 * since the last reset (completed launches only; call after a synchronise). */
int fock_prof_query(int kernel_id, int64_t *launches, double *total_ms, double *bytes);
int fock_prof_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* FOCK_H */
