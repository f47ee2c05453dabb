// C ABI of libfock: argument validation, workspace layout, the energy /
// adjoint-gradient pipeline, pool scoring, and the ADAPT state machine.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "bfgs.h"
#include "dense_internal.h"
#include "fuse_internal.h"
#include "pipeline.h"

namespace fock {

// ---------------------------------------------------------------- validation
int check_geometry(int L, int d, uint32_t *namp) {
  if (L < 1 || L > kMaxL) return set_error(FOCK_ERR_UNSUPPORTED, "L=%d outside [1, %d]", L, kMaxL);
  if (d < 2 || d > kMaxD) return set_error(FOCK_ERR_UNSUPPORTED, "d=%d outside [2, %d]", d, kMaxD);
  uint64_t n = 1;
  for (int r = 0; r < L; ++r) {
    n *= (uint64_t)d;
    if (n > (1ull << 31)) return set_error(FOCK_ERR_SIZE, "d^L = %d^%d exceeds 2^31 amplitudes", d, L);
  }
  *namp = (uint32_t)n;
  return FOCK_OK;
}

int check_ham_layout(const fock_ham_t *h, uint32_t *namp, bool allow_real) {
  if (!h) return set_error(FOCK_ERR_ARG, "ham is NULL");
  int rc = check_geometry(h->L, h->d, namp);
  if (rc) return rc;
  const double v[5] = {h->J, h->U, h->mu, h->Delta, h->K};
  for (double x : v)
    if (!std::isfinite(x)) return set_error(FOCK_ERR_NONFINITE, "non-finite Hamiltonian parameter");
  const int sector = h->layout & 3;
  if (sector > FOCK_LAYOUT_ODD || (h->layout & ~(3 | FOCK_LAYOUT_REAL)) != 0)
    return set_error(FOCK_ERR_ARG, "layout %d is not 0, 1 or 2, optionally with FOCK_LAYOUT_REAL (4)", h->layout);
  if (sector != FOCK_LAYOUT_FULL) {
    if (h->L != 8 || h->d != 8 || h->periodic)
      return set_error(FOCK_ERR_UNSUPPORTED, "the parity-halved layout is for open chains of L = 8, d = 8");
    *namp /= 2;
  }
  if (h->layout & FOCK_LAYOUT_REAL) {
    if (!allow_real) return set_error(FOCK_ERR_UNSUPPORTED, "this call takes complex64 states (no FOCK_LAYOUT_REAL)");
    if (h->L != 8 || h->d != 8 || h->periodic)
      return set_error(FOCK_ERR_UNSUPPORTED, "real states are taken for open chains of L = 8, d = 8");
  }
  return FOCK_OK;
}

int check_ham(const fock_ham_t *h, uint32_t *namp) {
  int rc = check_ham_layout(h, namp);
  if (rc) return rc;
  if (h->layout != FOCK_LAYOUT_FULL)
    return set_error(FOCK_ERR_UNSUPPORTED, "this call takes full d^L states (layout 0)");
  return FOCK_OK;
}

int check_op(const fock_op_t &op, int L) {
  if (op.type < FOCK_HR || op.type > FOCK_SI) return set_error(FOCK_ERR_ARG, "unknown op type %d", op.type);
  if (is_single_mode(op.type)) {
    if (op.i < 0 || op.i >= L) return set_error(FOCK_ERR_ARG, "mode %d out of range for L=%d", op.i, L);
    return FOCK_OK;
  }
  if (op.i < 0 || op.j < 0 || op.i >= L || op.j >= L)
    return set_error(FOCK_ERR_ARG, "mode pair (%d,%d) out of range for L=%d", op.i, op.j, L);
  if (op.i >= op.j) return set_error(FOCK_ERR_ARG, "mode pair (%d,%d) needs i < j", op.i, op.j);
  return FOCK_OK;
}

int check_ptr(const void *p, const char *name) {
  if (!p) return set_error(FOCK_ERR_ARG, "%s is NULL", name);
  if (((uintptr_t)p) & 15) return set_error(FOCK_ERR_ARG, "%s is not 16-byte aligned", name);
  return FOCK_OK;
}

HamArgs make_ham_args(const fock_ham_t &h) {
  HamArgs a;
  memset(&a, 0, sizeof(a));
  a.L = h.L;
  a.d = h.d;
  int nr = 1;
  for (int r = 1; r < h.L; ++r) nr *= h.d;
  a.nrows = nr;
  a.periodic_wrap = (h.periodic && h.L >= 3) ? 1 : 0;
  a.J = (float)h.J;
  a.Delta = (float)h.Delta;
  a.c2 = (float)(0.5 * h.U + h.K);
  a.mu = (float)h.mu;
  int s = 1;
  for (int r = 1; r < h.L; ++r) {
    a.srow[r] = s;
    s *= h.d;
  }
  for (int k = 0; k <= kMaxD; ++k) a.sq[k] = (float)std::sqrt((double)k);
  return a;
}

// ---------------------------------------------------------------- pinned staging
struct Pinned {
  void *p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
  int reserve(size_t bytes) {
    if (pending) {
      FOCK_HIP(hipEventSynchronize(ev));
      pending = false;
    }
    if (!ev) FOCK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (bytes > cap) {
      if (p) FOCK_HIP(hipHostFree(p));
      p = nullptr;
      size_t c = std::max<size_t>(bytes, 1 << 16);
      FOCK_HIP(hipHostMalloc(&p, c, hipHostMallocDefault));
      cap = c;
    }
    return FOCK_OK;
  }
  int mark(hipStream_t s) {
    FOCK_HIP(hipEventRecord(ev, s));
    pending = true;
    return FOCK_OK;
  }
};
static thread_local Pinned tl_in, tl_out;

// Results written by a kernel straight into host memory: fine-grained
// (coherent) pinned memory, so the stream synchronisation that follows the
// kernel is all the host waits for.  One per thread, sized for the longest
// circuit (energy, norm and 4096 gradients).
constexpr size_t kHostResults = 2 + 4096;
struct HostResults {
  double *p = nullptr;
  size_t cap = 0;
  int reserve(size_t count) {
    if (count <= cap) return FOCK_OK;
    if (p) FOCK_HIP(hipHostFree(p));
    p = nullptr;
    const size_t c = std::max<size_t>(count, kHostResults);
    FOCK_HIP(hipHostMalloc((void **)&p, sizeof(double) * c, hipHostMallocCoherent | hipHostMallocMapped));
    cap = c;
    return FOCK_OK;
  }
};
static thread_local HostResults tl_res;

// ---------------------------------------------------------------- workspace layout
static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(uint32_t namp, int Lm, int d, int P, int n, int half) {
  Layout L;
  const uint32_t nrows = namp / (uint32_t)d;
  L.G = (int)((nrows + kBlock - 1) / kBlock);
  L.G = std::max(L.G, (int)(nrows / (uint32_t)apply_h_tile_rows(Lm, d)));
  L.rs = L.G;
  if (Lm >= 2) {
    Geometry g{Lm, d, namp};
    g.half = half;
    L.rs = std::max(L.G, gate_blocks_max(g));
  }
  L.nmax = std::max(n, 1);
  L.pmax = std::min(std::max(P, 1), kMaxSlots);
  size_t o = 0;
  L.theta = o;
  o = al(o + sizeof(double) * L.nmax);
  L.recs = o;
  o = al(o + sizeof(GateRec) * L.nmax);
  L.utab = o;
  o = al(o + sizeof(float2) * (size_t)gate_stride(d) * L.nmax);
  L.partial = o;
  // gate rows, plus two rows after them for the energy partials of a gradient
  // evaluation on real states (reduced with the gate rows)
  const size_t rows = std::max<size_t>({2, (size_t)L.nmax + 2, (size_t)L.pmax});
  o = al(o + sizeof(double) * rows * std::max(L.G, L.rs));
  L.result = o;
  o = al(o + sizeof(double) * (2 + std::max(L.nmax, std::max(P, 1))));
  L.pairs = o;
  o = al(o + sizeof(PoolPair) * kMaxPairs);
  L.diags = o;
  o = al(o + sizeof(PoolDiag) * kMaxDiagOps);
  L.wdense = o;
  o = al(o + dense_w_bytes(d));
  L.total = o;
  return L;
}

// ---------------------------------------------------------------- shared pipeline
int make_ctx(const fock_ham_t &ham, uint32_t namp, int P, int n, void *ws, size_t ws_bytes, hipStream_t s,
                    Ctx *c) {
  c->g = {ham.L, ham.d, namp};
  c->h = make_ham_args(ham);
  if ((ham.layout & 3) != FOCK_LAYOUT_FULL) {
    c->g.half = c->h.half = 1;
    c->g.sector = c->h.sector = (ham.layout & 3) == FOCK_LAYOUT_ODD ? 1 : 0;
  }
  memset(&c->T, 0, sizeof(c->T));  // eigendata loaded below when the call applies gates
  {
    int rc = stencil_order_table(ham.L, ham.d, apply_h_blocks(c->h), &c->h.order);
    if (rc) return rc;
    if (stencil_schedule() == FOCK_SCHED_TWO_PASS)
      c->h.hi_m = apply_h_hi_modes(ham.L, ham.d, c->h.periodic_wrap);
    c->h.lanes = (stencil_variant() == FOCK_STENCIL_LANES && c->h.hi_m == 0 &&
                  lanes_stencil_ok(ham.L, ham.d, c->h.periodic_wrap)) ? 1 : 0;
    c->h.slab = (stencil_variant() == FOCK_STENCIL_SLAB && c->h.hi_m == 0 && slab_stencil_ok(ham.L, ham.d)) ? 1 : 0;
  }
  if (c->g.half && !c->h.slab)
    return set_error(FOCK_ERR_UNSUPPORTED, "the parity-halved layout needs the slab stencil with the one-pass schedule");
  c->s = s;
  c->ws = (char *)ws;
  c->L = make_layout(namp, ham.L, ham.d, P, n, c->g.half);
  if (!ws) return set_error(FOCK_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return set_error(FOCK_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < c->L.total)
    return set_error(FOCK_ERR_SIZE, "workspace too small: %zu < %zu bytes", ws_bytes, c->L.total);
  if (n > 0) {
    int rc = get_tables(ham.d, &c->T);
    if (rc) return rc;
  }
  return FOCK_OK;
}

int stage_gates(Ctx &c, const fock_op_t *ops, const double *theta, int n, const int *nblk) {
  const int stride = gate_stride(c.g.d);
  if (n <= kArgGates) {  // angles and records ride in the build kernel's arguments
    GateArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.n = n;
    const int Gd = diag_blocks_count(c.g);
    for (int k = 0; k < n; ++k) {
      if (!std::isfinite(theta[k])) return set_error(FOCK_ERR_NONFINITE, "theta[%d] is not finite", k);
      ga.theta[k] = theta[k];
      GateRec &r = ga.rec[k];
      r.type = ops[k].type;
      r.u_off = k * stride;
      r.nblk = nblk && nblk[k] > 0 ? nblk[k] : is_single_mode(ops[k].type) ? Gd : gate_blocks_count(c.g, ops[k].i);
    }
    return launch_gate_build_args(ga, c.T, (float2 *)(c.ws + c.L.utab), (double *)(c.ws + c.L.theta),
                                  (GateRec *)(c.ws + c.L.recs), c.s);
  }
  const size_t bt = sizeof(double) * n, br = sizeof(GateRec) * n;
  int rc = tl_in.reserve(c.L.recs + br);
  if (rc) return rc;
  char *hp = (char *)tl_in.p;
  double *th = (double *)(hp + c.L.theta);
  GateRec *rec = (GateRec *)(hp + c.L.recs);
  const int Gd = diag_blocks_count(c.g);
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(theta[k])) return set_error(FOCK_ERR_NONFINITE, "theta[%d] is not finite", k);
    th[k] = theta[k];
    rec[k].type = ops[k].type;
    rec[k].u_off = k * stride;
    rec[k].nblk = nblk && nblk[k] > 0 ? nblk[k] : is_single_mode(ops[k].type) ? Gd : gate_blocks_count(c.g, ops[k].i);
    rec[k].pad = 0;
  }
  (void)bt;
  FOCK_HIP(hipMemcpyAsync(c.ws + c.L.theta, hp + c.L.theta, c.L.recs + br - c.L.theta, hipMemcpyHostToDevice, c.s));
  rc = tl_in.mark(c.s);
  if (rc) return rc;
  return launch_gate_build((const double *)(c.ws + c.L.theta), (const GateRec *)(c.ws + c.L.recs), n, c.T,
                           (float2 *)(c.ws + c.L.utab), c.s);
}

static std::atomic<int> g_state_store{FOCK_STORE_AUTO};

// States up to this size stay in the 256 MiB Infinity Cache while gates update
// them in place, which then beats writing each forward state to a fresh buffer
// (measured: neutral at 134 MB, +10 % steps/s with the store at 1.07 GB).
constexpr size_t kStoreAutoMinBytes = (size_t)256 << 20;

// A store of nmax forward states for c, when switched on (always, or with
// FOCK_STORE_AUTO when one state exceeds the Infinity Cache) and the device has
// room (the store takes at most half of the free device memory); *owner
// receives the allocation, or nullptr when no store is kept (the in-place
// reverse sweep then runs).
int attach_state_store(Ctx &c, int nmax, void **owner) {
  *owner = nullptr;
  const int mode = g_state_store.load();
  const size_t sbytes = (sizeof(float2) * (size_t)c.g.n_amp + 255) & ~(size_t)255;
  if (mode == FOCK_STORE_OFF || nmax < 1) return FOCK_OK;
  if (mode == FOCK_STORE_AUTO && sbytes <= kStoreAutoMinBytes) return FOCK_OK;
  const size_t need = sbytes * (size_t)nmax;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess || need > fr / 2) {
    (void)hipGetLastError();
    return FOCK_OK;
  }
  void *p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    return FOCK_OK;
  }
  c.store = (float2 *)p;
  c.nstore = nmax;
  c.sstride = sbytes / sizeof(float2);
  *owner = p;
  return FOCK_OK;
}

static std::atomic<int> g_gate_variant{FOCK_GATE_BLOCK};

int gate_variant() { return g_gate_variant.load(); }

int forward_gate(Ctx &c, const fock_op_t &op, int k, bool dag, const float2 *src, float2 *psi) {
  const float2 *U = (const float2 *)(c.ws + c.L.utab) + (size_t)k * gate_stride(c.g.d);
  if (!is_single_mode(op.type) && !c.g.half && gate_variant() == FOCK_GATE_DENSE_MFMA && dense_supported(c.g.d)) {
    ProfScope ps(FOCK_K_GATE_DENSE, c.s, 16.0 * c.g.n_amp);
    return launch_gate_dense(c.g, op.i, op.j, gate_kind(op.type), dag, U, src, psi, (float *)(c.ws + c.L.wdense),
                             c.s);
  }
  ProfScope ps(is_single_mode(op.type) ? FOCK_K_DIAG : FOCK_K_GATE, c.s, 16.0 * c.g.n_amp);
  if (is_squeeze(op.type)) return launch_gate1(c.g, op.i, dag, U, src, psi, c.s);
  if (is_single_mode(op.type)) return launch_diag(c.g, op.i, op.type, dag, U, src, psi, c.s);
  return launch_gate(c.g, op.i, op.j, gate_kind(op.type), dag, U, src, psi, c.s);
}

int apply_h_dev(Ctx &c, const float2 *psi, float2 *hpsi, double *res2) {
  int G = 0;
  {
    ProfScope ps(FOCK_K_APPLY_H, c.s, 16.0 * c.g.n_amp);
    int rc = c.h.slab ? launch_apply_h2(c.h, psi, hpsi, (double *)(c.ws + c.L.partial), &G, c.s)
                      : launch_apply_h(c.h, psi, hpsi, (double *)(c.ws + c.L.partial), &G, c.s);
    if (rc) return rc;
  }
  return launch_reduce((const double *)(c.ws + c.L.partial), G, 2, res2, c.s);
}

int fetch_results(Ctx &c, int count, double *host) {
  int rc = tl_out.reserve(sizeof(double) * count);
  if (rc) return rc;
  FOCK_HIP(hipMemcpyAsync(tl_out.p, c.ws + c.L.result, sizeof(double) * count, hipMemcpyDeviceToHost, c.s));
  FOCK_HIP(hipStreamSynchronize(c.s));
  prof_harvest();
  memcpy(host, tl_out.p, sizeof(double) * count);
  return FOCK_OK;
}

// ---------------------------------------------------------------- gate fusion
static std::atomic<int> g_fuse{FOCK_FUSE_OFF};

bool fuse_supported(int d) { return d == 2 || d == 4 || d == 6 || d == 8; }

int fuse_max_modes(int L, int d) {
  int s = 0;
  for (long t = d; t <= 4096 && s < kMaxFuseModes && s < L; t *= d) ++s;
  return s;
}

// Greedy grouping: a group grows while the union of its gates' modes and mode
// 0 fits smax modes; its tile is that union filled up with the lowest other
// modes.  Kept when it has at least two gates and its tile holds mode 1 (rows
// of d^2 contiguous amplitudes) or at least three gates; groups whose tile
// count exceeds the partial-row stride are not fused.
static void plan_gate_groups(const Ctx &c, const fock_op_t *ops, int n, std::vector<GateGroup> *out) {
  out->clear();
  const int L = c.g.L, d = c.g.d, smax = fuse_max_modes(L, d);
  const bool on = !c.g.half && g_fuse.load() != FOCK_FUSE_OFF && fuse_supported(d) && smax >= 2;
  int k = 0;
  while (k < n) {
    GateGroup gr;
    gr.k0 = k;
    gr.k1 = k + 1;
    gr.s = 0;
    // consecutive single-mode phase gates commute: one diagonal pass
    const int k1 = diag_run_end(ops, n, k);
    if (k1 > k) {
      gr.k1 = k1;
      gr.diag = true;
      out->push_back(gr);
      k = k1;
      continue;
    }
    if (on) {
      unsigned mask = 1u;  // modes in the union (mode 0 always)
      auto modes = [&](const fock_op_t &o) { return is_single_mode(o.type) ? (1u << o.i) : ((1u << o.i) | (1u << o.j)); };
      mask |= modes(ops[k]);
      int k1 = k + 1;
      // squeezer gates are not fused: they run alone on the per-gate kernels
      while (!is_squeeze(ops[k].type) && k1 < n && k1 - k < kMaxFuseGates && !is_squeeze(ops[k1].type)) {
        const unsigned nm = mask | modes(ops[k1]);
        if (__builtin_popcount(nm) > smax) break;
        mask = nm;
        ++k1;
      }
      for (int r = 0; r < L && __builtin_popcount(mask) < smax; ++r) mask |= 1u << r;
      const int size = k1 - k;
      const int s = __builtin_popcount(mask);
      long ntile = 1;
      for (int r = 0; r < L - s; ++r) ntile *= d;
      if (size >= 2 && ((mask & 2u) || size >= 3) && ntile <= c.L.rs) {
        gr.k1 = k1;
        gr.s = 0;
        for (int r = 0; r < L; ++r)
          if (mask & (1u << r)) gr.m[gr.s++] = r;
      }
    }
    out->push_back(gr);
    k = gr.k1;
  }
}

static FuseArgs make_fuse_args(const Ctx &c, const GateGroup &gr, const fock_op_t *ops) {
  FuseArgs a;
  memset(&a, 0, sizeof(a));
  const int L = c.g.L, d = c.g.d;
  std::vector<uint32_t> pw(L, 1);
  for (int r = 1; r < L; ++r) pw[r] = pw[r - 1] * (uint32_t)d;
  a.s = gr.s;
  int pos[kMaxL];
  for (int r = 0; r < L; ++r) pos[r] = -1;
  for (int k = 0; k < gr.s; ++k) {
    a.tstride[k] = pw[gr.m[k]];
    pos[gr.m[k]] = k;
  }
  a.nc = 0;
  a.ntile = 1;
  for (int r = 0; r < L; ++r)
    if (pos[r] < 0) {
      a.cstride[a.nc++] = pw[r];
      a.ntile *= d;
    }
  int off = 0;
  for (int sb = 0; sb <= 2 * d - 2; ++sb) {
    a.boff[sb] = off;
    const int b = blk_hi(KIND_SUM, d, sb) - blk_lo(KIND_SUM, d, sb) + 1;
    off += b * b;
  }
  for (int t = 0; t < kTwoModeTypes; ++t) a.A[t] = c.T.A[t];
  a.ng = gr.k1 - gr.k0;
  for (int q = 0; q < a.ng; ++q) {
    const int k = gr.k0 + q;
    const fock_op_t &o = ops[k];
    FuseGate &g = a.g[q];
    g.type = o.type;
    g.kind = is_single_mode(o.type) ? 0 : gate_kind(o.type);
    g.ki = pos[o.i];
    g.kj = is_single_mode(o.type) ? -1 : pos[o.j];
    g.u_off = k * gate_stride(d);
    g.k = k;
  }
  return a;
}

// Stage the gate tables of a circuit (with the per-gate partial counts of the
// reverse step, which depend on how the gates are grouped) and plan its groups.
// Gates the parity-halved layout runs: two-mode HR..PI generators (they keep
// the total parity) on pairs below the top mode or on the top pair itself.
bool half_layout_op_ok(const fock_op_t &op, int L) {
  if (op.type < FOCK_HR || op.type > FOCK_PI || op.j < 0) return false;
  return op.j < L - 1 || op.i == L - 2;
}

static int stage_circuit(Ctx &c, const fock_op_t *ops, const double *theta, int n, std::vector<GateGroup> *groups) {
  if (n > c.L.nmax) return set_error(FOCK_ERR_SIZE, "circuit of %d gates exceeds the workspace's %d", n, c.L.nmax);
  if (c.g.half)
    for (int k = 0; k < n; ++k)
      if (!half_layout_op_ok(ops[k], c.g.L))
        return set_error(FOCK_ERR_UNSUPPORTED, "gate %d (type %d on (%d,%d)) in the parity-halved layout", k,
                         ops[k].type, ops[k].i, ops[k].j);
  plan_gate_groups(c, ops, n, groups);
  if (n == 0) return FOCK_OK;
  const bool fuse_rev = g_fuse.load() == FOCK_FUSE_ALL;
  std::vector<int> nblk(n, 0);
  for (const GateGroup &gr : *groups)
    if (gr.s > 0 && fuse_rev) {
      int nt = 1;
      for (int r = 0; r < c.g.L - gr.s; ++r) nt *= c.g.d;
      for (int k = gr.k0; k < gr.k1; ++k) nblk[k] = nt;
    }
  return stage_gates(c, ops, theta, n, nblk.data());
}

// True when a gradient evaluation of this circuit can keep its forward states:
// a store of at least n states, no fused gate runs and no squeezer gates
// (their reverse kernels always rewrite phi).
static bool use_store(const Ctx &c, const fock_op_t *ops, int n, const std::vector<GateGroup> &groups) {
  if (!c.store || n < 1 || n > c.nstore) return false;
  for (const GateGroup &gr : groups)
    if (gr.s > 0 || gr.diag) return false;
  for (int k = 0; k < n; ++k)
    if (is_squeeze(ops[k].type)) return false;
  return true;
}

static float2 *stored_state(const Ctx &c, int k) { return c.store + (size_t)(k - 1) * c.sstride; }

// Reverse sweep with the forward states kept: gate k reads phi_k from the
// store (read-only) and updates lam <- U_k^+ lam; 24 B per amplitude instead
// of 32.
static int reverse_sweep_stored(Ctx &c, const fock_op_t *ops, int n, float2 *lam, double *res) {
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  double *part = (double *)(c.ws + c.L.partial);
  const int stride = gate_stride(c.g.d);
  for (int k = n - 1; k >= 0; --k) {
    const fock_op_t &op = ops[k];
    const float2 *U = utab + (size_t)k * stride;
    double *pk = part + (size_t)k * c.L.rs;
    float2 *phik = stored_state(c, k + 1);
    ProfScope ps(is_single_mode(op.type) ? FOCK_K_DIAG : FOCK_K_ADJ, c.s, 24.0 * c.g.n_amp);
    const int rc = is_single_mode(op.type)
                       ? launch_diag_adj(c.g, op.i, op.type, U, phik, lam, pk, c.s, false)
                       : launch_gate_adj(c.g, op.i, op.j, gate_kind(op.type), U, c.T.A[table_slot(op.type)], phik, lam,
                                         pk, c.s, false);
    if (rc) return rc;
  }
  return launch_reduce_rows(part, c.L.rs, (const GateRec *)(c.ws + c.L.recs), n, res, c.s);
}

// Reverse sweep from phi = psi_n, lam = H psi_n (both overwritten): per-gate
// sums of Re<lam|A_k phi> reduced into res[0..n) (device), in stream order.
static int reverse_sweep(Ctx &c, const fock_op_t *ops, int n, const std::vector<GateGroup> &groups, float2 *phi,
                         float2 *lam, double *res) {
  if (n == 0) return FOCK_OK;
  int rc = FOCK_OK;
  const bool fuse_rev = g_fuse.load() == FOCK_FUSE_ALL;
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  double *part = (double *)(c.ws + c.L.partial);
  const int stride = gate_stride(c.g.d);
  for (int gi = (int)groups.size() - 1; gi >= 0; --gi) {
    const GateGroup &gr = groups[gi];
    if (gr.diag) {
      ProfScope ps(FOCK_K_DIAG, c.s, 32.0 * c.g.n_amp);
      rc = launch_diag_run_adj(c.g, diag_run_params(c.g, ops, gr.k0, gr.k1), utab + (size_t)gr.k0 * stride, phi, lam,
                               part + (size_t)gr.k0 * c.L.rs, c.L.rs, c.s);
      if (rc) return rc;
      continue;
    }
    if (gr.s > 0 && fuse_rev) {
      ProfScope ps(FOCK_K_ADJ, c.s, 32.0 * c.g.n_amp);
      rc = launch_fuse_adj(c.g.d, make_fuse_args(c, gr, ops), phi, lam, utab, part, c.L.rs, c.s);
      if (rc) return rc;
      continue;
    }
    for (int k = gr.k1 - 1; k >= gr.k0; --k) {
      const fock_op_t &op = ops[k];
      const float2 *U = utab + (size_t)k * stride;
      double *pk = part + (size_t)k * c.L.rs;
      ProfScope ps(is_single_mode(op.type) ? FOCK_K_DIAG : FOCK_K_ADJ, c.s, 32.0 * c.g.n_amp);
      if (is_squeeze(op.type))
        rc = launch_gate1_adj(c.g, op.i, U, c.T.A1[op.type == FOCK_SR ? 0 : 1], phi, lam, pk, c.s);
      else if (is_single_mode(op.type)) rc = launch_diag_adj(c.g, op.i, op.type, U, phi, lam, pk, c.s);
      else rc = launch_gate_adj(c.g, op.i, op.j, gate_kind(op.type), U, c.T.A[table_slot(op.type)], phi, lam, pk,
                                c.s);
      if (rc) return rc;
    }
  }
  return launch_reduce_rows(part, c.L.rs, (const GateRec *)(c.ws + c.L.recs), n, res, c.s);
}

// phi_k = O_k phi_{k-1} into store buffer k - 1 for k = 1..n (phi_0 = psi0).
static int forward_stored(Ctx &c, const fock_op_t *ops, int n, const void *psi0) {
  for (int k = 0; k < n; ++k) {
    const float2 *src = k == 0 ? (const float2 *)psi0 : stored_state(c, k);
    const int rc = forward_gate(c, ops[k], k, false, src, stored_state(c, k + 1));
    if (rc) return rc;
  }
  return FOCK_OK;
}

// phi = O_n..O_1 psi0 for a staged circuit (the first gate reads psi0 directly).
static int forward_circuit(Ctx &c, const fock_op_t *ops, int n, const std::vector<GateGroup> &groups,
                           const void *psi0, float2 *phi) {
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  if (n == 0)
    FOCK_HIP(hipMemcpyAsync(phi, psi0, sizeof(float2) * (size_t)c.g.n_amp, hipMemcpyDeviceToDevice, c.s));
  for (const GateGroup &gr : groups) {
    const float2 *src = gr.k0 == 0 ? (const float2 *)psi0 : phi;
    int rc;
    if (gr.diag) {
      ProfScope ps(FOCK_K_DIAG, c.s, 16.0 * c.g.n_amp);
      rc = launch_diag_run(c.g, diag_run_params(c.g, ops, gr.k0, gr.k1), false,
                           utab + (size_t)gr.k0 * gate_stride(c.g.d), src, phi, c.s);
    } else if (gr.s == 0) {
      rc = forward_gate(c, ops[gr.k0], gr.k0, false, src, phi);
    } else {
      ProfScope ps(FOCK_K_GATE, c.s, 16.0 * c.g.n_amp);
      rc = launch_fuse_fwd(c.g.d, make_fuse_args(c, gr, ops), src, phi, utab, c.s);
    }
    if (rc) return rc;
  }
  return FOCK_OK;
}

// ---------------------------------------------------------------- real states
static std::atomic<int> g_real_states{FOCK_REAL_AUTO};

int real_states_mode() { return g_real_states.load(); }

// An evaluation runs on real states when the context keeps them and every gate
// is HR or PR (real orthogonal) with a real-state kernel for its pair.
static bool real_eval(const Ctx &c, const fock_op_t *ops, int n) {
  if (!c.psi0_r) return false;
  for (int k = 0; k < n; ++k)
    if ((ops[k].type != FOCK_HR && ops[k].type != FOCK_PR) || !real_gate_supported(c.g, ops[k].i, ops[k].j))
      return false;
  return true;
}

static std::atomic<int> g_real_fusion{FOCK_RFUSE_ON};

// A run of a real-state evaluation: gates k0..k1-1 fused on modes a..a+2, or
// (a < 0) gate k0 by itself.
struct RealRun {
  int k0, k1, a;
};

// Greedy runs: extend while every pair of the run lies inside one window of
// three consecutive modes below the fusion's top mode; runs of one gate use the
// per-gate kernels.
static std::vector<RealRun> plan_real_runs(const Geometry &g, const fock_op_t *ops, int n) {
  std::vector<RealRun> runs;
  const bool on = g_real_fusion.load() == FOCK_RFUSE_ON && real_fuse_supported(g);
  const int top = on ? real_fuse_top(g) : 0;
  auto fusable = [&](int m) { return on && ops[m].i >= 0 && ops[m].j == ops[m].i + 1 && ops[m].j <= top; };
  for (int k = 0; k < n;) {
    int m = k + 1, lo = ops[k].i, hi = ops[k].i;
    if (fusable(k))
      for (; m < n && m - k < kRFuseMax && fusable(m); ++m) {
        const int nlo = std::min(lo, ops[m].i), nhi = std::max(hi, ops[m].i);
        if (nhi - nlo > 1) break;
        lo = nlo;
        hi = nhi;
      }
    if (m - k >= 2) {
      runs.push_back({k, m, std::min(lo, top - 2)});
    } else {
      runs.push_back({k, k + 1, -1});
      m = k + 1;
    }
    k = m;
  }
  return runs;
}

// Gate tables of a real-state evaluation, with the workgroup counts of the
// kernels that take each gate's reverse step as its partial counts.
static int stage_real(Ctx &c, const fock_op_t *ops, const double *theta, int n, std::vector<RealRun> *runs) {
  *runs = plan_real_runs(c.g, ops, n);
  std::vector<int> nblk(n > 0 ? n : 1);
  for (const RealRun &r : *runs)
    for (int k = r.k0; k < r.k1; ++k)
      nblk[k] = r.a >= 0 ? real_fuse_blocks(c.g, true) : real_gate_blocks(c.g, ops[k].i, ops[k].j);
  return stage_gates(c, ops, theta, n, nblk.data());
}

static void real_run_ops(const Ctx &c, const fock_op_t *ops, const RealRun &r, bool reverse, RFuseOp *fo) {
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  double *part = (double *)(c.ws + c.L.partial);
  const int stride = gate_stride(c.g.d);
  for (int k = r.k0; k < r.k1; ++k) {
    RFuseOp &f = fo[k - r.k0];
    f.kind = gate_kind(ops[k].type);
    f.o = ops[k].i - r.a;
    f.U = utab + (size_t)k * stride;
    f.A = reverse ? c.T.A[table_slot(ops[k].type)] : nullptr;
    f.part = reverse ? part + (size_t)k * c.L.rs : nullptr;
  }
}

// phi_r = O_n..O_1 psi0_r (staged gates), then (phi != nullptr) phi = phi_r
// widened to complex64.
static int forward_real(Ctx &c, const fock_op_t *ops, int n, const std::vector<RealRun> &runs, float2 *phi) {
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  const int stride = gate_stride(c.g.d);
  if (n == 0)
    FOCK_HIP(hipMemcpyAsync(c.phi_r, c.psi0_r, sizeof(float) * (size_t)c.g.n_amp, hipMemcpyDeviceToDevice, c.s));
  for (const RealRun &r : runs) {
    const float *src = r.k0 == 0 ? c.psi0_r : c.phi_r;
    int rc;
    if (r.a >= 0) {
      RFuseOp fo[kRFuseMax];
      real_run_ops(c, ops, r, false, fo);
      ProfScope ps(FOCK_K_RFUSE, c.s, 8.0 * c.g.n_amp);
      rc = launch_rfuse(c.g, r.a, r.k1 - r.k0, fo, src, c.phi_r, c.s);
    } else {
      const int k = r.k0;
      ProfScope ps(FOCK_K_RGATE, c.s, 8.0 * c.g.n_amp);
      rc = launch_rgate(c.g, ops[k].i, ops[k].j, gate_kind(ops[k].type), false, utab + (size_t)k * stride, src,
                        c.phi_r, c.s);
    }
    if (rc) return rc;
  }
  if (!phi) return FOCK_OK;
  ProfScope ps(FOCK_K_CONVERT, c.s, 12.0 * c.g.n_amp);
  return launch_real_convert(c.g.n_amp, true, c.phi_r, phi, c.s);
}

// H phi_r into lam_r and (<psi|H psi>, <psi|psi>) into res2, on real states;
// with defer, the energy partials go to the two rows after the n gate rows
// and *G receives their count, for reverse_real's reduction.
static int apply_h_real(Ctx &c, double *res2, int n = 0, bool defer = false, int *Gout = nullptr) {
  int G = 0;
  double *part = (double *)(c.ws + c.L.partial) + (defer ? (size_t)n * c.L.rs : 0);
  {
    ProfScope ps(FOCK_K_APPLY_H_REAL, c.s, 8.0 * c.g.n_amp);
    const int rc = launch_apply_h2_real(c.h, c.phi_r, c.lam_r, part, &G, c.s);
    if (rc) return rc;
  }
  if (defer) {
    if (G > std::max(c.L.G, c.L.rs) || n > c.L.nmax)  // rows n, n + 1 hold the 2 G partials
      return set_error(FOCK_ERR_SIZE, "energy partials beyond the workspace");
    *Gout = G;
    return FOCK_OK;
  }
  return launch_reduce(part, G, 2, res2, c.s);
}

// Reverse sweep on real states from phi_r and lam_r = H phi_r: per gate the
// partial sums of lam . A phi, then phi_r, lam_r <- U^T phi_r, U^T lam_r.
static int reverse_real(Ctx &c, const fock_op_t *ops, int n, const std::vector<RealRun> &runs, double *res,
                        int Ge = 0) {
  const float2 *utab = (const float2 *)(c.ws + c.L.utab);
  double *part = (double *)(c.ws + c.L.partial);
  const int stride = gate_stride(c.g.d);
  for (auto it = runs.rbegin(); it != runs.rend(); ++it) {
    const RealRun &r = *it;
    int rc;
    if (r.a >= 0) {
      RFuseOp fo[kRFuseMax];
      real_run_ops(c, ops, r, true, fo);
      ProfScope ps(FOCK_K_RFUSE_ADJ, c.s, 16.0 * c.g.n_amp);
      rc = launch_rfuse_adj(c.g, r.a, r.k1 - r.k0, fo, c.phi_r, c.lam_r, c.s);
    } else {
      const int k = r.k0;
      const fock_op_t &op = ops[k];
      ProfScope ps(FOCK_K_RADJ, c.s, 16.0 * c.g.n_amp);
      rc = launch_rgate_adj(c.g, op.i, op.j, gate_kind(op.type), utab + (size_t)k * stride,
                            c.T.A[table_slot(op.type)], c.phi_r, c.lam_r, part + (size_t)k * c.L.rs, c.s, true);
    }
    if (rc) return rc;
  }
  if (Ge > 0)  // with the energy partials of apply_h_real(defer): res[0..1] and res[2..]
    return launch_reduce_rows_energy(part, c.L.rs, (const GateRec *)(c.ws + c.L.recs), n, part + (size_t)n * c.L.rs,
                                     Ge, res, c.s);
  return launch_reduce_rows(part, c.L.rs, (const GateRec *)(c.ws + c.L.recs), n, res, c.s);
}

// State of a circuit, its energy and the pool gradients there, with the
// scoring fused where possible; g receives the raw 2 Re <H psi|A_k psi>.
int run_score(Ctx &c, const fock_op_t *ops, const double *theta, int n, const void *psi0, float2 *phi,
              float2 *lam, const fock_op_t *pool, int P, double *E, double *norm2, double *g) {
  std::vector<GateGroup> groups;
  std::vector<RealRun> runs;
  const bool real = real_eval(c, ops, n);
  int rc = real ? stage_real(c, ops, theta, n, &runs) : stage_circuit(c, ops, theta, n, &groups);
  if (rc) return rc;
  if ((rc = real ? forward_real(c, ops, n, runs, phi) : forward_circuit(c, ops, n, groups, psi0, phi))) return rc;
  double *res = (double *)(c.ws + c.L.result);
  if ((rc = score_dev(c, pool, P, phi, lam, res))) return rc;
  std::vector<double> host(2 + P);
  if ((rc = fetch_results(c, 2 + P, host.data()))) return rc;
  const double nrm = host[1];
  if (!std::isfinite(host[0]) || !std::isfinite(nrm) || nrm <= 0.0)
    return set_error(FOCK_ERR_NONFINITE, "non-finite energy or zero norm (E=%g, norm2=%g)", host[0], nrm);
  *E = host[0] / nrm;
  if (norm2) *norm2 = nrm;
  for (int k = 0; k < P; ++k) g[k] = host[2 + k];
  return FOCK_OK;
}

// Energy and (optionally) all dE/dtheta of a circuit; see fock_energy_grad_adjoint.
int run_circuit(Ctx &c, const fock_op_t *ops, const double *theta, int n, const void *psi0, float2 *phi,
                       float2 *lam, bool grad, double *E, double *norm2, double *dE) {
  std::vector<GateGroup> groups;
  std::vector<RealRun> runs;
  const bool real = real_eval(c, ops, n);
  int rc = real ? stage_real(c, ops, theta, n, &runs) : stage_circuit(c, ops, theta, n, &groups);
  if (rc) return rc;
  double *res = (double *)(c.ws + c.L.result);
  if (real) {
    // H psi on the real states when the slab passes take them, else on a
    // complex64 copy whose real part is kept
    const bool rh = apply_h2_real_supported(c.h) && c.h.slab;
    if ((rc = forward_real(c, ops, n, runs, rh ? nullptr : phi))) return rc;
    if (rh && grad && n > 0) {  // one reduction for the energy, the norm and all gradients,
      int Ge = 0;                 // written straight into host memory
      if ((rc = tl_res.reserve(2 + (size_t)n))) return rc;
      if ((rc = apply_h_real(c, res, n, true, &Ge))) return rc;
      if ((rc = reverse_real(c, ops, n, runs, tl_res.p, Ge))) return rc;
      FOCK_HIP(hipStreamSynchronize(c.s));
      prof_harvest();
      const double nrm = tl_res.p[1];
      if (!std::isfinite(tl_res.p[0]) || !std::isfinite(nrm) || nrm <= 0.0)
        return set_error(FOCK_ERR_NONFINITE, "non-finite energy or zero norm (E=%g, norm2=%g)", tl_res.p[0], nrm);
      *E = tl_res.p[0] / nrm;
      if (norm2) *norm2 = nrm;
      if (dE)
        for (int k = 0; k < n; ++k) dE[k] = 2.0 * tl_res.p[2 + k] / nrm;
      return FOCK_OK;
    } else {
      if (rh) {
        if ((rc = apply_h_real(c, res))) return rc;
      } else {
        if ((rc = apply_h_dev(c, phi, lam, res))) return rc;
        if (grad && n > 0) {
          ProfScope ps(FOCK_K_CONVERT, c.s, 12.0 * c.g.n_amp);
          if ((rc = launch_real_convert(c.g.n_amp, false, lam, c.lam_r, c.s))) return rc;
        }
      }
      if (grad && n > 0 && (rc = reverse_real(c, ops, n, runs, res + 2))) return rc;
    }
  } else if (grad && use_store(c, ops, n, groups)) {
    // forward states kept: H psi_n reads the last one; phi is not touched
    if ((rc = forward_stored(c, ops, n, psi0))) return rc;
    if ((rc = apply_h_dev(c, stored_state(c, n), lam, res))) return rc;
    if ((rc = reverse_sweep_stored(c, ops, n, lam, res + 2))) return rc;
  } else {
    if ((rc = forward_circuit(c, ops, n, groups, psi0, phi))) return rc;
    rc = apply_h_dev(c, phi, lam, res);
    if (rc) return rc;
    if (grad && n > 0) {
      rc = reverse_sweep(c, ops, n, groups, phi, lam, res + 2);
      if (rc) return rc;
    }
  }
  const int cnt = 2 + ((grad && n > 0) ? n : 0);
  std::vector<double> host(cnt);
  rc = fetch_results(c, cnt, host.data());
  if (rc) return rc;
  const double nrm = host[1];
  if (!std::isfinite(host[0]) || !std::isfinite(nrm) || nrm <= 0.0)
    return set_error(FOCK_ERR_NONFINITE, "non-finite energy or zero norm (E=%g, norm2=%g)", host[0], nrm);
  *E = host[0] / nrm;
  if (norm2) *norm2 = nrm;
  if (grad && dE)
    for (int k = 0; k < n; ++k) dE[k] = 2.0 * host[2 + k] / nrm;
  return FOCK_OK;
}

// All dE/dtheta by the reverse sweep alone, from phi = psi_n and lam = H psi_n
// left by an energy-only evaluation of the same circuit; see fock_adjoint_sweep.
int run_reverse(Ctx &c, const fock_op_t *ops, const double *theta, int n, float2 *phi, float2 *lam, double norm2,
                double *dE) {
  if (!(norm2 > 0.0) || !std::isfinite(norm2)) return set_error(FOCK_ERR_ARG, "norm2 must be finite and > 0");
  std::vector<GateGroup> groups;
  int rc = stage_circuit(c, ops, theta, n, &groups);
  if (rc || n == 0) return rc;
  double *res = (double *)(c.ws + c.L.result);
  rc = reverse_sweep(c, ops, n, groups, phi, lam, res);
  if (rc) return rc;
  std::vector<double> host(n);
  rc = fetch_results(c, n, host.data());
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(host[k])) return set_error(FOCK_ERR_NONFINITE, "non-finite gradient entry %d", k);
    dE[k] = 2.0 * host[k] / norm2;
  }
  return FOCK_OK;
}

// ---------------------------------------------------------------- parity-halved layout (ADAPT driver)
static std::atomic<int> g_sector_layout{FOCK_SECTOR_AUTO};

int sector_layout_mode() { return g_sector_layout.load(); }

// Whether the ADAPT driver may keep a parity-definite state of this chain in
// the parity-halved layout: switched on, an open L = 8, d = 8 chain under the
// slab stencil, a pool that the slab scoring takes whole (HR..PI on
// nearest-neighbour pairs, no repeats) and gates the layout runs.
bool half_layout_wanted(const fock_ham_t &h, const fock_op_t *pool, int P, const fock_op_t *ops, int n) {
  if (g_sector_layout.load() != FOCK_SECTOR_AUTO || h.L != 8 || h.d != 8 || h.periodic) return false;
  const int wrap = (h.periodic && h.L >= 3) ? 1 : 0;
  const int hi_m = stencil_schedule() == FOCK_SCHED_TWO_PASS ? apply_h_hi_modes(h.L, h.d, wrap) : 0;
  if (stencil_variant() != FOCK_STENCIL_SLAB || hi_m != 0 || !slab_stencil_ok(h.L, h.d)) return false;
  if (P < 1 || P > kMaxSlots) return false;
  bool seen[8][5] = {};
  for (int k = 0; k < P; ++k) {
    const fock_op_t &op = pool[k];
    if (op.type < FOCK_HR || op.type > FOCK_PI || op.j != op.i + 1 || op.i < 0 || op.i > 6) return false;
    if (seen[op.i][op.type]) return false;
    seen[op.i][op.type] = true;
  }
  for (int k = 0; k < n; ++k)
    if (!half_layout_op_ok(ops[k], h.L)) return false;
  return true;
}

// The whole pool as one slab-kernel chunk, when every entry is a two-mode
// generator (HR..PI) on a nearest-neighbour pair (p, p + 1), or on the ring pair
// (0, L - 1) of a ring, or a diagonal generator (at most kSlabDiag), with no
// duplicates and at most kMaxSlots entries; false otherwise.
static bool slab_pool_of(const Ctx &c, const fock_op_t *pool, int P, SlabPool *sp) {
  if (!c.h.slab || P < 1 || P > kMaxSlots) return false;
  memset(sp, 0, sizeof(*sp));
  for (int p = 0; p < 8; ++p)
    for (int t = 0; t < 5; ++t) sp->slot[p][t] = -1;
  for (int k = 0; k < P; ++k) {
    const fock_op_t &op = pool[k];
    if (is_pool_diagonal(op.type)) {
      if (c.g.half || sp->ndiag >= kSlabDiag) return false;
      sp->diag[sp->ndiag++] = {(int16_t)op.i, (int16_t)op.type, (int16_t)k, (int16_t)(op.type == FOCK_CK ? op.j : -1)};
      continue;
    }
    if (op.type > FOCK_PI) return false;  // squeezers
    int p = -1;
    if (op.j == op.i + 1 && op.i <= 6) p = op.i;
    else if (op.i == 0 && op.j == 7 && c.h.periodic_wrap) p = 7;
    if (p < 0 || sp->slot[p][op.type] >= 0) return false;
    sp->slot[p][op.type] = (int16_t)k;
  }
  sp->nslots = P;
  return true;
}

// H psi, (<psi|H psi>, <psi|psi>) into res[0..1] and the pool gradients
// 2 Re <H psi|A_k psi> into res[2..2+P), on the device: fused slab scoring when
// the pool fits it, else H psi followed by the pool pass.
int score_dev(Ctx &c, const fock_op_t *pool, int P, const float2 *psi, float2 *hpsi, double *res) {
  SlabPool sp;
  if (slab_pool_of(c, pool, P, &sp)) {
    double *ppart = (double *)(c.ws + c.L.partial);
    double *hpart = ppart + (size_t)pool_slab_blocks(c.h) * P;
    {
      ProfScope ps(FOCK_K_SCORE, c.s, 16.0 * c.g.n_amp);
      int rc = launch_score_slab(sp, c.h, psi, hpsi, hpart, ppart, c.s);
      if (rc) return rc;
    }
    int rc = launch_reduce(hpart, apply_h2_blocks(c.h), 2, res, c.s);
    if (rc) return rc;
    return launch_reduce(ppart, pool_slab_blocks(c.h), P, res + 2, c.s);
  }
  if (c.g.half) return set_error(FOCK_ERR_UNSUPPORTED, "pool outside the slab scoring in the parity-halved layout");
  int rc = apply_h_dev(c, psi, hpsi, res);
  if (rc) return rc;
  return pool_dev(c, pool, P, psi, hpsi, res + 2);
}

// Pool gradients 2 Re <hpsi|A_k psi> into res[0..P) on the device.
int pool_dev(Ctx &c, const fock_op_t *pool, int P, const float2 *psi, const float2 *hpsi, double *res) {
  if (c.g.half) {  // one slab chunk: nearest-neighbour pairs only
    SlabPool sp;
    if (!slab_pool_of(c, pool, P, &sp))
      return set_error(FOCK_ERR_UNSUPPORTED, "pool outside the slab scoring in the parity-halved layout");
    double *part = (double *)(c.ws + c.L.partial);
    int G = 0;
    {
      ProfScope ps(FOCK_K_POOL, c.s, 16.0 * c.g.n_amp);
      int rc = launch_pool_slab(sp, c.h, psi, hpsi, part, &G, c.s);
      if (rc) return rc;
    }
    return launch_reduce(part, G, P, res, c.s);
  }
  PoolArgs a;
  memset(&a, 0, sizeof(a));
  a.L = c.g.L;
  a.d = c.g.d;
  a.nrows = c.h.nrows;
  for (int r = 0; r < kMaxL; ++r) a.srow[r] = c.h.srow[r];
  for (int k = 0; k <= kMaxD; ++k) a.sq[k] = c.h.sq[k];
  a.order = c.h.order;  // same tiles as the Hamiltonian stencil
  double *part = (double *)(c.ws + c.L.partial);
  for (int k = 0; k < P; ++k)
    if (is_squeeze(pool[k].type) && c.T.d != c.g.d) {  // squeezer scoring reads the generator table
      int rc = get_tables(c.g.d, &c.T);
      if (rc) return rc;
      break;
    }
  int k0 = 0;
  while (k0 < P) {
    // chunk: up to kMaxSlots entries, kMaxPairs pairs, kMaxDiagOps single-mode ops
    std::vector<PoolPair> pairs;
    std::vector<PoolDiag> diags;
    std::map<std::pair<int, int>, int> pidx;
    std::vector<int> sq;  // squeezer entries: scored by their own pass after the chunk
    int k1 = k0;
    for (; k1 < P && k1 - k0 < kMaxSlots; ++k1) {
      const fock_op_t &op = pool[k1];
      const int slot = k1 - k0;
      if (is_squeeze(op.type)) {
        sq.push_back(k1);
        continue;
      }
      if (is_pool_diagonal(op.type)) {
        if ((int)diags.size() >= kMaxDiagOps) break;
        diags.push_back({(int16_t)op.i, (int16_t)op.type, (int16_t)slot, (int16_t)(op.type == FOCK_CK ? op.j : -1)});
        continue;
      }
      auto key = std::make_pair(op.i, op.j);
      auto it = pidx.find(key);
      if (it == pidx.end()) {
        if ((int)pairs.size() >= kMaxPairs) break;
        PoolPair pp;
        pp.i = (int16_t)op.i;
        pp.j = (int16_t)op.j;
        for (int t = 0; t < 5; ++t) pp.slot[t] = -1;
        pp.pad = 0;
        pidx[key] = (int)pairs.size();
        pairs.push_back(pp);
        it = pidx.find(key);
      }
      PoolPair &pp = pairs[it->second];
      if (pp.slot[op.type] >= 0) {
        // duplicate entry: start a new chunk so every slot keeps its own value
        break;
      }
      pp.slot[op.type] = (int16_t)slot;
    }
    if (k1 == k0) return set_error(FOCK_ERR_ARG, "cannot schedule pool entry %d", k0);
    // slab kernels (L = 8, d = 8): nearest-neighbour pairs, the ring pair and diagonal entries
    if (c.h.slab && (!pairs.empty() || !diags.empty())) {
      SlabPool sp;
      memset(&sp, 0, sizeof(sp));
      for (int p = 0; p < 8; ++p)
        for (int t = 0; t < 5; ++t) sp.slot[p][t] = -1;
      bool ok = (int)diags.size() <= kSlabDiag;
      for (const PoolPair &pp : pairs) {
        int p = -1;
        if (pp.j == pp.i + 1 && pp.i <= 6) p = pp.i;
        else if (pp.i == 0 && pp.j == 7 && c.h.periodic_wrap) p = 7;
        if (p < 0) {
          ok = false;
          break;
        }
        for (int t = 0; t < 5; ++t) sp.slot[p][t] = pp.slot[t];
      }
      if (ok) {
        sp.ndiag = (int)diags.size();
        for (int q = 0; q < sp.ndiag; ++q) sp.diag[q] = diags[q];
        sp.nslots = k1 - k0;
        int G = 0;
        {
          ProfScope ps(FOCK_K_POOL, c.s, 16.0 * c.g.n_amp);
          int rc = launch_pool_slab(sp, c.h, psi, hpsi, part, &G, c.s);
          if (rc) return rc;
        }
        int rc = launch_reduce(part, G, sp.nslots, res + k0, c.s);
        if (rc) return rc;
        for (int k : sq) {
          const fock_op_t &op = pool[k];
          int G1 = 0;
          {
            ProfScope ps(FOCK_K_POOL, c.s, 16.0 * c.g.n_amp);
            rc = launch_pool1(c.g, op.i, c.T.A1[op.type == FOCK_SR ? 0 : 1], psi, hpsi, part, &G1, c.s);
            if (rc) return rc;
          }
          rc = launch_reduce(part, G1, 1, res + k, c.s);
          if (rc) return rc;
        }
        k0 = k1;
        continue;
      }
    }
    a.npairs = (int)pairs.size();
    a.ndiag = (int)diags.size();
    a.nslots = k1 - k0;
    int rc = tl_in.reserve(c.L.diags + sizeof(PoolDiag) * kMaxDiagOps);
    if (rc) return rc;
    char *hp = (char *)tl_in.p;
    if (!pairs.empty()) memcpy(hp + c.L.pairs, pairs.data(), sizeof(PoolPair) * pairs.size());
    if (!diags.empty()) memcpy(hp + c.L.diags, diags.data(), sizeof(PoolDiag) * diags.size());
    FOCK_HIP(hipMemcpyAsync(c.ws + c.L.pairs, hp + c.L.pairs, c.L.diags + sizeof(PoolDiag) * kMaxDiagOps - c.L.pairs,
                            hipMemcpyHostToDevice, c.s));
    rc = tl_in.mark(c.s);
    if (rc) return rc;
    if (!pairs.empty() || !diags.empty()) {  // a chunk of squeezer entries only needs no stencil pass
      int G = 0;
      {
        ProfScope ps(FOCK_K_POOL, c.s, 16.0 * c.g.n_amp);
        rc = launch_pool(a, (const PoolPair *)(c.ws + c.L.pairs), (const PoolDiag *)(c.ws + c.L.diags), psi, hpsi,
                         part, &G, c.s);
        if (rc) return rc;
      }
      rc = launch_reduce(part, G, a.nslots, res + k0, c.s);
      if (rc) return rc;
    }
    for (int k : sq) {  // stream order: after the chunk's reduction has read the partials
      const fock_op_t &op = pool[k];
      int G1 = 0;
      {
        ProfScope ps(FOCK_K_POOL, c.s, 16.0 * c.g.n_amp);
        rc = launch_pool1(c.g, op.i, c.T.A1[op.type == FOCK_SR ? 0 : 1], psi, hpsi, part, &G1, c.s);
        if (rc) return rc;
      }
      rc = launch_reduce(part, G1, 1, res + k, c.s);
      if (rc) return rc;
    }
    k0 = k1;
  }
  return FOCK_OK;
}

}  // namespace fock

using namespace fock;

// ====================================================================== C ABI
extern "C" {

int fock_version(void) { return 1; }

int fock_prepare(int L, int d) {
  uint32_t namp = 0;
  int rc = check_geometry(L, d, &namp);
  if (rc) return rc;
  EigTables T;
  if ((rc = get_tables(d, &T))) return rc;
  fock_ham_t ham;
  memset(&ham, 0, sizeof(ham));
  ham.L = L;
  ham.d = d;
  for (int periodic = 0; periodic < 2; ++periodic) {
    ham.periodic = periodic;
    const HamArgs h = make_ham_args(ham);
    const int nt = apply_h_blocks(h);
    for (int scheme = 1; scheme < FOCK_SCHED_TWO_PASS; ++scheme) {
      const int *order = nullptr;
      if ((rc = stencil_order_table_for(L, d, nt, scheme, &order))) return rc;
    }
  }
  // pinned staging of this thread at its minimum size, and its results buffer
  if ((rc = tl_in.reserve(1))) return rc;
  if ((rc = tl_res.reserve(kHostResults))) return rc;
  return tl_out.reserve(1);
}

int fock_workspace_bytes(const fock_ham_t *ham, int n_pool, int n_ops, size_t *bytes) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp, true);
  if (rc) return rc;
  if (!bytes) return set_error(FOCK_ERR_ARG, "bytes is NULL");
  if (n_pool < 0 || n_pool > 4096 || n_ops < 0 || n_ops > 4096)
    return set_error(FOCK_ERR_ARG, "n_pool/n_ops out of range");
  *bytes = make_layout(namp, ham->L, ham->d, n_pool, n_ops, (ham->layout & 3) != FOCK_LAYOUT_FULL).total;
  return FOCK_OK;
}

int fock_apply_H(const fock_ham_t *ham, const void *psi, void *hpsi, double *E, double *norm2, void *ws,
                 size_t ws_bytes, fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp, true);
  if (rc) return rc;
  if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(hpsi, "hpsi"))) return rc;
  if (psi == hpsi) return set_error(FOCK_ERR_ARG, "psi and hpsi must not overlap");
  Ctx c;
  rc = make_ctx(*ham, namp, 0, 0, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  double *res = (double *)(c.ws + c.L.result);
  if (ham->layout & FOCK_LAYOUT_REAL) {
    c.phi_r = (float *)const_cast<void *>(psi);
    c.lam_r = (float *)hpsi;
    rc = apply_h_real(c, res);
  } else {
    rc = apply_h_dev(c, (const float2 *)psi, (float2 *)hpsi, res);
  }
  if (rc) return rc;
  if (E || norm2) {
    double h2[2];
    rc = fetch_results(c, 2, h2);
    if (rc) return rc;
    if (E) *E = h2[0];
    if (norm2) *norm2 = h2[1];
  }
  return FOCK_OK;
}

int fock_set_gate_variant(int variant) {
  if (variant != FOCK_GATE_BLOCK && variant != FOCK_GATE_DENSE_MFMA)
    return set_error(FOCK_ERR_ARG, "gate variant %d not in {0, 1}", variant);
  g_gate_variant.store(variant);
  return FOCK_OK;
}

int fock_get_gate_variant(void) { return g_gate_variant.load(); }

int fock_set_gate_fusion(int mode) {
  if (mode < FOCK_FUSE_OFF || mode > FOCK_FUSE_ALL)
    return set_error(FOCK_ERR_ARG, "gate fusion mode %d not in [0, 2]", mode);
  g_fuse.store(mode);
  return FOCK_OK;
}

int fock_get_gate_fusion(void) { return g_fuse.load(); }

int fock_autotune_stencil(const fock_ham_t *ham, const void *psi, void *hpsi, void *ws, size_t ws_bytes,
                          fock_stream_t stream, const char *cache_path, int *best_scheme) {
  uint32_t namp = 0;
  int rc = check_ham(ham, &namp);
  if (rc) return rc;
  if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(hpsi, "hpsi"))) return rc;
  if (psi == hpsi) return set_error(FOCK_ERR_ARG, "psi and hpsi must not overlap");
  hipDeviceProp_t prop;
  int dev = 0;
  FOCK_HIP(hipGetDevice(&dev));
  FOCK_HIP(hipGetDeviceProperties(&prop, dev));
  char key[256];
  snprintf(key, sizeof(key), "%s|stencil|L=%d|d=%d|periodic=%d|kitaev=%d", prop.gcnArchName, ham->L, ham->d,
           ham->periodic ? 1 : 0, ham->Delta != 0.0 ? 1 : 0);
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char line[512];
      int found = -1;
      while (fgets(line, sizeof(line), f)) {
        const char *k = strstr(line, key);
        const char *g = strstr(line, "\"scheme\": ");
        if (k && g) found = atoi(g + 10);
      }
      fclose(f);
      if (found >= 0 && found < FOCK_SCHED_NUM) {
        fock_set_stencil_schedule(found);
        if (best_scheme) *best_scheme = found;
        return FOCK_OK;
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  FOCK_HIP(hipEventCreate(&e0));
  FOCK_HIP(hipEventCreate(&e1));
  const int prev = fock_get_stencil_schedule();
  int best = prev;
  float best_ms = 1e30f;
  for (int sc = 0; sc < FOCK_SCHED_NUM && !rc; ++sc) {
    fock_set_stencil_schedule(sc);
    Ctx c;
    rc = make_ctx(*ham, namp, 0, 0, ws, ws_bytes, s, &c);
    if (rc) break;
    double *res = (double *)(c.ws + c.L.result);
    float t[5];
    for (int r = -1; r < 5 && !rc; ++r) {
      FOCK_HIP(hipEventRecord(e0, s));
      rc = apply_h_dev(c, (const float2 *)psi, (float2 *)hpsi, res);
      FOCK_HIP(hipEventRecord(e1, s));
      FOCK_HIP(hipEventSynchronize(e1));
      if (r >= 0) FOCK_HIP(hipEventElapsedTime(&t[r], e0, e1));
    }
    if (rc) break;
    std::sort(t, t + 5);
    if (t[2] < best_ms) {
      best_ms = t[2];
      best = sc;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  fock_set_stencil_schedule(rc ? prev : best);
  if (rc) return rc;
  if (best_scheme) *best_scheme = best;
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "{\"key\": \"%s\", \"scheme\": %d, \"ms\": %.5f}\n", key, best, best_ms);
      fclose(f);
    }
  }
  return FOCK_OK;
}

int fock_apply_gate2(int L, int d, fock_op_t op, double theta, int adjoint, void *psi, void *ws, size_t ws_bytes,
                     fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_geometry(L, d, &namp);
  if (rc) return rc;
  if ((rc = check_op(op, L)) || (rc = check_ptr(psi, "psi"))) return rc;
  if (!std::isfinite(theta)) return set_error(FOCK_ERR_NONFINITE, "theta is not finite");
  fock_ham_t ham;
  memset(&ham, 0, sizeof(ham));
  ham.L = L;
  ham.d = d;
  Ctx c;
  rc = make_ctx(ham, namp, 0, 1, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  rc = stage_gates(c, &op, &theta, 1, nullptr);
  if (rc) return rc;
  return forward_gate(c, op, 0, adjoint != 0, (const float2 *)psi, (float2 *)psi);
}

int fock_pool_grads(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi, const void *hpsi,
                    double *grads, void *ws, size_t ws_bytes, fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp);
  if (rc) return rc;
  if (P < 0 || P > 4096) return set_error(FOCK_ERR_ARG, "P=%d out of range", P);
  if (P == 0) return FOCK_OK;
  if (!pool || !grads) return set_error(FOCK_ERR_ARG, "pool/grads is NULL");
  if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(hpsi, "hpsi"))) return rc;
  for (int k = 0; k < P; ++k)
    if ((rc = check_op(pool[k], ham->L))) return rc;
  Ctx c;
  rc = make_ctx(*ham, namp, P, 0, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  rc = pool_dev(c, pool, P, (const float2 *)psi, (const float2 *)hpsi, (double *)(c.ws + c.L.result));
  if (rc) return rc;
  return fetch_results(c, P, grads);
}

int fock_energy_grad_adjoint(const fock_ham_t *ham, const fock_op_t *ops, const double *theta, int n,
                             const void *psi0, void *psi_work, void *lam_work, double *E, double *norm2,
                             double *dEdtheta, void *ws, size_t ws_bytes, fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp, true);
  if (rc) return rc;
  if (n < 0 || n > 4096) return set_error(FOCK_ERR_ARG, "n=%d out of range", n);
  if (n > 0 && (!ops || !theta)) return set_error(FOCK_ERR_ARG, "ops/theta is NULL");
  if (!E) return set_error(FOCK_ERR_ARG, "E is NULL");
  if ((rc = check_ptr(psi0, "psi0")) || (rc = check_ptr(psi_work, "psi_work")) ||
      (rc = check_ptr(lam_work, "lam_work")))
    return rc;
  if (psi_work == lam_work || psi_work == psi0 || lam_work == psi0)
    return set_error(FOCK_ERR_ARG, "psi0, psi_work and lam_work must be distinct");
  for (int k = 0; k < n; ++k)
    if ((rc = check_op(ops[k], ham->L))) return rc;
  Ctx c;
  rc = make_ctx(*ham, namp, 0, n, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  if (ham->layout & FOCK_LAYOUT_REAL) {
    // float32 states: psi0, psi_work and lam_work are the real-state buffers
    c.psi0_r = (float *)const_cast<void *>(psi0);
    c.phi_r = (float *)psi_work;
    c.lam_r = (float *)lam_work;
    if (!real_eval(c, ops, n))
      return set_error(FOCK_ERR_UNSUPPORTED, "real states take HR and PR gates only");
    if (!c.h.slab)  // the real H psi is the slab one; no complex copy fits these buffers
      return set_error(FOCK_ERR_UNSUPPORTED, "real states need the slab stencil with the one-pass schedule");
  }
  return run_circuit(c, ops, theta, n, psi0, (float2 *)psi_work, (float2 *)lam_work, dEdtheta != nullptr, E, norm2,
                     dEdtheta);
}

int fock_real_fusion_plan(const fock_ham_t *ham, const fock_op_t *ops, int n, int *run_k0, int *run_a,
                          int *nruns) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp, true);
  if (rc) return rc;
  if (n < 0 || n > 4096) return set_error(FOCK_ERR_ARG, "n=%d out of range", n);
  if (n > 0 && (!ops || !run_k0 || !run_a)) return set_error(FOCK_ERR_ARG, "ops/run_k0/run_a is NULL");
  if (!nruns) return set_error(FOCK_ERR_ARG, "nruns is NULL");
  for (int k = 0; k < n; ++k) {
    if ((rc = check_op(ops[k], ham->L))) return rc;
    if (ops[k].type != FOCK_HR && ops[k].type != FOCK_PR)
      return set_error(FOCK_ERR_UNSUPPORTED, "real states take HR and PR gates only (gate %d)", k);
  }
  Geometry g{ham->L, ham->d, namp};
  g.half = (ham->layout & 3) != FOCK_LAYOUT_FULL ? 1 : 0;
  const std::vector<RealRun> runs = plan_real_runs(g, ops, n);
  for (size_t r = 0; r < runs.size(); ++r) {
    run_k0[r] = runs[r].k0;
    run_a[r] = runs[r].a;
  }
  *nruns = (int)runs.size();
  return FOCK_OK;
}

int fock_score(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi, void *hpsi, double *E,
               double *norm2, double *grads, void *ws, size_t ws_bytes, fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp);
  if (rc) return rc;
  if (P < 1 || P > 4096) return set_error(FOCK_ERR_ARG, "P=%d out of range", P);
  if (!pool || !grads) return set_error(FOCK_ERR_ARG, "pool/grads is NULL");
  if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(hpsi, "hpsi"))) return rc;
  if (psi == hpsi) return set_error(FOCK_ERR_ARG, "psi and hpsi must not overlap");
  for (int k = 0; k < P; ++k)
    if ((rc = check_op(pool[k], ham->L))) return rc;
  Ctx c;
  rc = make_ctx(*ham, namp, P, 0, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  for (int k = 0; k < P; ++k)
    if (is_squeeze(pool[k].type) && c.T.d != c.g.d) {  // squeezer scoring reads the generator table
      rc = get_tables(c.g.d, &c.T);
      if (rc) return rc;
      break;
    }
  double *res = (double *)(c.ws + c.L.result);
  rc = score_dev(c, pool, P, (const float2 *)psi, (float2 *)hpsi, res);
  if (rc) return rc;
  std::vector<double> host(2 + P);
  rc = fetch_results(c, 2 + P, host.data());
  if (rc) return rc;
  if (E) *E = host[0];
  if (norm2) *norm2 = host[1];
  for (int k = 0; k < P; ++k) grads[k] = host[2 + k];
  return FOCK_OK;
}

int fock_set_state_store(int mode) {
  if (mode != FOCK_STORE_OFF && mode != FOCK_STORE_ON && mode != FOCK_STORE_AUTO)
    return set_error(FOCK_ERR_ARG, "state store mode %d is not OFF (0), ON (1) or AUTO (2)", mode);
  g_state_store.store(mode);
  return FOCK_OK;
}

int fock_get_state_store(void) { return g_state_store.load(); }

int fock_set_sector_layout(int mode) {
  if (mode != FOCK_SECTOR_OFF && mode != FOCK_SECTOR_AUTO)
    return set_error(FOCK_ERR_ARG, "sector layout mode %d is not OFF (0) or AUTO (1)", mode);
  g_sector_layout.store(mode);
  return FOCK_OK;
}

int fock_get_sector_layout(void) { return g_sector_layout.load(); }

int fock_set_real_states(int mode) {
  if (mode != FOCK_REAL_OFF && mode != FOCK_REAL_AUTO)
    return set_error(FOCK_ERR_ARG, "real-state mode %d is not OFF (0) or AUTO (1)", mode);
  g_real_states.store(mode);
  return FOCK_OK;
}

int fock_get_real_states(void) { return g_real_states.load(); }

int fock_set_real_fusion(int mode) {
  if (mode != FOCK_RFUSE_OFF && mode != FOCK_RFUSE_ON)
    return set_error(FOCK_ERR_ARG, "real fusion mode %d is not OFF (0) or ON (1)", mode);
  g_real_fusion.store(mode);
  return FOCK_OK;
}

int fock_get_real_fusion(void) { return g_real_fusion.load(); }

static int sector_convert(int L, int d, int layout, const void *src, void *dst, bool to_half, fock_stream_t stream) {
  if (d != 8) return set_error(FOCK_ERR_UNSUPPORTED, "the parity-halved layout needs d = 8 (d=%d)", d);
  if (layout != FOCK_LAYOUT_EVEN && layout != FOCK_LAYOUT_ODD)
    return set_error(FOCK_ERR_ARG, "layout %d is not EVEN (1) or ODD (2)", layout);
  int rc;
  if ((rc = check_ptr(src, "src")) || (rc = check_ptr(dst, "dst"))) return rc;
  if (src == dst) return set_error(FOCK_ERR_ARG, "src and dst must not overlap");
  return launch_sector_convert(L, layout == FOCK_LAYOUT_ODD ? 1 : 0, to_half, (const float2 *)src, (float2 *)dst,
                               (hipStream_t)stream);
}

int fock_sector_pack(int L, int d, int layout, const void *full, void *half, fock_stream_t stream) {
  return sector_convert(L, d, layout, full, half, true, stream);
}

int fock_sector_unpack(int L, int d, int layout, const void *half, void *full, fock_stream_t stream) {
  return sector_convert(L, d, layout, half, full, false, stream);
}

int fock_adjoint_sweep(const fock_ham_t *ham, const fock_op_t *ops, const double *theta, int n, void *psi_work,
                       void *lam_work, double norm2, double *dEdtheta, void *ws, size_t ws_bytes,
                       fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham_layout(ham, &namp);
  if (rc) return rc;
  if (n < 0 || n > 4096) return set_error(FOCK_ERR_ARG, "n=%d out of range", n);
  if (n > 0 && (!ops || !theta || !dEdtheta)) return set_error(FOCK_ERR_ARG, "ops/theta/dEdtheta is NULL");
  if ((rc = check_ptr(psi_work, "psi_work")) || (rc = check_ptr(lam_work, "lam_work"))) return rc;
  if (psi_work == lam_work) return set_error(FOCK_ERR_ARG, "psi_work and lam_work must be distinct");
  if (!(norm2 > 0.0) || !std::isfinite(norm2)) return set_error(FOCK_ERR_ARG, "norm2 must be finite and > 0");
  for (int k = 0; k < n; ++k)
    if ((rc = check_op(ops[k], ham->L))) return rc;
  Ctx c;
  rc = make_ctx(*ham, namp, 0, n, ws, ws_bytes, (hipStream_t)stream, &c);
  if (rc) return rc;
  return run_reverse(c, ops, theta, n, (float2 *)psi_work, (float2 *)lam_work, norm2, dEdtheta);
}

}  // extern "C"
