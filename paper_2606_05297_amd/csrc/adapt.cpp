// CV-ADAPT-VQE driver (Sec. IV.B, Sec. V.A) on top of the device pipeline:
// score the pool on the current state, test ||g||_2, select the largest
// |g_k| (lowest index inside a relative tie band), append exp(theta A_k) with
// theta = 0, and re-optimise all angles with BFGS (adjoint or finite-difference
// gradients).  An optional warm-up layer is optimised first and re-optimised
// with every later BFGS (Sec. IV.B, Appendix C).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bfgs.h"
#include "pipeline.h"

using namespace fock;

struct fock_adapt {
  fock_ham_t ham;
  uint32_t namp = 0;
  hipStream_t s = nullptr;
  fock_adapt_opts_t opt;
  std::vector<fock_op_t> pool;
  std::vector<fock_op_t> ops;
  std::vector<double> theta;
  std::vector<double> Hinv;
  void *dbuf = nullptr;
  float2 *psi0 = nullptr, *phi = nullptr, *lam = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Ctx ctx;
  int iter = 0;
  bool done = false;
  fock_adapt_report_t warm{};
  std::vector<double> proposal;
  bool has_prop = false;
  int prop_acc = 0;
  double prop_E = 0.0, plain_E = 0.0;
  // a step between adapt_step_select and adapt_step_finish
  bool pending = false;
  fock_adapt_report_t pend{};
  void *store_buf = nullptr;  // forward states of gradient evaluations (may be null)
  void *real_buf = nullptr;   // float32 psi0, phi, lam of real-state evaluations (may be null)
};

namespace {

// Total parity of a full d = 8 state: 0 or 1 when one of the two parity parts
// is exactly zero and the other is not, -1 otherwise.
int psi_sector(const void *psi, uint32_t namp, hipStream_t s, int *sector) {
  *sector = -1;
  const int G = sector_norms_blocks(namp);
  double *buf = nullptr;
  if (hipMalloc((void **)&buf, sizeof(double) * (2 * (size_t)G + 2)) != hipSuccess)
    return set_error(FOCK_ERR_HIP, "hipMalloc of the sector partials failed");
  double host[2] = {0.0, 0.0};
  int rc = launch_sector_norms((const float2 *)psi, namp, buf, s);
  if (!rc) rc = launch_reduce(buf, G, 2, buf + 2 * G, s);
  if (!rc && (hipMemcpyAsync(host, buf + 2 * G, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = set_error(FOCK_ERR_HIP, "sector norms of psi0 failed");
  (void)hipFree(buf);
  if (rc) return rc;
  if (host[1] == 0.0 && host[0] > 0.0) *sector = 0;
  else if (host[0] == 0.0 && host[1] > 0.0) *sector = 1;
  return FOCK_OK;
}

// Real-state buffers for st when switched on, d = 8 and every imaginary part of
// its (stored) psi0 is exactly zero; otherwise none.
int attach_real_states(fock_adapt *st) {
  if (real_states_mode() != FOCK_REAL_AUTO || st->ham.d != 8 || st->namp % 4 != 0) return FOCK_OK;
  unsigned int *flag = nullptr;
  if (hipMalloc((void **)&flag, sizeof(unsigned int)) != hipSuccess)
    return set_error(FOCK_ERR_HIP, "hipMalloc of the imaginary-part flag failed");
  unsigned int host = 1u;
  int rc = FOCK_OK;
  if (hipMemsetAsync(flag, 0, sizeof(unsigned int), st->s) != hipSuccess) rc = set_error(FOCK_ERR_HIP, "memset failed");
  if (!rc) rc = launch_imag_any(st->psi0, st->namp, flag, st->s);
  if (!rc && (hipMemcpyAsync(&host, flag, sizeof(host), hipMemcpyDeviceToHost, st->s) != hipSuccess ||
              hipStreamSynchronize(st->s) != hipSuccess))
    rc = set_error(FOCK_ERR_HIP, "imaginary-part check of psi0 failed");
  (void)hipFree(flag);
  if (rc || host != 0u) return rc;
  const size_t rb = (sizeof(float) * (size_t)st->namp + 255) & ~(size_t)255;
  if (hipMalloc(&st->real_buf, 3 * rb) != hipSuccess) {
    (void)hipGetLastError();
    st->real_buf = nullptr;
    return FOCK_OK;  // no room: complex evaluations only
  }
  char *b = (char *)st->real_buf;
  st->ctx.psi0_r = (float *)b;
  st->ctx.phi_r = (float *)(b + rb);
  st->ctx.lam_r = (float *)(b + 2 * rb);
  return launch_real_convert(st->namp, false, st->psi0, st->ctx.psi0_r, st->s);
}

int eval_energy(fock_adapt *st, const std::vector<double> &th, double *E, double *n2, std::vector<double> *g) {
  const int n = (int)st->ops.size();
  if (!g) return run_circuit(st->ctx, st->ops.data(), th.data(), n, st->psi0, st->phi, st->lam, false, E, n2, nullptr);
  g->assign(n, 0.0);
  if (st->opt.grad_mode == 0)
    return run_circuit(st->ctx, st->ops.data(), th.data(), n, st->psi0, st->phi, st->lam, true, E, n2, g->data());
  // plain method: central finite differences, 2n extra energy evaluations
  int rc = run_circuit(st->ctx, st->ops.data(), th.data(), n, st->psi0, st->phi, st->lam, false, E, n2, nullptr);
  if (rc) return rc;
  const double h = st->opt.fd_step;
  std::vector<double> t = th;
  for (int k = 0; k < n; ++k) {
    double ep = 0, em = 0;
    t[k] = th[k] + h;
    rc = run_circuit(st->ctx, st->ops.data(), t.data(), n, st->psi0, st->phi, st->lam, false, &ep, nullptr, nullptr);
    if (rc) return rc;
    t[k] = th[k] - h;
    rc = run_circuit(st->ctx, st->ops.data(), t.data(), n, st->psi0, st->phi, st->lam, false, &em, nullptr, nullptr);
    if (rc) return rc;
    t[k] = th[k];
    (*g)[k] = (ep - em) / (2.0 * h);
  }
  return FOCK_OK;
}

int optimise(fock_adapt *st, double gtol, fock_adapt_report_t *rep) {
  // every evaluation of this run, so that the energy and norm at the final
  // angles (always an evaluated point) are reported without evaluating again
  struct Seen {
    std::vector<double> x;
    double f, n2;
  };
  std::vector<Seen> seen;
  ObjFn fn = [st, &seen](const std::vector<double> &x, double *f, std::vector<double> *g) {
    double n2 = 0.0;
    const int rc = eval_energy(st, x, f, &n2, g);
    if (!rc) seen.push_back({x, *f, n2});
    return rc;
  };
  const int n = (int)st->theta.size();
  std::vector<double> *H = nullptr;
  if (st->opt.recycle_hessian) {
    // previous inverse Hessian padded with identity for the new angle (Appendix D)
    const int m = (int)std::lround(std::sqrt((double)st->Hinv.size()));
    if (m > 0 && m < n) {
      std::vector<double> Hn((size_t)n * n, 0.0);
      for (int r = 0; r < n; ++r) Hn[(size_t)r * n + r] = 1.0;
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) Hn[(size_t)r * n + c] = st->Hinv[(size_t)r * m + c];
      st->Hinv.swap(Hn);
    } else if (m != n) {
      st->Hinv.clear();
    }
    H = &st->Hinv;
  }
  BfgsOut bo;
  int rc = bfgs_minimize(st->theta, fn, gtol, st->opt.bfgs_maxiter, H, &bo, st->opt.noise_rel);
  if (rc) return rc;
  double E = 0.0, n2 = 0.0;
  const Seen *hit = nullptr;
  for (const Seen &e : seen)
    if (e.x == st->theta) hit = &e;
  if (hit) {
    E = hit->f;
    n2 = hit->n2;
  } else {
    rc = eval_energy(st, st->theta, &E, &n2, nullptr);
    if (rc) return rc;
  }
  rep->bfgs_iters = bo.iters;
  rep->bfgs_evals = bo.evals + (hit ? 0 : 1);
  rep->status = bo.status;
  rep->E = E;
  rep->norm2 = n2;
  rep->E_init = bo.f0;
  rep->n_params = n;
  return FOCK_OK;
}

double gtol_for(const fock_adapt *st, double gsel, double E) {
  const double paper = std::min(1e-6, 1e-5 * gsel);
  return std::max(paper, st->opt.gtol_floor_rel * std::max(1.0, std::fabs(E)));
}

}  // namespace

extern "C" {

void adapt_default_opts(fock_adapt_opts_t *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->max_iters = 60;
  o->bfgs_maxiter = 1000;
  o->grad_tol = 1e-3;
  o->tie_tau = 1e-4;
  o->gtol_floor_rel = 1e-5;
  o->warm_gtol = 1e-6;
  o->fd_step = 1e-3;
  o->noise_rel = 1e-7;
}

int adapt_create(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi0, const fock_adapt_opts_t *opts,
                 fock_stream_t stream, fock_adapt_t **out) {
  if (!out) return set_error(FOCK_ERR_ARG, "out is NULL");
  *out = nullptr;
  uint32_t namp = 0;
  int rc = check_ham(ham, &namp);
  if (rc) return rc;
  if (!opts) return set_error(FOCK_ERR_ARG, "opts is NULL");
  if (P < 1 || P > 4096 || !pool) return set_error(FOCK_ERR_ARG, "pool must hold 1..4096 ops");
  if ((rc = check_ptr(psi0, "psi0"))) return rc;
  for (int k = 0; k < P; ++k)
    if ((rc = check_op(pool[k], ham->L))) return rc;
  if (opts->warm_fixed != 0)
    return set_error(FOCK_ERR_UNSUPPORTED, "fixed warm-up angles are taken by the complex128 driver only");
  if (opts->n_warm < 0 || opts->n_warm > 4096 || (opts->n_warm > 0 && (!opts->warm_ops || !opts->warm_theta0)))
    return set_error(FOCK_ERR_ARG, "warm-up layer: 0..4096 ops with both arrays given");
  for (int k = 0; k < opts->n_warm; ++k)
    if ((rc = check_op(opts->warm_ops[k], ham->L))) return rc;
  if (opts->max_iters < 0 || opts->max_iters > 4000 || opts->bfgs_maxiter < 0 || !(opts->grad_tol >= 0.0))
    return set_error(FOCK_ERR_ARG, "invalid iteration caps (max_iters in 0..4000) or tolerance");
  if (opts->grad_mode == 1 && !(opts->fd_step > 0.0)) return set_error(FOCK_ERR_ARG, "fd_step must be > 0");

  if (ham->layout != FOCK_LAYOUT_FULL)
    return set_error(FOCK_ERR_ARG, "adapt_create takes a full d^L psi0 (layout 0); the driver picks its own layout");
  // A parity-definite psi0 under a parity-keeping pool stays in its sector:
  // the driver then keeps every state in the parity-halved layout.
  fock_ham_t hc = *ham;
  if (half_layout_wanted(*ham, pool, P, opts->warm_ops, opts->n_warm)) {
    int sector = -1;
    if ((rc = psi_sector(psi0, namp, (hipStream_t)stream, &sector))) return rc;
    if (sector >= 0) {
      hc.layout = sector ? FOCK_LAYOUT_ODD : FOCK_LAYOUT_EVEN;
      namp /= 2;
    }
  }

  fock_adapt *st = new fock_adapt();
  st->ham = hc;
  st->namp = namp;
  st->s = (hipStream_t)stream;
  st->opt = *opts;
  st->opt.warm_ops = nullptr;
  st->opt.warm_theta0 = nullptr;
  st->pool.assign(pool, pool + P);
  for (int k = 0; k < opts->n_warm; ++k) {
    st->ops.push_back(opts->warm_ops[k]);
    st->theta.push_back(opts->warm_theta0[k]);
  }
  const int nmax = opts->n_warm + opts->max_iters + 1;
  const Layout L = make_layout(namp, ham->L, ham->d, P, nmax, hc.layout != FOCK_LAYOUT_FULL);
  const size_t sbytes = (sizeof(float2) * (size_t)namp + 255) & ~(size_t)255;
  st->ws_bytes = L.total;
  if (hipMalloc(&st->dbuf, 3 * sbytes + st->ws_bytes) != hipSuccess) {
    delete st;
    return set_error(FOCK_ERR_HIP, "hipMalloc of %zu bytes failed", 3 * sbytes + L.total);
  }
  char *b = (char *)st->dbuf;
  st->psi0 = (float2 *)b;
  st->phi = (float2 *)(b + sbytes);
  st->lam = (float2 *)(b + 2 * sbytes);
  st->ws = b + 3 * sbytes;
  rc = make_ctx(hc, namp, P, nmax, st->ws, st->ws_bytes, st->s, &st->ctx);
  if (!rc) rc = attach_state_store(st->ctx, nmax, &st->store_buf);
  if (!rc && hc.layout != FOCK_LAYOUT_FULL)
    rc = launch_sector_convert(hc.L, st->ctx.g.sector, true, (const float2 *)psi0, st->psi0, st->s);
  else if (!rc && hipMemcpyAsync(st->psi0, psi0, sizeof(float2) * namp, hipMemcpyDeviceToDevice, st->s) != hipSuccess)
    rc = set_error(FOCK_ERR_HIP, "copy of psi0 failed");
  if (!rc) rc = attach_real_states(st);
  if (!rc) {
    st->warm.iter = 0;
    st->warm.k_sel = -1;
    if (opts->n_warm > 0) {
      double E0 = 0.0;
      rc = eval_energy(st, st->theta, &E0, nullptr, nullptr);
      if (!rc) rc = optimise(st, std::max(opts->warm_gtol, gtol_for(st, 0.0, E0)), &st->warm);
    } else {
      double E0 = 0.0, n2 = 0.0;
      rc = eval_energy(st, st->theta, &E0, &n2, nullptr);
      st->warm.E = E0;
      st->warm.E_init = E0;
      st->warm.norm2 = n2;
    }
  }
  if (rc) {
    (void)hipStreamSynchronize(st->s);
    (void)hipFree(st->dbuf);
    if (st->store_buf) (void)hipFree(st->store_buf);
    if (st->real_buf) (void)hipFree(st->real_buf);
    delete st;
    return rc;
  }
  st->Hinv.clear();
  *out = st;
  return FOCK_OK;
}

int adapt_warm_report(fock_adapt_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  *rep = st->warm;
  return FOCK_OK;
}

int adapt_step_select(fock_adapt_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (st->done) return set_error(FOCK_ERR_STATE, "ADAPT run already finished");
  if (st->pending) return set_error(FOCK_ERR_STATE, "a selected step awaits adapt_step_finish");
  memset(rep, 0, sizeof(*rep));
  st->iter += 1;
  rep->iter = st->iter;
  rep->k_sel = -1;
  // 1-2. state, energy and pool scoring at the current optimum (H psi and the
  // pool gradients from one fused pass where the pool allows it)
  double E = 0.0, n2 = 0.0;
  const int P = (int)st->pool.size();
  std::vector<double> g(P);
  int rc = run_score(st->ctx, st->ops.data(), st->theta.data(), (int)st->ops.size(), st->psi0, st->phi, st->lam,
                     st->pool.data(), P, &E, &n2, g.data());
  if (rc) return rc;
  double gn2 = 0.0, ginf = 0.0;
  for (auto &v : g) {
    v /= n2;
    gn2 += v * v;
    ginf = std::max(ginf, std::fabs(v));
  }
  gn2 = std::sqrt(gn2);
  rep->g_norm2 = gn2;
  rep->g_inf = ginf;
  rep->E = E;
  rep->E_init = E;
  rep->norm2 = n2;
  rep->n_params = (int)st->theta.size();
  if (gn2 < st->opt.grad_tol) {
    rep->converged = 1;
    st->done = true;
    return FOCK_OK;
  }
  if (st->iter > st->opt.max_iters) {
    rep->capped = 1;
    st->done = true;
    return FOCK_OK;
  }
  // 3. selection: lowest index inside the relative tie band
  int ks = 0;
  for (int k = 0; k < P; ++k)
    if (std::fabs(g[k]) >= (1.0 - st->opt.tie_tau) * ginf) {
      ks = k;
      break;
    }
  rep->k_sel = ks;
  rep->g_sel = std::fabs(g[ks]);
  // 4. append with theta = 0 (a proposal may replace the start in adapt_step_finish)
  st->ops.push_back(st->pool[ks]);
  st->theta.push_back(0.0);
  rep->n_params = (int)st->theta.size();
  st->pending = true;
  st->pend = *rep;
  return FOCK_OK;
}

int adapt_step_finish(fock_adapt_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (!st->pending) return set_error(FOCK_ERR_STATE, "no selected step (call adapt_step_select first)");
  st->pending = false;
  const fock_adapt_report_t sel = st->pend;
  const double E = sel.E;
  // 4b. start from {theta_prev, 0}, or from a proposal whose energy is not higher
  st->prop_acc = 0;
  st->plain_E = E;
  int rc = FOCK_OK;
  if (st->has_prop) {
    st->has_prop = false;
    if (st->proposal.size() == st->theta.size()) {
      double Ep = 0.0;
      rc = eval_energy(st, st->proposal, &Ep, nullptr, nullptr);
      if (rc) return rc;
      st->prop_E = Ep;
      if (Ep <= E) {
        st->theta = st->proposal;
        st->prop_acc = 1;
      }
    }
  }
  // 5. re-optimise all angles
  memset(rep, 0, sizeof(*rep));
  rc = optimise(st, gtol_for(st, sel.g_sel, E), rep);
  if (rc) return rc;
  rep->iter = sel.iter;
  rep->k_sel = sel.k_sel;
  rep->g_sel = sel.g_sel;
  rep->g_norm2 = sel.g_norm2;
  rep->g_inf = sel.g_inf;
  return FOCK_OK;
}

int adapt_step(fock_adapt_t *st, fock_adapt_report_t *rep) {
  int rc = adapt_step_select(st, rep);
  if (rc || rep->converged || rep->capped) return rc;
  return adapt_step_finish(st, rep);
}

int adapt_get_ansatz(fock_adapt_t *st, fock_op_t *ops, double *theta, int cap, int *n) {
  if (!st || !n) return set_error(FOCK_ERR_ARG, "NULL argument");
  *n = (int)st->ops.size();
  const int m = std::min(cap, *n);
  for (int k = 0; k < m; ++k) {
    if (ops) ops[k] = st->ops[k];
    if (theta) theta[k] = st->theta[k];
  }
  return FOCK_OK;
}

int adapt_propose(fock_adapt_t *st, const double *theta, int n) {
  if (!st || (!theta && n > 0)) return set_error(FOCK_ERR_ARG, "NULL argument");
  // before adapt_step_select the new angle is not appended yet; after it, it is
  const int want = (int)st->theta.size() + (st->pending ? 0 : 1);
  if (n != want) return set_error(FOCK_ERR_ARG, "proposal length %d != parameters of the step (%d)", n, want);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(theta[k])) return set_error(FOCK_ERR_NONFINITE, "proposal[%d] not finite", k);
  st->proposal.assign(theta, theta + n);
  st->has_prop = true;
  return FOCK_OK;
}

int adapt_last_proposal(fock_adapt_t *st, int *accepted, double *E_prop, double *E_plain) {
  if (!st) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (accepted) *accepted = st->prop_acc;
  if (E_prop) *E_prop = st->prop_E;
  if (E_plain) *E_plain = st->plain_E;
  return FOCK_OK;
}

int adapt_real(fock_adapt_t *st, int *real) {
  if (!st || !real) return set_error(FOCK_ERR_ARG, "NULL argument");
  *real = st->ctx.psi0_r != nullptr ? 1 : 0;
  return FOCK_OK;
}

int adapt_layout(fock_adapt_t *st, int *layout) {
  if (!st || !layout) return set_error(FOCK_ERR_ARG, "NULL argument");
  *layout = st->ham.layout;
  return FOCK_OK;
}

int adapt_state_store(fock_adapt_t *st, int *nstates) {
  if (!st || !nstates) return set_error(FOCK_ERR_ARG, "NULL argument");
  *nstates = st->ctx.nstore;
  return FOCK_OK;
}

int adapt_destroy(fock_adapt_t *st) {
  if (!st) return FOCK_OK;
  (void)hipStreamSynchronize(st->s);
  if (st->dbuf) (void)hipFree(st->dbuf);
  if (st->store_buf) (void)hipFree(st->store_buf);
  if (st->real_buf) (void)hipFree(st->real_buf);
  delete st;
  return FOCK_OK;
}

// Generic BFGS on a host objective (same minimiser the ADAPT driver uses).
int fock_bfgs_minimize(int n, double *x, fock_objective_fn fn, void *ctx, double gtol, int maxiter, double *Hinv,
                       int *iters, int *evals, double *fmin, int *status) {
  if (n < 1 || !x || !fn) return set_error(FOCK_ERR_ARG, "invalid BFGS arguments");
  std::vector<double> xv(x, x + n);
  ObjFn f = [fn, ctx](const std::vector<double> &xx, double *fx, std::vector<double> *gx) {
    gx->resize(xx.size());
    const int r = fn(ctx, (int)xx.size(), xx.data(), fx, gx->data());
    if (r) return set_error(r, "objective returned %d", r);
    return 0;
  };
  std::vector<double> H;
  if (Hinv) H.assign(Hinv, Hinv + (size_t)n * n);
  // an all-zero matrix means "no seed"
  bool seeded = false;
  for (double v : H) seeded |= v != 0.0;
  if (!seeded) H.clear();
  BfgsOut o;
  int rc = bfgs_minimize(xv, f, gtol, maxiter, Hinv ? &H : nullptr, &o);
  if (rc) return rc;
  std::copy(xv.begin(), xv.end(), x);
  if (Hinv) std::copy(H.begin(), H.end(), Hinv);
  if (iters) *iters = o.iters;
  if (evals) *evals = o.evals;
  if (fmin) *fmin = o.f;
  if (status) *status = o.status;
  return FOCK_OK;
}

}  // extern "C"
