// HVA-CV-VQE, the paper's fixed-structure baseline (Sec. IV.A, Eq.
// (HVA_ansatz)): P layers, each applying the exponentials of the
// Hamiltonian's own terms in a fixed order, grown one layer at a time.  Each
// new layer starts from caller-given angles (the paper draws them uniformly in
// [-0.05, 0.05]); the earlier layers start from their previous optimum, and
// BFGS re-optimises all angles (Sec. V.A: at most 1000 iterations, L-infinity
// gradient tolerance 1e-9, here with the complex64 noise floor of the ADAPT
// driver).  Energies and gradients come from the same device pipeline as
// adapt_step: forward gates, H psi, one adjoint sweep.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "bfgs.h"
#include "pipeline.h"

using namespace fock;

struct fock_hva {
  fock_ham_t ham;
  uint32_t namp = 0;
  hipStream_t s = nullptr;
  fock_adapt_opts_t opt;
  double gtol = 1e-9;
  int max_layers = 0;
  std::vector<fock_op_t> layer;
  std::vector<fock_op_t> ops;
  std::vector<double> theta;
  void *dbuf = nullptr;
  float2 *psi0 = nullptr, *phi = nullptr, *lam = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Ctx ctx;
  fock_adapt_report_t init{};
  void *store_buf = nullptr;  // forward states of gradient evaluations (may be null)
};

extern "C" {

int hva_create(const fock_ham_t *ham, const fock_op_t *layer, int n_layer, int max_layers, const void *psi0,
               const fock_adapt_opts_t *opts, double gtol, fock_stream_t stream, fock_hva_t **out) {
  if (!out) return set_error(FOCK_ERR_ARG, "out is NULL");
  *out = nullptr;
  uint32_t namp = 0;
  int rc = check_ham(ham, &namp);
  if (rc) return rc;
  if (!opts) return set_error(FOCK_ERR_ARG, "opts is NULL");
  if (!layer || n_layer < 1 || n_layer > 1024) return set_error(FOCK_ERR_ARG, "layer must hold 1..1024 ops");
  if (max_layers < 1 || (long)max_layers * n_layer > 4096)
    return set_error(FOCK_ERR_ARG, "max_layers * layer size must be in 1..4096");
  if (!(gtol > 0.0) || !std::isfinite(gtol)) return set_error(FOCK_ERR_ARG, "gtol must be finite and > 0");
  if (opts->bfgs_maxiter < 0) return set_error(FOCK_ERR_ARG, "invalid BFGS iteration cap");
  if ((rc = check_ptr(psi0, "psi0"))) return rc;
  for (int k = 0; k < n_layer; ++k)
    if ((rc = check_op(layer[k], ham->L))) return rc;
  fock_hva *st = new fock_hva();
  st->ham = *ham;
  st->namp = namp;
  st->s = (hipStream_t)stream;
  st->opt = *opts;
  st->opt.warm_ops = nullptr;
  st->opt.warm_theta0 = nullptr;
  st->gtol = gtol;
  st->max_layers = max_layers;
  st->layer.assign(layer, layer + n_layer);
  const int nmax = n_layer * max_layers;
  const Layout Lw = make_layout(namp, ham->L, ham->d, 0, nmax);
  const size_t sbytes = (sizeof(float2) * (size_t)namp + 255) & ~(size_t)255;
  st->ws_bytes = Lw.total;
  if (hipMalloc(&st->dbuf, 3 * sbytes + st->ws_bytes) != hipSuccess) {
    delete st;
    return set_error(FOCK_ERR_HIP, "hipMalloc of %zu bytes failed", 3 * sbytes + Lw.total);
  }
  char *b = (char *)st->dbuf;
  st->psi0 = (float2 *)b;
  st->phi = (float2 *)(b + sbytes);
  st->lam = (float2 *)(b + 2 * sbytes);
  st->ws = b + 3 * sbytes;
  rc = make_ctx(*ham, namp, 0, nmax, st->ws, st->ws_bytes, st->s, &st->ctx);
  if (!rc) rc = attach_state_store(st->ctx, nmax, &st->store_buf);
  if (!rc) {
    // the caller's psi0 must be complete before this stream copies it
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess ||
        hipMemcpyAsync(st->psi0, psi0, sizeof(float2) * namp, hipMemcpyDeviceToDevice, st->s) != hipSuccess)
      rc = set_error(FOCK_ERR_HIP, "copy of psi0 failed");
  }
  if (!rc) {
    double E = 0.0, n2 = 0.0;
    rc = run_circuit(st->ctx, nullptr, nullptr, 0, st->psi0, st->phi, st->lam, false, &E, &n2, nullptr);
    st->init.E = st->init.E_init = E;
    st->init.norm2 = n2;
    st->init.k_sel = -1;
  }
  if (rc) {
    (void)hipStreamSynchronize(st->s);
    (void)hipFree(st->dbuf);
    if (st->store_buf) (void)hipFree(st->store_buf);
    delete st;
    return rc;
  }
  *out = st;
  return FOCK_OK;
}

int hva_add_layer(fock_hva_t *st, const double *theta_new, fock_adapt_report_t *rep) {
  if (!st || !theta_new || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  const int nl = (int)st->layer.size();
  if ((int)st->ops.size() / nl >= st->max_layers)
    return set_error(FOCK_ERR_STATE, "already %d layers (the maximum)", st->max_layers);
  for (int k = 0; k < nl; ++k)
    if (!std::isfinite(theta_new[k])) return set_error(FOCK_ERR_NONFINITE, "theta_new[%d] not finite", k);
  memset(rep, 0, sizeof(*rep));
  st->ops.insert(st->ops.end(), st->layer.begin(), st->layer.end());
  st->theta.insert(st->theta.end(), theta_new, theta_new + nl);
  const int n = (int)st->theta.size();
  ObjFn fn = [st, n](const std::vector<double> &x, double *f, std::vector<double> *g) {
    g->assign(n, 0.0);
    return run_circuit(st->ctx, st->ops.data(), x.data(), n, st->psi0, st->phi, st->lam, true, f, nullptr,
                       g->data());
  };
  double E0 = 0.0;
  int rc = run_circuit(st->ctx, st->ops.data(), st->theta.data(), n, st->psi0, st->phi, st->lam, false, &E0, nullptr,
                       nullptr);
  if (rc) return rc;
  const double gtol = std::max(st->gtol, st->opt.gtol_floor_rel * std::max(1.0, std::fabs(E0)));
  BfgsOut bo;
  rc = bfgs_minimize(st->theta, fn, gtol, st->opt.bfgs_maxiter, nullptr, &bo, st->opt.noise_rel);
  if (rc) return rc;
  double E = 0.0, n2 = 0.0;
  rc = run_circuit(st->ctx, st->ops.data(), st->theta.data(), n, st->psi0, st->phi, st->lam, false, &E, &n2,
                   nullptr);
  if (rc) return rc;
  rep->iter = n / nl;
  rep->k_sel = -1;
  rep->status = bo.status;
  rep->bfgs_iters = bo.iters;
  rep->bfgs_evals = bo.evals + 2;
  rep->n_params = n;
  rep->g_inf = bo.ginf;
  rep->E = E;
  rep->norm2 = n2;
  rep->E_init = E0;
  return FOCK_OK;
}

int hva_initial_report(fock_hva_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  *rep = st->init;
  return FOCK_OK;
}

int hva_get_ansatz(fock_hva_t *st, fock_op_t *ops, double *theta, int cap, int *n) {
  if (!st || !n) return set_error(FOCK_ERR_ARG, "NULL argument");
  *n = (int)st->ops.size();
  const int m = std::min(cap, *n);
  for (int k = 0; k < m; ++k) {
    if (ops) ops[k] = st->ops[k];
    if (theta) theta[k] = st->theta[k];
  }
  return FOCK_OK;
}

int hva_destroy(fock_hva_t *st) {
  if (!st) return FOCK_OK;
  (void)hipStreamSynchronize(st->s);
  if (st->dbuf) (void)hipFree(st->dbuf);
  if (st->store_buf) (void)hipFree(st->store_buf);
  delete st;
  return FOCK_OK;
}

}  // extern "C"
