// CV-ADAPT-VQE (Sec. IV.B) on complex128 states: the same loop as adapt_step
// (pool scoring, tie band, append at theta = 0, BFGS re-optimisation with the
// L-inf tolerance and optional Hessian recycling), with every evaluation on
// the FP64 kernels of f64_kernels.hip.  For the small lattices whose runs
// must resolve energy differences far below the complex64 state's rounding.
//
// Two-parameter gates (Sec. II.B; FOCK_BS, FOCK_TMS, FOCK_SQ): the phase phi of
// the beam splitter, two-mode squeezer and squeezer is a conjugation by phase
// rotations R(a) = exp(i a N) of the phi = 0 gate,
//   BS(theta, phi)  = R_j(phi) exp(-theta HR) R_j(-phi)
//   TMS(theta, phi) = R_j(-phi) exp(theta PR) R_j(phi)
//   SQ(theta, phi)  = R_i(phi/2) exp(theta SR) R_i(-phi/2),
// so each expands to three gates with tied angles; dE/dtheta and dE/dphi
// follow by the chain rule from the three gates' adjoint gradients.  They are
// scored by |dE/dtheta| at theta = phi = 0 (dE/dphi vanishes there, Sec. IV.B)
// and enter the ansatz at (0, 0).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "bfgs.h"
#include "f64_internal.h"
#include "pipeline.h"

struct fock_adapt64 {
  fock::H64 h;
  int L = 0, d = 0;
  uint32_t namp = 0;
  std::vector<fock_op_t> pool, ops;  // ops: the ansatz's logical ops (two-parameter ones unexpanded)
  std::vector<double> theta, Hinv;   // theta: logical parameters (two per two-parameter op)
  std::vector<fock_op_t> gops;       // gates of the last evaluation
  std::vector<fock_op_t> rec_ops;    // gates whose records are on the device (recs)
  fock_adapt_opts_t opt;
  hipStream_t s = nullptr;
  fock::EigTables T;
  int cap = 0, Mmax = 0;  // gate capacity, largest local dimension
  // device buffers
  double2 *psi0 = nullptr, *phi = nullptr, *lam = nullptr, *utab = nullptr;
  double *partial = nullptr, *res = nullptr, *th_dev = nullptr;
  fock::GateRec *recs = nullptr;
  std::map<int, double2 *> A;  // dense generator per type
  int maxblk = 0;
  int iter = 0;
  bool done = false;
  fock_adapt_report_t warm{};  // warm-up optimisation done at creation (iter 0)
};

namespace fock {
namespace {

bool two_param(int t) { return t == FOCK_BS || t == FOCK_TMS || t == FOCK_SQ; }
int fixed_type(int t) { return t == FOCK_BS ? FOCK_HR : t == FOCK_TMS ? FOCK_PR : t == FOCK_SQ ? FOCK_SR : t; }
int local_dim(int d, int type) { return is_single_mode(fixed_type(type)) ? d : d * d; }

// Logical ansatz (ops, x) -> gates and gate angles.
void expand(const std::vector<fock_op_t> &lops, const std::vector<double> &x, std::vector<fock_op_t> *g,
            std::vector<double> *a) {
  g->clear();
  a->clear();
  size_t p = 0;
  for (const fock_op_t &op : lops) {
    if (!two_param(op.type)) {
      g->push_back(op);
      a->push_back(x[p++]);
      continue;
    }
    const double th = x[p], ph = x[p + 1];
    p += 2;
    const fock_op_t rot{FOCK_ROT, op.type == FOCK_SQ ? op.i : op.j, -1};
    const fock_op_t fix{fixed_type(op.type), op.i, op.type == FOCK_SQ ? -1 : op.j};
    const double r1 = op.type == FOCK_BS ? -ph : op.type == FOCK_TMS ? ph : -0.5 * ph;
    const double c = op.type == FOCK_BS ? -1.0 : 1.0;
    g->push_back(rot);
    a->push_back(r1);
    g->push_back(fix);
    a->push_back(c * th);
    g->push_back(rot);
    a->push_back(-r1);
  }
}

// Gate gradients -> logical gradients (chain rule through expand).
void contract(const std::vector<fock_op_t> &lops, const std::vector<double> &gg, std::vector<double> *gx) {
  gx->clear();
  size_t q = 0;
  for (const fock_op_t &op : lops) {
    if (!two_param(op.type)) {
      gx->push_back(gg[q++]);
      continue;
    }
    const double g1 = gg[q], g2 = gg[q + 1], g3 = gg[q + 2];
    q += 3;
    if (op.type == FOCK_BS) {
      gx->push_back(-g2);
      gx->push_back(g3 - g1);
    } else if (op.type == FOCK_TMS) {
      gx->push_back(g2);
      gx->push_back(g1 - g3);
    } else {
      gx->push_back(g2);
      gx->push_back(0.5 * (g3 - g1));
    }
  }
}

int generator64(fock_adapt64 *st, int type, const double2 **out) {
  auto it = st->A.find(type);
  if (it == st->A.end()) {
    std::vector<double> m;
    generator_dense(type, st->d, m);
    double2 *p = nullptr;
    FOCK_HIP(hipMalloc(&p, sizeof(double2) * m.size() / 2));
    FOCK_HIP(hipMemcpy(p, m.data(), sizeof(double) * m.size(), hipMemcpyHostToDevice));
    it = st->A.emplace(type, p).first;
  }
  *out = it->second;
  return FOCK_OK;
}

int fetch(fock_adapt64 *st, int n, double *host) {
  FOCK_HIP(hipMemcpyAsync(host, st->res, sizeof(double) * n, hipMemcpyDeviceToHost, st->s));
  FOCK_HIP(hipStreamSynchronize(st->s));
  return FOCK_OK;
}

// E (Rayleigh quotient), <psi|psi>, and the gate gradients when g != nullptr,
// for the gates st->gops at angles th.  Leaves phi = psi and lam = H psi when
// no gradient is asked for.
int eval_gates(fock_adapt64 *st, const std::vector<double> &th, double *E, double *n2, std::vector<double> *g) {
  const int n = (int)st->gops.size();
  if (n > st->cap) return set_error(FOCK_ERR_SIZE, "more gates (%d) than the run's capacity (%d)", n, st->cap);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(th[k])) return set_error(FOCK_ERR_NONFINITE, "theta[%d] is not finite", k);
  if (n > 0) {
    // gate records (table offset, reverse-step workgroups) change only with the gate list
    bool same = st->rec_ops.size() == st->gops.size();
    for (int k = 0; same && k < n; ++k)
      same = st->rec_ops[k].type == st->gops[k].type && st->rec_ops[k].i == st->gops[k].i &&
             st->rec_ops[k].j == st->gops[k].j;
    if (!same) {
      std::vector<GateRec> rec(n);
      for (int k = 0; k < n; ++k)
        rec[k] = GateRec{st->gops[k].type, k * st->Mmax * st->Mmax,
                         fib64_blocks(make_fib64(st->L, st->d, st->gops[k])), 0};
      FOCK_HIP(hipMemcpyAsync(st->recs, rec.data(), sizeof(GateRec) * n, hipMemcpyHostToDevice, st->s));
      st->rec_ops = st->gops;
    }
    FOCK_HIP(hipMemcpyAsync(st->th_dev, th.data(), sizeof(double) * n, hipMemcpyHostToDevice, st->s));
    int rc = launch64_build(st->th_dev, st->recs, n, st->T, st->Mmax, st->utab, st->s);
    if (rc) return rc;
  } else {
    FOCK_HIP(hipMemcpyAsync(st->phi, st->psi0, sizeof(double2) * st->namp, hipMemcpyDeviceToDevice, st->s));
  }
  for (int k = 0; k < n; ++k) {  // the first gate reads psi0 and writes phi
    const Fib64 a = make_fib64(st->L, st->d, st->gops[k]);
    int rc = launch64_fib_apply(a, k == 0 ? st->psi0 : st->phi, st->phi,
                                st->utab + (size_t)k * st->Mmax * st->Mmax, false, st->s);
    if (rc) return rc;
  }
  int G = 0;
  int rc = launch64_apply_h(st->h, st->phi, st->lam, st->partial, &G, st->s);
  if (rc) return rc;
  rc = launch_reduce(st->partial, G, 2, st->res, st->s);
  if (rc) return rc;
  if (g) {
    for (int k = n - 1; k >= 0; --k) {
      const Fib64 a = make_fib64(st->L, st->d, st->gops[k]);
      const double2 *A = nullptr;
      rc = generator64(st, st->gops[k].type, &A);
      if (rc) return rc;
      double *pk = st->partial + (size_t)(2 + k) * st->maxblk;
      rc = launch64_fib_adj(a, st->phi, st->lam, st->utab + (size_t)k * st->Mmax * st->Mmax, A, pk, st->s);
      if (rc) return rc;
    }
    // one launch sums every gate's row of partials (nblk of its record)
    rc = launch_reduce_rows(st->partial + (size_t)2 * st->maxblk, st->maxblk, st->recs, n, st->res + 2, st->s);
    if (rc) return rc;
  }
  std::vector<double> host(2 + (g ? n : 0));
  rc = fetch(st, (int)host.size(), host.data());
  if (rc) return rc;
  if (!std::isfinite(host[0]) || !(host[1] > 0.0))
    return set_error(FOCK_ERR_NONFINITE, "non-finite energy or zero norm (E=%g, norm2=%g)", host[0], host[1]);
  *E = host[0] / host[1];
  if (n2) *n2 = host[1];
  if (g) {
    g->resize(n);
    for (int k = 0; k < n; ++k) (*g)[k] = 2.0 * host[2 + k] / host[1];
  }
  return FOCK_OK;
}

// E, <psi|psi> and the logical gradient of the ansatz ops at logical parameters x.
int eval64(fock_adapt64 *st, const std::vector<fock_op_t> &lops, const std::vector<double> &x, double *E, double *n2,
           std::vector<double> *gx) {
  std::vector<double> a, gg;
  expand(lops, x, &st->gops, &a);
  int rc = eval_gates(st, a, E, n2, gx ? &gg : nullptr);
  if (rc || !gx) return rc;
  contract(lops, gg, gx);
  return FOCK_OK;
}

// 2 Re<H psi|A_k psi> for the whole pool on phi = psi, lam = H psi (the phi = 0
// generator of a two-parameter entry, with its sign in the expansion).
int pool64(fock_adapt64 *st, std::vector<double> *g) {
  const int P = (int)st->pool.size();
  for (int k = 0; k < P; ++k) {
    fock_op_t op = st->pool[k];
    if (op.type == FOCK_SQ) op.j = -1;
    op.type = fixed_type(op.type);
    const Fib64 a = make_fib64(st->L, st->d, op);
    const double2 *A = nullptr;
    int rc = generator64(st, op.type, &A);
    if (rc) return rc;
    double *pk = st->partial + (size_t)k * st->maxblk;
    rc = launch64_fib_pool(a, st->phi, st->lam, A, pk, st->s);
    if (rc) return rc;
    rc = launch_reduce(pk, fib64_blocks(a), 1, st->res + k, st->s);
    if (rc) return rc;
  }
  g->resize(P);
  int rc = fetch(st, P, g->data());
  if (rc) return rc;
  for (int k = 0; k < P; ++k)
    if (st->pool[k].type == FOCK_BS) (*g)[k] = -(*g)[k];
  return FOCK_OK;
}

void release(fock_adapt64 *st) {
  if (st->s) (void)hipStreamSynchronize(st->s);
  for (void *p : {(void *)st->psi0, (void *)st->phi, (void *)st->lam, (void *)st->utab, (void *)st->partial,
                  (void *)st->res, (void *)st->th_dev, (void *)st->recs})
    if (p) (void)hipFree(p);
  for (auto &kv : st->A) (void)hipFree(kv.second);
  if (st->s) (void)hipStreamDestroy(st->s);
}

}  // namespace
}  // namespace fock

using namespace fock;

extern "C" {

int adapt64_create(const fock_ham_t *ham, const fock_op_t *pool, int P, const void *psi0,
                   const fock_adapt_opts_t *opts, fock_stream_t stream, fock_adapt64_t **out) {
  if (!out) return set_error(FOCK_ERR_ARG, "out is NULL");
  *out = nullptr;
  uint32_t namp = 0;
  int rc = check_ham(ham, &namp);
  if (rc) return rc;
  if (!pool || P < 1 || P > 4096) return set_error(FOCK_ERR_ARG, "pool must hold 1..4096 ops");
  for (int k = 0; k < P; ++k) {
    const fock_op_t &op = pool[k];
    if (two_param(op.type)) {
      fock_op_t f = op;
      f.type = fixed_type(op.type);
      if (op.type == FOCK_SQ) f.j = -1;
      if ((rc = check_op(f, ham->L))) return rc;
    } else if ((rc = check_op(op, ham->L))) {
      return rc;
    }
  }
  if ((rc = check_ptr(psi0, "psi0"))) return rc;
  fock_adapt_opts_t o;
  adapt_default_opts(&o);
  if (opts) o = *opts;
  if (o.n_warm < 0 || o.n_warm > 4096 || (o.n_warm > 0 && (!o.warm_ops || !o.warm_theta0)))
    return set_error(FOCK_ERR_ARG, "warm-up layer arrays missing or too long");
  for (int k = 0; k < o.n_warm; ++k)  // one-parameter generators only (check_op refuses BS, TMS, SQ)
    if ((rc = check_op(o.warm_ops[k], ham->L))) return rc;
  if (o.grad_mode != 0) return set_error(FOCK_ERR_UNSUPPORTED, "the FP64 driver uses adjoint gradients only");
  if (o.max_iters < 0 || o.max_iters > 4000) return set_error(FOCK_ERR_ARG, "max_iters out of range");
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return set_error(FOCK_ERR_HIP, "caller stream error");
  fock_adapt64 *st = new fock_adapt64();
  st->L = ham->L;
  st->d = ham->d;
  st->namp = namp;
  st->h = H64{ham->L, ham->d, (ham->periodic && ham->L >= 3) ? 1 : 0, namp, ham->J, ham->Delta,
              0.5 * ham->U + ham->K, ham->mu};
  st->pool.assign(pool, pool + P);
  st->opt = o;
  st->opt.warm_ops = nullptr;
  st->opt.warm_theta0 = nullptr;
  for (int k = 0; k < o.n_warm; ++k) {  // the warm-up layer leads the ansatz and is re-optimised every step
    st->ops.push_back(o.warm_ops[k]);
    st->theta.push_back(o.warm_theta0[k]);
  }
  st->cap = o.n_warm + 3 * (o.max_iters + 1);  // gates: a two-parameter op expands to three
  st->Mmax = 0;
  for (int k = 0; k < P; ++k) st->Mmax = std::max(st->Mmax, local_dim(ham->d, pool[k].type));
  for (int k = 0; k < o.n_warm; ++k) st->Mmax = std::max(st->Mmax, local_dim(ham->d, o.warm_ops[k].type));
  // partial rows: the most workgroups of any launch (H psi, or fibres of d or d^2 amplitudes)
  st->maxblk = (int)((namp + kBlock - 1) / kBlock);
  for (int M : {ham->d, ham->d * ham->d}) {
    const uint32_t fpw = (uint32_t)std::max(1, kBlock / M), nf = namp / (uint32_t)M;
    st->maxblk = std::max(st->maxblk, (int)((nf + fpw - 1) / fpw));
  }
  const int rows = std::max(2 + st->cap, P) + 2;
  auto fail = [&](int code) {
    release(st);
    delete st;
    return code;
  };
  if (hipStreamCreateWithFlags(&st->s, hipStreamNonBlocking) != hipSuccess)
    return fail(set_error(FOCK_ERR_HIP, "stream creation failed"));
  const size_t bs = sizeof(double2) * namp;
  if (hipMalloc(&st->psi0, bs) != hipSuccess || hipMalloc(&st->phi, bs) != hipSuccess ||
      hipMalloc(&st->lam, bs) != hipSuccess ||
      hipMalloc(&st->utab, sizeof(double2) * (size_t)st->cap * st->Mmax * st->Mmax) != hipSuccess ||
      hipMalloc(&st->partial, sizeof(double) * (size_t)rows * st->maxblk) != hipSuccess ||
      hipMalloc(&st->res, sizeof(double) * rows) != hipSuccess ||
      hipMalloc(&st->th_dev, sizeof(double) * st->cap) != hipSuccess ||
      hipMalloc(&st->recs, sizeof(GateRec) * st->cap) != hipSuccess)
    return fail(set_error(FOCK_ERR_HIP, "device allocation failed"));
  // On the handle's own (non-blocking) stream, so that every later kernel is
  // ordered after it; the evaluation below synchronises that stream before
  // create returns, after which the caller may release psi0.
  if (hipMemcpyAsync(st->psi0, psi0, bs, hipMemcpyDeviceToDevice, st->s) != hipSuccess)
    return fail(set_error(FOCK_ERR_HIP, "copy of psi0 failed"));
  if ((rc = get_tables(ham->d, &st->T))) return fail(rc);
  st->warm.iter = 0;
  st->warm.k_sel = -1;
  double E0 = 0.0, n2 = 0.0;
  if ((rc = eval64(st, st->ops, st->theta, &E0, &n2, nullptr))) return fail(rc);
  st->warm.E = st->warm.E_init = E0;
  st->warm.norm2 = n2;
  st->warm.n_params = (int)st->theta.size();
  if (o.n_warm > 0 && !o.warm_fixed) {
    const double gtol = std::max(o.warm_gtol, o.gtol_floor_rel * std::max(1.0, std::fabs(E0)));
    ObjFn fn = [st](const std::vector<double> &x, double *f, std::vector<double> *gx) {
      return eval64(st, st->ops, x, f, nullptr, gx);
    };
    BfgsOut bo;
    if ((rc = bfgs_minimize(st->theta, fn, gtol, o.bfgs_maxiter, nullptr, &bo, 0.0))) return fail(rc);
    if ((rc = eval64(st, st->ops, st->theta, &E0, &n2, nullptr))) return fail(rc);
    st->warm.bfgs_iters = bo.iters;
    st->warm.bfgs_evals = bo.evals + 1;
    st->warm.status = bo.status;
    st->warm.E = E0;
    st->warm.E_init = bo.f0;
    st->warm.norm2 = n2;
  }
  *out = st;
  return FOCK_OK;
}

int adapt64_warm_report(fock_adapt64_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  *rep = st->warm;
  return FOCK_OK;
}

int adapt64_step(fock_adapt64_t *st, fock_adapt_report_t *rep) {
  if (!st || !rep) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (st->done) return set_error(FOCK_ERR_STATE, "ADAPT run already finished");
  memset(rep, 0, sizeof(*rep));
  st->iter += 1;
  rep->iter = st->iter;
  rep->k_sel = -1;
  double E = 0.0, n2 = 0.0;
  int rc = eval64(st, st->ops, st->theta, &E, &n2, nullptr);
  if (rc) return rc;
  std::vector<double> g;
  rc = pool64(st, &g);
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
  rep->E = rep->E_init = E;
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
  int ks = 0;
  for (int k = 0; k < (int)g.size(); ++k)
    if (std::fabs(g[k]) >= (1.0 - st->opt.tie_tau) * ginf) {
      ks = k;
      break;
    }
  rep->k_sel = ks;
  rep->g_sel = std::fabs(g[ks]);
  st->ops.push_back(st->pool[ks]);
  if (st->ops.back().type == FOCK_SQ) st->ops.back().j = -1;
  const int added = two_param(st->pool[ks].type) ? 2 : 1;
  for (int k = 0; k < added; ++k) st->theta.push_back(0.0);
  const int n = (int)st->theta.size();
  // BFGS runs over the free angles: all but a fixed warm-up layer's
  const int nf = st->opt.warm_fixed ? st->opt.n_warm : 0, nx = n - nf;
  std::vector<double> *H = nullptr;
  if (st->opt.recycle_hessian) {
    const int m = (int)std::lround(std::sqrt((double)st->Hinv.size()));
    std::vector<double> Hn((size_t)nx * nx, 0.0);
    for (int r = 0; r < nx; ++r) Hn[(size_t)r * nx + r] = 1.0;
    if (m == nx - added)
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) Hn[(size_t)r * nx + c] = st->Hinv[(size_t)r * m + c];
    st->Hinv.swap(Hn);
    H = &st->Hinv;
  }
  const double gtol = std::max(std::min(1e-6, 1e-5 * rep->g_sel), st->opt.gtol_floor_rel * std::max(1.0, std::fabs(E)));
  ObjFn fn = [st, nf](const std::vector<double> &x, double *f, std::vector<double> *gx) {
    if (nf == 0) return eval64(st, st->ops, x, f, nullptr, gx);
    std::vector<double> full(st->theta.begin(), st->theta.begin() + nf), g;
    full.insert(full.end(), x.begin(), x.end());
    const int r = eval64(st, st->ops, full, f, nullptr, gx ? &g : nullptr);
    if (!r && gx) gx->assign(g.begin() + nf, g.end());
    return r;
  };
  std::vector<double> x(st->theta.begin() + nf, st->theta.end());
  BfgsOut bo;
  rc = bfgs_minimize(x, fn, gtol, st->opt.bfgs_maxiter, H, &bo, 0.0);
  if (rc) return rc;
  std::copy(x.begin(), x.end(), st->theta.begin() + nf);
  double Ef = 0.0, n2f = 0.0;
  rc = eval64(st, st->ops, st->theta, &Ef, &n2f, nullptr);
  if (rc) return rc;
  rep->bfgs_iters = bo.iters;
  rep->bfgs_evals = bo.evals + 1;
  rep->status = bo.status;
  rep->E = Ef;
  rep->norm2 = n2f;
  rep->E_init = bo.f0;
  rep->n_params = n;
  return FOCK_OK;
}

int adapt64_get_ansatz(fock_adapt64_t *st, fock_op_t *ops, double *theta, int cap, int *n) {
  if (!st || !n) return set_error(FOCK_ERR_ARG, "NULL argument");
  std::vector<fock_op_t> g;
  std::vector<double> a;
  expand(st->ops, st->theta, &g, &a);
  *n = (int)g.size();
  const int m = std::min(cap, *n);
  for (int k = 0; k < m; ++k) {
    if (ops) ops[k] = g[k];
    if (theta) theta[k] = a[k];
  }
  return FOCK_OK;
}

int adapt64_energy_grad(fock_adapt64_t *st, const fock_op_t *ops, const double *theta, int n, double *E,
                        double *dEdtheta) {
  if (!st || !E || (n > 0 && (!ops || !theta))) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (n < 0 || n > st->cap) return set_error(FOCK_ERR_SIZE, "n = %d outside the run's capacity %d", n, st->cap);
  for (int k = 0; k < n; ++k) {
    int rc = check_op(ops[k], st->L);
    if (rc) return rc;
    if (local_dim(st->d, ops[k].type) > st->Mmax)
      return set_error(FOCK_ERR_ARG, "op %d needs a larger gate table than the pool's", k);
  }
  st->gops.assign(ops, ops + n);
  std::vector<double> th(theta, theta + n), g;
  const int rc = eval_gates(st, th, E, nullptr, dEdtheta ? &g : nullptr);
  if (rc) return rc;
  if (dEdtheta)
    for (int k = 0; k < n; ++k) dEdtheta[k] = g[k];
  return FOCK_OK;
}

int adapt64_destroy(fock_adapt64_t *st) {
  if (!st) return FOCK_OK;
  release(st);
  delete st;
  return FOCK_OK;
}

}  // extern "C"
