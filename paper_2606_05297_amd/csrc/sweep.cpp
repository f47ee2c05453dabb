// Batched sweep: CV-ADAPT-VQE (Sec. IV.B) on many Hamiltonian points of
// uneven (L, d) at once.  Every phase (forward gate layer k, H psi, reverse
// layer k, reductions, pool scoring) of all points runs as one batched launch
// per cutoff d; a whole energy+gradient evaluation round (angle upload, gate
// build, forward, H psi, reverse sweep, reductions, result download) is
// captured once per ADAPT iteration in a HIP graph and replayed for every
// lockstep BFGS round.  Each point keeps its own BFGS (Sec. V.A), run in a
// host thread whose objective calls are gathered into those rounds.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "bfgs.h"
#include "pipeline.h"
#include "sweep_internal.h"

using namespace fock;

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SPoint {
  fock_ham_t ham;
  Geometry g;
  HamArgs h;
  std::vector<fock_op_t> pool, ops;
  std::vector<double> theta;
  float2 *psi0 = nullptr, *phi = nullptr, *lam = nullptr;
  double *partial = nullptr, *res = nullptr;
  PoolPair *pairs = nullptr;
  PoolDiag *diags = nullptr;
  SweepPoolArgs pa;
  int G = 0, rs = 0, nmax = 0, P = 0, group = 0, gate_base = 0, res_off = 0;
  int GH = 0;  // workgroups (tiles) of H psi and pool scoring: apply_h_blocks()
  int iter = 0;
  bool done = false;
  fock_adapt_report_t warm{}, last{};
  // warm-start proposal for the next step (see fock_sweep_propose)
  std::vector<double> proposal;
  bool has_prop = false;
  int prop_acc = 0;
  double prop_E = 0.0, plain_E = 0.0;
  // lockstep BFGS
  bool want = false, finished = true;
  std::vector<double> x, grad;
  double f = 0.0, n2 = 0.0;
  int rc = 0;
};

struct DGroup {
  int d = 0;
  EigTables T;
  std::vector<int> pts;
  int ngates = 0;  // gate slots
  double *theta = nullptr;
  GateRec *recs = nullptr;
  float2 *utab = nullptr;
  size_t theta_off = 0;  // offset (doubles) of this group's angles in the upload block
};

}  // namespace

struct fock_sweep {
  std::vector<SPoint> pts;
  std::vector<DGroup> groups;
  fock_adapt_opts_t opt;
  hipStream_t s = nullptr;  // private non-blocking stream (graph capture needs one)
  void *dbuf = nullptr;
  int *active_d = nullptr;
  double *res_d = nullptr;
  double *up_d = nullptr;  // device upload block: angles of all groups
  size_t n_up = 0, n_res = 0;
  void *pin = nullptr;  // pinned: [angles][active flags][results]
  int grid = 1024;
  // item lists (device) for the current ansatz lengths
  void *items_d = nullptr;
  size_t items_cap = 0;
  // descriptors of the points' runs of phase gates (device), referenced by items
  DiagRun *runs_d = nullptr;
  size_t runs_cap = 0;
  struct Launch {
    int kind, d, n;  // kind: 0 gate, 1 H, 2 adj, 3 reduce
    size_t off;
  };
  std::vector<Launch> eval_launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int iter = 0;
};

namespace {

double *pin_up(fock_sweep *sw) { return (double *)sw->pin; }
int *pin_active(fock_sweep *sw) { return (int *)((char *)sw->pin + al256(sizeof(double) * sw->n_up)); }
double *pin_res(fock_sweep *sw) {
  return (double *)((char *)sw->pin + al256(sizeof(double) * sw->n_up) + al256(sizeof(int) * sw->pts.size()));
}

// ---------------------------------------------------------------- item lists
struct Lists {
  std::vector<std::vector<std::vector<SweepItem>>> fwd, rev;  // [k][2 * group + item class]
  std::vector<std::vector<SweepHItem>> h;                     // [group]
  std::vector<SweepRItem> red;
};

// A point's gate groups: [k0, k1) runs of phase gates (diag_run_end) or single gates.
void point_groups(const std::vector<fock_op_t> &ops, std::vector<std::pair<int, int>> *gr) {
  gr->clear();
  const int n = (int)ops.size();
  for (int k = 0; k < n;) {
    const int e = diag_run_end(ops.data(), n, k);
    const int k1 = e > k ? e : k + 1;
    gr->push_back({k, k1});
    k = k1;
  }
}

// Gate layers are the points' gate groups: layer l holds group l of every
// point, so a run of phase gates takes one layer and one pass.
int build_lists(fock_sweep *sw, const std::vector<char> &sel, bool grad, Lists *Ls) {
  const size_t npt = sw->pts.size();
  std::vector<std::vector<std::pair<int, int>>> groups(npt);
  std::vector<DiagRun> runs;
  std::vector<size_t> run_base(npt, 0);
  int maxn = 0;
  for (size_t p = 0; p < npt; ++p) {
    const SPoint &P = sw->pts[p];
    point_groups(P.ops, &groups[p]);
    run_base[p] = runs.size();
    for (auto &g : groups[p])
      if (g.second - g.first > 1) runs.push_back(diag_run_params(P.g, P.ops.data(), g.first, g.second));
    if (sel[p]) maxn = std::max(maxn, (int)groups[p].size());
  }
  if (runs.size() > sw->runs_cap) {
    if (sw->runs_d) FOCK_HIP(hipFree(sw->runs_d));
    sw->runs_d = nullptr;
    sw->runs_cap = 0;
    FOCK_HIP(hipMalloc(&sw->runs_d, sizeof(DiagRun) * runs.size() * 2));
    sw->runs_cap = runs.size() * 2;
  }
  if (!runs.empty())
    FOCK_HIP(hipMemcpy(sw->runs_d, runs.data(), sizeof(DiagRun) * runs.size(), hipMemcpyHostToDevice));
  const int NG = (int)sw->groups.size();
  Ls->fwd.assign(maxn, std::vector<std::vector<SweepItem>>(2 * NG));
  Ls->rev.assign(maxn, std::vector<std::vector<SweepItem>>(2 * NG));
  Ls->h.assign(NG, {});
  Ls->red.clear();
  for (size_t pi = 0; pi < npt; ++pi) {
    if (!sel[pi]) continue;
    SPoint &P = sw->pts[pi];
    const DGroup &G = sw->groups[P.group];
    const int stride = gate_stride(P.g.d);
    const int n = (int)P.ops.size();
    size_t ri = run_base[pi];
    for (size_t l = 0; l < groups[pi].size(); ++l) {
      const int k = groups[pi][l].first, k1 = groups[pi][l].second;
      const fock_op_t &op = P.ops[k];
      SweepItem it;
      memset(&it, 0, sizeof(it));
      it.p = (int)pi;
      it.U = G.utab + (size_t)(P.gate_base + k) * stride;
      int nb;
      if (k1 - k > 1) {
        it.variant = 3;
        it.kind = 0;
        it.rs = P.rs;
        it.run = sw->runs_d + ri++;
        nb = diag_blocks_count(P.g);
      } else if (is_single_mode(op.type)) {
        it.variant = 2;
        it.kind = 0;
        it.dl = diag_launch_params(P.g, op.i, op.type);
        nb = diag_blocks_count(P.g);
      } else {
        it.variant = op.i == 0 ? (sweep_m0_piped(P.g.d, (int)P.g.n_amp, 0) ? 4 : 1) : 0;
        it.kind = gate_kind(op.type);
        it.gl = gate_launch_params(P.g, op.i, op.j);
        it.A = G.T.A[table_slot(op.type)];
        nb = sweep_gate_blocks(P.g.d, (int)P.g.n_amp, op.i);
      }
      const bool m0 = it.variant == 1 || it.variant == 4;
      const int li = 2 * P.group + (m0 && sweep_split_classes(P.g.d) ? 1 : 0);  // item class list
      for (int vb = 0; vb < nb; ++vb) {
        SweepItem f = it;
        f.vb = vb;
        f.src = k == 0 ? P.psi0 : P.phi;
        f.dst = P.phi;
        Ls->fwd[l][li].push_back(f);
        if (grad) {
          SweepItem r = it;
          r.vb = vb;
          r.dst = P.phi;
          r.lam = P.lam;
          r.partial = P.partial + (size_t)k * P.rs;
          Ls->rev[l][li].push_back(r);
        }
      }
    }
    if (grad)
      for (int k = 0; k < n; ++k) {
        const fock_op_t &op = P.ops[k];
        const int nb = is_single_mode(op.type) ? diag_blocks_count(P.g)
                                               : sweep_gate_blocks(P.g.d, (int)P.g.n_amp, op.i);
        Ls->red.push_back(SweepRItem{(int)pi, 1, nb, 0, k, P.rs, P.partial, P.res + 2 + k});
      }
    const float2 *st = n > 0 ? P.phi : P.psi0;
    for (int vb = 0; vb < P.GH; ++vb) Ls->h[P.group].push_back(SweepHItem{(int)pi, vb, st, P.lam, P.partial});
  }
  // energy / norm reductions run before the reverse sweep reuses the partials
  return FOCK_OK;
}

template <class T>
size_t push_items(std::vector<char> &blob, const std::vector<T> &v) {
  const size_t off = al256(blob.size());
  blob.resize(off + sizeof(T) * v.size());
  if (!v.empty()) memcpy(blob.data() + off, v.data(), sizeof(T) * v.size());
  return off;
}

int upload_blob(fock_sweep *sw, const std::vector<char> &blob) {
  if (blob.size() > sw->items_cap) {
    if (sw->items_d) FOCK_HIP(hipFree(sw->items_d));
    sw->items_d = nullptr;
    const size_t cap = std::max(blob.size() * 2, (size_t)1 << 20);
    FOCK_HIP(hipMalloc(&sw->items_d, cap));
    sw->items_cap = cap;
  }
  if (!blob.empty()) FOCK_HIP(hipMemcpy(sw->items_d, blob.data(), blob.size(), hipMemcpyHostToDevice));
  return FOCK_OK;
}

// Gate records for the device-side build (type and slot of every gate).
int upload_recs(fock_sweep *sw) {
  for (auto &G : sw->groups) {
    std::vector<GateRec> recs(G.ngates);
    const int stride = gate_stride(G.d);
    for (int k = 0; k < G.ngates; ++k) recs[k] = GateRec{FOCK_ROT, k * stride, 0, 0};
    for (int pi : G.pts) {
      const SPoint &P = sw->pts[pi];
      for (size_t k = 0; k < P.ops.size(); ++k) recs[P.gate_base + k].type = P.ops[k].type;
    }
    FOCK_HIP(hipMemcpy(G.recs, recs.data(), sizeof(GateRec) * recs.size(), hipMemcpyHostToDevice));
  }
  return FOCK_OK;
}

// Enqueue one evaluation round (forward, H psi, optional reverse sweep,
// reductions) of the points in the current lists.
int enqueue_eval(fock_sweep *sw, const Lists &Ls, const std::vector<size_t> &offs, bool grad, bool upload) {
  hipStream_t s = sw->s;
  char *base = (char *)sw->items_d;
  size_t oi = 0;
  if (upload) {
    FOCK_HIP(hipMemcpyAsync(sw->up_d, pin_up(sw), sizeof(double) * sw->n_up, hipMemcpyHostToDevice, s));
    FOCK_HIP(hipMemcpyAsync(sw->active_d, pin_active(sw), sizeof(int) * sw->pts.size(), hipMemcpyHostToDevice, s));
    for (auto &G : sw->groups) {
      int rc = launch_gate_build(G.theta, G.recs, G.ngates, G.T, G.utab, s);
      if (rc) return rc;
    }
  }
  const int NG = (int)sw->groups.size();
  for (size_t k = 0; k < Ls.fwd.size(); ++k)
    for (int li = 0; li < 2 * NG; ++li) {
      const auto &v = Ls.fwd[k][li];
      int rc = sweep_launch_gate(sw->groups[li / 2].d, li % 2, (const SweepItem *)(base + offs[oi++]), (int)v.size(),
                                 sw->active_d, sw->grid, s);
      if (rc) return rc;
    }
  for (int gi = 0; gi < NG; ++gi) {
    const auto &v = Ls.h[gi];
    int rc = sweep_launch_h(sw->groups[gi].d, (const SweepHItem *)(base + offs[oi++]), (int)v.size(),
                            (const HamArgs *)(base + offs.back()), sw->active_d, sw->grid, s);
    if (rc) return rc;
  }
  // energy / norm of every point
  {
    const size_t off = offs[oi++];
    const int nr = (int)(offs[oi++]);
    int rc = sweep_launch_reduce((const SweepRItem *)(base + off), nr, sw->active_d, sw->grid, s);
    if (rc) return rc;
  }
  if (grad) {
    for (int k = (int)Ls.rev.size() - 1; k >= 0; --k)
      for (int li = 0; li < 2 * NG; ++li) {
        const auto &v = Ls.rev[k][li];
        int rc = sweep_launch_adj(sw->groups[li / 2].d, li % 2,
                                  (const SweepItem *)(base + offs[oi + (size_t)k * 2 * NG + li]), (int)v.size(),
                                  sw->active_d, sw->grid, s);
        if (rc) return rc;
      }
    oi += Ls.rev.size() * 2 * NG;
    int rc = sweep_launch_reduce((const SweepRItem *)(base + offs[oi]), (int)Ls.red.size(), sw->active_d, sw->grid,
                                 s);
    if (rc) return rc;
  }
  FOCK_HIP(hipMemcpyAsync(pin_res(sw), sw->res_d, sizeof(double) * sw->n_res, hipMemcpyDeviceToHost, s));
  return FOCK_OK;
}

// Lay out all item lists in one device blob; offs lists, in order: forward
// [k][2 g + class], H [g], E/norm reduce (offset, count), reverse
// [k][2 g + class], grad reduce,
// and finally the per-point HamArgs array.
int stage_lists(fock_sweep *sw, const Lists &Ls, bool grad, std::vector<size_t> *offs) {
  std::vector<char> blob;
  offs->clear();
  for (auto &lk : Ls.fwd)
    for (auto &v : lk) offs->push_back(push_items(blob, v));
  for (auto &v : Ls.h) offs->push_back(push_items(blob, v));
  std::vector<SweepRItem> en;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    const SPoint &P = sw->pts[pi];
    en.push_back(SweepRItem{(int)pi, 0, P.GH, 2, 0, 0, P.partial, P.res + 0});
    en.push_back(SweepRItem{(int)pi, 0, P.GH, 2, 1, 0, P.partial, P.res + 1});
  }
  offs->push_back(push_items(blob, en));
  offs->push_back(en.size());
  if (grad) {
    for (auto &lk : Ls.rev)
      for (auto &v : lk) offs->push_back(push_items(blob, v));
    offs->push_back(push_items(blob, Ls.red));
  }
  std::vector<HamArgs> hams;
  for (auto &P : sw->pts) hams.push_back(P.h);
  offs->push_back(push_items(blob, hams));
  return upload_blob(sw, blob);
}

void pack_angles(fock_sweep *sw) {
  double *up = pin_up(sw);
  for (auto &G : sw->groups)
    for (int pi : G.pts) {
      const SPoint &P = sw->pts[pi];
      const std::vector<double> &x = P.want ? P.x : P.theta;
      for (size_t k = 0; k < x.size(); ++k) up[G.theta_off + P.gate_base + k] = x[k];
    }
}

void unpack(fock_sweep *sw, bool grad) {
  const double *r = pin_res(sw);
  for (auto &P : sw->pts) {
    if (!P.want) continue;
    const double *pr = r + P.res_off;
    P.n2 = pr[1];
    P.f = pr[0] / pr[1];
    if (grad) {
      P.grad.resize(P.ops.size());
      for (size_t k = 0; k < P.ops.size(); ++k) P.grad[k] = 2.0 * pr[2 + k] / pr[1];
    }
    if (!std::isfinite(P.f) || !(P.n2 > 0.0)) P.rc = set_error(FOCK_ERR_NONFINITE, "non-finite energy in sweep");
  }
}

int destroy_graph(fock_sweep *sw) {
  if (sw->gexec) (void)hipGraphExecDestroy(sw->gexec);
  if (sw->graph) (void)hipGraphDestroy(sw->graph);
  sw->gexec = nullptr;
  sw->graph = nullptr;
  return FOCK_OK;
}

// Energy and norm of the selected points at their angles P.x (forward gates
// and H psi, direct launches); results in P.f, P.n2 (P.rc on failure).
int eval_forward(fock_sweep *sw, const std::vector<char> &sel) {
  Lists Lf;
  {
    const int brc = build_lists(sw, sel, false, &Lf);
    if (brc) return brc;
  }
  std::vector<size_t> offf;
  int rc = upload_recs(sw);
  if (rc) return rc;
  rc = stage_lists(sw, Lf, false, &offf);
  if (rc) return rc;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    SPoint &P = sw->pts[pi];
    P.want = sel[pi] != 0;
    pin_active(sw)[pi] = P.want ? 1 : 0;
  }
  pack_angles(sw);
  rc = enqueue_eval(sw, Lf, offf, false, true);
  if (rc) return rc;
  FOCK_HIP(hipStreamSynchronize(sw->s));
  unpack(sw, false);
  for (auto &P : sw->pts) P.want = false;
  return FOCK_OK;
}

// Lockstep BFGS over the points in `sel`: one thread per point runs the
// minimiser; the calling thread gathers their objective requests into rounds
// and replays the captured evaluation graph once per round.
int bfgs_phase(fock_sweep *sw, const std::vector<char> &sel, const std::vector<double> &gtol,
               std::vector<fock_adapt_report_t> *reps) {
  Lists Ls;
  {
    const int brc = build_lists(sw, sel, true, &Ls);
    if (brc) return brc;
  }
  std::vector<size_t> offs;
  int rc = stage_lists(sw, Ls, true, &offs);
  if (rc) return rc;
  rc = upload_recs(sw);
  if (rc) return rc;
  destroy_graph(sw);
  FOCK_HIP(hipStreamBeginCapture(sw->s, hipStreamCaptureModeThreadLocal));
  rc = enqueue_eval(sw, Ls, offs, true, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(sw->s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_error(FOCK_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  sw->graph = g;
  FOCK_HIP(hipGraphInstantiate(&sw->gexec, g, nullptr, nullptr, 0));

  std::mutex mu;
  std::condition_variable cv_req, cv_done;
  int waiting = 0, running = 0;
  uint64_t round = 0;
  std::vector<std::thread> th;
  std::vector<BfgsOut> outs(sw->pts.size());
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    if (!sel[pi]) continue;
    SPoint &P = sw->pts[pi];
    P.finished = false;
    P.rc = 0;
    ++running;
  }
  // energy and norm at each point's final angles, when the run evaluated them
  // (as the single-point driver does, so that both report the same values)
  std::vector<char> hit(sw->pts.size(), 0);
  std::vector<double> hit_f(sw->pts.size(), 0.0), hit_n2(sw->pts.size(), 0.0);
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    if (!sel[pi]) continue;
    th.emplace_back([&, pi]() {
      SPoint &P = sw->pts[pi];
      struct Seen {
        std::vector<double> x;
        double f, n2;
      };
      std::vector<Seen> seen;
      ObjFn fn = [&](const std::vector<double> &x, double *f, std::vector<double> *gg) -> int {
        std::unique_lock<std::mutex> lk(mu);
        P.x = x;
        P.want = true;
        const uint64_t my = round;
        ++waiting;
        cv_req.notify_one();
        cv_done.wait(lk, [&] { return round != my; });
        if (P.rc) return P.rc;
        *f = P.f;
        *gg = P.grad;
        seen.push_back({x, P.f, P.n2});
        return 0;
      };
      std::vector<double> th0 = P.theta;
      BfgsOut bo;
      int r = bfgs_minimize(th0, fn, gtol[pi], sw->opt.bfgs_maxiter, nullptr, &bo, sw->opt.noise_rel);
      std::unique_lock<std::mutex> lk(mu);
      for (const Seen &e : seen)
        if (e.x == th0) {
          hit[pi] = 1;
          hit_f[pi] = e.f;
          hit_n2[pi] = e.n2;
        }
      if (!r) P.theta = th0;
      if (r && !P.rc) P.rc = r;
      outs[pi] = bo;
      P.finished = true;
      --running;
      cv_req.notify_one();
    });
  }
  int err = 0;
  {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv_req.wait(lk, [&] { return waiting == running; });
      if (running == 0) break;
      // one round for every waiting point
      int *act = pin_active(sw);
      for (size_t pi = 0; pi < sw->pts.size(); ++pi) act[pi] = sw->pts[pi].want ? 1 : 0;
      pack_angles(sw);
      hipError_t le = hipGraphLaunch(sw->gexec, sw->s);
      if (le == hipSuccess) le = hipStreamSynchronize(sw->s);
      if (le != hipSuccess) {
        err = set_error(FOCK_ERR_HIP, "sweep graph launch failed: %s", hipGetErrorString(le));
        for (auto &P : sw->pts)
          if (P.want) P.rc = err;
      } else {
        unpack(sw, true);
      }
      for (auto &P : sw->pts) P.want = false;
      waiting = 0;
      ++round;
      cv_done.notify_all();
    }
  }
  for (auto &t : th) t.join();
  if (err) return err;
  // final energies at the accepted angles (forward only, graph-free) for the
  // points whose run did not evaluate them
  std::vector<char> need(sw->pts.size(), 0);
  bool any = false;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi)
    if (sel[pi]) {
      SPoint &P = sw->pts[pi];
      if (hit[pi]) {
        P.f = hit_f[pi];
        P.n2 = hit_n2[pi];
      } else {
        P.x = P.theta;
        need[pi] = 1;
        any = true;
      }
    }
  if (any && (rc = eval_forward(sw, need))) return rc;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    if (!sel[pi]) continue;
    SPoint &P = sw->pts[pi];
    if (P.rc) return P.rc;
    fock_adapt_report_t &r = (*reps)[pi];
    r.bfgs_iters = outs[pi].iters;
    r.bfgs_evals = outs[pi].evals + need[pi];
    r.status = outs[pi].status;
    r.E = P.f;
    r.norm2 = P.n2;
    r.E_init = outs[pi].f0;
    r.n_params = (int)P.theta.size();
  }
  return FOCK_OK;
}

// Forward + H psi + pool scoring for the selected points (direct launches).
int score_phase(fock_sweep *sw, const std::vector<char> &sel, std::vector<std::vector<double>> *grads) {
  Lists Ls;
  {
    const int brc = build_lists(sw, sel, false, &Ls);
    if (brc) return brc;
  }
  std::vector<size_t> offs;
  // pool items reuse the H tiles of every point
  std::vector<char> blob;
  int rc = upload_recs(sw);
  if (rc) return rc;
  rc = stage_lists(sw, Ls, false, &offs);
  if (rc) return rc;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    SPoint &P = sw->pts[pi];
    P.want = sel[pi] != 0;
    if (P.want) P.x = P.theta;
    pin_active(sw)[pi] = P.want ? 1 : 0;
  }
  pack_angles(sw);
  rc = enqueue_eval(sw, Ls, offs, false, true);
  if (rc) return rc;
  // pool scoring: items per group, then per-slot reductions into res[2..]
  std::vector<std::vector<SweepHItem>> pitems(sw->groups.size());
  std::vector<SweepRItem> red;
  std::vector<SweepPoolArgs> pargs;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    SPoint &P = sw->pts[pi];
    pargs.push_back(P.pa);
    if (!sel[pi]) continue;
    const float2 *st = P.ops.empty() ? P.psi0 : P.phi;
    for (int vb = 0; vb < P.GH; ++vb) pitems[P.group].push_back(SweepHItem{(int)pi, vb, st, P.lam, P.partial});
    for (int k = 0; k < P.P; ++k) red.push_back(SweepRItem{(int)pi, 0, P.GH, P.P, k, 0, P.partial, P.res + 2 + k});
  }
  // a second blob after the eval items: synchronise before reusing the item buffer
  FOCK_HIP(hipStreamSynchronize(sw->s));
  unpack(sw, false);
  std::vector<size_t> po;
  for (auto &v : pitems) po.push_back(push_items(blob, v));
  const size_t ro = push_items(blob, red);
  const size_t ao = push_items(blob, pargs);
  rc = upload_blob(sw, blob);
  if (rc) return rc;
  char *base = (char *)sw->items_d;
  for (size_t gi = 0; gi < sw->groups.size(); ++gi) {
    rc = sweep_launch_pool(sw->groups[gi].d, (const SweepHItem *)(base + po[gi]), (int)pitems[gi].size(),
                           (const SweepPoolArgs *)(base + ao), sw->active_d, sw->grid, sw->s);
    if (rc) return rc;
  }
  rc = sweep_launch_reduce((const SweepRItem *)(base + ro), (int)red.size(), sw->active_d, sw->grid, sw->s);
  if (rc) return rc;
  FOCK_HIP(hipMemcpyAsync(pin_res(sw), sw->res_d, sizeof(double) * sw->n_res, hipMemcpyDeviceToHost, sw->s));
  FOCK_HIP(hipStreamSynchronize(sw->s));
  const double *r = pin_res(sw);
  grads->assign(sw->pts.size(), {});
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    SPoint &P = sw->pts[pi];
    P.want = false;
    if (!sel[pi]) continue;
    (*grads)[pi].resize(P.P);
    for (int k = 0; k < P.P; ++k) (*grads)[pi][k] = r[P.res_off + 2 + k] / P.n2;
  }
  return FOCK_OK;
}

double gtol_for(const fock_adapt_opts_t &o, double gsel, double E) {
  const double paper = std::min(1e-6, 1e-5 * gsel);
  return std::max(paper, o.gtol_floor_rel * std::max(1.0, std::fabs(E)));
}

}  // namespace

extern "C" {

int fock_sweep_create(const fock_sweep_point_t *pts, int npts, const fock_adapt_opts_t *opts, fock_stream_t stream,
                      fock_sweep_t **out) {
  if (!out) return set_error(FOCK_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!pts || npts < 1 || npts > 4096) return set_error(FOCK_ERR_ARG, "npts must be in [1, 4096]");
  if (!opts) return set_error(FOCK_ERR_ARG, "opts is NULL");
  if (opts->warm_fixed != 0)
    return set_error(FOCK_ERR_UNSUPPORTED, "fixed warm-up angles are taken by the complex128 driver only");
  if (opts->max_iters < 0 || opts->max_iters > 4000) return set_error(FOCK_ERR_ARG, "max_iters out of range 0..4000");
  int rc = 0;
  for (int p = 0; p < npts; ++p) {
    uint32_t namp = 0;
    if ((rc = check_ham(&pts[p].ham, &namp))) return rc;
    if (!sweep_supports_d(pts[p].ham.d))
      return set_error(FOCK_ERR_UNSUPPORTED, "point %d: sweep kernels support d in {4, 6, 8}", p);
    if (pts[p].ham.L < 2) return set_error(FOCK_ERR_UNSUPPORTED, "point %d: sweep needs L >= 2", p);
    if (!pts[p].pool || pts[p].P < 1 || pts[p].P > kMaxSlots)
      return set_error(FOCK_ERR_ARG, "point %d: pool must hold 1..%d ops", p, kMaxSlots);
    if ((rc = check_ptr(pts[p].psi0, "psi0"))) return rc;
    for (int k = 0; k < pts[p].P; ++k) {
      if ((rc = check_op(pts[p].pool[k], pts[p].ham.L))) return rc;
      if (is_squeeze(pts[p].pool[k].type))
        return set_error(FOCK_ERR_UNSUPPORTED, "point %d: the sweep kernels do not take squeezer ops (pool %d)", p, k);
    }
    if (pts[p].n_warm < 0 || pts[p].n_warm > 4096 || (pts[p].n_warm > 0 && (!pts[p].warm_ops || !pts[p].warm_theta0)))
      return set_error(FOCK_ERR_ARG, "point %d: warm-up layer needs 0..4096 ops with both arrays given", p);
    for (int k = 0; k < pts[p].n_warm; ++k) {
      if ((rc = check_op(pts[p].warm_ops[k], pts[p].ham.L))) return rc;
      if (is_squeeze(pts[p].warm_ops[k].type))
        return set_error(FOCK_ERR_UNSUPPORTED, "point %d: the sweep kernels do not take squeezer ops (warm-up %d)", p,
                         k);
    }
  }
  // the caller's psi0 buffers must be ready before the private stream reads them
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return set_error(FOCK_ERR_HIP, "caller stream error");
  fock_sweep *sw = new fock_sweep();
  sw->opt = *opts;
  if (hipStreamCreateWithFlags(&sw->s, hipStreamNonBlocking) != hipSuccess) {
    delete sw;
    return set_error(FOCK_ERR_HIP, "stream creation failed");
  }
  sw->pts.resize(npts);
  std::map<int, int> gidx;
  size_t bytes = 0;
  std::vector<size_t> poff(npts);
  for (int p = 0; p < npts; ++p) {
    SPoint &P = sw->pts[p];
    const fock_sweep_point_t &in = pts[p];
    P.ham = in.ham;
    uint32_t namp = 0;
    check_ham(&in.ham, &namp);
    P.g = Geometry{in.ham.L, in.ham.d, namp};
    P.h = make_ham_args(in.ham);
    P.pool.assign(in.pool, in.pool + in.P);
    P.P = in.P;
    for (int k = 0; k < in.n_warm; ++k) {
      P.ops.push_back(in.warm_ops[k]);
      P.theta.push_back(in.warm_theta0[k]);
    }
    P.nmax = in.n_warm + opts->max_iters + 1;
    const Layout L = make_layout(namp, in.ham.L, in.ham.d, P.P, P.nmax);
    P.G = L.G;
    P.rs = L.rs;
    P.GH = apply_h_blocks(P.h);
    if (P.GH > P.G) {
      fock_sweep_destroy(sw);
      return set_error(FOCK_ERR_HIP, "internal: tile count exceeds the partial buffer");
    }
    if (!gidx.count(in.ham.d)) {
      gidx[in.ham.d] = (int)sw->groups.size();
      DGroup G;
      G.d = in.ham.d;
      sw->groups.push_back(G);
    }
    P.group = gidx[in.ham.d];
    DGroup &G = sw->groups[P.group];
    G.pts.push_back(p);
    P.gate_base = G.ngates;
    G.ngates += P.nmax;
    const size_t sb = al256(sizeof(float2) * namp);
    const size_t rows = std::max<size_t>({2, (size_t)P.nmax, (size_t)P.P});
    poff[p] = bytes;
    bytes += 3 * sb + al256(sizeof(double) * rows * std::max(P.G, P.rs)) + al256(sizeof(PoolPair) * kMaxPairs) +
             al256(sizeof(PoolDiag) * kMaxDiagOps);
    P.res_off = (int)sw->n_res;
    sw->n_res += 2 + std::max(P.nmax, P.P);
  }
  size_t goff = bytes;
  for (auto &G : sw->groups) {
    G.theta_off = sw->n_up;
    sw->n_up += G.ngates;
    bytes += al256(sizeof(GateRec) * G.ngates) + al256(sizeof(float2) * (size_t)gate_stride(G.d) * G.ngates);
  }
  const size_t up_off = bytes;
  bytes += al256(sizeof(double) * sw->n_up);
  const size_t res_off = bytes;
  bytes += al256(sizeof(double) * sw->n_res);
  const size_t act_off = bytes;
  bytes += al256(sizeof(int) * npts);
  if (hipMalloc(&sw->dbuf, bytes) != hipSuccess) {
    fock_sweep_destroy(sw);
    return set_error(FOCK_ERR_HIP, "hipMalloc of %zu bytes for the sweep failed", bytes);
  }
  char *b = (char *)sw->dbuf;
  sw->up_d = (double *)(b + up_off);
  sw->res_d = (double *)(b + res_off);
  sw->active_d = (int *)(b + act_off);
  for (auto &G : sw->groups) {
    G.recs = (GateRec *)(b + goff);
    goff += al256(sizeof(GateRec) * G.ngates);
    G.utab = (float2 *)(b + goff);
    goff += al256(sizeof(float2) * (size_t)gate_stride(G.d) * G.ngates);
    G.theta = sw->up_d + G.theta_off;
    if ((rc = get_tables(G.d, &G.T))) break;
  }
  const size_t pin_bytes =
      al256(sizeof(double) * sw->n_up) + al256(sizeof(int) * npts) + al256(sizeof(double) * sw->n_res);
  if (!rc && hipHostMalloc(&sw->pin, pin_bytes, hipHostMallocDefault) != hipSuccess)
    rc = set_error(FOCK_ERR_HIP, "pinned allocation failed");
  if (!rc) memset(sw->pin, 0, pin_bytes);
  for (int p = 0; p < npts && !rc; ++p) {
    SPoint &P = sw->pts[p];
    char *pb = b + poff[p];
    const size_t sb = al256(sizeof(float2) * P.g.n_amp);
    const size_t rows = std::max<size_t>({2, (size_t)P.nmax, (size_t)P.P});
    P.psi0 = (float2 *)pb;
    P.phi = (float2 *)(pb + sb);
    P.lam = (float2 *)(pb + 2 * sb);
    P.partial = (double *)(pb + 3 * sb);
    P.pairs = (PoolPair *)(pb + 3 * sb + al256(sizeof(double) * rows * std::max(P.G, P.rs)));
    P.diags = (PoolDiag *)((char *)P.pairs + al256(sizeof(PoolPair) * kMaxPairs));
    P.res = sw->res_d + P.res_off;
    if (hipMemcpyAsync(P.psi0, pts[p].psi0, sizeof(float2) * P.g.n_amp, hipMemcpyDeviceToDevice, sw->s) !=
        hipSuccess)
      rc = set_error(FOCK_ERR_HIP, "copy of psi0 failed");
    // pool description (one chunk: P <= kMaxSlots)
    std::vector<PoolPair> pairs;
    std::vector<PoolDiag> diags;
    std::map<std::pair<int, int>, int> pidx;
    for (int k = 0; k < P.P && !rc; ++k) {
      const fock_op_t &op = P.pool[k];
      if (is_pool_diagonal(op.type)) {
        diags.push_back({(int16_t)op.i, (int16_t)op.type, (int16_t)k, (int16_t)(op.type == FOCK_CK ? op.j : -1)});
        continue;
      }
      auto key = std::make_pair(op.i, op.j);
      if (!pidx.count(key)) {
        PoolPair pp;
        pp.i = (int16_t)op.i;
        pp.j = (int16_t)op.j;
        for (int t = 0; t < 5; ++t) pp.slot[t] = -1;
        pp.pad = 0;
        pidx[key] = (int)pairs.size();
        pairs.push_back(pp);
      }
      PoolPair &pp = pairs[pidx[key]];
      if (pp.slot[op.type] >= 0) rc = set_error(FOCK_ERR_ARG, "point %d: duplicate pool entry %d", p, k);
      pp.slot[op.type] = (int16_t)k;
    }
    if (!rc && ((int)pairs.size() > kMaxPairs || (int)diags.size() > kMaxDiagOps))
      rc = set_error(FOCK_ERR_ARG, "point %d: pool too large for one sweep launch", p);
    if (rc) break;
    if (!pairs.empty() &&
        hipMemcpy(P.pairs, pairs.data(), sizeof(PoolPair) * pairs.size(), hipMemcpyHostToDevice) != hipSuccess)
      rc = set_error(FOCK_ERR_HIP, "pool upload failed");
    if (!diags.empty() &&
        hipMemcpy(P.diags, diags.data(), sizeof(PoolDiag) * diags.size(), hipMemcpyHostToDevice) != hipSuccess)
      rc = set_error(FOCK_ERR_HIP, "pool upload failed");
    memset(&P.pa, 0, sizeof(P.pa));
    P.pa.args.L = P.g.L;
    P.pa.args.d = P.g.d;
    P.pa.args.nrows = P.h.nrows;
    P.pa.args.npairs = (int)pairs.size();
    P.pa.args.ndiag = (int)diags.size();
    P.pa.args.nslots = P.P;
    for (int r = 0; r < kMaxL; ++r) P.pa.args.srow[r] = P.h.srow[r];
    for (int k = 0; k <= kMaxD; ++k) P.pa.args.sq[k] = P.h.sq[k];
    P.pa.pairs = P.pairs;
    P.pa.diags = P.diags;
  }
  if (!rc && hipStreamSynchronize(sw->s) != hipSuccess) rc = set_error(FOCK_ERR_HIP, "stream error at create");
  // warm-up layer of the points that have one
  if (!rc) {
    std::vector<char> sel(npts, 0);
    bool any = false;
    for (int p = 0; p < npts; ++p)
      if (pts[p].n_warm > 0) sel[p] = any = true;
    std::vector<fock_adapt_report_t> reps(npts);
    std::vector<double> gt(npts, 0.0);
    if (any) {
      // energies at the initial angles set the FP32 tolerance floor
      std::vector<std::vector<double>> dummy;
      rc = score_phase(sw, sel, &dummy);
      for (int p = 0; p < npts && !rc; ++p)
        gt[p] = std::max(opts->warm_gtol, gtol_for(*opts, 0.0, sw->pts[p].f));
      if (!rc) rc = bfgs_phase(sw, sel, gt, &reps);
    }
    for (int p = 0; p < npts && !rc; ++p) {
      sw->pts[p].warm = reps[p];
      sw->pts[p].warm.iter = 0;
      sw->pts[p].warm.k_sel = -1;
    }
  }
  if (rc) {
    (void)hipStreamSynchronize(sw->s);
    fock_sweep_destroy(sw);
    return rc;
  }
  *out = sw;
  return FOCK_OK;
}

int fock_sweep_step(fock_sweep_t *sw, fock_adapt_report_t *reps, int *n_active) {
  if (!sw || !reps) return set_error(FOCK_ERR_ARG, "NULL argument");
  const int npts = (int)sw->pts.size();
  std::vector<char> sel(npts, 0);
  int nsel = 0;
  for (int p = 0; p < npts; ++p)
    if (!sw->pts[p].done) sel[p] = 1, ++nsel;
  if (n_active) *n_active = nsel;
  for (int p = 0; p < npts; ++p) {
    memset(&reps[p], 0, sizeof(reps[p]));
    reps[p].k_sel = -1;
    reps[p].iter = sw->pts[p].iter;
  }
  if (nsel == 0) return set_error(FOCK_ERR_STATE, "every sweep point has finished");
  std::vector<std::vector<double>> g;
  int rc = score_phase(sw, sel, &g);
  if (rc) return rc;
  std::vector<char> opt(npts, 0);
  std::vector<double> gt(npts, 0.0);
  for (int p = 0; p < npts; ++p) {
    if (!sel[p]) continue;
    SPoint &P = sw->pts[p];
    P.iter += 1;
    fock_adapt_report_t &r = reps[p];
    r.iter = P.iter;
    double gn2 = 0.0, ginf = 0.0;
    for (double v : g[p]) {
      gn2 += v * v;
      ginf = std::max(ginf, std::fabs(v));
    }
    gn2 = std::sqrt(gn2);
    r.g_norm2 = gn2;
    r.g_inf = ginf;
    r.E = r.E_init = P.f;
    r.norm2 = P.n2;
    r.n_params = (int)P.theta.size();
    if (gn2 < sw->opt.grad_tol) {
      r.converged = 1;
      P.done = true;
      continue;
    }
    if (P.iter > sw->opt.max_iters) {
      r.capped = 1;
      P.done = true;
      continue;
    }
    int ks = 0;
    for (int k = 0; k < P.P; ++k)
      if (std::fabs(g[p][k]) >= (1.0 - sw->opt.tie_tau) * ginf) {
        ks = k;
        break;
      }
    r.k_sel = ks;
    r.g_sel = std::fabs(g[p][ks]);
    P.ops.push_back(P.pool[ks]);
    P.theta.push_back(0.0);
    opt[p] = 1;
    gt[p] = gtol_for(sw->opt, r.g_sel, P.f);
  }
  // warm-start proposals: keep one only if its energy is not above the plain
  // start {theta_prev, 0} (whose energy is the one just scored)
  {
    std::vector<char> ps(npts, 0);
    bool anyp = false;
    for (int p = 0; p < npts; ++p) {
      SPoint &P = sw->pts[p];
      P.prop_acc = 0;
      if (!opt[p] || !P.has_prop) {
        P.has_prop = false;
        continue;
      }
      P.has_prop = false;
      if (P.proposal.size() != P.theta.size()) continue;
      P.plain_E = P.f;
      P.x = P.proposal;
      ps[p] = 1;
      anyp = true;
    }
    if (anyp) {
      rc = eval_forward(sw, ps);
      if (rc) return rc;
      for (int p = 0; p < npts; ++p) {
        if (!ps[p]) continue;
        SPoint &P = sw->pts[p];
        if (P.rc) return P.rc;
        P.prop_E = P.f;
        if (P.prop_E <= P.plain_E) {
          P.theta = P.proposal;
          P.prop_acc = 1;
        }
      }
    }
  }
  bool any = false;
  for (char c : opt) any |= c != 0;
  if (any) {
    std::vector<fock_adapt_report_t> br(npts);
    rc = bfgs_phase(sw, opt, gt, &br);
    if (rc) return rc;
    for (int p = 0; p < npts; ++p) {
      if (!opt[p]) continue;
      fock_adapt_report_t &r = reps[p];
      r.bfgs_iters = br[p].bfgs_iters;
      r.bfgs_evals = br[p].bfgs_evals;
      r.status = br[p].status;
      r.E = br[p].E;
      r.norm2 = br[p].norm2;
      r.E_init = br[p].E_init;
      r.n_params = br[p].n_params;
    }
  }
  for (int p = 0; p < npts; ++p) sw->pts[p].last = reps[p];
  sw->iter += 1;
  return FOCK_OK;
}

int fock_sweep_warm_reports(fock_sweep_t *sw, fock_adapt_report_t *reps) {
  if (!sw || !reps) return set_error(FOCK_ERR_ARG, "NULL argument");
  for (size_t p = 0; p < sw->pts.size(); ++p) reps[p] = sw->pts[p].warm;
  return FOCK_OK;
}

int fock_sweep_get_ansatz(fock_sweep_t *sw, int point, fock_op_t *ops, double *theta, int cap, int *n) {
  if (!sw || !n || point < 0 || point >= (int)sw->pts.size()) return set_error(FOCK_ERR_ARG, "bad point");
  const SPoint &P = sw->pts[point];
  *n = (int)P.ops.size();
  for (int k = 0; k < std::min(cap, *n); ++k) {
    if (ops) ops[k] = P.ops[k];
    if (theta) theta[k] = P.theta[k];
  }
  return FOCK_OK;
}

int fock_sweep_propose(fock_sweep_t *sw, int point, const double *theta, int n) {
  if (!sw || (!theta && n > 0)) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (point < 0 || point >= (int)sw->pts.size()) return set_error(FOCK_ERR_ARG, "point %d out of range", point);
  SPoint &P = sw->pts[point];
  if (n != (int)P.theta.size() + 1)
    return set_error(FOCK_ERR_ARG, "proposal length %d != current parameters + 1 (%d)", n, (int)P.theta.size() + 1);
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(theta[k])) return set_error(FOCK_ERR_NONFINITE, "proposal[%d] not finite", k);
  P.proposal.assign(theta, theta + n);
  P.has_prop = true;
  return FOCK_OK;
}

int fock_sweep_last_proposal(fock_sweep_t *sw, int point, int *accepted, double *E_prop, double *E_plain) {
  if (!sw) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (point < 0 || point >= (int)sw->pts.size()) return set_error(FOCK_ERR_ARG, "point %d out of range", point);
  const SPoint &P = sw->pts[point];
  if (accepted) *accepted = P.prop_acc;
  if (E_prop) *E_prop = P.prop_E;
  if (E_plain) *E_plain = P.plain_E;
  return FOCK_OK;
}

int fock_sweep_set_grid(fock_sweep_t *sw, int grid) {
  if (!sw || grid < 1 || grid > (1 << 20)) return set_error(FOCK_ERR_ARG, "bad grid");
  sw->grid = grid;
  return FOCK_OK;
}

// Autotuner: times one forward + H psi evaluation of every unfinished point
// for each candidate persistent-grid size (HIP events on the sweep's stream,
// median of 3 after a warm-up) and keeps the fastest.  With a cache file the
// choice is looked up first by (architecture, point count, amplitudes, gate
// slots) and appended after tuning, one JSON object per line.
int fock_sweep_autotune(fock_sweep_t *sw, const char *cache_path, int *best_grid) {
  if (!sw) return set_error(FOCK_ERR_ARG, "NULL sweep");
  hipDeviceProp_t prop;
  FOCK_HIP(hipGetDeviceProperties(&prop, 0));
  size_t amps = 0, gates = 0;
  for (auto &P : sw->pts) {
    amps += P.g.n_amp;
    gates += P.ops.size();
  }
  char key[256];
  snprintf(key, sizeof(key), "%s|sweep|npts=%zu|amps=%zu|gates=%zu", prop.gcnArchName, sw->pts.size(), amps, gates);
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char line[512];
      int found = -1;
      while (fgets(line, sizeof(line), f)) {
        const char *k = strstr(line, key);
        const char *g = strstr(line, "\"grid\": ");
        if (k && g) found = atoi(g + 8);
      }
      fclose(f);
      if (found > 0) {
        sw->grid = found;
        if (best_grid) *best_grid = found;
        return FOCK_OK;
      }
    }
  }
  std::vector<char> sel(sw->pts.size(), 0);
  for (size_t p = 0; p < sw->pts.size(); ++p) sel[p] = !sw->pts[p].done;
  Lists Ls;
  {
    const int brc = build_lists(sw, sel, false, &Ls);
    if (brc) return brc;
  }
  std::vector<size_t> offs;
  int rc = upload_recs(sw);
  if (rc) return rc;
  rc = stage_lists(sw, Ls, false, &offs);
  if (rc) return rc;
  for (size_t pi = 0; pi < sw->pts.size(); ++pi) {
    SPoint &P = sw->pts[pi];
    P.want = sel[pi] != 0;
    P.x = P.theta;
    pin_active(sw)[pi] = P.want ? 1 : 0;
  }
  pack_angles(sw);
  for (auto &P : sw->pts) P.want = false;
  hipEvent_t e0, e1;
  FOCK_HIP(hipEventCreate(&e0));
  FOCK_HIP(hipEventCreate(&e1));
  const int cand[] = {256, 512, 1024, 2048, 4096};
  int best = sw->grid;
  float best_ms = 1e30f;
  for (int c : cand) {
    sw->grid = c;
    float t[3];
    for (int r = -1; r < 3; ++r) {
      FOCK_HIP(hipEventRecord(e0, sw->s));
      rc = enqueue_eval(sw, Ls, offs, false, true);
      if (rc) break;
      FOCK_HIP(hipEventRecord(e1, sw->s));
      FOCK_HIP(hipEventSynchronize(e1));
      if (r >= 0) FOCK_HIP(hipEventElapsedTime(&t[r], e0, e1));
    }
    if (rc) break;
    std::sort(t, t + 3);
    if (t[1] < best_ms) {
      best_ms = t[1];
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  sw->grid = best;
  if (best_grid) *best_grid = best;
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "{\"key\": \"%s\", \"grid\": %d, \"ms\": %.4f}\n", key, best, best_ms);
      fclose(f);
    }
  }
  return FOCK_OK;
}

int fock_sweep_destroy(fock_sweep_t *sw) {
  if (!sw) return FOCK_OK;
  (void)hipStreamSynchronize(sw->s);
  destroy_graph(sw);
  if (sw->items_d) (void)hipFree(sw->items_d);
  if (sw->runs_d) (void)hipFree(sw->runs_d);
  if (sw->dbuf) (void)hipFree(sw->dbuf);
  if (sw->pin) (void)hipHostFree(sw->pin);
  if (sw->s) (void)hipStreamDestroy(sw->s);
  delete sw;
  return FOCK_OK;
}

}  // extern "C"
