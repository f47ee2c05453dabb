// Host-side support: error reporting, invariant division, local generator
// matrices, the Hermitian Jacobi eigensolver for the gate blocks, the
// library-owned device eigendata, and per-kernel event timing.
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <tuple>
#include <vector>
#include <mutex>

#include "fock_internal.h"

namespace fock {

// ---------------------------------------------------------------- errors
static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

const char *last_error() { return g_err; }

// ---------------------------------------------------------------- invariant division
FastDiv make_fastdiv(uint32_t v) {
  FastDiv f;
  f.v = v;
  uint32_t l = 0;
  while ((1ull << l) < v) ++l;
  f.sh = 32 + l;
  f.m = (uint64_t)((((unsigned __int128)1) << (32 + l)) / v) + 1;
  return f;
}

// ---------------------------------------------------------------- local generators
using cd = std::complex<double>;

bool is_single_mode(int type) { return type == FOCK_KERR || type == FOCK_ROT || type == FOCK_SR || type == FOCK_SI; }
bool is_squeeze(int type) { return type == FOCK_SR || type == FOCK_SI; }
bool is_pool_diagonal(int type) { return type == FOCK_KERR || type == FOCK_ROT || type == FOCK_CK; }

int diag_run_end(const fock_op_t *ops, int n, int k) {
  auto phase = [](const fock_op_t &o) { return o.type == FOCK_KERR || o.type == FOCK_ROT; };
  if (k + 1 >= n || !phase(ops[k]) || !phase(ops[k + 1])) return k;
  int k1 = k + 1;
  while (k1 < n && k1 - k < kMaxDiagRun && phase(ops[k1])) ++k1;
  return k1;
}
int gate_kind(int type) { return (type == FOCK_PR || type == FOCK_PI) ? KIND_DIFF : KIND_SUM; }

// Truncated annihilation operator, a|m> = sqrt(m)|m-1> (Sec. II.A).
static double lad(int d, int row, int col) { return (col >= 1 && row == col - 1) ? std::sqrt((double)col) : 0.0; }
static double cre(int d, int row, int col) { return lad(d, col, row); }

void generator_dense(int type, int d, std::vector<double> &m) {
  if (is_squeeze(type)) {
    // SR = (a^2 - a^+2) / 2, SI = i (a^2 + a^+2) / 2; a^2 |n> = sqrt(n (n-1)) |n-2>
    m.assign(2 * d * d, 0.0);
    for (int n = 2; n < d; ++n) {
      const double c = 0.5 * std::sqrt((double)n * (double)(n - 1));
      if (type == FOCK_SR) {
        m[2 * ((n - 2) * d + n)] = c;   // a^2: row n-2, column n
        m[2 * (n * d + (n - 2))] = -c;  // -a^+2: row n, column n-2
      } else {
        m[2 * ((n - 2) * d + n) + 1] = c;
        m[2 * (n * d + (n - 2)) + 1] = c;
      }
    }
    return;
  }
  if (is_single_mode(type)) {
    m.assign(2 * d * d, 0.0);
    for (int n = 0; n < d; ++n) m[2 * (n * d + n) + 1] = type == FOCK_KERR ? (double)n * n : (double)n;
    return;
  }
  const int D2 = d * d;
  m.assign(2 * D2 * D2, 0.0);
  for (int ip = 0; ip < d; ++ip)
    for (int jp = 0; jp < d; ++jp)
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          const double hop1 = cre(d, ip, i) * lad(d, jp, j);      // a_i^+ a_j
          const double hop2 = lad(d, ip, i) * cre(d, jp, j);      // a_i a_j^+ = a_j^+ a_i
          const double pr1 = lad(d, ip, i) * lad(d, jp, j);       // a_i a_j
          const double pr2 = cre(d, ip, i) * cre(d, jp, j);       // a_i^+ a_j^+
          // N_i a_i^+ : N acts after the creation, i.e. multiplies by the new n_i = ip
          const double dh1 = (double)ip * hop1;
          // a_i N_i : N acts first, multiplies by the old n_i = i
          const double dh2 = (double)i * hop2;
          double re = 0.0, im = 0.0;
          switch (type) {
            case FOCK_HR: re = hop1 - hop2; break;
            case FOCK_HI: im = hop1 + hop2; break;
            case FOCK_DH: im = dh1 + dh2; break;
            case FOCK_PR: re = pr1 - pr2; break;
            case FOCK_PI: im = pr1 + pr2; break;
            case FOCK_CK: im = (ip == i && jp == j) ? (double)(i * j) : 0.0; break;
            default: break;
          }
          const int r = ip * d + jp, c = i * d + j;
          m[2 * (r * D2 + c)] = re;
          m[2 * (r * D2 + c) + 1] = im;
        }
}

// ---------------------------------------------------------------- Hermitian Jacobi
// Cyclic Jacobi for a complex Hermitian n x n matrix H (row-major).  Each
// rotation J = diag(1, e^{-i phi}) [[c, s], [-s, c]] on (p, q) first makes
// H_pq real, then annihilates it with the symmetric Schur rotation (Golub &
// Van Loan, Alg. 8.4.1).  On return w holds the eigenvalues and column m of V
// the eigenvector of w[m].
static void herm_jacobi(int n, std::vector<cd> H, std::vector<double> &w, std::vector<cd> &V) {
  V.assign(n * n, cd(0.0, 0.0));
  for (int k = 0; k < n; ++k) V[k * n + k] = 1.0;
  double fro = 0.0;
  for (auto &x : H) fro += std::norm(x);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(H[p * n + q]);
    if (off <= 1e-32 * (fro + 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd hpq = H[p * n + q];
        const double mag = std::abs(hpq);
        if (mag < 1e-300) continue;
        const cd ph = hpq / mag;
        const double a = H[p * n + p].real(), c = H[q * n + q].real();
        const double tau = (c - a) / (2.0 * mag);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        const cd Jpp = cs, Jpq = sn, Jqp = -sn * std::conj(ph), Jqq = cs * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // H <- H J
          const cd hp = H[k * n + p], hq = H[k * n + q];
          H[k * n + p] = hp * Jpp + hq * Jqp;
          H[k * n + q] = hp * Jpq + hq * Jqq;
        }
        for (int k = 0; k < n; ++k) {  // H <- J^+ H
          const cd hp = H[p * n + k], hq = H[q * n + k];
          H[p * n + k] = std::conj(Jpp) * hp + std::conj(Jqp) * hq;
          H[q * n + k] = std::conj(Jpq) * hp + std::conj(Jqq) * hq;
        }
        for (int k = 0; k < n; ++k) {  // V <- V J
          const cd vp = V[k * n + p], vq = V[k * n + q];
          V[k * n + p] = vp * Jpp + vq * Jqp;
          V[k * n + q] = vp * Jpq + vq * Jqq;
        }
      }
  }
  w.resize(n);
  for (int k = 0; k < n; ++k) w[k] = H[k * n + k].real();
}

// ---------------------------------------------------------------- device eigendata
struct TableSet {
  EigTables T;
  void *dev = nullptr;
};

static std::mutex g_tab_mu;
static std::map<std::pair<int, int>, TableSet> g_tabs;

static int build_tables(int d, TableSet *ts) {
  const int ps = packed_size(d);
  // layout: [V: NT * ps complex double][lam: NT * d*d double][A: NT * ps float2], NT = kTwoModeTypes
  constexpr int NT = kTwoModeTypes;
  const size_t nV = (size_t)NT * ps * 2, nL = (size_t)NT * d * d, nA = (size_t)NT * ps * 2;
  std::vector<double> hv(nV + nL, 0.0);
  std::vector<float> ha(nA, 0.f);
  const int D2 = d * d;
  for (int t = 0; t < NT; ++t) {
    const int type = t == table_slot(FOCK_CK) ? FOCK_CK : t;
    std::vector<double> A;
    generator_dense(type, d, A);
    const int kind = gate_kind(type);
    int off = 0, loff = 0;
    double leak = 0.0;
    std::vector<char> covered((size_t)D2 * D2, 0);
    for (int s = 0; s <= 2 * d - 2; ++s) {
      const int lo = block_lo(kind, d, s), b = block_hi(kind, d, s) - lo + 1;
      std::vector<int> li(b);
      for (int p = 0; p < b; ++p) {
        const int a = lo + p;
        const int nj = kind == KIND_SUM ? s - a : a - (s - (d - 1));
        li[p] = a * d + nj;
      }
      std::vector<cd> G(b * b);
      for (int p = 0; p < b; ++p)
        for (int q = 0; q < b; ++q) {
          const size_t e = (size_t)li[p] * D2 + li[q];
          covered[e] = 1;
          const cd Aval(A[2 * e], A[2 * e + 1]);
          G[p * b + q] = cd(0.0, -1.0) * Aval;  // G = -i A, Hermitian
          ha[(size_t)t * ps * 2 + 2 * (off + p * b + q)] = (float)Aval.real();
          ha[(size_t)t * ps * 2 + 2 * (off + p * b + q) + 1] = (float)Aval.imag();
        }
      std::vector<double> w;
      std::vector<cd> V;
      herm_jacobi(b, G, w, V);
      // residual check |G - V diag(w) V^+|
      double res = 0.0;
      for (int p = 0; p < b; ++p)
        for (int q = 0; q < b; ++q) {
          cd acc = 0.0;
          for (int m = 0; m < b; ++m) acc += V[p * b + m] * w[m] * std::conj(V[q * b + m]);
          res = std::max(res, std::abs(acc - G[p * b + q]));
        }
      if (res > 1e-11) return set_error(FOCK_ERR_HIP, "gate eigendata residual %.3g (type %d, d %d)", res, type, d);
      for (int k = 0; k < b * b; ++k) {
        hv[(size_t)t * ps * 2 + 2 * (off + k)] = V[k].real();
        hv[(size_t)t * ps * 2 + 2 * (off + k) + 1] = V[k].imag();
      }
      for (int m = 0; m < b; ++m) hv[nV + (size_t)t * D2 + loff + m] = w[m];
      off += b * b;
      loff += b;
    }
    for (size_t e = 0; e < (size_t)D2 * D2; ++e)
      if (!covered[e]) leak += std::fabs(A[2 * e]) + std::fabs(A[2 * e + 1]);
    if (leak != 0.0) return set_error(FOCK_ERR_HIP, "generator type %d has entries outside its blocks", type);
  }
  // single-mode squeezers: dense d x d eigendata of G = -i A, appended as
  // [V1: 2 * d*d complex double][lam1: 2 * d double] and [A1: 2 * d*d float2]
  const size_t nV1 = (size_t)2 * D2 * 2, nL1 = (size_t)2 * d, nA1 = (size_t)2 * D2 * 2;
  hv.resize(nV + nL + nV1 + nL1, 0.0);
  ha.resize(nA + nA1, 0.f);
  for (int t = 0; t < 2; ++t) {
    const int type = t == 0 ? FOCK_SR : FOCK_SI;
    std::vector<double> A;
    generator_dense(type, d, A);
    std::vector<cd> G(D2);
    for (int e = 0; e < D2; ++e) {
      G[e] = cd(0.0, -1.0) * cd(A[2 * e], A[2 * e + 1]);  // Hermitian
      ha[nA + (size_t)t * D2 * 2 + 2 * e] = (float)A[2 * e];
      ha[nA + (size_t)t * D2 * 2 + 2 * e + 1] = (float)A[2 * e + 1];
    }
    std::vector<double> w;
    std::vector<cd> V;
    herm_jacobi(d, G, w, V);
    double res = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q) {
        cd acc = 0.0;
        for (int m = 0; m < d; ++m) acc += V[p * d + m] * w[m] * std::conj(V[q * d + m]);
        res = std::max(res, std::abs(acc - G[p * d + q]));
      }
    if (res > 1e-11) return set_error(FOCK_ERR_HIP, "squeezer eigendata residual %.3g (type %d, d %d)", res, type, d);
    for (int e = 0; e < D2; ++e) {
      hv[nV + nL + (size_t)t * D2 * 2 + 2 * e] = V[e].real();
      hv[nV + nL + (size_t)t * D2 * 2 + 2 * e + 1] = V[e].imag();
    }
    for (int m = 0; m < d; ++m) hv[nV + nL + nV1 + (size_t)t * d + m] = w[m];
  }
  const size_t bytesD = (nV + nL + nV1 + nL1) * sizeof(double), bytesA = (nA + nA1) * sizeof(float);
  void *dev = nullptr;
  FOCK_HIP(hipMalloc(&dev, bytesD + bytesA));
  FOCK_HIP(hipMemcpy(dev, hv.data(), bytesD, hipMemcpyHostToDevice));
  FOCK_HIP(hipMemcpy((char *)dev + bytesD, ha.data(), bytesA, hipMemcpyHostToDevice));
  ts->dev = dev;
  const double *dV = (const double *)dev;
  const double *dL = dV + nV;
  const float2 *dA = (const float2 *)((const char *)dev + bytesD);
  for (int t = 0; t < NT; ++t) {
    ts->T.V[t] = dV + (size_t)t * ps * 2;
    ts->T.lam[t] = dL + (size_t)t * D2;
    ts->T.A[t] = dA + (size_t)t * ps;
  }
  for (int t = 0; t < 2; ++t) {
    ts->T.V1[t] = dV + nV + nL + (size_t)t * D2 * 2;
    ts->T.lam1[t] = dV + nV + nL + nV1 + (size_t)t * d;
    ts->T.A1[t] = dA + (nA / 2) + (size_t)t * D2;
  }
  ts->T.d = d;
  ts->T.psize = ps;
  return FOCK_OK;
}

int get_tables(int d, EigTables *out) {
  int dev = 0;
  FOCK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto key = std::make_pair(dev, d);
  auto it = g_tabs.find(key);
  if (it == g_tabs.end()) {
    TableSet ts;
    int rc = build_tables(d, &ts);
    if (rc) return rc;
    it = g_tabs.emplace(key, ts).first;
  }
  *out = it->second.T;
  return FOCK_OK;
}

// ---------------------------------------------------------------- stencil tile schedules
// Tile t of the stencil kernels has digits c_0..c_{m-1} (base d; c_k is the
// occupation of mode K+1+k, the modes above the LDS tile).  Workgroup b runs on
// XCD b % 8 (round-robin dispatch), as its (b / 8)-th workgroup there.  A
// schedule assigns every tile to an XCD and orders each XCD's tiles:
//   1: XCD = contiguous run (top digits), the highest free digit fastest;
//   2: XCD = octant of the top three digits (upper or lower half of each),
//      natural order inside;
//   3: octants, with the three top digits fastest inside.
// A schedule that does not divide the tiles evenly over the XCDs falls back
// to scheme 0 (contiguous runs, natural order; no table).
static std::atomic<int> g_sched{0};
static std::mutex g_ord_mu;
static std::map<std::tuple<int, int, int, int, int>, int *> g_ord;

static bool build_tile_order(int d, int ntiles, int scheme, std::vector<int> *out) {
  if (ntiles % 8 || ntiles < 64) return false;
  int m = 0;
  for (long t = 1; t < ntiles; t *= d) ++m;
  long pw = 1;
  for (int k = 0; k < m; ++k) pw *= d;
  if (pw != ntiles) return false;
  const int q = ntiles / 8, h = d / 2;
  if ((scheme == 2 || scheme == 3) && (m < 3 || d % 2)) return false;
  std::vector<std::vector<std::pair<long, int>>> xs(8);
  std::vector<int> c(m);
  for (int t = 0; t < ntiles; ++t) {
    int u = t;
    for (int k = 0; k < m; ++k) {
      c[k] = u % d;
      u /= d;
    }
    int x = 0;
    long key = 0;
    if (scheme == 1) {
      x = t / q;
      for (int k = 0; k < m; ++k) key = key * d + c[k];  // c_0 most significant
    } else {
      x = 4 * (c[m - 1] >= h) + 2 * (c[m - 2] >= h) + (c[m - 3] >= h);
      if (scheme == 2) {
        key = t;
      } else {
        for (int k = 0; k < m - 3; ++k) key = key * d + c[m - 4 - k];
        for (int k = m - 3; k < m; ++k) key = key * h + (c[k] % h);
      }
    }
    xs[x].push_back({key, t});
  }
  for (auto &v : xs)
    if ((int)v.size() != q) return false;
  out->assign(ntiles, 0);
  for (int x = 0; x < 8; ++x) {
    std::sort(xs[x].begin(), xs[x].end());
    for (int p = 0; p < q; ++p) (*out)[p * 8 + x] = xs[x][p].second;
  }
  return true;
}

int stencil_schedule() { return g_sched.load(); }

static std::atomic<int> g_stencil_variant{FOCK_STENCIL_SLAB};
int stencil_variant() { return g_stencil_variant.load(); }
bool lanes_stencil_ok(int L, int d, int periodic_wrap) { return d == 8 && L >= 4 && L <= 10 && !periodic_wrap; }
bool slab_stencil_ok(int L, int d) { return L == 8 && d == 8; }

int stencil_order_table(int L, int d, int ntiles, const int **order) {
  return stencil_order_table_for(L, d, ntiles, g_sched.load(), order);
}

int stencil_order_table_for(int L, int d, int ntiles, int scheme, const int **order) {
  *order = nullptr;
  if (scheme == 0 || scheme == FOCK_SCHED_TWO_PASS) return FOCK_OK;
  int dev = 0;
  FOCK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ord_mu);
  const auto key = std::make_tuple(dev, L, d, ntiles, scheme);
  auto it = g_ord.find(key);
  if (it == g_ord.end()) {
    std::vector<int> ord;
    int *p = nullptr;
    if (build_tile_order(d, ntiles, scheme, &ord)) {
      FOCK_HIP(hipMalloc(&p, sizeof(int) * ord.size()));
      FOCK_HIP(hipMemcpy(p, ord.data(), sizeof(int) * ord.size(), hipMemcpyHostToDevice));
    }
    it = g_ord.emplace(key, p).first;
  }
  *order = it->second;
  return FOCK_OK;
}

}  // namespace fock

extern "C" int fock_set_stencil_schedule(int scheme) {
  if (scheme < 0 || scheme >= FOCK_SCHED_NUM)
    return fock::set_error(FOCK_ERR_ARG, "stencil schedule %d out of range [0, %d)", scheme, FOCK_SCHED_NUM);
  fock::g_sched.store(scheme);
  return FOCK_OK;
}

extern "C" int fock_get_stencil_schedule(void) { return fock::g_sched.load(); }

extern "C" int fock_set_stencil_variant(int variant) {
  if (variant != FOCK_STENCIL_ROWS && variant != FOCK_STENCIL_LANES && variant != FOCK_STENCIL_SLAB)
    return fock::set_error(FOCK_ERR_ARG, "stencil variant %d is not ROWS (0), LANES (1) or SLAB (2)", variant);
  fock::g_stencil_variant.store(variant);
  return FOCK_OK;
}

extern "C" int fock_get_stencil_variant(void) { return fock::g_stencil_variant.load(); }

extern "C" int fock_stencil_schedule_table(int L, int d, int scheme, int *order, int n) {
  if (!order || n <= 0) return fock::set_error(FOCK_ERR_ARG, "NULL or empty order buffer");
  std::vector<int> ord;
  if (scheme == 0 || scheme == FOCK_SCHED_TWO_PASS || !fock::build_tile_order(d, n, scheme, &ord)) {
    for (int b = 0; b < n; ++b) {
      const int q = n >> 3;
      order[b] = b >= (q << 3) ? b : (b & 7) * q + (b >> 3);
    }
    (void)L;
    return FOCK_OK;
  }
  std::copy(ord.begin(), ord.end(), order);
  return FOCK_OK;
}

namespace fock {

// ---------------------------------------------------------------- profiling
struct ProfAcc {
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};
struct Pending {
  int id;
  double bytes;
  hipEvent_t e0, e1;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static int g_prof_every = 1;              // time one launch in g_prof_every per kernel id
static int64_t g_prof_seen[FOCK_K_NUM];   // launches seen per kernel id while enabled
static ProfAcc g_prof[FOCK_K_NUM];
static std::vector<Pending> g_pending;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(int id_, hipStream_t s_, double bytes_) : id(id_), s(s_), bytes(bytes_) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  if (id >= 0 && id < FOCK_K_NUM && (g_prof_seen[id]++ % g_prof_every) != 0) return;
  e0 = take_event();
  e1 = take_event();
  if (e0) hipEventRecord(e0, s);
}

ProfScope::~ProfScope() {
  if (!e0 || !e1) return;
  hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.push_back({id, bytes, e0, e1});
}

void prof_harvest() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<Pending> keep;
  for (auto &p : g_pending) {
    if (hipEventQuery(p.e1) != hipSuccess) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess && p.id >= 0 && p.id < FOCK_K_NUM) {
      g_prof[p.id].launches += 1;
      g_prof[p.id].ms += ms;
      g_prof[p.id].bytes += p.bytes;
    }
    g_event_pool.push_back(p.e0);
    g_event_pool.push_back(p.e1);
  }
  g_pending.swap(keep);
}

}  // namespace fock

extern "C" {

const char *fock_last_error(void) { return fock::last_error(); }

int fock_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(fock::g_prof_mu);
  fock::g_prof_on = on != 0;
  return FOCK_OK;
}

int fock_prof_set_sample(int every) {
  if (every < 1) return fock::set_error(FOCK_ERR_ARG, "sampling interval %d < 1", every);
  std::lock_guard<std::mutex> lk(fock::g_prof_mu);
  fock::g_prof_every = every;
  return FOCK_OK;
}

int fock_prof_query(int id, int64_t *launches, double *total_ms, double *bytes) {
  if (id < 0 || id >= FOCK_K_NUM) return fock::set_error(FOCK_ERR_ARG, "kernel id %d out of range", id);
  fock::prof_harvest();
  std::lock_guard<std::mutex> lk(fock::g_prof_mu);
  if (launches) *launches = fock::g_prof[id].launches;
  if (total_ms) *total_ms = fock::g_prof[id].ms;
  if (bytes) *bytes = fock::g_prof[id].bytes;
  return FOCK_OK;
}

int fock_prof_reset(void) {
  fock::prof_harvest();
  std::lock_guard<std::mutex> lk(fock::g_prof_mu);
  for (auto &p : fock::g_prof) p = fock::ProfAcc();
  for (auto &n : fock::g_prof_seen) n = 0;
  return FOCK_OK;
}

}  // extern "C"
