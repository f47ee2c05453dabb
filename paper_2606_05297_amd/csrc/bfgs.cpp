#include "bfgs.h"

#include <algorithm>
#include <cmath>

#include "../../include/fock.h"

namespace fock {

namespace {

double dot(const std::vector<double> &a, const std::vector<double> &b) {
  double s = 0.0;
  for (size_t k = 0; k < a.size(); ++k) s += a[k] * b[k];
  return s;
}
double inf_norm(const std::vector<double> &a) {
  double m = 0.0;
  for (double v : a) m = std::max(m, std::fabs(v));
  return m;
}

// Minimiser of the cubic interpolating (a, fa, ga) and (b, fb, gb), if any,
// clipped into the interval; falls back to bisection (N&W eq. 3.59).
double cubic_step(double a, double fa, double ga, double b, double fb, double gb) {
  const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - ga * gb;
  const double lo = std::min(a, b), hi = std::max(a, b);
  if (disc >= 0.0) {
    const double d2 = (b > a ? 1.0 : -1.0) * std::sqrt(disc);
    const double den = gb - ga + 2.0 * d2;
    if (den != 0.0) {
      const double t = b - (b - a) * (gb + d2 - d1) / den;
      const double w = hi - lo;
      if (t > lo + 0.1 * w && t < hi - 0.1 * w) return t;
    }
  }
  return 0.5 * (a + b);
}

struct LsPoint {
  double a, f, g;  // step, phi(a), phi'(a)
  std::vector<double> grad;
};

}  // namespace

int bfgs_minimize(std::vector<double> &x, const ObjFn &fn, double gtol, int maxiter, std::vector<double> *Hinv,
                  BfgsOut *out, double noise_rel) {
  const int n = (int)x.size();
  BfgsOut o;
  std::vector<double> g(n), xn(n), gn(n), p(n), s(n), y(n), Hy(n);
  double f = 0.0;
  int rc = fn(x, &f, &g);
  o.evals = 1;
  if (rc) return rc;
  o.f0 = f;
  std::vector<double> H;
  bool scaled = false;
  if (Hinv && (int)Hinv->size() == n * n) {
    H = *Hinv;
    scaled = true;
  } else {
    H.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) H[(size_t)k * n + k] = 1.0;
  }
  double f_prev = f + 0.5 * std::sqrt(dot(g, g));
  const double c1 = 1e-4, c2 = 0.9;
  int it = 0;
  for (; it < maxiter; ++it) {
    if (inf_norm(g) < gtol) break;
    for (int r = 0; r < n; ++r) {
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += H[(size_t)r * n + c] * g[c];
      p[r] = -acc;
    }
    double dphi0 = dot(g, p);
    if (!(dphi0 < 0.0)) {  // not a descent direction: restart from steepest descent
      for (int k = 0; k < n * n; ++k) H[k] = 0.0;
      for (int k = 0; k < n; ++k) H[(size_t)k * n + k] = 1.0;
      for (int k = 0; k < n; ++k) p[k] = -g[k];
      dphi0 = dot(g, p);
      scaled = false;
    }
    // Noise floor: stop once the predicted decrease is below the energy's
    // resolution.  Not before the first line search: until then the inverse
    // Hessian holds no curvature of the new direction (identity or a padded
    // recycled matrix) and its prediction g^2 / 2 can be far below the decrease
    // available along a soft direction.
    if (noise_rel > 0.0 && it > 0 && -0.5 * dphi0 < noise_rel * std::max(1.0, std::fabs(f))) {
      o.noise_stop = 1;
      break;
    }
    // initial trial step (as in SciPy: from the previous decrease, at most 1)
    double a1 = 1.0;
    if (dphi0 != 0.0) a1 = std::min(1.0, 1.01 * 2.0 * (f - f_prev) / dphi0);
    if (!(a1 > 0.0)) a1 = 1.0;

    auto phi = [&](double a, LsPoint *pt) -> int {
      for (int k = 0; k < n; ++k) xn[k] = x[k] + a * p[k];
      std::vector<double> gg(n);
      double ff = 0.0;
      int r = fn(xn, &ff, &gg);
      o.evals += 1;
      if (r) return r;
      pt->a = a;
      pt->f = ff;
      pt->g = dot(gg, p);
      pt->grad = std::move(gg);
      return 0;
    };

    // Alg. 3.5 (bracketing) + Alg. 3.6 (zoom)
    LsPoint prev{0.0, f, dphi0, g}, cur, acc;
    bool found = false, fail = false;
    double a = a1;
    const int max_ls = 20;
    for (int k = 0; k < max_ls && !found && !fail; ++k) {
      rc = phi(a, &cur);
      if (rc) return rc;
      LsPoint lo, hi;
      bool zoom = false;
      if (!std::isfinite(cur.f) || cur.f > f + c1 * a * dphi0 || (k > 0 && cur.f >= prev.f)) {
        lo = prev;
        hi = cur;
        zoom = true;
      } else if (std::fabs(cur.g) <= -c2 * dphi0) {
        acc = cur;
        found = true;
      } else if (cur.g >= 0.0) {
        lo = cur;
        hi = prev;
        zoom = true;
      } else {
        prev = cur;
        a = std::min(2.0 * a, 1e6);
        continue;
      }
      if (zoom) {
        for (int z = 0; z < max_ls; ++z) {
          double aj;
          if (std::isfinite(hi.f)) aj = cubic_step(lo.a, lo.f, lo.g, hi.a, hi.f, hi.g);
          else aj = 0.5 * (lo.a + hi.a);
          if (std::fabs(hi.a - lo.a) < 1e-14 * std::max(1.0, std::fabs(lo.a))) break;
          LsPoint pj;
          rc = phi(aj, &pj);
          if (rc) return rc;
          if (!std::isfinite(pj.f) || pj.f > f + c1 * aj * dphi0 || pj.f >= lo.f) {
            hi = pj;
          } else {
            if (std::fabs(pj.g) <= -c2 * dphi0) {
              acc = pj;
              found = true;
              break;
            }
            if (pj.g * (hi.a - lo.a) >= 0.0) hi = lo;
            lo = pj;
          }
        }
        if (!found) {
          // accept a point with sufficient decrease if the zoom stalled
          if (lo.a > 0.0 && lo.f < f) {
            acc = lo;
            found = true;
          } else {
            fail = true;
          }
        }
      }
    }
    if (!found) {
      o.status = FOCK_ERR_LINESEARCH;
      break;
    }
    for (int k = 0; k < n; ++k) {
      s[k] = acc.a * p[k];
      xn[k] = x[k] + s[k];
      y[k] = acc.grad[k] - g[k];
    }
    const double ys = dot(y, s);
    if (!scaled && ys > 0.0) {  // N&W eq. (6.20): H0 = (y's / y'y) I before the first update
      const double gam = ys / dot(y, y);
      for (int k = 0; k < n * n; ++k) H[k] = 0.0;
      for (int k = 0; k < n; ++k) H[(size_t)k * n + k] = gam;
      scaled = true;
    }
    if (ys > 1e-300) {
      const double rho = 1.0 / ys;
      for (int r = 0; r < n; ++r) {
        double acc2 = 0.0;
        for (int c = 0; c < n; ++c) acc2 += H[(size_t)r * n + c] * y[c];
        Hy[r] = acc2;
      }
      const double yHy = dot(y, Hy);
      // H <- (I - rho s y')H(I - rho y s') + rho s s'
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c)
          H[(size_t)r * n + c] += -rho * (Hy[r] * s[c] + s[r] * Hy[c]) + (rho * rho * yHy + rho) * s[r] * s[c];
    }
    f_prev = f;
    x.swap(xn);
    f = acc.f;
    g = acc.grad;
  }
  o.iters = it;
  o.f = f;
  o.ginf = inf_norm(g);
  if (Hinv) *Hinv = H;
  *out = o;
  return 0;
}

}  // namespace fock
