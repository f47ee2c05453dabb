// Quasi-Newton minimiser used to re-optimise the ansatz angles (Sec. V.A:
// BFGS, L-infinity gradient tolerance, iteration cap).
#pragma once

#include <functional>
#include <vector>

namespace fock {

// f(x) and its gradient; returns 0 or a negative FOCK_ERR_* code.
using ObjFn = std::function<int(const std::vector<double> &x, double *f, std::vector<double> *g)>;

struct BfgsOut {
  int iters = 0, evals = 0, status = 0, noise_stop = 0;
  double f = 0.0, f0 = 0.0, ginf = 0.0;
};

// BFGS with a strong-Wolfe line search (Nocedal & Wright, Alg. 6.1 with
// Alg. 3.5/3.6, c1 = 1e-4, c2 = 0.9).  Stops when ||g||_inf < gtol or after
// maxiter iterations; on a line-search failure it keeps the last accepted
// point and reports FOCK_ERR_LINESEARCH.  If Hinv is non-null and holds an
// n x n matrix, it seeds the inverse Hessian (otherwise the first step is
// scaled by y's/y'y) and receives the final inverse Hessian.  With
// noise_rel > 0 the run also stops (successfully) once the decrease predicted
// for a full quasi-Newton step, -g'p/2, falls below noise_rel * max(1, |f|):
// below that level the objective's rounding noise hides any progress.
int bfgs_minimize(std::vector<double> &x, const ObjFn &fn, double gtol, int maxiter,
                  std::vector<double> *Hinv, BfgsOut *out, double noise_rel = 0.0);

}  // namespace fock
