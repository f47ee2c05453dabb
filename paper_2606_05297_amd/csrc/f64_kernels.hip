// FP64-state path (complex128 amplitudes) for runs that must resolve energy
// differences below the complex64 state's ~1e-7 relative rounding, as the
// paper's convergence to ~1e-10 does.  The kernels are plain (not tiled) and
// meant for the small lattices of those runs:
//   k64_apply_h     H psi (Sec. III), one thread per amplitude, every bond
//                   term read directly from global memory, FP64 energy/norm
//                   partials per workgroup;
//   k64_fib_apply   psi <- U psi (U^+ psi) with a dense M x M local matrix on
//                   every fibre (M = d^2 amplitudes over (n_i, n_j), or d over
//                   one mode), fibres (and matrices up to 36 x 36) staged in
//                   LDS, one thread per output;
//   k64_fib_adj     reverse step: Re<lam|A phi> per workgroup, then U^+ on
//                   phi and lam;
//   k64_fib_pool    2 Re<hpsi|A psi> per workgroup for one pool entry;
//   k64_build       dense U = exp(theta A) of every gate from the FP64
//                   eigendata (blocks of the two-mode types, dense d x d for
//                   the squeezers, phases for K and R).
#include "f64_internal.h"

namespace fock {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(kBlock) void k64_apply_h(const double2 *__restrict__ psi, double2 *__restrict__ hpsi,
                                                      double *__restrict__ partial, H64 h) {
  __shared__ double red[4];
  const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
  double e = 0.0, nn = 0.0;
  if (idx < h.n_amp) {
    int n[kMaxL];
    uint32_t st[kMaxL];
    {
      uint32_t t = idx, s = 1;
      for (int r = 0; r < h.L; ++r) {
        n[r] = (int)(t % (uint32_t)h.d);
        t /= (uint32_t)h.d;
        st[r] = s;
        s *= (uint32_t)h.d;
      }
    }
    const double2 x = psi[idx];
    double dg = 0.0;
    for (int r = 0; r < h.L; ++r) dg += h.c2 * n[r] * (n[r] - 1.0) - h.mu * n[r];
    double2 y = make_double2(dg * x.x, dg * x.y);
    const int nb = h.L - 1 + h.wrap;
    for (int b = 0; b < nb; ++b) {
      const int i = b < h.L - 1 ? b : 0, j = b < h.L - 1 ? b + 1 : h.L - 1;
      const int ni = n[i], nj = n[j];
      const uint32_t si = st[i], sj = st[j];
      auto add = [&](double c, uint32_t k) {
        const double2 v = psi[k];
        y.x += c * v.x;
        y.y += c * v.y;
      };
      if (h.J != 0.0) {
        if (ni >= 1 && nj <= h.d - 2) add(-h.J * sqrt((double)ni) * sqrt(nj + 1.0), idx - si + sj);
        if (ni <= h.d - 2 && nj >= 1) add(-h.J * sqrt(ni + 1.0) * sqrt((double)nj), idx + si - sj);
      }
      if (h.Delta != 0.0) {
        if (ni <= h.d - 2 && nj <= h.d - 2) add(h.Delta * sqrt(ni + 1.0) * sqrt(nj + 1.0), idx + si + sj);
        if (ni >= 1 && nj >= 1) add(h.Delta * sqrt((double)ni) * sqrt((double)nj), idx - si - sj);
      }
    }
    hpsi[idx] = y;
    e = x.x * y.x + x.y * y.y;
    nn = x.x * x.x + x.y * x.y;
  }
  const double se = block_sum_d(e, red);
  const double sn = block_sum_d(nn, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = se;
    partial[2 * blockIdx.x + 1] = sn;
  }
}

// Base amplitude of fibre f: its digits fill the modes other than i and j.
__device__ __forceinline__ uint32_t fib_base(uint32_t f, const Fib64 &a) {
  uint32_t base = 0, t = f, p = 1;
  for (int r = 0; r < a.L; ++r) {
    if (r != a.i && r != a.j) {
      base += (t % (uint32_t)a.d) * p;
      t /= (uint32_t)a.d;
    }
    p *= (uint32_t)a.d;
  }
  return base;
}

// Offset of member m (n_i d + n_j, or n_i for one mode) inside a fibre.
__device__ __forceinline__ uint32_t fib_off(int m, const Fib64 &a) {
  return a.j >= 0 ? (uint32_t)(m / a.d) * a.si + (uint32_t)(m % a.d) * a.sj : (uint32_t)m * a.si;
}

// Local matrices of up to kStage entries (M <= 36: every one-mode gate at
// d <= 36 and two-mode gates at d <= 6) are staged in LDS once per workgroup,
// so the per-thread loops below read LDS; larger ones are read from global
// memory (L2) as they are.
constexpr int kStage = 36 * 36;

template <bool STAGE>
__global__ __launch_bounds__(kBlock) void k64_fib_apply(const double2 *src, double2 *dst,
                                                        const double2 *__restrict__ U, Fib64 a, int dag) {
  __shared__ double2 x[kBlock];
  __shared__ double2 Us[STAGE ? kStage : 1];
  const int M = a.M, fpw = a.fpw;
  const int fl = threadIdx.x / M, p = threadIdx.x % M;
  const uint32_t f = blockIdx.x * (uint32_t)fpw + (uint32_t)fl;
  const bool on = fl < fpw && f < a.nfib;
  if constexpr (STAGE)
    for (int e = threadIdx.x; e < M * M; e += kBlock) Us[e] = U[e];
  uint32_t base = 0;
  if (on) {
    base = fib_base(f, a);
    x[threadIdx.x] = src[base + fib_off(p, a)];
  }
  __syncthreads();
  if (on) {
    const double2 *xf = x + fl * M;
    double yr = 0.0, yi = 0.0;
    for (int q = 0; q < M; ++q) {
      const int e = dag ? q * M + p : p * M + q;
      double2 u;
      if constexpr (STAGE) u = Us[e];
      else u = U[e];
      if (dag) u.y = -u.y;
      yr += u.x * xf[q].x - u.y * xf[q].y;
      yi += u.x * xf[q].y + u.y * xf[q].x;
    }
    dst[base + fib_off(p, a)] = make_double2(yr, yi);
  }
}

template <bool STAGE>
__global__ __launch_bounds__(kBlock) void k64_fib_adj(double2 *__restrict__ phi, double2 *__restrict__ lam,
                                                      const double2 *__restrict__ U, const double2 *__restrict__ A,
                                                      double *__restrict__ partial, Fib64 a) {
  __shared__ double2 x[kBlock], l[kBlock];
  __shared__ double2 Us[STAGE ? kStage : 1], As[STAGE ? kStage : 1];
  __shared__ double red[4];
  const int M = a.M, fpw = a.fpw;
  const int fl = threadIdx.x / M, p = threadIdx.x % M;
  const uint32_t f = blockIdx.x * (uint32_t)fpw + (uint32_t)fl;
  const bool on = fl < fpw && f < a.nfib;
  if constexpr (STAGE)
    for (int e = threadIdx.x; e < M * M; e += kBlock) {
      Us[e] = U[e];
      As[e] = A[e];
    }
  uint32_t base = 0;
  if (on) {
    base = fib_base(f, a);
    x[threadIdx.x] = phi[base + fib_off(p, a)];
    l[threadIdx.x] = lam[base + fib_off(p, a)];
  }
  __syncthreads();
  double g = 0.0;
  if (on) {
    const double2 *xf = x + fl * M, *lf = l + fl * M;
    double ar = 0.0, ai = 0.0, pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
    for (int q = 0; q < M; ++q) {
      double2 av, u;  // u = U[q][p]: (U^+)[p][q] = conj(U[q][p])
      if constexpr (STAGE) {
        av = As[p * M + q];
        u = Us[q * M + p];
      } else {
        av = A[(size_t)p * M + q];
        u = U[(size_t)q * M + p];
      }
      ar += av.x * xf[q].x - av.y * xf[q].y;
      ai += av.x * xf[q].y + av.y * xf[q].x;
      pr += u.x * xf[q].x + u.y * xf[q].y;
      pi += u.x * xf[q].y - u.y * xf[q].x;
      qr += u.x * lf[q].x + u.y * lf[q].y;
      qi += u.x * lf[q].y - u.y * lf[q].x;
    }
    g = lf[p].x * ar + lf[p].y * ai;  // Re(conj(lam_p) (A phi)_p)
    phi[base + fib_off(p, a)] = make_double2(pr, pi);
    lam[base + fib_off(p, a)] = make_double2(qr, qi);
  }
  const double s = block_sum_d(g, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <bool STAGE>
__global__ __launch_bounds__(kBlock) void k64_fib_pool(const double2 *__restrict__ psi,
                                                       const double2 *__restrict__ hpsi,
                                                       const double2 *__restrict__ A, double *__restrict__ partial,
                                                       Fib64 a) {
  __shared__ double2 x[kBlock];
  __shared__ double2 As[STAGE ? kStage : 1];
  __shared__ double red[4];
  const int M = a.M, fpw = a.fpw;
  const int fl = threadIdx.x / M, p = threadIdx.x % M;
  const uint32_t f = blockIdx.x * (uint32_t)fpw + (uint32_t)fl;
  const bool on = fl < fpw && f < a.nfib;
  if constexpr (STAGE)
    for (int e = threadIdx.x; e < M * M; e += kBlock) As[e] = A[e];
  uint32_t base = 0;
  double2 h = make_double2(0.0, 0.0);
  if (on) {
    base = fib_base(f, a);
    x[threadIdx.x] = psi[base + fib_off(p, a)];
    h = hpsi[base + fib_off(p, a)];
  }
  __syncthreads();
  double v = 0.0;
  if (on) {
    const double2 *xf = x + fl * M;
    double ar = 0.0, ai = 0.0;
    for (int q = 0; q < M; ++q) {
      double2 av;
      if constexpr (STAGE) av = As[p * M + q];
      else av = A[(size_t)p * M + q];
      ar += av.x * xf[q].x - av.y * xf[q].y;
      ai += av.x * xf[q].y + av.y * xf[q].x;
    }
    v = 2.0 * (h.x * ar + h.y * ai);
  }
  const double s = block_sum_d(v, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Dense U of gate k (recs[k]: type, offset of its M x M table) from the FP64
// eigendata; entry e = p M + q.
__global__ __launch_bounds__(kBlock) void k64_build(const double *__restrict__ theta, const GateRec *__restrict__ recs,
                                                    int n, EigTables T, double2 *__restrict__ utab) {
  const int k = blockIdx.y;
  if (k >= n) return;
  const GateRec r = recs[k];
  const int d = T.d;
  const bool one = r.type == FOCK_KERR || r.type == FOCK_ROT || r.type == FOCK_SR || r.type == FOCK_SI;
  const int M = one ? d : d * d;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= M * M) return;
  const int p = e / M, q = e % M;
  const double th = theta[k];
  double ur = 0.0, ui = 0.0;
  if (r.type == FOCK_KERR || r.type == FOCK_ROT) {
    if (p == q) {
      const double f = r.type == FOCK_KERR ? (double)p * p : (double)p;
      sincos(th * f, &ui, &ur);
    }
  } else if (one) {
    const int t = r.type == FOCK_SR ? 0 : 1;
    const double *V = T.V1[t], *lam = T.lam1[t];
    for (int m = 0; m < d; ++m) {
      double sn, cs;
      sincos(th * lam[m], &sn, &cs);
      const double pr = V[2 * (p * d + m)], pi = V[2 * (p * d + m) + 1];
      const double qr = V[2 * (q * d + m)], qi = V[2 * (q * d + m) + 1];
      const double tr = pr * cs - pi * sn, ti = pr * sn + pi * cs;
      ur += tr * qr + ti * qi;
      ui += ti * qr - tr * qi;
    }
  } else {
    // two-mode: members p = (a, b), q = (c, e) lie in one conserved block or U = 0
    const int kind = (r.type == FOCK_PR || r.type == FOCK_PI) ? KIND_DIFF : KIND_SUM;
    const int pa = p / d, pb = p % d, qa = q / d, qb = q % d;
    const int sp = kind == KIND_SUM ? pa + pb : pa - pb + (d - 1);
    const int sq = kind == KIND_SUM ? qa + qb : qa - qb + (d - 1);
    if (sp == sq) {
      int off = 0, loff = 0;
      for (int s = 0; s < sp; ++s) {
        const int bs = blk_hi(kind, d, s) - blk_lo(kind, d, s) + 1;
        off += bs * bs;
        loff += bs;
      }
      const int lo = blk_lo(kind, d, sp), b = blk_hi(kind, d, sp) - lo + 1;
      const int pl = pa - lo, ql = qa - lo;
      const int t = table_slot(r.type);
      const double *V = T.V[t] + 2 * off, *lam = T.lam[t] + loff;
      for (int m = 0; m < b; ++m) {
        double sn, cs;
        sincos(th * lam[m], &sn, &cs);
        const double pr = V[2 * (pl * b + m)], pi = V[2 * (pl * b + m) + 1];
        const double qr = V[2 * (ql * b + m)], qi = V[2 * (ql * b + m) + 1];
        const double tr = pr * cs - pi * sn, ti = pr * sn + pi * cs;
        ur += tr * qr + ti * qi;
        ui += ti * qr - tr * qi;
      }
    }
  }
  utab[(size_t)r.u_off + e] = make_double2(ur, ui);
}

Fib64 make_fib64(int L, int d, const fock_op_t &op) {
  Fib64 a;
  a.L = L;
  a.d = d;
  const bool one = op.j < 0;
  a.i = op.i;
  a.j = one ? -1 : op.j;
  uint32_t s = 1;
  for (int r = 0; r < op.i; ++r) s *= (uint32_t)d;
  a.si = s;
  s = 1;
  for (int r = 0; r < (one ? 0 : op.j); ++r) s *= (uint32_t)d;
  a.sj = one ? 0 : s;
  a.M = one ? d : d * d;
  uint32_t na = 1;
  for (int r = 0; r < L; ++r) na *= (uint32_t)d;
  a.nfib = na / (uint32_t)a.M;
  a.fpw = kBlock / a.M > 0 ? kBlock / a.M : 1;
  return a;
}

int fib64_blocks(const Fib64 &a) { return (int)((a.nfib + (uint32_t)a.fpw - 1) / (uint32_t)a.fpw); }

int launch64_apply_h(const H64 &h, const double2 *psi, double2 *hpsi, double *partial, int *nblocks, hipStream_t s) {
  *nblocks = (int)((h.n_amp + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k64_apply_h, dim3(*nblocks), dim3(kBlock), 0, s, psi, hpsi, partial, h);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch64_fib_apply(const Fib64 &a, const double2 *src, double2 *dst, const double2 *U, bool dag, hipStream_t s) {
  if (a.M * a.M <= kStage)
    hipLaunchKernelGGL(k64_fib_apply<true>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, src, dst, U, a, dag ? 1 : 0);
  else
    hipLaunchKernelGGL(k64_fib_apply<false>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, src, dst, U, a, dag ? 1 : 0);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch64_fib_adj(const Fib64 &a, double2 *phi, double2 *lam, const double2 *U, const double2 *A,
                     double *partial, hipStream_t s) {
  if (a.M * a.M <= kStage)
    hipLaunchKernelGGL(k64_fib_adj<true>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, phi, lam, U, A, partial, a);
  else
    hipLaunchKernelGGL(k64_fib_adj<false>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, phi, lam, U, A, partial, a);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch64_fib_pool(const Fib64 &a, const double2 *psi, const double2 *hpsi, const double2 *A, double *partial,
                      hipStream_t s) {
  if (a.M * a.M <= kStage)
    hipLaunchKernelGGL(k64_fib_pool<true>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, psi, hpsi, A, partial, a);
  else
    hipLaunchKernelGGL(k64_fib_pool<false>, dim3(fib64_blocks(a)), dim3(kBlock), 0, s, psi, hpsi, A, partial, a);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch64_build(const double *theta, const GateRec *recs, int n, const EigTables &T, int Mmax, double2 *utab,
                   hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  hipLaunchKernelGGL(k64_build, dim3((Mmax * Mmax + kBlock - 1) / kBlock, n), dim3(kBlock), 0, s, theta, recs, n, T,
                     utab);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace fock
