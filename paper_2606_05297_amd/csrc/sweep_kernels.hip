// Batched kernels for many ADAPT points of uneven (L, d) in one launch per
// phase.  A launch walks a list of work items (point, workgroup index) with a
// grid-stride loop over a grid sized to the GPU (persistent workgroups); each
// item runs exactly the per-workgroup device function the single-point
// kernels use, so every point's result is bit-identical to its unbatched run.
// Items of points whose BFGS is idle this round are skipped through a device
// "active" flag, so one captured graph serves every round of a phase.
#include "sweep_internal.h"

namespace fock {

// An item's run descriptor copied to LDS by the whole workgroup (items are
// uniform per workgroup).  The first barrier keeps the previous item's readers
// of the descriptor ahead of the copy.
__device__ __forceinline__ void load_run(const SweepItem &g, DiagRun *dst) {
  __syncthreads();
  const __attribute__((address_space(4))) int *src = (const __attribute__((address_space(4))) int *)g.run.p;
  int *d = (int *)dst;
  for (int e = threadIdx.x; e < (int)(sizeof(DiagRun) / 4); e += kBlock) d[e] = src[e];
  __syncthreads();
}

// Reverse step of a run item: all of its gates' workgroup sums.
template <int D>
__device__ __forceinline__ void sweep_run_adj(const SweepItem &g, DiagRun *srun, float2 *tb, float2 *t0,
                                              double (*dred)[kMaxDiagRun]) {
  load_run(g, srun);
  diag_run_adj_block<D, true>(g.vb, g.dst, g.lam, g.U, *srun, tb, t0, dred);
  if ((int)threadIdx.x < srun->ng) {
    const int q = threadIdx.x;
    g.partial[(size_t)q * g.rs + g.vb] = (dred[0][q] + dred[1][q]) + (dred[2][q] + dred[3][q]);
  }
}

// Gate and reverse-step items of one gate layer: at d = 8 they come in two
// classes launched separately, so that each kernel declares only the LDS its
// items use (64 kB of mode-0 tiles would otherwise cap the occupancy of the
// direct items): class 0 = two-mode gates on modes i >= 1 and single-mode
// phases, class 1 = two-mode gates on mode 0.  At d <= 6 the mode-0 tiles are
// small and one launch per layer runs all items (fewer launches for the small
// states, whose kernels are short).
template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_gate_all(const SweepItem *__restrict__ items, int n,
                                                           const int *__restrict__ active) {
  __shared__ float2 tile[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[lds_fibers<D>()];
  __shared__ float2 phs[kMaxD];
  __shared__ DiagRun srun;
  __shared__ float2 tb[kMaxDiagRun * D], t0[D];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    switch (g.variant * 2 + g.kind) {
      case 0: gate2_direct_block<D, KIND_SUM, false>(g.vb, g.src, g.dst, g.U, g.gl); break;
      case 1: gate2_direct_block<D, KIND_DIFF, false>(g.vb, g.src, g.dst, g.U, g.gl); break;
      case 2: gate2_m0_block<D, KIND_SUM, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase); break;
      case 3: gate2_m0_block<D, KIND_DIFF, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase); break;
      case 6:
        load_run(g, &srun);
        diag_run_block<D, false>(g.vb, g.src, g.dst, g.U, srun, tb, t0);
        break;
      default: diag_block<D, false>(g.vb, g.src, g.dst, g.U, g.dl, phs); break;
    }
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_adj_all(const SweepItem *__restrict__ items, int n,
                                                          const int *__restrict__ active) {
  __shared__ float2 tp[m0_tile_elems<D>()], tl[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[lds_fibers<D>()];
  __shared__ float2 phs[kMaxD];
  __shared__ double red[4];
  __shared__ DiagRun srun;
  __shared__ float2 tb[kMaxDiagRun * D], t0[D];
  __shared__ double dred[kBlock / 64][kMaxDiagRun];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    if (g.variant == 3) {
      sweep_run_adj<D>(g, &srun, tb, t0, dred);
      continue;
    }
    float gacc = 0.f;
    switch (g.variant * 2 + g.kind) {
      case 0: gacc = adj_direct_block<D, KIND_SUM>(g.vb, g.dst, g.lam, g.U, g.A, g.gl); break;
      case 1: gacc = adj_direct_block<D, KIND_DIFF>(g.vb, g.dst, g.lam, g.U, g.A, g.gl); break;
      case 2: gacc = adj_m0_block<D, KIND_SUM>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase); break;
      case 3: gacc = adj_m0_block<D, KIND_DIFF>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase); break;
      default: gacc = diag_adj_block<D>(g.vb, g.dst, g.lam, g.U, g.dl, phs); break;
    }
    const double sg = block_sum_d((double)gacc, red);
    if (threadIdx.x == 0) g.partial[g.vb] = sg;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_gate(const SweepItem *__restrict__ items, int n,
                                                       const int *__restrict__ active) {
  __shared__ float2 phs[kMaxD];
  __shared__ DiagRun srun;
  __shared__ float2 tb[kMaxDiagRun * D], t0[D];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    switch (g.variant * 2 + g.kind) {
      case 0: gate2_direct_block<D, KIND_SUM, false>(g.vb, g.src, g.dst, g.U, g.gl); break;
      case 1: gate2_direct_block<D, KIND_DIFF, false>(g.vb, g.src, g.dst, g.U, g.gl); break;
      case 6:
        load_run(g, &srun);
        diag_run_block<D, false>(g.vb, g.src, g.dst, g.U, srun, tb, t0);
        break;
      default: diag_block<D, false>(g.vb, g.src, g.dst, g.U, g.dl, phs); break;
    }
  }
}

// Mode-0 items at d = 8: variant 4 items run the pipelined multi-tile block of
// the single-point kernels (same tiles per workgroup, same summation order).
template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_gate_m0(const SweepItem *__restrict__ items, int n,
                                                          const int *__restrict__ active) {
  __shared__ float2 tile[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[2][lds_fibers<D>()];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    if (g.variant == 4) {
      __syncthreads();  // the previous item's readers of fbase are done
      if (g.kind == KIND_SUM) gate2_m0p_block<D, KIND_SUM, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase);
      else gate2_m0p_block<D, KIND_DIFF, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase);
    } else if (g.kind == KIND_SUM) {
      gate2_m0_block<D, KIND_SUM, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase[0]);
    } else {
      gate2_m0_block<D, KIND_DIFF, false>(g.vb, g.src, g.dst, g.U, g.gl, tile, fbase[0]);
    }
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_adj(const SweepItem *__restrict__ items, int n,
                                                      const int *__restrict__ active) {
  __shared__ float2 phs[kMaxD];
  __shared__ double red[4];
  __shared__ DiagRun srun;
  __shared__ float2 tb[kMaxDiagRun * D], t0[D];
  __shared__ double dred[kBlock / 64][kMaxDiagRun];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    if (g.variant == 3) {
      sweep_run_adj<D>(g, &srun, tb, t0, dred);
      continue;
    }
    float gacc = 0.f;
    switch (g.variant * 2 + g.kind) {
      case 0: gacc = adj_direct_block<D, KIND_SUM>(g.vb, g.dst, g.lam, g.U, g.A, g.gl); break;
      case 1: gacc = adj_direct_block<D, KIND_DIFF>(g.vb, g.dst, g.lam, g.U, g.A, g.gl); break;
      default: gacc = diag_adj_block<D>(g.vb, g.dst, g.lam, g.U, g.dl, phs); break;
    }
    const double sg = block_sum_d((double)gacc, red);
    if (threadIdx.x == 0) g.partial[g.vb] = sg;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_adj_m0(const SweepItem *__restrict__ items, int n,
                                                         const int *__restrict__ active) {
  __shared__ float2 tp[m0_tile_elems<D>()], tl[m0_tile_elems<D>()];
  __shared__ uint32_t fbase[2][lds_fibers<D>()];
  __shared__ double red[4];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepItem g = items[it];
    if (!active[g.p]) continue;
    float gacc;
    if (g.variant == 4) {
      __syncthreads();  // the previous item's readers of fbase are done
      gacc = g.kind == KIND_SUM ? adj_m0p_block<D, KIND_SUM>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase)
                                : adj_m0p_block<D, KIND_DIFF>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase);
    } else {
      gacc = g.kind == KIND_SUM ? adj_m0_block<D, KIND_SUM>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase[0])
                                : adj_m0_block<D, KIND_DIFF>(g.vb, g.dst, g.lam, g.U, g.A, g.gl, tp, tl, fbase[0]);
    }
    const double sg = block_sum_d((double)gacc, red);
    if (threadIdx.x == 0) g.partial[g.vb] = sg;
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_h(const SweepHItem *__restrict__ items, int n,
                                                    const HamArgs *__restrict__ hams, const int *__restrict__ active) {
  __shared__ double red[4];
  __shared__ float4 tile4[TileCfg<D>::PWORDS];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepHItem g = items[it];
    if (!active[g.p]) continue;
    float e = 0.f, nn = 0.f;
    hblock<D>(g.vb, g.psi, g.hpsi, hams[g.p], reinterpret_cast<float2 *>(tile4), e, nn);
    const double se = block_sum_d((double)e, red);
    const double sn = block_sum_d((double)nn, red);
    if (threadIdx.x == 0) {
      g.partial[2 * g.vb] = se;
      g.partial[2 * g.vb + 1] = sn;
    }
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sweep_pool(const SweepHItem *__restrict__ items, int n,
                                                       const SweepPoolArgs *__restrict__ pa,
                                                       const int *__restrict__ active) {
  __shared__ double acc[4][kMaxSlots];
  __shared__ float4 tile4[(PTile<D>::MAXROWS * PTile<D>::RS + 1) / 2];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepHItem g = items[it];
    if (!active[g.p]) continue;
    const SweepPoolArgs &a = pa[g.p];
    pool_block<D>(g.vb, g.psi, g.hpsi, g.partial, a.args, a.pairs, a.diags, reinterpret_cast<float2 *>(tile4), acc);
  }
}

// out = sum of a column (mode 0: partial[b * ncols + col], b < nblocks) or of
// a row (mode 1: partial[col * stride + b], b < nblocks), fixed order.
__global__ __launch_bounds__(kBlock) void k_sweep_reduce(const SweepRItem *__restrict__ items, int n,
                                                         const int *__restrict__ active) {
  __shared__ double red[4];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const SweepRItem g = items[it];
    if (!active[g.p]) continue;
    double s = 0.0;
    for (int b = threadIdx.x; b < g.nblocks; b += kBlock)
      s += g.mode == 0 ? g.partial[(size_t)b * g.ncols + g.col] : g.partial[(size_t)g.col * g.stride + b];
    s = block_sum_d(s, red);
    if (threadIdx.x == 0) g.out[0] = s;
  }
}

#define SWEEP_D_SWITCH(d, STMT)                                                    \
  switch (d) {                                                                     \
    case 4: { constexpr int D = 4; STMT; } break;                                  \
    case 6: { constexpr int D = 6; STMT; } break;                                  \
    case 8: { constexpr int D = 8; STMT; } break;                                  \
    default: return set_error(FOCK_ERR_UNSUPPORTED, "sweep kernels need d in {4, 6, 8}, got %d", d); \
  }

bool sweep_supports_d(int d) { return d == 4 || d == 6 || d == 8; }

bool sweep_split_classes(int d) { return d == 8; }

int sweep_launch_gate(int d, int cls, const SweepItem *items, int n, const int *active, int grid,
                      hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  const dim3 g(grid < n ? grid : n);
  if (!sweep_split_classes(d))
    SWEEP_D_SWITCH(d, hipLaunchKernelGGL(k_sweep_gate_all<D>, g, dim3(kBlock), 0, s, items, n, active))
  else if (cls == 0)
    hipLaunchKernelGGL(k_sweep_gate<8>, g, dim3(kBlock), 0, s, items, n, active);
  else
    hipLaunchKernelGGL(k_sweep_gate_m0<8>, g, dim3(kBlock), 0, s, items, n, active);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int sweep_launch_adj(int d, int cls, const SweepItem *items, int n, const int *active, int grid, hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  const dim3 g(grid < n ? grid : n);
  if (!sweep_split_classes(d))
    SWEEP_D_SWITCH(d, hipLaunchKernelGGL(k_sweep_adj_all<D>, g, dim3(kBlock), 0, s, items, n, active))
  else if (cls == 0)
    hipLaunchKernelGGL(k_sweep_adj<8>, g, dim3(kBlock), 0, s, items, n, active);
  else
    hipLaunchKernelGGL(k_sweep_adj_m0<8>, g, dim3(kBlock), 0, s, items, n, active);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int sweep_launch_h(int d, const SweepHItem *items, int n, const HamArgs *hams, const int *active, int grid,
                   hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  SWEEP_D_SWITCH(d, hipLaunchKernelGGL(k_sweep_h<D>, dim3(grid < n ? grid : n), dim3(kBlock), 0, s, items, n, hams,
                                       active));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int sweep_launch_pool(int d, const SweepHItem *items, int n, const SweepPoolArgs *pa, const int *active, int grid,
                      hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  SWEEP_D_SWITCH(d, hipLaunchKernelGGL(k_sweep_pool<D>, dim3(grid < n ? grid : n), dim3(kBlock), 0, s, items, n,
                                       pa, active));
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int sweep_launch_reduce(const SweepRItem *items, int n, const int *active, int grid, hipStream_t s) {
  if (n <= 0) return FOCK_OK;
  hipLaunchKernelGGL(k_sweep_reduce, dim3(grid < n ? grid : n), dim3(kBlock), 0, s, items, n, active);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

// The single-point kernels' launch geometry, needed to build item lists.
int sweep_gate_blocks(int d, int namp, int i) {
  int fpb = 64;
  const int nf = namp / (d * d);
  SWEEP_D_SWITCH(d, fpb = launch_fibers_per_block_d<D>(i, (uint32_t)nf));
  return (nf + fpb - 1) / fpb;
}

bool sweep_m0_piped(int d, int namp, int i) {
  return d == 8 && m0p_used<8>(i, (uint32_t)(namp / 64));
}

}  // namespace fock
