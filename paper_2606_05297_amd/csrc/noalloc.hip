// fock_apply_H_noalloc: H psi, <psi|H|psi> and <psi|psi> without any
// allocation, for callers that cannot allocate (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The per-workgroup energy/norm partials that fock_apply_H keeps in the
// caller's workspace live here in a file-scope device array of fixed size;
// the reduced pair goes to a caller-supplied device buffer instead of pinned
// host staging.  Same kernels and the same reduction order as fock_apply_H,
// hence bit-identical results.
#include <atomic>
#include <cstring>
#include <mutex>

#include "pipeline.h"

namespace fock {

namespace {

constexpr size_t kScratchDoubles = 131072;  // 1 MiB: partials of up to 65,536 workgroups
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// Device address of this device's copy of `scratch`, looked up once per device
// with that device current.  (In host code the array's name is only a host-side
// stand-in; kernels receive this address.)
int scratch_on_device(double **out) {
  int dev = 0;
  FOCK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(FOCK_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(FOCK_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return FOCK_OK;
}

}  // namespace

}  // namespace fock

using namespace fock;

extern "C" int fock_apply_H_noalloc(const fock_ham_t *ham, const void *psi, void *hpsi, double *res_dev,
                                    fock_stream_t stream) {
  uint32_t namp = 0;
  int rc = check_ham(ham, &namp);
  if (rc) return rc;
  if ((rc = check_ptr(psi, "psi")) || (rc = check_ptr(hpsi, "hpsi"))) return rc;
  if (psi == hpsi) return set_error(FOCK_ERR_ARG, "psi and hpsi must not overlap");
  if (res_dev && (((uintptr_t)res_dev) & 7)) return set_error(FOCK_ERR_ARG, "res_dev is not 8-byte aligned");
  // The H psi set-up of make_ctx without the workgroup-order table (tile
  // schedules 1-3 would allocate one): workgroups map to tiles by XCD runs.
  HamArgs h = make_ham_args(*ham);
  h.order = nullptr;
  if (stencil_schedule() == FOCK_SCHED_TWO_PASS) h.hi_m = apply_h_hi_modes(ham->L, ham->d, h.periodic_wrap);
  h.lanes = (stencil_variant() == FOCK_STENCIL_LANES && h.hi_m == 0 && lanes_stencil_ok(ham->L, ham->d, h.periodic_wrap))
                ? 1 : 0;
  h.slab = (stencil_variant() == FOCK_STENCIL_SLAB && h.hi_m == 0 && slab_stencil_ok(ham->L, ham->d)) ? 1 : 0;
  const size_t G = h.slab ? 512 : (size_t)apply_h_blocks(h);
  if (2 * G > kScratchDoubles)
    return set_error(FOCK_ERR_SIZE, "fock_apply_H_noalloc: %zu workgroup partials exceed the %zu-double scratch "
                     "(d^L too large; use fock_apply_H with a workspace)", 2 * G, kScratchDoubles);
  double *part = nullptr;
  if ((rc = scratch_on_device(&part))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int nb = 0;
  rc = h.slab ? launch_apply_h2(h, (const float2 *)psi, (float2 *)hpsi, part, &nb, s)
              : launch_apply_h(h, (const float2 *)psi, (float2 *)hpsi, part, &nb, s);
  if (rc) return rc;
  if ((size_t)nb != G) return set_error(FOCK_ERR_STATE, "apply-H launched %d workgroups, expected %zu", nb, G);
  if (res_dev) return launch_reduce(part, nb, 2, res_dev, s);
  return FOCK_OK;
}
