// Host side of the warm-start network: device buffers, the C ABI
// (fock_mlp_*), Adam bookkeeping.
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp_internal.h"

using namespace fock;
using namespace fock::mlp;

struct fock_mlp {
  int max_batch = 0, max_wg = 0;
  void *dev = nullptr;
  float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr;
  uint16_t *wb = nullptr;
  Count *cnt = nullptr;
  double *lossp = nullptr, *loss = nullptr;
  int step = 0;
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

Weights weights_of(const fock_mlp *n) {
  return Weights{n->params, n->wb + WB_W1, n->wb + WB_W2, n->wb + WB_W2T, n->wb + WB_W3, n->wb + WB_W3T};
}

int check_batch(const fock_mlp *n, int B) {
  if (B <= 0) return set_error(FOCK_ERR_ARG, "batch size %d must be positive", B);
  if (B > n->max_batch) return set_error(FOCK_ERR_SIZE, "batch size %d exceeds the maximum %d", B, n->max_batch);
  return FOCK_OK;
}

// Forward, backward and the loss of one batch; partials and the loss stay on
// the device.  Returns the number of workgroup partials.
int loss_grad_dev(fock_mlp *n, const float *X, const float *T, const int *nv, int B, hipStream_t s, int *nwg) {
  int rc = launch_mlp_count(nv, B, n->cnt, s);
  if (rc) return rc;
  *nwg = (B + ROWS - 1) / ROWS;
  {
    ProfScope ps(FOCK_K_MLP_TRAIN, s, 149504.0 * B);
    rc = launch_mlp(true, weights_of(n), X, T, nv, n->cnt, B, nullptr, n->partial, n->lossp, s);
    if (rc) return rc;
  }
  return launch_mlp_loss(n->lossp, *nwg, n->cnt, n->loss, s);
}

int fetch_loss(fock_mlp *n, double *loss, hipStream_t s) {
  FOCK_HIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  FOCK_HIP(hipStreamSynchronize(s));
  prof_harvest();
  return FOCK_OK;
}

}  // namespace

extern "C" {

int fock_mlp_create(int max_batch, fock_mlp_t **out) {
  if (!out) return set_error(FOCK_ERR_ARG, "NULL output");
  *out = nullptr;
  if (max_batch <= 0 || max_batch > (1 << 20))
    return set_error(FOCK_ERR_ARG, "max_batch %d outside [1, 2^20]", max_batch);
  fock_mlp *n = new fock_mlp;
  n->max_batch = max_batch;
  n->max_wg = (max_batch + ROWS - 1) / ROWS;
  const size_t sp = al256(sizeof(float) * NPAR);
  const size_t sizes[] = {sp, sp, sp, sp, al256(sizeof(float) * NPAR * (size_t)n->max_wg),
                          al256(sizeof(uint16_t) * WB_TOTAL), al256(sizeof(Count)),
                          al256(sizeof(double) * n->max_wg), al256(sizeof(double))};
  size_t total = 0;
  for (size_t x : sizes) total += x;
  if (hipMalloc(&n->dev, total) != hipSuccess) {
    delete n;
    return set_error(FOCK_ERR_HIP, "hipMalloc of %zu bytes for the network failed", total);
  }
  char *p = (char *)n->dev;
  n->params = (float *)p, p += sizes[0];
  n->m = (float *)p, p += sizes[1];
  n->v = (float *)p, p += sizes[2];
  n->grad = (float *)p, p += sizes[3];
  n->partial = (float *)p, p += sizes[4];
  n->wb = (uint16_t *)p, p += sizes[5];
  n->cnt = (Count *)p, p += sizes[6];
  n->lossp = (double *)p, p += sizes[7];
  n->loss = (double *)p;
  if (hipMemset(n->dev, 0, total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(n->dev);
    delete n;
    return set_error(FOCK_ERR_HIP, "clearing the network buffers failed");
  }
  *out = n;
  return FOCK_OK;
}

int fock_mlp_set_params(fock_mlp_t *n, const float *params, int count, fock_stream_t stream) {
  if (!n || !params) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (count != NPAR) return set_error(FOCK_ERR_SIZE, "expected %d parameters, got %d", NPAR, count);
  for (int k = 0; k < count; ++k)
    if (!std::isfinite(params[k])) return set_error(FOCK_ERR_NONFINITE, "parameter %d is not finite", k);
  hipStream_t s = (hipStream_t)stream;
  FOCK_HIP(hipMemcpyAsync(n->params, params, sizeof(float) * NPAR, hipMemcpyHostToDevice, s));
  FOCK_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * NPAR, s));
  FOCK_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * NPAR, s));
  AdamArgs off{};
  int rc = launch_mlp_update(n->partial, 0, n->grad, n->params, n->m, n->v, off, n->wb, s);
  if (rc) return rc;
  FOCK_HIP(hipStreamSynchronize(s));  // params is a caller buffer: finish the copy before returning
  n->step = 0;
  return FOCK_OK;
}

int fock_mlp_get_params(fock_mlp_t *n, float *params, int count, fock_stream_t stream) {
  if (!n || !params) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (count != NPAR) return set_error(FOCK_ERR_SIZE, "expected %d parameters, got %d", NPAR, count);
  hipStream_t s = (hipStream_t)stream;
  FOCK_HIP(hipMemcpyAsync(params, n->params, sizeof(float) * NPAR, hipMemcpyDeviceToHost, s));
  FOCK_HIP(hipStreamSynchronize(s));
  return FOCK_OK;
}

int fock_mlp_forward(fock_mlp_t *n, const float *X, int B, float *Y, fock_stream_t stream) {
  if (!n || !X || !Y) return set_error(FOCK_ERR_ARG, "NULL argument");
  int rc = check_batch(n, B);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps(FOCK_K_MLP_FWD, s, 50176.0 * B);
  return launch_mlp(false, weights_of(n), X, nullptr, nullptr, nullptr, B, Y, nullptr, nullptr, s);
}

int fock_mlp_loss_grad(fock_mlp_t *n, const float *X, const float *T, const int *nvalid, int B, double *loss,
                       float *grad, fock_stream_t stream) {
  if (!n || !X || !T || !nvalid) return set_error(FOCK_ERR_ARG, "NULL argument");
  int rc = check_batch(n, B);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int nwg = 0;
  rc = loss_grad_dev(n, X, T, nvalid, B, s, &nwg);
  if (rc) return rc;
  AdamArgs off{};
  rc = launch_mlp_update(n->partial, nwg, n->grad, n->params, n->m, n->v, off, n->wb, s);
  if (rc) return rc;
  if (grad) FOCK_HIP(hipMemcpyAsync(grad, n->grad, sizeof(float) * NPAR, hipMemcpyDeviceToHost, s));
  if (loss) return fetch_loss(n, loss, s);
  if (grad) FOCK_HIP(hipStreamSynchronize(s));
  return FOCK_OK;
}

int fock_mlp_adam_step(fock_mlp_t *n, const float *X, const float *T, const int *nvalid, int B, float lr,
                       double *loss, fock_stream_t stream) {
  if (!n || !X || !T || !nvalid) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (!(lr > 0.f) || !std::isfinite(lr)) return set_error(FOCK_ERR_ARG, "learning rate must be positive");
  int rc = check_batch(n, B);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int nwg = 0;
  rc = loss_grad_dev(n, X, T, nvalid, B, s, &nwg);
  if (rc) return rc;
  n->step += 1;
  AdamArgs ad;
  ad.on = 1;
  ad.lr = lr;
  ad.beta1 = 0.9f;
  ad.beta2 = 0.999f;
  ad.eps = 1e-8f;
  ad.bc1 = (float)(1.0 - std::pow(0.9, n->step));
  ad.bc2 = (float)(1.0 - std::pow(0.999, n->step));
  rc = launch_mlp_update(n->partial, nwg, n->grad, n->params, n->m, n->v, ad, n->wb, s);
  if (rc) return rc;
  if (loss) return fetch_loss(n, loss, s);
  return FOCK_OK;
}

int fock_mlp_destroy(fock_mlp_t *n) {
  if (!n) return FOCK_OK;
  (void)hipDeviceSynchronize();
  if (n->dev) (void)hipFree(n->dev);
  delete n;
  return FOCK_OK;
}

}  // extern "C"
