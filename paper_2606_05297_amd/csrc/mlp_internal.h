// Warm-start network: shapes, parameter layout and launchers.
#pragma once

#include "fock_internal.h"

namespace fock {
namespace mlp {

constexpr int NIN = 4, NH = 128, NOUT = 64;
constexpr int KIN = 32;   // layer-1 reduction padded to one MFMA step (entries >= NIN are zero)
constexpr int ROWS = 64;  // batch rows per workgroup

// FP32 master parameters, in this order; W is [out x in] row-major.
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, NPAR = OB3 + NOUT;

// bf16 weight copies (one allocation): W1 padded [NH][KIN], W2 [out][in],
// W2^T [in][out], W3 [out][in], W3^T [in][out].
constexpr int WB_W1 = 0, WB_W2 = WB_W1 + NH * KIN, WB_W2T = WB_W2 + NH * NH, WB_W3 = WB_W2T + NH * NH,
              WB_W3T = WB_W3 + NOUT * NH, WB_TOTAL = WB_W3T + NH * NOUT;

struct Weights {
  const float *params;  // FP32 master (biases are read from here)
  const uint16_t *w1b, *w2b, *w2t, *w3b, *w3t;
};

struct Count {
  double N;    // number of unmasked targets in the batch
  float invN;  // 1 / N (0 if N = 0)
  float pad;
};

struct AdamArgs {
  int on;
  float lr, beta1, beta2, eps, bc1, bc2;
};

int launch_mlp(bool bwd, const Weights &w, const float *X, const float *T, const int *nvalid, const Count *cnt, int B,
               float *Y, float *partial, double *lossp, hipStream_t s);
int launch_mlp_count(const int *nvalid, int B, Count *cnt, hipStream_t s);
int launch_mlp_loss(const double *lossp, int nwg, const Count *cnt, double *out, hipStream_t s);
int launch_mlp_update(const float *partial, int nwg, float *grad, float *params, float *m, float *v,
                      const AdamArgs &ad, uint16_t *wb, hipStream_t s);

}  // namespace mlp
}  // namespace fock
