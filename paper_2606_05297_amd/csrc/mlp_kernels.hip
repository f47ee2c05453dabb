// Warm-start network 4 -> 128 -> 128 -> 64 (SiLU, SiLU, linear) on bf16 MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Precision contract (the oracle follows the same steps in FP64): inputs and
// weights are rounded to bf16 (round to nearest even); biases stay FP32;
// hidden activations are rounded to bf16 after SiLU; the output is FP32.  The
// backward pass rounds the three error signals G3, G2, G1 to bf16 before their
// products (standard bf16 mixed precision); weight gradients are FP32 MFMA
// sums over a workgroup's 64 rows, then FP64 fixed-order sums over workgroups.
//
// One workgroup = 64 batch rows, 4 wavefronts; wavefront w owns rows
// 16w..16w+15 of every activation tile.  MFMA lane layout (16x16x32): lane l
// holds A[m = l % 16][k = 8 (l / 16) + i] and B[k = 8 (l / 16) + i][n = l % 16]
// for i < 8, and C[m = 4 (l / 16) + r][n = l % 16] for r < 4.
#include "mlp_internal.h"

namespace fock {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int XS = 40, AS = 136, GS = 72;  // LDS row strides in bf16 elements (multiples of 8)

// Round to nearest even (add 0x7fff plus the lowest kept bit, truncate).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
  const u16x8 v = *reinterpret_cast<const u16x8 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 gather8(const uint16_t *p, int stride) {
  u16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = p[i * stride];
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + expf(-z)); }

__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Forward for the workgroup's rows; with BWD also the masked-MSE error and
// this workgroup's share of every parameter gradient (partial + blockIdx.x *
// NPAR, parameter order) and of the loss numerator (lossp[blockIdx.x]).
template <bool BWD>
__global__ __launch_bounds__(256) void k_mlp(Weights w, const float *__restrict__ X, const float *__restrict__ T,
                                             const int *__restrict__ nvalid, const Count *__restrict__ cnt, int B,
                                             float *__restrict__ Y, float *__restrict__ partial,
                                             double *__restrict__ lossp) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[ROWS * XS];
  __shared__ __attribute__((aligned(16))) uint16_t a1s[ROWS * AS];  // A1, later G1
  __shared__ __attribute__((aligned(16))) uint16_t a2s[ROWS * AS];  // A2, later G2
  __shared__ __attribute__((aligned(16))) uint16_t g3s[ROWS * GS];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int row0 = blockIdx.x * ROWS, wr = wave * 16;

  for (int e = tid; e < ROWS * KIN; e += 256) {
    const int r = e / KIN, k = e % KIN;
    float v = 0.f;
    if (k < NIN && row0 + r < B) v = X[(size_t)(row0 + r) * NIN + k];
    xs[r * XS + k] = to_bf16(v);
  }
  __syncthreads();

  float ds1[8][4], ds2[8][4];  // SiLU'(Z1), SiLU'(Z2) in the C layout of this lane
  // layer 1: Z1 = Xb W1^T + b1 (K padded to 32 with zeros)
  {
    const bf16x8 a = ld8(xs + (wr + lr) * XS + 8 * lq);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 16 * t + lr;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      c = mma(a, ld8(w.w1b + n * KIN + 8 * lq), c);
      const float bias = w.params[OB1 + n];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z = c[r] + bias, s = sigm(z);
        a1s[(wr + 4 * lq + r) * AS + n] = to_bf16(z * s);
        ds1[t][r] = s * (1.f + z * (1.f - s));
      }
    }
  }
  __syncthreads();
  // layer 2: Z2 = A1 W2^T + b2
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int n = 16 * t + lr;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NH / 32; ++s)
      c = mma(ld8(a1s + (wr + lr) * AS + 32 * s + 8 * lq), ld8(w.w2b + n * NH + 32 * s + 8 * lq), c);
    const float bias = w.params[OB2 + n];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float z = c[r] + bias, sg = sigm(z);
      a2s[(wr + 4 * lq + r) * AS + n] = to_bf16(z * sg);
      ds2[t][r] = sg * (1.f + z * (1.f - sg));
    }
  }
  __syncthreads();
  // layer 3: Y = A2 W3^T + b3
  f32x4 y[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int n = 16 * t + lr;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NH / 32; ++s)
      c = mma(ld8(a2s + (wr + lr) * AS + 32 * s + 8 * lq), ld8(w.w3b + n * NH + 32 * s + 8 * lq), c);
    const float bias = w.params[OB3 + n];
#pragma unroll
    for (int r = 0; r < 4; ++r) y[t][r] = c[r] + bias;
  }
  if (Y) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int g = row0 + wr + 4 * lq + r;
        if (g < B) Y[(size_t)g * NOUT + 16 * t + lr] = y[t][r];
      }
  }
  if constexpr (!BWD) {
    return;
  } else {
    // G3 = bf16(2 M (Y - T) / N) and the loss numerator
    const float invN = cnt->invN;
    float lsum = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 4 * lq + r, g = row0 + row, n = 16 * t + lr;
        float gv = 0.f;
        if (g < B && n < nvalid[g]) {
          const float dl = y[t][r] - T[(size_t)g * NOUT + n];
          lsum = fmaf(dl, dl, lsum);
          gv = 2.f * dl * invN;
        }
        g3s[row * GS + n] = to_bf16(gv);
      }
    const double ls = block_sum((double)lsum, red);  // contains the barrier g3s needs
    if (tid == 0) lossp[blockIdx.x] = ls;
    float *P = partial + (size_t)blockIdx.x * NPAR;
    // dW3[out][in] = sum_rows G3[row][out] A2[row][in]: 4 x 8 tiles, 8 per wavefront
    for (int q = 0; q < 8; ++q) {
      const int tile = wave * 8 + q, tm = tile >> 3, tn = tile & 7;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < ROWS / 32; ++s)
        c = mma(gather8(g3s + (32 * s + 8 * lq) * GS + 16 * tm + lr, GS),
                gather8(a2s + (32 * s + 8 * lq) * AS + 16 * tn + lr, AS), c);
#pragma unroll
      for (int r = 0; r < 4; ++r) P[OW3 + (16 * tm + 4 * lq + r) * NH + 16 * tn + lr] = c[r];
    }
    if (tid < NOUT) {
      float s = 0.f;
      for (int row = 0; row < ROWS; ++row) s += from_bf16(g3s[row * GS + tid]);
      P[OB3 + tid] = s;
    }
    __syncthreads();
    // G2 = bf16((G3 W3) * SiLU'(Z2)), written over A2
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 16 * t + lr;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NOUT / 32; ++s)
        c = mma(ld8(g3s + (wr + lr) * GS + 32 * s + 8 * lq), ld8(w.w3t + n * NOUT + 32 * s + 8 * lq), c);
#pragma unroll
      for (int r = 0; r < 4; ++r) a2s[(wr + 4 * lq + r) * AS + n] = to_bf16(c[r] * ds2[t][r]);
    }
    __syncthreads();
    // dW2 = G2^T A1: 8 x 8 tiles, 16 per wavefront
    for (int q = 0; q < 16; ++q) {
      const int tile = wave * 16 + q, tm = tile >> 3, tn = tile & 7;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < ROWS / 32; ++s)
        c = mma(gather8(a2s + (32 * s + 8 * lq) * AS + 16 * tm + lr, AS),
                gather8(a1s + (32 * s + 8 * lq) * AS + 16 * tn + lr, AS), c);
#pragma unroll
      for (int r = 0; r < 4; ++r) P[OW2 + (16 * tm + 4 * lq + r) * NH + 16 * tn + lr] = c[r];
    }
    if (tid < NH) {
      float s = 0.f;
      for (int row = 0; row < ROWS; ++row) s += from_bf16(a2s[row * AS + tid]);
      P[OB2 + tid] = s;
    }
    __syncthreads();
    // G1 = bf16((G2 W2) * SiLU'(Z1)), written over A1
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 16 * t + lr;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NH / 32; ++s)
        c = mma(ld8(a2s + (wr + lr) * AS + 32 * s + 8 * lq), ld8(w.w2t + n * NH + 32 * s + 8 * lq), c);
#pragma unroll
      for (int r = 0; r < 4; ++r) a1s[(wr + 4 * lq + r) * AS + n] = to_bf16(c[r] * ds1[t][r]);
    }
    __syncthreads();
    // dW1 = G1^T Xb: 8 tiles of 16 outputs x 16 inputs (4 real), 2 per wavefront
    for (int q = 0; q < 2; ++q) {
      const int tm = wave * 2 + q;
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < ROWS / 32; ++s)
        c = mma(gather8(a1s + (32 * s + 8 * lq) * AS + 16 * tm + lr, AS), gather8(xs + (32 * s + 8 * lq) * XS + lr, XS),
                c);
      if (lr < NIN) {
#pragma unroll
        for (int r = 0; r < 4; ++r) P[OW1 + (16 * tm + 4 * lq + r) * NIN + lr] = c[r];
      }
    }
    if (tid < NH) {
      float s = 0.f;
      for (int row = 0; row < ROWS; ++row) s += from_bf16(a1s[row * AS + tid]);
      P[OB1 + tid] = s;
    }
  }
}

// N = sum_b min(max(n_b, 0), 64) and 1 / N (one workgroup).
__global__ __launch_bounds__(256) void k_mlp_count(const int *__restrict__ nvalid, int B, Count *__restrict__ cnt) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) s += (double)min(max(nvalid[b], 0), NOUT);
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    cnt->N = s;
    cnt->invN = s > 0.0 ? (float)(1.0 / s) : 0.f;
  }
}

// loss = sum of the workgroup numerators / N, fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_mlp_loss(const double *__restrict__ lossp, int nwg,
                                                  const Count *__restrict__ cnt, double *__restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nwg; b += 256) s += lossp[b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = cnt->N > 0.0 ? s / cnt->N : 0.0;
}

// One thread per parameter: fixed-order FP64 sum of the workgroup partials
// (nwg may be 0: no gradient), optional Adam update of the FP32 master value
// (Kingma & Ba, Algorithm 1; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t), then the
// bf16 copies the forward and backward kernels read.
__global__ __launch_bounds__(256) void k_mlp_update(const float *__restrict__ partial, int nwg, float *__restrict__ grad,
                                                    float *__restrict__ params, float *__restrict__ m,
                                                    float *__restrict__ v, AdamArgs ad, uint16_t *__restrict__ wb) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NPAR) return;
  double s = 0.0;
  for (int b = 0; b < nwg; ++b) s += (double)partial[(size_t)b * NPAR + p];
  const float g = (float)s;
  if (nwg > 0) grad[p] = g;
  float x = params[p];
  if (ad.on) {
    const float mm = ad.beta1 * m[p] + (1.f - ad.beta1) * g;
    const float vv = ad.beta2 * v[p] + (1.f - ad.beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    x -= ad.lr * (mm / ad.bc1) / (sqrtf(vv / ad.bc2) + ad.eps);
    params[p] = x;
  }
  const uint16_t h = to_bf16(x);
  if (p < OB1) {
    const int o = (p - OW1) / NIN, i = (p - OW1) % NIN;
    wb[WB_W1 + o * KIN + i] = h;
  } else if (p >= OW2 && p < OB2) {
    const int o = (p - OW2) / NH, i = (p - OW2) % NH;
    wb[WB_W2 + o * NH + i] = h;
    wb[WB_W2T + i * NH + o] = h;
  } else if (p >= OW3 && p < OB3) {
    const int o = (p - OW3) / NH, i = (p - OW3) % NH;
    wb[WB_W3 + o * NH + i] = h;
    wb[WB_W3T + i * NOUT + o] = h;
  }
}

int launch_mlp(bool bwd, const Weights &w, const float *X, const float *T, const int *nvalid, const Count *cnt, int B,
               float *Y, float *partial, double *lossp, hipStream_t s) {
  const int G = (B + ROWS - 1) / ROWS;
  if (G <= 0) return FOCK_OK;
  if (bwd) hipLaunchKernelGGL(k_mlp<true>, dim3(G), dim3(256), 0, s, w, X, T, nvalid, cnt, B, Y, partial, lossp);
  else hipLaunchKernelGGL(k_mlp<false>, dim3(G), dim3(256), 0, s, w, X, T, nvalid, cnt, B, Y, partial, lossp);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_mlp_count(const int *nvalid, int B, Count *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_count, dim3(1), dim3(256), 0, s, nvalid, B, cnt);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_mlp_loss(const double *lossp, int nwg, const Count *cnt, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, lossp, nwg, cnt, out);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

int launch_mlp_update(const float *partial, int nwg, float *grad, float *params, float *m, float *v,
                      const AdamArgs &ad, uint16_t *wb, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_update, dim3((NPAR + 255) / 256), dim3(256), 0, s, partial, nwg, grad, params, m, v, ad,
                     wb);
  FOCK_HIP(hipGetLastError());
  return FOCK_OK;
}

}  // namespace mlp
}  // namespace fock
