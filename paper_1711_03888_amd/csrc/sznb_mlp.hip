// Learned predictor selector: training and stand-alone inference kernels
// (gfx950, wave64).
//
// The network (16 -> 32 -> 32 -> 3, ReLU, 1699 parameters) picks a block's
// predictor from 16 block features (k_features); its labels are the
// exhaustive trial's choices.  Training is float32: softmax cross-entropy
// averaged over the batch, Adam with bias correction.  Every reduction runs
// in a fixed order, so a training step is deterministic.
//
//   mlp_fwd_bwd     one thread per sample: forward pass, loss, and the
//                   pre-activation gradients dz1, dz2, dz3 of the sample
//   mlp_grad        one thread per parameter: the batch sum of
//                   dz (outer) activation, samples in ascending order
//   mlp_loss        mean loss of the batch, fixed-shape tree
//   mlp_adam        one thread per parameter
//   mlp_infer       one wave per block: the bfloat16 inference used by the
//                   compressor's learned policy
#include "sznb_internal.h"

namespace sznb {

constexpr int kMlpThreads = 256;

// per-sample buffers, structure of arrays: row r holds sample s at r * B + s
enum : int { R_H1 = 0, R_H2 = 32, R_DZ1 = 64, R_DZ2 = 96, R_DZ3 = 128, R_LOSS = 131, R_ROWS = 132 };

__global__ __launch_bounds__(kMlpThreads) void mlp_fwd_bwd(const float *__restrict__ w, const float *__restrict__ feat,
                                                           const uint8_t *__restrict__ label, uint32_t B,
                                                           float *__restrict__ buf) {
  __shared__ float s_w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += kMlpThreads) s_w[i] = w[i];
  __syncthreads();
  const uint32_t s = blockIdx.x * kMlpThreads + threadIdx.x;
  if (s >= B) return;
  float x[kNFeat], z1[32], z2[32], z3[3];
#pragma unroll
  for (int k = 0; k < kNFeat; k++) x[k] = feat[(uint64_t)s * kNFeat + k];
#pragma unroll
  for (int j = 0; j < 32; j++) {
    float acc = s_w[kB1 + j];
#pragma unroll
    for (int k = 0; k < kNFeat; k++) acc = __builtin_fmaf(s_w[kW1 + 16 * j + k], x[k], acc);
    z1[j] = acc;
  }
#pragma unroll
  for (int j = 0; j < 32; j++) {
    float acc = s_w[kB2 + j];
#pragma unroll
    for (int k = 0; k < 32; k++) acc = __builtin_fmaf(s_w[kW2 + 32 * j + k], z1[k] > 0.0f ? z1[k] : 0.0f, acc);
    z2[j] = acc;
  }
#pragma unroll
  for (int j = 0; j < 3; j++) {
    float acc = s_w[kB3 + j];
#pragma unroll
    for (int k = 0; k < 32; k++) acc = __builtin_fmaf(s_w[kW3 + 32 * j + k], z2[k] > 0.0f ? z2[k] : 0.0f, acc);
    z3[j] = acc;
  }
  // softmax cross-entropy; gradient of the batch mean
  const float m = fmaxf(z3[0], fmaxf(z3[1], z3[2]));
  float e[3], se = 0.0f;
#pragma unroll
  for (int j = 0; j < 3; j++) { e[j] = expf(z3[j] - m); se += e[j]; }
  const int y = label[s] < 3 ? label[s] : 0;
  const float lse = m + logf(se);
  const float invB = 1.0f / (float)B;
  float dz3[3];
#pragma unroll
  for (int j = 0; j < 3; j++) dz3[j] = (e[j] / se - (j == y ? 1.0f : 0.0f)) * invB;
  float dz2[32], dz1[32];
#pragma unroll
  for (int k = 0; k < 32; k++) {
    float a = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; j++) a = __builtin_fmaf(s_w[kW3 + 32 * j + k], dz3[j], a);
    dz2[k] = z2[k] > 0.0f ? a : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 32; k++) {
    float a = 0.0f;
#pragma unroll
    for (int j = 0; j < 32; j++) a = __builtin_fmaf(s_w[kW2 + 32 * j + k], dz2[j], a);
    dz1[k] = z1[k] > 0.0f ? a : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 32; k++) {
    buf[(uint64_t)(R_H1 + k) * B + s] = z1[k] > 0.0f ? z1[k] : 0.0f;
    buf[(uint64_t)(R_H2 + k) * B + s] = z2[k] > 0.0f ? z2[k] : 0.0f;
    buf[(uint64_t)(R_DZ1 + k) * B + s] = dz1[k];
    buf[(uint64_t)(R_DZ2 + k) * B + s] = dz2[k];
  }
#pragma unroll
  for (int j = 0; j < 3; j++) buf[(uint64_t)(R_DZ3 + j) * B + s] = dz3[j];
  buf[(uint64_t)R_LOSS * B + s] = lse - z3[y];
}

// gradient of parameter p: sum over samples (ascending) of dz * input
__global__ __launch_bounds__(kMlpThreads) void mlp_grad(const float *__restrict__ feat, const float *__restrict__ buf,
                                                        uint32_t B, float *__restrict__ grad) {
  const int p = blockIdx.x * kMlpThreads + threadIdx.x;
  if (p >= kMlpParams) return;
  const float *dz, *in = nullptr;
  uint32_t in_stride = 0;
  if (p < kB1) {  // W1[j][k]
    const int j = p / 16, k = p % 16;
    dz = buf + (uint64_t)(R_DZ1 + j) * B; in = feat + k; in_stride = kNFeat;
  } else if (p < kW2) {
    dz = buf + (uint64_t)(R_DZ1 + p - kB1) * B;
  } else if (p < kB2) {  // W2[j][k]
    const int j = (p - kW2) / 32, k = (p - kW2) % 32;
    dz = buf + (uint64_t)(R_DZ2 + j) * B; in = buf + (uint64_t)(R_H1 + k) * B; in_stride = 1;
  } else if (p < kW3) {
    dz = buf + (uint64_t)(R_DZ2 + p - kB2) * B;
  } else if (p < kB3) {  // W3[j][k]
    const int j = (p - kW3) / 32, k = (p - kW3) % 32;
    dz = buf + (uint64_t)(R_DZ3 + j) * B; in = buf + (uint64_t)(R_H2 + k) * B; in_stride = 1;
  } else {
    dz = buf + (uint64_t)(R_DZ3 + p - kB3) * B;
  }
  float acc = 0.0f;
  if (in) {
    for (uint32_t s = 0; s < B; s++) acc = __builtin_fmaf(dz[s], in[(uint64_t)s * in_stride], acc);
  } else {
    for (uint32_t s = 0; s < B; s++) acc += dz[s];
  }
  grad[p] = acc;
}

// mean of the per-sample losses: fixed strided partial sums, then a fixed tree
__global__ __launch_bounds__(kMlpThreads) void mlp_loss(const float *__restrict__ buf, uint32_t B, float *loss) {
  __shared__ float s_part[kMlpThreads];
  const int t = threadIdx.x;
  const float *l = buf + (uint64_t)R_LOSS * B;
  float a = 0.0f;
  for (uint32_t s = t; s < B; s += kMlpThreads) a += l[s];
  s_part[t] = a;
  __syncthreads();
  for (int h = kMlpThreads / 2; h > 0; h >>= 1) {
    if (t < h) s_part[t] += s_part[t + h];
    __syncthreads();
  }
  if (t == 0) *loss = s_part[0] / (float)B;
}

// Adam (Kingma and Ba, 2015): m, v moving averages, bias-corrected step
__global__ __launch_bounds__(kMlpThreads) void mlp_adam(float *__restrict__ w, float *__restrict__ m,
                                                        float *__restrict__ v, const float *__restrict__ g,
                                                        uint32_t step, float lr, float beta1, float beta2, float eps) {
  const int p = blockIdx.x * kMlpThreads + threadIdx.x;
  if (p >= kMlpParams) return;
  const float gp = g[p];
  const float mp = beta1 * m[p] + (1.0f - beta1) * gp;
  const float vp = beta2 * v[p] + (1.0f - beta2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// bfloat16 inference, one wave per block: logits, choice and margin
__global__ __launch_bounds__(kMlpThreads) void mlp_infer(const float *__restrict__ w, const float *__restrict__ feat,
                                                         uint64_t nb, float *__restrict__ logits,
                                                         uint8_t *__restrict__ choice, float *__restrict__ margin) {
  __shared__ __align__(16) float s_w[kMlpLds];
  __shared__ __align__(16) float s_x[kMlpThreads / kWave][kNFeat];
  __shared__ __align__(16) float s_h[kMlpThreads / kWave][32];
  for (int i = threadIdx.x; i < kMlpParams; i += kMlpThreads) {
    const bool bias = (i >= kB1 && i < kW2) || (i >= kB2 && i < kW3) || i >= kB3;
    s_w[mlp_lds_slot(i)] = bias ? w[i] : bf16_round(w[i]);
  }
  __syncthreads();
  const uint64_t waves = (uint64_t)gridDim.x * (kMlpThreads / kWave);
  for (uint64_t b = (uint64_t)blockIdx.x * (kMlpThreads / kWave) + threadIdx.x / kWave; b < nb; b += waves) {
    const int w = threadIdx.x / kWave;
    wave_lds_order();  // the previous block's reads of s_x are done
    if (__lane_id() < (uint32_t)kNFeat) s_x[w][__lane_id()] = bf16_round(feat[b * kNFeat + __lane_id()]);
    float mg, z[3];
    const int top = mlp_select_wave(s_w, s_x[w], s_h[w], mg, z);
    if (__lane_id() == 0) {
      choice[b] = (uint8_t)top;
      margin[b] = mg;
      for (int k = 0; k < 3; k++) logits[b * 3 + k] = z[k];
    }
  }
}

}  // namespace sznb
