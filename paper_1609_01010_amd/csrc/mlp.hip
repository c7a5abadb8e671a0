// FP32 cost model of the plans: a 3-layer perceptron with hand-written
// forward, backward and Adam kernels.
//
//   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3
//   loss = (1/B) sum_b (y_b - t_b)^2
// Parameters are one float array: W1 [H][F], b1 [H], W2 [H][H], b2 [H],
// W3 [H], b3 [1].  Gradients are reduced over the batch in a fixed order
// (one thread per weight), so training is deterministic.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "mlp.h"

namespace pm {

// forward: one 64-thread block per sample; keeps h1, h2 for the backward
// (H1, H2 null: inference, only y)
__global__ void __launch_bounds__(kMlpH) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X, int B,
                                                       float* __restrict__ H1, float* __restrict__ H2,
                                                       float* __restrict__ Y) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const int j = threadIdx.x;
  const float* W1 = P + kOffW1;
  const float* b1 = P + kOffB1;
  const float* W2 = P + kOffW2;
  const float* b2 = P + kOffB2;
  const float* W3 = P + kOffW3;
  const float b3 = P[kOffB3];
  __shared__ float x[kMlpF];
  __shared__ float h1[kMlpH];
  __shared__ float part[kMlpH];
  if (j < kMlpF) x[j] = X[(size_t)b * kMlpF + j];
  __syncthreads();
  float z = b1[j];
  for (int f = 0; f < kMlpF; ++f) z = fmaf(W1[j * kMlpF + f], x[f], z);
  const float a1 = tanhf(z);
  h1[j] = a1;
  if (H1) H1[(size_t)b * kMlpH + j] = a1;
  __syncthreads();
  float z2 = b2[j];
  for (int k = 0; k < kMlpH; ++k) z2 = fmaf(W2[j * kMlpH + k], h1[k], z2);
  const float a2 = tanhf(z2);
  if (H2) H2[(size_t)b * kMlpH + j] = a2;
  part[j] = W3[j] * a2;
  __syncthreads();
  if (j == 0) {
    float y = b3;
    for (int k = 0; k < kMlpH; ++k) y += part[k];
    Y[b] = y;
  }
}

// backward, per sample: dy = 2 (y - t) / B, dz2 = dy W3 (1 - h2^2),
// dz1 = (W2^T dz2) (1 - h1^2)
__global__ void __launch_bounds__(kMlpH) k_mlp_deltas(const float* __restrict__ P, const float* __restrict__ T, int B,
                                                      const float* __restrict__ H1, const float* __restrict__ H2,
                                                      const float* __restrict__ Y, float* __restrict__ DY,
                                                      float* __restrict__ DZ1, float* __restrict__ DZ2) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const int j = threadIdx.x;
  const float* W2 = P + kOffW2;
  const float* W3 = P + kOffW3;
  __shared__ float dz2[kMlpH];
  const float dy = 2.0f * (Y[b] - T[b]) / (float)B;
  if (j == 0) DY[b] = dy;
  const float h2 = H2[(size_t)b * kMlpH + j];
  const float d2 = dy * W3[j] * (1.0f - h2 * h2);
  dz2[j] = d2;
  DZ2[(size_t)b * kMlpH + j] = d2;
  __syncthreads();
  float dh1 = 0.0f;
  for (int i = 0; i < kMlpH; ++i) dh1 = fmaf(W2[i * kMlpH + j], dz2[i], dh1);
  const float h1 = H1[(size_t)b * kMlpH + j];
  DZ1[(size_t)b * kMlpH + j] = dh1 * (1.0f - h1 * h1);
}

// gradient of every parameter: one thread per parameter, sum over the batch
__global__ void k_mlp_grads(const float* __restrict__ X, int B, const float* __restrict__ H1,
                            const float* __restrict__ H2, const float* __restrict__ DY,
                            const float* __restrict__ DZ1, const float* __restrict__ DZ2, float* __restrict__ G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float s = 0.0f;
  if (i < kOffB1) {  // W1[j][f]
    const int j = i / kMlpF, f = i % kMlpF;
    for (int b = 0; b < B; ++b) s = fmaf(DZ1[(size_t)b * kMlpH + j], X[(size_t)b * kMlpF + f], s);
  } else if (i < kOffW2) {  // b1[j]
    const int j = i - kOffB1;
    for (int b = 0; b < B; ++b) s += DZ1[(size_t)b * kMlpH + j];
  } else if (i < kOffB2) {  // W2[j][k]
    const int o = i - kOffW2, j = o / kMlpH, k = o % kMlpH;
    for (int b = 0; b < B; ++b) s = fmaf(DZ2[(size_t)b * kMlpH + j], H1[(size_t)b * kMlpH + k], s);
  } else if (i < kOffW3) {  // b2[j]
    const int j = i - kOffB2;
    for (int b = 0; b < B; ++b) s += DZ2[(size_t)b * kMlpH + j];
  } else if (i < kOffB3) {  // W3[j]
    const int j = i - kOffW3;
    for (int b = 0; b < B; ++b) s = fmaf(DY[b], H2[(size_t)b * kMlpH + j], s);
  } else {  // b3
    for (int b = 0; b < B; ++b) s += DY[b];
  }
  G[i] = s;
}

// mean squared error (one work-group, fixed reduction order)
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int B,
                                                  float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float d = Y[b] - T[b];
    s = fmaf(d, d, s);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0] / (float)B;
}

// Adam (Kingma & Ba), bias-corrected, in place
__global__ void k_mlp_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                           float* __restrict__ V, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  const float mh = m / c1;
  const float vh = v / c2;
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// host side

MlpDev::~MlpDev() { release(); }

void MlpDev::release() {
  for (float** p : {&P, &G, &M, &V, &X, &T, &H1, &H2, &Y, &DY, &DZ1, &DZ2, &L})
    if (*p) {
      hipFree(*p);
      *p = nullptr;
    }
  cap = 0;
}

pm_status MlpDev::ensure(int B) {
  if (!P) {
    if (hipMalloc(&P, kMlpParams * 4) || hipMalloc(&G, kMlpParams * 4) || hipMalloc(&M, kMlpParams * 4) ||
        hipMalloc(&V, kMlpParams * 4) || hipMalloc(&L, 4))
      return PM_ENOMEM;
  }
  if (B <= cap) return PM_OK;
  for (float** p : {&X, &T, &H1, &H2, &Y, &DY, &DZ1, &DZ2})
    if (*p) {
      hipFree(*p);
      *p = nullptr;
    }
  const size_t b = (size_t)B;
  if (hipMalloc(&X, b * kMlpF * 4) || hipMalloc(&T, b * 4) || hipMalloc(&H1, b * kMlpH * 4) ||
      hipMalloc(&H2, b * kMlpH * 4) || hipMalloc(&Y, b * 4) || hipMalloc(&DY, b * 4) ||
      hipMalloc(&DZ1, b * kMlpH * 4) || hipMalloc(&DZ2, b * kMlpH * 4))
    return PM_ENOMEM;
  cap = B;
  return PM_OK;
}

hipError_t MlpDev::forward(int B, hipStream_t s) {
  k_mlp_forward<<<B, kMlpH, 0, s>>>(P, X, B, H1, H2, Y);
  return hipGetLastError();
}

hipError_t MlpDev::loss_grad(int B, hipStream_t s) {
  hipError_t e = forward(B, s);
  if (e) return e;
  k_mlp_loss<<<1, 256, 0, s>>>(Y, T, B, L);
  k_mlp_deltas<<<B, kMlpH, 0, s>>>(P, T, B, H1, H2, Y, DY, DZ1, DZ2);
  k_mlp_grads<<<(kMlpParams + 255) / 256, 256, 0, s>>>(X, B, H1, H2, DY, DZ1, DZ2, G);
  return hipGetLastError();
}

hipError_t MlpDev::adam(int step, float lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_mlp_adam<<<(kMlpParams + 255) / 256, 256, 0, s>>>(P, G, M, V, kMlpParams, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

pm_status mlp_infer_init(MlpInfer* I) {
  const size_t rows = kMlpInferRows;
  if (hipStreamCreateWithFlags(&I->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&I->ev, hipEventDisableTiming) != hipSuccess)
    return PM_EDEVICE;
  if (hipMalloc(&I->dP, kMlpParams * 4) || hipMalloc(&I->dX, rows * kMlpF * 4) || hipMalloc(&I->dY, rows * 4) ||
      hipHostMalloc((void**)&I->hP, kMlpParams * 4, hipHostMallocDefault) ||
      hipHostMalloc((void**)&I->hX, rows * kMlpF * 4, hipHostMallocDefault) ||
      hipHostMalloc((void**)&I->hY, rows * 4, hipHostMallocDefault))
    return PM_ENOMEM;
  return PM_OK;
}

// Rows go through in chunks of kMlpInferRows: staged in pinned memory,
// copied and evaluated on the inference stream, and read back after its
// event (no device-wide synchronisation, no allocation).
pm_status mlp_infer(MlpInfer* I, const float* w, unsigned long ver, const float* X, int B, float* y) {
  std::lock_guard<std::mutex> lk(I->mu);
  if (I->ver != ver) {
    // the previous upload (if any) has completed: every call below waits for its event
    memcpy(I->hP, w, kMlpParams * 4);
    if (hipMemcpyAsync(I->dP, I->hP, kMlpParams * 4, hipMemcpyHostToDevice, I->s) != hipSuccess) return PM_EDEVICE;
    I->ver = ver;
  }
  for (int o = 0; o < B; o += kMlpInferRows) {
    const int n = B - o < kMlpInferRows ? B - o : kMlpInferRows;
    memcpy(I->hX, X + (size_t)o * kMlpF, (size_t)n * kMlpF * 4);
    if (hipMemcpyAsync(I->dX, I->hX, (size_t)n * kMlpF * 4, hipMemcpyHostToDevice, I->s) != hipSuccess)
      return PM_EDEVICE;
    k_mlp_forward<<<n, kMlpH, 0, I->s>>>(I->dP, I->dX, n, nullptr, nullptr, I->dY);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(I->hY, I->dY, (size_t)n * 4, hipMemcpyDeviceToHost, I->s) != hipSuccess ||
        hipEventRecord(I->ev, I->s) != hipSuccess || hipEventSynchronize(I->ev) != hipSuccess) {
      I->ver = 0;
      return PM_EDEVICE;
    }
    memcpy(y + o, I->hY, (size_t)n * 4);
  }
  return PM_OK;
}

}  // namespace pm

using namespace pm;

extern "C" {

size_t pm_mlp_num_params(void) { return kMlpParams; }

pm_status pm_mlp_loss_grad(const float* params, const float* X, const float* t, int B, float* loss, float* grads) {
  if (!params || !X || !t || B < 1 || !grads) return PM_EINVAL;
  MlpDev d;
  pm_status st = d.ensure(B);
  if (st) return st;
  if (hipMemcpy(d.P, params, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.X, X, (size_t)B * kMlpF * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.T, t, (size_t)B * 4, hipMemcpyHostToDevice))
    return PM_EDEVICE;
  if (d.loss_grad(B, 0) != hipSuccess) return PM_EDEVICE;
  if (hipMemcpy(grads, d.G, kMlpParams * 4, hipMemcpyDeviceToHost)) return PM_EDEVICE;
  if (loss && hipMemcpy(loss, d.L, 4, hipMemcpyDeviceToHost)) return PM_EDEVICE;
  return PM_OK;
}

pm_status pm_mlp_forward(const float* params, const float* X, int B, float* y) {
  if (!params || !X || B < 1 || !y) return PM_EINVAL;
  MlpDev d;
  pm_status st = d.ensure(B);
  if (st) return st;
  if (hipMemcpy(d.P, params, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.X, X, (size_t)B * kMlpF * 4, hipMemcpyHostToDevice))
    return PM_EDEVICE;
  if (d.forward(B, 0) != hipSuccess) return PM_EDEVICE;
  if (hipMemcpy(y, d.Y, (size_t)B * 4, hipMemcpyDeviceToHost)) return PM_EDEVICE;
  return PM_OK;
}

pm_status pm_mlp_train(float* params, const float* X, const float* t, int B, int steps, float lr, float* losses) {
  if (!params || !X || !t || B < 1 || steps < 0) return PM_EINVAL;
  MlpDev d;
  pm_status st = d.ensure(B);
  if (st) return st;
  if (hipMemcpy(d.P, params, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.X, X, (size_t)B * kMlpF * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.T, t, (size_t)B * 4, hipMemcpyHostToDevice) || hipMemset(d.M, 0, kMlpParams * 4) ||
      hipMemset(d.V, 0, kMlpParams * 4))
    return PM_EDEVICE;
  for (int i = 1; i <= steps; ++i) {
    if (d.loss_grad(B, 0) != hipSuccess || d.adam(i, lr, 0) != hipSuccess) return PM_EDEVICE;
    if (losses && hipMemcpy(&losses[i - 1], d.L, 4, hipMemcpyDeviceToHost)) return PM_EDEVICE;
  }
  if (hipMemcpy(params, d.P, kMlpParams * 4, hipMemcpyDeviceToHost)) return PM_EDEVICE;
  return PM_OK;
}

pm_status pm_mlp_adam(float* params, const float* grads, float* m, float* v, int step, float lr) {
  if (!params || !grads || !m || !v || step < 1) return PM_EINVAL;
  MlpDev d;
  pm_status st = d.ensure(1);
  if (st) return st;
  if (hipMemcpy(d.P, params, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.G, grads, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.M, m, kMlpParams * 4, hipMemcpyHostToDevice) ||
      hipMemcpy(d.V, v, kMlpParams * 4, hipMemcpyHostToDevice))
    return PM_EDEVICE;
  if (d.adam(step, lr, 0) != hipSuccess) return PM_EDEVICE;
  if (hipMemcpy(params, d.P, kMlpParams * 4, hipMemcpyDeviceToHost) ||
      hipMemcpy(m, d.M, kMlpParams * 4, hipMemcpyDeviceToHost) ||
      hipMemcpy(v, d.V, kMlpParams * 4, hipMemcpyDeviceToHost))
    return PM_EDEVICE;
  return PM_OK;
}

}  // extern "C"
