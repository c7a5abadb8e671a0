// Shapes of the plan cost model and its device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/polymul.h"

namespace pm {

constexpr int kMlpF = 17;  // features
constexpr int kMlpH = 64;  // hidden width
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpF;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 1;

struct MlpDev {
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;       // parameters, gradient, Adam moments
  float *X = nullptr, *T = nullptr, *H1 = nullptr, *H2 = nullptr;     // batch
  float *Y = nullptr, *DY = nullptr, *DZ1 = nullptr, *DZ2 = nullptr;  // activations and deltas
  float* L = nullptr;                                                 // loss
  int cap = 0;
  ~MlpDev();
  void release();
  pm_status ensure(int B);
  hipError_t forward(int B, hipStream_t s);
  hipError_t loss_grad(int B, hipStream_t s);
  hipError_t adam(int step, float lr, hipStream_t s);
};

}  // namespace pm
