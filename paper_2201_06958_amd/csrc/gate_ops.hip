// Learned error gate: a 384 -> 128 -> 128 -> 1 network with tanh-form GELU that
// predicts log10 of the reconstruction error of eq. (error) from 8 steps of the 16
// leading singular values of each core unfolding (eq. (rot)), its training kernels
// (forward, reverse-mode gradient, Adam) and the per-step inference that lets the
// error pass be skipped when the prediction sits far below the threshold.
//
// Parameters, one flat FP32 vector: W1 (128 x 384, row-major) | b1 | W2 (128 x 128) |
// b2 | w3 (128) | b3.
#include "tdb_common.h"
#include "gate.h"
#include <math.h>

namespace tdb {

__device__ __forceinline__ float gelu_f(float x) {
  const float c = 0.7978845608028654f;   // sqrt(2/pi)
  const float u = c * (x + 0.044715f * x * x * x);
  return 0.5f * x * (1.0f + tanhf(u));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float c = 0.7978845608028654f;
  const float u = c * (x + 0.044715f * x * x * x);
  const float t = tanhf(u);
  const float du = c * (1.0f + 3.0f * 0.044715f * x * x);
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * du;
}

__device__ __forceinline__ float block128_sum(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const float s = red[0] + red[1];
  __syncthreads();
  return s;
}

// Forward pass of one sample by a block of 128 threads; x (384 floats) in LDS.
// Optionally keeps the pre-activations and activations of both hidden layers.
__device__ float gate_mlp(const float* __restrict__ P, const float* x, float* a1s, float* red, float* h1o,
                          float* a1o, float* h2o, float* a2o) {
  const int j = threadIdx.x;
  const float* W1 = P + GATE_OFF_W1;
  float h1 = P[GATE_OFF_B1 + j];
  const float* wr = W1 + j * GATE_IN;
#pragma unroll 8
  for (int i = 0; i < GATE_IN; ++i) h1 += wr[i] * x[i];
  const float a1 = gelu_f(h1);
  a1s[j] = a1;
  if (h1o) { h1o[j] = h1; a1o[j] = a1; }
  __syncthreads();
  float h2 = P[GATE_OFF_B2 + j];
  const float* w2r = P + GATE_OFF_W2 + j * GATE_H;
#pragma unroll 8
  for (int k = 0; k < GATE_H; ++k) h2 += w2r[k] * a1s[k];
  const float a2 = gelu_f(h2);
  if (h2o) { h2o[j] = h2; a2o[j] = a2; }
  const float y = block128_sum(P[GATE_OFF_W3 + j] * a2, red) + P[GATE_OFF_B3];
  return y;
}

// ---------------------------------------------------------------- training
// One block per sample: forward pass, keeping what the gradient needs.
__global__ void __launch_bounds__(128) k_gate_fwd(const float* __restrict__ P, const float* __restrict__ X, int n,
                                                  float* H1, float* A1, float* H2, float* A2, float* y) {
  __shared__ float x[GATE_IN], a1s[GATE_H], red[2];
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < GATE_IN; i += 128) x[i] = X[(long long)s * GATE_IN + i];
  __syncthreads();
  const long long o = (long long)s * GATE_H;
  const float v = gate_mlp(P, x, a1s, red, H1 ? H1 + o : nullptr, A1 ? A1 + o : nullptr, H2 ? H2 + o : nullptr,
                           A2 ? A2 + o : nullptr);
  if (threadIdx.x == 0) y[s] = v;
}

// One block per sample: d loss / d pre-activation of both hidden layers and of the
// output (loss = mean squared error over the n samples).
__global__ void __launch_bounds__(128) k_gate_bwd(const float* __restrict__ P, const float* __restrict__ H1,
                                                  const float* __restrict__ H2, const float* __restrict__ y,
                                                  const float* __restrict__ t, int n, float* dH1, float* dH2,
                                                  float* dY) {
  __shared__ float d2[GATE_H];
  const int s = blockIdx.x, j = threadIdx.x;
  const float dy = 2.0f * (y[s] - t[s]) / (float)n;
  const long long o = (long long)s * GATE_H;
  const float g2 = dy * P[GATE_OFF_W3 + j] * gelu_grad_f(H2[o + j]);
  d2[j] = g2;
  dH2[o + j] = g2;
  if (j == 0) dY[s] = dy;
  __syncthreads();
  float da1 = 0.0f;
  const float* W2 = P + GATE_OFF_W2;
#pragma unroll 8
  for (int k = 0; k < GATE_H; ++k) da1 += W2[k * GATE_H + j] * d2[k];
  dH1[o + j] = da1 * gelu_grad_f(H1[o + j]);
}

// One thread per parameter: the gradient summed over the samples in order.
__global__ void __launch_bounds__(256) k_gate_pgrad(const float* __restrict__ X, const float* __restrict__ A1,
                                                    const float* __restrict__ A2, const float* __restrict__ dH1,
                                                    const float* __restrict__ dH2, const float* __restrict__ dY,
                                                    int n, float* G) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= GATE_NP) return;
  float acc = 0.0f;
  if (q < GATE_OFF_B1) {
    const int j = q / GATE_IN, i = q - (q / GATE_IN) * GATE_IN;
    for (int s = 0; s < n; ++s) acc += dH1[(long long)s * GATE_H + j] * X[(long long)s * GATE_IN + i];
  } else if (q < GATE_OFF_W2) {
    const int j = q - GATE_OFF_B1;
    for (int s = 0; s < n; ++s) acc += dH1[(long long)s * GATE_H + j];
  } else if (q < GATE_OFF_B2) {
    const int k = (q - GATE_OFF_W2) / GATE_H, j = (q - GATE_OFF_W2) - k * GATE_H;
    for (int s = 0; s < n; ++s) acc += dH2[(long long)s * GATE_H + k] * A1[(long long)s * GATE_H + j];
  } else if (q < GATE_OFF_W3) {
    const int k = q - GATE_OFF_B2;
    for (int s = 0; s < n; ++s) acc += dH2[(long long)s * GATE_H + k];
  } else if (q < GATE_OFF_B3) {
    const int k = q - GATE_OFF_W3;
    for (int s = 0; s < n; ++s) acc += dY[s] * A2[(long long)s * GATE_H + k];
  } else {
    for (int s = 0; s < n; ++s) acc += dY[s];
  }
  G[q] = acc;
}

// Mean squared error (one block).
__global__ void __launch_bounds__(256) k_gate_loss(const float* __restrict__ y, const float* __restrict__ t, int n,
                                                   float* out) {
  __shared__ float red[4];
  float v = 0.0f;
  for (int s = threadIdx.x; s < n; s += 256) {
    const float d = y[s] - t[s];
    v += d * d;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1] + red[2] + red[3]) / (float)n;
}

// Adam with bias correction; step counts from 1.
__global__ void __launch_bounds__(256) k_gate_adam(float* P, const float* __restrict__ G, float* M, float* V, int step,
                                                   float lr, float b1, float b2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= GATE_NP) return;
  const float g = G[q];
  const float m = b1 * M[q] + (1.0f - b1) * g;
  const float v = b2 * V[q] + (1.0f - b2) * g * g;
  M[q] = m;
  V[q] = v;
  const float mh = m / (1.0f - powf(b1, (float)step));
  const float vh = v / (1.0f - powf(b2, (float)step));
  P[q] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------- inference in a step
// One block of 128 threads per stream, after the post-step kernel has formed this
// step's singular values: append them to the stream's history, predict log10 of this
// step's error once 8 steps exist since the last reinitialisation, and decide whether
// the exact error pass runs.
__global__ void __launch_bounds__(128) kb_gate_infer(GateStepArgs g) {
  __shared__ float x[GATE_IN], a1s[GATE_H], red[2];
  __shared__ int runs;
  const int s = blockIdx.x;
  const CtrlState* c = g.ctrl[s];
  // a held step does not run at all; a step with non-finite data is not applied, so
  // its singular values (those of the kept state) join no history and the exact pass
  // runs (and reports the non-finite data)
  if (c->hold) return;
  if (c->numeric & NUM_NONFINITE) {
    if (threadIdx.x == 0) {
      g.yhat[s] = __builtin_nanf("");
      g.skip[s] = 0;
      g.would_skip[s] = 0;
    }
    return;
  }
  float* hist = g.hist + (long long)s * GATE_W * GATE_ROW;
  const int cnt = g.hcount[s];
  const int slot = cnt % GATE_W;
  for (int t = threadIdx.x; t < GATE_ROW; t += 128) {
    const int n = t / GATE_K, i = t - (t / GATE_K) * GATE_K;
    const double sv = n < c->p ? c->sigma[n][i] : 0.0;
    hist[slot * GATE_ROW + t] = log10f((float)fmax(sv, 1e-30));
  }
  __syncthreads();
  const int have = cnt + 1;
  float yhat = __builtin_nanf("");
  if (have >= GATE_W) {
    for (int t = threadIdx.x; t < GATE_IN; t += 128) {
      const int w = t / GATE_ROW, f = t - (t / GATE_ROW) * GATE_ROW;
      const int sl = (have - GATE_W + w) % GATE_W;
      x[t] = (hist[sl * GATE_ROW + f] - g.mean[t]) / g.stdv[t];
    }
    __syncthreads();
    yhat = gate_mlp(g.params, x, a1s, red, nullptr, nullptr, nullptr, nullptr);
  }
  if (threadIdx.x == 0) {
    int r = have < GATE_W || !(yhat < log10f((float)c->eps_th) - 0.5f);
    // the singular-value part of the removal test: keep exact errors while a mode could
    // drop its last direction within the budget
    const double B = c->gamma_th > 0.0 ? (1.0 - c->gamma_th / 100.0) * c->nu2 : 0.25 * c->eps_th * c->eps_th;
    for (int n = 0; n < c->p; ++n) {
      const double sv = c->sigma[n][c->ranks[n] - 1];
      if (sv * sv <= B) r = 1;
    }
    runs = r;
    g.hcount[s] = have;
    g.yhat[s] = yhat;
    g.skip[s] = (g.mode == GATE_ACTIVE && !r) ? 1 : 0;
    g.would_skip[s] = !r ? 1 : 0;
  }
}

// ---------------------------------------------------------------- launchers
hipError_t gate_forward(const float* P, const float* X, int n, float* H1, float* A1, float* H2, float* A2, float* y,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gate_fwd, dim3(n), dim3(128), 0, s, P, X, n, H1, A1, H2, A2, y);
  return hipGetLastError();
}

hipError_t gate_gradient(const float* P, const float* X, const float* t, int n, GateScratch w, float* G,
                         float* loss, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gate_fwd, dim3(n), dim3(128), 0, s, P, X, n, w.H1, w.A1, w.H2, w.A2, w.y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gate_bwd, dim3(n), dim3(128), 0, s, P, w.H1, w.H2, w.y, t, n, w.dH1, w.dH2, w.dY);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gate_pgrad, dim3((GATE_NP + 255) / 256), dim3(256), 0, s, X, w.A1, w.A2, w.dH1, w.dH2, w.dY,
                     n, G);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss) {
    hipLaunchKernelGGL(k_gate_loss, dim3(1), dim3(256), 0, s, w.y, t, n, loss);
    e = hipGetLastError();
  }
  return e;
}

hipError_t gate_adam(float* P, const float* G, float* M, float* V, int step, float lr, hipStream_t s) {
  hipLaunchKernelGGL(k_gate_adam, dim3((GATE_NP + 255) / 256), dim3(256), 0, s, P, G, M, V, step, lr, 0.9f, 0.999f,
                     1e-8f);
  return hipGetLastError();
}

hipError_t gate_infer(const GateStepArgs& g, int nstreams, hipStream_t s) {
  hipLaunchKernelGGL(kb_gate_infer, dim3(nstreams), dim3(128), 0, s, g);
  return hipGetLastError();
}

}  // namespace tdb
