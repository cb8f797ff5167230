// Learned error gate: sizes, parameter layout and launchers (see gate_ops.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "tdb_common.h"

namespace tdb {

constexpr int GATE_W = 8;                       // steps of history
constexpr int GATE_K = 16;                      // singular values per mode
constexpr int GATE_ROW = 3 * GATE_K;            // one step of features (three modes)
constexpr int GATE_IN = GATE_W * GATE_ROW;      // 384
constexpr int GATE_H = 128;
constexpr int GATE_OFF_W1 = 0;
constexpr int GATE_OFF_B1 = GATE_OFF_W1 + GATE_H * GATE_IN;
constexpr int GATE_OFF_W2 = GATE_OFF_B1 + GATE_H;
constexpr int GATE_OFF_B2 = GATE_OFF_W2 + GATE_H * GATE_H;
constexpr int GATE_OFF_W3 = GATE_OFF_B2 + GATE_H;
constexpr int GATE_OFF_B3 = GATE_OFF_W3 + GATE_H;
constexpr int GATE_NP = GATE_OFF_B3 + 1;        // 65921

enum { GATE_OFF = 0, GATE_RECORD = 1, GATE_ACTIVE = 2, GATE_SHADOW = 3 };

struct GateScratch {
  float *H1, *A1, *H2, *A2, *y, *dH1, *dH2, *dY;   // n x 128 (y, dY: n)
};

// Per-step inference over n streams (arrays of n entries, hist n x 8 x 48).
struct GateStepArgs {
  const float* params;
  const float* mean;        // 384
  const float* stdv;        // 384
  CtrlState* const* ctrl;
  float* hist;
  int* hcount;
  float* yhat;
  int* skip;
  int* would_skip;
  int mode;
};

hipError_t gate_forward(const float* P, const float* X, int n, float* H1, float* A1, float* H2, float* A2, float* y,
                        hipStream_t s);
hipError_t gate_gradient(const float* P, const float* X, const float* t, int n, GateScratch w, float* G,
                         float* loss, hipStream_t s);
hipError_t gate_adam(float* P, const float* G, float* M, float* V, int step, float lr, hipStream_t s);
hipError_t gate_infer(const GateStepArgs& g, int nstreams, hipStream_t s);

}  // namespace tdb
