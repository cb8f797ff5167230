// Shared device-side definitions of the TDB library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TDB_P 4          // largest tensor order handled by the kernels
#define TDB_RCAP 64      // largest rank cap per mode
#define TDB_WIN 64       // longest error-slope window
#define TDB_NEIG 512     // largest mode size for the device HOSVD eigensolver
#define TDB_BLOCK 256    // threads per block of the small FP64 kernels

// Pointers into device memory that the kernels take from argument tables held in
// device memory: the compiler cannot tell that they address global memory and would
// use flat instructions, and a flat access in flight makes every later wait drain all
// memory counters (no load can be kept in flight across a local-memory access). The
// kernels convert them once with gmem and keep the global type.
#define TDB_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ TDB_GLOBAL T* gmem(T* p) {
  return (TDB_GLOBAL T*)p;
}

// Controller events (same values as the TDB_EV_* codes of the public header).
enum { EV_NONE = 0, EV_REINIT = 1, EV_ADD = 2, EV_REMOVE = 3, EV_NUMERIC = 4 };

// Controller decisions taken on the device after the error pass.
// DEC_NONFINITE: the step's data derivative held NaN or Inf; the step was not applied
// (core and bases kept) and the host reports TDB_ENUMERIC.
enum { DEC_NONE = 0, DEC_ADD = 1, DEC_REMOVE = 2, DEC_NUMERIC = 3, DEC_INIT = 4, DEC_NONFINITE = 5 };

// Bits of CtrlState::numeric.
enum {
  NUM_CORE = 1,        // a stage's core Gram failed its Cholesky test (pseudo-inverse)
  NUM_BASIS = 2,       // a basis Gram failed its Cholesky test (re-orthonormalisation)
  NUM_NEXT = 4,        // the next step's core Gram failed (found by the post-step kernel)
  NUM_NONFINITE = 8    // the first stage's core derivative is not finite (NaN/Inf data)
};

// A direction whose full-data singular value is below this fraction of its mode's
// largest is numerically absent: adding it would make a core Gram matrix singular.
#define TDB_SIGMA_FLOOR 1e-6
// Jacobi rotations are skipped once |a_pq| <= TDB_JACOBI_TOL max_i |a_ii|: a few units
// of roundoff relative to the matrix norm, the accuracy any backward-stable symmetric
// eigensolver reaches (a tolerance relative to sqrt(a_pp a_qq) is never met by pairs
// of tiny diagonal entries next to large ones, and the sweeps would not terminate).
#define TDB_JACOBI_TOL 4e-16
// Core Gram matrices whose smallest Cholesky pivot falls below this fraction of the
// largest diagonal entry are treated as singular (a numerical event).
#define TDB_PIVOT_FLOOR 1e-12

// Device-resident controller state and per-step outputs (error control, Sec. 2.5).
struct CtrlState {
  // configuration
  double eps_th, gamma_th, dt;
  int adaptive, slope_window, p, pad0;
  int caps[TDB_P];
  long long dims[TDB_P];
  // evolving state
  double eps_trig;
  int unmet;
  int ranks[TDB_P];
  int wcount, whead;
  double window[TDB_WIN];
  // outputs of the last step
  int decision;       // DEC_*
  int event;          // TDB_EV_* (see tdb.h)
  int numeric;        // NUM_* bits: a failed Cholesky test or non-finite data
  int rank_changed;
  double eps2, nu2;   // from the error pass
  double eps, nu, eps_after;
  double sigma[TDB_P][TDB_RCAP];   // core unfolding singular values, descending
  int n_events[5];
  int gated;          // the learned gate skipped this step's error pass
  int would_skip;     // the gate's verdict (also when it only observes)
  double eps_pred;    // the gate's predicted error of this step (NaN without one)
  int hold;           // a decision awaits the host: the fused kernels of a step enqueued
                      // after it do nothing until the host has acted and cleared it
};

// Square root of a sum of squares: a tiny negative value from rounding becomes 0, and
// a NaN stays NaN (fmax(NaN, 0) would turn non-finite data into a zero error).
__device__ __forceinline__ double sqrt_sum_sq(double x) { return x >= 0.0 ? sqrt(x) : (x < 0.0 ? 0.0 : x); }

__device__ __forceinline__ double warp_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum (blockDim.x a multiple of 64, <= 1024); result valid in all threads.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = warp_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += scratch[i];   // same order in every thread
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_max(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = scratch[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, scratch[i]);
  __syncthreads();
  return s;
}

// Index helpers for a C-ordered tensor viewed as (outer, N_n, inner) around mode n.
struct ModeView {
  long long outer, inner;
  int n_len;
};
