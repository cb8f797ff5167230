// Device helpers shared by the plain and fused kernels (internal).
#pragma once
#include "tdb_common.h"

namespace tdb {

// ---------------------------------------------------------------- Jacobi eigensolver
// Cyclic Jacobi on a symmetric rn x rn LDS matrix A with round-robin pairing
// (rn/2 disjoint rotations per round). On exit the diagonal of A holds the
// eigenvalues; if V != nullptr it accumulates the eigenvectors (columns).
static __device__ void jacobi_lds(double* A, double* V, int rn, int* pairs) {
  __shared__ int rotated;
  __shared__ double cs[TDB_RCAP], sn[TDB_RCAP];
  const int m = rn + (rn & 1);               // even size with a dummy index
  if (V)
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) V[t] = (t / rn == t % rn) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      // round-robin schedule: index m-1 fixed, others rotate
      for (int k = threadIdx.x; k < m / 2; k += blockDim.x) {
        int p_, q_;
        if (k == 0) { p_ = m - 1; q_ = round; }
        else { p_ = (round + k) % (m - 1); q_ = (round - k + (m - 1)) % (m - 1); }
        if (p_ > q_) { const int t = p_; p_ = q_; q_ = t; }
        pairs[2 * k] = p_;
        pairs[2 * k + 1] = q_;
        double c = 1.0, s = 0.0;
        if (q_ < rn) {
          const double apq = A[p_ * rn + q_];
          const double app = A[p_ * rn + p_], aqq = A[q_ * rn + q_];
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
            rotated = 1;
          }
        }
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int t = threadIdx.x; t < (m / 2) * rn; t += blockDim.x) {
        const int k = t / rn, col = t % rn;
        const int p_ = pairs[2 * k], q_ = pairs[2 * k + 1];
        if (q_ >= rn || sn[k] == 0.0) continue;
        const double ap = A[p_ * rn + col], aq = A[q_ * rn + col];
        A[p_ * rn + col] = cs[k] * ap - sn[k] * aq;
        A[q_ * rn + col] = sn[k] * ap + cs[k] * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int t = threadIdx.x; t < (m / 2) * rn; t += blockDim.x) {
        const int k = t / rn, row = t % rn;
        const int p_ = pairs[2 * k], q_ = pairs[2 * k + 1];
        if (q_ >= rn || sn[k] == 0.0) continue;
        const double ap = A[row * rn + p_], aq = A[row * rn + q_];
        A[row * rn + p_] = cs[k] * ap - sn[k] * aq;
        A[row * rn + q_] = sn[k] * ap + cs[k] * aq;
        if (V) {
          const double vp = V[row * rn + p_], vq = V[row * rn + q_];
          V[row * rn + p_] = cs[k] * vp - sn[k] * vq;
          V[row * rn + q_] = sn[k] * vp + cs[k] * vq;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  __syncthreads();
}

static __device__ void jacobi_values(double* A, int rn, int* pairs) { jacobi_lds(A, nullptr, rn, pairs); }

// ---------------------------------------------------------------- controller
// Single thread (called by one thread): reads eps^2, nu^2 of the error pass and decides the step's event
// (Sec. 2.5): an add when eps exceeds the trigger, a removal check when the error
// slope over the window is negative with headroom and some mode's weakest direction
// fits in the budget, a restart on a numerical event.
static __device__ void controller_decide(CtrlState* c) {
  c->eps = sqrt(fmax(c->eps2, 0.0));
  c->nu = sqrt(fmax(c->nu2, 0.0));
  c->event = 0;
  c->eps_after = __builtin_nan("");
  c->rank_changed = 0;
  if (c->numeric & 3) { c->decision = DEC_NUMERIC; return; }
  if (!c->adaptive) { c->decision = DEC_NONE; return; }
  const double eps = c->eps;
  if (eps > c->eps_trig) { c->decision = DEC_ADD; return; }
  const int nw = c->slope_window;
  c->window[c->whead] = eps;
  c->whead = (c->whead + 1) % TDB_WIN;
  c->wcount += 1;
  c->decision = DEC_NONE;
  if (c->wcount < nw) return;
  const double last = c->window[(c->whead - 1 + TDB_WIN) % TDB_WIN];
  const double first = c->window[(c->whead - nw + TDB_WIN) % TDB_WIN];
  const double slope = (last - first) / ((nw - 1) * c->dt);
  if (!(slope < 0.0)) return;
  if (eps > 0.5 * c->eps_th) return;
  const double B = c->gamma_th > 0.0 ? (1.0 - c->gamma_th / 100.0) * c->nu2
                                     : 0.25 * c->eps_th * c->eps_th;
  for (int n = 0; n < c->p; ++n) {
    const double s = c->sigma[n][c->ranks[n] - 1];
    if (eps * eps + s * s <= B) { c->decision = DEC_REMOVE; return; }
  }
}


}  // namespace tdb
