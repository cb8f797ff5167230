// FP64 small-matrix kernels of the TDB step: core Gram pseudo-inverse, basis
// right-hand side and Heun stages, W-orthonormal CholeskyQR2 with the factor folded
// into the core, core-unfolding singular values, and the device controller.
//
// Everything here is O(sum N_n r_n + prod r_n * r) work; one workgroup handles one
// mode (or one stream), so a batch of streams maps to a grid of workgroups.
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "device_util.h"
#include <math.h>

namespace tdb {

// ---------------------------------------------------------------- helpers
// Mode-n unfolding of a C-ordered core with dims r[0..p-1]: element (a, col) of
// C_(n), where the columns enumerate the other indices in C order.
__device__ __forceinline__ long long unf_index(int a, long long col, int rn, long long inner) {
  const long long o = col / inner, in = col - o * inner;
  return (o * rn + a) * inner + in;
}

// sum_q w[q] x[q * sx] y[q * sy] for q < n in increasing order, with eight rows'
// loads in flight at a time.
__device__ __forceinline__ double wdot3(const double* __restrict__ w, const double* __restrict__ x, int sx,
                                        const double* __restrict__ y, int sy, long long n) {
  double s = 0.0;
  long long q = 0;
  for (; q + 8 <= n; q += 8) {
    double a[8], b[8], c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = w[q + u];
      b[u] = x[(q + u) * sx];
      c[u] = y[(q + u) * sy];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += a[u] * b[u] * c[u];
  }
  for (; q < n; ++q) s += w[q] * x[q * sx] * y[q * sy];
  return s;
}

// Gram matrix G = A A^T of the mode-n unfolding of a dense core, into LDS (ld = rn).
__device__ void core_gram(const double* __restrict__ C, int rn, long long R, long long inner,
                          double* G) {
  const int npair = rn * (rn + 1) / 2;
  for (int t = threadIdx.x; t < npair; t += blockDim.x) {
    // map t -> (a, b) with a >= b
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    while (a * (a + 1) / 2 > t) --a;
    const int b = t - a * (a + 1) / 2;
    // the columns c = o * inner + in in increasing order, without a division per term
    double s = 0.0;
    const long long nout = R / inner;
    for (long long o = 0; o < nout; ++o) {
      const double* pa = C + (o * rn + a) * inner;
      const double* pb = C + (o * rn + b) * inner;
      for (long long in = 0; in < inner; ++in) s += pa[in] * pb[in];
    }
    G[a * rn + b] = s;
    G[b * rn + a] = s;
  }
  __syncthreads();
}

// In-place lower Cholesky of an rn x rn LDS matrix (row-major, ld = rn). Returns
// false (in every thread) if a pivot is not positive or falls below
// TDB_PIVOT_FLOOR times the largest diagonal entry.
__device__ bool chol_lds(double* A, int rn, double* red) {
  __shared__ int bad;
  __shared__ double dmax;
  if (threadIdx.x == 0) {
    bad = 0;
    double m = 0.0;
    for (int i = 0; i < rn; ++i) m = fmax(m, A[i * rn + i]);
    dmax = m;
  }
  __syncthreads();
  for (int k = 0; k < rn; ++k) {
    if (threadIdx.x == 0) {
      const double piv = A[k * rn + k];
      if (!(piv > TDB_PIVOT_FLOOR * dmax) || !(piv > 0.0)) bad = 1;
      A[k * rn + k] = sqrt(fmax(piv, 1e-300));
    }
    __syncthreads();
    const double lkk = A[k * rn + k];
    for (int i = k + 1 + threadIdx.x; i < rn; i += blockDim.x) A[i * rn + k] /= lkk;
    __syncthreads();
    const int m = rn - k - 1;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) A[i * rn + j] -= A[i * rn + k] * A[j * rn + k];
    }
    __syncthreads();
  }
  // zero the strict upper triangle
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
    const int i = t / rn, j = t % rn;
    if (j > i) A[t] = 0.0;
  }
  __syncthreads();
  (void)red;
  return bad == 0;
}

// Inverse of a lower-triangular LDS matrix L (rn x rn) into Li (lower).
__device__ void tri_inv_lds(const double* L, double* Li, int rn) {
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Li[t] = 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < rn; j += blockDim.x) {
    // solve L x = e_j, x stored in column j of Li
    Li[j * rn + j] = 1.0 / L[j * rn + j];
    for (int i = j + 1; i < rn; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * rn + k] * Li[k * rn + j];
      Li[i * rn + j] = -s / L[i * rn + i];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- stage preparation
// blockIdx.x = mode n. Writes the weighted basis B_n = W_n U_n (compute type) and,
// unless the mode is full rank, the pseudo-inverse of the core unfolding
// P_n = C_(n)^T (C_(n) C_(n)^T)^-1 (least-squares solution of Sec. 2.2).
template <typename T>
__global__ void __launch_bounds__(TDB_BLOCK) k_stage_prep(StageArgs a, CtrlState* ctrl) {
  __shared__ double G[TDB_RCAP * TDB_RCAP];
  __shared__ double Li[TDB_RCAP * TDB_RCAP];
  __shared__ double red[16];
  const int n = blockIdx.x;
  const int rn = a.r[n];
  const long long Nn = a.N[n];
  const double* __restrict__ U = a.U[n];
  const double* __restrict__ w = a.w[n];
  T* __restrict__ B = (T*)a.B[n];
  for (long long t = threadIdx.x; t < Nn * rn; t += blockDim.x) {
    const long long i = t / rn;
    const int j = (int)(t - i * rn);
    B[t] = (T)(w[i] * U[i * a.ldU[n] + j]);
  }
  if (rn >= Nn) return;   // full-rank mode: its basis derivative vanishes
  long long inner = 1, R = 1;
  for (int k = 0; k < a.p; ++k) {
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  core_gram(a.C, rn, R, inner, G);
  const bool ok = chol_lds(G, rn, red);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 1);
    return;
  }
  tri_inv_lds(G, Li, rn);
  // G^-1 = Li^T Li, stored back into G
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
    const int i = t / rn, j = t % rn;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < rn; ++k) s += Li[k * rn + i] * Li[k * rn + j];
    G[t] = s;
  }
  __syncthreads();
  T* __restrict__ P = (T*)a.P[n];
  for (long long t = threadIdx.x; t < R * rn; t += blockDim.x) {
    const long long c = t / rn;
    const int j = (int)(t - c * rn);
    double s = 0.0;
    for (int b = 0; b < rn; ++b) s += a.C[unf_index(b, c, rn, inner)] * G[b * rn + j];
    P[t] = (T)s;
  }
}

// ---------------------------------------------------------------- basis RHS and Heun
// blockIdx.x = n < p: U_dot_n = (H_n - U_n (W_n U_n)^T H_n) / dt, the complement
// projection of eq. (basecont) written with U_n^T W_n F_(n) P_n = (W_n U_n)^T H_n.
// blockIdx.x == p: the core derivative of eq. (Corecont), C_dot = Cdot_raw * dscale.
// stage 1: k = RHS(S_k), S* = S_k + dt k.  stage 2: S_{k+1} = S_k + dt/2 (k + RHS(S*)).
__global__ void __launch_bounds__(TDB_BLOCK) k_rhs_stage(RhsArgs a, CtrlState* ctrl) {
  __shared__ double M[TDB_RCAP * TDB_RCAP];
  if (a.stage == 2 && ctrl->numeric) return;
  const int n = blockIdx.x;
  const double inv_dt = a.dscale;   // 1/dt for a difference quotient, 1 for a given derivative
  if (n == a.p) {
    const long long nc = a.core_size;
    for (long long t = blockIdx.y * blockDim.x + threadIdx.x; t < nc; t += (long long)gridDim.y * blockDim.x) {
      const double cd = a.Cdot[t] * inv_dt;
      if (a.stage == 1) {
        // NaN or Inf anywhere in the data derivative reaches every entry of C_dot
        if (!isfinite(cd)) atomicOr(&ctrl->numeric, NUM_NONFINITE);
        a.kC[t] = cd;
        a.Cs[t] = a.C0[t] + a.dt * cd;
      } else {
        a.C0[t] = a.C0[t] + 0.5 * a.dt * (a.kC[t] + cd);
      }
    }
    return;
  }
  if (blockIdx.y != 0) return;
  const int rn = a.r[n];
  const long long Nn = a.N[n];
  const int ld = a.ldU[n];
  const double* __restrict__ Ust = (a.stage == 1) ? a.U0[n] : a.Us[n];   // RHS state
  const double* __restrict__ H = a.H[n];
  const double* __restrict__ w = a.w[n];
  double* __restrict__ kU = a.kU[n];
  const bool full = rn >= Nn;
  if (!full) {
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
      const int i = t / rn, j = t % rn;
      M[t] = wdot3(w, Ust + i, ld, H + j, rn, Nn);
    }
  }
  __syncthreads();
  for (long long t = threadIdx.x; t < Nn * rn; t += blockDim.x) {
    const long long i = t / rn;
    const int j = (int)(t - i * rn);
    double ud = 0.0;
    if (!full) {
      double s = H[t];
      for (int k = 0; k < rn; ++k) s -= Ust[i * ld + k] * M[k * rn + j];
      ud = s * inv_dt;
    }
    if (a.stage == 1) {
      kU[i * ld + j] = ud;
      a.Us[n][i * ld + j] = a.U0[n][i * ld + j] + a.dt * ud;
    } else {
      a.U0[n][i * ld + j] += 0.5 * a.dt * (kU[i * ld + j] + ud);
    }
  }
}

// ---------------------------------------------------------------- QR and fold
// One workgroup per stream. For every mode: two rounds of Cholesky QR in the W inner
// product, U_n <- U_n R_n^-1 with U_n^T W_n U_n = R_n^T R_n, then C <- C x_n R_n, so
// the reconstruction is unchanged while eq. (orhonormality) is restored.
__global__ void __launch_bounds__(TDB_BLOCK) k_qr_fold(QrArgs a, CtrlState* ctrl) {
  __shared__ double L[TDB_RCAP * TDB_RCAP];
  __shared__ double Rt[TDB_RCAP * TDB_RCAP];
  __shared__ double Tmp[TDB_RCAP * TDB_RCAP];
  __shared__ double red[16];
  if (ctrl->numeric) return;
  long long csize = 1;
  for (int k = 0; k < a.p; ++k) csize *= a.r[k];
  for (int n = 0; n < a.p; ++n) {
    const int rn = a.r[n];
    const long long Nn = a.N[n];
    const int ld = a.ldU[n];
    double* __restrict__ U = a.U0[n];
    const double* __restrict__ w = a.w[n];
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Rt[t] = (t / rn == t % rn) ? 1.0 : 0.0;
    __syncthreads();
    for (int round = 0; round < 2; ++round) {
      for (int t = threadIdx.x; t < rn * (rn + 1) / 2; t += blockDim.x) {
        int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        while (i * (i + 1) / 2 > t) --i;
        const int j = t - i * (i + 1) / 2;
        const double s = wdot3(w, U + i, ld, U + j, ld, Nn);
        L[i * rn + j] = s;
        L[j * rn + i] = s;
      }
      __syncthreads();
      const bool ok = chol_lds(L, rn, red);
      if (!ok) {
        if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 2);
        return;
      }
      // rows: x L^T = u  (forward substitution, in place)
      for (long long q = threadIdx.x; q < Nn; q += blockDim.x) {
        double* row = U + q * ld;
        for (int j = 0; j < rn; ++j) {
          double s = row[j];
          for (int k = 0; k < j; ++k) s -= L[j * rn + k] * row[k];
          row[j] = s / L[j * rn + j];
        }
      }
      // Rt <- L^T Rt  (upper triangular product accumulates R_total = R2 R1)
      for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
        const int i = t / rn, j = t % rn;
        double s = 0.0;
        for (int k = i; k < rn; ++k) s += L[k * rn + i] * Rt[k * rn + j];
        Tmp[t] = s;
      }
      __syncthreads();
      for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Rt[t] = Tmp[t];
      __syncthreads();
    }
    // C <- C x_n Rt
    long long inner = 1;
    for (int k = n + 1; k < a.p; ++k) inner *= a.r[k];
    for (long long t = threadIdx.x; t < csize; t += blockDim.x) {
      const long long in = t % inner;
      const long long rest = t / inner;
      const int ai = (int)(rest % rn);
      const long long o = rest / rn;
      double s = 0.0;
      for (int b = ai; b < rn; ++b) s += Rt[ai * rn + b] * a.C0[(o * rn + b) * inner + in];
      a.Ctmp[t] = s;
    }
    __syncthreads();
    for (long long t = threadIdx.x; t < csize; t += blockDim.x) a.C0[t] = a.Ctmp[t];
    __syncthreads();
  }
}

// blockIdx.x = mode n: singular values of the core unfolding C_(n) (Sec. 2.4),
// descending, into ctrl->sigma[n]; with Psi != nullptr also the left singular
// vectors (the rotation of eq. (rot)), sign-fixed, row-major rn x rn.
__global__ void __launch_bounds__(TDB_BLOCK) k_core_sigma(SigmaArgs a, CtrlState* ctrl) {
  __shared__ double G[TDB_RCAP * TDB_RCAP];
  __shared__ double V[TDB_RCAP * TDB_RCAP];
  __shared__ int pairs[TDB_RCAP + 2];
  __shared__ int order[TDB_RCAP];
  const int n = blockIdx.x;
  const int rn = a.r[n];
  long long inner = 1, R = 1;
  for (int k = 0; k < a.p; ++k) {
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  core_gram(a.C, rn, R, inner, G);
  const bool vec = a.Psi[n] != nullptr;
  if (!vec) {
    // values only: one-wave tridiagonalisation and bisection
    __shared__ double lam_s[TDB_RCAP], ws_s[4 * TDB_RCAP];
    if (threadIdx.x < 64) {
      wave_eigvals(G, rn, lam_s, ws_s);
      for (int i = threadIdx.x; i < TDB_RCAP; i += 64)
        ctrl->sigma[n][i] = i < rn ? sqrt(fmax(lam_s[i], 0.0)) : 0.0;
    }
    return;
  }
  jacobi_lds(G, V, rn, pairs);
  if (threadIdx.x == 0) {
    // selection sort of the eigenvalues, descending (stable on ties)
    for (int i = 0; i < rn; ++i) order[i] = i;
    for (int i = 0; i < rn; ++i) {
      int best = i;
      for (int j = i + 1; j < rn; ++j)
        if (G[order[j] * rn + order[j]] > G[order[best] * rn + order[best]]) best = j;
      const int t = order[i]; order[i] = order[best]; order[best] = t;
    }
    for (int i = 0; i < TDB_RCAP; ++i)
      ctrl->sigma[n][i] = (i < rn) ? sqrt(fmax(G[order[i] * rn + order[i]], 0.0)) : 0.0;
  }
  __syncthreads();
  if (vec) {
    double* Psi = a.Psi[n];
    for (int j = threadIdx.x; j < rn; j += blockDim.x) {
      const int c = order[j];
      int imax = 0;
      double vmax = -1.0;
      for (int i = 0; i < rn; ++i)
        if (fabs(V[i * rn + c]) > vmax) { vmax = fabs(V[i * rn + c]); imax = i; }
      const double sg = V[imax * rn + c] < 0.0 ? -1.0 : 1.0;
      for (int i = 0; i < rn; ++i) Psi[i * rn + j] = sg * V[i * rn + c];
    }
  }
}

// ---------------------------------------------------------------- controller
__global__ void k_controller(CtrlState* c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  controller_decide(c);
}

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_stage_prep(const StageArgs& a, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_prep<T>, dim3(a.p), dim3(TDB_BLOCK), 0, s, a, ctrl);
  return hipGetLastError();
}
template hipError_t launch_stage_prep<float>(const StageArgs&, CtrlState*, hipStream_t);
template hipError_t launch_stage_prep<double>(const StageArgs&, CtrlState*, hipStream_t);

hipError_t launch_rhs_stage(const RhsArgs& a, CtrlState* ctrl, hipStream_t s) {
  int yb = (int)((a.core_size + TDB_BLOCK - 1) / TDB_BLOCK);
  if (yb > 64) yb = 64;
  if (yb < 1) yb = 1;
  hipLaunchKernelGGL(k_rhs_stage, dim3(a.p + 1, yb), dim3(TDB_BLOCK), 0, s, a, ctrl);
  return hipGetLastError();
}

hipError_t launch_qr_fold(const QrArgs& a, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_qr_fold, dim3(1), dim3(TDB_BLOCK), 0, s, a, ctrl);
  return hipGetLastError();
}

hipError_t launch_core_sigma(const SigmaArgs& a, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_core_sigma, dim3(a.p), dim3(TDB_BLOCK), 0, s, a, ctrl);
  return hipGetLastError();
}

hipError_t launch_controller(CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_controller, dim3(1), dim3(64), 0, s, ctrl);
  return hipGetLastError();
}

}  // namespace tdb
