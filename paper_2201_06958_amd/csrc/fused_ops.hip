// Fused path for third-order streams (p = 3), the production path of the library.
//
// One Heun stage is: a tiled pass over the snapshot pair that forms the data
// difference in LDS and contracts it, per tile, into every quantity the evolution
// equations need, already folded with the core pseudo-inverses (eqs. (Corecont) and
// (basecont)); a deterministic reduction of the per-tile partials; and a row-wise
// finish of the basis right-hand side and the Heun update. The step then
// re-orthonormalises the bases (CholeskyQR2 in the W inner product) and folds the
// triangular factors into the core, prepares the next stage, and runs the weighted
// error pass (eq. (error)) whose last workgroup also takes the controller decision.
//
// Tile of the stage pass: T1 slabs of mode 1 x T2 rows of mode 2 x all of mode 3.
// Per tile (D = V1 - V0 on the tile, B_n = W_n U_n, all local):
//   Z  = D x_3 B3^T                 (T1, T2, r3)
//   F1 = Z x_2 B2^T                 (T1, r2, r3)  rows of F_1 on this tile (partial in i2)
//   F2 = Z x_1 B1^T                 (r1, T2, r3)  rows of F_2 (partial in i1)
//   F3 = (D x_2 B2^T) x_1 B1^T      (r1, r2, N3)  F_3 partial (only if mode 3 is not full rank)
//   Cdot_p = F1 x_1 B1^T            (r1, r2, r3)
//   H_n,p = F_n,p(n) P_n, M_n,p = B_n(tile rows)^T H_n,p
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "device_util.h"
#include <math.h>

namespace tdb {

// ---------------------------------------------------------------- stage pass
template <typename TD, typename T>
__global__ void __launch_bounds__(256) k_fpass(FPassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int N2 = a.N2, N3 = a.N3, r1 = a.r1, r2 = a.r2, r3 = a.r3;
  const int T1 = a.T1, T2 = a.T2;
  const int t1 = blockIdx.x / a.nt2, t2 = blockIdx.x % a.nt2;
  const int i1_0 = t1 * T1, i2_0 = t2 * T2;
  const int n1 = min(T1, a.N1 - i1_0), n2 = min(T2, N2 - i2_0);
  // LDS carve-up
  T* Ds = sm;                               // T1*T2*N3
  T* Zs = Ds + T1 * T2 * N3;                // T1*T2*r3
  T* F1 = Zs + T1 * T2 * r3;                // T1*r2*r3
  T* F2 = F1 + T1 * r2 * r3;                // r1*T2*r3
  T* B1s = F2 + r1 * T2 * r3;               // T1*r1
  T* B2s = B1s + T1 * r1;                   // T2*r2
  T* B3s = B2s + T2 * r2;                   // N3*r3
  T* H1s = B3s + N3 * r3;                   // T1*r1
  T* H2s = H1s + T1 * r1;                   // T2*r2
  T* H3s = H2s + T2 * r2;                   // N3*r3
  T* Ys = H3s + N3 * r3;                    // T1*r2*N3 (need_f3)
  T* F3 = Ys + (a.need_f3 ? T1 * r2 * N3 : 0);   // r1*r2*N3 (need_f3)
  const int tid = threadIdx.x, nth = blockDim.x;

  // load the tile of the data difference and the local basis rows
  const int row = T2 * N3;
  for (int t = tid; t < T1 * row; t += nth) {
    const int i1l = t / row, rest = t - i1l * row;
    const int i2l = rest / N3;
    T v = (T)0;
    if (i1l < n1 && i2l < n2) {
      const long long g = ((long long)(i1_0 + i1l) * N2 + i2_0) * N3 + rest;
      v = (T)static_cast<const TD*>(a.V1)[g] - (T)static_cast<const TD*>(a.V0)[g];
    }
    Ds[t] = v;
  }
  const T* B1 = static_cast<const T*>(a.B1);
  const T* B2 = static_cast<const T*>(a.B2);
  const T* B3 = static_cast<const T*>(a.B3);
  for (int t = tid; t < T1 * r1; t += nth) {
    const int i = t / r1;
    B1s[t] = i < n1 ? B1[(long long)(i1_0 + i) * r1 + (t - i * r1)] : (T)0;
  }
  for (int t = tid; t < T2 * r2; t += nth) {
    const int i = t / r2;
    B2s[t] = i < n2 ? B2[(long long)(i2_0 + i) * r2 + (t - i * r2)] : (T)0;
  }
  for (int t = tid; t < N3 * r3; t += nth) B3s[t] = B3[t];
  __syncthreads();

  // Z = D x_3 B3^T ; Y = D x_2 B2^T
  for (int t = tid; t < T1 * T2 * r3; t += nth) {
    const int c2 = t % r3, q = t / r3;          // q = i1l*T2 + i2l
    const T* d = Ds + q * N3;
    T s = (T)0;
    for (int c = 0; c < N3; ++c) s += d[c] * B3s[c * r3 + c2];
    Zs[t] = s;
  }
  if (a.need_f3) {
    for (int t = tid; t < T1 * r2 * N3; t += nth) {
      const int c = t % N3, q = t / N3;
      const int b = q % r2, i1l = q / r2;
      T s = (T)0;
      for (int i2l = 0; i2l < T2; ++i2l) s += B2s[i2l * r2 + b] * Ds[(i1l * T2 + i2l) * N3 + c];
      Ys[t] = s;
    }
  }
  __syncthreads();

  // F1 = Z x_2 B2^T ; F2 = Z x_1 B1^T ; F3 = Y x_1 B1^T
  for (int t = tid; t < T1 * r2 * r3; t += nth) {
    const int c2 = t % r3, q = t / r3;
    const int b = q % r2, i1l = q / r2;
    T s = (T)0;
    for (int i2l = 0; i2l < T2; ++i2l) s += B2s[i2l * r2 + b] * Zs[(i1l * T2 + i2l) * r3 + c2];
    F1[t] = s;
  }
  for (int t = tid; t < r1 * T2 * r3; t += nth) {
    const int c2 = t % r3, q = t / r3;
    const int i2l = q % T2, ai = q / T2;
    T s = (T)0;
    for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + ai] * Zs[(i1l * T2 + i2l) * r3 + c2];
    F2[t] = s;
  }
  if (a.need_f3) {
    for (int t = tid; t < r1 * r2 * N3; t += nth) {
      const int c = t % N3, q = t / N3;
      const int b = q % r2, ai = q / r2;
      T s = (T)0;
      for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + ai] * Ys[(i1l * r2 + b) * N3 + c];
      F3[t] = s;
    }
  }
  __syncthreads();

  // partial outputs of this tile
  T* out = static_cast<T*>(a.part) + (long long)blockIdx.x * a.slot;
  T* oH1 = out;
  T* oH2 = oH1 + T1 * r1;
  T* oH3 = oH2 + T2 * r2;
  T* oC = oH3 + N3 * r3;
  T* oM1 = oC + r1 * r2 * r3;
  T* oM2 = oM1 + r1 * r1;
  T* oM3 = oM2 + r2 * r2;
  const T* P1 = static_cast<const T*>(a.P1);
  const T* P2 = static_cast<const T*>(a.P2);
  const T* P3 = static_cast<const T*>(a.P3);
  // core partial: Cdot_p[a][b][c2] = sum_i1 B1[i1][a] F1[i1][b][c2]
  for (int t = tid; t < r1 * r2 * r3; t += nth) {
    const int bc = t % (r2 * r3), ai = t / (r2 * r3);
    T s = (T)0;
    for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + ai] * F1[i1l * r2 * r3 + bc];
    oC[t] = s;
  }
  // H1_p[i1][a] = sum_(b,c2) F1[i1][b][c2] P1[(b,c2)][a]
  if (a.need_h1) {
    for (int t = tid; t < T1 * r1; t += nth) {
      const int ai = t % r1, i1l = t / r1;
      T s = (T)0;
      const T* f = F1 + i1l * r2 * r3;
      for (int k = 0; k < r2 * r3; ++k) s += f[k] * P1[k * r1 + ai];
      H1s[t] = s;
      oH1[t] = s;
    }
  }
  // H2_p[i2][b] = sum_(a,c2) F2[a][i2][c2] P2[(a,c2)][b]
  if (a.need_h2) {
    for (int t = tid; t < T2 * r2; t += nth) {
      const int b = t % r2, i2l = t / r2;
      T s = (T)0;
      for (int ai = 0; ai < r1; ++ai) {
        const T* f = F2 + (ai * T2 + i2l) * r3;
        const T* pp = P2 + (ai * r3) * r2 + b;
        for (int c2 = 0; c2 < r3; ++c2) s += f[c2] * pp[c2 * r2];
      }
      H2s[t] = s;
      oH2[t] = s;
    }
  }
  // H3_p[c][c2] = sum_(a,b) F3[a][b][c] P3[(a,b)][c2]  (rows of mode 3 are all here)
  if (a.need_f3) {
    for (int t = tid; t < N3 * r3; t += nth) {
      const int c2 = t % r3, c = t / r3;
      T s = (T)0;
      for (int k = 0; k < r1 * r2; ++k) s += F3[k * N3 + c] * P3[k * r3 + c2];
      H3s[t] = s;
      oH3[t] = s;
    }
  }
  __syncthreads();
  // M_n,p = B_n(rows)^T H_n,p
  if (a.need_h1) {
    for (int t = tid; t < r1 * r1; t += nth) {
      const int j = t % r1, i = t / r1;
      T s = (T)0;
      for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + i] * H1s[i1l * r1 + j];
      oM1[t] = s;
    }
  }
  if (a.need_h2) {
    for (int t = tid; t < r2 * r2; t += nth) {
      const int j = t % r2, i = t / r2;
      T s = (T)0;
      for (int i2l = 0; i2l < T2; ++i2l) s += B2s[i2l * r2 + i] * H2s[i2l * r2 + j];
      oM2[t] = s;
    }
  }
  if (a.need_f3) {
    for (int t = tid; t < r3 * r3; t += nth) {
      const int j = t % r3, i = t / r3;
      T s = (T)0;
      for (int c = 0; c < N3; ++c) s += B3s[c * r3 + i] * H3s[c * r3 + j];
      oM3[t] = s;
    }
  }
}

// ---------------------------------------------------------------- reduction
// Sums the per-tile partials in a fixed order (FP64) into H_n, M_n and C_dot, and
// applies the Heun update to the core (stage 1: k = C_dot/dt, C* = C + dt k;
// stage 2: C <- C + dt/2 (k + C_dot/dt)).
template <typename T>
__global__ void __launch_bounds__(256) k_freduce(FReduceArgs a, CtrlState* ctrl) {
  if (a.stage == 2 && ctrl->numeric) return;
  // A singular core found while preparing this step (bit 4, set by k_fpost) belongs
  // to this step's first stage, like the failure of its pseudo-inverse would.
  if (a.stage == 1 && blockIdx.x == 0 && threadIdx.x == 0 && (ctrl->numeric & 4)) ctrl->numeric = 1;
  const T* part = static_cast<const T*>(a.part);
  const long long nH1 = a.need_h1 ? (long long)a.N1 * a.r1 : 0;
  const long long nH2 = a.need_h2 ? (long long)a.N2 * a.r2 : 0;
  const long long nH3 = a.need_f3 ? (long long)a.N3 * a.r3 : 0;
  const long long nC = (long long)a.r1 * a.r2 * a.r3;
  const long long nM1 = a.need_h1 ? a.r1 * a.r1 : 0, nM2 = a.need_h2 ? a.r2 * a.r2 : 0;
  const long long nM3 = a.need_f3 ? a.r3 * a.r3 : 0;
  const long long total = nH1 + nH2 + nH3 + nC + nM1 + nM2 + nM3;
  const int ntiles = a.nt1 * a.nt2;
  const long long oH2 = (long long)a.T1 * a.r1, oH3 = oH2 + (long long)a.T2 * a.r2;
  const long long oC = oH3 + (long long)a.N3 * a.r3, oM1 = oC + nC, oM2 = oM1 + (long long)a.r1 * a.r1;
  const long long oM3 = oM2 + (long long)a.r2 * a.r2;
  const double inv_dt = 1.0 / a.dt;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    long long q = t;
    if (q < nH1) {
      const long long i1 = q / a.r1;
      const int ai = (int)(q - i1 * a.r1);
      const int t1 = (int)(i1 / a.T1), i1l = (int)(i1 - (long long)t1 * a.T1);
      for (int t2 = 0; t2 < a.nt2; ++t2)
        s += (double)part[(long long)(t1 * a.nt2 + t2) * a.slot + i1l * a.r1 + ai];
      a.H[0][q] = s;
      continue;
    }
    q -= nH1;
    if (q < nH2) {
      const long long i2 = q / a.r2;
      const int b = (int)(q - i2 * a.r2);
      const int t2 = (int)(i2 / a.T2), i2l = (int)(i2 - (long long)t2 * a.T2);
      for (int t1 = 0; t1 < a.nt1; ++t1)
        s += (double)part[(long long)(t1 * a.nt2 + t2) * a.slot + oH2 + i2l * a.r2 + b];
      a.H[1][q] = s;
      continue;
    }
    q -= nH2;
    if (q < nH3) {
      for (int k = 0; k < ntiles; ++k) s += (double)part[(long long)k * a.slot + oH3 + q];
      a.H[2][q] = s;
      continue;
    }
    q -= nH3;
    if (q < nC) {
      for (int k = 0; k < ntiles; ++k) s += (double)part[(long long)k * a.slot + oC + q];
      const double cd = s * inv_dt;
      if (a.stage == 1) {
        a.kC[q] = cd;
        a.Cs[q] = a.C0[q] + a.dt * cd;
      } else {
        a.C0[q] += 0.5 * a.dt * (a.kC[q] + cd);
      }
      continue;
    }
    q -= nC;
    long long off = oM1;
    int m = 0;
    if (q >= nM1) { q -= nM1; off = oM2; m = 1; if (q >= nM2) { q -= nM2; off = oM3; m = 2; } }
    for (int k = 0; k < ntiles; ++k) s += (double)part[(long long)k * a.slot + off + q];
    a.M[m][q] = s;
  }
}

// ---------------------------------------------------------------- prep helpers
// Core Gram of the mode-n unfolding into LDS G (rn x rn) from a core staged in LDS.
__device__ void gram_from(const double* Cl, int rn, long long R, long long inner, double* G) {
  const int npair = rn * (rn + 1) / 2;
  for (int t = threadIdx.x; t < npair; t += blockDim.x) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    const int j = t - i * (i + 1) / 2;
    double s = 0.0;
    for (long long c = 0; c < R; ++c) {
      const long long o = c / inner, in = c - o * inner;
      s += Cl[(o * rn + i) * inner + in] * Cl[(o * rn + j) * inner + in];
    }
    G[i * rn + j] = s;
    G[j * rn + i] = s;
  }
  __syncthreads();
}

// Cholesky with the singularity test (pivot below TDB_PIVOT_FLOOR x max diagonal).
__device__ bool chol_inplace(double* A, int rn) {
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
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x)
    if (t % rn > t / rn) A[t] = 0.0;
  __syncthreads();
  return bad == 0;
}

// P_n = C_(n)^T G^-1 from the Cholesky factor L (in G) of the core Gram; Li scratch.
template <typename T>
__device__ void write_pinv(const double* Cl, double* G, double* Li, int rn, long long R, long long inner,
                           T* P) {
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Li[t] = 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < rn; j += blockDim.x) {
    Li[j * rn + j] = 1.0 / G[j * rn + j];
    for (int i = j + 1; i < rn; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += G[i * rn + k] * Li[k * rn + j];
      Li[i * rn + j] = -s / G[i * rn + i];
    }
  }
  __syncthreads();
  // G <- Li^T Li = G^-1
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
    const int i = t / rn, j = t % rn;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < rn; ++k) s += Li[k * rn + i] * Li[k * rn + j];
    G[t] = s;   // safe: every thread reads only Li here
  }
  __syncthreads();
  for (long long t = threadIdx.x; t < R * rn; t += blockDim.x) {
    const long long c = t / rn;
    const int j = (int)(t - c * rn);
    const long long o = c / inner, in = c - o * inner;
    double s = 0.0;
    for (int b = 0; b < rn; ++b) s += Cl[(o * rn + b) * inner + in] * G[b * rn + j];
    P[t] = (T)s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- finish a stage
// Blocks [0, rowblocks): rows of every mode: U_dot = (H - U M)/dt, Heun update and,
// in stage 1, the weighted basis B_n = W_n U* of the next stage.
// Blocks [rowblocks, rowblocks + 3) (stage 1 only): pseudo-inverse P_n at the stage
// core C* (already updated by the reduction).
template <typename T>
__global__ void __launch_bounds__(256) k_ffinish(FFinishArgs a, CtrlState* ctrl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (a.stage == 2 && ctrl->numeric) return;
  const double inv_dt = 1.0 / a.dt;
  if ((int)blockIdx.x < a.rowblocks) {
    long long tot = 0;
    for (int n = 0; n < 3; ++n) tot += a.N[n] * a.r[n];
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (long long)a.rowblocks * blockDim.x) {
      long long q = t;
      int n = 0;
      while (q >= a.N[n] * a.r[n]) { q -= a.N[n] * a.r[n]; ++n; }
      const int rn = a.r[n], ld = a.ldU[n];
      const long long i = q / rn;
      const int j = (int)(q - i * rn);
      const double* Ust = a.stage == 1 ? a.U0[n] : a.Us[n];
      double ud = 0.0;
      if (rn < a.N[n]) {
        double s = a.H[n][q];
        const double* M = a.M[n];
        for (int k = 0; k < rn; ++k) s -= Ust[i * ld + k] * M[k * rn + j];
        ud = s * inv_dt;
      }
      if (a.stage == 1) {
        a.kU[n][i * ld + j] = ud;
        const double us = a.U0[n][i * ld + j] + a.dt * ud;
        a.Us[n][i * ld + j] = us;
        static_cast<T*>(a.B[n])[q] = (T)(a.w[n][i] * us);
      } else {
        a.U0[n][i * ld + j] += 0.5 * a.dt * (a.kU[n][i * ld + j] + ud);
      }
    }
    return;
  }
  // pseudo-inverse at the stage core
  const int n = blockIdx.x - a.rowblocks;
  const int rn = a.r[n];
  if (rn >= a.N[n]) return;
  long long inner = 1, R = 1, csz = 1;
  for (int k = 0; k < 3; ++k) {
    csz *= a.r[k];
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  double* G = lds;
  double* Li = G + TDB_RCAP * TDB_RCAP;
  double* Cl = Li + TDB_RCAP * TDB_RCAP;
  const double* Csrc = a.Cs;
  if (a.core_in_lds) {
    for (long long t = threadIdx.x; t < csz; t += blockDim.x) Cl[t] = Csrc[t];
    __syncthreads();
    Csrc = Cl;
  }
  gram_from(Csrc, rn, R, inner, G);
  if (!chol_inplace(G, rn)) {
    if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 1);
    return;
  }
  write_pinv<T>(Csrc, G, Li, rn, R, inner, static_cast<T*>(a.P[n]));
}

// ---------------------------------------------------------------- QR + fold
// Block n: two rounds of Cholesky QR of U_n in the W inner product (U_n <- U_n R^-1,
// R accumulated); the last block to finish folds every R_n into the core.
__global__ void __launch_bounds__(256) k_fqr(FQrArgs a, CtrlState* ctrl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int last, skip_s;
  // every block takes part in the completion count, even when there is nothing to do;
  // the flag is read once per block so that the whole block takes the same branch
  if (threadIdx.x == 0)
    skip_s = __hip_atomic_load(&ctrl->numeric, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  const bool skip = skip_s != 0;
  const int n = blockIdx.x;
  const int rn = a.r[n], ld = a.ldU[n];
  const long long Nn = a.N[n];
  double* L = lds;                          // rn*rn
  double* Rt = L + TDB_RCAP * TDB_RCAP;     // rn*rn
  double* Tm = Rt + TDB_RCAP * TDB_RCAP;    // rn*rn
  double* Ul = Tm + TDB_RCAP * TDB_RCAP;    // Nn*rn when staged
  double* U = a.U0[n];
  const double* w = a.w[n];
  const bool stage = a.u_in_lds[n] && !skip;
  if (stage) {
    for (long long t = threadIdx.x; t < Nn * rn; t += blockDim.x) {
      const long long i = t / rn;
      Ul[t] = U[i * ld + (t - i * rn)];
    }
  }
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Rt[t] = (t / rn == t % rn) ? 1.0 : 0.0;
  __syncthreads();
  double* Uw = stage ? Ul : U;
  const int ldw = stage ? rn : ld;
  bool ok = !skip;
  for (int round = 0; round < 2 && ok; ++round) {
    for (int t = threadIdx.x; t < rn * (rn + 1) / 2; t += blockDim.x) {
      int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while ((i + 1) * (i + 2) / 2 <= t) ++i;
      while (i * (i + 1) / 2 > t) --i;
      const int j = t - i * (i + 1) / 2;
      double s = 0.0;
      for (long long q = 0; q < Nn; ++q) s += w[q] * Uw[q * ldw + i] * Uw[q * ldw + j];
      L[i * rn + j] = s;
      L[j * rn + i] = s;
    }
    __syncthreads();
    ok = chol_inplace(L, rn);
    if (!ok) break;
    for (long long q = threadIdx.x; q < Nn; q += blockDim.x) {
      double* rowp = Uw + q * ldw;
      for (int j = 0; j < rn; ++j) {
        double s = rowp[j];
        for (int k = 0; k < j; ++k) s -= L[j * rn + k] * rowp[k];
        rowp[j] = s / L[j * rn + j];
      }
    }
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
      const int i = t / rn, j = t % rn;
      double s = 0.0;
      for (int k = i; k < rn; ++k) s += L[k * rn + i] * Rt[k * rn + j];
      Tm[t] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Rt[t] = Tm[t];
    __syncthreads();
  }
  if (skip) {
  } else if (!ok) {
    if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 2);
  } else {
    if (stage) {
      for (long long t = threadIdx.x; t < Nn * rn; t += blockDim.x) {
        const long long i = t / rn;
        U[i * ld + (t - i * rn)] = Ul[t];
      }
    }
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) a.Rq[n][t] = Rt[t];
  }
  // last block folds the factors into the core
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) *a.counter = 0u;
  if (__hip_atomic_load(&ctrl->numeric, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) return;
  long long csz = 1;
  for (int k = 0; k < 3; ++k) csz *= a.r[k];
  for (int m = 0; m < 3; ++m) {
    const int rm = a.r[m];
    for (int t = threadIdx.x; t < rm * rm; t += blockDim.x)
      Rt[t] = __hip_atomic_load(&a.Rq[m][t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    long long inner = 1;
    for (int k = m + 1; k < 3; ++k) inner *= a.r[k];
    for (long long t = threadIdx.x; t < csz; t += blockDim.x) {
      const long long in = t % inner, rest = t / inner;
      const int ai = (int)(rest % rm);
      const long long o = rest / rm;
      double s = 0.0;
      for (int b = ai; b < rm; ++b) s += Rt[ai * rm + b] * a.C0[(o * rm + b) * inner + in];
      a.Ctmp[t] = s;
    }
    __syncthreads();
    for (long long t = threadIdx.x; t < csz; t += blockDim.x) a.C0[t] = a.Ctmp[t];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- post-step
// Blocks [0, 3): for mode n at the new state: core singular values (Jacobi, into the
// controller), pseudo-inverse P_n and weighted basis B_n for the next stage 1.
// Blocks [3, 3 + eblocks): the partial expansion E = C x_2 U_2 x_3 U_3 used by the
// error pass, and the mode-1 basis in the compute type.
template <typename T>
__global__ void __launch_bounds__(256) k_fpost(FPostArgs a, CtrlState* ctrl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int pairs[TDB_RCAP + 2];
  __shared__ int order[TDB_RCAP];
  if ((int)blockIdx.x >= 3) {
    const int eb = blockIdx.x - 3;
    const int r1 = a.r[0], r2 = a.r[1], r3 = a.r[2];
    const long long N2 = a.N[1], N3 = a.N[2];
    const long long tot = (long long)r1 * N2 * N3;
    T* E = static_cast<T*>(a.E);
    for (long long t = (long long)eb * blockDim.x + threadIdx.x; t < tot; t += (long long)a.eblocks * blockDim.x) {
      const long long i3 = t % N3, q = t / N3;
      const long long i2 = q % N2;
      const int ai = (int)(q / N2);
      const double* u2 = a.U[1] + i2 * a.ldU[1];
      const double* u3 = a.U[2] + i3 * a.ldU[2];
      double s = 0.0;
      for (int b = 0; b < r2; ++b) {
        const double* cr = a.C + ((long long)ai * r2 + b) * r3;
        double s3 = 0.0;
        for (int c = 0; c < r3; ++c) s3 += cr[c] * u3[c];
        s += u2[b] * s3;
      }
      E[t] = (T)s;
    }
    const long long tu = a.N[0] * r1;
    T* U1c = static_cast<T*>(a.U1c);
    for (long long t = (long long)eb * blockDim.x + threadIdx.x; t < tu; t += (long long)a.eblocks * blockDim.x) {
      const long long i = t / r1;
      U1c[t] = (T)a.U[0][i * a.ldU[0] + (t - i * r1)];
    }
    return;
  }
  const int n = blockIdx.x;
  const int rn = a.r[n];
  long long inner = 1, R = 1, csz = 1;
  for (int k = 0; k < 3; ++k) {
    csz *= a.r[k];
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  // weighted basis of the next stage 1
  T* B = static_cast<T*>(a.B[n]);
  for (long long t = threadIdx.x; t < a.N[n] * rn; t += blockDim.x) {
    const long long i = t / rn;
    B[t] = (T)(a.w[n][i] * a.U[n][i * a.ldU[n] + (t - i * rn)]);
  }
  double* G = lds;
  double* Li = G + TDB_RCAP * TDB_RCAP;
  double* Cl = Li + TDB_RCAP * TDB_RCAP;
  const double* Csrc = a.C;
  if (a.core_in_lds) {
    for (long long t = threadIdx.x; t < csz; t += blockDim.x) Cl[t] = Csrc[t];
    __syncthreads();
    Csrc = Cl;
  }
  gram_from(Csrc, rn, R, inner, G);
  // singular values: Jacobi on a copy in Li
  for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Li[t] = G[t];
  __syncthreads();
  jacobi_values(Li, rn, pairs);
  if (threadIdx.x == 0) {
    for (int i = 0; i < rn; ++i) order[i] = i;
    for (int i = 0; i < rn; ++i) {
      int best = i;
      for (int j = i + 1; j < rn; ++j)
        if (Li[order[j] * rn + order[j]] > Li[order[best] * rn + order[best]]) best = j;
      const int tt = order[i]; order[i] = order[best]; order[best] = tt;
    }
    for (int i = 0; i < TDB_RCAP; ++i)
      ctrl->sigma[n][i] = (i < rn) ? sqrt(fmax(Li[order[i] * rn + order[i]], 0.0)) : 0.0;
  }
  __syncthreads();
  if (rn >= a.N[n] || !a.want_pinv) return;
  if (!chol_inplace(G, rn)) {
    if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 4);
    return;
  }
  write_pinv<T>(Csrc, G, Li, rn, R, inner, static_cast<T*>(a.P[n]));
}

// ---------------------------------------------------------------- error pass
// Tile = T1 slabs of mode 1. rec[i1][j] = sum_a U1[i1][a] E[a][j] (j over modes 2,3);
// partial sums of w (V - rec)^2 and w V^2 in FP64; the last block reduces them and
// runs the controller decision.
template <typename TD, typename T>
__global__ void __launch_bounds__(256) k_ferr(FErrArgs a, CtrlState* ctrl) {
  __shared__ double red[16];
  __shared__ int last;
  const long long M = a.M;      // N2*N3
  const int r1 = a.r1;
  const int i1_0 = blockIdx.y * a.T1;
  const int n1 = min(a.T1, a.N1 - i1_0);
  const T* E = static_cast<const T*>(a.E);
  const T* U1 = static_cast<const T*>(a.U1c);
  double se = 0.0, sv = 0.0;
  for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (long long)gridDim.x * blockDim.x) {
    T acc[FERR_T1];
    for (int q = 0; q < FERR_T1; ++q) acc[q] = (T)0;
    for (int ai = 0; ai < r1; ++ai) {
      const T e = E[(long long)ai * M + j];
      for (int q = 0; q < FERR_T1; ++q)
        if (q < n1) acc[q] += U1[(long long)(i1_0 + q) * r1 + ai] * e;
    }
    const double w23 = a.w23[j];
    for (int q = 0; q < FERR_T1; ++q) {
      if (q >= n1) break;
      const long long g = (long long)(i1_0 + q) * M + j;
      const TD v = static_cast<const TD*>(a.V)[g];
      const double d = (double)((T)v - acc[q]);
      const double ww = a.w1[i1_0 + q] * w23;
      se += ww * d * d;
      sv += ww * (double)v * (double)v;
    }
  }
  se = block_sum(se, red);
  sv = block_sum(sv, red);
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    a.part[2 * bid] = se;
    a.part[2 * bid + 1] = sv;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == gridDim.x * gridDim.y - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int nb = gridDim.x * gridDim.y;
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += __hip_atomic_load(&a.part[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s1 += __hip_atomic_load(&a.part[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    *a.counter = 0u;
    ctrl->eps2 = s0;
    ctrl->nu2 = s1;
    controller_decide(ctrl);
  }
}

// ---------------------------------------------------------------- launchers
template <typename TD, typename T>
hipError_t launch_fpass(const FPassArgs& a, size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fpass<TD, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fpass<TD, T>), dim3(a.nt1 * a.nt2), dim3(256), lds, s, a);
  return hipGetLastError();
}
template hipError_t launch_fpass<float, float>(const FPassArgs&, size_t, hipStream_t);
template hipError_t launch_fpass<float, double>(const FPassArgs&, size_t, hipStream_t);
template hipError_t launch_fpass<double, double>(const FPassArgs&, size_t, hipStream_t);
template hipError_t launch_fpass<double, float>(const FPassArgs&, size_t, hipStream_t);

template <typename T>
hipError_t launch_freduce(const FReduceArgs& a, CtrlState* c, hipStream_t s) {
  long long total = (long long)a.r1 * a.r2 * a.r3 + (a.need_h1 ? (long long)a.N1 * a.r1 + a.r1 * a.r1 : 0) +
                    (a.need_h2 ? (long long)a.N2 * a.r2 + a.r2 * a.r2 : 0) +
                    (a.need_f3 ? (long long)a.N3 * a.r3 + a.r3 * a.r3 : 0);
  long long blocks = (total + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_freduce<T>, dim3((unsigned)blocks), dim3(256), 0, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_freduce<float>(const FReduceArgs&, CtrlState*, hipStream_t);
template hipError_t launch_freduce<double>(const FReduceArgs&, CtrlState*, hipStream_t);

template <typename T>
hipError_t launch_ffinish(const FFinishArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_ffinish<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const int blocks = a.rowblocks + (a.stage == 1 ? 3 : 0);
  hipLaunchKernelGGL(k_ffinish<T>, dim3(blocks), dim3(256), lds, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_ffinish<float>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);
template hipError_t launch_ffinish<double>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);

hipError_t launch_fqr(const FQrArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fqr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fqr, dim3(3), dim3(256), lds, s, a, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fpost(const FPostArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fpost<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fpost<T>, dim3(3 + a.eblocks), dim3(256), lds, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_fpost<float>(const FPostArgs&, size_t, CtrlState*, hipStream_t);
template hipError_t launch_fpost<double>(const FPostArgs&, size_t, CtrlState*, hipStream_t);

template <typename TD, typename T>
hipError_t launch_ferr(const FErrArgs& a, CtrlState* c, hipStream_t s) {
  hipLaunchKernelGGL((k_ferr<TD, T>), dim3(a.gx, a.gy), dim3(256), 0, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_ferr<float, float>(const FErrArgs&, CtrlState*, hipStream_t);
template hipError_t launch_ferr<float, double>(const FErrArgs&, CtrlState*, hipStream_t);
template hipError_t launch_ferr<double, double>(const FErrArgs&, CtrlState*, hipStream_t);
template hipError_t launch_ferr<double, float>(const FErrArgs&, CtrlState*, hipStream_t);

}  // namespace tdb
