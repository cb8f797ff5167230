// Fused path for third-order streams (p = 3), the production path of the library.
//
// One Heun stage is: a tiled pass over the snapshot pair that forms the data
// difference in LDS and contracts it, per tile, into every quantity the evolution
// equations need, already folded with the core pseudo-inverses (eqs. (Corecont) and
// (basecont)); a deterministic reduction of the per-tile partials; and a row-wise
// finish of the basis right-hand side and the Heun update. The step then
// re-orthonormalises the bases (Cholesky QR in the W inner product) and folds the
// triangular factors into the core, prepares the next stage, and runs the weighted
// error pass (eq. (error)) followed by a one-workgroup kernel that sums its partials
// and takes the controller decision.
//
// The stage pass itself lives in its own source file.
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "device_util.h"
#include <hip/hip_ext.h>
#include <math.h>

namespace tdb {

// ---------------------------------------------------------------- reduction
// Sum of count values p[k*stride] in a fixed order with 8 independent partial sums
// (so that 8 loads are in flight per thread); deterministic for a given count.
template <typename T>
__device__ __forceinline__ double sum_strided(const T* __restrict__ p, long long stride, int count) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
  int k = 0;
  for (; k + 8 <= count; k += 8) {
    const T* q = p + (long long)k * stride;
    s0 += (double)q[0];
    s1 += (double)q[stride];
    s2 += (double)q[2 * stride];
    s3 += (double)q[3 * stride];
    s4 += (double)q[4 * stride];
    s5 += (double)q[5 * stride];
    s6 += (double)q[6 * stride];
    s7 += (double)q[7 * stride];
  }
  for (; k < count; ++k) {
    const double v = (double)p[(long long)k * stride];
    switch (k & 7) {
      case 0: s0 += v; break; case 1: s1 += v; break; case 2: s2 += v; break; case 3: s3 += v; break;
      case 4: s4 += v; break; case 5: s5 += v; break; case 6: s6 += v; break; default: s7 += v; break;
    }
  }
  return ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
}

// Sums the per-tile partials in a fixed order (FP64) into H_n and C_dot, and applies
// the Heun update to the core (stage 1: k = C_dot/dt, C* = C + dt k; stage 2:
// C <- C + dt/2 (k + C_dot/dt)). Each output is summed by L lanes of one wave (lane
// group j takes partials j, j + L, ...), combined by a fixed butterfly, so the order of
// the additions never depends on scheduling. A wave covers Q = 64/L consecutive
// outputs: lane = j*Q + (output within the wave), so neighbouring lanes read
// neighbouring partials of the same tile.
template <typename T>
__device__ __forceinline__ void freduce_body(const FReduceArgs& a, int stage, CtrlState* ctrl, int bx, int gx) {
  if (stage == 2 && ctrl->numeric) return;
  // A singular core found while preparing this step (bit 4, set by k_fpost) belongs
  // to this step's first stage, like the failure of its pseudo-inverse would.
  if (stage == 1 && bx == 0 && threadIdx.x == 0 && (ctrl->numeric & 4)) ctrl->numeric = 1;
  const T* part = static_cast<const T*>(a.part);
  const long long nH1 = a.need_h1 ? (long long)a.N1 * a.r1 : 0;
  const long long nH2 = a.need_h2 ? (long long)a.N2 * a.r2 : 0;
  const long long nH3 = a.need_f3 ? (long long)a.N3 * a.r3 : 0;
  const long long nC = (long long)a.r1 * a.r2 * a.r3;
  const int ntiles = a.nt1 * a.nt2;
  const int L1 = red_lanes(a.nt2), L2 = red_lanes(a.nt1), L3 = red_lanes(ntiles);
  const long long e1 = pad64(nH1 * L1), e2 = e1 + pad64(nH2 * L2), e3 = e2 + pad64(nH3 * L3);
  const long long e4 = e3 + pad64(nC * L3);
  const long long oH2 = (long long)a.T1 * a.r1, oH3 = oH2 + (long long)a.T2 * a.r2;
  const long long oC = oH3 + (long long)a.N3 * a.r3;
  const double inv_dt = 1.0 / a.dt;
  // e4 is a multiple of 64 and so is the stride: every wave runs the same trip count
  for (long long t = (long long)bx * blockDim.x + threadIdx.x; t < e4; t += (long long)gx * blockDim.x) {
    int kind, L;
    long long u;
    if (t < e1) { kind = 0; L = L1; u = t; }
    else if (t < e2) { kind = 1; L = L2; u = t - e1; }
    else if (t < e3) { kind = 2; L = L3; u = t - e2; }
    else { kind = 3; L = L3; u = t - e3; }
    const int Q = 64 / L;
    const int lw = (int)(u & 63);
    const long long q = (u >> 6) * Q + (lw % Q);
    const int j = lw / Q;
    const long long nq = kind == 0 ? nH1 : kind == 1 ? nH2 : kind == 2 ? nH3 : nC;
    const bool valid = q < nq;
    double s = 0.0;
    if (valid) {
      const T* base;
      long long stride;
      int count;
      if (kind == 0) {
        const long long i1 = q / a.r1;
        const int ai = (int)(q - i1 * a.r1);
        const int t1 = (int)(i1 / a.T1), i1l = (int)(i1 - (long long)t1 * a.T1);
        base = part + (long long)(t1 * a.nt2) * a.slot + i1l * a.r1 + ai;
        stride = a.slot;
        count = a.nt2;
      } else if (kind == 1) {
        const long long i2 = q / a.r2;
        const int b = (int)(q - i2 * a.r2);
        const int t2 = (int)(i2 / a.T2), i2l = (int)(i2 - (long long)t2 * a.T2);
        base = part + (long long)t2 * a.slot + oH2 + i2l * a.r2 + b;
        stride = (long long)a.nt2 * a.slot;
        count = a.nt1;
      } else {
        base = part + (kind == 2 ? oH3 : oC) + q;
        stride = a.slot;
        count = ntiles;
      }
      const int cnt = (count - j + L - 1) / L;
      if (cnt > 0) s = sum_strided(base + (long long)j * stride, stride * L, cnt);
    }
    for (int o = L >> 1; o >= 1; o >>= 1) s += __shfl_xor(s, o * Q, 64);
    if (!valid || j != 0) continue;
    if (kind == 0) {
      a.H[0][q] = s;
    } else if (kind == 1) {
      a.H[1][q] = s;
    } else if (kind == 2) {
      a.H[2][q] = s;
    } else {
      const double cd = s * inv_dt;
      if (stage == 1) {
        a.kC[q] = cd;
        a.Cs[q] = a.C0[q] + a.dt * cd;
      } else {
        a.Cdot2[q] = cd;
        a.C0[q] += 0.5 * a.dt * (a.kC[q] + cd);
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_freduce(FReduceArgs a, CtrlState* ctrl) {
  freduce_body<T>(a, a.stage, ctrl, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- prep helpers
// Core Gram of the mode-n unfolding into LDS G (rn x rn) from a core (LDS or global),
// with the unfolding columns walked as (outer, inner) loops.
__device__ void gram_from(const double* Cl, int rn, long long R_, long long inner_, double* G) {
  const int npair = rn * (rn + 1) / 2;
  const int inner = (int)inner_;
  const int outer = (int)(R_ / inner_);
  for (int t = threadIdx.x; t < npair; t += blockDim.x) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    const int j = t - i * (i + 1) / 2;
    double s0 = 0.0, s1 = 0.0;
    if (inner == 1) {
      const double* ci = Cl + i;
      const double* cj = Cl + j;
      int o = 0;
      for (; o + 2 <= outer; o += 2) {
        s0 += ci[o * rn] * cj[o * rn];
        s1 += ci[(o + 1) * rn] * cj[(o + 1) * rn];
      }
      if (o < outer) s0 += ci[o * rn] * cj[o * rn];
    } else {
      for (int o = 0; o < outer; ++o) {
        const double* ci = Cl + (o * rn + i) * inner;
        const double* cj = Cl + (o * rn + j) * inner;
        int in = 0;
        for (; in + 2 <= inner; in += 2) {
          s0 += ci[in] * cj[in];
          s1 += ci[in + 1] * cj[in + 1];
        }
        if (in < inner) s0 += ci[in] * cj[in];
      }
    }
    const double s = s0 + s1;
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

// P_n = C_(n)^T G^-1 from the inverse Gi (LDS), block-parallel.
template <typename T>
__device__ void write_p(const double* Cl, const double* Gi, int rn, long long R, long long inner, T* P) {
  const int Ri = (int)R, in_ = (int)inner;
  for (int t = threadIdx.x; t < Ri * rn; t += blockDim.x) {
    const int c = t / rn, j = t - (t / rn) * rn;
    const int o = c / in_, in = c - o * in_;
    const double* cp = Cl + (o * rn) * in_ + in;
    double s = 0.0;
    for (int b = 0; b < rn; ++b) s += cp[b * in_] * Gi[b * rn + j];
    P[t] = (T)s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- M_n of a stage
// Block n: M_n = U_n^T W_n F_(n) P_n = C_dot_(n) P_n, scaled by dt like the raw H_n
// (one r_n x r_n matrix per mode, shared by every row of the finish).
template <typename T>
__device__ __forceinline__ void fmprep_body(const FFinishArgs& a, int stage, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (stage == 2 && ctrl->numeric) return;
  const int n = bx;
  const int rr = a.r[n];
  if (rr >= a.N[n]) return;
  const double* cd = stage == 1 ? a.kC : a.Cdot2;   // this stage's C_dot
  const int csz = a.r[0] * a.r[1] * a.r[2];
  const int Rn = csz / rr;
  double* cdl = lds;
  T* pl = reinterpret_cast<T*>(cdl + csz);
  const T* Pn = static_cast<const T*>(a.Pcur[n]);
  for (int t = threadIdx.x; t < csz; t += blockDim.x) cdl[t] = cd[t];
  for (int t = threadIdx.x; t < Rn * rr; t += blockDim.x) pl[t] = Pn[t];
  __syncthreads();
  int inner = 1, outer = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < n) outer *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  for (int t = threadIdx.x; t < rr * rr; t += blockDim.x) {
    const int i = t / rr, j = t - (t / rr) * rr;
    double s = 0.0;
    for (int o = 0; o < outer; ++o) {
      const double* crow = cdl + (o * rr + i) * inner;
      const T* prow = pl + (o * inner) * rr + j;
      for (int in = 0; in < inner; ++in) s += crow[in] * (double)prow[in * rr];
    }
    a.M[n][t] = s * a.dt;   // H is the raw (undivided) projection, so M is too
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fmprep(FFinishArgs a, CtrlState* ctrl) {
  fmprep_body<T>(a, a.stage, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- finish a stage
// Blocks [0, rowblocks): rows of every mode: U_dot = (H - U M)/dt, Heun update and,
// in stage 1, the weighted basis B_n = W_n U* of the next stage.
// Blocks [rowblocks, rowblocks + 3) (stage 1 only): pseudo-inverse P_n at the stage
// core C* (already updated by the reduction).
template <typename T>
__device__ __forceinline__ void ffinish_body(const FFinishArgs& a, int stage, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (stage == 2 && ctrl->numeric) return;
  const double inv_dt = 1.0 / a.dt;
  if ((int)bx < a.rowblocks) {
    // M_n (r_n x r_n) into LDS: formed once per stage by k_fmprep, or here (a single
    // stream, where the extra launch would cost more than the repeated small product)
    double* Ml[3];
    if (a.m_inline) {
      const double* cd = stage == 1 ? a.kC : a.Cdot2;   // this stage's C_dot
      const int csz = a.r[0] * a.r[1] * a.r[2];
      double* cdl = lds;
      T* pl = reinterpret_cast<T*>(cdl + csz);
      for (int t = threadIdx.x; t < csz; t += blockDim.x) cdl[t] = cd[t];
      int poff[3], off = 0;
      for (int n = 0; n < 3; ++n) {
        poff[n] = off;
        if (a.r[n] < a.N[n]) {
          const T* Pn = static_cast<const T*>(a.Pcur[n]);
          for (int t = threadIdx.x; t < csz; t += blockDim.x) pl[off + t] = Pn[t];
          off += csz;
        }
      }
      __syncthreads();
      int moff = (int)((csz * 8 + off * (int)sizeof(T) + 7) / 8);
      for (int n = 0; n < 3; ++n) {
        Ml[n] = lds + moff;
        const int rr = a.r[n];
        if (rr < a.N[n]) {
          int inner = 1, outer = 1;
          for (int k = 0; k < 3; ++k) {
            if (k < n) outer *= a.r[k];
            if (k > n) inner *= a.r[k];
          }
          const T* Pn = pl + poff[n];
          for (int t = threadIdx.x; t < rr * rr; t += blockDim.x) {
            const int i = t / rr, j = t - (t / rr) * rr;
            double s = 0.0;
            for (int o = 0; o < outer; ++o) {
              const double* crow = cdl + (o * rr + i) * inner;
              const T* prow = Pn + (o * inner) * rr + j;
              for (int in = 0; in < inner; ++in) s += crow[in] * (double)prow[in * rr];
            }
            Ml[n][t] = s * a.dt;   // H is the raw (undivided) projection, so M is too
          }
        }
        moff += rr * rr;
      }
    } else {
      int off = 0;
      for (int n = 0; n < 3; ++n) {
        Ml[n] = lds + off;
        const int rr = a.r[n];
        if (rr < a.N[n])
          for (int t = threadIdx.x; t < rr * rr; t += blockDim.x) Ml[n][t] = a.M[n][t];
        off += rr * rr;
      }
    }
    __syncthreads();
    long long tot = 0;
    for (int n = 0; n < 3; ++n) tot += a.N[n] * a.r[n];
    for (long long t = (long long)bx * blockDim.x + threadIdx.x; t < tot;
         t += (long long)a.rowblocks * blockDim.x) {
      long long q = t;
      int n = 0;
      while (q >= a.N[n] * a.r[n]) { q -= a.N[n] * a.r[n]; ++n; }
      const int rn = a.r[n], ld = a.ldU[n];
      const long long i = q / rn;
      const int j = (int)(q - i * rn);
      const double* Ust = stage == 1 ? a.U0[n] : a.Us[n];
      double ud = 0.0;
      if (rn < a.N[n]) {
        double s = a.H[n][q];
        const double* M = Ml[n];
        const double* ur = Ust + i * ld;
        for (int k = 0; k < rn; ++k) s -= ur[k] * M[k * rn + j];
        ud = s * inv_dt;
      }
      if (stage == 1) {
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
  const int n = bx - a.rowblocks;
  const int rn = a.r[n];
  if (rn >= a.N[n]) return;
  long long inner = 1, R = 1, csz = 1;
  for (int k = 0; k < 3; ++k) {
    csz *= a.r[k];
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  const int rq = a.rmax;
  double* G = lds;
  double* Li = G + rq * rq;
  double* Gi = Li + rq * rq;
  double* Cl = Gi + rq * rq;
  __shared__ int ok_s;
  const double* Csrc = a.Cs;
  if (a.core_in_lds) {
    for (int t = threadIdx.x; t < (int)csz; t += blockDim.x) Cl[t] = Csrc[t];
    __syncthreads();
    Csrc = Cl;
  }
  gram_from(Csrc, rn, R, inner, G);
  if (threadIdx.x < 64) {
    const bool ok = wave_chol(G, rn);
    if (ok) {
      wave_tri_inv(G, Li, rn);
      wave_inv_from_linv(Li, Gi, rn);
    }
    if (threadIdx.x == 0) {
      ok_s = ok ? 1 : 0;
      if (!ok) atomicOr(&ctrl->numeric, 1);
    }
  }
  __syncthreads();
  if (!ok_s) return;
  write_p<T>(Csrc, Gi, rn, R, inner, static_cast<T*>(a.P[n]));
}

template <typename T>
__global__ void __launch_bounds__(256) k_ffinish(FFinishArgs a, CtrlState* ctrl) {
  ffinish_body<T>(a, a.stage, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- QR + fold
// Block n: Cholesky QR of U_n in the W inner product (one round: the Heun update leaves
// U_n W-orthonormal to O(dt^2), so a single round already reaches roundoff; a second
// round can be requested): the Gram matrix
// U^T W U from row-split partial sums (one quarter of the rows per wave, combined in
// a fixed order), its Cholesky factor R^T R and R^-1 by one wave, then U <- U R^-1
// row by row; R accumulates over the rounds. The last block to finish folds every
// R_n into the core (C <- C x_n R_n), so the reconstruction is unchanged.
__device__ __forceinline__ void fqr_body(const FQrArgs& a, CtrlState* ctrl, int bx, int gx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int last, skip_s, ok_s;
  // every block takes part in the completion count, even when there is nothing to do;
  // the flag is read once per block so that the whole block takes the same branch
  if (threadIdx.x == 0)
    skip_s = __hip_atomic_load(&ctrl->numeric, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  const bool skip = skip_s != 0;
  const int n = bx;
  const int rn = a.r[n], ld = a.ldU[n];
  const int Nn = (int)a.N[n];
  const int rq = a.rmax;
  const int np = rn * (rn + 1) / 2;
  const int npq = rq * (rq + 1) / 2;
  double* L = lds;                          // rq*rq
  double* Li = L + rq * rq;                 // rq*rq
  double* Rt = Li + rq * rq;                // rq*rq
  double* Tm = Rt + rq * rq;                // rq*rq
  double* Gp = Tm + rq * rq;                // 4*npq partial Grams
  double* wl = Gp + 4 * npq;                // Nn weights
  double* Ul = wl + TDB_NEIG;               // Nn*rn when staged (or the core for the fold)
  double* U = a.U0[n];
  const bool stage = a.u_in_lds[n] && !skip;
  if (!skip) {
    for (int t = threadIdx.x; t < Nn; t += blockDim.x) wl[t] = a.w[n][t];
    if (stage)
      for (int base = 0; base < Nn * rn; base += 8 * blockDim.x) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = base + u * blockDim.x + threadIdx.x;
          v[u] = 0.0;
          if (t < Nn * rn) { const int i = t / rn; v[u] = U[i * ld + (t - i * rn)]; }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = base + u * blockDim.x + threadIdx.x;
          if (t < Nn * rn) Ul[t] = v[u];
        }
      }
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) Rt[t] = (t / rn == t % rn) ? 1.0 : 0.0;
  }
  __syncthreads();
  double* Uw = stage ? Ul : U;
  const int ldw = stage ? rn : ld;
  bool ok = !skip;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int round = 0; round < a.rounds && ok; ++round) {
    // partial Grams: wave `wid` sums rows [q0, q1)
    const int per = (Nn + 3) / 4;
    const int q0 = wid * per, q1 = min(Nn, q0 + per);
    for (int pp = lane; pp < np; pp += 64) {
      int i = (int)((sqrt(8.0 * pp + 1.0) - 1.0) * 0.5);
      while ((i + 1) * (i + 2) / 2 <= pp) ++i;
      while (i * (i + 1) / 2 > pp) --i;
      const int j = pp - i * (i + 1) / 2;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int q = q0;
      for (; q + 4 <= q1; q += 4) {
        s0 += wl[q] * Uw[q * ldw + i] * Uw[q * ldw + j];
        s1 += wl[q + 1] * Uw[(q + 1) * ldw + i] * Uw[(q + 1) * ldw + j];
        s2 += wl[q + 2] * Uw[(q + 2) * ldw + i] * Uw[(q + 2) * ldw + j];
        s3 += wl[q + 3] * Uw[(q + 3) * ldw + i] * Uw[(q + 3) * ldw + j];
      }
      for (; q < q1; ++q) s0 += wl[q] * Uw[q * ldw + i] * Uw[q * ldw + j];
      Gp[wid * npq + pp] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int pp = threadIdx.x; pp < np; pp += blockDim.x) {
      int i = (int)((sqrt(8.0 * pp + 1.0) - 1.0) * 0.5);
      while ((i + 1) * (i + 2) / 2 <= pp) ++i;
      while (i * (i + 1) / 2 > pp) --i;
      const int j = pp - i * (i + 1) / 2;
      const double g = (Gp[pp] + Gp[npq + pp]) + (Gp[2 * npq + pp] + Gp[3 * npq + pp]);
      L[i * rn + j] = g;
      L[j * rn + i] = g;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const bool okw = wave_chol(L, rn);
      if (okw) wave_tri_inv(L, Li, rn);
      if (threadIdx.x == 0) ok_s = okw ? 1 : 0;
    }
    __syncthreads();
    ok = ok_s != 0;
    if (!ok) break;
    // U <- U R^-1 with R = L^T: x_j = sum_{k<=j} u_k Li[j][k], in place from the last column
    for (int q = threadIdx.x; q < Nn; q += blockDim.x) {
      double* rowp = Uw + q * ldw;
      for (int j = rn - 1; j >= 0; --j) {
        double s = 0.0;
        const double* lj = Li + j * rn;
        for (int k = 0; k <= j; ++k) s += rowp[k] * lj[k];
        rowp[j] = s;
      }
    }
    // Rt <- L^T Rt
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) {
      const int i = t / rn, j = t - (t / rn) * rn;
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
    if (stage)
      for (int t = threadIdx.x; t < Nn * rn; t += blockDim.x) {
        const int i = t / rn;
        U[i * ld + (t - i * rn)] = Ul[t];
      }
    for (int t = threadIdx.x; t < rn * rn; t += blockDim.x) a.Rq[n][t] = Rt[t];
  }
  // last block folds the factors into the core
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == gx - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) *a.counter = 0u;
  if (__hip_atomic_load(&ctrl->numeric, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) return;
  int csz = 1;
  for (int k = 0; k < 3; ++k) csz *= a.r[k];
  // core in LDS (two buffers) when it fits, else ping-pong through global memory
  double* ca = a.core_in_lds ? Ul : a.C0;
  double* cb = a.core_in_lds ? Ul + csz : a.Ctmp;
  if (a.core_in_lds) {
    for (int t = threadIdx.x; t < csz; t += blockDim.x)
      ca[t] = __hip_atomic_load(&a.C0[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (int m = 0; m < 3; ++m) {
    const int rm = a.r[m];
    for (int t = threadIdx.x; t < rm * rm; t += blockDim.x)
      Rt[t] = __hip_atomic_load(&a.Rq[m][t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int inner = 1;
    for (int k = m + 1; k < 3; ++k) inner *= a.r[k];
    for (int t = threadIdx.x; t < csz; t += blockDim.x) {
      const int in = t % inner, rest = t / inner;
      const int ai = rest % rm;
      const int o = rest / rm;
      double s = 0.0;
      for (int b = ai; b < rm; ++b) s += Rt[ai * rm + b] * ca[(o * rm + b) * inner + in];
      cb[t] = s;
    }
    __syncthreads();
    double* tswap = ca; ca = cb; cb = tswap;
  }
  for (int t = threadIdx.x; t < csz; t += blockDim.x) a.C0[t] = ca[t];
  // T3 = C x_3 U_3 of the folded core, for the error-pass expansion
  if (a.T3) {
    const int r12 = a.r[0] * a.r[1], r3 = a.r[2], N3 = (int)a.N[2], ld3 = a.ldU[2];
    for (int t = threadIdx.x; t < r12 * N3; t += blockDim.x) {
      const int ab = t / N3, i3 = t - (t / N3) * N3;
      double s = 0.0;
      for (int c = 0; c < r3; ++c)
        s += ca[ab * r3 + c] * __hip_atomic_load(&a.U0[2][i3 * ld3 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a.T3[t] = s;
    }
  }
}

__global__ void __launch_bounds__(256) k_fqr(FQrArgs a, CtrlState* ctrl) {
  fqr_body(a, ctrl, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- post-step
// Blocks [0, 3): for mode n at the new state: core singular values (Jacobi, into the
// controller), pseudo-inverse P_n and weighted basis B_n for the next stage 1.
// Blocks [3, 3 + eblocks): the partial expansion E = C x_2 U_2 x_3 U_3 used by the
// error pass, and the mode-1 basis in the compute type.
template <typename T>
__device__ __forceinline__ void fpost_body(const FPostArgs& a, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int pairs[TDB_RCAP + 2];
  __shared__ int order[TDB_RCAP];
  if ((int)bx >= 3) {
    // E[a][i2][i3] = sum_b U2[i2][b] T3[a][b][i3],  T3[a][b][i3] = sum_c C[a][b][c] U3[i3][c]
    const int eb = bx - 3;
    const int r1 = a.r[0], r2 = a.r[1], r3 = a.r[2];
    const long long N2 = a.N[1], N3 = a.N[2];
    double* T3 = lds;                                   // r1*r2*N3
    double* U2l = T3 + (long long)r1 * r2 * N3;         // rows of U2 of this block
    const long long per = (N2 + a.eblocks - 1) / a.eblocks;
    const long long i2a = (long long)eb * per, i2b = min(N2, i2a + per);
    if (i2a < i2b) {
      if (a.T3) {
        for (long long t = threadIdx.x; t < (long long)r1 * r2 * N3; t += blockDim.x) T3[t] = a.T3[t];
      } else {
        for (long long t = threadIdx.x; t < (long long)r1 * r2 * N3; t += blockDim.x) {
          const long long i3 = t % N3, ab = t / N3;
          const double* cr = a.C + ab * r3;
          const double* u3 = a.U[2] + i3 * a.ldU[2];
          double s = 0.0;
          for (int c = 0; c < r3; ++c) s += cr[c] * u3[c];
          T3[t] = s;
        }
      }
      for (long long t = threadIdx.x; t < (i2b - i2a) * r2; t += blockDim.x) {
        const long long i = t / r2;
        U2l[t] = a.U[1][(i2a + i) * a.ldU[1] + (t - i * r2)];
      }
      __syncthreads();
      T* E = static_cast<T*>(a.E);
      const long long nrow = i2b - i2a;
      for (long long t = threadIdx.x; t < (long long)r1 * nrow * N3; t += blockDim.x) {
        const long long i3 = t % N3, q = t / N3;
        const long long il = q % nrow;
        const int ai = (int)(q / nrow);
        const double* u2 = U2l + il * r2;
        const double* t3 = T3 + (long long)ai * r2 * N3 + i3;
        double s = 0.0;
        for (int b = 0; b < r2; ++b) s += u2[b] * t3[(long long)b * N3];
        E[((long long)ai * N2 + i2a + il) * N3 + i3] = (T)s;
      }
    }
    const long long tu = a.N[0] * r1;
    T* U1c = static_cast<T*>(a.U1c);
    for (long long t = (long long)eb * blockDim.x + threadIdx.x; t < tu; t += (long long)a.eblocks * blockDim.x) {
      const long long i = t / r1;
      U1c[t] = (T)a.U[0][i * a.ldU[0] + (t - i * r1)];
    }
    return;
  }
  const int n = bx;
  const int rn = a.r[n];
  long long inner = 1, R = 1, csz = 1;
  for (int k = 0; k < 3; ++k) {
    csz *= a.r[k];
    if (k != n) R *= a.r[k];
    if (k > n) inner *= a.r[k];
  }
  // weighted basis of the next stage 1
  {
    T* B = static_cast<T*>(a.B[n]);
    const int Nn = (int)a.N[n], ld = a.ldU[n];
    const double* U = a.U[n];
    const double* w = a.w[n];
    for (int i = threadIdx.x / 4; i < Nn; i += blockDim.x / 4) {
      const double wi = w[i];
      for (int j = threadIdx.x & 3; j < rn; j += 4) B[i * rn + j] = (T)(wi * U[i * ld + j]);
    }
  }
  const int rq = a.rmax;
  double* G = lds;
  double* Li = G + rq * rq;
  double* Gi = Li + rq * rq;
  double* ws = Gi + rq * rq;                 // 4*rq
  double* lam = ws + 4 * rq;                 // rq
  double* Cl = lam + rq;
  __shared__ int ok_s;
  const double* Csrc = a.C;
  if (a.core_in_lds) {
    for (int t = threadIdx.x; t < (int)csz; t += blockDim.x) Cl[t] = Csrc[t];
    __syncthreads();
    Csrc = Cl;
  }
  gram_from(Csrc, rn, R, inner, G);
  const bool need_p = rn < a.N[n] && a.want_pinv;
  if (threadIdx.x < 64) {
    if (a.G[n])
      for (int t = threadIdx.x; t < rn * rn; t += 64) a.G[n][t] = G[t];
    if (a.want_sigma) {
      // singular values of C_(n): eigenvalues of a copy of the Gram matrix
      for (int t = threadIdx.x; t < rn * rn; t += 64) Gi[t] = G[t];
      wave_fence();
      wave_eigvals(Gi, rn, lam, ws);
      for (int i = threadIdx.x; i < TDB_RCAP; i += 64)
        ctrl->sigma[n][i] = i < rn ? sqrt(fmax(lam[i], 0.0)) : 0.0;
    }
    bool ok = true;
    if (need_p) {
      ok = wave_chol(G, rn);
      if (ok) {
        wave_tri_inv(G, Li, rn);
        wave_inv_from_linv(Li, Gi, rn);
      }
    }
    if (threadIdx.x == 0) {
      ok_s = ok ? 1 : 0;
      if (!ok) atomicOr(&ctrl->numeric, 4);
    }
  }
  __syncthreads();
  if (!need_p || !ok_s) return;
  write_p<T>(Csrc, Gi, rn, R, inner, static_cast<T*>(a.P[n]));
}

template <typename T>
__global__ void __launch_bounds__(256) k_fpost(FPostArgs a, CtrlState* ctrl) {
  fpost_body<T>(a, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- error pass
// Tile = T1 slabs of mode 1. rec[i1][j] = sum_a U1[i1][a] E[a][j] (j over modes 2,3);
// partial sums of w (V - rec)^2 and w V^2 in FP64; the last block reduces them and
// runs the controller decision.
template <typename TD, typename T>
__device__ __forceinline__ void ferr_body(const FErrArgs& a, int bx, int by, int gx) {
  __shared__ double red[16];
  __shared__ double U1s[FERR_T1 * TDB_RCAP];
  if (a.skip && *a.skip) {
    // the learned gate skips this step's pass
    if (threadIdx.x == 0) {
      const int b0 = by * gx + bx;
      a.part[2 * b0] = 0.0;
      a.part[2 * b0 + 1] = 0.0;
    }
    return;
  }
  const long long M = a.M;      // N2*N3
  const int r1 = a.r1;
  const int i1_0 = by * a.T1;
  const int n1 = min(a.T1, a.N1 - i1_0);
  const T* E = static_cast<const T*>(a.E);
  for (int t = threadIdx.x; t < FERR_T1 * r1; t += blockDim.x) {
    const int q = t / r1;
    U1s[t] = q < n1 ? (double)static_cast<const T*>(a.U1c)[(long long)(i1_0 + q) * r1 + (t - q * r1)] : 0.0;
  }
  __syncthreads();
  double se = 0.0, sv = 0.0;
  for (long long j = (long long)bx * blockDim.x + threadIdx.x; j < M; j += (long long)gx * blockDim.x) {
    T acc[FERR_T1];
    for (int q = 0; q < FERR_T1; ++q) acc[q] = (T)0;
    for (int ai = 0; ai < r1; ++ai) {
      const T e = E[(long long)ai * M + j];
      for (int q = 0; q < FERR_T1; ++q)
        acc[q] += (T)U1s[q * r1 + ai] * e;
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
  const int bid = by * gx + bx;
  if (threadIdx.x == 0) {
    a.part[2 * bid] = se;
    a.part[2 * bid + 1] = sv;
  }
}

template <typename TD, typename T>
__global__ void __launch_bounds__(256) k_ferr(FErrArgs a, CtrlState* ctrl) {
  ferr_body<TD, T>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

// Controller of the fused path: the decision up to the removal test; only when that
// test has to run are the singular values of the core unfoldings formed, one wave per
// mode, from the Grams kept by the post-step kernel.
__device__ __forceinline__ void fused_decide(CtrlState* ctrl, const double* const* G, int rmax, const int* skip,
                                             const int* would_skip, const float* yhat) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int need;
  if (threadIdx.x == 0) {
    ctrl->gated = (skip && *skip) ? 1 : 0;
    ctrl->would_skip = would_skip ? *would_skip : 0;
    ctrl->eps_pred = (yhat && isfinite(*yhat)) ? pow(10.0, (double)*yhat) : __builtin_nan("");
    if (ctrl->gated) {
      // no exact error this step: no decision, and the slope window starts over so that
      // a removal always rests on consecutive exact errors
      ctrl->eps = __builtin_nan("");
      ctrl->event = 0;
      ctrl->eps_after = __builtin_nan("");
      ctrl->rank_changed = 0;
      ctrl->decision = DEC_NONE;
      ctrl->wcount = 0;
      need = 0;
    } else {
      need = controller_pre(ctrl) ? 1 : 0;
    }
  }
  __syncthreads();
  if (!need) return;
  const int w = threadIdx.x >> 6;
  if (w < 3 && G[w]) {
    const int rn = ctrl->ranks[w];
    double* A = lds + w * (rmax * rmax + 5 * rmax);
    double* lam = A + rmax * rmax;
    double* ws = lam + rmax;
    for (int t = threadIdx.x & 63; t < rn * rn; t += 64) A[t] = G[w][t];
    wave_fence();
    wave_eigvals(A, rn, lam, ws);
    for (int i = threadIdx.x & 63; i < TDB_RCAP; i += 64)
      ctrl->sigma[w][i] = i < rn ? sqrt(fmax(lam[i], 0.0)) : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) controller_remove(ctrl);
}

// One block: fixed-order sum of the error-pass partials, then the controller.
__global__ void __launch_bounds__(256) k_ferr_final(FErrArgs a, CtrlState* ctrl) {
  __shared__ double red[16];
  const int nb = a.gx * a.gy;
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += a.part[2 * i];
    s1 += a.part[2 * i + 1];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0 && !(a.skip && *a.skip)) {
    ctrl->eps2 = s0;
    ctrl->nu2 = s1;
  }
  __syncthreads();
  fused_decide(ctrl, a.G, a.rmax, a.skip, a.would_skip, a.yhat);
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_freduce(const FReduceArgs& a, CtrlState* c, hipStream_t s) {
  long long blocks = (freduce_items(a) + 255) / 256;
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

template <typename T>
hipError_t launch_fmprep(const FFinishArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fmprep<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fmprep<T>, dim3(3), dim3(256), lds, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_fmprep<float>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);
template hipError_t launch_fmprep<double>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);

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
hipError_t launch_ferr(const FErrArgs& a, CtrlState* c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipExtLaunchKernelGGL((k_ferr<TD, T>), dim3(a.gx, a.gy), dim3(256), 0u, s, ev0, ev1, 0u, a, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t fl = ferr_final_lds(a.rmax);
  e = hipFuncSetAttribute((const void*)k_ferr_final, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fl);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ferr_final, dim3(1), dim3(256), fl, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_ferr<float, float>(const FErrArgs&, CtrlState*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_ferr<float, double>(const FErrArgs&, CtrlState*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_ferr<double, double>(const FErrArgs&, CtrlState*, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_ferr<double, float>(const FErrArgs&, CtrlState*, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------- batched forms
template <typename T>
__global__ void __launch_bounds__(256) kb_freduce(const FReduceArgs* __restrict__ tab, CtrlState* const* ctab,
                                                  BatchMap m, int stage) {
  const int s = m.sid[blockIdx.x];
  const int b0 = m.start[s];
  freduce_body<T>(tab[s], stage, ctab[s], blockIdx.x - b0, m.start[s + 1] - b0);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_ffinish(const FFinishArgs* __restrict__ tab, CtrlState* const* ctab,
                                                  BatchMap m, int stage) {
  const int s = m.sid[blockIdx.x];
  ffinish_body<T>(tab[s], stage, ctab[s], blockIdx.x - m.start[s]);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_fmprep(const FFinishArgs* __restrict__ tab, CtrlState* const* ctab,
                                                 BatchMap m, int stage) {
  const int s = m.sid[blockIdx.x];
  fmprep_body<T>(tab[s], stage, ctab[s], blockIdx.x - m.start[s]);
}

__global__ void __launch_bounds__(256) kb_fqr(const FQrArgs* __restrict__ tab, CtrlState* const* ctab, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  const int b0 = m.start[s];
  fqr_body(tab[s], ctab[s], blockIdx.x - b0, m.start[s + 1] - b0);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_fpost(const FPostArgs* __restrict__ tab, CtrlState* const* ctab,
                                                BatchMap m) {
  const int s = m.sid[blockIdx.x];
  fpost_body<T>(tab[s], ctab[s], blockIdx.x - m.start[s]);
}

template <typename TD, typename T>
__global__ void __launch_bounds__(256) kb_ferr(const FErrArgs* __restrict__ tab, const void* const* v1, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  FErrArgs a = tab[s];
  a.V = v1[s];
  const int l = blockIdx.x - m.start[s];
  ferr_body<TD, T>(a, l % a.gx, l / a.gx, a.gx);
}

// One block per stream: the fixed-order sum of that stream's error-pass partials,
// its controller decision, and the summary the host reads.
__global__ void __launch_bounds__(256) kb_ferr_final(const FErrArgs* __restrict__ tab, CtrlState* const* ctab,
                                                     BatchSummary* out) {
  __shared__ double red[16];
  const int s = blockIdx.x;
  const double* part = tab[s].part;
  const int nb = tab[s].gx * tab[s].gy;
  CtrlState* ctrl = ctab[s];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0 && !(tab[s].skip && *tab[s].skip)) {
    ctrl->eps2 = s0;
    ctrl->nu2 = s1;
  }
  __syncthreads();
  fused_decide(ctrl, tab[s].G, tab[s].rmax, tab[s].skip, tab[s].would_skip, tab[s].yhat);
  if (threadIdx.x == 0) {
    BatchSummary q;
    q.decision = ctrl->decision;
    q.event = ctrl->event;
    q.numeric = ctrl->numeric;
    q.gated = ctrl->gated;
    for (int k = 0; k < 5; ++k) q.n_events[k] = ctrl->n_events[k];
    q.would_skip = ctrl->would_skip;
    q.eps = ctrl->eps;
    q.nu = ctrl->nu;
    q.eps2 = ctrl->eps2;
    q.nu2 = ctrl->nu2;
    q.eps_pred = ctrl->eps_pred;
    out[s] = q;
  }
}

template <typename T>
hipError_t launch_batch_freduce(const FReduceArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                                hipStream_t s) {
  hipLaunchKernelGGL(kb_freduce<T>, dim3(blocks), dim3(256), 0, s, tab, ctab, m, stage);
  return hipGetLastError();
}
template hipError_t launch_batch_freduce<float>(const FReduceArgs*, CtrlState* const*, BatchMap, int, int, hipStream_t);
template hipError_t launch_batch_freduce<double>(const FReduceArgs*, CtrlState* const*, BatchMap, int, int, hipStream_t);

template <typename T>
hipError_t launch_batch_ffinish(const FFinishArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                                size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_ffinish<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_ffinish<T>, dim3(blocks), dim3(256), lds, s, tab, ctab, m, stage);
  return hipGetLastError();
}
template hipError_t launch_batch_ffinish<float>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                                hipStream_t);
template hipError_t launch_batch_ffinish<double>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                                 hipStream_t);

template <typename T>
hipError_t launch_batch_fmprep(const FFinishArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                               size_t lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_fmprep<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_fmprep<T>, dim3(blocks), dim3(256), lds, s, tab, ctab, m, stage);
  return hipGetLastError();
}
template hipError_t launch_batch_fmprep<float>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                               hipStream_t);
template hipError_t launch_batch_fmprep<double>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                                hipStream_t);

hipError_t launch_batch_fqr(const FQrArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, size_t lds,
                            hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_fqr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_fqr, dim3(blocks), dim3(256), lds, s, tab, ctab, m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_fpost(const FPostArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, size_t lds,
                              hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_fpost<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_fpost<T>, dim3(blocks), dim3(256), lds, s, tab, ctab, m);
  return hipGetLastError();
}
template hipError_t launch_batch_fpost<float>(const FPostArgs*, CtrlState* const*, BatchMap, int, size_t, hipStream_t);
template hipError_t launch_batch_fpost<double>(const FPostArgs*, CtrlState* const*, BatchMap, int, size_t, hipStream_t);

template <typename TD, typename T>
hipError_t launch_batch_ferr(const FErrArgs* tab, const void* const* v1, BatchMap m, int blocks, int nstreams,
                             CtrlState* const* ctab, BatchSummary* out, size_t lds_final, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1) {
  hipExtLaunchKernelGGL((kb_ferr<TD, T>), dim3(blocks), dim3(256), 0u, s, ev0, ev1, 0u, tab, v1, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)kb_ferr_final, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_final);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_ferr_final, dim3(nstreams), dim3(256), lds_final, s, tab, ctab, out);
  return hipGetLastError();
}
template hipError_t launch_batch_ferr<float, float>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<float, double>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<double, double>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<double, float>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, size_t, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace tdb
