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
  __shared__ double dmax_l;
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < rn; ++i) mx = fmax(mx, fabs(A[i * rn + i]));
    dmax_l = mx;
  }
  __syncthreads();
  const double tol = TDB_JACOBI_TOL * dmax_l;
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
          if (fabs(apq) > 1e-300 && fabs(apq) > tol) {
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

// Eigenvalues of a symmetric rn x rn LDS matrix (rn <= 64) by cyclic Jacobi run by one
// wave (lanes 0..63 of the calling block, all of which must call it): round-robin
// pairing, rotations computed by one lane per pair, row and column updates spread
// over the lanes. Only wave-level ordering is needed, so no block barriers.
static __device__ void jacobi_wave(double* A, int rn, int* pairs) {
  __shared__ double cs_w[TDB_RCAP], sn_w[TDB_RCAP];
  __shared__ int rot_w;
  const int lane = threadIdx.x & 63;
  const int m = rn + (rn & 1);
  double mx = 0.0;
  for (int i = lane; i < rn; i += 64) mx = fmax(mx, fabs(A[i * rn + i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const double tol = TDB_JACOBI_TOL * mx;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (lane == 0) rot_w = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (int round = 0; round < m - 1; ++round) {
      for (int k = lane; k < m / 2; k += 64) {
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
          if (fabs(apq) > 1e-300 && fabs(apq) > tol) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
            rot_w = 1;
          }
        }
        cs_w[k] = c;
        sn_w[k] = s;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      for (int t = lane; t < (m / 2) * rn; t += 64) {
        const int k = t / rn, col = t % rn;
        const int p_ = pairs[2 * k], q_ = pairs[2 * k + 1];
        if (q_ >= rn || sn_w[k] == 0.0) continue;
        const double ap = A[p_ * rn + col], aq = A[q_ * rn + col];
        A[p_ * rn + col] = cs_w[k] * ap - sn_w[k] * aq;
        A[q_ * rn + col] = sn_w[k] * ap + cs_w[k] * aq;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      for (int t = lane; t < (m / 2) * rn; t += 64) {
        const int k = t / rn, row = t % rn;
        const int p_ = pairs[2 * k], q_ = pairs[2 * k + 1];
        if (q_ >= rn || sn_w[k] == 0.0) continue;
        const double ap = A[row * rn + p_], aq = A[row * rn + q_];
        A[row * rn + p_] = cs_w[k] * ap - sn_w[k] * aq;
        A[row * rn + q_] = sn_w[k] * ap + cs_w[k] * aq;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    if (!rot_w) break;
  }
}

// ---------------------------------------------------------------- controller
// Single thread (called by one thread): reads eps^2, nu^2 of the error pass and decides the step's event
// (Sec. 2.5): an add when eps exceeds the trigger, a removal check when the error
// slope over the window is negative with headroom and some mode's weakest direction
// fits in the budget, a restart on a numerical event.
// First part of the decision: error and norm, numerical events, additions, the slope
// window. Returns true when the removal test has to run, which needs the singular
// values of the core unfoldings (c->sigma).
static __device__ bool controller_pre(CtrlState* c) {
  c->eps = sqrt_sum_sq(c->eps2);
  c->nu = sqrt_sum_sq(c->nu2);
  c->event = 0;
  c->eps_after = __builtin_nan("");
  c->rank_changed = 0;
  // a numerical event (the state was kept) comes before an error that is not finite
  // only because of it; non-finite data come first
  if (!(c->numeric & NUM_NONFINITE) && (c->numeric & (NUM_CORE | NUM_BASIS))) {
    c->decision = DEC_NUMERIC;
    return false;
  }
  if ((c->numeric & NUM_NONFINITE) || !isfinite(c->eps2) || !isfinite(c->nu2)) {
    // non-finite data: the step was not applied; the flags its stages raised on the
    // non-finite values go with it (a failure of the next step's core Gram, found on
    // the kept state, stays for that step)
    c->numeric &= NUM_NEXT;
    c->eps = __builtin_nan("");
    c->decision = DEC_NONFINITE;
    return false;
  }
  if (!c->adaptive) { c->decision = DEC_NONE; return false; }
  const double eps = c->eps;
  if (eps > c->eps_trig) { c->decision = DEC_ADD; return false; }
  const int nw = c->slope_window;
  c->window[c->whead] = eps;
  c->whead = (c->whead + 1) % TDB_WIN;
  c->wcount += 1;
  c->decision = DEC_NONE;
  if (c->wcount < nw) return false;
  const double last = c->window[(c->whead - 1 + TDB_WIN) % TDB_WIN];
  const double first = c->window[(c->whead - nw + TDB_WIN) % TDB_WIN];
  const double slope = (last - first) / ((nw - 1) * c->dt);
  if (!(slope < 0.0)) return false;
  if (eps > 0.5 * c->eps_th) return false;
  return true;
}

// Removal test (after controller_pre returned true): drop a direction if the error
// stays within budget without it.
static __device__ void controller_remove(CtrlState* c) {
  const double eps = c->eps;
  const double B = c->gamma_th > 0.0 ? (1.0 - c->gamma_th / 100.0) * c->nu2 : 0.25 * c->eps_th * c->eps_th;
  for (int n = 0; n < c->p; ++n) {
    const double s = c->sigma[n][c->ranks[n] - 1];
    if (eps * eps + s * s <= B) { c->decision = DEC_REMOVE; return; }
  }
}

// The whole decision, with c->sigma already current.
static __device__ void controller_decide(CtrlState* c) {
  if (controller_pre(c)) controller_remove(c);
}


}  // namespace tdb

namespace tdb {

// floor(t / d) for 0 <= t < 2^22 and d >= 1, given inv = 1.0f / d: the float quotient
// is within one of the exact one (relative error below 2^-23), and the remainder
// corrects it.
__device__ __forceinline__ int small_div(int t, int d, float inv) {
  int q = (int)((float)t * inv);
  const int r = t - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// ===================================================================== block copies
// Copy n values from global memory into LDS (converted to the LDS type), with up to 16
// loads in flight per thread before any is stored, so that a short copy costs one
// memory round trip rather than one per loop iteration.
template <typename TS, typename TL>
__device__ __forceinline__ void g2l(TL* dst, const TS* src, int n) {
  for (int base = 0; base < n; base += 16 * (int)blockDim.x) {
    TS v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      v[u] = t < n ? src[t] : (TS)0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (t < n) dst[t] = (TL)v[u];
    }
  }
}

// Up to five such copies in one pass (one round trip for all of them); a segment with
// n = 0 is skipped.
__device__ __forceinline__ void g2l5(double* d0, const double* s0, int n0, double* d1, const double* s1, int n1,
                                     double* d2, const double* s2, int n2, double* d3, const double* s3, int n3,
                                     double* d4, const double* s4, int n4) {
  const int e0 = n0, e1 = e0 + n1, e2 = e1 + n2, e3 = e2 + n3, e4 = e3 + n4;
  for (int base = 0; base < e4; base += 16 * (int)blockDim.x) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      double x = 0.0;
      if (t < e0) x = s0[t];
      else if (t < e1) x = s1[t - e0];
      else if (t < e2) x = s2[t - e1];
      else if (t < e3) x = s3[t - e2];
      else if (t < e4) x = s4[t - e3];
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (t < e0) d0[t] = v[u];
      else if (t < e1) d1[t - e0] = v[u];
      else if (t < e2) d2[t - e1] = v[u];
      else if (t < e3) d3[t - e2] = v[u];
      else if (t < e4) d4[t - e3] = v[u];
    }
  }
}

// ===================================================================== one-wave kernels
// The routines below are run by one full wave (64 lanes) of the calling block on small
// (rn <= 64) row-major matrices in LDS. Lanes own rows or columns; ordering between
// lanes only needs wave-level memory ordering, so no block barriers are used.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// In-place lower Cholesky factor of the SPD matrix A (lane i owns row i). Returns false
// if a pivot is not positive or is below TDB_PIVOT_FLOOR times the largest diagonal.
static __device__ bool wave_chol(double* A, int rn) {
  const int i = threadIdx.x & 63;
  const double dmax = wave_max_d(i < rn ? A[i * rn + i] : 0.0);
  bool bad = false;
  for (int k = 0; k < rn; ++k) {
    const double piv = A[k * rn + k];
    bad = bad || !(piv > TDB_PIVOT_FLOOR * dmax) || !(piv > 0.0);
    const double lkk = sqrt(fmax(piv, 1e-300));
    wave_fence();
    if (i == k) A[k * rn + k] = lkk;
    if (i > k && i < rn) A[i * rn + k] /= lkk;
    wave_fence();
    if (i > k && i < rn) {
      const double lik = A[i * rn + k];
      double* ai = A + i * rn;
#pragma unroll 4
      for (int j = k + 1; j <= i; ++j) ai[j] -= lik * A[j * rn + k];
    }
    wave_fence();
  }
  if (i < rn)
    for (int j = i + 1; j < rn; ++j) A[i * rn + j] = 0.0;
  wave_fence();
  return !bad;
}

// Li = L^-1 for a lower-triangular L (lane j computes column j).
static __device__ void wave_tri_inv(const double* L, double* Li, int rn) {
  const int j = threadIdx.x & 63;
  if (j < rn) {
    for (int i = 0; i < j; ++i) Li[i * rn + j] = 0.0;
    Li[j * rn + j] = 1.0 / L[j * rn + j];
    for (int i = j + 1; i < rn; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * rn + k] * Li[k * rn + j];
      Li[i * rn + j] = -s / L[i * rn + i];
    }
  }
  wave_fence();
}

// L^-1 of the lower-triangular L (rn x rn, row-major in LDS) by one wave, lane j
// forming column j by forward substitution in registers; the entries of L are read
// from LDS at addresses common to all lanes, and rdiag holds 1 / L[i][i].
template <int RB>
__device__ __forceinline__ void wave_tri_inv_reg(const double* L, double* Li, int rn, const double* rdiag) {
  const int j = threadIdx.x & 63;
  double y[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    double s = (i == j) ? 1.0 : 0.0;
    if (i < rn) {
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i * rn + k] * y[k];
      s *= rdiag[i];
    }
    y[i] = s;
  }
  if (j < rn)
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if (i < rn) Li[i * rn + j] = y[i];
  wave_fence();
}

// L^-1 by one wave (rdiag: LDS scratch of rn doubles).
__device__ __forceinline__ void wave_tri_inv_fast(const double* L, double* Li, int rn, double* rdiag) {
  const int l = threadIdx.x & 63;
  for (int i = l; i < rn; i += 64) rdiag[i] = 1.0 / L[i * rn + i];
  wave_fence();
  if (rn <= 16) wave_tri_inv_reg<16>(L, Li, rn, rdiag);
  else if (rn <= 32) wave_tri_inv_reg<32>(L, Li, rn, rdiag);
  else wave_tri_inv(L, Li, rn);
}

// Gi = Li^T Li (the inverse of L L^T), lanes over entries.
static __device__ void wave_inv_from_linv(const double* Li, double* Gi, int rn) {
  const int lane = threadIdx.x & 63;
  for (int t = lane; t < rn * rn; t += 64) {
    const int i = t / rn, j = t - (t / rn) * rn;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < rn; ++k) s += Li[k * rn + i] * Li[k * rn + j];
    Gi[t] = s;
  }
  wave_fence();
}

// ------------------------------------------------ register-resident forms (rn <= 32)
// The same factorizations with the working rows or columns in registers: lane i keeps
// row i (or column i) in a fixed-size array indexed only by compile-time constants.
// Entries another lane owns are read with v_readlane during the factorization, and from
// LDS at wave-uniform addresses afterwards, so no step waits on a store-to-load chain
// through LDS. The whole wave must execute these (no lane may be masked off around the
// broadcasts). The arithmetic and its order are those of the LDS routines above.

// Value of v held by lane `src` (uniform), as a wave-uniform double.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// 1/sqrt(x) for x > 0 to full FP64 accuracy: the hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}

// The factorization runs over all RB indices without branches: rows and columns from
// rn to RB are those of the identity, which leaves the leading rn x rn block exactly
// as it would be alone. Entries above the diagonal are not read while factoring and
// are cleared at the end.
template <int RB>
__device__ __forceinline__ bool wave_chol_inv_rb(double* A, int rn, double* Li, double* Gi) {
  const int l = threadIdx.x & 63;
  double a[RB];
  double rdl = 0.0;                              // lane k: 1 / L[k][k]
#pragma unroll
  for (int j = 0; j < RB; ++j) a[j] = (l < rn && j < rn) ? A[l * rn + j] : (l == j ? 1.0 : 0.0);
  double dmax = 0.0;
#pragma unroll
  for (int k = 0; k < RB; ++k) dmax = fmax(dmax, k < rn ? lane_bcast(a[k], k) : 0.0);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const double piv = lane_bcast(a[k], k);
    bad = bad || (k < rn && (!(piv > TDB_PIVOT_FLOOR * dmax) || !(piv > 0.0)));
    const double pv = fmax(piv, 1e-300);
    const double r = rsqrt_nr(pv);
    rdl = (l == k) ? r : rdl;
    a[k] = (l == k) ? pv * r : a[k] * r;        // column k of L (lanes above k: unused)
#pragma unroll
    for (int j = k + 1; j < RB; ++j) a[j] -= a[k] * lane_bcast(a[k], j);
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) a[j] = (j > l) ? 0.0 : a[j];
  if (l < rn)
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < rn) A[l * rn + j] = a[j];
  if (!bad && Li) {
    // lane l: column l of L^-1 by forward substitution, column-oriented so that the
    // chain from one entry to the next is a single update; L[m][i] is lane m's a[i]
    double x[RB];
#pragma unroll
    for (int m = 0; m < RB; ++m) x[m] = (l == m) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      x[i] *= lane_bcast(rdl, i);
#pragma unroll
      for (int m = i + 1; m < RB; ++m) x[m] -= lane_bcast(a[i], m) * x[i];
    }
    if (l < rn)
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (i < rn) Li[i * rn + l] = x[i];
    if (Gi) {
      // lane l: column l of Li^T Li, Li[k][i] broadcast from lane i
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        double g = 0.0;
#pragma unroll
        for (int k = i; k < RB; ++k) g += lane_bcast(x[k], i) * x[k];
        if (l < rn && i < rn) Gi[i * rn + l] = g;
      }
    }
  }
  wave_fence();
  return !bad;
}

__device__ __attribute__((noinline)) bool wave_chol_inv_lds(double* A, int rn, double* Li, double* Gi) {
  const bool ok = wave_chol(A, rn);
  if (ok && Li) {
    wave_tri_inv(A, Li, rn);
    if (Gi) wave_inv_from_linv(Li, Gi, rn);
  }
  return ok;
}

__device__ __forceinline__ bool wave_chol_inv(double* A, int rn, double* Li, double* Gi) {
  if (rn <= 16) return wave_chol_inv_rb<16>(A, rn, Li, Gi);
  if (rn <= 32) return wave_chol_inv_rb<32>(A, rn, Li, Gi);
  return wave_chol_inv_lds(A, rn, Li, Gi);   // out of line: keeps the register forms' allocation lean
}

// Eigenvalues of the symmetric matrix A (destroyed), descending, into lam[0..rn):
// Householder reduction to tridiagonal form (lane i owns row i of the trailing block),
// then bisection on Sturm counts with one eigenvalue per lane. ws: LDS scratch of
// 4*rn doubles.
static __device__ void wave_eigvals(double* A, int rn, double* lam, double* ws) {
  const int lane = threadIdx.x & 63;
  double* d = ws;
  double* e2 = ws + rn;
  double* v = ws + 2 * rn;
  double* wv = ws + 3 * rn;
  for (int k = 0; k + 2 < rn; ++k) {
    const int m = rn - k - 1;
    const double x = lane < m ? A[(k + 1 + lane) * rn + k] : 0.0;
    const double ss = wave_sum_d(x * x);
    const double x0 = __shfl(x, 0, 64);
    double bk = 0.0, ek = x0;
    double vi = x;
    if (ss > 0.0) {
      const double xn = sqrt(ss);
      const double alpha = x0 > 0.0 ? -xn : xn;
      const double v0 = x0 - alpha;
      bk = 2.0 / (ss - x0 * x0 + v0 * v0);
      ek = alpha;
      if (lane == 0) vi = v0;
    }
    if (lane == 0) { d[k] = A[k * rn + k]; e2[k] = ek * ek; }
    if (lane < m) v[lane] = vi;
    wave_fence();
    if (bk != 0.0) {
      double p = 0.0;
      if (lane < m) {
        const double* row = A + (k + 1 + lane) * rn + (k + 1);
        for (int j = 0; j < m; ++j) p += row[j] * v[j];
        p *= bk;
      }
      const double Kc = 0.5 * bk * wave_sum_d(lane < m ? p * vi : 0.0);
      if (lane < m) wv[lane] = p - Kc * vi;
      wave_fence();
      if (lane < m) {
        double* row = A + (k + 1 + lane) * rn + (k + 1);
        const double wi = wv[lane];
        for (int j = 0; j < m; ++j) row[j] -= vi * wv[j] + wi * v[j];
      }
      wave_fence();
    }
  }
  if (lane == 0) {
    if (rn >= 2) {
      d[rn - 2] = A[(rn - 2) * rn + (rn - 2)];
      const double el = A[(rn - 1) * rn + (rn - 2)];
      e2[rn - 2] = el * el;
    }
    d[rn - 1] = A[(rn - 1) * rn + (rn - 1)];
  }
  wave_fence();
  // Gershgorin interval
  double lo = 1e300, hi = -1e300, mx = 0.0, me = 0.0;
  for (int i = lane; i < rn; i += 64) {
    const double off = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + (i + 1 < rn ? sqrt(e2[i]) : 0.0);
    lo = fmin(lo, d[i] - off);
    hi = fmax(hi, d[i] + off);
    mx = fmax(mx, fabs(d[i]) + off);
    if (i + 1 < rn) me = fmax(me, e2[i]);
  }
  lo = -wave_max_d(-lo);
  hi = wave_max_d(hi);
  mx = wave_max_d(mx);
  me = wave_max_d(me);
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, me);
  lo -= 4.0 * eps * mx + 2.0 * pivmin;
  hi += 4.0 * eps * mx + 2.0 * pivmin;
  // multisection: L lanes per eigenvalue evaluate Sturm counts at L interior points
  int L = 1;
  while (L < 16 && (2 * L) * rn <= 64) L *= 2;
  const int e = lane / L, sub = lane - (lane / L) * L;
  const int idx = rn - 1 - e;               // ascending index of the e-th largest
  double a = lo, b = hi;
  const double invL1 = 1.0 / (double)(L + 1);
  int its = 1;
  {
    int bits = 0;
    for (int q = L + 1; q > 1; q >>= 1) ++bits;      // floor(log2(L+1)) bits per round
    its = (56 + bits - 1) / bits + 1;
  }
  for (int it = 0; it < its; ++it) {
    const double x = a + (b - a) * ((double)(sub + 1) * invL1);
    int c = 0;
    if (e < rn) {
      double q = d[0] - x;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
      for (int i = 1; i < rn; ++i) {
        double r0 = __builtin_amdgcn_rcp(q);
        r0 = r0 * (2.0 - q * r0);
        r0 = r0 * (2.0 - q * r0);
        q = d[i] - x - e2[i - 1] * r0;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
      }
    }
    const unsigned long long mask = __ballot(c > idx);
    const unsigned grp = (unsigned)((mask >> (e * L)) & ((L == 64) ? ~0ull : ((1ull << L) - 1ull)));
    const int f = grp ? __builtin_ctz(grp) : L;   // first sub-point above the target
    const double na = (f == 0) ? a : a + (b - a) * ((double)f * invL1);
    const double nb = (f == L) ? b : a + (b - a) * ((double)(f + 1) * invL1);
    a = na;
    b = nb;
  }
  if (e < rn && sub == 0) lam[e] = 0.5 * (a + b);
  wave_fence();
}

}  // namespace tdb
