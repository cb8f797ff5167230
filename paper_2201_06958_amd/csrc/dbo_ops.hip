// Second-order streams with a tall mode (Sec. 2.2 for p = 2, the grouped spatial mode
// of Sec. 3.2): row passes over V (M x K, the short mode unit-stride) and the
// single-block FP64 kernels between them.
//
// Equations (Corecont) and (basecont) for p = 2 with the stage state (C, U1, U2):
//   F1 = D W2 U2 (M x r), F2 = D^T W1 U1 (K x r), C_dot = U1^T W1 F1,
//   U1_dot = (F1 - U1 C_dot) P1, U2_dot = (F2 - U2 C_dot^T) P2,
//   P1 = C^T (C C^T)^-1, P2 = C (C^T C)^-1.
// A row i of the tall mode needs only its own row of D and U1 plus r x r and K x r
// matrices; the sums over rows (C_dot, F2, Grams, the error) are formed per block and
// reduced by the next small kernel.
#include "dbo.h"
#include <math.h>

namespace tdb {

size_t dbo_lds_bytes(int nb) {
  const int TR = dbo_rows(nb);
  const size_t small = 5 * (size_t)nb * nb;   // two W2 U2, P1, M1 and E (or L^-1)
  return (small + (size_t)TR * (2 * (nb + 1) + (2 * nb + 1))) * sizeof(double);
}

// ---------------------------------------------------------------- row passes
template <int NB>
__device__ __forceinline__ void dbo_load_u(const double* U, long long i, int ld, int r, double (&u)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; ++q) u[q] = q < r ? U[i * ld + q] : 0.0;
}

// The row's stage derivative into LDS (doubles): D's row, or V1 - V0.
template <typename TD, int NB>
__device__ __forceinline__ void dbo_stage_d(const DboArgs& a, const void* D, long long i, double* out) {
  const int K = a.K;
  if (D) {
    const TD* p = static_cast<const TD*>(D) + i * K;
    for (int j = 0; j < K; ++j) out[j] = (double)p[j];
  } else {
    const TD* p1 = static_cast<const TD*>(a.V1) + i * K;
    const TD* p0 = static_cast<const TD*>(a.V0) + i * K;
    for (int j = 0; j < K; ++j) out[j] = (double)p1[j] - (double)p0[j];
  }
}

template <int NB>
__device__ __forceinline__ void dbo_stage_u(const double* U, long long i, int ld, int r, double* out) {
  for (int q = 0; q < r; ++q) out[q] = U[i * ld + q];
}

// f = d B: d (K entries) in LDS, B (K x r, stride NB, zero-padded) in LDS.
template <typename T, int NB>
__device__ __forceinline__ void dbo_dB_lds(const double* d, int K, const T* B, T (&f)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; ++q) f[q] = (T)0;
  for (int j = 0; j < K; ++j) {
    const T dj = (T)d[j];
#pragma unroll
    for (int q = 0; q < NB; ++q) f[q] += dj * B[j * NB + q];
  }
}

// y = (f P - u M) * s: f and u (r entries) in LDS, P and M (stride NB, zero-padded).
template <int NB>
__device__ __forceinline__ void dbo_rhs_lds(const double* f, const double* u, int r, const double* P,
                                            const double* Mm, double s, double (&y)[NB]) {
#pragma unroll
  for (int q = 0; q < NB; ++q) y[q] = 0.0;
  for (int c = 0; c < r; ++c) {
    const double fc = f[c], uc = u[c];
#pragma unroll
    for (int q = 0; q < NB; ++q) y[q] += fc * P[c * NB + q] - uc * Mm[c * NB + q];
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) y[q] *= s;
}

// Registers are bounded by the occupancy each bucket can reach (the compiler would
// otherwise issue every LDS operand of a phase at once).
template <typename TD, typename T, int NB, int PH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB <= 8 ? 4 : (NB <= 16 ? 2 : 1))))
k_dbo_rows(DboArgs a, CtrlState* ctrl) {
  extern __shared__ double lds[];
  if (PH != DBO_MAP && PH != DBO_FLIP && ctrl->numeric) return;
  const int K = a.K, r = a.r, TR = a.TR, tid = threadIdx.x;
  const int XS = NB + 1, YS = 2 * NB + 1;
  double* sP = lds;                  // P1 of the stage being finished (MAP: 1/sigma; FLIP: signs)
  double* sM = sP + NB * NB;         // M1 = C_dot_raw P1 of that stage
  double* sE = sM + NB * NB;         // E = C U2^T (r x K), or L^-1 (NORM), or Bmax2 (MAP)
  T* sB0 = reinterpret_cast<T*>(sE + NB * NB);   // W2 U2 at the stage-1 state
  T* sB1 = sB0 + NB * NB;                         // the same, stage 2
  double* X = lds + 5 * NB * NB;     // TR x XS (the W2 U2 pair takes at most 2 NB^2 doubles)
  double* Y = X + (size_t)TR * XS;   // TR x YS
  double* Z = Y + (size_t)TR * YS;   // TR x XS: each row's basis row
  const int cols = PH == DBO_MAP || PH == DBO_FLIP ? a.caps : r;
  // the stage matrices, zero-padded to NB x NB
  for (int t = tid; t < NB * NB; t += blockDim.x) {
    const int x = t / NB, y = t % NB;
    const T* B0 = static_cast<const T*>(a.Bt);
    const T* B1 = B0 + DBO_KMAX * DBO_RMAX;
    const bool kr = x < K && y < r;
    const bool rr = x < r && y < r;
    if (PH == DBO_MAP) {
      sE[t] = (x < K && y < a.caps) ? a.Bmax2[x * a.caps + y] : 0.0;
      const double sg = y < a.caps ? a.sig2[y] : 0.0;
      sP[t] = (x == 0 && y < a.caps && sg > 1e-14 * a.sig2[0] && sg > 0.0) ? 1.0 / sg : 0.0;
    } else if (PH == DBO_FLIP) {
      sP[t] = (x == 0 && y < a.caps) ? a.wk[DBO_WK_SG + y] : 0.0;
    } else if (PH == DBO_NORM) {
      sE[t] = rr ? a.wk[DBO_WK_LI + x * DBO_RMAX + y] : 0.0;
    } else {
      sB0[t] = kr ? B0[x * DBO_RMAX + y] : (T)0;
      sB1[t] = kr ? B1[x * DBO_RMAX + y] : (T)0;
      const int st = PH == DBO_FIN2 ? 1 : 0;
      sP[t] = rr ? a.wk[DBO_WK_P1 + st * DBO_RR + x * DBO_RMAX + y] : 0.0;
      sM[t] = rr ? a.wk[DBO_WK_M1 + st * DBO_RR + x * DBO_RMAX + y] : 0.0;
      sE[t] = (x < r && y < K) ? a.wk[DBO_WK_E + x * DBO_KMAX + y] : 0.0;
    }
  }
  __syncthreads();
  // outputs of the sums: X^T Y over the chunk's rows (nx x ny)
  int nx = 0, ny = 0;
  if (PH == DBO_PASS1 || PH == DBO_FIN1) { nx = r; ny = r + K; }
  if (PH == DBO_FIN2 || PH == DBO_FINE) { nx = r + 1; ny = r + 2; }
  const int nout = nx * ny;
  // outputs of at most 128 entries are split over row segments so that every thread works
  const int noutp = nout <= 64 ? 64 : (nout <= 128 ? 128 : 256);
  const int nseg = nout <= 128 ? 256 / noutp : 1;
  constexpr int NQ = (NB * 2 * NB + 255) / 256;   // >= outputs per thread when nseg == 1
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  // column argmax of the HOSVD map: (|x|, row, sign) kept by thread q < caps
  double bmax = -1.0, bsign = 1.0;
  long long brow = 0;

  const long long nchunk = (a.M + TR - 1) / TR;
  for (long long ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    // an offset the compiler cannot see through: the stage matrices are read from LDS
    // and the per-thread indices formed where they are used, not held in registers
    // across the chunks
    int zo = 0;
    asm volatile("" : "+s"(zo));
    const int tt = tid + zo;
    const long long i = ch * TR + tt;
    const int nrows = (int)min((long long)TR, a.M - ch * TR);
    const double* P = sP + zo;
    const double* Mm = sM + zo;
    const double* E = sE + zo;
    const T* B0 = sB0 + zo;
    const T* B1 = sB1 + zo;
    if (tt < TR && i < a.M) {
      double* xr = X + (size_t)tt * XS;
      double* yr = Y + (size_t)tt * YS;
      const double w1 = a.w1[i];
      double* zr = Z + (size_t)tt * XS;
      // the row's derivative goes to yr[r ..], its basis row to zr; the contractions
      // loop over the contracted index with only their outputs in registers
      if (PH == DBO_PASS1 || PH == DBO_FIN1) {
        dbo_stage_d<TD, NB>(a, a.D1, i, yr + r);
        dbo_stage_u<NB>(a.U1, i, a.ldU1, r, zr);
        T f[NB];
        dbo_dB_lds<T, NB>(yr + r, K, B0, f);
        if (PH == DBO_FIN1) {
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < r) yr[q] = (double)f[q];
          double ud[NB];
          dbo_rhs_lds<NB>(yr, zr, r, P, Mm, a.dscale, ud);
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < r) {
              a.kU1[i * a.ldU1 + q] = ud[q];
              zr[q] += a.dt * ud[q];
            }
          if (a.D2) dbo_stage_d<TD, NB>(a, a.D2, i, yr + r);
          dbo_dB_lds<T, NB>(yr + r, K, B1, f);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < r) {
            xr[q] = w1 * zr[q];
            yr[q] = (double)f[q];
          }
      } else if (PH == DBO_FIN2 || PH == DBO_FINE) {
        const void* Dst = PH == DBO_FIN2 ? (a.D2 ? a.D2 : a.D1) : a.D1;
        dbo_stage_d<TD, NB>(a, Dst, i, yr + r);
        dbo_stage_u<NB>(a.U1, i, a.ldU1, r, zr);
        if (PH == DBO_FIN2) {
          for (int q = 0; q < r; ++q) zr[q] += a.dt * a.kU1[i * a.ldU1 + q];
        }
        {
          T f[NB];
          dbo_dB_lds<T, NB>(yr + r, K, PH == DBO_FIN2 ? B1 : B0, f);
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q < r) xr[q] = (double)f[q];
        }
        double un[NB];
        dbo_rhs_lds<NB>(xr, zr, r, P, Mm, a.dscale, un);
        // un holds the stage's basis derivative; the new basis row from U1 and kU1
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (PH == DBO_FIN2)
            un[q] = q < r ? a.U1[i * a.ldU1 + q] + 0.5 * a.dt * (a.kU1[i * a.ldU1 + q] + un[q]) : 0.0;
          else
            un[q] = q < r ? a.U1[i * a.ldU1 + q] + a.dt * un[q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < r) a.U1[i * a.ldU1 + q] = un[q];
        // error of the advanced (not yet re-orthonormalised) factors: row i of
        // U1 C U2^T is un E
        const TD* vp = static_cast<const TD*>(a.V1) + i * K;
        double e = 0.0, nv = 0.0;
        for (int j = 0; j < K; ++j) {
          double rc = 0.0;
#pragma unroll
          for (int q = 0; q < NB; ++q) rc += un[q] * E[q * NB + j];
          const double v = (double)vp[j], dv = v - rc;
          e += a.w2[j] * dv * dv;
          nv += a.w2[j] * v * v;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < r) {
            xr[q] = w1 * un[q];
            yr[q] = un[q];
          }
        xr[r] = 1.0;
        yr[r] = w1 * e;
        yr[r + 1] = w1 * nv;
      } else if (PH == DBO_NORM) {
        double u[NB];
        dbo_load_u<NB>(a.U1, i, a.ldU1, r, u);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          double s = 0.0;
#pragma unroll
          for (int c = 0; c < NB; ++c) s += u[c] * E[q * NB + c];
          if (q < r) a.U1[i * a.ldU1 + q] = s;
        }
      } else if (PH == DBO_MAP) {
        double v[NB];
        const TD* vp = static_cast<const TD*>(a.V1) + i * K;
#pragma unroll
        for (int j = 0; j < NB; ++j) v[j] = j < K ? (double)vp[j] : 0.0;
        const double sw = sqrt(w1);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < NB; ++j) s += v[j] * E[j * NB + q];
          const double um = s * P[q];
          if (q < cols) {
            a.Umax1[i * a.ldU1 + q] = um;
            xr[q] = sw * um;
          }
        }
      } else {   // DBO_FLIP
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < cols) a.Umax1[i * a.ldU1 + q] *= P[q];
      }
    }
    if (PH == DBO_NORM || PH == DBO_FLIP) continue;
    __syncthreads();
    if (PH == DBO_MAP) {
      if (tt < cols) {
        for (int t = 0; t < nrows; ++t) {
          const double x = X[(size_t)t * XS + tt];
          if (fabs(x) > bmax) {
            bmax = fabs(x);
            brow = ch * TR + t;
            bsign = x < 0.0 ? -1.0 : 1.0;
          }
        }
      }
    } else {
      const int o0 = nseg > 1 ? tt % noutp : tt, seg = nseg > 1 ? tt / noutp : 0;
      const int rs = nseg > 1 ? (nrows * seg) / nseg : 0;
      const int re = nseg > 1 ? (nrows * (seg + 1)) / nseg : nrows;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int o = o0 + q * 256;
        if ((nseg > 1 && q > 0) || o >= nout) continue;
        const int ax = o / ny, by = o - (o / ny) * ny;
        double s = 0.0;
        for (int t = rs; t < re; ++t) s += X[(size_t)t * XS + ax] * Y[(size_t)t * YS + by];
        acc[q] += s;
      }
    }
    __syncthreads();
  }
  if (PH == DBO_NORM || PH == DBO_FLIP) return;
  const int slot = dbo_slot(PH, r, K);
  double* out = a.part + (size_t)blockIdx.x * slot;
  if (PH == DBO_MAP) {
    if (tid < cols) {
      out[3 * tid] = bmax;
      out[3 * tid + 1] = (double)brow;
      out[3 * tid + 2] = bsign;
    }
    return;
  }
  if (nseg > 1) {
    // segments in order: seg 0 + seg 1 (+ seg 2 + seg 3)
    const int o0 = tid % noutp, seg = tid / noutp;
    X[tid] = acc[0];
    __syncthreads();
    if (seg == 0 && o0 < nout) {
      double s = X[o0];
      for (int g = 1; g < nseg; ++g) s += X[g * noutp + o0];
      out[o0] = s;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int o = tid + q * 256;
      if (o < nout) out[o] = acc[q];
    }
  }
}

// ---------------------------------------------------------------- small kernels
// In-place lower Cholesky of an n x n LDS matrix (stride DBO_RMAX); false in every
// thread when a pivot is not positive or below TDB_PIVOT_FLOOR times the largest
// diagonal entry.
__device__ bool dbo_chol(double* A, int n) {
  __shared__ int bad;
  __shared__ double dmax;
  if (threadIdx.x == 0) {
    bad = 0;
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, A[i * DBO_RMAX + i]);
    dmax = m;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double piv = A[k * DBO_RMAX + k];
      if (!(piv > TDB_PIVOT_FLOOR * dmax) || !(piv > 0.0)) bad = 1;
      A[k * DBO_RMAX + k] = sqrt(fmax(piv, 1e-300));
    }
    __syncthreads();
    const double lkk = A[k * DBO_RMAX + k];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * DBO_RMAX + k] /= lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) A[i * DBO_RMAX + j] -= A[i * DBO_RMAX + k] * A[j * DBO_RMAX + k];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    if (j > i) A[i * DBO_RMAX + j] = 0.0;
  }
  __syncthreads();
  return bad == 0;
}

// Li = L^-1 for a lower-triangular LDS matrix (both stride DBO_RMAX).
__device__ void dbo_tri_inv(const double* L, double* Li, int n) {
  for (int t = threadIdx.x; t < DBO_RR; t += blockDim.x) Li[t] = 0.0;
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    Li[j * DBO_RMAX + j] = 1.0 / L[j * DBO_RMAX + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * DBO_RMAX + k] * Li[k * DBO_RMAX + j];
      Li[i * DBO_RMAX + j] = -s / L[i * DBO_RMAX + i];
    }
  }
  __syncthreads();
}

// Pseudo-inverses of both unfoldings of the r x r core C (global, row-major):
// P1 = C^T (C C^T)^-1 and P2 = C (C^T C)^-1 (P2 only when the short mode is not full
// rank), into the work area's slots of stage st. False when a Gram fails its test.
__device__ bool dbo_pinv(const DboArgs& a, const double* C, int st, double* G, double* Li, double* Gi) {
  const int r = a.r;
  for (int m = 0; m < 2; ++m) {
    if (m == 1 && a.full2) break;
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int x = t / r, y = t % r;
      double s = 0.0;
      for (int c = 0; c < r; ++c) s += m == 0 ? C[x * r + c] * C[y * r + c] : C[c * r + x] * C[c * r + y];
      G[x * DBO_RMAX + y] = s;
    }
    __syncthreads();
    if (!dbo_chol(G, r)) return false;
    dbo_tri_inv(G, Li, r);
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int x = t / r, y = t % r;
      double s = 0.0;
      for (int k = (x > y ? x : y); k < r; ++k) s += Li[k * DBO_RMAX + x] * Li[k * DBO_RMAX + y];
      Gi[x * DBO_RMAX + y] = s;
    }
    __syncthreads();
    double* P = a.wk + (m == 0 ? DBO_WK_P1 : DBO_WK_P2) + st * DBO_RR;
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int c = t / r, j = t % r;
      double s = 0.0;
      // P1[c][j] = sum_b C[b][c] Gi[b][j];  P2[c][j] = sum_b C[c][b] Gi[b][j]
      for (int b = 0; b < r; ++b) s += (m == 0 ? C[b * r + c] : C[c * r + b]) * Gi[b * DBO_RMAX + j];
      P[c * DBO_RMAX + j] = s;
    }
    __syncthreads();
  }
  return true;
}

template <typename T>
__device__ void dbo_weighted_basis(const DboArgs& a, const double* U2, int st) {
  T* B = static_cast<T*>(a.Bt) + st * DBO_KMAX * DBO_RMAX;
  for (int t = threadIdx.x; t < DBO_KMAX * DBO_RMAX; t += blockDim.x) {
    const int j = t / DBO_RMAX, q = t % DBO_RMAX;
    B[t] = (j < a.K && q < a.r) ? (T)(a.w2[j] * U2[j * a.ldU2 + q]) : (T)0;
  }
}

// Sums over the row blocks' partial slots: S[o] for o < slot. With fewer outputs than
// threads, G groups of threads each sum every G-th block (loads in flight together),
// and the groups' sums are added in group order; the order is fixed either way.
__device__ void dbo_reduce(const DboArgs& a, int slot, double* S, double* tmp) {
  const int G = slot >= (int)blockDim.x ? 1 : min((int)blockDim.x / slot, 16);
  const int t = threadIdx.x;
  if (G > 1) {
    if (t < G * slot) {
      const int o = t % slot, g = t / slot;
      double s = 0.0;
      int b = g;
      // eight loads in flight, added in the same order as one at a time
      for (; b + 7 * G < a.nblk; b += 8 * G) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = a.part[(size_t)(b + u * G) * slot + o];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; b < a.nblk; b += G) s += a.part[(size_t)b * slot + o];
      tmp[g * slot + o] = s;
    }
    __syncthreads();
    for (int o = t; o < slot; o += blockDim.x) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += tmp[g * slot + o];
      S[o] = s;
    }
  } else {
    for (int o = t; o < slot; o += blockDim.x) {
      double s = 0.0;
      for (int b = 0; b < a.nblk; ++b) s += a.part[(size_t)b * slot + o];
      S[o] = s;
    }
  }
  __syncthreads();
}

// The short mode's basis derivative of a stage: H2 = F2 P2, M2 = U2^T W2 H2,
// U2_dot = (H2 - U2 M2) * dscale (zero when the mode is full rank). S holds the
// stage's sums (r x (r + K): row a is [C_dot_raw[a][:] | F2^T[a][:]]).
__device__ void dbo_u2dot(const DboArgs& a, const double* S, const double* U2s, int st, double* H2, double* M2,
                          double* out) {
  const int r = a.r, K = a.K, ny = r + K;
  if (a.full2) {
    for (int t = threadIdx.x; t < K * r; t += blockDim.x) out[t] = 0.0;
    __syncthreads();
    return;
  }
  const double* P2 = a.wk + DBO_WK_P2 + st * DBO_RR;
  for (int t = threadIdx.x; t < K * r; t += blockDim.x) {
    const int j = t / r, c = t % r;
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += S[b * ny + r + j] * P2[b * DBO_RMAX + c];
    H2[j * DBO_RMAX + c] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
    const int q = t / r, c = t % r;
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += a.w2[j] * U2s[j * a.ldU2 + q] * H2[j * DBO_RMAX + c];
    M2[q * DBO_RMAX + c] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < K * r; t += blockDim.x) {
    const int j = t / r, c = t % r;
    double s = H2[j * DBO_RMAX + c];
    for (int q = 0; q < r; ++q) s -= U2s[j * a.ldU2 + q] * M2[q * DBO_RMAX + c];
    out[t] = s * a.dscale;
  }
  __syncthreads();
}

// M1 = C_dot_raw P1 of stage st (for the row passes) and C_dot = C_dot_raw * dscale
// into Cd; false (in every thread) when C_dot is not finite.
__device__ bool dbo_cdot(const DboArgs& a, const double* S, int st, double* Cd) {
  __shared__ int nonfinite;
  const int r = a.r, K = a.K, ny = r + K;
  if (threadIdx.x == 0) nonfinite = 0;
  __syncthreads();
  const double* P1 = a.wk + DBO_WK_P1 + st * DBO_RR;
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
    const int x = t / r, y = t % r;
    const double cd = S[x * ny + y] * a.dscale;
    if (!isfinite(cd)) nonfinite = 1;
    Cd[t] = cd;
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += S[x * ny + c] * P1[c * DBO_RMAX + y];
    a.wk[DBO_WK_M1 + st * DBO_RR + x * DBO_RMAX + y] = s;
  }
  __syncthreads();
  return nonfinite == 0;
}

// E = C U2^T (r x K) for the error of the advanced factors.
__device__ void dbo_expansion(const DboArgs& a) {
  const int r = a.r, K = a.K;
  for (int t = threadIdx.x; t < r * K; t += blockDim.x) {
    const int q = t / K, j = t % K;
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += a.C0[q * r + c] * a.U2[j * a.ldU2 + c];
    a.wk[DBO_WK_E + q * DBO_KMAX + j] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_dbo_small(DboArgs a, CtrlState* ctrl, int step) {
  __shared__ double G[DBO_RR], Li[DBO_RR], Gi[DBO_RR];
  __shared__ double S[DBO_RMAX * (DBO_RMAX + DBO_KMAX)];
  __shared__ double Cd[DBO_RR];
  __shared__ double U2d[DBO_KMAX * DBO_RMAX];
  const int r = a.r, K = a.K;
  // a singular core found while the previous step prepared this one belongs to this
  // step's first stage, like a failure of its own preparation
  if (step == DBO_MID1 && (ctrl->numeric & NUM_NEXT) && !(ctrl->numeric & ~NUM_NEXT)) {
    if (threadIdx.x == 0) {
      atomicOr(&ctrl->numeric, NUM_CORE);
      atomicAnd(&ctrl->numeric, ~NUM_NEXT);
    }
    return;
  }
  if (step != DBO_SIGN && ctrl->numeric) return;
  if (step == DBO_PREP) {
    if (!dbo_pinv(a, a.C0, 0, G, Li, Gi)) {
      if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_CORE);
      return;
    }
    dbo_weighted_basis<T>(a, a.U2, 0);
    return;
  }
  if (step == DBO_MID1 || step == DBO_MID2) {
    const int st = step == DBO_MID1 ? 0 : 1;
    dbo_reduce(a, r * (r + K), S, Cd);
    if (!dbo_cdot(a, S, st, Cd)) {
      if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_NONFINITE);
      return;
    }
    const double* U2s = st == 0 ? a.U2 : a.Us2;
    dbo_u2dot(a, S, U2s, st, G, Gi, U2d);
    const int cs = r * r;
    if (st == 0 && a.euler) {
      for (int t = threadIdx.x; t < cs; t += blockDim.x) a.C0[t] += a.dt * Cd[t];
      for (int t = threadIdx.x; t < K * r; t += blockDim.x) a.U2[(t / r) * a.ldU2 + t % r] += a.dt * U2d[t];
      __syncthreads();
      dbo_expansion(a);
      return;
    }
    if (st == 0) {
      for (int t = threadIdx.x; t < cs; t += blockDim.x) {
        a.kC[t] = Cd[t];
        a.Cs[t] = a.C0[t] + a.dt * Cd[t];
      }
      for (int t = threadIdx.x; t < K * r; t += blockDim.x) {
        const int j = t / r, c = t % r;
        a.kU2[j * a.ldU2 + c] = U2d[t];
        a.Us2[j * a.ldU2 + c] = a.U2[j * a.ldU2 + c] + a.dt * U2d[t];
      }
      __syncthreads();
      if (!dbo_pinv(a, a.Cs, 1, G, Li, Gi)) {
        if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_CORE);
        return;
      }
      dbo_weighted_basis<T>(a, a.Us2, 1);
      return;
    }
    for (int t = threadIdx.x; t < cs; t += blockDim.x) a.C0[t] += 0.5 * a.dt * (a.kC[t] + Cd[t]);
    for (int t = threadIdx.x; t < K * r; t += blockDim.x) {
      const int j = t / r, c = t % r;
      a.U2[j * a.ldU2 + c] += 0.5 * a.dt * (a.kU2[j * a.ldU2 + c] + U2d[t]);
    }
    __syncthreads();
    dbo_expansion(a);
    return;
  }
  if (step == DBO_END) {
    const int ny = r + 2;
    dbo_reduce(a, (r + 1) * ny, S, Cd);
    if (threadIdx.x == 0) {
      ctrl->eps2 = S[r * ny + r];
      ctrl->nu2 = S[r * ny + r + 1];
    }
    // one round of Cholesky QR per mode in the W inner product, R folded into the core
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) G[(t / r) * DBO_RMAX + t % r] = S[(t / r) * ny + t % r];
    __syncthreads();
    if (!dbo_chol(G, r)) {
      if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_BASIS);
      return;
    }
    dbo_tri_inv(G, Li, r);
    for (int t = threadIdx.x; t < r * r; t += blockDim.x)
      a.wk[DBO_WK_LI + (t / r) * DBO_RMAX + t % r] = Li[(t / r) * DBO_RMAX + t % r];
    // Cd = L1^T C
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int x = t / r, y = t % r;
      double s = 0.0;
      for (int c = x; c < r; ++c) s += G[c * DBO_RMAX + x] * a.C0[c * r + y];
      Cd[t] = s;
    }
    __syncthreads();
    // the short mode: Gram U2^T W2 U2 into Gi, its factor L2 in place
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int x = t / r, y = t % r;
      double s = 0.0;
      for (int j = 0; j < K; ++j) s += a.w2[j] * a.U2[j * a.ldU2 + x] * a.U2[j * a.ldU2 + y];
      Gi[x * DBO_RMAX + y] = s;
    }
    __syncthreads();
    if (!dbo_chol(Gi, r)) {
      if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_BASIS);
      return;
    }
    dbo_tri_inv(Gi, Li, r);
    // C = (L1^T C) L2
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
      const int x = t / r, y = t % r;
      double s = 0.0;
      for (int d = y; d < r; ++d) s += Cd[x * r + d] * Gi[d * DBO_RMAX + y];
      a.C0[t] = s;
    }
    // U2 <- U2 L2^-T
    for (int t = threadIdx.x; t < K * r; t += blockDim.x) {
      const int j = t / r, q = t % r;
      double s = 0.0;
      for (int c = 0; c <= q; ++c) s += a.U2[j * a.ldU2 + c] * Li[q * DBO_RMAX + c];
      U2d[t] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < K * r; t += blockDim.x) a.U2[(t / r) * a.ldU2 + t % r] = U2d[t];
    __syncthreads();
    // the next step's stage-1 pseudo-inverses and W2 U2 at the new state
    if (!dbo_pinv(a, a.C0, 0, G, Li, Gi)) {
      if (threadIdx.x == 0) atomicOr(&ctrl->numeric, NUM_NEXT);
      return;
    }
    dbo_weighted_basis<T>(a, a.U2, 0);
    return;
  }
  // DBO_SIGN: the HOSVD map's column argmax over the blocks (larger |x| wins, the
  // lower row on a tie), the tall mode's singular values, and the core at the caps,
  // diag(sign * sigma)
  const int cp = a.caps;
  for (int q = threadIdx.x; q < cp; q += blockDim.x) {
    double bm = -1.0, bs = 1.0, br = 0.0;
    for (int b = 0; b < a.nblk; ++b) {
      const double* pb = a.part + (size_t)b * (3 * DBO_RMAX) + 3 * q;
      if (pb[0] > bm || (pb[0] == bm && pb[1] < br)) {
        bm = pb[0];
        br = pb[1];
        bs = pb[2];
      }
    }
    a.wk[DBO_WK_SG + q] = bs;
  }
  for (int q = threadIdx.x; q <= cp; q += blockDim.x) a.sig1[q] = a.sig2[q];
  __syncthreads();
  for (int t = threadIdx.x; t < cp * cp; t += blockDim.x) {
    const int x = t / cp, y = t % cp;
    const double sg = a.sig2[x];
    const bool live = sg > 1e-14 * a.sig2[0] && sg > 0.0;
    a.Cmax[t] = (x == y && live) ? a.wk[DBO_WK_SG + x] * sg : 0.0;
  }
}

// ---------------------------------------------------------------- launchers
template <typename TD, typename T, int NB, int PH>
hipError_t dbo_rows_ph(const DboArgs& a, CtrlState* ctrl, hipStream_t s) {
  const size_t lds = dbo_lds_bytes(NB);
  static bool attr = false;   // the dynamic LDS limit is raised once per kernel
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_dbo_rows<TD, T, NB, PH>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_dbo_rows<TD, T, NB, PH>), dim3(a.nblk), dim3(256), lds, s, a, ctrl);
  return hipGetLastError();
}

template <typename TD, typename T, int NB>
hipError_t dbo_rows_nb(const DboArgs& a, int phase, CtrlState* ctrl, hipStream_t s) {
  switch (phase) {
    case DBO_PASS1: return dbo_rows_ph<TD, T, NB, DBO_PASS1>(a, ctrl, s);
    case DBO_FIN1: return dbo_rows_ph<TD, T, NB, DBO_FIN1>(a, ctrl, s);
    case DBO_FIN2: return dbo_rows_ph<TD, T, NB, DBO_FIN2>(a, ctrl, s);
    case DBO_FINE: return dbo_rows_ph<TD, T, NB, DBO_FINE>(a, ctrl, s);
    case DBO_NORM: return dbo_rows_ph<TD, T, NB, DBO_NORM>(a, ctrl, s);
    case DBO_MAP: return dbo_rows_ph<TD, T, NB, DBO_MAP>(a, ctrl, s);
    case DBO_FLIP: return dbo_rows_ph<TD, T, NB, DBO_FLIP>(a, ctrl, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TD, typename T>
hipError_t launch_dbo_rows(const DboArgs& a, int phase, CtrlState* ctrl, hipStream_t s) {
  const int nb = dbo_bucket(a.K);
  if (a.K > DBO_KMAX || a.r > a.K || a.caps > a.K || a.TR != dbo_rows(nb) || a.nblk < 1) return hipErrorInvalidValue;
  if (nb == 8) return dbo_rows_nb<TD, T, 8>(a, phase, ctrl, s);
  if (nb == 16) return dbo_rows_nb<TD, T, 16>(a, phase, ctrl, s);
  return dbo_rows_nb<TD, T, 32>(a, phase, ctrl, s);
}

template <typename T>
hipError_t launch_dbo_small(const DboArgs& a, int step, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_dbo_small<T>, dim3(1), dim3(256), 0, s, a, ctrl, step);
  return hipGetLastError();
}

template hipError_t launch_dbo_rows<double, double>(const DboArgs&, int, CtrlState*, hipStream_t);
template hipError_t launch_dbo_rows<float, float>(const DboArgs&, int, CtrlState*, hipStream_t);
template hipError_t launch_dbo_rows<float, double>(const DboArgs&, int, CtrlState*, hipStream_t);
template hipError_t launch_dbo_rows<double, float>(const DboArgs&, int, CtrlState*, hipStream_t);
template hipError_t launch_dbo_small<double>(const DboArgs&, int, CtrlState*, hipStream_t);
template hipError_t launch_dbo_small<float>(const DboArgs&, int, CtrlState*, hipStream_t);

}  // namespace tdb
