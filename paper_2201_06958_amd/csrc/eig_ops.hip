// Leading eigenpairs of the weighted mode Gram matrices of the HOSVD (Sec. 2.3):
// Householder reduction to tridiagonal form spread over many workgroups (one launch
// per reflector; the last reflectors in one workgroup per mode, the trailing block in
// LDS), bisection on Sturm counts for the leading K+1 eigenvalues, inverse iteration
// for the K leading eigenvectors (clusters of close eigenvalues
// orthogonalised within one wave), back-transformation by the stored reflectors and
// a sign convention (largest-magnitude entry positive, lowest index on a tie).
//
// Reflector k (k = 0..n-3) acts on indices k+1..n-1; it ends up in row k of G (entries
// k+1..n-1), its coefficient in beta[k]. While the distributed steps run it lives in
// one of two vectors vr (entries k+1..n-1), and the next launch copies it into G, so
// that row k of G, read in place of column k, is not overwritten while it is read. Launch k applies the rank-2 update
// of reflector k-1 to this workgroup's rows of the trailing block (columns k+1..n-1),
// forms column k and the diagonal entry k of the updated matrix on the fly from the
// not yet updated values (nobody writes them in this launch), computes reflector k
// redundantly in every workgroup (the same fixed-order sums everywhere), and the
// product p = beta A v for its rows into one of two buffers (the other still holds
// the previous reflector's product, which every workgroup reads in this launch).
#include "tdb_common.h"
#include "tdb_kernels.h"
#include <math.h>

namespace tdb {

#define NE TDB_NEIG
#define EC 8    // rows per chunk of the per-lane tridiagonal sweeps
#define TRI_TAIL 128   // largest trailing block reduced by a single workgroup
#define TT_PARTS 8     // thread groups of TRI_TAIL threads in that workgroup
#define TT_THREADS (TRI_TAIL * TT_PARTS)

// Per-mode workspace (after the K eigenvector columns): d, e, beta, p0, p1, vr0, vr1.
struct EigWs {
  double *X, *d, *e, *beta, *p[2], *vr[2];
};
__device__ __forceinline__ EigWs eig_ws(const EigArgs& a) {
  EigWs w;
  const long long n = a.Nn;
  w.X = a.work;
  w.d = a.work + n * a.k;
  w.e = w.d + n;
  w.beta = w.e + n;
  w.p[0] = w.beta + n;
  w.p[1] = w.p[0] + n;
  w.vr[0] = w.p[1] + n;
  w.vr[1] = w.vr[0] + n;
  return w;
}

// Step k of the distributed reduction for one mode, as workgroup bx of nblk.
// Every global load of a step (the previous reflector and its product, row k, and this
// workgroup's rows of the trailing block) is issued at entry into registers: one round
// trip to memory per launch rather than three. A wave owns at most TS_ROWS rows.
#define TS_ROWS 4
#define TS_COLS (NE / 64)
__device__ __forceinline__ void tri_step_body(const EigArgs& a, int k, int bx, int nblk, double* vp, double* wp,
                                              double* v, double* red) {
  const int n = a.Nn;
  if (k + 2 >= n || k >= a.k0) return;
  const EigWs w = eig_ws(a);
  double* G = a.G;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int mp = n - k, m = n - k - 1;
  const double* pp = ((k - 1) & 1) ? w.p[1] : w.p[0];
  const double* vq = ((k - 1) & 1) ? w.vr[1] : w.vr[0];
  // ---- loads
  const double bp = k > 0 ? w.beta[k - 1] : 0.0;
  const double dk0 = G[(long long)k * n + k];
  double vl[2], pl[2], cl[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = tid + 256 * u;
    vl[u] = (k > 0 && i < mp) ? vq[k + i] : 0.0;
    pl[u] = (k > 0 && i < mp) ? pp[k + i] : 0.0;
    cl[u] = i < m ? G[(long long)k * n + k + 1 + i] : 0.0;
  }
  double rv[TS_ROWS][TS_COLS];
#pragma unroll
  for (int q = 0; q < TS_ROWS; ++q) {
    const int i = bx + nblk * wid + 4 * nblk * q;
#pragma unroll
    for (int c = 0; c < TS_COLS; ++c) {
      const int j = lane + 64 * c;
      rv[q][c] = (i < m && j < m) ? G[(long long)(k + 1 + i) * n + k + 1 + j] : 0.0;
    }
  }
  // ---- the pending update of reflector k-1 (acting on indices k..n-1)
  if (bp != 0.0) {
    double pvv = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + 256 * u;
      if (i < mp) {
        vp[i] = vl[u];
        pvv += pl[u] * vl[u];
      }
    }
    pvv = block_sum(pvv, red);
    const double Kc = 0.5 * bp * pvv;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + 256 * u;
      if (i < mp) wp[i] = pl[u] - Kc * vl[u];
    }
    __syncthreads();
  }
  // column k below the diagonal and the diagonal entry of the updated matrix; the
  // trailing block stays exactly symmetric (each update forms the same two products and
  // only the order of their sum differs), so column k is read as the contiguous row k
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = tid + 256 * u;
    if (i < m) {
      double x = cl[u];
      if (bp != 0.0) x -= vp[0] * wp[1 + i] + wp[0] * vp[1 + i];
      v[i] = x;
      ss += x * x;
    }
  }
  ss = block_sum(ss, red);
  const double x0 = v[0];
  double dk = dk0;
  if (bp != 0.0) dk -= vp[0] * wp[0] + wp[0] * vp[0];
  double bk = 0.0, ek = x0;
  __syncthreads();
  if (ss > 0.0) {
    const double xn = sqrt(ss);
    const double alpha = x0 > 0.0 ? -xn : xn;
    const double v0 = x0 - alpha;
    const double vtv = ss - x0 * x0 + v0 * v0;
    bk = 2.0 / vtv;
    ek = alpha;
    if (tid == 0) v[0] = v0;
  }
  __syncthreads();
  // rows of this workgroup: k+1+i for i = bx + nblk*wid + 4*nblk*q; one wave per row
  double* pk = (k & 1) ? w.p[1] : w.p[0];
#pragma unroll
  for (int q = 0; q < TS_ROWS; ++q) {
    const int i = bx + nblk * wid + 4 * nblk * q;
    if (i < m) {
      double* row = G + (long long)(k + 1 + i) * n + (k + 1);
      double sv = 0.0;
      if (bp != 0.0) {
        const double vr = vp[1 + i], wr = wp[1 + i];
#pragma unroll
        for (int c = 0; c < TS_COLS; ++c) {
          const int j = lane + 64 * c;
          if (j < m) {
            const double x = rv[q][c] - (vr * wp[1 + j] + wr * vp[1 + j]);
            row[j] = x;
            sv += x * v[j];
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < TS_COLS; ++c) {
          const int j = lane + 64 * c;
          if (j < m) sv += rv[q][c] * v[j];
        }
      }
      sv = warp_sum(sv);
      if (lane == 0) pk[k + 1 + i] = bk * sv;
    }
  }
  if (bx == 0) {
    // this reflector into its vector; the previous one (read by every workgroup above,
    // from the other vector) into row k-1 of G, which nobody reads in this launch
    double* vk = (k & 1) ? w.vr[1] : w.vr[0];
    for (int i = tid; i < m; i += blockDim.x) vk[k + 1 + i] = v[i];
    if (k > 0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = tid + 256 * u;
        if (i < mp) G[(long long)(k - 1) * n + k + i] = vl[u];
      }
    }
    if (tid == 0) {
      w.d[k] = dk;
      w.e[k] = ek;
      w.beta[k] = bk;
    }
  }
}

__global__ void __launch_bounds__(256) k_tri_step(EigBatch batch, int k) {
  __shared__ double vp[NE], wp[NE], v[NE];
  __shared__ double red[16];
  tri_step_body(batch.m[blockIdx.y], k, blockIdx.x, gridDim.x, vp, wp, v, red);
}

// Reflectors k0 .. n-3 and the last 2 x 2 block in one workgroup per mode, with the
// trailing block A[k0..n-1][k0..n-1] (at most TRI_TAIL rows, full and symmetric) in
// LDS: the distributed steps above cost a launch each, and once the trailing block is
// this small a workgroup does a step in far less than a launch. It first applies the
// pending update of reflector k0-1, then runs the same reflector formulas as
// k_tri_step (sums in a fixed order), storing each reflector in row k of G for the
// back-transformation.
__global__ void __launch_bounds__(TT_THREADS) k_tri_tail(EigBatch batch) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, k0 = a.k0, T = n - k0;   // block size (<= TRI_TAIL)
  const EigWs w = eig_ws(a);
  double* G = a.G;
  double* v = A + (long long)T * T;            // TRI_TAIL
  double* wv = v + TRI_TAIL;                   // TRI_TAIL
  double* part = wv + TRI_TAIL;                // TT_PARTS * TRI_TAIL partial products
  __shared__ double red[16];
  const int tid = threadIdx.x;
  // thread layout over the block: column c = tid % TRI_TAIL, rows h, h + TT_PARTS, ...
  const int c = tid & (TRI_TAIL - 1), h = tid >> 7;
  if (n == 1) {
    if (tid == 0) { w.d[0] = G[0]; w.e[0] = 0.0; w.beta[0] = 0.0; }
    return;
  }
  if (c < T)
    for (int i = h; i < T; i += TT_PARTS) A[i * T + c] = G[(long long)(k0 + i) * n + k0 + c];
  __syncthreads();
  // the pending update of reflector k0-1 (acting on indices k0..n-1)
  const double bp = k0 > 0 ? w.beta[k0 - 1] : 0.0;
  if (k0 > 0) {
    // the last distributed reflector into row k0-1 of G
    const double* vq = ((k0 - 1) & 1) ? w.vr[1] : w.vr[0];
    for (int i = tid; i < T; i += blockDim.x) G[(long long)(k0 - 1) * n + k0 + i] = vq[k0 + i];
  }
  if (bp != 0.0) {
    const double* pp = ((k0 - 1) & 1) ? w.p[1] : w.p[0];
    const double* vq = ((k0 - 1) & 1) ? w.vr[1] : w.vr[0];
    double pvv = 0.0;
    for (int i = tid; i < T; i += blockDim.x) {
      const double vi = vq[k0 + i];
      v[i] = vi;
      pvv += pp[k0 + i] * vi;
    }
    pvv = block_sum(pvv, red);
    const double Kc = 0.5 * bp * pvv;
    for (int i = tid; i < T; i += blockDim.x) wv[i] = pp[k0 + i] - Kc * v[i];
    __syncthreads();
    if (c < T) {
      const double vc = v[c], wc = wv[c];
      for (int i = h; i < T; i += TT_PARTS) A[i * T + c] -= v[i] * wc + wv[i] * vc;
    }
    __syncthreads();
  }
  for (int k = k0; k + 2 < n; ++k) {
    const int r1 = k - k0 + 1;         // block row/column of index k+1
    const int m = n - k - 1;
    // column k below the diagonal
    double ss = 0.0;
    for (int i = tid; i < m; i += blockDim.x) {
      const double x = A[(r1 + i) * T + r1 - 1];
      v[i] = x;
      ss += x * x;
    }
    ss = block_sum(ss, red);
    const double x0 = v[0];
    double bk = 0.0, ek = x0;
    if (ss > 0.0) {
      const double xn = sqrt(ss);
      const double alpha = x0 > 0.0 ? -xn : xn;
      const double v0 = x0 - alpha;
      const double vtv = ss - x0 * x0 + v0 * v0;
      bk = 2.0 / vtv;
      ek = alpha;
    }
    __syncthreads();
    if (tid == 0) {
      if (ss > 0.0) v[0] = x0 - ek;
      w.d[k] = A[(r1 - 1) * T + r1 - 1];
      w.e[k] = ek;
      w.beta[k] = bk;
    }
    __syncthreads();
    for (int i = tid; i < m; i += blockDim.x) G[(long long)k * n + k + 1 + i] = v[i];
    if (bk != 0.0) {
      // p = bk A v over the trailing block: column c of A (= row c), the sum split in
      // TT_PARTS ranges over the workgroup's thread groups, added in a fixed order
      const int hm = (m + TT_PARTS - 1) / TT_PARTS;
      if (c < m) {
        double s = 0.0;
        const int j1 = min(m, (h + 1) * hm);
        for (int j = h * hm; j < j1; ++j) s += A[(r1 + j) * T + r1 + c] * v[j];
        part[h * TRI_TAIL + c] = s;
      }
      __syncthreads();
      double pv = 0.0;
      if (tid < m) {
        double ps = 0.0;
#pragma unroll
        for (int q = 0; q < TT_PARTS; ++q) ps += part[q * TRI_TAIL + tid];
        const double pi = bk * ps;
        wv[tid] = pi;
        pv = pi * v[tid];
      }
      pv = block_sum(pv, red);
      const double Kc = 0.5 * bk * pv;
      if (tid < m) wv[tid] -= Kc * v[tid];
      __syncthreads();
      if (c < m) {
        const double vc = v[c], wc = wv[c];
        for (int i = h; i < m; i += TT_PARTS) A[(r1 + i) * T + r1 + c] -= v[i] * wc + wv[i] * vc;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    const int k = n - 2, r0 = k - k0;
    w.d[k] = A[r0 * T + r0];
    w.e[k] = A[(r0 + 1) * T + r0];
    w.beta[k] = 0.0;
    w.d[k + 1] = A[(r0 + 1) * T + r0 + 1];
    w.e[k + 1] = 0.0;
  }
}

// Sturm count: number of eigenvalues of the tridiagonal (d, e2 = e^2) below x. The
// quotient e2/q of the recurrence is taken as e2 times the reciprocal of q from the
// hardware estimate and two Newton steps (full precision, a shorter dependent chain
// than a division).
__device__ int sturm_count2(const double* d, const double* e2, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    double r = __builtin_amdgcn_rcp(q);
    r = r * (2.0 - q * r);
    r = r * (2.0 - q * r);
    q = d[i] - x - e2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

__device__ __forceinline__ double hash_unit2(unsigned a, unsigned b) {
  unsigned x = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u);
  x ^= x >> 16; x *= 0x7FEB352Du; x ^= x >> 15; x *= 0x846CA68Bu; x ^= x >> 16;
  return (double)x * (2.0 / 4294967296.0) - 1.0;
}

// Grid (mode, eigenvalue): the K+1 leading eigenvalues by multisection on Sturm counts
// (the 64 lanes of one wave evaluate 64 interior points of the eigenvalue's interval,
// which shrinks 65-fold per round: a round costs one serial Sturm recurrence, so fewer
// rounds is what counts), the singular values sqrt(max(lambda, 0)), and the Gershgorin
// scale.
#define EV_PTS 64
__global__ void __launch_bounds__(EV_PTS) k_eig_values(EigBatch batch, double* lam_out) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const EigWs w = eig_ws(a);
  __shared__ double d[NE], e2[NE], red[16];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    d[i] = w.d[i];
    e2[i] = w.e[i] * w.e[i];
  }
  __syncthreads();
  double lo = 1e300, hi = -1e300, mx = 0.0, me = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double off = (i > 0 ? fabs(w.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(w.e[i]) : 0.0);
    lo = fmin(lo, d[i] - off);
    hi = fmax(hi, d[i] + off);
    mx = fmax(mx, fabs(d[i]) + off);
    if (i + 1 < n) me = fmax(me, e2[i]);
  }
  double gl = -block_max(-lo, red);
  double gu = block_max(hi, red);
  const double tn = block_max(mx, red);
  const double emax2 = block_max(me, red);
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  gl -= 4.0 * eps * tn + 2.0 * pivmin;
  gu += 4.0 * eps * tn + 2.0 * pivmin;
  double* lam = lam_out + (long long)blockIdx.x * (TDB_RCAP + 2);
  const int t = blockIdx.y, sub = threadIdx.x;   // eigenvalue, interior point
  double l = gl, h = gu;
  const bool live = t <= K && t < n;
  const int idx = n - 1 - t;                                  // ascending index of the t-th largest
  for (int it = 0; it < 80; ++it) {
    // converged to the accuracy of the eigenvalues themselves: a few ulps of the matrix
    // scale (an eigenvalue below that is numerically zero)
    bool done = !live || h - l <= fmax(2.0 * eps * fmax(fabs(l), fabs(h)), 4.0 * eps * tn) + pivmin;
    if (done) break;   // common to the wave
    const double x = l + (double)(sub + 1) * ((h - l) / (double)(EV_PTS + 1));
    const int c = sturm_count2(d, e2, n, x, pivmin);
    // first point whose count exceeds idx bounds the eigenvalue from above
    const unsigned long long above = __ballot(c > idx);
    {
      const int first = above ? __builtin_ctzll(above) : EV_PTS;   // EV_PTS: above all
      const double nl = first == 0 ? l : l + (double)first * ((h - l) / (double)(EV_PTS + 1));
      const double nh = first == EV_PTS ? h : l + (double)(first + 1) * ((h - l) / (double)(EV_PTS + 1));
      if (nl == l && nh == h) { h = l; }                  // no progress in floating point
      l = nl;
      h = nh;
    }
  }
  if (sub == 0 && t <= K) {
    const double lt = t < n ? 0.5 * (l + h) : 0.0;
    lam[t] = lt;
    a.sig[t] = t < n ? sqrt(fmax(lt, 0.0)) : 0.0;
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) lam[TDB_RCAP + 1] = tn;
}

// Inverse iteration for the K leading eigenvectors in rounds of two kernels: a solve
// (one wave per vector, its chains run by one lane out of LDS) and an orthonormalisation
// of all vectors of a mode in one workgroup (index order, each vector against the
// earlier members of its cluster). The first solve factors T - shift_j I with partial
// pivoting, eliminating the random start vector in the same top-down pass, and keeps
// the factors (multipliers, the two superdiagonals of U, reciprocal pivots, row
// interchanges) for the later rounds. Shifts inside a cluster are kept eps3 apart; a
// cluster starts where the gap to the previous eigenvalue exceeds 1e-3 of the matrix
// scale. Between the kernels the vectors live interleaved (entry i of vector j at
// i*64 + j) in a global workspace; the factors follow, one block of EIG_NF rows of NE
// per vector.
#define EIG_VPB 4   // vectors (waves) per workgroup of the solve
#define EIG_NF 5    // factor rows per vector: multiplier, U superdiagonals 1 and 2, 1/pivot, interchange

// Shift of vector j (the serial cluster walk over eigenvalues 0..j).
__device__ double eig_shift(const double* lam, int j, double ortol, double eps3) {
  double lam_prev = 0.0, lj = 0.0;
  for (int q = 0; q <= j; ++q) {
    lj = lam[q];
    if (!(q == 0 || lam[q - 1] - lj > ortol) && lam_prev - lj < eps3) lj = lam_prev - eps3;
    lam_prev = lj;
  }
  return lj;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(64 * EIG_VPB) k_eig_solve(EigBatch batch, const double* lam_in, double* scratch,
                                                           int first) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.y * EIG_VPB + wv;
  const EigWs w = eig_ws(a);
  const double* lam = lam_in + (long long)blockIdx.x * (TDB_RCAP + 2);
  const double tn = lam[TDB_RCAP + 1];
  double* xb = scratch + (long long)blockIdx.x * NE * 64 * (1 + EIG_NF);
  double* fac = xb + NE * 64 + (long long)j * EIG_NF * NE;
  __shared__ double d[NE], e[NE];
  __shared__ double F[EIG_VPB][EIG_NF][NE], rb[EIG_VPB][NE];
  if (first) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      d[i] = w.d[i];
      e[i] = i + 1 < n ? w.e[i] : 0.0;
    }
    __syncthreads();
  }
  if (j >= K) return;   // whole waves; no barrier follows
  double* fl = F[wv][0];   // multipliers
  double* u1 = F[wv][1];   // U superdiagonal 1
  double* u2 = F[wv][2];   // U superdiagonal 2
  double* rp = F[wv][3];   // 1 / pivot
  double* pv = F[wv][4];   // 1: rows i and i+1 interchanged
  double* x = rb[wv];
  if (first) {
    const double eps = 2.220446049250313e-16;
    double me = 0.0;
    for (int i = lane; i + 1 < n; i += 64) me = fmax(me, e[i] * e[i]);
    for (int off = 32; off > 0; off >>= 1) me = fmax(me, __shfl_xor(me, off, 64));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, me);
    const double ptiny = eps * tn + pivmin;
    for (int i = lane; i < n; i += 64) x[i] = hash_unit2((unsigned)i, (unsigned)j + 1u);
    wave_lds_sync();
    if (lane == 0) {
      const double lj = eig_shift(lam, j, 1e-3 * tn, 10.0 * eps * tn);
      // the running pivot row (cd, cu) and right-hand side entry cb stay in registers,
      // the next rows' entries are loaded EC at a time ahead of the chain
      double cd = d[0] - lj, cu = e[0], cb = x[0];
      for (int i0 = 0; i0 + 1 < n; i0 += EC) {
        double li_[EC], dn_[EC], un_[EC], nb_[EC];
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = min(i0 + u, n - 2);
          li_[u] = e[i];
          dn_[u] = d[i + 1] - lj;
          un_[u] = e[i + 1];   // zero past the end
          nb_[u] = x[i + 1];
        }
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = i0 + u;
          if (i + 1 >= n) break;
          const double li = li_[u], dn = dn_[u], un = un_[u], nb = nb_[u];
          if (fabs(cd) >= fabs(li)) {
            if (cd == 0.0) cd = ptiny;
            const double f = li / cd;
            fl[i] = f;
            rp[i] = 1.0 / cd;
            u1[i] = cu;
            u2[i] = 0.0;
            pv[i] = 0.0;
            x[i] = cb;
            cd = dn - f * cu;
            cu = un;
            cb = nb - f * cb;
          } else {
            const double f = cd / li;
            fl[i] = f;
            rp[i] = 1.0 / li;
            u1[i] = dn;
            u2[i] = un;
            pv[i] = 1.0;
            x[i] = nb;
            cd = cu - f * dn;
            cu = -f * un;
            cb = cb - f * nb;
          }
        }
      }
      if (cd == 0.0) cd = ptiny;
      rp[n - 1] = 1.0 / cd;
      u1[n - 1] = 0.0;
      u2[n - 1] = 0.0;
      fl[n - 1] = 0.0;
      pv[n - 1] = 0.0;
      x[n - 1] = cb;
    }
    wave_lds_sync();
    for (int t = lane; t < EIG_NF * NE; t += 64) {
      const int r = t / NE, i = t - r * NE;
      if (i < n) fac[t] = F[wv][r][i];
    }
  } else {
    for (int t = lane; t < EIG_NF * NE; t += 64) {
      const int r = t / NE, i = t - r * NE;
      if (i < n) F[wv][r][i] = fac[t];
    }
    for (int i = lane; i < n; i += 64) x[i] = xb[i * 64 + j];
    wave_lds_sync();
    if (lane == 0) {
      // forward elimination with the row interchanges, the running entry in a register
      double cur = x[0];
      for (int i0 = 0; i0 + 1 < n; i0 += EC) {
        double nx_[EC], l_[EC], p_[EC];
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = min(i0 + u, n - 2);
          nx_[u] = x[i + 1];
          l_[u] = fl[i];
          p_[u] = pv[i];
        }
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = i0 + u;
          if (i + 1 >= n) break;
          const double nx = nx_[u], l = l_[u];
          const bool sw = p_[u] != 0.0;
          x[i] = sw ? nx : cur;
          cur = sw ? cur - l * nx : nx - l * cur;
        }
      }
      x[n - 1] = cur;
    }
  }
  if (lane == 0) {
    // back substitution, the two later entries in registers
    double x1 = x[n - 1] * rp[n - 1], x2 = 0.0;
    x[n - 1] = x1;
    for (int i0 = n - 2; i0 >= 0; i0 -= EC) {
      double b_[EC], u1_[EC], u2_[EC], r_[EC];
#pragma unroll
      for (int u = 0; u < EC; ++u) {
        const int i = max(i0 - u, 0);
        b_[u] = x[i];
        u1_[u] = u1[i];
        u2_[u] = u2[i];
        r_[u] = rp[i];
      }
#pragma unroll
      for (int u = 0; u < EC; ++u) {
        const int i = i0 - u;
        if (i < 0) break;
        const double x0 = (b_[u] - u1_[u] * x1 - u2_[u] * x2) * r_[u];
        x[i] = x0;
        x2 = x1;
        x1 = x0;
      }
    }
  }
  wave_lds_sync();
  // scale to unit max-norm (keeps the later dot products in range)
  double mx = 0.0;
  for (int i = lane; i < n; i += 64) mx = fmax(mx, fabs(x[i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
  for (int i = lane; i < n; i += 64) xb[i * 64 + j] = x[i] * sc;
}

// Orthonormalisation of one mode's K vectors: wave g holds rows g*MGS_R .. g*MGS_R +
// MGS_R - 1 of all vectors, lane q those of vector q, in registers. Step j reads vector
// j's entries from lane j of each wave, forms every wave's partial squared norm of it
// and partial dot products with the later members of its cluster, and after one
// barrier normalises vector j and removes its component from those members (partials
// in LDS buffers that alternate between steps). The last round writes the column-major
// eigenvector block instead.
#define MGS_G 16
#define MGS_R (NE / MGS_G)
__device__ __forceinline__ double lane_get(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__global__ void __launch_bounds__(1024) k_eig_orth(EigBatch batch, const double* lam_in, double* scratch, int last) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const EigWs w = eig_ws(a);
  const double* lam = lam_in + (long long)blockIdx.x * (TDB_RCAP + 2);
  const double tn = lam[TDB_RCAP + 1];
  double* xb = scratch + (long long)blockIdx.x * NE * 64 * (1 + EIG_NF);
  __shared__ double part[2][MGS_G][64], red[2][MGS_G];
  __shared__ int cend[TDB_RCAP];
  const int q = threadIdx.x & 63, g = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    const double ortol = 1e-3 * tn;
    int cs = 0;
    for (int j = 1; j < K; ++j)
      if (lam[j - 1] - lam[j] > ortol) {
        for (int t = cs; t < j; ++t) cend[t] = j;
        cs = j;
      }
    for (int t = cs; t < K; ++t) cend[t] = K;
  }
  double x[MGS_R];
#pragma unroll
  for (int s = 0; s < MGS_R; ++s) {
    const int i = g * MGS_R + s;
    x[s] = (q < K && i < n) ? xb[i * 64 + q] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const int b = j & 1;
    const int ce = cend[j];
    double ps = 0.0, pd = 0.0;
#pragma unroll
    for (int s = 0; s < MGS_R; ++s) {
      const double y = lane_get(x[s], j);
      ps += y * y;
      pd += x[s] * y;
    }
    if (q == 0) red[b][g] = ps;
    part[b][g][q] = pd;
    __syncthreads();
    double nr = 0.0;
#pragma unroll
    for (int t = 0; t < MGS_G; ++t) nr += red[b][t];
    const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
    const bool act = q > j && q < ce;
    double c = 0.0;
    if (act) {
      double dq = 0.0;
#pragma unroll
      for (int t = 0; t < MGS_G; ++t) dq += part[b][t][q];
      c = dq * inv * inv;
    }
    const double sj = q == j ? inv : 1.0;
    if (j + 1 < ce || q == j) {
#pragma unroll
      for (int s = 0; s < MGS_R; ++s) {
        const double y = lane_get(x[s], j);
        x[s] = x[s] * sj - c * y;
      }
    }
  }
  if (q >= K) return;
#pragma unroll
  for (int s = 0; s < MGS_R; ++s) {
    const int i = g * MGS_R + s;
    if (i < n) {
      if (last) w.X[(long long)q * n + i] = x[s];
      else xb[i * 64 + q] = x[s];
    }
  }
}

// Back-transformation x <- H_0 H_1 ... H_{n-3} x and the sign convention; grid (mode,
// vector), one wave per vector. Lane l holds entries l, l+64, ... of the vector in
// registers; each reflector's entries are loaded one step ahead of its use.
#define BK_R (NE / 64)
#define BK_G 4   // reflectors per prefetch group
__global__ void __launch_bounds__(64) k_eig_back(EigBatch batch) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const int j = blockIdx.y;
  if (j >= K) return;
  const EigWs w = eig_ws(a);
  const int lane = threadIdx.x;
  const double* xj = w.X + (long long)j * n;
  const double* G = a.G;
  double x[BK_R];
#pragma unroll
  for (int r = 0; r < BK_R; ++r) {
    const int c = lane + 64 * r;
    x[r] = c < n ? xj[c] : 0.0;
  }
  // reflectors in groups of BK_G (k, k-1, ...), the next group's loads issued before
  // this group's arithmetic
  double va[BK_G][BK_R], vb[BK_G][BK_R], ba[BK_G], bb[BK_G];
  auto load = [&](int k0, double (&vv)[BK_G][BK_R], double (&bv)[BK_G]) {
#pragma unroll
    for (int g = 0; g < BK_G; ++g) {
      const int k = k0 - g;
      bv[g] = k >= 0 ? w.beta[k] : 0.0;
#pragma unroll
      for (int r = 0; r < BK_R; ++r) {
        const int c = lane + 64 * r;
        vv[g][r] = (k >= 0 && c > k && c < n) ? G[(long long)k * n + c] : 0.0;
      }
    }
  };
  load(n - 3, va, ba);
  for (int k0 = n - 3; k0 >= 0; k0 -= BK_G) {
    load(k0 - BK_G, vb, bb);
#pragma unroll
    for (int g = 0; g < BK_G; ++g) {
      if (ba[g] != 0.0) {
        double sv = 0.0;
#pragma unroll
        for (int r = 0; r < BK_R; ++r) sv += va[g][r] * x[r];
        for (int off = 32; off > 0; off >>= 1) sv += __shfl_xor(sv, off, 64);
        sv *= ba[g];
#pragma unroll
        for (int r = 0; r < BK_R; ++r) x[r] -= sv * va[g][r];
      }
    }
#pragma unroll
    for (int g = 0; g < BK_G; ++g) {
      ba[g] = bb[g];
#pragma unroll
      for (int r = 0; r < BK_R; ++r) va[g][r] = vb[g][r];
    }
  }
  // sign: the largest-magnitude entry positive (the lowest index on a tie)
  double best = -1.0, bval = 0.0;
  int bi = 0;
#pragma unroll
  for (int r = 0; r < BK_R; ++r) {
    const int c = lane + 64 * r;
    const double av = fabs(x[r]);
    if (c < n && av > best) { best = av; bi = c; bval = x[r]; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    const double ov = __shfl_xor(bval, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; bval = ov; }
  }
  const double sg = bval < 0.0 ? -1.0 : 1.0;
#pragma unroll
  for (int r = 0; r < BK_R; ++r) {
    const int i = lane + 64 * r;
    if (i < n) {
      const double q = sg * x[r];
      const double sw = sqrt(a.wn[i]);
      a.Umax[(long long)i * a.ldu + j] = q / sw;
      a.Bmax[(long long)i * K + j] = q * sw;
    }
  }
}

hipError_t launch_sym_eig(const EigBatch& b, double* lam_scratch, double* vec_scratch, hipStream_t s) {
  int nmax = 0, kmax = 0;
  for (int i = 0; i < b.count; ++i) {
    if (b.m[i].Nn > TDB_NEIG || b.m[i].k > TDB_RCAP || b.m[i].Nn < 1) return hipErrorInvalidValue;
    nmax = b.m[i].Nn > nmax ? b.m[i].Nn : nmax;
    kmax = b.m[i].k > kmax ? b.m[i].k : kmax;
  }
  // enough workgroups that each wave owns a row or two of the largest trailing block;
  // the last TRI_TAIL rows of every mode in one workgroup with the block in LDS
  const int nblk = nmax >= 512 ? 64 : nmax >= 128 ? 32 : 8;
  if (nmax > TDB_NEIG || 4 * nblk * TS_ROWS < nmax) return hipErrorInvalidValue;   // rows per wave in registers
  EigBatch bt = b;
  int kdist = 0;
  for (int i = 0; i < bt.count; ++i) {
    bt.m[i].k0 = bt.m[i].Nn > TRI_TAIL ? bt.m[i].Nn - TRI_TAIL : 0;
    kdist = bt.m[i].k0 > kdist ? bt.m[i].k0 : kdist;
  }
  for (int k = 0; k < kdist; ++k) {
    hipLaunchKernelGGL(k_tri_step, dim3(nblk, bt.count), dim3(256), 0, s, bt, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t tl = ((size_t)TRI_TAIL * TRI_TAIL + (2 + TT_PARTS) * TRI_TAIL) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_tri_tail, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_tail, dim3(bt.count), dim3(TT_THREADS), tl, s, bt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_values, dim3(b.count, kmax + 1), dim3(EV_PTS), 0, s, bt, lam_scratch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int it = 0; it < 3; ++it) {
    hipLaunchKernelGGL(k_eig_solve, dim3(b.count, (kmax + EIG_VPB - 1) / EIG_VPB), dim3(64 * EIG_VPB), 0, s, bt,
                       lam_scratch, vec_scratch, it == 0 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eig_orth, dim3(b.count), dim3(1024), 0, s, bt, lam_scratch, vec_scratch, it == 2 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_eig_back, dim3(b.count, kmax), dim3(64), 0, s, bt);
  return hipGetLastError();
}

}  // namespace tdb
