// Leading eigenpairs of the weighted mode Gram matrices of the HOSVD (Sec. 2.3):
// Householder reduction to tridiagonal form spread over many workgroups (one launch
// per reflector), bisection on Sturm counts for the leading K+1 eigenvalues, inverse
// iteration for the K leading eigenvectors (clusters of close eigenvalues
// orthogonalised within one wave), back-transformation by the stored reflectors and
// a sign convention (largest-magnitude entry positive, lowest index on a tie).
//
// Reflector k (k = 0..n-3) acts on indices k+1..n-1; it is stored in row k of G
// (entries k+1..n-1), its coefficient in beta[k]. Launch k applies the rank-2 update
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

// Per-mode workspace (after the K eigenvector columns): d, e, beta, p0, p1.
struct EigWs {
  double *X, *d, *e, *beta, *p[2];
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
  return w;
}

__global__ void __launch_bounds__(256) k_tri_step(EigBatch batch, int k) {
  const EigArgs a = batch.m[blockIdx.y];
  const int n = a.Nn;
  if (k + 2 >= n) return;
  const EigWs w = eig_ws(a);
  double* G = a.G;
  __shared__ double vp[NE], wp[NE], v[NE];
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nblk = gridDim.x;
  // the pending update of reflector k-1 (acting on indices k..n-1)
  const double bp = k > 0 ? w.beta[k - 1] : 0.0;
  const int mp = n - k;
  if (bp != 0.0) {
    const double* pp = ((k - 1) & 1) ? w.p[1] : w.p[0];
    double pvv = 0.0;
    for (int i = tid; i < mp; i += blockDim.x) {
      const double vi = G[(long long)(k - 1) * n + k + i];
      vp[i] = vi;
      pvv += pp[k + i] * vi;
    }
    pvv = block_sum(pvv, red);
    const double Kc = 0.5 * bp * pvv;
    for (int i = tid; i < mp; i += blockDim.x) wp[i] = pp[k + i] - Kc * vp[i];
    __syncthreads();
  }
  // column k below the diagonal and the diagonal entry of the updated matrix
  const int m = n - k - 1;
  double ss = 0.0;
  for (int i = tid; i < m; i += blockDim.x) {
    double x = G[(long long)(k + 1 + i) * n + k];
    if (bp != 0.0) x -= vp[1 + i] * wp[0] + wp[1 + i] * vp[0];
    v[i] = x;
    ss += x * x;
  }
  ss = block_sum(ss, red);
  const double x0 = v[0];
  double dk = G[(long long)k * n + k];
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
  // rows of this workgroup: k+1+i for i = blockIdx.x, blockIdx.x + nblk, ...; one wave per row
  double* pk = (k & 1) ? w.p[1] : w.p[0];
  for (int i = blockIdx.x + nblk * wid; i < m; i += nblk * 4) {
    double* row = G + (long long)(k + 1 + i) * n + (k + 1);
    double s = 0.0;
    if (bp != 0.0) {
      const double vr = vp[1 + i], wr = wp[1 + i];
      for (int j = lane; j < m; j += 64) {
        const double x = row[j] - (vr * wp[1 + j] + wr * vp[1 + j]);
        row[j] = x;
        s += x * v[j];
      }
    } else {
      for (int j = lane; j < m; j += 64) s += row[j] * v[j];
    }
    s = warp_sum(s);
    if (lane == 0) pk[k + 1 + i] = bk * s;
  }
  if (blockIdx.x == 0) {
    for (int i = tid; i < m; i += blockDim.x) G[(long long)k * n + k + 1 + i] = v[i];
    if (tid == 0) {
      w.d[k] = dk;
      w.e[k] = ek;
      w.beta[k] = bk;
    }
  }
}

// The last 2 x 2 block (with the pending update of reflector n-3), and e[n-1] = 0.
__global__ void __launch_bounds__(64) k_tri_final(EigBatch batch) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn;
  const EigWs w = eig_ws(a);
  const double* G = a.G;
  if (threadIdx.x != 0) return;
  if (n == 1) {
    w.d[0] = G[0];
    w.e[0] = 0.0;
    return;
  }
  const int k = n - 2;   // first index of the block
  double a00 = G[(long long)k * n + k], a10 = G[(long long)(k + 1) * n + k], a11 = G[(long long)(k + 1) * n + k + 1];
  const double bp = k > 0 ? w.beta[k - 1] : 0.0;
  if (bp != 0.0) {
    const double* pp = ((k - 1) & 1) ? w.p[1] : w.p[0];
    const double v0 = G[(long long)(k - 1) * n + k], v1 = G[(long long)(k - 1) * n + k + 1];
    const double Kc = 0.5 * bp * (pp[k] * v0 + pp[k + 1] * v1);
    const double w0 = pp[k] - Kc * v0, w1 = pp[k + 1] - Kc * v1;
    a00 -= v0 * w0 + w0 * v0;
    a10 -= v1 * w0 + w1 * v0;
    a11 -= v1 * w1 + w1 * v1;
  }
  w.d[k] = a00;
  w.e[k] = a10;
  w.beta[k] = 0.0;
  w.d[k + 1] = a11;
  w.e[k + 1] = 0.0;
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

// One block per mode: the K+1 leading eigenvalues by multisection on Sturm counts
// (8 lanes per eigenvalue evaluate 8 interior points of its interval, which shrinks
// 9-fold per round), the singular values sqrt(max(lambda, 0)), and the Gershgorin scale.
__global__ void __launch_bounds__(576) k_eig_values(EigBatch batch, double* lam_out) {
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
  const int t = threadIdx.x >> 3, sub = threadIdx.x & 7;   // eigenvalue slot, lane in the group
  double l = gl, h = gu;
  const bool live = t <= K && t < n;
  const int idx = n - 1 - t;                                  // ascending index of the t-th largest
  for (int it = 0; it < 80; ++it) {
    // converged to the accuracy of the eigenvalues themselves: a few ulps of the matrix
    // scale (an eigenvalue below that is numerically zero)
    bool done = !live || h - l <= fmax(2.0 * eps * fmax(fabs(l), fabs(h)), 4.0 * eps * tn) + pivmin;
    // the whole wave leaves together once every group in it has converged
    if (__all(done)) break;
    const double x = l + (double)(sub + 1) * ((h - l) / 9.0);
    const int c = live && !done ? sturm_count2(d, e2, n, x, pivmin) : 0;
    // first point whose count exceeds idx bounds the eigenvalue from above
    const unsigned long long above = __ballot(c > idx);
    const int base = (threadIdx.x & 63) & ~7;
    const unsigned grp = (unsigned)((above >> base) & 0xffull);
    if (live && !done) {
      const int first = grp ? __builtin_ctz(grp) : 8;     // points 0..7; 8: above all
      const double nl = first == 0 ? l : l + (double)first * ((h - l) / 9.0);
      const double nh = first == 8 ? h : l + (double)(first + 1) * ((h - l) / 9.0);
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
  if (threadIdx.x == 0) lam[TDB_RCAP + 1] = tn;
}

// Inverse iteration for the K leading eigenvectors, all at once: one block per mode.
// Vector j is shifted by its eigenvalue (shifts inside a cluster kept eps3 apart);
// lane j of the first wave factors T - shift_j I and solves with it (partial
// pivoting); after every solve round the whole block orthonormalises the vectors in
// index order, each against the earlier members of its cluster (a cluster starts where
// the gap to the previous eigenvalue exceeds 1e-3 of the matrix scale), so every
// vector keeps the direction of its own eigenvalue. Vectors live interleaved
// (entry i of vector j at i*64 + j) in a global workspace, as do the LU factors.
__global__ void __launch_bounds__(256) k_eig_vectors(EigBatch batch, const double* lam_in, double* scratch) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const EigWs w = eig_ws(a);
  const double* lam = lam_in + (long long)blockIdx.x * (TDB_RCAP + 2);
  const double tn = lam[TDB_RCAP + 1];
  double* xb = scratch + (long long)blockIdx.x * NE * 64 * 5;
  double* dd = xb + NE * 64;
  double* dl = dd + NE * 64;
  double* du = dl + NE * 64;
  double* du2 = du + NE * 64;
  __shared__ double sh[TDB_RCAP], part[4][TDB_RCAP], red[16], dots[TDB_RCAP], xj[NE];
  __shared__ int cend[TDB_RCAP];
  __shared__ unsigned long long pivbits[NE];   // bit j: row swap of vector j at step i
  const int tid = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  double me = 0.0;
  for (int i = tid; i + 1 < n; i += blockDim.x) me = fmax(me, w.e[i] * w.e[i]);
  me = block_max(me, red);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, me);
  const double ortol = 1e-3 * tn;
  const double eps3 = 10.0 * eps * tn;
  if (tid == 0) {
    double lam_prev = 0.0;
    int cs = 0;
    for (int j = 0; j < K; ++j) {
      double lj = lam[j];
      if (j == 0 || lam[j - 1] - lj > ortol) {
        for (int q = cs; q < j; ++q) cend[q] = j;
        cs = j;
      } else if (lam_prev - lj < eps3) {
        lj = lam_prev - eps3;   // keep shifts distinct in a cluster
      }
      lam_prev = lj;
      sh[j] = lj;
    }
    for (int q = cs; q < K; ++q) cend[q] = K;
  }
  for (int i = tid; i < n; i += blockDim.x) pivbits[i] = 0ull;
  __syncthreads();
  const double ptiny = eps * tn + pivmin;
  // factor and start vector: lane j of the first wave
  if (tid < K) {
    const int j = tid;
    const double lj = sh[j];
    for (int i = 0; i < n; ++i) {
      dd[i * 64 + j] = w.d[i] - lj;
      dl[i * 64 + j] = (i + 1 < n) ? w.e[i] : 0.0;
      du[i * 64 + j] = (i + 1 < n) ? w.e[i] : 0.0;
      du2[i * 64 + j] = 0.0;
      xb[i * 64 + j] = hash_unit2((unsigned)i, (unsigned)j + 1u);
    }
    // the running pivot row (cd, cu) and the next row's original entries are carried in
    // registers, so each step's loads do not wait for the previous step's stores
    // (rows are taken in chunks of EC: a chunk's loads are all issued before any of its
    // stores, so a chunk costs one memory round trip rather than one per row)
    double cd = dd[j], cu = du[j];
    for (int i0 = 0; i0 + 1 < n; i0 += EC) {
      double li_[EC], dn_[EC], un_[EC];
#pragma unroll
      for (int u = 0; u < EC; ++u) {
        const int i = min(i0 + u, n - 2);
        li_[u] = dl[i * 64 + j];
        dn_[u] = dd[(i + 1) * 64 + j];
        un_[u] = (i + 2 < n) ? du[(i + 1) * 64 + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < EC; ++u) {
        const int i = i0 + u;
        if (i + 1 >= n) break;
        const double li = li_[u], dn = dn_[u], un = un_[u];
        if (fabs(cd) >= fabs(li)) {
          if (cd == 0.0) cd = ptiny;
          const double f = li / cd;
          dd[i * 64 + j] = cd;
          dl[i * 64 + j] = f;
          du[i * 64 + j] = cu;
          cd = dn - f * cu;
          cu = un;
        } else {
          atomicOr(&pivbits[i], 1ull << j);
          const double f = cd / li;
          dd[i * 64 + j] = li;
          dl[i * 64 + j] = f;
          du[i * 64 + j] = dn;
          cd = cu - f * dn;
          if (i + 2 < n) {
            du2[i * 64 + j] = un;
            cu = -f * un;
          } else {
            cu = 0.0;
          }
        }
      }
    }
    dd[(n - 1) * 64 + j] = cd;
    if (dd[(n - 1) * 64 + j] == 0.0) dd[(n - 1) * 64 + j] = ptiny;
  }
  __syncthreads();
  const int qs = tid & 63, ig = tid >> 6;   // (vector slot, row group) of the block-wide passes
  for (int it = 0; it < 3; ++it) {
    if (tid < K) {
      const int j = tid;
      const unsigned long long bit = 1ull << j;
      // forward elimination with the row interchanges, the running entry in a register
      double cur = xb[j];
      for (int i0 = 0; i0 + 1 < n; i0 += EC) {
        double nx_[EC], l_[EC];
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = min(i0 + u, n - 2);
          nx_[u] = xb[(i + 1) * 64 + j];
          l_[u] = dl[i * 64 + j];
        }
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = i0 + u;
          if (i + 1 >= n) break;
          const double nx = nx_[u], l = l_[u];
          if (!(pivbits[i] & bit)) {
            xb[i * 64 + j] = cur;
            cur = nx - l * cur;
          } else {
            xb[i * 64 + j] = nx;
            cur = cur - l * nx;
          }
        }
      }
      // back substitution, the two later entries in registers
      double x1 = cur / dd[(n - 1) * 64 + j];
      xb[(n - 1) * 64 + j] = x1;
      double x2 = 0.0;
      if (n >= 2) {
        const double x0 = (xb[(n - 2) * 64 + j] - du[(n - 2) * 64 + j] * x1) / dd[(n - 2) * 64 + j];
        xb[(n - 2) * 64 + j] = x0;
        x2 = x1;
        x1 = x0;
      }
      for (int i0 = n - 3; i0 >= 0; i0 -= EC) {
        double b_[EC], u1_[EC], u2_[EC], d_[EC];
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = max(i0 - u, 0);
          b_[u] = xb[i * 64 + j];
          u1_[u] = du[i * 64 + j];
          u2_[u] = du2[i * 64 + j];
          d_[u] = dd[i * 64 + j];
        }
#pragma unroll
        for (int u = 0; u < EC; ++u) {
          const int i = i0 - u;
          if (i < 0) break;
          const double x0 = (b_[u] - u1_[u] * x1 - u2_[u] * x2) / d_[u];
          xb[i * 64 + j] = x0;
          x2 = x1;
          x1 = x0;
        }
      }
      // scale to unit max-norm (avoids overflow in the dot products)
      double mx = 0.0;
      for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(xb[i * 64 + j]));
      const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
      for (int i = 0; i < n; ++i) xb[i * 64 + j] *= sc;
    }
    __syncthreads();
    // orthonormalise in index order within clusters (vector j staged in LDS; each
    // thread's rows are loaded in batches of 8 before any of them is updated)
    for (int j = 0; j < K; ++j) {
      double nr = 0.0;
      for (int i = tid; i < n; i += blockDim.x) {
        const double x = xb[i * 64 + j];
        xj[i] = x;
        nr += x * x;
      }
      nr = block_sum(nr, red);
      const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
      for (int i = tid; i < n; i += blockDim.x) {
        const double x = xj[i] * inv;
        xj[i] = x;
        xb[i * 64 + j] = x;
      }
      __syncthreads();
      const int ce = cend[j];
      if (ce <= j + 1) continue;
      const int q = j + 1 + qs;
      const bool act = q < ce;
      double pd = 0.0;
      if (act) {
        for (int i0 = ig; i0 < n; i0 += 32) {
          double v8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + 4 * u;
            v8[u] = i < n ? xb[i * 64 + q] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + 4 * u;
            if (i < n) pd += v8[u] * xj[i];
          }
        }
      }
      part[ig][qs] = pd;
      __syncthreads();
      if (tid < 64) dots[tid] = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
      __syncthreads();
      if (act) {
        const double dq = dots[qs];
        for (int i0 = ig; i0 < n; i0 += 32) {
          double v8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + 4 * u;
            v8[u] = i < n ? xb[i * 64 + q] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + 4 * u;
            if (i < n) xb[i * 64 + q] = v8[u] - dq * xj[i];
          }
        }
      }
      __syncthreads();
    }
  }
  // out to the column-major eigenvector block
  for (long long t = tid; t < (long long)n * K; t += blockDim.x) {
    const int j = (int)(t / n), i = (int)(t - (long long)j * n);
    w.X[t] = xb[i * 64 + j];
  }
}

// Back-transformation x <- H_0 H_1 ... H_{n-3} x and the sign convention; grid (mode,
// vector), one wave per vector.
__global__ void __launch_bounds__(64) k_eig_back(EigBatch batch) {
  const EigArgs a = batch.m[blockIdx.x];
  const int n = a.Nn, K = a.k;
  const int j = blockIdx.y;
  if (j >= K) return;
  const EigWs w = eig_ws(a);
  const int lane = threadIdx.x;
  double* xj = w.X + (long long)j * n;
  const double* G = a.G;
  for (int k = n - 3; k >= 0; --k) {
    const double bk = w.beta[k];
    if (bk == 0.0) continue;
    const int m = n - k - 1;
    const double* vk = G + (long long)k * n + k + 1;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += vk[i] * xj[k + 1 + i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    s *= bk;
    for (int i = lane; i < m; i += 64) xj[k + 1 + i] -= s * vk[i];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
  double best = -1.0;
  int bi = 0;
  for (int i = lane; i < n; i += 64) {
    const double av = fabs(xj[i]);
    if (av > best) { best = av; bi = i; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  const double sg = xj[bi] < 0.0 ? -1.0 : 1.0;
  for (int i = lane; i < n; i += 64) {
    const double q = sg * xj[i];
    const double sw = sqrt(a.wn[i]);
    a.Umax[(long long)i * a.ldu + j] = q / sw;
    a.Bmax[(long long)i * K + j] = q * sw;
  }
}

hipError_t launch_sym_eig(const EigBatch& b, double* lam_scratch, double* vec_scratch, hipStream_t s) {
  int nmax = 0, kmax = 0;
  for (int i = 0; i < b.count; ++i) {
    if (b.m[i].Nn > TDB_NEIG || b.m[i].k > TDB_RCAP || b.m[i].Nn < 1) return hipErrorInvalidValue;
    nmax = b.m[i].Nn > nmax ? b.m[i].Nn : nmax;
    kmax = b.m[i].k > kmax ? b.m[i].k : kmax;
  }
  // enough workgroups that each wave owns a row or two of the largest trailing block
  const int nblk = nmax >= 512 ? 64 : nmax >= 128 ? 32 : 8;
  for (int k = 0; k + 2 < nmax; ++k) {
    hipLaunchKernelGGL(k_tri_step, dim3(nblk, b.count), dim3(256), 0, s, b, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tri_final, dim3(b.count), dim3(64), 0, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_values, dim3(b.count), dim3(576), 0, s, b, lam_scratch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_vectors, dim3(b.count), dim3(256), 0, s, b, lam_scratch, vec_scratch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eig_back, dim3(b.count, kmax), dim3(64), 0, s, b);
  return hipGetLastError();
}

}  // namespace tdb
