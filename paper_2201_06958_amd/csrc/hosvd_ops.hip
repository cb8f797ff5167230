// Device HOSVD for (re)initialisation (Sec. 2.3, 2.5): weighted Gram matrix of each
// mode unfolding, leading eigenpairs of that symmetric matrix (Householder
// tridiagonalisation, bisection on Sturm counts, inverse iteration with
// re-orthogonalisation inside eigenvalue clusters, back-transformation), and the
// rank selection that drives mode addition and removal (eq. (percentage)).
#include "tdb_common.h"
#include "tdb_kernels.h"
#include <math.h>

namespace tdb {

// ---------------------------------------------------------------- weighted Gram
// G = Vt_(n) Vt_(n)^T with Vt = V scaled by sqrt of all weights. Grid: (lower tile
// pairs of 64x64, K-chunks); each block writes a 64x64 partial (unscaled in mode n).
template <typename TV>
__global__ void __launch_bounds__(256) k_gram_partials(const TV* __restrict__ V, HosvdModeArgs m,
                                                       double* __restrict__ partials, long long kchunk,
                                                       int nchunks) {
  __shared__ double XA[16][65];
  __shared__ double XB[16][65];
  __shared__ long long kbase[16];
  __shared__ double kw[16];
  const int pair = blockIdx.x, chunk = blockIdx.y;
  int ti = (int)((sqrt(8.0 * pair + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= pair) ++ti;
  while (ti * (ti + 1) / 2 > pair) --ti;
  const int tj = pair - ti * (ti + 1) / 2;
  const long long K = m.A * m.Bsz;
  const long long k0 = (long long)chunk * kchunk;
  long long k1 = k0 + kchunk;
  if (k1 > K) k1 = K;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const bool kfast = m.Bsz >= 16;
  for (long long kk = k0; kk < k1; kk += 16) {
    if (threadIdx.x < 16) {
      const long long k = kk + threadIdx.x;
      if (k < k1) {
        const long long ai = k / m.Bsz, bi = k - ai * m.Bsz;
        kbase[threadIdx.x] = ai * m.Nn * m.Bsz + bi;
        kw[threadIdx.x] = m.wa[ai] * m.wb[bi];
      } else {
        kbase[threadIdx.x] = -1;
        kw[threadIdx.x] = 0.0;
      }
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      int il, kl;
      if (kfast) { kl = threadIdx.x & 15; il = (threadIdx.x >> 4) + 16 * q; }
      else { il = threadIdx.x & 63; kl = (threadIdx.x >> 6) + 4 * q; }
      const long long gi = (long long)ti * 64 + il, gj = (long long)tj * 64 + il;
      const long long kb = kbase[kl];
      double xa = 0.0, xb = 0.0;
      if (kb >= 0) {
        if (gi < m.Nn) xa = (double)V[kb + gi * m.Bsz] * kw[kl];
        if (gj < m.Nn) xb = (double)V[kb + gj * m.Bsz];
      }
      XA[kl][il] = xa;
      XB[kl][il] = xb;
    }
    __syncthreads();
    for (int kl = 0; kl < 16; ++kl) {
      double a[4], b[4];
      for (int q = 0; q < 4; ++q) {
        a[q] = XA[kl][ty * 4 + q];
        b[q] = XB[kl][tx * 4 + q];
      }
      for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
    }
    __syncthreads();
  }
  double* out = partials + ((long long)pair * nchunks + chunk) * 4096;
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y) out[(ty * 4 + x) * 64 + tx * 4 + y] = acc[x][y];
}

__global__ void __launch_bounds__(256) k_gram_reduce(const double* __restrict__ partials,
                                                     double* __restrict__ G, HosvdModeArgs m,
                                                     int nchunks) {
  const int pair = blockIdx.x;
  int ti = (int)((sqrt(8.0 * pair + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= pair) ++ti;
  while (ti * (ti + 1) / 2 > pair) --ti;
  const int tj = pair - ti * (ti + 1) / 2;
  for (int t = threadIdx.x; t < 4096; t += blockDim.x) {
    const int il = t / 64, jl = t % 64;
    const long long i = (long long)ti * 64 + il, j = (long long)tj * 64 + jl;
    if (i >= m.Nn || j >= m.Nn) continue;
    // a diagonal tile holds both (i, j) and (j, i), whose partial sums differ in rounding
    // (the weight multiplies one operand): only the lower entry writes both, so the
    // result never depends on which write lands last
    if (ti == tj && jl > il) continue;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partials[((long long)pair * nchunks + c) * 4096 + t];
    s *= sqrt(m.wn[i] * m.wn[j]);
    G[i * m.Nn + j] = s;
    G[j * m.Nn + i] = s;
  }
}

template <typename TV>
hipError_t launch_gram_partials(const TV* V, const HosvdModeArgs& m, double* partials, long long kchunk,
                                int nchunks, hipStream_t s) {
  const int nt = (int)((m.Nn + 63) / 64);
  hipLaunchKernelGGL(k_gram_partials<TV>, dim3(nt * (nt + 1) / 2, nchunks), dim3(256), 0, s, V, m,
                     partials, kchunk, nchunks);
  return hipGetLastError();
}
template hipError_t launch_gram_partials<float>(const float*, const HosvdModeArgs&, double*, long long, int,
                                                hipStream_t);
template hipError_t launch_gram_partials<double>(const double*, const HosvdModeArgs&, double*, long long,
                                                 int, hipStream_t);

hipError_t launch_gram_reduce(const double* partials, double* G, const HosvdModeArgs& m, int nchunks,
                              hipStream_t s) {
  const int nt = (int)((m.Nn + 63) / 64);
  hipLaunchKernelGGL(k_gram_reduce, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, partials, G, m, nchunks);
  return hipGetLastError();
}

// ---------------------------------------------------------------- symmetric eigensolver
#define NE TDB_NEIG

__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
  unsigned x = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u);
  x ^= x >> 16; x *= 0x7FEB352Du; x ^= x >> 15; x *= 0x846CA68Bu; x ^= x >> 16;
  return (double)x * (2.0 / 4294967296.0) - 1.0;
}

// Sturm count: number of eigenvalues of the tridiagonal (d, e2 = e^2) below x.
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ void __launch_bounds__(256) k_sym_eig(EigBatch batch) {
  const EigArgs a = batch.m[blockIdx.x];
  __shared__ double d[NE], e[NE], e2[NE], beta[NE], v[NE], pv[NE];
  __shared__ double lu_dl[NE], lu_dd[NE], lu_du[NE], lu_du2[NE], xs[NE];
  __shared__ unsigned char ipiv[NE];
  __shared__ double lam[TDB_RCAP + 1];
  __shared__ double red[16];
  const int n = a.Nn, K = a.k;
  double* G = a.G;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nwav = blockDim.x >> 6;

  // ---- 1. Householder reduction to tridiagonal form; reflector k is stored in row k.
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double ss = 0.0;
    for (int i = tid; i < m; i += blockDim.x) {
      const double x = G[(long long)(k + 1 + i) * n + k];
      v[i] = x;
      ss += x * x;
    }
    ss = block_sum(ss, red);
    const double x0 = v[0];
    double bk = 0.0;
    __syncthreads();
    if (ss > 0.0) {
      const double xn = sqrt(ss);
      const double alpha = x0 > 0.0 ? -xn : xn;
      const double v0 = x0 - alpha;
      const double vtv = ss - x0 * x0 + v0 * v0;
      bk = 2.0 / vtv;
      if (tid == 0) { v[0] = v0; e[k] = alpha; }
    } else if (tid == 0) {
      e[k] = x0;
    }
    if (tid == 0) { d[k] = G[(long long)k * n + k]; beta[k] = bk; }
    __syncthreads();
    for (int i = tid; i < m; i += blockDim.x) G[(long long)k * n + k + 1 + i] = v[i];
    if (bk == 0.0) { __syncthreads(); continue; }
    // pv = bk * A_sub v, one wave per row
    for (int i = wid; i < m; i += nwav) {
      const double* row = G + (long long)(k + 1 + i) * n + (k + 1);
      double s = 0.0;
      for (int j = lane; j < m; j += 64) s += row[j] * v[j];
      s = warp_sum(s);
      if (lane == 0) pv[i] = bk * s;
    }
    __syncthreads();
    double pvv = 0.0;
    for (int i = tid; i < m; i += blockDim.x) pvv += pv[i] * v[i];
    pvv = block_sum(pvv, red);
    const double Kc = 0.5 * bk * pvv;
    for (int i = tid; i < m; i += blockDim.x) pv[i] -= Kc * v[i];     // w
    __syncthreads();
    for (long long t = tid; t < (long long)m * m; t += blockDim.x) {
      const int i = (int)(t / m), j = (int)(t - (long long)i * m);
      G[(long long)(k + 1 + i) * n + (k + 1 + j)] -= v[i] * pv[j] + pv[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = G[(long long)(n - 2) * n + (n - 2)];
      e[n - 2] = G[(long long)(n - 1) * n + (n - 2)];
      beta[n - 2] = 0.0;
    }
    d[n - 1] = G[(long long)(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) e2[i] = e[i] * e[i];
  __syncthreads();

  // ---- 2. leading K+1 eigenvalues by bisection on Sturm counts
  double tn = 0.0, gl = 0.0, gu = 0.0, emax2 = 0.0;
  {
    double lo = 1e300, hi = -1e300, mx = 0.0, me = 0.0;
    for (int i = tid; i < n; i += blockDim.x) {
      const double off = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - off);
      hi = fmax(hi, d[i] + off);
      mx = fmax(mx, fabs(d[i]) + off);
      if (i + 1 < n) me = fmax(me, e2[i]);
    }
    gl = -block_max(-lo, red);
    gu = block_max(hi, red);
    tn = block_max(mx, red);
    emax2 = block_max(me, red);
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  gl -= 4.0 * eps * tn + 2.0 * pivmin;
  gu += 4.0 * eps * tn + 2.0 * pivmin;
  for (int t = tid; t <= K; t += blockDim.x) {
    if (t >= n) { lam[t] = 0.0; continue; }
    const int idx = n - 1 - t;           // ascending index of the t-th largest
    double lo = gl, hi = gu;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
      if (sturm_count(d, e2, n, mid, pivmin) > idx) hi = mid;
      else lo = mid;
    }
    lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();
  for (int t = tid; t <= K; t += blockDim.x) a.sig[t] = t < n ? sqrt(fmax(lam[t], 0.0)) : 0.0;

  // ---- 3. inverse iteration for the K leading eigenvectors (wave 0)
  double* X = a.work;                  // column-major n x K
  const double ortol = 1e-3 * tn;
  const double eps3 = 10.0 * eps * tn;
  if (wid == 0) {
    int cstart = 0;
    double lam_prev = 0.0;
    for (int j = 0; j < K; ++j) {
      double lj = lam[j];
      if (j > 0) {
        if (lam[j - 1] - lj > ortol) cstart = j;
        if (lam_prev - lj < eps3) lj = lam_prev - eps3;   // keep shifts distinct in a cluster
      }
      lam_prev = lj;
      for (int i = lane; i < n; i += 64) xs[i] = hash_unit((unsigned)i, (unsigned)j + 1u);
      if (lane == 0) {
        // LU with partial pivoting of T - lj I
        for (int i = 0; i < n; ++i) {
          lu_dd[i] = d[i] - lj;
          lu_dl[i] = (i + 1 < n) ? e[i] : 0.0;
          lu_du[i] = (i + 1 < n) ? e[i] : 0.0;
          lu_du2[i] = 0.0;
        }
        const double ptiny = eps * tn + pivmin;
        for (int i = 0; i + 1 < n; ++i) {
          if (fabs(lu_dd[i]) >= fabs(lu_dl[i])) {
            ipiv[i] = 0;
            if (lu_dd[i] == 0.0) lu_dd[i] = ptiny;
            const double f = lu_dl[i] / lu_dd[i];
            lu_dl[i] = f;
            lu_dd[i + 1] -= f * lu_du[i];
          } else {
            ipiv[i] = 1;
            const double f = lu_dd[i] / lu_dl[i];
            lu_dd[i] = lu_dl[i];
            lu_dl[i] = f;
            const double tmp = lu_du[i];
            lu_du[i] = lu_dd[i + 1];
            lu_dd[i + 1] = tmp - f * lu_dd[i + 1];
            if (i + 2 < n) {
              lu_du2[i] = lu_du[i + 1];
              lu_du[i + 1] = -f * lu_du[i + 1];
            }
          }
        }
        if (lu_dd[n - 1] == 0.0) lu_dd[n - 1] = ptiny;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      for (int it = 0; it < 3; ++it) {
        if (lane == 0) {
          for (int i = 0; i + 1 < n; ++i) {
            if (ipiv[i] == 0) {
              xs[i + 1] -= lu_dl[i] * xs[i];
            } else {
              const double tmp = xs[i];
              xs[i] = xs[i + 1];
              xs[i + 1] = tmp - lu_dl[i] * xs[i];
            }
          }
          xs[n - 1] /= lu_dd[n - 1];
          if (n >= 2) xs[n - 2] = (xs[n - 2] - lu_du[n - 2] * xs[n - 1]) / lu_dd[n - 2];
          for (int i = n - 3; i >= 0; --i)
            xs[i] = (xs[i] - lu_du[i] * xs[i + 1] - lu_du2[i] * xs[i + 2]) / lu_dd[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // scale to unit max-norm first (avoids overflow in the dot products)
        double mx = 0.0;
        for (int i = lane; i < n; i += 64) mx = fmax(mx, fabs(xs[i]));
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
        for (int i = lane; i < n; i += 64) xs[i] *= sc;
        for (int q = cstart; q < j; ++q) {
          const double* xq = X + (long long)q * n;
          double dt = 0.0;
          for (int i = lane; i < n; i += 64) dt += xs[i] * xq[i];
          for (int off = 32; off > 0; off >>= 1) dt += __shfl_xor(dt, off, 64);
          for (int i = lane; i < n; i += 64) xs[i] -= dt * xq[i];
        }
        double nr = 0.0;
        for (int i = lane; i < n; i += 64) nr += xs[i] * xs[i];
        for (int off = 32; off > 0; off >>= 1) nr += __shfl_xor(nr, off, 64);
        const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
        for (int i = lane; i < n; i += 64) xs[i] *= inv;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      }
      double* xj = X + (long long)j * n;
      for (int i = lane; i < n; i += 64) xj[i] = xs[i];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
  }
  __syncthreads();

  // ---- 4. back-transformation x <- H_0 H_1 ... H_{n-3} x, one wave per vector
  for (int j = wid; j < K; j += nwav) {
    double* xj = X + (long long)j * n;
    for (int k = n - 3; k >= 0; --k) {
      const double bk = beta[k];
      if (bk == 0.0) continue;
      const int m = n - k - 1;
      const double* vk = G + (long long)k * n + k + 1;
      double s = 0.0;
      for (int i = lane; i < m; i += 64) s += vk[i] * xj[k + 1 + i];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      s *= bk;
      for (int i = lane; i < m; i += 64) xj[k + 1 + i] -= s * vk[i];
    }
    // sign convention: largest-magnitude entry positive (lowest index on a tie)
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
}

hipError_t launch_sym_eig(const EigBatch& b, hipStream_t s) {
  for (int i = 0; i < b.count; ++i)
    if (b.m[i].Nn > TDB_NEIG || b.m[i].k > TDB_RCAP || b.m[i].Nn < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sym_eig, dim3(b.count), dim3(256), 0, s, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------- rank selection
struct SelShared {
  int r[TDB_P];
  int stop;
};

__device__ double sub_energy(const double* Cmax, const int* caps, const int* r, int p, double* red) {
  long long tot = 1;
  for (int k = 0; k < p; ++k) tot *= r[k];
  double s = 0.0;
  for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
    long long rem = t, idx = 0, mul = 1;
    long long id[TDB_P];
    for (int k = p - 1; k >= 0; --k) { id[k] = rem % r[k]; rem /= r[k]; }
    for (int k = p - 1; k >= 0; --k) { idx += id[k] * mul; mul *= caps[k]; }
    const double c = Cmax[idx];
    s += c * c;
  }
  return block_sum(s, red);
}

__device__ bool valid_ranks(const int* r, int p) {
  for (int n = 0; n < p; ++n) {
    long long o = 1;
    for (int k = 0; k < p; ++k) if (k != n) o *= r[k];
    if (r[n] > o) return false;
  }
  return true;
}

__device__ bool can_grow(const SelectArgs& a, const int* r, int n) {
  return r[n] < a.caps[n] && a.sig[n][r[n]] > TDB_SIGMA_FLOOR * a.sig[n][0];
}

// Grow modes until every r_n <= prod of the others (thread 0 edits sh.r).
__device__ void repair(const SelectArgs& a, int* r) {
  if (threadIdx.x == 0) {
    for (int guard = 0; guard < 100000 && !valid_ranks(r, a.p); ++guard) {
      int bad = 0;
      long long ob = 1;
      for (int n = 0; n < a.p; ++n) {
        long long o = 1;
        for (int k = 0; k < a.p; ++k) if (k != n) o *= r[k];
        if (r[n] > o) { bad = n; ob = o; break; }
      }
      int best = -1;
      for (int m = 0; m < a.p; ++m) {
        if (m == bad || !can_grow(a, r, m)) continue;
        if (best < 0 || a.sig[m][r[m]] > a.sig[best][r[best]]) best = m;
      }
      if (best < 0) r[bad] = (int)ob;
      else r[best] += 1;
    }
  }
  __syncthreads();
}

// Greedy rule: from r, grow the mode with the largest next singular value while the
// exact truncation error nu2 - ||Cmax[:r]||^2 exceeds the budget; then repair.
__device__ void greedy(const SelectArgs& a, int* r, double nu2, double B, double* red, int* stop) {
  while (true) {
    const double e2 = fmax(nu2 - sub_energy(a.Cmax, a.caps, r, a.p, red), 0.0);
    if (threadIdx.x == 0) {
      *stop = 1;
      if (e2 > B) {
        int best = -1;
        for (int n = 0; n < a.p; ++n) {
          if (!can_grow(a, r, n)) continue;
          if (best < 0 || a.sig[n][r[n]] > a.sig[best][r[best]]) best = n;
        }
        if (best >= 0) { r[best] += 1; *stop = 0; }
      }
    }
    __syncthreads();
    if (*stop) break;
    __syncthreads();
  }
  repair(a, r);
}

__global__ void __launch_bounds__(256) k_rank_select(SelectArgs a, CtrlState* c) {
  __shared__ int r[TDB_P], rr[TDB_P], cur[TDB_P];
  __shared__ int stop, doit;
  __shared__ double red[16];
  const int p = a.p;
  const double nu2h = *a.nu2h;
  const double nu2b = (a.mode == DEC_INIT) ? nu2h : c->nu2;
  const double B = c->gamma_th > 0.0 ? (1.0 - c->gamma_th / 100.0) * nu2b : 0.25 * c->eps_th * c->eps_th;
  if (threadIdx.x == 0) {
    for (int n = 0; n < p; ++n) cur[n] = c->ranks[n];
    doit = 1;
  }
  __syncthreads();
  int event = 0;
  if (a.mode == DEC_INIT) {
    bool given = false;
    for (int n = 0; n < p; ++n) given = given || a.rank_init[n] > 0;
    if (given) {
      if (threadIdx.x == 0) {
        for (int n = 0; n < p; ++n) {
          int v = a.rank_init[n] < 1 ? 1 : a.rank_init[n];
          r[n] = v > a.caps[n] ? a.caps[n] : v;
        }
        for (int guard = 0; guard < 100000 && !valid_ranks(r, p); ++guard) {
          for (int n = 0; n < p; ++n) {
            long long o = 1;
            for (int k = 0; k < p; ++k) if (k != n) o *= r[k];
            if (r[n] > o) { r[n] -= 1; break; }
          }
        }
      }
      __syncthreads();
    } else {
      if (threadIdx.x == 0) for (int n = 0; n < p; ++n) r[n] = 1;
      __syncthreads();
      greedy(a, r, nu2h, B, red, &stop);
    }
  } else if (a.mode == DEC_ADD) {
    if (threadIdx.x == 0) for (int n = 0; n < p; ++n) r[n] = cur[n];
    __syncthreads();
    const double e2 = fmax(nu2h - sub_energy(a.Cmax, a.caps, r, p, red), 0.0);
    event = EV_REINIT;
    if (sqrt(e2) > c->eps_th) {
      greedy(a, r, nu2h, B, red, &stop);
      bool same = true;
      for (int n = 0; n < p; ++n) same = same && r[n] == cur[n];
      if (!same) event = EV_ADD;
    }
  } else if (a.mode == DEC_REMOVE) {
    if (threadIdx.x == 0) for (int n = 0; n < p; ++n) rr[n] = 1;
    __syncthreads();
    greedy(a, rr, nu2h, B, red, &stop);
    if (threadIdx.x == 0) for (int n = 0; n < p; ++n) r[n] = rr[n] < cur[n] ? rr[n] : cur[n];
    __syncthreads();
    repair(a, r);
    bool same = true;
    for (int n = 0; n < p; ++n) same = same && r[n] == cur[n];
    if (same) {
      if (threadIdx.x == 0) { c->wcount = 0; c->whead = 0; doit = 0; }
      __syncthreads();
    } else {
      event = EV_REMOVE;
    }
  } else {   // DEC_NUMERIC: restart at ranks no larger than the data's numerical rank
    if (threadIdx.x == 0) {
      for (int n = 0; n < p; ++n) {
        int cnt = 0;
        for (int i = 0; i < a.caps[n]; ++i) cnt += (a.sig[n][i] > TDB_SIGMA_FLOOR * a.sig[n][0]) ? 1 : 0;
        if (cnt < 1) cnt = 1;
        r[n] = cur[n] < cnt ? cur[n] : cnt;
        rr[n] = 1;
      }
    }
    __syncthreads();
    if (c->adaptive) {
      greedy(a, rr, nu2h, B, red, &stop);
      if (threadIdx.x == 0) for (int n = 0; n < p; ++n) r[n] = rr[n] < r[n] ? rr[n] : r[n];
      __syncthreads();
    }
    repair(a, r);
    event = EV_NUMERIC;
  }
  __syncthreads();
  if (!doit) return;
  // truncate the HOSVD at r: C0 = Cmax[:r], U0 = Umax[:, :r]
  long long tot = 1;
  for (int k = 0; k < p; ++k) tot *= r[k];
  for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
    long long rem = t, idx = 0, mul = 1;
    long long id[TDB_P];
    for (int k = p - 1; k >= 0; --k) { id[k] = rem % r[k]; rem /= r[k]; }
    for (int k = p - 1; k >= 0; --k) { idx += id[k] * mul; mul *= a.caps[k]; }
    a.C0[t] = a.Cmax[idx];
  }
  for (int n = 0; n < p; ++n) {
    const long long tot_u = a.N[n] * a.ldU[n];
    for (long long t = threadIdx.x; t < tot_u; t += blockDim.x) a.U0[n][t] = a.Umax[n][t];
  }
  const double e2 = fmax(nu2h - sub_energy(a.Cmax, a.caps, r, p, red), 0.0);
  if (threadIdx.x == 0) {
    int changed = 0;
    for (int n = 0; n < p; ++n) { changed |= (r[n] != cur[n]); c->ranks[n] = r[n]; }
    c->rank_changed = changed;
    const double er = sqrt(e2);
    if (a.mode == DEC_INIT) {
      c->eps = er;
      c->nu = sqrt(nu2h);
      c->eps_after = __builtin_nan("");
      c->unmet = 0;
      c->eps_trig = c->eps_th;
      c->event = 0;
    } else {
      c->eps_after = er;
      c->event = event;
      c->n_events[event] += 1;
      if (er > c->eps_th) { c->unmet = 1; c->eps_trig = 2.0 * er; }
      else { c->unmet = 0; c->eps_trig = c->eps_th; }
    }
    c->wcount = 0;
    c->whead = 0;
    c->numeric = 0;
  }
}

hipError_t launch_rank_select(const SelectArgs& a, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_rank_select, dim3(1), dim3(256), 0, s, a, ctrl);
  return hipGetLastError();
}

// trace of an n x n matrix into *out (used as ||V||_W^2 = trace of any mode's Gram)
__global__ void __launch_bounds__(256) k_trace(const double* G, long long n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += G[i * n + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

hipError_t launch_trace(const double* G, long long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, G, n, out);
  return hipGetLastError();
}

}  // namespace tdb
