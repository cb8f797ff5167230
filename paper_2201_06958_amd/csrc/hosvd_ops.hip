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
    const double* pp = partials + (long long)pair * nchunks * 4096 + t;
    int c = 0;
    for (; c + 8 <= nchunks; c += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(long long)(c + u) * 4096];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunks; ++c) s += pp[(long long)c * 4096];
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
    const double e2 = nu2h - sub_energy(a.Cmax, a.caps, r, p, red);
    event = EV_REINIT;
    if (!(sqrt_sum_sq(e2) <= c->eps_th)) {
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
  const double e2 = nu2h - sub_energy(a.Cmax, a.caps, r, p, red);
  if (threadIdx.x == 0) {
    int changed = 0;
    for (int n = 0; n < p; ++n) { changed |= (r[n] != cur[n]); c->ranks[n] = r[n]; }
    c->rank_changed = changed;
    const double er = sqrt_sum_sq(e2);   // NaN stays NaN (non-finite data)
    if (a.mode == DEC_INIT) {
      c->eps = er;
      c->nu = sqrt_sum_sq(nu2h);
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
