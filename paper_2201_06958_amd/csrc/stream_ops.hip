// Bulk passes over S-sized tensors for the plain path: generic n-mode products (the
// chain of tensor-times-matrix projections of the data difference, and the
// reconstruction), the fold of a partial projection with the core pseudo-inverse,
// and the weighted error / norm reduction (eq. (error)).
#include "tdb_common.h"
#include "tdb_kernels.h"

namespace tdb {

template <typename TX, typename TC, typename TY>
__global__ void __launch_bounds__(256) k_ttm(const TX* __restrict__ X, const TX* __restrict__ X0,
                                             TY* __restrict__ Y, const TC* __restrict__ M,
                                             long long ms_i, long long ms_o, long long A, int Nin,
                                             int Nout, long long Bsz) {
  const long long total = A * (long long)Nout * Bsz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const long long b = idx % Bsz;
    const long long t = idx / Bsz;
    const int o = (int)(t % Nout);
    const long long a = t / Nout;
    const TX* xp = X + a * (long long)Nin * Bsz + b;
    const TC* mp = M + (long long)o * ms_o;
    TC acc = (TC)0;
    if (X0) {
      const TX* x0p = X0 + a * (long long)Nin * Bsz + b;
      for (int i = 0; i < Nin; ++i)
        acc += mp[(long long)i * ms_i] * ((TC)xp[(long long)i * Bsz] - (TC)x0p[(long long)i * Bsz]);
    } else {
      for (int i = 0; i < Nin; ++i) acc += mp[(long long)i * ms_i] * (TC)xp[(long long)i * Bsz];
    }
    Y[idx] = (TY)acc;
  }
}

template <typename TX, typename TC, typename TY>
hipError_t launch_ttm(const TX* X, const TX* X0, TY* Y, const TC* M, long long ms_i, long long ms_o,
                      long long A, int Nin, int Nout, long long Bsz, hipStream_t s) {
  const long long total = A * (long long)Nout * Bsz;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_ttm<TX, TC, TY>), dim3((unsigned)blocks), dim3(256), 0, s, X, X0, Y, M, ms_i,
                     ms_o, A, Nin, Nout, Bsz);
  return hipGetLastError();
}

#define TTM_INST(TX, TC, TY)                                                                   \
  template hipError_t launch_ttm<TX, TC, TY>(const TX*, const TX*, TY*, const TC*, long long,   \
                                             long long, long long, int, int, long long, hipStream_t);
TTM_INST(double, double, double)
TTM_INST(float, double, double)
TTM_INST(float, float, float)
TTM_INST(float, float, double)
TTM_INST(double, float, float)

// H[i, a] = sum_col F_(n)[i, col] P[col, a]; F has dims (outer, Nn, inner) C-ordered
// and its mode-n unfolding enumerates (o, in) with in fastest, like the core's.
// One block per row i: thread t takes output a = t % rn and every G-th column (G =
// blockDim / rn slices, columns in increasing order within a slice); the slices are
// added in slice order, so the sum's order is fixed.
template <typename T>
__global__ void __launch_bounds__(256) k_fold_h(const T* __restrict__ F, const T* __restrict__ P,
                                                double* __restrict__ H, long long Nn, int rn,
                                                long long outer, long long inner) {
  __shared__ double part[256];
  const int G = (int)blockDim.x / rn;
  const int t = threadIdx.x, a = t % rn, g = t / rn;
  const long long R = outer * inner;
  for (long long i = blockIdx.x; i < Nn; i += gridDim.x) {
    double acc = 0.0;
    if (g < G) {
      for (long long c = g; c < R; c += G) {
        const long long o = c / inner, in = c - o * inner;
        acc += (double)F[(o * Nn + i) * inner + in] * (double)P[c * rn + a];
      }
    }
    part[t] = acc;
    __syncthreads();
    if (t < rn) {
      double s = 0.0;
      for (int q = 0; q < G; ++q) s += part[q * rn + t];
      H[i * rn + t] = s;
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_fold_h(const T* F, const T* P, double* H, long long Nn, int rn, long long outer,
                         long long inner, hipStream_t s) {
  long long blocks = Nn;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fold_h<T>, dim3((unsigned)blocks), dim3(256), 0, s, F, P, H, Nn, rn, outer, inner);
  return hipGetLastError();
}
template hipError_t launch_fold_h<float>(const float*, const float*, double*, long long, int, long long,
                                         long long, hipStream_t);
template hipError_t launch_fold_h<double>(const double*, const double*, double*, long long, int,
                                          long long, long long, hipStream_t);

struct WPtrs {
  const double* w[TDB_P];
  long long N[TDB_P];
  int p;
};

template <typename TV, typename TR>
__global__ void __launch_bounds__(256) k_err_partials(const TV* __restrict__ V, const TR* __restrict__ R,
                                                      WPtrs wp, long long total, double* partials) {
  __shared__ double red[16];
  double se = 0.0, sv = 0.0;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    long long rem = idx;
    double w = 1.0;
    for (int k = wp.p - 1; k >= 0; --k) {
      const long long ik = rem % wp.N[k];
      rem /= wp.N[k];
      w *= wp.w[k][ik];
    }
    const double v = (double)V[idx];
    const double e = (double)((TR)V[idx] - R[idx]);
    se += w * e * e;
    sv += w * v * v;
  }
  se = block_sum(se, red);
  sv = block_sum(sv, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = se;
    partials[2 * blockIdx.x + 1] = sv;
  }
}

template <typename TV, typename TR>
hipError_t launch_err_partials(const TV* V, const TR* R, int p, const long long* N,
                               const double* const* w, double* partials, int nblocks, hipStream_t s) {
  WPtrs wp;
  long long total = 1;
  wp.p = p;
  for (int k = 0; k < TDB_P; ++k) {
    wp.w[k] = k < p ? w[k] : nullptr;
    wp.N[k] = k < p ? N[k] : 1;
    if (k < p) total *= N[k];
  }
  hipLaunchKernelGGL((k_err_partials<TV, TR>), dim3(nblocks), dim3(256), 0, s, V, R, wp, total, partials);
  return hipGetLastError();
}
template hipError_t launch_err_partials<double, double>(const double*, const double*, int, const long long*,
                                                        const double* const*, double*, int, hipStream_t);
template hipError_t launch_err_partials<float, float>(const float*, const float*, int, const long long*,
                                                      const double* const*, double*, int, hipStream_t);
template hipError_t launch_err_partials<float, double>(const float*, const double*, int, const long long*,
                                                       const double* const*, double*, int, hipStream_t);
template hipError_t launch_err_partials<double, float>(const double*, const float*, int, const long long*,
                                                       const double* const*, double*, int, hipStream_t);

__global__ void __launch_bounds__(256) k_err_final(const double* partials, int nb, CtrlState* ctrl) {
  __shared__ double red[16];
  double se = 0.0, sv = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    se += partials[2 * i];
    sv += partials[2 * i + 1];
  }
  se = block_sum(se, red);
  sv = block_sum(sv, red);
  if (threadIdx.x == 0) {
    ctrl->eps2 = se;
    ctrl->nu2 = sv;
  }
}

hipError_t launch_err_final(const double* partials, int nblocks, CtrlState* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_err_final, dim3(1), dim3(256), 0, s, partials, nblocks, ctrl);
  return hipGetLastError();
}

__global__ void k_flag_clear(int* flag) { *flag = 0; }

template <typename T>
__global__ void __launch_bounds__(256) k_nonfinite(const T* __restrict__ x, long long n, int* flag) {
  int bad = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    bad |= isfinite(x[i]) ? 0 : 1;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_nonfinite_check(const T* x, long long n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, s, flag);
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_nonfinite<T>), dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}
template hipError_t launch_nonfinite_check<float>(const float*, long long, int*, hipStream_t);
template hipError_t launch_nonfinite_check<double>(const double*, long long, int*, hipStream_t);

// The two stage derivatives of the second-order difference (Sec. 2.3): D1 at t_k by
// the central difference and D2 at t_{k+1} by the one-sided second-order difference,
// from the snapshots at t_{k-1} (Vm), t_k (V0) and t_{k+1} (V1). Formed in FP64 and
// stored in the data type; c = 1 / (2 dt). A grid-stride loop, one element per
// thread per pass (the loads of the three snapshots are coalesced).
template <typename T>
__global__ void __launch_bounds__(256) k_fd2(const T* __restrict__ Vm, const T* __restrict__ V0,
                                             const T* __restrict__ V1, T* __restrict__ D1, T* __restrict__ D2,
                                             long long n, double c) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double a = (double)Vm[i], b = (double)V0[i], x = (double)V1[i];
    D1[i] = (T)((x - a) * c);
    D2[i] = (T)((3.0 * x - 4.0 * b + a) * c);
  }
}

template <typename T>
hipError_t launch_fd2(const T* Vm, const T* V0, const T* V1, T* D1, T* D2, long long n, double dt, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_fd2<T>), dim3((unsigned)blocks), dim3(256), 0, s, Vm, V0, V1, D1, D2, n, 0.5 / dt);
  return hipGetLastError();
}
template hipError_t launch_fd2<float>(const float*, const float*, const float*, float*, float*, long long, double,
                                      hipStream_t);
template hipError_t launch_fd2<double>(const double*, const double*, const double*, double*, double*, long long,
                                       double, hipStream_t);

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (TO)in[i];
}

template <typename TI, typename TO>
hipError_t launch_convert(const TI* in, TO* out, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, long long, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, long long, hipStream_t);
template hipError_t launch_convert<float, float>(const float*, float*, long long, hipStream_t);

}  // namespace tdb
