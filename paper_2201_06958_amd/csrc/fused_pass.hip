// Stage pass of the fused third-order path: one streaming read of the snapshot
// pair per Heun stage (eqs. (Corecont) and (basecont)).
//
// Tile: T1 slabs of mode 1 x T2 rows of mode 2 x all of mode 3. Per tile
// (D = V1 - V0 on the tile, B_n = W_n U_n, all local):
//   Z  = D x_3 B3^T                 (T1, T2, r3)
//   F1 = Z x_2 B2^T                 (T1, r2, r3)  rows of F_1 on this tile (partial in i2)
//   F2 = Z x_1 B1^T                 (r1, T2, r3)  rows of F_2 (partial in i1)
//   F3 = (D x_2 B2^T) x_1 B1^T      (r1, r2, N3)  F_3 partial (only if mode 3 is not full rank)
//   Cdot_p = F1 x_1 B1^T            (r1, r2, r3)
//   H_n,p = F_n,p(n) P_n, M_n,p = B_n(tile rows)^T H_n,p
// Each tile writes its partials to its own slot; a separate reduction sums them in
// a fixed order, so results do not depend on scheduling.
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "device_util.h"
#include <hip/hip_ext.h>
#include <math.h>

namespace tdb {
// ---------------------------------------------------------------- stage pass
template <typename TD, typename T>
__device__ __forceinline__ void fpass_body(const FPassArgs& a, int bx) {
  if (a.hold && *a.hold) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int N2 = a.N2, N3 = a.N3, r1 = a.r1, r2 = a.r2, r3 = a.r3;
  const int T1 = a.T1, T2 = a.T2;
  const int t1 = bx / a.nt2, t2 = bx % a.nt2;
  const int i1_0 = t1 * T1, i2_0 = t2 * T2;
  const int n1 = min(T1, a.N1 - i1_0), n2 = min(T2, N2 - i2_0);
  const int R1 = r2 * r3, R2 = r1 * r3, R3 = r1 * r2;
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
  T* F3 = Ys + (a.need_f3 ? T1 * r2 * N3 : 0);       // r1*r2*N3 (need_f3)
  T* Pl = F3 + (a.need_f3 ? r1 * r2 * N3 : 0);       // staged P1 | P2 | P3
  const int tid = threadIdx.x, nth = blockDim.x;
  const T* P1 = static_cast<const T*>(a.P1);
  const T* P2 = static_cast<const T*>(a.P2);
  const T* P3 = static_cast<const T*>(a.P3);

  // load the tile of the data difference (8 loads of each snapshot in flight per thread),
  // the local basis rows and the pseudo-inverses
  const int row = T2 * N3;
  const int total = T1 * row, nvalid = n2 * N3;
  const TD* V1 = static_cast<const TD*>(a.V1);
  const TD* V0 = static_cast<const TD*>(a.V0);
  for (int base = 0; base < total; base += 8 * nth) {
    TD va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * nth + tid;
      va[u] = (TD)0;
      vb[u] = (TD)0;
      if (t < total) {
        const int i1l = t / row, rest = t - (t / row) * row;
        if (i1l < n1 && rest < nvalid) {
          const long long g = ((long long)(i1_0 + i1l) * N2 + i2_0) * N3 + rest;
          va[u] = V1[g];
          if (V0) vb[u] = V0[g];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * nth + tid;
      if (t < total) Ds[t] = (T)va[u] - (T)vb[u];
    }
  }
  const T* B1 = static_cast<const T*>(a.B1);
  const T* B2 = static_cast<const T*>(a.B2);
  const T* B3 = static_cast<const T*>(a.B3);
  for (int t = tid; t < T1 * r1; t += nth) B1s[t] = t < n1 * r1 ? B1[(long long)i1_0 * r1 + t] : (T)0;
  for (int t = tid; t < T2 * r2; t += nth) B2s[t] = t < n2 * r2 ? B2[(long long)i2_0 * r2 + t] : (T)0;
  for (int t = tid; t < N3 * r3; t += nth) B3s[t] = B3[t];
  if (a.stage_p) {
    T* p = Pl;
    if (a.need_h1) { for (int t = tid; t < R1 * r1; t += nth) p[t] = P1[t]; P1 = p; p += R1 * r1; }
    if (a.need_h2) { for (int t = tid; t < R2 * r2; t += nth) p[t] = P2[t]; P2 = p; p += R2 * r2; }
    if (a.need_f3) { for (int t = tid; t < R3 * r3; t += nth) p[t] = P3[t]; P3 = p; }
  }
  __syncthreads();

  // Z = D x_3 B3^T (one row of N3 values per thread iteration)
  for (int q = tid; q < T1 * T2; q += nth) {
    const T* d = Ds + q * N3;
    T* z = Zs + q * r3;
    for (int c2 = 0; c2 < r3; ++c2) {
      T s = (T)0;
      for (int c = 0; c < N3; ++c) s += d[c] * B3s[c * r3 + c2];
      z[c2] = s;
    }
  }
  // Y = D x_2 B2^T
  if (a.need_f3) {
    for (int t = tid; t < T1 * r2 * N3; t += nth) {
      const int c = t % N3, q = t / N3;
      const int b = q % r2, i1l = q / r2;
      const T* d = Ds + i1l * T2 * N3 + c;
      T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
      int i2l = 0;
      for (; i2l + 4 <= T2; i2l += 4) {
        s0 += B2s[i2l * r2 + b] * d[i2l * N3];
        s1 += B2s[(i2l + 1) * r2 + b] * d[(i2l + 1) * N3];
        s2 += B2s[(i2l + 2) * r2 + b] * d[(i2l + 2) * N3];
        s3 += B2s[(i2l + 3) * r2 + b] * d[(i2l + 3) * N3];
      }
      for (; i2l < T2; ++i2l) s0 += B2s[i2l * r2 + b] * d[i2l * N3];
      Ys[t] = (s0 + s1) + (s2 + s3);
    }
  }
  __syncthreads();

  // F1 = Z x_2 B2^T
  for (int t = tid; t < T1 * r2 * r3; t += nth) {
    const int c2 = t % r3, q = t / r3;
    const int b = q % r2, i1l = q / r2;
    const T* z = Zs + i1l * T2 * r3 + c2;
    T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
    int i2l = 0;
    for (; i2l + 4 <= T2; i2l += 4) {
      s0 += B2s[i2l * r2 + b] * z[i2l * r3];
      s1 += B2s[(i2l + 1) * r2 + b] * z[(i2l + 1) * r3];
      s2 += B2s[(i2l + 2) * r2 + b] * z[(i2l + 2) * r3];
      s3 += B2s[(i2l + 3) * r2 + b] * z[(i2l + 3) * r3];
    }
    for (; i2l < T2; ++i2l) s0 += B2s[i2l * r2 + b] * z[i2l * r3];
    F1[t] = (s0 + s1) + (s2 + s3);
  }
  // F2 = Z x_1 B1^T: one (i2l, c2) column per thread iteration, all a
  for (int q = tid; q < T2 * r3; q += nth) {
    const int i2l = q / r3, c2 = q - (q / r3) * r3;
    for (int ai = 0; ai < r1; ++ai) {
      T s = (T)0;
      for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + ai] * Zs[(i1l * T2 + i2l) * r3 + c2];
      F2[(ai * T2 + i2l) * r3 + c2] = s;
    }
  }
  // F3 = Y x_1 B1^T
  if (a.need_f3) {
    for (int q = tid; q < r2 * N3; q += nth) {
      for (int ai = 0; ai < r1; ++ai) {
        T s = (T)0;
        for (int i1l = 0; i1l < T1; ++i1l) s += B1s[i1l * r1 + ai] * Ys[i1l * r2 * N3 + q];
        F3[ai * r2 * N3 + q] = s;
      }
    }
  }
  __syncthreads();

  // partial outputs of this tile
  T* out = static_cast<T*>(a.part) + (long long)bx * a.slot;
  T* oH1 = out;
  T* oH2 = oH1 + T1 * r1;
  T* oH3 = oH2 + T2 * r2;
  T* oC = oH3 + N3 * r3;
  T* oM1 = oC + r1 * r2 * r3;
  T* oM2 = oM1 + r1 * r1;
  T* oM3 = oM2 + r2 * r2;
  // core partial: Cdot_p[a][b][c2] = sum_i1 B1[i1][a] F1[i1][b][c2] (one output per thread)
  for (int t = tid; t < r1 * R1; t += nth) {
    const int ai = t / R1, bc = t - (t / R1) * R1;
    T s0 = (T)0, s1 = (T)0;
    int i1l = 0;
    for (; i1l + 2 <= T1; i1l += 2) {
      s0 += B1s[i1l * r1 + ai] * F1[i1l * R1 + bc];
      s1 += B1s[(i1l + 1) * r1 + ai] * F1[(i1l + 1) * R1 + bc];
    }
    if (i1l < T1) s0 += B1s[i1l * r1 + ai] * F1[i1l * R1 + bc];
    oC[t] = s0 + s1;
  }
  // H1_p[i1][a] = sum_(b,c2) F1[i1][b][c2] P1[(b,c2)][a]: 4 lanes per output
  if (a.need_h1) {
    for (int t4 = tid; t4 < 4 * T1 * r1; t4 += nth) {
      const int t = t4 >> 2, part = t4 & 3;
      const int ai = t % r1, i1l = t / r1;
      const T* f = F1 + i1l * R1;
      T s = (T)0;
      for (int k = part; k < R1; k += 4) s += f[k] * P1[k * r1 + ai];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      if (part == 0) oH1[t] = s;
    }
  }
  // H2_p[i2][b] = sum_(a,c2) F2[a][i2][c2] P2[(a,c2)][b]: two outputs per iteration
  if (a.need_h2) {
    const int nout = T2 * r2;
    for (int t = tid; t < nout; t += 2 * nth) {
      const int tb = t + nth;
      const bool two = tb < nout;
      const int b0 = t % r2, i20 = t / r2;
      const int b1 = two ? tb % r2 : 0, i21 = two ? tb / r2 : 0;
      T s0 = (T)0, s1 = (T)0;
      for (int ai = 0; ai < r1; ++ai) {
        const T* f0 = F2 + (ai * T2 + i20) * r3;
        const T* f1 = F2 + (ai * T2 + i21) * r3;
        const T* pp = P2 + (ai * r3) * r2;
        for (int c2 = 0; c2 < r3; ++c2) {
          s0 += f0[c2] * pp[c2 * r2 + b0];
          s1 += f1[c2] * pp[c2 * r2 + b1];
        }
      }
      oH2[t] = s0;
      if (two) oH2[tb] = s1;
    }
  }
  // H3_p[c][c2] = sum_(a,b) F3[a][b][c] P3[(a,b)][c2]: 8 lanes per output
  if (a.need_f3) {
    for (int t8 = tid; t8 < 8 * N3 * r3; t8 += nth) {
      const int t = t8 >> 3, part = t8 & 7;
      const int c2 = t % r3, c = t / r3;
      T s = (T)0;
      for (int k = part; k < R3; k += 8) s += F3[k * N3 + c] * P3[k * r3 + c2];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (part == 0) oH3[t] = s;
    }
  }
}

template <typename TD, typename T>
__global__ void __launch_bounds__(256) k_fpass(FPassArgs a) {
  fpass_body<TD, T>(a, blockIdx.x);
}

template <typename TD, typename T>
hipError_t launch_fpass(const FPassArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fpass<TD, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL((k_fpass<TD, T>), dim3(a.nt1 * a.nt2), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, a);
  return hipGetLastError();
}
template hipError_t launch_fpass<float, float>(const FPassArgs&, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fpass<float, double>(const FPassArgs&, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fpass<double, double>(const FPassArgs&, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_fpass<double, float>(const FPassArgs&, size_t, hipStream_t, hipEvent_t, hipEvent_t);

// Batched form: one launch over the tiles of many streams.
template <typename TD, typename T>
__global__ void __launch_bounds__(256) kb_fpass(const FPassArgs* __restrict__ tab, const void* const* v1,
                                                const void* const* v0, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  FPassArgs a = tab[s];
  a.V1 = v1[s];
  a.V0 = v0[s];
  fpass_body<TD, T>(a, blockIdx.x - m.start[s]);
}

template <typename TD, typename T>
hipError_t launch_batch_fpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_fpass<TD, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL((kb_fpass<TD, T>), dim3(blocks), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, tab, v1, v0, m);
  return hipGetLastError();
}
template hipError_t launch_batch_fpass<float, float>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                                    size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_fpass<float, double>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                                    size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_fpass<double, double>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                                    size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_fpass<double, float>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                                    size_t, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace tdb
