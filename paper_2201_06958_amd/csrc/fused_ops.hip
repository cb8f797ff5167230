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
#include <type_traits>
#include <map>
#include <mutex>
#include "device_util.h"
#include <hip/hip_ext.h>
#include <math.h>

namespace tdb {

typedef double md4 __attribute__((ext_vector_type(4)));

// A kernel's dynamic-LDS limit raised only when a launch asks for more than it was given
// on the current device: the attribute call is otherwise a runtime call of a few
// microseconds on every launch of a single stream's step, which the host issues one
// kernel at a time.
static hipError_t lds_limit(const void* f, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> given;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  int& g = given[{f, dev}];
  if ((int)lds <= g) return hipSuccess;
  e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) g = (int)lds;
  return e;
}

// ---------------------------------------------------------------- reduction
// Sums the per-tile partials in a fixed order (FP64) into H_n and C_dot, and applies
// the Heun update to the core (stage 1: k = C_dot/dt, C* = C + dt k; stage 2:
// C <- C + dt/2 (k + C_dot/dt)). Each output is summed by L lanes of one wave (lane
// group j takes partials j, j + L, ...), combined by a fixed butterfly, so the order of
// the additions never depends on scheduling. A wave covers Q = 64/L consecutive
// outputs: lane = j*Q + (output within the wave), so neighbouring lanes read
// neighbouring partials of the same tile.
template <typename T>
__device__ __forceinline__ void freduce_body(const FReduceArgs& a, int stage, CtrlState* ctrl, int bx, int gx) {
  if (ctrl->hold || (stage == 2 && ctrl->numeric)) return;
  // A singular core found while preparing this step (bit 4, set by k_fpost) belongs
  // to this step's first stage, like the failure of its pseudo-inverse would.
  // (atomics: other blocks may be raising NUM_NONFINITE meanwhile)
  if (stage == 1 && bx == 0 && threadIdx.x == 0 && (ctrl->numeric & NUM_NEXT)) {
    atomicOr(&ctrl->numeric, NUM_CORE);
    atomicAnd(&ctrl->numeric, ~NUM_NEXT);
  }
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
  const double inv_dt = a.dscale;   // 1/dt for a difference quotient, 1 for a given derivative
  // e4 is a multiple of 64 and so is the stride: every wave runs the same trip count.
  // A thread takes RED_U outputs per pass, with the (at most 8) partials of all of them
  // loaded from clamped indices before any is added, so that a pass costs one memory
  // round trip; the partials of one lane are added in a fixed tree.
  const long long S = (long long)gx * blockDim.x;
  for (long long t0 = (long long)bx * blockDim.x + threadIdx.x; t0 < e4; t0 += RED_U * S) {
    double pv[RED_U][8];
    int cntv[RED_U], jv[RED_U], kindv[RED_U], Lv[RED_U], Qv[RED_U];
    long long qv[RED_U];
    const T* basev[RED_U];
    long long stv[RED_U];
#pragma unroll
    for (int u = 0; u < RED_U; ++u) {
      const long long t = t0 + u * S;
      int kind, L;
      long long uu;
      if (t < e1) { kind = 0; L = L1; uu = t; }
      else if (t < e2) { kind = 1; L = L2; uu = t - e1; }
      else if (t < e3) { kind = 2; L = L3; uu = t - e2; }
      else { kind = 3; L = L3; uu = t - e3; }
      const int Q = 64 / L;
      const int lw = (int)(uu & 63);
      const long long q = (uu >> 6) * Q + (lw % Q);
      const int j = lw / Q;
      const long long nq = kind == 0 ? nH1 : kind == 1 ? nH2 : kind == 2 ? nH3 : nC;
      const bool valid = t < e4 && q < nq;
      const T* base = part;
      long long stride = 0;
      int count = 0;
      if (valid) {
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
      }
      const int cnt = valid ? max((count - j + L - 1) / L, 0) : 0;
      base += (long long)j * stride;
      stride *= L;
#pragma unroll
      for (int k = 0; k < 8; ++k) pv[u][k] = (double)gmem(base)[(long long)min(k, max(cnt - 1, 0)) * stride];
      cntv[u] = cnt;
      jv[u] = j;
      kindv[u] = valid ? kind : -1;
      Lv[u] = L;
      Qv[u] = Q;
      qv[u] = q;
      basev[u] = base;
      stv[u] = stride;
    }
#pragma unroll
    for (int u = 0; u < RED_U; ++u) {
      if (t0 + u * S >= e4) break;   // wave-uniform
      const int cnt = cntv[u];
      double sk[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) sk[k] = k < cnt ? pv[u][k] : 0.0;
      // partials past the eighth (only for more than 8 L of them): added in the same
      // eight accumulators, in order
      for (int k = 8; k < cnt; ++k) sk[k & 7] += (double)basev[u][(long long)k * stv[u]];
      double s = ((sk[0] + sk[1]) + (sk[2] + sk[3])) + ((sk[4] + sk[5]) + (sk[6] + sk[7]));
      const int L = Lv[u], Q = Qv[u];
      for (int o = L >> 1; o >= 1; o >>= 1) s += __shfl_xor(s, o * Q, 64);
      const int kind = kindv[u];
      if (kind < 0 || jv[u] != 0) continue;
      const long long q = qv[u];
      if (kind == 0) {
        a.H[0][q] = s;
      } else if (kind == 1) {
        a.H[1][q] = s;
      } else if (kind == 2) {
        a.H[2][q] = s;
      } else {
        const double cd = s * inv_dt;
        if (stage == 1) {
          // every entry of the data derivative reaches every entry of C_dot, so NaN or
          // Inf anywhere in the snapshots shows here; the step is then not applied
          if (!isfinite(cd)) atomicOr(&ctrl->numeric, NUM_NONFINITE);
          a.kC[q] = cd;
          a.Cs[q] = a.C0[q] + a.dt * cd;
        } else {
          a.Cdot2[q] = cd;
          a.C0[q] += 0.5 * a.dt * (a.kC[q] + cd);
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_freduce(FReduceArgs a, CtrlState* ctrl) {
  freduce_body<T>(a, a.stage, ctrl, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- prep helpers
// G[i][j] = sum_k XA(i, k) XB(j, k) for i, j < n on the FP64 matrix cores (16x16x4),
// by the whole block (four waves). xa(i, k) and xb(j, k) return the operands (zero is
// never requested outside i, j < n, k < K). With sym only the blocks bi >= bj are
// formed and emit(r, c, v) is called for r >= c (the caller mirrors). A single output
// block is split over the waves along k and the four partials (part: 1024 doubles of
// LDS) are added in a fixed order; otherwise the waves share out the blocks and each
// covers all of k. Ends with a block barrier.
template <typename FA, typename FB, typename Emit>
__device__ __forceinline__ void block_xyt_f64(int n, int K, bool sym, FA xa, FB xb, Emit emit, double* part) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  const int nb = (n + 15) >> 4;
  const int nblk = sym ? nb * (nb + 1) / 2 : nb * nb;
  const bool split = nblk == 1;
  const int per = split ? (((K + 3) / 4 + 3) & ~3) : K;
  const int k0 = split ? wid * per : 0, k1 = split ? min(K, k0 + per) : K;
  for (int blk = split ? 0 : wid; blk < nblk; blk += split ? 1 : 4) {
    int bi, bj;
    if (sym) {
      bi = 0;
      while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
      bj = blk - bi * (bi + 1) / 2;
    } else {
      bi = blk / nb;
      bj = blk - bi * nb;
    }
    const int ia = 16 * bi + lm, jb = 16 * bj + lm;
    md4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = k0; kk < k1; kk += 4) {
      const int k = kk + lk;
      const double av = (k < k1 && ia < n) ? xa(ia, k) : 0.0;
      const double bv = (k < k1 && jb < n) ? xb(jb, k) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    // FP64 16x16x4 result: lane holds rows 16 bi + lk + 4 i, column 16 bj + lm
    if (split) {
#pragma unroll
      for (int i = 0; i < 4; ++i) part[wid * 256 + (lk + 4 * i) * 16 + lm] = acc[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * bi + lk + 4 * i, c = 16 * bj + lm;
        if (r < n && c < n && (!sym || bi > bj || r >= c)) emit(r, c, acc[i]);
      }
    }
  }
  __syncthreads();
  if (split) {
    const int t = threadIdx.x, r = t >> 4, c = t & 15;
    if (r < n && c < n && (!sym || r >= c)) emit(r, c, (part[t] + part[256 + t]) + (part[512 + t] + part[768 + t]));
    __syncthreads();
  }
}

// Entry (i, c) of the mode-n unfolding of a core stored with `inner` = prod_{k>n} r_k:
// column c = o*inner + in sits at (o*rn + i)*inner + in.
__device__ __forceinline__ int unfold_at(int i, int c, int rn, int inner) {
  const int o = c / inner;
  return (o * rn + i) * inner + (c - o * inner);
}

// Core Gram of the mode-n unfolding into LDS G (rn x rn) from a core (LDS or global);
// part: 1024 doubles of LDS scratch.
__device__ void gram_from(const double* Cl, int rn, long long R, long long inner_, double* G, double* part) {
  const int inner = (int)inner_;
  auto x = [&](int i, int c) { return Cl[unfold_at(i, c, rn, inner)]; };
  block_xyt_f64(rn, (int)R, true, x, x,
                [&](int r, int c, double v) {
                  G[r * rn + c] = v;
                  G[c * rn + r] = v;
                },
                part);
}

// M_n = C_dot_(n) P_n / dscale (rn x rn; dt C_dot_(n) P_n for a difference quotient) into
// Ml from LDS copies of C_dot and P_n (R x rn);
// part: 1024 doubles of LDS scratch.
template <typename T>
__device__ void form_m(const double* cdl, const T* Pn, int rn, int R, int inner, double dt, double* Ml, double* part) {
  block_xyt_f64(
      rn, R, false, [&](int i, int c) { return cdl[unfold_at(i, c, rn, inner)]; },
      [&](int j, int c) { return (double)Pn[c * rn + j]; },
      [&](int r, int c, double v) { Ml[r * rn + c] = v * dt; },   // H is the raw (undivided) projection, so M is too
      part);
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
  if (ctrl->hold || (stage == 2 && ctrl->numeric)) return;
  const int n = bx;
  const int rr = a.r[n];
  if (rr >= a.N[n]) return;
  const double* cd = stage == 1 ? a.kC : a.Cdot2;   // this stage's C_dot
  const int csz = a.r[0] * a.r[1] * a.r[2];
  const int Rn = csz / rr;
  double* cdl = lds;
  T* pl = reinterpret_cast<T*>(cdl + csz);
  const T* Pn = static_cast<const T*>(a.Pcur[n]);
  g2l(cdl, cd, csz);
  g2l(pl, Pn, Rn * rr);
  __syncthreads();
  int inner = 1;
  for (int k = n + 1; k < 3; ++k) inner *= a.r[k];
  double* Ml = lds + (csz * 8 + Rn * rr * (int)sizeof(T) + 7) / 8;
  double* part = Ml + rr * rr;
  form_m<T>(cdl, pl, rr, Rn, inner, 1.0 / a.dscale, Ml, part);
  for (int t = threadIdx.x; t < rr * rr; t += blockDim.x) a.M[n][t] = Ml[t];
}

template <typename T>
__global__ void __launch_bounds__(256) k_fmprep(FFinishArgs a, CtrlState* ctrl) {
  fmprep_body<T>(a, a.stage, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- finish a stage
// Per-lane choice among three per-mode values. The argument blocks sit in global
// memory (a batch's table) or the kernel arguments: indexing them with a lane-varying
// mode would turn every field access into a dependent vector load, so each field is
// read at a constant index (a scalar load) and chosen per lane.
template <typename V>
__device__ __forceinline__ V sel3(int n, V v0, V v1, V v2) {
  return n == 0 ? v0 : (n == 1 ? v1 : v2);
}

// One pass of a row block over EPT * blockDim.x consecutive elements from `base`
// of the flat order over the rows of the three bases (mode by mode, r_n entries a
// row). Element f needs the r_n entries of its row of U*, which lie within rmax - 1
// places of f in that order: the pass stages its elements and that halo into LDS (at
// most (EPT + 1) * blockDim.x values, ranks being at most 64), with every operand
// of the pass (and, in the first pass, the M_n) loaded in one round trip before any
// LDS store, instead of r_n dependent loads per element. The loads are unconditional,
// from indices clamped into range, so that no branch separates them; what a lane loads
// past the end is never used.
template <typename T, bool LOADM, int ST, int EPT>
__device__ __forceinline__ void fin_rows_pass(const FFinishArgs& a, long long base, long long tot,
                                              double* const* Ml, const int* mcnt, double* tile) {
  const int nt = (int)blockDim.x, tid = (int)threadIdx.x;
  const int halo = a.rmax - 1;
  const int tw = EPT * nt + 2 * halo;
  const int r0 = a.r[0], r1 = a.r[1], r2 = a.r[2];
  const long long L0 = a.N[0] * r0, L01 = L0 + a.N[1] * r1;
  const int ld0 = a.ldU[0], ld1 = a.ldU[1], ld2 = a.ldU[2];
  const bool act0 = r0 < a.N[0], act1 = r1 < a.N[1], act2 = r2 < a.N[2];
  // flat index f -> mode n, index q within the mode, row i, column j, entry e of U_n
  auto locate = [&](long long f, int& n, long long& q, long long& i, int& j, long long& e) {
    n = f < L0 ? 0 : (f < L01 ? 1 : 2);
    q = f - sel3<long long>(n, 0, L0, L01);
    const int rn = sel3(n, r0, r1, r2);
    i = q < 2147483647LL ? (long long)((unsigned)q / (unsigned)rn) : q / rn;
    j = (int)(q - i * rn);
    e = i * sel3(n, ld0, ld1, ld2) + j;
  };
  const double* U00 = a.U0[0];
  const double* U01 = a.U0[1];
  const double* U02 = a.U0[2];
  const double* Ust0 = ST == 1 ? U00 : a.Us[0];
  const double* Ust1 = ST == 1 ? U01 : a.Us[1];
  const double* Ust2 = ST == 1 ? U02 : a.Us[2];
  const int c01 = mcnt[0] + mcnt[1], call = c01 + mcnt[2];
  double mv[LOADM ? FIN_MU : 1];
  if (LOADM) {
#pragma unroll
    for (int u = 0; u < FIN_MU; ++u) {
      const int t = min(u * nt + tid, call - 1);
      const int n = t < mcnt[0] ? 0 : (t < c01 ? 1 : 2);
      mv[u] = *gmem(sel3<const double*>(n, a.M[0], a.M[1], a.M[2]) + (t - sel3(n, 0, mcnt[0], c01)));
    }
  }
  double tv[EPT + 1];
#pragma unroll
  for (int u = 0; u <= EPT; ++u) {
    const long long f = min(max(base - halo + u * nt + tid, 0LL), tot - 1);
    int n, j;
    long long q, i, e;
    locate(f, n, q, i, j, e);
    tv[u] = *gmem(sel3(n, Ust0, Ust1, Ust2) + e);
  }
  double hv[EPT], av[EPT], bv[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const long long t = min(base + u * nt + tid, tot - 1);
    int n, j;
    long long q, i, e;
    locate(t, n, q, i, j, e);
    // (a mode kept at full rank has no H_n: its lanes read U_n instead and ignore it)
    const double* hp = sel3(n, act0, act1, act2) ? sel3(n, a.H[0], a.H[1], a.H[2]) + q : sel3(n, U00, U01, U02) + e;
    hv[u] = *gmem(hp);
    if (ST == 1) {
      av[u] = *gmem(sel3(n, a.w[0], a.w[1], a.w[2]) + i);
      bv[u] = 0.0;
    } else {
      av[u] = *gmem(sel3<const double*>(n, a.kU[0], a.kU[1], a.kU[2]) + e);
      bv[u] = *gmem(sel3(n, U00, U01, U02) + e);
    }
  }
  if (LOADM) {
#pragma unroll
    for (int u = 0; u < FIN_MU; ++u) {
      const int t = u * nt + tid;
      if (t < call) {
        const int n = t < mcnt[0] ? 0 : (t < c01 ? 1 : 2);
        sel3(n, Ml[0], Ml[1], Ml[2])[t - sel3(n, 0, mcnt[0], c01)] = mv[u];
      }
    }
    // the rest of the M_n (rank caps above about 26 in every mode)
    for (int t = FIN_MU * nt + tid; t < call; t += nt) {
      const int n = t < mcnt[0] ? 0 : (t < c01 ? 1 : 2);
      const int e = t - sel3(n, 0, mcnt[0], c01);
      sel3(n, Ml[0], Ml[1], Ml[2])[e] = sel3<const double*>(n, a.M[0], a.M[1], a.M[2])[e];
    }
  }
#pragma unroll
  for (int u = 0; u <= EPT; ++u) {
    const int x = u * nt + tid;
    if (x < tw) tile[x] = tv[u];
  }
  __syncthreads();
  const double inv_dt = a.dscale;   // 1/dt for a difference quotient, 1 for a given derivative
  const double dt = a.dt;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const long long t = base + u * nt + tid;
    if (t < tot) {
      int n, j;
      long long q, i, e;
      locate(t, n, q, i, j, e);
      const int rn = sel3(n, r0, r1, r2);
      const int x = u * nt + tid + halo;   // element t in the tile
      double ud = 0.0;
      if (sel3(n, act0, act1, act2)) {
        const double* M = sel3(n, Ml[0], Ml[1], Ml[2]);
        const double* ur = tile + x - j;
        double s = hv[u];
        for (int k = 0; k < rn; ++k) s -= ur[k] * M[k * rn + j];
        ud = s * inv_dt;
      }
      if (ST == 1) {
        *gmem(sel3(n, a.kU[0], a.kU[1], a.kU[2]) + e) = ud;
        const double us = tile[x] + dt * ud;
        *gmem(sel3(n, a.Us[0], a.Us[1], a.Us[2]) + e) = us;
        *gmem(sel3(n, static_cast<T*>(a.B[0]), static_cast<T*>(a.B[1]), static_cast<T*>(a.B[2])) + q) =
            (T)(av[u] * us);
      } else {
        *gmem(sel3(n, a.U0[0], a.U0[1], a.U0[2]) + e) = bv[u] + 0.5 * dt * (av[u] + ud);
      }
    }
  }
  __syncthreads();
}

// All passes of one row block (EPT elements a thread and pass: FIN_EPT for a batch, whose
// grids are large, one for a single stream, whose blocks are few).
template <typename T, int ST, int EPT>
__device__ __forceinline__ void fin_rows(const FFinishArgs& a, long long tot, long long bx, double* const* Ml,
                                         const int* mcnt, double* tile) {
  const long long span = (long long)EPT * blockDim.x;
  const long long step = (long long)a.rowblocks * span;
  long long base = bx * span;
  if (mcnt[0] + mcnt[1] + mcnt[2] > 0) {
    fin_rows_pass<T, true, ST, EPT>(a, base, tot, Ml, mcnt, tile);
    base += step;
  }
  for (; base < tot; base += step) fin_rows_pass<T, false, ST, EPT>(a, base, tot, Ml, mcnt, tile);
}

// Blocks [0, rowblocks): rows of every mode: U_dot = (H - U M)/dt, Heun update and,
// in stage 1, the weighted basis B_n = W_n U* of the next stage.
// Blocks [rowblocks, rowblocks + 3) (stage 1 only): pseudo-inverse P_n at the stage
// core C* (already updated by the reduction). A batch launches the two roles as
// separate kernels (ROLE_ROWS, ROLE_PINV: block bx is mode bx), so that the row blocks
// do not carry the factorisation's registers.
template <typename T, int ROLE>
__device__ __forceinline__ void ffinish_body(const FFinishArgs& a, int stage, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  if (ctrl->hold || (stage == 2 && ctrl->numeric)) return;
  const double inv_dt = a.dscale;   // 1/dt for a difference quotient, 1 for a given derivative
  if (ROLE == ROLE_ROWS || (ROLE == ROLE_ALL && (int)bx < a.rowblocks)) {
    long long tot = 0;
    for (int n = 0; n < 3; ++n) tot += a.N[n] * a.r[n];
    // a batch sizes the grid for the rank caps: blocks past the current ranks' rows
    // leave before loading anything (block-uniform, ahead of every barrier)
    constexpr int EPT = ROLE == ROLE_ROWS ? FIN_EPT : 1;
    const long long span = (long long)EPT * blockDim.x;
    if ((long long)bx * span >= tot) return;
    // M_n (r_n x r_n) into LDS: formed once per stage by k_fmprep, or here (a single
    // stream, where the extra launch would cost more than the repeated small product)
    double* Ml[3];
    double* tile;                // the rows of the pass's elements (see fin_rows_pass)
    int mcnt[3] = {0, 0, 0};     // M_n values still to load
    if (ROLE == ROLE_ALL && a.m_inline) {   // (a batch forms M_n in its own kernel)
      const double* cd = stage == 1 ? a.kC : a.Cdot2;   // this stage's C_dot
      const int csz = a.r[0] * a.r[1] * a.r[2];
      double* cdl = lds;
      T* pl = reinterpret_cast<T*>(cdl + csz);
      int poff[3], off = 0;
      for (int n = 0; n < 3; ++n) {
        poff[n] = off;
        if (a.r[n] < a.N[n]) off += csz;
      }
      {
        // C_dot and the active P_n in one pass, 16 loads in flight per thread
        const T* P0 = static_cast<const T*>(a.Pcur[0]);
        const T* P1 = static_cast<const T*>(a.Pcur[1]);
        const T* P2 = static_cast<const T*>(a.Pcur[2]);
        const bool a0 = a.r[0] < a.N[0], a1 = a.r[1] < a.N[1];
        const T* Pfirst = a0 ? P0 : (a1 ? P1 : P2);
        const T* Psecond = (a0 && a1) ? P1 : P2;
        const int tot = csz + off;
        for (int base = 0; base < tot; base += 16 * blockDim.x) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int t = base + u * blockDim.x + threadIdx.x;
            double x = 0.0;
            if (t < csz) x = cd[t];
            else if (t < tot) {
              const int q = t - csz, seg = q / csz, e = q - seg * csz;
              const T* src = seg == 0 ? Pfirst : (seg == 1 ? Psecond : P2);
              x = (double)src[e];
            }
            v[u] = x;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int t = base + u * blockDim.x + threadIdx.x;
            if (t < csz) cdl[t] = v[u];
            else if (t < tot) pl[t - csz] = (T)v[u];
          }
        }
      }
      __syncthreads();
      int moff = (int)((csz * 8 + off * (int)sizeof(T) + 7) / 8);
      int msum = 0;
      for (int n = 0; n < 3; ++n) msum += a.r[n] * a.r[n];
      double* part = lds + moff + msum;
      tile = part + FIN_PART;
      for (int n = 0; n < 3; ++n) {
        Ml[n] = lds + moff;
        const int rr = a.r[n];
        if (rr < a.N[n]) {
          int inner = 1;
          for (int k = n + 1; k < 3; ++k) inner *= a.r[k];
          form_m<T>(cdl, pl + poff[n], rr, csz / rr, inner, 1.0 / a.dscale, Ml[n], part);
        }
        moff += rr * rr;
      }
      __syncthreads();
    } else {
      // the M_n arrive with the first pass's operands (one round trip for all of them)
      int off = 0;
      for (int n = 0; n < 3; ++n) {
        Ml[n] = lds + off;
        mcnt[n] = a.r[n] < a.N[n] ? a.r[n] * a.r[n] : 0;
        off += a.r[n] * a.r[n];
      }
      tile = lds + off;
    }
    if (stage == 1) fin_rows<T, 1, EPT>(a, tot, bx, Ml, mcnt, tile);
    else fin_rows<T, 2, EPT>(a, tot, bx, Ml, mcnt, tile);
    return;
  }
  if (ROLE == ROLE_ROWS) return;
  // pseudo-inverse at the stage core
  const int n = ROLE == ROLE_PINV ? bx : bx - a.rowblocks;
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
  double* Gp = Gi + rq * rq;                 // FQR_GP partial blocks
  double* Cl = Gp + FQR_GP;
  __shared__ int ok_s;
  // the core from LDS or from global memory (separate instances: fixed address spaces)
  auto pinv = [&](const double* Csrc) {
    gram_from(Csrc, rn, R, inner, G, Gp);
    if (threadIdx.x < 64) {
      const bool ok = wave_chol_inv(G, rn, Li, Gi);
      if (threadIdx.x == 0) {
        ok_s = ok ? 1 : 0;
        if (!ok) atomicOr(&ctrl->numeric, 1);
      }
    }
    __syncthreads();
    if (!ok_s) return;
    write_p<T>(Csrc, Gi, rn, R, inner, static_cast<T*>(a.P[n]));
  };
  if (a.core_in_lds) {
    g2l(Cl, a.Cs, (int)csz);
    __syncthreads();
    pinv(Cl);
  } else {
    pinv(a.Cs);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ffinish(FFinishArgs a, CtrlState* ctrl) {
  ffinish_body<T, ROLE_ALL>(a, a.stage, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- QR + fold
// One round of Cholesky QR of every U_n in the W inner product (the Heun update leaves
// U_n W-orthonormal to O(dt^2), so a single round reaches roundoff). Block (n, slab):
// the slab's partial Gram sum_q w_q u_q u_q^T. The last block to finish sums every
// mode's partials in slab order, factors the three Grams as L_n L_n^T (one wave per
// mode), publishes L_n^-1, and folds R_n = L_n^T into the core (C <- C x_n R_n, so the
// reconstruction is unchanged), forming T3 = C x_3 U_3 of the folded core on the way.
// The post-step then takes U_n <- U_n R_n^-1 = U_n L_n^-T (it reads every row anyway).
__device__ __forceinline__ int qr_mode(const FQrArgs& a, int bx, int& rb) {
  if (bx < a.nb[0]) { rb = bx; return 0; }
  bx -= a.nb[0];
  if (bx < a.nb[1]) { rb = bx; return 1; }
  rb = bx - a.nb[1];
  return 2;
}

// C <- C x_1 R_1 x_2 R_2 x_3 R_3 with R_m = L_m^T (L_m lower triangular with zeros
// above the diagonal, in LDS) and, between the second and third products,
// T3 = (C x_1 R_1 x_2 R_2) x_3 U_3 = C_new x_3 (U_3 R_3^-1) with U_3 before its
// normalisation. CM 2: the core is in LDS (X) and each product is taken in place
// through registers (at most FOLD_R outputs per thread); CM 1: the products alternate
// between two LDS buffers; CM 0: between C0 and Ctmp in global memory. They are
// separate instances so that every access has a fixed address space.
template <int CM>
__device__ __forceinline__ void fold_core(const FQrArgs& a, const double* L0, const double* L1, const double* L2,
                                          const double* Gp, double* X, int csz, bool u3l) {
  const int N3 = (int)a.N[2], ld3 = a.ldU[2];
  double* ca = CM ? X : a.C0;
  double* cb = CM == 2 ? X : (CM == 1 ? X + csz : a.Ctmp);
  for (int m = 0; m < 3; ++m) {
    const int rm = a.r[m];
    const double* Lm = m == 0 ? L0 : (m == 1 ? L1 : L2);
    if (m == 2 && a.T3) {
      const int r12 = a.r[0] * a.r[1], r3 = a.r[2];
      const float i_n3 = 1.0f / (float)N3;
      const bool fast = r12 * N3 < (1 << 22);
      if (u3l) {
        for (int t = threadIdx.x; t < r12 * N3; t += blockDim.x) {
          const int ab = fast ? small_div(t, N3, i_n3) : t / N3, i3 = t - ab * N3;
          double sv = 0.0;
          for (int c = 0; c < r3; ++c) sv += ca[ab * r3 + c] * Gp[i3 * ld3 + c];
          a.T3[t] = sv;
        }
      } else {
        const double* U3 = a.U0[2];
        for (int t = threadIdx.x; t < r12 * N3; t += blockDim.x) {
          const int ab = fast ? small_div(t, N3, i_n3) : t / N3, i3 = t - ab * N3;
          double sv = 0.0;
          for (int c = 0; c < r3; ++c) sv += ca[ab * r3 + c] * U3[i3 * ld3 + c];
          a.T3[t] = sv;
        }
      }
    }
    int inner = 1;
    for (int k = m + 1; k < 3; ++k) inner *= a.r[k];
    const float i_inner = 1.0f / (float)inner, i_rm = 1.0f / (float)rm;
    // output (o, ai, in) = sum_{b >= ai} R[ai][b] C[o][b][in], R[ai][b] = L[b][ai]
    // (zero for b < ai); outputs in groups of four with their sums interleaved
    if (CM == 2) {
      double sv[FOLD_R];
      const int nug = (csz + (int)blockDim.x - 1) / (int)blockDim.x;   // common to the block
#pragma unroll
      for (int g = 0; g < FOLD_R; g += 4) {
        sv[g] = sv[g + 1] = sv[g + 2] = sv[g + 3] = 0.0;
        if (g < nug) {
          int ai_[4], bs_[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int t = min((int)threadIdx.x + (g + u) * (int)blockDim.x, csz - 1);
            const int rest = small_div(t, inner, i_inner), in = t - rest * inner;
            const int o = small_div(rest, rm, i_rm);
            ai_[u] = rest - o * rm;
            bs_[u] = o * rm * inner + in;
          }
#pragma unroll 4
          for (int b = 0; b < rm; ++b) {
#pragma unroll
            for (int u = 0; u < 4; ++u) sv[g + u] += Lm[b * rm + ai_[u]] * ca[bs_[u] + b * inner];
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < FOLD_R; ++u) {
        const int t = (int)threadIdx.x + u * (int)blockDim.x;
        if (t < csz) ca[t] = sv[u];
      }
      __syncthreads();
    } else {
      for (int t0 = threadIdx.x; t0 < csz; t0 += 4 * (int)blockDim.x) {
        int ai_[4], bs_[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = min(t0 + u * (int)blockDim.x, csz - 1);
          const int rest = csz < (1 << 22) ? small_div(t, inner, i_inner) : t / inner, in = t - rest * inner;
          const int o = rest / rm;
          ai_[u] = rest - o * rm;
          bs_[u] = o * rm * inner + in;
        }
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int b = 0; b < rm; ++b) {
#pragma unroll
          for (int u = 0; u < 4; ++u) sv[u] += Lm[b * rm + ai_[u]] * ca[bs_[u] + b * inner];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = t0 + u * (int)blockDim.x;
          if (t < csz) cb[t] = sv[u];
        }
      }
      __syncthreads();
      double* tswap = ca; ca = cb; cb = tswap;
    }
  }
  if (CM) {
    for (int t = threadIdx.x; t < csz; t += blockDim.x) a.C0[t] = ca[t];
  } else if (ca != a.C0) {
    for (int t = threadIdx.x; t < csz; t += blockDim.x) a.C0[t] = ca[t];
  }
}

// Partial Gram sum_q w_q u_q u_q^T of slab rb of mode n (rows staged at Ul, weighted rows
// at Wl), upper triangle mirrored: stored to g, or added to g when acc (one block
// summing the slabs in order).
__device__ __forceinline__ void qr_slab_gram(const FQrArgs& a, int n, int rb, double* Ul, double* Wl, double* g,
                                             bool acc) {
  const int rn = a.r[n], ld = a.ldU[n];
  const int Nn = (int)a.N[n];
  const int rr = rn * rn;
  // the slab's rows u_q and w_q u_q, up to 8 loads in flight per thread
  const int q0 = rb * QR_ROWS, nr = min(QR_ROWS, Nn - q0);
  const double* U = a.U0[n] + (long long)q0 * ld;
  const double* w = a.w[n] + q0;
  const int tot = nr * rn;
  for (int base = 0; base < tot; base += 8 * (int)blockDim.x) {
    double v[8], wv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      const int q = t / rn;
      v[u] = t < tot ? U[q * ld + (t - q * rn)] : 0.0;
      wv[u] = t < tot ? w[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (t < tot) {
        Ul[t] = v[u];
        Wl[t] = wv[u] * v[u];
      }
    }
  }
  __syncthreads();
  // upper triangle (mirrored), four partial sums over the rows
  for (int e = threadIdx.x; e < rr; e += blockDim.x) {
    const int i = e / rn, j = e - (e / rn) * rn;
    if (j < i) continue;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = 0;
    for (; q + 4 <= nr; q += 4) {
      s0 += Wl[q * rn + i] * Ul[q * rn + j];
      s1 += Wl[(q + 1) * rn + i] * Ul[(q + 1) * rn + j];
      s2 += Wl[(q + 2) * rn + i] * Ul[(q + 2) * rn + j];
      s3 += Wl[(q + 3) * rn + i] * Ul[(q + 3) * rn + j];
    }
    for (; q < nr; ++q) s0 += Wl[q * rn + i] * Ul[q * rn + j];
    const double sv = (s0 + s1) + (s2 + s3);
    if (acc) {
      g[i * rn + j] += sv;
      if (j != i) g[j * rn + i] += sv;
    } else {
      g[i * rn + j] = sv;
      g[j * rn + i] = sv;
    }
  }
}

__device__ __forceinline__ void fqr_body(const FQrArgs& a, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int last, skip_s, ok_s[3];
  if (ctrl->hold) return;   // every block alike, so the completion count stays at zero
  // every block takes part in the completion count, even when there is nothing to do;
  // the flag is read once per block so that the whole block takes the same branch
  if (threadIdx.x == 0)
    skip_s = __hip_atomic_load(&ctrl->numeric, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  __syncthreads();
  const bool skip = skip_s != 0;
  const int r0 = a.r[0], r1 = a.r[1], r2 = a.r[2];
  const int rq = a.rmax;
  double* L0 = lds;                         // rq*rq each
  double* L1 = L0 + rq * rq;
  double* L2 = L1 + rq * rq;
  double* rdg = L2 + rq * rq;               // 3 x 64: reciprocal diagonals
  double* Gp = rdg + 3 * 64;                // FQR_GP (U_3 when it fits)
  double* X = Gp + FQR_GP;                  // the core (one or two buffers) when folded in LDS
  int csz = r0 * r1 * r2;
  const int N3 = (int)a.N[2], ld3 = a.ldU[2];
  const bool u3l = a.T3 && N3 * ld3 <= FQR_GP;
  if (a.whole) {
    // every slab in this block, the Grams summed in LDS in slab order
    if (ctrl->hold || skip) return;
    double* Ul = lds + a.slab_off;
    double* Wl = Ul + QR_ROWS * rq;
    for (int t = threadIdx.x; t < 3 * rq * rq; t += blockDim.x) L0[t] = 0.0;
    for (int n = 0; n < 3; ++n) {
      double* Ln = n == 0 ? L0 : (n == 1 ? L1 : L2);
      for (int rb = 0; rb < a.nb[n]; ++rb) {
        __syncthreads();
        qr_slab_gram(a, n, rb, Ul, Wl, Ln, true);
      }
    }
    for (int t = threadIdx.x; t < (a.core_in_lds ? csz : 0) + (u3l ? N3 * ld3 : 0); t += blockDim.x) {
      if (t < (a.core_in_lds ? csz : 0)) X[t] = a.C0[t];
      else Gp[t - (a.core_in_lds ? csz : 0)] = a.U0[2][t - (a.core_in_lds ? csz : 0)];
    }
    __syncthreads();
  } else {
    int rb;
    const int n = qr_mode(a, bx, rb);
    if (!skip) qr_slab_gram(a, n, rb, lds, lds + QR_ROWS * a.r[n], a.gpart[n] + (long long)rb * a.r[n] * a.r[n], false);
    // the last block factors the three Grams and folds the core
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned prev = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      last = (prev == (unsigned)(a.nb[0] + a.nb[1] + a.nb[2]) - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    // the fence orders the plain loads below after every block's stores of its partials
    __threadfence();
    if (threadIdx.x == 0) *a.counter = 0u;
    if (skip) return;
    {
      // one load phase: the summed Grams (partials in slab order), the core (when it is
      // folded in LDS) and U_3 (when it fits)
      const int g0 = r0 * r0, g1 = g0 + r1 * r1, g2 = g1 + r2 * r2;
      const int c1 = g2 + (a.core_in_lds ? csz : 0), tot = c1 + (u3l ? N3 * ld3 : 0);
      for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        if (t < g2) {
          const int m = t < g0 ? 0 : (t < g1 ? 1 : 2);
          const int e = t - (m == 0 ? 0 : (m == 1 ? g0 : g1));
          const int rr = m == 0 ? r0 * r0 : (m == 1 ? r1 * r1 : r2 * r2);
          const int nbm = m == 0 ? a.nb[0] : (m == 1 ? a.nb[1] : a.nb[2]);
          const double* gp = (m == 0 ? a.gpart[0] : (m == 1 ? a.gpart[1] : a.gpart[2])) + e;
          double sv = 0.0;
          int b = 0;
          for (; b + 8 <= nbm; b += 8) {
            double v[8];
  #pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = gp[(long long)(b + u) * rr];
  #pragma unroll
            for (int u = 0; u < 8; ++u) sv += v[u];
          }
          for (; b < nbm; ++b) sv += gp[(long long)b * rr];
          (m == 0 ? L0 : (m == 1 ? L1 : L2))[e] = sv;
        } else if (t < c1) {
          X[t - g2] = a.C0[t - g2];
        } else {
          Gp[t - c1] = a.U0[2][t - c1];
        }
      }
    }
    __syncthreads();
  }
  const int wid = threadIdx.x >> 6;
  if (wid < 3) {
    // wave m: L_m L_m^T = G_m and L_m^-1 (published for the post-step)
    const int rm = wid == 0 ? r0 : (wid == 1 ? r1 : r2);
    double* Lm = wid == 0 ? L0 : (wid == 1 ? L1 : L2);
    const bool ok = wave_chol_inv(Lm, rm, nullptr, nullptr);
    if (ok) wave_tri_inv_fast(Lm, wid == 0 ? a.Li[0] : (wid == 1 ? a.Li[1] : a.Li[2]), rm, rdg + 64 * wid);
    if ((threadIdx.x & 63) == 0) ok_s[wid] = ok ? 1 : 0;
  }
  __syncthreads();
  if (!(ok_s[0] && ok_s[1] && ok_s[2])) {
    if (threadIdx.x == 0) atomicOr(&ctrl->numeric, 2);
    return;
  }
  if (a.core_in_lds == 2) fold_core<2>(a, L0, L1, L2, Gp, X, csz, u3l);
  else if (a.core_in_lds == 1) fold_core<1>(a, L0, L1, L2, Gp, X, csz, u3l);
  else fold_core<0>(a, L0, L1, L2, Gp, X, csz, u3l);
}

__global__ void __launch_bounds__(256) k_fqr(FQrArgs a, CtrlState* ctrl) { fqr_body(a, ctrl, blockIdx.x); }

// The expansion rows E[a][i0 + il][i3] = sum_b U2r[il][b] T3[a][b][i3] for il < nr, the
// rows U2r (r2 a row) and T3 (r1 x r2 x N3) in LDS, the sum over b in order. The index
// decomposition takes small_div (a float reciprocal and one correction) below 2^22
// outputs, so that it does not outweigh the r2 multiply-adds of an output.
template <typename T>
__device__ __forceinline__ void expansion_rows(T* E, const double* U2r, const double* T3, int r1, int r2, int nr,
                                               int i0, long long N2, long long N3) {
  const long long tot = (long long)r1 * nr * N3;
  if (tot < (1LL << 22)) {
    const int n3 = (int)N3;
    const float i_n3 = 1.0f / (float)n3, i_nr = 1.0f / (float)nr;
    for (int t = threadIdx.x; t < (int)tot; t += blockDim.x) {
      const int q = small_div(t, n3, i_n3), i3 = t - q * n3;
      const int ai = small_div(q, nr, i_nr), il = q - ai * nr;
      const double* u2 = U2r + il * r2;
      const double* t3 = T3 + ai * r2 * n3 + i3;
      double sv = 0.0;
      for (int b = 0; b < r2; ++b) sv += u2[b] * t3[b * n3];
      E[((long long)ai * N2 + i0 + il) * N3 + i3] = (T)sv;
    }
  } else {
    for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
      const long long i3 = t % N3, q = t / N3;
      const int il = (int)(q % nr), ai = (int)(q / nr);
      const double* u2 = U2r + il * r2;
      const double* t3 = T3 + (long long)ai * r2 * N3 + i3;
      double sv = 0.0;
      for (int b = 0; b < r2; ++b) sv += u2[b] * t3[(long long)b * N3];
      E[((long long)ai * N2 + i0 + il) * N3 + i3] = (T)sv;
    }
  }
}

// ---------------------------------------------------------------- post-step
// Blocks [0, 3): for mode n at the new state: the core Gram (kept for the controller),
// its eigenvalues when asked for (core singular values) and the pseudo-inverse P_n for
// the next stage 1. Blocks [3, 3 + eblocks): the partial expansion E = C x_2 U_2 x_3 U_3
// used by the error pass, the mode-1 basis in the compute type and the weighted bases
// B_n of the next stage 1. A batch launches the two roles as separate kernels
// (ROLE_MODES: block bx is mode bx; ROLE_EXP: block bx is expansion block bx).
template <typename T, int ROLE>
__device__ __forceinline__ void fpost_body(const FPostArgs& a, CtrlState* ctrl, int bx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int pairs[TDB_RCAP + 2];
  __shared__ int order[TDB_RCAP];
  if (ctrl->hold) return;
  if (ROLE == ROLE_EXP || (ROLE == ROLE_ALL && (int)bx >= 3)) {
    // Block eb takes rows [eb*per_n, (eb+1)*per_n) of every mode, POST_CH at a time:
    // when the QR left U_n unnormalised, U_n <- U_n L_n^-T and the rows are written
    // back; then B_n = W_n U_n, the mode-1 basis in the compute type, and from the
    // mode-2 rows the expansion E[a][i2][i3] = sum_b U2[i2][b] T3[a][b][i3] with
    // T3[a][b][i3] = sum_c C[a][b][c] U3[i3][c].
    const int eb = ROLE == ROLE_EXP ? bx : bx - 3;
    const int r1 = a.r[0], r2 = a.r[1], r3 = a.r[2];
    const long long N2 = a.N[1], N3 = a.N[2];
    const int rq = a.rmax;
    double* T3 = lds;                                   // r1*r2*N3
    double* Lil = T3 + (long long)r1 * r2 * N3;         // rq*rq
    double* Ul = Lil + rq * rq;                         // POST_CH * rq (raw rows)
    double* Un = Ul + POST_CH * rq;                     // POST_CH * rq (normalised rows)
    // a step that was not applied (numerical event or non-finite data) skipped the QR:
    // U_n needs no normalisation and T3 is formed here from the kept state. NUM_NEXT
    // is left out: this kernel's own mode blocks may be raising it meanwhile.
    const bool kept = (ctrl->numeric & ~NUM_NEXT) != 0;
    const bool norm = a.Li[0] != nullptr && !kept;
    const long long per2 = (N2 + a.eblocks - 1) / a.eblocks;
    const bool erows = (long long)eb * per2 < N2;
    if (erows) {
      if (a.T3 && !kept) {
        g2l(T3, a.T3, r1 * r2 * (int)N3);
      } else {
        for (long long t = threadIdx.x; t < (long long)r1 * r2 * N3; t += blockDim.x) {
          const long long i3 = t % N3, ab = t / N3;
          const double* cr = a.C + ab * r3;
          const double* u3 = a.U[2] + i3 * a.ldU[2];
          double sv = 0.0;
          for (int c = 0; c < r3; ++c) sv += cr[c] * u3[c];
          T3[t] = sv;
        }
      }
    }
    if (a.stage_all) {
      // every input of the block in one load phase: T3 (already in LDS), the three
      // L^-1 and this block's rows of all three modes
      // (per-mode values in named scalars: a runtime mode index picks among them)
      double* base = Lil;
      int ia0, ia1, ia2, nr0, nr1, nr2;
      {
        int* iav[3] = {&ia0, &ia1, &ia2};
        int* nrv[3] = {&nr0, &nr1, &nr2};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const long long per = (a.N[m] + a.eblocks - 1) / a.eblocks;
          const long long ia = (long long)eb * per, ib = min(a.N[m], ia + per);
          *iav[m] = (int)ia;
          *nrv[m] = ia < ib ? (int)(ib - ia) : 0;
        }
      }
      const int q0 = a.r[0], q1 = a.r[1], q2 = a.r[2];
      const int l0 = norm ? q0 * q0 : 0, l1 = norm ? q1 * q1 : 0, l2 = norm ? q2 * q2 : 0;
      const int e0 = nr0 * q0, e1 = nr1 * q1, e2 = nr2 * q2;
      const int oL0 = 0, oL1 = l0, oL2 = l0 + l1;
      const int oU0 = l0 + l1 + l2, oU1 = oU0 + e0, oU2 = oU1 + e1;
      const int tot = oU2 + e2, nsum = e0 + e1 + e2;
      const int oN0 = tot, oN1 = tot + e0, oN2 = tot + e0 + e1;
      const double* Li0 = a.Li[0];
      const double* Li1 = a.Li[1];
      const double* Li2 = a.Li[2];
      const double* Ug0 = a.U[0] + (long long)ia0 * a.ldU[0];
      const double* Ug1 = a.U[1] + (long long)ia1 * a.ldU[1];
      const double* Ug2 = a.U[2] + (long long)ia2 * a.ldU[2];
      const int ld0 = a.ldU[0], ld1 = a.ldU[1], ld2 = a.ldU[2];
      for (int b0 = 0; b0 < tot; b0 += 16 * (int)blockDim.x) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = b0 + u * (int)blockDim.x + (int)threadIdx.x;
          double x = 0.0;
          if (t < tot) {
            if (t < oL1) x = Li0[t];
            else if (t < oL2) x = Li1[t - oL1];
            else if (t < oU0) x = Li2[t - oL2];
            else if (t < oU1) { const int e = t - oU0, q = e / q0; x = Ug0[(long long)q * ld0 + (e - q * q0)]; }
            else if (t < oU2) { const int e = t - oU1, q = e / q1; x = Ug1[(long long)q * ld1 + (e - q * q1)]; }
            else { const int e = t - oU2, q = e / q2; x = Ug2[(long long)q * ld2 + (e - q * q2)]; }
          }
          v[u] = x;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = b0 + u * (int)blockDim.x + (int)threadIdx.x;
          if (t < tot) base[t] = v[u];
        }
      }
      __syncthreads();
      if (norm) {
        // (U L^-T)[q][j] = sum_{k <= j} U[q][k] L^-1[j][k], four entries per thread at a time
        for (int t0 = threadIdx.x; t0 < nsum; t0 += 4 * (int)blockDim.x) {
          // entry u: row offset ur, L^-1 row offset lr, column jj, output index on
          int ur[4], lr[4], jj[4], on[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int t = min(t0 + u * (int)blockDim.x, nsum - 1);
            const int m = t < e0 ? 0 : (t < e0 + e1 ? 1 : 2);
            const int e = t - (m == 0 ? 0 : (m == 1 ? e0 : e0 + e1));
            const int rm = m == 0 ? q0 : (m == 1 ? q1 : q2);
            const int q = e / rm, j = e - q * rm;
            jj[u] = j;
            ur[u] = (m == 0 ? oU0 : (m == 1 ? oU1 : oU2)) + q * rm;
            lr[u] = (m == 0 ? oL0 : (m == 1 ? oL1 : oL2)) + j * rm;
            on[u] = (m == 0 ? oN0 : (m == 1 ? oN1 : oN2)) + e;
          }
          double sv[4] = {0.0, 0.0, 0.0, 0.0};
          const int kmax = max(max(jj[0], jj[1]), max(jj[2], jj[3]));
          for (int k = 0; k <= kmax; ++k) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (k <= jj[u]) sv[u] += base[ur[u] + k] * base[lr[u] + k];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (t0 + u * (int)blockDim.x < nsum) base[on[u]] = sv[u];
        }
        // (the normalised rows go back to U_n with the other stores below: a barrier
        // after global stores would wait for them)
        __syncthreads();
      }
      // the normalised rows
      const int oR0 = norm ? oN0 : oU0, oR1 = norm ? oN1 : oU1, oR2 = norm ? oN2 : oU2;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int rm = m == 0 ? q0 : (m == 1 ? q1 : q2);
        const int n_e = m == 0 ? e0 : (m == 1 ? e1 : e2);
        const int ia = m == 0 ? ia0 : (m == 1 ? ia1 : ia2);
        const double* Ur = base + (m == 0 ? oR0 : (m == 1 ? oR1 : oR2));
        const double* w = a.w[m] + ia;
        T* B = static_cast<T*>(a.B[m]) + (long long)ia * rm;
        const int ld = m == 0 ? ld0 : (m == 1 ? ld1 : ld2);
        double* Uw = norm ? a.Uw[m] + (long long)ia * ld : nullptr;
        for (int t = threadIdx.x; t < n_e; t += blockDim.x) {
          const int q = t / rm;
          const double u = Ur[t];
          B[t] = (T)(w[q] * u);
          if (norm) Uw[(long long)q * ld + (t - q * rm)] = u;
        }
        if (m == 0) {
          T* U1c = static_cast<T*>(a.U1c) + (long long)ia * rm;
          for (int t = threadIdx.x; t < n_e; t += blockDim.x) U1c[t] = (T)Ur[t];
        }
      }
      if (nr1 > 0) expansion_rows<T>(static_cast<T*>(a.E), base + oR1, T3, r1, r2, nr1, ia1, N2, N3);
      return;
    }
    for (int m = 0; m < 3; ++m) {
      const int rm = a.r[m], ld = a.ldU[m];
      const long long per = (a.N[m] + a.eblocks - 1) / a.eblocks;
      const long long ia = (long long)eb * per, ib = min(a.N[m], ia + per);
      if (ia >= ib) continue;
      if (norm) {
        __syncthreads();
        g2l(Lil, a.Li[m], rm * rm);
      }
      const double* w = a.w[m];
      T* B = static_cast<T*>(a.B[m]);
      for (long long c0 = ia; c0 < ib; c0 += POST_CH) {
        const int nr = (int)min((long long)POST_CH, ib - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < nr * rm; t += blockDim.x) {
          const int q = t / rm;
          Ul[t] = a.U[m][(c0 + q) * ld + (t - q * rm)];
        }
        __syncthreads();
        const double* Uc = Ul;
        if (norm) {
          // (U L^-T)[q][j] = sum_{k <= j} U[q][k] L^-1[j][k], four entries per thread at a time
          for (int t0 = threadIdx.x; t0 < nr * rm; t0 += 4 * (int)blockDim.x) {
            int qq[4], jj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int t = min(t0 + u * (int)blockDim.x, nr * rm - 1);
              qq[u] = t / rm;
              jj[u] = t - qq[u] * rm;
            }
            double sv[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < rm; ++k) {
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (k <= jj[u]) sv[u] += Ul[qq[u] * rm + k] * Lil[jj[u] * rm + k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int t = t0 + u * (int)blockDim.x;
              if (t < nr * rm) {
                Un[t] = sv[u];
                a.Uw[m][(c0 + qq[u]) * ld + jj[u]] = sv[u];
              }
            }
          }
          __syncthreads();
          Uc = Un;
        }
        for (int t = threadIdx.x; t < nr * rm; t += blockDim.x) {
          const int q = t / rm;
          B[(c0 + q) * rm + (t - q * rm)] = (T)(w[c0 + q] * Uc[t]);
        }
        if (m == 0) {
          T* U1c = static_cast<T*>(a.U1c);
          for (int t = threadIdx.x; t < nr * rm; t += blockDim.x) U1c[c0 * rm + t] = (T)Uc[t];
        }
        if (m == 1) expansion_rows<T>(static_cast<T*>(a.E), Uc, T3, r1, r2, nr, (int)c0, N2, N3);
      }
    }
    return;
  }
  if (ROLE == ROLE_EXP) return;
  const int n = bx;
  const int rn = a.r[n];
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
  double* ws = Gi + rq * rq;                 // 4*rq
  double* lam = ws + 4 * rq;                 // rq
  double* Gp = lam + rq;                     // FQR_GP partial blocks
  double* Cl = Gp + FQR_GP;
  __shared__ int ok_s;
  // the core from LDS or from global memory (separate instances: fixed address spaces)
  auto modes = [&](const double* Csrc) {
    gram_from(Csrc, rn, R, inner, G, Gp);
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
      if (need_p) ok = wave_chol_inv(G, rn, Li, Gi);
      if (threadIdx.x == 0) {
        ok_s = ok ? 1 : 0;
        if (!ok) atomicOr(&ctrl->numeric, 4);
      }
    }
    __syncthreads();
    if (!need_p || !ok_s) return;
    write_p<T>(Csrc, Gi, rn, R, inner, static_cast<T*>(a.P[n]));
  };
  if (a.core_in_lds) {
    g2l(Cl, a.C, (int)csz);
    __syncthreads();
    modes(Cl);
  } else {
    modes(a.C);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fpost(FPostArgs a, CtrlState* ctrl) {
  fpost_body<T, ROLE_ALL>(a, ctrl, blockIdx.x);
}

// ---------------------------------------------------------------- error pass
// Tile = T1 slabs of mode 1. rec[i1][j] = sum_a U1[i1][a] E[a][j] (j over modes 2,3);
// partial sums of w (V - rec)^2 and w V^2 in FP64; the last block reduces them and
// runs the controller decision.
template <typename TD, typename T>
__device__ __forceinline__ void ferr_body(const FErrArgs& a, int bx, int by, int gx) {
  __shared__ double red[16];
  // U1 rows of the slab, row q at q * TDB_RCAP, zero past r1 and past the slab's rows
  __shared__ T U1s[FERR_T1 * TDB_RCAP];
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
  const TD* V = static_cast<const TD*>(a.V);
  {
    T x[FERR_T1 * TDB_RCAP / 256];
#pragma unroll
    for (int u = 0; u < FERR_T1 * TDB_RCAP / 256; ++u) {
      const int t = u * 256 + threadIdx.x;
      const int q = t / TDB_RCAP, ai = t - q * TDB_RCAP;
      x[u] = static_cast<const T*>(a.U1c)[(long long)(i1_0 + min(q, n1 - 1)) * r1 + min(ai, r1 - 1)];
    }
#pragma unroll
    for (int u = 0; u < FERR_T1 * TDB_RCAP / 256; ++u) {
      const int t = u * 256 + threadIdx.x;
      const int q = t / TDB_RCAP, ai = t - q * TDB_RCAP;
      U1s[t] = q < n1 && ai < r1 ? x[u] : (T)0;
    }
  }
  __syncthreads();
  double se = 0.0, sv = 0.0;
  constexpr int EC = 16;        // entries of E per batch of loads
  for (long long j = (long long)bx * blockDim.x + threadIdx.x; j < M; j += (long long)gx * blockDim.x) {
    // the slab's snapshot values first (rows past the slab load the last row and are
    // dropped), then E in batches of EC, the next batch in flight while one is used
    TD vv[FERR_T1];
#pragma unroll
    for (int q = 0; q < FERR_T1; ++q) vv[q] = V[(long long)(i1_0 + min(q, n1 - 1)) * M + j];
    const double w23 = a.w23[j];
    T e[EC];
    auto eload = [&](int a0) {
#pragma unroll
      for (int k = 0; k < EC; ++k) e[k] = E[(long long)min(a0 + k, r1 - 1) * M + j];
    };
    T acc[FERR_T1];
#pragma unroll
    for (int q = 0; q < FERR_T1; ++q) acc[q] = (T)0;
    eload(0);
    for (int a0 = 0; a0 < r1; a0 += EC) {
      T cur[EC];
#pragma unroll
      for (int k = 0; k < EC; ++k) cur[k] = e[k];
      if (a0 + EC < r1) eload(a0 + EC);
#pragma unroll
      for (int k = 0; k < EC; ++k)
#pragma unroll
        for (int q = 0; q < FERR_T1; ++q) acc[q] += U1s[q * TDB_RCAP + a0 + k] * cur[k];
    }
#pragma unroll
    for (int q = 0; q < FERR_T1; ++q) {
      if (q < n1) {
        const double d = (double)((T)vv[q] - acc[q]);
        const double ww = a.w1[i1_0 + q] * w23;
        se += ww * d * d;
        sv += ww * (double)vv[q] * (double)vv[q];
      }
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
  if (ctrl->hold) return;
  ferr_body<TD, T>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

// Controller of the fused path: the decision up to the removal test; only when that
// test has to run are the singular values of the core unfoldings formed, one wave per
// mode, from the Grams kept by the post-step kernel.
// Whether the symmetric n x n matrix A (LDS, row-major) minus tau I has an eigenvalue
// at or below zero: its Cholesky factorisation, right-looking, meets a pivot that is not
// positive. One wave, lanes in step; A is overwritten.
__device__ __forceinline__ bool wave_shifted_not_pd(double* A, int n, double tau) {
  const int l = threadIdx.x & 63;
  for (int t = l; t < n; t += 64) A[t * n + t] -= tau;
  wave_fence();
  for (int k = 0; k < n; ++k) {
    const double piv = A[k * n + k];
    if (!(piv > 0.0)) return true;
    const double d = sqrt(piv);
    for (int i = k + 1 + l; i < n; i += 64) A[i * n + k] /= d;
    wave_fence();
    const int m = n - k - 1;
    for (int t = l; t < m * m; t += 64) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) A[i * n + j] -= A[i * n + k] * A[j * n + k];
    }
    wave_fence();
  }
  return false;
}

__device__ __forceinline__ void fused_decide(CtrlState* ctrl, const double* const* G, int rmax, const int* skip,
                                             const int* would_skip, const float* yhat) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  __shared__ int need;
  if (threadIdx.x == 0) {
    ctrl->gated = (skip && *skip) ? 1 : 0;
    ctrl->would_skip = would_skip ? *would_skip : 0;
    ctrl->eps_pred = (yhat && isfinite(*yhat)) ? pow(10.0, (double)*yhat) : __builtin_nan("");
    if (ctrl->gated && !(ctrl->numeric & NUM_NONFINITE)) {
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
  // The removal test of the controller: some mode whose weakest direction fits the
  // budget with the error, eps^2 + sigma_min(C_(n))^2 <= B. sigma_min^2 is the smallest
  // eigenvalue of the core Gram G_n, so the test is whether G_n - (B - eps^2) I has an
  // eigenvalue at or below zero: whether its Cholesky factorisation meets a pivot that
  // is not positive. One wave per mode.
  __shared__ int hit[3];
  if (threadIdx.x < 3) hit[threadIdx.x] = 0;
  __syncthreads();
  const double B = ctrl->gamma_th > 0.0 ? (1.0 - ctrl->gamma_th / 100.0) * ctrl->nu2
                                        : 0.25 * ctrl->eps_th * ctrl->eps_th;
  const double tau = B - ctrl->eps * ctrl->eps;
  const int w = threadIdx.x >> 6;
  if (w < 3 && G[w] && tau >= 0.0) {
    const int rn = ctrl->ranks[w];
    double* A = lds + w * (rmax * rmax + 5 * rmax);
    for (int t = threadIdx.x & 63; t < rn * rn; t += 64) A[t] = G[w][t];
    wave_fence();
    const bool not_pd = wave_shifted_not_pd(A, rn, tau);
    if ((threadIdx.x & 63) == 0) hit[w] = not_pd ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && (hit[0] || hit[1] || hit[2])) ctrl->decision = DEC_REMOVE;
}

// One block: fixed-order sum of the error-pass partials, then the controller. A
// decision other than none raises the hold flag for the host.
// The controller state copied by the whole block into its pinned host mirror, then
// the step's sequence number into its pinned word: the host spins on that word and
// reads the mirror once it holds the number it expects.
__device__ __forceinline__ void mirror_ctrl(const FErrArgs& a, const CtrlState* src) {
  static_assert(sizeof(CtrlState) % 8 == 0, "controller state copied in 8-byte words");
  if (!a.mirror) return;
  __syncthreads();
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(a.mirror);
  for (int i = threadIdx.x; i < (int)(sizeof(CtrlState) / 8); i += blockDim.x) d[i] = s[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0 && a.seq) {
    *reinterpret_cast<volatile unsigned long long*>(a.seq) = a.seq_val;
    __threadfence_system();
  }
}

// The controller state copied between global memory and LDS by the whole block in
// 8-byte words: the decision then reads and writes its few dozen fields in LDS instead
// of one dependent global round trip each.
__device__ __forceinline__ void ctrl_copy(CtrlState* dst, const CtrlState* src) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(CtrlState) / 8); i += blockDim.x) d[i] = q[i];
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_ferr_final(FErrArgs a, CtrlState* gctrl) {
  __shared__ double red[16];
  __shared__ CtrlState cs;
  ctrl_copy(&cs, gctrl);
  CtrlState* ctrl = &cs;
  if (ctrl->hold) {
    mirror_ctrl(a, ctrl);
    return;
  }
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
  // a discarded step (non-finite data) needs nothing from the host before the next one
  if (threadIdx.x == 0) ctrl->hold = (ctrl->decision != DEC_NONE && ctrl->decision != DEC_NONFINITE) ? 1 : 0;
  __syncthreads();
  ctrl_copy(gctrl, ctrl);
  mirror_ctrl(a, ctrl);
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
  hipError_t e = lds_limit((const void*)k_ffinish<T>, lds);
  if (e != hipSuccess) return e;
  const int blocks = a.rowblocks + (a.stage == 1 ? 3 : 0);
  hipLaunchKernelGGL(k_ffinish<T>, dim3(blocks), dim3(256), lds, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_ffinish<float>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);
template hipError_t launch_ffinish<double>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);

template <typename T>
hipError_t launch_fmprep(const FFinishArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = lds_limit((const void*)k_fmprep<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fmprep<T>, dim3(3), dim3(256), lds, s, a, c);
  return hipGetLastError();
}
template hipError_t launch_fmprep<float>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);
template hipError_t launch_fmprep<double>(const FFinishArgs&, size_t, CtrlState*, hipStream_t);

__global__ void __launch_bounds__(256) k_euler_commit(CommitArgs a, CtrlState* ctrl) {
  if (ctrl->hold || ctrl->numeric) return;
  const long long gs = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long t = t0; t < a.csz; t += gs) a.C0[t] = a.Cs[t];
  for (int n = 0; n < a.p; ++n) {
    const int rn = a.r[n], ld = a.ldU[n];
    const long long tot = a.N[n] * rn;
    for (long long t = t0; t < tot; t += gs) {
      const long long i = t / rn;
      const long long o = i * ld + (t - i * rn);
      a.U0[n][o] = a.Us[n][o];
    }
  }
}

hipError_t launch_euler_commit(const CommitArgs& a, CtrlState* c, hipStream_t s) {
  long long m = a.csz;
  for (int n = 0; n < a.p; ++n) m = std::max(m, a.N[n] * a.r[n]);
  const int blocks = (int)std::max<long long>(1, std::min<long long>(1024, (m + 255) / 256));
  hipLaunchKernelGGL(k_euler_commit, dim3(blocks), dim3(256), 0, s, a, c);
  return hipGetLastError();
}

hipError_t launch_fqr(const FQrArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = lds_limit((const void*)k_fqr, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fqr, dim3(a.nb[0] + a.nb[1] + a.nb[2]), dim3(256), lds, s, a, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fpost(const FPostArgs& a, size_t lds, CtrlState* c, hipStream_t s) {
  hipError_t e = lds_limit((const void*)k_fpost<T>, lds);
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
  e = lds_limit((const void*)k_ferr_final, fl);
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

template <typename T, int ROLE>
__global__ void __launch_bounds__(256) kb_ffinish(const FFinishArgs* __restrict__ tab, CtrlState* const* ctab,
                                                  BatchMap m, int stage) {
  const int s = m.sid[blockIdx.x];
  ffinish_body<T, ROLE>(tab[s], stage, ctab[s], blockIdx.x - m.start[s]);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_fmprep(const FFinishArgs* __restrict__ tab, CtrlState* const* ctab,
                                                 BatchMap m, int stage) {
  const int s = m.sid[blockIdx.x];
  fmprep_body<T>(tab[s], stage, ctab[s], blockIdx.x - m.start[s]);
}

// A batch's QR takes one workgroup per stream (all its slabs): 1024 threads, so that the
// slab loads, Grams and the fold of a stream are spread over sixteen waves.
__global__ void __launch_bounds__(1024) kb_fqr(const FQrArgs* __restrict__ tab, CtrlState* const* ctab, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  fqr_body(tab[s], ctab[s], blockIdx.x - m.start[s]);
}

template <typename T, int ROLE>
__global__ void __launch_bounds__(256) kb_fpost(const FPostArgs* __restrict__ tab, CtrlState* const* ctab,
                                                BatchMap m) {
  const int s = m.sid[blockIdx.x];
  fpost_body<T, ROLE>(tab[s], ctab[s], blockIdx.x - m.start[s]);
}

template <typename TD, typename T>
__global__ void __launch_bounds__(256) kb_ferr(const FErrArgs* __restrict__ tab, const void* const* v1, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  FErrArgs a = tab[s];
  if (a.hold && *gmem(a.hold)) return;   // a decision awaits the host
  a.V = v1[s];
  const int l = blockIdx.x - m.start[s];
  ferr_body<TD, T>(a, l % a.gx, l / a.gx, a.gx);
}

// One block per stream: the fixed-order sum of that stream's error-pass partials,
// its controller decision, and the summary the host reads. A decision that needs the
// host (any but none and a discarded step) raises the stream's hold flag: the kernels
// of steps enqueued behind it do nothing for that stream until the host has acted. A
// stream found held reports nothing (its step did not run). `out` may be pinned host
// memory: every block counts itself done after its summary is visible system-wide, and
// the last one resets the count and advances *seq, on which the host waits.
__global__ void __launch_bounds__(256) kb_ferr_final(const FErrArgs* __restrict__ tab, CtrlState* const* ctab,
                                                     BatchSummary* out, unsigned* counter,
                                                     unsigned long long* seq) {
  __shared__ double red[16];
  __shared__ CtrlState cs;
  const int s = blockIdx.x;
  CtrlState* gctrl = ctab[s];
  ctrl_copy(&cs, gctrl);
  CtrlState* ctrl = &cs;
  const int held = ctrl->hold;
  if (!held) {
    const double* part = tab[s].part;
    const int nb = tab[s].gx * tab[s].gy;
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
      ctrl->hold = (ctrl->decision != DEC_NONE && ctrl->decision != DEC_NONFINITE) ? 1 : 0;
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
    __syncthreads();
    ctrl_copy(gctrl, ctrl);
  }
  if (threadIdx.x == 0 && counter) {
    __threadfence_system();
    if (atomicAdd(counter, 1u) == gridDim.x - 1) {
      atomicExch(counter, 0u);
      __threadfence_system();
      volatile unsigned long long* w = seq;
      *w = *w + 1;
      __threadfence_system();
    }
  }
}

// The step's snapshot pointers from the pinned tables the host filled for it into the
// device tables the kernels read.
__global__ void kb_fetch_ptrs(const void* const* h1, const void* const* h0, const void** d1, const void** d0,
                              int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    d1[i] = h1[i];
    d0[i] = h0[i];
  }
}

// Streams with mask[i] set are held for a re-run of the other streams' step: their
// hold flag is saved and raised (restore = 0), or put back (restore = 1).
__global__ void kb_hold_mask(CtrlState* const* ctab, const int* mask, int* save, int n, int restore) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!mask[i]) continue;
    if (restore) {
      ctab[i]->hold = save[i];
    } else {
      save[i] = ctab[i]->hold;
      ctab[i]->hold = 1;
    }
  }
}

hipError_t launch_batch_fetch_ptrs(const void* const* h1, const void* const* h0, const void** d1, const void** d0,
                                   int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_fetch_ptrs, dim3((n + 255) / 256), dim3(256), 0, s, h1, h0, d1, d0, n);
  return hipGetLastError();
}

hipError_t launch_batch_hold_mask(CtrlState* const* ctab, const int* mask, int* save, int n, int restore,
                                  hipStream_t s) {
  hipLaunchKernelGGL(kb_hold_mask, dim3((n + 255) / 256), dim3(256), 0, s, ctab, mask, save, n, restore);
  return hipGetLastError();
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
                                size_t lds, int role, hipStream_t s) {
  const void* f = role == ROLE_PINV ? (const void*)kb_ffinish<T, ROLE_PINV> : (const void*)kb_ffinish<T, ROLE_ROWS>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (role == ROLE_PINV)
    hipLaunchKernelGGL((kb_ffinish<T, ROLE_PINV>), dim3(blocks), dim3(256), lds, s, tab, ctab, m, stage);
  else
    hipLaunchKernelGGL((kb_ffinish<T, ROLE_ROWS>), dim3(blocks), dim3(256), lds, s, tab, ctab, m, stage);
  return hipGetLastError();
}
template hipError_t launch_batch_ffinish<float>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                                int, hipStream_t);
template hipError_t launch_batch_ffinish<double>(const FFinishArgs*, CtrlState* const*, BatchMap, int, int, size_t,
                                                 int, hipStream_t);

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
  hipLaunchKernelGGL(kb_fqr, dim3(blocks), dim3(1024), lds, s, tab, ctab, m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_fpost(const FPostArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, size_t lds,
                              int role, hipStream_t s) {
  const void* f = role == ROLE_EXP ? (const void*)kb_fpost<T, ROLE_EXP> : (const void*)kb_fpost<T, ROLE_MODES>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (role == ROLE_EXP)
    hipLaunchKernelGGL((kb_fpost<T, ROLE_EXP>), dim3(blocks), dim3(256), lds, s, tab, ctab, m);
  else
    hipLaunchKernelGGL((kb_fpost<T, ROLE_MODES>), dim3(blocks), dim3(256), lds, s, tab, ctab, m);
  return hipGetLastError();
}
template hipError_t launch_batch_fpost<float>(const FPostArgs*, CtrlState* const*, BatchMap, int, size_t, int,
                                              hipStream_t);
template hipError_t launch_batch_fpost<double>(const FPostArgs*, CtrlState* const*, BatchMap, int, size_t, int,
                                               hipStream_t);

// Column-block error pass of batches (eq. (error)): block bx of a stream takes the
// FEC_COLS consecutive columns j = FEC_COLS bx + t of the mode-1 unfolding
// (j = i2*N3 + i3) with all N1 rows. Thread t keeps its column of E (a < r1, zero up to
// R1C) in registers; the rows of U1 (compute type) and w1 are staged in LDS FEC_ROWS at
// a time and read as broadcasts; the snapshot rows stream through, the next FEC_PF rows
// in flight while FEC_PF are used (loads past the last row clamp to it, so every load
// is issued on every path). A column's sums over its rows are w1[i] d_i^2 and
// w1[i] v_i^2 in FP64, scaled by w23[j] once; the block's fixed-order sum is its
// partial.
#define FEC_ROWS 128
#define FEC_PF 8
template <typename TD, typename T, int R1C>
__global__ void __launch_bounds__(FEC_COLS) kb_ferr_cols(const FErrArgs* __restrict__ tab, const void* const* v1,
                                                         BatchMap m) {
  __shared__ double red[16];
  __shared__ __align__(16) T U1s[FEC_ROWS * R1C];
  __shared__ double w1s[FEC_ROWS];
  const int s = m.sid[blockIdx.x];
  const FErrArgs a = tab[s];
  if (a.hold && *gmem(a.hold)) return;   // a decision awaits the host
  const int bx = blockIdx.x - m.start[s];
  TDB_GLOBAL double* part = gmem(a.part);
  if (a.skip && *gmem(a.skip)) {
    // the learned gate skips this step's pass
    if (threadIdx.x == 0) {
      part[2 * bx] = 0.0;
      part[2 * bx + 1] = 0.0;
    }
    return;
  }
  const long long M = a.M;
  const int N1 = a.N1, r1 = a.r1, tid = threadIdx.x;
  const long long j = (long long)bx * FEC_COLS + tid;
  const bool jok = j < M;
  const long long jc = jok ? j : M - 1;
  const TDB_GLOBAL TD* V = gmem(static_cast<const TD*>(v1[s])) + jc;
  const TDB_GLOBAL T* E = gmem(static_cast<const T*>(a.E)) + jc;
  const TDB_GLOBAL T* U1 = gmem(static_cast<const T*>(a.U1c));
  const TDB_GLOBAL double* w1 = gmem(a.w1);
  T e[R1C];
#pragma unroll
  for (int k = 0; k < R1C; ++k) {
    const T x = E[(long long)min(k, r1 - 1) * M];
    e[k] = k < r1 ? x : (T)0;
  }
  const double w23j = gmem(a.w23)[jc];
  double se = 0.0, sv = 0.0;
  TD va[FEC_PF], vb[FEC_PF];
  auto vload = [&](TD (&vv)[FEC_PF], int i0) {
#pragma unroll
    for (int q = 0; q < FEC_PF; ++q) vv[q] = V[(long long)min(i0 + q, N1 - 1) * M];
  };
  auto rows = [&](const TD (&vv)[FEC_PF], int g0, int nr) {
#pragma unroll
    for (int q = 0; q < FEC_PF; ++q) {
      const int il = g0 + q;
      if (il < nr) {
        const T* u = U1s + il * R1C;
        T x = (T)0;
#pragma unroll
        for (int k = 0; k < R1C; ++k) x += u[k] * e[k];
        const T v = (T)vv[q];
        const T d = v - x;
        const double wi = w1s[il];
        se += wi * (double)(d * d);
        sv += wi * (double)(v * v);
      }
    }
  };
  vload(va, 0);
  for (int c0 = 0; c0 < N1; c0 += FEC_ROWS) {
    const int nr = min(FEC_ROWS, N1 - c0);
    __syncthreads();
    {
      // rows c0 .. c0+nr of U1, zero-padded to R1C columns, eight loads in flight
      const int ne = nr * R1C;
      for (int t0 = 0; t0 < ne; t0 += 8 * FEC_COLS) {
        T x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = min(t0 + u * FEC_COLS + tid, ne - 1);
          const int q = t / R1C, k = t - (t / R1C) * R1C;
          x[u] = U1[(long long)(c0 + q) * r1 + min(k, r1 - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = t0 + u * FEC_COLS + tid;
          if (t < ne) U1s[t] = (t - (t / R1C) * R1C) < r1 ? x[u] : (T)0;
        }
      }
      if (tid < nr) w1s[tid] = w1[c0 + tid];
    }
    __syncthreads();
    // a full chunk ends with the first rows of the next one in flight in va
    for (int g0 = 0; g0 < nr; g0 += 2 * FEC_PF) {
      vload(vb, c0 + g0 + FEC_PF);
      rows(va, g0, nr);
      vload(va, c0 + g0 + 2 * FEC_PF);
      rows(vb, g0 + FEC_PF, nr);
    }
  }
  se = jok ? se * w23j : 0.0;
  sv = jok ? sv * w23j : 0.0;
  se = block_sum(se, red);
  sv = block_sum(sv, red);
  if (tid == 0) {
    part[2 * bx] = se;
    part[2 * bx + 1] = sv;
  }
}

// The same column-block error pass with the reconstruction U1 E on the matrix cores
// (FP32 compute): wave w of block bx takes the 64 columns FEC_COLS bx + 64 w + 16 c + q
// (c < 4 groups of 16), and each 16-row block of the mode-1 unfolding is reconstructed
// as four 16 x 16 FP32 products over K = R1C (16x16x4 instructions: lane (q, g) feeds
// U1[row q][4 kc + g] and E[4 kc + g][column q] and receives rows 4 g .. 4 g + 3 of
// column q). E stays in registers, the U1 rows and w1 are staged in LDS FEC_ROWS at a
// time, and the snapshot values of the next 16-row block are in flight while one is
// used. Sums as in kb_ferr_cols: w1[i] d^2 and w1[i] v^2 in FP64 per column, scaled by
// w23[j], then the block's fixed-order sum.
typedef float fec4 __attribute__((ext_vector_type(4)));
template <typename TD, int R1C>
__global__ void __launch_bounds__(FEC_COLS) kb_ferr_mf(const FErrArgs* __restrict__ tab, const void* const* v1,
                                                       BatchMap m) {
  constexpr int KC = R1C / 4;
  __shared__ double red[16];
  __shared__ __align__(16) float U1s[FEC_ROWS * R1C];
  __shared__ double w1s[FEC_ROWS];
  const int s = m.sid[blockIdx.x];
  const FErrArgs a = tab[s];
  if (a.hold && *gmem(a.hold)) return;   // a decision awaits the host
  const int bx = blockIdx.x - m.start[s];
  TDB_GLOBAL double* part = gmem(a.part);
  if (a.skip && *gmem(a.skip)) {
    // the learned gate skips this step's pass
    if (threadIdx.x == 0) {
      part[2 * bx] = 0.0;
      part[2 * bx + 1] = 0.0;
    }
    return;
  }
  const long long M = a.M;
  const int N1 = a.N1, r1 = a.r1, tid = threadIdx.x;
  const int lane = tid & 63, q = lane & 15, g = lane >> 4, wv = tid >> 6;
  long long jc[4];
  bool jok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long long j = (long long)bx * FEC_COLS + 64 * wv + 16 * c + q;
    jok[c] = j < M;
    jc[c] = jok[c] ? j : M - 1;
  }
  const TDB_GLOBAL TD* V = gmem(static_cast<const TD*>(v1[s]));
  const TDB_GLOBAL float* E = gmem(static_cast<const float*>(a.E));
  const TDB_GLOBAL float* U1 = gmem(static_cast<const float*>(a.U1c));
  const TDB_GLOBAL double* w1 = gmem(a.w1);
  float eB[4][KC];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int k = 4 * kc + g;
      const float x = E[(long long)min(k, r1 - 1) * M + jc[c]];
      eB[c][kc] = k < r1 ? x : 0.0f;
    }
  double w23[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) w23[c] = gmem(a.w23)[jc[c]];
  double se[4] = {0.0, 0.0, 0.0, 0.0}, sv[4] = {0.0, 0.0, 0.0, 0.0};
  // snapshot values of the 16-row block from row i0: rows i0 + 4g + ii of the four columns
  auto vload = [&](float (&vv)[16], int i0) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
        vv[4 * c + ii] = (float)V[(long long)min(i0 + 4 * g + ii, N1 - 1) * M + jc[c]];
  };
  // the 16-row block rb of the staged chunk from row c0 (its values in vv)
  auto block = [&](const float (&vv)[16], int c0, int rb) {
    fec4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = fec4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const float av = U1s[(16 * rb + q) * R1C + 4 * kc + g];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, eB[c][kc], acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int rl = 16 * rb + 4 * g + ii;
      if (c0 + rl < N1) {
        const double wi = w1s[rl];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float v = vv[4 * c + ii];
          const float d = v - acc[c][ii];
          se[c] += wi * (double)(d * d);
          sv[c] += wi * (double)(v * v);
        }
      }
    }
  };
  float va[16], vb[16];
  vload(va, 0);
  for (int c0 = 0; c0 < N1; c0 += FEC_ROWS) {
    const int nr = min(FEC_ROWS, N1 - c0);
    __syncthreads();
    {
      // rows c0 .. c0+nr of U1, zero-padded to R1C columns, eight loads in flight
      const int ne = nr * R1C;
      for (int t0 = 0; t0 < ne; t0 += 8 * FEC_COLS) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = min(t0 + u * FEC_COLS + tid, ne - 1);
          const int qq = t / R1C, k = t - (t / R1C) * R1C;
          x[u] = U1[(long long)(c0 + qq) * r1 + min(k, r1 - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = t0 + u * FEC_COLS + tid;
          if (t < ne) U1s[t] = (t - (t / R1C) * R1C) < r1 ? x[u] : 0.0f;
        }
      }
      if (tid < nr) w1s[tid] = w1[c0 + tid];
    }
    __syncthreads();
    // blocks in pairs: each has the next one's values in flight
    const int nb = (nr + 15) >> 4;
    for (int rb = 0; rb < nb; rb += 2) {
      vload(vb, c0 + 16 * rb + 16);
      block(va, c0, rb);
      if (rb + 1 < nb) {
        vload(va, c0 + 16 * rb + 32);
        block(vb, c0, rb + 1);
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) va[u] = vb[u];   // (the next chunk's first block)
      }
    }
  }
  double st = 0.0, sq = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    st += jok[c] ? se[c] * w23[c] : 0.0;
    sq += jok[c] ? sv[c] * w23[c] : 0.0;
  }
  st = block_sum(st, red);
  sq = block_sum(sq, red);
  if (tid == 0) {
    part[2 * bx] = st;
    part[2 * bx + 1] = sq;
  }
}

// The error pass's partials alone (no controller): the column-block form for r1c > 0.
template <typename TD, typename T>
hipError_t launch_batch_ferr_partials(const FErrArgs* tab, const void* const* v1, BatchMap m, int blocks, int r1c,
                                      hipStream_t s) {
  switch (r1c) {
#define FEC_CASE(R)                                                                                   \
  case R:                                                                                             \
    if constexpr (std::is_same<T, float>::value)                                                      \
      hipLaunchKernelGGL((kb_ferr_mf<TD, R>), dim3(blocks), dim3(FEC_COLS), 0u, s, tab, v1, m);       \
    else                                                                                              \
      hipLaunchKernelGGL((kb_ferr_cols<TD, T, R>), dim3(blocks), dim3(FEC_COLS), 0u, s, tab, v1, m);  \
    break;
    FEC_CASE(4) FEC_CASE(8) FEC_CASE(12) FEC_CASE(16) FEC_CASE(20) FEC_CASE(24) FEC_CASE(28) FEC_CASE(32)
#undef FEC_CASE
    default:
      hipLaunchKernelGGL((kb_ferr<TD, T>), dim3(blocks), dim3(256), 0u, s, tab, v1, m);
  }
  return hipGetLastError();
}
template hipError_t launch_batch_ferr_partials<float, float>(const FErrArgs*, const void* const*, BatchMap, int, int,
                                                             hipStream_t);
template hipError_t launch_batch_ferr_partials<float, double>(const FErrArgs*, const void* const*, BatchMap, int, int,
                                                              hipStream_t);
template hipError_t launch_batch_ferr_partials<double, double>(const FErrArgs*, const void* const*, BatchMap, int,
                                                               int, hipStream_t);
template hipError_t launch_batch_ferr_partials<double, float>(const FErrArgs*, const void* const*, BatchMap, int, int,
                                                              hipStream_t);

template <typename TD, typename T>
hipError_t launch_batch_ferr(const FErrArgs* tab, const void* const* v1, BatchMap m, int blocks, int nstreams,
                             CtrlState* const* ctab, BatchSummary* out, unsigned* counter, unsigned long long* seq,
                             size_t lds_final, int r1c, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  switch (r1c) {
#define FEC_CASE(R)                                                                                            \
  case R:                                                                                                      \
    if constexpr (std::is_same<T, float>::value)                                                               \
      hipExtLaunchKernelGGL((kb_ferr_mf<TD, R>), dim3(blocks), dim3(FEC_COLS), 0u, s, ev0, ev1, 0u, tab, v1, m); \
    else                                                                                                       \
      hipExtLaunchKernelGGL((kb_ferr_cols<TD, T, R>), dim3(blocks), dim3(FEC_COLS), 0u, s, ev0, ev1, 0u, tab, v1, \
                            m);                                                                                \
    break;
    FEC_CASE(4) FEC_CASE(8) FEC_CASE(12) FEC_CASE(16) FEC_CASE(20) FEC_CASE(24) FEC_CASE(28) FEC_CASE(32)
#undef FEC_CASE
    default:
      hipExtLaunchKernelGGL((kb_ferr<TD, T>), dim3(blocks), dim3(256), 0u, s, ev0, ev1, 0u, tab, v1, m);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)kb_ferr_final, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_final);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_ferr_final, dim3(nstreams), dim3(256), lds_final, s, tab, ctab, out, counter, seq);
  return hipGetLastError();
}
template hipError_t launch_batch_ferr<float, float>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, unsigned*, unsigned long long*, size_t, int,
                                                   hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<float, double>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, unsigned*, unsigned long long*, size_t, int,
                                                   hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<double, double>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, unsigned*, unsigned long long*, size_t, int,
                                                   hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_ferr<double, float>(const FErrArgs*, const void* const*, BatchMap, int, int, CtrlState* const*,
                                                   BatchSummary*, unsigned*, unsigned long long*, size_t, int,
                                                   hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace tdb
