// Stage pass on the matrix cores (eqs. (Corecont) and (basecont)) for third-order
// streams whose first two ranks are at most 32 and whose third mode has at most 8
// entries (the variables / species / components mode of the target workloads).
//
// Tile: 16 rows of mode 1 x T2 (16, 32 or 64) rows of mode 2 x all N3 of mode 3, run
// by 16, 8 or 4 waves (the kernels at the end of this file say when). The
// pseudo-inverses are staged in LDS with the tile when they fit. Z and D are kept in
// LDS as [c][i2][i1] with the mode-1 index XOR-swizzled by the low bits of i2, so that
// the operand reads of every product below fall in distinct LDS banks.
//   Z[c2][i1][i2] = sum_c D[i1][i2][c] B3[c][c2]        (VALU, from the loaded fibers)
//   Y[c][i1][b]   = sum_i2 D[c][i1][i2] B2[i2][b]      (only if mode 3 is not full rank)
//   F1[i1][b,c2]  = sum_i2 Z[c2][i1][i2] B2[i2][b]
//   F2[i2][a,c2]  = sum_i1 B1[i1][a] Z[c2][i1][i2]
//   F3[a,b][c]    = sum_i1 B1[i1][a] Y[c][i1][b]
//   H1p = F1 P1, H2p = F2 P2, H3p = F3^T P3, Cdot_p[a][b,c2] = sum_i1 B1[i1][a] F1[i1][b,c2]
// Every product above is a sum of 16 x 16 output blocks computed by one wave each,
// either with FP32 matrix instructions (16x16x4) or with BF16-split products
// (x = hi + lo, hi·hi + hi·lo + lo·hi on 16x16x32 BF16 instructions), always
// accumulated in FP32. The per-tile partial slot has the same layout as the generic
// pass, so the reduction and the rest of the step are shared.
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "mfma_util.h"
#include <hip/hip_ext.h>

namespace tdb {

// LDS floats of one tile (T1 = 16) for ranks (r1, r2, r3), N3 and T2; `pst` stages
// the pseudo-inverses that are needed (h1, h2, f3).
__host__ __device__ inline long long mpass_lds_floats(int r1, int r2, int r3, int N3, int T2, bool h1, bool h2,
                                                     bool f3, bool pst) {
  const long long R1 = (long long)r2 * r3, R2 = (long long)r1 * r3, R3 = (long long)r1 * r2;
  long long e = (long long)r3 * 16 * T2 + 16LL * r1 + (long long)T2 * r2 + 64 + 16 * R1;
  if (pst) e += (h1 ? R1 * r1 : 0) + (h2 ? R2 * r2 : 0) + (f3 ? R3 * r3 : 0);
  long long x = (long long)T2 * R2 + (f3 ? R3 * N3 : 0);
  if (f3) {
    const long long dsz = (long long)N3 * 16 * T2;
    x = x > dsz ? x : dsz;
    e += (long long)N3 * 16 * r2;
  }
  return e + x;
}

template <typename TD, int MF, int NW>
__device__ __forceinline__ void mpass_body(const FPassArgs& a, int bx) {
  if (a.hold && *a.hold) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* sm = reinterpret_cast<float*>(smem_raw);
  const int N2 = a.N2, N3 = a.N3, r1 = a.r1, r2 = a.r2, r3 = a.r3, T2 = a.T2;
  const int t1 = bx / a.nt2, t2 = bx - (bx / a.nt2) * a.nt2;
  const int i1_0 = t1 * 16, i2_0 = t2 * T2;
  const int n1 = min(16, a.N1 - i1_0), n2 = min(T2, N2 - i2_0);
  const int R1 = r2 * r3, R2 = r1 * r3, R3 = r1 * r2;
  const bool f3 = a.need_f3 != 0;
  const int TS = 16 * T2;                  // fibers per tile
  const int ZS = TS;                       // LDS floats of one Z (or D) slice
  float* Zs = sm;                          // r3 x (T2 x 16, swizzled)
  float* B1s = Zs + r3 * ZS;               // 16 x r1
  float* B2s = B1s + 16 * r1;              // T2 x r2
  float* B3s = B2s + T2 * r2;              // r3 x 8 (B3 transposed, <= 64)
  float* F1s = B3s + 64;                   // 16 x R1
  float* Pp = F1s + 16 * R1;               // staged P1 | P2 | P3
  const float* P1 = static_cast<const float*>(a.P1);
  const float* P2 = static_cast<const float*>(a.P2);
  const float* P3 = static_cast<const float*>(a.P3);
  const float* P1g = P1;                   // staging sources (P1..P3 switch to LDS)
  const float* P2g = P2;
  const float* P3g = P3;
  float* pend = Pp;
  if (a.stage_p) pend += (a.need_h1 ? R1 * r1 : 0) + (a.need_h2 ? R2 * r2 : 0) + (f3 ? R3 * r3 : 0);
  float* Ys = pend;                        // N3 x 16 x r2 (f3)
  float* X = Ys + (f3 ? N3 * 16 * r2 : 0); // D (N3 x T2 x 16), later F2 (T2 x R2) | F3 (R3 x N3)
  float* Ds = X;
  float* F2s = X;
  float* F3s = X + T2 * R2;
  // NW = 8 or 16: the first half of the waves load the snapshot fibers and form Z (and
  // D) while the second half stage the bases and pseudo-inverses; NW = 4: every wave
  // issues its staging loads, then its fiber loads, then stores the staged batch. All
  // waves share the products. FT threads load fibers (up to four each), ST stage.
  constexpr bool split = NW != 4;
  constexpr int FT = split ? NW * 32 : 256, ST = FT;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool stager = split && wave >= NW / 2;
  const int tid = stager ? (int)threadIdx.x - FT : (int)threadIdx.x;

  // 1. loads. The staging loads bring the bases of this tile and the pseudo-inverses
  // into LDS (B3 transposed, one column of 8 per c2, so that Z reads it as two
  // vectors); the fiber loads leave the snapshot differences in registers. Each source
  // array is copied through a register array of its own, one slot per ST entries,
  // so that a slot's source is fixed at compile time: a slot that holds none of the
  // wave's entries is skipped by a wave-uniform test, and entries past the end (or
  // past a ragged edge) load a valid entry and are dropped (or zeroed) when stored.
  // No register is written by anything but its load, so a batch's loads stay in
  // flight together.
  const float* B1 = static_cast<const float*>(a.B1) + (long long)i1_0 * r1;
  const float* B2 = static_cast<const float*>(a.B2) + (long long)i2_0 * r2;
  const float* B3 = static_cast<const float*>(a.B3);
  const bool sp = a.stage_p != 0;
  const int lB1 = 16 * r1, lB2 = T2 * r2, lB3 = N3 * r3;
  const int lP1 = sp && a.need_h1 ? R1 * r1 : 0;
  const int lP2 = sp && a.need_h2 ? R2 * r2 : 0;
  const int lP3 = sp && f3 ? R3 * r3 : 0;
  const int v0 = n1 * r1, v1 = n2 * r2;
  float* P1l = Pp;
  float* P2l = P1l + lP1;
  float* P3l = P2l + lP2;
  const int wq = 64 * (split ? wave % (NW / 2) : wave);
  // entries [j0, j0 + ST S) of an array of len entries, of which the first `valid`
  // exist in the source
  auto rload = [&](auto& r, const float* src, int len, int valid, int j0) {
    constexpr int S = sizeof(r) / sizeof(float);
#pragma unroll
    for (int u = 0; u < S; ++u)
      if (j0 + u * ST + wq < len) r[u] = src[min(j0 + u * ST + tid, valid - 1)];
  };
  auto rstore = [&](const auto& r, float* dst, int len, int valid, int j0) {
    constexpr int S = sizeof(r) / sizeof(float);
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int j = j0 + u * ST + tid;
      if (j0 + u * ST + wq < len && j < len) dst[j] = j < valid ? r[u] : 0.0f;
    }
  };
  constexpr int SB2 = 2048 / ST, SP = 1536 / ST;  // slots: B2 (T2 r2 <= 2048), each P batch
  float b1r[2], b2r[SB2], b3r[1], p1r[SP], p2r[SP], p3r[SP];
  auto load_bases = [&]() {
    rload(b1r, B1, lB1, v0, 0);
    rload(b2r, B2, lB2, v1, 0);
    rload(b3r, B3, lB3, lB3, 0);
  };
  auto store_bases = [&]() {
    rstore(b1r, B1s, lB1, v0, 0);
    rstore(b2r, B2s, lB2, v1, 0);
    if (wq < lB3 && tid < lB3) {
      const int c = tid / r3, c2 = tid - c * r3;
      B3s[c2 * 8 + c] = b3r[0];
    }
  };
  auto load_p = [&](int j0) {
    rload(p1r, P1g, lP1, lP1, j0);
    rload(p2r, P2g, lP2, lP2, j0);
    rload(p3r, P3g, lP3, lP3, j0);
  };
  auto store_p = [&](int j0) {
    rstore(p1r, P1l, lP1, lP1, j0);
    rstore(p2r, P2l, lP2, lP2, j0);
    rstore(p3r, P3l, lP3, lP3, j0);
  };
  const int lPmax = max(lP1, max(lP2, lP3));
  // the snapshot differences of this thread's fibers, every load issued before any
  // difference is formed
  float d[4][8];
  auto load_fibers = [&]() {
    const TD* V1 = static_cast<const TD*>(a.V1);
    const TD* V0 = static_cast<const TD*>(a.V0);
    if (sizeof(TD) == 4 && (N3 == 4 || N3 == 8) && ((reinterpret_cast<uintptr_t>(V1) | reinterpret_cast<uintptr_t>(V0)) & 15) == 0) {
      // whole fibers as 16-byte loads (a fiber of 4 or 8 FP32 values is 16-byte aligned)
      float4 x1[4][2], x0[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = tid + FT * u;
        const int i1 = q / T2, i2 = q - (q / T2) * T2;
        const bool ok = q < TS && i1 < n1 && i2 < n2;
        const long long g = ((long long)(i1_0 + i1) * N2 + i2_0 + i2) * N3;
        const float4* p1 = reinterpret_cast<const float4*>(V1 + g);
        const float4* p0 = reinterpret_cast<const float4*>(V0 + g);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          x1[u][h] = make_float4(0.f, 0.f, 0.f, 0.f);
          x0[u][h] = x1[u][h];
        }
        if (ok) {
          x1[u][0] = p1[0];
          if (N3 == 8) x1[u][1] = p1[1];
          if (V0) {
            x0[u][0] = p0[0];
            if (N3 == 8) x0[u][1] = p0[1];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        d[u][0] = x1[u][0].x - x0[u][0].x; d[u][1] = x1[u][0].y - x0[u][0].y;
        d[u][2] = x1[u][0].z - x0[u][0].z; d[u][3] = x1[u][0].w - x0[u][0].w;
        d[u][4] = x1[u][1].x - x0[u][1].x; d[u][5] = x1[u][1].y - x0[u][1].y;
        d[u][6] = x1[u][1].z - x0[u][1].z; d[u][7] = x1[u][1].w - x0[u][1].w;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = tid + FT * u;
        const int i1 = q / T2, i2 = q - (q / T2) * T2;
        const bool ok = q < TS && i1 < n1 && i2 < n2;
        const long long g = ((long long)(i1_0 + i1) * N2 + i2_0 + i2) * N3;
        TD y1[8], y0[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          y1[c] = TD(0);
          y0[c] = TD(0);
          if (ok && c < N3) {
            y1[c] = V1[g + c];
            if (V0) y0[c] = V0[g + c];
          }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) d[u][c] = (float)y1[c] - (float)y0[c];
      }
    }
  };
  // The first batch of pseudo-inverse loads is issued after the bases and kept in
  // registers through Z, F1 and F2 (only the folds read it); it is stored, and any
  // further batch copied, just before the folds. NW = 8 or 16: the staging waves do
  // this while the fiber waves load the snapshots; NW = 4: every wave does both.
  if (split) {
    if (stager) {
      load_bases();
      store_bases();
      load_p(0);
    } else {
      load_fibers();
    }
  } else {
    load_bases();
    load_fibers();
    store_bases();
    load_p(0);
  }
  if (lP1) P1 = P1l;
  if (lP2) P2 = P2l;
  if (lP3) P3 = P3l;
  __syncthreads();
  // 2. Z (and D for the third mode) into LDS
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (stager || FT * u >= TS) break;
    const int q = tid + FT * u;
    if (q >= TS) break;
    const int zo = zsw(q / T2, q - (q / T2) * T2);
    for (int c2 = 0; c2 < r3; ++c2) {
      const float4 b0 = *reinterpret_cast<const float4*>(B3s + c2 * 8);
      const float4 b1 = *reinterpret_cast<const float4*>(B3s + c2 * 8 + 4);
      const float bc[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      float s = 0.0f;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < N3) s += d[u][c] * bc[c];
      Zs[c2 * ZS + zo] = s;
    }
    if (f3)
      for (int c = 0; c < N3; ++c) Ds[c * ZS + zo] = d[u][c];
  }
  __syncthreads();
  const int nb1 = (r1 + 15) >> 4, nb2 = (r2 + 15) >> 4;
  // 3. F1 (and Y)
  {
    const int nF1 = r3 * nb2, nY = f3 ? N3 * nb2 : 0;
    for (int blk = wave; blk < nF1 + nY; blk += NW) {
      mf4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      if (blk < nF1) {
        const int c2 = blk / nb2, jb = blk - c2 * nb2;
        const float* Zc = Zs + c2 * ZS;
        const float* Bb = B2s + 16 * jb;
        acc = mma_blockf<MF>([&](int m, int k0, int j) { return Zc[zsw16(m, k0, j)]; }, 16,
                             [&](int k0, int j, int n) { return Bb[(k0 + j) * r2 + n]; }, r2 - 16 * jb, T2, acc);
        store_block(acc, F1s + (16 * jb) * r3 + c2, R1, r3, 16, r2 - 16 * jb);
      } else {
        const int q = blk - nF1;
        const int c = q / nb2, jb = q - c * nb2;
        const float* Dc = Ds + c * ZS;
        const float* Bb = B2s + 16 * jb;
        acc = mma_blockf<MF>([&](int m, int k0, int j) { return Dc[zsw16(m, k0, j)]; }, 16,
                             [&](int k0, int j, int n) { return Bb[(k0 + j) * r2 + n]; }, r2 - 16 * jb, T2, acc);
        store_block(acc, Ys + c * 16 * r2 + 16 * jb, r2, 1, 16, r2 - 16 * jb);
      }
    }
  }
  __syncthreads();
  // 4. F2 (over the former D) and F3
  {
    const int nib = T2 >> 4;
    const int nF2 = r3 * nb1 * nib, nF3 = f3 ? N3 * nb1 * nb2 : 0;
    for (int blk = wave; blk < nF2 + nF3; blk += NW) {
      mf4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      if (blk < nF2) {
        const int c2 = blk / (nb1 * nib), rem = blk - c2 * nb1 * nib;
        const int ab = rem / nib, ib = rem - ab * nib;
        // rows a (B1^T), columns i2 (Z[c2]), K = i1
        const float* Zc = Zs + c2 * ZS;
        const float* Ab = B1s + 16 * ab;
        const int i20 = 16 * ib;
        acc = mma_blockf<MF>([&](int m, int k0, int j) { return Ab[m + (k0 + j) * r1]; }, r1 - 16 * ab,
                             [&](int k0, int j, int n) { return Zc[(i20 + n) * 16 + ((k0 + j) ^ n)]; }, 16, 16, acc);
        // F2s[i2][a*r3 + c2]
        store_block(acc, F2s + (16 * ib) * R2 + (16 * ab) * r3 + c2, r3, R2, r1 - 16 * ab, 16);
      } else {
        const int q = blk - nF2;
        const int c = q / (nb1 * nb2), rem = q - c * nb1 * nb2;
        const int ab = rem / nb2, jb = rem - ab * nb2;
        acc = mma_block<MF>(B1s + 16 * ab, 1, r1, r1 - 16 * ab, Ys + c * 16 * r2 + 16 * jb, r2, 1, r2 - 16 * jb, 16,
                            acc);
        // F3s[(a*r2 + b)*N3 + c]
        store_block(acc, F3s + ((16 * ab) * r2 + 16 * jb) * N3 + c, r2 * N3, N3, r1 - 16 * ab, r2 - 16 * jb);
      }
    }
  }
  if (!split || stager) {
    store_p(0);
    for (int j0 = SP * ST; j0 < lPmax; j0 += SP * ST) {
      load_p(j0);
      store_p(j0);
    }
  }
  __syncthreads();
  // 5. folds into the partial slot
  float* out = static_cast<float*>(a.part) + (long long)bx * a.slot;
  float* oH1 = out;
  float* oH2 = oH1 + 16 * r1;
  float* oH3 = oH2 + T2 * r2;
  float* oC = oH3 + N3 * r3;
  const int nbR1 = (R1 + 15) >> 4;
  const int nC = nb1 * nbR1, nH1 = a.need_h1 ? nb1 : 0, nH2 = a.need_h2 ? (T2 >> 4) * nb2 : 0, nH3 = f3 ? 1 : 0;
  for (int blk = wave; blk < nC + nH1 + nH2 + nH3; blk += NW) {
    mf4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (blk < nC) {
      const int ab = blk / nbR1, kb = blk - ab * nbR1;
      acc = mma_block<MF>(B1s + 16 * ab, 1, r1, r1 - 16 * ab, F1s + 16 * kb, R1, 1, R1 - 16 * kb, 16, acc);
      store_block(acc, oC + (16 * ab) * R1 + 16 * kb, R1, 1, r1 - 16 * ab, R1 - 16 * kb);
    } else if (blk < nC + nH1) {
      const int ab = blk - nC;
      acc = mma_block<MF>(F1s, R1, 1, 16, P1 + 16 * ab, r1, 1, r1 - 16 * ab, R1, acc);
      store_block(acc, oH1 + 16 * ab, r1, 1, 16, r1 - 16 * ab);
    } else if (blk < nC + nH1 + nH2) {
      const int q = blk - nC - nH1;
      const int ib = q / nb2, jb = q - ib * nb2;
      acc = mma_block<MF>(F2s + (16 * ib) * R2, R2, 1, 16, P2 + 16 * jb, r2, 1, r2 - 16 * jb, R2, acc);
      store_block(acc, oH2 + (16 * ib) * r2 + 16 * jb, r2, 1, 16, r2 - 16 * jb);
    } else {
      // H3p[c][c2] = sum_k F3[k][c] P3[k][c2]
      acc = mma_block<MF>(F3s, 1, N3, N3, P3, r3, 1, r3, R3, acc);
      store_block(acc, oH3, r3, 1, N3, r3);
    }
  }
}

// Sixteen waves per tile, one tile per compute unit (tiles of 16 x 32 or more): for
// grids the chip holds at once, where a tile's latency is the launch's and a second
// tile on the same compute unit would only slow the first.
template <typename TD, int MF>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) k_mpass_w16(FPassArgs a) {
  mpass_body<TD, MF, 16>(a, blockIdx.x);
}

// Eight waves per tile, at most 128 registers so that two tiles share a compute unit.
template <typename TD, int MF>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_mpass(FPassArgs a) {
  mpass_body<TD, MF, 8>(a, blockIdx.x);
}

// Four waves per tile: more tiles per compute unit, for larger grids.
template <typename TD, int MF>
__global__ void __launch_bounds__(256) k_mpass_w4(FPassArgs a) {
  mpass_body<TD, MF, 4>(a, blockIdx.x);
}

template <typename TD, int MF>
__global__ void __launch_bounds__(256) kb_mpass(const FPassArgs* __restrict__ tab, const void* const* v1,
                                                const void* const* v0, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  FPassArgs a = tab[s];
  a.V1 = v1[s];
  a.V0 = v0[s];
  mpass_body<TD, MF, 4>(a, blockIdx.x - m.start[s]);
}

size_t mpass_lds_bytes(int r1, int r2, int r3, int N3, int T2, bool h1, bool h2, bool f3, bool pst) {
  return (size_t)mpass_lds_floats(r1, r2, r3, N3, T2, h1, h2, f3, pst) * sizeof(float);
}

int mpass_waves(int tiles, int T2) {
  if (tiles <= MPASS_W16_TILES && T2 >= 32) return 16;
  return tiles <= MPASS_W8_TILES ? 8 : 4;
}

template <typename TD>
hipError_t launch_mpass(const FPassArgs& a, int flavor, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const int tiles = a.nt1 * a.nt2;
  const int nw = mpass_waves(tiles, a.T2);
  const bool f32 = flavor == MPASS_F32;
  const void* f = nw == 16 ? (f32 ? (const void*)k_mpass_w16<TD, MPASS_F32> : (const void*)k_mpass_w16<TD, MPASS_BF16S>)
                  : nw == 8 ? (f32 ? (const void*)k_mpass<TD, MPASS_F32> : (const void*)k_mpass<TD, MPASS_BF16S>)
                            : (f32 ? (const void*)k_mpass_w4<TD, MPASS_F32> : (const void*)k_mpass_w4<TD, MPASS_BF16S>);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nw == 16) {
    if (f32)
      hipExtLaunchKernelGGL((k_mpass_w16<TD, MPASS_F32>), dim3(tiles), dim3(1024), (uint32_t)lds, s, ev0, ev1, 0u, a);
    else
      hipExtLaunchKernelGGL((k_mpass_w16<TD, MPASS_BF16S>), dim3(tiles), dim3(1024), (uint32_t)lds, s, ev0, ev1, 0u, a);
  } else if (nw == 8) {
    if (f32)
      hipExtLaunchKernelGGL((k_mpass<TD, MPASS_F32>), dim3(tiles), dim3(512), (uint32_t)lds, s, ev0, ev1, 0u, a);
    else
      hipExtLaunchKernelGGL((k_mpass<TD, MPASS_BF16S>), dim3(tiles), dim3(512), (uint32_t)lds, s, ev0, ev1, 0u, a);
  } else {
    if (f32)
      hipExtLaunchKernelGGL((k_mpass_w4<TD, MPASS_F32>), dim3(tiles), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, a);
    else
      hipExtLaunchKernelGGL((k_mpass_w4<TD, MPASS_BF16S>), dim3(tiles), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, a);
  }
  return hipGetLastError();
}
template hipError_t launch_mpass<float>(const FPassArgs&, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_mpass<double>(const FPassArgs&, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);

template <typename TD>
hipError_t launch_batch_mpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, int flavor, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const void* f =
      flavor == MPASS_F32 ? (const void*)kb_mpass<TD, MPASS_F32> : (const void*)kb_mpass<TD, MPASS_BF16S>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (flavor == MPASS_F32)
    hipExtLaunchKernelGGL((kb_mpass<TD, MPASS_F32>), dim3(blocks), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, tab, v1,
                          v0, m);
  else
    hipExtLaunchKernelGGL((kb_mpass<TD, MPASS_BF16S>), dim3(blocks), dim3(256), (uint32_t)lds, s, ev0, ev1, 0u, tab,
                          v1, v0, m);
  return hipGetLastError();
}
template hipError_t launch_batch_mpass<float>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                              int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_mpass<double>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                               int, size_t, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace tdb
