// Column-block stage pass on the matrix cores for batches of third-order streams
// (eqs. (Corecont) and (basecont): the TTM chain of one Runge-Kutta stage).
//
// A workgroup of 8 waves takes T2 columns of mode 2 with all of modes 1 and 3 and walks
// mode 1 in subtiles of 16 rows, so a stream has ceil(N2/T2) partial slots. With D the
// data difference, D_c its slice c of mode 3 and B_n = W_n U_n:
//   Y_c^T   = B2^T D_c^T           per subtile, K = the T2 columns
//   H1 rows = Y_(1) P1'            per subtile
//   F2'^T_c += D_c^T B1            K = the 16 rows, summed over the subtiles
// and after the subtiles
//   F3^T_c  = B2^T F2'^T_c,   H2 = F2'_(2) P2',   C_dot_p = F3 x_3 B3^T,   H3p = F3_(3)^T P3
// with P1'[(b,c)][a] = sum_c2 B3[c][c2] P1[(b,c2)][a] and P2'[(a,c)][b] likewise: every
// product is linear, so the mode-3 product is applied to the small results.
//
// Matrix-instruction convention of this file: a product is a sum of 16 x 16 blocks over
// 16-entry chunks of K; in a chunk, lane (q = l % 16, g = l / 16) feeds entries
// k = 4g .. 4g+3 of row q of A (column q of B), one per 16x16x4 instruction, and an
// accumulator lane (q, g) holds rows 4g .. 4g+3 of column q. An accumulator is therefore
// already, lane by lane, the A operand (its column index as m) or the B operand (as n)
// of a next product whose K runs over its rows: Y feeds H1 and F2'^T feeds F3 from the
// registers. The H1 blocks of the Y blocks (one per wave) are summed in a fixed order
// through LDS. Operand rows in LDS are plain with padded strides (16-byte reads).
//
// T2, the mode-3 extent (4 or 8, else at most 8 at run time) and the number of 16-wide
// rank blocks of modes 1 and 2 (1 or 2) are compile-time shapes; the slot layout
// [H1p rows (N1 rounded up to 16) | H2 rows (T2) | H3p | C_dot_p] is that of the other
// stage passes, so the fixed-order reduction and the rest of the step are shared. The
// next two subtiles' snapshot fibers are in flight while one is used (one for the
// BF16-split products and for FP64 data).
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "mfma_util.h"
#include <hip/hip_ext.h>

namespace tdb {

constexpr int RP_NW = 8;    // waves per workgroup
constexpr int RP_PS = 20;   // row stride (floats) of 16-entry operand rows in LDS

// Columns of mode 2 per workgroup: 64 or 32 for a mode-3 extent of 4, 32 otherwise
// (the F2' accumulators of 8 entries of mode 3 would not fit beside 64 columns).
int rpass_cols_for(int n3c) { return n3c == 4 ? 64 : 32; }
bool rpass_cols_ok(int n3c, int t2) { return t2 == 32 || (t2 == 64 && n3c == 4); }

// LDS regions (float offsets). Region X = [0, oB2) holds the raw copies of B2's rows, P1
// and B3 before the subtiles, D and the H1 blocks during them, and F2' (as A for H2) and
// F3 after them. B2^T and B3 stay for the whole block. Region S holds B1 and P1' during
// the subtiles and P2' after them (P2' is formed from global memory once the subtiles
// are done), so that a block fits twice in a compute unit's LDS at rank caps up to 24.
struct RpLayout {
  int nfc;                                       // 16-entry chunks of f = a*N3 + c
  int oHp, oF3, oB1, oB2, oP1, oP2, oB3, total;
};

__host__ __device__ inline RpLayout rp_layout(int T2, int r1, int r2, int N3) {
  RpLayout L;
  const int nb1 = (r1 + 15) >> 4, nb2 = (r2 + 15) >> 4, DS = T2 + 4;
  L.nfc = (r1 * N3 + 15) >> 4;
  const int d = N3 * 16 * DS;
  const int hp = N3 * nb2 * nb1 * 16 * RP_PS;
  const int fin = L.nfc * T2 * RP_PS + r1 * r2 * N3;
  const int raw = T2 * r2 + r1 * r2 * N3 + N3 * N3;   // r3 <= N3
  int x = d + hp;
  x = x > fin ? x : fin;
  x = x > raw ? x : raw;
  x = (x + 3) & ~3;
  L.oHp = d;
  L.oF3 = L.nfc * T2 * RP_PS;
  L.oB2 = x;
  L.oB3 = L.oB2 + nb2 * 16 * DS;
  const int oS = L.oB3 + ((N3 * N3 + 3) & ~3);
  L.oB1 = oS;
  L.oP1 = L.oB1 + nb1 * 16 * RP_PS;
  L.oP2 = oS;
  const int s1 = nb1 * 16 * RP_PS + N3 * nb2 * nb1 * 16 * RP_PS, s2 = L.nfc * nb2 * 16 * RP_PS;
  L.total = oS + (s1 > s2 ? s1 : s2);
  return L;
}

size_t rpass_lds_bytes(int T2, int r1, int r2, int N3) {
  return (size_t)rp_layout(T2, r1, r2, N3).total * sizeof(float);
}

bool rpass_shape_ok(int r1, int r2, int r3, int T2, int N3) {
  return N3 >= 1 && N3 <= 8 && r3 >= 1 && r3 <= N3 && r1 >= 1 && r2 >= 1 && r1 <= 32 && r2 <= 32 &&
         (T2 == 32 || (T2 == 64 && N3 == 4));
}

__device__ __forceinline__ mf4 ld4(const float* p) { return *reinterpret_cast<const mf4*>(p); }
__device__ __forceinline__ void st4(float* p, mf4 v) { *reinterpret_cast<mf4*>(p) = v; }

__device__ __forceinline__ void split_bf16(const float (&v)[8], mbf8& h, mbf8& l) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 x = (__bf16)v[j];
    h[j] = x;
    l[j] = (__bf16)(v[j] - (float)x);
  }
}

// acc += A B over one chunk (a: this lane's entries of A, b: of B). BF16-split: the
// chunk fills half of a 32-entry step, the other half zero.
template <int MF>
__device__ __forceinline__ mf4 mm16(mf4 acc, mf4 a, mf4 b) {
  if constexpr (MF == MPASS_F32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
  } else {
    const float av[8] = {a[0], a[1], a[2], a[3], 0.0f, 0.0f, 0.0f, 0.0f};
    const float bv[8] = {b[0], b[1], b[2], b[3], 0.0f, 0.0f, 0.0f, 0.0f};
    mbf8 ah, al, bh, bl;
    split_bf16(av, ah, al);
    split_bf16(bv, bh, bl);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  }
  return acc;
}

// Two chunks; BF16-split: one 32-entry step (the same slots for A and B).
template <int MF>
__device__ __forceinline__ mf4 mm32(mf4 acc, mf4 a0, mf4 b0, mf4 a1, mf4 b1) {
  if constexpr (MF == MPASS_F32) {
    acc = mm16<MF>(acc, a0, b0);
    return mm16<MF>(acc, a1, b1);
  } else {
    const float av[8] = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const float bv[8] = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    mbf8 ah, al, bh, bl;
    split_bf16(av, ah, al);
    split_bf16(bv, bh, bl);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    return acc;
  }
}

// acc += sum over nch chunks, chunk k of A at A + k*sa and of B at B + k*sb (both already
// at this lane's row/column and entry 4g).
template <int MF>
__device__ __forceinline__ mf4 mmk(mf4 acc, const float* A, int sa, const float* B, int sb, int nch) {
  if constexpr (MF == MPASS_F32) {
    for (int k = 0; k < nch; ++k) acc = mm16<MF>(acc, ld4(A + k * sa), ld4(B + k * sb));
  } else {
    int k = 0;
    for (; k + 1 < nch; k += 2)
      acc = mm32<MF>(acc, ld4(A + k * sa), ld4(B + k * sb), ld4(A + (k + 1) * sa), ld4(B + (k + 1) * sb));
    if (k < nch) acc = mm16<MF>(acc, ld4(A + k * sa), ld4(B + k * sb));
  }
  return acc;
}

template <typename TD, int MF, int N3C, bool VEC, int T2, int NB1, int NB2>
__device__ __forceinline__ void rpass_body(const FPassArgs& a, int bx) {
  constexpr int DS = T2 + 4;                            // row stride of D and B2^T
  constexpr int NBC = T2 / 16;                          // 16-column chunks of the block
  constexpr int N3M = N3C ? N3C : 8;                    // largest mode-3 extent
  constexpr int FPT = T2 / 32;                          // fibers per thread and subtile
  constexpr int GPW = (N3M * NB1 + RP_NW - 1) / RP_NW;  // F2' groups (c, a block) per wave
  constexpr int NYW = (N3M * NB2 + RP_NW - 1) / RP_NW;  // Y blocks (c, b block) per wave
  constexpr int NV = VEC ? (N3C ? N3C / 4 : 1) : 1;     // float4 per fiber
  constexpr int NS = VEC ? 1 : N3M;                     // scalar slots per fiber
  // subtiles in flight: two for FP32 products of FP32 data, else one (the register sets
  // of wider fibers or of the split products would not fit beside a second one)
  constexpr int DEPTH = (MF == MPASS_F32 && sizeof(TD) == 4) ? 2 : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* sm = reinterpret_cast<float*>(smem_raw);
  const int N3 = N3C ? N3C : a.N3;
  const int N1 = a.N1, N2 = a.N2, r1 = a.r1, r2 = a.r2, r3 = a.r3;
  const int i2_0 = bx * T2, ncol = min(T2, N2 - i2_0);
  const int nsub = (N1 + 15) >> 4;
  const RpLayout L = rp_layout(T2, r1, r2, N3);
  float* D = sm;              // slice c, subtile row i1: D + (c*16 + i1)*DS + i2
  float* Hp = sm + L.oHp;     // H1 block of Y block y, a block ab: Hp + ((y*NB1 + ab)*16 + a%16)*RP_PS + i1
  float* F2A = sm;            // after the subtiles: F2' chunk fc (f = a*N3 + c), column i2:
                              //   F2A + (fc*T2 + i2)*RP_PS + f%16
  float* F3s = sm + L.oF3;    // (a*r2 + b)*N3 + c
  float* B1T = sm + L.oB1;    // B1 of the subtile, column a, row i1: B1T + a*RP_PS + i1
  float* B2T = sm + L.oB2;    // B2^T: B2T + b*DS + i2
  float* P1T = sm + L.oP1;    // P1' block (c, jb), column a: P1T + ((c*NB2 + jb)*NB1*16 + a)*RP_PS + b%16
  float* P2T = sm + L.oP2;    // P2' chunk fc, column b: P2T + (fc*NB2*16 + b)*RP_PS + f%16
  float* B3s = sm + L.oB3;    // [c][c2]
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ln = tid & 63, q16 = ln & 15, g = ln >> 4;
  const bool has0 = a.V0 != nullptr;
  const TDB_GLOBAL TD* V1 = gmem(static_cast<const TD*>(a.V1));
  // without a previous snapshot the operand is V1 itself; V0 then aliases V1 so that
  // every load is issued on every path
  const TDB_GLOBAL TD* V0 = has0 ? gmem(static_cast<const TD*>(a.V0)) : V1;
  const TDB_GLOBAL float* B1 = gmem(static_cast<const float*>(a.B1));

  // ---- one subtile's snapshot fibers (16 rows x T2 columns) and B1 entries. Past the
  // last subtile, and past the tensor, addresses clamp to valid ones (the values are
  // zeroed when stored), so every load is unconditional: the count of memory operations
  // issued after each load is the same on every path and the waits for one subtile
  // leave the next one in flight. Offsets are 32-bit (the host admits tensors of fewer
  // than 2^31 entries).
  struct SubRegs {
    mf4 x1[FPT][NV], x0[FPT][NV];
    TD y1[FPT][NS], y0[FPT][NS];
    float b1r;
  };
  auto load_sub = [&](SubRegs& R, int s) {
    const int sc = min(s, nsub - 1);
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int q = tid + 512 * u;
      const int i1l = q / T2, i2l = q % T2;
      const int row = min(16 * sc + i1l, N1 - 1), col = i2_0 + min(i2l, ncol - 1);
      const int off = (row * N2 + col) * N3;
      if constexpr (VEC) {
        const TDB_GLOBAL mf4* p1 =
            reinterpret_cast<const TDB_GLOBAL mf4*>(reinterpret_cast<const TDB_GLOBAL float*>(V1) + off);
        const TDB_GLOBAL mf4* p0 =
            reinterpret_cast<const TDB_GLOBAL mf4*>(reinterpret_cast<const TDB_GLOBAL float*>(V0) + off);
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          R.x1[u][h] = p1[h];
          R.x0[u][h] = p0[h];
        }
      } else {
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          const int cc = min(c, N3 - 1);
          R.y1[u][c] = V1[off + cc];
          R.y0[u][c] = V0[off + cc];
        }
      }
    }
    const int t = min(tid, NB1 * 256 - 1);
    const int ai = min(t >> 4, r1 - 1), i1 = min(16 * sc + (t & 15), N1 - 1);
    R.b1r = B1[i1 * r1 + ai];
  };
  auto store_sub = [&](const SubRegs& R, int s) {
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
      const int q = tid + 512 * u;
      const int i1l = q / T2, i2l = q % T2;
      const bool ok = 16 * s + i1l < N1 && i2l < ncol;
      float d[NV * 4 > NS ? NV * 4 : NS];
      if constexpr (VEC) {
#pragma unroll
        for (int h = 0; h < NV; ++h)
#pragma unroll
          for (int j = 0; j < 4; ++j) d[4 * h + j] = has0 ? R.x1[u][h][j] - R.x0[u][h][j] : R.x1[u][h][j];
      } else {
#pragma unroll
        for (int c = 0; c < NS; ++c) d[c] = has0 ? (float)(R.y1[u][c] - R.y0[u][c]) : (float)R.y1[u][c];
      }
      float* Dp = D + i1l * DS + i2l;
#pragma unroll
      for (int c = 0; c < N3M; ++c)
        if (c < N3) Dp[c * 16 * DS] = ok ? d[c] : 0.0f;
    }
    if (tid < NB1 * 256) {
      const int ai = tid >> 4, i1l = tid & 15;
      B1T[ai * RP_PS + i1l] = (ai < r1 && 16 * s + i1l < N1) ? R.b1r : 0.0f;
    }
  };

  SubRegs ra, rb;
  load_sub(ra, 0);
  if constexpr (DEPTH == 2) load_sub(rb, 1);

  // ---- the block's B2 rows, P1 and B3, copied as they are into region X with all
  // loads of a round in flight together, then formed into the operand rows: B2^T and P1
  // folded with B3 (zero-padded)
  const int nB2 = ncol * r2, nP = r1 * r2 * r3, nB3 = N3 * r3;
  float* rB2 = sm;
  float* rP1 = rB2 + nB2;
  float* rB3 = rP1 + nP;
  {
    const TDB_GLOBAL float* gB2 = gmem(static_cast<const float*>(a.B2)) + i2_0 * r2;
    const TDB_GLOBAL float* gP1 = gmem(static_cast<const float*>(a.P1));
    const TDB_GLOBAL float* gB3 = gmem(static_cast<const float*>(a.B3));
    const int nP1 = a.need_h1 ? nP : 0;
    const int nmax = max(max(nB2, nP), nB3);
    for (int base = 0; base < nmax; base += 4 * 512) {
      float v[3][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = base + tid + u * 512;
        v[0][u] = gB2[min(t, nB2 - 1)];
        v[1][u] = nP1 ? gP1[min(t, nP1 - 1)] : 0.0f;
        v[2][u] = gB3[min(t, nB3 - 1)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = base + tid + u * 512;
        if (t < nB2) rB2[t] = v[0][u];
        if (t < nP1) rP1[t] = v[1][u];
        if (t < nB3) rB3[t] = v[2][u];
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < NB2 * 16 * T2; t += 512) {
    const int b = t / T2, i2 = t % T2;
    B2T[b * DS + i2] = (b < r2 && i2 < ncol) ? rB2[i2 * r2 + b] : 0.0f;
  }
  for (int t = tid; t < nB3; t += 512) B3s[t] = rB3[t];
  // P1'[(b,c)][a] = sum_c2 B3[c][c2] P1[(b*r3 + c2)][a], rows a of block (c, jb)
  for (int t = tid; t < N3 * NB2 * NB1 * 256; t += 512) {
    const int bl = t & 15, rest = t >> 4;
    const int aa = rest % (NB1 * 16), cj = rest / (NB1 * 16);
    const int c = cj / NB2, jb = cj % NB2, b = 16 * jb + bl;
    float v = 0.0f;
    if (a.need_h1 && aa < r1 && b < r2)
      for (int c2 = 0; c2 < r3; ++c2) v += rB3[c * r3 + c2] * rP1[(b * r3 + c2) * r1 + aa];
    P1T[rest * RP_PS + bl] = v;
  }
  // region X is read above and written by the first subtile
  __syncthreads();

  mf4 acc2[GPW][NBC];
#pragma unroll
  for (int gq = 0; gq < GPW; ++gq)
#pragma unroll
    for (int ib = 0; ib < NBC; ++ib) acc2[gq][ib] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
  TDB_GLOBAL float* out = gmem(static_cast<float*>(a.part)) + (long long)bx * a.slot;
  TDB_GLOBAL float* oH1 = out;
  TDB_GLOBAL float* oH2 = oH1 + a.T1 * r1;
  TDB_GLOBAL float* oH3 = oH2 + T2 * r2;
  TDB_GLOBAL float* oC = oH3 + N3 * r3;
  const int nY = N3 * NB2, nG = N3 * NB1;
  // this thread's output of the H1 rows of a subtile (row hi1, column ha)
  const int hi1 = tid / r1, ha = tid - (tid / r1) * r1;
  const bool hown = a.need_h1 && tid < 16 * r1;
  const float* Hq = Hp + ((ha >> 4) * 16 + (ha & 15)) * RP_PS + hi1;

  auto subtile = [&](SubRegs& R, int s) {
    store_sub(R, s);
    __syncthreads();
    load_sub(R, s + DEPTH);
    // Y blocks (c, jb) and, from their registers, their H1 blocks
#pragma unroll
    for (int t = 0; t < NYW; ++t) {
      const int yb = wave + RP_NW * t;
      if (yb < nY) {
        const int c = yb / NB2, jb = yb % NB2;
        mf4 y = {0.0f, 0.0f, 0.0f, 0.0f};
        y = mmk<MF>(y, B2T + (16 * jb + q16) * DS + 4 * g, 16, D + (c * 16 + q16) * DS + 4 * g, 16, NBC);
        const float* P = P1T + ((c * NB2 + jb) * NB1 * 16 + q16) * RP_PS + 4 * g;
#pragma unroll
        for (int ab = 0; ab < NB1; ++ab) {
          mf4 h = {0.0f, 0.0f, 0.0f, 0.0f};
          h = mm16<MF>(h, y, ld4(P + 16 * ab * RP_PS));
          st4(Hp + ((yb * NB1 + ab) * 16 + q16) * RP_PS + 4 * g, h);
        }
      }
    }
    // F2'^T blocks (c, ab, ib) += D_c^T B1 over the 16 rows
#pragma unroll
    for (int gq = 0; gq < GPW; ++gq) {
      const int gi = wave + RP_NW * gq;
      if (gi < nG) {
        const int c = gi / NB1, ab = gi % NB1;
        const mf4 bb = ld4(B1T + (16 * ab + q16) * RP_PS + 4 * g);
        const float* Dc = D + (c * 16 + 4 * g) * DS + q16;
#pragma unroll
        for (int ib = 0; ib < NBC; ++ib) {
          const mf4 av = {Dc[16 * ib], Dc[16 * ib + DS], Dc[16 * ib + 2 * DS], Dc[16 * ib + 3 * DS]};
          acc2[gq][ib] = mm16<MF>(acc2[gq][ib], av, bb);
        }
      }
    }
    __syncthreads();
    // the subtile's H1 rows: the Y blocks' H1 blocks summed in a fixed order
    if (hown && 16 * s + hi1 < N1) {
      float sv = 0.0f;
      for (int yb = 0; yb < nY; ++yb) sv += Hq[yb * NB1 * 16 * RP_PS];
      oH1[(16 * s + hi1) * r1 + ha] = sv;
    }
  };
  if constexpr (DEPTH == 2) {
    int s = 0;
    for (; s + 1 < nsub; s += 2) {
      subtile(ra, s);
      subtile(rb, s + 1);
    }
    if (s < nsub) subtile(ra, s);
  } else {
    for (int s = 0; s < nsub; ++s) subtile(ra, s);
  }
  // the last H1 rows read region X, the last subtile B1 and P1' (region S)
  __syncthreads();
  // ---- F3 from the F2'^T registers; F2' into the A rows of H2 (padded K entries zero)
  {
    const int K2 = r1 * N3;
    for (int t = tid; t < (16 * L.nfc - K2) * T2; t += 512) {
      const int f = K2 + t / T2, i2 = t % T2;
      F2A[((f >> 4) * T2 + i2) * RP_PS + (f & 15)] = 0.0f;
    }
#pragma unroll
    for (int gq = 0; gq < GPW; ++gq) {
      const int gi = wave + RP_NW * gq;
      if (gi < nG) {
        const int c = gi / NB1, ab = gi % NB1, aa = 16 * ab + q16;
#pragma unroll
        for (int jb = 0; jb < NB2; ++jb) {
          const float* A = B2T + (16 * jb + q16) * DS + 4 * g;
          mf4 f3 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int ib = 0; ib < NBC; ib += 2)
            f3 = mm32<MF>(f3, ld4(A + 16 * ib), acc2[gq][ib], ld4(A + 16 * (ib + 1)), acc2[gq][ib + 1]);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int b = 16 * jb + 4 * g + i;
            if (aa < r1 && b < r2) F3s[(aa * r2 + b) * N3 + c] = f3[i];
          }
        }
        if (aa < r1) {
          const int f = aa * N3 + c;
          float* F = F2A + (f >> 4) * T2 * RP_PS + (f & 15);
#pragma unroll
          for (int ib = 0; ib < NBC; ++ib)
#pragma unroll
            for (int i = 0; i < 4; ++i) F[(16 * ib + 4 * g + i) * RP_PS] = acc2[gq][ib][i];
        }
      }
    }
  }
  // P2'[f = a*N3 + c][b] = sum_c2 B3[c][c2] P2[(a*r3 + c2)][b] into region S: one thread
  // per (a, b) loads its r3 entries of P2 (all in flight, from clamped indices) once the
  // F2' registers are free
  constexpr int P2U = 2;   // (a, b) pairs per thread: r1 r2 <= 2 * 512 for ranks up to 32
  const int nab = a.need_h2 ? r1 * r2 : 0;
  float p2r[P2U][N3M];
  {
    const TDB_GLOBAL float* gP2 = gmem(static_cast<const float*>(a.P2));
#pragma unroll
    for (int u = 0; u < P2U; ++u) {
      const int t = min(tid + 512 * u, max(nab - 1, 0));
      const int ai = t / r2, b = t - (t / r2) * r2;
#pragma unroll
      for (int c2 = 0; c2 < N3M; ++c2) p2r[u][c2] = nab ? gP2[(ai * r3 + min(c2, r3 - 1)) * r2 + b] : 0.0f;
    }
  }

  // the padding of P2' (and all of it when H2 is not needed), while the loads are in flight
  for (int t = tid; t < L.nfc * NB2 * 256; t += 512) {
    const int fl = t & 15, rest = t >> 4;
    const int b = rest % (NB2 * 16), f = 16 * (rest / (NB2 * 16)) + fl;
    if (!(nab && b < r2 && f < r1 * N3)) P2T[rest * RP_PS + fl] = 0.0f;
  }
#pragma unroll
  for (int u = 0; u < P2U; ++u) {
    const int t = tid + 512 * u;
    if (t < nab) {
      const int ai = t / r2, b = t - (t / r2) * r2;
#pragma unroll
      for (int c = 0; c < N3M; ++c) {
        if (c < N3) {
          float v = 0.0f;
#pragma unroll
          for (int c2 = 0; c2 < N3M; ++c2)
            if (c2 < r3) v += B3s[c * r3 + c2] * p2r[u][c2];
          const int f = ai * N3 + c;
          P2T[((f >> 4) * NB2 * 16 + b) * RP_PS + (f & 15)] = v;
        }
      }
    }
  }
  __syncthreads();
  // H2 rows of this column block = F2'_(2) P2' (i2 blocks ib x b blocks jb, K = the nfc chunks)
  if (a.need_h2) {
    for (int blk = wave; blk < NBC * NB2; blk += RP_NW) {
      const int ib = blk / NB2, jb = blk % NB2;
      mf4 h = {0.0f, 0.0f, 0.0f, 0.0f};
      h = mmk<MF>(h, F2A + (16 * ib + q16) * RP_PS + 4 * g, T2 * RP_PS, P2T + (16 * jb + q16) * RP_PS + 4 * g,
                  NB2 * 16 * RP_PS, L.nfc);
      store_block(h, oH2 + (16 * ib) * r2 + 16 * jb, r2, 1, 16, r2 - 16 * jb);
    }
  }
  // C_dot_p[a][b][c2] = sum_c F3[a][b][c] B3[c][c2]
  for (int t = tid; t < r1 * r2 * r3; t += 512) {
    const int ab = t / r3, c2 = t - (t / r3) * r3;
    float sv = 0.0f;
    for (int c = 0; c < N3; ++c) sv += F3s[ab * N3 + c] * B3s[c * r3 + c2];
    oC[t] = sv;
  }
  // H3p[c][c2] = sum_(a,b) F3[a][b][c] P3[(a,b)][c2]
  if (a.need_f3 && wave == 0) {
    const TDB_GLOBAL float* P3 = gmem(static_cast<const float*>(a.P3));
    const int R3 = r1 * r2;
    for (int t = tid; t < N3 * r3; t += 64) {
      const int c = t / r3, c2 = t - (t / r3) * r3;
      float sv = 0.0f;
      for (int k = 0; k < R3; ++k) sv += F3s[k * N3 + c] * P3[k * r3 + c2];
      oH3[t] = sv;
    }
  }
}

template <typename TD, int MF, int N3C, bool VEC, int T2>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) kb_rpass(
    const FPassArgs* __restrict__ tab, const void* const* v1, const void* const* v0, BatchMap m) {
  const int s = m.sid[blockIdx.x];
  FPassArgs a = tab[s];
  a.V1 = v1[s];
  a.V0 = v0[s];
  if (a.hold && *gmem(a.hold)) return;
  const int bx = blockIdx.x - m.start[s];
  // rank blocks of modes 1 and 2 (the host admits ranks up to 32)
  const int sel = (a.r1 > 16 ? 2 : 0) + (a.r2 > 16 ? 1 : 0);
  if (sel == 0) rpass_body<TD, MF, N3C, VEC, T2, 1, 1>(a, bx);
  else if (sel == 1) rpass_body<TD, MF, N3C, VEC, T2, 1, 2>(a, bx);
  else if (sel == 2) rpass_body<TD, MF, N3C, VEC, T2, 2, 1>(a, bx);
  else rpass_body<TD, MF, N3C, VEC, T2, 2, 2>(a, bx);
}

template <typename TD, int MF, int N3C, bool VEC, int T2>
hipError_t launch_rpass_as(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m, int blocks,
                           size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  hipError_t e = hipFuncSetAttribute((const void*)kb_rpass<TD, MF, N3C, VEC, T2>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL((kb_rpass<TD, MF, N3C, VEC, T2>), dim3(blocks), dim3(RP_NW * 64), (uint32_t)lds, s, ev0, ev1,
                        0u, tab, v1, v0, m);
  return hipGetLastError();
}

template <typename TD, int MF>
hipError_t launch_rpass_mf(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m, int blocks,
                           int n3c, bool vec, int t2, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (sizeof(TD) == 4) {
    if (vec && n3c == 4)
      return t2 == 64 ? launch_rpass_as<TD, MF, 4, true, 64>(tab, v1, v0, m, blocks, lds, s, ev0, ev1)
                      : launch_rpass_as<TD, MF, 4, true, 32>(tab, v1, v0, m, blocks, lds, s, ev0, ev1);
    if (vec && n3c == 8) return launch_rpass_as<TD, MF, 8, true, 32>(tab, v1, v0, m, blocks, lds, s, ev0, ev1);
  }
  if (n3c == 4)
    return t2 == 64 ? launch_rpass_as<TD, MF, 4, false, 64>(tab, v1, v0, m, blocks, lds, s, ev0, ev1)
                    : launch_rpass_as<TD, MF, 4, false, 32>(tab, v1, v0, m, blocks, lds, s, ev0, ev1);
  if (n3c == 8) return launch_rpass_as<TD, MF, 8, false, 32>(tab, v1, v0, m, blocks, lds, s, ev0, ev1);
  return launch_rpass_as<TD, MF, 0, false, 32>(tab, v1, v0, m, blocks, lds, s, ev0, ev1);
}

// n3c: the mode-3 extent shared by every stream of the launch (4 or 8), else 0; t2: the
// columns of mode 2 every stream's plan uses (rpass_cols_ok). vw: 4 or 8 when every
// stream's snapshots are FP32 with N3 = vw on 16-byte addresses (whole fibers as float4
// loads), else 0.
template <typename TD>
hipError_t launch_batch_rpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, int flavor, int n3c, int t2, int vw, size_t lds, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
  if (n3c != 4 && n3c != 8) n3c = 0;
  if (!rpass_cols_ok(n3c, t2)) return hipErrorInvalidValue;
  const bool vec = sizeof(TD) == 4 && vw != 0 && vw == n3c;
  return flavor == MPASS_F32
             ? launch_rpass_mf<TD, MPASS_F32>(tab, v1, v0, m, blocks, n3c, vec, t2, lds, s, ev0, ev1)
             : launch_rpass_mf<TD, MPASS_BF16S>(tab, v1, v0, m, blocks, n3c, vec, t2, lds, s, ev0, ev1);
}
template hipError_t launch_batch_rpass<float>(const FPassArgs*, const void* const*, const void* const*, BatchMap, int,
                                              int, int, int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_batch_rpass<double>(const FPassArgs*, const void* const*, const void* const*, BatchMap,
                                               int, int, int, int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace tdb
