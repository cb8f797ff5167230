// Matrix-core helpers shared by the stage passes (gfx950, wave64): one 16 x 16 output
// block per wave with FP32 (16x16x4) or BF16-split (16x16x32, hi*hi + hi*lo + lo*hi)
// products accumulated in FP32, and the swizzled LDS layout of 16-row slices.
#pragma once
#include <hip/hip_runtime.h>
#include "fused.h"

namespace tdb {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef __bf16 mbf8 __attribute__((ext_vector_type(8)));

// One 16 x 16 block C += A B over K (valid K entries Kv): A(m, k) = fa(m, k0, j) and
// B(k, n) = fb(k0, j, n) with k = k0 + j, k0 a multiple of 16 and j < 16, for m < Mv,
// n < Nv, zero elsewhere. Lane l feeds row/column l % 16 and the K slice selected by
// l / 16. Operand reads are never predicated: lanes outside the block read a valid
// entry (indices clamped into the block) and zero it, so each group of 16 K entries
// is loaded in one go, and the next group while the current one's matrix
// instructions run.
// `l` is the lane (threadIdx.x & 63); a caller inside a loop may pass a copy the
// compiler cannot see through, so that the per-lane operand addresses are formed in
// each iteration instead of being hoisted out of the loop into many registers.
template <int MF, typename FA, typename FB>
__device__ __forceinline__ mf4 mma_blockf_l(int l, FA fa, int Mv, FB fb, int Nv, int Kv, mf4 acc) {
  const int mn = l & 15, kg = l >> 4;
  const bool am = mn < Mv, bn = mn < Nv;
  const int mc = am ? mn : Mv - 1, nc = bn ? mn : Nv - 1;
  if (MF == MPASS_F32) {
    const int nfull = Kv & ~15;
    float xa[4], xb[4];
    auto load = [&](int k0) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        xa[st] = fa(mc, k0, 4 * st + kg);
        xb[st] = fb(k0, 4 * st + kg, nc);
      }
    };
    if (nfull > 0) load(0);
    for (int k0 = 0; k0 < nfull; k0 += 16) {
      float a[4], b[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        a[st] = am ? xa[st] : 0.0f;
        b[st] = bn ? xb[st] : 0.0f;
      }
      if (k0 + 16 < nfull) load(k0 + 16);
#pragma unroll
      for (int st = 0; st < 4; ++st) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], b[st], acc, 0, 0, 0);
    }
    if (nfull < Kv) {
      float a[4], b[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int j = 4 * st + kg;
        const bool kv = nfull + j < Kv;
        const int jc = kv ? j : Kv - 1 - nfull;
        const float x = fa(mc, nfull, jc), y = fb(nfull, jc, nc);
        a[st] = (am && kv) ? x : 0.0f;
        b[st] = (bn && kv) ? y : 0.0f;
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], b[st], acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < Kv; k0 += 32) {
      mbf8 ah, al, bh, bl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + 8 * kg + j;
        const bool kv = k < Kv;
        const int kc = kv ? k : Kv - 1;
        const int kb = kc & ~15;
        const float x = fa(mc, kb, kc - kb), y = fb(kb, kc - kb, nc);
        const float a = (am && kv) ? x : 0.0f;
        const float b = (bn && kv) ? y : 0.0f;
        const __bf16 a1 = (__bf16)a, b1 = (__bf16)b;
        ah[j] = a1;
        al[j] = (__bf16)(a - (float)a1);
        bh[j] = b1;
        bl[j] = (__bf16)(b - (float)b1);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    }
  }
  return acc;
}

template <int MF, typename FA, typename FB>
__device__ __forceinline__ mf4 mma_blockf(FA fa, int Mv, FB fb, int Nv, int Kv, mf4 acc) {
  return mma_blockf_l<MF>((int)(threadIdx.x & 63), fa, Mv, fb, Nv, Kv, acc);
}

// The same with strided operands: A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn].
template <int MF>
__device__ __forceinline__ mf4 mma_block(const float* A, int sam, int sak, int Mv, const float* B, int sbk, int sbn,
                                         int Nv, int Kv, mf4 acc) {
  return mma_blockf<MF>([&](int m, int k0, int j) { return A[m * sam + (k0 + j) * sak]; }, Mv,
                        [&](int k0, int j, int n) { return B[(k0 + j) * sbk + n * sbn]; }, Nv, Kv, acc);
}

// Z and D slices in LDS: entry (i1, i2) of a 16 x T2 slice at i2*16 + (i1 ^ (i2 & 15)).
// Reading a 16-row column block along i2 (F1, Y) or a 16-column row block along i1
// (F2) then touches 64 distinct banks per instruction, with no padding.
__device__ __forceinline__ int zsw(int i1, int i2) { return i2 * 16 + (i1 ^ (i2 & 15)); }
// The same for i2 = k0 + j with k0 a multiple of 16 and j < 16.
__device__ __forceinline__ int zsw16(int i1, int k0, int j) { return (k0 + j) * 16 + (i1 ^ j); }

// Store a 16 x 16 block: lane l holds rows 4*(l/16) + i, column l % 16.
// C may be a generic or a global-memory pointer.
template <typename PC>
__device__ __forceinline__ void store_block(const mf4& acc, PC C, int scm, int scn, int Mv, int Nv) {
  const int l = threadIdx.x & 63;
  const int n = l & 15, m0 = 4 * (l >> 4);
  if (n >= Nv) return;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (m0 + i < Mv) C[(m0 + i) * scm + n * scn] = acc[i];
}


// ---- Packed operand layout. A 16 x 16 chunk of an operand (16 rows m of A, or 16
// columns n of B, by 16 entries of K) keeps row (or column) q at q*16 and entry k at
// (k % 4)*4 + k/4: lane (q = l % 16, g = l / 16) then finds the four entries it feeds
// to the four 16x16x4 instructions of the chunk (k = 4s + g, s = 0..3) in one 16-byte
// read. Padded rows, columns and K entries hold zeros, so no operand is masked.
__device__ __forceinline__ int pk(int q, int k) { return q * 16 + ((k & 3) << 2) + (k >> 2); }

// C += A B over nch chunks: A chunk c at A + c*sa, B chunk c at B + c*sb (packed,
// 16-byte aligned). BF16-split: chunks are taken in pairs; lane (q, g) feeds the four
// entries of chunk c to slots 0-3 and those of chunk c+1 to slots 4-7 of a 32-entry
// step, the same assignment for A and B, so the sum runs over every k once.
template <int MF>
__device__ __forceinline__ mf4 mma_pk(int l, const float* A, int sa, const float* B, int sb, int nch, mf4 acc) {
  const int off = (l & 15) * 16 + (l >> 4) * 4;
  if (MF == MPASS_F32) {
    for (int c = 0; c < nch; ++c) {
      const float4 a = *reinterpret_cast<const float4*>(A + c * sa + off);
      const float4 b = *reinterpret_cast<const float4*>(B + c * sb + off);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
    }
  } else {
    for (int c = 0; c < nch; c += 2) {
      const float4 a0 = *reinterpret_cast<const float4*>(A + c * sa + off);
      const float4 b0 = *reinterpret_cast<const float4*>(B + c * sb + off);
      float4 a1 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = a1;
      if (c + 1 < nch) {
        a1 = *reinterpret_cast<const float4*>(A + (c + 1) * sa + off);
        b1 = *reinterpret_cast<const float4*>(B + (c + 1) * sb + off);
      }
      const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      mbf8 ah, al, bh, bl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __bf16 x = (__bf16)av[j], y = (__bf16)bv[j];
        ah[j] = x;
        al[j] = (__bf16)(av[j] - (float)x);
        bh[j] = y;
        bl[j] = (__bf16)(bv[j] - (float)y);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    }
  }
  return acc;
}

// One chunk (16 entries of K) with A packed and B given per lane: b[s] is the entry
// k = 4s + g of this lane's column.
template <int MF>
__device__ __forceinline__ mf4 mma_pk1(int l, const float* A, const float (&b)[4], mf4 acc) {
  const int off = (l & 15) * 16 + (l >> 4) * 4;
  const float4 a = *reinterpret_cast<const float4*>(A + off);
  if (MF == MPASS_F32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b[3], acc, 0, 0, 0);
  } else {
    const float av[4] = {a.x, a.y, a.z, a.w};
    mbf8 ah, al, bh, bl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float xa = j < 4 ? av[j] : 0.0f, xb = j < 4 ? b[j] : 0.0f;
      const __bf16 x = (__bf16)xa, y = (__bf16)xb;
      ah[j] = x;
      al[j] = (__bf16)(xa - (float)x);
      bh[j] = y;
      bl[j] = (__bf16)(xb - (float)y);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  }
  return acc;
}

}  // namespace tdb
