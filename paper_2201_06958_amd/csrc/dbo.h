// Second-order streams with one tall mode: the dynamically bi-orthonormal (DBO) form
// that Sec. 2.2 recovers for p = 2, used in Sec. 3.2 (TDB-2) with the two spatial axes
// grouped into one mode of N1 N2 rows. V is M x K row-major (the tall mode first, the
// short mode of K <= 32 entries unit-stride); the ranks are equal, r1 = r2 = r <= K.
//
// A step walks the rows of V a few times, each row handled by one thread (the short
// mode and the ranks live in registers), with the sums over rows formed per block in
// LDS in a fixed order; single-block FP64 kernels do the r x r work between the row
// passes. The reinitialisation takes the tall mode's basis from the short mode's
// eigenvectors, U1 = V W2 U2 Sigma^-1 (the left singular vectors of the weighted
// unfolding), so no Gram of the tall mode is ever formed.
#pragma once
#include <hip/hip_runtime.h>
#include "tdb_common.h"

namespace tdb {

#define DBO_KMAX 32     // largest short mode
#define DBO_RMAX 32     // largest rank
#define DBO_GRID 512    // row blocks; each walks chunks of rows

// Row-kernel phases.
enum {
  DBO_PASS1 = 0,   // stage 1: sums of B1^T [F1 | D] (F1 = D W2 U2, B1 = W1 U1)
  DBO_FIN1 = 1,    // stage 1 basis derivative kU1, then the stage-2 sums at U1 + dt kU1
  DBO_FIN2 = 2,    // stage 2 basis update, Gram of the new U1, error and norm sums
  DBO_FINE = 3,    // explicit Euler: the basis update, Gram, error and norm sums
  DBO_NORM = 4,    // U1 <- U1 L^-T (Cholesky QR)
  DBO_MAP = 5,     // HOSVD: U1 = V Bmax2 Sigma^-1, with the per-column argmax sums
  DBO_FLIP = 6     // HOSVD: the sign of each column of U1
};
// Small-kernel steps.
enum { DBO_PREP = 0, DBO_MID1 = 1, DBO_MID2 = 2, DBO_END = 3, DBO_SIGN = 4 };

// Offsets (doubles) into the small FP64 work area: pseudo-inverses and M1 = Cdot P1 of
// both stages, E = C U2^T of the error, the inverse Cholesky factor of the QR, and
// the HOSVD column signs.
constexpr int DBO_RR = DBO_RMAX * DBO_RMAX;
constexpr int DBO_WK_P1 = 0;
constexpr int DBO_WK_P2 = 2 * DBO_RR;
constexpr int DBO_WK_M1 = 4 * DBO_RR;
constexpr int DBO_WK_E = 6 * DBO_RR;
constexpr int DBO_WK_LI = 6 * DBO_RR + DBO_RMAX * DBO_KMAX;
constexpr int DBO_WK_SG = 7 * DBO_RR + DBO_RMAX * DBO_KMAX;
constexpr int DBO_WK_SIZE = DBO_WK_SG + 2 * DBO_RMAX;

struct DboArgs {
  long long M;           // rows of the tall mode
  int K, r;              // short mode size, rank (both modes)
  int ldU1, ldU2;        // leading dimensions of U1, U2 (the caps)
  int full2;             // r == K: the short mode's basis derivative vanishes
  int euler;             // explicit Euler (one stage)
  int TR;                // rows per chunk (rows staged in LDS together)
  int nblk;              // row blocks launched (partial-sum slots)
  int caps;              // HOSVD: columns of the basis at the caps
  double dt, dscale;     // step; 1/dt for a difference of snapshots, 1 for a derivative
  const void* V1;        // snapshot at t_{k+1} (data type), M x K
  const void* V0;        // snapshot at t_k, or NULL when D1 is given
  const void* D1;        // given stage-1 derivative, or NULL
  const void* D2;        // given stage-2 derivative, or NULL (stage 1's)
  double* U1;            // M x ldU1 basis (updated in place)
  double* kU1;           // M x ldU1 stage-1 basis derivative
  const double* w1;      // M quadrature weights
  const double* w2;      // K quadrature weights
  double* part;          // nblk x slot partial sums
  double* wk;            // small work area (DBO_WK_SIZE)
  void* Bt;              // 2 x DBO_KMAX x DBO_RMAX compute type: W2 U2 of each stage
  double* C0;            // r x r core (updated in place)
  double* U2;            // K x ldU2 basis (updated in place)
  double *kU2, *Us2, *Cs, *kC;
  // HOSVD of the tall mode
  double* Umax1;         // M x ldU1
  const double* sig2;    // singular values of the short mode (descending)
  const double* Bmax2;   // W2 Umax2, K x ldU2
  double* sig1;          // the tall mode's singular values (the same)
  double* Cmax;          // caps x caps core of the truncated HOSVD
};

// Row bucket: the short mode rounded up to 8, 16 or 32.
__host__ __device__ inline int dbo_bucket(int K) { return K <= 8 ? 8 : (K <= 16 ? 16 : 32); }
// Rows per chunk for a bucket (each row's vectors sit in LDS: 74, 79 and 108 KB).
__host__ __device__ inline int dbo_rows(int nb) { return nb <= 8 ? 256 : (nb <= 16 ? 128 : 64); }
// Doubles of one partial-sum slot for a phase.
__host__ __device__ inline int dbo_slot(int phase, int r, int K) {
  if (phase == DBO_PASS1 || phase == DBO_FIN1) return r * (r + K);
  if (phase == DBO_FIN2 || phase == DBO_FINE) return (r + 1) * (r + 2);
  if (phase == DBO_MAP) return 3 * DBO_RMAX;
  return 0;
}
__host__ __device__ inline int dbo_slot_max(int K) {
  const int a = DBO_RMAX * (DBO_RMAX + K), b = (DBO_RMAX + 1) * (DBO_RMAX + 2), c = 3 * DBO_RMAX;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}
size_t dbo_lds_bytes(int nb);

template <typename TD, typename T>
hipError_t launch_dbo_rows(const DboArgs& a, int phase, CtrlState* ctrl, hipStream_t s);
template <typename T>
hipError_t launch_dbo_small(const DboArgs& a, int step, CtrlState* ctrl, hipStream_t s);

}  // namespace tdb
