// Argument blocks of the fused third-order path (internal).
#pragma once
#include "tdb_common.h"

namespace tdb {

#define FERR_T1 8   // mode-1 slabs per block of the error pass
#define FIN_PART 1024 // LDS doubles for the partial blocks of the small matrix-core products
#define FIN_EPT 2      // basis-row elements per thread in one pass of a batch's finish row block
#define RED_U 4        // outputs per thread in one pass of the partial reduction
#define FIN_MU 8       // M_n values per thread loaded together with the first pass's operands
#define FQR_GP 1024   // LDS doubles for the QR's partial Gram blocks (four 16 x 16)

struct FPassArgs {
  const void* V1;
  const void* V0;            // NULL: the operand is V1 itself (a given derivative), else V1 - V0
  int N1, N2, N3, r1, r2, r3;
  int T1, T2, nt1, nt2;
  int need_h1, need_h2, need_f3;
  int stage_p;               // pseudo-inverses staged in LDS
  long long slot;            // partial elements per tile
  const void *B1, *B2, *B3;  // weighted bases, compute type, packed (ld = r)
  const void *P1, *P2, *P3;  // pseudo-inverses, compute type
  void* part;                // tiles x slot partials
  const int* hold;           // the controller's hold flag (the pass does nothing while set)
};

struct FReduceArgs {
  int stage;
  double dt;
  double dscale;             // the data derivative is dscale times the pass's operand
  int N1, N2, N3, r1, r2, r3, T1, T2, nt1, nt2;
  int need_h1, need_h2, need_f3;
  long long slot;
  const void* part;
  double* H[3];
  double *C0, *Cs, *kC, *Cdot2;
};

struct FFinishArgs {
  int stage, rowblocks, core_in_lds, rmax;
  double dt;
  double dscale;             // the data derivative is dscale times the pass's operand
  long long N[3];
  int r[3], ldU[3];
  const double* H[3];
  const void* Pcur[3];       // pseudo-inverses used by this stage's pass
  const double* w[3];
  double* U0[3];
  double* Us[3];
  double* kU[3];
  void* B[3];
  void* P[3];                // stage 1 only: pseudo-inverses of the stage-2 core
  const double* Cs;
  const double* kC;          // C_dot of stage 1
  const double* Cdot2;       // C_dot of stage 2
  double* M[3];              // M_n = dt C_dot_(n) P_n (r_n x r_n), written by k_fmprep
  int m_inline;              // 1: each row block forms M_n itself (no k_fmprep launch)
};

#define QR_ROWS 64     // rows of U_n per block of the QR kernels
#define FOLD_R 8       // core entries per thread when the QR folds the core in place (256 threads)

struct FQrArgs {
  int core_in_lds, rmax;     // core_in_lds: 2 folded in place, 1 in two LDS buffers, 0 in global memory
  long long N[3];
  int r[3], ldU[3];
  int nb[3];                 // QR_ROWS-row slabs of U_n (one block each, unless whole)
  int whole;                 // one block takes every slab (no partials through global memory)
  int slab_off;              // whole: LDS offset (doubles) of the slab rows, past the fold's buffers
  double* U0[3];
  const double* w[3];
  double* Li[3];             // L_n^-1 (U_n <- U_n L_n^-T by the post-step)
  double* gpart[3];          // nb[n] slab partial Grams of r_n x r_n
  double* C0;
  double* Ctmp;
  unsigned* counter;         // blocks done
  double* T3;                // C x_3 U_3 (r1 x r2 x N3) of the folded core, for the error pass
};

struct FPostArgs {
  int eblocks, core_in_lds, want_pinv, rmax;
  long long N[3];
  int r[3], ldU[3];
  const double* C;
  const double* U[3];
  const double* w[3];
  void* B[3];
  void* P[3];
  void* E;                   // r1 x N2 x N3, compute type
  void* U1c;                 // N1 x r1, compute type
  const double* T3;          // C x_3 U_3 when already formed (else NULL: formed per block)
  int want_sigma;            // also form the singular values of the core unfoldings
  double* G[3];              // core Grams C_(n) C_(n)^T kept for a later singular-value test
  const double* Li[3];       // when set: U_n is not yet normalised, U_n <- U_n L_n^-T first
  double* Uw[3];             // U_n (written back normalised when Li is set)
  int stage_all;             // expansion blocks stage all their rows at once (else POST_CH at a time)
};
#define POST_CH 64           // rows per chunk of the expansion blocks

struct FErrArgs {
  const void* V;
  int N1, r1, T1, gx, gy;
  long long M;               // N2 * N3
  const void* E;
  const void* U1c;
  const double* w1;
  const double* w23;
  double* part;
  unsigned* counter;
  const double* G[3];        // core Grams of the committed state (lazy singular values)
  int rmax;                  // largest rank (LDS of the final kernel)
  const int* skip;           // the learned gate skips this pass (NULL: never)
  const int* hold;           // the controller's hold flag (batches: the pass does nothing while set)
  const int* would_skip;     // the gate's verdict, recorded in the controller state
  const float* yhat;         // the gate's prediction (log10 of the error)
  CtrlState* mirror;         // pinned host copy of the controller state the final kernel
                             // writes at its end (NULL: none)
  unsigned long long* seq;   // pinned word set to seq_val once the mirror is written
  unsigned long long seq_val;
};

// ev0/ev1 (may be null): events stamped by the dispatch itself at kernel start and end.
// Lanes that share one reduction output: a power of two (<= 64) such that each lane
// sums at most 8 partials when possible.
__host__ __device__ inline int red_lanes(int count) {
  int L = 1;
  while (L < 64 && L * 8 < count) L <<= 1;
  return L;
}
__host__ __device__ inline long long pad64(long long x) { return (x + 63) / 64 * 64; }
// Work items of the partial reduction (each output takes red_lanes(count) lanes; each
// kind of output starts on a wave boundary).
__host__ __device__ inline long long freduce_items(const FReduceArgs& a) {
  const long long nH1 = a.need_h1 ? (long long)a.N1 * a.r1 : 0;
  const long long nH2 = a.need_h2 ? (long long)a.N2 * a.r2 : 0;
  const long long nH3 = a.need_f3 ? (long long)a.N3 * a.r3 : 0;
  const long long nC = (long long)a.r1 * a.r2 * a.r3;
  const int L3 = red_lanes(a.nt1 * a.nt2);
  return pad64(nH1 * red_lanes(a.nt2)) + pad64(nH2 * red_lanes(a.nt1)) + pad64(nH3 * L3) + pad64(nC * L3);
}

template <typename TD, typename T>
hipError_t launch_fpass(const FPassArgs& a, size_t lds, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_freduce(const FReduceArgs& a, CtrlState* c, hipStream_t s);
template <typename T>
hipError_t launch_ffinish(const FFinishArgs& a, size_t lds, CtrlState* c, hipStream_t s);
template <typename T>
hipError_t launch_fmprep(const FFinishArgs& a, size_t lds, CtrlState* c, hipStream_t s);
hipError_t launch_fqr(const FQrArgs& a, size_t lds, CtrlState* c, hipStream_t s);
template <typename T>
hipError_t launch_fpost(const FPostArgs& a, size_t lds, CtrlState* c, hipStream_t s);
template <typename TD, typename T>
hipError_t launch_ferr(const FErrArgs& a, CtrlState* c, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// LDS of the final error kernel (singular values of three r x r Grams when needed).
inline size_t ferr_final_lds(int rmax) { return (size_t)3 * ((size_t)rmax * rmax + 5 * (size_t)rmax) * 8 + 64; }

// Explicit Euler: commit the stage-1 state (C* and U*_n) as the new state, unless the
// step is held or a factorisation failed.
struct CommitArgs {
  int p;
  long long csz;
  double* C0;
  const double* Cs;
  long long N[4];
  int r[4], ldU[4];
  double* U0[4];
  const double* Us[4];
};
hipError_t launch_euler_commit(const CommitArgs& a, CtrlState* c, hipStream_t s);

// ---------------------------------------------------------------- matrix-core pass
// Stage-pass flavours on the matrix cores (tile 16 x 64 x N3, N3 <= 8, r1, r2 <= 32).
enum { MPASS_NONE = 0, MPASS_F32 = 1, MPASS_BF16S = 2 };
size_t mpass_lds_bytes(int r1, int r2, int r3, int N3, int T2, bool h1, bool h2, bool f3, bool pst);
// Waves per tile of the single-stream matrix-core pass: 16 (one tile per compute unit)
// for up to MPASS_W16_TILES tiles of 16 x 32 or more, 8 (two per compute unit) for up
// to MPASS_W8_TILES, else 4.
#define MPASS_W16_TILES 256
#define MPASS_W8_TILES 512
int mpass_waves(int tiles, int T2);
template <typename TD>
hipError_t launch_mpass(const FPassArgs& a, int flavor, size_t lds, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);

// ---------------------------------------------------------------- batched streams
// Many independent streams in one launch per kernel: the global block index selects
// a stream through `sid` and the block's index inside that stream's grid through
// `start` (first global block of each stream, n + 1 entries). The per-stream
// argument structs live in device tables; snapshot pointers come from their own
// per-step tables.
struct BatchMap {
  const int* sid;
  const int* start;
};

// What the host needs from each stream after a batched step.
struct BatchSummary {
  int decision, event, numeric, gated;
  int n_events[5];
  int would_skip;
  double eps, nu, eps2, nu2, eps_pred;
};

template <typename TD, typename T>
hipError_t launch_batch_fpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, size_t lds, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);
// Column-block stage pass of batches (rpass.hip): T2 columns of mode 2 with all of
// modes 1 and 3 per workgroup of 8 waves; the mode-3 product is applied to the small
// results. T2 follows the mode-3 extent the batch's streams share (rpass_cols_for).
int rpass_cols_for(int n3c);
bool rpass_cols_ok(int n3c, int t2);
size_t rpass_lds_bytes(int T2, int r1, int r2, int N3);
bool rpass_shape_ok(int r1, int r2, int r3, int T2, int N3);
template <typename TD>
hipError_t launch_batch_rpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, int flavor, int n3c, int t2, int vw, size_t lds, hipStream_t s,
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename TD>
hipError_t launch_batch_mpass(const FPassArgs* tab, const void* const* v1, const void* const* v0, BatchMap m,
                              int blocks, int flavor, size_t lds, hipStream_t s, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_batch_freduce(const FReduceArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                                hipStream_t s);
// Roles of the finish and post-step kernels: the whole kernel (one stream), or one of
// its two block kinds launched on its own (a batch).
enum { ROLE_ALL = 0, ROLE_ROWS = 1, ROLE_PINV = 2, ROLE_MODES = 1, ROLE_EXP = 2 };
template <typename T>
hipError_t launch_batch_ffinish(const FFinishArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                                size_t lds, int role, hipStream_t s);
template <typename T>
hipError_t launch_batch_fmprep(const FFinishArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, int stage,
                               size_t lds, hipStream_t s);
hipError_t launch_batch_fqr(const FQrArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, size_t lds,
                            hipStream_t s);
template <typename T>
hipError_t launch_batch_fpost(const FPostArgs* tab, CtrlState* const* ctab, BatchMap m, int blocks, size_t lds,
                              int role, hipStream_t s);
// r1c (4..32, a multiple of 4): the column-block error pass compiled for r1 <= r1c
// (every stream's plan has gx = ceil(M/FEC_COLS) blocks of all rows, gy = 1); 0: the
// slab pass.
#define FEC_COLS 256
// The final kernel writes stream i's summary to out[i] (streams found held write
// nothing) and, with counter (device, zero between launches) given, advances *seq once
// every stream's summary is visible to the host.
template <typename TD, typename T>
hipError_t launch_batch_ferr(const FErrArgs* tab, const void* const* v1, BatchMap m, int blocks, int nstreams,
                             CtrlState* const* ctab, BatchSummary* out, unsigned* counter, unsigned long long* seq,
                             size_t lds_final, int r1c, hipStream_t s, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);
template <typename TD, typename T>
hipError_t launch_batch_ferr_partials(const FErrArgs* tab, const void* const* v1, BatchMap m, int blocks, int r1c,
                                      hipStream_t s);
hipError_t launch_batch_fetch_ptrs(const void* const* h1, const void* const* h0, const void** d1, const void** d0,
                                   int n, hipStream_t s);
hipError_t launch_batch_hold_mask(CtrlState* const* ctab, const int* mask, int* save, int n, int restore,
                                  hipStream_t s);

}  // namespace tdb
