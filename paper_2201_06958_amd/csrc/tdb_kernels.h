// Kernel argument blocks and launchers (internal to the library).
#pragma once
#include "tdb_common.h"

namespace tdb {

// Per-stage preparation: weighted bases B_n (compute type) and core pseudo-inverses.
struct StageArgs {
  int p;
  int r[TDB_P];
  long long N[TDB_P];
  int ldU[TDB_P];
  const double* C;            // dense core, dims r
  const double* U[TDB_P];     // FP64 bases, N_n x ldU
  const double* w[TDB_P];     // weights
  void* B[TDB_P];             // out: N_n x r_n, compute type
  void* P[TDB_P];             // out: R_n x r_n, compute type
};

struct RhsArgs {
  int p, stage;
  double dt;
  double dscale;         // the data derivative is dscale times the projected operand
  int r[TDB_P];
  long long N[TDB_P];
  int ldU[TDB_P];
  long long core_size;
  const double* Cdot;         // raw projection of the data difference (before 1/dt)
  const double* H[TDB_P];     // raw F_(n) P_n (before 1/dt), N_n x r_n
  const double* w[TDB_P];
  double* C0;                 // committed state
  double* U0[TDB_P];
  double* Cs;                 // stage state
  double* Us[TDB_P];
  double* kC;                 // first-stage slopes
  double* kU[TDB_P];
};

struct QrArgs {
  int p;
  int r[TDB_P];
  long long N[TDB_P];
  int ldU[TDB_P];
  double* C0;
  double* Ctmp;
  double* U0[TDB_P];
  const double* w[TDB_P];
};

struct SigmaArgs {
  int p;
  int r[TDB_P];
  const double* C;
  double* Psi[TDB_P];         // optional rotation output (nullptr = values only)
};

template <typename T>
hipError_t launch_stage_prep(const StageArgs& a, CtrlState* ctrl, hipStream_t s);
hipError_t launch_rhs_stage(const RhsArgs& a, CtrlState* ctrl, hipStream_t s);
hipError_t launch_qr_fold(const QrArgs& a, CtrlState* ctrl, hipStream_t s);
hipError_t launch_core_sigma(const SigmaArgs& a, CtrlState* ctrl, hipStream_t s);
hipError_t launch_controller(CtrlState* ctrl, hipStream_t s);

// ---- bulk passes (stream_ops.hip)
// Generic n-mode product on a C-ordered tensor viewed as (A, Nin, Bsz):
// Y[a, o, b] = sum_i M[i*ms_i + o*ms_o] * X[a, i, b]; with X0 != nullptr the input is
// the difference X - X0. TX: input type, TC: arithmetic type, TY: output type.
template <typename TX, typename TC, typename TY>
hipError_t launch_ttm(const TX* X, const TX* X0, TY* Y, const TC* M, long long ms_i, long long ms_o,
                      long long A, int Nin, int Nout, long long Bsz, hipStream_t s);
// H[i, a] = sum_col F_(n)[i, col] P[col, a] for a tensor F with dims (outer, Nn, inner).
template <typename T>
hipError_t launch_fold_h(const T* F, const T* P, double* H, long long Nn, int rn,
                         long long outer, long long inner, hipStream_t s);
// Weighted error and norm partial sums over a reconstruction R of V:
// sum w (V - R)^2, sum w V^2 with w = prod_n w_n[i_n]; partials[2*block + {0,1}].
template <typename TV, typename TR>
hipError_t launch_err_partials(const TV* V, const TR* R, int p, const long long* N,
                               const double* const* w, double* partials, int nblocks,
                               hipStream_t s);
hipError_t launch_err_final(const double* partials, int nblocks, CtrlState* ctrl, hipStream_t s);
// *flag (device int, set to 0 by the launcher) becomes 1 if any of the n values is NaN
// or infinite.
template <typename T>
hipError_t launch_nonfinite_check(const T* x, long long n, int* flag, hipStream_t s);
// Second-order stage derivatives from three consecutive snapshots (n values each):
// D1 = (V1 - Vm) / (2 dt) at t_k, D2 = (3 V1 - 4 V0 + Vm) / (2 dt) at t_{k+1}.
template <typename T>
hipError_t launch_fd2(const T* Vm, const T* V0, const T* V1, T* D1, T* D2, long long n, double dt, hipStream_t s);
// Elementwise conversions.
template <typename TI, typename TO>
hipError_t launch_convert(const TI* in, TO* out, long long n, hipStream_t s);

// ---- HOSVD (hosvd_ops.hip)
struct HosvdModeArgs {
  int n;                 // mode
  long long A, Nn, Bsz;  // tensor viewed as (A, Nn, Bsz) around mode n
  const double* wa;      // product of weights of the modes before n (length A)
  const double* wb;      // product of weights of the modes after n (length Bsz)
  const double* wn;      // weights of mode n
};
template <typename TV>
hipError_t launch_gram_partials(const TV* V, const HosvdModeArgs& m, double* partials,
                                long long kchunk, int nchunks, hipStream_t s);
hipError_t launch_gram_reduce(const double* partials, double* G, const HosvdModeArgs& m,
                              int nchunks, hipStream_t s);
// Leading `k` eigenpairs of the symmetric Nn x Nn matrix G (destroyed), k <= TDB_RCAP.
// Writes sig[0..k] (k+1 singular values sqrt(max(lambda,0)), descending) and
// Umax (Nn x ldu, unscaled bases Q / sqrt(w_n)) and Bmax (Nn x k, W Umax).
struct EigArgs {
  int Nn, k, ldu;
  int k0;                // first reflector of the single-workgroup tail (set by the launcher)
  double* G;
  double* work;          // >= Nn * (k + 7) doubles
  double* sig;           // k + 1
  double* Umax;
  double* Bmax;
  const double* wn;
};
struct EigBatch {
  int count;
  EigArgs m[TDB_P];
};
// lam_scratch: count x (TDB_RCAP + 2) doubles; vec_scratch: count x TDB_NEIG x 64 x 6
// doubles of device workspace.
hipError_t launch_sym_eig(const EigBatch& b, double* lam_scratch, double* vec_scratch, hipStream_t s);

struct SelectArgs {
  int p, mode;           // DEC_*
  int caps[TDB_P];
  long long N[TDB_P];
  int ldU[TDB_P];
  int rank_init[TDB_P];  // all zero => rank rule
  const double* Cmax;    // dense caps-shaped core of the HOSVD
  const double* sig[TDB_P];
  const double* Umax[TDB_P];
  const double* nu2h;    // ||V||_W^2 from the Gram trace
  double* C0;
  double* U0[TDB_P];
};
hipError_t launch_rank_select(const SelectArgs& a, CtrlState* ctrl, hipStream_t s);
hipError_t launch_trace(const double* G, long long n, double* out, hipStream_t s);

}  // namespace tdb
