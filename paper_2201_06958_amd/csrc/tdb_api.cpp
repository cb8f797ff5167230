// Host runtime and C ABI of the TDB compressor: validates configurations, owns the
// device workspace, sequences the kernels of one snapshot step and of the HOSVD
// (re)initialisation, and keeps the per-step statistics.
#include "../../include/tdb.h"
#include "tdb_kernels.h"
#include "fused.h"
#include "gate.h"
#include "noalloc.h"
#include "dbo.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <unordered_map>
#include <mutex>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace tdb;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct tdb_ctx {
  tdb_config cfg{};
  int p = 0;
  long long N[TDB_P] = {1, 1, 1, 1};
  long long S = 0;
  int caps[TDB_P] = {1, 1, 1, 1};
  int r[TDB_P] = {1, 1, 1, 1};
  int ldU[TDB_P] = {1, 1, 1, 1};
  bool f32 = false;          // bulk passes in FP32 (or BF16-split products with FP32 sums)
  bool bf16s = false;        // BF16-split products in the matrix-core stage pass
  bool no_mfma = false;      // keep the generic stage pass (a batch with mixed shapes)
  bool dbo = false;          // order 2 on the row passes (tall first mode, short second)
  bool tall = false;         // the first mode exceeds the eigensolver's size: its HOSVD
                             // basis comes from the second mode's eigenvectors
  double* dbo_wk = nullptr;  // small FP64 work area of the row passes
  void* dbo_bt = nullptr;    // W2 U2 of both stages in the compute type
  double* dbo_part = nullptr;
  int dbo_nblk = 1;
  bool dbo_prep = false;     // stage-1 operands of the current state are prepared
  bool no_rpass = false;     // keep the tile pass in a batch (streams that disagree)
  bool ferr_cols = false;    // batch member on the column-block error pass
  int rpass_cols = 64;       // columns of mode 2 per workgroup of the column-block pass
  bool data32 = false;       // snapshots stored as FP32
  size_t celt = 8;           // bytes per compute element
  size_t delt = 8;           // bytes per data element
  long long core_cap = 1;
  long long Rmax = 1;

  std::vector<void*> allocs;
  double *C0 = nullptr, *Cs = nullptr, *kC = nullptr, *Ctmp = nullptr, *Cdot = nullptr;
  double *U0[TDB_P] = {}, *Us[TDB_P] = {}, *kU[TDB_P] = {}, *H[TDB_P] = {}, *w[TDB_P] = {};
  void *B[TDB_P] = {}, *P[TDB_P] = {}, *Uc[TDB_P] = {};
  void *Cc = nullptr, *wsA = nullptr, *wsB = nullptr;
  void* wsZ[2] = {nullptr, nullptr};   // plain path: the two shared first contractions
  double *err_part = nullptr;
  int err_blocks = 1024;
  CtrlState* ctrl = nullptr;
  CtrlState* ctrl_h = nullptr;   // pinned mirror
  // HOSVD workspace
  double *G[TDB_P] = {}, *gpart = nullptr, *eigw[TDB_P] = {}, *sig[TDB_P] = {};
  double *Umax[TDB_P] = {}, *Bmax[TDB_P] = {}, *Cmax = nullptr, *hsA = nullptr, *hsB = nullptr;
  double *wa[TDB_P] = {}, *wb[TDB_P] = {}, *nu2h = nullptr;
  double* eig_lam = nullptr;     // eigenvalues of the mode Grams (per mode, TDB_RCAP + 2)
  double* eig_vec = nullptr;     // inverse-iteration vectors and factors (per mode, TDB_NEIG x 64 x 6)
  double *Psi[TDB_P] = {};
  // snapshots
  const void* Vprev = nullptr;
  void* Vcopy = nullptr;
  // second-order differences: the snapshot before Vprev (NULL until two are held), the
  // second copy buffer (TDB_COPY) and the two stage derivatives
  const void* Vprev2 = nullptr;
  void* Vcopy2 = nullptr;
  void* Dfd[2] = {nullptr, nullptr};
  // bookkeeping
  std::string err;
  tdb_stats stats{};
  double crbar_den = 0.0, t_now = 0.0;
  long long step = 0;
  bool ready = false;
  // fused third-order path
  bool fused = false;            // configuration allows the fused path
  bool post_valid = false;       // B_n, P_n, E of the current state are prepared
  int lds_max = 65536;
  void* fpart = nullptr;
  long long fpart_elems = 0;
  double* Cdot2 = nullptr;
  double *Lq[TDB_P] = {}, *qpart[TDB_P] = {};   // L_n^-1 of the QR; its slab partial Grams
  double *Mbuf[TDB_P] = {}, *T3buf = nullptr;   // M_n of a stage; C x_3 U_3 after the QR
  double* Gsave[TDB_P] = {};     // core Grams of the committed state (lazy singular values)
  bool sigma_every_step = false; // form the core singular values at every step
  void* P2[TDB_P] = {};          // pseudo-inverses of the stage-2 core
  void *E = nullptr, *U1c = nullptr;
  double *w23 = nullptr, *ferr_part = nullptr;
  unsigned* counters = nullptr;
  int ferr_gx = 1, ferr_gy = 1;
  long long fused_steps = 0, plain_steps = 0;
  long long n_nonfinite = 0;     // steps discarded for non-finite data
  int last_prec = -1;            // TDB_PREC_* the last step's stage pass ran in
  int last_path = 0;             // TDB_PATH_PLAIN or TDB_PATH_FUSED of the last step
  int* d_flag = nullptr;         // device word of the non-finite checks
  // learned gate of a single stream (fused path): the handle's own copy of the
  // parameters and feature statistics, the singular-value history and the verdicts
  int gate_mode = 0;             // GATE_*
  float *g_params = nullptr, *g_mean = nullptr, *g_std = nullptr, *g_hist = nullptr, *g_yhat = nullptr;
  int *g_hcount = nullptr, *g_skip = nullptr, *g_would = nullptr;
  CtrlState** g_ctab = nullptr;  // device array holding ctrl (the inference kernel takes a table)
  bool batch_owned = false;      // lives inside a tdb_batch
  tdb_batch_ctx* owner = nullptr;   // that batch (its pending step is resolved for reads)
  bool sigma_stale = false;      // stats.sigma not refreshed since the last batched step
  // pipelined ingest (fused path, borrowed snapshots): each call enqueues its step and
  // then reads the previous step's decision, so the device never waits for the host
  // between steps; a decision that needs the host holds the steps enqueued after it
  bool pipelined = false;
  bool pending = false;          // the newest step's decision has not been read yet
  const void* Vpend = nullptr;   // its snapshot (kept by the caller until the next call)
  hipStream_t pend_stream = nullptr;
  CtrlState* ctrl_hb[2] = {};    // pinned mirrors of the controller state, one per step in flight
  hipEvent_t ev_ctrl[2] = {};   // recorded on demand: another stream waits for a pending step
  unsigned long long* seq_h = nullptr;   // pinned words the final error kernel sets per mirror
  unsigned long long seq_next = 0, seq_want[2] = {0, 0};
  int mirror = 0;                // mirror of the newest step
  // optional pass timing (events recorded on the caller's stream), of every step or of
  // every prof_every-th step (prof_now: the step being enqueued is timed)
  bool prof = false;
  int prof_every = 1;
  long long prof_steps = 0;
  bool prof_now = true;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[2];
  // a second stream (default priority) for the kernels that run beside another one: the
  // stage-1 pseudo-inverses beside the row blocks, the post-step's mode blocks beside its
  // expansion blocks (fork and join by events, captured into the step's graph)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork[2] = {}, ev_join[2] = {};
  bool side_failed = false;

  ~tdb_ctx() {
    for (auto& v : ev_used)
      for (auto& e : v) { ev_pool.push_back(e.first); ev_pool.push_back(e.second); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_ctrl)
      if (e) (void)hipEventDestroy(e);
    for (void* q : allocs) (void)hipFree(q);
    for (CtrlState* m : ctrl_hb)
      if (m) (void)hipHostFree(m);
    if (seq_h) (void)hipHostFree(seq_h);
  }
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError(); /* clear it, or the next launch check reports it */   \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
      return TDB_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

namespace {

tdb_status dalloc(tdb_ctx* h, void** out, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    h->err = "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e);
    return TDB_ENOMEM;
  }
  h->allocs.push_back(q);
  *out = q;
  return TDB_OK;
}

template <typename T>
tdb_status dallocT(tdb_ctx* h, T** out, size_t count) {
  return dalloc(h, reinterpret_cast<void**>(out), count * sizeof(T));
}

#define TRY(expr)                          \
  do {                                     \
    tdb_status s_ = (expr);                \
    if (s_ != TDB_OK) return s_;           \
  } while (0)

tdb_status validate(const tdb_config* c, std::string& msg) {
  if (!c) { msg = "config is NULL"; return TDB_EINVAL; }
  if (c->order < 2 || c->order > TDB_MAX_ORDER) { msg = "order must be in [2, 8]"; return TDB_EINVAL; }
  if (c->order > TDB_P) { msg = "the library supports tensor order 2..4"; return TDB_EUNSUPPORTED; }
  for (int n = 0; n < c->order; ++n) {
    if (c->dims[n] < 1) { msg = "dims must be positive"; return TDB_EINVAL; }
    if (c->rank_max[n] < 1) { msg = "rank_max must be positive"; return TDB_EINVAL; }
    if (c->rank_max[n] > TDB_RCAP && c->rank_max[n] < c->dims[n]) {
      msg = "rank_max above 64 is not supported by the library";
      return TDB_EUNSUPPORTED;
    }
    if (c->dims[n] > TDB_NEIG && !(n == 0 && c->order == 2 && c->path != TDB_PATH_PLAIN && c->dims[1] <= DBO_KMAX)) {
      msg = c->order == 2 && n == 1 && c->dims[0] <= DBO_KMAX
                ? "an order-2 stream takes its tall mode first (V is N1 x N2 with N2 <= 32 unit-stride)"
                : "mode sizes above 512 are supported only for the first mode of an order-2 stream whose second "
                  "mode has at most 32 entries";
      return TDB_EUNSUPPORTED;
    }
    if (c->rank_init[n] < 0) { msg = "rank_init must be >= 0"; return TDB_EINVAL; }
    if (c->weights[n]) {
      for (long long i = 0; i < c->dims[n]; ++i)
        if (!(c->weights[n][i] > 0.0) || !std::isfinite(c->weights[n][i])) {
          msg = "weights must be positive and finite";
          return TDB_EINVAL;
        }
    }
  }
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) { msg = "dt must be positive"; return TDB_EINVAL; }
  if (c->data_dtype != TDB_F64 && c->data_dtype != TDB_F32) { msg = "bad data_dtype"; return TDB_EINVAL; }
  if (c->precision != TDB_PREC_F64 && c->precision != TDB_PREC_F32 && c->precision != TDB_PREC_BF16SPLIT) {
    msg = "bad precision";
    return TDB_EINVAL;
  }
  if (c->path != TDB_PATH_AUTO && c->path != TDB_PATH_PLAIN && c->path != TDB_PATH_FUSED) {
    msg = "bad path";
    return TDB_EINVAL;
  }
  if (c->snapshot_mode != TDB_COPY && c->snapshot_mode != TDB_BORROW) { msg = "bad snapshot_mode"; return TDB_EINVAL; }
  if (!(c->eps_th > 0.0) && c->adaptive) { msg = "eps_th must be positive for adaptive runs"; return TDB_EINVAL; }
  if (c->gamma_th >= 100.0) { msg = "gamma_th must be below 100"; return TDB_EINVAL; }
  if (c->slope_window < 0 || c->slope_window > TDB_WIN || c->slope_window == 1) {
    msg = "slope_window must be 0 (default) or in [2, 64]";
    return TDB_EINVAL;
  }
  if (c->integrator != TDB_INT_HEUN && c->integrator != TDB_INT_EULER) { msg = "bad integrator"; return TDB_EINVAL; }
  if (c->fd_order < 0 || c->fd_order > 2) { msg = "fd_order must be 0, 1 or 2"; return TDB_EINVAL; }
  return TDB_OK;
}

// K-chunks of the HOSVD Gram partials for a contraction of length K: about 256 terms per
// block (the kernel is latency-bound, so more, shorter blocks), at most 256 chunks.
long long gram_chunks(long long K) { return std::max<long long>(1, std::min<long long>(256, (K + 255) / 256)); }

long long prod_ll(const int* a, int p, int skip = -1) {
  long long q = 1;
  for (int k = 0; k < p; ++k)
    if (k != skip) q *= a[k];
  return q;
}

struct PassPlan {
  int T1 = 1, T2 = 1, nt1 = 1, nt2 = 1, stage_p = 0;
  int mfma = 0;              // MPASS_* flavour of the stage pass
  int rows = 0;              // 1: the column-block pass of batches (T1 = N1 padded, T2 columns)
  long long slot = 0;
  size_t lds = 0;
  bool ok = false;
};

// LDS bytes of one stage-pass tile of T1 x T2 x N3 at ranks r (without the staged
// pseudo-inverses), and the bytes of the staged pseudo-inverses. `worst` counts every
// optional term (a plan made at the caps must also hold smaller ranks, for which the
// third-mode terms may switch on).
size_t pass_lds(const tdb_ctx* h, const int* r, int T1, int T2, bool worst = false) {
  const long long N3 = h->N[2];
  const int r1 = r[0], r2 = r[1], r3 = r[2];
  long long e = (long long)T1 * T2 * N3 + (long long)T1 * T2 * r3 + (long long)T1 * r2 * r3 +
                (long long)r1 * T2 * r3 + 2LL * T1 * r1 + 2LL * T2 * r2 + 2LL * N3 * r3;
  if (r3 < N3 || worst) e += (long long)T1 * r2 * N3 + (long long)r1 * r2 * N3;
  return (size_t)e * h->celt;
}
size_t pass_p_bytes(const tdb_ctx* h, const int* r, bool worst = false) {
  const long long c = (long long)r[0] * r[1] * r[2];
  const long long pe = (r[0] < h->N[0] || worst ? c : 0) + (r[1] < h->N[1] || worst ? c : 0) +
                       (r[2] < h->N[2] || worst ? c : 0);
  return (size_t)pe * h->celt;
}
size_t mpass_bytes(const tdb_ctx* h, const int* r, int T2, bool pst, bool worst) {
  return mpass_lds_bytes(r[0], r[1], r[2], (int)h->N[2], T2, worst || r[0] < h->N[0], worst || r[1] < h->N[1],
                         worst || r[2] < h->N[2], pst);
}

// Whether the matrix-core stage pass takes ranks r (FP32 arithmetic, order 3,
// N3 <= 8, r1, r2 <= 32, LDS fits); TDB_MFMA=0 in the environment turns it off.
bool mfma_ok(const tdb_ctx* h, const int* r, bool worst) {
  if (!h->f32 || h->p != 3 || h->no_mfma || h->N[2] > 8 || r[0] > 32 || r[1] > 32 || r[2] > h->N[2]) return false;
  if (const char* env = std::getenv("TDB_MFMA"))
    if (env[0] == '0') return false;
  return mpass_bytes(h, r, 16, false, worst) <= (size_t)h->lds_max;
}

// Whether a batch member takes the column-block pass at ranks r (TDB_RPASS=0 turns it
// off).
bool rpass_ok(const tdb_ctx* h, const int* r, bool worst) {
  if (!h->batch_owned || h->no_rpass || !mfma_ok(h, r, worst)) return false;
  if (const char* env = std::getenv("TDB_RPASS"))
    if (env[0] == '0') return false;
  if (!rpass_shape_ok(r[0], r[1], r[2], h->rpass_cols, (int)h->N[2])) return false;
  if (h->N[0] * h->N[1] * h->N[2] >= (1LL << 31)) return false;   // 32-bit offsets
  return rpass_lds_bytes(h->rpass_cols, r[0], r[1], (int)h->N[2]) <= (size_t)h->lds_max;
}

// LDS up to which two matrix-core tiles still share a compute unit (160 KB each);
// the pseudo-inverses are staged only within it, since occupancy hides more latency
// than the staging saves.
size_t mpass_occupancy_budget(const tdb_ctx* h) { return std::min<size_t>((size_t)h->lds_max, 78 * 1024); }

// Tile shape of the fused stage pass for ranks r. Matrix-core tiles are 16 x T2 x N3
// with T2 the largest of 64, 32, 16 that fits and (for a single stream) still gives
// at least one tile per compute unit; generic tiles hold about `target` elements,
// shrunk until their LDS fits. `worst`: size for every rank up to r (batches).
PassPlan plan_pass(const tdb_ctx* h, const int* r, bool worst = false) {
  PassPlan pl;
  const long long N1 = h->N[0], N2 = h->N[1], N3 = h->N[2];
  if (rpass_ok(h, r, worst)) {
    const int T2 = h->rpass_cols;
    const int N1p = (int)((N1 + 15) & ~15LL);
    pl.mfma = h->bf16s ? MPASS_BF16S : MPASS_F32;
    pl.rows = 1;
    pl.T1 = N1p;
    pl.T2 = T2;
    pl.nt1 = 1;
    pl.nt2 = (int)((N2 + T2 - 1) / T2);
    pl.slot = (long long)N1p * r[0] + (long long)T2 * r[1] + N3 * r[2] + (long long)r[0] * r[1] * r[2];
    pl.lds = rpass_lds_bytes(T2, r[0], r[1], (int)N3);
    pl.ok = true;
    return pl;
  }
  if (mfma_ok(h, r, worst)) {
    int T2 = 64;
    while (T2 > 16 && mpass_bytes(h, r, T2, false, worst) > (size_t)h->lds_max) T2 /= 2;
    if (!h->batch_owned)
      while (T2 > 16 && ((N1 + 15) / 16) * ((N2 + T2 - 1) / T2) < MPASS_W16_TILES) T2 /= 2;
    pl.mfma = h->bf16s ? MPASS_BF16S : MPASS_F32;
    pl.T1 = 16;
    pl.T2 = T2;
    pl.nt1 = (int)((N1 + 15) / 16);
    pl.nt2 = (int)((N2 + T2 - 1) / T2);
    // a tile that has its compute unit to itself may stage into all of its LDS
    const bool alone = !h->batch_owned && mpass_waves(pl.nt1 * pl.nt2, T2) == 16;
    pl.stage_p = mpass_bytes(h, r, T2, true, worst) <= (alone ? (size_t)h->lds_max : mpass_occupancy_budget(h)) ? 1 : 0;
    pl.slot = 16LL * r[0] + (long long)T2 * r[1] + N3 * r[2] + (long long)r[0] * r[1] * r[2];
    pl.lds = mpass_bytes(h, r, T2, pl.stage_p != 0, worst);
    pl.ok = true;
    return pl;
  }
  long long target = h->f32 ? 4096 : 2048;
  if (const char* env = std::getenv("TDB_PASS_TILE")) {
    const long long v = std::atoll(env);
    if (v >= 64 && v <= (1 << 20)) target = v;
  }
  int T2 = (int)std::min<long long>(N2, 64);
  int T1 = (int)std::max<long long>(1, std::min<long long>(N1, target / std::max<long long>(1, T2 * N3)));
  while (pass_lds(h, r, T1, T2, worst) > (size_t)h->lds_max && T1 > 1) T1 = std::max(1, T1 / 2);
  while (pass_lds(h, r, T1, T2, worst) > (size_t)h->lds_max && T2 > 8) T2 = std::max(8, T2 / 2);
  if (pass_lds(h, r, T1, T2, worst) > (size_t)h->lds_max) return pl;
  // stage the pseudo-inverses too when they fit
  if (pass_lds(h, r, T1, T2, worst) + pass_p_bytes(h, r, worst) <= (size_t)h->lds_max) pl.stage_p = 1;
  pl.T1 = T1;
  pl.T2 = T2;
  pl.nt1 = (int)((N1 + T1 - 1) / T1);
  pl.nt2 = (int)((N2 + T2 - 1) / T2);
  pl.slot = (long long)T1 * r[0] + (long long)T2 * r[1] + N3 * r[2] + (long long)r[0] * r[1] * r[2];
  pl.lds = pass_lds(h, r, T1, T2, worst) + (pl.stage_p ? pass_p_bytes(h, r, worst) : 0);
  pl.ok = true;
  return pl;
}

// The plan `base` (made with `worst` for larger ranks) applied to ranks r: same tiles
// and LDS budget, the partial slot and the staging decision of r.
PassPlan plan_under(const tdb_ctx* h, const int* r, const PassPlan& base) {
  PassPlan pl = base;
  pl.slot = (long long)base.T1 * r[0] + (long long)base.T2 * r[1] + h->N[2] * r[2] + (long long)r[0] * r[1] * r[2];
  if (!base.ok) { pl.ok = false; return pl; }
  if (base.rows) {
    if (!rpass_shape_ok(r[0], r[1], r[2], base.T2, (int)h->N[2])) {
      pl.ok = false;
      return pl;
    }
    pl.lds = rpass_lds_bytes(base.T2, r[0], r[1], (int)h->N[2]);
    if (pl.lds > (size_t)h->lds_max) pl.ok = false;
    return pl;
  }
  if (base.mfma) {
    // LDS of the current ranks (a batch launches with the largest over its streams)
    if (r[0] > 32 || r[1] > 32 || mpass_bytes(h, r, base.T2, false, false) > (size_t)h->lds_max) {
      pl.ok = false;
      return pl;
    }
    const bool alone = !h->batch_owned && mpass_waves(base.nt1 * base.nt2, base.T2) == 16;
    pl.stage_p = mpass_bytes(h, r, base.T2, true, false) <= (alone ? (size_t)h->lds_max : mpass_occupancy_budget(h)) ? 1 : 0;
    pl.lds = mpass_bytes(h, r, base.T2, pl.stage_p != 0, false);
    return pl;
  }
  const size_t need = pass_lds(h, r, base.T1, base.T2);
  if (need > base.lds) { pl.ok = false; return pl; }
  pl.stage_p = need + pass_p_bytes(h, r) <= base.lds ? 1 : 0;
  pl.lds = need + (pl.stage_p ? pass_p_bytes(h, r) : 0);
  return pl;
}

tdb_status setup_fused(tdb_ctx* h, const std::vector<std::vector<double>>& wh);

tdb_status setup(tdb_ctx* h, const tdb_config* cfg) {
  h->cfg = *cfg;
  if (h->cfg.slope_window == 0) h->cfg.slope_window = 10;
  h->p = cfg->order;
  h->S = 1;
  for (int n = 0; n < h->p; ++n) {
    h->N[n] = cfg->dims[n];
    h->S *= h->N[n];
  }
  // caps: min(rank_max, N_n, 64), then <= product of the other caps
  for (int n = 0; n < h->p; ++n) {
    long long c = std::min<long long>(cfg->rank_max[n], h->N[n]);
    h->caps[n] = (int)std::min<long long>(c, TDB_RCAP);
  }
  for (int n = 0; n < h->p; ++n) {
    long long o = prod_ll(h->caps, h->p, n);
    if (h->caps[n] > o) h->caps[n] = (int)o;
  }
  for (int n = 0; n < h->p; ++n) h->ldU[n] = h->caps[n];
  h->f32 = cfg->precision != TDB_PREC_F64;
  h->bf16s = cfg->precision == TDB_PREC_BF16SPLIT;
  h->data32 = cfg->data_dtype == TDB_F32;
  h->celt = h->f32 ? 4 : 8;
  h->delt = h->data32 ? 4 : 8;
  h->core_cap = prod_ll(h->caps, h->p);
  h->Rmax = 1;
  for (int n = 0; n < h->p; ++n) h->Rmax = std::max(h->Rmax, prod_ll(h->caps, h->p, n));
  // order 2 with a short second mode steps on the row passes; a first mode beyond the
  // eigensolver's size takes its HOSVD basis from the second mode's eigenvectors
  h->dbo = h->p == 2 && cfg->path != TDB_PATH_PLAIN && h->N[1] <= DBO_KMAX && h->N[0] >= h->N[1];
  h->tall = h->dbo && h->N[0] > TDB_NEIG;

  // ---- state and stage buffers
  TRY(dallocT(h, &h->C0, h->core_cap));
  TRY(dallocT(h, &h->Cs, h->core_cap));
  TRY(dallocT(h, &h->kC, h->core_cap));
  TRY(dallocT(h, &h->Ctmp, h->core_cap));
  TRY(dallocT(h, &h->Cdot, h->core_cap));
  TRY(dalloc(h, &h->Cc, h->core_cap * h->celt));
  for (int n = 0; n < h->p; ++n) {
    const size_t nu = (size_t)h->N[n] * h->ldU[n];
    TRY(dallocT(h, &h->U0[n], nu));
    TRY(dallocT(h, &h->Us[n], nu));
    TRY(dallocT(h, &h->kU[n], nu));
    TRY(dallocT(h, &h->H[n], nu));
    TRY(dallocT(h, &h->w[n], h->N[n]));
    TRY(dalloc(h, &h->B[n], nu * h->celt));
    TRY(dalloc(h, &h->Uc[n], nu * h->celt));
    TRY(dalloc(h, &h->P[n], (size_t)h->Rmax * h->caps[n] * h->celt));
    TRY(dallocT(h, &h->Psi[n], (size_t)TDB_RCAP * TDB_RCAP));
  }
  TRY(dalloc(h, &h->wsA, (size_t)h->S * h->celt));
  TRY(dalloc(h, &h->wsB, (size_t)h->S * h->celt));
  for (int z = 0; z < 2; ++z) TRY(dalloc(h, &h->wsZ[z], (size_t)h->S * h->celt));
  TRY(dallocT(h, &h->err_part, 2 * (size_t)h->err_blocks));
  TRY(dallocT(h, &h->d_flag, 1));
  TRY(dalloc(h, reinterpret_cast<void**>(&h->ctrl), sizeof(CtrlState)));
  for (int m = 0; m < 2; ++m) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->ctrl_hb[m]), sizeof(CtrlState), hipHostMallocDefault);
    if (e != hipSuccess) { h->err = "hipHostMalloc failed"; return TDB_ENOMEM; }
    // no system-scope fence at the event: the host reads only the pinned mirror after
    // it, which the final error kernel has written and fenced at system scope itself
    HIPCHK(hipEventCreateWithFlags(&h->ev_ctrl[m], hipEventDisableTiming | hipEventDisableSystemFence));
  }
  {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->seq_h), 2 * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) { h->err = "hipHostMalloc failed"; return TDB_ENOMEM; }
    h->seq_h[0] = h->seq_h[1] = 0ull;
  }
  h->ctrl_h = h->ctrl_hb[0];
  {
    const char* env = std::getenv("TDB_PIPELINE");
    // second-order differences read three snapshots and step synchronously
    h->pipelined = cfg->snapshot_mode == TDB_BORROW && cfg->fd_order != 2 && !h->dbo && !(env && env[0] == '0');
  }
  // ---- HOSVD buffers
  size_t gpart = 0;
  for (int n = 0; n < h->p; ++n) {
    TRY(dallocT(h, &h->sig[n], (size_t)h->caps[n] + 1));
    TRY(dallocT(h, &h->Umax[n], (size_t)h->N[n] * h->ldU[n]));
    if (h->tall && n == 0) continue;   // no Gram of the tall mode (see hosvd_select)
    TRY(dallocT(h, &h->G[n], (size_t)h->N[n] * h->N[n]));
    TRY(dallocT(h, &h->eigw[n], (size_t)h->N[n] * (h->caps[n] + 7)));
    TRY(dallocT(h, &h->Bmax[n], (size_t)h->N[n] * h->caps[n]));
    const long long nt = (h->N[n] + 63) / 64;
    const long long K = h->S / h->N[n];
    const long long nch = gram_chunks(K);
    gpart = std::max(gpart, (size_t)(nt * (nt + 1) / 2 * nch * 4096));
  }
  TRY(dallocT(h, &h->gpart, gpart));
  TRY(dallocT(h, &h->Cmax, h->core_cap));
  TRY(dallocT(h, &h->hsA, (size_t)h->S));
  TRY(dallocT(h, &h->hsB, (size_t)h->S));
  TRY(dallocT(h, &h->nu2h, 1));
  TRY(dallocT(h, &h->eig_lam, (size_t)TDB_P * (TDB_RCAP + 2)));
  {
    long long nmax = 1;
    for (int n = 0; n < h->p; ++n) nmax = std::max(nmax, h->N[n]);
    (void)nmax;
    TRY(dallocT(h, &h->eig_vec, (size_t)TDB_P * TDB_NEIG * 64 * 6));
  }
  if (cfg->snapshot_mode == TDB_COPY) TRY(dalloc(h, &h->Vcopy, (size_t)h->S * h->delt));
  if (cfg->fd_order == 2) {
    if (cfg->snapshot_mode == TDB_COPY) TRY(dalloc(h, &h->Vcopy2, (size_t)h->S * h->delt));
    TRY(dalloc(h, &h->Dfd[0], (size_t)h->S * h->delt));
    TRY(dalloc(h, &h->Dfd[1], (size_t)h->S * h->delt));
  }

  // ---- weights and their mode-wise products
  std::vector<std::vector<double>> wh(h->p);
  for (int n = 0; n < h->p; ++n) {
    wh[n].resize(h->N[n]);
    for (long long i = 0; i < h->N[n]; ++i)
      wh[n][i] = cfg->weights[n] ? cfg->weights[n][i] : 1.0 / (double)h->N[n];
    HIPCHK(hipMemcpy(h->w[n], wh[n].data(), h->N[n] * sizeof(double), hipMemcpyHostToDevice));
  }
  for (int n = 0; n < h->p; ++n) {
    std::vector<double> a(1, 1.0), b(1, 1.0);
    for (int k = 0; k < n; ++k) {
      std::vector<double> t(a.size() * h->N[k]);
      for (size_t x = 0; x < a.size(); ++x)
        for (long long i = 0; i < h->N[k]; ++i) t[x * h->N[k] + i] = a[x] * wh[k][i];
      a.swap(t);
    }
    for (int k = n + 1; k < h->p; ++k) {
      std::vector<double> t(b.size() * h->N[k]);
      for (size_t x = 0; x < b.size(); ++x)
        for (long long i = 0; i < h->N[k]; ++i) t[x * h->N[k] + i] = b[x] * wh[k][i];
      b.swap(t);
    }
    TRY(dallocT(h, &h->wa[n], a.size()));
    TRY(dallocT(h, &h->wb[n], b.size()));
    HIPCHK(hipMemcpy(h->wa[n], a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->wb[n], b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // ---- controller state
  CtrlState c;
  std::memset(&c, 0, sizeof(c));
  c.eps_th = cfg->eps_th;
  c.gamma_th = cfg->gamma_th;
  c.dt = cfg->dt;
  c.adaptive = cfg->adaptive ? 1 : 0;
  c.slope_window = h->cfg.slope_window;
  c.p = h->p;
  for (int n = 0; n < TDB_P; ++n) {
    c.caps[n] = n < h->p ? h->caps[n] : 1;
    c.dims[n] = n < h->p ? h->N[n] : 1;
    c.ranks[n] = 1;
  }
  c.eps_trig = cfg->eps_th;
  *h->ctrl_h = c;
  HIPCHK(hipMemcpy(h->ctrl, h->ctrl_h, sizeof(CtrlState), hipMemcpyHostToDevice));
  TRY(setup_fused(h, wh));
  if (h->dbo) {
    const int tr = dbo_rows(dbo_bucket((int)h->N[1]));
    h->dbo_nblk = (int)std::max<long long>(1, std::min<long long>(DBO_GRID, (h->N[0] + tr - 1) / tr));
    TRY(dallocT(h, &h->dbo_wk, (size_t)DBO_WK_SIZE));
    TRY(dalloc(h, &h->dbo_bt, (size_t)2 * DBO_KMAX * DBO_RMAX * h->celt));
    TRY(dallocT(h, &h->dbo_part, (size_t)h->dbo_nblk * dbo_slot_max((int)h->N[1])));
  }
  return TDB_OK;
}

// Grows the stage-pass partial buffer to hold `elems` entries (a quarter more, for the
// ranks that follow), after the device has finished every step that used the old one.
tdb_status ensure_fpart(tdb_ctx* h, long long elems) {
  if (elems <= h->fpart_elems) return TDB_OK;
  if (h->fpart) HIPCHK(hipDeviceSynchronize());
  const long long want = elems + elems / 4;
  void* q = nullptr;
  TRY(dalloc(h, &q, (size_t)want * h->celt));
  if (h->fpart) {
    auto it = std::find(h->allocs.begin(), h->allocs.end(), h->fpart);
    if (it != h->allocs.end()) h->allocs.erase(it);
    HIPCHK(hipFree(h->fpart));
  }
  h->fpart = q;
  h->fpart_elems = want;
  return TDB_OK;
}

tdb_status setup_fused(tdb_ctx* h, const std::vector<std::vector<double>>& wh) {
  h->fused = h->p == 3 && h->cfg.path != TDB_PATH_PLAIN;
  if (!h->fused) return TDB_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int lds = 65536;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
  // dynamic LDS budget: the device limit minus room for the kernels' static LDS
  h->lds_max = lds - 4096;
  // partial buffer: the single-stream plans at ranks 1 and at the caps, with a quarter
  // more for the ranks between; a plan that needs more (other ranks, or the tiles of a
  // batch) grows it when its step is built (ensure_fpart)
  int ones[3] = {1, 1, 1};
  long long need = 1;
  for (const int* rr : {(const int*)ones, (const int*)h->caps}) {
    const PassPlan q = plan_pass(h, rr, false);
    if (q.ok) need = std::max(need, (long long)q.nt1 * q.nt2 * q.slot);
  }
  TRY(ensure_fpart(h, need));
  for (int n = 0; n < 3; ++n) {
    TRY(dallocT(h, &h->Lq[n], (size_t)TDB_RCAP * TDB_RCAP));
    TRY(dallocT(h, &h->qpart[n], (size_t)((h->N[n] + QR_ROWS - 1) / QR_ROWS) * h->caps[n] * h->caps[n]));
    TRY(dalloc(h, &h->P2[n], (size_t)h->Rmax * h->caps[n] * h->celt));
  }
  TRY(dallocT(h, &h->Cdot2, h->core_cap));
  for (int n = 0; n < 3; ++n) TRY(dallocT(h, &h->Mbuf[n], (size_t)TDB_RCAP * TDB_RCAP));
  for (int n = 0; n < 3; ++n) TRY(dallocT(h, &h->Gsave[n], (size_t)TDB_RCAP * TDB_RCAP));
  TRY(dallocT(h, &h->T3buf, (size_t)h->caps[0] * h->caps[1] * h->N[2]));
  TRY(dalloc(h, &h->E, (size_t)h->caps[0] * h->N[1] * h->N[2] * h->celt));
  TRY(dalloc(h, &h->U1c, (size_t)h->N[0] * h->caps[0] * h->celt));
  std::vector<double> w23((size_t)(h->N[1] * h->N[2]));
  for (long long i = 0; i < h->N[1]; ++i)
    for (long long j = 0; j < h->N[2]; ++j) w23[i * h->N[2] + j] = wh[1][i] * wh[2][j];
  TRY(dallocT(h, &h->w23, w23.size()));
  HIPCHK(hipMemcpy(h->w23, w23.data(), w23.size() * sizeof(double), hipMemcpyHostToDevice));
  const long long M = h->N[1] * h->N[2];
  h->ferr_gx = (int)std::max<long long>(1, std::min<long long>(64, (M + 255) / 256));
  h->ferr_gy = (int)((h->N[0] + FERR_T1 - 1) / FERR_T1);
  // partials of the slab error pass or of the column-block one (batches)
  TRY(dallocT(h, &h->ferr_part, 2 * std::max<size_t>((size_t)h->ferr_gx * h->ferr_gy, (size_t)((M + FEC_COLS - 1) / FEC_COLS))));
  TRY(dalloc(h, reinterpret_cast<void**>(&h->counters), 8 * sizeof(unsigned)));
  HIPCHK(hipMemset(h->counters, 0, 8 * sizeof(unsigned)));
  return TDB_OK;
}

// ---------------------------------------------------------------- sequencing helpers
template <typename T>
tdb_status stage_prep(tdb_ctx* h, const double* C, double* const* U, hipStream_t s) {
  StageArgs a{};
  a.p = h->p;
  a.C = C;
  for (int n = 0; n < h->p; ++n) {
    a.r[n] = h->r[n];
    a.N[n] = h->N[n];
    a.ldU[n] = h->ldU[n];
    a.U[n] = U[n];
    a.w[n] = h->w[n];
    a.B[n] = h->B[n];
    a.P[n] = h->P[n];
  }
  HIPCHK(launch_stage_prep<T>(a, h->ctrl, s));
  return TDB_OK;
}

// Plain projection pass: for every mode a chain of n-mode products of the data
// difference with W_k U_k over all other modes (eq. (basecont)), folded with the
// core pseudo-inverse into H_n; the core derivative (eq. (Corecont)) from F_1.
template <typename TD, typename T>
tdb_status project_plain(tdb_ctx* h, const TD* V1, const TD* V0, hipStream_t s) {
  const int p = h->p;
  // the two modes that reduce the data most (largest N/r), contracted first: every F_n
  // with n != a continues from D x_a B_a^T, F_a from D x_b B_b^T, so the snapshot pair is
  // read twice per stage instead of p times
  std::vector<int> ord(p);
  for (int k = 0; k < p; ++k) ord[k] = k;
  auto by_ratio = [&](int x, int y) {
    const double rx = (double)h->N[x] / h->r[x], ry = (double)h->N[y] / h->r[y];
    return rx != ry ? rx > ry : x < y;
  };
  std::sort(ord.begin(), ord.end(), by_ratio);
  const int first[2] = {ord[0], ord[1]};
  T* Z[2] = {static_cast<T*>(h->wsZ[0]), static_cast<T*>(h->wsZ[1])};
  for (int z = 0; z < 2; ++z) {
    const int k = first[z];
    long long A = 1, Bz = 1;
    for (int j = 0; j < k; ++j) A *= h->N[j];
    for (int j = k + 1; j < p; ++j) Bz *= h->N[j];
    HIPCHK((launch_ttm<TD, T, T>(V1, V0, Z[z], static_cast<const T*>(h->B[k]), h->r[k], 1, A, (int)h->N[k],
                                 h->r[k], Bz, s)));
  }
  T* bufs[2] = {static_cast<T*>(h->wsA), static_cast<T*>(h->wsB)};
  for (int n = 0; n < p; ++n) {
    const int zi = n == first[0] ? 1 : 0;
    const int done = first[zi];
    long long cd[TDB_P];
    for (int k = 0; k < p; ++k) cd[k] = h->N[k];
    cd[done] = h->r[done];
    std::vector<int> order;
    for (int k : ord)
      if (k != n && k != done) order.push_back(k);
    const T* cur = Z[zi];
    int next = 0;
    for (int k : order) {
      long long A = 1, Bz = 1;
      for (int j = 0; j < k; ++j) A *= cd[j];
      for (int j = k + 1; j < p; ++j) Bz *= cd[j];
      T* out = bufs[next];
      HIPCHK((launch_ttm<T, T, T>(cur, nullptr, out, static_cast<const T*>(h->B[k]), h->r[k], 1, A, (int)cd[k],
                                  h->r[k], Bz, s)));
      cd[k] = h->r[k];
      cur = out;
      next = 1 - next;
    }
    const T* F = cur;
    long long outer = 1, inner = 1;
    for (int k = 0; k < n; ++k) outer *= h->r[k];
    for (int k = n + 1; k < p; ++k) inner *= h->r[k];
    if (h->r[n] < h->N[n])
      HIPCHK(launch_fold_h<T>(F, static_cast<const T*>(h->P[n]), h->H[n], h->N[n], h->r[n], outer, inner, s));
    if (n == 0)
      HIPCHK((launch_ttm<T, T, double>(F, nullptr, h->Cdot, static_cast<const T*>(h->B[0]), h->r[0], 1, 1,
                                       (int)h->N[0], h->r[0], inner, s)));
  }
  return TDB_OK;
}

// Reconstruction C x_1 U_1 ... x_p U_p into one of the work buffers; returns it.
template <typename T>
tdb_status reconstruct_plain(tdb_ctx* h, T** result, hipStream_t s) {
  const int p = h->p;
  for (int n = 0; n < p; ++n)
    HIPCHK((launch_convert<double, T>(h->U0[n], static_cast<T*>(h->Uc[n]), h->N[n] * h->ldU[n], s)));
  HIPCHK((launch_convert<double, T>(h->C0, static_cast<T*>(h->Cc), prod_ll(h->r, p), s)));
  std::vector<int> order(p);
  for (int k = 0; k < p; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    const double rx = (double)h->N[x] / h->r[x], ry = (double)h->N[y] / h->r[y];
    return rx != ry ? rx < ry : x < y;
  });
  long long cd[TDB_P];
  for (int k = 0; k < p; ++k) cd[k] = h->r[k];
  T* bufs[2] = {static_cast<T*>(h->wsA), static_cast<T*>(h->wsB)};
  const T* in = static_cast<const T*>(h->Cc);
  int cur = -1;
  for (int q = 0; q < p; ++q) {
    const int k = order[q];
    long long A = 1, Bz = 1;
    for (int j = 0; j < k; ++j) A *= cd[j];
    for (int j = k + 1; j < p; ++j) Bz *= cd[j];
    T* out = bufs[cur == 0 ? 1 : 0];
    HIPCHK((launch_ttm<T, T, T>(in, nullptr, out, static_cast<const T*>(h->Uc[k]), 1, h->ldU[k], A,
                                (int)cd[k], (int)h->N[k], Bz, s)));
    cd[k] = h->N[k];
    cur = (cur == 0) ? 1 : 0;
    in = out;
  }
  *result = bufs[cur];
  return TDB_OK;
}

template <typename TD, typename T>
tdb_status error_pass_plain(tdb_ctx* h, const TD* V, hipStream_t s) {
  T* R = nullptr;
  TRY((reconstruct_plain<T>(h, &R, s)));
  const double* wp[TDB_P] = {};
  for (int n = 0; n < h->p; ++n) wp[n] = h->w[n];
  HIPCHK((launch_err_partials<TD, T>(V, R, h->p, h->N, wp, h->err_part, h->err_blocks, s)));
  HIPCHK(launch_err_final(h->err_part, h->err_blocks, h->ctrl, s));
  return TDB_OK;
}

tdb_status core_sigma(tdb_ctx* h, bool with_vectors, hipStream_t s) {
  SigmaArgs a{};
  a.p = h->p;
  a.C = h->C0;
  for (int n = 0; n < h->p; ++n) {
    a.r[n] = h->r[n];
    a.Psi[n] = with_vectors ? h->Psi[n] : nullptr;
  }
  HIPCHK(launch_core_sigma(a, h->ctrl, s));
  return TDB_OK;
}

DboArgs dbo_args(tdb_ctx* h) {
  DboArgs a{};
  a.M = h->N[0];
  a.K = (int)h->N[1];
  a.r = h->r[0];
  a.ldU1 = h->ldU[0];
  a.ldU2 = h->ldU[1];
  a.full2 = h->r[1] >= h->N[1] ? 1 : 0;
  a.euler = h->cfg.integrator == TDB_INT_EULER ? 1 : 0;
  a.TR = dbo_rows(dbo_bucket(a.K));
  a.nblk = h->dbo_nblk;
  a.caps = h->caps[0];
  a.dt = h->cfg.dt;
  a.dscale = 1.0 / h->cfg.dt;
  a.U1 = h->U0[0];
  a.kU1 = h->kU[0];
  a.w1 = h->w[0];
  a.w2 = h->w[1];
  a.part = h->dbo_part;
  a.wk = h->dbo_wk;
  a.Bt = h->dbo_bt;
  a.C0 = h->C0;
  a.U2 = h->U0[1];
  a.kU2 = h->kU[1];
  a.Us2 = h->Us[1];
  a.Cs = h->Cs;
  a.kC = h->kC;
  return a;
}

// HOSVD of an order-2 stream whose first mode is tall: the second mode's weighted Gram
// and eigenvectors Umax2 give the first mode's basis as the left singular vectors of
// the weighted unfolding, Umax1 = V (W2 Umax2) Sigma^-1, each column sign-fixed like
// an eigenvector (largest entry of W1^(1/2) Umax1 positive, lowest row on a tie); the
// core at the caps is diag(sign * sigma) (Sec. 2.3).
template <typename TD>
tdb_status hosvd_tall(tdb_ctx* h, const TD* V, int mode, hipStream_t s) {
  HIPCHK(hipMemsetAsync(&h->ctrl->hold, 0, sizeof(int), s));
  HosvdModeArgs m{};
  m.n = 1;
  m.A = h->N[0];
  m.Bsz = 1;
  m.Nn = h->N[1];
  m.wa = h->wa[1];
  m.wb = h->wb[1];
  m.wn = h->w[1];
  const long long K = m.A;
  const int nch = (int)gram_chunks(K);
  long long kchunk = (K + nch - 1) / nch;
  kchunk = (kchunk + 15) / 16 * 16;
  HIPCHK(launch_gram_partials<TD>(V, m, h->gpart, kchunk, nch, s));
  HIPCHK(launch_gram_reduce(h->gpart, h->G[1], m, nch, s));
  EigBatch eb{};
  eb.count = 1;
  EigArgs& e = eb.m[0];
  e.Nn = (int)h->N[1];
  e.k = h->caps[1];
  e.ldu = h->ldU[1];
  e.G = h->G[1];
  e.work = h->eigw[1];
  e.sig = h->sig[1];
  e.Umax = h->Umax[1];
  e.Bmax = h->Bmax[1];
  e.wn = h->w[1];
  HIPCHK(launch_trace(h->G[1], h->N[1], h->nu2h, s));
  HIPCHK(launch_sym_eig(eb, h->eig_lam, h->eig_vec, s));
  DboArgs a = dbo_args(h);
  a.V1 = V;
  a.r = 1;
  a.Umax1 = h->Umax[0];
  a.sig2 = h->sig[1];
  a.Bmax2 = h->Bmax[1];
  a.sig1 = h->sig[0];
  a.Cmax = h->Cmax;
  HIPCHK((launch_dbo_rows<TD, double>(a, DBO_MAP, h->ctrl, s)));
  HIPCHK(launch_dbo_small<double>(a, DBO_SIGN, h->ctrl, s));
  HIPCHK((launch_dbo_rows<TD, double>(a, DBO_FLIP, h->ctrl, s)));
  SelectArgs sa{};
  sa.p = 2;
  sa.mode = mode;
  sa.Cmax = h->Cmax;
  sa.nu2h = h->nu2h;
  sa.C0 = h->C0;
  for (int n = 0; n < 2; ++n) {
    sa.caps[n] = h->caps[n];
    sa.N[n] = h->N[n];
    sa.ldU[n] = h->ldU[n];
    sa.rank_init[n] = h->cfg.rank_init[n];
    sa.sig[n] = h->sig[n];
    sa.Umax[n] = h->Umax[n];
    sa.U0[n] = h->U0[n];
  }
  HIPCHK(launch_rank_select(sa, h->ctrl, s));
  return TDB_OK;
}

// Weighted HOSVD of V at the caps (Sec. 2.3) followed by the rank selection `mode`.
template <typename TD>
tdb_status hosvd_select(tdb_ctx* h, const TD* V, int mode, hipStream_t s) {
  if (h->tall) return hosvd_tall<TD>(h, V, mode, s);
  const int p = h->p;
  // the decision is being acted on: release the steps held behind it
  HIPCHK(hipMemsetAsync(&h->ctrl->hold, 0, sizeof(int), s));
  EigBatch eb{};
  eb.count = p;
  for (int n = 0; n < p; ++n) {
    HosvdModeArgs m{};
    m.n = n;
    m.A = 1;
    m.Bsz = 1;
    for (int k = 0; k < n; ++k) m.A *= h->N[k];
    for (int k = n + 1; k < p; ++k) m.Bsz *= h->N[k];
    m.Nn = h->N[n];
    m.wa = h->wa[n];
    m.wb = h->wb[n];
    m.wn = h->w[n];
    const long long K = m.A * m.Bsz;
    const int nch = (int)gram_chunks(K);
    long long kchunk = (K + nch - 1) / nch;
    kchunk = (kchunk + 15) / 16 * 16;
    HIPCHK(launch_gram_partials<TD>(V, m, h->gpart, kchunk, nch, s));
    HIPCHK(launch_gram_reduce(h->gpart, h->G[n], m, nch, s));
    EigArgs& e = eb.m[n];
    e.Nn = (int)h->N[n];
    e.k = h->caps[n];
    e.ldu = h->ldU[n];
    e.G = h->G[n];
    e.work = h->eigw[n];
    e.sig = h->sig[n];
    e.Umax = h->Umax[n];
    e.Bmax = h->Bmax[n];
    e.wn = h->w[n];
  }
  HIPCHK(launch_trace(h->G[0], h->N[0], h->nu2h, s));
  HIPCHK(launch_sym_eig(eb, h->eig_lam, h->eig_vec, s));
  // Cmax = V x_n (W_n Umax_n)^T over all modes, most reducing mode first
  std::vector<int> order(p);
  for (int k = 0; k < p; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    const double rx = (double)h->N[x] / h->caps[x], ry = (double)h->N[y] / h->caps[y];
    return rx != ry ? rx > ry : x < y;
  });
  long long cd[TDB_P];
  for (int k = 0; k < p; ++k) cd[k] = h->N[k];
  double* bufs[2] = {h->hsA, h->hsB};
  int cur = -1;
  for (int q = 0; q < p; ++q) {
    const int k = order[q];
    long long A = 1, Bz = 1;
    for (int j = 0; j < k; ++j) A *= cd[j];
    for (int j = k + 1; j < p; ++j) Bz *= cd[j];
    double* out = (q == p - 1) ? h->Cmax : bufs[cur == 0 ? 1 : 0];
    if (q == 0)
      HIPCHK((launch_ttm<TD, double, double>(V, nullptr, out, h->Bmax[k], h->caps[k], 1, A, (int)cd[k],
                                             h->caps[k], Bz, s)));
    else
      HIPCHK((launch_ttm<double, double, double>(bufs[cur], nullptr, out, h->Bmax[k], h->caps[k], 1, A,
                                                 (int)cd[k], h->caps[k], Bz, s)));
    cd[k] = h->caps[k];
    cur = (cur == 0) ? 1 : 0;
  }
  SelectArgs sa{};
  sa.p = p;
  sa.mode = mode;
  sa.Cmax = h->Cmax;
  sa.nu2h = h->nu2h;
  sa.C0 = h->C0;
  for (int n = 0; n < p; ++n) {
    sa.caps[n] = h->caps[n];
    sa.N[n] = h->N[n];
    sa.ldU[n] = h->ldU[n];
    sa.rank_init[n] = h->cfg.rank_init[n];
    sa.sig[n] = h->sig[n];
    sa.Umax[n] = h->Umax[n];
    sa.U0[n] = h->U0[n];
  }
  HIPCHK(launch_rank_select(sa, h->ctrl, s));
  return TDB_OK;
}

tdb_status pull_ctrl(tdb_ctx* h, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(h->ctrl_h, h->ctrl, sizeof(CtrlState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int n = 0; n < h->p; ++n) h->r[n] = h->ctrl_h->ranks[n];
  return TDB_OK;
}

double compression_ratio(const tdb_ctx* h) {
  double num = 1.0, den = 0.0, core = 1.0;
  for (int n = 0; n < h->p; ++n) {
    num *= (double)h->N[n];
    den += (double)h->r[n] * (double)h->N[n];
    core *= h->r[n];
  }
  return num / (den + core);
}

// batch members: their batch's newest step is read first; graph replay count
tdb_status batch_resolve(tdb_batch_ctx* b);
long long batch_graph_steps(const tdb_batch_ctx* b);

void fill_stats(tdb_ctx* h, bool initial) {
  const CtrlState& c = *h->ctrl_h;
  tdb_stats& st = h->stats;
  st.step = h->step;
  st.t = h->t_now;
  st.eps = c.eps;
  st.nu = c.nu;
  st.eps_after = initial ? NAN : c.eps_after;
  for (int n = 0; n < TDB_MAX_ORDER; ++n) st.ranks[n] = n < h->p ? h->r[n] : 0;
  st.event = initial ? 0 : c.event;
  for (int n = 0; n < 4; ++n)
    for (int i = 0; i < TDB_SIGMA_K; ++i)
      st.sigma[n][i] = (n < h->p && i < h->r[n]) ? c.sigma[n][i] : 0.0;
  st.cr = compression_ratio(h);
  if (!initial) h->crbar_den += h->cfg.dt / st.cr;
  st.crbar = (h->step > 0 && h->crbar_den > 0.0) ? (h->step * h->cfg.dt) / h->crbar_den : st.cr;
  st.n_reinit = c.n_events[EV_REINIT];
  st.n_add = c.n_events[EV_ADD];
  st.n_remove = c.n_events[EV_REMOVE];
  st.n_numeric = c.n_events[EV_NUMERIC];
  st.gated = initial ? 0 : c.gated;
  st.would_skip = initial ? 0 : c.would_skip;
  st.eps_pred = initial ? NAN : c.eps_pred;
  st.precision_used = h->last_prec;
  st.path_used = h->last_path;
  st.fused_steps = h->fused_steps;
  st.plain_steps = h->plain_steps;
  st.n_nonfinite = h->n_nonfinite;
  st.graph_steps = h->owner ? batch_graph_steps(h->owner) : 0;
}

hipEvent_t take_event(tdb_ctx* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Times a pass with a pair of events when profiling is on. By default the events
// bracket the pass on the stream; with by_dispatch the launcher hands them to the
// kernel dispatch itself (start and end of that one kernel), which leaves out any
// time the queue waits for the host to submit it.
struct PassTimer {
  tdb_ctx* h;
  int pass;
  hipStream_t s;
  bool by_dispatch;
  hipEvent_t a = nullptr, b = nullptr;
  PassTimer(tdb_ctx* h_, int pass_, hipStream_t s_, bool by_dispatch_ = false)
      : h(h_), pass(pass_), s(s_), by_dispatch(by_dispatch_) {
    if (!h->prof || !h->prof_now) return;
    a = take_event(h);
    b = take_event(h);
    if (a && b && !by_dispatch) (void)hipEventRecord(a, s);
  }
  hipEvent_t start() const { return a && b ? a : nullptr; }
  hipEvent_t stop() const { return a && b ? b : nullptr; }
  ~PassTimer() {
    if (!a || !b) return;
    if (!by_dispatch) (void)hipEventRecord(b, s);
    h->ev_used[pass].push_back({a, b});
  }
};

// V becomes the previous snapshot; with second-order differences the previous one
// becomes the one before (TDB_COPY alternates between two copy buffers).
template <typename TD>
tdb_status keep_previous(tdb_ctx* h, const TD* V, hipStream_t s) {
  const bool two = h->cfg.fd_order == 2;
  if (two) h->Vprev2 = h->Vprev;
  if (h->cfg.snapshot_mode == TDB_COPY) {
    void* dst = two && h->Vprev == h->Vcopy ? h->Vcopy2 : h->Vcopy;
    HIPCHK(hipMemcpyAsync(dst, V, (size_t)h->S * sizeof(TD), hipMemcpyDeviceToDevice, s));
    h->Vprev = dst;
  } else {
    h->Vprev = V;
  }
  return TDB_OK;
}

// *bad = whether any of the S values at x is NaN or infinite (synchronises s).
template <typename TD>
tdb_status has_nonfinite(tdb_ctx* h, const TD* x, hipStream_t s, bool* bad) {
  HIPCHK(launch_nonfinite_check<TD>(x, h->S, h->d_flag, s));
  int v = 0;
  HIPCHK(hipMemcpyAsync(&v, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *bad = v != 0;
  return TDB_OK;
}

tdb_status has_nonfinite_any(tdb_ctx* h, const void* x, hipStream_t s, bool* bad) {
  if (h->data32) return has_nonfinite<float>(h, static_cast<const float*>(x), s, bad);
  return has_nonfinite<double>(h, static_cast<const double*>(x), s, bad);
}

// A step whose data derivative held NaN or Inf was not applied on the device (the
// first stage's core derivative raised the flag, the later kernels kept the state):
// the snapshot still becomes the previous one, nothing else of the stream changes.
template <typename TD>
tdb_status discard_step(tdb_ctx* h, const TD* V1, hipStream_t s) {
  TRY(keep_previous<TD>(h, V1, s));
  h->n_nonfinite += 1;
  h->err = "non-finite values (NaN or Inf) in the data derivative: the step was not applied (core, bases and "
           "statistics are those of the last finite step)";
  return TDB_ENUMERIC;
}

tdb_status euler_commit(tdb_ctx* h, hipStream_t s);

// D (may be NULL): a given data derivative in place of (V1 - V_prev)/dt; D2 (may be
// NULL): the second stage's derivative when it differs from D.
template <typename TD, typename T>
tdb_status ingest_impl(tdb_ctx* h, const TD* V1, hipStream_t s, const TD* D = nullptr, const TD* D2 = nullptr) {
  h->prof_now = h->prof_every <= 1 || h->prof_steps++ % h->prof_every == 0;
  // the projected operand: V1 - V_prev (scaled by 1/dt), or D itself
  const TD* Vp = D ? D : V1;
  const TD* V0 = D ? nullptr : static_cast<const TD*>(h->Vprev);
  const int p = h->p;
  RhsArgs ra{};
  ra.p = p;
  ra.dt = h->cfg.dt;
  ra.dscale = D ? 1.0 : 1.0 / h->cfg.dt;
  ra.core_size = prod_ll(h->r, p);
  ra.Cdot = h->Cdot;
  ra.C0 = h->C0;
  ra.Cs = h->Cs;
  ra.kC = h->kC;
  for (int n = 0; n < p; ++n) {
    ra.r[n] = h->r[n];
    ra.N[n] = h->N[n];
    ra.ldU[n] = h->ldU[n];
    ra.H[n] = h->H[n];
    ra.w[n] = h->w[n];
    ra.U0[n] = h->U0[n];
    ra.Us[n] = h->Us[n];
    ra.kU[n] = h->kU[n];
  }
  // stage 1 at S_k
  TRY(stage_prep<T>(h, h->C0, h->U0, s));
  {
    PassTimer pt(h, TDB_PASS_PROJECT, s);
    TRY((project_plain<TD, T>(h, Vp, V0, s)));
  }
  ra.stage = 1;
  HIPCHK(launch_rhs_stage(ra, h->ctrl, s));
  if (h->cfg.integrator == TDB_INT_EULER) {
    TRY(euler_commit(h, s));
  } else {
    // stage 2 at S*
    TRY(stage_prep<T>(h, h->Cs, h->Us, s));
    {
      PassTimer pt(h, TDB_PASS_PROJECT, s);
      TRY((project_plain<TD, T>(h, D2 ? D2 : Vp, V0, s)));
    }
    ra.stage = 2;
    HIPCHK(launch_rhs_stage(ra, h->ctrl, s));
  }
  QrArgs qa{};
  qa.p = p;
  qa.C0 = h->C0;
  qa.Ctmp = h->Ctmp;
  for (int n = 0; n < p; ++n) {
    qa.r[n] = h->r[n];
    qa.N[n] = h->N[n];
    qa.ldU[n] = h->ldU[n];
    qa.U0[n] = h->U0[n];
    qa.w[n] = h->w[n];
  }
  HIPCHK(launch_qr_fold(qa, h->ctrl, s));
  TRY(core_sigma(h, false, s));
  {
    PassTimer pt(h, TDB_PASS_ERROR, s);
    TRY((error_pass_plain<TD, T>(h, V1, s)));
  }
  HIPCHK(launch_controller(h->ctrl, s));
  TRY(pull_ctrl(h, s));
  h->last_path = TDB_PATH_PLAIN;
  h->last_prec = h->f32 ? TDB_PREC_F32 : TDB_PREC_F64;
  h->plain_steps += 1;
  const int dec = h->ctrl_h->decision;
  if (dec == DEC_NONFINITE) return discard_step<TD>(h, V1, s);
  h->step += 1;
  h->t_now = h->step * h->cfg.dt;
  if (dec != DEC_NONE) {
    TRY(hosvd_select<TD>(h, V1, dec, s));
    TRY(pull_ctrl(h, s));
    TRY(core_sigma(h, false, s));
    TRY(pull_ctrl(h, s));
  }
  TRY(keep_previous<TD>(h, V1, s));
  // the host copy holds this step's singular values only after a reinit (pulled in
  // full) or when a single stream formed them and pulled the controller state
  h->sigma_stale = !(dec != DEC_NONE || (h->sigma_every_step && !h->batch_owned));
  fill_stats(h, false);
  return TDB_OK;
}

// One step of an order-2 stream on the row passes (Sec. 2.2 with p = 2; Heun or
// Euler, Sec. 2.4): stage preparation, the stage-1 sums, the stage-1 finish fused with
// the stage-2 sums, the stage-2 finish with the new basis' Gram and the error sums,
// the small kernels between them, and U1 <- U1 L^-T of the Cholesky QR. D, D2: given
// stage derivatives (or NULL for the difference of snapshots).
template <typename TD, typename T>
tdb_status ingest_dbo(tdb_ctx* h, const TD* V1, hipStream_t s, const TD* D = nullptr, const TD* D2 = nullptr) {
  h->prof_now = h->prof_every <= 1 || h->prof_steps++ % h->prof_every == 0;
  DboArgs a = dbo_args(h);
  a.V1 = V1;
  a.V0 = D ? nullptr : h->Vprev;
  a.D1 = D;
  a.D2 = D ? D2 : nullptr;
  a.dscale = D ? 1.0 : 1.0 / h->cfg.dt;
  CtrlState* c = h->ctrl;
  // the previous step's last kernel prepared this one's first stage, unless the host
  // has replaced the state since
  if (!h->dbo_prep) HIPCHK(launch_dbo_small<T>(a, DBO_PREP, c, s));
  h->dbo_prep = true;
  {
    PassTimer pt(h, TDB_PASS_PROJECT, s);
    HIPCHK((launch_dbo_rows<TD, T>(a, DBO_PASS1, c, s)));
  }
  HIPCHK(launch_dbo_small<T>(a, DBO_MID1, c, s));
  if (a.euler) {
    PassTimer pt(h, TDB_PASS_ERROR, s);
    HIPCHK((launch_dbo_rows<TD, T>(a, DBO_FINE, c, s)));
  } else {
    {
      PassTimer pt(h, TDB_PASS_PROJECT, s);
      HIPCHK((launch_dbo_rows<TD, T>(a, DBO_FIN1, c, s)));
    }
    HIPCHK(launch_dbo_small<T>(a, DBO_MID2, c, s));
    PassTimer pt(h, TDB_PASS_ERROR, s);
    HIPCHK((launch_dbo_rows<TD, T>(a, DBO_FIN2, c, s)));
  }
  HIPCHK(launch_dbo_small<T>(a, DBO_END, c, s));
  HIPCHK((launch_dbo_rows<TD, T>(a, DBO_NORM, c, s)));
  TRY(core_sigma(h, false, s));
  HIPCHK(launch_controller(c, s));
  TRY(pull_ctrl(h, s));
  h->last_path = TDB_PATH_FUSED;
  h->last_prec = h->f32 ? TDB_PREC_F32 : TDB_PREC_F64;
  h->fused_steps += 1;
  const int dec = h->ctrl_h->decision;
  if (dec == DEC_NONFINITE) return discard_step<TD>(h, V1, s);
  h->step += 1;
  h->t_now = h->step * h->cfg.dt;
  if (dec != DEC_NONE) {
    h->dbo_prep = false;
    TRY(hosvd_select<TD>(h, V1, dec, s));
    TRY(pull_ctrl(h, s));
    TRY(core_sigma(h, false, s));
    TRY(pull_ctrl(h, s));
  }
  TRY(keep_previous<TD>(h, V1, s));
  h->sigma_stale = !(dec != DEC_NONE || h->sigma_every_step);
  fill_stats(h, false);
  return TDB_OK;
}

int max_rank_of(const int* r, int p) {
  int m = 1;
  for (int n = 0; n < p; ++n) m = std::max(m, r[n]);
  return m;
}

// Where the QR folds a core of csz entries, given the LDS of its factors (fold) and
// the LDS available: 2 in place through registers, 1 in two LDS buffers, 0 in global
// memory.
int qr_core_mode(long long csz, size_t fold, size_t budget) {
  const size_t cneed = (size_t)csz * 8;
  if (csz <= (long long)FOLD_R * 256 && fold + cneed <= budget) return 2;
  if (fold + 2 * cneed <= budget) return 1;
  return 0;
}

// LDS of the post-step expansion blocks for ranks rl with eb blocks: T3, and either
// the three L_n^-1 with every row of the block before and after the normalisation
// (*all = true, when that fits) or one L_n^-1 and a chunk of rows.
size_t post_exp_lds(const tdb_ctx* h, const int* rl, int eb, bool* all) {
  const size_t rq = (size_t)max_rank_of(rl, 3);
  const size_t t3 = (size_t)rl[0] * rl[1] * (size_t)h->N[2];
  size_t rows = 0, ll = 0;
  for (int m = 0; m < 3; ++m) {
    rows += (size_t)((h->N[m] + eb - 1) / eb) * rl[m];
    ll += (size_t)rl[m] * rl[m];
  }
  const size_t staged = (t3 + ll + 2 * rows) * 8;
  *all = staged <= (size_t)h->lds_max;
  return *all ? staged : (t3 + rq * rq + 2 * (size_t)POST_CH * rq) * 8;
}

// LDS of the small per-mode kernels (finish, post) when sized for ranks rl.
size_t small_lds(const tdb_ctx* h, const int* rl, bool* core_in_lds, bool m_inline = false) {
  const long long csz = prod_ll(rl, h->p);
  const int rm = max_rank_of(rl, h->p);
  long long msum = 0;
  for (int n = 0; n < h->p; ++n) msum += (long long)rl[n] * rl[n];
  // finish rows stage the three M_n (and, forming them inline, C_dot and the three P_n)
  // and a tile of FIN_EPT * 256 row elements with rm - 1 on either side
  const size_t rows = (size_t)msum * 8 + (m_inline ? (size_t)csz * 8 + 3 * (size_t)csz * h->celt + 8 + FIN_PART * 8 : 0) +
                      (FIN_EPT * 256 + 2 * (size_t)rm) * 8;
  const size_t base = std::max<size_t>((3 * (size_t)rm * rm + 5 * (size_t)rm + 64 + FQR_GP) * 8, rows);
  *core_in_lds = base + (size_t)csz * 8 <= (size_t)h->lds_max;
  return base + (*core_in_lds ? (size_t)csz * 8 : 0);
}

// Everything one fused step launches, for the current ranks h->r. LDS budgets, tile
// shapes and grid sizes are taken for the ranks `rl` (h->r for a single stream; the
// caps for a batch, so that a batch's launch shapes never change).
struct StepArgs {
  PassPlan pl;
  FPassArgs fa[2];
  FReduceArgs ra;
  FFinishArgs ga[2];
  FQrArgs qa;
  FPostArgs pa;
  FErrArgs ea;
  size_t lds_fin = 0, lds_qr = 0, lds_post = 0, lds_mprep = 0;
  int blocks_pass = 1, blocks_red = 1, blocks_fin[2] = {1, 1}, blocks_qr = 3, blocks_post = 1, blocks_err = 1;
};

tdb_status build_post_args(tdb_ctx* h, const int* rl, FPostArgs& pa, size_t& lds) {
  pa = FPostArgs{};
  bool cil = false;
  lds = small_lds(h, rl, &cil);
  pa.core_in_lds = cil ? 1 : 0;
  pa.want_pinv = 1;
  pa.rmax = max_rank_of(rl, 3);
  const long long etot = (long long)rl[0] * h->N[1] * h->N[2];
  // a batch gives each expansion block four times the work (fewer blocks, each of which
  // stages T3 and the factors once)
  const long long eper = rl != h->r ? 2048 : 256;
  pa.eblocks = (int)std::max<long long>(1, std::min<long long>(std::min<long long>(256, h->N[1]), (etot + eper - 1) / eper));
  bool sall = false;
  const size_t elds = post_exp_lds(h, rl, pa.eblocks, &sall);
  pa.stage_all = sall ? 1 : 0;
  if (elds > (size_t)h->lds_max) { h->err = "error-pass expansion does not fit in LDS"; return TDB_EUNSUPPORTED; }
  lds = std::max(lds, elds);
  pa.C = h->C0;
  pa.E = h->E;
  pa.U1c = h->U1c;
  pa.T3 = nullptr;
  pa.want_sigma = 1;
  for (int n = 0; n < 3; ++n) pa.G[n] = h->Gsave[n];
  for (int n = 0; n < 3; ++n) {
    pa.N[n] = h->N[n];
    pa.r[n] = h->r[n];
    pa.ldU[n] = h->ldU[n];
    pa.U[n] = h->U0[n];
    pa.Uw[n] = h->U0[n];
    pa.w[n] = h->w[n];
    pa.B[n] = h->B[n];
    pa.P[n] = h->P[n];
  }
  return TDB_OK;
}

// Returns TDB_EUNSUPPORTED when the stage pass does not fit (the caller may fall back
// to the plain path).
// D (may be NULL): a given data derivative, projected in place of (V1 - V0)/dt; D2
// (may be NULL, only with D): the second stage's derivative.
tdb_status build_step_args(tdb_ctx* h, const int* rl, const void* V1, const void* V0, StepArgs& A,
                           const void* D = nullptr, const void* D2 = nullptr) {
  const PassPlan base = plan_pass(h, rl, rl != h->r);
  if (!base.ok) { h->err = "stage-pass tile does not fit in LDS"; return TDB_EUNSUPPORTED; }
  const PassPlan pl = rl == h->r ? base : plan_under(h, h->r, base);
  if (!pl.ok) {
    h->err = "stage-pass partials do not fit";
    return TDB_EUNSUPPORTED;
  }
  TRY(ensure_fpart(h, (long long)pl.nt1 * pl.nt2 * pl.slot));
  A.pl = pl;
  A.blocks_pass = pl.nt1 * pl.nt2;
  FPassArgs fa{};
  fa.V1 = D ? D : V1;
  fa.V0 = D ? nullptr : V0;
  const double dscale = D ? 1.0 : 1.0 / h->cfg.dt;
  fa.N1 = (int)h->N[0]; fa.N2 = (int)h->N[1]; fa.N3 = (int)h->N[2];
  fa.r1 = h->r[0]; fa.r2 = h->r[1]; fa.r3 = h->r[2];
  fa.T1 = pl.T1; fa.T2 = pl.T2; fa.nt1 = pl.nt1; fa.nt2 = pl.nt2;
  fa.need_h1 = h->r[0] < h->N[0];
  fa.need_h2 = h->r[1] < h->N[1];
  fa.need_f3 = h->r[2] < h->N[2];
  fa.stage_p = pl.stage_p;
  fa.slot = pl.slot;
  fa.B1 = h->B[0]; fa.B2 = h->B[1]; fa.B3 = h->B[2];
  fa.part = h->fpart;
  fa.hold = &h->ctrl->hold;
  A.fa[0] = fa;
  A.fa[0].P1 = h->P[0]; A.fa[0].P2 = h->P[1]; A.fa[0].P3 = h->P[2];
  A.fa[1] = fa;
  A.fa[1].P1 = h->P2[0]; A.fa[1].P2 = h->P2[1]; A.fa[1].P3 = h->P2[2];
  if (D && D2) A.fa[1].V1 = D2;

  FReduceArgs& ra = A.ra;
  ra = FReduceArgs{};
  ra.dt = h->cfg.dt;
  ra.dscale = dscale;
  ra.N1 = fa.N1; ra.N2 = fa.N2; ra.N3 = fa.N3; ra.r1 = fa.r1; ra.r2 = fa.r2; ra.r3 = fa.r3;
  ra.T1 = pl.T1; ra.T2 = pl.T2; ra.nt1 = pl.nt1; ra.nt2 = pl.nt2;
  ra.need_h1 = fa.need_h1; ra.need_h2 = fa.need_h2; ra.need_f3 = fa.need_f3;
  ra.slot = pl.slot;
  ra.part = h->fpart;
  ra.C0 = h->C0; ra.Cs = h->Cs; ra.kC = h->kC; ra.Cdot2 = h->Cdot2;
  for (int n = 0; n < 3; ++n) ra.H[n] = h->H[n];
  {
    // grid for the largest work the launch shape must cover (all outputs at the ranks rl)
    FReduceArgs big = ra;
    big.r1 = rl[0]; big.r2 = rl[1]; big.r3 = rl[2];
    big.need_h1 = big.need_h2 = big.need_f3 = 1;
    // (a batch gives each thread RED_U outputs: fewer blocks, each a single round trip)
    const long long per = rl != h->r ? 256LL * RED_U : 256LL;
    A.blocks_red = (int)std::max<long long>(1, std::min<long long>(1024, (freduce_items(big) + per - 1) / per));
  }

  FFinishArgs ga{};
  bool cil = false;
  // a single stream forms M_n in the row blocks when their LDS holds C_dot and the P_n
  ga.m_inline = (rl == h->r && small_lds(h, rl, &cil, true) <= (size_t)h->lds_max) ? 1 : 0;
  A.lds_fin = small_lds(h, rl, &cil, ga.m_inline != 0);
  ga.core_in_lds = cil ? 1 : 0;
  ga.rmax = max_rank_of(rl, 3);
  ga.dt = h->cfg.dt;
  ga.dscale = dscale;
  long long rows = 0;
  for (int n = 0; n < 3; ++n) rows += h->N[n] * rl[n];
  // row elements of one block pass: FIN_EPT a thread in a batch, one for a single stream
  const long long span = (rl != h->r ? (long long)FIN_EPT : 1LL) * 256;
  ga.rowblocks = (int)std::max<long long>(1, std::min<long long>(1024, (rows + span - 1) / span));
  ga.Cs = h->Cs;
  ga.kC = h->kC;
  ga.Cdot2 = h->Cdot2;
  for (int n = 0; n < 3; ++n) {
    ga.N[n] = h->N[n];
    ga.r[n] = h->r[n];
    ga.ldU[n] = h->ldU[n];
    ga.H[n] = h->H[n];
    ga.w[n] = h->w[n];
    ga.U0[n] = h->U0[n];
    ga.Us[n] = h->Us[n];
    ga.kU[n] = h->kU[n];
    ga.B[n] = h->B[n];
    ga.P[n] = h->P2[n];
    ga.M[n] = h->Mbuf[n];
  }
  {
    // M_n prep: the stage's C_dot and one P_n in LDS
    const long long csz = prod_ll(rl, 3);
    long long pmax = 0;
    for (int n = 0; n < 3; ++n) pmax = std::max(pmax, csz);
    const size_t rmq = (size_t)max_rank_of(rl, 3);
    A.lds_mprep = (size_t)csz * 8 + (size_t)pmax * h->celt + 16 + (rmq * rmq + FIN_PART) * 8;
  }
  for (int st = 0; st < 2; ++st) {
    A.ga[st] = ga;
    A.ga[st].stage = st + 1;
    for (int n = 0; n < 3; ++n) A.ga[st].Pcur[n] = st == 0 ? h->P[n] : h->P2[n];
    A.blocks_fin[st] = ga.rowblocks + (st == 0 ? 3 : 0);
  }

  FQrArgs& qa = A.qa;
  qa = FQrArgs{};
  qa.rmax = max_rank_of(rl, 3);
  {
    const size_t rq = (size_t)qa.rmax;
    // slab rows and weighted rows; then the Gram, its factors and the fold's buffers
    const size_t slab = 2 * (size_t)QR_ROWS * rq * 8;
    const size_t fold = (3 * rq * rq + 3 * 64 + FQR_GP) * 8;
    // the core folded in place through registers (FOLD_R entries per thread), else in
    // two LDS buffers, else in global memory
    const long long csz = prod_ll(rl, 3);
    const size_t cneed = (size_t)csz * 8;
    if (rl == h->r) {
      // one block per slab; the last one to finish factors and folds
      qa.core_in_lds = qr_core_mode(csz, fold, (size_t)h->lds_max);
      A.lds_qr = std::max(slab, fold + (qa.core_in_lds == 2 ? cneed : qa.core_in_lds == 1 ? 2 * cneed : 0));
    } else {
      // a batch: one block per stream takes every slab (its streams are small, and many
      // blocks each publishing partials cost a device-wide fence apiece); room for the
      // factors, an in-place fold of up to FOLD_R entries per thread and the slab rows.
      // The factors are laid out for the current ranks when the arguments are uploaded.
      qa.whole = 1;
      qa.core_in_lds = qr_core_mode(csz, fold, (size_t)h->lds_max - slab);
      qa.slab_off = (int)(fold / 8) + (qa.core_in_lds == 2 ? (int)csz : qa.core_in_lds == 1 ? 2 * (int)csz : 0);
      A.lds_qr = fold + slab + std::min(cneed, (size_t)FOLD_R * 256 * 8);
      if (qa.core_in_lds == 1) A.lds_qr = fold + slab + 2 * cneed;
    }
  }
  A.blocks_qr = 0;
  for (int n = 0; n < 3; ++n) {
    qa.nb[n] = (int)((h->N[n] + QR_ROWS - 1) / QR_ROWS);
    qa.N[n] = h->N[n];
    qa.r[n] = h->r[n];
    qa.ldU[n] = h->ldU[n];
    A.blocks_qr += qa.whole ? 0 : qa.nb[n];
    qa.U0[n] = h->U0[n];
    qa.w[n] = h->w[n];
    qa.Li[n] = h->Lq[n];
    qa.gpart[n] = h->qpart[n];
  }
  if (qa.whole) A.blocks_qr = 1;
  qa.C0 = h->C0;
  qa.Ctmp = h->Ctmp;
  qa.counter = h->counters;
  qa.T3 = h->T3buf;

  TRY(build_post_args(h, rl, A.pa, A.lds_post));
  A.pa.T3 = h->T3buf;   // formed by the QR of this step
  for (int n = 0; n < 3; ++n) A.pa.Li[n] = h->Lq[n];   // U_n normalised by the post-step
  A.pa.want_sigma = h->sigma_every_step ? 1 : 0;
  A.blocks_post = 3 + A.pa.eblocks;

  FErrArgs& ea = A.ea;
  ea = FErrArgs{};
  ea.V = V1;
  ea.N1 = (int)h->N[0];
  ea.r1 = h->r[0];
  ea.T1 = FERR_T1;
  ea.gx = h->ferr_gx;
  ea.gy = h->ferr_gy;
  ea.M = h->N[1] * h->N[2];
  ea.E = h->E;
  ea.U1c = h->U1c;
  ea.w1 = h->w[0];
  ea.w23 = h->w23;
  ea.part = h->ferr_part;
  ea.hold = &h->ctrl->hold;
  ea.counter = h->counters + 1;
  for (int n = 0; n < 3; ++n) ea.G[n] = h->Gsave[n];
  ea.rmax = max_rank_of(rl, 3);
  A.blocks_err = h->ferr_gx * h->ferr_gy;
  if (h->ferr_cols) {
    // column-block error pass: FEC_COLS columns of the mode-1 unfolding with all rows per block
    ea.T1 = 0;
    ea.gx = (int)((ea.M + FEC_COLS - 1) / FEC_COLS);
    ea.gy = 1;
    A.blocks_err = ea.gx;
  }
  // every small kernel's LDS must fit, or the step goes to the plain path
  const size_t lmax = (size_t)h->lds_max;
  if (A.lds_fin > lmax || (!ga.m_inline && A.lds_mprep > lmax) || A.lds_qr > lmax || A.lds_post > lmax ||
      ferr_final_lds(ea.rmax) > lmax) {
    h->err = "the fused step's small kernels do not fit in LDS at these ranks";
    return TDB_EUNSUPPORTED;
  }
  return TDB_OK;
}

// Explicit Euler: the stage-1 state becomes the state.
tdb_status euler_commit(tdb_ctx* h, hipStream_t s) {
  CommitArgs ca{};
  ca.p = h->p;
  ca.csz = prod_ll(h->r, h->p);
  ca.C0 = h->C0;
  ca.Cs = h->Cs;
  for (int n = 0; n < h->p; ++n) {
    ca.N[n] = h->N[n];
    ca.r[n] = h->r[n];
    ca.ldU[n] = h->ldU[n];
    ca.U0[n] = h->U0[n];
    ca.Us[n] = h->Us[n];
  }
  HIPCHK(launch_euler_commit(ca, h->ctrl, s));
  return TDB_OK;
}

// Post-step preparation of the fused path at the committed state: core singular
// values, B_n and P_n of the next stage 1, and the error-pass expansion E.
template <typename T>
tdb_status fused_post(tdb_ctx* h, hipStream_t s) {
  FPostArgs pa{};
  size_t lds = 0;
  TRY(build_post_args(h, h->r, pa, lds));
  HIPCHK(launch_fpost<T>(pa, lds, h->ctrl, s));
  h->post_valid = true;
  return TDB_OK;
}

// After a step's error pass: read the decision, reinitialise when one was taken,
// keep the snapshot for the next difference quotient, record the statistics.
template <typename TD, typename T>
tdb_status finish_step(tdb_ctx* h, const TD* V1, hipStream_t s) {
  const int dec = h->ctrl_h->decision;
  if (dec == DEC_NONFINITE) return discard_step<TD>(h, V1, s);
  h->step += 1;
  h->t_now = h->step * h->cfg.dt;
  if (dec != DEC_NONE) {
    TRY(hosvd_select<TD>(h, V1, dec, s));
    TRY(pull_ctrl(h, s));
    TRY(fused_post<T>(h, s));
    TRY(pull_ctrl(h, s));
    if (h->gate_mode != GATE_OFF && !h->batch_owned)   // the singular-value history starts over
      HIPCHK(hipMemsetAsync(h->g_hcount, 0, sizeof(int), s));
  }
  TRY(keep_previous<TD>(h, V1, s));
  // the host copy holds this step's singular values only after a reinit (pulled in
  // full) or when a single stream formed them and pulled the controller state
  h->sigma_stale = !(dec != DEC_NONE || (h->sigma_every_step && !h->batch_owned));
  fill_stats(h, false);
  return TDB_OK;
}

// The kernels of one fused step, enqueued on s (no host synchronisation).
template <typename TD, typename T>
tdb_status enqueue_fused_step(tdb_ctx* h, StepArgs& A, hipStream_t s) {
  h->prof_now = h->prof_every <= 1 || h->prof_steps++ % h->prof_every == 0;
  h->last_path = TDB_PATH_FUSED;
  h->last_prec = A.pl.mfma == MPASS_BF16S ? TDB_PREC_BF16SPLIT : (h->f32 ? TDB_PREC_F32 : TDB_PREC_F64);
  if (!h->post_valid) TRY(fused_post<T>(h, s));
  const int stages = h->cfg.integrator == TDB_INT_EULER ? 1 : 2;
  for (int stage = 1; stage <= stages; ++stage) {
    {
      PassTimer pt(h, TDB_PASS_PROJECT, s, true);
      if (A.pl.mfma)
        HIPCHK((launch_mpass<TD>(A.fa[stage - 1], A.pl.mfma, A.pl.lds, s, pt.start(), pt.stop())));
      else
        HIPCHK((launch_fpass<TD, T>(A.fa[stage - 1], A.pl.lds, s, pt.start(), pt.stop())));
    }
    A.ra.stage = stage;
    HIPCHK(launch_freduce<T>(A.ra, h->ctrl, s));
    if (!A.ga[stage - 1].m_inline) HIPCHK(launch_fmprep<T>(A.ga[stage - 1], A.lds_mprep, h->ctrl, s));
    HIPCHK(launch_ffinish<T>(A.ga[stage - 1], A.lds_fin, h->ctrl, s));
  }
  if (stages == 1) TRY(euler_commit(h, s));
  HIPCHK(launch_fqr(A.qa, A.lds_qr, h->ctrl, s));
  HIPCHK(launch_fpost<T>(A.pa, A.lds_post, h->ctrl, s));
  h->post_valid = true;
  if (h->gate_mode != GATE_OFF && !h->batch_owned) {
    // the learned gate predicts this step's error from the singular values the
    // post-step kernel just formed, and may skip the exact error pass
    GateStepArgs g{};
    g.params = h->g_params;
    g.mean = h->g_mean;
    g.stdv = h->g_std;
    g.ctrl = h->g_ctab;
    g.hist = h->g_hist;
    g.hcount = h->g_hcount;
    g.yhat = h->g_yhat;
    g.skip = h->g_skip;
    g.would_skip = h->g_would;
    g.mode = h->gate_mode;
    HIPCHK(gate_infer(g, 1, s));
    A.ea.skip = h->g_skip;
    A.ea.would_skip = h->g_would;
    A.ea.yhat = h->g_yhat;
  }
  {
    PassTimer pt(h, TDB_PASS_ERROR, s, true);
    HIPCHK((launch_ferr<TD, T>(A.ea, h->ctrl, s, pt.start(), pt.stop())));
  }
  return TDB_OK;
}

// Waits until the final error kernel of the step enqueued with mirror m has written
// that mirror (it sets the mirror's sequence word last). A step that has not reported
// after a long spin is left to the runtime: the stream is synchronised, which also
// reports a failed launch.
tdb_status wait_mirror(tdb_ctx* h, int m) {
  volatile unsigned long long* w = h->seq_h + m;
  const unsigned long long want = h->seq_want[m];
  for (long long it = 0; *w != want; ++it) {
    if (it == (1ll << 24)) {
      HIPCHK(hipStreamSynchronize(h->pend_stream));
      if (*w != want) {
        h->err = "the pending step did not report its controller state";
        return TDB_EHIP;
      }
      break;
    }
    __builtin_ia32_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return TDB_OK;
}

// Reads the decision of the newest enqueued step and acts on it (reinitialisation,
// statistics). Waits only for that step's controller state.
template <typename TD, typename T>
tdb_status resolve_step(tdb_ctx* h) {
  if (!h->pending) return TDB_OK;
  h->pending = false;
  TRY(wait_mirror(h, h->mirror));
  h->ctrl_h = h->ctrl_hb[h->mirror];
  for (int n = 0; n < h->p; ++n) h->r[n] = h->ctrl_h->ranks[n];
  return finish_step<TD, T>(h, static_cast<const TD*>(h->Vpend), h->pend_stream);
}

tdb_status resolve_pending(tdb_ctx* h) {
  if (h->owner) return batch_resolve(h->owner);
  if (!h->pending) return TDB_OK;
  if (h->data32) return h->f32 ? resolve_step<float, float>(h) : resolve_step<float, double>(h);
  return h->f32 ? resolve_step<double, float>(h) : resolve_step<double, double>(h);
}

// D (may be NULL): a given data derivative; such a step runs synchronously (D is read
// by this call only). D2 (may be NULL): the second stage's derivative.
template <typename TD, typename T>
tdb_status ingest_fused(tdb_ctx* h, const TD* V1, hipStream_t s, const TD* D = nullptr, const TD* D2 = nullptr) {
  if (D) TRY(resolve_pending(h));
  // work enqueued earlier on another stream comes first
  if (h->pending && h->pend_stream != s) {
    HIPCHK(hipEventRecord(h->ev_ctrl[h->mirror], h->pend_stream));
    HIPCHK(hipStreamWaitEvent(s, h->ev_ctrl[h->mirror], 0));
  }
  StepArgs A;
  tdb_status bs = build_step_args(h, h->r, V1, h->Vprev, A, D, D2);
  if (bs == TDB_EUNSUPPORTED) {
    TRY(resolve_pending(h));
    bs = build_step_args(h, h->r, V1, h->Vprev, A, D, D2);   // the ranks may have changed
  }
  if (bs == TDB_EUNSUPPORTED) {
    h->post_valid = false;
    return ingest_impl<TD, T>(h, V1, s, D, D2);
  }
  TRY(bs);
  h->fused_steps += 1;
  if (!h->pipelined || D) {
    TRY((enqueue_fused_step<TD, T>(h, A, s)));
    TRY(pull_ctrl(h, s));
    return finish_step<TD, T>(h, V1, s);
  }
  // Pipelined: enqueue this step, then read the previous one's decision. When that
  // decision needs the host, this step's kernels find the hold flag raised and do
  // nothing; the host acts on the decision and enqueues this step again.
  const int m_new = h->pending ? 1 - h->mirror : h->mirror;
  auto enqueue = [&](StepArgs& Ax) -> tdb_status {
    // the final error kernel writes the controller state into this step's pinned
    // mirror itself (no separate copy on the stream)
    Ax.ea.mirror = h->ctrl_hb[m_new];
    Ax.ea.seq = h->seq_h + m_new;
    Ax.ea.seq_val = ++h->seq_next;
    h->seq_want[m_new] = h->seq_next;
    TRY((enqueue_fused_step<TD, T>(h, Ax, s)));
    return TDB_OK;
  };
  TRY(enqueue(A));
  // TDB_ENUMERIC of the previous step (discarded for non-finite data) is returned once
  // this step is in flight
  tdb_status prev = TDB_OK;
  if (h->pending) {
    h->pending = false;
    TRY(wait_mirror(h, h->mirror));
    h->ctrl_h = h->ctrl_hb[h->mirror];
    for (int n = 0; n < h->p; ++n) h->r[n] = h->ctrl_h->ranks[n];
    const int dec = h->ctrl_h->decision;
    const bool acted = dec != DEC_NONE && dec != DEC_NONFINITE;   // the device holds the steps behind it
    if (acted) HIPCHK(hipStreamSynchronize(s));   // the held step has drained
    prev = finish_step<TD, T>(h, static_cast<const TD*>(h->Vpend), h->pend_stream);
    if (prev != TDB_OK && prev != TDB_ENUMERIC) return prev;
    if (acted) {
      StepArgs A2;
      tdb_status b2 = build_step_args(h, h->r, V1, h->Vprev, A2);
      if (b2 == TDB_EUNSUPPORTED) {
        h->post_valid = false;
        return ingest_impl<TD, T>(h, V1, s);
      }
      TRY(b2);
      TRY(enqueue(A2));
    }
  }
  h->Vprev = V1;
  h->Vpend = V1;
  h->pend_stream = s;
  h->mirror = m_new;
  h->pending = true;
  return prev;
}

// With second-order differences and two earlier snapshots held, the step's two stage
// derivatives are formed first (Sec. 2.3) and projected as given derivatives; the
// first step after init takes the first-order quotient.
template <typename TD>
tdb_status ingest_dispatch(tdb_ctx* h, const void* V, hipStream_t s, const void* D = nullptr) {
  const TD* Vt = static_cast<const TD*>(V);
  const TD* Dt = static_cast<const TD*>(D);
  const TD* D2t = nullptr;
  if (!D && h->cfg.fd_order == 2 && h->Vprev2) {
    TRY(resolve_pending(h));
    TD* d1 = static_cast<TD*>(h->Dfd[0]);
    TD* d2 = static_cast<TD*>(h->Dfd[1]);
    HIPCHK(launch_fd2<TD>(static_cast<const TD*>(h->Vprev2), static_cast<const TD*>(h->Vprev), Vt, d1, d2, h->S,
                          h->cfg.dt, s));
    Dt = d1;
    D2t = d2;
  }
  if (h->dbo) {
    if (h->f32) return ingest_dbo<TD, float>(h, Vt, s, Dt, D2t);
    return ingest_dbo<TD, double>(h, Vt, s, Dt, D2t);
  }
  if (h->fused) {
    if (h->f32) return ingest_fused<TD, float>(h, Vt, s, Dt, D2t);
    return ingest_fused<TD, double>(h, Vt, s, Dt, D2t);
  }
  if (h->f32) return ingest_impl<TD, float>(h, Vt, s, Dt, D2t);
  return ingest_impl<TD, double>(h, Vt, s, Dt, D2t);
}

template <typename TD>
tdb_status init_eps(tdb_ctx* h, const TD* V, hipStream_t s) {
  if (h->f32) TRY((error_pass_plain<TD, float>(h, V, s)));
  else TRY((error_pass_plain<TD, double>(h, V, s)));
  return TDB_OK;
}

tdb_status create(const tdb_config* cfg, tdb_ctx** out) {
  *out = nullptr;
  std::string msg;
  tdb_status st = validate(cfg, msg);
  if (st != TDB_OK) { g_create_error = msg; return st; }
  tdb_ctx* h = new (std::nothrow) tdb_ctx();
  if (!h) { g_create_error = "out of host memory"; return TDB_ENOMEM; }
  st = setup(h, cfg);
  if (st != TDB_OK) {
    g_create_error = h->err;
    delete h;
    return st;
  }
  *out = h;
  return TDB_OK;
}

// HOSVD initialisation of a freshly created context from its first snapshot.
tdb_status init_hosvd(tdb_ctx* h, const void* V0_dev, hipStream_t s) {
  if (h->data32) TRY(hosvd_select<float>(h, static_cast<const float*>(V0_dev), DEC_INIT, s));
  else TRY(hosvd_select<double>(h, static_cast<const double*>(V0_dev), DEC_INIT, s));
  TRY(pull_ctrl(h, s));
  TRY(core_sigma(h, false, s));
  TRY(pull_ctrl(h, s));
  if (h->data32) TRY(keep_previous<float>(h, static_cast<const float*>(V0_dev), s));
  else TRY(keep_previous<double>(h, static_cast<const double*>(V0_dev), s));
  fill_stats(h, true);
  return TDB_OK;
}

// ---------------------------------------------------------------- batches of streams
}  // namespace

struct tdb_batch_ctx {
  int n = 0;
  std::vector<tdb_ctx*> st;
  bool data32 = false, f32 = false;
  std::string err;
  std::vector<void*> dev, host;     // owned device / pinned host blocks
  // per-stream argument tables (device) and their pinned host mirrors
  FPassArgs *d_fa[2] = {}, *h_fa[2] = {};
  FReduceArgs *d_ra = nullptr, *h_ra = nullptr;
  FFinishArgs *d_ga[2] = {}, *h_ga[2] = {};
  FQrArgs *d_qa = nullptr, *h_qa = nullptr;
  FPostArgs *d_pa = nullptr, *h_pa = nullptr;
  FErrArgs *d_ea = nullptr, *h_ea = nullptr;
  CtrlState** d_ctab = nullptr;
  const void **d_v1 = nullptr, **d_v0 = nullptr;
  // A step's snapshot pointers go to pinned tables by step parity (a kernel copies them
  // to d_v1/d_v0), its summaries to pinned buffers by parity, and the last block of its
  // final error kernel advances the parity's sequence word. With pipelining (every
  // stream borrows its snapshots) the host reads a step while the next one runs; a
  // stream whose decision needs the host is held by the device until the host has
  // acted, and its next step runs again for it alone.
  const void** h_vt[2][2] = {};     // [parity][V1, V0], pinned
  BatchSummary* h_sumb[2] = {};     // pinned
  unsigned long long* seq_h = nullptr;   // pinned, one word per parity
  unsigned long long seq_want[2] = {0, 0};
  unsigned* d_counter = nullptr;
  int* h_mask = nullptr;            // pinned: streams held while the others' step runs again
  int* d_hsave = nullptr;
  bool pipelined = false, pending = false;
  int parity = 0;                   // parity of the next step
  std::vector<const void*> pend_V;
  hipStream_t pend_stream = nullptr;
  // the step's launches as one graph per parity (TDB_GRAPH=0: plain launches)
  bool use_graph = true;
  long long graph_steps = 0;        // launches replayed from a graph
  hipStream_t cap = nullptr;        // captures only (a graph launches on the caller's stream)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gkey[2] = {-1, -1};
  // block maps (fixed at creation: grids are sized at the caps)
  BatchMap m_pass{}, m_red{}, m_fin[2]{}, m_qr{}, m_qa{}, m_post{}, m_exp{}, m_err{};
  int g_pass = 0, g_red = 0, g_fin[2] = {0, 0}, g_qr = 0, g_qa = 0, g_post = 0, g_exp = 0, g_err = 0;
  size_t lds_pass = 0, lds_fin = 0, lds_qr = 0, lds_post = 0, lds_mprep = 0, lds_final = 0;
  size_t lds_rows = 0, lds_exp = 0;   // row blocks of the finish, expansion blocks of the post-step
  int mflavor = 0;                  // MPASS_* of the batched stage pass (one for all streams)
  int rows = 0;                     // 1: the row-block pass (every stream takes it)
  int vw = 0;                       // fiber load width of the row-block pass this step
  int rp_n3c = 0;                   // mode-3 extent the column-block kernel is built for (0: any)
  int rp_t2 = 64;                   // its columns of mode 2 per workgroup
  tdb_batch_plan_info tune{};       // the plan and how it was chosen
  int err_r1c = 0;                  // column-block error pass compiled for r1 <= err_r1c (0: slab pass)
  std::vector<int> pass_blocks, pass_T1, pass_T2;   // each stream's stage-pass grid, fixed at the caps
  double bytes_pass = 0.0, bytes_err = 0.0;
  bool dirty = true;
  bool prof = false;                // pass timing on
  int prof_every = 1;               // the passes of every prof_every-th step are timed
  long long prof_steps = 0;
  bool prof_now = false;            // this step is timed
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[2];
  // a second stream (default priority) for the kernels that run beside another one: the
  // stage-1 pseudo-inverses beside the row blocks, the post-step's mode blocks beside its
  // expansion blocks (fork and join by events, captured into the step's graph)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork[2] = {}, ev_join[2] = {};
  bool side_failed = false;
  // learned gate (parameters owned by the trainer that was attached)
  int gate_mode = GATE_OFF;
  const float* gate_params = nullptr;
  float *d_gmean = nullptr, *d_gstd = nullptr, *d_ghist = nullptr, *d_gyhat = nullptr;
  int *d_ghcount = nullptr, *d_gskip = nullptr, *d_gwould = nullptr;

  ~tdb_batch_ctx() {
    for (hipGraphExec_t& g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) (void)hipStreamDestroy(side);
    for (int k = 0; k < 2; ++k) {
      if (ev_fork[k]) (void)hipEventDestroy(ev_fork[k]);
      if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
    }
    for (auto& v : ev_used)
      for (auto& e : v) { ev_pool.push_back(e.first); ev_pool.push_back(e.second); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (tdb_ctx* h : st) delete h;
    for (void* q : dev) (void)hipFree(q);
    for (void* q : host) (void)hipHostFree(q);
  }
};

struct tdb_gate_ctx {
  int max_batch = 0;
  std::vector<void*> dev;
  float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr, *loss = nullptr;
  GateScratch w{};
  int step = 0;
  std::string err;
  ~tdb_gate_ctx() {
    for (void* q : dev) (void)hipFree(q);
  }
};

#define GHIPCHK(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError();                                                         \
      g->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
      return TDB_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

#define BHIPCHK(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError();                                                         \
      b->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
      return TDB_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

namespace {

template <typename X>
tdb_status balloc(tdb_batch_ctx* b, X** d, X** hp, size_t count) {
  void* q = nullptr;
  BHIPCHK(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(X)));
  b->dev.push_back(q);
  *d = static_cast<X*>(q);
  if (hp) {
    void* r = nullptr;
    BHIPCHK(hipHostMalloc(&r, std::max<size_t>(count, 1) * sizeof(X), hipHostMallocDefault));
    b->host.push_back(r);
    *hp = static_cast<X*>(r);
  }
  return TDB_OK;
}

template <typename X>
tdb_status halloc(tdb_batch_ctx* b, X** hp, size_t count) {
  void* r = nullptr;
  BHIPCHK(hipHostMalloc(&r, std::max<size_t>(count, 1) * sizeof(X), hipHostMallocDefault));
  b->host.push_back(r);
  *hp = static_cast<X*>(r);
  return TDB_OK;
}

// Block map of one batched kernel from the per-stream block counts. With `weight`
// (the work of one block of each stream) the streams' block ranges are laid out
// heaviest first, so the longest blocks are dispatched first and the short ones fill
// the end of the launch; start[i] is then the first block of stream i but start[i+1]
// is not its end, which only kernels that take their block count elsewhere may use.
tdb_status make_map(tdb_batch_ctx* b, const std::vector<int>& counts, BatchMap* m, int* total,
                    const std::vector<double>* weight = nullptr) {
  const size_t n = counts.size();
  std::vector<int> order(n);
  for (size_t i = 0; i < n; ++i) order[i] = (int)i;
  if (weight)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return (*weight)[x] > (*weight)[y]; });
  std::vector<int> start(n + 1, 0);
  int acc = 0;
  for (size_t j = 0; j < n; ++j) {
    start[order[j]] = acc;
    acc += counts[order[j]];
  }
  start[n] = acc;
  std::vector<int> sid(std::max(acc, 1), 0);
  for (size_t i = 0; i < n; ++i)
    for (int k = start[i]; k < start[i] + counts[i]; ++k) sid[k] = (int)i;
  int *d_sid = nullptr, *d_start = nullptr;
  TRY(balloc<int>(b, &d_sid, nullptr, sid.size()));
  TRY(balloc<int>(b, &d_start, nullptr, start.size()));
  BHIPCHK(hipMemcpy(d_sid, sid.data(), sid.size() * sizeof(int), hipMemcpyHostToDevice));
  BHIPCHK(hipMemcpy(d_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice));
  m->sid = d_sid;
  m->start = d_start;
  *total = start.back();
  return TDB_OK;
}

hipEvent_t take_bevent(tdb_batch_ctx* b) {
  if (!b->ev_pool.empty()) {
    hipEvent_t e = b->ev_pool.back();
    b->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Rebuild every stream's argument structs (current ranks, launch shapes at the caps)
// and upload them.
tdb_status batch_upload_args(tdb_batch_ctx* b, hipStream_t s) {
  size_t lds_pass = 0;
  for (int i = 0; i < b->n; ++i) {
    tdb_ctx* h = b->st[i];
    StepArgs A;
    tdb_status r = build_step_args(h, h->caps, nullptr, nullptr, A);
    if (r != TDB_OK) { b->err = "stream " + std::to_string(i) + ": " + h->err; return r; }
    // The launch (grid, block map, pass kernel) was fixed at the caps: the tiles at the
    // current ranks must be exactly those blocks, and their partial slots and LDS must
    // fit what was allocated, or the step is refused before any launch.
    if (A.pl.T1 != b->pass_T1[i] || A.pl.T2 != b->pass_T2[i] || A.blocks_pass != b->pass_blocks[i] ||
        A.pl.mfma != b->mflavor || A.pl.rows != b->rows || A.pl.lds > (size_t)h->lds_max ||
        (long long)A.pl.nt1 * A.pl.nt2 * A.pl.slot > h->fpart_elems) {
      b->err = "stream " + std::to_string(i) + ": the stage-pass tiles at ranks (" + std::to_string(h->r[0]) + ", " +
               std::to_string(h->r[1]) + ", " + std::to_string(h->r[2]) + ") do not fit the launch fixed at the caps";
      return TDB_EUNSUPPORTED;
    }
    lds_pass = std::max(lds_pass, A.pl.lds);
    b->h_fa[0][i] = A.fa[0];
    b->h_fa[1][i] = A.fa[1];
    A.ra.stage = 1;
    b->h_ra[i] = A.ra;
    b->h_ga[0][i] = A.ga[0];
    b->h_ga[1][i] = A.ga[1];
    b->h_qa[i] = A.qa;
    {
      // the QR's last block lays out its factors for the current ranks, which leaves
      // room in the batch's LDS (sized at the caps) to fold a core of the current size
      FQrArgs& q = b->h_qa[i];
      q.rmax = max_rank_of(h->r, 3);
      const size_t rq = (size_t)q.rmax;
      const size_t fold = (3 * rq * rq + 3 * 64 + FQR_GP) * 8, slab = 2 * (size_t)QR_ROWS * rq * 8;
      const long long csz = prod_ll(h->r, 3);
      q.core_in_lds = qr_core_mode(csz, fold, b->lds_qr - slab);
      q.slab_off = (int)(fold / 8) + (q.core_in_lds == 2 ? (int)csz : q.core_in_lds == 1 ? 2 * (int)csz : 0);
    }
    b->h_pa[i] = A.pa;
    b->h_ea[i] = A.ea;
    if (b->gate_mode != GATE_OFF) {
      b->h_ea[i].skip = b->d_gskip + i;
      b->h_ea[i].would_skip = b->d_gwould + i;
      b->h_ea[i].yhat = b->d_gyhat + i;
    }
  }
  const size_t n = (size_t)b->n;
  BHIPCHK(hipMemcpyAsync(b->d_fa[0], b->h_fa[0], n * sizeof(FPassArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_fa[1], b->h_fa[1], n * sizeof(FPassArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_ra, b->h_ra, n * sizeof(FReduceArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_ga[0], b->h_ga[0], n * sizeof(FFinishArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_ga[1], b->h_ga[1], n * sizeof(FFinishArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_qa, b->h_qa, n * sizeof(FQrArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_pa, b->h_pa, n * sizeof(FPostArgs), hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(b->d_ea, b->h_ea, n * sizeof(FErrArgs), hipMemcpyHostToDevice, s));
  b->lds_pass = lds_pass;   // the stage pass of the current ranks
  b->dirty = false;
  b->gkey[0] = b->gkey[1] = -1;   // launch shapes may have changed: capture again
  return TDB_OK;
}

// The batch's plan: which stage-pass kernel, its columns per block, which error pass.
struct BatchChoice {
  int pass_kind = 2;   // 0: vector-ALU tiles, 1: matrix-core tiles, 2: matrix-core column blocks
  int cols = 64;       // columns of mode 2 per column block
  int err_cols = 1;    // 1: column-block error pass, 0: row slabs
};

// Launch shapes at the caps and block maps for choice c (every stream the same kernel;
// the column-block pass only when every stream takes it, then the matrix-core tiles
// only when every stream takes those; else the vector-ALU tiles).
tdb_status batch_plan(tdb_batch_ctx* b, const BatchChoice& c) {
  const int n = b->n;
  for (int i = 0; i < n; ++i) {
    b->st[i]->no_rpass = c.pass_kind != 2;
    b->st[i]->no_mfma = c.pass_kind == 0;
    b->st[i]->rpass_cols = c.cols;
  }
  b->rp_t2 = c.cols;
  {
    bool all_rows = c.pass_kind == 2;
    for (int i = 0; i < n && all_rows; ++i) all_rows = plan_pass(b->st[i], b->st[i]->caps, true).rows == 1;
    if (!all_rows)
      for (int i = 0; i < n; ++i) b->st[i]->no_rpass = true;
    b->rows = all_rows ? 1 : 0;
    int first = -1;
    bool mixed = false;
    for (int i = 0; i < n; ++i) {
      const int f = plan_pass(b->st[i], b->st[i]->caps, true).mfma;
      if (first < 0) first = f;
      else if (f != first) mixed = true;
    }
    if (mixed)
      for (int i = 0; i < n; ++i) b->st[i]->no_mfma = true;
    b->mflavor = mixed ? 0 : first;
  }
  {
    // the column-block error pass keeps a column of E in registers: every stream's
    // mode-1 rank cap at most 32 (compiled for the cap rounded up to 4)
    int r1max = 0;
    for (int i = 0; i < n; ++i) r1max = std::max(r1max, b->st[i]->caps[0]);
    const bool cols = c.err_cols && r1max <= 32;
    b->err_r1c = cols ? (r1max + 3) / 4 * 4 : 0;
    for (int i = 0; i < n; ++i) b->st[i]->ferr_cols = cols;
  }
  b->pass_blocks.clear();
  b->pass_T1.clear();
  b->pass_T2.clear();
  b->lds_pass = b->lds_fin = b->lds_qr = b->lds_post = b->lds_mprep = b->lds_final = 0;
  b->lds_rows = b->lds_exp = 0;
  b->bytes_pass = b->bytes_err = 0.0;
  std::vector<int> c_pass(n), c_red(n), c_fin0(n), c_fin1(n), c_qr(n, 3), c_qa(n), c_post(n), c_exp(n), c_err(n);
  std::vector<double> w_pass(n, 0.0), w_err(n, 0.0);
  for (int i = 0; i < n; ++i) {
    tdb_ctx* h = b->st[i];
    StepArgs A;
    tdb_status r = build_step_args(h, h->caps, nullptr, nullptr, A);
    if (r != TDB_OK) { b->err = "stream " + std::to_string(i) + ": " + h->err; return r; }
    // the plan at the caps must also hold the partials of the caps
    const PassPlan pc = plan_pass(h, h->caps, true);
    if (ensure_fpart(h, (long long)pc.nt1 * pc.nt2 * pc.slot) != TDB_OK) {
      b->err = "stream " + std::to_string(i) + ": stage-pass partials at the caps: " + h->err;
      return TDB_ENOMEM;
    }
    c_pass[i] = A.blocks_pass;
    w_pass[i] = (double)A.pl.T1 * A.pl.T2 * h->N[2];
    b->pass_blocks.push_back(A.blocks_pass);
    b->pass_T1.push_back(A.pl.T1);
    b->pass_T2.push_back(A.pl.T2);
    c_red[i] = A.blocks_red;
    c_fin0[i] = A.blocks_fin[0];
    c_fin1[i] = A.blocks_fin[1];
    c_post[i] = A.blocks_post;
    c_qa[i] = A.blocks_qr;
    c_exp[i] = A.pa.eblocks;
    c_err[i] = A.blocks_err;
    w_err[i] = b->err_r1c ? (double)h->N[0] : 1.0;
    {
      // the three M_n and the row tile (FIN_EPT * 256 elements with rmax - 1 on either side)
      long long msum = 0;
      for (int k = 0; k < 3; ++k) msum += (long long)h->caps[k] * h->caps[k];
      const size_t tile = FIN_EPT * 256 + 2 * (size_t)max_rank_of(h->caps, 3);
      b->lds_rows = std::max(b->lds_rows, ((size_t)msum + tile) * 8);
      bool sall = false;
      b->lds_exp = std::max(b->lds_exp, post_exp_lds(h, h->caps, A.pa.eblocks, &sall));
    }
    b->lds_pass = std::max(b->lds_pass, pc.lds);
    b->lds_fin = std::max(b->lds_fin, A.lds_fin);
    b->lds_qr = std::max(b->lds_qr, A.lds_qr);
    b->lds_post = std::max(b->lds_post, A.lds_post);
    b->lds_mprep = std::max(b->lds_mprep, A.lds_mprep);
    b->lds_final = std::max(b->lds_final, ferr_final_lds(A.ea.rmax));
    b->bytes_pass += 2.0 * (double)h->S * (double)h->delt;
    b->bytes_err += (double)h->S * (double)h->delt;
  }
  TRY(make_map(b, c_pass, &b->m_pass, &b->g_pass, &w_pass));
  TRY(make_map(b, c_red, &b->m_red, &b->g_red));
  TRY(make_map(b, c_fin0, &b->m_fin[0], &b->g_fin[0]));
  TRY(make_map(b, c_fin1, &b->m_fin[1], &b->g_fin[1]));
  TRY(make_map(b, c_qr, &b->m_qr, &b->g_qr));
  TRY(make_map(b, c_qa, &b->m_qa, &b->g_qa));
  TRY(make_map(b, c_post, &b->m_post, &b->g_post));
  TRY(make_map(b, c_exp, &b->m_exp, &b->g_exp));
  TRY(make_map(b, c_err, &b->m_err, &b->g_err, &w_err));
  b->dirty = true;
  b->gkey[0] = b->gkey[1] = -1;
  return TDB_OK;
}

// Plans chosen by timing, per shape class of batch (storage and compute types and the
// members' extents and caps), for the life of the process.
std::mutex g_tune_mu;
std::unordered_map<std::string, BatchChoice> g_tune_cache;

std::string tune_key(const tdb_batch_ctx* b) {
  std::vector<std::array<long long, 6>> v;
  for (const tdb_ctx* h : b->st)
    v.push_back({h->N[0], h->N[1], h->N[2], h->caps[0], h->caps[1], h->caps[2]});
  std::sort(v.begin(), v.end());
  std::string k = std::to_string(b->data32) + "/" + std::to_string(b->f32) + "/" +
                  std::to_string(b->st[0]->bf16s ? 1 : 0) + ":";
  for (const auto& e : v)
    for (long long x : e) k += std::to_string(x) + ",";
  return k;
}

// Average duration (us) of `reps` launches of the stage pass (stage-1 tables) or of the
// error pass's partials under the current plan, after one untimed launch, on the first
// snapshots (their difference is zero: the kernels' cost does not depend on the values).
// Both only write partial buffers that every step overwrites.
template <typename TD, typename T>
tdb_status time_plan(tdb_batch_ctx* b, bool pass, hipStream_t s, double* us) {
  const int n = b->n, reps = 3;
  // the previous snapshot is a distinct buffer of the same size (the stream's HOSVD
  // scratch, idle after init), so that the timed launches read as much as a step does
  for (int i = 0; i < n; ++i) {
    b->h_vt[0][0][i] = b->st[i]->Vprev;
    b->h_vt[0][1][i] = b->st[i]->hsA;
  }
  b->vw = 0;
  if (sizeof(TD) == 4 && (b->st[0]->N[2] == 4 || b->st[0]->N[2] == 8)) {
    int vw = (int)b->st[0]->N[2];
    for (int i = 0; i < n && vw; ++i)
      if (b->st[i]->N[2] != vw || (reinterpret_cast<uintptr_t>(b->h_vt[0][0][i]) & 15) != 0) vw = 0;
    b->vw = vw;
  }
  TRY(batch_upload_args(b, s));
  BHIPCHK(launch_batch_fetch_ptrs(b->h_vt[0][0], b->h_vt[0][1], b->d_v1, b->d_v0, n, s));
  hipEvent_t e0 = take_bevent(b), e1 = take_bevent(b);
  if (!e0 || !e1) { b->err = "hipEventCreate failed"; return TDB_EHIP; }
  for (int k = 0; k <= reps; ++k) {
    if (k == 1) BHIPCHK(hipEventRecord(e0, s));
    if (pass) {
      if (b->rows)
        BHIPCHK((launch_batch_rpass<TD>(b->d_fa[0], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->mflavor, b->rp_n3c,
                                        b->rp_t2, b->vw, b->lds_pass, s)));
      else if (b->mflavor)
        BHIPCHK((launch_batch_mpass<TD>(b->d_fa[0], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->mflavor,
                                        b->lds_pass, s)));
      else
        BHIPCHK((launch_batch_fpass<TD, T>(b->d_fa[0], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->lds_pass, s)));
    } else {
      BHIPCHK((launch_batch_ferr_partials<TD, T>(b->d_ea, b->d_v1, b->m_err, b->g_err, b->err_r1c, s)));
    }
  }
  BHIPCHK(hipEventRecord(e1, s));
  BHIPCHK(hipEventSynchronize(e1));
  float ms = 0.0f;
  BHIPCHK(hipEventElapsedTime(&ms, e0, e1));
  b->ev_pool.push_back(e0);
  b->ev_pool.push_back(e1);
  *us = 1e3 * (double)ms / reps;
  return TDB_OK;
}

// Chooses the plan: the cached one of an earlier batch of the same shape class, else, when
// more than one candidate applies and TDB_AUTOTUNE is not 0, the fastest by time_plan
// (stage pass first: column blocks of 64 and of 32 columns for a shared mode-3 extent of
// 4, and the matrix-core tiles; then the error pass: column blocks and row slabs), else
// the fixed rule (column blocks of 64 columns for N3 = 4, else 32; column-block error
// pass).
template <typename TD, typename T>
tdb_status batch_tune(tdb_batch_ctx* b, hipStream_t s) {
  const int n = b->n;
  int n3c = (int)b->st[0]->N[2];
  for (int i = 1; i < n; ++i)
    if (b->st[i]->N[2] != n3c) n3c = 0;
  if (n3c != 4 && n3c != 8) n3c = 0;
  b->rp_n3c = n3c;
  BatchChoice rule;
  rule.pass_kind = 2;
  rule.cols = rpass_cols_for(n3c);
  rule.err_cols = 1;
  const char* env = std::getenv("TDB_AUTOTUNE");
  bool tune = !(env && env[0] == '0');
  if (const char* ce = std::getenv("TDB_RPASS_COLS")) {
    // a forced column count (32, or 64 with N3 = 4) takes the fixed rule with it
    const int tc = std::atoi(ce);
    if (rpass_cols_ok(n3c, tc)) {
      rule.cols = tc;
      tune = false;
    }
  }
  const std::string key = tune_key(b);
  b->tune = tdb_batch_plan_info{};
  if (tune) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      TRY(batch_plan(b, it->second));
      b->tune.source = 2;
      return TDB_OK;
    }
  }
  if (!tune) {
    TRY(batch_plan(b, rule));
    b->tune.source = 0;
    return TDB_OK;
  }
  // stage-pass candidates that apply to every stream
  std::vector<BatchChoice> cands;
  BatchChoice c64 = rule, c32 = rule, ctile = rule;
  c64.cols = 64;
  c32.cols = 32;
  ctile.pass_kind = 1;
  ctile.cols = 32;
  if (n3c == 4) cands.push_back(c64);
  cands.push_back(c32);
  cands.push_back(ctile);
  BatchChoice best = rule;
  double best_us = 1e30, rule_us = -1.0;
  int timed = 0;
  for (const BatchChoice& c : cands) {
    TRY(batch_plan(b, c));
    // a candidate the streams cannot all take falls back to another kernel: skip it
    if ((c.pass_kind == 2) != (b->rows == 1) || (c.pass_kind >= 1 && !b->mflavor)) continue;
    double us = 0.0;
    TRY((time_plan<TD, T>(b, true, s, &us)));
    const int slot = c.pass_kind == 1 ? 2 : (c.cols == 64 ? 0 : 1);
    b->tune.pass_us[slot] = us;
    ++timed;
    if (c.pass_kind == rule.pass_kind && c.cols == rule.cols) rule_us = us;
    if (us < best_us) { best_us = us; best = c; }
  }
  if (timed == 0) best = rule;
  // the rule's choice stays unless another is clearly faster: candidates within a few
  // percent of each other would otherwise swap from one creation to the next on noise
  if (rule_us > 0.0 && best_us > 0.95 * rule_us) best = rule;
  // error pass
  int r1max = 0;
  for (int i = 0; i < n; ++i) r1max = std::max(r1max, b->st[i]->caps[0]);
  if (r1max <= 32) {
    double eus[2] = {0.0, 0.0};
    for (int ec = 0; ec < 2; ++ec) {
      BatchChoice c = best;
      c.err_cols = ec;
      TRY(batch_plan(b, c));
      TRY((time_plan<TD, T>(b, false, s, &eus[ec])));
      b->tune.err_us[ec] = eus[ec];
    }
    best.err_cols = eus[1] <= eus[0] ? 1 : 0;
  } else {
    best.err_cols = 0;
  }
  TRY(batch_plan(b, best));
  b->tune.source = 1;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = best;
  return TDB_OK;
}

// Tables, pinned buffers and the plan of a new batch (its members initialised).
tdb_status batch_setup(tdb_batch_ctx* b, hipStream_t s) {
  const int n = b->n;
  const size_t nn = (size_t)n;
  TRY(balloc(b, &b->d_fa[0], &b->h_fa[0], nn));
  TRY(balloc(b, &b->d_fa[1], &b->h_fa[1], nn));
  TRY(balloc(b, &b->d_ra, &b->h_ra, nn));
  TRY(balloc(b, &b->d_ga[0], &b->h_ga[0], nn));
  TRY(balloc(b, &b->d_ga[1], &b->h_ga[1], nn));
  TRY(balloc(b, &b->d_qa, &b->h_qa, nn));
  TRY(balloc(b, &b->d_pa, &b->h_pa, nn));
  TRY(balloc(b, &b->d_ea, &b->h_ea, nn));
  TRY(balloc<const void*>(b, &b->d_v1, nullptr, nn));
  TRY(balloc<const void*>(b, &b->d_v0, nullptr, nn));
  for (int q = 0; q < 2; ++q) {
    TRY(halloc<const void*>(b, &b->h_vt[q][0], nn));
    TRY(halloc<const void*>(b, &b->h_vt[q][1], nn));
    TRY(halloc<BatchSummary>(b, &b->h_sumb[q], nn));
  }
  TRY(halloc<unsigned long long>(b, &b->seq_h, 2));
  b->seq_h[0] = b->seq_h[1] = 0;
  TRY(balloc<unsigned>(b, &b->d_counter, nullptr, 1));
  BHIPCHK(hipMemset(b->d_counter, 0, sizeof(unsigned)));
  TRY(halloc<int>(b, &b->h_mask, nn));
  TRY(balloc<int>(b, &b->d_hsave, nullptr, nn));
  {
    const char* env = std::getenv("TDB_PIPELINE");
    bool borrow = true;
    for (int i = 0; i < n; ++i) borrow = borrow && b->st[i]->cfg.snapshot_mode == TDB_BORROW;
    b->pipelined = borrow && !(env && env[0] == '0');
    const char* genv = std::getenv("TDB_GRAPH");
    b->use_graph = !(genv && genv[0] == '0');
  }
  std::vector<CtrlState*> ct(nn);
  for (int i = 0; i < n; ++i) ct[i] = b->st[i]->ctrl;
  TRY(balloc<CtrlState*>(b, &b->d_ctab, nullptr, nn));
  BHIPCHK(hipMemcpy(b->d_ctab, ct.data(), nn * sizeof(CtrlState*), hipMemcpyHostToDevice));
  tdb_status r;
  if (b->data32) r = b->f32 ? batch_tune<float, float>(b, s) : batch_tune<float, double>(b, s);
  else r = b->f32 ? batch_tune<double, float>(b, s) : batch_tune<double, double>(b, s);
  TRY(r);
  BHIPCHK(hipStreamSynchronize(s));
  return TDB_OK;
}

// The launches of one batched step for snapshot parity p (no host synchronisation).
template <typename TD, typename T>
tdb_status batch_kernels(tdb_batch_ctx* b, int p, hipStream_t s) {
  const int n = b->n;
  BHIPCHK(launch_batch_fetch_ptrs(b->h_vt[p][0], b->h_vt[p][1], b->d_v1, b->d_v0, n, s));
  for (int st = 0; st < 2; ++st) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->prof_now) {
      e0 = take_bevent(b);
      e1 = take_bevent(b);
      if (e0 && e1) b->ev_used[TDB_PASS_PROJECT].push_back({e0, e1});
      else e0 = e1 = nullptr;
    }
    if (b->rows)
      BHIPCHK((launch_batch_rpass<TD>(b->d_fa[st], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->mflavor, b->rp_n3c,
                                      b->rp_t2, b->vw, b->lds_pass, s, e0, e1)));
    else if (b->mflavor)
      BHIPCHK((launch_batch_mpass<TD>(b->d_fa[st], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->mflavor, b->lds_pass,
                                      s, e0, e1)));
    else
      BHIPCHK((launch_batch_fpass<TD, T>(b->d_fa[st], b->d_v1, b->d_v0, b->m_pass, b->g_pass, b->lds_pass, s, e0,
                                         e1)));
    BHIPCHK(launch_batch_freduce<T>(b->d_ra, b->d_ctab, b->m_red, b->g_red, st + 1, s));
    // the row blocks (both stages) and the stage-1 pseudo-inverses as separate kernels;
    // the pseudo-inverses need only the stage core and share no buffer with the M prep
    // or the row blocks (a single stream runs the two finish roles as one launch), so
    // with a side stream they run beside those
    const bool fork = st == 0 && b->side;
    if (fork) {
      BHIPCHK(hipEventRecord(b->ev_fork[0], s));
      BHIPCHK(hipStreamWaitEvent(b->side, b->ev_fork[0], 0));
      BHIPCHK(launch_batch_ffinish<T>(b->d_ga[st], b->d_ctab, b->m_qr, b->g_qr, st + 1, b->lds_fin, ROLE_PINV,
                                      b->side));
      BHIPCHK(hipEventRecord(b->ev_join[0], b->side));
    }
    BHIPCHK(launch_batch_fmprep<T>(b->d_ga[st], b->d_ctab, b->m_qr, b->g_qr, st + 1, b->lds_mprep, s));
    BHIPCHK(launch_batch_ffinish<T>(b->d_ga[st], b->d_ctab, b->m_fin[1], b->g_fin[1], st + 1, b->lds_rows, ROLE_ROWS,
                                    s));
    if (fork)
      BHIPCHK(hipStreamWaitEvent(s, b->ev_join[0], 0));
    else if (st == 0)
      BHIPCHK(launch_batch_ffinish<T>(b->d_ga[st], b->d_ctab, b->m_qr, b->g_qr, st + 1, b->lds_fin, ROLE_PINV, s));
  }
  BHIPCHK(launch_batch_fqr(b->d_qa, b->d_ctab, b->m_qa, b->g_qa, b->lds_qr, s));
  // the post-step's mode blocks (core Grams, next pseudo-inverses) and expansion blocks
  // likewise share no buffer
  if (b->side) {
    BHIPCHK(hipEventRecord(b->ev_fork[1], s));
    BHIPCHK(hipStreamWaitEvent(b->side, b->ev_fork[1], 0));
    BHIPCHK(launch_batch_fpost<T>(b->d_pa, b->d_ctab, b->m_qr, b->g_qr, b->lds_post, ROLE_MODES, b->side));
    BHIPCHK(hipEventRecord(b->ev_join[1], b->side));
    BHIPCHK(launch_batch_fpost<T>(b->d_pa, b->d_ctab, b->m_exp, b->g_exp, b->lds_exp, ROLE_EXP, s));
    BHIPCHK(hipStreamWaitEvent(s, b->ev_join[1], 0));
  } else {
    BHIPCHK(launch_batch_fpost<T>(b->d_pa, b->d_ctab, b->m_qr, b->g_qr, b->lds_post, ROLE_MODES, s));
    BHIPCHK(launch_batch_fpost<T>(b->d_pa, b->d_ctab, b->m_exp, b->g_exp, b->lds_exp, ROLE_EXP, s));
  }
  if (b->gate_mode != GATE_OFF) {
    GateStepArgs g{};
    g.params = b->gate_params;
    g.mean = b->d_gmean;
    g.stdv = b->d_gstd;
    g.ctrl = b->d_ctab;
    g.hist = b->d_ghist;
    g.hcount = b->d_ghcount;
    g.yhat = b->d_gyhat;
    g.skip = b->d_gskip;
    g.would_skip = b->d_gwould;
    g.mode = b->gate_mode;
    BHIPCHK(gate_infer(g, n, s));
  }
  {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->prof_now) {
      e0 = take_bevent(b);
      e1 = take_bevent(b);
      if (e0 && e1) b->ev_used[TDB_PASS_ERROR].push_back({e0, e1});
      else e0 = e1 = nullptr;
    }
    BHIPCHK((launch_batch_ferr<TD, T>(b->d_ea, b->d_v1, b->m_err, b->g_err, n, b->d_ctab, b->h_sumb[p], b->d_counter,
                                      b->seq_h + p, b->lds_final, b->err_r1c, s, e0, e1)));
  }
  return TDB_OK;
}

// Enqueues the step of parity p: a replay of the parity's graph when it was captured
// with the current launch shapes (argument tables and LDS sizes change only through
// batch_upload_args, which drops the graphs; the fiber width is the key), else the
// launches themselves, captured first when graphs are on. A capture that fails turns
// graphs off for the batch and the launches run as they are.
template <typename TD, typename T>
tdb_status batch_enqueue(tdb_batch_ctx* b, int p, hipStream_t s) {
  if (!b->side && !b->side_failed) {
    // the side stream and its events, made once, before any capture (without them every
    // kernel runs on s)
    bool ok = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
      ok = hipEventCreateWithFlags(&b->ev_fork[k], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      if (b->side) (void)hipStreamDestroy(b->side);
      b->side = nullptr;
      b->side_failed = true;
    }
  }
  const bool graph = b->use_graph && !b->prof_now;
  const int key = b->vw;
  if (graph && b->gexec[p] && b->gkey[p] == key) {
    BHIPCHK(hipGraphLaunch(b->gexec[p], s));
    b->graph_steps += 1;
  } else if (graph) {
    if (b->gexec[p]) {
      (void)hipGraphExecDestroy(b->gexec[p]);
      b->gexec[p] = nullptr;
      b->gkey[p] = -1;
    }
    bool ok = b->cap || hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    tdb_status r = TDB_OK;
    hipGraph_t g = nullptr;
    if (ok) {
      r = batch_kernels<TD, T>(b, p, b->cap);
      ok = hipStreamEndCapture(b->cap, &g) == hipSuccess && g != nullptr && r == TDB_OK;
      if (ok) ok = hipGraphInstantiate(&b->gexec[p], g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
    }
    (void)hipGetLastError();
    if (ok) {
      b->gkey[p] = key;
      BHIPCHK(hipGraphLaunch(b->gexec[p], s));
      b->graph_steps += 1;
    } else {
      if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
      b->gexec[p] = nullptr;
      b->use_graph = false;
      TRY((batch_kernels<TD, T>(b, p, s)));
    }
  } else {
    TRY((batch_kernels<TD, T>(b, p, s)));
  }
  b->seq_want[p] += 1;
  return TDB_OK;
}

// Waits for the summaries of the newest step of parity p (the sequence word of the
// parity reaches the number of final kernels enqueued for it; a step that does not
// report after a long spin is left to the runtime, which also reports a failed launch)
// and applies them, stream by stream. acted[i]: stream i's decision needed the host
// (which then drained the device before acting on it).
template <typename TD, typename T>
tdb_status batch_process(tdb_batch_ctx* b, int p, const std::vector<const void*>& V, hipStream_t s,
                         std::vector<char>& acted) {
  const int n = b->n;
  {
    volatile unsigned long long* w = b->seq_h + p;
    const unsigned long long want = b->seq_want[p];
    for (long long it = 0; *w != want; ++it) {
      if (it == (1ll << 24)) {
        BHIPCHK(hipStreamSynchronize(s));
        if (*w != want) {
          b->err = "the pending batch step did not report its summaries";
          return TDB_EHIP;
        }
        break;
      }
      __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
  }
  acted.assign(n, 0);
  bool drained = false;
  int first_bad = -1, n_bad = 0;
  for (int i = 0; i < n; ++i) {
    tdb_ctx* h = b->st[i];
    const BatchSummary& q = b->h_sumb[p][i];
    CtrlState& c = *h->ctrl_h;
    c.decision = q.decision;
    c.event = q.event;
    c.numeric = q.numeric;
    for (int k = 0; k < 5; ++k) c.n_events[k] = q.n_events[k];
    c.eps = q.eps;
    c.nu = q.nu;
    c.eps2 = q.eps2;
    c.nu2 = q.nu2;
    c.eps_after = NAN;   // as the controller leaves it on a step without an event
    c.gated = q.gated;
    c.would_skip = q.would_skip;
    c.eps_pred = q.eps_pred;
    h->post_valid = true;
    acted[i] = q.decision != DEC_NONE && q.decision != DEC_NONFINITE;
    if (acted[i] && !drained) {   // the step enqueued behind this one (held for it) drains first
      BHIPCHK(hipStreamSynchronize(s));
      drained = true;
    }
    const int r0[3] = {h->r[0], h->r[1], h->r[2]};
    tdb_status r = finish_step<TD, T>(h, static_cast<const TD*>(V[i]), s);
    if (r == TDB_ENUMERIC) {   // this stream's step was discarded; the others went on
      if (first_bad < 0) first_bad = i;
      ++n_bad;
    } else if (r != TDB_OK) {
      b->err = "stream " + std::to_string(i) + ": " + h->err;
      return r;
    }
    if (h->r[0] != r0[0] || h->r[1] != r0[1] || h->r[2] != r0[2]) b->dirty = true;
    if (q.decision != DEC_NONE && b->gate_mode != GATE_OFF)   // the singular values start over
      BHIPCHK(hipMemsetAsync(b->d_ghcount + i, 0, sizeof(int), s));
    h->fused_steps += 1;
    h->last_path = TDB_PATH_FUSED;
    h->last_prec = b->mflavor == MPASS_BF16S ? TDB_PREC_BF16SPLIT : (h->f32 ? TDB_PREC_F32 : TDB_PREC_F64);
  }
  if (n_bad > 0) {
    b->err = std::to_string(n_bad) + " stream(s), the first " + std::to_string(first_bad) +
             ", had non-finite data: their steps were not applied (the other streams advanced)";
    return TDB_ENUMERIC;
  }
  return TDB_OK;
}

// One batched step. Pipelined: enqueue it, then read the previous step and act on its
// decisions; the streams that needed the host were held by the device during this
// step, which then runs again for them alone (the others held meanwhile). Without
// pipelining the step is read at once. TDB_ENUMERIC reports a discarded step of the
// step read by this call.
template <typename TD, typename T>
tdb_status batch_step(tdb_batch_ctx* b, const void* const* V, hipStream_t s) {
  const int n = b->n;
  const int p = b->parity;
  for (int i = 0; i < n; ++i) {
    b->h_vt[p][0][i] = V[i];
    b->h_vt[p][1][i] = b->st[i]->Vprev;
  }
  {
    // whole fibers as float4 loads when every stream's snapshots allow it
    int vw = (sizeof(TD) == 4) ? (int)b->st[0]->N[2] : 0;
    if (vw != 4 && vw != 8) vw = 0;
    for (int i = 0; i < n && vw; ++i) {
      const uintptr_t a1 = reinterpret_cast<uintptr_t>(b->h_vt[p][0][i]);
      const uintptr_t a0 = reinterpret_cast<uintptr_t>(b->h_vt[p][1][i]);
      if (b->st[i]->N[2] != vw || ((a1 | a0) & 15) != 0 || !b->h_vt[p][1][i]) vw = 0;
    }
    b->vw = vw;
  }
  if (b->dirty) TRY(batch_upload_args(b, s));
  b->prof_now = b->prof && b->prof_steps++ % b->prof_every == 0;
  TRY((batch_enqueue<TD, T>(b, p, s)));
  tdb_status prev = TDB_OK;
  std::vector<char> acted;
  if (b->pending) {
    b->pending = false;
    prev = batch_process<TD, T>(b, 1 - p, b->pend_V, b->pend_stream, acted);
    if (prev != TDB_OK && prev != TDB_ENUMERIC) return prev;
    int na = 0;
    for (int i = 0; i < n; ++i) na += acted[i] ? 1 : 0;
    if (na > 0) {
      for (int i = 0; i < n; ++i) b->h_mask[i] = acted[i] ? 0 : 1;
      BHIPCHK(launch_batch_hold_mask(b->d_ctab, b->h_mask, b->d_hsave, n, 0, s));
      if (b->dirty) TRY(batch_upload_args(b, s));
      TRY((batch_enqueue<TD, T>(b, p, s)));
      BHIPCHK(launch_batch_hold_mask(b->d_ctab, b->h_mask, b->d_hsave, n, 1, s));
    }
  }
  for (int i = 0; i < n; ++i) b->st[i]->Vprev = V[i];
  b->pend_V.assign(V, V + n);
  b->pend_stream = s;
  b->pending = true;
  b->parity = 1 - p;
  if (!b->pipelined) {
    b->pending = false;
    return batch_process<TD, T>(b, p, b->pend_V, s, acted);
  }
  return prev;
}

template <typename TD, typename T>
tdb_status batch_resolve_as(tdb_batch_ctx* b) {
  if (!b->pending) return TDB_OK;
  b->pending = false;
  std::vector<char> acted;
  return batch_process<TD, T>(b, 1 - b->parity, b->pend_V, b->pend_stream, acted);
}

long long batch_graph_steps(const tdb_batch_ctx* b) { return b->graph_steps; }

// Reads the newest batched step if it has not been read (the calls that return results
// of a batch member come here first).
tdb_status batch_resolve(tdb_batch_ctx* b) {
  if (b->data32) return b->f32 ? batch_resolve_as<float, float>(b) : batch_resolve_as<float, double>(b);
  return b->f32 ? batch_resolve_as<double, float>(b) : batch_resolve_as<double, double>(b);
}

}  // namespace

extern "C" {

tdb_status tdb_init(const tdb_config* cfg, const void* V0_dev, void* stream, tdb_handle* out) {
  if (!out) { g_create_error = "out is NULL"; return TDB_EINVAL; }
  *out = nullptr;
  if (!V0_dev) { g_create_error = "V0_dev is NULL"; return TDB_EINVAL; }
  tdb_ctx* h = nullptr;
  tdb_status st = create(cfg, &h);
  if (st != TDB_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto run = [&]() -> tdb_status {
    bool bad = false;
    TRY(has_nonfinite_any(h, V0_dev, s, &bad));
    if (bad) { h->err = "non-finite values (NaN or Inf) in the first snapshot"; return TDB_ENUMERIC; }
    return init_hosvd(h, V0_dev, s);
  };
  st = run();
  if (st != TDB_OK) {
    g_create_error = h->err;
    delete h;
    return st;
  }
  h->ready = true;
  *out = h;
  return TDB_OK;
}

tdb_status tdb_init_from_factors(const tdb_config* cfg, const void* V0_dev, const int32_t* ranks,
                                 const double* C_host, const double* const* U_host, void* stream,
                                 tdb_handle* out) {
  if (!out) { g_create_error = "out is NULL"; return TDB_EINVAL; }
  *out = nullptr;
  if (!V0_dev || !ranks || !C_host || !U_host) { g_create_error = "NULL argument"; return TDB_EINVAL; }
  tdb_ctx* h = nullptr;
  tdb_status st = create(cfg, &h);
  if (st != TDB_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto run = [&]() -> tdb_status {
    bool bad = false;
    TRY(has_nonfinite_any(h, V0_dev, s, &bad));
    if (bad) { h->err = "non-finite values (NaN or Inf) in the first snapshot"; return TDB_ENUMERIC; }
    for (int n = 0; n < h->p; ++n) {
      if (ranks[n] < 1 || ranks[n] > h->caps[n] || !U_host[n]) {
        h->err = "ranks must be in [1, cap] with a basis for every mode";
        return TDB_EINVAL;
      }
      h->r[n] = ranks[n];
    }
    {
      bool fin = true;
      const long long csz = prod_ll(h->r, h->p);
      for (long long i = 0; i < csz; ++i) fin = fin && std::isfinite(C_host[i]);
      for (int n = 0; n < h->p; ++n)
        for (long long i = 0; i < h->N[n] * h->r[n]; ++i) fin = fin && std::isfinite(U_host[n][i]);
      if (!fin) { h->err = "non-finite values in the given core or bases"; return TDB_ENUMERIC; }
    }
    for (int n = 0; n < h->p; ++n)
      if (h->r[n] > prod_ll(h->r, h->p, n)) {
        h->err = "each rank must not exceed the product of the others";
        return TDB_EINVAL;
      }
    HIPCHK(hipMemcpy(h->C0, C_host, prod_ll(h->r, h->p) * sizeof(double), hipMemcpyHostToDevice));
    for (int n = 0; n < h->p; ++n) {
      HIPCHK(hipMemset(h->U0[n], 0, (size_t)h->N[n] * h->ldU[n] * sizeof(double)));
      HIPCHK(hipMemcpy2D(h->U0[n], h->ldU[n] * sizeof(double), U_host[n], h->r[n] * sizeof(double),
                         h->r[n] * sizeof(double), h->N[n], hipMemcpyHostToDevice));
    }
    for (int n = 0; n < h->p; ++n) h->ctrl_h->ranks[n] = h->r[n];
    HIPCHK(hipMemcpy(h->ctrl, h->ctrl_h, sizeof(CtrlState), hipMemcpyHostToDevice));
    if (h->data32) TRY(init_eps<float>(h, static_cast<const float*>(V0_dev), s));
    else TRY(init_eps<double>(h, static_cast<const double*>(V0_dev), s));
    TRY(core_sigma(h, false, s));
    TRY(pull_ctrl(h, s));
    h->ctrl_h->eps = std::sqrt(std::max(h->ctrl_h->eps2, 0.0));   // finite: V0 and the factors were checked
    h->ctrl_h->nu = std::sqrt(std::max(h->ctrl_h->nu2, 0.0));
    HIPCHK(hipMemcpy(h->ctrl, h->ctrl_h, sizeof(CtrlState), hipMemcpyHostToDevice));
    if (h->data32) TRY(keep_previous<float>(h, static_cast<const float*>(V0_dev), s));
    else TRY(keep_previous<double>(h, static_cast<const double*>(V0_dev), s));
    fill_stats(h, true);
    return TDB_OK;
  };
  st = run();
  if (st != TDB_OK) {
    g_create_error = h->err;
    delete h;
    return st;
  }
  h->ready = true;
  *out = h;
  return TDB_OK;
}

tdb_status tdb_ingest_snapshot(tdb_handle h, const void* V_dev, void* stream) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  if (!V_dev) { h->err = "V_dev is NULL"; return TDB_EINVAL; }
  if (h->batch_owned) { h->err = "this stream belongs to a batch: use tdb_batch_ingest"; return TDB_ESTATE; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->data32 ? ingest_dispatch<float>(h, V_dev, s) : ingest_dispatch<double>(h, V_dev, s);
}

tdb_status tdb_ingest_with_derivative(tdb_handle h, const void* V_dev, const void* D_dev, void* stream) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  if (!V_dev || !D_dev) { h->err = "V_dev and D_dev must not be NULL"; return TDB_EINVAL; }
  if (h->batch_owned) { h->err = "this stream belongs to a batch: use tdb_batch_ingest"; return TDB_ESTATE; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(resolve_pending(h));
  // the derivative reaches the core derivative (and the device check) but the snapshot
  // only the error pass, after the state is advanced: both are checked first
  bool bad_v = false, bad_d = false;
  TRY(has_nonfinite_any(h, V_dev, s, &bad_v));
  TRY(has_nonfinite_any(h, D_dev, s, &bad_d));
  if (bad_v || bad_d) {
    h->n_nonfinite += 1;
    h->err = std::string("non-finite values (NaN or Inf) in the ") + (bad_v ? "snapshot" : "derivative") +
             ": the step was not taken";
    return TDB_ENUMERIC;
  }
  return h->data32 ? ingest_dispatch<float>(h, V_dev, s, D_dev) : ingest_dispatch<double>(h, V_dev, s, D_dev);
}

tdb_status tdb_flush(tdb_handle h) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  return resolve_pending(h);
}

tdb_status tdb_get_core_and_bases(tdb_handle h, int32_t rotate, int32_t* ranks_out, double* C_host,
                                  double* const* U_host) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  TRY(resolve_pending(h));
  HIPCHK(hipDeviceSynchronize());
  if (ranks_out)
    for (int n = 0; n < TDB_MAX_ORDER; ++n) ranks_out[n] = n < h->p ? h->r[n] : 0;
  const long long csz = prod_ll(h->r, h->p);
  if (!rotate) {
    if (C_host) HIPCHK(hipMemcpy(C_host, h->C0, csz * sizeof(double), hipMemcpyDeviceToHost));
    if (U_host)
      for (int n = 0; n < h->p; ++n)
        if (U_host[n])
          HIPCHK(hipMemcpy2D(U_host[n], h->r[n] * sizeof(double), h->U0[n], h->ldU[n] * sizeof(double),
                             h->r[n] * sizeof(double), h->N[n], hipMemcpyDeviceToHost));
    return TDB_OK;
  }
  // energetic rotation eq. (rot): U_n Psi_n and C x_n Psi_n^T
  hipStream_t s = nullptr;
  TRY(core_sigma(h, true, s));
  HIPCHK(hipMemcpyAsync(h->hsA, h->C0, csz * sizeof(double), hipMemcpyDeviceToDevice, s));
  double* cur = h->hsA;
  double* nxt = h->hsB;
  for (int n = 0; n < h->p; ++n) {
    long long A = 1, Bz = 1;
    for (int j = 0; j < n; ++j) A *= h->r[j];
    for (int j = n + 1; j < h->p; ++j) Bz *= h->r[j];
    HIPCHK((launch_ttm<double, double, double>(cur, nullptr, nxt, h->Psi[n], h->r[n], 1, A, h->r[n],
                                                h->r[n], Bz, s)));
    std::swap(cur, nxt);
  }
  if (C_host) HIPCHK(hipMemcpyAsync(C_host, cur, csz * sizeof(double), hipMemcpyDeviceToHost, s));
  if (U_host) {
    for (int n = 0; n < h->p; ++n) {
      if (!U_host[n]) continue;
      // dense copy of U_n, then U_n Psi_n viewed as (N_n, r_n, 1) x_2 Psi^T
      HIPCHK(hipMemcpy2DAsync(nxt, h->r[n] * sizeof(double), h->U0[n], h->ldU[n] * sizeof(double),
                              h->r[n] * sizeof(double), h->N[n], hipMemcpyDeviceToDevice, s));
      double* outb = (nxt == h->hsA) ? h->hsB : h->hsA;
      if (outb == cur) outb = static_cast<double*>(h->wsA);
      HIPCHK((launch_ttm<double, double, double>(nxt, nullptr, outb, h->Psi[n], h->r[n], 1, h->N[n], h->r[n],
                                                  h->r[n], 1, s)));
      HIPCHK(hipMemcpyAsync(U_host[n], outb, h->N[n] * h->r[n] * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return TDB_OK;
}

tdb_status tdb_reconstruct(tdb_handle h, void* out_dev, void* stream) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  TRY(resolve_pending(h));
  if (!out_dev) { h->err = "out_dev is NULL"; return TDB_EINVAL; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->f32) {
    float* R = nullptr;
    TRY(reconstruct_plain<float>(h, &R, s));
    if (h->data32) HIPCHK(hipMemcpyAsync(out_dev, R, h->S * 4, hipMemcpyDeviceToDevice, s));
    else HIPCHK((launch_convert<float, double>(R, static_cast<double*>(out_dev), h->S, s)));
  } else {
    double* R = nullptr;
    TRY(reconstruct_plain<double>(h, &R, s));
    if (h->data32) HIPCHK((launch_convert<double, float>(R, static_cast<float*>(out_dev), h->S, s)));
    else HIPCHK(hipMemcpyAsync(out_dev, R, h->S * 8, hipMemcpyDeviceToDevice, s));
  }
  return TDB_OK;
}

tdb_status tdb_set_threshold(tdb_handle h, double eps_th, double gamma_th) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  if (!(eps_th > 0.0) || gamma_th >= 100.0) { h->err = "bad threshold"; return TDB_EINVAL; }
  TRY(resolve_pending(h));
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(h->ctrl_h, h->ctrl, sizeof(CtrlState), hipMemcpyDeviceToHost));
  h->ctrl_h->eps_th = eps_th;
  h->ctrl_h->gamma_th = gamma_th;
  if (!h->ctrl_h->unmet) h->ctrl_h->eps_trig = eps_th;
  HIPCHK(hipMemcpy(h->ctrl, h->ctrl_h, sizeof(CtrlState), hipMemcpyHostToDevice));
  h->cfg.eps_th = eps_th;
  h->cfg.gamma_th = gamma_th;
  return TDB_OK;
}

tdb_status tdb_get_stats(tdb_handle h, tdb_stats* out) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!out) { h->err = "out is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  TRY(resolve_pending(h));
  if (h->sigma_stale) {
    // fused steps form the core singular values only when the controller needs them;
    // the statistics form them on demand from the committed core
    HIPCHK(hipDeviceSynchronize());
    TRY(core_sigma(h, false, nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(h->ctrl_h->sigma, h->ctrl->sigma, sizeof(h->ctrl_h->sigma), hipMemcpyDeviceToHost));
    for (int n = 0; n < 4; ++n)
      for (int i = 0; i < TDB_SIGMA_K; ++i)
        h->stats.sigma[n][i] = (n < h->p && i < h->r[n]) ? h->ctrl_h->sigma[n][i] : 0.0;
    h->sigma_stale = false;
  }
  // counters that also move on a step that was not applied
  h->stats.fused_steps = h->fused_steps;
  h->stats.plain_steps = h->plain_steps;
  h->stats.n_nonfinite = h->n_nonfinite;
  h->stats.graph_steps = h->owner ? batch_graph_steps(h->owner) : 0;
  *out = h->stats;
  return TDB_OK;
}

void tdb_destroy(tdb_handle h) {
  if (!h || h->batch_owned) return;
  (void)hipDeviceSynchronize();
  delete h;
}

tdb_status tdb_profile_enable(tdb_handle h, int32_t on) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  TRY(resolve_pending(h));
  HIPCHK(hipDeviceSynchronize());
  for (auto& v : h->ev_used) {
    for (auto& e : v) { h->ev_pool.push_back(e.first); h->ev_pool.push_back(e.second); }
    v.clear();
  }
  h->prof = on != 0;
  h->prof_every = on > 1 ? on : 1;
  h->prof_steps = 0;
  h->prof_now = true;
  return TDB_OK;
}

tdb_status tdb_profile_read(tdb_handle h, int32_t pass, int64_t* launches, double* total_ms,
                            double* bytes_per_launch) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  TRY(resolve_pending(h));
  if (pass != TDB_PASS_PROJECT && pass != TDB_PASS_ERROR) { h->err = "bad pass id"; return TDB_EINVAL; }
  double ms = 0.0;
  for (auto& e : h->ev_used[pass]) {
    HIPCHK(hipEventSynchronize(e.second));
    float x = 0.0f;
    HIPCHK(hipEventElapsedTime(&x, e.first, e.second));
    ms += x;
  }
  if (launches) *launches = (int64_t)h->ev_used[pass].size();
  if (total_ms) *total_ms = ms;
  if (bytes_per_launch)
    *bytes_per_launch = (double)h->S * (double)h->delt * (pass == TDB_PASS_PROJECT ? 2.0 : 1.0);
  return TDB_OK;
}

tdb_status tdb_batch_create(int32_t n, const tdb_config* cfgs, const void* const* V0_dev, void* stream,
                            tdb_batch* out) {
  if (!out) { g_create_error = "out is NULL"; return TDB_EINVAL; }
  *out = nullptr;
  if (n < 1 || !cfgs || !V0_dev) { g_create_error = "need n >= 1 configurations and snapshots"; return TDB_EINVAL; }
  tdb_batch_ctx* b = new (std::nothrow) tdb_batch_ctx();
  if (!b) { g_create_error = "out of host memory"; return TDB_ENOMEM; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto run = [&]() -> tdb_status {
    b->n = n;
    b->data32 = cfgs[0].data_dtype == TDB_F32;
    b->f32 = cfgs[0].precision != TDB_PREC_F64;   // FP32 buffers for F32 and BF16SPLIT alike
    for (int i = 0; i < n; ++i) {
      const tdb_config& c = cfgs[i];
      if (c.order != 3 || c.path == TDB_PATH_PLAIN) {
        b->err = "stream " + std::to_string(i) + ": batches take third-order streams on the fused path";
        return TDB_EUNSUPPORTED;
      }
      if (c.integrator != TDB_INT_HEUN) {
        b->err = "stream " + std::to_string(i) + ": batches step with the Heun integrator only";
        return TDB_EUNSUPPORTED;
      }
      if (c.fd_order == 2) {
        b->err = "stream " + std::to_string(i) + ": batches take the first-order difference quotient only";
        return TDB_EUNSUPPORTED;
      }
      if ((c.data_dtype == TDB_F32) != b->data32 || c.precision != cfgs[0].precision) {
        b->err = "all streams of a batch share data_dtype and precision";
        return TDB_EINVAL;
      }
      if (!V0_dev[i]) { b->err = "stream " + std::to_string(i) + ": V0 is NULL"; return TDB_EINVAL; }
      std::string msg;
      const tdb_status v = validate(&c, msg);
      if (v != TDB_OK) { b->err = "stream " + std::to_string(i) + ": " + msg; return v; }
    }
    for (int i = 0; i < n; ++i) {
      const tdb_config& c = cfgs[i];
      tdb_ctx* h = nullptr;
      tdb_status r = create(&c, &h);
      if (r != TDB_OK) { b->err = "stream " + std::to_string(i) + ": " + g_create_error; return r; }
      b->st.push_back(h);
      h->batch_owned = true;
      h->owner = b;
      if (h->f32 != b->f32 || h->data32 != b->data32) {
        b->err = "internal: stream " + std::to_string(i) + " buffer precision differs from the batch";
        return TDB_EINVAL;
      }
      bool bad = false;
      r = has_nonfinite_any(h, V0_dev[i], s, &bad);
      if (r == TDB_OK && bad) {
        h->err = "non-finite values (NaN or Inf) in the first snapshot";
        r = TDB_ENUMERIC;
      }
      if (r == TDB_OK) r = init_hosvd(h, V0_dev[i], s);
      if (r == TDB_OK) r = b->f32 ? fused_post<float>(h, s) : fused_post<double>(h, s);
      if (r == TDB_OK) r = pull_ctrl(h, s);
      if (r != TDB_OK) { b->err = "stream " + std::to_string(i) + ": " + h->err; return r; }
      h->ready = true;
    }
    return batch_setup(b, s);
  };
  tdb_status st = run();
  if (st != TDB_OK) {
    g_create_error = b->err;
    delete b;
    return st;
  }
  *out = b;
  return TDB_OK;
}

tdb_status tdb_batch_ingest(tdb_batch b, const void* const* V_dev, void* stream) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  if (!V_dev) { b->err = "V_dev is NULL"; return TDB_EINVAL; }
  for (int i = 0; i < b->n; ++i)
    if (!V_dev[i]) { b->err = "snapshot " + std::to_string(i) + " is NULL"; return TDB_EINVAL; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  tdb_status st;
  if (b->data32) st = b->f32 ? batch_step<float, float>(b, V_dev, s) : batch_step<float, double>(b, V_dev, s);
  else st = b->f32 ? batch_step<double, float>(b, V_dev, s) : batch_step<double, double>(b, V_dev, s);
  return st;
}

tdb_status tdb_batch_stream(tdb_batch b, int32_t i, tdb_handle* out) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  if (!out || i < 0 || i >= b->n) { b->err = "bad stream index"; return TDB_EINVAL; }
  *out = b->st[i];
  return TDB_OK;
}

tdb_status tdb_batch_profile_enable(tdb_batch b, int32_t on) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  {
    const tdb_status r = batch_resolve(b);
    if (r != TDB_OK && r != TDB_ENUMERIC) return r;
  }
  BHIPCHK(hipDeviceSynchronize());
  for (auto& v : b->ev_used) {
    for (auto& e : v) { b->ev_pool.push_back(e.first); b->ev_pool.push_back(e.second); }
    v.clear();
  }
  b->prof = on != 0;
  b->prof_every = on > 1 ? on : 1;
  b->prof_steps = 0;
  return TDB_OK;
}

tdb_status tdb_batch_profile_read(tdb_batch b, int32_t pass, int64_t* launches, double* total_ms,
                                  double* bytes_per_launch) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  if (pass != TDB_PASS_PROJECT && pass != TDB_PASS_ERROR) { b->err = "bad pass id"; return TDB_EINVAL; }
  {
    const tdb_status r = batch_resolve(b);
    if (r != TDB_OK && r != TDB_ENUMERIC) return r;
  }
  double ms = 0.0;
  for (auto& e : b->ev_used[pass]) {
    BHIPCHK(hipEventSynchronize(e.second));
    float x = 0.0f;
    BHIPCHK(hipEventElapsedTime(&x, e.first, e.second));
    ms += x;
  }
  if (launches) *launches = (int64_t)b->ev_used[pass].size();
  if (total_ms) *total_ms = ms;
  if (bytes_per_launch) *bytes_per_launch = pass == TDB_PASS_PROJECT ? b->bytes_pass : b->bytes_err;
  return TDB_OK;
}

void tdb_batch_destroy(tdb_batch b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  delete b;
}

tdb_status tdb_batch_plan(tdb_batch b, tdb_batch_plan_info* out) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  if (!out) { b->err = "out is NULL"; return TDB_EINVAL; }
  tdb_batch_plan_info q = b->tune;
  q.pass_kind = b->rows ? 2 : (b->mflavor ? 1 : 0);
  q.pass_cols = b->rows ? b->rp_t2 : (b->pass_T2.empty() ? 0 : b->pass_T2[0]);
  q.err_kind = b->err_r1c ? 1 : 0;
  *out = q;
  return TDB_OK;
}

tdb_status tdb_batch_flush(tdb_batch b) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  return batch_resolve(b);
}

const char* tdb_batch_last_error(tdb_batch b) {
  if (!b) return g_create_error.c_str();
  return b->err.c_str();
}

tdb_status tdb_gate_create(int32_t max_batch, tdb_gate* out) {
  if (!out) { g_create_error = "out is NULL"; return TDB_EINVAL; }
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 20)) { g_create_error = "max_batch must be in [1, 2^20]"; return TDB_EINVAL; }
  tdb_gate_ctx* g = new (std::nothrow) tdb_gate_ctx();
  if (!g) { g_create_error = "out of host memory"; return TDB_ENOMEM; }
  auto al = [&](float** p, size_t count) -> tdb_status {
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(float)) != hipSuccess) { g->err = "hipMalloc failed"; return TDB_ENOMEM; }
    g->dev.push_back(q);
    *p = static_cast<float*>(q);
    return TDB_OK;
  };
  auto run = [&]() -> tdb_status {
    g->max_batch = max_batch;
    TRY(al(&g->P, GATE_NP));
    TRY(al(&g->M, GATE_NP));
    TRY(al(&g->V, GATE_NP));
    TRY(al(&g->G, GATE_NP));
    TRY(al(&g->loss, 4));
    const size_t nh = (size_t)max_batch * GATE_H;
    TRY(al(&g->w.H1, nh));
    TRY(al(&g->w.A1, nh));
    TRY(al(&g->w.H2, nh));
    TRY(al(&g->w.A2, nh));
    TRY(al(&g->w.dH1, nh));
    TRY(al(&g->w.dH2, nh));
    TRY(al(&g->w.y, (size_t)max_batch));
    TRY(al(&g->w.dY, (size_t)max_batch));
    GHIPCHK(hipMemset(g->P, 0, GATE_NP * sizeof(float)));
    GHIPCHK(hipMemset(g->M, 0, GATE_NP * sizeof(float)));
    GHIPCHK(hipMemset(g->V, 0, GATE_NP * sizeof(float)));
    return TDB_OK;
  };
  tdb_status st = run();
  if (st != TDB_OK) {
    g_create_error = g->err;
    delete g;
    return st;
  }
  *out = g;
  return TDB_OK;
}

tdb_status tdb_gate_set_params(tdb_gate g, const float* params_host) {
  if (!g) { g_create_error = "gate is NULL"; return TDB_EINVAL; }
  if (!params_host) { g->err = "params is NULL"; return TDB_EINVAL; }
  GHIPCHK(hipDeviceSynchronize());
  GHIPCHK(hipMemcpy(g->P, params_host, GATE_NP * sizeof(float), hipMemcpyHostToDevice));
  GHIPCHK(hipMemset(g->M, 0, GATE_NP * sizeof(float)));
  GHIPCHK(hipMemset(g->V, 0, GATE_NP * sizeof(float)));
  g->step = 0;
  return TDB_OK;
}

tdb_status tdb_gate_get_params(tdb_gate g, float* params_host) {
  if (!g) { g_create_error = "gate is NULL"; return TDB_EINVAL; }
  if (!params_host) { g->err = "params is NULL"; return TDB_EINVAL; }
  GHIPCHK(hipDeviceSynchronize());
  GHIPCHK(hipMemcpy(params_host, g->P, GATE_NP * sizeof(float), hipMemcpyDeviceToHost));
  return TDB_OK;
}

tdb_status tdb_gate_forward(tdb_gate g, const float* X_dev, int32_t n, float* y_dev, void* stream) {
  if (!g) { g_create_error = "gate is NULL"; return TDB_EINVAL; }
  if (!X_dev || !y_dev || n < 0) { g->err = "bad arguments"; return TDB_EINVAL; }
  GHIPCHK(gate_forward(g->P, X_dev, n, nullptr, nullptr, nullptr, nullptr, y_dev, static_cast<hipStream_t>(stream)));
  return TDB_OK;
}

tdb_status tdb_gate_grad(tdb_gate g, const float* X_dev, const float* t_dev, int32_t n, float* grad_dev,
                         float* loss_host, void* stream) {
  if (!g) { g_create_error = "gate is NULL"; return TDB_EINVAL; }
  if (!X_dev || !t_dev || n < 1 || n > g->max_batch) { g->err = "bad arguments (1 <= n <= max_batch)"; return TDB_EINVAL; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  GHIPCHK(gate_gradient(g->P, X_dev, t_dev, n, g->w, grad_dev ? grad_dev : g->G, loss_host ? g->loss : nullptr, s));
  if (loss_host) {
    GHIPCHK(hipMemcpyAsync(loss_host, g->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
  }
  return TDB_OK;
}

tdb_status tdb_gate_train_step(tdb_gate g, const float* X_dev, const float* t_dev, int32_t n, float lr,
                               float* loss_host, void* stream) {
  if (!g) { g_create_error = "gate is NULL"; return TDB_EINVAL; }
  if (!X_dev || !t_dev || n < 1 || n > g->max_batch || !(lr > 0.0f)) { g->err = "bad arguments"; return TDB_EINVAL; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  GHIPCHK(gate_gradient(g->P, X_dev, t_dev, n, g->w, g->G, loss_host ? g->loss : nullptr, s));
  g->step += 1;
  GHIPCHK(gate_adam(g->P, g->G, g->M, g->V, g->step, lr, s));
  if (loss_host) {
    GHIPCHK(hipMemcpyAsync(loss_host, g->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
  }
  return TDB_OK;
}

void tdb_gate_destroy(tdb_gate g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  delete g;
}

const char* tdb_gate_last_error(tdb_gate g) {
  if (!g) return g_create_error.c_str();
  return g->err.c_str();
}

tdb_status tdb_batch_gate_attach(tdb_batch b, tdb_gate g, const float* feat_mean_std_host, int32_t mode) {
  if (!b) { g_create_error = "batch is NULL"; return TDB_EINVAL; }
  if (mode < GATE_OFF || mode > GATE_SHADOW) { b->err = "bad gate mode"; return TDB_EINVAL; }
  if (mode != GATE_OFF && mode != GATE_RECORD && (!g || !feat_mean_std_host)) {
    b->err = "a gate and its feature statistics are needed";
    return TDB_EINVAL;
  }
  {
    const tdb_status r = batch_resolve(b);
    if (r != TDB_OK && r != TDB_ENUMERIC) return r;
  }
  BHIPCHK(hipDeviceSynchronize());
  const size_t n = (size_t)b->n;
  if (!b->d_ghist) {
    TRY(balloc<float>(b, &b->d_gmean, nullptr, GATE_IN));
    TRY(balloc<float>(b, &b->d_gstd, nullptr, GATE_IN));
    TRY(balloc<float>(b, &b->d_ghist, nullptr, n * GATE_W * GATE_ROW));
    TRY(balloc<float>(b, &b->d_gyhat, nullptr, n));
    TRY(balloc<int>(b, &b->d_ghcount, nullptr, n));
    TRY(balloc<int>(b, &b->d_gskip, nullptr, n));
    TRY(balloc<int>(b, &b->d_gwould, nullptr, n));
  }
  std::vector<float> ms(2 * GATE_IN, 0.0f);
  for (int i = 0; i < GATE_IN; ++i) ms[GATE_IN + i] = 1.0f;
  if (feat_mean_std_host) {
    for (int i = 0; i < 2 * GATE_IN; ++i) ms[i] = feat_mean_std_host[i];
    for (int i = 0; i < GATE_IN; ++i)
      if (!(ms[GATE_IN + i] > 0.0f)) { b->err = "feature standard deviations must be positive"; return TDB_EINVAL; }
  }
  BHIPCHK(hipMemcpy(b->d_gmean, ms.data(), GATE_IN * sizeof(float), hipMemcpyHostToDevice));
  BHIPCHK(hipMemcpy(b->d_gstd, ms.data() + GATE_IN, GATE_IN * sizeof(float), hipMemcpyHostToDevice));
  BHIPCHK(hipMemset(b->d_ghcount, 0, n * sizeof(int)));
  BHIPCHK(hipMemset(b->d_gskip, 0, n * sizeof(int)));
  BHIPCHK(hipMemset(b->d_gwould, 0, n * sizeof(int)));
  // RECORD without a network only keeps the singular values every step
  b->gate_params = g ? g->P : nullptr;
  b->gate_mode = (mode == GATE_RECORD && !g) ? GATE_OFF : mode;
  for (tdb_ctx* h : b->st) h->sigma_every_step = mode != GATE_OFF;
  b->dirty = true;
  return TDB_OK;
}

tdb_status tdb_gate_load(tdb_handle h, const float* params_host, const float* feat_mean_std_host, int32_t n_params,
                         int32_t mode) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
  if (h->batch_owned) { h->err = "this stream belongs to a batch: use tdb_batch_gate_attach"; return TDB_ESTATE; }
  if (mode < GATE_OFF || mode > GATE_SHADOW) { h->err = "bad gate mode"; return TDB_EINVAL; }
  const bool net = mode == GATE_ACTIVE || mode == GATE_SHADOW;
  if (mode != GATE_OFF && !h->fused) {
    h->err = "the learned gate runs on the fused third-order path only";
    return TDB_EUNSUPPORTED;
  }
  if (net && (!params_host || !feat_mean_std_host || n_params != GATE_NP)) {
    h->err = "active and shadow modes need TDB_GATE_PARAMS parameters and 768 feature statistics";
    return TDB_EINVAL;
  }
  TRY(resolve_pending(h));
  HIPCHK(hipDeviceSynchronize());
  if (!h->g_params) {
    TRY(dallocT(h, &h->g_params, (size_t)GATE_NP));
    TRY(dallocT(h, &h->g_mean, (size_t)GATE_IN));
    TRY(dallocT(h, &h->g_std, (size_t)GATE_IN));
    TRY(dallocT(h, &h->g_hist, (size_t)GATE_W * GATE_ROW));
    TRY(dallocT(h, &h->g_yhat, 1));
    TRY(dallocT(h, &h->g_hcount, 1));
    TRY(dallocT(h, &h->g_skip, 1));
    TRY(dallocT(h, &h->g_would, 1));
    TRY(dallocT(h, &h->g_ctab, 1));
    HIPCHK(hipMemcpy(h->g_ctab, &h->ctrl, sizeof(CtrlState*), hipMemcpyHostToDevice));
  }
  if (net) {
    for (int i = 0; i < GATE_NP; ++i)
      if (!std::isfinite(params_host[i])) { h->err = "non-finite gate parameter"; return TDB_EINVAL; }
    for (int i = 0; i < GATE_IN; ++i)
      if (!(feat_mean_std_host[GATE_IN + i] > 0.0f) || !std::isfinite(feat_mean_std_host[i])) {
        h->err = "feature means must be finite and standard deviations positive";
        return TDB_EINVAL;
      }
    HIPCHK(hipMemcpy(h->g_params, params_host, GATE_NP * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->g_mean, feat_mean_std_host, GATE_IN * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->g_std, feat_mean_std_host + GATE_IN, GATE_IN * sizeof(float), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemset(h->g_hcount, 0, sizeof(int)));
  HIPCHK(hipMemset(h->g_skip, 0, sizeof(int)));
  HIPCHK(hipMemset(h->g_would, 0, sizeof(int)));
  // RECORD keeps the singular values every step (for training histories), no network
  h->gate_mode = mode == GATE_RECORD ? GATE_OFF : mode;
  h->sigma_every_step = mode != GATE_OFF;
  return TDB_OK;
}

static_assert(NOALLOC_SCRATCH_DOUBLES == TDB_NOALLOC_SCRATCH, "scratch size of the header and the library");

tdb_status tdb_reconstruct_noalloc(int32_t order, const int64_t* dims, const int32_t* ranks, const double* C_dev,
                                   const double* const* U_dev, int32_t data_dtype, void* out_dev, void* stream) {
  // (messages are set on failure only: a successful call allocates nothing at all)
  if (order < 2 || order > TDB_P) { g_create_error = "order must be 2..4"; return TDB_EINVAL; }
  if (!dims || !ranks || !C_dev || !U_dev || !out_dev) { g_create_error = "NULL argument"; return TDB_EINVAL; }
  if (data_dtype != TDB_F64 && data_dtype != TDB_F32) { g_create_error = "bad data_dtype"; return TDB_EINVAL; }
  long long d[TDB_P] = {1, 1, 1, 1};
  int r[TDB_P] = {1, 1, 1, 1};
  double S = 1.0;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || ranks[n] < 1 || ranks[n] > dims[n] || !U_dev[n]) {
      g_create_error = "need 1 <= ranks[n] <= dims[n] and a basis for every mode";
      return TDB_EINVAL;
    }
    d[n] = dims[n];
    r[n] = ranks[n];
    S *= (double)dims[n];
  }
  if (S > 9.0e15) { g_create_error = "tensor too large"; return TDB_EINVAL; }
  const NoallocPlan pl = noalloc_plan(order, d, r);
  if (pl.max_inter > NOALLOC_SCRATCH_DOUBLES / 2) {
    g_create_error = "an intermediate of the product chain exceeds the fixed scratch (TDB_NOALLOC_SCRATCH / 2 doubles)";
    return TDB_EINVAL;
  }
  const hipError_t e = noalloc_reconstruct(pl, d, r, C_dev, U_dev, data_dtype == TDB_F32 ? 1 : 0, out_dev,
                                           static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g_create_error = std::string("tdb_reconstruct_noalloc: ") + hipGetErrorString(e);
    return TDB_EHIP;
  }
  return TDB_OK;
}

void tdb_struct_sizes(int64_t* config_bytes, int64_t* stats_bytes) {
  if (config_bytes) *config_bytes = (int64_t)sizeof(tdb_config);
  if (stats_bytes) *stats_bytes = (int64_t)sizeof(tdb_stats);
}

const char* tdb_last_error(tdb_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
