// Host runtime and C ABI of the TDB compressor: validates configurations, owns the
// device workspace, sequences the kernels of one snapshot step and of the HOSVD
// (re)initialisation, and keeps the per-step statistics.
#include "../../include/tdb.h"
#include "tdb_kernels.h"
#include "fused.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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
  bool f32 = false;          // bulk passes in FP32
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
  double *err_part = nullptr;
  int err_blocks = 1024;
  CtrlState* ctrl = nullptr;
  CtrlState* ctrl_h = nullptr;   // pinned mirror
  // HOSVD workspace
  double *G[TDB_P] = {}, *gpart = nullptr, *eigw[TDB_P] = {}, *sig[TDB_P] = {};
  double *Umax[TDB_P] = {}, *Bmax[TDB_P] = {}, *Cmax = nullptr, *hsA = nullptr, *hsB = nullptr;
  double *wa[TDB_P] = {}, *wb[TDB_P] = {}, *nu2h = nullptr;
  double *Psi[TDB_P] = {};
  // snapshots
  const void* Vprev = nullptr;
  void* Vcopy = nullptr;
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
  double *Rq[TDB_P] = {}, *Cdot2 = nullptr;
  void* P2[TDB_P] = {};          // pseudo-inverses of the stage-2 core
  void *E = nullptr, *U1c = nullptr;
  double *w23 = nullptr, *ferr_part = nullptr;
  unsigned* counters = nullptr;
  int ferr_gx = 1, ferr_gy = 1;
  long long fused_steps = 0, plain_steps = 0;
  // optional pass timing (events recorded on the caller's stream)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[2];

  ~tdb_ctx() {
    for (auto& v : ev_used)
      for (auto& e : v) { ev_pool.push_back(e.first); ev_pool.push_back(e.second); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* q : allocs) (void)hipFree(q);
    if (ctrl_h) (void)hipHostFree(ctrl_h);
  }
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
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
  if (c->order > TDB_P) { msg = "this build supports tensor order 2..4"; return TDB_EUNSUPPORTED; }
  for (int n = 0; n < c->order; ++n) {
    if (c->dims[n] < 1) { msg = "dims must be positive"; return TDB_EINVAL; }
    if (c->rank_max[n] < 1) { msg = "rank_max must be positive"; return TDB_EINVAL; }
    if (c->rank_max[n] > TDB_RCAP && c->rank_max[n] < c->dims[n]) {
      msg = "rank_max above 64 is not supported by this build";
      return TDB_EUNSUPPORTED;
    }
    if (c->dims[n] > TDB_NEIG) { msg = "mode sizes above 512 are not supported by this build"; return TDB_EUNSUPPORTED; }
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
  if (c->precision != TDB_PREC_F64 && c->precision != TDB_PREC_F32) { msg = "bad precision"; return TDB_EINVAL; }
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
  return TDB_OK;
}

long long prod_ll(const int* a, int p, int skip = -1) {
  long long q = 1;
  for (int k = 0; k < p; ++k)
    if (k != skip) q *= a[k];
  return q;
}

struct PassPlan {
  int T1 = 1, T2 = 1, nt1 = 1, nt2 = 1, stage_p = 0;
  long long slot = 0;
  size_t lds = 0;
  bool ok = false;
};

// Tile shape of the fused stage pass for ranks r: about `target` elements per tile,
// shrunk until its LDS footprint fits.
PassPlan plan_pass(const tdb_ctx* h, const int* r) {
  PassPlan pl;
  const long long N1 = h->N[0], N2 = h->N[1], N3 = h->N[2];
  const int r1 = r[0], r2 = r[1], r3 = r[2];
  const bool f3 = r3 < N3;
  const size_t te = h->celt;
  long long target = h->f32 ? 4096 : 2048;
  if (const char* env = std::getenv("TDB_PASS_TILE")) {
    const long long v = std::atoll(env);
    if (v >= 64 && v <= (1 << 20)) target = v;
  }
  int T2 = (int)std::min<long long>(N2, 64);
  int T1 = (int)std::max<long long>(1, std::min<long long>(N1, target / std::max<long long>(1, T2 * N3)));
  auto lds_of = [&](int t1, int t2) {
    long long e = (long long)t1 * t2 * N3 + (long long)t1 * t2 * r3 + (long long)t1 * r2 * r3 +
                  (long long)r1 * t2 * r3 + 2LL * t1 * r1 + 2LL * t2 * r2 + 2LL * N3 * r3;
    if (f3) e += (long long)t1 * r2 * N3 + (long long)r1 * r2 * N3;
    return (size_t)e * te;
  };
  while (lds_of(T1, T2) > (size_t)h->lds_max && T1 > 1) T1 = std::max(1, T1 / 2);
  while (lds_of(T1, T2) > (size_t)h->lds_max && T2 > 8) T2 = std::max(8, T2 / 2);
  if (lds_of(T1, T2) > (size_t)h->lds_max) return pl;
  // stage the pseudo-inverses too when they fit
  const long long pe = (r1 < N1 ? (long long)r1 * r2 * r3 : 0) + (r2 < N2 ? (long long)r1 * r2 * r3 : 0) +
                       (f3 ? (long long)r1 * r2 * r3 : 0);
  if (lds_of(T1, T2) + (size_t)pe * te <= (size_t)h->lds_max) pl.stage_p = 1;
  pl.T1 = T1;
  pl.T2 = T2;
  pl.nt1 = (int)((N1 + T1 - 1) / T1);
  pl.nt2 = (int)((N2 + T2 - 1) / T2);
  pl.slot = (long long)T1 * r1 + (long long)T2 * r2 + N3 * r3 + (long long)r1 * r2 * r3;
  pl.lds = lds_of(T1, T2) + (pl.stage_p ? (size_t)pe * te : 0);
  pl.ok = true;
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
  h->f32 = cfg->precision == TDB_PREC_F32;
  h->data32 = cfg->data_dtype == TDB_F32;
  h->celt = h->f32 ? 4 : 8;
  h->delt = h->data32 ? 4 : 8;
  h->core_cap = prod_ll(h->caps, h->p);
  h->Rmax = 1;
  for (int n = 0; n < h->p; ++n) h->Rmax = std::max(h->Rmax, prod_ll(h->caps, h->p, n));

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
  TRY(dallocT(h, &h->err_part, 2 * (size_t)h->err_blocks));
  TRY(dalloc(h, reinterpret_cast<void**>(&h->ctrl), sizeof(CtrlState)));
  {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->ctrl_h), sizeof(CtrlState), hipHostMallocDefault);
    if (e != hipSuccess) { h->err = "hipHostMalloc failed"; return TDB_ENOMEM; }
  }
  // ---- HOSVD buffers
  size_t gpart = 0;
  for (int n = 0; n < h->p; ++n) {
    TRY(dallocT(h, &h->G[n], (size_t)h->N[n] * h->N[n]));
    TRY(dallocT(h, &h->eigw[n], (size_t)h->N[n] * (h->caps[n] + 4)));
    TRY(dallocT(h, &h->sig[n], (size_t)h->caps[n] + 1));
    TRY(dallocT(h, &h->Umax[n], (size_t)h->N[n] * h->ldU[n]));
    TRY(dallocT(h, &h->Bmax[n], (size_t)h->N[n] * h->caps[n]));
    const long long nt = (h->N[n] + 63) / 64;
    const long long K = h->S / h->N[n];
    const long long nch = std::max<long long>(1, std::min<long long>(64, (K + 4095) / 4096));
    gpart = std::max(gpart, (size_t)(nt * (nt + 1) / 2 * nch * 4096));
  }
  TRY(dallocT(h, &h->gpart, gpart));
  TRY(dallocT(h, &h->Cmax, h->core_cap));
  TRY(dallocT(h, &h->hsA, (size_t)h->S));
  TRY(dallocT(h, &h->hsB, (size_t)h->S));
  TRY(dallocT(h, &h->nu2h, 1));
  if (cfg->snapshot_mode == TDB_COPY) TRY(dalloc(h, &h->Vcopy, (size_t)h->S * h->delt));

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
  // partial buffer: enough for the ranks-1 plan and the caps plan
  int ones[3] = {1, 1, 1};
  PassPlan p1 = plan_pass(h, ones), pc = plan_pass(h, h->caps);
  long long tiles = std::max<long long>(p1.ok ? (long long)p1.nt1 * p1.nt2 : 1, pc.ok ? (long long)pc.nt1 * pc.nt2 : 1);
  long long slot = pc.ok ? pc.slot : (p1.ok ? p1.slot : 1);
  long long capslot = (long long)h->caps[0] * h->caps[1] * h->caps[2] + 3LL * 64 * 64 + 64 * (h->N[0] + h->N[1] + h->N[2]);
  slot = std::max(slot, std::min(capslot, slot * 4));
  h->fpart_elems = tiles * slot;
  TRY(dalloc(h, &h->fpart, (size_t)h->fpart_elems * h->celt));
  for (int n = 0; n < 3; ++n) {
    TRY(dallocT(h, &h->Rq[n], (size_t)TDB_RCAP * TDB_RCAP));
    TRY(dalloc(h, &h->P2[n], (size_t)h->Rmax * h->caps[n] * h->celt));
  }
  TRY(dallocT(h, &h->Cdot2, h->core_cap));
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
  TRY(dallocT(h, &h->ferr_part, 2 * (size_t)h->ferr_gx * h->ferr_gy));
  TRY(dalloc(h, reinterpret_cast<void**>(&h->counters), 4 * sizeof(unsigned)));
  HIPCHK(hipMemset(h->counters, 0, 4 * sizeof(unsigned)));
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
  for (int n = 0; n < p; ++n) {
    std::vector<int> order;
    for (int k = 0; k < p; ++k)
      if (k != n) order.push_back(k);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const double rx = (double)h->N[x] / h->r[x], ry = (double)h->N[y] / h->r[y];
      return rx != ry ? rx > ry : x < y;
    });
    long long cd[TDB_P];
    for (int k = 0; k < p; ++k) cd[k] = h->N[k];
    T* bufs[2] = {static_cast<T*>(h->wsA), static_cast<T*>(h->wsB)};
    int cur = -1;
    for (size_t q = 0; q < order.size(); ++q) {
      const int k = order[q];
      long long A = 1, Bz = 1;
      for (int j = 0; j < k; ++j) A *= cd[j];
      for (int j = k + 1; j < p; ++j) Bz *= cd[j];
      T* out = bufs[cur == 0 ? 1 : 0];
      if (q == 0) {
        HIPCHK((launch_ttm<TD, T, T>(V1, V0, out, static_cast<const T*>(h->B[k]), h->r[k], 1, A,
                                     (int)cd[k], h->r[k], Bz, s)));
      } else {
        HIPCHK((launch_ttm<T, T, T>(bufs[cur], nullptr, out, static_cast<const T*>(h->B[k]), h->r[k], 1,
                                    A, (int)cd[k], h->r[k], Bz, s)));
      }
      cd[k] = h->r[k];
      cur = (cur == 0) ? 1 : 0;
    }
    const T* F = bufs[cur];
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

// Weighted HOSVD of V at the caps (Sec. 2.3) followed by the rank selection `mode`.
template <typename TD>
tdb_status hosvd_select(tdb_ctx* h, const TD* V, int mode, hipStream_t s) {
  const int p = h->p;
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
    const int nch = (int)std::max<long long>(1, std::min<long long>(64, (K + 4095) / 4096));
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
  HIPCHK(launch_sym_eig(eb, s));
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
    if (!h->prof) return;
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

template <typename TD>
tdb_status keep_previous(tdb_ctx* h, const TD* V, hipStream_t s) {
  if (h->cfg.snapshot_mode == TDB_COPY) {
    HIPCHK(hipMemcpyAsync(h->Vcopy, V, (size_t)h->S * sizeof(TD), hipMemcpyDeviceToDevice, s));
    h->Vprev = h->Vcopy;
  } else {
    h->Vprev = V;
  }
  return TDB_OK;
}

template <typename TD, typename T>
tdb_status ingest_impl(tdb_ctx* h, const TD* V1, hipStream_t s) {
  const TD* V0 = static_cast<const TD*>(h->Vprev);
  const int p = h->p;
  RhsArgs ra{};
  ra.p = p;
  ra.dt = h->cfg.dt;
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
    TRY((project_plain<TD, T>(h, V1, V0, s)));
  }
  ra.stage = 1;
  HIPCHK(launch_rhs_stage(ra, h->ctrl, s));
  // stage 2 at S*
  TRY(stage_prep<T>(h, h->Cs, h->Us, s));
  {
    PassTimer pt(h, TDB_PASS_PROJECT, s);
    TRY((project_plain<TD, T>(h, V1, V0, s)));
  }
  ra.stage = 2;
  HIPCHK(launch_rhs_stage(ra, h->ctrl, s));
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
  h->step += 1;
  h->t_now = h->step * h->cfg.dt;
  const int dec = h->ctrl_h->decision;
  if (dec != DEC_NONE) {
    TRY(hosvd_select<TD>(h, V1, dec, s));
    TRY(pull_ctrl(h, s));
    TRY(core_sigma(h, false, s));
    TRY(pull_ctrl(h, s));
  }
  TRY(keep_previous<TD>(h, V1, s));
  fill_stats(h, false);
  return TDB_OK;
}

int max_rank(const tdb_ctx* h) {
  int m = 1;
  for (int n = 0; n < h->p; ++n) m = std::max(m, h->r[n]);
  return m;
}

size_t small_lds(const tdb_ctx* h, bool* core_in_lds) {
  const long long csz = prod_ll(h->r, h->p);
  const int rm = max_rank(h);
  long long msum = 0;
  for (int n = 0; n < h->p; ++n) msum += (long long)h->r[n] * h->r[n];
  // finish rows stage C_dot, the three P_n and the three M_n
  long long pel = 0;
  for (int n = 0; n < h->p; ++n) pel += (csz / h->r[n]) * h->r[n];
  const size_t rows = (size_t)csz * 8 + (size_t)pel * h->celt + 8 + (size_t)msum * 8;
  const size_t base = std::max<size_t>((3 * (size_t)rm * rm + 5 * (size_t)rm + 64) * 8, rows);
  *core_in_lds = base + (size_t)csz * 8 <= (size_t)h->lds_max;
  return base + (*core_in_lds ? (size_t)csz * 8 : 0);
}

// Post-step preparation of the fused path at the committed state: core singular
// values, B_n and P_n of the next stage 1, and the error-pass expansion E.
template <typename T>
tdb_status fused_post(tdb_ctx* h, hipStream_t s) {
  FPostArgs pa{};
  bool cil = false;
  size_t lds = small_lds(h, &cil);
  pa.core_in_lds = cil ? 1 : 0;
  pa.want_pinv = 1;
  pa.rmax = max_rank(h);
  const long long etot = (long long)h->r[0] * h->N[1] * h->N[2];
  pa.eblocks = (int)std::max<long long>(1, std::min<long long>(std::min<long long>(256, h->N[1]), (etot + 255) / 256));
  const long long per = (h->N[1] + pa.eblocks - 1) / pa.eblocks;
  const size_t elds = ((size_t)h->r[0] * h->r[1] * h->N[2] + (size_t)per * h->r[1]) * 8;
  if (elds > (size_t)h->lds_max) { h->err = "error-pass expansion does not fit in LDS"; return TDB_EUNSUPPORTED; }
  lds = std::max(lds, elds);
  pa.C = h->C0;
  pa.E = h->E;
  pa.U1c = h->U1c;
  for (int n = 0; n < 3; ++n) {
    pa.N[n] = h->N[n];
    pa.r[n] = h->r[n];
    pa.ldU[n] = h->ldU[n];
    pa.U[n] = h->U0[n];
    pa.w[n] = h->w[n];
    pa.B[n] = h->B[n];
    pa.P[n] = h->P[n];
  }
  HIPCHK(launch_fpost<T>(pa, lds, h->ctrl, s));
  h->post_valid = true;
  return TDB_OK;
}

template <typename TD, typename T>
tdb_status ingest_fused(tdb_ctx* h, const TD* V1, hipStream_t s) {
  const TD* V0 = static_cast<const TD*>(h->Vprev);
  const PassPlan pl = plan_pass(h, h->r);
  if (!pl.ok || (long long)pl.nt1 * pl.nt2 * pl.slot > h->fpart_elems) {
    h->post_valid = false;
    h->plain_steps += 1;
    return ingest_impl<TD, T>(h, V1, s);
  }
  h->fused_steps += 1;
  if (!h->post_valid) TRY(fused_post<T>(h, s));
  FPassArgs fa{};
  fa.V1 = V1;
  fa.V0 = V0;
  fa.N1 = (int)h->N[0]; fa.N2 = (int)h->N[1]; fa.N3 = (int)h->N[2];
  fa.r1 = h->r[0]; fa.r2 = h->r[1]; fa.r3 = h->r[2];
  fa.T1 = pl.T1; fa.T2 = pl.T2; fa.nt1 = pl.nt1; fa.nt2 = pl.nt2;
  fa.need_h1 = h->r[0] < h->N[0];
  fa.need_h2 = h->r[1] < h->N[1];
  fa.need_f3 = h->r[2] < h->N[2];
  fa.stage_p = pl.stage_p;
  fa.slot = pl.slot;
  fa.B1 = h->B[0]; fa.B2 = h->B[1]; fa.B3 = h->B[2];
  fa.P1 = h->P[0]; fa.P2 = h->P[1]; fa.P3 = h->P[2];
  fa.part = h->fpart;
  FReduceArgs ra{};
  ra.dt = h->cfg.dt;
  ra.N1 = fa.N1; ra.N2 = fa.N2; ra.N3 = fa.N3; ra.r1 = fa.r1; ra.r2 = fa.r2; ra.r3 = fa.r3;
  ra.T1 = pl.T1; ra.T2 = pl.T2; ra.nt1 = pl.nt1; ra.nt2 = pl.nt2;
  ra.need_h1 = fa.need_h1; ra.need_h2 = fa.need_h2; ra.need_f3 = fa.need_f3;
  ra.slot = pl.slot;
  ra.part = h->fpart;
  ra.C0 = h->C0; ra.Cs = h->Cs; ra.kC = h->kC; ra.Cdot2 = h->Cdot2;
  FFinishArgs ga{};
  bool cil = false;
  const size_t slds = small_lds(h, &cil);
  ga.core_in_lds = cil ? 1 : 0;
  ga.rmax = max_rank(h);
  ga.dt = h->cfg.dt;
  long long rows = 0;
  for (int n = 0; n < 3; ++n) rows += h->N[n] * h->r[n];
  ga.rowblocks = (int)std::max<long long>(1, std::min<long long>(1024, (rows + 255) / 256));
  ga.Cs = h->Cs;
  ga.kC = h->kC;
  ga.Cdot2 = h->Cdot2;
  for (int n = 0; n < 3; ++n) {
    ra.H[n] = h->H[n];
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
  }
  for (int stage = 1; stage <= 2; ++stage) {
    void* const* Pst = stage == 1 ? h->P : h->P2;
    fa.P1 = Pst[0]; fa.P2 = Pst[1]; fa.P3 = Pst[2];
    for (int n = 0; n < 3; ++n) ga.Pcur[n] = Pst[n];
    {
      PassTimer pt(h, TDB_PASS_PROJECT, s, true);
      HIPCHK((launch_fpass<TD, T>(fa, pl.lds, s, pt.start(), pt.stop())));
    }
    ra.stage = stage;
    HIPCHK(launch_freduce<T>(ra, h->ctrl, s));
    ga.stage = stage;
    HIPCHK(launch_ffinish<T>(ga, slds, h->ctrl, s));
  }
  FQrArgs qa{};
  qa.rmax = max_rank(h);
  qa.rounds = 1;
  const size_t npq = (size_t)qa.rmax * (qa.rmax + 1) / 2;
  size_t qlds = (4 * (size_t)qa.rmax * qa.rmax + 4 * npq + TDB_NEIG) * 8;
  size_t ustage = 0;
  for (int n = 0; n < 3; ++n) {
    const size_t need = (size_t)h->N[n] * h->r[n] * 8;
    qa.u_in_lds[n] = qlds + need <= (size_t)h->lds_max ? 1 : 0;
    if (qa.u_in_lds[n]) ustage = std::max(ustage, need);
    qa.N[n] = h->N[n];
    qa.r[n] = h->r[n];
    qa.ldU[n] = h->ldU[n];
    qa.U0[n] = h->U0[n];
    qa.w[n] = h->w[n];
    qa.Rq[n] = h->Rq[n];
  }
  const size_t cneed = 2 * (size_t)prod_ll(h->r, 3) * 8;
  qa.core_in_lds = qlds + cneed <= (size_t)h->lds_max ? 1 : 0;
  if (qa.core_in_lds) ustage = std::max(ustage, cneed);
  qa.C0 = h->C0;
  qa.Ctmp = h->Ctmp;
  qa.counter = h->counters;
  HIPCHK(launch_fqr(qa, qlds + ustage, h->ctrl, s));
  TRY(fused_post<T>(h, s));
  FErrArgs ea{};
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
  ea.counter = h->counters + 1;
  {
    PassTimer pt(h, TDB_PASS_ERROR, s, true);
    HIPCHK((launch_ferr<TD, T>(ea, h->ctrl, s, pt.start(), pt.stop())));
  }
  TRY(pull_ctrl(h, s));
  h->step += 1;
  h->t_now = h->step * h->cfg.dt;
  const int dec = h->ctrl_h->decision;
  if (dec != DEC_NONE) {
    TRY(hosvd_select<TD>(h, V1, dec, s));
    TRY(pull_ctrl(h, s));
    TRY(fused_post<T>(h, s));
    TRY(pull_ctrl(h, s));
  }
  TRY(keep_previous<TD>(h, V1, s));
  fill_stats(h, false);
  return TDB_OK;
}

template <typename TD>
tdb_status ingest_dispatch(tdb_ctx* h, const void* V, hipStream_t s) {
  if (h->fused) {
    if (h->f32) return ingest_fused<TD, float>(h, static_cast<const TD*>(V), s);
    return ingest_fused<TD, double>(h, static_cast<const TD*>(V), s);
  }
  if (h->f32) return ingest_impl<TD, float>(h, static_cast<const TD*>(V), s);
  return ingest_impl<TD, double>(h, static_cast<const TD*>(V), s);
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
    if (h->data32) TRY(hosvd_select<float>(h, static_cast<const float*>(V0_dev), DEC_INIT, s));
    else TRY(hosvd_select<double>(h, static_cast<const double*>(V0_dev), DEC_INIT, s));
    TRY(pull_ctrl(h, s));
    TRY(core_sigma(h, false, s));
    TRY(pull_ctrl(h, s));
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
    for (int n = 0; n < h->p; ++n) {
      if (ranks[n] < 1 || ranks[n] > h->caps[n] || !U_host[n]) {
        h->err = "ranks must be in [1, cap] with a basis for every mode";
        return TDB_EINVAL;
      }
      h->r[n] = ranks[n];
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
    h->ctrl_h->eps = std::sqrt(std::max(h->ctrl_h->eps2, 0.0));
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
  hipStream_t s = static_cast<hipStream_t>(stream);
  tdb_status st = h->data32 ? ingest_dispatch<float>(h, V_dev, s) : ingest_dispatch<double>(h, V_dev, s);
  if (st == TDB_OK && !std::isfinite(h->stats.eps)) {
    h->err = "non-finite reconstruction error (NaN or Inf in the snapshot?)";
    return TDB_ENUMERIC;
  }
  return st;
}

tdb_status tdb_get_core_and_bases(tdb_handle h, int32_t rotate, int32_t* ranks_out, double* C_host,
                                  double* const* U_host) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  if (!h->ready) { h->err = "handle is not initialised"; return TDB_ESTATE; }
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
  *out = h->stats;
  return TDB_OK;
}

void tdb_destroy(tdb_handle h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

tdb_status tdb_profile_enable(tdb_handle h, int32_t on) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
  HIPCHK(hipDeviceSynchronize());
  for (auto& v : h->ev_used) {
    for (auto& e : v) { h->ev_pool.push_back(e.first); h->ev_pool.push_back(e.second); }
    v.clear();
  }
  h->prof = on != 0;
  return TDB_OK;
}

tdb_status tdb_profile_read(tdb_handle h, int32_t pass, int64_t* launches, double* total_ms,
                            double* bytes_per_launch) {
  if (!h) { g_create_error = "handle is NULL"; return TDB_EINVAL; }
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

void tdb_struct_sizes(int64_t* config_bytes, int64_t* stats_bytes) {
  if (config_bytes) *config_bytes = (int64_t)sizeof(tdb_config);
  if (stats_bytes) *stats_bytes = (int64_t)sizeof(tdb_stats);
}

const char* tdb_last_error(tdb_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
