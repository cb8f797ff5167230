/*
 * tdb.h -- C ABI of the MI355X (gfx950) in situ compressor built on time-dependent
 * bases (TDB): each streaming snapshot tensor V(t) of order p is kept as a core
 * tensor C(t) times one orthonormal basis U_n(t) per mode, and advanced snapshot by
 * snapshot with the paper's closed-form evolution equations.
 *
 * Paper: Zamani Ashtiani, Malik, Babaee, "Scalable In Situ Compression of Transient
 * Simulation Data Using Time-Dependent Bases" (arXiv 2201.06958).
 *   - problem statement: streaming multidimensional data, modes as groups of
 *     variables, weighted inner products (Sec. 2.1, eq. (inner));
 *   - the decomposition into core and bases (Sec. 2.2, eq. (reconstructed));
 *   - discrete space-time form, quadrature weights, finite-difference derivative,
 *     HOSVD initialisation (Sec. 2.3);
 *   - error control and mode addition/removal (Sec. 2.5, eqs. (error), (percentage));
 *   - storage of core and bases, compression ratio (Sec. 2.6).
 *
 * Conventions for every entry point:
 *   - Return value: TDB_OK (0) or a positive tdb_status error code. No exception or
 *     abort crosses the ABI; tdb_last_error() gives a message for the last failure
 *     on a handle (or, for a NULL handle, for the last failed create call).
 *   - Device pointers ("_dev") are HIP device addresses on the current device;
 *     host pointers ("_host") are ordinary host memory and are copied before return.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work is
 *     enqueued on it; calls that return host data synchronise it.
 *   - Snapshots are dense C-contiguous tensors over (N_1, ..., N_p) in the
 *     configured storage type (mode p has unit stride).
 *   - A handle is not re-entrant: use one handle from one host thread at a time.
 */
#ifndef TDB_H
#define TDB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tdb_status;
enum {
  TDB_OK = 0,
  TDB_EINVAL = 1,        /* bad argument or configuration                         */
  TDB_ENOMEM = 2,        /* device or host allocation failed                      */
  TDB_EHIP = 3,          /* a HIP runtime call failed                             */
  TDB_ESTATE = 4,        /* call out of order (e.g. ingest before init)           */
  TDB_ENUMERIC = 5,      /* non-finite data, or an unrecoverable singular core    */
  TDB_EUNSUPPORTED = 6   /* a valid request the library does not implement        */
};

enum { TDB_F64 = 0, TDB_F32 = 1 };                      /* snapshot storage type  */
enum { TDB_PREC_F64 = 0, TDB_PREC_F32 = 1, TDB_PREC_BF16SPLIT = 2 };  /* bulk-pass arithmetic */
enum { TDB_PATH_AUTO = 0, TDB_PATH_PLAIN = 1, TDB_PATH_FUSED = 2 };
enum { TDB_COPY = 0, TDB_BORROW = 1 };                  /* previous-snapshot mode */
enum {                                                   /* controller events      */
  TDB_EV_NONE = 0, TDB_EV_REINIT = 1, TDB_EV_ADD = 2, TDB_EV_REMOVE = 3, TDB_EV_NUMERIC = 4
};

#define TDB_MAX_ORDER 8       /* ABI array size; the library supports 2 <= p <= 4 */
#define TDB_SIGMA_K 16        /* leading core singular values reported per mode    */

typedef struct tdb_ctx* tdb_handle;

/* Configuration of one stream (Sec. 2.3, 2.5). Copied at init.
 *
 * Order 2 with a short second mode (dims[1] <= 32, dims[0] >= dims[1], path AUTO or
 * FUSED) is the DBO form of Sec. 2.2 and TDB-2 of Sec. 3.2: a snapshot is the
 * dims[0] x dims[1] row-major matrix, e.g. a field (x1, x2, variables) with x1 and x2
 * grouped into the first mode (weights the product of the two axes' weights). Such a
 * stream steps on row passes and synchronously; its first mode may exceed 512 entries
 * (its HOSVD basis is then taken from the second mode's eigenvectors). Every other mode
 * of every stream has at most 512 entries. */
typedef struct {
  int32_t order;                       /* p, 2..4 in this library                      */
  int64_t dims[TDB_MAX_ORDER];         /* N_n; a mode may be a flattened group of axes */
  int32_t rank_init[TDB_MAX_ORDER];    /* all 0 => chosen by the rank rule at init     */
  int32_t rank_max[TDB_MAX_ORDER];     /* caps; clamped to N_n and to the product of
                                          the other caps; each <= 64 in this library   */
  const double* weights[TDB_MAX_ORDER];/* host arrays of N_n positive quadrature
                                          weights (diagonal W^(n)); NULL => 1/N_n      */
  double dt;                           /* uniform snapshot spacing, > 0                */
  int32_t data_dtype;                  /* TDB_F64 | TDB_F32                            */
  int32_t precision;                   /* TDB_PREC_F64 | TDB_PREC_F32 |
                                          TDB_PREC_BF16SPLIT (projection and error
                                          passes; the small r x r work and the state
                                          are always FP64). BF16SPLIT: the stage pass
                                          on matrix cores with x = hi + lo in BF16
                                          and the products hi*hi + hi*lo + lo*hi
                                          accumulated in FP32, where the shapes allow
                                          (order 3, N_3 <= 8, r_1, r_2 <= 32), else
                                          as F32 (tdb_stats.precision_used reports
                                          what each step ran); the error pass in FP32 */
  int32_t path;                        /* TDB_PATH_*: AUTO picks FUSED where supported */
  int32_t adaptive;                    /* 0 = fixed ranks (eps is still reported)      */
  int32_t snapshot_mode;               /* TDB_COPY: the library keeps its own copy of
                                          the previous snapshot; TDB_BORROW: the caller
                                          keeps the previous snapshot's buffer intact
                                          until the next ingest has completed          */
  double eps_th;                       /* error threshold on the weighted error eq. (error) */
  double gamma_th;                     /* > 0: percentage budget of eq. (percentage),
                                          (1 - gamma_th/100) ||V||^2; <= 0: (eps_th/2)^2 */
  int32_t slope_window;                /* error-slope window for removal; 0 => 10      */
  int32_t integrator;                  /* TDB_INT_HEUN (0, default): the second-order
                                          Runge-Kutta (Heun) step; TDB_INT_EULER: the
                                          explicit first-order Euler step (Sec. 2.4,
                                          the time-scheme comparison of Sec. 3.1);
                                          single streams only                          */
  int32_t fd_order;                    /* data derivative (Sec. 2.3): 0 or 1, the first-
                                          order quotient (V_{k+1} - V_k)/dt held over
                                          both stages; 2, second-order differences from
                                          V_{k-1}, V_k, V_{k+1}: the central difference
                                          at t_k for the first stage, the one-sided
                                          (3 V_{k+1} - 4 V_k + V_{k-1})/(2 dt) at t_{k+1}
                                          for the second (the first step after init
                                          takes the first-order quotient). 2 keeps two
                                          earlier snapshots (TDB_COPY: two copies;
                                          TDB_BORROW: the caller keeps the last two
                                          snapshots intact), needs two more data-sized
                                          buffers and steps synchronously; single
                                          streams only                                 */
} tdb_config;

#define TDB_INT_HEUN 0
#define TDB_INT_EULER 1

/* Per-step record (Sec. 2.5, 2.6). */
typedef struct {
  int64_t step;                        /* snapshots ingested since init                */
  double t;                            /* step * dt                                    */
  double eps;                          /* ||V - C x_n U_n||_W of the evolved state     */
  double nu;                           /* ||V||_W                                      */
  double eps_after;                    /* error after this step's reinit (NaN if none) */
  int32_t ranks[TDB_MAX_ORDER];        /* ranks held after the step                    */
  int32_t event;                       /* TDB_EV_* taken at this step                  */
  double sigma[4][TDB_SIGMA_K];        /* leading singular values of each core
                                          unfolding after the step (0-padded)          */
  double cr;                           /* compression ratio at the current ranks       */
  double crbar;                        /* time-weighted ratio since init               */
  int32_t n_reinit, n_add, n_remove, n_numeric;
  int32_t gated;                       /* 1: the learned gate skipped the exact error
                                          pass of this step (eps is then NaN)          */
  int32_t would_skip;                  /* the gate's verdict, also when it observes    */
  double eps_pred;                     /* the gate's predicted eps (NaN without one)   */
  int32_t precision_used;              /* TDB_PREC_* the last step's stage pass ran in
                                          (-1 before the first step)                   */
  int32_t path_used;                   /* TDB_PATH_FUSED or TDB_PATH_PLAIN of the last
                                          step (0 before the first step)               */
  int64_t fused_steps, plain_steps;    /* steps taken on each path since init (a fused
                                          stream falls back to the plain path for a step
                                          whose stage pass does not fit the LDS)       */
  int64_t n_nonfinite;                 /* steps not applied for NaN/Inf data           */
  int64_t graph_steps;                 /* batch members: launches of the batch's step
                                          replayed from a HIP graph (0 otherwise)      */
} tdb_stats;

/* Initialise from the first snapshot by a weighted HOSVD (Sec. 2.3). V0_dev: device
 * tensor in data_dtype. Allocates all device workspace (sized by the caps). On
 * success *out owns it; on failure *out is NULL (TDB_ENUMERIC when V0 holds NaN or
 * Inf). */
tdb_status tdb_init(const tdb_config* cfg, const void* V0_dev, void* stream, tdb_handle* out);

/* Initialise from given factors instead of a HOSVD (parity and restart use).
 * ranks[n] gives the core shape; C_host is the C-contiguous r_1 x ... x r_p core;
 * U_host[n] is the row-major N_n x r_n basis, expected W-orthonormal. TDB_ENUMERIC
 * for NaN or Inf in V0 or the factors. A rank-deficient core is accepted: the first
 * step then finds its pseudo-inverse singular (Sec. 2.2) and restarts from a HOSVD
 * of that step's snapshot (event TDB_EV_NUMERIC). */
tdb_status tdb_init_from_factors(const tdb_config* cfg, const void* V0_dev,
                                 const int32_t* ranks, const double* C_host,
                                 const double* const* U_host, void* stream, tdb_handle* out);

/* Advance from t_k to t_{k+1} with snapshot V_dev (Sec. 2.2-2.5): difference quotient,
 * two Heun stages of eqs. (Corecont)/(basecont), W-orthonormal QR with the factor
 * folded into the core, weighted error pass, controller (and HOSVD reinit when it
 * fires).
 * Non-finite data: when the difference quotient holds NaN or Inf (the first stage's
 * core derivative is then not finite, which the device checks), the step is not
 * applied: core, bases, ranks, step count and statistics stay those of the last
 * finite step and TDB_ENUMERIC is returned (by the call that reads the step, see
 * below). The snapshot still becomes the previous snapshot, so the next step's
 * difference quotient is also non-finite and is not applied either; the stream goes
 * on from the snapshot after that.
 * With TDB_COPY snapshots it returns after one small read-back of the controller
 * result, so the step is complete. With TDB_BORROW snapshots on the fused third-order
 * path the call is pipelined: it enqueues this step on `stream`, then reads the
 * previous step's decision and acts on it (a reinitialisation, with the previous
 * snapshot, which the caller keeps until this call returns; this step is then enqueued
 * again), so the device never waits for the host between steps. The newest step's
 * decision is read by the next ingest or by any call that returns results
 * (tdb_get_stats, tdb_get_core_and_bases, tdb_reconstruct, tdb_set_threshold,
 * tdb_profile_*) or tdb_flush; TDB_ENUMERIC for a non-finite error is reported by the
 * call that reads it. Reads of V_dev are ordered on `stream`: overwrite it only in
 * work ordered after the next call's. Setting TDB_PIPELINE=0 in the environment
 * turns the pipelining off. */
tdb_status tdb_ingest_snapshot(tdb_handle h, const void* V_dev, void* stream);

/* One step with a given data derivative (Sec. 2.3, and the exact-derivative runs of
 * the time-scheme study, Sec. 3.1): as tdb_ingest_snapshot with snapshot V_dev at
 * t_{k+1}, except that the stage projections use D_dev (same shape, dtype and layout
 * as a snapshot; the derivative of the data, held over the step's stages as the
 * difference quotient is) instead of (V_{k+1} - V_k)/dt. V_dev still serves the
 * weighted error and becomes the previous snapshot of the next difference quotient.
 * The step runs synchronously (any pipelined step is resolved first): D_dev is read
 * by this call only. TDB_EINVAL for NULL pointers; TDB_ENUMERIC, with nothing
 * changed, when V_dev or D_dev holds NaN or Inf; otherwise as tdb_ingest_snapshot. */
tdb_status tdb_ingest_with_derivative(tdb_handle h, const void* V_dev, const void* D_dev, void* stream);

/* Read the newest enqueued step's decision and act on it (see tdb_ingest_snapshot);
 * afterwards every step is complete and the statistics are those of the last one.
 * No effect when nothing is pending. TDB_ENUMERIC if that step was not applied for
 * non-finite data. */
tdb_status tdb_flush(tdb_handle h);

/* Copy the current ranks, core and bases to the host. ranks_out: TDB_MAX_ORDER ints
 * (may be NULL). C_host (prod r_n doubles) and U_host[n] (N_n x r_n row-major) may
 * be NULL to skip. rotate != 0 applies the energetic rotation eq. (rot) first. */
tdb_status tdb_get_core_and_bases(tdb_handle h, int32_t rotate, int32_t* ranks_out,
                                  double* C_host, double* const* U_host);

/* Write the dense reconstruction of eq. (reconstructed) (Sec. 2.2), the Tucker product
 * C x_1 U_1 ... x_p U_p, into out_dev: S values in data_dtype, C-contiguous over
 * (N_1, ..., N_p), caller-owned device memory. Enqueued on `stream` after any
 * pending step is resolved. TDB_EINVAL for a NULL out_dev. */
tdb_status tdb_reconstruct(tdb_handle h, void* out_dev, void* stream);

/* Change the error threshold eps_th of eq. (error) and the captured-energy
 * percentage gamma_th of eq. (percentage) (Sec. 2.5: mode addition when the error
 * exceeds eps_th, removal and rank choice within the budget); gamma_th <= 0 uses
 * the budget (eps_th/2)^2. Applies from the next ingest; a stream in the state
 * where the caps cannot meet the threshold keeps its raised trigger until a
 * reinitialisation meets it. TDB_EINVAL unless eps_th > 0 and gamma_th < 100. */
tdb_status tdb_set_threshold(tdb_handle h, double eps_th, double gamma_th);

/* Statistics of the last applied step (or of init) into *out: the weighted error
 * eq. (error) and ||V||_W (Sec. 2.5), the ranks and event, the leading singular values
 * of the core unfoldings (Sec. 2.4, the diagonal of eq. (rot)), the compression ratio
 * CR and its time-weighted mean (Sec. 2.6), event counts, the gate's fields and the
 * path and precision the last step ran in. Resolves a pending step first. */
tdb_status tdb_get_stats(tdb_handle h, tdb_stats* out);

/* Free everything the handle owns. NULL-safe. */
void tdb_destroy(tdb_handle h);

/* Kernel timing for measurement tools. While enabled, the library brackets the
 * launches of a bulk pass with a pair of HIP events recorded on the caller's stream:
 * TDB_PASS_PROJECT is one Heun stage's projection of the data difference (two per
 * snapshot), TDB_PASS_ERROR is the weighted error pass (one per snapshot). on = 0
 * turns timing off, on = 1 times every launch, on = k > 1 times the passes of every
 * k-th step only (the events themselves cost time on the stream; the averages are
 * over the timed launches). Enabling clears the counters. tdb_profile_read
 * synchronises the recorded events and returns the number of timed launches, their
 * summed duration in milliseconds and the algorithmic bytes one launch must read
 * (snapshot bytes it streams). */
enum { TDB_PASS_PROJECT = 0, TDB_PASS_ERROR = 1 };
tdb_status tdb_profile_enable(tdb_handle h, int32_t on);
tdb_status tdb_profile_read(tdb_handle h, int32_t pass, int64_t* launches, double* total_ms,
                            double* bytes_per_launch);

/* ---- Many independent streams in one set of launches.
 * Each stream is its own TDB of a third-order tensor (Sec. 2; the stochastic flow of
 * Sec. 3.3 has one field per sample, here taken as independent streams of uneven
 * sizes). A batch step runs every kernel of a fused step once for all streams, with
 * tile shapes, grids and LDS sized at each stream's rank caps so that the launch
 * sequence does not change when ranks do; the host reads one small summary per
 * stream per step and reinitialises only the streams whose controller decided so.
 *
 * tdb_batch_create: n >= 1 configurations (order 3, path AUTO or FUSED, one common
 *   data_dtype and precision) and n device snapshots V0_dev[i]; runs each stream's
 *   HOSVD initialisation. TDB_EUNSUPPORTED when a stream's stage pass does not fit
 *   the LDS at its caps.
 * tdb_batch_ingest: V_dev is a host array of n device pointers, one snapshot per
 *   stream, each C-contiguous in data_dtype. Snapshot ownership as in
 *   tdb_ingest_snapshot, per stream. When every stream has TDB_BORROW snapshots the
 *   call is pipelined as tdb_ingest_snapshot is: it enqueues this step for all
 *   streams on `stream`, then reads the previous step's summaries (without
 *   synchronising the device) and acts on the decisions that need the host; the
 *   device holds such a stream's part of this step, which then runs again for those
 *   streams alone. The newest step is read by the next ingest, by tdb_batch_flush or
 *   by any call that returns a member's results; TDB_ENUMERIC is reported by the call
 *   that reads the step. The launches of a step are replayed from a HIP graph, one per
 *   step parity, captured again when the launch shapes change (TDB_GRAPH=0 in the
 *   environment launches them one by one; TDB_PIPELINE=0 reads every step at once).
 *   Two kernels of a step run on a second stream the batch owns (default priority),
 *   forked from and joined back to `stream` by events within the step, so work that
 *   follows on `stream`, or a synchronisation of it, sees the whole step.
 * tdb_batch_flush: reads the newest step if it has not been read; returns its
 *   status.
 * tdb_batch_stream: a handle of stream i for tdb_get_stats, tdb_get_core_and_bases,
 *   tdb_reconstruct and tdb_set_threshold. The batch owns it: tdb_ingest_snapshot on
 *   it returns TDB_ESTATE and tdb_destroy ignores it.
 * tdb_batch_profile_enable / _read: as tdb_profile_enable / _read for the batched
 *   stage pass and error pass (one launch covers all streams; the bytes per launch
 *   are summed over streams). A timed step is launched without its graph (the events
 *   are stamped by the dispatches themselves).
 * tdb_batch_destroy frees the batch and all its streams; NULL-safe. */
typedef struct tdb_batch_ctx* tdb_batch;
tdb_status tdb_batch_create(int32_t n, const tdb_config* cfgs, const void* const* V0_dev, void* stream,
                            tdb_batch* out);
tdb_status tdb_batch_ingest(tdb_batch b, const void* const* V_dev, void* stream);
tdb_status tdb_batch_flush(tdb_batch b);

/* The batch's kernel plan, chosen once at creation (host-written struct, caller-owned).
 * The stage pass of every member is one kernel: matrix-core column blocks of all rows
 * (pass_kind 2; pass_cols columns of mode 2 per workgroup), matrix-core tiles (1) or
 * vector-ALU tiles (0); the error pass takes column blocks of the mode-1 unfolding
 * (err_kind 1) or row slabs (0). With more than one candidate, each is timed on the
 * first snapshots (the pass over three launches after one untimed; the partials only,
 * no state changes) and the fastest kept; the choice is cached for the process per
 * shape class (storage and compute types, the members' extents and caps).
 * source: 0 the fixed rule (TDB_AUTOTUNE=0 in the environment, or TDB_RPASS_COLS
 * forcing the column count), 1 timed at creation,
 * 2 the cached plan of an earlier batch of the same class. pass_us: the timed
 * candidates' average launch (column blocks of 64, of 32 columns, matrix-core tiles;
 * 0 = not timed); err_us: row slabs, column blocks. */
typedef struct {
  int32_t pass_kind, pass_cols, err_kind, source;
  double pass_us[3];
  double err_us[2];
} tdb_batch_plan_info;
tdb_status tdb_batch_plan(tdb_batch b, tdb_batch_plan_info* out);
tdb_status tdb_batch_stream(tdb_batch b, int32_t i, tdb_handle* out);
tdb_status tdb_batch_profile_enable(tdb_batch b, int32_t on);
tdb_status tdb_batch_profile_read(tdb_batch b, int32_t pass, int64_t* launches, double* total_ms,
                                  double* bytes_per_launch);
void tdb_batch_destroy(tdb_batch b);
const char* tdb_batch_last_error(tdb_batch b);

/* ---- Learned error gate (not in the paper: a predictor of eq. (error) from the
 * singular values of the core unfoldings, eq. (rot), so that the exact error pass of
 * Sec. 2.5 can be skipped when the error is predicted to sit far below the threshold).
 * Network 384 -> 128 -> 128 -> 1, tanh-form GELU, FP32; inputs: 8 consecutive steps x
 * 3 modes x the 16 leading singular values, as log10(max(sigma, 1e-30)), oldest step
 * first, mode-major, standardised per feature; output: log10 of the step's error.
 * Parameters: one FP32 vector of TDB_GATE_PARAMS entries, W1 (128 x 384 row-major),
 * b1, W2 (128 x 128), b2, w3 (128), b3.
 *
 * tdb_gate_create: a trainer owning the parameters, Adam moments and scratch for
 *   batches of up to max_batch samples (device memory of the current device).
 * tdb_gate_set_params / _get_params: host copies (set also clears Adam's moments).
 * tdb_gate_forward: y_dev[i] = network(X_dev row i), X_dev n x 384 FP32 (device).
 * tdb_gate_grad: gradient of the mean squared error against t_dev (n) into grad_dev
 *   (TDB_GATE_PARAMS floats, device; NULL keeps it inside the trainer) and the loss
 *   into *loss_host (NULL: not read back).
 * tdb_gate_train_step: tdb_gate_grad, then one Adam step (lr; betas 0.9, 0.999;
 *   eps 1e-8; bias correction by the trainer's own step count).
 * tdb_batch_gate_attach: use trainer g's current parameters in batch b (not copied:
 *   keep g alive). feat_mean_std_host: 384 means then 384 standard deviations
 *   (copied). mode: TDB_GATE_OFF, TDB_GATE_RECORD (singular values every step, exact
 *   pass always), TDB_GATE_ACTIVE (skip the exact pass when the gate allows), or
 *   TDB_GATE_SHADOW (exact pass always; stats.would_skip reports the verdict).
 * The gate runs the exact pass when fewer than 8 steps exist since the last
 * reinitialisation, when the prediction is within half a decade of the threshold or
 * above it, or when some mode's last singular value alone fits the removal budget. */
enum { TDB_GATE_PARAMS = 65921, TDB_GATE_INPUTS = 384 };
enum { TDB_GATE_OFF = 0, TDB_GATE_RECORD = 1, TDB_GATE_ACTIVE = 2, TDB_GATE_SHADOW = 3 };
typedef struct tdb_gate_ctx* tdb_gate;
tdb_status tdb_gate_create(int32_t max_batch, tdb_gate* out);
tdb_status tdb_gate_set_params(tdb_gate g, const float* params_host);
tdb_status tdb_gate_get_params(tdb_gate g, float* params_host);
tdb_status tdb_gate_forward(tdb_gate g, const float* X_dev, int32_t n, float* y_dev, void* stream);
tdb_status tdb_gate_grad(tdb_gate g, const float* X_dev, const float* t_dev, int32_t n, float* grad_dev,
                         float* loss_host, void* stream);
tdb_status tdb_gate_train_step(tdb_gate g, const float* X_dev, const float* t_dev, int32_t n, float lr,
                               float* loss_host, void* stream);
void tdb_gate_destroy(tdb_gate g);
const char* tdb_gate_last_error(tdb_gate g);
tdb_status tdb_batch_gate_attach(tdb_batch b, tdb_gate g, const float* feat_mean_std_host, int32_t mode);

/* The gate on a single stream (the fused third-order path; batch members use
 * tdb_batch_gate_attach). params_host: n_params == TDB_GATE_PARAMS FP32 values in the
 * layout above; feat_mean_std_host: 384 means then 384 standard deviations. Both are
 * copied into the handle (no trainer needs to stay alive). mode as for batches:
 * TDB_GATE_ACTIVE skips the exact error pass of eq. (error) (Sec. 2.5) when the
 * prediction allows (that step's eps is then NaN and it takes no add/remove
 * decision), TDB_GATE_SHADOW only reports the verdict, TDB_GATE_RECORD forms the
 * core singular values every step (params may be NULL), TDB_GATE_OFF detaches.
 * Resolves a pending step first. TDB_EUNSUPPORTED on the plain path; TDB_ESTATE for
 * a batch member; TDB_EINVAL for a wrong count, non-finite parameters or
 * non-positive standard deviations. */
tdb_status tdb_gate_load(tdb_handle h, const float* params_host, const float* feat_mean_std_host, int32_t n_params,
                         int32_t mode);

/* ---- For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.
 * The dense reconstruction of tdb_reconstruct, C x_1 U_1 ... x_p U_p, from factors the
 * caller holds on the device, with the intermediates of the n-mode product chain in a
 * fixed scratch array inside the library: TDB_NOALLOC_SCRATCH doubles (64 MiB) per GPU,
 * held from the first call on that GPU until the process ends. The call allocates no
 * memory (no hipMalloc, no host allocation on success).
 * order: 2..4; dims[n] = N_n and ranks[n] = r_n with 1 <= r_n <= N_n; C_dev: the
 * C-contiguous r_1 x ... x r_p FP64 core; U_dev: a host array of `order` device
 * pointers, U_dev[n] the row-major N_n x r_n FP64 basis; out_dev: S values in
 * data_dtype (TDB_F64 | TDB_F32), C-contiguous, caller-owned. Enqueued on `stream`
 * (products in FP64, rounded once into data_dtype).
 * TDB_EINVAL for bad arguments or when an intermediate exceeds TDB_NOALLOC_SCRATCH / 2
 * doubles (the modes are contracted in order of increasing N_n / r_n; the largest
 * intermediate is the product of all but the last such mode's size and that rank);
 * TDB_EHIP for a failed launch; messages from tdb_last_error(NULL).
 * Every call on one GPU shares that GPU's array and leaves the last call's
 * intermediates in it: calls that overlap on one GPU (on different streams or
 * threads) race and must be ordered by the caller. */
#define TDB_NOALLOC_SCRATCH 8388608
tdb_status tdb_reconstruct_noalloc(int32_t order, const int64_t* dims, const int32_t* ranks, const double* C_dev,
                                   const double* const* U_dev, int32_t data_dtype, void* out_dev, void* stream);

/* Layout check for language bindings: writes sizeof(tdb_config) and sizeof(tdb_stats)
 * (either pointer may be NULL). Needs no device. */
void tdb_struct_sizes(int64_t* config_bytes, int64_t* stats_bytes);

/* Message for the last non-OK status on h (or of the last failed create when h is
 * NULL). Owned by the library; valid until the next call on the same handle. */
const char* tdb_last_error(tdb_handle h);

#ifdef __cplusplus
}
#endif
#endif /* TDB_H */
