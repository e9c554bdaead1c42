/*
 * fcsdnn.h - C ABI of the MI355X (gfx950) FC-SDNN per-stage solver.
 *
 * The method is the multi-patch FC-SDNN shock-dynamics solver of
 * Leibovici & Bruno, "General-domain FC-based shock-dynamics solver II"
 * (arXiv 2506.19370).  Section references below are to that paper.
 *
 * Conventions shared by every entry point
 *   - Arrays described as "host" are read (or written) by the call only and
 *     remain owned by the caller; "device" arrays are GPU memory owned by the
 *     caller.
 *   - Subpatch fields are (n2, n1) arrays, q^1 (index i) fastest.
 *   - Every call returns an fcs_status; no C++ exception crosses the ABI.
 *     Context-bound calls leave a message for fcs_last_error().
 *   - The library never allocates device memory: the caller binds one
 *     device workspace (fcs_bind) and a HIP stream; all device work is
 *     enqueued on that stream, in order.
 */
#ifndef FCSDNN_H
#define FCSDNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FCS_OK = 0,
  FCS_EINVAL = 1,      /* bad argument, shape or parameter                    */
  FCS_EOVERLAP = 2,    /* a fringe point has no eligible donor (Sec. 3.2.3)   */
  FCS_ENOMEM = 3,      /* workspace too small / host allocation failed        */
  FCS_ENONFINITE = 4,  /* the state became non-finite or non-physical (sticky)*/
  FCS_EHIP = 5,        /* a HIP runtime call failed                           */
  FCS_ESTATE = 6       /* call out of order (e.g. advance before bind)        */
} fcs_status;

/* Kinds of the sides of a subpatch index box and of the mask boundary
 * (Sec. 3.3: internal sides receive fringe data, external sides carry
 * boundary conditions). */
enum {
  FCS_SIDE_INTERNAL = 0,
  FCS_SIDE_INFLOW = 1,   /* Dirichlet: the subpatch's inflow state          */
  FCS_SIDE_OUTFLOW = 2,  /* supersonic outflow: nothing imposed              */
  FCS_SIDE_SLIP = 3,     /* inviscid wall: zero normal momentum, p kept     */
  FCS_SIDE_EXACT = 4,    /* n_f-point layer set to the exact vortex solution */
  FCS_SIDE_NOSLIP = 5    /* no-slip adiabatic wall (the paper's obstacle
                            conditions, Sec. 7): zero momentum, rho kept,
                            theta = p/((gamma-1) rho) chosen so that the FC
                            first derivative along the grid line ending at
                            the wall vanishes there (both ends of a line
                            solved together; at a node ending two such lines,
                            the line along q^2)                             */
};

/* Patch types of Sec. 3.1 (informational; C1 requires a mask). */
enum { FCS_PATCH_I = 0, FCS_PATCH_S = 1, FCS_PATCH_C1 = 2, FCS_PATCH_C2 = 3 };

/* Arithmetic of the FC derivative contractions (the state, the RK
 * accumulation and the operator construction are always FP64). */
enum {
  FCS_PREC_FP64 = 0,    /* FP64 MFMA                                         */
  FCS_PREC_FP32 = 1,    /* FP32 operands, FP32 MFMA accumulation             */
  FCS_PREC_BF16X3 = 2,  /* split-BF16 hi/lo products (3 MFMAs), FP32 accum.  */
  FCS_PREC_BF16X6 = 3   /* split-BF16 hi/mid/lo products (6 MFMAs), FP32
                           accumulators per magnitude order, FP64 sum       */
};

/* Smoothness classifier for the artificial viscosity (Sec. 4, Alg. 3). */
enum {
  FCS_AV_OFF = 0,
  FCS_AV_MODAL = 1,     /* modal-decay fallback indicator                   */
  FCS_AV_SDNN = 2,      /* trained network (weights in fcs_params)           */
  FCS_AV_FROZEN = 3     /* classes supplied by fcs_set_tau (testing)         */
};

/* Kinds of dense FC operators: first and second derivative (index units),
 * the filter of Alg. 4 (t > 0: exp(-16 ln 10 eta^36) of the mode
 * eta = 2|m|/(n + C)), and the stronger filter of the initial-data smearing
 * (the same with eta^8). */
enum { FCS_OP_D1 = 0, FCS_OP_D2 = 1, FCS_OP_FILTER = 2, FCS_OP_SMEAR = 3 };

/* Fields for fcs_get_field. */
enum {
  FCS_FIELD_RHO = 0, FCS_FIELD_MX = 1, FCS_FIELD_MY = 2, FCS_FIELD_E = 3,
  FCS_FIELD_P = 4, FCS_FIELD_MACH = 5, FCS_FIELD_MU = 6,
  FCS_FIELD_TAU0 = 7, FCS_FIELD_TAU1 = 8, FCS_FIELD_MUHAT = 9
};

/* Variables accepted by fcs_set_state. */
enum { FCS_VARS_CONS = 0, FCS_VARS_PRIM = 1 };

/* SDNN parameter blob: W1 (64x16), b1 (64), W2 (64x64), b2 (64), W3 (3x64),
 * b3 (3), row-major, FP32, in this order. */
#define FCS_SDNN_WINDOW 16
#define FCS_SDNN_HIDDEN 64
#define FCS_SDNN_CLASSES 3
#define FCS_SDNN_NPARAM (64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3)

typedef struct {
  double gamma;        /* heat-capacity ratio (Sec. 2), 1.4                  */
  double cfl;          /* CFL number of the adaptive step                    */
  double c_mu;         /* viscosity scale of the preliminary viscosity       */
  double dt_fixed;     /* > 0: use this step instead of the adaptive one     */
  int32_t fc_d;        /* FC-Gram matching points d (Sec. 2)                 */
  int32_t fc_C;        /* FC-Gram continuation points C                      */
  int32_t n_f;         /* fringe width (Sec. 3.3; the paper uses 5)          */
  int32_t n_v;         /* overlap / viscosity-window parameter (9)           */
  int32_t precision;   /* FCS_PREC_*                                         */
  int32_t av_mode;     /* FCS_AV_*                                           */
  int32_t filter;      /* nonzero: spectral filter every step t > 0 (Alg. 4) */
  int32_t use_graph;   /* nonzero: replay whole steps as a captured hipGraph */
  int32_t autotune;    /* nonzero: time the contraction tile shapes on the
                          first advance and keep the fastest               */
  int32_t visc_all_lines; /* nonzero: evaluate the viscous derivatives on
                          every grid line.  0 (default): on lattice
                          subpatches a row or column along which mu vanishes
                          in a step is skipped; its derivatives only meet
                          exact zeros there (Sec. 4, localized viscosity),
                          so the state is the same                         */
  const float* sdnn_weights; /* host, FCS_SDNN_NPARAM floats; copied        */
  double vortex[5];    /* EXACT sides: beta, x0, y0, u0, v0 of the isentropic
                          vortex (background rho = p = 1)                    */
  int32_t smear;       /* nonzero: localized smearing of the initial data in
                          the first step from t = 0 (Alg. 4, t = 0; Sec. 5
                          item 3): where the step's classes flag a
                          discontinuity, rho, rho u, rho v and theta are
                          blended with their FCS_OP_SMEAR-filtered values by
                          a window localized as the viscosity is, and E is
                          rebuilt.  Needs av_mode != FCS_AV_OFF           */
} fcs_params;

typedef struct {
  int32_t type;            /* FCS_PATCH_*                                    */
  int32_t n1, n2;          /* index box; each >= 2 fc_d, <= 512              */
  const double* x;         /* host (n2, n1) node coordinates; copied         */
  const double* y;
  const uint8_t* mask;     /* host (n2, n1), 1 = active, or NULL; every row
                              and column must hold one run of active points  */
  int32_t side[4];         /* kinds of sides W (i=0), E, S (j=0), N          */
  int32_t notch;           /* kind of the mask boundary                      */
  double inflow[4];        /* primitive (rho, u, v, p) for INFLOW sides      */
} fcs_patch_desc;

typedef struct {
  int64_t steps;           /* completed steps                                */
  int64_t stages;          /* completed stages                               */
  double t;                /* simulated time                                 */
  double dt;               /* last step size                                 */
  double mass, energy;     /* sums of rho and E over active points (no
                              overlap weighting)                             */
  int64_t npoints;         /* active points, all subpatches                  */
  int32_t stage_variant;   /* contraction tile variant of the stage launches
                              (index for fcs_gemm_variant_name)             */
  int32_t reserved;
} fcs_stats_t;

typedef struct fcs_ctx fcs_ctx;

int fcs_version(void);

/* Build a solver for a set of subpatches (Alg. 2 on one GPU): grids and
 * metrics (Sec. 5 item 1), dense FC operators for every line length
 * (Sec. 2), fringe interpolation and viscosity blend tables (Sec. 3.3,
 * Sec. 4).  Host-only; validates the minimum-overlap condition
 * (FCS_EOVERLAP).  On success *out must be released with fcs_destroy. */
fcs_status fcs_create(const fcs_params* prm, int32_t npatch,
                      const fcs_patch_desc* patches, fcs_ctx** out);

/* Bytes of device workspace the context needs. */
fcs_status fcs_workspace_size(const fcs_ctx* ctx, size_t* bytes);

/* Bind a device workspace (>= fcs_workspace_size bytes, 256-byte aligned)
 * and a HIP stream (hipStream_t, may be NULL for the null stream); uploads
 * the static tables.  The context uses both until fcs_destroy. */
fcs_status fcs_bind(fcs_ctx* ctx, void* workspace, size_t bytes, void* stream);

/* Set the state of one subpatch from (4, n2, n1) conserved or primitive
 * values (host or device; vars = FCS_VARS_*); masked points are ignored.
 * The copy is complete when the call returns (it synchronizes the bound
 * stream).  Only at a step boundary: inside a partial step (after an
 * fcs_advance whose stage count was not a multiple of 5) it fails with
 * FCS_ESTATE and changes nothing.  Together with fcs_get_field and
 * fcs_set_time it checkpoints and resumes a run (Alg. 1 output): a context
 * given the conserved fields and the time of another at a step boundary
 * continues it bit for bit (same parameters and contraction tile shape). */
fcs_status fcs_set_state(fcs_ctx* ctx, int32_t patch, int32_t vars,
                         const double* src, int32_t src_on_device);
/* Set the simulated time t (finite).  The filter of Alg. 4 applies to every
 * step that starts at t > 0, so resuming at t > 0 filters the first step as
 * the uninterrupted run does.  FCS_ESTATE inside a partial step; FCS_EINVAL
 * for a non-finite t.  Synchronizes the bound stream. */
fcs_status fcs_set_time(fcs_ctx* ctx, double t);

/* Frozen smoothness classes (FCS_AV_FROZEN): (2, n2, n1) uint8 values of
 * tau along q^1 and q^2, host. */
fcs_status fcs_set_tau(fcs_ctx* ctx, int32_t patch, const uint8_t* tau);

/* Advance n_stages SSPRK stages (Alg. 1).  The viscosity, filter and step
 * size are evaluated at step boundaries; a partial step resumes on the next
 * call.  Asynchronous unless t_out is non-NULL (then synchronizes and
 * returns the time).  FCS_ENONFINITE once a stage produced a non-finite
 * value or rho <= 0 or p <= 0 (checked when synchronizing). */
fcs_status fcs_advance(fcs_ctx* ctx, int64_t n_stages, double* t_out);

/* Copy one field of one subpatch, (n2, n1) doubles (FCS_FIELD_*), to host or
 * device memory.  Host destinations synchronize the stream. */
fcs_status fcs_get_field(fcs_ctx* ctx, int32_t patch, int32_t field,
                         double* dst, int32_t dst_on_device);

/* Counters, time, last step and integrals (synchronizes). */
fcs_status fcs_stats(fcs_ctx* ctx, fcs_stats_t* out);

/* Stage-contraction autotuner results of the context (autotune in
 * fcs_params; the tuning runs at the first advance): the average launch
 * time in ms of every candidate variant, in the order of
 * fcs_gemm_variant_name, written to ms[0 .. n-1] (host; n <= 16; 0 for
 * candidates not timed).  FCS_EINVAL for n out of range or a NULL ms. */
fcs_status fcs_autotune_times(const fcs_ctx* ctx, int32_t n, double* ms);

/* Tune again (autotune in fcs_params): the next advance times the
 * candidates on the current state, with the viscous lines its viscosity
 * needs, keeps the fastest and captures its step graphs anew.  For runs
 * whose localized viscosity grows or shrinks far from where the first
 * tuning saw it.  Synchronizes the stream; the state is not changed.
 * FCS_ESTATE before fcs_bind. */
fcs_status fcs_retune(fcs_ctx* ctx);

/* Pin the stage-contraction tile shape to candidate `index` (the order of
 * fcs_gemm_variant_name for the context's precision) instead of tuning it;
 * a later fcs_retune tunes again.  Synchronizes the stream; the step graphs
 * are captured anew at the next advance.  FCS_EINVAL for an index out of
 * range, FCS_ESTATE before fcs_bind. */
fcs_status fcs_set_stage_variant(fcs_ctx* ctx, int32_t index);

/* Average duration (ms) of the dominant derivative-contraction launch (the
 * stage contraction of stages 2 to 5 of each step; the first stage's launch
 * also carries the viscosity gradient) over the advance calls since the last
 * reset, measured with HIP events on the bound stream, and the algorithmic
 * flops and bytes of one such launch, averaged over the same launches: the
 * lines each step needed (viscous lines skipped in a step, see
 * visc_all_lines, are not counted; before any profiled step, all lines).
 * Profiling synchronizes the stream after every step.
 * Timing is recorded only after fcs_profile_enable(ctx, 1).  Whole steps
 * then replay a separate graph that carries event-record nodes around each
 * stage contraction and one empty pair of event nodes; *event_latency_ms
 * (nullable) is the average interval of that empty pair, the latency an
 * event pair adds to each measured interval.  Without a stream or graphs
 * the events are recorded eagerly and *event_latency_ms is 0. */
fcs_status fcs_profile_enable(fcs_ctx* ctx, int32_t on);
/* The stage contraction of the last step, timed alone: `reps` launches back
 * to back on the bound stream between two HIP events (after one untimed
 * launch), on the current state with the tiles the last step's viscosity
 * needed; *avg_ms is the average per launch, *flops and *bytes (nullable)
 * the useful work of one launch, as for fcs_profile_read.  The launches
 * overwrite the stage derivatives only, which every stage recomputes before
 * reading them, so the solution is not changed.  Synchronizes the stream.
 * FCS_EINVAL for reps <= 0 or a NULL avg_ms; FCS_ESTATE before the first
 * advance. */
fcs_status fcs_profile_stage(fcs_ctx* ctx, int32_t reps, double* avg_ms, double* flops, double* bytes);
fcs_status fcs_profile_read(fcs_ctx* ctx, double* avg_ms, double* flops_per_launch,
                            double* bytes_per_launch, int64_t* launches, double* event_latency_ms);

const char* fcs_last_error(const fcs_ctx* ctx);
void fcs_destroy(fcs_ctx* ctx);

/* ---------------------------------------------------------------------
 * FC operators (host).
 * fcs_fc_continuation: FC-Gram construction (Sec. 2, with the continuation
 * reading documented with the library): Q (d x d) Gram basis at the matching
 * points, A (C x d) continuation of each Gram polynomial; row-major.
 * fcs_fc_operator: the n x n matrix (row t, column s, row-major) of the FC
 * first derivative, second derivative (index units) or filter for lines of
 * n points (2 d <= n <= 1024). */
fcs_status fcs_fc_continuation(int32_t d, int32_t C, double* Q, double* A);
fcs_status fcs_fc_operator(int32_t n, int32_t d, int32_t C, int32_t kind, double* out);

/* ---------------------------------------------------------------------
 * Batched derivative sweep: d/dq^1 and d/dq^2 of ncomp fields on many
 * rectangular patches of uneven sizes in one grouped launch (the FC
 * derivative contraction of the stage algorithm, Sec. 5).
 * Input and outputs are device arrays holding, patch after patch,
 * (ncomp, n2, n1) doubles; outputs are in index units (d/di, d/dj). */
typedef struct fcs_sweep fcs_sweep;
fcs_status fcs_sweep_create(int32_t npatch, const int32_t* n1n2 /* host, 2*npatch */,
                            int32_t ncomp, int32_t precision, int32_t d, int32_t C,
                            fcs_sweep** out);
fcs_status fcs_sweep_workspace_size(const fcs_sweep* s, size_t* bytes);
fcs_status fcs_sweep_bind(fcs_sweep* s, void* workspace, size_t bytes, void* stream);
fcs_status fcs_sweep_run(fcs_sweep* s, const double* in, double* d1, double* d2);
/* HIP-event timing of the grouped launch: on = 1 starts (and resets), 0
 * stops, -1 only reads.  Returns the average ms per launch since the start,
 * the algorithmic flops (2 n per point and line direction and component)
 * and bytes (FP64 operand and result once) of one launch.  Synchronizes. */
fcs_status fcs_sweep_profile(fcs_sweep* s, int32_t on, double* avg_ms, double* flops, double* bytes,
                             int64_t* launches);
fcs_status fcs_sweep_points(const fcs_sweep* s, int64_t* npoints);
/* Autotuner: runs every candidate tile shape of the contraction kernel on
 * the given device arrays (results overwritten), keeps the fastest, and
 * writes the per-candidate ms (fcs_gemm_variant_count(precision) doubles,
 * host) to ms if non-NULL.  Synchronizes. */
fcs_status fcs_sweep_autotune(fcs_sweep* s, const double* in, double* d1, double* d2, double* ms);
/* Candidate tile variants of the grouped contraction for a precision
 * (FCS_PREC_*; 0 for an unknown precision), and the explicit choice of one
 * of them (0 <= index < count) for a sweep, in the autotuner's order.
 * FCS_EINVAL for an index out of range. */
int32_t fcs_gemm_variant_count(int32_t precision);
/* Kernel name of a variant (as profilers list it, without namespaces), NUL
 * terminated in buf (len bytes, host); FCS_EINVAL for an unknown variant. */
fcs_status fcs_gemm_variant_name(int32_t precision, int32_t index, char* buf, int32_t len);
fcs_status fcs_sweep_set_variant(fcs_sweep* s, int32_t index);
void fcs_sweep_destroy(fcs_sweep* s);

/* ---------------------------------------------------------------------
 * Smoothness classification of 16-point windows (Sec. 4, Alg. 3).
 * windows: device, nwin x 16 doubles (raw proxy values); tau: device uint8.
 * fcs_sdnn_infer uses the network in params (device, FCS_SDNN_NPARAM floats)
 * with BF16 MFMA products and FP32 accumulation; logits (device, nwin x 3
 * floats) may be NULL.  fcs_modal_infer is the modal-decay fallback. */
fcs_status fcs_sdnn_infer(const float* params, const double* windows, int64_t nwin,
                          uint8_t* tau, float* logits, void* stream);
fcs_status fcs_modal_infer(const double* windows, int64_t nwin, uint8_t* tau, void* stream);

/* One training step of the network: forward, softmax cross-entropy with
 * per-class weights, backward and Adam (lr, beta1 0.9, beta2 0.999,
 * eps 1e-8, step number t >= 1).  x: device, batch x 16 normalized windows
 * (FP32); labels: device int32; class_weight: device, 3 floats; params, m, v:
 * device FP32 (FCS_SDNN_NPARAM each), updated in place; loss: device float;
 * grads: device FP32 (FCS_SDNN_NPARAM) or NULL.  Default: forward and
 * backward on the BF16 matrix cores (inputs, weights and hidden activations
 * rounded to bf16, the back-propagated errors entering the products as two
 * bf16 parts, FP32 accumulation and FP32 elsewhere; the batch sums in a fixed
 * order, so a step is deterministic).  workspace: device,
 * fcs_sdnn_train_workspace bytes. */
size_t fcs_sdnn_train_workspace(int32_t batch);
/* flags bit 0: FP32 activations and products, no bf16 rounding (the
 * gradient-check mode; scalar FP32 kernels, not the matrix cores). */
fcs_status fcs_sdnn_train_step(float* params, float* m, float* v, int32_t t, float lr,
                               const float* x, const int32_t* labels, const float* class_weight,
                               int32_t batch, float* loss, float* grads, int32_t flags,
                               void* workspace, size_t bytes, void* stream);

/* Allocation-free form of fcs_sdnn_train_step, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc).  Same arguments and
 * results without the workspace: the per-sample scratch is a library-owned
 * device array sized for FCS_SDNN_TRAIN_MAX_BATCH samples (9.8 MB), of which
 * each GPU holds its own copy from the first call on it until the process
 * ends.  The call allocates nothing.  batch > FCS_SDNN_TRAIN_MAX_BATCH (or any
 * argument fcs_sdnn_train_step rejects) -> FCS_EINVAL; a failed symbol lookup
 * or launch -> FCS_EHIP.  All calls on one GPU share its array: calls that
 * overlap in time on that GPU (unordered streams, other threads) race and
 * must be serialized by the caller. */
#define FCS_SDNN_TRAIN_MAX_BATCH 8192
fcs_status fcs_sdnn_train_step_noalloc(float* params, float* m, float* v, int32_t t, float lr,
                                       const float* x, const int32_t* labels,
                                       const float* class_weight, int32_t batch, float* loss,
                                       float* grads, int32_t flags, void* stream);


/* Apply a dense FC operator (FCS_OP_*) along lines: nlines lines of n
 * points, device in/out (nlines x n doubles), FP64.  workspace: device,
 * fcs_lines_workspace(n, nlines) bytes.  Synchronizes the stream.  Used to
 * pass training lines through the solver's filter. */
size_t fcs_lines_workspace(int32_t n, int64_t nlines);
fcs_status fcs_lines_apply(int32_t n, int64_t nlines, int32_t kind, int32_t d, int32_t C,
                           const double* in, double* out, void* workspace, size_t bytes,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FCSDNN_H */
