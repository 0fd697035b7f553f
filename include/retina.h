/*
 * libretina: the optimisation-based Artificial Retina track finder
 * (Borisyak, Ustyuzhanin, Derkach, Belous, "Numerical optimization for
 * Artificial Retina Algorithm", arXiv:1709.08610) on AMD Instinct MI355X
 * (gfx950).
 *
 * Problem statement (Section 2, Algorithm 1): hits in, line parameters out.
 * The response of a line hypothesis theta to an event's hits X is Eq. (1),
 *     R(theta) = sum_k exp(-s(x_k, theta)^2 / sigma^2),
 * with s the Euclidean distance between hit k and the line's intersection
 * with the hit's detector plane (Section 3).  Track finding locates the local
 * maxima of R by many independent truncated-Newton ascents from seeds
 * (Algorithm 1), then clusters the converged solutions and keeps, per
 * cluster, the highest response above a threshold R0.
 *
 * Conventions shared by every entry point
 *   - C ABI, C99 types only.  Every function returns int: RETINA_OK (0) or a
 *     negative retina_status; no exception or abort crosses the boundary.
 *     The message of the last failure is retina_last_error(ctx).
 *   - Geometry: planes perpendicular to z at plane_z[p] (host memory, FP32,
 *     any order).  meas_dim 2: a hit is (plane, x, y) and a line is
 *     theta = (x0, y0, tx, ty) with x(z) = x0 + tx z, y(z) = y0 + ty z.
 *     meas_dim 1 (the 2D toy of Section 2, Fig. 1): a hit is (plane, u) with
 *     u stored in x (y unused, may be NULL) and theta = (x0, tx), u(z) = x0 +
 *     tx z.  n_par = 2*meas_dim.
 *   - Hits: CSR over events: event e owns hits event_offsets[e] ..
 *     event_offsets[e+1]-1 in any order.  x, y FP32; plane int32.
 *   - Memory: retina_hits.mem says where the hit arrays, the event offsets,
 *     explicit seeds and every output array live (RETINA_MEM_HOST: ordinary
 *     host memory; RETINA_MEM_DEVICE: device memory of the context's device,
 *     e.g. torch tensors' data_ptr()).  Device-memory calls are ordered on
 *     the context's stream and return after that stream has finished them.
 *   - Ownership: the caller owns every input and output buffer; the library
 *     keeps no caller pointer after a call returns.  The library owns the
 *     context (device pool, stream, captured graphs) until retina_destroy.
 *   - Validation happens before any result is written: NaN/Inf hit
 *     coordinates or plane positions, plane index outside [0, n_planes),
 *     decreasing offsets, sigma <= 0 or non-finite, meas_dim not 1 or 2, NULL
 *     required pointers and negative sizes all give RETINA_ERR_INVALID_ARG
 *     and leave outputs untouched.  An event without hits is valid (R = 0,
 *     no tracks).
 *   - Threading: one context per host thread; a context is not thread-safe.
 */
#ifndef RETINA_H
#define RETINA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct retina_ctx retina_ctx;

typedef enum {
    RETINA_OK = 0,
    RETINA_ERR_INVALID_ARG = -1,
    RETINA_ERR_OUT_OF_MEMORY = -2,
    RETINA_ERR_DEVICE = -3,     /* no usable gfx950 device, or a HIP runtime failure */
    RETINA_ERR_CAPACITY = -4,   /* an output array is too small; see retina_find_tracks */
    RETINA_ERR_INTERNAL = -6
} retina_status;

enum { RETINA_MEM_HOST = 0, RETINA_MEM_DEVICE = 1 };
enum { RETINA_WANT_R = 1, RETINA_WANT_GRAD = 2, RETINA_WANT_HESS = 4 };
enum { RETINA_SEED_LATTICE = 0, RETINA_SEED_EXPLICIT = 1 };
/* Update rule of Algorithm 1's inner loop (Section 3 reports trying several
 * optimisation methods and keeping truncated Newton). */
enum { RETINA_UPDATE_NEWTON = 0, RETINA_UPDATE_GRADIENT = 1, RETINA_UPDATE_BFGS = 2 };

/* per-seed / per-track flag bits */
enum {
    RETINA_CONVERGED = 1,  /* -H positive definite at the last FP64 Newton polish and its
                              scaled step <= conv_tol * sigma_final */
    RETINA_STALLED = 2,    /* some line search accepted none of its step lengths */
    RETINA_NOT_PD = 4,     /* -H not positive definite at the last polish */
    RETINA_NEGCURV = 8     /* some Newton-CG direction met non-positive curvature */
};

typedef struct {
    int32_t meas_dim;       /* 1 or 2 */
    int32_t n_planes;       /* 1 .. RETINA_MAX_PLANES */
    const float* plane_z;   /* host memory, n_planes finite values */
} retina_geometry;

#define RETINA_MAX_PLANES 64
#define RETINA_MAX_SIGMA 16
#define RETINA_MAX_LATTICE_SIDE 8192   /* cells per dimension of a seed lattice or search grid */
#define RETINA_NOALLOC_SCRATCH_BYTES (64ull << 20)  /* fixed workspace of retina_response_noalloc, per device */

typedef struct {
    int32_t mem;                   /* RETINA_MEM_HOST or RETINA_MEM_DEVICE */
    int64_t n_events;              /* >= 0 */
    const int64_t* event_offsets;  /* n_events+1, [0] = 0, non-decreasing */
    const float* x;
    const float* y;                /* NULL allowed when meas_dim == 1 */
    const int32_t* plane;
} retina_hits;

/* Method parameters of Algorithm 1 as this library reads it.  A trajectory
 * takes n_sigma continuation steps (sigma[0..n_sigma-1], one truncated-Newton
 * step each; Section 3 changes the bandwidth with every step) and then
 * n_final_steps steps at sigma_final, followed by n_polish FP64 Newton
 * iterations at sigma_final.  The number of updates is fixed (Section 2:
 * no early exit). */
typedef struct {
    int32_t n_sigma;            /* 0 .. RETINA_MAX_SIGMA */
    const float* sigma;         /* host memory */
    float sigma_final;
    int32_t n_final_steps;
    int32_t n_polish;           /* >= 1 */
    int32_t ls_trials;          /* backtracking step lengths 1, 1/2, .., 2^-(ls_trials-1); >= 1 */
    float armijo_c1;            /* sufficient-increase constant */
    float step_cap_sigmas;      /* scaled step capped at step_cap_sigmas * sigma */
    float small_step_sigmas;    /* Newton steps (no negative curvature) with scaled length
                                   <= small_step_sigmas * sigma are taken without a search */
    int32_t n_slope_steps;      /* meas_dim 2: the first n_slope_steps steps move only (tx, ty);
                                   the count runs on into the polish iterations, so a value
                                   >= steps + n_polish holds the offsets at their seed values
                                   throughout (lines through the origin) */
    float conv_tol;             /* converged iff last polish step <= conv_tol * sigma_final */
    float R0;                   /* keep clusters whose best response is >= R0 */
    float d_merge;              /* cluster radius: largest in-plane separation over the two
                                   end planes of the detector */
    int32_t seed_mode;          /* RETINA_SEED_LATTICE or RETINA_SEED_EXPLICIT */
    int32_t lattice_n[2];       /* lattice: dims (tx, ty) for meas_dim 2 (x0 = y0 = 0),
                                   (tx, x0) for meas_dim 1; dim 0 is the slow index;
                                   each 1 .. RETINA_MAX_LATTICE_SIDE, at most 2^24 seeds */
    float lattice_lo[2];
    float lattice_hi[2];        /* cell centres: FP32(lo + (j + 1/2)(hi - lo)/n) formed in FP64 */
    const double* seeds;        /* EXPLICIT: n_par doubles per seed (rounded to FP32 for the
                                   ascent), in the hits' memory space; a seed that is not
                                   finite after that rounding gives RETINA_ERR_INVALID_ARG
                                   (host memory: before any device work; device memory:
                                   found by the ascent, no output written) */
    const int64_t* seed_offsets;/* EXPLICIT: n_events+1, in the hits' memory space */
    int32_t update;             /* RETINA_UPDATE_NEWTON: truncated Newton (Newton-CG in scaled
                                   coordinates); RETINA_UPDATE_GRADIENT: a scaled step of one
                                   bandwidth along the scaled gradient; RETINA_UPDATE_BFGS:
                                   quasi-Newton, the BFGS inverse-Hessian model of -R in scaled
                                   coordinates, (sigma / |g~|) I whenever sigma changes, updated
                                   when s~.y > 0.  Every rule keeps the line search, the step cap
                                   and the FP64 Newton polish. */
    float prune_u;              /* 0: every pass sums over every hit (exact).  > 0: a pass skips
                                   the hits of a plane whose first coordinate lies farther than
                                   sqrt(prune_u) * sigma from that of every candidate a wavefront
                                   holds; each skipped term is below exp(-prune_u), so R moves by
                                   less than n_hits * exp(-prune_u) (e.g. 30: 1e-13 per hit).
                                   Hits are then sorted by that coordinate within each plane;
                                   events with a plane of more than 4096 hits stay exact.
                                   Truncated-Newton rule only. */
} retina_params;

/* One reconstructed track (48 bytes). */
typedef struct {
    double theta[4];    /* (x0, y0, tx, ty); meas_dim 1: (x0, tx, 0, 0) */
    float R;            /* response at sigma_final from the last polish evaluation */
    int32_t n_members;  /* converged seeds in the cluster */
    int32_t seed_index; /* the leader's seed index within its event */
    int32_t flags;      /* the leader's RETINA_* flag bits */
} retina_track;

/* Optional per-seed results (diagnostics and parity checks).  Arrays in the
 * hits' memory space, indexed by global seed number (events in order). */
typedef struct {
    double* theta;      /* n_seeds * n_par, or NULL */
    float* R;           /* n_seeds, or NULL */
    int32_t* flags;     /* n_seeds, or NULL */
    int32_t* n_reval;   /* n_seeds: R-only evaluations spent in line searches, or NULL */
    int64_t capacity;   /* number of seeds the arrays hold */
} retina_seed_out;

/* Create a context on HIP device `device_ordinal` (must be gfx950).  Creates
 * a library-owned stream of default priority.  RETINA_ERR_DEVICE when no such
 * device exists; *out is NULL then. */
int retina_create(int device_ordinal, retina_ctx** out);

/* Release the context and everything it owns.  NULL-safe. */
void retina_destroy(retina_ctx* ctx);

/* Message of the last failure on ctx (static text when ctx is NULL).  Valid
 * until the next call on ctx. */
const char* retina_last_error(const retina_ctx* ctx);

/* Order the context's device work on `hip_stream` (a hipStream_t of the
 * context's device, e.g. torch.cuda.current_stream().cuda_stream); NULL
 * restores the library's own stream. */
int retina_set_stream(retina_ctx* ctx, void* hip_stream);

/* Upper bound (bytes) on the device pool; 0 = unlimited.  Calls whose
 * working set would exceed it return RETINA_ERR_OUT_OF_MEMORY. */
int retina_set_max_device_bytes(retina_ctx* ctx, int64_t max_bytes);

/* Kernel timing with HIP events recorded on the context's stream around each
 * launch of retina_find_tracks / retina_response (and the proposer stage of
 * retina_propose_seeds / retina_find_tracks_learned) while enabled.  Times
 * accumulate (milliseconds) until retina_profile_reset. */
typedef struct {
    int64_t calls;        /* profiled calls since the last reset */
    double ms_stage;      /* hit validation + per-plane sort */
    double ms_plan;       /* work list */
    double ms_hot;        /* ascent (find_tracks) or response kernel */
    double ms_merge;      /* clustering + selection + output */
    double ms_total;      /* first kernel start to last kernel end */
    double exec_pairs;    /* hit-candidate pairs the ascent kernel executed: every lane
                             of a wave holding a seed in the full passes, every
                             thread in the line-search rounds */
    double exec_rpairs;   /* ... of which in R-only line-search rounds */
    double ms_propose;    /* learned seeds: binning, network and seed selection */
} retina_profile;

int retina_set_profiling(retina_ctx* ctx, int32_t enable);
int retina_get_profile(const retina_ctx* ctx, retina_profile* out);
int retina_profile_reset(retina_ctx* ctx);

/* Launch shape of the hot kernels (the autotuner's knobs).
 *   kernel     0: the ascent kernel of retina_find_tracks for batches of at
 *              least 512 seeds per event on average (dense seeding, e.g. a
 *              lattice); 2: the same kernel for sparser batches (e.g. learned
 *              seeds); 1: retina_response
 *   cand       candidate lines per lane: 1 or 2
 *   tile_hits  hits held in LDS per work-group (events with more hits are
 *              streamed through it tile by tile): 256 .. 16384 for
 *              meas_dim 2, 256 .. 32768 for meas_dim 1
 * Results differ between shapes only by FP32 summation order.  The
 * persistent grid is sized from the resulting occupancy. */
int retina_set_tuning(retina_ctx* ctx, int32_t meas_dim, int32_t kernel, int32_t cand,
                      int32_t tile_hits);

/* Current shape: *cand, *tile_hits and the persistent grid size *grid. */
int retina_get_tuning(const retina_ctx* ctx, int32_t meas_dim, int32_t kernel, int32_t* cand,
                      int32_t* tile_hits, int32_t* grid);

/* retina_find_tracks replays one captured HIP graph per (meas_dim, launch
 * shape, profiling) for every batch (default on); 0 launches the kernels one
 * by one.  Results are identical either way. */
int retina_set_graphs(retina_ctx* ctx, int32_t enable);

/* Autotuner: time retina_find_tracks on `sample` (a batch representative of
 * the workload, with `params`) for each ascent launch shape (cand 1, 2 x
 * tile_hits 2048 .. 12288 that fit the device's LDS) and install the
 * fastest.  With cache_path != NULL the choice is stored in that text file
 * keyed by (device arch, meas_dim, workload class = floor(log2(mean hits per
 * event)), seeds per event class) and later calls with the same key reuse it
 * without timing.  The sample's mean seeds per event decide which ascent
 * shape (kernel 0 or 2 of retina_set_tuning) is tuned.  *cand / *tile_hits
 * (may be NULL) receive the choice. */
int retina_autotune(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* sample,
                    const retina_params* params, const char* cache_path, int32_t* cand,
                    int32_t* tile_hits);

/* Eq. (1) and its derivatives at caller-given line parameters.
 *   theta        n_theta * n_par FP32 values, in the hits' memory space
 *   n_theta      number of parameter vectors (>= 0)
 *   theta_offsets n_events+1 offsets into theta (non-decreasing, [0] = 0,
 *                last = n_theta), hits' memory space; NULL allowed when
 *                n_events == 1 (all n_theta belong to event 0)
 *   sigma        bandwidth (> 0)
 *   want         RETINA_WANT_R is implied; | RETINA_WANT_GRAD | RETINA_WANT_HESS
 *   R            n_theta floats
 *   grad         n_theta * n_par floats (NULL unless WANT_GRAD):
 *                dR/dtheta in theta's component order
 *   hess         n_theta * n_par(n_par+1)/2 floats (NULL unless WANT_HESS):
 *                upper triangle row-major (00,01,..,11,12,..)
 * FP32 arithmetic.  Residuals are never formed from a rounded line position:
 * once per (line, plane) the position o + t z is split exactly into a
 * rounded value s and its error l (the product error of one fma plus the
 * error of one addition), and each hit's residual is (x - s) - l, two
 * subtractions whose first is exact for hits near the line. */
int retina_response(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* hits,
                    const float* theta, int64_t n_theta, const int64_t* theta_offsets,
                    float sigma, uint32_t want, float* R, float* grad, float* hess);

/* retina_response for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as retina_response, except:
 *   - hits, theta, theta_offsets, R, grad and hess must be device memory
 *     (hits.mem == RETINA_MEM_DEVICE), else RETINA_ERR_INVALID_ARG;
 *   - the call's workspace (staged hits, per-event offsets, the work list and
 *     the hit-part partial sums) comes from a fixed array of
 *     RETINA_NOALLOC_SCRATCH_BYTES in device memory, one per device, which
 *     the library holds from its load until the process ends; the call
 *     itself makes no hipMalloc / hipFree or other allocation;
 *   - a call whose workspace does not fit returns RETINA_ERR_CAPACITY with
 *     the sizes in retina_last_error, before any device work (about
 *     4 meas_dim bytes per hit plus 4 (n_planes + 7) bytes per event);
 *     when the hit-part partial sums alone do not fit, fewer parts are used,
 *     which changes R, grad and hess only in FP32 summation order.
 * Every call on one device shares that device's array and leaves its
 * contents behind (nothing in it has to start at zero: each call writes what
 * it reads).  Calls that overlap in time on one device, from any context or
 * stream, race on it and must be serialised by the caller. */
int retina_response_noalloc(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* hits,
                            const float* theta, int64_t n_theta, const int64_t* theta_offsets,
                            float sigma, uint32_t want, float* R, float* grad, float* hess);

/* Algorithm 1 on every event of the batch in one device pass: seeds (lattice
 * or explicit), truncated-Newton ascents with sigma continuation, FP64 Newton
 * polish, clustering and selection.
 *   tracks         capacity retina_track slots; event e's tracks are
 *                  tracks[track_offsets[e] .. track_offsets[e+1]-1], in the
 *                  order their clusters were founded (decreasing R)
 *   track_offsets  n_events+1
 *   event_flags    n_events (or NULL): bit 1 (RETINA_STALLED) if any seed of
 *                  the event stalled
 *   seeds_out      optional per-seed results (NULL to skip)
 * RETINA_ERR_CAPACITY: the tracks do not fit; then only
 * track_offsets[n_events] is written, with the required total. */
int retina_find_tracks(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* hits,
                       const retina_params* params, retina_track* tracks, int64_t capacity,
                       int64_t* track_offsets, int32_t* event_flags,
                       const retina_seed_out* seeds_out);

/* ------------------------------------------------------------------------
 * Grid-search Artificial Retina: the grid-based algorithm family that the
 * optimisation method replaces (Section 2: the response at every cell of a
 * parameter grid, groups of high-response cells, one estimate per group).
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n[2];           /* cells per dimension, 1 .. RETINA_MAX_LATTICE_SIDE */
    float lo[2], hi[2];     /* box (finite, lo < hi); cell centres as the seed
                               lattice: FP32(lo + (i + 1/2)(hi - lo)/n), dimension
                               0 slow; meas_dim 2: dims (tx, ty) at x0 = y0 = 0;
                               meas_dim 1: dims (tx, x0) */
    float sigma;            /* bandwidth of the grid response (> 0) */
    float R0;               /* activation threshold (> 0) */
} retina_grid;

/* For every event: R of Eq. (1) at every cell centre (FP32, as
 * retina_response); a peak is a cell whose R reaches R0 and exceeds the R of
 * each of its (up to 8) neighbouring cells inside the grid (an equal
 * neighbour: no peak).  Each peak gives one retina_track: the parameters the
 * grid spans are the R-weighted mean of the centres of the peak's 3 x 3
 * neighbourhood (cells inside the grid, FP64 sums), the others 0; R is the
 * peak cell's response; n_members counts the neighbourhood's cells with
 * R >= R0; seed_index is the peak's cell index; flags 0.
 *   R_grid         n_events * n[0] * n[1] floats (event-major, cell index
 *                  i0 * n[1] + i1), or NULL
 *   tracks         capacity slots; event e's peaks are
 *                  tracks[track_offsets[e] .. track_offsets[e+1]-1] in cell order
 *   track_offsets  n_events+1
 * All arrays in the hits' memory space.  RETINA_ERR_CAPACITY as
 * retina_find_tracks (only track_offsets[n_events] is written). */
int retina_grid_search(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* hits,
                       const retina_grid* grid, float* R_grid, retina_track* tracks, int64_t capacity,
                       int64_t* track_offsets);

/* ------------------------------------------------------------------------
 * Learned seed proposer (a workload extension, not part of the paper).
 *
 * An event's hits are binned into a 128 x 128 image over slope space
 * (x/z, y/z) in [-0.35, 0.35)^2 with two channels (planes of the first and of
 * the second half of the detector), counts log1p-scaled, stored BF16.  A
 * four-layer 3x3 convolutional network (2 -> 64 -> 128 -> 96 -> 1 channels,
 * ReLU between layers, zero padding, 186,625 parameters) maps it to a heatmap
 * whose sigmoid is the probability that a track's slopes fall in the bin.
 * Products run on BF16 MFMA with FP32 accumulation; the FP32 master weights
 * are trained by Adam on a weighted binary cross-entropy (positive weight
 * pos_weight) against targets placed at the bins of given track slopes.
 * Seeds (retina_proposal) are the bin centres, with x0 = y0 = 0, of the best
 * k_max candidate bins by probability (ties to the lower bin index); a bin is
 * a candidate when its probability exceeds tau and, with nms = 1, it is also
 * a strict 3 x 3 local maximum (equal neighbours: the lower index wins).  An
 * event whose best probability is below conf_min (or that has no candidate)
 * falls back to the lattice of the parameters.
 * Parameter layout (retina_model_get_params): per layer W[co][tap][ci] with
 * tap = 3 (dr + 1) + (dc + 1) for input offset (dr, dc) in (row, column) =
 * (tx bin, ty bin), then b[co]; layers in order.
 * ---------------------------------------------------------------------- */
typedef struct retina_model retina_model;

#define RETINA_MODEL_PARAMS 186625

typedef struct retina_proposal {
    int32_t k_max;    /* seeds per event at most, 1 .. 4096 */
    float tau;        /* candidate threshold on the probability, in (0, 1) */
    float conf_min;   /* per-event lattice fallback threshold, in [0, 1] */
    int32_t nms;      /* 1: candidates must be strict 3 x 3 local maxima; 0: any bin */
} retina_proposal;

/* New model on ctx's device: He-normal weights (sd sqrt(2 / (9 Cin))) drawn
 * from a counter-based generator keyed by init_key, zero biases except the
 * last layer's (logit of 0.01). */
int retina_model_create(retina_ctx* ctx, uint64_t init_key, retina_model** out);
/* Binary file: magic, version, step, parameters, Adam moments, checksum. */
int retina_model_save(const retina_model* model, const char* path);
int retina_model_load(retina_ctx* ctx, const char* path, retina_model** out);
void retina_model_free(retina_model* model);
/* RETINA_MODEL_PARAMS FP32 values in the layout above (host memory). */
int retina_model_get_params(const retina_model* model, float* out);
int retina_model_set_params(retina_model* model, const float* in);
/* Adam steps taken so far. */
int64_t retina_model_step(const retina_model* model);

/* One Adam step on a batch: hits (meas_dim 2) and, per event, the slope pairs
 * (tx, ty) to mark in the target heatmap (target_offsets: n_events+1), all in
 * the hits' memory space.  *loss receives the batch's mean loss before the
 * step.  With lr = 0 the step only computes (grad may be non-NULL then:
 * RETINA_MODEL_PARAMS FP32 host values, the gradient of the mean loss). */
int retina_train_step(retina_ctx* ctx, retina_model* model, const retina_geometry* geom,
                      const retina_hits* hits, const double* targets,
                      const int64_t* target_offsets, float lr, float pos_weight, float* loss,
                      float* grad);

/* Network evaluation for inspection: the binned images (n_events * 128 * 128
 * * 2 BF16 values as uint16, may be NULL) and the logits (n_events * 128 *
 * 128 FP32, may be NULL), both in the hits' memory space, row = tx bin. */
int retina_model_forward(retina_ctx* ctx, const retina_model* model, const retina_geometry* geom,
                         const retina_hits* hits, uint16_t* image, float* logits);

/* Seeds from the network for every event: seeds (4 doubles each, (0, 0, tx,
 * ty)) in slots seed_offsets[e] .. seed_offsets[e+1]-1; confidence[e] = the
 * event's best probability; fallback[e] = 1 when the event got the lattice of
 * `params` instead.  Arrays in the hits' memory space; RETINA_ERR_CAPACITY
 * (with seed_offsets[n_events] = the required count) when seeds do not fit. */
int retina_propose_seeds(retina_ctx* ctx, const retina_geometry* geom, const retina_hits* hits,
                         const retina_model* model, const retina_proposal* proposal,
                         const retina_params* params, double* seeds, int64_t capacity,
                         int64_t* seed_offsets, float* confidence, int32_t* fallback);

/* Algorithm 1 with learned seeds: the results of retina_propose_seeds
 * followed by retina_find_tracks on those seeds (explicit seeds), computed in
 * one device pass: staging, network, seed selection, ascent and merge are
 * replayed from one captured HIP graph (graphs enabled), with the work
 * buffers sized by the proposal bound n_events * max(k_max, lattice cells),
 * so no count returns to the host between the proposer and the ascent (the
 * hit total is read at the start and the counters at the end).  The ascent's
 * launch shape follows the bound: the sparse-seeding shape (retina_set_tuning
 * kernel 2) when k_max < 512, the small-cache merge when k_max <= 1024.
 * params gives the method's constants and the fallback lattice; event_flags
 * bit 4 (value 16) marks events that fell back to the lattice.  Outputs and
 * errors as retina_find_tracks. */
int retina_find_tracks_learned(retina_ctx* ctx, const retina_geometry* geom,
                               const retina_hits* hits, const retina_params* params,
                               const retina_model* model, const retina_proposal* proposal,
                               retina_track* tracks, int64_t capacity,
                               int64_t* track_offsets, int32_t* event_flags);

#ifdef __cplusplus
}
#endif

#endif /* RETINA_H */
