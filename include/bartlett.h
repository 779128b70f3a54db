/*
 * bartlett.h - C-ABI of the MI355X batched Bartlett grid search.
 *
 * The operation (paper: "Soft-Coherent Direct Multipath SLAM", Sec. IV-D.2,
 * "An Efficient Birth Proposal PDF"): for every candidate direction u_g of a
 * grid, the Bartlett cost of the observation against the candidate's steering
 * vector, then the candidate(s) of maximum cost and, optionally, the
 * cost-weighted proposal moments. Read for one array and T snapshots with
 * independent source phases:
 *
 *     R     = (1/T) sum_t y_t y_t^H                         (sample covariance)
 *     P[g]  = Re(a_g^H R a_g) / M^2 = (1/T) sum_t |a_g^H y_t|^2 / M^2
 *     a_g[m] = exp(+j 2 pi p_m . u_g)                        (eq. spatial-response-y/z,
 *                                                             directional cosines, Suppl. S-II)
 *
 * Element positions p_m are in wavelengths; observations follow the signal
 * model of eq. (observation-generative) (Sec. II-B).
 *
 * Conventions for every call:
 *  - Pointers marked "dev" are HIP device pointers on the plan's device;
 *    "host" pointers are ordinary host memory, read before the call returns.
 *  - The caller allocates and frees every input, output and workspace buffer.
 *    A plan owns only its own tables. No call except ba_plan_create (and the
 *    other *_create calls) allocates device memory.
 *  - Complex values are interleaved (re, im) float32 pairs ("c64").
 *  - Calls that take a stream enqueue asynchronously on it (NULL = the null
 *    stream). Argument errors are detected and returned before anything is
 *    enqueued. A launch failure returns BA_ERR_DEVICE; faults inside kernels
 *    surface at the caller's next synchronisation.
 *  - A plan may be used by one host thread at a time. Calls that share a
 *    workspace must not overlap.
 *  - No C++ exception crosses this interface.
 */
#ifndef BARTLETT_H
#define BARTLETT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ba_status;
#define BA_OK              0
#define BA_ERR_ARG        -1   /* invalid argument (sizes, null pointers, enums) */
#define BA_ERR_DEVICE     -2   /* a HIP call or kernel launch failed */
#define BA_ERR_NOMEM      -3   /* device allocation failed (plan creation only) */
#define BA_ERR_UNSUPPORTED -4  /* valid request outside what the library implements */
#define BA_ERR_STATE      -5   /* plan not in a state that allows the call */

typedef struct ba_plan_s* ba_plan;

/* Arithmetic of the grid projection (the dominant contraction). Covariance
 * accumulation is always FP32; peak refinement and moments are FP64. */
#define BA_PREC_F32     1   /* FP32 operands, FP32 accumulate (MFMA f32) */
#define BA_PREC_BF16X3  2   /* hi/lo BF16 split, three BF16 MFMA passes, FP32 accumulate */
#define BA_PREC_BF16    3   /* single BF16 pass (precision ablation only) */
#define BA_PREC_F32_VALU 4  /* FP32 on the vector ALUs: the unfused reference kernel, for A/B timing */

/* Grid kinds. */
#define BA_GRID_DIRS      0  /* grid = host double [G][3] unit direction vectors */
#define BA_GRID_ULA_DEG   1  /* grid = host double [G] angles t from broadside (deg), u = (cos t, sin t, 0) */
#define BA_GRID_AZEL_DEG  2  /* grid = host double [G][2] (az, el) deg, u = (cos el cos az, cos el sin az, sin el) */

/* Status as text (static storage). */
const char* ba_status_string(ba_status s);

/* Text of the last error raised on this host thread (static per-thread storage). */
const char* ba_last_error(void);

/* Library version as text. */
const char* ba_version(void);

/*
 * Create a plan: geometry + grid + precision. Builds the steering tables on the
 * host in FP64 (phase p_m . u_g reduced to [-1/2, 1/2) before the complex
 * exponential) and uploads them to the current HIP device, which the plan is
 * then bound to.
 *   n_elem       M, 1 <= M <= 256.
 *   elem_pos_wl  host double [M][3], element positions in wavelengths.
 *   grid_kind    BA_GRID_*; grid host double as described above.
 *   n_grid       G >= 1, G == grid_shape0 * max(grid_shape1, 1).
 *   grid_shape0, grid_shape1  adjacency for peak search: flat g = i0*shape1 + i1;
 *                shape1 <= 1 means a 1-D grid.
 *   wrap0        0: no wrap; 1: dim0 periodic with period shape0; 2: dim0
 *                periodic with period shape0-1, its last row duplicating the
 *                first (never a peak, never a neighbour). Period must be >= 3.
 *   precision    BA_PREC_*.
 * Errors: BA_ERR_ARG, BA_ERR_NOMEM, BA_ERR_DEVICE. On error *out is NULL.
 */
ba_status ba_plan_create(ba_plan* out, int32_t n_elem, const double* elem_pos_wl,
                         int32_t grid_kind, int64_t n_grid, const double* grid,
                         int32_t grid_shape0, int32_t grid_shape1, int32_t wrap0,
                         int32_t precision);

/* Destroy a plan (NULL is accepted). Synchronises the plan's device first. */
ba_status ba_plan_destroy(ba_plan p);

/* Plan facts: M, G, number of refined coordinates per peak (1 for 1-D grids, 2 for 2-D). */
ba_status ba_plan_info(ba_plan p, int32_t* n_elem, int64_t* n_grid, int32_t* ndim);

/*
 * Workspace bytes that ba_run needs for n_trials trials; with_spectrum_out = 0
 * means ba_run is called with P == NULL, so the spectrum is staged in the
 * workspace, except on plans that ba_spectrum_candidates serves: there the
 * workspace holds the covariances and the peak candidates (sized for k = 16)
 * and the spectrum is written only to a P the caller passes.
 */
ba_status ba_workspace_size(ba_plan p, int32_t n_trials, int32_t n_snap,
                            int32_t with_spectrum_out, size_t* bytes);

/*
 * Sample covariance (the R of the Bartlett cost, 1/T normalisation, no mean
 * removal) of B trials.
 *   Y  dev c64 [B][T][M], snapshot-major (each snapshot one contiguous M-vector).
 *   R  dev c64 [B][M][M], row-major R[m][n] = (1/T) sum_t y_t[m] conj(y_t[n]);
 *      both triangles written, exactly Hermitian.
 * Requires B >= 0 (0 is a no-op), T >= 1.
 */
ba_status ba_covariance(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, void* R,
                        void* stream);

/*
 * Workspace bytes ba_spectrum needs for n_trials trials (0 for plans of up to
 * 64 elements; otherwise the real-equivalent covariance of every trial,
 * (2 Mp)^2 * 4 bytes per trial with Mp the padded element count, 128 or 256).
 */
ba_status ba_spectrum_workspace_size(ba_plan p, int32_t n_trials, size_t* bytes);

/*
 * Bartlett spectrum from covariances: P[b][g] = Re(a_g^H R_b a_g) / M^2, computed
 * as x_g^T Q_b x_g / M^2 with x_g = [Re a_g; Im a_g] and Q_b = [[Re R_b, -Im R_b],
 * [Im R_b, Re R_b]] on the matrix cores, in the plan's precision.
 *   R          dev c64 [B][M][M] as written by ba_covariance (any Hermitian matrix).
 *   P          dev float [B][G].
 *   workspace  dev, >= ba_spectrum_workspace_size bytes, 256-byte aligned (may be
 *              NULL when that size is 0).
 */
ba_status ba_spectrum(ba_plan p, int32_t n_trials, const void* R, float* P, void* workspace,
                      size_t workspace_bytes, void* stream);

/*
 * Bartlett spectrum straight from snapshots (snapshot route, cheaper when T < M):
 * P[b][g] = (1/T) sum_t |a_g^H y_t|^2 / M^2.
 */
ba_status ba_spectrum_snapshots(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y,
                                float* P, void* stream);

/*
 * Peak pick and refinement (generalising the paper's argmax candidate to the K
 * largest local maxima). A point is a local maximum when it is strictly
 * greater than every neighbour before it in raster order and greater than or
 * equal to every neighbour after it (8-neighbourhood on 2-D grids, wrap as in
 * the plan); missing neighbours are not compared and any comparison with NaN
 * is false. Peaks are ordered by value, ties to the lower index.
 *   P        dev float [B][G].
 *   k        1 <= k <= 16.
 *   idx      dev int32 [B][k] flat grid index, -1 where fewer than k maxima exist.
 *   val      dev float [B][k] P at the peak, NaN where idx = -1.
 *   refined  dev double [B][k][ndim] (may be NULL): fractional grid index per
 *            axis, i + d with the parabolic vertex d = (P- - P+) / (2 (P- - 2 P0 + P+))
 *            clamped to [-1/2, 1/2], computed in FP64 from the FP32 values; d = 0
 *            on a non-wrapping edge or a zero denominator; NaN where idx = -1.
 */
ba_status ba_peaks(ba_plan p, int32_t n_trials, const float* P, int32_t k, int32_t* idx,
                   float* val, double* refined, void* stream);

/*
 * Spectrum and peak candidates in one pass (Sec. IV-D.2: the cost over the
 * candidate set and its maximum, as ba_spectrum followed by ba_peaks): the
 * projection's epilogue applies the peak rule of ba_peaks to each column range
 * a workgroup covers and keeps that range's k best interior maxima with their
 * neighbour values, plus the values at the range's two ends; ba_peaks_merge
 * then finishes the pick per trial. The spectrum is not re-read, and not
 * written at all when P is NULL.
 * Plans of up to 64 elements on 1-D grids in BA_PREC_F32, BA_PREC_BF16X3 or
 * BA_PREC_BF16 (the register-resident kernels) only; BA_ERR_UNSUPPORTED
 * otherwise, from all three calls.
 *   R      dev c64 [B][M][M] (ba_covariance).
 *   k      1 <= k <= 16; the same k must reach ba_peaks_merge.
 *   P      dev float [B][G] or NULL; when given, bit-identical to ba_spectrum
 *          of the same plan.
 *   cand   dev, >= ba_candidates_size(p, B, k) bytes, 16-byte aligned; opaque
 *          records owned by the caller, every byte of the sized part written.
 */
ba_status ba_candidates_size(ba_plan p, int32_t n_trials, int32_t k, size_t* bytes);
ba_status ba_spectrum_candidates(ba_plan p, int32_t n_trials, const void* R, int32_t k, float* P,
                                 void* cand, size_t cand_bytes, void* stream);

/*
 * Per-trial merge of the records ba_spectrum_candidates wrote for the same
 * plan, n_trials and k (enqueue it after that call on the same stream).
 *   idx/val/refined as ba_peaks, with identical values (same rule, same order,
 *   the refinement from the same three FP32 values).
 */
ba_status ba_peaks_merge(ba_plan p, int32_t n_trials, int32_t k, const void* cand, int32_t* idx,
                         float* val, double* refined, void* stream);

/*
 * Proposal moments of Sec. IV-D.2: weights w_g = P_g / sum P over the distinct
 * grid points, mean mu = coordinates of the global maximum (lowest index among
 * equal maxima), covariance C = sum_g w_g (x_g - mu)(x_g - mu)^T. Coordinates x
 * are degrees for angle grids (azimuth differences wrapped into [-180, 180))
 * and the unit vector for BA_GRID_DIRS; d = 1, 2 or 3 accordingly.
 *   mu_cov  dev double [B][d + d*d]: mu then C row-major.
 */
ba_status ba_proposal_moments(ba_plan p, int32_t n_trials, const float* P, double* mu_cov,
                              void* stream);

/*
 * Gaussian birth proposal of Sec. IV-D.2 from the moments above: particle n
 * of trial b is mu + L z[b][n] with C = L L^T, and its importance weight is
 * proportional to the indicator of the search region over the proposal
 * density (the target being uniform on the region), normalised to sum to one
 * per trial. The region is the span of the grid's coordinates; on an az/el
 * grid whose azimuth axis wraps, azimuth is periodic (always inside; the
 * particle is reported wrapped, its density taken at the unwrapped draw).
 *   mu_cov     dev double [B][d + d*d] (ba_proposal_moments).
 *   z          dev double [B][N][d]: standard normal draws, supplied by the caller.
 *   particles  dev double [B][N][d]; weights dev double [B][N].
 * A covariance that is not positive definite gives particles = mu and equal
 * weights; a trial with no particle inside the region gets NaN weights.
 * Angle grids only: BA_ERR_UNSUPPORTED for BA_GRID_DIRS.
 */
ba_status ba_proposal_sample(ba_plan p, int32_t n_trials, const double* mu_cov, int32_t n_particles,
                             const double* z, double* particles, double* weights, void* stream);

/*
 * The whole path for B trials: covariance -> spectrum -> peaks (+refinement);
 * on plans that ba_spectrum_candidates serves, covariance -> spectrum with
 * candidates -> merge (same results).
 *   Y          dev c64 [B][T][M].
 *   P          dev float [B][G] or NULL (then staged in the workspace, or not
 *              written at all on the candidate path).
 *   idx/val/refined as ba_peaks (refined may be NULL).
 *   workspace  dev, at least ba_workspace_size(p, B, T, P != NULL) bytes,
 *              256-byte aligned.
 */
ba_status ba_run(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, int32_t k,
                 float* P, int32_t* idx, float* val, double* refined,
                 void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of the fixed device scratch array behind ba_run_noalloc (one per GPU). */
#define BA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/*
 * ba_run without a workspace argument and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). The workspace is a
 * file-scope device array of BA_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends; its address is looked
 * up once per device, on the first call there.
 *   Arguments, layouts and results are those of ba_run (same kernels, same
 *   values bit for bit). The plan's device must be the current device.
 *   Errors: BA_ERR_ARG when ba_workspace_size(p, n_trials, n_snap, P != NULL)
 *   exceeds BA_NOALLOC_SCRATCH_BYTES (split the batch, or pass P so the
 *   spectrum is not staged), and every error of ba_run; BA_ERR_DEVICE if the
 *   array's address cannot be obtained.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (other streams or host threads) race.
 */
ba_status ba_run_noalloc(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, int32_t k,
                         float* P, int32_t* idx, float* val, double* refined, void* stream);


/* ------------------------------------------------------------------ ragged batches */

/* Route of one trial through the spectrum: the covariance form a^H R a, or the
 * snapshot form (1/T) sum_t |a^H y_t|^2 (fewer flops when T < M). Both give the
 * same Bartlett cost. */
#define BA_ROUTE_AUTO      -1   /* tuned table if ba_ragged_autotune ran, else snapshots iff T < M */
#define BA_ROUTE_COV        0
#define BA_ROUTE_SNAPSHOTS  1

/* One trial of an uneven batch. */
typedef struct {
  int64_t y_offset;  /* complex offset of the trial's [T][M] snapshot block in the pool */
  int32_t n_elem;    /* M, 1 <= M <= min(128, plan elements): the plan's first M elements */
  int32_t n_snap;    /* T >= 1 */
  int32_t k;         /* peaks wanted, 1 <= k <= kmax */
  int32_t route;     /* BA_ROUTE_*; the snapshot route needs T <= the padded size (8, 16, 32, 64, 128) */
} ba_trial;

typedef struct ba_ragged_s* ba_ragged;

/*
 * Prepare an uneven batch of trials (different M, T and K) that share the
 * plan's grid and the first elements of its geometry (a uniform array sliced
 * to M elements is the same array up to a phase centre, which leaves the
 * Bartlett cost unchanged). Builds per-size-class steering tables, orders the
 * trials longest first, and captures one persistent fused launch
 * (covariance -> spectrum -> peaks per trial, trials taken from an atomic
 * ticket) in a HIP graph. On 1-D grids, trials of up to 32 elements on the
 * covariance route run packed by default: one per wave, eight per ticket
 * (ba_ragged_autotune decides per class). Buffers are bound here
 * (ba_ragged_bind rebinds them); ba_ragged_launch replays.
 *   plan        FP32 plan, G <= 16384, 1-D or 2-D grid.
 *   desc        host, n_trials entries (copied).
 *   kmax        1..8: output row width; entries past a trial's k are -1 / NaN.
 *   Y_pool      dev c64 [pool_elems]; every trial's block must lie inside.
 *   P           dev float [B][G] or NULL; idx dev int32 [B][kmax]; val dev float
 *               [B][kmax]; refined dev double [B][kmax][ndim] or NULL.
 * Allocates device memory (tables, descriptors); errors: BA_ERR_ARG,
 * BA_ERR_NOMEM, BA_ERR_DEVICE.
 */
ba_status ba_ragged_create(ba_ragged* out, ba_plan plan, int32_t n_trials, const ba_trial* desc,
                           int32_t kmax, const void* Y_pool, int64_t pool_elems, float* P,
                           int32_t* idx, float* val, double* refined);

/* Replay the captured launch on a stream. The plan and the bound buffers must
 * stay alive; replays on one handle must not overlap. */
ba_status ba_ragged_launch(ba_ragged r, void* stream);

/*
 * Bind other buffers to the handle for the replays that follow on `stream`
 * (same meaning and sizes as in ba_ragged_create; the trials' layout in the
 * pool is the one given at creation). The captured launch reads its buffer
 * addresses from device memory, so the new buffers take effect in stream
 * order without re-capturing: a replay already enqueued keeps the old ones.
 *   pool_elems  must cover every trial's block.
 * Errors: BA_ERR_ARG, BA_ERR_DEVICE.
 */
ba_status ba_ragged_bind(ba_ragged r, const void* Y_pool, int64_t pool_elems, float* P, int32_t* idx, float* val,
                         double* refined, void* stream);

/*
 * Autotune on this batch: per size class, the MFMA tile (waves along rows vs
 * along grid columns); for the 8-, 16- and 32-element classes on 1-D grids,
 * packed (one trial per wave) or one trial per workgroup; per (size class,
 * log2 T bucket), the route. Candidates are timed with HIP events on up to
 * max_probe trials each (32 * max_probe for the packing choice, so that
 * both layouts fill as many workgroups for several rounds; best of `repeats`
 * launches after one warm-up). Results are cached in cache_path (text, may be
 * NULL) keyed by device, grid size and class/bucket; the graph is re-captured.
 * Synchronous; writes outputs of the probed trials as a side effect.
 */
ba_status ba_ragged_autotune(ba_ragged r, const char* cache_path, int32_t repeats, int32_t max_probe);

/* Route each trial takes (host int32 [B], BA_ROUTE_COV or BA_ROUTE_SNAPSHOTS). */
ba_status ba_ragged_routes(ba_ragged r, int32_t* routes);

/* Waves along rows chosen per size class (host int32 [5], classes 8..128). */
ba_status ba_ragged_config(ba_ragged r, int32_t* wr_per_class);

/* Whether each size class runs packed, one trial per wave (host int32 [5],
 * classes 8..128; 1 = packed; only the first three classes on 1-D grids can be). */
ba_status ba_ragged_packed(ba_ragged r, int32_t* packed_per_class);

/* Destroy (NULL accepted); synchronises the device first. */
ba_status ba_ragged_destroy(ba_ragged r);

/* ------------------------------------------------------------------ learned proposal network */

/* The paper has no learned part (hybrid learned / model-based processing is
 * named as future work in its conclusions). This network predicts coarse
 * directions from the sample covariance so that only narrow windows of the
 * Bartlett grid are scanned; the full grid search is its fallback. */

typedef struct ba_mlp_s* ba_mlp;

/*
 * Pack covariances for the network: per trial, M diagonal real parts, then the
 * strict upper triangle's real parts, then its imaginary parts (row-major),
 * all times M / tr(R): M^2 floats.
 *   R  dev c64 [B][M][M];  X  dev float [B][M*M].
 */
ba_status ba_pack_covariance(int32_t n_elem, int32_t n_trials, const void* R, float* X, void* stream);

/*
 * Network d_in -> n_hidden x (affine + exact GELU, d_hidden wide) -> affine ->
 * d_out, weights W [out][in] and biases, FP32 master copies. precision
 * BA_PREC_BF16: GEMM operands rounded to BF16 (round to nearest even), FP32
 * accumulate; BA_PREC_F32: FP32 throughout. Allocates parameters, Adam moments
 * and activations for up to max_batch rows; the calls below allocate nothing.
 * Weights start uniform in +-1/sqrt(fan_in) from `seed`.
 */
ba_status ba_mlp_create(ba_mlp* out, int32_t d_in, int32_t d_hidden, int32_t n_hidden, int32_t d_out,
                        int32_t max_batch, int32_t precision, uint64_t seed);
ba_status ba_mlp_destroy(ba_mlp n);
ba_status ba_mlp_num_params(ba_mlp n, int64_t* count);

/* Host copies of all parameters, in the order W1, b1, W2, b2, ... (row-major).
 * set_weights also clears the Adam moments and step count. Synchronous. */
ba_status ba_mlp_get_weights(ba_mlp n, float* host, int64_t count);
ba_status ba_mlp_set_weights(ba_mlp n, const float* host, int64_t count);

/* Y = net(X) for B rows (any B >= 0; processed max_batch rows at a time).
 * X dev float [B][d_in]; Y dev float [B][d_out]. */
ba_status ba_mlp_forward(ba_mlp n, int32_t B, const float* X, float* Y, void* stream);

/*
 * Masked mean-squared error L = sum m (y - t)^2 / sum m and its gradient with
 * respect to every parameter (same order as the weights), B <= max_batch.
 *   T, mask  dev float [B][d_out] (mask may be NULL = all ones);
 *   grads_out dev float [num_params]; loss_out dev float scalar or NULL.
 */
ba_status ba_mlp_gradients(ba_mlp n, int32_t B, const float* X, const float* T, const float* mask,
                           float* grads_out, float* loss_out, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradients of the loss above, B <= max_batch. */
ba_status ba_mlp_train_step(ba_mlp n, int32_t B, const float* X, const float* T, const float* mask,
                            float lr, float* loss_out, void* stream);

/* Input and output widths of a network. */
ba_status ba_mlp_dims(ba_mlp n, int32_t* d_in, int32_t* d_out);

/* Workspace bytes of ba_propose_refine. */
ba_status ba_propose_workspace_size(ba_plan plan, int32_t n_trials, int32_t d_out, int32_t k, size_t* bytes);

/*
 * Learned proposal + refinement: pack R, run the network (its first k outputs
 * are sin(direction) of the sources), scan only the full-grid points within
 * +-half_window of each proposal (nearest full-grid index), and take each
 * window's maximum (ties to the lower index) as a peak, refined as on the
 * full grid. A trial falls back to the full-grid search (covariance already
 * given) when a proposal or any spectrum value inside a window is NaN, when a
 * window maximum lies on a window edge that is not a grid edge, when two
 * windows find the same point, or when a peak's normalised cost P M / tr(R)
 * is not at least tau. Outputs are then the full-grid ones.
 *   plan        FP32 plan, M <= 64, uniform 1-D angle grid (BA_GRID_ULA_DEG).
 *   net         d_in = M^2, d_out >= k.
 *   R           dev c64 [B][M][M]; k in [1, 8]; half_window in [1, 100]; tau in [0, 1].
 *   idx, val, refined  dev [B][k] (refined in grid units); fell_back dev uint8 [B].
 *   n_fallback  dev int32 (may be NULL): receives the number of trials that
 *               fell back (written on the stream; 0 when n_trials = 0).
 * Enqueues everything and never waits for the device: the fallback kernels
 * are launched for the whole batch and read the number of fallback trials on
 * the device (so the call can be captured in a graph).
 */
ba_status ba_propose_refine(ba_plan plan, ba_mlp net, int32_t n_trials, const void* R, int32_t k,
                            int32_t half_window, float tau, int32_t* idx, float* val, double* refined,
                            uint8_t* fell_back, int32_t* n_fallback, void* workspace, size_t workspace_bytes,
                            void* stream);

/* ---------------------------------------------------------------- residual projector
 *
 * Sec. IV-D.2: before the Bartlett cost is evaluated, each observation is
 * replaced by its residual z~ = Pi z, Pi = I - Psi Psi^+, the component
 * orthogonal to the span of the steering vectors Psi of the features already
 * known. For T snapshots the residuals' covariance is R~ = Pi R Pi.
 */

/*
 * Residual covariance R~ = Pi R Pi for every trial.
 *   R      dev c64 [B][M][M], Hermitian (as ba_covariance writes it; the kernel
 *          reads both triangles as one Hermitian matrix).
 *   S      columns of Psi per trial, 0..16 (0 copies R).
 *   Psi    dev c64 [B][S][M]: column s of trial b is the contiguous M-vector at
 *          Psi + (b S + s) M. Columns whose part orthogonal to the earlier
 *          columns has squared norm <= 1e-10 of their own (duplicates, zero
 *          columns) add nothing to the span.
 *   R_out  dev c64 [B][M][M], exactly Hermitian; may be R itself (in place).
 * The projector algebra runs in FP64; R~ is rounded to FP32 once.
 * Errors: BA_ERR_ARG for S outside [0, 16] or NULL buffers, synchronously.
 */
ba_status ba_residual_covariance(ba_plan p, int32_t n_trials, const void* R, int32_t S, const void* Psi,
                                 void* R_out, void* stream);

/* Workspace bytes of ba_sequential_peaks (256-byte aligned base required). */
ba_status ba_sequential_workspace_size(ba_plan p, int32_t n_trials, size_t* bytes);

/*
 * Project-out-and-rescan detection: pass 0 takes the largest local maximum
 * of the plain spectrum; pass j > 0 projects the steering vectors of the
 * j grid points found so far out of R (ba_residual_covariance with Psi the
 * plan's steering columns), evaluates the spectrum of the residual
 * covariance at the plan's precision, and takes its largest local maximum.
 *   R        dev c64 [B][M][M] (not modified).
 *   k        passes, 1..16.
 *   idx      dev int32 [B][k] in detection order (-1 if a pass finds no
 *            local maximum; such a pass adds no column).
 *   val      dev f32 [B][k]: the residual spectrum at the point, in its pass.
 *   refined  dev f64 [B][k][ndim] (may be NULL): parabolic vertex on that
 *            pass's spectrum, grid units.
 * Cost: k spectrum evaluations per trial. Asynchronous on stream.
 */
ba_status ba_sequential_peaks(ba_plan p, int32_t n_trials, const void* R, int32_t k, int32_t* idx, float* val,
                              double* refined, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- coherent multi-array cost
 *
 * The paper's own birth-proposal workload (Sec. IV-D.2): the coherent
 * Bartlett spectrum P(s) = |sum_j (1/N_z) z_j^H psi_j(s)|^2 over J arrays for
 * candidate SFV positions s, where psi_j(s) is the path-loss compensated
 * wideband URA response (Sec. II-B) of the path that the surface with SFV s
 * creates between the terminal and array j: virtual anchor, Householder mirror
 * and array rotation of Sec. II-A. Element order of psi_j: frequency slowest,
 * then the horizontal element, then the vertical one (b (x) a_y (x) a_z); the
 * pilot spectrum is flat; baseband frequencies are equally spaced over the
 * bandwidth and centred on zero; elements sit at half a wavelength, centred.
 */
typedef struct ba_coherent_s* ba_coherent;

/*
 * Plan of one geometry: builds the steering table of every candidate at every
 * array on the device (FP64 geometry and phases, stored FP32).
 *   pa_pos      host double [J][3]: array positions (m).
 *   pa_rot      host double [J][3][3] row-major: array rotations (local -> global).
 *   n_y, n_z    URA elements per axis (1..16); n_f baseband frequencies (1..64);
 *               J * n_f * n_y * n_z <= 2048.
 *   fc          carrier (Hz); bandwidth (Hz, >= 0).
 *   p_mt        host double [3]: terminal position (m).
 *   candidates  host double [n_cand][3]: SFV positions (m), nonzero, n_cand <= 2^26.
 * Table memory: 8 * J * N_z * ceil(n_cand / 128) * 128 bytes.
 */
ba_status ba_coherent_create(ba_coherent* out, int32_t n_arrays, const double* pa_pos, const double* pa_rot,
                             int32_t n_y, int32_t n_z, int32_t n_f, double fc, double bandwidth,
                             const double* p_mt, int64_t n_cand, const double* candidates);
ba_status ba_coherent_destroy(ba_coherent h);
/* n_obs = J * N_z (complex values per trial), n_cand = candidates. */
ba_status ba_coherent_info(ba_coherent h, int32_t* n_obs, int64_t* n_cand);
/* Workspace bytes of ba_coherent_spectrum and ba_coherent_moments (one buffer
 * serves both; 256-byte aligned base required). */
ba_status ba_coherent_workspace_size(ba_coherent h, int32_t n_trials, size_t* bytes);

/*
 * The cost for every (trial, candidate).
 *   Z  dev c64 [B][J][N_z]: each trial's (residual) observations, array by array.
 *   P  dev float [B][n_cand].
 * FP32 MFMA with FP32 accumulation. Asynchronous on stream.
 */
ba_status ba_coherent_spectrum(ba_coherent h, int32_t n_trials, const void* Z, float* P, void* workspace,
                               size_t workspace_bytes, void* stream);

/*
 * Proposal moments over the candidates (Sec. IV-D.2): weights P / sum P, mean
 * = the candidate of maximum cost (lowest index among equal maxima),
 * covariance = weighted second central moment, in metres, accumulated in FP64
 * about the maximum (sum P (x - mu)(x - mu)^T / sum P).
 *   mu_cov  dev double [B][3 + 9].
 */
ba_status ba_coherent_moments(ba_coherent h, int32_t n_trials, const float* P, double* mu_cov, void* workspace,
                              size_t workspace_bytes, void* stream);

/*
 * Birth particles of the new feature's SFV position (Sec. IV-D.2 proposal
 * density, and the birth-particle weights of Sec. IV-D): particle n of trial
 * b is mu + L z[b][n] with C = L L^T from ba_coherent_moments, and its
 * importance weight is proportional to the indicator of the partition over
 * the proposal density (a target uniform on the partition), normalised to
 * sum to one per trial. The partition is the axis-aligned box spanned by the
 * plan's candidates (candidates are drawn from the partition).
 *   mu_cov     dev double [B][12] (ba_coherent_moments).
 *   z          dev double [B][N][3]: standard normal draws, supplied by the caller.
 *   particles  dev double [B][N][3] (m); weights dev double [B][N].
 * A covariance that is not positive definite gives particles = mu and equal
 * weights; a trial with no particle inside the box gets NaN weights.
 */
ba_status ba_coherent_sample(ba_coherent h, int32_t n_trials, const double* mu_cov, int32_t n_particles,
                             const double* z, double* particles, double* weights, void* stream);


/* ---------------------------------------------------------------- particle update messages
 *
 * The likelihood-to-variable update messages of the particle-based BP step
 * (Sec. IV-C; Supplementary Sec. S-V, efficient implementation), each a
 * complex Gaussian log-density log CN(z_j; mu, C) of the observation z_j of
 * array j with covariance eta I plus a low-rank part:
 *   iota  MT state message at every (MT particle p, array j);
 *   nu    noise variance message at every (noise particle eta^(j,p), array j);
 *   kappa PF state message at every (feature s, PF particle p, array j), PF
 *         existence r = 1, and per (s, j) at r = 0;
 *   omega PR existence message per (s, j) at r = 0 and r = 1.
 * Feature s = 0 is the line-of-sight path, s >= 1 surfaces given by SFVs. PF
 * particle p of every feature is paired with MT particle p, so a_s^(j,p) is
 * the response at array j of feature s's path for MT position x^p and SFV
 * v_s^p (geometry of Sec. II-A, response of Sec. II-B, as for the coherent
 * cost above: path loss included, element order b (x) a_y (x) a_z, centred
 * half-wavelength supports and frequency bins).
 * Moments (rho_s = sum_p w_alpha,s^p, zeta_s = zeta_s^(j)(1), eta~_j =
 * sum_p w_xi^(j,p) eta^(j,p)):
 *   iota: mu = sum_s zeta_s rho_s mu_s^p a_s, C = eta~ I + sum_s c_s a_s a_s^H,
 *         c_s = zeta_s rho_s (gamma_s^p + |mu_s^p|^2 (1 - zeta_s rho_s));
 *   kappa: mu = r zeta_s mu_s^p a_s + sum_{t != s} m3_t,
 *          C = r q a_s a_s^H + eta~ I + sum_{t != s} m_t m_t^H,
 *          q = zeta_s (gamma_s^p + |mu_s^p|^2 (1 - zeta_s));
 *   omega: mu = r m4_s + sum_{t != s} m3_t, C = r w_s w_s^H + eta~ I + sum_{t != s} m_t m_t^H;
 *   nu:   mu = sum_t m3_t, C = eta^(j,p) I + sum_t m_t m_t^H;
 * with the particle averages (weights w_beta^p of the MT particles)
 *   m_s = rho_s zeta_s sum_p w_beta^p sqrt(gamma_s^p + |mu_s^p|^2 (1 - zeta_s rho_s)) a_s^(j,p),
 *   w_s = rho_s sum_p w_beta^p sqrt(gamma_s^p + |mu_s^p|^2 (1 - rho_s)) a_s^(j,p),
 *   m4_s = rho_s sum_p w_beta^p mu_s^p a_s^(j,p), m3_s = zeta_s m4_s.
 * Values are full log-densities (normalisation included). FP64 throughout.
 */
typedef struct ba_msgs_s* ba_msgs;

/*
 * Geometry of the arrays (copied to the device).
 *   pa_pos  host double [J][3] (m); pa_rot host double [J][3][3] row-major
 *           (local -> global); J in [1, 16].
 *   n_y, n_z in [1, 16]; n_f in [1, 64]; N_z = n_f n_y n_z <= 1024.
 *   fc (Hz) > 0; bandwidth (Hz) >= 0 (bins spaced bandwidth / (n_f - 1)).
 */
ba_status ba_msgs_create(ba_msgs* out, int32_t n_arrays, const double* pa_pos, const double* pa_rot, int32_t n_y,
                         int32_t n_z, int32_t n_f, double fc, double bandwidth);
ba_status ba_msgs_destroy(ba_msgs h);
/* Workspace bytes for n_feat features and n_part particles (256-byte aligned base required). */
ba_status ba_msgs_workspace_size(ba_msgs h, int32_t n_feat, int32_t n_part, size_t* bytes);

/* One time step's inputs; every pointer is device memory, complex values are
 * interleaved (re, im) doubles. */
typedef struct {
  int32_t n_feat;        /* S in [1, 16], LOS included */
  int32_t n_part;        /* P in [1, 2^26] */
  const void* z;         /* complex [J][N_z] observations */
  const double* mt_pos;  /* [P][3] MT position particles (m) */
  const double* w_beta;  /* [P] MT particle weights */
  const double* sfv;     /* [S][P][3] SFV particles (m), nonzero for s >= 1; row 0 unused */
  const double* gamma;   /* [S][P] amplitude prior variance particles (>= 0) */
  const void* mu;        /* complex [S][P] amplitude prior mean particles */
  const double* w_alpha; /* [S][P] PF particle weights (sum = existence probability) */
  const double* zeta;    /* [S][J] PR existence probabilities zeta(r = 1) */
  const double* eta;     /* [J][P] noise variance particles (> 0) */
  const double* w_xi;    /* [J][P] noise particle weights */
} ba_msg_inputs;

/* Outputs (device memory, double); any may be NULL to skip it. */
typedef struct {
  double* log_iota;   /* [J][P] */
  double* log_nu;     /* [J][P] */
  double* log_kappa;  /* [S][J][P], r = 1 */
  double* log_kappa0; /* [S][J], r = 0 */
  double* log_omega;  /* [S][J][2], r = 0 then r = 1 */
} ba_msg_outputs;

/*
 * Evaluate the messages of one time step. Argument errors (sizes, NULL
 * inputs, workspace smaller than ba_msgs_workspace_size) return BA_ERR_ARG
 * before anything is enqueued; values are not checked on the host (a
 * non-positive eta or a zero SFV gives NaN or Inf). Asynchronous on stream.
 */
ba_status ba_update_messages(ba_msgs h, const ba_msg_inputs* in, const ba_msg_outputs* out, void* workspace,
                             size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BARTLETT_H */
