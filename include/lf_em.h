/*
 * lf_em.h -- C ABI of the MI355X (gfx950) implementation of the EM static-
 * background reconstruction with a rectified linear camera array
 * (Kaveti, Katt and Singh, "Removing Dynamic Objects for Static Scene
 * Reconstruction using Light Fields", 2020).
 *
 * Problem (Sec. III-A, III-B): K rectified views I_k of a horizontal camera
 * array, the per-view semantic segmentation prior S_P (probability that a
 * pixel is static; S_P = 0 means dynamic) and a dense prior disparity map mu_T
 * interpolated from a triangulation T.  For every pixel of the reference view
 * the library estimates the static-background disparity d (M-step, Sec. III-C,
 * Eq. 6), the posterior q_k that the ray into view k is static (E-step,
 * Sec. III-D, Eq. 7) and the refocused image of the static scene (Eq. 2).
 *
 * Conventions shared by every entry point:
 *   - View k is sampled at x - baselines[k] * d on the same row (Eq. 1 for a
 *     rectified linear array), with linear interpolation along x for
 *     non-integral positions and indices clamped to the image.
 *   - Disparity levels are d_j = d_min + j * d_step, j = 0..D-1.
 *   - Layouts are C order: views uint8 [K][H][W][3] (RGB), S_P float
 *     [K][H][W], mu_T float [H][W], q float [K][H][W], d_idx int32 [H][W]
 *     (level index j), rgb float [H][W][3] in [0,1], hole uint8 [H][W].
 *   - Pointers are host memory unless the flags say device memory
 *     (LF_INPUTS_ON_DEVICE for inputs, LF_OUTPUTS_ON_DEVICE for outputs).
 *   - Every call returns a status code; no exception crosses the ABI.  On an
 *     error lf_last_error() describes it (thread-local, valid until the next
 *     call on the same thread).
 *   - All descriptor, likelihood and posterior arithmetic is FP32 on the GPU;
 *     `storage` only sets the precision in which descriptors and S_P are held
 *     (values are rounded once, to nearest even).
 */
#ifndef LF_EM_H
#define LF_EM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lf_status;
#define LF_OK       0
#define LF_EINVAL   1   /* invalid argument; nothing was launched                    */
#define LF_ENOMEM   2   /* device memory (or the server's HBM budget) exhausted      */
#define LF_EDEVICE  3   /* HIP runtime error or device-side failure                  */
#define LF_EAGAIN   4   /* server queue full; retry later                            */
#define LF_ESTATE   5   /* call out of order (e.g. refocus before any iteration)     */

#define LF_MAX_VIEWS 16

/* Storage precision of descriptors and S_P (arithmetic is always FP32). */
#define LF_F32   0
#define LF_F16   1
#define LF_BF16  2

/* E-step form.  SOFT: posterior P(S_k = 1) of each ray under the per-view
 * factorised likelihood (static exp(lambda - beta/K |f_k - m|^2), dynamic 1);
 * HARD: its arg max per view, the paper's delta / hard assignment (Sec. III-C
 * and III-D).  ENUM_SOFT / ENUM_HARD: the E-step as the paper states it, over
 * all 2^K labelings S (Sec. III-C, last sentence; Sec. III-D): the log weight
 * of S is sum_k ln P(S_k | rho_k) - beta Var_S, Var_S the variance of the
 * static descriptors normalised by their count (0 for fewer than two static
 * views, no lambda); ENUM_SOFT returns the marginals P(S_k = 1), ENUM_HARD
 * the labeling of largest weight (ties: the largest mask, bit k = view k).
 * The enumeration modes need K <= 12.  The M-step is the same in every mode. */
#define LF_SOFT       0
#define LF_HARD       1
#define LF_ENUM_SOFT  2
#define LF_ENUM_HARD  3
#define LF_ENUM_MAX_VIEWS 12

/* flags */
#define LF_INPUTS_ON_DEVICE   0x1u  /* views, S_P, mu_T, q_warm are device pointers   */
#define LF_OUTPUTS_ON_DEVICE  0x2u  /* rgb, d_idx, q, hole, L_pix are device pointers  */
#define LF_EXHAUSTIVE_SWEEP   0x4u  /* evaluate every level with the two-pass spread:   */
                                    /* same results, slower; for verification          */
/* Work-avoiding variants (the paper's speed levers):
 * LF_PRIOR_WINDOW: the M-step searches only the levels within 3 sigma of
 *   mu_T (the level nearest mu_T when none is), the prior "reducing the
 *   search space" (Sec. III-C, disparity prior).
 * LF_DYNAMIC_ONLY: only pixels whose reference ray is dynamic by the prior
 *   threshold (rho_ref < tau_init) are reconstructed, as the paper refocuses
 *   only the dynamic pixels (Sec. III-F, IV-B).  Every other pixel keeps its
 *   first weights, takes the level nearest mu_T, adds nothing to the
 *   objective, and its refocused colour is its reference colour (hole = 0).
 *   The plain context builds a list of the dynamic pixels on the device
 *   when the frame is loaded (lf_em_load) and runs EM over that list only;
 *   the frame server masks the static pixels in its tiles instead. */
#define LF_PRIOR_WINDOW       0x8u
#define LF_DYNAMIC_ONLY       0x10u
/* LF_DEFERRED_CHECK (with LF_INPUTS_ON_DEVICE): lf_em_load / lf_em_init
 * return without waiting for the device-side value check of the inputs, so
 * frames can be queued back to back.  Invalid values are counted on the
 * device (the count stays set across frames) and reported as LF_EINVAL by
 * the next call that waits for the stream (lf_em_check, lf_em_iterate with
 * an objective, or an output copied to the host), which also unloads the
 * frame; results of frames with invalid inputs are meaningless. */
#define LF_DEFERRED_CHECK     0x20u

typedef struct {
    int32_t K, H, W;            /* views, rows, columns; 2 <= K <= 16                 */
    int32_t ref;                /* reference view, baselines[ref] must be 0 (Sec. III-F) */
    float baselines[LF_MAX_VIEWS]; /* view k samples x - baselines[k] * d              */
    float d_min, d_step;        /* disparity levels d_j = d_min + j * d_step, d_step > 0 */
    int32_t D;                  /* number of levels, D >= 1                           */
    float beta;                 /* likelihood sharpness beta >= 0 (Sec. III-C)         */
    float lambda;               /* log ratio static/dynamic likelihood normalisers;   */
                                /* NaN: derived as ln(beta'/pi) + 2 ln(2R),            */
                                /* beta' = beta/K, R = 3060/4096 (needs beta > 0)      */
    float gamma, sigma;         /* disparity prior ln(gamma + exp(-(d-mu)^2/(2 sigma^2))) */
    float tau_init;             /* first-iteration threshold: static iff rho >= tau (0.7) */
    int32_t storage;            /* LF_F32, LF_F16, LF_BF16                            */
    int32_t mode;               /* LF_SOFT, LF_HARD, LF_ENUM_SOFT, LF_ENUM_HARD        */
    uint32_t flags;             /* LF_INPUTS_ON_DEVICE | LF_OUTPUTS_ON_DEVICE |       */
                                /* LF_EXHAUSTIVE_SWEEP | LF_PRIOR_WINDOW |            */
                                /* LF_DYNAMIC_ONLY | LF_DEFERRED_CHECK                */
} lf_params;

typedef struct lf_ctx lf_ctx;   /* opaque; owns all device buffers of one frame shape */

/*
 * lf_em_init -- create a context for frames of shape (K, H, W) and load the
 * first frame: descriptors (3x3 Sobel responses of R+G+B, Sec. III-C), the ray
 * prior rho_k = S_P of view k at the footprint x - b_k mu_T, and the first
 * weights q0_k = [rho_k >= tau_init] (Sec. III-F) or q_warm when given.
 *   out     : receives the context (NULL on failure).
 *   p       : parameters, copied.
 *   views   : uint8 [K][H][W][3]; S_P float [K][H][W] in [0,1];
 *             mu_T float [H][W] finite; q_warm float [K][H][W] in [0,1] or NULL.
 *   hip_stream : hipStream_t all work of this context is queued on (NULL is
 *             the device's null stream); the caller keeps it alive until
 *             lf_em_destroy.
 * Host inputs are copied before return (the caller may free them).  Device
 * inputs must stay valid until the next lf_em_load or lf_em_destroy.
 * Errors: LF_EINVAL (checked before any device work: K outside [2,16], H or W
 * < 1, ref out of range, baselines[ref] != 0, non-finite baselines, D < 1,
 * d_step <= 0, beta < 0, lambda NaN with beta == 0, gamma <= 0, sigma <= 0,
 * tau_init outside [0,1], bad storage/mode/flags, K > 12 in an enumeration mode, max |baseline * level|
 * above 1e6, S_P outside [0,1] or NaN, mu_T not finite or |mu_T| above 1e6,
 * q_warm outside [0,1]; a disparity halo too wide for one workgroup's LDS);
 * LF_ENOMEM; LF_EDEVICE.  Value checks of device-resident inputs run on the
 * device before the frame counts as loaded (one stream synchronisation).
 */
lf_status lf_em_init(lf_ctx **out, const lf_params *p, const uint8_t *views, const float *S_P,
                     const float *mu_T, const float *q_warm, void *hip_stream);

/*
 * lf_em_load -- load a new frame of the same shape and parameters into an
 * existing context (no allocation): recomputes descriptors, ray prior and the
 * first weights exactly as lf_em_init does, and resets the iteration count.
 * Arguments and errors as lf_em_init.
 */
lf_status lf_em_load(lf_ctx *c, const uint8_t *views, const float *S_P, const float *mu_T,
                     const float *q_warm);

/*
 * lf_em_iterate -- run n_iters EM iterations (each an M-step followed by an
 * E-step, the M-step first, Sec. III-B) on the current state.
 *   objective : NULL, or host double [n_iters] receiving the frame objective
 *               sum_p L_t(p) after each iteration, L_t(p) = ln(gamma +
 *               exp(-(d_t-mu)^2/(2 sigma^2))) + sum_k logaddexp(a1_k, a0_k)
 *               (SOFT) or sum_k max(a1_k, a0_k) (HARD); in the enumeration
 *               modes the log prior plus the log of the summed labeling
 *               weights (ENUM_SOFT) or of the largest one (ENUM_HARD), which
 *               EM does not guarantee to be monotone; summed in FP64.
 *               With NULL the call only queues work and returns, and only the
 *               last iteration's objective is formed (for lf_em_state).
 * iterate(a) followed by iterate(b) gives bit-identical state to iterate(a+b).
 * Errors: LF_EINVAL (n_iters < 0), LF_ESTATE (no frame loaded), LF_EDEVICE.
 */
lf_status lf_em_iterate(lf_ctx *c, int32_t n_iters, double *objective);

/*
 * lf_refocus -- refocused image of the static scene at the current disparity
 * (Eq. 2): the mean of the views whose posterior is q_k >= 0.5, each sampled
 * at x - b_k d.  Where no view is static the reference pixel is kept and
 * hole = 1 (Sec. IV-B).  Also returns the state.
 *   rgb    : float [H][W][3] in [0,1] (required).
 *   d_idx  : int32 [H][W] level indices, or NULL.
 *   q      : float [K][H][W] posteriors, or NULL.
 *   hole   : uint8 [H][W], or NULL.
 *   median : 0, or 3 for a 3x3 per-channel median of rgb (Sec. III-E); the
 *            median is applied to every pixel, holes included.
 * Host outputs are complete on return; device outputs are complete when the
 * context's stream reaches this point.
 * Errors: LF_EINVAL (rgb NULL, median not 0 or 3), LF_ESTATE (no iteration
 * since the last load), LF_EDEVICE.
 */
lf_status lf_refocus(lf_ctx *c, float *rgb, int32_t *d_idx, float *q, uint8_t *hole, int32_t median);

/*
 * lf_segmentation_maps -- the updated segmentation (Sec. III-D) of every view
 * in the view's own pixel grid, from the current levels and weights.  The ray
 * of reference pixel (x, y) lands in view k at u = x - baselines[k] * d, taken
 * to the nearest pixel floor(u + 1/2) on row y; where several rays land on one
 * pixel the one with the largest level (the nearest surface) is seen.
 *   labels : uint8 [K][H][W] (device memory with LF_OUTPUTS_ON_DEVICE):
 *            1 = static (q_k >= 0.5), 0 = dynamic, 2 = no reference ray
 *            lands on the pixel.
 * Errors: LF_EINVAL (NULL arguments, W > 65535, D > 32767), LF_ESTATE (no EM
 * iteration since the last load), LF_EDEVICE.
 */
lf_status lf_segmentation_maps(lf_ctx *c, uint8_t *labels);

/*
 * lf_em_sweep_count -- diagnostics of the M-step's work: runs n_iters EM
 * iterations exactly as lf_em_iterate (the same state afterwards) and
 * returns in *level_steps the number of level steps the sweeps took, summed
 * over the waves of 64 pixels and the iterations: a wave that sweeps n
 * levels for its pixels counts n, so 64 * level_steps / (H * W * D * n_iters)
 * is the share of the full sweep's level evaluations the hardware issued
 * (the prior bound skips levels that cannot win; lanes of a wave sweep
 * together).  Waits for the stream.
 * Errors: as lf_em_iterate, LF_EINVAL (level_steps NULL).
 */
lf_status lf_em_sweep_count(lf_ctx *c, int32_t n_iters, uint64_t *level_steps);

/*
 * lf_em_check -- wait for all work queued on the context's stream and report
 * a deferred input check (LF_DEFERRED_CHECK): LF_EINVAL when any frame loaded
 * since the last report had invalid values (the frame is then unloaded).
 * Errors: LF_EINVAL, LF_EDEVICE.
 */
lf_status lf_em_check(lf_ctx *c);

/*
 * lf_em_state -- copy out the current state without refocusing.
 *   q      : float [K][H][W] current weights (q0 before the first iteration), or NULL.
 *   d_idx  : int32 [H][W] disparity levels of the last iteration, or NULL.
 *   L_pix  : float [H][W] per-pixel objective L_t(p) of the last iteration, or NULL.
 * Errors: LF_ESTATE (d_idx or L_pix requested before any iteration), LF_EDEVICE.
 */
lf_status lf_em_state(lf_ctx *c, float *q, int32_t *d_idx, float *L_pix);

/*
 * lf_em_intermediates -- copy out the current frame's per-view inputs to the
 * EM iterations.
 *   feat : [K][H][W][2] descriptors (Gx, Gy) * 2^-12 of the 3x3 Sobel
 *          responses of R+G+B (Sec. III-C), in the storage precision: float
 *          for LF_F32, IEEE binary16 for LF_F16, bfloat16 for LF_BF16
 *          (8 or 4 bytes per pixel), or NULL.
 *   rho  : float [K][H][W] ray prior, S_P of view k (rounded to the storage
 *          precision) interpolated at x - b_k mu_T (Sec. III-B), or NULL.
 * Errors: LF_ESTATE (no frame loaded), LF_EDEVICE.
 */
lf_status lf_em_intermediates(lf_ctx *c, void *feat, float *rho);

/*
 * lf_em_frame_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one whole frame, the work of lf_em_init, lf_em_iterate(n_iters)
 * and lf_refocus with device inputs and outputs, giving the same bits, with
 * no allocation of any kind.  The intermediate buffers (descriptors, ray
 * prior, per-pixel objective, the objective's block sums, the median's input,
 * the dynamic-only work list) live in one fixed device array of
 * LF_NOALLOC_SCRATCH_BYTES that each GPU
 * holds from the library's first use on it until the process ends.
 *   p          : parameters as lf_em_init; the pointer flags are implied
 *                (every pointer below is device memory) and LF_DEFERRED_CHECK
 *                is ignored.
 *   views, S_P, mu_T, q_warm : device inputs as lf_em_init (q_warm nullable).
 *   n_iters    : EM iterations, 1 <= n_iters <= 100000.
 *   rgb        : device float [H][W][3]; hole device uint8 [H][W] or NULL.
 *   d_idx, q   : device int32 [H][W] and float [K][H][W]: the EM state,
 *                written in place (required).
 *   median     : 0 or 3, as lf_refocus.
 *   objective  : device double [n_iters] or NULL: the frame objective after
 *                each iteration, as lf_em_iterate.
 *   invalid    : device uint32 or NULL: receives the number of invalid input
 *                values (S_P outside [0,1], mu_T not finite, q_warm outside
 *                [0,1]); results of a frame with invalid inputs are
 *                meaningless.
 *   hip_stream : stream the work is queued on (NULL: the null stream); the
 *                call returns without waiting for it.
 * Every call on one GPU uses that GPU's one scratch array, which keeps the
 * last call's contents: calls that overlap on one GPU (queued on different
 * streams, or from several threads) race and give undefined results.
 * Errors: LF_EINVAL (as lf_em_init, plus NULL rgb, d_idx or q, n_iters or
 * median out of range, a frame whose buffers exceed the scratch array: about
 * K*H*W*(pair bytes + 8) + H*W*4, plus H*W*12 with the median), LF_EDEVICE.
 */
#define LF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
lf_status lf_em_frame_noalloc(const lf_params *p, const uint8_t *views, const float *S_P, const float *mu_T,
                              const float *q_warm, int32_t n_iters, float *rgb, int32_t *d_idx, float *q,
                              uint8_t *hole, int32_t median, double *objective, uint32_t *invalid,
                              void *hip_stream);

/* lf_em_destroy -- wait for the context's work, free it.  NULL is a no-op. */
void lf_em_destroy(lf_ctx *c);

/* lf_last_error -- message of the last failing call on this thread ("" if none). */
const char *lf_last_error(void);

/* ------------------------------------------------------------------------ */
/* Frame server: continuous batching of frames from many camera streams.     */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Disparity prior construction (Sec. III-C, disparity prior)                */
/* ------------------------------------------------------------------------ */

/* Support-point parameters (the paper follows ELAS and states no numbers;
 * the defaults below are this library's readings). */
typedef struct {
    int32_t step;          /* grid spacing of candidate points, pixels (5)         */
    int32_t radius;        /* matching window (2r+1)^2, r in [0,7] (2)              */
    int32_t texture_min;   /* min sum of |Gx|+|Gy| over the window (2000)           */
    int32_t ratio_num, ratio_den; /* unique iff best*den < second*num (85, 100)     */
    int32_t incon_radius;  /* consistency neighbourhood, pixels (10)                */
    int32_t incon_levels;  /* max level difference of a consistent neighbour (2)    */
    int32_t incon_min;     /* min consistent neighbours to keep a point (3)         */
    int32_t static_min;    /* min static pixels (S_P >= tau_init) in the window (20) */
} lf_support_params;

/*
 * lf_build_prior -- build the dense prior disparity mu_T from the views and
 * S_P (Sec. III-C): support points are matched along the epipolar line over
 * all levels (sum of absolute differences of the integer Sobel responses of
 * R+G+B over the window; the views left and right of the matched view are
 * summed apart and the smaller sum counts), kept when static (the point and
 * static_min window pixels have S_P >= tau_init), textured and unique (the
 * second best taken over levels at least 2 away).  Grid points of the
 * reference are matched against all other views; grid points of every other
 * view a against its non-reference neighbours a-1, a+1, and moved to the
 * reference column x + baselines[a] * d where the reference is dynamic
 * (S_P_ref < tau_init), one per reference pixel (lowest view, then lowest x).
 * Points with fewer than incon_min neighbours (within incon_radius pixels and
 * incon_levels levels) are dropped, the rest sorted by (y, u), and the four
 * image corners added at the level of their nearest point.  mu_T is the
 * piecewise-linear interpolation of the levels' disparities over a Delaunay
 * triangulation of the points (the lowest-index triangle holding a pixel,
 * edges included); with no point, the middle of the level range.
 *   p      : parameters as lf_em_init; integer baselines and levels only,
 *            H, W <= 16384; flags LF_INPUTS_ON_DEVICE / LF_OUTPUTS_ON_DEVICE
 *            place views, S_P / mu_T.
 *   views  : uint8 [K][H][W][3]; S_P float [K][H][W] in [0,1].
 *   mu_T   : float [H][W], written.
 *   points : host int32 [max_points][4] = (u, y, level, view; view -1 for a
 *            corner) or NULL; n_points (nullable) receives the total count.
 *   tris   : host int32 [max_tris][3] counter-clockwise point indices or
 *            NULL; n_tris (nullable) receives the total count.
 *   hip_stream : stream for the device work (NULL: the null stream).
 * Allocates and frees temporary device memory; synchronises the stream.
 * Errors: LF_EINVAL (as lf_em_init, plus fractional geometry, bad support
 * parameters, frames above 16384), LF_ENOMEM, LF_EDEVICE.
 */
/*
 * lf_triangulate -- a Delaunay triangulation of any point set on the host:
 * incremental insertion along a Hilbert curve with exact integer predicates
 * (a point on a circumcircle does not count as inside; points already
 * present are skipped).  lf_build_prior triangulates its points on the
 * device (row strips and side pockets, then rounds of edge flips) and uses
 * this one only if the flip rounds do not settle; where points are
 * cocircular the two may pick different valid triangulations.
 *   xy     : int32 [n][2] points, coordinates in [0, 16383].
 *   tris   : int32 [max_tris][3] counter-clockwise indices or NULL;
 *            n_tris (nullable) receives the count.
 * No device work.  Errors: LF_EINVAL.
 */
lf_status lf_triangulate(const int32_t *xy, int32_t n, int32_t *tris, int32_t max_tris, int32_t *n_tris);

lf_status lf_build_prior(const lf_params *p, const lf_support_params *sp, const uint8_t *views, const float *S_P,
                         float *mu_T, int32_t *points, int32_t max_points, int32_t *n_points, int32_t *tris,
                         int32_t max_tris, int32_t *n_tris, void *hip_stream);

typedef struct lf_server lf_server;   /* opaque */

/* Called once per submitted frame from one of the server's worker threads,
 * after the frame's outputs are in the caller's buffers (status LF_OK), or
 * when the frame failed (LF_EINVAL: invalid values in device inputs;
 * LF_EDEVICE).  A worker in a callback takes no new batch: callbacks should
 * not block for long.  May call lf_submit_frame but not lf_server_drain or
 * lf_server_destroy. */
typedef void (*lf_done_fn)(int64_t frame_id, lf_status status, void *user);

typedef struct {
    int64_t submitted, completed, failed, rejected;  /* rejected: LF_EAGAIN at submission   */
    int64_t batches;                                  /* device launches of admitted frames   */
    double mean_batch_frames;                         /* frames per launch                    */
    double p50_ms, p99_ms, mean_ms, max_ms;           /* submission -> outputs delivered      */
    double wall_s;                                    /* first submission -> last completion  */
    double frames_per_s;                              /* completed / wall_s                   */
    int64_t hbm_in_use, hbm_peak;                     /* bytes of the HBM arena               */
    int64_t max_batch_frames;                         /* most frames in one launch            */
} lf_server_stats_t;

/*
 * lf_server_create -- start a server.  The whole method of Sec. III runs per
 * frame (descriptors, ray prior, n_iters EM iterations, refocus, Eq. 2) for
 * frames of any size, view count (K <= 9), level count and storage, with the
 * previous frame's weights of the same stream (same K, H, W) as its first
 * weights instead of the 0.7 threshold (warm start).  Four worker threads,
 * each with its own HIP stream, take batches of pending frames: every frame
 * of the oldest admissible frame's kernel key (storage, K, integer or
 * fractional shifts, search window or not) that is admissible then, up to 16,
 * runs in one kernel launch.  A frame is admissible when no earlier frame of
 * its stream is running and its buffers fit the HBM budget.
 *   hbm_budget_bytes : device arena (>= 64 KiB) every admitted frame's buffers and every
 *                      stream's warm-start weights come from; frames wait for
 *                      admission until theirs fit.  When nothing running will
 *                      free memory, the warm starts of idle streams are given
 *                      up, oldest first (those streams start cold).
 *   max_streams      : stream ids are 0..max_streams-1.
 *   n_iters          : EM iterations per frame.
 *   staging_bytes    : pinned host staging for host inputs and outputs (0: the
 *                      smaller of the budget and 1 GiB); when full, submission
 *                      of a frame with host buffers returns LF_EAGAIN.  (An
 *                      argument beyond the paper's problem statement: the host
 *                      side of the server's memory budget.)
 * Errors: LF_EINVAL, LF_ENOMEM (arena allocation), LF_EDEVICE.
 */
lf_status lf_server_create(lf_server **out, size_t hbm_budget_bytes, int32_t max_streams, int32_t n_iters,
                           size_t staging_bytes);

/*
 * lf_submit_frame -- queue one frame of stream `stream_id`.
 *   p      : parameters as lf_em_init.  Flags: LF_INPUTS_ON_DEVICE (views,
 *            S_P, mu_T are device memory, used in place: the caller keeps
 *            them unchanged until `done` has run; their values are checked on
 *            the device and a frame with invalid values completes with
 *            LF_EINVAL), LF_OUTPUTS_ON_DEVICE (rgb_out, d_out, q_out are
 *            device memory, written by the kernel), LF_PRIOR_WINDOW,
 *            LF_DYNAMIC_ONLY.  The server's HIP streams do not wait for the
 *            caller's: device inputs must be complete, and device outputs
 *            free of pending work of the caller, when the call is made.
 *   views, S_P, mu_T : inputs as lf_em_init; host inputs are checked and
 *            copied before return.
 *   rgb_out : float [H][W][3] (required); d_out int32 [H][W] (nullable);
 *            q_out float [K][H][W] (nullable).  Written before `done` runs.
 * Frames of one stream complete in submission order; frames of different
 * streams run concurrently, batched into shared launches as they are
 * admitted.  Results do not depend on what else is running.  Output buffers
 * must stay valid until `done` has run for the frame (or lf_server_drain /
 * lf_server_destroy has returned).
 * Errors: LF_EINVAL (as lf_em_init, plus K > 9, stream_id out of range,
 * LF_EXHAUSTIVE_SWEEP or LF_DEFERRED_CHECK set, a frame larger than the
 * arenas), LF_EAGAIN (staging full), or the error a previous device failure
 * left.
 */
lf_status lf_submit_frame(lf_server *s, int32_t stream_id, const lf_params *p, const uint8_t *views,
                          const float *S_P, const float *mu_T, float *rgb_out, int32_t *d_out, float *q_out,
                          lf_done_fn done, void *user, int64_t *frame_id);

/* lf_server_hold -- hold (hold != 0) or release admission: while held, no
 * new batch starts and submitted frames queue, so that a group of frames
 * submitted together is admitted together (they share launches as their
 * kernel keys allow).  lf_server_drain releases a hold. */
lf_status lf_server_hold(lf_server *s, int32_t hold);

/* lf_server_drain -- block until every submitted frame has completed. */
lf_status lf_server_drain(lf_server *s);

/* lf_server_stats / lf_server_reset_stats -- counters and latency percentiles. */
lf_status lf_server_stats(lf_server *s, lf_server_stats_t *out);
lf_status lf_server_reset_stats(lf_server *s);

/* lf_server_destroy -- drain, stop the service thread, free everything. */
void lf_server_destroy(lf_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LF_EM_H */
