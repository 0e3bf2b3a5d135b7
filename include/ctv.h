/*
 * ctv.h - C ABI of the MI355X (gfx950) complex constrained total-variation
 * denoiser and its proximal-gradient phase-retrieval application.
 *
 * Method: Gao & Cao, "A Complex Constrained Total Variation Image Denoising
 * Algorithm with Application to Phase Retrieval" (arXiv 2109.05496).
 *   problem        min_{x in C} 0.5 ||x - b||_F^2 + lambda ||x||_TV      (Eq. 1)
 *   TV kinds       type-I / type-II, isotropic / anisotropic             (Eqs. 7-10)
 *   constraint C   none (C = C^{m x n}) or |x_jk| <= 1                   (Eq. 25, projection Eq. 26)
 *                  optionally intersected with a 0/1 support mask (x = 0 where the mask is 0)
 *   solver         fast gradient projection on the dual                  (Algorithm 2, Eqs. 16-20, 33-37)
 *   output         x = P_C(b - lambda L^T q_K)                           (Eq. 18)
 *   PR application FISTA (Algorithm 1) with angular-spectrum propagation (Eq. 23),
 *                  amplitude data term (Eq. 24) and its gradient (Eq. 27).
 *
 * Conventions for every entry point
 *   - Images are complex64, interleaved (re, im) float pairs, row-major
 *     [batch][m][n]; m = rows (the paper's index j), n = columns (index k).
 *   - Pointers are DEVICE pointers unless the name ends in _host.
 *   - The caller owns every buffer. Only *_plan_create (and the batched
 *     autotuner, per candidate plan) allocates device memory (freed in
 *     *_plan_destroy); no other call allocates. ctv_denoise (every schedule),
 *     ctv_denoise_backward, pr_prox_grad with a fixed step and the stage entry
 *     points enqueue kernels only, so they can be captured into a HIP graph;
 *     ctv_denoise_batched is itself one graph launch, and the autotuners and
 *     pr_prox_grad's line search synchronise the host.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL = the
 *     default stream). They return after enqueueing work.
 *   - Arguments are validated before any device work; on error nothing is
 *     enqueued and a message is available from ctv_last_error() (thread-local).
 *   - NaN/Inf inputs are not checked; they propagate.
 *   - FGP state ("dual state") layout: float[batch][2][m][n][4]. Plane 0 holds
 *     q_k, plane 1 holds the extrapolated point r_{k+1} of Algorithm 2, line 5.
 *     Per pixel the four floats are (r1, s1, r2, s2) = (Re Q1, Im Q1, Re Q2,
 *     Im Q2) with Q1 = r^(1) + i s^(1) (vertical differences) and
 *     Q2 = r^(2) + i s^(2) (horizontal differences); the entries that do not
 *     exist in the paper (Q1 on the last row, Q2 on the last column) are 0.
 */
#ifndef CTV_H
#define CTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ctv_status;
#define CTV_OK 0
#define CTV_ERR_INVALID_ARG (-1)
#define CTV_ERR_WORKSPACE (-2)
#define CTV_ERR_HIP (-3)
#define CTV_ERR_UNSUPPORTED (-4)

/* TV kinds: type-I isotropic (Eq. 7), type-I anisotropic (Eq. 8),
 * type-II isotropic (Eq. 9), type-II anisotropic (Eq. 10). */
#define CTV_TV_1I 0
#define CTV_TV_1A 1
#define CTV_TV_2I 2
#define CTV_TV_2A 3

/* Constraint sets: CTV_C_NONE is C = C^{m x n} (the unconstrained "TV" model of
 * Section VI-A); CTV_C_MODULUS is Eq. (25), |x_jk| <= 1. */
#define CTV_C_NONE 0
#define CTV_C_MODULUS 1

/* Dual iteration: the fast gradient projection (Algorithm 2) or the plain
 * gradient projection (Eq. 21). Both share the step and the projections; the
 * plain one drops the momentum (beta_k = 0), converging as O(1/k) instead of
 * O(1/k^2) in the dual objective. */
#define CTV_M_FGP 0
#define CTV_M_GP 1

/* Launch schedule of ctv_denoise (a tuning choice, never a change of result).
 * CTV_S_FLOW needs ckpt_every = 0, iters > 0 and the default 8 x 8 column tile;
 * its tiles pass the dual state through device-coherent accesses and wait (a
 * bounded wait) for their neighbours. CTV_S_AUTO uses CTV_S_STEPS, which is
 * faster on MI355X, except that an image of at most 64 x 64 pixels (default
 * tile, no checkpoints) runs up to 480 iterations per launch in one tile with
 * no halo. */
#define CTV_S_AUTO 0
#define CTV_S_STEPS 1
#define CTV_S_FLOW 2

typedef void* ctv_stream_t; /* hipStream_t */

typedef struct {
  uint32_t struct_size; /* sizeof(ctv_params) */
  int32_t tv_kind;      /* CTV_TV_* */
  float alpha;          /* type-II weight in [0, 1] (Eqs. 9-10); ignored for type-I */
  int32_t constraint;   /* CTV_C_* */
  int32_t iters;        /* K >= 0, FGP iterations (Algorithm 2) */
  int32_t fuse;         /* at most this many iterations fused per kernel launch, 1..16 (a run is
                           split into the fewest launches, iterations spread evenly); 0 = automatic */
  int32_t tile_waves;   /* tile shape (tuning): 0 = automatic; 4, 8 or 16 wave64s per workgroup in
                           the column-register tile; -1 = the LDS-staged tile (4 waves); -2 = the
                           row-sweep tile (8 waves sweeping down a 64-column strip one iteration
                           behind each other, no vertical halo; at most 10 fused iterations) */
  int32_t tile_rows;    /* rows per thread: 0 = automatic; column tile 4 or 8 (with waves 4: 8 only);
                           LDS tile 4, 8 or 16; row-sweep tile: output rows of a tile, a multiple of 4 in
                           [16, 1024] */
  int32_t method;       /* CTV_M_FGP: Algorithm 2 with the t_k extrapolation; CTV_M_GP: the
                           unaccelerated gradient projection of Eq. (21), r_k = q_{k-1} */
  int32_t schedule;     /* CTV_S_AUTO, CTV_S_STEPS (one kernel launch per fused step) or
                           CTV_S_FLOW (one persistent launch; tiles wait only on their
                           neighbours' previous step). Results are identical. */
} ctv_params;

/* Library version (major*10000 + minor*100 + patch) and last error message. */
int32_t ctv_version(void);
const char* ctv_last_error(void);

/* Test hook for the failure path of CTV_S_FLOW (callers: the library's own
 * tests). on != 0 makes every later CTV_S_FLOW launch in this process start
 * with its wait-failure flag raised, so each neighbour wait gives up at once,
 * as after a real timeout; the kernels still exit normally and x (and
 * state_out) come back NaN. on = 0 restores normal runs. Always CTV_OK. */
ctv_status ctv_debug_flow_fail_waits(int32_t on);

/* Workspace (and checkpoint storage) needed by ctv_denoise /
 * ctv_denoise_backward for `batch` images of m x n.
 *   ws_bytes    : scratch for ctv_denoise; ctv_denoise_backward needs
 *                 ctv_backward_workspace_size() instead.
 *   saved_bytes : size of the `saved` checkpoint buffer for ckpt_every > 0
 *                 (ceil(K / ckpt_every) - 1 dual states), else 0.
 * Either output pointer may be NULL. */
ctv_status ctv_workspace_size(const ctv_params* p, int32_t batch, int32_t m, int32_t n,
                              int32_t ckpt_every, size_t* ws_bytes, size_t* saved_bytes);

/* Launch configuration ctv_denoise uses for these sizes: iterations fused per
 * kernel launch, tile region rows (tiles are 64 columns wide) and the tile
 * shape in ctv_params' tile_waves / tile_rows terms. Host-only; any output
 * pointer may be NULL.
 * Fails with CTV_ERR_INVALID_ARG for an unsupported tile_waves/tile_rows pair. */
ctv_status ctv_tiling(const ctv_params* p, int32_t batch, int32_t m, int32_t n, int32_t* fuse_out,
                      int32_t* region_rows_out, int32_t* tile_waves_out, int32_t* tile_rows_out);

/* ctv_denoise - K FGP iterations (Algorithm 2) on each of `batch` equally
 * sized images followed by Eq. (18).
 *   b           [batch][m][n] complex64 observation.
 *   lambda_host [batch] host floats, lambda >= 0 per image. lambda = 0 or K = 0
 *               gives x = P_C(b), the exact solution / Eq. (18) at q = 0.
 *   support     [m][n] uint8 (0 = outside the support), shared by the batch; NULL = none.
 *   x           [batch][m][n] complex64 output (may not alias b).
 *   gap         [batch] doubles (device) receiving the duality gap
 *               lambda * sum_groups(||(L x)_g|| - <q_g, (L x)_g>) >= 0 at the
 *               returned x (derived from Appendix A); NULL = not computed.
 *   state_in    dual state (layout above) to resume from after k0 iterations
 *               already done; NULL = cold start q_0 = 0 (Algorithm 2, line 1), then k0 must be 0.
 *   k0          iterations already performed (t_{k0} continues the t sequence).
 *   state_out   dual state after k0 + K iterations, or NULL.
 *   ckpt_every  0, or c > 0 to store the dual state at k = c, 2c, ... < K in
 *               `saved` (the state at k = 0 is the cold start); needed by
 *               ctv_denoise_backward; requires state_in == NULL.
 *   saved       [ceil(K/c) - 1][batch][2][m][n][4] floats, or NULL when no slot is needed.
 *   ws          workspace of at least ctv_workspace_size() bytes.
 * With a support and a cold start, the dual stays exactly zero at pixels that
 * are outside the support and have no support pixel below or to the right
 * (from q_0 = 0, y vanishes at every pixel their differences read), and x = 0
 * there: tiles made only of such pixels are not computed (results are bitwise
 * those of computing them, for finite b). The call then launches two small
 * kernels per tiling that list the other tiles.
 * Errors: CTV_ERR_INVALID_ARG (null/negative/out-of-range arguments, unknown
 * kind/constraint, alpha outside [0,1], lambda < 0, non-finite or inside
 * (0, 1e-12) - there the float32 dual step 1/(8 lambda) and the backward's
 * 1/(8 lambda^2) overflow; pass 0 instead: since P_C is nonexpansive and
 * |L^T q| <= 4 per channel on the dual set, P_C(b) is within 6 lambda of the
 * K-step result at every pixel - m or n < 1, struct_size mismatch),
 * CTV_ERR_WORKSPACE (ws_bytes too small), CTV_ERR_HIP (a launch failed).
 * CTV_S_FLOW's neighbour waits are bounded (about a second each); if one gives
 * up, the affected pixels of x and of state_out are NaN (never silently wrong
 * values). */
ctv_status ctv_denoise(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                       const float* lambda_host, const uint8_t* support, float* x, double* gap,
                       const float* state_in, int32_t k0, float* state_out, int32_t ckpt_every,
                       float* saved, void* ws, size_t ws_bytes, ctv_stream_t stream);

/* ctv_denoise_noalloc - ctv_denoise for callers that cannot allocate device
 * memory (code under HIP-graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same cold-start solve (no resume state, no
 * checkpoints) with the workspace taken from a fixed device array that the
 * library holds on every GPU it runs on until the process ends, instead of a
 * caller buffer. The call allocates nothing; results are bitwise those of
 * ctv_denoise. The current device must be the one `stream` belongs to.
 *   Arguments as in ctv_denoise (gap may be NULL).
 *   Limit: ctv_workspace_size(p, batch, m, n, 0) must not exceed
 *   CTV_NOALLOC_SCRATCH_BYTES (72 MiB: one 1024 x 1024 image, or four
 *   512 x 512 images); larger problems fail with CTV_ERR_WORKSPACE before any
 *   device work.
 *   Calls on one GPU share that GPU's array: two calls that may overlap in time
 *   (different streams, or different host threads without ordering) race and
 *   give wrong results; calls ordered on one stream are safe. Nothing needs to
 *   start at zero: the kernels write every workspace word they read.
 * Errors: those of ctv_denoise, plus CTV_ERR_WORKSPACE above the limit. */
#define CTV_NOALLOC_SCRATCH_BYTES (72u * 1024u * 1024u)
ctv_status ctv_denoise_noalloc(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                               const float* lambda_host, const uint8_t* support, float* x, double* gap,
                               ctv_stream_t stream);

/* ---------------------------------------------------------------------------
 * Batched ragged denoising: many images of different sizes, each with its own
 * lambda, TV kind, alpha and K, in one HIP-graph launch. Per image the result
 * equals ctv_denoise on that image alone (bitwise, for the same fuse setting).
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t offset;          /* first pixel of the image in the packed buffers (complex elements) */
  int32_t m, n;            /* rows, columns (>= 1) */
  float lambda;            /* >= 0 */
  int32_t tv_kind;         /* CTV_TV_* */
  float alpha;             /* [0, 1] */
  int32_t iters;           /* K >= 0 */
  int64_t support_offset;  /* byte offset of this image's m x n mask in the packed support buffer; -1 = none */
} ctv_image_desc;

typedef struct ctv_batched_plan ctv_batched_plan;

/* Builds the tile work list, the momentum table and a HIP graph with one
 * kernel node per fused step; allocates the plan's device tables. `common`
 * supplies constraint and fuse (tv_kind/alpha/iters are taken per image).
 * Images must not overlap in the packed buffers. */
ctv_status ctv_batched_plan_create(const ctv_image_desc* descs_host, int32_t count,
                                   const ctv_params* common, ctv_batched_plan** plan);
ctv_status ctv_batched_workspace_size(const ctv_batched_plan* plan, size_t* ws_bytes);
/* Runs the plan: b_packed and x_packed are complex64 buffers addressed by the
 * descriptors' offsets; support_packed is a uint8 buffer (NULL if no image has
 * a mask). One graph launch on `stream`; kernel arguments are refreshed when
 * the pointers change between calls. As in ctv_denoise, the tiles of images
 * with a support whose pixels all keep a zero dual are not computed (two
 * graph nodes ahead of the steps list the others). */
ctv_status ctv_denoise_batched(ctv_batched_plan* plan, const float* b_packed,
                               const uint8_t* support_packed, float* x_packed, void* ws,
                               size_t ws_bytes, ctv_stream_t stream);
ctv_status ctv_batched_plan_destroy(ctv_batched_plan* plan);
/* Launch configuration the plan was built with (iterations fused per launch,
 * tile_waves, tile_rows); any output pointer may be NULL. */
ctv_status ctv_batched_plan_tiling(const ctv_batched_plan* plan, int32_t* fuse_out,
                                   int32_t* tile_waves_out, int32_t* tile_rows_out);

/* ---------------------------------------------------------------------------
 * Autotuning of the fused forward kernel's launch configuration: the tile
 * shape and the number of FGP iterations fused per launch (the tiling and
 * temporal fusion of the iteration loop of Algorithm 2; the paper runs it
 * unfused). Every configuration computes the same iterates bit for bit, so a
 * tuning choice changes only the speed.
 *
 * ctv_autotune runs ctv_denoise on the caller's problem (same arguments as a
 * plain call without gap, state or checkpoints) once per candidate (tile
 * shape, fuse) pair, times `reps` further calls of each on `stream` with HIP
 * events (median), and records the fastest in a process-wide table keyed by
 * the device's architecture, its CU count and the HIP runtime version, and by (tv_kind, constraint, method,
 * batch, m, n, iters); the support mask is not part of the key. ctv_denoise,
 * ctv_tiling and pr_prox_grad (its inner prox) use a recorded entry whenever
 * params.fuse, tile_waves and tile_rows are all 0 (and schedule is not
 * CTV_S_FLOW); ctv_denoise_backward always uses the default.
 * ctv_batched_autotune does the same for a batched plan: it builds, runs and
 * destroys one plan per candidate and records the fastest under a key derived
 * from (constraint, method, and per image m, n, effective K, tv_kind, has
 * support); ctv_batched_plan_create with fuse and tile 0 then uses it. Its
 * ws must hold ctv_batched_workspace_size() bytes of a plan of these images
 * (the same for every configuration).
 *   reps         1..100 timed calls per candidate.
 *   results      host array of max_results entries (may be NULL with
 *                max_results = 0): every candidate timed, in the order tried.
 *   num_results  host: number of candidates timed (may be NULL).
 *   best         host: the recorded configuration (may be NULL).
 * x (x_packed) holds the solution afterwards: every candidate computes it.
 * Both calls block the host (they synchronize on their events), allocate
 * nothing in ctv_autotune (ctv_batched_autotune allocates and frees each
 * candidate's plan tables) and fail with CTV_ERR_INVALID_ARG while `stream`
 * is being captured. The table is shared by all threads (guarded by a lock).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t fuse;        /* at most this many iterations fused per launch */
  int32_t tile_waves;  /* as ctv_params.tile_waves */
  int32_t tile_rows;   /* as ctv_params.tile_rows */
  float ms;            /* median time of one call, milliseconds */
} ctv_tuning;

ctv_status ctv_autotune(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                        const float* lambda_host, const uint8_t* support, float* x, void* ws,
                        size_t ws_bytes, int32_t reps, ctv_tuning* results, int32_t max_results,
                        int32_t* num_results, ctv_tuning* best, ctv_stream_t stream);
ctv_status ctv_batched_autotune(const ctv_image_desc* descs_host, int32_t count, const ctv_params* common,
                                const float* b_packed, const uint8_t* support_packed, float* x_packed,
                                void* ws, size_t ws_bytes, int32_t reps, ctv_tuning* results, int32_t max_results,
                                int32_t* num_results, ctv_tuning* best, ctv_stream_t stream);
/* Whether the table holds an entry for this plain problem on the current
 * device (*found = 1, *entry = the entry) or not (*found = 0). entry may be NULL. */
ctv_status ctv_tune_lookup(const ctv_params* p, int32_t batch, int32_t m, int32_t n, int32_t* found,
                           ctv_tuning* entry);
/* The same for a batched plan of these images (the key of ctv_batched_autotune). */
ctv_status ctv_batched_tune_lookup(const ctv_image_desc* descs_host, int32_t count, const ctv_params* common,
                                   int32_t* found, ctv_tuning* entry);
/* The tuning table as text, one JSON object per line ("arch", "key", "fuse",
 * "tile_waves", "tile_rows", "ms", "what"). Loading merges the file's entries
 * into the table (an entry with the same arch and key is replaced); a
 * malformed line fails with CTV_ERR_INVALID_ARG and merges nothing. Entries of
 * other architectures are kept and saved again but never used. */
ctv_status ctv_tune_cache_save(const char* path);
ctv_status ctv_tune_cache_load(const char* path);
ctv_status ctv_tune_cache_clear(void);
int32_t ctv_tune_cache_size(void);

/* ---------------------------------------------------------------------------
 * ctv_denoise_backward - exact reverse-mode derivative of the K-step map
 * (b, lambda) -> x of ctv_denoise (chain rule through Algorithm 2 and Eq. 18).
 * Requires the forward call's checkpoints (ckpt_every > 0, same b, lambda,
 * support and params). Complex gradients use the real-pair convention of
 * Section II: grad = dL/dRe + i dL/dIm (what PyTorch returns for a real loss).
 * At the non-smooth points of the projections the Jacobian is the identity
 * when the norm is <= the radius (zero for a zero radius). With a support, the
 * reverse steps skip the tiles where the adjoint state provably stays zero
 * (the pixels where ctv_denoise's dual does), as ctv_denoise does.
 *   grad_x       [batch][m][n] complex64 incoming gradient.
 *   grad_b       [batch][m][n] complex64 output.
 *   grad_lambda  [batch] floats (device) output; 0 where lambda = 0 or K = 0.
 *   ws           at least ctv_backward_workspace_size() bytes.
 * ------------------------------------------------------------------------- */
ctv_status ctv_backward_workspace_size(const ctv_params* p, int32_t batch, int32_t m, int32_t n,
                                       int32_t ckpt_every, size_t* ws_bytes);
ctv_status ctv_denoise_backward(const ctv_params* p, int32_t batch, int32_t m, int32_t n,
                                const float* b, const float* lambda_host, const uint8_t* support,
                                int32_t ckpt_every, const float* saved, const float* grad_x,
                                float* grad_b, float* grad_lambda, void* ws, size_t ws_bytes,
                                ctv_stream_t stream);

/* ---------------------------------------------------------------------------
 * Phase retrieval (Section V): FISTA (Algorithm 1) on
 *   F(x) + tau ||x||_TV + I_C(x),  F(x) = sum_d 0.5 || |A_d x| - sqrt(y_d) ||^2 (Eq. 24),
 * A_d = angular-spectrum propagation over distance d (Eq. 23), gradient Eq. (27),
 * prox = ctv FGP with lambda = tau * gamma (Eq. 15), cold dual start per prox
 * unless warm_start is set.
 * Step size: fixed, or (line_search = 1) chosen by backtracking in the manner of
 * Beck and Teboulle's FISTA, since Section III-B selects gamma by a line search
 * without naming one: starting from the previous step, gamma is multiplied by
 * ls_shrink until x = prox(z - gamma grad F(z)) satisfies
 *   F(x) <= F(z) + Re<grad F(z), x - z> + ||x - z||^2 / (2 gamma),
 * at most ls_max_trials prox evaluations per outer iteration (the last one is
 * accepted). Each test reads four doubles back to the host, so a call with the
 * line search synchronises `stream` once per trial.
 * m and n must be powers of two in [2, 4096].
 * ------------------------------------------------------------------------- */
typedef struct {
  uint32_t struct_size;          /* sizeof(pr_params) */
  int32_t num_meas;              /* D >= 1 */
  const double* distances_host;  /* [D] propagation distances (m) */
  double wavelength;             /* illumination wavelength (m), > 0 */
  double pixel;                  /* sampling pitch (m), > 0 */
  float tau;                     /* TV weight: 0, or tau * (initial gamma) >= 1e-12 (a smaller prox
                                    weight, reachable only by backtracking, is taken as 0) */
  float gamma;                   /* step size > 0 (0 = 1/D) */
  int32_t outer_iters;           /* K_out >= 0 */
  ctv_params inner;              /* prox: kind, alpha, constraint, iters = K_in, fuse */
  int32_t init_backprop;         /* 1: x0 = (1/D) sum_d A_d^H sqrt(y_d); 0: x0 is read from x */
  int32_t accelerate;            /* 1: FISTA (Algorithm 1); 0: plain proximal gradient (Eq. 14) */
  int32_t line_search;           /* 1: backtracking step (above); 0: fixed gamma */
  float ls_shrink;               /* backtracking factor in (0, 1) (line_search = 1) */
  int32_t ls_max_trials;         /* >= 1 prox evaluations per outer iteration (line_search = 1) */
  int32_t warm_start;            /* 1: each prox starts from the previous prox's last dual iterate
                                    (momentum restarted: r_1 = q_0, t_1 = 1); 0: q_0 = 0 */
} pr_params;

ctv_status pr_workspace_size(const pr_params* p, int32_t m, int32_t n, size_t* ws_bytes);
/*   y           [D][m][n] float intensities (>= 0).
 *   x           [m][n] complex64: input x0 when init_backprop = 0; output x_K.
 *   loss_trace  [K_out] floats (device) receiving F(z_k) at each gradient point, or NULL.
 *   gamma_trace [K_out] floats (device) receiving the step used in each outer iteration, or NULL. */
ctv_status pr_prox_grad(const pr_params* p, int32_t m, int32_t n, const float* y, float* x,
                        float* loss_trace, float* gamma_trace, void* ws, size_t ws_bytes,
                        ctv_stream_t stream);

/* pr_ip - the iterative projection (IP) method that Section VI-A compares
 * against: K = outer_iters iterations, each projecting the estimate onto the
 * measured-modulus set of every distance in turn,
 *   x <- P_C(A_d^H[sqrt(y_d) A_d x / |A_d x|])   for d = 0 .. D-1
 * (unit phasor where A_d x = 0; P_C of Eq. 26 with C from inner.constraint:
 * CTV_C_MODULUS is the nonnegative-absorption set of Eq. 25, CTV_C_NONE
 * projects nothing). With several distances the paper does not fix the order;
 * the distances are taken in turn. Uses num_meas, distances_host, wavelength,
 * pixel, outer_iters, init_backprop and inner.constraint (inner must be a
 * valid ctv_params); tau, gamma and the prox settings are ignored.
 *   y, x, ws, ws_bytes as in pr_prox_grad.
 *   loss_trace [K] floats (device) receiving F(x_k) (Eq. 24 summed over d) at
 *              the start of each iteration, or NULL.
 * Errors as pr_prox_grad's. */
ctv_status pr_ip(const pr_params* p, int32_t m, int32_t n, const float* y, float* x, float* loss_trace, void* ws,
                 size_t ws_bytes, ctv_stream_t stream);

/* Stage entry points of the phase-retrieval path (same conventions).
 * ctv_fft2: 2-D DFT of a complex64 [batch][m][n] array (m, n powers of two in
 *   [2, 4096]); out = sum x exp(-2 pi i (j j'/m + k k'/n)); inverse: + sign and
 *   1/(m n). out may equal in. ws: ctv_fft2_workspace_size() bytes (twiddles and
 *   one transposed copy of the batch).
 * pr_forward: out[d] = A_d x for every distance (out is [D][m][n] complex64).
 * pr_gradient: grad = sum_d A_d^H[(A_d x / |A_d x|)(|A_d x| - sqrt(y_d))] (Eq. 27,
 *   unit phasor where A_d x = 0), and loss (device float, may be NULL) = F(x).
 * Both take the workspace of pr_workspace_size(). */
ctv_status ctv_fft2_workspace_size(int32_t batch, int32_t m, int32_t n, size_t* ws_bytes);
ctv_status ctv_fft2(int32_t batch, int32_t m, int32_t n, const float* in, float* out, int32_t inverse,
                    void* ws, size_t ws_bytes, ctv_stream_t stream);
ctv_status pr_forward(const pr_params* p, int32_t m, int32_t n, const float* x, float* out,
                      void* ws, size_t ws_bytes, ctv_stream_t stream);
ctv_status pr_gradient(const pr_params* p, int32_t m, int32_t n, const float* y, const float* x,
                       float* grad, float* loss, void* ws, size_t ws_bytes, ctv_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CTV_H */
