/*
 * msibm.h - C ABI of the MI355X (gfx950) multi-scale hierarchical block matching
 * library (libmsibm.so).
 *
 * The method (Kaushik and Lall, "Fast Hierarchical depth map computation from
 * stereo", Section III): build a K-level Gaussian pyramid of a rectified stereo
 * pair, find every pixel's disparity at the coarsest level by a full
 * winner-take-all search of the zero-mean normalised cross-correlation (ZNCC,
 * Eq. 2) over the disparity search image of Eq. 1 (Eqs. 3-4), then at each finer
 * level search only a small interval around the nearest-neighbour-upsampled
 * coarser disparity (Eqs. 8-9, first branch).  On the plain per-pair forward
 * the library also runs the paper's optional steps: the confidence gating
 * (the full search where the bicubic-doubled coarser cost is low, Eqs. 8-9
 * second branch; the re-pick by neighbourhood-averaged scores, Eqs. 5-7), the
 * selective median filter (Eq. 10) and a blurred level 0.  Two additions are not
 * in the paper: a differentiable finest level (soft-argmax with its backward)
 * and a soft output at every level with the backward through the pyramid.
 *
 * Conventions used by every entry point
 *   - All image, map and gradient pointers are DEVICE pointers allocated by the
 *     caller (for instance by torch).  The library never allocates memory that
 *     the caller sees; scratch comes from a caller-provided workspace whose size
 *     the *_workspace_size functions give.  Pointers are not retained after a
 *     call returns (except inside a captured graph, see MSIBM_FLAG_GRAPH).
 *     Internally the batched path keeps pinned host staging, a capture stream
 *     and cached graphs per device until the process ends.
 *   - Images are row-major with a row pitch counted in ELEMENTS (pitch >= width).
 *     Pixel (i, j) is row i, column j.
 *   - Disparity convention: left pixel (i, j) is compared with right pixel
 *     (i, j - z) (left-reference convention for rectified pairs).  Candidate z
 *     is valid iff 0 <= z <= min(D_k - 1, j).
 *   - Level k has height ceil(H_{k-1}/2) and width ceil(W_{k-1}/2) and searches
 *     D_k = ceil(D / 2^k) candidates (the paper's d_max^k = D_max / 2^k with D
 *     counting candidates).
 *   - Window reads clamp to the nearest edge pixel.  A window whose variance is
 *     at most var_eps is flat and scores 0.  Ties break to the lowest z.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *     call only enqueues work on that stream and returns; outputs are valid once
 *     the stream has reached that point.
 *   - Every entry point validates its arguments before enqueuing anything.  On
 *     a validation error nothing is enqueued and a negative msibm_status is
 *     returned; msibm_last_error() then describes it (thread-local string).
 *     MSIBM_ERR_HIP reports a failure of the HIP runtime (launch or capture).
 */
#ifndef MSIBM_H
#define MSIBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t msibm_status;

#define MSIBM_OK 0
#define MSIBM_ERR_INVALID_ARG (-1) /* null pointer, negative size, bad enum   */
#define MSIBM_ERR_SHAPE (-2)       /* sizes inconsistent or too small/large   */
#define MSIBM_ERR_WORKSPACE (-3)   /* workspace missing or too small          */
#define MSIBM_ERR_UNSUPPORTED (-4) /* parameter outside the compiled range    */
#define MSIBM_ERR_HIP (-5)         /* HIP runtime error                       */

/* element types of input images */
#define MSIBM_U8 0  /* uint8_t, intensity range 0..255 */
#define MSIBM_F32 1 /* float                             */

#define MSIBM_MAX_LEVELS 8        /* K <= 8                                  */
#define MSIBM_MAX_HALF_WINDOW 6   /* n <= 6: windows up to 13 x 13           */
#define MSIBM_MAX_RADIUS 4        /* refine and soft radius <= 4             */
#define MSIBM_MAX_DISP 2048       /* D <= 2048                               */
#define MSIBM_MAX_PAIRS 256       /* pairs per msibm_disparity call          */

/* flags of msibm_config.flags */
#define MSIBM_FLAG_BATCHED 1    /* one launch per stage for all pairs together  */
#define MSIBM_FLAG_GRAPH 2      /* with BATCHED: capture once, replay a hipGraph */
#define MSIBM_FLAG_PREBLUR 8    /* plain and batched forward: level 0 is matched on the
                                   input blurred with the pyramid's 5x5 binomial
                                   kernel (every pixel, clamp-to-edge; the blur
                                   of the original image of Section IV)         */
#define MSIBM_FLAG_MEDIAN 16    /* plain and batched forward: every level's hard map goes
                                   through the selective median filter (Eq. 10)
                                   with threshold median_alpha                  */
#define MSIBM_FLAG_GATED 32     /* plain and batched forward: the confidence gating of
                                   Sections III.B-C at every hard level: below the
                                   coarsest level, the full search where the
                                   bicubic-doubled coarser cost is <= gate_beta
                                   (Eqs. 8-9); then the re-pick of pixels with
                                   cost <= gate_alpha by the 5x5-averaged scores
                                   (Eqs. 5-7); the cost carried down and returned
                                   is that of Eq. 7                             */
#define MSIBM_FLAG_PERSISTENT 4 /* reserved: single-launch persistent scheduler;
                                   switched off, fails with UNSUPPORTED       */

/* One rectified stereo pair.  left/right are device pointers of `dtype`. */
typedef struct msibm_pair {
    const void* left;
    const void* right;
    int32_t dtype;      /* MSIBM_U8 or MSIBM_F32                               */
    int32_t height;     /* H >= 1                                              */
    int32_t width;      /* W >= 1                                              */
    int32_t pitch;      /* row pitch of left and right, elements, >= W         */
    int32_t max_disp;   /* D: candidates 0..D-1 at level 0, 1 <= D <= 2048     */
    int32_t num_levels; /* K: pyramid images (level 0 = input); 0 = automatic:
                           the smallest K with D_{K-1} <= 32                   */
} msibm_pair;

/* Matching parameters shared by all pairs of a call. */
typedef struct msibm_config {
    int32_t half_window;   /* n: windows are (2n+1) x (2n+1), 1 <= n <= 6       */
    int32_t refine_radius; /* r: restricted search [c-r, c+r], 0 <= r <= 4       */
    float var_eps;         /* flat-window variance floor, intensity^2 units     */
    int32_t soft_radius;   /* r_s: 0 = hard WTA at level 0; 1..4 = level 0 also
                              computes the soft-argmax over [c-r_s, c+r_s] and
                              its hard WTA is taken over that interval          */
    float tau;             /* soft-argmax temperature, > 0 when soft_radius > 0 */
    int32_t flags;         /* MSIBM_FLAG_*                                      */
    int32_t half_window_levels[MSIBM_MAX_LEVELS];
                           /* per-level n: entry k (1 <= n_k <= 6) replaces
                              half_window at level k, 0 keeps half_window; for
                              the block size that shrinks by 2 per level
                              (Section III), e.g. {5, 2, 1}                    */
    float median_alpha;    /* with MSIBM_FLAG_MEDIAN: pixels with matched cost
                              <= median_alpha are filtered (the paper: 0.9)      */
    float gate_alpha;      /* with MSIBM_FLAG_GATED: re-pick threshold alpha    */
    float gate_beta;       /* with MSIBM_FLAG_GATED: full-search threshold beta
                              (the paper: alpha = beta = 0.9)                   */
} msibm_config;

/* Thread-local description of the last error of this thread ("" if none). */
const char* msibm_last_error(void);

/* Library version string. */
const char* msibm_version(void);

/*
 * Kernel shapes of the matching kernel (bits of a variant):
 *   1  right window statistics staged in LDS with the right tile (full
 *      searches only; otherwise each thread reads them from global memory),
 *   2  XCD-aware tile order (each of the 8 XCDs takes one contiguous run of
 *      tiles, so neighbouring tiles share their halos in one L2),
 *   4  candidate split (full and restricted searches, not the soft level):
 *      2-row tiles whose 4 waves score disjoint windows of candidates for the
 *      same pixels (every 4th window of a full search; a quarter of each
 *      block's 2r + 1 candidates in a restricted one) and combine their
 *      winners; four times the workgroups, a fraction of each thread's work
 *      (for small levels),
 *   8  fixed window (restricted searches whose whole candidate range, about
 *      D_k candidates, fits one staged chunk): both tiles are staged at once
 *      before any prior is read, with no workgroup-wide range step,
 *  16  short right chunk: the right tile is staged 48 (full search) or 128
 *      (restricted search) candidates at a time instead of 96 or 320 (less
 *      LDS per workgroup, more chunks where a tile's candidates spread),
 *  32  tall tiles: 16 pixel rows and 8 waves per workgroup instead of 8 rows
 *      and 4 waves (fewer halo rows staged per pixel row; not combined with
 *      the candidate split, which keeps its 2-row tiles).
 * Per thread the shapes score 4 pixel windows (a 2 x 2 block) at all of its
 * candidates, or (candidate split) at a quarter of them.  Results do not
 * depend on the shape.  The batched path uses the fixed window and the
 * default chunk and tile height for every stage.
 *
 * msibm_force_variant - pin the shape for every later call in this process
 * (bits that do not apply to a launch are ignored); -1 restores the automatic
 * choice.  Errors: INVALID_ARG (outside -1..63).
 */
msibm_status msibm_force_variant(int32_t variant);

/*
 * msibm_autotune - with enable != 0, the first launch of each matching shape
 * (mode, n, candidates per window, dtype, H, W, D_k) not yet in the table is
 * timed in every applicable kernel shape (three interleaved rounds of one
 * warm-up and three launches each, synchronising the caller's stream; never
 * while the stream is being captured); the default shape is kept unless
 * another's best round is at least 2% faster, and the choice is used from then
 * on.  cache_path (may be NULL) names a text
 * file read now and rewritten after each new measurement, one line per shape:
 * "mode n nc dtype H W Dk variant microseconds".  The environment variables
 * MSIBM_AUTOTUNE=1 and MSIBM_TUNE_CACHE=<path> do the same at load time.
 * Errors: INVALID_ARG (cache file present but not a tuning table).
 */
msibm_status msibm_autotune(int32_t enable, const char* cache_path);

/* The tuning table as text (format above); copies at most len - 1 bytes and a
 * terminating NUL into buf (may be NULL) and returns the full length. */
int64_t msibm_autotune_table(char* buf, size_t len);

/*
 * msibm_pyramid - the K-level Gaussian pyramid of one image (Section III).
 * The blur is the separable 5-tap binomial [1 4 6 4 1]/16 with clamp-to-edge
 * reads, sampled at even rows and columns.
 *   img         device image of `dtype`, H x W, row pitch `pitch` elements.
 *   levels[k]   K device float pointers; levels[0] receives img converted to
 *               float (exact for uint8), levels[k] the level-k image of size
 *               H_k x W_k with row pitch level_pitch[k] >= W_k.
 *   level_pitch host array of K pitches.
 * Errors: INVALID_ARG (null pointer, bad dtype), SHAPE (H, W < 1, pitches),
 *         UNSUPPORTED (K outside 1..MSIBM_MAX_LEVELS), HIP.
 */
msibm_status msibm_pyramid(const void* img, int32_t dtype, int32_t H, int32_t W, int32_t pitch,
                           int32_t K, float* const* levels, const int32_t* level_pitch,
                           void* stream);

/*
 * msibm_median_filter - selective median filtering (Section III.D, Eq. 10): a
 * pixel whose matched cost is at most alpha takes the median disparity of the
 * pixels of its 5x5 patch (only those inside the image) whose cost exceeds
 * alpha; the lower median for an even count; without such pixels it keeps its
 * disparity.  Costs are compared with alpha in double precision.
 *   d_in     device int16 H x W (row pitch in_pitch), the unfiltered map.
 *   cost     device float H x W (row pitch cost_pitch), the matched costs.
 *   d_out    device int16 H x W (row pitch out_pitch); must not overlap d_in.
 * Errors: INVALID_ARG (null pointers, overlapping maps, non-finite alpha),
 *         SHAPE (sizes, pitches), HIP.
 */
msibm_status msibm_median_filter(const int16_t* d_in, int32_t in_pitch, const float* cost, int32_t cost_pitch,
                                 int32_t H, int32_t W, double alpha, int16_t* d_out, int32_t out_pitch,
                                 void* stream);

/*
 * msibm_upsample_cost - bicubic doubling of a coarser cost map (Section III.C),
 * the map the gated search compares with beta.  Fine pixel (i, j) sits at the
 * coarse position ((i + 1/2)/2 - 1/2, (j + 1/2)/2 - 1/2); Keys' cubic kernel
 * with a = -1/2 over the 4 x 4 nearest taps, clamped to the map; evaluated in
 * double as a fixed-order 16-term sum.
 *   coarse   device float Hc x Wc (row pitch coarse_pitch).
 *   out      device double H x W (row pitch out_pitch) with Hc = ceil(H/2),
 *            Wc = ceil(W/2).
 * Errors: INVALID_ARG (null pointers), SHAPE (sizes, pitches), HIP.
 */
msibm_status msibm_upsample_cost(const float* coarse, int32_t Hc, int32_t Wc, int32_t coarse_pitch, int32_t H,
                                 int32_t W, double* out, int32_t out_pitch, void* stream);

/*
 * msibm_pyramid_adjoint - the transpose of one pyramid reduction (the chain rule
 * through the binomial reduce of Section III): g_fine += R^T g_coarse, where
 * R maps an H x W image to its ceil(H/2) x ceil(W/2) reduction.  Each fine pixel
 * gathers, from at most 3 x 3 coarse pixels, the binomial weights of the taps
 * that read it (clamped taps at the border add up).  Accumulates into g_fine.
 *   g_coarse  device float Hc x Wc (row pitch coarse_pitch), Hc = ceil(H/2).
 *   g_fine    device float H x W (row pitch fine_pitch), read and written.
 * Errors: INVALID_ARG (null pointers), SHAPE (sizes, pitches), HIP.
 */
msibm_status msibm_pyramid_adjoint(const float* g_coarse, int32_t Hc, int32_t Wc, int32_t coarse_pitch,
                                   float* g_fine, int32_t H, int32_t W, int32_t fine_pitch, void* stream);

/*
 * Soft output at every level (an extension of the paper).  The coarsest level
 * is the hard full search; every finer level k takes the soft-argmax of
 * msibm_disparity's soft level (radius soft_radius, temperature tau) around its
 * doubled prior, the hard map of level k+1, and its hard winner over the same
 * interval is the prior of level k-1.  One pair; config flags must be 0,
 * soft_radius >= 1, K >= 2.
 *
 * msibm_levels_workspace_size - workspace bytes of both calls below (0 if the
 *   pair or config is invalid).
 * msibm_disparity_levels - the forward.
 *   soft[k]   k = 0..K-2: device float H_k x W_k (pitch W_k), d_soft of level k.
 *   maps[k]   k = 0..K-1: device int16 H_k x W_k (pitch W_k), the hard maps.
 * msibm_backward_levels - gradient of sum_k sum_p grad_soft[k](p) d_soft^k(p)
 *   with respect to both level-0 images (float pairs only), every level's prior
 *   held fixed: each level's soft-level backward on its own pyramid images, and
 *   the sum carried down level by level with msibm_pyramid_adjoint.
 *   maps[k]        k = 1..K-1: the forward's hard maps (maps[0] is not read).
 *   grad_soft[k]   k = 0..K-2: device float H_k x W_k (pitch W_k), or NULL for a
 *                  level without loss.
 *   grad_left/right device float H x W (pitch W), overwritten.
 * Errors: INVALID_ARG, SHAPE, UNSUPPORTED (flags, K < 2, non-float backward),
 *         WORKSPACE, HIP.
 */
size_t msibm_levels_workspace_size(const msibm_pair* pair, const msibm_config* cfg);
msibm_status msibm_disparity_levels(const msibm_pair* pair, const msibm_config* cfg, float* const* soft,
                                    int16_t* const* maps, void* workspace, size_t ws_bytes, void* stream);
msibm_status msibm_backward_levels(const msibm_pair* pair, const msibm_config* cfg, const int16_t* const* maps,
                                   const float* const* grad_soft, float* grad_left, float* grad_right,
                                   void* workspace, size_t ws_bytes, void* stream);

/* Bytes of workspace msibm_match_level needs for an H x W level. */
size_t msibm_level_workspace_size(int32_t H, int32_t W);

/*
 * msibm_match_level - winner-take-all ZNCC matching of one pyramid level.
 *   prior == NULL: full search of z in [0, min(D_k - 1, j)] (Eqs. 3-4; also
 *                  standard block matching when applied at level 0 with D).
 *   prior != NULL: restricted search (Eqs. 8-9, first branch).  `prior` is the
 *                  level-(k+1) disparity map, Hc x Wc int16 with Hc =
 *                  ceil(H/2), Wc = ceil(W/2), row pitch prior_pitch; pixel
 *                  (i, j) takes c = min(2 prior(i/2, j/2), j) and searches
 *                  [max(0, c - r), min(D_k - 1, j, c + r)].
 *   L, R       device images of `dtype` (MSIBM_U8 or MSIBM_F32), H x W, pitch.
 *   d_out      device int16 H x W (row pitch out_pitch): lowest z of the best score.
 *   cost_out   device float H x W or NULL: the best score (Eq. 4 / Eq. 9).
 *   costvol    NULL, or (for testing) device float H x W x D_k, entry
 *              (i W + j) D_k + z: the clamped score of every candidate the
 *              search scores, -2 for every other z (the buffer is filled first).
 *   workspace  device scratch of msibm_level_workspace_size(H, W) bytes.
 * Errors: INVALID_ARG, SHAPE (sizes, pitches, prior shape), UNSUPPORTED (n, r,
 *         D_k out of range), WORKSPACE, HIP.
 */
msibm_status msibm_match_level(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                               int32_t pitch, int32_t n, int32_t Dk, const int16_t* prior,
                               int32_t Hc, int32_t Wc, int32_t prior_pitch, int32_t r,
                               float var_eps, int16_t* d_out, float* cost_out, int32_t out_pitch,
                               float* costvol, void* workspace, size_t ws_bytes, void* stream);

/*
 * msibm_match_level_gated - confidence-gated matching of a finer level (Eqs.
 * 8-9): the restricted search of msibm_match_level around `prior`, except at
 * pixels whose bicubic-doubled coarser cost (msibm_upsample_cost of
 * prior_cost, compared in double) is <= beta, which take the full search of z
 * in [0, min(D_k - 1, j)].  Ties go to the lowest z in both branches.
 *   prior, prior_cost  device int16 and float Hc x Wc maps of level k+1 (its
 *                      disparities and costs), Hc = ceil(H/2), Wc = ceil(W/2),
 *                      both with row pitch prior_pitch.
 *   d_out, cost_out    device int16 / float H x W, row pitch out_pitch (both
 *                      required).
 *   workspace          msibm_level_workspace_size(H, W) bytes.
 * Errors: as msibm_match_level; INVALID_ARG for a NULL prior, prior_cost or
 *         cost_out, or a non-finite beta.
 */
msibm_status msibm_match_level_gated(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                                     int32_t pitch, int32_t n, int32_t Dk, const int16_t* prior,
                                     const float* prior_cost, int32_t Hc, int32_t Wc, int32_t prior_pitch,
                                     int32_t r, double beta, float var_eps, int16_t* d_out, float* cost_out,
                                     int32_t out_pitch, void* workspace, size_t ws_bytes, void* stream);

/*
 * msibm_aggregate_refine - disparity refinement by the neighbourhood-averaged
 * disparity search image (Eqs. 5-7), in place.  A pixel whose cost is <= alpha
 * (compared in double) takes the z of [0, min(D_k - 1, j)] that maximises the
 * mean over its 5x5 neighbourhood (clipped to the image) of the neighbours'
 * scores at z, a neighbour in column q counting only for z <= q; its cost
 * becomes that maximum (ties to the lowest z).  Other pixels keep d and cost.
 *   d, cost    device int16 / float H x W, row pitch dc_pitch (read and written).
 *   workspace  msibm_level_workspace_size(H, W) bytes.
 * Errors: INVALID_ARG (null pointers, non-finite alpha, var_eps), SHAPE,
 *         UNSUPPORTED (n, D_k), WORKSPACE, HIP.
 */
msibm_status msibm_aggregate_refine(const void* L, const void* R, int32_t dtype, int32_t H, int32_t W,
                                    int32_t pitch, int32_t n, int32_t Dk, int16_t* d, float* cost,
                                    int32_t dc_pitch, double alpha, float var_eps, void* workspace,
                                    size_t ws_bytes, void* stream);

/* Bytes of workspace msibm_disparity / msibm_backward need for these pairs. */
size_t msibm_workspace_size(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg);

/*
 * msibm_disparity - the hierarchical forward pass for n_pairs stereo pairs.
 * For each pair: pyramid of both views, full search at level K-1, restricted
 * search at levels K-2..0, each level's prior being the next coarser map.
 *   pairs, cfg     host arrays/structs (copied; need not outlive the call unless
 *                  MSIBM_FLAG_GRAPH, which caches by shape, see below).
 *   disp[p]        device int16 H x W (row pitch = pairs[p].width): level-0 map.
 *   cost[p]        NULL or NULL entries, or device float H x W: level-0 score.
 *   soft_disp[p]   required iff cfg->soft_radius > 0: device float H x W,
 *                  sum_z p_z z with p = softmax(score / tau) over level 0's
 *                  candidates (an addition to the paper: the differentiable form).
 *   prior1[p]      NULL, or device int16 H_1 x W_1 (pitch W_1) receiving the
 *                  level-1 map (the prior of level 0) that msibm_backward needs;
 *                  unused when K == 1.
 *   workspace      device scratch of msibm_workspace_size(pairs, n_pairs, cfg).
 * Without MSIBM_FLAG_BATCHED the pairs run one after another (plain path, per
 * pair: one launch per three pyramid steps, one statistics launch, one matching
 * launch per level).  With it the pairs advance together, one launch per stage
 * covering every pair's tiles: per pyramid step the level's statistics beside
 * the reduce to the next level, then per level (coarsest first) one matching
 * launch per (mode, dtype) present;
 * the outputs are bit-identical to the plain path.  The launches find their
 * tiles through a small table that is copied into the workspace on `stream`
 * from library-owned pinned host memory.  With MSIBM_FLAG_GRAPH too, the first
 * call captures the launch sequence into a hipGraph (on a library-owned stream,
 * with a library-owned device copy of the table) keyed by the device, the pairs
 * (pointers, shapes, D, K), cfg, the output pointers and the workspace; later
 * calls with the same key replay it on `stream`.  The graph keeps using those
 * buffers: the caller keeps them alive and unchanged in size while it replays.
 * MSIBM_FLAG_GRAPH without MSIBM_FLAG_BATCHED is INVALID_ARG.
 * Errors: INVALID_ARG, SHAPE, UNSUPPORTED, WORKSPACE, HIP.
 */
msibm_status msibm_disparity(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                             int16_t* const* disp, float* const* cost, float* const* soft_disp,
                             int16_t* const* prior1, void* workspace, size_t ws_bytes,
                             void* stream);

/* Bytes of device scratch msibm_disparity_noalloc holds on each device: enough
 * for a 1920 x 1080 pair with any of PREBLUR, MEDIAN and GATED. */
#define MSIBM_NOALLOC_SCRATCH_BYTES (96u << 20)

/*
 * msibm_disparity_noalloc - msibm_disparity for ONE pair on the plain per-pair
 * path, with no workspace argument and no allocation of any kind.  For callers
 * that cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.
 *   pair, cfg   as for msibm_disparity with n_pairs = 1; cfg->flags may hold
 *               PREBLUR, MEDIAN and GATED, not BATCHED or GRAPH.
 *   disp, cost, soft_disp, prior1   as msibm_disparity's entries of the pair
 *               (cost and prior1 may be NULL; soft_disp is required iff
 *               soft_radius > 0).  The caller owns them.
 * Scratch: a device array of MSIBM_NOALLOC_SCRATCH_BYTES inside the library,
 * one per device, held from the device's first call until the process ends;
 * the first call on a device looks up its address with that device current.
 * No call calls hipMalloc, hipFree, an allocating library routine or creates
 * an event: the autotuner only reads kernel shapes it measured before (it
 * never measures here) and per-launch timing records nothing.  Every call on a
 * device uses that device's one array, which keeps the last call's contents
 * (the forward writes every scratch byte it reads, so nothing is cleared):
 * calls that overlap in time on one device (several streams or host threads)
 * race and must be serialised by the caller.
 * Errors: INVALID_ARG, SHAPE, UNSUPPORTED (as msibm_disparity; BATCHED or
 *         GRAPH), WORKSPACE (the pair needs more scratch than
 *         MSIBM_NOALLOC_SCRATCH_BYTES: msibm_workspace_size gives its need),
 *         HIP.
 */
msibm_status msibm_disparity_noalloc(const msibm_pair* pair, const msibm_config* cfg, int16_t* disp, float* cost,
                                     float* soft_disp, int16_t* prior1, void* stream);

/*
 * msibm_backward - gradient of sum_{ij} g(i,j) d_soft(i,j) with respect to the
 * level-0 left and right images, with the level-1 prior held fixed (it is
 * piecewise constant in the images).  Recomputes every window statistic and
 * score; no cost volume is stored.  The gradient flows through
 *   d_soft = sum_z p_z z,  p = softmax(rho / tau)  ->  dd/drho_z = p_z (z - d_soft) / tau,
 *   rho = C / sqrt(A B)  ->  drho/dl = (r - mu_r)/sqrt(AB) - rho (l - mu_l)/A  (and
 *   symmetrically for r); flat candidates contribute nothing and a clamped read
 *   passes its gradient to the edge pixel it read.
 *   pairs[p]        must be MSIBM_F32 (UNSUPPORTED otherwise), K >= 2.
 *   cfg             as in the forward call, soft_radius >= 1.
 *   prior1[p]       device int16 level-1 map saved by msibm_disparity.
 *   grad_soft[p]    device float H x W (pitch W): dL/dd_soft.
 *   grad_left[p], grad_right[p]  device float H x W (pitch W), OVERWRITTEN.
 *   workspace       as for msibm_disparity.
 * Without MSIBM_FLAG_BATCHED each pair takes three launches (level-0 statistics,
 * gradient zeroing, backward tiles).  With it those three launches cover every
 * pair; with MSIBM_FLAG_GRAPH too they are captured and replayed as described
 * for msibm_disparity (keyed by pairs, cfg, the prior, gradient and workspace
 * pointers).  Gradients are summed with float atomics, so the low bits depend
 * on the summation order (not bit-reproducible between runs).
 * Errors: INVALID_ARG, SHAPE, UNSUPPORTED, WORKSPACE, HIP.
 */
msibm_status msibm_backward(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                            const int16_t* const* prior1, const float* const* grad_soft,
                            float* const* grad_left, float* const* grad_right, void* workspace,
                            size_t ws_bytes, void* stream);

/*
 * msibm_fwd_bwd_l1 - the forward, the masked mean-L1 loss and the backward of
 * n_pairs float pairs in one call (a training step's work on the
 * differentiable finest level; not in the paper, which has no loss).  Per pair
 *   L = (1/|M|) sum_{(i,j) in M} |d_soft(i,j) - gt(i,j)|   (L = 0 when M is empty)
 * and dL/dd_soft = sign(d_soft - gt)/|M| on M (sign(0) = 0), 0 elsewhere,
 * carried to both images as msibm_backward does.  Levels K-1..1 run as in
 * msibm_disparity; level 0 is one fused launch that computes the soft level,
 * forms each pixel's loss gradient from its d_soft and runs the backward with
 * it (no soft-level launch of its own, no dL/dd_soft buffer, and the level-0
 * window statistics of the forward are reused).  The d_soft, winner and score
 * it writes are those msibm_disparity computes, up to the summation order of
 * the window sums (the backward's pixel-row order), within the forward's
 * tolerances.
 *   pairs[p]        MSIBM_F32, K >= 2; cfg: soft_radius >= 1, no PREBLUR,
 *                   MEDIAN or GATED.
 *   d_gt[p]         device float H x W (pitch W): target disparity.
 *   mask[p]         device uint8 H x W (pitch W): nonzero on the loss pixels M.
 *   disp[p], cost[p] (cost may be NULL), soft_disp[p], prior1[p] (may be NULL)
 *                   outputs as for msibm_disparity.
 *   grad_left[p], grad_right[p]  device float H x W (pitch W), OVERWRITTEN.
 *   loss[p]         device float, receives L.
 *   workspace       msibm_workspace_size(pairs, n_pairs, cfg) bytes.
 * Without MSIBM_FLAG_BATCHED the pairs run one after another; with it every
 * stage is one launch for all pairs; with MSIBM_FLAG_GRAPH too the whole
 * sequence (forward, loss and backward) is one captured graph, replayed as
 * described for msibm_disparity (keyed by the pairs, cfg and every buffer
 * pointer).  Gradients and the loss sum use float atomics (low bits depend on
 * the summation order).
 * Errors: INVALID_ARG, SHAPE, UNSUPPORTED, WORKSPACE, HIP.
 */
msibm_status msibm_fwd_bwd_l1(const msibm_pair* pairs, int32_t n_pairs, const msibm_config* cfg,
                              const float* const* d_gt, const uint8_t* const* mask, int16_t* const* disp,
                              float* const* cost, float* const* soft_disp, int16_t* const* prior1,
                              float* const* grad_left, float* const* grad_right, float* const* loss,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * Launch timing (instrumentation, off by default).  While enabled, every kernel
 * launch that msibm_disparity and msibm_backward enqueue is bracketed by two HIP
 * events on the launch stream, labelled by kernel and level (for example
 * "match_refine_l0").  Enabling or disabling clears the accumulated totals.
 */
msibm_status msibm_timing_enable(int32_t on);

/*
 * Waits for every pending timed launch, folds it into per-label totals and
 * writes up to `cap` entries: labels (64 chars each, NUL-terminated, may be
 * NULL), total milliseconds and launch counts.  Returns the entry count.
 */
int32_t msibm_timing_read(int32_t cap, char* labels, double* total_ms, int32_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* MSIBM_H */
