/*
 * bsm.h - C ABI of the MI355X (gfx950) Binary Stereo Matching library.
 *
 * The library computes the hot path of Zhang et al., "Binary Stereo
 * Matching" (Section 3): a BRIEF descriptor per pixel of both views
 * (Eq. 2-3), a binary support mask for the reference view (Eq. 5-7), the
 * masked Hamming cost by XOR / AND / popcount on packed words (Eq. 8; Eq. 4
 * without the mask) and the winner-take-all disparity over
 * d in [0, dmax - 1] (Eq. 1).  Input: a rectified RGB pair and dmax, as in
 * the problem statement of Section 1; output: an integer disparity map and,
 * on request, the cost volume.  Every step runs in HIP kernels on the GPU.
 *
 * Conventions shared by all calls
 * -------------------------------
 * Views      The left view is the reference; pixel x = (u, v) of the left
 *            view is compared with x_d = (u - d, v) of the right view.
 * Images     uint8 RGB, interleaved, rows `stride` bytes apart
 *            (stride >= 3 * W).
 * Intensity  I = (77 R + 150 G + 29 B + 128) >> 8 (the paper says only
 *            "intensity"; this is integer BT.601 luma).
 * CIELAB     8-bit L8 = L*255/100, a8 = a + 128, b8 = b + 128 for sRGB with
 *            the D65 white, computed with integer tables (the paper names
 *            the colour space only).
 * Borders    A sample outside the image takes the nearest edge pixel.
 * Pattern    int8 [n][4] rows (px, py, qx, qy): pair i compares
 *            x + (px, py) with x + (qx, qy) (Section 3, after Eq. 2).
 * Bits       Pair i (1-based) is bit (i-1) % 64 of word (i-1) / 64: the
 *            weight 2^(i-1) of Eq. 2 and Eq. 7.
 * desc/mask  uint64 [H][W][n/64], pixel-major ("words of pixel (u, v)
 *            start at ((v * W) + u) * n/64").
 * Threshold  T(x) = k-th smallest pair weight, k = n/4 by default (the
 *            "quarter smallest value" after Eq. 6); delta_i = [w_i <= T].
 * Cost       C(x, d) = popcount((B_L(x) XOR B_R(x_d)) AND Phi(x)); with no
 *            mask, popcount(B_L(x) XOR B_R(x_d)).  C <= n.
 * Volume     int16 [dmax][H][W]; entries with u - d < 0 hold 32767.
 * Disparity  int32 [H][W]: the smallest d that attains min_d C(x, d).
 *
 * Pointers   "device" = memory of the context's GPU (e.g. a torch CUDA
 *            tensor's data_ptr()); "host" = ordinary CPU memory.  Device
 *            calls take a HIP stream (hipStream_t, NULL = default stream),
 *            are stream-ordered and return once the work is enqueued.
 *            desc/mask buffers must be 16-byte aligned, disp/cost/packed
 *            4-byte aligned; buffers must not overlap.  The caller owns
 *            every buffer it passes.
 * Errors     Every call returns a status and never aborts.  Arguments are
 *            validated before any device work (BSM_EINVAL).  A failed HIP
 *            call returns BSM_EDEVICE and marks the context dead: every
 *            later call on it returns BSM_EDEVICE.  bsm_last_error() gives a
 *            message for the calling thread's last failure.
 * Threads    A context may be used from one thread at a time, except
 *            bsm_submit / bsm_poll / bsm_drain, which lock internally.
 * Streams    Device calls are ordered on the stream they are given.  The
 *            single-pair calls (bsm_color / bsm_describe / bsm_match /
 *            bsm_match_right / bsm_vote_refine) share context scratch: a
 *            call on a different stream than the previous such call first
 *            waits for the device to be idle, so one stream per context is
 *            the fast way to use them.
 */
#ifndef BSM_H
#define BSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSM_OK = 0,
    BSM_EINVAL = -1,    /* invalid argument; nothing was enqueued          */
    BSM_ENOMEM = -2,    /* device or host allocation failed                */
    BSM_EDEVICE = -3,   /* HIP error (sticky on the context)               */
    BSM_EAGAIN = -4,    /* serving queue full; try again later             */
    BSM_ETOOBIG = -5,   /* pair larger than the serving admission cap      */
    BSM_ENOTFOUND = -6  /* unknown ticket                                  */
} bsm_status;

typedef struct bsm_ctx bsm_ctx;

typedef struct {
    int32_t n_bits;         /* n: descriptor length, multiple of 64 in
                               [64, 4096] (the paper uses 4096, Section 4.1) */
    int32_t window;         /* S: side of the sampling window, 2..63
                               (the paper uses 26); offsets lie in
                               [-S/2, (S-1)/2]                              */
    double sigma;           /* spread of the Gaussian sampling; <= 0 selects
                               4 * S / 26 (the paper's 4 at S = 26)         */
    uint64_t seed;          /* seed for the pattern when pattern == NULL    */
    const int8_t *pattern;  /* host [n][4] pattern to use, or NULL to draw
                               one with bsm_make_pattern(seed, ...); copied */
    int32_t mask_rank;      /* k of the threshold, 1..n; 0 selects n/4      */
    int32_t use_mask;       /* bsm_match / batch / serving: 1 = Eq. 8
                               (masked cost), 0 = Eq. 4 (plain Hamming)     */
} bsm_params;

/* One stereo pair for bsm_match_batch (device pointers) or bsm_submit
 * (host pointers). */
typedef struct {
    const uint8_t *left;    /* RGB [H][stride]                              */
    const uint8_t *right;   /* RGB [H][stride]                              */
    int32_t width, height, stride, dmax;
    int32_t *disp;          /* out int32 [H][W]                             */
    int16_t *cost;          /* out int16 [dmax][H][W], or NULL              */
} bsm_pair;

/* Serving timestamps, seconds on the host's CLOCK_MONOTONIC. */
typedef struct {
    double t_arrive;        /* bsm_submit was called                        */
    double t_admit;         /* admitted under the memory cap                */
    double t_start;         /* its first GPU work was enqueued              */
    double t_end;           /* results were in host memory                  */
} bsm_times;

/* Creates a context on HIP device `hip_device`: validates the parameters,
 * copies or draws the point-pair pattern (Section 3, after Eq. 2), builds
 * the integer colour tables and uploads both.  On success *out owns them.
 * BSM_EINVAL on bad parameters, BSM_EDEVICE / BSM_ENOMEM on HIP failure. */
bsm_status bsm_create(const bsm_params *params, int32_t hip_device,
                      bsm_ctx **out);

/* Waits for the context's in-flight work, stops its serving thread and
 * frees everything it owns.  NULL is ignored. */
void bsm_destroy(bsm_ctx *ctx);

/* Message of the calling thread's last failed call ("" if none). */
const char *bsm_last_error(void);

/* Host only: draws the pattern of Section 3 (after Eq. 2): each of the
 * 4 n coordinates is floor(sigma * z + 0.5), z a standard normal from the
 * basic Box-Muller transform of two splitmix64 outputs (seeded with `seed`),
 * redrawn while outside [-S/2, (S-1)/2]; q is redrawn while q == p.
 * out: host int8 [n][4].  n in [1, 4096], S in [2, 63], sigma > 0. */
bsm_status bsm_make_pattern(uint64_t seed, int32_t n, int32_t S, double sigma,
                            int8_t *out);

/* Copies the context's pattern to host int8 [n][4]. */
bsm_status bsm_pattern(const bsm_ctx *ctx, int8_t *out);

/* Device bytes bsm_match needs for one W x H pair (its internal scratch:
 * colour planes and descriptors), plus the volume if want_cost.  0 on
 * invalid arguments. */
size_t bsm_footprint(const bsm_ctx *ctx, int32_t W, int32_t H, int32_t dmax,
                     int32_t want_cost);

/* Colour pre-pass (the intensity of Eq. 3 and the CIELAB values of Eq. 5):
 * packed uint32 [H][W], byte 0 = L8, 1 = a8, 2 = b8, 3 = I.  With
 * want_lab == 0 bytes 0-2 are 0.  img: device RGB; packed: device. */
bsm_status bsm_color(bsm_ctx *ctx, const uint8_t *img, int32_t W, int32_t H,
                     int32_t stride, uint32_t *packed, int32_t want_lab,
                     void *hip_stream);

/* Descriptor B (Eq. 2-3) of every pixel of one view, and its binary mask Phi
 * (Eq. 5-7) when mask != NULL (the reference view).  img: device RGB;
 * desc, mask: device uint64 [H][W][n/64].  Uses context scratch. */
bsm_status bsm_describe(bsm_ctx *ctx, const uint8_t *img, int32_t W,
                        int32_t H, int32_t stride, uint64_t *desc,
                        uint64_t *mask, void *hip_stream);

/* Descriptor and optional mask from the colour pre-pass output (bsm_color
 * with want_lab = 1 when mask != NULL): the same as bsm_describe without its
 * colour step.  packed: device uint32 [H][W]; desc, mask as bsm_describe. */
bsm_status bsm_describe_packed(bsm_ctx *ctx, const uint32_t *packed, int32_t W,
                               int32_t H, uint64_t *desc, uint64_t *mask,
                               void *hip_stream);

/* Masked cost (Eq. 8, or Eq. 4 when maskL == NULL) fused with the
 * winner-take-all of Eq. 1 (lowest d among equal costs).  The H x W x dmax
 * volume is written only when cost != NULL; entries with u - d < 0 hold
 * 32767.  descL, maskL, descR: device uint64 [H][W][n/64], 16-byte
 * aligned; disp: device int32 [H][W]; cost: device int16 [dmax][H][W] or
 * NULL.  1 <= dmax <= W.  The matrix-core and bitwise kernels (bsm_tuning
 * cost_mfma) give identical results. */
bsm_status bsm_cost_wta(bsm_ctx *ctx, const uint64_t *descL,
                        const uint64_t *maskL, const uint64_t *descR,
                        int32_t W, int32_t H, int32_t dmax, int32_t *disp,
                        int16_t *cost, void *hip_stream);

/* The whole hot path for one pair: colour pre-pass and descriptors of both
 * views, mask of the left view (if params.use_mask), cost and WTA.
 * left/right: device RGB; disp/cost as in bsm_cost_wta.  Uses context
 * scratch (bsm_footprint bytes).  The other view's colour pass and
 * descriptor run on an internal stream of the context that first waits for
 * the work already queued on hip_stream, and hip_stream waits for it before
 * the cost kernel: the call as a whole stays ordered on hip_stream. */
bsm_status bsm_match(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right,
                     int32_t W, int32_t H, int32_t stride, int32_t dmax,
                     int32_t *disp, int16_t *cost, void *hip_stream);

/* bsm_match for callers that cannot allocate device memory (work under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as bsm_match; the pair's scratch (two
 * colour planes and three descriptor planes, bsm_footprint without the
 * volume) lives in a fixed device array of the library, of
 * BSM_NOALLOC_MAX_BYTES (64 MiB) per GPU, held from bsm_create until the
 * process ends.  The call allocates nothing and creates no stream or event:
 * all its work is enqueued on hip_stream.  A 450 x 375 pair at n = 1024
 * fits; a pair whose scratch exceeds the array returns BSM_ETOOBIG before
 * any device work.  Every context on one GPU shares that GPU's array and
 * nothing in it needs clearing (each call overwrites what it reads), but
 * calls whose work overlaps on one GPU race: the caller must order them
 * (one stream, or events between streams). */
#define BSM_NOALLOC_MAX_BYTES ((size_t)64 << 20)
bsm_status bsm_match_noalloc(bsm_ctx *ctx, const uint8_t *left,
                             const uint8_t *right, int32_t W, int32_t H,
                             int32_t stride, int32_t dmax, int32_t *disp,
                             int16_t *cost, void *hip_stream);

/* Right-reference matching: the second depth map of the left/right check
 * that opens the refinement step of Section 3.  The right view is the
 * reference: pixel (u, v) of the right view is compared with (u + d, v) of
 * the left view, with the right view's own mask (Eq. 5-7 on the right
 * image); volume entries with u + d > W - 1 hold 32767; ties take the
 * lowest d.  Same arguments, buffers and errors as bsm_match; disp and cost
 * are indexed by right-view pixels.  Runs the left-reference kernels on the
 * horizontally mirrored views with the mirrored pattern and reverses the
 * results' rows. */
bsm_status bsm_match_right(bsm_ctx *ctx, const uint8_t *left,
                           const uint8_t *right, int32_t W, int32_t H,
                           int32_t stride, int32_t dmax, int32_t *disp,
                           int16_t *cost, void *hip_stream);

/* Left/right consistency check (Section 3, refinement step): out(u, v) =
 * dL(u, v) where |dL(u, v) - dR(u - dL(u, v), v)| <= tol (the pixel is
 * valid), else -1 (invalid; also when u - dL(u, v) < 0).  disp_left,
 * disp_right, out: device int32 [H][W], 4-byte aligned; out may be
 * disp_left (in place) but not disp_right.  tol >= 0 (1 is customary). */
bsm_status bsm_lr_check(bsm_ctx *ctx, const int32_t *disp_left,
                        const int32_t *disp_right, int32_t W, int32_t H,
                        int32_t tol, int32_t *out, void *hip_stream);

/* Voting refinement (Section 3, Eq. 9-10) of the pixels a left/right check
 * marked invalid (checked < 0): d(x) = the d in [0, dmax - 1] with the
 * largest W(x, d), the sum over valid pixels p (checked >= 0) with
 * disparity d in the (2 radius + 1)^2 window around x (inside the image) of
 * exp(-(c(x, p) / lambda_c + e(x, p) / lambda_e)), c = Euclidean distance
 * of the 8-bit CIELAB colours of the left view, e = Euclidean distance of
 * the positions (the paper's lambda_c = 9, lambda_e = 16; it leaves the
 * window and the colour space open, this library takes the matching window
 * and CIELAB).  Ties take the lowest d; an invalid pixel without voters
 * takes fallback(x) (e.g. the WTA disparity); valid pixels keep checked(x).
 * Votes are summed in fp32 in a fixed order: the same result on every
 * run, which may differ from an exact sum only at near-ties.  left: device
 * RGB; checked, fallback, out: device int32 [H][W], 4-byte aligned; out may
 * be fallback but not checked.  1 <= dmax <= 4096, 0 <= radius <= 63.
 * Uses context scratch. */
bsm_status bsm_vote_refine(bsm_ctx *ctx, const uint8_t *left, int32_t W,
                           int32_t H, int32_t stride, const int32_t *checked,
                           const int32_t *fallback, int32_t dmax,
                           int32_t radius, float lambda_c, float lambda_e,
                           int32_t *out, void *hip_stream);

/* Many pairs of uneven size and dmax at once.  The tiles of all pairs go
 * into device work queues (largest pair first) served by one persistent
 * kernel per stage (colour, describe+mask, describe, cost+WTA with and
 * without volume); the launches are captured once per context into a HIP
 * graph that every later batch replays, whatever its shapes.  All pointers
 * in `pairs` are device pointers; `pairs` itself is host memory.  Results
 * equal npairs calls of bsm_match.  The persistent path needs n in
 * {64, 128, 256, 512, 1024} and at least five pairs; otherwise the pairs
 * run one after another with the per-pair kernels (on up to four pairs they
 * are faster than the persistent launch, whose fixed cost is about 0.1 ms).
 * Uses context scratch (the sum of the pairs' bsm_footprint without
 * volumes). */
bsm_status bsm_match_batch(bsm_ctx *ctx, const bsm_pair *pairs,
                           int32_t npairs, void *hip_stream);

/* Launch choices of a context.  They change speed only, never results. */
typedef struct {
    int32_t desc_tile_w;      /* describe+mask tile width: 16 or 32 pixels   */
    int32_t cost_dchunk;      /* disparities per LDS window of the bitwise
                                 cost kernel: 32 or 64                      */
    int32_t blocks_per_cu[4]; /* persistent batch launches, 0 = default:
                                 [0] colour, [1] the two describe stages
                                 (one launch), [3] cost: workgroups per CU
                                 (0 = as many as fit, max 64); [2]: one
                                 describe workgroup in this many starts on
                                 the descriptor-only tiles (0 = 4)          */
    int32_t cost_mfma;        /* 1 (default): cost + WTA on the matrix cores
                                 (the cost as an integer dot product) for
                                 n <= 1024 and 16 < dmax (<= 256 with a
                                 volume; single pairs, and batch pairs
                                 without one); 0: the bitwise VALU kernel */
    int32_t batch_tile_h;     /* describe+mask tile height of the persistent
                                 batch: 8 or 16 rows (default 16)           */
    int32_t pair_desc_th;     /* single pairs (and batches of up to four):
                                 describe+mask tile height, 4 or 8 rows;
                                 0 (default): 4 below 4096 tiles of 8 rows,
                                 else 8                                     */
    int32_t pair_right_px;    /* single pairs: pixels per lane of the
                                 descriptor-only kernel, 1 or 4; 0
                                 (default): 4 from 1024 tiles of 4 x 256
                                 pixels on, else 1                          */
    int32_t mfma_min_dmax;    /* smallest dmax that takes the matrix-core
                                 cost kernel when cost_mfma = 1, 2..257
                                 (default 17)                               */
} bsm_tuning;

bsm_status bsm_get_tuning(const bsm_ctx *ctx, bsm_tuning *out);
/* BSM_EINVAL on values outside the ranges above. */
bsm_status bsm_set_tuning(bsm_ctx *ctx, const bsm_tuning *tuning);

/* Autotuner: times bsm_match_batch on `pairs` (device pointers, as for
 * bsm_match_batch; outputs are overwritten) for each candidate tuning,
 * `reps` timed runs each after one untimed run, keeps the fastest on the
 * context and returns it in *best with its mean time per batch in *best_ms
 * (either may be NULL).  Blocks until done.  Candidates for the persistent
 * batch: desc_tile_w 16/32 x batch_tile_h 8/16 x blocks_per_cu[2] (the
 * describe split) 3/4/5/6/8, and, when a pair has a volume, cost_dchunk
 * 32/64 x blocks_per_cu[3] 0/2.  For pairs that run one by one (a single
 * pair, or up to four): desc_tile_w 16/32 x pair_desc_th 4/8 x
 * pair_right_px 1/4 x cost_mfma 1/0 (0 only where the matrix-core kernel
 * applies). */
bsm_status bsm_autotune(bsm_ctx *ctx, const bsm_pair *pairs, int32_t npairs,
                        int32_t reps, void *hip_stream, bsm_tuning *best,
                        double *best_ms);

/* Autotuner with a persistent cache.  cache_path names a JSON file (one
 * object, one entry per line) mapping a key to a tuning and its time.  The
 * key holds the GPU architecture, n, S, the mask mode and the shape class
 * of `pairs`: the path they take ("batch" or "pairs"), the pair count, the
 * largest dmax and the mean pixel count in thousands (each rounded up to a
 * power of two) and whether a volume is wanted.  If the file holds the key,
 * its tuning is set on the context without running anything and *hit = 1;
 * otherwise bsm_autotune runs, its winner is added to the file (written to
 * cache_path.tmp, then renamed) and *hit = 0.  cache_path NULL: no cache.
 * best, best_ms, hit may be NULL.  BSM_EINVAL if the file cannot be
 * written (the context keeps the tuned choice). */
bsm_status bsm_autotune_cached(bsm_ctx *ctx, const bsm_pair *pairs,
                               int32_t npairs, int32_t reps,
                               void *hip_stream, const char *cache_path,
                               bsm_tuning *best, double *best_ms,
                               int32_t *hit);

/* Measurement of a batch's stages: runs `pairs` like bsm_match_batch (same
 * work list, kernels and results) but launches the stage kernels directly
 * on the stream instead of replaying the graph, with HIP events between
 * them; waits for the batch and writes each stage's time in milliseconds
 * to the host array stage_ms[4]: [0] colour pre-pass of all views,
 * [1] both describe stages (descriptor + mask of the left views,
 * descriptor of the right views, one launch), [2] cost + WTA of the pairs
 * without a volume, [3] of the pairs with one.  Needs the persistent path
 * (n in {64, 128, 256, 512, 1024} and at least five pairs), else
 * BSM_EINVAL. */
bsm_status bsm_batch_stage_times(bsm_ctx *ctx, const bsm_pair *pairs,
                                 int32_t npairs, void *hip_stream,
                                 float *stage_ms);

/* Serving: admission cap on the device working set of pairs in flight
 * (bytes; default 32 GiB), the maximum number of queued requests (default
 * 4096) and the most pairs one group may hold (0 = the default, 4).  A
 * server starts on the first serving call; it admits waiting pairs in
 * arrival order while their device bytes fit under the cap and runs each
 * admitted group as one batch on one of three executor slots, so groups
 * overlap on the device and pairs that arrive meanwhile join the next group
 * (continuous batching). */
bsm_status bsm_serve_config(bsm_ctx *ctx, size_t cap_bytes, int32_t max_queue,
                            int32_t max_group);

/* Serving: queues one pair given in HOST memory and returns a ticket.  The
 * library copies the images to the device when the pair is admitted and
 * writes disp (and cost) back to the host buffers; the caller keeps all
 * four buffers alive until bsm_poll reports it done or failed.
 * BSM_ETOOBIG if the pair alone exceeds the cap, BSM_EAGAIN if the queue is
 * full. */
bsm_status bsm_submit(bsm_ctx *ctx, const bsm_pair *pair, uint64_t *ticket);

/* Serving: state of a ticket (0 pending, 1 done, -1 failed) and its
 * timestamps (times may be NULL).  A done or failed ticket is forgotten
 * after it is reported once.  BSM_ENOTFOUND for unknown tickets. */
bsm_status bsm_poll(bsm_ctx *ctx, uint64_t ticket, int32_t *state,
                    bsm_times *times);

/* Serving: blocks until every submitted pair is done or failed. */
bsm_status bsm_drain(bsm_ctx *ctx);

/* Serving counters since the server started. */
typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t groups;              /* groups started on executor slots        */
    uint64_t max_in_flight_bytes; /* largest admitted working set            */
    int32_t max_group;            /* most pairs in one group                 */
    int32_t max_slots_busy;       /* most groups running at once             */
} bsm_serve_counters;

/* Serving: copies the counters to *out (all zero before the first serving
 * call).  BSM_EINVAL if ctx or out is NULL. */
bsm_status bsm_serve_stats(bsm_ctx *ctx, bsm_serve_counters *out);

#ifdef __cplusplus
}
#endif

#endif /* BSM_H */
