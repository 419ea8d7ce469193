/*
 * CPU oracle for the Binary Stereo Matching hot path (Zhang et al., "Binary
 * Stereo Matching", Section 3 "Proposed Approach", Eq. 1-8).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check the GPU library
 * against a plain, slow, obviously correct definition.  It shares no code,
 * header, table or constant with the GPU library and must never be linked
 * into, or called by, the product path.
 *
 * Layouts (all row-major, little-endian):
 *   rgb   : uint8  [H][stride]  interleaved R,G,B; stride >= 3*W bytes
 *   luma  : uint8  [H][W]
 *   lab   : uint8  [H][W][3]    (L8, a8, b8)
 *   desc  : uint64 [H][W][n/64] bit (i-1)%64 of word (i-1)/64 = pair i
 *   mask  : uint64 [H][W][n/64] same bit order as desc
 *   cost  : int16  [dmax][H][W] ; 32767 where u - d < 0
 *   disp  : int32  [H][W]
 */
#ifndef BSM_ORACLE_H
#define BSM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of worker threads the row loops may use (OpenMP); 1 = serial. */
void oracle_set_threads(int threads);
int oracle_get_threads(void);

/* splitmix64: state += golden gamma, then the published finaliser. */
uint64_t oracle_splitmix64_next(uint64_t *state);

/* Standard normal draw by the basic Box-Muller transform (cosine branch)
 * from two consecutive splitmix64 outputs. */
double oracle_normal(uint64_t *state);

/* Point-pair pattern (Section 3, the sentence after Eq. 2; parameters of
 * Section 4.1).  Writes n rows of (px, py, qx, qy).  Returns 0, or -1 on
 * invalid arguments. */
int oracle_make_pattern(uint64_t seed, int n, int S, double sigma,
                        int8_t *out);

/* Intensity I(x) used by the binary test of Eq. 3. */
void oracle_luma(const uint8_t *rgb, int W, int H, int stride, uint8_t *out);

/* Integer CIELAB tables and conversion used by the SAD of Eq. 5. */
void oracle_lab8_tables(uint16_t *lin256, int32_t *mq9, uint16_t *f65536);
void oracle_lab8(const uint8_t *rgb, int W, int H, int stride, uint8_t *out);

/* BRIEF descriptor B(x) of Eq. 2-3 for every pixel. */
int oracle_describe(const uint8_t *rgb, int W, int H, int stride,
                    const int8_t *pattern, int n, uint64_t *desc);

/* Pair weights w(x,p_i,q_i) of Eq. 5 for one pixel (u, v). */
int oracle_weights(const uint8_t *rgb, int W, int H, int stride,
                   const int8_t *pattern, int n, int u, int v, int32_t *w);

/* Binary mask Phi(x) of Eq. 6-7 for every pixel; T (optional, [H][W])
 * receives the per-pixel threshold, the k-th smallest weight. */
int oracle_mask(const uint8_t *rgb, int W, int H, int stride,
                const int8_t *pattern, int n, int k, uint64_t *mask,
                int32_t *T);

/* Cost volume of Eq. 8 (Eq. 4 when mask == NULL). */
int oracle_cost_volume(const uint64_t *descL, const uint64_t *maskL,
                       const uint64_t *descR, int W, int H, int n, int dmax,
                       int16_t *cost);

/* Winner-take-all of Eq. 1 over a cost volume, lowest d on ties. */
int oracle_wta(const int16_t *cost, int W, int H, int dmax, int32_t *disp);

/* Whole hot path for one pair: descriptors of both views, mask of the left
 * (reference) view, cost, WTA.  cost may be NULL. */
int oracle_match(const uint8_t *left, const uint8_t *right, int W, int H,
                 int stride, const int8_t *pattern, int n, int k,
                 int use_mask, int dmax, int32_t *disp, int16_t *cost);

/* Right-reference matching, the second depth map of the left/right check
 * that opens the refinement step of Section 3: the right view is the
 * reference, pixel (u, v) of the right view is compared with (u + d, v) of
 * the left view, the mask is the right view's own (Eq. 5-7 on the right
 * image), a partner outside the image (u + d > W - 1) has no cost (32767),
 * ties take the lowest d.  cost may be NULL. */
int oracle_match_right(const uint8_t *left, const uint8_t *right, int W, int H,
                       int stride, const int8_t *pattern, int n, int k,
                       int use_mask, int dmax, int32_t *disp, int16_t *cost);

/* Left/right consistency check (Section 3, refinement step): out = dL
 * where |dL(u, v) - dR(u - dL(u, v), v)| <= tol, else -1. */
int oracle_lr_check(const int32_t *dL, const int32_t *dR, int W, int H,
                    int tol, int32_t *out);

/* Voting refinement (Section 3, Eq. 9-10) of the pixels the left/right
 * check marked invalid (checked < 0): d_x = argmax over d in [0, dmax - 1]
 * of W(x, d), the sum over valid pixels p (checked >= 0) with disparity d
 * in the (2 radius + 1)^2 window around x, inside the image, of
 * exp(-(c(x, p) / lambda_c + e(x, p) / lambda_e)); c = Euclidean distance of
 * the 8-bit CIELAB colours, e = Euclidean distance of the positions.  Ties
 * take the lowest d; an invalid pixel without any valid pixel in its window
 * keeps fallback(x); valid pixels keep checked(x).  Double precision.
 * W_out (optional, [H][W][dmax]) receives W(x, d) of invalid pixels (0
 * elsewhere). */
int oracle_vote_refine(const uint8_t *rgb, int W, int H, int stride,
                       const int32_t *checked, const int32_t *fallback,
                       int radius, int dmax, double lambda_c, double lambda_e,
                       int32_t *out, double *W_out);

#ifdef __cplusplus
}
#endif

#endif
