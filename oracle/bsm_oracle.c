/*
 * CPU oracle for the Binary Stereo Matching hot path (Zhang et al., "Binary
 * Stereo Matching", Section 3, Eq. 1-8).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the
 * benchmark's CPU-baseline leg.  It shares no code with the GPU library.
 *
 * Every step is the plain definition, written for a reader to check against
 * the paper by eye: no bit tricks beyond packing bits into uint64 words, no
 * blocking, no fusion.  Where the paper is silent the reading taken is named
 * at the step (intensity from RGB, CIELAB quantisation, image borders,
 * u - d < 0, tie-breaks).
 */
#include "bsm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

void oracle_set_threads(int threads) { g_threads = threads < 1 ? 1 : threads; }
int oracle_get_threads(void) { return g_threads; }

static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ------------------------------------------------------------------------ */
/* Step 0: the point-pair pattern.                                           */
/* Section 3 (after Eq. 2): n pairs <p_i, q_i>, each sampled from an         */
/* isotropic Gaussian centred on x inside an S x S window.  Section 4.1      */
/* fixes n = 4096, S = 26 and a spread of 4.  Reading: p and q are           */
/* independent draws; each coordinate is an integer offset                   */
/* floor(sigma*z + 0.5), redrawn while outside the window [-S/2, (S-1)/2];   */
/* q is redrawn while q == p.  z comes from splitmix64 (Steele, Lea and      */
/* Flood 2014) through the basic Box-Muller transform.                       */
/* ------------------------------------------------------------------------ */

uint64_t oracle_splitmix64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ull;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double oracle_normal(uint64_t *state)
{
    /* u1 in (0, 1], u2 in [0, 1), both with 53 random bits. */
    uint64_t a = oracle_splitmix64_next(state);
    uint64_t b = oracle_splitmix64_next(state);
    double u1 = (double)((a >> 11) + 1) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    double radius = sqrt(-2.0 * log(u1));
    double angle = 6.283185307179586 * u2;
    return radius * cos(angle);
}

static int draw_offset(uint64_t *state, double sigma, int lo, int hi)
{
    for (;;) {
        double z = oracle_normal(state);
        double o = floor(sigma * z + 0.5);
        if (o >= (double)lo && o <= (double)hi)
            return (int)o;
    }
}

int oracle_make_pattern(uint64_t seed, int n, int S, double sigma, int8_t *out)
{
    int lo = -(S / 2), hi = (S - 1) / 2;
    uint64_t state = seed;
    if (n < 1 || S < 2 || S > 64 || !(sigma > 0.0) || !out)
        return -1;
    for (int i = 0; i < n; i++) {
        int px = draw_offset(&state, sigma, lo, hi);
        int py = draw_offset(&state, sigma, lo, hi);
        int qx, qy;
        do {
            qx = draw_offset(&state, sigma, lo, hi);
            qy = draw_offset(&state, sigma, lo, hi);
        } while (qx == px && qy == py);
        out[4 * i + 0] = (int8_t)px;
        out[4 * i + 1] = (int8_t)py;
        out[4 * i + 2] = (int8_t)qx;
        out[4 * i + 3] = (int8_t)qy;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 1: intensity I(x) of Eq. 3.  The paper says only "intensity".        */
/* Reading: integer BT.601 luma, weights 77/150/29 summing to 256, so a      */
/* grey pixel keeps its value exactly.                                       */
/* ------------------------------------------------------------------------ */

void oracle_luma(const uint8_t *rgb, int W, int H, int stride, uint8_t *out)
{
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            const uint8_t *px = rgb + (size_t)v * stride + 3 * (size_t)u;
            int I = (77 * px[0] + 150 * px[1] + 29 * px[2] + 128) >> 8;
            out[(size_t)v * W + u] = (uint8_t)I;
        }
}

/* ------------------------------------------------------------------------ */
/* Step 2: CIELAB for the SAD of Eq. 5.  The paper names the colour space    */
/* only.  Reading: sRGB (IEC 61966-2-1) with the D65 white, L*a*b* from the  */
/* CIE 1976 definition, stored as 8-bit L8 = L*255/100, a8 = a+128,          */
/* b8 = b+128.  Floating point is used only to build three tables; the       */
/* per-pixel conversion is integer:                                          */
/*   LIN[c]  = round(65535 * decode(c/255))                                  */
/*   t_r     = (sum_c MQ[r][c] * LIN[c] + 8192) >> 14, MQ = Q14 of the       */
/*             sRGB->XYZ matrix with rows divided by the white point         */
/*             (rows then sum to exactly 16384)                              */
/*   F[t]    = round(65535 * f(t/65535)), f the CIE companding function      */
/*   L8 = rdiv(255*(116*F_Y - 16*65535), 100*65535)                          */
/*   a8 = 128 + rdiv(500*(F_X - F_Y), 65535)                                 */
/*   b8 = 128 + rdiv(200*(F_Y - F_Z), 65535)        (each clamped to 0..255) */
/* round() is half away from zero; rdiv(a,b) = floor((2a + b) / 2b).         */
/* ------------------------------------------------------------------------ */

static const double SRGB_TO_XYZ[3][3] = {
    {0.4124, 0.3576, 0.1805},
    {0.2126, 0.7152, 0.0722},
    {0.0193, 0.1192, 0.9505},
};

static double srgb_decode(double u)
{
    return u <= 0.04045 ? u / 12.92 : pow((u + 0.055) / 1.055, 2.4);
}

static double cie_f(double t)
{
    const double e = 6.0 / 29.0;
    return t > e * e * e ? cbrt(t) : t / (3.0 * e * e) + 4.0 / 29.0;
}

void oracle_lab8_tables(uint16_t *lin256, int32_t *mq9, uint16_t *f65536)
{
    for (int c = 0; c < 256; c++)
        lin256[c] = (uint16_t)lround(65535.0 * srgb_decode(c / 255.0));
    for (int r = 0; r < 3; r++) {
        double white = SRGB_TO_XYZ[r][0] + SRGB_TO_XYZ[r][1] + SRGB_TO_XYZ[r][2];
        int sum = 0, big = 0;
        for (int c = 0; c < 3; c++) {
            mq9[3 * r + c] = (int32_t)lround(16384.0 * SRGB_TO_XYZ[r][c] / white);
            sum += mq9[3 * r + c];
            if (mq9[3 * r + c] > mq9[3 * r + big])
                big = c;
        }
        mq9[3 * r + big] += 16384 - sum;
    }
    for (int t = 0; t < 65536; t++)
        f65536[t] = (uint16_t)lround(65535.0 * cie_f(t / 65535.0));
}

static int64_t rdiv(int64_t a, int64_t b)
{
    int64_t num = 2 * a + b, den = 2 * b;
    int64_t q = num / den;
    if ((num % den != 0) && (num < 0))
        q -= 1; /* floor, not truncation */
    return q;
}

void oracle_lab8(const uint8_t *rgb, int W, int H, int stride, uint8_t *out)
{
    uint16_t lin[256];
    int32_t mq[9];
    uint16_t *F = (uint16_t *)malloc(65536 * sizeof(uint16_t));
    oracle_lab8_tables(lin, mq, F);
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            const uint8_t *px = rgb + (size_t)v * stride + 3 * (size_t)u;
            int64_t fxyz[3];
            for (int r = 0; r < 3; r++) {
                int64_t acc = 0;
                for (int c = 0; c < 3; c++)
                    acc += (int64_t)mq[3 * r + c] * lin[px[c]];
                fxyz[r] = F[(acc + 8192) >> 14];
            }
            int64_t L = rdiv(255 * (116 * fxyz[1] - 16 * 65535), 100 * 65535);
            int64_t a = 128 + rdiv(500 * (fxyz[0] - fxyz[1]), 65535);
            int64_t b = 128 + rdiv(200 * (fxyz[1] - fxyz[2]), 65535);
            uint8_t *o = out + 3 * ((size_t)v * W + u);
            o[0] = (uint8_t)clampi((int)L, 0, 255);
            o[1] = (uint8_t)clampi((int)a, 0, 255);
            o[2] = (uint8_t)clampi((int)b, 0, 255);
        }
    free(F);
}

/* ------------------------------------------------------------------------ */
/* Step 3 (borders): the paper is silent.  Reading: a sample position        */
/* outside the image takes the nearest edge pixel (clamp each coordinate).  */
/* ------------------------------------------------------------------------ */

static int valid_pattern_args(int W, int H, int n, const int8_t *pattern)
{
    return W >= 1 && H >= 1 && n >= 64 && n % 64 == 0 && pattern != NULL;
}

/* ------------------------------------------------------------------------ */
/* Step 4: the BRIEF descriptor, Eq. 2 with the binary test of Eq. 3:        */
/*   B(x) = sum_{i=1..n} 2^(i-1) tau(p_i, q_i),  tau = [I(p_i) > I(q_i)].    */
/* Weight 2^(i-1) puts pair i at bit (i-1) mod 64 of word (i-1)/64.          */
/* ------------------------------------------------------------------------ */

static void describe_from_luma(const uint8_t *I, int W, int H,
                               const int8_t *pat, int n, uint64_t *desc)
{
    int nw = n / 64;
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            uint64_t *B = desc + ((size_t)v * W + u) * nw;
            for (int j = 0; j < nw; j++)
                B[j] = 0;
            for (int i = 1; i <= n; i++) {
                const int8_t *o = pat + 4 * (i - 1);
                int pu = clampi(u + o[0], 0, W - 1), pv = clampi(v + o[1], 0, H - 1);
                int qu = clampi(u + o[2], 0, W - 1), qv = clampi(v + o[3], 0, H - 1);
                int tau = I[(size_t)pv * W + pu] > I[(size_t)qv * W + qu] ? 1 : 0;
                B[(i - 1) / 64] |= (uint64_t)tau << ((i - 1) % 64);
            }
        }
}

int oracle_describe(const uint8_t *rgb, int W, int H, int stride,
                    const int8_t *pattern, int n, uint64_t *desc)
{
    if (!valid_pattern_args(W, H, n, pattern) || stride < 3 * W || !rgb || !desc)
        return -1;
    uint8_t *I = (uint8_t *)malloc((size_t)W * H);
    oracle_luma(rgb, W, H, stride, I);
    describe_from_luma(I, W, H, pattern, n, desc);
    free(I);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 5: the binary mask, Eq. 5-7, reference (left) view only.             */
/*   SAD(x,y)  = sum over L,a,b of |I_c(x) - I_c(y)|                          */
/*   w_i       = max(SAD(x,p_i), SAD(x,q_i))                       (Eq. 5)   */
/*   T         = the "quarter smallest" w: the k-th smallest, k = n/4 by     */
/*               default (1-indexed)                                          */
/*   delta_i   = [w_i <= T]                                        (Eq. 6)   */
/*   Phi(x)    = sum 2^(i-1) delta_i, same bit order as B          (Eq. 7)   */
/* ------------------------------------------------------------------------ */

static int sad_lab(const uint8_t *a, const uint8_t *b)
{
    return abs((int)a[0] - (int)b[0]) + abs((int)a[1] - (int)b[1]) +
           abs((int)a[2] - (int)b[2]);
}

static void weights_from_lab(const uint8_t *lab, int W, int H,
                             const int8_t *pat, int n, int u, int v,
                             int32_t *w)
{
    const uint8_t *x = lab + 3 * ((size_t)v * W + u);
    for (int i = 1; i <= n; i++) {
        const int8_t *o = pat + 4 * (i - 1);
        int pu = clampi(u + o[0], 0, W - 1), pv = clampi(v + o[1], 0, H - 1);
        int qu = clampi(u + o[2], 0, W - 1), qv = clampi(v + o[3], 0, H - 1);
        int sp = sad_lab(x, lab + 3 * ((size_t)pv * W + pu));
        int sq = sad_lab(x, lab + 3 * ((size_t)qv * W + qu));
        w[i - 1] = sp > sq ? sp : sq;
    }
}

int oracle_weights(const uint8_t *rgb, int W, int H, int stride,
                   const int8_t *pattern, int n, int u, int v, int32_t *w)
{
    if (!valid_pattern_args(W, H, n, pattern) || stride < 3 * W || !rgb || !w ||
        u < 0 || u >= W || v < 0 || v >= H)
        return -1;
    uint8_t *lab = (uint8_t *)malloc((size_t)W * H * 3);
    oracle_lab8(rgb, W, H, stride, lab);
    weights_from_lab(lab, W, H, pattern, n, u, v, w);
    free(lab);
    return 0;
}

static int cmp_int32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void mask_from_lab(const uint8_t *lab, int W, int H, const int8_t *pat,
                          int n, int k, uint64_t *mask, int32_t *Tout)
{
    int nw = n / 64;
#pragma omp parallel num_threads(g_threads)
    {
        int32_t *w = (int32_t *)malloc(sizeof(int32_t) * n);
        int32_t *sorted = (int32_t *)malloc(sizeof(int32_t) * n);
#pragma omp for schedule(dynamic)
        for (int v = 0; v < H; v++)
            for (int u = 0; u < W; u++) {
                weights_from_lab(lab, W, H, pat, n, u, v, w);
                memcpy(sorted, w, sizeof(int32_t) * n);
                qsort(sorted, n, sizeof(int32_t), cmp_int32);
                int32_t T = sorted[k - 1];
                uint64_t *M = mask + ((size_t)v * W + u) * nw;
                for (int j = 0; j < nw; j++)
                    M[j] = 0;
                for (int i = 1; i <= n; i++) {
                    int delta = w[i - 1] <= T ? 1 : 0;
                    M[(i - 1) / 64] |= (uint64_t)delta << ((i - 1) % 64);
                }
                if (Tout)
                    Tout[(size_t)v * W + u] = T;
            }
        free(w);
        free(sorted);
    }
}

int oracle_mask(const uint8_t *rgb, int W, int H, int stride,
                const int8_t *pattern, int n, int k, uint64_t *mask, int32_t *T)
{
    if (!valid_pattern_args(W, H, n, pattern) || stride < 3 * W || !rgb ||
        !mask || k < 1 || k > n)
        return -1;
    uint8_t *lab = (uint8_t *)malloc((size_t)W * H * 3);
    oracle_lab8(rgb, W, H, stride, lab);
    mask_from_lab(lab, W, H, pattern, n, k, mask, T);
    free(lab);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 6: the cost of Eq. 8 (Eq. 4 when no mask is given):                  */
/*   C(x,d) = || (B(x) XOR B(x_d)) AND Phi(x) ||_1,   x_d = (u - d, v).       */
/* Readings: the left view is the reference; XOR binds before AND (the mask  */
/* selects which differing bits count); d ranges over [0, dmax - 1]; a       */
/* partner outside the image (u - d < 0) has no cost and is stored as 32767. */
/* ------------------------------------------------------------------------ */

#define ORACLE_INVALID_COST 32767

static int cost_at(const uint64_t *descL, const uint64_t *maskL,
                   const uint64_t *descR, int W, int nw, int u, int v, int d)
{
    const uint64_t *BL = descL + ((size_t)v * W + u) * nw;
    const uint64_t *BR = descR + ((size_t)v * W + (u - d)) * nw;
    const uint64_t *M = maskL ? maskL + ((size_t)v * W + u) * nw : NULL;
    int c = 0;
    for (int j = 0; j < nw; j++) {
        uint64_t x = BL[j] ^ BR[j];
        if (M)
            x &= M[j];
        c += __builtin_popcountll(x);
    }
    return c;
}

int oracle_cost_volume(const uint64_t *descL, const uint64_t *maskL,
                       const uint64_t *descR, int W, int H, int n, int dmax,
                       int16_t *cost)
{
    int nw = n / 64;
    if (W < 1 || H < 1 || n < 64 || n % 64 || dmax < 1 || dmax > W || !descL ||
        !descR || !cost)
        return -1;
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int v = 0; v < H; v++)
        for (int d = 0; d < dmax; d++)
            for (int u = 0; u < W; u++)
                cost[((size_t)d * H + v) * W + u] =
                    (int16_t)(u - d < 0 ? ORACLE_INVALID_COST
                                        : cost_at(descL, maskL, descR, W, nw, u, v, d));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 7: winner-take-all, Eq. 1: d_x = argmin_d C(x,d) over [0, dmax-1].   */
/* Reading: ties go to the lowest d.  d = 0 is always valid (u - 0 >= 0).    */
/* ------------------------------------------------------------------------ */

int oracle_wta(const int16_t *cost, int W, int H, int dmax, int32_t *disp)
{
    if (W < 1 || H < 1 || dmax < 1 || !cost || !disp)
        return -1;
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            int best_d = 0;
            int best_c = cost[((size_t)0 * H + v) * W + u];
            for (int d = 1; d < dmax; d++) {
                int c = cost[((size_t)d * H + v) * W + u];
                if (c < best_c) {
                    best_c = c;
                    best_d = d;
                }
            }
            disp[(size_t)v * W + u] = best_d;
        }
    return 0;
}

int oracle_match(const uint8_t *left, const uint8_t *right, int W, int H,
                 int stride, const int8_t *pattern, int n, int k, int use_mask,
                 int dmax, int32_t *disp, int16_t *cost)
{
    int nw = n / 64;
    if (!valid_pattern_args(W, H, n, pattern) || stride < 3 * W || !left ||
        !right || !disp || dmax < 1 || dmax > W || (use_mask && (k < 1 || k > n)))
        return -1;
    size_t npx = (size_t)W * H;
    uint8_t *I = (uint8_t *)malloc(npx);
    uint64_t *descL = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
    uint64_t *descR = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
    uint64_t *maskL = NULL;

    oracle_luma(left, W, H, stride, I);
    describe_from_luma(I, W, H, pattern, n, descL);
    oracle_luma(right, W, H, stride, I);
    describe_from_luma(I, W, H, pattern, n, descR);
    if (use_mask) {
        uint8_t *lab = (uint8_t *)malloc(npx * 3);
        maskL = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
        oracle_lab8(left, W, H, stride, lab);
        mask_from_lab(lab, W, H, pattern, n, k, maskL, NULL);
        free(lab);
    }

#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            int best_d = 0, best_c = 0;
            for (int d = 0; d < dmax; d++) {
                int c = u - d < 0 ? ORACLE_INVALID_COST
                                  : cost_at(descL, maskL, descR, W, nw, u, v, d);
                if (cost)
                    cost[((size_t)d * H + v) * W + u] = (int16_t)c;
                if (d == 0 || c < best_c) {
                    best_c = c;
                    best_d = d;
                }
            }
            disp[(size_t)v * W + u] = best_d;
        }

    free(I);
    free(descL);
    free(descR);
    free(maskL);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-reference matching and the left/right check (Section 3, the first  */
/* part of the refinement step: two depth maps, one per reference view,     */
/* classify each left pixel as valid or invalid).  Reading: the right map    */
/* uses the same pattern, the right view's own mask, x_d = (u + d, v), and   */
/* a pixel is valid when the two maps agree within 1 (the customary check   */
/* of the cited two-view methods).                                          */
/* ------------------------------------------------------------------------ */

int oracle_match_right(const uint8_t *left, const uint8_t *right, int W, int H,
                       int stride, const int8_t *pattern, int n, int k,
                       int use_mask, int dmax, int32_t *disp, int16_t *cost)
{
    int nw = n / 64;
    if (!valid_pattern_args(W, H, n, pattern) || stride < 3 * W || !left ||
        !right || !disp || dmax < 1 || dmax > W || (use_mask && (k < 1 || k > n)))
        return -1;
    size_t npx = (size_t)W * H;
    uint8_t *I = (uint8_t *)malloc(npx);
    uint64_t *descL = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
    uint64_t *descR = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
    uint64_t *maskR = NULL;

    oracle_luma(left, W, H, stride, I);
    describe_from_luma(I, W, H, pattern, n, descL);
    oracle_luma(right, W, H, stride, I);
    describe_from_luma(I, W, H, pattern, n, descR);
    if (use_mask) {
        uint8_t *lab = (uint8_t *)malloc(npx * 3);
        maskR = (uint64_t *)malloc(npx * nw * sizeof(uint64_t));
        oracle_lab8(right, W, H, stride, lab);
        mask_from_lab(lab, W, H, pattern, n, k, maskR, NULL);
        free(lab);
    }

#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            const uint64_t *BR = descR + ((size_t)v * W + u) * nw;
            const uint64_t *M = maskR ? maskR + ((size_t)v * W + u) * nw : NULL;
            int best_d = 0, best_c = 0;
            for (int d = 0; d < dmax; d++) {
                int c = ORACLE_INVALID_COST;
                if (u + d <= W - 1) {
                    const uint64_t *BL = descL + ((size_t)v * W + (u + d)) * nw;
                    c = 0;
                    for (int j = 0; j < nw; j++) {
                        uint64_t x = BR[j] ^ BL[j];
                        if (M)
                            x &= M[j];
                        c += __builtin_popcountll(x);
                    }
                }
                if (cost)
                    cost[((size_t)d * H + v) * W + u] = (int16_t)c;
                if (d == 0 || c < best_c) {
                    best_c = c;
                    best_d = d;
                }
            }
            disp[(size_t)v * W + u] = best_d;
        }

    free(I);
    free(descL);
    free(descR);
    free(maskR);
    return 0;
}

int oracle_lr_check(const int32_t *dL, const int32_t *dR, int W, int H,
                    int tol, int32_t *out)
{
    if (W < 1 || H < 1 || tol < 0 || !dL || !dR || !out)
        return -1;
    for (int v = 0; v < H; v++)
        for (int u = 0; u < W; u++) {
            int d = dL[(size_t)v * W + u];
            int ok = 0;
            if (d >= 0 && u - d >= 0) {
                int e = d - dR[(size_t)v * W + (u - d)];
                ok = (e < 0 ? -e : e) <= tol;
            }
            out[(size_t)v * W + u] = ok ? d : -1;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Voting refinement, Eq. 9-10 (the second part of Section 3's refinement   */
/* step).  Readings: the voters of x are the valid pixels of the window of  */
/* radius `radius` around x that lie inside the image; c is the Euclidean   */
/* distance of the Lab8 colours (the colour space of the mask); e is the    */
/* Euclidean distance of the pixel positions; argmax ties take the lowest  */
/* d; a pixel without voters keeps the fallback disparity.                 */
/* ------------------------------------------------------------------------ */

int oracle_vote_refine(const uint8_t *rgb, int W, int H, int stride,
                       const int32_t *checked, const int32_t *fallback,
                       int radius, int dmax, double lambda_c, double lambda_e,
                       int32_t *out, double *W_out)
{
    if (W < 1 || H < 1 || stride < 3 * W || !rgb || !checked || !fallback || !out ||
        radius < 0 || dmax < 1 || !(lambda_c > 0) || !(lambda_e > 0))
        return -1;
    size_t npx = (size_t)W * H;
    uint8_t *lab = (uint8_t *)malloc(npx * 3);
    oracle_lab8(rgb, W, H, stride, lab);
    if (W_out)
        memset(W_out, 0, npx * dmax * sizeof(double));
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int v = 0; v < H; v++) {
        double *acc = (double *)malloc(sizeof(double) * dmax);
        for (int u = 0; u < W; u++) {
            size_t x = (size_t)v * W + u;
            if (checked[x] >= 0) {
                out[x] = checked[x];
                continue;
            }
            for (int d = 0; d < dmax; d++)
                acc[d] = 0.0;
            int voters = 0;
            const uint8_t *cx = lab + 3 * x;
            for (int dy = -radius; dy <= radius; dy++)
                for (int dx = -radius; dx <= radius; dx++) {
                    int pu = u + dx, pv = v + dy;
                    if (pu < 0 || pu >= W || pv < 0 || pv >= H)
                        continue;
                    size_t p = (size_t)pv * W + pu;
                    int d = checked[p];
                    if (d < 0 || d >= dmax)
                        continue;
                    const uint8_t *cp = lab + 3 * p;
                    double dl = (double)cx[0] - cp[0], da = (double)cx[1] - cp[1],
                           db = (double)cx[2] - cp[2];
                    double c = sqrt(dl * dl + da * da + db * db);
                    double e = sqrt((double)dx * dx + (double)dy * dy);
                    acc[d] += exp(-(c / lambda_c + e / lambda_e));
                    voters++;
                }
            int best = fallback[x];
            if (voters > 0) {
                best = 0;
                for (int d = 1; d < dmax; d++)
                    if (acc[d] > acc[best])
                        best = d;
            }
            out[x] = best;
            if (W_out)
                memcpy(W_out + x * dmax, acc, sizeof(double) * dmax);
        }
        free(acc);
    }
    free(lab);
    return 0;
}
