// HIP kernels of the BSM hot path for gfx950 (CDNA4, wave64).
//
//   k_color     colour pre-pass: intensity (Eq. 3) and 8-bit CIELAB (Eq. 5)
//   k_describe  BRIEF descriptor (Eq. 2-3) and binary mask (Eq. 5-7)
//   k_cost_wta  masked Hamming cost (Eq. 8 / Eq. 4) fused with WTA (Eq. 1)
//
// Nothing on this path is a dense contraction, so there is no MFMA: the
// kernels are bound by integer VALU issue (cost, descriptor) or HBM (colour).
#include "bsm_internal.h"

namespace bsm {
namespace {

// ---------------------------------------------------------------------------
// K1: colour pre-pass.  One thread per pixel; output uint32 per pixel:
// byte 0 L8, byte 1 a8, byte 2 b8, byte 3 intensity I.
// ---------------------------------------------------------------------------

// floor((2a + b) / (2b)) for b > 0: a / b rounded to nearest, halves up.
__device__ __forceinline__ int32_t nearest_div(int64_t a, int64_t b) {
  const int64_t num = 2 * a + b, den = 2 * b;
  int64_t q = num / den;
  if (q * den > num) --q;
  return static_cast<int32_t>(q);
}

__device__ __forceinline__ uint32_t clamp_u8(int32_t x) {
  return static_cast<uint32_t>(x < 0 ? 0 : (x > 255 ? 255 : x));
}

constexpr int kColorTX = 64, kColorTY = 4;

__global__ __launch_bounds__(256) void k_color(const uint8_t *__restrict__ img, int W, int H,
                                               int stride, uint32_t *__restrict__ out,
                                               const uint16_t *__restrict__ lin,
                                               const uint16_t *__restrict__ ftab, Mq mq,
                                               int want_lab) {
  const int u = blockIdx.x * kColorTX + (threadIdx.x % kColorTX);
  const int v = blockIdx.y * kColorTY + (threadIdx.x / kColorTX);
  if (u >= W || v >= H) return;
  const uint8_t *px = img + (size_t)v * stride + 3 * (size_t)u;
  const int32_t R = px[0], G = px[1], B = px[2];
  uint32_t word = static_cast<uint32_t>((77 * R + 150 * G + 29 * B + 128) >> 8) << 24;
  if (want_lab) {
    const int32_t lr = lin[R], lg = lin[G], lb = lin[B];
    const int32_t fx = ftab[(mq.m[0] * lr + mq.m[1] * lg + mq.m[2] * lb + 8192) >> 14];
    const int32_t fy = ftab[(mq.m[3] * lr + mq.m[4] * lg + mq.m[5] * lb + 8192) >> 14];
    const int32_t fz = ftab[(mq.m[6] * lr + mq.m[7] * lg + mq.m[8] * lb + 8192) >> 14];
    const uint32_t L8 = clamp_u8(nearest_div(255 * (116 * (int64_t)fy - 16 * 65535), 100 * 65535));
    const uint32_t a8 = clamp_u8(128 + nearest_div(500 * (int64_t)(fx - fy), 65535));
    const uint32_t b8 = clamp_u8(128 + nearest_div(200 * (int64_t)(fy - fz), 65535));
    word |= L8 | (a8 << 8) | (b8 << 16);
  }
  out[(size_t)v * W + u] = word;
}

// ---------------------------------------------------------------------------
// K2: descriptor and mask.  A block stages a TH x TW tile of packed pixels
// plus a halo of `radius` in LDS (coordinates clamped to the image, which is
// exactly the border rule).  Each wave then walks its pixels one at a time
// with the 64 lanes spread over point pairs: lane l of word j evaluates pair
// 64 j + l, so the wave-wide ballot of the binary test IS word j of B(x)
// (bit l = pair 64 j + l + 1).  For the mask each lane keeps its pair
// weights in registers and the k-th smallest weight T is found by bisection
// on [0, 765], each probe counting ballot(w <= t) words with a popcount.
// ---------------------------------------------------------------------------
constexpr int kDescTW = 32, kDescTH = 8, kDescThreads = 256;

template <int NWMAX, bool MASK>
__global__ __launch_bounds__(kDescThreads) void k_describe(
    const uint32_t *__restrict__ packed, int W, int H, const int8_t *__restrict__ pattern, int nw,
    int radius, int pitch, int k, uint64_t *__restrict__ desc, uint64_t *__restrict__ mask) {
  extern __shared__ uint32_t tile[];
  const int u0 = blockIdx.x * kDescTW, v0 = blockIdx.y * kDescTH;
  const int rows = kDescTH + 2 * radius, cols = kDescTW + 2 * radius;
  for (int i = threadIdx.x; i < rows * cols; i += kDescThreads) {
    const int ty = i / cols, tx = i - ty * cols;
    const int gv = min(max(v0 - radius + ty, 0), H - 1);
    const int gu = min(max(u0 - radius + tx, 0), W - 1);
    tile[ty * pitch + tx] = packed[(size_t)gv * W + gu];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // LDS offsets (relative to the centre) of this lane's pairs.
  int offp[NWMAX], offq[NWMAX];
  const int32_t *pat32 = reinterpret_cast<const int32_t *>(pattern);
#pragma unroll
  for (int j = 0; j < NWMAX; ++j) {
    offp[j] = offq[j] = 0;
    if (j < nw) {
      const int32_t e = pat32[64 * j + lane];
      const int px = (int8_t)(e & 0xff), py = (int8_t)((e >> 8) & 0xff);
      const int qx = (int8_t)((e >> 16) & 0xff), qy = (int8_t)((e >> 24) & 0xff);
      offp[j] = py * pitch + px;
      offq[j] = qy * pitch + qx;
    }
  }
  __syncthreads();

  constexpr int kPixPerWave = kDescTW * kDescTH / (kDescThreads / 64);
  for (int p = 0; p < kPixPerWave; ++p) {
    const int ty = wave * (kPixPerWave / kDescTW) + p / kDescTW, tx = p % kDescTW;
    const int u = u0 + tx, v = v0 + ty;
    if (u >= W || v >= H) continue;  // uniform across the wave
    const int c = (ty + radius) * pitch + (tx + radius);
    const uint32_t centre = tile[c] & 0xffffffu;
    uint64_t out_desc = 0, out_mask = 0;
    uint32_t w[NWMAX];
#pragma unroll
    for (int j = 0; j < NWMAX; ++j) {
      w[j] = 0;
      if (j < nw) {
        const uint32_t a = tile[c + offp[j]], b = tile[c + offq[j]];
        const uint64_t bits = __ballot((a >> 24) > (b >> 24));  // tau of Eq. 3
        if (lane == j) out_desc = bits;
        if (MASK) {
          const uint32_t sp = __builtin_amdgcn_sad_u8(a & 0xffffffu, centre, 0u);
          const uint32_t sq = __builtin_amdgcn_sad_u8(b & 0xffffffu, centre, 0u);
          w[j] = sp > sq ? sp : sq;  // Eq. 5
        }
      }
    }
    if (MASK) {
      // smallest t with #{w <= t} >= k, i.e. the k-th smallest weight
      int lo = 0, hi = 3 * 255;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        int count = 0;
#pragma unroll
        for (int j = 0; j < NWMAX; ++j)
          if (j < nw) count += __popcll(__ballot(w[j] <= (uint32_t)mid));
        if (count >= k)
          hi = mid;
        else
          lo = mid + 1;
      }
#pragma unroll
      for (int j = 0; j < NWMAX; ++j)
        if (j < nw) {
          const uint64_t bits = __ballot(w[j] <= (uint32_t)lo);  // Eq. 6-7
          if (lane == j) out_mask = bits;
        }
    }
    const size_t base = ((size_t)v * W + u) * nw;
    if (lane < nw) {
      desc[base + lane] = out_desc;
      if (MASK) mask[base + lane] = out_mask;
    }
  }
}

// ---------------------------------------------------------------------------
// K3 (fast): masked cost fused with winner-take-all, n = 64 NW bits,
// NW in {1, 2, 4, 8, 16}.
//
// One wave per (row v, 128-pixel tile).  Lane l owns the two adjacent left
// pixels a = u0 + 2l and b = a + 1, with their B_L and Phi in registers.
// Disparities are walked in order; at step d lane l reads B_R(a - d) from
// LDS and uses it for (a, d) now and for (b, d + 1) at the next step, since
// b - (d + 1) = a - d: every right descriptor fetched from LDS serves two
// evaluations.  The right descriptors of the window a disparity chunk needs
// sit in LDS word-major and split by parity, so at any step the 64 lanes
// read 64 consecutive 8-byte words (no bank conflicts).  Each evaluation is
// (bl ^ br) & m per 32-bit half (one v_bitop3_b32) plus a popcount that
// accumulates for free (v_bcnt_u32_b32); the running minimum of the key
// (C << 16) | d gives the lowest d among equal costs.  The cost volume, when
// wanted, is stored [d][v][u], so the two int16 costs of a lane form one
// coalesced 32-bit store per step.
// ---------------------------------------------------------------------------
constexpr int kCostTX = 128;     // pixels per wave
constexpr int kCostDC = 64;      // disparities per LDS window
constexpr int kCostHP = 97;      // words per parity half (>= (127 + 64) / 2, odd)

__device__ __forceinline__ uint32_t masked_cost(const uint64_t *bl, const uint64_t *m,
                                                const uint64_t *br, int nwords, bool use_mask) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < nwords; ++j) {
    const uint64_t x = use_mask ? ((bl[j] ^ br[j]) & m[j]) : (bl[j] ^ br[j]);
    c += __popcll(x);
  }
  return c;
}

template <int NW, bool MASK, bool VOL>
__global__ __launch_bounds__(64) void k_cost_wta_fast(const uint64_t *__restrict__ descL,
                                                      const uint64_t *__restrict__ maskL,
                                                      const uint64_t *__restrict__ descR, int W,
                                                      int H, int dmax, int32_t *__restrict__ disp,
                                                      int16_t *__restrict__ cost) {
  extern __shared__ uint64_t win[];  // [NW][2][kCostHP]
  const int lane = threadIdx.x;
  const int v = blockIdx.y;
  const int u0 = blockIdx.x * kCostTX;
  const int a = u0 + 2 * lane, b = a + 1;
  const bool has_a = a < W, has_b = b < W;

  uint64_t bla[NW], blb[NW], ma[NW], mb[NW];
  {
    const uint64_t *pa = descL + ((size_t)v * W + (has_a ? a : 0)) * NW;
    const uint64_t *pb = descL + ((size_t)v * W + (has_b ? b : 0)) * NW;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      bla[j] = has_a ? pa[j] : 0;
      blb[j] = has_b ? pb[j] : 0;
    }
    if (MASK) {
      const uint64_t *qa = maskL + ((size_t)v * W + (has_a ? a : 0)) * NW;
      const uint64_t *qb = maskL + ((size_t)v * W + (has_b ? b : 0)) * NW;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        ma[j] = has_a ? qa[j] : 0;
        mb[j] = has_b ? qb[j] : 0;
      }
    }
  }
  const uint64_t *rowR = descR + (size_t)v * W * NW;
  uint32_t best_a = 0xffffffffu, best_b = 0xffffffffu;

  for (int dc0 = 0; dc0 < dmax; dc0 += kCostDC) {
    const int dc1 = min(dmax, dc0 + kCostDC);
    const int r_lo = u0 - dc1 + 1;               // first right pixel of the window
    const int P = kCostTX - 1 + (dc1 - dc0);     // window width
    __syncthreads();                             // previous window fully consumed
    for (int i = lane; i < P * NW; i += 64) {
      const int rel = i / NW, j = i % NW;
      const int r = r_lo + rel;
      const uint64_t val = (r >= 0 && r < W) ? rowR[(size_t)r * NW + j] : 0;
      win[(j * 2 + (rel & 1)) * kCostHP + (rel >> 1)] = val;
    }
    __syncthreads();

    // B_R(b - dc0): relative index 2l + (dc1 - dc0)
    uint64_t prev[NW], cur[NW];
    {
      const int rel = 2 * lane + (dc1 - dc0);
#pragma unroll
      for (int j = 0; j < NW; ++j) prev[j] = win[(j * 2 + (rel & 1)) * kCostHP + (rel >> 1)];
    }
    const bool edge = u0 < dc1 - 1;  // some a - d < 0 inside this chunk
    for (int d = dc0; d < dc1; ++d) {
      const int e = dc1 - 1 - d;  // B_R(a - d): relative index 2l + e
      const uint64_t *src = win + (e & 1) * kCostHP + lane + (e >> 1);
#pragma unroll
      for (int j = 0; j < NW; ++j) cur[j] = src[j * 2 * kCostHP];
      const uint32_t ca = masked_cost(bla, ma, cur, NW, MASK);
      const uint32_t cb = masked_cost(blb, mb, prev, NW, MASK);
      const bool va = !edge || a - d >= 0, vb = !edge || b - d >= 0;
      const uint32_t ka = (ca << 16) | (uint32_t)d, kb = (cb << 16) | (uint32_t)d;
      if (va) best_a = min(best_a, ka);
      if (vb) best_b = min(best_b, kb);
      if (VOL) {
        const uint32_t sa = va ? ca : (uint32_t)kInvalidCost;
        const uint32_t sb = vb ? cb : (uint32_t)kInvalidCost;
        int16_t *plane = cost + ((size_t)d * H + v) * W;
        if (has_b && ((((size_t)d * H + v) * W) & 1) == 0) {
          *reinterpret_cast<uint32_t *>(plane + a) = sa | (sb << 16);
        } else {
          if (has_a) plane[a] = (int16_t)sa;
          if (has_b) plane[b] = (int16_t)sb;
        }
      }
#pragma unroll
      for (int j = 0; j < NW; ++j) prev[j] = cur[j];
    }
  }
  if (has_a) disp[(size_t)v * W + a] = (int32_t)(best_a & 0xffffu);
  if (has_b) disp[(size_t)v * W + b] = (int32_t)(best_b & 0xffffu);
}

// ---------------------------------------------------------------------------
// K3 (generic): any n = 64 nw bits, nw <= 64.  Lanes over disparities; the
// left descriptor and mask of the current pixel are wave-uniform (scalar
// loads); the right descriptors of the window sit in LDS word-major.
// ---------------------------------------------------------------------------
constexpr int kGenTX = 32;
constexpr int kGenWin = kGenTX + 63;  // right pixels per window

__global__ __launch_bounds__(64) void k_cost_wta_generic(const uint64_t *__restrict__ descL,
                                                         const uint64_t *__restrict__ maskL,
                                                         const uint64_t *__restrict__ descR, int W,
                                                         int H, int nw, int dmax,
                                                         int32_t *__restrict__ disp,
                                                         int16_t *__restrict__ cost) {
  extern __shared__ uint64_t gwin[];  // [nw][kGenWin]
  const int lane = threadIdx.x;
  const int v = blockIdx.y;
  const int u0 = blockIdx.x * kGenTX;
  const uint64_t *rowR = descR + (size_t)v * W * nw;
  uint32_t best = 0xffffffffu;  // lane p < kGenTX: best key of pixel u0 + p
  for (int dc0 = 0; dc0 < dmax; dc0 += 64) {
    const int r_lo = u0 - dc0 - 63;
    __syncthreads();
    for (int i = lane; i < kGenWin * nw; i += 64) {
      const int rel = i / nw, j = i - rel * nw;
      const int r = r_lo + rel;
      gwin[j * kGenWin + rel] = (r >= 0 && r < W) ? rowR[(size_t)r * nw + j] : 0;
    }
    __syncthreads();
    const int d = dc0 + lane;
    for (int p = 0; p < kGenTX; ++p) {
      const int u = u0 + p;
      if (u >= W) break;
      const uint64_t *bl = descL + ((size_t)v * W + u) * nw;
      const uint64_t *m = maskL ? maskL + ((size_t)v * W + u) * nw : nullptr;
      const int rel = p + 63 - lane;  // right pixel u - d
      uint32_t c = 0;
      for (int j = 0; j < nw; ++j) {
        uint64_t x = bl[j] ^ gwin[j * kGenWin + rel];
        if (m) x &= m[j];
        c += __popcll(x);
      }
      const bool valid = d < dmax && u - d >= 0;
      uint32_t key = valid ? ((c << 16) | (uint32_t)d) : 0xffffffffu;
      if (cost && d < dmax) cost[((size_t)d * H + v) * W + u] = (int16_t)(valid ? c : kInvalidCost);
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) key = min(key, (uint32_t)__shfl_xor((int)key, s));
      if (lane == p) best = min(best, key);
    }
  }
  if (lane < kGenTX && u0 + lane < W) disp[(size_t)v * W + u0 + lane] = (int32_t)(best & 0xffffu);
}

template <int NWMAX>
hipError_t launch_describe_t(const uint32_t *packed, int W, int H, const DeviceTables &t,
                             uint64_t *desc, uint64_t *mask, hipStream_t s) {
  const int pitch = kDescTW + 2 * t.radius + 1;
  const size_t lds = describe_lds_bytes(t.radius);
  dim3 grid((W + kDescTW - 1) / kDescTW, (H + kDescTH - 1) / kDescTH);
  if (mask)
    hipLaunchKernelGGL((k_describe<NWMAX, true>), grid, dim3(kDescThreads), lds, s, packed, W, H,
                       t.pattern, t.nw, t.radius, pitch, t.k, desc, mask);
  else
    hipLaunchKernelGGL((k_describe<NWMAX, false>), grid, dim3(kDescThreads), lds, s, packed, W, H,
                       t.pattern, t.nw, t.radius, pitch, t.k, desc, mask);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_cost_fast(const uint64_t *descL, const uint64_t *maskL, const uint64_t *descR,
                            int W, int H, int dmax, int32_t *disp, int16_t *cost, hipStream_t s) {
  dim3 grid((W + kCostTX - 1) / kCostTX, H);
  const size_t lds = (size_t)NW * 2 * kCostHP * sizeof(uint64_t);
#define BSM_LAUNCH_COST(M, V)                                                                     \
  hipLaunchKernelGGL((k_cost_wta_fast<NW, M, V>), grid, dim3(64), lds, s, descL, maskL, descR, W, \
                     H, dmax, disp, cost)
  if (maskL) {
    if (cost) BSM_LAUNCH_COST(true, true);
    else BSM_LAUNCH_COST(true, false);
  } else {
    if (cost) BSM_LAUNCH_COST(false, true);
    else BSM_LAUNCH_COST(false, false);
  }
#undef BSM_LAUNCH_COST
  return hipGetLastError();
}

}  // namespace

size_t describe_lds_bytes(int radius) {
  const int pitch = kDescTW + 2 * radius + 1;
  return (size_t)(kDescTH + 2 * radius) * pitch * sizeof(uint32_t);
}

hipError_t launch_color(const uint8_t *img, int W, int H, int stride, uint32_t *packed,
                        int want_lab, const DeviceTables &t, hipStream_t s) {
  dim3 grid((W + kColorTX - 1) / kColorTX, (H + kColorTY - 1) / kColorTY);
  hipLaunchKernelGGL(k_color, grid, dim3(kColorTX * kColorTY), 0, s, img, W, H, stride, packed,
                     t.lin, t.f, t.mq, want_lab);
  return hipGetLastError();
}

hipError_t launch_describe(const uint32_t *packed, int W, int H, const DeviceTables &t,
                           uint64_t *desc, uint64_t *mask, hipStream_t s) {
  if (t.nw <= 1) return launch_describe_t<1>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 2) return launch_describe_t<2>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 4) return launch_describe_t<4>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 8) return launch_describe_t<8>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 16) return launch_describe_t<16>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 32) return launch_describe_t<32>(packed, W, H, t, desc, mask, s);
  return launch_describe_t<64>(packed, W, H, t, desc, mask, s);
}

hipError_t launch_cost_wta(const uint64_t *descL, const uint64_t *maskL, const uint64_t *descR,
                           int W, int H, int nw, int dmax, int32_t *disp, int16_t *cost,
                           hipStream_t s) {
  switch (nw) {
    case 1: return launch_cost_fast<1>(descL, maskL, descR, W, H, dmax, disp, cost, s);
    case 2: return launch_cost_fast<2>(descL, maskL, descR, W, H, dmax, disp, cost, s);
    case 4: return launch_cost_fast<4>(descL, maskL, descR, W, H, dmax, disp, cost, s);
    case 8: return launch_cost_fast<8>(descL, maskL, descR, W, H, dmax, disp, cost, s);
    case 16: return launch_cost_fast<16>(descL, maskL, descR, W, H, dmax, disp, cost, s);
    default: break;
  }
  dim3 grid((W + kGenTX - 1) / kGenTX, H);
  const size_t lds = (size_t)nw * kGenWin * sizeof(uint64_t);
  hipLaunchKernelGGL(k_cost_wta_generic, grid, dim3(64), lds, s, descL, maskL, descR, W, H, nw,
                     dmax, disp, cost);
  return hipGetLastError();
}

}  // namespace bsm
