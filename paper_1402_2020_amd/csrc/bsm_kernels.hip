// HIP kernels of the BSM hot path for gfx950 (CDNA4, wave64).
//
//   colour        intensity (Eq. 3) and 8-bit CIELAB (Eq. 5) per pixel
//   describe+mask BRIEF descriptor (Eq. 2-3) and binary mask (Eq. 5-7)
//   describe      BRIEF descriptor only (the non-reference view)
//   cost+WTA      masked Hamming cost (Eq. 8 / Eq. 4) fused with WTA (Eq. 1)
//
// Each stage is a per-tile device function.  The single-pair kernels map
// one workgroup to one tile; the batch kernels are persistent and pull the
// tiles of many pairs from a device work list, so both paths run the same
// per-tile code.  The kernels are bound by integer VALU/SALU issue or by
// HBM, except the cost + WTA without a volume, which runs the masked Hamming
// cost as an int8 dot product on the matrix cores.
#include <type_traits>

#include "bsm_internal.h"

namespace bsm {
namespace {

constexpr int kXcds = 8;  // accelerator complex dies of an MI355X

// A wave-uniform value pinned to scalar registers.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <typename T>
__device__ __forceinline__ T *uniform(T *p) {
  const uint64_t x = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
  const uint32_t hi =
      static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x >> 32)));
  return reinterpret_cast<T *>((static_cast<uint64_t>(hi) << 32) | lo);
}

// The wave's index in its workgroup, marked wave-uniform: derived from
// threadIdx.x, it would otherwise make every row and address computed from
// it per-lane vector arithmetic (64-bit multiplies included).
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// ===========================================================================
// Colour pre-pass.  Output uint32 per pixel: byte 0 L8, byte 1 a8, byte 2 b8,
// byte 3 intensity I.  Tiles of 64 x (4 RPT) pixels, RPT rows per thread:
// one for the single-pair kernel (even a 128 x 96 view gets 48 workgroups),
// eight for the persistent batch kernel (fewer queue pulls).
// ===========================================================================
constexpr int kColorTX = 64, kColorThreads = 256;
constexpr int kColorRows = kColorThreads / kColorTX;     // rows per pass
constexpr int kColorRPT = 1, kBatchColorRPT = 8;        // passes per tile
constexpr int kColorTY = kColorRows * kColorRPT, kBatchColorTY = kColorRows * kBatchColorRPT;

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

// mirror != 0 writes pixel u of a row to column W - 1 - u (the horizontally
// mirrored view, used for right-reference matching).
template <int RPT>
__device__ __forceinline__ void color_tile(const uint8_t *__restrict__ img, int W, int H,
                                           int stride, uint32_t *__restrict__ out,
                                           const uint16_t *__restrict__ lin,
                                           const uint16_t *__restrict__ ftab, const Mq &mq,
                                           int want_lab, int mirror, int u0, int v0) {
  const int u = u0 + (threadIdx.x % kColorTX);
  if (u >= W) return;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int v = v0 + r * kColorRows + (threadIdx.x / kColorTX);
    if (v >= H) return;
    const uint8_t *px = img + (size_t)v * stride + 3 * (size_t)u;
    const int32_t R = px[0], G = px[1], B = px[2];
    uint32_t word = static_cast<uint32_t>((77 * R + 150 * G + 29 * B + 128) >> 8) << 24;
    if (want_lab) {
      const int32_t lr = lin[R], lg = lin[G], lb = lin[B];
      const int32_t fx = ftab[(mq.m[0] * lr + mq.m[1] * lg + mq.m[2] * lb + 8192) >> 14];
      const int32_t fy = ftab[(mq.m[3] * lr + mq.m[4] * lg + mq.m[5] * lb + 8192) >> 14];
      const int32_t fz = ftab[(mq.m[6] * lr + mq.m[7] * lg + mq.m[8] * lb + 8192) >> 14];
      const uint32_t L8 =
          clamp_u8(nearest_div(255 * (116 * (int64_t)fy - 16 * 65535), 100 * 65535));
      const uint32_t a8 = clamp_u8(128 + nearest_div(500 * (int64_t)(fx - fy), 65535));
      const uint32_t b8 = clamp_u8(128 + nearest_div(200 * (int64_t)(fy - fz), 65535));
      word |= L8 | (a8 << 8) | (b8 << 16);
    }
    out[(size_t)v * W + (mirror ? W - 1 - u : u)] = word;
  }
}

__global__ __launch_bounds__(kColorThreads) void k_color(const uint8_t *__restrict__ img, int W,
                                                         int H, int stride,
                                                         uint32_t *__restrict__ out,
                                                         const uint16_t *__restrict__ lin,
                                                         const uint16_t *__restrict__ ftab, Mq mq,
                                                         int want_lab, int mirror) {
  color_tile<kColorRPT>(img, W, H, stride, out, lin, ftab, mq, want_lab, mirror,
                        blockIdx.x * kColorTX, blockIdx.y * kColorTY);
}

// Reverses every row of a [rows][W] array in place (maps results of the
// mirrored frame back to image columns).
template <typename T>
__global__ __launch_bounds__(256) void k_reverse_rows(T *__restrict__ data, int W, int rows) {
  const int u = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y + blockIdx.z * 65535;
  if (r >= rows || u >= W / 2) return;
  T *row = data + (size_t)r * W;
  const T a = row[u], b = row[W - 1 - u];
  row[u] = b;
  row[W - 1 - u] = a;
}

// Left/right consistency check of two disparity maps (the first part of the
// refinement step of Section 3): dL where |dL(u) - dR(u - dL(u))| <= tol,
// else -1.
__global__ __launch_bounds__(256) void k_lr_check(const int32_t *__restrict__ dL,
                                                  const int32_t *__restrict__ dR, int W, int H,
                                                  int tol, int32_t *__restrict__ out) {
  const int u = blockIdx.x * 256 + threadIdx.x, v = blockIdx.y;
  if (u >= W || v >= H) return;
  const size_t row = (size_t)v * W;
  const int d = dL[row + u];
  bool ok = false;
  if (d >= 0 && u - d >= 0) {
    const int e = d - dR[row + u - d];
    ok = (e < 0 ? -e : e) <= tol;
  }
  out[row + u] = ok ? d : -1;
}

// ===========================================================================
// Descriptor + mask (reference view).  A block stages a TH x TW tile of
// packed pixels plus a halo of `radius` in LDS (coordinates clamped to the
// image, which is exactly the border rule).  Each wave walks its pixels one
// at a time with the 64 lanes spread over the point pairs and every pair
// weight kept in registers.  T, the k-th smallest weight, is the smallest t
// with #{w <= t} >= k: a counting search on the vector unit (see
// kth_smallest) that starts from the wave's previous pixel's T, since
// neighbouring pixels have close thresholds.
//
// Pair-to-lane maps (NW = nw rounded up to a power of two, padded pairs
// compare the centre with itself: weight 0, and each shifts the rank of T
// by one):
//   NW >= 8  lane l owns pairs NW l .. NW l + NW - 1, so its binary tests
//            are NW consecutive bits of the descriptor (and of the mask):
//            the lane shifts them into a register and stores its NW / 8
//            bytes itself; the wave's stores cover the pixel's words.
//   NW <= 4  lane l of word j owns pair 64 j + l, so the ballot of the
//            wave's tests IS word j, moved into lane j with v_writelane.
// ===========================================================================
// Tile height (rows) of the describe+mask tiles: eight rows when the image
// has tiles enough to fill the GPU about once (fewer halo rows per output
// row), four rows otherwise (twice the tiles, shorter tails).  The
// persistent batch kernel takes the height its tuning names (8 or 16 rows).
constexpr int kDescTH = 8, kDescTHSmall = 4, kDescThreads = 256;
constexpr long long kDescTallMinTiles = 1024;  // one round of the GPU at four blocks per CU

// Pair index of slot j of lane `lane` (0-based).
template <int NW>
__device__ __forceinline__ int pair_of(int lane, int j) {
  return NW >= 8 ? NW * lane + j : 64 * j + lane;
}

// v_writelane_b32 through the LLVM intrinsic (this clang has no builtin for
// it), so that the compiler's hazard handling sees it: an SGPR written by a
// VALU compare must not be read by v_writelane in the very next cycles.
__device__ int writelane_i32(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Puts the wave-uniform 64-bit value `bits` into lane J of (lo, hi).
template <int J>
__device__ __forceinline__ void put_word(uint64_t bits, uint32_t &lo, uint32_t &hi) {
  lo = static_cast<uint32_t>(writelane_i32(static_cast<int>(static_cast<uint32_t>(bits)), J,
                                           static_cast<int>(lo)));
  hi = static_cast<uint32_t>(writelane_i32(static_cast<int>(static_cast<uint32_t>(bits >> 32)), J,
                                           static_cast<int>(hi)));
}

// Applies f<J>() for J = 0 .. N-1 (compile-time lane indices).
template <int N, int J = 0, typename F>
__device__ __forceinline__ void for_words(F &&f) {
  if constexpr (J < N) {
    f(std::integral_constant<int, J>{});
    for_words<N, J + 1>(f);
  }
}

// ---- T, the k-th smallest weight (Eq. 6), by a counting search ----------
// Weights lie in [0, 765] (three byte differences) and sit two per dword in
// 16-bit halves; a half that holds no weight holds 0x7fff.  The rank of a
// threshold t, #{w <= t}, is counted on the vector unit: w - (t + 1) is
// negative exactly when w <= t, v_perm_b32 turns the sign bits of four
// halves into four bytes of 0x00 / 0xff and v_bcnt_u32_b32 adds 8 per set
// sign.  A wave reduction with DPP row shifts and row broadcasts sums the
// lanes' counts.  The search keeps a bracket lo < T <= hi with known ranks
// (rank(lo) < k <= rank(hi)); the next probe is the secant through the
// bracket once both ends have been probed, and before that a step of
// (k - rank) / density from the last probe.  The density (weights per unit
// of t near T) is a running average over the wave's previous pixels, taken
// from their first two probes.  The first probe is the previous pixel's T.
// The steps are scalar integer arithmetic: a division by d <= 4096 is a
// multiply-high by floor((2^32 - 1) / d) from a constant table.
constexpr int kTop = 765;  // largest weight: rank(765) counts every weight

// The state carried from one pixel to the next by a wave.
struct SearchHint {
  int t;      // previous pixel's T
  int dens4;  // 4 x the running average of the rank density near T, 1..4096
};

// floor((2^32 - 1) / d) for d = 1 .. 4096 (entry 0 unused).
struct RecipTable {
  uint32_t v[4097];
  constexpr RecipTable() : v() {
    v[0] = 0xffffffffu;
    for (int d = 1; d <= 4096; ++d) v[d] = static_cast<uint32_t>(0xffffffffull / d);
  }
};
__constant__ RecipTable kRecip = RecipTable{};

// About num / den rounded up (within one) for 1 <= den <= 4096 and
// num < 2^24; wave-uniform.  kShortChain: from v_rcp_f32 instead of the
// table, for kernels too short to hide a scalar load per probe (few
// weights a lane: few waves, few probes' worth of work between loads).
template <bool kShortChain>
__device__ __forceinline__ int div_up(uint32_t num, int den) {
  if constexpr (kShortChain)
    return __builtin_amdgcn_readfirstlane(static_cast<int>(
               static_cast<float>(num) * __builtin_amdgcn_rcpf(static_cast<float>(den)))) +
           1;
  else
    return static_cast<int>(__umulhi(num, kRecip.v[den])) + 1;
}

// Packs two weights (each <= 765) into the 16-bit halves of a dword.
__device__ __forceinline__ uint32_t pack_halves(uint32_t lo, uint32_t hi) {
  return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// Halves of a minus halves of b, each mod 2^16 (v_pk_sub_u16).
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t b) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}

// 8 * #{weights of this lane <= t}; t1x2 holds t + 1 in both halves.
template <int NP>
__device__ __forceinline__ uint32_t lane_rank8(const uint32_t *P, uint32_t t1x2) {
  uint32_t c = 0;
#pragma unroll
  for (int m = 0; m + 1 < NP; m += 2) {
    // bytes 0-3: signs of P[m + 1].lo, P[m + 1].hi, P[m].lo, P[m].hi
    const uint32_t z = __builtin_amdgcn_perm(pk_sub16(P[m], t1x2), pk_sub16(P[m + 1], t1x2),
                                             0x0b0a0908u);
    c = __builtin_popcount(z) + c;
  }
  if constexpr (NP & 1) {
    const uint32_t z = __builtin_amdgcn_perm(0u, pk_sub16(P[NP - 1], t1x2), 0x0c0c0908u);
    c = __builtin_popcount(z) + c;
  }
  return c;
}

// Sum of v over the wave's 64 lanes (wave-uniform result).
__device__ __forceinline__ int wave_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// #{w <= t} over the wave's packed weights (t wave-uniform, 0 <= t < 765).
// With at most four weights a lane (n <= 256) ballots and scalar popcounts
// make the shorter chain; with more, the vector count and DPP sum.
template <int NP>
__device__ __forceinline__ int wave_rank(const uint32_t *P, int t) {
  if constexpr (NP <= 2) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      c += __popcll(__ballot((P[q] & 0xffffu) <= static_cast<uint32_t>(t)));
      c += __popcll(__ballot((P[q] >> 16) <= static_cast<uint32_t>(t)));
    }
    return c;
  } else {
    const uint32_t t1 = static_cast<uint32_t>(t + 1);
    return wave_sum(static_cast<int>(lane_rank8<NP>(P, t1 | (t1 << 16)))) >> 3;
  }
}

// A probe of the search: the bracket lo < T <= hi with rank(lo) < k <=
// rank(hi) takes in (t, rank(t)).
struct Bracket {
  int lo, hi, rlo, rhi;
  __device__ __forceinline__ void take(int t, int r, int k) {
    const bool reached = r >= k;
    hi = reached ? t : hi;
    rhi = reached ? r : rhi;
    lo = reached ? lo : t;
    rlo = reached ? rlo : r;
  }
  __device__ __forceinline__ bool open() const { return hi - lo > 1; }
};

// The next probe after (t, r): the secant through the bracket when both of
// its ends have been probed, else a step of (k - r) / density from t (at
// least one), clamped inside the bracket.
template <bool kShortChain>
__device__ __forceinline__ int next_probe(const Bracket &b, int t, int r, int k, int dens4) {
  const bool secant = b.lo >= 0 && b.hi < kTop;
  const bool down = !secant && r >= k;
  const int base = secant ? b.lo : t;
  const uint32_t num = secant ? static_cast<uint32_t>((k - b.rlo) * (b.hi - b.lo))
                              : 4u * static_cast<uint32_t>(down ? r - k : k - r);
  const int step = div_up<kShortChain>(num, secant ? b.rhi - b.rlo : dens4);
  const int next = down ? base - step : base + step;
  return min(max(next, b.lo + 1), b.hi - 1);
}

// The k-th smallest of the wave's weights (nwts of them), searched from the
// hint, which is updated for the next pixel.
// The same search for lanes with at most four weights (n <= 256), where a
// probe is a few ballots: galloping from the hint in steps of 8, 16, ...
// until T is bracketed, then bisection.  Each step is one scalar add, which
// beats the secant's longer chain of scalar and vector work per probe when
// the kernel has few waves to overlap.
template <int NP>
__device__ __forceinline__ int kth_smallest_gallop(const uint32_t *P, int k, SearchHint &h) {
  int lo, hi;  // rank not reached at lo, reached at hi
  const int g = min(max(h.t, 0), kTop - 1);
  if (wave_rank<NP>(P, g) >= k) {
    hi = g;
    for (int step = 8;; step <<= 1) {
      const int t = hi - step;
      if (t < 0) {
        lo = -1;
        break;
      }
      if (wave_rank<NP>(P, t) < k) {
        lo = t;
        break;
      }
      hi = t;
    }
  } else {
    lo = g;
    for (int step = 8;; step <<= 1) {
      const int t = lo + step;
      if (t >= kTop) {
        hi = kTop;
        break;
      }
      if (wave_rank<NP>(P, t) >= k) {
        hi = t;
        break;
      }
      lo = t;
    }
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (wave_rank<NP>(P, mid) >= k)
      hi = mid;
    else
      lo = mid;
  }
  h.t = hi;
  return hi;
}

template <int NP>
__device__ __forceinline__ int kth_smallest(const uint32_t *P, int k, int nwts, SearchHint &h) {
  if constexpr (NP <= 2) return kth_smallest_gallop<NP>(P, k, h);
  constexpr bool kShort = false;
  Bracket b{-1, kTop, 0, nwts};
  const int t0 = min(max(h.t, 0), kTop - 1);
  const int r0 = wave_rank<NP>(P, t0);
  b.take(t0, r0, k);
  if (b.open()) {
    const int t1 = next_probe<kShort>(b, t0, r0, k, h.dens4);
    const int r1 = wave_rank<NP>(P, t1);
    b.take(t1, r1, k);
    // 4 x the rank density between the first two probes, averaged over pixels
    const int dt = t1 > t0 ? t1 - t0 : t0 - t1;
    const int d4 = div_up<kShort>(4u * static_cast<uint32_t>(r1 > r0 ? r1 - r0 : r0 - r1), dt);
    h.dens4 = min((3 * h.dens4 + d4) >> 2, 4096);
    int t = t1, r = r1;
    while (b.open()) {
      t = next_probe<kShort>(b, t, r, k, h.dens4);
      r = wave_rank<NP>(P, t);
      b.take(t, r, k);
    }
  }
  h.t = b.hi;
  return b.hi;
}

// Pair weights of Eq. 5: max of the CIELAB SADs of the two samples to the
// centre.  Packed pixels hold L8, a8, b8 in bytes 0-2 and I in byte 3.
// v_msad_u8 leaves out the bytes where its second operand is 0, so with the
// centre's byte 3 cleared it sums exactly the three colour differences, as
// long as none of the centre's colour bytes is 0; otherwise the samples'
// byte 3 is masked off first.  `centre` is wave-uniform.
template <int NW>
__device__ __forceinline__ void pair_weights(const uint32_t *a, const uint32_t *b,
                                             uint32_t centre, uint32_t *w) {
  const uint32_t c = centre & 0xffffffu;
  const bool colour_nonzero = (c & 0xffu) && (c & 0xff00u) && (c & 0xff0000u);
  if (colour_nonzero) {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const uint32_t sp = __builtin_amdgcn_msad_u8(a[j], c, 0u);
      const uint32_t sq = __builtin_amdgcn_msad_u8(b[j], c, 0u);
      w[j] = sp > sq ? sp : sq;
    }
  } else {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const uint32_t sp = __builtin_amdgcn_sad_u8(a[j] & 0xffffffu, c, 0u);
      const uint32_t sq = __builtin_amdgcn_sad_u8(b[j] & 0xffffffu, c, 0u);
      w[j] = sp > sq ? sp : sq;
    }
  }
}

// The lane's NW pair weights (Eq. 5), two per dword (P[q] holds pairs 2q in
// the low half and 2q + 1 in the high half; a lone last pair has 0x7fff
// beside it, which no threshold counts).
template <int NW>
__device__ __forceinline__ void packed_weights(const uint32_t *a, const uint32_t *b,
                                               uint32_t centre, uint32_t *P) {
  uint32_t w[NW];
  pair_weights<NW>(a, b, centre, w);
#pragma unroll
  for (int q = 0; q < NW / 2; ++q) P[q] = pack_halves(w[2 * q], w[2 * q + 1]);
  if constexpr (NW & 1) P[NW / 2] = pack_halves(w[NW - 1], 0x7fffu);
}

// The lane's mask bits (Eq. 6-7) for NW >= 8 pairs packed two per dword in
// P: bit j of m[j / 32] is [w_j <= T], t1 = T + 1.  Eight pairs at a time:
// the signs of their halves of P - t1 become bytes of 0x00 / 0xff
// (v_perm_b32 sign selectors, four pairs per dword), a mask keeps 2^i in
// the byte of pair i of the eight, and v_sad_u8 adds the bytes up on top of
// the register's higher groups shifted up by eight bits.
template <int NW>
__device__ __forceinline__ void mask_bits(const uint32_t *P, uint32_t t1, uint32_t *m) {
  static_assert(NW % 8 == 0, "whole groups of eight pairs");
  const uint32_t t1x2 = t1 | (t1 << 16);
  constexpr int kRegs = (NW + 31) / 32;
#pragma unroll
  for (int r = 0; r < kRegs; ++r) {
    constexpr int kGroups = NW / 8 < 4 ? NW / 8 : 4;  // groups of eight in a register
    uint32_t acc = 0;
#pragma unroll
    for (int g = kGroups - 1; g >= 0; --g) {
      const int q = 16 * r + 4 * g;  // dwords q .. q + 3 hold pairs 2q .. 2q + 7
      // bytes 0-3: signs of P[q].lo, P[q].hi, P[q + 1].lo, P[q + 1].hi
      const uint32_t lo = __builtin_amdgcn_perm(pk_sub16(P[q + 1], t1x2), pk_sub16(P[q], t1x2),
                                                0x0b0a0908u) & 0x08040201u;
      const uint32_t hi = __builtin_amdgcn_perm(pk_sub16(P[q + 3], t1x2),
                                                pk_sub16(P[q + 2], t1x2), 0x0b0a0908u) &
                          0x80402010u;
      acc = __builtin_amdgcn_sad_u8(hi, 0u, __builtin_amdgcn_sad_u8(lo, 0u, acc << 8));
    }
    m[r] = acc;
  }
}

// Stores a lane's NW consecutive bits (NW >= 8) at byte NW / 8 * lane of
// the pixel's words.
template <int NW>
__device__ __forceinline__ void store_lane_bits(uint64_t *out, int lane, const uint32_t *bits) {
  if constexpr (NW == 8) {
    reinterpret_cast<uint8_t *>(out)[lane] = static_cast<uint8_t>(bits[0]);
  } else if constexpr (NW == 16) {
    reinterpret_cast<uint16_t *>(out)[lane] = static_cast<uint16_t>(bits[0]);
  } else if constexpr (NW == 32) {
    reinterpret_cast<uint32_t *>(out)[lane] = bits[0];
  } else {
    static_assert(NW == 64, "lane-major descriptors need NW in {8, 16, 32, 64}");
    reinterpret_cast<uint2 *>(out)[lane] = make_uint2(bits[0], bits[1]);
  }
}

// One pixel of the descriptor and mask.  ap/aq: LDS byte addresses of this
// lane's samples for the group's first pixel; `shift` (bytes, compile-time
// after unrolling) moves them to this pixel through the instruction's
// immediate offset.  out: this pixel's words in desc / mask.
template <int NW>
__device__ __forceinline__ void describe_pixel(const char *lds, const int *ap, const int *aq,
                                              int centre_addr, int shift, int lane, int n,
                                              int k_eff, SearchHint &hint,
                                              uint64_t *out_desc, uint64_t *out_mask) {
  uint32_t a[NW], b[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    a[j] = *reinterpret_cast<const uint32_t *>(lds + ap[j] + shift);
    b[j] = *reinterpret_cast<const uint32_t *>(lds + aq[j] + shift);
  }
  const uint32_t centre = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(
      *reinterpret_cast<const int *>(lds + centre_addr)));
  if constexpr (NW >= 8) {
    // tau of Eq. 3 and delta of Eq. 6, slot j -> bit j of the lane's chunk.
    // Each test is the sign of a difference, shifted in by v_alignbit:
    // I(q) - I(p) < 0 exactly when tau = 1, w - T - 1 < 0 exactly when
    // delta = 1 (both differences are small, so nothing wraps).  The
    // descriptor bits are taken first so that the samples are dead during
    // the threshold search.
    constexpr int kRegs = (NW + 31) / 32;
    uint32_t d[kRegs], m[kRegs];
#pragma unroll
    for (int r = 0; r < kRegs; ++r) d[r] = m[r] = 0;
#pragma unroll
    for (int j = NW - 1; j >= 0; --j)
      d[j / 32] = __builtin_amdgcn_alignbit(d[j / 32], (b[j] >> 24) - (a[j] >> 24), 31);
    // Keep the descriptor bits here: otherwise the compiler computes them at
    // the store, after the search, and the samples stay live through it.
#pragma unroll
    for (int r = 0; r < kRegs; ++r) asm volatile("" : "+v"(d[r]));
    uint32_t P[NW / 2];
    packed_weights<NW>(a, b, centre, P);
    const uint32_t t1 = static_cast<uint32_t>(kth_smallest<NW / 2>(P, k_eff, 64 * NW, hint) + 1);
    mask_bits<NW>(P, t1, m);
    if (NW * lane < n) {
      store_lane_bits<NW>(out_desc, lane, d);
      store_lane_bits<NW>(out_mask, lane, m);
    }
  } else {
    uint32_t d_lo = 0, d_hi = 0, m_lo = 0, m_hi = 0;
    for_words<NW>([&](auto J) {  // Eq. 3
      put_word<J.value>(__ballot((a[J.value] >> 24) > (b[J.value] >> 24)), d_lo, d_hi);
    });
    constexpr int NP = (NW + 1) / 2;
    uint32_t P[NP];
    packed_weights<NW>(a, b, centre, P);
    const uint32_t T = static_cast<uint32_t>(kth_smallest<NP>(P, k_eff, 64 * NW, hint));
    for_words<NW>([&](auto J) {  // Eq. 6-7
      const uint32_t wj = (J.value & 1) ? P[J.value / 2] >> 16 : P[J.value / 2] & 0xffffu;
      put_word<J.value>(__ballot(wj <= T), m_lo, m_hi);
    });
    if (lane < n / 64) {
      out_desc[lane] = (static_cast<uint64_t>(d_hi) << 32) | d_lo;
      out_mask[lane] = (static_cast<uint64_t>(m_hi) << 32) | m_lo;
    }
  }
}

// Parameters of the describe kernels that are fixed per context.
struct DescribeConsts {
  const int8_t *pattern;  // [n][4]
  int nw, radius, pitch, k;
  int table_off;  // single-pair kernel: LDS byte offset of the pair-offset table
};

// The pair-offset table in LDS: for lane l and slot j, the byte offsets in
// the tile, relative to the centre, of the pair's two samples (0 for padded
// pairs), as int2 at ((j / 2) * 64 + l) * 2 + j % 2, so that a lane reads two
// slots with one 16-byte load and the 64 lanes read 1 KB without bank
// conflicts.  The offsets depend only on the lane and the tile pitch: one
// wave writes the table once per launch and every wave of the workgroup
// reads it, which keeps them out of the registers.
template <int NW>
__host__ __device__ constexpr int pair_table_bytes() {
  return NW >= 32 ? (NW / 4) * 64 * 16 : ((NW + 1) / 2) * 64 * 16;
}

template <int NW>
__device__ __forceinline__ void write_pair_table(const DescribeConsts &c, int2 *tab) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x, n = 64 * c.nw;
  const int32_t *pat32 = reinterpret_cast<const int32_t *>(c.pattern);
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int i = pair_of<NW>(lane, j);
    const int32_t e = i < n ? pat32[i] : 0;
    const int px = (int8_t)(e & 0xff), py = (int8_t)((e >> 8) & 0xff);
    const int qx = (int8_t)((e >> 16) & 0xff), qy = (int8_t)((e >> 24) & 0xff);
    tab[((j >> 1) * 64 + lane) * 2 + (j & 1)] =
        make_int2(4 * (py * c.pitch + px), 4 * (qy * c.pitch + qx));
  }
}

// Where a wave finds its lanes' pair offsets: TableOffsets reads the LDS
// table per group of pixels (registers free for a fifth wave per SIMD);
// RegOffsets holds them in 2 NW registers (no LDS load before the gathers,
// which matters where descriptor-only tiles keep the LDS busy).
template <int NW>
struct TableOffsets {
  const int2 *tab;
  // ap[j] / aq[j] = c0 + the offsets of slot j for this lane
  __device__ __forceinline__ void addresses(int c0, int lane, int *ap, int *aq) const {
    if constexpr (NW == 1) {
      const int2 e = tab[2 * lane];
      ap[0] = c0 + e.x;
      aq[0] = c0 + e.y;
    } else {
#pragma unroll
      for (int j = 0; j < NW; j += 2) {
        const int4 e = *reinterpret_cast<const int4 *>(tab + ((j >> 1) * 64 + lane) * 2);
        ap[j] = c0 + e.x;
        aq[j] = c0 + e.y;
        ap[j + 1] = c0 + e.z;
        aq[j + 1] = c0 + e.w;
      }
    }
  }
};

template <int NW>
struct RegOffsets {
  int p[NW], q[NW];
  __device__ __forceinline__ RegOffsets(const DescribeConsts &c, int lane) {
    const int n = 64 * c.nw;
    const int32_t *pat32 = reinterpret_cast<const int32_t *>(c.pattern);
    // (loads without a branch, so that all of them are in flight at once)
    int32_t pe[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) pe[j] = pat32[min(pair_of<NW>(lane, j), n - 1)];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int32_t e = pair_of<NW>(lane, j) < n ? pe[j] : 0;
      const int px = (int8_t)(e & 0xff), py = (int8_t)((e >> 8) & 0xff);
      const int qx = (int8_t)((e >> 16) & 0xff), qy = (int8_t)((e >> 24) & 0xff);
      p[j] = 4 * (py * c.pitch + px);
      q[j] = 4 * (qy * c.pitch + qx);
    }
  }
  __device__ __forceinline__ void addresses(int c0, int, int *ap, int *aq) const {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      ap[j] = c0 + p[j];
      aq[j] = c0 + q[j];
    }
  }
};

// For NW >= 32 (n >= 2048) the offsets are 16-bit halves of one dword per
// slot, p low and q high (|offset| < 2^15 for any window and tile pitch),
// at (j / 4) * 64 + l in dwords of four: a lane reads four slots with one
// 16-byte load.  Wide pixels take their slots in chunks of 16 and read each
// chunk's offsets as they go, so no group of addresses stays in registers.
template <int NW>
__device__ __forceinline__ void write_pair_table16(const DescribeConsts &c, uint32_t *tab) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x, n = 64 * c.nw;
  const int32_t *pat32 = reinterpret_cast<const int32_t *>(c.pattern);
#pragma unroll 4
  for (int j = 0; j < NW; ++j) {
    const int i = pair_of<NW>(lane, j);
    const int32_t e = i < n ? pat32[i] : 0;
    const int px = (int8_t)(e & 0xff), py = (int8_t)((e >> 8) & 0xff);
    const int qx = (int8_t)((e >> 16) & 0xff), qy = (int8_t)((e >> 24) & 0xff);
    const int op = 4 * (py * c.pitch + px), oq = 4 * (qy * c.pitch + qx);
    tab[((j >> 2) * 64 + lane) * 4 + (j & 3)] =
        (static_cast<uint32_t>(op) & 0xffffu) | (static_cast<uint32_t>(oq) << 16);
  }
}

template <int NW>
struct WideOffsets {
  const uint32_t *tab;
  // ap[j] / aq[j] = c0 + the offsets of slot 16 ch + j, j < 16
  __device__ __forceinline__ void chunk(int c0, int lane, int ch, int *ap, int *aq) const {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 e = *reinterpret_cast<const uint4 *>(tab + ((4 * ch + k) * 64 + lane) * 4);
      const uint32_t v[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ap[4 * k + i] = c0 + (static_cast<int>(v[i] << 16) >> 16);
        aq[4 * k + i] = c0 + (static_cast<int>(v[i]) >> 16);
      }
    }
  }
};

// One pixel of the descriptor and mask for NW >= 32, the slots in chunks of
// 16: the chunk's offsets, samples, descriptor bits and packed weights, then
// the next chunk, so that only one chunk's samples and addresses are live.
// Chunks go from the last so that the descriptor bits shift in from slot
// NW - 1 down to 0, as in describe_pixel.
template <int NW>
__device__ __forceinline__ void describe_pixel_wide(const char *lds, const WideOffsets<NW> &off,
                                                    int centre_addr, int lane, int n, int k_eff,
                                                    SearchHint &hint, uint64_t *out_desc,
                                                    uint64_t *out_mask) {
  static_assert(NW >= 32, "wide pixels have whole 32-bit descriptor registers");
  constexpr int kChunk = 16, kRegs = NW / 32;
  const uint32_t centre = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(
      *reinterpret_cast<const int *>(lds + centre_addr)));
  uint32_t d[kRegs], m[kRegs];
#pragma unroll
  for (int r = 0; r < kRegs; ++r) d[r] = m[r] = 0;
  uint32_t P[NW / 2];
#pragma unroll
  for (int ch = NW / kChunk - 1; ch >= 0; --ch) {
    int ap[kChunk], aq[kChunk];
    off.chunk(centre_addr, lane, ch, ap, aq);
    uint32_t a[kChunk], b[kChunk];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      a[j] = *reinterpret_cast<const uint32_t *>(lds + ap[j]);
      b[j] = *reinterpret_cast<const uint32_t *>(lds + aq[j]);
    }
#pragma unroll
    for (int j = kChunk - 1; j >= 0; --j) {
      const int slot = kChunk * ch + j;
      d[slot / 32] = __builtin_amdgcn_alignbit(d[slot / 32], (b[j] >> 24) - (a[j] >> 24), 31);
    }
    packed_weights<kChunk>(a, b, centre, P + (kChunk / 2) * ch);
    // Finish the chunk here: sunk to their uses (the search, the stores),
    // its descriptor bits and packing would keep every chunk's samples and
    // weights live at once.
#pragma unroll
    for (int q = 0; q < kChunk / 2; ++q) asm volatile("" : "+v"(P[(kChunk / 2) * ch + q]));
#pragma unroll
    for (int r = 0; r < kRegs; ++r) asm volatile("" : "+v"(d[r]));
  }
  const uint32_t t1 = static_cast<uint32_t>(kth_smallest<NW / 2>(P, k_eff, 64 * NW, hint) + 1);
  mask_bits<NW>(P, t1, m);
  if (NW * lane < n) {
    store_lane_bits<NW>(out_desc, lane, d);
    store_lane_bits<NW>(out_mask, lane, m);
  }
}

// Rows of the tile go to the waves either fixed (TH / 4 consecutive rows
// each) or, with PULL_ROWS, one at a time from the LDS counter *row_next as
// the waves become free: a wave whose pixels needed fewer search probes then
// takes another row instead of waiting at the next barrier of a persistent
// kernel for the others.
template <int NW, int TW, int TH, bool PULL_ROWS, typename Offsets>
__device__ __forceinline__ void describe_mask_tile(uint32_t *tile, int *row_next,
                                                   const uint32_t *__restrict__ packed, int W,
                                                   int H, const DescribeConsts &c,
                                                   const Offsets &off,
                                                   uint64_t *__restrict__ desc,
                                                   uint64_t *__restrict__ mask, int u0, int v0) {
  const int radius = c.radius, pitch = c.pitch, nw = c.nw, n = 64 * nw;
  const int rows = TH + 2 * radius, cols = TW + 2 * radius;
  const int total = rows * cols;
  __syncthreads();  // the previous tile (persistent kernels) is done with LDS
  // Stage the tile with kBatch independent loads in flight per thread.
  constexpr int kBatch = 8;
  for (int first = threadIdx.x; first < total; first += kDescThreads * kBatch) {
    uint32_t staged[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int i = first + b * kDescThreads;
      staged[b] = 0;
      if (i < total) {
        const int ty = i / cols, tx = i - ty * cols;
        const int gv = min(max(v0 - radius + ty, 0), H - 1);
        const int gu = min(max(u0 - radius + tx, 0), W - 1);
        staged[b] = packed[(size_t)gv * W + gu];
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int i = first + b * kDescThreads;
      if (i < total) {
        const int ty = i / cols, tx = i - ty * cols;
        tile[ty * pitch + tx] = staged[b];
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int k_eff = c.k + (64 * NW - n);
  if (PULL_ROWS && threadIdx.x == 0) *row_next = 0;
  __syncthreads();

  const char *lds = reinterpret_cast<const char *>(tile);
  constexpr int kRowsPerWave = TH / (kDescThreads / 64);
  constexpr int kGroup = 4;  // pixels whose LDS addresses share one base
  SearchHint hint{64, NW * 2};  // the first pixel starts at t = 64, density n / 128
  for (int r = 0;; ++r) {
    int ty;
    if constexpr (PULL_ROWS) {
      int pulled = 0;
      if (lane == 0) pulled = atomicAdd(row_next, 1);
      ty = __builtin_amdgcn_readfirstlane(pulled);
      if (ty >= TH) break;  // uniform
    } else {
      if (r == kRowsPerWave) break;
      ty = wave * kRowsPerWave + r;
    }
    const int v = v0 + ty;
    if (v >= H) break;  // uniform
    // the row's first word, from scalar registers (v W < 2^31)
    const size_t row_words = static_cast<size_t>(uniform(v * W)) * static_cast<size_t>(nw);
    if constexpr (NW >= 32) {
      for (int g = 0; g < TW; ++g) {
        const int u = u0 + g;
        if (u >= W) break;  // uniform
        describe_pixel_wide<NW>(lds, off, 4 * ((ty + radius) * pitch + (g + radius)), lane, n,
                                k_eff, hint, uniform(desc + row_words + uniform(u * nw)),
                                uniform(mask + row_words + uniform(u * nw)));
      }
    } else {
      for (int g = 0; g < TW; g += kGroup) {
        if (u0 + g >= W) break;  // uniform
        const int c0 = 4 * ((ty + radius) * pitch + (g + radius));
        int ap[NW], aq[NW];
        off.addresses(c0, lane, ap, aq);
#pragma unroll
        for (int t = 0; t < kGroup; ++t) {
          const int u = u0 + g + t;
          if (u >= W) break;  // uniform
          // the words' addresses on the scalar unit (used only under the
          // lanes' store condition, they would be computed per lane there)
          describe_pixel<NW>(lds, ap, aq, c0 + 4 * t, 4 * t, lane, n, k_eff, hint,
                             uniform(desc + row_words + uniform(u * nw)),
                             uniform(mask + row_words + uniform(u * nw)));
        }
      }
    }
  }
}

template <int NW, int TW, int TH>
__global__ __launch_bounds__(kDescThreads) void k_describe_mask(
    const uint32_t *__restrict__ packed, int W, int H, DescribeConsts c,
    uint64_t *__restrict__ desc, uint64_t *__restrict__ mask) {
  extern __shared__ uint32_t tile[];
  if constexpr (NW >= 32) {
    uint32_t *tab = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(tile) + c.table_off);
    write_pair_table16<NW>(c, tab);  // the tile function's first barrier publishes it
    describe_mask_tile<NW, TW, TH, false>(tile, nullptr, packed, W, H, c, WideOffsets<NW>{tab},
                                          desc, mask, blockIdx.x * TW, blockIdx.y * TH);
  } else if constexpr (NW >= 16) {
    // 4 NW offset registers would cap the kernel at four waves per SIMD
    int2 *tab = reinterpret_cast<int2 *>(reinterpret_cast<char *>(tile) + c.table_off);
    write_pair_table<NW>(c, tab);  // the tile function's first barrier publishes it
    describe_mask_tile<NW, TW, TH, false>(tile, nullptr, packed, W, H, c, TableOffsets<NW>{tab},
                                          desc, mask, blockIdx.x * TW, blockIdx.y * TH);
  } else {
    // few offsets: in registers, so that no LDS load precedes the gathers
    describe_mask_tile<NW, TW, TH, false>(tile, nullptr, packed, W, H, c,
                                          RegOffsets<NW>(c, threadIdx.x & 63), desc, mask,
                                          blockIdx.x * TW, blockIdx.y * TH);
  }
}

// ===========================================================================
// Descriptor only (the non-reference view).  One wave per row of a tile of
// 64 PX pixels; lane l owns the PX adjacent pixels PX l .. PX l + PX - 1 and
// the point pairs are walked in a uniform loop.  The intensity tile sits in
// LDS one byte per pixel, its interior starting on a 4-byte boundary and
// its pitch a multiple of 4, so for pair i the PX samples x + p_i of a
// lane's pixels are PX consecutive bytes at the same alignment in every
// lane: (PX = 4) two aligned dword reads and one v_alignbyte (shift = the
// offset's low two bits, wave-uniform) fetch all four.  The pair offsets
// (bytes in the tile) are wave-uniform and come through scalar loads.  Each
// pixel's binary tests go bit by bit into its own registers with
// v_alignbit, most significant pair first, so pair 64 j + 32 h + b ends at
// bit b of half h of word j.  With one pixel per lane the words are
// produced 16 at a time (128 bytes of the pixel's string) and stored
// straight from registers; with four pixels per lane (which would need 128
// registers for that) every two finished words are staged in LDS as
// [word][pixel] and written out pixel by pixel as 16-byte chunks.
// ===========================================================================
constexpr int kRightPx = 4;                         // pixels per lane (wide tiles)
constexpr int kRightTW = 64 * kRightPx, kRightTH = 4, kRightThreads = 256;
constexpr int kRightGroup = 16;                     // words per pass (one pixel per lane)
constexpr int kDescRightEvery = 4;  // batch: one describe workgroup in this many starts right
constexpr int kRightStageWords = 2;                 // words per LDS stage (four per lane)
constexpr int kRightRegWords = 8;  // words per pass in registers (four per lane, nw % 8 == 0)
// Images with fewer wide tiles than this run one pixel per lane (64-pixel
// tiles), which gives four times as many workgroups.
constexpr int kRightWideMinBlocks = 1024;

__host__ __device__ constexpr int right_halo(int radius) { return (radius + 3) / 4 * 4; }

// LDS bytes of the describe-only kernels with PX pixels per lane: the
// output staging (four pixels per lane only), then the intensity tile
// (pitch bytes per row).
__host__ __device__ constexpr size_t right_stage_bytes(int px) {
  return px == 1 ? 0 : (size_t)(kRightThreads / 64) * kRightStageWords * 64 * px * sizeof(uint64_t);
}
__host__ __device__ constexpr size_t right_lds_bytes(int px, int radius, int pitch) {
  return right_stage_bytes(px) + (size_t)(kRightTH + 2 * radius) * pitch;
}

struct RightConsts {
  const int2 *offs;  // [n] (p, q) byte offsets in the intensity tile
  int n, nw, radius, pitch;
};

// Bytes x + 0 .. x + PX - 1 of the tile at byte address a + o, where a is a
// multiple of 4: for PX = 4 two aligned dwords and a funnel shift by
// o mod 4, for PX = 1 one byte.
template <int PX>
__device__ __forceinline__ uint32_t tile_bytes(const uint8_t *tile, int a, int o) {
  if constexpr (PX == 1) {
    return tile[a + o];
  } else {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(tile + a + (o & ~3));
    return __builtin_amdgcn_alignbyte(w[1], w[0], static_cast<uint32_t>(o & 3));
  }
}

// An int2 table read through the constant address space: the table is
// never written while a kernel runs and its indices are wave-uniform, so
// every read is a scalar load, also where descriptor stores share the loop.
struct ConstInt2Table {
  const int2 *p;
  __device__ __forceinline__ int2 operator[](int i) const {
    const __attribute__((address_space(4))) long long *q =
        (const __attribute__((address_space(4))) long long *)p;
    const long long v = q[i];
    return make_int2(static_cast<int>(v), static_cast<int>(v >> 32));
  }
};

// Bytes x + 0 .. x + 3 for the lane whose first pixel sits at the 4-byte
// aligned LDS address lp, at tile offset o: two dwords and a funnel shift.
__device__ __forceinline__ uint32_t lane_bytes4(const uint8_t *lp, int o) {
  const uint32_t *w = reinterpret_cast<const uint32_t *>(lp + (o & ~3));
  return __builtin_amdgcn_alignbyte(w[1], w[0], static_cast<uint32_t>(o & 3));
}

// kWhole: the words come in whole register groups (nw a multiple of
// kRightGroup for PX = 1, of kRightRegWords for PX = 4); the other case has
// a kernel of its own, so that neither shapes the other's code.
template <int PX, bool kWhole>
__device__ __forceinline__ void describe_right_tile(uint8_t *lds,
                                                    const uint32_t *__restrict__ packed, int W,
                                                    int H, const RightConsts &c,
                                                    uint64_t *__restrict__ desc, int u0, int v0) {
  constexpr int TW = 64 * PX;
  uint64_t *stage_all = reinterpret_cast<uint64_t *>(lds);
  // The register path stages nothing, so its tile starts at the bottom of
  // LDS, and a sample's address is one add from the lane's base.
  uint8_t *itile = lds + (kWhole && PX == 4 ? 0 : right_stage_bytes(PX));
  const int radius = c.radius, pitch = c.pitch, nw = c.nw;
  const int hx = right_halo(radius);  // tile column of pixel u0
  const int rows = kRightTH + 2 * radius, cols = hx + TW + radius;
  const int total = rows * cols;
  __syncthreads();  // the previous tile is done with LDS
  constexpr int kBatch = 8;
  for (int first = threadIdx.x; first < total; first += kRightThreads * kBatch) {
    uint32_t staged[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int i = first + b * kRightThreads;
      staged[b] = 0;
      if (i < total) {
        const int ty = i / cols, tx = i - ty * cols;
        const int gv = min(max(v0 - radius + ty, 0), H - 1);
        const int gu = min(max(u0 - hx + tx, 0), W - 1);
        staged[b] = packed[(size_t)gv * W + gu];
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int i = first + b * kRightThreads;
      if (i < total) {
        const int ty = i / cols, tx = i - ty * cols;
        itile[ty * pitch + tx] = static_cast<uint8_t>(staged[b] >> 24);
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = wave_index();
  const int ty = wave, v = v0 + ty;  // one row per wave
  if (v >= H) return;                // no barrier follows in this tile
  const int base = (ty + radius) * pitch + hx + PX * lane;  // multiple of 4 for PX = 4
  const int px0 = u0 + PX * lane;                           // the lane's first pixel
  const ConstInt2Table offs{c.offs};
  if constexpr (PX == 1) {
    uint64_t *out = desc + ((size_t)v * W + px0) * nw;
    if constexpr (kWhole) {
      // Whole groups (n a multiple of 1024): word indices are compile-time
      // constants and no word is skipped, so the 32 accumulators stay in
      // registers and leave as eight 16-byte stores.
      for (int g0 = 0; g0 < nw; g0 += kRightGroup) {
        uint32_t acc[kRightGroup][2];
        for_words<kRightGroup>([&](auto J) {
          constexpr int jj = J.value;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            acc[jj][h] = 0;
#pragma unroll 8
            for (int b = 31; b >= 0; --b) {
              const int2 o = offs[64 * (g0 + jj) + 32 * h + b];  // uniform: scalar load
              const uint32_t diff =
                  tile_bytes<1>(itile, base, o.y) - tile_bytes<1>(itile, base, o.x);
              acc[jj][h] = __builtin_amdgcn_alignbit(acc[jj][h], diff, 31);
            }
          }
        });
        if (px0 < W) {
          for_words<kRightGroup / 2>([&](auto K) {
            constexpr int jj = 2 * K.value;
            *reinterpret_cast<uint4 *>(out + g0 + jj) =
                make_uint4(acc[jj][0], acc[jj][1], acc[jj + 1][0], acc[jj + 1][1]);
          });
        }
      }
      return;
    }
    for (int g0 = 0; g0 < nw; g0 += kRightGroup) {
      uint32_t acc[kRightGroup][2];
#pragma unroll
      for (int jj = 0; jj < kRightGroup; ++jj) {
        if (g0 + jj >= nw) break;  // uniform
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[jj][h] = 0;
#pragma unroll 8
          for (int b = 31; b >= 0; --b) {
            // (a plain load: in this loop, with its early exit, vector loads
            // of the same address by every lane run further ahead than
            // scalar ones)
            const int2 o = c.offs[64 * (g0 + jj) + 32 * h + b];
            // tau of Eq. 3: for bytes p, q the difference q - p has bit 31
            // set exactly when p > q; alignbit shifts that bit into acc.
            const uint32_t diff = tile_bytes<1>(itile, base, o.y) - tile_bytes<1>(itile, base, o.x);
            acc[jj][h] = __builtin_amdgcn_alignbit(acc[jj][h], diff, 31);
          }
        }
      }
      // the pixel's words g0 .. g0 + G - 1 (contiguous)
      const int G = min(kRightGroup, nw - g0);
      if (px0 < W) {
        uint64_t *dst = out + g0;
        if ((nw & 1) == 0) {  // 16-byte aligned pairs of words
#pragma unroll
          for (int jj = 0; jj < kRightGroup; jj += 2) {
            if (jj >= G) break;  // uniform
            *reinterpret_cast<uint4 *>(dst + jj) =
                make_uint4(acc[jj][0], acc[jj][1], acc[jj + 1][0], acc[jj + 1][1]);
          }
        } else {
#pragma unroll
          for (int jj = 0; jj < kRightGroup; ++jj) {
            if (jj >= G) break;  // uniform
            dst[jj] = (static_cast<uint64_t>(acc[jj][1]) << 32) | acc[jj][0];
          }
        }
      }
    }
  } else {
    if constexpr (kWhole) {
      // Eight words (64 bytes) of each of the lane's four pixels in
      // registers, then each pixel's 64 bytes as four 16-byte stores in a
      // row: the half-lines are complete when they leave, so no partly
      // written line waits in the cache for the rest of the pixel's string.
      //
      // The four pixels' tests of one pair are one byte-parallel compare:
      // byte k of P and Q holds I(p), I(q) of pixel k, and the top bit of
      // byte k of lt is [I(q) < I(p)] (the compare of the low seven bits
      // in the top bit of (Q | 0x80) - (P & 0x7f), which borrows across no
      // byte, then the top bits decide).  Eight pairs shift into byte k of
      // e from the top, so e holds eight bits of each pixel; four such
      // registers are transposed into the pixels' 32-bit halves.
      const uint8_t *lp = itile + base;  // the lane's first pixel, 4-byte aligned
      uint64_t *out = desc + ((size_t)v * W + px0) * nw;
      static_assert(PX == 4, "byte-parallel tests of four pixels");
      constexpr uint32_t kTop = 0x80808080u;
      for (int g0 = 0; g0 < nw; g0 += kRightRegWords) {
        uint32_t words[kRightRegWords][2][PX];
        for_words<kRightRegWords>([&](auto J) {
          constexpr int jj = J.value;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            // e[3 - r] after the loop: pairs 8r .. 8r + 7 (a rolled loop
            // keeps the offsets of one group of eight in scalar registers)
            uint32_t e[4] = {0, 0, 0, 0};
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
              uint32_t x = 0;
#pragma unroll
              for (int b = 8 * r; b < 8 * r + 8; ++b) {
                const int2 o = offs[64 * (g0 + jj) + 32 * h + b];  // uniform: scalar load
                const uint32_t P = lane_bytes4(lp, o.x), Q = lane_bytes4(lp, o.y);
                const uint32_t low = (Q | kTop) - (P & ~kTop);
                // top bits: (!q7 & p7) | (!(q7 ^ p7) & !low7), as one
                // three-input bit operation (truth table on Q = 0xf0,
                // P = 0xcc, low = 0xaa)
                const uint32_t lt = __builtin_amdgcn_bitop3_b32(Q, P, low, 0x4d);
                x = (lt & kTop) | ((x >> 1) & ~kTop);
              }
              e[3] = e[2];
              e[2] = e[1];
              e[1] = e[0];
              e[0] = x;
            }
            // halves of pixels 0-3: bytes k of e[3], e[2], e[1], e[0]
            const uint32_t t01 = __builtin_amdgcn_perm(e[2], e[3], 0x05010400u);
            const uint32_t t23 = __builtin_amdgcn_perm(e[0], e[1], 0x05010400u);
            const uint32_t u01 = __builtin_amdgcn_perm(e[2], e[3], 0x07030602u);
            const uint32_t u23 = __builtin_amdgcn_perm(e[0], e[1], 0x07030602u);
            words[jj][h][0] = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
            words[jj][h][1] = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
            words[jj][h][2] = __builtin_amdgcn_perm(u23, u01, 0x05040100u);
            words[jj][h][3] = __builtin_amdgcn_perm(u23, u01, 0x07060302u);
          }
        });
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          if (px0 + k < W) {
            uint4 *dst = reinterpret_cast<uint4 *>(out + (size_t)k * nw + g0);
#pragma unroll
            for (int q = 0; q < kRightRegWords / 2; ++q)
              dst[q] = make_uint4(words[2 * q][0][k], words[2 * q][1][k], words[2 * q + 1][0][k],
                                  words[2 * q + 1][1][k]);
          }
        }
      }
      return;
    }
    uint64_t *stage = stage_all + wave * kRightStageWords * TW;
    const int valid = min(TW, W - u0);  // pixels of this tile inside the image
    uint64_t *row_out = desc + ((size_t)v * W + u0) * nw;
    for (int g0 = 0; g0 < nw; g0 += kRightStageWords) {
      const int G = min(kRightStageWords, nw - g0);
      for (int jj = 0; jj < G; ++jj) {
        const int j = g0 + jj;
        uint32_t half[2][PX];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint32_t acc[PX] = {};
#pragma unroll 8
          for (int b = 31; b >= 0; --b) {
            const int2 o = offs[64 * j + 32 * h + b];  // uniform: scalar load
            const uint32_t P = tile_bytes<PX>(itile, base, o.x);
            const uint32_t Q = tile_bytes<PX>(itile, base, o.y);
#pragma unroll
            for (int k = 0; k < PX; ++k) {
              const uint32_t diff = ((Q >> (8 * k)) & 0xffu) - ((P >> (8 * k)) & 0xffu);
              acc[k] = __builtin_amdgcn_alignbit(acc[k], diff, 31);
            }
          }
#pragma unroll
          for (int k = 0; k < PX; ++k) half[h][k] = acc[k];
        }
#pragma unroll
        for (int k = 0; k < PX; ++k)
          stage[jj * TW + PX * lane + k] = (static_cast<uint64_t>(half[1][k]) << 32) | half[0][k];
      }
      // Copy the group out: pixel p's words g0 .. g0+G-1 are contiguous in
      // global memory (the staging writes and reads are by the same wave,
      // in order).
      if (G == 2) {
        for (int p = lane; p < valid; p += 64)
          *reinterpret_cast<ulonglong2 *>(row_out + (size_t)p * nw + g0) =
              make_ulonglong2(stage[p], stage[TW + p]);
      } else {
        for (int p = lane; p < valid; p += 64) row_out[(size_t)p * nw + g0] = stage[p];
      }
    }
  }
}

template <int PX, bool kWhole>
__global__ __launch_bounds__(kRightThreads) void k_describe_right(
    const uint32_t *__restrict__ packed, int W, int H, RightConsts c,
    uint64_t *__restrict__ desc) {
  extern __shared__ uint8_t rlds[];
  describe_right_tile<PX, kWhole>(rlds, packed, W, H, c, desc, blockIdx.x * 64 * PX,
                                  blockIdx.y * kRightTH);
}

// ===========================================================================
// Masked cost fused with winner-take-all, n = 64 NW bits, NW in
// {1, 2, 4, 8, 16}.
//
// One wave per (row v, 128-pixel tile).  Lane l owns the two adjacent left
// pixels a = u0 + 2l and b = a + 1, with their B_L and Phi in registers.
// Disparities are walked in order; at step d lane l reads B_R(a - d) from
// LDS and uses it for (a, d) now and for (b, d + 1) at the next step, since
// b - (d + 1) = a - d: every right descriptor fetched from LDS serves two
// evaluations.  The right descriptors of the window a chunk of DC
// disparities needs sit in LDS split by parity, so at any step the 64 lanes
// read 64 consecutive 16-byte chunks (no bank conflicts).  Each evaluation is
// (bl ^ br) & m per 32-bit half (one v_bitop3_b32) plus a popcount that
// accumulates for free (v_bcnt_u32_b32); the running minimum of the key
// (C << 16) | d gives the lowest d among equal costs.  The cost volume, when
// wanted, is stored [d][v][u], so the two int16 costs of a lane form one
// coalesced 32-bit store per step.
// ===========================================================================
constexpr int kCostTX = 128;  // pixels per wave

// c + popcount(x) as one v_bcnt_u32_b32.  Written out so that the compiler
// keeps one accumulating chain instead of re-associating the sum into trees
// of extra adds.
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t c) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(c));
  return r;
}

// (a ^ b) & m in one v_bitop3_b32: the immediate is the truth table of the
// function evaluated on the operand patterns 0xF0, 0xCC, 0xAA.
constexpr unsigned kXorAnd = (0xF0 ^ 0xCC) & 0xAA;

// popcount((bl ^ br) & m) over nwords 64-bit words, on 32-bit halves: one
// v_bitop3_b32 and one accumulating v_bcnt_u32_b32 per half.
__device__ __forceinline__ uint32_t masked_cost(const uint64_t *bl, const uint64_t *m,
                                                const uint64_t *br, int nwords, bool use_mask) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < nwords; ++j) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t a = static_cast<uint32_t>(bl[j] >> (32 * h));
      const uint32_t b = static_cast<uint32_t>(br[j] >> (32 * h));
      const uint32_t x =
          use_mask ? __builtin_amdgcn_bitop3_b32(a, b, static_cast<uint32_t>(m[j] >> (32 * h)),
                                                 kXorAnd)
                   : (a ^ b);
      c = bcnt_acc(x, c);
    }
  }
  return c;
}

// LDS window of right descriptors for one chunk of DC disparities.  Elements
// are chunks of CW consecutive words of one pixel (16 bytes when n >= 128);
// the layout is [chunk jc][parity of pixel][pixel / 2][CW words], so at every
// step the 64 lanes (which read pixels of one parity, 2 apart) touch 64
// consecutive chunks, and the chunk index only moves a compile-time
// immediate offset.
template <int NW, int DC>
struct Window {
  static constexpr int CW = NW >= 2 ? 2 : 1;       // words per chunk
  static constexpr int CPP = NW / CW;               // chunks per pixel
  static constexpr int P = kCostTX - 1 + DC;         // pixels in the window
  static constexpr int HP = (P + 1) / 2 + 1;         // pixels per parity half
  static constexpr size_t kBytes = (size_t)CPP * 2 * HP * CW * sizeof(uint64_t);
  // u64 index of (chunk jc, relative pixel rel)
  __device__ static int index(int jc, int rel) {
    return ((jc * 2 + (rel & 1)) * HP + (rel >> 1)) * CW;
  }
};

// Copies the right descriptors of pixels [r_lo, r_lo + P) (zeros outside the
// image) into the LDS window.  Pixel r's words are contiguous in global
// memory, so the wave reads coalesced chunks with up to kBatch loads in
// flight per lane before writing them to LDS.
template <int NW, int DC>
__device__ __forceinline__ void stage_window(const uint64_t *__restrict__ rowR, int r_lo, int P,
                                             int W, int lane, uint64_t *win) {
  using Win = Window<NW, DC>;
  constexpr int kBatch = 8;
  const int total = P * Win::CPP;
  for (int first = lane; first < total; first += 64 * kBatch) {
    uint64_t staged[kBatch][Win::CW];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int c = first + 64 * b;
      const int rel = c / Win::CPP, jc = c % Win::CPP;
      const int r = r_lo + rel;
#pragma unroll
      for (int w = 0; w < Win::CW; ++w) staged[b][w] = 0;
      if (c < total && r >= 0 && r < W) {
        if (Win::CW == 2) {
          const ulonglong2 x =
              *reinterpret_cast<const ulonglong2 *>(rowR + (size_t)r * NW + 2 * jc);
          staged[b][0] = x.x;
          staged[b][Win::CW - 1] = x.y;
        } else {
          staged[b][0] = rowR[(size_t)r * NW + jc];
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int c = first + 64 * b;
      if (c < total) {
        const int rel = c / Win::CPP, jc = c % Win::CPP;
        uint64_t *dst = win + Win::index(jc, rel);
        if (Win::CW == 2)
          *reinterpret_cast<ulonglong2 *>(dst) = make_ulonglong2(staged[b][0], staged[b][Win::CW - 1]);
        else
          dst[0] = staged[b][0];
      }
    }
  }
}

// Loads the NW words of relative pixel `rel` from the window.
template <int NW, int DC>
__device__ __forceinline__ void load_right(const uint64_t *win, int rel, uint64_t *out) {
  using Win = Window<NW, DC>;
#pragma unroll
  for (int jc = 0; jc < Win::CPP; ++jc) {
    const uint64_t *src = win + Win::index(jc, rel);
    if (Win::CW == 2) {
      const ulonglong2 x = *reinterpret_cast<const ulonglong2 *>(src);
      out[2 * jc] = x.x;
      out[2 * jc + Win::CW - 1] = x.y;
    } else {
      out[jc] = src[0];
    }
  }
}

// Per-lane state of the fused cost + WTA tile.
template <int NW>
struct CostLane {
  uint64_t bla[NW], ma[NW], blb[NW], mb[NW];
  uint32_t best_a, best_b;
  int a, b;
  bool has_a, has_b;
};

// One disparity step d for the lane's pixels a and b: `cur` receives
// B_R(a - d) (relative pixel 2 lane + e), `prev` holds B_R(b - d).
template <int NW, int DC, bool MASK, bool VOL, bool EDGE>
__device__ __forceinline__ void cost_step(const uint64_t *win, int lane, int e, int d,
                                          CostLane<NW> &s, const uint64_t *prev, uint64_t *cur,
                                          int16_t *__restrict__ cost, int H, int W, int v) {
  load_right<NW, DC>(win, 2 * lane + e, cur);
  const uint32_t ca = masked_cost(s.bla, s.ma, cur, NW, MASK);
  const uint32_t cb = masked_cost(s.blb, s.mb, prev, NW, MASK);
  const bool va = !EDGE || s.a - d >= 0, vb = !EDGE || s.b - d >= 0;
  const uint32_t ka = (ca << 16) | (uint32_t)d, kb = (cb << 16) | (uint32_t)d;
  if (va) s.best_a = min(s.best_a, ka);
  if (vb) s.best_b = min(s.best_b, kb);
  if (VOL) {
    const uint32_t sa = va ? ca : (uint32_t)kInvalidCost;
    const uint32_t sb = vb ? cb : (uint32_t)kInvalidCost;
    int16_t *plane = cost + ((size_t)d * H + v) * W;
    if (s.has_b && ((((size_t)d * H + v) * W) & 1) == 0) {
      *reinterpret_cast<uint32_t *>(plane + s.a) = sa | (sb << 16);
    } else {
      if (s.has_a) plane[s.a] = (int16_t)sa;
      if (s.has_b) plane[s.b] = (int16_t)sb;
    }
  }
}

// All steps d in [dc0, dc1) of one window, two per iteration so that the two
// register buffers swap roles without copies.
template <int NW, int DC, bool MASK, bool VOL, bool EDGE>
__device__ __forceinline__ void cost_chunk(const uint64_t *win, int lane, int dc0, int dc1,
                                           CostLane<NW> &s, int16_t *__restrict__ cost, int H,
                                           int W, int v) {
  uint64_t x[NW], y[NW];
  load_right<NW, DC>(win, 2 * lane + (dc1 - dc0), x);  // B_R(b - dc0)
  int d = dc0;
  for (; d + 1 < dc1; d += 2) {
    cost_step<NW, DC, MASK, VOL, EDGE>(win, lane, dc1 - 1 - d, d, s, x, y, cost, H, W, v);
    cost_step<NW, DC, MASK, VOL, EDGE>(win, lane, dc1 - 2 - d, d + 1, s, y, x, cost, H, W, v);
  }
  if (d < dc1) cost_step<NW, DC, MASK, VOL, EDGE>(win, lane, dc1 - 1 - d, d, s, x, y, cost, H, W, v);
}

// One 128-pixel tile of row v starting at u0 (a single wave).
template <int NW, int DC, bool MASK, bool VOL>
__device__ __forceinline__ void cost_tile(uint64_t *win, const uint64_t *__restrict__ descL,
                                          const uint64_t *__restrict__ maskL,
                                          const uint64_t *__restrict__ descR, int W, int H,
                                          int dmax, int32_t *__restrict__ disp,
                                          int16_t *__restrict__ cost, int v, int u0) {
  const int lane = threadIdx.x;
  CostLane<NW> s;
  s.a = u0 + 2 * lane;
  s.b = s.a + 1;
  s.has_a = s.a < W;
  s.has_b = s.b < W;
  {
    const uint64_t *pa = descL + ((size_t)v * W + (s.has_a ? s.a : 0)) * NW;
    const uint64_t *pb = descL + ((size_t)v * W + (s.has_b ? s.b : 0)) * NW;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      s.bla[j] = s.has_a ? pa[j] : 0;
      s.blb[j] = s.has_b ? pb[j] : 0;
    }
    if (MASK) {
      const uint64_t *qa = maskL + ((size_t)v * W + (s.has_a ? s.a : 0)) * NW;
      const uint64_t *qb = maskL + ((size_t)v * W + (s.has_b ? s.b : 0)) * NW;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        s.ma[j] = s.has_a ? qa[j] : 0;
        s.mb[j] = s.has_b ? qb[j] : 0;
      }
    }
  }
  s.best_a = s.best_b = 0xffffffffu;
  const uint64_t *rowR = descR + (size_t)v * W * NW;

  for (int dc0 = 0; dc0 < dmax; dc0 += DC) {
    const int dc1 = min(dmax, dc0 + DC);
    const int r_lo = u0 - dc1 + 1;            // first right pixel of the window
    const int P = kCostTX - 1 + (dc1 - dc0);  // window width
    __syncthreads();                          // previous window fully consumed
    stage_window<NW, DC>(rowR, r_lo, P, W, lane, win);
    __syncthreads();
    if (u0 < dc1 - 1)  // some a - d < 0 inside this chunk
      cost_chunk<NW, DC, MASK, VOL, true>(win, lane, dc0, dc1, s, cost, H, W, v);
    else
      cost_chunk<NW, DC, MASK, VOL, false>(win, lane, dc0, dc1, s, cost, H, W, v);
  }
  if (s.has_a) disp[(size_t)v * W + s.a] = (int32_t)(s.best_a & 0xffffu);
  if (s.has_b) disp[(size_t)v * W + s.b] = (int32_t)(s.best_b & 0xffffu);
}

template <int NW, int DC, bool MASK, bool VOL>
__global__ __launch_bounds__(64, 2) void k_cost_wta_fast(const uint64_t *__restrict__ descL,
                                                      const uint64_t *__restrict__ maskL,
                                                      const uint64_t *__restrict__ descR, int W,
                                                      int H, int dmax, int32_t *__restrict__ disp,
                                                      int16_t *__restrict__ cost) {
  extern __shared__ uint64_t win[];
  // XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round-robin by
  // id, so ids b, b + 8, b + 16, ... share one XCD and its L2.  Rows are dealt
  // the same way (row v to XCD v mod 8) and all tiles of a row go to that
  // XCD, so the row's right descriptors, which every tile of the row reads
  // with a dmax halo, are fetched from HBM into a single L2.
  const int tiles = (W + kCostTX - 1) / kCostTX;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int v = xcd + kXcds * (slot / tiles);
  if (v >= H) return;  // whole block: ids past the last row of this XCD
  cost_tile<NW, DC, MASK, VOL>(win, descL, maskL, descR, W, H, dmax, disp, cost, v,
                               (slot % tiles) * kCostTX);
}

// ===========================================================================
// Masked cost + WTA on the matrix cores, n = 64 NW bits.
//
// The masked Hamming distance of Eq. 8 is a dot product.  For bits a (B_L),
// m (Phi_L) and b (B_R), m (a ^ b) = m a + m (1 - 2a) b, so
//   popcount((a ^ b) & m) = popcount(a & m) + sum_i v_i b_i,
// with v_i = m_i (1 - 2 a_i) in {-1, 0, 1}; Eq. 4 is the case m = all ones.
// popcount(a & m) is fixed per left pixel and cannot move its minimum over
// d, so the WTA ranks n + sum_i v_i b_i (in [0, 2n]) instead.  For one row,
// these sums for a tile of 32 left pixels against a block of 32 right pixels
// are one 32 x 32 matrix product over the n bits: left v as rows, right bits
// as columns.  Lane (c, h) = (l % 32, l / 32) supplies the bits of left
// pixel u0 + c (A operand, kept in registers) and of right pixel r0 + c (B
// operand, expanded from the packed words for each product); the two lane
// halves share out the bits of each product.  Which bit sits in which
// operand slot is free as long as A and B agree.  Right block q holds the
// pixels u0 - 32q + j, so entry (i, j) is disparity 32q + i - j and the
// blocks q = 0 .. Q-1 cover [0, dmax).  The accumulator gives lane (c, h)
// row 8(e/4) + 4h + e%4 of column c in its element e; the lane keeps the
// running minimum of the key (sum << 16) + d per element, and a butterfly
// over the 32 columns ends the WTA with the lowest d among equal costs.
// Every sum is exact, so the winners equal the bitwise kernel's.
// The products are fp4 ones (below).  An earlier int8 form
// (v_mfma_i32_32x32x32_i8, one byte per bit, 32 bits per product) took
// twice the products and about twice the vector instructions per bit.
// ===========================================================================
typedef int v4i32 __attribute__((ext_vector_type(4)));

constexpr int kMfmaTX = 32;     // left pixels per wave
// Row pitch (int16) of a wave's volume slab [d][pixel]: an odd number of
// dwords, so the 32 lanes of a half, which write 32 consecutive disparities
// of one pixel, hit 32 different LDS banks (a 32-entry pitch put them on 4).
constexpr int kSlabPitch = kMfmaTX + 2;
constexpr int kMfmaWaves = 4;   // tiles (waves) per workgroup, consecutive in a row

// Largest dmax of the matrix-core kernel with a volume: the wave's slab of
// the volume (dmax x 32 costs) is assembled in LDS.
constexpr int kMfmaVolMaxD = 256;

// ---------------------------------------------------------------------------
// The fp4 products.  v_mfma_scale_f32_32x32x64_f8f6f4 with e2m1 operands
// (and unit scales) takes 64 bits of the strings per product, at the issue
// cost of a 32-bit int8 product, so lane (c, h) supplies a whole
// 32-bit chunk: chunk h NW + k of the string in product k.  An e2m1 nibble
// with one bit set is 0.5, 1 or 2 (bit 0, 1, 2) or a sign (bit 3).  B dword t
// keeps the right bits 4j + t of the chunk where they are (nibble j worth
// 0.5, 1, 2 for t = 0, 1, 2: one AND), and dword 3 takes bits 4j + 3 one
// place down (worth 2).  A dword t carries v / (B's value) for the same bits:
// magnitude 2, 1, 0.5, 0.5 (nibble bit 2, 1, 0, 0) with the sign bit for
// v = -1.  Every product is v b exactly, every partial sum is a small
// integer, so the fp32 sums are exact.  With 2^23 + n added to a block's
// sum (fp32 steps by 1 there) the bit pattern is 0x4b000000 + (n + sum v b),
// and its low 16 bits shifted up give the key's cost half.
// ---------------------------------------------------------------------------
typedef float v16f32 __attribute__((ext_vector_type(16)));

// The four A dwords of one 32-bit chunk: a = B_L bits, m = Phi_L bits.
__device__ __forceinline__ void a_nibbles(uint32_t a, uint32_t m, v4i32 &A) {
  // m & a restricted to one bit of every nibble (0x80: x & y & z)
  const uint32_t n0 = __builtin_amdgcn_bitop3_b32(m, a, 0x11111111u, 0x80);
  const uint32_t n1 = __builtin_amdgcn_bitop3_b32(m, a, 0x22222222u, 0x80);
  const uint32_t n2 = __builtin_amdgcn_bitop3_b32(m, a, 0x44444444u, 0x80);
  const uint32_t n3 = __builtin_amdgcn_bitop3_b32(m, a, 0x88888888u, 0x80);
  A[0] = static_cast<int>(((m & 0x11111111u) << 2) | (n0 << 3));  // 2, sign
  A[1] = static_cast<int>((m & 0x22222222u) | (n1 << 2));         // 1, sign
  A[2] = static_cast<int>(((m >> 2) & 0x11111111u) | (n2 << 1));  // 0.5, sign
  A[3] = static_cast<int>(((m >> 3) & 0x11111111u) | n3);         // 0.5, sign
}

__device__ __forceinline__ v16f32 mfma_fp4(const v4i32 &A, const v4i32 &B, const v16f32 &C) {
  constexpr int kE2M1 = 4, kUnitScale = 127;  // operand format; E8M0 2^0
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
      __builtin_shufflevector(A, A, 0, 1, 2, 3, -1, -1, -1, -1),
      __builtin_shufflevector(B, B, 0, 1, 2, 3, -1, -1, -1, -1), C, kE2M1, kE2M1, 0,
      kUnitScale, 0, kUnitScale);
}

// The lane's NW 32-bit chunks of one string: chunks h NW .. h NW + NW - 1 of
// the 2 NW at p (16 bytes at a time when NW >= 4).
template <int NW>
__device__ __forceinline__ void load_chunks(const uint64_t *p, int h, uint32_t *out) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) u32x4 *GlobalU4;
  typedef const __attribute__((address_space(1))) u32x2 *GlobalU2;
  typedef const __attribute__((address_space(1))) uint32_t *GlobalU1;
  const uint32_t *q = reinterpret_cast<const uint32_t *>(p) + h * NW;
  if constexpr (NW >= 4) {
#pragma unroll
    for (int i = 0; i < NW / 4; ++i) {
      const u32x4 x = ((GlobalU4)q)[i];
      out[4 * i] = x[0];
      out[4 * i + 1] = x[1];
      out[4 * i + 2] = x[2];
      out[4 * i + 3] = x[3];
    }
  } else if constexpr (NW == 2) {
    const u32x2 x = *(GlobalU2)q;
    out[0] = x[0];
    out[1] = x[1];
  } else {
    out[0] = *(GlobalU1)q;
  }
}

// The A operands of left pixel ua of row v for the lane's half h of the
// chunks (zero past the row's end, where the loads read a clamped pixel, so
// no load sits behind a branch); with VOL also popcount(a & m) of that half.
template <int NW, bool MASK, bool VOL = false>
__device__ __forceinline__ void a_operands_of(const uint64_t *__restrict__ descL,
                                              const uint64_t *__restrict__ maskL, int W, int v,
                                              int ua, int h, v4i32 *A, int *am = nullptr) {
  const bool has_a = ua < W;
  const size_t pa_off = ((size_t)v * W + (has_a ? ua : W - 1)) * NW;
  uint32_t aw[NW], mw[NW];
  load_chunks<NW>(descL + pa_off, h, aw);
  if (MASK) load_chunks<NW>(maskL + pa_off, h, mw);
  int pc = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    if (!MASK) mw[k] = 0xffffffffu;
    if (!has_a) aw[k] = mw[k] = 0;
    if (VOL) pc += __builtin_popcount(aw[k] & mw[k]);
    a_nibbles(aw[k], mw[k], A[k]);
  }
  if (VOL) *am = pc;
}

// One wave: the 32 left pixels of row v from u0.  With VOL, `slab` is the
// wave's LDS (dmax x 32 int16): each cost goes there first, at [d][i], and
// the slab leaves as whole 64-byte rows of cost[d][v][u0 .. u0 + 31].
template <int NW, bool MASK, bool VOL = false>
__device__ __forceinline__ void cost_tile_mfma(const uint64_t *__restrict__ descL,
                                               const uint64_t *__restrict__ maskL,
                                               const uint64_t *__restrict__ descR, int W,
                                               int H, int dmax, int32_t *__restrict__ disp,
                                               int16_t *__restrict__ cost, int16_t *slab, int v,
                                               int u0) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 31, h = lane >> 5;
  int am = 0;  // popcount(a & m) of the lane's half of its left pixel (volume only)
  v4i32 A[NW];
  a_operands_of<NW, MASK, VOL>(descL, maskL, W, v, u0 + c, h, A, &am);
  // costs: C = popcount(a & m) + sum v b = am_row - n + (n + sum v b), the
  // last term the low 16 bits of the block's sum plus 2^23 + n
  int cbase[16];
  if (VOL) {
    am += __shfl_xor(am, 32);  // both halves of the pixel
#pragma unroll
    for (int e = 0; e < 16; ++e) cbase[e] = __shfl(am, 8 * (e / 4) + 4 * h + (e % 4)) - 64 * NW;
  }
  // The key of element e in block q is ((n + sum v b) << 16) + 32 q +
  // kKeyBias.  The rest of d = 32 q + row(e) - c is the lane's own and the
  // same in every block, so it joins the low half once, after the blocks
  // (the bias keeps the low half from borrowing: row(e) - c >= -31).  Within
  // an element a lower key is a lower cost or, on equal costs, a lower q, d.
  constexpr uint32_t kKeyBias = 64;
  constexpr float kBias = 8388608.0f + 64.0f * NW;  // 2^23 + n
  const v16f32 zero = {};
  uint32_t best[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) best[e] = 0xffffffffu;
  const uint64_t *rowR = descR + (size_t)v * W * NW;
  const int nq = (dmax + 30) / kMfmaTX + 1;  // right blocks
  // The lane's right pixel of block q, clamped into the row for loading.
  auto right_px = [&](int q) { return min(max(u0 - kMfmaTX * q + c, 0), W - 1); };
  uint32_t bw[NW];
  load_chunks<NW>(rowR + (size_t)right_px(0) * NW, h, bw);
  // One right block; with `fast` every entry of the block is valid.
  auto block = [&](int q, auto fast) {
    // The next block's chunks load into bw as this block's products use them
    // up (16 bytes per four products), so that they have the whole block to
    // arrive.  The loads are unconditional (after the last block they read
    // a clamped pixel of the row again).
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) u32x4 *GlobalU4;
    const uint64_t *next_px = rowR + (size_t)right_px(q + 1) * NW;
    const GlobalU4 next = (GlobalU4)(reinterpret_cast<const uint32_t *>(next_px) + h * NW);
    const int rb = u0 - kMfmaTX * q + c;  // the lane's right pixel
    // a missing right pixel gives B = 0
    const uint32_t ones = (rb >= 0 && rb < W) ? 0xffffffffu : 0u;
    const uint32_t b0 = ones & 0x11111111u, b1 = ones & 0x22222222u, b2 = ones & 0x44444444u;
    v16f32 acc;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const uint32_t x = bw[k];
      v4i32 B;
      B[0] = static_cast<int>(x & b0);
      B[1] = static_cast<int>(x & b1);
      B[2] = static_cast<int>(x & b2);
      B[3] = static_cast<int>((x >> 1) & b2);
      acc = mfma_fp4(A[k], B, k == 0 ? zero : acc);
      if constexpr (NW >= 4) {
        if ((k & 3) == 3) {
          const u32x4 y = next[k / 4];
          bw[k - 3] = y[0];
          bw[k - 2] = y[1];
          bw[k - 1] = y[2];
          bw[k] = y[3];
          // keep the load here: scheduled freely, the loads move to one end
          // of the block
          __builtin_amdgcn_sched_barrier(0);
        }
      } else if (k == NW - 1) {
        load_chunks<NW>(next_px, h, bw);
      }
    }
    // d of element e is dbase + row(e); valid when 0 <= d < dmax and the
    // right pixel exists (u - d = rb >= 0).
    const int dbase = kMfmaTX * q - c;
    const uint32_t key_lo = kMfmaTX * q + kKeyBias;  // wave-uniform
    uint32_t sum[16];  // n + sum v b in the low 16 bits
#pragma unroll
    for (int e = 0; e < 16; ++e) sum[e] = __float_as_uint(acc[e] + kBias);
    if (VOL) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int d = dbase + 8 * (e / 4) + 4 * h + (e % 4);
        if (d >= 0 && d < dmax)
          slab[d * kSlabPitch + 8 * (e / 4) + 4 * h + (e % 4)] = static_cast<int16_t>(
              rb >= 0 ? cbase[e] + static_cast<int>(sum[e] & 0xffffu)
                      : kInvalidCost);
      }
    }
    if constexpr (decltype(fast)::value) {
#pragma unroll
      for (int e = 0; e < 16; ++e)
        best[e] = min(best[e], (sum[e] << 16) + key_lo);
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int d = dbase + 8 * (e / 4) + 4 * h + (e % 4);
        const uint32_t key = (sum[e] << 16) + key_lo;
        if (d >= 0 && d < dmax && rb >= 0) best[e] = min(best[e], key);
      }
    }
  };
  // Every entry of block q is valid for 1 <= q <= q_fast (d in [1, dmax),
  // right pixel in the row); the condition only weakens as q grows, so the
  // blocks run as three loops without per-block branches.
  const int q_fast =
      min(nq - 1, min(dmax >= kMfmaTX ? (dmax - kMfmaTX) / kMfmaTX : 0, u0 / kMfmaTX));
  block(0, std::false_type{});
  for (int q = 1; q <= q_fast; ++q) block(q, std::true_type{});
  for (int q = max(q_fast + 1, 1); q < nq; ++q) block(q, std::false_type{});
  // the lane's part of d (an element no block updated stays above every
  // real key: 0xffffffff less at most 95)
#pragma unroll
  for (int e = 0; e < 16; ++e)
    best[e] += static_cast<uint32_t>(8 * (e / 4) + 4 * h + (e % 4) - c) - kKeyBias;
  // WTA across the 32 columns of each half.
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
#pragma unroll
    for (int e = 0; e < 16; ++e)
      best[e] = min(best[e], static_cast<uint32_t>(__shfl_xor(static_cast<int>(best[e]), off)));
  }
  if (c < 16) {
    uint32_t key = best[0];
#pragma unroll
    for (int e = 1; e < 16; ++e)
      if (c == e) key = best[e];
    const int u = u0 + 8 * (c / 4) + 4 * h + (c % 4);
    if (u < W) disp[(size_t)v * W + u] = static_cast<int32_t>(key & 0xffffu);
  }
  if (VOL) {
    // The slab was written by the lanes of this wave only; LDS accesses of
    // one wave are performed in order, so a wave-level fence suffices.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // four rows per pass: lane l takes row 4k + l / 16, pixels 2 (l % 16), + 1
    const int pr = lane >> 4, px = 2 * (lane & 15), u = u0 + px;
    for (int d = pr; d < dmax; d += 4) {
      const uint32_t two = *reinterpret_cast<const uint32_t *>(slab + d * kSlabPitch + px);
      int16_t *dst = cost + ((size_t)d * H + v) * W + u;
      if (u + 1 < W && (reinterpret_cast<uintptr_t>(dst) & 3u) == 0) {
        *reinterpret_cast<uint32_t *>(dst) = two;
      } else {
        if (u < W) dst[0] = static_cast<int16_t>(two & 0xffffu);
        if (u + 1 < W) dst[1] = static_cast<int16_t>(two >> 16);
      }
    }
  }
}

// Two adjacent tiles in one wave, left pixels u0 .. u0 + 63 (both tiles
// start inside the row).  Right block b (pixels u0 + 32 - 32 b + j) is block
// q = b of tile 1 and block q = b - 1 of tile 0, so its B operands, expanded
// once, feed the products of both tiles: blocks b = 0 .. nq, the first for
// tile 1 alone and the last for tile 0 alone.  Keys as in cost_tile_mfma.
template <int NW, bool MASK>
__device__ __forceinline__ void cost_tile_pair_mfma(const uint64_t *__restrict__ descL,
                                                    const uint64_t *__restrict__ maskL,
                                                    const uint64_t *__restrict__ descR, int W,
                                                    int dmax, int32_t *__restrict__ disp, int v,
                                                    int u0) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 31, h = lane >> 5;
  v4i32 A0[NW], A1[NW];
  a_operands_of<NW, MASK>(descL, maskL, W, v, u0 + c, h, A0);
  a_operands_of<NW, MASK>(descL, maskL, W, v, u0 + kMfmaTX + c, h, A1);
  constexpr uint32_t kKeyBias = 64;
  constexpr float kBias = 8388608.0f + 64.0f * NW;  // 2^23 + n
  const v16f32 zero = {};
  uint32_t best0[16], best1[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) best0[e] = best1[e] = 0xffffffffu;
  const uint64_t *rowR = descR + (size_t)v * W * NW;
  const int nq = (dmax + 30) / kMfmaTX + 1;  // right blocks of each tile
  const int u1 = u0 + kMfmaTX;                // tile 1's first pixel
  auto right_px = [&](int b) { return min(max(u1 - kMfmaTX * b + c, 0), W - 1); };
  uint32_t bw[NW];
  load_chunks<NW>(rowR + (size_t)right_px(0) * NW, h, bw);
  // tile t's entries of one block into its running minima
  auto fold = [&](const v16f32 &acc, uint32_t *best, int q, int rb, auto fast) {
    const uint32_t key_lo = kMfmaTX * q + kKeyBias;  // wave-uniform
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t key = (__float_as_uint(acc[e] + kBias) << 16) + key_lo;
      if constexpr (decltype(fast)::value) {
        best[e] = min(best[e], key);
      } else {
        const int d = kMfmaTX * q - c + 8 * (e / 4) + 4 * h + (e % 4);
        if (d >= 0 && d < dmax && rb >= 0) best[e] = min(best[e], key);
      }
    }
  };
  // Right block b for tile 0 (USE0: q = b - 1) and tile 1 (USE1: q = b);
  // with `fast` every entry of both is valid.
  auto block = [&](int b, auto use0, auto use1, auto fast) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) u32x4 *GlobalU4;
    const uint64_t *next_px = rowR + (size_t)right_px(b + 1) * NW;
    const GlobalU4 next = (GlobalU4)(reinterpret_cast<const uint32_t *>(next_px) + h * NW);
    const int rb = u1 - kMfmaTX * b + c;  // the lane's right pixel (both tiles)
    const uint32_t ones = (rb >= 0 && rb < W) ? 0xffffffffu : 0u;
    const uint32_t b0 = ones & 0x11111111u, b1 = ones & 0x22222222u, b2 = ones & 0x44444444u;
    v16f32 acc0, acc1;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const uint32_t x = bw[k];
      v4i32 B;
      B[0] = static_cast<int>(x & b0);
      B[1] = static_cast<int>(x & b1);
      B[2] = static_cast<int>(x & b2);
      B[3] = static_cast<int>((x >> 1) & b2);
      if constexpr (decltype(use1)::value) acc1 = mfma_fp4(A1[k], B, k == 0 ? zero : acc1);
      if constexpr (decltype(use0)::value) acc0 = mfma_fp4(A0[k], B, k == 0 ? zero : acc0);
      if constexpr (NW >= 4) {
        if ((k & 3) == 3) {
          const u32x4 y = next[k / 4];
          bw[k - 3] = y[0];
          bw[k - 2] = y[1];
          bw[k - 1] = y[2];
          bw[k] = y[3];
          __builtin_amdgcn_sched_barrier(0);
        }
      } else if (k == NW - 1) {
        load_chunks<NW>(next_px, h, bw);
      }
    }
    if constexpr (decltype(use1)::value) fold(acc1, best1, b, rb, fast);
    if constexpr (decltype(use0)::value) fold(acc0, best0, b - 1, rb, fast);
  };
  // Every entry of both tiles is valid for 2 <= b <= b_fast (tile 0's
  // q = b - 1 >= 1, d < dmax for tile 1's q = b, right pixels in the row);
  // the condition only weakens as b grows.
  const int b_fast =
      min(nq - 1, min(dmax >= kMfmaTX ? (dmax - kMfmaTX) / kMfmaTX : 0, u1 / kMfmaTX));
  block(0, std::false_type{}, std::true_type{}, std::false_type{});
  if (nq > 1) block(1, std::true_type{}, std::true_type{}, std::false_type{});
  for (int b = 2; b <= b_fast; ++b) block(b, std::true_type{}, std::true_type{}, std::true_type{});
  for (int b = max(b_fast + 1, 2); b < nq; ++b)
    block(b, std::true_type{}, std::true_type{}, std::false_type{});
  block(nq, std::true_type{}, std::false_type{}, std::false_type{});
  // the lane's part of d, then the WTA across the 32 columns of each half
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint32_t part = static_cast<uint32_t>(8 * (e / 4) + 4 * h + (e % 4) - c) - kKeyBias;
    best0[e] += part;
    best1[e] += part;
  }
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      best0[e] = min(best0[e], static_cast<uint32_t>(__shfl_xor(static_cast<int>(best0[e]), off)));
      best1[e] = min(best1[e], static_cast<uint32_t>(__shfl_xor(static_cast<int>(best1[e]), off)));
    }
  }
  if (c < 16) {
    uint32_t key0 = best0[0], key1 = best1[0];
#pragma unroll
    for (int e = 1; e < 16; ++e)
      if (c == e) {
        key0 = best0[e];
        key1 = best1[e];
      }
    const int u = u0 + 8 * (c / 4) + 4 * h + (c % 4);
    if (u < W) disp[(size_t)v * W + u] = static_cast<int32_t>(key0 & 0xffffu);
    if (u + kMfmaTX < W) disp[(size_t)v * W + u + kMfmaTX] = static_cast<int32_t>(key1 & 0xffffu);
  }
}

template <int NW, bool MASK>
__global__ __launch_bounds__(64 * kMfmaWaves, 2) void k_cost_wta_mfma(
    const uint64_t *__restrict__ descL, const uint64_t *__restrict__ maskL,
    const uint64_t *__restrict__ descR, int W, int H, int dmax, int32_t *__restrict__ disp) {
  // XCD-aware order (see k_cost_wta_fast), in groups of kMfmaWaves waves of
  // two tiles each (a duo).
  const int duos = (W + 2 * kMfmaTX - 1) / (2 * kMfmaTX);
  const int groups = (duos + kMfmaWaves - 1) / kMfmaWaves;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int v = xcd + kXcds * (slot / groups);
  const int duo = (slot % groups) * kMfmaWaves + wave_index();
  if (v >= H || duo >= duos) return;  // whole wave; no barrier follows
  const int u0 = duo * 2 * kMfmaTX;
  if (u0 + kMfmaTX < W)
    cost_tile_pair_mfma<NW, MASK>(descL, maskL, descR, W, dmax, disp, v, u0);
  else
    cost_tile_mfma<NW, MASK>(descL, maskL, descR, W, H, dmax, disp, nullptr, nullptr, v, u0);
}

// With the volume (dmax <= kMfmaVolMaxD): dynamic LDS of kMfmaWaves slabs.
template <int NW, bool MASK>
__global__ __launch_bounds__(64 * kMfmaWaves, 2) void k_cost_wta_mfma_vol(
    const uint64_t *__restrict__ descL, const uint64_t *__restrict__ maskL,
    const uint64_t *__restrict__ descR, int W, int H, int dmax, int32_t *__restrict__ disp,
    int16_t *__restrict__ cost) {
  extern __shared__ int16_t slabs[];
  const int tiles = (W + kMfmaTX - 1) / kMfmaTX;
  const int groups = (tiles + kMfmaWaves - 1) / kMfmaWaves;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int v = xcd + kXcds * (slot / groups);
  const int wave = wave_index();
  const int tile = (slot % groups) * kMfmaWaves + wave;
  if (v >= H || tile >= tiles) return;  // whole wave; no barrier follows
  cost_tile_mfma<NW, MASK, true>(descL, maskL, descR, W, H, dmax, disp, cost,
                                 slabs + (size_t)wave * dmax * kSlabPitch, v, tile * kMfmaTX);
}

// ===========================================================================
// Matrix-core cost + WTA for long descriptors: nw a multiple of 8 above 16
// (n = 1536, 2048, ..., 4096), no volume, dmax <= 256, with cost_tile_mfma's
// fp4 products.  The A operands of a tile's 32 left pixels for all n bits
// would need 2 nw registers a lane, so the bits go in passes of 512 (8
// words): a pass builds A for its 16 chunks (8 a lane half), then runs every
// right block q over them, adding into block q's accumulator, which lives
// across the passes (nine blocks at dmax 256: 144 registers).  Within a
// pass, block q + 1's right words load 16 bytes at a time while block q's
// products run.  Bounded to two waves per SIMD (256 registers a lane, one
// value spilled), which hide the chains of dependent products far better
// than one.
// The sums stay exact integers (|sum v b| <= n); the key takes n + sum v b
// from the low mantissa bits of the sum plus 2^23 + n, as cost_tile_mfma.
// ===========================================================================
constexpr int kLongPassWords = 8;
constexpr int kLongMaxBlocks = 9;  // right blocks, (dmax + 30) / 32 + 1, at dmax 256
constexpr int kLongMaxDmax = 256;

template <bool MASK>
__device__ __forceinline__ void cost_tile_mfma_long(const uint64_t *__restrict__ descL,
                                                    const uint64_t *__restrict__ maskL,
                                                    const uint64_t *__restrict__ descR, int W,
                                                    int nw, int dmax, int32_t *__restrict__ disp,
                                                    int v, int u0) {
  constexpr int kChunks = kLongPassWords;  // 32-bit chunks of a pass per lane half
  const int lane = threadIdx.x & 63;
  const int c = lane & 31, h = lane >> 5;
  const int ua = u0 + c;
  const bool has_a = ua < W;
  const size_t pa_off = ((size_t)v * W + (has_a ? ua : W - 1)) * nw;
  const uint64_t *rowR = descR + (size_t)v * W * nw;
  const int nq = (dmax + 30) / kMfmaTX + 1;  // right blocks, <= kLongMaxBlocks
  auto right_px = [&](int q) { return min(max(u0 - kMfmaTX * q + c, 0), W - 1); };
  v16f32 acc[kLongMaxBlocks];
#pragma unroll
  for (int q = 0; q < kLongMaxBlocks; ++q)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
  for (int w0 = 0; w0 < nw; w0 += kLongPassWords) {
    // A operands of this pass: the lane half's chunks 2 w0 + 8 h .. + 7
    v4i32 A[kChunks];
    {
      uint32_t aw[kChunks], mw[kChunks];
      load_chunks<kChunks>(descL + pa_off + w0, h, aw);
      if (MASK) load_chunks<kChunks>(maskL + pa_off + w0, h, mw);
#pragma unroll
      for (int k = 0; k < kChunks; ++k) {
        if (!MASK) mw[k] = 0xffffffffu;
        if (!has_a) aw[k] = mw[k] = 0;
        a_nibbles(aw[k], mw[k], A[k]);
      }
    }
    uint32_t bw[kChunks];  // right chunks of the block being multiplied
    load_chunks<kChunks>(rowR + (size_t)right_px(0) * nw + w0, h, bw);
#pragma unroll
    for (int q = 0; q < kLongMaxBlocks; ++q) {
      if (q < nq) {  // uniform
        const int rb = u0 - kMfmaTX * q + c;
        const uint32_t ones = (rb >= 0 && rb < W) ? 0xffffffffu : 0u;
        const uint32_t b0 = ones & 0x11111111u, b1 = ones & 0x22222222u,
                       b2 = ones & 0x44444444u;
        // the next block's chunks of this pass load as these are used up,
        // as in cost_tile_mfma (right_px clamps, so after the last block
        // the load stays in the row and its words go unused)
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(1))) u32x4 *GlobalU4;
        const GlobalU4 next = (GlobalU4)(reinterpret_cast<const uint32_t *>(
                                             rowR + (size_t)right_px(q + 1) * nw + w0) +
                                         h * kChunks);
#pragma unroll
        for (int k = 0; k < kChunks; ++k) {
          const uint32_t x = bw[k];
          v4i32 B;
          B[0] = static_cast<int>(x & b0);
          B[1] = static_cast<int>(x & b1);
          B[2] = static_cast<int>(x & b2);
          B[3] = static_cast<int>((x >> 1) & b2);
          acc[q] = mfma_fp4(A[k], B, acc[q]);
          if ((k & 3) == 3) {
            const u32x4 y = next[k / 4];
            bw[k - 3] = y[0];
            bw[k - 2] = y[1];
            bw[k - 1] = y[2];
            bw[k] = y[3];
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
  }
  // WTA: element e of block q is d = 32 q - c + row(e), valid when
  // 0 <= d < dmax and the right pixel exists
  const float bias = 8388608.0f + 64.0f * static_cast<float>(nw);  // 2^23 + n
  uint32_t best[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) best[e] = 0xffffffffu;
#pragma unroll
  for (int q = 0; q < kLongMaxBlocks; ++q) {
    if (q < nq) {
      const int rb = u0 - kMfmaTX * q + c;
      const int dbase = kMfmaTX * q - c;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int d = dbase + 8 * (e / 4) + 4 * h + (e % 4);
        const uint32_t key = (__float_as_uint(acc[q][e] + bias) << 16) | static_cast<uint32_t>(d);
        if (d >= 0 && d < dmax && rb >= 0) best[e] = min(best[e], key);
      }
    }
  }
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
#pragma unroll
    for (int e = 0; e < 16; ++e)
      best[e] = min(best[e], static_cast<uint32_t>(__shfl_xor(static_cast<int>(best[e]), off)));
  }
  if (c < 16) {
    uint32_t key = best[0];
#pragma unroll
    for (int e = 1; e < 16; ++e)
      if (c == e) key = best[e];
    const int u = u0 + 8 * (c / 4) + 4 * h + (c % 4);
    if (u < W) disp[(size_t)v * W + u] = static_cast<int32_t>(key & 0xffffu);
  }
}

template <bool MASK>
__global__ __launch_bounds__(64 * kMfmaWaves, 2) void k_cost_wta_mfma_long(
    const uint64_t *__restrict__ descL, const uint64_t *__restrict__ maskL,
    const uint64_t *__restrict__ descR, int W, int H, int nw, int dmax,
    int32_t *__restrict__ disp) {
  // XCD-aware order, as k_cost_wta_mfma
  const int tiles = (W + kMfmaTX - 1) / kMfmaTX;
  const int groups = (tiles + kMfmaWaves - 1) / kMfmaWaves;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int v = xcd + kXcds * (slot / groups);
  const int tile = (slot % groups) * kMfmaWaves + wave_index();
  if (v >= H || tile >= tiles) return;  // whole wave; no barrier follows
  cost_tile_mfma_long<MASK>(descL, maskL, descR, W, nw, dmax, disp, v, tile * kMfmaTX);
}

// ===========================================================================
// Cost + WTA for any n = 64 nw bits (nw outside the register-resident
// kernel's set, up to n = 4096).  Same tiling and diagonal reuse as above
// (one wave per row tile of 128 pixels, lane l owns a = u0 + 2l and b = a +
// 1, B_R(a - d) serves (a, d) and (b, d + 1)), but the words of the
// descriptors are walked in chunks of kChunkWords: for each chunk of
// kChunkD disparities the lane keeps the partial costs of its two pixels in
// registers and adds one chunk of words at a time, with the left words of
// its pixels loaded from global memory and the right words of the window
// staged in LDS as [word][parity][pixel / 2].  Words past nw are zero.
// ===========================================================================
constexpr int kChunkD = 32, kChunkWords = 4;
constexpr int kChunkP = kCostTX - 1 + kChunkD;      // window pixels
constexpr int kChunkHP = (kChunkP + 1) / 2 + 1;     // pixels per parity half
constexpr size_t kChunkLds = 2 * (size_t)(kChunkWords / 2) * 2 * kChunkHP * 2 * sizeof(uint64_t);

__device__ __forceinline__ uint32_t masked_cost1(uint64_t bl, uint64_t m, uint64_t br, bool use_mask,
                                                 uint32_t c) {
  const uint32_t lo = use_mask ? __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(bl),
                                                             static_cast<uint32_t>(br),
                                                             static_cast<uint32_t>(m), kXorAnd)
                               : static_cast<uint32_t>(bl ^ br);
  const uint32_t hi = use_mask ? __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(bl >> 32),
                                                             static_cast<uint32_t>(br >> 32),
                                                             static_cast<uint32_t>(m >> 32), kXorAnd)
                               : static_cast<uint32_t>((bl ^ br) >> 32);
  return bcnt_acc(hi, bcnt_acc(lo, c));
}

// Window elements a lane stages per chunk: kChunkP pixels x kChunkWords,
// taken as 16-byte pairs of words.
constexpr int kChunkPairs = kChunkWords / 2;
constexpr int kChunkStage = (kChunkP * kChunkPairs + 63) / 64;

// The steps of a tile are (disparity chunk, word chunk) pairs in order; the
// global loads of step s + 1 (right window into registers, then LDS; the
// lane's left words and mask words) are issued before step s computes, so
// their latency hides behind a step's arithmetic.  Words travel in 16-byte
// pairs when nw is even (every pixel's words are then 16-byte aligned).
struct ChunkLoads {
  uint64_t win[kChunkStage][2];
  uint64_t la[kChunkWords], lb[kChunkWords], ma[kChunkWords], mb[kChunkWords];
};

// Words j, j + 1 of a pixel's string p (zeros past nw or for a missing
// pixel); `pairs` = nw is even.
__device__ __forceinline__ void load_word_pair(const uint64_t *p, int j, int nw, bool present,
                                               bool pairs, uint64_t &x, uint64_t &y) {
  x = y = 0;
  if (!present || j >= nw) return;
  if (pairs) {
    const ulonglong2 t = *reinterpret_cast<const ulonglong2 *>(p + j);
    x = t.x;
    y = t.y;
  } else {
    x = p[j];
    if (j + 1 < nw) y = p[j + 1];
  }
}

template <bool MASK>
__device__ __forceinline__ void chunk_load(ChunkLoads &L, const uint64_t *__restrict__ rowR,
                                           const uint64_t *la, const uint64_t *lb,
                                           const uint64_t *qa, const uint64_t *qb, bool has_a,
                                           bool has_b, int W, int nw, int r_lo, int j0,
                                           int lane) {
  const bool pairs = (nw & 1) == 0;
#pragma unroll
  for (int k = 0; k < kChunkStage; ++k) {
    const int i = lane + 64 * k;
    const int rel = i / kChunkPairs, h = i - rel * kChunkPairs;
    const int r = r_lo + rel;
    load_word_pair(rowR + (size_t)(r >= 0 ? r : 0) * nw, j0 + 2 * h, nw,
                   i < kChunkP * kChunkPairs && r >= 0 && r < W, pairs, L.win[k][0], L.win[k][1]);
  }
#pragma unroll
  for (int h = 0; h < kChunkPairs; ++h) {
    const int j = j0 + 2 * h;
    load_word_pair(la, j, nw, has_a, pairs, L.la[2 * h], L.la[2 * h + 1]);
    load_word_pair(lb, j, nw, has_b, pairs, L.lb[2 * h], L.lb[2 * h + 1]);
    if (MASK) {
      load_word_pair(qa, j, nw, has_a, pairs, L.ma[2 * h], L.ma[2 * h + 1]);
      load_word_pair(qb, j, nw, has_b, pairs, L.mb[2 * h], L.mb[2 * h + 1]);
    } else {
      L.ma[2 * h] = L.ma[2 * h + 1] = L.mb[2 * h] = L.mb[2 * h + 1] = 0;
    }
  }
}

__device__ __forceinline__ void chunk_store_window(const ChunkLoads &L, ulonglong2 *buf, int lane) {
#pragma unroll
  for (int k = 0; k < kChunkStage; ++k) {
    const int i = lane + 64 * k;
    if (i < kChunkP * kChunkPairs) {
      const int rel = i / kChunkPairs, h = i - rel * kChunkPairs;
      buf[(h * 2 + (rel & 1)) * kChunkHP + (rel >> 1)] = make_ulonglong2(L.win[k][0], L.win[k][1]);
    }
  }
}

template <bool MASK, bool VOL>
__global__ __launch_bounds__(64) void k_cost_wta_chunked(const uint64_t *__restrict__ descL,
                                                         const uint64_t *__restrict__ maskL,
                                                         const uint64_t *__restrict__ descR, int W,
                                                         int H, int nw, int dmax,
                                                         int32_t *__restrict__ disp,
                                                         int16_t *__restrict__ cost) {
  extern __shared__ ulonglong2 cwin[];  // two buffers of [kChunkPairs][2][kChunkHP]
  constexpr int kBuf = kChunkPairs * 2 * kChunkHP;
  const int tiles = (W + kCostTX - 1) / kCostTX;
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const int v = xcd + kXcds * (slot / tiles);
  if (v >= H) return;  // whole block
  const int u0 = (slot % tiles) * kCostTX;
  const int lane = threadIdx.x;
  const int a = u0 + 2 * lane, b = a + 1;
  const bool has_a = a < W, has_b = b < W;
  const uint64_t *rowR = descR + (size_t)v * W * nw;
  const uint64_t *la = descL + ((size_t)v * W + (has_a ? a : 0)) * nw;
  const uint64_t *lb = descL + ((size_t)v * W + (has_b ? b : 0)) * nw;
  const uint64_t *qa = MASK ? maskL + ((size_t)v * W + (has_a ? a : 0)) * nw : nullptr;
  const uint64_t *qb = MASK ? maskL + ((size_t)v * W + (has_b ? b : 0)) * nw : nullptr;
  const int nwc = (nw + kChunkWords - 1) / kChunkWords;   // word chunks
  const int ndc = (dmax + kChunkD - 1) / kChunkD;         // disparity chunks
  const int steps = nwc * ndc;
  uint32_t best_a = 0xffffffffu, best_b = 0xffffffffu;
  uint32_t ca[kChunkD], cb[kChunkD];

  ChunkLoads cur, next;
  // right pixel of relative index 0 for disparity chunk dc: u0 - dc*kChunkD - kChunkD + 1
  chunk_load<MASK>(cur, rowR, la, lb, qa, qb, has_a, has_b, W, nw, u0 - kChunkD + 1, 0, lane);
  chunk_store_window(cur, cwin, lane);
  __syncthreads();

  for (int s = 0; s < steps; ++s) {
    const int dci = s / nwc, wci = s - dci * nwc;
    const int dc0 = dci * kChunkD;
    if (wci == 0) {
#pragma unroll
      for (int i = 0; i < kChunkD; ++i) ca[i] = cb[i] = 0;
    }
    if (s + 1 < steps) {  // prefetch step s + 1
      const int dn = (s + 1) / nwc, wn = (s + 1) - dn * nwc;
      chunk_load<MASK>(next, rowR, la, lb, qa, qb, has_a, has_b, W, nw,
                       u0 - dn * kChunkD - kChunkD + 1, wn * kChunkWords, lane);
    }
    const ulonglong2 *buf = cwin + (s & 1) * kBuf;
#pragma unroll
    for (int h = 0; h < kChunkPairs; ++h) {
      const ulonglong2 *ww = buf + h * 2 * kChunkHP;
      const uint64_t la0 = cur.la[2 * h], la1 = cur.la[2 * h + 1];
      const uint64_t lb0 = cur.lb[2 * h], lb1 = cur.lb[2 * h + 1];
      const uint64_t ma0 = cur.ma[2 * h], ma1 = cur.ma[2 * h + 1];
      const uint64_t mb0 = cur.mb[2 * h], mb1 = cur.mb[2 * h + 1];
      {
        const int rel = 2 * lane + kChunkD;  // right pixel b - dc0
        const ulonglong2 br = ww[(rel & 1) * kChunkHP + (rel >> 1)];
        cb[0] = masked_cost1(lb1, mb1, br.y, MASK, masked_cost1(lb0, mb0, br.x, MASK, cb[0]));
      }
#pragma unroll
      for (int i = 0; i < kChunkD; ++i) {
        const int rel = 2 * lane + (kChunkD - 1 - i);  // right pixel a - (dc0 + i)
        const ulonglong2 br = ww[(rel & 1) * kChunkHP + (rel >> 1)];
        ca[i] = masked_cost1(la1, ma1, br.y, MASK, masked_cost1(la0, ma0, br.x, MASK, ca[i]));
        if (i + 1 < kChunkD)
          cb[i + 1] =
              masked_cost1(lb1, mb1, br.y, MASK, masked_cost1(lb0, mb0, br.x, MASK, cb[i + 1]));
      }
    }
    if (wci == nwc - 1) {  // the disparity chunk is complete
      const int nd = min(kChunkD, dmax - dc0);
#pragma unroll
      for (int i = 0; i < kChunkD; ++i) {
        if (i < nd) {
          const int d = dc0 + i;
          const bool va = a - d >= 0, vb = b - d >= 0;
          if (va) best_a = min(best_a, (ca[i] << 16) | (uint32_t)d);
          if (vb) best_b = min(best_b, (cb[i] << 16) | (uint32_t)d);
          if (VOL) {
            int16_t *plane = cost + ((size_t)d * H + v) * W;
            const uint32_t sa = va ? ca[i] : (uint32_t)kInvalidCost;
            const uint32_t sb = vb ? cb[i] : (uint32_t)kInvalidCost;
            if (has_b && ((((size_t)d * H + v) * W) & 1) == 0) {
              *reinterpret_cast<uint32_t *>(plane + a) = sa | (sb << 16);
            } else {
              if (has_a) plane[a] = (int16_t)sa;
              if (has_b) plane[b] = (int16_t)sb;
            }
          }
        }
      }
    }
    if (s + 1 < steps) {
      // the other buffer was last read in step s - 1, which every lane of
      // this one-wave workgroup has finished
      chunk_store_window(next, cwin + ((s + 1) & 1) * kBuf, lane);
      cur = next;
      __syncthreads();
    }
  }
  if (has_a) disp[(size_t)v * W + a] = (int32_t)(best_a & 0xffffu);
  if (has_b) disp[(size_t)v * W + b] = (int32_t)(best_b & 0xffffu);
}

// ===========================================================================
// Voting refinement (Eq. 9-10) of the pixels the left/right check marked
// invalid.  One wave per pixel: the lanes walk the (2 radius + 1)^2 window
// 64 positions at a time, and every valid pixel p brings its bilateral
// weight exp(-(c / lambda_c + e / lambda_e)) (c: Euclidean distance of the
// Lab8 colours, e: of the positions) as a vote for its disparity.  Within
// one step the votes for one d are summed by a fixed butterfly over the
// lanes (zeros from lanes voting for another d), taking the step's d values
// in the order of their lowest lane, and one lane adds the sum to the
// wave's histogram bin in LDS.  Every bin thus receives its votes in the
// same order on every run, so the fp32 sums, and the argmax, are
// deterministic.  The wave then takes the largest vote, the lowest d among
// equal votes.  A pixel without voters keeps its fallback disparity; valid
// pixels keep theirs.
// ===========================================================================
constexpr int kVoteWaves = 4;

__global__ __launch_bounds__(64 * kVoteWaves) void k_vote_refine(
    const uint32_t *__restrict__ packed, const int32_t *__restrict__ checked,
    const int32_t *__restrict__ fallback, int W, int H, int dmax, int radius, float lambda_c,
    float lambda_e, int32_t *__restrict__ out) {
  extern __shared__ float votes[];  // [kVoteWaves][dmax]
  const int lane = threadIdx.x & 63, wave = wave_index();
  const long long x = (long long)blockIdx.x * kVoteWaves + wave;
  const bool live = x < (long long)W * H;
  const int u = live ? (int)(x % W) : 0, v = live ? (int)(x / W) : 0;
  const int own = live ? checked[x] : 0;
  const bool refine = live && own < 0;  // wave-uniform
  float *hist = votes + wave * dmax;
  if (refine)
    for (int d = lane; d < dmax; d += 64) hist[d] = 0.0f;
  __syncthreads();
  bool voted = false;
  if (refine) {
    const uint32_t cx = packed[x];
    const int side = 2 * radius + 1, area = side * side;
    for (int base = 0; base < area; base += 64) {
      const int i = base + lane;
      int d = -1;
      float wgt = 0.0f;
      if (i < area) {
        const int dy = i / side - radius, dx = i % side - radius;
        const int pu = u + dx, pv = v + dy;
        if (pu >= 0 && pu < W && pv >= 0 && pv < H) {
          const size_t p = (size_t)pv * W + pu;
          const int dp = checked[p];
          if (dp >= 0 && dp < dmax) {
            const uint32_t cp = packed[p];
            const float dl = (float)(int)(cx & 0xff) - (float)(int)(cp & 0xff);
            const float da = (float)(int)((cx >> 8) & 0xff) - (float)(int)((cp >> 8) & 0xff);
            const float db = (float)(int)((cx >> 16) & 0xff) - (float)(int)((cp >> 16) & 0xff);
            const float c = sqrtf(dl * dl + da * da + db * db);
            const float e = sqrtf((float)(dx * dx + dy * dy));
            d = dp;
            wgt = expf(-(c / lambda_c + e / lambda_e));
          }
        }
      }
      unsigned long long pending = __ballot(d >= 0);
      if (pending) voted = true;
      while (pending) {  // uniform
        const int leader = __builtin_ctzll(pending);
        const int dl = __shfl(d, leader);
        const bool mine = d == dl;
        float sum = mine ? wgt : 0.0f;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane == 0) hist[dl] += sum;  // the bin's only writer
        pending &= ~__ballot(mine);
      }
    }
  }
  __syncthreads();
  if (!refine) {
    if (live && lane == 0) out[x] = own;
    return;
  }
  float best = -1.0f;
  int best_d = 0;
  for (int d = lane; d < dmax; d += 64) {
    const float w = hist[d];
    if (w > best) {  // ascending d: keeps the lowest d among equal votes
      best = w;
      best_d = d;
    }
  }
#pragma unroll
  for (int sft = 32; sft >= 1; sft >>= 1) {
    const float ow = __shfl_xor(best, sft);
    const int od = __shfl_xor(best_d, sft);
    if (ow > best || (ow == best && od < best_d)) {
      best = ow;
      best_d = od;
    }
  }
  if (lane == 0) out[x] = voted ? best_d : fallback[x];
}

// ===========================================================================
// Persistent batch kernels.  Every stage kernel loops: a workgroup takes the
// next tile index of its queue with one atomic add, finds the pair that owns
// it (binary search over per-pair prefix sums; pairs are listed largest work
// first) and runs the same per-tile function as the single-pair kernels.
// Stages run one after another on the stream, so a stage only reads what the
// previous stages completed; no workgroup ever waits for another.
// ===========================================================================

// Largest i in [0, npairs) with start[i] <= t (start[npairs] > t).
__device__ __forceinline__ int owner(const int *start, int npairs, int t) {
  int lo = 0, hi = npairs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Queue head read coherently across the XCDs.  Heads only grow during a
// stage, so a head at or past a queue's length proves the queue drained and
// spares the atomic that would only confirm it (every workgroup ends each
// queue it visits with such a pull, on one counter).
__device__ __forceinline__ int queue_head(int *counter) {
  return __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A workgroup's pulls from one queue of `total` items (thread 0 pulls; the
// value goes to every thread through LDS and is uniform, so everything
// derived from it stays in scalar registers).  While at least a grid's
// worth of items lies beyond the current one, the next item is claimed when
// the current one starts, so the atomic's round trip overlaps the work;
// near the end of the queue pulls wait for the current item, so that no
// item waits behind a busy workgroup while others idle.
struct WgQueue {
  int *counter;
  int total;
  int *slot;
  int claimed;  // thread 0: item claimed ahead, or -1
  // First pull; `check` first reads the head (a queue likely drained).
  __device__ __forceinline__ int first(bool check) {
    int v = 0;
    if (threadIdx.x == 0) {
      const int h = check ? queue_head(counter) : 0;
      v = h >= total ? h : atomicAdd(counter, 1);
    }
    return publish(v);
  }
  // Called when item `cur` starts.
  __device__ __forceinline__ void begin(int cur) {
    claimed = -1;
    if (threadIdx.x == 0 && cur + static_cast<int>(gridDim.x) < total)
      claimed = atomicAdd(counter, 1);
  }
  // Called when the current item is done: the next item.
  __device__ __forceinline__ int next() {
    int v = 0;
    if (threadIdx.x == 0) v = claimed >= 0 ? claimed : atomicAdd(counter, 1);
    return publish(v);
  }
  __device__ __forceinline__ int publish(int v) {
    __syncthreads();  // everyone has read the previous value
    if (threadIdx.x == 0) *slot = v;
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
  }
};

__global__ void k_batch_reset(int *counters) {
  if (threadIdx.x < kBatchQueues) counters[threadIdx.x * kCounterStride] = 0;
}

__global__ __launch_bounds__(kColorThreads) void k_batch_color(const BatchWork *__restrict__ bw,
                                                               const uint16_t *__restrict__ lin,
                                                               const uint16_t *__restrict__ ftab,
                                                               Mq mq, int use_mask) {
  __shared__ int slot;
  const int *start = bw->start + kQueueColor * (bw->npairs + 1);
  WgQueue qu{bw->counters + kQueueColor * kCounterStride, uniform(start[bw->npairs]), &slot, -1};
  for (int t = qu.first(false); t < qu.total; t = qu.next()) {
    qu.begin(t);
    const int i = uniform(owner(start, bw->npairs, t));
    const BatchPair &p = bw->pairs[bw->order[i]];
    const int tx = (p.W + kColorTX - 1) / kColorTX;
    const int ty = (p.H + kBatchColorTY - 1) / kBatchColorTY;
    const int local = t - start[i], view = local / (tx * ty), tile = local % (tx * ty);
    color_tile<kBatchColorRPT>(view ? p.right : p.left, p.W, p.H, p.stride,
                               view ? p.packedR : p.packedL, lin, ftab, mq,
                               view == 0 && use_mask, 0, (tile % tx) * kColorTX,
                               (tile / tx) * kBatchColorTY);
  }
}

// Both describe stages of a batch in one persistent launch.  One workgroup
// in `right_every` starts on the descriptor-only queue, the others on the
// describe+mask queue, and each turns to the other queue when its own is
// empty: the LDS-bound descriptor-only tiles and the issue-bound
// describe+mask tiles share the CUs instead of following each other.
template <int NW, int TW, int TH>
__global__ __launch_bounds__(kDescThreads, 4) void k_batch_describe(
    const BatchWork *__restrict__ bw, DescribeConsts cm, RightConsts cr, int right_every) {
  static_assert(kDescThreads == kRightThreads, "one workgroup shape for both stages");
  extern __shared__ uint32_t dlds[];
  __shared__ int slot, row_next;
  const int n = bw->npairs;
  const bool right_first = blockIdx.x % right_every == 0;
  for (int phase = 0; phase < 2; ++phase) {
    if ((phase == 0) == right_first) {
      const int *start = bw->start + kQueueDescribe * (n + 1);
      WgQueue qu{bw->counters + kQueueDescribe * kCounterStride, uniform(start[n]), &slot, -1};
      if (qu.total == 0) continue;
      for (int t = qu.first(phase == 1); t < qu.total; t = qu.next()) {
        qu.begin(t);
        const int i = uniform(owner(start, n, t));
        const BatchPair &p = bw->pairs[bw->order[i]];
        const int W = uniform(p.W), H = uniform(p.H);
        const int tx = (W + kRightTW - 1) / kRightTW, ty = (H + kRightTH - 1) / kRightTH;
        const int local = t - start[i], view = local / (tx * ty), tile = local % (tx * ty);
        // view 0 is the right view; view 1 (mask off only) the left view
        describe_right_tile<kRightPx, NW % kRightRegWords == 0>(reinterpret_cast<uint8_t *>(dlds),
                                      uniform(view ? p.packedL : p.packedR), W, H, cr,
                                      uniform(view ? p.descL : p.descR),
                                      uniform((tile % tx) * kRightTW),
                                      uniform((tile / tx) * kRightTH));
      }
    } else {
      const int *start = bw->start + kQueueDescribeMask * (n + 1);
      WgQueue qu{bw->counters + kQueueDescribeMask * kCounterStride, uniform(start[n]), &slot, -1};
      if (qu.total == 0) continue;
      for (int t = qu.first(phase == 1); t < qu.total; t = qu.next()) {
        qu.begin(t);
        const int i = uniform(owner(start, n, t));
        const BatchPair &p = bw->pairs[bw->order[i]];
        const int W = uniform(p.W), H = uniform(p.H);
        const int tx = (W + TW - 1) / TW;
        const int local = t - start[i];
        // offsets in registers, per tile, so that they hold none during
        // descriptor-only tiles
        const RegOffsets<NW> off(cm, threadIdx.x & 63);
        describe_mask_tile<NW, TW, TH, true>(dlds, &row_next, uniform(p.packedL), W, H, cm, off,
                                             uniform(p.descL), uniform(p.maskL),
                                             uniform((local % tx) * TW),
                                             uniform((local / tx) * TH));
      }
    }
  }
}

// Pulls of one wave on its own (no barrier): lane 0 adds.  claim() starts a
// pull and returns lane 0's pending value; value() makes it the wave's,
// waiting for the atomic only then, so a pull started before an item's work
// overlaps it.
__device__ __forceinline__ int wave_claim(int *counter) {
  int t = 0;
  if ((threadIdx.x & 63) == 0) t = atomicAdd(counter, 1);
  return t;
}
__device__ __forceinline__ int wave_value(int claimed) {
  return __builtin_amdgcn_readfirstlane(claimed);
}
// A queue a wave visits after its own: drained when its head has reached
// its length.
__device__ __forceinline__ bool wave_drained(int *counter, int total) {
  int h = 0;
  if ((threadIdx.x & 63) == 0) h = queue_head(counter);
  return __builtin_amdgcn_readfirstlane(h) >= total;
}

// Cost tiles.  Queue x (one per XCD) holds the tiles of the rows v = x mod 8
// of every pair; a workgroup serves the queue of its own XCD first (so a
// row's tiles share one L2) and then helps the others.  Pairs with and
// without a cost volume have their own queues and kernels.  The next item is
// claimed before the current tile runs, so the atomic's latency is hidden,
// and the owning pair is looked up again only when an item leaves it.
template <int NW, int DC, bool MASK, bool VOL>
__global__ __launch_bounds__(64, 2) void k_batch_cost(const BatchWork *__restrict__ bw) {
  extern __shared__ uint64_t win[];
  const int home = blockIdx.x % kXcds;
  const int n = bw->npairs;
  for (int qi = 0; qi < kXcds; ++qi) {
    const int x = (home + qi) % kXcds;
    const int q = (VOL ? kQueueCostVol0 : kQueueCost0) + x;
    const int *start = bw->start + q * (n + 1);
    const int total = start[n];
    int *counter = bw->counters + q * kCounterStride;
    if (total == 0 || (qi > 0 && wave_drained(counter, total))) continue;
    int cur = wave_value(wave_claim(counter));
    int i = 0, i_end = -1;  // pair of the last item and the end of its range
    while (cur < total) {
      const int next = wave_claim(counter);
      if (cur >= i_end || cur < start[i]) {
        i = owner(start, n, cur);
        i_end = start[i + 1];
      }
      const BatchPair &p = bw->pairs[bw->order[i]];
      const int tiles = (p.W + kCostTX - 1) / kCostTX;
      const int local = cur - start[i];
      cost_tile<NW, DC, MASK, VOL>(win, p.descL, p.maskL, p.descR, p.W, p.H, p.dmax, p.disp,
                                   p.cost, x + kXcds * (local / tiles),
                                   (local % tiles) * kCostTX);
      cur = wave_value(next);
    }
  }
}

// The no-volume cost queues on the matrix cores.  An item is one 32-pixel
// row tile, and each wave pulls items on its own: the waves of a workgroup
// share nothing, so they never wait for one another at a barrier.  The
// next item is claimed before the current one runs.  Bounded to three waves
// per SIMD (168 registers, nothing spilled to memory), which hide more of
// each block's chain of dependent products than two.
template <int NW, bool MASK>
__global__ __launch_bounds__(64 * kMfmaWaves, 3) void k_batch_cost_mfma(
    const BatchWork *__restrict__ bw) {
  const int home = blockIdx.x % kXcds;
  const int n = bw->npairs;
  for (int qi = 0; qi < kXcds; ++qi) {
    const int x = (home + qi) % kXcds;
    const int q = kQueueCost0 + x;
    const int *start = bw->start + q * (n + 1);
    const int total = start[n];
    int *counter = bw->counters + q * kCounterStride;
    if (total == 0 || (qi > 0 && wave_drained(counter, total))) continue;
    int cur = wave_value(wave_claim(counter));
    int i = 0, i_end = -1;  // pair of the last item and the end of its range
    while (cur < total) {
      const int next = wave_claim(counter);
      if (cur >= i_end || cur < start[i]) {
        i = owner(start, n, cur);
        i_end = start[i + 1];
      }
      const BatchPair &p = bw->pairs[bw->order[i]];
      const int W = uniform(p.W);
      const int tiles = (W + kMfmaTX - 1) / kMfmaTX;
      const int local = cur - start[i];
      const int v = x + kXcds * (local / tiles);
      cost_tile_mfma<NW, MASK>(uniform(p.descL), uniform(p.maskL), uniform(p.descR), W,
                               uniform(p.H), uniform(p.dmax), uniform(p.disp), nullptr, nullptr,
                               v, (local % tiles) * kMfmaTX);
      cur = wave_value(next);
    }
  }
}

// ===========================================================================
// Launchers
// ===========================================================================
DescribeConsts describe_consts(const DeviceTables &t) {
  return DescribeConsts{t.pattern, t.nw, t.radius, t.left_pitch_for(t.tune.desc_tile_w), t.k, 0};
}

RightConsts right_consts(const DeviceTables &t) {
  return RightConsts{t.right_offs, t.n, t.nw, t.radius, t.right_pitch};
}

// LDS of a describe+mask tile (TH + 2 radius rows at the tile pitch).
size_t mask_tile_bytes(const DeviceTables &t, int tw, int th) {
  return (size_t)(th + 2 * t.radius) * t.left_pitch_for(tw) * sizeof(uint32_t);
}

size_t round16(size_t x) { return (x + 15) / 16 * 16; }

template <int NW, int TW>
hipError_t launch_describe_mask_t(const uint32_t *packed, int W, int H, const DeviceTables &t,
                                  uint64_t *desc, uint64_t *mask, hipStream_t s) {
  DescribeConsts c = describe_consts(t);
  c.pitch = t.left_pitch_for(TW);
  const long long tall_tiles = (long long)((W + TW - 1) / TW) * ((H + kDescTH - 1) / kDescTH);
  const bool tall = t.tune.pair_desc_th ? t.tune.pair_desc_th == kDescTH
                                        : tall_tiles >= kDescTallMinTiles;
  const int th = tall ? kDescTH : kDescTHSmall;
  c.table_off = static_cast<int>(round16(mask_tile_bytes(t, TW, th)));
  const size_t lds = c.table_off + pair_table_bytes<NW>();
  dim3 grid((W + TW - 1) / TW, (H + th - 1) / th);
  if (tall)
    hipLaunchKernelGGL((k_describe_mask<NW, TW, kDescTH>), grid, dim3(kDescThreads), lds, s,
                       packed, W, H, c, desc, mask);
  else
    hipLaunchKernelGGL((k_describe_mask<NW, TW, kDescTHSmall>), grid, dim3(kDescThreads), lds,
                       s, packed, W, H, c, desc, mask);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_describe_mask_nw(const uint32_t *packed, int W, int H, const DeviceTables &t,
                                   uint64_t *desc, uint64_t *mask, hipStream_t s) {
  return t.tune.desc_tile_w == 32
             ? launch_describe_mask_t<NW, 32>(packed, W, H, t, desc, mask, s)
             : launch_describe_mask_t<NW, 16>(packed, W, H, t, desc, mask, s);
}

// Raises a kernel's dynamic LDS limit above the 64 KiB default.  The describe
// kernels need at most ~75 KiB (n = 4096, S = 63); 128 KiB leaves room for the
// kernels' static LDS within the 160 KiB of a workgroup.
hipError_t allow_big_lds(const void *kernel) {
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
}

template <int NW, int DC>
hipError_t launch_cost_fast_dc(const uint64_t *descL, const uint64_t *maskL,
                               const uint64_t *descR, int W, int H, int dmax, int32_t *disp,
                               int16_t *cost, hipStream_t s) {
  const int tiles = (W + kCostTX - 1) / kCostTX;
  dim3 grid(kXcds * tiles * ((H + kXcds - 1) / kXcds));
  const size_t lds = Window<NW, DC>::kBytes;
#define BSM_LAUNCH_COST(M, V)                                                                  \
  hipLaunchKernelGGL((k_cost_wta_fast<NW, DC, M, V>), grid, dim3(64), lds, s, descL, maskL, \
                     descR, W, H, dmax, disp, cost)
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

template <int NW>
hipError_t launch_cost_mfma(const uint64_t *descL, const uint64_t *maskL, const uint64_t *descR,
                            int W, int H, int dmax, int32_t *disp, int16_t *cost, hipStream_t s) {
  const int rows = (H + kXcds - 1) / kXcds;  // rows per XCD
  if (cost) {
    const int tiles = (W + kMfmaTX - 1) / kMfmaTX;  // a wave per tile
    const dim3 grid(kXcds * ((tiles + kMfmaWaves - 1) / kMfmaWaves) * rows);
    static const hipError_t attr[2] = {
        allow_big_lds(reinterpret_cast<const void *>(k_cost_wta_mfma_vol<NW, false>)),
        allow_big_lds(reinterpret_cast<const void *>(k_cost_wta_mfma_vol<NW, true>))};
    if (attr[0] != hipSuccess) return attr[0];
    if (attr[1] != hipSuccess) return attr[1];
    const size_t lds = (size_t)kMfmaWaves * dmax * kSlabPitch * sizeof(int16_t);
    if (maskL)
      hipLaunchKernelGGL((k_cost_wta_mfma_vol<NW, true>), grid, dim3(64 * kMfmaWaves), lds, s,
                         descL, maskL, descR, W, H, dmax, disp, cost);
    else
      hipLaunchKernelGGL((k_cost_wta_mfma_vol<NW, false>), grid, dim3(64 * kMfmaWaves), lds, s,
                         descL, maskL, descR, W, H, dmax, disp, cost);
    return hipGetLastError();
  }
  const int duos = (W + 2 * kMfmaTX - 1) / (2 * kMfmaTX);  // a wave per two tiles
  const dim3 grid(kXcds * ((duos + kMfmaWaves - 1) / kMfmaWaves) * rows);
  if (maskL)
    hipLaunchKernelGGL((k_cost_wta_mfma<NW, true>), grid, dim3(64 * kMfmaWaves), 0, s, descL,
                       maskL, descR, W, H, dmax, disp);
  else
    hipLaunchKernelGGL((k_cost_wta_mfma<NW, false>), grid, dim3(64 * kMfmaWaves), 0, s, descL,
                       maskL, descR, W, H, dmax, disp);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_cost_fast(const uint64_t *descL, const uint64_t *maskL, const uint64_t *descR,
                            int W, int H, int dmax, int32_t *disp, int16_t *cost, int dc,
                            hipStream_t s) {
  return dc == 32 ? launch_cost_fast_dc<NW, 32>(descL, maskL, descR, W, H, dmax, disp, cost, s)
                  : launch_cost_fast_dc<NW, 64>(descL, maskL, descR, W, H, dmax, disp, cost, s);
}

// Persistent grid: `per_cu` workgroups per CU (0: as many as fit), rounded
// to a multiple of the XCD count.
template <typename K>
int persistent_grid(K kernel, int threads, size_t lds, int per_cu) {
  int dev = 0, cus = 0, fit = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, reinterpret_cast<const void *>(kernel),
                                                     threads, lds);
  if (cus < 1) cus = 256;
  if (fit < 1) fit = 1;
  const int k = per_cu > 0 ? std::min(per_cu, fit) : fit;
  return std::max(kXcds, (cus * k + kXcds - 1) / kXcds * kXcds);
}

template <int NW, int TW, int TH, int DC>
hipError_t launch_batch_t(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                          hipStream_t s) {
  const Tuning &tu = t.tune;
  const BatchWork *bw = bl.work;
  // Optional stage marks (eager launches): before the colour stage and
  // after each stage.
  auto mark = [&](int i) -> hipError_t {
    return bl.marks ? hipEventRecord(bl.marks[i], s) : hipSuccess;
  };
  hipError_t me;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, bl.counters);
  if ((me = mark(0)) != hipSuccess) return me;
  const int g0 = persistent_grid(k_batch_color, kColorThreads, 0, tu.blocks_per_cu[0]);
  hipLaunchKernelGGL(k_batch_color, dim3(g0), dim3(kColorThreads), 0, s, bw, t.lin, t.f,
                     t.mq, use_mask);
  if ((me = mark(1)) != hipSuccess) return me;
  {
    // both describe stages (the describe+mask queue is empty without a mask)
    static const hipError_t attr =
        allow_big_lds(reinterpret_cast<const void *>(k_batch_describe<NW, TW, TH>));
    if (attr != hipSuccess) return attr;
    DescribeConsts cm = describe_consts(t);
    cm.pitch = t.left_pitch_for(TW);
    const size_t lds = std::max(mask_tile_bytes(t, TW, TH),
                                right_lds_bytes(kRightPx, t.radius, t.right_pitch));
    const int g1 = persistent_grid(k_batch_describe<NW, TW, TH>, kDescThreads, lds,
                                   tu.blocks_per_cu[1]);
    const int right_every = tu.blocks_per_cu[2] > 0 ? tu.blocks_per_cu[2] : kDescRightEvery;
    hipLaunchKernelGGL((k_batch_describe<NW, TW, TH>), dim3(g1), dim3(kDescThreads), lds, s, bw,
                       cm, right_consts(t), use_mask ? right_every : 1);
  }
  if ((me = mark(2)) != hipSuccess) return me;
  {
    // pairs without a volume, then pairs with one (each kernel's queues are
    // empty when the batch has no pair of its kind)
    const size_t lds = Window<NW, DC>::kBytes;
#define BSM_LAUNCH_BATCH_COST(M, V)                                                          \
  do {                                                                                       \
    const int g3 = persistent_grid(k_batch_cost<NW, DC, M, V>, 64, lds, tu.blocks_per_cu[3]); \
    hipLaunchKernelGGL((k_batch_cost<NW, DC, M, V>), dim3(g3), dim3(64), lds, s, bw);        \
  } while (0)
#define BSM_LAUNCH_BATCH_COST_MFMA(M)                                                          \
  do {                                                                                        \
    const int g3 = persistent_grid(k_batch_cost_mfma<NW, M>, 64 * kMfmaWaves, 0,            \
                                   tu.blocks_per_cu[3]);                                        \
    hipLaunchKernelGGL((k_batch_cost_mfma<NW, M>), dim3(g3), dim3(64 * kMfmaWaves), 0, s, bw); \
  } while (0)
    if (use_mask) {
      if (tu.cost_mfma) BSM_LAUNCH_BATCH_COST_MFMA(true);
      else BSM_LAUNCH_BATCH_COST(true, false);
      if ((me = mark(3)) != hipSuccess) return me;
      BSM_LAUNCH_BATCH_COST(true, true);
    } else {
      if (tu.cost_mfma) BSM_LAUNCH_BATCH_COST_MFMA(false);
      else BSM_LAUNCH_BATCH_COST(false, false);
      if ((me = mark(3)) != hipSuccess) return me;
      BSM_LAUNCH_BATCH_COST(false, true);
    }
    if ((me = mark(4)) != hipSuccess) return me;
#undef BSM_LAUNCH_BATCH_COST
#undef BSM_LAUNCH_BATCH_COST_MFMA
  }
  return hipGetLastError();
}

template <int NW, int TW, int TH>
hipError_t launch_batch_th(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                           hipStream_t s) {
  return t.tune.cost_dchunk == 32 ? launch_batch_t<NW, TW, TH, 32>(bl, t, use_mask, s)
                                  : launch_batch_t<NW, TW, TH, 64>(bl, t, use_mask, s);
}

template <int NW, int TW>
hipError_t launch_batch_tw(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                           hipStream_t s) {
  return t.tune.batch_tile_h == 8 ? launch_batch_th<NW, TW, 8>(bl, t, use_mask, s)
                                  : launch_batch_th<NW, TW, 16>(bl, t, use_mask, s);
}

template <int NW>
hipError_t launch_batch_nw(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                           hipStream_t s) {
  return t.tune.desc_tile_w == 32 ? launch_batch_tw<NW, 32>(bl, t, use_mask, s)
                                  : launch_batch_tw<NW, 16>(bl, t, use_mask, s);
}

}  // namespace

int describe_left_cols(int radius, int tile_w) { return tile_w + 2 * radius; }
// Row pitch (bytes) of the intensity tile: halo rounded up to 4, the tile,
// the right halo and one dword of slack for the funnel reads, rounded to 4.
int describe_right_cols(int radius) {
  return (right_halo(radius) + kRightTW + radius + 4 + 3) / 4 * 4;
}

void batch_tile_counts(int W, int H, int use_mask, int want_cost, int desc_tile_w,
                       int desc_tile_h, int cost_mfma, int counts[kBatchQueues]) {
  counts[kQueueColor] =
      2 * ((W + kColorTX - 1) / kColorTX) * ((H + kBatchColorTY - 1) / kBatchColorTY);
  counts[kQueueDescribeMask] =
      use_mask ? ((W + desc_tile_w - 1) / desc_tile_w) * ((H + desc_tile_h - 1) / desc_tile_h)
               : 0;
  counts[kQueueDescribe] =
      (use_mask ? 1 : 2) * ((W + kRightTW - 1) / kRightTW) * ((H + kRightTH - 1) / kRightTH);
  // The bitwise kernels take 128-pixel items; the matrix-core kernel takes
  // single 32-pixel tiles, so that the rows open at once on an XCD (whose
  // right descriptors its L2 must hold) are as few as in one pair's launch.
  const int tiles = (W + kCostTX - 1) / kCostTX;
  const int cost_tiles = cost_mfma ? (W + kMfmaTX - 1) / kMfmaTX : tiles;
  for (int x = 0; x < kXcds; ++x) {
    const int rows = H > x ? (H - x + kXcds - 1) / kXcds : 0;
    counts[kQueueCost0 + x] = want_cost ? 0 : cost_tiles * rows;
    counts[kQueueCostVol0 + x] = want_cost ? tiles * rows : 0;
  }
}

bool batch_supported(int nw) { return nw == 1 || nw == 2 || nw == 4 || nw == 8 || nw == 16; }

hipError_t launch_color(const uint8_t *img, int W, int H, int stride, uint32_t *packed,
                        int want_lab, int mirror, const DeviceTables &t, hipStream_t s) {
  dim3 grid((W + kColorTX - 1) / kColorTX, (H + kColorTY - 1) / kColorTY);
  hipLaunchKernelGGL(k_color, grid, dim3(kColorThreads), 0, s, img, W, H, stride, packed, t.lin,
                     t.f, t.mq, want_lab, mirror);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reverse_rows_t(T *data, int W, int rows, hipStream_t s) {
  if (W < 2 || rows < 1) return hipSuccess;
  const int ry = rows < 65535 ? rows : 65535;
  dim3 grid((W / 2 + 255) / 256, ry, (rows + 65534) / 65535);
  hipLaunchKernelGGL(k_reverse_rows<T>, grid, dim3(256), 0, s, data, W, rows);
  return hipGetLastError();
}

hipError_t launch_reverse_rows(int32_t *data, int W, int rows, hipStream_t s) {
  return launch_reverse_rows_t(data, W, rows, s);
}

hipError_t launch_reverse_rows(int16_t *data, int W, int rows, hipStream_t s) {
  return launch_reverse_rows_t(data, W, rows, s);
}

hipError_t launch_vote_refine(const uint32_t *packed, const int32_t *checked,
                              const int32_t *fallback, int W, int H, int dmax, int radius,
                              float lambda_c, float lambda_e, int32_t *out, hipStream_t s) {
  const long long px = (long long)W * H;
  dim3 grid((unsigned)((px + kVoteWaves - 1) / kVoteWaves));
  hipLaunchKernelGGL(k_vote_refine, grid, dim3(64 * kVoteWaves),
                     (size_t)kVoteWaves * dmax * sizeof(float), s, packed, checked, fallback, W, H,
                     dmax, radius, lambda_c, lambda_e, out);
  return hipGetLastError();
}

hipError_t launch_lr_check(const int32_t *dL, const int32_t *dR, int W, int H, int tol,
                           int32_t *out, hipStream_t s) {
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(k_lr_check, grid, dim3(256), 0, s, dL, dR, W, H, tol, out);
  return hipGetLastError();
}

hipError_t launch_describe(const uint32_t *packed, int W, int H, const DeviceTables &t,
                           uint64_t *desc, uint64_t *mask, hipStream_t s) {
  if (!mask) {
    static const hipError_t attr[4] = {
        allow_big_lds(reinterpret_cast<const void *>(k_describe_right<1, true>)),
        allow_big_lds(reinterpret_cast<const void *>(k_describe_right<1, false>)),
        allow_big_lds(reinterpret_cast<const void *>(k_describe_right<kRightPx, true>)),
        allow_big_lds(reinterpret_cast<const void *>(k_describe_right<kRightPx, false>))};
    for (hipError_t a : attr)
      if (a != hipSuccess) return a;
    const int rows = (H + kRightTH - 1) / kRightTH;
    const int wide = (W + kRightTW - 1) / kRightTW;
    const bool four = t.tune.pair_right_px ? t.tune.pair_right_px == kRightPx
                                           : (long long)wide * rows >= kRightWideMinBlocks;
    const RightConsts rc = right_consts(t);
    if (four) {
      const size_t lds = right_lds_bytes(kRightPx, t.radius, t.right_pitch);
      if (t.nw % kRightRegWords == 0)
        hipLaunchKernelGGL((k_describe_right<kRightPx, true>), dim3(wide, rows),
                           dim3(kRightThreads), lds, s, packed, W, H, rc, desc);
      else
        hipLaunchKernelGGL((k_describe_right<kRightPx, false>), dim3(wide, rows),
                           dim3(kRightThreads), lds, s, packed, W, H, rc, desc);
    } else {
      const size_t lds = right_lds_bytes(1, t.radius, t.right_pitch);
      const dim3 grid((W + 63) / 64, rows);
      if (t.nw % kRightGroup == 0)
        hipLaunchKernelGGL((k_describe_right<1, true>), grid, dim3(kRightThreads), lds, s,
                           packed, W, H, rc, desc);
      else
        hipLaunchKernelGGL((k_describe_right<1, false>), grid, dim3(kRightThreads), lds, s,
                           packed, W, H, rc, desc);
    }
    return hipGetLastError();
  }
  if (t.nw <= 1) return launch_describe_mask_nw<1>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 2) return launch_describe_mask_nw<2>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 4) return launch_describe_mask_nw<4>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 8) return launch_describe_mask_nw<8>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 16) return launch_describe_mask_nw<16>(packed, W, H, t, desc, mask, s);
  if (t.nw <= 32) return launch_describe_mask_nw<32>(packed, W, H, t, desc, mask, s);
  return launch_describe_mask_nw<64>(packed, W, H, t, desc, mask, s);
}

hipError_t launch_cost_wta(const uint64_t *descL, const uint64_t *maskL, const uint64_t *descR,
                           int W, int H, int nw, int dmax, int32_t *disp, int16_t *cost,
                           const DeviceTables &t, hipStream_t s) {
  const int dc = t.tune.cost_dchunk;
  // Matrix-core kernel, except for short disparity ranges (a tile computes
  // at least two 32-wide blocks, most of them wasted when dmax <= 16).
  if (t.tune.cost_mfma && dmax >= t.tune.mfma_min_dmax && (!cost || dmax <= kMfmaVolMaxD)) {
    switch (nw) {
      case 1: return launch_cost_mfma<1>(descL, maskL, descR, W, H, dmax, disp, cost, s);
      case 2: return launch_cost_mfma<2>(descL, maskL, descR, W, H, dmax, disp, cost, s);
      case 4: return launch_cost_mfma<4>(descL, maskL, descR, W, H, dmax, disp, cost, s);
      case 8: return launch_cost_mfma<8>(descL, maskL, descR, W, H, dmax, disp, cost, s);
      case 16: return launch_cost_mfma<16>(descL, maskL, descR, W, H, dmax, disp, cost, s);
      default: break;
    }
  }
  if (t.tune.cost_mfma && !cost && nw > kLongPassWords && nw % kLongPassWords == 0 &&
      dmax >= t.tune.mfma_min_dmax && dmax <= kLongMaxDmax) {
    const int tiles = (W + kMfmaTX - 1) / kMfmaTX;
    const int groups = (tiles + kMfmaWaves - 1) / kMfmaWaves;
    dim3 grid(kXcds * groups * ((H + kXcds - 1) / kXcds));
    if (maskL)
      hipLaunchKernelGGL((k_cost_wta_mfma_long<true>), grid, dim3(64 * kMfmaWaves), 0, s, descL,
                         maskL, descR, W, H, nw, dmax, disp);
    else
      hipLaunchKernelGGL((k_cost_wta_mfma_long<false>), grid, dim3(64 * kMfmaWaves), 0, s, descL,
                         maskL, descR, W, H, nw, dmax, disp);
    return hipGetLastError();
  }
  switch (nw) {
    case 1: return launch_cost_fast<1>(descL, maskL, descR, W, H, dmax, disp, cost, dc, s);
    case 2: return launch_cost_fast<2>(descL, maskL, descR, W, H, dmax, disp, cost, dc, s);
    case 4: return launch_cost_fast<4>(descL, maskL, descR, W, H, dmax, disp, cost, dc, s);
    case 8: return launch_cost_fast<8>(descL, maskL, descR, W, H, dmax, disp, cost, dc, s);
    case 16: return launch_cost_fast<16>(descL, maskL, descR, W, H, dmax, disp, cost, dc, s);
    default: break;
  }
  const int tiles = (W + kCostTX - 1) / kCostTX;
  dim3 grid(kXcds * tiles * ((H + kXcds - 1) / kXcds));
#define BSM_LAUNCH_CHUNKED(M, V)                                                             \
  hipLaunchKernelGGL((k_cost_wta_chunked<M, V>), grid, dim3(64), kChunkLds, s, descL, maskL, \
                     descR, W, H, nw, dmax, disp, cost)
  if (maskL) {
    if (cost) BSM_LAUNCH_CHUNKED(true, true);
    else BSM_LAUNCH_CHUNKED(true, false);
  } else {
    if (cost) BSM_LAUNCH_CHUNKED(false, true);
    else BSM_LAUNCH_CHUNKED(false, false);
  }
#undef BSM_LAUNCH_CHUNKED
  return hipGetLastError();
}

hipError_t launch_batch(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                        hipStream_t s) {
  switch (t.nw) {
    case 1: return launch_batch_nw<1>(bl, t, use_mask, s);
    case 2: return launch_batch_nw<2>(bl, t, use_mask, s);
    case 4: return launch_batch_nw<4>(bl, t, use_mask, s);
    case 8: return launch_batch_nw<8>(bl, t, use_mask, s);
    case 16: return launch_batch_nw<16>(bl, t, use_mask, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bsm
