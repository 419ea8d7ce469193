// Host runtime of the BSM library: error plumbing, parameter validation,
// the point-pair pattern, the integer colour tables, context lifetime and
// the single-pair entry points.  All pixel work is done by the kernels in
// bsm_kernels.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <ctime>

#include "bsm_internal.h"

namespace bsm {

static thread_local std::string g_last_error;

void clear_error() { g_last_error.clear(); }

bsm_status fail(bsm_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

bsm_status device_fail(bsm_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();  // allocation failures are not sticky
    return fail(BSM_ENOMEM, "%s: out of device memory", what);
  }
  if (ctx) {
    ctx->dead = true;
    ctx->dead_reason = std::string(what) + ": " + hipGetErrorString(e);
  }
  return fail(BSM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bsm_status check_alive(bsm_ctx *ctx) {
  if (!ctx) return fail(BSM_EINVAL, "context is NULL");
  if (ctx->dead)
    return fail(BSM_EDEVICE, "context is dead after an earlier device error (%s)",
                ctx->dead_reason.c_str());
  return BSM_OK;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

bsm_status validate_image(const void *img, int W, int H, int stride) {
  if (!img) return fail(BSM_EINVAL, "image pointer is NULL");
  if (W < 1 || H < 1) return fail(BSM_EINVAL, "image size %dx%d must be positive", W, H);
  if (W > kMaxSide || H > kMaxSide)
    return fail(BSM_EINVAL, "image size %dx%d exceeds %d", W, H, kMaxSide);
  if (stride < 3 * W) return fail(BSM_EINVAL, "stride %d < 3*W = %d", stride, 3 * W);
  return BSM_OK;
}

bsm_status validate_dmax(int W, int dmax) {
  if (dmax < 1 || dmax > W)
    return fail(BSM_EINVAL, "dmax %d must be in [1, W=%d]", dmax, W);
  if (dmax > 32767) return fail(BSM_EINVAL, "dmax %d too large", dmax);
  return BSM_OK;
}

double now_seconds() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

// ---------------------------------------------------------------------------
// Point-pair pattern (Section 3, after Eq. 2).  Coordinates are drawn from
// splitmix64 (Steele, Lea and Flood, 2014) through the basic Box-Muller
// transform (cosine branch): z = sqrt(-2 ln u1) cos(2 pi u2) with
// u1 in (0, 1] and u2 in [0, 1) carrying 53 random bits each.  An offset is
// floor(sigma z + 0.5), redrawn while outside [-S/2, (S-1)/2]; p is drawn
// (x then y) before q, and q is redrawn while it equals p.
// ---------------------------------------------------------------------------
namespace {
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

double gaussian(SplitMix64 &g) {
  const double two_pow_53 = 9007199254740992.0;
  uint64_t x1 = g.next(), x2 = g.next();
  double u1 = (double)((x1 >> 11) + 1) * (1.0 / two_pow_53);
  double u2 = (double)(x2 >> 11) * (1.0 / two_pow_53);
  double r = std::sqrt(-2.0 * std::log(u1));
  return r * std::cos(6.283185307179586 * u2);
}

int offset_in_window(SplitMix64 &g, double sigma, int lo, int hi) {
  while (true) {
    double o = std::floor(sigma * gaussian(g) + 0.5);
    if (o >= lo && o <= hi) return static_cast<int>(o);
  }
}
}  // namespace

bsm_status make_pattern(uint64_t seed, int n, int S, double sigma, int8_t *out) {
  if (!out) return fail(BSM_EINVAL, "pattern output is NULL");
  if (n < 1 || n > kMaxBits) return fail(BSM_EINVAL, "n %d out of [1, %d]", n, kMaxBits);
  if (S < 2 || S > kMaxWindow) return fail(BSM_EINVAL, "window %d out of [2, %d]", S, kMaxWindow);
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(BSM_EINVAL, "sigma must be > 0");
  const int lo = -(S / 2), hi = (S - 1) / 2;
  SplitMix64 g{seed};
  for (int i = 0; i < n; ++i) {
    int p[2], q[2];
    p[0] = offset_in_window(g, sigma, lo, hi);
    p[1] = offset_in_window(g, sigma, lo, hi);
    do {
      q[0] = offset_in_window(g, sigma, lo, hi);
      q[1] = offset_in_window(g, sigma, lo, hi);
    } while (q[0] == p[0] && q[1] == p[1]);
    int8_t *row = out + 4 * i;
    row[0] = (int8_t)p[0];
    row[1] = (int8_t)p[1];
    row[2] = (int8_t)q[0];
    row[3] = (int8_t)q[1];
  }
  return BSM_OK;
}

// ---------------------------------------------------------------------------
// Integer CIELAB tables.  sRGB decoding (IEC 61966-2-1), the sRGB->XYZ matrix
// of the same standard with each row divided by the D65 white (its row sum)
// and rounded to Q14 so that each row sums to 16384 exactly (greys map to
// a = b = 0), and the CIE companding function f on a 16-bit grid.  Doubles
// are rounded half away from zero.
// ---------------------------------------------------------------------------
void build_color_tables(ColorTables *t) {
  for (int c = 0; c < 256; ++c) {
    double x = c / 255.0;
    double lin = x <= 0.04045 ? x / 12.92 : std::pow((x + 0.055) / 1.055, 2.4);
    t->lin[c] = (uint16_t)std::lround(65535.0 * lin);
  }
  static const double M[3][3] = {{0.4124, 0.3576, 0.1805},
                                 {0.2126, 0.7152, 0.0722},
                                 {0.0193, 0.1192, 0.9505}};
  for (int r = 0; r < 3; ++r) {
    const double white = M[r][0] + M[r][1] + M[r][2];
    int32_t *row = t->mq + 3 * r;
    int largest = 0;
    for (int c = 0; c < 3; ++c) {
      row[c] = (int32_t)std::lround(16384.0 * M[r][c] / white);
      if (row[c] > row[largest]) largest = c;
    }
    row[largest] += 16384 - (row[0] + row[1] + row[2]);
  }
  t->f.resize(65536);
  const double e = 6.0 / 29.0;
  for (int i = 0; i < 65536; ++i) {
    double x = i / 65535.0;
    double f = x > e * e * e ? std::cbrt(x) : x / (3.0 * e * e) + 4.0 / 29.0;
    t->f[i] = (uint16_t)std::lround(65535.0 * f);
  }
}

// ---------------------------------------------------------------------------
// LDS pitch of the descriptor+mask tile.  In that kernel the 64 lanes of a
// wave gather the samples of 64 pairs at once, at LDS word offsets
// py * pitch + px from the same centre; LDS serves 32 lanes per cycle and a
// half-wave takes as many cycles as its most loaded bank (32 banks of 4
// bytes).  The offsets are random, but the pitch changes how they fall into
// banks, so try the pitches [cols, cols + 32) and keep the one with the
// fewest cycles summed over all words and both samples.
// ---------------------------------------------------------------------------
int choose_left_pitch(const int8_t *pattern, int n, int cols) {
  // The describe+mask kernel's gathers: for slot j, lane l reads the
  // samples of pair NW l + j (NW >= 8) or 64 j + l (NW <= 4); pairs past n
  // read the centre.  Each half-wave's 32 lanes are served together, one
  // cycle per lane that shares a bank with earlier ones.
  int NW = 1;
  while (NW < n / 64) NW *= 2;
  int best_pitch = cols, best_cycles = -1;
  for (int pitch = cols; pitch < cols + 32; ++pitch) {
    int cycles = 0;
    for (int j = 0; j < NW; ++j)
      for (int sample = 0; sample < 2; ++sample)
        for (int half = 0; half < 2; ++half) {
          int load[32] = {0}, worst = 0;
          for (int l = 32 * half; l < 32 * half + 32; ++l) {
            const int i = NW >= 8 ? NW * l + j : 64 * j + l;
            int dx = 0, dy = 0;
            if (i < n) {
              dx = pattern[4 * i + 2 * sample];
              dy = pattern[4 * i + 2 * sample + 1];
            }
            const int bank = ((dy * pitch + dx) % 32 + 32) % 32;
            worst = std::max(worst, ++load[bank]);
          }
          cycles += worst;
        }
    if (best_cycles < 0 || cycles < best_cycles) {
      best_cycles = cycles;
      best_pitch = pitch;
    }
  }
  return best_pitch;
}

// ---------------------------------------------------------------------------
Scratch::~Scratch() {
  if (used_) (void)wait_last_use();
  if (ev_) (void)hipEventDestroy(ev_);
  if (ptr_) (void)hipFree(ptr_);
}

hipError_t Scratch::wait_last_use() {
  return tracked_ ? hipEventSynchronize(ev_) : hipDeviceSynchronize();
}

void *Scratch::acquire(size_t bytes, hipStream_t s, hipError_t *err) {
  *err = hipSuccess;
  if (tracked_ && !ev_) {
    *err = hipEventCreateWithFlags(&ev_, hipEventDisableTiming);
    if (*err != hipSuccess) return nullptr;
  }
  if (bytes > cap_) {
    if (used_) {
      *err = wait_last_use();
      if (*err != hipSuccess) return nullptr;
      used_ = false;
    }
    if (ptr_) (void)hipFree(ptr_);
    ptr_ = nullptr;
    cap_ = 0;
    *err = hipMalloc(&ptr_, bytes);
    if (*err != hipSuccess) {
      ptr_ = nullptr;
      return nullptr;
    }
    cap_ = bytes;
  } else if (used_ && last_ != s) {
    *err = tracked_ ? hipStreamWaitEvent(s, ev_, 0) : hipDeviceSynchronize();
    if (*err != hipSuccess) return nullptr;
  }
  return ptr_;
}

hipError_t Scratch::release(hipStream_t s) {
  used_ = true;
  last_ = s;
  return tracked_ ? hipEventRecord(ev_, s) : hipSuccess;
}

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t match_scratch_bytes(const bsm_ctx *ctx, int W, int H) {
  size_t px = (size_t)W * H;
  size_t plane = round_up(px * 4, 256);
  size_t desc = round_up(px * ctx->nw * 8, 256);
  return 2 * plane + 3 * desc;
}

SideLane::~SideLane() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  if (stream) (void)hipStreamDestroy(stream);
}

hipError_t SideLane::ensure() {
  hipError_t e = hipSuccess;
  if (!fork && (e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess) return e;
  if (!join && (e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess) return e;
  if (!stream) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  return e;
}

// The whole hot path of one pair on stream s; `scratch` holds
// match_scratch_bytes(W, H).  With right_reference the right view is the
// reference (partner (u + d, v) in the left view, the right view's mask):
// that is left-reference matching of the mirrored pair (mirrored right view
// as reference, mirrored left view as the other) with the mirrored pattern,
// whose results are reversed back row by row.  With a side lane (and an
// image large enough) the other view's colour pass and descriptor run
// there, forked after everything already queued on s and joined back
// before the cost kernel.
bsm_status match_on_stream(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right,
                           int W, int H, int stride, int dmax, int32_t *disp,
                           int16_t *cost, void *scratch, hipStream_t s, SideLane *side,
                           bool right_reference) {
  size_t px = (size_t)W * H;
  char *base = static_cast<char *>(scratch);
  const size_t plane = round_up(px * 4, 256);
  uint32_t *packedA = reinterpret_cast<uint32_t *>(base);
  uint32_t *packedB = reinterpret_cast<uint32_t *>(base + plane);
  size_t desc_bytes = round_up(px * ctx->nw * 8, 256);
  uint64_t *descA = reinterpret_cast<uint64_t *>(base + 2 * plane);
  uint64_t *maskA = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(descA) + desc_bytes);
  uint64_t *descB = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(maskA) + desc_bytes);
  const bool m = ctx->use_mask != 0;
  const DeviceTables t = right_reference ? mirrored_tables(ctx) : ctx->dt;
  const uint8_t *ref = right_reference ? right : left;
  const uint8_t *other = right_reference ? left : right;
  const int mirror = right_reference ? 1 : 0;
  hipError_t e;
  hipStream_t so = s;  // stream of the other view
  // Below ~64 K pixels the kernels are too short for the cross-stream
  // waits to pay for themselves.
  constexpr size_t kSideMinPixels = 1 << 16;
  if (side && px >= kSideMinPixels) {
    if ((e = side->ensure()) != hipSuccess || (e = hipEventRecord(side->fork, s)) != hipSuccess ||
        (e = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess)
      return device_fail(ctx, e, "forking the other view's stream");
    so = side->stream;
  }
  if ((e = launch_color(other, W, H, stride, packedB, 0, mirror, t, so)) != hipSuccess)
    return device_fail(ctx, e, "colour pre-pass (other view)");
  if ((e = launch_describe(packedB, W, H, t, descB, nullptr, so)) != hipSuccess)
    return device_fail(ctx, e, "describe (other view)");
  if (so != s && (e = hipEventRecord(side->join, so)) != hipSuccess)
    return device_fail(ctx, e, "joining the other view's stream");
  if ((e = launch_color(ref, W, H, stride, packedA, m, mirror, t, s)) != hipSuccess)
    return device_fail(ctx, e, "colour pre-pass (reference view)");
  if ((e = launch_describe(packedA, W, H, t, descA, m ? maskA : nullptr, s)) != hipSuccess)
    return device_fail(ctx, e, "describe (reference view)");
  if (so != s && (e = hipStreamWaitEvent(s, side->join, 0)) != hipSuccess)
    return device_fail(ctx, e, "joining the other view's stream");
  if ((e = launch_cost_wta(descA, m ? maskA : nullptr, descB, W, H, ctx->nw, dmax, disp, cost, t,
                           s)) != hipSuccess)
    return device_fail(ctx, e, "cost + WTA");
  if (right_reference) {
    if ((e = launch_reverse_rows(disp, W, H, s)) != hipSuccess ||
        (cost && (e = launch_reverse_rows(cost, W, dmax * H, s)) != hipSuccess))
      return device_fail(ctx, e, "mirroring results back");
  }
  return BSM_OK;
}

DeviceTables mirrored_tables(const bsm_ctx *ctx) {
  DeviceTables t = ctx->dt;
  t.pattern = ctx->d_pattern_m;
  t.right_offs = ctx->d_right_offs_m;
  t.left_pitch16 = ctx->left_pitch16_m;
  t.left_pitch32 = ctx->left_pitch32_m;
  return t;
}

}  // namespace bsm

namespace bsm {

bsm_status check_tuning(const bsm_tuning *in) {
  if (!in) return fail(BSM_EINVAL, "tuning must not be NULL");
  if (in->desc_tile_w != 16 && in->desc_tile_w != 32)
    return fail(BSM_EINVAL, "desc_tile_w must be 16 or 32");
  if (in->cost_dchunk != 32 && in->cost_dchunk != 64)
    return fail(BSM_EINVAL, "cost_dchunk must be 32 or 64");
  for (int i = 0; i < 4; ++i)
    if (in->blocks_per_cu[i] < 0 || in->blocks_per_cu[i] > 64)
      return fail(BSM_EINVAL, "blocks_per_cu[%d] out of [0, 64]", i);
  if (in->cost_mfma != 0 && in->cost_mfma != 1) return fail(BSM_EINVAL, "cost_mfma must be 0 or 1");
  if (in->batch_tile_h != 8 && in->batch_tile_h != 16)
    return fail(BSM_EINVAL, "batch_tile_h must be 8 or 16");
  if (in->pair_desc_th != 0 && in->pair_desc_th != 4 && in->pair_desc_th != 8)
    return fail(BSM_EINVAL, "pair_desc_th must be 0, 4 or 8");
  if (in->pair_right_px != 0 && in->pair_right_px != 1 && in->pair_right_px != 4)
    return fail(BSM_EINVAL, "pair_right_px must be 0, 1 or 4");
  if (in->mfma_min_dmax < 2 || in->mfma_min_dmax > 257)
    return fail(BSM_EINVAL, "mfma_min_dmax must be in [2, 257]");
  return BSM_OK;
}

}  // namespace bsm

using namespace bsm;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *bsm_last_error(void) { return g_last_error.c_str(); }

bsm_status bsm_make_pattern(uint64_t seed, int32_t n, int32_t S, double sigma, int8_t *out) {
  clear_error();
  return make_pattern(seed, n, S, sigma, out);
}

bsm_status bsm_create(const bsm_params *p, int32_t hip_device, bsm_ctx **out) {
  clear_error();
  if (!p || !out) return fail(BSM_EINVAL, "params and out must not be NULL");
  *out = nullptr;
  if (p->n_bits < 64 || p->n_bits > kMaxBits || p->n_bits % 64)
    return fail(BSM_EINVAL, "n_bits %d must be a multiple of 64 in [64, %d]", p->n_bits, kMaxBits);
  if (p->window < 2 || p->window > kMaxWindow)
    return fail(BSM_EINVAL, "window %d out of [2, %d]", p->window, kMaxWindow);
  if (!std::isfinite(p->sigma)) return fail(BSM_EINVAL, "sigma is not finite");
  const int k = p->mask_rank == 0 ? p->n_bits / 4 : p->mask_rank;
  if (k < 1 || k > p->n_bits)
    return fail(BSM_EINVAL, "mask_rank %d out of [1, n=%d]", p->mask_rank, p->n_bits);
  if (p->use_mask != 0 && p->use_mask != 1) return fail(BSM_EINVAL, "use_mask must be 0 or 1");
  std::unique_ptr<bsm_ctx> ctx(new bsm_ctx);
  ctx->device = hip_device;
  ctx->n = p->n_bits;
  ctx->nw = p->n_bits / 64;
  ctx->S = p->window;
  ctx->k = k;
  ctx->use_mask = p->use_mask;
  ctx->sigma = p->sigma > 0 ? p->sigma : 4.0 * p->window / 26.0;
  ctx->seed = p->seed;
  ctx->pattern.resize(4 * (size_t)ctx->n);
  const int lo = -(ctx->S / 2), hi = (ctx->S - 1) / 2;
  if (p->pattern) {
    for (int i = 0; i < 4 * ctx->n; ++i) {
      int o = p->pattern[i];
      if (o < lo || o > hi)
        return fail(BSM_EINVAL, "pattern entry %d (pair %d) = %d outside [%d, %d]", i, i / 4 + 1, o,
                    lo, hi);
      ctx->pattern[i] = p->pattern[i];
    }
  } else {
    bsm_status st = make_pattern(ctx->seed, ctx->n, ctx->S, ctx->sigma, ctx->pattern.data());
    if (st != BSM_OK) return st;
  }
  int radius = 0;
  for (int8_t o : ctx->pattern) radius = std::max(radius, std::abs((int)o));
  ctx->radius = radius;
  build_color_tables(&ctx->tables);

  // host-side validation is complete; from here on the device is touched
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(BSM_EDEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= ndev)
    return fail(BSM_EINVAL, "device %d out of [0, %d)", hip_device, ndev);

  // LDS layouts of the describe kernels: the pitch of the descriptor+mask
  // tile is chosen for this pattern; the intensity tile needs no padding.
  const int left_pitch16 =
      choose_left_pitch(ctx->pattern.data(), ctx->n, describe_left_cols(radius, 16));
  const int left_pitch32 =
      choose_left_pitch(ctx->pattern.data(), ctx->n, describe_left_cols(radius, 32));
  const int right_pitch = describe_right_cols(radius);
  std::vector<int2> right_offs(ctx->n);
  for (int i = 0; i < ctx->n; ++i) {
    const int8_t *o = &ctx->pattern[4 * i];
    right_offs[i] = make_int2(o[1] * right_pitch + o[0], o[3] * right_pitch + o[2]);
  }
  // The same for the mirrored pattern (right-reference matching).
  std::vector<int8_t> mirrored(ctx->pattern);
  for (int i = 0; i < ctx->n; ++i) {
    mirrored[4 * i] = static_cast<int8_t>(-mirrored[4 * i]);
    mirrored[4 * i + 2] = static_cast<int8_t>(-mirrored[4 * i + 2]);
  }
  ctx->left_pitch16_m = choose_left_pitch(mirrored.data(), ctx->n, describe_left_cols(radius, 16));
  ctx->left_pitch32_m = choose_left_pitch(mirrored.data(), ctx->n, describe_left_cols(radius, 32));
  std::vector<int2> right_offs_m(ctx->n);
  for (int i = 0; i < ctx->n; ++i) {
    const int8_t *o = &mirrored[4 * i];
    right_offs_m[i] = make_int2(o[1] * right_pitch + o[0], o[3] * right_pitch + o[2]);
  }

  DeviceGuard g(hip_device);
  if (g.err() != hipSuccess) return device_fail(nullptr, g.err(), "hipSetDevice");
  hipError_t e;
  // the device address of bsm_match_noalloc's fixed array, once per device
  if ((e = noalloc_setup(hip_device)) != hipSuccess) {
    bsm_destroy(ctx.release());
    return device_fail(nullptr, e, "taking the address of the no-allocation scratch array");
  }
  if ((e = hipMalloc(&ctx->d_pattern, ctx->pattern.size())) != hipSuccess ||
      (e = hipMalloc(&ctx->d_lin, 256 * sizeof(uint16_t))) != hipSuccess ||
      (e = hipMalloc(&ctx->d_f, 65536 * sizeof(uint16_t))) != hipSuccess ||
      (e = hipMalloc(&ctx->d_right_offs, right_offs.size() * sizeof(int2))) != hipSuccess ||
      (e = hipMalloc(&ctx->d_pattern_m, mirrored.size())) != hipSuccess ||
      (e = hipMalloc(&ctx->d_right_offs_m, right_offs_m.size() * sizeof(int2))) != hipSuccess) {
    bsm_destroy(ctx.release());
    return device_fail(nullptr, e, "allocating context tables");
  }
  if ((e = hipMemcpy(ctx->d_pattern, ctx->pattern.data(), ctx->pattern.size(),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->d_lin, ctx->tables.lin, 256 * sizeof(uint16_t), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(ctx->d_f, ctx->tables.f.data(), 65536 * sizeof(uint16_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->d_right_offs, right_offs.data(), right_offs.size() * sizeof(int2),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->d_pattern_m, mirrored.data(), mirrored.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(ctx->d_right_offs_m, right_offs_m.data(), right_offs_m.size() * sizeof(int2),
                     hipMemcpyHostToDevice)) != hipSuccess) {
    bsm_destroy(ctx.release());
    return device_fail(nullptr, e, "uploading context tables");
  }
  DeviceTables &dt = ctx->dt;
  dt.pattern = ctx->d_pattern;
  dt.lin = ctx->d_lin;
  dt.f = ctx->d_f;
  dt.right_offs = ctx->d_right_offs;
  dt.left_pitch16 = left_pitch16;
  dt.left_pitch32 = left_pitch32;
  dt.right_pitch = right_pitch;
  std::memcpy(dt.mq.m, ctx->tables.mq, sizeof dt.mq.m);
  dt.n = ctx->n;
  dt.nw = ctx->nw;
  dt.k = ctx->k;
  dt.radius = ctx->radius;
  *out = ctx.release();
  return BSM_OK;
}

void bsm_destroy(bsm_ctx *ctx) {
  if (!ctx) return;
  if (ctx->server) server_stop(ctx->server);
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->batch) batch_state_free(ctx->batch);
  if (ctx->d_pattern) (void)hipFree(ctx->d_pattern);
  if (ctx->d_lin) (void)hipFree(ctx->d_lin);
  if (ctx->d_f) (void)hipFree(ctx->d_f);
  if (ctx->d_right_offs) (void)hipFree(ctx->d_right_offs);
  if (ctx->d_pattern_m) (void)hipFree(ctx->d_pattern_m);
  if (ctx->d_right_offs_m) (void)hipFree(ctx->d_right_offs_m);
  delete ctx;  // scratch buffers are released with the device still current
}

bsm_status bsm_pattern(const bsm_ctx *ctx, int8_t *out) {
  clear_error();
  if (!ctx || !out) return fail(BSM_EINVAL, "context and out must not be NULL");
  std::memcpy(out, ctx->pattern.data(), ctx->pattern.size());
  return BSM_OK;
}

size_t bsm_footprint(const bsm_ctx *ctx, int32_t W, int32_t H, int32_t dmax, int32_t want_cost) {
  clear_error();
  if (!ctx || W < 1 || H < 1 || dmax < 1 || dmax > W) return 0;
  size_t bytes = match_scratch_bytes(ctx, W, H);
  if (want_cost) bytes += (size_t)dmax * W * H * sizeof(int16_t);
  return bytes;
}

bsm_status bsm_color(bsm_ctx *ctx, const uint8_t *img, int32_t W, int32_t H, int32_t stride,
                     uint32_t *packed, int32_t want_lab, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(img, W, H, stride)) != BSM_OK) return st;
  if (!packed || (reinterpret_cast<uintptr_t>(packed) & 3u))
    return fail(BSM_EINVAL, "packed output must be a 4-byte aligned device pointer");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipError_t e = launch_color(img, W, H, stride, packed, want_lab ? 1 : 0, 0, ctx->dt,
                              static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? BSM_OK : device_fail(ctx, e, "colour pre-pass");
}

bsm_status bsm_describe(bsm_ctx *ctx, const uint8_t *img, int32_t W, int32_t H, int32_t stride,
                        uint64_t *desc, uint64_t *mask, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(img, W, H, stride)) != BSM_OK) return st;
  if (!desc || !aligned16(desc)) return fail(BSM_EINVAL, "desc must be a 16-byte aligned device pointer");
  if (mask && !aligned16(mask)) return fail(BSM_EINVAL, "mask must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  void *buf = ctx->describe_scratch.acquire((size_t)W * H * 4, s, &e);
  if (!buf) return device_fail(ctx, e, "describe scratch");
  if ((e = launch_color(img, W, H, stride, static_cast<uint32_t *>(buf), mask != nullptr, 0, ctx->dt,
                        s)) !=
      hipSuccess)
    return device_fail(ctx, e, "colour pre-pass");
  if ((e = launch_describe(static_cast<uint32_t *>(buf), W, H, ctx->dt, desc, mask, s)) != hipSuccess)
    return device_fail(ctx, e, "describe");
  if ((e = ctx->describe_scratch.release(s)) != hipSuccess)
    return device_fail(ctx, e, "describe scratch event");
  return BSM_OK;
}

bsm_status bsm_describe_packed(bsm_ctx *ctx, const uint32_t *packed, int32_t W, int32_t H,
                               uint64_t *desc, uint64_t *mask, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(packed, W, H, 3 * W)) != BSM_OK) return st;
  if (reinterpret_cast<uintptr_t>(packed) & 3u) return fail(BSM_EINVAL, "packed must be 4-byte aligned");
  if (!desc || !aligned16(desc)) return fail(BSM_EINVAL, "desc must be a 16-byte aligned device pointer");
  if (mask && !aligned16(mask)) return fail(BSM_EINVAL, "mask must be 16-byte aligned");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipError_t e = launch_describe(packed, W, H, ctx->dt, desc, mask, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? BSM_OK : device_fail(ctx, e, "describe");
}

bsm_status bsm_cost_wta(bsm_ctx *ctx, const uint64_t *descL, const uint64_t *maskL,
                        const uint64_t *descR, int32_t W, int32_t H, int32_t dmax, int32_t *disp,
                        int16_t *cost, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (W < 1 || H < 1 || W > kMaxSide || H > kMaxSide)
    return fail(BSM_EINVAL, "image size %dx%d out of range", W, H);
  if ((st = validate_dmax(W, dmax)) != BSM_OK) return st;
  if (!descL || !descR || !disp) return fail(BSM_EINVAL, "descL, descR and disp must not be NULL");
  if (!aligned16(descL) || !aligned16(descR) || (maskL && !aligned16(maskL)) ||
      (reinterpret_cast<uintptr_t>(disp) & 3u) || (reinterpret_cast<uintptr_t>(cost) & 3u))
    return fail(BSM_EINVAL, "misaligned device pointer");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipError_t e = launch_cost_wta(descL, maskL, descR, W, H, ctx->nw, dmax, disp, cost, ctx->dt,
                                 static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? BSM_OK : device_fail(ctx, e, "cost + WTA");
}

bsm_status bsm_get_tuning(const bsm_ctx *ctx, bsm_tuning *out) {
  clear_error();
  if (!ctx || !out) return fail(BSM_EINVAL, "context and out must not be NULL");
  const Tuning &t = ctx->dt.tune;
  out->desc_tile_w = t.desc_tile_w;
  out->cost_dchunk = t.cost_dchunk;
  for (int i = 0; i < 4; ++i) out->blocks_per_cu[i] = t.blocks_per_cu[i];
  out->cost_mfma = t.cost_mfma;
  out->batch_tile_h = t.batch_tile_h;
  out->pair_desc_th = t.pair_desc_th;
  out->pair_right_px = t.pair_right_px;
  out->mfma_min_dmax = t.mfma_min_dmax;
  return BSM_OK;
}

bsm_status bsm_set_tuning(bsm_ctx *ctx, const bsm_tuning *in) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = check_tuning(in)) != BSM_OK) return st;
  Tuning t;
  t.desc_tile_w = in->desc_tile_w;
  t.cost_dchunk = in->cost_dchunk;
  for (int i = 0; i < 4; ++i) t.blocks_per_cu[i] = in->blocks_per_cu[i];
  t.cost_mfma = in->cost_mfma;
  t.batch_tile_h = in->batch_tile_h;
  t.pair_desc_th = in->pair_desc_th;
  t.pair_right_px = in->pair_right_px;
  t.mfma_min_dmax = in->mfma_min_dmax;
  {
    // batch states compare this with the choices their graphs hold
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->dt.tune = t;
  }
  return BSM_OK;
}

static bsm_status match_entry(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right, int32_t W,
                              int32_t H, int32_t stride, int32_t dmax, int32_t *disp,
                              int16_t *cost, void *hip_stream, bool right_reference) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(left, W, H, stride)) != BSM_OK) return st;
  if ((st = validate_image(right, W, H, stride)) != BSM_OK) return st;
  if ((st = validate_dmax(W, dmax)) != BSM_OK) return st;
  if (!disp || (reinterpret_cast<uintptr_t>(disp) & 3u) || (reinterpret_cast<uintptr_t>(cost) & 3u))
    return fail(BSM_EINVAL, "disp must be a 4-byte aligned device pointer (cost too)");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  void *buf = ctx->match_scratch.acquire(match_scratch_bytes(ctx, W, H), s, &e);
  if (!buf) return device_fail(ctx, e, "match scratch");
  st = match_on_stream(ctx, left, right, W, H, stride, dmax, disp, cost, buf, s, &ctx->side,
                       right_reference);
  if (st != BSM_OK) return st;
  if ((e = ctx->match_scratch.release(s)) != hipSuccess)
    return device_fail(ctx, e, "match scratch event");
  return BSM_OK;
}

bsm_status bsm_match(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right, int32_t W, int32_t H,
                     int32_t stride, int32_t dmax, int32_t *disp, int16_t *cost, void *hip_stream) {
  return match_entry(ctx, left, right, W, H, stride, dmax, disp, cost, hip_stream, false);
}

bsm_status bsm_match_right(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right, int32_t W,
                           int32_t H, int32_t stride, int32_t dmax, int32_t *disp, int16_t *cost,
                           void *hip_stream) {
  return match_entry(ctx, left, right, W, H, stride, dmax, disp, cost, hip_stream, true);
}

bsm_status bsm_lr_check(bsm_ctx *ctx, const int32_t *disp_left, const int32_t *disp_right,
                        int32_t W, int32_t H, int32_t tol, int32_t *out, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (W < 1 || H < 1 || W > kMaxSide || H > kMaxSide)
    return fail(BSM_EINVAL, "image size %d x %d out of [1, %d]", W, H, kMaxSide);
  if (tol < 0) return fail(BSM_EINVAL, "tol must be >= 0");
  if (!disp_left || !disp_right || !out)
    return fail(BSM_EINVAL, "disp_left, disp_right and out must not be NULL");
  if ((reinterpret_cast<uintptr_t>(disp_left) | reinterpret_cast<uintptr_t>(disp_right) |
       reinterpret_cast<uintptr_t>(out)) & 3u)
    return fail(BSM_EINVAL, "disparity maps must be 4-byte aligned");
  if (out == disp_right) return fail(BSM_EINVAL, "out must not alias disp_right");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipError_t e = launch_lr_check(disp_left, disp_right, W, H, tol, out,
                                 static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(ctx, e, "left/right check");
  return BSM_OK;
}

bsm_status bsm_vote_refine(bsm_ctx *ctx, const uint8_t *left, int32_t W, int32_t H,
                           int32_t stride, const int32_t *checked, const int32_t *fallback,
                           int32_t dmax, int32_t radius, float lambda_c, float lambda_e,
                           int32_t *out, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(left, W, H, stride)) != BSM_OK) return st;
  if (dmax < 1 || dmax > kMaxVoteDmax)
    return fail(BSM_EINVAL, "dmax %d out of [1, %d]", dmax, kMaxVoteDmax);
  if (radius < 0 || radius > kMaxWindow)
    return fail(BSM_EINVAL, "radius %d out of [0, %d]", radius, kMaxWindow);
  if (!(lambda_c > 0.0f) || !(lambda_e > 0.0f))
    return fail(BSM_EINVAL, "lambda_c and lambda_e must be > 0");
  if (!checked || !fallback || !out)
    return fail(BSM_EINVAL, "checked, fallback and out must not be NULL");
  if ((reinterpret_cast<uintptr_t>(checked) | reinterpret_cast<uintptr_t>(fallback) |
       reinterpret_cast<uintptr_t>(out)) & 3u)
    return fail(BSM_EINVAL, "disparity maps must be 4-byte aligned");
  if (out == checked) return fail(BSM_EINVAL, "out must not alias checked");
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  void *buf = ctx->describe_scratch.acquire((size_t)W * H * 4, s, &e);
  if (!buf) return device_fail(ctx, e, "refinement scratch");
  uint32_t *packed = static_cast<uint32_t *>(buf);
  if ((e = launch_color(left, W, H, stride, packed, 1, 0, ctx->dt, s)) != hipSuccess)
    return device_fail(ctx, e, "colour pre-pass (refinement)");
  if ((e = launch_vote_refine(packed, checked, fallback, W, H, dmax, radius, lambda_c, lambda_e,
                              out, s)) != hipSuccess)
    return device_fail(ctx, e, "voting refinement");
  if ((e = ctx->describe_scratch.release(s)) != hipSuccess)
    return device_fail(ctx, e, "refinement scratch event");
  return BSM_OK;
}

}  // extern "C"
