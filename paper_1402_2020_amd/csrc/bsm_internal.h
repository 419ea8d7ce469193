// Internal declarations of the BSM library (host runtime <-> kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bsm.h"

namespace bsm {

// Upper limits of the device code.
constexpr int kMaxBits = 4096;
constexpr int kMaxWords = kMaxBits / 64;
constexpr int kMaxWindow = 63;
constexpr int kInvalidCost = 32767;
constexpr int kMaxSide = 32768;  // largest W or H (grid y limit)

// Integer colour tables (built on the host, used by the colour kernel).
struct ColorTables {
  uint16_t lin[256];      // sRGB decode, 65535 * s(c / 255)
  int32_t mq[9];          // Q14 rows of the white-normalised sRGB->XYZ matrix
  std::vector<uint16_t> f;  // 65536 entries, 65535 * f(t / 65535)
};

void build_color_tables(ColorTables *t);
bsm_status make_pattern(uint64_t seed, int n, int S, double sigma, int8_t *out);

// Small matrix passed to the colour kernel by value.
struct Mq {
  int32_t m[9];
};

// Launch choices the autotuner may change (all results are identical).
struct Tuning {
  int desc_tile_w = 16;                // describe+mask tile width: 16 or 32 pixels
  int cost_dchunk = 64;                // disparities per cost LDS window: 32 or 64
  int blocks_per_cu[4] = {0, 0, 0, 0};  // persistent batch grids (0: all that fit)
  int cost_mfma = 1;                    // no-volume cost + WTA on the matrix cores
  int batch_tile_h = 16;                // describe+mask tile height of the batch: 8 or 16
  // Single-pair launch choices (0 = the size rule of the launcher).
  int pair_desc_th = 0;                 // describe+mask tile height: 4 or 8 rows
  int pair_right_px = 0;                // descriptor-only pixels per lane: 1 or 4
  int mfma_min_dmax = 17;               // smallest dmax on the matrix-core cost kernel
};

// Device-side view of the constant data of a context.
struct DeviceTables {
  const int8_t *pattern;   // [n][4]
  const uint16_t *lin;     // [256]
  const uint16_t *f;       // [65536]
  const int2 *right_offs;  // [n] (p, q) byte offsets in the intensity tile
  Mq mq;
  int n, nw, k, radius;
  int left_pitch16, left_pitch32;  // LDS row pitch (words) of the descriptor+mask
                                   // tile for tile widths 16 and 32
  int right_pitch;                 // LDS row pitch (bytes) of the intensity tile
  Tuning tune;
  int left_pitch_for(int tile_w) const { return tile_w == 32 ? left_pitch32 : left_pitch16; }
};

// Tile geometry of the describe kernels (bsm_kernels.hip).
int describe_left_cols(int radius, int tile_w);  // tile width incl. halo, pixels
int describe_right_cols(int radius);
// LDS pitch (pixels) for the descriptor+mask tile that minimises the bank
// conflicts of the pattern's gathers (host search, bsm_host.cpp).
int choose_left_pitch(const int8_t *pattern, int n, int cols);

// ---- batch work lists (device memory) -------------------------------------
// Queues of the persistent batch kernels.  Cost tiles have one queue per
// XCD, separately for pairs without and with a cost volume.
constexpr int kQueueColor = 0, kQueueDescribeMask = 1, kQueueDescribe = 2, kQueueCost0 = 3;
constexpr int kQueueCostVol0 = kQueueCost0 + 8;
constexpr int kBatchQueues = kQueueCostVol0 + 8;
// Queue heads sit 128 bytes apart, so that the atomics of different queues
// do not contend for one cache line.
constexpr int kCounterStride = 32;

// One pair of a batch with its scratch planes.
struct BatchPair {
  const uint8_t *left, *right;
  int32_t W, H, stride, dmax;
  int32_t *disp;
  int16_t *cost;
  uint32_t *packedL, *packedR;
  uint64_t *descL, *maskL, *descR;
};

// The work list: pairs in scheduling order and, per queue, the prefix sums
// of their tile counts (start[q * (npairs + 1) + i]).
struct BatchWork {
  const BatchPair *pairs;
  const int *order;
  const int *start;
  int *counters;  // head of queue q at counters[q * kCounterStride]
  int npairs;
};

// Host-side handle of a device BatchWork.
struct BatchLaunch {
  const BatchWork *work;  // device pointer
  int *counters;          // device pointer (== work->counters)
  // Optional (eager launches only): kBatchMarks events recorded on the
  // stream before the colour stage and after each of the four stages.
  const hipEvent_t *marks = nullptr;
};
constexpr int kBatchStages = 4;  // colour, describe (both views), cost, cost with a volume
constexpr int kBatchMarks = kBatchStages + 1;

// ---- kernel launchers (bsm_kernels.hip) -----------------------------------
hipError_t launch_color(const uint8_t *img, int W, int H, int stride,
                        uint32_t *packed, int want_lab, int mirror,
                        const DeviceTables &t, hipStream_t s);
// In-place reversal of each of `rows` rows of W elements.
hipError_t launch_reverse_rows(int32_t *data, int W, int rows, hipStream_t s);
hipError_t launch_reverse_rows(int16_t *data, int W, int rows, hipStream_t s);
hipError_t launch_lr_check(const int32_t *dL, const int32_t *dR, int W, int H, int tol,
                           int32_t *out, hipStream_t s);
hipError_t launch_vote_refine(const uint32_t *packed, const int32_t *checked,
                              const int32_t *fallback, int W, int H, int dmax, int radius,
                              float lambda_c, float lambda_e, int32_t *out, hipStream_t s);
constexpr int kMaxVoteDmax = 4096;  // LDS histogram of the voting kernel
hipError_t launch_describe(const uint32_t *packed, int W, int H,
                           const DeviceTables &t, uint64_t *desc,
                           uint64_t *mask, hipStream_t s);
hipError_t launch_cost_wta(const uint64_t *descL, const uint64_t *maskL,
                           const uint64_t *descR, int W, int H, int nw,
                           int dmax, int32_t *disp, int16_t *cost,
                           const DeviceTables &t, hipStream_t s);
// The four persistent stage kernels of a batch (after a counter reset).
hipError_t launch_batch(const BatchLaunch &bl, const DeviceTables &t, int use_mask,
                        hipStream_t s);
bool batch_supported(int nw);
// Tiles per stage of one pair, as the batch kernels number them (cost_mfma:
// the matrix-core cost kernel takes the pairs without a volume).
void batch_tile_counts(int W, int H, int use_mask, int want_cost, int desc_tile_w,
                       int desc_tile_h, int cost_mfma, int counts[kBatchQueues]);

// ---- batch (bsm_batch.cpp) --------------------------------------------------
struct BatchState;
void batch_state_free(BatchState *b);
bsm_status batch_state_create(bsm_ctx *ctx, BatchState **out);
// Runs pairs (device pointers) as one batch with the given state, tables and
// launch choices on stream s.
bsm_status batch_run(bsm_ctx *ctx, BatchState &b, const DeviceTables &dt, const bsm_pair *pairs,
                     int npairs, hipStream_t s);
// The persistent path with its stages launched directly on s (no graph) and
// `marks` (kBatchMarks events) recorded between them.
bsm_status batch_run_marked(bsm_ctx *ctx, BatchState &b, const DeviceTables &dt,
                            const bsm_pair *pairs, int npairs, hipStream_t s,
                            const hipEvent_t *marks);

// ---- device scratch with stream-ordered reuse ---------------------------
// A growable device buffer.  Every use is recorded with an event; a use on
// another stream first waits for that event, and growing waits for it on the
// host, so reuse never races with earlier work.
class Scratch {
 public:
  // tracked = true: every use is recorded with an event, so a use on another
  // stream waits only for that event.  tracked = false (the single-pair
  // entry points, called over and over on one stream): uses are not
  // recorded; a use on another stream, growth and destruction wait for the
  // whole device instead.  An event per call costs about 5 us of command
  // processing on the stream, a device-wide wait only when the stream
  // changes.
  explicit Scratch(bool tracked = true) : tracked_(tracked) {}
  ~Scratch();
  // Returns a buffer of at least `bytes` usable on stream s (nullptr on
  // failure; *err holds the HIP error).
  void *acquire(size_t bytes, hipStream_t s, hipError_t *err);
  // Records that the buffer was last used on stream s.
  hipError_t release(hipStream_t s);
  size_t capacity() const { return cap_; }

 private:
  hipError_t wait_last_use();  // host waits until the last use has finished
  bool tracked_;
  void *ptr_ = nullptr;
  size_t cap_ = 0;
  hipEvent_t ev_ = nullptr;
  bool used_ = false;
  hipStream_t last_ = nullptr;
};

// A second stream with a fork and a join event.  The two views of a pair
// are independent until the cost kernel, so the other view's colour pass
// and descriptor run on the side stream while the reference view's run on
// the caller's stream: on images too small to fill the GPU alone the two
// describe kernels then share it.  Created on first use, with default
// priority; one owner at a time (a context, or one batch state).
class SideLane {
 public:
  ~SideLane();
  hipError_t ensure();  // creates the stream and events once
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct Server;
void server_stop(Server *s);

}  // namespace bsm

struct bsm_ctx {
  int device = 0;
  int n = 0, nw = 0, S = 0, k = 0, use_mask = 1, radius = 0;
  double sigma = 0;
  uint64_t seed = 0;
  std::vector<int8_t> pattern;
  bsm::ColorTables tables;
  // device copies
  int8_t *d_pattern = nullptr;
  uint16_t *d_lin = nullptr;
  uint16_t *d_f = nullptr;
  int2 *d_right_offs = nullptr;
  bsm::DeviceTables dt{};
  // The pattern mirrored horizontally (x offsets negated) and its LDS
  // layouts: right-reference matching runs the left-reference kernels on
  // the mirrored views with it.
  int8_t *d_pattern_m = nullptr;
  int2 *d_right_offs_m = nullptr;
  int left_pitch16_m = 0, left_pitch32_m = 0;
  std::mutex tune_mu;  // guards dt.tune between its setters and the serving thread
  bsm::Scratch describe_scratch{false};  // packed colour plane of bsm_describe
  bsm::Scratch match_scratch{false};     // planes + descriptors of bsm_match
  bsm::SideLane side;             // other-view stream of bsm_match
  bool dead = false;
  std::string dead_reason;
  bsm::BatchState *batch = nullptr;
  bsm::Server *server = nullptr;
  std::mutex server_mu;  // guards lazy creation of `server`
};

namespace bsm {
// RAII: makes the context's device current and restores the caller's.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) err_ = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
  }
  hipError_t err() const { return err_; }

 private:
  int prev_ = -1;
  hipError_t err_ = hipSuccess;
};

// Error plumbing (bsm_host.cpp).
bsm_status fail(bsm_status st, const char *fmt, ...);
bsm_status device_fail(bsm_ctx *ctx, hipError_t e, const char *what);
bsm_status check_alive(bsm_ctx *ctx);
void clear_error();
// Validation shared by the entry points.
bsm_status validate_image(const void *img, int W, int H, int stride);
bsm_status validate_dmax(int W, int dmax);
bool aligned8(const void *p);
bool aligned16(const void *p);
size_t match_scratch_bytes(const bsm_ctx *ctx, int W, int H);
// BSM_EINVAL (with a message) unless every field is in its documented range.
bsm_status check_tuning(const bsm_tuning *t);
// The context's tables with the mirrored pattern in place of the pattern.
DeviceTables mirrored_tables(const bsm_ctx *ctx);
// `side`: a lane for the other view's work (nullptr: everything on s).
bsm_status match_on_stream(bsm_ctx *ctx, const uint8_t *left,
                           const uint8_t *right, int W, int H, int stride,
                           int dmax, int32_t *disp, int16_t *cost,
                           void *scratch, hipStream_t s, SideLane *side,
                           bool right_reference = false);
double now_seconds();
// Entry point without allocation (bsm_noalloc.hip): size of its fixed device
// array, and its set-up, run once per device with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_setup(int device);
}  // namespace bsm
