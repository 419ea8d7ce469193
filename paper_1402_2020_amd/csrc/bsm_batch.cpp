// Batched matching of many uneven pairs (bsm_match_batch) and the autotuner.
//
// A batch is described to the device by a work list (BatchWork): the pairs
// with their scratch planes, a scheduling order (largest W*H*dmax first) and
// per-queue prefix sums of tile counts.  The persistent stage kernels read
// everything from that list, so their launches never change with the batch:
// they are captured once into a HIP graph and replayed for every batch.  The
// list travels host -> device through a pinned staging buffer just before
// the graph launch, on the same stream.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <vector>

#include "bsm_internal.h"

namespace bsm {

namespace {
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
}  // namespace

// Batches of at most this many pairs take the per-pair kernels.
constexpr int kSequentialMaxPairs = 4;

struct BatchState {
  Scratch scratch;               // per-pair planes and descriptors
  SideLane side;                 // other-view stream of the per-pair path
  // d_work and d_counters live in one allocation at a fixed device address:
  // both are baked into the captured graph, so neither may move while the
  // graph exists.  The tables (which grow with the batch) are only reached
  // through d_work.
  BatchWork *d_work = nullptr;
  int *d_counters = nullptr;     // queue heads, kCounterStride ints apart
  char *d_tables = nullptr;      // pairs | order | start
  size_t d_tables_cap = 0;
  Tuning tune;                   // launch choices the graph was captured with
  char *h_stage = nullptr;       // pinned staging of BatchWork + tables
  size_t h_stage_cap = 0;
  hipEvent_t done = nullptr;     // last batch finished with the tables
  hipEvent_t staged = nullptr;   // last batch's upload has read the staging buffer
  hipStream_t last_stream = nullptr;  // stream of the last batch
  bool launched = false;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~BatchState() {
    if (done) {
      if (launched) (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (staged) (void)hipEventDestroy(staged);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
    if (d_work) (void)hipFree(d_work);
    if (d_tables) (void)hipFree(d_tables);
    if (h_stage) (void)hipHostFree(h_stage);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

void batch_state_free(BatchState *b) { delete b; }

namespace {

// Scratch bytes of one pair in a batch: both colour planes, descriptors of
// both views and the left mask.
size_t pair_scratch_bytes(const bsm_ctx *ctx, int W, int H) {
  const size_t px = (size_t)W * H;
  return 2 * align_up(px * 4, 256) + 3 * align_up(px * ctx->nw * 8, 256);
}

}  // namespace

bsm_status batch_state_create(bsm_ctx *ctx, BatchState **out) {
  std::unique_ptr<BatchState> b(new BatchState);
  hipError_t e;
  const size_t work_bytes = align_up(sizeof(BatchWork), 256);
  if ((e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipMalloc(&b->d_work, work_bytes + kBatchQueues * kCounterStride * sizeof(int))) !=
          hipSuccess)
    return device_fail(ctx, e, "batch state");
  b->d_counters = reinterpret_cast<int *>(reinterpret_cast<char *>(b->d_work) + work_bytes);
  *out = b.release();
  return BSM_OK;
}

namespace {

bsm_status validate_pairs(const bsm_pair *pairs, int npairs) {
  if (npairs < 0 || (npairs > 0 && !pairs)) return fail(BSM_EINVAL, "invalid pair list");
  for (int i = 0; i < npairs; ++i) {
    const bsm_pair &p = pairs[i];
    bsm_status st;
    if ((st = validate_image(p.left, p.width, p.height, p.stride)) != BSM_OK ||
        (st = validate_image(p.right, p.width, p.height, p.stride)) != BSM_OK ||
        (st = validate_dmax(p.width, p.dmax)) != BSM_OK)
      return fail(st, "pair %d: %s", i, bsm_last_error());
    if (!p.disp || (reinterpret_cast<uintptr_t>(p.disp) & 3u) ||
        (reinterpret_cast<uintptr_t>(p.cost) & 3u))
      return fail(BSM_EINVAL, "pair %d: misaligned or NULL output", i);
  }
  return BSM_OK;
}

// Pairs one after another with the per-pair kernels.
bsm_status batch_sequential(bsm_ctx *ctx, BatchState &b, const bsm_pair *pairs, int npairs,
                            hipStream_t s) {
  size_t need = 0;
  for (int i = 0; i < npairs; ++i)
    need = std::max(need, match_scratch_bytes(ctx, pairs[i].width, pairs[i].height));
  hipError_t e;
  void *buf = b.scratch.acquire(need, s, &e);
  if (!buf) return device_fail(ctx, e, "batch scratch");
  for (int i = 0; i < npairs; ++i) {
    const bsm_pair &p = pairs[i];
    bsm_status st = match_on_stream(ctx, p.left, p.right, p.width, p.height, p.stride, p.dmax,
                                    p.disp, p.cost, buf, s, &b.side);
    if (st != BSM_OK) return st;
  }
  if ((e = b.scratch.release(s)) != hipSuccess)
    return device_fail(ctx, e, "batch scratch event");
  return BSM_OK;
}

bool same_tuning(const Tuning &a, const Tuning &b) {
  if (a.desc_tile_w != b.desc_tile_w || a.cost_dchunk != b.cost_dchunk ||
      a.cost_mfma != b.cost_mfma || a.batch_tile_h != b.batch_tile_h)
    return false;
  for (int i = 0; i < 4; ++i)
    if (a.blocks_per_cu[i] != b.blocks_per_cu[i]) return false;
  return true;
}

// marks != nullptr: the stages are launched directly on s with the events
// recorded between them (the graph is neither used nor captured).
bsm_status batch_persistent(bsm_ctx *ctx, BatchState &b, const DeviceTables &dt,
                            const bsm_pair *pairs, int npairs, hipStream_t s,
                            const hipEvent_t *marks = nullptr) {
  const int use_mask = ctx->use_mask;
  hipError_t e;

  // Schedule: largest cost work first, so the longest tiles start early.
  std::vector<int> order(npairs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const double wx = (double)pairs[x].width * pairs[x].height * pairs[x].dmax;
    const double wy = (double)pairs[y].width * pairs[y].height * pairs[y].dmax;
    return wx > wy;
  });

  // Scratch planes of every pair.
  std::vector<size_t> offset(npairs);
  size_t total = 0;
  for (int i = 0; i < npairs; ++i) {
    offset[i] = total;
    total += pair_scratch_bytes(ctx, pairs[i].width, pairs[i].height);
  }
  void *scratch = b.scratch.acquire(total, s, &e);
  if (!scratch) return device_fail(ctx, e, "batch scratch");

  // Table layout (device and pinned staging alike).
  const size_t n1 = npairs + 1;
  const size_t off_pairs = 0;
  const size_t off_order = align_up(off_pairs + npairs * sizeof(BatchPair), 256);
  const size_t off_start = align_up(off_order + npairs * sizeof(int), 256);
  const size_t table_bytes = align_up(off_start + kBatchQueues * n1 * sizeof(int), 256);
  const size_t stage_bytes = table_bytes + sizeof(BatchWork);

  // The pinned staging buffer may be rewritten once the previous batch's
  // upload has run, which is as soon as that batch starts.  The device
  // tables and work list are rewritten by this batch's upload, queued on the
  // same stream behind the previous batch's kernels, so only a change of
  // stream, tables or staging that must grow, or a graph captured with other
  // launch choices (it does not match the tile numbering below) make the
  // host wait for the previous batch to finish.
  const bool retune = b.exec && !same_tuning(b.tune, dt.tune);
  if (b.launched) {
    const bool drain = s != b.last_stream || retune || table_bytes > b.d_tables_cap ||
                       stage_bytes > b.h_stage_cap;
    if ((e = hipEventSynchronize(drain ? b.done : b.staged)) != hipSuccess)
      return device_fail(ctx, e, "waiting for the previous batch");
  }
  if (retune) b.drop_graph();
  if (table_bytes > b.d_tables_cap) {
    if (b.d_tables) (void)hipFree(b.d_tables);
    b.d_tables = nullptr;
    b.d_tables_cap = 0;
    if ((e = hipMalloc(&b.d_tables, table_bytes)) != hipSuccess)
      return device_fail(ctx, e, "batch tables");
    b.d_tables_cap = table_bytes;
  }
  if (stage_bytes > b.h_stage_cap) {
    if (b.h_stage) (void)hipHostFree(b.h_stage);
    b.h_stage = nullptr;
    b.h_stage_cap = 0;
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&b.h_stage), stage_bytes,
                           hipHostMallocDefault)) != hipSuccess)
      return device_fail(ctx, e, "batch staging buffer");
    b.h_stage_cap = stage_bytes;
  }

  char *h = b.h_stage;
  BatchPair *hp = reinterpret_cast<BatchPair *>(h + off_pairs);
  int *horder = reinterpret_cast<int *>(h + off_order);
  int *hstart = reinterpret_cast<int *>(h + off_start);
  for (int i = 0; i < npairs; ++i) {
    const bsm_pair &p = pairs[i];
    const size_t px = (size_t)p.width * p.height;
    char *base = static_cast<char *>(scratch) + offset[i];
    BatchPair &q = hp[i];
    q.left = p.left;
    q.right = p.right;
    q.W = p.width;
    q.H = p.height;
    q.stride = p.stride;
    q.dmax = p.dmax;
    q.disp = p.disp;
    q.cost = p.cost;
    q.packedL = reinterpret_cast<uint32_t *>(base);
    q.packedR = reinterpret_cast<uint32_t *>(base + align_up(px * 4, 256));
    char *d0 = base + 2 * align_up(px * 4, 256);
    const size_t db = align_up(px * ctx->nw * 8, 256);
    q.descL = reinterpret_cast<uint64_t *>(d0);
    q.maskL = reinterpret_cast<uint64_t *>(d0 + db);
    q.descR = reinterpret_cast<uint64_t *>(d0 + 2 * db);
  }
  for (int q = 0; q < kBatchQueues; ++q) hstart[q * n1] = 0;
  for (int i = 0; i < npairs; ++i) {
    const bsm_pair &p = pairs[order[i]];
    horder[i] = order[i];
    int counts[kBatchQueues];
    batch_tile_counts(p.width, p.height, use_mask, p.cost != nullptr, dt.tune.desc_tile_w,
                      dt.tune.batch_tile_h, dt.tune.cost_mfma, counts);
    for (int q = 0; q < kBatchQueues; ++q) hstart[q * n1 + i + 1] = hstart[q * n1 + i] + counts[q];
  }
  BatchWork *hw = reinterpret_cast<BatchWork *>(h + table_bytes);
  hw->pairs = reinterpret_cast<const BatchPair *>(b.d_tables + off_pairs);
  hw->order = reinterpret_cast<const int *>(b.d_tables + off_order);
  hw->start = reinterpret_cast<const int *>(b.d_tables + off_start);
  hw->counters = b.d_counters;  // zeroed by the graph's first node
  hw->npairs = npairs;

  if ((e = hipMemcpyAsync(b.d_tables, h, table_bytes, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(b.d_work, hw, sizeof(BatchWork), hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return device_fail(ctx, e, "uploading the batch work list");
  if ((e = hipEventRecord(b.staged, s)) != hipSuccess) return device_fail(ctx, e, "batch event");

  if (marks) {
    const BatchLaunch bl{b.d_work, b.d_counters, marks};
    if ((e = launch_batch(bl, dt, use_mask, s)) != hipSuccess)
      return device_fail(ctx, e, "launching the batch stages");
  } else {
    const BatchLaunch bl{b.d_work, b.d_counters};
    if (!b.exec) {
      // Capture the stage launches once; they read everything else from the
      // work list, so the graph serves every later batch of this context.
      if ((e = hipStreamBeginCapture(b.capture, hipStreamCaptureModeRelaxed)) != hipSuccess)
        return device_fail(ctx, e, "beginning batch graph capture");
      hipError_t le = launch_batch(bl, dt, use_mask, b.capture);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(b.capture, &g);
      if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return device_fail(ctx, le != hipSuccess ? le : e, "capturing the batch graph");
      }
      b.graph = g;
      if ((e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0)) != hipSuccess) {
        b.drop_graph();
        return device_fail(ctx, e, "instantiating the batch graph");
      }
      b.tune = dt.tune;
    }
    if ((e = hipGraphLaunch(b.exec, s)) != hipSuccess)
      return device_fail(ctx, e, "launching the batch graph");
  }
  if ((e = hipEventRecord(b.done, s)) != hipSuccess) return device_fail(ctx, e, "batch event");
  b.launched = true;
  b.last_stream = s;
  if ((e = b.scratch.release(s)) != hipSuccess) return device_fail(ctx, e, "batch scratch event");
  return BSM_OK;
}

}  // namespace

bsm_status batch_run_marked(bsm_ctx *ctx, BatchState &b, const DeviceTables &dt,
                            const bsm_pair *pairs, int npairs, hipStream_t s,
                            const hipEvent_t *marks) {
  if (!batch_supported(ctx->nw) || npairs <= kSequentialMaxPairs)
    return fail(BSM_EINVAL, "stage times need the persistent path (n in {64, 128, 256, 512, "
                            "1024} and more than %d pairs)", kSequentialMaxPairs);
  return batch_persistent(ctx, b, dt, pairs, npairs, s, marks);
}

bsm_status batch_run(bsm_ctx *ctx, BatchState &b, const DeviceTables &dt, const bsm_pair *pairs,
                     int npairs, hipStream_t s) {
  // Up to kSequentialMaxPairs pairs run one after another with the per-pair
  // kernels (identical results): the persistent launch costs about 0.1 ms
  // more than it saves below five pairs, whatever their size (measured on
  // copies of the 128x96, 450x375 and 1400x1100 pairs: two to four of them
  // run 10-100 % faster pair by pair; six 450x375 pairs break even).
  if (!batch_supported(ctx->nw) || npairs <= kSequentialMaxPairs)
    return batch_sequential(ctx, b, pairs, npairs, s);
  return batch_persistent(ctx, b, dt, pairs, npairs, s);
}

namespace {

bsm_status ensure_batch_state(bsm_ctx *ctx) {
  if (ctx->batch) return BSM_OK;
  return batch_state_create(ctx, &ctx->batch);
}

bsm_status run_batch(bsm_ctx *ctx, const bsm_pair *pairs, int npairs, hipStream_t s) {
  bsm_status st = ensure_batch_state(ctx);
  if (st != BSM_OK) return st;
  return batch_run(ctx, *ctx->batch, ctx->dt, pairs, npairs, s);
}

// RAII device switch for the entry points of this file.
struct OnDevice {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit OnDevice(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~OnDevice() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace
}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_match_batch(bsm_ctx *ctx, const bsm_pair *pairs, int32_t npairs,
                                      void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_pairs(pairs, npairs)) != BSM_OK) return st;
  if (npairs == 0) return BSM_OK;
  OnDevice g(ctx->device);
  if (g.err != hipSuccess) return device_fail(ctx, g.err, "hipSetDevice");
  return run_batch(ctx, pairs, npairs, static_cast<hipStream_t>(hip_stream));
}

extern "C" bsm_status bsm_batch_stage_times(bsm_ctx *ctx, const bsm_pair *pairs,
                                            int32_t npairs, void *hip_stream,
                                            float *stage_ms) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_pairs(pairs, npairs)) != BSM_OK) return st;
  if (!stage_ms) return fail(BSM_EINVAL, "stage_ms is NULL");
  OnDevice g(ctx->device);
  if (g.err != hipSuccess) return device_fail(ctx, g.err, "hipSetDevice");
  if ((st = ensure_batch_state(ctx)) != BSM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipEvent_t ev[kBatchMarks] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < kBatchMarks && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  if (e == hipSuccess) {
    st = batch_run_marked(ctx, *ctx->batch, ctx->dt, pairs, npairs, s, ev);
    if (st == BSM_OK) e = hipEventSynchronize(ev[kBatchMarks - 1]);
    for (int i = 0; i < kBatchStages && st == BSM_OK && e == hipSuccess; ++i)
      e = hipEventElapsedTime(&stage_ms[i], ev[i], ev[i + 1]);
  }
  for (int i = 0; i < kBatchMarks; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  if (st != BSM_OK) return st;
  if (e != hipSuccess) return device_fail(ctx, e, "batch stage events");
  return BSM_OK;
}

namespace bsm {
namespace {

bool takes_persistent_path(const bsm_ctx *ctx, int npairs) {
  return batch_supported(ctx->nw) && npairs > kSequentialMaxPairs;
}

// Candidate tunings.  The persistent batch: describe tile width x height x
// share of the describe workgroups that start on the descriptor-only tiles
// (one in 3 .. 8) and, only when a pair has a volume (they belong to the
// bitwise kernel), cost window and cost occupancy.  Pairs run one by one
// (batches of up to four, single pairs): describe tile width x tile height
// x pixels per lane of the descriptor-only kernel x matrix-core or bitwise
// cost kernel (the latter only where the matrix-core kernel applies).
std::vector<Tuning> autotune_candidates(const bsm_ctx *ctx, const bsm_pair *pairs, int npairs) {
  bool any_volume = false, mfma_possible = false;
  for (int i = 0; i < npairs; ++i) {
    any_volume = any_volume || pairs[i].cost != nullptr;
    mfma_possible = mfma_possible ||
                    (pairs[i].dmax > 16 && (!pairs[i].cost || pairs[i].dmax <= 256));
  }
  std::vector<Tuning> out;
  if (takes_persistent_path(ctx, npairs)) {
    for (int tw : {16, 32})
      for (int th : {8, 16})
        for (int dc : {32, 64})
          for (int cost_bpc : {0, 2})
            for (int right_every : {3, 4, 5, 6, 8}) {
              if (!any_volume && (dc == 32 || cost_bpc == 2)) continue;
              Tuning t;
              t.desc_tile_w = tw;
              t.batch_tile_h = th;
              t.cost_dchunk = dc;
              t.blocks_per_cu[2] = right_every;
              t.blocks_per_cu[3] = cost_bpc;
              out.push_back(t);
            }
  } else {
    const bool fast_nw = batch_supported(ctx->nw);
    for (int tw : {16, 32})
      for (int th : {4, 8})
        for (int px : {1, 4})
          for (int mfma : {1, 0}) {
            if (mfma == 0 && !(mfma_possible && fast_nw)) continue;
            Tuning t;
            t.desc_tile_w = tw;
            t.pair_desc_th = th;
            t.pair_right_px = px;
            t.cost_mfma = mfma;
            out.push_back(t);
          }
  }
  return out;
}

// Times every candidate on `pairs` (one untimed run, then `reps` timed
// runs each) and returns the fastest with its mean time per call.
bsm_status autotune_search(bsm_ctx *ctx, const bsm_pair *pairs, int npairs, int reps,
                           hipStream_t s, Tuning *best_t, double *best_time) {
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return device_fail(ctx, e, "autotune events");
  }
  bsm_status st = BSM_OK;
  *best_t = ctx->dt.tune;
  *best_time = -1;
  for (const Tuning &cand : autotune_candidates(ctx, pairs, npairs)) {
    DeviceTables dt = ctx->dt;
    dt.tune = cand;
    if ((st = batch_run(ctx, *ctx->batch, dt, pairs, npairs, s)) != BSM_OK) break;
    if ((e = hipEventRecord(t0, s)) != hipSuccess) break;
    for (int r = 0; r < reps && st == BSM_OK; ++r)
      st = batch_run(ctx, *ctx->batch, dt, pairs, npairs, s);
    if (st != BSM_OK) break;
    if ((e = hipEventRecord(t1, s)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess)
      break;
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
    const double per = ms / reps;
    if (*best_time < 0 || per < *best_time) {
      *best_time = per;
      *best_t = cand;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st == BSM_OK && e != hipSuccess) st = device_fail(ctx, e, "autotune timing");
  return st;
}

void tuning_to_c(const Tuning &t, bsm_tuning *out) {
  out->desc_tile_w = t.desc_tile_w;
  out->cost_dchunk = t.cost_dchunk;
  for (int i = 0; i < 4; ++i) out->blocks_per_cu[i] = t.blocks_per_cu[i];
  out->cost_mfma = t.cost_mfma;
  out->batch_tile_h = t.batch_tile_h;
  out->pair_desc_th = t.pair_desc_th;
  out->pair_right_px = t.pair_right_px;
  out->mfma_min_dmax = t.mfma_min_dmax;
}

void set_context_tuning(bsm_ctx *ctx, const Tuning &t) {
  std::lock_guard<std::mutex> lk(ctx->tune_mu);
  ctx->dt.tune = t;
}

int pow2_at_least(double x) {
  int p = 1;
  while (p < x && p < (1 << 30)) p <<= 1;
  return p;
}

// Cache key: GPU architecture, n, S, mask mode and the shape class of the
// pairs (path, pair count, largest dmax, mean pixels in thousands, each
// rounded up to a power of two, and whether a volume is wanted).
std::string autotune_key(const bsm_ctx *ctx, const bsm_pair *pairs, int npairs) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  int max_dmax = 1;
  double px = 0;
  bool vol = false;
  for (int i = 0; i < npairs; ++i) {
    max_dmax = std::max(max_dmax, pairs[i].dmax);
    px += (double)pairs[i].width * pairs[i].height;
    vol = vol || pairs[i].cost != nullptr;
  }
  char buf[256];
  snprintf(buf, sizeof buf, "%s n%d S%d mask%d %s pairs%d dmax%d kpx%d vol%d", arch.c_str(),
           ctx->n, ctx->S, ctx->use_mask, takes_persistent_path(ctx, npairs) ? "batch" : "pairs",
           pow2_at_least(npairs), pow2_at_least(max_dmax), pow2_at_least(px / npairs / 1000.0),
           vol ? 1 : 0);
  return buf;
}

// The cache file is one JSON object with one entry per line:
//   "<key>": {"desc_tile_w": 32, ..., "ms": 52.9},
constexpr const char *kEntryFormat =
    "{\"desc_tile_w\": %d, \"cost_dchunk\": %d, \"blocks_per_cu\": [%d, %d, %d, %d], "
    "\"cost_mfma\": %d, \"batch_tile_h\": %d, \"pair_desc_th\": %d, \"pair_right_px\": %d, "
    "\"mfma_min_dmax\": %d, \"ms\": %lf}";

// Entries of the file as (key, rest of the line); unreadable lines are
// dropped.
std::vector<std::pair<std::string, std::string>> cache_read(const char *path) {
  std::vector<std::pair<std::string, std::string>> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    const size_t c = line.find('{', b == std::string::npos ? a : b);
    if (b == std::string::npos || c == std::string::npos) continue;
    std::string rest = line.substr(c);
    while (!rest.empty() && (rest.back() == ',' || rest.back() == ' ' || rest.back() == '\r'))
      rest.pop_back();
    out.emplace_back(line.substr(a + 1, b - a - 1), rest);
  }
  return out;
}

bool parse_entry(const std::string &text, Tuning *t, double *ms) {
  Tuning x;
  const int got = sscanf(text.c_str(), kEntryFormat, &x.desc_tile_w, &x.cost_dchunk,
                         &x.blocks_per_cu[0], &x.blocks_per_cu[1], &x.blocks_per_cu[2],
                         &x.blocks_per_cu[3], &x.cost_mfma, &x.batch_tile_h, &x.pair_desc_th,
                         &x.pair_right_px, &x.mfma_min_dmax, ms);
  if (got != 12) return false;
  bsm_tuning c;
  tuning_to_c(x, &c);
  if (check_tuning(&c) != BSM_OK) return false;
  *t = x;
  return true;
}

bool cache_write(const char *path, const std::vector<std::pair<std::string, std::string>> &e) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    for (size_t i = 0; i < e.size(); ++i)
      f << "\"" << e[i].first << "\": " << e[i].second << (i + 1 < e.size() ? ",\n" : "\n");
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace
}  // namespace bsm

extern "C" bsm_status bsm_autotune(bsm_ctx *ctx, const bsm_pair *pairs, int32_t npairs,
                                   int32_t reps, void *hip_stream, bsm_tuning *best,
                                   double *best_ms) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_pairs(pairs, npairs)) != BSM_OK) return st;
  if (npairs < 1 || reps < 1 || reps > 1000)
    return fail(BSM_EINVAL, "need npairs >= 1 and 1 <= reps <= 1000");
  OnDevice g(ctx->device);
  if (g.err != hipSuccess) return device_fail(ctx, g.err, "hipSetDevice");
  if ((st = ensure_batch_state(ctx)) != BSM_OK) return st;
  Tuning best_t;
  double best_time = -1;
  st = autotune_search(ctx, pairs, npairs, reps, static_cast<hipStream_t>(hip_stream), &best_t,
                       &best_time);
  if (st != BSM_OK) return st;
  set_context_tuning(ctx, best_t);
  if (best) tuning_to_c(best_t, best);
  if (best_ms) *best_ms = best_time;
  return BSM_OK;
}

extern "C" bsm_status bsm_autotune_cached(bsm_ctx *ctx, const bsm_pair *pairs, int32_t npairs,
                                          int32_t reps, void *hip_stream, const char *cache_path,
                                          bsm_tuning *best, double *best_ms, int32_t *hit) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_pairs(pairs, npairs)) != BSM_OK) return st;
  if (npairs < 1 || reps < 1 || reps > 1000)
    return fail(BSM_EINVAL, "need npairs >= 1 and 1 <= reps <= 1000");
  if (hit) *hit = 0;
  const std::string key = cache_path ? autotune_key(ctx, pairs, npairs) : std::string();
  std::vector<std::pair<std::string, std::string>> entries;
  if (cache_path) {
    entries = cache_read(cache_path);
    for (const auto &en : entries) {
      Tuning t;
      double ms = 0;
      if (en.first == key && parse_entry(en.second, &t, &ms)) {
        set_context_tuning(ctx, t);
        if (best) tuning_to_c(t, best);
        if (best_ms) *best_ms = ms;
        if (hit) *hit = 1;
        return BSM_OK;
      }
    }
  }
  OnDevice g(ctx->device);
  if (g.err != hipSuccess) return device_fail(ctx, g.err, "hipSetDevice");
  if ((st = ensure_batch_state(ctx)) != BSM_OK) return st;
  Tuning best_t;
  double best_time = -1;
  st = autotune_search(ctx, pairs, npairs, reps, static_cast<hipStream_t>(hip_stream), &best_t,
                       &best_time);
  if (st != BSM_OK) return st;
  set_context_tuning(ctx, best_t);
  if (best) tuning_to_c(best_t, best);
  if (best_ms) *best_ms = best_time;
  if (cache_path) {
    char text[512];
    snprintf(text, sizeof text, kEntryFormat, best_t.desc_tile_w, best_t.cost_dchunk,
             best_t.blocks_per_cu[0], best_t.blocks_per_cu[1], best_t.blocks_per_cu[2],
             best_t.blocks_per_cu[3], best_t.cost_mfma, best_t.batch_tile_h, best_t.pair_desc_th,
             best_t.pair_right_px, best_t.mfma_min_dmax, best_time);
    bool replaced = false;
    for (auto &en : entries)
      if (en.first == key) {
        en.second = text;
        replaced = true;
      }
    if (!replaced) entries.emplace_back(key, text);
    if (!cache_write(cache_path, entries))
      return fail(BSM_EINVAL, "tuned, but could not write the cache file %s", cache_path);
  }
  return BSM_OK;
}
