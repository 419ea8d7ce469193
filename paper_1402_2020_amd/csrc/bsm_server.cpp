// Serving on the GPU: the HIP executor behind the serving core, and the C
// entry points bsm_serve_config / bsm_submit / bsm_poll / bsm_drain.
//
// Each executor slot owns a stream, an event and its own batch state (work
// list, scratch and captured graph).  A group of admitted requests is staged
// into pinned host memory, copied to device buffers taken from the device's
// stream-ordered memory pool, matched as one batch and copied back; groups on
// different slots overlap on the device.  When the slot's event completes,
// the results are copied from pinned memory into the caller's buffers.
#include <cstring>
#include <functional>
#include <map>

#include "bsm_internal.h"
#include "bsm_serve_core.h"

namespace bsm {

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Pinned host buffers kept for reuse, keyed by size.  At most kCachedBytes
// of idle buffers are kept; beyond that a returned buffer is freed.
class PinnedPool {
 public:
  static constexpr size_t kCachedBytes = size_t(2) << 30;
  ~PinnedPool() {
    for (auto &kv : free_)
      for (void *p : kv.second) (void)hipHostFree(p);
  }
  void *get(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.lower_bound(bytes);
    if (it != free_.end() && it->first <= 2 * bytes && !it->second.empty()) {
      void *p = it->second.back();
      it->second.pop_back();
      cached_ -= it->first;
      size_[p] = it->first;
      return p;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    size_[p] = bytes;
    return p;
  }
  void put(void *p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = size_.find(p);
    const size_t bytes = it->second;
    size_.erase(it);
    if (cached_ + bytes > kCachedBytes) {
      (void)hipHostFree(p);
      return;
    }
    free_[bytes].push_back(p);
    cached_ += bytes;
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void *>> free_;  // idle buffers by size
  std::map<void *, size_t> size_;               // buffers handed out
  size_t cached_ = 0;                           // bytes in free_
};

// A few host threads that run copy tasks beside the calling thread.  Host
// copies between the caller's pageable buffers and pinned staging are the
// serving path's host-side cost; spreading them over threads keeps the
// server thread free to retire and admit.
class CopyPool {
 public:
  explicit CopyPool(int workers) {
    for (int i = 0; i < workers; ++i) threads_.emplace_back([this] { work(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : threads_) t.join();
  }
  // Runs fn(i) for i in [0, n) on the workers and the calling thread and
  // returns when all calls have returned.  One run at a time.
  void run(int n, const std::function<void(int)> &fn) {
    if (n <= 0) return;
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_ = 0;
      pending_ = n;
      ++gen_;
    }
    cv_.notify_all();
    drain_tasks();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [this] { return pending_ == 0; });
    fn_ = nullptr;
  }

 private:
  void drain_tasks() {
    for (;;) {
      int i;
      const std::function<void(int)> *fn;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (!fn_ || next_ >= n_) return;
        i = next_++;
        fn = fn_;
      }
      (*fn)(i);
      bool last;
      {
        std::lock_guard<std::mutex> lk(mu_);
        last = --pending_ == 0;
      }
      if (last) done_.notify_all();
    }
  }
  void work() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      drain_tasks();
    }
  }

  std::mutex mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)> *fn_ = nullptr;
  int n_ = 0, next_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
  std::vector<std::thread> threads_;
};

// One strided block copy (rows of `bytes` bytes).
struct CopyTask {
  char *dst;
  const char *src;
  size_t dst_pitch, src_pitch, bytes;
  int rows;
};

// Appends the copy of `rows` rows as tasks of about 512 KiB each.
void add_rows(std::vector<CopyTask> &tasks, char *dst, size_t dst_pitch, const char *src,
              size_t src_pitch, size_t bytes, int rows) {
  const int per = (int)std::max<size_t>(1, (512 << 10) / std::max<size_t>(bytes, 1));
  for (int r = 0; r < rows; r += per)
    tasks.push_back(CopyTask{dst + r * dst_pitch, src + r * src_pitch, dst_pitch, src_pitch, bytes,
                             std::min(per, rows - r)});
}

void run_copies(CopyPool &pool, const std::vector<CopyTask> &tasks) {
  pool.run((int)tasks.size(), [&](int i) {
    const CopyTask &t = tasks[i];
    if (t.dst_pitch == t.bytes && t.src_pitch == t.bytes) {
      std::memcpy(t.dst, t.src, t.bytes * t.rows);
      return;
    }
    for (int r = 0; r < t.rows; ++r) std::memcpy(t.dst + r * t.dst_pitch, t.src + r * t.src_pitch, t.bytes);
  });
}

// Layout of one request's device buffer and pinned staging buffer.
struct Layout {
  size_t img, disp, cost, total, in_bytes;
  explicit Layout(const bsm_pair &p) {
    const size_t px = (size_t)p.width * p.height;
    img = align256(px * 3);                     // compact RGB, one view
    disp = align256(px * 4);
    cost = p.cost ? align256(px * p.dmax * 2) : 0;
    in_bytes = 2 * img;
    total = 2 * img + disp + cost;
  }
};

constexpr int kCopyThreads = 3;  // plus the server thread

class HipExecutor : public Executor {
 public:
  HipExecutor(bsm_ctx *ctx, int nslots) : ctx_(ctx), slots_(nslots) {}
  ~HipExecutor() override {
    for (Slot &s : slots_) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.batch) batch_state_free(s.batch);
      if (s.event) (void)hipEventDestroy(s.event);
      if (s.stream) (void)hipStreamDestroy(s.stream);
    }
  }
  int slots() const override { return (int)slots_.size(); }

  bool start(int slot, const std::vector<Request *> &group) override {
    Slot &s = slots_[slot];
    if (hipSetDevice(ctx_->device) != hipSuccess) return false;
    if (!s.stream && !init(s)) return false;
    s.pinned.assign(group.size(), nullptr);
    std::vector<char *> device(group.size(), nullptr);
    std::vector<bsm_pair> pairs(group.size());
    std::vector<CopyTask> tasks;
    bool ok = true;
    for (size_t i = 0; i < group.size() && ok; ++i) {
      const bsm_pair &p = group[i]->pair;
      const Layout L(p);
      char *h = static_cast<char *>(pool_.get(L.total));
      char *d = nullptr;
      if (!h || hipMallocAsync(reinterpret_cast<void **>(&d), L.total, s.stream) != hipSuccess) {
        if (h) pool_.put(h);
        ok = false;
        break;
      }
      s.pinned[i] = h;
      device[i] = d;
      // the caller's rows, compacted into pinned memory
      const size_t row = (size_t)p.width * 3;
      add_rows(tasks, h, row, reinterpret_cast<const char *>(p.left), p.stride, row, p.height);
      add_rows(tasks, h + L.img, row, reinterpret_cast<const char *>(p.right), p.stride, row,
               p.height);
      pairs[i] = bsm_pair{reinterpret_cast<const uint8_t *>(d),
                          reinterpret_cast<const uint8_t *>(d + L.img),
                          p.width,
                          p.height,
                          p.width * 3,
                          p.dmax,
                          reinterpret_cast<int32_t *>(d + L.in_bytes),
                          p.cost ? reinterpret_cast<int16_t *>(d + L.in_bytes + L.disp) : nullptr};
    }
    if (ok) {
      run_copies(copies_, tasks);
      for (size_t i = 0; i < group.size() && ok; ++i)
        ok = hipMemcpyAsync(device[i], s.pinned[i], Layout(group[i]->pair).in_bytes,
                            hipMemcpyHostToDevice, s.stream) == hipSuccess;
    }
    if (ok) {
      DeviceTables dt;
      {
        std::lock_guard<std::mutex> lk(ctx_->tune_mu);
        dt = ctx_->dt;
      }
      ok = batch_run(ctx_, *s.batch, dt, pairs.data(), (int)pairs.size(), s.stream) == BSM_OK;
    }
    for (size_t i = 0; i < group.size(); ++i) {
      if (!device[i]) continue;
      if (ok) {
        const Layout L(group[i]->pair);
        ok = hipMemcpyAsync(static_cast<char *>(s.pinned[i]) + L.in_bytes, device[i] + L.in_bytes,
                            L.total - L.in_bytes, hipMemcpyDeviceToHost, s.stream) == hipSuccess;
      }
      (void)hipFreeAsync(device[i], s.stream);
    }
    if (ok) ok = hipEventRecord(s.event, s.stream) == hipSuccess;
    if (!ok) {
      // nothing may still write the pinned buffers when they go back
      (void)hipStreamSynchronize(s.stream);
      release(s);
    }
    return ok;
  }

  int query(int slot) override {
    const hipError_t e = hipEventQuery(slots_[slot].event);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    release(slots_[slot]);
    return -1;
  }

  bool finish(int slot, const std::vector<Request *> &group) override {
    Slot &s = slots_[slot];
    std::vector<CopyTask> tasks;
    for (size_t i = 0; i < group.size(); ++i) {
      const bsm_pair &p = group[i]->pair;
      const Layout L(p);
      const char *h = static_cast<const char *>(s.pinned[i]);
      const size_t row = (size_t)p.width * 4;
      add_rows(tasks, reinterpret_cast<char *>(p.disp), row, h + L.in_bytes, row, row, p.height);
      if (p.cost)
        add_rows(tasks, reinterpret_cast<char *>(p.cost), row / 2, h + L.in_bytes + L.disp, row / 2,
                 row / 2, p.height * p.dmax);
    }
    run_copies(copies_, tasks);
    release(s);
    return true;
  }

 private:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    BatchState *batch = nullptr;
    std::vector<void *> pinned;  // staging of the group in flight
  };

  bool init(Slot &s) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&s.event, hipEventDisableTiming) != hipSuccess) return false;
    if (batch_state_create(ctx_, &s.batch) != BSM_OK) return false;
    // keep freed device memory in the pool for the next requests
    hipMemPool_t mp;
    if (hipDeviceGetDefaultMemPool(&mp, ctx_->device) == hipSuccess) {
      uint64_t keep = UINT64_MAX;
      (void)hipMemPoolSetAttribute(mp, hipMemPoolAttrReleaseThreshold, &keep);
    }
    return true;
  }

  void release(Slot &s) {
    for (void *&p : s.pinned)
      if (p) {
        pool_.put(p);
        p = nullptr;
      }
  }

  bsm_ctx *ctx_;
  std::vector<Slot> slots_;
  PinnedPool pool_;
  CopyPool copies_{kCopyThreads};
};

constexpr size_t kDefaultCap = size_t(32) << 30;  // 32 GiB
constexpr int kDefaultQueue = 4096;
constexpr int kDefaultGroup = 4;
constexpr int kSlots = 3;

// Device bytes one request holds while admitted: its buffers (images,
// disparity, volume) and the batch scratch of the pair.
size_t request_bytes(const bsm_ctx *ctx, const bsm_pair &p) {
  const Layout L(p);
  const size_t px = (size_t)p.width * p.height;
  return L.total + 2 * align256(px * 4) + 3 * align256(px * ctx->nw * 8);
}

Server *server_of(bsm_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  if (!ctx->server)
    ctx->server =
        new Server(std::unique_ptr<Executor>(new HipExecutor(ctx, kSlots)), kDefaultCap,
                   kDefaultQueue, kDefaultGroup);
  return ctx->server;
}

}  // namespace

void server_stop(Server *s) { delete s; }

}  // namespace bsm

using namespace bsm;

extern "C" {

bsm_status bsm_serve_config(bsm_ctx *ctx, size_t cap_bytes, int32_t max_queue,
                            int32_t max_group) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (cap_bytes == 0 || max_queue < 1 || max_group < 0)
    return fail(BSM_EINVAL, "need cap_bytes > 0, max_queue >= 1 and max_group >= 0");
  server_of(ctx)->configure(cap_bytes, max_queue, max_group ? max_group : kDefaultGroup);
  return BSM_OK;
}

bsm_status bsm_serve_stats(bsm_ctx *ctx, bsm_serve_counters *out) {
  clear_error();
  if (!ctx || !out) return fail(BSM_EINVAL, "context and out must not be NULL");
  Server *s;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    s = ctx->server;
  }
  *out = bsm_serve_counters{};
  if (!s) return BSM_OK;
  const Server::Stats st = s->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->failed = st.failed;
  out->groups = st.groups;
  out->max_in_flight_bytes = st.max_in_flight_bytes;
  out->max_group = st.max_group;
  out->max_slots_busy = st.max_slots_busy;
  return BSM_OK;
}

bsm_status bsm_submit(bsm_ctx *ctx, const bsm_pair *pair, uint64_t *ticket) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (!pair || !ticket) return fail(BSM_EINVAL, "pair and ticket must not be NULL");
  if ((st = validate_image(pair->left, pair->width, pair->height, pair->stride)) != BSM_OK ||
      (st = validate_image(pair->right, pair->width, pair->height, pair->stride)) != BSM_OK ||
      (st = validate_dmax(pair->width, pair->dmax)) != BSM_OK)
    return st;
  if (!pair->disp) return fail(BSM_EINVAL, "disp must not be NULL");
  st = server_of(ctx)->submit(*pair, request_bytes(ctx, *pair), ticket);
  if (st == BSM_ETOOBIG) return fail(st, "pair needs more device memory than the admission cap");
  if (st == BSM_EAGAIN) return fail(st, "serving queue is full");
  return st;
}

bsm_status bsm_poll(bsm_ctx *ctx, uint64_t ticket, int32_t *state, bsm_times *times) {
  clear_error();
  if (!ctx) return fail(BSM_EINVAL, "context is NULL");
  Server *s;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    s = ctx->server;
  }
  if (!s) return fail(BSM_ENOTFOUND, "no request was submitted");
  bsm_status st = s->poll(ticket, state, times);
  if (st == BSM_ENOTFOUND) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
  return st;
}

bsm_status bsm_drain(bsm_ctx *ctx) {
  clear_error();
  if (!ctx) return fail(BSM_EINVAL, "context is NULL");
  Server *s;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    s = ctx->server;
  }
  if (s) s->drain();
  return BSM_OK;
}

}  // extern "C"
