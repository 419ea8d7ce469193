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
#include <map>

#include "bsm_internal.h"
#include "bsm_serve_core.h"

namespace bsm {

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Pinned host buffers kept for reuse, keyed by size.
class PinnedPool {
 public:
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
    free_[size_[p]].push_back(p);
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void *>> free_;
  std::map<void *, size_t> size_;
};

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
    s.device.assign(group.size(), nullptr);
    std::vector<bsm_pair> pairs(group.size());
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
      s.device[i] = d;
      // compact the caller's rows into pinned memory, then copy to the device
      const size_t row = (size_t)p.width * 3;
      for (int v = 0; v < p.height; ++v) {
        std::memcpy(h + v * row, p.left + (size_t)v * p.stride, row);
        std::memcpy(h + L.img + v * row, p.right + (size_t)v * p.stride, row);
      }
      ok = hipMemcpyAsync(d, h, L.in_bytes, hipMemcpyHostToDevice, s.stream) == hipSuccess;
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
      DeviceTables dt;
      {
        std::lock_guard<std::mutex> lk(ctx_->tune_mu);
        dt = ctx_->dt;
      }
      ok = batch_run(ctx_, *s.batch, dt, pairs.data(), (int)pairs.size(), s.stream) == BSM_OK;
    }
    for (size_t i = 0; i < group.size(); ++i) {
      if (!s.device[i]) continue;
      if (ok) {
        const Layout L(group[i]->pair);
        ok = hipMemcpyAsync(static_cast<char *>(s.pinned[i]) + L.in_bytes,
                            static_cast<char *>(s.device[i]) + L.in_bytes, L.total - L.in_bytes,
                            hipMemcpyDeviceToHost, s.stream) == hipSuccess;
      }
      (void)hipFreeAsync(s.device[i], s.stream);
      s.device[i] = nullptr;
    }
    if (ok) ok = hipEventRecord(s.event, s.stream) == hipSuccess;
    if (!ok) release(s);
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
    for (size_t i = 0; i < group.size(); ++i) {
      const bsm_pair &p = group[i]->pair;
      const Layout L(p);
      const char *h = static_cast<const char *>(s.pinned[i]);
      std::memcpy(p.disp, h + L.in_bytes, (size_t)p.width * p.height * 4);
      if (p.cost)
        std::memcpy(p.cost, h + L.in_bytes + L.disp, (size_t)p.width * p.height * p.dmax * 2);
    }
    release(s);
    return true;
  }

 private:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    BatchState *batch = nullptr;
    std::vector<void *> pinned, device;
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
};

constexpr size_t kDefaultCap = size_t(32) << 30;  // 32 GiB
constexpr int kDefaultQueue = 4096;
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
                   kDefaultQueue);
  return ctx->server;
}

}  // namespace

void server_stop(Server *s) { delete s; }

}  // namespace bsm

using namespace bsm;

extern "C" {

bsm_status bsm_serve_config(bsm_ctx *ctx, size_t cap_bytes, int32_t max_queue) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (cap_bytes == 0 || max_queue < 1)
    return fail(BSM_EINVAL, "cap_bytes must be > 0 and max_queue >= 1");
  server_of(ctx)->configure(cap_bytes, max_queue);
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
