// Test shim: the serving core (bsm_serve_core.cpp) driven by a fake executor,
// so admission, batching and ticket handling can be tested on the CPU.
//
// The fake executor "runs" a group for a fixed time per slot and writes, for
// every request, disp[i] = left[3 i] + right[3 i] + dmax, so tests can check
// that each result belongs to its own request.  It can be told to fail the
// next groups at start or at completion.
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>

#include "../paper_1402_2020_amd/csrc/bsm_serve_core.h"

using namespace bsm;

namespace {

class FakeExecutor : public Executor {
 public:
  FakeExecutor(int slots, double work_ms) : end_(slots), work_ms_(work_ms) {}
  int slots() const override { return (int)end_.size(); }
  bool start(int slot, const std::vector<Request *> &group) override {
    if (fail_start_ > 0) {
      --fail_start_;
      return false;
    }
    for (Request *r : group) {
      const bsm_pair &p = r->pair;
      for (int i = 0; i < p.width * p.height; ++i)
        p.disp[i] = p.left[3 * i] + p.right[3 * i] + p.dmax;
    }
    end_[slot] = Server::now() + work_ms_ * 1e-3;
    fail_[slot] = fail_finish_ > 0 ? (--fail_finish_, true) : false;
    return true;
  }
  int query(int slot) override {
    if (Server::now() < end_[slot]) return 0;
    return fail_[slot] ? -1 : 1;
  }
  bool finish(int, const std::vector<Request *> &) override { return true; }
  std::atomic<int> fail_start_{0}, fail_finish_{0};

 private:
  std::vector<double> end_;
  bool fail_[64] = {};
  double work_ms_;
};

struct Shim {
  FakeExecutor *exec;
  Server *server;
};

}  // namespace

extern "C" {

void *shim_create(size_t cap, int max_queue, int slots, double work_ms, int max_group) {
  auto *e = new FakeExecutor(slots, work_ms);
  auto *s = new Shim{e, nullptr};
  s->server = new Server(std::unique_ptr<Executor>(e), cap, max_queue, max_group);
  return s;
}

void shim_destroy(void *h) {
  auto *s = static_cast<Shim *>(h);
  delete s->server;
  delete s;
}

void shim_configure(void *h, size_t cap, int max_queue, int max_group) {
  static_cast<Shim *>(h)->server->configure(cap, max_queue, max_group);
}

int shim_submit(void *h, const uint8_t *left, const uint8_t *right, int W, int H, int dmax,
                int32_t *disp, size_t bytes, uint64_t *ticket) {
  bsm_pair p{left, right, W, H, 3 * W, dmax, disp, nullptr};
  return static_cast<Shim *>(h)->server->submit(p, bytes, ticket);
}

int shim_poll(void *h, uint64_t ticket, int32_t *state, double *times4) {
  bsm_times t{};
  const int st = static_cast<Shim *>(h)->server->poll(ticket, state, &t);
  if (times4) {
    times4[0] = t.t_arrive;
    times4[1] = t.t_admit;
    times4[2] = t.t_start;
    times4[3] = t.t_end;
  }
  return st;
}

void shim_drain(void *h) { static_cast<Shim *>(h)->server->drain(); }

void shim_fail(void *h, int at_start, int at_finish) {
  static_cast<Shim *>(h)->exec->fail_start_ = at_start;
  static_cast<Shim *>(h)->exec->fail_finish_ = at_finish;
}

// submitted, completed, failed, groups, max_in_flight_bytes, max_group, max_slots_busy
void shim_stats(void *h, uint64_t *out7) {
  const Server::Stats st = static_cast<Shim *>(h)->server->stats();
  out7[0] = st.submitted;
  out7[1] = st.completed;
  out7[2] = st.failed;
  out7[3] = st.groups;
  out7[4] = st.max_in_flight_bytes;
  out7[5] = (uint64_t)st.max_group;
  out7[6] = (uint64_t)st.max_slots_busy;
}

double shim_now() { return Server::now(); }

}  // extern "C"

#ifdef SHIM_STRESS_MAIN
// Stand-alone stress run for ThreadSanitizer: 4 client threads submit,
// poll and drain concurrently.  Exit code 0 iff every request completed with
// its own result.
#include <cstdio>
#include <vector>
int main() {
  void *h = shim_create(1000, 64, 3, 0.2, 4);
  std::atomic<int> bad{0};
  std::vector<std::thread> clients;
  for (int c = 0; c < 4; ++c)
    clients.emplace_back([&, c] {
      const int W = 8, H = 4;
      for (int k = 0; k < 200; ++k) {
        std::vector<uint8_t> L(3 * W * H, (uint8_t)(c + k)), R(3 * W * H, (uint8_t)k);
        std::vector<int32_t> D(W * H, -1);
        uint64_t t = 0;
        int st;
        while ((st = shim_submit(h, L.data(), R.data(), W, H, c, D.data(), 100 + k % 300, &t)) ==
               BSM_EAGAIN)
          std::this_thread::yield();
        if (st != BSM_OK) {
          ++bad;
          continue;
        }
        int32_t state = 0;
        do {
          std::this_thread::yield();
          if (shim_poll(h, t, &state, nullptr) != BSM_OK) {
            ++bad;
            break;
          }
        } while (state == 0);
        if (state != 1 || D[0] != (uint8_t)(c + k) + (uint8_t)k + c) ++bad;
      }
    });
  for (auto &t : clients) t.join();
  shim_drain(h);
  uint64_t stats[7];
  shim_stats(h, stats);
  shim_destroy(h);
  std::printf("bad=%d submitted=%llu completed=%llu groups=%llu max_bytes=%llu\n", bad.load(),
              (unsigned long long)stats[0], (unsigned long long)stats[1],
              (unsigned long long)stats[3], (unsigned long long)stats[4]);
  return bad.load() == 0 && stats[4] <= 1000 ? 0 : 1;
}
#endif
