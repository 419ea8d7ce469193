// Serving core (no HIP): see bsm_serve_core.h.
#include "bsm_serve_core.h"

#include <algorithm>

namespace bsm {

// Clock of the server's timed waits.  GCC 11's ThreadSanitizer does not
// intercept pthread_cond_clockwait, which libstdc++ uses for steady-clock
// waits, and then reports false double locks; the sanitizer build of the
// tests waits on the system clock (pthread_cond_timedwait) instead.
#ifdef BSM_TSAN_SYSTEM_CLOCK_WAITS
using WaitClock = std::chrono::system_clock;
#else
using WaitClock = std::chrono::steady_clock;
#endif

double Server::now() {
  return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

Server::Server(std::unique_ptr<Executor> exec, size_t cap_bytes, int max_queue, int max_group)
    : exec_(std::move(exec)), cap_(cap_bytes), max_queue_(max_queue), max_group_(max_group) {
  running_.resize(exec_->slots());
  thread_ = std::thread([this] { loop(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  wake_.notify_all();
  if (thread_.joinable()) thread_.join();
}

void Server::configure(size_t cap_bytes, int max_queue, int max_group) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    cap_ = cap_bytes;
    max_queue_ = max_queue;
    max_group_ = max_group;
  }
  wake_.notify_all();
}

bsm_status Server::submit(const bsm_pair &pair, size_t bytes, uint64_t *ticket) {
  const double t = now();
  std::lock_guard<std::mutex> lk(mu_);
  if (bytes > cap_) return BSM_ETOOBIG;
  if ((int)waiting_.size() >= max_queue_) return BSM_EAGAIN;
  std::unique_ptr<Request> r(new Request);
  r->ticket = next_ticket_++;
  r->pair = pair;
  r->bytes = bytes;
  r->times.t_arrive = t;
  waiting_.push_back(r.get());
  *ticket = r->ticket;
  all_[r->ticket] = std::move(r);
  ++unfinished_;
  ++stats_.submitted;
  wake_.notify_all();
  return BSM_OK;
}

bsm_status Server::poll(uint64_t ticket, int32_t *state, bsm_times *times) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) return BSM_ENOTFOUND;
  Request &r = *it->second;
  if (state) *state = r.state;
  if (times) *times = r.times;
  if (r.state != 0) all_.erase(it);  // reported once, then forgotten
  return BSM_OK;
}

void Server::drain() {
  std::unique_lock<std::mutex> lk(mu_);
  idle_.wait(lk, [this] { return unfinished_ == 0 || stop_; });
}

Server::Stats Server::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  return stats_;
}

void Server::finish_group(int slot, bool ok) {
  std::vector<Request *> group;
  {
    std::lock_guard<std::mutex> lk(mu_);
    group.swap(running_[slot]);
  }
  if (ok) ok = exec_->finish(slot, group);
  const double t = now();
  {
    std::lock_guard<std::mutex> lk(mu_);
    for (Request *r : group) {
      r->state = ok ? 1 : -1;
      r->times.t_end = t;
      in_flight_ -= r->bytes;
      --unfinished_;
      if (ok)
        ++stats_.completed;
      else
        ++stats_.failed;
    }
  }
  idle_.notify_all();
  wake_.notify_all();
}

void Server::loop() {
  const int slots = (int)running_.size();
  for (;;) {
    // 1. Retire finished groups.
    bool busy = false;
    for (int s = 0; s < slots; ++s) {
      bool has;
      {
        std::lock_guard<std::mutex> lk(mu_);
        has = !running_[s].empty();
      }
      if (!has) continue;
      const int q = exec_->query(s);
      if (q != 0)
        finish_group(s, q == 1);
      else
        busy = true;
    }
    // 2. Admit waiting requests onto a free slot (FIFO, under the cap).
    int free_slot = -1;
    std::vector<Request *> group;
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (stop_ && waiting_.empty() && !busy) break;
      int busy_slots = 0;
      for (int s = 0; s < slots; ++s) {
        if (running_[s].empty() && free_slot < 0) free_slot = s;
        busy_slots += running_[s].empty() ? 0 : 1;
      }
      if (free_slot >= 0) {
        const double t = now();
        while (!waiting_.empty() && (int)group.size() < max_group_ &&
               in_flight_ + waiting_.front()->bytes <= cap_) {
          Request *r = waiting_.front();
          waiting_.pop_front();
          r->times.t_admit = t;
          in_flight_ += r->bytes;
          group.push_back(r);
        }
        if (!group.empty()) {
          running_[free_slot] = group;
          ++stats_.groups;
          stats_.max_group = std::max<int>(stats_.max_group, (int)group.size());
          stats_.max_in_flight_bytes = std::max(stats_.max_in_flight_bytes, in_flight_);
          stats_.max_slots_busy = std::max(stats_.max_slots_busy, busy_slots + 1);
        }
      }
      if (group.empty() && !busy && free_slot >= 0 && !waiting_.empty()) {
        // Nothing runs and the head still does not fit: the cap was lowered
        // below its footprint after it was queued.  It can never run.
        Request *r = waiting_.front();
        waiting_.pop_front();
        r->state = -1;
        r->times.t_end = now();
        --unfinished_;
        ++stats_.failed;
        idle_.notify_all();
        continue;
      }
      if (group.empty()) {
        // Nothing to start: sleep until a submit, or briefly while work runs.
        if (busy)
          wake_.wait_until(lk, WaitClock::now() + std::chrono::microseconds(20));
        else if (waiting_.empty() || free_slot < 0)
          wake_.wait_until(lk, WaitClock::now() + std::chrono::milliseconds(5),
                           [this] { return stop_ || !waiting_.empty(); });
        continue;
      }
    }
    // 3. Start the group outside the lock.
    {
      std::lock_guard<std::mutex> lk(mu_);
      const double t = now();
      for (Request *r : group) r->times.t_start = t;
    }
    if (!exec_->start(free_slot, group)) finish_group(free_slot, false);
  }
}

}  // namespace bsm
