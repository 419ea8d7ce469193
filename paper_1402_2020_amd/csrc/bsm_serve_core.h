// Serving core: admission, continuous batching and ticket bookkeeping.
//
// No HIP here.  The device work goes through the Executor interface, so the
// same scheduler runs with the HIP executor in the library and with a fake
// executor in CPU tests.
//
// Requests wait in arrival order.  Whenever an executor slot is free, the
// server admits the longest prefix of the waiting queue (at most max_group
// requests) whose device footprints fit under the cap next to everything in
// flight, hands that group to the slot and goes on; groups on different
// slots run at the same time.  A request is in one of: waiting, running,
// done or failed.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/bsm.h"

namespace bsm {

struct Request {
  uint64_t ticket = 0;
  bsm_pair pair{};        // host pointers given to bsm_submit
  size_t bytes = 0;       // device footprint counted against the cap
  int state = 0;          // 0 pending, 1 done, -1 failed
  bsm_times times{};
};

// Device side of serving: `slots()` independent lanes of work.
class Executor {
 public:
  virtual ~Executor() = default;
  virtual int slots() const = 0;
  // Starts the group on a free slot; false on failure (the group fails).
  virtual bool start(int slot, const std::vector<Request *> &group) = 0;
  // 1: finished, 0: still running, -1: failed.
  virtual int query(int slot) = 0;
  // Called once after query() returned 1 (results to the caller's buffers).
  virtual bool finish(int slot, const std::vector<Request *> &group) = 0;
};

class Server {
 public:
  using Clock = std::chrono::steady_clock;
  Server(std::unique_ptr<Executor> exec, size_t cap_bytes, int max_queue, int max_group);
  ~Server();  // stops the thread after the work in flight ends

  void configure(size_t cap_bytes, int max_queue, int max_group);
  // BSM_ETOOBIG if bytes > cap; BSM_EAGAIN if the waiting queue is full.
  bsm_status submit(const bsm_pair &pair, size_t bytes, uint64_t *ticket);
  // BSM_ENOTFOUND for unknown (or already reported finished) tickets.
  bsm_status poll(uint64_t ticket, int32_t *state, bsm_times *times);
  void drain();
  // Seconds on the clock the timestamps use.
  static double now();

  struct Stats {
    uint64_t submitted = 0, completed = 0, failed = 0, groups = 0;
    size_t max_in_flight_bytes = 0;
    int max_group = 0, max_slots_busy = 0;
  };
  Stats stats();

 private:
  void loop();
  void finish_group(int slot, bool ok);

  std::unique_ptr<Executor> exec_;
  std::mutex mu_;
  std::condition_variable wake_;   // new work, stop
  std::condition_variable idle_;   // something finished
  std::deque<Request *> waiting_;
  std::map<uint64_t, std::unique_ptr<Request>> all_;
  std::vector<std::vector<Request *>> running_;  // per slot
  size_t cap_ = 0, in_flight_ = 0;
  int max_queue_ = 0, max_group_ = 1;
  uint64_t next_ticket_ = 1;
  uint64_t unfinished_ = 0;  // waiting + running
  bool stop_ = false;
  Stats stats_;
  std::thread thread_;
};

}  // namespace bsm
