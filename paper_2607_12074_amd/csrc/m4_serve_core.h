// m4_serve_core.h -- the host side of the serving loop: request queue,
// first-come first-served admission against a device-memory budget, lanes of
// fused launches and the worker for graphs beyond one workgroup.  It holds no
// device code and includes no HIP header: the device side is the template
// parameter Dev (the HIP one is in m4_serve.hip; a CPU test drives this same
// code with a mock device under a thread sanitizer).
//
// Dev provides:
//   void thread_init();                            first call of each core thread
//   struct Lane;                                   per-lane device state
//   static constexpr int kLanes;
//   double now_ms();
//   bool launch_done(Lane&);                       non-blocking
//   void launch(Lane&, std::vector<ServeReq*>&);   may throw; enqueues the fused launch
//   void collect(Lane&, std::vector<ServeReq*>&);  statuses and counts of a finished launch
//   uint64_t lane_bytes(const Lane&);              device bytes the lane holds
//   uint64_t lane_need(int64_t G, int64_t sum_n, int64_t sum_nnz);  bytes a launch needs
//   uint64_t lane_bytes_after(uint64_t held, uint64_t need);        lane size after it
//   void lane_release(Lane&);
//   uint64_t base_bytes();                         planning context
//   int run_big(ServeReq*, uint64_t reserve);      worker thread: one graph, status
//   uint64_t big_bytes();                          what the worker keeps between jobs
//   void big_release();
#pragma once
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/m4.h"

namespace m4 {

struct ServeReq {
  uint64_t id = 0, tag = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  uint64_t footprint = 0;  // device bytes admission reserves (big requests)
  bool big = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = M4_OK;
  uint64_t counts[6] = {0, 0, 0, 0, 0, 0};
};

constexpr int kMaxBatchGraphs = 4096;

template <class Dev>
class ServeCore {
 public:
  ServeCore(Dev& dev, uint64_t budget, int max_queue)
      : dev_(dev), budget_(budget), max_queue_(max_queue > 0 ? max_queue : 1 << 20) {}
  ~ServeCore() { stop(); }

  void start() {
    sched_ = std::thread([this] { scheduler(); });
    worker_ = std::thread([this] { big_worker(); });
  }

  // Joins the threads once every admitted launch has finished.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    cv_big_.notify_all();
    if (sched_.joinable()) sched_.join();
    cv_big_.notify_all();
    if (worker_.joinable()) worker_.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (ServeReq* r : queue_) delete r;
    for (ServeReq* r : results_) delete r;
    queue_.clear();
    results_.clear();
  }

  // Takes ownership of r (its id is set); M4_EBUSY when the queue is full.
  int submit(ServeReq* r, uint64_t* id) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if ((int64_t)queue_.size() >= max_queue_) return M4_EBUSY;
      r->id = next_id_++;
      r->t_submit = dev_.now_ms();
      queue_.push_back(r);
      submitted_++;
      if (id) *id = r->id;
    }
    cv_.notify_all();
    return M4_OK;
  }

  // Up to max finished requests, oldest completion first; the caller deletes them.
  int poll(std::vector<ServeReq*>& out, int max) {
    std::lock_guard<std::mutex> lk(mu_);
    int k = 0;
    while (k < max && !results_.empty()) {
      out.push_back(results_.front());
      results_.pop_front();
      k++;
    }
    return k;
  }

  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.notify_all();
    cv_done_.wait(lk, [&] { return completed_ == submitted_; });
  }

  void stats(uint64_t* max_device_bytes, uint64_t* launches, uint64_t* completed) {
    std::lock_guard<std::mutex> lk(mu_);
    if (max_device_bytes) *max_device_bytes = max_device_bytes_;
    if (launches) *launches = launches_;
    if (completed) *completed = completed_;
  }

  // f(lane) for every lane's device state (before start or after stop)
  template <class F>
  void for_each_lane(F&& f) {
    for (LaneSlot& L : lanes_) f(L.dl);
  }

  // Device memory held now (callers hold mu_): lane arenas (at least the
  // running launch's), the worker's workspaces (at least the running job's
  // reserve) and the planning context.
  uint64_t held_bytes_locked() const {
    uint64_t h = dev_.base_bytes();
    for (const LaneSlot& L : lanes_) h += std::max<uint64_t>(dev_.lane_bytes(L.dl), L.busy ? L.need : 0);
    h += big_busy_ ? std::max(big_retained_, big_job_->footprint) : big_retained_;
    return h;
  }

 private:
  struct LaneSlot {
    typename Dev::Lane dl;
    std::vector<ServeReq*> reqs;
    uint64_t need = 0;  // device bytes of the running launch
    bool busy = false;
  };

  void finish(ServeReq* r) {
    r->t_done = dev_.now_ms();
    results_.push_back(r);
    completed_++;
  }

  // Frees what idle lanes and an idle worker keep; true if anything was freed.
  bool release_idle() {
    bool freed = false;
    for (LaneSlot& L : lanes_)
      if (!L.busy && dev_.lane_bytes(L.dl) > 0) {
        dev_.lane_release(L.dl);
        freed = true;
      }
    if (!big_busy_ && big_retained_ > 0) {
      dev_.big_release();
      big_retained_ = dev_.big_bytes();
      freed = true;
    }
    return freed;
  }

  void scheduler() {
    dev_.thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      bool progress = false;
      // completions
      for (LaneSlot& L : lanes_) {
        if (L.busy && dev_.launch_done(L.dl)) {
          dev_.collect(L.dl, L.reqs);
          for (ServeReq* r : L.reqs) finish(r);
          L.reqs.clear();
          L.busy = false;
          progress = true;
        }
      }
      if (big_finished_) {
        big_finished_ = false;
        big_busy_ = false;
        finish(big_job_);
        big_job_ = nullptr;
        progress = true;
      }
      // admission, first come first served
      while (!queue_.empty()) {
        ServeReq* r = queue_.front();
        const uint64_t alone = r->big ? r->footprint : dev_.lane_need(1, r->n, r->nnz);
        if (alone + dev_.base_bytes() > budget_) {
          queue_.pop_front();
          r->status = M4_ENOMEM;
          r->t_admit = dev_.now_ms();
          finish(r);
          progress = true;
          continue;
        }
        if (r->big) {
          if (big_busy_) break;
          auto after = [&] {
            return held_bytes_locked() - big_retained_ + std::max(big_retained_, r->footprint);
          };
          if (after() > budget_ && !(release_idle() && after() <= budget_)) break;
          queue_.pop_front();
          r->t_admit = dev_.now_ms();
          big_job_ = r;
          big_busy_ = true;
          max_device_bytes_ = std::max(max_device_bytes_, held_bytes_locked());
          cv_big_.notify_one();
          progress = true;
          continue;
        }
        LaneSlot* free_lane = nullptr;
        for (LaneSlot& L : lanes_)
          if (!L.busy) {
            free_lane = &L;
            break;
          }
        if (!free_lane) break;
        // consecutive small requests that fit join this launch
        LaneSlot& L = *free_lane;
        L.reqs.clear();
        int64_t sn = 0, snnz = 0;
        bool retried = false;
        while (!queue_.empty() && (int)L.reqs.size() < kMaxBatchGraphs) {
          ServeReq* q = queue_.front();
          if (q->big) break;
          const uint64_t need = dev_.lane_need((int64_t)L.reqs.size() + 1, sn + q->n, snnz + q->nnz);
          const uint64_t held = dev_.lane_bytes(L.dl);
          const uint64_t after = held_bytes_locked() - held + dev_.lane_bytes_after(held, need);
          if (after > budget_) {
            // the first request of a launch may make room by freeing idle memory
            if (L.reqs.empty() && !retried) {
              retried = true;
              if (release_idle()) continue;
            }
            break;
          }
          queue_.pop_front();
          q->t_admit = dev_.now_ms();
          L.reqs.push_back(q);
          sn += q->n;
          snnz += q->nnz;
          L.need = need;
        }
        if (L.reqs.empty()) break;
        L.busy = true;
        launches_++;
        max_device_bytes_ = std::max(max_device_bytes_, held_bytes_locked());
        lk.unlock();
        bool ok = true;
        try {
          dev_.launch(L.dl, L.reqs);
        } catch (...) {
          ok = false;
        }
        lk.lock();
        if (!ok) {
          for (ServeReq* q : L.reqs) {
            q->status = M4_EDEVICE;
            finish(q);
          }
          L.reqs.clear();
          L.busy = false;
        }
        progress = true;
      }
      if (completed_ == submitted_) cv_done_.notify_all();
      bool any_busy = big_busy_;
      for (LaneSlot& L : lanes_) any_busy |= L.busy;
      if (stop_ && !any_busy && queue_.empty()) break;
      if (!progress) {
        // poll running launches every 50 us; sleep until woken when idle (the
        // deadline is on the system clock: a timed wait on it is the plain
        // pthread timed wait, which thread sanitizers model)
        const auto wait = any_busy ? std::chrono::microseconds(50) : std::chrono::microseconds(20000);
        cv_.wait_until(lk, std::chrono::system_clock::now() + wait);
      }
    }
  }

  void big_worker() {
    dev_.thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_big_.wait(lk, [&] { return stop_ || (big_job_ && !big_finished_ && big_busy_); });
      if (!big_job_ || big_finished_) {
        if (stop_) break;
        continue;
      }
      ServeReq* r = big_job_;
      lk.unlock();
      // the job runs within the reserve it was admitted with
      const int rc = dev_.run_big(r, r->footprint);
      const uint64_t kept = dev_.big_bytes();
      lk.lock();
      big_retained_ = kept;
      r->status = rc;
      big_finished_ = true;
      cv_.notify_all();
    }
  }

  Dev& dev_;
  const uint64_t budget_;
  const int64_t max_queue_;
  std::mutex mu_;
  std::condition_variable cv_;       // scheduler wake-up
  std::condition_variable cv_done_;  // drain
  std::condition_variable cv_big_;   // worker wake-up
  std::deque<ServeReq*> queue_;
  std::deque<ServeReq*> results_;
  uint64_t next_id_ = 1, submitted_ = 0, completed_ = 0, launches_ = 0;
  uint64_t big_retained_ = 0, max_device_bytes_ = 0;
  bool stop_ = false;
  LaneSlot lanes_[Dev::kLanes];
  ServeReq* big_job_ = nullptr;
  bool big_busy_ = false, big_finished_ = false;
  std::thread sched_, worker_;
};

}  // namespace m4
