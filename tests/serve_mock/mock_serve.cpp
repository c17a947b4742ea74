// Drives the serving core (m4_serve_core.h) with a mock device from many
// threads: submitters, pollers, the core's scheduler and worker.  Built with a
// thread sanitizer by tests/test_serve_admission.py.  Checks that every
// request comes back exactly once with its own result, that requests beyond
// the budget are refused, that admission is first come first served, and
// that the device memory the mock holds never exceeds the budget.
#include <stdio.h>

#include <atomic>
#include <map>
#include <random>

#include "../../paper_2607_12074_amd/csrc/m4_serve_core.h"

using m4::ServeReq;

namespace {

constexpr uint64_t kBudget = 8u << 20;
constexpr uint64_t kBase = 1u << 16;

double clock_ms() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct MockDev {
  static constexpr int kLanes = 3;
  struct Lane {
    uint64_t cap = 0;
    std::chrono::steady_clock::time_point ready;
    unsigned seed = 1;
  };
  // device bytes the mock holds: lane arenas and the worker's workspaces
  std::atomic<int64_t> held{0}, peak{0};
  std::atomic<int> over{0};
  uint64_t big_kept = 0;  // worker thread, or the scheduler while the worker is idle

  void grow(int64_t bytes) {
    const int64_t h = held.fetch_add(bytes) + bytes;
    int64_t p = peak.load();
    while (h > p && !peak.compare_exchange_weak(p, h)) {
    }
    if ((uint64_t)h + kBase > kBudget) over++;
  }
  void thread_init() {}
  double now_ms() const { return clock_ms(); }
  bool launch_done(Lane& L) { return std::chrono::steady_clock::now() >= L.ready; }
  void launch(Lane& L, std::vector<ServeReq*>& reqs) {
    int64_t sn = 0, snnz = 0;
    for (ServeReq* r : reqs) {
      if (r->big) over++;  // a lane only takes small requests
      sn += r->n;
      snnz += r->nnz;
    }
    const uint64_t need = lane_need((int64_t)reqs.size(), sn, snnz);
    const uint64_t after = lane_bytes_after(L.cap, need);
    if (after > L.cap) {
      grow((int64_t)(after - L.cap));
      L.cap = after;
    }
    L.seed = L.seed * 1103515245u + 12345u;
    L.ready = std::chrono::steady_clock::now() + std::chrono::microseconds(20 + L.seed % 400);
  }
  void collect(Lane&, std::vector<ServeReq*>& reqs) {
    for (ServeReq* r : reqs) {
      r->status = M4_OK;
      r->counts[0] = (uint64_t)r->n;
      r->counts[1] = (uint64_t)r->nnz;
      r->counts[5] = r->tag;
    }
  }
  uint64_t lane_bytes(const Lane& L) const { return L.cap; }
  uint64_t lane_need(int64_t G, int64_t sn, int64_t snnz) const {
    return 4096 + 64 * (uint64_t)G + 40 * (uint64_t)sn + 10 * (uint64_t)snnz;
  }
  uint64_t lane_bytes_after(uint64_t held_now, uint64_t need) const {
    return need <= held_now ? held_now : need + need / 8 + 65536;
  }
  void lane_release(Lane& L) {
    grow(-(int64_t)L.cap);
    L.cap = 0;
  }
  uint64_t base_bytes() const { return kBase; }
  int run_big(ServeReq* r, uint64_t reserve) {
    // the job's workspaces stay within its reserve
    const uint64_t want = reserve - reserve / 8;
    if (want > big_kept) {
      grow((int64_t)(want - big_kept));
      big_kept = want;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100 + r->n % 900));
    r->counts[0] = (uint64_t)r->n;
    r->counts[1] = (uint64_t)r->nnz;
    r->counts[5] = r->tag;
    return M4_OK;
  }
  uint64_t big_bytes() const { return big_kept; }
  void big_release() {
    grow(-(int64_t)big_kept);
    big_kept = 0;
  }
};

struct Sent {
  int64_t n, nnz;
  bool big, oversize;
};

}  // namespace

int main() {
  MockDev dev;
  m4::ServeCore<MockDev> core(dev, kBudget, 64);
  core.start();
  constexpr int kSubmitters = 6, kPerSubmitter = 300, kPollers = 2;
  std::mutex mu;
  std::map<uint64_t, Sent> sent;
  std::map<uint64_t, ServeReq> got;
  std::atomic<int> dup{0}, wrong{0}, submitters_left{kSubmitters};
  std::vector<std::thread> th;
  for (int t = 0; t < kSubmitters; t++)
    th.emplace_back([&, t] {
      std::mt19937_64 rng(1000 + t);
      for (int i = 0; i < kPerSubmitter; i++) {
        ServeReq* r = new ServeReq();
        r->n = 10 + (int64_t)(rng() % 5000);
        r->nnz = 8 * r->n;
        r->tag = (uint64_t)t * 100000 + i;
        const unsigned kind = rng() % 100;
        r->big = kind < 6;
        r->footprint = r->big ? (1u << 20) * (1 + rng() % 6) : 0;
        bool oversize = false;
        if (kind == 99) {  // beyond the budget
          r->big = true;
          r->footprint = kBudget * 2;
          oversize = true;
        }
        const Sent s{r->n, r->nnz, r->big, oversize};
        uint64_t id = 0;
        int rc;
        {
          // hold the map lock across the submit so the record exists before
          // a poller can see the result
          std::lock_guard<std::mutex> lk(mu);
          rc = core.submit(r, &id);
          if (rc == M4_OK) sent[id] = s;
        }
        while (rc == M4_EBUSY) {
          std::this_thread::sleep_for(std::chrono::microseconds(50));
          std::lock_guard<std::mutex> lk(mu);
          rc = core.submit(r, &id);
          if (rc == M4_OK) sent[id] = s;
        }
        if (rc != M4_OK) wrong++;
      }
      submitters_left--;
    });
  const int total = kSubmitters * kPerSubmitter;
  for (int p = 0; p < kPollers; p++)
    th.emplace_back([&] {
      while (true) {
        std::vector<ServeReq*> out;
        core.poll(out, 32);
        {
          std::lock_guard<std::mutex> lk(mu);
          for (ServeReq* r : out) {
            if (got.count(r->id)) dup++;
            got[r->id] = *r;
            delete r;
          }
          if ((int)got.size() == total) break;
        }
        if (out.empty()) std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    });
  for (auto& x : th) x.join();
  core.drain();
  uint64_t max_dev = 0, launches = 0, completed = 0;
  core.stats(&max_dev, &launches, &completed);
  core.stop();

  int bad = 0;
  double last_admit = -1;
  for (auto& kv : got) {  // ascending ids
    const Sent& s = sent.at(kv.first);
    const ServeReq& r = kv.second;
    if (s.oversize) {
      if (r.status != M4_ENOMEM) bad++;
      continue;
    }
    if (r.status != M4_OK || r.counts[0] != (uint64_t)s.n || r.counts[1] != (uint64_t)s.nnz ||
        r.counts[5] != r.tag)
      bad++;
    // first come first served: admission times follow submission order
    if (r.t_admit < last_admit) bad++;
    last_admit = r.t_admit;
    if (!(r.t_submit <= r.t_admit && r.t_admit <= r.t_done)) bad++;
  }
  printf("results %zu of %d, duplicates %d, wrong %d, bad %d, over-budget %d, "
         "peak %lld + %llu of %llu bytes, max reported %llu, launches %llu, completed %llu\n",
         got.size(), total, dup.load(), wrong.load(), bad, dev.over.load(),
         (long long)dev.peak.load(), (unsigned long long)kBase, (unsigned long long)kBudget,
         (unsigned long long)max_dev, (unsigned long long)launches,
         (unsigned long long)completed);
  const bool ok = (int)got.size() == total && dup == 0 && wrong == 0 && bad == 0 &&
                  dev.over == 0 && max_dev <= kBudget && completed == (uint64_t)total &&
                  launches > 0;
  printf(ok ? "OK\n" : "FAILED\n");
  return ok ? 0 : 1;
}
