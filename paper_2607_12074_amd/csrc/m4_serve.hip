// m4_serve.hip -- request loop with continuous batching.
//
// Submitted graphs are copied into library-owned memory and queued in
// arrival order.  A scheduler thread admits them while their device
// footprint fits the HBM budget: consecutive small graphs are packed into one
// arena and counted by one persistent fused launch on a free lane (each lane
// has its own stream, arena and pinned buffers, so launches of different
// lanes overlap on the device); a graph larger than one workgroup's share
// goes to a worker thread that runs the multi-kernel single-graph path on its
// own context and stream.  Whenever a lane's launch completes its results are
// published and the next requests are admitted, so requests arriving while
// others run join as soon as a lane and memory free up.  Admission counts
// the device memory the server holds: every lane's arena (kept for the next
// launches, and counted at the size the next launch grows it to), the
// worker context's workspaces as its last job left them (at least the
// running job's reserve); when the next request does not fit, idle lanes'
// arenas and an idle worker's workspaces are freed first.  Admission is strictly first-come first-served (no request
// overtakes an earlier one that does not fit yet), which rules out
// starvation.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "m4_batch.h"

namespace m4 {

namespace {

constexpr int kLanes = 3;
constexpr int kMaxBatchGraphs = 4096;

struct Req {
  uint64_t id = 0, tag = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  uint64_t footprint = 0;
  bool big = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = M4_OK;
  uint64_t counts[6] = {0, 0, 0, 0, 0, 0};
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  BatchBuffers buf;
  BatchPlan plan;
  std::vector<Req*> reqs;
  std::vector<int64_t> voff, eoff, rowp;
  std::vector<int32_t> col;
  uint64_t need = 0;  // device bytes of the running launch
  bool busy = false;
};

// device bytes a small request occupies inside a lane arena (CSR copy plus
// the per-graph work arrays of the fused kernel)
uint64_t small_footprint(int64_t n, int64_t nnz) {
  return (uint64_t)(8 * (n + 1) + 4 * nnz) + (uint64_t)(16 * n + 16 * (n + 1) + 4 * nnz + 2 * nnz) +
         64;
}
// device bytes of the single-graph path (workspace of the resident pipeline)
uint64_t big_footprint(int64_t n, int64_t nnz) {
  return prep_bytes(n, nnz) + stage_tmp_bytes(n, nnz, 1, 256) + (uint64_t)(8 * (n + 1) + 4 * nnz) +
         (uint64_t)nnz * 8 + (64ull << 20);
}

}  // namespace

}  // namespace m4

struct m4_server {
  m4_ctx* ctx = nullptr;      // lanes (fused kernel planning)
  m4_ctx* big_ctx = nullptr;  // single-graph path of the worker thread
  uint64_t budget = 0;
  int max_queue = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;       // scheduler wake-up
  std::condition_variable cv_done;  // drain
  std::deque<m4::Req*> queue;
  std::deque<m4::Req*> results;
  uint64_t next_id = 1, submitted = 0, completed = 0;
  uint64_t inflight_bytes = 0, launches = 0;
  uint64_t big_retained = 0;     // workspaces the worker context keeps between jobs
  uint64_t max_device_bytes = 0;  // largest device memory held at once
  bool stop = false;
  m4::Lane lanes[m4::kLanes];
  std::thread sched, worker;
  // big-request worker
  m4::Req* big_job = nullptr;
  bool big_busy = false, big_finished = false;
  std::condition_variable cv_big;

  double now() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace m4 {

namespace {

void finish(m4_server* s, Req* r) {
  r->t_done = s->now();
  s->inflight_bytes -= r->footprint;
  s->results.push_back(r);
  s->completed++;
}

// Packs lane.reqs into the lane arena and enqueues the fused launch.
void launch_lane(m4_server* s, Lane& L) {
  const int64_t G = (int64_t)L.reqs.size();
  L.voff.assign(G + 1, 0);
  L.eoff.assign(G + 1, 0);
  for (int64_t g = 0; g < G; g++) {
    L.voff[g + 1] = L.voff[g] + L.reqs[g]->n;
    L.eoff[g + 1] = L.eoff[g] + L.reqs[g]->nnz;
  }
  L.rowp.resize(L.voff[G] + G);
  L.col.resize(L.eoff[G] > 0 ? L.eoff[G] : 1);
  for (int64_t g = 0; g < G; g++) {
    const Req* r = L.reqs[g];
    memcpy(L.rowp.data() + L.voff[g] + g, r->rp.data(), (r->n + 1) * 8);
    if (r->nnz) memcpy(L.col.data() + L.eoff[g], r->col.data(), r->nnz * 4);
  }
  batch_prepare(s->ctx, L.buf, L.plan, G, L.voff.data(), L.eoff.data(), nullptr,
                s->ctx->tune.batch_variant, s->ctx->tune.batch_light, 0, 0, L.stream);
  batch_stage(L.buf, L.plan, L.voff.data(), L.eoff.data(), L.rowp.data(), L.col.data());
  batch_enqueue(L.buf, L.plan, L.stream);
  M4_HIP(hipEventRecord(L.done, L.stream));
  L.busy = true;
  s->launches++;
}

void collect_lane(m4_server* s, Lane& L) {
  for (size_t g = 0; g < L.reqs.size(); g++) {
    Req* r = L.reqs[g];
    const int st = L.buf.h_status[g];
    r->status = st == 0 ? M4_OK : (st == 3 ? M4_EOVERFLOW : M4_EINTERNAL);
    memcpy(r->counts, L.buf.h_out + 6 * g, 48);
    finish(s, r);
  }
  L.reqs.clear();
  L.busy = false;
}

// Device memory the server holds now: lane arenas (at least the running
// launch's), the worker's workspaces (at least the running job's reserve)
// and the lanes' planning context.
uint64_t held_bytes(const m4_server* s) {
  uint64_t h = s->ctx->held_bytes();
  for (const Lane& L : s->lanes) h += std::max<uint64_t>(L.buf.dev.cap, L.busy ? L.need : 0);
  h += s->big_busy ? std::max(s->big_retained, s->big_job->footprint) : s->big_retained;
  return h;
}

// Frees what idle lanes and an idle worker keep; true if anything was freed.
bool release_idle(m4_server* s) {
  bool freed = false;
  for (Lane& L : s->lanes)
    if (!L.busy && L.buf.dev.cap > 0) {
      (void)hipStreamSynchronize(L.stream);
      L.buf.dev.release();
      freed = true;
    }
  if (!s->big_busy && s->big_retained > 0) {
    s->big_ctx->release_resident();
    s->big_retained = s->big_ctx->held_bytes();
    freed = true;
  }
  return freed;
}

uint64_t lane_need(int64_t G, int64_t sum_n, int64_t sum_nnz) {
  return batch_layout(G, sum_n, sum_nnz, true).need;
}

// a lane arena's size after a launch that needs `need` bytes (DevBuf::ensure
// grows by an eighth plus 1 MiB, so that slowly growing batches do not
// reallocate every launch)
uint64_t lane_cap_after(uint64_t cap, uint64_t need) {
  return need <= cap ? cap : need + need / 8 + (1u << 20);
}

void scheduler(m4_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    bool progress = false;
    // completions
    for (Lane& L : s->lanes) {
      if (L.busy && hipEventQuery(L.done) == hipSuccess) {
        collect_lane(s, L);
        progress = true;
      }
    }
    if (s->big_finished) {
      s->big_finished = false;
      s->big_busy = false;
      finish(s, s->big_job);
      s->big_job = nullptr;
      progress = true;
    }
    // admission, first come first served
    while (!s->queue.empty()) {
      Req* r = s->queue.front();
      const uint64_t alone = r->big ? r->footprint : lane_need(1, r->n, r->nnz);
      if (alone + s->ctx->held_bytes() > s->budget) {
        s->queue.pop_front();
        r->status = M4_ENOMEM;
        r->t_admit = s->now();
        s->inflight_bytes += r->footprint;
        finish(s, r);
        progress = true;
        continue;
      }
      if (r->big) {
        if (s->big_busy) break;
        auto after = [&] {
          return held_bytes(s) - s->big_retained + std::max(s->big_retained, r->footprint);
        };
        if (after() > s->budget && !(release_idle(s) && after() <= s->budget)) break;
        s->queue.pop_front();
        r->t_admit = s->now();
        s->inflight_bytes += r->footprint;
        s->big_job = r;
        s->big_busy = true;
        s->max_device_bytes = std::max(s->max_device_bytes, held_bytes(s));
        s->cv_big.notify_one();
        progress = true;
        continue;
      }
      Lane* free_lane = nullptr;
      for (Lane& L : s->lanes)
        if (!L.busy) {
          free_lane = &L;
          break;
        }
      if (!free_lane) break;
      // consecutive small requests that fit join this launch
      Lane& L = *free_lane;
      L.reqs.clear();
      int64_t sn = 0, snnz = 0;
      bool retried = false;
      while (!s->queue.empty() && (int)L.reqs.size() < kMaxBatchGraphs) {
        Req* q = s->queue.front();
        if (q->big) break;
        const uint64_t need = lane_need((int64_t)L.reqs.size() + 1, sn + q->n, snnz + q->nnz);
        const uint64_t after = held_bytes(s) - L.buf.dev.cap + lane_cap_after(L.buf.dev.cap, need);
        if (after > s->budget) {
          // the first request of a launch may make room by freeing idle memory
          if (L.reqs.empty() && !retried) {
            retried = true;
            if (release_idle(s)) continue;
          }
          break;
        }
        s->queue.pop_front();
        q->t_admit = s->now();
        s->inflight_bytes += q->footprint;
        L.reqs.push_back(q);
        sn += q->n;
        snnz += q->nnz;
        L.need = need;
      }
      if (L.reqs.empty()) break;
      L.busy = true;
      s->max_device_bytes = std::max(s->max_device_bytes, held_bytes(s));
      lk.unlock();
      bool ok = true;
      try {
        launch_lane(s, L);
      } catch (...) {
        ok = false;
      }
      lk.lock();
      if (!ok) {
        for (Req* q : L.reqs) {
          q->status = M4_EDEVICE;
          finish(s, q);
        }
        L.reqs.clear();
        L.busy = false;
      }
      progress = true;
    }
    if (s->completed == s->submitted) s->cv_done.notify_all();
    bool any_busy = s->big_busy;
    for (Lane& L : s->lanes) any_busy |= L.busy;
    if (s->stop && !any_busy && s->queue.empty()) break;
    if (!progress) {
      // poll running launches every 50 us; sleep until woken when idle
      if (any_busy) s->cv.wait_for(lk, std::chrono::microseconds(50));
      else s->cv.wait_for(lk, std::chrono::milliseconds(20));
    }
  }
}

void big_worker(m4_server* s) {
  (void)hipSetDevice(s->big_ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_big.wait(lk, [&] { return s->stop || (s->big_job && !s->big_finished && s->big_busy); });
    if (!s->big_job || s->big_finished) {
      if (s->stop) break;
      continue;
    }
    Req* r = s->big_job;
    lk.unlock();
    m4_csr g;
    g.n = r->n;
    g.nnz = r->nnz;
    g.row_ptr = r->rp.data();
    g.col = r->col.data();
    g.on_device = 0;
    // the job runs within the reserve it was admitted with (the resident
    // path when that holds it, else halo partitions)
    m4_opts o{};
    o.device_budget_bytes = r->footprint;
    const int rc = m4_count_motifs4_ex(s->big_ctx, &g, &o, r->counts, nullptr);
    const uint64_t kept = s->big_ctx->held_bytes();
    lk.lock();
    s->big_retained = kept;
    r->status = rc;
    s->big_finished = true;
    s->cv.notify_all();
  }
}

}  // namespace

}  // namespace m4

extern "C" int m4_server_create(m4_ctx* ctx, uint64_t budget, int max_queue, m4_server** out) {
  if (!ctx || !out || budget == 0) return M4_EINVAL;
  *out = nullptr;
  m4_server* s = new (std::nothrow) m4_server();
  if (!s) return M4_ENOMEM;
  int rc = m4_ctx_create(ctx->device, &s->ctx);
  if (rc == M4_OK) rc = m4_ctx_create(ctx->device, &s->big_ctx);
  if (rc != M4_OK) {
    m4_ctx_destroy(s->ctx);
    delete s;
    return rc;
  }
  s->ctx->tune = ctx->tune;
  s->big_ctx->tune = ctx->tune;
  s->budget = budget;
  s->max_queue = max_queue > 0 ? max_queue : 1 << 20;
  s->t0 = std::chrono::steady_clock::now();
  try {
    for (m4::Lane& L : s->lanes) {
      M4_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
      M4_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    }
  } catch (const m4::HipFail&) {
    m4_server_destroy(s);
    return M4_EDEVICE;
  }
  s->sched = std::thread(m4::scheduler, s);
  s->worker = std::thread(m4::big_worker, s);
  *out = s;
  return M4_OK;
}

extern "C" int m4_server_submit(m4_server* s, const m4_csr* g, uint64_t tag, uint64_t* id) {
  if (!s || !g) return M4_EINVAL;
  int rc = m4::check_csr_args(g);
  if (rc) return rc;
  if (g->on_device) return M4_EINVAL;  // requests arrive from the host
  if (g->row_ptr[g->n] != g->nnz) return M4_ERANGE;
  m4::Req* r = new (std::nothrow) m4::Req();
  if (!r) return M4_ENOMEM;
  try {
    r->rp.assign(g->row_ptr, g->row_ptr + g->n + 1);
    r->col.assign(g->col, g->col + g->nnz);
  } catch (...) {
    delete r;
    return M4_ENOMEM;
  }
  r->n = g->n;
  r->nnz = g->nnz;
  r->tag = tag;
  r->big = !m4::batch_graph_fits(g->n, g->row_ptr, s->ctx->tune.batch_variant);
  r->footprint = r->big ? m4::big_footprint(g->n, g->nnz) : m4::small_footprint(g->n, g->nnz);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)s->queue.size() >= s->max_queue) {
      delete r;
      return M4_EBUSY;
    }
    r->id = s->next_id++;
    r->t_submit = s->now();
    s->queue.push_back(r);
    s->submitted++;
  }
  s->cv.notify_all();
  if (id) *id = r->id;
  return M4_OK;
}

extern "C" int m4_server_poll(m4_server* s, m4_result* res, int max_results, int* got) {
  if (!s || !got || (max_results > 0 && !res)) return M4_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int k = 0;
  while (k < max_results && !s->results.empty()) {
    m4::Req* r = s->results.front();
    s->results.pop_front();
    m4_result& o = res[k++];
    o.id = r->id;
    o.tag = r->tag;
    o.status = r->status;
    memcpy(o.counts, r->counts, 48);
    o.t_submit_ms = r->t_submit;
    o.t_admit_ms = r->t_admit;
    o.t_done_ms = r->t_done;
    delete r;
  }
  *got = k;
  return M4_OK;
}

extern "C" int m4_server_drain(m4_server* s) {
  if (!s) return M4_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_all();
  s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
  return M4_OK;
}

extern "C" int m4_server_stats(const m4_server* s, uint64_t* max_inflight_bytes,
                               uint64_t* launches, uint64_t* completed) {
  if (!s) return M4_EINVAL;
  m4_server* m = const_cast<m4_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  if (max_inflight_bytes) *max_inflight_bytes = m->max_device_bytes;
  if (launches) *launches = m->launches;
  if (completed) *completed = m->completed;
  return M4_OK;
}

extern "C" void m4_server_destroy(m4_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->cv_big.notify_all();
  if (s->sched.joinable()) s->sched.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_big.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (m4::Lane& L : s->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    L.buf.release();
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  for (m4::Req* r : s->queue) delete r;
  for (m4::Req* r : s->results) delete r;
  m4_ctx_destroy(s->ctx);
  m4_ctx_destroy(s->big_ctx);
  delete s;
}

extern "C" double m4_server_now_ms(const m4_server* s) { return s ? s->now() : 0.0; }
