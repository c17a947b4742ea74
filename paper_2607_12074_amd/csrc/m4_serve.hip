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
// arenas and an idle worker's workspaces are freed first.  Admission is
// strictly first-come first-served (no request overtakes an earlier one that
// does not fit yet), which rules out starvation.  The queue, admission and
// threads are the device-independent core in m4_serve_core.h; this file is
// its device side.
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
#include "m4_serve_core.h"

namespace m4 {

namespace {

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

// The device side of the serving core: three lanes, each with its own
// stream, arena and pinned buffers running one persistent fused launch over
// the requests packed into it, and a worker context that runs the
// single-graph path.
struct HipServeDev {
  static constexpr int kLanes = 3;
  struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    BatchBuffers buf;
    BatchPlan plan;
    std::vector<int64_t> voff, eoff, rowp;
    std::vector<int32_t> col;
  };
  m4_ctx* ctx = nullptr;      // lanes (fused kernel planning)
  m4_ctx* big_ctx = nullptr;  // single-graph path of the worker thread
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  void thread_init() { (void)hipSetDevice(ctx->device); }
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
  bool launch_done(Lane& L) { return hipEventQuery(L.done) == hipSuccess; }
  // packs the requests into the lane arena and enqueues the fused launch
  void launch(Lane& L, std::vector<ServeReq*>& reqs) {
    const int64_t G = (int64_t)reqs.size();
    L.voff.assign(G + 1, 0);
    L.eoff.assign(G + 1, 0);
    for (int64_t g = 0; g < G; g++) {
      L.voff[g + 1] = L.voff[g] + reqs[g]->n;
      L.eoff[g + 1] = L.eoff[g] + reqs[g]->nnz;
    }
    L.rowp.resize(L.voff[G] + G);
    L.col.resize(L.eoff[G] > 0 ? L.eoff[G] : 1);
    for (int64_t g = 0; g < G; g++) {
      const ServeReq* r = reqs[g];
      memcpy(L.rowp.data() + L.voff[g] + g, r->rp.data(), (r->n + 1) * 8);
      if (r->nnz) memcpy(L.col.data() + L.eoff[g], r->col.data(), r->nnz * 4);
    }
    batch_prepare(ctx, L.buf, L.plan, G, L.voff.data(), L.eoff.data(), nullptr,
                  ctx->tune.batch_variant, ctx->tune.batch_light, 0, 0, L.stream);
    batch_stage(L.buf, L.plan, L.voff.data(), L.eoff.data(), L.rowp.data(), L.col.data());
    batch_enqueue(L.buf, L.plan, L.stream);
    M4_HIP(hipEventRecord(L.done, L.stream));
  }
  void collect(Lane& L, std::vector<ServeReq*>& reqs) {
    for (size_t g = 0; g < reqs.size(); g++) {
      ServeReq* r = reqs[g];
      const int st = L.buf.h_status[g];
      r->status = st == 0 ? M4_OK : (st == 3 ? M4_EOVERFLOW : M4_EINTERNAL);
      memcpy(r->counts, L.buf.h_out + 6 * g, 48);
    }
  }
  uint64_t lane_bytes(const Lane& L) const { return L.buf.dev.cap; }
  uint64_t lane_need(int64_t G, int64_t sum_n, int64_t sum_nnz) const {
    return batch_layout(G, sum_n, sum_nnz, true).need;
  }
  // DevBuf::ensure grows by an eighth plus 1 MiB, so that slowly growing
  // batches do not reallocate every launch
  uint64_t lane_bytes_after(uint64_t held, uint64_t need) const {
    return need <= held ? held : need + need / 8 + (1u << 20);
  }
  void lane_release(Lane& L) {
    (void)hipStreamSynchronize(L.stream);
    L.buf.dev.release();
  }
  uint64_t base_bytes() const { return ctx->held_bytes(); }
  int run_big(ServeReq* r, uint64_t reserve) {
    m4_csr g;
    g.n = r->n;
    g.nnz = r->nnz;
    g.row_ptr = r->rp.data();
    g.col = r->col.data();
    g.on_device = 0;
    // within the reserve it was admitted with (the resident path when that
    // holds it, else halo partitions)
    m4_opts o{};
    o.device_budget_bytes = reserve;
    return m4_count_motifs4_ex(big_ctx, &g, &o, r->counts, nullptr);
  }
  uint64_t big_bytes() const { return big_ctx->held_bytes(); }
  void big_release() { big_ctx->release_resident(); }
};

}  // namespace

}  // namespace m4

struct m4_server {
  m4::HipServeDev dev;
  m4::ServeCore<m4::HipServeDev>* core = nullptr;
  int batch_variant = 0;
};

extern "C" int m4_server_create(m4_ctx* ctx, uint64_t budget, int max_queue, m4_server** out) {
  if (!ctx || !out || budget == 0) return M4_EINVAL;
  *out = nullptr;
  m4_server* s = new (std::nothrow) m4_server();
  if (!s) return M4_ENOMEM;
  int rc = m4_ctx_create(ctx->device, &s->dev.ctx);
  if (rc == M4_OK) rc = m4_ctx_create(ctx->device, &s->dev.big_ctx);
  if (rc != M4_OK) {
    m4_ctx_destroy(s->dev.ctx);
    delete s;
    return rc;
  }
  s->dev.ctx->tune = ctx->tune;
  s->dev.big_ctx->tune = ctx->tune;
  s->batch_variant = ctx->tune.batch_variant;
  s->core = new (std::nothrow) m4::ServeCore<m4::HipServeDev>(s->dev, budget, max_queue);
  if (!s->core) {
    m4_server_destroy(s);
    return M4_ENOMEM;
  }
  try {
    s->core->for_each_lane([&](m4::HipServeDev::Lane& L) {
      M4_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
      M4_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    });
  } catch (const m4::HipFail&) {
    m4_server_destroy(s);
    return M4_EDEVICE;
  }
  s->core->start();
  *out = s;
  return M4_OK;
}

extern "C" int m4_server_submit(m4_server* s, const m4_csr* g, uint64_t tag, uint64_t* id) {
  if (!s || !g) return M4_EINVAL;
  int rc = m4::check_csr_args(g);
  if (rc) return rc;
  if (g->on_device) return M4_EINVAL;  // requests arrive from the host
  if (g->row_ptr[g->n] != g->nnz) return M4_ERANGE;
  m4::ServeReq* r = new (std::nothrow) m4::ServeReq();
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
  r->big = !m4::batch_graph_fits(g->n, g->row_ptr, s->batch_variant);
  r->footprint = r->big ? m4::big_footprint(g->n, g->nnz) : m4::small_footprint(g->n, g->nnz);
  rc = s->core->submit(r, id);
  if (rc != M4_OK) delete r;
  return rc;
}

extern "C" int m4_server_poll(m4_server* s, m4_result* res, int max_results, int* got) {
  if (!s || !got || (max_results > 0 && !res)) return M4_EINVAL;
  std::vector<m4::ServeReq*> done;
  const int k = s->core->poll(done, max_results);
  for (int i = 0; i < k; i++) {
    m4::ServeReq* r = done[i];
    m4_result& o = res[i];
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
  s->core->drain();
  return M4_OK;
}

extern "C" int m4_server_stats(const m4_server* s, uint64_t* max_inflight_bytes,
                               uint64_t* launches, uint64_t* completed) {
  if (!s) return M4_EINVAL;
  s->core->stats(max_inflight_bytes, launches, completed);
  return M4_OK;
}

extern "C" void m4_server_destroy(m4_server* s) {
  if (!s) return;
  if (s->core) {
    s->core->stop();
    s->core->for_each_lane([&](m4::HipServeDev::Lane& L) {
      if (L.stream) (void)hipStreamSynchronize(L.stream);
      L.buf.release();
      if (L.done) (void)hipEventDestroy(L.done);
      if (L.stream) (void)hipStreamDestroy(L.stream);
    });
    delete s->core;
  }
  m4_ctx_destroy(s->dev.ctx);
  m4_ctx_destroy(s->dev.big_ctx);
  delete s;
}

extern "C" double m4_server_now_ms(const m4_server* s) { return s ? s->dev.now_ms() : 0.0; }
