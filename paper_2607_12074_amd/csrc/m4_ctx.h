// m4_ctx.h -- the context object behind the C ABI.
#pragma once
#include <string>

#include "m4_internal.h"

namespace m4 {

// A fixed region of device memory handed out front to back (the
// allocation-free entry point's workspaces).
struct ScratchPool {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

// Growable device buffer owned by a context.
// ensure() over-allocates by 1/8 (plus 1 MiB) so that slowly growing inputs
// do not reallocate every call; exact = true allocates exactly `bytes` and
// also shrinks a larger buffer (the budgeted path must not hold more).  With
// a pool, ensure() carves the bytes from it instead (a buffer can grow only
// while it is the pool's last carve) and fails with M4_ENOMEM when they do
// not fit; nothing is allocated or freed.
struct DevBuf {
  char* ptr = nullptr;
  size_t cap = 0;
  ScratchPool* pool = nullptr;
  void ensure(size_t bytes, hipStream_t s, bool exact = false);
  void release();
};

constexpr int kNumEvents = 8;

struct BatchState;
struct PartState;

size_t prep_bytes(int64_t n, int64_t nnz);
Prep carve_prep(char* base, int64_t n, int64_t nnz);
size_t stage_tmp_bytes(int64_t n, int64_t nnz, int64_t dmax, int num_cu);
// full_rows: the per-row records of resident runs (partitions store prefixes)
size_t c4_tmp_bytes(int64_t n, bool full_rows = true);
int set_error(m4_ctx* ctx, int code, const std::string& msg);
// status and message of the error bits a call left in Scal::err
int scal_error(m4_ctx* ctx, int err);
int check_csr_args(const m4_csr* g);
Tuning tuning_for(const m4_ctx* c, const m4_opts* o);
void run_resident(m4_ctx* c, const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz,
                  const m4_opts* o, hipStream_t s, Prep& P, bool want_timing);
// m4_noalloc.hip: the fixed scratch of the allocation-free entry point;
// noalloc_setup() looks up its address on the current device (once per
// device, from m4_ctx_create; a failed lookup leaves that entry point
// reporting M4_EDEVICE on the device)
void noalloc_setup(int device);

// m4_part.hip
bool needs_partition(m4_ctx* c, const m4_csr* g, const m4_opts* o);
int count_partitioned(m4_ctx* c, const m4_csr* g, const m4_opts* o, uint64_t out[6],
                      m4_stats* st);
void destroy_ctx_extras(m4_ctx* c);
// m4_batch.hip -- one persistent fused launch over a packed arena
struct BatchArgs;
struct BatchBuffers {
  DevBuf dev;
  unsigned long long* h_out = nullptr;  // pinned [G][6]
  int* h_status = nullptr;              // pinned [G]
  char* h_stage = nullptr;              // pinned copy of a host arena
  size_t h_out_cap = 0, h_stage_cap = 0;
  void release();
};
struct BatchPlan;
void destroy_batch_state(m4_ctx* c);

}  // namespace m4

struct m4_ctx {
  int device = 0;
  int num_cu = 256;
  std::string arch;
  hipStream_t stream = nullptr;
  m4::Scal* scal = nullptr;       // device
  m4::Scal* scal_host = nullptr;  // pinned
  hipStream_t stream2 = nullptr;  // the 4-cycle stage, overlapped with the triangle stage
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  m4::DevBuf prep, tmp, big, big2, input, tout, extra;
  hipEvent_t ev[m4::kNumEvents] = {};
  m4::KTimer ktimer;
  m4::Tuning tune;
  std::string last_error;
  m4::BatchState* batch = nullptr;
  m4::PartState* part = nullptr;
  m4::BasisChoice basis;                  // cycle/path basis of the last resident count
  unsigned long long cost_pair[2] = {0, 0};  // its objective's inputs, read back
  bool no_alloc = false;  // inside the allocation-free entry point
  // device bytes the context holds now (workspaces, batch buffers, Scal)
  size_t held_bytes() const;
  // frees every workspace except the budgeted path's (c->extra)
  void release_resident();
};
