// m4_api.hip -- C ABI of the motif-count library: contexts, workspace and the
// single-graph pipeline (CSR builder -> triangle/4-clique anchors -> 4-cycle
// anchor -> closure -> exact inverse).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "m4_device.h"
#include "m4_ctx.h"

using namespace m4;

// ----------------------------------------------------------------- context

namespace m4 {

void DevBuf::ensure(size_t bytes, hipStream_t s, bool exact) {
  if (pool) {
    if (bytes <= cap) return;
    const size_t off = ptr ? (size_t)(ptr - pool->base) : ((pool->used + 255) & ~size_t(255));
    if ((ptr && off + cap != pool->used) || off + bytes > pool->cap)
      throw Fail(M4_ENOMEM, "workspace of " + std::to_string(bytes) +
                                " bytes does not fit in the fixed scratch of " +
                                std::to_string(pool->cap) + " bytes");
    ptr = pool->base + off;
    cap = bytes;
    pool->used = off + bytes;
    return;
  }
  if (exact ? bytes == cap : bytes <= cap) return;
  if (ptr) {
    M4_HIP(hipStreamSynchronize(s));
    M4_HIP(hipFree(ptr));
    ptr = nullptr;
    cap = 0;
  }
  size_t want = exact ? bytes : bytes + bytes / 8 + (1 << 20);
  hipError_t e = hipMalloc((void**)&ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc((void**)&ptr, bytes);
    want = bytes;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    throw Fail(M4_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  cap = want;
}

void DevBuf::release() {
  if (ptr && !pool) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t batch_held_bytes(const m4_ctx* c);
void batch_release(m4_ctx* c);

}  // namespace m4

size_t m4_ctx::held_bytes() const {
  return prep.cap + tmp.cap + big.cap + big2.cap + input.cap + tout.cap + extra.cap +
         m4::batch_held_bytes(this) + sizeof(m4::Scal);
}

void m4_ctx::release_resident() {
  (void)hipStreamSynchronize(stream);
  (void)hipStreamSynchronize(stream2);
  prep.release();
  tmp.release();
  big.release();
  big2.release();
  input.release();
  tout.release();
  m4::batch_release(this);
}

namespace m4 {

size_t prep_bytes(int64_t n, int64_t nnz) {
  size_t b = 0;
  b += 5 * align256((size_t)n * 4 + 4);
  b += 2 * align256((size_t)(n + 1) * 8);
  b += align256((size_t)(nnz + NCOL_PAD) * 4);
  b += align256((size_t)(nnz / 2) * 4 + 4);
  return b + 4096;
}

Prep carve_prep(char* base, int64_t n, int64_t nnz) {
  Arena a;
  a.base = base;
  a.cap = prep_bytes(n, nnz);
  Prep P;
  P.perm = a.take<int32_t>(n + 1);
  P.rank = a.take<int32_t>(n + 1);
  P.dr = a.take<int32_t>(n + 1);
  P.dlo = a.take<int32_t>(n + 1);
  P.dplus = a.take<int32_t>(n + 1);
  P.nptr = a.take<int64_t>(n + 1);
  P.optr = a.take<int64_t>(n + 1);
  P.ncol = a.take<int32_t>(nnz + NCOL_PAD);
  P.t = a.take<uint32_t>(nnz / 2 + 1);
  return P;
}

size_t stage_tmp_bytes(int64_t n, int64_t nnz, int64_t dmax, int num_cu) {
  size_t build = build_tmp_bytes(n, nnz);
  size_t tri = 5 * align256((size_t)n * 4 + 4) + align256(radix_tmp_elems(n, 4) * 8) +
               align256((size_t)(n + 1) * 8 + 8) + align256(scan_tmp_elems(n) * 8) + 4096;
  (void)dmax;
  (void)num_cu;
  // the triangle and 4-cycle stages hold their workspaces at the same time
  return std::max(build, tri + c4_tmp_bytes(n)) + (1 << 16);
}

size_t c4_tmp_bytes(int64_t n, bool full_rows) {
  return 2 * align256((size_t)(n + 1) * 8 + 8) + 3 * align256((size_t)n * 4 + 4) +
         (full_rows ? align256((size_t)n * 16 + 16) : 0) +
         align256(radix_tmp_elems(n, C4_KEY_BITS) * 8) + align256(scan_tmp_elems(n) * 8) +
         align256(32 * 8) + 4096;
}

int set_error(m4_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int scal_error(m4_ctx* ctx, int err) {
  if (err & ERR_INVALID) return set_error(ctx, M4_EINVAL, "CSR is not simple, symmetric and sorted");
  if (err & ERR_PROBE)
    return set_error(ctx, M4_EINTERNAL, "an open-addressing probe ran past its table size");
  if (err) return set_error(ctx, M4_EINTERNAL, "4-cycle range plan exceeded its bound");
  return M4_OK;
}

}  // namespace m4

extern "C" int m4_ctx_create(int device, m4_ctx** out) {
  if (!out) return M4_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return M4_EDEVICE;
  }
  m4_ctx* c = new (std::nothrow) m4_ctx();
  if (!c) return M4_ENOMEM;
  c->device = device;
  try {
    M4_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    M4_HIP(hipGetDeviceProperties(&prop, device));
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->arch = std::string(prop.gcnArchName) + " " + std::to_string(c->num_cu) + " CU";
    M4_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    M4_HIP(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
    M4_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    M4_HIP(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    M4_HIP(hipMalloc((void**)&c->scal, sizeof(Scal)));
    M4_HIP(hipHostMalloc((void**)&c->scal_host, sizeof(Scal), hipHostMallocDefault));
    for (int i = 0; i < kNumEvents; i++) M4_HIP(hipEventCreate(&c->ev[i]));
    for (int k = 0; k < M4_NK; k++)
      for (int j = 0; j < 2; j++) M4_HIP(hipEventCreate(&c->ktimer.ev[k][j]));
    noalloc_setup(device);
  } catch (const HipFail& f) {
    (void)hipGetLastError();
    m4_ctx_destroy(c);
    return M4_EDEVICE;
  }
  *out = c;
  return M4_OK;
}

extern "C" void m4_ctx_destroy(m4_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->stream2) (void)hipStreamSynchronize(c->stream2);
  c->prep.release();
  c->tmp.release();
  c->big.release();
  c->big2.release();
  c->input.release();
  c->tout.release();
  c->extra.release();
  if (c->scal) (void)hipFree(c->scal);
  if (c->scal_host) (void)hipHostFree(c->scal_host);
  for (int i = 0; i < kNumEvents; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (int k = 0; k < M4_NK; k++)
    for (int j = 0; j < 2; j++)
      if (c->ktimer.ev[k][j]) (void)hipEventDestroy(c->ktimer.ev[k][j]);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  if (c->stream2) (void)hipStreamDestroy(c->stream2);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  destroy_ctx_extras(c);
  delete c;
}

extern "C" const char* m4_last_error(const m4_ctx* c) {
  return c ? c->last_error.c_str() : "no context";
}

extern "C" const char* m4_ctx_device(const m4_ctx* c) { return c ? c->arch.c_str() : "no context"; }

extern "C" const char* m4_strerror(int st) {
  switch (st) {
    case M4_OK: return "ok";
    case M4_EINVAL: return "invalid argument or malformed CSR";
    case M4_ERANGE: return "size out of range (n or nnz >= 2^31, or nnz != row_ptr[n])";
    case M4_EOVERFLOW: return "a count does not fit in 64 bits";
    case M4_ENOMEM: return "out of memory or device budget too small";
    case M4_EDEVICE: return "HIP device error";
    case M4_EBUSY: return "queue full";
    case M4_EINTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

namespace m4 {

int check_csr_args(const m4_csr* g) {
  if (!g) return M4_EINVAL;
  if (g->n < 0 || g->nnz < 0) return M4_EINVAL;
  // column positions (plus the row slack of aligned loads) must fit 32 bits
  if (g->n >= (int64_t(1) << 31) || g->nnz > (int64_t(1) << 31) - 1024) return M4_ERANGE;
  if (g->nnz % 2) return M4_EINVAL;
  if (!g->row_ptr) return M4_EINVAL;
  if (g->nnz > 0 && !g->col) return M4_EINVAL;
  return M4_OK;
}

// Brings the CSR to the device (copying host arrays into the context's input
// buffer) and returns device pointers.
void stage_input(m4_ctx* c, const m4_csr* g, hipStream_t s, const int64_t** rp,
                 const int32_t** col, double* h2d_bytes) {
  if (g->on_device) {
    *rp = g->row_ptr;
    *col = g->col;
    return;
  }
  size_t rb = align256((size_t)(g->n + 1) * 8), cb = (size_t)g->nnz * 4 + 4;
  c->input.ensure(rb + cb, s);
  int64_t* drp = reinterpret_cast<int64_t*>(c->input.ptr);
  int32_t* dcol = reinterpret_cast<int32_t*>(c->input.ptr + rb);
  M4_HIP(hipMemcpyAsync(drp, g->row_ptr, (size_t)(g->n + 1) * 8, hipMemcpyHostToDevice, s));
  if (g->nnz)
    M4_HIP(hipMemcpyAsync(dcol, g->col, (size_t)g->nnz * 4, hipMemcpyHostToDevice, s));
  if (h2d_bytes) *h2d_bytes += (double)((g->n + 1) * 8 + g->nnz * 4);
  *rp = drp;
  *col = dcol;
}

Tuning tuning_for(const m4_ctx* c, const m4_opts* o) {
  Tuning tu = c->tune;
  if (o && o->tri_wave_max > 0) tu.tri_wave_max = tu.tri_wave_far = o->tri_wave_max;
  if (o && o->c4_light_max > 0) tu.c4_light_max = o->c4_light_max;
  if (o && o->c4_med_max != 0) tu.c4_med_max = o->c4_med_max < 0 ? 0 : o->c4_med_max;
  // the light table holds C4_HASH_SLOTS keys at load <= 1/2, the medium one
  // C4_MED_SLOTS keys at load <= 3/4 in one pass
  tu.c4_light_max = std::max(0, std::min(tu.c4_light_max, C4_HASH_SLOTS / 2));
  tu.c4_med_max = std::max(0, std::min(tu.c4_med_max, 3 * C4_MED_SLOTS / 4));
  // the binned 4-cycle owners take scratch sized by the CU count, which a
  // device budget and the fixed scratch do not provide for
  if ((o && o->device_budget_bytes > 0) || c->no_alloc) tu.c4_bin_win = 0;
  return tu;
}

// The resident single-graph pipeline.  Leaves the prepared graph in c->prep
// (P) and the results in c->scal; the caller reads them back.
void run_resident(m4_ctx* c, const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz,
                  const m4_opts* o, hipStream_t s, Prep& P, bool want_timing) {
  KTimer* kt = nullptr;
  if (o && (o->flags & M4_TIMING)) {
    kt = &c->ktimer;
    kt->on = true;
    for (int i = 0; i < M4_NK; i++) kt->used[i] = false;
  }
  const uint32_t flags = o ? o->flags : 0;
  const uint32_t cache_rows = o ? o->cache_rows : 0;
  const Tuning tu = tuning_for(c, o);
  c->prep.ensure(prep_bytes(n, nnz), s);
  P = carve_prep(c->prep.ptr, n, nnz);
  fill_u32(c->scal, 0, sizeof(Scal) / 4, s);
  if (nnz / 2) fill_u32(P.t, 0, (size_t)(nnz / 2), s);
  if (want_timing) M4_HIP(hipEventRecord(c->ev[0], s));
  c->tmp.ensure(stage_tmp_bytes(n, nnz, 1, c->num_cu), s);
  Arena a;
  a.base = c->tmp.ptr;
  a.cap = c->tmp.cap;
  Classes C{};
  if (kt) kt->begin(M4_K_BUILD, s);
  build_prep(rp, col, n, nnz, (flags & M4_VALIDATE) != 0, P, C, c->scal, c->scal_host, a, s);
  if (kt) kt->end(M4_K_BUILD, s);
  // the cycle/path anchor basis (Section III-A): wedges or edge anchors
  c->basis = choose_basis(P, tu, flags, o && o->device_budget_bytes > 0, c->scal, c->cost_pair, s);
  if (want_timing) M4_HIP(hipEventRecord(c->ev[1], s));
  auto big = [c, s](size_t bytes) -> char* {
    c->big.ensure(bytes, s);
    return c->big.ptr;
  };
  auto big2 = [c, s](size_t bytes) -> char* {
    c->big2.ensure(bytes, s);
    return c->big2.ptr;
  };
  // both anchor stages are planned first, each in its own part of the
  // workspace; their heavy kernels then run concurrently, the 4-cycle stage
  // on the context's second stream (forked from and joined back into s), so
  // that each fills the CUs the other's tail leaves idle (triangle kernels
  // are queued first: measured slightly ahead of the reverse order).  When
  // 4-cycle owners are binned the stages run in order: the binning kernel
  // keeps two persistent workgroups and all of the LDS on every CU, and
  // sharing the CUs with the triangle kernels measured slower.
  const size_t c4_bytes = c4_tmp_bytes(n);
  Arena at, ac;
  at.base = c->tmp.ptr;
  at.cap = c->tmp.cap - c4_bytes;
  ac.base = c->tmp.ptr + at.cap;
  ac.cap = c4_bytes;
  Launch tri = tri_plan(P, c->scal, tu, flags, cache_rows, at, s, c->num_cu, big, kt);
  bool binned = false;
  Launch c4 = c->basis.edge ? edge_plan(P, c->scal, flags, c->num_cu, kt)
                            : c4_plan(P, C, c->scal, tu, flags, ac, s, c->num_cu, kt, big2, &binned);
  if ((flags & M4_SERIAL) || binned) {
    tri(s);
    if (want_timing) M4_HIP(hipEventRecord(c->ev[2], s));
    c4(s);
  } else {
    M4_HIP(hipEventRecord(c->fork_ev, s));
    M4_HIP(hipStreamWaitEvent(c->stream2, c->fork_ev, 0));
    tri(s);
    c4(c->stream2);
    if (want_timing) M4_HIP(hipEventRecord(c->ev[2], s));
    M4_HIP(hipEventRecord(c->join_ev, c->stream2));
    M4_HIP(hipStreamWaitEvent(s, c->join_ev, 0));
  }
  if (want_timing) M4_HIP(hipEventRecord(c->ev[3], s));
  if (kt) kt->begin(M4_K_CLOSURE, s);
  closure_run(P, c->scal, flags, s);
  finalize_run(c->scal, s, c->basis.edge);
  if (kt) kt->end(M4_K_CLOSURE, s);
  if (want_timing) M4_HIP(hipEventRecord(c->ev[4], s));
}

void fill_stats(m4_ctx* c, const Scal& h, m4_stats* st, bool timing) {
  if (!st) return;
  for (int i = 0; i < 8; i++) st->basis[i] = h.basis[i];
  st->intersect_steps = h.stat[ST_STEPS];
  st->wedges = h.stat[ST_WEDGES];
  st->cache_lookups = h.stat[ST_LOOKUPS];
  st->cache_hits = h.stat[ST_HITS];
  st->basis_used = c->basis.edge ? 1u : 0u;
  st->cost_wedge = c->basis.cost_wedge;
  st->cost_edge = c->basis.cost_edge;
  for (int k = 0; k < M4_NK; k++) {
    st->k_elems[k] = h.kstat[k][0];
    st->k_rows[k] = h.kstat[k][1];
    st->k_aux[k] = h.kstat[k][2];
    st->k_aux2[k] = h.kstat[k][3];
  }
  if (c->ktimer.on) {
    for (int k = 0; k < M4_NK; k++) {
      float ms = 0;
      if (c->ktimer.used[k] &&
          hipEventElapsedTime(&ms, c->ktimer.ev[k][0], c->ktimer.ev[k][1]) == hipSuccess)
        st->ms_kernel[k] = ms;
    }
    c->ktimer.on = false;
  }
  if (timing) {
    float ms[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; i++) (void)hipEventElapsedTime(&ms[i], c->ev[i], c->ev[i + 1]);
    st->ms_build = ms[0];
    st->ms_tri = ms[1];
    st->ms_c4 = ms[2];
    st->ms_closure = ms[3];
  }
}

}  // namespace m4

#define M4_GUARD_BEGIN try {
#define M4_GUARD_END                                                                      \
  }                                                                                       \
  catch (const HipFail& f) {                                                              \
    char buf[512];                                                                        \
    snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", f.what, hipGetErrorString(f.e),   \
             f.file, f.line);                                                             \
    (void)hipGetLastError();                                                              \
    return set_error(ctx, M4_EDEVICE, buf);                                               \
  }                                                                                       \
  catch (const Fail& f) {                                                                 \
    return set_error(ctx, f.code, f.msg);                                                 \
  }                                                                                       \
  catch (const std::bad_alloc&) {                                                         \
    return set_error(ctx, M4_ENOMEM, "host allocation failed");                           \
  }                                                                                       \
  catch (...) {                                                                           \
    return set_error(ctx, M4_EINTERNAL, "unexpected exception");                          \
  }

extern "C" int m4_count_motifs4_ex(m4_ctx* ctx, const m4_csr* g, const m4_opts* o,
                                   uint64_t out[6], m4_stats* st) {
  if (!ctx || !out) return M4_EINVAL;
  int rc = check_csr_args(g);
  if (rc) return set_error(ctx, rc, "bad CSR arguments");
  M4_GUARD_BEGIN
  M4_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : ctx->stream;
  const bool timing = st && o && (o->flags & (M4_STATS | M4_TIMING));
  if (st) memset(st, 0, sizeof(*st));
  if (g->n < 4 || g->nnz == 0) {
    for (int i = 0; i < 6; i++) out[i] = 0;
    if (st) st->partitions = 1;
    return M4_OK;
  }
  if (needs_partition(ctx, g, o)) return count_partitioned(ctx, g, o, out, st);
  double h2d = 0;
  if (timing) M4_HIP(hipEventRecord(ctx->ev[5], s));
  const int64_t* rp;
  const int32_t* col;
  stage_input(ctx, g, s, &rp, &col, &h2d);
  if (!g->on_device) {
    // row_ptr[n] must equal nnz
    int64_t last = 0;
    M4_HIP(hipMemcpyAsync(&last, rp + g->n, 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    if (last != g->nnz) return set_error(ctx, M4_ERANGE, "row_ptr[n] != nnz");
  }
  if (timing) M4_HIP(hipEventRecord(ctx->ev[6], s));
  Prep P;
  run_resident(ctx, rp, col, g->n, g->nnz, o, s, P, timing);
  M4_HIP(hipMemcpyAsync(ctx->scal_host, ctx->scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  const Scal& h = *ctx->scal_host;
  if (h.err) return scal_error(ctx, h.err);
  if (h.status == 3) return set_error(ctx, M4_EOVERFLOW, "a count is >= 2^64");
  if (h.status != 0) return set_error(ctx, M4_EINTERNAL, "closure consistency check failed");
  for (int i = 0; i < 6; i++) out[i] = h.out[i];
  if (st) {
    fill_stats(ctx, h, st, timing);
    st->k_elems[M4_K_BUILD] = (uint64_t)g->nnz;
    st->k_rows[M4_K_BUILD] = (uint64_t)g->n;
    st->k_elems[M4_K_CLOSURE] = (uint64_t)(g->nnz / 2);
    st->k_rows[M4_K_CLOSURE] = (uint64_t)g->n;
    st->partitions = 1;
    st->h2d_bytes = (uint64_t)h2d;
    st->device_bytes = ctx->held_bytes();
    if (timing) {
      float ms = 0, mh = 0;
      (void)hipEventElapsedTime(&ms, ctx->ev[5], ctx->ev[4]);
      (void)hipEventElapsedTime(&mh, ctx->ev[5], ctx->ev[6]);
      st->ms_total = ms;
      st->ms_h2d = mh;
    }
  }
  return M4_OK;
  M4_GUARD_END
}

extern "C" int m4_edge_triangles(m4_ctx* ctx, const m4_csr* g, const m4_opts* o, uint32_t* t_out) {
  if (!ctx || !t_out) return M4_EINVAL;
  int rc = check_csr_args(g);
  if (rc) return set_error(ctx, rc, "bad CSR arguments");
  M4_GUARD_BEGIN
  M4_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : ctx->stream;
  if (g->nnz == 0) return M4_OK;
  const int64_t* rp;
  const int32_t* col;
  stage_input(ctx, g, s, &rp, &col, nullptr);
  Prep P;
  const uint32_t flags = o ? o->flags : 0;
  const Tuning tu = tuning_for(ctx, o);
  ctx->prep.ensure(prep_bytes(g->n, g->nnz), s);
  P = carve_prep(ctx->prep.ptr, g->n, g->nnz);
  fill_u32(ctx->scal, 0, sizeof(Scal) / 4, s);
  fill_u32(P.t, 0, (size_t)(g->nnz / 2), s);
  ctx->tmp.ensure(stage_tmp_bytes(g->n, g->nnz, 1, ctx->num_cu), s);
  Arena a;
  a.base = ctx->tmp.ptr;
  a.cap = ctx->tmp.cap;
  Classes C{};
  build_prep(rp, col, g->n, g->nnz, (flags & M4_VALIDATE) != 0, P, C, ctx->scal, ctx->scal_host,
             a, s);
  a.used = 0;
  auto big = [ctx, s](size_t bytes) -> char* {
    ctx->big.ensure(bytes, s);
    return ctx->big.ptr;
  };
  tri_run(P, ctx->scal, tu, flags, o ? o->cache_rows : 0, a, s, ctx->num_cu, big, nullptr);
  uint32_t* dst = t_out;
  if (!g->on_device) {
    ctx->tout.ensure((size_t)g->nnz * 4, s);
    dst = reinterpret_cast<uint32_t*>(ctx->tout.ptr);
  }
  edge_t_to_input(P, rp, col, dst, s);
  if (!g->on_device)
    M4_HIP(hipMemcpyAsync(t_out, dst, (size_t)g->nnz * 4, hipMemcpyDeviceToHost, s));
  M4_HIP(hipMemcpyAsync(ctx->scal_host, ctx->scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  if (ctx->scal_host->err) return scal_error(ctx, ctx->scal_host->err);
  return M4_OK;
  M4_GUARD_END
}

extern "C" int m4_count_orbits4(m4_ctx* ctx, const m4_csr* g, const m4_opts* o,
                                uint64_t* orbits) {
  if (!ctx || !orbits) return M4_EINVAL;
  int rc = check_csr_args(g);
  if (rc) return set_error(ctx, rc, "bad CSR arguments");
  if (o && o->device_budget_bytes > 0)
    return set_error(ctx, M4_EINVAL, "orbit counts need the whole graph resident (no budget)");
  M4_GUARD_BEGIN
  M4_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : ctx->stream;
  const int64_t n = g->n;
  if (n == 0) return M4_OK;
  const size_t out_bytes = (size_t)n * 11 * sizeof(uint64_t);
  if (g->nnz == 0) {
    if (g->on_device) {
      fill_u32(orbits, 0, out_bytes / 4, s);
      M4_HIP(hipStreamSynchronize(s));
    } else {
      memset(orbits, 0, out_bytes);
    }
    return M4_OK;
  }
  const int64_t* rp;
  const int32_t* col;
  stage_input(ctx, g, s, &rp, &col, nullptr);
  if (!g->on_device) {
    int64_t last = 0;
    M4_HIP(hipMemcpyAsync(&last, rp + n, 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    if (last != g->nnz) return set_error(ctx, M4_ERANGE, "row_ptr[n] != nnz");
  }
  const uint32_t flags = o ? (o->flags & M4_VALIDATE) : 0;
  const Tuning tu = tuning_for(ctx, o);
  ctx->prep.ensure(prep_bytes(n, g->nnz), s);
  Prep P = carve_prep(ctx->prep.ptr, n, g->nnz);
  fill_u32(ctx->scal, 0, sizeof(Scal) / 4, s);
  fill_u32(P.t, 0, (size_t)(g->nnz / 2), s);
  ctx->tmp.ensure(stage_tmp_bytes(n, g->nnz, 1, ctx->num_cu), s);
  Arena a;
  a.base = ctx->tmp.ptr;
  a.cap = ctx->tmp.cap;
  Classes C{};
  build_prep(rp, col, n, g->nnz, (flags & M4_VALIDATE) != 0, P, C, ctx->scal, ctx->scal_host, a,
             s);
  a.used = 0;
  auto big = [ctx, s](size_t bytes) -> char* {
    ctx->big.ensure(bytes, s);
    return ctx->big.ptr;
  };
  tri_run(P, ctx->scal, tu, flags, 0, a, s, ctx->num_cu, big, nullptr);
  // statistics (8 n words) and the bitmap slices of out-degrees above the
  // LDS bound in big2; the 4-cycle counters (4 n bytes per workgroup, 8 n
  // from degree 2^16, at most 16 GiB, at most one workgroup per CU: more
  // workgroups measured slower, their counters crowding the caches) in big
  const int kmax = local_dplus_max(P, ctx->scal, s);
  const size_t arr_bytes = align256((size_t)n * 8 * 8);
  int gblocks = 0;
  size_t g_bytes = 0;
  if (kmax > 512) {
    const size_t per = local_glob_stride_words(kmax) * 8;
    gblocks = (int)std::max<size_t>(1, std::min<size_t>((size_t(1) << 30) / per, 64));
    g_bytes = (size_t)gblocks * per;
  }
  ctx->big2.ensure(arr_bytes + g_bytes, s);
  const bool wide = C.dmax >= 65536;
  const int64_t cword = wide ? 8 : 4;
  const int cblocks = (int)std::max<int64_t>(
      1, std::min<int64_t>((int64_t(16) << 30) / ((int64_t)n * cword), (int64_t)ctx->num_cu));
  ctx->big.ensure((size_t)cblocks * (size_t)n * (size_t)cword, s);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(orbits);
  if (!g->on_device) {
    ctx->tout.ensure(out_bytes, s);
    dst = reinterpret_cast<unsigned long long*>(ctx->tout.ptr);
  }
  local_orbits(P, C, ctx->scal, reinterpret_cast<unsigned long long*>(ctx->big2.ptr),
               ctx->big.ptr, wide, cblocks,
               gblocks ? reinterpret_cast<unsigned long long*>(ctx->big2.ptr + arr_bytes) : nullptr,
               gblocks, kmax, dst, ctx->num_cu, s);
  if (!g->on_device) M4_HIP(hipMemcpyAsync(orbits, dst, out_bytes, hipMemcpyDeviceToHost, s));
  M4_HIP(hipMemcpyAsync(ctx->scal_host, ctx->scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  const Scal& h = *ctx->scal_host;
  if (h.err & 8) return set_error(ctx, M4_EINTERNAL, "per-vertex orbit inverse went negative");
  if (h.err) return scal_error(ctx, h.err);
  if (h.status == 3) return set_error(ctx, M4_EOVERFLOW, "an orbit count is >= 2^64");
  return M4_OK;
  M4_GUARD_END
}

static std::once_flag g_default_once;
static m4_ctx* g_default = nullptr;
static int g_default_rc = M4_OK;
static std::mutex g_default_mu;

extern "C" int m4_count_motifs4(const m4_csr* g, uint64_t out[6]) {
  std::call_once(g_default_once, [] { g_default_rc = m4_ctx_create(0, &g_default); });
  if (g_default_rc != M4_OK) return g_default_rc;
  std::lock_guard<std::mutex> lk(g_default_mu);
  return m4_count_motifs4_ex(g_default, g, nullptr, out, nullptr);
}
