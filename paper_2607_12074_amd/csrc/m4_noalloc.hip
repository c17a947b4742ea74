// m4_noalloc.hip -- the single-graph count for callers that cannot allocate
// device memory: every workspace of the resident count is carved from one
// fixed array in device memory instead of the context's growable buffers.
//
// scratch is a file-scope __device__ array; each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is
// only a stand-in symbol): noalloc_setup() looks up the device address once
// per device with hipGetSymbolAddress, with that device current, and every
// use goes through that address.
#include <mutex>

#include "m4_ctx.h"

namespace m4 {

constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    // the other entry points do not need it: this one reports M4_EDEVICE
    (void)hipGetLastError();
    return;
  }
  g_scratch_ptr[device] = static_cast<char*>(p);
}

static char* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace m4

using namespace m4;

extern "C" int m4_count_motifs4_noalloc(m4_ctx* ctx, const m4_csr* g, const m4_opts* o,
                                        uint64_t out[6]) {
  if (!ctx || !out) return M4_EINVAL;
  int rc = check_csr_args(g);
  if (rc) return set_error(ctx, rc, "bad CSR arguments");
  if (!g->on_device) return set_error(ctx, M4_EINVAL, "the CSR must be in device memory");
  if (o && o->device_budget_bytes > 0)
    return set_error(ctx, M4_EINVAL, "no device budget here: the scratch is the budget");
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : ctx->stream;
  try {
    M4_HIP(hipSetDevice(ctx->device));
    char* base = scratch_of(ctx->device);
    if (!base) return set_error(ctx, M4_EDEVICE, "fixed scratch address unknown on this device");
    if (g->n < 4 || g->nnz == 0) {
      for (int i = 0; i < 6; i++) out[i] = 0;
      return M4_OK;
    }
    // the prepared graph and the stage workspace are known up front; the
    // hub tables and 4-cycle descriptors are carved while the stages are
    // planned and fail the call (before their kernels) if they do not fit
    const size_t need = ((prep_bytes(g->n, g->nnz) + 255) & ~size_t(255)) +
                        stage_tmp_bytes(g->n, g->nnz, 1, ctx->num_cu);
    if (need > kNoAllocBytes)
      return set_error(ctx, M4_ENOMEM,
                       "graph needs " + std::to_string(need) + " bytes of workspace; the fixed " +
                           "scratch holds " + std::to_string(kNoAllocBytes));
    ScratchPool pool;
    pool.base = base;
    pool.cap = kNoAllocBytes;
    // the context's own buffers are set aside for the call and put back
    // after it, whatever happens
    struct Swap {
      m4_ctx* c;
      DevBuf saved[4];
      explicit Swap(m4_ctx* c_, ScratchPool* p) : c(c_) {
        DevBuf* bufs[4] = {&c->prep, &c->tmp, &c->big, &c->big2};
        for (int i = 0; i < 4; i++) {
          saved[i] = *bufs[i];
          *bufs[i] = DevBuf{};
          bufs[i]->pool = p;
        }
        c->no_alloc = true;
      }
      ~Swap() {
        DevBuf* bufs[4] = {&c->prep, &c->tmp, &c->big, &c->big2};
        for (int i = 0; i < 4; i++) *bufs[i] = saved[i];
        c->no_alloc = false;
      }
    } swap(ctx, &pool);
    m4_opts oo{};
    if (o) oo = *o;
    oo.flags &= ~(uint32_t)(M4_TIMING | M4_FORCE_PARTITION);
    Prep P;
    run_resident(ctx, g->row_ptr, g->col, g->n, g->nnz, &oo, s, P, false);
    M4_HIP(hipMemcpyAsync(ctx->scal_host, ctx->scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    const Scal& h = *ctx->scal_host;
    if (h.err) return scal_error(ctx, h.err);
    if (h.status == 3) return set_error(ctx, M4_EOVERFLOW, "a count is >= 2^64");
    if (h.status != 0) return set_error(ctx, M4_EINTERNAL, "closure consistency check failed");
    for (int i = 0; i < 6; i++) out[i] = h.out[i];
    return M4_OK;
  } catch (const HipFail& f) {
    (void)hipGetLastError();
    return set_error(ctx, M4_EDEVICE, std::string(f.what) + " failed: " + hipGetErrorString(f.e));
  } catch (const Fail& f) {
    // a workspace that did not fit: the launches queued before it finish
    // before the scratch can be handed to another call
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(ctx->stream2);
    return set_error(ctx, f.code, f.msg);
  } catch (...) {
    return set_error(ctx, M4_EINTERNAL, "unexpected exception");
  }
}
