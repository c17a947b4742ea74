// m4_part.hip -- halo-partitioned path (graphs larger than a device budget).
#include "m4_ctx.h"

namespace m4 {

bool needs_partition(m4_ctx* c, const m4_csr* g, const m4_opts* o) {
  (void)c;
  (void)g;
  if (!o) return false;
  return (o->flags & M4_FORCE_PARTITION) || o->device_budget_bytes > 0;
}

int count_partitioned(m4_ctx* c, const m4_csr* g, const m4_opts* o, uint64_t out[6],
                      m4_stats* st) {
  (void)g;
  (void)o;
  (void)out;
  (void)st;
  return set_error(c, M4_EINVAL, "partitioned path not available");
}

void destroy_ctx_extras(m4_ctx* c) { (void)c; }

}  // namespace m4

extern "C" int m4_count_batch(m4_ctx* ctx, const m4_batch* b, const m4_opts* o, uint64_t* out,
                              m4_stats* st) {
  (void)b;
  (void)o;
  (void)out;
  (void)st;
  return m4::set_error(ctx, M4_EINVAL, "batch path not available");
}
extern "C" int m4_server_create(m4_ctx*, uint64_t, int, m4_server** out) {
  if (out) *out = nullptr;
  return M4_EINVAL;
}
extern "C" int m4_server_submit(m4_server*, const m4_csr*, uint64_t, uint64_t*) { return M4_EINVAL; }
extern "C" int m4_server_poll(m4_server*, m4_result*, int, int* got) {
  if (got) *got = 0;
  return M4_EINVAL;
}
extern "C" int m4_server_drain(m4_server*) { return M4_EINVAL; }
extern "C" void m4_server_destroy(m4_server*) {}
extern "C" double m4_server_now_ms(const m4_server*) { return 0.0; }
