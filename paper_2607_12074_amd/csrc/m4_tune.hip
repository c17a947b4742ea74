// m4_tune.hip -- autotuner of the degree-bucket and tile thresholds.
//
// Candidate settings are timed on a caller-supplied sample (a graph for the
// single-graph path, an arena for the fused batched launch); the fastest is
// kept in the context.  Every candidate must give the same counts -- the
// thresholds only move owners between kernels -- and a disagreement is an
// internal error, not a tuning choice.
#include <string.h>

#include <chrono>
#include <vector>

#include "m4_ctx.h"

namespace m4 {
int count_batch_impl(m4_ctx* c, const m4_batch* b, const m4_opts* o, uint64_t* out,
                     m4_stats* st);
}

using namespace m4;

namespace {

double wall_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void to_public(const Tuning& t, m4_tuning* out) {
  memset(out, 0, sizeof(*out));
  out->tri_wave_max = t.tri_wave_max;
  out->c4_light_max = t.c4_light_max;
  out->batch_variant = t.batch_variant;
  out->batch_light = t.batch_light;
  out->hub_min = t.hub_min;
  out->c4_med_max = t.c4_med_max;
  out->probe_w = t.probe_w;
  out->c4_med_win = t.c4_med_win;
  out->c4_bin_win = t.c4_bin_win;
  out->c4_bin_cap = t.c4_bin_cap;
  out->c4_bin_dense = t.c4_bin_dense;
  out->probe_w_far = t.probe_w_far;
  out->tri_wave_far = t.tri_wave_far;
}

}  // namespace

extern "C" int m4_get_tuning(const m4_ctx* ctx, m4_tuning* out) {
  if (!ctx || !out) return M4_EINVAL;
  to_public(ctx->tune, out);
  return M4_OK;
}

extern "C" int m4_set_tuning(m4_ctx* ctx, const m4_tuning* t) {
  if (!ctx || !t) return M4_EINVAL;
  if (t->tri_wave_max < 2 || t->tri_wave_max > 64 || t->c4_light_max < 1 ||
      t->c4_light_max > C4_HASH_SLOTS / 2 || (t->batch_variant != 0 && t->batch_variant != 1) ||
      t->batch_light < 1 || t->batch_light > 256 ||
      (t->hub_min != 0 && (t->hub_min < 4 || t->hub_min > 65536)) || t->c4_med_max < 0 ||
      t->c4_med_max > 3 * C4_MED_SLOTS / 4 || t->probe_w < 1 || t->probe_w > 256 ||
      t->c4_med_win < 0 || t->c4_med_win > 65536 || t->c4_bin_win < 0 || t->c4_bin_win > 65536 ||
      (t->c4_bin_cap != 0 && (t->c4_bin_cap < 64 || t->c4_bin_cap > (1 << 24))) ||
      (t->c4_bin_dense != 0 && (t->c4_bin_dense < 64 || t->c4_bin_dense > (1 << 20))) ||
      t->probe_w_far < 1 || t->probe_w_far > 256 || t->tri_wave_far < 2 || t->tri_wave_far > 64)
    return set_error(ctx, M4_EINVAL, "tuning value out of range");
  ctx->tune.tri_wave_max = t->tri_wave_max;
  ctx->tune.c4_light_max = t->c4_light_max;
  ctx->tune.batch_variant = t->batch_variant;
  ctx->tune.batch_light = t->batch_light;
  ctx->tune.hub_min = t->hub_min;
  ctx->tune.c4_med_max = t->c4_med_max;
  ctx->tune.probe_w = t->probe_w;
  ctx->tune.c4_med_win = t->c4_med_win;
  ctx->tune.c4_bin_win = t->c4_bin_win;
  ctx->tune.c4_bin_cap = t->c4_bin_cap;
  ctx->tune.c4_bin_dense = t->c4_bin_dense;
  ctx->tune.probe_w_far = t->probe_w_far;
  ctx->tune.tri_wave_far = t->tri_wave_far;
  return M4_OK;
}

extern "C" int m4_autotune(m4_ctx* ctx, const m4_csr* graph, const m4_batch* batch, int reps,
                           m4_tuning* out) {
  if (!ctx || (!graph && !batch)) return M4_EINVAL;
  if (reps < 1) reps = 3;
  const Tuning start = ctx->tune;
  Tuning best = start;
  try {
    if (graph) {
      // one candidate: a warm run, then the best of reps timed runs; every
      // candidate must reproduce the first one's counts
      uint64_t ref[6];
      bool have_ref = false;
      auto time_cfg = [&](const Tuning& t, double* ms) -> int {
        ctx->tune = t;
        uint64_t cnt[6];
        int rc = m4_count_motifs4_ex(ctx, graph, nullptr, cnt, nullptr);
        if (rc != M4_OK) return rc;
        if (!have_ref) {
          memcpy(ref, cnt, sizeof(ref));
          have_ref = true;
        } else if (memcmp(ref, cnt, sizeof(ref)) != 0) {
          return set_error(ctx, M4_EINTERNAL, "autotune: thresholds changed the counts");
        }
        *ms = 1e300;
        for (int r = 0; r < reps; r++) {
          const double t0 = wall_ms();
          rc = m4_count_motifs4_ex(ctx, graph, nullptr, cnt, nullptr);
          if (rc != M4_OK) return rc;
          *ms = std::min(*ms, wall_ms() - t0);
        }
        return M4_OK;
      };
      double best_ms = 1e300;
      auto try_cfg = [&](const Tuning& t) -> int {
        double ms;
        const int rc = time_cfg(t, &ms);
        if (rc == M4_OK && ms < best_ms) {
          best_ms = ms;
          best = t;
        }
        return rc;
      };
      // bucket bounds first, then the hub-table threshold with the probe
      // weight, then the medium 4-cycle bucket, each at the best setting
      // found so far
      const int waves[] = {16, 32, 64};
      const int lights[] = {256, 512, 1024, 2048};
      for (int w : waves)
        for (int l : lights) {
          Tuning t = start;
          t.tri_wave_max = w;  // the sample graph decides which of the two bounds applies
          t.tri_wave_far = w;
          t.c4_light_max = l;
          const int rc = try_cfg(t);
          if (rc != M4_OK) {
            ctx->tune = start;
            return rc;
          }
        }
      const int hub_mins[] = {0, 16, 32, 64, 128};
      const int probe_ws[] = {4, 8, 16, 32};
      const Tuning after_buckets = best;
      for (int hm : hub_mins)
        for (int pw : probe_ws) {
          if (hm == 0 && pw != probe_ws[0]) continue;  // no tables: the weight is unused
          Tuning t = after_buckets;
          t.hub_min = hm;
          t.probe_w = pw;  // the sample graph decides which of the two weights applies
          t.probe_w_far = pw;
          const int rc = try_cfg(t);
          if (rc != M4_OK) {
            ctx->tune = start;
            return rc;
          }
        }
      const int meds[] = {0, 6144, 12288};
      const int med_wins[] = {0, 32, 64, 128};
      const Tuning after_hubs = best;
      for (int md : meds)
        for (int mw : med_wins) {
          if (md == 0 && mw != med_wins[0]) continue;  // no medium bucket at all
          Tuning t = after_hubs;
          t.c4_med_max = md;
          t.c4_med_win = mw;
          const int rc = try_cfg(t);
          if (rc != M4_OK) {
            ctx->tune = start;
            return rc;
          }
        }
      const int bin_wins[] = {0, 2, 4, 6, 8, 16};
      const int bin_denses[] = {0, 4096, 8192, 16384};
      const Tuning after_med = best;
      for (int bw : bin_wins)
        for (int bd : bin_denses) {
          if (bw == 0 && bd != bin_denses[0]) continue;  // nothing binned
          Tuning t = after_med;
          t.c4_bin_win = bw;
          t.c4_bin_dense = bd;
          const int rc = try_cfg(t);
          if (rc != M4_OK) {
            ctx->tune = start;
            return rc;
          }
        }
      ctx->tune = start;
    }
    if (batch) {
      const int64_t G = batch->num_graphs;
      if (G <= 0) return set_error(ctx, M4_EINVAL, "autotune: empty batch");
      std::vector<uint64_t> ref((size_t)G * 6), cnt((size_t)G * 6);
      bool have_ref = false;
      double best_ms = 1e300;
      const int lights[] = {32, 64, 128, 256};
      for (int variant = 0; variant < 2; variant++)
        for (int l : lights) {
          ctx->tune.batch_variant = variant;
          ctx->tune.batch_light = l;
          m4_opts o{};
          int rc = count_batch_impl(ctx, batch, &o, cnt.data(), nullptr);  // plan + capture
          if (rc != M4_OK) {
            ctx->tune = start;
            return rc;
          }
          if (!have_ref) {
            ref = cnt;
            have_ref = true;
          } else if (ref != cnt) {
            ctx->tune = start;
            return set_error(ctx, M4_EINTERNAL, "autotune: thresholds changed the counts");
          }
          double ms = 1e300;
          for (int r = 0; r < reps; r++) {
            const double t0 = wall_ms();
            rc = count_batch_impl(ctx, batch, &o, cnt.data(), nullptr);  // replay
            if (rc != M4_OK) {
              ctx->tune = start;
              return rc;
            }
            ms = std::min(ms, wall_ms() - t0);
          }
          if (ms < best_ms) {
            best_ms = ms;
            best.batch_variant = variant;
            best.batch_light = l;
          }
        }
    }
  } catch (const HipFail& f) {
    (void)hipGetLastError();
    ctx->tune = start;
    return set_error(ctx, M4_EDEVICE, std::string(f.what) + ": " + hipGetErrorString(f.e));
  } catch (const Fail& f) {
    ctx->tune = start;
    return set_error(ctx, f.code, f.msg);
  }
  ctx->tune = best;
  if (out) to_public(best, out);
  return M4_OK;
}
