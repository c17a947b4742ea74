// m4_part.hip -- halo-partitioned path for graphs larger than a device budget
// (ownership-preserving partitioned derivation, Section III-E).
//
// The graph stays in host memory.  Its degree order is computed on the device
// (n-sized arrays only), then the relabelled, sorted rank-space CSR is built
// by streaming chunks of rows through the row-sort kernels into pinned host
// memory.  The anchors are then counted over contiguous rank ranges of
// owners, each range uploaded with its halo (the rows its anchors read):
//   triangles / 4-cliques: owner = lowest vertex; the range's out-lists plus
//     the out-lists of their out-neighbours (radius-1 oriented halo);
//   4-cycles: owner = highest vertex; the lower lists of the range plus the
//     rows of their lower neighbours, cut below the range's upper end;
//   closure: owner = lower end of every oriented edge; out-lists only.
// Every anchor is counted by exactly the one range holding its owner, linear
// sums add across ranges, and the per-edge triangle counts live in one device
// array that every range adds into, so the closure sees complete t_e (the
// sum of C(t_e, 2) is not linear in the ranges).  Integer adds commute, so
// the result equals the resident count bit for bit.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "m4_ctx.h"
#include "m4_device.h"

namespace m4 {

namespace {

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// nptr_p[v] = val for every (v, val) of a partition's row table
__global__ void k_scatter_rows(const int64_t* __restrict__ pairs, int64_t cnt,
                               int64_t* __restrict__ nptr_p, int32_t* __restrict__ row_len,
                               const int32_t* __restrict__ lens) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int64_t v = pairs[2 * i], off = pairs[2 * i + 1];
  nptr_p[v] = off;
  if (row_len) row_len[v] = lens[i];
}

struct Pinned {
  char* p = nullptr;
  size_t cap = 0;
  void ensure(size_t b) {
    if (b <= cap) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    M4_HIP(hipHostMalloc((void**)&p, b, hipHostMallocDefault));
    cap = b;
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

// rank-space CSR in host memory
struct HostCsr {
  int64_t n = 0, nnz = 0, m = 0;
  std::vector<int32_t> perm, rank, dr, dlo, dplus;
  std::vector<int64_t> nptr, optr;
  Pinned ncol;  // int32[nnz]
  const int32_t* col() const { return reinterpret_cast<const int32_t*>(ncol.p); }
};

// Host threads for the halo planning and gathers (at most 16).
int host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, h));
}

// f(begin, end) over [0, n) split evenly across nt threads (the caller's
// thread takes the first share); f must not throw.
template <class F>
void parallel_for(int64_t n, int nt, F&& f) {
  if (n <= 0) return;
  nt = (int)std::min<int64_t>(nt, n);
  if (nt <= 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; t++) th.emplace_back([&, t] { f(n * t / nt, n * (t + 1) / nt); });
  f(int64_t(0), n / nt);
  for (auto& x : th) x.join();
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// A row of a partition: entries [first, first + len) of row v.
struct RowPart {
  int32_t v;
  int64_t first;
  int32_t len;
};

// Rank-space rows in host memory, as the range planners read them.
struct HostRows {
  int64_t n = 0;
  const int64_t* nptr = nullptr;
  const int32_t* col = nullptr;
  const int32_t* dr = nullptr;
  const int32_t* dlo = nullptr;
  const int32_t* dplus = nullptr;
};

// Owner ranges of the triangle / 4-clique anchor (owner = lowest vertex):
// a range holds its owners' out-lists and the out-lists of their
// out-neighbours (radius-1 oriented halo), 4 bytes per entry and 28 per row.
struct TriPlanner {
  const HostRows& H;
  std::vector<uint32_t> mark;
  uint32_t stamp = 0;
  explicit TriPlanner(const HostRows& h) : H(h), mark(h.n, 0) {}
  // the largest range [lo, hi) whose rows fit cap bytes (at least one owner;
  // bytes then tells whether even that one fits)
  int64_t next(int64_t lo, size_t cap, std::vector<RowPart>& rows, size_t& bytes) {
    stamp++;
    rows.clear();
    bytes = 0;
    int64_t hi = lo;
    auto need_row = [&](int32_t v) {
      return mark[v] == stamp ? (size_t)0 : (size_t)H.dplus[v] * 4 + 28;
    };
    auto put = [&](int32_t v) {
      if (mark[v] == stamp) return;
      mark[v] = stamp;
      rows.push_back({v, (int64_t)H.dlo[v], H.dplus[v]});
    };
    while (hi < H.n) {
      size_t add = need_row((int32_t)hi);
      const int64_t b0 = H.nptr[hi] + H.dlo[hi];
      const int32_t dp = H.dplus[hi];
      constexpr int kAhead = 16;  // mark[] and the degree arrays miss the caches
      for (int32_t j = 0; j < dp; j++) {
        if (j + kAhead < dp) {
          const int32_t w = H.col[b0 + j + kAhead];
          __builtin_prefetch(&mark[w]);
          __builtin_prefetch(&H.dplus[w]);
          __builtin_prefetch(&H.dlo[w]);
        }
        add += need_row(H.col[b0 + j]);
      }
      if (bytes + add > cap && hi > lo) break;
      bytes += add;
      put((int32_t)hi);
      for (int32_t j = 0; j < dp; j++) put(H.col[b0 + j]);
      hi++;
    }
    return hi;
  }
};

// Owner ranges of the 4-cycle anchor (owner = highest vertex, from r1): a
// range holds the rows of its owners and of their lower neighbours, each cut
// below the range's end: 4 bytes per entry, 32 per row, 16 per lower
// neighbour of an owner (segment descriptor) and 4 per owner, plus 512 of
// alignment.
struct C4Planner {
  const HostRows& H;
  int64_t r1;
  std::vector<int64_t> lptr;
  std::vector<int32_t> ulen;  // per lower entry of an owner: row v's entries up to the owner
  struct Held {
    uint32_t stamp;
    int32_t len;
  };
  std::vector<Held> held;
  uint32_t stamp = 0;
  // For every lower neighbour v of an owner u, u sits at position j of row
  // v's upper part, and v's slot in u's lower part is the count of lower
  // neighbours of u below v, so one ascending sweep over the rows fills
  // every slot.  Each host thread sweeps all rows for the owners of its own
  // share (balanced by lower entries), keeping per-owner cursors.
  C4Planner(const HostRows& h, int64_t r1_, int nthreads)
      : H(h), r1(r1_), lptr(h.n + 1, 0), held(h.n, Held{0, 0}) {
    const int64_t n = H.n;
    for (int64_t u = 0; u < n; u++) lptr[u + 1] = lptr[u] + (u >= r1 ? H.dlo[u] : 0);
    ulen.assign((size_t)lptr[n] + 1, 0);
    std::vector<int64_t> cut(nthreads + 1, n);
    cut[0] = std::min(r1, n);
    for (int t = 1; t < nthreads; t++)
      cut[t] = std::lower_bound(lptr.begin(), lptr.end(), lptr[n] * t / nthreads) - lptr.begin();
    for (int t = 1; t <= nthreads; t++) cut[t] = std::max(cut[t], cut[t - 1]);
    parallel_for(nthreads, nthreads, [&](int64_t a, int64_t b) {
      for (int64_t t = a; t < b; t++) {
        const int64_t ua = cut[t], ube = cut[t + 1];
        if (ua >= ube) continue;
        std::vector<int32_t> cur(ube - ua, 0);
        // rows from ube on cannot hold an owner of this share in their upper part
        for (int64_t v = 0; v < ube; v++) {
          const int32_t* rb = H.col + H.nptr[v];
          int32_t j = H.dlo[v];
          const int32_t e = H.dr[v];
          if (e - j > 16) j = (int32_t)(std::lower_bound(rb + j, rb + e, (int32_t)ua) - rb);
          for (; j < e; j++) {
            const int32_t u = rb[j];
            if (u >= ube) break;
            if (u < ua) continue;
            ulen[lptr[u] + cur[u - ua]++] = j + 1;
          }
        }
      }
    });
  }
  int64_t next(int64_t lo, size_t cap, std::vector<RowPart>& rows, size_t& bytes) {
    stamp++;
    rows.clear();
    std::vector<int32_t> members;
    bytes = 512;
    int64_t hi = lo;
    while (hi < H.n) {
      const int64_t u = hi;
      const int64_t ub = H.nptr[u];
      const int32_t dl = H.dlo[u];
      const int32_t* lu = ulen.data() + lptr[u];
      // a held row v in L(u) gains the entry u when the end moves past u; a
      // new one is stored up to and including u; u's own lower part joins
      // (its later entries come as the end moves on)
      size_t add = (size_t)dl * 4 + 32 + (size_t)dl * 16 + 4;
      constexpr int kAhead = 16;  // held[] is far larger than the caches
      for (int32_t j = 0; j < dl; j++) {
        if (j + kAhead < dl) __builtin_prefetch(&held[H.col[ub + j + kAhead]]);
        const Held& h = held[H.col[ub + j]];
        add += h.stamp == stamp ? 4 : (size_t)lu[j] * 4 + 32;
      }
      if (bytes + add > cap && hi > lo) break;
      bytes += add;
      for (int32_t j = 0; j < dl; j++) {
        const int32_t v = H.col[ub + j];
        Held& h = held[v];
        if (h.stamp == stamp) {
          h.len++;
        } else {
          h.stamp = stamp;
          h.len = lu[j];
          members.push_back(v);
        }
      }
      held[u] = Held{stamp, dl};
      members.push_back((int32_t)u);
      hi++;
    }
    for (int32_t v : members) rows.push_back({v, 0, held[v].len});
    return hi;
  }
};

}  // namespace

struct PartState {
  HostCsr H;
  Pinned stage[2];
  std::vector<int64_t> pairs;
  std::vector<int32_t> lens;
};

size_t resident_bytes(int64_t n, int64_t nnz, int num_cu) {
  return prep_bytes(n, nnz) + stage_tmp_bytes(n, nnz, 1, num_cu) + (size_t)(n + 1) * 8 +
         (size_t)nnz * 4 + (size_t)nnz * 8;
}

bool needs_partition(m4_ctx* c, const m4_csr* g, const m4_opts* o) {
  if (!o) return false;
  if (o->flags & M4_FORCE_PARTITION) return true;
  return o->device_budget_bytes > 0 &&
         resident_bytes(g->n, g->nnz, c->num_cu) > o->device_budget_bytes;
}

void destroy_ctx_extras(m4_ctx* c) {
  destroy_batch_state(c);
  delete c->part;
  c->part = nullptr;
}

namespace {

// Device arena carved from c->extra, never larger than the budget.
struct Dev {
  char* base;
  size_t cap, used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t b = al(count * sizeof(T) + 8);
    if (used + b > cap) throw Fail(M4_ENOMEM, "device budget too small for this partition");
    T* p = reinterpret_cast<T*>(base + used);
    used += b;
    return p;
  }
};

}  // namespace

int count_partitioned(m4_ctx* c, const m4_csr* g, const m4_opts* o, uint64_t out[6],
                      m4_stats* st) {
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : c->stream;
  const uint32_t flags = o ? o->flags : 0;
  Tuning tu = tuning_for(c, o);
  // the binned 4-cycle owners need scratch a partition's budget cannot spare
  tu.c4_bin_win = 0;
  const int64_t n = g->n, nnz = g->nnz, m = nnz / 2;
  uint64_t budget = o ? o->device_budget_bytes : 0;
  if (budget == 0) budget = resident_bytes(n, nnz, c->num_cu) / 3 + (1 << 20);
  const double t_start = now_ms();
  double t_h2d = 0, t_host = 0, t_phase[4] = {0, 0, 0, 0};
  uint64_t h2d_bytes = 0, halo_rows = 0, parts = 0;

  if (!c->part) c->part = new PartState();
  PartState& PS = *c->part;
  HostCsr& H = PS.H;
  H.n = n;
  H.nnz = nnz;
  H.m = m;

  // host copy of the input when it lives on the device
  std::vector<int64_t> hrp;
  std::vector<int32_t> hcol;
  const int64_t* rp = g->row_ptr;
  const int32_t* col = g->col;
  if (g->on_device) {
    hrp.resize(n + 1);
    hcol.resize(nnz);
    M4_HIP(hipMemcpyAsync(hrp.data(), g->row_ptr, (n + 1) * 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipMemcpyAsync(hcol.data(), g->col, nnz * 4, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    rp = hrp.data();
    col = hcol.data();
  }
  if (rp[n] != nnz) return set_error(c, M4_ERANGE, "row_ptr[n] != nnz");

  // The device side of the whole call lives in c->extra.  Workspaces of
  // earlier resident calls are freed first, and the region is allocated at
  // exactly the budget less a reserve for the context's result block and the
  // allocator's rounding, so the context never holds more than the budget.
  c->release_resident();
  constexpr uint64_t kReserve = 16 << 10;  // the result block and rounding
  if (budget <= 4 * kReserve) return set_error(c, M4_ENOMEM, "device budget below 64 KiB");
  const uint64_t region = (budget - kReserve) & ~uint64_t(255);
  c->extra.ensure(region, s, true);
  Dev D{c->extra.ptr, region};
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    const double t0 = now_ms();
    M4_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    M4_HIP(hipStreamSynchronize(s));
    t_h2d += now_ms() - t0;
    h2d_bytes += bytes;
  };
  auto down = [&](void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    M4_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
  };

  fill_u32(c->scal, 0, sizeof(Scal) / 4, s);

  // ---- 1. degree order on the device (n-sized arrays)
  Classes C{};
  {
    D.used = 0;
    int64_t* drp = D.take<int64_t>(n + 1);
    Prep P0;
    P0.perm = D.take<int32_t>(n + 1);
    P0.rank = D.take<int32_t>(n + 1);
    P0.dr = D.take<int32_t>(n + 1);
    P0.nptr = D.take<int64_t>(n + 1);
    Arena a;
    a.base = c->extra.ptr + D.used;
    a.cap = D.cap - D.used;
    if (a.cap < build_tmp_bytes(n, nnz)) throw Fail(M4_ENOMEM, "device budget below the degree sort");
    up(drp, rp, (n + 1) * 8);
    degree_order(drp, nullptr, n, nnz, false, P0, C, c->scal, c->scal_host, a, s);
    H.perm.resize(n);
    H.rank.resize(n);
    H.dr.resize(n);
    H.nptr.resize(n + 1);
    down(H.perm.data(), P0.perm, n * 4);
    down(H.rank.data(), P0.rank, n * 4);
    down(H.dr.data(), P0.dr, n * 4);
    down(H.nptr.data(), P0.nptr, (n + 1) * 8);
  }
  H.dlo.assign(n, 0);
  H.dplus.assign(n, 0);
  H.ncol.ensure((size_t)nnz * 4 + 4);

  // ---- 2. rank-space rows, streamed in chunks through the row-sort kernels
  {
    D.used = 0;
    int32_t* drank = D.take<int32_t>(n + 1);
    up(drank, H.rank.data(), n * 4);
    const size_t fixed = D.used + 64 * 1024;
    // per row 8 (rp) + 4 (perm) + 8 (nptr) + 12 (dr, dlo, dplus), per entry 8
    const size_t avail = D.cap > fixed ? D.cap - fixed : 0;
    int64_t dmax = C.dmax;
    if ((size_t)dmax * 8 + 64 * 64 > avail) throw Fail(M4_ENOMEM, "device budget below one row");
    const size_t base_used = D.used;
    int64_t r0 = 0;
    while (r0 < n) {
      // rows [r0, r1): entries * 8 + rows * 40 within the free budget
      int64_t r1 = r0, ent = 0;
      while (r1 < n) {
        const int64_t d = H.dr[r1];
        if ((size_t)(ent + d) * 8 + (size_t)(r1 - r0 + 1) * 48 + 8 * 256 > avail) break;
        ent += d;
        r1++;
      }
      if (r1 == r0) throw Fail(M4_ENOMEM, "device budget below one row");
      const int64_t R = r1 - r0;
      D.used = base_used;
      int64_t* crp = D.take<int64_t>(R + 1);
      int32_t* cperm = D.take<int32_t>(R);
      int64_t* cnptr = D.take<int64_t>(R + 1);
      int32_t* cdr = D.take<int32_t>(R);
      int32_t* cdlo = D.take<int32_t>(R);
      int32_t* cdplus = D.take<int32_t>(R);
      int32_t* ccol = D.take<int32_t>(ent + 1);
      int32_t* cout = D.take<int32_t>(ent + 1);
      // host staging: input rows of perm[r0..r1) in rank order
      Pinned& S = PS.stage[0];
      const size_t sb = al((R + 1) * 8) + al(R * 4) + al((R + 1) * 8) + al(R * 4) + al(ent * 4 + 4);
      S.ensure(sb);
      int64_t* hrp2 = reinterpret_cast<int64_t*>(S.p);
      int32_t* hperm = reinterpret_cast<int32_t*>(S.p + al((R + 1) * 8));
      int64_t* hnptr = reinterpret_cast<int64_t*>(S.p + al((R + 1) * 8) + al(R * 4));
      int32_t* hdr = reinterpret_cast<int32_t*>(S.p + 2 * al((R + 1) * 8) + al(R * 4));
      int32_t* hcc = reinterpret_cast<int32_t*>(S.p + 2 * al((R + 1) * 8) + 2 * al(R * 4));
      hrp2[0] = 0;
      for (int64_t i = 0; i < R; i++) {
        const int32_t v = H.perm[r0 + i];
        hrp2[i + 1] = hrp2[i] + (rp[v + 1] - rp[v]);
      }
      const double tg = now_ms();
      parallel_for(R, host_threads(), [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; i++) {
          const int32_t v = H.perm[r0 + i];
          const int64_t d = hrp2[i + 1] - hrp2[i];
          memcpy(hcc + hrp2[i], col + rp[v], d * 4);
          hperm[i] = (int32_t)i;
          hnptr[i] = hrp2[i];
          hdr[i] = (int32_t)d;
        }
      });
      t_host += now_ms() - tg;
      hnptr[R] = hrp2[R];
      up(crp, hrp2, (R + 1) * 8);
      up(cperm, hperm, R * 4);
      up(cnptr, hnptr, (R + 1) * 8);
      up(cdr, hdr, R * 4);
      up(ccol, hcc, ent * 4);
      sort_rows(crp, ccol, cperm, drank, cnptr, cdr, n, r0, r1, C.bound, cout, cdlo, cdplus, r0, s);
      down(H.ncol.p + H.nptr[r0] * 4, cout, ent * 4);
      down(H.dlo.data() + r0, cdlo, R * 4);
      down(H.dplus.data() + r0, cdplus, R * 4);
      r0 = r1;
    }
  }
  H.optr.assign(n + 1, 0);
  {
    // oriented offsets: device scan of the out-degrees
    D.used = 0;
    int32_t* ddp = D.take<int32_t>(n + 1);
    int64_t* dop = D.take<int64_t>(n + 2);
    int64_t* stmp = D.take<int64_t>(scan_tmp_elems(n));
    up(ddp, H.dplus.data(), n * 4);
    scan_i32(ddp, n, dop, stmp, s);
    down(H.optr.data(), dop, (n + 1) * 8);
  }

  // ---- fixed device arrays of the anchor phases
  D.used = 0;
  Prep P;
  P.n = n;
  P.nnz = nnz;
  P.m = m;
  P.nptr = D.take<int64_t>(n + 1);  // per-partition offsets into the row buffer
  P.optr = D.take<int64_t>(n + 1);
  P.dlo = D.take<int32_t>(n + 1);
  P.dplus = D.take<int32_t>(n + 1);
  P.dr = D.take<int32_t>(n + 1);
  P.t = D.take<uint32_t>(m + 1);
  int32_t* rowlen = D.take<int32_t>(n + 1);
  up(P.optr, H.optr.data(), (n + 1) * 8);
  up(P.dlo, H.dlo.data(), n * 4);
  up(P.dplus, H.dplus.data(), n * 4);
  up(P.dr, H.dr.data(), n * 4);
  fill_u32(P.t, 0, (size_t)m, s);
  const size_t fixed_used = D.used;
  const size_t tri_tmp = 2 * al(n * 4 + 4) + al(radix_tmp_elems(n, 4) * 8) + 4096;
  const size_t c4_tmp = c4_tmp_bytes(n, false);
  // scratch that a kernel stage sizes at run time comes from the tail of the
  // budget region, after the stage's work arrays
  size_t scratch_floor = 0;
  auto big = [&D, &scratch_floor](size_t bytes) -> char* {
    const size_t b = al(bytes);
    if (scratch_floor + b > D.cap) return nullptr;
    return D.base + (D.cap - b);
  };
  const int nthreads = host_threads();
  const int32_t* hc = H.col();

  // Uploads rows of a partition: (row, first stored entry, count) triples.
  std::vector<RowPart> rows;
  HostRows HR;
  HR.n = n;
  HR.nptr = H.nptr.data();
  HR.col = hc;
  HR.dr = H.dr.data();
  HR.dlo = H.dlo.data();
  HR.dplus = H.dplus.data();
  // A range's rows gathered into a pinned buffer: (row, offset) pairs, stored
  // prefix lengths, then the entries.
  struct Staged {
    int64_t lo = 0, hi = 0, nrows = 0, ent = 0;
    int err = M4_OK;
    std::string msg;
  };
  auto gather_rows = [&](const std::vector<RowPart>& rr, Pinned& S, Staged& st) {
    int64_t ent = 0;
    for (const RowPart& r : rr) ent += r.len;
    const size_t nr = rr.size();
    S.ensure(al((2 * nr + 2) * 8) + al((nr + 1) * 4) + al(ent * 4 + 4));
    int64_t* hp = reinterpret_cast<int64_t*>(S.p);
    int32_t* hl = reinterpret_cast<int32_t*>(S.p + al((2 * nr + 2) * 8));
    int32_t* hcc = reinterpret_cast<int32_t*>(S.p + al((2 * nr + 2) * 8) + al((nr + 1) * 4));
    // row offsets in the buffer, then the copies on all host threads
    int64_t off = 0;
    for (size_t i = 0; i < nr; i++) {
      hp[2 * i + 1] = off;
      off += rr[i].len;
    }
    parallel_for((int64_t)nr, nthreads, [&](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; i++) {
        const RowPart& r = rr[i];
        const int64_t o = hp[2 * i + 1];
        memcpy(hcc + o, hc + H.nptr[r.v] + r.first, (size_t)r.len * 4);
        hp[2 * i] = r.v;
        hp[2 * i + 1] = o - r.first;  // so that nptr[v] + index-in-row addresses the buffer
        hl[i] = (int32_t)(r.first + r.len);  // stored prefix length (when the row starts at 0)
      }
    });
    st.nrows = (int64_t)nr;
    st.ent = ent;
  };
  auto upload_staged = [&](const Staged& st, const Pinned& S, bool with_len) -> int32_t* {
    const size_t nr = (size_t)st.nrows;
    D.used = fixed_used;
    int64_t* dpairs = D.take<int64_t>(2 * nr + 2);
    int32_t* dlens = D.take<int32_t>(nr + 1);
    int32_t* dcol = D.take<int32_t>(st.ent + NCOL_PAD);
    up(dpairs, S.p, nr * 16);
    up(dlens, S.p + al((2 * nr + 2) * 8), nr * 4);
    up(dcol, S.p + al((2 * nr + 2) * 8) + al((nr + 1) * 4), (size_t)st.ent * 4);
    k_scatter_rows<<<(unsigned)ceil_div((int64_t)nr + 1, 256), 256, 0, s>>>(
        dpairs, (int64_t)nr, P.nptr, with_len ? rowlen : nullptr, dlens);
    halo_rows += nr;
    parts++;
    return dcol;
  };
  auto upload_rows = [&](bool with_len, int64_t) -> int32_t* {
    Staged st;
    Pinned& S = PS.stage[parts & 1];
    const double tg = now_ms();
    gather_rows(rows, S, st);
    t_host += now_ms() - tg;
    return upload_staged(st, S, with_len);
  };
  // Owner ranges from `next` (lo -> hi, filling its row list, throwing Fail
  // on a budget error) counted by `count` (lo, hi) after their rows are on
  // the device.  A host thread plans and gathers range k + 1 into the other
  // pinned buffer while the device counts range k.
  auto run_ranges = [&](int64_t start, bool with_len,
                        const std::function<int64_t(int64_t, std::vector<RowPart>&)>& next,
                        const std::function<void(int64_t, int64_t, int32_t*)>& count) {
    if (start >= n) return;
    std::mutex mu;
    std::condition_variable cv;
    Staged slot[2];
    bool ready[2] = {false, false}, done = false;
    double host_ms = 0;
    std::thread producer([&] {
      (void)hipSetDevice(c->device);
      std::vector<RowPart> rr;
      int64_t lo = start;
      for (int k = 0;; k++) {
        const int b = k & 1;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return !ready[b] || done; });
          if (done) return;
        }
        Staged st;
        const double t0 = now_ms();
        try {
          st.lo = lo;
          st.hi = lo < n ? next(lo, rr) : n;
          if (lo < n) gather_rows(rr, PS.stage[b], st);
        } catch (const Fail& f) {
          st.err = f.code;
          st.msg = f.msg;
        } catch (const std::exception& e) {
          st.err = M4_ENOMEM;
          st.msg = e.what();
        }
        const double t1 = now_ms();
        std::lock_guard<std::mutex> lk(mu);
        host_ms += t1 - t0;
        slot[b] = st;
        ready[b] = true;
        cv.notify_all();
        if (st.err != M4_OK || lo >= n) return;
        lo = st.hi;
      }
    });
    auto stop = [&] {
      {
        std::lock_guard<std::mutex> lk(mu);
        done = true;
      }
      cv.notify_all();
      producer.join();
    };
    try {
      for (int k = 0;; k++) {
        const int b = k & 1;
        Staged st;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return ready[b]; });
          st = slot[b];
        }
        if (st.err != M4_OK) throw Fail(st.err, st.msg);
        if (st.lo >= n) break;
        int32_t* dcol = upload_staged(st, PS.stage[b], with_len);  // synchronous copies
        {
          std::lock_guard<std::mutex> lk(mu);
          ready[b] = false;
        }
        cv.notify_all();
        count(st.lo, st.hi, dcol);
      }
    } catch (...) {
      stop();
      t_host += host_ms;
      throw;
    }
    stop();
    t_host += host_ms;
  };
  auto tmp_arena = [&](size_t need) {
    Arena a;
    a.base = c->extra.ptr + D.used;
    a.cap = need;
    if (D.used + need > D.cap)
      throw Fail(M4_ENOMEM, "device budget too small for a partition's work arrays");
    scratch_floor = D.used + need;
    return a;
  };

  t_phase[0] = now_ms() - t_start;
  double t_mark = now_ms();
  // ---- 3. triangle / 4-clique anchors over owner ranges with oriented halos
  {
    const size_t cap_rows = D.cap > fixed_used + tri_tmp ? D.cap - fixed_used - tri_tmp : 0;
    TriPlanner plan(HR);
    run_ranges(
        0, false,
        [&](int64_t lo, std::vector<RowPart>& rr) {
          size_t bytes = 0;
          const int64_t hi = plan.next(lo, cap_rows, rr, bytes);
          if (bytes > cap_rows) throw Fail(M4_ENOMEM, "device budget below one owner's halo");
          return hi;
        },
        [&](int64_t lo, int64_t hi, int32_t* dcol) {
          P.ncol = dcol;
          P.own_lo = lo;
          P.own_hi = hi;
          Arena a = tmp_arena(tri_tmp);
          tri_run(P, c->scal, tu, flags, o ? o->cache_rows : 0, a, s, c->num_cu, big, nullptr);
          M4_HIP(hipStreamSynchronize(s));
        });
  }

  t_phase[1] = now_ms() - t_mark;
  t_mark = now_ms();
  // ---- 4. 4-cycle anchor over owner ranges with lower halos cut below hi
  // (owners below r1 have degree <= 1 and no 4-cycle)
  {
    const size_t cap_rows = D.cap > fixed_used + c4_tmp ? D.cap - fixed_used - c4_tmp : 0;
    const double tq = now_ms();
    C4Planner plan(HR, C.r1, nthreads);
    t_host += now_ms() - tq;
    run_ranges(
        C.r1, true,
        [&](int64_t lo, std::vector<RowPart>& rr) {
          size_t bytes = 0;
          const int64_t hi = plan.next(lo, cap_rows, rr, bytes);
          if (bytes > cap_rows) throw Fail(M4_ENOMEM, "device budget below one owner's halo");
          return hi;
        },
        [&](int64_t lo, int64_t hi, int32_t* dcol) {
          P.ncol = dcol;
          P.row_len = rowlen;
          P.own_lo = lo;
          P.own_hi = hi;
          Arena a = tmp_arena(c4_tmp);
          c4_run(P, C, c->scal, tu, flags, a, s, c->num_cu, nullptr, big);
          M4_HIP(hipStreamSynchronize(s));
          P.row_len = nullptr;
        });
  }

  t_phase[2] = now_ms() - t_mark;
  t_mark = now_ms();
  // ---- 5. closure over owner ranges (out-lists only), then the inverse
  {
    const size_t cap_rows = D.cap > fixed_used + 4096 ? D.cap - fixed_used - 4096 : 0;
    int64_t lo = 0;
    while (lo < n) {
      rows.clear();
      size_t bytes = 0;
      int64_t hi = lo;
      const double tp = now_ms();
      while (hi < n) {
        const size_t add = (size_t)H.dplus[hi] * 4 + 28;
        if (bytes + add > cap_rows && hi > lo) break;
        bytes += add;
        rows.push_back({(int32_t)hi, (int64_t)H.dlo[hi], H.dplus[hi]});
        hi++;
      }
      t_host += now_ms() - tp;
      P.ncol = upload_rows(false, 1);
      P.own_lo = lo;
      P.own_hi = hi;
      closure_run(P, c->scal, flags, s);
      M4_HIP(hipStreamSynchronize(s));
      lo = hi;
    }
  }
  finalize_run(c->scal, s);
  M4_HIP(hipMemcpyAsync(c->scal_host, c->scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  t_phase[3] = now_ms() - t_mark;
  const Scal& h = *c->scal_host;
  if (h.err) return scal_error(c, h.err);
  if (h.status == 3) return set_error(c, M4_EOVERFLOW, "a count is >= 2^64");
  if (h.status != 0) return set_error(c, M4_EINTERNAL, "closure consistency check failed");
  for (int i = 0; i < 6; i++) out[i] = h.out[i];
  if (st) {
    for (int i = 0; i < 8; i++) st->basis[i] = h.basis[i];
    st->intersect_steps = h.stat[ST_STEPS];
    st->wedges = h.stat[ST_WEDGES];
    st->cache_lookups = h.stat[ST_LOOKUPS];
    st->cache_hits = h.stat[ST_HITS];
    st->partitions = parts;
    st->h2d_bytes = h2d_bytes;
    st->halo_rows = halo_rows;
    st->ms_total = now_ms() - t_start;
    st->ms_h2d = t_h2d;
    st->ms_build = t_phase[0];
    st->ms_tri = t_phase[1];
    st->ms_c4 = t_phase[2];
    st->ms_closure = t_phase[3];
    st->ms_host = t_host;
    st->device_bytes = c->held_bytes();
    st->basis_used = 0;  // halo partitions hold 1-hop rows: the wedge basis
    st->cost_wedge = st->cost_edge = 0;
  }
  return M4_OK;
}

}  // namespace m4

extern "C" int m4_plan_partitions(int kind, int64_t n, const int64_t* nptr, const int32_t* col,
                                  const int32_t* dlo, const int32_t* dplus, int64_t r1,
                                  uint64_t cap_bytes, int64_t max_ranges, int64_t max_rows,
                                  int64_t* range_end, int64_t* range_rows, int32_t* rows_v,
                                  int64_t* rows_first, int32_t* rows_len, int64_t* nranges) {
  using namespace m4;
  if ((kind != 0 && kind != 1) || n < 0 || !nranges || (n > 0 && (!nptr || !col || !dlo || !dplus)))
    return M4_EINVAL;
  if (kind == 1 && (r1 < 0 || r1 > n)) return M4_EINVAL;
  try {
    std::vector<int32_t> dr(n);
    for (int64_t v = 0; v < n; v++) dr[v] = (int32_t)(nptr[v + 1] - nptr[v]);
    HostRows H;
    H.n = n;
    H.nptr = nptr;
    H.col = col;
    H.dr = dr.data();
    H.dlo = dlo;
    H.dplus = dplus;
    std::vector<RowPart> rows;
    int64_t k = 0, nr = 0;
    auto emit = [&](int64_t hi, size_t bytes) -> int {
      if (bytes > cap_bytes) return M4_ENOMEM;
      if (k >= max_ranges || nr + (int64_t)rows.size() > max_rows) return M4_ERANGE;
      range_end[k] = hi;
      for (const RowPart& r : rows) {
        rows_v[nr] = r.v;
        rows_first[nr] = r.first;
        rows_len[nr] = r.len;
        nr++;
      }
      range_rows[k] = nr;
      k++;
      return M4_OK;
    };
    int rc = M4_OK;
    if (kind == 0) {
      TriPlanner plan(H);
      for (int64_t lo = 0; lo < n && rc == M4_OK;) {
        size_t bytes = 0;
        const int64_t hi = plan.next(lo, cap_bytes, rows, bytes);
        rc = emit(hi, bytes);
        lo = hi;
      }
    } else {
      C4Planner plan(H, r1, host_threads());
      for (int64_t lo = r1; lo < n && rc == M4_OK;) {
        size_t bytes = 0;
        const int64_t hi = plan.next(lo, cap_bytes, rows, bytes);
        rc = emit(hi, bytes);
        lo = hi;
      }
    }
    *nranges = k;
    return rc;
  } catch (const std::bad_alloc&) {
    return M4_ENOMEM;
  }
}

