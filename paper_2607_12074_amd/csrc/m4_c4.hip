// m4_c4.hip -- non-induced 4-cycle anchor (C4_ni).
//
// A 4-cycle is counted once, at its highest-ranked vertex u with opposite
// corner w: for every w < u let c_u[w] be the number of common neighbours v
// of u and w with v < u; each pair of them closes one cycle u-v-w-v', so
//   C4_ni = sum_u sum_w C(c_u[w], 2)
// (degree-ordered wedges, Chiba and Nishizeki 1985).  This is the cycle term
// of the paper's edge closure (Section III-F, adjacent pairs of A_e x B_e),
// reached through wedges instead of edge anchors.  The wedge endpoints of u
// are the prefixes below u of the sorted rows of its lower neighbours.  The
// sum is accumulated incrementally: every increment of c_u[w] adds the old
// value, so no second pass over the counters is needed.
//
// Vertices of degree <= 1 have rank < r1 and never contribute (c <= 1), so
// endpoints below r1 are skipped.  Owners are split by the wedge bound
// W_u = sum_{v in L(u)} (d(v) - 1):
//   hash bucket   -- small W_u: 256 threads, 4096-slot open-addressing
//                    table in LDS;
//   medium bucket -- W_u up to 3/4 of 16384: 1024 threads, 16384-slot table;
//   window bucket -- large W_u: one 1024-thread workgroup, dense counters in
//                    LDS over windows of 128 KiB; a counter is 4 bits wide
//                    for endpoints of degree <= 15, 8 bits for degree <= 255
//                    and 32 bits beyond (c_u[w] never exceeds d(w)), so a
//                    window spans up to 262144 ranks; every lower neighbour
//                    keeps a cursor into its sorted row so each window reads
//                    exactly its own endpoints.
// A table costs per wedge; a window costs per rank of the owner's range, so
// owners whose endpoints are sparse over many windows belong in a table.
#include <limits.h>

#include <algorithm>
#include <array>
#include <type_traits>

#include "m4_device.h"

namespace m4 {

namespace {

struct C4Args {
  const int32_t* order;
  const int64_t* start;
  const int64_t* nptr;
  const int32_t* ncol;
  const int32_t* dr;
  const int32_t* dlo;
  const int64_t* wub;
  const int32_t* row_len;  // stored prefix of every row (null: full rows)
  int64_t r1;
  int bucket;
  int slot;
  unsigned int* work;
  Scal* scal;
  uint32_t flags;
  const int64_t* seg_off;  // window and binned owners: first descriptor of each owner
  int4* desc;              // ... per-segment cursor descriptors
  const int64_t* seg_pre;  // ... exclusive prefix of segment lengths within the owner
  const int32_t* seg_cnt;  // ... non-empty segments of each owner
  int32_t* bins;           // binned owners: per-block scratch of bin_cap endpoints
  int64_t bin_cap;
  // counter zones of the window owners (ranks >= r1): 4-bit counters for
  // ranks [r1, z1) (degree <= 15), 8-bit for [z1, z2) (degree <= 255), 32-bit
  // from z2 on; aw and bw are the words of the first two zones
  int32_t z1, z2, aw, bw, zr1;  // zr1: r1 as a 32-bit rank
};

// first ranks with degree > 15 and > 255 (degrees are sorted by rank)
__global__ void k_zone_bounds(const int32_t* __restrict__ dr, int64_t n, int64_t* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= 2) return;
  const int thr = i == 0 ? 15 : 255;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (dr[mid] <= thr) lo = mid + 1;
    else hi = mid;
  }
  out[i] = lo;
}

// Multi-pass medium owners (wedge bound above 3/4 of the table) are counted
// over rank ranges cut from a histogram with bins of 2^hs ranks, 2^hs <=
// C4_MED_BIN_MAX, so one bin never holds more distinct endpoints than a pass
// may insert; their rank span must fit C4_MED_SLOTS such bins.  A wedge
// bound of at most C4_MED_MAX needs at most 12 ranges.
constexpr int C4_MED_BIN_MAX = 8192;
constexpr int C4_MED_RANGES = 32;
constexpr int64_t C4_MED_SPAN = (int64_t)C4_MED_SLOTS * C4_MED_BIN_MAX;
constexpr int64_t C4_MED_CAP = 3 * C4_MED_SLOTS / 4;
// most counter windows of a binned owner (its per-bucket histogram, over
// buckets 16 times finer, is in LDS)
constexpr int C4_BIN_KMAX = 248;

// Windows of dense counters owner u needs over ranks [r1, u); zb holds the
// first ranks of degree > 15 and > 255 (the zone bounds).
__device__ __forceinline__ int64_t c4_windows(const int64_t* zb, int64_t r1, int64_t u) {
  const int64_t z1 = zb[0] > r1 ? zb[0] : r1, z2 = zb[1] > z1 ? zb[1] : z1;
  const int64_t aw = (z1 - r1 + 7) >> 3, bw = (z2 - z1 + 3) >> 2;
  int64_t words;
  if (u <= r1) words = 0;
  else if (u <= z1) words = (u - r1 + 7) >> 3;
  else if (u <= z2) words = aw + ((u - z1 + 3) >> 2);
  else words = aw + bw + (u - z2);
  return (words + C4_WIN_WORDS - 1) / C4_WIN_WORDS;
}

// Bucket of owner u with wedge bound w > 0.  A table pass costs about one
// read of every wedge endpoint and a window costs a pass over the owner's
// lower neighbours, so an owner above the single-pass bound goes to the
// ranged table only when its endpoints are thin over many windows:
// 16 windows >= med_win ranges (med_win 0: never).
// Beyond the one-pass table, an owner whose endpoints span at least bin_win
// windows (and at most C4_BIN_KMAX) is binned: its endpoints are sorted into
// per-window bins in device memory before counting, so a window costs only
// its own endpoints instead of a pass over every lower neighbour's cursor;
// unless they average at least bin_dense per window, where a dense window's
// fixed cost is small beside its endpoints.
struct C4Plan {
  int light_max, med_max, med_win, bin_win, bin_dense;
  const int64_t* zb;
  int64_t r1;
};
__device__ __forceinline__ uint32_t c4_bucket(const C4Plan& pl, int64_t w, int64_t u) {
  if (w <= pl.light_max) return CB_HASH;
  if (pl.med_max > 0 && w <= pl.med_max && w <= C4_MED_CAP) return CB_MED;
  const int64_t nwin = c4_windows(pl.zb, pl.r1, u);
  if (pl.bin_win > 0 && nwin >= pl.bin_win && nwin <= C4_BIN_KMAX &&
      (pl.bin_dense <= 0 || w < (int64_t)pl.bin_dense * nwin))
    return CB_BIN;
  if (pl.med_max <= 0) return CB_WIN;
  if (pl.med_win > 0 && w <= C4_MED_MAX && u - pl.r1 < C4_MED_SPAN &&
      16 * nwin >= (int64_t)pl.med_win * ((w + C4_MED_CAP - 1) / C4_MED_CAP))
    return CB_MED;
  return CB_WIN;
}

// wedge bound of every owner: G lanes cooperate on one row, 4 loads in flight
template <int G>
__global__ __launch_bounds__(256) void k_c4_plan(const int64_t* __restrict__ nptr,
                                                 const int32_t* __restrict__ ncol,
                                                 const int32_t* __restrict__ dr,
                                                 const int32_t* __restrict__ dlo, int64_t r_lo,
                                                 int64_t r_hi, int64_t r1, C4Plan pl,
                                                 int64_t* __restrict__ wub,
                                                 uint32_t* __restrict__ key, int64_t own_lo,
                                                 int64_t own_hi) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t u = r_lo + t / G;
  int j = (int)(t % G);
  bool ok = u < r_hi;
  if (ok && (u < own_lo || u >= own_hi)) {
    if (j == 0) key[u] = CB_NONE;
    ok = false;
  }
  int nl = ok ? dlo[u] : 0;
  int64_t b = ok ? nptr[u] : 0;
  int64_t s = 0;
  int i = j;
  for (; i + 3 * G < nl; i += 4 * G) {
    int32_t v0 = ncol[b + i], v1 = ncol[b + i + G], v2 = ncol[b + i + 2 * G], v3 = ncol[b + i + 3 * G];
    s += (int64_t)dr[v0] + dr[v1] + dr[v2] + dr[v3] - 4;
  }
  for (; i < nl; i += G) s += dr[ncol[b + i]] - 1;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
  if (ok && j == 0) {
    wub[u] = s;
    uint32_t k = CB_NONE;
    if (u >= r1 && nl >= 2 && s > 0) k = c4_bucket(pl, s, u);
    key[u] = k;
  }
}

// rows too long for one wavefront: one 1024-thread workgroup per row
__global__ __launch_bounds__(1024) void k_c4_plan_big(const int64_t* __restrict__ nptr,
                                                      const int32_t* __restrict__ ncol,
                                                      const int32_t* __restrict__ dr,
                                                      const int32_t* __restrict__ dlo, int64_t r_lo,
                                                      int64_t r1, C4Plan pl,
                                                      int64_t* __restrict__ wub,
                                                      uint32_t* __restrict__ key, int64_t own_lo,
                                                      int64_t own_hi) {
  int64_t u = r_lo + blockIdx.x;
  if (u < own_lo || u >= own_hi) {
    if (threadIdx.x == 0) key[u] = CB_NONE;
    return;
  }
  int nl = dlo[u];
  int64_t b = nptr[u];
  int64_t s = 0;
  for (int i = threadIdx.x; i < nl; i += 1024) s += dr[ncol[b + i]] - 1;
  int64_t tot;
  block_excl_scan64<1024>(s, &tot);
  if (threadIdx.x == 0) {
    wub[u] = tot;
    uint32_t k = CB_NONE;
    if (u >= r1 && nl >= 2 && tot > 0) k = c4_bucket(pl, tot, u);
    key[u] = k;
  }
}

// --------------------------------------------------------- hash buckets
// Streams the wedge endpoints x in [r1, u) of owner u to fn: the rows of the
// lower neighbours, NT at a time, are flattened by a scan of their lengths;
// every thread takes UNR endpoints per round with their loads in flight
// together.  Called by every thread of the workgroup.
template <int NT, int UNR, class F>
__device__ __forceinline__ void c4_endpoints(const C4Args& A, int32_t u, int nl, int64_t base,
                                             int32_t* sst, int32_t* spref,
                                             unsigned long long& reads, F&& fn) {
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < nl; c0 += NT) {
    const int nc = nl - c0 < NT ? nl - c0 : NT;
    int len = 0;
    if (tid < nc) {
      const int32_t v = A.ncol[base + c0 + tid];
      sst[tid] = (int32_t)A.nptr[v];
      len = A.row_len ? A.row_len[v] : A.dr[v];
    }
    int64_t tot;
    const int64_t ex = block_excl_scan64<NT>(len, &tot);
    if (tid < nc) spref[tid] = (int32_t)ex;
    if (tid == 0) spref[nc] = (int32_t)tot;
    __syncthreads();
    const int total = (int)tot;
    if (tid == 0) reads += (unsigned long long)total;
    for (int q0 = 0; q0 < total; q0 += NT * UNR) {
      int32_t w[UNR];
#pragma unroll
      for (int j = 0; j < UNR; j++) {
        const int q = q0 + j * NT + tid;
        w[j] = INT_MAX;
        if (q < total) {
          const int si = upper_index(spref, nc, q);
          w[j] = A.ncol[sst[si] + (q - spref[si])];
        }
      }
#pragma unroll
      for (int j = 0; j < UNR; j++)
        if (w[j] >= A.r1 && w[j] < u) fn(w[j]);
    }
    __syncthreads();
  }
}

// One owner at a time per workgroup, counting in an open-addressing table in
// LDS (linear probing, keys inserted with compare-and-swap).  The table is
// sized to a power of two of at least twice the wedge bound, capped at
// SLOTS; the number of distinct endpoints never exceeds the wedge bound, so
// while that bound is at most 3/4 of SLOTS a probe always ends.  Owners of
// the medium bucket with a larger bound (1024 threads only) are counted in
// rank ranges: a first pass histograms their endpoints over bins of ranks,
// the bins are cut greedily into ranges of at most 3/4 SLOTS endpoints (or
// one bin, which holds at most C4_MED_BIN_MAX distinct ranks), and every
// range is one pass over the rows that inserts only its own endpoints.  Each
// endpoint lies in exactly one range, so every c_u[w] is complete in its
// pass.
template <int NT, int SLOTS, int UNR>
__global__ __launch_bounds__(NT) void k_c4_hash(C4Args A) {
  __shared__ int32_t hkey[SLOTS];
  __shared__ uint32_t hcnt[SLOTS];
  __shared__ int32_t sst[NT];
  __shared__ int32_t spref[NT + 1];
  __shared__ int32_t s_rng[C4_MED_RANGES + 1];
  __shared__ int s_item, s_nr;
  __shared__ uint32_t s_tot;
  constexpr uint32_t CAP = 3 * SLOTS / 4;
  const int tid = threadIdx.x;
  const int64_t b0 = A.start[A.bucket], cnt = A.start[A.bucket + 1] - b0;
  u128_t acc = 0;
  unsigned long long wedges = 0, owners = 0, segs = 0, reads = 0;
  for (int i = tid; i < SLOTS; i += NT) {
    hkey[i] = -1;
    hcnt[i] = 0;
  }
  const int GRAB = NT >= 1024 ? 1 : 8;
  int64_t item = 0, last = 0;
  for (;;) {
    if (item == last) {
      if (tid == 0) s_item = (int)atomicAdd(A.work, (unsigned)GRAB);
      __syncthreads();
      item = s_item;
      __syncthreads();
      if (item >= cnt) break;
      last = item + GRAB < cnt ? item + GRAB : cnt;
    }
    const int32_t u = A.order[b0 + item];
    item++;
    const int nl = A.dlo[u];
    const int64_t base = A.nptr[u];
    const int64_t wb = A.wub[u];
    int S = 64;
    while (S < 2 * wb && S < SLOTS) S <<= 1;
    const uint32_t mask = (uint32_t)S - 1;
    const int shift = 32 - __ffs(S) + 1;
    if (tid == 0) {
      owners++;
      segs += (unsigned long long)nl;
    }
    // at most 3/4 S distinct keys: every probe meets x or a free slot within
    // S steps (a longer one means a broken bound and is reported, not spun)
    auto insert = [&](int32_t x) {
      uint32_t h = ((uint32_t)x * 0x9E3779B1u) >> shift;
      bool ok = false;
      for (int probes = 0; probes < S; probes++) {
        const int32_t k = hkey[h];
        if (k == x) {
          ok = true;
          break;
        }
        if (k == -1) {
          const int32_t prev = atomicCAS(&hkey[h], -1, x);
          if (prev == -1 || prev == x) {
            ok = true;
            break;
          }
        }
        h = (h + 1) & mask;
      }
      if (!ok) {
        atomicOr(&A.scal->err, ERR_PROBE);
        return;
      }
      acc += atomicAdd(&hcnt[h], 1u);
      wedges++;
    };
    if (NT < 1024 || wb <= (int64_t)CAP) {
      c4_endpoints<NT, UNR>(A, u, nl, base, sst, spref, reads, insert);
    } else {
      // histogram of the endpoints over bins of 2^hs ranks (in hcnt)
      const int32_t span = u - (int32_t)A.r1;
      int hs = 0;
      while ((span >> hs) >= SLOTS) hs++;
      c4_endpoints<NT, UNR>(A, u, nl, base, sst, spref, reads, [&](int32_t x) {
        atomicAdd(&hcnt[(x - (int32_t)A.r1) >> hs], 1u);
      });
      // exclusive prefix of the bins, in place
      constexpr int PER = SLOTS / NT;
      uint32_t loc[PER], sum = 0;
#pragma unroll
      for (int i = 0; i < PER; i++) {
        loc[i] = hcnt[tid * PER + i];
        sum += loc[i];
      }
      int64_t tot;
      uint32_t run = (uint32_t)block_excl_scan64<NT>((int64_t)sum, &tot);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < PER; i++) {
        hcnt[tid * PER + i] = run;
        run += loc[i];
      }
      if (tid == 0) s_tot = (uint32_t)tot;
      __syncthreads();
      // greedy ranges: as many bins as fit in CAP endpoints, at least one
      if (tid == 0) {
        auto pre = [&](int b) { return b >= SLOTS ? s_tot : hcnt[b]; };
        int nr = 0, lo = 0;
        s_rng[0] = (int32_t)A.r1;
        while (lo < SLOTS && nr < C4_MED_RANGES) {
          const uint32_t p0 = pre(lo);
          int l = lo + 1, h = SLOTS;  // largest b in [lo + 1, SLOTS] with pre(b) - p0 <= CAP
          if (pre(l) - p0 > CAP) {
            h = l;
          } else {
            while (l < h) {
              const int mid = (l + h + 1) >> 1;
              if (pre(mid) - p0 <= CAP) l = mid;
              else h = mid - 1;
            }
            h = l;
          }
          nr++;
          const int64_t rk = (int64_t)A.r1 + ((int64_t)h << hs);
          s_rng[nr] = h >= SLOTS || rk >= u ? u : (int32_t)rk;
          lo = h;
          if (s_rng[nr] >= u) break;
        }
        if (s_rng[nr] < u) {  // more ranges than planned for: not counted
          atomicOr(&A.scal->err, ERR_RANGES);
          nr = 0;
        }
        s_nr = nr;
      }
      __syncthreads();
      for (int i = tid; i < SLOTS; i += NT) hcnt[i] = 0;
      __syncthreads();
      const int nr = s_nr;
      for (int r = 0; r < nr; r++) {
        const int32_t lo = s_rng[r], hi = s_rng[r + 1];
        c4_endpoints<NT, UNR>(A, u, nl, base, sst, spref, reads, [&](int32_t x) {
          if (x >= lo && x < hi) insert(x);
        });
        if (r + 1 < nr) {
          for (int i = tid; i < S; i += NT) {
            hkey[i] = -1;
            hcnt[i] = 0;
          }
          __syncthreads();
        }
      }
    }
    for (int i = tid; i < S; i += NT) {
      hkey[i] = -1;
      hcnt[i] = 0;
    }
    __syncthreads();
  }
  block_add_u128<NT>(&A.scal->acc[ACC_C4], acc);
  if (A.flags & M4_STATS) {
    block_add_u64<NT>(&A.scal->stat[ST_WEDGES], wedges);
    block_add_u64<NT>(&A.scal->kstat[A.slot][0], wedges);
    block_add_u64<NT>(&A.scal->kstat[A.slot][1], owners);
    block_add_u64<NT>(&A.scal->kstat[A.slot][2], segs);
    block_add_u64<NT>(&A.scal->kstat[A.slot][3], reads);
  }
}

// -------------------------------------------------------- window bucket
// Segment descriptors of the window and binned owners: for lower neighbour v
// of owner u the cursor into row v (first entry >= r1), the segment's end
// (for a binned owner the position of u in row v: entries from there on are
// not below u; for a window owner the row's end), and the values at the
// cursor and 7 entries after it.  Only non-empty segments are
// kept (a lower neighbour of degree 1, say, has none), packed from the
// owner's first slot; seg_cnt[h] is their number and seg_pre (binned owners
// only) the exclusive prefix of their lengths.  One block per owner.
__global__ __launch_bounds__(256) void k_c4_desc(const int32_t* __restrict__ order,
                                                 const int64_t* __restrict__ start,
                                                 const int64_t* __restrict__ seg_off,
                                                 const int64_t* __restrict__ nptr,
                                                 const int32_t* __restrict__ dlo,
                                                 const int32_t* __restrict__ ncol,
                                                 const int4* __restrict__ vmeta,
                                                 const int32_t* __restrict__ row_len, int64_t r1,
                                                 int4* __restrict__ desc,
                                                 int64_t* __restrict__ seg_pre,
                                                 int32_t* __restrict__ seg_cnt) {
  const int64_t h = blockIdx.x;
  const int32_t u = order[start[CB_WIN] + h];
  const int64_t so = seg_off[h], base = nptr[u];
  const int nl = dlo[u];
  // binned owners walk positions and need each segment's exact end (u's
  // place in the row); the window kernel stops at u by value, so its
  // segments may run to the row's end
  const bool exact = h >= start[CB_BIN] - start[CB_WIN];
  int64_t run = 0, kept = 0;
  for (int i0 = 0; i0 < nl; i0 += 256) {
    const int i = i0 + (int)threadIdx.x;
    int64_t len = 0, c = 0, e = 0;
    if (i < nl) {
      const int32_t v = ncol[base + i];
      if (vmeta) {
        // full rows: one 16-byte record per vertex
        const int4 m = vmeta[v];
        const int64_t rs = m.x;
        // u is an out-neighbour of v: search the out-part of row v
        e = exact ? lower_index(ncol, rs + m.z, rs + m.y, u) : rs + m.y;
        c = rs + m.w;
      } else {
        const int64_t rs = nptr[v];
        const int64_t rend = row_len ? rs + row_len[v] : nptr[v + 1];
        e = exact ? lower_index(ncol, rs + dlo[v], rend, u) : rend;
        // first entry >= r1, searched in the stored prefix
        c = lower_index(ncol, rs, e, (int32_t)r1);
      }
      if (c > e) c = e;
      len = e - c;
    }
    int64_t tot, ktot;
    const int64_t ex = block_excl_scan64<256>(len, &tot);
    const int64_t kx = block_excl_scan64<256>(len > 0 ? 1 : 0, &ktot);
    if (len > 0) {
      const int64_t at = so + kept + kx;
      desc[at] = make_int4((int)c, (int)e, ncol[c], c + 7 < e ? ncol[c + 7] : INT_MAX);
      if (seg_pre) seg_pre[at] = run + ex;
    }
    run += tot;
    kept += ktot;
  }
  if (threadIdx.x == 0) seg_cnt[h] = (int32_t)kept;
}

// per full row: {row offset, degree, lower neighbours, entries below r1
// (degree <= 1) at its head}; row offsets fit 32 bits (CSR positions do)
__global__ void k_vmeta(const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                        const int32_t* __restrict__ dr, const int32_t* __restrict__ dlo, int64_t n,
                        int64_t r1, int4* __restrict__ vmeta) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t rs = nptr[v];
  const int32_t cut = (int32_t)(lower_index(ncol, rs, nptr[v + 1], (int32_t)r1) - rs);
  vmeta[v] = make_int4((int)rs, dr[v], dlo[v], cut);
}

__global__ void k_c4_heavy_len(const int32_t* __restrict__ order, const int64_t* __restrict__ start,
                               const int32_t* __restrict__ dlo, int32_t* __restrict__ len) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = start[CB_WIN], H = start[CB_BIN + 1] - b;
  if (h < H) len[h] = dlo[order[b + h]];
}

constexpr int W_NT = 1024, W_GL = 8, W_NG = W_NT / W_GL, W_SHORT = 8;
constexpr int W_LD = 2;  // 16-byte loads per lane and step of a long visit
constexpr int W_BATCH = 2048;  // segments per pass (bounds the long-visit queue)
constexpr int W_RPT = W_BATCH / W_NT;  // segments per thread and pass

// Counter of rank x (x >= r1) in the zoned layout: a 4-bit counter while the
// degree of x is <= 15, 8-bit while <= 255, else 32-bit.  c_u[x] counts
// common neighbours of u and x, so it never exceeds the degree of x and no
// counter overflows into its neighbour.
__device__ __forceinline__ void zone_slot(const C4Args& A, int32_t x, int32_t& word, int& shift) {
  if (x < A.z1) {
    const int32_t k = x - A.zr1;
    word = k >> 3;
    shift = (k & 7) * 4;
  } else if (x < A.z2) {
    const int32_t k = x - A.z1;
    word = A.aw + (k >> 2);
    shift = (k & 3) * 8;
  } else {
    word = A.aw + A.bw + (x - A.z2);
    shift = 0;
  }
}

// first rank whose counter lies in word w
__device__ __forceinline__ int32_t zone_rank(const C4Args& A, int32_t w) {
  if (w < A.aw) return A.zr1 + 8 * w;
  if (w < A.aw + A.bw) return A.z1 + 4 * (w - A.aw);
  return A.z2 + (w - A.aw - A.bw);
}

// words holding the counters of ranks [r1, u)
__device__ __forceinline__ int32_t zone_words(const C4Args& A, int32_t u) {
  if (u <= A.zr1) return 0;
  if (u <= A.z1) return (u - A.zr1 + 7) >> 3;
  if (u <= A.z2) return A.aw + ((u - A.z1 + 3) >> 2);
  return A.aw + A.bw + (u - A.z2);
}

// one wedge endpoint x of the window starting at word wlo: returns the old
// count c (every increment of c_u[x] from c to c + 1 adds c to the sum of
// C(c_u[x], 2))
__device__ __forceinline__ uint32_t window_inc(const C4Args& A, uint32_t* cnt, int32_t wlo,
                                               int32_t x) {
  int32_t word;
  int shift;
  zone_slot(A, x, word, shift);
  const uint32_t mask = x < A.z1 ? 0xfu : (x < A.z2 ? 0xffu : 0xffffffffu);
  const uint32_t old = atomicAdd(&cnt[word - wlo], 1u << shift);
  return (old >> shift) & mask;
}

// The same increment for a window that lies inside one zone (KIND 0: 4-bit
// counters, 1: 8-bit, 2: 32-bit; 3: the window crosses a zone bound): with
// base the first rank of the window's first word, the counter word is
// (x - base) >> log2(counters per word), so the zone tests and the shifted
// zone offsets drop out of the per-endpoint work.
template <int KIND>
__device__ __forceinline__ uint32_t window_inc_k(const C4Args& A, uint32_t* cnt, int32_t wlo,
                                                 int32_t base, int32_t x) {
  if constexpr (KIND == 0) {
    const int32_t k = x - base;
    const int sh = (k & 7) << 2;
    return (atomicAdd(&cnt[k >> 3], 1u << sh) >> sh) & 0xfu;
  } else if constexpr (KIND == 1) {
    const int32_t k = x - base;
    const int sh = (k & 3) << 3;
    return (atomicAdd(&cnt[k >> 2], 1u << sh) >> sh) & 0xffu;
  } else if constexpr (KIND == 2) {
    return atomicAdd(&cnt[x - base], 1u);
  } else {
    return window_inc(A, cnt, wlo, x);
  }
}

// word holding the counter of rank x (x >= r1)
__device__ __forceinline__ int32_t zone_word(const C4Args& A, int32_t x) {
  int32_t word;
  int shift;
  zone_slot(A, x, word, shift);
  return word;
}

__device__ __forceinline__ int32_t row_at(const int32_t* ncol, int64_t i, int64_t e) {
  return i < e ? ncol[i] : INT_MAX;
}

__device__ __forceinline__ int32_t comp(const int4& v, int r) {
  return r == 0 ? v.x : (r == 1 ? v.y : (r == 2 ? v.z : v.w));
}

// A visit of at most 7 entries by one thread: entries c .. c+14 from five
// aligned 16-byte loads, the entries below hi counted, the descriptor
// advanced (the new cursor's value and the one 7 later are among them).
template <int KIND>
__device__ __forceinline__ int short_visit(const C4Args& A, const int4* __restrict__ ncol4,
                                           uint32_t* cnt, int4& d, int32_t wlo, int32_t base,
                                           int32_t hi, u128_t& acc) {
  const int64_t c = d.x, e = d.y, c4 = c & ~int64_t(3);
  const int off = (int)(c - c4);
  int4 v[5];
#pragma unroll
  for (int q = 0; q < 5; q++) v[q] = ncol4[(c4 >> 2) + q];
  int32_t x[W_SHORT + 7];
#pragma unroll
  for (int j = 0; j < W_SHORT + 7; j++) {
    int32_t val;
    switch (off) {
      default: val = comp(v[j >> 2], j & 3); break;
      case 1: val = comp(v[(j + 1) >> 2], (j + 1) & 3); break;
      case 2: val = comp(v[(j + 2) >> 2], (j + 2) & 3); break;
      case 3: val = comp(v[(j + 3) >> 2], (j + 3) & 3); break;
    }
    x[j] = c + j < e ? val : INT_MAX;
  }
  int took = 0;
  uint64_t part = 0;
#pragma unroll
  for (int j = 0; j < W_SHORT; j++)
    if (x[j] < hi) {
      part += window_inc_k<KIND>(A, cnt, wlo, base, x[j]);
      took++;
    }
  acc += part;
  int32_t z = x[0], w = x[7];
#pragma unroll
  for (int j = 1; j < W_SHORT; j++)
    if (j == took) {
      z = x[j];
      w = x[j + 7];
    }
  d = make_int4((int)(c + took), (int)e, z, w);
  return took;
}

// One heavy owner per workgroup, windows of counters in LDS in rank order.
// A segment is one lower neighbour's row; its descriptor holds the cursor
// (the first entry not yet counted), the row end, and the values at the
// cursor and 7 entries after it, so the length of its visit to a window is
// known to be 0, at most 7, or more without reading the row.  Rows are read
// with 16-byte loads aligned below the cursor (entries before the cursor lie
// below the window, entries from the row end on are masked; the array has
// slack after its last row).  Per pass over W_BATCH segments every thread
// first takes whole segments by itself (an empty visit costs nothing for
// descriptors held in registers, a short one five 16-byte loads); longer
// visits are queued in LDS and walked by 8-lane groups, 64 entries (two
// 16-byte loads per lane) per step, the next step's loads issued before a
// step is counted, and the next queued segment's first
// step in flight.  The next window starts at the smallest value any cursor
// points at, so windows without endpoints are never visited.
__global__ __launch_bounds__(W_NT) void k_c4_window(C4Args A) {
  constexpr int WORDS = C4_WIN_WORDS;
  constexpr int STEP = 4 * W_GL * W_LD;
  static_assert(STEP <= NCOL_PAD, "a step may read STEP entries past a cursor");
  __shared__ uint32_t cnt[WORDS];
  __shared__ int32_t queue[W_BATCH];
  __shared__ int s_item, s_q, s_minz;
  const int tid = threadIdx.x;
  const int g = tid / W_GL, gl = tid & (W_GL - 1);
  const int64_t b0 = A.start[A.bucket], cnt_items = A.start[A.bucket + 1] - b0;
  const int64_t hbase = b0 - A.start[CB_WIN];
  const int4* __restrict__ ncol4 = reinterpret_cast<const int4*>(A.ncol);
  const int4 kNone = make_int4(0, 0, INT_MAX, INT_MAX);
  u128_t acc = 0;
  unsigned long long wedges = 0, owners = 0, segs = 0, visits = 0;
  // counters start at zero; every window clears the words it used
  for (int i = tid; i < WORDS; i += W_NT) cnt[i] = 0;
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt_items) break;
    // heaviest owners (highest ranks) first
    const int64_t pos = cnt_items - 1 - item;
    const int32_t u = A.order[b0 + pos];
    const int64_t so = A.seg_off[hbase + pos];
    const int nl = A.seg_cnt[hbase + pos];
    int4* D = A.desc + so;
    // owners with at most W_BATCH segments keep each thread's descriptors in
    // registers from window to window
    const bool resident = nl <= W_BATCH;
    int4 rdesc[W_RPT];
    uint32_t stale = (1u << W_RPT) - 1u;
    if (tid == 0) {
      owners++;
      segs += (unsigned long long)nl;
    }
    const int32_t uwords = zone_words(A, u);
    int32_t wlo = 0;
    while (wlo < uwords) {
      // ranks past the last word of a zone map beyond the owner: hi = u
      const int32_t hnext = wlo + WORDS >= uwords ? u : zone_rank(A, wlo + WORDS);
      const int32_t hi = (int32_t)(hnext < u ? hnext : u);
      if (tid == 0) {
        visits += (unsigned long long)nl;
        s_minz = INT_MAX;
      }
      // the window's zone: one zone lets the counter index skip the zone tests
      const int32_t wr = zone_rank(A, wlo);
      const int kind = hi <= A.z1 ? 0 : (wr >= A.z1 && hi <= A.z2 ? 1 : (wr >= A.z2 ? 2 : 3));
      const int32_t base = wr;
      auto pass = [&](auto kind_tag) {
        constexpr int KIND = decltype(kind_tag)::value;
        for (int s0 = 0; s0 < nl; s0 += W_BATCH) {
          const int s1 = s0 + W_BATCH < nl ? s0 + W_BATCH : nl;
          if (tid == 0) s_q = 0;
          __syncthreads();
          // ---- whole segments per thread
          int32_t zmin = INT_MAX;
          if (resident) {
            // descriptors stay in registers across windows; one that a group
            // advances (a long visit) is stored before and reloaded after
#pragma unroll
            for (int j = 0; j < W_RPT; j++) {
              const int sg = tid + j * W_NT;
              if (sg < nl) {
                if ((stale >> j) & 1u) {
                  rdesc[j] = D[sg];
                  stale &= ~(1u << j);
                }
                if (rdesc[j].z < hi && rdesc[j].w < hi) {
                  D[sg] = rdesc[j];
                  queue[atomicAdd(&s_q, 1)] = sg;
                  stale |= 1u << j;
                } else {
                  if (rdesc[j].z < hi)
                    wedges += short_visit<KIND>(A, ncol4, cnt, rdesc[j], wlo, base, hi, acc);
                  zmin = min(zmin, rdesc[j].z);
                }
              }
            }
          } else {
            for (int sg = s0 + tid; sg < s1; sg += W_NT) {
              int4 d = D[sg];
              if (d.z < hi && d.w < hi) {  // 8 entries or more: queue it
                queue[atomicAdd(&s_q, 1)] = sg;
                continue;
              }
              if (d.z < hi) {
                wedges += short_visit<KIND>(A, ncol4, cnt, d, wlo, base, hi, acc);
                D[sg] = d;
              }
              zmin = min(zmin, d.z);
            }
          }
          if (zmin != INT_MAX) atomicMin(&s_minz, zmin);
          __syncthreads();
          // ---- queued long segments, one 8-lane group each: a step reads the
          // STEP entries [p, p + STEP); lane gl holds entries
          // 4 (W_GL k + gl) + r (k < W_LD, r < 4) of the step
          const int nq = s_q;
          int qi = g;
          int4 dA = qi < nq ? D[queue[qi]] : kNone;
          int64_t pA = (int64_t)dA.x & ~int64_t(STEP - 1);
          int4 a[W_LD];
#pragma unroll
          for (int k = 0; k < W_LD; k++)
            a[k] = qi < nq ? ncol4[(pA >> 2) + W_GL * k + gl] : make_int4(0, 0, 0, 0);
          while (qi < nq) {  // uniform in the group
            const int sg = queue[qi];
            const int qn = qi + W_NG;
            const int4 dB = qn < nq ? D[queue[qn]] : kNone;
            const int64_t pB = (int64_t)dB.x & ~int64_t(STEP - 1);
            int4 bn[W_LD];
#pragma unroll
            for (int k = 0; k < W_LD; k++)
              bn[k] = qn < nq ? ncol4[(pB >> 2) + W_GL * k + gl] : make_int4(0, 0, 0, 0);
            // positions fit 32 bits: the column array holds < 2^31 - 1024 entries
            const int32_t c0 = dA.x, e = dA.y;
            int32_t p = (int32_t)pA;
            int32_t cend = c0;  // new cursor
            for (;;) {
              // the next step's loads go out before this step's counting
              const bool more = p + STEP < e;
              int4 nx[W_LD];
#pragma unroll
              for (int k = 0; k < W_LD; k++)
                nx[k] = more ? ncol4[((p + STEP) >> 2) + W_GL * k + gl] : make_int4(0, 0, 0, 0);
              int mine = 0;
              // counts of one-zone windows of 4- or 8-bit counters sum below
              // 2^32 over a step; wider ones need 64 bits
              std::conditional_t<(KIND <= 1), uint32_t, uint64_t> part = 0;
              // the step's entries from the cursor on and before the row end,
              // as a bit mask over this lane's 4 W_LD entries
              const int lo_o = c0 > p ? c0 - p : 0;
              const int hi_o = e - p < STEP ? e - p : STEP;
              uint32_t pm = 0;
#pragma unroll
              for (int k = 0; k < W_LD; k++) {
                const int b = 4 * (W_GL * k + gl);
                const int lk = min(max(lo_o - b, 0), 4), hk = min(max(hi_o - b, 0), 4);
                pm |= ((1u << hk) - (1u << lk)) << (4 * k);  // lo_o <= hi_o, so lk <= hk
              }
#pragma unroll
              for (int k = 0; k < W_LD; k++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                  const int32_t xv = comp(a[k], r);
                  if (((pm >> (4 * k + r)) & 1u) && xv < hi) {
                    part += window_inc_k<KIND>(A, cnt, wlo, base, xv);
                    mine++;
                  }
                }
              acc += (uint64_t)part;
              wedges += (unsigned long long)mine;
              // entries in the window form a run from the cursor: its length is
              // the group's total
              int tot = mine;
#pragma unroll
              for (int o = 1; o < W_GL; o <<= 1) tot += __shfl_xor(tot, o, WAVE);
              const int32_t first = p > c0 ? p : c0;
              cend = first + tot;
              if (cend < p + STEP || !more) break;  // the run ends in this step
              p += STEP;
#pragma unroll
              for (int k = 0; k < W_LD; k++) a[k] = nx[k];
            }
            if (gl == 0) {
              const int32_t vnext = row_at(A.ncol, cend, e);
              D[sg] = make_int4((int)cend, (int)e, vnext, row_at(A.ncol, cend + 7, e));
              atomicMin(&s_minz, vnext);
            }
            qi = qn;
            dA = dB;
            pA = pB;
#pragma unroll
            for (int k = 0; k < W_LD; k++) a[k] = bn[k];
          }
          __syncthreads();
        }
      };
      switch (kind) {
        case 0: pass(std::integral_constant<int, 0>{}); break;
        case 1: pass(std::integral_constant<int, 1>{}); break;
        case 2: pass(std::integral_constant<int, 2>{}); break;
        default: pass(std::integral_constant<int, 3>{}); break;
      }
      // clear the counters; the next window starts at the word of the
      // smallest value a cursor points at
      const int32_t minz = s_minz;
      const int used = uwords - wlo < WORDS ? uwords - wlo : WORDS;
      for (int i = tid; i < used; i += W_NT) cnt[i] = 0;
      __syncthreads();
      wlo = minz >= u ? uwords : zone_word(A, minz);
    }
  }
  block_add_u128<W_NT>(&A.scal->acc[ACC_C4], acc);
  if (A.flags & M4_STATS) {
    block_add_u64<W_NT>(&A.scal->stat[ST_WEDGES], wedges);
    block_add_u64<W_NT>(&A.scal->kstat[A.slot][0], wedges);
    block_add_u64<W_NT>(&A.scal->kstat[A.slot][1], owners);
    block_add_u64<W_NT>(&A.scal->kstat[A.slot][2], segs);
    block_add_u64<W_NT>(&A.scal->kstat[A.slot][3], visits);
  }
}

// ----------------------------------------------------------- binned bucket
// One owner at a time per 512-thread workgroup (two per CU), heaviest first.
// Its wedge endpoints are the concatenation of its non-empty segments (rows
// of the lower neighbours from the first rank >= r1 up to u).  The counter
// words of the ranks [r1, u) are cut into fine buckets of BF_WORDS words.
//   pass 1: each wave walks a contiguous share of the concatenation, 64
//           endpoints a step and BF_UNROLL steps in flight, and counts the
//           endpoints per bucket in LDS (one atomic per run of lanes with
//           the same segment and bucket); a block prefix turns the counts
//           into bucket starts;
//   pass 2: the same walk scatters the endpoints into their buckets in the
//           block's device scratch (one cursor atomic per run);
//   pass 3: waves take groups of consecutive buckets, a group being the
//           buckets that start within one stretch of BF_GROUP positions of
//           the scatter, and count each in a private 8 KiB LDS region: the
//           group's small buckets in an open-addressing table of (rank,
//           count) pairs, a bucket above BF_GROUP endpoints alone in dense
//           zoned counters (it spans BF_WORDS words); every increment adds
//           the counter's old value.  Dense buckets above BF_BIG endpoints
//           are counted afterwards by the whole block.
// No barrier is taken per bucket.  The scratch holds `cap` endpoints: an
// owner with more is scattered in consecutive bucket ranges that fit, one
// pass 2 and 3 per range; a single bucket above `cap` is counted straight
// from the rows by a walk that keeps only its endpoints.
constexpr int BN_NT = 512, BN_NW = BN_NT / WAVE;
constexpr int BF_SHIFT = 11, BF_WORDS = 1 << BF_SHIFT;  // 8 KiB of counters per wave
constexpr int BF_KMAX = 3968;    // fine buckets per owner (two workgroups' LDS per CU)
constexpr int BF_GROUP = 192;    // scatter positions per group
constexpr int BF_HBITS = BF_SHIFT - 1, BF_HSLOTS = 1 << BF_HBITS;  // 64-bit slots
constexpr int BF_BIG = 4096;     // dense buckets above this: the whole block
constexpr int BF_BIGLIST = 48;
constexpr int BF_SB = 16;        // staging buffer entries per target (four 16-byte stores)
constexpr int BF_NTS = 620;      // targets with a staging buffer (20 words each)
constexpr int BF_PAD = 16;       // targets start at multiples of this many entries
static_assert((int64_t)C4_BIN_KMAX * C4_WIN_WORDS <= (int64_t)BF_KMAX * BF_WORDS,
              "a binned owner's fine buckets must fit the LDS histogram");
static_assert(2 * BF_GROUP <= BF_HSLOTS / 2, "a hash group must keep its table half empty");
static_assert(BF_KMAX + (4 + BF_SB) * BF_NTS <= BN_NW * BF_WORDS && (BF_KMAX + 4 * BF_NTS) % 4 == 0,
              "scatter cursors and staging buffers fit the counter regions, the buffers 16-byte aligned");

__device__ __forceinline__ int32_t fbin_of(const C4Args& A, int32_t x) {
  return zone_word(A, x) >> BF_SHIFT;
}

// a wave-uniform value held in scalar registers (LDS and vector loads
// return it in vector registers)
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Per-wave view of 64 consecutive segments from sbase: lane j holds the
// concatenated start of segment sbase + 1 + j (far beyond the end past the
// last segment) and, for segment sbase + j, its row index minus its
// concatenated start (so an endpoint at position q of that segment sits at
// ncol[q + delta]; both are below 2^31).
struct SegView {
  int sbase;
  int64_t B;
  int32_t delta;
};
constexpr int64_t SEG_FAR = int64_t(1) << 62;
constexpr int WALK_PER = 4;                     // positions per lane and step
constexpr int WALK_STEP = WAVE * WALK_PER;      // positions per wave and step

__device__ __forceinline__ void seg_view_load(const int4* __restrict__ D,
                                              const int64_t* __restrict__ pre, int nl, int sbase,
                                              SegView& v) {
  const int j = sbase + (int)(threadIdx.x & (WAVE - 1));
  v.sbase = sbase;
  v.B = j + 1 < nl ? pre[j + 1] : SEG_FAR;
  v.delta = j < nl ? (int32_t)((int64_t)D[j].x - pre[j]) : 0;
}

// Walks the endpoints [q_lo, q_hi) of one owner on one wave (s_lo: the
// segment holding q_lo); emit(x, valid) sees every position once.  A step
// gives each lane WALK_PER consecutive positions; the segment of each is the
// view's boundaries at or below it, counted over the few boundaries inside
// the step.  Where 64 segments end within a step (very short segments) the
// step falls back to one position per lane.
template <int WALK_UNROLL = 2, class F>
__device__ __forceinline__ void bin_walk(const int32_t* __restrict__ ncol,
                                         const int4* __restrict__ D,
                                         const int64_t* __restrict__ pre, int nl, int64_t q_lo,
                                         int64_t q_hi, int s_lo, F&& emit) {
  const int lane = threadIdx.x & (WAVE - 1);
  if (q_lo >= q_hi) return;
  SegView v;
  seg_view_load(D, pre, nl, s_lo, v);
  int64_t q0 = q_lo;
  while (q0 < q_hi) {
    int64_t b63 = readlane64(v.B, WAVE - 1);
    if (b63 <= q0 + WALK_STEP - 1) {
      // the view may miss boundaries of this step: move it to the segment
      // holding q0
      seg_view_load(D, pre, nl, v.sbase + __popcll(__ballot(v.B <= q0)), v);
      b63 = readlane64(v.B, WAVE - 1);
    }
    if (b63 > q0 + WALK_STEP * WALK_UNROLL - 1) {
      // WALK_UNROLL steps of WALK_PER positions per lane, loads in flight together
      int32_t xs[WALK_UNROLL][WALK_PER];
      const int base_rel = __popcll(__ballot(v.B <= q0));
      uint64_t inside = __ballot(v.B > q0 && v.B <= q0 + WALK_STEP * WALK_UNROLL - 1);
      int rel[WALK_UNROLL][WALK_PER];
#pragma unroll
      for (int u = 0; u < WALK_UNROLL; u++)
#pragma unroll
        for (int k = 0; k < WALK_PER; k++) rel[u][k] = base_rel;
      while (inside) {
        const int j = __ffsll((long long)inside) - 1;
        inside &= inside - 1;
        const int64_t bj = readlane64(v.B, j);
#pragma unroll
        for (int u = 0; u < WALK_UNROLL; u++)
#pragma unroll
          for (int k = 0; k < WALK_PER; k++)
            rel[u][k] += q0 + u * WALK_STEP + lane * WALK_PER + k >= bj ? 1 : 0;
      }
#pragma unroll
      for (int u = 0; u < WALK_UNROLL; u++)
#pragma unroll
        for (int k = 0; k < WALK_PER; k++) {
          const int64_t p = q0 + u * WALK_STEP + lane * WALK_PER + k;
          const int32_t d = __shfl(v.delta, rel[u][k], WAVE);
          xs[u][k] = p < q_hi ? ncol[p + d] : INT_MAX;
        }
#pragma unroll
      for (int u = 0; u < WALK_UNROLL; u++)
#pragma unroll
        for (int k = 0; k < WALK_PER; k++)
          emit(xs[u][k], q0 + u * WALK_STEP + lane * WALK_PER + k < q_hi);
      q0 += WALK_STEP * WALK_UNROLL;
    } else if (b63 > q0 + WALK_STEP - 1) {
      int32_t xs[WALK_PER];
      int rel[WALK_PER];
      const int base_rel = __popcll(__ballot(v.B <= q0));
      uint64_t inside = __ballot(v.B > q0 && v.B <= q0 + WALK_STEP - 1);
#pragma unroll
      for (int k = 0; k < WALK_PER; k++) rel[k] = base_rel;
      while (inside) {
        const int j = __ffsll((long long)inside) - 1;
        inside &= inside - 1;
        const int64_t bj = readlane64(v.B, j);
#pragma unroll
        for (int k = 0; k < WALK_PER; k++) rel[k] += q0 + lane * WALK_PER + k >= bj ? 1 : 0;
      }
#pragma unroll
      for (int k = 0; k < WALK_PER; k++) {
        const int64_t p = q0 + lane * WALK_PER + k;
        const int32_t d = __shfl(v.delta, rel[k], WAVE);
        xs[k] = p < q_hi ? ncol[p + d] : INT_MAX;
      }
#pragma unroll
      for (int k = 0; k < WALK_PER; k++) emit(xs[k], q0 + lane * WALK_PER + k < q_hi);
      q0 += WALK_STEP;
    } else {
      // one position per lane: after the move above at most 63 boundaries
      // lie in (q0, q0 + 63], all in the view
      int rel = __popcll(__ballot(v.B <= q0));
      uint64_t inside = __ballot(v.B > q0 && v.B <= q0 + WAVE - 1);
      while (inside) {
        const int j = __ffsll((long long)inside) - 1;
        inside &= inside - 1;
        rel += q0 + lane >= readlane64(v.B, j) ? 1 : 0;
      }
      const int32_t d = __shfl(v.delta, rel, WAVE);
      const bool valid = q0 + lane < q_hi;
      emit(valid ? ncol[q0 + lane + d] : INT_MAX, valid);
      q0 += WAVE;
    }
  }
}

// First b in [lo, hi] with key(b) >= target (key non-decreasing), hi + 1 if
// none; hi - lo < 4096.  Two probes per lane.
template <class KeyF>
__device__ __forceinline__ int wave_first_ge(int lo, int hi, int64_t target, KeyF&& key) {
  const int lane = threadIdx.x & (WAVE - 1);
  int pb = lo + lane * WAVE + WAVE - 1;
  if (pb > hi) pb = hi;
  const uint64_t m1 = __ballot(lo + lane * WAVE <= hi && key(pb) >= target);
  if (!m1) return hi + 1;
  const int c = __ffsll((long long)m1) - 1;
  const int b = lo + c * WAVE + lane;
  const uint64_t m2 = __ballot(b <= hi && key(b) >= target);
  return lo + c * WAVE + __ffsll((long long)m2) - 1;
}

// hash slot of rank x in a table of BF_HSLOTS (rank + 1, count) pairs
__device__ __forceinline__ uint32_t bin_hash_inc(uint64_t* tab, int32_t x, int* err) {
  const uint64_t key = (uint64_t)(uint32_t)(x + 1) << 32;
  uint32_t h = ((uint32_t)x * 0x9E3779B1u) >> (32 - BF_HBITS);
  for (int p = 0; p < BF_HSLOTS; p++) {
    uint64_t cur = tab[h];
    if (cur == 0) {
      const uint64_t o = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[h]), 0ull,
                                   (unsigned long long)(key | 1u));
      if (o == 0) return 0;
      cur = o;
    }
    if ((cur & 0xffffffff00000000ull) == key)
      return (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(&tab[h]), 1ull);
    h = (h + 1) & (BF_HSLOTS - 1);
  }
  atomicOr(err, ERR_PROBE);
  return 0;
}

// The same for up to N endpoints of one lane (x < 0: none): the home slots
// are read for all of them first, then the empty ones claimed and the
// matching ones incremented, each step issued for all N before any result is
// used; a lost claim or an occupied home slot probes on.
template <int N>
__device__ __forceinline__ uint64_t bin_hash_batch(uint64_t* tab, const int32_t (&x)[N], int* err) {
  auto home = [](int32_t v) { return ((uint32_t)v * 0x9E3779B1u) >> (32 - BF_HBITS); };
  auto key = [](int32_t v) { return (uint64_t)(uint32_t)(v + 1) << 32; };
  uint64_t o[N];
#pragma unroll
  for (int k = 0; k < N; k++) o[k] = x[k] >= 0 ? tab[home(x[k])] : 1;  // 1: no endpoint
  uint32_t won = 0;
#pragma unroll
  for (int k = 0; k < N; k++)
    if (x[k] >= 0 && o[k] == 0) {
      o[k] = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[home(x[k])]), 0ull,
                       (unsigned long long)(key(x[k]) | 1u));
      if (o[k] == 0) won |= 1u << k;
    }
  uint64_t sum = 0;
  uint32_t rest = 0;
#pragma unroll
  for (int k = 0; k < N; k++) {
    if (x[k] < 0 || ((won >> k) & 1)) continue;
    if ((o[k] & 0xffffffff00000000ull) == key(x[k]))
      sum += (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(&tab[home(x[k])]), 1ull);
    else
      rest |= 1u << k;
  }
#pragma unroll
  for (int k = 0; k < N; k++)
    if ((rest >> k) & 1) sum += bin_hash_inc(tab, x[k], err);
  return sum;
}

__device__ __forceinline__ void region_clear(uint32_t* r) {
  const int lane = threadIdx.x & (WAVE - 1);
  uint4* r4 = reinterpret_cast<uint4*>(r);
#pragma unroll
  for (int k = lane; k < BF_WORDS / 4; k += WAVE) r4[k] = make_uint4(0, 0, 0, 0);
}

__global__ __launch_bounds__(BN_NT, 4) void k_c4_bin(C4Args A) {
  __shared__ uint4 cnt4[BN_NW * BF_WORDS / 4];
  __shared__ int32_t off[BF_KMAX + 1];
  __shared__ int16_t bigl[BF_BIGLIST];
  __shared__ int s_item, s_nbig, s_b1, s_next, s_nt;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(cnt4);
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  const int64_t b0i = A.start[A.bucket], cnt_items = A.start[A.bucket + 1] - b0i;
  const int64_t hbase = b0i - A.start[CB_WIN];
  // per block: the scratch plus up to 7 padding entries per target
  int32_t* bins = A.bins + (int64_t)blockIdx.x * (A.bin_cap + BF_PAD * BF_KMAX);
  uint32_t* mycnt = cnt + wid * BF_WORDS;
  u128_t acc = 0;
  // counters kept equal across a wave (scalar registers); lane 0 of each
  // wave contributes its wave's, the block-wide ones counted by wave 0
  unsigned long long wedges = 0, owners = 0, segs = 0, reads = 0;
  region_clear(mycnt);
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = uni(s_item);
    if (item >= cnt_items) break;
    const int64_t pos = cnt_items - 1 - item;  // heaviest owners (highest ranks) first
    const int32_t u = uni(A.order[b0i + pos]);
    const int64_t so = uni64(A.seg_off[hbase + pos]);
    const int nl = uni(A.seg_cnt[hbase + pos]);
    const int4* D = A.desc + so;
    const int64_t* pre = A.seg_pre + so;
    const int64_t total = uni64(nl > 0 ? pre[nl - 1] + (D[nl - 1].y - D[nl - 1].x) : 0);
    const int32_t uwords = zone_words(A, u);
    const int K = (uwords + BF_WORDS - 1) >> BF_SHIFT;
    for (int i = tid; i <= K; i += BN_NT) off[i] = 0;
    // each wave's contiguous share of the endpoints, in whole steps, and the
    // segment holding its first endpoint
    constexpr int SHARE = WALK_STEP * 2;
    const int64_t steps = (total + SHARE - 1) / SHARE;
    const int64_t q_lo = std::min(total, (steps * wid / BN_NW) * SHARE);
    const int64_t q_hi = std::min(total, (steps * (wid + 1) / BN_NW) * SHARE);
    int s_lo = 0;
    if (q_lo < q_hi) {
      // last segment with start <= q_lo: 64-ary search over the starts
      int lo = 0, hi = nl - 1;
      while (hi - lo >= WAVE) {
        const int64_t stride = (hi - lo + WAVE) / WAVE;
        const int64_t p = lo + stride * lane;
        const uint64_t m = __ballot(p <= hi && pre[p] <= q_lo);
        const int c = 63 - __clzll((long long)m);  // lane 0 (p = lo) always qualifies
        const int nlo = (int)(lo + stride * c);
        hi = (int)std::min<int64_t>(hi, nlo + stride - 1);
        lo = nlo;
      }
      const uint64_t m = __ballot(lo + lane <= hi && pre[lo + lane] <= q_lo);
      s_lo = lo + 63 - __clzll((long long)m);
    }
    owners++;
    segs += (unsigned long long)nl;
    __syncthreads();
    // ---- pass 1: endpoints per bucket
    bin_walk(A.ncol, D, pre, nl, q_lo, q_hi, s_lo, [&](int32_t x, bool valid) {
      if (valid) atomicAdd(&off[fbin_of(A, x)], 1);
    });
    reads += (unsigned long long)total;
    __syncthreads();
    // exclusive prefix: off[b] = first scatter position of bucket b
    {
      constexpr int PER = (BF_KMAX + 1 + BN_NT - 1) / BN_NT;
      int32_t v[PER];
      int64_t sum = 0;
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int b = tid * PER + k;
        v[k] = b < K ? off[b] : 0;
        sum += v[k];
      }
      int64_t tot;
      int64_t run = block_excl_scan64<BN_NT>(sum, &tot);
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int b = tid * PER + k;
        if (b <= K) off[b] = (int32_t)run;
        run += v[k];
      }
    }
    __syncthreads();
    int b0 = 0;
    while (b0 < K) {
      // ---- the next bucket range whose endpoints fit the scratch
      const int64_t p0 = uni(off[b0]);
      if (wid == 0) {
        const int f = wave_first_ge(b0 + 1, K, p0 + A.bin_cap + 1,
                                    [&](int b) { return (int64_t)off[b]; });
        if (lane == 0) {
          s_b1 = f - 1;
          s_nbig = 0;
        }
      }
      __syncthreads();
      const int b1 = uni(s_b1);
      const int64_t off_end = uni(off[b1]);  // first position past the range
      if (b1 == b0) {
        // one bucket alone beyond the scratch: counted straight from the rows
        const int32_t wlo = b0 << BF_SHIFT;
        uint64_t part = 0;
        bin_walk(A.ncol, D, pre, nl, q_lo, q_hi, s_lo, [&](int32_t x, bool valid) {
          if (valid && fbin_of(A, x) == b0) part += window_inc(A, cnt, wlo, x);
        });
        acc += part;
        if (wid == 0) wedges += (unsigned long long)(off[b0 + 1] - off[b0]);
        reads += (unsigned long long)total;
        __syncthreads();
        for (int i = tid; i < BF_WORDS; i += BN_NT) cnt[i] = 0;
        if (tid == 0) off[b0] = off[b0 + 1];  // the end of bucket b0
        __syncthreads();
        b0++;
        continue;
      }
      // ---- targets: runs of consecutive buckets that start within one
      // stretch of BF_GROUP positions (hash targets), a bucket holding more
      // than BF_GROUP endpoints alone (a dense target; it always ends its
      // stretch).  Each bucket's target goes to off; the scatter state sits in
      // the counter regions, unused until pass 3: per target its write
      // cursor (bit 31: dense), and for the last BF_NTS targets a BF_SB-entry
      // staging buffer (its fill and completion counts, and a tail cursor for
      // endpoints that arrive while it is full).  Targets start at multiples
      // of 8 scratch entries, so a full buffer leaves as aligned 16-byte
      // stores instead of BF_SB scattered ones.
      uint32_t* head = cnt;
      uint32_t* tail = cnt + BF_KMAX;
      uint32_t* tend = tail + BF_NTS;
      uint32_t* fill = tend + BF_NTS;
      uint32_t* done = fill + BF_NTS;
      int32_t* stage = reinterpret_cast<int32_t*>(done + BF_NTS);
      {
        constexpr int PER = (BF_KMAX + BN_NT - 1) / BN_NT;
        uint32_t beg = 0, big = 0;
        // positions relative to p0 are below the scratch size (< 2^31)
        for (int k = 0; k < PER; k++) {
          const int b = b0 + tid * PER + k;
          if (b < b1) {
            const uint32_t sr = (uint32_t)(off[b] - p0), er = (uint32_t)(off[b + 1] - p0);
            const uint32_t pr = b == b0 ? 0u : (uint32_t)(off[b - 1] - p0);
            if (er - sr > BF_GROUP) big |= 1u << k;
            if (b == b0 || er - sr > BF_GROUP || sr / BF_GROUP != pr / BF_GROUP) beg |= 1u << k;
          }
        }
        int64_t ntot;
        int t = (int)block_excl_scan64<BN_NT>(__popc(beg), &ntot) - 1;
        // every read of a neighbour's entry of off is done (the scan
        // synchronised); each thread now rewrites only its own entries.
        // head[t] takes the target's first position for now.
        for (int k = 0; k < PER; k++) {
          const int b = b0 + tid * PER + k;
          if (b < b1) {
            if ((beg >> k) & 1) {
              t++;
              head[t] = (uint32_t)(off[b] - p0) | (((big >> k) & 1u) << 31);
            }
            off[b] = t;
          }
        }
        if (tid == 0) s_nt = (int)ntot;
        __syncthreads();
        // padded starts: each target's count rounded up to a multiple of BF_PAD
        const int nt = (int)ntot;
        const int sb = nt > BF_NTS ? nt - BF_NTS : 0;  // first target with a buffer
        const uint32_t span = (uint32_t)(off_end - p0);
        uint32_t st[PER + 1], kinds = 0, psum = 0;
        for (int k = 0; k <= PER; k++) {
          const int tt = tid * PER + k;
          st[k] = tt < nt ? head[tt] : span;
          if (k < PER && (st[k] >> 31)) kinds |= 1u << k;
          st[k] &= 0x7fffffffu;
        }
        for (int k = 0; k < PER; k++)
          if (tid * PER + k < nt) psum += (st[k + 1] - st[k] + BF_PAD - 1) & ~(BF_PAD - 1u);
        uint32_t ps = (uint32_t)block_excl_scan64<BN_NT>(psum, nullptr);
        for (int k = 0; k < PER; k++) {
          const int tt = tid * PER + k;
          if (tt < nt) {
            const uint32_t c = st[k + 1] - st[k];
            head[tt] = ps | (((kinds >> k) & 1u) << 31);
            if (tt >= sb) {
              tail[tt - sb] = tend[tt - sb] = ps + c;
              fill[tt - sb] = done[tt - sb] = 0;
            }
            ps += (c + BF_PAD - 1) & ~(BF_PAD - 1u);
          }
        }
      }
      __syncthreads();
      const int ntargets = uni(s_nt);
      // the last BF_NTS targets (the highest ranks, whose buckets of 32-bit
      // counters span the fewest ranks and hold the most endpoints) have
      // staging buffers
      const int sbase = ntargets > BF_NTS ? ntargets - BF_NTS : 0;
      // ---- pass 2: scatter the range's endpoints by target (one step in
      // flight: its stores, not its loads, bound this pass)
      bin_walk<1>(A.ncol, D, pre, nl, q_lo, q_hi, s_lo, [&](int32_t x, bool valid) {
        bool flush = false;
        int t = 0, sl = 0;
        if (valid) {
          const int w = fbin_of(A, x);
          if (w >= b0 && w < b1) {
            t = off[w];
            sl = t - sbase;
            if (sl >= 0) {
              const uint32_t slot = atomicAdd(&fill[sl], 1u);
              if (slot < BF_SB) {
                stage[sl * BF_SB + slot] = x;
                flush = atomicAdd(&done[sl], 1u) == BF_SB - 1;
              } else {
                bins[atomicSub(&tail[sl], 1u) - 1] = x;
              }
            } else {
              bins[atomicAdd(&head[t], 1u) & 0x7fffffffu] = x;
            }
          }
        }
        if (flush) {
          // every slot of the buffer is written: it leaves as aligned
          // 16-byte stores, two at a time, and only then are the counters
          // reset (no new entry lands in the buffer before that)
          const int4* sv = reinterpret_cast<const int4*>(stage + sl * BF_SB);
          const uint32_t at = atomicAdd(&head[t], (uint32_t)BF_SB) & 0x7fffffffu;
          int4* dst = reinterpret_cast<int4*>(bins + at);
#pragma unroll
          for (int k = 0; k < BF_SB / 4; k += 2) {
            const int4 v0 = sv[k], v1 = sv[k + 1];
            dst[k] = v0;
            dst[k + 1] = v1;
          }
          done[sl] = 0;
          fill[sl] = 0;
        }
      });
      reads += (unsigned long long)total;
      __syncthreads();
      // buffers still holding entries, then the target ends (bit 31: dense)
      // move to off[b0 ..) and the regions are cleared
      for (int t = sbase + tid; t < ntargets; t += BN_NT) {
        const uint32_t at = head[t] & 0x7fffffffu;
        for (uint32_t k = 0; k < done[t - sbase]; k++) bins[at + k] = stage[(t - sbase) * BF_SB + k];
      }
      __syncthreads();
      for (int t = tid; t < ntargets; t += BN_NT)
        off[b0 + t] = (int32_t)((t >= sbase ? tend[t - sbase] : head[t] & 0x7fffffffu) |
                                (head[t] & 0x80000000u));
      __syncthreads();
      for (int i = tid; i < BN_NW * BF_WORDS / 4; i += BN_NT) cnt4[i] = make_uint4(0, 0, 0, 0);
      if (tid == 0) {
        s_next = 0;
        s_nbig = 0;
      }
      __syncthreads();
      // ---- pass 3: targets taken one at a time by waves; the next one is
      // taken and its first endpoints loaded before the current is counted
      uint64_t* tab = reinterpret_cast<uint64_t*>(mycnt);
      constexpr int HPER = (2 * BF_GROUP + WAVE - 1) / WAVE;  // hash-target endpoints per lane
      // target t occupies [tbeg(t), its end): ends are exact, starts padded
      auto tbeg = [&](int t) -> int64_t {
        return t == 0 ? 0
                      : (int64_t)((((uint32_t)off[b0 + t - 1] & 0x7fffffffu) + BF_PAD - 1) &
                                  ~(BF_PAD - 1u));
      };
      auto grab = [&]() {
        int g = 0;
        if (lane == 0) g = atomicAdd(&s_next, 1);
        return uni(__shfl(g, 0, WAVE));
      };
      struct Tgt {
        int t;
        bool dense;
        int64_t s, e;
      };
      auto fetch = [&](int t, Tgt& T, int32_t (&xv)[HPER]) {
        T.t = t;
        T.dense = false;
        T.s = T.e = 0;
        if (t < ntargets) {
          const uint32_t ev = (uint32_t)uni(off[b0 + t]);
          T.s = uni64(tbeg(t));
          T.e = ev & 0x7fffffffu;
          T.dense = (ev >> 31) != 0;
        }
#pragma unroll
        for (int k = 0; k < HPER; k++) {
          const int64_t q = T.s + lane + k * WAVE;
          xv[k] = q < T.e ? bins[q] : -1;
        }
      };
      Tgt cur, nxt;
      int32_t xc[HPER], xn[HPER];
      fetch(grab(), nxt, xn);
      while (nxt.t < ntargets) {
        cur = nxt;
#pragma unroll
        for (int k = 0; k < HPER; k++) xc[k] = xn[k];
        fetch(grab(), nxt, xn);
        const int64_t n_e = cur.e - cur.s;
        if (n_e == 0) continue;
        if (!cur.dense) {
          // a hash target: fewer than 2 * BF_GROUP endpoints, all loaded
          acc += bin_hash_batch(tab, xc, &A.scal->err);
          wedges += (unsigned long long)n_e;
          wave_sync();
          region_clear(mycnt);
          wave_sync();
          continue;
        }
        const int l = fbin_of(A, __shfl(xc[0], 0, WAVE));
        if (n_e > BF_BIG) {
          if (lane == 0) {
            const int k = atomicAdd(&s_nbig, 1);
            if (k < BF_BIGLIST) bigl[k] = (int16_t)cur.t;
          }
          continue;
        }
        // ---- one dense bucket in this wave's region
        const int32_t wlo = l << BF_SHIFT;
        uint64_t part = 0;
#pragma unroll
        for (int k = 0; k < HPER; k++)
          if (xc[k] >= 0) part += window_inc(A, mycnt, wlo, xc[k]);
        int64_t q = cur.s + HPER * WAVE + lane;
        for (; q + 3 * WAVE < cur.e; q += 4 * WAVE) {
          int32_t xv[4];
#pragma unroll
          for (int k = 0; k < 4; k++) xv[k] = bins[q + k * WAVE];
#pragma unroll
          for (int k = 0; k < 4; k++) part += window_inc(A, mycnt, wlo, xv[k]);
        }
        for (; q < cur.e; q += WAVE) part += window_inc(A, mycnt, wlo, bins[q]);
        acc += part;
        wedges += (unsigned long long)n_e;
        wave_sync();
        region_clear(mycnt);
        wave_sync();
      }
      __syncthreads();
      // dense targets too large for one wave: the whole block, one region
      // (listed, or found by a scan of the targets when the list overflowed)
      const int nbig = uni(s_nbig);
      auto count_big = [&](int t) {
        const int64_t bs = tbeg(t), be = off[b0 + t] & 0x7fffffff;
        const int32_t wlo = fbin_of(A, bins[bs]) << BF_SHIFT;
        uint64_t part = 0;
        for (int64_t q = bs + tid; q < be; q += BN_NT) part += window_inc(A, cnt, wlo, bins[q]);
        acc += part;
        if (wid == 0) wedges += (unsigned long long)(be - bs);
        __syncthreads();
        for (int i = tid; i < BF_WORDS; i += BN_NT) cnt[i] = 0;
        __syncthreads();
      };
      if (nbig <= BF_BIGLIST) {
        for (int k = 0; k < nbig; k++) count_big(bigl[k]);
      } else {
        for (int t = 0; t < ntargets; t++) {
          const uint32_t ev = (uint32_t)off[b0 + t];
          if ((ev >> 31) && (int64_t)(ev & 0x7fffffffu) - tbeg(t) > BF_BIG) count_big(t);
        }
      }
      b0 = b1;
      __syncthreads();
    }
  }
  block_add_u128<BN_NT>(&A.scal->acc[ACC_C4], acc);
  if (A.flags & M4_STATS) {
    const unsigned long long wv = lane == 0 ? wedges : 0, b0v = tid == 0 ? 1 : 0;
    block_add_u64<BN_NT>(&A.scal->stat[ST_WEDGES], wv);
    block_add_u64<BN_NT>(&A.scal->kstat[A.slot][0], wv);
    block_add_u64<BN_NT>(&A.scal->kstat[A.slot][1], owners * b0v);
    block_add_u64<BN_NT>(&A.scal->kstat[A.slot][2], segs * b0v);
    block_add_u64<BN_NT>(&A.scal->kstat[A.slot][3], reads * b0v);
  }
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)ceil_div(n > 0 ? n : 1, nt); }

}  // namespace

Launch c4_plan(const Prep& P, const Classes& C, Scal* scal, const Tuning& tu, uint32_t flags,
               Arena& tmp, hipStream_t s, int num_cu, KTimer* kt,
               const std::function<char*(size_t)>& big_scratch, bool* binned) {
  const int64_t n = P.n;
  if (n == 0 || P.m == 0) return [](hipStream_t) {};
  int64_t* wub = tmp.take<int64_t>(n);
  uint32_t* key = tmp.take<uint32_t>(n);
  int32_t* order = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, C4_KEY_BITS));
  // bucket starts (C4_START_SLOTS), then the two zone bounds
  int64_t* start = tmp.take<int64_t>(C4_START_SLOTS + 2);
  int32_t* hlen = tmp.take<int32_t>(n);
  int64_t* seg_off = tmp.take<int64_t>(n + 1);
  int64_t* stmp = tmp.take<int64_t>(scan_tmp_elems(n));
  // per-row records of full rows (a partition stores row prefixes instead)
  int4* vmeta = P.row_len ? nullptr : tmp.take<int4>(n);
  if (!wub || !key || !order || !rtmp || !start || !hlen || !seg_off || !stmp ||
      (!P.row_len && !vmeta))
    throw Fail(M4_EINTERNAL, "workspace too small (c4)");
  fill_u32(&scal->work_c4[0], 0, 8, s);
  // zone bounds first: the planner needs every owner's window count
  int64_t* zbounds = start + C4_START_SLOTS;
  k_zone_bounds<<<1, 64, 0, s>>>(P.dr, n, zbounds);
  C4Plan pl{tu.c4_light_max, tu.c4_med_max, tu.c4_med_win, tu.c4_bin_win, tu.c4_bin_dense,
            zbounds, C.r1};
  // rows by degree: <= 64 with 8 lanes, <= 4096 with a wavefront, longer
  // rows with a workgroup
  const int64_t b64 = C.bound[4], b4096 = C.bound[7];
  if (kt) kt->begin(M4_K_C4_PLAN, s);
  if (b64 > 0)
    k_c4_plan<8><<<blocks_for(b64 * 8, 256), 256, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, 0, b64,
                                                          C.r1, pl, wub, key, P.own_lo, P.hi());
  if (b4096 > b64)
    k_c4_plan<64><<<blocks_for((b4096 - b64) * 64, 256), 256, 0, s>>>(
        P.nptr, P.ncol, P.dr, P.dlo, b64, b4096, C.r1, pl, wub, key, P.own_lo, P.hi());
  if (n > b4096)
    k_c4_plan_big<<<(unsigned)(n - b4096), 1024, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, b4096, C.r1,
                                                         pl, wub, key, P.own_lo, P.hi());
  radix_pass(key, nullptr, n, 0, C4_KEY_BITS, nullptr, order, rtmp, start, s);
  std::array<int64_t, C4_START_SLOTS + 2> hstart;
  M4_HIP(hipMemcpyAsync(hstart.data(), start, sizeof(int64_t) * hstart.size(),
                        hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  // counter zones of the window and binned owners
  const int64_t z1 = std::max<int64_t>(hstart[C4_START_SLOTS], C.r1);
  const int64_t z2 = std::max<int64_t>(hstart[C4_START_SLOTS + 1], z1);
  const int64_t aw = (z1 - C.r1 + 7) >> 3, bw = (z2 - z1 + 3) >> 2;
  // window and binned owners are adjacent in the bucket order: one set of
  // segment descriptors serves both
  const int64_t H = hstart[CB_BIN + 1] - hstart[CB_WIN];
  const int64_t HB = hstart[CB_BIN + 1] - hstart[CB_BIN];
  if (binned) *binned = HB > 0;
  int4* desc = nullptr;
  int64_t* seg_pre = nullptr;
  int32_t* seg_cnt = nullptr;
  int32_t* bins = nullptr;
  int64_t bin_cap = 0;
  unsigned bin_grid = 0;
  if (H > 0) {
    k_c4_heavy_len<<<blocks_for(H, 256), 256, 0, s>>>(order, start, P.dlo, hlen);
    scan_i32(hlen, H, seg_off, stmp, s);
    int64_t nseg = 0;
    M4_HIP(hipMemcpyAsync(&nseg, seg_off + H, 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    const size_t db = ((size_t)(nseg > 0 ? nseg : 1) * sizeof(int4) + 255) & ~size_t(255);
    const size_t cb = ((size_t)H * 4 + 255) & ~size_t(255);
    // length prefixes: binned owners only (their slots, after the window owners')
    const size_t pb = HB > 0 ? ((size_t)(nseg > 0 ? nseg : 1) * 8 + 255) & ~size_t(255) : 0;
    // binned owners: two workgroups per CU, each with a scratch of at most
    // 2^20 endpoints by default (no owner has more endpoints than the graph
    // has CSR entries)
    size_t bb = 0;
    if (HB > 0) {
      const int64_t cap = tu.c4_bin_cap > 0 ? tu.c4_bin_cap : int64_t(1) << 20;
      bin_cap = (std::min<int64_t>(cap, std::max<int64_t>(P.nnz, 1)) + BF_PAD - 1) &
                ~int64_t(BF_PAD - 1);
      bin_grid = (unsigned)std::min<int64_t>(2 * (int64_t)num_cu, HB);
      bb = (size_t)bin_grid * (size_t)(bin_cap + BF_PAD * BF_KMAX) * 4;
    }
    char* scr = big_scratch(db + cb + pb + bb);
    if (!scr) throw Fail(M4_ENOMEM, "no room for 4-cycle segment descriptors");
    desc = reinterpret_cast<int4*>(scr);
    seg_cnt = reinterpret_cast<int32_t*>(scr + db);
    if (HB > 0) {
      seg_pre = reinterpret_cast<int64_t*>(scr + db + cb);
      bins = reinterpret_cast<int32_t*>(scr + db + cb + pb);
    }
  }
  if (kt) kt->end(M4_K_C4_PLAN, s);

  C4Args A{};
  A.order = order;
  A.start = start;
  A.nptr = P.nptr;
  A.ncol = P.ncol;
  A.dr = P.dr;
  A.dlo = P.dlo;
  A.wub = wub;
  A.row_len = P.row_len;
  A.r1 = C.r1;
  A.scal = scal;
  A.flags = flags;
  A.seg_off = seg_off;
  A.desc = desc;
  A.seg_pre = seg_pre;
  A.seg_cnt = seg_cnt;
  A.bins = bins;
  A.bin_cap = bin_cap;
  A.z1 = (int32_t)z1;
  A.z2 = (int32_t)z2;
  A.aw = (int32_t)aw;
  A.bw = (int32_t)bw;
  A.zr1 = (int32_t)C.r1;
  // everything below runs on the launch stream, after the plan above
  return [=](hipStream_t ls) mutable {
    if (H > 0) {
      if (kt) kt->begin(M4_K_C4_DESC, ls);
      // with stored prefixes only the partition's rows are valid: no full pass
      if (!P.row_len)
        k_vmeta<<<blocks_for(n, 256), 256, 0, ls>>>(P.nptr, P.ncol, P.dr, P.dlo, n, C.r1, vmeta);
      k_c4_desc<<<(unsigned)H, 256, 0, ls>>>(order, start, seg_off, P.nptr, P.dlo, P.ncol,
                                             P.row_len ? nullptr : vmeta, P.row_len, C.r1,
                                             desc, seg_pre, seg_cnt);
      if (kt) kt->end(M4_K_C4_DESC, ls);
    }
    // heavy owners first: one 1024-thread workgroup per CU
    if (HB > 0) {
      A.bucket = CB_BIN;
      A.slot = M4_K_C4_BIN;
      A.work = &scal->work_c4[CB_BIN];
      if (kt) kt->begin(M4_K_C4_BIN, ls);
      k_c4_bin<<<bin_grid, BN_NT, 0, ls>>>(A);
      if (kt) kt->end(M4_K_C4_BIN, ls);
    }
    if (hstart[CB_WIN + 1] > hstart[CB_WIN]) {
      A.bucket = CB_WIN;
      A.slot = M4_K_C4_WINDOW;
      A.work = &scal->work_c4[CB_WIN];
      if (kt) kt->begin(M4_K_C4_WINDOW, ls);
      k_c4_window<<<(unsigned)num_cu, W_NT, 0, ls>>>(A);
      if (kt) kt->end(M4_K_C4_WINDOW, ls);
    }
    if (hstart[CB_MED + 1] > hstart[CB_MED]) {
      A.bucket = CB_MED;
      A.slot = M4_K_C4_MED;
      A.work = &scal->work_c4[CB_MED];
      if (kt) kt->begin(M4_K_C4_MED, ls);
      k_c4_hash<1024, C4_MED_SLOTS, 4><<<(unsigned)num_cu, 1024, 0, ls>>>(A);
      if (kt) kt->end(M4_K_C4_MED, ls);
    }
    if (hstart[CB_HASH + 1] > hstart[CB_HASH]) {
      A.bucket = CB_HASH;
      A.slot = M4_K_C4_HASH;
      A.work = &scal->work_c4[CB_HASH];
      if (kt) kt->begin(M4_K_C4_HASH, ls);
      k_c4_hash<256, C4_HASH_SLOTS, 4><<<(unsigned)(num_cu * 4), 256, 0, ls>>>(A);
      if (kt) kt->end(M4_K_C4_HASH, ls);
    }
  };
}

}  // namespace m4
