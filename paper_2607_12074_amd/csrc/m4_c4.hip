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
//   hash bucket   -- small W_u: one workgroup, open-addressing table in LDS;
//   window bucket -- large W_u: one 1024-thread workgroup, dense counters in
//                    LDS over windows of 128 KiB; a counter is 4 bits wide
//                    for endpoints of degree <= 15, 8 bits for degree <= 255
//                    and 32 bits beyond (c_u[w] never exceeds d(w)), so a
//                    window spans up to 262144 ranks; every lower neighbour
//                    keeps a cursor into its sorted row so each window reads
//                    exactly its own endpoints.
#include <limits.h>

#include <algorithm>
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
  const int64_t* seg_off;  // window owners: first descriptor of each owner
  int4* desc;              // window owners: per-segment cursor descriptors
  // counter zones of the window owners (ranks >= r1): 4-bit counters for
  // ranks [r1, z1) (degree <= 15), 8-bit for [z1, z2) (degree <= 255), 32-bit
  // from z2 on; aw and bw are the words of the first two zones
  int64_t z1, z2, aw, bw;
};

// wedge bound of every owner: G lanes cooperate on one row, 4 loads in flight
template <int G>
__global__ __launch_bounds__(256) void k_c4_plan(const int64_t* __restrict__ nptr,
                                                 const int32_t* __restrict__ ncol,
                                                 const int32_t* __restrict__ dr,
                                                 const int32_t* __restrict__ dlo, int64_t r_lo,
                                                 int64_t r_hi, int64_t r1, int light_max,
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
    if (u >= r1 && nl >= 2 && s > 0) {
      if (s <= light_max) k = CB_HASH;
      else k = CB_WIN16;
    }
    key[u] = k;
  }
}

// rows too long for one wavefront: one 1024-thread workgroup per row
__global__ __launch_bounds__(1024) void k_c4_plan_big(const int64_t* __restrict__ nptr,
                                                      const int32_t* __restrict__ ncol,
                                                      const int32_t* __restrict__ dr,
                                                      const int32_t* __restrict__ dlo, int64_t r_lo,
                                                      int64_t r1, int light_max,
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
    if (u >= r1 && nl >= 2 && tot > 0) {
      if (tot <= light_max) k = CB_HASH;
      else k = CB_WIN16;
    }
    key[u] = k;
  }
}

// ---------------------------------------------------------- hash bucket
constexpr int H_NT = 256, H_SLOTS = C4_HASH_SLOTS, H_CHUNK = H_NT;

__global__ __launch_bounds__(H_NT) void k_c4_hash(C4Args A) {
  __shared__ int32_t hkey[H_SLOTS];
  __shared__ uint32_t hcnt[H_SLOTS];
  __shared__ int32_t sst[H_CHUNK];
  __shared__ int32_t spref[H_CHUNK + 1];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int64_t b0 = A.start[A.bucket], cnt = A.start[A.bucket + 1] - b0;
  u128_t acc = 0;
  unsigned long long wedges = 0, owners = 0, segs = 0, reads = 0;
  for (int i = tid; i < H_SLOTS; i += H_NT) {
    hkey[i] = -1;
    hcnt[i] = 0;
  }
  constexpr int GRAB = 8;
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
    int64_t wb = A.wub[u];
    int S = 64;
    while (S < 2 * wb && S < H_SLOTS) S <<= 1;
    const uint32_t mask = (uint32_t)S - 1;
    const int shift = 32 - __ffs(S) + 1;
    if (tid == 0) {
      owners++;
      segs += (unsigned long long)nl;
    }
    for (int c0 = 0; c0 < nl; c0 += H_CHUNK) {
      const int nc = nl - c0 < H_CHUNK ? nl - c0 : H_CHUNK;
      int len = 0;
      if (tid < nc) {
        int32_t v = A.ncol[base + c0 + tid];
        sst[tid] = (int32_t)A.nptr[v];
        len = A.row_len ? A.row_len[v] : A.dr[v];
      }
      int64_t tot;
      int64_t ex = block_excl_scan64<H_NT>(len, &tot);
      if (tid < nc) spref[tid] = (int32_t)ex;
      if (tid == 0) spref[nc] = (int32_t)tot;
      __syncthreads();
      const int total = (int)tot;
      if (tid == 0) reads += (unsigned long long)total;
      for (int q = tid; q < total; q += H_NT) {
        int si = upper_index(spref, nc, q);
        int32_t w = A.ncol[sst[si] + (q - spref[si])];
        if (w < A.r1 || w >= u) continue;
        uint32_t h = ((uint32_t)w * 0x9E3779B1u) >> shift;
        for (;;) {
          int32_t k = hkey[h];
          if (k == w) break;
          if (k == -1) {
            int32_t prev = atomicCAS(&hkey[h], -1, w);
            if (prev == -1 || prev == w) break;
          }
          h = (h + 1) & mask;
        }
        acc += atomicAdd(&hcnt[h], 1u);
        wedges++;
      }
      __syncthreads();
    }
    for (int i = tid; i < S; i += H_NT) {
      hkey[i] = -1;
      hcnt[i] = 0;
    }
    __syncthreads();
  }
  block_add_u128<H_NT>(&A.scal->acc[ACC_C4], acc);
  if (A.flags & M4_STATS) {
    block_add_u64<H_NT>(&A.scal->stat[ST_WEDGES], wedges);
    block_add_u64<H_NT>(&A.scal->kstat[A.slot][0], wedges);
    block_add_u64<H_NT>(&A.scal->kstat[A.slot][1], owners);
    block_add_u64<H_NT>(&A.scal->kstat[A.slot][2], segs);
    block_add_u64<H_NT>(&A.scal->kstat[A.slot][3], reads);
  }
}

// -------------------------------------------------------- window bucket
// Segment descriptors of the window owners: for lower neighbour v of owner u
// the cursor into row v (first entry >= r1), the end of the stored row and
// the values at the cursor and 7 entries after it.  The windows stop at the first entry >= their
// upper end, so the position of u in row v is never needed.  Built once per
// owner by a block of its own.
__global__ __launch_bounds__(256) void k_c4_desc(const int32_t* __restrict__ order,
                                                 const int64_t* __restrict__ start,
                                                 const int64_t* __restrict__ seg_off,
                                                 const int64_t* __restrict__ nptr,
                                                 const int32_t* __restrict__ dlo,
                                                 const int32_t* __restrict__ ncol,
                                                 const int32_t* __restrict__ lowcut,
                                                 const int32_t* __restrict__ row_len, int64_t r1,
                                                 int4* __restrict__ desc) {
  const int64_t h = blockIdx.x;
  const int32_t u = order[start[CB_WIN16] + h];
  const int64_t so = seg_off[h], base = nptr[u];
  const int nl = dlo[u];
  for (int i = threadIdx.x; i < nl; i += 256) {
    const int32_t v = ncol[base + i];
    const int64_t rs = nptr[v];
    const int64_t rend = row_len ? rs + row_len[v] : nptr[v + 1];
    // first entry >= r1: precomputed for full rows, searched for stored prefixes
    int64_t c = lowcut ? rs + lowcut[v] : lower_index(ncol, rs, rend, (int32_t)r1);
    desc[so + i] = make_int4((int)c, (int)rend, c < rend ? ncol[c] : INT_MAX,
                             c + 7 < rend ? ncol[c + 7] : INT_MAX);
  }
}

// entries below r1 (degree <= 1) at the head of every sorted row
__global__ void k_lowcut(const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                         const int32_t* __restrict__ row_len, int64_t n, int64_t r1,
                         int32_t* __restrict__ lowcut) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t rend = row_len ? nptr[v] + row_len[v] : nptr[v + 1];
  lowcut[v] = (int32_t)(lower_index(ncol, nptr[v], rend, (int32_t)r1) - nptr[v]);
}

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

__global__ void k_c4_heavy_len(const int32_t* __restrict__ order, const int64_t* __restrict__ start,
                               const int32_t* __restrict__ dlo, int32_t* __restrict__ len) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = start[CB_WIN16], H = start[CB_WIN32 + 1] - b;
  if (h < H) len[h] = dlo[order[b + h]];
}

constexpr int W_NT = 1024, W_GL = 8, W_NG = W_NT / W_GL, W_SHORT = 8;
constexpr int W_BATCH = 4096;  // segments per pass (bounds the long-visit queue)
constexpr int W_RPT = W_BATCH / W_NT;  // segments per thread and pass

// Counter of rank x (x >= r1) in the zoned layout: a 4-bit counter while the
// degree of x is <= 15, 8-bit while <= 255, else 32-bit.  c_u[x] counts
// common neighbours of u and x, so it never exceeds the degree of x and no
// counter overflows into its neighbour.
__device__ __forceinline__ void zone_slot(const C4Args& A, int64_t x, int64_t& word, int& shift) {
  if (x < A.z1) {
    const int64_t k = x - A.r1;
    word = k >> 3;
    shift = (int)(k & 7) * 4;
  } else if (x < A.z2) {
    const int64_t k = x - A.z1;
    word = A.aw + (k >> 2);
    shift = (int)(k & 3) * 8;
  } else {
    word = A.aw + A.bw + (x - A.z2);
    shift = 0;
  }
}

// first rank whose counter lies in word w
__device__ __forceinline__ int64_t zone_rank(const C4Args& A, int64_t w) {
  if (w < A.aw) return A.r1 + 8 * w;
  if (w < A.aw + A.bw) return A.z1 + 4 * (w - A.aw);
  return A.z2 + (w - A.aw - A.bw);
}

// words holding the counters of ranks [r1, u)
__device__ __forceinline__ int64_t zone_words(const C4Args& A, int64_t u) {
  if (u <= A.r1) return 0;
  if (u <= A.z1) return (u - A.r1 + 7) >> 3;
  if (u <= A.z2) return A.aw + ((u - A.z1 + 3) >> 2);
  return A.aw + A.bw + (u - A.z2);
}

// one wedge endpoint x of the window starting at word wlo (no value returned:
// the sum of C(c, 2) is taken from the counters when the window closes)
__device__ __forceinline__ void window_inc(const C4Args& A, uint32_t* cnt, int64_t wlo,
                                           int32_t x) {
  int64_t word;
  int shift;
  zone_slot(A, x, word, shift);
  atomicAdd(&cnt[word - wlo], 1u << shift);
}

// Adds sum C(c, 2) over the counters in words [wlo, wlo + words) of a closing
// window and clears them for the next one.
__device__ __forceinline__ void window_close(const C4Args& A, uint32_t* cnt, int64_t wlo,
                                             int words, u128_t& acc) {
  uint64_t s = 0;
  for (int i = threadIdx.x; i < words; i += W_NT) {
    const uint32_t w = cnt[i];
    if (w) {
      const int64_t gw = wlo + i;
      if (gw < A.aw) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const uint64_t c = (w >> (4 * k)) & 0xfu;
          s += c * (c - 1) / 2;
        }
      } else if (gw < A.aw + A.bw) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const uint64_t c = (w >> (8 * k)) & 0xffu;
          s += c * (c - 1) / 2;
        }
      } else {
        s += (uint64_t)w * (w - 1) / 2;
      }
      cnt[i] = 0;
    }
  }
  acc += s;
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
__device__ __forceinline__ int short_visit(const C4Args& A, const int4* __restrict__ ncol4,
                                           uint32_t* cnt, int4& d, int64_t wlo, int32_t hi) {
  const int64_t c = d.x, e = d.y, base = c & ~int64_t(3);
  const int off = (int)(c - base);
  int4 v[5];
#pragma unroll
  for (int q = 0; q < 5; q++) v[q] = ncol4[(base >> 2) + q];
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
#pragma unroll
  for (int j = 0; j < W_SHORT; j++)
    if (x[j] < hi) {
      window_inc(A, cnt, wlo, x[j]);
      took++;
    }
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

// One heavy owner per workgroup, windows of counters in LDS in order.  A
// segment is one lower neighbour's row; its descriptor holds the cursor (the
// first entry not yet counted), the row end, and the values at the cursor and
// 7 entries after it, so the length of its visit to a window is known to be
// 0, at most 7, or more without reading the row.  Rows are read with 16-byte
// loads aligned below the cursor (entries before the cursor lie below the
// window, entries from the row end on are masked; the array has slack after
// its last row).  Per pass over W_BATCH segments, every thread first takes
// whole segments by itself: an empty visit costs the descriptor only, a
// short one five 16-byte loads; longer visits are queued in LDS and walked
// by 8-lane groups, 64 entries (two 16-byte loads per lane) per step with
// the next queued segment's first step in flight.
__global__ __launch_bounds__(W_NT) void k_c4_window(C4Args A) {
  constexpr int WORDS = C4_WIN_WORDS;
  __shared__ uint32_t cnt[WORDS];
  __shared__ int32_t queue[W_BATCH];
  __shared__ int s_item, s_q;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const int g = tid / W_GL, gl = tid & (W_GL - 1);
  const int gshift = lane & ~(W_GL - 1);
  const uint64_t gmask = (1ull << W_GL) - 1;
  const int64_t b0 = A.start[A.bucket], cnt_items = A.start[A.bucket + 1] - b0;
  const int64_t hbase = b0 - A.start[CB_WIN16];
  const int4* __restrict__ ncol4 = reinterpret_cast<const int4*>(A.ncol);
  u128_t acc = 0;
  unsigned long long wedges = 0, owners = 0, segs = 0, visits = 0;
  // counters start at zero; every window clears the ones it used
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
    const int nl = (int)(A.seg_off[hbase + pos + 1] - so);
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
    const int64_t uwords = zone_words(A, u);
    if (tid == 0)
      visits += (unsigned long long)nl * (unsigned long long)((uwords + WORDS - 1) / WORDS);
    for (int64_t wlo = 0; wlo < uwords; wlo += WORDS) {
      const int64_t lo = zone_rank(A, wlo);
      const int64_t hnext = zone_rank(A, wlo + WORDS);
      const int32_t hi = (int32_t)(hnext < u ? hnext : u);
      for (int s0 = 0; s0 < nl; s0 += W_BATCH) {
        const int s1 = s0 + W_BATCH < nl ? s0 + W_BATCH : nl;
        if (tid == 0) s_q = 0;
        __syncthreads();
        // ---- whole segments per thread
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
              if (rdesc[j].z < hi) {
                if (rdesc[j].w < hi) {
                  D[sg] = rdesc[j];
                  queue[atomicAdd(&s_q, 1)] = sg;
                  stale |= 1u << j;
                } else {
                  wedges += short_visit(A, ncol4, cnt, rdesc[j], wlo, hi);
                }
              }
            }
          }
        } else {
          for (int sg = s0 + tid; sg < s1; sg += W_NT) {
            int4 d = D[sg];
            if (d.z >= hi) continue;  // nothing in this window
            if (d.w < hi) {           // 8 entries or more: queue it
              queue[atomicAdd(&s_q, 1)] = sg;
              continue;
            }
            wedges += short_visit(A, ncol4, cnt, d, wlo, hi);
            D[sg] = d;
          }
        }
        __syncthreads();
        // ---- queued long segments, one 8-lane group each: step k reads the
        // 64 entries [base + 64k, base + 64k + 64); lane gl holds entries
        // 4 gl .. 4 gl + 3 and 32 + 4 gl .. 32 + 4 gl + 3 of the step
        const int nq = s_q;
        int qi = g;
        int4 dA = qi < nq ? D[queue[qi]] : make_int4(0, 0, INT_MAX, INT_MAX);
        int64_t pA = (int64_t)dA.x & ~int64_t(63);  // first step, aligned to 64 entries
        int4 a0 = qi < nq ? ncol4[(pA >> 2) + gl] : make_int4(0, 0, 0, 0);
        int4 a1 = qi < nq ? ncol4[(pA >> 2) + 8 + gl] : make_int4(0, 0, 0, 0);
        while (qi < nq) {  // uniform in the group
          const int sg = queue[qi];
          const int qn = qi + W_NG;
          const int4 dB = qn < nq ? D[queue[qn]] : make_int4(0, 0, INT_MAX, INT_MAX);
          const int64_t pB = (int64_t)dB.x & ~int64_t(63);
          int4 b0v = qn < nq ? ncol4[(pB >> 2) + gl] : make_int4(0, 0, 0, 0);
          int4 b1v = qn < nq ? ncol4[(pB >> 2) + 8 + gl] : make_int4(0, 0, 0, 0);
          const int64_t c0 = dA.x, e = dA.y;
          int64_t p = pA;
          int64_t cend = c0;  // new cursor
          for (;;) {
            // the 8 entries of this lane in this step
            int32_t xs[8];
            xs[0] = a0.x; xs[1] = a0.y; xs[2] = a0.z; xs[3] = a0.w;
            xs[4] = a1.x; xs[5] = a1.y; xs[6] = a1.z; xs[7] = a1.w;
            int mine = 0;
#pragma unroll
            for (int r = 0; r < 8; r++) {
              const int64_t idx = p + (r < 4 ? 4 * gl + r : 32 + 4 * gl + (r - 4));
              const bool in = idx >= c0 && idx < e && xs[r] < hi;
              if (in) {
                window_inc(A, cnt, wlo, xs[r]);
                mine++;
              }
            }
            wedges += (unsigned long long)mine;
            // entries in the window form a run from the cursor: its length is
            // the group's total
            int tot = mine;
#pragma unroll
            for (int o = 1; o < W_GL; o <<= 1) tot += __shfl_xor(tot, o, WAVE);
            const int64_t first = p > c0 ? p : c0;
            cend = first + tot;
            if (cend < p + 64 || p + 64 >= e) break;  // the run ends in this step
            p += 64;
            a0 = ncol4[(p >> 2) + gl];
            a1 = ncol4[(p >> 2) + 8 + gl];
          }
          if (gl == 0)
            D[sg] = make_int4((int)cend, (int)e, row_at(A.ncol, cend, e), row_at(A.ncol, cend + 7, e));
          qi = qn;
          dA = dB;
          pA = pB;
          a0 = b0v;
          a1 = b1v;
        }
        __syncthreads();
      }
      window_close(A, cnt, wlo, (int)(uwords - wlo < WORDS ? uwords - wlo : WORDS), acc);
      __syncthreads();
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

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)ceil_div(n > 0 ? n : 1, nt); }

}  // namespace

void c4_run(const Prep& P, const Classes& C, Scal* scal, const Tuning& tu, uint32_t flags,
            Arena& tmp, hipStream_t s, int num_cu, KTimer* kt,
            const std::function<char*(size_t)>& big_scratch) {
  const int64_t n = P.n;
  if (n == 0 || P.m == 0) return;
  int64_t* wub = tmp.take<int64_t>(n);
  uint32_t* key = tmp.take<uint32_t>(n);
  int32_t* order = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, 2));
  int64_t* start = tmp.take<int64_t>(CB_N + 3);
  int32_t* hlen = tmp.take<int32_t>(n);
  int64_t* seg_off = tmp.take<int64_t>(n + 1);
  int64_t* stmp = tmp.take<int64_t>(scan_tmp_elems(n));
  int32_t* lowcut = tmp.take<int32_t>(n);
  if (!wub || !key || !order || !rtmp || !start || !hlen || !seg_off || !stmp || !lowcut)
    throw Fail(M4_EINTERNAL, "workspace too small (c4)");
  fill_u32(&scal->work[0], 0, 8, s);
  const int light = tu.c4_light_max;
  // rows by degree: <= 64 with 8 lanes, <= 4096 with a wavefront, longer
  // rows with a workgroup
  const int64_t b64 = C.bound[4], b4096 = C.bound[7];
  if (kt) kt->begin(M4_K_C4_PLAN, s);
  if (b64 > 0)
    k_c4_plan<8><<<blocks_for(b64 * 8, 256), 256, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, 0, b64,
                                                          C.r1, light, wub, key, P.own_lo, P.hi());
  if (b4096 > b64)
    k_c4_plan<64><<<blocks_for((b4096 - b64) * 64, 256), 256, 0, s>>>(
        P.nptr, P.ncol, P.dr, P.dlo, b64, b4096, C.r1, light, wub, key, P.own_lo, P.hi());
  if (n > b4096)
    k_c4_plan_big<<<(unsigned)(n - b4096), 1024, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, b4096, C.r1,
                                                         light, wub, key, P.own_lo, P.hi());
  radix_pass(key, nullptr, n, 0, 2, nullptr, order, rtmp, start, s);
  k_zone_bounds<<<1, 64, 0, s>>>(P.dr, n, start + CB_N + 1);
  int64_t hstart[CB_N + 3];
  M4_HIP(hipMemcpyAsync(hstart, start, sizeof(hstart), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  // counter zones of the window owners
  const int64_t z1 = std::max<int64_t>(hstart[CB_N + 1], C.r1);
  const int64_t z2 = std::max<int64_t>(hstart[CB_N + 2], z1);
  const int64_t aw = (z1 - C.r1 + 7) >> 3, bw = (z2 - z1 + 3) >> 2;
  const int64_t H = hstart[CB_WIN32 + 1] - hstart[CB_WIN16];
  int4* desc = nullptr;
  if (H > 0) {
    k_c4_heavy_len<<<blocks_for(H, 256), 256, 0, s>>>(order, start, P.dlo, hlen);
    scan_i32(hlen, H, seg_off, stmp, s);
    int64_t nseg = 0;
    M4_HIP(hipMemcpyAsync(&nseg, seg_off + H, 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    desc = reinterpret_cast<int4*>(big_scratch((size_t)(nseg > 0 ? nseg : 1) * sizeof(int4)));
    if (!desc) throw Fail(M4_ENOMEM, "no room for 4-cycle segment descriptors");
    // with stored prefixes only the partition's rows are valid: no full pass
    if (!P.row_len)
      k_lowcut<<<blocks_for(n, 256), 256, 0, s>>>(P.nptr, P.ncol, P.row_len, n, C.r1, lowcut);
    k_c4_desc<<<(unsigned)H, 256, 0, s>>>(order, start, seg_off, P.nptr, P.dlo, P.ncol,
                                          P.row_len ? nullptr : lowcut, P.row_len, C.r1, desc);
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
  A.z1 = z1;
  A.z2 = z2;
  A.aw = aw;
  A.bw = bw;
  // heavy owners first: one 1024-thread workgroup per CU
  if (hstart[CB_WIN16 + 1] > hstart[CB_WIN16]) {
    A.bucket = CB_WIN16;
    A.slot = M4_K_C4_WIN16;
    A.work = &scal->work[CB_WIN16];
    if (kt) kt->begin(M4_K_C4_WIN16, s);
    k_c4_window<<<(unsigned)num_cu, W_NT, 0, s>>>(A);
    if (kt) kt->end(M4_K_C4_WIN16, s);
  }
  if (hstart[CB_HASH + 1] > hstart[CB_HASH]) {
    A.bucket = CB_HASH;
    A.slot = M4_K_C4_HASH;
    A.work = &scal->work[CB_HASH];
    if (kt) kt->begin(M4_K_C4_HASH, s);
    k_c4_hash<<<(unsigned)(num_cu * 4), H_NT, 0, s>>>(A);
    if (kt) kt->end(M4_K_C4_HASH, s);
  }
}

}  // namespace m4
