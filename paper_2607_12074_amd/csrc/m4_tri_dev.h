// m4_tri_dev.h -- device routine of the triangle / 4-clique anchor for one
// owner, shared by the single-graph kernels and the batched kernel.
#pragma once
#include "m4_device.h"

namespace m4 {

// signature of a cached frontier: (j, slot, required-adjacency mask,
// required-non-adjacency mask); a lookup matches only on all four fields.
__host__ __device__ __forceinline__ uint32_t sig_key(uint32_t j, uint32_t slot, uint32_t mplus,
                                                     uint32_t mminus) {
  return (j << 28) | ((mplus & 0xfu) << 24) | ((mminus & 0xfu) << 20) | (slot & 0xfffffu);
}

struct TriArgs {
  const int32_t* order;   // owners sorted by bucket
  const int64_t* start;   // bucket ranges (device, in Scal)
  const int64_t* nptr;
  const int64_t* optr;
  const int32_t* ncol;
  const int32_t* dlo;
  const int32_t* dplus;
  uint32_t* t;
  Scal* scal;
  uint32_t flags;
  uint32_t cache_rows;
  int bucket;
  int slot;  // kernel slot of the work counters
  int grab;  // owners taken per atomic on the work counter
  unsigned int* work;     // atomic owner counter for this bucket
  // global-bitmap variant scratch (per block), sized for kmax
  int kmax;
  uint64_t* gbits;
  int32_t* garr;
  // hub tables: open-addressing tables of the out-lists of vertices with
  // out-degree >= hub_min (entry = key << 32 | position, empty = ~0)
  const int32_t* hoff;    // table offset per vertex, -1 without a table
  const unsigned long long* htab;
  int hub_min;            // 0: no tables
  int probe_w;            // row i is probed when probe_w (k-1-i) < 3 |N+(a[i])|
  // bit ERR_PROBE is set here when a probe sequence runs past its table size
  // (a broken table invariant); the probe then stops instead of spinning
  int* err;
};

constexpr unsigned long long HUB_EMPTY = ~0ull;

// log2 of the slots of the table of a vertex with out-degree L >= 1: the
// power of two >= 2L (load factor <= 1/2).
__host__ __device__ __forceinline__ int hub_bits(int L) { return 32 - __builtin_clz(2u * L - 1u); }

__device__ __forceinline__ uint32_t hub_hash(int32_t x, int bits) {
  return ((uint32_t)x * 0x9E3779B1u) >> (32 - bits);
}

template <typename T>
__device__ __forceinline__ T ld(const T* p, bool fresh) {
  if (fresh) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

// |C(u, a[i]) & N+(a[p])| recomputed from the lists, for frontiers that are
// not held in the signature cache.
__device__ __forceinline__ uint64_t k4_recompute(const int32_t* ncol, const int32_t* a, int k,
                                                 int p, int64_t si, int li, int64_t sp, int lp) {
  uint64_t c = 0;
  for (int jj = 0; jj < lp; jj++) {
    int32_t x = ncol[sp + jj];
    int64_t q = lower_index(a, (int64_t)p + 1, (int64_t)k, x);
    if (q >= k || a[q] != x) continue;
    int64_t r = lower_index(ncol, si, si + li, x);
    if (r < si + li && ncol[r] == x) c++;
  }
  return c;
}

#define TRI_SYNC()                \
  do {                            \
    if (WAVE_ONLY) wave_sync();   \
    else __syncthreads();         \
  } while (0)

// One owner processed by NT threads with per-owner arrays in `a..colcnt`
// (LDS or global) and bitmap rows of W words each in `B`.
// HASH: positions of the out-list are found through an LDS hash table
// (hk/hv, 2H >= 2k slots) instead of a binary search over a[].
// PROBE: a row i whose head v = a[i] has a hub table is resolved by probing
// that table for the later entries a[i+1..k) when that is cheaper than
// scanning N+(v): k-1-i probes, each weighted probe_w / 3 scanned elements
// (4/3 reads per probe at load 1/2; larger weights account for a probe
// fetching a whole cache line where a scan streams 4 bytes); the table
// returns the position of the hit in N+(v), which indexes the far edge's
// triangle count.  Both ways find the same triangles.
// Work counters: steps (elements looked up or probed), looks/hits (frontier
// cache), ksum (out-list entries of the owner), escan (sum of |N+(v)| over the
// owner's out-neighbours v, the elements a scanning intersection reads),
// wread (4-byte words this routine reads from the out-lists and hub tables:
// one per scanned element, two per 8-byte table slot probed).
template <int NT, bool FRESH, bool WAVE_ONLY = false, bool HASH = false, bool PROBE = false>
__device__ __forceinline__ void tri_owner(const TriArgs& A, int32_t u, const int tid, int32_t* a,
                                          int32_t* sst,
                                          int32_t* soe, int32_t* slen, int32_t* spref,
                                          uint32_t* colcnt, uint32_t* tag, uint64_t* B,
                                          u128_t& k4acc,
                                          unsigned long long& steps, unsigned long long& looks,
                                          unsigned long long& hits, unsigned long long& ksum,
                                          unsigned long long& wread,
                                          unsigned long long& escan, int32_t* hk = nullptr,
                                          int16_t* hv = nullptr) {
  const int k = A.dplus[u];
  const int64_t rb = A.nptr[u] + A.dlo[u];
  const int64_t oe_u = A.optr[u];
  const int W = (k + 63) >> 6;
  if (tid == 0) ksum += (unsigned long long)k;
  for (int i = tid; i < k; i += NT) {
    int32_t v = A.ncol[rb + i];
    a[i] = v;
    const int L = A.dplus[v];
    int32_t st = (int32_t)(A.nptr[v] + A.dlo[v]);
    if (PROBE && A.hub_min > 0 && L >= A.hub_min && A.probe_w * (k - 1 - i) < 3 * L) {
      const int32_t off = A.hoff[v];
      if (off >= 0) st = -1 - off;  // probe row: table offset, negated
    }
    sst[i] = st;
    soe[i] = (int32_t)A.optr[v];
    slen[i] = L;
    colcnt[i] = 0;
  }
  for (int i = tid; i < k * W; i += NT) B[i] = 0;
  int H = 16, hshift = 28;
  if (HASH) {
    while (H < 2 * k) {
      H <<= 1;
      hshift--;
    }
    for (int i = tid; i < H; i += NT) hk[i] = -1;
  }
  TRI_SYNC();
  if (HASH) {
    // k distinct keys in H >= 2k slots: a free slot is met within H probes
    for (int i = tid; i < k; i += NT) {
      const int32_t key = a[i];
      uint32_t h = ((uint32_t)key * 0x9E3779B1u) >> hshift;
      int probes = 0;
      while (atomicCAS(&hk[h], -1, key) != -1) {
        h = (h + 1) & (uint32_t)(H - 1);
        if (++probes >= H) {
          atomicOr(A.err, ERR_PROBE);
          break;
        }
      }
      if (probes < H) hv[h] = (int16_t)i;
    }
  }
  // exclusive prefix of the row work of a[0..k) into spref[0..k]: |N+(a[i])|
  // elements for a scanned row, k-1-i probes for a probed row
  {
    const int per = (k + NT - 1) / NT;
    const int lo = tid * per;
    int64_t s = 0;
    for (int i = lo; i < lo + per && i < k; i++) {
      s += (PROBE && sst[i] < 0) ? (k - 1 - i) : slen[i];
      escan += (unsigned long long)slen[i];
    }
    int64_t tot;
    int64_t run = block_excl_scan64<NT>(s, &tot);
    for (int i = lo; i < lo + per && i < k; i++) {
      spref[i] = (int32_t)run;
      run += (PROBE && sst[i] < 0) ? (k - 1 - i) : slen[i];
    }
    if (tid == 0) spref[k] = (int32_t)tot;
  }
  TRI_SYNC();
  const int total = spref[k];
  // Flattened (row, element) pairs: thread tid takes q = tid, tid + NT, ...;
  // the row index only moves forward, and four element loads (or first
  // probes) are issued before the four lookups so that their latencies
  // overlap.
  int i = tid < total ? upper_index(spref, k, tid) : 0;
  int ii[4], jj[4];
  int32_t xx[4];
  uint32_t hh[4];
  unsigned long long ee[4];
  auto fetch = [&](int q0) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int q = q0 + r * NT;
      ii[r] = -1;
      if (q < total) {
        while (spref[i + 1] <= q) i++;
        ii[r] = i;
        jj[r] = q - spref[i];
        const int32_t st = sst[i];
        if (PROBE && st < 0) {
          const int32_t x = a[i + 1 + jj[r]];
          const uint32_t h = hub_hash(x, hub_bits(slen[i]));
          xx[r] = x;
          hh[r] = h;
          ee[r] = A.htab[(int64_t)(-1 - st) + h];
        } else {
          xx[r] = A.ncol[st + jj[r]];
        }
      }
    }
  };
  fetch(tid);
  for (int q0 = tid; q0 < total; q0 += 4 * NT) {
    int ci[4], cj[4];
    int32_t cx[4];
    uint32_t ch[4];
    unsigned long long ce[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      ci[r] = ii[r];
      cj[r] = jj[r];
      cx[r] = xx[r];
      ch[r] = hh[r];
      ce[r] = ee[r];
    }
    if (q0 + 4 * NT < total) fetch(q0 + 4 * NT);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      if (ci[r] < 0) continue;
      const int ir = ci[r];
      const int32_t x = cx[r];
      int p, pos;
      if (PROBE && sst[ir] < 0) {
        // x = a[p] looked up in the table of a[ir]
        p = ir + 1 + cj[r];
        const int64_t off = -1 - (int64_t)sst[ir];
        const uint32_t mask = (1u << hub_bits(slen[ir])) - 1u;
        uint32_t h = ch[r];
        unsigned long long e = ce[r];
        pos = -1;
        wread += 2;
        // load <= 1/2: an empty slot ends every probe within mask + 1 steps
        for (uint32_t probes = 0; e != HUB_EMPTY; probes++) {
          if ((int32_t)(e >> 32) == x) {
            pos = (int)(uint32_t)e;
            break;
          }
          if (probes >= mask) {
            atomicOr(A.err, ERR_PROBE);
            break;
          }
          h = (h + 1) & mask;
          e = A.htab[off + h];
          wread += 2;
        }
        if (pos < 0) p = -1;
      } else if (HASH) {
        // x > a[ir], so a hit is always a position after ir
        pos = cj[r];
        wread++;
        uint32_t h = ((uint32_t)x * 0x9E3779B1u) >> hshift;
        p = -1;
        for (int probes = 0;; probes++) {
          const int32_t key = hk[h];
          if (key == x) {
            p = hv[h];
            break;
          }
          if (key == -1) break;
          if (probes >= H) {
            atomicOr(A.err, ERR_PROBE);
            break;
          }
          h = (h + 1) & (uint32_t)(H - 1);
        }
      } else {
        pos = cj[r];
        wread++;
        p = (int)lower_index(a, (int64_t)ir + 1, (int64_t)k, x);
        if (p >= k || a[p] != x) p = -1;
      }
      steps++;
      if (p >= 0) {
        atomicOr((unsigned long long*)&B[ir * W + (p >> 6)], 1ull << (p & 63));
        atomicAdd(&colcnt[p], 1u);
        atomicAdd(&A.t[soe[ir] + pos], 1u);
      }
    }
  }
  TRI_SYNC();
  // triangles on the owner's own out-edges: (u, a[i], *) and (u, *, a[i])
  for (int i = tid; i < k; i += NT) {
    uint32_t rc = 0;
    for (int w = 0; w < W; w++) rc += __popcll(ld(&B[i * W + w], FRESH));
    uint32_t c = rc + ld(&colcnt[i], FRESH);
    if (c) atomicAdd(&A.t[oe_u + i], c);
  }
  // The rows that fit the cache capacity are published with their signature
  // (j = 2, slot i, adjacency to both embedded vertices required, no
  // non-adjacency); other rows stay unpublished and are recomputed.
  const bool cache_on = !(A.flags & M4_NO_CACHE);
  const uint32_t cap = A.cache_rows ? A.cache_rows : 0xffffffffu;
  for (int i = tid; i < k; i += NT)
    tag[i] = (cache_on && (uint32_t)i < cap) ? sig_key(2, (uint32_t)i, 3, 0) : 0u;
  TRI_SYNC();
  // 4-cliques: for every triangle (u, a[i], a[p]) intersect the two frontiers
  for (int i = tid; i < k; i += NT) {
    const bool ci = tag[i] == sig_key(2, (uint32_t)i, 3, 0);
    for (int w = 0; w < W; w++) {
      uint64_t bits = ld(&B[i * W + w], FRESH);
      while (bits) {
        int p = (w << 6) + __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        looks++;
        const bool cp = tag[p] == sig_key(2, (uint32_t)p, 3, 0);
        if (ci && cp) {
          hits++;
          uint64_t c = 0;
          for (int ww = p >> 6; ww < W; ww++)
            c += __popcll(ld(&B[i * W + ww], FRESH) & ld(&B[p * W + ww], FRESH));
          k4acc += c;
        } else {
          // probed rows keep a table offset in sst[]: take the list start again
          const int64_t si = (PROBE && sst[i] < 0) ? A.nptr[a[i]] + A.dlo[a[i]] : sst[i];
          const int64_t sp = (PROBE && sst[p] < 0) ? A.nptr[a[p]] + A.dlo[a[p]] : sst[p];
          k4acc += k4_recompute(A.ncol, a, k, p, si, slen[i], sp, slen[p]);
        }
      }
    }
  }
  TRI_SYNC();
}


}  // namespace m4
