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
//                    LDS over windows of 64K ranks (16-bit counters while
//                    |L(u)| < 65536, else 32K ranks of 32-bit counters);
//                    every lower neighbour keeps a cursor into its sorted row
//                    so each window reads exactly its own endpoints.
#include <limits.h>

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
  int64_t r1;
  int bucket;
  int slot;
  unsigned int* work;
  Scal* scal;
  uint32_t flags;
  int32_t* cur;  // per-block cursor scratch (window bucket)
  int32_t* end;
  int64_t seg_cap;
};

// wedge bound of every owner: G lanes cooperate on one row, 4 loads in flight
template <int G>
__global__ __launch_bounds__(256) void k_c4_plan(const int64_t* __restrict__ nptr,
                                                 const int32_t* __restrict__ ncol,
                                                 const int32_t* __restrict__ dr,
                                                 const int32_t* __restrict__ dlo, int64_t r_lo,
                                                 int64_t r_hi, int64_t r1, int light_max,
                                                 int64_t* __restrict__ wub,
                                                 uint32_t* __restrict__ key) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t u = r_lo + t / G;
  int j = (int)(t % G);
  bool ok = u < r_hi;
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
      else if (nl < 65535) k = CB_WIN16;
      else k = CB_WIN32;
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
                                                      uint32_t* __restrict__ key) {
  int64_t u = r_lo + blockIdx.x;
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
      else if (nl < 65535) k = CB_WIN16;
      else k = CB_WIN32;
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
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt) break;
    const int32_t u = A.order[b0 + item];
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
        len = A.dr[v];
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
constexpr int W_NT = 1024, W_GROUP = 16, W_GROUPS = W_NT / W_GROUP;

template <bool NARROW>
__global__ __launch_bounds__(W_NT) void k_c4_window(C4Args A) {
  constexpr int WIN = NARROW ? C4_WIN16 : C4_WIN32;
  constexpr int WORDS = NARROW ? WIN / 2 : WIN;
  __shared__ uint32_t cnt[WORDS];
  __shared__ int s_item;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const int g = tid / W_GROUP, gl = tid & (W_GROUP - 1);
  const int gshift = lane & ~(W_GROUP - 1);
  const int64_t b0 = A.start[A.bucket], cnt_items = A.start[A.bucket + 1] - b0;
  int32_t* cur = A.cur + (int64_t)blockIdx.x * A.seg_cap;
  int32_t* end = A.end + (int64_t)blockIdx.x * A.seg_cap;
  u128_t acc = 0;
  unsigned long long wedges = 0, owners = 0, segs = 0, visits = 0;
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt_items) break;
    // heaviest owners (highest ranks) first
    const int32_t u = A.order[b0 + cnt_items - 1 - item];
    const int nl = A.dlo[u];
    const int64_t base = A.nptr[u];
    if (tid == 0) {
      owners++;
      segs += (unsigned long long)nl;
      visits += (unsigned long long)nl * (unsigned long long)((u - A.r1 + WIN - 1) / WIN);
    }
    for (int i = tid; i < nl; i += W_NT) {
      int32_t v = A.ncol[base + i];
      int64_t rs = A.nptr[v];
      int64_t e = lower_index(A.ncol, rs + A.dlo[v], A.nptr[v + 1], u);  // position of u
      int64_t c = lower_index(A.ncol, rs, e, (int32_t)A.r1);
      cur[i] = (int32_t)c;
      end[i] = (int32_t)e;
    }
    __syncthreads();
    for (int64_t lo = A.r1; lo < u; lo += WIN) {
      const int64_t hi = lo + WIN < u ? lo + WIN : u;
      for (int i = tid; i < WORDS; i += W_NT) cnt[i] = 0;
      __syncthreads();
      for (int sgi = g; sgi < nl; sgi += W_GROUPS) {
        int32_t c = cur[sgi];
        const int32_t e = end[sgi];
        for (;;) {
          const int32_t idx = c + gl;
          const int32_t w = idx < e ? A.ncol[idx] : INT_MAX;
          const bool in = w < hi;
          if (in) {
            const uint32_t o = (uint32_t)(w - lo);
            if (NARROW) {
              const uint32_t sh = (o & 1u) << 4;
              const uint32_t old = atomicAdd(&cnt[o >> 1], 1u << sh);
              acc += (old >> sh) & 0xffffu;
            } else {
              acc += atomicAdd(&cnt[o], 1u);
            }
            wedges++;
          }
          const uint64_t bal = (__ballot(in) >> gshift) & ((1ull << W_GROUP) - 1);
          const int nin = __popcll(bal);
          c += nin;
          if (nin < W_GROUP) break;
        }
        if (gl == 0) cur[sgi] = c;
      }
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
            Arena& tmp, hipStream_t s, int num_cu, KTimer* kt) {
  const int64_t n = P.n;
  if (n == 0 || P.m == 0) return;
  int64_t* wub = tmp.take<int64_t>(n);
  uint32_t* key = tmp.take<uint32_t>(n);
  int32_t* order = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, 2));
  int64_t* start = tmp.take<int64_t>(8);
  const int64_t seg_cap = C.dmax > 0 ? C.dmax : 1;
  int32_t* cur = tmp.take<int32_t>((size_t)seg_cap * num_cu);
  int32_t* end = tmp.take<int32_t>((size_t)seg_cap * num_cu);
  if (!wub || !key || !order || !rtmp || !start || !cur || !end)
    throw Fail(M4_EINTERNAL, "workspace too small (c4)");
  fill_u32(&scal->work[0], 0, 8, s);
  const int light = tu.c4_light_max;
  // rows by degree: <= 64 with 8 lanes, <= 4096 with a wavefront, longer
  // rows with a workgroup
  const int64_t b64 = C.bound[4], b4096 = C.bound[7];
  if (kt) kt->begin(M4_K_C4_PLAN, s);
  if (b64 > 0)
    k_c4_plan<8><<<blocks_for(b64 * 8, 256), 256, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, 0, b64,
                                                          C.r1, light, wub, key);
  if (b4096 > b64)
    k_c4_plan<64><<<blocks_for((b4096 - b64) * 64, 256), 256, 0, s>>>(
        P.nptr, P.ncol, P.dr, P.dlo, b64, b4096, C.r1, light, wub, key);
  if (n > b4096)
    k_c4_plan_big<<<(unsigned)(n - b4096), 1024, 0, s>>>(P.nptr, P.ncol, P.dr, P.dlo, b4096, C.r1,
                                                         light, wub, key);
  radix_pass(key, nullptr, n, 0, 2, nullptr, order, rtmp, start, s);
  if (kt) kt->end(M4_K_C4_PLAN, s);

  C4Args A{};
  A.order = order;
  A.start = start;
  A.nptr = P.nptr;
  A.ncol = P.ncol;
  A.dr = P.dr;
  A.dlo = P.dlo;
  A.wub = wub;
  A.r1 = C.r1;
  A.scal = scal;
  A.flags = flags;
  A.cur = cur;
  A.end = end;
  A.seg_cap = seg_cap;
  // heavy owners first: one 1024-thread workgroup per CU
  A.bucket = CB_WIN16;
  A.slot = M4_K_C4_WIN16;
  A.work = &scal->work[CB_WIN16];
  if (kt) kt->begin(M4_K_C4_WIN16, s);
  k_c4_window<true><<<(unsigned)num_cu, W_NT, 0, s>>>(A);
  if (kt) kt->end(M4_K_C4_WIN16, s);
  A.bucket = CB_WIN32;
  A.slot = M4_K_C4_WIN32;
  A.work = &scal->work[CB_WIN32];
  if (kt) kt->begin(M4_K_C4_WIN32, s);
  k_c4_window<false><<<(unsigned)num_cu, W_NT, 0, s>>>(A);
  if (kt) kt->end(M4_K_C4_WIN32, s);
  A.bucket = CB_HASH;
  A.slot = M4_K_C4_HASH;
  A.work = &scal->work[CB_HASH];
  if (kt) kt->begin(M4_K_C4_HASH, s);
  k_c4_hash<<<(unsigned)(num_cu * 4), H_NT, 0, s>>>(A);
  if (kt) kt->end(M4_K_C4_HASH, s);
}

}  // namespace m4
