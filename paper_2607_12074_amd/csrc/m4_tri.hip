// m4_tri.hip -- triangle and 4-clique anchors (per-edge t_e, K4).
//
// Owner rule: a triangle u<v<w and a 4-clique u<v<w<x (rank order) belong to
// their lowest vertex u.  For an owner u with out-list a = N+(u) (k entries,
// sorted) the kernel builds the induced subgraph of G on a as k bitmap rows:
// bit p of row i is set iff a[p] is in N+(a[i]).  Row i is the candidate
// frontier C(u, a[i]) = N+(u) & N+(a[i]) of the partial embedding (u, a[i]):
// every set bit is a triangle (u, a[i], a[p]), and the frontier is reused by
// every triangle that extends it to a 4-clique, |C(u,a[i]) & C(u,a[p])|
// (induced-signature reuse, Section III-C; the stored state has j = 2 and
// requires adjacency to both embedded vertices, no non-adjacency).
//
// Rows are filled by ordered set intersection (Section III-D): every element
// x of N+(a[i]) is looked up by binary search in a[i+1..k).  Owners are split
// by k: one wavefront (k <= 64, one 64-bit word per row), one workgroup with
// the bitmap in LDS (k <= 1024), or one workgroup with the bitmap in global
// scratch (larger k).  Block-local sums are folded into one 128-bit atomic
// per workgroup (block-local aggregation).
#include <limits.h>

#include "m4_device.h"

namespace m4 {

namespace {

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
  unsigned int* work;     // atomic owner counter for this bucket
  // global-bitmap variant scratch (per block), sized for kmax
  int kmax;
  uint64_t* gbits;
  int32_t* garr;
};

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

// One owner processed by NT threads with per-owner arrays in `a..colcnt`
// (LDS or global) and bitmap rows of W words each in `B`.
template <int NT, bool FRESH>
__device__ __forceinline__ void tri_owner(const TriArgs& A, int32_t u, int32_t* a, int32_t* sst,
                                          int32_t* soe, int32_t* slen, int32_t* spref,
                                          uint32_t* colcnt, uint32_t* tag, uint64_t* B,
                                          u128_t& k4acc,
                                          unsigned long long& steps, unsigned long long& looks,
                                          unsigned long long& hits, unsigned long long& ksum,
                                          unsigned long long& tris) {
  const int tid = threadIdx.x;
  const int k = A.dplus[u];
  const int64_t rb = A.nptr[u] + A.dlo[u];
  const int64_t oe_u = A.optr[u];
  const int W = (k + 63) >> 6;
  if (tid == 0) ksum += (unsigned long long)k;
  for (int i = tid; i < k; i += NT) {
    int32_t v = A.ncol[rb + i];
    a[i] = v;
    sst[i] = (int32_t)(A.nptr[v] + A.dlo[v]);
    soe[i] = (int32_t)A.optr[v];
    slen[i] = A.dplus[v];
    colcnt[i] = 0;
  }
  for (int i = tid; i < k * W; i += NT) B[i] = 0;
  __syncthreads();
  // exclusive prefix of the out-degrees of a[0..k) into spref[0..k]
  {
    const int per = (k + NT - 1) / NT;
    const int lo = tid * per;
    int64_t s = 0;
    for (int i = lo; i < lo + per && i < k; i++) s += slen[i];
    int64_t tot;
    int64_t run = block_excl_scan64<NT>(s, &tot);
    for (int i = lo; i < lo + per && i < k; i++) {
      spref[i] = (int32_t)run;
      run += slen[i];
    }
    if (tid == 0) spref[k] = (int32_t)tot;
  }
  __syncthreads();
  const int total = spref[k];
  for (int q = tid; q < total; q += NT) {
    int i = upper_index(spref, k, q);
    int j = q - spref[i];
    int32_t x = A.ncol[sst[i] + j];
    int p = (int)lower_index(a, (int64_t)i + 1, (int64_t)k, x);
    steps++;
    if (p < k && a[p] == x) {
      atomicOr((unsigned long long*)&B[i * W + (p >> 6)], 1ull << (p & 63));
      atomicAdd(&colcnt[p], 1u);
      atomicAdd(&A.t[soe[i] + j], 1u);
    }
  }
  __syncthreads();
  // triangles on the owner's own out-edges: (u, a[i], *) and (u, *, a[i])
  for (int i = tid; i < k; i += NT) {
    uint32_t rc = 0;
    for (int w = 0; w < W; w++) rc += __popcll(ld(&B[i * W + w], FRESH));
    uint32_t c = rc + ld(&colcnt[i], FRESH);
    tris += rc;
    if (c) atomicAdd(&A.t[oe_u + i], c);
  }
  // The rows that fit the cache capacity are published with their signature
  // (j = 2, slot i, adjacency to both embedded vertices required, no
  // non-adjacency); other rows stay unpublished and are recomputed.
  const bool cache_on = !(A.flags & M4_NO_CACHE);
  const uint32_t cap = A.cache_rows ? A.cache_rows : 0xffffffffu;
  for (int i = tid; i < k; i += NT)
    tag[i] = (cache_on && (uint32_t)i < cap) ? sig_key(2, (uint32_t)i, 3, 0) : 0u;
  __syncthreads();
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
          k4acc += k4_recompute(A.ncol, a, k, p, sst[i], slen[i], sst[p], slen[p]);
        }
      }
    }
  }
  __syncthreads();
}

template <int KMAX, int NT>
__global__ __launch_bounds__(NT) void k_tri_lds(TriArgs A) {
  constexpr int WMAX = (KMAX + 63) / 64;
  __shared__ int32_t a[KMAX], sst[KMAX], soe[KMAX], slen[KMAX], spref[KMAX + 1];
  __shared__ uint32_t colcnt[KMAX], tag[KMAX];
  __shared__ uint64_t B[KMAX * WMAX];
  __shared__ int s_item;
  const int64_t b0 = A.start[A.bucket], cnt = A.start[A.bucket + 1] - b0;
  u128_t k4 = 0;
  unsigned long long steps = 0, looks = 0, hits = 0, ksum = 0, tris = 0, owners = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt) break;
    tri_owner<NT, false>(A, A.order[b0 + item], a, sst, soe, slen, spref, colcnt, tag, B, k4,
                         steps, looks, hits, ksum, tris);
    owners++;
  }
  block_add_u128<NT>(&A.scal->acc[ACC_K4], k4);
  if (A.flags & M4_STATS) {
    block_add_u64<NT>(&A.scal->stat[ST_STEPS], steps);
    block_add_u64<NT>(&A.scal->stat[ST_LOOKUPS], looks);
    block_add_u64<NT>(&A.scal->stat[ST_HITS], hits);
    block_add_u64<NT>(&A.scal->kstat[A.slot][0], steps);
    block_add_u64<NT>(&A.scal->kstat[A.slot][1], threadIdx.x == 0 ? owners : 0);
    block_add_u64<NT>(&A.scal->kstat[A.slot][2], ksum);
    block_add_u64<NT>(&A.scal->kstat[A.slot][3], tris);
  }
}

// Owners whose bitmap does not fit in LDS: the same algorithm over a
// per-block slice of global scratch (atomic loads read past the L1).
template <int NT>
__global__ __launch_bounds__(NT) void k_tri_global(TriArgs A) {
  __shared__ int s_item;
  const int64_t b0 = A.start[A.bucket], cnt = A.start[A.bucket + 1] - b0;
  const int64_t K = A.kmax, WK = (K + 63) / 64;
  uint64_t* B = A.gbits + (int64_t)blockIdx.x * K * WK;
  int32_t* base = A.garr + (int64_t)blockIdx.x * (7 * K + 2);
  int32_t *a = base, *sst = base + K, *soe = base + 2 * K, *slen = base + 3 * K;
  int32_t* spref = base + 4 * K;
  uint32_t* colcnt = (uint32_t*)(base + 5 * K + 1);
  uint32_t* tag = (uint32_t*)(base + 6 * K + 1);
  u128_t k4 = 0;
  unsigned long long steps = 0, looks = 0, hits = 0, ksum = 0, tris = 0, owners = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt) break;
    tri_owner<NT, true>(A, A.order[b0 + item], a, sst, soe, slen, spref, colcnt, tag, B, k4,
                        steps, looks, hits, ksum, tris);
    owners++;
    __threadfence();
  }
  block_add_u128<NT>(&A.scal->acc[ACC_K4], k4);
  if (A.flags & M4_STATS) {
    block_add_u64<NT>(&A.scal->stat[ST_STEPS], steps);
    block_add_u64<NT>(&A.scal->stat[ST_LOOKUPS], looks);
    block_add_u64<NT>(&A.scal->stat[ST_HITS], hits);
    block_add_u64<NT>(&A.scal->kstat[A.slot][0], steps);
    block_add_u64<NT>(&A.scal->kstat[A.slot][1], threadIdx.x == 0 ? owners : 0);
    block_add_u64<NT>(&A.scal->kstat[A.slot][2], ksum);
    block_add_u64<NT>(&A.scal->kstat[A.slot][3], tris);
  }
}

// bucket of every owner by its out-degree k
enum { TK_NONE = 0, TK_WAVE, TK_128, TK_256, TK_512, TK_1024, TK_GLOBAL, TK_N };

__global__ void k_tri_keys(const int32_t* __restrict__ dplus, int64_t n, int wave_max,
                           uint32_t* __restrict__ key, Scal* scal) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int k = dplus[u];
  uint32_t b;
  if (k < 2) b = TK_NONE;
  else if (k <= wave_max) b = TK_WAVE;
  else if (k <= 128) b = TK_128;
  else if (k <= 256) b = TK_256;
  else if (k <= 512) b = TK_512;
  else if (k <= TRI_LDS_MAX) b = TK_1024;
  else {
    b = TK_GLOBAL;
    atomicMax((unsigned int*)&scal->work[7], (unsigned int)k);
  }
  key[u] = b;
}

}  // namespace

// host-side replica of the signature key, for tests of its distinctness
extern "C" uint32_t m4_internal_sig_key(uint32_t j, uint32_t slot, uint32_t mplus, uint32_t mminus) {
  return sig_key(j, slot, mplus, mminus);
}

size_t tri_tmp_bytes(int64_t n, int64_t nnz, int kmax_global) {
  (void)nnz;
  return (size_t)n * 8 + radix_tmp_elems(n, 4) * 8 + 16 * 8 + 8192 +
         (size_t)(kmax_global > 0 ? 64 : 0) *
             ((size_t)kmax_global * ((kmax_global + 63) / 64) * 8 + (7 * (size_t)kmax_global + 2) * 4);
}

void tri_run(const Prep& P, Scal* scal, const Tuning& tu, uint32_t flags, uint32_t cache_rows,
             Arena& tmp, hipStream_t s, int num_cu,
             const std::function<char*(size_t)>& big_scratch, KTimer* kt) {
  const int64_t n = P.n;
  if (n == 0 || P.m == 0) return;
  uint32_t* key = tmp.take<uint32_t>(n);
  int32_t* order = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, 4));
  int64_t* start = tmp.take<int64_t>(17);
  if (!key || !order || !rtmp || !start) throw Fail(M4_EINTERNAL, "workspace too small (tri)");
  fill_u32(&scal->work[0], 0, 8, s);
  int wave_max = tu.tri_wave_max < 2 ? 2 : (tu.tri_wave_max > 64 ? 64 : tu.tri_wave_max);
  k_tri_keys<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(P.dplus, n, wave_max, key, scal);
  radix_pass(key, nullptr, n, 0, 4, nullptr, order, rtmp, start, s);
  // largest out-degree of the global bucket decides its scratch size
  unsigned int kmax_g = 0;
  int64_t hstart[17];
  M4_HIP(hipMemcpyAsync(&kmax_g, &scal->work[7], sizeof(kmax_g), hipMemcpyDeviceToHost, s));
  M4_HIP(hipMemcpyAsync(hstart, start, sizeof(hstart), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));

  TriArgs A{};
  A.order = order;
  A.start = start;
  A.nptr = P.nptr;
  A.optr = P.optr;
  A.ncol = P.ncol;
  A.dlo = P.dlo;
  A.dplus = P.dplus;
  A.t = P.t;
  A.scal = scal;
  A.flags = flags;
  A.cache_rows = cache_rows;

  auto run_lds = [&](auto kmax_tag, auto nt_tag, int bucket, int slot, int blocks_per_cu) {
    constexpr int KM = decltype(kmax_tag)::value;
    constexpr int NT = decltype(nt_tag)::value;
    if (hstart[bucket + 1] == hstart[bucket]) return;
    A.bucket = bucket;
    A.slot = slot;
    A.work = &scal->work[bucket];
    int64_t blocks = (int64_t)num_cu * blocks_per_cu;
    if (blocks > hstart[bucket + 1] - hstart[bucket]) blocks = hstart[bucket + 1] - hstart[bucket];
    if (kt) kt->begin(slot, s);
    k_tri_lds<KM, NT><<<(unsigned)blocks, NT, 0, s>>>(A);
    if (kt) kt->end(slot, s);
  };
  // heaviest buckets first so that their tails overlap the light ones
  if (kmax_g > 0) {
    size_t K = kmax_g, WK = (K + 63) / 64;
    size_t per_block = K * WK * 8 + (7 * K + 2) * 4;
    int64_t owners = hstart[TK_GLOBAL + 1] - hstart[TK_GLOBAL];
    int64_t blocks = (int64_t)((size_t(1) << 30) / per_block);
    if (blocks > 64) blocks = 64;
    if (blocks > owners) blocks = owners;
    if (blocks < 1) blocks = 1;
    size_t bits_bytes = ((size_t)blocks * K * WK * 8 + 255) & ~size_t(255);
    char* big = big_scratch(bits_bytes + (size_t)blocks * (7 * K + 2) * 4);
    if (!big) throw Fail(M4_ENOMEM, "scratch for dense out-lists does not fit");
    uint64_t* gbits = reinterpret_cast<uint64_t*>(big);
    int32_t* garr = reinterpret_cast<int32_t*>(big + bits_bytes);
    A.bucket = TK_GLOBAL;
    A.slot = M4_K_TRI_GLOBAL;
    A.work = &scal->work[TK_GLOBAL];
    A.kmax = (int)K;
    A.gbits = gbits;
    A.garr = garr;
    if (kt) kt->begin(M4_K_TRI_GLOBAL, s);
    k_tri_global<256><<<(unsigned)blocks, 256, 0, s>>>(A);
    if (kt) kt->end(M4_K_TRI_GLOBAL, s);
  }
  using std::integral_constant;
  run_lds(integral_constant<int, 1024>{}, integral_constant<int, 256>{}, TK_1024, M4_K_TRI_1024, 1);
  run_lds(integral_constant<int, 512>{}, integral_constant<int, 256>{}, TK_512, M4_K_TRI_512, 3);
  run_lds(integral_constant<int, 256>{}, integral_constant<int, 256>{}, TK_256, M4_K_TRI_256, 8);
  run_lds(integral_constant<int, 128>{}, integral_constant<int, 256>{}, TK_128, M4_K_TRI_128, 8);
  run_lds(integral_constant<int, 64>{}, integral_constant<int, 64>{}, TK_WAVE, M4_K_TRI_WAVE, 32);
}

}  // namespace m4
