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

#include <array>

#include "m4_tri_dev.h"

namespace m4 {

namespace {

// At least 5 wavefronts per SIMD: the register cap (<= 96 VGPRs) trades a few
// spills for a fifth resident wavefront, which hides more of the load and
// probe latency of the owners whose LDS footprint allows it (out-degree up
// to 256); the larger owners are bound by LDS either way.
template <int KMAX, int NT>
__global__ __launch_bounds__(NT, 5) void k_tri_lds(TriArgs A) {
  constexpr int WMAX = (KMAX + 63) / 64;
  constexpr bool HASH = KMAX <= 512;  // the hash table fits beside the bitmap
  constexpr int HSLOTS = HASH ? 2 * KMAX : 1;
  __shared__ int32_t a[KMAX], sst[KMAX], soe[KMAX], slen[KMAX], spref[KMAX + 1];
  __shared__ uint32_t colcnt[KMAX], tag[KMAX];
  __shared__ uint64_t B[KMAX * WMAX];
  __shared__ int32_t hk[HSLOTS];
  __shared__ int16_t hv[HSLOTS];
  __shared__ int s_item;
  const int64_t b0 = A.start[A.bucket], cnt = A.start[A.bucket + 1] - b0;
  u128_t k4 = 0;
  unsigned long long steps = 0, looks = 0, hits = 0, ksum = 0, wread = 0, owners = 0,
                     escan = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(A.work, (unsigned)A.grab);
    __syncthreads();
    const int64_t first = s_item;
    __syncthreads();
    if (first >= cnt) break;
    const int64_t last = first + A.grab < cnt ? first + A.grab : cnt;
    for (int64_t item = first; item < last; item++) {
      tri_owner<NT, false, false, HASH, true>(A, A.order[b0 + item], threadIdx.x, a, sst, soe,
                                              slen, spref, colcnt, tag, B, k4, steps, looks,
                                              hits, ksum, wread, escan, hk, hv);
      owners++;
    }
  }
  block_add_u128<NT>(&A.scal->acc[ACC_K4], k4);
  if (A.flags & M4_STATS) {
    block_add_u64<NT>(&A.scal->stat[ST_STEPS], steps);
    block_add_u64<NT>(&A.scal->stat[ST_LOOKUPS], looks);
    block_add_u64<NT>(&A.scal->stat[ST_HITS], hits);
    block_add_u64<NT>(&A.scal->kstat[A.slot][0], escan);
    block_add_u64<NT>(&A.scal->kstat[A.slot][1], threadIdx.x == 0 ? owners : 0);
    block_add_u64<NT>(&A.scal->kstat[A.slot][2], ksum);
    block_add_u64<NT>(&A.scal->kstat[A.slot][3], wread);
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
  unsigned long long steps = 0, looks = 0, hits = 0, ksum = 0, wread = 0, owners = 0,
                     escan = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= cnt) break;
    tri_owner<NT, true, false, false, true>(A, A.order[b0 + item], threadIdx.x, a, sst, soe, slen,
                                            spref, colcnt, tag, B, k4, steps, looks, hits, ksum,
                                            wread, escan);
    owners++;
    __threadfence();
  }
  block_add_u128<NT>(&A.scal->acc[ACC_K4], k4);
  if (A.flags & M4_STATS) {
    block_add_u64<NT>(&A.scal->stat[ST_STEPS], steps);
    block_add_u64<NT>(&A.scal->stat[ST_LOOKUPS], looks);
    block_add_u64<NT>(&A.scal->stat[ST_HITS], hits);
    block_add_u64<NT>(&A.scal->kstat[A.slot][0], escan);
    block_add_u64<NT>(&A.scal->kstat[A.slot][1], threadIdx.x == 0 ? owners : 0);
    block_add_u64<NT>(&A.scal->kstat[A.slot][2], ksum);
    block_add_u64<NT>(&A.scal->kstat[A.slot][3], wread);
  }
}

// bucket of every owner by its out-degree k
enum { TK_NONE = 0, TK_WAVE, TK_128, TK_256, TK_512, TK_1024, TK_GLOBAL, TK_N };

__global__ void k_tri_keys(const int32_t* __restrict__ dplus, int64_t n, int64_t own_lo,
                           int64_t own_hi, int wave_max, uint32_t* __restrict__ key, Scal* scal) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int k = (u >= own_lo && u < own_hi) ? dplus[u] : 0;
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

// Hub tables (a vertex with out-degree >= hub_min gets an open-addressing
// table of its out-list, mapping a rank to its position in N+(v)).
__global__ void k_hub_size(const int32_t* __restrict__ dplus, int64_t n, int hub_min,
                           int32_t* __restrict__ hsz, int32_t* __restrict__ hubs,
                           unsigned int* __restrict__ nhub) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int L = dplus[v];
  const bool hub = L >= hub_min;
  hsz[v] = hub ? (1 << hub_bits(L)) : 0;
  if (hub) hubs[atomicAdd(nhub, 1u)] = (int32_t)v;
}

__global__ void k_hub_off(const int32_t* __restrict__ hsz, const int64_t* __restrict__ off64,
                          int64_t n, int32_t* __restrict__ hoff) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  hoff[v] = hsz[v] ? (int32_t)off64[v] : -1;
}

// one wavefront per hub (grid-stride over the hub list); lanes insert the
// out-list entries with 64-bit compare-and-swap
__global__ __launch_bounds__(256) void k_hub_insert(const int32_t* __restrict__ dplus,
                                                    const int64_t* __restrict__ nptr,
                                                    const int32_t* __restrict__ dlo,
                                                    const int32_t* __restrict__ ncol,
                                                    const int32_t* __restrict__ hoff,
                                                    const int32_t* __restrict__ hubs,
                                                    const unsigned int* __restrict__ nhub,
                                                    unsigned long long* __restrict__ htab,
                                                    int* __restrict__ err) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
  const int64_t nh = *nhub;
  for (int64_t hix = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; hix < nh;
       hix += nw) {
    const int32_t v = hubs[hix];
    const int32_t off = hoff[v];
    const int L = dplus[v];
    const int bits = hub_bits(L);
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t st = nptr[v] + dlo[v];
    for (int j = lane; j < L; j += WAVE) {
      const int32_t x = ncol[st + j];
      uint32_t h = hub_hash(x, bits);
      const unsigned long long e = ((unsigned long long)(uint32_t)x << 32) | (uint32_t)j;
      // L distinct keys in 2^bits >= 2L slots: a free slot within 2^bits probes
      for (uint32_t probes = 0;
           atomicCAS(&htab[(int64_t)off + h], HUB_EMPTY, e) != HUB_EMPTY; probes++) {
        if (probes >= mask) {
          atomicOr(err, ERR_PROBE);
          break;
        }
        h = (h + 1) & mask;
      }
    }
  }
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

Launch tri_plan(const Prep& P, Scal* scal, const Tuning& tu, uint32_t flags, uint32_t cache_rows,
                Arena& tmp, hipStream_t s, int num_cu,
                const std::function<char*(size_t)>& big_scratch, KTimer* kt) {
  const int64_t n = P.n;
  if (n == 0 || P.m == 0) return [](hipStream_t) {};
  uint32_t* key = tmp.take<uint32_t>(n);
  int32_t* order = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, 4));
  int64_t* start = tmp.take<int64_t>(17);
  if (!key || !order || !rtmp || !start) throw Fail(M4_EINTERNAL, "workspace too small (tri)");
  fill_u32(&scal->work[0], 0, 8, s);
  // one wavefront per owner reaches more owners when the out-lists it scans
  // stream from HBM rather than from the Infinity Cache
  const int wave_req = (size_t)P.m * 4 > kInfinityCacheBytes ? tu.tri_wave_far : tu.tri_wave_max;
  int wave_max = wave_req < 2 ? 2 : (wave_req > 64 ? 64 : wave_req);
  k_tri_keys<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(P.dplus, n, P.own_lo, P.hi(), wave_max,
                                                         key, scal);
  radix_pass(key, nullptr, n, 0, 4, nullptr, order, rtmp, start, s);
  // hub tables: resident runs only (a partition holds only its halo rows)
  const bool hubs = tu.hub_min > 0 && P.own_hi < 0 && !P.row_len;
  int32_t* hsz = nullptr;
  int32_t* hoff = nullptr;
  int32_t* hub_list = nullptr;
  int64_t* hoff64 = nullptr;
  if (hubs) {
    hsz = tmp.take<int32_t>(n);
    hoff = tmp.take<int32_t>(n);
    hub_list = tmp.take<int32_t>(n);
    hoff64 = tmp.take<int64_t>(n + 1);
    int64_t* hst = tmp.take<int64_t>(scan_tmp_elems(n));
    if (!hsz || !hoff || !hub_list || !hoff64 || !hst)
      throw Fail(M4_EINTERNAL, "workspace too small (hubs)");
    fill_u32(&scal->nhub, 0, 1, s);
    k_hub_size<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(P.dplus, n, tu.hub_min, hsz, hub_list,
                                                          &scal->nhub);
    scan_i32(hsz, n, hoff64, hst, s);
  }
  // largest out-degree of the global bucket decides its scratch size
  unsigned int kmax_g = 0;
  int64_t hstart[17];
  int64_t hub_slots = 0;
  M4_HIP(hipMemcpyAsync(&kmax_g, &scal->work[7], sizeof(kmax_g), hipMemcpyDeviceToHost, s));
  M4_HIP(hipMemcpyAsync(hstart, start, sizeof(hstart), hipMemcpyDeviceToHost, s));
  if (hubs) M4_HIP(hipMemcpyAsync(&hub_slots, hoff64 + n, 8, hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  // scratch: hub tables, then the dense-owner bitmaps
  size_t hub_bytes = 0, dense_bytes = 0, dense_bits = 0, dense_blocks = 0;
  const bool use_hubs = hubs && hub_slots > 0 && hub_slots < (int64_t(1) << 31);
  if (use_hubs) hub_bytes = ((size_t)hub_slots * 8 + 255) & ~size_t(255);
  if (kmax_g > 0) {
    size_t K = kmax_g, WK = (K + 63) / 64;
    size_t per_block = K * WK * 8 + (7 * K + 2) * 4;
    int64_t owners = hstart[TK_GLOBAL + 1] - hstart[TK_GLOBAL];
    int64_t blocks = (int64_t)((size_t(1) << 30) / per_block);
    if (blocks > 64) blocks = 64;
    if (blocks > owners) blocks = owners;
    if (blocks < 1) blocks = 1;
    dense_blocks = (size_t)blocks;
    dense_bits = ((size_t)blocks * K * WK * 8 + 255) & ~size_t(255);
    dense_bytes = dense_bits + (size_t)blocks * (7 * K + 2) * 4;
  }
  char* scratch = nullptr;
  if (hub_bytes + dense_bytes > 0) {
    scratch = big_scratch(hub_bytes + dense_bytes);
    if (!scratch) throw Fail(M4_ENOMEM, "scratch for hub tables and dense out-lists does not fit");
  }

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
  A.err = &scal->err;
  A.flags = flags;
  A.cache_rows = cache_rows;
  std::array<int64_t, 17> hst;
  for (int i = 0; i < 17; i++) hst[i] = hstart[i];
  // everything below runs on the launch stream, after the plan above
  return [=](hipStream_t ls) mutable {
    if (use_hubs) {
      if (kt) kt->begin(M4_K_TRI_HUBS, ls);
      unsigned long long* htab = reinterpret_cast<unsigned long long*>(scratch);
      k_hub_off<<<(unsigned)ceil_div(n, 256), 256, 0, ls>>>(hsz, hoff64, n, hoff);
      fill_u32(htab, 0xffffffffu, (size_t)hub_slots * 2, ls);
      k_hub_insert<<<(unsigned)(num_cu * 8), 256, 0, ls>>>(P.dplus, P.nptr, P.dlo, P.ncol, hoff,
                                                            hub_list, &scal->nhub, htab,
                                                            &scal->err);
      A.hoff = hoff;
      A.htab = htab;
      A.hub_min = tu.hub_min;
      // a probe reads one line of a table: from the Infinity Cache while
      // the tables fit there, else from HBM, where it weighs more against
      // a scan's sequential reads
      A.probe_w = hub_bytes > kInfinityCacheBytes ? tu.probe_w_far : tu.probe_w;
      if (kt) kt->end(M4_K_TRI_HUBS, ls);
    }
    auto run_lds = [&](auto kmax_tag, auto nt_tag, int bucket, int slot, int blocks_per_cu) {
      constexpr int KM = decltype(kmax_tag)::value;
      constexpr int NT = decltype(nt_tag)::value;
      if (hst[bucket + 1] == hst[bucket]) return;
      A.bucket = bucket;
      A.slot = slot;
      A.work = &scal->work[bucket];
      A.grab = KM <= 64 ? 16 : (KM <= 128 ? 4 : 1);
      int64_t blocks = (int64_t)num_cu * blocks_per_cu;
      if (blocks > hst[bucket + 1] - hst[bucket]) blocks = hst[bucket + 1] - hst[bucket];
      if (kt) kt->begin(slot, ls);
      k_tri_lds<KM, NT><<<(unsigned)blocks, NT, 0, ls>>>(A);
      if (kt) kt->end(slot, ls);
    };
    // heaviest buckets first so that their tails overlap the light ones
    if (kmax_g > 0) {
      const size_t K = kmax_g;
      A.bucket = TK_GLOBAL;
      A.slot = M4_K_TRI_GLOBAL;
      A.grab = 1;
      A.work = &scal->work[TK_GLOBAL];
      A.kmax = (int)K;
      A.gbits = reinterpret_cast<uint64_t*>(scratch + hub_bytes);
      A.garr = reinterpret_cast<int32_t*>(scratch + hub_bytes + dense_bits);
      if (kt) kt->begin(M4_K_TRI_GLOBAL, ls);
      k_tri_global<256><<<(unsigned)dense_blocks, 256, 0, ls>>>(A);
      if (kt) kt->end(M4_K_TRI_GLOBAL, ls);
    }
    using std::integral_constant;
    run_lds(integral_constant<int, 1024>{}, integral_constant<int, 256>{}, TK_1024, M4_K_TRI_1024,
            1);
    run_lds(integral_constant<int, 512>{}, integral_constant<int, 256>{}, TK_512, M4_K_TRI_512, 3);
    run_lds(integral_constant<int, 256>{}, integral_constant<int, 256>{}, TK_256, M4_K_TRI_256, 8);
    run_lds(integral_constant<int, 128>{}, integral_constant<int, 256>{}, TK_128, M4_K_TRI_128, 8);
    run_lds(integral_constant<int, 64>{}, integral_constant<int, 64>{}, TK_WAVE, M4_K_TRI_WAVE, 32);
  };
}

}  // namespace m4
