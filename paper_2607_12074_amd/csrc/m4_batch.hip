// m4_batch.hip -- many small graphs counted by one persistent fused launch.
//
// Every workgroup repeatedly takes the next graph of the arena (largest
// first) and runs the whole method on it without leaving the kernel:
//   A. CSR builder: degree order by a bitonic sort of (degree, id) keys in
//      LDS, relabelled rows sorted per row, out-list offsets;
//   B. triangle and 4-clique anchors: owners with out-degree <= 64 one per
//      wavefront, larger owners one at a time by the whole workgroup with the
//      frontier bitmap in LDS (or in global scratch beyond its capacity);
//   C. 4-cycle anchor: light owners one per wavefront with an LDS hash table,
//      heavy owners by the whole workgroup with dense LDS counters;
//   D. closure sums and the exact inverse, written as the graph's six counts.
// Graphs larger than the workgroup's LDS structures are flagged for the
// multi-kernel single-graph path.  The launch is captured once in a hipGraph
// per arena layout and replayed.
#include <limits.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "m4_batch.h"
#include "m4_tri_dev.h"

namespace m4 {

namespace {

// LDS bytes of the per-owner triangle arrays plus bitmap for out-degree k
__host__ __device__ constexpr int tri_lds_bytes(int k) {
  return 7 * 4 * (k + 1) + 8 + 8 * k * ((k + 63) / 64);
}
template <int UB>
__host__ __device__ constexpr int tri_lds_kmax() {
  int k = 64;
  while (tri_lds_bytes(k + 64) <= UB) k += 64;
  return k;
}

constexpr int PW_TRI = 2560;  // per-wavefront triangle arrays (k <= 64)
constexpr int PW_HASH = 512;  // per-wavefront hash slots of the light 4-cycle owners
constexpr int64_t kBatchWorkMax = int64_t(1) << 26;  // sum of d^2 of a fused-kernel graph

template <int NT>
__device__ __forceinline__ void bitonic_u32(uint32_t* s, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        int ixj = i ^ j;
        if (ixj > i) {
          uint32_t a = s[i], b = s[ixj];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int NT, int UB>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs A) {
  constexpr int NW = NT / WAVE;
  static_assert(NW * PW_TRI <= UB, "per-wave triangle arrays");
  static_assert(NW * (PW_HASH * 8 + 2 * 65 * 4 + 16) <= UB, "per-wave hash tables");
  static_assert(B_NMAX * 4 <= UB, "degree keys");
  __shared__ __align__(16) unsigned char U[UB];
  __shared__ int16_t rankL[B_NMAX];
  __shared__ int16_t dlist[B_NMAX];
  __shared__ int s_item, s_r1, s_ndef, s_below, s_err;
  __shared__ unsigned int s_dmax;
  __shared__ unsigned long long s_d2;
  __shared__ U128 gacc[7];
  constexpr int KB = tri_lds_kmax<UB>();
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(A.work, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= A.norder) break;
    const int64_t g = A.order ? A.order[item] : item;
    const int64_t v0 = A.voff[g], e0 = A.eoff[g], v1 = A.voff[g + 1], e1 = A.eoff[g + 1];
    unsigned long long* outg = A.out + 6 * g;
    // the graph's slices of the work arrays must lie inside them
    if (v0 < 0 || e0 < 0 || v1 < v0 || e1 < e0 || v1 > A.vcap || e1 > A.ecap || (e1 - e0) % 2) {
      if (tid == 0) A.status[g] = M4_EINVAL;
      continue;
    }
    const int64_t nn = v1 - v0;
    const int n = nn > B_NMAX ? B_NMAX + 1 : (int)nn;
    const int64_t nnz = e1 - e0;
    if (n < 4 || nnz == 0) {
      if (tid < 6) outg[tid] = 0;
      if (tid == 0) A.status[g] = 0;
      continue;
    }
    if (n > B_NMAX) {
      if (tid == 0) A.status[g] = A.too_big;
      continue;
    }
    const int64_t* rp = A.rowp + v0 + g;
    // The graph is counted here only when every per-owner structure fits the
    // workgroup's LDS (out-degree <= KB) and its work is modest; this is
    // decided from the arena's contents on every launch, so a replayed launch
    // never trusts an earlier routing.  Other graphs are left to the
    // single-graph path (status B_TOO_BIG).
    if (tid == 0) {
      s_dmax = 0;
      s_d2 = 0;
      s_err = 0;
    }
    __syncthreads();
    {
      unsigned int dm = 0;
      unsigned long long d2 = 0;
      for (int v = tid; v < n; v += NT) {
        const int64_t d = rp[v + 1] - rp[v];
        const unsigned int du = d < 0 ? 0xffffffffu : (d > 0x7fffffff ? 0x7fffffffu : (unsigned)d);
        dm = du > dm ? du : dm;
        d2 += (unsigned long long)du * du;
      }
      if (dm) atomicMax(&s_dmax, dm);
      if (d2) atomicAdd(&s_d2, d2);
    }
    __syncthreads();
    if (s_dmax > (unsigned)KB || s_dmax >= (unsigned)n || s_d2 > (unsigned long long)kBatchWorkMax ||
        rp[0] != 0 || rp[n] != nnz) {
      if (tid == 0) A.status[g] = A.too_big;
      continue;
    }
    const int32_t* cl = A.col + e0;
    int32_t* perm = A.perm + v0;
    int32_t* dr = A.dr + v0;
    int32_t* dlo = A.dlo + v0;
    int32_t* dplus = A.dplus + v0;
    int64_t* nptr = A.nptr + v0 + g;
    int64_t* optr = A.optr + v0 + g;
    int32_t* ncol = A.ncol + e0;
    uint32_t* t = A.t + e0 / 2;
    if (tid < 7) gacc[tid].lo = gacc[tid].hi = 0;
    if (tid == 0) {
      s_r1 = n;
      s_ndef = 0;
    }

    // ---- A. degree order (bitonic sort of (degree << 13 | id) keys)
    uint32_t* keys = reinterpret_cast<uint32_t*>(U);
    int P = 1;
    while (P < n) P <<= 1;
    for (int v = tid; v < P; v += NT)
      keys[v] = v < n ? (((uint32_t)(rp[v + 1] - rp[v]) << 13) | (uint32_t)v) : 0xffffffffu;
    __syncthreads();
    bitonic_u32<NT>(keys, P);
    for (int r = tid; r < n; r += NT) {
      const uint32_t key = keys[r];
      const int v = (int)(key & 0x1fffu), d = (int)(key >> 13);
      perm[r] = v;
      dr[r] = d;
      rankL[v] = (int16_t)r;
      if (d >= 2 && (r == 0 || (keys[r - 1] >> 13) < 2)) s_r1 = r;
    }
    {
      const int per = (n + NT - 1) / NT, lo = tid * per;
      int64_t sum = 0;
      for (int r = lo; r < lo + per && r < n; r++) sum += keys[r] >> 13;
      int64_t tot;
      int64_t run = block_excl_scan64<NT>(sum, &tot);
      for (int r = lo; r < lo + per && r < n; r++) {
        nptr[r] = run;
        run += keys[r] >> 13;
      }
      if (tid == 0) nptr[n] = tot;
    }
    __syncthreads();
    const int r1 = s_r1;
    // rows of degree <= 64: one wavefront each, sorted position by counting
    for (int r = wid; r < n; r += NW) {
      const uint32_t key = keys[r];
      const int d = (int)(key >> 13);
      if (d > WAVE) {
        if (lane == 0) dlist[atomicAdd(&s_ndef, 1)] = (int16_t)r;
        continue;
      }
      const int v = (int)(key & 0x1fffu);
      int x = INT_MAX;
      if (lane < d) x = rankL[cl[rp[v] + lane]];
      int pos = 0;
      for (int k2 = 0; k2 < WAVE; k2++) pos += (__shfl(x, k2, WAVE) < x);
      const uint64_t below = __ballot(lane < d && x < r);
      if (lane < d) ncol[nptr[r] + pos] = x;
      if (lane == 0) {
        const int b = __popcll(below);
        dlo[r] = b;
        dplus[r] = d - b;
      }
    }
    __syncthreads();
    // longer rows: the whole workgroup sorts one row at a time in LDS
    const int ndef = s_ndef;
    for (int idx = 0; idx < ndef; idx++) {
      const int r = dlist[idx];
      const int d = dr[r], v = perm[r];
      int32_t* buf = reinterpret_cast<int32_t*>(U);
      int Pd = 1;
      while (Pd < d) Pd <<= 1;
      if (tid == 0) s_below = 0;
      __syncthreads();
      int mb = 0;
      for (int i = tid; i < Pd; i += NT) {
        int x = INT_MAX;
        if (i < d) {
          x = rankL[cl[rp[v] + i]];
          mb += x < r;
        }
        buf[i] = x;
      }
      if (mb) atomicAdd(&s_below, mb);
      __syncthreads();
      bitonic_u32<NT>(reinterpret_cast<uint32_t*>(buf), Pd);
      for (int i = tid; i < d; i += NT) ncol[nptr[r] + i] = buf[i];
      if (tid == 0) {
        dlo[r] = s_below;
        dplus[r] = d - s_below;
      }
      __syncthreads();
    }
    {
      const int per = (n + NT - 1) / NT, lo = tid * per;
      int64_t sum = 0;
      for (int r = lo; r < lo + per && r < n; r++) sum += dplus[r];
      int64_t tot;
      int64_t run = block_excl_scan64<NT>(sum, &tot);
      for (int r = lo; r < lo + per && r < n; r++) {
        optr[r] = run;
        run += dplus[r];
      }
      if (tid == 0) optr[n] = tot;
    }
    for (int64_t i = tid; i < nnz / 2; i += NT) t[i] = 0;
    if (tid == 0) s_ndef = 0;
    __syncthreads();

    // ---- B. triangle and 4-clique anchors
    TriArgs T{};
    T.nptr = nptr;
    T.optr = optr;
    T.ncol = ncol;
    T.dlo = dlo;
    T.dplus = dplus;
    T.t = t;
    T.flags = A.flags;
    T.cache_rows = A.cache_rows;
    T.err = &s_err;
    u128_t k4 = 0;
    unsigned long long st0 = 0, st1 = 0, st2 = 0, st3 = 0, st4 = 0, st5 = 0;
    {
      unsigned char* w = U + wid * PW_TRI;
      int32_t* a = reinterpret_cast<int32_t*>(w);
      int32_t* sst = a + 64;
      int32_t* soe = sst + 64;
      int32_t* slen = soe + 64;
      int32_t* spref = slen + 64;  // 65 entries
      uint32_t* colcnt = reinterpret_cast<uint32_t*>(spref + 68);
      uint32_t* tag = colcnt + 64;
      uint64_t* B = reinterpret_cast<uint64_t*>(tag + 64);
      for (int r = wid; r < n; r += NW) {
        const int k = dplus[r];
        if (k < 2) continue;
        if (k > WAVE) {
          if (lane == 0) dlist[atomicAdd(&s_ndef, 1)] = (int16_t)r;
          continue;
        }
        tri_owner<WAVE, false, true>(T, r, lane, a, sst, soe, slen, spref, colcnt, tag, B, k4,
                                     st0, st1, st2, st3, st4, st5);
      }
    }
    __syncthreads();
    const int nbig = s_ndef;
    for (int idx = 0; idx < nbig; idx++) {
      const int r = dlist[idx];
      const int k = dplus[r];
      // the planner only sends graphs whose out-degrees fit the LDS bitmap
      int32_t* a = reinterpret_cast<int32_t*>(U);
      int32_t* sst = a + k;
      int32_t* soe = sst + k;
      int32_t* slen = soe + k;
      int32_t* spref = slen + k;
      uint32_t* colcnt = reinterpret_cast<uint32_t*>(spref + k + 1);
      uint32_t* tag = colcnt + k;
      uint64_t* B =
          reinterpret_cast<uint64_t*>(U + ((7 * 4 * (size_t)(k + 1) + 7) & ~(size_t)7));
      tri_owner<NT, false, false>(T, r, tid, a, sst, soe, slen, spref, colcnt, tag, B, k4, st0,
                                  st1, st2, st3, st4, st5);
      __syncthreads();
    }
    if (tid == 0) s_ndef = 0;
    __syncthreads();

    // ---- C. 4-cycle anchor
    u128_t c4 = 0;
    {
      unsigned char* w = U + wid * (PW_HASH * 8 + 2 * 65 * 4 + 16);
      int32_t* hkey = reinterpret_cast<int32_t*>(w);
      uint32_t* hcnt = reinterpret_cast<uint32_t*>(hkey + PW_HASH);
      int32_t* sst = reinterpret_cast<int32_t*>(hcnt + PW_HASH);
      int32_t* spref = sst + 65;
      for (int r = wid; r < n; r += NW) {
        const int nl = dlo[r];
        if (r < r1 || nl < 2) continue;
        const int64_t base = nptr[r];
        int64_t wb = 0;
        for (int i = lane; i < nl; i += WAVE) wb += dr[ncol[base + i]] - 1;
        for (int o = WAVE / 2; o > 0; o >>= 1) wb += __shfl_xor(wb, o, WAVE);
        if (wb == 0) continue;
        if (wb > A.light || 2 * wb > PW_HASH) {
          if (lane == 0) dlist[atomicAdd(&s_ndef, 1)] = (int16_t)r;
          continue;
        }
        int S = 16;
        while (S < 2 * wb) S <<= 1;
        const uint32_t mask = (uint32_t)S - 1;
        const int shift = 32 - __ffs(S) + 1;
        for (int i = lane; i < S; i += WAVE) {
          hkey[i] = -1;
          hcnt[i] = 0;
        }
        wave_sync();
        for (int c0 = 0; c0 < nl; c0 += WAVE) {
          const int nc = nl - c0 < WAVE ? nl - c0 : WAVE;
          int len = 0;
          if (lane < nc) {
            const int32_t v = ncol[base + c0 + lane];
            sst[lane] = (int32_t)nptr[v];
            len = dr[v];
          }
          int64_t tot;
          const int64_t ex = block_excl_scan64<WAVE>(len, &tot);
          if (lane < nc) spref[lane] = (int32_t)ex;
          wave_sync();
          for (int q = lane; q < (int)tot; q += WAVE) {
            const int si = upper_index(spref, nc, q);
            const int32_t x = ncol[sst[si] + (q - spref[si])];
            if (x < r1 || x >= r) continue;
            // at most wb <= S / 2 distinct keys: x or a free slot within S probes
            uint32_t h = ((uint32_t)x * 0x9E3779B1u) >> shift;
            bool found = false;
            for (int probes = 0; probes < S; probes++) {
              const int32_t kk = hkey[h];
              if (kk == x) {
                found = true;
                break;
              }
              if (kk == -1) {
                const int32_t prev = atomicCAS(&hkey[h], -1, x);
                if (prev == -1 || prev == x) {
                  found = true;
                  break;
                }
              }
              h = (h + 1) & mask;
            }
            if (found) c4 += atomicAdd(&hcnt[h], 1u);
            else atomicOr(&s_err, ERR_PROBE);
          }
          wave_sync();
        }
      }
    }
    __syncthreads();
    const int nheavy = s_ndef;
    for (int idx = 0; idx < nheavy; idx++) {
      const int r = dlist[idx];
      const int nl = dlo[r];
      const int64_t base = nptr[r];
      uint32_t* cnt = reinterpret_cast<uint32_t*>(U);
      int32_t* sst = reinterpret_cast<int32_t*>(U + 4 * B_NMAX);
      int32_t* spref = sst + NT;
      for (int i = tid; i < r - r1; i += NT) cnt[i] = 0;
      __syncthreads();
      for (int c0 = 0; c0 < nl; c0 += NT) {
        const int nc = nl - c0 < NT ? nl - c0 : NT;
        int len = 0;
        if (tid < nc) {
          const int32_t v = ncol[base + c0 + tid];
          sst[tid] = (int32_t)nptr[v];
          len = dr[v];
        }
        int64_t tot;
        const int64_t ex = block_excl_scan64<NT>(len, &tot);
        if (tid < nc) spref[tid] = (int32_t)ex;
        __syncthreads();
        for (int q = tid; q < (int)tot; q += NT) {
          const int si = upper_index(spref, nc, q);
          const int32_t x = ncol[sst[si] + (q - spref[si])];
          if (x >= r1 && x < r) c4 += atomicAdd(&cnt[x - r1], 1u);
        }
        __syncthreads();
      }
    }

    // ---- D. closure and exact inverse
    u128_t S = 0, Pp = 0, D = 0, Paw2 = 0, St = 0;
    for (int r = tid; r < n; r += NT) {
      const uint64_t du = (uint32_t)dr[r];
      if (du >= 3) S += (u128_t)du * (du - 1) * (du - 2) / 6;
      const int k = dplus[r];
      const int64_t rb = nptr[r] + dlo[r], oe = optr[r];
      for (int j = 0; j < k; j++) {
        const uint64_t dv = (uint32_t)dr[ncol[rb + j]];
        const uint64_t te = t[oe + j];
        Pp += (u128_t)((du - 1) * (dv - 1));
        St += te;
        D += (u128_t)(te * (te - 1) / 2);
        if (te) Paw2 += (u128_t)(te * (du + dv - 4));
      }
    }
    const u128_t parts[7] = {k4, c4, S, Pp, D, Paw2, St};
    for (int i = 0; i < 7; i++)
      if (parts[i]) atomic_add_u128(&gacc[i], parts[i]);
    __syncthreads();
    if (tid == 0) {
      u128_t in[7];
      for (int i = 0; i < 7; i++) in[i] = load_u128(&gacc[i]);
      unsigned long long res[6], bas[8];
      const int fs = finalize_basis(in, res, bas);
      A.status[g] = s_err ? 7 : fs;
      for (int i = 0; i < 6; i++) outg[i] = res[i];
      if (A.basis)
        for (int i = 0; i < 8; i++) A.basis[8 * g + i] = bas[i];
    }
    __syncthreads();
  }
}

__global__ void k_batch_reset(unsigned int* work) { *work = 0; }

}  // namespace

// ---------------------------------------------------------------- host side

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

void BatchBuffers::release() {
  dev.release();
  if (h_out) (void)hipHostFree(h_out);
  if (h_status) (void)hipHostFree(h_status);
  if (h_stage) (void)hipHostFree(h_stage);
  h_out = nullptr;
  h_status = nullptr;
  h_stage = nullptr;
  h_out_cap = h_stage_cap = 0;
}

int batch_variant_kb(int variant) {
  return variant == 1 ? tri_lds_kmax<40960>() : tri_lds_kmax<98304>();
}

bool batch_graph_fits(int64_t n, const int64_t* rp, int variant) {
  if (n > B_NMAX) return false;
  const int64_t KB = batch_variant_kb(variant);
  int64_t d2 = 0;
  for (int64_t v = 0; v < n; v++) {
    const int64_t d = rp[v + 1] - rp[v];
    if (d > KB) return false;
    d2 += d * d;
  }
  return d2 <= kBatchWorkMax;
}

// Plans a launch over an arena whose offsets are readable on the host, and
// lays out the device buffers.  The plan depends on the offsets only: a graph
// with more than B_NMAX vertices goes to the single-graph path at once, every
// other one is queued for the fused kernel (largest first), which itself
// checks the graph's degrees and work against its LDS structures on every
// launch.
// dev_arena: device pointers of the arena, or null to stage the host arena
// into pinned memory and upload it within the launch.
BatchLayout batch_layout(int64_t G, int64_t sum_n, int64_t sum_nnz, bool staged) {
  BatchLayout L{};
  size_t need = 0;
  auto add = [&](size_t bytes) {
    size_t o2 = need;
    need += al(bytes + 8);
    return o2;
  };
  L.o_perm = add(sum_n * 4);
  L.o_dr = add(sum_n * 4);
  L.o_dlo = add(sum_n * 4);
  L.o_dplus = add(sum_n * 4);
  L.o_nptr = add((sum_n + G) * 8);
  L.o_optr = add((sum_n + G) * 8);
  L.o_ncol = add(sum_nnz * 4);
  L.o_t = add(sum_nnz / 2 * 4);
  L.o_order = add(G * 4);
  L.o_out = add(G * 48);
  L.o_status = add(G * 4);
  L.o_work = add(64);
  L.arena_bytes = (size_t)(G + 1) * 16 + (sum_n + G) * 8 + sum_nnz * 4;
  if (staged) L.o_arena = add(L.arena_bytes);
  L.need = need;
  return L;
}

void batch_prepare(m4_ctx* c, BatchBuffers& B, BatchPlan& P, int64_t G, const int64_t* hvoff,
                   const int64_t* heoff, const m4_batch* dev_arena, int variant, int light,
                   uint32_t flags, uint32_t cache_rows, hipStream_t s) {
  const int64_t sum_n = hvoff[G], sum_nnz = heoff[G];
  std::vector<int64_t> nnz(G);
  P.order.clear();
  P.big.clear();
  for (int64_t g = 0; g < G; g++) {
    nnz[g] = heoff[g + 1] - heoff[g];
    if (hvoff[g + 1] - hvoff[g] <= B_NMAX) P.order.push_back((int32_t)g);
    else P.big.push_back(g);
  }
  // largest graphs first
  std::stable_sort(P.order.begin(), P.order.end(),
                   [&](int32_t x, int32_t y) { return nnz[x] > nnz[y]; });
  P.variant = variant;
  P.G = G;
  P.sum_n = sum_n;
  P.sum_nnz = sum_nnz;
  int grid = c->num_cu * (variant == 1 ? 2 : 1);
  if ((int64_t)grid > (int64_t)P.order.size()) grid = (int)std::max<size_t>(1, P.order.size());
  P.grid = grid;

  P.staged = dev_arena == nullptr;
  const BatchLayout Lo = batch_layout(G, sum_n, sum_nnz, P.staged);
  const size_t o_perm = Lo.o_perm, o_dr = Lo.o_dr, o_dlo = Lo.o_dlo, o_dplus = Lo.o_dplus,
               o_nptr = Lo.o_nptr, o_optr = Lo.o_optr, o_ncol = Lo.o_ncol, o_t = Lo.o_t,
               o_order = Lo.o_order, o_out = Lo.o_out, o_status = Lo.o_status,
               o_work = Lo.o_work;
  P.arena_bytes = Lo.arena_bytes;
  if (P.staged) P.o_arena = Lo.o_arena;
  B.dev.ensure(Lo.need, s);
  char* d = B.dev.ptr;
  if (B.h_out_cap < (size_t)G) {
    if (B.h_out) (void)hipHostFree(B.h_out);
    if (B.h_status) (void)hipHostFree(B.h_status);
    B.h_out = nullptr;
    B.h_status = nullptr;
    M4_HIP(hipHostMalloc((void**)&B.h_out, G * 48, hipHostMallocDefault));
    M4_HIP(hipHostMalloc((void**)&B.h_status, G * 4, hipHostMallocDefault));
    B.h_out_cap = G;
  }
  if (P.staged && B.h_stage_cap < P.arena_bytes) {
    if (B.h_stage) (void)hipHostFree(B.h_stage);
    B.h_stage = nullptr;
    M4_HIP(hipHostMalloc((void**)&B.h_stage, P.arena_bytes, hipHostMallocDefault));
    B.h_stage_cap = P.arena_bytes;
  }
  if (!P.order.empty())
    M4_HIP(hipMemcpyAsync(d + o_order, P.order.data(), P.order.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  BatchArgs& A = P.args;
  A = BatchArgs{};
  A.G = G;
  if (!P.staged) {
    A.voff = dev_arena->voff;
    A.eoff = dev_arena->eoff;
    A.rowp = dev_arena->row_ptr;
    A.col = dev_arena->col;
  } else {
    int64_t* av = reinterpret_cast<int64_t*>(d + P.o_arena);
    A.voff = av;
    A.eoff = av + (G + 1);
    A.rowp = av + 2 * (G + 1);
    A.col = reinterpret_cast<const int32_t*>(av + 2 * (G + 1) + (sum_n + G));
  }
  A.order = reinterpret_cast<int32_t*>(d + o_order);
  A.norder = (int64_t)P.order.size();
  A.work = reinterpret_cast<unsigned int*>(d + o_work);
  A.perm = reinterpret_cast<int32_t*>(d + o_perm);
  A.dr = reinterpret_cast<int32_t*>(d + o_dr);
  A.dlo = reinterpret_cast<int32_t*>(d + o_dlo);
  A.dplus = reinterpret_cast<int32_t*>(d + o_dplus);
  A.nptr = reinterpret_cast<int64_t*>(d + o_nptr);
  A.optr = reinterpret_cast<int64_t*>(d + o_optr);
  A.ncol = reinterpret_cast<int32_t*>(d + o_ncol);
  A.t = reinterpret_cast<uint32_t*>(d + o_t);
  A.out = reinterpret_cast<unsigned long long*>(d + o_out);
  A.status = reinterpret_cast<int*>(d + o_status);
  A.light = light;
  A.flags = flags;
  A.cache_rows = cache_rows;
  A.too_big = B_TOO_BIG;
  A.vcap = sum_n;
  A.ecap = sum_nnz;
}

// Copies a host arena into the pinned staging buffer of a prepared plan.
void batch_stage(BatchBuffers& B, const BatchPlan& P, const int64_t* voff, const int64_t* eoff,
                 const int64_t* rowp, const int32_t* col) {
  const int64_t G = P.G;
  char* p = B.h_stage;
  memcpy(p, voff, (G + 1) * 8);
  memcpy(p + (G + 1) * 8, eoff, (G + 1) * 8);
  memcpy(p + (G + 1) * 16, rowp, (P.sum_n + G) * 8);
  memcpy(p + (G + 1) * 16 + (P.sum_n + G) * 8, col, P.sum_nnz * 4);
}

// Enqueues [upload] -> counter reset -> fused kernel -> results to pinned
// host memory on stream s (also used inside a stream capture).
void batch_enqueue(BatchBuffers& B, const BatchPlan& P, hipStream_t s) {
  const BatchArgs& A = P.args;
  if (P.staged)
    M4_HIP(hipMemcpyAsync(B.dev.ptr + P.o_arena, B.h_stage, P.arena_bytes, hipMemcpyHostToDevice,
                          s));
  k_batch_reset<<<1, 1, 0, s>>>(A.work);
  fill_u32(A.status, (uint32_t)B_TOO_BIG, (size_t)P.G, s);
  if (A.norder > 0) {
    if (P.variant == 1)
      k_batch<512, 40960><<<P.grid, 512, 0, s>>>(A);
    else
      k_batch<1024, 98304><<<P.grid, 1024, 0, s>>>(A);
  }
  M4_HIP(hipMemcpyAsync(B.h_out, A.out, P.G * 48, hipMemcpyDeviceToHost, s));
  M4_HIP(hipMemcpyAsync(B.h_status, A.status, P.G * 4, hipMemcpyDeviceToHost, s));
}

// The captured launch of the last arena.  It is replayed only when the new
// arena has the same offsets (compared by content) and, for a device arena,
// the same device pointers (they are baked into the captured kernel
// arguments); the arena's rows and columns may differ freely, because the
// kernel decides per launch which graphs it counts.
void batch_launch_fused(const BatchArgs& A, int grid, hipStream_t s) {
  k_batch<1024, 98304><<<grid, 1024, 0, s>>>(A);
}

int batch_light_max() { return PW_HASH / 2; }

struct BatchState {
  std::vector<int64_t> voff, eoff;
  const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
  int variant = -1, light = -1;
  uint32_t flags = 0, cache_rows = 0;
  bool on_device = false;
  hipStream_t stream = nullptr;
  BatchBuffers buf;
  BatchPlan plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~BatchState() {
    drop_graph();
    buf.release();
  }
};

size_t batch_held_bytes(const m4_ctx* c) { return c->batch ? c->batch->buf.dev.cap : 0; }

void batch_release(m4_ctx* c) { destroy_batch_state(c); }

void destroy_batch_state(m4_ctx* c) {
  delete c->batch;
  c->batch = nullptr;
}

int count_batch_impl(m4_ctx* c, const m4_batch* b, const m4_opts* o, uint64_t* out,
                     m4_stats* st) {
  if (!b || !out || b->num_graphs < 0) return set_error(c, M4_EINVAL, "bad batch arguments");
  const int64_t G = b->num_graphs;
  if (G == 0) return M4_OK;
  if (!b->voff || !b->eoff || !b->row_ptr || !b->col)
    return set_error(c, M4_EINVAL, "bad batch arguments");
  hipStream_t s = (o && o->hip_stream) ? (hipStream_t)o->hip_stream : c->stream;
  const uint32_t flags = o ? o->flags : 0;
  const uint32_t cache_rows = o ? o->cache_rows : 0;
  const int variant = c->tune.batch_variant;
  int light = (o && o->c4_light_max > 0) ? o->c4_light_max : c->tune.batch_light;
  light = std::max(1, std::min(light, PW_HASH / 2));
  if (!c->batch) c->batch = new BatchState();
  BatchState& S = *c->batch;
  hipEvent_t e0 = c->ev[0], e1 = c->ev[1];
  const bool timing = st && (flags & (M4_STATS | M4_TIMING));

  std::vector<int64_t> hv, he;
  const int64_t* hvoff;
  const int64_t* heoff;
  if (b->on_device) {
    hv.resize(G + 1);
    he.resize(G + 1);
    M4_HIP(hipMemcpyAsync(hv.data(), b->voff, (G + 1) * 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipMemcpyAsync(he.data(), b->eoff, (G + 1) * 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    hvoff = hv.data();
    heoff = he.data();
  } else {
    hvoff = b->voff;
    heoff = b->eoff;
  }
  const int64_t sum_nnz = heoff[G];
  if (hvoff[0] != 0 || heoff[0] != 0 || sum_nnz >= (int64_t(1) << 31))
    return set_error(c, M4_ERANGE, "batch offsets out of range");
  for (int64_t g = 0; g < G; g++)
    if (hvoff[g + 1] < hvoff[g] || heoff[g + 1] < heoff[g] || (heoff[g + 1] - heoff[g]) % 2)
      return set_error(c, M4_EINVAL, "batch offsets are not a partition");
  if (flags & M4_PLAIN_LOOP) {
    // one complete single-graph count per graph, on the same stream
    if (timing) M4_HIP(hipEventRecord(e0, s));
    int rc = M4_OK;
    for (int64_t g = 0; g < G && rc == M4_OK; g++) {
      m4_csr sub;
      sub.n = hvoff[g + 1] - hvoff[g];
      sub.nnz = heoff[g + 1] - heoff[g];
      sub.row_ptr = b->row_ptr + hvoff[g] + g;
      sub.col = b->col + heoff[g];
      sub.on_device = b->on_device;
      m4_opts o2{};
      if (o) o2 = *o;
      o2.hip_stream = s;
      o2.flags &= ~(uint32_t)(M4_STATS | M4_TIMING | M4_PLAIN_LOOP);
      rc = m4_count_motifs4_ex(c, &sub, &o2, out + 6 * g, nullptr);
    }
    if (timing) M4_HIP(hipEventRecord(e1, s));
    if (st) {
      memset(st, 0, sizeof(*st));
      if (timing) {
        M4_HIP(hipEventSynchronize(e1));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        st->ms_total = ms;
      }
    }
    return rc;
  }

  const bool dev_same = !b->on_device || (S.key[0] == b->voff && S.key[1] == b->eoff &&
                                           S.key[2] == b->row_ptr && S.key[3] == b->col);
  const bool same = S.exec && dev_same && S.voff.size() == (size_t)(G + 1) &&
                    memcmp(S.voff.data(), hvoff, (G + 1) * 8) == 0 &&
                    memcmp(S.eoff.data(), heoff, (G + 1) * 8) == 0 && S.variant == variant &&
                    S.light == light && S.flags == flags && S.cache_rows == cache_rows &&
                    S.on_device == (b->on_device != 0) && S.stream == s;
  if (!same) {
    S.drop_graph();
    batch_prepare(c, S.buf, S.plan, G, hvoff, heoff, b->on_device ? b : nullptr, variant, light,
                  flags, cache_rows, s);
    // capture the whole launch once; later calls on this layout replay it
    M4_HIP(hipStreamSynchronize(s));
    M4_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    batch_enqueue(S.buf, S.plan, s);
    M4_HIP(hipStreamEndCapture(s, &S.graph));
    M4_HIP(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
    S.voff.assign(hvoff, hvoff + G + 1);
    S.eoff.assign(heoff, heoff + G + 1);
    S.key[0] = b->voff;
    S.key[1] = b->eoff;
    S.key[2] = b->row_ptr;
    S.key[3] = b->col;
    S.variant = variant;
    S.light = light;
    S.flags = flags;
    S.cache_rows = cache_rows;
    S.on_device = b->on_device != 0;
    S.stream = s;
  }
  if (!b->on_device) batch_stage(S.buf, S.plan, b->voff, b->eoff, b->row_ptr, b->col);
  if (timing) M4_HIP(hipEventRecord(e0, s));
  M4_HIP(hipGraphLaunch(S.exec, s));
  if (timing) M4_HIP(hipEventRecord(e1, s));
  M4_HIP(hipStreamSynchronize(s));
  int rc = M4_OK;
  std::vector<int64_t> single;
  for (int64_t g = 0; g < G; g++) {
    const int sg = S.buf.h_status[g];
    if (sg == B_TOO_BIG) {
      single.push_back(g);
      continue;
    }
    if (sg == 3 && rc == M4_OK) rc = set_error(c, M4_EOVERFLOW, "a count is >= 2^64");
    if (sg != 0 && sg != 3 && rc == M4_OK)
      rc = set_error(c, M4_EINTERNAL, "closure consistency or probe bound check failed");
    memcpy(out + 6 * g, S.buf.h_out + 6 * g, 48);
  }
  // graphs the fused kernel left alone: the multi-kernel single-graph path
  for (int64_t g : single) {
    m4_csr sub;
    sub.n = hvoff[g + 1] - hvoff[g];
    sub.nnz = heoff[g + 1] - heoff[g];
    sub.row_ptr = b->row_ptr + hvoff[g] + g;
    sub.col = b->col + heoff[g];
    sub.on_device = b->on_device;
    m4_opts o2{};
    if (o) o2 = *o;
    o2.hip_stream = s;
    o2.flags &= ~(uint32_t)(M4_STATS | M4_TIMING);
    int r2 = m4_count_motifs4_ex(c, &sub, &o2, out + 6 * g, nullptr);
    if (r2 != M4_OK && rc == M4_OK) rc = r2;
  }
  if (st) {
    memset(st, 0, sizeof(*st));
    st->partitions = 1;
    if (timing) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      st->ms_total = ms;
    }
  }
  return rc;
}

}  // namespace m4

extern "C" int m4_count_batch(m4_ctx* ctx, const m4_batch* b, const m4_opts* o, uint64_t* out,
                              m4_stats* st) {
  if (!ctx) return M4_EINVAL;
  try {
    M4_HIP(hipSetDevice(ctx->device));
    return m4::count_batch_impl(ctx, b, o, out, st);
  } catch (const m4::HipFail& f) {
    (void)hipGetLastError();
    return m4::set_error(ctx, M4_EDEVICE, std::string(f.what) + ": " + hipGetErrorString(f.e));
  } catch (const m4::Fail& f) {
    return m4::set_error(ctx, f.code, f.msg);
  } catch (...) {
    return m4::set_error(ctx, M4_EINTERNAL, "unexpected exception");
  }
}
