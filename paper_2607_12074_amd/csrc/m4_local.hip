// m4_local.hip -- per-vertex graphlet orbit counts of the connected 4-vertex
// graphs (orbits 4..14 in Przulj's numbering, the one ORCA uses; the paper
// names ORCA's orbit equations in its related work, Section V).
//
// The same closure idea as the global count (Section III-F), one vertex at a
// time: local statistics give, for every vertex v and orbit o, the number
// N_o(v) of non-induced copies (edge subsets) of o's pattern in which v sits
// at o, and a unit upper-triangular inverse turns them into induced counts.
// With d = d(v), t_e the triangles on edge e, t_v the triangles at v and
// S_v = sum over u in N(v) of (d(u) - 1):
//   N4  = sum_{a in N(v)} S_a - d (d - 1) - 2 t_v       path end
//   N5  = (d - 1) S_v - 2 t_v                           path middle
//   N6  = sum_{u in N(v)} C(d(u) - 1, 2)                claw leaf
//   N7  = C(d, 3)                                       claw centre
//   N8  = 4-cycles through v                            cycle
//   N9  = sum_{a in N(v)} (t_a - t_va)                  paw tail
//   N10 = sum_{a in N(v)} t_va (d(a) - 2)               paw, triangle, degree 2
//   N11 = t_v (d - 2)                                   paw, degree 3
//   N12 = sum over triangles (v, a, b) of (t_ab - 1)    diamond, degree 2
//   N13 = sum_{u in N(v)} C(t_vu, 2)                    diamond, degree 3
//   N14 = 4-cliques through v                           clique
// and, counting the spanning copies of each orbit inside the denser ones at
// the same vertex (a diamond holds one cycle, two paws where a degree-2
// vertex is the tail, ...):
//   N14 = I14
//   N13 = I13 + 3 I14                 N12 = I12 + 3 I14
//   N11 = I11 + 2 I13 + 3 I14         N10 = I10 + 2 I12 + 2 I13 + 6 I14
//   N9  = I9 + 2 I12 + 3 I14          N8  = I8 + I12 + I13 + 3 I14
//   N7  = I7 + I11 + I13 + I14        N6  = I6 + I9 + I10 + 2 I12 + I13 + 3 I14
//   N5  = I5 + 2 I8 + I10 + 2 I11 + 2 I12 + 4 I13 + 6 I14
//   N4  = I4 + 2 I8 + 2 I9 + I10 + 4 I12 + 2 I13 + 6 I14
//
// Kernels, after the CSR builder and the triangle stage (t_e complete):
//   k_loc_rows     per vertex, G lanes a row: t_v, S_v and the N6, N10, N13 sums
//   k_loc_cliques  per triangle owner u (lowest vertex): the induced subgraph
//                  on N+(u) as bitmap rows (LDS up to out-degree 512, device
//                  scratch beyond); every triangle credits its three vertices
//                  for N12, every 4-clique (row ANDs) its four for N14
//   k_loc_cycles   per 4-cycle owner u (highest vertex): wedge counters c[w]
//                  over the lower neighbours' rows; u and w gain C(c[w], 2),
//                  a middle vertex v the c[w] - 1 other middles of its wedge
//   k_loc_final    per vertex: the neighbour sums of N4 and N9, the inverse,
//                  and the row of the caller's vertex id
#include <algorithm>

#include "m4_ctx.h"
#include "m4_device.h"

namespace m4 {

namespace {

constexpr int LOC_NT = 256;
constexpr int LOC_NW = LOC_NT / WAVE;
constexpr int LOC_K_LDS = 512;             // out-degree bound of the LDS bitmap
constexpr int LOC_W_LDS = LOC_K_LDS / 64;  // its words per row
constexpr int LOC_SINGLE = 65536;          // heaviest 4-cycle owners taken one at a time
constexpr int LOC_CHUNK = 32;              // ... the rest in runs of this many ranks
constexpr int LOC_TRI_CHUNK = 16;          // triangle owners per grab
constexpr int CYC_NT = 512, CYC_NW = CYC_NT / WAVE;  // 4-cycle credits: 8 wavefronts per counter array
constexpr int ERR_LOCAL = 8;               // an orbit inverse went negative

struct LocIn {
  const int64_t* nptr;
  const int64_t* optr;
  const int32_t* ncol;
  const int32_t* dr;
  const int32_t* dlo;
  const int32_t* dplus;
  const uint32_t* t;
  const int32_t* perm;
  int64_t n;
};

// per-vertex statistics by rank
struct LocArrays {
  unsigned long long *tv, *S, *A6, *A10, *A13, *N8, *N12, *N14;
};

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int o) {
  return __shfl_xor(v, o, WAVE);
}

template <int G>
__device__ __forceinline__ unsigned long long group_sum(unsigned long long v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += shfl_xor_u64(v, o);
  return v;
}

// 128-bit sum over a group of G lanes (a carry per step)
template <int G>
__device__ __forceinline__ u128_t group_sum128(u128_t v) {
  unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const unsigned long long l2 = shfl_xor_u64(lo, o), h2 = shfl_xor_u64(hi, o);
    const unsigned long long s = lo + l2;
    hi = hi + h2 + (s < lo ? 1ull : 0ull);
    lo = s;
  }
  return ((u128_t)hi << 64) | lo;
}

// position of key in the sorted ncol[lo, hi), or -1
__device__ __forceinline__ int64_t find_in_row(const int32_t* __restrict__ a, int64_t lo,
                                               int64_t hi, int32_t key) {
  const int64_t p = lower_index(a, lo, hi, key);
  return (p < hi && a[p] == key) ? p : -1;
}

// t of the edge between v and its row entry u at position p of row v
__device__ __forceinline__ int64_t edge_t(const LocIn& in, int32_t v, int64_t p, int32_t u) {
  const int64_t vb = in.nptr[v];
  const int dl = in.dlo[v];
  if (p - vb >= dl) return in.t[in.optr[v] + (p - vb - dl)];
  // u is below v: the edge is u's out-edge to v
  const int64_t lo = in.nptr[u] + in.dlo[u], hi = in.nptr[u] + in.dr[u];
  const int64_t q = find_in_row(in.ncol, lo, hi, v);
  return q < 0 ? -1 : (int64_t)in.t[in.optr[u] + (q - lo)];
}

__device__ __forceinline__ void store_u64(unsigned long long* dst, u128_t v, Scal* scal) {
  if ((unsigned long long)(v >> 64)) scal->status = 3;
  *dst = (unsigned long long)v;
}

// ranks [r_lo, r_hi), G lanes per row
template <int G>
__global__ __launch_bounds__(256) void k_loc_rows(LocIn in, int64_t r_lo, int64_t r_hi,
                                                  LocArrays L, Scal* scal) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(gt % G);
  const int64_t groups = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t v = r_lo + gt / G; v < r_hi; v += groups) {
    const int64_t vb = in.nptr[v];
    const int d = in.dr[v];
    unsigned long long s = 0, t2 = 0;
    u128_t a6 = 0, a10 = 0, a13 = 0;
    bool bad = false;
    for (int p = j; p < d; p += G) {
      const int32_t u = in.ncol[vb + p];
      const unsigned long long du = (unsigned long long)in.dr[u];
      const int64_t te = edge_t(in, (int32_t)v, vb + p, u);
      if (te < 0) {
        bad = true;
        continue;
      }
      const unsigned long long tt = (unsigned long long)te;
      s += du - 1;
      t2 += tt;
      a6 += (u128_t)((du - 1) * (du >= 2 ? du - 2 : 0) / 2);
      if (tt) a10 += (u128_t)tt * (du - 2);  // a common neighbour makes d(u) >= 2
      a13 += (u128_t)(tt * (tt - (tt ? 1 : 0)) / 2);
    }
    if (bad) atomicOr(&scal->err, ERR_INVALID);
    s = group_sum<G>(s);
    t2 = group_sum<G>(t2);
    a6 = group_sum128<G>(a6);
    a10 = group_sum128<G>(a10);
    a13 = group_sum128<G>(a13);
    if (j == 0) {
      L.tv[v] = t2 / 2;
      L.S[v] = s;
      store_u64(&L.A6[v], a6, scal);
      store_u64(&L.A10[v], a10, scal);
      store_u64(&L.A13[v], a13, scal);
    }
  }
}

// A word of the clique kernel's bitmap or credit arrays, written by atomics of
// other wavefronts: from LDS, or from device scratch past the CU's L1 (the
// atomics are performed in the L2).
template <bool GLOB>
__device__ __forceinline__ unsigned long long ld_word(const unsigned long long* p) {
  if (GLOB) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

// A wavefront's bit list: in LDS, or in device scratch (written and read by
// the same wavefront; the device-scope loads skip the L1).
template <bool GLOB>
__device__ __forceinline__ int ld_list(const int32_t* p) {
  if (GLOB) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}
template <bool GLOB>
__device__ __forceinline__ void wave_list_sync() {
  if (GLOB) __threadfence();
  wave_sync();
}

// Triangle owners u (their lowest vertex) with out-degree k in [k_lo, k_hi],
// ranks from r_start up, LOC_TRI_CHUNK per grab.  Row i of the bitmap holds
// bit j when a[j] is in N+(a[i]), a = N+(u) (so j > i: rows are the
// induced subgraph's out-lists).  GLOB keeps the bitmap, the credit arrays
// and a in a per-block slice of device scratch (stride words).
template <bool GLOB>
__global__ __launch_bounds__(LOC_NT) void k_loc_cliques(LocIn in, LocArrays L, int64_t r_start,
                                                        int k_lo, int k_hi,
                                                        unsigned long long* gscr, int64_t stride,
                                                        unsigned int* work, Scal* scal) {
  __shared__ unsigned long long s_bits[GLOB ? 1 : LOC_K_LDS * LOC_W_LDS];
  __shared__ unsigned long long s_c12[GLOB ? 1 : LOC_K_LDS], s_c14[GLOB ? 1 : LOC_K_LDS];
  __shared__ int32_t s_a[GLOB ? 1 : LOC_K_LDS];
  __shared__ int32_t s_list[GLOB ? 1 : LOC_NW * LOC_K_LDS];
  __shared__ int64_t s_g;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  unsigned long long* bits;
  unsigned long long *c12, *c14;
  int32_t *a, *list;
  int64_t list_cap;
  if (GLOB) {
    unsigned long long* base = gscr + (int64_t)blockIdx.x * stride;
    const int64_t W = (k_hi + 63) / 64;
    bits = base;
    c12 = base + (int64_t)k_hi * W;
    c14 = c12 + k_hi;
    a = reinterpret_cast<int32_t*>(c14 + k_hi);
    list = a + k_hi;
    list_cap = k_hi;
  } else {
    bits = s_bits;
    c12 = s_c12;
    c14 = s_c14;
    a = s_a;
    list = s_list;
    list_cap = LOC_K_LDS;
  }
  for (;;) {
    if (tid == 0) s_g = (int64_t)atomicAdd(work, 1u) * LOC_TRI_CHUNK + r_start;
    __syncthreads();
    const int64_t u0 = s_g;
    __syncthreads();
    if (u0 >= in.n) break;
    const int64_t u1 = u0 + LOC_TRI_CHUNK < in.n ? u0 + LOC_TRI_CHUNK : in.n;
    for (int64_t u = u0; u < u1; u++) {
      const int k = in.dplus[u];
      if (k < 2 || k < k_lo || k > k_hi) continue;
      const int W = (k + 63) / 64;
      const int64_t ub = in.nptr[u] + in.dlo[u], oe = in.optr[u];
      for (int i = tid; i < k; i += LOC_NT) {
        a[i] = in.ncol[ub + i];
        c12[i] = 0;
        c14[i] = 0;
      }
      for (int64_t i = tid; i < (int64_t)k * W; i += LOC_NT) bits[i] = 0;
      __syncthreads();
      // rows: a wavefront per row, lanes over N+(a[i])
      unsigned long long cu12 = 0, cu14 = 0;
      for (int i = wv; i < k; i += LOC_NW) {
        const int32_t v = a[i];
        const int64_t vb = in.nptr[v] + in.dlo[v], ve = in.nptr[v] + in.dr[v], ov = in.optr[v];
        const unsigned long long t_uv = in.t[oe + i];
        unsigned long long ci = 0;
        for (int64_t p = vb + lane; p < ve; p += WAVE) {
          const int32_t x = in.ncol[p];
          // x in a[i+1 .. k)?
          int lo = i + 1, hi = k;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a[mid] < x) lo = mid + 1;
            else hi = mid;
          }
          if (lo < k && a[lo] == x) {
            const int jx = lo;
            atomicOr(&bits[(int64_t)i * W + (jx >> 6)], 1ull << (jx & 63));
            // triangle (u, v, x): each vertex gains t of its opposite edge - 1
            cu12 += (unsigned long long)in.t[ov + (p - vb)] - 1;
            ci += (unsigned long long)in.t[oe + jx] - 1;
            atomicAdd(&c12[jx], t_uv - 1);
          }
        }
        ci = group_sum<WAVE>(ci);
        if (lane == 0 && ci) atomicAdd(&c12[i], ci);
      }
      __syncthreads();
      // 4-cliques u < a[i] < a[j] < a[l]: bits l of row i AND row j, for
      // every bit j of row i.  A wavefront lists row i's bits (each lane
      // its words' bits at its offset of a wave prefix), then its lanes
      // take the listed j's.
      int32_t* lst = list + (int64_t)wv * list_cap;
      for (int i = wv; i < k; i += LOC_NW) {
        const unsigned long long* ri = bits + (int64_t)i * W;
        int mine = 0;
        for (int w = lane; w < W; w += WAVE) mine += __popcll(ld_word<GLOB>(ri + w));
        int incl = mine;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
          const int y = __shfl_up(incl, o, WAVE);
          if (lane >= o) incl += y;
        }
        const int total = __shfl(incl, WAVE - 1, WAVE);
        int q = incl - mine;
        for (int w = lane; w < W; w += WAVE) {
          unsigned long long m = ld_word<GLOB>(ri + w);
          while (m) {
            lst[q++] = w * 64 + __builtin_ctzll(m);
            m &= m - 1;
          }
        }
        wave_list_sync<GLOB>();
        unsigned long long ci = 0;
        for (int e = lane; e < total; e += WAVE) {
          const int jx = ld_list<GLOB>(lst + e);
          const unsigned long long* rj = bits + (int64_t)jx * W;
          unsigned long long cj = 0;
          for (int y = jx >> 6; y < W; y++) {
            unsigned long long andw = ld_word<GLOB>(ri + y) & ld_word<GLOB>(rj + y);
            cj += (unsigned long long)__popcll(andw);
            while (andw) {
              const int lx = y * 64 + __builtin_ctzll(andw);
              andw &= andw - 1;
              atomicAdd(&c14[lx], 1ull);
            }
          }
          if (cj) {
            ci += cj;
            cu14 += cj;
            atomicAdd(&c14[jx], cj);
          }
        }
        ci = group_sum<WAVE>(ci);
        if (lane == 0 && ci) atomicAdd(&c14[i], ci);
        // the list is rewritten for the next row only after every lane
        // has read it
        wave_list_sync<GLOB>();
      }
      __syncthreads();
      for (int i = tid; i < k; i += LOC_NT) {
        const unsigned long long x12 = ld_word<GLOB>(c12 + i), x14 = ld_word<GLOB>(c14 + i);
        if (x12) atomicAdd(&L.N12[a[i]], x12);
        if (x14) atomicAdd(&L.N14[a[i]], x14);
      }
      block_add_u64<LOC_NT>(&L.N12[u], cu12);
      block_add_u64<LOC_NT>(&L.N14[u], cu14);
    }
  }
}

// 4-cycle owners u (their highest vertex), heaviest first.  Each block keeps
// n wedge counters of type CT, all zero between owners: the low half counts
// a wedge endpoint's wedges in the first pass, the high half its visits in
// the second, whose last visitor credits the endpoint and clears the
// counter.  An endpoint's wedges come from distinct lower neighbours of u,
// so 16-bit halves hold them while degrees stay below 2^16.  The counters of
// the highest ranks (the hubs, where most wedges end) sit in LDS, the rest
// in the block's slice of device scratch.
constexpr int LOC_HOT_BYTES = 128 * 1024;

template <typename CT>
__device__ __forceinline__ CT hot_or_dev_add(CT* hot, CT* c, int32_t w, int64_t hot_base, CT v) {
  return w >= hot_base ? atomicAdd(&hot[w - hot_base], v) : atomicAdd(&c[w], v);
}

template <typename CT>
__global__ __launch_bounds__(CYC_NT) void k_loc_cycles(LocIn in, int64_t r1, LocArrays L,
                                                       CT* cscr, unsigned int* work) {
  constexpr int HALF = (int)sizeof(CT) * 4;
  constexpr CT LOC_LOW = (CT(1) << HALF) - 1;
  constexpr int HOT = LOC_HOT_BYTES / (int)sizeof(CT);
  __shared__ CT hot[HOT];
  __shared__ int64_t s_g;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int64_t n = in.n;
  const int64_t hot_base = n > HOT ? n - HOT : 0;
  CT* c = cscr + (int64_t)blockIdx.x * n;
  for (int i = tid; i < HOT; i += CYC_NT) hot[i] = 0;
  for (;;) {
    if (tid == 0) s_g = (int64_t)atomicAdd(work, 1u);
    __syncthreads();
    const int64_t g = s_g;
    __syncthreads();
    int64_t hi, lo;  // owners hi, hi - 1, ..., lo + 1
    if (g < LOC_SINGLE) {
      hi = n - 1 - g;
      lo = hi - 1;
    } else {
      hi = n - 1 - LOC_SINGLE - (g - LOC_SINGLE) * LOC_CHUNK;
      lo = hi - LOC_CHUNK;
    }
    if (hi < r1) break;
    if (lo < r1 - 1) lo = r1 - 1;
    for (int64_t u = hi; u > lo; u--) {
      const int nl = in.dlo[u];
      if (nl < 2) continue;
      const int64_t ub = in.nptr[u];
      // pass 1: c[w] for the wedges u - v - w with v, w below u; the old
      // values sum to the cycles at u
      unsigned long long pairs = 0;
      for (int i = wv; i < nl; i += CYC_NW) {
        const int32_t v = in.ncol[ub + i];
        const int64_t vb = in.nptr[v];
        const int64_t pe = lower_index(in.ncol, vb, vb + in.dr[v], (int32_t)u);
        for (int64_t p = vb + lane; p < pe; p += WAVE)
          pairs += (unsigned long long)(hot_or_dev_add(hot, c, in.ncol[p], hot_base, CT(1)) &
                                        LOC_LOW);
      }
      __syncthreads();
      // pass 2: a middle vertex v shares each of its wedges with c[w] - 1
      // others; the c[w]-th visit of w gives w its C(c[w], 2) cycles with
      // u and clears the counter
      for (int i = wv; i < nl; i += CYC_NW) {
        const int32_t v = in.ncol[ub + i];
        const int64_t vb = in.nptr[v];
        const int64_t pe = lower_index(in.ncol, vb, vb + in.dr[v], (int32_t)u);
        unsigned long long acc = 0;
        for (int64_t p = vb + lane; p < pe; p += WAVE) {
          const int32_t w = in.ncol[p];
          const CT old = hot_or_dev_add(hot, c, w, hot_base, CT(1) << HALF);
          const unsigned long long k = (unsigned long long)(old & LOC_LOW);
          acc += k - 1;
          if ((unsigned long long)(old >> HALF) == k - 1) {
            if (w >= hot_base) atomicExch(&hot[w - hot_base], CT(0));
            else atomicExch(&c[w], CT(0));
            if (k >= 2) atomicAdd(&L.N8[w], k * (k - 1) / 2);
          }
        }
        acc = group_sum<WAVE>(acc);
        if (lane == 0 && acc) atomicAdd(&L.N8[v], acc);
      }
      block_add_u64<CYC_NT>(&L.N8[u], pairs);
    }
  }
}

__device__ __forceinline__ __int128 c3(__int128 d) { return d >= 3 ? d * (d - 1) * (d - 2) / 6 : 0; }

template <int G>
__global__ __launch_bounds__(256) void k_loc_final(LocIn in, int64_t r_lo, int64_t r_hi,
                                                   LocArrays L, unsigned long long* out,
                                                   Scal* scal) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(gt % G);
  const int64_t groups = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t v = r_lo + gt / G; v < r_hi; v += groups) {
    const int64_t vb = in.nptr[v];
    const int d = in.dr[v];
    u128_t b4 = 0;
    unsigned long long b9 = 0;
    for (int p = j; p < d; p += G) {
      const int32_t a = in.ncol[vb + p];
      b4 += (u128_t)L.S[a];
      b9 += L.tv[a];
    }
    b4 = group_sum128<G>(b4);
    b9 = group_sum<G>(b9);
    if (j != 0) continue;
    typedef __int128 i128;
    const i128 dd = d, tv = (i128)L.tv[v];
    i128 N[15];
    N[4] = (i128)b4 - dd * (dd - 1) - 2 * tv;
    N[5] = (dd - 1) * (i128)L.S[v] - 2 * tv;
    N[6] = (i128)L.A6[v];
    N[7] = c3(dd);
    N[8] = (i128)L.N8[v];
    N[9] = (i128)b9 - 2 * tv;
    N[10] = (i128)L.A10[v];
    N[11] = d >= 2 ? tv * (dd - 2) : 0;
    N[12] = (i128)L.N12[v];
    N[13] = (i128)L.A13[v];
    N[14] = (i128)L.N14[v];
    i128 I[15];
    I[14] = N[14];
    I[13] = N[13] - 3 * I[14];
    I[12] = N[12] - 3 * I[14];
    I[11] = N[11] - 2 * I[13] - 3 * I[14];
    I[10] = N[10] - 2 * I[12] - 2 * I[13] - 6 * I[14];
    I[9] = N[9] - 2 * I[12] - 3 * I[14];
    I[8] = N[8] - I[12] - I[13] - 3 * I[14];
    I[7] = N[7] - I[11] - I[13] - I[14];
    I[6] = N[6] - I[9] - I[10] - 2 * I[12] - I[13] - 3 * I[14];
    I[5] = N[5] - 2 * I[8] - I[10] - 2 * I[11] - 2 * I[12] - 4 * I[13] - 6 * I[14];
    I[4] = N[4] - 2 * I[8] - 2 * I[9] - I[10] - 4 * I[12] - 2 * I[13] - 6 * I[14];
    unsigned long long* row = out + (int64_t)in.perm[v] * 11;
    for (int o = 4; o <= 14; o++) {
      if (I[o] < 0) atomicOr(&scal->err, ERR_LOCAL);
      else if ((I[o] >> 64) != 0) scal->status = 3;
      row[o - 4] = (unsigned long long)I[o];
    }
  }
}

__global__ void k_loc_dplus_max(const int32_t* __restrict__ dplus, int64_t n,
                                unsigned int* __restrict__ out) {
  unsigned int k = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    k = std::max(k, (unsigned int)dplus[v]);
  for (int o = WAVE / 2; o > 0; o >>= 1) k = std::max(k, (unsigned int)__shfl_xor((int)k, o, WAVE));
  if ((threadIdx.x & (WAVE - 1)) == 0 && k) atomicMax(out, k);
}

}  // namespace

// Orbit counts of the prepared graph P (t complete) into out (uint64[n][11],
// device memory, caller's vertex ids).  arrays: 8 n words; cscr: the 4-cycle
// counters, cblocks x n of 32 bits (64 when wide: degrees of 2^16 and more); gscr: the bitmap slices of out-degrees above
// the LDS bound (kmax > LOC_K_LDS), gblocks slices.
void local_orbits(const Prep& P, const Classes& C, Scal* scal, unsigned long long* arrays,
                  void* cscr, bool wide, int cblocks, unsigned long long* gscr, int gblocks,
                  int kmax, unsigned long long* out, int num_cu, hipStream_t s) {
  const int64_t n = P.n;
  LocIn in{P.nptr, P.optr, P.ncol, P.dr, P.dlo, P.dplus, P.t, P.perm, n};
  LocArrays L{arrays,         arrays + n,     arrays + 2 * n, arrays + 3 * n,
              arrays + 4 * n, arrays + 5 * n, arrays + 6 * n, arrays + 7 * n};
  fill_u32(arrays, 0, (size_t)n * 16, s);
  fill_u32(&scal->work[0], 0, 8, s);
  const int64_t b64 = std::min<int64_t>(C.bound[4], n);  // degree <= 64: 8 lanes a row
  const unsigned cap = (unsigned)num_cu * 64;
  auto grid_for = [&](int64_t rows, int G) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows * G, 256), cap));
  };
  if (b64 > 0) k_loc_rows<8><<<grid_for(b64, 8), 256, 0, s>>>(in, 0, b64, L, scal);
  if (n > b64) k_loc_rows<64><<<grid_for(n - b64, 64), 256, 0, s>>>(in, b64, n, L, scal);
  // triangle owners have out-degree >= 2, so degree >= 2
  const int64_t r_tri = std::min<int64_t>(C.bound[0], n);
  k_loc_cliques<false><<<(unsigned)(num_cu * 4), LOC_NT, 0, s>>>(in, L, r_tri, 2, LOC_K_LDS,
                                                                 nullptr, 0, &scal->work[0], scal);
  if (kmax > LOC_K_LDS && gblocks > 0) {
    // out-degree above 512 needs degree above 256
    const int64_t stride = (int64_t)local_glob_stride_words(kmax);
    k_loc_cliques<true><<<(unsigned)gblocks, LOC_NT, 0, s>>>(
        in, L, std::min<int64_t>(C.bound[5], n), LOC_K_LDS + 1, kmax, gscr, stride,
        &scal->work[1], scal);
  }
  if (cblocks > 0) {
    fill_u32(cscr, 0, (size_t)cblocks * (size_t)n * (wide ? 2 : 1), s);
    if (wide)
      k_loc_cycles<unsigned long long><<<(unsigned)cblocks, CYC_NT, 0, s>>>(
          in, C.r1, L, reinterpret_cast<unsigned long long*>(cscr), &scal->work[2]);
    else
      k_loc_cycles<unsigned int><<<(unsigned)cblocks, CYC_NT, 0, s>>>(
          in, C.r1, L, reinterpret_cast<unsigned int*>(cscr), &scal->work[2]);
  }
  if (b64 > 0) k_loc_final<8><<<grid_for(b64, 8), 256, 0, s>>>(in, 0, b64, L, out, scal);
  if (n > b64) k_loc_final<64><<<grid_for(n - b64, 64), 256, 0, s>>>(in, b64, n, L, out, scal);
}

int local_dplus_max(const Prep& P, Scal* scal, hipStream_t s) {
  fill_u32(&scal->work[3], 0, 1, s);
  const int64_t n = P.n;
  k_loc_dplus_max<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096)), 256,
                    0, s>>>(P.dplus, n, &scal->work[3]);
  unsigned int k = 0;
  M4_HIP(hipMemcpyAsync(&k, &scal->work[3], 4, hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  return (int)k;
}

// per block: the bitmap (kmax rows of ceil(kmax / 64) words), the two
// credit arrays, a (kmax int32) and one bit list per wavefront (kmax int32)
size_t local_glob_stride_words(int kmax) {
  const int64_t W = (kmax + 63) / 64;
  return (size_t)((int64_t)kmax * W + 2 * (int64_t)kmax + ((int64_t)kmax * (1 + LOC_NW) + 1) / 2);
}

}  // namespace m4
