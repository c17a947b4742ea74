// m4_build.hip -- CSR builder: degrees, degree order, relabelled sorted rows
// and the oriented out-list offsets.
//
// The canonical order is (degree, id) (Section III-D: sorted CSR adjacency
// and canonical ordering constraints).  Vertex v is renamed rank(v), its
// position in that order, so that "u precedes w" is the integer test u < w,
// every row in rank space is sorted, and the out-list N+(r) (neighbours of
// higher rank) is the suffix of row r that starts at dlo[r].
#include <limits.h>

#include <type_traits>
#include <utility>

#include "m4_internal.h"

namespace m4 {

namespace {

__global__ void k_degree(const int64_t* __restrict__ rp, int64_t n, uint32_t* __restrict__ deg,
                         Scal* scal) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t d = 0;
  if (v < n) {
    d = (uint32_t)(rp[v + 1] - rp[v]);
    deg[v] = d;
  }
  // block max, one atomic per block
  __shared__ uint32_t bmax;
  if (threadIdx.x == 0) bmax = 0;
  __syncthreads();
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    uint32_t e = __shfl_xor(d, o, WAVE);
    d = d > e ? d : e;
  }
  if ((threadIdx.x & (WAVE - 1)) == 0 && d) atomicMax(&bmax, d);
  __syncthreads();
  if (threadIdx.x == 0 && bmax) atomicMax(&scal->dmax, bmax);
}

__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ rp, int64_t n, int64_t q) {
  int64_t lo = 0, hi = n;  // last v with rp[v] <= q
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (rp[mid] <= q) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool has(const int32_t* __restrict__ col, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (col[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return col[lo] == x;
}

__global__ void k_validate_rows(const int64_t* __restrict__ rp, int64_t n, int64_t nnz, Scal* scal) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  bool bad = false;
  if (v == 0 && rp[0] != 0) bad = true;
  if (v == n && rp[n] != nnz) bad = true;
  if (v < n && rp[v + 1] < rp[v]) bad = true;
  if (bad) atomicOr(&scal->err, ERR_INVALID);
}

__global__ void k_validate_entries(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                   int64_t n, int64_t nnz, Scal* scal) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  int64_t v = row_of(rp, n, q);
  int32_t x = col[q];
  bool bad = x < 0 || x >= n || x == v || (q > rp[v] && col[q - 1] >= x);
  if (!bad) {
    int64_t lo = rp[x], hi = rp[x + 1];
    bad = lo >= hi || !has(col, lo, hi - 1, (int32_t)v);
  }
  if (bad) atomicOr(&scal->err, ERR_INVALID);
}

__global__ void k_identity(int32_t* __restrict__ p, uint32_t* __restrict__ k, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    p[i] = (int32_t)i;
    k[i] = 0;
  }
}

__global__ void k_rank(const int32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ rank) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) rank[perm[r]] = (int32_t)r;
}

// First rank whose degree exceeds each threshold (degrees are sorted).
__global__ void k_classes(const int32_t* __restrict__ dr, int64_t n, const int* thr, int nthr,
                          int64_t* __restrict__ out) {
  int i = threadIdx.x;
  if (i >= nthr) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (dr[mid] <= thr[i]) lo = mid + 1;
    else hi = mid;
  }
  out[i] = lo;
}

// Rows of degree <= G: G lanes per row; each lane maps one neighbour to its
// rank and computes its sorted position by comparing with the other lanes.
template <int G>
__global__ __launch_bounds__(256) void k_row_small(const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ rank,
                                                   const int64_t* __restrict__ nptr,
                                                   const int32_t* __restrict__ dr, int64_t r_lo,
                                                   int64_t r_hi, int32_t* __restrict__ ncol,
                                                   int32_t* __restrict__ dlo,
                                                   int32_t* __restrict__ dplus, int64_t r_base) {
  // r is the rank (compared with the relabelled neighbours); li = r - r_base
  // indexes the per-row arrays, which may hold a chunk of rows only
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t r = r_lo + t / G;
  int j = (int)(t % G);
  bool rowok = r < r_hi;
  const int64_t li = rowok ? r - r_base : 0;
  int d = rowok ? dr[li] : 0;
  bool mine = rowok && j < d;
  int32_t x = INT_MAX;
  if (mine) x = rank[col[rp[perm[li]] + j]];
  const int lane = threadIdx.x & (WAVE - 1);
  const int gbase = lane & ~(G - 1);
  int pos = 0;
#pragma unroll
  for (int k = 0; k < G; k++) {
    int32_t y = __shfl(x, gbase + k, WAVE);
    pos += (y < x);
  }
  uint64_t below = __ballot(mine && x < r);
  uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1) << gbase);
  if (mine) ncol[nptr[li] + pos] = x;
  if (rowok && j == 0) {
    int b = __popcll(below & gmask);
    dlo[li] = b;
    dplus[li] = d - b;
  }
}

// Rows of degree in (64, CAP]: one workgroup, bitonic sort in LDS.
template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_row_bitonic(const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ rank,
                                                    const int64_t* __restrict__ nptr,
                                                    const int32_t* __restrict__ dr, int64_t r_lo,
                                                    int32_t* __restrict__ ncol,
                                                    int32_t* __restrict__ dlo,
                                                    int32_t* __restrict__ dplus, int64_t r_base) {
  __shared__ int32_t s[CAP];
  __shared__ int below;
  const int64_t r = r_lo + blockIdx.x, li = r - r_base;
  const int d = dr[li];
  const int64_t in0 = rp[perm[li]];
  int P = 1;
  while (P < d) P <<= 1;
  if (threadIdx.x == 0) below = 0;
  __syncthreads();
  int mybelow = 0;
  for (int i = threadIdx.x; i < P; i += NT) {
    int32_t x = INT_MAX;
    if (i < d) {
      x = rank[col[in0 + i]];
      mybelow += (x < r);
    }
    s[i] = x;
  }
  if (mybelow) atomicAdd(&below, mybelow);
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = threadIdx.x; i < P; i += NT) {
        int ixj = i ^ jj;
        if (ixj > i) {
          int32_t a = s[i], b = s[ixj];
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
  int32_t* out = ncol + nptr[li];
  for (int i = threadIdx.x; i < d; i += NT) out[i] = s[i];
  if (threadIdx.x == 0) {
    dlo[li] = below;
    dplus[li] = d - below;
  }
}

// Rows longer than the LDS sort: set bits of a 2^20-wide window of ranks in
// an LDS bitmap and emit them in order, window after window.
constexpr int BM_NT = 1024, BM_WORDS = 32768;  // 1M bits = 128 KiB
__global__ __launch_bounds__(BM_NT) void k_row_bitmap(const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ rank,
                                                      const int64_t* __restrict__ nptr,
                                                      const int32_t* __restrict__ dr, int64_t n,
                                                      int64_t r_lo, int32_t* __restrict__ ncol,
                                                      int32_t* __restrict__ dlo,
                                                      int32_t* __restrict__ dplus, int64_t r_base) {
  __shared__ uint32_t bm[BM_WORDS];
  __shared__ int64_t wsum[BM_NT / WAVE];
  __shared__ int below;
  const int64_t r = r_lo + blockIdx.x, li = r - r_base;
  const int d = dr[li];
  const int64_t in0 = rp[perm[li]];
  int32_t* out = ncol + nptr[li];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  if (tid == 0) below = 0;
  int64_t written = 0;
  int mybelow = 0;
  for (int64_t lo = 0; lo < n; lo += (int64_t)BM_WORDS * 32) {
    for (int i = tid; i < BM_WORDS; i += BM_NT) bm[i] = 0;
    __syncthreads();
    for (int i = tid; i < d; i += BM_NT) {
      int64_t x = rank[col[in0 + i]];
      if (lo == 0) mybelow += (x < r);
      if (x >= lo && x < lo + (int64_t)BM_WORDS * 32) {
        int64_t o = x - lo;
        atomicOr(&bm[o >> 5], 1u << (o & 31));
      }
    }
    __syncthreads();
    constexpr int PER = BM_WORDS / BM_NT;
    int64_t c = 0;
#pragma unroll
    for (int k = 0; k < PER; k++) c += __popc(bm[tid * PER + k]);
    int64_t inc = c;
    for (int o = 1; o < WAVE; o <<= 1) {
      int64_t u = __shfl_up(inc, o, WAVE);
      if (lane >= o) inc += u;
    }
    if (lane == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, tot = 0;
    for (int k = 0; k < BM_NT / WAVE; k++) {
      if (k < w) before += wsum[k];
      tot += wsum[k];
    }
    int64_t pos = written + before + inc - c;
    for (int k = 0; k < PER; k++) {
      uint32_t word = bm[tid * PER + k];
      while (word) {
        int b = __ffs(word) - 1;
        word &= word - 1;
        out[pos++] = (int32_t)(lo + (int64_t)(tid * PER + k) * 32 + b);
      }
    }
    written += tot;
    __syncthreads();
  }
  if (mybelow) atomicAdd(&below, mybelow);
  __syncthreads();
  if (tid == 0) {
    dlo[li] = below;
    dplus[li] = d - below;
  }
}

__global__ void k_edge_t_out(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             int64_t n, int64_t nnz, const int32_t* __restrict__ rank,
                             const int64_t* __restrict__ nptr, const int32_t* __restrict__ dlo,
                             const int64_t* __restrict__ optr, const int32_t* __restrict__ ncol,
                             const uint32_t* __restrict__ t, uint32_t* __restrict__ t_out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  int64_t v = row_of(rp, n, q);
  int32_t a = rank[v], b = rank[col[q]];
  int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  int64_t s = nptr[lo] + dlo[lo], e = nptr[lo + 1];
  int64_t l = s, h = e;
  while (l < h) {
    int64_t mid = (l + h) >> 1;
    if (ncol[mid] < hi) l = mid + 1;
    else h = mid;
  }
  t_out[q] = t[optr[lo] + (l - s)];
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)ceil_div(n > 0 ? n : 1, nt); }

}  // namespace

// Degree thresholds of the row-sort classes; the same table decides which
// kernel sorts each rank range.
static const int kThr[] = {1, 8, 16, 32, 64, 256, 1024, 2048, 8192, 16384};
static constexpr int kNThr = sizeof(kThr) / sizeof(kThr[0]);

void sort_rows(const int64_t* rp, const int32_t* col, const int32_t* perm, const int32_t* rank,
               const int64_t* nptr, const int32_t* dr, int64_t n, int64_t r_lo, int64_t r_hi,
               const int64_t* bnd, int32_t* ncol, int32_t* dlo, int32_t* dplus, int64_t r_base,
               hipStream_t s) {
  // class boundaries clipped to [r_lo, r_hi)
  int64_t b[kNThr];
  for (int i = 0; i < kNThr; i++) b[i] = std::min(std::max(bnd[i], r_lo), r_hi);
  auto small = [&](auto tag, int64_t lo, int64_t hi) {
    constexpr int G = decltype(tag)::value;
    if (hi <= lo) return;
    int64_t threads = (hi - lo) * G;
    k_row_small<G><<<blocks_for(threads, 256), 256, 0, s>>>(rp, col, perm, rank, nptr, dr, lo, hi,
                                                            ncol, dlo, dplus, r_base);
  };
  small(std::integral_constant<int, 1>{}, r_lo, b[0]);
  small(std::integral_constant<int, 8>{}, b[0], b[1]);
  small(std::integral_constant<int, 16>{}, b[1], b[2]);
  small(std::integral_constant<int, 32>{}, b[2], b[3]);
  small(std::integral_constant<int, 64>{}, b[3], b[4]);
  if (b[5] > b[4])
    k_row_bitonic<256, 128><<<(unsigned)(b[5] - b[4]), 128, 0, s>>>(
        rp, col, perm, rank, nptr, dr, b[4], ncol, dlo, dplus, r_base);
  if (b[6] > b[5])
    k_row_bitonic<1024, 256><<<(unsigned)(b[6] - b[5]), 256, 0, s>>>(
        rp, col, perm, rank, nptr, dr, b[5], ncol, dlo, dplus, r_base);
  if (b[7] > b[6])
    k_row_bitonic<2048, 512><<<(unsigned)(b[7] - b[6]), 512, 0, s>>>(
        rp, col, perm, rank, nptr, dr, b[6], ncol, dlo, dplus, r_base);
  // up to 16384 entries a row is one bitonic sort in LDS (gathering each
  // entry's rank once); longer rows take the bitmap windows
  if (b[8] > b[7])
    k_row_bitonic<8192, 1024><<<(unsigned)(b[8] - b[7]), 1024, 0, s>>>(
        rp, col, perm, rank, nptr, dr, b[7], ncol, dlo, dplus, r_base);
  if (b[9] > b[8])
    k_row_bitonic<16384, 1024><<<(unsigned)(b[9] - b[8]), 1024, 0, s>>>(
        rp, col, perm, rank, nptr, dr, b[8], ncol, dlo, dplus, r_base);
  if (r_hi > b[9])
    k_row_bitmap<<<(unsigned)(r_hi - b[9]), BM_NT, 0, s>>>(rp, col, perm, rank, nptr, dr, n, b[9],
                                                           ncol, dlo, dplus, r_base);
}

int row_class_count() { return kNThr; }
const int* row_class_thresholds() { return kThr; }

void degree_order(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz, bool validate,
                  Prep& P, Classes& C, Scal* scal, Scal* scal_host, Arena& tmp, hipStream_t s) {
  P.n = n;
  P.nnz = nnz;
  P.m = nnz / 2;
  const int NT = 256;
  if (validate) {
    k_validate_rows<<<blocks_for(n + 1, NT), NT, 0, s>>>(rp, n, nnz, scal);
    if (nnz > 0) k_validate_entries<<<blocks_for(nnz, NT), NT, 0, s>>>(rp, col, n, nnz, scal);
  }
  // degrees and the stable sort by degree
  uint32_t* kA = tmp.take<uint32_t>(n);
  uint32_t* kB = tmp.take<uint32_t>(n);
  int32_t* vB = tmp.take<int32_t>(n);
  int64_t* rtmp = tmp.take<int64_t>(radix_tmp_elems(n, 8));
  if (!kA || !kB || !vB || !rtmp) throw Fail(M4_EINTERNAL, "workspace too small (build)");
  k_degree<<<blocks_for(n, 1024), 1024, 0, s>>>(rp, n, kA, scal);
  M4_HIP(hipMemcpyAsync(scal_host, scal, sizeof(Scal), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  if (scal_host->err) throw Fail(M4_EINVAL, "CSR is not simple, symmetric and sorted");
  const uint32_t dmax = scal_host->dmax;
  C.dmax = (int)dmax;
  int passes = 0;
  while (passes < 4 && (dmax >> (8 * passes)) != 0) passes++;
  uint32_t* kin = kA;
  int32_t* vin = nullptr;  // identity on the first pass
  uint32_t* kout = kB;
  int32_t* vout = P.perm;
  int32_t* vother = vB;
  for (int p = 0; p < passes; p++) {
    radix_pass(kin, vin, n, 8 * p, 8, kout, vout, rtmp, nullptr, s);
    std::swap(kin, kout);
    vin = vout;
    std::swap(vout, vother);
  }
  // sorted degrees are in kin, the permutation in vin
  if (passes == 0) {
    k_identity<<<blocks_for(n, NT), NT, 0, s>>>(P.perm, kB, n);
    kin = kB;
    vin = P.perm;
  }
  if (vin != P.perm)
    M4_HIP(hipMemcpyAsync(P.perm, vin, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  M4_HIP(hipMemcpyAsync(P.dr, kin, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  k_rank<<<blocks_for(n, NT), NT, 0, s>>>(P.perm, n, P.rank);
  int64_t* stmp = tmp.take<int64_t>(scan_tmp_elems(n));
  int* thr_d = tmp.take<int>(kNThr);
  int64_t* bounds_d = tmp.take<int64_t>(kNThr);
  if (!stmp || !thr_d || !bounds_d) throw Fail(M4_EINTERNAL, "workspace too small (build)");
  scan_i32(P.dr, n, P.nptr, stmp, s);
  M4_HIP(hipMemcpyAsync(thr_d, kThr, sizeof(kThr), hipMemcpyHostToDevice, s));
  k_classes<<<1, 64, 0, s>>>(P.dr, n, thr_d, kNThr, bounds_d);
  int64_t b[kNThr];
  M4_HIP(hipMemcpyAsync(b, bounds_d, sizeof(b), hipMemcpyDeviceToHost, s));
  M4_HIP(hipStreamSynchronize(s));
  C.r1 = b[0];
  for (int i = 0; i < kNThr; i++) C.bound[i] = b[i];
}

void build_prep(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz, bool validate,
                Prep& P, Classes& C, Scal* scal, Scal* scal_host, Arena& tmp, hipStream_t s) {
  degree_order(rp, col, n, nnz, validate, P, C, scal, scal_host, tmp, s);
  // relabel and sort every row, by degree class
  sort_rows(rp, col, P.perm, P.rank, P.nptr, P.dr, n, 0, n, C.bound, P.ncol, P.dlo, P.dplus, 0, s);
  int64_t* stmp = tmp.take<int64_t>(scan_tmp_elems(n));
  if (!stmp) throw Fail(M4_EINTERNAL, "workspace too small (build)");
  scan_i32(P.dplus, n, P.optr, stmp, s);
}

void edge_t_to_input(const Prep& P, const int64_t* rp, const int32_t* col, uint32_t* t_out,
                     hipStream_t s) {
  if (P.nnz == 0) return;
  k_edge_t_out<<<blocks_for(P.nnz, 256), 256, 0, s>>>(rp, col, P.n, P.nnz, P.rank, P.nptr, P.dlo,
                                                      P.optr, P.ncol, P.t, t_out);
}

size_t build_tmp_bytes(int64_t n, int64_t nnz) {
  (void)nnz;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(n * 4);
  add(n * 4);
  add(n * 4);
  add(radix_tmp_elems(n, 8) * 8);
  add(scan_tmp_elems(n) * 8);
  add(scan_tmp_elems(n) * 8);
  add(64 * 4);
  add(64 * 8);
  return b + 4096;
}

}  // namespace m4
