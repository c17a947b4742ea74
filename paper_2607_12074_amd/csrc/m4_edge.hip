// m4_edge.hip -- the edge-anchor basis of the path / cycle counts and the
// anchor-selection objective that chooses between it and the wedge basis
// (Sections III-A and III-F).
//
// For an edge e = (u, v) with C_e = N(u) ∩ N(v), A_e = N(u) \ (C_e ∪ {v}) and
// B_e = N(v) \ (C_e ∪ {u}), a pair (x, y) of A_e × B_e is an induced 4-path
// x-u-v-y when x and y are not adjacent and an induced 4-cycle when they are
// (Section III-F).  The only statistic this basis adds to the triangle
// anchor's is Z = Σ_e |{(x, y) ∈ A_e × B_e : (x, y) ∈ E}| = 4 · cycle; then
// C4_ni = Z / 4 + D_ni - 3 K4 (every 4-cycle subgraph is an induced 4-cycle,
// a diamond or one of the three in a 4-clique), and the closure inverse runs
// unchanged.  The wedge basis instead counts C4_ni directly, each cycle once
// at its highest vertex (m4_c4.hip).
#include <math.h>

#include <algorithm>

#include "m4_ctx.h"
#include "m4_device.h"

namespace m4 {

namespace {

// index of key in the sorted a[lo, hi), or -1
__device__ __forceinline__ int64_t find_sorted(const int32_t* __restrict__ a, int64_t lo,
                                               int64_t hi, int32_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t v = a[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// Inputs of the objective, exact from the prepared graph: the wedge
// endpoints the wedge basis streams, sum over v of (d(v) - 1) d+(v) (every
// lower neighbour v of an owner lends its row but the owner), and the row
// entries the edge basis scans, sum over u of d+(u) * sum over a in N(u) of
// d(a) (each edge owned by its lower end scans the rows of the lower end's
// neighbours).  The first pass reads degrees only and gives the wedge term
// and a lower bound of the edge term (every neighbour has degree >= 1 and u
// itself is in each neighbour's row: sum over u of d+(u) d(u)); the second
// reads the rows and is run only when that bound does not settle the
// choice.
__global__ void k_edge_cost(const int32_t* __restrict__ dr, const int32_t* __restrict__ dplus,
                            int64_t n, unsigned long long* __restrict__ out) {
  unsigned long long wedge = 0, lower = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = dr[u];
    if (d >= 2) wedge += (unsigned long long)(d - 1) * (unsigned long long)dplus[u];
    lower += (unsigned long long)d * (unsigned long long)dplus[u];
  }
  block_add_u64<256>(&out[0], wedge);
  block_add_u64<256>(&out[1], lower);
}

__global__ void k_edge_scan_cost(const int64_t* __restrict__ nptr,
                                 const int32_t* __restrict__ ncol,
                                 const int32_t* __restrict__ dr,
                                 const int32_t* __restrict__ dplus, int64_t n,
                                 unsigned long long* __restrict__ out) {
  unsigned long long scan = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    if (dplus[u] == 0) continue;
    unsigned long long sum = 0;
    for (int64_t p = nptr[u]; p < nptr[u] + dr[u]; p++) sum += (unsigned long long)dr[ncol[p]];
    scan += sum * (unsigned long long)dplus[u];
  }
  block_add_u64<256>(out, scan);
}

// Z over the edges owned by their lower end: one 256-thread workgroup per
// owner u at a time (persistent, owners from a counter), its threads over
// the pairs (v, x) with v in N+(u) and x in N(u); for x in A_e, every y in
// N(x) that lies in N(v) but not in N(u) ∪ {u} is an adjacent pair.  Rows
// are sorted, so membership is a binary search.
__global__ __launch_bounds__(256) void k_edge_pairs(const int64_t* __restrict__ nptr,
                                                     const int32_t* __restrict__ ncol,
                                                     const int32_t* __restrict__ dr,
                                                     const int32_t* __restrict__ dlo, int64_t n,
                                                     unsigned int* work, Scal* scal,
                                                     uint32_t flags) {
  __shared__ int s_u;
  u128_t z = 0;
  unsigned long long scanned = 0, pairs = 0, owners = 0;
  for (;;) {
    if (threadIdx.x == 0) s_u = (int)atomicAdd(work, 1u);
    __syncthreads();
    const int64_t u = s_u;
    __syncthreads();
    if (u >= n) break;
    const int64_t ub = nptr[u], d = dr[u], dl = dlo[u];
    const int64_t np = (d - dl) * d;  // (v, x) pairs
    if (threadIdx.x == 0 && np > 0) owners++;
    for (int64_t q = threadIdx.x; q < np; q += 256) {
      const int32_t v = ncol[ub + dl + q / d];
      const int32_t x = ncol[ub + q % d];
      pairs++;
      if (x == v) continue;
      const int64_t vb = nptr[v], ve = vb + dr[v];
      if (find_sorted(ncol, vb, ve, x) >= 0) continue;  // x in C_e
      const int64_t xb = nptr[x], xe = xb + dr[x];
      scanned += (unsigned long long)(xe - xb);
      for (int64_t p = xb; p < xe; p++) {
        const int32_t y = ncol[p];
        if (y == (int32_t)u) continue;
        if (find_sorted(ncol, vb, ve, y) < 0) continue;      // y not in N(v)
        if (find_sorted(ncol, ub, ub + d, y) >= 0) continue;  // y in C_e
        z += 1;
      }
    }
  }
  block_add_u128<256>(&scal->acc[ACC_Z], z);
  if (flags & M4_STATS) {
    block_add_u64<256>(&scal->kstat[M4_K_EDGE][0], scanned);
    block_add_u64<256>(&scal->kstat[M4_K_EDGE][1], owners);
    block_add_u64<256>(&scal->kstat[M4_K_EDGE][2], pairs);
  }
}

}  // namespace

BasisChoice choose_basis(const Prep& P, const Tuning& tu, uint32_t flags, bool budgeted,
                         Scal* scal, unsigned long long* host_pair, hipStream_t s) {
  BasisChoice b;
  host_pair[0] = host_pair[1] = 0;
  const bool forced = (flags & (M4_BASIS_WEDGE | M4_BASIS_EDGE)) != 0;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(std::max<int64_t>(P.n, 1), 256), 4096);
  if (P.n > 0) {
    k_edge_cost<<<grid, 256, 0, s>>>(P.dr, P.dplus, P.n, &scal->stat[ST_COST]);
    M4_HIP(hipMemcpyAsync(host_pair, &scal->stat[ST_COST], 16, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
  }
  // Eq. (1) over the two cycle/path bases: the triangle anchor, the
  // recoverable counts (closure yield: all six for both) and the reuse
  // (none for either) are shared and drop out; enumeration plus
  // intersection work, each element weighted by its measured cost on this
  // device, plus a fixed stage cost (launches and the host read-backs of the
  // wedge plan), and the halo term: the edge basis reads 2-hop rows, which
  // the halo partitions do not hold, so it is infinite under a budget.
  b.cost_wedge = tu.cost_wedge_ns * (double)host_pair[0] + tu.cost_wedge_fixed_us * 1e3;
  b.cost_edge = tu.cost_edge_ns * (double)host_pair[1];  // a lower bound so far
  if (budgeted) {
    b.cost_edge = INFINITY;
  } else if (P.n > 0 && (b.cost_edge < b.cost_wedge || forced)) {
    fill_u32(&scal->stat[ST_COST + 1], 0, 2, s);
    k_edge_scan_cost<<<grid, 256, 0, s>>>(P.nptr, P.ncol, P.dr, P.dplus, P.n,
                                          &scal->stat[ST_COST + 1]);
    M4_HIP(hipMemcpyAsync(host_pair + 1, &scal->stat[ST_COST + 1], 8, hipMemcpyDeviceToHost, s));
    M4_HIP(hipStreamSynchronize(s));
    b.cost_edge = tu.cost_edge_ns * (double)host_pair[1];
  }
  if (flags & M4_BASIS_EDGE) b.edge = !budgeted;
  else if (flags & M4_BASIS_WEDGE) b.edge = false;
  else b.edge = b.cost_edge < b.cost_wedge;
  return b;
}

Launch edge_plan(const Prep& P, Scal* scal, uint32_t flags, int num_cu, KTimer* kt) {
  return [=](hipStream_t ls) {
    if (kt) kt->begin(M4_K_EDGE, ls);
    if (P.n > 0)
      k_edge_pairs<<<(unsigned)(num_cu * 4), 256, 0, ls>>>(P.nptr, P.ncol, P.dr, P.dlo, P.n,
                                                          &scal->work_c4[0], scal, flags);
    if (kt) kt->end(M4_K_EDGE, ls);
  };
}

}  // namespace m4
