// m4_closure.hip -- closure pass and the exact inverse (Section III-F).
//
// Streams every oriented edge u -> v once with d_u, d_v and t_e, and every
// vertex with d_v, into 128-bit sums:
//   S     = sum_v C(d_v, 3)              non-induced 3-stars
//   P     = sum_e (d_u - 1)(d_v - 1)     4-paths + 3 T (wedge pairs on e)
//   D_ni  = sum_e C(t_e, 2)              non-induced diamonds
//   Paw2  = sum_e t_e (d_u + d_v - 4)    2 x non-induced paws
//   sum_t = sum_e t_e                    3 T
// Only these sufficient statistics are materialised (Section III-D).  The
// induced counts then follow from the non-induced ones by a unit upper
// triangular system (the number of spanning copies of each pattern inside
// each larger one); evaluated from the densest pattern down, every partial
// value is itself a count, so an unsigned underflow can only mean a bug.
// The per-vertex star formula of Section III-F sums to the same star count:
// with m(H_u) = triangles at u and deg_H(v) = t_uv it reads
// star = S - Paw_ni + 2 D_ni - 4 K4.
#include "m4_device.h"

namespace m4 {

namespace {

constexpr int CL_NT = 256, CL_G = 8;

// CL_G lanes per vertex: the out-list, its heads' degrees and its t_e are
// read by consecutive lanes, several vertices per wavefront.
__global__ __launch_bounds__(CL_NT) void k_closure(const int64_t* __restrict__ nptr,
                                                   const int32_t* __restrict__ dlo,
                                                   const int32_t* __restrict__ dplus,
                                                   const int64_t* __restrict__ optr,
                                                   const int32_t* __restrict__ ncol,
                                                   const int32_t* __restrict__ dr,
                                                   const uint32_t* __restrict__ t, int64_t lo,
                                                   int64_t hi, Scal* scal) {
  u128_t S = 0, P = 0, D = 0, Paw2 = 0, St = 0;
  const int gl = threadIdx.x & (CL_G - 1);
  const int64_t groups = (int64_t)gridDim.x * (CL_NT / CL_G);
  for (int64_t u = lo + ((int64_t)blockIdx.x * CL_NT + threadIdx.x) / CL_G; u < hi; u += groups) {
    const uint64_t du = (uint32_t)dr[u];
    if (gl == 0 && du >= 3) S += (u128_t)du * (du - 1) * (du - 2) / 6;
    const int k = dplus[u];
    const int64_t rb = nptr[u] + dlo[u], oe = optr[u];
    uint64_t st = 0;  // sum of t_e over this lane's edges of u: < 2^31 * 2^32
    for (int j = gl; j < k; j += CL_G) {
      const uint64_t dv = (uint32_t)dr[ncol[rb + j]];
      const uint64_t te = t[oe + j];
      P += (u128_t)((du - 1) * (dv - 1));  // each product < 2^62
      st += te;
      D += (u128_t)(te * (te - 1) / 2);     // te < 2^32: < 2^63 per edge
      if (te) Paw2 += (u128_t)te * (du + dv - 4);
    }
    St += st;
  }
  block_add_u128<CL_NT>(&scal->acc[ACC_S], S);
  block_add_u128<CL_NT>(&scal->acc[ACC_P], P);
  block_add_u128<CL_NT>(&scal->acc[ACC_D], D);
  block_add_u128<CL_NT>(&scal->acc[ACC_PAW2], Paw2);
  block_add_u128<CL_NT>(&scal->acc[ACC_SUMT], St);
}

// status: 0 ok, 3 a count >= 2^64, 7 internal check failed
__global__ void k_finalize(Scal* scal, int zbasis) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const u128_t K4 = load_u128(&scal->acc[ACC_K4]), D = load_u128(&scal->acc[ACC_D]);
  u128_t C4 = load_u128(&scal->acc[ACC_C4]);
  int zstatus = 0;
  if (zbasis) {
    // edge-anchor basis: Z = 4 * cycle (each induced 4-cycle is an adjacent
    // pair of A_e x B_e for each of its four edges), and a 4-cycle subgraph
    // is an induced 4-cycle, a diamond (D_ni - 6 K4) or one of the three in
    // a 4-clique
    const u128_t Z = load_u128(&scal->acc[ACC_Z]);
    if (Z % 4 != 0 || D < 3 * K4) zstatus = 7;
    else C4 = Z / 4 + D - 3 * K4;
  }
  const u128_t in[7] = {K4, C4, load_u128(&scal->acc[ACC_S]), load_u128(&scal->acc[ACC_P]), D,
                        load_u128(&scal->acc[ACC_PAW2]), load_u128(&scal->acc[ACC_SUMT])};
  const int st = finalize_basis(in, scal->out, scal->basis);
  scal->status = zstatus ? zstatus : st;
}

}  // namespace

void closure_run(const Prep& P, Scal* scal, uint32_t flags, hipStream_t s) {
  (void)flags;
  const int64_t lo = P.own_lo, hi = P.hi();
  if (hi <= lo) return;
  int64_t blocks = ceil_div((hi - lo) * CL_G, CL_NT);
  if (blocks > 4096) blocks = 4096;
  k_closure<<<(unsigned)blocks, CL_NT, 0, s>>>(P.nptr, P.dlo, P.dplus, P.optr, P.ncol, P.dr, P.t,
                                               lo, hi, scal);
}

void finalize_run(Scal* scal, hipStream_t s, bool zbasis) {
  k_finalize<<<1, 64, 0, s>>>(scal, zbasis ? 1 : 0);
}

}  // namespace m4
