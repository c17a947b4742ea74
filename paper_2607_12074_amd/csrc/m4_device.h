// m4_device.h -- small device helpers shared by the kernels.
#pragma once
#include "m4_internal.h"

namespace m4 {

// Orders the LDS accesses of one wavefront (all lanes run in lockstep; the
// fence keeps the compiler from moving LDS loads above earlier stores).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

typedef unsigned __int128 u128_t;

// Exact 128-bit add into memory (global or LDS) from two 64-bit atomics.
__device__ __forceinline__ void atomic_add_u128(U128* a, u128_t v) {
  unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
  if (lo) {
    unsigned long long old = atomicAdd(&a->lo, lo);
    if (old + lo < old) hi += 1;
  }
  if (hi) atomicAdd(&a->hi, hi);
}

__device__ __forceinline__ u128_t load_u128(const U128* a) {
  return ((u128_t)a->hi << 64) | a->lo;
}

// Reduce one u128 per thread over the block into `dst` (global).
template <int NT>
__device__ __forceinline__ void block_add_u128(U128* dst, u128_t v) {
  __shared__ U128 red;
  if (threadIdx.x == 0) red.lo = red.hi = 0;
  __syncthreads();
  if (v) atomic_add_u128(&red, v);
  __syncthreads();
  if (threadIdx.x == 0) {
    u128_t tot = load_u128(&red);
    if (tot) atomic_add_u128(dst, tot);
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ void block_add_u64(unsigned long long* dst, unsigned long long v) {
  __shared__ unsigned long long red;
  if (threadIdx.x == 0) red = 0;
  __syncthreads();
  if (v) atomicAdd(&red, v);
  __syncthreads();
  if (threadIdx.x == 0 && red) atomicAdd(dst, red);
  __syncthreads();
}

// Exclusive prefix over one int64 per thread of an NT-thread block.
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan64(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[NT / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  int64_t inc = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t u = __shfl_up(inc, o, WAVE);
    if (lane >= o) inc += u;
  }
  if (NT == WAVE) {
    if (total) *total = __shfl(inc, WAVE - 1, WAVE);
    return inc - v;
  }
  if (lane == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; i++) {
    if (i < w) before += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return before + inc - v;
}

// Index of the last entry <= key in a non-decreasing array a[0..len).
template <typename T, typename K>
__device__ __forceinline__ int upper_index(const T* a, int len, K key) {
  int lo = 0, hi = len;  // first index with a[i] > key
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// First index in [lo, hi) with a[i] >= key.
template <typename T, typename K>
__device__ __forceinline__ int64_t lower_index(const T* a, int64_t lo, int64_t hi, K key) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Induced counts from the non-induced basis (Section III-F closure): the
// inverse of the unit upper-triangular "spanning copies" system, densest
// pattern first.  in[] = {K4, C4_ni, S, P, D_ni, Paw2, sum_t} as 128-bit sums.
// Returns 0, 3 (a value >= 2^64) or 7 (a consistency check failed).
__device__ __forceinline__ int finalize_basis(const u128_t in[7], unsigned long long out[6],
                                              unsigned long long basis[8]) {
  const u128_t K4 = in[0], C4 = in[1], S = in[2], P = in[3], D = in[4], Paw2 = in[5],
               St = in[6];
  int status = 0;
  if (St % 3 != 0 || Paw2 % 2 != 0) status = 7;
  const u128_t T = St / 3, PawN = Paw2 / 2;
  u128_t clique = K4, diamond = 0, cycle = 0, paw = 0, star = 0, path = 0;
  if (D >= 6 * clique) diamond = D - 6 * clique; else status = 7;
  if (C4 >= diamond + 3 * clique) cycle = C4 - diamond - 3 * clique; else status = 7;
  if (PawN >= 4 * diamond + 12 * clique) paw = PawN - 4 * diamond - 12 * clique; else status = 7;
  if (S >= paw + 2 * diamond + 4 * clique) star = S - paw - 2 * diamond - 4 * clique; else status = 7;
  const u128_t pathN = P >= 3 * T ? P - 3 * T : 0;
  const u128_t sub = 2 * paw + 4 * cycle + 6 * diamond + 12 * clique;
  if (P >= 3 * T && pathN >= sub) path = pathN - sub; else status = 7;
  const u128_t res[6] = {star, path, paw, cycle, diamond, clique};
  const u128_t b[8] = {T, K4, C4, S, pathN, PawN, D, St};
  for (int i = 0; i < 8; i++) {
    if (b[i] >> 64) { if (!status) status = 3; if (basis) basis[i] = ~0ull; }
    else if (basis) basis[i] = (unsigned long long)b[i];
  }
  for (int i = 0; i < 6; i++) {
    if (res[i] >> 64) { if (!status) status = 3; out[i] = ~0ull; }
    else out[i] = (unsigned long long)res[i];
  }
  return status;
}

}  // namespace m4
