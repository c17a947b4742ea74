// m4_prims.hip -- device-wide scan and stable radix pass (gfx950, wave64).
#include "m4_internal.h"

namespace m4 {

namespace {

constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;
constexpr int RAD_T = 256, RAD_ROUNDS = 16, RAD_TILE = RAD_T * RAD_ROUNDS;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t u = __shfl_up(v, o, WAVE);
    if (lane >= o) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[SCAN_T / WAVE];
  int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  int64_t inc = wave_incl_scan(v, lane);
  if (lane == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_T / WAVE; i++) {
    if (i < w) before += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return before + inc - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_T) void k_scan_tile_sums(const T* __restrict__ in, int64_t count,
                                                           int64_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_I; k++) {
    int64_t i = base + k * SCAN_T + threadIdx.x;
    if (i < count) s += (int64_t)in[i];
  }
  int64_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const T* __restrict__ in, int64_t count,
                                                       const int64_t* __restrict__ offs,
                                                       int64_t* __restrict__ out) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
  int64_t v[SCAN_I];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_I; k++) {
    int64_t i = base + k;
    v[k] = i < count ? (int64_t)in[i] : 0;
    sum += v[k];
  }
  int64_t run = block_excl_scan(sum, nullptr) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < SCAN_I; k++) {
    int64_t i = base + k;
    if (i < count) out[i] = run;
    run += v[k];
  }
  if (base < count && count - 1 < base + SCAN_I) out[count] = run;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

template <typename T>
void scan_impl(const T* in, int64_t count, int64_t* out, int64_t* tmp, hipStream_t s) {
  if (count <= 0) {
    k_set_i64<<<1, 1, 0, s>>>(out, 0);
    return;
  }
  int64_t nb = ceil_div(count, SCAN_TILE);
  if (nb == 1) {
    k_scan_tiles<T><<<1, SCAN_T, 0, s>>>(in, count, nullptr, out);
    return;
  }
  int64_t* sums = tmp;
  int64_t* offs = tmp + nb;
  int64_t* rest = tmp + 2 * nb + 1;
  k_scan_tile_sums<T><<<(unsigned)nb, SCAN_T, 0, s>>>(in, count, sums);
  scan_impl<int64_t>(sums, nb, offs, rest, s);
  k_scan_tiles<T><<<(unsigned)nb, SCAN_T, 0, s>>>(in, count, offs, out);
}

// ------------------------------------------------------------- radix pass

template <int BITS>
__global__ __launch_bounds__(RAD_T) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t count,
                                                      int shift, int64_t* __restrict__ hist) {
  constexpr int NB = 1 << BITS;
  __shared__ unsigned int h[NB];
  for (int d = threadIdx.x; d < NB; d += RAD_T) h[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RAD_TILE;
#pragma unroll 4
  for (int r = 0; r < RAD_ROUNDS; r++) {
    int64_t i = base + r * RAD_T + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & (NB - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < NB; d += RAD_T)
    hist[(int64_t)d * gridDim.x + blockIdx.x] = (int64_t)h[d];
}

// Stable scatter: items keep their input order within each digit.  Round r
// of a tile covers items base + r*256 + [0, 256); inside a round, the rank of
// an item among equal digits of its wavefront comes from BITS ballots, and
// earlier wavefronts / rounds are added through LDS counters.
template <int BITS>
__global__ __launch_bounds__(RAD_T) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                         const int32_t* __restrict__ vals_in,
                                                         int64_t count, int shift,
                                                         const int64_t* __restrict__ offs,
                                                         uint32_t* __restrict__ keys_out,
                                                         int32_t* __restrict__ vals_out) {
  constexpr int NB = 1 << BITS;
  constexpr int NW = RAD_T / WAVE;
  __shared__ unsigned int run[NB];
  __shared__ unsigned int wcnt[NW][NB];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  for (int d = tid; d < NB; d += RAD_T) {
    run[d] = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) wcnt[k][d] = 0;
  }
  __syncthreads();
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
  int64_t base = (int64_t)blockIdx.x * RAD_TILE;
  for (int r = 0; r < RAD_ROUNDS; r++) {
    int64_t i = base + r * RAD_T + tid;
    bool valid = i < count;
    uint32_t key = valid ? keys_in[i] : 0u;
    uint32_t dig = (key >> shift) & (NB - 1);
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; b++) {
      uint64_t bb = __ballot((dig >> b) & 1u);
      match &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    unsigned int rk = (unsigned int)__popcll(match & lt);
    if (valid && rk == 0) wcnt[w][dig] = (unsigned int)__popcll(match);
    __syncthreads();
    if (valid) {
      unsigned int pre = run[dig];
      for (int k = 0; k < w; k++) pre += wcnt[k][dig];
      int64_t pos = offs[(int64_t)dig * gridDim.x + blockIdx.x] + pre + rk;
      if (keys_out) keys_out[pos] = key;
      vals_out[pos] = vals_in ? vals_in[i] : (int32_t)i;
    }
    __syncthreads();
    for (int d = tid; d < NB; d += RAD_T) {
      unsigned int add = 0;
#pragma unroll
      for (int k = 0; k < NW; k++) {
        add += wcnt[k][d];
        wcnt[k][d] = 0;
      }
      run[d] += add;
    }
    __syncthreads();
  }
}

__global__ void k_bucket_starts(const int64_t* offs, int64_t nb, int NB, int64_t count,
                                int64_t* bucket_start) {
  int d = threadIdx.x;
  if (d < NB) bucket_start[d] = offs[(int64_t)d * nb];
  if (d == NB) bucket_start[NB] = count;
}

__global__ void k_zero_starts(int64_t* bucket_start, int NB) {
  int d = threadIdx.x;
  if (d <= NB) bucket_start[d] = 0;
}

template <int BITS>
void radix_pass_t(const uint32_t* keys_in, const int32_t* vals_in, int64_t count, int shift,
                  uint32_t* keys_out, int32_t* vals_out, int64_t* tmp, int64_t* bucket_start,
                  hipStream_t s) {
  constexpr int NB = 1 << BITS;
  if (count <= 0) {
    if (bucket_start) k_zero_starts<<<1, NB + 1, 0, s>>>(bucket_start, NB);
    return;
  }
  int64_t nb = ceil_div(count, RAD_TILE);
  int64_t* hist = tmp;
  int64_t* offs = tmp + NB * nb;
  int64_t* stmp = offs + NB * nb + 1;
  k_radix_hist<BITS><<<(unsigned)nb, RAD_T, 0, s>>>(keys_in, count, shift, hist);
  scan_impl<int64_t>(hist, NB * nb, offs, stmp, s);
  k_radix_scatter<BITS><<<(unsigned)nb, RAD_T, 0, s>>>(keys_in, vals_in, count, shift, offs,
                                                        keys_out, vals_out);
  if (bucket_start) k_bucket_starts<<<1, NB + 1, 0, s>>>(offs, nb, NB, count, bucket_start);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

size_t scan_tmp_elems(int64_t count) {
  size_t tot = 0;
  while (count > SCAN_TILE) {
    int64_t nb = ceil_div(count, SCAN_TILE);
    tot += 2 * nb + 1;
    count = nb;
  }
  return tot + 1;
}

void scan_i32(const int32_t* in, int64_t count, int64_t* out, int64_t* tmp, hipStream_t s) {
  scan_impl<int32_t>(in, count, out, tmp, s);
}
void scan_i64(const int64_t* in, int64_t count, int64_t* out, int64_t* tmp, hipStream_t s) {
  scan_impl<int64_t>(in, count, out, tmp, s);
}

size_t radix_tmp_elems(int64_t count, int bits) {
  int64_t nb = ceil_div(count > 0 ? count : 1, RAD_TILE);
  int64_t NB = 1 << bits;
  return (size_t)(2 * NB * nb + 1) + scan_tmp_elems(NB * nb);
}

void radix_pass(const uint32_t* keys_in, const int32_t* vals_in, int64_t count, int shift, int bits,
                uint32_t* keys_out, int32_t* vals_out, int64_t* tmp, int64_t* bucket_start,
                hipStream_t s) {
  switch (bits) {
    case 2: radix_pass_t<2>(keys_in, vals_in, count, shift, keys_out, vals_out, tmp, bucket_start, s); break;
    case 4: radix_pass_t<4>(keys_in, vals_in, count, shift, keys_out, vals_out, tmp, bucket_start, s); break;
    case 8: radix_pass_t<8>(keys_in, vals_in, count, shift, keys_out, vals_out, tmp, bucket_start, s); break;
    default: throw Fail(M4_EINTERNAL, "radix_pass: unsupported digit width");
  }
}

void fill_u32(void* p, uint32_t v, size_t count32, hipStream_t s) {
  if (count32 == 0) return;
  size_t blocks = (count32 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(static_cast<uint32_t*>(p), v, count32);
}

}  // namespace m4
