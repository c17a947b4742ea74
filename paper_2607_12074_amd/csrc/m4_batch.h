// m4_batch.h -- plan and launch of the persistent fused batch kernel
// (shared by the batch entry point and the serving loop).
#pragma once
#include <vector>

#include "m4_ctx.h"

namespace m4 {

constexpr int B_NMAX = 8192;  // vertices of a graph handled in one workgroup
constexpr int B_TOO_BIG = 9;  // per-graph status: needs the single-graph path

struct BatchArgs {
  int64_t G;
  const int64_t* voff;
  const int64_t* eoff;
  const int64_t* rowp;
  const int32_t* col;
  const int32_t* order;
  int64_t norder;
  unsigned int* work;
  int32_t* perm;
  int32_t* dr;
  int32_t* dlo;
  int32_t* dplus;
  int64_t* nptr;
  int64_t* optr;
  int32_t* ncol;
  uint32_t* t;
  unsigned long long* out;    // [G][6]
  int* status;                // [G]
  unsigned long long* basis;  // [G][8] or null
  int light;
  uint32_t flags;
  uint32_t cache_rows;
  int kbig;
  uint64_t* gbits;
  int32_t* garr;
};

struct BatchPlan {
  int64_t G = 0, sum_n = 0, sum_nnz = 0;
  std::vector<int32_t> order;  // graphs for the fused kernel, largest first
  std::vector<int64_t> big;    // graphs for the single-graph path
  int kbig = 0, variant = 0, grid = 1;
  size_t arena_bytes = 0, o_arena = 0;
  bool staged = false;
  BatchArgs args{};
};

int batch_variant_kb(int variant);
// true when graph (n, rp) is counted by the fused kernel rather than by the
// single-graph path
bool batch_graph_fits(int64_t n, const int64_t* rp, int variant);
void batch_prepare(m4_ctx* c, BatchBuffers& B, BatchPlan& P, int64_t G, const int64_t* hvoff,
                   const int64_t* heoff, const int64_t* hrowp, const m4_batch* dev_arena,
                   int variant, int light, uint32_t flags, uint32_t cache_rows, hipStream_t s);
void batch_stage(BatchBuffers& B, const BatchPlan& P, const int64_t* voff, const int64_t* eoff,
                 const int64_t* rowp, const int32_t* col);
void batch_enqueue(BatchBuffers& B, const BatchPlan& P, hipStream_t s);

}  // namespace m4
