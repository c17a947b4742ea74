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
  const int32_t* order;  // graphs in launch order (null: 0, 1, ..., norder - 1)
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
  int too_big;  // status of a graph the kernel leaves to another path
  // vertices and CSR entries the work arrays hold: a graph whose offsets
  // reach past them gets status M4_EINVAL and is not touched
  int64_t vcap, ecap;
};

struct BatchPlan {
  int64_t G = 0, sum_n = 0, sum_nnz = 0;
  std::vector<int32_t> order;  // graphs for the fused kernel, largest first
  std::vector<int64_t> big;    // graphs for the single-graph path
  int variant = 0, grid = 1;
  size_t arena_bytes = 0, o_arena = 0;
  bool staged = false;
  BatchArgs args{};
};

// Device layout of one fused launch over G graphs (staged: the packed arena
// is copied in from pinned host memory); need is the device bytes it takes.
struct BatchLayout {
  size_t o_perm, o_dr, o_dlo, o_dplus, o_nptr, o_optr, o_ncol, o_t, o_order, o_out, o_status,
      o_work, o_arena, arena_bytes, need;
};
BatchLayout batch_layout(int64_t G, int64_t sum_n, int64_t sum_nnz, bool staged);

int batch_variant_kb(int variant);
// true when graph (n, rp) is counted by the fused kernel rather than by the
// single-graph path (the kernel applies the same test to the arena itself)
bool batch_graph_fits(int64_t n, const int64_t* rp, int variant);
void batch_prepare(m4_ctx* c, BatchBuffers& B, BatchPlan& P, int64_t G, const int64_t* hvoff,
                   const int64_t* heoff, const m4_batch* dev_arena, int variant, int light,
                   uint32_t flags, uint32_t cache_rows, hipStream_t s);
void batch_stage(BatchBuffers& B, const BatchPlan& P, const int64_t* voff, const int64_t* eoff,
                 const int64_t* rowp, const int32_t* col);
void batch_enqueue(BatchBuffers& B, const BatchPlan& P, hipStream_t s);
// the fused kernel alone (1024 threads, 96 KiB of LDS tiles) on grid workgroups
void batch_launch_fused(const BatchArgs& A, int grid, hipStream_t s);
// largest wedge bound of the fused kernel's per-wavefront 4-cycle hash
int batch_light_max();

}  // namespace m4
