// m4_internal.h -- shared declarations of the MI355X motif-count library.
// Device arrays of a graph prepared in "rank space": vertices are relabelled
// by the degree order (d, id) (the canonical order of Section III-D), every
// row is sorted, and the oriented out-list N+(r) of vertex r is the suffix of
// its row holding the neighbours of higher rank.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>

#include "../../include/m4.h"

namespace m4 {

constexpr int WAVE = 64;
// the MI355X's last-level cache (Infinity Cache) in front of HBM
constexpr size_t kInfinityCacheBytes = size_t(256) << 20;

// 128-bit unsigned accumulator in device memory, added to with two 64-bit
// atomics (exact: the carry of the low word is derived from its own old value).
struct U128 {
  unsigned long long lo, hi;
};

enum Acc { ACC_K4 = 0, ACC_C4, ACC_S, ACC_P, ACC_PAW2, ACC_D, ACC_SUMT, ACC_N };
// adjacent pairs of A_e x B_e over all edges (edge-anchor basis), in the
// spare accumulator
constexpr int ACC_Z = ACC_N;
// ST_COST, ST_COST + 1: the anchor-selection inputs (wedge endpoints bound,
// edge-basis row entries)
enum Stat { ST_STEPS = 0, ST_WEDGES, ST_LOOKUPS, ST_HITS, ST_COST, ST_N = 8 };

// Triangle-owner buckets by out-degree k = d+(u).
enum TriBucket { TB_NONE = 0, TB_WAVE, TB_LDS, TB_GLOBAL, TB_N = 4 };
// 4-cycle-owner buckets by wedge bound.
enum C4Bucket { CB_NONE = 0, CB_HASH, CB_MED, CB_WIN, CB_BIN, CB_N = 5 };
// radix digits of the 4-cycle bucket keys and slots of their bucket starts
constexpr int C4_KEY_BITS = 4;
constexpr int C4_START_SLOTS = (1 << C4_KEY_BITS) + 1;

// Largest out-degree handled with the bitmap rows in LDS.
constexpr int TRI_LDS_MAX = 1024;
// 4-cycle window: 32768 words (128 KiB of LDS) of zoned counters.
constexpr int C4_WIN_WORDS = 32768;
constexpr int C4_HASH_SLOTS = 4096;   // light owners: 256 threads, load <= 1/2
constexpr int C4_MED_SLOTS = 16384;   // medium owners: 1024 threads, load <= 3/4
constexpr int C4_MED_MAX = 65536;     // largest wedge bound of the medium bucket
// Entries of slack after the last row of a rank-space CSR, so that 16-byte
// vector loads aligned below a cursor may run past the end of the array.
constexpr int NCOL_PAD = 256;

// Error bits of Scal::err
constexpr int ERR_INVALID = 1;  // malformed CSR (M4_VALIDATE)
constexpr int ERR_RANGES = 2;   // ranged 4-cycle plan exceeded its bound
constexpr int ERR_PROBE = 4;    // an open-addressing probe ran past its table size

struct Scal {
  U128 acc[ACC_N + 1];
  unsigned long long stat[ST_N];
  unsigned int dmax;
  int err;
  unsigned int work[8];     // owner counters of the triangle stage
  unsigned int work_c4[8];  // ... of the 4-cycle stage (the stages may overlap)
  unsigned int nhub;  // vertices with a hub table (triangle stage)
  unsigned int pad2;
  int64_t tri_start[TB_N + 1];
  int64_t c4_start[CB_N + 1];
  unsigned long long out[6];
  unsigned long long basis[8];  // T, K4, C4_ni, S, P_ni, Paw_ni, D_ni, sum_t
  unsigned long long kstat[M4_NK][4];  // per kernel slot: elems, rows, aux, aux2
  int status;
  int pad;
};

struct Prep {
  int64_t n = 0, nnz = 0, m = 0;
  int32_t* perm = nullptr;  // rank -> input id
  int32_t* rank = nullptr;  // input id -> rank
  int32_t* dr = nullptr;    // degree by rank (non-decreasing)
  int32_t* dlo = nullptr;   // neighbours of lower rank
  int32_t* dplus = nullptr; // neighbours of higher rank = |N+(r)|
  int64_t* nptr = nullptr;  // row offsets in rank space [n+1]
  int64_t* optr = nullptr;  // oriented edge offsets [n+1]
  int32_t* ncol = nullptr;  // rows in rank space, sorted [nnz]
  uint32_t* t = nullptr;    // triangles per oriented edge [m]
  // Partitioned runs: only owners in [own_lo, own_hi) are processed and rows
  // may be stored as a prefix of row_len[v] entries (null: full rows).
  int64_t own_lo = 0, own_hi = -1;
  const int32_t* row_len = nullptr;
  int64_t hi() const { return own_hi < 0 ? n : own_hi; }
};

// Rank boundaries of degree classes, read back once per graph.
struct Classes {
  int64_t r1;            // first rank with degree >= 2
  int64_t bound[16];     // first rank with degree > thr[i]
  int dmax;
};

// ------------------------------------------------------------ workspace
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (used + bytes > cap) return nullptr;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

struct Tuning {
  int tri_wave_max = 32;    // <= WAVE
  int c4_light_max = 2048;  // wedge bound for the hash bucket
  int c4_med_max = 12288;   // wedge bound for the one-pass medium hash (0: no medium bucket)
  int grid_mult = 8;        // persistent blocks per CU for light kernels
  int batch_variant = 0;    // batched kernel: 0 = 1024 threads / 96 KiB, 1 = 512 / 40 KiB
  int batch_light = 128;    // batched kernel: wedge bound of the wavefront hash
  int hub_min = 32;         // out-degree from which a vertex gets a hub table (0: none)
  int probe_w = 4;          // weight of a hub-table probe against a scanned element (x 1/3)
  int c4_med_win = 64;      // ranged medium owners: 16 windows >= this per range (0: none)
  int c4_bin_win = 6;       // owners above the one-pass medium bound whose endpoints span at
                            // least this many counter windows are binned by window (0: never)
  int c4_bin_cap = 0;       // endpoints of a binning workgroup's scratch (0: 2^20)
  int c4_bin_dense = 16384; // endpoints per window from which an owner keeps dense windows (0: never)
  int probe_w_far = 16;     // probe_w when the hub tables do not fit in the Infinity Cache
  int tri_wave_far = 64;    // tri_wave_max when the out-lists do not fit in the Infinity Cache
  // weights of the anchor-selection objective, from stage times measured on
  // the MI355X over graphs of 10^2 to 10^7 edges: ns per wedge endpoint
  // bound, fixed us of the wedge stage (its plan kernels and host
  // read-backs), ns per row entry the edge basis scans
  double cost_wedge_ns = 0.005, cost_wedge_fixed_us = 300.0, cost_edge_ns = 0.03;
};

// Optional per-launch HIP event pairs (M4_TIMING).
struct KTimer {
  bool on = false;
  hipEvent_t ev[M4_NK][2] = {};
  bool used[M4_NK] = {};
  void begin(int k, hipStream_t s) {
    if (on) {
      (void)hipEventRecord(ev[k][0], s);
      used[k] = true;
    }
  }
  void end(int k, hipStream_t s) {
    if (on) (void)hipEventRecord(ev[k][1], s);
  }
};

// ------------------------------------------------------ launch helpers
struct Err {
  int code = M4_OK;
  std::string msg;
};

#define M4_HIP(expr)                                                       \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      throw ::m4::HipFail(e_, #expr, __FILE__, __LINE__);                  \
    }                                                                      \
  } while (0)

struct HipFail {
  hipError_t e;
  const char* what;
  const char* file;
  int line;
  HipFail(hipError_t e_, const char* w, const char* f, int l) : e(e_), what(w), file(f), line(l) {}
};

struct Fail {
  int code;
  std::string msg;
  Fail(int c, std::string m) : code(c), msg(std::move(m)) {}
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------- primitives (m4_prims)
// Exclusive scan: out[0..count] with out[count] = total.  tmp must hold
// scan_tmp_elems(count) int64.
size_t scan_tmp_elems(int64_t count);
void scan_i32(const int32_t* in, int64_t count, int64_t* out, int64_t* tmp, hipStream_t s);
void scan_i64(const int64_t* in, int64_t count, int64_t* out, int64_t* tmp, hipStream_t s);

// Stable partition of items [0, count) by a small key (bucket id < 2^bits),
// and the general stable radix pass used by the degree sort.
size_t radix_tmp_elems(int64_t count, int bits);
void radix_pass(const uint32_t* keys_in, const int32_t* vals_in, int64_t count, int shift,
                int bits, uint32_t* keys_out, int32_t* vals_out, int64_t* tmp,
                int64_t* bucket_start /* nullable, [2^bits + 1] */, hipStream_t s);

void fill_u32(void* p, uint32_t v, size_t count32, hipStream_t s);

// --------------------------------------------------- stages (per file)
// m4_build.hip
size_t build_tmp_bytes(int64_t n, int64_t nnz);
void build_prep(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz, bool validate,
                Prep& P, Classes& C, Scal* scal, Scal* scal_host, Arena& tmp, hipStream_t s);
// First half of build_prep: degrees, degree order (perm, dr, rank), row
// offsets nptr and the rank boundaries of the degree classes.
void degree_order(const int64_t* rp, const int32_t* col, int64_t n, int64_t nnz, bool validate,
                  Prep& P, Classes& C, Scal* scal, Scal* scal_host, Arena& tmp, hipStream_t s);
void edge_t_to_input(const Prep& P, const int64_t* rp, const int32_t* col, uint32_t* t_out,
                     hipStream_t s);
// Relabels rows [r_lo, r_hi) (ranks) through rank[] and sorts them; per-row
// arrays (perm, nptr, dr, dlo, dplus) are indexed by rank - r_base; bnd are
// the rank boundaries of the degree classes (row_class_thresholds()).
void sort_rows(const int64_t* rp, const int32_t* col, const int32_t* perm, const int32_t* rank,
               const int64_t* nptr, const int32_t* dr, int64_t n, int64_t r_lo, int64_t r_hi,
               const int64_t* bnd, int32_t* ncol, int32_t* dlo, int32_t* dplus, int64_t r_base,
               hipStream_t s);
int row_class_count();
const int* row_class_thresholds();

// An anchor stage is planned on stream s (small kernels and host read-backs
// of bucket sizes) and returns the launches of its heavy kernels, to be
// issued on any stream ordered after s; the stage's workspace and scratch
// stay reserved until those kernels are done.
using Launch = std::function<void(hipStream_t)>;

// m4_tri.hip
size_t tri_tmp_bytes(int64_t n, int64_t nnz, int dplus_max_bound);
// big_scratch(bytes) returns device memory for the hub tables and for owners
// whose bitmap does not fit in LDS (only called when those exist).
Launch tri_plan(const Prep& P, Scal* scal, const Tuning& tu, uint32_t flags, uint32_t cache_rows,
                Arena& tmp, hipStream_t s, int num_cu,
                const std::function<char*(size_t)>& big_scratch, KTimer* kt);
inline void tri_run(const Prep& P, Scal* scal, const Tuning& tu, uint32_t flags,
                    uint32_t cache_rows, Arena& tmp, hipStream_t s, int num_cu,
                    const std::function<char*(size_t)>& big_scratch, KTimer* kt) {
  tri_plan(P, scal, tu, flags, cache_rows, tmp, s, num_cu, big_scratch, kt)(s);
}

// m4_local.hip: per-vertex orbit counts of a prepared graph (t complete)
void local_orbits(const Prep& P, const Classes& C, Scal* scal, unsigned long long* arrays,
                  void* cscr, bool wide, int cblocks, unsigned long long* gscr, int gblocks,
                  int kmax, unsigned long long* out, int num_cu, hipStream_t s);
size_t local_glob_stride_words(int kmax);
int local_dplus_max(const Prep& P, Scal* scal, hipStream_t s);

// m4_edge.hip: the cycle/path anchor basis chosen by the anchor-selection
// objective (estimates in ns; edge = adjacent pairs of A_e x B_e)
struct BasisChoice {
  bool edge = false;
  double cost_wedge = 0, cost_edge = 0;
};
BasisChoice choose_basis(const Prep& P, const Tuning& tu, uint32_t flags, bool budgeted,
                         Scal* scal, unsigned long long* host_pair, hipStream_t s);
Launch edge_plan(const Prep& P, Scal* scal, uint32_t flags, int num_cu, KTimer* kt);

// m4_c4.hip (binned, if given, is set when owners go to the binning kernel,
// which holds every CU with persistent workgroups and all of their LDS)
Launch c4_plan(const Prep& P, const Classes& C, Scal* scal, const Tuning& tu, uint32_t flags,
               Arena& tmp, hipStream_t s, int num_cu, KTimer* kt,
               const std::function<char*(size_t)>& big_scratch, bool* binned = nullptr);
inline void c4_run(const Prep& P, const Classes& C, Scal* scal, const Tuning& tu, uint32_t flags,
                   Arena& tmp, hipStream_t s, int num_cu, KTimer* kt,
                   const std::function<char*(size_t)>& big_scratch) {
  c4_plan(P, C, scal, tu, flags, tmp, s, num_cu, kt, big_scratch)(s);
}

// m4_closure.hip
void closure_run(const Prep& P, Scal* scal, uint32_t flags, hipStream_t s);
// zbasis: the 4-cycle statistic is Z of the edge-anchor basis, not C4_ni
void finalize_run(Scal* scal, hipStream_t s, bool zbasis = false);

}  // namespace m4
