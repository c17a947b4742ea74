/*
 * m4.h -- exact counts of the six connected induced 4-node motifs on an
 * AMD MI355X (gfx950), C ABI.
 *
 * Problem (HARP-ME, Section II): G = (V, E) is a simple undirected graph.  An
 * induced occurrence of a connected 4-node pattern p is a 4-vertex subset S
 * whose induced subgraph G[S] is isomorphic to p; N_p is the number of such
 * subsets.  The library returns N_p for the six connected 4-node patterns in
 * this order (m4_motif):
 *
 *   [0] 3-star (claw)   [1] 4-path   [2] tailed triangle (paw)
 *   [3] 4-cycle         [4] diamond  [5] 4-clique
 *
 * Method (Section III): only an anchor basis is enumerated -- per-edge
 * triangle counts t_e, 4-cliques and non-induced 4-cycles, found by sorted
 * neighbour-list intersections over a degree-oriented CSR (Section III-D) --
 * and the remaining counts follow from exact closure relations over degrees,
 * wedges and t_e (Section III-F).
 *
 * Conventions for every entry point:
 *   - Return value is an m4_status; outputs are untouched on error.
 *   - The caller owns every input and output buffer.  The library keeps no
 *     caller pointer after a call returns.
 *   - Device pointers refer to memory of the context's device.
 *   - A context is not thread-safe: one host thread per context at a time.
 *   - Nothing throws across this boundary.
 */
#ifndef M4_H
#define M4_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  M4_OK = 0,
  M4_EINVAL = 1,    /* bad argument, or a CSR that is not simple/symmetric/
                       sorted (detected only with M4_VALIDATE)               */
  M4_ERANGE = 2,    /* n >= 2^31, nnz > 2^31 - 1024, or nnz != row_ptr[n]   */
  M4_EOVERFLOW = 3, /* a count, or an intermediate sum, is >= 2^64          */
  M4_ENOMEM = 4,    /* device or pinned host allocation failed, or the
                       device budget cannot hold even one partition        */
  M4_EDEVICE = 5,   /* a HIP call failed; m4_last_error() has the text      */
  M4_EBUSY = 6,     /* server queue full                                    */
  M4_EINTERNAL = 7  /* internal consistency check failed (a library bug)    */
} m4_status;

typedef enum {
  M4_STAR = 0, M4_PATH = 1, M4_PAW = 2, M4_CYCLE = 3, M4_DIAMOND = 4, M4_CLIQUE = 5
} m4_motif;

/* Symmetric CSR of a simple undirected graph: row v lists N(v), strictly
 * increasing, without v itself; every edge appears in both rows.  nnz = 2|E|.
 * on_device = 1: row_ptr/col are device pointers, 0: host pointers. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* row_ptr; /* int64[n+1] */
  const int32_t* col;     /* int32[nnz] */
  int32_t on_device;
} m4_csr;

/* option flags */
#define M4_VALIDATE 0x1u        /* check the CSR on the device first (O(m log d)) */
#define M4_NO_CACHE 0x2u        /* disable induced-signature frontier reuse         */
#define M4_FORCE_PARTITION 0x4u /* take the halo-partition path even if it fits      */
#define M4_STATS 0x8u           /* fill the work counters of m4_stats               */
#define M4_TIMING 0x10u         /* time every kernel launch with HIP events         */
#define M4_SERIAL 0x40u         /* single graph: run the triangle and 4-cycle stages
                                   one after the other on one stream (by default
                                   they overlap on two streams, except when
                                   4-cycle owners are binned)                      */
#define M4_BASIS_WEDGE 0x80u    /* single graph: count 4-cycles with degree-ordered
                                   wedges, each at its highest vertex            */
#define M4_BASIS_EDGE 0x100u    /* single graph: count 4-cycles and 4-paths from
                                   edge anchors, the adjacent pairs of A_e x B_e
                                   (Section III-F); resident calls only.  With
                                   neither flag the anchor-selection objective
                                   of Section III-A chooses per graph            */
#define M4_PLAIN_LOOP 0x20u     /* m4_count_batch: one single-graph call per graph
                                   (the reference point of the batched launch)     */

typedef struct {
  uint64_t device_budget_bytes; /* 0 = no budget (whole device)                    */
  uint32_t flags;               /* M4_* flags above                                */
  uint32_t cache_rows;          /* signature-cache rows per owner (0 = unlimited)  */
  void* hip_stream;             /* hipStream_t to run on (NULL = context stream)   */
  /* tuning (0 = library default / autotuned value) */
  int32_t tri_wave_max;   /* owners with out-degree <= this use one wavefront
                             (overrides both of the context's wave bounds)     */
  int32_t c4_light_max;   /* owners with wedge bound <= this use the LDS hash      */
  int32_t c4_med_max;     /* ... <= this the medium LDS hash (-1: none)            */
  int32_t reserved[3];
} m4_opts;

/* Kernel slots of m4_stats.ms_kernel / k_* (one slot per kernel launch of
 * the resident pipeline; M4_K_BUILD covers all CSR-builder kernels). */
enum {
  M4_K_BUILD = 0,     /* degrees, degree sort, relabel + row sort, offsets      */
  M4_K_TRI_GLOBAL,    /* triangle/4-clique owners, out-degree > 1024           */
  M4_K_TRI_1024,      /* ... out-degree in (512, 1024], bitmap rows in LDS      */
  M4_K_TRI_512,       /* ... (256, 512]                                        */
  M4_K_TRI_256,       /* ... (128, 256]                                        */
  M4_K_TRI_128,       /* ... (wave max, 128]                                   */
  M4_K_TRI_WAVE,      /* ... out-degree <= tri_wave_max, one wavefront each    */
  M4_K_C4_PLAN,       /* 4-cycle wedge bounds and owner buckets                 */
  M4_K_C4_WINDOW,     /* 4-cycle owners with windows of dense LDS counters     */
  M4_K_C4_MED,        /* ... medium wedge bound, 16384-slot LDS hash table     */
  M4_K_C4_HASH,       /* ... small wedge bound, 4096-slot LDS hash table       */
  M4_K_CLOSURE,       /* closure sums and exact inverse                         */
  M4_K_TRI_HUBS,      /* hub tables of the long out-lists (triangle probes)     */
  M4_K_C4_DESC,       /* 4-cycle window owners' segment descriptors             */
  M4_K_C4_BIN,        /* 4-cycle owners binned by counter window                */
  M4_K_EDGE,          /* edge-anchor basis: adjacent pairs of A_e x B_e         */
  M4_NK = 16
};

/* Work and timing counters of one call.  basis[] is filled for every call
 * with a non-NULL m4_stats; the k_* counters need M4_STATS and ms_kernel[]
 * needs M4_TIMING.  Per slot:
 *   triangle slots: k_elems = sum of |N+(v)| over the owners' out-neighbours
 *                   v (elements a scanning intersection reads), k_rows = owners,
 *                   k_aux = out-list entries of the owners, k_aux2 = 4-byte
 *                   words the kernel read from out-lists and hub tables (one
 *                   per scanned element, two per 8-byte table slot probed)
 *   4-cycle slots:  k_elems = wedge endpoints counted, k_rows = owners,
 *                   k_aux = lower neighbours (segments), k_aux2 = segment
 *                   visits (window slot), row entries read (table slots;
 *                   an owner counted in rank ranges reads its rows once per
 *                   pass) or row entries read by the histogram and scatter
 *                   passes (binned slot)
 *   edge basis:     k_elems = row entries scanned, k_rows = owners with an
 *                   out-neighbour, k_aux = (out-neighbour, neighbour) pairs
 *   closure:        k_elems = oriented edges, k_rows = vertices
 *   build:          k_elems = CSR entries, k_rows = vertices */
typedef struct {
  /* non-induced basis: T, K4, C4_ni, S = sum C(d,3), P_ni, Paw_ni, D_ni,
   * sum_e t_e (each < 2^64, else the call returns M4_EOVERFLOW) */
  uint64_t basis[8];
  uint64_t intersect_steps; /* list elements looked up plus hub-table probes
                               (triangle anchors)                               */
  uint64_t wedges;          /* 4-cycle wedge endpoints counted                   */
  uint64_t cache_lookups;   /* frontier requests of the 4-clique stage           */
  uint64_t cache_hits;      /* ... served from the signature cache               */
  uint64_t partitions;      /* halo partitions processed (1 = resident)          */
  uint64_t h2d_bytes;       /* host-to-device bytes moved by the call            */
  uint64_t halo_rows;       /* rows copied as halo over all partitions           */
  uint64_t k_elems[M4_NK], k_rows[M4_NK], k_aux[M4_NK], k_aux2[M4_NK];
  double ms_kernel[M4_NK];  /* per-slot kernel time (M4_TIMING)                  */
  /* stage times (M4_TIMING): ms_tri runs from the end of the build to the end
   * of the triangle stage, ms_c4 from there to the end of both anchor stages
   * (the two overlap unless M4_SERIAL) */
  double ms_total, ms_build, ms_tri, ms_c4, ms_closure, ms_h2d;
  /* device memory the context held when the call returned: its workspaces at
   * their largest for this call (the footprint of the call).  Under a device
   * budget it never exceeds device_budget_bytes: the call first frees the
   * workspaces of earlier unbudgeted calls and allocates exactly the budget. */
  uint64_t device_bytes;
  /* partitioned calls: host time spent planning the owner ranges and
   * gathering their halo rows into pinned memory (ms_build, ms_tri, ms_c4 and
   * ms_closure then hold the wall time of each phase)                        */
  double ms_host;
  /* cycle/path anchor basis of a resident call: 0 degree-ordered wedges,
   * 1 edge anchors (A_e x B_e); the anchor-selection objective's estimate of
   * each, in ns (for the edge basis a lower bound when that already exceeds
   * the wedge estimate; infinite under a device budget)                     */
  uint32_t basis_used;
  double cost_wedge, cost_edge;
} m4_stats;

typedef struct m4_ctx m4_ctx;

/* Context bound to one device.  It owns a stream, a growable device
 * workspace and pinned staging buffers; reuse it across calls so that the
 * steady state allocates nothing. */
int m4_ctx_create(int device, m4_ctx** out);
void m4_ctx_destroy(m4_ctx* ctx);
/* Text of the last error raised in this context (never NULL). */
const char* m4_last_error(const m4_ctx* ctx);
/* Architecture name and compute-unit count of the context's device, e.g.
 * "gfx950:sramecc+:xnack- 256 CU" (owned by the context, never NULL). */
const char* m4_ctx_device(const m4_ctx* ctx);
const char* m4_strerror(int status);

/* Blocking count on device 0 with a process-wide default context. */
int m4_count_motifs4(const m4_csr* g, uint64_t out[6]);

/* Full entry point: counts on ctx's device, blocking until out[] is written.
 * opts and st may be NULL. */
int m4_count_motifs4_ex(m4_ctx* ctx, const m4_csr* g, const m4_opts* opts,
                        uint64_t out[6], m4_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of m4_count_motifs4_ex on a CSR already in device memory (g->on_device),
 * with every workspace carved from a fixed 256 MiB array in device memory
 * that the library holds on each GPU it runs on until the process ends.  It
 * calls no hipMalloc / hipFree and no allocating library routine.  The CSR
 * and out[] stay the caller's.  opts may be NULL; M4_TIMING and
 * M4_FORCE_PARTITION are ignored and a device budget is M4_EINVAL.  A graph
 * whose prepared CSR and stage workspace exceed the array is rejected with
 * M4_ENOMEM before any launch; hub tables or 4-cycle descriptors that do not
 * fit fail the call with M4_ENOMEM while the stages are planned, before
 * their kernels run.  Every call on one GPU shares that GPU's array (it
 * keeps the last call's contents; the call clears what must start at zero):
 * calls that overlap on one GPU race, so serialise them. */
int m4_count_motifs4_noalloc(m4_ctx* ctx, const m4_csr* g, const m4_opts* opts, uint64_t out[6]);

/* Per-edge triangle counts t_e = |N(u) & N(v)| for every CSR entry of g, in
 * g's own layout (t_out[p] for col[p]); t_out is a device pointer when
 * g->on_device, else host.  Same anchor kernels as the count. */
int m4_edge_triangles(m4_ctx* ctx, const m4_csr* g, const m4_opts* opts,
                      uint32_t* t_out);

/* Per-vertex graphlet orbit counts of the connected 4-vertex graphs: for every
 * vertex v and orbit o in 4..14 (Przulj's numbering, the one of ORCA, whose
 * orbit equations the paper names in its related work, Section V), the number
 * of induced 4-sets containing v in which v sits at o -- 4/5 path end/middle,
 * 6/7 claw leaf/centre, 8 cycle, 9/10/11 paw tail / degree-2 / degree-3
 * vertex, 12/13 diamond degree-2 / degree-3 vertex, 14 clique.  The same
 * closure idea as the count (Section III-F) applied per vertex: non-induced
 * local statistics from the triangle anchor (t_e, the induced subgraph on
 * N+(u)) and the wedge 4-cycle anchor, then the per-vertex inverse.
 *   orbits  uint64[n][11], row v = the caller's vertex v, column o - 4;
 *           device memory when g->on_device, else host; caller-owned.
 * Only M4_VALIDATE of opts->flags is used; a device budget is not supported
 * (M4_EINVAL).  M4_EOVERFLOW when a count is >= 2^64, M4_EINTERNAL when the
 * per-vertex inverse is inconsistent.  The graph and 8n words of statistics
 * stay resident, plus the 4-cycle counters (4n bytes per workgroup, 8n from
 * degree 2^16; at most one workgroup per CU and 16 GiB in all). */
int m4_count_orbits4(m4_ctx* ctx, const m4_csr* g, const m4_opts* opts, uint64_t* orbits);

/* --------------------------------------------------------------- tuning --
 * Degree-bucket and tile thresholds of a context.  They move owners between
 * kernels and never change a count.  m4_autotune times every candidate on
 * the given sample (a graph for the single-graph path and/or an arena for
 * the fused batched launch, reps timed runs each after one warm run), checks
 * that all candidates agree on every count (else M4_EINTERNAL), keeps the
 * fastest in the context and returns it in out (may be NULL).  On error the
 * context's tuning is unchanged. */
typedef struct {
  int32_t tri_wave_max;  /* single graph: owners with out-degree <= this use one
                            64-thread workgroup (2..64, default 32), while the
                            out-lists (4 m bytes) fit in the 256 MiB Infinity
                            Cache                                              */
  int32_t c4_light_max;  /* single graph: owners with wedge bound <= this use the
                            LDS hash (1..2048, default 2048)                   */
  int32_t batch_variant; /* fused batched kernel: 0 = 1024 threads with 96 KiB of
                            LDS tiles (out-degrees up to 768), 1 = 512 threads
                            with 40 KiB (up to 448); default 0                 */
  int32_t batch_light;   /* fused batched kernel: wedge bound of the per-
                            wavefront 4-cycle hash (1..256, default 128)      */
  int32_t hub_min;       /* single graph: vertices with out-degree >= this get a
                            hash table of their out-list, and a triangle owner
                            probes it for its later out-neighbours instead of
                            scanning the list when that is cheaper (0 = never,
                            else 4..65536, default 32)                        */
  int32_t c4_med_max;    /* single graph: owners with wedge bound in
                            (c4_light_max, c4_med_max] use the 16384-slot LDS
                            hash in one pass, heavier ones the counter windows
                            (0 = no medium bucket, else up to 12288, default
                            12288)                                            */
  int32_t probe_w;       /* single graph: a triangle row is probed in the hub
                            table when probe_w * (probes) < 3 * (elements a
                            scan would read) (1..256, default 4), while the
                            hub tables fit in the 256 MiB Infinity Cache     */
  int32_t c4_med_win;    /* single graph: an owner with wedge bound in
                            (12288, 65536] also uses the medium table, one
                            pass per rank range of at most 12288 endpoints,
                            when 16 * (windows it needs) >= c4_med_win *
                            ceil(bound / 12288), i.e. its endpoints are thin
                            over many windows (0 = never, default 64; needs
                            c4_med_max > 0)                                   */
  int32_t c4_bin_win;    /* single graph: an owner above the one-pass medium
                            bound whose endpoints span at least this many
                            counter windows is counted by binning: its
                            endpoints are sorted into per-window bins in
                            device memory, then each bin is counted in LDS
                            (0 = never, default 6)                            */
  int32_t c4_bin_cap;    /* single graph: endpoints one binning workgroup's
                            device scratch holds (0 = 2^20, else 64..2^24);
                            an owner with more is binned in several rank
                            ranges                                           */
  int32_t c4_bin_dense;  /* single graph: an owner that c4_bin_win would bin
                            keeps the dense counter windows when its wedge
                            bound is at least this many endpoints per window
                            it needs (0 = never, else 64..2^20, default
                            16384)                                            */
  int32_t probe_w_far;   /* single graph: probe_w when the hub tables exceed
                            the Infinity Cache, so that a probe is a line
                            read from HBM (1..256, default 16)                */
  int32_t tri_wave_far;  /* single graph: tri_wave_max when the out-lists
                            exceed the Infinity Cache (2..64, default 64)     */
} m4_tuning;

int m4_get_tuning(const m4_ctx* ctx, m4_tuning* out);
int m4_set_tuning(m4_ctx* ctx, const m4_tuning* t);
int m4_autotune(m4_ctx* ctx, const m4_csr* graph, const struct m4_batch_s* batch, int reps,
                m4_tuning* out);

/* ---------------------------------------------------------------- batch --
 * Many independent graphs packed in one arena: graph i has vertices
 * [voff[i], voff[i+1]) and CSR entries [eoff[i], eoff[i+1]) of row_ptr/col;
 * row_ptr holds local offsets (row_ptr[voff[i]] == 0 for every graph ... see
 * layout below) and col holds LOCAL vertex ids in [0, n_i).
 *   row_ptr: int64[voff[G] + G]  -- graph i uses row_ptr[voff[i] + i ...
 *            voff[i+1] + i], its own n_i + 1 offsets starting at 0
 *   col    : int32[eoff[G]]      -- graph i uses col[eoff[i] ... eoff[i+1])
 * All arrays live on the device when on_device, else on the host.  out is a
 * host array of G * 6 counts.  One persistent launch counts every graph. */
typedef struct m4_batch_s {
  int64_t num_graphs;
  const int64_t* voff;    /* int64[G+1] */
  const int64_t* eoff;    /* int64[G+1] */
  const int64_t* row_ptr; /* int64[voff[G] + G] */
  const int32_t* col;     /* int32[eoff[G]] */
  int32_t on_device;
} m4_batch;

int m4_count_batch(m4_ctx* ctx, const m4_batch* b, const m4_opts* opts,
                   uint64_t* out, m4_stats* st);

/* ------------------------------------------------ partition planning ----
 * The host planner of the halo-partitioned path (Section III-E), exposed so
 * that its ranges can be checked without a GPU.  Input: a rank-space CSR in
 * host memory (rows sorted, ranks in (degree, id) order, dlo[v] entries of
 * row v below v and dplus[v] above it).  kind 0 plans triangle / 4-clique
 * owner ranges over [0, n) (a range holds its owners' out-lists and their
 * out-neighbours' out-lists); kind 1 plans 4-cycle owner ranges over
 * [r1, n) (a range holds the rows of its owners and of their lower
 * neighbours, each cut below the range's end).  Every range but a lone owner
 * fits cap_bytes by the path's own accounting.  Output, caller-owned: range k
 * ends at range_end[k] (starting where range k-1 ended) and owns rows
 * [range_rows[k-1], range_rows[k]) of rows_v / rows_first / rows_len (entries
 * [first, first + len) of row v); *nranges = ranges written.  Returns
 * M4_ENOMEM when one owner alone exceeds cap_bytes (the ranges before it are
 * written), M4_ERANGE when max_ranges or max_rows is too small, M4_EINVAL on
 * bad arguments.  Host only; no device is touched. */
int m4_plan_partitions(int kind, int64_t n, const int64_t* nptr, const int32_t* col,
                       const int32_t* dlo, const int32_t* dplus, int64_t r1,
                       uint64_t cap_bytes, int64_t max_ranges, int64_t max_rows,
                       int64_t* range_end, int64_t* range_rows, int32_t* rows_v,
                       int64_t* rows_first, int32_t* rows_len, int64_t* nranges);

/* -------------------------------------------------------------- serving --
 * A request loop with continuous batching: submitted graphs are copied into
 * pinned staging, admitted to the device while their CSR and work arrays fit
 * the HBM budget, and counted together with whatever else is resident. */
typedef struct m4_server m4_server;
typedef struct {
  uint64_t id;       /* value returned by m4_server_submit */
  uint64_t tag;      /* caller tag                          */
  int32_t status;    /* m4_status of this request           */
  uint64_t counts[6];
  double t_submit_ms, t_admit_ms, t_done_ms; /* server clock */
} m4_result;

int m4_server_create(m4_ctx* ctx, uint64_t hbm_budget_bytes, int max_queue,
                     m4_server** out);
int m4_server_submit(m4_server* s, const m4_csr* g, uint64_t tag, uint64_t* id);
int m4_server_poll(m4_server* s, m4_result* res, int max_results, int* got);
/* Blocks until every submitted request has a result ready for polling. */
int m4_server_drain(m4_server* s);
void m4_server_destroy(m4_server* s);
/* Milliseconds on the server clock (the clock of m4_result times). */
double m4_server_now_ms(const m4_server* s);
/* Largest device memory the server held at once (lane arenas, the worker's
 * workspaces and the running work's reserve; never above the budget), number
 * of fused launches and completed requests so far. */
int m4_server_stats(const m4_server* s, uint64_t* max_inflight_bytes, uint64_t* launches,
                    uint64_t* completed);

#ifdef __cplusplus
}
#endif
#endif
