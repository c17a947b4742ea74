/*
 * m4gen.h -- seeded synthetic graph generators (inputs only).
 *
 * This library produces the simple undirected graphs that the motif counter
 * and its CPU oracle both read.  It holds none of the counting arithmetic:
 * it draws random numbers, builds edge lists and turns them into a symmetric
 * CSR with strictly increasing rows, no self-loops and no duplicate edges.
 *
 * Randomness is counter based: every draw is splitmix64 (Steele, Lea and
 * Flood, OOPSLA 2014, the finaliser of SplitMix64) applied to a key derived
 * from (seed, stream) plus a draw index, so every output depends only on the
 * seed and never on the number of threads.
 *
 * Ownership: each generator allocates g->row_ptr (int64[n+1]) and g->col
 * (int32[nnz]) with malloc; the caller releases both with m4gen_free().
 * Return value: 0 on success, -1 on bad arguments, -2 when out of memory.
 * On error *g is left zeroed.
 */
#ifndef M4GEN_H
#define M4GEN_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t n;        /* vertices                                       */
  int64_t nnz;      /* CSR entries = 2 * undirected edges              */
  int64_t* row_ptr; /* int64[n+1]                                      */
  int32_t* col;     /* int32[nnz], each row strictly increasing         */
} m4gen_graph;

/* Uniform draw in [0,1) number `ctr` of stream (seed, stream). */
double m4gen_uniform(uint64_t seed, uint64_t stream, uint64_t ctr);

/* G(n, m): uniform over simple graphs with exactly m edges
 * (m is clipped to n(n-1)/2). */
int m4gen_gnm(int64_t n, int64_t m, uint64_t seed, m4gen_graph* g);

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale vertices,
 * edge_factor * 2^scale sampled arcs, quadrant probabilities a, b, c and
 * d = 1-a-b-c at every level, no noise.  If permute != 0 the ids are
 * relabelled by a seeded random permutation.  Self-loops are dropped, the
 * arcs are symmetrised and duplicates removed. */
int m4gen_rmat(int scale, int64_t edge_factor, double a, double b, double c,
               uint64_t seed, int permute, m4gen_graph* g);

/* Barabasi-Albert preferential attachment: the seed graph is a star on
 * m_ba+1 vertices, then every new vertex attaches to m_ba distinct earlier
 * vertices drawn with probability proportional to degree. */
int m4gen_ba(int64_t n, int m_ba, uint64_t seed, m4gen_graph* g);

/* Chung-Lu power law: weight of vertex i is (i+1)^(-1/(beta-1)), scaled to
 * mean mean_deg and capped at sqrt(sum of weights); round(n*mean_deg/2)
 * endpoint pairs are drawn with probability proportional to the weights,
 * then loops and duplicates are dropped; ids are randomly permuted. */
int m4gen_chunglu(int64_t n, double beta, double mean_deg, uint64_t seed,
                  m4gen_graph* g);

/* Random geometric graph in the unit square with radius
 * r = sqrt(mean_deg / (pi n)); vertices closer than r are adjacent. */
int m4gen_rgg(int64_t n, double mean_deg, uint64_t seed, m4gen_graph* g);

/* Build a simple symmetric CSR from an arbitrary edge list (either
 * direction, loops and duplicates allowed and removed). */
int m4gen_from_edges(int64_t n, int64_t ne, const int32_t* src,
                     const int32_t* dst, m4gen_graph* g);

void m4gen_free(m4gen_graph* g);

#ifdef __cplusplus
}
#endif
#endif
