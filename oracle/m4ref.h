/*
 * m4ref.h -- CPU oracle for connected induced 4-node motif counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Input: a simple undirected graph as a symmetric CSR -- row_ptr int64[n+1],
 * col int32[row_ptr[n]], every row strictly increasing, no self-loops.  The
 * oracle does not repair bad input; m4ref_validate() reports it.
 *
 * Output order of the six counts (induced occurrences are vertex subsets S of
 * size 4 whose induced subgraph G[S] is isomorphic to the pattern, as in the
 * paper's problem definition, Section II):
 *   out[0] 3-star (claw)   out[1] 4-path        out[2] tailed triangle (paw)
 *   out[3] 4-cycle         out[4] diamond       out[5] 4-clique
 *
 * Return codes: 0 ok, 1 bad argument, 3 a count does not fit in 64 bits,
 * 4 out of memory, 7 graph too large for the chosen method.
 */
#ifndef M4REF_H
#define M4REF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Checks the CSR is simple, symmetric and sorted.  0 ok, 1 bad. */
int m4ref_validate(int64_t n, const int64_t* row_ptr, const int32_t* col);

/* O1: every 4-vertex subset is classified by the sorted degree sequence of
 * its induced subgraph (Section II definition).  n <= 1024. */
int m4ref_brute(int64_t n, const int64_t* row_ptr, const int32_t* col,
                uint64_t out[6]);

/* O2: ESU enumeration (Wernicke 2006) visits every connected 4-vertex set
 * exactly once and classifies it as O1 does. */
int m4ref_esu(int64_t n, const int64_t* row_ptr, const int32_t* col,
              uint64_t out[6]);

/* O3: the closure equations of Section III-F applied as printed: triangle
 * attachment classes X_j(T), edge sides A_e x B_e, and the per-vertex star
 * formula over H_u = G[N(u)].  Sums over undirected edges take each edge once. */
int m4ref_paper(int64_t n, const int64_t* row_ptr, const int32_t* col,
                uint64_t out[6]);

/* O4: plain closure counter (also the CPU timing baseline).  Lists every
 * triangle once under the degree order (d, id), accumulates per-edge triangle
 * counts t_e, counts 4-cliques over the triangles, counts non-induced 4-cycles
 * by wedges at their highest vertex, and converts the non-induced counts to
 * induced ones by the exact triangular inverse.  threads <= 0 means all.
 *
 * Optional outputs (NULL to skip):
 *   t_csr  uint32[row_ptr[n]]: t_e at both CSR positions of every edge.
 *   basis  uint64[8]: { T, K4, C4_ni, S, P_ni, Paw_ni, D_ni, sum_e t_e }
 *          (triangles, 4-cliques, non-induced 4-cycles, sum C(d,3),
 *           non-induced 4-paths, non-induced paws, non-induced diamonds). */
int m4ref_closure(int64_t n, const int64_t* row_ptr, const int32_t* col,
                  int threads, uint64_t out[6], uint32_t* t_csr,
                  uint64_t basis[8]);

/* Per-vertex graphlet orbit counts of the connected 4-vertex graphs: orb is
 * uint64[n][11], entry [v][o - 4] the number of induced 4-sets S containing v
 * in which v occupies orbit o (Przulj's numbering, as used by ORCA, which the
 * paper names in its related work, Section V): 4/5 path end/middle, 6/7 claw
 * leaf/centre, 8 cycle, 9/10/11 paw tail / degree-2 / degree-3, 12/13
 * diamond degree-2 / degree-3, 14 clique.  The orbit of v follows from the
 * class of G[S] and v's degree inside S.
 *   m4ref_orbits_brute: every 4-vertex subset (n <= 1024);
 *   m4ref_orbits_esu:   every connected 4-set once by ESU. */
int m4ref_orbits_brute(int64_t n, const int64_t* row_ptr, const int32_t* col, uint64_t* orb);
int m4ref_orbits_esu(int64_t n, const int64_t* row_ptr, const int32_t* col, uint64_t* orb);

/* |N(u) intersect N(v)| by a plain merge of the two sorted rows. */
int64_t m4ref_common(int64_t n, const int64_t* row_ptr, const int32_t* col,
                     int32_t u, int32_t v);

/* Number of threads the O4 loops use for a request of `threads`. */
int m4ref_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
