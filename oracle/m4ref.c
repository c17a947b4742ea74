/*
 * m4ref.c -- CPU oracle for connected induced 4-node motif counts.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.  Plain, slow and
 * written to be checked by eye against the paper:
 *   - Section II defines an induced occurrence of a pattern as a 4-vertex
 *     subset S whose induced subgraph G[S] is isomorphic to the pattern.
 *     O1 (all subsets) and O2 (ESU) apply that definition directly.
 *   - Section III-F gives the closure equations (triangle attachment
 *     classes, edge sides, per-vertex star formula).  O3 applies them as
 *     printed.
 *   - O4 counts the non-induced anchor basis (triangles with per-edge counts,
 *     4-cliques, 4-cycles) plus degree sums and inverts the relation between
 *     non-induced and induced counts.
 * Build: gcc -O2 -fopenmp -shared -fPIC m4ref.c -o libm4ref.so
 */
#include "m4ref.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;
typedef __int128 i128;

enum { STAR = 0, PATH = 1, PAW = 2, CYCLE = 3, DIAMOND = 4, CLIQUE = 5 };

/* --------------------------------------------------------------- helpers */

static int adjacent(const int64_t* rp, const int32_t* col, int32_t u, int32_t v) {
  int64_t lo = rp[u], hi = rp[u + 1];
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < rp[u + 1] && col[lo] == v;
}

/* Position of v inside row u (v must be a neighbour of u). */
static int64_t position(const int64_t* rp, const int32_t* col, int32_t u, int32_t v) {
  int64_t lo = rp[u], hi = rp[u + 1];
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* Class of a 4-vertex induced subgraph from its degrees inside S, or -1 when
 * the subgraph is disconnected.  The sorted degree sequence identifies each
 * connected 4-vertex graph uniquely:
 *   (1,1,1,3) claw, (1,1,2,2) path, (1,2,2,3) paw, (2,2,2,2) cycle,
 *   (2,2,3,3) diamond, (3,3,3,3) clique. */
static int classify(int d0, int d1, int d2, int d3) {
  int d[4] = {d0, d1, d2, d3};
  for (int i = 1; i < 4; i++)
    for (int j = i; j > 0 && d[j - 1] > d[j]; j--) {
      int t = d[j]; d[j] = d[j - 1]; d[j - 1] = t;
    }
  int key = d[0] * 1000 + d[1] * 100 + d[2] * 10 + d[3];
  switch (key) {
    case 1113: return STAR;
    case 1122: return PATH;
    case 1223: return PAW;
    case 2222: return CYCLE;
    case 2233: return DIAMOND;
    case 3333: return CLIQUE;
    default: return -1;
  }
}

static int classify_set(const int64_t* rp, const int32_t* col, const int32_t s[4]) {
  int deg[4] = {0, 0, 0, 0};
  for (int i = 0; i < 4; i++)
    for (int j = i + 1; j < 4; j++)
      if (adjacent(rp, col, s[i], s[j])) { deg[i]++; deg[j]++; }
  return classify(deg[0], deg[1], deg[2], deg[3]);
}

/* Orbit of a vertex inside a connected induced 4-vertex graph of class c,
 * from its degree d inside the set.  Graphlet orbits 4-14 in the numbering of
 * Przulj's graphlet degree vectors (the one ORCA uses): path ends 4, path
 * middles 5, claw leaves 6, claw centre 7, cycle 8, paw tail 9, paw triangle
 * vertices of degree 2 10, paw vertex of degree 3 11, diamond vertices of
 * degree 2 12 and of degree 3 13, clique 14.  In each class the degree inside
 * the set tells the orbits apart. */
static int orbit_of(int c, int d) {
  switch (c) {
    case PATH: return d == 1 ? 4 : 5;
    case STAR: return d == 1 ? 6 : 7;
    case CYCLE: return 8;
    case PAW: return d == 1 ? 9 : (d == 2 ? 10 : 11);
    case DIAMOND: return d == 2 ? 12 : 13;
    case CLIQUE: return 14;
    default: return -1;
  }
}

/* Adds the induced 4-set s to the orbit counts of its four vertices. */
static void add_orbits(const int64_t* rp, const int32_t* col, const int32_t s[4], uint64_t* orb) {
  int deg[4] = {0, 0, 0, 0};
  for (int i = 0; i < 4; i++)
    for (int j = i + 1; j < 4; j++)
      if (adjacent(rp, col, s[i], s[j])) { deg[i]++; deg[j]++; }
  int c = classify(deg[0], deg[1], deg[2], deg[3]);
  if (c < 0) return;
  for (int i = 0; i < 4; i++) orb[(int64_t)s[i] * 11 + orbit_of(c, deg[i]) - 4]++;
}

int m4ref_threads(int threads) {
#ifdef _OPENMP
  return threads > 0 ? threads : omp_get_max_threads();
#else
  (void)threads;
  return 1;
#endif
}

int m4ref_validate(int64_t n, const int64_t* rp, const int32_t* col) {
  if (n < 0 || n > 2147483647LL || !rp) return 1;
  if (rp[0] != 0) return 1;
  for (int64_t v = 0; v < n; v++) {
    if (rp[v + 1] < rp[v]) return 1;
    for (int64_t p = rp[v]; p < rp[v + 1]; p++) {
      int32_t w = col[p];
      if (w < 0 || w >= n || w == v) return 1;
      if (p > rp[v] && col[p - 1] >= w) return 1;
      if (!adjacent(rp, col, w, (int32_t)v)) return 1;
    }
  }
  return 0;
}

int64_t m4ref_common(int64_t n, const int64_t* rp, const int32_t* col,
                     int32_t u, int32_t v) {
  if (u < 0 || v < 0 || u >= n || v >= n) return -1;
  int64_t i = rp[u], j = rp[v], c = 0;
  while (i < rp[u + 1] && j < rp[v + 1]) {
    if (col[i] < col[j]) i++;
    else if (col[i] > col[j]) j++;
    else { c++; i++; j++; }
  }
  return c;
}

/* ------------------------------------------------------ O1: all subsets */

int m4ref_brute(int64_t n, const int64_t* rp, const int32_t* col, uint64_t out[6]) {
  if (n < 0) return 1;
  if (n > 1024) return 7;
  memset(out, 0, 6 * sizeof(uint64_t));
  if (n < 4) return 0;
  unsigned char* A = (unsigned char*)calloc((size_t)(n * n), 1);
  if (!A) return 4;
  for (int64_t u = 0; u < n; u++)
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) A[u * n + col[p]] = 1;
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++)
      for (int64_t c = b + 1; c < n; c++)
        for (int64_t d = c + 1; d < n; d++) {
          int ab = A[a * n + b], ac = A[a * n + c], ad = A[a * n + d];
          int bc = A[b * n + c], bd = A[b * n + d], cd = A[c * n + d];
          int k = classify(ab + ac + ad, ab + bc + bd, ac + bc + cd, ad + bd + cd);
          if (k >= 0) out[k]++;
        }
  free(A);
  return 0;
}

/* -------------------------------------------------------------- O2: ESU */

typedef struct {
  const int64_t* rp;
  const int32_t* col;
  int32_t root;
  int32_t sub[4];
  int32_t* ext[4]; /* extension buffer per depth */
  uint64_t cnt[6];
  uint64_t* orb;   /* n x 11 orbit counts, or NULL */
} esu_state;

/* u is in the closed neighbourhood of the current subgraph sub[0..k) */
static int touches_sub(const esu_state* s, int k, int32_t u) {
  for (int i = 0; i < k; i++)
    if (s->sub[i] == u || adjacent(s->rp, s->col, s->sub[i], u)) return 1;
  return 0;
}

/* ExtendSubgraph(V_sub = sub[0..k), V_ext = ext[k][0..len)) */
static void esu_extend(esu_state* s, int k, int64_t len) {
  if (k == 4) {
    int c = classify_set(s->rp, s->col, s->sub);
    if (c >= 0) s->cnt[c]++;
    if (s->orb) add_orbits(s->rp, s->col, s->sub, s->orb);
    return;
  }
  int32_t* E = s->ext[k];
  while (len > 0) {
    int32_t w = E[--len];
    /* V_ext' = remaining V_ext plus the exclusive neighbours of w that are
     * larger than the root */
    int32_t* E2 = s->ext[k + 1];
    int64_t len2 = 0;
    if (k + 1 < 4) {
      memcpy(E2, E, (size_t)len * sizeof(int32_t));
      len2 = len;
      for (int64_t p = s->rp[w]; p < s->rp[w + 1]; p++) {
        int32_t u = s->col[p];
        if (u > s->root && !touches_sub(s, k, u) && u != w) E2[len2++] = u;
      }
    }
    s->sub[k] = w;
    esu_extend(s, k + 1, len2);
  }
}

int m4ref_esu(int64_t n, const int64_t* rp, const int32_t* col, uint64_t out[6]) {
  if (n < 0) return 1;
  memset(out, 0, 6 * sizeof(uint64_t));
  int64_t dmax = 0;
  for (int64_t v = 0; v < n; v++)
    if (rp[v + 1] - rp[v] > dmax) dmax = rp[v + 1] - rp[v];
  size_t cap = (size_t)(4 * dmax + 8);
  esu_state s;
  memset(&s, 0, sizeof(s));
  s.rp = rp;
  s.col = col;
  for (int i = 0; i < 4; i++) {
    s.ext[i] = (int32_t*)malloc(cap * sizeof(int32_t));
    if (!s.ext[i]) {
      for (int j = 0; j < i; j++) free(s.ext[j]);
      return 4;
    }
  }
  for (int64_t v = 0; v < n; v++) {
    s.root = (int32_t)v;
    s.sub[0] = (int32_t)v;
    int64_t len = 0;
    for (int64_t p = rp[v]; p < rp[v + 1]; p++)
      if (col[p] > v) s.ext[1][len++] = col[p];
    esu_extend(&s, 1, len);
  }
  memcpy(out, s.cnt, sizeof(s.cnt));
  for (int i = 0; i < 4; i++) free(s.ext[i]);
  return 0;
}

/* ------------------------------------------ per-vertex orbit counts (O1, O2) */

int m4ref_orbits_brute(int64_t n, const int64_t* rp, const int32_t* col, uint64_t* orb) {
  if (n < 0) return 1;
  if (n > 1024) return 7;
  memset(orb, 0, (size_t)n * 11 * sizeof(uint64_t));
  for (int32_t a = 0; a < n; a++)
    for (int32_t b = a + 1; b < n; b++)
      for (int32_t c = b + 1; c < n; c++)
        for (int32_t d = c + 1; d < n; d++) {
          const int32_t set[4] = {a, b, c, d};
          add_orbits(rp, col, set, orb);
        }
  return 0;
}

int m4ref_orbits_esu(int64_t n, const int64_t* rp, const int32_t* col, uint64_t* orb) {
  if (n < 0) return 1;
  memset(orb, 0, (size_t)n * 11 * sizeof(uint64_t));
  int64_t dmax = 0;
  for (int64_t v = 0; v < n; v++)
    if (rp[v + 1] - rp[v] > dmax) dmax = rp[v + 1] - rp[v];
  size_t cap = (size_t)(4 * dmax + 8);
  esu_state s;
  memset(&s, 0, sizeof(s));
  s.rp = rp;
  s.col = col;
  s.orb = orb;
  for (int i = 0; i < 4; i++) {
    s.ext[i] = (int32_t*)malloc(cap * sizeof(int32_t));
    if (!s.ext[i]) {
      for (int j = 0; j < i; j++) free(s.ext[j]);
      return 4;
    }
  }
  for (int64_t v = 0; v < n; v++) {
    s.root = (int32_t)v;
    s.sub[0] = (int32_t)v;
    int64_t len = 0;
    for (int64_t p = rp[v]; p < rp[v + 1]; p++)
      if (col[p] > v) s.ext[1][len++] = col[p];
    esu_extend(&s, 1, len);
  }
  for (int i = 0; i < 4; i++) free(s.ext[i]);
  return 0;
}

/* --------------------------------------- O3: closure equations as printed */

int m4ref_paper(int64_t n, const int64_t* rp, const int32_t* col, uint64_t out[6]) {
  if (n < 0) return 1;
  memset(out, 0, 6 * sizeof(uint64_t));
  u128 X[4] = {0, 0, 0, 0};
  u128 path_pairs = 0, cycle_pairs = 0;
  i128 star = 0;
  int32_t* mark = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int32_t* degH = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  if (!mark || !degH) { free(mark); free(degH); return 4; }

  /* Triangle closure: for every triangle T = {a < b < c}, X_j(T) counts the
   * vertices outside T adjacent to exactly j vertices of T. */
  for (int32_t a = 0; a < n; a++)
    for (int64_t pb = rp[a]; pb < rp[a + 1]; pb++) {
      int32_t b = col[pb];
      if (b <= a) continue;
      for (int64_t pc = rp[b]; pc < rp[b + 1]; pc++) {
        int32_t c = col[pc];
        if (c <= b || !adjacent(rp, col, a, c)) continue;
        /* three-way merge of N(a), N(b), N(c) */
        int64_t i = rp[a], j = rp[b], k = rp[c];
        for (;;) {
          int32_t x = 2147483647;
          if (i < rp[a + 1] && col[i] < x) x = col[i];
          if (j < rp[b + 1] && col[j] < x) x = col[j];
          if (k < rp[c + 1] && col[k] < x) x = col[k];
          if (x == 2147483647) break;
          int mult = 0;
          if (i < rp[a + 1] && col[i] == x) { mult++; i++; }
          if (j < rp[b + 1] && col[j] == x) { mult++; j++; }
          if (k < rp[c + 1] && col[k] == x) { mult++; k++; }
          if (x != a && x != b && x != c) X[mult]++;
        }
      }
    }

  /* Edge closure: for every undirected edge e = (u < v), C_e = N(u) & N(v),
   * A_e = N(u) \ (C_e + v), B_e = N(v) \ (C_e + u); adjacent pairs of
   * A_e x B_e close 4-cycles, non-adjacent pairs are induced 4-paths. */
  for (int32_t u = 0; u < n; u++) {
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) mark[col[p]] = 1;
    for (int64_t pv = rp[u]; pv < rp[u + 1]; pv++) {
      int32_t v = col[pv];
      if (v <= u) continue;
      for (int64_t px = rp[u]; px < rp[u + 1]; px++) {
        int32_t x = col[px];
        if (x == v || adjacent(rp, col, v, x)) continue; /* x in A_e */
        for (int64_t py = rp[v]; py < rp[v + 1]; py++) {
          int32_t y = col[py];
          if (y == u || mark[y]) continue; /* y in B_e */
          if (adjacent(rp, col, x, y)) cycle_pairs++;
          else path_pairs++;
        }
      }
    }
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) mark[col[p]] = 0;
  }

  /* Star closure: per vertex u with H_u = G[N(u)],
   * C(d,3) - m(H_u)(d-2) + sum_v C(deg_H(v),2) - tau(H_u). */
  for (int32_t u = 0; u < n; u++) {
    int64_t d = rp[u + 1] - rp[u];
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) mark[col[p]] = 1;
    i128 mH2 = 0, sum_c2 = 0, tau = 0;
    for (int64_t pv = rp[u]; pv < rp[u + 1]; pv++) {
      int32_t v = col[pv];
      int64_t dh = 0;
      for (int64_t q = rp[v]; q < rp[v + 1]; q++) dh += mark[col[q]];
      degH[v] = (int32_t)dh;
      mH2 += dh;
      sum_c2 += (i128)dh * (dh - 1) / 2;
    }
    /* triangles of H_u: v < w < x, all in N(u), pairwise adjacent */
    for (int64_t pv = rp[u]; pv < rp[u + 1]; pv++) {
      int32_t v = col[pv];
      for (int64_t pw = rp[v]; pw < rp[v + 1]; pw++) {
        int32_t w = col[pw];
        if (w <= v || !mark[w]) continue;
        for (int64_t px = rp[w]; px < rp[w + 1]; px++) {
          int32_t x = col[px];
          if (x <= w || !mark[x]) continue;
          if (adjacent(rp, col, v, x)) tau++;
        }
      }
    }
    i128 c3 = (i128)d * (d - 1) * (d - 2) / 6;
    star += c3 - (mH2 / 2) * (d - 2) + sum_c2 - tau;
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) mark[col[p]] = 0;
  }
  free(mark);
  free(degH);

  if (X[2] % 2 || X[3] % 4 || cycle_pairs % 4 || star < 0) return 1;
  u128 res[6];
  res[STAR] = (u128)star;
  res[PATH] = path_pairs;
  res[PAW] = X[1];
  res[CYCLE] = cycle_pairs / 4;
  res[DIAMOND] = X[2] / 2;
  res[CLIQUE] = X[3] / 4;
  for (int i = 0; i < 6; i++) {
    if (res[i] >> 64) return 3;
    out[i] = (uint64_t)res[i];
  }
  return 0;
}

/* ------------------------------------------------- O4: plain closure counter */

/* degree order: a precedes b iff (d_a, a) < (d_b, b) */
static inline int before(const int64_t* rp, int32_t a, int32_t b) {
  int64_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
  return da < db || (da == db && a < b);
}

int m4ref_closure(int64_t n, const int64_t* rp, const int32_t* col, int threads,
                  uint64_t out[6], uint32_t* t_csr, uint64_t basis[8]) {
  if (n < 0 || n > 2147483647LL) return 1;
  memset(out, 0, 6 * sizeof(uint64_t));
  if (basis) memset(basis, 0, 8 * sizeof(uint64_t));
  int nt = m4ref_threads(threads);
  int64_t nnz = rp[n];
  uint32_t* t = t_csr;
  int own_t = 0;
  if (!t) {
    t = (uint32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(uint32_t));
    if (!t) return 4;
    own_t = 1;
  }
  memset(t, 0, (size_t)nnz * sizeof(uint32_t));

  /* out-lists N+(u) = { v in N(u) : u precedes v }, kept in id order */
  int64_t* optr = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  int32_t* ocol = (int32_t*)malloc((size_t)(nnz / 2 + 1) * sizeof(int32_t));
  if (!optr || !ocol) {
    free(optr); free(ocol);
    if (own_t) free(t);
    return 4;
  }
  optr[0] = 0;
  for (int64_t u = 0; u < n; u++) {
    int64_t k = 0;
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) k += before(rp, (int32_t)u, col[p]);
    optr[u + 1] = optr[u] + k;
  }
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
  for (int64_t u = 0; u < n; u++) {
    int64_t k = optr[u];
    for (int64_t p = rp[u]; p < rp[u + 1]; p++)
      if (before(rp, (int32_t)u, col[p])) ocol[k++] = col[p];
  }

  u128 K4 = 0, C4 = 0;
  int fail = 0;
#pragma omp parallel num_threads(nt) reduction(+ : K4, C4) reduction(| : fail)
  {
    unsigned char* inU = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    unsigned char* inV = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    uint32_t* cnt = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!inU || !inV || !cnt || !touched) fail = 1;
#pragma omp for schedule(dynamic, 64)
    for (int64_t uu = 0; uu < n; uu++) {
      if (fail) continue;
      int32_t u = (int32_t)uu;
      /* triangles u < v < w (degree order) and 4-cliques u < v < w < x */
      for (int64_t p = optr[u]; p < optr[u + 1]; p++) inU[ocol[p]] = 1;
      for (int64_t pv = optr[u]; pv < optr[u + 1]; pv++) {
        int32_t v = ocol[pv];
        for (int64_t p = optr[v]; p < optr[v + 1]; p++) inV[ocol[p]] = 1;
        for (int64_t pw = optr[v]; pw < optr[v + 1]; pw++) {
          int32_t w = ocol[pw];
          if (!inU[w]) continue;
          /* triangle {u, v, w}: one more triangle on each of its edges */
          int64_t pos[6] = {position(rp, col, u, v), position(rp, col, v, u),
                            position(rp, col, u, w), position(rp, col, w, u),
                            position(rp, col, v, w), position(rp, col, w, v)};
          for (int i = 0; i < 6; i++) {
#pragma omp atomic
            t[pos[i]]++;
          }
          for (int64_t px = optr[w]; px < optr[w + 1]; px++) {
            int32_t x = ocol[px];
            if (inU[x] && inV[x]) K4++;
          }
        }
        for (int64_t p = optr[v]; p < optr[v + 1]; p++) inV[ocol[p]] = 0;
      }
      for (int64_t p = optr[u]; p < optr[u + 1]; p++) inU[ocol[p]] = 0;

      /* non-induced 4-cycles whose highest vertex is u: for every w below u,
       * cnt[w] = #{v below u adjacent to both u and w}; each pair of such v
       * closes one cycle u-v-w-v'. */
      int64_t nt2 = 0;
      for (int64_t pv = rp[u]; pv < rp[u + 1]; pv++) {
        int32_t v = col[pv];
        if (!before(rp, v, u)) continue;
        for (int64_t pw = rp[v]; pw < rp[v + 1]; pw++) {
          int32_t w = col[pw];
          if (!before(rp, w, u)) continue;
          if (cnt[w]++ == 0) touched[nt2++] = w;
        }
      }
      for (int64_t i = 0; i < nt2; i++) {
        uint64_t c = cnt[touched[i]];
        C4 += (u128)c * (c - 1) / 2;
        cnt[touched[i]] = 0;
      }
    }
    free(inU);
    free(inV);
    free(cnt);
    free(touched);
  }
  free(optr);
  free(ocol);
  if (fail) {
    if (own_t) free(t);
    return 4;
  }

  /* sums over undirected edges (each edge once, from its smaller id end) and
   * over vertices */
  u128 sum_t = 0, P = 0, Paw2 = 0, D = 0, S = 0;
  for (int64_t u = 0; u < n; u++) {
    u128 du = (u128)(rp[u + 1] - rp[u]);
    if (du >= 3) S += du * (du - 1) * (du - 2) / 6;
    for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
      int32_t v = col[p];
      if (v <= u) continue;
      u128 dv = (u128)(rp[v + 1] - rp[v]);
      u128 te = t[p];
      sum_t += te;
      P += (du - 1) * (dv - 1);
      if (te) Paw2 += te * (du + dv - 4);
      D += te * (te - 1) / 2;
    }
  }
  if (own_t) free(t);

  /* Non-induced counts of each pattern and the exact inverse.  A non-induced
   * count of pattern p sums, over induced patterns q, the number of spanning
   * copies of p inside q times the induced count of q:
   *   S      = star + paw + 2 diamond + 4 clique
   *   P_ni   = path + 2 paw + 4 cycle + 6 diamond + 12 clique
   *   Paw_ni = paw + 4 diamond + 12 clique
   *   C4_ni  = cycle + diamond + 3 clique
   *   D_ni   = diamond + 6 clique
   * with P_ni = sum_e (d_u-1)(d_v-1) - 3T, Paw_ni = sum_e t_e (d_u+d_v-4) / 2
   * and D_ni = sum_e C(t_e, 2). */
  if (sum_t % 3 || Paw2 % 2) return 1;
  u128 T = sum_t / 3;
  u128 Pni = P - 3 * T;
  u128 Pawni = Paw2 / 2;
  u128 res[6];
  res[CLIQUE] = K4;
  if (D < 6 * K4) return 1;
  res[DIAMOND] = D - 6 * K4;
  if (C4 < res[DIAMOND] + 3 * K4) return 1;
  res[CYCLE] = C4 - res[DIAMOND] - 3 * K4;
  if (Pawni < 4 * res[DIAMOND] + 12 * K4) return 1;
  res[PAW] = Pawni - 4 * res[DIAMOND] - 12 * K4;
  if (S < res[PAW] + 2 * res[DIAMOND] + 4 * K4) return 1;
  res[STAR] = S - res[PAW] - 2 * res[DIAMOND] - 4 * K4;
  u128 sub = 2 * res[PAW] + 4 * res[CYCLE] + 6 * res[DIAMOND] + 12 * K4;
  if (Pni < sub) return 1;
  res[PATH] = Pni - sub;
  u128 b[8] = {T, K4, C4, S, Pni, Pawni, D, sum_t};
  for (int i = 0; i < 8; i++)
    if (b[i] >> 64) return 3;
  for (int i = 0; i < 6; i++) {
    if (res[i] >> 64) return 3;
    out[i] = (uint64_t)res[i];
  }
  if (basis)
    for (int i = 0; i < 8; i++) basis[i] = (uint64_t)b[i];
  return 0;
}
