/*
 * m4gen.c -- seeded synthetic graph generators.  See m4gen.h.
 * Build: gcc -O3 -fopenmp -shared -fPIC m4gen.c -o libm4gen.so -lm
 */
#include "m4gen.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- RNG -- */

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return sm64_mix(seed ^ sm64_mix(stream * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL));
}
static inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return sm64_mix(key + (ctr + 1) * 0x9e3779b97f4a7c15ULL);
}
static inline double unif(uint64_t key, uint64_t ctr) {
  return (double)(draw(key, ctr) >> 11) * (1.0 / 9007199254740992.0);
}
/* uniform integer in [0, k) by 128-bit multiply (Lemire), k >= 1 */
static inline uint64_t below(uint64_t key, uint64_t ctr, uint64_t k) {
  return (uint64_t)(((unsigned __int128)draw(key, ctr) * k) >> 64);
}

double m4gen_uniform(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return unif(stream_key(seed, stream), ctr);
}

/* ----------------------------------------------------- CSR from edges -- */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static void sort_row(int32_t* r, int64_t len) {
  if (len <= 32) {
    for (int64_t i = 1; i < len; i++) {
      int32_t x = r[i];
      int64_t j = i - 1;
      while (j >= 0 && r[j] > x) { r[j + 1] = r[j]; j--; }
      r[j + 1] = x;
    }
  } else {
    qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

int m4gen_from_edges(int64_t n, int64_t ne, const int32_t* src,
                     const int32_t* dst, m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n < 0 || ne < 0 || n > 2147483647LL) return -1;
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
  int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
  for (int64_t i = 0; i < ne; i++) {
    int32_t u = src[i], v = dst[i];
    if (u < 0 || v < 0 || u >= n || v >= n) { bad = 1; continue; }
    if (u == v) continue;
#pragma omp atomic
    cnt[u]++;
#pragma omp atomic
    cnt[v]++;
  }
  if (bad) { free(cnt); return -1; }
  int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!off) { free(cnt); return -2; }
  off[0] = 0;
  for (int64_t v = 0; v < n; v++) off[v + 1] = off[v] + cnt[v];
  int64_t tot = off[n];
  int32_t* tmp = (int32_t*)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  if (!tmp) { free(cnt); free(off); return -2; }
  memset(cnt, 0, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ne; i++) {
    int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    int64_t pu, pv;
#pragma omp atomic capture
    pu = cnt[u]++;
#pragma omp atomic capture
    pv = cnt[v]++;
    tmp[off[u] + pu] = v;
    tmp[off[v] + pv] = u;
  }
  /* sort + dedup every row in place, remember the new lengths in cnt */
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; v++) {
    int32_t* r = tmp + off[v];
    int64_t len = off[v + 1] - off[v];
    sort_row(r, len);
    int64_t k = 0;
    for (int64_t i = 0; i < len; i++)
      if (k == 0 || r[i] != r[k - 1]) r[k++] = r[i];
    cnt[v] = k;
  }
  int64_t* rp = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!rp) { free(cnt); free(off); free(tmp); return -2; }
  rp[0] = 0;
  for (int64_t v = 0; v < n; v++) rp[v + 1] = rp[v] + cnt[v];
  int64_t nnz = rp[n];
  int32_t* col = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!col) { free(cnt); free(off); free(tmp); free(rp); return -2; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; v++)
    memcpy(col + rp[v], tmp + off[v], (size_t)cnt[v] * sizeof(int32_t));
  free(cnt);
  free(off);
  free(tmp);
  g->n = n;
  g->nnz = nnz;
  g->row_ptr = rp;
  g->col = col;
  return 0;
}

void m4gen_free(m4gen_graph* g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  memset(g, 0, sizeof(*g));
}

/* ------------------------------------------------------------ G(n, m) -- */

typedef struct {
  uint64_t* keys;
  uint64_t mask;
} pairset;

static int pairset_init(pairset* s, int64_t want) {
  uint64_t cap = 16;
  while (cap < (uint64_t)want * 2 + 16) cap <<= 1;
  s->keys = (uint64_t*)malloc(cap * sizeof(uint64_t));
  if (!s->keys) return -2;
  memset(s->keys, 0xff, cap * sizeof(uint64_t));
  s->mask = cap - 1;
  return 0;
}
/* returns 1 if inserted, 0 if already present */
static int pairset_add(pairset* s, uint64_t k) {
  uint64_t h = sm64_mix(k) & s->mask;
  for (;;) {
    if (s->keys[h] == ~0ULL) { s->keys[h] = k; return 1; }
    if (s->keys[h] == k) return 0;
    h = (h + 1) & s->mask;
  }
}
static int pairset_has(const pairset* s, uint64_t k) {
  uint64_t h = sm64_mix(k) & s->mask;
  for (;;) {
    if (s->keys[h] == ~0ULL) return 0;
    if (s->keys[h] == k) return 1;
    h = (h + 1) & s->mask;
  }
}

int m4gen_gnm(int64_t n, int64_t m, uint64_t seed, m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n < 0 || m < 0 || n > 2147483647LL) return -1;
  int64_t maxm = n * (n - 1) / 2;
  if (m > maxm) m = maxm;
  uint64_t key = stream_key(seed, 0x676e6dULL);
  /* dense requests sample the complement instead */
  int complement = (m > maxm / 2);
  int64_t want = complement ? maxm - m : m;
  pairset s;
  if (pairset_init(&s, want)) return -2;
  int64_t got = 0;
  uint64_t ctr = 0;
  while (got < want) {
    uint64_t u = below(key, ctr++, (uint64_t)n);
    uint64_t v = below(key, ctr++, (uint64_t)n);
    if (u == v) continue;
    if (u > v) { uint64_t t = u; u = v; v = t; }
    got += pairset_add(&s, (u << 32) | v);
  }
  int32_t* src = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!src || !dst) { free(s.keys); free(src); free(dst); return -2; }
  int64_t k = 0;
  if (!complement) {
    for (uint64_t h = 0; h <= s.mask; h++)
      if (s.keys[h] != ~0ULL) {
        src[k] = (int32_t)(s.keys[h] >> 32);
        dst[k] = (int32_t)(s.keys[h] & 0xffffffffULL);
        k++;
      }
  } else {
    for (int64_t u = 0; u < n; u++)
      for (int64_t v = u + 1; v < n; v++)
        if (!pairset_has(&s, ((uint64_t)u << 32) | (uint64_t)v)) {
          src[k] = (int32_t)u;
          dst[k] = (int32_t)v;
          k++;
        }
  }
  free(s.keys);
  int rc = m4gen_from_edges(n, k, src, dst, g);
  free(src);
  free(dst);
  return rc;
}

/* -------------------------------------------------------------- R-MAT -- */

static int32_t* random_permutation(int64_t n, uint64_t key) {
  int32_t* p = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!p) return NULL;
  for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)below(key, (uint64_t)i, (uint64_t)i + 1);
    int32_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
  return p;
}

int m4gen_rmat(int scale, int64_t edge_factor, double a, double b, double c,
               uint64_t seed, int permute, m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (scale < 1 || scale > 30 || edge_factor < 0 || a < 0 || b < 0 || c < 0 ||
      a + b + c > 1.0)
    return -1;
  int64_t n = 1LL << scale;
  int64_t ne = n * edge_factor;
  uint64_t key = stream_key(seed, 0x726d6174ULL);
  int32_t* src = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  if (!src || !dst) { free(src); free(dst); return -2; }
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ne; i++) {
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; l++) {
      double r = unif(key, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
      uint32_t bu, bv;
      if (r < a) { bu = 0; bv = 0; }
      else if (r < ab) { bu = 0; bv = 1; }
      else if (r < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  if (permute) {
    int32_t* p = random_permutation(n, stream_key(seed, 0x7065726dULL));
    if (!p) { free(src); free(dst); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; i++) {
      src[i] = p[src[i]];
      dst[i] = p[dst[i]];
    }
    free(p);
  }
  int rc = m4gen_from_edges(n, ne, src, dst, g);
  free(src);
  free(dst);
  return rc;
}

/* ---------------------------------------------------- Barabasi-Albert -- */

int m4gen_ba(int64_t n, int m_ba, uint64_t seed, m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n < 0 || m_ba < 1 || n > 2147483647LL) return -1;
  uint64_t key = stream_key(seed, 0x6261ULL);
  int64_t s0 = (n < (int64_t)m_ba + 1) ? n : (int64_t)m_ba + 1;
  int64_t maxe = (s0 > 0 ? s0 - 1 : 0) + (n > s0 ? (n - s0) * (int64_t)m_ba : 0);
  int32_t* src = (int32_t*)malloc((size_t)(maxe > 0 ? maxe : 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)(maxe > 0 ? maxe : 1) * sizeof(int32_t));
  /* endpoint list: every vertex appears once per incident edge */
  int32_t* ends = (int32_t*)malloc((size_t)(2 * maxe > 0 ? 2 * maxe : 1) * sizeof(int32_t));
  int32_t* pick = (int32_t*)malloc((size_t)m_ba * sizeof(int32_t));
  if (!src || !dst || !ends || !pick) {
    free(src); free(dst); free(ends); free(pick);
    return -2;
  }
  int64_t k = 0, ne = 0;
  uint64_t ctr = 0;
  for (int64_t v = 1; v < s0; v++) { /* star seed graph centred on 0 */
    src[k] = 0; dst[k] = (int32_t)v; k++;
    ends[ne++] = 0; ends[ne++] = (int32_t)v;
  }
  for (int64_t t = s0; t < n; t++) {
    int got = 0;
    while (got < m_ba) {
      int32_t w = ends[below(key, ctr++, (uint64_t)ne)];
      int dup = 0;
      for (int i = 0; i < got; i++) dup |= (pick[i] == w);
      if (!dup) pick[got++] = w;
    }
    for (int i = 0; i < m_ba; i++) {
      src[k] = (int32_t)t; dst[k] = pick[i]; k++;
      ends[ne++] = (int32_t)t; ends[ne++] = pick[i];
    }
  }
  free(ends);
  free(pick);
  int rc = m4gen_from_edges(n, k, src, dst, g);
  free(src);
  free(dst);
  return rc;
}

/* ---------------------------------------------------------- Chung-Lu -- */

int m4gen_chunglu(int64_t n, double beta, double mean_deg, uint64_t seed,
                  m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n < 1 || beta <= 1.0 || mean_deg < 0 || n > 2147483647LL) return -1;
  double* cdf = (double*)malloc((size_t)n * sizeof(double));
  if (!cdf) return -2;
  double ex = -1.0 / (beta - 1.0), tot = 0.0;
  for (int64_t i = 0; i < n; i++) { cdf[i] = pow((double)(i + 1), ex); tot += cdf[i]; }
  double scale = mean_deg * (double)n / tot, cap = sqrt(mean_deg * (double)n);
  double acc = 0.0;
  for (int64_t i = 0; i < n; i++) {
    double w = cdf[i] * scale;
    if (w > cap) w = cap;
    acc += w;
    cdf[i] = acc;
  }
  int64_t ne = (int64_t)llround((double)n * mean_deg / 2.0);
  uint64_t key = stream_key(seed, 0x636cULL);
  int32_t* src = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  int32_t* p = random_permutation(n, stream_key(seed, 0x636c70ULL));
  if (!src || !dst || !p) { free(cdf); free(src); free(dst); free(p); return -2; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ne; i++) {
    int32_t e[2];
    for (int s = 0; s < 2; s++) {
      double r = unif(key, 2 * (uint64_t)i + (uint64_t)s) * acc;
      int64_t lo = 0, hi = n - 1;
      while (lo < hi) { /* first index with cdf > r */
        int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > r) hi = mid; else lo = mid + 1;
      }
      e[s] = p[lo];
    }
    src[i] = e[0];
    dst[i] = e[1];
  }
  free(cdf);
  free(p);
  int rc = m4gen_from_edges(n, ne, src, dst, g);
  free(src);
  free(dst);
  return rc;
}

/* ---------------------------------------------- random geometric graph -- */

int m4gen_rgg(int64_t n, double mean_deg, uint64_t seed, m4gen_graph* g) {
  memset(g, 0, sizeof(*g));
  if (n < 1 || mean_deg < 0 || n > 2147483647LL) return -1;
  uint64_t key = stream_key(seed, 0x726767ULL);
  double r = sqrt(mean_deg / (M_PI * (double)n));
  int64_t G = (int64_t)floor(1.0 / (r > 0 ? r : 1.0));
  if (G < 1) G = 1;
  if (G > 65536) G = 65536;
  double* x = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  int64_t* cell_start = (int64_t*)calloc((size_t)(G * G + 1), sizeof(int64_t));
  int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* cur = (int64_t*)malloc((size_t)(G * G) * sizeof(int64_t));
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  if (!x || !y || !cell_start || !order || !cur || !cnt) {
    free(x); free(y); free(cell_start); free(order); free(cur); free(cnt);
    return -2;
  }
  for (int64_t i = 0; i < n; i++) {
    x[i] = unif(key, 2 * (uint64_t)i);
    y[i] = unif(key, 2 * (uint64_t)i + 1);
    int64_t cx = (int64_t)(x[i] * (double)G), cy = (int64_t)(y[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    cell_start[cx * G + cy + 1]++;
  }
  for (int64_t c = 0; c < G * G; c++) cell_start[c + 1] += cell_start[c];
  memcpy(cur, cell_start, (size_t)(G * G) * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) {
    int64_t cx = (int64_t)(x[i] * (double)G), cy = (int64_t)(y[i] * (double)G);
    if (cx >= G) cx = G - 1;
    if (cy >= G) cy = G - 1;
    order[cur[cx * G + cy]++] = (int32_t)i;
  }
  free(cur);
  const double r2 = r * r;
  /* two passes over the same neighbourhood scan: count, then emit */
  int64_t* eoff = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!eoff) { free(x); free(y); free(cell_start); free(order); free(cnt); return -2; }
  int32_t *src = NULL, *dst = NULL;
  for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
      int64_t cx = (int64_t)(x[i] * (double)G), cy = (int64_t)(y[i] * (double)G);
      if (cx >= G) cx = G - 1;
      if (cy >= G) cy = G - 1;
      int64_t k = 0;
      for (int64_t dx = -1; dx <= 1; dx++)
        for (int64_t dy = -1; dy <= 1; dy++) {
          int64_t ax = cx + dx, ay = cy + dy;
          if (ax < 0 || ay < 0 || ax >= G || ay >= G) continue;
          int64_t c = ax * G + ay;
          for (int64_t q = cell_start[c]; q < cell_start[c + 1]; q++) {
            int32_t j = order[q];
            if (j <= i) continue;
            double ddx = x[i] - x[j], ddy = y[i] - y[j];
            if (ddx * ddx + ddy * ddy < r2) {
              if (pass == 1) {
                src[eoff[i] + k] = (int32_t)i;
                dst[eoff[i] + k] = j;
              }
              k++;
            }
          }
        }
      if (pass == 0) cnt[i] = k;
    }
    if (pass == 0) {
      eoff[0] = 0;
      for (int64_t i = 0; i < n; i++) eoff[i + 1] = eoff[i] + cnt[i];
      src = (int32_t*)malloc((size_t)(eoff[n] > 0 ? eoff[n] : 1) * sizeof(int32_t));
      dst = (int32_t*)malloc((size_t)(eoff[n] > 0 ? eoff[n] : 1) * sizeof(int32_t));
      if (!src || !dst) {
        free(x); free(y); free(cell_start); free(order); free(cnt); free(eoff);
        free(src); free(dst);
        return -2;
      }
    }
  }
  int64_t ne = eoff[n];
  free(x); free(y); free(cell_start); free(order); free(cnt); free(eoff);
  int rc = m4gen_from_edges(n, ne, src, dst, g);
  free(src);
  free(dst);
  return rc;
}
