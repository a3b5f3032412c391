/*
 * graphgen.c -- seeded synthetic graph generators.
 *
 * This module only produces inputs: simple undirected graphs in CSR form
 * (int32 row pointers, int32 column indices, every row sorted ascending, no
 * self-loops, no duplicate entries, symmetric).  It contains none of the
 * k-clique method's arithmetic and is shared by the tests and the benchmark;
 * neither the oracle nor the GPU library includes or links it.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based
 * stream: state_i = seed + i * 0x9e3779b97f4a7c15, output = mix(state_i).
 *
 * Generators:
 *   - Erdos-Renyi G(n,p) by geometric skipping over the pair index
 *     (Batagelj and Brandes, "Efficient generation of large random networks",
 *     Phys. Rev. E 71, 2005), plus planted cliques on uniform vertex sets.
 *   - Chung-Lu expected-degree graphs, p_ij = min(1, w_i w_j / sum(w)), with
 *     power-law weights w_i = w_max * ((i + i0) / i0)^(-1/(gamma-1)); i0 is
 *     found by bisection so that mean(w) equals the requested average degree.
 *     Sampled in O(n + m) with the skipping method of Miller and Hagberg
 *     ("Efficient generation of networks with given expected degrees", WAW
 *     2011).  Vertex ids are randomly permuted afterwards.
 *   - R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) without noise, plus
 *     planted dense communities (each intra pair present with probability q).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ rng */
typedef struct { uint64_t s; } gg_rng;

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static inline uint64_t gg_next(gg_rng* r) {
  r->s += 0x9e3779b97f4a7c15ULL;
  return gg_mix(r->s);
}
/* uniform double in [0, 1) with 53 random bits */
static inline double gg_unif(gg_rng* r) { return (double)(gg_next(r) >> 11) * (1.0 / 9007199254740992.0); }
/* uniform double in (0, 1] (safe for log) */
static inline double gg_unif_pos(gg_rng* r) { return ((double)(gg_next(r) >> 11) + 1.0) * (1.0 / 9007199254740992.0); }
/* uniform integer in [0, m) (m > 0), multiply-shift with rejection */
static uint64_t gg_below(gg_rng* r, uint64_t m) {
  uint64_t lim = (uint64_t)(-m) % m;
  for (;;) {
    uint64_t x = gg_next(r);
    unsigned __int128 p = (unsigned __int128)x * m;
    if ((uint64_t)p >= lim) return (uint64_t)(p >> 64);
  }
}

uint64_t gg_stream_seed(uint64_t seed, uint64_t substream) {
  return gg_mix(seed ^ gg_mix(substream + 0x632be59bd9b4e019ULL));
}

/* ------------------------------------------------------------ edge list */
typedef struct {
  uint64_t* e; /* (u << 32) | v */
  size_t len, cap;
} gg_edges;

static int edges_push(gg_edges* el, uint32_t u, uint32_t v) {
  if (u == v) return 0; /* self-loops are dropped */
  if (el->len == el->cap) {
    size_t nc = el->cap ? el->cap * 2 : 1024;
    uint64_t* ne = (uint64_t*)realloc(el->e, nc * sizeof(uint64_t));
    if (!ne) return -1;
    el->e = ne;
    el->cap = nc;
  }
  el->e[el->len++] = ((uint64_t)u << 32) | v;
  return 0;
}

/* ------------------------------------------------------------- graph */
typedef struct {
  int32_t n;
  int64_t nnz;
  int32_t* row_ptr; /* n+1 (int32: nnz must stay below 2^31) */
  int32_t* col;
  int32_t status; /* 0 ok, -1 out of memory, -2 too large */
} gg_graph;

static void insertion_sort_i32(int32_t* a, int64_t len) {
  for (int64_t i = 1; i < len; ++i) {
    int32_t x = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
    a[j + 1] = x;
  }
}
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Symmetrise, sort rows, drop duplicates; consumes the edge list. */
static gg_graph* csr_from_edges(int32_t n, gg_edges* el) {
  gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph));
  if (!g) return NULL;
  g->n = n;
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) { g->status = -1; free(el->e); el->e = NULL; return g; }
  for (size_t i = 0; i < el->len; ++i) {
    uint32_t u = (uint32_t)(el->e[i] >> 32), v = (uint32_t)el->e[i];
    deg[u]++;
    deg[v]++;
  }
  int64_t total = 0;
  for (int32_t i = 0; i < n; ++i) { int64_t d = deg[i]; deg[i] = total; total += d; }
  deg[n] = total;
  int32_t* col = (int32_t*)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  int64_t* fill = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!col || !fill) { free(col); free(fill); free(deg); g->status = -1; free(el->e); el->e = NULL; return g; }
  memcpy(fill, deg, ((size_t)n + 1) * sizeof(int64_t));
  for (size_t i = 0; i < el->len; ++i) {
    uint32_t u = (uint32_t)(el->e[i] >> 32), v = (uint32_t)el->e[i];
    col[fill[u]++] = (int32_t)v;
    col[fill[v]++] = (int32_t)u;
  }
  free(el->e);
  el->e = NULL;
  el->len = el->cap = 0;
  free(fill);
  /* sort + dedup each row, compacting in place */
  int64_t out = 0;
  int32_t* rp = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  if (!rp) { free(col); free(deg); g->status = -1; return g; }
  for (int32_t u = 0; u < n; ++u) {
    int64_t b = deg[u], e = deg[u + 1], len = e - b;
    if (len > 48) qsort(col + b, (size_t)len, sizeof(int32_t), cmp_i32);
    else insertion_sort_i32(col + b, len);
    rp[u] = (int32_t)out;
    int64_t start = out;
    for (int64_t i = b; i < e; ++i) {
      if (out > start && col[out - 1] == col[i]) continue;
      col[out++] = col[i];
    }
    if (out > INT32_MAX) { free(rp); free(col); free(deg); g->status = -2; return g; }
  }
  rp[n] = (int32_t)out;
  free(deg);
  g->nnz = out;
  g->row_ptr = rp;
  int32_t* shrunk = (int32_t*)realloc(col, (size_t)(out ? out : 1) * sizeof(int32_t));
  g->col = shrunk ? shrunk : col;
  return g;
}

/* ---------------------------------------------------------- planting */
/* Adds a clique on `size` distinct uniform vertices (partial Fisher-Yates). */
static int plant_clique(gg_edges* el, int32_t n, int32_t size, gg_rng* r, int32_t* perm, int32_t* members) {
  if (size > n) size = n;
  for (int32_t i = 0; i < size; ++i) {
    int32_t j = i + (int32_t)gg_below(r, (uint64_t)(n - i));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    members[i] = perm[i];
  }
  for (int32_t i = 0; i < size; ++i)
    for (int32_t j = i + 1; j < size; ++j)
      if (edges_push(el, (uint32_t)members[i], (uint32_t)members[j])) return -1;
  return 0;
}
/* Adds a community on `size` uniform vertices with each pair kept w.p. q. */
static int plant_community(gg_edges* el, int32_t n, int32_t size, double q, gg_rng* r, int32_t* perm,
                           int32_t* members) {
  if (size > n) size = n;
  for (int32_t i = 0; i < size; ++i) {
    int32_t j = i + (int32_t)gg_below(r, (uint64_t)(n - i));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    members[i] = perm[i];
  }
  for (int32_t i = 0; i < size; ++i)
    for (int32_t j = i + 1; j < size; ++j)
      if (gg_unif(r) < q)
        if (edges_push(el, (uint32_t)members[i], (uint32_t)members[j])) return -1;
  return 0;
}

static int32_t* identity_perm(int32_t n) {
  int32_t* p = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
  if (p)
    for (int32_t i = 0; i < n; ++i) p[i] = i;
  return p;
}

static int plant_list(gg_edges* el, int32_t n, int32_t n_planted, const int32_t* sizes, gg_rng* r) {
  if (n_planted <= 0) return 0;
  int32_t* perm = identity_perm(n);
  int32_t maxs = 0;
  for (int32_t i = 0; i < n_planted; ++i) maxs = sizes[i] > maxs ? sizes[i] : maxs;
  int32_t* mem = (int32_t*)malloc(((size_t)maxs + 1) * sizeof(int32_t));
  int rc = (!perm || !mem) ? -1 : 0;
  for (int32_t i = 0; i < n_planted && !rc; ++i) rc = plant_clique(el, n, sizes[i], r, perm, mem);
  free(perm);
  free(mem);
  return rc;
}

/* --------------------------------------------------------------- ER */
gg_graph* gg_erdos_renyi(int32_t n, double p, int32_t n_planted, const int32_t* planted_sizes, uint64_t seed) {
  gg_edges el = {0};
  gg_rng r = {gg_stream_seed(seed, 1)};
  int rc = 0;
  if (n >= 2 && p > 0.0) {
    if (p >= 1.0) {
      for (int32_t v = 1; v < n && !rc; ++v)
        for (int32_t w = 0; w < v && !rc; ++w) rc = edges_push(&el, (uint32_t)v, (uint32_t)w);
    } else {
      /* Batagelj-Brandes: walk the lower triangle (v > w) with geometric skips */
      double lq = log(1.0 - p);
      int64_t v = 1, w = -1;
      while (v < n && !rc) {
        double u = gg_unif_pos(&r);
        w = w + 1 + (int64_t)floor(log(u) / lq);
        while (w >= v && v < n) { w -= v; v++; }
        if (v < n) rc = edges_push(&el, (uint32_t)v, (uint32_t)w);
      }
    }
  }
  gg_rng rp = {gg_stream_seed(seed, 2)};
  if (!rc) rc = plant_list(&el, n, n_planted, planted_sizes, &rp);
  if (rc) { free(el.e); gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -1; return g; }
  return csr_from_edges(n, &el);
}

/* ---------------------------------------------------------- Chung-Lu */
static double cl_mean(int32_t n, double gamma, double wmax, double i0) {
  double ex = -1.0 / (gamma - 1.0), s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += wmax * pow(((double)i + i0) / i0, ex);
  return s / (double)n;
}

/* Solves i0 so that mean weight equals avg_deg (returns < 0 if impossible). */
double gg_chung_lu_i0(int32_t n, double avg_deg, double gamma, double w_max) {
  if (!(avg_deg > 0.0) || !(w_max > avg_deg) || !(gamma > 1.0) || n <= 0) return -1.0;
  double lo = log(1e-9), hi = log(1e15);
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (cl_mean(n, gamma, w_max, exp(mid)) < avg_deg) lo = mid; else hi = mid;
  }
  return exp(0.5 * (lo + hi));
}

gg_graph* gg_chung_lu(int32_t n, double avg_deg, double gamma, double w_max, int32_t n_planted,
                      const int32_t* planted_sizes, uint64_t seed) {
  gg_edges el = {0};
  int rc = 0;
  double* w = (double*)malloc(((size_t)n + 1) * sizeof(double));
  double i0 = gg_chung_lu_i0(n, avg_deg, gamma, w_max);
  if (!w || i0 <= 0.0) { free(w); gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -3; return g; }
  double ex = -1.0 / (gamma - 1.0), S = 0.0;
  for (int32_t i = 0; i < n; ++i) { w[i] = w_max * pow(((double)i + i0) / i0, ex); S += w[i]; }
  gg_rng r = {gg_stream_seed(seed, 3)};
  /* weights are non-increasing in i, so p(u, v) is non-increasing in v > u */
  for (int32_t u = 0; u < n - 1 && !rc; ++u) {
    int64_t v = u + 1;
    double p = w[u] * w[v] / S;
    if (p > 1.0) p = 1.0;
    while (v < n && p > 0.0 && !rc) {
      if (p < 1.0) {
        double x = gg_unif_pos(&r);
        v += (int64_t)floor(log(x) / log(1.0 - p));
      }
      if (v < n) {
        double q = w[u] * w[v] / S;
        if (q > 1.0) q = 1.0;
        if (gg_unif(&r) < q / p) rc = edges_push(&el, (uint32_t)u, (uint32_t)v);
        p = q;
        v++;
      }
    }
  }
  free(w);
  gg_rng rp = {gg_stream_seed(seed, 4)};
  if (!rc) rc = plant_list(&el, n, n_planted, planted_sizes, &rp);
  /* random relabelling so that ids carry no weight information */
  if (!rc) {
    int32_t* perm = identity_perm(n);
    if (!perm) rc = -1;
    else {
      gg_rng rr = {gg_stream_seed(seed, 5)};
      for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)gg_below(&rr, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
      }
      for (size_t i = 0; i < el.len; ++i) {
        uint32_t a = (uint32_t)(el.e[i] >> 32), b = (uint32_t)el.e[i];
        el.e[i] = ((uint64_t)(uint32_t)perm[a] << 32) | (uint32_t)perm[b];
      }
      free(perm);
    }
  }
  if (rc) { free(el.e); gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -1; return g; }
  return csr_from_edges(n, &el);
}

/* ------------------------------------------------------------- R-MAT */
gg_graph* gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, int32_t n_comm,
                  int32_t comm_min, int32_t comm_max, double comm_p, uint64_t seed) {
  gg_edges el = {0};
  int rc = 0;
  if (scale < 1 || scale > 30) { gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -3; return g; }
  int32_t n = (int32_t)1 << scale;
  int64_t samples = (int64_t)edge_factor << scale;
  gg_rng r = {gg_stream_seed(seed, 6)};
  double ab = a + b, abc = a + b + c;
  for (int64_t s = 0; s < samples && !rc; ++s) {
    uint32_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double x = gg_unif(&r);
      uint32_t bu, bv;
      if (x < a) { bu = 0; bv = 0; }
      else if (x < ab) { bu = 0; bv = 1; }
      else if (x < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    rc = edges_push(&el, u, v);
  }
  if (!rc && n_comm > 0) {
    gg_rng rc2 = {gg_stream_seed(seed, 7)};
    int32_t* perm = identity_perm(n);
    int32_t* mem = (int32_t*)malloc(((size_t)comm_max + 1) * sizeof(int32_t));
    if (!perm || !mem) rc = -1;
    for (int32_t i = 0; i < n_comm && !rc; ++i) {
      int32_t size = comm_min + (int32_t)gg_below(&rc2, (uint64_t)(comm_max - comm_min + 1));
      rc = plant_community(&el, n, size, comm_p, &rc2, perm, mem);
    }
    free(perm);
    free(mem);
  }
  if (rc) { free(el.e); gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -1; return g; }
  return csr_from_edges(n, &el);
}

/* ------------------------------------------------ explicit edge list */
gg_graph* gg_from_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  gg_edges el = {0};
  int rc = 0;
  for (int64_t i = 0; i < m && !rc; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) continue;
    rc = edges_push(&el, (uint32_t)src[i], (uint32_t)dst[i]);
  }
  if (rc) { free(el.e); gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph)); if (g) g->status = -1; return g; }
  return csr_from_edges(n, &el);
}

/* --------------------------------------------------------- accessors */
int32_t gg_status(const gg_graph* g) { return g ? g->status : -1; }
int32_t gg_n(const gg_graph* g) { return g ? g->n : 0; }
int64_t gg_nnz(const gg_graph* g) { return g ? g->nnz : 0; }
void gg_copy(const gg_graph* g, int32_t* row_ptr, int32_t* col) {
  if (!g || g->status) return;
  memcpy(row_ptr, g->row_ptr, ((size_t)g->n + 1) * sizeof(int32_t));
  if (g->nnz) memcpy(col, g->col, (size_t)g->nnz * sizeof(int32_t));
}
void gg_free(gg_graph* g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  free(g);
}

/* Raw stream access so that tests can check the generator against its
 * published definition. */
void gg_stream(uint64_t seed, uint64_t substream, int64_t count, uint64_t* out) {
  gg_rng r = {gg_stream_seed(seed, substream)};
  for (int64_t i = 0; i < count; ++i) out[i] = gg_next(&r);
}
