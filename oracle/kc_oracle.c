/*
 * kc_oracle.c -- CPU oracle for exact k-clique counting.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Graphs are simple undirected graphs in CSR form: row_ptr[n+1] and
 * col[row_ptr[n]] (int32), rows sorted ascending, symmetric, no loops.
 *
 * Contents and where each piece comes from in the paper
 * ("Efficient k-clique Listing with Set Intersection Speedup"):
 *
 *   orc_binom            C(n, k) exactly, with overflow detection (used for
 *                        the clique components of Pre-List, Sec. 5.2).
 *   orc_count_brute      plain definition of the result (Def. 2 and the
 *                        problem statement of Sec. 3.1): every k-subset is
 *                        tested for pairwise adjacency.  n <= 30.
 *   orc_count_idorder    the same result by the textbook ordered recursion
 *                        (the kClist scheme of Alg. 2 with eta = vertex id):
 *                        each clique is counted once, from its smallest id.
 *                        Optional per-vertex participation counts.
 *   orc_list_idorder     listing: the same recursion writing each clique's ids.
 *   orc_vertex_count     per-vertex participation of one vertex v: the number
 *                        of (k-1)-cliques in the subgraph induced by N(v).
 *   orc_core_numbers     core numbers by the bucket algorithm of Batagelj and
 *                        Zaversnik (the "classic core decomposition" the
 *                        paper cites for degeneracy, Sec. 3).
 *   orc_precore          Pre-Core, Alg. 3 (queue-based (k-1)-core peel).
 *   orc_prelist          Pre-List, Alg. 4 (components that are cliques).
 *   orc_degree_dag       degree ordering of Sec. 6.2: u -> v iff
 *                        (d_u, u) < (d_v, v) on the reduced graph.
 *   orc_degeneracy_dag   degeneracy ordering (Sec. 7.4) as a synchronous peel.
 *   orc_sdegree_dag      SDegree, Alg. 5, instrumented per root (orc_sdegree_roots:
 *                        the same from a list of roots).
 *   orc_greedy_color     greedy coloring in inverse degree order (Sec. 7.1).
 *   orc_bitcol_dag       BitCol, Alg. 6, instrumented per root.
 *
 * Readings of passages that are ambiguous or garbled in the paper:
 *   - Pre-Core removes vertices of degree < k-1 (Alg. 3), keeping the
 *     (k-1)-core.
 *   - Pre-List's clique test counts adjacency entries in both directions:
 *     a component with n_c vertices is a clique iff its degree sum equals
 *     n_c (n_c - 1).  It contributes C(n_c, k) cliques and C(n_c-1, k-1) to
 *     each member.
 *   - Degree ordering uses the degrees of the graph left by Pre-Core and
 *     Pre-List; ties go to the smaller vertex id.
 *   - Degeneracy ordering: a synchronous peel.  Level c starts at 0; each
 *     round removes every live vertex of live degree <= c at once and gives
 *     them the next round number; when a round finds nothing, c grows by one.
 *     u -> v iff (round_u, u) < (round_v, v).  Out-degree <= core number.
 *   - Greedy coloring order: descending degree inside G_u, ties by ascending
 *     vertex id; colors are 1-based; a vertex takes the smallest color not
 *     used by an already-colored neighbour.
 *   - BitCol bitmaps: bit i of word j stands for local vertex j*L + i (least
 *     significant bit first, as in the paper's encoding table); local vertices
 *     are the members of N+(u) in ascending id order; B(v) holds the
 *     neighbours of v in G_u of strictly smaller color.
 *   - Work per root: `nodes` counts calls of the listing procedure (the top
 *     call included), `isect` counts set intersections (merge joins or
 *     BitJoins), `elems` adds |C| + d+_u per merge join (the cost term of
 *     Lemma 2) and `words` adds ceil(s / 32) per BitJoin.
 *
 * Parity status: counts, per-vertex counts, Pre-Core, Pre-List, both
 * orientations, the coloring and the encoding are pinned by the CPU tests
 * (brute force, closed forms, core numbers, the paper's worked examples and
 * encoding table).  The per-root work counters are pinned by hand-derived
 * traces of the paper's own examples: SDegree's (nodes, isect, elems) by the
 * Example 4 recursion from v2 and v5, BitCol's (count, nodes, isect, words,
 * colors, |E_u|) by Alg. 6 run by hand on the Example 6 / Table 3 local graph
 * at k = 3..6; plus the Lemma 4 bound.  The paper itself prints no per-root
 * work values, so beyond those traces they rest on the readings above.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-3)
#define ORC_EBUDGET (-6)

typedef unsigned __int128 u128;

static int add_checked(uint64_t* acc, uint64_t x) {
  uint64_t s = *acc + x;
  if (s < *acc) return 1;
  *acc = s;
  return 0;
}

/* ----------------------------------------------------------- binomial */
int orc_binom(uint64_t n, uint64_t k, uint64_t* out) {
  if (k > n) { *out = 0; return ORC_OK; }
  if (k > n - k) k = n - k;
  /* r_i = C(n-k+i, i); r_i = r_{i-1} * (n-k+i) / i is exact */
  u128 r = 1;
  for (uint64_t i = 1; i <= k; ++i) {
    r = r * (u128)(n - k + i);
    r /= i;
    if (r > (u128)UINT64_MAX) return ORC_EOVERFLOW;
  }
  *out = (uint64_t)r;
  return ORC_OK;
}

/* ---------------------------------------------------- input validation */
int orc_validate(int32_t n, const int32_t* rp, const int32_t* col) {
  if (n < 0) return ORC_EINVAL;
  if (n == 0) return ORC_OK;
  if (rp[0] != 0) return ORC_EINVAL;
  for (int32_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) return ORC_EINVAL;
    for (int32_t i = rp[v]; i < rp[v + 1]; ++i) {
      int32_t w = col[i];
      if (w < 0 || w >= n || w == v) return ORC_EINVAL;
      if (i > rp[v] && col[i - 1] >= w) return ORC_EINVAL;
      /* symmetry: v must appear in w's row (binary search) */
      int32_t lo = rp[w], hi = rp[w + 1];
      while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (lo >= rp[w + 1] || col[lo] != v) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

/* ----------------------------------------------------- O0: brute force */
int orc_count_brute(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, uint64_t* count,
                    uint64_t* pv) {
  if (n < 0 || n > 30 || k < 1) return ORC_EINVAL;
  uint32_t adj[30];
  for (int32_t v = 0; v < n; ++v) {
    adj[v] = 0;
    for (int32_t i = rp[v]; i < rp[v + 1]; ++i) adj[v] |= 1u << col[i];
  }
  if (pv)
    for (int32_t v = 0; v < n; ++v) pv[v] = 0;
  *count = 0;
  if (k > n) return ORC_OK;
  /* walk all k-subsets of {0..n-1} as bit masks in increasing order */
  uint64_t s = (k == 0) ? 0 : ((uint64_t)1 << k) - 1;
  uint64_t limit = (uint64_t)1 << n;
  while (s < limit) {
    int ok = 1;
    for (int32_t v = 0; v < n && ok; ++v)
      if ((s >> v) & 1) {
        uint32_t others = (uint32_t)s & ~(1u << v);
        if ((others & adj[v]) != others) ok = 0;
      }
    if (ok) {
      (*count)++;
      if (pv)
        for (int32_t v = 0; v < n; ++v)
          if ((s >> v) & 1) pv[v]++;
    }
    /* next subset of the same size (Gosper) */
    uint64_t c = s & (~s + 1), r = s + c;
    s = (((r ^ s) >> 2) / c) | r;
  }
  return ORC_OK;
}

/* ------------------------------------------ O1: ordered recursion by id */
typedef struct {
  const int32_t* rp;
  const int32_t* col;
  uint64_t* pv;
  int32_t* R;      /* chosen vertices, R[0..depth) */
  int32_t* buf;    /* candidate lists, one block per depth */
  int32_t stride;  /* block size (max degree + 1) */
  uint64_t budget; /* max intersections (0 = unlimited) */
  uint64_t isects;
  double deadline; /* CLOCK_MONOTONIC seconds (0 = none) */
  int status;
} idrec_t;

static double mono_now(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* out = {w in N(v) : w > v} intersected with cand[0..len); returns |out| */
static int32_t isect_up(const idrec_t* S, int32_t v, const int32_t* cand, int32_t len, int32_t* out) {
  int32_t a = S->rp[v], ae = S->rp[v + 1], b = 0, o = 0;
  while (a < ae && S->col[a] <= v) a++;
  while (a < ae && b < len) {
    int32_t x = S->col[a], y = cand[b];
    if (x == y) { out[o++] = x; a++; b++; }
    else if (x < y) a++;
    else b++;
  }
  return o;
}

/* Counts cliques R + (l vertices from cand) whose vertices ascend by id. */
static uint64_t idrec(idrec_t* S, int32_t l, const int32_t* cand, int32_t len, int32_t depth) {
  if (S->status) return 0;
  if (l == 0) {
    if (S->pv)
      for (int32_t i = 0; i < depth; ++i) S->pv[S->R[i]]++;
    return 1;
  }
  if (l == 1) {
    if (S->pv) {
      for (int32_t i = 0; i < depth; ++i) S->pv[S->R[i]] += (uint64_t)len;
      for (int32_t i = 0; i < len; ++i) S->pv[cand[i]]++;
    }
    return (uint64_t)len;
  }
  uint64_t total = 0;
  int32_t* next = S->buf + (size_t)(depth + 1) * (size_t)S->stride;
  for (int32_t i = 0; i < len; ++i) {
    int32_t v = cand[i];
    S->isects++;
    if (S->budget && S->isects > S->budget) { S->status = ORC_EBUDGET; return 0; }
    if (S->deadline > 0.0 && (S->isects & 0xffff) == 0 && mono_now() > S->deadline) {
      S->status = ORC_EBUDGET;
      return total;
    }
    int32_t m = isect_up(S, v, cand + i + 1, len - i - 1, next);
    if (m < l - 1) continue;
    S->R[depth] = v;
    uint64_t sub = idrec(S, l - 1, next, m, depth + 1);
    if (add_checked(&total, sub)) { S->status = ORC_EOVERFLOW; return 0; }
  }
  return total;
}

static int32_t max_degree(int32_t n, const int32_t* rp) {
  int32_t d = 0;
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] - rp[v] > d) d = rp[v + 1] - rp[v];
  return d;
}

/* Counts over roots in roots[0..nroots) (NULL: all vertices).  Cliques are
 * attributed to their smallest vertex id.  With a deadline, the count covers
 * only the cliques found before it expired and the status is ORC_EBUDGET;
 * *roots_done reports how many roots were completed. */
int orc_count_idorder_roots(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, const int32_t* roots,
                            int32_t nroots, double seconds, uint64_t* count, uint64_t* pv, int32_t* roots_done) {
  if (n < 0 || k < 1) return ORC_EINVAL;
  if (pv)
    for (int32_t v = 0; v < n; ++v) pv[v] = 0;
  *count = 0;
  if (roots_done) *roots_done = 0;
  if (n == 0) return ORC_OK;
  idrec_t S;
  memset(&S, 0, sizeof(S));
  S.rp = rp;
  S.col = col;
  S.pv = pv;
  S.stride = max_degree(n, rp) + 1;
  S.R = (int32_t*)malloc(sizeof(int32_t) * ((size_t)k + 1));
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 2));
  if (!S.R || !S.buf) { free(S.R); free(S.buf); return ORC_ENOMEM; }
  S.deadline = seconds > 0.0 ? mono_now() + seconds : 0.0;
  int32_t total_roots = roots ? nroots : n;
  for (int32_t t = 0; t < total_roots && !S.status; ++t) {
    int32_t u = roots ? roots[t] : t;
    /* candidates: neighbours with larger id */
    int32_t m = 0;
    for (int32_t i = rp[u]; i < rp[u + 1]; ++i)
      if (col[i] > u) S.buf[m++] = col[i];
    S.R[0] = u;
    uint64_t sub = idrec(&S, k - 1, S.buf, m, 1);
    if (add_checked(count, sub)) S.status = ORC_EOVERFLOW;
    if (!S.status && roots_done) (*roots_done)++;
  }
  free(S.R);
  free(S.buf);
  return S.status;
}

int orc_count_idorder(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, uint64_t* count, uint64_t* pv) {
  return orc_count_idorder_roots(n, rp, col, k, NULL, 0, 0.0, count, pv, NULL);
}

/* Listing (Sec. 3.1): every k-clique as its k vertex ids in ascending order,
 * by the same ordered recursion (each clique reached once, from its smallest
 * id, then in ascending id order).  Rows go to out[cap][k] in the order the
 * recursion meets them; *written receives min(count, cap), *count the total. */
typedef struct {
  const int32_t* rp;
  const int32_t* col;
  int32_t k;
  int32_t* R;
  int32_t* buf;
  int32_t stride;
  int32_t* out;
  int64_t cap, rows;
} idlist_t;

static void idlist(idlist_t* S, int32_t l, const int32_t* cand, int32_t len, int32_t depth) {
  if (l == 0) {
    if (S->rows < S->cap)
      for (int32_t i = 0; i < S->k; ++i) S->out[S->rows * S->k + i] = S->R[i];
    S->rows++;
    return;
  }
  int32_t* next = S->buf + (size_t)(depth + 1) * (size_t)S->stride;
  for (int32_t i = 0; i < len; ++i) {
    int32_t v = cand[i];
    /* next = {w in N(v) : w > v} intersected with cand[i+1..len) */
    int32_t a = S->rp[v], ae = S->rp[v + 1], b = i + 1, m = 0;
    while (a < ae && S->col[a] <= v) a++;
    while (a < ae && b < len) {
      int32_t x = S->col[a], y = cand[b];
      if (x == y) { next[m++] = x; a++; b++; }
      else if (x < y) a++;
      else b++;
    }
    if (m < l - 1) continue;
    S->R[depth] = v;
    idlist(S, l - 1, next, m, depth + 1);
  }
}

int orc_list_idorder(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, int32_t* out, int64_t cap,
                     int64_t* written, uint64_t* count) {
  if (n < 0 || k < 1 || cap < 0) return ORC_EINVAL;
  *written = 0;
  *count = 0;
  if (n == 0) return ORC_OK;
  idlist_t S;
  memset(&S, 0, sizeof(S));
  S.rp = rp;
  S.col = col;
  S.k = k;
  S.out = out;
  S.cap = cap;
  S.stride = max_degree(n, rp) + 1;
  S.R = (int32_t*)malloc(sizeof(int32_t) * ((size_t)k + 1));
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 2));
  if (!S.R || !S.buf) { free(S.R); free(S.buf); return ORC_ENOMEM; }
  for (int32_t u = 0; u < n; ++u) {
    int32_t m = 0;
    for (int32_t i = rp[u]; i < rp[u + 1]; ++i)
      if (col[i] > u) S.buf[m++] = col[i];
    S.R[0] = u;
    if (k == 1) {
      if (S.rows < S.cap) S.out[S.rows * k] = u;
      S.rows++;
      continue;
    }
    idlist(&S, k - 1, S.buf, m, 1);
  }
  free(S.R);
  free(S.buf);
  *count = (uint64_t)S.rows;
  *written = S.rows < cap ? S.rows : cap;
  return ORC_OK;
}

/* Participation of vertex v: (k-1)-cliques inside G[N(v)].  `budget` caps the
 * number of intersections (0 = unlimited); ORC_EBUDGET when exceeded. */
int orc_vertex_count(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, int32_t v, uint64_t budget,
                     uint64_t* out) {
  if (n < 0 || k < 1 || v < 0 || v >= n) return ORC_EINVAL;
  *out = 0;
  if (k == 1) { *out = 1; return ORC_OK; }
  idrec_t S;
  memset(&S, 0, sizeof(S));
  S.rp = rp;
  S.col = col;
  S.budget = budget;
  S.stride = max_degree(n, rp) + 1;
  S.R = (int32_t*)malloc(sizeof(int32_t) * ((size_t)k + 2));
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 3));
  if (!S.R || !S.buf) { free(S.R); free(S.buf); return ORC_ENOMEM; }
  int32_t m = rp[v + 1] - rp[v];
  memcpy(S.buf, col + rp[v], sizeof(int32_t) * (size_t)m);
  /* (k-1)-cliques of G[N(v)]: the ordered recursion restricted to N(v) */
  uint64_t total = idrec(&S, k - 1, S.buf, m, 0);
  int st = S.status;
  free(S.R);
  free(S.buf);
  if (st) return st;
  *out = total;
  return ORC_OK;
}

/* ------------------------------------------------------- core numbers */
int orc_core_numbers(int32_t n, const int32_t* rp, const int32_t* col, int32_t* core) {
  if (n < 0) return ORC_EINVAL;
  if (n == 0) return ORC_OK;
  int32_t md = max_degree(n, rp);
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* bin = (int32_t*)calloc((size_t)md + 2, sizeof(int32_t));
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!deg || !bin || !pos || !vert) { free(deg); free(bin); free(pos); free(vert); return ORC_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) { deg[v] = rp[v + 1] - rp[v]; bin[deg[v]]++; }
  int32_t start = 0;
  for (int32_t d = 0; d <= md; ++d) { int32_t c = bin[d]; bin[d] = start; start += c; }
  for (int32_t v = 0; v < n; ++v) { pos[v] = bin[deg[v]]; vert[pos[v]] = v; bin[deg[v]]++; }
  for (int32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t v = vert[i];
    for (int32_t j = rp[v]; j < rp[v + 1]; ++j) {
      int32_t u = col[j];
      if (deg[u] > deg[v]) {
        int32_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) { pos[u] = pw; vert[pu] = w; pos[w] = pu; vert[pw] = u; }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  memcpy(core, deg, sizeof(int32_t) * (size_t)n);
  free(deg); free(bin); free(pos); free(vert);
  return ORC_OK;
}

/* ------------------------------------------------------------ Pre-Core */
/* removed[v] = 1 for every vertex Alg. 3 eliminates (degree < k-1 cascade). */
int orc_precore(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, uint8_t* removed) {
  if (n < 0 || k < 1) return ORC_EINVAL;
  if (n == 0) return ORC_OK;
  int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* Q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!d || !Q) { free(d); free(Q); return ORC_ENOMEM; }
  int32_t head = 0, tail = 0;
  for (int32_t u = 0; u < n; ++u) {
    d[u] = rp[u + 1] - rp[u];
    removed[u] = 0;
    if (d[u] < k - 1) { Q[tail++] = u; removed[u] = 1; }
  }
  while (head < tail) {
    int32_t u = Q[head++];
    for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
      int32_t v = col[i];
      d[v]--;
      if (d[v] < k - 1 && !removed[v]) { removed[v] = 1; Q[tail++] = v; }
    }
  }
  free(d);
  free(Q);
  return ORC_OK;
}

/* ------------------------------------------------------------ Pre-List */
/* On the graph without `removed` vertices: every connected component whose
 * degree sum is n_c(n_c-1) is a clique; its C(n_c,k) cliques are added to
 * *count, C(n_c-1,k-1) to pv of each member (if pv), and it is marked in
 * removed.  *n_cliques_out receives the number of such components. */
int orc_prelist(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, uint8_t* removed, uint64_t* count,
                uint64_t* pv, int32_t* n_clique_comps) {
  if (n < 0 || k < 1) return ORC_EINVAL;
  *count = 0;
  if (n_clique_comps) *n_clique_comps = 0;
  if (n == 0) return ORC_OK;
  int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* Q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!comp || !Q) { free(comp); free(Q); return ORC_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) comp[v] = -1;
  int st = ORC_OK;
  for (int32_t s = 0; s < n && !st; ++s) {
    if (removed[s] || comp[s] >= 0) continue;
    /* BFS */
    int32_t head = 0, tail = 0;
    Q[tail++] = s;
    comp[s] = s;
    int64_t degsum = 0;
    while (head < tail) {
      int32_t u = Q[head++];
      for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
        int32_t v = col[i];
        if (removed[v]) continue;
        degsum++;
        if (comp[v] < 0) { comp[v] = s; Q[tail++] = v; }
      }
    }
    int64_t nc = tail;
    if (degsum == nc * (nc - 1)) {
      uint64_t c, cv = 0;
      if (orc_binom((uint64_t)nc, (uint64_t)k, &c)) { st = ORC_EOVERFLOW; break; }
      if (pv && orc_binom((uint64_t)nc - 1, (uint64_t)k - 1, &cv)) { st = ORC_EOVERFLOW; break; }
      if (add_checked(count, c)) { st = ORC_EOVERFLOW; break; }
      for (int32_t i = 0; i < tail; ++i) {
        removed[Q[i]] = 1;
        if (pv) pv[Q[i]] += cv;
      }
      if (n_clique_comps) (*n_clique_comps)++;
    }
  }
  free(comp);
  free(Q);
  return st;
}

/* -------------------------------------------------------- orientations */
/* Builds the out-neighbour lists of the live graph (removed[v] == 0) under a
 * total order given by key[] (ties by id): u -> v iff (key_u,u) < (key_v,v).
 * out_rp[n+1], out_col[<= nnz/2]; lists keep ascending id order. */
static void build_dag(int32_t n, const int32_t* rp, const int32_t* col, const uint8_t* removed, const int64_t* key,
                      int32_t* out_rp, int32_t* out_col) {
  int32_t o = 0;
  for (int32_t u = 0; u < n; ++u) {
    out_rp[u] = o;
    if (removed[u]) continue;
    for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
      int32_t v = col[i];
      if (removed[v]) continue;
      if (key[u] < key[v] || (key[u] == key[v] && u < v)) out_col[o++] = v;
    }
  }
  out_rp[n] = o;
}

int orc_degree_dag(int32_t n, const int32_t* rp, const int32_t* col, const uint8_t* removed, int32_t* out_rp,
                   int32_t* out_col) {
  if (n < 0) return ORC_EINVAL;
  int64_t* key = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!key) return ORC_ENOMEM;
  for (int32_t u = 0; u < n; ++u) {
    int64_t d = 0;
    if (!removed[u])
      for (int32_t i = rp[u]; i < rp[u + 1]; ++i) d += !removed[col[i]];
    key[u] = d;
  }
  build_dag(n, rp, col, removed, key, out_rp, out_col);
  free(key);
  return ORC_OK;
}

/* Synchronous peel; round[v] and core[v] for live vertices (-1 if removed). */
int orc_degeneracy_dag(int32_t n, const int32_t* rp, const int32_t* col, const uint8_t* removed, int32_t* out_rp,
                       int32_t* out_col, int32_t* round_out, int32_t* core_out) {
  if (n < 0) return ORC_EINVAL;
  int64_t* key = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t* d = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  uint8_t* alive = (uint8_t*)malloc((size_t)n + 1);
  int32_t* F = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!key || !d || !alive || !F) { free(key); free(d); free(alive); free(F); return ORC_ENOMEM; }
  int32_t live = 0;
  for (int32_t u = 0; u < n; ++u) {
    alive[u] = !removed[u];
    d[u] = 0;
    key[u] = -1;
    if (core_out) core_out[u] = -1;
    if (!alive[u]) continue;
    live++;
    for (int32_t i = rp[u]; i < rp[u + 1]; ++i) d[u] += !removed[col[i]];
  }
  int32_t c = 0, round = 0;
  while (live > 0) {
    int32_t f = 0;
    for (int32_t u = 0; u < n; ++u)
      if (alive[u] && d[u] <= c) F[f++] = u;
    if (f == 0) { c++; continue; }
    for (int32_t i = 0; i < f; ++i) {
      int32_t u = F[i];
      key[u] = round;
      if (core_out) core_out[u] = c;
      alive[u] = 0;
    }
    for (int32_t i = 0; i < f; ++i) {
      int32_t u = F[i];
      for (int32_t j = rp[u]; j < rp[u + 1]; ++j)
        if (alive[col[j]]) d[col[j]]--;
    }
    live -= f;
    round++;
  }
  build_dag(n, rp, col, removed, key, out_rp, out_col);
  if (round_out)
    for (int32_t u = 0; u < n; ++u) round_out[u] = (int32_t)key[u];
  free(key); free(d); free(alive); free(F);
  return ORC_OK;
}

/* ------------------------------------------------------ SDegree, Alg. 5 */
typedef struct {
  const int32_t* drp; /* DAG */
  const int32_t* dcol;
  int32_t stride;
  int32_t* buf;
  uint64_t count, nodes, isect, elems;
  int status;
  int noprune; /* ablation: no d+ <= l-2 skip, recurse into any non-empty C' */
  double deadline; /* CLOCK_MONOTONIC seconds (0 = none) */
} sdeg_t;

static int32_t merge_join(const int32_t* a, int32_t na, const int32_t* b, int32_t nb, int32_t* out) {
  int32_t i = 0, j = 0, o = 0;
  while (i < na && j < nb) {
    if (a[i] == b[j]) { out[o++] = a[i]; i++; j++; }
    else if (a[i] < b[j]) i++;
    else j++;
  }
  return o;
}

/* exported for the worked-example test of the merge join (Sec. 6.3) */
int32_t orc_merge_join(const int32_t* a, int32_t na, const int32_t* b, int32_t nb, int32_t* out) {
  return merge_join(a, na, b, nb, out);
}

static void sdegree_list(sdeg_t* S, int32_t l, const int32_t* C, int32_t nc, int32_t depth) {
  S->nodes++;
  int32_t* next = S->buf + (size_t)(depth + 1) * (size_t)S->stride;
  for (int32_t i = 0; i < nc && !S->status; ++i) {
    int32_t u = C[i];
    int32_t du = S->drp[u + 1] - S->drp[u];
    if (!S->noprune && du <= l - 2) continue;
    int32_t m = merge_join(S->dcol + S->drp[u], du, C, nc, next);
    S->isect++;
    S->elems += (uint64_t)nc + (uint64_t)du;
    if (S->deadline > 0.0 && (S->isect & 0xffff) == 0 && mono_now() > S->deadline) {
      S->status = ORC_EBUDGET;
      return;
    }
    if (l == 2) {
      if (add_checked(&S->count, (uint64_t)m)) S->status = ORC_EOVERFLOW;
    } else if (S->noprune ? m > 0 : m > l - 2) {
      sdegree_list(S, l - 1, next, m, depth + 1);
    }
  }
}

/* SDegree from root u with the out-neighbour reduction of Sec. 7.2: the
 * recursion runs on the DAG G_u induced by N+(u), whose vertices are the
 * positions 0..s-1 of N+(u) and whose out-lists are L_i = N+(x_i) restricted
 * to N+(u) (x_i = N+(u)[i]).  Alg. 5 then runs unchanged on G_u from the top
 * call C = all of G_u: its joins are L_x with C, its pruning uses the
 * out-degree |L_x| in G_u, and Lemma 2's cost of a join is |C| + |L_x|. */
static int sdegree_reduced_root(sdeg_t* S, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t u) {
  const int32_t s = drp[u + 1] - drp[u];
  if (s < k - 1) return ORC_OK;
  const int32_t* ids = dcol + drp[u];
  size_t cap = 0;
  for (int32_t i = 0; i < s; ++i) {
    const int32_t d = drp[ids[i] + 1] - drp[ids[i]];
    cap += (size_t)(d < s ? d : s);
  }
  int32_t* lrp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)s + 1));
  int32_t* lcol = (int32_t*)malloc(sizeof(int32_t) * (cap + 1));
  if (!lrp || !lcol) { free(lrp); free(lcol); return ORC_ENOMEM; }
  lrp[0] = 0;
  for (int32_t i = 0; i < s; ++i) {
    /* L_i: positions j with ids[j] in N+(x_i); both lists ascend by id */
    const int32_t x = ids[i];
    int32_t a = drp[x], ae = drp[x + 1], j = 0, o = lrp[i];
    while (a < ae && j < s) {
      if (dcol[a] == ids[j]) { lcol[o++] = j; a++; j++; }
      else if (dcol[a] < ids[j]) a++;
      else j++;
    }
    lrp[i + 1] = o;
  }
  const int32_t* save_rp = S->drp;
  const int32_t* save_col = S->dcol;
  S->drp = lrp;
  S->dcol = lcol;
  for (int32_t i = 0; i < s; ++i) S->buf[i] = i;
  sdegree_list(S, k - 1, S->buf, s, 0);
  S->drp = save_rp;
  S->dcol = save_col;
  free(lrp);
  free(lcol);
  return ORC_OK;
}

/* SDegree on a DAG.  Per root u (index = vertex id) the arrays receive the
 * cliques found from u and the work counters (any may be NULL).  k >= 3. */
static int sdegree_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int noprune, int reduce,
                       uint64_t* count, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                       uint64_t* root_elems);

int orc_sdegree_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, uint64_t* count,
                    uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect, uint64_t* root_elems) {
  return sdegree_dag(n, drp, dcol, k, 0, 0, count, root_count, root_nodes, root_isect, root_elems);
}

/* The same with the out-neighbour reduction (Sec. 7.2) on every root. */
int orc_sdegree_reduced_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, uint64_t* count,
                            uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect, uint64_t* root_elems) {
  return sdegree_dag(n, drp, dcol, k, 0, 1, count, root_count, root_nodes, root_isect, root_elems);
}

static int sdegree_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int noprune, int reduce,
                       uint64_t* count, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                       uint64_t* root_elems) {
  if (n < 0 || k < 3) return ORC_EINVAL;
  *count = 0;
  int32_t md = 0;
  for (int32_t u = 0; u < n; ++u)
    if (drp[u + 1] - drp[u] > md) md = drp[u + 1] - drp[u];
  sdeg_t S;
  memset(&S, 0, sizeof(S));
  S.drp = drp;
  S.dcol = dcol;
  S.noprune = noprune;
  S.stride = md + 1;
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 2));
  if (!S.buf) return ORC_ENOMEM;
  for (int32_t u = 0; u < n && !S.status; ++u) {
    int32_t du = drp[u + 1] - drp[u];
    uint64_t c0 = S.count, n0 = S.nodes, i0 = S.isect, e0 = S.elems;
    if (reduce) {
      const int st = sdegree_reduced_root(&S, drp, dcol, k, u);
      if (st) { free(S.buf); return st; }
    } else if (du >= k - 1) {
      memcpy(S.buf, dcol + drp[u], sizeof(int32_t) * (size_t)du);
      sdegree_list(&S, k - 1, S.buf, du, 0);
    }
    if (root_count) root_count[u] = S.count - c0;
    if (root_nodes) root_nodes[u] = S.nodes - n0;
    if (root_isect) root_isect[u] = S.isect - i0;
    if (root_elems) root_elems[u] = S.elems - e0;
  }
  free(S.buf);
  if (S.status) return S.status;
  *count = S.count;
  return ORC_OK;
}

/* The same for a list of roots only (sampled or sliced runs on large graphs):
 * entry i of each output describes roots[i]. */
static int sdegree_roots(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int reduce, int32_t nroots,
                         const int32_t* roots, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                         uint64_t* root_elems);

int orc_sdegree_roots(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t nroots,
                      const int32_t* roots, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                      uint64_t* root_elems) {
  return sdegree_roots(n, drp, dcol, k, 0, nroots, roots, root_count, root_nodes, root_isect, root_elems);
}

int orc_sdegree_reduced_roots(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t nroots,
                              const int32_t* roots, uint64_t* root_count, uint64_t* root_nodes,
                              uint64_t* root_isect, uint64_t* root_elems) {
  return sdegree_roots(n, drp, dcol, k, 1, nroots, roots, root_count, root_nodes, root_isect, root_elems);
}

static int sdegree_roots(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int reduce, int32_t nroots,
                         const int32_t* roots, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                         uint64_t* root_elems) {
  if (n < 0 || k < 3 || nroots < 0) return ORC_EINVAL;
  for (int32_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return ORC_EINVAL;
  int32_t md = 0;
  for (int32_t u = 0; u < n; ++u)
    if (drp[u + 1] - drp[u] > md) md = drp[u + 1] - drp[u];
  sdeg_t S;
  memset(&S, 0, sizeof(S));
  S.drp = drp;
  S.dcol = dcol;
  S.stride = md + 1;
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 2));
  if (!S.buf) return ORC_ENOMEM;
  for (int32_t i = 0; i < nroots && !S.status; ++i) {
    int32_t u = roots[i];
    int32_t du = drp[u + 1] - drp[u];
    uint64_t c0 = S.count, n0 = S.nodes, i0 = S.isect, e0 = S.elems;
    if (reduce) {
      const int st = sdegree_reduced_root(&S, drp, dcol, k, u);
      if (st) { free(S.buf); return st; }
    } else if (du >= k - 1) {
      memcpy(S.buf, dcol + drp[u], sizeof(int32_t) * (size_t)du);
      sdegree_list(&S, k - 1, S.buf, du, 0);
    }
    root_count[i] = S.count - c0;
    if (root_nodes) root_nodes[i] = S.nodes - n0;
    if (root_isect) root_isect[i] = S.isect - i0;
    if (root_elems) root_elems[i] = S.elems - e0;
  }
  free(S.buf);
  return S.status;
}

/* ----------------------------------------------------- greedy coloring */
/* Local graph on s vertices given by a dense 0/1 matrix adj[s*s] and their
 * global ids.  order_out[i] = local index colored i-th; color_out[v] >= 1. */
int orc_greedy_color(int32_t s, const uint8_t* adj, const int32_t* ids, int32_t* order_out, int32_t* color_out) {
  if (s < 0) return ORC_EINVAL;
  if (s == 0) return ORC_OK;
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)s);
  uint8_t* used = (uint8_t*)malloc((size_t)s + 2);
  if (!deg || !used) { free(deg); free(used); return ORC_ENOMEM; }
  for (int32_t v = 0; v < s; ++v) {
    deg[v] = 0;
    for (int32_t w = 0; w < s; ++w) deg[v] += adj[(size_t)v * s + w] ? 1 : 0;
    order_out[v] = v;
  }
  /* insertion sort: degree descending, then id ascending */
  for (int32_t i = 1; i < s; ++i) {
    int32_t x = order_out[i], j = i - 1;
    while (j >= 0) {
      int32_t y = order_out[j];
      int before = deg[x] > deg[y] || (deg[x] == deg[y] && ids[x] < ids[y]);
      if (!before) break;
      order_out[j + 1] = y;
      --j;
    }
    order_out[j + 1] = x;
  }
  for (int32_t v = 0; v < s; ++v) color_out[v] = 0;
  for (int32_t i = 0; i < s; ++i) {
    int32_t v = order_out[i];
    memset(used, 0, (size_t)s + 2);
    for (int32_t w = 0; w < s; ++w)
      if (adj[(size_t)v * s + w] && color_out[w] > 0 && color_out[w] <= s) used[color_out[w]] = 1;
    int32_t c = 1;
    while (used[c]) c++;
    color_out[v] = c;
  }
  free(deg);
  free(used);
  return ORC_OK;
}

/* ------------------------------------------------------- BitCol, Alg. 6 */
typedef struct {
  int32_t s, L, nw;      /* local size, bits per word, words per bitmap */
  const uint32_t* B;     /* s bitmaps of nw words */
  const int32_t* color;  /* per local vertex */
  uint32_t* stack;       /* candidate bitmaps, one per depth */
  uint64_t count, nodes, isect, words;
  int status;
  int noprune;           /* ablation: no color(v) < l skip */
  double deadline;       /* CLOCK_MONOTONIC seconds (0 = none) */
} bitcol_t;

static int32_t bits_set(const uint32_t* x, int32_t nw) {
  int32_t c = 0;
  for (int32_t i = 0; i < nw; ++i) c += __builtin_popcount(x[i]);
  return c;
}

static void bitcol_list(bitcol_t* S, int32_t l, const uint32_t* CB, int32_t depth) {
  S->nodes++;
  uint32_t* next = S->stack + (size_t)(depth + 1) * (size_t)S->nw;
  for (int32_t v = 0; v < S->s && !S->status; ++v) {
    /* decode: v is a member of CB */
    if (!((CB[v / S->L] >> (v % S->L)) & 1u)) continue;
    if (!S->noprune && S->color[v] < l) continue;
    const uint32_t* Bv = S->B + (size_t)v * S->nw;
    for (int32_t i = 0; i < S->nw; ++i) next[i] = Bv[i] & CB[i]; /* BitJoin */
    S->isect++;
    S->words += (uint64_t)((S->s + 31) / 32);
    if (S->deadline > 0.0 && (S->isect & 0xffff) == 0 && mono_now() > S->deadline) {
      S->status = ORC_EBUDGET;
      return;
    }
    int32_t p = bits_set(next, S->nw);
    if (l == 2) {
      if (add_checked(&S->count, (uint64_t)p)) S->status = ORC_EOVERFLOW;
    } else if (p >= l - 1) {
      bitcol_list(S, l - 1, next, depth + 1);
    }
  }
}

/* Encodes one local graph: colors and bitmaps B (s x ceil(s/L) words, L <= 32)
 * of the color-ordered DAG.  ids[] are the global ids (tie-break). */
int orc_bitcol_encode(int32_t s, const uint8_t* adj, const int32_t* ids, int32_t L, int32_t* color,
                      uint32_t* B) {
  if (s < 0 || L < 1 || L > 32) return ORC_EINVAL;
  if (s == 0) return ORC_OK;
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)s);
  if (!order) return ORC_ENOMEM;
  int st = orc_greedy_color(s, adj, ids, order, color);
  free(order);
  if (st) return st;
  int32_t nw = (s + L - 1) / L;
  memset(B, 0, sizeof(uint32_t) * (size_t)s * (size_t)nw);
  for (int32_t v = 0; v < s; ++v)
    for (int32_t w = 0; w < s; ++w)
      if (adj[(size_t)v * s + w] && color[w] < color[v]) B[(size_t)v * nw + w / L] |= 1u << (w % L);
  return ORC_OK;
}

/* Work space of the per-root BitCol evaluation. */
typedef struct {
  int32_t md, nwmax;
  uint8_t* adj;
  int32_t* ids;
  int32_t* color;
  uint32_t* B;
  uint32_t* stack;
  int32_t* pos;
} bitcol_ws_t;

static void bitcol_ws_free(bitcol_ws_t* w) {
  free(w->adj); free(w->ids); free(w->color); free(w->B); free(w->stack); free(w->pos);
}

static int bitcol_ws_init(bitcol_ws_t* w, int32_t n, const int32_t* drp, int32_t k, int32_t L) {
  memset(w, 0, sizeof(*w));
  for (int32_t u = 0; u < n; ++u)
    if (drp[u + 1] - drp[u] > w->md) w->md = drp[u + 1] - drp[u];
  w->nwmax = (w->md + L - 1) / L + 1;
  w->adj = (uint8_t*)malloc((size_t)w->md * (size_t)w->md + 1);
  w->ids = (int32_t*)malloc(sizeof(int32_t) * ((size_t)w->md + 1));
  w->color = (int32_t*)malloc(sizeof(int32_t) * ((size_t)w->md + 1));
  w->B = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)w->md + 1) * (size_t)w->nwmax);
  w->stack = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)w->nwmax * ((size_t)k + 2));
  w->pos = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!w->adj || !w->ids || !w->color || !w->B || !w->stack || !w->pos) {
    bitcol_ws_free(w);
    return ORC_ENOMEM;
  }
  for (int32_t v = 0; v < n; ++v) w->pos[v] = -1;
  return ORC_OK;
}

/* SDegree from roots[0..nroots) in that order until `seconds` have passed (a
 * timing sample), with the out-neighbour reduction when `reduce` is set;
 * outputs and status as orc_bitcol_roots_timed below. */
int orc_sdegree_roots_timed(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t reduce,
                            int32_t nroots, const int32_t* roots, double seconds, uint64_t* count,
                            int32_t* roots_done) {
  if (n < 0 || k < 3 || nroots < 0 || seconds <= 0.0) return ORC_EINVAL;
  for (int32_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return ORC_EINVAL;
  *count = 0;
  *roots_done = 0;
  int32_t md = 0;
  for (int32_t u = 0; u < n; ++u)
    if (drp[u + 1] - drp[u] > md) md = drp[u + 1] - drp[u];
  sdeg_t S;
  memset(&S, 0, sizeof(S));
  S.drp = drp;
  S.dcol = dcol;
  S.stride = md + 1;
  S.deadline = mono_now() + seconds;
  S.buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)S.stride * ((size_t)k + 2));
  if (!S.buf) return ORC_ENOMEM;
  for (int32_t i = 0; i < nroots && !S.status; ++i) {
    int32_t u = roots[i];
    int32_t du = drp[u + 1] - drp[u];
    if (reduce) {
      const int st = sdegree_reduced_root(&S, drp, dcol, k, u);
      if (st) { free(S.buf); return st; }
    } else if (du >= k - 1) {
      memcpy(S.buf, dcol + drp[u], sizeof(int32_t) * (size_t)du);
      sdegree_list(&S, k - 1, S.buf, du, 0);
    }
    if (!S.status) (*roots_done)++;
    if (!S.status && mono_now() > S.deadline) S.status = ORC_EBUDGET;
  }
  free(S.buf);
  *count = S.count;
  return S.status;
}

/* BitCol (Alg. 6) from one root u of the DAG: builds G_u from N+(u), colors
 * and encodes it, and runs the listing from the top call.  Adds to S's
 * counters; reports the number of colors and |E_u|. */
static int bitcol_root(bitcol_t* S, bitcol_ws_t* w, const int32_t* drp, const int32_t* dcol, int32_t k,
                       int32_t L, int32_t u, int32_t* ncolors_out, int64_t* edges_out) {
  int32_t s = drp[u + 1] - drp[u];
  *ncolors_out = 0;
  *edges_out = 0;
  if (s < k - 1) return ORC_OK;
  /* G_u: induced by N+(u), local index = position in N+(u) */
  for (int32_t i = 0; i < s; ++i) { w->ids[i] = dcol[drp[u] + i]; w->pos[w->ids[i]] = i; }
  memset(w->adj, 0, (size_t)s * (size_t)s);
  int64_t ecount = 0;
  for (int32_t i = 0; i < s; ++i) {
    int32_t v = w->ids[i];
    for (int32_t j = drp[v]; j < drp[v + 1]; ++j) {
      int32_t x = dcol[j];
      if (w->pos[x] >= 0) {
        w->adj[(size_t)i * s + w->pos[x]] = 1;
        w->adj[(size_t)w->pos[x] * s + i] = 1;
        ecount++;
      }
    }
  }
  for (int32_t i = 0; i < s; ++i) w->pos[w->ids[i]] = -1;
  int st = orc_bitcol_encode(s, w->adj, w->ids, L, w->color, w->B);
  if (st) return st;
  int32_t ncolors = 0;
  for (int32_t i = 0; i < s; ++i) ncolors = w->color[i] > ncolors ? w->color[i] : ncolors;
  S->L = L;
  S->stack = w->stack;
  S->s = s;
  S->nw = (s + L - 1) / L;
  S->B = w->B;
  S->color = w->color;
  /* top call: C_B = every local vertex (B_u(u)) */
  for (int32_t i = 0; i < S->nw; ++i) w->stack[i] = 0;
  for (int32_t i = 0; i < s; ++i) w->stack[i / L] |= 1u << (i % L);
  bitcol_list(S, k - 1, w->stack, 0);
  *ncolors_out = ncolors;
  *edges_out = ecount;
  return S->status;
}

/* BitCol on a DAG (normally the degeneracy DAG).  Per root u: cliques found,
 * work counters, and the features d+_u, number of colors of G_u, |E_u|. */
static int bitcol_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t L, int noprune,
                      uint64_t* count, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                      uint64_t* root_words, int32_t* root_colors, int64_t* root_edges);

int orc_bitcol_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t L, uint64_t* count,
                   uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect, uint64_t* root_words,
                   int32_t* root_colors, int64_t* root_edges) {
  return bitcol_dag(n, drp, dcol, k, L, 0, count, root_count, root_nodes, root_isect, root_words, root_colors,
                    root_edges);
}

static int bitcol_dag(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t L, int noprune,
                      uint64_t* count, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                      uint64_t* root_words, int32_t* root_colors, int64_t* root_edges) {
  if (n < 0 || k < 3 || L < 1 || L > 32) return ORC_EINVAL;
  *count = 0;
  bitcol_ws_t w;
  if (bitcol_ws_init(&w, n, drp, k, L)) return ORC_ENOMEM;
  bitcol_t S;
  memset(&S, 0, sizeof(S));
  S.noprune = noprune;
  int st = ORC_OK;
  for (int32_t u = 0; u < n && !st; ++u) {
    uint64_t c0 = S.count, n0 = S.nodes, i0 = S.isect, w0 = S.words;
    int32_t nc = 0;
    int64_t ec = 0;
    st = bitcol_root(&S, &w, drp, dcol, k, L, u, &nc, &ec);
    if (root_count) root_count[u] = S.count - c0;
    if (root_nodes) root_nodes[u] = S.nodes - n0;
    if (root_isect) root_isect[u] = S.isect - i0;
    if (root_words) root_words[u] = S.words - w0;
    if (root_colors) root_colors[u] = nc;
    if (root_edges) root_edges[u] = ec;
  }
  bitcol_ws_free(&w);
  if (st) return st;
  *count = S.count;
  return ORC_OK;
}

/* The same for a list of roots only (sampled checks on large graphs):
 * entry i of each output describes roots[i]. */
int orc_bitcol_roots(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t L, int32_t nroots,
                     const int32_t* roots, uint64_t* root_count, uint64_t* root_nodes, uint64_t* root_isect,
                     uint64_t* root_words) {
  if (n < 0 || k < 3 || L < 1 || L > 32 || nroots < 0) return ORC_EINVAL;
  for (int32_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return ORC_EINVAL;
  bitcol_ws_t w;
  if (bitcol_ws_init(&w, n, drp, k, L)) return ORC_ENOMEM;
  bitcol_t S;
  memset(&S, 0, sizeof(S));
  int st = ORC_OK;
  for (int32_t i = 0; i < nroots && !st; ++i) {
    uint64_t c0 = S.count, n0 = S.nodes, i0 = S.isect, w0 = S.words;
    int32_t nc = 0;
    int64_t ec = 0;
    st = bitcol_root(&S, &w, drp, dcol, k, L, roots[i], &nc, &ec);
    root_count[i] = S.count - c0;
    if (root_nodes) root_nodes[i] = S.nodes - n0;
    if (root_isect) root_isect[i] = S.isect - i0;
    if (root_words) root_words[i] = S.words - w0;
  }
  bitcol_ws_free(&w);
  return st;
}

/* BitCol from roots[0..nroots) in that order until `seconds` have passed (a
 * timing sample): *count receives the cliques found, including those of a
 * root cut short by the deadline, *roots_done the roots completed.  Returns
 * ORC_EBUDGET when the deadline cut the run short. */
int orc_bitcol_roots_timed(int32_t n, const int32_t* drp, const int32_t* dcol, int32_t k, int32_t L,
                           int32_t nroots, const int32_t* roots, double seconds, uint64_t* count,
                           int32_t* roots_done) {
  if (n < 0 || k < 3 || L < 1 || L > 32 || nroots < 0 || seconds <= 0.0) return ORC_EINVAL;
  for (int32_t i = 0; i < nroots; ++i)
    if (roots[i] < 0 || roots[i] >= n) return ORC_EINVAL;
  *count = 0;
  *roots_done = 0;
  bitcol_ws_t w;
  if (bitcol_ws_init(&w, n, drp, k, L)) return ORC_ENOMEM;
  bitcol_t S;
  memset(&S, 0, sizeof(S));
  S.deadline = mono_now() + seconds;
  int st = ORC_OK;
  for (int32_t i = 0; i < nroots && !st; ++i) {
    int32_t nc = 0;
    int64_t ec = 0;
    st = bitcol_root(&S, &w, drp, dcol, k, L, roots[i], &nc, &ec);
    if (!st) (*roots_done)++;
    if (!st && mono_now() > S.deadline) st = ORC_EBUDGET;
  }
  bitcol_ws_free(&w);
  *count = S.count;
  return st;
}

/* ------------------------------------------- whole methods (Alg. 5, 6) */
/* Pre-Core, Pre-List, orientation and listing, as the paper orders them.
 * method 0 = SDegree (degree DAG), 1 = BitCol (degeneracy DAG, L bits),
 * 2 = SDegree on the degeneracy DAG (Sec. 6.2: any vertex order), 3 and 4 =
 * methods 0 and 2 with the out-neighbour reduction (Sec. 7.2).
 * disable: ablation bits 1 = skip Pre-Core, 2 = skip Pre-List, 4 = no
 * pruning (SDegree: no d+ <= l-2 skip, children with any member entered;
 * BitCol: no color(v) < l skip).  Returns the total count (Pre-List cliques
 * included); the per-root arrays (size n, may be NULL) describe the listing
 * phase only. */
int orc_method_count(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, int32_t method, int32_t L,
                     int32_t disable, uint64_t* count, uint64_t* prelist_count, uint64_t* root_count,
                     uint64_t* root_nodes, uint64_t* root_isect, uint64_t* root_work, int32_t* root_dplus,
                     int32_t* root_core, int32_t* root_colors, int64_t* root_edges) {
  if (n < 0 || k < 3 || method < 0 || method > 4) return ORC_EINVAL;
  *count = 0;
  if (prelist_count) *prelist_count = 0;
  if (n == 0) return ORC_OK;
  uint8_t* removed = (uint8_t*)malloc((size_t)n);
  int32_t* drp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* dcol = (int32_t*)malloc(sizeof(int32_t) * ((size_t)rp[n] / 2 + 1));
  int32_t* core = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!removed || !drp || !dcol || !core) { free(removed); free(drp); free(dcol); free(core); return ORC_ENOMEM; }
  int st = ORC_OK;
  if (disable & 1) memset(removed, 0, (size_t)n);
  else st = orc_precore(n, rp, col, k, removed);
  uint64_t pl = 0;
  if (!st && !(disable & 2)) st = orc_prelist(n, rp, col, k, removed, &pl, NULL, NULL);
  if (!st) {
    if (method == 0 || method == 3) st = orc_degree_dag(n, rp, col, removed, drp, dcol);
    else st = orc_degeneracy_dag(n, rp, col, removed, drp, dcol, NULL, core);
  }
  uint64_t c = 0;
  const int noprune = (disable & 4) != 0;
  if (!st) {
    if (method == 1)
      st = bitcol_dag(n, drp, dcol, k, L, noprune, &c, root_count, root_nodes, root_isect, root_work, root_colors,
                      root_edges);
    else st = sdegree_dag(n, drp, dcol, k, noprune, method >= 3, &c, root_count, root_nodes, root_isect, root_work);
  }
  if (!st) {
    if (root_dplus)
      for (int32_t u = 0; u < n; ++u) root_dplus[u] = drp[u + 1] - drp[u];
    if (root_core && method != 0 && method != 3) memcpy(root_core, core, sizeof(int32_t) * (size_t)n);
    if (add_checked(&c, pl)) st = ORC_EOVERFLOW;
  }
  if (!st) {
    *count = c;
    if (prelist_count) *prelist_count = pl;
  }
  free(removed); free(drp); free(dcol); free(core);
  return st;
}
