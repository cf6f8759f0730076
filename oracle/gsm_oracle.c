/*
 * CPU oracle for the subgraph matcher.  TEST INFRASTRUCTURE ONLY: tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the matching
 * library never does.  It shares no code with the HIP path.
 *
 * oracle_match — the result the paper's method produces (Sec. 3.2, Alg. 1:
 *   inputs a query Q and a data graph G, both undirected, labelled or not;
 *   outputs the number of matched subgraphs and their listing).  An embedding
 *   is an injective map f from the query vertices to data vertices that keeps
 *   vertex labels and maps every query edge onto a data edge (non-induced; the
 *   verification step only tests connections to already-matched vertices,
 *   Sec. 3.2, verification).  Every such map is counted, automorphic images
 *   included; rows are reported in query-vertex-id order.
 *   Method: plain depth-first backtracking (the tree-search family of Sec. 2),
 *   visiting query vertices in BFS order from vertex 0 with ascending neighbour
 *   ids; candidates for a vertex are the neighbours of its BFS parent's image;
 *   each candidate is tested for label, injectivity and every edge back to
 *   earlier query vertices.  No pruning, no candidate filter.
 *   Optional root slice: only maps with splitmix64(f(root)) mod M == R, where
 *   splitmix64 is the output of one step of Steele, Lea and Flood's generator
 *   from state x, i.e. the finaliser applied to x + 0x9E3779B97F4A7C15.
 *   Optional threads: root candidates are dealt out dynamically.
 *   Optional induced semantics (the other common reading of subgraph
 *   isomorphism, Sec. 1): non-adjacent query vertices must also map to
 *   non-adjacent data vertices; every earlier non-neighbour is tested too.
 *   Optional edge labels (the labelled graphs of Sec. 3.1 carry node and edge
 *   labels): every query edge {a, b} must map onto a data edge with the same
 *   label.  Graph edge labels are given per CSR entry (both directions of an
 *   edge carry its label; none given = every edge has label 0); query edge
 *   labels per query edge (none given = no edge-label constraint).
 *
 * oracle_filter — the candidate sets of the filtering stage (Sec. 3.2,
 *   filtering; Alg. 1 Filter_candidate_set): v is a candidate of query
 *   vertex u when labels are equal, deg(v) >= deg(u) and NE(v) >= NE(u), with
 *   the neighbourhood encoding NE(x) = sum over neighbours w of (label(w) + 1)
 *   (so an unlabelled graph gives NE = degree).  Each refinement round keeps
 *   only candidates whose degree and NE, recomputed over neighbours that are
 *   still a candidate of some query vertex, pass the same tests.
 *   Output: one uint16 per data vertex, bit u set when v is a candidate of u.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OQ_MAX 16

static uint64_t slice_hash(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t oracle_slice_hash(uint64_t x) { return slice_hash(x); }

/* CSR position of b in the row of a, or -1. */
static int64_t edge_pos(const int64_t *rp, const int32_t *col, int32_t a, int32_t b) {
  int64_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < rp[a + 1] && col[lo] == b) ? lo : -1;
}

static int has_edge(const int64_t *rp, const int32_t *col, int32_t a, int32_t b) {
  int64_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < rp[a + 1] && col[lo] == b;
}

typedef struct {
  int q;
  int order[OQ_MAX];      /* query vertex visited at depth k */
  int parent[OQ_MAX];     /* query vertex whose image's neighbours are scanned */
  int nback[OQ_MAX];      /* further earlier neighbours to test, per depth */
  int back[OQ_MAX][OQ_MAX];
  int nnon[OQ_MAX];       /* earlier non-neighbours, per depth (induced only) */
  int non[OQ_MAX][OQ_MAX];
  int32_t label[OQ_MAX];  /* label per query vertex (0 when unlabelled) */
  int has_elab;           /* query edge labels given */
  int32_t elab[OQ_MAX][OQ_MAX]; /* label of query edge {a, b} */
} OPlan;

/* BFS order from query vertex 0, neighbours in ascending id.  -1 if not connected. */
static int make_plan(int q, int ne, const int32_t *edges, const int32_t *qlab, const int32_t *qelab, OPlan *p) {
  int A[OQ_MAX][OQ_MAX];
  memset(A, 0, sizeof(A));
  p->has_elab = qelab != NULL;
  for (int e = 0; e < ne; ++e) {
    int a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || b < 0 || a >= q || b >= q || a == b) return -1;
    A[a][b] = A[b][a] = 1;
    if (qelab) p->elab[a][b] = p->elab[b][a] = qelab[e];
  }
  p->q = q;
  for (int u = 0; u < q; ++u) p->label[u] = qlab ? qlab[u] : 0;
  int depth_of[OQ_MAX];
  for (int u = 0; u < q; ++u) depth_of[u] = -1;
  int head = 0, tail = 0;
  p->order[tail] = 0;
  p->parent[tail] = -1;
  depth_of[0] = tail++;
  while (head < tail) {
    int u = p->order[head++];
    for (int w = 0; w < q; ++w)
      if (A[u][w] && depth_of[w] < 0) {
        p->order[tail] = w;
        p->parent[tail] = u;
        depth_of[w] = tail++;
      }
  }
  if (tail != q) return -1;
  for (int k = 0; k < q; ++k) {
    int u = p->order[k];
    p->nback[k] = 0;
    p->nnon[k] = 0;
    for (int j = 0; j < k; ++j) {
      int w = p->order[j];
      if (A[u][w] && w != p->parent[k]) p->back[k][p->nback[k]++] = w;
      if (!A[u][w]) p->non[k][p->nnon[k]++] = w;
    }
  }
  return 0;
}

typedef struct {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const int32_t *lab;
  const int32_t *elab;  /* per CSR entry, or NULL */
  const OPlan *p;
  int root_q;
  uint32_t root_mod, root_rem;
  int want_rows;
  int induced;
  /* shared root dispenser */
  int64_t next_root;
  pthread_mutex_t mu;
} Shared;

typedef struct {
  Shared *s;
  int32_t f[OQ_MAX];
  uint8_t *used;
  uint64_t count;
  int32_t *rows;
  uint64_t nrows, cap;
  int oom;
} Worker;

static void emit(Worker *w) {
  Shared *s = w->s;
  w->count++;
  if (!s->want_rows || w->oom) return;
  if (w->nrows == w->cap) {
    uint64_t nc = w->cap ? 2 * w->cap : 1024;
    int32_t *r = (int32_t *)realloc(w->rows, nc * (uint64_t)s->p->q * sizeof(int32_t));
    if (!r) {
      w->oom = 1;
      return;
    }
    w->rows = r;
    w->cap = nc;
  }
  memcpy(w->rows + w->nrows * (uint64_t)s->p->q, w->f, (size_t)s->p->q * sizeof(int32_t));
  w->nrows++;
}

/* Label of the data edge at CSR position e (0 when the graph has none). */
static int32_t data_elab(const Shared *s, int64_t e) { return s->elab ? s->elab[e] : 0; }

/* v for query vertex order[k]; e = CSR position of v in its parent image's
 * row (-1 at depth 0). */
static int admissible(Worker *w, int k, int32_t v, int64_t e) {
  Shared *s = w->s;
  const OPlan *p = s->p;
  int u = p->order[k];
  if ((s->lab ? s->lab[v] : 0) != p->label[u]) return 0;
  if (w->used[v]) return 0;
  if (u == s->root_q && s->root_mod > 0 && slice_hash((uint64_t)v) % s->root_mod != s->root_rem)
    return 0;
  if (p->has_elab && e >= 0 && data_elab(s, e) != p->elab[p->parent[k]][u]) return 0;
  for (int b = 0; b < p->nback[k]; ++b) {
    const int x = p->back[k][b];
    if (!p->has_elab) {
      if (!has_edge(s->rp, s->col, w->f[x], v)) return 0;
    } else {
      const int64_t pos = edge_pos(s->rp, s->col, w->f[x], v);
      if (pos < 0 || data_elab(s, pos) != p->elab[x][u]) return 0;
    }
  }
  if (s->induced)
    for (int b = 0; b < p->nnon[k]; ++b)
      if (has_edge(s->rp, s->col, w->f[p->non[k][b]], v)) return 0;
  return 1;
}

static void dfs(Worker *w, int k) {
  Shared *s = w->s;
  const OPlan *p = s->p;
  if (k == p->q) {
    emit(w);
    return;
  }
  int u = p->order[k];
  int32_t a = w->f[p->parent[k]];
  for (int64_t e = s->rp[a]; e < s->rp[a + 1]; ++e) {
    int32_t v = s->col[e];
    if (!admissible(w, k, v, e)) continue;
    w->f[u] = v;
    w->used[v] = 1;
    dfs(w, k + 1);
    w->used[v] = 0;
  }
}

static void *worker_main(void *arg) {
  Worker *w = (Worker *)arg;
  Shared *s = w->s;
  const OPlan *p = s->p;
  const int64_t grain = 64;
  for (;;) {
    pthread_mutex_lock(&s->mu);
    int64_t b = s->next_root;
    s->next_root += grain;
    pthread_mutex_unlock(&s->mu);
    if (b >= s->n) break;
    int64_t e = b + grain < s->n ? b + grain : s->n;
    for (int64_t v = b; v < e; ++v) {
      if (!admissible(w, 0, (int32_t)v, -1)) continue;
      w->f[p->order[0]] = (int32_t)v;
      w->used[v] = 1;
      dfs(w, 1);
      w->used[v] = 0;
    }
  }
  return NULL;
}

/*
 * Returns 0 on success, -1 for an invalid query, -2 when out of memory.
 * *count gets the number of embeddings.  When want_rows, *rows_out gets a
 * malloc'd array of count*q int32 (query-id columns, unsorted; release with
 * oracle_free).  nthreads <= 1 runs on the calling thread only.
 */
int oracle_match_el(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab,
                    const int32_t *elab, int32_t q, int32_t ne, const int32_t *edges, const int32_t *qlab,
                    const int32_t *qelab, int32_t root_q, uint32_t root_mod, uint32_t root_rem,
                    int32_t want_rows, int32_t nthreads, int32_t induced, uint64_t *count,
                    int32_t **rows_out) {
  OPlan p;
  if (q < 1 || q > OQ_MAX || make_plan(q, ne, edges, qlab, qelab, &p) != 0) return -1;
  Shared s;
  s.n = n;
  s.rp = rp;
  s.col = col;
  s.lab = lab;
  s.elab = elab;
  s.p = &p;
  s.root_q = root_q;
  s.root_mod = root_mod;
  s.root_rem = root_rem;
  s.want_rows = want_rows;
  s.induced = induced != 0;
  s.next_root = 0;
  pthread_mutex_init(&s.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  Worker *ws = (Worker *)calloc((size_t)nthreads, sizeof(Worker));
  if (!ws) return -2;
  int rc = 0;
  for (int t = 0; t < nthreads; ++t) {
    ws[t].s = &s;
    ws[t].used = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    if (!ws[t].used) rc = -2;
  }
  if (rc == 0) {
    if (nthreads == 1) {
      worker_main(&ws[0]);
    } else {
      pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
      for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker_main, &ws[t]);
      for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
      free(th);
    }
  }
  uint64_t total = 0, nrows = 0;
  for (int t = 0; t < nthreads; ++t) {
    total += ws[t].count;
    nrows += ws[t].nrows;
    if (ws[t].oom) rc = -2;
  }
  if (rc == 0 && want_rows) {
    int32_t *all = (int32_t *)malloc((size_t)(nrows ? nrows : 1) * (size_t)q * sizeof(int32_t));
    if (!all) {
      rc = -2;
    } else {
      uint64_t off = 0;
      for (int t = 0; t < nthreads; ++t) {
        memcpy(all + off * (uint64_t)q, ws[t].rows, (size_t)ws[t].nrows * (size_t)q * sizeof(int32_t));
        off += ws[t].nrows;
      }
      *rows_out = all;
    }
  }
  for (int t = 0; t < nthreads; ++t) {
    free(ws[t].used);
    free(ws[t].rows);
  }
  free(ws);
  pthread_mutex_destroy(&s.mu);
  if (rc == 0) *count = total;
  return rc;
}

/* oracle_match_el without edge labels. */
int oracle_match_ex(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab, int32_t q,
                    int32_t ne, const int32_t *edges, const int32_t *qlab, int32_t root_q,
                    uint32_t root_mod, uint32_t root_rem, int32_t want_rows, int32_t nthreads,
                    int32_t induced, uint64_t *count, int32_t **rows_out) {
  return oracle_match_el(n, rp, col, lab, NULL, q, ne, edges, qlab, NULL, root_q, root_mod, root_rem, want_rows,
                         nthreads, induced, count, rows_out);
}

/* oracle_match_ex with non-induced semantics. */
int oracle_match(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab, int32_t q,
                 int32_t ne, const int32_t *edges, const int32_t *qlab, int32_t root_q,
                 uint32_t root_mod, uint32_t root_rem, int32_t want_rows, int32_t nthreads,
                 uint64_t *count, int32_t **rows_out) {
  return oracle_match_ex(n, rp, col, lab, q, ne, edges, qlab, root_q, root_mod, root_rem, want_rows, nthreads, 0,
                         count, rows_out);
}

void oracle_free(void *p) { free(p); }

/* --------------------------------------------------------------- filter -- */

int oracle_filter(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab, int32_t q,
                  int32_t ne, const int32_t *edges, const int32_t *qlab, int32_t rounds,
                  int32_t use_deg, int32_t use_ne, int32_t root_q, uint32_t root_mod,
                  uint32_t root_rem, uint16_t *out) {
  if (q < 1 || q > OQ_MAX) return -1;
  /* query degree and NE */
  int64_t qdeg[OQ_MAX];
  uint64_t qne[OQ_MAX];
  int32_t ql[OQ_MAX];
  for (int u = 0; u < q; ++u) {
    qdeg[u] = 0;
    qne[u] = 0;
    ql[u] = qlab ? qlab[u] : 0;
  }
  for (int e = 0; e < ne; ++e) {
    int a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || b < 0 || a >= q || b >= q || a == b) return -1;
    qdeg[a]++;
    qdeg[b]++;
    qne[a] += (uint64_t)ql[b] + 1;
    qne[b] += (uint64_t)ql[a] + 1;
  }
  int64_t *deg = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  uint64_t *nev = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
  uint16_t *prev = (uint16_t *)malloc((size_t)(n ? n : 1) * sizeof(uint16_t));
  if (!deg || !nev || !prev) {
    free(deg);
    free(nev);
    free(prev);
    return -2;
  }
  /* round 0: all neighbours count */
  for (int64_t v = 0; v < n; ++v) {
    deg[v] = rp[v + 1] - rp[v];
    uint64_t s = 0;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += (uint64_t)(lab ? lab[col[e]] : 0) + 1;
    nev[v] = s;
  }
  for (int64_t v = 0; v < n; ++v) {
    uint16_t m = 0;
    int32_t lv = lab ? lab[v] : 0;
    for (int u = 0; u < q; ++u) {
      if (lv != ql[u]) continue;
      if (use_deg && deg[v] < qdeg[u]) continue;
      if (use_ne && nev[v] < qne[u]) continue;
      if (u == root_q && root_mod > 0 && slice_hash((uint64_t)v) % root_mod != root_rem) continue;
      m |= (uint16_t)(1u << u);
    }
    out[v] = m;
  }
  /* refinement rounds: degree and NE over neighbours still alive */
  for (int r = 0; r < rounds; ++r) {
    memcpy(prev, out, (size_t)n * sizeof(uint16_t));
    for (int64_t v = 0; v < n; ++v) {
      int64_t d = 0;
      uint64_t s = 0;
      for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
        int32_t w = col[e];
        if (prev[w] == 0) continue;
        d++;
        s += (uint64_t)(lab ? lab[w] : 0) + 1;
      }
      uint16_t m = 0;
      for (int u = 0; u < q; ++u) {
        if (!((prev[v] >> u) & 1)) continue;
        if (use_deg && d < qdeg[u]) continue;
        if (use_ne && s < qne[u]) continue;
        m |= (uint16_t)(1u << u);
      }
      out[v] = m;
    }
  }
  free(deg);
  free(nev);
  free(prev);
  return 0;
}
