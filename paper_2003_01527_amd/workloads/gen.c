/*
 * Seeded synthetic workload generators for the subgraph matcher.
 *
 * This module holds no matching arithmetic.  It produces the inputs that both
 * the CPU oracle and the HIP path consume:
 *   - Erdos-Renyi G(n, m) graphs, uniform over vertex pairs;
 *   - R-MAT graphs (Graph500-style quadrant recursion, seeded vertex
 *     permutation, self-loops dropped, symmetrised, deduplicated);
 *   - vertex labels, uniform or Zipf(s);
 *   - query graphs drawn by random walk on the data graph (the label-scalability
 *     protocol the paper borrows from Yan et al., Sec. 4 "Scalability of
 *     query-graph size and label count"), either as the induced subgraph of the
 *     walk's vertices or as a fixed shape found among them;
 *   - a tractability bound for a query: the labelled homomorphism count of a
 *     BFS spanning tree of the query, which upper-bounds the embedding count;
 *   - Poisson arrival times.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, OOPSLA 2014) seeds
 * xoshiro256** (Blackman and Vigna, 2018).  No libc random or distribution
 * routines are used, so a seed gives the same workload on every machine.
 *
 * Graphs are returned as CSR: row_ptr (int64, n+1) and col (int32, row_ptr[n]),
 * simple, symmetric, with each row sorted ascending.  Arrays returned through
 * pointer-to-pointer arguments are malloc'd here and released with gen_free().
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- PRNG -- */

static inline uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t s[4];
} xo256;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xo256 *x, uint64_t seed) {
  uint64_t sm = seed;
  for (int i = 0; i < 4; ++i) x->s[i] = sm64_next(&sm);
}

static inline uint64_t xo_next(xo256 *x) {
  uint64_t *s = x->s;
  const uint64_t r = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return r;
}

/* uniform double in [0, 1) with 53 random bits */
static inline double xo_unit(xo256 *x) { return (double)(xo_next(x) >> 11) * 0x1.0p-53; }

/* integer in [0, n), by the multiply-shift map of a 64-bit draw */
static inline uint64_t xo_below(xo256 *x, uint64_t n) {
  return (uint64_t)(((unsigned __int128)xo_next(x) * n) >> 64);
}

/* the seed of sub-stream k of a master seed */
uint64_t gen_substream_seed(uint64_t master, uint64_t k) {
  uint64_t s = master * 0x100000001B3ULL + k;
  return sm64_next(&s);
}

void gen_free(void *p) { free(p); }

/* -------------------------------------------------- edge list -> CSR -- */

static void isort_i32(int32_t *a, int64_t n) {
  for (int64_t i = 1; i < n; ++i) {
    int32_t v = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > v) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = v;
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Builds a simple symmetric CSR from an undirected edge list: self-loops are
 * dropped, each edge is stored in both directions, rows are sorted and
 * duplicates removed.  Returns 2m (CSR entries) or -1 on allocation failure.
 */
static int64_t edges_to_csr(int64_t n, int64_t ne, const uint32_t *src, const uint32_t *dst,
                            int64_t **rp_out, int32_t **col_out) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
  for (int64_t e = 0; e < ne; ++e) {
    if (src[e] == dst[e]) continue;
    cnt[src[e] + 1]++;
    cnt[dst[e] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int64_t total = cnt[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  if (!tmp || !fill) {
    free(cnt);
    free(tmp);
    free(fill);
    return -1;
  }
  memcpy(fill, cnt, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < ne; ++e) {
    uint32_t u = src[e], v = dst[e];
    if (u == v) continue;
    tmp[fill[u]++] = (int32_t)v;
    tmp[fill[v]++] = (int32_t)u;
  }
  free(fill);
  /* sort and deduplicate each row, compacting in place */
  int64_t *rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!rp) {
    free(cnt);
    free(tmp);
    return -1;
  }
  int64_t w = 0;
  rp[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t b = cnt[v], e = cnt[v + 1], d = e - b;
    if (d <= 32)
      isort_i32(tmp + b, d);
    else
      qsort(tmp + b, (size_t)d, sizeof(int32_t), cmp_i32);
    int32_t last = -1;
    for (int64_t k = b; k < e; ++k) {
      if (tmp[k] != last) {
        tmp[w++] = tmp[k];
        last = tmp[k];
      }
    }
    rp[v + 1] = w;
  }
  free(cnt);
  int32_t *col = (int32_t *)realloc(tmp, (size_t)(w ? w : 1) * sizeof(int32_t));
  *rp_out = rp;
  *col_out = col ? col : tmp;
  return w;
}

/* ------------------------------------------------------- Erdos-Renyi -- */

/* G(n, m): m distinct unordered pairs drawn uniformly.  Returns 2m or -1. */
int64_t gen_er_csr(int64_t n, int64_t m, uint64_t seed, int64_t **rp_out, int32_t **col_out) {
  if (n < 2 || m < 0 || (double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
  uint64_t cap = 16;
  while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
  uint64_t *set = (uint64_t *)malloc(cap * sizeof(uint64_t));
  uint32_t *src = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
  uint32_t *dst = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
  if (!set || !src || !dst) {
    free(set);
    free(src);
    free(dst);
    return -1;
  }
  memset(set, 0xff, cap * sizeof(uint64_t));
  xo256 x;
  xo_seed(&x, seed);
  int64_t got = 0;
  while (got < m) {
    uint64_t a = xo_below(&x, (uint64_t)n), b = xo_below(&x, (uint64_t)n);
    if (a == b) continue;
    if (a > b) {
      uint64_t t = a;
      a = b;
      b = t;
    }
    uint64_t key = a * (uint64_t)n + b;
    uint64_t h = (key * 0x9E3779B97F4A7C15ULL) & (cap - 1);
    int fresh = 1;
    while (set[h] != ~0ULL) {
      if (set[h] == key) {
        fresh = 0;
        break;
      }
      h = (h + 1) & (cap - 1);
    }
    if (!fresh) continue;
    set[h] = key;
    src[got] = (uint32_t)a;
    dst[got] = (uint32_t)b;
    ++got;
  }
  free(set);
  int64_t r = edges_to_csr(n, m, src, dst, rp_out, col_out);
  free(src);
  free(dst);
  return r;
}

/* ------------------------------------------------------------- R-MAT -- */

/*
 * R-MAT with 2^scale vertices and round(ef * 2^scale) generated tuples.  Each
 * tuple picks one quadrant per bit with probabilities (a, b, c, 1-a-b-c); no
 * noise.  Vertex ids are then relabelled by a seeded random permutation, as in
 * Graph500's Kronecker generator.  Returns 2m or -1.
 */
int64_t gen_rmat_csr(int scale, double ef, double a, double b, double c, uint64_t seed,
                     int64_t **rp_out, int32_t **col_out) {
  if (scale < 1 || scale > 30) return -1;
  int64_t n = (int64_t)1 << scale;
  int64_t ne = (int64_t)llround(ef * (double)n);
  uint32_t *src = (uint32_t *)malloc((size_t)ne * sizeof(uint32_t));
  uint32_t *dst = (uint32_t *)malloc((size_t)ne * sizeof(uint32_t));
  uint32_t *perm = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!src || !dst || !perm) {
    free(src);
    free(dst);
    free(perm);
    return -1;
  }
  xo256 x;
  xo_seed(&x, seed);
  const uint64_t ta = (uint64_t)(a * 4294967296.0);
  const uint64_t tab = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tabc = (uint64_t)((a + b + c) * 4294967296.0);
  for (int64_t e = 0; e < ne; ++e) {
    uint32_t u = 0, v = 0;
    uint64_t r = 0;
    for (int bit = 0; bit < scale; ++bit) {
      if ((bit & 1) == 0) r = xo_next(&x);
      uint64_t d = (bit & 1) ? (r >> 32) : (r & 0xffffffffULL);
      uint32_t ub, vb;
      if (d < ta) {
        ub = 0;
        vb = 0;
      } else if (d < tab) {
        ub = 0;
        vb = 1;
      } else if (d < tabc) {
        ub = 1;
        vb = 0;
      } else {
        ub = 1;
        vb = 1;
      }
      u = (u << 1) | ub;
      v = (v << 1) | vb;
    }
    src[e] = u;
    dst[e] = v;
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  for (int64_t i = n - 1; i > 0; --i) { /* Fisher-Yates */
    int64_t j = (int64_t)xo_below(&x, (uint64_t)i + 1);
    uint32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  for (int64_t e = 0; e < ne; ++e) {
    src[e] = perm[src[e]];
    dst[e] = perm[dst[e]];
  }
  free(perm);
  int64_t r = edges_to_csr(n, ne, src, dst, rp_out, col_out);
  free(src);
  free(dst);
  return r;
}

/* ------------------------------------------------------------ labels -- */

void gen_labels_uniform(int64_t n, int32_t L, uint64_t seed, int32_t *out) {
  xo256 x;
  xo_seed(&x, seed);
  for (int64_t v = 0; v < n; ++v) out[v] = (int32_t)xo_below(&x, (uint64_t)L);
}

/* Zipf(s) over labels 0..L-1: P(k) proportional to 1/(k+1)^s. */
void gen_labels_zipf(int64_t n, int32_t L, double s, uint64_t seed, int32_t *out) {
  double *cdf = (double *)malloc((size_t)L * sizeof(double));
  double acc = 0.0;
  for (int k = 0; k < L; ++k) {
    acc += 1.0 / pow((double)(k + 1), s);
    cdf[k] = acc;
  }
  for (int k = 0; k < L; ++k) cdf[k] /= acc;
  cdf[L - 1] = 1.0;
  xo256 x;
  xo_seed(&x, seed);
  for (int64_t v = 0; v < n; ++v) {
    double u = xo_unit(&x);
    int lo = 0, hi = L - 1;
    while (lo < hi) {
      int mid = (lo + hi) / 2;
      if (u < cdf[mid])
        hi = mid;
      else
        lo = mid + 1;
    }
    out[v] = lo;
  }
  free(cdf);
}

/* ----------------------------------------------------------- queries -- */

static int adj(const int64_t *rp, const int32_t *col, int32_t a, int32_t b) {
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

/*
 * Random walk from a uniformly drawn non-isolated vertex until k distinct
 * vertices have been seen (or max_steps steps).  verts[] gets them in order of
 * first visit.  Returns the number of distinct vertices reached.
 */
static int walk(int64_t n, const int64_t *rp, const int32_t *col, int k, xo256 *x, int32_t *verts) {
  int32_t v;
  int tries = 0;
  do {
    v = (int32_t)xo_below(x, (uint64_t)n);
    if (++tries > 1000000) return 0;
  } while (rp[v + 1] == rp[v]);
  int got = 0;
  verts[got++] = v;
  const int max_steps = 64 * k + 64;
  for (int step = 0; step < max_steps && got < k; ++step) {
    int64_t d = rp[v + 1] - rp[v];
    v = col[rp[v] + (int64_t)xo_below(x, (uint64_t)d)];
    int seen = 0;
    for (int i = 0; i < got; ++i)
      if (verts[i] == v) seen = 1;
    if (!seen) verts[got++] = v;
  }
  return got;
}

/* ------------------------------------------- spanning-tree hom bound -- */

typedef struct {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const int32_t *lab; /* NULL = unlabelled */
  int32_t nlab;
  int64_t *cls_start; /* nlab+1 */
  int32_t *cls_vert;  /* vertices grouped by label */
  int32_t *cls_index; /* position of v inside its label class */
} LabelIndex;

static int build_label_index(LabelIndex *ix, int64_t n, const int64_t *rp, const int32_t *col,
                             const int32_t *lab) {
  ix->n = n;
  ix->rp = rp;
  ix->col = col;
  ix->lab = lab;
  int32_t L = 1;
  if (lab)
    for (int64_t v = 0; v < n; ++v)
      if (lab[v] + 1 > L) L = lab[v] + 1;
  ix->nlab = L;
  ix->cls_start = (int64_t *)calloc((size_t)L + 1, sizeof(int64_t));
  ix->cls_vert = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  ix->cls_index = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!ix->cls_start || !ix->cls_vert || !ix->cls_index) return -1;
  for (int64_t v = 0; v < n; ++v) ix->cls_start[(lab ? lab[v] : 0) + 1]++;
  for (int32_t l = 0; l < L; ++l) ix->cls_start[l + 1] += ix->cls_start[l];
  int64_t *fill = (int64_t *)malloc((size_t)L * sizeof(int64_t));
  memcpy(fill, ix->cls_start, (size_t)L * sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) {
    int32_t l = lab ? lab[v] : 0;
    ix->cls_index[v] = (int32_t)(fill[l] - ix->cls_start[l]);
    ix->cls_vert[fill[l]++] = (int32_t)v;
  }
  free(fill);
  return 0;
}

static void free_label_index(LabelIndex *ix) {
  free(ix->cls_start);
  free(ix->cls_vert);
  free(ix->cls_index);
}

/*
 * Number of label-preserving homomorphisms of a BFS spanning tree of the
 * query (rooted at query vertex 0) into G.  Every embedding of the query
 * restricts to one such homomorphism, so this bounds the embedding count.
 * h_u(v) = [l(v) = l(u)] * prod_{children c} sum_{w in N(v)} h_c(w), stored
 * only over the label class of l(u).  Returned as a double (may exceed 2^64).
 */
static double tree_hom_bound(const LabelIndex *ix, int q, int ne, const int32_t *qe,
                             const int32_t *ql) {
  int par[16], ord[16], nadj[16], adjq[16][16];
  memset(nadj, 0, sizeof(nadj));
  for (int e = 0; e < ne; ++e) {
    int a = qe[2 * e], b = qe[2 * e + 1];
    adjq[a][nadj[a]++] = b;
    adjq[b][nadj[b]++] = a;
  }
  int seen[16] = {0};
  int head = 0, tail = 0;
  ord[tail++] = 0;
  seen[0] = 1;
  par[0] = -1;
  while (head < tail) {
    int u = ord[head++];
    /* neighbours in ascending id */
    int tmp[16], m = nadj[u];
    memcpy(tmp, adjq[u], (size_t)m * sizeof(int));
    for (int i = 1; i < m; ++i)
      for (int j = i; j > 0 && tmp[j - 1] > tmp[j]; --j) {
        int t = tmp[j];
        tmp[j] = tmp[j - 1];
        tmp[j - 1] = t;
      }
    for (int i = 0; i < m; ++i)
      if (!seen[tmp[i]]) {
        seen[tmp[i]] = 1;
        par[tmp[i]] = u;
        ord[tail++] = tmp[i];
      }
  }
  if (tail != q) return INFINITY; /* disconnected */
  double *h[16];
  int ok = 1;
  for (int u = 0; u < q; ++u) {
    int32_t l = ql ? ql[u] : 0;
    int64_t sz = (l < ix->nlab) ? ix->cls_start[l + 1] - ix->cls_start[l] : 0;
    h[u] = (double *)malloc((size_t)(sz ? sz : 1) * sizeof(double));
    if (!h[u]) ok = 0;
  }
  double total = 0.0;
  if (ok) {
    for (int oi = q - 1; oi >= 0; --oi) {
      int u = ord[oi];
      int32_t l = ql ? ql[u] : 0;
      if (l >= ix->nlab) {
        total = 0.0;
        goto done;
      }
      int64_t cb = ix->cls_start[l], ce = ix->cls_start[l + 1];
      for (int64_t t = cb; t < ce; ++t) h[u][t - cb] = 1.0;
      for (int c = 0; c < q; ++c) {
        if (par[c] != u) continue;
        int32_t lc = ql ? ql[c] : 0;
        for (int64_t t = cb; t < ce; ++t) {
          int32_t v = ix->cls_vert[t];
          double s = 0.0;
          for (int64_t k = ix->rp[v]; k < ix->rp[v + 1]; ++k) {
            int32_t w = ix->col[k];
            if ((ix->lab ? ix->lab[w] : 0) == lc) s += h[c][ix->cls_index[w]];
          }
          h[u][t - cb] *= s;
        }
      }
    }
    int32_t l0 = ql ? ql[0] : 0;
    int64_t cb = ix->cls_start[l0], ce = ix->cls_start[l0 + 1];
    for (int64_t t = cb; t < ce; ++t) total += h[0][t - cb];
  }
done:
  for (int u = 0; u < q; ++u) free(h[u]);
  return ok ? total : INFINITY;
}

/* ------------------------------------------------- query set driver -- */

/* Fixed shapes for the small plain config (4 query vertices each). */
enum { SHAPE_INDUCED = 0, SHAPE_PAW = 1, SHAPE_P4 = 2, SHAPE_C4 = 3, SHAPE_STAR = 4 };

static int shape_edges(int shape, int32_t *e) {
  switch (shape) {
    case SHAPE_PAW: { /* triangle 0-1-2 plus pendant 3 on 0 */
      int32_t s[] = {0, 1, 1, 2, 0, 2, 0, 3};
      memcpy(e, s, sizeof(s));
      return 4;
    }
    case SHAPE_P4: {
      int32_t s[] = {0, 1, 1, 2, 2, 3};
      memcpy(e, s, sizeof(s));
      return 3;
    }
    case SHAPE_C4: {
      int32_t s[] = {0, 1, 1, 2, 2, 3, 0, 3};
      memcpy(e, s, sizeof(s));
      return 4;
    }
    case SHAPE_STAR: {
      int32_t s[] = {0, 1, 0, 2, 0, 3};
      memcpy(e, s, sizeof(s));
      return 3;
    }
  }
  return 0;
}

typedef struct {
  int32_t kind;      /* SHAPE_* */
  int32_t k_min, k_max;
  int32_t e_min, e_max;
  double dens_min, dens_max;
  double cap;        /* reject if the spanning-tree bound exceeds cap; <= 0: no cap */
} QueryParams;

typedef struct {
  int ok;
  int32_t q, ne;
  int32_t edges[2 * 120];
  int32_t labels[16];
  int32_t source[16];
  double bound;
} Candidate;

/* Draws candidate number idx of a query stream and decides acceptance. */
static void draw_candidate(const LabelIndex *ix, const QueryParams *p, uint64_t seed, uint64_t idx,
                           Candidate *out) {
  out->ok = 0;
  xo256 x;
  xo_seed(&x, gen_substream_seed(seed, idx));
  int k = p->k_min + (int)xo_below(&x, (uint64_t)(p->k_max - p->k_min + 1));
  if (k > 16) return;
  int32_t verts[16];
  if (walk(ix->n, ix->rp, ix->col, k, &x, verts) < k) return;
  if (p->kind == SHAPE_INDUCED) {
    int ne = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if (adj(ix->rp, ix->col, verts[i], verts[j])) {
          out->edges[2 * ne] = i;
          out->edges[2 * ne + 1] = j;
          ++ne;
        }
    if (ne < p->e_min || ne > p->e_max) return;
    double dens = (k > 1) ? (double)ne / (0.5 * k * (k - 1)) : 1.0;
    if (dens < p->dens_min || dens > p->dens_max) return;
    out->q = k;
    out->ne = ne;
    for (int i = 0; i < k; ++i) {
      out->source[i] = verts[i];
      out->labels[i] = ix->lab ? ix->lab[verts[i]] : 0;
    }
  } else {
    if (k != 4) return;
    int32_t se[8];
    int sne = shape_edges(p->kind, se);
    /* first permutation (lexicographic) mapping every shape edge onto G */
    int perm[4] = {0, 1, 2, 3}, found = 0;
    for (int it = 0; it < 24 && !found; ++it) {
      int good = 1;
      for (int e = 0; e < sne && good; ++e)
        good = adj(ix->rp, ix->col, verts[perm[se[2 * e]]], verts[perm[se[2 * e + 1]]]);
      if (good) {
        found = 1;
        break;
      }
      /* next permutation */
      int i = 2;
      while (i >= 0 && perm[i] > perm[i + 1]) --i;
      if (i < 0) break;
      int j = 3;
      while (perm[j] < perm[i]) --j;
      int t = perm[i];
      perm[i] = perm[j];
      perm[j] = t;
      for (int l = i + 1, r = 3; l < r; ++l, --r) {
        t = perm[l];
        perm[l] = perm[r];
        perm[r] = t;
      }
    }
    if (!found) return;
    out->q = 4;
    out->ne = sne;
    memcpy(out->edges, se, (size_t)sne * 2 * sizeof(int32_t));
    for (int s = 0; s < 4; ++s) {
      out->source[s] = verts[perm[s]];
      out->labels[s] = ix->lab ? ix->lab[verts[perm[s]]] : 0;
    }
  }
  out->bound = -1.0;
  if (p->cap > 0.0) {
    out->bound = tree_hom_bound(ix, out->q, out->ne, out->edges, out->labels);
    if (!(out->bound <= p->cap)) return;
  }
  out->ok = 1;
}

typedef struct {
  const LabelIndex *ix;
  const QueryParams *p;
  uint64_t seed;
  uint64_t base;
  int count;
  Candidate *cands;
  int next;
  pthread_mutex_t mu;
} Pool;

static void *pool_worker(void *arg) {
  Pool *pl = (Pool *)arg;
  for (;;) {
    pthread_mutex_lock(&pl->mu);
    int i = pl->next++;
    pthread_mutex_unlock(&pl->mu);
    if (i >= pl->count) break;
    draw_candidate(pl->ix, pl->p, pl->seed, pl->base + (uint64_t)i, &pl->cands[i]);
  }
  return NULL;
}

/*
 * Draws `want` accepted queries from the candidate stream of `seed`, in
 * candidate-index order (the result does not depend on nthreads).
 * Outputs, per accepted query j: q[j], ne[j], edges[j*240 ...], labels[j*16 ...],
 * source[j*16 ...], bound[j].  Returns the number of candidates examined, or
 * -1 if max_candidates were examined before `want` were accepted.
 */
int64_t gen_query_set(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab,
                      int32_t kind, int32_t k_min, int32_t k_max, int32_t e_min, int32_t e_max,
                      double dens_min, double dens_max, double cap, uint64_t seed, int32_t want,
                      int64_t max_candidates, int32_t nthreads, int32_t *q_out, int32_t *ne_out,
                      int32_t *edges_out, int32_t *labels_out, int32_t *source_out,
                      double *bound_out) {
  LabelIndex ix;
  if (build_label_index(&ix, n, rp, col, lab) != 0) return -1;
  QueryParams p = {kind, k_min, k_max, e_min, e_max, dens_min, dens_max, cap};
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  const int batch = 8 * nthreads;
  Candidate *cands = (Candidate *)malloc((size_t)batch * sizeof(Candidate));
  int32_t got = 0;
  uint64_t base = 0;
  while (got < want && (int64_t)base < max_candidates) {
    Pool pl;
    pl.ix = &ix;
    pl.p = &p;
    pl.seed = seed;
    pl.base = base;
    pl.count = batch;
    pl.cands = cands;
    pl.next = 0;
    pthread_mutex_init(&pl.mu, NULL);
    pthread_t th[64];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, pool_worker, &pl);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&pl.mu);
    for (int i = 0; i < batch && got < want; ++i) {
      if ((int64_t)(base + (uint64_t)i) >= max_candidates) break;
      Candidate *c = &cands[i];
      if (!c->ok) continue;
      q_out[got] = c->q;
      ne_out[got] = c->ne;
      memcpy(edges_out + (int64_t)got * 240, c->edges, (size_t)c->ne * 2 * sizeof(int32_t));
      memcpy(labels_out + (int64_t)got * 16, c->labels, (size_t)c->q * sizeof(int32_t));
      memcpy(source_out + (int64_t)got * 16, c->source, (size_t)c->q * sizeof(int32_t));
      bound_out[got] = c->bound;
      if (++got == want) {
        base += (uint64_t)i + 1;
        goto finished;
      }
    }
    base += (uint64_t)batch;
  }
finished:
  free(cands);
  free_label_index(&ix);
  return got == want ? (int64_t)base : -1;
}

/* Spanning-tree homomorphism bound of one query (see tree_hom_bound). */
double gen_tree_hom_bound(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab,
                          int32_t q, int32_t ne, const int32_t *edges, const int32_t *qlab) {
  LabelIndex ix;
  if (build_label_index(&ix, n, rp, col, lab) != 0) return -1.0;
  double b = tree_hom_bound(&ix, q, ne, edges, qlab);
  free_label_index(&ix);
  return b;
}

/* Poisson process: arrival times (seconds) with exponential gaps of mean 1/rate. */
void gen_poisson_arrivals(int64_t count, double rate, uint64_t seed, double *out) {
  xo256 x;
  xo_seed(&x, seed);
  double t = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    t += -log(1.0 - xo_unit(&x)) / rate;
    out[i] = t;
  }
}
