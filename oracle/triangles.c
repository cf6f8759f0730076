/*
 * Textbook triangle count, used as an independent pin of the oracle on the
 * triangle query.  TEST INFRASTRUCTURE ONLY.
 *
 * The "forward" algorithm (Schank and Wagner, 2005; Latapy, 2008): rank the
 * vertices by (degree, id), orient every edge from lower to higher rank, and
 * for each oriented edge (v, w) count the common higher-ranked neighbours of v
 * and w by merging the two sorted out-lists.  Each triangle is counted exactly
 * once.  The number of triangle embeddings is six times this count.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const int64_t *orp;
  const int32_t *ocol;
  int64_t next;
  pthread_mutex_t mu;
} TriShared;

typedef struct {
  TriShared *s;
  uint64_t count;
} TriWorker;

static int ranks_above(const int64_t *rp, int32_t v, int32_t w) {
  int64_t dv = rp[v + 1] - rp[v], dw = rp[w + 1] - rp[w];
  return dw > dv || (dw == dv && w > v);
}

static void *tri_worker(void *arg) {
  TriWorker *t = (TriWorker *)arg;
  TriShared *s = t->s;
  const int64_t grain = 256;
  for (;;) {
    pthread_mutex_lock(&s->mu);
    int64_t b = s->next;
    s->next += grain;
    pthread_mutex_unlock(&s->mu);
    if (b >= s->n) break;
    int64_t e = b + grain < s->n ? b + grain : s->n;
    for (int64_t v = b; v < e; ++v) {
      for (int64_t k = s->orp[v]; k < s->orp[v + 1]; ++k) {
        int32_t w = s->ocol[k];
        int64_t i = s->orp[v], ie = s->orp[v + 1];
        int64_t j = s->orp[w], je = s->orp[w + 1];
        while (i < ie && j < je) {
          if (s->ocol[i] < s->ocol[j])
            ++i;
          else if (s->ocol[i] > s->ocol[j])
            ++j;
          else {
            t->count++;
            ++i;
            ++j;
          }
        }
      }
    }
  }
  return NULL;
}

/* Number of triangles (unordered vertex triples); -1 on allocation failure. */
int64_t oracle_triangles(int64_t n, const int64_t *rp, const int32_t *col, int32_t nthreads) {
  int64_t *orp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!orp) return -1;
  orp[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t c = 0;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) c += ranks_above(rp, (int32_t)v, col[e]);
    orp[v + 1] = orp[v] + c;
  }
  int32_t *ocol = (int32_t *)malloc((size_t)(orp[n] ? orp[n] : 1) * sizeof(int32_t));
  if (!ocol) {
    free(orp);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) {
    int64_t k = orp[v];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
      if (ranks_above(rp, (int32_t)v, col[e])) ocol[k++] = col[e];
  }
  TriShared s = {n, rp, col, orp, ocol, 0};
  pthread_mutex_init(&s.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  TriWorker *ws = (TriWorker *)calloc((size_t)nthreads, sizeof(TriWorker));
  pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
  for (int t = 0; t < nthreads; ++t) {
    ws[t].s = &s;
    pthread_create(&th[t], NULL, tri_worker, &ws[t]);
  }
  uint64_t total = 0;
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], NULL);
    total += ws[t].count;
  }
  pthread_mutex_destroy(&s.mu);
  free(ws);
  free(th);
  free(orp);
  free(ocol);
  return (int64_t)total;
}
