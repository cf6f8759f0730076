// Host pre-computation of the query (the paper's Alg. 1 PreCompute_on_CPUs,
// Sec. 3.2): visiting order, spanning-tree parents and non-tree edges, plus
// the query-side degree and neighbourhood encoding used by the filter.
#include <cstring>

#include "gsm_internal.h"

namespace gsm {

namespace {

// count(label l) * count(deg >= d): P_f scaled by n^2 (both factors share the
// denominator n), compared exactly in integers.
unsigned __int128 pf_scaled(const gsm_graph &g, int32_t l, int64_t d) {
  const int64_t lc = (l >= 0 && (size_t)l < g.label_count.size()) ? g.label_count[l] : 0;
  const int64_t dc = (d < (int64_t)g.deg_ge.size()) ? g.deg_ge[d] : 0;
  return (unsigned __int128)lc * (unsigned __int128)dc;
}

}  // namespace

Plan make_plan(const gsm_graph &g, const gsm_query &q) {
  Plan p;
  std::memset(&p, 0, sizeof(p));
  p.q = q.q;
  int64_t qdeg[kMaxQ];
  unsigned __int128 pf[kMaxQ];
  for (int u = 0; u < q.q; ++u) {
    qdeg[u] = __builtin_popcount(q.adj[u]);
    pf[u] = pf_scaled(g, q.label[u], qdeg[u]);
    uint64_t ne = 0;
    for (int w = 0; w < q.q; ++w)
      if ((q.adj[u] >> w) & 1) ne += (uint64_t)q.label[w] + 1;
    p.qdeg[u] = qdeg[u];
    p.qne[u] = ne;
    p.qlab[u] = q.label[u];
  }
  // Greedy order: larger d_M, then smaller P_f, then larger degree, then smaller id.
  int dM[kMaxQ] = {0};
  uint32_t taken = 0;
  for (int i = 0; i < q.q; ++i) {
    int best = -1;
    for (int u = 0; u < q.q; ++u) {
      if ((taken >> u) & 1) continue;
      if (best < 0) {
        best = u;
        continue;
      }
      bool better = false;
      if (dM[u] != dM[best])
        better = dM[u] > dM[best];
      else if (pf[u] != pf[best])
        better = pf[u] < pf[best];
      else if (qdeg[u] != qdeg[best])
        better = qdeg[u] > qdeg[best];
      if (better) best = u;  // equal on all three: the smaller id (scanned first) stays
    }
    p.order[i] = best;
    p.pos[best] = i;
    taken |= 1u << best;
    for (int w = 0; w < q.q; ++w)
      if (((q.adj[best] >> w) & 1) && !((taken >> w) & 1)) dM[w]++;
  }
  for (int i = 0; i < q.q; ++i) {
    const int u = p.order[i];
    uint32_t m = 0;
    for (int j = 0; j < i; ++j)
      if ((q.adj[u] >> p.order[j]) & 1) m |= 1u << j;
    p.backmask[i] = m;
    p.parent[i] = m ? __builtin_ctz(m) : -1;
  }
  return p;
}

namespace {

// Is there an automorphism of q that fixes every vertex of `fixed` and maps
// v to w?  Backtracking over vertices in id order; a vertex's image must keep
// its label and degree and the adjacency to every vertex placed before it.
bool find_automorphism(const gsm_query &q, uint32_t fixed, int v, int w) {
  int img[kMaxQ];
  uint32_t used = 0;
  for (int u = 0; u < q.q; ++u) img[u] = -1;
  for (int u = 0; u < q.q; ++u)
    if ((fixed >> u) & 1) {
      img[u] = u;
      used |= 1u << u;
    }
  if (img[v] >= 0 && img[v] != w) return false;
  if (img[v] < 0) {
    if ((used >> w) & 1) return false;
    img[v] = w;
    used |= 1u << w;
  }
  auto consistent = [&](int u, int x) {
    if (q.label[u] != q.label[x]) return false;
    if (__builtin_popcount(q.adj[u]) != __builtin_popcount(q.adj[x])) return false;
    for (int t = 0; t < q.q; ++t) {
      if (img[t] < 0 || t == u) continue;
      if (((q.adj[u] >> t) & 1) != ((q.adj[x] >> img[t]) & 1)) return false;
      if (q.has_elab && ((q.adj[u] >> t) & 1) && q.elab[u][t] != q.elab[x][img[t]]) return false;
    }
    return true;
  };
  // the pre-placed vertices must agree with each other
  for (int u = 0; u < q.q; ++u)
    if (img[u] >= 0 && !consistent(u, img[u])) return false;
  int order[kMaxQ], n = 0;
  for (int u = 0; u < q.q; ++u)
    if (img[u] < 0) order[n++] = u;
  // iterative backtracking: cand[d] is the next image to try at depth d
  int cand[kMaxQ];
  int d = 0;
  if (n == 0) return true;
  cand[0] = 0;
  while (d >= 0) {
    const int u = order[d];
    if (img[u] >= 0) {  // undo this depth's current choice
      used &= ~(1u << img[u]);
      img[u] = -1;
    }
    int x = cand[d];
    while (x < q.q && (((used >> x) & 1) || !consistent(u, x))) ++x;
    if (x == q.q) {
      --d;
      continue;
    }
    img[u] = x;
    used |= 1u << x;
    cand[d] = x + 1;
    if (d + 1 == n) return true;
    ++d;
    cand[d] = 0;
  }
  return false;
}

}  // namespace

// Symmetry breaking for the unique-subgraph mode (the paper visits equivalent
// query nodes in increasing id order so each combination is produced once,
// Sec. 3.3).  Stabilizer chain (Grochow and Kellis, RECOMB 2007): take the
// smallest vertex v whose orbit under the automorphisms fixing the vertices
// chosen so far has more than one vertex, require f(v) < f(w) for every other
// w of that orbit, fix v, repeat.  Exactly one embedding of every class
// {f o s : s in Aut(Q)} satisfies all constraints, and |Aut(Q)| is the
// product of the orbit sizes.
void compute_symmetry(gsm_query &q) {
  q.aut = 1;
  q.sym_pairs.clear();
  uint32_t fixed = 0;
  for (;;) {
    bool found = false;
    for (int v = 0; v < q.q && !found; ++v) {
      if ((fixed >> v) & 1) continue;
      int orbit[kMaxQ], m = 0;
      for (int w = 0; w < q.q; ++w)
        if (!((fixed >> w) & 1) && (w == v || find_automorphism(q, fixed, v, w))) orbit[m++] = w;
      if (m < 2) continue;
      for (int k = 0; k < m; ++k)
        if (orbit[k] != v) {
          q.sym_pairs.push_back(v);
          q.sym_pairs.push_back(orbit[k]);
        }
      q.aut *= (uint64_t)m;
      fixed |= 1u << v;
      found = true;
    }
    if (!found) break;
  }
}

}  // namespace gsm
