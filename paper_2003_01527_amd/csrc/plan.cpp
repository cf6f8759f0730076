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

}  // namespace gsm
