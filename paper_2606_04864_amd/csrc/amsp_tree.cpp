// Sparse coarse factorisation, host symbolic phase: nested dissection of the
// subdomain graph, supernodes, front structure, and the index tables the
// numeric kernels read (see amsp_tree.h).  Integer work only.
#include "amsp_tree.h"

#include <algorithm>
#include <cstdint>
#include <functional>
#include <numeric>

namespace amsp {

namespace {

struct Graph {
  int n = 0;
  std::vector<int> ptr, adj;  // CSR without self loops
};

// BFS over the nodes of `in` (mark[v] == tag) from `src`; returns the level
// of every visited node in lev (others untouched) and the visit order.
int bfs(const Graph &g, const std::vector<int> &mark, int tag, int src, std::vector<int> &lev,
        std::vector<int> &order) {
  order.clear();
  order.push_back(src);
  lev[src] = 0;
  int maxl = 0;
  for (size_t h = 0; h < order.size(); ++h) {
    const int v = order[h];
    for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
      const int w = g.adj[e];
      if (mark[w] != tag || lev[w] >= 0) continue;
      lev[w] = lev[v] + 1;
      maxl = std::max(maxl, lev[w]);
      order.push_back(w);
    }
  }
  return maxl;
}

struct Builder {
  const Graph &g;
  const std::vector<int> &m;  // coarse dofs per node
  int leaf_dofs;
  std::vector<int> mark, lev;
  int tag = 0;
  // supernodes, in creation order (children before parents)
  std::vector<std::vector<int>> sn_nodes;
  std::vector<std::vector<int>> sn_children;

  Builder(const Graph &g_, const std::vector<int> &m_, int leaf)
      : g(g_), m(m_), leaf_dofs(leaf), mark(g_.n, -1), lev(g_.n, -1) {}

  int new_sn(std::vector<int> nodes, std::vector<int> children) {
    std::sort(nodes.begin(), nodes.end());
    sn_nodes.push_back(std::move(nodes));
    sn_children.push_back(std::move(children));
    return (int)sn_nodes.size() - 1;
  }

  long long weight(const std::vector<int> &s) const {
    long long w = 0;
    for (int v : s) w += m[v];
    return w;
  }

  // Dissects the node set S; returns the root supernodes of its forest.
  std::vector<int> dissect(const std::vector<int> &S) {
    if (S.empty()) return {};
    const int t = ++tag;
    for (int v : S) {
      mark[v] = t;
      lev[v] = -1;
    }
    // connected components of S
    std::vector<std::vector<int>> comps;
    std::vector<int> order;
    for (int v : S) {
      if (lev[v] >= 0) continue;
      bfs(g, mark, t, v, lev, order);
      comps.push_back(order);
    }
    std::vector<int> roots;
    for (auto &C : comps) {
      std::vector<int> r = dissect_connected(C);
      roots.insert(roots.end(), r.begin(), r.end());
    }
    return roots;
  }

  std::vector<int> dissect_connected(const std::vector<int> &C) {
    if (weight(C) <= leaf_dofs || C.size() <= 2) return {new_sn(C, {})};
    const int t = ++tag;
    for (int v : C) {
      mark[v] = t;
      lev[v] = -1;
    }
    // pseudo-peripheral start: two sweeps from the lowest-numbered node
    std::vector<int> order;
    int src = *std::min_element(C.begin(), C.end());
    bfs(g, mark, t, src, lev, order);
    src = order.back();
    for (int v : C) lev[v] = -1;
    const int maxl = bfs(g, mark, t, src, lev, order);
    if (maxl < 2) return {new_sn(C, {})};  // no level set separates: one dense supernode
    // the level whose cumulative weight first reaches half, kept inside 1..maxl-1
    std::vector<long long> wl(maxl + 1, 0);
    for (int v : C) wl[lev[v]] += m[v];
    const long long half = weight(C) / 2;
    long long acc = 0;
    int L = 1;
    for (int l = 0; l <= maxl; ++l) {
      acc += wl[l];
      if (acc >= half) {
        L = l;
        break;
      }
    }
    L = std::min(std::max(L, 1), maxl - 1);
    std::vector<int> A, B, Sep;
    for (int v : C) (lev[v] < L ? A : lev[v] > L ? B : Sep).push_back(v);
    std::vector<int> ch = dissect(A);
    std::vector<int> chb = dissect(B);
    ch.insert(ch.end(), chb.begin(), chb.end());
    return {new_sn(Sep, ch)};
  }
};

}  // namespace

bool build_tree_plan(int N, const std::vector<int> &mi, const std::vector<int> &coff,
                     const std::vector<int> &pair_i, const std::vector<int> &pair_j, TreePlan &tp,
                     std::string &msg) {
  tp = TreePlan();
  const size_t np = pair_i.size();
  // subdomain graph (nodes with m_i > 0)
  Graph g;
  g.n = N;
  g.ptr.assign(N + 1, 0);
  for (size_t q = 0; q < np; ++q)
    if (pair_i[q] != pair_j[q]) g.ptr[pair_i[q] + 1]++;
  for (int i = 0; i < N; ++i) g.ptr[i + 1] += g.ptr[i];
  g.adj.resize(g.ptr[N]);
  {
    std::vector<int> fill(g.ptr.begin(), g.ptr.end() - 1);
    for (size_t q = 0; q < np; ++q)
      if (pair_i[q] != pair_j[q]) g.adj[fill[pair_i[q]]++] = pair_j[q];
  }
  std::vector<int> nodes;
  for (int i = 0; i < N; ++i)
    if (mi[i] > 0) nodes.push_back(i);
  Builder b(g, mi, TS);
  std::vector<int> roots = b.dissect(nodes);
  const int ns = (int)b.sn_nodes.size();
  // parents
  std::vector<int> sparent(ns, -1);
  for (int s = 0; s < ns; ++s)
    for (int c : b.sn_children[s]) sparent[c] = s;
  // nested-dissection position of every subdomain: supernodes in creation
  // order (a postorder: children first), their subdomains ascending
  std::vector<int> pos(N, -1), sn_of(N, -1);
  {
    int q = 0;
    for (int s = 0; s < ns; ++s)
      for (int v : b.sn_nodes[s]) {
        pos[v] = q++;
        sn_of[v] = s;
      }
    if (q != (int)nodes.size()) {
      msg = "coarse tree: nested dissection lost subdomains";
      return false;
    }
  }
  // symbolic structure: struct(s) = subdomains adjacent to s's own or in its
  // children's structures, placed after s (ancestors), sorted by position
  std::vector<std::vector<int>> st(ns);
  for (int s = 0; s < ns; ++s) {
    const int last = pos[b.sn_nodes[s].back()];
    std::vector<int> cand;
    for (int v : b.sn_nodes[s])
      for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e)
        if (pos[g.adj[e]] > last) cand.push_back(g.adj[e]);
    for (int c : b.sn_children[s])
      for (int v : st[c])
        if (pos[v] > last) cand.push_back(v);
    std::sort(cand.begin(), cand.end(), [&](int a, int c) { return pos[a] < pos[c]; });
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    st[s] = std::move(cand);
  }
  // levels (height above the leaves)
  std::vector<int> height(ns, 0);
  for (int s = 0; s < ns; ++s)
    for (int c : b.sn_children[s]) height[s] = std::max(height[s], height[c] + 1);
  int nlevel = 0;
  for (int s = 0; s < ns; ++s) nlevel = std::max(nlevel, height[s] + 1);
  // front numbering: level by level, creation order inside a level
  std::vector<int> fid(ns), sn_at;
  tp.lvl_ptr.assign(nlevel + 1, 0);
  for (int s = 0; s < ns; ++s) tp.lvl_ptr[height[s] + 1]++;
  for (int h = 0; h < nlevel; ++h) tp.lvl_ptr[h + 1] += tp.lvl_ptr[h];
  {
    std::vector<int> fill(tp.lvl_ptr.begin(), tp.lvl_ptr.end() - 1);
    sn_at.resize(ns);
    for (int s = 0; s < ns; ++s) {
      fid[s] = fill[height[s]]++;
      sn_at[fid[s]] = s;
    }
  }
  tp.nfront = ns;
  tp.nlevel = nlevel;
  tp.K.resize(ns);
  tp.T.resize(ns);
  tp.kdof.resize(ns);
  tp.udof.resize(ns);
  tp.fbase.resize(ns);
  tp.xbase.resize(ns);
  tp.dbase.resize(ns);
  tp.rbase.resize(ns);
  tp.vbase.resize(ns);
  tp.parent.resize(ns);
  // first front row of each subdomain within its own front and within the
  // fronts whose update set holds it are computed per front below
  for (int f = 0; f < ns; ++f) {
    const int s = sn_at[f];
    long long kd = 0, ud = 0;
    for (int v : b.sn_nodes[s]) kd += mi[v];
    for (int v : st[s]) ud += mi[v];
    tp.kdof[f] = (int)kd;
    tp.udof[f] = (int)ud;
    tp.K[f] = (int)((kd + TS - 1) / TS);
    tp.T[f] = tp.K[f] + (int)((ud + TS - 1) / TS);
    tp.parent[f] = sparent[s] >= 0 ? fid[sparent[s]] : -1;
    tp.fbase[f] = tp.ftiles;
    tp.ftiles += (long long)tp.T[f] * (tp.T[f] + 1) / 2;
    tp.xbase[f] = tp.xtiles;
    tp.xtiles += (long long)tp.T[f] * tp.K[f];
    tp.dbase[f] = tp.dtiles;
    tp.dtiles += tp.K[f];
    tp.rbase[f] = tp.nrows;
    tp.nrows += TS * tp.T[f];
    tp.vbase[f] = tp.nvec;
    tp.nvec += (int)ud;
    tp.max_T = std::max(tp.max_T, tp.T[f]);
    tp.max_K = std::max(tp.max_K, tp.K[f]);
    for (int k = 0; k < tp.K[f]; ++k) {
      const double t = tp.T[f] - k - 1;
      tp.flops += 1.0 + t + t * (t + 1) / 2 + (k + 1) * (1.0 + t);  // potrf, trsm, syrk, X
    }
  }
  tp.flops *= 2.0 * TS * TS * TS;
  // row tables; the front row of a subdomain's first dof in each front
  tp.row_coarse.assign(tp.nrows, -1);
  std::vector<std::vector<std::pair<int, int>>> first_row(ns);  // (subdomain, row), by position
  for (int f = 0; f < ns; ++f) {
    const int s = sn_at[f];
    int r = 0;
    auto &fr = first_row[f];
    for (int v : b.sn_nodes[s]) {
      fr.push_back({v, r});
      for (int a = 0; a < mi[v]; ++a) tp.row_coarse[tp.rbase[f] + r + a] = coff[v] + a;
      r += mi[v];
    }
    r = TS * tp.K[f];
    for (int v : st[s]) {
      fr.push_back({v, r});
      for (int a = 0; a < mi[v]; ++a) tp.row_coarse[tp.rbase[f] + r + a] = coff[v] + a;
      r += mi[v];
    }
    std::sort(fr.begin(), fr.end());
  }
  auto row_of = [&](int f, int v) -> int {
    const auto &fr = first_row[f];
    auto it = std::lower_bound(fr.begin(), fr.end(), std::make_pair(v, -1));
    return (it != fr.end() && it->first == v) ? it->second : -1;
  };
  // extend-add rows and forward gather lists
  tp.ea_row.assign(tp.nvec, -1);
  std::vector<std::vector<int>> gl(tp.nrows);
  for (int f = 0; f < ns; ++f) {
    const int s = sn_at[f], pf = tp.parent[f];
    int t = 0;
    for (int v : st[s]) {
      const int pr0 = pf >= 0 ? row_of(pf, v) : -1;
      if (pr0 < 0) {
        msg = "coarse tree: an update subdomain is missing from the parent front";
        return false;
      }
      for (int a = 0; a < mi[v]; ++a, ++t) {
        tp.ea_row[tp.vbase[f] + t] = pr0 + a;
        gl[tp.rbase[pf] + pr0 + a].push_back(tp.vbase[f] + t);
      }
    }
  }
  tp.gptr.assign(tp.nrows + 1, 0);
  for (int r = 0; r < tp.nrows; ++r) tp.gptr[r + 1] = tp.gptr[r] + (int)gl[r].size();
  tp.gsrc.reserve(tp.gptr.back());
  for (int r = 0; r < tp.nrows; ++r) tp.gsrc.insert(tp.gsrc.end(), gl[r].begin(), gl[r].end());
  // children by level and slot
  std::vector<int> nslot(ns, 0), slot(ns, 0);
  for (int f = 0; f < ns; ++f)
    if (tp.parent[f] >= 0) slot[f] = nslot[tp.parent[f]]++;
  for (int f = 0; f < ns; ++f) tp.max_slots = std::max(tp.max_slots, nslot[f]);
  const int MS = std::max(tp.max_slots, 1);
  tp.ch_ptr.assign((size_t)nlevel * MS + 1, 0);
  std::vector<std::vector<int>> lists((size_t)nlevel * MS);
  for (int f = 0; f < ns; ++f) {
    const int pf = tp.parent[f];
    if (pf < 0) continue;
    lists[(size_t)height[sn_at[pf]] * MS + slot[f]].push_back(f);
  }
  for (size_t q = 0; q < lists.size(); ++q) {
    tp.ch_ptr[q + 1] = tp.ch_ptr[q] + (int)lists[q].size();
    tp.ch_front.insert(tp.ch_front.end(), lists[q].begin(), lists[q].end());
  }
  // A0 assembly entries
  std::vector<int> rev(np, -1);
  {
    // pairs of subdomain i are sorted by j: find (j, i) by binary search
    std::vector<int> first(N + 1, (int)np);
    for (size_t q = np; q-- > 0;) first[pair_i[q]] = (int)q;
    for (int i = N - 1; i >= 0; --i)
      if (first[i] == (int)np) first[i] = first[i + 1];
    for (size_t q = 0; q < np; ++q) {
      const int i = pair_i[q], j = pair_j[q];
      int lo = first[j], hi = first[j + 1];
      auto it = std::lower_bound(pair_j.begin() + lo, pair_j.begin() + hi, i);
      if (it == pair_j.begin() + hi || *it != i) {
        msg = "coarse tree: the coupled pairs are not symmetric";
        return false;
      }
      rev[q] = (int)(it - pair_j.begin());
    }
  }
  for (size_t q = 0; q < np; ++q) {
    const int i = pair_i[q], j = pair_j[q];
    if (mi[i] == 0 || mi[j] == 0 || pos[i] < pos[j]) continue;
    const int f = fid[sn_of[j]];  // eliminated first: j's front holds both
    const int ri = row_of(f, i), rj = row_of(f, j);
    if (ri < 0 || rj < 0) {
      msg = "coarse tree: a coupled pair falls outside its front";
      return false;
    }
    tp.as_pair.push_back((int)q);
    tp.as_rev.push_back(rev[q]);
    tp.as_front.push_back(f);
    tp.as_ri.push_back(ri);
    tp.as_rj.push_back(rj);
  }
  // per-level maxima
  tp.lvl_maxT.assign(nlevel, 0);
  tp.lvl_maxK.assign(nlevel, 0);
  tp.lvl_maxU.assign(nlevel, 0);
  for (int h = 0; h < nlevel; ++h)
    for (int f = tp.lvl_ptr[h]; f < tp.lvl_ptr[h + 1]; ++f) {
      tp.lvl_maxT[h] = std::max(tp.lvl_maxT[h], tp.T[f]);
      tp.lvl_maxK[h] = std::max(tp.lvl_maxK[h], tp.K[f]);
      const int U = tp.T[f] - tp.K[f];
      tp.lvl_maxU[h] = std::max(tp.lvl_maxU[h], U * (U + 1) / 2);
    }
  return true;
}

}  // namespace amsp
