// Host-side input validation and index planning (integer work only).
//
// Planning turns (CSR pattern, partition, overlap) into the per-subdomain
// index sets the device kernels consume:
//   * cores Omega_i from the partition and regions Omega_i^delta by delta
//     rounds of graph growth (Section 3.1: non-overlapping graph subdomains
//     and an overlapping support region around each);
//   * a local order per region (reverse Cuthill-McKee by default) and the
//     region's local CSR in that order;
//   * the 64x64 tile profile of each local lower triangle;
//   * dof multiplicities and the inverse map dof -> (subdomain, local index);
//   * extended regions (one more layer) and the subdomain pairs whose
//     supports couple through A, used to form A0 = R0 A R0^T.
#include "amsp_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace amsp {

int validate_inputs(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                    int32_t overlap, std::string &msg) {
  if (!A || !part || !A->row_ptr || !A->col_idx || !A->val) {
    msg = "null pointer argument";
    return AMSP_ERR_ARG;
  }
  if (nev < 0 || nev > MAXNEV) {
    msg = "nev must be in [0, " + std::to_string(MAXNEV) + "]";
    return AMSP_ERR_ARG;
  }
  if (overlap < 0 || overlap > 64) {
    msg = "overlap must be in [0, 64]";
    return AMSP_ERR_ARG;
  }
  const int64_t n = A->n;
  if (n < 1 || n > (int64_t)1 << 30) {
    msg = "n out of range";
    return n < 1 ? AMSP_ERR_ARG : AMSP_ERR_OOM;
  }
  if (nparts < 1 || nparts > n) {
    msg = "nparts must be in [1, n]";
    return AMSP_ERR_PARTITION;
  }
  const int64_t *rp = A->row_ptr;
  if (rp[0] != 0 || rp[n] != A->nnz || A->nnz >= ((int64_t)1 << 31)) {
    msg = "row_ptr[0] must be 0, row_ptr[n] == nnz < 2^31";
    return AMSP_ERR_CSR;
  }
  double amax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) {
      msg = "row_ptr not monotone at row " + std::to_string(i);
      return AMSP_ERR_CSR;
    }
    bool diag = false;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t c = A->col_idx[e];
      if (c < 0 || c >= n || (e > rp[i] && c <= A->col_idx[e - 1])) {
        msg = "column index out of range or unsorted in row " + std::to_string(i);
        return AMSP_ERR_CSR;
      }
      const double v = A->val[e];
      if (!std::isfinite(v)) {
        msg = "non-finite value in row " + std::to_string(i);
        return AMSP_ERR_CSR;
      }
      if (c == i) diag = true;
      amax = std::max(amax, std::fabs(v));
    }
    if (!diag) {
      msg = "missing diagonal entry in row " + std::to_string(i);
      return AMSP_ERR_CSR;
    }
  }
  const double tol = 1e-14 * amax;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t c = A->col_idx[e];
      if (c == i) continue;
      const int32_t *b = A->col_idx + rp[c], *en = A->col_idx + rp[c + 1];
      const int32_t *f = std::lower_bound(b, en, (int32_t)i);
      if (f == en || *f != i) {
        msg = "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(c) + ")";
        return AMSP_ERR_NONSYM;
      }
      if (std::fabs(A->val[rp[c] + (f - b)] - A->val[e]) > tol) {
        msg = "values not symmetric at (" + std::to_string(i) + "," + std::to_string(c) + ")";
        return AMSP_ERR_NONSYM;
      }
    }
  }
  std::vector<int64_t> cnt(nparts, 0);
  for (int64_t j = 0; j < n; ++j) {
    if (part[j] < 0 || part[j] >= nparts) {
      msg = "partition value out of range at dof " + std::to_string(j);
      return AMSP_ERR_PARTITION;
    }
    cnt[part[j]]++;
  }
  for (int32_t k = 0; k < nparts; ++k)
    if (cnt[k] == 0) {
      msg = "empty subdomain " + std::to_string(k);
      return AMSP_ERR_PARTITION;
    }
  return AMSP_OK;
}

// Reverse Cuthill-McKee order of a small graph given as adjacency lists
// (local indices).  Each component starts from a pseudo-peripheral node;
// neighbours are visited by increasing degree, ties by index.
static void rcm_order(const std::vector<int> &adj_ptr, const std::vector<int> &adj,
                      std::vector<int> &order) {
  const int n = (int)adj_ptr.size() - 1;
  std::vector<int> deg(n), level(n, -1);
  for (int v = 0; v < n; ++v) deg[v] = adj_ptr[v + 1] - adj_ptr[v];
  std::vector<char> vis(n, 0);
  order.clear();
  order.reserve(n);
  std::vector<int> q;
  q.reserve(n);
  auto bfs_last_min = [&](int s, int &ecc) {
    // BFS within the component (unvisited nodes); return min-degree node of the last level
    q.clear();
    q.push_back(s);
    std::vector<int> touched{s};
    level[s] = 0;
    size_t h = 0;
    int last = 0;
    while (h < q.size()) {
      int v = q[h++];
      last = std::max(last, level[v]);
      for (int e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e) {
        int w = adj[e];
        if (!vis[w] && level[w] < 0) {
          level[w] = level[v] + 1;
          q.push_back(w);
          touched.push_back(w);
        }
      }
    }
    int best = -1;
    for (int v : q)
      if (level[v] == last && (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)))
        best = v;
    for (int v : touched) level[v] = -1;
    ecc = last;
    return best;
  };
  for (int s0 = 0; s0 < n; ++s0) {
    if (vis[s0]) continue;
    // pseudo-peripheral node (George-Liu)
    int s = s0, ecc = -1;
    for (int it = 0; it < 8; ++it) {
      int e2;
      int cand = bfs_last_min(s, e2);
      if (e2 <= ecc) break;
      ecc = e2;
      s = cand;
    }
    // Cuthill-McKee from s
    size_t start = order.size();
    order.push_back(s);
    vis[s] = 1;
    size_t h = start;
    std::vector<int> nb;
    while (h < order.size()) {
      int v = order[h++];
      nb.clear();
      for (int e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e)
        if (!vis[adj[e]]) nb.push_back(adj[e]);
      std::sort(nb.begin(), nb.end(), [&](int a, int b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      for (int w : nb)
        if (!vis[w]) {
          vis[w] = 1;
          order.push_back(w);
        }
    }
  }
  std::reverse(order.begin(), order.end());
}

int build_plan(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
               const amsp_options &opt, HostPlan &P, std::string &msg) {
  const int n = (int)A->n;
  const int64_t *rp = A->row_ptr;
  const int32_t *ci = A->col_idx;
  const double *va = A->val;
  const int N = nparts;
  const int delta = opt.overlap;
  P.n = n;
  P.N = N;
  P.nev = nev;
  // cores: stable bucket by part
  std::vector<int> core_ptr(N + 1, 0), core(n);
  for (int j = 0; j < n; ++j) core_ptr[part[j] + 1]++;
  for (int i = 0; i < N; ++i) core_ptr[i + 1] += core_ptr[i];
  {
    std::vector<int> pos(core_ptr.begin(), core_ptr.end() - 1);
    for (int j = 0; j < n; ++j) core[pos[part[j]]++] = j;
  }
  std::vector<int> stamp(n, -1), loc(n, -1);
  P.sd_ptr.assign(1, 0);
  P.sd_dofs.clear();
  P.vp_ptr.assign(1, 0);
  P.trow_ptr.assign(1, 0);
  P.tfirst.clear();
  P.toff.clear();
  P.loc_rowptr.assign(1, 0);
  P.loc_col.clear();
  P.loc_src.clear();
  P.mult.assign(n, 0);
  P.mi.assign(N, 0);
  P.coff.assign(1, 0);
  P.ext_ptr.assign(1, 0);
  P.ext_rowptr.assign(1, 0);
  P.ext_src.clear();
  P.ext_loc.clear();
  std::vector<int> ext_dofs;  // concatenated extended regions (ascending global)
  long long tiles = 0;
  P.max_ni = 0;
  P.max_npad = 0;
  std::vector<int> region, frontier, next, adj_ptr, adj, order, mincol;
  for (int i = 0; i < N; ++i) {
    region.assign(core.begin() + core_ptr[i], core.begin() + core_ptr[i + 1]);
    for (int g : region) stamp[g] = i;
    frontier = region;
    const int layers = delta + (nev > 0 ? 1 : 0);
    size_t region_size = region.size();
    for (int d = 0; d < layers; ++d) {
      next.clear();
      for (int g : frontier)
        for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
          const int c = ci[e];
          if (c != g && va[e] != 0.0 && stamp[c] != i) {
            stamp[c] = i;
            next.push_back(c);
          }
        }
      region.insert(region.end(), next.begin(), next.end());
      if (d == delta - 1) region_size = region.size();
      frontier.swap(next);
    }
    if (delta == 0) region_size = core_ptr[i + 1] - core_ptr[i];
    std::vector<int> ext(region.begin(), region.end());
    region.resize(region_size);
    std::sort(region.begin(), region.end());
    const int ni = (int)region.size();
    // local adjacency in ascending-global order
    for (int k = 0; k < ni; ++k) loc[region[k]] = k;
    adj_ptr.assign(ni + 1, 0);
    adj.clear();
    for (int k = 0; k < ni; ++k) {
      const int g = region[k];
      for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
        const int c = ci[e];
        if (c != g && va[e] != 0.0 && loc[c] >= 0) adj.push_back(loc[c]);
      }
      adj_ptr[k + 1] = (int)adj.size();
    }
    if (opt.local_order == AMSP_ORDER_RCM) {
      rcm_order(adj_ptr, adj, order);
    } else {
      order.resize(ni);
      for (int k = 0; k < ni; ++k) order[k] = k;
    }
    // final local order: local index k -> global region[order[k]]
    const int base = P.sd_ptr.back();
    for (int k = 0; k < ni; ++k) {
      const int g = region[order[k]];
      P.sd_dofs.push_back(g);
      loc[g] = k;
      P.mult[g]++;
    }
    // local CSR in the final order
    mincol.assign(ni, 0);
    std::vector<std::pair<int, int>> row;
    for (int k = 0; k < ni; ++k) {
      const int g = P.sd_dofs[base + k];
      row.clear();
      for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
        const int c = ci[e];
        if (loc[c] >= 0) row.emplace_back(loc[c], (int)e);
      }
      std::sort(row.begin(), row.end());
      mincol[k] = row.empty() ? k : std::min(k, row.front().first);
      for (auto &pr : row) {
        P.loc_col.push_back(pr.first);
        P.loc_src.push_back(pr.second);
      }
      P.loc_rowptr.push_back((int)P.loc_col.size());
    }
    // tile profile
    const int nt = (ni + TS - 1) / TS;
    for (int I = 0; I < nt; ++I) {
      int f = I;
      if (opt.dense_tiles) {
        f = 0;
      } else {
        for (int k = I * TS; k < std::min(ni, (I + 1) * TS); ++k) f = std::min(f, mincol[k] / TS);
      }
      P.tfirst.push_back(f);
      P.toff.push_back(tiles);
      tiles += I - f + 1;
    }
    P.trow_ptr.push_back(P.trow_ptr.back() + nt);
    P.sd_ptr.push_back(base + ni);
    P.vp_ptr.push_back(P.vp_ptr.back() + nt * TS);
    P.max_ni = std::max(P.max_ni, ni);
    P.max_npad = std::max(P.max_npad, nt * TS);
    const int m = std::min(nev, ni);
    P.mi[i] = m;
    P.coff.push_back(P.coff.back() + m);
    // extended region (one more layer) for A Phi_i
    if (nev > 0) {
      std::sort(ext.begin(), ext.end());
      for (int g : ext) {
        ext_dofs.push_back(g);
        for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
          const int c = ci[e];
          if (loc[c] >= 0) {
            P.ext_src.push_back((int)e);
            P.ext_loc.push_back(loc[c]);
          }
        }
        P.ext_rowptr.push_back((int)P.ext_src.size());
      }
      P.ext_ptr.push_back((int)ext_dofs.size());
    }
    for (int k = 0; k < ni; ++k) loc[P.sd_dofs[base + k]] = -1;
  }
  P.ntiles = tiles;
  P.nc = P.coff.back();
  // inverse map: dof -> (subdomain, local index), subdomains ascending
  P.inv_ptr.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) P.inv_ptr[j + 1] = P.inv_ptr[j] + P.mult[j];
  const int tot = P.inv_ptr[n];
  P.inv_sd.assign(tot, 0);
  P.inv_loc.assign(tot, 0);
  {
    std::vector<int> pos(P.inv_ptr.begin(), P.inv_ptr.end() - 1);
    for (int i = 0; i < N; ++i)
      for (int k = P.sd_ptr[i]; k < P.sd_ptr[i + 1]; ++k) {
        const int g = P.sd_dofs[k];
        P.inv_sd[pos[g]] = i;
        P.inv_loc[pos[g]] = k - P.sd_ptr[i];
        pos[g]++;
      }
  }
  for (int j = 0; j < n; ++j)
    if (P.mult[j] == 0) {
      msg = "dof not covered by any region";
      return AMSP_ERR_PARTITION;
    }
  // coupled subdomain pairs for A0
  P.pair_i.clear();
  P.pair_j.clear();
  P.pair_ptr.assign(1, 0);
  P.pair_l.clear();
  P.pair_e.clear();
  if (nev > 0 && P.nc > 0) {
    // dof -> list of (j, e) with dof = ext_dofs[ext_ptr[j] + e]
    std::vector<int> xptr(n + 1, 0);
    for (int g : ext_dofs) xptr[g + 1]++;
    for (int j = 0; j < n; ++j) xptr[j + 1] += xptr[j];
    std::vector<int> xj(ext_dofs.size()), xe(ext_dofs.size());
    {
      std::vector<int> pos(xptr.begin(), xptr.end() - 1);
      for (int j = 0; j < N; ++j)
        for (int e = P.ext_ptr[j]; e < P.ext_ptr[j + 1]; ++e) {
          const int g = ext_dofs[e];
          xj[pos[g]] = j;
          xe[pos[g]] = e - P.ext_ptr[j];
          pos[g]++;
        }
    }
    std::vector<std::array<int, 3>> trip;
    for (int i = 0; i < N; ++i) {
      if (P.mi[i] == 0) continue;
      trip.clear();
      for (int k = P.sd_ptr[i]; k < P.sd_ptr[i + 1]; ++k) {
        const int g = P.sd_dofs[k];
        for (int q = xptr[g]; q < xptr[g + 1]; ++q)
          if (P.mi[xj[q]] > 0) trip.push_back({xj[q], k - P.sd_ptr[i], xe[q]});
      }
      std::stable_sort(trip.begin(), trip.end(),
                       [](const std::array<int, 3> &a, const std::array<int, 3> &b) { return a[0] < b[0]; });
      size_t s = 0;
      while (s < trip.size()) {
        size_t e = s;
        while (e < trip.size() && trip[e][0] == trip[s][0]) ++e;
        P.pair_i.push_back(i);
        P.pair_j.push_back(trip[s][0]);
        for (size_t u = s; u < e; ++u) {
          P.pair_l.push_back(trip[u][1]);
          P.pair_e.push_back(trip[u][2]);
        }
        P.pair_ptr.push_back((int)P.pair_l.size());
        s = e;
      }
    }
  }
  return AMSP_OK;
}

}  // namespace amsp
