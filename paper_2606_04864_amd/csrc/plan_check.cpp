// Host-only check program for the index planner, built with AddressSanitizer
// and UndefinedBehaviorSanitizer (see build.py: build_plan_check).  It runs
// the planner's validation and both planning phases on a set of grid
// matrices (2D five-point and 3D seven-point, ragged sizes, all option
// combinations the library exposes), on inputs each check must reject, from
// two threads at once (the worker pool's busy path), then releases the
// caches, plans again (pools and caches re-created) and exits, so that the
// exit handler's teardown also runs under the sanitizers.  It checks the
// plan's basic invariants (every core inside its region, pointers monotone,
// regions sorted sets once ordered) and prints one line per case.
// Exit status 0 means every case behaved.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "amsp_plan.h"
#include "tree_check.h"

using namespace amsp;

namespace {

struct Grid {
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> va;
  std::vector<int32_t> part;
  int nparts = 1;
  amsp_csr csr() const {
    return amsp_csr{(int64_t)rp.size() - 1, (int64_t)ci.size(), rp.data(), ci.data(), va.data()};
  }
};

// Symmetric M-matrix on an nx x ny x nz grid (nz = 1: five-point), with
// face coefficients from a fixed integer hash so that rows differ; the
// partition cuts the grid into px x py x pz boxes.
Grid make_grid(int nx, int ny, int nz, int px, int py, int pz) {
  Grid g;
  const int n = nx * ny * nz;
  auto id = [&](int x, int y, int z) { return x + nx * (y + ny * z); };
  auto coef = [](int a, int b) {
    unsigned h = (unsigned)std::min(a, b) * 2654435761u ^ (unsigned)std::max(a, b) * 40503u;
    return 1.0 + (double)(h % 1000) / 10.0;
  };
  g.rp.push_back(0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int i = id(x, y, z);
        std::vector<std::pair<int, double>> row;
        double d = 0.5;  // boundary term keeps the matrix definite
        const int nb[6][3] = {{x - 1, y, z}, {x + 1, y, z}, {x, y - 1, z},
                              {x, y + 1, z}, {x, y, z - 1}, {x, y, z + 1}};
        for (const auto &q : nb) {
          if (q[0] < 0 || q[0] >= nx || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nz) continue;
          const int j = id(q[0], q[1], q[2]);
          const double c = coef(i, j);
          row.push_back({j, -c});
          d += c;
        }
        row.push_back({i, d});
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
          g.ci.push_back(e.first);
          g.va.push_back(e.second);
        }
        g.rp.push_back((int64_t)g.ci.size());
      }
  g.part.resize(n);
  g.nparts = px * py * pz;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        g.part[id(x, y, z)] =
            (x * px / nx) + px * ((y * py / ny) + py * (z * pz / nz));
  return g;
}

int failures = 0;

void expect(bool ok, const std::string &what) {
  if (!ok) {
    ++failures;
    std::printf("FAIL %s\n", what.c_str());
  }
}

// Plans g with the options and checks the plan's invariants.
void plan_case(const Grid &g, int nev, int overlap, int order, int dense, const char *name) {
  amsp_options opt{};  // the planner reads only the fields set here
  opt.overlap = overlap;
  opt.local_order = order;
  opt.dense_tiles = dense;
  const amsp_csr A = g.csr();
  std::string msg;
  int64_t zeros = -1;
  int s = validate_inputs(&A, g.part.data(), g.nparts, nev, overlap, msg, &zeros);
  expect(s == AMSP_OK && zeros == 0, std::string(name) + ": validate " + msg);
  HostPlan P;
  P.offdiag_zeros = zeros != 0;  // the planner's column-only reads
  s = build_plan(&A, g.part.data(), g.nparts, nev, opt, P, msg);
  expect(s == AMSP_OK, std::string(name) + ": plan " + msg);
  if (s != AMSP_OK) return;
  {  // the same plan when every visited value is read
    HostPlan Q;
    Q.offdiag_zeros = true;
    s = build_plan(&A, g.part.data(), g.nparts, nev, opt, Q, msg);
    expect(s == AMSP_OK && Q.sd_dofs == P.sd_dofs && Q.loc_rowptr == P.loc_rowptr &&
               Q.tfirst == P.tfirst && Q.ext_ptr == P.ext_ptr && Q.ext_src == P.ext_src &&
               Q.pair_j == P.pair_j && Q.pair_e == P.pair_e,
           std::string(name) + ": plan with value reads differs");
  }
  const int N = g.nparts;
  expect((int)P.sd_ptr.size() == N + 1, std::string(name) + ": sd_ptr size");
  bool mono = true, cores_in = true, sets = true;
  for (int i = 0; i < N; ++i) {
    mono &= P.sd_ptr[i] <= P.sd_ptr[i + 1] && P.vp_ptr[i] <= P.vp_ptr[i + 1] &&
            P.trow_ptr[i] <= P.trow_ptr[i + 1];
    std::vector<int> d(P.sd_dofs.begin() + P.sd_ptr[i], P.sd_dofs.begin() + P.sd_ptr[i + 1]);
    std::sort(d.begin(), d.end());
    sets &= std::adjacent_find(d.begin(), d.end()) == d.end() && !d.empty() && d.front() >= 0 &&
            d.back() < (int)A.n;
    for (int64_t j = 0; j < A.n; ++j)
      if (g.part[j] == i) cores_in &= std::binary_search(d.begin(), d.end(), (int)j);
  }
  expect(mono, std::string(name) + ": pointers monotone");
  expect(sets, std::string(name) + ": regions are sets of valid dofs");
  expect(cores_in, std::string(name) + ": cores inside regions");
  std::printf("ok %s: N %d, sum n_i %d, tiles %lld, pairs %zu\n", name, N, P.sd_ptr[N],
              P.ntiles, P.pair_i.size());
  if (nev > 0) {  // the sparse coarse factorisation on this plan's coupling
    TreePlan tp;
    s = build_tree_plan(N, P.mi, P.coff, P.pair_i, P.pair_j, tp, msg) ? 0 : 1;
    expect(s == 0, std::string(name) + ": tree plan " + msg);
    const double err = tree_emulate(N, nev, P.mi, P.coff, P.pair_i, P.pair_j, 7u, msg);
    expect(err >= 0 && err < 1e-11, std::string(name) + ": tree solve " + msg + " err " +
                                        std::to_string(err));
    std::printf("ok %s: coarse tree %d fronts, %d levels, max front %d tiles, solve err %.2e\n",
                name, tp.nfront, tp.nlevel, tp.max_T, err);
  }
}

void reject_case(Grid g, int what, int want, const char *name) {
  const int nev = 4, overlap = 1;
  if (what == 0) std::swap(g.ci[1], g.ci[2]);           // unsorted columns
  if (what == 1) g.va[g.rp[3]] *= 1.5;                   // asymmetric value (row 3, column 2)
  if (what == 2) g.part[5] = g.nparts + 3;               // part out of range
  if (what == 3) g.va[0] = 0.0 / 0.0;                    // non-finite value
  if (what == 4) g.rp[2] = g.rp[3] + 1;                  // row pointers not monotone
  const amsp_csr A = g.csr();
  std::string msg;
  const int s = validate_inputs(&A, g.part.data(), g.nparts, nev, overlap, msg);
  expect(s == want, std::string(name) + ": got " + std::to_string(s) + " " + msg);
  std::printf("ok %s: rejected (%d)\n", name, s);
}

}  // namespace

int main() {
  const Grid g2 = make_grid(61, 53, 1, 5, 4, 1);     // ragged 2D, 20 parts
  const Grid g3 = make_grid(14, 13, 11, 3, 2, 2);    // ragged 3D, 12 parts
  const Grid one = make_grid(9, 7, 1, 1, 1, 1);      // a single part
  for (int order = 0; order < 2; ++order)
    for (int dense = 0; dense < 2; ++dense) {
      plan_case(g2, 6, 2, order, dense, "2d delta2");
      plan_case(g3, 8, 1, order, dense, "3d delta1");
    }
  plan_case(g2, 0, 0, 0, 0, "2d no overlap, nev 0");
  // deeper coarse trees: 256 parts in 2D, 216 in 3D
  plan_case(make_grid(128, 128, 1, 16, 16, 1), 4, 1, 0, 0, "2d 256 parts");
  plan_case(make_grid(24, 24, 24, 6, 6, 6), 4, 1, 0, 0, "3d 216 parts");
  plan_case(one, 3, 1, 0, 0, "one part");
  reject_case(g2, 0, AMSP_ERR_CSR, "unsorted columns");
  reject_case(g2, 1, AMSP_ERR_NONSYM, "asymmetric");
  reject_case(g2, 2, AMSP_ERR_PARTITION, "partition out of range");
  reject_case(g2, 3, AMSP_ERR_CSR, "non-finite value");
  reject_case(g2, 4, AMSP_ERR_CSR, "row pointers");
  {  // two planners at once: one of them finds the worker pool busy
    std::thread t([&] { plan_case(g3, 8, 1, 0, 0, "thread A"); });
    plan_case(g2, 6, 2, 0, 0, "thread B");
    t.join();
  }
  plan_release_caches();
  plan_case(g3, 8, 1, 0, 0, "after release");  // pool and cache re-created
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "PASSED", failures);
  return failures ? 1 : 0;  // the exit handler releases the caches again
}
