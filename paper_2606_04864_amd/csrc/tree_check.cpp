// CPU emulation of k_tree.hip (see tree_check.h).  Host check program only.
#include "tree_check.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <stdexcept>

namespace amsp {

namespace {

struct Arr {
  std::vector<double> v;
  const char *name;
  double &at(long long i) {
    if (i < 0 || i >= (long long)v.size())
      throw std::runtime_error(std::string("out of bounds: ") + name + " [" + std::to_string(i) +
                               "] of " + std::to_string(v.size()));
    return v[i];
  }
};

void tri_index(int b, int &ii, int &jj) {
  ii = (int)((std::sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= b) ++ii;
  while (ii * (ii + 1) / 2 > b) --ii;
  jj = b - ii * (ii + 1) / 2;
}

// 64x64 tile products on row-major tiles
void chol_tile(double *a, double *inv, bool &fail) {  // a: lower -> L; inv = L^{-1}
  for (int k = 0; k < TS; ++k) {
    double d = a[k * TS + k];
    for (int j = 0; j < k; ++j) d -= a[k * TS + j] * a[k * TS + j];
    if (!(d > 0)) {
      fail = true;
      d = 1.0;
    }
    const double l = std::sqrt(d);
    a[k * TS + k] = l;
    for (int i = k + 1; i < TS; ++i) {
      double s = a[i * TS + k];
      for (int j = 0; j < k; ++j) s -= a[i * TS + j] * a[k * TS + j];
      a[i * TS + k] = s / l;
    }
  }
  for (int i = 0; i < TS; ++i)
    for (int j = i + 1; j < TS; ++j) a[i * TS + j] = 0.0;
  for (int c = 0; c < TS; ++c)
    for (int r = 0; r < TS; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) s -= a[r * TS + k] * inv[k * TS + c];
      inv[r * TS + c] = r < c ? 0.0 : s / a[r * TS + r];
    }
}

}  // namespace

double tree_emulate(int N, int nev, const std::vector<int> &mi, const std::vector<int> &coff,
                    const std::vector<int> &pair_i, const std::vector<int> &pair_j, unsigned seed,
                    std::string &msg) {
  TreePlan tp;
  if (!build_tree_plan(N, mi, coff, pair_i, pair_j, tp, msg)) return -1.0;
  const int nc = coff[N], np = (int)pair_i.size(), nn = nev * nev;
  try {
    // random SPD A0 with the block sparsity of the pairs: pair blocks
    // symmetric by construction, diagonal dominant
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    Arr pb{std::vector<double>((size_t)np * nn, 0.0), "pb"};
    std::vector<double> A0((size_t)nc * nc, 0.0);
    std::vector<int> first(N + 1, np);
    for (int q = np - 1; q >= 0; --q) first[pair_i[q]] = q;
    for (int i = N - 1; i >= 0; --i)
      if (first[i] == np) first[i] = first[i + 1];
    for (int q = 0; q < np; ++q) {
      const int i = pair_i[q], j = pair_j[q];
      if (i > j) continue;
      int r = -1;
      for (int t = first[j]; t < first[j + 1]; ++t)
        if (pair_j[t] == i) r = t;
      if (r < 0) throw std::runtime_error("pairs not symmetric");
      for (int a = 0; a < mi[i]; ++a)
        for (int b = 0; b < mi[j]; ++b) {
          double v = U(rng);
          if (i == j) v = (a == b) ? 0.0 : 0.0;
          pb.at((long long)q * nn + a * nev + b) = v;
          pb.at((long long)r * nn + b * nev + a) = v;
          A0[(size_t)(coff[i] + a) * nc + coff[j] + b] = v;
          A0[(size_t)(coff[j] + b) * nc + coff[i] + a] = v;
        }
    }
    for (int i = 0; i < N; ++i) {  // diagonal blocks: dominant SPD
      int q = -1;
      for (int t = first[i]; t < first[i + 1]; ++t)
        if (pair_j[t] == i) q = t;
      if (q < 0 && mi[i] > 0) throw std::runtime_error("missing diagonal pair");
      for (int a = 0; a < mi[i]; ++a)
        for (int b = 0; b <= a; ++b) {
          double v = 0.0;
          if (a == b) {
            double rs = 0.0;
            for (int c = 0; c < nc; ++c) rs += std::fabs(A0[(size_t)(coff[i] + a) * nc + c]);
            v = rs + 1.0 + 0.5 * std::fabs(U(rng));
          } else {
            v = 0.1 * U(rng);
          }
          pb.at((long long)q * nn + a * nev + b) = v;
          pb.at((long long)q * nn + b * nev + a) = v;
          A0[(size_t)(coff[i] + a) * nc + coff[i] + b] = v;
          A0[(size_t)(coff[i] + b) * nc + coff[i] + a] = v;
        }
    }
    Arr F{std::vector<double>((size_t)tp.ftiles * TE, 0.0), "F"};
    Arr X{std::vector<double>((size_t)tp.xtiles * TE, 0.0), "X"};
    Arr D{std::vector<double>((size_t)std::max(tp.dtiles, 1) * TE, 0.0), "dinv"};
    auto ft = [&](int f, int I, int J) -> long long {
      if (J > I || I >= tp.T[f]) throw std::runtime_error("front tile index");
      return (tp.fbase[f] + (long long)I * (I + 1) / 2 + J) * TE;
    };
    auto fe = [&](int f, int R, int C) -> double & {
      return F.at(ft(f, R >> 6, C >> 6) + (R & 63) * TS + (C & 63));
    };
    auto xt = [&](int f, int I, int J) -> long long {
      if (J >= tp.K[f] || I >= tp.T[f]) throw std::runtime_error("X tile index");
      return (tp.xbase[f] + (long long)I * tp.K[f] + J) * TE;
    };
    // k_tree_diag_init
    for (int f = 0; f < tp.nfront; ++f)
      for (int r = 0; r < tp.K[f] * TS; ++r) {
        if (r >= tp.kdof[f]) fe(f, r, r) = 1.0;
        X.at(xt(f, r >> 6, r >> 6) + (r & 63) * TS + (r & 63)) = 1.0;
      }
    // k_tree_assemble
    for (size_t e = 0; e < tp.as_pair.size(); ++e) {
      const int pr = tp.as_pair[e], rv = tp.as_rev[e], f = tp.as_front[e];
      const int i = pair_i[pr], j = pair_j[pr];
      for (int a = 0; a < mi[i]; ++a)
        for (int b = 0; b < mi[j]; ++b) {
          const int R = tp.as_ri[e] + a, C = tp.as_rj[e] + b;
          if (R < C) continue;
          fe(f, R, C) = 0.5 * (pb.at((long long)pr * nn + a * nev + b) + pb.at((long long)rv * nn + b * nev + a));
        }
    }
    bool fail = false;
    const int MS = std::max(tp.max_slots, 1);
    std::vector<double> tmp(TE);
    for (int lv = 0; lv < tp.nlevel; ++lv) {
      const int f0 = tp.lvl_ptr[lv], f1 = tp.lvl_ptr[lv + 1], maxT = tp.lvl_maxT[lv];
      for (int cs = 0; cs < tp.max_slots; ++cs) {  // k_tree_extend_add
        for (int q = tp.ch_ptr[(size_t)lv * MS + cs]; q < tp.ch_ptr[(size_t)lv * MS + cs + 1]; ++q) {
          const int c = tp.ch_front[q];
          const int Kc = tp.K[c], Uc = tp.T[c] - Kc, ud = tp.udof[c], pf = tp.parent[c];
          if (pf < f0 || pf >= f1) throw std::runtime_error("child's parent not in this level");
          for (int b = 0; b < Uc * (Uc + 1) / 2; ++b) {
            int ii, jj;
            tri_index(b, ii, jj);
            const long long src = ft(c, Kc + ii, Kc + jj);
            for (int e = 0; e < TE; ++e) {
              const int r = e >> 6, cc = e & 63, t1 = TS * ii + r, t2 = TS * jj + cc;
              if (t1 >= ud || t2 >= ud || (ii == jj && cc > r)) continue;
              const int P1 = tp.ea_row.at(tp.vbase[c] + t1), P2 = tp.ea_row.at(tp.vbase[c] + t2);
              if (P1 < P2) throw std::runtime_error("extend-add map not increasing");
              fe(pf, P1, P2) += F.at(src + e);
            }
          }
        }
      }
      for (int k = 0; k < tp.lvl_maxK[lv]; ++k) {
        for (int f = f0; f < f1; ++f) {  // potrf, trsm, syrk
          if (k >= tp.K[f]) continue;
          const int T = tp.T[f];
          const long long dk = (long long)(tp.dbase[f] + k) * TE;
          chol_tile(&F.at(ft(f, k, k)), &D.at(dk), fail);
          for (int i = k + 1; i < T && i < maxT; ++i) {
            double *a = &F.at(ft(f, i, k));
            for (int r = 0; r < TS; ++r)
              for (int c = 0; c < TS; ++c) {
                double s = 0.0;
                for (int q = 0; q < TS; ++q) s += a[r * TS + q] * D.at(dk + c * TS + q);
                tmp[r * TS + c] = s;
              }
            std::copy(tmp.begin(), tmp.end(), a);
          }
          const int m = maxT - k - 1;
          for (int b = 0; b < m * (m + 1) / 2; ++b) {
            if (b >= (T - k - 1) * (T - k) / 2) continue;
            int ii, jj;
            tri_index(b, ii, jj);
            const int i = k + 1 + ii, j = k + 1 + jj;
            double *c = &F.at(ft(f, i, j));
            const double *li = &F.at(ft(f, i, k)), *lj = &F.at(ft(f, j, k));
            for (int r = 0; r < TS; ++r)
              for (int cc = 0; cc < TS; ++cc) {
                double s = 0.0;
                for (int q = 0; q < TS; ++q) s += li[r * TS + q] * lj[cc * TS + q];
                c[r * TS + cc] -= s;
              }
          }
        }
      }
      for (int k = 0; k < tp.lvl_maxK[lv]; ++k) {
        for (int f = f0; f < f1; ++f) {  // inv_row, inv_update
          if (k >= tp.K[f]) continue;
          const long long dk = (long long)(tp.dbase[f] + k) * TE;
          for (int j = 0; j <= k; ++j) {
            double *w = &X.at(xt(f, k, j));
            for (int r = 0; r < TS; ++r)
              for (int c = 0; c < TS; ++c) {
                double s = 0.0;
                for (int q = 0; q < TS; ++q) s += D.at(dk + r * TS + q) * w[q * TS + c];
                tmp[r * TS + c] = s;
              }
            std::copy(tmp.begin(), tmp.end(), w);
          }
          for (int b = 0; b < (maxT - k - 1) * (k + 1); ++b) {
            const int i = k + 1 + b / (k + 1), j = b % (k + 1);
            if (i >= tp.T[f]) continue;
            double *c = &X.at(xt(f, i, j));
            const double *l = &F.at(ft(f, i, k)), *xk = &X.at(xt(f, k, j));
            for (int r = 0; r < TS; ++r)
              for (int cc = 0; cc < TS; ++cc) {
                double s = 0.0;
                for (int q = 0; q < TS; ++q) s += l[r * TS + q] * xk[q * TS + cc];
                c[r * TS + cc] -= s;
              }
          }
        }
      }
    }
    if (fail) throw std::runtime_error("a pivot failed in the emulated factorisation");
    // solve: c random; forward levels up, backward levels down
    std::vector<double> c(nc), y(std::max(nc, 1), 0.0), v(std::max(tp.nvec, 1), 0.0),
        x(nc, 0.0);
    for (double &e : c) e = U(rng);
    for (int lv = 0; lv < tp.nlevel; ++lv)
      for (int f = tp.lvl_ptr[lv]; f < tp.lvl_ptr[lv + 1]; ++f) {
        const int K = tp.K[f], T = tp.T[f], rb = tp.rbase[f];
        std::vector<double> cs(K * TS);
        for (int r = 0; r < K * TS; ++r) {
          const int rc = tp.row_coarse.at(rb + r);
          double s = rc >= 0 ? c.at(rc) : 0.0;
          for (int g = tp.gptr.at(rb + r); g < tp.gptr.at(rb + r + 1); ++g) s += v.at(tp.gsrc.at(g));
          cs[r] = s;
        }
        for (int I = 0; I < T; ++I) {
          const int jn = I < K ? I + 1 : K;
          for (int row = 0; row < TS; ++row) {
            double s = 0.0;
            for (int J = 0; J < jn; ++J)
              for (int e = 0; e < TS; ++e) s += X.at(xt(f, I, J) + row * TS + e) * cs[J * TS + e];
            const int R = I * TS + row;
            if (I < K) {
              const int rc = tp.row_coarse.at(rb + R);
              if (rc >= 0) y.at(rc) = s;
            } else {
              const int u = R - K * TS;
              if (u < tp.udof[f]) {
                for (int g = tp.gptr.at(rb + R); g < tp.gptr.at(rb + R + 1); ++g) s += v.at(tp.gsrc.at(g));
                v.at(tp.vbase[f] + u) = s;
              }
            }
          }
        }
      }
    for (int lv = tp.nlevel - 1; lv >= 0; --lv)
      for (int f = tp.lvl_ptr[lv]; f < tp.lvl_ptr[lv + 1]; ++f) {
        const int K = tp.K[f], T = tp.T[f], rb = tp.rbase[f];
        for (int J = 0; J < K; ++J) {
          std::vector<double> z(T * TS, 0.0);
          for (int r = J * TS; r < T * TS; ++r) {
            const int rc = tp.row_coarse.at(rb + r);
            z[r] = rc < 0 ? 0.0 : (r < K * TS ? y.at(rc) : x.at(rc));
          }
          for (int col = 0; col < TS; ++col) {
            double s = 0.0;
            for (int I = J; I < T; ++I)
              for (int r = 0; r < TS; ++r) s += X.at(xt(f, I, J) + r * TS + col) * z[I * TS + r];
            const int rc = tp.row_coarse.at(rb + J * TS + col);
            if (rc >= 0) x.at(rc) = s;
          }
        }
      }
    // dense reference: A0 x = c by Cholesky
    std::vector<double> L(A0);
    for (int k = 0; k < nc; ++k) {
      double d = L[(size_t)k * nc + k];
      for (int j = 0; j < k; ++j) d -= L[(size_t)k * nc + j] * L[(size_t)k * nc + j];
      if (!(d > 0)) throw std::runtime_error("reference matrix not SPD");
      L[(size_t)k * nc + k] = std::sqrt(d);
      for (int i = k + 1; i < nc; ++i) {
        double s = L[(size_t)i * nc + k];
        for (int j = 0; j < k; ++j) s -= L[(size_t)i * nc + j] * L[(size_t)k * nc + j];
        L[(size_t)i * nc + k] = s / L[(size_t)k * nc + k];
      }
    }
    std::vector<double> w(c);
    for (int i = 0; i < nc; ++i) {
      for (int j = 0; j < i; ++j) w[i] -= L[(size_t)i * nc + j] * w[j];
      w[i] /= L[(size_t)i * nc + i];
    }
    for (int i = nc - 1; i >= 0; --i) {
      for (int j = i + 1; j < nc; ++j) w[i] -= L[(size_t)j * nc + i] * w[j];
      w[i] /= L[(size_t)i * nc + i];
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i < nc; ++i) {
      num += (x[i] - w[i]) * (x[i] - w[i]);
      den += w[i] * w[i];
    }
    return std::sqrt(num / den);
  } catch (const std::exception &e) {
    msg = e.what();
    return -1.0;
  }
}

}  // namespace amsp
