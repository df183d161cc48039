// Several right-hand sides at once: z_k = M^{-1} r_k for up to EIGP columns
// with one pass over the local factors.  With many columns the local solves
// become triangular solves with a block of right-hand sides, whose diagonal
// products run on the matrix cores: the same block solve the eigensolver
// uses (k_env_solve_block), here with the Dirichlet factor of the apply.
//
// Layouts: the columns of r and z are n apart (column-major n x nr); the
// gathered block X and the solved block Y hold, per region, npad_i rows of
// EIGP doubles in the local (RCM) order at row vp_ptr[i]; XN holds the
// region outputs (local solve plus coarse prolongation) in the region's
// ascending-global-index layout, the layout the scatter reads.  Columns nr ..
// EIGP-1 and padding rows are zero.
#include "k_common.h"

namespace amsp {

// X[vp_i + l][k] = r_k[dof(l)] for real rows and k < nr, zero otherwise;
// thread per row (its EIGP entries are one contiguous 128-byte row of X).
__global__ void __launch_bounds__(WG) k_gather_multi(Plan p, int n, int nr,
                                                     const double *__restrict__ r,
                                                     double *__restrict__ X) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int v0 = p.vp_ptr[i], npad = p.vp_ptr[i + 1] - v0;
  for (int l = threadIdx.x; l < npad; l += WG) {
    const int dof = l < ni ? p.sd_dofs[r0 + l] : -1;
    double v[EIGP];
#pragma unroll
    for (int k = 0; k < EIGP; ++k) v[k] = (dof >= 0 && k < nr) ? r[(size_t)k * n + dof] : 0.0;
    double2 *dst = reinterpret_cast<double2 *>(X + (size_t)(v0 + l) * EIGP);
#pragma unroll
    for (int k = 0; k < EIGP / 2; ++k) dst[k] = make_double2(v[2 * k], v[2 * k + 1]);
  }
}

// Restriction of every column: c_k[coff_i + q] = sum_l phi_i[l][q] X[l][k].
// Thread (row group g, column k) adds rows g, g + 16, ... for all q (GU rows'
// loads issued together); the 16 group sums are then added in group order.
// The coarse vectors are ncp apart (their padding stays zero).
template <typename TB>
__global__ void __launch_bounds__(WG) k_restrict_multi(Plan p, int nr, size_t ncp,
                                                       const TB *__restrict__ phi,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ c) {
  constexpr int RGS = WG / EIGP;  // row groups
  __shared__ double sh[RGS][MAXNEV][EIGP];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0, m = p.mi[i], nev = p.nev;
  const int k = threadIdx.x % EIGP, g = threadIdx.x / EIGP;
  const double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  if (m > 0)
    with_km(nev, [&](auto km) __attribute__((always_inline)) {
      constexpr int KM = decltype(km)::value, GU = 4;
      double acc[KM];
#pragma unroll
      for (int q = 0; q < KM; ++q) acc[q] = 0.0;
      for (int l0 = g; l0 < ni; l0 += GU * RGS) {
        double x[GU];
        TB raw[GU][KM];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
          const int l = l0 + u * RGS, lc = min(l, ni - 1);
          x[u] = l < ni ? Xi[(size_t)lc * EIGP + k] : 0.0;
          basis_row_load<KM>(phi + (size_t)(r0 + lc) * nev, 1, m, raw[u]);
        }
#pragma unroll
        for (int u = 0; u < GU; ++u)
#pragma unroll
          for (int q = 0; q < KM; ++q) acc[q] = fma(basis_coef<KM>(raw[u], q, m), x[u], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < KM; ++q)
        if (q < m) sh[g][q][k] = acc[q];
    });
  __syncthreads();
  if ((int)threadIdx.x < m * EIGP) {
    const int q = threadIdx.x / EIGP, kk = threadIdx.x % EIGP;
    double s = 0.0;
    for (int gg = 0; gg < RGS; ++gg) s += sh[gg][q][kk];
    if (kk < nr) c[(size_t)kk * ncp + p.coff[i] + q] = s;
  }
}

// XN[vp_i + nat(l)][k] = Y[vp_i + l][k] + sum_q phi_i[l][q] t_k[coff_i + q]
// (without the coarse part when t is null; without the local part when Y is).
// The region's coarse values are staged in LDS; thread per row.
template <typename TB>
__global__ void __launch_bounds__(WG) k_prolong_multi(Plan p, int nr, size_t ncp,
                                                      const TB *__restrict__ phi,
                                                      const double *__restrict__ t,
                                                      const double *__restrict__ Y,
                                                      double *__restrict__ XN) {
  __shared__ double tl[MAXNEV][EIGP];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0, m = p.mi[i], nev = p.nev;
  const size_t v0 = p.vp_ptr[i];
  const int co = p.coff[i];
  if (t && (int)threadIdx.x < MAXNEV * EIGP) {
    const int q = threadIdx.x / EIGP, k = threadIdx.x % EIGP;
    tl[q][k] = (q < m && k < nr) ? t[(size_t)k * ncp + co + q] : 0.0;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < ni; l += WG) {
    double v[EIGP];
    if (Y) {
      const double2 *src = reinterpret_cast<const double2 *>(Y + (v0 + l) * EIGP);
#pragma unroll
      for (int k = 0; k < EIGP / 2; ++k) {
        const double2 y = src[k];
        v[2 * k] = y.x;
        v[2 * k + 1] = y.y;
      }
    } else {
#pragma unroll
      for (int k = 0; k < EIGP; ++k) v[k] = 0.0;
    }
    if (t && m > 0)
      with_km(nev, [&](auto km) __attribute__((always_inline)) {
        constexpr int KM = decltype(km)::value;
        TB raw[KM];
        basis_row_load<KM>(phi + (size_t)(r0 + l) * nev, 1, m, raw);
#pragma unroll
        for (int q = 0; q < KM; ++q)
          if (q < m) {  // the loads above are already in flight
            const double a = basis_coef<KM>(raw, q, m);
#pragma unroll
            for (int k = 0; k < EIGP; ++k) v[k] = fma(a, tl[q][k], v[k]);
          }
      });
#pragma unroll
    for (int k = 0; k < EIGP; ++k)
      if (k >= nr) v[k] = 0.0;
    double2 *dst = reinterpret_cast<double2 *>(XN + (v0 + p.nat[r0 + l]) * EIGP);
#pragma unroll
    for (int k = 0; k < EIGP / 2; ++k) dst[k] = make_double2(v[2 * k], v[2 * k + 1]);
  }
}

// z_k[j] = sum over the copies of dof j (fixed map order) of XN[copy][k];
// thread per dof, the copies' rows read whole, each column written coalesced.
__global__ void __launch_bounds__(WG) k_scatter_multi(int n, int nr, const int *__restrict__ inv_ptr,
                                                      const int *__restrict__ ix,
                                                      const double *__restrict__ XN,
                                                      double *__restrict__ z) {
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= n) return;
  double s[EIGP];
#pragma unroll
  for (int k = 0; k < EIGP; ++k) s[k] = 0.0;
  for (int e = inv_ptr[j]; e < inv_ptr[j + 1]; ++e) {
    const double2 *row = reinterpret_cast<const double2 *>(XN + (size_t)ix[e] * EIGP);
#pragma unroll
    for (int k = 0; k < EIGP / 2; ++k) {
      const double2 x = row[k];
      s[2 * k] += x.x;
      s[2 * k + 1] += x.y;
    }
  }
#pragma unroll
  for (int k = 0; k < EIGP; ++k)
    if (k < nr) z[(size_t)k * n + j] = s[k];
}

// Coarse solve of every column: the product with the tiles of W0 (or W0^T)
// for all columns at once, so W0 is read once.  Workgroup per lower tile
// (I, J); the input block (64 rows x EIGP columns of tile K = J, or I
// transposed) is staged in LDS; part[(O * T0 + K)][row][k] holds the tile's
// contribution to output tile O (I, or J transposed).
template <typename T>
__global__ void __launch_bounds__(WG) k_trmm_tiles(const T *__restrict__ Wt, int T0,
                                                   const double *__restrict__ x, size_t ncp, int nr,
                                                   double *__restrict__ part, int transpose) {
  __shared__ double xs[TS][EIGP];
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;  // J <= I
  const T *w = Wt + ((size_t)I * T0 + J) * TE;
  const int K = transpose ? I : J, O = transpose ? J : I;
  for (int e = threadIdx.x; e < TS * EIGP; e += WG) {
    const int rr = e / EIGP, k = e % EIGP;
    xs[rr][k] = k < nr ? x[(size_t)k * ncp + K * TS + rr] : 0.0;
  }
  __syncthreads();
  const int o = threadIdx.x % TS, kq = threadIdx.x / TS;  // output row o, columns 4kq..4kq+3
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int c = 0; c < TS; ++c) {
    const double wv = transpose ? (double)w[c * TS + o] : (double)w[o * TS + c];
    a0 = fma(wv, xs[c][4 * kq], a0);
    a1 = fma(wv, xs[c][4 * kq + 1], a1);
    a2 = fma(wv, xs[c][4 * kq + 2], a2);
    a3 = fma(wv, xs[c][4 * kq + 3], a3);
  }
  double *dst = part + (((size_t)O * T0 + K) * TS + o) * EIGP + 4 * kq;
  dst[0] = a0;
  dst[1] = a1;
  dst[2] = a2;
  dst[3] = a3;
}

// y_k[O*64 + r] = sum over input tiles K (in order) of part[(O*T0 + K)][r][k]
__global__ void __launch_bounds__(TS * EIGP) k_trmm_reduce(int T0, const double *__restrict__ part,
                                                           double *__restrict__ y, size_t ncp,
                                                           int nr, int transpose) {
  const int O = blockIdx.x, r = threadIdx.x / EIGP, k = threadIdx.x % EIGP;
  const int k0 = transpose ? O : 0, k1 = transpose ? T0 : O + 1;
  double s = 0.0;
#pragma unroll 4
  for (int K = k0; K < k1; ++K) s += part[(((size_t)O * T0 + K) * TS + r) * EIGP + k];
  if (k < nr) y[(size_t)k * ncp + O * TS + r] = s;
}

// The mixed forms keep their f32 factor only as the two per-sweep streams;
// the block solve reads packed diagonal tiles and the envelope (row and
// column forms).  One workgroup per tile row g copies them back out: the
// forward block of g is [row-form segments | padding | diagonal tile], the
// backward block [column-form segments | padding | diagonal tile].
__global__ void __launch_bounds__(WG) k_streams_to_env(Plan p, const float *__restrict__ fst,
                                                       const float *__restrict__ bst,
                                                       float *__restrict__ dg,
                                                       float *__restrict__ er,
                                                       float *__restrict__ ec) {
  const int g = blockIdx.x;
  const int i = find_segment(p.trow_ptr, p.N, g);
  const int I = g - p.trow_ptr[i], r0 = I * TS;
  const int *ep = p.eptr + p.vp_ptr[i] + i, *up = p.uptr + p.vp_ptr[i] + i;
  const long long eb = p.ebase[i];
  {
    const float *blk = fst + p.sfr[i] + p.sfb[g];
    const int base = ep[r0], T = ep[r0 + TS] - base, Tp = (T + 3) & ~3;
    for (int k = threadIdx.x; k < T; k += WG) er[eb + base + k] = blk[k];
    for (int e = threadIdx.x; e < DE; e += WG) dg[(size_t)g * DE + e] = blk[Tp + e];
  }
  {
    const float *blk = bst + p.sbr[i] + p.sbb[g];
    const int base = up[r0], T = up[r0 + TS] - base;
    for (int k = threadIdx.x; k < T; k += WG) ec[eb + base + k] = blk[k];
  }
}

// ------------------------------------------ CG on several columns at once ---
// Independent CG recurrences, one per column, that share every operator
// application.  Columns are ld apart; per-column scalars come from device
// arrays (alpha, beta); converged columns carry alpha = beta = 0.

// Y_k = A X_k for k < nr on the sliced copy of A: a row's entries are
// loaded once and used for every column.
__global__ void __launch_bounds__(WG) k_spmm_sell(int n, const long long *__restrict__ sptr,
                                                  const int *__restrict__ scol,
                                                  const double *__restrict__ sval, size_t ld,
                                                  int nr, const double *__restrict__ X,
                                                  double *__restrict__ Y) {
  constexpr int JU = 8;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const int sl = i >> 6, lane = i & 63;
  const long long base = sptr[sl];
  const int wd = (int)((sptr[sl + 1] - base) >> 6);
  int c[JU];
  double v[JU];
#pragma unroll
  for (int j = 0; j < JU; ++j) {
    const bool in = j < wd;
    const long long e = base + (long long)j * 64 + lane;
    c[j] = in ? scol[e] : i;
    v[j] = in ? sval[e] : 0.0;
  }
  for (int k = 0; k < nr; ++k) {
    const double *x = X + (size_t)k * ld;
    // every slot's x is loaded (c[j] is a valid row for the slots past the
    // slice width), and those slots are dropped by a select, so that the
    // loads are in flight together
    double xv[JU];
#pragma unroll
    for (int j = 0; j < JU; ++j) xv[j] = x[c[j]];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < JU; ++j) {
      const double t = fma(v[j], xv[j], s);
      s = j < wd ? t : s;
    }
    for (int j = JU; j < wd; ++j) {
      const long long e = base + (long long)j * 64 + lane;
      s = fma(sval[e], x[scol[e]], s);
    }
    Y[(size_t)k * ld + i] = s;
  }
}

// part[k * gridDim.x + b] = sum over rows of block-stride b of A_k . B_k
__global__ void __launch_bounds__(WG) k_col_dots(int n, size_t ld, int nr,
                                                 const double *__restrict__ A,
                                                 const double *__restrict__ B,
                                                 double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  const int k = blockIdx.y;
  if (k >= nr) return;  // uniform over the workgroup
  const double *a = A + (size_t)k * ld, *b = B + (size_t)k * ld;
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) acc = fma(a[i], b[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = t;
}

// x_k += alpha_k p_k, r_k -= alpha_k q_k, partial sums of r_k . r_k
__global__ void __launch_bounds__(WG) k_col_update(int n, size_t ld, int nr,
                                                   const double *__restrict__ alpha,
                                                   const double *__restrict__ P,
                                                   const double *__restrict__ Q,
                                                   double *__restrict__ X,
                                                   double *__restrict__ R,
                                                   double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  const int k = blockIdx.y;
  if (k >= nr) return;
  const double a = alpha[k];
  const size_t o = (size_t)k * ld;
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    X[o + i] = fma(a, P[o + i], X[o + i]);
    const double ri = fma(-a, Q[o + i], R[o + i]);
    R[o + i] = ri;
    acc = fma(ri, ri, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = t;
}

// p_k = z_k + beta_k p_k
__global__ void __launch_bounds__(WG) k_col_direction(int n, size_t ld, int nr,
                                                      const double *__restrict__ beta,
                                                      const double *__restrict__ Z,
                                                      double *__restrict__ P) {
  const int k = blockIdx.y;
  if (k >= nr) return;
  const double b = beta[k];
  const size_t o = (size_t)k * ld;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG)
    P[o + i] = fma(b, P[o + i], Z[o + i]);
}

// out[k] = sum of part[k * nb .. k * nb + nb) in a fixed order
__global__ void __launch_bounds__(WG) k_col_reduce(int nb, const double *__restrict__ part,
                                                   double *__restrict__ out) {
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += WG) acc += part[(size_t)blockIdx.x * nb + b];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// ------------------------------------------------------------- launchers ---
void launch_streams_to_env(hipStream_t s, const Plan &p, int ntilerows, const float *fst,
                           const float *bst, float *dg, float *er, float *ec) {
  if (ntilerows <= 0) return;
  hipLaunchKernelGGL(k_streams_to_env, dim3(ntilerows), dim3(WG), 0, s, p, fst, bst, dg, er, ec);
}

void launch_gather_multi(hipStream_t s, const Plan &p, int n, int nr, const double *r, double *X) {
  hipLaunchKernelGGL(k_gather_multi, dim3(p.N), dim3(WG), 0, s, p, n, nr, r, X);
}

template <typename TB>
void launch_restrict_multi(hipStream_t s, const Plan &p, int nr, size_t ncp, const TB *phi,
                           const double *X, double *c) {
  hipLaunchKernelGGL((k_restrict_multi<TB>), dim3(p.N), dim3(WG), 0, s, p, nr, ncp, phi, X, c);
}

template <typename TB>
void launch_prolong_multi(hipStream_t s, const Plan &p, int nr, size_t ncp, const TB *phi,
                          const double *t, const double *Y, double *XN) {
  hipLaunchKernelGGL((k_prolong_multi<TB>), dim3(p.N), dim3(WG), 0, s, p, nr, ncp, phi, t, Y, XN);
}

void launch_scatter_multi(hipStream_t s, int n, int nr, const int *inv_ptr, const int *ix,
                          const double *XN, double *z) {
  const unsigned b = (unsigned)(((long long)n + WG - 1) / WG);
  if (b == 0) return;
  hipLaunchKernelGGL(k_scatter_multi, dim3(b), dim3(WG), 0, s, n, nr, inv_ptr, ix, XN, z);
}

template <typename T>
void launch_trmm(hipStream_t s, const T *Wt, int T0, const double *x, size_t ncp, int nr,
                 double *part, double *y, int transpose) {
  const int nb = T0 * (T0 + 1) / 2;
  if (nb == 0) return;
  hipLaunchKernelGGL((k_trmm_tiles<T>), dim3(nb), dim3(WG), 0, s, Wt, T0, x, ncp, nr, part,
                     transpose);
  hipLaunchKernelGGL(k_trmm_reduce, dim3(T0), dim3(TS * EIGP), 0, s, T0, part, y, ncp, nr,
                     transpose);
}
template void launch_trmm<double>(hipStream_t, const double *, int, const double *, size_t, int,
                                  double *, double *, int);
template void launch_trmm<float>(hipStream_t, const float *, int, const double *, size_t, int,
                                 double *, double *, int);

static int col_blocks(int n) {
  int b = (n + WG - 1) / WG;
  return b > 256 ? 256 : (b < 1 ? 1 : b);
}

void launch_spmm_sell(hipStream_t s, int n, const long long *sptr, const int *scol,
                      const double *sval, size_t ld, int nr, const double *X, double *Y) {
  const unsigned b = (unsigned)(((long long)n + WG - 1) / WG);
  if (b == 0 || nr <= 0) return;
  hipLaunchKernelGGL(k_spmm_sell, dim3(b), dim3(WG), 0, s, n, sptr, scol, sval, ld, nr, X, Y);
}

void launch_col_dots(hipStream_t s, int n, size_t ld, int nr, const double *A, const double *B,
                     double *part, double *out) {
  const int nb = col_blocks(n);
  hipLaunchKernelGGL(k_col_dots, dim3(nb, nr), dim3(WG), 0, s, n, ld, nr, A, B, part);
  hipLaunchKernelGGL(k_col_reduce, dim3(nr), dim3(WG), 0, s, nb, part, out);
}

void launch_col_update(hipStream_t s, int n, size_t ld, int nr, const double *alpha,
                       const double *P, const double *Q, double *X, double *R, double *part,
                       double *rr) {
  const int nb = col_blocks(n);
  hipLaunchKernelGGL(k_col_update, dim3(nb, nr), dim3(WG), 0, s, n, ld, nr, alpha, P, Q, X, R,
                     part);
  hipLaunchKernelGGL(k_col_reduce, dim3(nr), dim3(WG), 0, s, nb, part, rr);
}

__global__ void __launch_bounds__(64) k_col_alpha(int nr, ColCgState *cs,
                                                  const double *__restrict__ pq,
                                                  double *__restrict__ alpha) {
  const int k = threadIdx.x;
  if (k >= nr) return;
  double c = 0.0;
  bool brk = false;
  if (cs->active[k]) {
    const double q = cs->rz[k] / pq[k];
    if (!(pq[k] > 0.0) || !isfinite(q)) {
      brk = true;
      cs->active[k] = 0;
    } else {
      c = q;
    }
  }
  alpha[k] = c;
  const unsigned long long m = __ballot(brk);
  if (k == 0 && m) cs->breakdown |= (int)m;
}

__global__ void __launch_bounds__(64) k_col_beta(int nr, ColCgState *cs,
                                                 const double *__restrict__ rr,
                                                 const double *__restrict__ rz, double rtol2,
                                                 double *__restrict__ beta) {
  const int k = threadIdx.x;
  int act = 0;
  bool brk = false;
  if (k < nr) {
    double c = 0.0;
    cs->rr[k] = rr[k];
    if (cs->active[k]) {
      cs->its[k] += 1;
      if (!isfinite(rr[k])) {
        brk = true;
        cs->active[k] = 0;
      } else if (rr[k] <= rtol2 * cs->f2[k]) {
        cs->active[k] = 0;
      } else {
        c = rz[k] / cs->rz[k];
        cs->rz[k] = rz[k];
      }
    }
    beta[k] = c;
    act = cs->active[k];
  }
  const unsigned long long m = __ballot(act != 0), bm = __ballot(brk);
  if (k == 0) {
    cs->nact = __popcll(m);
    if (bm) cs->breakdown |= (int)bm;
  }
}

void launch_col_alpha(hipStream_t s, int nr, ColCgState *cs, const double *pq, double *alpha) {
  hipLaunchKernelGGL(k_col_alpha, dim3(1), dim3(64), 0, s, nr, cs, pq, alpha);
}

void launch_col_beta(hipStream_t s, int nr, ColCgState *cs, const double *rr, const double *rz,
                     double rtol2, double *beta) {
  hipLaunchKernelGGL(k_col_beta, dim3(1), dim3(64), 0, s, nr, cs, rr, rz, rtol2, beta);
}

void launch_col_direction(hipStream_t s, int n, size_t ld, int nr, const double *beta,
                          const double *Z, double *P) {
  hipLaunchKernelGGL(k_col_direction, dim3(col_blocks(n), nr), dim3(WG), 0, s, n, ld, nr, beta, Z, P);
}

#define AMSP_MULTI_INST(TB)                                                                  \
  template void launch_restrict_multi<TB>(hipStream_t, const Plan &, int, size_t, const TB *, \
                                          const double *, double *);                          \
  template void launch_prolong_multi<TB>(hipStream_t, const Plan &, int, size_t, const TB *,  \
                                         const double *, const double *, double *);
AMSP_MULTI_INST(double)
AMSP_MULTI_INST(float)
AMSP_MULTI_INST(__hip_bfloat16)
#undef AMSP_MULTI_INST

}  // namespace amsp
