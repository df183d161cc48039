// Sparse coarse factorisation, numeric phase (see amsp_tree.h): multifrontal
// Cholesky of A0 = R0 A R0^T over a nested-dissection tree of supernodes, and
// the coarse solve through it.
//
// A front of T x T tiles (64x64, row-major inside a tile) keeps only its
// lower tiles, packed: tile (I, J), J <= I, at fbase + I(I+1)/2 + J.  Its
// first K tile rows are its own coarse dofs, the rest its update dofs.  The
// right-looking tile Cholesky runs over the own columns k < K; afterwards the
// trailing tiles hold the Schur complement that the parent adds in.
// X (T x K tiles, full) is formed by a right-looking solve of
// [L11 0; L21 I] X = [I; 0], so X = [inv(L11); -L21 inv(L11)].
// Kernels of one step take a 2D grid: y = front (inside a level's range), x =
// work item of that front; items past a front's work return at once.
#include "amsp_tree.h"
#include "k_common.h"

namespace amsp {

__device__ __forceinline__ double *ftile(double *F, const TreeDev &t, int f, int I, int J) {
  return F + ((size_t)t.fbase[f] + (size_t)I * (I + 1) / 2 + J) * TE;
}
__device__ __forceinline__ const double *ftile(const double *F, const TreeDev &t, int f, int I,
                                               int J) {
  return F + ((size_t)t.fbase[f] + (size_t)I * (I + 1) / 2 + J) * TE;
}
__device__ __forceinline__ double &fentry(double *F, const TreeDev &t, int f, int R, int C) {
  return ftile(F, t, f, R >> 6, C >> 6)[(R & 63) * TS + (C & 63)];
}
template <typename T>
__device__ __forceinline__ T *xtile(T *X, const TreeDev &t, int f, int I, int J) {
  return X + ((size_t)t.xbase[f] + (size_t)I * t.K[f] + J) * TE;
}

// (ii, jj), jj <= ii, of packed lower-triangle index b
__device__ __forceinline__ void tri_index(int b, int &ii, int &jj) {
  ii = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= b) ++ii;
  while (ii * (ii + 1) / 2 > b) --ii;
  jj = b - ii * (ii + 1) / 2;
}

// ------------------------------------------------------------ assembly ---
// Block (i, j) of A0 for every coupled pair: Phi_i^T (A Phi_j) summed over the
// pair's overlap list in fixed segments, into pb[pair][a][b] (nev x nev).
__global__ void __launch_bounds__(WG) k_pair_blocks(Plan p, CoarsePlan c,
                                                    const double *__restrict__ phi,
                                                    const double *__restrict__ W,
                                                    double *__restrict__ pb) {
  const int pr = blockIdx.x;
  const int i = c.pair_i[pr], j = c.pair_j[pr];
  const int nev = p.nev, nn = nev * nev, nseg = WG / nn;
  const int mi = p.mi[i], mj = p.mi[j];
  __shared__ double part[WG];
  const int t = threadIdx.x, ab = t % nn, seg = t / nn;
  const int a = ab / nev, b = ab % nev;
  double s = 0.0;
  if (seg < nseg && a < mi && b < mj) {
    const int q0 = c.pair_ptr[pr], len = c.pair_ptr[pr + 1] - q0;
    const int s0 = q0 + (int)(((long long)len * seg) / nseg);
    const int s1 = q0 + (int)(((long long)len * (seg + 1)) / nseg);
    const int ri = p.sd_ptr[i];
    for (int q = s0; q < s1; ++q)
      s = fma(phi[(size_t)(ri + c.pair_l[q]) * nev + a],
              W[(size_t)(c.ext_ptr[j] + c.pair_e[q]) * nev + b], s);
  }
  part[t] = s;
  __syncthreads();
  if (t < nn) {
    double tot = 0.0;
    for (int g = 0; g < nseg; ++g) tot += part[g * nn + t];
    pb[(size_t)pr * nn + t] = (a < mi && b < mj) ? tot : 0.0;
  }
}

// Unit diagonal on the own padding rows of every front and the identity in
// X's own diagonal tiles (F and X zero-filled before).
__global__ void __launch_bounds__(WG) k_tree_diag_init(TreeDev t, double *__restrict__ F,
                                                       double *__restrict__ X) {
  const int f = blockIdx.x;
  const int K = t.K[f], kd = t.kdof[f];
  for (int r = threadIdx.x; r < K * TS; r += WG) {
    if (r >= kd) fentry(F, t, f, r, r) = 1.0;
    xtile(X, t, f, r >> 6, r >> 6)[(r & 63) * TS + (r & 63)] = 1.0;
  }
}

// Lower entries of the pair blocks that land in fronts, symmetrised:
// 0.5 (B_ij[a][b] + B_ji[b][a]).
__global__ void __launch_bounds__(WG) k_tree_assemble(Plan p, TreeDev t,
                                                      const double *__restrict__ pb,
                                                      double *__restrict__ F) {
  const int e = blockIdx.x;
  const int pr = t.as_pair[e], rv = t.as_rev[e], f = t.as_front[e];
  const int i = t.pair_i[pr], j = t.pair_j[pr];
  const int nev = p.nev, nn = nev * nev;
  const int a = threadIdx.x / nev, b = threadIdx.x % nev;
  if ((int)threadIdx.x >= nn || a >= p.mi[i] || b >= p.mi[j]) return;
  const int R = t.as_ri[e] + a, C = t.as_rj[e] + b;
  if (R < C) return;  // diagonal block: its upper half is the transpose
  fentry(F, t, f, R, C) = 0.5 * (pb[(size_t)pr * nn + a * nev + b] + pb[(size_t)rv * nn + b * nev + a]);
}

// Children's Schur complements into their parents: one workgroup per lower
// tile of a child's update block; each child of the launch has its own
// parent, and a child's update rows map to distinct parent rows (increasing),
// so no two workgroups add into the same entry.
__global__ void __launch_bounds__(WG) k_tree_extend_add(TreeDev t, const int *__restrict__ children,
                                                        double *__restrict__ F) {
  const int c = children[blockIdx.y];
  const int Kc = t.K[c], U = t.T[c] - Kc, ud = t.udof[c];
  const int b = blockIdx.x;
  if (b >= U * (U + 1) / 2) return;
  int ii, jj;
  tri_index(b, ii, jj);
  const double *src = ftile(F, t, c, Kc + ii, Kc + jj);
  const int pf = t.parent[c];
  const int *ea = t.ea_row + t.vbase[c];
  for (int e = threadIdx.x; e < TE; e += WG) {
    const int r = e >> 6, cc = e & 63;
    const int t1 = TS * ii + r, t2 = TS * jj + cc;
    if (t1 >= ud || t2 >= ud || (ii == jj && cc > r)) continue;
    fentry(F, t, pf, ea[t1], ea[t2]) += src[e];
  }
}

// --------------------------------------------------- factor, step k -------
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_tree_potrf(TreeDev t, int f0, int k, double *F, double *dinv, int *status) {
  extern __shared__ double lds[];
  double *A = lds, *Y = lds + TS * LDT;
  __shared__ int fail;
  const int f = f0 + blockIdx.y;
  if (k >= t.K[f]) return;
  if (threadIdx.x == 0) fail = 0;
  double *a = ftile(F, t, f, k, k);
  tile_to_lds(a, A);
  __syncthreads();
  lds_potrf_trtri<32>(A, Y, &fail);
  lds_to_tile(A, a);
  lds_to_tile(Y, dinv + (size_t)(t.dbase[f] + k) * TE);
  __syncthreads();
  if (threadIdx.x == 0 && fail) atomicOr(status, 1);
}

// L_ik = A_ik inv(L_kk)^T, k < i < T (in place: each wavefront reads only
// its own rows of A_ik before writing them)
__global__ void __launch_bounds__(WG) k_tree_trsm(TreeDev t, int f0, int k, double *F,
                                                  const double *dinv) {
  const int f = f0 + blockIdx.y, i = k + 1 + blockIdx.x;
  if (k >= t.K[f] || i >= t.T[f]) return;
  double *a = ftile(F, t, f, i, k);
  Acc4 o;
  acc_zero(o);
  acc_mma_abt(o, a, TS, dinv + (size_t)(t.dbase[f] + k) * TE, TS, 1.0);
  acc_store(o, a);
}

// A_ij -= L_ik L_jk^T, k < j <= i < T
__global__ void __launch_bounds__(WG) k_tree_syrk(TreeDev t, int f0, int k, double *F) {
  const int f = f0 + blockIdx.y;
  const int T = t.T[f];
  if (k >= t.K[f]) return;
  const int m = T - k - 1;
  if ((int)blockIdx.x >= m * (m + 1) / 2) return;
  int ii, jj;
  tri_index(blockIdx.x, ii, jj);
  const int i = k + 1 + ii, j = k + 1 + jj;
  __shared__ double Ly[TS * LDT];  // every wavefront multiplies by the whole L_jk
  tile_to_lds(ftile(F, t, f, j, k), Ly);
  double *c = ftile(F, t, f, i, j);
  Acc4 o;
  acc_load(o, c);
  __syncthreads();
  acc_mma_abt(o, ftile(F, t, f, i, k), TS, Ly, LDT, -1.0);
  acc_store(o, c);
}

// X_kj <- inv(L_kk) X_kj, j <= k
__global__ void __launch_bounds__(WG) k_tree_inv_row(TreeDev t, int f0, int k, double *X,
                                                     const double *dinv) {
  extern __shared__ double lds[];
  const int f = f0 + blockIdx.y, j = blockIdx.x;
  if (k >= t.K[f] || j > k) return;
  double *w = xtile(X, t, f, k, j);
  tile_to_lds(w, lds);
  __syncthreads();
  Acc4 o;
  acc_zero(o);
  acc_mma_ab(o, dinv + (size_t)(t.dbase[f] + k) * TE, TS, lds, LDT, 1.0);
  acc_store(o, w);
}

// X_ij -= L_ik X_kj, k < i < T, j <= k
__global__ void __launch_bounds__(WG) k_tree_inv_update(TreeDev t, int f0, int k,
                                                        const double *F, double *X) {
  const int f = f0 + blockIdx.y;
  if (k >= t.K[f]) return;
  const int i = k + 1 + (int)blockIdx.x / (k + 1), j = (int)blockIdx.x % (k + 1);
  if (i >= t.T[f]) return;
  __shared__ double Xk[TS * LDT];
  tile_to_lds(xtile(X, t, f, k, j), Xk);
  double *c = xtile(X, t, f, i, j);
  Acc4 o;
  acc_load(o, c);
  __syncthreads();
  acc_mma_ab(o, ftile(F, t, f, i, k), TS, Xk, LDT, -1.0);
  acc_store(o, c);
}

__global__ void k_x_to_f32(const double *__restrict__ src, float *__restrict__ dst, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// ----------------------------------------------------------- the solve ---
// Forward, one level: workgroup (front f, row tile I) forms the front's own
// input cs = c + the children's contributions, then rows 64I.. of X cs:
// own rows give y (by coarse index), update rows give the front's update
// vector v_f = (X cs) + the children's contributions to those rows.
template <typename TX>
__global__ void __launch_bounds__(WG) k_tree_fwd(TreeDev t, int f0, const TX *__restrict__ X,
                                                 const double *__restrict__ c,
                                                 double *__restrict__ y, double *__restrict__ v,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ double cs[];  // 64 K
  const int f = f0 + blockIdx.y, I = blockIdx.x;
  const int K = t.K[f];
  if (I >= t.T[f]) return;
  const int rb = t.rbase[f];
  for (int r = threadIdx.x; r < K * TS; r += WG) {
    const int rc = t.row_coarse[rb + r];
    double s = rc >= 0 ? c[rc] : 0.0;
    for (int g = t.gptr[rb + r]; g < t.gptr[rb + r + 1]; ++g) s += v[t.gsrc[g]];
    cs[r] = s;
  }
  __syncthreads();
  const int row = threadIdx.x >> 2, q = threadIdx.x & 3;
  const int jn = I < K ? I + 1 : K;  // inv(L11) is lower triangular
  double s = 0.0;
  for (int J = 0; J < jn; ++J) {
    const TX *x = xtile(X, t, f, I, J) + row * TS + 16 * q;
    const double *cc = cs + J * TS + 16 * q;
#pragma unroll
    for (int e = 0; e < 16; ++e) s = fma((double)x[e], cc[e], s);
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (q != 0) return;
  const int R = I * TS + row;
  if (I < K) {
    const int rc = t.row_coarse[rb + R];
    if (rc >= 0) y[rc] = s;
  } else {
    const int u = R - K * TS;
    if (u < t.udof[f]) {
      for (int g = t.gptr[rb + R]; g < t.gptr[rb + R + 1]; ++g) s += v[t.gsrc[g]];
      v[t.vbase[f] + u] = s;
    }
  }
}

// Backward, one level: workgroup (front f, column tile J) forms
// z = [y on the own rows; x on the update rows (ancestors, solved)] and
// x[own rows 64J..] = (X^T z) restricted to those columns.
template <typename TX>
__global__ void __launch_bounds__(WG) k_tree_bwd(TreeDev t, int f0, const TX *__restrict__ X,
                                                 const double *__restrict__ y,
                                                 double *__restrict__ x,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ double z[];  // 64 T
  __shared__ double red[4][TS];
  const int f = f0 + blockIdx.y, J = blockIdx.x;
  const int K = t.K[f], T = t.T[f];
  if (J >= K) return;
  const int rb = t.rbase[f];
  for (int r = J * TS + threadIdx.x; r < T * TS; r += WG) {
    const int rc = t.row_coarse[rb + r];
    z[r] = rc < 0 ? 0.0 : (r < K * TS ? y[rc] : x[rc]);
  }
  __syncthreads();
  const int col = threadIdx.x & 63, g = threadIdx.x >> 6;
  double s = 0.0;
  for (int I = J; I < T; ++I) {
    const TX *xt = xtile(X, t, f, I, J) + (16 * g) * TS + col;
    const double *zz = z + I * TS + 16 * g;
#pragma unroll
    for (int r = 0; r < 16; ++r) s = fma((double)xt[r * TS], zz[r], s);
  }
  red[g][col] = s;
  __syncthreads();
  if (g == 0) {
    const int rc = t.row_coarse[rb + J * TS + col];
    if (rc >= 0) x[rc] = (red[0][col] + red[1][col]) + (red[2][col] + red[3][col]);
  }
}

// ------------------------------------------------------------- launchers ---
static size_t two_tiles() { return (size_t)(2 * TS * LDT) * sizeof(double); }
static size_t one_tile() { return (size_t)(TS * LDT) * sizeof(double); }

void launch_pair_blocks(hipStream_t s, const Plan &p, const CoarsePlan &c, const double *phi,
                        const double *W, double *pb) {
  if (c.npairs == 0) return;
  hipLaunchKernelGGL(k_pair_blocks, dim3(c.npairs), dim3(WG), 0, s, p, c, phi, W, pb);
}

void launch_tree_init(hipStream_t s, const TreeDev &t, int nfront, int, double *F, double *X) {
  if (nfront == 0) return;
  hipLaunchKernelGGL(k_tree_diag_init, dim3(nfront), dim3(WG), 0, s, t, F, X);
}

void launch_tree_assemble(hipStream_t s, const Plan &p, const TreeDev &t, int nas, const double *pb,
                          double *F) {
  if (nas == 0) return;
  hipLaunchKernelGGL(k_tree_assemble, dim3(nas), dim3(WG), 0, s, p, t, pb, F);
}

void launch_tree_extend_add(hipStream_t s, const TreeDev &t, const int *children, int nchild,
                            int maxU, double *F) {
  if (nchild == 0 || maxU == 0) return;
  hipLaunchKernelGGL(k_tree_extend_add, dim3(maxU, nchild), dim3(WG), 0, s, t, children, F);
}

void launch_tree_factor_step(hipStream_t s, const TreeDev &t, int f0, int f1, int maxT, int k,
                             double *F, double *dinv, int *status) {
  const int nf = f1 - f0, m = maxT - k - 1;
  if (nf <= 0) return;
  allow_lds(k_tree_potrf, two_tiles());
  hipLaunchKernelGGL(k_tree_potrf, dim3(1, nf), dim3(WG), two_tiles(), s, t, f0, k, F, dinv, status);
  if (m <= 0) return;
  hipLaunchKernelGGL(k_tree_trsm, dim3(m, nf), dim3(WG), 0, s, t, f0, k, F, dinv);
  hipLaunchKernelGGL(k_tree_syrk, dim3(m * (m + 1) / 2, nf), dim3(WG), 0, s, t, f0, k, F);
}

void launch_tree_inverse_step(hipStream_t s, const TreeDev &t, int f0, int f1, int maxT, int k,
                              const double *F, const double *dinv, double *X) {
  const int nf = f1 - f0, m = maxT - k - 1;
  if (nf <= 0) return;
  hipLaunchKernelGGL(k_tree_inv_row, dim3(k + 1, nf), dim3(WG), one_tile(), s, t, f0, k, X, dinv);
  if (m <= 0) return;
  hipLaunchKernelGGL(k_tree_inv_update, dim3(m * (k + 1), nf), dim3(WG), 0, s, t, f0, k, F, X);
}

void launch_tree_x_to_f32(hipStream_t s, const double *X, float *Xf, long long ntiles) {
  const size_t n = (size_t)ntiles * TE;
  if (n == 0) return;
  size_t b = (n + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_x_to_f32, dim3((unsigned)b), dim3(WG), 0, s, X, Xf, n);
}

template <typename TX>
void launch_tree_solve(hipStream_t s, const TreeDev &t, const std::vector<int> &lvl_ptr,
                       const std::vector<int> &lvl_maxT, const std::vector<int> &lvl_maxK,
                       int maxK, int maxT, const TX *X, const double *c, double *y, double *v,
                       double *x, const int *done) {
  const int nl = (int)lvl_ptr.size() - 1;
  allow_lds(k_tree_fwd<TX>, (size_t)maxK * TS * sizeof(double));
  allow_lds(k_tree_bwd<TX>, (size_t)maxT * TS * sizeof(double));
  for (int h = 0; h < nl; ++h) {
    const int f0 = lvl_ptr[h], nf = lvl_ptr[h + 1] - f0;
    hipLaunchKernelGGL((k_tree_fwd<TX>), dim3(lvl_maxT[h], nf), dim3(WG),
                       (size_t)lvl_maxK[h] * TS * sizeof(double), s, t, f0, X, c, y, v, done);
  }
  for (int h = nl - 1; h >= 0; --h) {
    const int f0 = lvl_ptr[h], nf = lvl_ptr[h + 1] - f0;
    hipLaunchKernelGGL((k_tree_bwd<TX>), dim3(lvl_maxK[h], nf), dim3(WG),
                       (size_t)lvl_maxT[h] * TS * sizeof(double), s, t, f0, X, y, x, done);
  }
}
template void launch_tree_solve<double>(hipStream_t, const TreeDev &, const std::vector<int> &,
                                        const std::vector<int> &, const std::vector<int> &, int,
                                        int, const double *, const double *, double *, double *,
                                        double *, const int *);
template void launch_tree_solve<float>(hipStream_t, const TreeDev &, const std::vector<int> &,
                                       const std::vector<int> &, const std::vector<int> &, int, int,
                                       const float *, const double *, double *, double *, double *,
                                       const int *);

}  // namespace amsp
