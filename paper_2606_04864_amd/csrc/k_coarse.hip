// Coarse level: Galerkin matrix A0 = R0 A R0^T (Section 3.1), its tiled
// dense Cholesky factorisation A0 = L0 L0^T, the inverse factor W0 = inv(L0),
// and the coarse solve A0^{-1} c = W0^T (W0 c) as two fully parallel
// triangular matrix-vector products.
//
// A0 is stored as T0 x T0 row-major 64x64 tiles (tile (I,J) at (I*T0+J)*64*64);
// rows/columns past N_c are padding with a unit diagonal.
#include "k_common.h"

namespace amsp {

// W_j = A Phi_j on the extended region of subdomain j (region grown by one
// layer), one workgroup per subdomain.  Row stride of W and Phi: nev.
__global__ void __launch_bounds__(WG) k_apply_A_to_basis(Plan p, CoarsePlan c,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ phi,
                                                         double *__restrict__ W) {
  const int j = blockIdx.x;
  const int nev = p.nev, m = p.mi[j];
  const int e0 = c.ext_ptr[j], e1 = c.ext_ptr[j + 1];
  const int r0 = p.sd_ptr[j];
  for (int e = e0 + threadIdx.x; e < e1; e += WG) {
    if (m == 0) {
      for (int k = 0; k < nev; ++k) W[(size_t)e * nev + k] = 0.0;
      continue;
    }
    with_km(nev, [&](auto km) __attribute__((always_inline)) {
      constexpr int KM = decltype(km)::value;
      double acc[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) acc[k] = 0.0;
      for (int q = c.ext_rowptr[e]; q < c.ext_rowptr[e + 1]; ++q) {
        const double a = val[c.ext_src[q]];
        double raw[KM];
        basis_row_load<KM>(phi + (size_t)(r0 + c.ext_loc[q]) * nev, 1, m, raw);
#pragma unroll
        for (int k = 0; k < KM; ++k) acc[k] = fma(a, basis_coef<KM>(raw, k, m), acc[k]);
      }
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (k < nev) W[(size_t)e * nev + k] = (k < m) ? acc[k] : 0.0;
    });
  }
}

__device__ __forceinline__ size_t a0_index(int R, int C, int T0) {
  return ((size_t)(R >> 6) * T0 + (C >> 6)) * TE + (size_t)(R & 63) * TS + (C & 63);
}

// Block (i,j) of A0: Phi_i^T W_j summed over the overlap list of the pair.
// Thread t handles entry (a,b) = (t % (nev*nev)) and list segment t / (nev*nev);
// segments are combined in fixed order.
__global__ void __launch_bounds__(WG) k_pair_products(Plan p, CoarsePlan c,
                                                      const double *__restrict__ phi,
                                                      const double *__restrict__ W,
                                                      double *__restrict__ A0t, int T0) {
  const int pr = blockIdx.x;
  const int i = c.pair_i[pr], j = c.pair_j[pr];
  const int nev = p.nev;
  const int mi = p.mi[i], mj = p.mi[j];
  const int nn = nev * nev;
  const int nseg = WG / nn;
  __shared__ double part[WG];
  const int t = threadIdx.x;
  const int q0 = c.pair_ptr[pr], q1 = c.pair_ptr[pr + 1];
  double s = 0.0;
  const int ab = t % nn, seg = t / nn;
  const int a = ab / nev, b = ab % nev;
  if (seg < nseg && a < mi && b < mj) {
    const int len = q1 - q0;
    const int s0 = q0 + (int)(((long long)len * seg) / nseg);
    const int s1 = q0 + (int)(((long long)len * (seg + 1)) / nseg);
    const int ri = p.sd_ptr[i], ej = 0;
    (void)ej;
    for (int q = s0; q < s1; ++q) {
      s = fma(phi[(size_t)(ri + c.pair_l[q]) * nev + a], W[(size_t)(c.ext_ptr[j] + c.pair_e[q]) * nev + b], s);
    }
  }
  part[t] = s;
  __syncthreads();
  if (t < nn && a < mi && b < mj) {
    double tot = 0.0;
    for (int g = 0; g < nseg; ++g) tot += part[g * nn + t];
    A0t[a0_index(p.coff[i] + a, p.coff[j] + b, T0)] = tot;
  }
}

// Both triangles <- (A0 + A0^T)/2, padding diagonal <- 1.  One workgroup per
// lower tile pair (I, J), J <= I: tiles (I, J) and (J, I) go through LDS, so
// that every global access is a whole tile row.
__global__ void __launch_bounds__(WG) k_symmetrize(double *__restrict__ A0t, int T0, int nc) {
  __shared__ double X[TS * LDT], Y[TS * LDT];
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  double *xt = A0t + ((size_t)I * T0 + J) * TE, *yt = A0t + ((size_t)J * T0 + I) * TE;
  for (int e = threadIdx.x; e < TE; e += WG) {
    X[(e >> 6) * LDT + (e & 63)] = xt[e];
    Y[(e >> 6) * LDT + (e & 63)] = yt[e];
  }
  __syncthreads();
  // element (r, c) of tile (I, J) is A0[R][C], R = 64I + r, C = 64J + c; its
  // mirror A0[C][R] is element (c, r) of tile (J, I)
  for (int e = threadIdx.x; e < TE; e += WG) {
    const int r = e >> 6, c = e & 63, R = I * TS + r, C = J * TS + c;
    double v;
    if (R >= nc || C >= nc)
      v = R == C ? 1.0 : 0.0;
    else
      v = 0.5 * (X[r * LDT + c] + Y[c * LDT + r]);
    xt[e] = v;
    Y[c * LDT + r] = v;  // read above by this thread only
  }
  if (I == J) return;
  __syncthreads();
  for (int e = threadIdx.x; e < TE; e += WG) yt[e] = Y[(e >> 6) * LDT + (e & 63)];
}

// ------------------------------------- singular problems: A0 + alpha u u^T ---
// When A's null space is the constant vector (homogeneous Neumann problem),
// A0 = R0 A R0^T is singular along the c with R0^T c = 1.  The coarse term is
// applied with (A0 + alpha u u^T)^{-1}, u = R0 1: for any b = R0 r with
// 1.r = 0 this is A0^+ b plus a multiple of c, whose prolongation is a
// constant vector that A annihilates.
// u[coff_i + k] = sum over the region's rows of phi_i[:, k] (R0 1).
__global__ void __launch_bounds__(WG) k_basis_colsum(Plan p, const double *__restrict__ phi,
                                                     double *__restrict__ u) {
  __shared__ double sh[WG / 64];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0, m = p.mi[i], nev = p.nev;
  for (int k = 0; k < m; ++k) {  // uniform
    double acc = 0.0;
    for (int l = threadIdx.x; l < ni; l += WG) acc += phi[(size_t)(r0 + l) * nev + k];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) u[p.coff[i] + k] = t;
  }
}

// alpha = trace(A0) / u.u (so that alpha u u^T is on A0's scale); one workgroup
__global__ void __launch_bounds__(WG) k_rank1_scale(const double *__restrict__ A0t, int T0, int nc,
                                                    const double *__restrict__ u,
                                                    double *__restrict__ alpha) {
  __shared__ double sh[WG / 64];
  double tr = 0.0, uu = 0.0;
  for (int k = threadIdx.x; k < nc; k += WG) {
    tr += A0t[a0_index(k, k, T0)];
    uu = fma(u[k], u[k], uu);
  }
  tr = block_sum(tr, sh);
  uu = block_sum(uu, sh);
  if (threadIdx.x == 0) *alpha = uu > 0.0 ? tr / uu : 0.0;
}

// A0 += alpha u u^T on every stored tile (entries of the padding untouched)
__global__ void k_rank1_update(double *__restrict__ A0t, int T0, int nc,
                               const double *__restrict__ u, const double *__restrict__ alpha) {
  const size_t npad = (size_t)T0 * TS;
  const double a = *alpha;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < npad * npad;
       e += (size_t)gridDim.x * blockDim.x) {
    const int R = (int)(e / npad), C = (int)(e % npad);
    if (R < nc && C < nc) A0t[a0_index(R, C, T0)] += a * u[R] * u[C];
  }
}

// ------------------------------------------------- dense tiled Cholesky ---
__device__ __forceinline__ double *tile_ptr(double *A, int T0, int I, int J) {
  return A + ((size_t)I * T0 + J) * TE;
}

// Step k: factor diagonal tile, store L_kk in place and inv(L_kk) in dinv.
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1))) k_dense_potrf_diag(double *A0t, int T0, int k, double *dinv,
                                                         int *status) {
  extern __shared__ double lds[];
  double *X = lds, *Y = lds + TS * LDT;
  __shared__ int fail;
  __builtin_amdgcn_s_setprio(3);  // critical path: issue ahead of concurrent update kernels
  if (threadIdx.x == 0) fail = 0;
  tile_to_lds(tile_ptr(A0t, T0, k, k), X);
  __syncthreads();
  lds_potrf_trtri<32>(X, Y, &fail);
  lds_to_tile(X, tile_ptr(A0t, T0, k, k));
  lds_to_tile(Y, dinv + (size_t)k * TE);
  __syncthreads();
  if (threadIdx.x == 0 && fail) *status |= 1;
}

// L_ik = A_ik inv(L_kk)^T for i > k (each wavefront reads only its own rows
// of A_ik before writing them, so the product can be formed in place)
__global__ void __launch_bounds__(WG) k_dense_trsm_panel(double *A0t, int T0, int k,
                                                         const double *dinv) {
  const int i = k + 1 + blockIdx.x;
  double *a = tile_ptr(A0t, T0, i, k);
  __builtin_amdgcn_s_setprio(3);  // critical path
  Acc4 o;
  acc_zero(o);
  acc_mma_abt(o, a, TS, dinv + (size_t)k * TE, TS, 1.0);
  acc_store(o, a);
}

// A_ij -= L_ik L_jk^T over the tiles j0 <= j <= i (tri = 1), or over the
// single tile column j = j0, i >= j0 (tri = 0).
__global__ void __launch_bounds__(WG) k_dense_syrk_update(double *A0t, int T0, int k, int j0,
                                                          int tri) {
  const int b = blockIdx.x;
  int ii = b, jj = 0;
  if (!tri) __builtin_amdgcn_s_setprio(3);  // next tile column: critical path
  if (tri) {
    ii = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((ii + 1) * (ii + 2) / 2 <= b) ++ii;
    while (ii * (ii + 1) / 2 > b) --ii;
    jj = b - ii * (ii + 1) / 2;
  }
  const int i = j0 + ii, j = j0 + jj;
  // every wavefront multiplies by the whole L_jk: stage it once in LDS
  __shared__ double Ly[TS * LDT];
  tile_to_lds(tile_ptr(A0t, T0, j, k), Ly);
  double *c = tile_ptr(A0t, T0, i, j);
  Acc4 o;
  acc_load(o, c);
  __syncthreads();
  acc_mma_abt(o, tile_ptr(A0t, T0, i, k), TS, Ly, LDT, -1.0);
  acc_store(o, c);
}

// Step k's update of the next tile column, fused with step k+1's diagonal
// factor: tile (k+1+b, k+1) -= L_{k+1+b,k} L_{k+1,k}^T for every b (as
// k_dense_syrk_update over that column); workgroup 0 holds the next diagonal
// tile, which it then factors in LDS as k_dense_potrf_diag does (L in place,
// its inverse in dinv).  One launch and one launch gap less per step on the
// critical path.
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_dense_next_potrf(double *A0t, int T0, int k, double *dinv, int *status) {
  extern __shared__ double lds[];
  double *Ly = lds, *Y = lds + TS * LDT;  // Ly then holds the tile to factor
  __shared__ int fail;
  const int b = blockIdx.x, j = k + 1, i = j + b;
  __builtin_amdgcn_s_setprio(3);  // critical path
  if (threadIdx.x == 0) fail = 0;
  tile_to_lds(tile_ptr(A0t, T0, j, k), Ly);
  double *c = tile_ptr(A0t, T0, i, j);
  Acc4 o;
  acc_load(o, c);
  __syncthreads();
  acc_mma_abt(o, tile_ptr(A0t, T0, i, k), TS, Ly, LDT, -1.0);
  if (b != 0) {  // uniform over the workgroup
    acc_store(o, c);
    return;
  }
  __syncthreads();  // every wavefront has finished reading L_{k+1,k}
  acc_to_lds(o, Ly);
  __syncthreads();
  lds_potrf_trtri<32>(Ly, Y, &fail);
  lds_to_tile(Ly, c);
  lds_to_tile(Y, dinv + (size_t)j * TE);
  __syncthreads();
  if (threadIdx.x == 0 && fail) *status |= 1;
}

// Inverse factor by a right-looking solve of L X = I, step k:
//   row k:   X_kj <- inv(L_kk) B_kj  (j <= k)
//   update:  B_ij -= L_ik X_kj        (i > k, j <= k)
__global__ void __launch_bounds__(WG) k_dense_inv_row(double *Wt, int T0, int k,
                                                      const double *dinv) {
  extern __shared__ double lds[];
  const int j = blockIdx.x;  // 0..k
  double *w = tile_ptr(Wt, T0, k, j);
  tile_to_lds(w, lds);
  __syncthreads();
  Acc4 o;
  acc_zero(o);
  acc_mma_ab(o, dinv + (size_t)k * TE, TS, lds, LDT, 1.0);
  acc_store(o, w);
}

__global__ void __launch_bounds__(WG) k_dense_inv_update(const double *Lt, double *Wt, int T0,
                                                         int k) {
  const int i = k + 1 + blockIdx.x / (k + 1);
  const int j = blockIdx.x % (k + 1);
  // every wavefront multiplies by the whole X_kj: stage it once in LDS
  __shared__ double Xk[TS * LDT];
  tile_to_lds(Wt + ((size_t)k * T0 + j) * TE, Xk);
  double *c = tile_ptr(Wt, T0, i, j);
  Acc4 o;
  acc_load(o, c);
  __syncthreads();
  acc_mma_ab(o, Lt + ((size_t)i * T0 + k) * TE, TS, Xk, LDT, -1.0);
  acc_store(o, c);
}

__global__ void k_tiles_identity(double *Wt, int T0) {
  const size_t tot = (size_t)T0 * T0 * TE;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t tile = e / TE;
    const int I = (int)(tile / T0), J = (int)(tile % T0);
    const int r = (int)((e % TE) / TS), c = (int)(e % TS);
    Wt[e] = (I == J && r == c) ? 1.0 : 0.0;
  }
}

__global__ void k_tiles_to_f32_lower(const double *__restrict__ src, float *__restrict__ dst,
                                     int T0) {
  const size_t tot = (size_t)T0 * T0 * TE;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// ------------------------------------------------ coarse solve (TRMV) -----
// y = W x (transpose = 0) or y = W^T x (transpose = 1) for the lower tiles
// of W.  Stage 1: one workgroup per lower tile writes its 64-vector product
// into part[(out tile) * T0 + (in tile)]; stage 2 sums in tile order.
template <typename T>
__global__ void __launch_bounds__(WG) k_trmv_tiles(const T *__restrict__ Wt, int T0,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ part, int transpose,
                                                   const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double xs[TS];
  __shared__ double red[4][TS];
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;  // J <= I
  const T *w = Wt + ((size_t)I * T0 + J) * TE;
  const int t = threadIdx.x;
  if (!transpose) {
    if (t < TS) xs[t] = x[J * TS + t];
    __syncthreads();
    const int r = t >> 2, q = t & 3;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) s = fma((double)w[r * TS + 16 * q + c], xs[16 * q + c], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (q == 0) part[((size_t)I * T0 + J) * TS + r] = s;
  } else {
    if (t < TS) xs[t] = x[I * TS + t];
    __syncthreads();
    const int c = t & 63, g = t >> 6;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) s = fma((double)w[(16 * g + r) * TS + c], xs[16 * g + r], s);
    red[g][c] = s;
    __syncthreads();
    if (g == 0) part[((size_t)J * T0 + I) * TS + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  }
}

// y[O*64 + r] = sum over input tiles K (in order) of part[(O*T0 + K)*64 + r],
// K ranging over J <= O (no transpose) or I >= O (transpose).  RG groups of
// 64 threads per output tile split the K range into fixed consecutive
// pieces (a few loads each, issued together), combined in group order.
constexpr int RG = TRMV_RG;
__global__ void __launch_bounds__(RG * TS) k_trmv_reduce(int T0, const double *__restrict__ part,
                                                         double *__restrict__ y, int transpose,
                                                         const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double red[RG][TS];
  const int O = blockIdx.x, r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int k0 = transpose ? O : 0, k1 = transpose ? T0 : O + 1;
  const int len = k1 - k0;
  const int a = k0 + (len * g) / RG, b = k0 + (len * (g + 1)) / RG;
  double s = 0.0;
#pragma unroll 4
  for (int K = a; K < b; ++K) s += part[((size_t)O * T0 + K) * TS + r];
  red[g][r] = s;
  __syncthreads();
  if (g == 0) {
    double tot = 0.0;
#pragma unroll
    for (int gg = 0; gg < RG; ++gg) tot += red[gg][r];
    y[O * TS + r] = tot;
  }
}

// ------------------------------------------------------------- launchers ---
static size_t two_tiles_lds() { return (size_t)(2 * TS * LDT) * sizeof(double); }
static size_t one_tile_lds() { return (size_t)(TS * LDT) * sizeof(double); }

void launch_apply_A_to_basis(hipStream_t s, const Plan &p, const CoarsePlan &c,
                             const double *val, const double *phi, double *W) {
  hipLaunchKernelGGL(k_apply_A_to_basis, dim3(p.N), dim3(WG), 0, s, p, c, val, phi, W);
}

void launch_pair_products(hipStream_t s, const Plan &p, const CoarsePlan &c, const double *phi,
                          const double *W, double *A0t, int T0) {
  if (c.npairs == 0) return;
  hipLaunchKernelGGL(k_pair_products, dim3(c.npairs), dim3(WG), 0, s, p, c, phi, W, A0t, T0);
}

void launch_singular_regularize(hipStream_t s, const Plan &p, const double *phi, double *A0t,
                                int T0, int nc, double *u, double *alpha) {
  hipLaunchKernelGGL(k_basis_colsum, dim3(p.N), dim3(WG), 0, s, p, phi, u);
  hipLaunchKernelGGL(k_rank1_scale, dim3(1), dim3(WG), 0, s, A0t, T0, nc, u, alpha);
  size_t tot = (size_t)T0 * TS * T0 * TS;
  size_t b = (tot + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_rank1_update, dim3((unsigned)b), dim3(WG), 0, s, A0t, T0, nc, u, alpha);
}

void launch_symmetrize_tiles(hipStream_t s, double *A0t, int T0, int nc) {
  const unsigned nb = (unsigned)((size_t)T0 * (T0 + 1) / 2);
  if (nb > 0) hipLaunchKernelGGL(k_symmetrize, dim3(nb), dim3(WG), 0, s, A0t, T0, nc);
}

void launch_dense_potrf_diag(hipStream_t s, double *A0t, int T0, int k, double *dinv, int *status) {
  allow_lds(k_dense_potrf_diag, two_tiles_lds());
  hipLaunchKernelGGL(k_dense_potrf_diag, dim3(1), dim3(WG), two_tiles_lds(), s, A0t, T0, k, dinv,
                     status);
}

void launch_dense_trsm_panel(hipStream_t s, double *A0t, int T0, int k, const double *dinv) {
  const int nb = T0 - k - 1;
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_dense_trsm_panel, dim3(nb), dim3(WG), 0, s, A0t, T0, k, dinv);
}

void launch_dense_next_potrf(hipStream_t s, double *A0t, int T0, int k, double *dinv,
                             int *status) {
  const int m = T0 - k - 1;
  if (m <= 0) return;
  allow_lds(k_dense_next_potrf, two_tiles_lds());
  hipLaunchKernelGGL(k_dense_next_potrf, dim3(m), dim3(WG), two_tiles_lds(), s, A0t, T0, k, dinv,
                     status);
}

void launch_dense_syrk_rest(hipStream_t s, double *A0t, int T0, int k) {
  const int m = T0 - k - 2;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_dense_syrk_update, dim3(m * (m + 1) / 2), dim3(WG), 0, s, A0t, T0, k, k + 2,
                     1);
}

void launch_dense_inv_row(hipStream_t s, double *Wt, int T0, int k, const double *dinv) {
  hipLaunchKernelGGL(k_dense_inv_row, dim3(k + 1), dim3(WG), one_tile_lds(), s, Wt, T0, k, dinv);
}

void launch_dense_inv_update(hipStream_t s, const double *Lt, double *Wt, int T0, int k) {
  const int m = T0 - k - 1;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_dense_inv_update, dim3(m * (k + 1)), dim3(WG), 0, s, Lt, Wt, T0, k);
}

void launch_tiles_identity(hipStream_t s, double *Wt, int T0) {
  size_t tot = (size_t)T0 * T0 * TE;
  size_t b = (tot + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_tiles_identity, dim3((unsigned)b), dim3(WG), 0, s, Wt, T0);
}

void launch_dense_tiles_to_f32(hipStream_t s, const double *src, float *dst, int T0) {
  size_t tot = (size_t)T0 * T0 * TE;
  size_t b = (tot + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_tiles_to_f32_lower, dim3((unsigned)b), dim3(WG), 0, s, src, dst, T0);
}

template <typename T>
void launch_trmv(hipStream_t s, const T *Wt, int T0, const double *x, double *part, double *y,
                 int transpose, const int *done) {
  const int nb = T0 * (T0 + 1) / 2;
  hipLaunchKernelGGL((k_trmv_tiles<T>), dim3(nb), dim3(WG), 0, s, Wt, T0, x, part, transpose, done);
  if (y)
    hipLaunchKernelGGL(k_trmv_reduce, dim3(T0), dim3(RG * TS), 0, s, T0, part, y, transpose, done);
}
template void launch_trmv<double>(hipStream_t, const double *, int, const double *, double *,
                                  double *, int, const int *);
template void launch_trmv<float>(hipStream_t, const float *, int, const double *, double *,
                                 double *, int, const int *);

}  // namespace amsp
