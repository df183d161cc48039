// Per-subdomain local matrices, their batched tile-profile Cholesky
// factorisation, and the local solves of the additive Schwarz term.
//
// Local matrices (Section 3.2): A_i = R_i A R_i^T on the overlapping region,
// hat A_i = A_i with the diagonal replaced by minus the sum of the row's
// off-diagonals (couplings inside the region only), S_i = diag(hat A_i) and
// the standard-form eigen-operator B_i = S^{-1/2} hat A_i S^{-1/2}.
//
// Storage: each region is ordered locally (RCM by default) and stored as
// 64x64 row-major tiles of its lower triangle, restricted to the tile
// profile: tile row I holds tiles J = first(I)..I.  Cholesky fill stays
// inside the row envelope, so the profile of the factor equals that of A_i.
// After factorisation each diagonal tile holds inv(L_II) (the local solves
// then need only matrix-vector products) and the off-diagonal tiles hold L_IJ.
#include <hip/hip_ext.h>

#include "k_common.h"

namespace amsp {

// ------------------------------------------------------------ S_i ---------
__global__ void __launch_bounds__(WG) k_neumann_diag(Plan p, const double *__restrict__ val,
                                                     double *__restrict__ sdiag,
                                                     int *__restrict__ status) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], r1 = p.sd_ptr[i + 1];
  int bad = 0;
  for (int R = r0 + threadIdx.x; R < r1; R += WG) {
    const int l = R - r0;
    double s = 0.0;
    for (int e = p.loc_rowptr[R]; e < p.loc_rowptr[R + 1]; ++e)
      if (p.loc_col[e] != l) s -= val[p.loc_src[e]];
    sdiag[R] = s;
    if (!(s > 0.0)) bad = 1;
  }
  if (bad) status[i] |= 1;
}

// ----------------------------------------------------- tile extraction ----
// One workgroup per tile row.  Thread t fills row (t>>2) of each tile, columns
// 16*(t&3) .. +15, by scanning that local CSR row once.
__global__ void __launch_bounds__(WG) k_extract_tiles(Plan p, int nrows_total,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ sdiag,
                                                      double *__restrict__ tiles, int mode,
                                                      double sigma) {
  const int g = blockIdx.x;
  const int i = find_segment(p.trow_ptr, p.N, g);
  const int I = g - p.trow_ptr[i];
  const int r0 = p.sd_ptr[i];
  const int ni = p.sd_ptr[i + 1] - r0;
  const int fI = p.tfirst[g];
  const long long t0 = p.toff[g];
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  const int l = I * TS + r;
  const bool real = l < ni;
  const int e0 = real ? p.loc_rowptr[r0 + l] : 0, e1 = real ? p.loc_rowptr[r0 + l + 1] : 0;
  const double sl = (real && mode == 1) ? sdiag[r0 + l] : 1.0;
  for (int J = fI; J <= I; ++J) {
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0.0;
    const int cbase = J * TS + 16 * q;
    if (real) {
      for (int e = e0; e < e1; ++e) {
        const int lc = p.loc_col[e];
        const int off = lc - cbase;
        if (off >= 0 && off < 16) {
          double a = val[p.loc_src[e]];
          if (mode == 1) a = (lc == l) ? 1.0 + sigma : a / sqrt(sl * sdiag[r0 + lc]);
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c == off) v[c] = a;
        }
      }
    } else {
      // padding rows: identity on the diagonal
      const int off = l - cbase;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c == off) v[c] = 1.0;
    }
    double *dst = tiles + tile_elem(t0 + (J - fI)) + r * TS + 16 * q;
#pragma unroll
    for (int c = 0; c < 16; ++c) dst[c] = v[c];
  }
}

// ------------------------------------------------ batched Cholesky --------
// One workgroup per region, left-looking over tile rows.  For tile (I,J):
//   C = A_IJ - sum_K L_IK L_JK^T  (K over tiles present in both rows; MFMA)
//   J < I : L_IJ = C inv(L_JJ)^T   (MFMA)
//   J = I : L_II = chol(C) in LDS; the tile then stores inv(L_II).
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) k_profile_cholesky(Plan p, double *__restrict__ tiles, int bit,
                                                         int *__restrict__ status) {
  extern __shared__ double lds[];
  double *X = lds;             // 64 x LDT
  double *Y = lds + TS * LDT;  // 64 x LDT
  __shared__ int fail;
  const int i = blockIdx.x;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int I = 0; I < nt; ++I) {
    const int fI = p.tfirst[g0 + I];
    const long long tI = p.toff[g0 + I];
    for (int J = fI; J <= I; ++J) {
      const int fJ = p.tfirst[g0 + J];
      const long long tJ = p.toff[g0 + J];
      double *cij = tiles + tile_elem(tI + (J - fI));
      Acc4 c;
      acc_load(c, cij);
      const int k0 = fI > fJ ? fI : fJ;
      for (int K = k0; K < J; ++K)
        acc_mma_abt(c, tiles + tile_elem(tI + (K - fI)), TS, tiles + tile_elem(tJ + (K - fJ)), TS, -1.0);
      acc_to_lds(c, X);
      __syncthreads();
      if (J < I) {
        Acc4 o;
        acc_zero(o);
        acc_mma_abt(o, X, LDT, tiles + tile_elem(tJ + (J - fJ)), TS, 1.0);  // C inv(L_JJ)^T
        acc_store(o, cij);
      } else {
        lds_potrf_trtri<16>(X, Y, &fail);
        lds_to_tile(Y, cij);
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0 && fail) status[i] |= bit;
}

__global__ void k_tiles_to_f32(const double *__restrict__ src, float *__restrict__ dst,
                               size_t count) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// ------------------------------------------------ local solves (1 rhs) ----
// Row-mapped tile-vector product: thread t owns row t>>2 and 16 columns.
template <typename T, typename C>
__device__ __forceinline__ C tile_row_dot(const T *__restrict__ tile, const C *v) {
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  const T *row = tile + r * TS + 16 * q;
  const C *vv = v + 16 * q;
  C s = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) s = fma((C)row[c], vv[c], s);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  return s;  // full row sum in all 4 lanes of the row
}

// The 16 entries of one tile row that a thread holds in the row mapping
// (row t>>2, columns 16(t&3) ..), loaded ahead of their use.
template <typename T>
struct RowFrag {
  T a[16];
};

template <typename T>
__device__ __forceinline__ void row_frag_load(RowFrag<T> &f, const T *__restrict__ tile) {
  const T *row = tile + (threadIdx.x >> 2) * TS + 16 * (threadIdx.x & 3);
#pragma unroll
  for (int c = 0; c < 16; ++c) f.a[c] = row[c];
}

template <typename T, typename C>
__device__ __forceinline__ C row_frag_dot(const RowFrag<T> &f, const C *v) {
  const C *vv = v + 16 * (threadIdx.x & 3);
  C s = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) s = fma((C)f.a[c], vv[c], s);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  return s;  // full row sum in all 4 lanes of the row
}

// The 16 entries a thread holds in the column-ownership mapping: wavefront w
// owns columns 16w .. 16w+15; lane l covers column 16w + (l & 15) and rows
// 16(l >> 4) .. +15, so a column's 64 rows sit in four lanes 16 apart.
template <typename T>
struct ColFrag {
  T a[16];
};

template <typename T>
__device__ __forceinline__ void col_frag_load(ColFrag<T> &f, const T *__restrict__ tile) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T *src = tile + (16 * (l >> 4)) * TS + 16 * w + (l & 15);
#pragma unroll
  for (int r = 0; r < 16; ++r) f.a[r] = src[r * TS];
}

// sum_r tile[r][col] x[r] for this lane's column, complete in all four lanes
// of the column (x: the 64-vector the tile multiplies, in LDS)
template <typename T, typename C>
__device__ __forceinline__ C col_frag_dot(const ColFrag<T> &f, const C *x) {
  const C *xx = x + 16 * ((threadIdx.x & 63) >> 4);
  C s = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) s = fma((C)f.a[r], xx[r], s);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

// Column-mapped transposed product: thread t owns column t&63 and 16 rows;
// partial sums over the 4 row groups are combined through LDS.
template <typename T, typename C>
__device__ __forceinline__ C tile_col_dot(const T *__restrict__ tile, const C *v) {
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  C s = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) s = fma((C)tile[(16 * g + r) * TS + c], v[16 * g + r], s);
  return s;
}

// Fused additive-Schwarz local kernel for one region per workgroup:
//   gather r on the region, coarse restriction c_i = Phi_i^T r_i (optional),
//   forward/backward substitution with the tile-profile factor (optional),
//   store the local correction into the padded local vector xloc.
// T: factor storage type, C: compute type, TB: basis storage type.
template <typename T, typename C, typename TB>
__global__ void __launch_bounds__(WG) k_local_apply(Plan p, const double *__restrict__ r,
                                                    const T *__restrict__ tiles,
                                                    const TB *__restrict__ phi,
                                                    double *__restrict__ xloc,
                                                    double *__restrict__ cvec, int do_local,
                                                    int do_coarse, const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ char smem_raw[];
  C *v = reinterpret_cast<C *>(smem_raw);          // whole local vector (padded)
  C *tmp = v + (p.vp_ptr[blockIdx.x + 1] - p.vp_ptr[blockIdx.x]);  // 64
  C *part = tmp + TS;                               // 4 x 64
  __shared__ double red[MAXNEV + 1][WG / 64];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  const int npad = nt * TS;
  const int nev = p.nev;
  const int m = p.mi[i];
  double cacc[MAXNEV];
#pragma unroll
  for (int k = 0; k < MAXNEV; ++k) cacc[k] = 0.0;
  for (int l = threadIdx.x; l < npad; l += WG) {
    double rv = 0.0;
    if (l < ni) {
      rv = r[p.sd_dofs[r0 + l]];
      if (do_coarse) {
        const TB *ph = phi + (size_t)(r0 + l) * nev;
#pragma unroll
        for (int k = 0; k < MAXNEV; ++k)
          if (k < m) cacc[k] = fma(to_d(ph[k]), rv, cacc[k]);
      }
    }
    v[l] = (C)rv;
  }
  if (do_coarse) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < m; ++k) {
      double s = wave_sum(cacc[k]);
      if (lane == 0) red[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < m) {
      double s = 0.0;
      for (int ww = 0; ww < WG / 64; ++ww) s += red[threadIdx.x][ww];
      cvec[p.coff[i] + threadIdx.x] = s;
    }
  }
  __syncthreads();
  if (!do_local) return;
  const int rr = threadIdx.x >> 2, q = threadIdx.x & 3;
  const int cc = threadIdx.x & 63, gg = threadIdx.x >> 6;
  // Both sweeps stream the region's tiles: the forward sweep in storage
  // order (each row's off-diagonal tiles, then its diagonal), the backward
  // sweep in reverse.  D + 1 register slots hold the next tiles; the slot
  // loop is unrolled so each slot is refilled in place right after its tile
  // is used (no register copies, which would wait for the loads in flight).
  constexpr int D = sizeof(T) == 4 ? 3 : 1;  // keeps 4 workgroups per CU resident
  const long long t0 = p.toff[g0];
  const int ntl = (int)(p.toff[g0 + nt - 1] + (nt - 1 - p.tfirst[g0 + nt - 1]) + 1 - t0);
  const T *pool = tiles + tile_elem(t0);
  // forward: y_I = inv(L_II) (b_I - sum_J L_IJ y_J)
  {
    RowFrag<T> f[D + 1];
#pragma unroll
    for (int d = 0; d <= D; ++d)
      if (d < ntl) row_frag_load(f[d], pool + tile_elem(d));
    int I = 0, J = p.tfirst[g0];
    C acc = v[rr];
    for (int k0 = 0; k0 < ntl; k0 += D + 1) {
#pragma unroll
      for (int sl = 0; sl <= D; ++sl) {
        const int k = k0 + sl;
        if (k < ntl) {
          if (J < I) {
            acc -= row_frag_dot<T, C>(f[sl], v + J * TS);
            ++J;
          } else {
            if (q == 0) tmp[rr] = acc;
            __syncthreads();
            const C y = row_frag_dot<T, C>(f[sl], tmp);
            if (q == 0) v[I * TS + rr] = y;
            __syncthreads();
            ++I;
            if (I < nt) {
              J = p.tfirst[g0 + I];
              acc = v[I * TS + rr];
            }
          }
          if (k + D + 1 < ntl) row_frag_load(f[sl], pool + tile_elem(k + D + 1));
        }
      }
    }
  }
  // backward, right-looking: for I = nt-1 .. 0, x_I = inv(L_II)^T y_I, then
  // y_J -= L_IJ^T x_I for the off-diagonal tiles J of row I (storage order
  // reversed: the diagonal first, then J descending).  Wavefront w owns
  // columns 16w .. 16w+15 of every product, so each y_J entry has a single
  // writer and a row needs two barriers.
  {
    ColFrag<T> f[D + 1];
#pragma unroll
    for (int d = 0; d <= D; ++d)
      if (d < ntl) col_frag_load(f[d], pool + tile_elem(ntl - 1 - d));
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = 16 * w + (l & 15);
    const bool head = (l >> 4) == 0;  // one lane of the four that share a column
    int I = nt - 1, J = nt - 1, fI = p.tfirst[g0 + nt - 1];
    for (int k0 = 0; k0 < ntl; k0 += D + 1) {
#pragma unroll
      for (int sl = 0; sl <= D; ++sl) {
        const int k = k0 + sl;
        if (k < ntl) {
          if (J == I) {
            __syncthreads();  // y_I complete (updates from rows > I)
            const C x = col_frag_dot<T, C>(f[sl], v + I * TS);
            if (head) tmp[col] = x;
            __syncthreads();  // x_I visible in tmp; all reads of y_I done
            if (head) v[I * TS + col] = x;
          } else {
            const C s2 = col_frag_dot<T, C>(f[sl], tmp);
            if (head) v[J * TS + col] -= s2;
          }
          if (J > fI) {
            --J;
          } else {
            --I;
            if (I >= 0) {
              J = I;
              fI = p.tfirst[g0 + I];
            }
          }
          if (k + D + 1 < ntl) col_frag_load(f[sl], pool + tile_elem(ntl - 1 - (k + D + 1)));
        }
      }
    }
    __syncthreads();
  }
  // local correction in the region's ascending-global-index layout, so that
  // the scatter reads contiguous runs
  double *dst = xloc + p.vp_ptr[i];
  for (int l = threadIdx.x; l < ni; l += WG) dst[p.nat[r0 + l]] = (double)v[l];
}

// ------------------------------------------- block solve (EIGP rhs) -------
// In-place (L L^T)^{-1} X for a row-major padded block X[rows][EIGP], one
// workgroup per region; regions flagged in skip[] are left untouched.
template <typename T>
__global__ void __launch_bounds__(WG) k_profile_solve_block(Plan p, const T *__restrict__ tiles,
                                                            double *__restrict__ X,
                                                            const int *__restrict__ skip) {
  const int i = blockIdx.x;
  if (skip && skip[i]) return;
  extern __shared__ double lds[];
  double *Lt = lds;                    // 64 x LDT
  double *V = lds + TS * LDT;          // 64 x (EIGP+1) right-hand block
  double *Acc = V + TS * (EIGP + 1);   // 64 x (EIGP+1)
  constexpr int LV = EIGP + 1;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 4;
  // forward
  for (int I = 0; I < nt; ++I) {
    const int fI = p.tfirst[g0 + I];
    const long long tI = p.toff[g0 + I];
    double acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = Xi[(size_t)(I * TS + r) * EIGP + c0 + j];
    for (int J = fI; J < I; ++J) {
      __syncthreads();
      tile_to_lds(tiles + tile_elem(tI + (J - fI)), Lt);
      for (int e = threadIdx.x; e < TS * EIGP; e += WG)
        V[(e / EIGP) * LV + (e % EIGP)] = Xi[(size_t)J * TS * EIGP + e];
      __syncthreads();
      for (int k = 0; k < TS; ++k) {
        const double a = Lt[r * LDT + k];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fma(-a, V[k * LV + c0 + j], acc[j]);
      }
    }
    __syncthreads();
    tile_to_lds(tiles + tile_elem(tI + (I - fI)), Lt);
#pragma unroll
    for (int j = 0; j < 4; ++j) Acc[r * LV + c0 + j] = acc[j];
    __syncthreads();
    double y[4] = {0, 0, 0, 0};
    for (int k = 0; k < TS; ++k) {
      const double a = Lt[r * LDT + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = fma(a, Acc[k * LV + c0 + j], y[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Xi[(size_t)(I * TS + r) * EIGP + c0 + j] = y[j];
  }
  // backward
  for (int I = nt - 1; I >= 0; --I) {
    __syncthreads();
    double acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = Xi[(size_t)(I * TS + r) * EIGP + c0 + j];
    for (int J = I + 1; J < nt; ++J) {
      const int fJ = p.tfirst[g0 + J];
      if (fJ > I) continue;
      __syncthreads();
      tile_to_lds(tiles + tile_elem(p.toff[g0 + J] + (I - fJ)), Lt);
      for (int e = threadIdx.x; e < TS * EIGP; e += WG)
        V[(e / EIGP) * LV + (e % EIGP)] = Xi[(size_t)J * TS * EIGP + e];
      __syncthreads();
      // acc[r][:] -= sum_k L_JI[k][r] V[k][:]
      for (int k = 0; k < TS; ++k) {
        const double a = Lt[k * LDT + r];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fma(-a, V[k * LV + c0 + j], acc[j]);
      }
    }
    __syncthreads();
    const int fI = p.tfirst[g0 + I];
    tile_to_lds(tiles + tile_elem(p.toff[g0 + I] + (I - fI)), Lt);
#pragma unroll
    for (int j = 0; j < 4; ++j) Acc[r * LV + c0 + j] = acc[j];
    __syncthreads();
    double y[4] = {0, 0, 0, 0};
    for (int k = 0; k < TS; ++k) {
      const double a = Lt[k * LDT + r];  // inv(L_II)^T
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = fma(a, Acc[k * LV + c0 + j], y[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Xi[(size_t)(I * TS + r) * EIGP + c0 + j] = y[j];
  }
}

// ------------------------------------ block solve on MFMA (EIGP rhs) ------
// Same operation as k_profile_solve_block, one workgroup (4 wavefronts) per
// region: wavefront w owns rows 16w..16w+15 of the 64 x EIGP block of the
// current tile row.  A 64x64 tile times the 64x16 block is 16 MFMA steps;
// K-slot q of step s stands for column k = 16q + s, so that each lane reads
// 16 contiguous entries of one tile row (non-transposed products) and the
// transposed products read 16 consecutive columns per instruction.
template <typename T>
__device__ __forceinline__ d4 mfma_tile_rhs(const T *__restrict__ tile, const double *rhs, int w,
                                            int transpose, d4 acc, double sign) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, q = l >> 4;
  double a[16];
  if (!transpose) {
    const T *row = tile + (16 * w + i) * TS + 16 * q;
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = (double)row[s];
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = (double)tile[(16 * q + s) * TS + 16 * w + i];
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) acc = mfma16x16x4(sign * a[s], rhs[(16 * q + s) * (EIGP + 1) + i], acc);
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(WG) k_profile_solve_block_mfma(Plan p, const T *__restrict__ tiles,
                                                                 const double *Xin, double *X,
                                                                 const int *__restrict__ skip) {
  const int i = blockIdx.x;
  if (skip && skip[i]) return;
  __shared__ double V[TS * (EIGP + 1)];    // right-hand block of a neighbour tile row
  __shared__ double Acc[TS * (EIGP + 1)];  // current accumulated block
  constexpr int LV = EIGP + 1;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  const double *Xin_i = Xin + (size_t)p.vp_ptr[i] * EIGP;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int col = l & 15, rb = 16 * w + (l >> 4);  // D register r: row rb + 4r, column col
  auto load_block = [&](int J, double *dst) {
    for (int e = threadIdx.x; e < TS * EIGP; e += WG) dst[(e / EIGP) * LV + (e % EIGP)] = Xi[(size_t)J * TS * EIGP + e];
  };
  // forward: Y_I = inv(L_II) (X_I - sum_J L_IJ Y_J)
  for (int I = 0; I < nt; ++I) {
    const int fI = p.tfirst[g0 + I];
    const long long tI = p.toff[g0 + I];
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = Xin_i[(size_t)(I * TS + rb + 4 * r) * EIGP + col];
    for (int J = fI; J < I; ++J) {
      __syncthreads();
      load_block(J, V);
      __syncthreads();
      acc = mfma_tile_rhs<T>(tiles + tile_elem(tI + (J - fI)), V, w, 0, acc, -1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Acc[(rb + 4 * r) * LV + col] = acc[r];
    __syncthreads();
    d4 y = {0.0, 0.0, 0.0, 0.0};
    y = mfma_tile_rhs<T>(tiles + tile_elem(tI + (I - fI)), Acc, w, 0, y, 1.0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xi[(size_t)(I * TS + rb + 4 * r) * EIGP + col] = y[r];
    __syncthreads();
  }
  // backward: X_I = inv(L_II)^T (Y_I - sum_{J>I} L_JI^T X_J)
  for (int I = nt - 1; I >= 0; --I) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = Xi[(size_t)(I * TS + rb + 4 * r) * EIGP + col];
    for (int J = I + 1; J < nt; ++J) {
      const int fJ = p.tfirst[g0 + J];
      if (fJ > I) continue;
      __syncthreads();
      load_block(J, V);
      __syncthreads();
      acc = mfma_tile_rhs<T>(tiles + tile_elem(p.toff[g0 + J] + (I - fJ)), V, w, 1, acc, -1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Acc[(rb + 4 * r) * LV + col] = acc[r];
    __syncthreads();
    const int fI = p.tfirst[g0 + I];
    d4 y = {0.0, 0.0, 0.0, 0.0};
    y = mfma_tile_rhs<T>(tiles + tile_elem(p.toff[g0 + I] + (I - fI)), Acc, w, 1, y, 1.0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Xi[(size_t)(I * TS + rb + 4 * r) * EIGP + col] = y[r];
    __syncthreads();
  }
}

// Device self-test of the MFMA operand/result layout used above: D = A B
// for A (16x4) and B (4x16) given row-major, D written row-major (16x16).
__global__ void k_selftest_mfma(const double *A, const double *B, double *D) {
  const int l = threadIdx.x;
  d4 c = {0.0, 0.0, 0.0, 0.0};
  c = mfma16x16x4(A[(l & 15) * 4 + (l >> 4)], B[(l >> 4) * 16 + (l & 15)], c);
#pragma unroll
  for (int r = 0; r < 4; ++r) D[((l >> 4) + 4 * r) * 16 + (l & 15)] = c[r];
}

void launch_selftest_mfma(hipStream_t s, const double *A, const double *B, double *D) {
  hipLaunchKernelGGL(k_selftest_mfma, dim3(1), dim3(64), 0, s, A, B, D);
}

// ------------------------------------------------------------ scatter -----
// z[j] = sum over regions containing j of (local correction + Phi t) and the
// partial r.z, in the fixed order of the inverse map (no atomics).  The local
// corrections and the basis copy are in each region's ascending-global-index
// layout and inv_loc holds that position, so consecutive dofs of a region
// read consecutive entries.
template <typename TB>
__global__ void __launch_bounds__(WG) k_scatter_sum(int n, const int *__restrict__ inv_ptr,
                                                    const int *__restrict__ inv_sd,
                                                    const int *__restrict__ inv_loc, Plan p,
                                                    const double *__restrict__ xloc,
                                                    const TB *__restrict__ phi,  // natural layout
                                                    const double *__restrict__ t,
                                                    double *__restrict__ z,
                                                    const double *__restrict__ r,
                                                    double *__restrict__ partial, int do_local,
                                                    int do_coarse, const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[WG / 64];
  constexpr int U = 4;  // independent dofs per thread and trip (overlapping load chains)
  const int nev = p.nev;
  const int stride = gridDim.x * WG;
  double acc = 0.0;
  for (int j0 = blockIdx.x * WG + threadIdx.x; j0 < n; j0 += U * stride) {
    int e[U], e1[U];
    double zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * stride;
      e[u] = j < n ? inv_ptr[j] : 0;
      e1[u] = j < n ? inv_ptr[j + 1] : 0;
      zj[u] = 0.0;
    }
    for (;;) {
      bool any = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e[u] >= e1[u]) continue;
        any = true;
        const int sd = inv_sd[e[u]], l = inv_loc[e[u]];
        ++e[u];
        double v = 0.0;
        if (do_local) v = xloc[p.vp_ptr[sd] + l];
        if (do_coarse) {
          const int m = p.mi[sd];
          const TB *ph = phi + (size_t)(p.sd_ptr[sd] + l) * nev;
          const double *tt = t + p.coff[sd];
#pragma unroll
          for (int k = 0; k < MAXNEV; ++k)  // predicated: all loads issue together
            if (k < m) v = fma(to_d(ph[k]), tt[k], v);
        }
        zj[u] += v;
      }
      if (!any) break;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * stride;
      if (j < n) {
        z[j] = zj[u];
        if (r) acc = fma(r[j], zj[u], acc);
      }
    }
  }
  double tot = block_sum(acc, sh);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename TB>
__global__ void __launch_bounds__(WG) k_basis_to_natural(Plan p, const TB *__restrict__ src,
                                                         TB *__restrict__ dst) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0, nev = p.nev;
  for (int e = threadIdx.x; e < ni * nev; e += WG) {
    const int l = e / nev, c = e % nev;
    dst[(size_t)(r0 + p.nat[r0 + l]) * nev + c] = src[(size_t)(r0 + l) * nev + c];
  }
}

// ------------------------------------------------------------- launchers ---
template <typename TB>
void launch_basis_to_natural(hipStream_t s, const Plan &p, const TB *src, TB *dst) {
  hipLaunchKernelGGL((k_basis_to_natural<TB>), dim3(p.N), dim3(WG), 0, s, p, src, dst);
}
template void launch_basis_to_natural<double>(hipStream_t, const Plan &, const double *, double *);
template void launch_basis_to_natural<float>(hipStream_t, const Plan &, const float *, float *);
template void launch_basis_to_natural<__hip_bfloat16>(hipStream_t, const Plan &,
                                                      const __hip_bfloat16 *, __hip_bfloat16 *);

void launch_neumann_diag(hipStream_t s, const Plan &p, const double *val, double *sdiag,
                         int *status) {
  hipLaunchKernelGGL(k_neumann_diag, dim3(p.N), dim3(WG), 0, s, p, val, sdiag, status);
}

void launch_extract_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *val,
                          const double *sdiag, double *tiles, int mode, double sigma) {
  hipLaunchKernelGGL(k_extract_tiles, dim3(ntilerows), dim3(WG), 0, s, p, ntilerows, val, sdiag,
                     tiles, mode, sigma);
}

void launch_profile_cholesky(hipStream_t s, const Plan &p, double *tiles, int *status, int bit) {
  size_t sm = (size_t)(2 * TS * LDT) * sizeof(double);
  allow_lds(k_profile_cholesky, sm);
  hipLaunchKernelGGL(k_profile_cholesky, dim3(p.N), dim3(WG), sm, s, p, tiles, bit, status);
}

void launch_tiles_to_f32(hipStream_t s, const double *src, float *dst, size_t count) {
  size_t b = (count + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_tiles_to_f32, dim3((unsigned)b), dim3(WG), 0, s, src, dst, count);
}

template <typename T, typename C, typename TB>
void launch_local_apply_t(hipStream_t s, const Plan &p, int max_npad, const double *r,
                          const T *tiles, const TB *phi, double *xloc, double *cvec, int do_local,
                          int do_coarse, const int *done, hipEvent_t ev_start, hipEvent_t ev_stop) {
  size_t sm = (size_t)(max_npad + TS + 4 * TS) * sizeof(C);
  allow_lds(k_local_apply<T, C, TB>, sm);
  if (ev_start || ev_stop)  // events bound to this dispatch: exact kernel duration
    hipExtLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, ev_start, ev_stop,
                          0, p, r, tiles, phi, xloc, cvec, do_local, do_coarse, done);
  else
    hipLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, p, r, tiles, phi,
                       xloc, cvec, do_local, do_coarse, done);
}

template void launch_local_apply_t<double, double, double>(hipStream_t, const Plan &, int,
                                                           const double *, const double *,
                                                           const double *, double *, double *,
                                                           int, int, const int *, hipEvent_t,
                                                           hipEvent_t);
template void launch_local_apply_t<float, float, float>(hipStream_t, const Plan &, int,
                                                        const double *, const float *,
                                                        const float *, double *, double *, int,
                                                        int, const int *, hipEvent_t, hipEvent_t);
template void launch_local_apply_t<float, float, __hip_bfloat16>(
    hipStream_t, const Plan &, int, const double *, const float *, const __hip_bfloat16 *,
    double *, double *, int, int, const int *, hipEvent_t, hipEvent_t);

template <typename T>
void launch_profile_solve_block(hipStream_t s, const Plan &p, const T *tiles, const double *X,
                                double *Y, const int *skip) {
  hipLaunchKernelGGL((k_profile_solve_block_mfma<T>), dim3(p.N), dim3(WG), 0, s, p, tiles, X, Y,
                     skip);
}
template void launch_profile_solve_block<double>(hipStream_t, const Plan &, const double *,
                                                 const double *, double *, const int *);
template void launch_profile_solve_block<float>(hipStream_t, const Plan &, const float *,
                                                const double *, double *, const int *);

template <typename TB>
void launch_scatter_sum_t(hipStream_t s, int n, const int *inv_ptr, const int *inv_sd,
                          const int *inv_loc, const Plan &p, const double *xloc, const TB *phi,
                          const double *t, double *z, const double *r, double *partial,
                          int do_local, int do_coarse, const int *done) {
  hipLaunchKernelGGL((k_scatter_sum<TB>), dim3(reduce_blocks(n)), dim3(WG), 0, s, n, inv_ptr,
                     inv_sd, inv_loc, p, xloc, phi, t, z, r, partial, do_local, do_coarse, done);
}
template void launch_scatter_sum_t<double>(hipStream_t, int, const int *, const int *, const int *,
                                           const Plan &, const double *, const double *,
                                           const double *, double *, const double *, double *,
                                           int, int, const int *);
template void launch_scatter_sum_t<float>(hipStream_t, int, const int *, const int *, const int *,
                                          const Plan &, const double *, const float *,
                                          const double *, double *, const double *, double *, int,
                                          int, const int *);
template void launch_scatter_sum_t<__hip_bfloat16>(hipStream_t, int, const int *, const int *,
                                                   const int *, const Plan &, const double *,
                                                   const __hip_bfloat16 *, const double *,
                                                   double *, const double *, double *, int, int,
                                                   const int *);

}  // namespace amsp
