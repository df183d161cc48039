// Per-subdomain local matrices, their batched tile-profile Cholesky
// factorisation, and the local solves of the additive Schwarz term.
//
// Local matrices (Section 3.2): A_i = R_i A R_i^T on the overlapping region,
// hat A_i = A_i with the diagonal replaced by minus the sum of the row's
// off-diagonals (couplings inside the region only), S_i = diag(hat A_i) and
// the standard-form eigen-operator B_i = S^{-1/2} hat A_i S^{-1/2}.
//
// Storage: each region is ordered locally (RCM by default) and stored as
// 64x64 tiles of its lower triangle, restricted to the tile profile: tile row
// I holds tiles J = first(I)..I.  Cholesky fill stays inside the row
// envelope, so the profile of the factor equals that of A_i.  Off-diagonal
// tiles are row-major; diagonal tiles keep only their lower triangle, packed
// (see dpos_row), in a second pool behind the first.  After factorisation
// each diagonal tile holds inv(L_II) (the local solves then need only
// matrix-vector products) and the off-diagonal tiles hold L_IJ.
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
    if (J < I) {
      double *dst = tiles + tile_elem(t0 + (J - fI)) + r * TS + 16 * q;
#pragma unroll
      for (int c = 0; c < 16; ++c) dst[c] = v[c];
    } else {  // packed lower triangle, zero padding right of the diagonal
      double *dst = tiles + diag_elem(p, g) + dpos_row(r) + 16 * q;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (16 * q + (c & ~3) <= r) dst[c] = (16 * q + c <= r) ? v[c] : 0.0;
    }
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
      double *cij = J < I ? tiles + tile_elem(tI + (J - fI)) : tiles + diag_elem(p, g0 + I);
      Acc4 c;
      if (J < I) {
        acc_load(c, cij);
        packed_to_lds(tiles + diag_elem(p, g0 + J), Y);  // inv(L_JJ)
      } else {
        acc_load_packed(c, cij);  // lower triangle is all the factorisation reads
      }
      const int k0 = fI > fJ ? fI : fJ;
      for (int K = k0; K < J; ++K)
        acc_mma_abt(c, tiles + tile_elem(tI + (K - fI)), TS, tiles + tile_elem(tJ + (K - fJ)), TS, -1.0);
      acc_to_lds(c, X);
      __syncthreads();
      if (J < I) {
        Acc4 o;
        acc_zero(o);
        acc_mma_abt(o, X, LDT, Y, LDT, 1.0);  // C inv(L_JJ)^T
        acc_store(o, cij);
      } else {
        lds_potrf_trtri<16>(X, Y, &fail);
        lds_to_packed(Y, cij);
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

// ------------------------------------------------ envelope copy ----------
// The local solves of the apply read the factor's off-diagonal part in
// envelope form instead of tiles: below the diagonal tiles, row r of block I
// (rows 64I .. 64I+63) is nonzero at most in columns fenv[r] .. 64I-1, with
// fenv nondecreasing (see the planner), so both
//   row form    (forward sweep):  row r, columns 64I - len_r .. 64I - 1
//   column form (backward sweep): column c of block J, rows 64(J+1) .. +len_c - 1
// are contiguous segments; eptr / uptr hold their starts.  One workgroup per
// tile row g; entries outside the tile profile are zero.
template <typename T>
__global__ void __launch_bounds__(WG) k_env_from_tiles(Plan p, const double *__restrict__ tiles,
                                                       T *__restrict__ erow, T *__restrict__ ecol) {
  const int g = blockIdx.x;
  const int i = find_segment(p.trow_ptr, p.N, g);
  const int g0 = p.trow_ptr[i], I = g - g0;
  const int *ep = p.eptr + p.vp_ptr[i] + i;
  const int *up = p.uptr + p.vp_ptr[i] + i;
  const long long eb = p.ebase[i];
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  const int l = I * TS + r;
  {
    const int e0 = ep[l], len = ep[l + 1] - e0, c0 = I * TS - len;
    const int fI = p.tfirst[g];
    for (int k = q; k < len; k += 4) {
      const int c = c0 + k, J = c / TS;
      const double v =
          J >= fI ? tiles[tile_elem(p.toff[g] + (J - fI)) + r * TS + (c - J * TS)] : 0.0;
      erow[eb + e0 + k] = (T)v;
    }
  }
  {
    const int e0 = up[l], len = up[l + 1] - e0, r1 = (I + 1) * TS;
    for (int k = q; k < len; k += 4) {
      const int rw = r1 + k, Ir = rw / TS, gr = g0 + Ir;
      const int fr = p.tfirst[gr];
      const double v =
          I >= fr ? tiles[tile_elem(p.toff[gr] + (I - fr)) + (rw - Ir * TS) * TS + r] : 0.0;
      ecol[eb + e0 + k] = (T)v;
    }
  }
}

// ------------------------------------------------ local solves (1 rhs) ----
// What one thread holds of a streamed piece of the factor: 16 entries, and
// for an envelope chunk the vector index paired with a[0] (entry s pairs with
// cb + 4s) and the bound kv (entries with 4s >= kv lie past the segment and
// are zero).
template <typename T>
struct Frag {
  T a[16];
  int cb, kv;
};

// Row mapping of a packed diagonal tile: row t>>2, columns 16(t&3) .. +15.
template <typename T>
__device__ __forceinline__ void row_frag_load_diag(Frag<T> &f, const T *__restrict__ dtile) {
  packed_row16(f.a, dtile, threadIdx.x >> 2, 16 * (threadIdx.x & 3));
}

template <typename T, typename C>
__device__ __forceinline__ C row_frag_dot(const Frag<T> &f, const C *v) {
  const C *vv = v + 16 * (threadIdx.x & 3);
  C s = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) s = fma((C)f.a[c], vv[c], s);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  return s;  // full row sum in all 4 lanes of the row
}

// Column mapping of a packed diagonal tile: wavefront w owns columns
// 16w .. 16w+15; lane l covers column 16w + (l & 15) and rows 16(l >> 4) ..
// +15, so a column's 64 rows sit in four lanes 16 apart.
template <typename T>
__device__ __forceinline__ void col_frag_load_diag(Frag<T> &f, const T *__restrict__ dtile) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = 16 * w + (l & 15), r0 = 16 * (l >> 4);
#pragma unroll
  for (int r = 0; r < 16; ++r) f.a[r] = packed_at(dtile, r0 + r, col);
}

// sum_r tile[r][col] x[r] for this lane's column, complete in all four lanes
// of the column (x: the 64-vector the tile multiplies, in LDS)
template <typename T, typename C>
__device__ __forceinline__ C col_frag_dot(const Frag<T> &f, const C *x) {
  const C *xx = x + 16 * ((threadIdx.x & 63) >> 4);
  C s = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) s = fma((C)f.a[r], xx[r], s);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

// Chunk j of this thread's envelope segment (seg: its first entry, len: its
// length, v0: the vector index of entry 0): entries k = 64j + (t&3) + 4s.
template <typename T>
__device__ __forceinline__ void env_chunk_load(Frag<T> &f, const T *__restrict__ seg, int len,
                                               int v0, int j) {
  const int kb = TS * j + (threadIdx.x & 3);
  f.cb = v0 + kb;
  f.kv = len - kb;
#pragma unroll
  for (int s = 0; s < 16; ++s) f.a[s] = 4 * s < f.kv ? seg[kb + 4 * s] : T(0);
}

// acc -= sum over the chunk's entries of a[s] x[cb + 4s] (partial: this
// thread's share of the segment)
template <typename T, typename C>
__device__ __forceinline__ C env_chunk_dot(const Frag<T> &f, const C *x, C acc) {
#pragma unroll
  for (int s = 0; s < 16; ++s)
    if (4 * s < f.kv) acc = fma(-(C)f.a[s], x[f.cb + 4 * s], acc);
  return acc;
}

size_t local_apply_lds_bytes(int max_npad, size_t csize) {
  return (size_t)(max_npad + TS) * csize + 2 * (size_t)(max_npad + 1) * sizeof(int);
}

// Fused additive-Schwarz local kernel for one region per workgroup:
//   gather r on the region, coarse restriction c_i = Phi_i^T r_i (optional),
//   forward/backward substitution with the factor (optional),
//   store the local correction into the padded local vector xloc.
// T: factor storage type, C: compute type, TB: basis storage type.
template <typename T, typename C, typename TB>
__global__ void __launch_bounds__(WG) k_local_apply(Plan p, const double *__restrict__ r,
                                                    const T *__restrict__ diag,
                                                    const T *__restrict__ erow,
                                                    const T *__restrict__ ecol,
                                                    const TB *__restrict__ phi,
                                                    double *__restrict__ xloc,
                                                    double *__restrict__ cvec, int do_local,
                                                    int do_coarse, const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ char smem_raw[];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  const int npad = nt * TS;
  C *v = reinterpret_cast<C *>(smem_raw);  // whole local vector (padded)
  C *tmp = v + npad;                         // 64
  int *er = reinterpret_cast<int *>(tmp + TS);  // npad + 1 row-form segment starts
  int *eu = er + npad + 1;                       // npad + 1 column-form segment starts
  __shared__ double red[MAXNEV + 1][WG / 64];
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
  if (do_local) {
    const int *ep = p.eptr + p.vp_ptr[i] + i, *up = p.uptr + p.vp_ptr[i] + i;
    for (int l = threadIdx.x; l <= npad; l += WG) {
      er[l] = ep[l];
      eu[l] = up[l];
    }
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
  const T *dpool = diag + (size_t)g0 * DE;
  const T *erow_i = erow + p.ebase[i];
  const T *ecol_i = ecol + p.ebase[i];
  // Each sweep streams, per block of 64 rows, the block's envelope chunks
  // (64 entries of every row segment each) and then its diagonal tile.  A
  // load cursor walks that sequence D + 1 pieces ahead of the consuming one;
  // D + 1 register slots hold the pieces in flight, and the slot loop is
  // unrolled so each slot is refilled in place right after its piece is used
  // (no register copies, which would wait for the loads in flight).  Segment
  // lengths are monotone inside a block (fenv nondecreasing), so the block's
  // chunk count comes from its first row (row form) or last column (column
  // form).
  constexpr int D = sizeof(T) == 4 ? 3 : 1;  // keeps 4 workgroups per CU resident
  auto nch_row = [&](int I) { return (er[I * TS + 1] - er[I * TS] + TS - 1) / TS; };
  auto nch_col = [&](int I) { return (eu[I * TS + TS] - eu[I * TS + TS - 1] + TS - 1) / TS; };
  // forward: y_I = inv(L_II) (b_I - sum_{c < 64I} L[., c] y_c)
  {
    Frag<T> f[D + 1];
    int lI = 0, lj = 0, lnch = nch_row(0);  // load cursor: block lI, chunk lj
    auto load_next = [&](Frag<T> &fr) {
      if (lj < lnch) {
        const int row = lI * TS + rr;
        const int e0 = er[row], len = er[row + 1] - e0;
        env_chunk_load(fr, erow_i + e0, len, lI * TS - len, lj);
        ++lj;
      } else {
        row_frag_load_diag(fr, dpool + (size_t)lI * DE);
        ++lI;
        lj = 0;
        if (lI < nt) lnch = nch_row(lI);
      }
    };
#pragma unroll
    for (int d = 0; d <= D; ++d)
      if (lI < nt) load_next(f[d]);
    int I = 0, j = 0, nch = nch_row(0);
    C acc = 0;
    for (;;) {
#pragma unroll
      for (int sl = 0; sl <= D; ++sl) {
        if (I < nt) {
          if (j < nch) {
            acc = env_chunk_dot<T, C>(f[sl], v, acc);
            ++j;
          } else {
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            if (q == 0) tmp[rr] = v[I * TS + rr] + acc;
            __syncthreads();
            const C y = row_frag_dot<T, C>(f[sl], tmp);
            if (q == 0) v[I * TS + rr] = y;
            __syncthreads();
            ++I;
            j = 0;
            acc = 0;
            if (I < nt) nch = nch_row(I);
          }
          if (lI < nt) load_next(f[sl]);
        }
      }
      if (I >= nt) break;
    }
  }
  // backward: x_J = inv(L_JJ)^T (y_J - sum_{r >= 64(J+1)} L[r, .]^T x_r),
  // J = nt-1 .. 0, with the column form (row c of L^T).
  {
    Frag<T> f[D + 1];
    int lI = nt - 1, lj = 0, lnch = nch_col(nt - 1);
    auto load_next = [&](Frag<T> &fr) {
      if (lj < lnch) {
        const int c = lI * TS + rr;
        const int e0 = eu[c], len = eu[c + 1] - e0;
        env_chunk_load(fr, ecol_i + e0, len, (lI + 1) * TS, lj);
        ++lj;
      } else {
        col_frag_load_diag(fr, dpool + (size_t)lI * DE);
        --lI;
        lj = 0;
        if (lI >= 0) lnch = nch_col(lI);
      }
    };
#pragma unroll
    for (int d = 0; d <= D; ++d)
      if (lI >= 0) load_next(f[d]);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = 16 * w + (l & 15);
    const bool head = (l >> 4) == 0;  // one lane of the four that share a column
    int I = nt - 1, j = 0, nch = nch_col(nt - 1);
    C acc = 0;
    for (;;) {
#pragma unroll
      for (int sl = 0; sl <= D; ++sl) {
        if (I >= 0) {
          if (j < nch) {
            acc = env_chunk_dot<T, C>(f[sl], v, acc);
            ++j;
          } else {
            acc += __shfl_xor(acc, 1, 64);
            acc += __shfl_xor(acc, 2, 64);
            if (q == 0) tmp[rr] = v[I * TS + rr] + acc;
            __syncthreads();  // tmp complete
            const C x = col_frag_dot<T, C>(f[sl], tmp);
            if (head) v[I * TS + col] = x;
            __syncthreads();  // x_I visible; all reads of tmp done
            --I;
            j = 0;
            acc = 0;
            if (I >= 0) nch = nch_col(I);
          }
          if (lI >= 0) load_next(f[sl]);
        }
      }
      if (I < 0) break;
    }
  }
  // local correction in the region's ascending-global-index layout, so that
  // the scatter reads contiguous runs
  double *dst = xloc + p.vp_ptr[i];
  for (int l = threadIdx.x; l < ni; l += WG) dst[p.nat[r0 + l]] = (double)v[l];
}

// ------------------------------------ block solve on MFMA (EIGP rhs) ------
// In-place (L L^T)^{-1} X for a row-major padded block X[rows][EIGP] (the
// subspace block of the local eigensolver), one workgroup (4 wavefronts) per
// region; regions flagged in skip[] are left untouched.  Wavefront w owns
// rows 16w..16w+15 of the 64 x EIGP block of the
// current tile row.  A 64x64 tile times the 64x16 block is 16 MFMA steps;
// K-slot q of step s stands for column k = 16q + s, so that each lane reads
// 16 contiguous entries of one tile row (non-transposed products) and the
// transposed products read 16 consecutive columns per instruction.
// packed: the tile is a packed diagonal tile (zero above the diagonal).
template <typename T>
__device__ __forceinline__ d4 mfma_tile_rhs(const T *__restrict__ tile, const double *rhs, int w,
                                            int transpose, int packed, d4 acc, double sign) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, q = l >> 4;
  T t[16];
  if (!transpose) {
    if (packed) {
      packed_row16(t, tile, 16 * w + i, 16 * q);
    } else {
      const T *row = tile + (16 * w + i) * TS + 16 * q;
#pragma unroll
      for (int s = 0; s < 16; ++s) t[s] = row[s];
    }
  } else if (packed) {
#pragma unroll
    for (int s = 0; s < 16; ++s) t[s] = packed_at(tile, 16 * q + s, 16 * w + i);
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) t[s] = tile[(16 * q + s) * TS + 16 * w + i];
  }
#pragma unroll
  for (int s = 0; s < 16; ++s)
    acc = mfma16x16x4(sign * (double)t[s], rhs[(16 * q + s) * (EIGP + 1) + i], acc);
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
      acc = mfma_tile_rhs<T>(tiles + tile_elem(tI + (J - fI)), V, w, 0, 0, acc, -1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Acc[(rb + 4 * r) * LV + col] = acc[r];
    __syncthreads();
    d4 y = {0.0, 0.0, 0.0, 0.0};
    y = mfma_tile_rhs<T>(tiles + diag_elem(p, g0 + I), Acc, w, 0, 1, y, 1.0);
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
      acc = mfma_tile_rhs<T>(tiles + tile_elem(p.toff[g0 + J] + (I - fJ)), V, w, 1, 0, acc, -1.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Acc[(rb + 4 * r) * LV + col] = acc[r];
    __syncthreads();
    d4 y = {0.0, 0.0, 0.0, 0.0};
    y = mfma_tile_rhs<T>(tiles + diag_elem(p, g0 + I), Acc, w, 1, 1, y, 1.0);
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

template <typename T>
void launch_env_from_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *tiles,
                           T *erow, T *ecol) {
  hipLaunchKernelGGL((k_env_from_tiles<T>), dim3(ntilerows), dim3(WG), 0, s, p, tiles, erow, ecol);
}
template void launch_env_from_tiles<double>(hipStream_t, const Plan &, int, const double *,
                                            double *, double *);
template void launch_env_from_tiles<float>(hipStream_t, const Plan &, int, const double *,
                                           float *, float *);

template <typename T, typename C, typename TB>
void launch_local_apply_t(hipStream_t s, const Plan &p, int max_npad, const double *r,
                          const T *diag, const T *erow, const T *ecol, const TB *phi,
                          double *xloc, double *cvec, int do_local, int do_coarse,
                          const int *done, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const size_t sm = local_apply_lds_bytes(max_npad, sizeof(C));
  allow_lds(k_local_apply<T, C, TB>, sm);
  if (ev_start || ev_stop)  // events bound to this dispatch: exact kernel duration
    hipExtLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, ev_start, ev_stop,
                          0, p, r, diag, erow, ecol, phi, xloc, cvec, do_local, do_coarse, done);
  else
    hipLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, p, r, diag, erow,
                       ecol, phi, xloc, cvec, do_local, do_coarse, done);
}

#define AMSP_LOCAL_APPLY_INST(T, C, TB)                                                        \
  template void launch_local_apply_t<T, C, TB>(hipStream_t, const Plan &, int, const double *, \
                                               const T *, const T *, const T *, const TB *,    \
                                               double *, double *, int, int, const int *,      \
                                               hipEvent_t, hipEvent_t);
AMSP_LOCAL_APPLY_INST(double, double, double)
AMSP_LOCAL_APPLY_INST(float, float, float)
AMSP_LOCAL_APPLY_INST(float, float, __hip_bfloat16)
#undef AMSP_LOCAL_APPLY_INST

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
