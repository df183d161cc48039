// Per-subdomain local matrices, their batched tile-profile Cholesky
// factorisation, the envelope copy the solves read, and the scatter that sums
// the additive Schwarz terms.
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
#include "k_common.h"

namespace amsp {

// ------------------------------------------------------- inverse map -----
// mult[j] = number of regions containing dof j, inv_ptr = exclusive scan of
// mult, and each dof's list (subdomain, position in the region's
// ascending-global-index layout) ordered by subdomain: counts and fill by
// atomic increments, then every short list sorted in place, so the result
// does not depend on the order of the increments.
// mult = fill = 0, *max_mult = 0
__global__ void k_fill_int_dev(int n, int *__restrict__ mult, int *__restrict__ fill,
                               int *__restrict__ max_mult) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    mult[j] = 0;
    fill[j] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *max_mult = 0;
}

__global__ void __launch_bounds__(WG) k_count_mult(Plan p, int *__restrict__ mult) {
  const int i = blockIdx.x;
  for (int k = p.sd_ptr[i] + threadIdx.x; k < p.sd_ptr[i + 1]; k += WG)
    atomicAdd(&mult[p.sd_dofs[k]], 1);
}

// exclusive scan in three passes: block totals (SCB entries per block), a
// scan of the totals by one workgroup, then each block's entries
constexpr int SCB = 4 * WG;
__global__ void __launch_bounds__(WG) k_scan_totals(int n, const int *__restrict__ in,
                                                    int *__restrict__ tot) {
  __shared__ int sh[WG / 64];
  const int b0 = blockIdx.x * SCB;
  int acc = 0;
  for (int u = 0; u < 4; ++u) {
    const int j = b0 + u * WG + threadIdx.x;
    if (j < n) acc += in[j];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < WG / 64; ++w) t += sh[w];
    tot[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(WG) k_scan_offsets(int nb, int *__restrict__ tot) {
  __shared__ int sh[WG];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += WG) {
    const int j = c0 + threadIdx.x;
    const int v = j < nb ? tot[j] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < WG; o <<= 1) {  // inclusive scan (Hillis-Steele)
      const int a = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += a;
      __syncthreads();
    }
    if (j < nb) tot[j] = carry + sh[threadIdx.x] - v;  // exclusive
    carry += sh[WG - 1];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(WG) k_scan_apply(int n, const int *__restrict__ in,
                                                   const int *__restrict__ off,
                                                   int *__restrict__ out) {
  __shared__ int wt[WG / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j0 = blockIdx.x * SCB + 4 * t;  // this thread's four consecutive entries
  int v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = j0 + u < n ? in[j0 + u] : 0;
  const int s4 = v[0] + v[1] + v[2] + v[3];
  int x = s4;  // inclusive scan over the wavefront
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wt[w] = x;
  __syncthreads();
  int e = off[blockIdx.x] + x - s4;
  for (int ww = 0; ww < w; ++ww) e += wt[ww];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (j0 + u < n) out[j0 + u] = e;
    e += v[u];
  }
  if (blockIdx.x == gridDim.x - 1 && t == WG - 1) out[n] = e;  // the total (entries past n are 0)
}

__global__ void __launch_bounds__(WG) k_fill_inverse(Plan p, const int *__restrict__ inv_ptr,
                                                     int *__restrict__ fill, int *__restrict__ inv_sd,
                                                     int *__restrict__ inv_loc) {
  const int i = blockIdx.x;
  for (int k = p.sd_ptr[i] + threadIdx.x; k < p.sd_ptr[i + 1]; k += WG) {
    const int g = p.sd_dofs[k];
    const int at = inv_ptr[g] + atomicAdd(&fill[g], 1);
    inv_sd[at] = i;
    inv_loc[at] = p.nat[k];
  }
}

__global__ void __launch_bounds__(WG) k_sort_inverse(int n, const int *__restrict__ inv_ptr,
                                                     int *__restrict__ inv_sd,
                                                     int *__restrict__ inv_loc,
                                                     int *__restrict__ max_mult) {
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= n) return;
  const int a = inv_ptr[j], b = inv_ptr[j + 1];
  for (int e = a + 1; e < b; ++e) {
    const int sd = inv_sd[e], lc = inv_loc[e];
    int y = e;
    while (y > a && inv_sd[y - 1] > sd) {
      inv_sd[y] = inv_sd[y - 1];
      inv_loc[y] = inv_loc[y - 1];
      --y;
    }
    inv_sd[y] = sd;
    inv_loc[y] = lc;
  }
  atomicMax(max_mult, b - a);
}

// ----------------------------------------------------- local CSR ---------
// The local CSR of every region, rows in local order, columns ascending:
// the entries of A's row dof(l) whose column is in the region, with their
// local index and the position of the value in A's CSR.  One workgroup per
// region; the region's dofs sorted by global index (and the local index of
// each) are staged in LDS (or in global scratch when the largest region does
// not fit), looked up by binary search; each row is written in place by
// insertion (rows are short).  Row pointers come from the host plan.
__global__ void __launch_bounds__(WG) k_local_csr(Plan p, const int *__restrict__ rowptr,
                                                  const int *__restrict__ col,
                                                  int *__restrict__ loc_col,
                                                  int *__restrict__ loc_src, int *gscratch,
                                                  int use_lds) {
  extern __shared__ int lds_i[];
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  int *sorted = use_lds ? lds_i : gscratch + 2 * (size_t)r0;
  int *r2l = sorted + ni;
  for (int l = threadIdx.x; l < ni; l += WG) {
    const int rk = p.nat[r0 + l];
    sorted[rk] = p.sd_dofs[r0 + l];
    r2l[rk] = l;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < ni; l += WG) {
    const int g = p.sd_dofs[r0 + l];
    const int o0 = p.loc_rowptr[r0 + l];
    int cnt = 0;
    for (int e = rowptr[g]; e < rowptr[g + 1]; ++e) {
      const int c = col[e];
      int lo = 0, hi = ni;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sorted[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo == ni || sorted[lo] != c) continue;
      const int lc = r2l[lo];
      int y = o0 + cnt++;
      while (y > o0 && loc_col[y - 1] > lc) {
        loc_col[y] = loc_col[y - 1];
        loc_src[y] = loc_src[y - 1];
        --y;
      }
      loc_col[y] = lc;
      loc_src[y] = e;
    }
  }
}

void launch_inverse_map(hipStream_t s, const Plan &p, int n, int *mult, int *inv_ptr,
                        int *inv_sd, int *inv_loc, int *work, int *max_mult) {
  if (n <= 0 || p.N == 0) return;
  const int nb = (n + SCB - 1) / SCB;
  int *fill = work, *tot = work + n;  // work: n + nb ints
  const int zb = (n + WG - 1) / WG;
  hipLaunchKernelGGL(k_fill_int_dev, dim3(zb < 16384 ? zb : 16384), dim3(WG), 0, s, n, mult, fill,
                     max_mult);
  hipLaunchKernelGGL(k_count_mult, dim3(p.N), dim3(WG), 0, s, p, mult);
  hipLaunchKernelGGL(k_scan_totals, dim3(nb), dim3(WG), 0, s, n, mult, tot);
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(WG), 0, s, nb, tot);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(WG), 0, s, n, mult, tot, inv_ptr);
  hipLaunchKernelGGL(k_fill_inverse, dim3(p.N), dim3(WG), 0, s, p, inv_ptr, fill, inv_sd, inv_loc);
  hipLaunchKernelGGL(k_sort_inverse, dim3((n + WG - 1) / WG), dim3(WG), 0, s, n, inv_ptr, inv_sd,
                     inv_loc, max_mult);
}

size_t local_csr_lds_bytes(int max_ni) { return (size_t)2 * max_ni * sizeof(int); }

void launch_local_csr(hipStream_t s, const Plan &p, int max_ni, const int *rowptr, const int *col,
                      int *loc_col, int *loc_src, int *gscratch) {
  if (p.N == 0) return;
  const size_t sm = local_csr_lds_bytes(max_ni);
  const int use_lds = sm <= LOCAL_CSR_LDS_MAX ? 1 : 0;
  if (use_lds) allow_lds(k_local_csr, sm);
  hipLaunchKernelGGL(k_local_csr, dim3(p.N), dim3(WG), use_lds ? sm : 0, s, p, rowptr, col, loc_col,
                     loc_src, gscratch, use_lds);
}

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
  // the row's first RE entries (local column and value, scaled in mode 1),
  // loaded once for all its tiles with clamped indices, every load issued;
  // longer rows take the rest one by one in each tile
  constexpr int RE = 8;
  int ec[RE];
  double ea[RE];
#pragma unroll
  for (int k = 0; k < RE; ++k) {
    ec[k] = -TS;
    ea[k] = 0.0;
  }
  if (real) {  // a row of the region has at least its diagonal entry
    const int el = e1 - 1;
    int es[RE];
#pragma unroll
    for (int k = 0; k < RE; ++k) {
      const int e = min(e0 + k, el);
      ec[k] = p.loc_col[e];
      es[k] = p.loc_src[e];
    }
#pragma unroll
    for (int k = 0; k < RE; ++k) ea[k] = val[es[k]];
    if (mode == 1) {
      double sc[RE];
#pragma unroll
      for (int k = 0; k < RE; ++k) sc[k] = sdiag[r0 + ec[k]];
#pragma unroll
      for (int k = 0; k < RE; ++k) ea[k] = (ec[k] == l) ? 1.0 + sigma : ea[k] / sqrt(sl * sc[k]);
    }
#pragma unroll
    for (int k = 0; k < RE; ++k)
      if (e0 + k >= e1) ec[k] = -TS;  // no entry: never inside a tile
  }
  for (int J = fI; J <= I; ++J) {
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = 0.0;
    const int cbase = J * TS + 16 * q;
    if (real) {
#pragma unroll
      for (int k = 0; k < RE; ++k) {
        const int off = ec[k] - cbase;
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c == off) v[c] = ea[k];
      }
      for (int e = e0 + RE; e < e1; ++e) {
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

// Per-sweep streams of the f32 factor (layout in amsp_internal.h), one
// workgroup per tile row g: the forward block of g (row-form segments,
// padding, diagonal) and its backward block (column-form segments, padding,
// diagonal).
__global__ void __launch_bounds__(WG) k_stream_from_tiles(Plan p, const double *__restrict__ tiles,
                                                          float *__restrict__ fst,
                                                          float *__restrict__ bst) {
  const int g = blockIdx.x;
  const int i = find_segment(p.trow_ptr, p.N, g);
  const int g0 = p.trow_ptr[i], I = g - g0;
  const int *ep = p.eptr + p.vp_ptr[i] + i, *up = p.uptr + p.vp_ptr[i] + i;
  const int r0 = I * TS;
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
  const int l = r0 + r;
  const double *dg = tiles + diag_elem(p, g);
  // forward block
  {
    float *blk = fst + p.sfr[i] + p.sfb[g];
    const int base = ep[r0], T = ep[r0 + TS] - base, Tp = (T + 3) & ~3;
    const int e0 = ep[l] - base, len = ep[l + 1] - ep[l], c0 = r0 - len;
    const int fI = p.tfirst[g];
    for (int k = q; k < len; k += 4) {
      const int c = c0 + k, J = c / TS;
      const double v =
          J >= fI ? tiles[tile_elem(p.toff[g] + (J - fI)) + r * TS + (c - J * TS)] : 0.0;
      blk[e0 + k] = (float)v;
    }
    if ((int)threadIdx.x < Tp - T) blk[T + threadIdx.x] = 0.f;
    for (int e = threadIdx.x; e < DE; e += WG) blk[Tp + e] = (float)dg[e];
  }
  // backward block
  {
    float *blk = bst + p.sbr[i] + p.sbb[g];
    const int base = up[r0], T = up[r0 + TS] - base, Tp = (T + 3) & ~3;
    const int e0 = up[l] - base, len = up[l + 1] - up[l], r1 = r0 + TS;
    for (int k = q; k < len; k += 4) {
      const int rw = r1 + k, Ir = rw / TS, gr = g0 + Ir;
      const int fr = p.tfirst[gr];
      const double v =
          I >= fr ? tiles[tile_elem(p.toff[gr] + (I - fr)) + (rw - Ir * TS) * TS + r] : 0.0;
      blk[e0 + k] = (float)v;
    }
    if ((int)threadIdx.x < Tp - T) blk[T + threadIdx.x] = 0.f;
    for (int e = threadIdx.x; e < DE; e += WG) blk[Tp + e] = (float)dg[e];
  }
}

void launch_stream_from_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *tiles,
                              float *fst, float *bst) {
  hipLaunchKernelGGL(k_stream_from_tiles, dim3(ntilerows), dim3(WG), 0, s, p, tiles, fst, bst);
}

// Device self-test of the MFMA operand/result layout the kernels rely on: D = A B
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
// Direct indices of the inverse map, formed once at setup so that the scatter
// reads each entry's operands without going through its region's offsets:
//   ix = vp_ptr[sd] + l     (local correction),
//   ip = sd_ptr[sd] + l     (basis row, ascending-index layout),
//   ic = coff[sd] * 16 + m_sd  (coarse offset and count; m <= MAXNEV < 16).
__global__ void k_inverse_direct(int ne, const int *__restrict__ inv_sd,
                                 const int *__restrict__ inv_loc, Plan p, int *__restrict__ ix) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x)
    ix[e] = p.vp_ptr[inv_sd[e]] + inv_loc[e];
}

// Coarse prolongation per region, into the local output: w_i = x_i + Phi_i t_i
// (or Phi_i t_i alone without the local part), in the region's
// ascending-global-index layout, with Phi_i = D_i psi (the basis copy in that
// layout, column after column).  Grid (row block, region); one row per thread.
template <typename TB>
__global__ void __launch_bounds__(WG) k_prolong_local(Plan p, const TB *__restrict__ phi,
                                                      const double *__restrict__ t,
                                                      double *__restrict__ xloc, int do_local,
                                                      const int *__restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.y;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int pos = blockIdx.x * WG + threadIdx.x;
  if (pos >= ni) return;
  const int m = p.mi[i], nev = p.nev;
  const double *tt = t + p.coff[i];
  double *dst = xloc + p.vp_ptr[i] + pos;
  double v = do_local ? *dst : 0.0;
  if (m == 0) {
    *dst = v;
    return;
  }
  with_km(nev, [&](auto km) __attribute__((always_inline)) {
    constexpr int KM = decltype(km)::value;
    TB raw[KM];
    double tk[KM];
    basis_row_load<KM>(phi + (size_t)r0 * nev + pos, (size_t)ni, m, raw);
#pragma unroll
    for (int q = 0; q < KM; ++q) tk[q] = tt[min(q, m - 1)];
#pragma unroll
    for (int q = 0; q < KM; ++q) v = fma(basis_coef<KM>(raw, q, m), tk[q], v);
  });
  *dst = v;
}

// z[j] = sum over the copies of dof j (regions containing j, in the fixed
// order of the inverse map; no atomics) of the region outputs, and the
// partial r.z.  A thread takes SU consecutive dofs, whose copies are one
// contiguous run of the map: the first SC copies are loaded together (index,
// then value), any further ones one by one.
constexpr int SU = 4, SC = 8;
__global__ void __launch_bounds__(WG) k_scatter_sum(int n, const int *__restrict__ inv_ptr,
                                                    const int *__restrict__ ix,
                                                    const double *__restrict__ xloc,
                                                    double *__restrict__ z,
                                                    const double *__restrict__ r,
                                                    double *__restrict__ partial,
                                                    const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[WG / 64];
  const int stride = gridDim.x * WG;
  double acc = 0.0;
  for (int g = blockIdx.x * WG + threadIdx.x; g < (n + SU - 1) / SU; g += stride) {
    const int j0 = g * SU;
    int e[SU + 1];
#pragma unroll
    for (int u = 0; u <= SU; ++u) e[u] = inv_ptr[min(j0 + u, n)];
    double rj[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) rj[u] = r ? r[min(j0 + u, n - 1)] : 0.0;
    // the first SC copies' indices, then values, with the positions clamped
    // into the run and every load issued (a load under a per-lane condition
    // would be waited for inside its branch); copies past the run are
    // dropped by the range test of the sums
    const int klast = max(e[SU] - 1, 0);
    int idx[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) idx[c] = ix[min(e[0] + c, klast)];
    double x[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) x[c] = xloc[idx[c]];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      double zj = 0.0;
#pragma unroll
      for (int c = 0; c < SC; ++c) {
        const int k = e[0] + c;
        if (k >= e[u] && k < e[u + 1]) zj += x[c];
      }
      for (int k = max(e[u], e[0] + SC); k < e[u + 1]; ++k) zj += xloc[ix[k]];
      const int j = j0 + u;
      if (j < n) {
        z[j] = zj;
        if (r) acc = fma(rj[u], zj, acc);
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
    dst[(size_t)r0 * nev + (size_t)c * ni + p.nat[r0 + l]] = src[(size_t)(r0 + l) * nev + c];
  }
}

// asc[r0 + nat[r0 + l]] = sd_dofs[r0 + l], lop[r0 + nat[r0 + l]] = l: each
// region's dofs in ascending order (the row order of the ascending-index
// layout) and their local indices.
__global__ void __launch_bounds__(WG) k_ascending_dofs(Plan p, int *__restrict__ asc,
                                                       int *__restrict__ lop) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  for (int l = threadIdx.x; l < ni; l += WG) {
    const int pos = r0 + p.nat[r0 + l];
    asc[pos] = p.sd_dofs[r0 + l];
    lop[pos] = l;
  }
}

// ------------------------------------------------------------- launchers ---
void launch_ascending_dofs(hipStream_t s, const Plan &p, int *asc, int *lop) {
  hipLaunchKernelGGL(k_ascending_dofs, dim3(p.N), dim3(WG), 0, s, p, asc, lop);
}

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


void launch_inverse_direct(hipStream_t s, int ne, const int *inv_sd, const int *inv_loc,
                           const Plan &p, int *ix) {
  size_t b = ((size_t)ne + WG - 1) / WG;
  if (b > 65535) b = 65535;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_inverse_direct, dim3((unsigned)b), dim3(WG), 0, s, ne, inv_sd, inv_loc, p, ix);
}

template <typename TB>
void launch_scatter_sum_t(hipStream_t s, const Plan &p, int max_ni, int n, const int *inv_ptr,
                          const int *ix, double *xloc, const TB *phi, const double *t, double *z,
                          const double *r, double *partial, int do_local, int do_coarse,
                          const int *done) {
  if (do_coarse && max_ni > 0)
    hipLaunchKernelGGL((k_prolong_local<TB>), dim3((max_ni + WG - 1) / WG, p.N), dim3(WG), 0, s, p,
                       phi, t, xloc, do_local, done);
  // one partial per workgroup of the usual reduction grid, which the
  // consumers of r.z expect (the surplus workgroups add zeros)
  hipLaunchKernelGGL(k_scatter_sum, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, inv_ptr, ix, xloc, z,
                     r, partial, done);
}
#define AMSP_SCATTER_INST(TB)                                                                   \
  template void launch_scatter_sum_t<TB>(hipStream_t, const Plan &, int, int, const int *,     \
                                         const int *, double *, const TB *, const double *,    \
                                         double *, const double *, double *, int, int,         \
                                         const int *);
AMSP_SCATTER_INST(double)
AMSP_SCATTER_INST(float)
AMSP_SCATTER_INST(__hip_bfloat16)
#undef AMSP_SCATTER_INST

}  // namespace amsp
