// The local solves of the additive Schwarz term (Section 3.2): one fused
// kernel per application of the preconditioner gathers the residual on every
// region, runs the forward and backward substitutions with the region's
// factor, stored as packed inverse diagonal tiles plus the envelope below
// them (see k_local.hip), and adds the coarse prolongation Phi_i t_i to the
// region's output.  The coarse restriction Phi_i^T r_i, which the coarse
// solve needs first, is a kernel of its own (k_restrict).
#include <hip/hip_ext.h>

#include "k_common.h"

namespace amsp {

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

// dst[l] = src[l] for l < cnt (LDS from global), each thread's loads all in
// flight together when cnt <= U * WG: they are clamped into range and
// issued unconditionally, and the stores of rows past cnt go to
// junk[threadIdx.x % 64] (scratch), so that no load waits inside a branch.
template <int U>
__device__ __forceinline__ void copy_ints_to_lds(int *dst, const int *__restrict__ src, int cnt,
                                                 int *junk) {
  if (cnt <= U * WG) {
    int x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = src[min((int)threadIdx.x + u * WG, cnt - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = threadIdx.x + u * WG;
      (l < cnt ? dst[l] : junk[threadIdx.x & (TS - 1)]) = x[u];
    }
  } else {
    for (int l = threadIdx.x; l < cnt; l += WG) dst[l] = src[l];
  }
}

// Restriction of one region with at most KM basis coefficients per row (see
// k_restrict).
template <int KM, typename TB>
__device__ __forceinline__ void restrict_region(const Plan &p, int i, const double *__restrict__ r,
                                                const TB *__restrict__ phi,
                                                double *__restrict__ cvec, double (*red)[WG / 64]) {
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int m = p.mi[i];
  if (m == 0) return;
  const TB *phr = phi + (size_t)r0 * p.nev;
  double cacc[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) cacc[k] = 0.0;
  // rows per thread per pass (one pass covers regions up to GU * WG rows)
  constexpr int GU = (sizeof(TB) == 8 ? 4 : 8) / (KM <= 8 ? 1 : 2);
  for (int l0 = threadIdx.x; l0 < ni; l0 += GU * WG) {
    int dof[GU];
    double rv[GU];
    TB raw[GU][KM];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int lc = min(l0 + u * WG, ni - 1);  // clamped: every load is issued
      dof[u] = p.asc[r0 + lc];
      basis_row_load<KM>(phr + lc, (size_t)ni, m, raw[u]);
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) rv[u] = r[dof[u]];
#pragma unroll
    for (int u = 0; u < GU; ++u) rv[u] = l0 + u * WG < ni ? rv[u] : 0.0;
#pragma unroll
    for (int u = 0; u < GU; ++u)
#pragma unroll
      for (int k = 0; k < KM; ++k) cacc[k] = fma(basis_coef<KM>(raw[u], k, m), rv[u], cacc[k]);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < KM; ++k)
    if (k < m) {
      const double s = wave_sum(cacc[k]);
      if (lane == 0) red[k][w] = s;
    }
  __syncthreads();
  if (threadIdx.x < m) {
    double s = 0.0;
    for (int ww = 0; ww < WG / 64; ++ww) s += red[threadIdx.x][ww];
    cvec[p.coff[i] + threadIdx.x] = s;
  }
}

// Coarse restriction c_i = Phi_i^T r_i (the coarse term R0 r of the two-level
// operator, Section 3.1), one region per workgroup, over the region's rows in
// ascending global order (Plan::asc) with the basis stored column after
// column in that order, so that neighbouring lanes read neighbouring entries
// of r and of every basis column.  Each thread takes the rows t, t + WG, ...
// in order (several rows' loads issued together), then the wavefronts' sums
// are added in a fixed order (no atomics).
template <typename TB>
__global__ void __launch_bounds__(WG) k_restrict(Plan p, const double *__restrict__ r,
                                                 const TB *__restrict__ phi,
                                                 double *__restrict__ cvec,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double red[MAXNEV][WG / 64];
  with_km(p.nev, [&](auto km) __attribute__((always_inline)) {
    restrict_region<decltype(km)::value>(p, blockIdx.x, r, phi, cvec, red);
  });
}

// Region i's output with the prolongation added (at most KM coefficients per
// row), row by row in the ascending-index layout: dst[pos] = x_l +
// sum_q Phi_i[pos][q] t_q for the local index l of position pos, the
// coefficients taken in order (the same arithmetic as k_prolong_local).
template <int KM, typename TB, typename V>
__device__ __forceinline__ void store_local_prolong(const Plan &p, int r0, int ni, int m,
                                                    const V *v, const TB *__restrict__ phi,
                                                    const double *tt, double *__restrict__ dst) {
  const TB *phr = phi + (size_t)r0 * p.nev;
  double tk[KM];
#pragma unroll
  for (int q = 0; q < KM; ++q) tk[q] = q < m ? tt[min(q, m - 1)] : 0.0;
  constexpr int GU = KM <= 8 ? 2 : 1;
  for (int l0 = threadIdx.x; l0 < ni; l0 += GU * WG) {
    TB raw[GU][KM];
    int lo[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int pos = min(l0 + u * WG, ni - 1);
      lo[u] = p.lop[r0 + pos];
      basis_row_load<KM>(phr + pos, (size_t)ni, m, raw[u]);
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int pos = l0 + u * WG;
      if (pos < ni) {
        double x = (double)v[lo[u]];
#pragma unroll
        for (int q = 0; q < KM; ++q) x = fma(basis_coef<KM>(raw[u], q, m), tk[q], x);
        dst[pos] = x;
      }
    }
  }
}

// Region i's output x_i (v, local order) into xloc in the region's
// ascending-global-index layout (written in that order); with the region's
// coarse values tq (its m_i entries of the coarse solution; else nullptr),
// the prolongation Phi_i t_i is added (phi: the basis copy in that layout,
// column after column).
template <typename TB, typename V>
__device__ __forceinline__ void store_local(const Plan &p, int i, int r0, int ni, const V *v,
                                            const TB *__restrict__ phi, const double *tq,
                                            double *__restrict__ xloc) {
  double *dst = xloc + p.vp_ptr[i];
  const int m = tq ? p.mi[i] : 0;
  if (m == 0) {
    for (int pos = threadIdx.x; pos < ni; pos += WG) dst[pos] = (double)v[p.lop[r0 + pos]];
  } else {
    with_km(p.nev, [&](auto km) __attribute__((always_inline)) {
      store_local_prolong<decltype(km)::value>(p, r0, ni, m, v, phi, tq, dst);
    });
  }
}

// The region's coarse values from the per-tile products of W0^T t1
// (launch_trmv with y == nullptr), summed exactly as k_trmv_reduce sums
// them.  Thread (q, g) = (t / TRMV_RG, t % TRMV_RG), q < m_i, adds piece g
// of entry coff_i + q (coarse_partial_load, early: its loads then overlap the
// gather); coarse_partial_finish adds the pieces in order inside each
// 16-lane group and leaves the m_i values in tq (LDS; visible after the
// next barrier).
static_assert(MAXNEV * TRMV_RG <= WG, "one thread per (coarse value, piece)");
__device__ __forceinline__ double coarse_partial_load(const Plan &p, int i,
                                                      const double *__restrict__ part, int T0) {
  const int q = threadIdx.x / TRMV_RG, g = threadIdx.x % TRMV_RG;
  double s = 0.0;
  if (q < p.mi[i]) {
    const int gi = p.coff[i] + q, O = gi / TS, r = gi % TS;
    const int len = T0 - O;
    const int a = O + (len * g) / TRMV_RG, b = O + (len * (g + 1)) / TRMV_RG;
    const double *src = part + (size_t)O * T0 * TS + r;
    constexpr int U = 8;  // loads in flight together; added in order
    for (int K0 = a; K0 < b; K0 += U) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = K0 + u < b ? src[(size_t)(K0 + u) * TS] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (K0 + u < b) s += x[u];
    }
  }
  return s;
}
__device__ __forceinline__ void coarse_partial_finish(const Plan &p, int i, double s, double *tq) {
  const int lane = threadIdx.x & 63, base = lane & ~(TRMV_RG - 1);
  double tot = 0.0;
#pragma unroll
  for (int g = 0; g < TRMV_RG; ++g) tot += __shfl(s, base + g, 64);
  const int q = threadIdx.x / TRMV_RG;
  if (threadIdx.x % TRMV_RG == 0 && q < p.mi[i]) tq[q] = tot;
}

size_t local_apply_lds_bytes(int max_npad, size_t csize) {
  return (size_t)(max_npad + TS) * csize + 2 * (size_t)(max_npad + 1) * sizeof(int);
}

// Fused additive-Schwarz local kernel for one region per workgroup:
//   gather r on the region, forward/backward substitution with the factor,
//   store the local correction (plus Phi_i t_i when t is given) into xloc.
// T: factor storage type, C: compute type, TB: basis storage type.
template <typename T, typename C, typename TB>
__global__ void __launch_bounds__(WG) k_local_apply(Plan p, const double *__restrict__ r,
                                                    const T *__restrict__ diag,
                                                    const T *__restrict__ erow,
                                                    const T *__restrict__ ecol,
                                                    const TB *__restrict__ phi,
                                                    const double *__restrict__ t,
                                                    const double *__restrict__ tpart, int T0,
                                                    double *__restrict__ xloc,
                                                    const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ char smem_raw[];
  __shared__ double tq_s[16];  // the region's coarse values (a multiple of 16 bytes)
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  const int npad = nt * TS;
  C *v = reinterpret_cast<C *>(smem_raw);  // whole local vector (padded)
  C *tmp = v + npad;                         // 64
  int *er = reinterpret_cast<int *>(tmp + TS);  // npad + 1 row-form segment starts
  int *eu = er + npad + 1;                       // npad + 1 column-form segment starts
  const double cps = tpart ? coarse_partial_load(p, i, tpart, T0) : 0.0;
  {  // gather, nothing conditional (as in the stream kernel; tmp takes the
     // stores of rows past the padding)
    constexpr int GU = 4;
    for (int l0 = threadIdx.x; l0 < npad; l0 += GU * WG) {
      int dof[GU];
      double rv[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) dof[u] = p.sd_dofs[r0 + min(l0 + u * WG, ni - 1)];
#pragma unroll
      for (int u = 0; u < GU; ++u) rv[u] = r[dof[u]];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int l = l0 + u * WG;
        v[l < npad ? l : npad + (threadIdx.x & (TS - 1))] = l < ni ? (C)rv[u] : C(0);
      }
    }
  }
  {
    const int *ep = p.eptr + p.vp_ptr[i] + i, *up = p.uptr + p.vp_ptr[i] + i;
    int *junk = reinterpret_cast<int *>(tmp);  // scratch until the sweeps
    copy_ints_to_lds<8>(er, ep, npad + 1, junk);
    copy_ints_to_lds<8>(eu, up, npad + 1, junk);
  }
  if (tpart) coarse_partial_finish(p, i, cps, tq_s);
  const double *tq = tpart ? tq_s : (t ? t + p.coff[i] : nullptr);
  __syncthreads();
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
  // local correction (+ prolongation) in the region's ascending-global-index
  // layout, so that the scatter reads contiguous runs
  store_local(p, i, r0, ni, v, phi, tq, xloc);
}

// ------------------------------------ local solves on the f32 streams -----
// The mixed-form local apply reads each sweep's data as one contiguous
// stream per region (envelope segments then packed diagonal tile, block by
// block in sweep order).  The workgroup loads it in 4 KB units (16 bytes per
// thread, every byte used), in batches of NS units: while one batch is used
// the next is in flight.  An arriving batch is copied into an LDS ring of RU
// units behind one barrier, and the row and column products read the ring.
// Envelope entries are used as soon as their unit has arrived; a block's
// diagonal step runs once its whole tile is in the ring.
// The ring is large enough that a unit is overwritten only after every read
// of it has finished.  While batch j (units k .. k + NS - 1) is used, reads
// touch envelope entries of batch j and diagonal tiles that end in batch j,
// which start no earlier than unit k - 3 (DE = 2.125 units).  Writing batch
// j + 1 replaces units k + NS - RU .. k + 2 NS - 1 - RU, i.e. batch j - 1 when
// RU = 2 NS.  Every diagonal step ends with a barrier, so the writer of batch
// j + 1 can overlap only envelope reads of batch j; and the diagonal tiles
// read in batch j + 1 start no earlier than unit k + NS - 3 >= k for NS >= 3.
namespace stream {
typedef float f4 __attribute__((ext_vector_type(4)));  // one thread's 16 bytes of a unit
constexpr int UE = 4 * WG;   // floats per unit
constexpr int NS = 3;        // units per batch (and in flight per thread)
constexpr int RU = 2 * NS;   // units in the LDS ring
constexpr int RSZ = RU * UE;
static_assert(NS >= 3, "a diagonal tile may start three units before the batch it ends in");
}  // namespace stream

// The region's coarse values (MAXNEV doubles, padded to 16 so that what
// follows stays 16-byte aligned) head the stream kernel's LDS.
constexpr size_t TQ_BYTES = 16 * sizeof(double);
static_assert(MAXNEV <= 16, "coarse values of one region");

size_t local_apply_stream_lds_bytes(int max_npad) {
  // coarse values + v (npad) + tmp (64) + ring + one form's segment starts (npad + 1)
  return TQ_BYTES + (size_t)(max_npad + TS + stream::RSZ) * sizeof(float) +
         (size_t)(max_npad + 1) * sizeof(int);
}

// One sweep.  FWD: blocks I = 0 .. nt-1, row form, y_I = inv(L_II)(b_I - env);
// otherwise blocks nt-1 .. 0, column form, x_I = inv(L_II)^T (y_I - env).
// es: the form's segment starts of this region in LDS; boff: block starts.
template <bool FWD>
__device__ __forceinline__ void stream_sweep(int nt, const int *es, const int *__restrict__ boff,
                                             const float *__restrict__ S, int L,
                                             const float *__restrict__ tail, float *v, float *tmp,
                                             float *ring) {
  using namespace stream;
  const int t = threadIdx.x, rr = t >> 2, q = t & 3;
  const int nunits = (L + UE - 1) / UE;
  // Every step loads and stores unconditionally (units past the stream read
  // the shared tail), so that the compiler can count the loads in flight and
  // wait for the oldest one only.
  const long long tail_off = tail - S;  // one offset select, one load per unit
  auto unit_src = [&](int u) {
    const long long off = u < nunits ? (long long)u * UE : tail_off;
    return reinterpret_cast<const f4 *>(S + off) + t;
  };
  f4 f[NS];
  // issue in slot order (the copy below waits for slot sl with the NS - 1
  // younger loads still in flight; the scheduler must not reorder these)
  static_for<0, NS>([&](auto slc) __attribute__((always_inline)) {
    f[decltype(slc)::value] = *unit_src(decltype(slc)::value);
    __builtin_amdgcn_sched_barrier(0);
  });
  // current block: index b in sweep order, its tile row I, stream start bs,
  // envelope size T and this thread's segment [bs + e0, bs + e0 + len)
  int b = 0, I = FWD ? 0 : nt - 1;
  int bs = nt > 0 ? boff[I] : 0, T = es[I * TS + TS] - es[I * TS];
  int e0 = es[I * TS + rr] - es[I * TS], len = es[I * TS + rr + 1] - es[I * TS + rr];
  int cons = bs;  // stream position up to which this block's envelope has been used
  float acc = 0.f;
  bool fin = nt == 0;
  for (int k0 = 0; k0 < nunits; k0 += NS) {
    // slots are unrolled at compile time (f[] must not be indexed at run time)
    static_for<0, NS>([&](auto slc) __attribute__((always_inline)) {
      constexpr int sl = decltype(slc)::value;
      const int u = k0 + sl;
      reinterpret_cast<f4 *>(ring + (u % RU) * UE)[t] = f[sl];
      f[sl] = *unit_src(u + NS);
    });
    __syncthreads();  // batch in the ring
    const int avail = min(L, (k0 + NS) * UE);
    while (!fin) {
      const int dI = bs + ((T + 3) & ~3), eI = dI + DE;
      const int hi = min(avail, dI);
      if (hi > cons) {  // envelope entries that arrived: [cons, hi)
        const int s0 = bs + e0;
        const int kl = max(cons - s0, 0), kh = min(hi - s0, len);
        const int v0 = FWD ? I * TS - len : I * TS + TS;
        int k = kl + ((q - kl) & 3);
        int ri = (s0 + k) % RSZ;  // ring index of entry k, advanced with a wrap
        for (; k < kh; k += 4) {
          acc = fmaf(-ring[ri], v[v0 + k], acc);
          ri += 4;
          ri = ri >= RSZ ? ri - RSZ : ri;
        }
        cons = hi;
      }
      if (avail < eI) break;
      // diagonal step of block I; the next block's segment bounds are read
      // now, off the path that follows the barriers
      const int In = FWD ? b + 1 : nt - 2 - b;
      int Tn = 0, e0n = 0, lenn = 0;
      if (b + 1 < nt) {
        const int sI = es[In * TS];
        Tn = es[In * TS + TS] - sI;
        e0n = es[In * TS + rr] - sI;
        lenn = es[In * TS + rr + 1] - es[In * TS + rr];
      }
      acc += dpp_quad_f<0xB1>(acc);  // the row's four partial sums (lanes 4rr .. 4rr+3)
      acc += dpp_quad_f<0x4E>(acc);
      if (q == 0) tmp[rr] = v[I * TS + rr] + acc;
      __syncthreads();  // tmp complete
      const int dr = dI % RSZ;  // ring index of the diagonal tile
      // Every LDS read of the diagonal step is issued before the first
      // product, so that the step waits for LDS once.  Entries outside the
      // triangle are read too (they lie inside the packed tile, which is
      // whole in the ring) and dropped by a select.
      if (FWD) {
        // y[rr] = sum_c inv(L_II)[rr][c] tmp[c]: row rr, columns 16q .. 16q+15
        int ri = dr + dpos_row(rr) + 16 * q;
        ri = ri >= RSZ ? ri - RSZ : ri;
        f4 a[4], tt[4];
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          const int rc = ri + 4 * c4 >= RSZ ? ri + 4 * c4 - RSZ : ri + 4 * c4;
          a[c4] = *reinterpret_cast<const f4 *>(ring + rc);
          tt[c4] = *reinterpret_cast<const f4 *>(tmp + 16 * q + 4 * c4);
        }
        float y = 0.f;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          float s4 = a[c4][0] * tt[c4][0];
          s4 = fmaf(a[c4][1], tt[c4][1], s4);
          s4 = fmaf(a[c4][2], tt[c4][2], s4);
          s4 = fmaf(a[c4][3], tt[c4][3], s4);
          y += (16 * q + 4 * c4 <= rr) ? s4 : 0.f;
        }
        y += dpp_quad_f<0xB1>(y);
        y += dpp_quad_f<0x4E>(y);
        if (q == 0) v[I * TS + rr] = y;
      } else {
        // x[col] = sum_r inv(L_II)[r][col] tmp[r]: lanes 4c .. 4c+3 of
        // wavefront w hold column col = 16w + c; lane qq takes rows 4s + qq
        const int l = t & 63, w = t >> 6;
        const int col = 16 * w + (l >> 2), qq = l & 3;
        const int base = dr + col + 4 * qq;  // entry (4s + qq, col) at base +
        float rv[16], tv[16];                // dpos_row(4s + qq) - 4 qq
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4) {
          int ri = base + 4 * qq * s4 + 8 * s4 * (s4 + 1);
          ri = ri >= RSZ ? ri - RSZ : ri;
          rv[s4] = ring[ri];
          tv[s4] = tmp[4 * s4 + qq];
        }
        float x0 = 0.f, x1 = 0.f;  // two chains: rows 4s + qq for even and odd s
#pragma unroll
        for (int s4 = 0; s4 < 16; s4 += 2) {
          const float p0 = rv[s4] * tv[s4], p1 = rv[s4 + 1] * tv[s4 + 1];
          x0 += (col <= 4 * s4 + qq) ? p0 : 0.f;
          x1 += (col <= 4 * s4 + 4 + qq) ? p1 : 0.f;
        }
        float x = x0 + x1;
        x += dpp_quad_f<0xB1>(x);
        x += dpp_quad_f<0x4E>(x);
        if (qq == 0) v[I * TS + col] = x;
      }
      __syncthreads();  // block I final in v; tmp free
      acc = 0.f;
      if (++b == nt) {
        fin = true;
        break;
      }
      I = In;
      bs = eI;
      T = Tn;
      e0 = e0n;
      len = lenn;
      cons = bs;
    }
  }
}

template <typename TB>
__global__ void __launch_bounds__(WG) k_local_apply_stream(Plan p, const double *__restrict__ r,
                                                           const float *__restrict__ fst,
                                                           const float *__restrict__ bst,
                                                           const TB *__restrict__ phi,
                                                           const double *__restrict__ t,
                                                           const double *__restrict__ tpart,
                                                           int T0, double *__restrict__ xloc,
                                                           const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) char smem_raw[];  // 16-byte ring accesses
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int g0 = p.trow_ptr[i], nt = p.trow_ptr[i + 1] - g0;
  const int npad = nt * TS;
  double *tq_s = reinterpret_cast<double *>(smem_raw);  // the region's coarse values
  float *v = reinterpret_cast<float *>(smem_raw + TQ_BYTES);  // whole local vector (padded)
  float *tmp = v + npad;                             // 64
  float *ring = tmp + TS;                            // stream::RSZ
  int *es = reinterpret_cast<int *>(ring + stream::RSZ);  // npad + 1 segment starts
  const double cps = tpart ? coarse_partial_load(p, i, tpart, T0) : 0.0;
  // gather, GU rows per thread per pass with all index loads, then all value
  // loads, issued before use.  Nothing here is conditional: the loads are
  // clamped to the region's last row, padding rows are zeroed by a select,
  // and rows past the padding are stored into tmp (scratch until the sweeps)
  // (a load or store under a per-row condition would be waited for inside
  // its branch, one row after the other)
  constexpr int GU = 4;
  for (int l0 = threadIdx.x; l0 < npad; l0 += GU * WG) {
    int dof[GU];
    double rv[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) dof[u] = p.sd_dofs[r0 + min(l0 + u * WG, ni - 1)];
#pragma unroll
    for (int u = 0; u < GU; ++u) rv[u] = r[dof[u]];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int l = l0 + u * WG;
      v[l < npad ? l : npad + (threadIdx.x & (TS - 1))] = l < ni ? (float)rv[u] : 0.f;
    }
  }
  const int *ep = p.eptr + p.vp_ptr[i] + i, *up = p.uptr + p.vp_ptr[i] + i;
  // the backward sweep's segment starts are loaded now and kept in registers
  // (regions up to UPR * WG - 1 padded rows), so that no global load sits
  // between the two sweeps
  constexpr int UPR = 8;
  const bool up_regs = npad < UPR * WG;
  int upv[UPR];
#pragma unroll
  for (int u = 0; u < UPR; ++u) {
    const int l = threadIdx.x + u * WG;
    upv[u] = (up_regs && l <= npad) ? up[l] : 0;
  }
  copy_ints_to_lds<UPR>(es, ep, npad + 1, reinterpret_cast<int *>(tmp));  // tmp: scratch here
  if (tpart) coarse_partial_finish(p, i, cps, tq_s);
  const double *tq = tpart ? tq_s : (t ? t + p.coff[i] : nullptr);
  __syncthreads();
  const int Lf = (int)(p.sfr[i + 1] - p.sfr[i]), Lb = (int)(p.sbr[i + 1] - p.sbr[i]);
  stream_sweep<true>(nt, es, p.sfb + g0, fst + p.sfr[i], Lf, fst + p.sfr[p.N], v, tmp, ring);
  if (up_regs) {
#pragma unroll
    for (int u = 0; u < UPR; ++u) {
      const int l = threadIdx.x + u * WG;
      if (l <= npad) es[l] = upv[u];
    }
  } else {
    for (int l = threadIdx.x; l <= npad; l += WG) es[l] = up[l];
  }
  __syncthreads();
  stream_sweep<false>(nt, es, p.sbb + g0, bst + p.sbr[i], Lb, bst + p.sbr[p.N], v, tmp, ring);
  // local correction (+ prolongation) in the region's ascending-global-index layout
  store_local(p, i, r0, ni, v, phi, tq, xloc);
}

// ------------------------------------------------------------- launchers ---
template <typename TB>
void launch_restrict(hipStream_t s, const Plan &p, const double *r, const TB *phi, double *cvec,
                     const int *done) {
  hipLaunchKernelGGL((k_restrict<TB>), dim3(p.N), dim3(WG), 0, s, p, r, phi, cvec, done);
}
template void launch_restrict<double>(hipStream_t, const Plan &, const double *, const double *,
                                      double *, const int *);
template void launch_restrict<float>(hipStream_t, const Plan &, const double *, const float *,
                                     double *, const int *);
template void launch_restrict<__hip_bfloat16>(hipStream_t, const Plan &, const double *,
                                              const __hip_bfloat16 *, double *, const int *);

template <typename T, typename C, typename TB>
void launch_local_apply_t(hipStream_t s, const Plan &p, int max_npad, const double *r,
                          const T *diag, const T *erow, const T *ecol, const TB *phi,
                          const double *t, const double *tpart, int T0, double *xloc,
                          const int *done, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const size_t sm = local_apply_lds_bytes(max_npad, sizeof(C));
  allow_lds(k_local_apply<T, C, TB>, sm);
  if (ev_start || ev_stop)  // events bound to this dispatch: exact kernel duration
    hipExtLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, ev_start, ev_stop,
                          0, p, r, diag, erow, ecol, phi, t, tpart, T0, xloc, done);
  else
    hipLaunchKernelGGL((k_local_apply<T, C, TB>), dim3(p.N), dim3(WG), sm, s, p, r, diag, erow,
                       ecol, phi, t, tpart, T0, xloc, done);
}

#define AMSP_LOCAL_APPLY_INST(T, C, TB)                                                        \
  template void launch_local_apply_t<T, C, TB>(hipStream_t, const Plan &, int, const double *, \
                                               const T *, const T *, const T *, const TB *,    \
                                               const double *, const double *, int, double *,  \
                                               const int *, hipEvent_t, hipEvent_t);
AMSP_LOCAL_APPLY_INST(double, double, double)
#undef AMSP_LOCAL_APPLY_INST

template <typename TB>
void launch_local_apply_stream(hipStream_t s, const Plan &p, int max_npad, const double *r,
                               const float *fst, const float *bst, const TB *phi, const double *t,
                               const double *tpart, int T0, double *xloc, const int *done,
                               hipEvent_t ev_start, hipEvent_t ev_stop) {
  const size_t sm = local_apply_stream_lds_bytes(max_npad);
  allow_lds(k_local_apply_stream<TB>, sm);
  if (ev_start || ev_stop)  // events bound to this dispatch: exact kernel duration
    hipExtLaunchKernelGGL((k_local_apply_stream<TB>), dim3(p.N), dim3(WG), sm, s, ev_start,
                          ev_stop, 0, p, r, fst, bst, phi, t, tpart, T0, xloc, done);
  else
    hipLaunchKernelGGL((k_local_apply_stream<TB>), dim3(p.N), dim3(WG), sm, s, p, r, fst, bst, phi,
                       t, tpart, T0, xloc, done);
}
template void launch_local_apply_stream<float>(hipStream_t, const Plan &, int, const double *,
                                               const float *, const float *, const float *,
                                               const double *, const double *, int, double *,
                                               const int *, hipEvent_t, hipEvent_t);
template void launch_local_apply_stream<__hip_bfloat16>(hipStream_t, const Plan &, int,
                                                        const double *, const float *,
                                                        const float *, const __hip_bfloat16 *,
                                                        const double *, const double *, int,
                                                        double *, const int *, hipEvent_t,
                                                        hipEvent_t);

}  // namespace amsp
