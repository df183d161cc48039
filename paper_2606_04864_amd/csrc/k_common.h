// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include "amsp_internal.h"

namespace amsp {

constexpr int LDT = TS + 1;  // padded LDS row stride (doubles) for 64x64 tiles

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over the workgroup; result valid in every thread.
// sh must hold WG/64 doubles; the call contains two barriers.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < WG / 64; ++i) t += sh[i];
  return t;
}

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(__hip_bfloat16 x) { return (double)__bfloat162float(x); }
__device__ __forceinline__ float to_f(double x) { return (float)x; }
__device__ __forceinline__ float to_f(__hip_bfloat16 x) { return __bfloat162float(x); }

// Binary search: index i with ptr[i] <= x < ptr[i+1] (ptr nondecreasing, n+1 entries).
__device__ __forceinline__ int find_segment(const int *ptr, int n, int x) {
  int lo = 0, hi = n;  // invariant ptr[lo] <= x < ptr[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (ptr[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ size_t tile_elem(long long tile) { return (size_t)tile * (size_t)TE; }

// Packed diagonal tiles.  The factor pool holds the off-diagonal 64x64 tiles
// (row-major, TE entries each) followed by one lower-triangular diagonal tile
// per tile row.  Row R of a packed tile keeps columns 0..R, zero-padded to a
// multiple of 4 entries, and starts at dpos_row(R), a multiple of 4: rows are
// 16-byte aligned in fp32 and fp64, so they load in 4-entry vectors.
__host__ __device__ constexpr int dpos_row(int R) {
  return 4 * ((R >> 2) + 1) * (2 * (R >> 2) + (R & 3));
}
static_assert(dpos_row(TS) == DE, "packed diagonal tile size");
static_assert((DE * 4) % 16 == 0 && (TE * 4) % 16 == 0, "16-byte aligned tiles");

// first entry of the packed diagonal tile of global tile row g
__device__ __forceinline__ size_t diag_elem(const Plan &p, int g) {
  return (size_t)p.noff * TE + (size_t)g * DE;
}

// Entries c0 .. c0+15 (c0 a multiple of 16) of row R of a packed diagonal
// tile; entries above the diagonal are zero.  Each 4-entry group that starts
// right of the diagonal is not read.
template <typename T>
__device__ __forceinline__ void packed_row16(T (&a)[16], const T *__restrict__ dtile, int R,
                                             int c0) {
  const T *row = dtile + dpos_row(R) + c0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (c0 + 4 * u <= R) {
      if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(row + 4 * u);
        a[4 * u] = v.x;
        a[4 * u + 1] = v.y;
        a[4 * u + 2] = v.z;
        a[4 * u + 3] = v.w;
      } else {
        const double2 v0 = *reinterpret_cast<const double2 *>(row + 4 * u);
        const double2 v1 = *reinterpret_cast<const double2 *>(row + 4 * u + 2);
        a[4 * u] = v0.x;
        a[4 * u + 1] = v0.y;
        a[4 * u + 2] = v1.x;
        a[4 * u + 3] = v1.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) a[4 * u + j] = T(0);
    }
  }
}

// Entry (R, C) of a packed diagonal tile (zero above the diagonal).
template <typename T>
__device__ __forceinline__ T packed_at(const T *__restrict__ dtile, int R, int C) {
  return C <= R ? dtile[dpos_row(R) + C] : T(0);
}

// gfx950 gives a workgroup up to 160 KB of LDS; raise the dynamic-LDS limit
// of a kernel once before its first launch with more than 64 KB.
template <typename F>
inline void allow_lds(F *kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------- MFMA ----
// v_mfma_f64_16x16x4f64: D(16x16) = A(16x4) B(4x16) + C, wave64.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; D is returned in four
// registers, D[l/16 + 4r][l%16] in register r (checked on the device by
// amsp_selftest_mfma).
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Copy a 64x64 row-major tile from global memory into padded LDS (coalesced).
template <typename T>
__device__ __forceinline__ void tile_to_lds(const T *__restrict__ g, double *lds) {
  for (int e = threadIdx.x; e < TE; e += WG) lds[(e >> 6) * LDT + (e & 63)] = to_d(g[e]);
}

__device__ __forceinline__ void lds_to_tile(const double *lds, double *__restrict__ g) {
  for (int e = threadIdx.x; e < TE; e += WG) g[e] = lds[(e >> 6) * LDT + (e & 63)];
}

// Packed diagonal tile <-> full tile in padded LDS (upper triangle zero).
__device__ __forceinline__ void packed_to_lds(const double *__restrict__ g, double *lds) {
  for (int e = threadIdx.x; e < TE; e += WG) lds[(e >> 6) * LDT + (e & 63)] = packed_at(g, e >> 6, e & 63);
}

__device__ __forceinline__ void lds_to_packed(const double *lds, double *__restrict__ g) {
  for (int e = threadIdx.x; e < TE; e += WG) {
    const int r = e >> 6, c = e & 63;
    if (c < 4 * ((r >> 2) + 1)) g[dpos_row(r) + c] = c <= r ? lds[r * LDT + c] : 0.0;
  }
}

// Synchronisation of the lanes of one wavefront around LDS traffic: LDS
// operations of a wavefront complete in order; the fences keep the compiler
// from moving loads or stores across the point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast lane `src` (a compile-time constant in the callers' unrolled
// loops) of a double to the whole wavefront.
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(d) for d > 0 to double precision: hardware estimate refined by two
// Newton steps y <- y (3 - d y^2) / 2 (each squares the relative error).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double hd = -0.5 * d;
  y = y * fma(hd, y * y, 1.5);
  y = y * fma(hd, y * y, 1.5);
  return y;
}

__device__ __forceinline__ int opaque_int(int v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

// Compile-time loop: f(std::integral_constant<int, v>) for v = B, B+S, ... < E.
template <int B, int E, int S = 1, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + S, E, S>(f);
  }
}

// Basis rows with m <= MAXNEV kept coefficients are read as KM = 4, 8 or 16
// values (the smallest that holds nev): with_km(nev, f) calls f with
// std::integral_constant<int, KM>.
template <typename F>
__device__ __forceinline__ void with_km(int nev, F &&f) {
  static_assert(MAXNEV <= 16, "basis rows are read as at most 16 coefficients");
  if (nev <= 4)
    f(std::integral_constant<int, 4>{});
  else if (nev <= 8)
    f(std::integral_constant<int, 8>{});
  else
    f(std::integral_constant<int, 16>{});
}

// Coefficients 0 .. KM-1 of a basis row with m >= 1 kept coefficients, entry
// k at ph[k * stride]; those for k >= m read as zero (basis_coef).  The loads
// are clamped into the m kept entries and issued unconditionally, so that all
// of them are in flight together: a load under "k < m" (a branch on a value
// the compiler cannot see) would be waited for before the next is issued.
template <int KM, typename TB>
__device__ __forceinline__ void basis_row_load(const TB *__restrict__ ph, size_t stride, int m,
                                               TB (&raw)[KM]) {
#pragma unroll
  for (int k = 0; k < KM; ++k) raw[k] = ph[(size_t)min(k, m - 1) * stride];
}
template <int KM, typename TB>
__device__ __forceinline__ double basis_coef(const TB (&raw)[KM], int k, int m) {
  return k < m ? to_d(raw[k]) : 0.0;
}

// Quad permutation of a double across lanes (DPP, no LDS traffic); CTRL is a
// quad_perm control word: 0xB1 swaps neighbours (lane ^ 1), 0x4E swaps pairs
// (lane ^ 2).
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same for a float.
template <int CTRL>
__device__ __forceinline__ float dpp_quad_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Cholesky factor of a 64x64 SPD tile and the inverse of the factor, in LDS.
//   a (stride LDT): lower triangle of the tile on entry, L on exit (upper 0)
//   w (stride LDT): inv(L) on exit (upper 0)
// Factorisation: wavefront 0, lane i holds row i in registers (right-looking).
// At step k the entry L[k+1][k] that the next pivot waits for is taken from
// lane k+1 directly; the other entries of column k are broadcast through LDS
// (double-buffered, read in batches of CH).  A single wavefront's LDS
// accesses complete in program order, so the steps need no barriers.
// Inverse: all four wavefronts; each column of inv(L) is solved by four
// adjacent lanes that split every row's dot product and combine it with quad
// permutations; the next row of L is fetched while the current one is used.
// A non-positive or non-finite pivot sets *fail and is replaced by 1 so that
// the result stays finite.  Needs blockDim.x == 256.
template <int CH>
__device__ __forceinline__ void lds_potrf_trtri(double *a, double *w, int *fail) {
  // The lane index and the LDS base pass once through an opaque move, so
  // that callers' loops cannot hoist the lane-dependent masks or the
  // constant LDS addresses below out of the loop and keep them live.
  const int lane_id = opaque_int((int)threadIdx.x);
  const int z = opaque_int(0);
  double *aa = a + z, *ww = w + z;
  double *ls = ww;        // rows of L with stride 64 for the inverse phase
  double *rdg = ww + TE;  // 1 / L_kk  (TE + 64 <= TS * LDT)
  if (threadIdx.x < 64) {
    const int i = lane_id;
    double *col = aa;  // two column buffers (a is free once its rows are in registers)
    double r[TS];      // row i; entries right of the diagonal are never used
    static_for<0, TS>([&](auto jc) __attribute__((always_inline)) {
      r[jc.value] = aa[i * LDT + jc.value];
    });
    wave_sync();
    bool bad = false;
    // column k of L for this lane's row, given the updated r[k]
    auto pivot = [&](auto kc) __attribute__((always_inline)) {
      constexpr int k = decltype(kc)::value;
      double d = readlane_d(r[k], k);
      const bool bk = !(d > 0.0) || !isfinite(d);
      bad = bad || bk;
      d = bk ? 1.0 : d;
      const double inv = rsqrt_nr(d);
      r[k] = (i == k) ? d * inv : r[k] * inv;
      rdg[k] = inv;
      col[(k & 1) * TS + i] = r[k];
    };
    pivot(std::integral_constant<int, 0>{});
    // Step k: the reads of column k go out first; the next pivot (which
    // needs only column k+1, updated through a lane read) and its column
    // write overlap their latency; then the bulk update of columns >= k+2.
    static_for<0, TS - 1>([&](auto kc) __attribute__((always_inline)) {
      constexpr int k = decltype(kc)::value;
      constexpr int nb = (TS - (k + 2) + CH - 1) / CH;  // batches of columns >= k+2
      const double *cb = col + (k & 1) * TS;
      const double lk = r[k];
      double cva[CH], cvb[CH];
      auto load_batch = [&](auto bc, double(&cv)[CH]) __attribute__((always_inline)) {
        constexpr int j0 = k + 2 + CH * decltype(bc)::value;
        constexpr int j1 = j0 + CH < TS ? j0 + CH : TS;
        static_for<j0, j1>([&](auto jc) __attribute__((always_inline)) {
          cv[jc.value - j0] = cb[jc.value];
        });
      };
      if constexpr (nb > 0) load_batch(std::integral_constant<int, 0>{}, cva);
      r[k + 1] = fma(-lk, readlane_d(lk, k + 1), r[k + 1]);
      pivot(std::integral_constant<int, k + 1>{});
      static_for<0, nb>([&](auto bc) __attribute__((always_inline)) {
        constexpr int bi = decltype(bc)::value;
        double(&cur)[CH] = (bi & 1) ? cvb : cva;
        double(&nxt)[CH] = (bi & 1) ? cva : cvb;
        if constexpr (bi + 1 < nb) load_batch(std::integral_constant<int, bi + 1>{}, nxt);
        constexpr int j0 = k + 2 + CH * bi;
        constexpr int j1 = j0 + CH < TS ? j0 + CH : TS;
        static_for<j0, j1>([&](auto jc) __attribute__((always_inline)) {
          r[jc.value] = fma(-lk, cur[jc.value - j0], r[jc.value]);
        });
      });
    });
    if (bad && i == 0) *fail = 1;
    wave_sync();
    static_for<0, TS>([&](auto jc) __attribute__((always_inline)) {
      aa[i * LDT + jc.value] = r[jc.value];
      ls[i * TS + jc.value] = r[jc.value];
    });
  }
  __syncthreads();
  {
    // column j of inv(L): x_m = (delta_mj - sum_{q<m} L_mq x_q) / L_mm.
    // Lane (j, p): p = lane & 3 owns x_q for q = 4t + p (xs[t]).
    const int p = lane_id & 3;
    const int j = lane_id >> 2;  // 0..63
    double xs[TS / 4];  // zero-initialised: masked products must see finite values
    static_for<0, TS / 4>([&](auto tc) __attribute__((always_inline)) { xs[tc.value] = 0.0; });
    double lva[TS / 4], lvb[TS / 4];  // rows m (even / odd) of L, entries q = 4t + p
    auto load_row = [&](auto mc, double(&lv)[TS / 4]) __attribute__((always_inline)) {
      constexpr int m = decltype(mc)::value;
      static_for<0, (m + 3) / 4>([&](auto tc) __attribute__((always_inline)) {
        constexpr int t = decltype(tc)::value;
        const int q = 4 * t + p;
        lv[t] = (q < m) ? ls[m * TS + q] : 0.0;
      });
    };
    load_row(std::integral_constant<int, 1>{}, lvb);
    static_for<0, TS>([&](auto mc) __attribute__((always_inline)) {
      constexpr int m = decltype(mc)::value;
      constexpr int nt = (m + 3) / 4;
      double(&cur)[TS / 4] = (m & 1) ? lvb : lva;
      double(&nxt)[TS / 4] = (m & 1) ? lva : lvb;
      if constexpr (m + 1 < TS) load_row(std::integral_constant<int, m + 1>{}, nxt);
      double s0 = 0.0, s1 = 0.0;
      static_for<0, nt>([&](auto tc) __attribute__((always_inline)) {
        constexpr int t = decltype(tc)::value;
        if constexpr ((t & 1) == 0)
          s0 = fma(-cur[t], xs[t], s0);
        else
          s1 = fma(-cur[t], xs[t], s1);
      });
      double sum = s0 + s1;
      sum += dpp_quad<0xB1>(sum);
      sum += dpp_quad<0x4E>(sum);
      const double xm = ((j == m) ? 1.0 + sum : sum) * rdg[m];
      constexpr int tm = m / 4;
      xs[tm] = (p == (m & 3)) ? xm : xs[tm];
    });
    __syncthreads();  // all reads of ls / rdg done before w is overwritten
    static_for<0, TS / 4>([&](auto tc) __attribute__((always_inline)) {
      constexpr int t = decltype(tc)::value;
      ww[(4 * t + p) * LDT + j] = xs[t];  // exact zeros above the diagonal
    });
  }
  for (int e = threadIdx.x; e < TE; e += blockDim.x) {
    const int r = e >> 6, c = e & 63;
    if (c > r) a[r * LDT + c] = 0.0;
  }
  __syncthreads();
}

// ------------------------------------------------ MFMA tile products ------
// One 64x64 output tile per workgroup: wavefront w owns rows 16w..16w+15 as
// four 16x16 MFMA blocks (acc[cb] = columns 16cb..).  K-slot q of MFMA step s
// stands for k = 16q + s, so each lane reads 16 contiguous entries of a row.
// Tiles are row-major 64x64 in global memory.
struct Acc4 {
  d4 v[4];
};

__device__ __forceinline__ void acc_load(Acc4 &c, const double *__restrict__ g) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) c.v[cb][r] = g[(16 * wv + (l >> 4) + 4 * r) * TS + 16 * cb + (l & 15)];
}

// acc_load of a packed diagonal tile (zero above the diagonal)
__device__ __forceinline__ void acc_load_packed(Acc4 &c, const double *__restrict__ g) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      c.v[cb][r] = packed_at(g, 16 * wv + (l >> 4) + 4 * r, 16 * cb + (l & 15));
}

__device__ __forceinline__ void acc_zero(Acc4 &c) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) c.v[cb] = d4{0.0, 0.0, 0.0, 0.0};
}

__device__ __forceinline__ void acc_store(const Acc4 &c, double *__restrict__ g) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) g[(16 * wv + (l >> 4) + 4 * r) * TS + 16 * cb + (l & 15)] = c.v[cb][r];
}

__device__ __forceinline__ void acc_to_lds(const Acc4 &c, double *lds) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) lds[(16 * wv + (l >> 4) + 4 * r) * LDT + 16 * cb + (l & 15)] = c.v[cb][r];
}

// c += sign * X Y^T, X and Y with row stride ldx/ldy (global or LDS)
__device__ __forceinline__ void acc_mma_abt(Acc4 &c, const double *X, int ldx, const double *Y,
                                            int ldy, double sign) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = l & 15, q = l >> 4;
  double xa[16];
  const double *xr = X + (16 * wv + i) * ldx + 16 * q;
#pragma unroll
  for (int s = 0; s < 16; ++s) xa[s] = sign * xr[s];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const double *yr = Y + (16 * cb + i) * ldy + 16 * q;
    double yb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) yb[s] = yr[s];
#pragma unroll
    for (int s = 0; s < 16; ++s) c.v[cb] = mfma16x16x4(xa[s], yb[s], c.v[cb]);
  }
}

// c += sign * X Y
__device__ __forceinline__ void acc_mma_ab(Acc4 &c, const double *X, int ldx, const double *Y,
                                           int ldy, double sign) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = l & 15, q = l >> 4;
  double xa[16];
  const double *xr = X + (16 * wv + i) * ldx + 16 * q;
#pragma unroll
  for (int s = 0; s < 16; ++s) xa[s] = sign * xr[s];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int s = 0; s < 16; ++s) c.v[cb] = mfma16x16x4(xa[s], Y[(16 * q + s) * ldy + 16 * cb + i], c.v[cb]);
  }
}

}  // namespace amsp
