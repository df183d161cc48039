// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once
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

// Register block of a tile owned by one thread: rows (t>>4)+16*i, cols (t&15)+16*j.
struct Blk {
  double v[4][4];
};

__device__ __forceinline__ void blk_load(Blk &b, const double *__restrict__ g) {
  const int r0 = threadIdx.x >> 4, c0 = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) b.v[i][j] = g[(r0 + 16 * i) * TS + c0 + 16 * j];
}

__device__ __forceinline__ void blk_store(const Blk &b, double *__restrict__ g) {
  const int r0 = threadIdx.x >> 4, c0 = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) g[(r0 + 16 * i) * TS + c0 + 16 * j] = b.v[i][j];
}

__device__ __forceinline__ void blk_to_lds(const Blk &b, double *lds) {
  const int r0 = threadIdx.x >> 4, c0 = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) lds[(r0 + 16 * i) * LDT + c0 + 16 * j] = b.v[i][j];
}

// b -= X * Y^T  (X, Y 64x64 in padded LDS)
__device__ __forceinline__ void blk_sub_abt(Blk &b, const double *X, const double *Y) {
  const int r0 = threadIdx.x >> 4, c0 = threadIdx.x & 15;
  for (int k = 0; k < TS; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = X[(r0 + 16 * i) * LDT + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = Y[(c0 + 16 * j) * LDT + k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) b.v[i][j] = fma(-x[i], y[j], b.v[i][j]);
  }
}

// b -= X * Y  (X, Y 64x64 in padded LDS)
__device__ __forceinline__ void blk_sub_ab(Blk &b, const double *X, const double *Y) {
  const int r0 = threadIdx.x >> 4, c0 = threadIdx.x & 15;
  for (int k = 0; k < TS; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = X[(r0 + 16 * i) * LDT + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = Y[k * LDT + c0 + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) b.v[i][j] = fma(-x[i], y[j], b.v[i][j]);
  }
}

// out = X * Y^T (fresh block)
__device__ __forceinline__ void blk_abt(Blk &b, const double *X, const double *Y) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) b.v[i][j] = 0.0;
  blk_sub_abt(b, X, Y);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) b.v[i][j] = -b.v[i][j];
}

// out = X * Y (fresh block)
__device__ __forceinline__ void blk_ab(Blk &b, const double *X, const double *Y) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) b.v[i][j] = 0.0;
  blk_sub_ab(b, X, Y);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) b.v[i][j] = -b.v[i][j];
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

// Cholesky factor of a 64x64 SPD tile and the inverse of the factor, in LDS.
//   a (stride LDT): lower triangle of the tile on entry, L on exit (upper 0)
//   w (stride LDT): inv(L) on exit (upper 0)
// Wavefront 0 does the work in registers: for the factorisation lane i holds
// row i (right-looking; column k of L is broadcast through LDS at step k),
// for the inverse lane j holds column j of inv(L) (forward substitution
// against broadcast rows of L).  Other wavefronts only meet the closing
// barrier.  A non-positive or non-finite pivot sets *fail and is replaced by
// 1 so that the result stays finite.
__device__ __forceinline__ int opaque_int(int v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

__device__ void lds_potrf_trtri(double *a, double *w, int *fail) {
  if (threadIdx.x < 64) {
    // Lane-dependent compares go through opaque_int at their point of use so
    // that callers' loops cannot hoist 64 masks (or the constant LDS
    // addresses, via z) out of the loop and keep them live.
    const int z = opaque_int(0);
    double *aa = a + z, *ww = w + z;
    const int i = threadIdx.x;
    double *col = aa;      // column k of L (a is free once its rows are in registers)
    double *ls = ww;       // rows of L with stride 64 for the inverse phase
    double *rdg = ww + TE; // 1 / L_kk  (TE + 64 <= TS * LDT)
    double r[TS];          // row i; entries right of the diagonal are never used
#pragma unroll
    for (int j = 0; j < TS; ++j) r[j] = aa[i * LDT + j];
    wave_sync();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < TS; ++k) {
      double d = readlane_d(r[k], k);
      if (!(d > 0.0) || !isfinite(d)) {
        bad = true;
        d = 1.0;
      }
      const double sq = sqrt(d);
      const double inv = 1.0 / sq;
      r[k] = (opaque_int(i) == k) ? sq : r[k] * inv;
      rdg[k] = inv;
      col[i] = r[k];
      wave_sync();
#pragma unroll
      for (int j = k + 1; j < TS; ++j) r[j] = fma(-r[k], col[j], r[j]);
      wave_sync();
    }
    if (bad && i == 0) *fail = 1;
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      aa[i * LDT + j] = r[j];
      ls[i * TS + j] = r[j];
    }
    wave_sync();
    // column j = i of inv(L): x_m = (delta_mj - sum_{q<m} L_mq x_q) / L_mm
    double x[TS];
#pragma unroll
    for (int m = 0; m < TS; ++m) {
      double s0 = (opaque_int(i) == m) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
      for (int q = 0; q + 1 < m; q += 2) {
        s0 = fma(-ls[m * TS + q], x[q], s0);
        s1 = fma(-ls[m * TS + q + 1], x[q + 1], s1);
      }
      if (m & 1) s0 = fma(-ls[m * TS + m - 1], x[m - 1], s0);
      x[m] = (s0 + s1) * rdg[m];
    }
    wave_sync();
#pragma unroll
    for (int m = 0; m < TS; ++m) ww[m * LDT + i] = x[m];  // exact zeros above the diagonal
  }
  __syncthreads();
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
