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

// In-LDS Cholesky of the lower triangle of a 64x64 SPD tile (padded stride).
// Non-positive pivots set *fail and are replaced by 1 so that the
// factorisation always finishes with finite values.
__device__ __forceinline__ void lds_potrf(double *a, int *fail) {
  const int t = threadIdx.x;
  for (int k = 0; k < TS; ++k) {
    if (t == 0) {
      double d = a[k * LDT + k];
      if (!(d > 0.0) || !isfinite(d)) {
        *fail = 1;
        d = 1.0;
      }
      a[k * LDT + k] = sqrt(d);
    }
    __syncthreads();
    if (t > k && t < TS) a[t * LDT + k] /= a[k * LDT + k];
    __syncthreads();
    for (int e = t; e < TE; e += WG) {
      const int i = e >> 6, j = e & 63;
      if (j > k && j <= i) a[i * LDT + j] = fma(-a[i * LDT + k], a[j * LDT + k], a[i * LDT + j]);
    }
    __syncthreads();
  }
  // clear the strict upper triangle
  for (int e = t; e < TE; e += WG) {
    const int i = e >> 6, j = e & 63;
    if (j > i) a[i * LDT + j] = 0.0;
  }
  __syncthreads();
}

// x = inv(L) for lower-triangular L in LDS (both padded).  part: 4*64 doubles.
__device__ __forceinline__ void lds_trtri(const double *L, double *x, double *part) {
  const int t = threadIdx.x;
  const int j = t & 63, seg = t >> 6;
  for (int e = t; e < TE; e += WG) x[(e >> 6) * LDT + (e & 63)] = 0.0;
  __syncthreads();
  for (int i = 0; i < TS; ++i) {
    // x[i][j] = -(sum_{k=j}^{i-1} L[i][k] x[k][j]) / L[i][i]  for j < i
    double s = 0.0;
    if (j < i) {
      const int len = i - j;
      const int k0 = j + (len * seg) / 4, k1 = j + (len * (seg + 1)) / 4;
      for (int k = k0; k < k1; ++k) s = fma(L[i * LDT + k], x[k * LDT + j], s);
    }
    part[seg * TS + j] = s;
    __syncthreads();
    if (seg == 0) {
      const double lii = L[i * LDT + i];
      if (j < i) {
        const double tot = (part[j] + part[TS + j]) + (part[2 * TS + j] + part[3 * TS + j]);
        x[i * LDT + j] = -tot / lii;
      } else if (j == i) {
        x[i * LDT + i] = 1.0 / lii;
      }
    }
    __syncthreads();
  }
}

}  // namespace amsp
