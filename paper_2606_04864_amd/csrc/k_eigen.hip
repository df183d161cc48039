// Batched local eigensolver and coarse-basis construction.
//
// For every region the lowest eigenpairs of the local eigenproblem
// hat A_i psi = lambda S_i psi (Section 3.2) are computed through the
// standard form B_i z = lambda z with B_i = S^{-1/2} hat A_i S^{-1/2} and
// psi = S^{-1/2} z (Section 5, parameter test).  Method: block shift-invert
// subspace iteration (Bathe-Wilson) with EIGP columns: Y = (B_i + sigma I)^{-1} X
// (tile-profile Cholesky solves, k_profile_solve_block), then a Rayleigh-Ritz
// step here: CholQR2 orthonormalisation of Y, H = Y^T B_i Y with the sparse
// B_i, cyclic Jacobi on the EIGP x EIGP matrix H, X = Y V sorted ascending,
// and residuals ||B_i x - theta x|| for the m_i + 1 lowest pairs.  Regions
// with n_i <= EIGP are solved directly by Jacobi on the dense B_i.
#include "k_common.h"

namespace amsp {

constexpr int HP = EIGP + 1;  // padded row stride of the small matrices
static_assert(WG == EIGP * EIGP, "one thread per entry of the EIGP x EIGP Gram matrices");

__device__ __forceinline__ double hash_uniform(unsigned a, unsigned b) {
  // SplitMix-style integer hash of (a, b) mapped to (-1, 1)
  unsigned long long x = ((unsigned long long)a << 32) ^ (unsigned long long)b;
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  x ^= x >> 31;
  return ((double)(x >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

// X: column 0 = S^{1/2} 1 (the exact null vector of B_i), others pseudo-random
// functions of (global dof, column); padding rows zero.
__global__ void __launch_bounds__(WG) k_eig_init(Plan p, const double *__restrict__ sdiag,
                                                 double *__restrict__ X) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int npad = p.vp_ptr[i + 1] - p.vp_ptr[i];
  double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  for (int e = threadIdx.x; e < npad * EIGP; e += WG) {
    const int l = e / EIGP, c = e % EIGP;
    double v = 0.0;
    if (l < ni) v = (c == 0) ? sqrt(sdiag[r0 + l]) : hash_uniform((unsigned)p.sd_dofs[r0 + l], (unsigned)c);
    Xi[e] = v;
  }
}

// Cyclic Jacobi on the symmetric EIGP x EIGP matrix H (LDS, stride HP);
// V accumulates the rotations.  Round-robin ordering: 8 disjoint pairs per
// round, 15 rounds per sweep.
__device__ void jacobi16(double *H, double *V, double *cs, int *flag) {
  const int t = threadIdx.x;
  for (int e = t; e < EIGP * EIGP; e += WG) V[(e / EIGP) * HP + e % EIGP] = (e / EIGP == e % EIGP) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (t == 0) {
      double off = 0.0, tot = 0.0;
      for (int a = 0; a < EIGP; ++a)
        for (int b = 0; b < EIGP; ++b) {
          const double h2 = H[a * HP + b] * H[a * HP + b];
          tot += h2;
          if (a != b) off += h2;
        }
      *flag = (off <= 1e-32 * tot) ? 1 : 0;
    }
    __syncthreads();
    if (*flag) break;
    for (int rnd = 0; rnd < EIGP - 1; ++rnd) {
      if (t < EIGP / 2) {
        int pp, qq;
        if (t == 0) {
          pp = rnd;
          qq = EIGP - 1;
        } else {
          pp = (rnd + t) % (EIGP - 1);
          qq = (rnd - t + (EIGP - 1)) % (EIGP - 1);
        }
        if (pp > qq) {
          int tmp = pp;
          pp = qq;
          qq = tmp;
        }
        const double apq = H[pp * HP + qq];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (H[qq * HP + qq] - H[pp * HP + pp]) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        cs[4 * t + 0] = c;
        cs[4 * t + 1] = s;
        cs[4 * t + 2] = (double)pp;
        cs[4 * t + 3] = (double)qq;
      }
      __syncthreads();
      if (t < (EIGP / 2) * EIGP) {  // rows: H <- J^T H
        const int pr = t / EIGP, k = t % EIGP;
        const double c = cs[4 * pr], s = cs[4 * pr + 1];
        const int pp = (int)cs[4 * pr + 2], qq = (int)cs[4 * pr + 3];
        const double hp = H[pp * HP + k], hq = H[qq * HP + k];
        H[pp * HP + k] = c * hp - s * hq;
        H[qq * HP + k] = s * hp + c * hq;
      }
      __syncthreads();
      if (t < (EIGP / 2) * EIGP) {  // columns: H <- H J
        const int pr = t / EIGP, k = t % EIGP;
        const double c = cs[4 * pr], s = cs[4 * pr + 1];
        const int pp = (int)cs[4 * pr + 2], qq = (int)cs[4 * pr + 3];
        const double hp = H[k * HP + pp], hq = H[k * HP + qq];
        H[k * HP + pp] = c * hp - s * hq;
        H[k * HP + qq] = s * hp + c * hq;
      } else if (t < EIGP * EIGP) {  // V <- V J
        const int u = t - (EIGP / 2) * EIGP;
        const int pr = u / EIGP, k = u % EIGP;
        const double c = cs[4 * pr], s = cs[4 * pr + 1];
        const int pp = (int)cs[4 * pr + 2], qq = (int)cs[4 * pr + 3];
        const double vp = V[k * HP + pp], vq = V[k * HP + qq];
        V[k * HP + pp] = c * vp - s * vq;
        V[k * HP + qq] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

// G = Y^T Y style product of two row-major [n][EIGP] blocks into LDS (stride HP).
__device__ void gram16(const double *__restrict__ A, const double *__restrict__ B, int n, double *G) {
  const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
  double s = 0.0;
  for (int l = 0; l < n; ++l) s = fma(A[(size_t)l * EIGP + a], B[(size_t)l * EIGP + b], s);
  G[a * HP + b] = s;
}

// In-place Y <- Y L^{-T} with G = L L^T (one CholQR pass).
__device__ void cholqr_pass(double *__restrict__ Y, int n, double *G, double *Li) {
  gram16(Y, Y, n, G);
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int a = 0; a < EIGP; ++a) tr += G[a * HP + a];
    const double floor_ = 1e-28 * (tr > 0.0 ? tr : 1.0);
    // Cholesky G = L L^T (lower, in place)
    for (int k = 0; k < EIGP; ++k) {
      double d = G[k * HP + k];
      for (int j = 0; j < k; ++j) d -= G[k * HP + j] * G[k * HP + j];
      if (!(d > floor_)) d = floor_;
      d = sqrt(d);
      G[k * HP + k] = d;
      for (int r = k + 1; r < EIGP; ++r) {
        double v = G[r * HP + k];
        for (int j = 0; j < k; ++j) v -= G[r * HP + j] * G[k * HP + j];
        G[r * HP + k] = v / d;
      }
    }
    // Li = L^{-1}
    for (int a = 0; a < EIGP; ++a)
      for (int b = 0; b < EIGP; ++b) Li[a * HP + b] = 0.0;
    for (int j = 0; j < EIGP; ++j) {
      Li[j * HP + j] = 1.0 / G[j * HP + j];
      for (int r = j + 1; r < EIGP; ++r) {
        double s = 0.0;
        for (int k = j; k < r; ++k) s += G[r * HP + k] * Li[k * HP + j];
        Li[r * HP + j] = -s / G[r * HP + r];
      }
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < n; l += WG) {
    double y[EIGP], o[EIGP];
#pragma unroll
    for (int k = 0; k < EIGP; ++k) y[k] = Y[(size_t)l * EIGP + k];
#pragma unroll
    for (int j = 0; j < EIGP; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k <= j; ++k) s = fma(y[k], Li[j * HP + k], s);
      o[j] = s;
    }
#pragma unroll
    for (int k = 0; k < EIGP; ++k) Y[(size_t)l * EIGP + k] = o[k];
  }
  __syncthreads();
}

// Rayleigh-Ritz step of the subspace iteration (see file header).
__global__ void __launch_bounds__(WG) k_eig_rr(Plan p, const double *__restrict__ val,
                                               const double *__restrict__ sdiag,
                                               double *X, double *Y,
                                               double *__restrict__ BQ, double tol,
                                               int *__restrict__ conv, double *__restrict__ lam) {
  const int i = blockIdx.x;
  if (conv[i]) return;
  __shared__ double H[EIGP * HP], V[EIGP * HP], Li[EIGP * HP];
  __shared__ double cs[4 * EIGP / 2];
  __shared__ double res[EIGP][WG / 64];
  __shared__ int perm[EIGP];
  __shared__ double theta[EIGP];
  __shared__ int flag;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int npad = p.vp_ptr[i + 1] - p.vp_ptr[i];
  double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  double *Yi = Y + (size_t)p.vp_ptr[i] * EIGP;
  double *Bi = BQ + (size_t)p.vp_ptr[i] * EIGP;
  const int m = p.mi[i];
  const int t = threadIdx.x;
  const bool small = ni <= EIGP;

  if (small) {
    // dense B_i (n_i <= EIGP) padded with a diagonal above the spectrum [0, 2]
    for (int e = t; e < EIGP * EIGP; e += WG) {
      const int a = e / EIGP, b = e % EIGP;
      H[a * HP + b] = (a == b) ? (a < ni ? 1.0 : 3.0 + a) : 0.0;
    }
    __syncthreads();
    if (t < ni) {
      const int a = t;
      const double sa = sdiag[r0 + a];
      for (int e = p.loc_rowptr[r0 + a]; e < p.loc_rowptr[r0 + a + 1]; ++e) {
        const int b = p.loc_col[e];
        if (b != a) H[a * HP + b] = val[p.loc_src[e]] / sqrt(sa * sdiag[r0 + b]);
      }
    }
    __syncthreads();
  } else {
    cholqr_pass(Yi, ni, H, Li);
    cholqr_pass(Yi, ni, H, Li);
    // BQ = B_i Y (sparse, unit diagonal)
    for (int l = t; l < ni; l += WG) {
      double acc[EIGP];
#pragma unroll
      for (int k = 0; k < EIGP; ++k) acc[k] = Yi[(size_t)l * EIGP + k];
      const double sl = sdiag[r0 + l];
      for (int e = p.loc_rowptr[r0 + l]; e < p.loc_rowptr[r0 + l + 1]; ++e) {
        const int c = p.loc_col[e];
        if (c == l) continue;
        const double b = val[p.loc_src[e]] / sqrt(sl * sdiag[r0 + c]);
#pragma unroll
        for (int k = 0; k < EIGP; ++k) acc[k] = fma(b, Yi[(size_t)c * EIGP + k], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < EIGP; ++k) Bi[(size_t)l * EIGP + k] = acc[k];
    }
    __syncthreads();
    gram16(Yi, Bi, ni, H);
    __syncthreads();
    {  // symmetrise
      const int a = t >> 4, b = t & 15;
      double hs = 0.5 * (H[a * HP + b] + H[b * HP + a]);
      __syncthreads();
      H[a * HP + b] = hs;
    }
    __syncthreads();
  }
  jacobi16(H, V, cs, &flag);
  if (t == 0) {
    for (int a = 0; a < EIGP; ++a) {
      perm[a] = a;
      theta[a] = H[a * HP + a];
    }
    for (int a = 1; a < EIGP; ++a) {  // insertion sort, ascending
      int pa = perm[a];
      double th = theta[a];
      int b = a - 1;
      while (b >= 0 && theta[b] > th) {
        theta[b + 1] = theta[b];
        perm[b + 1] = perm[b];
        --b;
      }
      theta[b + 1] = th;
      perm[b + 1] = pa;
    }
  }
  __syncthreads();
  const int nchk = (m + 1 < ni ? m + 1 : ni);  // pairs that must converge
  if (small) {
    for (int e = t; e < npad * EIGP; e += WG) {
      const int l = e / EIGP, j = e % EIGP;
      Xi[e] = (l < ni) ? V[l * HP + perm[j]] : 0.0;
    }
  } else {
    double rs[EIGP];
#pragma unroll
    for (int j = 0; j < EIGP; ++j) rs[j] = 0.0;
    for (int l = t; l < ni; l += WG) {
      double y[EIGP], b[EIGP];
#pragma unroll
      for (int k = 0; k < EIGP; ++k) {
        y[k] = Yi[(size_t)l * EIGP + k];
        b[k] = Bi[(size_t)l * EIGP + k];
      }
#pragma unroll
      for (int j = 0; j < EIGP; ++j) {
        const int pj = perm[j];
        double x = 0.0, bx = 0.0;
#pragma unroll
        for (int k = 0; k < EIGP; ++k) {
          const double v = V[k * HP + pj];
          x = fma(y[k], v, x);
          bx = fma(b[k], v, bx);
        }
        Xi[(size_t)l * EIGP + j] = x;
        const double rr = bx - theta[j] * x;
        rs[j] = fma(rr, rr, rs[j]);
      }
    }
    const int lane = t & 63, w = t >> 6;
#pragma unroll
    for (int j = 0; j < EIGP; ++j) {
      double s = wave_sum(rs[j]);
      if (lane == 0) res[j][w] = s;
    }
  }
  __syncthreads();
  if (t == 0) {
    double worst = 0.0;
    if (!small) {
      for (int j = 0; j < nchk; ++j) {
        double s = 0.0;
        for (int w = 0; w < WG / 64; ++w) s += res[j][w];
        s = sqrt(s);
        if (s > worst || !(s == s)) worst = (s == s) ? s : 1e300;
      }
    }
    conv[i] = (worst <= tol) ? 1 : 0;
    const int ld = p.nev + 1;
    for (int j = 0; j < ld; ++j) lam[(size_t)i * ld + j] = (j < nchk) ? theta[j] : __builtin_nan("");
  }
}

// psi = S^{-1/2} z for the m_i kept columns, sign: largest |psi| entry
// positive (ties: lowest global dof), Phi = psi / multiplicity (pou == 0).
__global__ void __launch_bounds__(WG) k_build_basis(Plan p, const double *__restrict__ sdiag,
                                                    const double *__restrict__ X,
                                                    double *__restrict__ phi, int pou) {
  const int i = blockIdx.x;
  const int r0 = p.sd_ptr[i], ni = p.sd_ptr[i + 1] - r0;
  const int m = p.mi[i], nev = p.nev;
  const double *Xi = X + (size_t)p.vp_ptr[i] * EIGP;
  __shared__ double bestv[WG / 64], bests[WG / 64];
  __shared__ int bestg[WG / 64];
  __shared__ double sgn[EIGP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = 0; k < m; ++k) {
    double bv = -1.0;
    int bg = 0x7fffffff;
    double bs = 1.0;
    for (int l = threadIdx.x; l < ni; l += WG) {
      const double ps = Xi[(size_t)l * EIGP + k] / sqrt(sdiag[r0 + l]);
      const double a = fabs(ps);
      const int g = p.sd_dofs[r0 + l];
      if (a > bv || (a == bv && g < bg)) {
        bv = a;
        bg = g;
        bs = ps < 0.0 ? -1.0 : 1.0;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int og = __shfl_xor(bg, o, 64);
      const double os = __shfl_xor(bs, o, 64);
      if (ov > bv || (ov == bv && og < bg)) {
        bv = ov;
        bg = og;
        bs = os;
      }
    }
    __syncthreads();
    if (lane == 0) {
      bestv[w] = bv;
      bestg[w] = bg;
      bests[w] = bs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = bestv[0];
      int g = bestg[0];
      double s = bests[0];
      for (int u = 1; u < WG / 64; ++u)
        if (bestv[u] > v || (bestv[u] == v && bestg[u] < g)) {
          v = bestv[u];
          g = bestg[u];
          s = bests[u];
        }
      sgn[k] = s;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ni * nev; e += WG) {
    const int l = e / nev, k = e % nev;
    double v = 0.0;
    if (k < m) {
      v = sgn[k] * Xi[(size_t)l * EIGP + k] / sqrt(sdiag[r0 + l]);
      if (pou == 0) v /= (double)p.mult[p.sd_dofs[r0 + l]];
    }
    phi[(size_t)(r0 + l) * nev + k] = v;
  }
}

__global__ void k_basis_convert(const double *__restrict__ src, void *__restrict__ dst,
                                size_t count, int bf16) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x) {
    if (bf16)
      reinterpret_cast<__hip_bfloat16 *>(dst)[e] = __float2bfloat16((float)src[e]);
    else
      reinterpret_cast<float *>(dst)[e] = (float)src[e];
  }
}

// ------------------------------------------------------------- launchers ---
void launch_eig_init(hipStream_t s, const Plan &p, const double *sdiag, double *X) {
  hipLaunchKernelGGL(k_eig_init, dim3(p.N), dim3(WG), 0, s, p, sdiag, X);
}

void launch_eig_rr(hipStream_t s, const Plan &p, const double *val, const double *sdiag, double *X,
                   double *Y, double *BQ, double tol, int *conv, double *lam) {
  hipLaunchKernelGGL(k_eig_rr, dim3(p.N), dim3(WG), 0, s, p, val, sdiag, X, Y, BQ, tol, conv, lam);
}

void launch_build_basis(hipStream_t s, const Plan &p, const double *sdiag, const double *X,
                        double *phi, int pou) {
  hipLaunchKernelGGL(k_build_basis, dim3(p.N), dim3(WG), 0, s, p, sdiag, X, phi, pou);
}

void launch_basis_convert(hipStream_t s, const double *phi, void *dst, size_t count, int bf16) {
  if (count == 0) return;
  size_t b = (count + WG - 1) / WG;
  if (b > 65535) b = 65535;
  hipLaunchKernelGGL(k_basis_convert, dim3((unsigned)b), dim3(WG), 0, s, phi, dst, count, bf16);
}

}  // namespace amsp
