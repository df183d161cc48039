// Independent problems solved together (a block-diagonal system whose blocks
// are the problems): one CG recurrence per (problem, column) pair, sharing
// every matrix product and preconditioner application, which act on all
// problems and columns at once.  The vector work is split into row blocks
// that never cross a problem boundary, so every reduction is a fixed-order
// sum of whole blocks per (problem, column): results are bitwise
// reproducible, and a problem's scalars do not depend on the others.
//
// Recurrence r = k * nseg + s (column k, problem s).  Rows of block b:
// [brow[b], brow[b+1]), its problem bseg[b]; problem s owns blocks
// [sblk[s], sblk[s+1]).
#include "k_common.h"

namespace amsp {

struct SegCgState {
  double *rz, *f2, *rr;  // nrec each
  int *active, *its;     // nrec each
  int *broken;           // nrec: 1 once the recurrence broke down
  int *flags;            // [1] active recurrences after the step
};

// part[k * nblk + b] = sum over the block's rows of A_k . B_k
__global__ void __launch_bounds__(WG) k_seg_dots(int nblk, const long long *__restrict__ brow,
                                                 size_t ld, const double *__restrict__ A,
                                                 const double *__restrict__ B,
                                                 double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  const int b = blockIdx.x, k = blockIdx.y;
  const double *a = A + (size_t)k * ld, *bb = B + (size_t)k * ld;
  double acc = 0.0;
  for (long long i = brow[b] + threadIdx.x; i < brow[b + 1]; i += WG) acc = fma(a[i], bb[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)k * nblk + b] = t;
}

// out[k * nseg + s] = sum of the problem's block partials, in block order
__global__ void __launch_bounds__(WG) k_seg_reduce(int nseg, int nblk, const int *__restrict__ sblk,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ out) {
  __shared__ double sh[WG / 64];
  const int s = blockIdx.x, k = blockIdx.y;
  double acc = 0.0;
  for (int b = sblk[s] + threadIdx.x; b < sblk[s + 1]; b += WG) acc += part[(size_t)k * nblk + b];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(size_t)k * nseg + s] = t;
}

// x += alpha p, r -= alpha q with the block's problem's alpha; partials of r.r
__global__ void __launch_bounds__(WG) k_seg_update(int nblk, int nseg,
                                                   const long long *__restrict__ brow,
                                                   const int *__restrict__ bseg, size_t ld,
                                                   const double *__restrict__ alpha,
                                                   const double *__restrict__ P,
                                                   const double *__restrict__ Q,
                                                   double *__restrict__ X, double *__restrict__ R,
                                                   double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  const int b = blockIdx.x, k = blockIdx.y;
  const double a = alpha[(size_t)k * nseg + bseg[b]];
  const size_t o = (size_t)k * ld;
  double acc = 0.0;
  for (long long i = brow[b] + threadIdx.x; i < brow[b + 1]; i += WG) {
    X[o + i] = fma(a, P[o + i], X[o + i]);
    const double ri = fma(-a, Q[o + i], R[o + i]);
    R[o + i] = ri;
    acc = fma(ri, ri, acc);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)k * nblk + b] = t;
}

// p = z + beta p with the block's problem's beta
__global__ void __launch_bounds__(WG) k_seg_direction(int nseg, const long long *__restrict__ brow,
                                                      const int *__restrict__ bseg, size_t ld,
                                                      const double *__restrict__ beta,
                                                      const double *__restrict__ Z,
                                                      double *__restrict__ P) {
  const int b = blockIdx.x, k = blockIdx.y;
  const double be = beta[(size_t)k * nseg + bseg[b]];
  const size_t o = (size_t)k * ld;
  for (long long i = brow[b] + threadIdx.x; i < brow[b + 1]; i += WG) P[o + i] = fma(be, P[o + i], Z[o + i]);
}

// alpha_r = (r.z)_r / (p.Ap)_r for active recurrences (0 otherwise); p.Ap <= 0
// or a non-finite ratio stops the recurrence and marks it broken
__global__ void __launch_bounds__(WG) k_seg_alpha(int nrec, SegCgState st,
                                                  const double *__restrict__ pq,
                                                  double *__restrict__ alpha) {
  const int r = blockIdx.x * WG + threadIdx.x;
  if (r >= nrec) return;
  double c = 0.0;
  if (st.active[r]) {
    const double q = st.rz[r] / pq[r];
    if (!(pq[r] > 0.0) || !isfinite(q)) {
      st.broken[r] = 1;
      st.active[r] = 0;
    } else {
      c = q;
    }
  }
  alpha[r] = c;
}

// After the update (one workgroup): an active recurrence with r.r <= rtol2 f.f
// stops; the others take beta = (r.z)' / (r.z).  Counts the active ones.
__global__ void __launch_bounds__(WG) k_seg_beta(int nrec, SegCgState st,
                                                 const double *__restrict__ rr,
                                                 const double *__restrict__ rz, double rtol2,
                                                 double *__restrict__ beta) {
  __shared__ int cnt[WG / 64];
  int act = 0;
  for (int r = threadIdx.x; r < nrec; r += WG) {
    double c = 0.0;
    st.rr[r] = rr[r];
    if (st.active[r]) {
      st.its[r] += 1;
      if (!isfinite(rr[r])) {
        st.broken[r] = 1;
        st.active[r] = 0;
      } else if (rr[r] <= rtol2 * st.f2[r]) {
        st.active[r] = 0;
      } else {
        c = rz[r] / st.rz[r];
        st.rz[r] = rz[r];
      }
    }
    beta[r] = c;
    act += st.active[r];
  }
  for (int off = 32; off > 0; off >>= 1) act += __shfl_xor(act, off, 64);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = act;
  __syncthreads();
  if (threadIdx.x == 0) st.flags[1] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// w_i = sum_j |a_ij| |u_j| (the attainable-accuracy floor of the residual)
__global__ void __launch_bounds__(WG) k_abs_spmv_rows(int n, const int *__restrict__ rp,
                                                      const int *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ u,
                                                      double *__restrict__ w) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) s = fma(fabs(val[e]), fabs(u[col[e]]), s);
  w[i] = s;
}

// R = F - Q for every column
__global__ void __launch_bounds__(WG) k_sub_columns(size_t tot, const double *__restrict__ F,
                                                    const double *__restrict__ Q,
                                                    double *__restrict__ R) {
  for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < tot; e += (size_t)gridDim.x * WG)
    R[e] = F[e] - Q[e];
}

// flag[0] = 1 if a stored entry couples two problems (row and column in
// different ones); problem of a row by binary search in sptr (nseg + 1)
__global__ void __launch_bounds__(WG) k_check_blocks(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ col, int nseg,
                                                     const long long *__restrict__ sptr,
                                                     int *__restrict__ flag) {
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = nseg;  // sptr[lo] <= i < sptr[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sptr[mid] <= i) lo = mid; else hi = mid;
  }
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (col[e] < sptr[lo] || col[e] >= sptr[lo + 1]) {
      atomicOr(flag, 1);
      return;
    }
}

// ------------------------------------------------------------- launchers ---
void launch_seg_dots(hipStream_t s, int nblk, int nseg, const long long *brow, const int *sblk,
                     size_t ld, int nr, const double *A, const double *B, double *part,
                     double *out) {
  hipLaunchKernelGGL(k_seg_dots, dim3(nblk, nr), dim3(WG), 0, s, nblk, brow, ld, A, B, part);
  hipLaunchKernelGGL(k_seg_reduce, dim3(nseg, nr), dim3(WG), 0, s, nseg, nblk, sblk, part, out);
}

void launch_seg_update(hipStream_t s, int nblk, int nseg, const long long *brow, const int *bseg,
                       const int *sblk, size_t ld, int nr, const double *alpha, const double *P,
                       const double *Q, double *X, double *R, double *part, double *rr) {
  hipLaunchKernelGGL(k_seg_update, dim3(nblk, nr), dim3(WG), 0, s, nblk, nseg, brow, bseg, ld,
                     alpha, P, Q, X, R, part);
  hipLaunchKernelGGL(k_seg_reduce, dim3(nseg, nr), dim3(WG), 0, s, nseg, nblk, sblk, part, rr);
}

void launch_seg_direction(hipStream_t s, int nblk, int nseg, const long long *brow,
                          const int *bseg, size_t ld, int nr, const double *beta, const double *Z,
                          double *P) {
  hipLaunchKernelGGL(k_seg_direction, dim3(nblk, nr), dim3(WG), 0, s, nseg, brow, bseg, ld, beta,
                     Z, P);
}

void launch_seg_alpha(hipStream_t s, int nrec, double *rz, double *f2, double *rr, int *active,
                      int *its, int *broken, int *flags, const double *pq, double *alpha) {
  const SegCgState st{rz, f2, rr, active, its, broken, flags};
  hipLaunchKernelGGL(k_seg_alpha, dim3((nrec + WG - 1) / WG), dim3(WG), 0, s, nrec, st, pq, alpha);
}

void launch_seg_beta(hipStream_t s, int nrec, double *rz, double *f2, double *rr, int *active,
                     int *its, int *broken, int *flags, const double *rrn, const double *rzn,
                     double rtol2, double *beta) {
  const SegCgState st{rz, f2, rr, active, its, broken, flags};
  hipLaunchKernelGGL(k_seg_beta, dim3(1), dim3(WG), 0, s, nrec, st, rrn, rzn, rtol2, beta);
}

void launch_abs_spmv_rows(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                          const double *u, double *w) {
  hipLaunchKernelGGL(k_abs_spmv_rows, dim3((n + WG - 1) / WG), dim3(WG), 0, s, n, rp, col, val, u,
                     w);
}

void launch_sub_columns(hipStream_t s, size_t tot, const double *F, const double *Q, double *R) {
  size_t b = (tot + WG - 1) / WG;
  if (b > 65535) b = 65535;
  if (b == 0) return;
  hipLaunchKernelGGL(k_sub_columns, dim3((unsigned)b), dim3(WG), 0, s, tot, F, Q, R);
}

void launch_check_blocks(hipStream_t s, int n, const int *rp, const int *col, int nseg,
                         const long long *sptr, int *flag) {
  hipLaunchKernelGGL(k_check_blocks, dim3((n + WG - 1) / WG), dim3(WG), 0, s, n, rp, col, nseg,
                     sptr, flag);
}

}  // namespace amsp
