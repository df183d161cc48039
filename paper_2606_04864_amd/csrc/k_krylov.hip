// CSR SpMV and the fused CG vector updates with deterministic reductions.
//
// Every reduction is two-stage: each workgroup writes one partial (wavefront
// shuffles, then a fixed-order LDS sum) and a single-workgroup kernel adds the
// partials in index order, so results are bitwise reproducible run to run.
// Scalars (alpha, beta, residual norms, the convergence flag) stay on the
// device; kernels read the 'done' flag first and return at once after
// convergence, which lets the host launch CG iterations in chunks.
#include "k_common.h"

namespace amsp {

int reduce_blocks(int n) {
  int b = (n + WG - 1) / WG;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return b;
}

// q = A p, partial p.q per workgroup (one row per thread, grid-stride).
__global__ void __launch_bounds__(WG) k_spmv(int n, const int *__restrict__ rp,
                                             const int *__restrict__ col,
                                             const double *__restrict__ val,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             double *__restrict__ partial,
                                             const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    double s = 0.0;
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) s = fma(val[e], x[col[e]], s);
    y[i] = s;
    acc = fma(x[i], s, acc);
  }
  double tot = block_sum(acc, sh);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// p_new = z + beta p_old (for the rows this thread owns) and q = A p_new,
// where the neighbours' p_new entries are recomputed from z and p_old;
// partial p_new.q.
__global__ void __launch_bounds__(WG) k_spmv_pupdate(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ z,
                                                     const double *__restrict__ pold,
                                                     double *__restrict__ pnew,
                                                     double *__restrict__ q,
                                                     double *__restrict__ partial,
                                                     const PcgState *__restrict__ st) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  const double beta = st->beta;
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    double s = 0.0;
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) {
      const int c = col[e];
      s = fma(val[e], fma(beta, pold[c], z[c]), s);
    }
    const double pi = fma(beta, pold[i], z[i]);
    pnew[i] = pi;
    q[i] = s;
    acc = fma(pi, s, acc);
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(WG) k_dot(int n, const double *__restrict__ a,
                                            const double *__restrict__ b,
                                            double *__restrict__ partial,
                                            const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) acc = fma(a[i], b[i], acc);
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// x += alpha p; r -= alpha q; partial r.r and, when zold is given, the
// partial r_new.z_old used by the flexible (Polak-Ribiere) beta
__global__ void __launch_bounds__(WG) k_axpy_update(int n, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ q,
                                                    const PcgState *__restrict__ st,
                                                    double *__restrict__ partial,
                                                    const double *__restrict__ zold,
                                                    double *__restrict__ partial_rzo) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  const double alpha = st->alpha;
  double acc = 0.0, acc2 = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    acc = fma(ri, ri, acc);
    if (zold) acc2 = fma(ri, zold[i], acc2);
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
  if (zold) {
    tot = block_sum(acc2, sh);
    if (threadIdx.x == 0) partial_rzo[blockIdx.x] = tot;
  }
}

// r = f - Ax, partial r.r
__global__ void __launch_bounds__(WG) k_residual(int n, const double *__restrict__ f,
                                                 const double *__restrict__ Ax,
                                                 double *__restrict__ r,
                                                 double *__restrict__ partial) {
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    const double ri = f[i] - Ax[i];
    r[i] = ri;
    acc = fma(ri, ri, acc);
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// partial sums of (|A| |x|)_i^2: the scale of the rounding error of any
// float64 residual f - A x (attainable-accuracy floor of the solve)
__global__ void __launch_bounds__(WG) k_abs_spmv_sq(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ partial) {
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s = fma(fabs(val[e]), fabs(x[col[e]]), s);
    acc = fma(s, s, acc);
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_copy_scale(int n, const double *__restrict__ a, double *__restrict__ b,
                             double alpha) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    b[i] = alpha * a[i];
}

__global__ void k_fill(size_t n, double *__restrict__ a, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_fill_int(size_t n, int *__restrict__ a, int v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Fixed-order sum of nb partials by one workgroup.
__device__ double sum_partials(const double *__restrict__ partial, int nb, double *sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += WG) acc += partial[i];
  return block_sum(acc, sh);
}

__global__ void __launch_bounds__(WG) k_sum_partials(const double *partial, int nb, double *out) {
  __shared__ double sh[WG / 64];
  double t = sum_partials(partial, nb, sh);
  if (threadIdx.x == 0) *out = t;
}

// Start (or restart) of CG: rr = r.r, rz = r.z, flags.
__global__ void __launch_bounds__(WG) k_pcg_init(PcgState *st, const double *prr, int nbrr,
                                                 const double *prz, int nbrz, double rtol,
                                                 int maxit) {
  __shared__ double sh[WG / 64];
  const double rr = sum_partials(prr, nbrr, sh);
  const double rz = sum_partials(prz, nbrz, sh);
  if (threadIdx.x == 0) {
    if (rtol >= 0.0) {  // fresh start: r = f
      st->f2 = rr;
      st->tol2 = rtol * rtol * rr;
      st->it = 0;
      st->breakdown = 0;
      st->maxit = maxit;
    }
    st->rr = rr;
    st->rz = rz;
    st->rz_old = rz;
    if (st->hist && st->it < st->hist_cap) st->hist[st->it] = rr;
    st->beta = 0.0;
    st->alpha = 0.0;
    int done = (rr <= st->tol2) ? 1 : 0;
    if (!isfinite(rr) || !isfinite(rz)) {
      st->breakdown = 1;
      done = 1;
    } else if (!done && !(rz > 0.0)) {
      st->breakdown = 1;
      done = 1;
    }
    if (st->it >= st->maxit) done = 1;
    st->done = done;
  }
}

__global__ void __launch_bounds__(WG) k_pcg_alpha(PcgState *st, const double *partial, int nb) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  const double pq = sum_partials(partial, nb, sh);
  if (threadIdx.x == 0) {
    st->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      st->breakdown = 1;
      st->done = 1;
      st->alpha = 0.0;
    } else {
      st->alpha = st->rz / pq;
    }
  }
}

__global__ void __launch_bounds__(WG) k_pcg_rr(PcgState *st, const double *partial, int nb) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  const double rr = sum_partials(partial, nb, sh);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->it += 1;
    if (st->hist && st->it < st->hist_cap) st->hist[st->it] = rr;
    if (!isfinite(rr)) {
      st->breakdown = 1;
      st->done = 1;
    } else if (rr <= st->tol2 || st->it >= st->maxit) {
      st->done = 1;
    }
  }
}

// beta = rz_new / rz (flexible: (rz_new - r_new.z_old) / rz)
__global__ void __launch_bounds__(WG) k_pcg_beta(PcgState *st, const double *prz, int nb,
                                                 const double *przo, int flexible) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  const double rz = sum_partials(prz, nb, sh);
  double rzo = 0.0;
  if (flexible) rzo = sum_partials(przo, nb, sh);
  if (threadIdx.x == 0) {
    double num = flexible ? (rz - rzo) : rz;
    if (!isfinite(rz) || !(rz > 0.0)) {
      st->breakdown = 1;
      st->done = 1;
      st->beta = 0.0;
    } else {
      st->beta = num / st->rz;
      st->rz_old = st->rz;
      st->rz = rz;
    }
  }
}

// ------------------------------------------------------------- launchers ---
void launch_spmv(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                 const double *x, double *y, double *partial, const int *done) {
  hipLaunchKernelGGL(k_spmv, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, rp, col, val, x, y,
                     partial, done);
}

void launch_spmv_pupdate_st(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                            const double *z, const double *pold, double *pnew, double *q,
                            double *partial, const PcgState *st) {
  hipLaunchKernelGGL(k_spmv_pupdate, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, rp, col, val, z,
                     pold, pnew, q, partial, st);
}

void launch_dot(hipStream_t s, int n, const double *a, const double *b, double *partial,
                const int *done) {
  hipLaunchKernelGGL(k_dot, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, a, b, partial, done);
}

void launch_axpy_update_st(hipStream_t s, int n, double *x, double *r, const double *p,
                           const double *q, const PcgState *st, double *partial,
                           const double *zold, double *partial_rzo) {
  hipLaunchKernelGGL(k_axpy_update, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, x, r, p, q, st,
                     partial, zold, partial_rzo);
}

void launch_residual(hipStream_t s, int n, const double *f, const double *Ax, double *r,
                     double *partial) {
  hipLaunchKernelGGL(k_residual, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, f, Ax, r, partial);
}

void launch_abs_spmv_sq(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                        const double *x, double *partial) {
  hipLaunchKernelGGL(k_abs_spmv_sq, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, rp, col, val, x,
                     partial);
}

void launch_copy_scale(hipStream_t s, int n, const double *a, double *b, double alpha) {
  hipLaunchKernelGGL(k_copy_scale, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, a, b, alpha);
}

void launch_fill(hipStream_t s, size_t n, double *a, double v) {
  if (n == 0) return;
  size_t b = (n + WG - 1) / WG;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)b), dim3(WG), 0, s, n, a, v);
}

void launch_fill_int(hipStream_t s, size_t n, int *a, int v) {
  if (n == 0) return;
  size_t b = (n + WG - 1) / WG;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)b), dim3(WG), 0, s, n, a, v);
}

void launch_sum_partials(hipStream_t s, const double *partial, int nb, double *out) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, s, partial, nb, out);
}

void launch_pcg_init(hipStream_t s, PcgState *st, const double *prr, int nbrr, const double *prz,
                     int nbrz, double rtol, int maxit) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(WG), 0, s, st, prr, nbrr, prz, nbrz, rtol, maxit);
}

void launch_pcg_alpha(hipStream_t s, PcgState *st, const double *partial, int nb) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(WG), 0, s, st, partial, nb);
}

void launch_pcg_rr(hipStream_t s, PcgState *st, const double *partial, int nb) {
  hipLaunchKernelGGL(k_pcg_rr, dim3(1), dim3(WG), 0, s, st, partial, nb);
}

void launch_pcg_beta(hipStream_t s, PcgState *st, const double *prz, int nb, const double *przo,
                     int flexible) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(WG), 0, s, st, prz, nb, przo, flexible);
}

}  // namespace amsp
