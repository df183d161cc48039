// CSR SpMV and the fused CG vector updates with deterministic reductions.
//
// Every reduction is two-stage: each workgroup writes one partial (wavefront
// shuffles, then a fixed-order LDS sum) and the consumer adds the partials in
// index order, so results are bitwise reproducible run to run.  In the CG
// iteration the consumer is the next kernel itself: each of its workgroups
// sums the (at most 1024) partials redundantly, obtains the same scalar, and
// workgroup 0 records it in the device state; no single-workgroup kernels
// and no atomics.  Kernels read the 'done' flag first and return at once
// after convergence, which lets the host launch iterations in chunks.
#include "k_common.h"

namespace amsp {

int reduce_blocks(int n) {
  int b = (n + WG - 1) / WG;
  if (b > MAX_PARTIALS) b = MAX_PARTIALS;
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
    st->rz_ring[st->it & 1] = rz;
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

// CG step t, direction part.  Unless this is the first step after a (re)start,
// iteration t-1 has just finished: r.r (partials from k_cg_update), r.z
// (partials from the preconditioner's scatter) and, for the flexible form,
// r.z_old decide convergence and beta; then p_new = z + beta p_old and
// q = A p_new (neighbours' p_new entries recomputed from z and p_old), with
// partials p_new.q.  rz of step t is kept in rz_ring[t & 1] so that no
// workgroup reads a value this kernel is writing.
__global__ void __launch_bounds__(WG) k_cg_dir(int n, const long long *__restrict__ sptr,
                                               const int *__restrict__ scol,
                                               const double *__restrict__ sval,
                                               const double *__restrict__ z,
                                               const double *__restrict__ pold,
                                               double *__restrict__ pnew, double *__restrict__ q,
                                               double *__restrict__ part_pq, PcgState *st,
                                               const double *__restrict__ part_rr,
                                               const double *__restrict__ part_rz,
                                               const double *__restrict__ part_rzo, int nb, int t,
                                               int first, int flexible) {
  if (st->done) return;
  __shared__ double sh[3][WG / 64];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // q = A p with p = z + beta p_old formed on the fly, on the sliced layout:
  // U rows per thread (one 64-row slice per wavefront each), the first JU
  // entries of every row loaded together.  The first rows' entries do not
  // depend on beta: they are loaded before the partial sums are reduced, so
  // that the two latencies overlap.
  constexpr int U = 2, JU = 8;
  const int stride = gridDim.x * WG;
  long long base[U];
  int wd[U];
  int cj[U][JU];
  double vj[U][JU];
  auto load_rows = [&](int i0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      const int sl = i >> 6;
      base[u] = i < n ? sptr[sl] : 0;
      wd[u] = i < n ? (int)((sptr[sl + 1] - base[u]) >> 6) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < JU; ++j) {
        const bool in = j < wd[u];
        const long long e = base[u] + (long long)j * 64 + lane;
        cj[u][j] = in ? scol[e] : 0;
        vj[u][j] = in ? sval[e] : 0.0;
      }
  };
  int i0 = blockIdx.x * WG + threadIdx.x;
  if (i0 < n) load_rows(i0);
  double beta = 0.0;
  if (!first) {
    // the three fixed-order sums of partials in one pass (the same order in
    // every workgroup, so every workgroup takes the same beta)
    double a[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += WG) {
      a[0] += part_rr[k];
      a[1] += part_rz[k];
      if (flexible) a[2] += part_rzo[k];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) a[m] = wave_sum(a[m]);
    if (lane == 0) {
#pragma unroll
      for (int m = 0; m < 3; ++m) sh[m][w] = a[m];
    }
    __syncthreads();
    double rsum[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int v = 0; v < WG / 64; ++v) rsum[m] += sh[m][v];
    const double rr = rsum[0], rz = rsum[1], rzo = flexible ? rsum[2] : 0.0;
    int stop = 0, brk = 0;
    if (!isfinite(rr)) {
      stop = brk = 1;
    } else if (rr <= st->tol2 || t >= st->maxit) {
      stop = 1;
    } else if (!isfinite(rz) || !(rz > 0.0)) {
      stop = brk = 1;
    }
    if (!stop) beta = (flexible ? rz - rzo : rz) / st->rz_ring[(t - 1) & 1];
    if (lead) {
      st->rr = rr;
      st->it = t;
      if (st->hist && t < st->hist_cap) st->hist[t] = rr;
      if (stop) {
        st->breakdown |= brk;
        st->done = 1;
      } else {
        st->rz_ring[t & 1] = rz;
        st->rz = rz;
        st->beta = beta;
      }
    }
    if (stop) return;
  }
  double acc = 0.0;
  for (; i0 < n; i0 += U * stride) {
    double sacc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) sacc[u] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < JU; ++j)
        if (j < wd[u]) {
          const int c = cj[u][j];
          sacc[u] = fma(vj[u][j], fma(beta, pold[c], z[c]), sacc[u]);
        }
#pragma unroll
    for (int u = 0; u < U; ++u)
      for (int j = JU; j < wd[u]; ++j) {  // rows longer than JU entries
        const long long e = base[u] + (long long)j * 64 + lane;
        const int c = scol[e];
        sacc[u] = fma(sval[e], fma(beta, pold[c], z[c]), sacc[u]);
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      if (i < n) {
        const double pi = fma(beta, pold[i], z[i]);
        pnew[i] = pi;
        q[i] = sacc[u];
        acc = fma(pi, sacc[u], acc);
      }
    }
    if (i0 + U * stride < n) load_rows(i0 + U * stride);
  }
  double tot = block_sum(acc, sh[0]);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = tot;
}

// Sliced copy of the CSR matrix for the CG matrix product: 64-row slices,
// slice s holding (sptr[s+1] - sptr[s]) / 64 entries per row, column-major
// inside the slice (entry j of row 64s + l at sptr[s] + 64j + l), short rows
// padded with zero values pointing at their own row.
__global__ void k_csr_to_sell(int n, const int *__restrict__ rp, const int *__restrict__ col,
                              const double *__restrict__ val, const long long *__restrict__ sptr,
                              int *__restrict__ scol, double *__restrict__ sval) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int sl = i >> 6, lane = i & 63;
    const long long base = sptr[sl];
    const int w = (int)((sptr[sl + 1] - base) >> 6);
    const int e0 = rp[i], len = rp[i + 1] - e0;
    for (int j = 0; j < w; ++j) {
      const long long e = base + (long long)j * 64 + lane;
      scol[e] = j < len ? col[e0 + j] : i;
      sval[e] = j < len ? val[e0 + j] : 0.0;
    }
  }
}

// CG step t, update part: alpha = rz_t / p.q (p.q from this step's direction
// partials), x += alpha p, r -= alpha q, partials r.r and, when zold is
// given, r_new.z_old for the flexible beta.
__global__ void __launch_bounds__(WG) k_cg_update(int n, double *__restrict__ x,
                                                  double *__restrict__ r,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ q, PcgState *st,
                                                  const double *__restrict__ part_pq, int nb, int t,
                                                  double *__restrict__ part_rr,
                                                  const double *__restrict__ zold,
                                                  double *__restrict__ part_rzo) {
  if (st->done) return;
  __shared__ double sh[WG / 64];
  // this thread's first row is loaded before the partial sums are reduced
  // (it does not depend on alpha), so that the two latencies overlap
  int i = blockIdx.x * WG + threadIdx.x;
  double xv = 0.0, pv = 0.0, qv = 0.0, rv = 0.0, zv = 0.0;
  if (i < n) {
    xv = x[i];
    pv = p[i];
    qv = q[i];
    rv = r[i];
    if (zold) zv = zold[i];
  }
  const double pq = sum_partials(part_pq, nb, sh);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead) {
      st->pq = pq;
      st->alpha = 0.0;
      st->breakdown = 1;
      st->done = 1;
    }
    return;
  }
  const double alpha = st->rz_ring[t & 1] / pq;
  if (lead) {
    st->pq = pq;
    st->alpha = alpha;
  }
  double acc = 0.0, acc2 = 0.0;
  for (; i < n; i += gridDim.x * WG) {
    x[i] = fma(alpha, pv, xv);
    const double ri = fma(-alpha, qv, rv);
    r[i] = ri;
    acc = fma(ri, ri, acc);
    if (zold) acc2 = fma(ri, zv, acc2);
    const int inext = i + gridDim.x * WG;
    if (inext < n) {
      xv = x[inext];
      pv = p[inext];
      qv = q[inext];
      rv = r[inext];
      if (zold) zv = zold[inext];
    }
  }
  double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = tot;
  if (zold) {
    tot = block_sum(acc2, sh);
    if (threadIdx.x == 0) part_rzo[blockIdx.x] = tot;
  }
}

// y = A x on the sliced copy of A (64-row slices, column-major inside a
// slice): one row per thread, a wavefront per slice, so every entry load is
// one coalesced access; the first JU entries of a row load together.
__global__ void __launch_bounds__(WG) k_spmv_sell(int n, const long long *__restrict__ sptr,
                                                  const int *__restrict__ scol,
                                                  const double *__restrict__ sval,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y,
                                                  const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int JU = 8;
  const int i = blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const int sl = i >> 6, lane = i & 63;
  const long long base = sptr[sl];
  const int wd = (int)((sptr[sl + 1] - base) >> 6);
  int c[JU];
  double v[JU];
#pragma unroll
  for (int j = 0; j < JU; ++j) {
    const bool in = j < wd;
    const long long e = base + (long long)j * 64 + lane;
    c[j] = in ? scol[e] : i;
    v[j] = in ? sval[e] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < JU; ++j)
    if (j < wd) s = fma(v[j], x[c[j]], s);
  for (int j = JU; j < wd; ++j) {  // rows longer than JU entries
    const long long e = base + (long long)j * 64 + lane;
    s = fma(sval[e], x[scol[e]], s);
  }
  y[i] = s;
}

void launch_spmv_sell(hipStream_t s, int n, const long long *sptr, const int *scol,
                      const double *sval, const double *x, double *y, const int *done) {
  const unsigned b = (unsigned)(((long long)n + WG - 1) / WG);
  if (b == 0) return;
  hipLaunchKernelGGL(k_spmv_sell, dim3(b), dim3(WG), 0, s, n, sptr, scol, sval, x, y, done);
}

// ------------------------------------------ multiplicative two-grid cycle ---
// Vector steps of z = x2 + w S (r - A x2), x2 = x1 + C (r - A x1), x1 = w S r;
// every kernel returns at once after convergence (done flag), like the rest
// of the CG step.
__global__ void __launch_bounds__(WG) k_scale_done(int n, double a, double *__restrict__ x,
                                                   const int *__restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) x[i] *= a;
}

__global__ void __launch_bounds__(WG) k_sub_done(int n, const double *__restrict__ r,
                                                 const double *__restrict__ q,
                                                 double *__restrict__ t,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) t[i] = r[i] - q[i];
}

// y += a x; with partial != 0 also the partial sums of r.y
__global__ void __launch_bounds__(WG) k_axpy_dot(int n, double a, const double *__restrict__ x,
                                                 double *__restrict__ y,
                                                 const double *__restrict__ r,
                                                 double *__restrict__ partial,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    const double yi = fma(a, x[i], y[i]);
    y[i] = yi;
    if (r) acc = fma(r[i], yi, acc);
  }
  if (partial) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

void launch_scale_done(hipStream_t s, int n, double a, double *x, const int *done) {
  hipLaunchKernelGGL(k_scale_done, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, a, x, done);
}
void launch_sub_done(hipStream_t s, int n, const double *r, const double *q, double *t,
                     const int *done) {
  hipLaunchKernelGGL(k_sub_done, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, r, q, t, done);
}
void launch_axpy_dot(hipStream_t s, int n, double a, const double *x, double *y, const double *r,
                     double *partial, const int *done) {
  hipLaunchKernelGGL(k_axpy_dot, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, a, x, y, r, partial,
                     done);
}

// grad[k] = -lambda[row k] * u[col k] over the CSR entries (adjoint of the
// solve; one thread per row).
__global__ void __launch_bounds__(WG) k_grad_values(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col,
                                                    const double *__restrict__ lambda,
                                                    const double *__restrict__ u,
                                                    double *__restrict__ grad) {
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    const double li = lambda[i];
    for (int e = rp[i]; e < rp[i + 1]; ++e) grad[e] = -li * u[col[e]];
  }
}

void launch_grad_values(hipStream_t s, int n, const int *rp, const int *col, const double *lambda,
                        const double *u, double *grad) {
  size_t b = ((size_t)n + WG - 1) / WG;
  if (b > 65535) b = 65535;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_grad_values, dim3((unsigned)b), dim3(WG), 0, s, n, rp, col, lambda, u, grad);
}

// ------------------------------------------------------------- launchers ---
void launch_spmv(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                 const double *x, double *y, double *partial, const int *done) {
  hipLaunchKernelGGL(k_spmv, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, rp, col, val, x, y,
                     partial, done);
}

void launch_cg_dir(hipStream_t s, int n, const long long *sptr, const int *scol,
                   const double *sval, const double *z, const double *pold, double *pnew, double *q,
                   double *part_pq, PcgState *st, const double *part_rr, const double *part_rz,
                   const double *part_rzo, int t, int first, int flexible) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(WG), 0, s, n, sptr, scol, sval, z, pold, pnew, q,
                     part_pq, st, part_rr, part_rz, part_rzo, nb, t, first, flexible);
}

void launch_csr_to_sell(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                        const long long *sptr, int *scol, double *sval) {
  size_t b = ((size_t)n + WG - 1) / WG;
  if (b > 65535) b = 65535;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_csr_to_sell, dim3((unsigned)b), dim3(WG), 0, s, n, rp, col, val, sptr, scol,
                     sval);
}

void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q,
                      PcgState *st, const double *part_pq, int t, double *part_rr,
                      const double *zold, double *part_rzo) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(WG), 0, s, n, x, r, p, q, st, part_pq, nb, t,
                     part_rr, zold, part_rzo);
}

void launch_dot(hipStream_t s, int n, const double *a, const double *b, double *partial,
                const int *done) {
  hipLaunchKernelGGL(k_dot, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, a, b, partial, done);
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

// ------------------------------------------------------ GMRES (Arnoldi) ---
// Classical Gram-Schmidt passes over the basis V (column k at V + k * ldv),
// used twice per step.  Dots: workgroup (b, c) adds rows b, b + nb, ... of
// columns 8c .. 8c+7 into part[k * nb + b]; the reduce kernel then sums each
// column's nb partials in a fixed order.
constexpr int GSC = 8;
__global__ void __launch_bounds__(WG) k_gs_dots(int n, const double *__restrict__ V, size_t ldv,
                                                int k1, const double *__restrict__ w,
                                                double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  const int nb = gridDim.x, c0 = blockIdx.y * GSC;
  double acc[GSC];
#pragma unroll
  for (int c = 0; c < GSC; ++c) acc[c] = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += nb * WG) {
    const double wi = w[i];
    // columns clamped to the last one and loaded unconditionally, so that
    // the GSC loads are in flight together; the surplus ones are dropped
    double vc[GSC];
#pragma unroll
    for (int c = 0; c < GSC; ++c) vc[c] = V[(size_t)min(c0 + c, k1 - 1) * ldv + i];
#pragma unroll
    for (int c = 0; c < GSC; ++c) acc[c] = c0 + c < k1 ? fma(vc[c], wi, acc[c]) : acc[c];
  }
#pragma unroll
  for (int c = 0; c < GSC; ++c) {
    if (c0 + c >= k1) break;  // uniform
    const double t = block_sum(acc[c], sh);
    if (threadIdx.x == 0) part[(size_t)(c0 + c) * nb + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(WG) k_gs_reduce(int nb, const double *__restrict__ part,
                                                  double *__restrict__ out) {
  __shared__ double sh[WG / 64];
  const double t = sum_partials(part + (size_t)blockIdx.x * nb, nb, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// w -= V h (columns 0 .. k1-1, in that order); with part != 0 also the
// partial sums of the updated w.w.
__global__ void __launch_bounds__(WG) k_gs_update(int n, const double *__restrict__ V, size_t ldv,
                                                  int k1, const double *__restrict__ h,
                                                  double *__restrict__ w,
                                                  double *__restrict__ part) {
  __shared__ double sh[WG / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    double wi = w[i];
    // GSC columns' loads at a time (clamped, all issued), used in order
    for (int k0 = 0; k0 < k1; k0 += GSC) {
      double vc[GSC], hc[GSC];
#pragma unroll
      for (int c = 0; c < GSC; ++c) {
        const int k = min(k0 + c, k1 - 1);
        vc[c] = V[(size_t)k * ldv + i];
        hc[c] = h[k];
      }
#pragma unroll
      for (int c = 0; c < GSC; ++c)
        if (k0 + c < k1) wi = fma(-vc[c], hc[c], wi);
    }
    w[i] = wi;
    acc = fma(wi, wi, acc);
  }
  if (part) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// v = w / sqrt(*nrm2) (zero when the norm is zero: the Krylov space is exhausted)
__global__ void __launch_bounds__(WG) k_gs_normalize(int n, const double *__restrict__ w,
                                                     const double *__restrict__ nrm2,
                                                     double *__restrict__ v) {
  const double nr = sqrt(*nrm2);
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG)
    v[i] = nr > 0.0 ? w[i] / nr : 0.0;
}

// x += Z y (columns 0 .. k-1, in that order)
__global__ void __launch_bounds__(WG) k_basis_combine(int n, const double *__restrict__ Z,
                                                      size_t ldz, int k,
                                                      const double *__restrict__ y,
                                                      double *__restrict__ x) {
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(Z[(size_t)j * ldz + i], y[j], s);
    x[i] += s;
  }
}

void launch_gs_dots(hipStream_t s, int n, const double *V, size_t ldv, int k1, const double *w,
                    double *part, double *out) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_gs_dots, dim3(nb, (k1 + GSC - 1) / GSC), dim3(WG), 0, s, n, V, ldv, k1, w,
                     part);
  hipLaunchKernelGGL(k_gs_reduce, dim3(k1), dim3(WG), 0, s, nb, part, out);
}

void launch_gs_update(hipStream_t s, int n, const double *V, size_t ldv, int k1, const double *h,
                      double *w, double *part) {
  hipLaunchKernelGGL(k_gs_update, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, V, ldv, k1, h, w, part);
}

void launch_gs_normalize(hipStream_t s, int n, const double *w, const double *nrm2, double *v) {
  hipLaunchKernelGGL(k_gs_normalize, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, w, nrm2, v);
}

void launch_basis_combine(hipStream_t s, int n, const double *Z, size_t ldz, int k, const double *y,
                          double *x) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_basis_combine, dim3(reduce_blocks(n)), dim3(WG), 0, s, n, Z, ldz, k, y, x);
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

}  // namespace amsp
