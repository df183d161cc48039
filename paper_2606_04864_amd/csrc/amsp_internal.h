// Internal declarations shared by the host library and the HIP kernels.
// Not part of the public ABI (see include/amsp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "amsp_consts.h"

namespace amsp {

// Device view of the planned subdomain structure (all arrays on the device).
struct Plan {
  int N;                    // subdomains
  int nev;                  // requested eigenvectors (row stride of basis arrays)
  const int *sd_ptr;        // [N+1] offsets of each region in the concatenated local vectors
  const int *sd_dofs;       // [sum n_i] global dof of each local index (local order)
  const int *nat;           // [sum n_i] rank of that dof among the region's dofs by global
                            // index: position in the ascending-index layout of the
                            // local corrections and of the basis copy read by the apply
  const int *asc;           // [sum n_i] the region's dofs in ascending order, and the local
  const int *lop;           //   index of each: asc[r0 + nat[r0 + l]] = sd_dofs[r0 + l],
                            //   lop[r0 + nat[r0 + l]] = l
  const int *vp_ptr;        // [N+1] padded offsets (multiples of 64) for tile-aligned vectors
  const int *trow_ptr;      // [N+1] offsets into the per-tile-row arrays
  const int *tfirst;        // [sum nt_i] first tile column of each tile row
  const long long *toff;    // [sum nt_i] pool index of the first off-diagonal tile of each
                            // tile row (tiles J = first(I) .. I-1 follow in order)
  long long noff;           // off-diagonal tiles in the pool; the packed diagonal tiles
                            // follow at entry noff*TE, DE entries per tile row
  const int *eptr;          // [sum npad_i + N] envelope of the factor below the diagonal
  const int *uptr;          //   tiles, per region npad_i + 1 segment starts relative to
  const long long *ebase;   //   ebase[i]: row form (eptr) and column form (uptr)
  const int *sfb, *sbb;     // [sum nt_i] start of each 64-row block in its region's forward
  const long long *sfr;     //   / backward stream; [N+1] region starts of the forward
  const long long *sbr;     //   / backward streams (see launch_local_apply_stream)
  const int *loc_rowptr;    // [sum n_i + 1] local CSR of A_i (rows in local order)
  const int *loc_col;       //   local column index
  const int *loc_src;       //   index of the value in the global CSR
  const int *mi;            // [N] kept eigenvectors m_i
  const int *coff;          // [N+1] coarse offsets
  const int *mult;          // [n] dof multiplicity
};

// PCG scalar state kept on the device.
struct PcgState {
  double rz, rz_ring[2], pq, rr, alpha, beta, tol2, f2;
  int it, done, breakdown, maxit;
  double *hist;   // rr after each iteration (hist[it]); may be null
  int hist_cap;
};

// ---------------------------------------------------------------- krylov ---
int reduce_blocks(int n);
void launch_spmv(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                 const double *x, double *y, double *partial, const int *done);
// One CG step t in two kernels (direction + update); the scalar reductions
// of the previous kernels are folded in (see k_krylov.hip).
// The direction kernel's matrix product reads the sliced copy of A (64-row
// slices, column-major inside a slice; see launch_csr_to_sell).
void launch_cg_dir(hipStream_t s, int n, const long long *sptr, const int *scol,
                   const double *sval, const double *z, const double *pold, double *pnew, double *q,
                   double *part_pq, PcgState *st, const double *part_rr, const double *part_rz,
                   const double *part_rzo, int t, int first, int flexible);
// y = A x on the sliced copy (amsp_spmv).
void launch_spmv_sell(hipStream_t s, int n, const long long *sptr, const int *scol,
                      const double *sval, const double *x, double *y, const int *done = nullptr);
// Multiplicative cycle steps (all return at once when *done is set):
// x *= a; t = r - q; y += a x with optional partial sums of r.y.
void launch_scale_done(hipStream_t s, int n, double a, double *x, const int *done);
void launch_sub_done(hipStream_t s, int n, const double *r, const double *q, double *t,
                     const int *done);
void launch_axpy_dot(hipStream_t s, int n, double a, const double *x, double *y, const double *r,
                     double *partial, const int *done);
// Sliced copy of A: sptr[s] = first entry of slice s (ceil(n/64) + 1 entries).
void launch_csr_to_sell(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                        const long long *sptr, int *scol, double *sval);
void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p, const double *q,
                      PcgState *st, const double *part_pq, int t, double *part_rr,
                      const double *zold, double *part_rzo);
void launch_dot(hipStream_t s, int n, const double *a, const double *b, double *partial,
                const int *done);
// grad[k] = -lambda[row k] * u[col k] for the CSR entries k
void launch_grad_values(hipStream_t s, int n, const int *rp, const int *col, const double *lambda,
                        const double *u, double *grad);
void launch_residual(hipStream_t s, int n, const double *f, const double *Ax, double *r,
                     double *partial);
void launch_copy_scale(hipStream_t s, int n, const double *a, double *b, double alpha);
// GMRES (restarted, flexible right preconditioning) building blocks.  The
// basis columns are V + k * ldv.  out[k] = V_k . w for k < k1 (part holds
// k1 * reduce_blocks(n) partials); w -= V h with optional w.w partials;
// v = w / sqrt(*nrm2); x += Z y.
void launch_gs_dots(hipStream_t s, int n, const double *V, size_t ldv, int k1, const double *w,
                    double *part, double *out);
void launch_gs_update(hipStream_t s, int n, const double *V, size_t ldv, int k1, const double *h,
                      double *w, double *part);
void launch_gs_normalize(hipStream_t s, int n, const double *w, const double *nrm2, double *v);
void launch_basis_combine(hipStream_t s, int n, const double *Z, size_t ldz, int k, const double *y,
                          double *x);

void launch_abs_spmv_sq(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                        const double *x, double *partial);
void launch_fill(hipStream_t s, size_t n, double *a, double v);
void launch_fill_int(hipStream_t s, size_t n, int *a, int v);
void launch_sum_partials(hipStream_t s, const double *partial, int nb, double *out);
void launch_pcg_init(hipStream_t s, PcgState *st, const double *partial_rr, int nb_rr,
                     const double *partial_rz, int nb_rz, double rtol, int maxit);

// ----------------------------------------------------------------- local ---
// s = diag(hat A_i) for every local row; status[i] |= 1 if some s <= 0.
void launch_neumann_diag(hipStream_t s, const Plan &p, const double *val, double *sdiag,
                         int *status);
// Tile-profile storage: mode 0 -> A_i, mode 1 -> S^{-1/2} hat A_i S^{-1/2} + sigma I.
void launch_extract_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *val,
                          const double *sdiag, double *tiles, int mode, double sigma);
// In-place batched profile Cholesky; diagonal tiles then hold inv(L_II).
// status[i] |= bit on a non-positive pivot.
void launch_profile_cholesky(hipStream_t s, const Plan &p, double *tiles, int *status, int bit);
void launch_tiles_to_f32(hipStream_t s, const double *src, float *dst, size_t count);
// Envelope copy (row and column forms, type T) of the off-diagonal part of a
// factored tile pool.
template <typename T>
void launch_env_from_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *tiles,
                           T *erow, T *ecol);
// Dynamic LDS of the local apply for regions of up to max_npad padded rows
// and compute type of csize bytes.
size_t local_apply_lds_bytes(int max_npad, size_t csize);
// Per-sweep streams of an f32 factor: for every region, its 64-row blocks in
// sweep order (forward: ascending, envelope row form; backward: descending,
// column form), each block's envelope segments zero-padded to a multiple of
// 4 entries and followed by the block's packed inverse diagonal tile.  The
// arrays carry STREAM_TAIL extra entries (read, never used).
constexpr int STREAM_TAIL = 4 * WG;
void launch_stream_from_tiles(hipStream_t s, const Plan &p, int ntilerows, const double *tiles,
                              float *fst, float *bst);
size_t local_apply_stream_lds_bytes(int max_npad);
// Coarse restriction c = R0 r: c_i = Phi_i^T r_i for every region (TB basis
// type; the copy made by launch_basis_to_natural).
template <typename TB>
void launch_restrict(hipStream_t s, const Plan &p, const double *r, const TB *phi, double *cvec,
                     const int *done);
// The mixed-form local apply on the streams (same operation as
// launch_local_apply_t with float factors).
template <typename TB>
void launch_local_apply_stream(hipStream_t s, const Plan &p, int max_npad, const double *r,
                               const float *fst, const float *bst, const TB *phi, const double *t,
                               const double *tpart, int T0, double *xloc, const int *done,
                               hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Local apply: gather r, envelope forward/backward solve, store into xloc;
// with the coarse solution t (else nullptr) the prolongation Phi_i t_i is
// added to each region's output (phi: the copy made by
// launch_basis_to_natural).  With tpart (else nullptr) the coarse solution
// is instead summed from the per-tile products of W0^T (launch_trmv with
// y == nullptr; T0 tiles), as the reduction would sum them.  diag: the packed inverse diagonal tiles
// (DE entries per tile row), erow/ecol: the envelope.  T factor, C compute,
// TB basis type.  ev_start / ev_stop (optional, created with timing): bound
// to the dispatch itself (no extra packets in the stream).
template <typename T, typename C, typename TB>
void launch_local_apply_t(hipStream_t s, const Plan &p, int max_npad, const double *r,
                          const T *diag, const T *erow, const T *ecol, const TB *phi,
                          const double *t, const double *tpart, int T0, double *xloc,
                          const int *done, hipEvent_t ev_start = nullptr,
                          hipEvent_t ev_stop = nullptr);
void launch_selftest_mfma(hipStream_t s, const double *A, const double *B, double *D);
// The regions' dofs in ascending order and their local indices (Plan::asc,
// Plan::lop).
void launch_ascending_dofs(hipStream_t s, const Plan &p, int *asc, int *lop);
// Direct operand indices of the inverse map (see k_inverse_direct).
void launch_inverse_direct(hipStream_t s, int ne, const int *inv_sd, const int *inv_loc,
                           const Plan &p, int *ix);
// z = sum_i R_i^T (x_i + D_i psi_i t_i): with the coarse part, first adds the
// prolongation into the local outputs xloc (overwrites them without the local
// part), then sums every dof's copies; partial r.z per workgroup when r != 0.
template <typename TB>
void launch_scatter_sum_t(hipStream_t s, const Plan &p, int max_ni, int n, const int *inv_ptr,
                          const int *ix, double *xloc, const TB *phi, const double *t, double *z,
                          const double *r, double *partial, int do_local, int do_coarse,
                          const int *done);

// ------------------------------------------------------- several columns ---
// Up to EIGP right-hand sides per pass (k_multi.hip): gather into X (per
// region npad_i rows of EIGP doubles, local order), restriction of every
// column into c (columns ncp apart), prolongation + local solution into XN
// (ascending-global-index layout), scatter into z (columns n apart).
void launch_gather_multi(hipStream_t s, const Plan &p, int n, int nr, const double *r, double *X);
template <typename TB>
void launch_restrict_multi(hipStream_t s, const Plan &p, int nr, size_t ncp, const TB *phi,
                           const double *X, double *c);
template <typename TB>
void launch_prolong_multi(hipStream_t s, const Plan &p, int nr, size_t ncp, const TB *phi,
                          const double *t, const double *Y, double *XN);
void launch_scatter_multi(hipStream_t s, int n, int nr, const int *inv_ptr, const int *ix,
                          const double *XN, double *z);
// y_k = W0 x_k (transpose 0) or W0^T x_k (1) for k < nr, vectors ncp apart,
// reading W0's tiles once; part holds T0 * T0 * 64 * EIGP doubles.
template <typename T>
void launch_trmm(hipStream_t s, const T *Wt, int T0, const double *x, size_t ncp, int nr,
                 double *part, double *y, int transpose);
// CG on nr columns ld apart, one recurrence per column: Y = A X (entries
// read once for all columns); out[k] = A_k . B_k (part: 256 * nr doubles);
// x_k += alpha_k p_k, r_k -= alpha_k q_k with rr[k] = r_k . r_k; p_k = z_k +
// beta_k p_k.  alpha, beta, out and rr are device arrays of nr doubles.
void launch_spmm_sell(hipStream_t s, int n, const long long *sptr, const int *scol,
                      const double *sval, size_t ld, int nr, const double *X, double *Y);
void launch_col_dots(hipStream_t s, int n, size_t ld, int nr, const double *A, const double *B,
                     double *part, double *out);
void launch_col_update(hipStream_t s, int n, size_t ld, int nr, const double *alpha,
                       const double *P, const double *Q, double *X, double *R, double *part,
                       double *rr);
void launch_col_direction(hipStream_t s, int n, size_t ld, int nr, const double *beta,
                          const double *Z, double *P);
// Scalars of the per-column CG recurrences, kept on the device (nr <= EIGP).
struct ColCgState {
  double rz[EIGP], f2[EIGP], rr[EIGP];  // r.z, f.f and r.r (after the last update) per column
  int active[EIGP], its[EIGP];
  int breakdown, nact;  // bit k: column k broke down; columns still active
};
// alpha_k = (r.z)_k / (p.Ap)_k for active columns (0 otherwise); a column with
// p.Ap <= 0 or a non-finite ratio stops and sets its breakdown bit.
void launch_col_alpha(hipStream_t s, int nr, ColCgState *cs, const double *pq, double *alpha);
// After the update: an active column with r.r <= rtol2 f.f stops (a
// non-finite r.r stops it with breakdown); the others take beta_k =
// (r.z)'_k / (r.z)_k and keep (r.z)'.  Copies rr into the state, counts the
// active columns.
void launch_col_beta(hipStream_t s, int nr, ColCgState *cs, const double *rr, const double *rz,
                     double rtol2, double *beta);
// f32 factor of the mixed forms from its streams back into packed diagonal
// tiles + envelope (the layout of launch_env_solve_block)
void launch_streams_to_env(hipStream_t s, const Plan &p, int ntilerows, const float *fst,
                           const float *bst, float *dg, float *er, float *ec);

// mult[j] (regions containing dof j), inv_ptr (n + 1) and the per-dof lists
// (subdomain, ascending-index position) ordered by subdomain; work holds
// n + ceil(n / 1024) ints; *max_mult receives the largest multiplicity.
void launch_inverse_map(hipStream_t s, const Plan &p, int n, int *mult, int *inv_ptr,
                        int *inv_sd, int *inv_loc, int *work, int *max_mult);
// Local CSR entries (loc_col, loc_src) of every region from the plan's row
// pointers, dofs and ranks, and A's device CSR.  gscratch (2 * sum n_i ints)
// is used only when 2 * max_ni ints exceed LOCAL_CSR_LDS_MAX bytes of LDS.
constexpr size_t LOCAL_CSR_LDS_MAX = 128 * 1024;
size_t local_csr_lds_bytes(int max_ni);
void launch_local_csr(hipStream_t s, const Plan &p, int max_ni, const int *rowptr, const int *col,
                      int *loc_col, int *loc_src, int *gscratch);

// ---------------------------------------------------------------- eigen ---
void launch_eig_init(hipStream_t s, const Plan &p, const double *sdiag, double *X);
// dst[sd_ptr[i] * nev + c * n_i + nat[k]] = src[(sd_ptr[i] + k) * nev + c]: the
// basis in each region's ascending-global-index order, one column after the
// other (read by the single-vector apply's restriction and prolongation).
template <typename TB>
void launch_basis_to_natural(hipStream_t s, const Plan &p, const TB *src, TB *dst);
// Off-diagonal values of the scaled local operators B_i per local CSR entry.
void launch_eig_bval(hipStream_t s, const Plan &p, const double *val, const double *sdiag,
                     double *bval);
// Y = (L L^T)^{-1} X on row-major [rows][EIGP] padded blocks, L given as
// packed inverse diagonal tiles + envelope (as for the local apply).
template <typename T>
void launch_env_solve_block(hipStream_t s, const Plan &p, const T *diag, const T *erow,
                            const T *ecol, const double *X, double *Y, const int *skip);
// Rayleigh-Ritz step on the solve output Y, writing the Ritz vectors into X
// (distinct buffer), residuals, convergence flags and eigenvalues.
// BY: scratch like Y; GK: N*2*EIGP*EIGP doubles; CC: N*(EIGP*EIGP+EIGP).
void launch_eig_rr(hipStream_t s, const Plan &p, int max_ni, const double *val,
                   const double *sdiag, const double *bval, const double *Y, double *BY, double *X,
                   double *GK, double *CC, double tol, int *conv, double *lam,
                   bool test_next);
void launch_build_basis(hipStream_t s, const Plan &p, const double *sdiag, const double *X,
                        double *phi, int pou);
void launch_basis_convert(hipStream_t s, const double *phi, void *dst, size_t count, int bf16);
// phi[e] := phi[e] rounded to float32 (bf16 = 0) or bfloat16 (bf16 = 1), in place
void launch_basis_round(hipStream_t s, double *phi, size_t count, int bf16);

// ---------------------------------------------------------------- coarse ---
struct CoarsePlan {
  int N;
  int nev;
  const int *ext_ptr;       // [N+1] offsets of the extended regions
  const int *ext_rowptr;    // [sum |E_i| + 1] entries coupling each row to region i
  const int *ext_src;       //   global CSR value index
  const int *ext_loc;       //   local index in region i
  int npairs;
  const int *pair_i, *pair_j;
  const int *pair_ptr;      // [npairs+1]
  const int *pair_l;        // local index in region i
  const int *pair_e;        // index in the extended region of j
};
void launch_apply_A_to_basis(hipStream_t s, const Plan &p, const CoarsePlan &c,
                             const double *val, const double *phi, double *W);
void launch_pair_products(hipStream_t s, const Plan &p, const CoarsePlan &c, const double *phi,
                          const double *W, double *A0t, int T0);
void launch_symmetrize_tiles(hipStream_t s, double *A0t, int T0, int nc);
// Singular problems (null space = constants): u = R0 1 (u holds nc doubles),
// alpha = trace(A0) / u.u, A0 += alpha u u^T.
void launch_singular_regularize(hipStream_t s, const Plan &p, const double *phi, double *A0t,
                                int T0, int nc, double *u, double *alpha);
void launch_dense_potrf_diag(hipStream_t s, double *A0t, int T0, int k, double *dinv, int *status);
void launch_dense_trsm_panel(hipStream_t s, double *A0t, int T0, int k, const double *dinv);
// Trailing update of Cholesky step k split for lookahead: the next tile
// column (j = k + 1), in one launch with step k + 1's diagonal factor (the
// next diagonal tile is factored by the workgroup that updates it), and the
// rest (j >= k + 2).
void launch_dense_next_potrf(hipStream_t s, double *A0t, int T0, int k, double *dinv,
                             int *status);
void launch_dense_syrk_rest(hipStream_t s, double *A0t, int T0, int k);
void launch_dense_inv_row(hipStream_t s, double *Wt, int T0, int k, const double *dinv);
void launch_dense_inv_update(hipStream_t s, const double *Lt, double *Wt, int T0, int k);
void launch_tiles_identity(hipStream_t s, double *Wt, int T0);
void launch_dense_tiles_to_f32(hipStream_t s, const double *src, float *dst, int T0);
// y = W x (transpose 0) or W^T x (transpose 1) over the lower tiles of W;
// part: T0*T0*64 doubles of scratch holding the per-tile products.  With
// y == nullptr only the per-tile products are formed: entry O*64 + r of
// W^T x is then the sum over K = O .. T0-1 of part[(O*T0 + K)*64 + r], split
// into TRMV_RG consecutive pieces of K (piece g: K from O + len*g/TRMV_RG,
// len = T0 - O), each summed in order and the pieces added in order from 0.
constexpr int TRMV_RG = 16;
template <typename T>
void launch_trmv(hipStream_t s, const T *Wt, int T0, const double *x, double *part, double *y,
                 int transpose, const int *done);

// ------------------------------------ independent problems (k_batch.hip) ---
// Recurrence r = k * nseg + s (column k, problem s); row blocks never cross
// a problem boundary (rows of block b: [brow[b], brow[b+1]), problem bseg[b];
// problem s owns blocks [sblk[s], sblk[s+1])).
void launch_seg_dots(hipStream_t s, int nblk, int nseg, const long long *brow, const int *sblk,
                     size_t ld, int nr, const double *A, const double *B, double *part,
                     double *out);
void launch_seg_update(hipStream_t s, int nblk, int nseg, const long long *brow, const int *bseg,
                       const int *sblk, size_t ld, int nr, const double *alpha, const double *P,
                       const double *Q, double *X, double *R, double *part, double *rr);
void launch_seg_direction(hipStream_t s, int nblk, int nseg, const long long *brow,
                          const int *bseg, size_t ld, int nr, const double *beta, const double *Z,
                          double *P);
void launch_seg_alpha(hipStream_t s, int nrec, double *rz, double *f2, double *rr, int *active,
                      int *its, int *broken, int *flags, const double *pq, double *alpha);
void launch_seg_beta(hipStream_t s, int nrec, double *rz, double *f2, double *rr, int *active,
                     int *its, int *broken, int *flags, const double *rrn, const double *rzn,
                     double rtol2, double *beta);
void launch_abs_spmv_rows(hipStream_t s, int n, const int *rp, const int *col, const double *val,
                          const double *u, double *w);
void launch_sub_columns(hipStream_t s, size_t tot, const double *F, const double *Q, double *R);
void launch_check_blocks(hipStream_t s, int n, const int *rp, const int *col, int nseg,
                         const long long *sptr, int *flag);

}  // namespace amsp
