// Sparse coarse factorisation: host symbolic phase and device launchers.
//
// The coarse matrix A0 = R0 A R0^T (Section 3.1) couples two subdomains only
// when their supports touch, so it is block-sparse with the sparsity of the
// subdomain graph.  The paper factors it with a sparse direct solver
// (Section 5, solver set-up); this is the device counterpart: a multifrontal
// Cholesky factorisation over a nested-dissection order of the subdomains.
//
// Symbolic phase (host, integer work):
//   * nested dissection of the subdomain graph (recursive bisection by BFS
//     level sets from a pseudo-peripheral subdomain; a level set is a vertex
//     separator), down to leaves of at most one 64-row tile of coarse dofs;
//   * one supernode per separator or leaf; a front's rows are its own coarse
//     dofs (padded to whole 64-row tiles) followed by its update dofs, the
//     coarse dofs of the ancestor subdomains its subtree is coupled to (the
//     symbolic Cholesky structure at subdomain granularity);
//   * levels: a front's level is one more than its highest child's, so the
//     fronts of one level are independent and factor together.
// Numeric phase (device, one level after another): assemble A0's blocks and
// the children's Schur complements (extend-add) into each front, factor its
// own tile columns (right-looking tile Cholesky, matrix-core tile updates),
// and form X = [inv(L11); -L21 inv(L11)] (T x K tiles; the first K block
// columns of the inverse of [L11 0; L21 I]), the matrix both triangular
// solves read:
//   forward:  [y_s; v_s - w_s] = X c_s, i.e. y_s = inv(L11) c_s and
//             v_s = w_s - L21 y_s, passed to the parent (w_s: the children's
//             contributions to the update rows);
//   backward: x_s = X^T [y_s; x_upd] = inv(L11)^T (y_s - L21^T x_upd).
// Each level of a solve is one launch whose workgroups each own a row tile
// (forward) or a column tile (backward) of one front.
#pragma once
#include <string>
#include <vector>

#include "amsp_internal.h"

namespace amsp {

struct TreePlan {
  int nfront = 0, nlevel = 0;
  int max_T = 0, max_K = 0;         // largest front (tiles) and own part (tiles)
  std::vector<int> lvl_ptr;         // fronts of level h: [lvl_ptr[h], lvl_ptr[h+1])
  // per front (fronts numbered level by level)
  std::vector<int> K, T, kdof, udof;  // own tiles, front tiles, own dofs, update dofs
  std::vector<long long> fbase;     // packed lower tiles of the front: tile (I,J), J <= I,
                                    // at fbase + I(I+1)/2 + J
  std::vector<long long> xbase;     // X: T x K tiles, tile (I,J) at xbase + I*K + J
  std::vector<int> dbase;           // inverse diagonal tiles of L11: dbase + k
  std::vector<int> rbase;           // first row of the front in the row tables (64 T rows)
  std::vector<int> vbase;           // first entry of the front's update vector (udof entries)
  std::vector<int> parent;          // -1 for a root
  long long ftiles = 0, xtiles = 0;
  int dtiles = 0, nrows = 0, nvec = 0;
  // row tables (64 T_s rows per front): the coarse index (the library's
  // subdomain-major numbering) of each row, -1 for padding rows
  std::vector<int> row_coarse;
  // forward gather: for each front row, the children's update-vector entries
  // that add into it (indices into the concatenated update vectors)
  std::vector<int> gptr, gsrc;
  // extend-add: for each front, the parent front row of each of its update
  // rows (udof entries), at vbase
  std::vector<int> ea_row;
  // children of each level's fronts, by child slot: for level h and slot c,
  // the child fronts at [ch_ptr[h * max_slots + c], ch_ptr[h * max_slots + c + 1])
  int max_slots = 0;
  std::vector<int> ch_ptr, ch_front;
  // A0 assembly: one entry per coupled pair (i, j) whose block lands in the
  // lower triangle of a front (ND position of i >= that of j): the pair, its
  // transpose's pair, the front and the first front rows of i and j
  std::vector<int> as_pair, as_rev, as_front, as_ri, as_rj;
  // per level: largest number of row tiles, of own tiles, of update-block
  // tiles (packed lower) over its fronts, and fronts in the level
  std::vector<int> lvl_maxT, lvl_maxK, lvl_maxU;
  double flops = 0.0;               // factor + X: sum over fronts of the tile products (x 2*64^3)
};

// Builds the plan from the coupled pairs (both orders present, i == j
// included), the kept eigenvectors m_i and the coarse offsets.  Subdomains
// with m_i = 0 take no part.  Returns false (with msg) on inconsistent input.
bool build_tree_plan(int N, const std::vector<int> &mi, const std::vector<int> &coff,
                     const std::vector<int> &pair_i, const std::vector<int> &pair_j, TreePlan &tp,
                     std::string &msg);

// Device view of the plan (all arrays on the device).
struct TreeDev {
  int nfront;
  const int *K, *T, *kdof, *udof, *dbase, *rbase, *vbase, *parent;
  const long long *fbase, *xbase;
  const int *row_coarse, *gptr, *gsrc, *ea_row, *ch_front;
  const int *as_pair, *as_rev, *as_front, *as_ri, *as_rj;
  const int *pair_i, *pair_j;  // the coupled pairs (CoarsePlan)
};

// Numeric phase.
void launch_pair_blocks(hipStream_t s, const Plan &p, const CoarsePlan &c, const double *phi,
                        const double *W, double *pb);
void launch_tree_init(hipStream_t s, const TreeDev &t, int nfront, int maxT, double *F, double *X);
void launch_tree_assemble(hipStream_t s, const Plan &p, const TreeDev &t, int nas, const double *pb,
                          double *F);
void launch_tree_extend_add(hipStream_t s, const TreeDev &t, const int *children, int nchild,
                            int maxU, double *F);
// Factor step k of the fronts [f0, f1) (maxT: their largest front in tiles).
void launch_tree_factor_step(hipStream_t s, const TreeDev &t, int f0, int f1, int maxT, int k,
                             double *F, double *dinv, int *status);
void launch_tree_inverse_step(hipStream_t s, const TreeDev &t, int f0, int f1, int maxT, int k,
                              const double *F, const double *dinv, double *X);
void launch_tree_x_to_f32(hipStream_t s, const double *X, float *Xf, long long ntiles);
// Coarse solve x = A0^{-1} c (c, x: the library's coarse numbering, padded);
// y: own-row values (nc), v: update vectors (nvec).
template <typename TX>
void launch_tree_solve(hipStream_t s, const TreeDev &t, const std::vector<int> &lvl_ptr,
                       const std::vector<int> &lvl_maxT, const std::vector<int> &lvl_maxK,
                       int maxK, int maxT, const TX *X, const double *c, double *y, double *v,
                       double *x, const int *done);

}  // namespace amsp
