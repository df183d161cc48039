// Host index planner (integer work) shared by the library's setup.
#pragma once
#include <array>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/amsp.h"
#include "amsp_consts.h"

namespace amsp {

// Host blocks of 1 MiB and more are recycled through a process-wide cache
// (at most 4 GiB held), so repeated setups do not pay fresh page faults for
// their index arrays; smaller requests go to operator new.
void *plan_alloc(size_t bytes);
void plan_free(void *p, size_t bytes);
// fn(c) for c in [0, count) on the planner's worker threads (at most 16,
// dynamic schedule); returns when all have run.
void plan_parallel_for(int count, const std::function<void(int)> &fn);
// Joins the planner's worker threads and releases the free blocks of the
// cache (blocks still in use stay valid and return to the cache later).
// Also run by an exit handler.  Not to be called while a plan is being built.
void plan_release_caches();

// Allocator whose resize() leaves new elements uninitialised (large index
// arrays are first written by the threads that fill them), backed by the
// recycling cache above.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U> &) {}
  T *allocate(size_t n) { return static_cast<T *>(plan_alloc(n * sizeof(T))); }
  void deallocate(T *p, size_t n) { plan_free(p, n * sizeof(T)); }
  template <typename U>
  void construct(U *p) noexcept {
    ::new ((void *)p) U;
  }
  template <typename U, typename... Args>
  void construct(U *p, Args &&...args) {
    ::new ((void *)p) U(std::forward<Args>(args)...);
  }
};
using ivec = std::vector<int, NoInitAlloc<int>>;

struct HostPlan {
  // Set by the caller before planning: whether A may store off-diagonal
  // zeros.  The graph of A leaves such entries out, so the planner reads the
  // value of every entry it visits; when validation counted none, it reads
  // only the column indices.
  bool offdiag_zeros = true;
  int n = 0, N = 0, nev = 0, nc = 0;
  int max_ni = 0, max_npad = 0;
  long long ntiles = 0;  // all profile tiles (off-diagonal + one diagonal per tile row)
  long long noff = 0;    // off-diagonal tiles
  std::vector<int> sd_ptr, vp_ptr, trow_ptr, tfirst;
  ivec sd_dofs;
  ivec nat;  // [sum n_i] rank of each local dof among its region's dofs by global index
  std::vector<long long> toff;  // first off-diagonal tile of each tile row
  // envelope storage of the factor below the diagonal tiles: per region,
  // npad_i + 1 segment starts of the row form (eptr) and of the column form
  // (uptr), relative to the region's base ebase[i]; nenv entries in all
  ivec eptr, uptr;
  std::vector<long long> ebase;
  long long nenv = 0;
  // local CSR of every region (rows in local order, columns ascending): the
  // row pointers here; the nloc column indices and source entries are built on
  // the device (launch_local_csr)
  ivec loc_rowptr;
  long long nloc = 0;
  std::vector<int> mi, coff;
  std::vector<int> ext_ptr;
  ivec ext_rowptr, ext_src, ext_loc;
  std::vector<int> pair_i, pair_j, pair_ptr;
  ivec pair_l, pair_e;
};

// On success *offdiag_zeros (when given) receives the number of stored
// off-diagonal entries whose value is zero (-1 on failure).
int validate_inputs(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                    int32_t overlap, std::string &msg, int64_t *offdiag_zeros = nullptr);
// Regions, local orders, local CSR and tile profiles (everything the local
// factorisations and eigensolves need).
int build_plan_local(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                     const amsp_options &opt, HostPlan &P, std::string &msg);
// Multiplicities, inverse map, extended regions and coupled pairs (needed by
// the basis, A0 and the apply); reads what build_plan_local produced.
int build_plan_coupling(const amsp_csr *A, const amsp_options &opt, HostPlan &P, std::string &msg);
// Both phases in order.
int build_plan(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
               const amsp_options &opt, HostPlan &P, std::string &msg);

}  // namespace amsp
