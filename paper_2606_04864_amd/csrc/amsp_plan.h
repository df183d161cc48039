// Host index planner (integer work) shared by the library's setup.
#pragma once
#include <array>
#include <string>
#include <vector>

#include "../../include/amsp.h"
#include "amsp_consts.h"

namespace amsp {

struct HostPlan {
  int n = 0, N = 0, nev = 0, nc = 0;
  int max_ni = 0, max_npad = 0;
  long long ntiles = 0;
  std::vector<int> sd_ptr, sd_dofs, vp_ptr, trow_ptr, tfirst;
  std::vector<long long> toff;
  std::vector<int> loc_rowptr, loc_col, loc_src;
  std::vector<int> mult, mi, coff;
  std::vector<int> inv_ptr, inv_sd, inv_loc;
  std::vector<int> ext_ptr, ext_rowptr, ext_src, ext_loc;
  std::vector<int> pair_i, pair_j, pair_ptr, pair_l, pair_e;
};

int validate_inputs(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                    int32_t overlap, std::string &msg);
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
