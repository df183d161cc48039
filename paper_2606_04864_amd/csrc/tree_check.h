// CPU emulation of the sparse coarse factorisation's kernels (k_tree.hip):
// the same index formulas, grid ranges and early exits, with every array
// access bounds-checked, on a random symmetric positive definite matrix with
// the block sparsity of the coupled pairs.  The solve is compared with a
// dense Cholesky solve.  Used by the host check program only.
#pragma once
#include <string>
#include <vector>

#include "amsp_tree.h"

namespace amsp {

// Returns the relative error of the emulated coarse solve (negative on a
// bounds or structure failure, with msg).
double tree_emulate(int N, int nev, const std::vector<int> &mi, const std::vector<int> &coff,
                    const std::vector<int> &pair_i, const std::vector<int> &pair_j,
                    unsigned seed, std::string &msg);

}  // namespace amsp
