"""C-ABI checks that need no GPU: exported symbols, host-side validation and
error codes, and the host index planner against the oracle's region sets."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from workloads import configs

import paper_2606_04864_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "amsp.h")).read()
    declared = set(re.findall(r"\b(amsp_[a-z_0-9]+)\s*\(", header))
    assert len(declared) >= 15
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in amsp.h but not exported"
    assert declared <= set(P.EXPORTED) | {"amsp_default_options"}


def test_default_options():
    o = P.default_options()
    assert o["overlap"] == 1 and o["precision"] == 0 and o["eig_maxit"] >= 40
    assert o["eig_shift"] > 0 and o["chunk"] >= 1


def _csr_parts(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64)


def _small():
    w = configs.channels(nx=8, nparts=4, overlap=1, nev=2)
    return w, w.A.to_scipy()


def test_error_codes_forced_from_host():
    w, A = _small()
    rp, ci, va = _csr_parts(A)
    part = w.part
    ok = P.setup_error_code(rp, ci, va, part, 4, 2)
    assert ok[0] == "AMSP_OK"
    # unsorted / out-of-range column index
    ci2 = ci.copy()
    ci2[1], ci2[2] = ci2[2], ci2[1]
    assert P.setup_error_code(rp, ci2, va, part, 4, 2)[0] == "AMSP_ERR_CSR"
    ci3 = ci.copy()
    ci3[3] = A.shape[0] + 5
    assert P.setup_error_code(rp, ci3, va, part, 4, 2)[0] == "AMSP_ERR_CSR"
    # missing diagonal
    B = A.tolil()
    B[0, 0] = 0
    B = sp.csr_matrix(B)
    B.eliminate_zeros()
    assert P.setup_error_code(*_csr_parts(B), part, 4, 2)[0] == "AMSP_ERR_CSR"
    # non-finite value
    va2 = va.copy()
    va2[0] = np.nan
    assert P.setup_error_code(rp, ci, va2, part, 4, 2)[0] == "AMSP_ERR_CSR"
    # asymmetric values: the lowest row with a mismatched upper entry is named
    C = A.tolil()
    C[0, 1] = C[0, 1] * 1.5
    assert P.setup_error_code(*_csr_parts(C), part, 4, 2)[0] == "AMSP_ERR_NONSYM"
    C = A.tolil()
    C[50, 51] = C[50, 51] * 1.5
    C[20, 21] = C[20, 21] * 1.5
    code, msg = P.setup_error_code(*_csr_parts(C), part, 4, 2)
    assert code == "AMSP_ERR_NONSYM" and msg.endswith("row 20"), msg
    # a mismatch below 1e-14 max|a| is accepted
    C = A.tolil()
    C[20, 21] = C[20, 21] + 1e-16 * abs(A).max()
    assert P.setup_error_code(*_csr_parts(sp.csr_matrix(C)), part, 4, 2)[0] == "AMSP_OK"
    # asymmetric pattern with as many lower as upper entries: (3, 17) and
    # (12, 5) without their mirrors
    D = A.tolil()
    D[3, 17] = -1e-3
    D[12, 5] = -1e-3
    code, msg = P.setup_error_code(*_csr_parts(sp.csr_matrix(D)), part, 4, 2)
    assert code == "AMSP_ERR_NONSYM" and msg.endswith("row 3"), msg
    # partition value out of range, empty part, bad nparts
    p2 = part.copy()
    p2[0] = 7
    assert P.setup_error_code(rp, ci, va, p2, 4, 2)[0] == "AMSP_ERR_PARTITION"
    p3 = part.copy()
    p3[p3 == 3] = 2
    assert P.setup_error_code(rp, ci, va, p3, 4, 2)[0] == "AMSP_ERR_PARTITION"
    assert P.setup_error_code(rp, ci, va, part, 0, 2)[0] == "AMSP_ERR_PARTITION"
    # nev out of range, overlap negative
    assert P.setup_error_code(rp, ci, va, part, 4, -1)[0] == "AMSP_ERR_ARG"
    assert P.setup_error_code(rp, ci, va, part, 4, 16)[0] == "AMSP_ERR_ARG"
    assert P.setup_error_code(rp, ci, va, part, 4, 2, overlap=-1)[0] == "AMSP_ERR_ARG"


@pytest.mark.parametrize("name,overlap", [("channels64", 0), ("channels64", 1), ("channels64", 3),
                                          ("gauss128", 2)])
def test_planner_regions_match_oracle(name, overlap):
    w = W.get(name)
    A = w.A.to_scipy()
    regs, nt, npairs = P.plan_regions(w.A.row_ptr, w.A.col_idx, w.A.val, w.part, w.nparts, w.nev,
                                      overlap=overlap)
    cores = O.cores(w.part, w.nparts)
    for r, c in zip(regs, cores):
        ref = O.grow(A, c, overlap)
        assert len(r) == len(ref) and len(set(r.tolist())) == len(r)
        assert np.array_equal(np.sort(r), ref)
    assert npairs >= w.nparts  # every subdomain couples at least with itself


def test_planner_orders_and_profiles():
    w = configs.gauss_inclusions(nx=128, nparts=16)
    args = (w.A.row_ptr, w.A.col_idx, w.A.val, w.part, w.nparts, w.nev)
    r_rcm, t_rcm, _ = P.plan_regions(*args, overlap=2)
    r_nat, t_nat, _ = P.plan_regions(*args, overlap=2, local_order="natural")
    r_den, t_den, _ = P.plan_regions(*args, overlap=2, dense_tiles=True)
    for a, b in zip(r_rcm, r_nat):
        assert np.array_equal(np.sort(a), b)  # natural order is ascending global index
    nts = [(len(r) + 63) // 64 for r in r_den]
    assert t_den == sum(k * (k + 1) // 2 for k in nts)
    assert t_rcm < t_den and t_rcm <= t_nat
    # the RCM order's tile profile covers every nonzero of the local matrices
    A = w.A.to_scipy()
    for r in r_rcm[:4]:
        Ai = A[r][:, r].tocoo()
        low = Ai.row >= Ai.col
        band = (Ai.row[low] // 64) - (Ai.col[low] // 64)
        assert band.max() <= (len(r) + 63) // 64


def test_planner_is_deterministic():
    w = W.get("gauss128")
    a = P.plan_regions(w.A.row_ptr, w.A.col_idx, w.A.val, w.part, w.nparts, w.nev, overlap=2)
    b = P.plan_regions(w.A.row_ptr, w.A.col_idx, w.A.val, w.part, w.nparts, w.nev, overlap=2)
    assert a[1:] == b[1:]
    assert all(np.array_equal(x, y) for x, y in zip(a[0], b[0]))


def test_planner_repeatable_across_problem_sizes():
    """The planner keeps its workers' scratch between calls (index maps sized
    for the largest problem seen); plans must not depend on what ran before:
    a large problem, a smaller one, then the large one again give the same
    regions in the same local (RCM) order, tile count and pair count."""
    big = W.get("gauss128")
    small = configs.channels(nx=24, nparts=9, overlap=1, nev=3)

    def plan(w):
        return P.plan_regions(w.A.row_ptr, w.A.col_idx, w.A.val, w.part, w.nparts, w.nev,
                              overlap=2)

    r1, nt1, np1 = plan(big)
    rs, nts, nps = plan(small)
    r2, nt2, np2 = plan(big)
    rs2, nts2, nps2 = plan(small)
    assert (nt1, np1) == (nt2, np2) and (nts, nps) == (nts2, nps2)
    assert all(np.array_equal(a, b) for a, b in zip(r1, r2))
    assert all(np.array_equal(a, b) for a, b in zip(rs, rs2))
