"""Generator and partitioner checks (host inputs shared by oracle and HIP path)."""
import numpy as np
import pytest

import workloads as W
from workloads import configs, darcy


def _check_mmatrix(A):
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0
    off = S.copy()
    off.setdiag(0)
    assert off.data.max() <= 0.0
    assert np.asarray(S.sum(axis=1)).min() >= -1e-12 * abs(S).max()
    assert (S.diagonal() > 0).all()
    # sorted columns
    for i in range(0, A.n, max(1, A.n // 50)):
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert (np.diff(c) > 0).all()


def test_channels64_shape_and_mmatrix():
    w = W.get("channels64")
    assert w.n == 4096 and w.A.nnz == 5 * 4096 - 4 * 64
    _check_mmatrix(w.A)
    assert set(np.unique(w.kappa)) == {1.0, 1e4}


def test_3d_tpfa_nnz_and_anisotropy():
    k = np.ones((6, 6, 6))
    A = darcy.tpfa_matrix(k, 0.1 * k)
    assert A.n == 216 and A.nnz == 7 * 216 - 6 * 36
    _check_mmatrix(A)
    S = A.to_scipy()
    # x coupling h^(d-2)*harm(1,1) = 1/6; z coupling a tenth of that
    assert np.isclose(S[0, 1], -1.0 / 6) and np.isclose(S[0, 36], -0.1 / 6)


def test_seeds_reproduce():
    a = configs.gauss_inclusions(nx=64, nparts=4)
    b = configs.gauss_inclusions(nx=64, nparts=4)
    assert np.array_equal(a.A.val, b.A.val) and np.array_equal(a.b, b.b)
    assert a.part_sha256() == b.part_sha256()


@pytest.mark.parametrize("nparts", [1, 3, 16, 37])
def test_partition_covers_balanced(nparts):
    w = configs.channels(nx=40, nparts=nparts)
    cnt = np.bincount(w.part, minlength=nparts)
    assert cnt.sum() == 1600 and (cnt > 0).all()
    assert cnt.max() - cnt.min() <= 2


def test_grf_statistics():
    rng = np.random.default_rng(0)
    f = darcy.gaussian_random_field((256, 256), 4.0, 0.05, rng)
    assert abs(f.var() - 4.0) < 1.5
    assert abs(f.mean()) < 1.5


def test_torch_assembly_equals_generator():
    """workloads.tpfa_torch (the differentiable forward model) gives the
    generator's CSR values in the same order, 2D and 3D."""
    torch = pytest.importorskip("torch")
    from workloads.tpfa_torch import TpfaAssembly
    rng = np.random.default_rng(3)
    for shape in [(9, 7), (5, 4, 3)]:
        th = 2.0 * rng.standard_normal(shape)
        M = darcy.tpfa_matrix(np.exp(th))
        v = TpfaAssembly(shape, M.row_ptr, M.col_idx).values(torch.tensor(th)).numpy()
        assert np.abs(v - M.val).max() <= 1e-15 * np.abs(M.val).max()


def test_adjoint_workload():
    w = configs.adjoint(nx=32, nparts=4)
    assert w.theta.shape == (32, 32) and np.allclose(np.exp(w.theta), w.kappa)
    A = w.A.to_scipy()
    # u_obs solves the perturbed problem, not this one
    r = np.linalg.norm(A @ w.u_obs - w.b) / np.linalg.norm(w.b)
    assert r > 1e-3
    assert abs(w.theta.var() - 4.0) < 2.0


def test_shifted_operator_breaks_cg_with_spd_local_factors():
    """The breakdown cases' premise: A - sigma I is indefinite, every
    overlapping region's Dirichlet matrix stays SPD (the oracle's local
    Cholesky factors exist), and the oracle's CG meets p.Ap <= 0 within a
    few steps on the right-hand sides those cases draw."""
    import scipy.sparse as sp

    import oracle as O
    from conftest import cg_breakdown_step, shifted_indefinite
    w, As, val, sigma = shifted_indefinite()
    assert np.linalg.eigvalsh(As.toarray())[0] < 0
    # the shifted values in the workload's CSR order are the shifted matrix
    S = sp.csr_matrix((val, w.A.col_idx, w.A.row_ptr), shape=As.shape)
    assert abs(S - As).max() == 0
    st = O.setup(As, w.part, w.nparts, 0, 1)
    R = np.random.default_rng(71).standard_normal((w.n, 3))
    for j in (1, 2):
        t, xt = cg_breakdown_step(As, R[:, j], st.apply)
        assert 2 <= t <= 10
