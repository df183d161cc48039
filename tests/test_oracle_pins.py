"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses a hand-derived
worked example, a closed form, a brute-force computation on a tiny input, an
identity stated in the paper, or an independent library routine.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from workloads import configs


def _small(nx=16, nparts=4, overlap=1, nev=2, contrast=1e4, nchan=3):
    w = configs.channels(nx=nx, nparts=nparts, overlap=overlap, nev=nev, contrast=contrast,
                         nchan=nchan)
    return w, w.A.to_scipy()


# ---------------------------------------------------------------- golden ---
@pytest.mark.parametrize("case", ["overlap0", "overlap1"])
def test_worked_example_1d(golden, case):
    g = golden("worked_1d_4cell.txt")
    A = sp.csr_matrix(g["A"])
    part = g["part"].astype(np.int32)
    overlap = 0 if case == "overlap0" else 1
    st = O.setup(A, part, 2, 1, overlap=overlap)
    for r, ref in zip(st.regions, g[f"{case}.regions"]):
        np.testing.assert_array_equal(r, ref.astype(int))
    Ai = O.local_matrix(A, st.regions[0])
    Ah = O.neumann_matrix(Ai)
    np.testing.assert_allclose(Ah, g[f"{case}.neumann0"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(O.weighting(Ah), g[f"{case}.S0"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(st.lam[0], g[f"{case}.lambda0"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(st.psi[0][:, 0], g[f"{case}.psi0"], rtol=1e-13)
    if case == "overlap1":
        np.testing.assert_array_equal(st.mult, g["overlap1.mult"].astype(int))
        np.testing.assert_allclose(st.R0T.toarray(), g["overlap1.R0T"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(st.A0, g[f"{case}.A0"], rtol=1e-13)
    np.testing.assert_allclose(st.apply(g["f"]), g[f"{case}.Minv_f"], rtol=1e-13)
    res = O.pcg(A, g["f"], st.apply, rtol=1e-14, maxit=10)
    assert res.iterations <= 4
    np.testing.assert_allclose(res.x, g["u"], rtol=1e-12)


# ------------------------------------------------- Neumann matrix, S_i -----
def test_neumann_rowsums_and_edge_sum_identity():
    """Row sums of hat A_i vanish (Section 3.2) and x^T hat A_i x equals the
    edge sum 1/2 sum_{j!=k} (-A_jk)(x_j - x_k)^2 (proof of Lemma 2)."""
    w, A = _small(nx=20, nparts=4, overlap=2)
    rng = np.random.default_rng(0)
    st_regions = [O.grow(A, c, 2) for c in O.cores(w.part, w.nparts)]
    for dofs in st_regions:
        Ai = O.local_matrix(A, dofs)
        Ah = O.neumann_matrix(Ai)
        assert np.abs(Ah.sum(axis=1)).max() <= 1e-13 * np.abs(Ah).max()
        s = O.weighting(Ah)
        assert (s > 0).all()
        x = rng.standard_normal(len(dofs))
        # brute force edge loop, written from the definition
        e = 0.0
        for j in range(len(dofs)):
            for k in range(len(dofs)):
                if j != k and Ai[j, k] != 0.0:
                    e += 0.5 * (-Ai[j, k]) * (x[j] - x[k]) ** 2
        assert abs(x @ Ah @ x - e) <= 1e-12 * abs(e)


# ------------------------------------------------------------ eigenpairs ---
def test_hep_equals_ghep_bruteforce():
    """The standard form S^{-1/2} hat A S^{-1/2} (Section 5) has the same
    spectrum as the generalized pencil (hat A, S) solved by a full dense GHEP."""
    w, A = _small(nx=16, nparts=4, overlap=1, nev=5)
    for c in O.cores(w.part, w.nparts):
        dofs = O.grow(A, c, 1)
        Ah = O.neumann_matrix(O.local_matrix(A, dofs))
        s = O.weighting(Ah)
        lam, psi = O.local_eigenpairs(Ah, s, 5, dofs)
        full = sla.eigh(Ah, np.diag(s), eigvals_only=True)
        np.testing.assert_allclose(lam, full[:6], rtol=0, atol=1e-12)
        # psi solves the generalized problem and is S-orthonormal
        np.testing.assert_allclose(Ah @ psi, (s[:, None] * psi) * lam[None, :5], atol=1e-10)
        np.testing.assert_allclose(psi.T @ (s[:, None] * psi), np.eye(5), atol=1e-12)


def test_first_eigenpair_is_constant():
    """Row sums of hat A vanish, so lambda_1 = 0 with psi_1 constant on a
    connected region."""
    w, A = _small(nx=16, nparts=4, overlap=1)
    for c in O.cores(w.part, w.nparts):
        dofs = O.grow(A, c, 1)
        Ah = O.neumann_matrix(O.local_matrix(A, dofs))
        s = O.weighting(Ah)
        lam, psi = O.local_eigenpairs(Ah, s, 2, dofs)
        assert abs(lam[0]) < 1e-12
        v = psi[:, 0]
        np.testing.assert_allclose(v, v.mean(), rtol=1e-10)
        np.testing.assert_allclose(v @ (s * v), 1.0, rtol=1e-12)


@pytest.mark.parametrize("n", [5, 12, 33])
def test_path_graph_closed_form(n):
    """Uniform chain: the pencil (Laplacian, degree) has lambda_k =
    1 - cos(pi k/(n-1)) and psi_k(j) proportional to cos(pi k j/(n-1))."""
    w = 3.7
    L = np.zeros((n, n))
    for j in range(n - 1):
        L[j, j + 1] = L[j + 1, j] = -w
    Ah = O.neumann_matrix(L)
    s = O.weighting(Ah)
    m = n - 1
    lam, psi = O.local_eigenpairs(Ah, s, m)
    k = np.arange(n)
    np.testing.assert_allclose(lam, 1 - np.cos(np.pi * k / (n - 1)), atol=1e-13)
    j = np.arange(n)
    for kk in range(1, min(m, 6)):
        ref = np.cos(np.pi * kk * j / (n - 1))
        ref = ref / np.sqrt(ref @ (s * ref))
        if ref[np.argmax(np.abs(ref))] < 0:
            ref = -ref
        assert min(np.abs(psi[:, kk] - ref).max(), np.abs(psi[:, kk] + ref).max()) < 1e-10


def test_weighted_three_node_path_spectrum():
    """Any weighted 3-node path: the normalised pencil spectrum is {0, 1, 2}
    (bipartite graph; hand derivation)."""
    for a, b in [(2.0, 5.0), (1e-6, 1e6), (3.0, 3.0)]:
        L = np.array([[0, -a, 0], [-a, 0, -b], [0, -b, 0]], dtype=float)
        Ah = O.neumann_matrix(L)
        lam, _ = O.local_eigenpairs(Ah, O.weighting(Ah), 2)
        np.testing.assert_allclose(lam, [0, 1, 2], atol=1e-12 * max(1, b / a))


# ------------------------------------------------------------ theory -------
def _nonoverlap_setup(nev, contrast=1e4):
    w, A = _small(nx=14, nparts=4, overlap=0, nev=nev, contrast=contrast)
    st = O.setup(A, w.part, w.nparts, nev, overlap=0, pou="none")
    return w, A, st


def test_lemma1_s_norm_additivity():
    w, A, st = _nonoverlap_setup(2)
    rng = np.random.default_rng(1)
    n = A.shape[0]
    Sglob = np.zeros(n)
    total = 0.0
    v = np.zeros(n)
    for dofs in st.regions:
        s = O.weighting(O.neumann_matrix(O.local_matrix(A, dofs)))
        Sglob[dofs] = s
        x = rng.standard_normal(len(dofs))
        total += x @ (s * x)
        v[dofs] += x
    assert abs(v @ (Sglob * v) - total) <= 1e-13 * total


def test_lemma2_energy_splitting():
    w, A, st = _nonoverlap_setup(2)
    rng = np.random.default_rng(2)
    for _ in range(5):
        x = rng.standard_normal(A.shape[0])
        lhs = sum(x[d] @ O.neumann_matrix(O.local_matrix(A, d)) @ x[d] for d in st.regions)
        assert lhs <= x @ (A @ x) * (1 + 1e-13)


@pytest.mark.parametrize("nev", [1, 3])
def test_theorem2_approximation_constant(nev):
    """K = max_x min_{x_c in coarse space} ||x - x_c||_S^2 / ||x||_A^2 <= 1/mu_c
    with mu_c = min_i lambda_{m_i+1}, by a dense generalized eigenproblem."""
    w, A, st = _nonoverlap_setup(nev)
    n = A.shape[0]
    Sg = np.zeros(n)
    for dofs in st.regions:
        Sg[dofs] = O.weighting(O.neumann_matrix(O.local_matrix(A, dofs)))
    P = st.R0T.toarray()  # no PoU scaling: Boolean zero extension
    S = np.diag(Sg)
    # S-orthogonal projector onto the coarse space, error operator I - Pi
    Pi = P @ np.linalg.solve(P.T @ S @ P, P.T @ S)
    E = np.eye(n) - Pi
    K = sla.eigh(E.T @ S @ E, A.toarray(), eigvals_only=True)[-1]
    mu_c = min(l[nev] for l in st.lam)
    assert K <= (1.0 / mu_c) * (1 + 1e-9)


# ------------------------------------------------------- coarse operator ---
def test_coarse_operator_galerkin_identities():
    w, A = _small(nx=16, nparts=4, overlap=1, nev=3)
    st = O.setup(A, w.part, w.nparts, 3, overlap=1)
    Ad = A.toarray()
    R0T = st.R0T.toarray()
    C = R0T @ np.linalg.solve(st.A0, R0T.T)
    np.testing.assert_allclose(C @ Ad @ C, C, atol=1e-12 * np.abs(C).max())
    np.testing.assert_allclose(R0T.T @ (np.eye(A.shape[0]) - Ad @ C), 0,
                               atol=1e-12 * np.abs(R0T).max())


def test_full_coarse_space_is_exact_inverse():
    """overlap 0 and nev = n_i everywhere: R0^T is square and invertible, so
    R0^T A0^{-1} R0 = A^{-1}."""
    w, A = _small(nx=8, nparts=4, overlap=0)
    ni = np.bincount(w.part).max()
    st = O.setup(A, w.part, w.nparts, int(ni), overlap=0, pou="none")
    assert st.nc == A.shape[0]
    rng = np.random.default_rng(3)
    r = rng.standard_normal(A.shape[0])
    np.testing.assert_allclose(O.coarse_part(st, r), spla.spsolve(A.tocsc(), r), rtol=1e-10)


# ------------------------------------------------------- preconditioner ---
def test_preconditioner_is_spd():
    w, A = _small(nx=16, nparts=4, overlap=1, nev=2)
    st = O.setup(A, w.part, w.nparts, 2, overlap=1)
    n = A.shape[0]
    M = np.column_stack([st.apply(e) for e in np.eye(n)])
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_condition_number_dense_vs_lanczos():
    w, A = _small(nx=16, nparts=4, overlap=1, nev=2)
    st = O.setup(A, w.part, w.nparts, 2, overlap=1)
    n = A.shape[0]
    M = np.column_stack([st.apply(e) for e in np.eye(n)])
    ev = np.sort(np.linalg.eigvals(M @ A.toarray()).real)
    kappa = ev[-1] / ev[0]
    res = O.pcg(A, np.random.default_rng(4).standard_normal(n), st.apply, rtol=1e-14, maxit=n)
    est = O.lanczos_condition(res.alphas, res.betas)
    assert abs(est - kappa) <= 1e-3 * kappa


# ------------------------------------------------------------------ PCG ----
def test_pcg_identity_matches_scipy_cg():
    w, A = _small(nx=12, nparts=4)
    f = np.random.default_rng(5).standard_normal(A.shape[0])
    ours = O.pcg(A, f, lambda r: r.copy(), rtol=1e-30, maxit=15)
    iterates = []
    spla.cg(A, f, x0=np.zeros_like(f), rtol=1e-30, maxiter=15, callback=lambda x: iterates.append(x.copy()))
    assert len(iterates) >= 15
    np.testing.assert_allclose(ours.x, iterates[14], rtol=1e-9, atol=1e-12 * np.abs(iterates[14]).max())


def test_pcg_solution_matches_direct_solve():
    w = W.get("channels64")
    A = w.A.to_scipy()
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
    res = O.pcg(A, w.b, st.apply, rtol=1e-8)
    assert res.converged and res.relres_true <= 1e-8 * 1.01
    u = spla.spsolve(A.tocsc(), w.b)
    assert np.linalg.norm(res.x - u) / np.linalg.norm(u) < 1e-5
    assert res.iterations <= A.shape[0]


def test_contrast_flatness():
    """Iteration counts stay flat as the channel contrast grows (the trend of
    the paper's contrast tables), while one-level Schwarz (nev = 0) degrades."""
    its, its0 = [], []
    for c in [0, 2, 4, 6]:
        w = configs.channels(contrast=10.0 ** c)
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, 4, 1)
        its.append(O.pcg(A, w.b, st.apply, 1e-8).iterations)
        st0 = O.setup(A, w.part, w.nparts, 0, 1)
        its0.append(O.pcg(A, w.b, st0.apply, 1e-8).iterations)
    assert max(its) <= 1.5 * its[0], its
    assert its0[-1] > its[-1], (its0, its)


# -------------------------------------------- planted-mistake detection ----
def test_planted_mistakes_are_caught(monkeypatch):
    """Each plausible slip in the oracle breaks one of the pins above."""
    g = __import__("conftest").load_golden("worked_1d_4cell.txt")
    A = sp.csr_matrix(g["A"])
    part = g["part"].astype(np.int32)

    def minv_f(**patch):
        for k, v in patch.items():
            monkeypatch.setattr(O.amsp_oracle, k, v)
        try:
            return O.setup(A, part, 2, 1, overlap=1).apply(g["f"])
        except O.OracleError:
            return None  # the slip is rejected outright
        finally:
            monkeypatch.undo()

    ref = g["overlap1.Minv_f"]
    np.testing.assert_allclose(minv_f(), ref, rtol=1e-13)

    real_neu = O.amsp_oracle.neumann_matrix
    real_pro = O.amsp_oracle.prolongation
    # wrong sign of the Neumann diagonal (diag = +sum of off-diagonals)
    def flipped(Ai):
        M = real_neu(Ai)
        np.fill_diagonal(M, -np.diag(M))
        return M
    bad1 = minv_f(neumann_matrix=flipped)
    # Dirichlet diagonal kept instead of the Neumann one
    bad2 = minv_f(neumann_matrix=lambda Ai: Ai.copy())
    # partition of unity dropped
    bad3 = minv_f(prolongation=lambda n, reg, psis, mult, pou="mult": real_pro(n, reg, psis, mult, "none"))
    # eigenvectors not scaled back by S^{-1/2}
    real_eig = O.amsp_oracle.local_eigenpairs
    def unscaled(Ah, s, m, gdofs=None):
        lam, psi = real_eig(Ah, s, m, gdofs)
        return lam, psi * np.sqrt(s)[:, None]
    bad4 = minv_f(local_eigenpairs=unscaled)
    for bad in (bad1, bad2, bad3, bad4):
        assert bad is None or np.abs(bad - ref).max() > 1e-3


# ---------------------------------------------------------------- adjoint ---
def _loss(A, f, uobs):
    u = spla.spsolve(sp.csc_matrix(A), f)
    return 0.5 * float(np.sum((u - uobs) ** 2))


def test_adjoint_diagonal_closed_form():
    # A = diag(d): u = f/d and dJ/dd_i = -(u_i - uobs_i) u_i / d_i exactly
    rng = np.random.default_rng(11)
    d = rng.uniform(1.0, 3.0, 9)
    f, uobs = rng.standard_normal(9), rng.standard_normal(9)
    A = sp.diags(d).tocsr()
    u, lam, g = O.adjoint_gradients(A, f, f / d - uobs)
    np.testing.assert_allclose(u, f / d, rtol=1e-15)
    np.testing.assert_allclose(g, -(f / d - uobs) * (f / d) / d, rtol=1e-13)
    np.testing.assert_allclose(lam, (f / d - uobs) / d, rtol=1e-13)


def test_adjoint_matches_central_differences():
    # single stored entries (the perturbed matrix is unsymmetric, so a
    # transposed index lam_j u_i would fail) and entries of f, on a
    # high-contrast two-point-flux matrix; central differences with a step of
    # 1e-4 of the entry (truncation ~1e-8 relative), tolerance relative to the
    # entry plus a floor from the largest gradient (solve rounding)
    w, A = _small(nx=12, nparts=4, overlap=1, nev=2)
    A = sp.csr_matrix(A)
    A.sort_indices()
    rng = np.random.default_rng(12)
    f = rng.standard_normal(A.shape[0])
    uobs = rng.standard_normal(A.shape[0])
    u = spla.spsolve(A.tocsc(), f)
    _, lam, g = O.adjoint_gradients(A, f, u - uobs)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    off = np.nonzero(rows != A.indices)[0]
    dia = np.nonzero(rows == A.indices)[0]
    # the largest off-diagonal gradients, where a wrong index shows most
    big = off[np.argsort(-np.abs(g[off]))[:8]]
    picks = list(big) + list(rng.choice(off, 8, replace=False)) + list(rng.choice(dia, 6, replace=False))
    gmax = np.abs(g).max()
    for k in picks:
        h = 1e-4 * abs(A.data[k])
        Ap, Am = A.copy(), A.copy()
        Ap.data[k] += h
        Am.data[k] -= h
        fd = (_loss(Ap, f, uobs) - _loss(Am, f, uobs)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * abs(g[k]) + 1e-9 * gmax, (k, fd, g[k])
    # a transposed gradient would differ from the true one on these entries
    cols = A.indices
    wrong = -lam[cols] * u[rows]
    assert np.abs(wrong[big] - g[big]).max() > 1e-3 * gmax
    # dJ/df = lam
    lmax = np.abs(lam).max()
    for i in rng.choice(A.shape[0], 6, replace=False):
        e = np.zeros(A.shape[0])
        e[i] = 1.0
        h = 1e-4 * max(abs(f[i]), 1.0)
        fd = (_loss(A, f + h * e, uobs) - _loss(A, f - h * e, uobs)) / (2 * h)
        assert abs(fd - lam[i]) <= 1e-5 * abs(lam[i]) + 1e-9 * lmax


# ---------------------------------------------------------------- GMRES ----
def _nonsym(n=40, seed=11):
    """A small well-conditioned nonsymmetric matrix (GMRES does not need symmetry)."""
    rng = np.random.default_rng(seed)
    return sp.csr_matrix(np.eye(n) * 4.0 + rng.standard_normal((n, n)) / np.sqrt(n))


def test_gmres_identity_reaches_direct_solution():
    """Unrestarted, unpreconditioned GMRES solves an n x n system in at most n
    steps (the Krylov space is then all of R^n)."""
    for A in (_nonsym(), _small(nx=6, nparts=2)[1]):
        n = A.shape[0]
        f = np.random.default_rng(12).standard_normal(n)
        res = O.gmres(A, f, lambda v: v.copy(), restart=n, rtol=1e-10, maxit=n)
        assert res.converged and res.iterations <= n
        u = np.linalg.solve(A.toarray(), f)
        np.testing.assert_allclose(res.x, u, rtol=0, atol=1e-7 * np.abs(u).max())


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_gmres_iterate_is_the_krylov_least_squares_minimiser(k):
    """After k steps, x_k minimises ||f - A x|| over x in M^{-1} K_k(A M^{-1}, f):
    brute force with the explicit Krylov matrix, Householder QR and lstsq."""
    w, A = _small(nx=12, nparts=4, nev=2)
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
    f = np.random.default_rng(13).standard_normal(A.shape[0])
    res = O.gmres(A, f, st.apply, restart=50, rtol=0.0, maxit=k)
    assert res.iterations == k
    K = np.empty((A.shape[0], k))
    v = f.copy()
    for j in range(k):
        K[:, j] = v
        v = A @ st.apply(v)
    Q, _ = np.linalg.qr(K)
    S = np.column_stack([st.apply(Q[:, j]) for j in range(k)])
    y, *_ = np.linalg.lstsq(A @ S, f, rcond=None)
    xs = S @ y
    np.testing.assert_allclose(res.x, xs, rtol=0, atol=1e-9 * np.abs(xs).max())
    rel = np.linalg.norm(f - A @ xs) / np.linalg.norm(f)
    assert abs(res.relres_history[-1] - rel) <= 1e-9 * rel + 1e-15


def test_gmres_residual_never_above_pcg():
    """With the same SPD preconditioner and x0 = 0, PCG's k-th iterate lies in
    the space GMRES minimises over, so GMRES's residual is never larger."""
    w = W.get("channels64")
    A = w.A.to_scipy()
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
    cg = O.pcg(A, w.b, st.apply, rtol=1e-10)
    gm = O.gmres(A, w.b, st.apply, restart=400, rtol=1e-10, maxit=cg.iterations)
    k = min(len(cg.relres_history), len(gm.relres_history))
    h_cg = np.array(cg.relres_history[:k])
    h_gm = np.array(gm.relres_history[:k])
    assert np.all(h_gm <= h_cg * (1 + 1e-8) + 1e-14), np.max(h_gm / h_cg)
    assert gm.iterations <= cg.iterations


def test_gmres_restarted_history_and_true_residual():
    """Restarted GMRES: the residual never grows (each cycle starts from the
    current iterate), the estimate equals the true residual at every restart,
    and the result meets the tolerance."""
    w = W.get("channels64")
    A = w.A.to_scipy()
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
    res = O.gmres(A, w.b, st.apply, restart=10, rtol=1e-6)
    h = np.array(res.relres_history)
    assert res.converged and res.restarts >= 1
    assert np.all(np.diff(h) <= 1e-12), np.diff(h).max()
    assert res.relres_true <= 1e-6 and abs(res.relres_true - h[-1]) <= 1e-8 * h[-1]
    u = spla.spsolve(A.tocsc(), w.b)
    assert np.linalg.norm(A @ res.x - w.b) <= 1e-6 * np.linalg.norm(w.b)
    assert np.linalg.norm(res.x - u) / np.linalg.norm(u) < 1e-3


# ------------------------------------------------ Neumann-singular problem ----
def _neumann_setup():
    w = W.get("neumann64")
    A = w.A.to_scipy()
    return w, A, O.setup(A, w.part, w.nparts, w.nev, w.overlap, singular=True)


def test_neumann_matrix_null_space():
    """Without Dirichlet faces every row sums to zero (the constant vector is
    in the null space) and the source is consistent."""
    w, A, _ = _neumann_setup()
    assert np.abs(A @ np.ones(w.n)).max() <= 1e-10 * np.abs(A.diagonal()).max()
    assert abs(w.b.sum()) <= 1e-12 * np.abs(w.b).sum()


def test_neumann_coarse_null_space_is_the_constant():
    """A0 = R0 A R0^T is singular exactly along the c with R0^T c = 1: every
    region's first mode is constant and the partition of unity sums to one."""
    w, A, st = _neumann_setup()
    ev, Q = np.linalg.eigh(st.A0)
    assert ev[0] <= 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1], ev[:3]
    v = st.R0T @ Q[:, 0]
    np.testing.assert_allclose(v, v.mean(), rtol=0, atol=1e-8 * np.abs(v).max())


def test_pseudo_inverse_penrose_conditions():
    """The four Penrose conditions, and agreement with the library's pinv."""
    _, _, st = _neumann_setup()
    M, X = st.A0, st.A0_pinv
    s = np.abs(M).max()
    assert np.abs(M @ X @ M - M).max() <= 1e-9 * s
    assert np.abs(X @ M @ X - X).max() <= 1e-9 * np.abs(X).max()
    assert np.abs(M @ X - (M @ X).T).max() <= 1e-9
    assert np.abs(X @ M - (X @ M).T).max() <= 1e-9
    ref = np.linalg.pinv(M, rcond=1e-10, hermitian=True)
    assert np.abs(X - ref).max() <= 1e-8 * np.abs(ref).max()


def test_neumann_preconditioner_spd_on_the_range():
    """On vectors orthogonal to the null space the preconditioner with the
    pseudo-inverse is symmetric and positive."""
    w, A, st = _neumann_setup()
    rng = np.random.default_rng(21)
    for _ in range(3):
        x, y = rng.standard_normal(w.n), rng.standard_normal(w.n)
        x -= x.mean()
        y -= y.mean()
        mx, my = st.apply(x), st.apply(y)
        assert abs(x @ my - y @ mx) <= 1e-10 * np.linalg.norm(x) * np.linalg.norm(my)
        assert x @ mx > 0


def test_neumann_pcg_matches_grounded_direct_solve():
    """PCG on the consistent singular system reaches rtol; modulo the null
    space its solution is the direct solution with one dof grounded."""
    w, A, st = _neumann_setup()
    res = O.pcg(A, w.b, st.apply, rtol=1e-10)
    assert res.converged and res.relres_true <= 1e-9
    Ag = A[1:, 1:].tocsc()
    ug = np.concatenate([[0.0], spla.spsolve(Ag, w.b[1:])])
    a, b = res.x - res.x.mean(), ug - ug.mean()
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-6


# ------------------------------------------- multiplicative two-grid cycle ----
def _dense_ops(st, n):
    I = np.eye(n)
    S = np.column_stack([O.local_part(st, I[:, j]) for j in range(n)])
    C = np.column_stack([O.coarse_part(st, I[:, j]) for j in range(n)])
    M = np.column_stack([st.apply(I[:, j]) for j in range(n)])
    return S, C, M


@pytest.mark.parametrize("omega", [None, 0.5])
def test_two_grid_cycle_is_the_xz_identity(omega):
    """The cycle's error propagation E = I - M^{-1} A has the energy norm the
    Xu-Zikatanov identity gives (the identity Section 4 builds on):
    ||E||_A = 1 - 1/K, K = max_v min_{v_c} ||v - v_c||^2 / ||v||_A^2 in the
    norm of the inverse symmetrised smoother 2R - R A R, R = omega S.  A
    dropped smoothing step, a wrong sign or a missing coarse term breaks it."""
    w, A = _small(nx=12, nparts=4, overlap=1, nev=2, contrast=1e4, nchan=3)
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap, cycle="multiplicative", omega=omega)
    n = A.shape[0]
    Ad = A.toarray()
    S, C, M = _dense_ops(st, n)
    E = np.eye(n) - M @ Ad
    Ah = sla.sqrtm(Ad).real
    normE = np.linalg.norm(Ah @ E @ np.linalg.inv(Ah), 2)
    R = st.omega * S
    Rt = 2 * R - R @ Ad @ R
    Rti = np.linalg.inv(0.5 * (Rt + Rt.T))
    P = st.R0T.toarray()
    Q = P @ np.linalg.solve(P.T @ Rti @ P, P.T @ Rti)
    M1 = (np.eye(n) - Q).T @ Rti @ (np.eye(n) - Q)
    K = sla.eigh(0.5 * (M1 + M1.T), Ad, eigvals_only=True).max()
    assert abs(normE - (1 - 1 / K)) <= 1e-9, (normE, 1 - 1 / K)
    assert normE < 1


def test_two_grid_cycle_is_spd_and_beats_additive():
    """With omega = 1 / max multiplicity the cycle is a symmetric positive
    definite preconditioner; on the correctness workload it needs fewer CG
    iterations than the additive form."""
    w, A = _small(nx=12, nparts=4, overlap=1, nev=2, contrast=1e4, nchan=3)
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap, cycle="multiplicative")
    _, _, M = _dense_ops(st, A.shape[0])
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    wb = W.get("channels64")
    Ab = wb.A.to_scipy()
    add = O.setup(Ab, wb.part, wb.nparts, wb.nev, wb.overlap)
    mul = O.setup(Ab, wb.part, wb.nparts, wb.nev, wb.overlap, cycle="multiplicative")
    ra, rm = O.pcg(Ab, wb.b, add.apply, 1e-8), O.pcg(Ab, wb.b, mul.apply, 1e-8)
    assert rm.converged and rm.iterations < ra.iterations, (rm.iterations, ra.iterations)


@pytest.mark.parametrize("shape", [(7, 5), (4, 3, 3), (1, 6)])
def test_theta_gradient_matches_central_differences(shape):
    """dJ/dtheta for theta = log kappa (the adjoint of the solve chained
    through the two-point-flux assembly) against central differences of J
    computed with the generator's own assembly and sparse direct solves: a
    dropped boundary term, a swapped kP/kQ in dT/dkappa or a missing factor
    kappa = dkappa/dtheta fails this."""
    from workloads import darcy
    rng = np.random.default_rng(91)
    theta = 1.5 * rng.standard_normal(shape)
    A = darcy.tpfa_matrix(np.exp(theta)).to_scipy()
    n = A.shape[0]
    f, uobs = rng.standard_normal(n), rng.standard_normal(n)
    u, J, g = O.theta_gradient(A, f, uobs, np.exp(theta))
    assert np.allclose(u, spla.spsolve(A.tocsc(), f), rtol=1e-12, atol=1e-14)

    def J_of(th):
        x = spla.spsolve(darcy.tpfa_matrix(np.exp(th)).to_scipy().tocsc(), f)
        return 0.5 * (x - uobs) @ (x - uobs)

    assert abs(J_of(theta) - J) <= 1e-12 * J
    for _ in range(6):
        d = rng.standard_normal(shape)
        d /= np.linalg.norm(d)
        h = 1e-5
        fd = (J_of(theta + h * d) - J_of(theta - h * d)) / (2 * h)
        assert abs(fd - (g * d).sum()) <= 1e-8 * np.linalg.norm(g)


def test_theta_gradient_single_cell_closed_form():
    """One cell (1x1 grid, 2D): A = 4 * 2 kappa (four Dirichlet faces, s = 1),
    u = f / (8 kappa), J = 0.5 (u - uobs)^2, so
    dJ/dtheta = (u - uobs) * du/dtheta = -(u - uobs) u."""
    kappa, f, uobs = 3.0, 2.0, 0.01
    A = sp.csr_matrix(np.array([[8.0 * kappa]]))
    u, J, g = O.theta_gradient(A, np.array([f]), np.array([uobs]), np.array([[kappa]]))
    uu = f / (8 * kappa)
    assert abs(u[0] - uu) <= 1e-15
    assert abs(g[0, 0] - (-(uu - uobs) * uu)) <= 1e-15


def test_validate_rejects_bad_inputs():
    """The oracle refuses what the method is not defined for: a non-square or
    asymmetric matrix, a non-positive diagonal, a partition out of range or
    with an empty subdomain."""
    A = W.darcy.tpfa_matrix(np.ones((4, 4))).to_scipy()
    part = np.repeat(np.arange(2), 8)
    O.validate(A, part, 2)  # a valid input passes
    with pytest.raises(O.OracleError, match="square"):
        O.validate(sp.csr_matrix(np.ones((3, 4))), np.zeros(3, dtype=int), 1)
    B = A.tolil()
    B[0, 1] = B[0, 1] * 2.0
    with pytest.raises(O.OracleError, match="symmetric"):
        O.validate(B.tocsr(), part, 2)
    C = A.tolil()
    C[3, 3] = 0.0
    with pytest.raises(O.OracleError, match="diagonal"):
        O.validate(C.tocsr(), part, 2)
    with pytest.raises(O.OracleError, match="range"):
        O.validate(A, part, 1)
    with pytest.raises(O.OracleError, match="range"):
        O.validate(A, part[:-1], 2)
    with pytest.raises(O.OracleError, match="empty"):
        O.validate(A, part, 3)


def blocks_problem(nb=3, side=8):
    """Uniform coefficient on a grid of nb x nb square cores of side cells:
    with one overlap layer the centre region is a plus shape (the core and a
    strip of side cells on each of its four sides), symmetric under all
    reflections of the square."""
    nx = nb * side
    A = W.darcy.tpfa_matrix(np.ones((nx, nx))).to_scipy()
    ix, iy = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    part = ((ix // side) + nb * (iy // side)).ravel()
    return A, part


def test_symmetric_region_gives_a_degenerate_cut():
    """The reading of the gap flags (lambda_{m+1} - lambda_m tiny): on a region
    invariant under the square's reflections, with a uniform coefficient, the
    Neumann pencil (hat A_i, S_i) has the same symmetry, so its second and
    third eigenvalues coincide (a two-dimensional symmetry class) while the
    first is zero (constants).  A cut after the second mode is then
    degenerate there, a cut after the first is not."""
    A, part = blocks_problem()
    st = O.setup(A, part, 9, 2, overlap=1)
    c = 4  # the centre core
    assert len(st.regions[c]) == 64 + 4 * 8
    lam = st.lam[c]
    assert abs(lam[0]) < 1e-12
    assert abs(lam[2] - lam[1]) <= 1e-10 * lam[2], lam
    st1 = O.setup(A, part, 9, 1, overlap=1)
    assert st1.lam[c][1] - st1.lam[c][0] > 1e-3
