"""Plain FP64 CPU oracle of the two-grid algebraic multiscale preconditioner.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the HIP library: numpy/scipy (LAPACK) in float64, written
to be read against the paper, not to be fast.

Paper: "An algebraic multiscale preconditioner for large sparse SPD matrices"
(Zhou, Fu, Chung).  Section references below are to that paper.

Readings where the paper is silent (each also listed in the design notes):
  * overlap: the support region around a core subdomain (Section 3.1, "an
    overlapping region constructed around Omega_i") is delta rounds of
    adding graph neighbours; the local problems live on that region;
  * Neumann diagonal (Section 3.2): only couplings inside the region count;
  * partition of unity: each zero-extended eigenvector is divided by the
    number of regions that contain the dof (the paper zero-extends only);
  * preconditioner: additive two-level Schwarz, the paper's coarse term
    R0^T A0^{-1} R0 (Section 3.1) plus local solves sum_i R_i^T A_i^{-1} R_i,
    so that the operator is SPD and usable in CG;
  * Krylov method: preconditioned CG stopping on the unpreconditioned 2-norm
    ||r|| <= rtol ||f|| from x0 = 0; and the paper's own GMRES (Section 5),
    right-preconditioned in flexible form so that it minimises and reports
    the same residual, restarted every 30 steps unless told otherwise;
  * normalisation/sign: psi^T S psi = 1, largest-|entry| positive (lowest
    global index on ties).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class OracleError(ValueError):
    pass


# --------------------------------------------------------------------------
# Input checks (Section 1: A is symmetric positive definite; Section 3.1: the
# non-overlapping partition covers every dof).
# --------------------------------------------------------------------------
def validate(A: sp.csr_matrix, part: np.ndarray, nparts: int) -> None:
    n = A.shape[0]
    if A.shape != (n, n):
        raise OracleError("A must be square")
    if abs(A - A.T).max() > 1e-14 * abs(A).max():
        raise OracleError("A must be symmetric")
    if (A.diagonal() <= 0).any():
        raise OracleError("diagonal of A must be positive")
    if len(part) != n or part.min() < 0 or part.max() >= nparts:
        raise OracleError("partition out of range")
    if (np.bincount(part, minlength=nparts) == 0).any():
        raise OracleError("empty subdomain")


# --------------------------------------------------------------------------
# Subdomains (Section 3.1): cores Omega_i from the partition, then the
# overlapping region Omega_i^delta by delta rounds of graph growth.
# --------------------------------------------------------------------------
def cores(part: np.ndarray, nparts: int) -> list[np.ndarray]:
    order = np.argsort(part, kind="stable")
    counts = np.bincount(part, minlength=nparts)
    splits = np.cumsum(counts)[:-1]
    return [np.sort(c) for c in np.split(order, splits)]


def grow(A: sp.csr_matrix, dofs: np.ndarray, delta: int) -> np.ndarray:
    """Omega^delta: add every dof coupled (nonzero off-diagonal) to the set, delta times."""
    cur = np.asarray(dofs, dtype=np.int64)
    for _ in range(delta):
        rows = A[cur]
        nb = rows.indices[rows.data != 0]
        cur = np.union1d(cur, nb)
    return cur


def multiplicity(n: int, regions: list[np.ndarray]) -> np.ndarray:
    mult = np.zeros(n, dtype=np.int64)
    for r in regions:
        mult[r] += 1
    return mult


# --------------------------------------------------------------------------
# Local matrices (Section 3.2).
# --------------------------------------------------------------------------
def local_matrix(A: sp.csr_matrix, dofs: np.ndarray) -> np.ndarray:
    """A_i = R_i A R_i^T (Boolean restriction to the region, dense)."""
    return A[dofs][:, dofs].toarray()


def neumann_matrix(Ai: np.ndarray) -> np.ndarray:
    """hat A_i: keep the off-diagonals of A_i, set each diagonal entry to minus
    the sum of the off-diagonal entries of its row, so that row sums vanish."""
    Ah = Ai.copy()
    np.fill_diagonal(Ah, 0.0)
    np.fill_diagonal(Ah, -Ah.sum(axis=1))
    return Ah


def weighting(Ah: np.ndarray) -> np.ndarray:
    """S_i = diag(hat A_i), returned as the vector of its diagonal."""
    s = np.diag(Ah).copy()
    if (s <= 0).any():
        raise OracleError("weighting matrix S_i must have a positive diagonal")
    return s


def local_eigenpairs(Ah: np.ndarray, s: np.ndarray, m: int, gdofs: np.ndarray | None = None):
    """Smallest eigenpairs of hat A psi = lambda S psi (the algebraic local
    eigenproblem of Section 3.2), solved through the equivalent standard
    problem S^{-1/2} hat A S^{-1/2} z = lambda z with psi = S^{-1/2} z
    (Section 5, parameter test).

    Returns (lam, psi): lam holds min(m+1, n_i) eigenvalues (the last one is
    the first eigenvalue left out of the coarse space, used for mu_c of
    Theorem 2); psi holds the first m_i = min(m, n_i) eigenvectors,
    normalised psi^T S psi = 1, sign: largest |entry| positive.
    """
    ni = Ah.shape[0]
    mi = min(m, ni)
    k = min(m + 1, ni)
    dm = 1.0 / np.sqrt(s)
    B = dm[:, None] * Ah * dm[None, :]
    B = 0.5 * (B + B.T)
    lam, Z = sla.eigh(B, subset_by_index=[0, k - 1])
    psi = dm[:, None] * Z[:, :mi]
    if gdofs is None:
        gdofs = np.arange(ni)
    for c in range(mi):
        a = np.abs(psi[:, c])
        cand = np.flatnonzero(a == a.max())
        j = cand[np.argmin(gdofs[cand])]
        if psi[j, c] < 0:
            psi[:, c] = -psi[:, c]
    return lam, psi


# --------------------------------------------------------------------------
# Coarse space (Section 3.1 and 3.2): R0^T columns are the (scaled,
# zero-extended) local eigenvectors; A0 = R0 A R0^T.
# --------------------------------------------------------------------------
def prolongation(n: int, regions, psis, mult, pou: str = "mult") -> sp.csr_matrix:
    cols, rows, vals = [], [], []
    c0 = 0
    for dofs, psi in zip(regions, psis):
        for k in range(psi.shape[1]):
            v = psi[:, k].copy()
            if pou == "mult":
                v = v / mult[dofs]
            rows.append(dofs)
            cols.append(np.full(len(dofs), c0 + k))
            vals.append(v)
        c0 += psi.shape[1]
    if c0 == 0:
        return sp.csr_matrix((n, 0))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, c0))


def coarse_matrix(A: sp.csr_matrix, R0T: sp.csr_matrix) -> np.ndarray:
    """A0 = R0 A R0^T (Galerkin projection), symmetrised."""
    A0 = (R0T.T @ (A @ R0T)).toarray()
    return 0.5 * (A0 + A0.T)


# --------------------------------------------------------------------------
# The preconditioner M^{-1} r = sum_i R_i^T A_i^{-1} R_i r + R0^T A0^{-1} R0 r.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Setup:
    n: int
    regions: list
    mult: np.ndarray
    local_chol: list
    lam: list
    psi: list
    R0T: sp.csr_matrix
    A0: np.ndarray
    A0_chol: object
    nev: int
    overlap: int
    A0_pinv: np.ndarray | None = None  # singular problems: the pseudo-inverse of A0
    A: sp.csr_matrix | None = None      # kept for the multiplicative cycle
    cycle: str = "additive"
    omega: float = 1.0                  # smoother weight of the multiplicative cycle

    @property
    def nc(self) -> int:
        return self.R0T.shape[1]

    def apply(self, r: np.ndarray) -> np.ndarray:
        return apply(self, r) if self.cycle == "additive" else apply_multiplicative(self, r)


def setup(A, part, nparts, nev, overlap=1, pou="mult", local_order="ascending",
          local_solves=True, singular=False, cycle="additive", omega=None,
          progress=None) -> Setup:
    """singular=True: A is positive semidefinite with a null space (the
    paper's homogeneous Neumann problem, Section 5); the coarse term then
    uses the pseudo-inverse of A0, as the two-level operator of Section 3.1
    is written.

    cycle="multiplicative": the symmetric two-grid cycle of the paper's
    two-grid algorithm and Section 4 (pre-smoothing, coarse correction,
    post-smoothing) with the damped additive Schwarz smoother
    omega * sum_i R_i^T A_i^{-1} R_i; omega defaults to 1 / (the largest
    number of regions containing one dof).

    progress: optional callable(i, N) called after subdomain i's local work
    (reporting only; it does not change any result)."""
    A = sp.csr_matrix(A)
    validate(A, part, nparts)
    if nev < 0:
        raise OracleError("nev must be >= 0")
    n = A.shape[0]
    regions = [grow(A, c, overlap) for c in cores(part, nparts)]
    if local_order == "descending":
        regions = [r[::-1].copy() for r in regions]
    mult = multiplicity(n, regions)
    chol, lams, psis = [], [], []
    for dofs in regions:
        Ai = local_matrix(A, dofs)
        if local_solves:
            try:
                chol.append(sla.cho_factor(Ai, lower=True))
            except np.linalg.LinAlgError as e:
                raise OracleError("local matrix not SPD") from e
        if nev > 0:
            Ah = neumann_matrix(Ai)
            s = weighting(Ah)
            lam, psi = local_eigenpairs(Ah, s, nev, dofs)
        else:
            lam, psi = np.zeros(0), np.zeros((len(dofs), 0))
        lams.append(lam)
        psis.append(psi)
        if progress is not None:
            progress(len(psis) - 1, len(regions))
    R0T = prolongation(n, regions, psis, mult, pou)
    A0p = None
    if R0T.shape[1] > 0:
        A0 = coarse_matrix(A, R0T)
        if singular:
            A0c, A0p = None, pseudo_inverse(A0)
        else:
            try:
                A0c = sla.cho_factor(A0, lower=True)
            except np.linalg.LinAlgError as e:
                raise OracleError("coarse matrix not SPD") from e
    else:
        A0, A0c = np.zeros((0, 0)), None
    if cycle not in ("additive", "multiplicative"):
        raise OracleError("cycle must be additive or multiplicative")
    om = float(omega) if omega is not None else 1.0 / float(mult.max())
    return Setup(n, regions, mult, chol, lams, psis, R0T, A0, A0c, nev, overlap, A0p, A, cycle, om)


def pseudo_inverse(M: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Moore-Penrose inverse of a symmetric positive semidefinite matrix from
    its eigendecomposition: eigenvalues below rtol * the largest count as
    zero."""
    w, Q = np.linalg.eigh(M)
    keep = w > rtol * w.max()
    return (Q[:, keep] / w[keep]) @ Q[:, keep].T


def local_part(st: Setup, r: np.ndarray) -> np.ndarray:
    z = np.zeros_like(r)
    for dofs, c in zip(st.regions, st.local_chol):
        z[dofs] += sla.cho_solve(c, r[dofs])
    return z


def coarse_part(st: Setup, r: np.ndarray) -> np.ndarray:
    if st.nc == 0:
        return np.zeros_like(r)
    c = st.R0T.T @ r
    if st.A0_pinv is not None:
        return st.R0T @ (st.A0_pinv @ c)
    return st.R0T @ sla.cho_solve(st.A0_chol, c)


def apply(st: Setup, r: np.ndarray) -> np.ndarray:
    """M^{-1} r: additive local solves plus the coarse correction."""
    return local_part(st, r) + coarse_part(st, r)


def apply_multiplicative(st: Setup, r: np.ndarray) -> np.ndarray:
    """One symmetric two-grid cycle from x = 0 for A x = r: x1 = S r,
    x2 = x1 + C (r - A x1), x3 = x2 + S (r - A x2), with the smoother
    S = omega * (local solves) and C = R0^T A0^{-1} R0."""
    A = st.A
    x = st.omega * local_part(st, r)
    x = x + coarse_part(st, r - A @ x)
    return x + st.omega * local_part(st, r - A @ x)


# --------------------------------------------------------------------------
# Preconditioned conjugate gradients (Hestenes-Stiefel; Saad, Iterative
# Methods for Sparse Linear Systems, Algorithm 9.1), x0 = 0.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    converged: bool
    relres_history: list
    relres_true: float
    alphas: list
    betas: list


def pcg(A, f, Minv, rtol=1e-8, maxit=1000) -> PCGResult:
    A = sp.csr_matrix(A)
    x = np.zeros_like(f)
    r = f.copy()
    nf = np.linalg.norm(f)
    hist = [1.0 if nf > 0 else 0.0]
    alphas, betas = [], []
    if nf == 0.0:
        return PCGResult(x, 0, True, hist, 0.0, alphas, betas)
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    it = 0
    converged = False
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        alphas.append(alpha)
        rel = np.linalg.norm(r) / nf
        hist.append(rel)
        if rel <= rtol:
            converged = True
            break
        z = Minv(r)
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    true = np.linalg.norm(f - A @ x) / nf
    return PCGResult(x, it, converged, hist, true, alphas, betas)


def lanczos_condition(alphas, betas) -> float:
    """kappa(M^{-1}A) estimate from the CG coefficients (the Lanczos
    tridiagonal T: diag 1/a_k + b_{k-1}/a_{k-1}, offdiag sqrt(b_k)/a_k)."""
    k = len(alphas)
    if k == 0:
        return 1.0
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    for j in range(k):
        d[j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j < k - 1:
            e[j] = np.sqrt(betas[j]) / alphas[j]
    ev = sla.eigh_tridiagonal(d, e, eigvals_only=True)
    return float(ev[-1] / ev[0])


# --------------------------------------------------------------------------
# Preconditioned GMRES, the Krylov method of the paper's experiments
# (Section 5: GMRES with the two-level preconditioner, stopped once the
# relative residual has dropped by 1e-6).  Readings: right preconditioning
# in its flexible form (Saad, Iterative Methods for Sparse Linear Systems,
# Section 9.4.1: the preconditioned vectors z_j = M^{-1} v_j are kept and
# x = x0 + Z y), so the minimised and reported quantity is the true residual
# ||f - A x||_2 relative to ||f|| (x0 = 0); restart length m (30 by default,
# as the paper does not state one); Arnoldi by modified Gram-Schmidt; the
# small least-squares problem by Givens rotations.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class GMRESResult:
    x: np.ndarray
    iterations: int
    converged: bool
    relres_history: list   # |g_{j+1}| / ||f|| after each inner step (entry 0: 1)
    relres_true: float
    restarts: int


def gmres(A, f, Minv, restart=30, rtol=1e-6, maxit=1000) -> GMRESResult:
    A = sp.csr_matrix(A)
    n = f.shape[0]
    x = np.zeros_like(f)
    nf = np.linalg.norm(f)
    hist = [1.0 if nf > 0 else 0.0]
    if nf == 0.0:
        return GMRESResult(x, 0, True, hist, 0.0, 0)
    r = f.copy()
    beta = nf
    it = 0
    cycles = 0
    converged = False
    while it < maxit:
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[:, 0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[:, j] = Minv(V[:, j])
            w = A @ Z[:, j]
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = V[:, i] @ w
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            a, b = H[j, j], H[j + 1, j]
            rho = np.hypot(a, b)
            cs[j], sn[j] = (a / rho, b / rho) if rho > 0.0 else (1.0, 0.0)
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nf)
            if abs(g[j + 1]) <= rtol * nf or it >= maxit or H[k - 1, k - 1] == 0.0:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k], lower=False)
        x = x + Z[:, :k] @ y
        r = f - A @ x
        beta = np.linalg.norm(r)
        cycles += 1
        if beta <= rtol * nf:
            converged = True
            break
    true = np.linalg.norm(f - A @ x) / nf
    return GMRESResult(x, it, converged, hist, true, cycles - 1)


# --------------------------------------------------------------------------
# Adjoint of the solve.  Not part of the paper's method: it differentiates
# the solve u = A^{-1} f that the preconditioner serves, for a scalar loss
# J(u).  From A u = f, a change dA gives A du = -dA u, so
#   dJ = g . du = -(A^{-T} g) . (dA u),   g = dJ/du.
# With lam = A^{-T} g:  dJ/df = lam  and  dJ/dA_ij = -lam_i u_j  for every
# stored entry (i, j), each entry taken as an independent value.  Both
# solves are sparse direct (SuperLU); the transpose is kept explicit.
def adjoint_gradients(A, f, dJdu):
    """Returns (u, lam, grad_vals) with grad_vals in the CSR entry order of A."""
    A = sp.csr_matrix(A)
    u = spla.spsolve(A.tocsc(), f)
    lam = spla.spsolve(A.T.tocsc(), dJdu)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    return u, lam, -lam[rows] * u[A.indices]


# --------------------------------------------------------------------------
# Gradient with respect to the log-permeability theta = log kappa of a
# two-point-flux Darcy matrix on an nx x ny (x nz) cell grid with h = 1/nx,
# the same kappa on every face direction, homogeneous Dirichlet faces.
# Not part of the paper's method: it chains the adjoint of the solve (above)
# through the matrix assembly.  For the interior face f between cells P and
# Q, T_f = s 2 kP kQ / (kP + kQ) with s = h^(d-2) enters A as A_PQ = A_QP =
# -T_f and adds T_f to A_PP and A_QQ; a Dirichlet face of P adds s 2 kP to
# A_PP.  Hence
#   dJ/dT_f = g_PP + g_QQ - g_PQ - g_QP,
#   dT_f/dkP = s 2 kQ^2 / (kP + kQ)^2,   d(s 2 kP)/dkP = 2 s,
#   dkP/dthetaP = kP,
# with g = dJ/dvals from adjoint_gradients.  Cells are numbered
# j = ix + nx (iy + ny iz); faces are read off the grid, not off A.
def theta_gradient(A, f, u_obs, kappa):
    """dJ/dtheta for J = 0.5 ||A(theta)^{-1} f - u_obs||^2 (kappa indexed
    [ix, iy] or [ix, iy, iz]).  Returns (u, J, grad_theta indexed like kappa)."""
    A = sp.csr_matrix(A)
    u = adjoint_gradients(A, f, np.zeros(A.shape[0]))[0]
    u, lam, g = adjoint_gradients(A, f, u - u_obs)
    J = 0.5 * float((u - u_obs) @ (u - u_obs))
    shape = kappa.shape
    d = len(shape)
    h = 1.0 / shape[0]
    s = h ** (d - 2)
    n = int(np.prod(shape))
    k = np.ascontiguousarray(kappa.T).ravel()  # cell j = ix + nx (iy + ny iz)
    cell = np.arange(n).reshape(shape[::-1]).T  # cell[ix, iy(, iz)]

    def entry(i, j):  # positions of the stored entries (i, j) in A's CSR order
        pos = np.empty(len(i), dtype=np.int64)
        for t, (a, b) in enumerate(zip(i, j)):
            lo, hi = A.indptr[a], A.indptr[a + 1]
            pos[t] = lo + np.searchsorted(A.indices[lo:hi], b)
        return pos

    diag = entry(np.arange(n), np.arange(n))
    grad_k = np.zeros(n)
    for a in range(d):
        # interior faces between consecutive cells along axis a
        P = np.take(cell, np.arange(shape[a] - 1), axis=a).ravel()
        Q = np.take(cell, np.arange(1, shape[a]), axis=a).ravel()
        kP, kQ = k[P], k[Q]
        dJdT = g[diag[P]] + g[diag[Q]] - g[entry(P, Q)] - g[entry(Q, P)]
        np.add.at(grad_k, P, dJdT * s * 2.0 * kQ * kQ / (kP + kQ) ** 2)
        np.add.at(grad_k, Q, dJdT * s * 2.0 * kP * kP / (kP + kQ) ** 2)
        # Dirichlet faces at both ends of axis a
        for end in (0, shape[a] - 1):
            B = np.take(cell, [end], axis=a).ravel()
            np.add.at(grad_k, B, g[diag[B]] * 2.0 * s)
    grad_theta = grad_k * k
    return u, J, grad_theta.reshape(shape[::-1]).T
