"""Named workloads: seeded synthetic heterogeneous Darcy problems.

Each workload bundles the matrix, the right-hand side, the host partition and
the preconditioner parameters (overlap layers, eigenvectors per subdomain).
Seeds: workload K uses numpy default_rng seeded from SeedSequence(260604864 + K)
with spawned sub-streams for field, source and geometry.

The paper's fields exist only as figures, so these recipes stand in for them:
  * channels64   -- 64x64, background 1 with 8 straight channels (width 2,
                    kappa 1e4), f = 1, 16 parts, 1 overlap layer, 4 eigenvectors.
  * gauss1024    -- 1024x1024, kappa = exp(GRF(var 4, corr 0.05)) times 1e6 in 200
                    disks of radius 3-10 cells, f ~ N(0,1), 1024 parts, 2 overlap
                    layers, 6 eigenvectors.
  * layered128   -- 128^3 7-point, 32 layers of extruded exp(GRF(var 3)) with two
                    sinuous channels (x1e6) per layer, kz = 0.1 kx, 4096 parts,
                    1 overlap layer, 8 eigenvectors.
  * gauss<N>     -- the gauss1024 recipe at a smaller side N (parity sizes).
  * adjoint256   -- 256x256, theta = log kappa = GRF(var 4, corr 0.05), f = 1, u_obs
                    from theta + GRF(var 0.25, corr 0.1), 64 parts, 2 overlap layers,
                    6 eigenvectors (the loss J = 0.5 ||u - u_obs||^2).
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from . import darcy
from .partition import partition, partition_hash

SEED_BASE = 260604864


@dataclasses.dataclass
class Workload:
    name: str
    A: darcy.CSR
    b: np.ndarray
    part: np.ndarray
    nparts: int
    overlap: int
    nev: int
    kappa: np.ndarray
    grid: tuple

    @property
    def n(self) -> int:
        return self.A.n

    def part_sha256(self) -> str:
        return partition_hash(self.part)


def _streams(k: int, count: int = 4):
    ss = np.random.SeedSequence(SEED_BASE + k)
    return [np.random.default_rng(s) for s in ss.spawn(count)]


def channels(nx: int = 64, nparts: int = 16, overlap: int = 1, nev: int = 4,
             contrast: float = 1e4, nchan: int = 8, seed_key: int = 1) -> Workload:
    rng_geo, _, _, _ = _streams(seed_key)
    kappa = darcy.channel_field_2d(nx, nchan, 2, contrast, rng_geo)
    A = darcy.tpfa_matrix(kappa)
    b = darcy.rhs_from_source(np.ones((nx, nx)))
    part = partition(A.row_ptr, A.col_idx, nparts)
    return Workload(f"channels{nx}", A, b, part, nparts, overlap, nev, kappa, (nx, nx))


def gauss_inclusions(nx: int = 1024, nparts: int = 1024, overlap: int = 2, nev: int = 6,
                     var: float = 4.0, corr: float = 0.05, ndisks: int | None = None,
                     factor: float = 1e6, seed_key: int = 2) -> Workload:
    rng_field, rng_src, rng_geo, _ = _streams(seed_key)
    logk = darcy.gaussian_random_field((nx, nx), var, corr, rng_field)
    kappa = np.exp(logk)
    if ndisks is None:
        ndisks = max(1, round(200 * (nx / 1024) ** 2))
    kappa = darcy.disk_inclusions_2d(kappa, ndisks, 3.0, 10.0, factor, rng_geo)
    A = darcy.tpfa_matrix(kappa)
    b = darcy.rhs_from_source(rng_src.standard_normal((nx, nx)))
    part = partition(A.row_ptr, A.col_idx, nparts)
    return Workload(f"gauss{nx}", A, b, part, nparts, overlap, nev, kappa, (nx, nx))


def layered(n: int = 128, nparts: int = 4096, overlap: int = 1, nev: int = 8,
            seed_key: int = 3) -> Workload:
    rng_field, rng_src, _, _ = _streams(seed_key)
    nlayers = 32 if n >= 32 else max(1, n // 4)
    kx = darcy.layered_channel_field_3d(n, nlayers, 3.0, 0.1, 2, 3, 1e6, rng_field)
    A = darcy.tpfa_matrix(kx, 0.1 * kx)
    b = darcy.rhs_from_source(rng_src.standard_normal((n, n, n)))
    part = partition(A.row_ptr, A.col_idx, nparts)
    return Workload(f"layered{n}", A, b, part, nparts, overlap, nev, kx, (n, n, n))


def neumann(nx: int = 64, nparts: int = 16, overlap: int = 1, nev: int = 4,
            contrast: float = 1e4, nchan: int = 8, seed_key: int = 5) -> Workload:
    """The paper's boundary condition (Section 5: homogeneous Neumann): the
    channel field of `channels` without Dirichlet faces, so A is singular
    with the constant vector as its null space, and a source with zero mean
    (f ~ N(0, 1) minus its mean) so that A u = f is consistent."""
    rng_geo, rng_src, _, _ = _streams(seed_key)
    kappa = darcy.channel_field_2d(nx, nchan, 2, contrast, rng_geo)
    A = darcy.tpfa_matrix(kappa, neumann=True)
    src = rng_src.standard_normal((nx, nx))
    b = darcy.rhs_from_source(src - src.mean())
    b -= b.mean()
    part = partition(A.row_ptr, A.col_idx, nparts)
    return Workload(f"neumann{nx}", A, b, part, nparts, overlap, nev, kappa, (nx, nx))


@dataclasses.dataclass
class AdjointWorkload(Workload):
    """The adjoint configuration: theta = log kappa and the observation."""
    theta: np.ndarray = None
    u_obs: np.ndarray = None


def adjoint(nx: int = 256, nparts: int = 64, overlap: int = 2, nev: int = 6,
            seed_key: int = 5) -> AdjointWorkload:
    """The adjoint configuration: theta = log kappa = GRF(var 4, corr 0.05)
    on nx x nx cells, f = 1, J = 0.5 ||u(theta) - u_obs||^2 with u_obs the
    solution for theta_obs = theta + GRF(var 0.25, corr 0.1).  Seeds: the
    third and fourth sub-streams of SeedSequence(260604864 + 5) (the first
    two serve `neumann`).  u_obs is a sparse direct solve (SuperLU): an input,
    not a result of the preconditioner."""
    import scipy.sparse.linalg as spla
    streams = _streams(seed_key)
    rng_theta, rng_obs = streams[2], streams[3]
    theta = darcy.gaussian_random_field((nx, nx), 4.0, 0.05, rng_theta)
    theta_obs = theta + darcy.gaussian_random_field((nx, nx), 0.25, 0.1, rng_obs)
    kappa = np.exp(theta)
    A = darcy.tpfa_matrix(kappa)
    b = darcy.rhs_from_source(np.ones((nx, nx)))
    A_obs = darcy.tpfa_matrix(np.exp(theta_obs)).to_scipy().tocsc()
    u_obs = spla.spsolve(A_obs, b)
    part = partition(A.row_ptr, A.col_idx, nparts)
    return AdjointWorkload(f"adjoint{nx}", A, b, part, nparts, overlap, nev, kappa, (nx, nx),
                           theta=theta, u_obs=u_obs)


@dataclasses.dataclass
class BatchWorkload:
    """Independent problems concatenated into one block-diagonal system: A
    (CSR), the concatenated partition (part ids offset per problem), the
    right-hand sides B (n x nrhs, C order: column k is B[:, k]) and the
    problems' row offsets seg_ptr (nprob + 1)."""
    name: str
    A: darcy.CSR
    B: np.ndarray
    part: np.ndarray
    nparts: int
    overlap: int
    nev: int
    seg_ptr: np.ndarray
    sides: list
    variances: list

    @property
    def n(self) -> int:
        return self.A.n

    @property
    def nprob(self) -> int:
        return len(self.sides)

    def problem(self, p: int):
        """(A_p as scipy CSR, its partition with ids from 0, its nparts, its rows)."""
        a, b = int(self.seg_ptr[p]), int(self.seg_ptr[p + 1])
        Ap = self.A.to_scipy()[a:b, a:b].tocsr()
        pp = self.part[a:b]
        return Ap, pp - pp.min(), int(pp.max() - pp.min() + 1), slice(a, b)


def box_partition(nx: int, ny: int, px: int, py: int) -> np.ndarray:
    """Cells (ix, iy), index ix + nx iy, in px x py rectangular boxes."""
    ix = np.arange(nx) * px // nx
    iy = np.arange(ny) * py // ny
    return (ix[None, :] + px * iy[:, None]).ravel().astype(np.int32)


def batch(nprob: int = 64, smin: int = 128, smax: int = 512, nrhs: int = 8, overlap: int = 1,
          nev: int = 6, corr: float = 0.05, seed_key: int = 4, box: int = 32,
          first: int | None = None) -> BatchWorkload:
    """The batched configuration: nprob independent 2D two-point-flux Darcy
    problems of side s ~ U{smin..smax}, log kappa = GRF(variance ~ U[2, 6],
    correlation length 0.05), nrhs right-hand sides from N(0, 1) sources.
    Each problem is cut into round(s/box)^2 rectangular boxes (box = 32: ~1024
    cells; a graph partition of its grid), one overlap layer, 6 eigenvectors.
    Seeds: sub-streams of SeedSequence(260604864 + 4): sizes and variances,
    then one stream per problem for its field and sources.  first: keep only
    the first problems of the batch (a sample of the same problems)."""
    ss = np.random.SeedSequence(SEED_BASE + seed_key)
    kids = ss.spawn(nprob + 1)
    rng0 = np.random.default_rng(kids[0])
    sides = [int(x) for x in rng0.integers(smin, smax + 1, size=nprob)]
    variances = [float(x) for x in rng0.uniform(2.0, 6.0, size=nprob)]
    if first is not None:
        sides, variances = sides[:first], variances[:first]
    mats, rhs, parts = [], [], []
    poff = 0
    for p, (s_, var) in enumerate(zip(sides, variances)):
        rng = np.random.default_rng(kids[p + 1])
        logk = darcy.gaussian_random_field((s_, s_), var, corr, rng)
        Ap = darcy.tpfa_matrix(np.exp(logk)).to_scipy()
        B = np.stack([darcy.rhs_from_source(rng.standard_normal((s_, s_))) for _ in range(nrhs)],
                     axis=1)
        nb = max(1, round(s_ / box))
        part = box_partition(s_, s_, nb, nb) + poff
        poff += nb * nb
        mats.append(Ap)
        rhs.append(B)
        parts.append(part)
    import scipy.sparse as sp
    A = darcy.CSR.from_scipy(sp.block_diag(mats, format="csr"))
    seg = np.concatenate([[0], np.cumsum([m.shape[0] for m in mats])]).astype(np.int64)
    return BatchWorkload(f"batch{len(sides)}", A, np.ascontiguousarray(np.concatenate(rhs, axis=0)),
                         np.concatenate(parts), poff, overlap, nev, seg, sides, variances)


@functools.lru_cache(maxsize=8)
def get(name: str) -> Workload:
    """Workloads by name; cached per process."""
    if name == "channels64":
        return channels()
    if name == "gauss1024":
        return gauss_inclusions()
    if name == "layered128":
        return layered()
    if name.startswith("gauss"):
        nx = int(name[5:])
        nparts = max(4, (nx * nx) // 1024)
        return gauss_inclusions(nx=nx, nparts=nparts)
    if name.startswith("adjoint"):
        nx = int(name[7:])
        return adjoint(nx=nx, nparts=max(4, (nx * nx) // 1024))
    if name.startswith("neumann"):
        nx = int(name[7:])
        return neumann(nx=nx, nparts=max(4, (nx * nx) // 256))
    if name.startswith("channels"):
        nx = int(name[8:])
        return channels(nx=nx, nparts=max(4, (nx * nx) // 256))
    raise KeyError(name)
