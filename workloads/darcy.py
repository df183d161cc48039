"""Seeded synthetic heterogeneous Darcy matrices (two-point-flux finite volumes).

This module only produces inputs: the SPD matrix A (CSR), the right-hand side
and the permeability field.  It contains none of the preconditioner's
arithmetic, so both the CPU oracle and the HIP path consume its output.

The paper's experiments use an elliptic pressure equation -div(kappa grad u) = f
with heterogeneous kappa (Section 2, the model problem; Section 5, the Darcy
tests).  Its own discretisation (lowest-order Raviart-Thomas with velocity
elimination) reduces on Cartesian grids to the cell-centred two-point stencil
built here.  Boundary: homogeneous Dirichlet u = 0, imposed through a
half-cell transmissibility 2*kappa_P, so A is a symmetric M-matrix with
nonnegative row sums (the property the paper's energy-splitting lemma uses).

Cell index j = ix + nx*(iy + ny*iz); h = 1/nx; interior face transmissibility
T = h^(d-2) * 2 kP kQ / (kP + kQ); Dirichlet face T_b = h^(d-2) * 2 kP;
A_PP = sum of T, A_PQ = -T, b_P = h^d f_P.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int64 row_ptr, int32 col_idx (sorted per row), float64 val."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx.astype(np.int64), self.row_ptr),
                             shape=(self.n, self.n))

    @staticmethod
    def from_scipy(M) -> "CSR":
        M = sp.csr_matrix(M)
        M.sort_indices()
        M.sum_duplicates()
        return CSR(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32),
                   M.data.astype(np.float64))


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def tpfa_matrix(kx: np.ndarray, kz: np.ndarray | None = None, neumann: bool = False) -> CSR:
    """Assemble the TPFA matrix for a 2D (nx, ny) or 3D (nx, ny, nz) field.

    kx is indexed [ix, iy] or [ix, iy, iz]; kx is used for x and y faces and
    kz (default kx) for z faces.  neumann=True drops the Dirichlet boundary
    faces (homogeneous Neumann problem: every row sums to zero and the
    constant vector spans the null space).
    """
    d = kx.ndim
    shape = kx.shape
    nx = shape[0]
    h = 1.0 / nx
    scale = h ** (d - 2)
    if kz is None:
        kz = kx
    # flatten with ix fastest: transpose so that C-order ravel gives ix fastest
    kflat = np.ascontiguousarray(kx.T).ravel()
    kzflat = np.ascontiguousarray(kz.T).ravel()
    n = kflat.size
    idx = np.arange(n, dtype=np.int64).reshape(shape[::-1])  # [iz,iy,ix] or [iy,ix]
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    axes = list(range(d))
    for ax_field in axes:  # field axis 0 = x
        arr_axis = d - 1 - ax_field  # axis in the reversed-shape index array
        kk = kzflat if ax_field == 2 else kflat
        lo = np.take(idx, np.arange(shape[ax_field] - 1), axis=arr_axis).ravel()
        hi = np.take(idx, np.arange(1, shape[ax_field]), axis=arr_axis).ravel()
        t = scale * _harm(kk[lo], kk[hi])
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-t, -t]
        np.add.at(diag, lo, t)
        np.add.at(diag, hi, t)
        # Dirichlet faces on both ends of this axis
        for end in ((0, shape[ax_field] - 1) if not neumann else ()):
            b = np.take(idx, [end], axis=arr_axis).ravel()
            np.add.at(diag, b, scale * 2.0 * kk[b])
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    return CSR.from_scipy(M)


def rhs_from_source(f_cells: np.ndarray) -> np.ndarray:
    """b_P = h^d f_P with the same cell ordering as tpfa_matrix (ix fastest)."""
    d = f_cells.ndim
    h = 1.0 / f_cells.shape[0]
    return (h ** d) * np.ascontiguousarray(f_cells.T).ravel().astype(np.float64)


def gaussian_random_field(shape, var: float, corr_len: float, rng: np.random.Generator) -> np.ndarray:
    """Zero-mean stationary Gaussian field, covariance var*exp(-r^2/(2 l^2)).

    Coordinates are cell centres on the unit square/cube (spacing 1/shape[0]).
    Sampled by circulant embedding on a 2x periodic padding (negative
    embedding eigenvalues are clipped to zero), then cropped.
    """
    h = 1.0 / shape[0]
    pshape = tuple(2 * s for s in shape)
    grids = np.meshgrid(*[np.minimum(np.arange(p), p - np.arange(p)) * h for p in pshape],
                        indexing="ij")
    r2 = sum(g * g for g in grids)
    c = var * np.exp(-r2 / (2.0 * corr_len ** 2))
    lam = np.fft.fftn(c).real
    lam = np.maximum(lam, 0.0)
    M = c.size
    xi = rng.standard_normal(pshape) + 1j * rng.standard_normal(pshape)
    y = np.fft.fftn(np.sqrt(lam / M) * xi)
    sl = tuple(slice(0, s) for s in shape)
    return np.ascontiguousarray(y.real[sl])


def channel_field_2d(nx: int, nchan: int, width: int, value: float, rng) -> np.ndarray:
    """Background 1 with nchan full-length axis-aligned straight channels."""
    k = np.ones((nx, nx))
    for _ in range(nchan):
        orient = int(rng.integers(0, 2))
        off = int(rng.integers(0, nx - width + 1))
        if orient == 0:
            k[:, off:off + width] = value  # channel along x
        else:
            k[off:off + width, :] = value  # channel along y
    return k


def disk_inclusions_2d(k: np.ndarray, ndisks: int, rmin: float, rmax: float,
                       factor: float, rng) -> np.ndarray:
    nx = k.shape[0]
    cx = rng.uniform(0, nx, ndisks)
    cy = rng.uniform(0, nx, ndisks)
    rad = rng.uniform(rmin, rmax, ndisks)
    mask = np.zeros(k.shape, dtype=bool)
    ii = np.arange(nx) + 0.5
    for x0, y0, r in zip(cx, cy, rad):
        x_lo, x_hi = max(0, int(x0 - r) - 1), min(nx, int(x0 + r) + 2)
        y_lo, y_hi = max(0, int(y0 - r) - 1), min(nx, int(y0 + r) + 2)
        X, Y = np.meshgrid(ii[x_lo:x_hi], ii[y_lo:y_hi], indexing="ij")
        mask[x_lo:x_hi, y_lo:y_hi] |= (X - x0) ** 2 + (Y - y0) ** 2 <= r * r
    out = k.copy()
    out[mask] *= factor
    return out


def layered_channel_field_3d(n: int, nlayers: int, var: float, corr_len: float,
                             chan_per_layer: int, chan_width: int, factor: float, rng) -> np.ndarray:
    """Layered 3D field: each horizontal layer holds a 2D log-normal field
    extruded through the layer, times `factor` inside sinuous channels."""
    k = np.empty((n, n, n))
    lz = n // nlayers
    xc = (np.arange(n) + 0.5) / n
    for L in range(nlayers):
        logk = gaussian_random_field((n, n), var, corr_len, rng)
        kl = np.exp(logk)
        for _ in range(chan_per_layer):
            y0 = rng.uniform(0.1, 0.9)
            a = rng.uniform(0.05, 0.15)
            lam = rng.uniform(0.3, 1.0)
            phi = rng.uniform(0, 2 * np.pi)
            yc = y0 + a * np.sin(2 * np.pi * xc / lam + phi)  # per ix
            iy = (np.arange(n) + 0.5) / n
            mask = np.abs(iy[None, :] - yc[:, None]) * n <= chan_width / 2.0
            kl = np.where(mask, kl * factor, kl)
        k[:, :, L * lz:(L + 1) * lz] = kl[:, :, None]
    return k
