"""The two-point-flux Darcy assembly of darcy.tpfa_matrix written in torch
operations, so that a loss of the solution can be differentiated with respect
to theta = log kappa by chaining the solve's adjoint (the gradient with
respect to the stored values of A) through the assembly.

This is the application's forward model, not the preconditioner: the values
it produces are the CSR values of darcy.tpfa_matrix(exp(theta)) in the same
order (sorted columns per row), for a 2D or 3D grid with the same kappa on
every face direction and homogeneous Dirichlet faces:
  interior face (P, Q): T = s 2 kP kQ / (kP + kQ), s = h^(d-2), h = 1/nx,
      A_PQ = A_QP = -T, and T is added to A_PP and A_QQ;
  Dirichlet face of P: s 2 kP added to A_PP.
"""
from __future__ import annotations

import numpy as np


class TpfaAssembly:
    """Index maps of one grid (built once with numpy); values(theta) then
    assembles in torch on theta's device."""

    def __init__(self, shape, row_ptr: np.ndarray, col_idx: np.ndarray):
        import torch
        self.shape = tuple(shape)
        d = len(shape)
        n = int(np.prod(shape))
        self.n, self.nnz = n, int(row_ptr[-1])
        self.s = (1.0 / shape[0]) ** (d - 2)
        cell = np.arange(n).reshape(self.shape[::-1]).T  # cell[ix, iy(, iz)]
        rows = np.repeat(np.arange(n), np.diff(row_ptr))
        key = rows.astype(np.int64) * n + col_idx  # CSR entries are sorted by this key

        def pos(i, j):
            p = np.searchsorted(key, i.astype(np.int64) * n + j)
            assert np.all(key[p] == i.astype(np.int64) * n + j), "entry missing from the pattern"
            return p

        P, Q = [], []
        nb = np.zeros(n)
        for a in range(d):
            P.append(np.take(cell, np.arange(shape[a] - 1), axis=a).ravel())
            Q.append(np.take(cell, np.arange(1, shape[a]), axis=a).ravel())
            for end in (0, shape[a] - 1):
                np.add.at(nb, np.take(cell, [end], axis=a).ravel(), 1.0)
        P, Q = np.concatenate(P), np.concatenate(Q)
        diag = pos(np.arange(n), np.arange(n))
        t = lambda x: torch.as_tensor(x)
        self._P, self._Q = t(P), t(Q)
        self._pq, self._qp = t(pos(P, Q)), t(pos(Q, P))
        self._dp, self._dq, self._diag = t(diag[P]), t(diag[Q]), t(diag)
        self._nb = t(nb)
        self._dev = None

    def _to(self, device):
        if self._dev != device:
            for name in ("_P", "_Q", "_pq", "_qp", "_dp", "_dq", "_diag", "_nb"):
                setattr(self, name, getattr(self, name).to(device))
            self._dev = device

    def values(self, theta):
        """CSR values of A(exp(theta)); theta: float64 tensor of the grid's
        shape indexed [ix, iy(, iz)] (differentiable)."""
        import torch
        self._to(theta.device)
        k = theta.permute(*reversed(range(theta.dim()))).reshape(-1).exp()  # cell order
        kP, kQ = k[self._P], k[self._Q]
        T = self.s * 2.0 * kP * kQ / (kP + kQ)
        vals = torch.zeros(self.nnz, dtype=theta.dtype, device=theta.device)
        vals = vals.index_add(0, self._pq, -T).index_add(0, self._qp, -T)
        vals = vals.index_add(0, self._dp, T).index_add(0, self._dq, T)
        return vals.index_add(0, self._diag, self.s * 2.0 * k * self._nb)
