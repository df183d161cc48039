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
        nf = [len(x) for x in P]
        P, Q = np.concatenate(P), np.concatenate(Q)
        # faces of every cell, 2 per axis (as P, as Q), the missing ones
        # pointing at a zero appended to the face values: the diagonal is a
        # row sum of this table, a fixed order (a scatter-add onto repeated
        # indices would add in an order that changes from run to run)
        faces = np.full((n, 2 * d), len(P), dtype=np.int64)
        f0 = 0
        for a in range(d):
            fa = np.arange(f0, f0 + nf[a])
            faces[P[fa], 2 * a] = fa
            faces[Q[fa], 2 * a + 1] = fa
            f0 += nf[a]
        diag = pos(np.arange(n), np.arange(n))
        t = lambda x: torch.as_tensor(x)
        self._P, self._Q = t(P), t(Q)
        self._pq, self._qp = t(pos(P, Q)), t(pos(Q, P))
        self._diag, self._faces = t(diag), t(faces)
        self._nb = t(nb)
        self._dev = None

    def _to(self, device):
        if self._dev != device:
            for name in ("_P", "_Q", "_pq", "_qp", "_diag", "_faces", "_nb"):
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
        Tz = torch.cat([T, T.new_zeros(1)])
        dg = Tz[self._faces].sum(dim=1) + self.s * 2.0 * k * self._nb
        # every CSR position is written once: no accumulation, a fixed result
        vals = torch.zeros(self.nnz, dtype=theta.dtype, device=theta.device)
        vals = vals.index_put((self._pq,), -T).index_put((self._qp,), -T)
        return vals.index_put((self._diag,), dg)
