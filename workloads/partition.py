"""Deterministic algebraic graph partitioner (host input, computed once).

The paper splits the graph of A into non-overlapping subdomains with METIS
(Section 3.1 and Section 5).  METIS is not available here, so this module
provides a plain recursive graph bisection that uses only the sparsity
pattern of A (no coordinates): for a node set R it finds a pseudo-diameter
pair (u, v) by repeated breadth-first search inside R, orders the nodes of R
by (d_u - d_v, d_u, index) and cuts at the count that keeps the two halves
proportional to the number of parts each half will receive.

The partition is an input of the preconditioner: it is computed once, hashed,
and the very same int32 array is handed to the oracle and to the HIP path.
"""
from __future__ import annotations

import hashlib

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path


def _bfs_dist(G: sp.csr_matrix, src: int) -> np.ndarray:
    d = shortest_path(G, method="D", unweighted=True, directed=False, indices=[src])[0]
    return d


def _far(d: np.ndarray) -> int:
    finite = np.isfinite(d)
    m = d[finite].max()
    return int(np.flatnonzero(finite & (d == m))[0])


def _bisect(G: sp.csr_matrix, n_left: int) -> np.ndarray:
    """Return a boolean mask (len = G.shape[0]) selecting n_left nodes."""
    m = G.shape[0]
    # pseudo-peripheral node: two BFS sweeps from node 0
    d = _bfs_dist(G, 0)
    u = _far(d)
    du = _bfs_dist(G, u)
    v = _far(du)
    dv = _bfs_dist(G, v)
    # disconnected pieces (infinite distances) go to the end of the order
    big = float(m + 1)
    du = np.where(np.isfinite(du), du, big)
    dv = np.where(np.isfinite(dv), dv, big)
    key1 = du - dv
    order = np.lexsort((np.arange(m), du, key1))
    mask = np.zeros(m, dtype=bool)
    mask[order[:n_left]] = True
    return mask


def partition(row_ptr: np.ndarray, col_idx: np.ndarray, nparts: int) -> np.ndarray:
    """Partition the graph of a symmetric CSR pattern into nparts non-empty parts."""
    n = len(row_ptr) - 1
    if nparts < 1 or nparts > n:
        raise ValueError("nparts must be in [1, n]")
    G = sp.csr_matrix((np.ones(len(col_idx), dtype=np.int8), col_idx.astype(np.int64),
                       row_ptr.astype(np.int64)), shape=(n, n))
    G.setdiag(0)
    G.eliminate_zeros()
    part = np.empty(n, dtype=np.int32)
    # work list of (node array, first part id, number of parts)
    stack = [(np.arange(n, dtype=np.int64), 0, nparts)]
    while stack:
        nodes, p0, k = stack.pop()
        if k == 1:
            part[nodes] = p0
            continue
        k_left = k // 2
        n_left = int(round(len(nodes) * k_left / k))
        sub = G[nodes][:, nodes]
        mask = _bisect(sub, n_left)
        stack.append((nodes[~mask], p0 + k_left, k - k_left))
        stack.append((nodes[mask], p0, k_left))
    return part


def partition_hash(part: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(part, dtype=np.int32).tobytes()).hexdigest()
