import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def load_golden(name):
    """Parse a tests/golden text fixture: 'key: numbers' lines, ';' separates
    matrix rows, '|' separates lists; '#' starts a comment."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line or ":" not in line:
                continue
            key, val = line.split(":", 1)
            val = val.strip()
            if "|" in val:
                out[key.strip()] = [np.array([float(x) for x in part.split()]) for part in val.split("|")]
            elif ";" in val:
                out[key.strip()] = np.array([[float(x) for x in row.split()] for row in val.split(";")])
            else:
                out[key.strip()] = np.array([float(x) for x in val.split()])
    return out


@pytest.fixture
def golden():
    return load_golden


def shifted_indefinite(nx=32, nparts=16, seed_key=1):
    """A channels problem shifted to A - sigma I with lambda_min(A) < sigma <
    the smallest eigenvalue of every overlapping region's Dirichlet matrix
    A_i: the operator is indefinite while every local factor stays SPD, so
    the one-level setup (nev = 0) succeeds and CG meets p.Ap <= 0 after a
    few steps (the breakdown cases).  Returns (workload, shifted scipy
    matrix, shifted values in the workload's CSR order, sigma)."""
    import scipy.sparse as sp

    import oracle as O
    from workloads import configs
    w = configs.channels(nx=nx, nparts=nparts, overlap=1, nev=0, seed_key=seed_key)
    A = w.A.to_scipy()
    regions = O.setup(A, w.part, w.nparts, 0, 1).regions
    lo = np.linalg.eigvalsh(A.toarray())[0]
    hi = min(np.linalg.eigvalsh(A[d][:, d].toarray())[0] for d in regions)
    assert lo < hi, (lo, hi)
    sigma = 0.5 * (lo + hi)
    rows = np.repeat(np.arange(w.n), np.diff(w.A.row_ptr))
    val = w.A.val - sigma * (rows == w.A.col_idx)
    return w, (A - sigma * sp.identity(w.n, format="csr")).tocsr(), val, sigma


def cg_breakdown_step(A, f, Minv, maxit=200):
    """The oracle's CG run until its first step with p.Ap <= 0: returns
    (t, x_t), t the steps completed before it and x_t the iterate then."""
    import oracle as O
    for t in range(maxit):
        res = O.pcg(A, f, Minv, 0.0, t + 1)
        if not res.alphas[-1] > 0:
            return t, O.pcg(A, f, Minv, 0.0, t).x
    raise AssertionError("no breakdown")
