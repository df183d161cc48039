"""The paper's homogeneous Neumann problem (singular A, pseudo-inverse of
A0) through the C ABI against the oracle.

The device applies A0^+ as (A0 + alpha u u^T)^{-1} with u = R0 1; on vectors
orthogonal to the constants this differs from the oracle's pseudo-inverse by
a multiple of the constant vector only, and solutions of the singular system
are defined up to a constant.  So every comparison removes the mean first.
Bars as for the Dirichlet cases: M^{-1} v within max(1e-10, 10 F) with F the
oracle's own floor (reversed local order); PCG to 1e-8 with the iteration
count of the oracle up to 1 plus the steps within 3x of rtol; solutions
within 1e-6 of the grounded direct solve modulo constants.
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2606_04864_amd as P  # noqa: E402

_C = {}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def case():
    if not _C:
        w = W.get("neumann64")
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, w.nev, w.overlap, singular=True)
        ug = np.concatenate([[0.0], spla.spsolve(A[1:, 1:].tocsc(), w.b[1:])])
        _C.update(w=w, A=A, st=st, ug=ug - ug.mean())
    return _C["w"], _C["A"], _C["st"], _C["ug"]


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def centred(x):
    return x - x.mean()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_neumann_apply_parity():
    w, A, st, _ = case()
    say("neumann apply parity")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, singular=True, keep_a0=True)
    alt = O.setup(A, w.part, w.nparts, w.nev, w.overlap, singular=True, local_order="descending")
    rng = np.random.default_rng(31)
    for _ in range(2):
        v = centred(rng.standard_normal(w.n))
        ref = centred(st.apply(v))
        floor = relerr(centred(alt.apply(v)), ref)
        got = centred(host(pc.apply(dev(v))))
        assert relerr(got, ref) <= max(1e-10, 10 * floor), (relerr(got, ref), floor)
    # the exported A0 is the Galerkin product itself, singular along R0^T c = 1
    ev = np.linalg.eigvalsh(pc.coarse_matrix())
    ref_ev = np.linalg.eigvalsh(st.A0)
    assert abs(ev[0]) <= 1e-12 * ref_ev[-1]
    np.testing.assert_allclose(ev[1:], ref_ev[1:], rtol=1e-8)
    pc.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_neumann_pcg(prec):
    w, A, st, ug = case()
    say("neumann pcg", prec)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, singular=True, precision=prec)
    u, info = pc.pcg(dev(w.b), 1e-8, 1000)
    assert info["converged"] == 1 and info["relres_true"] <= max(1e-8, info["relres_floor"])
    uh = host(u)
    assert np.linalg.norm(w.b - A @ uh) <= 1.01 * max(1e-8, info["relres_floor"]) * np.linalg.norm(w.b)
    assert relerr(centred(uh), ug) < 1e-6
    if prec == "fp64":
        ref = O.pcg(A, w.b, st.apply, 1e-8)
        h = np.array(ref.relres_history)
        slack = 1 + int(np.sum((h > 1e-8) & (h < 3e-8)))
        assert abs(info["iterations"] - ref.iterations) <= slack, (info["iterations"], ref.iterations)
    pc.close()


def test_neumann_gmres():
    w, A, st, ug = case()
    say("neumann gmres")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, singular=True)
    u, info = pc.gmres(dev(w.b), rtol=1e-6)
    ref = O.gmres(A, w.b, st.apply, restart=30, rtol=1e-6)
    assert info["converged"] == 1 and ref.converged
    assert abs(info["iterations"] - ref.iterations) <= 1, (info["iterations"], ref.iterations)
    uh = host(u)
    assert np.linalg.norm(w.b - A @ uh) <= 1e-6 * np.linalg.norm(w.b)
    assert relerr(centred(uh), ug) < 1e-3
    pc.close()
