"""Several right-hand sides per pass (amsp_apply with nrhs >= 2) against the
oracle, column by column.

FP64 form: every column within max(1e-10, 10 F) of the oracle's M^{-1} r_k,
F the oracle's own floor under a rounding-only change (reversed local
order), for both terms together and each alone; widths 2, 5, 16 and 17
(16 + a single column).  Mixed forms: the block path uses the same f32-stored
factor with float64 arithmetic, so each column is at least as close to the
FP64 oracle as the single-column f32 path (within 10x, or 1e-6).
"""
import sys

import numpy as np
import pytest

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


def case(name):
    if name not in _C:
        w = W.get(name)
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
        alt = O.setup(A, w.part, w.nparts, w.nev, w.overlap, local_order="descending")
        _C[name] = (w, A, st, alt)
    return _C[name]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


FN = {3: O.apply, 1: O.local_part, 2: O.coarse_part}


@pytest.mark.parametrize("name,k,parts", [("channels64", 2, 3), ("channels64", 17, 3),
                                          ("gauss128", 16, 3), ("gauss128", 5, 1),
                                          ("gauss128", 5, 2)])
def test_multi_apply_parity(name, k, parts):
    w, A, st, alt = case(name)
    say("multi apply", name, k, parts)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    R = np.random.default_rng(51).standard_normal((w.n, k))
    Z = host(pc.apply(torch.tensor(R, device="cuda"), parts=parts))
    f = FN[parts]
    for j in range(k):
        ref = f(st, R[:, j])
        floor = relerr(f(alt, R[:, j]), ref)
        assert relerr(Z[:, j], ref) <= max(1e-10, 10 * floor), (j, relerr(Z[:, j], ref), floor)
    pc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_multi_apply_mixed(prec):
    w, A, st, _ = case("gauss128")
    say("multi apply mixed", prec)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
    R = np.random.default_rng(52).standard_normal((w.n, 6))
    Rt = torch.tensor(R, device="cuda")
    Z = host(pc.apply(Rt))
    for j in range(6):
        ref = st.apply(R[:, j])
        single = host(pc.apply(Rt[:, j].contiguous()))
        e_single, e_block = relerr(single, ref), relerr(Z[:, j], ref)
        assert e_block <= max(10 * e_single, 1e-6), (j, e_block, e_single)
    pc.close()
