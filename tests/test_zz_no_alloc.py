"""amsp_apply_noalloc (the allocation-free block apply) through the C ABI
against amsp_apply, the entry point it is a variant of: both run the same
block kernels, so the results are bitwise equal; two calls in a row share the
per-device scratch array, the second with a smaller input (fewer columns, then
a smaller problem on another handle).  Also: the single-column case against
amsp_apply's single-column path and the oracle, the mixed form's
precondition, and the rejection of a workspace beyond the array."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2606_04864_amd as P  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_noalloc_matches_apply_two_calls():
    wa, wb = W.get("gauss128"), W.get("channels64")
    pa = P.setup(wa.A, wa.part, wa.nparts, wa.nev, overlap=wa.overlap)
    pb = P.setup(wb.A, wb.part, wb.nparts, wb.nev, overlap=wb.overlap)
    rng = np.random.default_rng(71)
    calls = [(pa, wa, 6, 3), (pa, wa, 2, 3), (pb, wb, 3, 3), (pb, wb, 2, 2), (pa, wa, 5, 1)]
    for pc, w, k, parts in calls:
        say(f"noalloc {w.name} columns {k} parts {parts}")
        R = torch.tensor(rng.standard_normal((w.n, k)), device="cuda")
        ref = host(pc.apply(R, parts=parts))
        z = host(pc.apply_noalloc(R, parts=parts))
        assert np.array_equal(z, ref), (w.name, k, parts, np.abs(z - ref).max())
    pa.close()
    pb.close()


def test_noalloc_single_column_and_oracle():
    w = W.get("gauss128")
    A = w.A.to_scipy()
    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
    alt = O.setup(A, w.part, w.nparts, w.nev, w.overlap, local_order="descending")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    r = np.random.default_rng(72).standard_normal(w.n)
    rt = torch.tensor(r, device="cuda")
    z = host(pc.apply_noalloc(rt))
    ref = st.apply(r)
    bar = max(1e-10, 10 * relerr(alt.apply(r), ref))
    say(f"single column: vs oracle {relerr(z, ref):.2e} (bar {bar:.2e}), vs amsp_apply "
        f"{relerr(z, host(pc.apply(rt))):.2e}")
    assert relerr(z, ref) <= bar
    assert relerr(z, host(pc.apply(rt))) <= bar
    pc.close()


def test_noalloc_mixed_needs_block_factor_copy():
    w = W.get("channels64")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision="fp32")
    R = torch.tensor(np.random.default_rng(73).standard_normal((w.n, 4)), device="cuda")
    # the coarse term alone needs no factor copy
    assert np.array_equal(host(pc.apply_noalloc(R, parts=2)), host(pc.apply(R, parts=2)))
    with pytest.raises(P.AmspError) as e:
        pc.apply_noalloc(R)
    assert e.value.name == "AMSP_ERR_ARG"
    ref = host(pc.apply(R))  # builds the copy
    assert np.array_equal(host(pc.apply_noalloc(R)), ref)
    pc.close()


def test_noalloc_rejects_workspace_beyond_the_array():
    w = configs.gauss_inclusions(nx=512, nparts=256, overlap=2, nev=6)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    R = torch.zeros((w.n, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(P.AmspError) as e:
        pc.apply_noalloc(R)
    assert e.value.name == "AMSP_ERR_ARG" and "exceeds" in e.value.msg
    pc.close()
