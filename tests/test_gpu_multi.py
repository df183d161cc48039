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
from conftest import cg_breakdown_step, shifted_indefinite

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
        if name == "nev12":  # more than 8 kept vectors: basis rows read as 16 values
            w = W.configs.channels(nx=64, nparts=16, overlap=1, nev=12)
        else:
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
                                          ("gauss128", 5, 2), ("nev12", 3, 3)])
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


@pytest.mark.parametrize("name,k", [("channels64", 4), ("gauss128", 3)])
def test_block_pcg_parity(name, k):
    """Columns solved together: each reaches rtol with the oracle's solution
    (bar of the one-column PCG parity), and the summed iteration count is
    the oracle's up to one step per column."""
    w, A, st, alt = case(name)
    say("block pcg", name, k)
    rng = np.random.default_rng(53)
    F = np.column_stack([w.b] + [rng.standard_normal(w.n) for _ in range(k - 1)])
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    U, info = pc.pcg(torch.tensor(F, device="cuda"), 1e-8, 1000)
    U = host(U)
    assert info["converged"] == 1
    its = 0
    for j in range(k):
        ref = O.pcg(A, F[:, j], st.apply, 1e-8)
        its += ref.iterations
        floor = relerr(O.pcg(A, F[:, j], alt.apply, 1e-8).x, ref.x)
        err = relerr(U[:, j], ref.x)
        say(f"  column {j}: u err {err:.2e} bar {max(1e-10, 10 * floor):.2e}")
        assert err <= max(1e-10, 10 * floor), (j, err, floor)
        rel = np.linalg.norm(F[:, j] - A @ U[:, j]) / np.linalg.norm(F[:, j])
        assert rel <= 1.01 * max(1e-8, info["relres_floor"]), (j, rel)
    assert abs(info["iterations"] - its) <= k, (info["iterations"], its)
    pc.close()


def test_block_pcg_mixed_and_edges():
    w, A, _, _ = case("gauss128")
    say("block pcg mixed")
    rng = np.random.default_rng(54)
    F = np.column_stack([w.b, rng.standard_normal(w.n), np.zeros(w.n), rng.standard_normal(w.n)])
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision="fp32")
    Ft = torch.tensor(F, device="cuda")
    U, info = pc.pcg(Ft, 1e-8, 2000)
    U = host(U)
    assert info["converged"] == 1
    assert np.all(U[:, 2] == 0)
    single = 0
    for j in (0, 1, 3):
        rel = np.linalg.norm(F[:, j] - A @ U[:, j]) / np.linalg.norm(F[:, j])
        assert rel <= 1.01 * max(1e-8, info["relres_floor"]), (j, rel)
        single += pc.pcg(Ft[:, j].contiguous(), 1e-8, 2000)[1]["iterations"]
    assert info["iterations"] <= 1.2 * single + 6, (info["iterations"], single)
    bad = F.copy()
    bad[5, 1] = np.nan
    with pytest.raises(P.AmspError) as e:
        pc.pcg(torch.tensor(bad, device="cuda"), 1e-8, 100)
    assert e.value.name == "AMSP_ERR_BREAKDOWN"
    u, info = pc.pcg(Ft[:, 0].contiguous(), 1e-8, 2000)  # the handle still solves
    assert info["converged"] == 1
    pc.close()


def test_block_pcg_breaks_down_mid_solve():
    """An indefinite operator (A - sigma I, every local factor SPD, nev = 0):
    each column stops on the device at its own first p.Ap <= 0 and keeps the
    iterate of the step before, equal to the oracle's CG iterate of that
    step; a zero column is untouched.  The call reports AMSP_ERR_BREAKDOWN
    with u and info written for every column."""
    w, As, val, sigma = shifted_indefinite()
    st = O.setup(As, w.part, w.nparts, 0, 1)
    alt = O.setup(As, w.part, w.nparts, 0, 1, local_order="descending")
    pc = P.Preconditioner(w.A.row_ptr, w.A.col_idx, val, w.part, w.nparts, 0, overlap=1)
    R = np.random.default_rng(71).standard_normal((w.n, 3))
    F = np.column_stack([R[:, 1], np.zeros(w.n), R[:, 2]])
    with pytest.raises(P.AmspError) as e:
        pc.pcg(torch.tensor(F, device="cuda"), 1e-8, 500)
    assert e.value.name == "AMSP_ERR_BREAKDOWN" and e.value.result is not None
    U, info = e.value.result
    U = host(U)
    assert info["converged"] == 0 and np.all(U[:, 1] == 0)
    steps = 0
    for j in (0, 2):
        t, xt = cg_breakdown_step(As, F[:, j], st.apply)
        ta, xa = cg_breakdown_step(As, F[:, j], alt.apply)
        assert t == ta and t >= 2
        err, bar = relerr(U[:, j], xt), max(1e-10, 10 * relerr(xa, xt))
        say(f"breakdown column {j}: oracle stops after {t} steps (sigma {sigma:.4f}), "
            f"iterate err {err:.2e} bar {bar:.2e}")
        assert err <= bar
        steps += t
    assert info["iterations"] == steps
    # the one-column path stops on the same condition
    with pytest.raises(P.AmspError) as e:
        pc.pcg(torch.tensor(F[:, 0], device="cuda"), 1e-8, 500)
    assert e.value.name == "AMSP_ERR_BREAKDOWN"
    pc.close()


def test_column_layout_bindings_match():
    """apply_columns / pcg_columns take the right-hand sides as rows of a
    (k, n) tensor (the C layout); the results equal the (n, k) calls exactly."""
    w, A, _, _ = case("channels64")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    R = torch.tensor(np.random.default_rng(55).standard_normal((w.n, 5)), device="cuda")
    Zc = host(pc.apply_columns(R.t().contiguous()))
    Zr = host(pc.apply(R))
    assert np.array_equal(Zc, Zr.T)
    Uc, ic = pc.pcg_columns(R.t().contiguous(), 1e-8, 500)
    Ur, ir = pc.pcg(R, 1e-8, 500)
    assert np.array_equal(host(Uc), host(Ur).T) and ic["iterations"] == ir["iterations"]
    with pytest.raises(ValueError):
        pc.apply_columns(R)
    pc.close()
