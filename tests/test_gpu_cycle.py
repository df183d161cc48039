"""The multiplicative two-grid cycle (amsp_options.cycle = 1) through the C
ABI against the oracle's apply_multiplicative.

Bars as for the additive operator: M^{-1} v within max(1e-10, 10 F), F the
oracle's own floor under a rounding-only change (reversed local order); the
operator symmetric to 1e-12 relative (x.My against y.Mx); PCG iteration
counts equal up to 1 plus the oracle steps within 3x of rtol; solutions
within max(1e-10, 10 F) of the oracle's.  Mixed forms: converge to the
attainable residual with fewer iterations than the additive operator.
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


def case(name, omega=None):
    key = (name, omega)
    if key not in _C:
        w = W.get(name)
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, w.nev, w.overlap, cycle="multiplicative", omega=omega)
        alt = O.setup(A, w.part, w.nparts, w.nev, w.overlap, cycle="multiplicative", omega=omega,
                      local_order="descending")
        _C[key] = (w, A, st, alt)
    return _C[key]


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,omega", [("channels64", None), ("gauss128", None),
                                        ("channels64", 0.5)])
def test_cycle_apply_parity(name, omega):
    w, A, st, alt = case(name, omega)
    say("cycle apply", name, omega)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, cycle="multiplicative",
                 smoother_weight=omega or 0.0)
    rng = np.random.default_rng(41)
    x, y = rng.standard_normal(w.n), rng.standard_normal(w.n)
    ref = st.apply(x)
    floor = relerr(alt.apply(x), ref)
    mx, my = host(pc.apply(dev(x))), host(pc.apply(dev(y)))
    assert relerr(mx, ref) <= max(1e-10, 10 * floor), (relerr(mx, ref), floor)
    assert abs(x @ my - y @ mx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(my)
    assert x @ mx > 0
    pc.close()


@pytest.mark.parametrize("name", ["channels64", "gauss128"])
def test_cycle_pcg_parity(name):
    w, A, st, alt = case(name)
    say("cycle pcg", name)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, cycle="multiplicative")
    u, info = pc.pcg(dev(w.b), 1e-8, 1000)
    ref = O.pcg(A, w.b, st.apply, 1e-8)
    assert info["converged"] == 1 and info["relres_true"] <= max(1e-8, info["relres_floor"])
    h = np.array(ref.relres_history)
    slack = 1 + int(np.sum((h > 1e-8) & (h < 3e-8)))
    assert abs(info["iterations"] - ref.iterations) <= slack, (info["iterations"], ref.iterations)
    floor = relerr(O.pcg(A, w.b, alt.apply, 1e-8).x, ref.x)
    err = relerr(host(u), ref.x)
    say(f"  u err {err:.2e} bar {max(1e-10, 10 * floor):.2e}")
    assert err <= max(1e-10, 10 * floor), (err, floor)
    pc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cycle_mixed_forms(prec):
    w = W.get("gauss128")
    say("cycle mixed", prec)
    add = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
    _, ia = add.pcg(dev(w.b), 1e-8, 2000)
    add.close()
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec,
                 cycle="multiplicative")
    u, info = pc.pcg(dev(w.b), 1e-8, 2000)
    assert info["converged"] == 1 and info["relres_true"] <= max(1e-8, info["relres_floor"])
    assert info["iterations"] < ia["iterations"], (info["iterations"], ia["iterations"])
    _, ig = pc.gmres(dev(w.b), rtol=1e-6)
    assert ig["converged"] == 1
    pc.close()


def test_cycle_neumann_and_options():
    w = W.get("neumann64")
    A = w.A.to_scipy()
    say("cycle neumann")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, singular=True,
                 cycle="multiplicative")
    u, info = pc.pcg(dev(w.b), 1e-8, 1000)
    assert info["converged"] == 1
    uh = host(u)
    assert np.linalg.norm(w.b - A @ uh) <= 1.01 * max(1e-8, info["relres_floor"]) * np.linalg.norm(w.b)
    pc.close()
    for kw in ({"cycle": "multiplicative", "smoother_weight": -1.0},
               {"cycle": "multiplicative", "smoother_weight": float("nan")}):
        with pytest.raises(P.AmspError) as e:
            P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, **kw)
        assert e.value.name == "AMSP_ERR_ARG"
