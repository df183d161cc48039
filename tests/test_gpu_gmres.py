"""GMRES through the C ABI (amsp_gmres) against the oracle's GMRES.

Both sides run flexible right-preconditioned restarted GMRES from u = 0 with
the same preconditioner definition; the oracle orthogonalises by modified
Gram-Schmidt, the device by classical Gram-Schmidt applied twice.  Both are
backward-stable ways of computing the same minimisers, so (FP64 form):
  * residual estimates after each step agree, while they are above 1e-9,
    within 100x the oracle's own step-by-step divergence under a
    rounding-only change (reversed local order), at least 1e-8 relative: the
    preconditioner's rounding grows with the contrast (its own parity bar is
    10x the same self-floor), and each step's minimiser inherits it;
  * the step count and the restart count are equal, up to one step when an
    oracle estimate lies within 1.01x of rtol;
  * the two solutions differ by at most 1e-8 ||f|| in the residual norm
    ||A (u - u_oracle)||.
Mixed forms: the true residual meets rtol; steps within 1.5x of FP64.
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

_CACHE = {}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def case(name):
    if name not in _CACHE:
        w = W.get(name)
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
        _CACHE[name] = (w, A, st)
    return _CACHE[name]


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name,restart,rtol", [("channels64", 30, 1e-6), ("channels64", 10, 1e-6),
                                               ("channels64", 64, 1e-10), ("gauss128", 30, 1e-6)])
def test_gmres_parity(name, restart, rtol):
    w, A, st = case(name)
    say("gmres parity", name, restart, rtol)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    u, info = pc.gmres(dev(w.b), rtol=rtol, restart=restart, maxit=2000)
    res = O.gmres(A, w.b, st.apply, restart=restart, rtol=rtol, maxit=2000)
    assert res.converged and info["converged"] == 1
    assert info["relres_true"] <= rtol
    near = int(np.sum(np.abs(np.array(res.relres_history) / rtol - 1.0) < 0.01))
    assert abs(info["iterations"] - res.iterations) <= near, (info["iterations"], res.iterations)
    assert info["restarts"] == res.restarts or near > 0, (info["restarts"], res.restarts)
    hist = pc.pcg_history()
    ref = np.array(res.relres_history)
    alt = np.array(O.gmres(A, w.b, O.setup(A, w.part, w.nparts, w.nev, w.overlap,
                                            local_order="descending").apply,
                           restart=restart, rtol=rtol, maxit=2000).relres_history)
    k = min(len(hist), len(ref), len(alt))
    sel = ref[:k] > 1e-9
    self_div = np.maximum.accumulate(np.abs(alt[:k] - ref[:k]) / ref[:k])[sel]
    rel = np.abs(hist[:k][sel] - ref[:k][sel]) / ref[:k][sel]
    assert np.all(rel <= np.maximum(1e-8, 100 * self_div)), (rel, self_div)
    du = host(u) - res.x
    assert np.linalg.norm(A @ du) <= 1e-8 * np.linalg.norm(w.b)
    pc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_gmres_mixed_forms(prec):
    w, A, st = case("gauss128")
    say("gmres mixed", prec)
    pc64 = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    _, i64 = pc64.gmres(dev(w.b), rtol=1e-6)
    pc64.close()
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
    u, info = pc.gmres(dev(w.b), rtol=1e-6)
    assert info["converged"] == 1 and info["relres_true"] <= 1e-6
    r = w.b - A @ host(u)
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(w.b)
    assert info["iterations"] <= 1.5 * i64["iterations"] + 2, (info["iterations"], i64["iterations"])
    pc.close()


def test_gmres_status_paths():
    w, A, _ = case("channels64")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    u, info = pc.gmres(dev(w.b), rtol=1e-6, maxit=3, raise_on_noconv=False)
    assert info["status"] == "AMSP_ERR_PCG_NOCONV" and info["iterations"] == 3
    assert info["relres_true"] > 1e-6
    z, info = pc.gmres(dev(np.zeros(w.n)), rtol=1e-6)
    assert info["iterations"] == 0 and info["converged"] == 1 and np.all(host(z) == 0)
    bad = w.b.copy()
    bad[3] = np.nan
    with pytest.raises(P.AmspError) as e:
        pc.gmres(dev(bad), rtol=1e-6)
    assert e.value.name == "AMSP_ERR_BREAKDOWN"
    for restart in (0, 65):
        with pytest.raises(P.AmspError) as e:
            pc.gmres(dev(w.b), restart=restart)
        assert e.value.name == "AMSP_ERR_ARG"
    # the handle still solves after the error paths
    u, info = pc.gmres(dev(w.b), rtol=1e-6)
    assert info["converged"] == 1
    pc.close()
