"""Full-size checks on the 3D configuration: layered128 (128^3 7-point
two-point-flux Darcy, n = 2,097,152; 32 layers with 1e6-contrast channels and
kz = 0.1 kx; 4096 parts, 1 overlap layer, 8 eigenvectors; N_c = 32,768).

As for the 2D benchmark size, the oracle checks samples it can compute one by
one (local eigenpairs of sampled subdomains, the local solves hit by a vector
supported on one core) and properties that hold at any size check the rest:
M^{-1} symmetric and positive (FP64 form), both forms reach the attainable
residual, agree on the solution and need similar iteration counts.
"""
import sys
import time

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2606_04864_amd as P  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def big3d():
    t = time.time()
    w = W.get("layered128")
    say(f"layered128 generated: n={w.n} parts={w.nparts} ({time.time() - t:.0f} s)")
    A = w.A.to_scipy()
    t = time.time()
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    torch.cuda.synchronize()
    say(f"fp64 setup {1e3 * (time.time() - t):.0f} ms, nc={pc.info['nc']}")
    yield w, A, pc
    pc.close()


def test_layered_eigen_samples(big3d):
    w, A, pc = big3d
    assert pc.info["eig_unconverged"] == 0
    lam = pc.eigenvalues()
    cores = O.cores(w.part, w.nparts)
    for i in np.linspace(0, w.nparts - 1, 5).astype(int):
        d = O.grow(A, cores[i], w.overlap)
        Ah = O.neumann_matrix(O.local_matrix(A, d))
        ref, _ = O.local_eigenpairs(Ah, O.weighting(Ah), w.nev, d)
        err = np.abs(lam[i, :len(ref)] - ref).max()
        say(f"  subdomain {i}: n_i={len(d)} eigenvalue error {err:.1e}")
        assert err <= 1e-10


def test_layered_local_solves_sample(big3d):
    w, A, pc = big3d
    rng = np.random.default_rng(21)
    cores = O.cores(w.part, w.nparts)
    i = w.nparts // 3
    r = np.zeros(w.n)
    r[cores[i]] = rng.standard_normal(len(cores[i]))
    z = pc.apply(torch.tensor(r, device="cuda"), parts=1)
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    ref = np.zeros(w.n)
    hit = 0
    for j in range(w.nparts):
        d = O.grow(A, cores[j], w.overlap)
        if not np.any(r[d]):
            continue
        hit += 1
        ref[d] += sla.cho_solve(sla.cho_factor(O.local_matrix(A, d), lower=True), r[d])
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say(f"  local solves: {hit} regions hit, relative error {err:.1e}")
    assert hit >= 2
    assert err <= 1e-9


def test_layered_symmetry_and_pcg(big3d):
    w, A, pc = big3d
    rng = np.random.default_rng(22)
    x, y = rng.standard_normal(w.n), rng.standard_normal(w.n)
    mx = pc.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    my = pc.apply(torch.tensor(y, device="cuda")).cpu().numpy()
    assert abs(x @ my - y @ mx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(my)
    assert x @ mx > 0
    f = torch.tensor(w.b, device="cuda")
    u64, i64 = pc.pcg(f, 1e-8, 3000)
    say(f"  fp64 pcg: {i64['iterations']} its, true {i64['relres_true']:.2e}, "
        f"floor {i64['relres_floor']:.2e}")
    assert i64["converged"] == 1 and i64["relres_true"] <= max(1e-8, i64["relres_floor"])
    t = time.time()
    pm = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision="fp32")
    torch.cuda.synchronize()
    say(f"  mixed setup {1e3 * (time.time() - t):.0f} ms")
    u32, i32 = pm.pcg(f, 1e-8, 3000)
    say(f"  mixed pcg: {i32['iterations']} its, true {i32['relres_true']:.2e}")
    assert i32["converged"] == 1 and i32["relres_true"] <= max(1e-8, i32["relres_floor"])
    assert abs(i32["iterations"] - i64["iterations"]) <= max(3, 0.1 * i64["iterations"])
    d = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
    say(f"  mixed vs fp64 solution: {d:.1e}")
    assert d < 1e-5
    pm.close()
