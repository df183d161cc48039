"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (FP64 form):
  * SpMV, region sets, local/coarse index work: exact or 1e-14 relative;
  * local eigenvalues of S^{-1/2} hat A S^{-1/2} (spectrum in [0, 2]): 1e-10
    absolute (eigensolver residual bound 1e-12 -> eigenvalue error <= 1e-12);
  * A0 spectrum: 1e-10 relative to its largest eigenvalue;
  * M^{-1} v and the PCG solution: max(1e-10, 10 F) relative, where F is the
    oracle's own floor for that same quantity, measured as the difference
    between two oracle runs that differ only in the local ordering (ascending
    vs descending global index); the same bar per core subdomain in the max
    norm (a wrong low-magnitude region cannot hide under a global 2-norm);
  * PCG: recursive residual histories within 100x the oracle's own
    iteration-by-iteration divergence under a rounding-only change (reversed
    local order), at least 1e-5 decades; iteration counts equal up to 1 plus
    the number of oracle iterations whose residual lies within 3x of rtol.
Mixed forms: true relative residual below max(1e-8, attainable floor) and the
solution within 1e-6 of the oracle's.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from workloads import configs

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
        if name == "channels64":
            w = W.get("channels64")
        elif name == "gauss128":
            w = W.get("gauss128")
        elif name == "tiny16":  # subdomains with n_i <= 16: direct small eigen path
            w = configs.channels(nx=12, nparts=16, overlap=0, nev=3)
        elif name == "ragged":  # n not a multiple of 64, uneven parts
            w = configs.gauss_inclusions(nx=61, nparts=7, overlap=1, nev=5, ndisks=6)
        elif name == "nev12":  # more than 8 kept vectors: basis rows read as 16 values
            w = configs.channels(nx=64, nparts=16, overlap=1, nev=12)
        else:
            raise KeyError(name)
        A = w.A.to_scipy()
        st = O.setup(A, w.part, w.nparts, w.nev, w.overlap)
        _CACHE[name] = (w, A, st)
    return _CACHE[name]


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_ALT = {}


def alt_setup(name):
    """The oracle with the reversed local ordering (a rounding-only change)."""
    if name not in _ALT:
        w, A, _ = case(name)
        _ALT[name] = O.setup(A, w.part, w.nparts, w.nev, w.overlap, local_order="descending")
    return _ALT[name]


def oracle_floor(name, r, which="both"):
    """F: oracle vs oracle with the reversed local ordering, and the same
    difference per core subdomain (max norm)."""
    w, A, st = case(name)
    f = {"local": O.local_part, "coarse": O.coarse_part, "both": O.apply}[which]
    a, b = f(st, r), f(alt_setup(name), r)
    return relerr(b, a), core_errors(b, a, w.part, w.nparts)


def core_errors(z, ref, part, nparts):
    """max |z - ref| / max |ref| on every core subdomain."""
    order = np.argsort(part, kind="stable")
    cuts = np.searchsorted(part[order], np.arange(nparts + 1))
    d = np.abs(z - ref)[order]
    a = np.abs(ref)[order]
    return np.array([d[cuts[i]:cuts[i + 1]].max() / max(a[cuts[i]:cuts[i + 1]].max(), 1e-300)
                     for i in range(nparts)])


def check_cores(z, ref, w, fcore, what):
    """Per-core bar: max(1e-10, 10 F_i) with F_i the oracle's own per-core floor."""
    e = core_errors(z, ref, w.part, w.nparts)
    bar = np.maximum(1e-10, 10 * fcore)
    k = int(np.argmax(e / bar))
    say(f"  {what}: worst core {k}: err {e[k]:.2e} bar {bar[k]:.2e} (max core err {e.max():.2e})")
    assert np.all(e <= bar), (what, k, e[k], bar[k])


def test_mfma_layout_selftest():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((16, 4))
    b = rng.standard_normal((4, 16))
    d = P.selftest_mfma(a, b)
    np.testing.assert_allclose(d, a @ b, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("name", ["channels64", "gauss128", "ragged"])
def test_spmv(name):
    w, A, st = case(name)
    say("spmv", name)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    x = np.random.default_rng(1).standard_normal(w.n)
    y = host(pc.spmv(dev(x)))
    ref = A @ x
    assert relerr(y, ref) < 1e-14
    pc.close()


@pytest.mark.parametrize("name", ["channels64", "gauss128", "tiny16", "ragged"])
def test_setup_parity(name):
    w, A, st = case(name)
    say("setup parity", name)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, keep_a0=True)
    info = pc.info
    assert info["eig_unconverged"] == 0
    assert info["nc"] == st.nc
    for i in range(w.nparts):
        d, phi = pc.region(i)
        assert np.array_equal(np.sort(d), st.regions[i])
    lam = pc.eigenvalues()
    for i in range(w.nparts):
        k = len(st.lam[i])
        np.testing.assert_allclose(lam[i, :k], st.lam[i], rtol=0, atol=1e-10)
    A0 = pc.coarse_matrix()
    assert np.abs(A0 - A0.T).max() == 0.0
    e_gpu = np.linalg.eigvalsh(A0)
    e_ref = np.linalg.eigvalsh(st.A0)
    a0err = np.abs(e_gpu - e_ref).max() / np.abs(e_ref).max()
    say(f"  A0 spectrum relerr {a0err:.2e} (nc {st.nc})")
    assert a0err <= 1e-10
    # each exported basis block spans the oracle's (up to rotation and sign):
    # projector difference, S-orthonormality after undoing the PoU scaling
    for i in range(0, w.nparts, max(1, w.nparts // 5)):
        d, phi = pc.region(i)
        order = np.argsort(d)
        psi = (phi[order] * st.mult[d[order]][:, None])[:, :st.psi[i].shape[1]]
        ref = st.psi[i]
        s = O.weighting(O.neumann_matrix(O.local_matrix(A, st.regions[i])))
        G = psi.T @ (s[:, None] * psi)
        np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-8)
        Pg = psi @ psi.T @ np.diag(s)
        Pr = ref @ ref.T @ np.diag(s)
        assert np.abs(Pg - Pr).max() < 1e-6 * max(1.0, np.abs(Pr).max())
    pc.close()


@pytest.mark.parametrize("name", ["channels64", "gauss128", "tiny16", "ragged", "nev12"])
def test_apply_parity(name):
    w, A, st = case(name)
    say("apply parity", name)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    r = np.random.default_rng(2).standard_normal(w.n)
    for parts, which, ref in [(1, "local", O.local_part(st, r)), (2, "coarse", O.coarse_part(st, r)),
                              (3, "both", O.apply(st, r))]:
        z = host(pc.apply(dev(r), parts=parts))
        F, fcore = oracle_floor(name, r, which)
        tol = max(1e-10, 10 * F)
        err = relerr(z, ref)
        say(f"  parts={parts} err={err:.2e} tol={tol:.2e}")
        assert err <= tol
        check_cores(z, ref, w, fcore, f"parts={parts}")
    pc.close()


def test_preconditioner_symmetric_positive():
    w, A, st = case("gauss128")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x, y = rng.standard_normal(w.n), rng.standard_normal(w.n)
        mx, my = host(pc.apply(dev(x))), host(pc.apply(dev(y)))
        assert abs(x @ my - y @ mx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(my)
        assert x @ mx > 0
    pc.close()


@pytest.mark.parametrize("name", ["channels64", "gauss128", "ragged", "nev12"])
def test_pcg_parity(name):
    w, A, st = case(name)
    say("pcg parity", name)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    u, info = pc.pcg(dev(w.b), 1e-8, 1000)
    res = O.pcg(A, w.b, st.apply, 1e-8)
    assert info["converged"] == 1
    assert info["relres_true"] <= max(1e-8, info["relres_floor"])
    # Residual histories: CG in floating point amplifies rounding differences
    # from iteration to iteration, so the bar per iteration is 10x the
    # oracle's own divergence (ascending vs descending local order, i.e. a
    # rounding-only change) times 100, at least 1e-5 decades (the GPU path
    # differs from the oracle in more rounding sources than a reordering).
    hist = pc.pcg_history()
    ref = np.array(res.relres_history)
    res_alt = O.pcg(A, w.b, alt_setup(name).apply, 1e-8)
    alt = np.array(res_alt.relres_history)
    k = min(len(hist), len(ref), len(alt))
    self_div = np.maximum.accumulate(np.abs(np.log10(ref[:k]) - np.log10(alt[:k])))
    gpu_div = np.abs(np.log10(hist[:k]) - np.log10(ref[:k]))
    assert np.all(gpu_div <= np.maximum(1e-5, 100 * self_div)), (gpu_div, self_div)
    # the stopping step is ambiguous while the residual hovers within 3x of rtol
    near = int(np.sum((ref > 1e-8) & (ref < 3e-8)))
    slack = 1 + near + abs(len(ref) - len(alt))
    assert abs(info["iterations"] - res.iterations) <= slack, (info["iterations"], res.iterations)
    # the solution: F is the oracle's own PCG solution under the reordering
    uh = host(u)
    F = relerr(res_alt.x, res.x)
    err = relerr(uh, res.x)
    say(f"  u err {err:.2e} bar {max(1e-10, 10 * F):.2e} (its {info['iterations']}, first "
        f"segment {info['first_segment']}, restarts {info['restarts']}; oracle {res.iterations})")
    assert abs(info["first_segment"] - res.iterations) <= slack
    assert err <= max(1e-10, 10 * F), (err, F)
    check_cores(uh, res.x, w, core_errors(res_alt.x, res.x, w.part, w.nparts), "u")
    pc.close()


@pytest.mark.parametrize("prec,name", [("fp32", "gauss128"), ("bf16", "gauss128"),
                                       ("fp32", "nev12")])
def test_mixed_forms_converge(prec, name):
    w, A, st = case(name)
    say("mixed", prec)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
    u, info = pc.pcg(dev(w.b), 1e-8, 2000)
    res = O.pcg(A, w.b, st.apply, 1e-8)
    assert info["converged"] == 1 and info["relres_true"] <= max(1e-8, info["relres_floor"])
    assert info["iterations"] <= 1.5 * res.iterations + 5
    assert relerr(host(u), res.x) < 1e-6
    pc.close()


def test_determinism_bitwise():
    w, A, st = case("gauss128")
    outs = []
    for _ in range(2):
        pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
        u, info = pc.pcg(dev(w.b), 1e-8, 1000)
        outs.append((host(u), info["iterations"], pc.eigenvalues()))
        pc.close()
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][2], outs[1][2], equal_nan=True)


def test_one_level_schwarz_nev0():
    w, A, _ = case("channels64")
    pc = P.setup(w.A, w.part, w.nparts, 0, overlap=1)
    st0 = O.setup(A, w.part, w.nparts, 0, 1)
    r = np.random.default_rng(4).standard_normal(w.n)
    assert relerr(host(pc.apply(dev(r))), st0.apply(r)) < 1e-10
    u, info = pc.pcg(dev(w.b), 1e-8, 1000)
    res = O.pcg(A, w.b, st0.apply, 1e-8)
    assert abs(info["iterations"] - res.iterations) <= 1
    pc.close()


def test_single_subdomain_is_exact_solve():
    w = configs.channels(nx=20, nparts=1, overlap=0, nev=2)
    pc = P.setup(w.A, w.part, 1, 2, overlap=0)
    u, info = pc.pcg(dev(w.b), 1e-8, 50)
    # local solve = A^{-1}, the coarse term adds a rank-2 SPD piece: at most 3 steps
    assert info["iterations"] <= 3 and info["converged"] == 1
    pc.close()


@pytest.mark.parametrize("opts", [dict(local_order="natural"), dict(dense_tiles=True),
                                  dict(pou=1)])
def test_layout_options_same_operator(opts):
    w, A, st = case("channels64")
    say("layout", opts)
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, **opts)
    r = np.random.default_rng(5).standard_normal(w.n)
    ref = st.apply(r) if opts.get("pou", 0) == 0 else O.apply(
        O.setup(A, w.part, w.nparts, w.nev, w.overlap, pou="none"), r)
    assert relerr(host(pc.apply(dev(r))), ref) < 1e-9
    pc.close()


def test_pcg_status_paths():
    w, A, _ = case("channels64")
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap)
    u, info = pc.pcg(dev(w.b), 1e-8, 1, raise_on_noconv=False)
    assert info["status"] == "AMSP_ERR_PCG_NOCONV" and info["iterations"] == 1
    z, info = pc.pcg(dev(np.zeros(w.n)), 1e-8, 10)
    assert info["iterations"] == 0 and np.all(host(z) == 0)
    bad = w.b.copy()
    bad[3] = np.nan
    with pytest.raises(P.AmspError) as e:
        pc.pcg(dev(bad), 1e-8, 10)
    assert e.value.name == "AMSP_ERR_BREAKDOWN"
    pc.close()


def test_device_error_codes():
    # a negative diagonal entry makes the local Dirichlet matrix indefinite
    w = configs.channels(nx=16, nparts=4, overlap=1, nev=2)
    val = w.A.val.copy()
    for r in range(w.n):
        for e in range(w.A.row_ptr[r], w.A.row_ptr[r + 1]):
            if w.A.col_idx[e] == r and r == 37:
                val[e] = -val[e]
    with pytest.raises(P.AmspError) as e:
        P.Preconditioner(w.A.row_ptr, w.A.col_idx, val, w.part, 4, 2, overlap=1)
    assert e.value.name == "AMSP_ERR_LOCAL_NOT_SPD"
    # a positive off-diagonal pair that drives S_jj <= 0
    val = w.A.val.copy()
    j = 40
    for e in range(w.A.row_ptr[j], w.A.row_ptr[j + 1]):
        c = w.A.col_idx[e]
        if c != j:
            val[e] = 100.0
            for f in range(w.A.row_ptr[c], w.A.row_ptr[c + 1]):
                if w.A.col_idx[f] == j:
                    val[f] = 100.0
    with pytest.raises(P.AmspError) as e:
        P.Preconditioner(w.A.row_ptr, w.A.col_idx, val, w.part, 4, 2, overlap=1)
    assert e.value.name in ("AMSP_ERR_NEUMANN_DIAG", "AMSP_ERR_LOCAL_NOT_SPD")


def test_gap_flags_and_mu_c_match_the_oracle():
    """The setup's gap flags (lambda_{m+1} - lambda_m below 1e-8 relative) and
    mu_c = min_i lambda_{m_i+1} against the oracle's eigenvalues, on a grid of
    3 x 3 square cores with a uniform coefficient: the centre region is
    symmetric under the square's reflections, so a cut after its second mode
    is degenerate (one flag) and a cut after the first is not (none)."""
    from test_oracle_pins import blocks_problem
    A, part = blocks_problem()
    Ac = sp.csr_matrix(A)
    Ac.sort_indices()
    for nev, want in ((2, 1), (1, 0)):
        st = O.setup(A, part, 9, nev, overlap=1)
        flags = sum(1 for lam in st.lam if len(lam) > nev
                    and lam[nev] - lam[nev - 1] < 1e-8 * max(lam[nev], 1e-12))
        mu = min(lam[nev] for lam in st.lam)
        assert flags == want
        pc = P.Preconditioner(Ac.indptr.astype(np.int64), Ac.indices.astype(np.int32), Ac.data,
                              part.astype(np.int32), 9, nev, overlap=1)
        si = pc.info
        say(f"nev {nev}: gap flags {si['n_gap_flags']} (oracle {flags}), mu_c {si['mu_c']:.12g} "
            f"(oracle {mu:.12g})")
        assert si["n_gap_flags"] == flags
        assert abs(si["mu_c"] - mu) <= 1e-10 * mu
        pc.close()
