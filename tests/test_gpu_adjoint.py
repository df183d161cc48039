"""Adjoint of the solve through the C ABI: the gradient of a scalar loss
J(u) = 0.5 ||u - u_obs||^2 of u = A^{-1} f with respect to the stored values of
A and to f (paper_2606_04864_amd.solve, amsp_grad_values).  Not part of the
paper's method; it differentiates the solve the preconditioner serves.

Checked against the oracle's gradient from direct sparse solves, and against
central differences of the GPU solve itself.  On the adjoint configuration
(adjoint256) the gradient with respect to theta = log kappa chains the solve's
adjoint through the torch two-point-flux assembly (workloads.tpfa_torch):
against the oracle's theta_gradient at 1e-8 and against central differences
on 50 random unit directions (h = 1e-4, those solves to 1e-13) at 1e-6 of
||dJ/dtheta||, for the FP64 and the mixed form.  The solves run to a relative
residual of 1e-12; the bars (max-abs error over max-abs value): u and the
gradients 1e-8 (FP64 form) and 1e-7 (mixed form, whose preconditioner differs
but whose CG runs in FP64); central differences 1e-5 plus 1e-7 of the largest
gradient (solve tolerance over the step).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2606_04864_amd as P  # noqa: E402

RTOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _problem():
    w = W.get("channels64")
    A = sp.csr_matrix((w.A.val, w.A.col_idx, w.A.row_ptr), shape=(w.n, w.n))
    rng = np.random.default_rng(2606)
    f = rng.standard_normal(w.n)
    uobs = rng.standard_normal(w.n)
    return w, A, f, uobs


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _gpu_grads(w, f, uobs, precision):
    vals = torch.tensor(w.A.val, dtype=torch.float64, device="cuda", requires_grad=True)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
    u = P.solve(vals, ft, w.A.row_ptr, w.A.col_idx, w.part, w.nparts, w.nev, rtol=RTOL,
                overlap=w.overlap, precision=precision)
    J = 0.5 * ((u - torch.tensor(uobs, device="cuda")) ** 2).sum()
    J.backward()
    torch.cuda.synchronize()
    return (u.detach().cpu().numpy(), vals.grad.cpu().numpy(), ft.grad.cpu().numpy(),
            float(J.detach()))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-8), ("fp32", 1e-7)])
def test_solve_gradient_matches_oracle(precision, bar):
    w, A, f, uobs = _problem()
    say(f"adjoint vs oracle: channels64, precision={precision}")
    u, gv, gf, _ = _gpu_grads(w, f, uobs, precision)
    uo = O.adjoint_gradients(A, f, np.zeros(w.n))[0]
    _, lam, go = O.adjoint_gradients(A, f, uo - uobs)
    eu, ev, ef = _rel(u, uo), _rel(gv, go), _rel(gf, lam)
    say(f"  u {eu:.2e}  dJ/dvals {ev:.2e}  dJ/df {ef:.2e}")
    assert eu <= bar and ev <= bar and ef <= bar


def test_solve_gradient_central_differences():
    w, A, f, uobs = _problem()
    say("adjoint vs central differences of the GPU solve: channels64, fp64")
    _, gv, _, _ = _gpu_grads(w, f, uobs, "fp64")
    rows = np.repeat(np.arange(w.n), np.diff(w.A.row_ptr))
    off = np.nonzero(rows != w.A.col_idx)[0]
    dia = np.nonzero(rows == w.A.col_idx)[0]
    rng = np.random.default_rng(7)
    gmax = np.abs(gv).max()
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    ut = torch.tensor(uobs, dtype=torch.float64, device="cuda")

    def loss(vals):
        u = P.solve(torch.tensor(vals, dtype=torch.float64, device="cuda"), ft, w.A.row_ptr,
                    w.A.col_idx, w.part, w.nparts, w.nev, rtol=RTOL, overlap=w.overlap)
        return float(0.5 * ((u - ut) ** 2).sum())

    # symmetric pairs (the solver needs symmetric A): the change of J is the
    # sum of the pair's gradients; diagonal entries alone
    big = off[np.argsort(-np.abs(gv[off]))[:2]]
    for k in list(big) + list(rng.choice(dia, 2, replace=False)):
        i, j = rows[k], w.A.col_idx[k]
        ks = [k] if i == j else [k, int(np.nonzero((rows == j) & (w.A.col_idx == i))[0][0])]
        h = 1e-4 * abs(w.A.val[k])
        vp, vm = w.A.val.copy(), w.A.val.copy()
        vp[ks] += h
        vm[ks] -= h
        fd = (loss(vp) - loss(vm)) / (2 * h)
        an = float(gv[ks].sum())
        say(f"  entry {k} ({i},{j}): fd {fd:.8e} adjoint {an:.8e}")
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7 * gmax


# --------------------------------------------------------------------------
# The adjoint configuration: 256 x 256, theta = log kappa (GRF, variance 4),
# J = 0.5 ||u(theta) - u_obs||^2; dJ/dtheta by the adjoint solve chained
# through the torch two-point-flux assembly (the forward model), against the
# oracle's gradient (sparse direct solves + the closed-form derivatives of
# the assembly) and against central differences on 50 random unit
# directions (h = 1e-4, solves to 1e-13).
_ADJ = {}


def _adjoint_case():
    if "w" not in _ADJ:
        from workloads.tpfa_torch import TpfaAssembly
        w = W.get("adjoint256")
        A = w.A.to_scipy()
        _, J, g = O.theta_gradient(A, w.b, w.u_obs, w.kappa)
        _ADJ["w"] = (w, TpfaAssembly(w.grid, w.A.row_ptr, w.A.col_idx), J, g)
    return _ADJ["w"]


def _theta_loss(w, asm, theta, precision, ft, ut, rtol=RTOL):
    vals = asm.values(theta)
    u = P.solve(vals, ft, w.A.row_ptr, w.A.col_idx, w.part, w.nparts, w.nev, rtol=rtol,
                overlap=w.overlap, precision=precision)
    return 0.5 * ((u - ut) ** 2).sum()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_theta_gradient_matches_oracle(precision):
    w, asm, Jo, go = _adjoint_case()
    say(f"dJ/dtheta vs oracle: adjoint256, precision={precision}")
    ft = torch.tensor(w.b, device="cuda")
    ut = torch.tensor(w.u_obs, device="cuda")
    theta = torch.tensor(w.theta, device="cuda", requires_grad=True)
    J = _theta_loss(w, asm, theta, precision, ft, ut)
    J.backward()
    g = theta.grad.detach().cpu().numpy()
    eJ, eg = abs(float(J.detach()) - Jo) / Jo, _rel(g, go)
    say(f"  J {float(J.detach()):.10e} (oracle {Jo:.10e}, rel {eJ:.2e}); dJ/dtheta {eg:.2e}")
    assert eJ <= 1e-8 and eg <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_theta_gradient_central_differences_50_directions(precision):
    w, asm, Jo, go = _adjoint_case()
    say(f"dJ/dtheta vs central differences, 50 directions: adjoint256, precision={precision}")
    ft = torch.tensor(w.b, device="cuda")
    ut = torch.tensor(w.u_obs, device="cuda")
    th0 = torch.tensor(w.theta, device="cuda", requires_grad=True)
    _theta_loss(w, asm, th0, precision, ft, ut).backward()
    g = th0.grad.detach()
    gn = float(torch.linalg.norm(g))
    rng = np.random.default_rng(2605)
    # central differences: truncation error O(h^2), rounding error O(eps_J / h)
    # with eps_J the loss's error from solves run to 1e-13; h = 1e-4 sits near
    # the balance of the two (at 1e-5 the rounding part alone reached 0.8 of
    # the bar)
    h = 1e-4
    worst = 0.0
    for k in range(50):
        d = torch.tensor(rng.standard_normal(w.grid), device="cuda")
        d /= torch.linalg.norm(d)
        with torch.no_grad():
            jp = float(_theta_loss(w, asm, th0 + h * d, precision, ft, ut, rtol=1e-13))
            jm = float(_theta_loss(w, asm, th0 - h * d, precision, ft, ut, rtol=1e-13))
        fd = (jp - jm) / (2 * h)
        an = float((g * d).sum())
        worst = max(worst, abs(fd - an) / gn)
        assert abs(fd - an) <= 1e-6 * gn, (k, fd, an, gn)
    say(f"  worst |fd - g.d| / ||g|| over 50 directions: {worst:.2e}")
