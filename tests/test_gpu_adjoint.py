"""GPU parity of the steady adjoint (dk_eff/dgamma) against the FP64 oracle.

The oracle solves (dR/de)^T psi = -g with its own transposed operator
(scatter form) by GMRES; the GPU runs the transposed synthetic iteration
with reversed sweeps.  Both start from their own converged forward
solution.  Bars: FP64 1e-11, FP32 1e-5 (relative to max |grad|).
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from oracle.adjoint import keff_weights, steady_adjoint
from tests.helpers import geo, mat, rel_err, small_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def adjoint_cases():
    """Geometries with a periodic x axis carrying the temperature drop, and
    every other boundary kind on the remaining faces and pores.  Geometries
    without a thermalizing wall have no heat source (else no steady state)."""
    out = {k: v for k, v in small_cases().items() if k in ("periodic2d", "box3d")}
    rng = np.random.default_rng(77)
    b3 = I.bands(rng, 3, 1e-12, 1e-9)
    solid = np.ones(12 * 9, dtype=np.uint8)
    solid[[26, 27, 38, 39, 70, 95]] = 0
    out["specular2d"] = (geo(2, (12, 9), (120e-9, 90e-9),
                             [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_SPECULAR,
                              I.BC_SPECULAR], pdT=(1.0, 0, 0), solid=solid, pore_bc=I.BC_SPECULAR),
                         mat(b3, 2, 2), None, rng.uniform(0, 1e11, 108))   # no sink: no source either
    out["thermal2d"] = (geo(2, (11, 10), (110e-9, 100e-9),
                            [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_THERMAL, I.BC_DIFFUSE, I.BC_SPECULAR,
                             I.BC_SPECULAR], bcT=[300, 300, 300.3, 300, 300, 300], pdT=(0.7, 0, 0)),
                        mat(b3, 1, 3), rng.uniform(0, 1e17, 110), rng.uniform(0, 1e11, 110))
    out["bulk1d"] = (geo(1, (70,), (140e-9,), [I.BC_PERIODIC, I.BC_PERIODIC] + [I.BC_SPECULAR] * 4,
                         pdT=(1.0, 0, 0)),
                     mat(I.bands(rng, 4, 1e-12, 1e-10), 6), None, rng.uniform(0, 1e11, 70))
    # 3D with more than one 64-lane chunk per octant (6 bands x 12 directions
    # = 72 lanes per octant), pores, periodic x with the drop, periodic z and
    # diffuse y walls: the column walk of the transposed residual and the 3D
    # adjoint sweep over several chunks
    solid = np.ones(7 * 6 * 5, dtype=np.uint8)
    solid[[9, 10, 16, 52, 53, 101, 150, 151]] = 0
    out["chunks3d"] = (geo(3, (7, 6, 5), (0.21e-6, 0.18e-6, 0.15e-6),
                           [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_DIFFUSE, I.BC_DIFFUSE, I.BC_PERIODIC,
                            I.BC_PERIODIC], pdT=(1.0, 0, 0), solid=solid),
                       mat(I.bands(rng, 6, 1e-12, 1e-9), 3, 4), None, rng.uniform(0, 1e11, 210))
    return out


CASES = list(adjoint_cases().keys())


def dev(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


_REF = {}


def oracle_grad(name):
    if name not in _REF:
        g, m, P, gam = adjoint_cases()[name]
        case = O.Case(g, m, P=P, gamma=gam)
        e, _ = O.steady(case, scheme=1, tol_T=1e-15, tol_q=1e-15, max_iter=20000, cg_rtol=1e-14)
        _, grad = steady_adjoint(case, e, keff_weights(case))
        _REF[name] = grad
    return _REF[name]


def gpu_grad(B, name, prec, scheme=1, tol=1e-13):
    g, m, P, gam = adjoint_cases()[name]
    prob = B.Problem(g, m, dict(precision=prec, scheme=scheme, limiter=B.LIM_NONE, adjoint=True,
                                residual_temp=1e-14 if prec == B.F64 else 1e-7,
                                residual_flux=1e-13 if prec == B.F64 else 1e-6,
                                max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000))
    prob.set_fields(dev(P), dev(gam))
    e = prob.zeros()
    prob.steady_solve(e, init=True, allow_not_converged=(prec == B.F32))
    prob.set_control(precision=prec, scheme=scheme, limiter=B.LIM_NONE, adjoint=True, residual_temp=tol,
                     max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
    grad, st = prob.adjoint(e, allow_not_converged=(prec == B.F32))
    torch.cuda.synchronize()
    return host(grad), st, prob


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("scheme", [1, 0])
def test_adjoint_fp64_matches_oracle(B, name, scheme):
    ref = oracle_grad(name)
    grad, st, _ = gpu_grad(B, name, B.F64, scheme=scheme)
    assert st["converged"], st
    print(name, scheme, "adjoint sweeps", st["iters"], "residual", st["eps_T"])
    assert rel_err(grad, ref) < 1e-11, (rel_err(grad, ref), st)
    g, m, P, gam = adjoint_cases()[name]
    if g.get("solid") is not None:
        assert np.all(grad[np.asarray(g["solid"]) == 0] == 0.0)


def test_adjoint_synthetic_needs_fewer_sweeps(B):
    _, st1, _ = gpu_grad(B, "thermal2d", B.F64, scheme=1, tol=1e-10)
    _, st0, _ = gpu_grad(B, "thermal2d", B.F64, scheme=0, tol=1e-10)
    assert st1["iters"] <= st0["iters"], (st1["iters"], st0["iters"])


@pytest.mark.parametrize("name", ["specular2d", "box3d", "chunks3d"])
def test_adjoint_fp32_matches_oracle(B, name):
    ref = oracle_grad(name)
    grad, st, _ = gpu_grad(B, name, B.F32, tol=1e-6)
    assert rel_err(grad, ref) < 1e-5, (rel_err(grad, ref), st)


def test_adjoint_argument_errors(B):
    g, m, P, gam = adjoint_cases()["periodic2d"]
    prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_NONE))   # no adjoint workspace
    e = prob.zeros()
    with pytest.raises(B.BteError, match="STATE"):
        prob.adjoint(e)
    prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_MC, adjoint=True))
    with pytest.raises(B.BteError, match="UNSUPPORTED"):
        prob.adjoint(prob.zeros())
    g2 = dict(g, pdT=[0.0, 0.0, 0.0])
    prob = B.Problem(g2, m, dict(precision=B.F64, limiter=B.LIM_NONE, adjoint=True))
    with pytest.raises(B.BteError, match="ARG"):
        prob.adjoint(prob.zeros())


def test_two_forwards_then_one_backward(B):
    """k(gamma_1) - k(gamma_2) from two KeffSteady forwards on one problem,
    then one backward: each gradient is the adjoint at its own fields
    (the backward re-applies the forward's gamma before the adjoint)."""
    g, m, P, gam = adjoint_cases()["periodic2d"]
    ctl = dict(precision=B.F64, scheme=B.SYNTHETIC, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-13,
               residual_flux=1e-12, max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
    prob = B.Problem(g, m, ctl)
    g1 = dev(gam).requires_grad_(True)
    g2 = dev(3.0 * gam + 2e10).requires_grad_(True)
    k1 = B.KeffSteady.apply(g1, prob, None)
    k2 = B.KeffSteady.apply(g2, prob, None)
    (k1 - k2).sum().backward()
    ref = []
    for gg in (gam, 3.0 * gam + 2e10):
        one = B.Problem(g, m, ctl)
        one.set_fields(None, dev(gg))
        e = one.zeros()
        one.steady_solve(e, init=True)
        grad, st = one.adjoint(e)
        assert st["converged"], st
        ref.append(host(grad))
    err1 = rel_err(host(g1.grad), ref[0])
    err2 = rel_err(host(g2.grad), -ref[1])
    assert max(err1, err2) < 1e-11, (err1, err2)
    # the two fields give clearly different gradients, so a mix-up would show
    assert rel_err(ref[0], ref[1]) > 1e-2
