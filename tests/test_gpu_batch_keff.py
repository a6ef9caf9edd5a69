"""GPU parity of k_eff (single and batched geometries) and of the adjoint
gradient behind torch.autograd against central finite differences.

k_eff = (L_x / dT_x) (1/N_cells) sum_solid q_x (pores count as zero).  A
batch of porous films is solved in one problem (one sweep launch per tile
diagonal covers every film) and each film's k_eff is compared with the
oracle's solve of that film alone.
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def dev(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def small_batch():
    return I.porous2d_batch_case(seed=5, n_films=6, sides=(16, 24, 32), n_bands=4, n_theta=1, n_phi=2)


_REF = {}


def oracle_keff(geo, mat, gamma=None, limiter=O.LIM_NONE):
    case = O.Case(geo, mat, gamma=gamma, limiter=limiter)
    e, st = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e-12, max_iter=5000, cg_rtol=1e-14)
    assert st["converged"], st
    return O.keff(case, e)


@pytest.mark.parametrize("prec,lim", [("f64", "none"), ("f32", "none"), ("f64", "mc"), ("f32", "mc"),
                                      ("f64", "minmod"), ("f32", "minmod")])
def test_batched_films_keff_matches_oracle(B, prec, lim):
    cfg = small_batch()
    films, mat = cfg["films"], cfg["material"]
    p = B.F64 if prec == "f64" else B.F32
    gl, ol = {"none": (B.LIM_NONE, O.LIM_NONE), "mc": (B.LIM_MC, O.LIM_MC),
              "minmod": (B.LIM_MINMOD, O.LIM_MINMOD)}[lim]
    prob = B.Problem(films, mat, dict(precision=p, scheme=B.SYNTHETIC, limiter=gl,
                                      residual_temp=2e-13 if p == B.F64 else 1e-7,
                                      residual_flux=2e-12 if p == B.F64 else 1e-6,
                                      max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000))
    e = prob.zeros()
    st = prob.steady_solve(e, init=True, allow_not_converged=(p == B.F32))
    k = prob.keff(e).cpu().numpy()
    if lim not in _REF:
        _REF[lim] = np.array([oracle_keff(g, mat, limiter=ol) for g in films])
    ref = _REF[lim]
    print(prec, "iters", st["iters"], "updates", st["updates"], "k_eff", k, "oracle", ref)
    # converged films leave the sweep: never more updates than every film for every iteration
    assert 0 < st["updates"] <= prob.n_unknowns * st["iters"]
    tol = 1e-11 if p == B.F64 else 1e-5
    assert np.all(np.abs(k - ref) <= tol * np.abs(ref)), (k, ref, np.abs(k / ref - 1).max())


def test_batched_equals_separate_solves(B):
    """The batch couples nothing: each film's field equals its own solve."""
    cfg = small_batch()
    films, mat = cfg["films"][:3], cfg["material"]
    ctl = dict(precision=B.F64, scheme=B.SYNTHETIC, limiter=B.LIM_NONE, residual_temp=1e-12,
               residual_flux=1e-11, max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
    prob = B.Problem(films, mat, ctl)
    e = prob.zeros()
    prob.steady_solve(e, init=True)
    T, _, q = prob.moments(e)
    off = 0
    for g in films:
        one = B.Problem(g, mat, ctl)
        e1 = one.zeros()
        one.steady_solve(e1, init=True)
        T1, _, q1 = one.moments(e1)
        n = one.n_cells
        errs = (rel_err(T[off:off + n].cpu().numpy(), T1.cpu().numpy(), 300.0),
                rel_err(q[off:off + n].cpu().numpy(), q1.cpu().numpy()))
        assert max(errs) < 1e-11, errs
        off += n


def test_keff_bulk_closed_form(B):
    """Pore-free periodic film: k_eff = sum C v^2 tau M_xx exactly."""
    b = dict(C=np.array([7e5, 9e5]), v=np.array([5000.0, 2000.0]), tau=np.array([2e-12, 3e-10]))
    g = dict(dim=2, n=[12, 10, 1], len=[120e-9, 100e-9, 1.0], bc=[I.BC_PERIODIC] * 4 + [I.BC_SPECULAR] * 2,
             bcT=[300.0] * 6, pdT=[1.0, 0.0, 0.0], solid=None, pore_bc=I.BC_DIFFUSE)
    m = dict(b, n_theta=2, n_phi=2, Tref=300.0)
    prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_NONE, residual_temp=1e-13, residual_flux=1e-12,
                                max_iter=5000, cg_rtol=1e-12))
    e = prob.zeros()
    prob.steady_solve(e, init=True)
    k = prob.keff(e).item()
    case = O.Case(g, m)
    Mxx = (case.w * case.s[:, 0] ** 2).sum() / (4 * np.pi)
    expect = (b["C"] * b["v"] ** 2 * b["tau"]).sum() * Mxx
    assert abs(k / expect - 1) < 1e-10, (k, expect)


def test_autograd_gradient_matches_central_differences(B):
    """KeffSteady backward (adjoint) against central differences of the GPU
    k_eff on a small porous 3D cube (h = 1e-4 relative, FP64)."""
    cfg = I.porous3d_adjoint_case(seed=9, n=10, n_bands=4, n_theta=1, n_phi=2)
    g, m, gam0 = cfg["geometry"], cfg["material"], cfg["gamma"]
    ctl = dict(precision=B.F64, scheme=B.SYNTHETIC, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-13,
               residual_flux=1e-12, max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
    prob = B.Problem(g, m, ctl)
    gamma = dev(gam0).requires_grad_(True)
    k = B.KeffSteady.apply(gamma, prob, None)
    k.sum().backward()
    grad = gamma.grad.cpu().numpy()
    solid = np.asarray(g["solid"]).astype(bool)
    assert np.all(grad[~solid] == 0.0)
    rng = np.random.default_rng(3)
    cells = rng.choice(np.flatnonzero(solid), 5, replace=False)
    for c in cells:
        h = 1e-4 * max(gam0[c], 1e10)
        ks = []
        for sg in (1, -1):
            g2 = gam0.copy()
            g2[c] += sg * h
            prob.set_fields(None, dev(g2))
            e = prob.zeros()
            prob.steady_solve(e, init=True)
            ks.append(prob.keff(e).item())
        fd = (ks[0] - ks[1]) / (2 * h)
        print("cell", c, "fd", fd, "adjoint", grad[c])
        assert abs(fd - grad[c]) <= 1e-5 * np.abs(grad).max(), (c, fd, grad[c])
