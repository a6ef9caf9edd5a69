"""GPU parity for two-dimensional materials (in-plane directions, total
angle 2 pi; Sec. 2.1 and Sec. 5 MaterialDimension) through the C ABI,
against the FP64 oracle on the same seeded inputs: moments, residual (three
limiters), explicit steps, converged steady solves (both schemes), the
steady adjoint d k_eff / d gamma and the checkpointed transient adjoint, on
a slab and on 2D geometries with every wall kind, pores and a periodic axis
with a temperature drop; and the paper-size transient grating against the
exact Fourier-mode recurrence with Omega = 2 pi.

Bars as in the bulk parity tests: FP64 1e-11 (steady 1e-10, adjoint 1e-9),
FP32 storage 1e-5 (residual 2e-5, steady 1e-5 in T and T_L, 1e-4 in q).
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from oracle.adjoint import keff_weights, steady_adjoint, transient_adjoint
from tests.helpers import geo, mat, rel_err, ttg_discrete_mode

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def mat2(b, nt):
    m = mat(b, nt, 1)
    m["material_dim"] = 2
    return m


def cases():
    rng = np.random.default_rng(202)
    b = I.bands(rng, 4, 1e-12, 1e-9)
    out = {}
    out["slab1d"] = (geo(1, (40,), (80e-9,), [I.BC_THERMAL, I.BC_THERMAL] + [I.BC_SPECULAR] * 4,
                         bcT=[301.0, 299.0, 300, 300, 300, 300]),
                     mat2(b, 8), rng.uniform(0, 1e17, 40), rng.uniform(0, 1e11, 40))
    solid = np.ones(11 * 9, dtype=np.uint8)
    solid[[24, 25, 35, 36, 70]] = 0
    out["walls2d"] = (geo(2, (11, 9), (110e-9, 90e-9),
                          [I.BC_THERMAL, I.BC_DIFFUSE, I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_SPECULAR, I.BC_SPECULAR],
                          bcT=[300.5] * 6, solid=solid),
                      mat2(b, 3), rng.uniform(0, 1e17, 99), rng.uniform(0, 1e11, 99))
    solid = np.ones(10 * 8, dtype=np.uint8)
    solid[[22, 23, 55]] = 0
    out["periodic2d"] = (geo(2, (10, 8), (100e-9, 80e-9),
                             [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_THERMAL, I.BC_DIFFUSE, I.BC_SPECULAR,
                              I.BC_SPECULAR], bcT=[300, 300, 300.2, 300, 300, 300], pdT=(0.8, 0, 0),
                             solid=solid),
                         mat2(b, 5), rng.uniform(0, 1e17, 80), rng.uniform(0, 1e11, 80))
    return out


CASES = list(cases().keys())


def dev(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def build(B, name, prec, limiter=O.LIM_NONE, **ctl):
    g, m, P, gam = cases()[name]
    case = O.Case(g, m, P=P, gamma=gam, limiter=limiter)
    control = dict(precision=prec, limiter=limiter)
    control.update(ctl)
    prob = B.Problem(g, m, control)
    prob.set_fields(dev(P), dev(gam))
    return case, prob


def seeded_e(case, seed):
    rng = np.random.default_rng(seed)
    T = rng.uniform(-1, 1, case.nc)
    e = (case.C[None, None, :] * T[:, None, None] / (2 * np.pi)) * np.ones((1, case.na, 1))
    e = e + 0.05 * np.abs(e).max() * rng.normal(size=e.shape)
    if case.solid is not None:
        e[case.solid == 0] = 0.0
    return e.reshape(-1)


def to_gpu(prob, e):
    return torch.as_tensor(np.asarray(e), device="cuda").to(prob.dtype).contiguous()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", CASES)
def test_moments(B, name, prec):
    case, prob = build(B, name, prec)
    eg = to_gpu(prob, np.random.default_rng(1).normal(size=case.size) * 10.0)
    e = host(eg)
    T, TL, q = prob.moments(eg)
    To, TLo, qo = O.moments(case, e)
    assert rel_err(host(T), To, 300) < 1e-12
    assert rel_err(host(TL), TLo, 300) < 1e-12
    assert rel_err(host(q), qo) < 1e-12


@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC, O.LIM_MINMOD])
@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", CASES)
def test_residual(B, name, prec, lim):
    case, prob = build(B, name, prec, limiter=lim)
    eg = to_gpu(prob, seeded_e(case, 2))
    e = host(eg)
    R = host(prob.residual(eg))
    err = rel_err(R, O.residual(case, e))
    assert err < (1e-11 if prec == 1 else 1e-5), (name, lim, err)


@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC])
@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", CASES)
def test_transient_steps(B, name, prec, lim):
    dt = 0.05e-12 if name == "slab1d" else 0.2e-12
    case, prob = build(B, name, prec, limiter=lim, dt=dt)
    eg = to_gpu(prob, seeded_e(case, 3))
    e = host(eg)
    pulse = (1e-12, 2e-12)
    prob.transient_step(eg, 7, 0.0, pulse)
    eo, _ = O.transient(case, e.copy(), 7, dt, 0.0, pulse)
    assert rel_err(host(eg), eo) < (1e-11 if prec == 1 else 1e-5)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", CASES)
def test_steady_converged(B, name, prec, scheme):
    tolT = 2e-13 if prec == 1 else 1e-7
    case, prob = build(B, name, prec, scheme=scheme, max_iter=8000, residual_temp=tolT, residual_flux=tolT * 10,
                       cg_rtol=1e-12)
    eg = prob.zeros()
    st = prob.steady_solve(eg, init=True)
    assert st["converged"]
    eo, _ = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e-13, max_iter=20000, cg_rtol=1e-13)
    T, TL, q = prob.moments(eg)
    To, TLo, qo = O.moments(case, eo)
    tol = 1e-11 if prec == 1 else 1e-5
    errs = (rel_err(host(T), To, 300), rel_err(host(TL), TLo, 300), rel_err(host(q), qo))
    print(name, prec, scheme, "steady T, T_L, q rel err", errs, "iters", st["iters"])
    assert max(errs) < tol, (name, prec, scheme, errs)


def test_keff_and_steady_adjoint(B):
    """k_eff of the periodic film and d k_eff / d gamma (FP64) against the
    oracle's forward solve and GMRES adjoint."""
    name = "periodic2d"
    g, m, P, gam = cases()[name]
    case = O.Case(g, m, P=P, gamma=gam)
    e, _ = O.steady(case, scheme=1, tol_T=1e-15, tol_q=1e-15, max_iter=20000, cg_rtol=1e-14)
    _, grad_ref = steady_adjoint(case, e, keff_weights(case))
    prob = B.Problem(g, m, dict(precision=B.F64, scheme=1, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-14,
                                residual_flux=1e-13, max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000))
    prob.set_fields(dev(P), dev(gam))
    eg = prob.zeros()
    prob.steady_solve(eg, init=True)
    k = prob.keff(eg).item()
    assert abs(k - O.keff(case, e)) < 1e-11 * abs(O.keff(case, e)), (k, O.keff(case, e))
    prob.set_control(precision=B.F64, scheme=1, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-13,
                     max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
    grad, st = prob.adjoint(eg)
    assert st["converged"], st
    assert rel_err(host(grad), grad_ref) < 1e-11, rel_err(host(grad), grad_ref)


@pytest.mark.parametrize("name", ["walls2d", "periodic2d", "slab1d"])
def test_transient_adjoint(B, name):
    g, m, P, gam = cases()[name]
    case = O.Case(g, m, P=P, gamma=gam)
    w = np.random.default_rng(5).uniform(0, 1, case.nc)
    if case.solid is not None:
        w = w * (case.solid > 0)
    dt = 0.05e-12 if name == "slab1d" else 0.2e-12
    n, pulse = 12, (1e-12, 2e-12)
    J_ref, grad_ref = transient_adjoint(case, case.zeros(), n, dt, 0.0, pulse, w)
    prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_NONE, dt=dt, adjoint=True))
    prob.set_fields(dev(P), dev(gam))
    J, grad, st = prob.transient_adjoint(prob.zeros(), n, dev(w), 0.0, pulse, every=5)
    assert abs(J - J_ref) < 1e-11 * max(abs(J_ref), 1e-300)
    assert rel_err(grad.cpu().numpy(), grad_ref) < 1e-11, rel_err(grad.cpu().numpy(), grad_ref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ttg_paper_size_against_mode_recurrence(B, prec):
    cfg = I.ttg(1.0)
    m = dict(cfg["material"], material_dim=2)
    p = B.F64 if prec == "f64" else B.F32
    prob = B.Problem(cfg["geometry"], m, dict(precision=p, limiter=B.LIM_NONE, dt=cfg["dt"]))
    prob.set_fields(None, None)
    case = O.Case(cfg["geometry"], m)
    c = m["C"][0]
    e0 = (c * (cfg["T0"] - 300.0) / (2 * np.pi))[:, None] * np.ones(case.na)[None, :]
    e = torch.as_tensor(e0.reshape(-1), device="cuda").to(prob.dtype)
    n = int(round(1.0 * cfg["tau"] / cfg["dt"]))
    prob.transient_step(e, n)
    T, _, _ = prob.moments(e)
    ref = ttg_discrete_mode(case.s[:, 0], case.w, m["v"][0], cfg["tau"], 1000, 1e-6, cfg["dt"], n, c,
                            cfg["amplitude"], omega=2 * np.pi)
    err = float(np.abs(T.cpu().numpy() - 300.0 - ref).max())
    print(prec, "2D-material grating, steps", n, "err", err)
    assert err < (1e-11 if prec == "f64" else 1e-5) * cfg["amplitude"], err


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batched_films_keff(B, prec):
    """A batch of porous films of a two-dimensional material: k_eff of every
    film against the oracle's own solve of that film."""
    cfg = I.porous2d_batch_case(seed=5, n_films=4, sides=(16, 24), n_bands=4, n_theta=2, n_phi=1)
    films, m = cfg["films"], dict(cfg["material"], material_dim=2)
    p = B.F64 if prec == "f64" else B.F32
    prob = B.Problem(films, m, dict(precision=p, scheme=B.SYNTHETIC, limiter=B.LIM_NONE,
                                    residual_temp=1e-12 if p == B.F64 else 1e-7,
                                    residual_flux=1e-11 if p == B.F64 else 1e-6,
                                    max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000))
    e = prob.zeros()
    prob.steady_solve(e, init=True, allow_not_converged=(p == B.F32))
    k = prob.keff(e).cpu().numpy()
    ref = []
    for g in films:
        case = O.Case(g, m)
        eo, st = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e-12, max_iter=5000, cg_rtol=1e-14)
        assert st["converged"], st
        ref.append(O.keff(case, eo))
    ref = np.array(ref)
    print(prec, "k_eff", k, "oracle", ref)
    tol = 1e-11 if p == B.F64 else 1e-5
    assert np.all(np.abs(k - ref) <= tol * np.abs(ref)), (k, ref, np.abs(k / ref - 1).max())
