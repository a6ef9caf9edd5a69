"""Tile shapes of the LDS-tile kernels: every candidate shape gives the
oracle's results (sweep iterates in 1D and 3D, explicit steps in 1D and 2D,
the steady adjoint gradient in 3D and the transient adjoint in 2D), and the
autotuner times every candidate and keeps one.

The shape only changes how the same arithmetic is blocked: bars as in the
other parity tests (FP64 1e-10 on iterates, 1e-11 on steps, 1e-9 on
gradients; FP32 1e-5 on steps)."""
import numpy as np
import pytest

import oracle as O
from oracle.adjoint import transient_adjoint
from tests.helpers import rel_err, small_cases
from tests.test_gpu_adjoint import adjoint_cases, oracle_grad
from tests.test_gpu_parity import build, dev, host, seeded_e, to_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def candidates(B, name, prec, kind):
    _, prob = build(B, name, prec)
    return prob.tile_candidates(kind)


@pytest.mark.parametrize("name,prec,lim", [("box3d", 1, O.LIM_NONE), ("slab1d", 1, O.LIM_NONE),
                                            ("walls2d", 1, O.LIM_NONE), ("periodic2d", 1, O.LIM_NONE),
                                            ("walls2d", 0, O.LIM_MC), ("periodic2d", 0, O.LIM_MINMOD)])
def test_sweep_tiles_match_oracle(B, name, prec, lim):
    """Every sweep candidate: LDS tiles in 1D, column segments in 3D, in 2D
    the register tile with each number of rows per wavefront (per-diagonal
    launches and one launch per sweep) and the LDS tiles (walls2d has ragged
    8 x 8 tiles, every wall kind and pores)."""
    shapes = [(B.TUNE_SWEEP, t) for t in candidates(B, name, prec, B.TUNE_SWEEP)]
    assert len(shapes) >= 3
    shapes += [(B.TUNE_SWEEP_ONE_LAUNCH, t) for t in candidates(B, name, prec, B.TUNE_SWEEP_ONE_LAUNCH)]
    assert (len(shapes) > len(candidates(B, name, prec, B.TUNE_SWEEP))) == name.endswith("2d")
    eo = None
    for kind, tile in shapes:
        case, prob = build(B, name, prec, limiter=lim, scheme=1, max_iter=3, residual_temp=0.0, residual_flux=0.0,
                           cg_rtol=1e-13, cg_max_iter=20000)
        prob.set_tiles(kind, tile)
        e = seeded_e(case, 4)
        eg = to_gpu(prob, e)
        e = host(eg)
        st = prob.steady_solve(eg, init=False, allow_not_converged=True)
        assert st["iters"] == 3
        if name.endswith("2d"):   # more than one tile diagonal in these films
            assert (st["sweep_launches"] == 3) == (kind == B.TUNE_SWEEP_ONE_LAUNCH)
        if eo is None:
            eo, _ = O.steady(case, scheme=1, tol_T=0.0, tol_q=0.0, max_iter=3, cg_rtol=1e-13, cg_maxit=20000,
                             e=e.copy())
        err = rel_err(host(eg), eo)
        print(name, prec, lim, kind, tile, err)
        assert err < (1e-11 if prec == 1 else 1e-5), (kind, tile, err)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", ["walls2d", "periodic2d", "slab1d"])
def test_transient_tiles_match_oracle(B, name, prec):
    shapes = candidates(B, name, prec, B.TUNE_TRANSIENT)
    assert len(shapes) >= 2
    dt = 0.05e-12 if name == "slab1d" else 0.2e-12
    pulse = (1e-12, 2e-12)
    eo = None
    for tile in shapes:
        case, prob = build(B, name, prec, limiter=O.LIM_MC, dt=dt)
        prob.set_tiles(B.TUNE_TRANSIENT, tile)
        e = seeded_e(case, 3)
        eg = to_gpu(prob, e)
        e = host(eg)
        prob.transient_step(eg, 5, 0.0, pulse)
        if eo is None:
            eo, _ = O.transient(case, e.copy(), 5, dt, 0.0, pulse)
        err = rel_err(host(eg), eo)
        print(name, prec, tile, err)
        assert err < (1e-11 if prec == 1 else 1e-5), (tile, err)


def test_adjoint_sweep_tiles_match_oracle(B):
    ref = oracle_grad("box3d")
    g, m, P, gam = adjoint_cases()["box3d"]
    for tile in candidates(B, "box3d", 1, B.TUNE_SWEEP)[:4]:
        prob = B.Problem(g, m, dict(precision=B.F64, scheme=1, limiter=B.LIM_NONE, adjoint=True,
                                    residual_temp=1e-14, residual_flux=1e-13, max_iter=20000, cg_rtol=1e-12,
                                    cg_max_iter=5000))
        prob.set_tiles(B.TUNE_SWEEP, tile)
        prob.set_fields(dev(P), dev(gam))
        e = prob.zeros()
        prob.steady_solve(e, init=True)
        prob.set_control(precision=B.F64, scheme=1, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-13,
                         max_iter=20000, cg_rtol=1e-12, cg_max_iter=5000)
        grad, st = prob.adjoint(e)
        err = rel_err(host(grad), ref)
        print(tile, err, st["iters"])
        assert err < 1e-11, (tile, err)


def test_transient_adjoint_tiles_match_oracle(B):
    g, m, P, gam = small_cases()["walls2d"]
    rng = np.random.default_rng(8)
    w = rng.uniform(0, 1, 143) * (np.asarray(g["solid"]) > 0)
    dt, n = 0.2e-12, 12
    case = O.Case(g, m, P=P, gamma=gam)
    Jr, gr = transient_adjoint(case, case.zeros(), n, dt, 0.0, None, w)
    shapes = None
    for i in range(8):
        prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_NONE, dt=dt, adjoint=True))
        shapes = shapes or prob.tile_candidates(B.TUNE_TRANSIENT)
        if i >= len(shapes):
            break
        prob.set_tiles(B.TUNE_TRANSIENT, shapes[i])
        prob.set_fields(dev(P), dev(gam))
        J, grad, _ = prob.transient_adjoint(prob.zeros(), n, dev(w), 0.0, None, every=5)
        err = rel_err(host(grad), gr)
        print(shapes[i], err)
        assert abs(J - Jr) <= 1e-12 * abs(Jr) and err < 1e-11, (shapes[i], err)


@pytest.mark.parametrize("name", ["box3d", "walls2d"])
@pytest.mark.parametrize("prec", [1, 0])
def test_autotune_keeps_one_candidate(B, prec, name):
    case, prob = build(B, name, prec, scheme=1, max_iter=3, residual_temp=0.0, residual_flux=0.0,
                       cg_rtol=1e-13, cg_max_iter=20000)
    kinds = (B.TUNE_SWEEP, B.TUNE_SWEEP_ONE_LAUNCH)
    shapes = [(k, t) for k in kinds for t in prob.tile_candidates(k)]
    ent = prob.autotune(reps=2)
    # the two sweep kinds are one choice: shape and launch form
    sweep = [x for x in ent if x["kind"] in kinds]
    assert [(x["kind"], x["tile"]) for x in sweep] == shapes
    assert sum(x["chosen"] for x in sweep) == 1 and all(x["ms"] > 0 for x in sweep)
    best = min(sweep, key=lambda x: x["ms"])
    assert best["chosen"]
    # the problem still solves with the kept shape
    e = seeded_e(case, 4)
    eg = to_gpu(prob, e)
    e = host(eg)
    st = prob.steady_solve(eg, init=False, allow_not_converged=True)
    if name.endswith("2d"):
        assert (st["sweep_launches"] == 3) == (best["kind"] == B.TUNE_SWEEP_ONE_LAUNCH)
    eo, _ = O.steady(case, scheme=1, tol_T=0.0, tol_q=0.0, max_iter=3, cg_rtol=1e-13, cg_maxit=20000, e=e.copy())
    err = rel_err(host(eg), eo)
    assert err < (1e-11 if prec == 1 else 1e-5), err


def test_set_tiles_rejects_non_candidates(B):
    _, prob = build(B, "box3d", 0)
    with pytest.raises(RuntimeError):
        prob.set_tiles(B.TUNE_SWEEP, (5, 5, 5))
    with pytest.raises(RuntimeError):
        prob.set_tiles(B.TUNE_SWEEP, (16, 4, 1))
