"""HIP graphs of the steady iteration give the same results as plain
launches: the sweep graphs (one per buffer parity) and the CG graph are
replayed every source iteration, with the host's convergence check and
synchronisation between replays; the final fields must be bitwise equal to
those of the same solve with plain launches.

The tests of the work-queue form of the two-dimensional sweep (one launch
whose blocks take the tiles in diagonal order and wait for their upwind
tiles) are skipped: that form hung its first GPU run and was taken out; the
entry point that selects it now refuses."""
import numpy as np
import pytest

import bte_inputs as I
from tests.helpers import small_cases

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


def solve(B, geo, mat, P, gam, prec, lim, graphs, cg_max_iter, persistent=None, max_iter=400):
    prob = B.Problem(geo, mat, dict(precision=prec, scheme=B.SYNTHETIC, limiter=lim, residual_temp=1e-9,
                                    residual_flux=1e-8, max_iter=max_iter, cg_rtol=1e-10, cg_max_iter=cg_max_iter))
    prob.set_graphs(graphs)
    if persistent is not None:
        prob.set_persistent(persistent)
    prob.set_fields(dev(P), dev(gam))
    e = prob.zeros()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    return e.cpu().numpy(), st


@pytest.mark.parametrize("name", ["walls2d", "periodic2d", "box3d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replays_equal_plain_launches(B, name, prec):
    cases = small_cases()
    if name not in cases:
        pytest.skip("case not defined")
    g, m, P, gam = cases[name]
    p = B.F64 if prec == "f64" else B.F32
    a, sa = solve(B, g, m, P, gam, p, B.LIM_NONE, False, 30)
    b, sb = solve(B, g, m, P, gam, p, B.LIM_NONE, True, 30)
    assert sa["iters"] == sb["iters"] and sa["iters"] > 2
    assert np.array_equal(a, b)


def test_graph_batch_with_masks_equals_plain_launches(B):
    cfg = I.porous2d_batch_case(seed=5, n_films=5, sides=(16, 24, 32), n_bands=4, n_theta=1, n_phi=2)
    films, mat = cfg["films"], cfg["material"]
    a, sa = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, False, 40)
    b, sb = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, True, 40)
    assert sa["iters"] == sb["iters"] and sa["updates"] == sb["updates"]
    assert np.array_equal(a, b)


QUEUE_SKIP = pytest.mark.skip(reason="the work-queue sweep hung its first GPU run (a steady solve of walls2d "
                                     "timed out); it was taken out and bte_set_persistent(1) refuses")


@QUEUE_SKIP
@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("lim", ["none", "mc"])
@pytest.mark.parametrize("name", ["walls2d", "periodic2d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_queue_sweep_equals_diagonal_launches(B, name, prec, lim, graphs):
    g, m, P, gam = small_cases()[name]
    p = B.F64 if prec == "f64" else B.F32
    L = B.LIM_NONE if lim == "none" else B.LIM_MC
    a, sa = solve(B, g, m, P, gam, p, L, graphs, 30, persistent=False, max_iter=60)
    b, sb = solve(B, g, m, P, gam, p, L, graphs, 30, persistent=True, max_iter=60)
    assert sa["iters"] == sb["iters"] and sa["iters"] > 2
    assert sb["sweep_launches"] == sb["iters"]
    assert np.array_equal(a, b)


@QUEUE_SKIP
def test_queue_sweep_many_items_per_block(B):
    # 64 x 64 cells: 64 tiles x 4 octants x 10 chunks = 2560 items, several
    # per resident block of the queue launch
    cfg = I.square2d_source_case(n=64)
    for prec in (B.F32, B.F64):
        a, sa = solve(B, cfg["geometry"], cfg["material"], cfg["P"], None, prec, B.LIM_NONE, True, 30,
                      persistent=False, max_iter=12)
        b, sb = solve(B, cfg["geometry"], cfg["material"], cfg["P"], None, prec, B.LIM_NONE, True, 30,
                      persistent=True, max_iter=12)
        assert sa["iters"] == sb["iters"] == 12
        assert np.array_equal(a, b)


@QUEUE_SKIP
def test_queue_sweep_batch_with_masks(B):
    cfg = I.porous2d_batch_case(seed=5, n_films=5, sides=(16, 24, 32), n_bands=4, n_theta=1, n_phi=2)
    films, mat = cfg["films"], cfg["material"]
    a, sa = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, True, 40, persistent=False)
    b, sb = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, True, 40, persistent=True)
    assert sa["iters"] == sb["iters"] and sa["updates"] == sb["updates"]
    assert np.array_equal(a, b)


def test_work_queue_sweep_is_refused(B):
    g, m, P, gam = small_cases()["walls2d"]
    prob = B.Problem(g, m, dict(precision=B.F32))
    prob.set_persistent(False)
    with pytest.raises(RuntimeError):
        prob.set_persistent(True)
