"""HIP graphs of the steady iteration give the same results as plain
launches: the sweep graphs (one per buffer parity) and the CG graph are
replayed every source iteration, with the host's convergence check and
synchronisation between replays; the final fields must be bitwise equal to
those of the same solve with plain launches.

The one-launch form of the two-dimensional sweep (bte_set_persistent: one
launch per sweep whose blocks take the items in sweep order by ticket and
wait for the items of their upwind tiles) does the same arithmetic as the
launch-per-diagonal form: its fields are bitwise equal to those, with and
without graphs, for every rows-per-wavefront variant, batches with
per-geometry masks included."""
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


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_queue_sweep_square_every_row_split(B, prec):
    # 64 x 64 cells: 64 tiles x 4 quadrants x 10 chunks = 2560 items in one
    # launch, for each number of tile rows per wavefront
    cfg = I.square2d_source_case(n=64)
    p = B.F32 if prec == "f32" else B.F64
    shapes = [(8, 8, 2), (8, 8, 1)] + ([(8, 8, 4)] if p == B.F32 else [])
    for tile in shapes:
        out = []
        for persistent in (False, True):
            prob = B.Problem(cfg["geometry"], cfg["material"], dict(precision=p, scheme=B.SYNTHETIC,
                                                                    limiter=B.LIM_NONE, residual_temp=0.0,
                                                                    residual_flux=0.0, max_iter=12, cg_rtol=1e-10,
                                                                    cg_max_iter=30))
            prob.set_tiles(B.TUNE_SWEEP, tile)
            prob.set_persistent(persistent)
            prob.set_fields(dev(cfg["P"]), None)
            e = prob.zeros()
            st = prob.steady_solve(e, init=True, allow_not_converged=True)
            assert st["iters"] == 12
            assert st["sweep_launches"] == (12 if persistent else 12 * 15)
            out.append(e.cpu().numpy())
        print(prec, tile, "equal", np.array_equal(out[0], out[1]))
        assert np.array_equal(out[0], out[1]), tile


def test_queue_sweep_batch_with_masks(B):
    cfg = I.porous2d_batch_case(seed=5, n_films=5, sides=(16, 24, 32), n_bands=4, n_theta=1, n_phi=2)
    films, mat = cfg["films"], cfg["material"]
    a, sa = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, True, 40, persistent=False)
    b, sb = solve(B, films, mat, None, None, B.F32, B.LIM_MINMOD, True, 40, persistent=True)
    assert sa["iters"] == sb["iters"] and sa["updates"] == sb["updates"]
    assert np.array_equal(a, b)


def test_one_launch_sweep_is_refused_in_3d(B):
    g, m, P, gam = small_cases()["box3d"]
    prob = B.Problem(g, m, dict(precision=B.F32))
    prob.set_persistent(False)
    with pytest.raises(RuntimeError):
        prob.set_persistent(True)
