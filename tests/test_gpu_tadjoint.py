"""GPU parity of the transient adjoint (checkpointed reverse mode of the
explicit steps) against the oracle's store-all reverse mode, checkpoint
independence, and central differences of J on the GPU.

J = sum_c a_c T_c(e^N) / sum_c a_c after N steps from e0 (limiter NONE).
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from oracle.adjoint import transient_adjoint
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


def dev(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def cases():
    rng = np.random.default_rng(21)
    b = I.bands(rng, 3, 1e-12, 1e-9)
    out = {}
    g = geo(3, (5, 4, 6), (0.25e-6, 0.2e-6, 0.3e-6), [I.BC_THERMAL] * 5 + [I.BC_DIFFUSE])
    wts = np.zeros(120)
    wts[100:] = rng.uniform(0.5, 1.0, 20)            # top layer
    out["laser3d"] = (g, mat(b, 1, 2), rng.uniform(0, 1e18, 120), rng.uniform(0, 1e11, 120), wts,
                      0.5e-12, 24, (4e-12, 4e-12))
    g2, m2, P2, gam2 = small_cases()["walls2d"]
    w2 = rng.uniform(0, 1, 143) * (np.asarray(g2["solid"]) > 0)
    out["walls2d"] = (g2, m2, P2, gam2, w2, 0.2e-12, 20, None)
    g3, m3, _, gam3 = small_cases()["periodic2d"]
    w3 = rng.uniform(0, 1, 90) * (np.asarray(g3["solid"]) > 0)
    out["periodic2d"] = (g3, m3, rng.uniform(0, 1e17, 90), gam3, w3, 0.2e-12, 16, (1e-12, 2e-12))
    # three-dimensional column paths: periodic x / y with pores, specular,
    # diffuse and thermalizing walls; a periodic z axis with pores; a column
    # longer than one 64-cell run of per-cell records
    g4, m4, P4, gam4 = small_cases()["box3d"]
    w4 = rng.uniform(0, 1, 270) * (np.asarray(g4["solid"]) > 0)
    out["box3d"] = (g4, m4, P4, gam4, w4, 0.2e-12, 12, (1e-12, 2e-12))
    solid = np.ones(4 * 3 * 5, dtype=np.uint8)
    solid[[5, 17, 30, 46]] = 0
    g5 = geo(3, (4, 3, 5), (0.2e-6, 0.15e-6, 0.25e-6),
             [I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_THERMAL, I.BC_SPECULAR, I.BC_PERIODIC, I.BC_PERIODIC],
             pdT=(0, 0, 0.4), bcT=[300, 300, 299.5, 300, 300, 300], solid=solid)
    out["zper3d"] = (g5, mat(b, 1, 2), rng.uniform(0, 1e17, 60), rng.uniform(0, 1e11, 60),
                     rng.uniform(0, 1, 60) * solid, 0.2e-12, 10, (1e-12, 2e-12))
    g6 = geo(3, (2, 2, 70), (0.1e-6, 0.1e-6, 3.5e-6),
             [I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_SPECULAR, I.BC_SPECULAR, I.BC_THERMAL, I.BC_DIFFUSE],
             bcT=[300, 300, 300, 300, 300.5, 300])
    out["tall3d"] = (g6, mat(b, 1, 2), rng.uniform(0, 1e17, 280), rng.uniform(0, 1e11, 280),
                     rng.uniform(0, 1, 280), 0.3e-12, 8, (1e-12, 2e-12))
    return out


_REF = {}


def oracle_ref(name):
    if name not in _REF:
        g, m, P, gam, w, dt, n, pulse = cases()[name]
        case = O.Case(g, m, P=P, gamma=gam)
        _REF[name] = transient_adjoint(case, case.zeros(), n, dt, 0.0, pulse, w)
    return _REF[name]


def gpu_run(B, name, prec, every):
    g, m, P, gam, w, dt, n, pulse = cases()[name]
    prob = B.Problem(g, m, dict(precision=prec, limiter=B.LIM_NONE, dt=dt, adjoint=True))
    prob.set_fields(dev(P), dev(gam))
    J, grad, st = prob.transient_adjoint(prob.zeros(), n, dev(w), 0.0, pulse, every=every)
    torch.cuda.synchronize()
    return J, grad.cpu().numpy(), prob


@pytest.mark.parametrize("name", ["laser3d", "walls2d", "periodic2d", "box3d", "zper3d", "tall3d"])
def test_transient_adjoint_fp64_matches_oracle(B, name):
    Jr, gr = oracle_ref(name)
    J, g, _ = gpu_run(B, name, B.F64, every=7)
    assert abs(J - Jr) <= 1e-12 * abs(Jr), (J, Jr)
    assert rel_err(g, gr) < 1e-11, rel_err(g, gr)


@pytest.mark.parametrize("name", ["laser3d", "box3d"])
def test_transient_adjoint_fp32_matches_oracle(B, name):
    Jr, gr = oracle_ref(name)
    J, g, _ = gpu_run(B, name, B.F32, every=5)
    assert abs(J - Jr) <= 1e-6 * abs(Jr), (J, Jr)
    assert rel_err(g, gr) < 1e-5, rel_err(g, gr)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_checkpoint_interval_does_not_change_the_gradient(B, prec):
    p = B.F64 if prec == "f64" else B.F32
    ref = None
    for every in (1, 5, 24, 100):
        J, g, _ = gpu_run(B, "laser3d", p, every=every)
        if ref is None:
            ref = (J, g)
        else:
            assert J == ref[0]
            assert np.array_equal(g, ref[1]), every


def test_transient_adjoint_against_central_differences(B):
    name = "laser3d"
    g, m, P, gam, w, dt, n, pulse = cases()[name]
    J, grad, prob = gpu_run(B, name, B.F64, every=8)
    for c in (7, 33, 61, 110):
        h = 1e-4 * max(gam[c], 1e10)
        Js = []
        for sg in (1, -1):
            g2 = gam.copy()
            g2[c] += sg * h
            prob.set_fields(dev(P), dev(g2))
            e = prob.zeros()
            prob.transient_step(e, n, 0.0, pulse)
            T, _, _ = prob.moments(e)
            Js.append(float((T.cpu().numpy() * w).sum() / w.sum()))
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(fd - grad[c]) <= 1e-5 * np.abs(grad).max(), (c, fd, grad[c])


def test_autograd_tave_transient(B):
    g, m, P, gam, w, dt, n, pulse = cases()["laser3d"]
    prob = B.Problem(g, m, dict(precision=B.F64, limiter=B.LIM_NONE, dt=dt, adjoint=True))
    gamma = dev(gam).requires_grad_(True)
    J = B.TaveTransient.apply(gamma, prob, dev(P), n, dev(w), 0.0, pulse, 6)
    (2.0 * J).backward()
    Jr, gr = oracle_ref("laser3d")
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    assert rel_err(gamma.grad.cpu().numpy(), 2.0 * gr) < 1e-10
