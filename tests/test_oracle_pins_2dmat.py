"""Pins of the oracle for two-dimensional materials (Sec. 2.1: for a
two-dimensional material the solid angle is replaced by the in-plane polar
angle; Sec. 5, MaterialDimension): directions in the x-y plane, total angle
Omega = 2 pi, e0 = C T_L / 2 pi.  Each test checks the oracle against a
closed form or an independent construction; none re-uses the oracle's
formulas."""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from tests.helpers import geo, mat, ttg_discrete_mode

TWOPI = 2 * np.pi


def mat2(b, n_theta, Tref=300.0):
    m = mat(b, n_theta, 1, Tref)
    m["material_dim"] = 2
    return m


@pytest.mark.parametrize("dim,nt", [(1, 8), (2, 1), (2, 6), (2, 8)])
def test_quadrature_in_plane(dim, nt):
    s, w = O.quadrature(dim, nt, 1, material_dim=2)
    assert len(w) == 2 * nt if dim == 1 else 4 * nt
    assert np.all(w > 0)
    assert abs(w.sum() - TWOPI) < 1e-13
    assert np.all(s[:, 2] == 0.0)
    if dim == 2:
        np.testing.assert_allclose((s ** 2).sum(1), 1.0, atol=1e-15)
        for a in (0, 1):
            m = s.copy()
            m[:, a] *= -1
            # the mirror of every direction is in the set with the same weight
            d = np.abs(m[:, None, :] - s[None, :, :]).sum(2)
            j = d.argmin(1)
            assert np.all(d[np.arange(len(w)), j] < 1e-15)
            np.testing.assert_allclose(w[j], w, rtol=1e-15)
    if dim == 2 and nt == 1:
        # one node per quadrant: the four diagonals, pi/2 each
        np.testing.assert_allclose(np.abs(s[:, :2]), np.sqrt(0.5), atol=1e-15)
        np.testing.assert_allclose(w, np.pi / 2, rtol=1e-15)
    if nt >= 6:
        # second moment of the circle: <s_x^2> = 1/2 (<s_y^2> = 1/2 in 2D)
        assert abs((w * s[:, 0] ** 2).sum() / TWOPI - 0.5) < 1e-13
        # half-range first moment: int_{-pi/2}^{pi/2} cos = 2
        assert abs((w * s[:, 0] * (s[:, 0] > 0)).sum() - 2.0) < 1e-10


def test_three_dimensional_geometry_rejected():
    with pytest.raises(ValueError):
        O.quadrature(3, 2, 2, material_dim=2)


def test_equilibrium_moments_and_fourier_flux():
    """e = C (T - Tref) / 2 pi gives T = T_L = T exactly and no flux; the
    first-order anisotropic part carries q = -(1/2) sum C v^2 tau grad T
    (the in-plane conductivity of a two-dimensional material)."""
    rng = np.random.default_rng(3)
    b = I.bands(rng, 5, 1e-12, 1e-9)
    g = geo(2, (3, 4), (1e-7, 1e-7), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2)
    case = O.Case(g, mat2(b, 8))
    Tst = 300 + rng.uniform(-2, 2, case.nc)
    e = (b["C"][None, None, :] * (Tst - 300)[:, None, None] / TWOPI * np.ones((1, case.na, 1))).reshape(-1)
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(T, Tst, rtol=0, atol=1e-12)
    np.testing.assert_allclose(TL, Tst, rtol=0, atol=1e-12)
    assert np.abs(q).max() < 1e-14 * (b["C"] * b["v"]).sum()
    grad = np.array([2e7, -1e7, 0.0])
    sg = case.s @ grad
    e2 = b["C"][None, :] / TWOPI * (-(b["tau"] * b["v"])[None, :] * sg[:, None])
    e2 = np.broadcast_to(e2, (case.nc, case.na, case.nl)).reshape(-1)
    _, _, q2 = O.moments(case, e2)
    k = (b["C"] * b["v"] ** 2 * b["tau"]).sum()
    np.testing.assert_allclose(q2[0, :2], -0.5 * k * grad[:2], rtol=1e-12)


def test_gray_lattice_equals_local_temperature():
    rng = np.random.default_rng(5)
    b = dict(C=np.array([1.6e6]), v=np.array([3000.0]), tau=np.array([2e-11]))
    g = geo(2, (3, 3), (1e-7, 1e-7), [O.BC_THERMAL] * 4 + [O.BC_SPECULAR] * 2)
    case = O.Case(g, mat2(b, 4))
    e = rng.normal(size=case.size)
    T, TL, _ = O.moments(case, e)
    np.testing.assert_allclose(T, TL, rtol=0, atol=1e-13)


@pytest.mark.parametrize("walls", ["periodic", "specular", "diffuse", "mixed"])
def test_closed_domain_zero_net_flux(walls):
    rng = np.random.default_rng(11)
    b = I.bands(rng, 3, 1e-12, 1e-9)
    bc = {"periodic": [O.BC_PERIODIC] * 4, "specular": [O.BC_SPECULAR] * 4, "diffuse": [O.BC_DIFFUSE] * 4,
          "mixed": [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_DIFFUSE, O.BC_SPECULAR]}[walls] + [O.BC_SPECULAR] * 2
    solid = np.ones(30, dtype=np.uint8)
    solid[[7, 8, 21]] = 0
    g = geo(2, (6, 5), (1e-7, 1.2e-7), bc, solid=solid)
    for lim in (O.LIM_NONE, O.LIM_MC):
        case = O.Case(g, mat2(b, 3), limiter=lim)
        e = rng.normal(size=case.size)
        D = O.flux_div(case, e).reshape(case.nc, case.na, case.nl)
        tot = (case.w[None, :, None] * D).sum()
        scale = (case.w[None, :, None] * np.abs(D)).sum()
        assert abs(tot) < 1e-13 * scale, (walls, lim, tot, scale)


def test_equilibrium_is_fixed_point_with_walls_at_same_temperature():
    rng = np.random.default_rng(2)
    b = I.bands(rng, 4, 1e-12, 1e-9)
    bc = [O.BC_THERMAL, O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_THERMAL, O.BC_SPECULAR, O.BC_SPECULAR]
    g = geo(2, (4, 3), (1e-7, 1e-7), bc, bcT=[302.5] * 6)
    case = O.Case(g, mat2(b, 3))
    e, st = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e30, max_iter=5)
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(T, 302.5, atol=1e-12)
    assert np.abs(q).max() < 1e-13 * (b["C"] * b["v"]).sum() * 2.5
    assert st["iters"] <= 2


@pytest.mark.parametrize("dim", [1, 2])
def test_periodic_bulk_exact_linear_solution(dim):
    """Periodic bulk with a temperature jump: e = C/2pi [T(x) - tau v s_x
    dT/dx] with linear T solves the discrete equations, so q_x = k dT / L
    with k = sum C v^2 tau <s_x^2> and <s_x^2> -> 1/2."""
    rng = np.random.default_rng(21)
    b = dict(C=np.array([8e5, 8.6e5]), v=np.array([6000.0, 2500.0]), tau=np.array([1e-12, 5e-10]))
    n, L, dT = 12, 120e-9, 1.0
    if dim == 1:
        g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4, pdT=(dT, 0, 0))
    else:
        g = geo(2, (n, 3), (L, 30e-9), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2, pdT=(dT, 0, 0))
    case = O.Case(g, mat2(b, 8))
    e0 = rng.normal(size=case.size) * 1e2
    e, st = O.steady(case, scheme=1, tol_T=1e-14, tol_q=1e-13, max_iter=3000, cg_rtol=1e-13, e=e0)
    T, TL, q = O.moments(case, e)
    k = (b["C"] * b["v"] ** 2 * b["tau"]).sum() * 0.5
    np.testing.assert_allclose(q[:, 0], k * dT / L, rtol=1e-9)
    x = (np.arange(case.nc) % n + 0.5) * L / n
    Tex = 300 - dT * (x - L / 2) / L
    np.testing.assert_allclose(T - 300, Tex - 300, atol=1e-9)
    ex = (b["C"][None, None, :] / TWOPI * ((Tex - 300)[:, None, None]
          + (b["tau"] * b["v"])[None, None, :] * case.s[None, :, 0, None] * dT / L))
    np.testing.assert_allclose(e, ex.reshape(-1), atol=1e-9 * np.abs(ex).max())


def test_ballistic_casimir_limit():
    """tau -> infinity between thermalizing walls 2 K apart: each direction
    carries its wall's equilibrium, q = 2 K sum C v (1/2pi) int_{-pi/2}^{pi/2}
    cos = 2 K sum C v / pi, and T is the mean."""
    b = dict(C=np.array([6e5, 1e6]), v=np.array([3000.0, 7000.0]), tau=np.array([1e-3, 1e-3]))
    g = geo(1, (40,), (100e-9,), [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4,
            bcT=[301.0, 299.0, 300, 300, 300, 300])
    case = O.Case(g, mat2(b, 16))
    e, st = O.steady(case, scheme=1, tol_T=1e-13, max_iter=200)
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(q[:, 0], 2.0 * (b["C"] * b["v"]).sum() / np.pi, rtol=1e-6)
    np.testing.assert_allclose(T, 300.0, atol=1e-6)


def test_ttg_ballistic_bessel():
    """Transient grating, gray, tau -> infinity: each in-plane direction
    advects its cosine undamped, so the temperature amplitude is the circle
    average of cos(q v t cos(theta)), i.e. J0(q v t) for continuous angles;
    the oracle's grating follows the discrete-ordinates sum."""
    from scipy.special import j0
    v, L, n = 2000.0, 1e-6, 200
    b = dict(C=np.array([1.6e6]), v=np.array([v]), tau=np.array([1.0]))
    g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    case = O.Case(g, mat2(b, 16))
    x = (np.arange(n) + 0.5) * L / n
    e = (b["C"][0] * 0.5 * np.cos(2 * np.pi * x / L) / TWOPI)[:, None] * np.ones(case.na)[None, :]
    dt = 0.05 * (L / n) / v
    nsteps = 400
    e, _ = O.transient(case, e.reshape(-1), nsteps, dt)
    T, _, _ = O.moments(case, e)
    t = nsteps * dt
    qk = 2 * np.pi / L
    amp = 2 * np.mean((T - 300) * np.cos(qk * x))
    expect = 0.5 * (case.w * np.cos(qk * v * case.s[:, 0] * t)).sum() / TWOPI
    assert abs(amp - expect) < 2e-3 * 0.5
    assert abs(expect / 0.5 - j0(qk * v * t)) < 1e-6


def test_ttg_diffusive_decay():
    """Kn << 1: the grating decays as exp(-q^2 v^2 tau t / 2) (in-plane
    diffusivity v^2 tau / 2)."""
    v, tau, L, n = 2000.0, 1e-12, 2e-6, 100
    b = dict(C=np.array([1.6e6]), v=np.array([v]), tau=np.array([tau]))
    g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    case = O.Case(g, mat2(b, 8))
    x = (np.arange(n) + 0.5) * L / n
    e = (b["C"][0] * np.cos(2 * np.pi * x / L) / TWOPI)[:, None] * np.ones(case.na)[None, :]
    dt = 0.25e-12
    nsteps = 4000
    e, _ = O.transient(case, e.reshape(-1), nsteps, dt)
    T, _, _ = O.moments(case, e)
    qk = 2 * np.pi / L
    amp = 2 * np.mean((T - 300) * np.cos(qk * x))
    expect = np.exp(-qk ** 2 * v ** 2 * tau * 0.5 * nsteps * dt)
    assert abs(amp / expect - 1) < 0.02


def test_ttg_paper_size_matches_fourier_mode():
    """The grating at the paper's size with in-plane directions: the oracle
    equals the exact single-mode recurrence with Omega = 2 pi."""
    cfg = I.ttg(2.0)
    m = dict(cfg["material"], material_dim=2)
    case = O.Case(cfg["geometry"], m)
    c = m["C"][0]
    e = (c * (cfg["T0"] - 300.0) / TWOPI)[:, None] * np.ones(case.na)[None, :]
    n_steps = 60
    e, _ = O.transient(case, e.reshape(-1), n_steps, cfg["dt"])
    T, _, _ = O.moments(case, e)
    ref = ttg_discrete_mode(case.s[:, 0], case.w, m["v"][0], cfg["tau"], 1000, 1e-6, cfg["dt"], n_steps, c,
                            cfg["amplitude"], omega=TWOPI)
    assert np.abs((T - 300.0) - ref).max() < 1e-12 * cfg["amplitude"]


@pytest.mark.parametrize("scheme", [0, 1])
def test_iterative_solution_equals_dense_solve(scheme):
    """Tiny 2D geometry with every wall kind: the converged source iteration
    equals the direct solve of the assembled linear system."""
    from oracle import dense
    rng = np.random.default_rng(9)
    b = I.bands(rng, 2, 1e-12, 1e-10)
    bc = [O.BC_THERMAL, O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_PERIODIC, O.BC_SPECULAR, O.BC_SPECULAR]
    bc[2] = O.BC_PERIODIC
    g = geo(2, (4, 3), (4e-8, 3e-8), bc, bcT=[301.0, 300.0, 300, 300, 300, 300], pdT=(0, 0.5, 0))
    P = rng.uniform(0, 1e17, 12)
    case = O.Case(g, mat2(b, 2), P=P)
    ed = dense.solve_steady(case, floating=False)
    e, st = O.steady(case, scheme=scheme, tol_T=1e-14, tol_q=1e-14, max_iter=20000, cg_rtol=1e-13)
    T, _, q = O.moments(case, e)
    Td, _, qd = O.moments(case, ed)
    assert np.abs(T - Td).max() <= 1e-10 * np.abs(Td - 300).max()
    assert np.abs(q - qd).max() <= 1e-8 * np.abs(qd).max()
