"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them.
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from oracle import dense
from oracle.adjoint import keff_weights, steady_adjoint, transient_adjoint

FOURPI = 4 * np.pi


def gray(v=2677.0, tau=39.9e-12, C=1627600.0):
    """Gray silicon parameters quoted in the verification section (Sec. 3.6)."""
    return dict(C=np.array([C]), v=np.array([v]), tau=np.array([tau]))


def mat(b, n_theta, n_phi=1, Tref=300.0):
    m = dict(b)
    m.update(n_theta=n_theta, n_phi=n_phi, Tref=Tref)
    return m


def geo(dim, n, length, bc, bcT=None, pdT=(0, 0, 0), solid=None, pore_bc=O.BC_DIFFUSE):
    n = list(n) + [1] * (3 - len(n))
    length = list(length) + [1.0] * (3 - len(length))
    return dict(dim=dim, n=n, len=length, bc=bc, bcT=bcT or [300.0] * 6, pdT=list(pdT),
                solid=solid, pore_bc=pore_bc)


# ------------------------------------------------------------------ quadrature

@pytest.mark.parametrize("dim,nt,nph", [(1, 8, 1), (3, 2, 8), (3, 4, 4), (3, 2, 4), (3, 3, 4)])
def test_quadrature_symmetry(dim, nt, nph):
    s, w = O.quadrature(dim, nt, nph)
    assert len(w) == (2 * nt if dim == 1 else 8 * nt * nph)
    assert np.all(w > 0)
    assert abs(w.sum() - FOURPI) < 1e-13
    np.testing.assert_allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-14) if dim > 1 else None
    for a in range(3):
        assert abs((w * s[:, a]).sum()) < 1e-13
        for b in range(a + 1, 3):
            assert abs((w * s[:, a] * s[:, b]).sum()) < 1e-13


def test_quadrature_nodes_match_closed_forms():
    """Gauss-Legendre nodes/weights from their closed forms (golden fixture)
    mapped to theta in (0, pi/2) as Sec. 3.2 prescribes: the 1D direction set
    is cos(theta) per hemisphere with w proportional to w_theta sin(theta)."""
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "gauss_legendre.txt"))
    for n in (2, 3, 4):
        x, wg = rows[rows[:, 0] == n, 1], rows[rows[:, 0] == n, 2]
        th = (x + 1) * np.pi / 4
        wt = 2 * np.pi * wg * np.pi / 4 * np.sin(th)
        wt *= 2 * np.pi / wt.sum()          # each hemisphere carries 2 pi
        s, w = O.quadrature(1, n, 1)
        hemi = s[:, 0] > 0
        order = np.argsort(-np.cos(th))
        np.testing.assert_allclose(np.sort(s[hemi, 0])[::-1], np.cos(th)[order], rtol=0, atol=1e-15)
        np.testing.assert_allclose(w[hemi][np.argsort(-s[hemi, 0])], wt[order], rtol=1e-14)
        np.testing.assert_allclose(np.sort(-s[~hemi, 0])[::-1], np.cos(th)[order], rtol=0, atol=1e-15)


def test_quadrature_moments_close_to_sphere():
    # 1D: 8 Gauss-Legendre theta nodes per hemisphere integrate mu^2 almost exactly
    s, w = O.quadrature(1, 8, 1)
    assert abs((w * s[:, 0] ** 2).sum() / FOURPI - 1 / 3) < 1e-11
    # hemisphere flux sum_{s_x>0} w s_x -> pi
    assert abs((w * s[:, 0] * (s[:, 0] > 0)).sum() - np.pi) < 1e-11
    # 3D: finer quadratures approach the continuous second moment
    errs = []
    for nt, nph in [(2, 4), (4, 4), (8, 8)]:
        s, w = O.quadrature(3, nt, nph)
        errs.append(abs((w * s[:, 2] ** 2).sum() / FOURPI - 1 / 3))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-9


# ------------------------------------------------------------- closure/moments

def test_scattering_conserves_energy():
    """With no streaming (v = 0) R = -(e - e0)/tau + Q; the closure of
    eq. BTE_get_e0 makes sum_{alpha,lambda} w R equal to the heat input P."""
    rng = np.random.default_rng(7)
    b = dict(C=rng.uniform(1e5, 5e5, 4), v=np.zeros(4), tau=10 ** rng.uniform(-12, -9, 4))
    g = geo(2, (5, 4), (1e-7, 1e-7), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2)
    P = rng.uniform(0, 1e15, 20)
    gam = rng.uniform(0, 1e11, 20)
    case = O.Case(g, mat(b, 2, 2), P=P, gamma=gam)
    e = rng.normal(size=case.size) * 1e3
    R = O.residual(case, e).reshape(case.nc, case.na, case.nl)
    tot = (case.w[None, :, None] * R).sum(axis=(1, 2))
    np.testing.assert_allclose(tot, P, rtol=1e-12, atol=1e-12 * np.abs(R).max())


def test_moments_equilibrium_and_flux():
    rng = np.random.default_rng(3)
    b = I.bands(rng, 5, 1e-12, 1e-9)
    g = geo(3, (3, 2, 2), (1e-7, 1e-7, 1e-7), [O.BC_PERIODIC] * 6)
    case = O.Case(g, mat(b, 2, 4))
    Tst = 300 + rng.uniform(-2, 2, case.nc)
    e = (b["C"][None, None, :] * (Tst - 300)[:, None, None] / FOURPI * np.ones((1, case.na, 1))).reshape(-1)
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(T, Tst, rtol=0, atol=1e-12)
    np.testing.assert_allclose(TL, Tst, rtol=0, atol=1e-12)
    qscale = FOURPI * (b["C"] * b["v"]).sum() * 2 / FOURPI
    assert np.abs(q).max() < 1e-14 * qscale
    # first-order anisotropic part carries the Fourier flux q = -k_disc grad T
    grad = np.array([2e7, -1e7, 5e6])
    sg = case.s @ grad
    e2 = (b["C"][None, :] / FOURPI * (0.0 - (b["tau"] * b["v"])[None, :] * sg[:, None]))
    e2 = np.broadcast_to(e2, (case.nc, case.na, case.nl)).reshape(-1)
    _, _, q2 = O.moments(case, e2)
    M = (case.w[:, None, None] * case.s[:, :, None] * case.s[:, None, :]).sum(0) / FOURPI
    k = (b["C"] * b["v"] ** 2 * b["tau"]).sum()
    np.testing.assert_allclose(q2[0], -k * M @ grad, rtol=1e-12)


def test_gray_lattice_equals_local_temperature():
    rng = np.random.default_rng(5)
    g = geo(1, (6,), (1e-7,), [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4)
    case = O.Case(g, mat(gray(), 8))
    e = rng.normal(size=case.size)
    T, TL, _ = O.moments(case, e)
    np.testing.assert_allclose(T, TL, rtol=0, atol=1e-13)


# --------------------------------------------------------------- flux operator

@pytest.mark.parametrize("walls", ["periodic", "specular", "diffuse", "mixed"])
def test_closed_domain_zero_net_flux(walls):
    """Face fluxes telescope between neighbours and adiabatic walls (specular,
    diffuse with the discrete normalisation) carry zero net energy, so for a
    closed domain sum_cells sum_{alpha,lambda} w D = 0 for ANY e."""
    rng = np.random.default_rng(11)
    b = I.bands(rng, 3, 1e-12, 1e-9)
    bc = {"periodic": [O.BC_PERIODIC] * 6, "specular": [O.BC_SPECULAR] * 6,
          "diffuse": [O.BC_DIFFUSE] * 6,
          "mixed": [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_SPECULAR, O.BC_DIFFUSE]}[walls]
    solid = np.ones(60, dtype=np.uint8)
    solid[[7, 8, 31, 44]] = 0
    g = geo(3, (5, 4, 3), (1e-7, 1.2e-7, 0.9e-7), bc, solid=solid)
    for lim in (O.LIM_NONE, O.LIM_MC):
        case = O.Case(g, mat(b, 2, 3), limiter=lim)
        e = rng.normal(size=case.size)
        D = O.flux_div(case, e).reshape(case.nc, case.na, case.nl)
        tot = (case.w[None, :, None] * D).sum()
        scale = (case.w[None, :, None] * np.abs(D)).sum()
        assert abs(tot) < 1e-13 * scale, (walls, lim, tot, scale)


def test_equilibrium_is_fixed_point_with_walls_at_same_temperature():
    rng = np.random.default_rng(2)
    b = I.bands(rng, 4, 1e-12, 1e-9)
    bc = [O.BC_THERMAL, O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_THERMAL, O.BC_DIFFUSE, O.BC_THERMAL]
    g = geo(3, (4, 3, 3), (1e-7,) * 3, bc, bcT=[302.5] * 6)
    case = O.Case(g, mat(b, 2, 2))
    e, st = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e30, max_iter=5)
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(T, 302.5, atol=1e-12)
    qscale = (b["C"] * b["v"]).sum() * 2.5
    assert np.abs(q).max() < 1e-13 * qscale
    assert st["iters"] <= 2


# ----------------------------------------------------------- steady solutions

@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC])
@pytest.mark.parametrize("dim", [1, 2])
def test_periodic_bulk_exact_linear_solution(dim, lim):
    """Periodic bulk with a temperature jump: the discrete equations are
    solved exactly by e = C/4pi [T(x) - tau v s_x dT/dx] with linear T, so
    q_x = k_disc dT/L with k_disc = sum C v^2 tau M_xx at any Knudsen number."""
    rng = np.random.default_rng(21)
    b = dict(C=np.array([8e5, 8.6e5]), v=np.array([6000.0, 2500.0]), tau=np.array([1e-12, 5e-10]))
    n, L, dT = 12, 120e-9, 1.0
    if dim == 1:
        g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4, pdT=(dT, 0, 0))
        m = mat(b, 8)
    else:
        g = geo(2, (n, 3), (L, 30e-9), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2, pdT=(dT, 0, 0))
        m = mat(b, 2, 2)
    case = O.Case(g, m, limiter=lim)
    e0 = rng.normal(size=case.size) * 1e2
    e, st = O.steady(case, scheme=1, tol_T=1e-14, tol_q=1e-13, max_iter=3000, cg_rtol=1e-13, e=e0)
    T, TL, q = O.moments(case, e)
    Mxx = (case.w * case.s[:, 0] ** 2).sum() / FOURPI
    kd = (b["C"] * b["v"] ** 2 * b["tau"]).sum() * Mxx
    np.testing.assert_allclose(q[:, 0], kd * dT / L, rtol=2e-10)
    x = (np.arange(case.nc) % n + 0.5) * L / n
    Tex = 300 - dT * (x - L / 2) / L
    np.testing.assert_allclose(T - 300, Tex - 300, atol=1e-9)
    ex = (b["C"][None, None, :] / FOURPI * ((Tex - 300)[:, None, None]
          + (b["tau"] * b["v"])[None, None, :] * case.s[None, :, 0, None] * dT / L))
    np.testing.assert_allclose(e, ex.reshape(-1), atol=1e-9 * np.abs(ex).max())


def test_ballistic_casimir_limit():
    """tau -> infinity between thermalizing walls: each direction carries its
    wall value, q = dT sum_lambda C v (sum_{s_x>0} w s_x)/4pi and T is the mean."""
    b = dict(C=np.array([6e5, 1e6]), v=np.array([3000.0, 7000.0]), tau=np.array([1e-3, 1e-3]))
    g = geo(1, (40,), (100e-9,), [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4,
            bcT=[301.0, 299.0, 300, 300, 300, 300])
    case = O.Case(g, mat(b, 8))
    e, st = O.steady(case, scheme=1, tol_T=1e-13, max_iter=200)
    T, TL, q = O.moments(case, e)
    hemi = (case.w * case.s[:, 0] * (case.s[:, 0] > 0)).sum()
    qc = 2.0 * (b["C"] * b["v"]).sum() * hemi / FOURPI
    np.testing.assert_allclose(q[:, 0], qc, rtol=1e-6)
    np.testing.assert_allclose(T, 300.0, atol=1e-6)


def test_diffusive_limit_approaches_fourier():
    """Kn -> 0 with the mesh resolving the mean free path (dx <= Lambda/2):
    q -> k dT/L, with a first-order-in-Kn deficit from the wall slip."""
    errs = []
    L, n = 200e-9, 200
    for tau in (4e-12, 2e-12, 1e-12):
        b = dict(C=np.array([1.6e6]), v=np.array([2000.0]), tau=np.array([tau]))
        g = geo(1, (n,), (L,), [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4,
                bcT=[301.0, 299.0, 300, 300, 300, 300])
        case = O.Case(g, mat(b, 8))
        e, st = O.steady(case, scheme=1, tol_T=1e-12, max_iter=5000)
        assert st["converged"]
        _, _, q = O.moments(case, e)
        Mxx = (case.w * case.s[:, 0] ** 2).sum() / FOURPI
        qf = 1.6e6 * 2000.0 ** 2 * tau * Mxx * 2.0 / L
        errs.append(1.0 - q[:, 0].mean() / qf)
    assert all(0 < x < 0.1 for x in errs)
    # deficit halves with Kn (first order)
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


def test_slab_antisymmetry_and_face_flux_conservation():
    cfg = I.slab1d_case(n_cells=60)
    case = O.Case(cfg["geometry"], cfg["material"])
    e, st = O.steady(case, scheme=1, tol_T=1e-13, tol_q=1e-13, max_iter=5000)
    assert st["converged"]
    T, TL, q = O.moments(case, e)
    np.testing.assert_allclose(T - 300, -(T[::-1] - 300), atol=1e-11)
    # face fluxes: telescoping makes the per-cell divergence zero at convergence
    D = O.flux_div(case, e).reshape(case.nc, case.na, case.nl)
    divq = (case.w[None, :, None] * D).sum(axis=(1, 2))
    assert np.abs(divq).max() < 1e-8 * np.abs(q[:, 0]).max() / (100e-9 / 60)


# ------------------------------------------------ iteration vs direct solve

def _tiny_cases():
    rng = np.random.default_rng(99)
    b = I.bands(rng, 2, 1e-12, 1e-9)
    out = []
    g = geo(1, (12,), (60e-9,), [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4,
            bcT=[301.0, 299.5, 300, 300, 300, 300])
    out.append(("slab", O.Case(g, mat(b, 4), P=rng.uniform(0, 1e17, 12)), False))
    solid = np.ones(30, dtype=np.uint8)
    solid[[8, 14]] = 0
    g = geo(2, (6, 5), (60e-9, 50e-9), [O.BC_THERMAL, O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_DIFFUSE,
                                         O.BC_SPECULAR, O.BC_SPECULAR],
            bcT=[300.5] * 6, solid=solid)
    out.append(("walls2d", O.Case(g, mat(b, 1, 2), P=rng.uniform(0, 1e17, 30),
                                  gamma=rng.uniform(0, 1e11, 30)), False))
    g = geo(2, (5, 4), (50e-9, 40e-9), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2, pdT=(1.0, 0, 0),
            solid=np.array([1] * 6 + [0] + [1] * 13, dtype=np.uint8))
    out.append(("porous2d", O.Case(g, mat(b, 1, 2)), True))
    return out


@pytest.mark.parametrize("idx", [0, 1, 2])
@pytest.mark.parametrize("scheme", [0, 1])
def test_iterative_solution_equals_dense_solve(idx, scheme):
    name, case, floating = _tiny_cases()[idx]
    ed = dense.solve_steady(case, floating=floating)
    e, st = O.steady(case, scheme=scheme, tol_T=1e-14, tol_q=1e-14, max_iter=20000, cg_rtol=1e-13)
    T, _, q = O.moments(case, e)
    Td, _, qd = O.moments(case, ed)
    assert np.abs(T - Td).max() <= 1e-10 * np.abs(Td - 300).max()
    assert np.abs(q - qd).max() <= 1e-8 * np.abs(qd).max()


def test_transient_reaches_steady_solution():
    name, case, floating = _tiny_cases()[0]
    es, _ = O.steady(case, scheme=1, tol_T=1e-14, tol_q=1e-14, max_iter=20000)
    e = case.zeros()
    dt = 0.2e-12
    for _ in range(200):
        e_prev = e.copy()
        e, _ = O.transient(case, e, 500, dt)
        if np.abs(e - e_prev).max() < 1e-14 * np.abs(e).max():
            break
    np.testing.assert_allclose(e, es, atol=1e-10 * np.abs(es).max())


# ------------------------------------------------------------------ transient

def test_transient_energy_balance_closed_domain():
    """Per explicit step: Delta sum_cells sum w e = dt sum_cells P (scattering
    conserves energy, fluxes telescope, adiabatic/periodic walls are closed)."""
    rng = np.random.default_rng(4)
    b = I.bands(rng, 3, 1e-12, 1e-9)
    g = geo(3, (4, 4, 3), (1e-7,) * 3, [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_DIFFUSE, O.BC_SPECULAR,
                                        O.BC_DIFFUSE, O.BC_DIFFUSE])
    P = rng.uniform(0, 1e16, 48)
    for lim in (O.LIM_NONE, O.LIM_MC):
        case = O.Case(g, mat(b, 2, 2), P=P, limiter=lim)
        e = rng.normal(size=case.size) * 10
        dt = 0.1e-12
        E0 = (case.w[None, :, None] * e.reshape(case.nc, case.na, case.nl)).sum()
        e1, _ = O.transient(case, e.copy(), 1, dt, 5e-12, pulse=(6e-12, 3e-12))
        E1 = (case.w[None, :, None] * e1.reshape(case.nc, case.na, case.nl)).sum()
        fac = np.exp(-4 * np.log(2) * 1e-24 / 9e-24)
        np.testing.assert_allclose(E1 - E0, dt * P.sum() * fac, rtol=1e-9)


def test_ttg_ballistic_discrete_ordinates():
    """Transient thermal grating, gray, tau -> infinity: each direction
    advects its cosine undamped, so the amplitude of T is
    sum_alpha w cos(q v mu_alpha t)/4pi (the discrete-ordinates form of
    sin(qvt)/(qvt)); second-order upwind on 200 cells/period adds a small
    numerical damping only."""
    v, L, n = 2000.0, 1e-6, 200
    b = dict(C=np.array([1.6e6]), v=np.array([v]), tau=np.array([1.0]))
    g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    case = O.Case(g, mat(b, 8))
    x = (np.arange(n) + 0.5) * L / n
    A0 = 0.5
    e = (b["C"][0] * A0 * np.cos(2 * np.pi * x / L) / FOURPI)[:, None] * np.ones(case.na)[None, :]
    dt = 0.05 * (L / n) / v
    nsteps = 400
    e, _ = O.transient(case, e.reshape(-1), nsteps, dt)
    T, _, _ = O.moments(case, e)
    t = nsteps * dt
    qk = 2 * np.pi / L
    amp = 2 * np.mean((T - 300) * np.cos(qk * x))
    expect = A0 * (case.w * np.cos(qk * v * case.s[:, 0] * t)).sum() / FOURPI
    assert abs(amp - expect) < 2e-3 * A0
    # continuous-angle limit for reference
    cont = A0 * np.sin(qk * v * t) / (qk * v * t)
    assert abs(expect - cont) < 1e-3


def test_ttg_diffusive_decay():
    """Kn << 1: the grating amplitude decays as exp(-q^2 v^2 tau M_xx t)."""
    v, tau, L, n = 2000.0, 1e-12, 2e-6, 100
    b = dict(C=np.array([1.6e6]), v=np.array([v]), tau=np.array([tau]))
    g = geo(1, (n,), (L,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    case = O.Case(g, mat(b, 8))
    x = (np.arange(n) + 0.5) * L / n
    e = (b["C"][0] * np.cos(2 * np.pi * x / L) / FOURPI)[:, None] * np.ones(case.na)[None, :]
    dt = 0.25e-12
    nsteps = 4000
    e, _ = O.transient(case, e.reshape(-1), nsteps, dt)
    T, _, _ = O.moments(case, e)
    qk = 2 * np.pi / L
    amp = 2 * np.mean((T - 300) * np.cos(qk * x))
    Mxx = (case.w * case.s[:, 0] ** 2).sum() / FOURPI
    expect = np.exp(-qk ** 2 * v ** 2 * tau * Mxx * nsteps * dt)
    assert abs(amp / expect - 1) < 0.02


@pytest.mark.parametrize("xi", [0.5, 5.0])
def test_ttg_paper_size_matches_fourier_mode(xi):
    """The transient grating at the paper's size (1000 cells, 512
    directions, gray, periodic): on a uniform periodic grid one Fourier mode
    stays one mode, so the explicit second-order upwind scheme with
    relaxation reduces to a 512 x 512 complex recurrence (derived from the
    face-value symbol, not from the oracle's code).  The oracle's field must
    equal it to rounding."""
    from tests.helpers import ttg_discrete_mode
    cfg = I.ttg(xi)
    case = O.Case(cfg["geometry"], cfg["material"])
    c = cfg["material"]["C"][0]
    e = (c * (cfg["T0"] - 300.0) / FOURPI)[:, None] * np.ones(case.na)[None, :]
    n_steps = 60
    e, _ = O.transient(case, e.reshape(-1), n_steps, cfg["dt"])
    T, _, _ = O.moments(case, e)
    ref = ttg_discrete_mode(case.s[:, 0], case.w, cfg["material"]["v"][0], cfg["tau"], 1000, 1e-6, cfg["dt"],
                            n_steps, c, cfg["amplitude"])
    assert np.abs((T - 300.0) - ref).max() < 1e-12 * cfg["amplitude"]


# -------------------------------------------------------------------- adjoint

def test_adjoint_dot_product():
    """<(dR/de) x, y> = <x, (dR/de)^T y>: the transposed operator (scatter
    form) against the forward residual (gather form)."""
    for name, case, floating in _tiny_cases():
        rng = np.random.default_rng(17)
        x = rng.normal(size=case.size)
        y = rng.normal(size=case.size)
        Mx = O.residual(case, x) - O.residual(case, np.zeros(case.size))
        lhs = Mx @ y
        rhs = x @ O.apply_jac_T(case, y)
        assert abs(lhs - rhs) < 1e-12 * (np.abs(Mx).max() * np.abs(y).sum())


def test_adjoint_dot_product_3d_pores():
    rng = np.random.default_rng(8)
    b = I.bands(rng, 2, 1e-12, 1e-9)
    solid = np.ones(48, dtype=np.uint8)
    solid[[5, 6, 21, 40]] = 0
    g = geo(3, (4, 4, 3), (1e-7, 1e-7, 0.8e-7), [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_SPECULAR,
                                                O.BC_DIFFUSE, O.BC_THERMAL, O.BC_DIFFUSE],
            pdT=(1.0, 0, 0), solid=solid)
    case = O.Case(g, mat(b, 1, 2), gamma=rng.uniform(0, 1e11, 48))
    x = rng.normal(size=case.size)
    y = rng.normal(size=case.size)
    Mx = O.residual(case, x) - O.residual(case, np.zeros(case.size))
    assert abs(Mx @ y - x @ O.apply_jac_T(case, y)) < 1e-12 * np.abs(Mx).max() * np.abs(y).sum()


def test_steady_adjoint_against_central_differences():
    rng = np.random.default_rng(31)
    b = I.bands(rng, 2, 1e-12, 1e-9)
    solid = np.ones(20, dtype=np.uint8)
    solid[7] = 0
    g = geo(2, (5, 4), (50e-9, 40e-9), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2, pdT=(1.0, 0, 0),
            solid=solid)
    gam = rng.uniform(0, 1e11, 20)
    case = O.Case(g, mat(b, 1, 2), gamma=gam)
    e, _ = O.steady(case, scheme=1, tol_T=1e-15, tol_q=1e-15, max_iter=20000, cg_rtol=1e-14)
    psi, grad = steady_adjoint(case, e, keff_weights(case))
    for c in (0, 3, 11, 18):
        h = 1e-4 * max(gam[c], 1e10)
        ks = []
        for sg in (+1, -1):
            g2 = gam.copy()
            g2[c] += sg * h
            c2 = case.with_(gamma=g2)
            e2, _ = O.steady(c2, scheme=1, tol_T=1e-15, tol_q=1e-15, max_iter=20000, cg_rtol=1e-14, e=e)
            ks.append(O.keff(c2, e2))
        fd = (ks[0] - ks[1]) / (2 * h)
        assert abs(fd - grad[c]) <= 1e-4 * np.abs(grad).max(), (c, fd, grad[c])
    assert grad[7] == 0.0


def test_steady_adjoint_uniform_gamma_sum_rule():
    """Periodic bulk: k_eff = sum C v^2 tau_eff M_xx, so sum_i dk/dgamma_i =
    -sum C v^2 tau_eff^2 M_xx, shared equally by all cells."""
    b = dict(C=np.array([7e5, 9e5]), v=np.array([5000.0, 2000.0]), tau=np.array([2e-12, 3e-10]))
    g = geo(2, (6, 3), (60e-9, 30e-9), [O.BC_PERIODIC] * 4 + [O.BC_SPECULAR] * 2, pdT=(1.0, 0, 0))
    gam = np.full(18, 4e10)
    case = O.Case(g, mat(b, 1, 2), gamma=gam)
    e, _ = O.steady(case, scheme=1, tol_T=1e-15, tol_q=1e-15, max_iter=20000, cg_rtol=1e-14)
    _, grad = steady_adjoint(case, e, keff_weights(case))
    Mxx = (case.w * case.s[:, 0] ** 2).sum() / FOURPI
    te = 1 / (1 / b["tau"] + 4e10)
    expect = -(b["C"] * b["v"] ** 2 * te ** 2).sum() * Mxx
    np.testing.assert_allclose(grad.sum(), expect, rtol=1e-9)
    np.testing.assert_allclose(grad, expect / 18, rtol=1e-8)


def test_transient_adjoint_against_central_differences():
    rng = np.random.default_rng(12)
    b = I.bands(rng, 2, 1e-12, 1e-9)
    g = geo(3, (3, 3, 3), (0.3e-6,) * 3, [O.BC_THERMAL] * 5 + [O.BC_DIFFUSE])
    P = rng.uniform(0, 1e18, 27)
    gam = rng.uniform(0, 1e11, 27)
    case = O.Case(g, mat(b, 1, 2), P=P, gamma=gam)
    wts = np.zeros(27)
    wts[18:] = rng.uniform(0.5, 1.0, 9)
    e0 = case.zeros()
    J, grad = transient_adjoint(case, e0, 30, 0.5e-12, 0.0, (5e-12, 4e-12), wts)
    for c in (4, 13, 22):
        h = 1e-4 * max(gam[c], 1e10)
        Js = []
        for sg in (+1, -1):
            g2 = gam.copy()
            g2[c] += sg * h
            Jp, _ = transient_adjoint(case.with_(gamma=g2), e0, 30, 0.5e-12, 0.0, (5e-12, 4e-12), wts)
            Js.append(Jp)
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(fd - grad[c]) <= 1e-5 * np.abs(grad).max(), (c, fd, grad[c])
