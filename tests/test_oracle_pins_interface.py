"""Pins of the oracle's interfacial boundary condition between two materials
(Sec. 2.2 (v)) and of its per-cell materials.

The interface passes back into material A, diffusely, the fraction beta_BA
of the energy flux that B sends toward it and the fraction 1 - beta_AB of
A's own outgoing flux; in the discrete form
    e_in,A = [beta_BA (v_B / v_A) F_B + (1 - beta_AB) F_A] / W,
with F_X the outgoing flux sum_{s.n > 0} w (s.n) e_face of side X and
W = sum_{s.n < 0} w |s.n| (the diffuse wall's normalisation).  Pins:

* Conservation for any state: with every outer wall adiabatic (specular or
  diffuse) the total flux divergence sum_c sum_{alpha, lambda} w D vanishes
  for a random e, interfaces included (flux leaving A through the face equals
  the flux entering B, whatever beta).  Dropping the speed ratio breaks it
  (checked by planting the slip in the oracle); swapping beta_AB and
  beta_BA does not (that is another conserving interface), but it breaks
  the closed form and the equilibrium below (planted likewise).
* beta = 0 is a diffuse wall on both sides: the residual of the
  two-material slab equals, cell by cell, that of each half alone with a
  diffuse wall at the cut.
* Ballistic closed form: a slab between two thermalizing walls with the
  interface in the middle and no scattering to speak of (tau = 1 s) carries,
  per band, q = W [beta_AB v_A e_A+ - beta_BA v_B e_B-], e_A+ = C_A dT_1 / 4 pi
  and e_B- = C_B dT_2 / 4 pi the emitted values of the two walls (four-flux
  bookkeeping of the forward and backward values on each side); the
  converged oracle's q_x matches in every cell.
* Equilibrium: with beta_BA C_B v_B = beta_AB C_A v_A per band (detailed
  balance) a uniform temperature is a fixed point: the residual of
  e = C_m dT / 4 pi vanishes in every cell, the interface cells included
  (without the speed ratio it does not).
"""
import numpy as np
import pytest

import oracle as O

FOURPI = 4 * np.pi
TREF = 300.0

MAT_A = dict(C=np.array([1.0e5, 2.0e5, 3.0e5]), v=np.array([1000.0, 2000.0, 3000.0]),
             tau=np.array([1e-10, 3e-10, 2e-11]), n_theta=4, n_phi=3, Tref=TREF)
MAT_B = dict(C=np.array([2.0e5, 1.0e5, 4.0e5]), v=np.array([1500.0, 700.0, 2500.0]),
             tau=np.array([5e-11, 2e-10, 1e-10]), n_theta=4, n_phi=3, Tref=TREF)
BETA_AB = np.array([0.3, 0.55, 0.8])
BETA_BA = np.array([0.6, 0.25, 0.45])


def beta(ab, ba):
    b = np.zeros((2, 2, 3))
    b[0, 1], b[1, 0] = ab, ba
    return b


def slab(n, bc, bcT=None, mat=None, length=None):
    """1D slab of n cells of 50 nm, materials per cell (None: one)."""
    g = dict(dim=1, n=[n, 1, 1], len=[length or 50e-9 * n, 1.0, 1.0], bc=bc, bcT=bcT or [TREF] * 6,
             pdT=[0, 0, 0], solid=None, pore_bc=O.BC_DIFFUSE)
    if mat is not None:
        g["mat"] = np.asarray(mat, dtype=np.int32)
    return g


def halves(n):
    return np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.int32)


def seeded(case, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, case.size) * 1e3


def total_divergence(case, e):
    D = O.flux_div(case, e).reshape(case.nc, case.na, case.nl)
    return np.einsum("a,cal->", case.w, D), np.einsum("a,cal->", case.w, np.abs(D))


@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC])
def test_interface_conserves_energy_for_any_state_1d(lim):
    n = 12
    g = slab(n, [O.BC_SPECULAR, O.BC_DIFFUSE] + [O.BC_SPECULAR] * 4, mat=halves(n))
    case = O.Case(g, [MAT_A, MAT_B], beta=beta(BETA_AB, BETA_BA), limiter=lim)
    for seed in range(3):
        tot, scale = total_divergence(case, seeded(case, seed))
        assert abs(tot) <= 1e-13 * scale, (tot, scale)


def test_interface_conserves_energy_for_any_state_2d():
    """Two interfaces (A | B | A along x), pores, periodic y."""
    nx, ny = 9, 6
    mat = np.zeros((ny, nx), dtype=np.int32)
    mat[:, 3:6] = 1
    solid = np.ones((ny, nx), dtype=np.uint8)
    solid[2, 7] = 0
    g = dict(dim=2, n=[nx, ny, 1], len=[nx * 50e-9, ny * 50e-9, 1.0],
             bc=[O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_PERIODIC, O.BC_PERIODIC, O.BC_SPECULAR, O.BC_SPECULAR],
             bcT=[TREF] * 6, pdT=[0, 0, 0], solid=solid.reshape(-1), pore_bc=O.BC_DIFFUSE, mat=mat.reshape(-1))
    case = O.Case(g, [MAT_A, MAT_B], beta=beta(BETA_AB, BETA_BA))
    for seed in range(2):
        e = seeded(case, seed)
        e.reshape(case.nc, -1)[solid.reshape(-1) == 0] = 0.0
        tot, scale = total_divergence(case, e)
        assert abs(tot) <= 1e-13 * scale, (tot, scale)


def test_zero_transmission_is_a_diffuse_wall_on_both_sides():
    n = 10
    T1, T2 = TREF + 2.0, TREF - 1.0
    bcT = [T1, T2] + [TREF] * 4
    bc = [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4
    both = O.Case(slab(n, bc, bcT, mat=halves(n)), [MAT_A, MAT_B], beta=beta(np.zeros(3), np.zeros(3)),
                  limiter=O.LIM_MC)
    left = O.Case(slab(n // 2, [O.BC_THERMAL, O.BC_DIFFUSE] + [O.BC_SPECULAR] * 4, [T1, TREF] + [TREF] * 4),
                  MAT_A, limiter=O.LIM_MC)
    right = O.Case(slab(n // 2, [O.BC_DIFFUSE, O.BC_THERMAL] + [O.BC_SPECULAR] * 4, [TREF, T2] + [TREF] * 4),
                   MAT_B, limiter=O.LIM_MC)
    e = seeded(both, 7)
    half = both.size // 2
    TL = np.random.default_rng(8).uniform(-1, 1, n)
    R = O.residual(both, e, TL)
    Rl = O.residual(left, e[:half], TL[: n // 2])
    Rr = O.residual(right, e[half:], TL[n // 2:])
    np.testing.assert_allclose(R[:half], Rl, rtol=0, atol=1e-12 * np.abs(Rl).max())
    np.testing.assert_allclose(R[half:], Rr, rtol=0, atol=1e-12 * np.abs(Rr).max())


@pytest.mark.parametrize("scheme", [0, 1])
def test_ballistic_slab_matches_the_four_flux_closed_form(scheme):
    n = 16
    dT1, dT2 = 1.0, -0.5
    ma = dict(MAT_A, tau=np.ones(3))
    mb = dict(MAT_B, tau=np.ones(3))
    bc = [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4
    case = O.Case(slab(n, bc, [TREF + dT1, TREF + dT2] + [TREF] * 4, mat=halves(n)), [ma, mb],
                  beta=beta(BETA_AB, BETA_BA))
    e, st = O.steady(case, scheme=scheme, tol_T=1e-13, tol_q=1e-13, max_iter=400)
    assert st["converged"]
    _, _, q = O.moments(case, e)
    W = float(np.sum(case.w[case.s[:, 0] > 0] * case.s[case.s[:, 0] > 0, 0]))
    eA = ma["C"] * dT1 / FOURPI
    eB = mb["C"] * dT2 / FOURPI
    q_ref = float(np.sum(W * (BETA_AB * ma["v"] * eA - BETA_BA * mb["v"] * eB)))
    np.testing.assert_allclose(q[:, 0], q_ref, rtol=1e-7)


def test_detailed_balance_keeps_a_uniform_temperature():
    n = 8
    dT = 1.5
    GA, GB = MAT_A["C"] * MAT_A["v"], MAT_B["C"] * MAT_B["v"]
    b_ab = np.array([0.2, 0.1, 0.7])
    b_ba = b_ab * GA / GB
    assert np.all(b_ba <= 1)
    bc = [O.BC_THERMAL, O.BC_THERMAL] + [O.BC_SPECULAR] * 4
    case = O.Case(slab(n, bc, [TREF + dT] * 2 + [TREF] * 4, mat=halves(n)), [MAT_A, MAT_B],
                  beta=beta(b_ab, b_ba), limiter=O.LIM_MC)
    mat = halves(n)
    C = np.where(mat[:, None] == 0, MAT_A["C"][None, :], MAT_B["C"][None, :])   # [nc, nl]
    e = np.repeat(C[:, None, :] * dT / FOURPI, case.na, axis=1).reshape(-1)
    R = O.residual(case, e, np.full(n, dT))
    assert np.abs(R).max() <= 1e-12 * np.abs(e).max() * (1.0 / MAT_A["tau"].min())


def test_adjoint_refuses_several_materials():
    n = 6
    case = O.Case(slab(n, [O.BC_THERMAL] * 2 + [O.BC_SPECULAR] * 4, mat=halves(n)), [MAT_A, MAT_B],
                  beta=beta(BETA_AB, BETA_BA))
    with pytest.raises(RuntimeError):
        O.apply_jac_T(case, case.zeros())
