"""Pins of two oracle parts that the other pins reach only indirectly:
the limited slopes of the face reconstruction and the per-iterate operator
of the transport sweep.

* Limited slopes (the slope limiting that the second-order face value
  e_f = e_m + grad e_m . l of Sec. 3.3 takes when a limiter is chosen).  The
  definitions used are the published ones:
    - minmod (Roe): minmod(a, b) = sign(a) min(|a|, |b|) if a b > 0, else 0;
    - monotonised central (van Leer): MC(a, b) = minmod(2a, 2b, (a + b) / 2);
    - none: the least-squares gradient, which on a uniform Cartesian grid is
      the central difference (a + b) / 2;
  with a = (e_i - e_{i-1}) / h and b = (e_{i+1} - e_i) / h.  The expected
  slopes below are worked out by hand for a ten-cell periodic pattern with a
  plateau, a peak, unequal one-sided differences (clipped by 2|a| and by
  2|b|) and descending runs.
* Limiter property: forward-Euler advection with the MUSCL face values is
  total-variation diminishing for every limiter function 0 <= phi(r) <= 2,
  0 <= phi(r) / r <= 2 at a Courant number <= 1/2 (Harten's condition), so
  MC and minmod make no new extrema from a step; the unlimited central
  gradient overshoots.
* Sweep operator: the stiffness matrix of eq. "Linear system" (Sec. 3.5),
    A_ii = 1/tau_i + sum_{faces} (1/V) v s.n Theta(v s.n) S,
    A_ij = (1/V) v s.n Theta(-v s.n) S  (interior faces; boundary and
    periodic inflow lagged into b),
  assembled densely from the geometry alone, and A de = b with b the
  residual of eq. B_BTE, solved with numpy, must equal one oracle sweep.
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O

FOURPI = 4 * np.pi


def geo(dim, n, length, bc, bcT=None, pdT=(0, 0, 0), solid=None, pore_bc=O.BC_DIFFUSE):
    n = list(n) + [1] * (3 - len(n))
    length = list(length) + [1.0] * (3 - len(length))
    return dict(dim=dim, n=n, len=length, bc=bc, bcT=bcT or [300.0] * 6, pdT=list(pdT),
                solid=solid, pore_bc=pore_bc)


# ---------------------------------------------------------- limited slopes

# cell values of the pattern (periodic: cell 9 is followed by cell 0)
PATTERN = np.array([0.0, 0.0, 2.0, 5.0, 5.5, 11.0, 7.0, 3.0, 2.0, 0.0])

# Hand-derived slopes times h.  Per cell: a = e_i - e_{i-1}, b = e_{i+1} - e_i
#   cell 0: a = 0,    b = 0     plateau                      none 0     MC 0     minmod 0
#   cell 1: a = 0,    b = 2     one side flat                none 1     MC 0     minmod 0
#   cell 2: a = 2,    b = 3     MC = central (2.5 < 4, 6)    none 2.5   MC 2.5   minmod 2
#   cell 3: a = 3,    b = 0.5   MC clipped by 2|b| = 1       none 1.75  MC 1     minmod 0.5
#   cell 4: a = 0.5,  b = 5.5   MC clipped by 2|a| = 1       none 3     MC 1     minmod 0.5
#   cell 5: a = 5.5,  b = -4    peak (sign change)           none 0.75  MC 0     minmod 0
#   cell 6: a = -4,   b = -4    equal, descending            none -4    MC -4    minmod -4
#   cell 7: a = -4,   b = -1    MC clipped by 2|b| = 2       none -2.5  MC -2    minmod -1
#   cell 8: a = -1,   b = -2    MC = central (1.5 < 2, 4)    none -1.5  MC -1.5  minmod -1
#   cell 9: a = -2,   b = 0     one side flat                none -1    MC 0     minmod 0
SLOPES_H = {
    O.LIM_NONE: np.array([0.0, 1.0, 2.5, 1.75, 3.0, 0.75, -4.0, -2.5, -1.5, -1.0]),
    O.LIM_MC: np.array([0.0, 0.0, 2.5, 1.0, 1.0, 0.0, -4.0, -2.0, -1.5, 0.0]),
    O.LIM_MINMOD: np.array([0.0, 0.0, 2.0, 0.5, 0.5, 0.0, -4.0, -1.0, -1.0, 0.0]),
}


def _pattern_case(lim):
    b = dict(C=np.array([1.0e6]), v=np.array([3000.0]), tau=np.array([5e-11]))
    n, h = len(PATTERN), 1e-9
    g = geo(1, (n,), (n * h,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    m = dict(b, n_theta=3, n_phi=1, Tref=300.0)
    return O.Case(g, m, limiter=lim), h


@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC, O.LIM_MINMOD])
def test_limited_slopes_hand_values(lim):
    """The residual of an isotropic field on a gray periodic slab is -D (the
    equilibrium closure makes e0 = e, so scattering drops out exactly), and
    D is fixed by the face values e_i +- (h/2) slope_i:
      s_x > 0:  D_i = (v s_x / h) [(e_i + sig_i/2) - (e_{i-1} + sig_{i-1}/2)]
      s_x < 0:  D_i = (v s_x / h) [(e_{i+1} - sig_{i+1}/2) - (e_i - sig_i/2)]
    with sig = slope * h from the hand-derived table."""
    case, h = _pattern_case(lim)
    e = np.repeat(PATTERN[:, None], case.na * case.nl, axis=1).reshape(-1)
    R = O.residual(case, e).reshape(case.nc, case.na)
    sig = SLOPES_H[lim]
    v = case.v[0]
    up = np.roll(PATTERN, 1), np.roll(sig, 1)      # cell i-1
    dn = np.roll(PATTERN, -1), np.roll(sig, -1)    # cell i+1
    for al in range(case.na):
        mu = case.s[al, 0]
        if mu > 0:
            D = v * mu / h * ((PATTERN + sig / 2) - (up[0] + up[1] / 2))
        else:
            D = v * mu / h * ((dn[0] - dn[1] / 2) - (PATTERN - sig / 2))
        np.testing.assert_allclose(R[:, al], -D, rtol=0, atol=1e-12 * v / h * 11.0)


def _advect_step(lim, n_steps, cfl=0.5):
    """A square wave carried by every direction of a gray slab with no
    scattering to speak of (tau = 1000 s) for n_steps explicit steps with
    the largest Courant number v |s_x| dt / h equal to `cfl`."""
    n, h = 64, 1e-9
    b = dict(C=np.array([1.0e6]), v=np.array([2000.0]), tau=np.array([1.0e3]))
    g = geo(1, (n,), (n * h,), [O.BC_PERIODIC] * 2 + [O.BC_SPECULAR] * 4)
    case = O.Case(g, dict(b, n_theta=4, n_phi=1, Tref=300.0), limiter=lim)
    x = np.arange(n)
    wave = ((x >= n // 4) & (x < 3 * n // 4)).astype(float)
    e = np.repeat(wave[:, None], case.na, axis=1).reshape(-1)
    dt = cfl * h / (b["v"][0] * np.abs(case.s[:, 0]).max())
    e, _ = O.transient(case, e, n_steps, dt)
    return e.reshape(n, case.na)


@pytest.mark.parametrize("lim", [O.LIM_MC, O.LIM_MINMOD])
def test_limited_advection_makes_no_new_extrema(lim):
    e = _advect_step(lim, 150)
    assert e.max() <= 1.0 + 1e-12 and e.min() >= -1e-12, (e.min(), e.max())
    # the wave has moved and been smeared in every direction
    assert np.all(((e > 0.01) & (e < 0.99)).sum(axis=0) >= 2)


def test_unlimited_advection_overshoots():
    e = _advect_step(O.LIM_NONE, 150)
    assert e.max() > 1.02 or e.min() < -0.02, (e.min(), e.max())


# ------------------------------------------------------ sweep operator


def _dense_sweep_operator(case, al, l):
    """A_{alpha,lambda} of eq. "Linear system" on the Cartesian grid, built
    from the geometry: face area over cell volume is 1/h_a per axis, every
    axis with s_a != 0 has one outflow face (interior or boundary) and one
    inflow face; the inflow face couples to the upwind cell only if that cell
    is a solid cell reached without crossing the domain boundary (boundary
    and periodic inflow are lagged into b).  Pore cells carry identity rows
    (they have no unknowns)."""
    n = case.n
    nc = case.nc
    A = np.zeros((nc, nc))
    s = case.s[al]
    v = case.v[l]
    solid = np.ones(nc, dtype=bool) if case.solid is None else case.solid.astype(bool)
    gam = np.zeros(nc) if case.gamma is None else case.gamma
    for c in range(nc):
        if not solid[c]:
            A[c, c] = 1.0
            continue
        idx = [c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]
        A[c, c] = 1.0 / case.tau[l] + gam[c]
        for a in range(case.dim):
            if s[a] == 0.0:
                continue
            h = case.len[a] / n[a]
            ca = v * abs(s[a]) / h
            A[c, c] += ca                        # outflow face: Theta(v s.n) = 1
            k = idx[a] - (1 if s[a] > 0 else -1)  # upwind neighbour along axis a
            if 0 <= k < n[a]:
                j_idx = list(idx)
                j_idx[a] = k
                j = j_idx[0] + n[0] * (j_idx[1] + n[1] * j_idx[2])
                if solid[j]:
                    A[c, j] -= ca                # inflow face: v s.n = -|v s_a|
    return A


def _operator_cases():
    rng = np.random.default_rng(314)
    b = I.bands(rng, 2, 1e-12, 1e-9)
    out = []
    solid = np.ones(6 * 5, dtype=np.uint8)
    solid[[8, 9, 21]] = 0
    g = geo(2, (6, 5), (60e-9, 45e-9), [O.BC_THERMAL, O.BC_DIFFUSE, O.BC_PERIODIC, O.BC_PERIODIC,
                                         O.BC_SPECULAR, O.BC_SPECULAR],
            bcT=[301.0, 300, 300, 300, 300, 300], pdT=(0, 0.7, 0), solid=solid)
    out.append(O.Case(g, dict(b, n_theta=1, n_phi=2, Tref=300.0), P=rng.uniform(0, 1e17, 30),
                      gamma=rng.uniform(0, 1e11, 30)))
    solid = np.ones(4 * 3 * 3, dtype=np.uint8)
    solid[[5, 17]] = 0
    g = geo(3, (4, 3, 3), (40e-9, 30e-9, 30e-9), [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_DIFFUSE, O.BC_SPECULAR,
                                                   O.BC_THERMAL, O.BC_DIFFUSE],
            bcT=[300, 300, 300, 300, 299.0, 300], pdT=(0.5, 0, 0), solid=solid)
    out.append(O.Case(g, dict(b, n_theta=1, n_phi=1, Tref=300.0), gamma=rng.uniform(0, 1e11, 36)))
    g = geo(1, (9,), (45e-9,), [O.BC_THERMAL, O.BC_DIFFUSE] + [O.BC_SPECULAR] * 4,
            bcT=[301.0, 300, 300, 300, 300, 300])
    out.append(O.Case(g, dict(b, n_theta=3, n_phi=1, Tref=300.0), P=rng.uniform(0, 1e17, 9)))
    return out


@pytest.mark.parametrize("lim", [O.LIM_NONE, O.LIM_MC])
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_sweep_is_the_dense_linear_system(idx, lim):
    case = _operator_cases()[idx].with_(limiter=lim)
    rng = np.random.default_rng(7 + idx)
    e = rng.normal(size=case.size) * 50.0
    if case.solid is not None:
        e.reshape(case.nc, -1)[case.solid == 0] = 0.0
    TL = rng.normal(size=case.nc) * 0.3
    b = O.residual(case, e, TLdev=TL).reshape(case.nc, case.na, case.nl)
    out = O.sweep(case, e, TL).reshape(case.nc, case.na, case.nl)
    de = out - e.reshape(case.nc, case.na, case.nl)
    scale = np.abs(de).max()
    for al in range(case.na):
        for l in range(case.nl):
            A = _dense_sweep_operator(case, al, l)
            ref = np.linalg.solve(A, b[:, al, l])
            np.testing.assert_allclose(de[:, al, l], ref, rtol=0, atol=1e-13 * scale)
