"""Pins of the unstructured-mesh oracle (oracle/mesh.py; Sec. 3.3 eq.
disretized_BTE with the least-squares gradient, Sec. 3.5's stiffness matrix).

* Cartesian reduction: on a uniform grid of quadrilaterals the least-squares
  gradient is the central (one-sided at a wall) difference, so residual,
  moments and one sweep equal the structured-grid oracle's, which is pinned
  on its own, for thermalizing, specular and diffuse walls.
* Linear exactness on distorted hybrid meshes: the least-squares gradient of
  a linear field is exact on any mesh, and so is the second-order face
  value; the flux divergence of every cell away from the walls is then
  v s . grad e exactly (a wrong l vector, upwind side or normal fails).
* Geometry: the areas sum to the rectangle's, every cell is closed
  (sum_f n S = 0) and its normals point outward.
* Conservation: with adiabatic walls (specular, diffuse) the total flux
  divergence sum_i V_i sum_k w D vanishes for any state.
* Equilibrium: e = C dT / 4 pi with every wall thermalizing at T_ref + dT is
  a fixed point (R = 0).
* Sweep: the increment solves A de = R with A assembled here from the
  geometry (first-order upwind operator of Sec. 3.5), lane by lane.
* Upwind order: no coupling is lagged on these meshes (2D conforming meshes
  of convex cells give acyclic graphs), and a hand-built cycle is lagged by
  the stated rule.
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from oracle import mesh as M

MAT = dict(C=np.array([1e5, 2e5, 3e5]), v=np.array([1000.0, 2000.0, 3000.0]),
           tau=np.array([1e-10, 3e-10, 2e-11]), n_theta=2, n_phi=2, Tref=300.0)


def structured(nx, ny, lx, ly, bc4, bcT4):
    g = dict(dim=2, n=[nx, ny, 1], len=[lx, ly, 1.0], bc=list(bc4) + [O.BC_SPECULAR] * 2,
             bcT=list(bcT4) + [300.0, 300.0], pdT=[0.0, 0.0, 0.0], pore_bc=O.BC_DIFFUSE)
    return O.Case(g, MAT)


@pytest.mark.parametrize("bc4", [(O.BC_THERMAL, O.BC_THERMAL, O.BC_SPECULAR, O.BC_SPECULAR),
                                 (O.BC_DIFFUSE, O.BC_THERMAL, O.BC_DIFFUSE, O.BC_SPECULAR),
                                 (O.BC_SPECULAR, O.BC_DIFFUSE, O.BC_THERMAL, O.BC_DIFFUSE)])
def test_cartesian_mesh_equals_the_structured_oracle(bc4):
    nx, ny, lx, ly = 6, 5, 6e-7, 5e-7
    bcT4 = (301.0, 299.5, 300.5, 299.0)
    mc = M.MeshCase(I.mesh2d(0, nx, ny, lx, ly, jitter=0.0, quad_frac=1.0, bc=bc4, bcT=bcT4, gradient_stencil=1),
                    MAT, P=np.linspace(0, 1e15, nx * ny))
    sc = structured(nx, ny, lx, ly, bc4, bcT4).with_(P=np.linspace(0, 1e15, nx * ny))
    rng = np.random.default_rng(1)
    e = rng.normal(size=sc.size) * 1e3
    TL = rng.normal(size=sc.nc)
    R1, R2 = M.residual(mc, e, TL), O.residual(sc, e, TL)
    assert np.abs(R1 - R2).max() <= 1e-13 * np.abs(R2).max()
    s1, s2 = M.sweep(mc, e, TL), O.sweep(sc, e, TL)
    assert np.abs(s1 - s2).max() <= 1e-13 * np.abs(s2).max()
    T1, TL1, q1 = M.moments(mc, e)
    T2, TL2, q2 = O.moments(sc, e)
    assert np.abs(T1 - T2).max() <= 1e-12 and np.abs(TL1 - TL2).max() <= 1e-12
    assert np.abs(q1 - q2).max() <= 1e-13 * np.abs(q2).max()


def hybrid(seed=3, nx=7, ny=6, bc=(O.BC_THERMAL, O.BC_THERMAL, O.BC_SPECULAR, O.BC_SPECULAR)):
    return I.mesh2d(seed, nx, ny, 7e-7, 6e-7, jitter=0.3, quad_frac=0.4, bc=bc)


def test_geometry_closed_cells_outward_normals_total_area():
    mc = M.MeshCase(hybrid(), MAT)
    assert abs(mc.V.sum() - 7e-7 * 6e-7) <= 1e-12 * 7e-7 * 6e-7
    for c in range(mc.nc):
        tot = sum(S * n for _, _, S, n, _ in mc.faces[c])
        assert np.abs(tot).max() <= 1e-12 * 1e-7
        for _, _, _, n, xf in mc.faces[c]:
            assert n @ (xf - mc.xc[c]) > 0
    # both kinds of cell occur
    sides = {len(f) for f in mc.faces}
    assert sides == {3, 4}
    # the cell centre is the area centroid: the area-weighted mean of the
    # centroids of a triangle fan from the first vertex
    m = hybrid()
    xy, ptr, vtx = m["xy"], m["cell_ptr"], m["cell_vtx"]
    for c in range(mc.nc):
        P = xy[vtx[ptr[c]:ptr[c + 1]]]
        num, den = np.zeros(2), 0.0
        for k in range(1, len(P) - 1):
            a, b = P[k] - P[0], P[k + 1] - P[0]
            A = 0.5 * (a[0] * b[1] - a[1] * b[0])
            num += A * (P[0] + P[k] + P[k + 1]) / 3.0
            den += A
        assert np.abs(mc.xc[c] - num / den).max() <= 1e-12 * 1e-7
        assert abs(mc.V[c] - den) <= 1e-12 * den


@pytest.mark.parametrize("stencil", [0, 1])
def test_least_squares_gradient_and_face_values_exact_for_linear_fields(stencil):
    mc = M.MeshCase(dict(hybrid(), gradient_stencil=stencil), MAT)
    rng = np.random.default_rng(2)
    a0, ax, ay = (rng.normal(size=mc.nk) for _ in range(3))
    ax, ay = ax * 1e9, ay * 1e9
    e = a0[None, :] + mc.xc[:, :1] * ax[None, :] + mc.xc[:, 1:] * ay[None, :]
    g = M.grad(mc, e)
    assert np.abs(g[:, 0] - ax).max() <= 1e-9 * np.abs(ax).max()
    assert np.abs(g[:, 1] - ay).max() <= 1e-9 * np.abs(ay).max()
    # interior cells (no boundary face, no boundary-touching upwind
    # neighbour needed): D = v s . grad e
    D = M.flux_div(mc, e.reshape(-1)).reshape(mc.nc, mc.nk)
    v = mc.lanes_v()
    sx, sy = np.repeat(mc.s[:, 0], mc.nl), np.repeat(mc.s[:, 1], mc.nl)
    exact = v * (sx * ax + sy * ay)
    interior = [c for c in range(mc.nc) if all(nb >= 0 for nb, *_ in mc.faces[c])]
    assert len(interior) > 10
    for c in interior:
        assert np.abs(D[c] - exact).max() <= 1e-8 * np.abs(exact).max()


PORES = [(2.2e-7, 3.0e-7, 1.1e-7), (5.3e-7, 2.0e-7, 0.8e-7)]


@pytest.mark.parametrize("bc,pores", [((O.BC_SPECULAR,) * 4, ()),
                                      ((O.BC_DIFFUSE, O.BC_SPECULAR, O.BC_DIFFUSE, O.BC_DIFFUSE), ()),
                                      ((O.BC_SPECULAR,) * 4, PORES)])
def test_adiabatic_walls_conserve_energy_for_any_state(bc, pores):
    mesh = I.mesh2d(3, 7, 6, 7e-7, 6e-7, jitter=0.3, quad_frac=0.4, bc=bc, pores=pores)
    if pores:
        assert (mesh["edge_tag"] == 4).sum() > 8     # pore surfaces (diffuse)
    mc = M.MeshCase(mesh, MAT)
    rng = np.random.default_rng(4)
    for _ in range(2):
        e = rng.normal(size=mc.size) * 1e3
        D = M.flux_div(mc, e).reshape(mc.nc, mc.na, mc.nl)
        tot = np.einsum("c,a,cal->", mc.V, mc.w, D)
        scale = np.einsum("c,a,cal->", mc.V, mc.w, np.abs(D))
        assert abs(tot) <= 1e-13 * scale


def test_equilibrium_is_a_fixed_point():
    dT = 1.5
    mc = M.MeshCase(I.mesh2d(5, 6, 5, 6e-7, 5e-7, jitter=0.3, quad_frac=0.5,
                             bc=(O.BC_THERMAL,) * 4, bcT=(301.5,) * 4), MAT)
    e = np.tile(mc.lanes_C4() * dT, mc.nc)
    R = M.residual(mc, e)
    assert np.abs(R).max() <= 1e-12 * np.abs(e).max() / mc.tau.min()


def test_sweep_solves_the_first_order_upwind_system():
    mc = M.MeshCase(hybrid(seed=7, nx=5, ny=4), MAT)
    rng = np.random.default_rng(5)
    e = rng.normal(size=mc.size) * 1e3
    TL = rng.normal(size=mc.nc)
    b = M.residual(mc, e, TL).reshape(mc.nc, mc.na, mc.nl)
    de = (M.sweep(mc, e, TL) - e).reshape(mc.nc, mc.na, mc.nl)
    for al in range(mc.na):
        s = mc.s[al]
        for l in range(mc.nl):
            A = np.diag(np.full(mc.nc, 1.0 / mc.tau[l]))
            for c in range(mc.nc):
                for nb, _, S, n, _ in mc.faces[c]:
                    sn = s[0] * n[0] + s[1] * n[1]
                    if sn > 0:
                        A[c, c] += mc.v[l] * sn * S / mc.V[c]
                    elif sn < 0 and nb >= 0:
                        A[c, nb] -= mc.v[l] * (-sn) * S / mc.V[c]
            r = A @ de[:, al, l] - b[:, al, l]
            assert np.abs(r).max() <= 1e-12 * np.abs(b[:, al, l]).max()


def test_no_lagging_on_conforming_meshes_and_the_cycle_rule():
    mc = M.MeshCase(hybrid(seed=9, nx=8, ny=7), MAT)
    for al in range(mc.na):
        order, lagged = M.upwind_order(mc, al)
        assert sorted(order) == list(range(mc.nc)) and not lagged
    # a three-cell cycle built by hand (cells 0 -> 1 -> 2 -> 0 plus a cell 3
    # downstream of 2): the smallest-index cell, 0, is taken first with its
    # coupling to 2 lagged

    class Ring:
        nc = 4
        s = np.array([[1.0, 0.0, 0.0]])

    r = Ring()
    out = lambda nb: (nb, -1, 1.0, np.array([-1.0, 0.0]), None)   # noqa: E731  inflow from nb
    r.faces = [[out(2)], [out(0)], [out(1)], [out(2)]]
    order, lagged = M.upwind_order(r, 0)
    assert order == [0, 1, 2, 3] and lagged == {(0, 2)}


def test_vertex_stencil_on_a_cartesian_grid_is_the_three_by_three_fit():
    """Interior cell of a uniform grid: the eight cells around it, X =
    diag(6 hx^2, 6 hy^2), so d e/dx = (east column - west column) / (6 hx)."""
    nx, ny, hx, hy = 5, 4, 60e-9, 50e-9
    mc = M.MeshCase(I.mesh2d(0, nx, ny, nx * hx, ny * hy, jitter=0.0, quad_frac=1.0), MAT)
    rng = np.random.default_rng(6)
    e = rng.normal(size=(mc.nc, mc.nk))
    g = M.grad(mc, e)
    at = lambda i, j: e[i + nx * j]   # noqa: E731
    for (i, j) in [(1, 1), (2, 2), (3, 1)]:
        gx = (at(i + 1, j - 1) + at(i + 1, j) + at(i + 1, j + 1) - at(i - 1, j - 1) - at(i - 1, j) - at(i - 1, j + 1))
        gy = (at(i - 1, j + 1) + at(i, j + 1) + at(i + 1, j + 1) - at(i - 1, j - 1) - at(i, j - 1) - at(i + 1, j - 1))
        c = i + nx * j
        assert np.abs(g[c, 0] - gx / (6 * hx)).max() <= 1e-6 * np.abs(gx / hx).max()
        assert np.abs(g[c, 1] - gy / (6 * hy)).max() <= 1e-6 * np.abs(gy / hy).max()


def test_sequential_iteration_contracts_on_triangles_with_the_vertex_stencil():
    """The iteration e <- e + A^-1 R(e) converges on a distorted triangle
    mesh (ratio of successive updates below 1): the property the paper
    relies on for its sequential scheme."""
    mesh = I.mesh2d(13, 10, 8, 10 * 60e-9, 8 * 50e-9, jitter=0.3, quad_frac=0.0, bc=(I.BC_THERMAL,) * 4)
    mc = M.MeshCase(mesh, dict(MAT, tau=np.array([2e-9, 1e-9, 5e-10])))
    e = mc.zeros()
    prev, ratios = None, []
    for _ in range(15):
        e1 = M.sweep(mc, e, M.moments(mc, e)[1] - mc.Tref)
        d = np.abs(e1 - e).max()
        if prev:
            ratios.append(d / prev)
        prev, e = d, e1
    assert max(ratios[-5:]) < 0.7, ratios


def test_explicit_steps_conserve_energy_with_adiabatic_walls():
    """Algorithm 2 on the mesh: with specular and diffuse walls and no
    source, sum_i V_i sum_k w e is invariant (the flux divergence sums to
    zero and the scattering term sum w (e - C T_L / 4 pi) / tau vanishes by
    the definition of T_L); taking T_L from the wrong moment breaks it."""
    mc = M.MeshCase(hybrid(bc=(I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_DIFFUSE, I.BC_SPECULAR)), MAT)
    rng = np.random.default_rng(8)
    e0 = rng.normal(size=mc.size) * 1e3
    energy = lambda x: np.einsum("c,a,cal->", mc.V, mc.w, x.reshape(mc.nc, mc.na, mc.nl))   # noqa: E731
    e1 = M.transient(mc, e0, 5, 1e-13)
    scale = np.einsum("c,a,cal->", mc.V, mc.w, np.abs(e0.reshape(mc.nc, mc.na, mc.nl)))
    assert abs(energy(e1) - energy(e0)) <= 1e-12 * scale
    assert np.abs(e1 - e0).max() > 1e-3 * np.abs(e0).max()     # the state did move


# ---------------------------------------------------------------- tetrahedra

def tets(seed=1, n=(4, 3, 3), bc=(O.BC_THERMAL, O.BC_THERMAL) + (O.BC_SPECULAR,) * 4, **kw):
    L = [x * 1e-7 for x in n]
    return I.mesh3d(seed, *n, *L, jitter=0.15, bc=bc, **kw)


def test_tet_geometry_closed_cells_outward_normals_total_volume():
    mc = M.TetMeshCase(tets(), MAT)
    assert abs(mc.V.sum() - 4e-7 * 3e-7 * 3e-7) <= 1e-12 * 3.6e-20
    for c in range(mc.nc):
        tot = sum(S * n for _, _, S, n, _ in mc.faces[c])
        assert np.abs(tot).max() <= 1e-12 * 1e-14
        for _, _, _, n, xf in mc.faces[c]:
            assert n @ (xf - mc.xc[c]) > 0
        # volume from the divergence theorem: V = (1/3) sum_f (x_f . n) S
        assert abs(sum(xf @ n * S for _, _, S, n, xf in mc.faces[c]) / 3.0 - mc.V[c]) <= 1e-10 * mc.V[c]


@pytest.mark.parametrize("stencil", [0, 1])
def test_tet_gradient_and_flux_divergence_exact_for_linear_fields(stencil):
    mc = M.TetMeshCase(dict(tets(n=(5, 4, 4)), gradient_stencil=stencil), MAT)
    rng = np.random.default_rng(2)
    a0, ax, ay, az = (rng.normal(size=mc.nk) for _ in range(4))
    ax, ay, az = ax * 1e9, ay * 1e9, az * 1e9
    e = a0[None, :] + mc.xc[:, :1] * ax + mc.xc[:, 1:2] * ay + mc.xc[:, 2:] * az
    g = M.grad(mc, e)
    # exact wherever the stencil spans space (with the face stencil a
    # boundary tetrahedron may have one or two neighbours: pseudo-inverse)
    full = np.array([np.linalg.matrix_rank(mc.Xinv[c]) == 3 for c in range(mc.nc)])
    assert full.mean() > (0.999 if stencil == 0 else 0.6)
    for q, a in enumerate((ax, ay, az)):
        assert np.abs(g[full, q] - a).max() <= 1e-8 * np.abs(a).max()
    D = M.flux_div(mc, e.reshape(-1)).reshape(mc.nc, mc.nk)
    sx, sy, sz = (np.repeat(mc.s[:, q], mc.nl) for q in range(3))
    exact = mc.lanes_v() * (sx * ax + sy * ay + sz * az)
    interior = [c for c in range(mc.nc) if all(nb >= 0 and full[nb] for nb, *_ in mc.faces[c]) and full[c]]
    assert len(interior) > 20
    for c in interior:
        assert np.abs(D[c] - exact).max() <= 1e-8 * np.abs(exact).max()


@pytest.mark.parametrize("bc,pores", [((O.BC_SPECULAR,) * 6, ()),
                                      ((O.BC_DIFFUSE, O.BC_SPECULAR) * 3, ()),
                                      ((O.BC_SPECULAR,) * 6, [(2e-7, 1.5e-7, 1.5e-7, 0.9e-7)])])
def test_tet_adiabatic_walls_conserve_energy(bc, pores):
    mesh = tets(bc=bc, pores=pores)
    if pores:
        assert (mesh["face_tag"] == 6).sum() > 8
    mc = M.TetMeshCase(mesh, MAT)
    e = np.random.default_rng(4).normal(size=mc.size) * 1e3
    D = M.flux_div(mc, e).reshape(mc.nc, mc.na, mc.nl)
    tot = np.einsum("c,a,cal->", mc.V, mc.w, D)
    assert abs(tot) <= 1e-13 * np.einsum("c,a,cal->", mc.V, mc.w, np.abs(D))
    e1 = M.transient(mc, e, 3, 1e-13)
    energy = lambda x: np.einsum("c,a,cal->", mc.V, mc.w, x.reshape(mc.nc, mc.na, mc.nl))   # noqa: E731
    assert abs(energy(e1) - energy(e)) <= 1e-12 * np.einsum("c,a,cal->", mc.V, mc.w, np.abs(e.reshape(mc.nc, mc.na, mc.nl)))


def test_tet_equilibrium_and_sweep_system():
    mc = M.TetMeshCase(tets(bc=(O.BC_THERMAL,) * 6, bcT=(301.5,) * 6), MAT)
    e = np.tile(mc.lanes_C4() * 1.5, mc.nc)
    assert np.abs(M.residual(mc, e)).max() <= 1e-12 * np.abs(e).max() / mc.tau.min()
    rng = np.random.default_rng(5)
    e = rng.normal(size=mc.size) * 1e3
    TL = rng.normal(size=mc.nc)
    b = M.residual(mc, e, TL).reshape(mc.nc, mc.na, mc.nl)
    de = (M.sweep(mc, e, TL) - e).reshape(mc.nc, mc.na, mc.nl)
    for al in range(0, mc.na, 5):
        _, lagged = M.upwind_order(mc, al)
        for l in range(mc.nl):
            A = np.diag(np.full(mc.nc, 1.0 / mc.tau[l]))
            for c in range(mc.nc):
                for nb, _, S, n, _ in mc.faces[c]:
                    sn = mc.s[al] @ n
                    if sn > 0:
                        A[c, c] += mc.v[l] * sn * S / mc.V[c]
                    elif sn < 0 and nb >= 0 and (c, nb) not in lagged:
                        A[c, nb] -= mc.v[l] * (-sn) * S / mc.V[c]
            r = A @ de[:, al, l] - b[:, al, l]
            assert np.abs(r).max() <= 1e-12 * np.abs(b[:, al, l]).max()
