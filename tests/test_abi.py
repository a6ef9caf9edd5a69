"""C-ABI library checks that need no GPU: it loads, exports every symbol
declared in include/bte.h, validates arguments and builds the quadrature
on the host (compared with numpy's Gauss-Legendre nodes via the oracle)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import bte_inputs as I
import oracle as O
from tests.helpers import geo, mat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_14181_amd import bte
    return bte.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "bte.h")).read()
    declared = set(re.findall(r"\b(bte_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    from paper_2306_14181_amd import bte
    assert declared == set(bte.EXPORTS)


def _setup(lib, g, m, ctl=None):
    from paper_2306_14181_amd import bte
    s, keep = bte._geometry_struct(g)
    arr = (bte.Geometry * 1)(s)
    bands = [np.ascontiguousarray(m[k], dtype=np.float64) for k in ("C", "v", "tau")]
    mm = bte.Material()
    mm.n_bands = len(bands[0])
    mm.C, mm.v, mm.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in bands]
    mm.n_theta, mm.n_phi, mm.T_ref = m["n_theta"], m.get("n_phi", 1), m["Tref"]
    mm.material_dim = int(m.get("material_dim", 3))
    c = bte.Control()
    for k, v in (ctl or {}).items():
        setattr(c, k, v)
    h = C.c_void_p()
    st = lib.bte_setup(arr, 1, C.byref(mm), C.byref(c), C.byref(h))
    return st, h


@pytest.mark.parametrize("dim,nt,nph", [(1, 8, 1), (2, 2, 8), (3, 4, 4), (3, 3, 4), (2, 2, 4)])
def test_directions_match_oracle_quadrature(lib, dim, nt, nph):
    b = I.bands(0, 2)
    g = geo(dim, (4,) * dim, (1e-7,) * dim, [I.BC_SPECULAR] * 6)
    st, h = _setup(lib, g, mat(b, nt, nph))
    assert st == 0, lib.bte_last_error(h)
    na = lib.bte_num_directions(h)
    s = np.empty((na, 3))
    w = np.empty(na)
    assert lib.bte_get_directions(h, s.ctypes.data_as(C.POINTER(C.c_double)),
                                  w.ctypes.data_as(C.POINTER(C.c_double))) == 0
    so, wo = O.quadrature(dim, nt, nph)
    np.testing.assert_allclose(s, so, atol=2e-15)
    np.testing.assert_allclose(w, wo, rtol=1e-14)
    assert lib.bte_num_unknowns(h) == 4 ** dim * na * 2
    assert lib.bte_workspace_bytes(h) > 0
    lib.bte_destroy(h)


@pytest.mark.parametrize("dim,nt", [(1, 8), (2, 1), (2, 5)])
def test_two_dimensional_material_directions_match_oracle(lib, dim, nt):
    """In-plane directions of a two-dimensional material (total angle 2 pi)."""
    b = I.bands(0, 2)
    g = geo(dim, (4,) * dim, (1e-7,) * dim, [I.BC_SPECULAR] * 6)
    m = mat(b, nt, 1)
    m["material_dim"] = 2
    st, h = _setup(lib, g, m)
    assert st == 0, lib.bte_last_error(h)
    na = lib.bte_num_directions(h)
    s = np.empty((na, 3))
    w = np.empty(na)
    assert lib.bte_get_directions(h, s.ctypes.data_as(C.POINTER(C.c_double)),
                                  w.ctypes.data_as(C.POINTER(C.c_double))) == 0
    so, wo = O.quadrature(dim, nt, 1, material_dim=2)
    np.testing.assert_allclose(s, so, atol=2e-15)
    np.testing.assert_allclose(w, wo, rtol=1e-14)
    lib.bte_destroy(h)


@pytest.mark.parametrize("md", [1, 4, 2])
def test_material_dimension_checked(lib, md):
    """material_dim must be 0, 2 or 3, and a two-dimensional material needs
    a 1D or 2D geometry."""
    b = I.bands(0, 2)
    g = geo(3, (4, 4, 4), (1e-7,) * 3, [I.BC_SPECULAR] * 6)
    m = mat(b, 2, 2)
    m["material_dim"] = md
    st, h = _setup(lib, g, m)
    assert st == 1   # BTE_ERR_ARG
    assert lib.bte_last_error(h)
    lib.bte_destroy(h)


@pytest.mark.parametrize("bad", ["dim", "periodic_pair", "bands", "n_theta", "precision", "dT_nonperiodic",
                                 "all_pores"])
def test_setup_rejects_invalid_arguments(lib, bad):
    b = I.bands(0, 2)
    g = geo(2, (4, 4), (1e-7, 1e-7), [I.BC_THERMAL] * 6)
    m = mat(b, 1, 2)
    ctl = {}
    if bad == "dim":
        g["dim"] = 4
    elif bad == "periodic_pair":
        g["bc"][0] = I.BC_PERIODIC
    elif bad == "bands":
        m["tau"] = np.array([1e-12, -1.0])
    elif bad == "n_theta":
        m["n_theta"] = 0
    elif bad == "precision":
        ctl = {"precision": 7}
    elif bad == "dT_nonperiodic":
        g["pdT"] = [1.0, 0, 0]
    elif bad == "all_pores":
        g["solid"] = np.zeros(16, dtype=np.uint8)
    st, h = _setup(lib, g, m, ctl)
    assert st == 1
    assert len(lib.bte_last_error(h)) > 0
    lib.bte_destroy(h)


def test_device_calls_need_a_workspace(lib):
    b = I.bands(0, 2)
    g = geo(1, (8,), (1e-7,), [I.BC_THERMAL] * 6)
    st, h = _setup(lib, g, mat(b, 2))
    assert st == 0
    dummy = C.c_void_p(0x1000)
    assert lib.bte_moments(h, dummy, None, None, None, None) == 7
    assert lib.bte_steady_solve(h, dummy, 1, None, None) == 7
    assert lib.bte_bind(h, dummy, C.c_size_t(16)) == 1
    lib.bte_destroy(h)


@pytest.mark.parametrize("dim,prec", [(1, 0), (2, 0), (2, 1), (3, 0), (3, 1)])
def test_tile_candidates(lib, dim, prec):
    """Candidate tile shapes: the default first and a choice for every kind
    the kernels have one for (sweeps in 1D: LDS tiles; in 2D: the register
    tile with 2, 1 or (FP32) 4 tile rows per wavefront, written as 8 x 8 x
    rows, then LDS tiles; in 3D: column segments; explicit steps in 1D/2D;
    the one-launch sweep: the 2D register shapes);
    LDS tiles have at most 64 cells; no shape can be set before a workspace
    is bound."""
    b = I.bands(0, 3)
    g = geo(dim, (8,) * dim, (1e-7,) * dim, [I.BC_SPECULAR] * 6)
    st, h = _setup(lib, g, mat(b, 2, 2), {"precision": prec})
    assert st == 0, lib.bte_last_error(h)
    got = {}
    for kind in (0, 1, 2):
        buf = (C.c_int * 96)()
        n = C.c_int()
        assert lib.bte_tile_candidates(h, kind, buf, 32, C.byref(n)) == 0
        shapes = [tuple(buf[3 * i:3 * i + 3]) for i in range(n.value)]
        if kind == 2:
            # the one-launch 2D sweep: the register shapes, nothing in 1D/3D
            assert shapes == ([] if dim != 2 else [(8, 8, 2), (8, 8, 1), (8, 8, 4)] if prec == 0
                              else [(8, 8, 2), (8, 8, 1)])
            got[kind] = shapes
            continue
        reg = [s for s in shapes if dim == 2 and kind == 0 and s[:2] == (8, 8)]
        lds = [s for s in shapes if s not in reg]
        assert all(x * y * z <= 64 and min(x, y, z) >= 1 for x, y, z in lds)
        assert all(s[dim:] == (1,) * (3 - dim) for s in lds)
        if dim == 2 and kind == 0:
            assert reg == ([(8, 8, 2), (8, 8, 1), (8, 8, 4)] if prec == 0 else [(8, 8, 2), (8, 8, 1)])
            assert shapes[:len(reg)] == reg and len(lds) >= 1
        got[kind] = shapes
    # 3D sweeps walk column segments of 1 x 1 x z cells: 16 by default, at
    # most the column height (8 here)
    default_sweep = {1: (64, 1, 1), 2: (8, 8, 2), 3: (1, 1, 8)}[dim]
    assert got[0][0] == default_sweep
    if dim == 3:
        assert all(x == 1 and y == 1 and z <= 8 for x, y, z in got[0]) and len(set(got[0])) == len(got[0])
    assert len(got[0]) > 1
    assert (len(got[1]) > 1) == (dim != 3)
    t = (C.c_int * 3)(*got[0][0])
    assert lib.bte_set_tiles(h, 0, t) == 7   # BTE_ERR_STATE: no workspace
    assert lib.bte_set_tiles(h, 5, t) == 1   # BTE_ERR_ARG
    lib.bte_destroy(h)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_one_launch_sweep_is_the_2d_register_sweeps(lib, dim):
    """bte_set_persistent(1): the 2D sweep in one launch (its work list
    passed the order check at setup: every item after its upwind items);
    refused in 1D and 3D; switching it off is always accepted."""
    b = I.bands(0, 3)
    g = geo(dim, (13,) * dim, (1e-7,) * dim, [I.BC_SPECULAR] * 6)
    st, h = _setup(lib, g, mat(b, 2, 2), {"precision": 0})
    assert st == 0, lib.bte_last_error(h)
    assert lib.bte_set_persistent(h, 0) == 0
    assert lib.bte_set_persistent(h, 1) == (0 if dim == 2 else 2)   # BTE_ERR_UNSUPPORTED
    lib.bte_destroy(h)


def _setup_multi(lib, geos, mats, geo_mat, ifcs):
    from paper_2306_14181_amd import bte
    keep = []
    arr = (bte.Geometry * len(geos))()
    for i, g in enumerate(geos):
        s, k = bte._geometry_struct(g)
        arr[i] = s
        keep.append(k)
    marr = (bte.Material * len(mats))()
    for i, m in enumerate(mats):
        bands = [np.ascontiguousarray(m[k], dtype=np.float64) for k in ("C", "v", "tau")]
        keep.append(bands)
        mm = marr[i]
        mm.n_bands = len(bands[0])
        mm.C, mm.v, mm.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in bands]
        mm.n_theta, mm.n_phi, mm.T_ref = m["n_theta"], m.get("n_phi", 1), m["Tref"]
        mm.material_dim = int(m.get("material_dim", 3))
    gm = (C.c_int * len(geo_mat))(*geo_mat)
    iarr = (bte.Interface * max(len(ifcs), 1))()
    for i, q in enumerate(ifcs):
        ab = np.ascontiguousarray(q["beta_ab"], dtype=np.float64)
        ba = np.ascontiguousarray(q["beta_ba"], dtype=np.float64)
        keep += [ab, ba]
        iarr[i].geo_a, iarr[i].face_a, iarr[i].geo_b, iarr[i].face_b = q["geo_a"], q["face_a"], q["geo_b"], q["face_b"]
        iarr[i].beta_ab = ab.ctypes.data_as(C.POINTER(C.c_double))
        iarr[i].beta_ba = ba.ctypes.data_as(C.POINTER(C.c_double))
    c = bte.Control()
    h = C.c_void_p()
    st = lib.bte_setup_multi(arr, len(geos), marr, len(mats), gm, iarr, len(ifcs), C.byref(c), C.byref(h))
    return st, h


@pytest.mark.parametrize("what", ["ok", "3d", "unmatched_face", "same_side", "no_interface", "beta", "twice",
                                  "bands", "floating"])
def test_setup_multi_validates_interfaces(lib, what):
    """bte_setup_multi: two geometries of two materials joined at A's +x and
    B's -x face (2D, and 3D); each broken variant is refused with
    BTE_ERR_ARG (or BTE_ERR_UNSUPPORTED for a geometry without a
    thermalizing wall), nothing on the device."""
    dim = 3 if what == "3d" else 2
    b = I.bands(0, 3)
    ma, mb = mat(b, 2, 2), mat(dict(b, C=b["C"] * 2.0, v=b["v"] * 0.5), 2, 2)
    if what == "bands":
        mb = mat(I.bands(0, 4), 2, 2)
    n = (6, 5, 4)[:dim]
    nB = (8, 5, 4)[:dim] if what != "unmatched_face" else (8, 4, 4)[:dim]
    bcA = [I.BC_THERMAL, 4] + [I.BC_SPECULAR] * 4
    bcB = [4 if what != "no_interface" else I.BC_DIFFUSE, I.BC_THERMAL if what != "floating" else I.BC_DIFFUSE] \
        + [I.BC_SPECULAR] * 4
    gA = geo(dim, n, tuple(1e-7 * k for k in n), bcA)
    gB = geo(dim, nB, tuple(1e-7 * k for k in nB), bcB)
    q = dict(geo_a=0, face_a=1, geo_b=1, face_b=0 if what != "same_side" else 1,
             beta_ab=np.full(3, 0.4 if what != "beta" else 1.2), beta_ba=np.full(3, 0.5))
    ifcs = [q, q] if what == "twice" else [q]
    st, h = _setup_multi(lib, [gA, gB], [ma, mb], [0, 1], ifcs)
    expect = {"ok": 0, "3d": 0, "floating": 2}.get(what, 1)
    assert st == expect, (what, lib.bte_last_error(h))
    lib.bte_destroy(h)


def test_transient_adjoint_buffer_and_interval(lib):
    """Checkpoint buffer of the transient adjoint: (m + every - 2) states and
    (m + every - 1) T_L fields for m = ceil(n / every); the interval helper
    returns the smallest interval that fits a byte budget."""
    b = I.bands(0, 2)
    g = geo(3, (4, 4, 4), (1e-7,) * 3, [I.BC_THERMAL] * 6)
    st, h = _setup(lib, g, mat(b, 2, 2), dict(precision=1, dt=1e-13, adjoint=1))
    assert st == 0, lib.bte_last_error(h)
    nc = lib.bte_num_cells(h)
    S = 8 * lib.bte_num_unknowns(h)
    size = lambda n, e: lib.bte_transient_adjoint_bytes(h, n, e)
    for n, e in ((500, 50), (500, 1), (500, 2), (7, 3), (1, 1), (5, 9)):
        ee = min(e, n)
        m = -(-n // ee)
        assert size(n, e) == (m + ee - 2) * S + (m + ee - 1) * 8 * nc, (n, e)
    assert size(500, 0) == 0 and size(0, 5) == 0
    pick = lambda n, budget: lib.bte_transient_adjoint_interval(h, n, C.c_size_t(budget))
    assert pick(500, size(500, 1)) == 1
    assert pick(500, size(500, 1) - 1) == 2
    sizes = [size(500, e) for e in range(1, 501)]
    smallest = min(sizes)
    assert sizes.index(smallest) + 1 == 20          # 43 states at every = 20, 21, 22
    assert pick(500, smallest) == 20
    assert pick(500, smallest - 1) == 0
    for budget in (size(500, 3), size(500, 7) + 12345, size(500, 40)):
        e = pick(500, budget)
        assert size(500, e) <= budget and all(size(500, j) > budget for j in range(1, e))
    lib.bte_destroy(h)


def _mesh_setup(lib, mesh, m, **ctl):
    from paper_2306_14181_amd import bte
    ms, keep = bte.mesh_struct(mesh)
    bands = [np.ascontiguousarray(m[k], dtype=np.float64) for k in ("C", "v", "tau")]
    mm = bte.Material()
    mm.n_bands = len(bands[0])
    mm.C, mm.v, mm.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in bands]
    mm.n_theta, mm.n_phi, mm.T_ref = m["n_theta"], m.get("n_phi", 1), m["Tref"]
    mm.material_dim = int(m.get("material_dim", 3))
    c = bte._control_struct(dict(dict(scheme=0, limiter=0), **ctl))
    h = C.c_void_p()
    st = lib.bte_mesh_setup(C.byref(ms), C.byref(mm), C.byref(c), C.byref(h))
    return st, h, keep


MESH_MAT = dict(C=np.array([1e5, 2e5, 3e5]), v=np.array([1000.0, 2000.0, 3000.0]),
                tau=np.array([1e-10, 3e-10, 2e-11]), n_theta=2, n_phi=2, Tref=300.0)


def test_mesh_levels_match_the_oracle_upwind_graphs(lib):
    """The host schedule: one level per step of the deepest direction's
    dependency graph (computed here from the oracle's upwind order)."""
    from oracle import mesh as M
    mesh = I.mesh2d(3, 9, 7, 9e-7, 7e-7, jitter=0.3, quad_frac=0.4)
    st, h, keep = _mesh_setup(lib, mesh, MESH_MAT)
    assert st == 0, lib.bte_mesh_last_error(h)
    mc = M.MeshCase(mesh, MESH_MAT)
    depth = 0
    for al in range(mc.na):
        order, lagged = M.upwind_order(mc, al)
        lev = {}
        for c in order:
            ups = [nb for nb, _, _, n, _ in mc.faces[c]
                   if nb >= 0 and mc.s[al, 0] * n[0] + mc.s[al, 1] * n[1] < 0 and (c, nb) not in lagged]
            lev[c] = 1 + max((lev[j] for j in ups), default=-1)
        depth = max(depth, max(lev.values()))
    assert lib.bte_mesh_num_levels(h) == depth + 1
    assert lib.bte_mesh_num_lagged(h) == 0
    assert lib.bte_mesh_num_cells(h) == mc.nc and lib.bte_mesh_num_directions(h) == mc.na
    assert lib.bte_mesh_workspace_bytes(h) > 0
    lib.bte_mesh_destroy(h)


@pytest.mark.parametrize("what", ["cw", "pentagon", "untagged", "tag_range", "slanted_specular", "synthetic",
                                  "limiter", "planar", "shared3", "stencil"])
def test_mesh_setup_validates(lib, what):
    mesh = I.mesh2d(1, 4, 3, 4e-7, 3e-7, jitter=0.2, quad_frac=0.5)
    mesh = {k: np.array(v, copy=True) for k, v in mesh.items()}
    ctl, mat, want = {}, dict(MESH_MAT), 1
    if what == "cw":
        a, b = mesh["cell_ptr"][0], mesh["cell_ptr"][1]
        mesh["cell_vtx"][a:b] = mesh["cell_vtx"][a:b][::-1].copy()
    elif what == "pentagon":
        mesh["cell_ptr"] = mesh["cell_ptr"].copy()
        mesh["cell_ptr"][1] = 5
    elif what == "untagged":
        i = int(np.flatnonzero(mesh["edge_tag"] >= 0)[0])
        mesh["edge_tag"][i] = -1
    elif what == "tag_range":
        i = int(np.flatnonzero(mesh["edge_tag"] >= 0)[0])
        mesh["edge_tag"][i] = 7
    elif what == "slanted_specular":
        # a specular wall on a slanted edge: move a corner vertex inward
        mesh["tag_bc"][:] = I.BC_SPECULAR
        mesh["xy"][0] = [0.3e-7, 0.2e-7]
    elif what == "stencil":
        mesh["gradient_stencil"] = 2
    elif what == "synthetic":
        ctl, want = dict(scheme=1), 2
    elif what == "limiter":
        ctl, want = dict(limiter=1), 2
    elif what == "planar":
        mat["material_dim"], want = 2, 2
    elif what == "shared3":
        # a third cell on an existing edge
        ptr, vtx = mesh["cell_ptr"], mesh["cell_vtx"]
        mesh["cell_vtx"] = np.concatenate([vtx, vtx[ptr[0]:ptr[0] + 2][::-1], [len(mesh["xy"])]]).astype(np.int32)
        mesh["cell_ptr"] = np.concatenate([ptr, [ptr[-1] + 3]]).astype(np.int32)
        mesh["edge_tag"] = np.concatenate([mesh["edge_tag"], [-1, 0, 0]]).astype(np.int32)
        mesh["xy"] = np.concatenate([mesh["xy"], [[0.5e-7, -1e-7]]])
    st, h, keep = _mesh_setup(lib, mesh, mat, **ctl)
    assert st == want, (what, st, lib.bte_mesh_last_error(h))
    assert len(lib.bte_mesh_last_error(h)) > 0
    lib.bte_mesh_destroy(h)


def test_tet_mesh_levels_and_lagging_match_the_oracle(lib):
    """Tetrahedral schedule: levels and lagged couplings (3D upwind graphs
    may have cycles) as the oracle's rule gives them."""
    from paper_2306_14181_amd import bte
    from oracle import mesh as M
    mesh = I.mesh3d(2, 4, 4, 3, 4e-7, 4e-7, 3e-7, jitter=0.15)
    ms, keep = bte.mesh_struct(mesh)
    bands = [np.ascontiguousarray(MESH_MAT[k], dtype=np.float64) for k in ("C", "v", "tau")]
    mm = bte.Material()
    mm.n_bands = 3
    mm.C, mm.v, mm.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in bands]
    mm.n_theta, mm.n_phi, mm.T_ref, mm.material_dim = 2, 2, 300.0, 3
    c = bte._control_struct(dict(scheme=0, limiter=0))
    h = C.c_void_p()
    st = lib.bte_mesh_setup_tet(C.byref(ms), C.byref(mm), C.byref(c), C.byref(h))
    assert st == 0, lib.bte_mesh_last_error(h)
    mc = M.TetMeshCase(mesh, MESH_MAT)
    depth, nlag = 0, 0
    for al in range(mc.na):
        order, lagged = M.upwind_order(mc, al)
        nlag += len(lagged)
        lev = {}
        for cc in order:
            ups = [nb for nb, _, _, n, _ in mc.faces[cc]
                   if nb >= 0 and mc.s[al] @ n < 0 and (cc, nb) not in lagged]
            lev[cc] = 1 + max((lev[j] for j in ups), default=-1)
        depth = max(depth, max(lev.values()))
    assert lib.bte_mesh_num_levels(h) == depth + 1
    assert lib.bte_mesh_num_lagged(h) == nlag
    assert lib.bte_mesh_num_cells(h) == mc.nc and lib.bte_mesh_num_directions(h) == mc.na
    lib.bte_mesh_destroy(h)
