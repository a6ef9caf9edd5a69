"""FP64 oracle of the steady BTE on unstructured two-dimensional meshes of
triangles and quadrilaterals (test infrastructure only: imported by
``tests/`` alone, shares no code with the HIP library).

What it computes, in the paper's notation (Sec. 3.3, eq. disretized_BTE,
with the stiffness matrix and right-hand side of Sec. 3.5):

* cell i of volume (area) V_i, faces ij of length S_ij, exterior unit normal
  n_ij, centre x_f; cell centre x_i = the polygon's centroid;
* least-squares gradient (Sec. 3.3, the matrix X of Sec. 3.5): over the
  stencil cells j of i, d_ij = x_j - x_i, X_i = sum_j d_ij d_ij^T and
  grad e_i = X_i^+ sum_j d_ij (e_j - e_i)  (boundary faces do not enter;
  X^+ is the inverse, or the pseudo-inverse with eigenvalues below 1e-10 of
  the largest dropped when the offsets do not span the plane).  The paper
  does not name the stencil: mesh["gradient_stencil"] = 0 (default) takes
  every cell sharing a vertex with i, 1 the face neighbours only (on a
  Cartesian grid that is the central / one-sided difference of the
  structured-grid oracle; on triangles it makes the sequential iteration
  diverge, the vertex stencil does not);
* second-order upwind face value: e_ij = e_m + grad e_m . l_{m,ij} with m the
  upwind cell (s . n_ij > 0 for m) and l the vector from x_m to x_f;
  across a boundary face the incoming value is the wall's (Sec. 2.2):
  thermalizing C (T_w - T_ref) / 4 pi; specular the mirror direction's
  outgoing face value (edges parallel to x or y only, where the mirror is a
  quadrature direction); diffuse the outgoing energy flux of the face over
  the incoming weight, sum_{s.n>0} w s.n e_f / sum_{s.n<0} w |s.n|;
* residual R_i = -(1/V_i) sum_j v (s . n_ij) S_ij e_ij - (e_i - e0_i)/tau + Q_i
  with e0 = C T_L / 4 pi and Q = P C / (4 pi C_tot);
* moments as on the structured grids: T = T_ref + sum w e / C_tot,
  T_L = T_ref + sum w e / tau / sum C / tau, q = sum w v s e;
* one source iteration (sequential scheme, Sec. 3.4): T_L from the moments
  of e^n, then A de = R(e^n) with the first-order upwind operator
  A_ii = 1/tau + (1/V_i) sum_{s.n>0} v s.n S, A_ij = -(1/V_i) v |s.n| S for
  the upwind neighbour j across an interior face (wall inflow enters R
  only), solved by marching the cells of each direction in upwind order,
  e^{n+1} = e^n + de;
* an explicit transient step (Sec. 4.1, Algorithm 2): e^{n+1} = e^n +
  dt R(e^n), T_L from the moments of e^n.

Upwind order: for each direction the cells form a dependency graph (i
depends on j when j is upwind across an interior face).  Cells are taken in
Kahn order; if the graph has a cycle, the smallest-index cell left is taken
with its unresolved upwind couplings lagged (their increments count as zero
in that iteration), and Kahn order resumes.  The lagged set depends only on
the graph, so any implementation of this rule lags the same couplings.
"""
import numpy as np

from .oracle import quadrature, BC_THERMAL, BC_SPECULAR, BC_DIFFUSE

FOURPI = 4.0 * np.pi


class MeshCase:
    """Mesh (dict of xy, cell_ptr, cell_vtx, edge_tag, tag_bc, tag_T: see
    bte_inputs.mesh2d) + bands (dict C, v, tau, n_theta, n_phi, Tref) + an
    optional heat source P[nc] (W/m^3)."""

    def __init__(self, mesh, material, P=None):
        xy = np.asarray(mesh["xy"], dtype=np.float64)
        ptr = np.asarray(mesh["cell_ptr"], dtype=np.int64)
        vtx = np.asarray(mesh["cell_vtx"], dtype=np.int64)
        etag = np.asarray(mesh["edge_tag"], dtype=np.int64)
        self.tag_bc = np.asarray(mesh["tag_bc"], dtype=np.int64)
        self.tag_T = np.asarray(mesh["tag_T"], dtype=np.float64)
        nc = len(ptr) - 1
        self.nc = nc
        self.dim = 2
        # polygon area and centroid (shoelace)
        self.V = np.zeros(nc)
        self.xc = np.zeros((nc, 2))
        for c in range(nc):
            P_ = xy[vtx[ptr[c]:ptr[c + 1]]]
            Q_ = np.roll(P_, -1, axis=0)
            cr = P_[:, 0] * Q_[:, 1] - Q_[:, 0] * P_[:, 1]
            A = 0.5 * cr.sum()
            self.V[c] = A
            self.xc[c] = ((P_ + Q_) * cr[:, None]).sum(axis=0) / (6.0 * A)
        # faces: edge k of cell c runs from vertex k to vertex k + 1
        owner = {}
        for c in range(nc):
            m = ptr[c + 1] - ptr[c]
            for k in range(m):
                a, b = vtx[ptr[c] + k], vtx[ptr[c] + (k + 1) % m]
                owner.setdefault((min(a, b), max(a, b)), []).append(c)
        self.faces = []   # per cell: list of (neighbour or -1, tag, S, n[2], xf[2])
        for c in range(nc):
            m = ptr[c + 1] - ptr[c]
            fl = []
            for k in range(m):
                a, b = vtx[ptr[c] + k], vtx[ptr[c] + (k + 1) % m]
                d = xy[b] - xy[a]
                S = float(np.hypot(d[0], d[1]))
                n = np.array([d[1], -d[0]]) / S     # exterior for a counter-clockwise cell
                xf = 0.5 * (xy[a] + xy[b])
                others = [o for o in owner[(min(a, b), max(a, b))] if o != c]
                nb = others[0] if others else -1
                tag = int(etag[ptr[c] + k])
                if nb < 0 and tag < 0:
                    raise ValueError("boundary edge without a tag")
                fl.append((nb, tag, S, n, xf))
            self.faces.append(fl)
        # least-squares stencils: cells sharing a vertex (0) or a face (1)
        self.stencil = int(mesh.get("gradient_stencil", 0))
        if self.stencil == 0:
            vcells = {}
            for c in range(nc):
                for v in vtx[ptr[c]:ptr[c + 1]]:
                    vcells.setdefault(int(v), set()).add(c)
            self.lsn = []
            for c in range(nc):
                near = set()
                for v in vtx[ptr[c]:ptr[c + 1]]:
                    near |= vcells[int(v)]
                near.discard(c)
                self.lsn.append(sorted(near))
        else:
            self.lsn = [[nb for nb, _, _, _, _ in self.faces[c] if nb >= 0] for c in range(nc)]
        # least-squares matrices; a cell whose offsets do not span the plane
        # (one neighbour) takes the pseudo-inverse: the gradient along the
        # offsets it has, none across them (on a Cartesian grid with the face
        # stencil: zero slope along an axis without neighbours, as the
        # structured oracle)
        self.Xinv = np.zeros((nc, 2, 2))
        for c in range(nc):
            X = np.zeros((2, 2))
            for nb in self.lsn[c]:
                d = self.xc[nb] - self.xc[c]
                X += np.outer(d, d)
            self.Xinv[c] = np.linalg.pinv(X, rcond=1e-10, hermitian=True)
        m = material
        self.s, self.w = quadrature(2, int(m["n_theta"]), int(m.get("n_phi", 1)), 3)
        self.C = np.asarray(m["C"], dtype=np.float64)
        self.v = np.asarray(m["v"], dtype=np.float64)
        self.tau = np.asarray(m["tau"], dtype=np.float64)
        self.Tref = float(m["Tref"])
        self.na, self.nl = len(self.w), len(self.C)
        self.nk = self.na * self.nl
        self.C4 = self.C / FOURPI
        self.Ctot = self.C.sum()
        self.Ssum = (self.C / self.tau).sum()
        self.P = None if P is None else np.asarray(P, dtype=np.float64)
        # mirror directions for walls parallel to x (flip s_y) or y (flip s_x)
        self.mirror = np.zeros((2, self.na), dtype=np.int64)
        for a in range(2):
            for al in range(self.na):
                t = self.s[al].copy()
                t[a] = -t[a]
                dd = np.abs(self.s - t).sum(axis=1)
                self.mirror[a, al] = int(np.argmin(dd))
        for c in range(nc):
            for nb, tag, _, n, _ in self.faces[c]:
                if nb < 0 and self.tag_bc[tag] == BC_SPECULAR and min(abs(n[0]), abs(n[1])) > 1e-12:
                    raise ValueError("specular walls must be parallel to x or y")
        self._order = None

    @property
    def size(self):
        return self.nc * self.nk

    def zeros(self):
        return np.zeros(self.size)

    def sn(self, n):
        """s . n for every direction (n has the mesh's dimension)."""
        out = self.s[:, 0] * n[0] + self.s[:, 1] * n[1]
        return out + self.s[:, 2] * n[2] if len(n) == 3 else out

    def lanes_v(self):
        return np.tile(self.v, self.na)           # v of lane k = al * nl + l

    def lanes_tau(self):
        return np.tile(self.tau, self.na)

    def lanes_C4(self):
        return np.tile(self.C4, self.na)


def _dot(s, n):
    """s . n with n in the mesh's dimension."""
    out = s[0] * n[0] + s[1] * n[1]
    return out + s[2] * n[2] if len(n) == 3 else out


def grad(case, e):
    """Least-squares gradient [nc, dim, nk] (Sec. 3.3)."""
    e = np.asarray(e, dtype=np.float64).reshape(case.nc, case.nk)
    D = case.dim
    g = np.zeros((case.nc, D, case.nk))
    for c in range(case.nc):
        y = np.zeros((D, case.nk))
        for nb in case.lsn[c]:
            d = case.xc[nb] - case.xc[c]
            y += np.outer(d, e[nb] - e[c])
        g[c] = case.Xinv[c] @ y
    return g


def _face_out(case, e, g, c, xf):
    """Outgoing second-order face value of cell c at face centre xf, all lanes."""
    l = xf - case.xc[c]
    out = e[c] + g[c, 0] * l[0] + g[c, 1] * l[1]
    return out + g[c, 2] * l[2] if case.dim == 3 else out


def _wall_in(case, e, g, c, tag, n, xf):
    """Incoming value of every lane at the boundary face (only the lanes with
    s . n < 0 are used)."""
    kind = case.tag_bc[tag]
    nl = case.nl
    if kind == BC_THERMAL:
        return np.tile(case.C4 * (case.tag_T[tag] - case.Tref), case.na)
    out = _face_out(case, e, g, c, xf).reshape(case.na, nl)
    if kind == BC_SPECULAR:
        a = int(np.argmax(np.abs(n)))      # the wall's normal axis: flip that component
        return out[case.mirror[a]].reshape(-1)
    if kind == BC_DIFFUSE:
        sn = case.sn(n)
        num = ((case.w * np.where(sn > 0, sn, 0.0))[:, None] * out).sum(axis=0)
        den = (case.w * np.where(sn < 0, -sn, 0.0)).sum()
        return np.tile(num / den, case.na)
    raise ValueError("unsupported boundary condition %d" % kind)


def flux_div(case, e):
    """(1/V_i) sum_j v (s . n_ij) S_ij e_ij for every cell and lane [nc*nk]."""
    e = np.asarray(e, dtype=np.float64).reshape(case.nc, case.nk)
    g = grad(case, e)
    v = case.lanes_v()
    D = np.zeros((case.nc, case.nk))
    for c in range(case.nc):
        acc = np.zeros(case.nk)
        for nb, tag, S, n, xf in case.faces[c]:
            sn = np.repeat(case.sn(n), case.nl)
            eo = _face_out(case, e, g, c, xf)
            ei = _face_out(case, e, g, nb, xf) if nb >= 0 else _wall_in(case, e, g, c, tag, n, xf)
            ef = np.where(sn > 0, eo, ei)
            acc += v * sn * S * ef
        D[c] = acc / case.V[c]
    return D.reshape(-1)


def moments(case, e):
    """T (K), T_L (K), q [nc, 3] (W/m^2)."""
    e = np.asarray(e, dtype=np.float64).reshape(case.nc, case.na, case.nl)
    we = case.w[None, :, None] * e
    T = case.Tref + we.sum(axis=(1, 2)) / case.Ctot
    TL = case.Tref + (we / case.tau[None, None, :]).sum(axis=(1, 2)) / case.Ssum
    q = np.einsum("cal,ai,l->ci", we, case.s, case.v)
    return T, TL, q


def residual(case, e, TLdev=None):
    """R = -D - (e - C T_L / 4 pi) / tau + Q; TLdev: T_L - T_ref per cell
    (None: from e)."""
    e = np.asarray(e, dtype=np.float64).reshape(-1)
    if TLdev is None:
        TLdev = moments(case, e)[1] - case.Tref
    D = flux_div(case, e).reshape(case.nc, case.nk)
    e2 = e.reshape(case.nc, case.nk)
    C4 = case.lanes_C4()
    R = -D - (e2 - C4[None, :] * np.asarray(TLdev)[:, None]) / case.lanes_tau()[None, :]
    if case.P is not None:
        R += (case.P[:, None] / case.Ctot) * C4[None, :]
    return R.reshape(-1)


def upwind_order(case, al):
    """Cells of direction al in upwind order and the lagged couplings
    (set of (cell, neighbour)), by the rule of the module docstring."""
    s = case.s[al]
    deps = [set() for _ in range(case.nc)]
    down = [[] for _ in range(case.nc)]
    for c in range(case.nc):
        for nb, _, _, n, _ in case.faces[c]:
            if nb >= 0 and _dot(s, n) < 0:
                deps[c].add(nb)
                down[nb].append(c)
    indeg = [len(x) for x in deps]
    done = [False] * case.nc
    order, lagged = [], set()
    ready = [c for c in range(case.nc) if indeg[c] == 0]
    head = 0
    while len(order) < case.nc:
        if head == len(ready):
            c = min(i for i in range(case.nc) if not done[i])
            for j in deps[c]:
                if not done[j]:
                    lagged.add((c, j))
            indeg[c] = 0
            ready.append(c)
        c = ready[head]
        head += 1
        done[c] = True
        order.append(c)
        for d in down[c]:
            if (d, c) in lagged:
                continue
            indeg[d] -= 1
            if indeg[d] == 0 and not done[d]:
                ready.append(d)
    return order, lagged


def sweep(case, e, TLdev):
    """One source iteration's transport solve: e + de with A de = R(e)."""
    e = np.asarray(e, dtype=np.float64).reshape(-1)
    b = residual(case, e, TLdev).reshape(case.nc, case.na, case.nl)
    de = np.zeros((case.nc, case.na, case.nl))
    if case._order is None:
        case._order = [upwind_order(case, al) for al in range(case.na)]
    for al in range(case.na):
        order, lagged = case._order[al]
        s = case.s[al]
        for c in order:
            A = 1.0 / case.tau
            num = b[c, al].copy()
            for nb, _, S, n, _ in case.faces[c]:
                sn = _dot(s, n)
                if sn > 0:
                    A = A + case.v * sn * S / case.V[c]
                elif sn < 0 and nb >= 0 and (c, nb) not in lagged:
                    num += case.v * (-sn) * S / case.V[c] * de[nb, al]
            de[c, al] = num / A
    return e + de.reshape(-1)


def steady(case, e=None, tol_T=1e-12, max_iter=10000):
    """Source iterations from e (default: equilibrium at T_ref) until the
    largest change of T between iterations is at most tol_T times the
    largest |T - T_ref|."""
    e = case.zeros() if e is None else np.asarray(e, dtype=np.float64).copy()
    T0 = moments(case, e)[0]
    for it in range(1, max_iter + 1):
        TL = moments(case, e)[1] - case.Tref
        e = sweep(case, e, TL)
        T1 = moments(case, e)[0]
        ref = max(np.abs(T1 - case.Tref).max(), 1e-300)
        if np.abs(T1 - T0).max() <= tol_T * ref:
            return e, dict(iters=it, converged=True)
        T0 = T1
    return e, dict(iters=max_iter, converged=False)


def transient(case, e, n_steps, dt):
    """Explicit steps (Sec. 4.1, Algorithm 2): e^{n+1} = e^n + dt R(e^n) with
    T_L from the moments of e^n."""
    e = np.asarray(e, dtype=np.float64).copy()
    for _ in range(n_steps):
        TL = moments(case, e)[1] - case.Tref
        e = e + dt * residual(case, e, TL)
    return e


class TetMeshCase(MeshCase):
    """Tetrahedral mesh (dict of xyz, cell_vtx [nc][4], face_tag [nc][4]
    with face k opposite vertex k, tag_bc, tag_T, optional
    gradient_stencil; see bte_inputs.mesh3d) + bands + optional P.  Cell
    volume |det| / 6, centre = vertex mean (the centroid of a
    tetrahedron); face area |cross| / 2, centre = vertex mean, normal away
    from the opposite vertex; specular walls on faces normal to x, y or z.
    The functions of this module (grad, flux_div, residual, moments, sweep,
    steady, transient) take it like a two-dimensional case."""

    def __init__(self, mesh, material, P=None):
        xyz = np.asarray(mesh["xyz"], dtype=np.float64)
        cells = np.asarray(mesh["cell_vtx"], dtype=np.int64).reshape(-1, 4)
        ftag = np.asarray(mesh["face_tag"], dtype=np.int64).reshape(-1, 4)
        self.tag_bc = np.asarray(mesh["tag_bc"], dtype=np.int64)
        self.tag_T = np.asarray(mesh["tag_T"], dtype=np.float64)
        nc = len(cells)
        self.nc, self.dim = nc, 3
        P4 = xyz[cells]                                        # [nc, 4, 3]
        self.xc = P4.mean(axis=1)
        self.V = np.abs(np.linalg.det(P4[:, 1:] - P4[:, :1])) / 6.0
        owner = {}
        for c in range(nc):
            for k in range(4):
                owner.setdefault(tuple(sorted(np.delete(cells[c], k))), []).append(c)
        self.faces = []
        for c in range(nc):
            fl = []
            for k in range(4):
                f = np.delete(cells[c], k)
                a, b, d = xyz[f]
                cr = np.cross(b - a, d - a)
                S = 0.5 * float(np.linalg.norm(cr))
                n = cr / np.linalg.norm(cr)
                xf = (a + b + d) / 3.0
                if n @ (xf - xyz[cells[c][k]]) < 0:
                    n = -n
                others = [o for o in owner[tuple(sorted(f))] if o != c]
                nb = others[0] if others else -1
                tag = int(ftag[c][k])
                if nb < 0 and tag < 0:
                    raise ValueError("boundary face without a tag")
                fl.append((nb, tag, S, n, xf))
            self.faces.append(fl)
        self.stencil = int(mesh.get("gradient_stencil", 0))
        if self.stencil == 0:
            vcells = {}
            for c in range(nc):
                for v in cells[c]:
                    vcells.setdefault(int(v), set()).add(c)
            self.lsn = []
            for c in range(nc):
                near = set()
                for v in cells[c]:
                    near |= vcells[int(v)]
                near.discard(c)
                self.lsn.append(sorted(near))
        else:
            self.lsn = [[nb for nb, _, _, _, _ in self.faces[c] if nb >= 0] for c in range(nc)]
        self.Xinv = np.zeros((nc, 3, 3))
        for c in range(nc):
            X = np.zeros((3, 3))
            for nb in self.lsn[c]:
                d = self.xc[nb] - self.xc[c]
                X += np.outer(d, d)
            self.Xinv[c] = np.linalg.pinv(X, rcond=1e-10, hermitian=True)
        m = material
        self.s, self.w = quadrature(3, int(m["n_theta"]), int(m.get("n_phi", 1)), 3)
        self.C = np.asarray(m["C"], dtype=np.float64)
        self.v = np.asarray(m["v"], dtype=np.float64)
        self.tau = np.asarray(m["tau"], dtype=np.float64)
        self.Tref = float(m["Tref"])
        self.na, self.nl = len(self.w), len(self.C)
        self.nk = self.na * self.nl
        self.C4 = self.C / FOURPI
        self.Ctot = self.C.sum()
        self.Ssum = (self.C / self.tau).sum()
        self.P = None if P is None else np.asarray(P, dtype=np.float64)
        self.mirror = np.zeros((3, self.na), dtype=np.int64)
        for a in range(3):
            for al in range(self.na):
                t = self.s[al].copy()
                t[a] = -t[a]
                self.mirror[a, al] = int(np.argmin(np.abs(self.s - t).sum(axis=1)))
        for c in range(nc):
            for nb, tag, _, n, _ in self.faces[c]:
                if nb < 0 and self.tag_bc[tag] == BC_SPECULAR and np.sort(np.abs(n))[1] > 1e-12:
                    raise ValueError("specular walls must be normal to x, y or z")
        self._order = None
