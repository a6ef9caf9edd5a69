"""Seeded synthetic inputs for the phonon-BTE workloads.

This module only draws random numbers and lays out geometry, band tables and
source fields.  It contains none of the solver's arithmetic and is the only
code shared by the oracle side and the HIP side of the tests and benchmark.

Band tables stand in for first-principles silicon data (not available here):
v ~ U[1e3, 8e3] m/s, log10(tau) ~ U[lo, hi], C_raw ~ U(0, 1] rescaled so that
sum C = 1.66e6 J/(m^3 K).  Draw order: v, then log10 tau, then C.
Porous geometries: non-overlapping circular (2D) or spherical (3D) pores with
a ligament of at least two cells (periodic wrap), added until the porosity
reaches the target within 0.01; solid islands not connected to the main
body are filled; the solid must percolate along x.
"""
import numpy as np

BC_THERMAL, BC_SPECULAR, BC_DIFFUSE, BC_PERIODIC, BC_INTERFACE = 0, 1, 2, 3, 4
LIM_NONE, LIM_MC, LIM_MINMOD = 0, 1, 2
SCHEME_SEQUENTIAL, SCHEME_SYNTHETIC = 0, 1

C_TOTAL = 1.66e6


def bands(rng, n_bands, tau_lo=1e-12, tau_hi=1e-10, v_lo=1e3, v_hi=8e3, c_total=C_TOTAL):
    """Seeded band table (C, v, tau) as float64 arrays."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    v = rng.uniform(v_lo, v_hi, n_bands)
    tau = 10.0 ** rng.uniform(np.log10(tau_lo), np.log10(tau_hi), n_bands)
    c = 1.0 - rng.random(n_bands)
    c *= c_total / c.sum()
    return dict(C=c.astype(np.float64), v=v.astype(np.float64), tau=tau.astype(np.float64))


def _geometry(dim, n, length, bc, bcT=None, pdT=(0.0, 0.0, 0.0), solid=None, pore_bc=BC_DIFFUSE,
              Tref=300.0):
    n = list(n) + [1] * (3 - len(n))
    length = list(length) + [1.0] * (3 - len(length))
    return dict(dim=dim, n=n, len=length, bc=list(bc), bcT=list(bcT or [Tref] * 6),
                pdT=list(pdT), solid=solid, pore_bc=pore_bc)


def _cell_centres(n, length):
    """Cell-centre coordinates, arrays of shape n[::-1] (z, y, x order flattened as c)."""
    axes = [(np.arange(n[a]) + 0.5) * (length[a] / n[a]) for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def _keep_percolating(solid, n, dim):
    """Fill solid islands not connected (periodically) to the main body; return
    None if the main body does not span x."""
    from scipy import ndimage
    shape = tuple(n[a] for a in range(dim))[::-1]
    s = solid.reshape(shape).astype(bool)
    # periodic labelling by tiling 3x along each axis
    reps = (3,) * dim
    big = np.tile(s, reps)
    lab, nl = ndimage.label(big)
    sl = tuple(slice(shape[k], 2 * shape[k]) for k in range(dim))
    centre = lab[sl]
    if nl == 0:
        return None
    counts = np.bincount(centre.reshape(-1))
    counts[0] = 0
    main = counts.argmax()
    keep = centre == main
    # percolation along x (last array axis): main label in the first and last column
    if not (keep[..., 0].any() and keep[..., -1].any()):
        return None
    return keep.reshape(-1).astype(np.uint8)


def porous(rng, dim, n, dx, porosity, r_lo=0.05, r_hi=0.15, ligament=2, max_tries=20000):
    """Random circular/spherical pores on a periodic grid of n cells (uniform dx)."""
    n = list(n) + [1] * (3 - len(n))
    side = min(n[a] for a in range(dim)) * dx
    length = [n[a] * dx for a in range(3)]
    x, y, z = _cell_centres(n, length)
    coords = [x, y, z][:dim]
    solid = np.ones(int(np.prod(n)), dtype=np.uint8)
    pores = []
    tries = 0
    while tries < max_tries:
        tries += 1
        phi = 1.0 - solid.mean()
        if phi >= porosity - 0.01:
            break
        r = rng.uniform(r_lo, r_hi) * side
        ctr = [rng.uniform(0, length[a]) for a in range(dim)]
        ok = True
        for (c2, r2) in pores:
            d2 = 0.0
            for a in range(dim):
                d = abs(ctr[a] - c2[a])
                d = min(d, length[a] - d)
                d2 += d * d
            if np.sqrt(d2) < r + r2 + ligament * dx:
                ok = False
                break
        if not ok:
            continue
        d2 = np.zeros_like(x)
        for a in range(dim):
            d = np.abs(coords[a] - ctr[a])
            d = np.minimum(d, length[a] - d)
            d2 += d * d
        trial = solid.copy()
        trial[d2 < r * r] = 0
        if 1.0 - trial.mean() > porosity + 0.01:
            continue
        solid = trial
        pores.append((ctr, r))
    kept = _keep_percolating(solid, n, dim)
    return kept


# ------------------------------------------------------------------ workloads

def slab1d_case(seed=0, n_cells=200, n_bands=10):
    """1D cross-plane slab, L = 100 nm, walls at 301 K / 299 K, Tref 300 K,
    16 polar directions (8 per hemisphere), FP64 steady synthetic."""
    rng = np.random.default_rng(seed)
    mat = bands(rng, n_bands, 1e-12, 1e-10)
    mat.update(n_theta=8, n_phi=1, Tref=300.0)
    bc = [BC_THERMAL, BC_THERMAL] + [BC_SPECULAR] * 4
    bcT = [301.0, 299.0] + [300.0] * 4
    geo = _geometry(1, (n_cells,), (100e-9,), bc, bcT)
    return dict(name="slab1d", geometry=geo, material=mat, P=None, gamma=None,
                limiter=LIM_NONE, scheme=SCHEME_SYNTHETIC, tol_T=1e-10)


def square2d_source_case(seed=1, n=256, n_bands=20, n_theta=2, n_phi=8):
    """2D 1 um square, 256^2 cells; heat sink y=0 edge at 300 K, other edges
    diffuse; Gaussian source (sigma 50 nm, peak 1e17 W/m^3) at the centre."""
    rng = np.random.default_rng(seed)
    mat = bands(rng, n_bands, 1e-12, 1e-9)
    mat.update(n_theta=n_theta, n_phi=n_phi, Tref=300.0)
    bc = [BC_DIFFUSE, BC_DIFFUSE, BC_THERMAL, BC_DIFFUSE, BC_SPECULAR, BC_SPECULAR]
    L = 1e-6
    geo = _geometry(2, (n, n), (L, L), bc)
    x, y, _ = _cell_centres(geo["n"], geo["len"])
    sig = 50e-9
    P = 1e17 * np.exp(-((x - L / 2) ** 2 + (y - L / 2) ** 2) / (2 * sig * sig))
    return dict(name="square2d_source", geometry=geo, material=mat, P=P, gamma=None,
                limiter=LIM_NONE, scheme=SCHEME_SYNTHETIC)


def interface2d_case(seed=5, n=256, n_bands=20, n_theta=2, n_phi=8):
    """Two materials side by side in a 1 um square (the shape of the paper's
    interface verification case): material A on the left half between a
    thermalizing wall at 301 K and the interface, material B on the right
    half between the interface and a wall at 299 K, specular top and bottom;
    n/2 x n cells per half.  Both band tables are seeded draws (B with twice
    the heat capacity, 0.4-0.9x the speeds, its own relaxation times); the
    transmittances follow the diffuse-mismatch form per band,
    beta_AB = C_B v_B / (C_A v_A + C_B v_B), beta_BA = 1 - beta_AB (which keeps
    a uniform temperature in equilibrium)."""
    rng = np.random.default_rng(seed)
    ma = bands(rng, n_bands, 1e-12, 1e-9)
    mb = bands(rng, n_bands, 1e-12, 1e-9)
    mb["C"] = ma["C"] * 2.0
    mb["v"] = ma["v"] * rng.uniform(0.4, 0.9, n_bands)
    for m in (ma, mb):
        m.update(n_theta=n_theta, n_phi=n_phi, Tref=300.0)
    ga, gb = ma["C"] * ma["v"], mb["C"] * mb["v"]
    beta_ab = gb / (ga + gb)
    L, h = 1e-6, n // 2
    spec = [BC_SPECULAR] * 4
    gA = _geometry(2, (h, n), (L / 2, L), [BC_THERMAL, BC_INTERFACE] + spec, [301.0, 300.0] + [300.0] * 4)
    gB = _geometry(2, (h, n), (L / 2, L), [BC_INTERFACE, BC_THERMAL] + spec, [300.0, 299.0] + [300.0] * 4)
    ifc = dict(geo_a=0, face_a=1, geo_b=1, face_b=0, beta_ab=beta_ab, beta_ba=1.0 - beta_ab)
    return dict(name="interface2d", geometries=[gA, gB], materials=[ma, mb], geo_mat=[0, 1], interfaces=[ifc],
                limiter=LIM_NONE, scheme=SCHEME_SYNTHETIC)


def laser_profile(geo, q0=4.64e18, w0=200e-9, depth=1.5e-6):
    """Spatial part of the top-face laser source: Q0 exp(-2 r^2/w0^2) exp(-d/h)."""
    x, y, z = _cell_centres(geo["n"], geo["len"])
    Lx, Ly, Lz = geo["len"]
    r2 = (x - Lx / 2) ** 2 + (y - Ly / 2) ** 2
    d = Lz - z
    return q0 * np.exp(-2 * r2 / (w0 * w0)) * np.exp(-d / depth)


def tave_weights(geo, w0=200e-9):
    """Weights of the surface-average temperature: top-layer cells with r < 2 w0,
    weight exp(-2 r^2 / w0^2)."""
    x, y, z = _cell_centres(geo["n"], geo["len"])
    Lx, Ly, Lz = geo["len"]
    hz = Lz / geo["n"][2]
    r2 = (x - Lx / 2) ** 2 + (y - Ly / 2) ** 2
    top = z > Lz - hz
    return np.where(top & (r2 < 4 * w0 * w0), np.exp(-2 * r2 / (w0 * w0)), 0.0)


def cube3d_laser_case(seed=2, n=64, n_bands=40, n_theta=4, n_phi=4, length=2e-6):
    """3D (2 um)^3 cube, n^3 cells, top (+z) face diffuse, other faces at
    300 K; Gaussian laser pulse (200 nm spot, 10 ps FWHM centred at 20 ps);
    dt = 0.5 ps explicit steps; MC limiter.  `length` shrinks the cube (a
    reduced grid with the cell size, and so the Courant numbers, of the
    64^3 case: length = n * 2 um / 64)."""
    rng = np.random.default_rng(seed)
    mat = bands(rng, n_bands, 1e-12, 1e-9)
    mat.update(n_theta=n_theta, n_phi=n_phi, Tref=300.0)
    bc = [BC_THERMAL] * 5 + [BC_DIFFUSE]
    L = float(length)
    geo = _geometry(3, (n, n, n), (L, L, L), bc)
    P = laser_profile(geo)
    return dict(name="cube3d_laser", geometry=geo, material=mat, P=P, gamma=None,
                limiter=LIM_MC, dt=0.5e-12, n_steps=2000, pulse=(20e-12, 10e-12),
                hist_weights=tave_weights(geo))


def porous2d_batch_case(seed=3, n_films=64, sides=(32, 64, 128, 192, 256), n_bands=20, n_theta=2, n_phi=4):
    """Batch of 2D porous films (periodic x with dT = 1 K, periodic y, diffuse
    pores), dx = 1 um / 256; returns a list of film geometries and one band table.

    The films are solved with the minmod limiter: with the unlimited central
    gradient, plain and synthetic source iteration both diverge on some of
    the seeded films, and with the MC limiter the iteration settles into a
    limit cycle (relative change per iteration about 1.5e-5) on the larger
    ballistic films; with minmod every film converges to the FP32 floor."""
    rng = np.random.default_rng(seed)
    mat = bands(rng, n_bands, 1e-12, 1e-9)
    mat.update(n_theta=n_theta, n_phi=n_phi, Tref=300.0)
    dx = 1e-6 / 256
    films = []
    for child in rng.spawn(n_films):
        for _ in range(50):
            side = int(child.choice(sides))
            phi = child.uniform(0.1, 0.4)
            solid = porous(child, 2, (side, side), dx, phi)
            if solid is not None:
                break
        bc = [BC_PERIODIC] * 4 + [BC_SPECULAR] * 2
        films.append(_geometry(2, (side, side), (side * dx, side * dx), bc, pdT=(1.0, 0.0, 0.0),
                               solid=solid))
    return dict(name="porous2d_batch", films=films, material=mat, limiter=LIM_MINMOD,
                scheme=SCHEME_SYNTHETIC)


def porous3d_adjoint_case(seed=4, n=48, n_bands=40, n_theta=3, n_phi=4, porosity=0.2):
    """3D (1 um)^3 porous cube (spherical pores), periodic xyz with dT = 1 K
    along x, per-cell extra scattering rate gamma ~ U[0, 1e11] 1/s."""
    rng = np.random.default_rng(seed)
    mat = bands(rng, n_bands, 1e-12, 1e-9)
    mat.update(n_theta=n_theta, n_phi=n_phi, Tref=300.0)
    dx = 1e-6 / n
    solid = None
    for _ in range(50):
        solid = porous(rng, 3, (n, n, n), dx, porosity)
        if solid is not None:
            break
    gamma = rng.uniform(0.0, 1e11, n ** 3)
    bc = [BC_PERIODIC] * 6
    geo = _geometry(3, (n, n, n), (n * dx,) * 3, bc, pdT=(1.0, 0.0, 0.0), solid=solid)
    return dict(name="porous3d_adjoint", geometry=geo, material=mat, P=None, gamma=gamma,
                limiter=LIM_NONE, scheme=SCHEME_SYNTHETIC)


def ttg(xi, n_cells=1000, n_theta=256, period=1e-6, v=1e3, c=C_TOTAL, amplitude=1.0, cfl=0.05):
    """Transient thermal grating (Sec. 6, transient verification): one period
    of a 1D domain with periodic ends (no temperature drop), a gray material
    (one band) whose Knudsen number v tau / period is xi / (2 pi), and an
    initial temperature Tref + amplitude cos(2 pi x / period) at the cell
    centres.  The paper's size is 1000 cells and 512 directions (256 per
    hemisphere).  dt = cfl * h / v (and at most tau / 10); the default
    Courant number 0.05 keeps the slow growth of mid-wavenumber rounding
    noise under the explicit unlimited scheme below the relaxation rate of
    the ballistic case."""
    tau = xi * period / (2.0 * np.pi * v)
    mat = dict(C=np.array([c]), v=np.array([v]), tau=np.array([tau]), n_theta=n_theta, n_phi=1, Tref=300.0)
    bc = [BC_PERIODIC, BC_PERIODIC] + [BC_SPECULAR] * 4
    geo = _geometry(1, (n_cells,), (period,), bc)
    x, _, _ = _cell_centres(geo["n"], geo["len"])
    h = period / n_cells
    dt = min(cfl * h / v, 0.1 * tau)
    T = 300.0 + amplitude * np.cos(2.0 * np.pi * x / period)
    return dict(name="ttg1d", geometry=geo, material=mat, P=None, gamma=None, limiter=LIM_NONE, dt=dt, T0=T,
                tau=tau, amplitude=amplitude)


def modes(seed, n_modes, frac_zero_v=0.02, c_total=C_TOTAL):
    """Seeded synthetic mode-level list (stand-in for first-principles
    phonon data): group speed v ~ U[0, 8e3] m/s with a fraction of
    zero-speed modes, log10 tau ~ U[-13, -8], C ~ U(0, 1] rescaled to sum
    c_total.  Draw order: v, zero-speed mask, log10 tau, C."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 8e3, n_modes)
    v[rng.random(n_modes) < frac_zero_v] = 0.0
    tau = 10.0 ** rng.uniform(-13.0, -8.0, n_modes)
    c = 1.0 - rng.random(n_modes)
    c *= c_total / c.sum()
    return dict(C=c, v=v, tau=tau)


def random_field(seed, size, scale=1.0):
    """Seeded uniform random array in [-scale, scale) (test perturbations)."""
    rng = np.random.default_rng(seed)
    return scale * (2.0 * rng.random(size) - 1.0)


def mesh2d(seed, nx, ny, lx, ly, jitter=0.25, quad_frac=0.3, bc=(BC_THERMAL, BC_THERMAL, BC_SPECULAR, BC_SPECULAR),
           bcT=(301.0, 299.0, 300.0, 300.0), gradient_stencil=0, pores=(), pore_bc=BC_DIFFUSE):
    """Unstructured 2D mesh of the rectangle [0, lx] x [0, ly] (topology and
    vertices only): an nx x ny grid whose interior vertices are moved by up to
    `jitter` of a cell size, each quadrilateral kept with probability
    quad_frac (a hybrid mesh) or split into two triangles along a random
    diagonal.  Cells are counter-clockwise vertex lists in grid order (row by
    row; a split square gives two consecutive cells).  edge_tag[i] is the
    boundary side of the edge from vertex i of its cell to the next (0: x = 0,
    1: x = lx, 2: y = 0, 3: y = ly), -1 inside; tag_bc / tag_T give each
    side's boundary condition and wall temperature; gradient_stencil is
    passed through (0: least-squares gradients over the cells sharing a
    vertex, 1: over the face neighbours).  pores: circles (cx, cy, r); the
    cells whose vertex mean lies inside one are left out, and the edges
    they shared with kept cells get tag 4 (pore surface, condition pore_bc).
    With jitter = 0 and quad_frac = 1 it is the Cartesian grid, cell
    ix + nx iy."""
    rng = np.random.default_rng(seed)
    hx, hy = lx / nx, ly / ny
    X, Y = np.meshgrid(np.arange(nx + 1) * hx, np.arange(ny + 1) * hy)   # [ny+1, nx+1]
    X, Y = X.copy(), Y.copy()
    if jitter > 0:
        dx = rng.uniform(-jitter, jitter, X.shape) * hx
        dy = rng.uniform(-jitter, jitter, Y.shape) * hy
        X[1:-1, 1:-1] += dx[1:-1, 1:-1]
        Y[1:-1, 1:-1] += dy[1:-1, 1:-1]
    xy = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    vid = lambda i, j: j * (nx + 1) + i   # noqa: E731

    def side_of(a, b):
        ia, ja = a % (nx + 1), a // (nx + 1)
        ib, jb = b % (nx + 1), b // (nx + 1)
        if ia == 0 and ib == 0:
            return 0
        if ia == nx and ib == nx:
            return 1
        if ja == 0 and jb == 0:
            return 2
        if ja == ny and jb == ny:
            return 3
        return -1

    cells = []
    for j in range(ny):
        for i in range(nx):
            v00, v10, v11, v01 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if quad_frac >= 1.0 or rng.uniform() < quad_frac:
                cells.append([v00, v10, v11, v01])
            elif rng.uniform() < 0.5:
                cells += [[v00, v10, v11], [v00, v11, v01]]
            else:
                cells += [[v00, v10, v01], [v10, v11, v01]]
    if pores:
        def inside(c):
            m = xy[c].mean(axis=0)
            return any((m[0] - px) ** 2 + (m[1] - py) ** 2 < r * r for px, py, r in pores)
        cells = [c for c in cells if not inside(c)]
    count = {}
    for c in cells:
        for k in range(len(c)):
            key = (min(c[k], c[(k + 1) % len(c)]), max(c[k], c[(k + 1) % len(c)]))
            count[key] = count.get(key, 0) + 1

    def tag_of(a, b):
        t = side_of(a, b)
        if t < 0 and count[(min(a, b), max(a, b))] == 1:
            return 4                     # an edge left open by a pore
        return t

    ptr = np.zeros(len(cells) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(c) for c in cells])
    vtx = np.array([v for c in cells for v in c], dtype=np.int32)
    tag = np.array([tag_of(c[k], c[(k + 1) % len(c)]) for c in cells for k in range(len(c))], dtype=np.int32)
    return dict(xy=xy, cell_ptr=ptr, cell_vtx=vtx, edge_tag=tag,
                tag_bc=np.asarray(list(bc) + [pore_bc], dtype=np.int32),
                tag_T=np.asarray(list(bcT) + [300.0], dtype=np.float64), gradient_stencil=int(gradient_stencil))


def mesh3d(seed, nx, ny, nz, lx, ly, lz, jitter=0.15,
           bc=(BC_THERMAL, BC_THERMAL, BC_SPECULAR, BC_SPECULAR, BC_SPECULAR, BC_SPECULAR),
           bcT=(301.0, 299.0, 300.0, 300.0, 300.0, 300.0), gradient_stencil=0, pores=(), pore_bc=BC_DIFFUSE):
    """Tetrahedral mesh of the box [0, lx] x [0, ly] x [0, lz] (topology and
    vertices only): an nx x ny x nz grid whose interior vertices are moved by
    up to `jitter` of a cell size, each cube split into the six tetrahedra
    around its diagonal from its lowest to its highest corner (the same
    split in every cube, so faces match).  cell_vtx[c] holds the four
    vertices of tetrahedron c (any order); face_tag[c][k] is the boundary
    side of the face opposite vertex k (0: x = 0, 1: x = lx, 2: y = 0,
    3: y = ly, 4: z = 0, 5: z = lz), -1 inside; pores are spheres
    (cx, cy, cz, r) whose tetrahedra (by vertex mean) are left out, the
    faces they open getting tag 6 (condition pore_bc)."""
    rng = np.random.default_rng(seed)
    h = np.array([lx / nx, ly / ny, lz / nz])
    g = np.stack(np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij"), axis=-1)
    xyz = (g * h).astype(np.float64)                        # [nx+1, ny+1, nz+1, 3]
    if jitter > 0:
        d = rng.uniform(-jitter, jitter, xyz.shape) * h
        xyz[1:-1, 1:-1, 1:-1] += d[1:-1, 1:-1, 1:-1]
    xyz = xyz.reshape(-1, 3)
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k   # noqa: E731
    unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    cells = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                for p in perms:
                    a = [i, j, k]
                    t = [vid(*a)]
                    for ax in p:
                        a = [a[q] + unit[ax][q] for q in range(3)]
                        t.append(vid(*a))
                    cells.append(t)
    if pores:
        def inside(c):
            m = xyz[c].mean(axis=0)
            return any(((m - np.array(pc[:3])) ** 2).sum() < pc[3] ** 2 for pc in pores)
        cells = [c for c in cells if not inside(c)]
    cells = np.array(cells, dtype=np.int32)
    P = xyz[cells]
    if (np.linalg.det(P[:, 1:] - P[:, :1]) == 0).any():
        raise ValueError("degenerate tetrahedron: lower the jitter")
    ijk = np.stack(np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij"),
                   axis=-1).reshape(-1, 3)
    top = np.array([nx, ny, nz])
    # faces: vertices other than vertex q, for every cell and q
    others = np.array([[r for r in range(4) if r != q] for q in range(4)])
    F = cells[:, others]                                     # [nc, 4, 3]
    keys = np.sort(F, axis=2).reshape(-1, 3)
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    once = (cnt[inv.reshape(-1)] == 1).reshape(len(cells), 4)
    tag = np.full((len(cells), 4), -1, dtype=np.int32)
    G = ijk[F]                                               # [nc, 4, 3 vertices, 3 axes]
    for ax in range(3):
        tag[(G[..., ax] == 0).all(axis=2)] = 2 * ax
        tag[(G[..., ax] == top[ax]).all(axis=2)] = 2 * ax + 1
    tag[(tag < 0) & once] = 6
    return dict(xyz=xyz, cell_vtx=cells, face_tag=tag, tag_bc=np.asarray(list(bc) + [pore_bc], dtype=np.int32),
                tag_T=np.asarray(list(bcT) + [300.0], dtype=np.float64), gradient_stencil=int(gradient_stencil))
