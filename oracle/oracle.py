"""ctypes wrapper around the C oracle (test infrastructure only).

Quadrature (Sec. 3.2, eq. directiondis): Gauss-Legendre nodes on the first
octant, theta in (0, pi/2) and phi in (0, pi/2), weight w = w_theta w_phi
sin(theta), mirrored to the eight octants and renormalised so that the
weights sum to 4 pi exactly (without that, equilibrium is not a fixed point
of the discrete scattering operator).  Directions are ordered octant-major
(octant bits: 1 = s_x < 0, 2 = s_y < 0, 4 = s_z < 0), then theta (ascending),
then phi (ascending).  For a one-dimensional slab the polar axis is x and the
azimuth is integrated: n_theta nodes per hemisphere, w = 2 pi w_theta sin(theta),
s = (cos(theta), 0, 0); hemisphere 0 has s_x > 0.

Two-dimensional materials (material_dim = 2; Sec. 2.1 replaces the solid
angle by the in-plane polar angle, Sec. 5 MaterialDimension): directions lie
in the x-y plane, s = (cos(theta), sin(theta), 0), with n_theta
Gauss-Legendre nodes of theta in (0, pi/2) per quadrant, weight w_theta,
mirrored to the four quadrants (bits 1 = s_x < 0, 2 = s_y < 0) and
renormalised to 2 pi; on a one-dimensional slab the two signs of s_y merge:
s = (+-cos(theta), 0, 0) with w = 2 w_theta per hemisphere.  The total angle
Omega (4 pi or 2 pi) replaces 4 pi wherever an isotropic value is formed
(e0 = C T_L / Omega, wall emission, source split, periodic jump).  Only
one- and two-dimensional geometries take two-dimensional materials.
"""
import ctypes as C
import os
import subprocess

import numpy as np

BC_THERMAL, BC_SPECULAR, BC_DIFFUSE, BC_PERIODIC, BC_INTERFACE = 0, 1, 2, 3, 4
LIM_NONE, LIM_MC, LIM_MINMOD = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bte_oracle.c")


def lib_path():
    return os.path.join(_HERE, "_build", "liboracle.so")


def build(force=False):
    """Compile the oracle with gcc (-O3 -fopenmp, no fast-math)."""
    out = lib_path()
    if os.path.exists(out) and not force and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-std=c11", "-fPIC", "-shared",
                           "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)
    return out


_lib = None


def _L():
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(_CCase)
        for name, args, res in [
            ("orc_moments", [cp, dp, dp, dp, dp], C.c_int),
            ("orc_residual", [cp, dp, dp, C.c_double, dp], C.c_int),
            ("orc_flux_div", [cp, dp, dp], C.c_int),
            ("orc_sweep", [cp, dp, dp, dp, C.POINTER(C.c_int), C.c_int], C.c_int),
            ("orc_cg", [cp, C.c_int, dp, dp, C.c_double, C.c_int], C.c_int),
            ("orc_diffusion_T", [cp, dp, C.c_double, C.c_int], C.c_int),
            ("orc_steady", [cp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                            C.c_int, dp, C.POINTER(_CStats)], C.c_int),
            ("orc_keff", [cp, dp], C.c_double),
            ("orc_transient", [cp, dp, C.c_int, C.c_double, C.c_double, dp, dp, dp], C.c_int),
            ("orc_apply_jac_T", [cp, dp, dp], C.c_int),
            ("orc_dR_dgamma", [cp, dp, dp, dp], C.c_int),
            ("orc_sweep_T", [cp, dp, dp], C.c_int),
        ]:
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = res
    return _lib


class _CCase(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("len", C.c_double * 3),
        ("solid", C.POINTER(C.c_uint8)),
        ("bc", C.c_int * 6), ("bcT", C.c_double * 6), ("pdT", C.c_double * 3),
        ("pore_bc", C.c_int), ("pore_T", C.c_double),
        ("na", C.c_int), ("s", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
        ("nl", C.c_int), ("C", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
        ("tau", C.POINTER(C.c_double)), ("Tref", C.c_double),
        ("gamma", C.POINTER(C.c_double)), ("P", C.POINTER(C.c_double)),
        ("limiter", C.c_int), ("omega", C.c_double),
        ("nmat", C.c_int), ("mat", C.POINTER(C.c_int)), ("beta", C.POINTER(C.c_double)),
    ]


class _CStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cg_iters", C.c_int), ("eps_T", C.c_double),
                ("eps_q", C.c_double), ("converged", C.c_int)]


def quadrature(dim, n_theta, n_phi, material_dim=3):
    """Directions s[na,3] and weights w[na] (see module docstring)."""
    xt, wt = np.polynomial.legendre.leggauss(n_theta)
    theta = (xt + 1.0) * np.pi / 4.0
    wt = wt * np.pi / 4.0
    if material_dim == 2:
        if dim not in (1, 2):
            raise ValueError("two-dimensional materials take 1D or 2D geometries")
        s, w = [], []
        if dim == 1:
            for sg in (1.0, -1.0):
                for k in range(n_theta):
                    s.append((sg * np.cos(theta[k]), 0.0, 0.0))
                    w.append(2.0 * wt[k])
        else:
            for o in range(4):
                sx = -1.0 if o & 1 else 1.0
                sy = -1.0 if o & 2 else 1.0
                for k in range(n_theta):
                    s.append((sx * np.cos(theta[k]), sy * np.sin(theta[k]), 0.0))
                    w.append(wt[k])
        s = np.array(s, dtype=np.float64)
        w = np.array(w, dtype=np.float64)
        w *= 2.0 * np.pi / w.sum()
        return s, w
    if dim == 1:
        s, w = [], []
        for sg in (1.0, -1.0):
            for k in range(n_theta):
                s.append((sg * np.cos(theta[k]), 0.0, 0.0))
                w.append(2.0 * np.pi * wt[k] * np.sin(theta[k]))
    else:
        xp, wp = np.polynomial.legendre.leggauss(n_phi)
        phi = (xp + 1.0) * np.pi / 4.0
        wp = wp * np.pi / 4.0
        s, w = [], []
        for o in range(8):
            sx = -1.0 if o & 1 else 1.0
            sy = -1.0 if o & 2 else 1.0
            sz = -1.0 if o & 4 else 1.0
            for i in range(n_theta):
                for j in range(n_phi):
                    st = np.sin(theta[i])
                    s.append((sx * st * np.cos(phi[j]), sy * st * np.sin(phi[j]), sz * np.cos(theta[i])))
                    w.append(wt[i] * wp[j] * st)
    s = np.array(s, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    w *= 4.0 * np.pi / w.sum()
    return s, w


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class Case:
    """A problem instance: geometry + bands + quadrature + fields.

    geometry: dict(dim, n(3), len(3), solid (uint8 [nc]) or None, bc(6),
              bcT(6) absolute K, pdT(3), pore_bc, optional mat (int [nc]):
              the material of each cell)
    material: dict(C, v, tau arrays, n_theta, n_phi, Tref, optional
              material_dim: 3 (default) or 2), or a list of such dicts (one
              per material: same bands, directions and Tref)
    beta:     with several materials, [nmat][nmat][nl] transmittances of the
              interfaces between them (Sec. 2.2 (v)): beta[a][b][l] is the
              fraction of band l's energy flux from material a crossing into b
    """

    def __init__(self, geometry, material, P=None, gamma=None, limiter=LIM_NONE, beta=None):
        g = geometry
        mats = list(material) if isinstance(material, (list, tuple)) else [material]
        m = mats[0]
        for mm in mats[1:]:
            for key in ("n_theta", "n_phi", "Tref", "material_dim"):
                if mm.get(key) != m.get(key):
                    raise ValueError("materials differ in %s" % key)
            if len(mm["C"]) != len(m["C"]):
                raise ValueError("materials differ in their number of bands")
        self.nmat = len(mats)
        self.mat = None if g.get("mat") is None else np.ascontiguousarray(g["mat"], dtype=np.int32)
        self.beta = None if beta is None else np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
        self.dim = int(g["dim"])
        self.n = [int(x) for x in g["n"]]
        self.len = [float(x) for x in g["len"]]
        self.nc = self.n[0] * self.n[1] * self.n[2]
        self.solid = None if g.get("solid") is None else np.ascontiguousarray(g["solid"], dtype=np.uint8)
        self.material_dim = int(m.get("material_dim", 3))
        self.omega = 2.0 * np.pi if self.material_dim == 2 else 4.0 * np.pi
        self.s, self.w = quadrature(self.dim, int(m["n_theta"]), int(m.get("n_phi", 1)), self.material_dim)
        self.C = np.ascontiguousarray(np.concatenate([np.asarray(x["C"], dtype=np.float64) for x in mats]))
        self.v = np.ascontiguousarray(np.concatenate([np.asarray(x["v"], dtype=np.float64) for x in mats]))
        self.tau = np.ascontiguousarray(np.concatenate([np.asarray(x["tau"], dtype=np.float64) for x in mats]))
        self.Tref = float(m["Tref"])
        self.na, self.nl = len(self.w), len(m["C"])
        self.P = None if P is None else np.ascontiguousarray(P, dtype=np.float64)
        self.gamma = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
        self.limiter = int(limiter)
        self.bc = [int(x) for x in g["bc"]]
        self.bcT = [float(x) for x in g.get("bcT", [self.Tref] * 6)]
        self.pdT = [float(x) for x in g.get("pdT", [0.0, 0.0, 0.0])]
        self.pore_bc = int(g.get("pore_bc", BC_DIFFUSE))
        self._c = self._make()

    def _make(self):
        c = _CCase()
        c.dim = self.dim
        c.n[:] = self.n
        c.len[:] = self.len
        c.solid = self.solid.ctypes.data_as(C.POINTER(C.c_uint8)) if self.solid is not None else None
        c.bc[:] = self.bc
        c.bcT[:] = self.bcT
        c.pdT[:] = self.pdT
        c.pore_bc = self.pore_bc
        c.pore_T = self.Tref
        c.na, c.nl = self.na, self.nl
        c.s, c.w = _dp(self.s), _dp(self.w)
        c.C, c.v, c.tau = _dp(self.C), _dp(self.v), _dp(self.tau)
        c.Tref = self.Tref
        c.gamma = _dp(self.gamma)
        c.P = _dp(self.P)
        c.limiter = self.limiter
        c.omega = self.omega
        c.nmat = self.nmat
        c.mat = self.mat.ctypes.data_as(C.POINTER(C.c_int)) if self.mat is not None else None
        c.beta = _dp(self.beta)
        return c

    def with_(self, **kw):
        """Copy with some fields replaced (gamma, P, limiter)."""
        import copy
        o = copy.copy(self)
        for k, v in kw.items():
            if k in ("gamma", "P") and v is not None:
                v = np.ascontiguousarray(v, dtype=np.float64)
            setattr(o, k, v)
        o._c = o._make()
        return o

    @property
    def size(self):
        return self.nc * self.na * self.nl

    def zeros(self):
        return np.zeros(self.size, dtype=np.float64)

    @property
    def ptr(self):
        return C.byref(self._c)


def moments(case, e):
    """Return T (K), T_L (K), q[nc,3] (W/m^2) of e."""
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    T, TL, q = np.empty(case.nc), np.empty(case.nc), np.empty(3 * case.nc)
    _L().orc_moments(case.ptr, _dp(e), _dp(T), _dp(TL), _dp(q))
    return T, TL, q.reshape(-1, 3)


def residual(case, e, TLdev=None, src_scale=1.0):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    R = np.empty_like(e)
    tl = None if TLdev is None else np.ascontiguousarray(TLdev, dtype=np.float64)
    if _L().orc_residual(case.ptr, _dp(e), _dp(tl), float(src_scale), _dp(R)):
        raise RuntimeError("orc_residual failed")
    return R


def flux_div(case, e):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    D = np.empty_like(e)
    _L().orc_flux_div(case.ptr, _dp(e), _dp(D))
    return D


def sweep(case, e, TLdev, lanes=None, out=None):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    out = e.copy() if out is None else out
    tl = np.ascontiguousarray(TLdev, dtype=np.float64)
    if lanes is None:
        lp, nlanes = None, 0
    else:
        la = np.ascontiguousarray(lanes, dtype=np.int32)
        lp, nlanes = la.ctypes.data_as(C.POINTER(C.c_int)), len(la)
    if _L().orc_sweep(case.ptr, _dp(e), _dp(tl), _dp(out), lp, nlanes):
        raise RuntimeError("orc_sweep failed")
    return out


def cg(case, rhs, rtol=1e-14, maxit=100000, corr=False):
    """Solve the heat-diffusion operator (corr=False) or the synthetic
    correction operator (corr=True) with Jacobi-preconditioned CG."""
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty(case.nc)
    it = _L().orc_cg(case.ptr, int(bool(corr)), _dp(rhs), _dp(x), float(rtol), int(maxit))
    return x, it


def diffusion_T(case, rtol=1e-14, maxit=100000):
    """Heat-diffusion temperature deviation (initial guess)."""
    x = np.empty(case.nc)
    _L().orc_diffusion_T(case.ptr, _dp(x), float(rtol), int(maxit))
    return x


def steady(case, scheme=1, tol_T=1e-10, tol_q=1e30, max_iter=10000, cg_rtol=1e-12,
           cg_maxit=100000, e=None):
    """Steady solve.  Returns (e, stats dict).  e=None starts from diffusion."""
    init = 1 if e is None else 0
    e = case.zeros() if e is None else np.array(e, dtype=np.float64).reshape(-1)
    st = _CStats()
    if _L().orc_steady(case.ptr, int(scheme), float(tol_T), float(tol_q), int(max_iter),
                       float(cg_rtol), int(cg_maxit), init, _dp(e), C.byref(st)):
        raise RuntimeError("orc_steady failed")
    return e, dict(iters=st.iters, cg_iters=st.cg_iters, eps_T=st.eps_T, eps_q=st.eps_q,
                   converged=bool(st.converged))


def keff(case, e):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    return float(_L().orc_keff(case.ptr, _dp(e)))


def transient(case, e, n_steps, dt, t0=0.0, pulse=None, hist_weights=None):
    """Advance e in place by n_steps explicit steps; returns (e, hist or None)."""
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    pl = None if pulse is None else np.ascontiguousarray(pulse, dtype=np.float64)
    hw = None if hist_weights is None else np.ascontiguousarray(hist_weights, dtype=np.float64)
    hist = None if hw is None else np.empty(n_steps)
    _L().orc_transient(case.ptr, _dp(e), int(n_steps), float(dt), float(t0), _dp(pl), _dp(hw), _dp(hist))
    return e, hist


def apply_jac_T(case, x):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.empty_like(x)
    if _L().orc_apply_jac_T(case.ptr, _dp(x), _dp(y)):
        raise RuntimeError("orc_apply_jac_T failed (limiter must be NONE)")
    return y


def dR_dgamma(case, e, psi):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
    out = np.empty(case.nc)
    _L().orc_dR_dgamma(case.ptr, _dp(e), _dp(psi), _dp(out))
    return out


def sweep_T(case, rhs):
    rhs = np.ascontiguousarray(rhs, dtype=np.float64).reshape(-1)
    z = np.empty_like(rhs)
    _L().orc_sweep_T(case.ptr, _dp(rhs), _dp(z))
    return z
