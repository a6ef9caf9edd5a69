"""ctypes binding of the gfx950 phonon-BTE library (include/bte.h).

Argument marshalling only: every step of the hot path runs in the HIP
library ``_lib/libbte.so``.  Device buffers are torch tensors on a ROCm
device; the stream is torch's current stream.  If the library is missing
the import of this module fails loudly -- there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libbte.so")

BTE_OK, BTE_ERR_ARG, BTE_ERR_UNSUPPORTED, BTE_ERR_HIP = 0, 1, 2, 3
BTE_ERR_NOT_CONVERGED, BTE_ERR_NONFINITE, BTE_ERR_CFL, BTE_ERR_STATE = 4, 5, 6, 7
F32, F64 = 0, 1
BC_THERMAL, BC_SPECULAR, BC_DIFFUSE, BC_PERIODIC, BC_INTERFACE = 0, 1, 2, 3, 4
SEQUENTIAL, SYNTHETIC = 0, 1
LIM_NONE, LIM_MC, LIM_MINMOD = 0, 1, 2
OBJ_KEFF_X = 0
TUNE_SWEEP, TUNE_TRANSIENT, TUNE_SWEEP_ONE_LAUNCH = 0, 1, 2

STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_UNSUPPORTED", 3: "ERR_HIP", 4: "ERR_NOT_CONVERGED",
                5: "ERR_NONFINITE", 6: "ERR_CFL", 7: "ERR_STATE"}

EXPORTS = ["bte_setup", "bte_setup_multi", "bte_set_control", "bte_workspace_bytes", "bte_num_unknowns", "bte_num_cells", "bte_num_directions",
           "bte_bind", "bte_set_fields", "bte_moments", "bte_moments_static", "bte_residual", "bte_transient_step",
           "bte_steady_solve", "bte_keff", "bte_adjoint", "bte_transient_adjoint", "bte_transient_adjoint_bytes",
           "bte_transient_adjoint_interval",
           "bte_set_timing", "bte_set_graphs", "bte_set_persistent", "bte_tile_candidates", "bte_set_tiles",
           "bte_autotune", "bte_last_stats",
           "bte_get_directions", "bte_band_discretize", "bte_band_discretize_dev",
           "bte_band_discretize_scratch_bytes", "bte_last_error", "bte_destroy",
           "bte_mesh_setup", "bte_mesh_setup_tet", "bte_mesh_workspace_bytes", "bte_mesh_bind", "bte_mesh_num_cells",
           "bte_mesh_num_directions", "bte_mesh_num_levels", "bte_mesh_num_lagged", "bte_mesh_set_source",
           "bte_mesh_moments", "bte_mesh_residual", "bte_mesh_steady_solve", "bte_mesh_transient_step",
           "bte_mesh_last_error", "bte_mesh_destroy"]


class BteError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("len", C.c_double * 3),
                ("solid", C.POINTER(C.c_uint8)), ("bc", C.c_int * 6), ("bc_T", C.c_double * 6),
                ("periodic_dT", C.c_double * 3), ("pore_bc", C.c_int)]


class Material(C.Structure):
    _fields_ = [("n_bands", C.c_int), ("C", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("tau", C.POINTER(C.c_double)), ("n_theta", C.c_int), ("n_phi", C.c_int),
                ("T_ref", C.c_double), ("material_dim", C.c_int)]


class Interface(C.Structure):
    _fields_ = [("geo_a", C.c_int), ("face_a", C.c_int), ("geo_b", C.c_int), ("face_b", C.c_int),
                ("beta_ab", C.POINTER(C.c_double)), ("beta_ba", C.POINTER(C.c_double))]


class Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int), ("xy", C.POINTER(C.c_double)), ("n_cells", C.c_int),
                ("cell_ptr", C.POINTER(C.c_int)), ("cell_vtx", C.POINTER(C.c_int)), ("edge_tag", C.POINTER(C.c_int)),
                ("n_tags", C.c_int), ("tag_bc", C.POINTER(C.c_int)), ("tag_T", C.POINTER(C.c_double)),
                ("gradient_stencil", C.c_int)]


class TetMesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int), ("xyz", C.POINTER(C.c_double)), ("n_cells", C.c_int),
                ("cell_vtx", C.POINTER(C.c_int)), ("face_tag", C.POINTER(C.c_int)), ("n_tags", C.c_int),
                ("tag_bc", C.POINTER(C.c_int)), ("tag_T", C.POINTER(C.c_double)), ("gradient_stencil", C.c_int)]


class Control(C.Structure):
    _fields_ = [("precision", C.c_int), ("scheme", C.c_int), ("limiter", C.c_int),
                ("residual_temp", C.c_double), ("residual_flux", C.c_double), ("max_iter", C.c_int),
                ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int), ("dt", C.c_double), ("adjoint", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cg_iters", C.c_int), ("eps_T", C.c_double), ("eps_q", C.c_double),
                ("converged", C.c_int), ("ms_total", C.c_double), ("ms_sweep", C.c_double),
                ("ms_walls", C.c_double), ("ms_post", C.c_double), ("ms_cg", C.c_double),
                ("sweep_launches", C.c_int), ("updates", C.c_double)]

    def as_dict(self):
        return {k: (bool(getattr(self, k)) if k == "converged" else getattr(self, k)) for k, _ in self._fields_}


class TuneEntry(C.Structure):
    _fields_ = [("kind", C.c_int), ("tile", C.c_int * 3), ("ms", C.c_double), ("chosen", C.c_int)]


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbte.so not built (run python -m paper_2306_14181_amd.build): %s" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
    sig = {
        "bte_setup": ([C.POINTER(Geometry), C.c_int, C.POINTER(Material), C.POINTER(Control),
                       C.POINTER(vp)], st),
        "bte_setup_multi": ([C.POINTER(Geometry), C.c_int, C.POINTER(Material), C.c_int, C.POINTER(C.c_int),
                             C.POINTER(Interface), C.c_int, C.POINTER(Control), C.POINTER(vp)], st),
        "bte_set_control": ([vp, C.POINTER(Control)], st),
        "bte_workspace_bytes": ([vp], C.c_size_t),
        "bte_num_unknowns": ([vp], C.c_size_t),
        "bte_num_cells": ([vp], C.c_int),
        "bte_num_directions": ([vp], C.c_int),
        "bte_bind": ([vp, vp, C.c_size_t], st),
        "bte_set_fields": ([vp, vp, vp, vp], st),
        "bte_moments": ([vp, vp, vp, vp, vp, vp], st),
        "bte_moments_static": ([vp, vp, vp, vp, vp, vp], st),
        "bte_residual": ([vp, vp, vp, vp], st),
        "bte_transient_step": ([vp, vp, C.c_int, C.c_double, dp, vp], st),
        "bte_steady_solve": ([vp, vp, C.c_int, C.POINTER(SolveStats), vp], st),
        "bte_keff": ([vp, vp, vp, vp], st),
        "bte_adjoint": ([vp, vp, C.c_int, vp, C.POINTER(SolveStats), vp], st),
        "bte_transient_adjoint": ([vp, vp, C.c_int, C.c_double, dp, vp, C.c_int, vp, C.c_size_t, dp, vp,
                                   C.POINTER(SolveStats), vp], st),
        "bte_transient_adjoint_bytes": ([vp, C.c_int, C.c_int], C.c_size_t),
        "bte_transient_adjoint_interval": ([vp, C.c_int, C.c_size_t], C.c_int),
        "bte_set_timing": ([vp, C.c_int], st),
        "bte_set_graphs": ([vp, C.c_int], st),
        "bte_set_persistent": ([vp, C.c_int], st),
        "bte_tile_candidates": ([vp, C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)], st),
        "bte_set_tiles": ([vp, C.c_int, C.POINTER(C.c_int)], st),
        "bte_autotune": ([vp, vp, C.c_int, C.POINTER(TuneEntry), C.c_int, C.POINTER(C.c_int), vp], st),
        "bte_last_stats": ([vp, C.POINTER(SolveStats)], st),
        "bte_get_directions": ([vp, dp, dp], st),
        "bte_band_discretize": ([dp, dp, dp, C.c_longlong, C.c_int, dp, dp, dp, C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)], st),
        "bte_band_discretize_dev": ([vp, vp, vp, C.c_longlong, C.c_int, vp, vp, vp, C.POINTER(C.c_int), vp, vp,
                                     C.c_size_t, vp], st),
        "bte_band_discretize_scratch_bytes": ([C.c_int], C.c_size_t),
        "bte_last_error": ([vp], C.c_char_p),
        "bte_destroy": ([vp], None),
        "bte_mesh_setup": ([C.POINTER(Mesh), C.POINTER(Material), C.POINTER(Control), C.POINTER(vp)], st),
        "bte_mesh_setup_tet": ([C.POINTER(TetMesh), C.POINTER(Material), C.POINTER(Control), C.POINTER(vp)], st),
        "bte_mesh_workspace_bytes": ([vp], C.c_size_t),
        "bte_mesh_bind": ([vp, vp, C.c_size_t], st),
        "bte_mesh_num_cells": ([vp], C.c_int),
        "bte_mesh_num_directions": ([vp], C.c_int),
        "bte_mesh_num_levels": ([vp], C.c_int),
        "bte_mesh_num_lagged": ([vp], C.c_int),
        "bte_mesh_set_source": ([vp, vp, vp], st),
        "bte_mesh_moments": ([vp, vp, vp, vp, vp, vp], st),
        "bte_mesh_residual": ([vp, vp, vp, vp, vp], st),
        "bte_mesh_steady_solve": ([vp, vp, C.c_int, C.POINTER(SolveStats), vp], st),
        "bte_mesh_transient_step": ([vp, vp, C.c_int, vp], st),
        "bte_mesh_last_error": ([vp], C.c_char_p),
        "bte_mesh_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def band_discretize(C_mode, v_mode, tau_mode, n_bands):
    """Mean-free-path band discretisation of a mode-level list (eq. banddis,
    computed by bte_band_discretize).  Returns a material dict part
    {"C", "v", "tau"} of the non-empty bands and each mode's band index."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (C_mode, v_mode, tau_mode)]
    n = len(arrs[0])
    if any(len(a) != n for a in arrs):
        raise ValueError("C, v, tau must have the same length")
    outs = [np.zeros(max(int(n_bands), 1)) for _ in range(3)]
    band = np.zeros(max(n, 1), dtype=np.int32)
    nout = C.c_int(0)
    dptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    st = load().bte_band_discretize(dptr(arrs[0]), dptr(arrs[1]), dptr(arrs[2]), n, int(n_bands),
                                    dptr(outs[0]), dptr(outs[1]), dptr(outs[2]), C.byref(nout),
                                    band.ctypes.data_as(C.POINTER(C.c_int)))
    if st != 0:
        raise BteError(st, "bte_band_discretize: invalid mode list or band count")
    k = nout.value
    return dict(C=outs[0][:k].copy(), v=outs[1][:k].copy(), tau=outs[2][:k].copy()), band[:n].copy()


def band_discretize_dev(C_mode, v_mode, tau_mode, n_bands):
    """band_discretize with the mode list on the device (float64 cuda tensors;
    bte_band_discretize_dev).  Returns ({"C", "v", "tau"} float64 cuda tensors of
    the non-empty bands, band index of every mode as an int32 cuda tensor)."""
    lib = load()
    mode = [t.detach().to(torch.float64).contiguous() for t in (C_mode, v_mode, tau_mode)]
    n = mode[0].numel()
    if any(t.numel() != n or t.device.type != "cuda" for t in mode):
        raise ValueError("C, v, tau must be cuda tensors of the same length")
    dev = mode[0].device
    nb_cap = max(int(n_bands), 1)
    outs = [torch.zeros(nb_cap, dtype=torch.float64, device=dev) for _ in range(3)]
    band = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nbytes = lib.bte_band_discretize_scratch_bytes(int(n_bands))
    scratch = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=dev)
    base = (scratch.data_ptr() + 255) & ~255
    nout = C.c_int(0)
    st = lib.bte_band_discretize_dev(*[C.c_void_p(t.data_ptr()) for t in mode], n, int(n_bands),
                                     *[C.c_void_p(t.data_ptr()) for t in outs], C.byref(nout),
                                     C.c_void_p(band.data_ptr()), C.c_void_p(base), C.c_size_t(nbytes),
                                     C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        raise BteError(st, "bte_band_discretize_dev: invalid mode list, band count or scratch")
    k = nout.value
    return dict(C=outs[0][:k], v=outs[1][:k], tau=outs[2][:k]), band[:n]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _geometry_struct(g):
    s = Geometry()
    s.dim = int(g["dim"])
    n = list(g["n"]) + [1] * (3 - len(g["n"]))
    ln = list(g["len"]) + [1.0] * (3 - len(g["len"]))
    s.n[:] = [int(x) for x in n[:3]]
    s.len[:] = [float(x) for x in ln[:3]]
    keep = None
    if g.get("solid") is not None:
        import numpy as np
        keep = np.ascontiguousarray(g["solid"], dtype=np.uint8)
        s.solid = keep.ctypes.data_as(C.POINTER(C.c_uint8))
    s.bc[:] = [int(x) for x in g["bc"]]
    s.bc_T[:] = [float(x) for x in g.get("bcT", [300.0] * 6)]
    s.periodic_dT[:] = [float(x) for x in g.get("pdT", [0.0, 0.0, 0.0])]
    s.pore_bc = int(g.get("pore_bc", BC_DIFFUSE))
    return s, keep


def _control_struct(control):
    c = Control()
    c.precision = int(control.get("precision", F32))
    c.scheme = int(control.get("scheme", SYNTHETIC))
    c.limiter = int(control.get("limiter", LIM_NONE))
    c.residual_temp = float(control.get("residual_temp", 1e-5))
    c.residual_flux = float(control.get("residual_flux", 1e-3))
    c.max_iter = int(control.get("max_iter", 10000))
    c.cg_rtol = float(control.get("cg_rtol", 1e-10))
    c.cg_max_iter = int(control.get("cg_max_iter", 2000))
    c.dt = float(control.get("dt", 0.0))
    c.adjoint = int(bool(control.get("adjoint", False)))
    return c


class Problem:
    """One problem (a geometry or a batch of geometries) bound to a device workspace.

    geometries: dict or list of dicts (dim, n, len, solid, bc, bcT, pdT, pore_bc)
    material:   dict(C, v, tau, n_theta, n_phi, Tref), or a list of such dicts
                (several materials: geo_mat[g] is the material of geometry g)
    control:    dict(precision, scheme, limiter, residual_temp, residual_flux,
                     max_iter, cg_rtol, cg_max_iter, dt, adjoint)
    interfaces: list of dict(geo_a, face_a, geo_b, face_b, beta_ab, beta_ba)
                (bte_setup_multi)
    """

    def __init__(self, geometries, material, control, device="cuda", geo_mat=None, interfaces=None):
        import numpy as np
        lib = load()
        if isinstance(geometries, dict):
            geometries = [geometries]
        self.device = torch.device(device)
        structs, self._keep = [], []
        for g in geometries:
            s, keep = _geometry_struct(g)
            structs.append(s)
            self._keep.append(keep)
        garr = (Geometry * len(structs))(*structs)
        mats = list(material) if isinstance(material, (list, tuple)) else [material]
        self._bands = []
        marr = (Material * len(mats))()
        for i, mt in enumerate(mats):
            bands = [np.ascontiguousarray(mt[k], dtype=np.float64) for k in ("C", "v", "tau")]
            self._bands.append(bands)
            m = marr[i]
            m.n_bands = len(bands[0])
            m.C, m.v, m.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in bands]
            m.n_theta = int(mt["n_theta"])
            m.n_phi = int(mt.get("n_phi", 1))
            m.T_ref = float(mt["Tref"])
            m.material_dim = int(mt.get("material_dim", 3))
        m = marr[0]
        gm = None
        if geo_mat is not None:
            self._geo_mat = np.ascontiguousarray(geo_mat, dtype=np.int32)
            gm = self._geo_mat.ctypes.data_as(C.POINTER(C.c_int))
        interfaces = interfaces or []
        iarr = (Interface * max(len(interfaces), 1))()
        self._ibeta = []
        for i, q in enumerate(interfaces):
            ab = np.ascontiguousarray(q["beta_ab"], dtype=np.float64)
            ba = np.ascontiguousarray(q["beta_ba"], dtype=np.float64)
            self._ibeta += [ab, ba]
            iarr[i].geo_a, iarr[i].face_a = int(q["geo_a"]), int(q["face_a"])
            iarr[i].geo_b, iarr[i].face_b = int(q["geo_b"]), int(q["face_b"])
            iarr[i].beta_ab = ab.ctypes.data_as(C.POINTER(C.c_double))
            iarr[i].beta_ba = ba.ctypes.data_as(C.POINTER(C.c_double))
        c = _control_struct(control)
        self.control = dict(control)
        self.precision = c.precision
        self.dtype = torch.float64 if c.precision == F64 else torch.float32
        h = C.c_void_p()
        st = lib.bte_setup_multi(garr, len(structs), marr, len(mats), gm, iarr, len(interfaces), C.byref(c),
                                 C.byref(h))
        self._h = h
        if st != BTE_OK:
            msg = lib.bte_last_error(h).decode() if h else "setup failed"
            if h:
                lib.bte_destroy(h)
                self._h = None
            raise BteError(st, msg)
        self._finish_init(lib, h, m, structs)

    def _finish_init(self, lib, h, m, structs):
        self.n_cells = lib.bte_num_cells(h)
        self.n_dirs = lib.bte_num_directions(h)
        self.n_bands = m.n_bands
        self.n_unknowns = lib.bte_num_unknowns(h)
        self.n_geo = len(structs)
        ncell = [int(st.n[0]) * int(st.n[1]) * int(st.n[2]) for st in structs]
        self.cell_geometry = torch.repeat_interleave(torch.arange(self.n_geo, device=self.device),
                                                     torch.tensor(ncell, device=self.device))
        nbytes = lib.bte_workspace_bytes(h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(lib.bte_bind(h, C.c_void_p(aligned), C.c_size_t(nbytes)))

    # ------------------------------------------------------------------ utils
    def _check(self, st, ok=(BTE_OK,)):
        if st not in ok:
            raise BteError(st, load().bte_last_error(self._h).decode())
        return st

    def _e(self, e):
        if not (isinstance(e, torch.Tensor) and e.device.type == "cuda" and e.dtype == self.dtype
                and e.is_contiguous() and e.numel() == self.n_unknowns):
            raise ValueError("e must be a contiguous %s cuda tensor with %d elements"
                             % (self.dtype, self.n_unknowns))
        return _ptr(e)

    def _cells(self, x, width=1):
        if x is None:
            return None
        if not (isinstance(x, torch.Tensor) and x.device.type == "cuda" and x.dtype == torch.float64
                and x.is_contiguous() and x.numel() == self.n_cells * width):
            raise ValueError("expected a contiguous float64 cuda tensor with %d elements" % (self.n_cells * width))
        return _ptr(x)

    def set_control(self, **kw):
        """Update control fields (precision excluded)."""
        self.control.update(kw)
        self._check(load().bte_set_control(self._h, C.byref(_control_struct(self.control))))

    def zeros(self):
        return torch.zeros(self.n_unknowns, dtype=self.dtype, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                torch.cuda.synchronize(self.device)
                _lib.bte_destroy(h)
            except Exception:
                pass
            self._h = None

    # -------------------------------------------------------------------- API
    def directions(self):
        import numpy as np
        s = np.empty((self.n_dirs, 3))
        w = np.empty(self.n_dirs)
        self._check(load().bte_get_directions(self._h, s.ctypes.data_as(C.POINTER(C.c_double)),
                                              w.ctypes.data_as(C.POINTER(C.c_double))))
        return s, w

    def set_fields(self, P=None, gamma=None):
        self._check(load().bte_set_fields(self._h, self._cells(P), self._cells(gamma), _stream()))

    def moments(self, e):
        T = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        TL = torch.empty_like(T)
        q = torch.empty(self.n_cells * 3, dtype=torch.float64, device=self.device)
        self._check(load().bte_moments(self._h, self._e(e), _ptr(T), _ptr(TL), _ptr(q), _stream()))
        return T, TL, q.view(-1, 3)

    def moments_static(self, e):
        """moments() through bte_moments_static: the library's static device
        scratch instead of the workspace (allocates nothing in the library)."""
        T = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        TL = torch.empty_like(T)
        q = torch.empty(self.n_cells * 3, dtype=torch.float64, device=self.device)
        self._check(load().bte_moments_static(self._h, self._e(e), _ptr(T), _ptr(TL), _ptr(q), _stream()))
        return T, TL, q.view(-1, 3)

    def residual(self, e):
        R = torch.empty_like(e)
        self._check(load().bte_residual(self._h, self._e(e), _ptr(R), _stream()))
        return R

    def transient_step(self, e, n_steps, t0=0.0, pulse=None):
        pl = None
        if pulse is not None:
            pl = (C.c_double * 2)(float(pulse[0]), float(pulse[1]))
        self._check(load().bte_transient_step(self._h, self._e(e), int(n_steps), float(t0), pl, _stream()))
        return e

    def transient_adjoint_bytes(self, n_steps, every):
        """Bytes of the checkpoint buffer for n_steps with checkpoints every
        `every` steps (0 on invalid arguments)."""
        return int(load().bte_transient_adjoint_bytes(self._h, int(n_steps), int(every)))

    def transient_adjoint_interval(self, n_steps, max_bytes):
        """The smallest checkpoint interval whose buffer fits in max_bytes
        (0 if none)."""
        return int(load().bte_transient_adjoint_interval(self._h, int(n_steps), C.c_size_t(int(max_bytes))))

    def transient_adjoint(self, e0, n_steps, weights, t0=0.0, pulse=None, every=50):
        """J = sum a T(e^N) / sum a after n_steps explicit steps from e0, and
        dJ/dgamma per cell (checkpoints every `every` steps)."""
        lib = load()
        nbytes = lib.bte_transient_adjoint_bytes(self._h, int(n_steps), int(every))
        if nbytes == 0:
            raise ValueError("invalid n_steps / every")
        ck = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = (ck.data_ptr() + 255) & ~255
        a = self._cells(weights)
        g = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        J = C.c_double(0.0)
        pl = None if pulse is None else (C.c_double * 2)(float(pulse[0]), float(pulse[1]))
        st = SolveStats()
        self._check(lib.bte_transient_adjoint(self._h, self._e(e0), int(n_steps), float(t0), pl, a, int(every),
                                              C.c_void_p(base), C.c_size_t(nbytes), C.byref(J), _ptr(g),
                                              C.byref(st), _stream()))
        del ck
        return J.value, g, st.as_dict()

    def set_timing(self, on=True):
        """Device timers for transient_step (makes it synchronous)."""
        self._check(load().bte_set_timing(self._h, int(bool(on))))

    def set_graphs(self, on=True):
        """Capture the steady sweep and CG launches in HIP graphs (default on)."""
        self._check(load().bte_set_graphs(self._h, int(bool(on))))

    def set_persistent(self, on=False):
        """Launch form of the two-dimensional register-tile sweep: one launch per tile diagonal
        (on=False) or one launch per sweep (on=True; BteError in 1D and 3D)."""
        self._check(load().bte_set_persistent(self._h, int(bool(on))))

    def tile_candidates(self, kind):
        """Candidate tile shapes (x, y, z) of TUNE_SWEEP, TUNE_SWEEP_ONE_LAUNCH or TUNE_TRANSIENT,
        the default first."""
        n = C.c_int()
        buf = (C.c_int * 96)()
        self._check(load().bte_tile_candidates(self._h, int(kind), buf, 32, C.byref(n)))
        return [tuple(buf[3 * i:3 * i + 3]) for i in range(min(n.value, 32))]

    def set_tiles(self, kind, tile):
        """Use tile shape `tile` (one of tile_candidates(kind)); TUNE_SWEEP_ONE_LAUNCH also turns
        the one-launch sweep on, TUNE_SWEEP turns it off."""
        t = (C.c_int * 3)(*tile)
        self._check(load().bte_set_tiles(self._h, int(kind), t))

    def autotune(self, reps=3, scratch=None):
        """Time every candidate tile shape, keep the fastest; returns one dict per candidate.
        The two sweep kinds are one choice: one entry of either is chosen (shape and launch form).
        `scratch` (a state tensor, overwritten) defaults to a fresh one."""
        e = self.zeros() if scratch is None else scratch
        out = (TuneEntry * 64)()
        n = C.c_int()
        self._check(load().bte_autotune(self._h, self._e(e), int(reps), out, 64, C.byref(n), _stream()))
        return [dict(kind=x.kind, tile=tuple(x.tile), ms=x.ms, chosen=bool(x.chosen)) for x in out[:min(n.value, 64)]]

    def last_stats(self):
        st = SolveStats()
        self._check(load().bte_last_stats(self._h, C.byref(st)))
        return st.as_dict()

    def steady_solve(self, e, init=True, allow_not_converged=False):
        st = SolveStats()
        ok = (BTE_OK, BTE_ERR_NOT_CONVERGED) if allow_not_converged else (BTE_OK,)
        self._check(load().bte_steady_solve(self._h, self._e(e), int(bool(init)), C.byref(st), _stream()), ok)
        return st.as_dict()

    def keff(self, e):
        k = torch.empty(self.n_geo, dtype=torch.float64, device=self.device)
        self._check(load().bte_keff(self._h, self._e(e), _ptr(k), _stream()))
        return k

    def adjoint(self, e, objective=OBJ_KEFF_X, allow_not_converged=False):
        """dJ/dgamma per cell (float64 tensor) and the adjoint solve statistics."""
        g = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        st = SolveStats()
        ok = (BTE_OK, BTE_ERR_NOT_CONVERGED) if allow_not_converged else (BTE_OK,)
        self._check(load().bte_adjoint(self._h, self._e(e), int(objective), _ptr(g), C.byref(st), _stream()), ok)
        return g, st.as_dict()


class KeffSteady(torch.autograd.Function):
    """k_eff of every geometry of a problem as a function of the per-cell extra
    scattering rate gamma (float64 tensor of n_cells on the problem's device).

    forward: bte_set_fields(P, gamma), steady solve from the heat-diffusion
    guess, bte_keff.  backward: bte_set_fields with the forward's own P and
    gamma (another forward or set_fields on the same problem may have run in
    between; the problem keeps these fields afterwards), then one bte_adjoint
    solve; geometries are independent, so the gradient of sum_f w_f k_f is
    w_{f(c)} dk/dgamma_c.  The problem must be built with limiter NONE and
    control adjoint=True.

        k = KeffSteady.apply(gamma, prob, P)
    """

    @staticmethod
    def forward(ctx, gamma, prob, P=None):
        gam = gamma.detach().to(torch.float64).contiguous().clone()
        Pf = None if P is None else P.detach().to(torch.float64).contiguous().clone()
        prob.set_fields(Pf, gam)
        e = prob.zeros()
        prob.steady_solve(e, init=True)
        k = prob.keff(e)
        ctx.prob, ctx.e, ctx.gamma, ctx.P = prob, e, gam, Pf
        return k

    @staticmethod
    def backward(ctx, grad_k):
        prob = ctx.prob
        # the adjoint linearises about e for the fields e was solved with
        prob.set_fields(ctx.P, ctx.gamma)
        g, _ = prob.adjoint(ctx.e)
        w = grad_k.to(torch.float64)[prob.cell_geometry]
        return g * w, None, None



class TaveTransient(torch.autograd.Function):
    """Weighted mean local temperature J = sum a T / sum a after n_steps
    explicit steps from rest (e = 0), as a function of the per-cell extra
    scattering rate gamma.  The forward call runs bte_transient_adjoint, which
    returns J and dJ/dgamma together (checkpoints every `every` steps);
    backward scales the stored gradient.  Limiter NONE, control adjoint=True.

        J = TaveTransient.apply(gamma, prob, P, n_steps, weights, t0, pulse, every)
    """

    @staticmethod
    def forward(ctx, gamma, prob, P, n_steps, weights, t0=0.0, pulse=None, every=50):
        prob.set_fields(P, gamma.detach().to(torch.float64).contiguous())
        J, g, _ = prob.transient_adjoint(prob.zeros(), n_steps, weights, t0, pulse, every)
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_J):
        (g,) = ctx.saved_tensors
        return g * grad_J.to(torch.float64), None, None, None, None, None, None, None


def mesh_struct(mesh):
    """ctypes bte_mesh of a 2D mesh dict (xy, cell_ptr, cell_vtx, edge_tag,
    tag_bc, tag_T, optional gradient_stencil; see bte_inputs.mesh2d), or
    bte_tet_mesh of a tetrahedral one (xyz, cell_vtx [n][4], face_tag
    [n][4], tag_bc, tag_T; bte_inputs.mesh3d), and the arrays it points
    into."""
    import numpy as np
    if "xyz" in mesh:
        xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64).reshape(-1, 3)
        vtx = np.ascontiguousarray(mesh["cell_vtx"], dtype=np.int32).reshape(-1, 4)
        tag = np.ascontiguousarray(mesh["face_tag"], dtype=np.int32).reshape(-1, 4)
        tbc = np.ascontiguousarray(mesh["tag_bc"], dtype=np.int32)
        tT = np.ascontiguousarray(mesh["tag_T"], dtype=np.float64)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))   # noqa: E731
        m = TetMesh()
        m.n_vertices, m.xyz = len(xyz), xyz.ctypes.data_as(C.POINTER(C.c_double))
        m.n_cells, m.cell_vtx, m.face_tag = len(vtx), ip(vtx), ip(tag)
        m.n_tags, m.tag_bc, m.tag_T = len(tbc), ip(tbc), tT.ctypes.data_as(C.POINTER(C.c_double))
        m.gradient_stencil = int(mesh.get("gradient_stencil", 0))
        return m, (xyz, vtx, tag, tbc, tT)
    xy = np.ascontiguousarray(mesh["xy"], dtype=np.float64).reshape(-1, 2)
    ptr = np.ascontiguousarray(mesh["cell_ptr"], dtype=np.int32)
    vtx = np.ascontiguousarray(mesh["cell_vtx"], dtype=np.int32)
    tag = np.ascontiguousarray(mesh["edge_tag"], dtype=np.int32)
    tbc = np.ascontiguousarray(mesh["tag_bc"], dtype=np.int32)
    tT = np.ascontiguousarray(mesh["tag_T"], dtype=np.float64)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))   # noqa: E731
    m = Mesh()
    m.n_vertices, m.xy = len(xy), xy.ctypes.data_as(C.POINTER(C.c_double))
    m.n_cells, m.cell_ptr, m.cell_vtx, m.edge_tag = len(ptr) - 1, ip(ptr), ip(vtx), ip(tag)
    m.n_tags, m.tag_bc, m.tag_T = len(tbc), ip(tbc), tT.ctypes.data_as(C.POINTER(C.c_double))
    m.gradient_stencil = int(mesh.get("gradient_stencil", 0))
    return m, (xy, ptr, vtx, tag, tbc, tT)


class MeshProblem:
    """Steady solves and explicit transient steps on an unstructured mesh
    (2D triangles / quadrilaterals or tetrahedra; bte_mesh_*), bound to a
    device workspace.  control: precision,
    max_iter, residual_temp, dt (scheme SEQUENTIAL and limiter NONE)."""

    def __init__(self, mesh, material, control, device="cuda"):
        import numpy as np
        lib = load()
        self.device = torch.device(device)
        ms, self._keep = mesh_struct(mesh)
        self._bands = [np.ascontiguousarray(material[k], dtype=np.float64) for k in ("C", "v", "tau")]
        mt = Material()
        mt.n_bands = len(self._bands[0])
        mt.C, mt.v, mt.tau = [b.ctypes.data_as(C.POINTER(C.c_double)) for b in self._bands]
        mt.n_theta, mt.n_phi = int(material["n_theta"]), int(material.get("n_phi", 1))
        mt.T_ref, mt.material_dim = float(material["Tref"]), int(material.get("material_dim", 3))
        ctl = dict(scheme=SEQUENTIAL, limiter=LIM_NONE)
        ctl.update(control)
        c = _control_struct(ctl)
        self.dtype = torch.float64 if c.precision == F64 else torch.float32
        h = C.c_void_p()
        setup = lib.bte_mesh_setup_tet if isinstance(ms, TetMesh) else lib.bte_mesh_setup
        st = setup(C.byref(ms), C.byref(mt), C.byref(c), C.byref(h))
        self._h = h
        if st != BTE_OK:
            msg = lib.bte_mesh_last_error(h).decode() if h else "setup failed"
            if h:
                lib.bte_mesh_destroy(h)
                self._h = None
            raise BteError(st, msg)
        self.n_cells = lib.bte_mesh_num_cells(h)
        self.n_dirs = lib.bte_mesh_num_directions(h)
        self.n_bands = mt.n_bands
        self.n_unknowns = self.n_cells * self.n_dirs * self.n_bands
        self.n_levels = lib.bte_mesh_num_levels(h)
        self.n_lagged = lib.bte_mesh_num_lagged(h)
        nbytes = lib.bte_mesh_workspace_bytes(h)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._check(lib.bte_mesh_bind(h, C.c_void_p(aligned), C.c_size_t(nbytes)))

    def _check(self, st, ok=(BTE_OK,)):
        if st not in ok:
            raise BteError(st, load().bte_mesh_last_error(self._h).decode())
        return st

    def _e(self, e):
        if not (isinstance(e, torch.Tensor) and e.device.type == "cuda" and e.dtype == self.dtype
                and e.is_contiguous() and e.numel() == self.n_unknowns):
            raise ValueError("e must be a contiguous %s cuda tensor with %d elements"
                             % (self.dtype, self.n_unknowns))
        return _ptr(e)

    def zeros(self):
        return torch.zeros(self.n_unknowns, dtype=self.dtype, device=self.device)

    def set_source(self, P):
        Pt = None if P is None else torch.as_tensor(P, dtype=torch.float64, device=self.device).contiguous()
        self._check(load().bte_mesh_set_source(self._h, _ptr(Pt), _stream()))
        torch.cuda.current_stream().synchronize()

    def moments(self, e):
        T = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        TL = torch.empty_like(T)
        q = torch.empty(self.n_cells, 3, dtype=torch.float64, device=self.device)
        self._check(load().bte_mesh_moments(self._h, self._e(e), _ptr(T), _ptr(TL), _ptr(q), _stream()))
        return T, TL, q

    def residual(self, e, TLdev=None):
        R = torch.empty_like(e)
        tl = None if TLdev is None else torch.as_tensor(TLdev, dtype=torch.float64, device=self.device).contiguous()
        self._check(load().bte_mesh_residual(self._h, self._e(e), _ptr(tl), _ptr(R), _stream()))
        return R

    def steady_solve(self, e, init=True, allow_not_converged=False):
        st = SolveStats()
        ok = (BTE_OK, BTE_ERR_NOT_CONVERGED) if allow_not_converged else (BTE_OK,)
        self._check(load().bte_mesh_steady_solve(self._h, self._e(e), int(init), C.byref(st), _stream()), ok)
        return st.as_dict()

    def transient_step(self, e, n_steps):
        """n_steps explicit steps (control dt) on e in place."""
        self._check(load().bte_mesh_transient_step(self._h, self._e(e), int(n_steps), _stream()))
        return e

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                load().bte_mesh_destroy(h)
            except Exception:
                pass
            self._h = None
