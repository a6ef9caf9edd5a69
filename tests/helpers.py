"""Shared test helpers: build the oracle case and the GPU problem from the
same seeded inputs, and the relative-error metric used by the parity tests
(max |x - x_ref| / max |x_ref - offset|; offset T_ref for temperatures, 0
otherwise)."""
import numpy as np

import bte_inputs as I


def geo(dim, n, length, bc, bcT=None, pdT=(0, 0, 0), solid=None, pore_bc=I.BC_DIFFUSE):
    n = list(n) + [1] * (3 - len(n))
    length = list(length) + [1.0] * (3 - len(length))
    return dict(dim=dim, n=n, len=length, bc=list(bc), bcT=list(bcT or [300.0] * 6), pdT=list(pdT),
                solid=solid, pore_bc=pore_bc)


def mat(b, n_theta, n_phi=1, Tref=300.0):
    m = dict(b)
    m.update(n_theta=n_theta, n_phi=n_phi, Tref=Tref)
    return m


def rel_err(x, ref, offset=0.0):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref - offset).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def small_cases():
    """A set of small geometries covering every boundary type, pores,
    periodic jumps, sources, per-cell scattering, 1D/2D/3D and ragged tiles."""
    rng = np.random.default_rng(1234)
    b2 = I.bands(rng, 3, 1e-12, 1e-9)
    out = {}
    out["slab1d"] = (geo(1, (70,), (70e-9,), [I.BC_THERMAL, I.BC_THERMAL] + [I.BC_SPECULAR] * 4,
                         bcT=[301.0, 299.0, 300, 300, 300, 300]),
                     mat(I.bands(rng, 5, 1e-12, 1e-10), 8), rng.uniform(0, 1e16, 70), None)
    solid = np.ones(13 * 11, dtype=np.uint8)
    solid[[20, 21, 33, 34, 60, 100]] = 0
    out["walls2d"] = (geo(2, (13, 11), (130e-9, 110e-9),
                          [I.BC_THERMAL, I.BC_DIFFUSE, I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_SPECULAR, I.BC_SPECULAR],
                          bcT=[300.5, 300, 300, 300, 300, 300], solid=solid),
                      mat(b2, 2, 2), rng.uniform(0, 1e17, 143), rng.uniform(0, 1e11, 143))
    solid = np.ones(10 * 9, dtype=np.uint8)
    solid[[11, 12, 44, 45, 77]] = 0
    out["periodic2d"] = (geo(2, (10, 9), (100e-9, 90e-9), [I.BC_PERIODIC] * 4 + [I.BC_SPECULAR] * 2,
                             pdT=(1.0, 0, 0), solid=solid),
                         mat(b2, 1, 3), None, rng.uniform(0, 1e11, 90))
    solid = np.ones(9 * 6 * 5, dtype=np.uint8)
    solid[[7, 8, 50, 51, 120, 200]] = 0
    out["box3d"] = (geo(3, (9, 6, 5), (0.3e-6, 0.2e-6, 0.15e-6),
                        [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_SPECULAR, I.BC_DIFFUSE, I.BC_THERMAL, I.BC_DIFFUSE],
                        pdT=(0.5, 0, 0), bcT=[300, 300, 300, 300, 299.0, 300], solid=solid),
                    mat(b2, 1, 2), rng.uniform(0, 1e17, 270), rng.uniform(0, 1e11, 270))
    return out


# ------------------------------------------------ transient thermal grating

def ttg_discrete_mode(mu, w, v, tau, n_cells, period, dt, n_steps, c, amplitude, omega=4.0 * np.pi):
    """Temperature deviation T_i - Tref after n_steps of the explicit scheme
    on a gray transient grating, computed in Fourier space (independent of
    the oracle).  On a periodic uniform grid a single mode exp(i theta j),
    theta = 2 pi / n, stays a single mode: with the central least-squares
    slope the face difference of the second-order upwind flux has the symbol
      S = 1 + (e^{i theta} - e^{-i theta}) / 4 - e^{-i theta} - (1 - e^{-2 i theta}) / 4
    for s_x > 0 (its conjugate for s_x < 0), so each direction's complex
    amplitude a obeys forward Euler on
      da/dt = -(v |mu| / h) S a + (sum_b w_b a_b / 4 pi - a) / tau
    (gray: e0 = C T_L / 4 pi and T_L = sum w e / C).  The initial state is
    the equilibrium of amplitude cos(2 pi x / period) at the cell centres,
    i.e. a = (C amplitude / 4 pi) e^{i theta / 2} for every direction.  For a
    two-dimensional material the total angle omega = 2 pi replaces 4 pi."""
    n = n_cells
    h = period / n
    th = 2.0 * np.pi / n
    z = np.exp(1j * th)
    S = 1.0 + (z - 1.0 / z) / 4.0 - 1.0 / z - (1.0 - z ** -2) / 4.0
    Sd = np.where(np.asarray(mu) > 0, S, np.conj(S))
    lam = v * np.abs(mu) * Sd / h
    w = np.asarray(w, dtype=np.float64)
    a = np.full(len(w), c * amplitude / omega * np.exp(0.5j * th), dtype=np.complex128)
    for _ in range(n_steps):
        a = a + dt * (-lam * a + ((w @ a) / omega - a) / tau)
    phase = np.exp(1j * th * np.arange(n))
    return np.real((w @ a) * phase) / c


def ttg_continuous_amplitude(xi_tau_t, v, tau, period, n_mu=2000):
    """A(t)/A0 of the gray transient grating with continuous space, time and
    angle (the reference solution the paper compares against): per
    direction cosine mu the mode amplitude obeys
      da/dt = -i q v mu a + (1/2 int a dmu' - a) / tau,  q = 2 pi / period,
    a(0) = 1, solved exactly (matrix exponential) on n_mu Gauss-Legendre
    nodes in mu; A/A0 = 1/2 sum w a.  xi_tau_t: times in units of tau."""
    from scipy.linalg import expm
    mu, wq = np.polynomial.legendre.leggauss(n_mu)
    q = 2.0 * np.pi / period
    M = -1j * q * v * np.diag(mu) + (0.5 * np.outer(np.ones(n_mu), wq) - np.eye(n_mu)) / tau
    out = []
    for ts in xi_tau_t:
        a = expm(M * (ts * tau)) @ np.ones(n_mu)
        out.append(float(np.real(0.5 * wq @ a)))
    return np.array(out)
