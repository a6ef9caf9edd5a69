"""Dense brute force for tiny grids (test infrastructure only).

With the limiter off, the steady residual R(e) (Sec. 3.3, eq. disretized_BTE
with e0 from the lattice-temperature closure) is affine in e.  Assembling
M = dR/de column by column from unit vectors and solving M e = -R(0)
directly gives the discrete steady solution without any iteration, which
pins the sweep / synthetic-correction / conjugate-gradient machinery of the
iterative solvers to the fixed point they claim to reach.
"""
import numpy as np

from . import oracle as O


def assemble(case, src_scale=1.0):
    """Return (M, r0) with R(e) = M e + r0 (dense; tiny cases only)."""
    n = case.size
    if n > 6000:
        raise ValueError("dense assembly is for tiny cases (n=%d)" % n)
    z = np.zeros(n)
    r0 = O.residual(case, z, None, src_scale)
    M = np.empty((n, n))
    for k in range(n):
        z[k] = 1.0
        M[:, k] = O.residual(case, z, None, src_scale) - r0
        z[k] = 0.0
    return M, r0


def equilibrium_mode(case):
    """Uniform equilibrium shift e = C/(4 pi) on solid cells (null mode of floating domains)."""
    solid = np.ones(case.nc) if case.solid is None else case.solid.astype(np.float64)
    return (solid[:, None, None] * np.ones(case.na)[None, :, None] * (case.C / case.omega)[None, None, :]).reshape(-1)


def solid_unknowns(case):
    """Boolean mask over e of the unknowns that live on solid cells."""
    solid = np.ones(case.nc, bool) if case.solid is None else case.solid.astype(bool)
    return np.repeat(solid, case.na * case.nl)


def solve_steady(case, floating=False):
    """Direct solution of R(e) = 0 over the solid-cell unknowns; floating
    domains fix the mean local temperature deviation to zero with one extra
    constraint row."""
    M, r0 = assemble(case)
    keep = solid_unknowns(case)
    Ms, rs = M[np.ix_(keep, keep)], r0[keep]
    x = np.zeros(case.size)
    if not floating:
        x[keep] = np.linalg.solve(Ms, -rs)
        return x
    # constraint: sum_c (T_c - Tref) = 0  <=>  sum w e over solid cells = 0
    row = (np.ones(case.nc)[:, None, None] * case.w[None, :, None]
           * np.ones(case.nl)[None, None, :]).reshape(-1)[keep]
    row *= np.abs(Ms).max() / np.abs(row).max()
    A = np.vstack([Ms, row[None, :]])
    b = np.concatenate([-rs, [0.0]])
    x[keep], *_ = np.linalg.lstsq(A, b, rcond=None)
    return x
