"""FP64 CPU oracle for the phonon-BTE hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library under ``paper_2306_14181_amd/`` and never serves as
a fallback for it.

The arithmetic lives in ``bte_oracle.c`` (plain C, FP64, OpenMP); this module
computes the angular quadrature (Sec. 3.2, eq. directiondis) with numpy's
Gauss-Legendre routine and marshals arguments.
"""
from .oracle import (  # noqa: F401
    Case, quadrature, build, lib_path, moments, residual, flux_div, sweep,
    cg, diffusion_T, steady, keff, transient, apply_jac_T, dR_dgamma, sweep_T,
    BC_THERMAL, BC_SPECULAR, BC_DIFFUSE, BC_PERIODIC, BC_INTERFACE, LIM_NONE, LIM_MC, LIM_MINMOD,
)
