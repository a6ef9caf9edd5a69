"""MI355X (gfx950) phonon-BTE hot path: discrete-ordinates transport step,
moments, steady source iteration with synthetic correction, explicit
transient step and adjoint, behind the C ABI of include/bte.h.

``paper_2306_14181_amd.bte`` is the ctypes binding of the HIP library
(import it explicitly; building the package needs no GPU).
"""
