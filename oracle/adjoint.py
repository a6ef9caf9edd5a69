"""Adjoint gradients for the oracle (test infrastructure only).

Steady: R(e, gamma) = 0 and J = g.e (k_eff is linear in e).  The adjoint
psi solves (dR/de)^T psi = -g and dJ/dgamma_i = sum_{alpha,lambda} psi
dR/dgamma_i.  The transposed Jacobian is applied by the C oracle
(``orc_apply_jac_T``); the linear system is solved with scipy's GMRES,
left-preconditioned by the transposed first-order sweep.

Transient: J = sum_c a_c T_c(e^N) after N explicit steps
e^{n+1} = e^n + dt R(e^n); reverse-mode accumulation with all states kept.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, gmres

from . import oracle as O


def keff_weights(case):
    """g with k_eff = g.e : (L_x / (dT N_cells)) w_alpha v_lambda s_alpha,x on solid cells."""
    nc, na, nl = case.nc, case.na, case.nl
    solid = np.ones(nc) if case.solid is None else case.solid.astype(np.float64)
    fac = case.len[0] / (case.pdT[0] * nc)
    g = fac * solid[:, None, None] * (case.w * case.s[:, 0])[None, :, None] * case.v[None, None, :]
    return g.reshape(-1)


def steady_adjoint(case, e, g, rtol=1e-13, maxiter=2000):
    """Solve (dR/de)^T psi = -g; return psi and dJ/dgamma per cell."""
    n = case.size

    def mv(x):
        return -O.sweep_T(case, O.apply_jac_T(case, x))

    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    b = O.sweep_T(case, g)
    psi, info = gmres(op, b, rtol=rtol, atol=0.0, restart=200, maxiter=maxiter)
    if info != 0:
        raise RuntimeError("adjoint GMRES did not converge (info=%d)" % info)
    return psi, O.dR_dgamma(case, e, psi)


def tave_grad_T(case, weights):
    """dJ/de for J = sum_c a_c T_c / sum_c a_c with T the local temperature."""
    a = np.asarray(weights, dtype=np.float64) / np.sum(weights)
    ct = case.C.sum()
    return (a[:, None, None] * (case.w / ct)[None, :, None] * np.ones(case.nl)[None, None, :]).reshape(-1)


def transient_adjoint(case, e0, n_steps, dt, t0=0.0, pulse=None, weights=None):
    """J = weighted mean of T after n_steps; returns (J, dJ/dgamma)."""
    states = [np.array(e0, dtype=np.float64).reshape(-1)]
    e = states[0].copy()
    for k in range(n_steps):
        e, _ = O.transient(case, e, 1, dt, t0 + k * dt, pulse)
        states.append(e.copy())
    T, _, _ = O.moments(case, states[-1])
    a = np.asarray(weights, dtype=np.float64)
    J = float(np.sum(a * T) / np.sum(a))
    lam = tave_grad_T(case, weights)
    grad = np.zeros(case.nc)
    for k in range(n_steps - 1, -1, -1):
        # e^{k+1} = e^k + dt R(e^k):  dJ/dgamma += dt lam^{k+1} . dR/dgamma(e^k)
        grad += dt * O.dR_dgamma(case, states[k], lam)
        lam = lam + dt * O.apply_jac_T(case, lam)
    return J, grad
