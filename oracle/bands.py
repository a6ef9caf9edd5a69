"""Mean-free-path band discretisation, written from Sec. 3.1, eq. banddis
(test infrastructure only, like the rest of oracle/).

The mode list (C, v, tau) is isotropic (the paper's assumption).  The mean
free path Lambda = v tau of the modes with Lambda > 0 spans
[Lambda_min, Lambda_max]; the paper divides that range into bands without
saying how, and the reading here is equal widths in log(Lambda): mode i
falls in interval floor(n (log Lambda_i - log Lambda_min) / (log Lambda_max -
log Lambda_min)), the last interval closed; modes with v = 0 join the
first.  For each band the representative properties are the eq. banddis
sums: C_b = sum C, v_b = sum C v / sum C, tau_b = sum C v^2 tau / (v_b sum C v).
Intervals whose sum C v is zero are dropped.  Plain Python loops with
math.log (the same libm as the library's host code, so the interval of a
mode is decided identically).
"""
import math


def band_discretize(C, v, tau, n_bands):
    """Returns (C_b, v_b, tau_b) lists in ascending mean free path and the
    band index of every mode (-1 for a mode of a dropped interval)."""
    n = len(C)
    lam = [float(v[i]) * float(tau[i]) for i in range(n)]
    pos = [x for x in lam if x > 0]
    if n < 1 or n_bands < 1 or not pos:
        raise ValueError("need modes with a positive mean free path and n_bands >= 1")
    lo, hi = min(pos), max(pos)
    l0 = math.log(lo)
    span = math.log(hi) - l0
    interval = []
    for x in lam:
        k = 0
        if x > 0 and span > 0:
            k = int(math.floor((math.log(x) - l0) / span * n_bands))
            k = min(max(k, 0), n_bands - 1)
        interval.append(k)
    sums = [[0.0, 0.0, 0.0] for _ in range(n_bands)]   # sum C, sum C v, sum C v^2 tau
    for i in range(n):
        s = sums[interval[i]]
        c, vi, ti = float(C[i]), float(v[i]), float(tau[i])
        s[0] += c
        s[1] += c * vi
        s[2] += c * vi * vi * ti
    Cb, vb, tb, index = [], [], [], [-1] * n_bands
    for k in range(n_bands):
        sc, scv, scvt = sums[k]
        if sc > 0 and scv > 0:
            index[k] = len(Cb)
            Cb.append(sc)
            vb.append(scv / sc)
            tb.append(scvt / ((scv / sc) * scv))
    return Cb, vb, tb, [index[k] for k in interval]
