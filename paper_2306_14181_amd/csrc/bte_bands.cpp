// bte_bands.cpp -- mean-free-path band discretisation (Sec. 3.1, eq.
// banddis): the step that turns a mode-level list of phonon properties into
// the bands of the PHONON input.  Host code: one pass to find the range of
// the mean free path, one pass that bins every mode and accumulates the
// three band sums, one pass over the bins.
#include <cmath>
#include <vector>

#include "../../include/bte.h"

extern "C" bte_status bte_band_discretize(const double *C, const double *v, const double *tau, long long n_modes,
                                          int n_bands, double *C_out, double *v_out, double *tau_out, int *n_out,
                                          int *band_of_mode)
{
    if (!C || !v || !tau || !C_out || !v_out || !tau_out || !n_out || n_modes < 1 || n_bands < 1)
        return BTE_ERR_ARG;
    *n_out = 0;
    double lmin = 0, lmax = 0;
    bool any = false;
    for (long long i = 0; i < n_modes; ++i) {
        if (!(C[i] >= 0) || !(v[i] >= 0) || !(tau[i] > 0)) return BTE_ERR_ARG;
        const double L = v[i] * tau[i];
        if (L > 0) {
            if (!any || L < lmin) lmin = L;
            if (!any || L > lmax) lmax = L;
            any = true;
        }
    }
    if (!any) return BTE_ERR_ARG;
    const double l0 = std::log(lmin), span = std::log(lmax) - l0;
    // band sums: C, C v, C v^2 tau (accumulated in mode order)
    std::vector<double> sc(n_bands, 0.0), scv(n_bands, 0.0), scvt(n_bands, 0.0);
    std::vector<int> bin(n_modes);
    for (long long i = 0; i < n_modes; ++i) {
        const double L = v[i] * tau[i];
        int k = 0;
        if (L > 0 && span > 0) {
            const double x = (std::log(L) - l0) / span * n_bands;
            k = (int)std::floor(x);
            k = k < 0 ? 0 : (k > n_bands - 1 ? n_bands - 1 : k);
        }
        bin[i] = k;
        const double cv = C[i] * v[i];
        sc[k] += C[i];
        scv[k] += cv;
        scvt[k] += cv * v[i] * tau[i];
    }
    // non-empty bins in ascending mean free path; the lowest bin always
    // holds the mode of the smallest positive mean free path, so every
    // band has sum C v > 0
    std::vector<int> renum(n_bands, -1);
    int nb = 0;
    for (int k = 0; k < n_bands; ++k) {
        if (!(sc[k] > 0) || !(scv[k] > 0)) continue;
        const double vb = scv[k] / sc[k];
        C_out[nb] = sc[k];
        v_out[nb] = vb;
        tau_out[nb] = scvt[k] / (vb * scv[k]);
        renum[k] = nb++;
    }
    if (nb == 0) return BTE_ERR_ARG;
    if (band_of_mode)
        for (long long i = 0; i < n_modes; ++i) band_of_mode[i] = renum[bin[i]];
    *n_out = nb;
    return BTE_OK;
}
