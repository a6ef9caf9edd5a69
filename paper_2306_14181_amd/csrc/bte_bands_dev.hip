// bte_bands_dev.hip -- mean-free-path band discretisation (Sec. 3.1, eq.
// banddis) with the mode list in device memory: the range of the mean free
// path (one block), the interval of every mode, the three band sums of each
// interval (one block per interval, a fixed summation order, so the result
// is the same on every call), the compaction of the non-empty intervals and
// the renumbering of the modes' band indices.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/bte.h"

namespace bte {

namespace {

constexpr int kBdThreads = 256;

// scratch layout: header of 4 doubles (lmin, lmax, flags as doubles),
// then 3 n_bands band sums, then n_bands ints (interval -> band index)
struct BdScratch {
    double *hdr;
    double *sums;
    int *renum;
};

__host__ __device__ inline BdScratch bd_layout(void *base, int n_bands)
{
    BdScratch s;
    s.hdr = static_cast<double *>(base);
    s.sums = s.hdr + 4;
    s.renum = reinterpret_cast<int *>(s.sums + 3 * (size_t)n_bands);
    return s;
}

// Range of the mean free path v tau over the modes with v tau > 0 and the
// validity of the list: hdr = {lmin, lmax, number of invalid modes, number of
// modes with a positive mean free path}.  One block.
__global__ __launch_bounds__(1024) void k_bd_range(const double *__restrict__ C, const double *__restrict__ v,
                                                   const double *__restrict__ tau, long long n, double *hdr)
{
    __shared__ double smin[1024], smax[1024];
    __shared__ long long sbad[1024], spos[1024];
    double lo = INFINITY, hi = 0.0;
    long long bad = 0, pos = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const double c = C[i], vi = v[i], ti = tau[i];
        if (!(c >= 0.0) || !(vi >= 0.0) || !(ti > 0.0)) ++bad;
        const double L = vi * ti;
        if (L > 0.0) {
            ++pos;
            lo = fmin(lo, L);
            hi = fmax(hi, L);
        }
    }
    const int t = threadIdx.x;
    smin[t] = lo;
    smax[t] = hi;
    sbad[t] = bad;
    spos[t] = pos;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) {
            smin[t] = fmin(smin[t], smin[t + o]);
            smax[t] = fmax(smax[t], smax[t + o]);
            sbad[t] += sbad[t + o];
            spos[t] += spos[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        hdr[0] = smin[0];
        hdr[1] = smax[0];
        hdr[2] = (double)sbad[0];
        hdr[3] = (double)spos[0];
    }
}

// Interval of every mode: equal widths in log(Lambda) over [lmin, lmax], the
// last closed; modes without a mean free path (v = 0) join interval 0.
__global__ __launch_bounds__(kBdThreads) void k_bd_bin(const double *__restrict__ v, const double *__restrict__ tau,
                                                       long long n, double l0, double span, int n_bands,
                                                       int *__restrict__ bin)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L = v[i] * tau[i];
    int k = 0;
    if (L > 0.0 && span > 0.0) {
        const double x = (log(L) - l0) / span * n_bands;
        k = (int)floor(x);
        k = k < 0 ? 0 : (k > n_bands - 1 ? n_bands - 1 : k);
    }
    bin[i] = k;
}

// Band sums of interval blockIdx.x: sum C, sum C v, sum C v^2 tau.  Thread t
// takes the modes t, t + 256, ... in order; the 256 partials are then added
// in a fixed tree order.
__global__ __launch_bounds__(kBdThreads) void k_bd_sum(const double *__restrict__ C, const double *__restrict__ v,
                                                       const double *__restrict__ tau, const int *__restrict__ bin,
                                                       long long n, double *__restrict__ sums)
{
    __shared__ double sh[3][kBdThreads];
    const int k = blockIdx.x, t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long long i = t; i < n; i += kBdThreads) {
        if (bin[i] != k) continue;
        const double cv = C[i] * v[i];
        s0 += C[i];
        s1 += cv;
        s2 += cv * v[i] * tau[i];
    }
    sh[0][t] = s0;
    sh[1][t] = s1;
    sh[2][t] = s2;
    __syncthreads();
    for (int o = kBdThreads / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + o];
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < 3; ++q) sums[3 * (size_t)k + q] = sh[q][0];
}

// Compaction of the non-empty intervals in ascending mean free path (one
// thread): the representative band values of eq. banddis and the band index
// of each interval (-1: dropped, its sum C v is zero); hdr[2] = bands kept.
__global__ void k_bd_final(const double *__restrict__ sums, int n_bands, double *C_out, double *v_out,
                           double *tau_out, int *renum, double *hdr)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nb = 0;
    for (int k = 0; k < n_bands; ++k) {
        const double sc = sums[3 * k], scv = sums[3 * k + 1], scvt = sums[3 * k + 2];
        renum[k] = -1;
        if (!(sc > 0.0) || !(scv > 0.0)) continue;
        const double vb = scv / sc;
        C_out[nb] = sc;
        v_out[nb] = vb;
        tau_out[nb] = scvt / (vb * scv);
        renum[k] = nb++;
    }
    hdr[2] = (double)nb;
}

__global__ __launch_bounds__(kBdThreads) void k_bd_renum(int *__restrict__ bin, const int *__restrict__ renum,
                                                         long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bin[i] = renum[bin[i]];
}

}  // namespace

}  // namespace bte

using namespace bte;

extern "C" size_t bte_band_discretize_scratch_bytes(int n_bands)
{
    if (n_bands < 1) return 0;
    const size_t b = 8 * (4 + 3 * (size_t)n_bands) + 4 * (size_t)n_bands;
    return (b + 255) & ~size_t(255);
}

extern "C" bte_status bte_band_discretize_dev(const double *C, const double *v, const double *tau, long long n_modes,
                                              int n_bands, double *C_out, double *v_out, double *tau_out,
                                              int *n_out, int *band_of_mode, void *scratch, size_t scratch_bytes,
                                              void *stream)
{
    if (!C || !v || !tau || !C_out || !v_out || !tau_out || !n_out || !band_of_mode || !scratch || n_modes < 1 ||
        n_bands < 1 || n_modes > 2147483647ll)
        return BTE_ERR_ARG;
    if (scratch_bytes < bte_band_discretize_scratch_bytes(n_bands) || ((uintptr_t)scratch & 255)) return BTE_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const BdScratch S = bd_layout(scratch, n_bands);
    hipLaunchKernelGGL(k_bd_range, dim3(1), dim3(1024), 0, s, C, v, tau, n_modes, S.hdr);
    double hdr[4];
    if (hipMemcpyAsync(hdr, S.hdr, sizeof hdr, hipMemcpyDeviceToHost, s) != hipSuccess) return BTE_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BTE_ERR_HIP;
    // invalid values or no mode with a mean free path: nothing is written
    if (hdr[2] != 0.0 || !(hdr[3] > 0.0)) return BTE_ERR_ARG;
    const double l0 = log(hdr[0]), span = log(hdr[1]) - l0;
    const unsigned grid = (unsigned)((n_modes + kBdThreads - 1) / kBdThreads);
    hipLaunchKernelGGL(k_bd_bin, dim3(grid), dim3(kBdThreads), 0, s, v, tau, n_modes, l0, span, n_bands,
                       band_of_mode);
    hipLaunchKernelGGL(k_bd_sum, dim3(n_bands), dim3(kBdThreads), 0, s, C, v, tau, band_of_mode, n_modes, S.sums);
    hipLaunchKernelGGL(k_bd_final, dim3(1), dim3(64), 0, s, S.sums, n_bands, C_out, v_out, tau_out, S.renum, S.hdr);
    hipLaunchKernelGGL(k_bd_renum, dim3(grid), dim3(kBdThreads), 0, s, band_of_mode, S.renum, n_modes);
    if (hipGetLastError() != hipSuccess) return BTE_ERR_HIP;
    double nb = 0.0;
    if (hipMemcpyAsync(&nb, S.hdr + 2, sizeof nb, hipMemcpyDeviceToHost, s) != hipSuccess) return BTE_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return BTE_ERR_HIP;
    *n_out = (int)nb;
    return nb > 0 ? BTE_OK : BTE_ERR_ARG;
}
