// bte_adjoint.hip -- kernels of the adjoint (transposed) iteration for the
// gradient of the effective conductivity with respect to a per-cell extra
// scattering rate gamma (1/tau_i = 1/tau + gamma_i).
//
// The steady residual R(e, gamma) = 0 (Sec. 3.3 / 3.5 with the closures of
// Sec. 2.2) defines e(gamma); for J = g.e the gradient is
//   dJ/dgamma_i = sum_{alpha,lambda} psi dR/dgamma_i,   J_e^T psi = -g.
// The forward synthetic iteration e <- e + M R(e) has
//   M = (I + P L^-1 Q) A^-1
// (A: first-order upwind sweep operator, Q x = sum w x / tau per cell,
// L: correction diffusion operator, P: isotropic prolongation C/(4 pi)).
// The adjoint runs its transpose,
//   psi <- psi + A^-T (I + Q^T L^-1 P^T) (J^T psi + g),
// whose iteration matrix is the transpose of the forward one: same
// convergence rate.  Per iteration: diffuse-wall sums of psi (k_walls_adj),
// y = J^T psi + g with its per-cell moments P^T y and |y|^2 (k_adj_res),
// the CG solve L v = P^T y, and the reversed sweep (k_sweep_tile<ADJ>).
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tile.h"
#include "bte_tilelds.h"
#include "bte_adjflux.h"

namespace bte {

// Per diffuse wall record and band: sum over the lanes that enter the cell
// through that wall of cpl psi, divided by sum_{incoming} w |s.n|.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_walls_adj(Dev d, const T *__restrict__ psi, const int *__restrict__ wrec,
                                                       const double *__restrict__ wden, double *__restrict__ dinA,
                                                       int nw)
{
    __shared__ double sh[kBlock];
    const int r = blockIdx.x;
    if (r >= nw) return;
    const int c = wrec[2 * r], f = wrec[2 * r + 1];
    const int a = f >> 1, side = (f & 1) ? 1 : -1;
    const Film &fm = d.film[d.fid[c]];
    const int G = kBlock / d.nl;
    const int grp = threadIdx.x / d.nl, l = threadIdx.x - grp * d.nl;
    double sum = 0.0;
    if (grp < G) {
        const double cv = d.v[l] * fm.ih[a];
        for (int al = grp; al < d.na; al += G) {
            const double sa = d.s[3 * al + a];
            if (sa * side >= 0.0) continue;
            sum += cv * fabs(sa) * (double)psi[(size_t)c * d.nk + al * d.nl + l];
        }
    }
    sh[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x < d.nl) {
        double t = 0.0;
        for (int g2 = 0; g2 < G; ++g2) t += sh[g2 * d.nl + threadIdx.x];
        dinA[(size_t)r * d.nl + threadIdx.x] = t / wden[f];
    }
}

// y = J^T psi + g on a tile, every lane chunk of the reversed octant; per
// cell the block accumulates sum C/(4 pi) y (= P^T y) and sum y^2 and writes
// them once: part[(oct * 2 + q) * nc + cell].  X = per-cell isotropic term
// (sum C/(4 pi) (1/tau) psi / S, the transposed scattering closure).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_res(Dev d, const T *__restrict__ psi, const double *__restrict__ X,
                                                 const double *__restrict__ dinA, const TileItem *__restrict__ items,
                                                 int nitems, int3 tdim, int na_oct, int nchunk_oct, int cap,
                                                 double *__restrict__ part)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ T sy[4][8][64];
    __shared__ double sc4[64];
    TileSmem<T> S = tile_smem<T>(smem, cap, false);
    const int nb = gridDim.x, bb = blockIdx.x;
    const int lb = (bb & 7) * (nb >> 3) + (bb >> 3);
    if (lb >= nitems) return;
    const TileItem it = items[lb];
    const Film &fm = d.film[it.film];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const TileCtx t = tile_make(fm, d.dim, octant_sign(d, it.oct, na_oct, 0), octant_sign(d, it.oct, na_oct, 1),
                                octant_sign(d, it.oct, na_oct, 2), it.tile, tdim);
    tile_tables<T>(t, fm, d, S, X, nullptr, false);
    for (int i = threadIdx.x; i < 128; i += blockDim.x) S.mom[i] = 0.0;
    __syncthreads();
    tile_modes<T>(t, d, S, true);
    const int loct = it.oct ^ ((1 << d.dim) - 1);
    const int kbeg = loct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const double gfac = fm.pdT[0] != 0.0 ? fm.len[0] / (fm.pdT[0] * fm.ncell) : 0.0;
    for (int ch = 0; ch < nchunk_oct; ++ch) {
        const int k = kbeg + ch * 64 + lane;
        const bool active = k < kend;
        const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
        T wsa[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) wsa[a] = (T)(L.w * fabs(d.s[3 * L.al + a]));
        const T gl = (T)(gfac * L.wv[0]);
        if (wave == 0) sc4[lane] = active ? d.C4[L.l] : 0.0;
        tile_load<T>(t, S, psi, k, active, L.C4, static_cast<const T *>(d.zrow));
        __syncthreads();
        T *const ys = &sy[wave][0][0];
        const int nmine = (t.nt - wave + 3) / 4;   // cells i = wave + 4 m
        for (int m0 = 0; m0 < nmine; m0 += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int m = m0 + j;
                T y = (T)0;
                if (m < nmine) {
                    const int i = wave + 4 * m;
                    if (active && (uni(S.code[i]) & kSolidBit)) {
                        int up_out[3];
                        const T tf = tile_flux_adj<T, DIM>(d, t, S, i, L, wsa, lane, psi, dinA, up_out);
                        const T ec = S.box[i * 64 + lane];
                        const T itc = L.itau + (T)S.gam[i];
                        y = tf - ec * itc + (T)L.w * itc * (T)S.tl[i] + gl;
                    }
                }
                ys[j * 64 + lane] = y;
            }
            const int j = lane >> 3, p8 = lane & 7;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int l2 = 8 * p8 + q;
                const double y = (double)ys[j * 64 + l2];
                a0 += sc4[l2] * y;
                a1 += y * y;
            }
            a0 += dpp_f64<0xB1>(a0);
            a0 += dpp_f64<0x4E>(a0);
            a0 += dpp_f64<0x141>(a0);
            a1 += dpp_f64<0xB1>(a1);
            a1 += dpp_f64<0x4E>(a1);
            a1 += dpp_f64<0x141>(a1);
            const int mj = m0 + j;
            if (p8 == 0 && mj < nmine) {
                const int i = wave + 4 * mj;
                S.mom[2 * i] += a0;
                S.mom[2 * i + 1] += a1;
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < t.nt; i += blockDim.x) {
        part[((size_t)it.oct * 2) * d.nc + S.cell[i]] = S.mom[2 * i];
        part[((size_t)it.oct * 2 + 1) * d.nc + S.cell[i]] = S.mom[2 * i + 1];
    }
}

// u = P^T y and |y|^2 per cell from the per-octant partials
__global__ void k_adj_post(Dev d, const double *__restrict__ part, int noct, double *__restrict__ u,
                           double *__restrict__ r2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    double a = 0, b = 0;
    for (int o = 0; o < noct; ++o) {
        a += part[((size_t)o * 2) * d.nc + c];
        b += part[((size_t)o * 2 + 1) * d.nc + c];
    }
    const bool solid = d.code[c] & kSolidBit;
    u[c] = solid ? a : 0.0;
    r2[c] = solid ? b : 0.0;
}

// X = sum_p part[p][c][0] / S_c (slot 0 of the sweep's moment partials)
__global__ void k_adj_phi(Dev d, const double *__restrict__ part, int np, double *__restrict__ X)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    double a = 0;
    for (int p = 0; p < np; ++p) a += part[((size_t)p * d.nc + c) * kMomN];
    X[c] = (d.code[c] & kSolidBit) ? a / d.S[c] : 0.0;
}

// dJ/dgamma_c = sum psi dR/dgamma_c with
//   dR/dgamma_c = -(e - C T_L/4pi) + C/(4 pi tau_c) dT_L/dgamma_c,
//   dT_L/dgamma_c = C_tot (T_c - T_L,c) / S_c   (deviations from T_ref),
// i.e. -sum psi e + T_L sum psi C/4pi + C_tot (T - T_L) X_c (X as above).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_grad(Dev d, const T *__restrict__ e, const T *__restrict__ psi,
                                                      const double *__restrict__ Tdev,
                                                      const double *__restrict__ TLdev,
                                                      const double *__restrict__ X, double *__restrict__ grad)
{
    __shared__ double sh[4 * 2];
    const int c = blockIdx.x;
    double acc[2] = {0, 0};
    const bool solid = d.code[c] & kSolidBit;
    if (solid) {
        for (int k = threadIdx.x; k < d.nk; k += kBlock) {
            const int l = k % d.nl;
            const double ps = (double)psi[(size_t)c * d.nk + k];
            acc[0] += ps * (double)e[(size_t)c * d.nk + k];
            acc[1] += ps * d.C4[l];
        }
    }
    // block reduction (fixed order)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double x = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        acc[q] = x;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[2 * wave] = acc[0];
        sh[2 * wave + 1] = acc[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double A = sh[0] + sh[2] + sh[4] + sh[6], B = sh[1] + sh[3] + sh[5] + sh[7];
        grad[c] = solid ? -A + TLdev[c] * B + d.Ctot * (Tdev[c] - TLdev[c]) * X[c] : 0.0;
    }
}


// Transposed explicit step of the transient adjoint (reverse mode of
// e^{k+1} = e^k + dt R(e^k)):  lam^k = lam^{k+1} + dt J^T lam^{k+1}, with the
// forward state e^k read alongside for the gradient and TLk = T_L(e^k), the
// lattice temperature the forward step of e^k used.  Per (octant, cell) the
// block writes two partial sums, part[(oct * 2 + q) * nc + cell]:
//   q = 0: sum C/(4 pi) (1/tau) lam^k        (closure term of the next step)
//   q = 1: sum lam^{k+1} (C/(4 pi) T_L - e^k) + w X e^k
// (the gradient's sums over (direction, band) in one: with X = Phi(lam^{k+1})
// and T = sum w e^k / C_tot, the per-cell term -sum lam e + T_L sum lam C/4pi
// + C_tot (T - T_L) X is q = 1 minus C_tot T_L X).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_adj_step(Dev d, const T *__restrict__ lam, T *__restrict__ lout,
                                                  const T *__restrict__ ek, const double *__restrict__ X,
                                                  const double *__restrict__ TLk, const double *__restrict__ dinA,
                                                  const TileItem *__restrict__ items, int nitems, int3 tdim,
                                                  int na_oct, int nchunk_oct, int cap, double dt,
                                                  double *__restrict__ part)
{
    extern __shared__ __align__(16) char smem[];
    TileSmem<T> S = tile_smem<T>(smem, cap, false);
    const int nb = gridDim.x, bb = blockIdx.x;
    const int lb = (bb & 7) * (nb >> 3) + (bb >> 3);
    if (lb >= nitems) return;
    const TileItem it = items[lb];
    const Film &fm = d.film[it.film];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const TileCtx t = tile_make(fm, d.dim, octant_sign(d, it.oct, na_oct, 0), octant_sign(d, it.oct, na_oct, 1),
                                octant_sign(d, it.oct, na_oct, 2), it.tile, tdim);
    tile_tables<T>(t, fm, d, S, X, nullptr, false);
    for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) S.mom[i] = 0.0;
    __syncthreads();
    tile_modes<T>(t, d, S, true);
    const int loct = it.oct ^ ((1 << d.dim) - 1);
    const int kbeg = loct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const T tdt = (T)dt;
    for (int ch = 0; ch < nchunk_oct; ++ch) {
        const int k = kbeg + ch * 64 + lane;
        const bool active = k < kend;
        const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
        T wsa[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) wsa[a] = (T)(L.w * fabs(d.s[3 * L.al + a]));
        const double c4 = d.C4[L.l], it0 = d.itau[L.l];
        tile_load<T>(t, S, lam, k, active, L.C4, static_cast<const T *>(d.zrow));
        __syncthreads();
        for (int i = wave; i < t.nt; i += 4) {
            const int c = uni(S.cell[i]);
            const bool solid = uni(S.code[i]) & kSolidBit;
            double acc[2] = {0, 0};
            if (active) {
                if (solid) {
                    int up_out[3];
                    const T tf = tile_flux_adj<T, DIM>(d, t, S, i, L, wsa, lane, lam, dinA, up_out);
                    const T lc = S.box[i * 64 + lane];
                    const T itc = L.itau + (T)S.gam[i];
                    const T ln = lc + tdt * (tf - lc * itc + (T)L.w * itc * (T)S.tl[i]);
                    lout[(size_t)c * d.nk + k] = ln;
                    const double x = (double)ek[(size_t)c * d.nk + k];
                    acc[0] = c4 * (it0 + S.gam[i]) * (double)ln;
                    acc[1] = (double)lc * (c4 * TLk[c] - x) + L.w * X[c] * x;
                } else {
                    lout[(size_t)c * d.nk + k] = (T)0;
                }
            }
            wave_sum_t<2>(acc);
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < 2; ++q) S.mom[2 * i + q] += acc[q];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < t.nt; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < 2; ++q) part[((size_t)it.oct * 2 + q) * d.nc + S.cell[i]] = S.mom[2 * i + q];
}

// Per cell after a transposed step (two partials per octant, or per (octant,
// chunk) column group, as the step kernels write them): the next closure
// term Xn = Phi(lam^k) and
//   grad += dt (-sum lam e + T_L sum lam C/4pi + C_tot (T - T_L) X)
//         = dt (part_1 - C_tot T_L X)
// with T, T_L the deviations of e^k, T_L = TLk, and X = Phi(lam^{k+1})
// (dR/dgamma as in the steady gradient).
// 64 cells per block, the partials split over the four wavefronts as in
// k_finalize_tl.
__global__ __launch_bounds__(kBlock) void k_adj_step_post(Dev d, const double *__restrict__ part, int noct,
                                                          const double *__restrict__ X,
                                                          const double *__restrict__ TLk, double *__restrict__ Xn,
                                                          double *__restrict__ grad, double dt)
{
    __shared__ double sh[2][4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    double s[2] = {0, 0};
    if (c < d.nc)
        for (int o = w; o < noct; o += 4)
            for (int q = 0; q < 2; ++q) s[q] += part[((size_t)o * 2 + q) * d.nc + c];
    sh[0][w][lane] = s[0];
    sh[1][w][lane] = s[1];
    __syncthreads();
    if (w != 0 || c >= d.nc) return;
    if (!(d.code[c] & kSolidBit)) {
        Xn[c] = 0.0;
        return;
    }
    const double s0 = (sh[0][0][lane] + sh[0][1][lane]) + (sh[0][2][lane] + sh[0][3][lane]);
    const double s1 = (sh[1][0][lane] + sh[1][1][lane]) + (sh[1][2][lane] + sh[1][3][lane]);
    grad[c] += dt * (s1 - d.Ctot * TLk[c] * X[c]);
    Xn[c] = s0 / d.S[c];
}

// lam^N = dJ/de^N for J = sum_c a_c T_c / sum_c a_c:  a_c w / (A C_tot)
template <typename T>
__global__ void k_adj_tave_init(Dev d, const double *__restrict__ a, double inv_sum_a, T *__restrict__ lam)
{
    const size_t n = (size_t)d.nc * d.nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / d.nk), k = (int)(i - (size_t)c * d.nk);
        const int al = k / d.nl;
        lam[i] = (d.code[c] & kSolidBit) ? (T)(a[c] * inv_sum_a * d.w[al] / d.Ctot) : (T)0;
    }
}

// Phi(lam) = sum C/(4 pi) (1/tau) lam / S per cell (one block per cell)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_phi_cell(Dev d, const T *__restrict__ lam, double *__restrict__ X)
{
    __shared__ double sh[4];
    const int c = blockIdx.x;
    double acc = 0;
    const bool solid = d.code[c] & kSolidBit;
    if (solid) {
        const double g = d.gamma[c];
        for (int k = threadIdx.x; k < d.nk; k += kBlock) {
            const int l = k % d.nl;
            acc += d.C4[l] * (d.itau[l] + g) * (double)lam[(size_t)c * d.nk + k];
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) X[c] = solid ? (sh[0] + sh[1] + sh[2] + sh[3]) / d.S[c] : 0.0;
}

// J = sum a T / sum a, T absolute (one block; T from the moments)
__global__ __launch_bounds__(kBlock) void k_tave(Dev d, const double *__restrict__ a, const double *__restrict__ T,
                                                 double *__restrict__ out)
{
    __shared__ double sh[8];
    double x = 0, y = 0;
    for (int c = threadIdx.x; c < d.nc; c += kBlock) {
        x += a[c] * T[c];
        y += a[c];
    }
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = x;
        sh[4 + (threadIdx.x >> 6)] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (sh[0] + sh[1] + sh[2] + sh[3]) / (sh[4] + sh[5] + sh[6] + sh[7]);
        out[1] = sh[4] + sh[5] + sh[6] + sh[7];
    }
}

// ------------------------------------------------------------------ launchers

template <typename T>
void launch_walls_adj(const Dev &d, const T *psi, const int *wrec, const double *wden, double *dinA, int nw,
                      hipStream_t s)
{
    if (nw > 0) hipLaunchKernelGGL(k_walls_adj<T>, dim3(nw), dim3(kBlock), 0, s, d, psi, wrec, wden, dinA, nw);
}

template <typename T, int DIM>
void adj_res_launch(const Dev &d, const T *psi, const double *X, const double *dinA, const TileItem *items,
                    int nitems, int3 tdim, int na_oct, int nchunk_oct, int cap, double *part, hipStream_t s)
{
    const size_t sm = tile_smem_bytes(cap, sizeof(T), false);
    const int grid = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((k_adj_res<T, DIM>), dim3(grid), dim3(256), sm, s, d, psi, X, dinA, items, nitems, tdim,
                       na_oct, nchunk_oct, cap, part);
}

template <typename T>
hipError_t launch_adj_res(const Dev &d, const T *psi, const double *X, const double *dinA, const TileItem *items,
                          int nitems, int3 tdim, int na_oct, int nchunk_oct, int cap, double *part, hipStream_t s)
{
    if (d.dim == 1) adj_res_launch<T, 1>(d, psi, X, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, part, s);
    if (d.dim == 2) adj_res_launch<T, 2>(d, psi, X, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, part, s);
    if (d.dim == 3) adj_res_launch<T, 3>(d, psi, X, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, part, s);
    return hipGetLastError();
}

void launch_adj_post(const Dev &d, const double *part, int noct, double *u, double *r2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_post, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, part, noct, u, r2);
}

void launch_adj_phi(const Dev &d, const double *part, int np, double *X, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_phi, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, part, np, X);
}

template <typename T>
void launch_adj_grad(const Dev &d, const T *e, const T *psi, const double *Tdev, const double *TLdev, const double *X,
                     double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_grad<T>, dim3(d.nc), dim3(kBlock), 0, s, d, e, psi, Tdev, TLdev, X, grad);
}


template <typename T, int DIM>
void adj_step_launch(const Dev &d, const T *lam, T *lout, const T *ek, const double *X, const double *TLk,
                     const double *dinA, const TileItem *items, int nitems, int3 tdim, int na_oct, int nchunk_oct,
                     int cap, double dt, double *part, hipStream_t s)
{
    const size_t sm = tile_smem_bytes(cap, sizeof(T), false);
    const int grid = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((k_adj_step<T, DIM>), dim3(grid), dim3(256), sm, s, d, lam, lout, ek, X, TLk, dinA, items,
                       nitems, tdim, na_oct, nchunk_oct, cap, dt, part);
}

template <typename T>
hipError_t launch_adj_step(const Dev &d, const T *lam, T *lout, const T *ek, const double *X, const double *TLk,
                           const double *dinA, const TileItem *items, int nitems, int3 tdim, int na_oct,
                           int nchunk_oct, int cap, double dt, double *part, hipStream_t s)
{
    if (d.dim == 1)
        adj_step_launch<T, 1>(d, lam, lout, ek, X, TLk, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, dt, part, s);
    if (d.dim == 2)
        adj_step_launch<T, 2>(d, lam, lout, ek, X, TLk, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, dt, part, s);
    if (d.dim == 3)
        adj_step_launch<T, 3>(d, lam, lout, ek, X, TLk, dinA, items, nitems, tdim, na_oct, nchunk_oct, cap, dt, part, s);
    return hipGetLastError();
}

void launch_adj_step_post(const Dev &d, const double *part, int noct, const double *X, const double *TLk, double *Xn,
                          double *grad, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_step_post, dim3((d.nc + 63) / 64), dim3(kBlock), 0, s, d, part, noct, X, TLk, Xn, grad,
                       dt);
}

template <typename T>
void launch_adj_tave_init(const Dev &d, const double *a, double inv_sum_a, T *lam, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_tave_init<T>, dim3(4096), dim3(kBlock), 0, s, d, a, inv_sum_a, lam);
}

template <typename T> void launch_adj_phi_cell(const Dev &d, const T *lam, double *X, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_phi_cell<T>, dim3(d.nc), dim3(kBlock), 0, s, d, lam, X);
}

void launch_tave(const Dev &d, const double *a, const double *T, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_tave, dim3(1), dim3(kBlock), 0, s, d, a, T, out);
}

template <typename T> hipError_t set_lds_adj(size_t bytes)
{
    hipError_t r = hipSuccess, x;
    // k_adj_res also has static LDS (its staging of 8 cells per wavefront)
    const int res_bytes = (int)bytes - (int)(sizeof(T) * 4 * 8 * 64 + 8 * 64);
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_res<T, 1>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, res_bytes)) != hipSuccess) r = x;
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_res<T, 2>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, res_bytes)) != hipSuccess) r = x;
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_res<T, 3>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, res_bytes)) != hipSuccess) r = x;
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_step<T, 1>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) r = x;
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_step<T, 2>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) r = x;
    if ((x = hipFuncSetAttribute(reinterpret_cast<const void *>(k_adj_step<T, 3>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)) != hipSuccess) r = x;
    return r;
}

hipError_t adj_kernels_init(size_t max_bytes)
{
    hipError_t a = set_lds_adj<float>(max_bytes), b = set_lds_adj<double>(max_bytes);
    return a != hipSuccess ? a : b;
}

template void launch_walls_adj<float>(const Dev &, const float *, const int *, const double *, double *, int,
                                      hipStream_t);
template void launch_walls_adj<double>(const Dev &, const double *, const int *, const double *, double *, int,
                                       hipStream_t);
template hipError_t launch_adj_res<float>(const Dev &, const float *, const double *, const double *,
                                          const TileItem *, int, int3, int, int, int, double *, hipStream_t);
template hipError_t launch_adj_res<double>(const Dev &, const double *, const double *, const double *,
                                           const TileItem *, int, int3, int, int, int, double *, hipStream_t);
template void launch_adj_grad<float>(const Dev &, const float *, const float *, const double *, const double *,
                                     const double *, double *, hipStream_t);
template void launch_adj_grad<double>(const Dev &, const double *, const double *, const double *, const double *,
                                      const double *, double *, hipStream_t);

template hipError_t launch_adj_step<float>(const Dev &, const float *, float *, const float *, const double *,
                                           const double *, const double *, const TileItem *, int, int3, int, int, int,
                                           double, double *, hipStream_t);
template hipError_t launch_adj_step<double>(const Dev &, const double *, double *, const double *, const double *,
                                            const double *, const double *, const TileItem *, int, int3, int, int, int,
                                            double, double *, hipStream_t);
template void launch_adj_tave_init<float>(const Dev &, const double *, double, float *, hipStream_t);
template void launch_adj_tave_init<double>(const Dev &, const double *, double, double *, hipStream_t);
template void launch_adj_phi_cell<float>(const Dev &, const float *, double *, hipStream_t);
template void launch_adj_phi_cell<double>(const Dev &, const double *, double *, hipStream_t);

}  // namespace bte
