// bte_kernels.hip -- gfx950 kernels of the phonon-BTE hot path.
//
// Streaming kernels work on e[cell][k] with k = alpha*n_bands + lambda; a
// 256-thread block covers 256 consecutive k of one cell (coalesced 1 KiB
// rows for FP32) and loops over a few cells.  Moments (eqs. BTE_get_e0,
// getTQ) are accumulated in FP64 and reduced deterministically: a butterfly
// within each 64-wide wavefront, then a fixed-order sum over the block's
// wavefronts, then a fixed-order sum over k-chunks in a finalize kernel.
#include <algorithm>

#include "bte_internal.h"
#include "bte_stencil.h"

namespace bte {

// ----------------------------------------------------------------- reductions

template <int N>
__device__ inline void wave_sum(double (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
}

// Sum over a 256-thread block; the result is valid in thread 0.
template <int N>
__device__ inline void block_sum(double (&v)[N], double *sh)
{
    wave_sum<N>(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) sh[wave * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = sh[i] + sh[N + i] + sh[2 * N + i] + sh[3 * N + i];
    __syncthreads();
}

// XCD-aware block numbering: consecutive dispatch slots go round-robin over
// the 8 XCDs, so give each XCD a contiguous range of logical blocks (its own
// k-chunk / cell range) to keep stencil neighbours in its L2.  grid % 8 == 0.
__device__ inline int xcd_logical_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// ------------------------------------------------------------------- per cell

// S_c = sum C (1/tau + gamma_c); per-axis conductivities of the heat-diffusion
// operator, k = sum C v^2 tau_c M_aa (M_aa = sum w s_a^2 / Omega, Omega the total
// angle: 4 pi, or 2 pi for a two-dimensional material), and of the
// correction operator, which adds the conduction of the sweep's first-order
// upwind increment, sum C v h_a H_a / Omega (H_a = sum_{s_a>0} w s_a).
__global__ void k_cell_setup(Dev d, double *S, double *kdif, double *kcor, double m0, double m1, double m2,
                             double H0, double H1, double H2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const double g = d.gamma ? d.gamma[c] : 0.0;
    const Film &fm = d.film[d.fid[c]];
    const int mo = fm.moff;   // the geometry's material
    double sm = 0, k = 0, cv = 0;
    for (int l = 0; l < d.nl; ++l) {
        const double C = d.C4[mo + l] * d.omega;
        const double it = d.itau[mo + l] + g;
        const double v = d.v[mo + l];
        sm += C * it;
        k += C * v * v / it;
        cv += C * v;
    }
    S[c] = sm;
    const double m[3] = {m0, m1, m2}, H[3] = {H0, H1, H2};
    for (int a = 0; a < 3; ++a) {
        kdif[a * d.nc + c] = k * m[a];
        kcor[a * d.nc + c] = k * m[a] + cv * fm.h[a] * H[a] / d.omega;
    }
}

// ------------------------------------------------------------------- moments

// Moments of e per cell (eqs. BTE_get_e0 and getTQ: sum w e, sum w e (1/tau +
// gamma), sum w v s_a e) into part[c * 5 + m].  One wavefront per cell, four
// cells per block; a lane reads 16 consecutive bytes (4 FP32 or 2 FP64
// elements) per load, 64 lanes a contiguous 1 KiB, and the direction and
// band of its elements advance incrementally; the quadrature and band
// constants come from LDS tables loaded once per block.  FP64 accumulation,
// then a butterfly over the 64 lanes.  Needs a 16-byte aligned e, nk a
// multiple of the vector width and the tables to fit (k_moments_block
// otherwise).
template <typename T>
__global__ __launch_bounds__(256) void k_moments_wave(Dev d, const T *__restrict__ e,
                                                      const double *__restrict__ dpend, double *__restrict__ part)
{
    constexpr int kV = 16 / (int)sizeof(T);
    extern __shared__ double tab[];
    const int na = d.na, nl = d.nl, nk = d.nk;
    double *tw = tab, *ts0 = tab + na, *ts1 = tab + 2 * na, *ts2 = tab + 3 * na;
    const int nml = d.nmat * nl;   // band tables of every material
    double *tv0 = tab + 4 * na, *tit0 = tv0 + nml, *tc40 = tv0 + 2 * nml;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        tw[i] = d.w[i];
        ts0[i] = d.s[3 * i];
        ts1[i] = d.s[3 * i + 1];
        ts2[i] = d.s[3 * i + 2];
    }
    for (int i = threadIdx.x; i < nml; i += blockDim.x) {
        tv0[i] = d.v[i];
        tit0[i] = d.itau[i];
        tc40[i] = d.C4[i];
    }
    __syncthreads();
    const int c = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (c >= d.nc) return;
    const int lane = threadIdx.x & 63;
    double acc[kMomN] = {0, 0, 0, 0, 0};
    if (d.code[c] & kSolidBit) {
        const int mo = d.nmat > 1 ? d.film[d.fid[c]].moff : 0;
        const double *tv = tv0 + mo, *tit = tit0 + mo, *tc4 = tc40 + mo;
        const double g = d.gamma[c];
        const double dp = dpend ? dpend[c] : 0.0;
        // (direction, band) of the lane's first element and the advance per
        // step of 64 kV elements
        const int k0 = kV * lane, step = 64 * kV;
        int al = k0 / nl, l = k0 - al * nl;
        const int dA = step / nl, dL = step - dA * nl;
        const T *row = e + (size_t)c * nk;
        // two vector loads in flight per lane (the second clamped to the
        // row's last vector when past its end, and then not accumulated)
        auto load = [&](int kb, T (&v)[kV]) {
            if constexpr (kV == 4) {
                const float4 q = *reinterpret_cast<const float4 *>(row + kb);
                v[0] = q.x;
                v[1] = q.y;
                v[2] = q.z;
                v[3] = q.w;
            } else {
                const double2 q = *reinterpret_cast<const double2 *>(row + kb);
                v[0] = q.x;
                v[1] = q.y;
            }
        };
        const bool corr = dp != 0.0;   // uniform: the C/(4 pi) table is read only with a pending correction
        auto accumulate = [&](const T (&v)[kV]) {
            int a = al, b = l;
#pragma unroll
            for (int u = 0; u < kV; ++u) {
                const double x = corr ? (double)v[u] + tc4[b] * dp : (double)v[u];
                const double wx = tw[a] * x;
                acc[0] += wx;
                acc[1] += wx * (tit[b] + g);
                const double vw = wx * tv[b];
                acc[2] += vw * ts0[a];
                acc[3] += vw * ts1[a];
                acc[4] += vw * ts2[a];
                if (++b == nl) {
                    b = 0;
                    ++a;
                }
            }
            al += dA;
            l += dL;
            if (l >= nl) {
                l -= nl;
                ++al;
            }
        };
        for (int kb = k0; kb < nk; kb += 2 * step) {
            const int kb2 = kb + step < nk ? kb + step : nk - kV;
            T v0[kV], v1[kV];
            load(kb, v0);
            load(kb2, v1);
            accumulate(v0);
            if (kb + step < nk) accumulate(v1);
        }
    }
#pragma unroll
    for (int m = 0; m < kMomN; ++m)
        for (int off = 32; off > 0; off >>= 1) acc[m] += __shfl_xor(acc[m], off, 64);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < kMomN; ++m) part[(size_t)c * kMomN + m] = acc[m];
}

// Band-factored form (used when the lanes of a row can keep their bands
// from one load to the next: nl a multiple of the vector width kV, and nL
// lanes of kV values covering a multiple of nl): the moments of a cell are
//   sum_k w_a x,  sum_k w_a (1/tau_b + gamma) x,  sum_k w_a s_a v_b x
// with k = (a, b), so each lane sums its kV values x (same direction a)
// unweighted, weighted by 1/tau_b and by v_b -- band constants it holds in
// registers for the whole row -- and only then applies the direction's
// weights (w_a, w_a s_a) from LDS: two LDS doubles per kV values instead of
// six per value.  One wavefront per cell; lanes nL .. 63 only load nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_moments_band(Dev d, const T *__restrict__ e,
                                                      const double *__restrict__ dpend, double *__restrict__ part,
                                                      int nL)
{
    constexpr int kV = 16 / (int)sizeof(T);
    extern __shared__ double tab[];   // per direction: w, w s0, w s1, w s2
    const int na = d.na, nl = d.nl, nk = d.nk;
    for (int i = threadIdx.x; i < na; i += blockDim.x) {
        const double w = d.w[i];
        tab[4 * i] = w;
        tab[4 * i + 1] = w * d.s[3 * i];
        tab[4 * i + 2] = w * d.s[3 * i + 1];
        tab[4 * i + 3] = w * d.s[3 * i + 2];
    }
    __syncthreads();
    const int c = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (c >= d.nc) return;
    const int lane = threadIdx.x & 63;
    double acc[kMomN] = {0, 0, 0, 0, 0};
    if ((d.code[c] & kSolidBit) && lane < nL) {
        const double g = d.gamma[c];
        const double dp = dpend ? dpend[c] : 0.0;
        const int k0 = kV * lane, step = kV * nL;   // step: a multiple of nl
        const int b0 = k0 % nl, dA = step / nl;
        int a = k0 / nl;
        double it[kV], vb[kV], c4[kV];
        const int mo = d.nmat > 1 ? d.film[d.fid[c]].moff : 0;   // the cell's material
#pragma unroll
        for (int u = 0; u < kV; ++u) {
            it[u] = d.itau[mo + b0 + u];
            vb[u] = d.v[mo + b0 + u];
            c4[u] = d.C4[mo + b0 + u] * dp;   // pending correction of value u
        }
        const T *row = e + (size_t)c * nk;
        auto load = [&](int kb, T (&v)[kV]) {
            if constexpr (kV == 4) {
                const float4 q = *reinterpret_cast<const float4 *>(row + kb);
                v[0] = q.x;
                v[1] = q.y;
                v[2] = q.z;
                v[3] = q.w;
            } else {
                const double2 q = *reinterpret_cast<const double2 *>(row + kb);
                v[0] = q.x;
                v[1] = q.y;
            }
        };
        auto accumulate = [&](const T (&v)[kV], int aa) {
            double X = 0.0, Y = 0.0, V = 0.0;
#pragma unroll
            for (int u = 0; u < kV; ++u) {
                const double x = (double)v[u] + c4[u];
                X += x;
                Y += it[u] * x;
                V += vb[u] * x;
            }
            const double *t = tab + 4 * aa;
            acc[0] += t[0] * X;
            acc[1] += t[0] * Y;
            acc[2] += t[1] * V;
            acc[3] += t[2] * V;
            acc[4] += t[3] * V;
        };
        // two vector loads in flight per lane (the second clamped to the
        // row's last vector when past its end, and then not accumulated)
        for (int kb = k0; kb < nk; kb += 2 * step) {
            const int kb2 = kb + step < nk ? kb + step : nk - kV;
            T v0[kV], v1[kV];
            load(kb, v0);
            load(kb2, v1);
            accumulate(v0, a);
            if (kb + step < nk) accumulate(v1, a + dA);
            a += 2 * dA;
        }
        acc[1] += g * acc[0];
    }
#pragma unroll
    for (int m = 0; m < kMomN; ++m)
        for (int off = 32; off > 0; off >>= 1) acc[m] += __shfl_xor(acc[m], off, 64);
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < kMomN; ++m) part[(size_t)c * kMomN + m] = acc[m];
}

// General form: one block per cell.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments_block(Dev d, const T *__restrict__ e,
                                                          const double *__restrict__ dpend, double *__restrict__ part)
{
    __shared__ double sh[4 * kMomN];
    const int c = blockIdx.x;
    double acc[kMomN] = {0, 0, 0, 0, 0};
    if (d.code[c] & kSolidBit) {
        const double g = d.gamma[c];
        const double dp = dpend ? dpend[c] : 0.0;
        const int mo = d.nmat > 1 ? d.film[d.fid[c]].moff : 0;
        for (int k = threadIdx.x; k < d.nk; k += kBlock) {
            const LaneConst L = lane_const(d, k, mo);
            const double x = (double)e[(size_t)c * d.nk + k] + L.C4 * dp;
            const double wx = L.w * x;
            acc[0] += wx;
            acc[1] += wx * (L.itau + g);
            const double vw = wx * L.v;
            acc[2] += vw * L.s[0];
            acc[3] += vw * L.s[1];
            acc[4] += vw * L.s[2];
        }
    }
    block_sum<kMomN>(acc, sh);
    if (threadIdx.x == 0)
        for (int i = 0; i < kMomN; ++i) part[(size_t)c * kMomN + i] = acc[i];
}

// Sum np partials per cell -> T, T_L (absolute), q, T_L deviation, |q|.
__global__ void k_finalize(Dev d, const double *__restrict__ part, int np, double Tref, double *T, double *TL,
                           double *q, double *TLdev, double *Tdev, double *qmag)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    double s[kMomN] = {0, 0, 0, 0, 0};
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < kMomN; ++i) s[i] += part[((size_t)p * d.nc + c) * kMomN + i];
    const bool solid = d.code[c] & kSolidBit;
    const double td = solid ? s[0] / d.film[d.fid[c]].Ctot : 0.0;
    const double tl = solid ? s[1] / d.S[c] : 0.0;
    if (T) T[c] = Tref + td;
    if (TL) TL[c] = Tref + tl;
    if (q)
        for (int a = 0; a < 3; ++a) q[3 * c + a] = solid ? s[2 + a] : 0.0;
    if (TLdev) TLdev[c] = tl;
    if (Tdev) Tdev[c] = td;
    if (qmag) qmag[c] = solid ? sqrt(s[2] * s[2] + s[3] * s[3] + s[4] * s[4]) : 0.0;
}

// T_L deviation from per-octant (or per (octant, chunk)) partials of
// sum w e/tau (transient step).  64 cells per block: wavefront w sums the
// partials p = w mod 4 (four independent load chains per cell instead of
// one), then the four sums are added in a fixed order.
__global__ __launch_bounds__(kBlock) void k_finalize_tl(Dev d, const double *__restrict__ part, int np,
                                                        double *__restrict__ TLdev)
{
    __shared__ double sh[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    double s = 0;
    if (c < d.nc)
        for (int p = w; p < np; p += 4) s += part[(size_t)p * d.nc + c];
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && c < d.nc) {
        const double t = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
        TLdev[c] = (d.code[c] & kSolidBit) ? t / d.S[c] : 0.0;
    }
}

// ---------------------------------------------------------------- diffuse walls

// Incoming value of each wall record.  Diffuse wall (Sec. 2.2 (iii), eq.
// diff_bound, with the discrete normalisation): sum_{s.n>0} w s.n e_face /
// sum_{s.n<0} w |s.n|.  Interface (Sec. 2.2 (v)) between the record's cell
// (material A) and the cell across the face (material B):
// [beta_BA (v_B / v_A) F_B + (1 - beta_AB) F_A] / sum_{s.n<0} w |s.n|, with
// F_X the outgoing sum_{s.n>0} w |s.n| e_face of side X; the fractions act
// on energy fluxes, hence the speed ratio.  Face values: the cell value plus
// the one-sided slope toward the face (unlimited scheme only).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_walls(Dev d, const T *__restrict__ e, const double *__restrict__ dpend,
                                                   const int *__restrict__ wrec, const double *__restrict__ wden,
                                                   double *__restrict__ din, int nw)
{
    __shared__ double sh[2][kBlock];
    const int r = blockIdx.x;
    if (r >= nw) return;
    const int c = wrec[2 * r], f = wrec[2 * r + 1];
    const int a = f >> 1, side = (f & 1) ? 1 : -1;
    const Film &fm = d.film[d.fid[c]];
    const int jp = d.wpart[r];   // the cell across an interface, -1 for a diffuse wall
    const Film &fp = d.film[d.fid[jp >= 0 ? jp : c]];
    const int G = kBlock / d.nl;     // groups of n_bands threads (n_bands <= 256)
    const int grp = threadIdx.x / d.nl, l = threadIdx.x - grp * d.nl;
    // the outgoing face value of cell x through its face on side sx, for lane k
    auto face_out = [&](const Film &fx, int x, int sx, int k, T C4) -> T {
        const uint32_t ab = axis_bits(d.code[x], a);
        const bool hb = side_is_cell(ab, -sx);
        const T ex = ld_e(e, dpend, d, x, k, C4);
        if (d.limiter != LIM_NONE || !hb) return ex;
        const int jb = d.nb[face_of(a, -sx) * d.nc + x];
        const T J = C4 * (T)fx.pdT[a];
        const T jump = side_wraps(ab, -sx) ? (T)sx * J : (T)0;
        return ex + (T)(0.5 * fx.h[a]) * ((ex - (ld_e(e, dpend, d, jb, k, C4) + jump)) * (T)fx.ih[a]);
    };
    double sum = 0.0, sumb = 0.0;
    if (grp < G) {
        const T C4 = (T)d.C4[fm.moff + l], C4p = (T)d.C4[fp.moff + l];
        for (int al = grp; al < d.na; al += G) {
            const double sa = d.s[3 * al + a];
            const int k = al * d.nl + l;
            if (sa * side > 0.0) sum += d.w[al] * fabs(sa) * (double)face_out(fm, c, side, k, C4);
            else if (jp >= 0 && sa * side < 0.0) sumb += d.w[al] * fabs(sa) * (double)face_out(fp, jp, -side, k, C4p);
        }
    }
    sh[0][threadIdx.x] = sum;
    sh[1][threadIdx.x] = sumb;
    __syncthreads();
    if (threadIdx.x < d.nl) {
        double t = 0.0, tb = 0.0;
        for (int g2 = 0; g2 < G; ++g2) {
            t += sh[0][g2 * d.nl + threadIdx.x];
            tb += sh[1][g2 * d.nl + threadIdx.x];
        }
        double v = t;
        if (jp >= 0) {
            const double *bt = d.wbeta + 2 * (size_t)r * d.nl;
            const double ratio = d.v[fp.moff + threadIdx.x] / d.v[fm.moff + threadIdx.x];
            v = bt[threadIdx.x] * ratio * tb + (1.0 - bt[d.nl + threadIdx.x]) * t;
        }
        din[(size_t)r * d.nl + threadIdx.x] = v / wden[f];
    }
}

// Steady residual R(e) with e0 from TLdev (right-hand side of eq. B_BTE).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(Dev d, const T *__restrict__ e, T *__restrict__ R,
                                                      const double *__restrict__ TLdev, const double *__restrict__ din,
                                                      int nchunk, int ngroup, int cpb)
{
    const int lb = xcd_logical_block();
    const int chunk = lb / ngroup, grp = lb - chunk * ngroup;
    if (chunk >= nchunk) return;
    const int k = chunk * kBlock + threadIdx.x;
    if (k >= d.nk) return;
    const LaneConst L0 = lane_const(d, k, 0);
    for (int ci = 0; ci < cpb; ++ci) {
        const int c = grp * cpb + ci;
        if (c >= d.nc) break;
        const uint32_t code = d.code[c];
        if (!(code & kSolidBit)) {
            R[(size_t)c * d.nk + k] = (T)0;
            continue;
        }
        const Film &fm = d.film[d.fid[c]];
        const LaneConst L = d.nmat > 1 ? lane_const(d, k, fm.moff) : L0;
        const double itc = L.itau + d.gamma[c];
        const double qsrc = d.P ? d.P[c] / fm.Ctot : 0.0;
        const T ec = e[(size_t)c * d.nk + k];
        const StencilOut<T> so = stencil<T>(e, nullptr, din, d, fm, c, code, L, ec);
        const T e0 = (T)(L.C4 * TLdev[c]);
        R[(size_t)c * d.nk + k] = -so.D - (ec - e0) * (T)itc + (T)(L.C4 * qsrc);
    }
}

// -------------------------------------------------------------- cell kernels

// e = C (T - T_ref)/4pi for every direction (pores: 0)
template <typename T>
__global__ void k_set_equilibrium(Dev d, T *__restrict__ e, const double *__restrict__ Tdev)
{
    const size_t n = (size_t)d.nc * d.nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / d.nk), k = (int)(i - (size_t)c * d.nk);
        const int l = k % d.nl + (d.nmat > 1 ? d.film[d.fid[c]].moff : 0);
        e[i] = (d.code[c] & kSolidBit) ? (T)(d.C4[l] * Tdev[c]) : (T)0;
    }
}

// out = in + C (dpend_c - shift_film)/4pi   (final correction and gauge)
template <typename T>
__global__ void k_apply_shift(Dev d, const T *__restrict__ in, T *__restrict__ out, const double *__restrict__ dpend,
                              const double *__restrict__ fshift)
{
    const size_t n = (size_t)d.nc * d.nk;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / d.nk), k = (int)(i - (size_t)c * d.nk);
        const int l = k % d.nl + (d.nmat > 1 ? d.film[d.fid[c]].moff : 0);
        double sft = (dpend ? dpend[c] : 0.0) - (fshift ? fshift[d.fid[c]] : 0.0);
        out[i] = (d.code[c] & kSolidBit) ? (T)((double)in[i] + d.C4[l] * sft) : in[i];
    }
}

// Steady bookkeeping after a sweep: moments of e^{n+1} (T_L^kin, T, |q|),
// the synthetic defect r = S (T_L^kin - T_L^n) and the squared changes.
__global__ void k_steady_post(Dev d, const double *__restrict__ part, int np, const double *__restrict__ TLn,
                              double *__restrict__ TLkin, double *__restrict__ Tnew, double *__restrict__ qnew,
                              double *__restrict__ r, int synthetic)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    double s[kMomN] = {0, 0, 0, 0, 0};
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < kMomN; ++i) s[i] += part[((size_t)p * d.nc + c) * kMomN + i];
    const bool solid = d.code[c] & kSolidBit;
    const double tl = solid ? s[1] / d.S[c] : 0.0;
    TLkin[c] = tl;
    Tnew[c] = solid ? s[0] / d.film[d.fid[c]].Ctot : 0.0;
    qnew[c] = solid ? sqrt(s[2] * s[2] + s[3] * s[3] + s[4] * s[4]) : 0.0;
    // a converged geometry gets no further correction
    if (synthetic) r[c] = (solid && !d.fdone[d.fid[c]]) ? d.S[c] * (tl - TLn[c]) : 0.0;
}

// Per-geometry convergence measures (Sec. 3.4), in two stages: blocks of
// kFilmSeg cells of a geometry write partials, then one wavefront per
// geometry combines them in a fixed order.
// out[f] = {sum dT^2, max|T-Tref|, sum d|q|^2, max|q|, sum (T-Tref)}.
constexpr int kFilmSeg = 2048;

__global__ __launch_bounds__(kBlock) void k_film_eps_part(Dev d, const double *__restrict__ T0,
                                                           const double *__restrict__ T1,
                                                           const double *__restrict__ q0,
                                                           const double *__restrict__ q1, double *__restrict__ part)
{
    __shared__ double sh[4 * 5];
    __shared__ double shm[8];
    const int f = blockIdx.y, sgm = blockIdx.x;
    const Film &fm = d.film[f];
    const int i0 = sgm * kFilmSeg, i1 = min(fm.ncell, i0 + kFilmSeg);
    double a[5] = {0, 0, 0, 0, 0};
    double mT = 0, mq = 0;
    // branch-free body (pores contribute zeros) so that the loads of
    // consecutive iterations overlap
#pragma unroll 4
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int c = fm.cell0 + i;
        const double sl = (d.code[c] & kSolidBit) ? 1.0 : 0.0;
        const double t1 = T1[c], u1 = q1[c];
        const double dT = (T0[c] - t1) * sl, dq = (q0[c] - u1) * sl;
        a[0] += dT * dT;
        a[2] += dq * dq;
        a[4] += t1 * sl;
        mT = fmax(mT, fabs(t1) * sl);
        mq = fmax(mq, fabs(u1) * sl);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mT = fmax(mT, __shfl_xor(mT, off, 64));
        mq = fmax(mq, __shfl_xor(mq, off, 64));
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        shm[wave] = mT;
        shm[4 + wave] = mq;
    }
    block_sum<5>(a, sh);
    if (threadIdx.x == 0) {
        double *o = part + 5 * ((size_t)f * gridDim.x + sgm);
        o[0] = a[0];
        o[1] = fmax(fmax(shm[0], shm[1]), fmax(shm[2], shm[3]));
        o[2] = a[2];
        o[3] = fmax(fmax(shm[4], shm[5]), fmax(shm[6], shm[7]));
        o[4] = a[4];
    }
}

__global__ __launch_bounds__(64) void k_film_eps_fin(const double *__restrict__ part, int nseg,
                                                     double *__restrict__ out)
{
    const int f = blockIdx.x, lane = threadIdx.x;
    double a[5] = {0, 0, 0, 0, 0};
    for (int s = lane; s < nseg; s += 64) {
        const double *p = part + 5 * ((size_t)f * nseg + s);
        a[0] += p[0];
        a[1] = fmax(a[1], p[1]);
        a[2] += p[2];
        a[3] = fmax(a[3], p[3]);
        a[4] += p[4];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a[0] += __shfl_xor(a[0], off, 64);
        a[1] = fmax(a[1], __shfl_xor(a[1], off, 64));
        a[2] += __shfl_xor(a[2], off, 64);
        a[3] = fmax(a[3], __shfl_xor(a[3], off, 64));
        a[4] += __shfl_xor(a[4], off, 64);
    }
    if (lane == 0)
        for (int i = 0; i < 5; ++i) out[5 * f + i] = a[i];
}

// Per-geometry mean over solid cells of x, in the same two stages.
__global__ __launch_bounds__(kBlock) void k_film_mean_part(Dev d, const double *__restrict__ x,
                                                            double *__restrict__ part)
{
    __shared__ double sh[4];
    const int f = blockIdx.y, sgm = blockIdx.x;
    const Film &fm = d.film[f];
    const int i0 = sgm * kFilmSeg, i1 = min(fm.ncell, i0 + kFilmSeg);
    double a[1] = {0};
#pragma unroll 4
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int c = fm.cell0 + i;
        a[0] += (d.code[c] & kSolidBit) ? x[c] : 0.0;
    }
    block_sum<1>(a, sh);
    if (threadIdx.x == 0) part[(size_t)f * gridDim.x + sgm] = a[0];
}

__global__ __launch_bounds__(64) void k_film_mean_fin(Dev d, const double *__restrict__ part, int nseg,
                                                      double *__restrict__ mean)
{
    const int f = blockIdx.x, lane = threadIdx.x;
    double a = 0;
    for (int s = lane; s < nseg; s += 64) a += part[(size_t)f * nseg + s];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) mean[f] = a / d.film[f].nsolid;
}

// x -= mean of its geometry, only for floating geometries (no thermalizing wall)
__global__ void k_sub_film_mean(Dev d, double *__restrict__ x, const double *__restrict__ mean)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const int f = d.fid[c];
    if (d.film[f].floating && (d.code[c] & kSolidBit)) x[c] -= mean[f];
}

// T_L^{n+1} = T_L^kin + delta, pending correction = delta (cells of
// converged geometries keep both, when fid / fdone are given)
__global__ void k_tl_update(int n, const double *__restrict__ TLkin, const double *__restrict__ delta,
                            double *__restrict__ TL, double *__restrict__ dpend, const int *__restrict__ fid,
                            const int *__restrict__ fdone)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (fdone && fdone[fid[c]]) return;
    const double dl = delta ? delta[c] : 0.0;
    TL[c] = TLkin[c] + dl;
    if (dpend) dpend[c] = dl;
}

// ------------------------------------------------------------------- CG
//
// Finite-volume diffusion operator -div(k grad x) per unit volume: harmonic
// face conductivity, thermalizing walls through a wall conductance, other
// walls zero flux, periodic faces wrap.  Used for the heat-diffusion initial
// guess (Sec. 3.5, eq. diff) and, with the correction conductivities, for the
// synthetic correction.  Jacobi-preconditioned CG; the scalars live on the
// device, the host only polls a convergence flag every few iterations.

__device__ inline double wall_cond(const Dev &d, const CgArgs &g, int c, int a, const Film &fm)
{
    const double kd = 2.0 * g.kax[a * d.nc + c] * fm.ih[a];
    if (!g.corr) return kd;
    return 1.0 / (1.0 / kd + 1.0 / fm.Hm[a]);
}

// Face couplings and diagonal of the diffusion operator per unit volume:
// harmonic-mean face conductivity k_f / h^2 between solid neighbours (periodic
// faces wrap), a thermalizing wall adds its conductance / h to the diagonal,
// other walls nothing.
__global__ void k_cg_coef(Dev d, CgArgs g, double *coef, double *dgo)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const uint32_t code = d.code[c];
    for (int f = 0; f < 6; ++f) coef[f * d.nc + c] = 0.0;
    double diag = 0.0;
    if (code & kSolidBit) {
        const Film &fm = d.film[d.fid[c]];
        for (int a = 0; a < d.dim; ++a) {
            const double ih2 = fm.ih[a] * fm.ih[a];
            const double ki = g.kax[a * d.nc + c];
            const uint32_t ab = axis_bits(code, a);
            for (int side = -1; side <= 1; side += 2) {
                if (side_is_cell(ab, side)) {
                    const int j = d.nb[face_of(a, side) * d.nc + c];
                    const double kj = g.kax[a * d.nc + j];
                    const double kf = 2.0 * ki * kj / (ki + kj) * ih2;
                    coef[face_of(a, side) * d.nc + c] = kf;
                    diag += kf;
                } else if (side_wall(ab, side) == kWallInterface) {
                    // the half cells in series with the interface conductance
                    const double G = fm.gif[face_of(a, side)];
                    if (G > 0.0) {
                        const int j = d.nb[face_of(a, side) * d.nc + c];
                        const double kj = g.kax[a * d.nc + j];
                        const double kf = fm.ih[a] / (0.5 * fm.h[a] / ki + 1.0 / G + 0.5 * fm.h[a] / kj);
                        coef[face_of(a, side) * d.nc + c] = kf;
                        diag += kf;
                    }
                } else if (side_wall(ab, side) == 0) {
                    diag += wall_cond(d, g, c, a, fm) * fm.ih[a];
                }
            }
        }
    }
    dgo[c] = (code & kSolidBit) && diag > 0 ? diag : 1.0;
}

// ---- CG with one ordinary launch per iteration (Chronopoulos-Gear form of
// Jacobi-preconditioned CG: the two inner products of an iteration come from
// one reduction).  With u = r / diag, w = A u and s = A p:
//   p_i = u_i + beta_i p_(i-1),  s_i = w_i + beta_i s_(i-1),
//   x += alpha_i p_i,  r_(i+1) = r_i - alpha_i s_i,  w_(i+1) = A u_(i+1),
//   gamma = r.u, delta = w.u (and r.r for the stopping test) of step i + 1,
//   beta_(i+1) = gamma_(i+1) / gamma_i,
//   alpha_(i+1) = gamma_(i+1) / (delta_(i+1) - beta_(i+1) gamma_(i+1) / alpha_i).
// A u_(i+1) needs u_(i+1) at the neighbours: it is recomputed there from
// r_i, w_i and s_(i-1), so r, w and s alternate between two buffers by
// iteration parity.  The launch boundary is the grid-wide barrier (far
// cheaper than a cooperative grid barrier on this part); every block reduces
// the block partials of the previous launch itself, in the same fixed order,
// so all blocks take the same decisions.
// scal: [1] |b|^2, [5] done, [6] iterations of this solve, [9] iterations
// accumulated, [10 + parity] gamma, [12 + parity] alpha.
__device__ inline void part_sum3(const double *__restrict__ part, int n, double *sh, double &a, double &b, double &c)
{
    double v[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < n; i += kBlock) {
        v[0] += part[3 * i];
        v[1] += part[3 * i + 1];
        v[2] += part[3 * i + 2];
    }
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        sh[0] = v[0];
        sh[1] = v[1];
        sh[2] = v[2];
    }
    __syncthreads();
    a = sh[0];
    b = sh[1];
    c = sh[2];
    __syncthreads();
}

__device__ inline void write_part3(double *part, double a, double b, double c, double *sh)
{
    double v[3] = {a, b, c};
    block_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

// x = 0, p = 0, s_(-1) = 0, r_0 = b (solid cells), w_0 = A (r_0 / diag);
// partials (gamma, delta, r.r) of step 0
__global__ __launch_bounds__(kBlock) void k_cg_start(Dev d, CgArgs g, const double *__restrict__ b)
{
    __shared__ double sh[32];
    const int nthr = gridDim.x * kBlock, nf = 2 * d.dim;
    double ga = 0, de = 0, rr = 0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < d.nc; c += nthr) {
        const double dg = g.dg[c];
        const double rc = (d.code[c] & kSolidBit) ? b[c] : 0.0;
        const double uc = rc / dg;
        double acc = dg * uc;
        for (int f = 0; f < nf; ++f) {
            const double cf = g.coef[f * d.nc + c];
            const int j = cf != 0.0 ? d.nb[f * d.nc + c] : c;   // coupled faces join solid cells
            acc -= cf * (b[j] / g.dg[j]);
        }
        g.x[c] = 0.0;
        g.p[c] = 0.0;
        g.rb[0][c] = rc;
        g.wb[0][c] = acc;
        g.sb[1][c] = 0.0;
        ga += rc * uc;
        de += acc * uc;
        rr += rc * rc;
    }
    write_part3(g.part, ga, de, rr, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.scal[5] = 0.0;
        g.scal[6] = 0.0;
    }
}

// step it: scalars from the partials of the previous launch, stopping test,
// then the vector updates of step it and the partials of step it + 1
// Everything one cell of k_cg_iter reads: none of it depends on the
// scalars of the step, so the first cell's loads are issued before the
// reduction of the previous launch's partials.
struct CgCell {
    double dg, R, W, S, p, x;
    double cf[6], Rj[6], Wj[6], Sj[6], dgj[6];
};

__device__ inline void cg_cell_load(const Dev &d, const CgArgs &g, const double *__restrict__ R,
                                    const double *__restrict__ W, const double *__restrict__ S, int c, CgCell &q)
{
    q.dg = g.dg[c];
    q.R = R[c];
    q.W = W[c];
    q.S = S[c];
    q.p = g.p[c];
    q.x = g.x[c];
    int j[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {   // unused faces have a zero coupling: they read the cell itself
        q.cf[f] = g.coef[f * d.nc + c];
        j[f] = q.cf[f] != 0.0 ? d.nb[f * d.nc + c] : c;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        q.Rj[f] = R[j[f]];
        q.Wj[f] = W[j[f]];
        q.Sj[f] = S[j[f]];
        q.dgj[f] = g.dg[j[f]];
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_iter(Dev d, CgArgs g, int it)
{
    __shared__ double sh[32];
    const int nb = gridDim.x, nthr = nb * kBlock;
    const int cur = it & 1, nxt = cur ^ 1;
    // the solve's flag and scalars are loaded together with the first
    // cell's values; the flag is tested once the partials are reduced (a
    // finished solve's launches then return without writing)
    const double done = g.scal[5], bn2s = g.scal[1], gprev = g.scal[10 + nxt], aprev = g.scal[12 + nxt];
    const double *__restrict__ R = g.rb[cur];
    const double *__restrict__ W = g.wb[cur];
    const double *__restrict__ S = g.sb[nxt];   // s_(it-1)
    double *__restrict__ RN = g.rb[nxt];
    double *__restrict__ WN = g.wb[nxt];
    double *__restrict__ SN = g.sb[cur];        // s_it
    const int c0 = blockIdx.x * kBlock + threadIdx.x;
    CgCell q;
    cg_cell_load(d, g, R, W, S, c0 < d.nc ? c0 : 0, q);
    double ga, de, rr;
    part_sum3(g.part + 3 * nb * cur, nb, sh, ga, de, rr);
    if (done != 0.0) return;
    const double bn2 = it == 0 ? rr : bn2s;
    double alpha = 0.0, beta = 0.0;
    bool stop = !(rr > g.rtol2 * bn2) || !(ga > 0.0);
    if (!stop) {
        if (it == 0) {
            alpha = ga / de;
        } else {
            beta = ga / gprev;
            alpha = ga / (de - beta * ga / aprev);
        }
        stop = !(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta);
    }
    if (stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (it == 0) g.scal[1] = bn2;
            g.scal[5] = 1.0;
        }
        return;
    }
    double gn = 0, dn = 0, rn2 = 0;
    for (int c = c0; c < d.nc; c += nthr) {
        if (c != c0) cg_cell_load(d, g, R, W, S, c, q);
        const double uc = q.R / q.dg;
        const double pc = uc + beta * q.p;
        const double sc = q.W + beta * q.S;
        g.p[c] = pc;
        SN[c] = sc;
        g.x[c] = q.x + alpha * pc;
        const double rc = q.R - alpha * sc;
        RN[c] = rc;
        const double un = rc / q.dg;
        double acc = q.dg * un;
#pragma unroll
        for (int f = 0; f < 6; ++f) acc -= q.cf[f] * ((q.Rj[f] - alpha * (q.Wj[f] + beta * q.Sj[f])) / q.dgj[f]);
        WN[c] = acc;
        gn += rc * un;
        dn += acc * un;
        rn2 += rc * rc;
    }
    write_part3(g.part + 3 * nb * nxt, gn, dn, rn2, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (it == 0) g.scal[1] = bn2;
        g.scal[10 + cur] = ga;
        g.scal[12 + cur] = alpha;
        g.scal[6] = it + 1;
        g.scal[9] += 1.0;
    }
}

int cg_blocks(const Dev &d) { return std::max(1, std::min(1024, (d.nc + kBlock - 1) / kBlock)); }

void launch_cg_begin(const Dev &d, const CgArgs &g, const double *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_start, dim3(cg_blocks(d)), dim3(kBlock), 0, s, d, g, b);
}

void launch_cg_iters(const Dev &d, const CgArgs &g, int it0, int n, hipStream_t s)
{
    const int nb = cg_blocks(d);
    for (int it = it0; it < it0 + n; ++it) hipLaunchKernelGGL(k_cg_iter, dim3(nb), dim3(kBlock), 0, s, d, g, it);
}

// right-hand side of the heat-diffusion initial guess: P plus thermalizing
// wall and periodic-jump terms
__global__ void k_diff_rhs(Dev d, CgArgs g, double *__restrict__ b)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const uint32_t code = d.code[c];
    if (!(code & kSolidBit)) {
        b[c] = 0.0;
        return;
    }
    const Film &fm = d.film[d.fid[c]];
    double acc = d.P ? d.P[c] : 0.0;
    for (int a = 0; a < d.dim; ++a) {
        const double ih2 = fm.ih[a] * fm.ih[a];
        const double ki = g.kax[a * d.nc + c];
        const uint32_t ab = axis_bits(code, a);
        for (int side = -1; side <= 1; side += 2) {
            if (side_is_cell(ab, side)) {
                if (side_wraps(ab, side)) {
                    const int j = d.nb[face_of(a, side) * d.nc + c];
                    const double kj = g.kax[a * d.nc + j];
                    acc += 2.0 * ki * kj / (ki + kj) * ih2 * (-side) * fm.pdT[a];
                }
            } else if (side_wall(ab, side) == 0) {
                const double Tw = side_outer(code, a, side) ? fm.wallT[face_of(a, side)] : d.poreT;
                acc += wall_cond(d, g, c, a, fm) * fm.ih[a] * Tw;
            }
        }
    }
    b[c] = acc;
}

// k_eff per geometry: (L_x/dT) (1/N_cells) sum_solid q_x  (one block per geometry)
__global__ __launch_bounds__(kBlock) void k_keff(Dev d, const double *__restrict__ q, double *__restrict__ keff)
{
    __shared__ double sh[4];
    const Film &fm = d.film[blockIdx.x];
    double a[1] = {0};
    for (int i = threadIdx.x; i < fm.ncell; i += kBlock) a[0] += q[3 * (fm.cell0 + i)];
    block_sum<1>(a, sh);
    if (threadIdx.x == 0) keff[blockIdx.x] = fm.len[0] / fm.pdT[0] * a[0] / fm.ncell;
}

// ---------------------------------------------------------------- launchers

template <typename T>
void launch_moments(const Dev &d, const T *e, const double *dpend, double *part, hipStream_t s)
{
    constexpr int kV = 16 / (int)sizeof(T);
    const size_t tab = 8 * (4 * (size_t)d.na + 3 * (size_t)d.nl * d.nmat);
    const bool aligned = d.nk % kV == 0 && (reinterpret_cast<uintptr_t>(e) & 15) == 0;
    // lanes per step of the band-factored form: at most 64, kV nL a multiple of nl
    int nL = 0;
    if (d.nl % kV == 0)
        for (int l = 64; l >= 1 && !nL; --l)
            if ((kV * l) % d.nl == 0) nL = l;
    if (aligned && nL >= 32 && 8 * 4 * (size_t)d.na <= 48 * 1024)
        hipLaunchKernelGGL(k_moments_band<T>, dim3((d.nc + 3) / 4), dim3(256), 8 * 4 * (size_t)d.na, s, d, e, dpend,
                           part, nL);
    else if (aligned && tab <= 48 * 1024)
        hipLaunchKernelGGL(k_moments_wave<T>, dim3((d.nc + 3) / 4), dim3(256), tab, s, d, e, dpend, part);
    else
        hipLaunchKernelGGL(k_moments_block<T>, dim3(d.nc), dim3(kBlock), 0, s, d, e, dpend, part);
}

template <typename T>
void launch_walls(const Dev &d, const T *e, const double *dpend, const int *wrec, const double *wden, double *din,
                  int nw, hipStream_t s)
{
    if (nw > 0) hipLaunchKernelGGL(k_walls<T>, dim3(nw), dim3(kBlock), 0, s, d, e, dpend, wrec, wden, din, nw);
}

static inline void stream_grid(const Dev &d, int cpb, int &nchunk, int &ngroup, int &grid)
{
    nchunk = (d.nk + kBlock - 1) / kBlock;
    ngroup = (d.nc + cpb - 1) / cpb;
    grid = nchunk * ngroup;
    grid = (grid + 7) / 8 * 8;
}

template <typename T>
void launch_residual(const Dev &d, const T *e, T *R, const double *TLdev, const double *din, int cpb, hipStream_t s)
{
    int nchunk, ngroup, grid;
    stream_grid(d, cpb, nchunk, ngroup, grid);
    hipLaunchKernelGGL(k_residual<T>, dim3(grid), dim3(kBlock), 0, s, d, e, R, TLdev, din, nchunk, ngroup, cpb);
}

template <typename T>
void launch_set_equilibrium(const Dev &d, T *e, const double *Tdev, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_equilibrium<T>, dim3(2048), dim3(kBlock), 0, s, d, e, Tdev);
}

template <typename T>
void launch_apply_shift(const Dev &d, const T *in, T *out, const double *dpend, const double *fshift, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply_shift<T>, dim3(2048), dim3(kBlock), 0, s, d, in, out, dpend, fshift);
}

void launch_keff(const Dev &d, const double *q, double *keff, hipStream_t s)
{
    hipLaunchKernelGGL(k_keff, dim3(d.nfilm), dim3(kBlock), 0, s, d, q, keff);
}

#define BTE_INST(T)                                                                                                   \
    template void launch_moments<T>(const Dev &, const T *, const double *, double *, hipStream_t);                  \
    template void launch_walls<T>(const Dev &, const T *, const double *, const int *, const double *, double *,     \
                                  int, hipStream_t);                                                                 \
    template void launch_residual<T>(const Dev &, const T *, T *, const double *, const double *, int, hipStream_t); \
    template void launch_set_equilibrium<T>(const Dev &, T *, const double *, hipStream_t);                          \
    template void launch_apply_shift<T>(const Dev &, const T *, T *, const double *, const double *, hipStream_t);
BTE_INST(float)
BTE_INST(double)

void launch_cell_setup(const Dev &d, double *S, double *kdif, double *kcor, const double M[3], const double H[3],
                       hipStream_t s)
{
    const int grid = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_cell_setup, dim3(grid), dim3(kBlock), 0, s, d, S, kdif, kcor, M[0], M[1], M[2], H[0], H[1],
                       H[2]);
}

void launch_finalize(const Dev &d, const double *part, int np, double Tref, double *T, double *TL, double *q,
                     double *TLdev, double *Tdev, double *qmag, hipStream_t s)
{
    const int grid = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kBlock), 0, s, d, part, np, Tref, T, TL, q, TLdev, Tdev, qmag);
}

void launch_finalize_tl(const Dev &d, const double *part, int np, double *TLdev, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_tl, dim3((d.nc + 63) / 64), dim3(kBlock), 0, s, d, part, np, TLdev);
}

void launch_steady_post(const Dev &d, const double *part, int np, const double *TLn, double *TLkin, double *Tnew,
                        double *qnew, double *r, int synthetic, hipStream_t s)
{
    const int grid = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_steady_post, dim3(grid), dim3(kBlock), 0, s, d, part, np, TLn, TLkin, Tnew, qnew, r,
                       synthetic);
}

int film_segments(int max_cells) { return std::max(1, (max_cells + kFilmSeg - 1) / kFilmSeg); }

// part: scratch of 5 * nfilm * nseg doubles, nseg = film_segments(largest geometry)
void launch_film_eps(const Dev &d, const double *T0, const double *T1, const double *q0, const double *q1,
                     double *out, double *part, int nseg, hipStream_t s)
{
    hipLaunchKernelGGL(k_film_eps_part, dim3(nseg, d.nfilm), dim3(kBlock), 0, s, d, T0, T1, q0, q1, part);
    hipLaunchKernelGGL(k_film_eps_fin, dim3(d.nfilm), dim3(64), 0, s, part, nseg, out);
}

void launch_film_mean(const Dev &d, const double *x, double *mean, double *part, int nseg, hipStream_t s)
{
    hipLaunchKernelGGL(k_film_mean_part, dim3(nseg, d.nfilm), dim3(kBlock), 0, s, d, x, part);
    hipLaunchKernelGGL(k_film_mean_fin, dim3(d.nfilm), dim3(64), 0, s, d, part, nseg, mean);
}

void launch_sub_film_mean(const Dev &d, double *x, const double *mean, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_film_mean, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, x, mean);
}

void launch_tl_update(int n, const double *TLkin, const double *delta, double *TL, double *dpend, const int *fid,
                      const int *fdone, hipStream_t s)
{
    hipLaunchKernelGGL(k_tl_update, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, TLkin, delta, TL, dpend,
                       fid, fdone);
}

void launch_cg_coef(const Dev &d, const CgArgs &g, double *coef, double *dg, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_coef, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, g, coef, dg);
}

void launch_diff_rhs(const Dev &d, const CgArgs &g, double *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_diff_rhs, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, g, b);
}

}  // namespace bte
