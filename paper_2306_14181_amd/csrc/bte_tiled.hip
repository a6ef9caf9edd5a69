// bte_tiled.hip -- LDS-staged transport kernels: the steady sweep (tile
// wavefronts) and the explicit transient step.  See bte_tile.h for the
// staging scheme.
//
// Per-element work is kept small: everything that depends only on the cell
// (neighbour slots, wall kind, T_L, source, scattering rate) is prepared once
// per tile in LDS and read as wavefront-uniform scalars; everything that
// depends only on the lane (direction, band) is prepared once per lane chunk.
// Interior cells take a short path (second-order upwind with the central
// least-squares slope, or the MC / minmod slopes); cells next to walls,
// pores or a domain edge take the general path.
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tile.h"
#include "bte_tilelds.h"
#include "bte_adjflux.h"

namespace bte {

// General path for one axis: slopes with missing neighbours, limiters, wall inflow.
template <typename T, int LIM>
__device__ inline T axis_general(const Dev &d, const Film &fm, const TileSmem<T> &S, int i, int a,
                                                    int m, int sd, const T *__restrict__ e,
                                                    const double *__restrict__ dpend,
                                                    const double *__restrict__ din, int al, int l, T C4, T hh, T ih,
                                                    int sg, T ec, T e1, T e2, T ed)
{
    const bool hu = m & M_HU, hu2 = m & M_HU2, hd = m & M_HD;
    const T fout = ec + hh * slope_flow<T>(LIM, hu, hd, e1, ec, ed, ih);
    T fin;
    if (hu) {
        fin = e1 + hh * slope_flow<T>(LIM, hu2, true, e2, e1, ec, ih);
    } else {
        const int kind = (m >> M_KSHIFT) & 3;
        const uint32_t code = S.code[i];
        const int c = S.cell[i];
        const int su = -sg;
        if (kind == 0) {
            const double Tw = side_outer(code, a, su) ? fm.wallT[face_of(a, su)] : d.poreT;
            fin = C4 * (T)Tw;
        } else if (kind == 1) {
            // specular: outgoing face value of the mirror direction, whose
            // upwind side is this lane's downwind side
            const int km = d.mirror[a * d.na + al] * d.nl + l;
            const T em = e[(size_t)c * d.nk + km] + C4 * (T)(dpend ? dpend[c] : 0.0);
            T gm = (T)0;
            if (LIM == LIM_NONE && hd) {
                const long long od = S.slot_off[sd];
                const T edm = e[od + km] + C4 * (T)S.slot_x[sd];
                gm = (em - edm) * ih;
            }
            fin = em + hh * gm;
        } else {
            const int rec = diffuse_index(d, c, code, face_of(a, su));
            fin = (T)din[(size_t)rec * d.nl + l];
        }
    }
    return fout - fin;
}

// Flux divergence of tile cell i for one lane.  up_out[a]: compact dup index
// of an implicitly coupled upwind neighbour outside the tile (sweep), or -1.
template <typename T, int DIM, int LIM>
__device__ inline T tile_flux(const Dev &d, const Film &fm, const TileCtx t, const TileSmem<T> &S, int i,
                              const LaneT<T> &L, int lane, const T *__restrict__ e, const double *__restrict__ dpend,
                              const double *__restrict__ din, int up_out[3])
{
    const T ec = S.box[i * 64 + lane];
    T D = (T)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int m = uni(S.mode[3 * i + a]);
        const int s1 = uni(S.stn[9 * i + 3 * a]), s2 = uni(S.stn[9 * i + 3 * a + 1]),
                  sd = uni(S.stn[9 * i + 3 * a + 2]);
        const T e1 = S.box[s1 * 64 + lane];
        const T e2 = (m & M_HU2) ? S.box[s2 * 64 + lane] : (T)0;
        const T ed = S.box[sd * 64 + lane];
        T delta;
        if ((m & (M_HU | M_HU2 | M_HD)) == (M_HU | M_HU2 | M_HD)) {
            if (LIM == LIM_NONE) {
                // e_f = e_m + (h/2) (e_{m+1} - e_{m-1}) / (2h) on both faces
                delta = (ec - e1) + (T)0.25 * ((ed - e1) - (ec - e2));
            } else {
                const T d0 = e1 - e2, d1 = ec - e1, d2 = ed - ec;
                delta = d1 + (T)0.5 * (lim_diff<T, LIM>(d1, d2) - lim_diff<T, LIM>(d0, d1));
            }
        } else {
            const int sg = a == 0 ? t.sg0 : (a == 1 ? t.sg1 : t.sg2);
            delta = axis_general<T, LIM>(d, fm, S, i, a, m, sd, e, dpend, din, L.al, L.l, L.C4, L.hh[a], L.ih[a], sg,
                                         ec, e1, e2, ed);
        }
        D += L.cpl[a] * delta;
        up_out[a] = ((m & M_HU) && !(m & M_WRAP) && s1 >= t.nt) ? S.slot_up1[s1] : -1;
    }
    return D;
}


// ----------------------------------------------------------------- sweep
//
// One work item = one tile of one geometry for 64 lanes of one octant.
//   phase A (4 wavefronts): b = R(e^n; T_L^n) for every tile cell plus the
//     increments of the already-swept upstream tiles (first-order implicit
//     coupling), into LDS;
//   phase B (wavefront 0): upwind recurrence across the tile;
//   phase C (4 wavefronts): e^{n+1} = e^n + de and FP64 moment partials.

//
// ADJ = true: the transposed sweep of the adjoint iteration.  The item's
// octant fixes the tile frame and the diagonal order; the lanes are those of
// the opposite octant (all active axes reversed), so the frame is the lanes'
// reversed flow and the recurrence solves A^T.  The right-hand side is
// (J^T psi + g) + w (1/tau) X with X the per-cell isotropic term (TLdev),
// and the moment partial is sum C/(4 pi) (1/tau) psi^{n+1} (slot 0).
template <typename T, int DIM, int LIM, bool ADJ = false>
__global__ __launch_bounds__(256) void k_sweep_tile(Dev d, const T *__restrict__ ein, T *__restrict__ eout,
                                                    const double *__restrict__ dpend,
                                                    const double *__restrict__ TLdev,
                                                    const double *__restrict__ din,
                                                    const SweepItem *__restrict__ items, int item0, int3 tdim,
                                                    int na_oct, int nchunk_oct, int cap, double *__restrict__ part)
{
    extern __shared__ __align__(16) char smem[];
    TileSmem<T> S = tile_smem<T>(smem, cap, true);
    const SweepItem it = items[item0 + blockIdx.x];
    if (!ADJ && d.nfilm > 1 && d.fdone[it.film]) return;   // converged geometry of a batch (uniform)
    const Film &fm = d.film[it.film];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int loct = ADJ ? (it.oct ^ ((1 << d.dim) - 1)) : it.oct;
    const int kbeg = loct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
    const TileCtx t = tile_make(fm, d.dim, octant_sign(d, it.oct, na_oct, 0), octant_sign(d, it.oct, na_oct, 1),
                                octant_sign(d, it.oct, na_oct, 2), it.tile, tdim);
    tile_tables<T>(t, fm, d, S, TLdev, dpend, !ADJ);
    __syncthreads();
    tile_modes<T>(t, d, S, ADJ);
    tile_load<T>(t, S, ein, k, active, L.C4, static_cast<const T *>(d.zrow), eout);
    __syncthreads();

    // lane constants of the moment partials (phase C), FP64: forward
    // w, w/tau, w v s_a; adjoint C/(4 pi) /tau, C/(4 pi)
    constexpr int NM = ADJ ? 2 : kMomN;
    double *const lc = S.mom;   // [64][NM]
    if (wave == 0) {
        double cst[kMomN];
        if constexpr (ADJ) {
            cst[0] = d.C4[L.l] * d.itau[L.l];
            cst[1] = d.C4[L.l];
        } else {
            cst[0] = L.w;
            cst[1] = L.witau;
            cst[2] = L.wv[0];
            cst[3] = L.wv[1];
            cst[4] = L.wv[2];
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) lc[lane * NM + m] = active ? cst[m] : 0.0;
    }
    T wsa[3] = {(T)0, (T)0, (T)0};
    T gl = (T)0;
    if (ADJ) {
#pragma unroll
        for (int a = 0; a < 3; ++a) wsa[a] = (T)(L.w * fabs(d.s[3 * L.al + a]));
        // objective k_eff along x: g = (L_x / (dT_x N_cells)) w v s_x
        gl = fm.pdT[0] != 0.0 ? (T)(fm.len[0] / (fm.pdT[0] * fm.ncell) * L.wv[0]) : (T)0;
    }
    for (int i = wave; i < t.nt; i += 4) {
        T b = (T)0;
        if (active && (uni(S.code[i]) & kSolidBit)) {
            int up_out[3];
            const T ec = S.box[i * 64 + lane];
            const T itc = L.itau + (T)S.gam[i];
            if constexpr (ADJ) {
                const T tf = tile_flux_adj<T, DIM>(d, t, S, i, L, wsa, lane, ein, din, up_out);
                b = tf - ec * itc + (T)L.w * itc * (T)S.tl[i] + gl;
            } else {
                const T D = tile_flux<T, DIM, LIM>(d, fm, t, S, i, L, lane, ein, dpend, din, up_out);
                b = -D - (ec - L.C4 * (T)S.tl[i]) * itc + L.C4 * (T)S.qs[i];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                if (up_out[a] >= 0) b += L.cpl[a] * S.dup[up_out[a] * 64 + lane];
        }
        S.bsh[i * 64 + lane] = b;
    }
    __syncthreads();

    if (wave == 0 && active) {
        const T cp0 = L.cpl[0], cp1 = DIM > 1 ? L.cpl[1] : (T)0, cp2 = DIM > 2 ? L.cpl[2] : (T)0;
        const T A0 = cp0 + cp1 + cp2 + L.itau;
        for (int i = 0; i < t.nt; ++i) {
            if (!(uni(S.code[i]) & kSolidBit)) continue;
            T num = S.bsh[i * 64 + lane];
            const int u0 = uni(S.upin[3 * i]), u1 = uni(S.upin[3 * i + 1]), u2 = uni(S.upin[3 * i + 2]);
            if (u0 >= 0) num += cp0 * S.bsh[u0 * 64 + lane];
            if (DIM > 1 && u1 >= 0) num += cp1 * S.bsh[u1 * 64 + lane];
            if (DIM > 2 && u2 >= 0) num += cp2 * S.bsh[u2 * 64 + lane];
            const T den = A0 + (T)S.gam[i];
            if constexpr (sizeof(T) == 4) S.bsh[i * 64 + lane] = num * __builtin_amdgcn_rcpf(den);
            else S.bsh[i * 64 + lane] = num / den;
        }
    }
    __syncthreads();

    // phase C: new values, and the moment partials of each wavefront's cells
    // (i = wave + 4 m) by a transposed reduction: 8 cells' values are staged
    // in LDS (the upwind-increment buffer, free after phase A), then lane
    // 8 j + p sums cell j over lanes 8 p .. 8 p + 7 and three data-parallel
    // moves finish the 64-lane sums.
    const int pidx = it.oct * nchunk_oct + it.chunk;
    T *const xs = S.dup + (size_t)wave * 8 * 64;
    const int nmine = (t.nt - wave + 3) / 4;
    for (int m0 = 0; m0 < nmine; m0 += 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            T xv = (T)0;
            const int m = m0 + j;
            if (m < nmine) {
                const int i = wave + 4 * m;
                const int c = uni(S.cell[i]);
                const bool solid = uni(S.code[i]) & kSolidBit;
                if (active) {
                    if (solid) {
                        const T en = S.box[i * 64 + lane] + S.bsh[i * 64 + lane];
                        eout[(size_t)c * d.nk + k] = en;
                        xv = en;
                    } else {
                        eout[(size_t)c * d.nk + k] = ein[(size_t)c * d.nk + k];
                    }
                }
            }
            xs[j * 64 + lane] = xv;
        }
        const int j = lane >> 3, p8 = lane & 7;
        double acc[NM];
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[m] = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int l2 = 8 * p8 + q;
            const double x = (double)xs[j * 64 + l2];
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] += lc[l2 * NM + m] * x;
        }
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double v = acc[m];
            v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
            v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
            v += dpp_f64<0x141>(v);   // row_half_mirror
            acc[m] = v;
        }
        // every lane of the 8-lane group j now holds cell j's total
        const int mj = m0 + j;
        if (p8 == 0 && mj < nmine) {
            const int i = wave + 4 * mj;
            const int c = S.cell[i];
            const double g = S.gam[i];
            double *o = part + ((size_t)pidx * d.nc + c) * kMomN;
            if constexpr (ADJ) {
                o[0] = acc[0] + g * acc[1];
            } else {
                o[0] = acc[0];
                o[1] = acc[1] + g * acc[0];
                o[2] = acc[2];
                o[3] = acc[3];
                o[4] = acc[4];
            }
        }
    }
}

// ------------------------------------------------------------ transient step

// Explicit step (Sec. 4.1) on a tile for every lane chunk of one octant.  The
// next step needs only the lattice temperature, so the block accumulates the
// octant's part of sum w e/tau per cell in LDS and writes it once
// (part[octant][cell]).  Items are numbered so that each XCD gets a
// contiguous run of tiles.
template <typename T, int DIM, int LIM>
__global__ __launch_bounds__(256) void k_transient_tile(Dev d, const T *__restrict__ ein, T *__restrict__ eout,
                                                        const double *__restrict__ TLdev,
                                                        const double *__restrict__ din,
                                                        const TileItem *__restrict__ items, int nitems, int3 tdim,
                                                        int na_oct, int nchunk_oct, int cap, double src, double dt,
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
    tile_tables<T>(t, fm, d, S, TLdev, nullptr);
    for (int i = threadIdx.x; i < 64; i += blockDim.x) S.mom[i] = 0.0;
    __syncthreads();
    tile_modes<T>(t, d, S);
    const int kbeg = it.oct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const T tdt = (T)dt, tsrc = (T)src;
    for (int ch = 0; ch < nchunk_oct; ++ch) {
        const int k = kbeg + ch * 64 + lane;
        const bool active = k < kend;
        const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
        tile_load<T>(t, S, ein, k, active, L.C4, static_cast<const T *>(d.zrow));
        __syncthreads();
        for (int i = wave; i < t.nt; i += 4) {
            const int c = uni(S.cell[i]);
            const bool solid = uni(S.code[i]) & kSolidBit;
            double acc[1] = {0};
            if (active) {
                if (solid) {
                    int up_out[3];
                    const T D = tile_flux<T, DIM, LIM>(d, fm, t, S, i, L, lane, ein, nullptr, din, up_out);
                    const T ec = S.box[i * 64 + lane];
                    const T itc = L.itau + (T)S.gam[i];
                    const T en = ec + tdt * (-D - (ec - L.C4 * (T)S.tl[i]) * itc + L.C4 * tsrc * (T)S.qs[i]);
                    eout[(size_t)c * d.nk + k] = en;
                    acc[0] = (L.witau + L.w * S.gam[i]) * (double)en;
                } else {
                    eout[(size_t)c * d.nk + k] = ein[(size_t)c * d.nk + k];
                }
            }
            wave_sum_t<1>(acc);
            if (lane == 0) S.mom[i] += acc[0];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < t.nt; i += blockDim.x) part[(size_t)it.oct * d.nc + S.cell[i]] = S.mom[i];
}

// --------------------------------------------------------------- launchers

// three-dimensional sweeps walk column segments (bte_sweep3d.hip); a
// segment item is a tile of 1 x 1 x tdim.z cells
template <typename T>
hipError_t launch_sweep3d(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev,
                          const double *din, const SweepItem *items, int item0, int count, int zseg, int na_oct,
                          int nchunk_oct, double *part, hipStream_t s);
template <typename T>
hipError_t launch_sweep3d_adj(const Dev &d, const T *ein, T *eout, const double *X, const double *dinA,
                              const SweepItem *items, int item0, int count, int zseg, int na_oct, int nchunk_oct,
                              double *part, hipStream_t s);

template <typename T, int DIM, int LIM>
void sweep_launch(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev, const double *din,
                  const SweepItem *items, int item0, int count, int3 tdim, int na_oct, int nchunk_oct, int cap,
                  double *part, hipStream_t s)
{
    const size_t sm = tile_smem_bytes(cap, sizeof(T), true);
    hipLaunchKernelGGL((k_sweep_tile<T, DIM, LIM>), dim3(count), dim3(256), sm, s, d, ein, eout, dpend, TLdev, din,
                       items, item0, tdim, na_oct, nchunk_oct, cap, part);
}

template <typename T>
hipError_t launch_sweep_tile(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev,
                             const double *din, const SweepItem *items, int item0, int count, int3 tdim,
                             int na_oct, int nchunk_oct, int cap, double *part, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (d.dim == 3)
        return launch_sweep3d<T>(d, ein, eout, dpend, TLdev, din, items, item0, count, tdim.z, na_oct, nchunk_oct,
                                 part, s);
#define BTE_SWEEP(DIM, LIM)                                                                                          \
    if (d.dim == DIM && d.limiter == LIM)                                                                            \
        sweep_launch<T, DIM, LIM>(d, ein, eout, dpend, TLdev, din, items, item0, count, tdim, na_oct, nchunk_oct,    \
                                  cap, part, s);
    BTE_SWEEP(1, 0) BTE_SWEEP(1, 1) BTE_SWEEP(1, 2)
    BTE_SWEEP(2, 0) BTE_SWEEP(2, 1) BTE_SWEEP(2, 2)
#undef BTE_SWEEP
    return hipGetLastError();
}

template <typename T, int DIM>
void sweep_adj_launch(const Dev &d, const T *ein, T *eout, const double *X, const double *dinA,
                      const SweepItem *items, int item0, int count, int3 tdim, int na_oct, int nchunk_oct, int cap,
                      double *part, hipStream_t s)
{
    const size_t sm = tile_smem_bytes(cap, sizeof(T), true);
    hipLaunchKernelGGL((k_sweep_tile<T, DIM, LIM_NONE, true>), dim3(count), dim3(256), sm, s, d, ein, eout, nullptr,
                       X, dinA, items, item0, tdim, na_oct, nchunk_oct, cap, part);
}

template <typename T>
hipError_t launch_sweep_adj(const Dev &d, const T *ein, T *eout, const double *X, const double *dinA,
                            const SweepItem *items, int item0, int count, int3 tdim, int na_oct, int nchunk_oct,
                            int cap, double *part, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (d.dim == 1) sweep_adj_launch<T, 1>(d, ein, eout, X, dinA, items, item0, count, tdim, na_oct, nchunk_oct, cap, part, s);
    if (d.dim == 2) sweep_adj_launch<T, 2>(d, ein, eout, X, dinA, items, item0, count, tdim, na_oct, nchunk_oct, cap, part, s);
    if (d.dim == 3)
        return launch_sweep3d_adj<T>(d, ein, eout, X, dinA, items, item0, count, tdim.z, na_oct, nchunk_oct, part, s);
    return hipGetLastError();
}

template <typename T, int DIM, int LIM>
void transient_launch(const Dev &d, const T *ein, T *eout, const double *TLdev, const double *din,
                      const TileItem *items, int nitems, int3 tdim, int na_oct, int nchunk_oct, int cap, double src,
                      double dt, double *part, hipStream_t s)
{
    const size_t sm = tile_smem_bytes(cap, sizeof(T), false);
    const int grid = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((k_transient_tile<T, DIM, LIM>), dim3(grid), dim3(256), sm, s, d, ein, eout, TLdev, din,
                       items, nitems, tdim, na_oct, nchunk_oct, cap, src, dt, part);
}

template <typename T>
hipError_t launch_transient_tile(const Dev &d, const T *ein, T *eout, const double *TLdev, const double *din,
                                 const TileItem *items, int nitems, int3 tdim, int na_oct, int nchunk_oct, int cap,
                                 double src, double dt, double *part, hipStream_t s)
{
#define BTE_TRANS(DIM, LIM)                                                                                          \
    if (d.dim == DIM && d.limiter == LIM)                                                                            \
        transient_launch<T, DIM, LIM>(d, ein, eout, TLdev, din, items, nitems, tdim, na_oct, nchunk_oct, cap, src,   \
                                      dt, part, s);
    BTE_TRANS(1, 0) BTE_TRANS(1, 1) BTE_TRANS(1, 2)
    BTE_TRANS(2, 0) BTE_TRANS(2, 1) BTE_TRANS(2, 2)
    BTE_TRANS(3, 0) BTE_TRANS(3, 1) BTE_TRANS(3, 2)
#undef BTE_TRANS
    return hipGetLastError();
}

template <typename T, int DIM, int LIM> hipError_t set_lds(size_t bytes)
{
    hipError_t a = hipSuccess, c = hipSuccess;
    if constexpr (DIM < 3) {
        a = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep_tile<T, DIM, LIM>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (LIM == LIM_NONE)
            c = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep_tile<T, DIM, LIM_NONE, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    }
    hipError_t b = hipFuncSetAttribute(reinterpret_cast<const void *>(k_transient_tile<T, DIM, LIM>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return a != hipSuccess ? a : (b != hipSuccess ? b : c);
}

// allow the dynamic LDS the tiles need (above the 64 KiB default)
hipError_t tile_kernels_init(size_t max_bytes)
{
    hipError_t e = hipSuccess, r;
#define BTE_LDS(T, DIM, LIM)                                                                                         \
    if ((r = set_lds<T, DIM, LIM>(max_bytes)) != hipSuccess) e = r;
    BTE_LDS(float, 1, 0) BTE_LDS(float, 1, 1) BTE_LDS(float, 1, 2)
    BTE_LDS(float, 2, 0) BTE_LDS(float, 2, 1) BTE_LDS(float, 2, 2)
    BTE_LDS(float, 3, 0) BTE_LDS(float, 3, 1) BTE_LDS(float, 3, 2)
    BTE_LDS(double, 1, 0) BTE_LDS(double, 1, 1) BTE_LDS(double, 1, 2)
    BTE_LDS(double, 2, 0) BTE_LDS(double, 2, 1) BTE_LDS(double, 2, 2)
    BTE_LDS(double, 3, 0) BTE_LDS(double, 3, 1) BTE_LDS(double, 3, 2)
#undef BTE_LDS
    return e;
}

size_t tile_smem_size(int cap, int esize, int with_bsh) { return tile_smem_bytes(cap, esize, with_bsh != 0); }

template hipError_t launch_sweep_tile<float>(const Dev &, const float *, float *, const double *, const double *,
                                             const double *, const SweepItem *, int, int, int3, int, int, int,
                                             double *, hipStream_t);
template hipError_t launch_sweep_tile<double>(const Dev &, const double *, double *, const double *, const double *,
                                              const double *, const SweepItem *, int, int, int3, int, int, int,
                                              double *, hipStream_t);
template hipError_t launch_transient_tile<float>(const Dev &, const float *, float *, const double *, const double *,
                                                 const TileItem *, int, int3, int, int, int, double, double, double *,
                                                 hipStream_t);
template hipError_t launch_transient_tile<double>(const Dev &, const double *, double *, const double *,
                                                  const double *, const TileItem *, int, int3, int, int, int, double,
                                                  double, double *, hipStream_t);

template hipError_t launch_sweep_adj<float>(const Dev &, const float *, float *, const double *, const double *,
                                            const SweepItem *, int, int, int3, int, int, int, double *, hipStream_t);
template hipError_t launch_sweep_adj<double>(const Dev &, const double *, double *, const double *, const double *,
                                             const SweepItem *, int, int, int3, int, int, int, double *, hipStream_t);

}  // namespace bte
