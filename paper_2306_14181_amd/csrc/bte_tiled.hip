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

namespace bte {

template <int N> __device__ inline void wave_sum_t(double (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
}

__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// per (cell, axis) stencil mode bits
enum : int { M_HU = 1, M_HU2 = 2, M_HD = 4, M_WRAP = 8, M_KSHIFT = 4 };   // wall kind in bits 4-5

// Dynamic LDS layout of a tile block.
template <typename T> struct TileSmem {
    T *box;                // [cap][64]
    T *bsh;                // [64][64] right-hand side, then increments (sweep)
    T *dup;                // [48][64] increments of first-layer upwind halo cells (sweep)
    double *slot_x;        // [cap] pending correction + periodic jump (units of C/4pi)
    double *mom;           // [64][5] moment accumulators
    double *gam;           // [64] extra scattering rate
    double *tl;            // [64] lattice temperature deviation T_L^n
    double *qs;            // [64] P / Ctot
    long long *slot_off;   // [cap] element offset of the slot's cell (c * nk) or -1
    int *cell;             // [64] global cell of tile cell (pores included)
    uint32_t *code;        // [64]
    short *stn;            // [64][3][3] slots: upwind, second upwind, downwind per axis
    short *slot_up1;       // [cap] compact first-upwind-layer index or -1 (sweep inflow)
    signed char *upin;     // [64][3] in-tile upwind neighbour per axis or -1
    unsigned char *mode;   // [64][3] stencil mode bits
};

__host__ __device__ inline size_t tile_smem_bytes(int cap, int esize, bool with_bsh)
{
    size_t b = (size_t)cap * 64 * esize + (with_bsh ? (size_t)(64 + 48) * 64 * esize : 0);
    b += (size_t)cap * 8 + 64 * 5 * 8 + 3 * 64 * 8;   // slot_x, mom, gam, tl, qs
    b += (size_t)cap * 8;                              // slot_off
    b += 64 * 4 * 2;                                   // cell, code
    b += 64 * 9 * 2 + (size_t)cap * 2;                 // stn, slot_up1
    b += 64 * 3 * 2;                                   // upin, mode
    return (b + 255) & ~size_t(255);
}

template <typename T> __device__ inline TileSmem<T> tile_smem(char *base, int cap, bool with_bsh)
{
    TileSmem<T> m;
    char *p = base;
    m.box = reinterpret_cast<T *>(p);
    p += (size_t)cap * 64 * sizeof(T);
    m.bsh = reinterpret_cast<T *>(p);
    if (with_bsh) p += (size_t)64 * 64 * sizeof(T);
    m.dup = reinterpret_cast<T *>(p);
    if (with_bsh) p += (size_t)48 * 64 * sizeof(T);
    m.slot_x = reinterpret_cast<double *>(p);
    p += (size_t)cap * 8;
    m.mom = reinterpret_cast<double *>(p);
    p += 64 * 5 * 8;
    m.gam = reinterpret_cast<double *>(p);
    p += 64 * 8;
    m.tl = reinterpret_cast<double *>(p);
    p += 64 * 8;
    m.qs = reinterpret_cast<double *>(p);
    p += 64 * 8;
    m.slot_off = reinterpret_cast<long long *>(p);
    p += (size_t)cap * 8;
    m.cell = reinterpret_cast<int *>(p);
    p += 64 * 4;
    m.code = reinterpret_cast<uint32_t *>(p);
    p += 64 * 4;
    m.stn = reinterpret_cast<short *>(p);
    p += 64 * 9 * 2;
    m.slot_up1 = reinterpret_cast<short *>(p);
    p += (size_t)cap * 2;
    m.upin = reinterpret_cast<signed char *>(p);
    p += 64 * 3;
    m.mode = reinterpret_cast<unsigned char *>(p);
    return m;
}

// Slot and tile-cell tables (all threads).  dpend (pending isotropic
// correction, may be null) and the periodic jump are folded into slot_x.
template <typename T>
__device__ inline void tile_tables(const TileCtx t, const Film &fm, const Dev &d, TileSmem<T> &S,
                                   const double *__restrict__ TLdev, const double *__restrict__ dpend)
{
    for (int s = threadIdx.x; s < t.nslot; s += blockDim.x) {
        int f0, f1, f2, jmp;
        const int a = tile_pos(t, s, f0, f1, f2);
        const int c = tile_cell(t, fm, d, f0, f1, f2, jmp);
        const double pdt = (a == 0) * fm.pdT[0] + (a == 1) * fm.pdT[1] + (a == 2) * fm.pdT[2];
        S.slot_off[s] = c >= 0 ? (long long)c * d.nk : -1;
        S.slot_x[s] = c >= 0 ? (dpend ? dpend[c] : 0.0) + jmp * pdt : 0.0;
        S.slot_up1[s] = (short)((c >= 0 && jmp == 0) ? tile_up1(t, s) : -1);
        if (s < t.nt) {
            const int craw = tile_raw_cell(t, fm, f0, f1, f2);
            S.cell[s] = craw;
            S.code[s] = d.code[craw];
            S.gam[s] = d.gamma[craw];
            S.tl[s] = TLdev ? TLdev[craw] : 0.0;
            S.qs[s] = d.P ? d.P[craw] / d.Ctot : 0.0;
            short *st = S.stn + 9 * s;
            st[0] = (short)tile_slot(t, f0 - 1, f1, f2);
            st[1] = (short)tile_slot(t, f0 - 2, f1, f2);
            st[2] = (short)tile_slot(t, f0 + 1, f1, f2);
            st[3] = (short)tile_slot(t, f0, f1 - 1, f2);
            st[4] = (short)tile_slot(t, f0, f1 - 2, f2);
            st[5] = (short)tile_slot(t, f0, f1 + 1, f2);
            st[6] = (short)tile_slot(t, f0, f1, f2 - 1);
            st[7] = (short)tile_slot(t, f0, f1, f2 - 2);
            st[8] = (short)tile_slot(t, f0, f1, f2 + 1);
        }
    }
}

// Stencil modes and in-tile upwind links (after the slot table is complete).
template <typename T> __device__ inline void tile_modes(const TileCtx t, const Dev &d, TileSmem<T> &S)
{
    for (int i = threadIdx.x; i < t.nt; i += blockDim.x) {
        const uint32_t code = S.code[i];
        const bool solid = code & kSolidBit;
        const int f0 = i % t.e0, f1 = (i / t.e0) % t.e1, f2 = i / (t.e0 * t.e1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int s1 = S.stn[9 * i + 3 * a], s2 = S.stn[9 * i + 3 * a + 1], sd = S.stn[9 * i + 3 * a + 2];
            const int fa = a == 0 ? f0 : (a == 1 ? f1 : f2);
            const int stride = a == 0 ? 1 : (a == 1 ? t.e0 : t.e0 * t.e1);
            const int sg = a == 0 ? t.sg0 : (a == 1 ? t.sg1 : t.sg2);
            int m = 0;
            if (a < d.dim && solid) {
                const bool hu = S.slot_off[s1] >= 0;
                if (hu) m |= M_HU;
                if (hu && S.slot_off[s2] >= 0) m |= M_HU2;
                if (S.slot_off[sd] >= 0) m |= M_HD;
                if (hu && S.slot_up1[s1] < 0 && s1 >= t.nt) m |= M_WRAP;   // periodic inflow: lagged
                if (!hu) m |= side_wall(axis_bits(code, a), -sg) << M_KSHIFT;
            }
            S.mode[3 * i + a] = (unsigned char)m;
            S.upin[3 * i + a] = (signed char)((a < d.dim && solid && fa > 0 && (m & M_HU)) ? i - stride : -1);
        }
    }
}

// Stage the star for lane k (wave w loads slots w, w+4, ...) in register
// batches.  If eout is given (sweep), the increments e^{n+1} - e^n of the
// first upwind halo layer (not periodic) go to `dup`.
template <typename T, int NB = 16>
__device__ inline void tile_load(const TileCtx t, TileSmem<T> &S, const T *__restrict__ e, int k, bool active, T C4,
                                 const T *__restrict__ eout = nullptr)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s0 = wave; s0 < t.nslot; s0 += 4 * NB) {
        T v[NB], w[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int s = s0 + 4 * j;
            v[j] = (T)0;
            w[j] = (T)0;
            if (s < t.nslot) {
                const long long off = S.slot_off[s];
                if (active && off >= 0) {
                    v[j] = e[off + k];
                    if (eout && S.slot_up1[s] >= 0) w[j] = eout[off + k];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int s = s0 + 4 * j;
            if (s < t.nslot) {
                const T corr = C4 * (T)S.slot_x[s];
                S.box[s * 64 + lane] = v[j] + corr;
                if (eout) {
                    const int u = S.slot_up1[s];
                    if (u >= 0) S.dup[u * 64 + lane] = w[j] - (v[j] + corr);
                }
            }
        }
    }
}

// Limited slope times h (a difference) from the one-sided differences
// dl = e_m - e_{m-1}, dr = e_{m+1} - e_m: MC = minmod(2 dl, 2 dr, (dl + dr)/2),
// MINMOD = minmod(dl, dr); the face value is e_m + lim/2.
template <typename T, int LIM> __device__ inline T lim_diff(T dl, T dr)
{
    T m;
    if (LIM == LIM_MC) m = fmin(fmin((T)2 * fabs(dl), (T)2 * fabs(dr)), (T)0.5 * fabs(dl + dr));
    else m = fmin(fabs(dl), fabs(dr));
    return dl * dr > (T)0 ? copysign(m, dl) : (T)0;
}

// Lane constants of one (direction, band) lane.
template <typename T> struct LaneT {
    int k, al, l;
    T C4, itau, cpl[3], hh[3], ih[3];
    double w, wv[3], witau;
};

template <typename T> __device__ inline LaneT<T> lane_make(const Dev &d, const Film &fm, int k)
{
    LaneT<T> L;
    L.k = k;
    L.al = k / d.nl;
    L.l = k - L.al * d.nl;
    L.w = d.w[L.al];
    const double v = d.v[L.l], it = d.itau[L.l];
    L.C4 = (T)d.C4[L.l];
    L.itau = (T)it;
    L.witau = L.w * it;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double sa = d.s[3 * L.al + a];
        L.cpl[a] = (T)(v * fabs(sa) * fm.ih[a]);
        L.hh[a] = (T)(0.5 * fm.h[a]);
        L.ih[a] = (T)fm.ih[a];
        L.wv[a] = L.w * v * sa;
    }
    return L;
}

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

__device__ inline int octant_sign(const Dev &d, int oct, int na_oct, int a)
{
    return d.s[3 * (oct * na_oct) + a] > 0 ? 1 : -1;
}

// ----------------------------------------------------------------- sweep
//
// One work item = one tile of one geometry for 64 lanes of one octant.
//   phase A (4 wavefronts): b = R(e^n; T_L^n) for every tile cell plus the
//     increments of the already-swept upstream tiles (first-order implicit
//     coupling), into LDS;
//   phase B (wavefront 0): upwind recurrence across the tile;
//   phase C (4 wavefronts): e^{n+1} = e^n + de and FP64 moment partials.

template <typename T, int DIM, int LIM>
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
    const Film &fm = d.film[it.film];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kbeg = it.oct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
    const TileCtx t = tile_make(fm, d.dim, octant_sign(d, it.oct, na_oct, 0), octant_sign(d, it.oct, na_oct, 1),
                                octant_sign(d, it.oct, na_oct, 2), it.tile, tdim);
    tile_tables<T>(t, fm, d, S, TLdev, dpend);
    __syncthreads();
    tile_modes<T>(t, d, S);
    tile_load<T>(t, S, ein, k, active, L.C4, eout);
    __syncthreads();

    for (int i = wave; i < t.nt; i += 4) {
        T b = (T)0;
        if (active && (uni(S.code[i]) & kSolidBit)) {
            int up_out[3];
            const T D = tile_flux<T, DIM, LIM>(d, fm, t, S, i, L, lane, ein, dpend, din, up_out);
            const T ec = S.box[i * 64 + lane];
            const T itc = L.itau + (T)S.gam[i];
            b = -D - (ec - L.C4 * (T)S.tl[i]) * itc + L.C4 * (T)S.qs[i];
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
            S.bsh[i * 64 + lane] = num / (A0 + (T)S.gam[i]);
        }
    }
    __syncthreads();

    const int pidx = it.oct * nchunk_oct + it.chunk;
    for (int i = wave; i < t.nt; i += 4) {
        const int c = uni(S.cell[i]);
        const bool solid = uni(S.code[i]) & kSolidBit;
        double acc[kMomN] = {0, 0, 0, 0, 0};
        if (active) {
            if (solid) {
                const T en = S.box[i * 64 + lane] + S.bsh[i * 64 + lane];
                eout[(size_t)c * d.nk + k] = en;
                const double x = (double)en;
                acc[0] = L.w * x;
                acc[1] = (L.witau + L.w * S.gam[i]) * x;
                acc[2] = L.wv[0] * x;
                acc[3] = L.wv[1] * x;
                acc[4] = L.wv[2] * x;
            } else {
                eout[(size_t)c * d.nk + k] = ein[(size_t)c * d.nk + k];
            }
        }
        wave_sum_t<kMomN>(acc);
        if (lane == 0)
            for (int q = 0; q < kMomN; ++q) part[((size_t)pidx * d.nc + c) * kMomN + q] = acc[q];
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
        tile_load<T>(t, S, ein, k, active, L.C4);
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
#define BTE_SWEEP(DIM, LIM)                                                                                          \
    if (d.dim == DIM && d.limiter == LIM)                                                                            \
        sweep_launch<T, DIM, LIM>(d, ein, eout, dpend, TLdev, din, items, item0, count, tdim, na_oct, nchunk_oct,    \
                                  cap, part, s);
    BTE_SWEEP(1, 0) BTE_SWEEP(1, 1) BTE_SWEEP(1, 2)
    BTE_SWEEP(2, 0) BTE_SWEEP(2, 1) BTE_SWEEP(2, 2)
    BTE_SWEEP(3, 0) BTE_SWEEP(3, 1) BTE_SWEEP(3, 2)
#undef BTE_SWEEP
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
    hipError_t a = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep_tile<T, DIM, LIM>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipError_t b = hipFuncSetAttribute(reinterpret_cast<const void *>(k_transient_tile<T, DIM, LIM>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return a != hipSuccess ? a : b;
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

}  // namespace bte
