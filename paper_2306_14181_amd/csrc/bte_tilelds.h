// bte_tilelds.h -- LDS layout and set-up of a tile block, shared by the
// forward transport kernels and their transposes (adjoint).
//
// A block owns one tile of one geometry (see bte_tile.h for the star of
// slots) and works on 64 (direction, band) lanes of one octant at a time.
// Everything that depends only on the cell (neighbour slots, wall kinds,
// T_L, source, scattering rate) is prepared once per tile in LDS and read as
// wavefront-uniform scalars; everything that depends only on the lane is
// prepared once per lane chunk.
#pragma once
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

// Per (cell, axis) stencil mode bits, in the flow frame of the tile:
//   M_HU / M_HU2 first / second upwind cell exists, M_HD downwind cell exists,
//   M_WRAP the upwind cell is reached through a periodic face,
//   bits 4-5 wall kind on the upwind side (when there is no upwind cell),
//   and for the transposed operators only:
//   bits 6-7 wall kind on the upwind side of the upwind cell (M_HU, no M_HU2),
//   M_HD2 the downwind cell has a downwind cell of its own.
enum : int { M_HU = 1, M_HU2 = 2, M_HD = 4, M_WRAP = 8, M_KSHIFT = 4, M_K2SHIFT = 6, M_HD2 = 256 };

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
    unsigned short *mode;  // [64][3] stencil mode bits
};

__host__ __device__ inline size_t tile_smem_bytes(int cap, int esize, bool with_bsh)
{
    size_t b = (size_t)cap * 64 * esize + (with_bsh ? (size_t)(64 + 48) * 64 * esize : 0);
    b += (size_t)cap * 8 + 64 * 5 * 8 + 3 * 64 * 8;   // slot_x, mom, gam, tl, qs
    b += (size_t)cap * 8;                              // slot_off
    b += 64 * 4 * 2;                                   // cell, code
    b += 64 * 9 * 2 + (size_t)cap * 2;                 // stn, slot_up1
    b += 64 * 3 * 3;                                   // upin, mode
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
    m.mode = reinterpret_cast<unsigned short *>(p);
    return m;
}

// Slot and tile-cell tables (all threads).  dpend (pending isotropic
// correction, may be null) and, if `jumps`, the periodic jump are folded
// into slot_x (the transposed operators are linear: no jump).
template <typename T>
__device__ inline void tile_tables(const TileCtx t, const Film &fm, const Dev &d, TileSmem<T> &S,
                                   const double *__restrict__ TLdev, const double *__restrict__ dpend,
                                   bool jumps = true)
{
    for (int s = threadIdx.x; s < t.nslot; s += blockDim.x) {
        int f0, f1, f2, jmp;
        const int a = tile_pos(t, s, f0, f1, f2);
        const int c = tile_cell(t, fm, d, f0, f1, f2, jmp);
        const double pdt = (a == 0) * fm.pdT[0] + (a == 1) * fm.pdT[1] + (a == 2) * fm.pdT[2];
        S.slot_off[s] = c >= 0 ? (long long)c * d.nk : -1;
        S.slot_x[s] = c >= 0 ? (dpend ? dpend[c] : 0.0) + (jumps ? jmp * pdt : 0.0) : 0.0;
        S.slot_up1[s] = (short)((c >= 0 && jmp == 0) ? tile_up1(t, s) : -1);
        if (s < t.nt) {
            const int craw = tile_raw_cell(t, fm, f0, f1, f2);
            S.cell[s] = craw;
            S.code[s] = d.code[craw];
            S.gam[s] = d.gamma[craw];
            S.tl[s] = TLdev ? TLdev[craw] : 0.0;
            S.qs[s] = d.P ? d.P[craw] / fm.Ctot : 0.0;
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
// `adj` adds the bits only the transposed operators read.
template <typename T>
__device__ inline void tile_modes(const TileCtx t, const Dev &d, TileSmem<T> &S, bool adj = false)
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
                if (adj) {
                    if (m & M_HD) {
                        const int cd = (int)(S.slot_off[sd] / d.nk);
                        if (side_is_cell(axis_bits(d.code[cd], a), sg)) m |= M_HD2;
                    }
                    if (hu && !(m & M_HU2)) {
                        const int c1 = (int)(S.slot_off[s1] / d.nk);
                        m |= side_wall(axis_bits(d.code[c1], a), -sg) << M_K2SHIFT;
                    }
                }
            }
            S.mode[3 * i + a] = (unsigned short)m;
            S.upin[3 * i + a] = (signed char)((a < d.dim && solid && fa > 0 && (m & M_HU)) ? i - stride : -1);
        }
    }
}

// Stage the star for lane k (wave w loads slots w, w+4, ...) in register
// batches.  If eout is given (sweep), the increments e^{n+1} - e^n of the
// first upwind halo layer (not periodic) go to `dup`.  The loads are
// unconditional: a missing cell reads the zero row, an inactive lane reads
// element 0 of a valid row (never stored), and the batch index is clamped;
// a load under a branch would be waited for before the branch joins.
template <typename T, int NB = 16>
__device__ inline void tile_load(const TileCtx t, TileSmem<T> &S, const T *__restrict__ e, int k, bool active, T C4,
                                 const T *__restrict__ zrow, const T *__restrict__ eout = nullptr)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kk = active ? k : 0;
    for (int s0 = wave; s0 < t.nslot; s0 += 4 * NB) {
        T v[NB], w[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int s = min(s0 + 4 * j, t.nslot - 1);
            const long long off = S.slot_off[s];
            const T *row = off >= 0 ? e + off : zrow;
            v[j] = row[kk];
            w[j] = (T)0;
            if (eout) {
                const T *ro = (off >= 0 && S.slot_up1[s] >= 0) ? eout + off : zrow;
                w[j] = ro[kk];
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
// In single precision both are medians: minmod(a, b) = med3(a, b, 0) and
// MC(a, b) = med3(4 minmod(a, b), a + b, 0) / 2 (the scalings are exact).
template <typename T, int LIM> __device__ inline T lim_diff(T dl, T dr)
{
    if constexpr (sizeof(T) == 4) {
        const float mm = __builtin_amdgcn_fmed3f(dl, dr, 0.0f);
        if (LIM == LIM_MC) return 0.5f * __builtin_amdgcn_fmed3f(4.0f * mm, dl + dr, 0.0f);
        return mm;
    } else {
        T m;
        if (LIM == LIM_MC) m = fmin(fmin((T)2 * fabs(dl), (T)2 * fabs(dr)), (T)0.5 * fabs(dl + dr));
        else m = fmin(fabs(dl), fabs(dr));
        return dl * dr > (T)0 ? copysign(m, dl) : (T)0;
    }
}

// Cross-lane move of a double inside a row of 16 lanes (DPP control CTRL).
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Limited or least-squares slope difference of the fast path: face value
// difference f(i) - f(i-1) along the flow with all three neighbours present.
template <typename T, int LIM>
__device__ inline T delta_fast(T e2, T e1, T ec, T ed)
{
    if (LIM == LIM_NONE) return (ec - e1) + (T)0.25 * ((ed - e1) - (ec - e2));
    const T d0 = e1 - e2, d1 = ec - e1, d2 = ed - ec;
    return d1 + (T)0.5 * (lim_diff<T, LIM>(d1, d2) - lim_diff<T, LIM>(d0, d1));
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
    const int mb = fm.moff + L.l;   // the band in the geometry's material
    const double v = d.v[mb], it = d.itau[mb];
    L.C4 = (T)d.C4[mb];
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

__device__ inline int octant_sign(const Dev &d, int oct, int na_oct, int a)
{
    return d.s[3 * (oct * na_oct) + a] > 0 ? 1 : -1;
}

}  // namespace bte
