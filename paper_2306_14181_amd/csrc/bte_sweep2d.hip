// bte_sweep2d.hip -- register-resident tile sweep for two-dimensional
// geometries (the steady transport sweep of Sec. 3.3-3.5, Algorithm 1, in
// delta form with the first-order upwind implicit operator).
//
// One wavefront per work item (tile of TX x TY cells, octant, chunk of 64
// (direction, band) lanes).  The tile is walked row by row in the flow
// frame of the octant: a window of four rows of e (two upwind rows, the
// current row with its x halo, the next row) lives in registers, so the
// stencil of every cell is read from registers, the right-hand side and the
// upwind recurrence of a row are computed together, and no barrier is needed
// inside the tile.  Everything that depends only on the cell (global index,
// geometry code, T_L, scattering rate, source, pending correction) is loaded
// once, one cell per lane, and broadcast with readlane.  The FP64 moment
// partials of a row are reduced through a small LDS transpose.
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tile.h"
#include "bte_tilelds.h"

namespace bte {

namespace {

constexpr int kTX = 8, kTY = 8;

struct Frame2 {
    int o0, o1, e0, e1, sg0, sg1, n0, n1, cell0, per0, per1;
    double pdT0, pdT1;
};

__device__ inline Frame2 frame2(const Film &fm, int sg0, int sg1, int tile)
{
    Frame2 F;
    F.n0 = fm.n[0];
    F.n1 = fm.n[1];
    const int nt0 = (F.n0 + kTX - 1) / kTX;
    const int tc0 = tile % nt0, tc1 = tile / nt0;
    F.o0 = tc0 * kTX;
    F.o1 = tc1 * kTY;
    F.e0 = min(kTX, F.n0 - F.o0);
    F.e1 = min(kTY, F.n1 - F.o1);
    F.sg0 = sg0;
    F.sg1 = sg1;
    F.cell0 = fm.cell0;
    F.per0 = fm.periodic[0];
    F.per1 = fm.periodic[1];
    F.pdT0 = fm.pdT[0];
    F.pdT1 = fm.pdT[1];
    return F;
}

// Global cell of flow position (f0, f1) and the periodic jump of the value
// there (units of C/4pi); -1 outside a non-periodic domain or in a pore.
__device__ inline int cell2(const Dev &d, const Frame2 &F, int f0, int f1, double &jump)
{
    int i0 = F.o0 + (F.sg0 > 0 ? f0 : F.e0 - 1 - f0);
    int i1 = F.o1 + (F.sg1 > 0 ? f1 : F.e1 - 1 - f1);
    jump = 0.0;
    if (i0 < 0 || i0 >= F.n0) {
        if (!F.per0) return -1;
        jump += (i0 < 0 ? 1.0 : -1.0) * F.pdT0;   // the low face adds +C dT/4pi
        i0 = ((i0 % F.n0) + F.n0) % F.n0;
    }
    if (i1 < 0 || i1 >= F.n1) {
        if (!F.per1) return -1;
        jump += (i1 < 0 ? 1.0 : -1.0) * F.pdT1;
        i1 = ((i1 % F.n1) + F.n1) % F.n1;
    }
    const int c = F.cell0 + i0 + F.n0 * i1;
    return (d.code[c] & kSolidBit) ? c : -1;
}

// Halo positions, one per lane: h < 8: row -2, h < 16: row -1, h < 24: row
// e1 (downwind), h < 48: x halo of row r = (h - 24) / 3 at f0 = -2, -1, e0.
__device__ inline bool halo_pos(const Frame2 &F, int h, int &f0, int &f1)
{
    if (h < 24) {
        f0 = h & 7;
        f1 = h < 8 ? -2 : (h < 16 ? -1 : F.e1);
        return f0 < F.e0;
    }
    if (h < 48) {
        const int r = (h - 24) / 3, w = (h - 24) - 3 * r;
        f1 = r;
        f0 = w == 0 ? -2 : (w == 1 ? -1 : F.e0);
        return r < F.e1;
    }
    return false;
}

__device__ inline int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ inline double rl(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of the lane's element at a broadcast cell c (with correction x in
// units of C/4pi), 0 if c < 0
template <typename T>
__device__ inline T ldc(const T *__restrict__ e, int c, int nk, int k, bool active, T C4, double x)
{
    if (c < 0 || !active) return (T)0;
    return e[(size_t)c * nk + k] + C4 * (T)x;
}

}  // namespace

// Limited or least-squares slope difference of the fast path: face value
// difference f(i) - f(i-1) along the flow with all three neighbours present.
template <typename T, int LIM>
__device__ inline T delta_fast(T e2, T e1, T ec, T ed)
{
    if (LIM == LIM_NONE) return (ec - e1) + (T)0.25 * ((ed - e1) - (ec - e2));
    const T d0 = e1 - e2, d1 = ec - e1, d2 = ed - ec;
    return d1 + (T)0.5 * (lim_diff<T, LIM>(d1, d2) - lim_diff<T, LIM>(d0, d1));
}

// General face-value difference of one axis (missing neighbours, walls).
template <typename T, int LIM>
__device__ inline T delta_general(const Dev &d, const Film &fm, const T *__restrict__ e,
                                  const double *__restrict__ din, int c, uint32_t code, int a, int sg, bool hu,
                                  bool hu2, bool hd, T e2, T e1, T ec, T ed, int cd, double xd, double xc, int al,
                                  int l, int k, bool active, T C4, T hh, T ih, int nk)
{
    const T fout = ec + hh * slope_flow<T>(LIM, hu, hd, e1, ec, ed, ih);
    T fin;
    if (hu) {
        fin = e1 + hh * slope_flow<T>(LIM, hu2, true, e2, e1, ec, ih);
    } else {
        const int su = -sg;
        const int kind = side_wall(axis_bits(code, a), su);
        if (kind == 0) {
            const double Tw = side_outer(code, a, su) ? fm.wallT[face_of(a, su)] : d.poreT;
            fin = C4 * (T)Tw;
        } else if (kind == 1) {
            const int km = d.mirror[a * d.na + al] * d.nl + l;
            const T em = active ? e[(size_t)c * nk + km] + C4 * (T)xc : (T)0;
            T gm = (T)0;
            if (LIM == LIM_NONE && hd && active) gm = (em - (e[(size_t)cd * nk + km] + C4 * (T)xd)) * ih;
            fin = em + hh * gm;
        } else {
            const int rec = diffuse_index(d, c, code, face_of(a, su));
            fin = (T)din[(size_t)rec * d.nl + l];
        }
    }
    (void)k;
    return fout - fin;
}

// Per tile cell mode word (built once per wave, read as a uniform value)
enum : uint32_t {
    W_SOLID = 1u, W_FX = 2u, W_FY = 4u,        // solid; interior stencil along x / y
    W_CX = 8u, W_CY = 16u                      // implicit coupling to the upwind cell along x / y
};

template <typename T, int LIM>
__global__ __launch_bounds__(64) void k_sweep2d(Dev d, const T *__restrict__ ein, T *__restrict__ eout,
                                                const double *__restrict__ dpend, const double *__restrict__ TLdev,
                                                const double *__restrict__ din,
                                                const SweepItem *__restrict__ items, int item0, int na_oct,
                                                int nchunk_oct, double *__restrict__ part)
{
    __shared__ double lc[64][kMomN + 1];
    __shared__ T xs[64 * 65];        // [lane][cell], padded: conflict-free both ways
    __shared__ T wx[kTX + 3][64];    // row window of the general path: x halo + row
    __shared__ T wy[3][kTX][64];     // rows f1-2, f1-1, f1+1
    __shared__ T gd[kTX][64];        // flux divergence of general cells

    const SweepItem it = items[item0 + blockIdx.x];
    const Film &fm = d.film[it.film];
    const int lane = threadIdx.x;
    const int kbeg = it.oct * na_oct * d.nl, kend = kbeg + na_oct * d.nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const int nk = d.nk;
    const LaneT<T> L = lane_make<T>(d, fm, active ? k : kbeg);
    lc[lane][0] = active ? L.w : 0.0;
    lc[lane][1] = active ? L.witau : 0.0;
    lc[lane][2] = active ? L.wv[0] : 0.0;
    lc[lane][3] = active ? L.wv[1] : 0.0;
    lc[lane][4] = active ? L.wv[2] : 0.0;
    const Frame2 F = frame2(fm, octant_sign(d, it.oct, na_oct, 0), octant_sign(d, it.oct, na_oct, 1), it.tile);
    const int e0 = F.e0, e1 = F.e1;
    const int sg0 = F.sg0, sg1 = F.sg1;
    const int sx = sg0 > 0 ? 1 : -1;
    const int rowstep = sg1 > 0 ? F.n0 : -F.n0;
    const int cbase = F.cell0 + (sg0 > 0 ? F.o0 : F.o0 + e0 - 1) + F.n0 * (sg1 > 0 ? F.o1 : F.o1 + e1 - 1);

    // ---- cell records, one cell per lane, broadcast with readlane:
    //   tile cell t = f0 + 8 f1 in lane t: global cell (any; -1 outside the
    //   tile), mode word, T_L, gamma, P/C_tot, pending correction;
    //   halo cell h (see halo_pos) in lane h: solid cell or -1, correction
    //   (pending correction + periodic jump).
    int t_c = -1;
    uint32_t t_w = 0;
    T t_tl = 0, t_gam = 0, t_qs = 0, t_x = 0;
    int h_c = -1;
    T h_x = 0;
    {
        const int f0 = lane & 7, f1 = lane >> 3;
        if (f0 < e0 && f1 < e1) {
            const int c = cbase + rowstep * f1 + sx * f0;
            t_c = c;
            const uint32_t code = d.code[c];
            if (code & kSolidBit) {
                const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1);
                const bool hu0 = side_is_cell(ab0, -sg0), hu1 = side_is_cell(ab1, -sg1);
                bool hu20 = false, hu21 = false;
                if (hu0) hu20 = side_is_cell(axis_bits(d.code[d.nb[face_of(0, -sg0) * d.nc + c]], 0), -sg0);
                if (hu1) hu21 = side_is_cell(axis_bits(d.code[d.nb[face_of(1, -sg1) * d.nc + c]], 1), -sg1);
                uint32_t w = W_SOLID;
                if (hu0 && hu20 && side_is_cell(ab0, sg0)) w |= W_FX;
                if (hu1 && hu21 && side_is_cell(ab1, sg1)) w |= W_FY;
                if (hu0 && !side_wraps(ab0, -sg0)) w |= W_CX;
                if (hu1 && !side_wraps(ab1, -sg1)) w |= W_CY;
                t_w = w;
                t_tl = TLdev ? (T)TLdev[c] : (T)0;
                t_gam = (T)d.gamma[c];
                t_qs = d.P ? (T)(d.P[c] / d.Ctot) : (T)0;   // P is null without a heat source
                t_x = dpend ? (T)dpend[c] : (T)0;
            }
        }
        int h0, h1;
        if (halo_pos(F, lane, h0, h1)) {
            double jmp;
            h_c = cell2(d, F, h0, h1, jmp);
            if (h_c >= 0) h_x = (T)((dpend ? dpend[h_c] : 0.0) + jmp);
        }
    }
    auto rlt = [&](T v, int l) -> T {
        if constexpr (sizeof(T) == 4) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
        else return rl((double)v, l);
    };
    // slot s: tile cell (s < 64) or halo cell 64 + h
    auto slot_c = [&](int s) { return s < 64 ? rl(t_c, s) : rl(h_c, s - 64); };
    auto slot_x = [&](int s) { return s < 64 ? rlt(t_x, s) : rlt(h_x, s - 64); };

    const T C4 = L.C4, cp0 = L.cpl[0], cp1 = L.cpl[1];
    const T A0 = cp0 + cp1 + L.itau;
    // Loads are unconditional (a missing cell or an inactive lane reads a
    // valid element and the value is dropped afterwards): a load under a
    // branch would be waited for before the branch joins, and the wavefront
    // would then pay the full memory latency once per load.
    // A missing cell reads the zero row (and has no correction); inactive
    // lanes read a valid element whose value is never stored.  Values are
    // prefetched raw (the load is not consumed) one row ahead of their use;
    // the pending correction and periodic jump (C/4pi x) are added when the
    // row becomes current.
    const int kk = active ? k : kbeg;
    const T *zrow = static_cast<const T *>(d.zrow);
    auto raw = [&](const T *base, int slot) -> T {
        const int c = slot_c(slot);
        const T *row = c >= 0 ? base + (size_t)c * nk : zrow;
        return row[kk];
    };
    // tile row r < e1: the cell index is arithmetic (pores are read too and
    // masked by the codes)
    auto raw_tile = [&](int r, int j) -> T {
        const T *row = j < e0 ? ein + (size_t)(cbase + rowstep * r + sx * j) * nk : zrow;
        return row[kk];
    };
    auto corr = [&](int slot) -> T { return C4 * slot_x(slot); };
    auto row_slot = [&](int r, int j) { return r < e1 ? 8 * r + j : 64 + 16 + j; };

    // window: rows f1-2, f1-1, f1 (cur), f1+1 (yp1) as final values; raw
    // prefetch of row f1+2 and of the x halo (-2, -1, e0) and x-upwind
    // increment of row f1+1; increments of row f1-1 (dpr)
    T ym2[kTX], ym1[kTX], cur[kTX], yp1[kTX], pr2[kTX], dpr[kTX];
    T xh0, xh1, xh2, dupx, pxh0, pxh1, pxh2, pdup;
#pragma unroll
    for (int j = 0; j < kTX; ++j) {
        ym2[j] = raw(ein, 64 + j);
        ym1[j] = raw(ein, 64 + 8 + j);
        dpr[j] = raw(eout, 64 + 8 + j);
        cur[j] = raw_tile(0, j);
        yp1[j] = e1 > 1 ? raw_tile(1, j) : raw(ein, 64 + 16 + j);
    }
    pxh0 = raw(ein, 64 + 24);
    pxh1 = raw(ein, 64 + 25);
    pxh2 = raw(ein, 64 + 26);
    pdup = raw(eout, 64 + 25);
#pragma unroll
    for (int j = 0; j < kTX; ++j) {
        ym2[j] += corr(64 + j);
        ym1[j] += corr(64 + 8 + j);
        dpr[j] = dpr[j] - ym1[j];
        cur[j] += corr(j);
        yp1[j] += corr(row_slot(1, j));
    }

    for (int f1 = 0; f1 < e1; ++f1) {
        const int hx = 64 + 24 + 3 * f1;
        // current x halo from the prefetch
        xh0 = pxh0 + corr(hx);
        xh1 = pxh1 + corr(hx + 1);
        xh2 = pxh2 + corr(hx + 2);
        dupx = pdup - xh1;
        // prefetch (unconditional, clamped: a load under a branch would be
        // waited for at the join): row f1 + 2, the downwind halo row when
        // f1 + 2 == e1; the x halo of row f1 + 1
        {
            const int r2 = f1 + 2;
#pragma unroll
            for (int j = 0; j < kTX; ++j) pr2[j] = r2 < e1 ? raw_tile(r2, j) : raw(ein, 64 + 16 + j);
            const int hn = f1 + 1 < e1 ? hx + 3 : hx;
            pxh0 = raw(ein, hn);
            pxh1 = raw(ein, hn + 1);
            pxh2 = raw(ein, hn + 2);
            pdup = raw(eout, hn + 1);
        }

        // flux divergence: interior cells here, the others (walls, pores,
        // missing neighbours) in one loop over the row window in LDS
        T D[kTX];
        uint32_t gmask = 0;
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            D[j] = (T)0;
            const uint32_t w = (uint32_t)rl((int)t_w, 8 * f1 + j);
            if ((w & (W_SOLID | W_FX | W_FY)) == (W_SOLID | W_FX | W_FY)) {
                const T ex2 = j >= 2 ? cur[j - 2] : (j == 1 ? xh1 : xh0);
                const T ex1 = j >= 1 ? cur[j - 1] : xh1;
                const T exd = j + 1 < e0 ? cur[j + 1] : xh2;
                D[j] = cp0 * delta_fast<T, LIM>(ex2, ex1, cur[j], exd) +
                       cp1 * delta_fast<T, LIM>(ym2[j], ym1[j], cur[j], yp1[j]);
            } else if (w & W_SOLID) {
                gmask |= 1u << j;
            }
        }
        if (gmask) {
            wx[0][lane] = xh0;
            wx[1][lane] = xh1;
#pragma unroll
            for (int j = 0; j < kTX; ++j) {
                wx[j + 2][lane] = cur[j];
                wy[0][j][lane] = ym2[j];
                wy[1][j][lane] = ym1[j];
                wy[2][j][lane] = yp1[j];
            }
            wx[e0 + 2][lane] = xh2;
            for (uint32_t m = gmask; m; m &= m - 1) {
                const int j = __builtin_ctz(m);
                const int t = 8 * f1 + j;
                const int c = rl(t_c, t);
                const uint32_t code = d.code[c];
                const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1);
                const uint32_t w = (uint32_t)rl((int)t_w, t);
                const bool hu0 = side_is_cell(ab0, -sg0), hd0 = side_is_cell(ab0, sg0);
                const bool hu1 = side_is_cell(ab1, -sg1), hd1 = side_is_cell(ab1, sg1);
                // second upwind cell: from the upwind cell's code
                const int cu0 = hu0 ? d.nb[face_of(0, -sg0) * d.nc + c] : -1;
                const int cu1 = hu1 ? d.nb[face_of(1, -sg1) * d.nc + c] : -1;
                const bool hu20 = cu0 >= 0 && side_is_cell(axis_bits(d.code[cu0], 0), -sg0);
                const bool hu21 = cu1 >= 0 && side_is_cell(axis_bits(d.code[cu1], 1), -sg1);
                const T ex2 = wx[j][lane], ex1 = wx[j + 1][lane], ec = wx[j + 2][lane], exd = wx[j + 3][lane];
                const T ey2 = wy[0][j][lane], ey1 = wy[1][j][lane], eyd = wy[2][j][lane];
                const double xc = (double)rlt(t_x, t);
                T dx, dy;
                if (w & W_FX) {
                    dx = delta_fast<T, LIM>(ex2, ex1, ec, exd);
                } else {
                    // downwind cell and its correction (the x halo or the next cell of the row)
                    const int sd = j + 1 < e0 ? t + 1 : hx + 2;
                    const int cd = hd0 ? slot_c(sd) : -1;
                    dx = delta_general<T, LIM>(d, fm, ein, din, c, code, 0, sg0, hu0, hu20, hd0, ex2, ex1, ec, exd,
                                               cd, (double)slot_x(sd), xc, L.al, L.l, k, active, C4, L.hh[0], L.ih[0], nk);
                }
                if (w & W_FY) {
                    dy = delta_fast<T, LIM>(ey2, ey1, ec, eyd);
                } else {
                    const int sd = f1 + 1 < e1 ? t + 8 : 64 + 16 + j;
                    const int cd = hd1 ? slot_c(sd) : -1;
                    dy = delta_general<T, LIM>(d, fm, ein, din, c, code, 1, sg1, hu1, hu21, hd1, ey2, ey1, ec, eyd,
                                               cd, (double)slot_x(sd), xc, L.al, L.l, k, active, C4, L.hh[1], L.ih[1], nk);
                }
                gd[j][lane] = cp0 * dx + cp1 * dy;
            }
#pragma unroll
            for (int j = 0; j < kTX; ++j)
                if (gmask & (1u << j)) D[j] = gd[j][lane];
        }

        // right-hand side and upwind recurrence along the row
        const int b = cbase + rowstep * f1;
        T dl = dupx;   // increment of the upwind x neighbour
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            if (j < e0) {
                const int t = 8 * f1 + j;
                const int c = b + sx * j;
                const uint32_t w = (uint32_t)rl((int)t_w, t);
                T en = (T)0;
                if (w & W_SOLID) {
                    const T ec = cur[j];
                    const T gam = rlt(t_gam, t);
                    const T itc = L.itau + gam;
                    T num = -D[j] - (ec - C4 * rlt(t_tl, t)) * itc + C4 * rlt(t_qs, t);
                    // implicit upwind couplings (not across periodic faces)
                    if (w & W_CX) num += cp0 * dl;
                    if (w & W_CY) num += cp1 * dpr[j];
                    const T den = A0 + gam;
                    T dlt;
                    if constexpr (sizeof(T) == 4) dlt = num * __builtin_amdgcn_rcpf(den);
                    else dlt = num / den;
                    en = ec + dlt;
                    dl = dlt;
                    dpr[j] = dlt;
                    if (active) eout[(size_t)c * nk + k] = en;
                } else {
                    dl = (T)0;
                    dpr[j] = (T)0;
                    if (active) eout[(size_t)c * nk + k] = ein[(size_t)c * nk + k];
                }
                xs[lane * 65 + t] = active ? en : (T)0;
            }
        }
        // advance the window
        const int s2 = row_slot(min(f1 + 2, e1), 0);
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            ym2[j] = ym1[j];
            ym1[j] = cur[j];
            cur[j] = yp1[j];
            yp1[j] = pr2[j] + corr(s2 + j);
        }
    }
    __syncthreads();
    // moment partials: lane = tile cell (f0 + 8 f1), sum over the 64 lanes
    {
        const int c = t_c;
        if (c >= 0) {
            double acc[kMomN] = {0, 0, 0, 0, 0};
            if (t_w & W_SOLID) {
#pragma unroll 4
                for (int l2 = 0; l2 < 64; ++l2) {
                    const double x = (double)xs[l2 * 65 + lane];
#pragma unroll
                    for (int m = 0; m < kMomN; ++m) acc[m] += lc[l2][m] * x;
                }
                acc[1] += d.gamma[c] * acc[0];
            }
            double *o = part + ((size_t)(it.oct * nchunk_oct + it.chunk) * d.nc + c) * kMomN;
#pragma unroll
            for (int m = 0; m < kMomN; ++m) o[m] = acc[m];
        }
    }
}

template <typename T, int LIM>
void sweep2d_launch(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev, const double *din,
                    const SweepItem *items, int item0, int count, int na_oct, int nchunk_oct, double *part,
                    hipStream_t s)
{
    hipLaunchKernelGGL((k_sweep2d<T, LIM>), dim3(count), dim3(64), 0, s, d, ein, eout, dpend, TLdev, din, items,
                       item0, na_oct, nchunk_oct, part);
}

template <typename T>
hipError_t launch_sweep2d(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev,
                          const double *din, const SweepItem *items, int item0, int count, int na_oct,
                          int nchunk_oct, double *part, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (d.limiter == LIM_NONE)
        sweep2d_launch<T, LIM_NONE>(d, ein, eout, dpend, TLdev, din, items, item0, count, na_oct, nchunk_oct, part, s);
    else if (d.limiter == LIM_MC)
        sweep2d_launch<T, LIM_MC>(d, ein, eout, dpend, TLdev, din, items, item0, count, na_oct, nchunk_oct, part, s);
    else
        sweep2d_launch<T, LIM_MINMOD>(d, ein, eout, dpend, TLdev, din, items, item0, count, na_oct, nchunk_oct, part,
                                      s);
    return hipGetLastError();
}

template hipError_t launch_sweep2d<float>(const Dev &, const float *, float *, const double *, const double *,
                                          const double *, const SweepItem *, int, int, int, int, double *,
                                          hipStream_t);
template hipError_t launch_sweep2d<double>(const Dev &, const double *, double *, const double *, const double *,
                                           const double *, const SweepItem *, int, int, int, int, double *,
                                           hipStream_t);

}  // namespace bte
