// bte_tile.h -- LDS-staged stencil evaluation over a tile of cells.
//
// A block works on a tile of up to 64 cells for 64 (direction, band) lanes of
// one octant, so every lane shares the upwind side along each axis.  The
// tile is described in flow coordinates (position increases along the flow
// of the octant).  The second-order upwind face reconstruction of a cell
// reads 2 upwind and 1 downwind neighbours per axis, so the block stages the
// tile plus three halo layers per active axis -- a "star" of slots -- in LDS:
//   slots [0, nt)                    tile cells, flow-lexicographic order
//   slots nt + hoff[a] + L*cs[a] + x axis-a halo, layer L = 0 (two upwind),
//                                    1 (one upwind), 2 (one downwind),
//                                    x = position in the tile cross-section.
// Each slot holds the energy deviation of its cell in the tile's frame
// (periodic faces add the temperature-jump term) or is invalid (wall, pore
// or outside a non-periodic domain).  All stencil values then come from LDS.
#pragma once
#include "bte_internal.h"
#include "bte_stencil.h"

namespace bte {

// Scalars only (no arrays): the descriptor must stay in registers, and
// selects between its fields are written as arithmetic blends so that the
// compiler never turns them into loads from a computed address.
struct TileCtx {
    int sg0, sg1, sg2;   // flow sign per axis
    int o0, o1, o2;      // index-space origin
    int e0, e1, e2;      // extent (1 on inactive axes)
    int nt;              // tile cells
    int cs0, cs1, cs2;   // cross-section size per axis
    int h1, h2;          // halo block offsets of axes 1 and 2 (axis 0: 0)
    int nslot;
};

__device__ inline int pick3(int a, int x0, int x1, int x2)
{
    return x0 * (a == 0) + x1 * (a == 1) + x2 * (a == 2);
}

__device__ inline TileCtx tile_make(const Film &fm, int dim, int sg0, int sg1, int sg2, int tile, int3 tdim)
{
    TileCtx t;
    const int n0 = fm.n[0], n1 = fm.n[1], n2 = fm.n[2];
    const int nt0 = (n0 + tdim.x - 1) / tdim.x, nt1 = (n1 + tdim.y - 1) / tdim.y;
    const int tc0 = tile % nt0, tc1 = (tile / nt0) % nt1, tc2 = tile / (nt0 * nt1);
    t.sg0 = sg0;
    t.sg1 = sg1;
    t.sg2 = sg2;
    t.o0 = tc0 * tdim.x;
    t.o1 = tc1 * tdim.y;
    t.o2 = tc2 * tdim.z;
    t.e0 = min(tdim.x, n0 - t.o0);
    t.e1 = min(tdim.y, n1 - t.o1);
    t.e2 = min(tdim.z, n2 - t.o2);
    t.nt = t.e0 * t.e1 * t.e2;
    t.cs0 = t.e1 * t.e2;
    t.cs1 = t.e0 * t.e2;
    t.cs2 = t.e0 * t.e1;
    t.h1 = 3 * t.cs0;
    t.h2 = t.h1 + (dim > 1 ? 3 * t.cs1 : 0);
    t.nslot = t.nt + t.h2 + (dim > 2 ? 3 * t.cs2 : 0);
    return t;
}

// slot of flow position (f0, f1, f2) (at most one coordinate outside the
// tile), -1 if none
__device__ inline int tile_slot(const TileCtx t, int f0, int f1, int f2)
{
    const int o0 = f0 < 0 || f0 >= t.e0, o1 = f1 < 0 || f1 >= t.e1, o2 = f2 < 0 || f2 >= t.e2;
    const int nout = o0 + o1 + o2;
    if (nout == 0) return f0 + t.e0 * (f1 + t.e1 * f2);
    if (nout > 1) return -1;
    const int a = o1 + 2 * o2;
    const int fa = pick3(a, f0, f1, f2), ea = pick3(a, t.e0, t.e1, t.e2);
    const int cs = pick3(a, t.cs0, t.cs1, t.cs2), off = pick3(a, 0, t.h1, t.h2);
    const int x = pick3(a, f1 + t.e1 * f2, f0 + t.e0 * f2, f0 + t.e0 * f1);
    if (fa < -2 || fa > ea) return -1;
    const int L = fa < 0 ? fa + 2 : 2;
    return t.nt + off + L * cs + x;
}

// halo axis of slot s (-1 for tile cells) and its offset inside the axis block
__device__ inline int tile_axis(const TileCtx t, int s, int &r)
{
    if (s < t.nt) return -1;
    const int r0 = s - t.nt;
    const int a = (r0 >= t.h1) + (r0 >= t.h2);
    r = r0 - pick3(a, 0, t.h1, t.h2);
    return a;
}

// flow position of slot s; axis of the halo block (-1 for tile cells)
__device__ inline int tile_pos(const TileCtx t, int s, int &f0, int &f1, int &f2)
{
    if (s < t.nt) {
        f0 = s % t.e0;
        f1 = (s / t.e0) % t.e1;
        f2 = s / (t.e0 * t.e1);
        return -1;
    }
    int r;
    const int a = tile_axis(t, s, r);
    const int cs = pick3(a, t.cs0, t.cs1, t.cs2);
    const int L = r / cs, x = r - L * cs;
    const int fa = L < 2 ? L - 2 : pick3(a, t.e0, t.e1, t.e2);
    // the cross-section is indexed by the two other axes in increasing order
    const int eb = a == 0 ? t.e1 : t.e0;
    const int xb = x % eb, xc = x / eb;
    f0 = a == 0 ? fa : xb;
    f1 = a == 1 ? fa : (a == 0 ? xb : xc);
    f2 = a == 2 ? fa : xc;
    return a;
}

// compact index of slot s among the first upwind halo layers (layer 1 of
// every axis), -1 for other slots
__device__ inline int tile_up1(const TileCtx t, int s)
{
    int r;
    const int a = tile_axis(t, s, r);
    if (a < 0) return -1;
    const int cs = pick3(a, t.cs0, t.cs1, t.cs2);
    if (r < cs || r >= 2 * cs) return -1;
    return pick3(a, 0, t.cs0, t.cs0 + t.cs1) + r - cs;
}

// global cell of flow position f and the signed count of periodic crossings;
// returns -1 for walls, pores and positions outside a non-periodic domain
// Whole periods between position i and the cell range [0, n): floor(i / n).
__host__ __device__ inline int periods(int i, int n) { return i >= 0 ? i / n : -((n - 1 - i) / n); }

__device__ inline int tile_cell(const TileCtx t, const Film &fm, const Dev &d, int f0, int f1, int f2, int &jump)
{
    int i0 = t.o0 + (t.sg0 > 0 ? f0 : t.e0 - 1 - f0);
    int i1 = t.o1 + (t.sg1 > 0 ? f1 : t.e1 - 1 - f1);
    int i2 = t.o2 + (t.sg2 > 0 ? f2 : t.e2 - 1 - f2);
    jump = 0;
    const int n0 = fm.n[0], n1 = fm.n[1], n2 = fm.n[2];
    // every crossing of the low face adds +C dT/4pi, of the high face
    // -C dT/4pi (a slot two cells out on an axis of one cell is two periods away)
    if (i0 < 0 || i0 >= n0) {
        if (!fm.periodic[0]) return -1;
        const int w = periods(i0, n0);
        jump -= w;
        i0 -= w * n0;
    }
    if (i1 < 0 || i1 >= n1) {
        if (!fm.periodic[1]) return -1;
        const int w = periods(i1, n1);
        jump -= w;
        i1 -= w * n1;
    }
    if (i2 < 0 || i2 >= n2) {
        if (!fm.periodic[2]) return -1;
        const int w = periods(i2, n2);
        jump -= w;
        i2 -= w * n2;
    }
    const int c = fm.cell0 + i0 + n0 * (i1 + n1 * i2);
    return (d.code[c] & kSolidBit) ? c : -1;
}

// raw global cell of a tile position (no wrap, pores included)
__device__ inline int tile_raw_cell(const TileCtx t, const Film &fm, int f0, int f1, int f2)
{
    const int i0 = t.o0 + (t.sg0 > 0 ? f0 : t.e0 - 1 - f0);
    const int i1 = t.o1 + (t.sg1 > 0 ? f1 : t.e1 - 1 - f1);
    const int i2 = t.o2 + (t.sg2 > 0 ? f2 : t.e2 - 1 - f2);
    return fm.cell0 + i0 + fm.n[0] * (i1 + fm.n[1] * i2);
}

}  // namespace bte
