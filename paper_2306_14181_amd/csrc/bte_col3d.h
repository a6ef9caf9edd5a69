// bte_col3d.h -- helpers of the column-walk kernels on three-dimensional
// geometries (explicit step, its transpose, the steady sweep): periodic
// positions, the general-path face-value difference of one axis (walls,
// missing neighbours) and its transpose.
#pragma once
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tilelds.h"

namespace bte {

__device__ inline double rl_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Position i along an axis of n cells: itself inside, the periodic image
// outside (jump +1 per crossing of the low face, -1 per crossing of the high
// face, in units of C dT / 4pi), -1 outside a non-periodic domain.
__device__ inline int wrap_pos(int i, int n, int per, int &jump)
{
    jump = 0;
    if (i >= 0 && i < n) return i;
    if (!per) return -1;
    const int w = periods(i, n);
    jump = -w;
    return i - w * n;
}

// Face-value difference of one axis on the general path (missing
// neighbours, walls): outgoing face value minus incoming face value, the
// incoming one from the upwind cell or from the wall (thermalizing,
// specular: the mirror direction's outgoing value, diffuse: the wall record).
// xc, xd: additive terms of the mirror lane's values at the cell and at its
// downwind neighbour cd (pending correction, periodic jump).
template <typename T, int LIM>
__device__ inline T delta_wall3(const Dev &d, const Film &fm, const T *__restrict__ e, const double *__restrict__ din,
                                int c, uint32_t code, int a, int sg, bool hu, bool hu2, bool hd, T e2, T e1, T ec,
                                T ed, int cd, T xd, int al, int l, T C4, T hh, T ih, T xc = (T)0)
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
            const T em = e[(size_t)c * d.nk + km] + xc;
            T gm = (T)0;
            if (LIM == LIM_NONE && hd) gm = (em - (e[(size_t)cd * d.nk + km] + xd)) * ih;
            fin = em + hh * gm;
        } else {
            const int rec = diffuse_index(d, c, code, face_of(a, su));
            fin = (T)din[(size_t)rec * d.nl + l];
        }
    }
    return fout - fin;
}


// One axis of (J^T lam) on the general path (missing neighbours, walls).
template <typename T>
__device__ inline T adj_axis3(const Dev &d, const T *__restrict__ lam, const double *__restrict__ dinA, int c,
                              uint32_t code, int c1, uint32_t code1, int a, int sg, bool hu, bool hu2, bool hd,
                              bool hd2, T lc, T a1, T a2, T ad, int al, int l, T cpl, T wsa)
{
    const T cjj = hu ? (hd ? (T)1 : (T)0.5) : (hd ? (T)1.5 : (T)1);
    T tx = cjj * (hu ? a1 - lc : -lc);
    if (hd) tx += (hd2 ? (T)0.25 : (T)0.5) * (lc - ad);
    if (hu) tx += hu2 ? (T)-0.25 * (a2 - a1) : (T)0.5 * a1;
    T out = cpl * tx;
    if (!hu) {
        // wall on the frame's upwind side of this cell
        const int kind = side_wall(axis_bits(code, a), -sg);
        const T cw = hd ? (T)1.5 : (T)1;
        if (kind == 1) {
            const int km = d.mirror[a * d.na + al] * d.nl + l;
            out += cpl * cw * lam[(size_t)c * d.nk + km];
        } else if (kind == 2) {
            const int rec = diffuse_index(d, c, code, face_of(a, -sg));
            out += wsa * cw * (T)dinA[(size_t)rec * d.nl + l];
        }
    } else if (!hu2 && c1 >= 0) {
        // wall on the frame's upwind side of the upwind cell
        const int kind2 = side_wall(axis_bits(code1, a), -sg);
        if (kind2 == 1) {
            const int km = d.mirror[a * d.na + al] * d.nl + l;
            out -= (T)0.5 * cpl * lam[(size_t)c1 * d.nk + km];
        } else if (kind2 == 2) {
            const int rec = diffuse_index(d, c1, code1, face_of(a, -sg));
            out -= (T)0.5 * wsa * (T)dinA[(size_t)rec * d.nl + l];
        }
    }
    return out;
}

}  // namespace bte
