// bte_stencil.h -- per-element discrete operators of the phonon BTE on a
// structured grid, evaluated by one thread for one (cell, direction, band).
//
// Face reconstruction (Sec. 3.3): the face value is taken from the upwind
// cell m as e_m + grad e_m . l_{m,f}.  On a Cartesian grid the least-squares
// gradient (Sec. 3.5, X^{-1} y over the face neighbours) decouples per axis:
// a central difference with both neighbours, one-sided with one, zero with
// none.  Optional MC / minmod limiters (zero slope next to a wall) replace it.
// Everything is written in "flow coordinates" along each axis: the upwind
// side is -sign(s_a), so the stencil of a cell is (u2, u1, c, d1).
#pragma once
#include "bte_internal.h"

namespace bte {

enum { LIM_NONE = 0, LIM_MC = 1, LIM_MINMOD = 2 };

// Constants of one (direction, band) lane.
struct LaneConst {
    int k, al, l;
    double w, s[3], v, C4, itau;
};

// Constants of lane k (direction, band) for the material whose band tables
// start at moff.
__device__ inline LaneConst lane_const(const Dev &d, int k, int moff)
{
    LaneConst c;
    c.k = k;
    c.al = k / d.nl;
    c.l = k - c.al * d.nl;
    c.w = d.w[c.al];
    c.s[0] = d.s[3 * c.al + 0];
    c.s[1] = d.s[3 * c.al + 1];
    c.s[2] = d.s[3 * c.al + 2];
    c.v = d.v[moff + c.l];
    c.C4 = d.C4[moff + c.l];
    c.itau = d.itau[moff + c.l];
    return c;
}

// Energy deviation of element (j, k) including the pending isotropic
// correction C delta_j / 4pi of the synthetic scheme (dpend may be null).
template <typename T>
__device__ inline T ld_e(const T *__restrict__ e, const double *__restrict__ dpend, const Dev &d, int j,
                         int k, T C4)
{
    T x = e[(size_t)j * d.nk + k];
    if (dpend) x += C4 * (T)dpend[j];
    return x;
}

// Slope along the flow direction (units of e per metre).
template <typename T>
__device__ inline T slope_flow(int lim, bool hu, bool hd, T eu, T ec, T ed, T ih)
{
    if (lim == LIM_NONE) {
        if (hu && hd) return (T)0.5 * (ed - eu) * ih;
        if (hd) return (ed - ec) * ih;
        if (hu) return (ec - eu) * ih;
        return (T)0;
    }
    if (!(hu && hd)) return (T)0;
    T dl = (ec - eu) * ih, dr = (ed - ec) * ih;
    if (dl * dr <= (T)0) return (T)0;
    T adl = fabs(dl), adr = fabs(dr);
    T m = (lim == LIM_MC) ? fmin(fmin((T)2 * adl, (T)2 * adr), (T)0.5 * fabs(dl + dr)) : fmin(adl, adr);
    return dl > (T)0 ? m : -m;
}

// Index of the diffuse-wall record of face f of cell c: records are numbered
// cell by cell in face order -x,+x,-y,+y,-z,+z.
__device__ inline int diffuse_index(const Dev &d, int c, uint32_t code, int f)
{
    int idx = d.dbase[c];
    for (int g = 0; g < f; ++g) {
        int a = g >> 1, side = (g & 1) ? 1 : -1;
        uint32_t ab = axis_bits(code, a);
        if (a < d.dim && !side_is_cell(ab, side) && side_record(ab, side)) ++idx;
    }
    return idx;
}

// Result of evaluating the stencil of one element.
template <typename T>
struct StencilOut {
    T D;             // (1/V) sum_f e_f v s.n S   (flux divergence)
    T cup[3];        // coupling |v s_a|/h_a of the implicit first-order operator
    int jup[3];      // upwind neighbour coupled implicitly (-1: wall or periodic)
    T eup[3];        // its corrected energy deviation (no periodic jump)
};

// Flux divergence of element (c, lane) from e (plus pending correction),
// with boundary inflow from the same field (thermalizing: C (T_w - T_ref)/4pi,
// specular: mirror direction's outgoing face value, diffuse: din record,
// periodic: neighbour across the face plus the temperature jump).
template <typename T>
__device__ inline StencilOut<T> stencil(const T *__restrict__ e, const double *__restrict__ dpend,
                                        const double *__restrict__ din, const Dev &d, const Film &fm, int c,
                                        uint32_t code, const LaneConst &L, T ec)
{
    StencilOut<T> o;
    o.D = (T)0;
    const T C4 = (T)L.C4;
    for (int a = 0; a < 3; ++a) {
        o.cup[a] = (T)0;
        o.jup[a] = -1;
        o.eup[a] = (T)0;
    }
    for (int a = 0; a < d.dim; ++a) {
        const double sa = L.s[a];
        const int sg = sa > 0 ? 1 : -1;
        const int su = -sg, sd = sg;
        const T ih = (T)fm.ih[a], hh = (T)(0.5 * fm.h[a]);
        const T J = C4 * (T)fm.pdT[a];
        const uint32_t ab = axis_bits(code, a);
        const bool hu = side_is_cell(ab, su), hd = side_is_cell(ab, sd);
        T eu1 = (T)0, eu2 = (T)0, ed1 = (T)0;
        bool hu2 = false;
        int j1 = -1, jd = -1;
        T jump1 = (T)0;
        if (hu) {
            j1 = d.nb[face_of(a, su) * d.nc + c];
            jump1 = side_wraps(ab, su) ? (T)sg * J : (T)0;
            T raw1 = ld_e(e, dpend, d, j1, L.k, C4);
            eu1 = raw1 + jump1;
            const uint32_t ab1 = axis_bits(d.code[j1], a);
            hu2 = side_is_cell(ab1, su);
            if (hu2) {
                int j2 = d.nb[face_of(a, su) * d.nc + j1];
                T jump2 = side_wraps(ab1, su) ? (T)sg * J : (T)0;
                eu2 = ld_e(e, dpend, d, j2, L.k, C4) + jump1 + jump2;
            }
            if (!side_wraps(ab, su)) {
                o.jup[a] = j1;
                o.eup[a] = raw1;
            }
        }
        if (hd) {
            jd = d.nb[face_of(a, sd) * d.nc + c];
            ed1 = ld_e(e, dpend, d, jd, L.k, C4) + (side_wraps(ab, sd) ? -(T)sg * J : (T)0);
        }
        const T gc = slope_flow<T>(d.limiter, hu, hd, eu1, ec, ed1, ih);
        const T fout = ec + hh * gc;
        T fin;
        if (hu) {
            const T g1 = slope_flow<T>(d.limiter, hu2, true, eu2, eu1, ec, ih);
            fin = eu1 + hh * g1;
        } else {
            const int kind = side_wall(ab, su);
            if (kind == 0) {
                const double Tw = side_outer(code, a, su) ? fm.wallT[face_of(a, su)] : d.poreT;
                fin = C4 * (T)Tw;
            } else if (kind == 1) {
                // specular: outgoing face value of the mirror direction, whose
                // upwind side is our downwind side
                const int km = d.mirror[a * d.na + L.al] * d.nl + L.l;
                const T em = ld_e(e, dpend, d, c, km, C4);
                T gm = (T)0;
                if (d.limiter == LIM_NONE && hd) {
                    const T edm = ld_e(e, dpend, d, jd, km, C4) + (side_wraps(ab, sd) ? -(T)sg * J : (T)0);
                    gm = (em - edm) * ih;
                }
                fin = em + hh * gm;
            } else {
                const int rec = diffuse_index(d, c, code, face_of(a, su));
                fin = (T)din[(size_t)rec * d.nl + L.l];
            }
        }
        const T cpl = (T)(L.v * fabs(sa)) * ih;
        o.D += cpl * (fout - fin);
        o.cup[a] = cpl;
    }
    return o;
}

}  // namespace bte
