// bte_adjflux.h -- transposed transport stencil of one tile cell (adjoint).
//
// With the central least-squares slope (no limiter) the steady residual R(e)
// is affine in e, and its Jacobian J = dR/de is fixed by the face
// reconstruction (Sec. 3.3 and 3.5: second-order upwind face values from
// the per-axis least-squares gradient) and by the boundary closures
// (Sec. 2.2).  The adjoint needs (J^T psi) for every (cell, direction, band).
//
// Along one axis, in the flow frame of the lane, the outgoing face value of
// cell k is f(k) = e_k + sigma_k / 2 (sigma_k: central, one-sided or zero
// slope difference, depending on which neighbours exist), and the lane's
// residual gets -cpl (f(i) - f(i-1)) with cpl = v |s_a| / h (or the wall
// value instead of f(i-1)).  Collecting the coefficient of e_j gives
//   (J^T psi)_j = sum_{k = j-1, j, j+1} (df(k)/de_j) mu_k,
//   mu_k = cpl (psi_{k+1} [link k,k+1] - psi_k),
// a stencil with two downstream cells and one upstream cell.  The kernels
// evaluate it in the reversed frame of the lane (tile signs flipped), where
// it has the same shape as the forward stencil (two "upwind" cells, one
// "downwind" cell) and, in the interior, the same coefficients:
//   (J^T psi)_j = cpl [(a1 - c) + ((c - ad) - (a2 - a1)) / 4]
// with c = psi_j, a1, a2 the first and second cells upwind in the reversed
// frame and ad the cell downwind.
//
// Walls.  A specular wall makes the inflow of lane alpha the outgoing face
// value of its mirror lane alpha', so its transpose feeds psi of alpha into
// alpha' at the wall cell (coefficient 3/2 or 1) and at its neighbour
// (coefficient -1/2).  A diffuse wall makes the inflow of every incoming lane
// the w |s.n| weighted mean of the outgoing face values; its transpose feeds
// W = sum_{incoming} cpl psi / sum_{incoming} w |s.n| (k_walls_adj) back into
// every outgoing lane with weight w |s_a|.  Thermalizing walls and periodic
// temperature jumps are constants and drop out.
#pragma once
#include "bte_tilelds.h"

namespace bte {

// General case of one axis: missing neighbours and wall terms.  `sg` is the
// reversed-frame sign of the axis (its upwind side is the lane's downstream side).
template <typename T>
__device__ inline T axis_adj_general(const Dev &d, const TileSmem<T> &S, int i, int a, int m, int s1, int sg,
                                     const T *__restrict__ psi, const double *__restrict__ dinA, int al, int l,
                                     T cpl, T wsa, T c, T a1, T a2, T ad)
{
    const bool hu = m & M_HU, hu2 = m & M_HU2, hd = m & M_HD, hd2 = m & M_HD2;
    // k = j: df(j)/de_j = 1 (central or no slope), 1/2 (one-sided towards the
    // lane's downstream cell), 3/2 (one-sided towards its upstream cell)
    const T cjj = hu ? (hd ? (T)1 : (T)0.5) : (hd ? (T)1.5 : (T)1);
    T tx = cjj * (hu ? a1 - c : -c);
    // k = lane-upstream cell (ad): its slope reaches e_j with 1/4 (central) or 1/2
    if (hd) tx += (hd2 ? (T)0.25 : (T)0.5) * (c - ad);
    // k = lane-downstream cell (a1): its slope reaches e_j with -1/4 or -1/2
    if (hu) tx += hu2 ? (T)-0.25 * (a2 - a1) : (T)0.5 * a1;
    T out = cpl * tx;
    if (!hu) {
        // wall on the lane's downstream side of this cell
        const int kind = (m >> M_KSHIFT) & 3;
        const T cw = hd ? (T)1.5 : (T)1;
        const int cc = S.cell[i];
        if (kind == 1) {
            const int km = d.mirror[a * d.na + al] * d.nl + l;
            out += cpl * cw * psi[(size_t)cc * d.nk + km];
        } else if (kind == 2) {
            const int rec = diffuse_index(d, cc, S.code[i], face_of(a, -sg));
            out += wsa * cw * (T)dinA[(size_t)rec * d.nl + l];
        }
    } else if (!hu2) {
        // wall on the lane's downstream side of the downstream cell
        const int kind2 = (m >> M_K2SHIFT) & 3;
        if (kind2 != 0) {
            const int c1 = (int)(S.slot_off[s1] / d.nk);
            if (kind2 == 1) {
                const int km = d.mirror[a * d.na + al] * d.nl + l;
                out -= (T)0.5 * cpl * psi[(size_t)c1 * d.nk + km];
            } else {
                const int rec = diffuse_index(d, c1, d.code[c1], face_of(a, -sg));
                out -= (T)0.5 * wsa * (T)dinA[(size_t)rec * d.nl + l];
            }
        }
    }
    return out;
}

// Transport part of (J^T psi) at tile cell i for one lane (reversed frame).
// up_out[a]: compact dup index of an implicitly coupled upwind neighbour
// outside the tile (sweep), or -1.
template <typename T, int DIM>
__device__ inline T tile_flux_adj(const Dev &d, const TileCtx t, const TileSmem<T> &S, int i, const LaneT<T> &L,
                                  const T (&wsa)[3], int lane, const T *__restrict__ psi,
                                  const double *__restrict__ dinA, int up_out[3])
{
    const T c = S.box[i * 64 + lane];
    T out = (T)0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int m = uni(S.mode[3 * i + a]);
        const int s1 = uni(S.stn[9 * i + 3 * a]), s2 = uni(S.stn[9 * i + 3 * a + 1]),
                  sd = uni(S.stn[9 * i + 3 * a + 2]);
        const T a1 = S.box[s1 * 64 + lane];
        const T a2 = (m & M_HU2) ? S.box[s2 * 64 + lane] : (T)0;
        const T ad = S.box[sd * 64 + lane];
        if ((m & (M_HU | M_HU2 | M_HD | M_HD2)) == (M_HU | M_HU2 | M_HD | M_HD2)) {
            out += L.cpl[a] * ((a1 - c) + (T)0.25 * ((c - ad) - (a2 - a1)));
        } else {
            const int sg = a == 0 ? t.sg0 : (a == 1 ? t.sg1 : t.sg2);
            out += axis_adj_general<T>(d, S, i, a, m, s1, sg, psi, dinA, L.al, L.l, L.cpl[a], wsa[a], c, a1, a2, ad);
        }
        up_out[a] = ((m & M_HU) && !(m & M_WRAP) && s1 >= t.nt) ? S.slot_up1[s1] : -1;
    }
    return out;
}

}  // namespace bte
