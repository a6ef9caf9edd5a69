// bte_sweep3d.hip -- steady transport sweep (the source iteration of
// Algorithm 1 in delta form, Sec. 3.3-3.5: right-hand side eq. B_BTE, the
// first-order upwind operator of eq. "Linear system") on three-dimensional
// geometries, and its transpose for the adjoint.
//
// Work item: a segment of zseg cells of one (x, y) column, for 64
// (direction, band) lanes of one octant; one wavefront per item, four
// independent wavefronts per block.  The wavefront walks its segment along z
// in the flow direction of the octant: the z stencil (two upwind cells, the
// cell, the downwind cell) is a window of registers that shifts by one load
// per cell, the increment of the z-upwind cell is the previous cell's, and
// the upwind recurrence of the cell is solved right after its right-hand
// side, in registers.  The x / y neighbours are read from memory together
// with the increments e^{n+1} - e^n of the x- and y-upwind cells, which
// belong to segments of earlier launches: the segments are launched by
// hyperplanes fx + fy + fz (flow coordinates of the column and of the
// segment), so every upwind segment is complete when a segment starts.
// Per-cell values (geometry codes, T_L, scattering rate, source, pending
// synthetic correction of the cell and of its x / y neighbours) are loaded
// one cell per lane for the segment and broadcast with readlane.  FP64
// moment partials of eight cells at a time are reduced transposed through
// LDS (lane = 8 cell + part) and written per (octant, chunk, cell).
//
// ADJ: the transposed sweep of the adjoint iteration.  The item's octant
// fixes the frame and the hyperplane order; the lanes are those of the
// opposite octant, so the frame is the lanes' reversed flow, the transposed
// stencil has the forward shape and the recurrence solves A^T.  The
// right-hand side is (J^T psi + g) - psi/tau + w X/tau (X: isotropic closure
// term), and the moment partial is sum C/(4 pi) (1/tau) psi^{n+1}.
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tilelds.h"
#include "bte_col3d.h"

namespace bte {

namespace {

// per-cell mode word of the segment records
enum : uint32_t {
    S3_SOLID = 1u,   // solid cell
    S3_FAST = 2u,    // interior stencil on every axis
    S3_CX = 4u,      // implicit coupling to the upwind cell along x (solid, not across a periodic face)
    S3_CY = 8u,
    S3_CZ = 16u
};

__device__ inline float rl_f(float v, int q) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q)); }

template <typename T> __device__ inline T rl_t(T v, int q)
{
    if constexpr (sizeof(T) == 4) return rl_f(v, q);
    else return rl_d(v, q);
}

}  // namespace

// ADD: the stencil values carry additive terms (pending correction of the
// synthetic scheme, periodic temperature jumps); false: plain values.
template <typename T, int LIM, bool ADJ, bool ADD>
__global__ __launch_bounds__(256) void k_sweep3d(Dev d, const T *__restrict__ ein, T *__restrict__ eout,
                                                 const double *__restrict__ dpend, const double *__restrict__ TLdev,
                                                 const double *__restrict__ din, const SweepItem *__restrict__ items,
                                                 int item0, int count, int zseg, int na_oct, int nchunk_oct,
                                                 double *__restrict__ part)
{
    constexpr int NM = ADJ ? 2 : kMomN;
    __shared__ double lcs[4][64][NM];   // per-lane moment constants of each wavefront
    __shared__ T xs[4][8][64];          // new values of eight cells of each wavefront
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * 4 + wv;
    if (idx >= count) return;
    const SweepItem it = items[item0 + idx];
    if (!ADJ && d.nfilm > 1 && d.fdone[it.film]) return;   // converged geometry of a batch
    const Film &fm = d.film[it.film];
    const int n0 = fm.n[0], n1 = fm.n[1], n2 = fm.n[2], plane = n0 * n1;
    const int col = it.tile % plane, tz = it.tile / plane;
    const int x = col % n0, y = col / n0;
    const int sg0 = octant_sign(d, it.oct, na_oct, 0), sg1 = octant_sign(d, it.oct, na_oct, 1),
              sg2 = octant_sign(d, it.oct, na_oct, 2);
    // the segment in flow order along z: flow index f is geometric z = f
    // (sg2 > 0) or n2 - 1 - f
    const int gz0 = tz * zseg, gz1 = min(gz0 + zseg, n2);
    const int fb = sg2 > 0 ? gz0 : n2 - gz1, fe = sg2 > 0 ? gz1 : n2 - gz0;
    const int nl = d.nl, nk = d.nk, nc = d.nc;
    const int loct = ADJ ? (it.oct ^ 7) : it.oct;
    const int kbeg = loct * na_oct * nl, kend = kbeg + na_oct * nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const int kk = active ? k : kbeg;
    const LaneT<T> L = lane_make<T>(d, fm, kk);
    const T C4 = L.C4;
    {
        double cst[NM];
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
        for (int m = 0; m < NM; ++m) lcs[wv][lane][m] = active ? cst[m] : 0.0;
    }
    T wsa[3] = {(T)0, (T)0, (T)0};
    T gl = (T)0;
    if constexpr (ADJ) {
#pragma unroll
        for (int a = 0; a < 3; ++a) wsa[a] = (T)(L.w * fabs(d.s[3 * L.al + a]));
        // objective k_eff along x: g = (L_x / (dT_x N_cells)) w v s_x
        gl = fm.pdT[0] != 0.0 ? (T)(fm.len[0] / (fm.pdT[0] * fm.ncell) * L.wv[0]) : (T)0;
    }

    const int cb = fm.cell0 + x + n0 * y;   // cell of (x, y, 0)
    int jx1, jx2, jxd, jy1, jy2, jyd;
    const int px1 = wrap_pos(x - sg0, n0, fm.periodic[0], jx1), px2 = wrap_pos(x - 2 * sg0, n0, fm.periodic[0], jx2),
              pxd = wrap_pos(x + sg0, n0, fm.periodic[0], jxd);
    const int py1 = wrap_pos(y - sg1, n1, fm.periodic[1], jy1), py2 = wrap_pos(y - 2 * sg1, n1, fm.periodic[1], jy2),
              pyd = wrap_pos(y + sg1, n1, fm.periodic[1], jyd);
    const int bx1 = px1 >= 0 ? fm.cell0 + px1 + n0 * y : -1, bx2 = px2 >= 0 ? fm.cell0 + px2 + n0 * y : -1,
              bxd = pxd >= 0 ? fm.cell0 + pxd + n0 * y : -1;
    const int by1 = py1 >= 0 ? fm.cell0 + x + n0 * py1 : -1, by2 = py2 >= 0 ? fm.cell0 + x + n0 * py2 : -1,
              byd = pyd >= 0 ? fm.cell0 + x + n0 * pyd : -1;
    // cell of the column at flow index f (periodic image outside the
    // column, -1 outside a non-periodic column) and its jump in C dT / 4pi
    auto zcell = [&](int f, int &jz) -> int {
        const int zg = wrap_pos(sg2 > 0 ? f : n2 - 1 - f, n2, fm.periodic[2], jz);
        return zg >= 0 ? cb + plane * zg : -1;
    };
    auto plus = [](int base, int off) { return base >= 0 ? base + off : -1; };
    const T *zrow = static_cast<const T *>(d.zrow);
    const double *zd = static_cast<const double *>(d.zrow);
    const unsigned koff = (unsigned)kk * (unsigned)sizeof(T);
    auto at = [&](const T *row) -> T { return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + koff); };

    // ---- records of the segment, one flow position per lane: lane q holds
    // flow index fb - 2 + q (the window reaches two cells before the
    // segment and two after it; zseg <= 48 keeps that within 64 lanes)
    uint32_t r_code = 0, r_cxu = 0, r_cyu = 0, r_czu = 0, r_cxd = 0, r_cyd = 0, r_czd = 0, r_mode = 0;
    double r_gam = 0.0;
    T r_tl = (T)0, r_qs = (T)0, r_az = (T)0;
    T r_ax1 = (T)0, r_ax2 = (T)0, r_axd = (T)0, r_ay1 = (T)0, r_ay2 = (T)0, r_ayd = (T)0;
    {
        const int fr = fb - 2 + lane;
        const int fcl = min(max(fr, 0), n2 - 1);
        const int zo = plane * (sg2 > 0 ? fcl : n2 - 1 - fcl);
        const int c = cb + zo;
        r_code = d.code[c];
        {
            const uint32_t cxu = d.code[bx1 >= 0 ? bx1 + zo : c], cyu = d.code[by1 >= 0 ? by1 + zo : c];
            r_cxu = bx1 >= 0 ? cxu : 0u;
            r_cyu = by1 >= 0 ? cyu : 0u;
            int jz;
            const int cu = zcell(fcl - 1, jz);
            const uint32_t v = d.code[cu >= 0 ? cu : c];
            r_czu = cu >= 0 ? v : 0u;
            if constexpr (ADJ) {
                const uint32_t cxd = d.code[bxd >= 0 ? bxd + zo : c], cyd = d.code[byd >= 0 ? byd + zo : c];
                r_cxd = bxd >= 0 ? cxd : 0u;
                r_cyd = byd >= 0 ? cyd : 0u;
                const int cdz = zcell(fcl + 1, jz);
                const uint32_t w = d.code[cdz >= 0 ? cdz : c];
                r_czd = cdz >= 0 ? w : 0u;
            }
        }
        r_gam = d.gamma[c];
        r_tl = (T)TLdev[c];   // ADJ: the isotropic closure term X
        if constexpr (!ADJ) r_qs = (T)(*(d.P ? d.P + c : zd) / fm.Ctot);   // P is null without a heat source
        if constexpr (ADD) {
            // additive terms (units of C/4pi): pending correction plus the
            // periodic jump of the value as seen from this column
            auto dp = [&](int cell) -> double { return dpend ? dpend[cell] : 0.0; };
            int jz;
            const int cz = zcell(fr, jz);
            r_az = cz >= 0 ? (T)(dp(cz) + jz * fm.pdT[2]) : (T)0;
            r_ax1 = bx1 >= 0 ? (T)(dp(bx1 + zo) + jx1 * fm.pdT[0]) : (T)0;
            r_ax2 = bx2 >= 0 ? (T)(dp(bx2 + zo) + jx2 * fm.pdT[0]) : (T)0;
            r_axd = bxd >= 0 ? (T)(dp(bxd + zo) + jxd * fm.pdT[0]) : (T)0;
            r_ay1 = by1 >= 0 ? (T)(dp(by1 + zo) + jy1 * fm.pdT[1]) : (T)0;
            r_ay2 = by2 >= 0 ? (T)(dp(by2 + zo) + jy2 * fm.pdT[1]) : (T)0;
            r_ayd = byd >= 0 ? (T)(dp(byd + zo) + jyd * fm.pdT[1]) : (T)0;
        }
        const uint32_t ab0 = axis_bits(r_code, 0), ab1 = axis_bits(r_code, 1), ab2 = axis_bits(r_code, 2);
        const bool hu0 = side_is_cell(ab0, -sg0), hu1 = side_is_cell(ab1, -sg1), hu2 = side_is_cell(ab2, -sg2);
        const bool hd0 = side_is_cell(ab0, sg0), hd1 = side_is_cell(ab1, sg1), hd2 = side_is_cell(ab2, sg2);
        bool fast = hu0 && hd0 && side_is_cell(axis_bits(r_cxu, 0), -sg0) && hu1 && hd1 &&
                    side_is_cell(axis_bits(r_cyu, 1), -sg1) && hu2 && hd2 && side_is_cell(axis_bits(r_czu, 2), -sg2);
        if constexpr (ADJ)
            fast = fast && side_is_cell(axis_bits(r_cxd, 0), sg0) && side_is_cell(axis_bits(r_cyd, 1), sg1) &&
                   side_is_cell(axis_bits(r_czd, 2), sg2);
        uint32_t m = (r_code & kSolidBit) ? S3_SOLID : 0u;
        if (m && fast) m |= S3_FAST;
        if (m && hu0 && !side_wraps(ab0, -sg0)) m |= S3_CX;
        if (m && hu1 && !side_wraps(ab1, -sg1)) m |= S3_CY;
        if (m && hu2 && !side_wraps(ab2, -sg2)) m |= S3_CZ;
        r_mode = m;
    }
    auto rlu = [&](uint32_t v, int q) -> uint32_t { return (uint32_t)__builtin_amdgcn_readlane((int)v, q); };

    // ---- stencil rows.  The x / y neighbour rows (and the new values of the
    // x- and y-upwind cells) and the column's own rows are addressed from
    // one base per buffer (the lowest of the rows involved, one plane below
    // the segment's lowest plane where there is one) by 32-bit byte offsets
    // that move one plane per cell; an absent neighbour points at the
    // column's own row (its value is never used: the mode bits say it is
    // absent), so every offset moves by the same step.
    const int own = cb;
    auto pick = [&](int b) { return b >= 0 ? b : own; };
    const int cx1 = pick(bx1), cx2 = pick(bx2), cxd = pick(bxd), cy1 = pick(by1), cy2 = pick(by2), cyd = pick(byd);
    const int cmin = min(min(min(cx1, cx2), min(cxd, cy1)), min(min(cy2, cyd), own));
    const size_t rowb = (size_t)nk * sizeof(T);
    const int zbase = gz0 > 0 ? gz0 - 1 : 0;
    const size_t basecell = (size_t)cmin + (size_t)plane * zbase;
    const char *eb = reinterpret_cast<const char *>(ein) + basecell * rowb;
    char *ob = reinterpret_cast<char *>(eout) + basecell * rowb;
    const int zgb = sg2 > 0 ? fb : n2 - 1 - fb;
    const unsigned zb0 = (unsigned)((size_t)(zgb - zbase) * plane * rowb);
    const int zstepb = (sg2 > 0 ? 1 : -1) * (int)((size_t)plane * rowb);
    auto off0 = [&](int c) -> unsigned { return (unsigned)((size_t)(c - cmin) * rowb) + zb0 + koff; };
    unsigned vx1 = off0(cx1), vx2 = off0(cx2), vxd = off0(cxd), vy1 = off0(cy1), vy2 = off0(cy2), vyd = off0(cyd);
    // the column's own row at the cell being swept, and at the flow index
    // the next z value is prefetched from (inside the column, up to flow
    // index fe, one past the segment: at most one plane below the segment's
    // lowest or above its highest plane)
    unsigned vc = off0(own), vzn = off0(own) + (unsigned)zstepb;
    auto atb = [&](const char *b, unsigned o) -> T { return *reinterpret_cast<const T *>(b + o); };
    auto zraw = [&](int f) -> T {
        int jz;
        const int c = zcell(f, jz);
        return at(c >= 0 ? ein + (size_t)c * nk : zrow);
    };
    // corrected value of the column at flow index f (record lane f - fb + 2)
    auto zval = [&](int f, T raw) -> T {
        if constexpr (ADD) return raw + C4 * rl_t(r_az, f - fb + 2);
        else return raw;
    };

    struct Pre {
        T nz, x1, x2, xd, y1, y2, yd, ux, uy;
    };
    // loads of cell fn (x / y neighbours, new values of the x- / y-upwind
    // cells) and the raw column value at fn + 1 (by the running offset
    // inside the column, past its end the periodic image or zero); the x / y
    // offsets stop at the segment's last cell
    auto prefetch = [&](int fn, Pre &q) {
        q.x1 = atb(eb, vx1);
        q.x2 = atb(eb, vx2);
        q.xd = atb(eb, vxd);
        q.y1 = atb(eb, vy1);
        q.y2 = atb(eb, vy2);
        q.yd = atb(eb, vyd);
        q.ux = atb(ob, vx1);
        q.uy = atb(ob, vy1);
        if (fn < fe) {
            q.nz = fn + 1 < n2 ? atb(eb, vzn) : zraw(fn + 1);
            vzn += (unsigned)zstepb;
        } else {
            q.nz = (T)0;   // past the segment: never used
        }
        if (fn + 1 < fe) {
            vx1 += zstepb;
            vx2 += zstepb;
            vxd += zstepb;
            vy1 += zstepb;
            vy2 += zstepb;
            vyd += zstepb;
        }
    };

    // z window (corrected) and the increment of the z-upwind cell: inside the
    // column it is the last cell of the previous segment (an earlier launch)
    T ez2 = zval(fb - 2, zraw(fb - 2)), ez1 = zval(fb - 1, zraw(fb - 1)), ec = zval(fb, zraw(fb));
    T dzu = (T)0;
    if (fb > 0) {
        int jz;
        const int cu = zcell(fb - 1, jz);
        dzu = at(eout + (size_t)cu * nk) - ez1;
    }
    T lz_up = (LIM == LIM_NONE) ? (T)0 : lim_diff<T, LIM>(ez1 - ez2, ec - ez1);
    const T itau = L.itau;
    const T cp0 = L.cpl[0], cp1 = L.cpl[1], cp2 = L.cpl[2];
    const T A0 = cp0 + cp1 + cp2 + itau;
    const int pidx = it.oct * nchunk_oct + it.chunk;

    auto step = [&](int f, const Pre &in, Pre &out) {
        prefetch(f + 1, out);
        const int q = f - fb + 2;
        const int zo = plane * (sg2 > 0 ? f : n2 - 1 - f);
        const int c = cb + zo;
        const uint32_t mode = rlu(r_mode, q);
        const T ezd = zval(f + 1, in.nz);
        // limited z slope of this cell (also the upwind slope of the next cell)
        const T lz = (LIM == LIM_NONE) ? (T)0 : lim_diff<T, LIM>(ec - ez1, ezd - ec);
        T en = ec, de = (T)0;
        if (mode & S3_SOLID) {
            T ex1 = in.x1, ex2 = in.x2, exd = in.xd, ey1 = in.y1, ey2 = in.y2, eyd = in.yd;
            if constexpr (ADD) {
                ex1 += C4 * rl_t(r_ax1, q);
                ex2 += C4 * rl_t(r_ax2, q);
                exd += C4 * rl_t(r_axd, q);
                ey1 += C4 * rl_t(r_ay1, q);
                ey2 += C4 * rl_t(r_ay2, q);
                eyd += C4 * rl_t(r_ayd, q);
            }
            const T gam = rl_t((T)r_gam, q);
            const T itc = itau + gam;
            T b;
            if constexpr (!ADJ) {
                T dx, dy, dz;
                if (mode & S3_FAST) {
                    dx = delta_fast<T, LIM>(ex2, ex1, ec, exd);
                    dy = delta_fast<T, LIM>(ey2, ey1, ec, eyd);
                    if (LIM == LIM_NONE) dz = delta_fast<T, LIM>(ez2, ez1, ec, ezd);
                    else dz = (ec - ez1) + (T)0.5 * (lz - lz_up);
                } else {
                    const uint32_t code = rlu(r_code, q);
                    const uint32_t cxu = rlu(r_cxu, q), cyu = rlu(r_cyu, q), czu = rlu(r_czu, q);
                    const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1), ab2 = axis_bits(code, 2);
                    const bool hu0 = side_is_cell(ab0, -sg0), hd0 = side_is_cell(ab0, sg0);
                    const bool hu1 = side_is_cell(ab1, -sg1), hd1 = side_is_cell(ab1, sg1);
                    const bool hu2 = side_is_cell(ab2, -sg2), hd2 = side_is_cell(ab2, sg2);
                    const bool hu20 = hu0 && side_is_cell(axis_bits(cxu, 0), -sg0);
                    const bool hu21 = hu1 && side_is_cell(axis_bits(cyu, 1), -sg1);
                    const bool hu22 = hu2 && side_is_cell(axis_bits(czu, 2), -sg2);
                    const T xc = ADD ? C4 * rl_t(r_az, q) : (T)0;
                    if (hu0 && hu20 && hd0) dx = delta_fast<T, LIM>(ex2, ex1, ec, exd);
                    else
                        dx = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 0, sg0, hu0, hu20, hd0, ex2, ex1, ec, exd,
                                                 plus(bxd, zo), ADD ? C4 * rl_t(r_axd, q) : (T)0, L.al, L.l, C4,
                                                 L.hh[0], L.ih[0], xc);
                    if (hu1 && hu21 && hd1) dy = delta_fast<T, LIM>(ey2, ey1, ec, eyd);
                    else
                        dy = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 1, sg1, hu1, hu21, hd1, ey2, ey1, ec, eyd,
                                                 plus(byd, zo), ADD ? C4 * rl_t(r_ayd, q) : (T)0, L.al, L.l, C4,
                                                 L.hh[1], L.ih[1], xc);
                    if (hu2 && hu22 && hd2) {
                        if (LIM == LIM_NONE) dz = delta_fast<T, LIM>(ez2, ez1, ec, ezd);
                        else dz = (ec - ez1) + (T)0.5 * (lz - lz_up);
                    } else {
                        int jd;
                        const int cdz = zcell(f + 1, jd);
                        dz = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 2, sg2, hu2, hu22, hd2, ez2, ez1, ec, ezd,
                                                 cdz, ADD ? C4 * rl_t(r_az, q + 1) : (T)0, L.al, L.l, C4, L.hh[2],
                                                 L.ih[2], xc);
                    }
                }
                const T D = cp0 * dx + cp1 * dy + cp2 * dz;
                b = -D - (ec - C4 * rl_t(r_tl, q)) * itc + C4 * rl_t(r_qs, q);
            } else {
                T tf;
                if (mode & S3_FAST) {
                    const T tx = cp0 * ((ex1 - ec) + (T)0.25 * ((ec - exd) - (ex2 - ex1)));
                    const T ty = cp1 * ((ey1 - ec) + (T)0.25 * ((ec - eyd) - (ey2 - ey1)));
                    const T tzv = cp2 * ((ez1 - ec) + (T)0.25 * ((ec - ezd) - (ez2 - ez1)));
                    tf = (tx + ty) + tzv;
                } else {
                    const uint32_t code = rlu(r_code, q);
                    const uint32_t cxu = rlu(r_cxu, q), cyu = rlu(r_cyu, q), czu = rlu(r_czu, q);
                    const uint32_t cxd = rlu(r_cxd, q), cyd = rlu(r_cyd, q), czd = rlu(r_czd, q);
                    const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1), ab2 = axis_bits(code, 2);
                    const bool hu0 = side_is_cell(ab0, -sg0), hd0 = side_is_cell(ab0, sg0);
                    const bool hu1 = side_is_cell(ab1, -sg1), hd1 = side_is_cell(ab1, sg1);
                    const bool hu2 = side_is_cell(ab2, -sg2), hd2 = side_is_cell(ab2, sg2);
                    const bool hu20 = hu0 && side_is_cell(axis_bits(cxu, 0), -sg0);
                    const bool hu21 = hu1 && side_is_cell(axis_bits(cyu, 1), -sg1);
                    const bool hu22 = hu2 && side_is_cell(axis_bits(czu, 2), -sg2);
                    const bool hd20 = hd0 && side_is_cell(axis_bits(cxd, 0), sg0);
                    const bool hd21 = hd1 && side_is_cell(axis_bits(cyd, 1), sg1);
                    const bool hd22 = hd2 && side_is_cell(axis_bits(czd, 2), sg2);
                    int jz;
                    const T tx = adj_axis3<T>(d, ein, din, c, code, plus(bx1, zo), cxu, 0, sg0, hu0, hu20, hd0, hd20,
                                              ec, ex1, ex2, exd, L.al, L.l, cp0, wsa[0]);
                    const T ty = adj_axis3<T>(d, ein, din, c, code, plus(by1, zo), cyu, 1, sg1, hu1, hu21, hd1, hd21,
                                              ec, ey1, ey2, eyd, L.al, L.l, cp1, wsa[1]);
                    const T tzv = adj_axis3<T>(d, ein, din, c, code, zcell(f - 1, jz), czu, 2, sg2, hu2, hu22, hd2,
                                               hd22, ec, ez1, ez2, ezd, L.al, L.l, cp2, wsa[2]);
                    tf = (tx + ty) + tzv;
                }
                b = tf - ec * itc + (T)L.w * itc * rl_t(r_tl, q) + gl;
            }
            // upwind recurrence of the cell: increments of the coupled
            // upwind cells (an uncoupled one is dropped by a select: its value
            // may be anything, e.g. the other buffer across a periodic face)
            const T ux = (mode & S3_CX) ? in.ux - ex1 : (T)0;
            const T uy = (mode & S3_CY) ? in.uy - ey1 : (T)0;
            const T uz = (mode & S3_CZ) ? dzu : (T)0;
            const T num = b + cp0 * ux + cp1 * uy + cp2 * uz;
            const T den = A0 + gam;
            if constexpr (sizeof(T) == 4) de = num * __builtin_amdgcn_rcpf(den);
            else de = num / den;
            en = ec + de;
            if (active) *reinterpret_cast<T *>(ob + vc) = en;
        } else if (active) {
            *reinterpret_cast<T *>(ob + vc) = atb(eb, vc);
        }
        vc += (unsigned)zstepb;
        // moment partials: eight cells staged, then reduced transposed
        const int mloc = f - fb;
        xs[wv][mloc & 7][lane] = (active && (mode & S3_SOLID)) ? en : (T)0;
        if ((mloc & 7) == 7 || f == fe - 1) {
            const int j = lane >> 3, p8 = lane & 7;
            double acc[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] = 0.0;
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
                const int l2 = 8 * p8 + qq;
                const double xv = (double)xs[wv][j][l2];
#pragma unroll
                for (int m = 0; m < NM; ++m) acc[m] += lcs[wv][l2][m] * xv;
            }
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                double v = acc[m];
                v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
                v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
                v += dpp_f64<0x141>(v);   // row_half_mirror
                acc[m] = v;
            }
            // every lane of the 8-lane group j holds cell j's totals
            const int fj = fb + (mloc & ~7) + j;
            const double g = __shfl(r_gam, min(fj - fb + 2, 63), 64);
            if (p8 == 0 && fj <= f) {
                const int cj = cb + plane * (sg2 > 0 ? fj : n2 - 1 - fj);
                double *o = part + ((size_t)pidx * nc + cj) * kMomN;
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
        // shift the window
        ez2 = ez1;
        ez1 = ec;
        ec = ezd;
        lz_up = lz;
        dzu = de;
    };

    Pre A, B;
    prefetch(fb, A);
    int f = fb;
    for (; f + 1 < fe; f += 2) {
        step(f, A, B);
        step(f + 1, B, A);
    }
    if (f < fe) step(f, A, B);
}

// --------------------------------------------------------------- launchers

// Segment lengths the kernel takes (the host also keeps (zseg + 2) planes
// of rows of every geometry below 4 GiB: the row offsets are 32-bit).
static bool sweep3d_fits(const Dev &, int zseg, size_t) { return zseg >= 1 && zseg <= 48; }

template <typename T, int LIM, bool ADJ, bool ADD>
void sweep3d_launch(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev, const double *din,
                    const SweepItem *items, int item0, int count, int zseg, int na_oct, int nchunk_oct, double *part,
                    hipStream_t s)
{
    const int blocks = (count + 3) / 4;
    hipLaunchKernelGGL((k_sweep3d<T, LIM, ADJ, ADD>), dim3(blocks), dim3(256), 0, s, d, ein, eout, dpend, TLdev, din,
                       items, item0, count, zseg, na_oct, nchunk_oct, part);
}

// Forward sweep of the items [item0, item0 + count) (one hyperplane).
template <typename T>
hipError_t launch_sweep3d(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev,
                          const double *din, const SweepItem *items, int item0, int count, int zseg, int na_oct,
                          int nchunk_oct, double *part, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (!sweep3d_fits(d, zseg, sizeof(T))) return hipErrorInvalidValue;
    const bool add = dpend != nullptr || d.jumps;
#define BTE_S3(LIM)                                                                                                  \
    if (d.limiter == LIM) {                                                                                          \
        if (add)                                                                                                     \
            sweep3d_launch<T, LIM, false, true>(d, ein, eout, dpend, TLdev, din, items, item0, count, zseg, na_oct,  \
                                                nchunk_oct, part, s);                                                \
        else                                                                                                         \
            sweep3d_launch<T, LIM, false, false>(d, ein, eout, dpend, TLdev, din, items, item0, count, zseg, na_oct, \
                                                 nchunk_oct, part, s);                                               \
    }
    BTE_S3(LIM_NONE) BTE_S3(LIM_MC) BTE_S3(LIM_MINMOD)
#undef BTE_S3
    return hipGetLastError();
}

// Transposed sweep of the adjoint iteration (X: isotropic closure term).
template <typename T>
hipError_t launch_sweep3d_adj(const Dev &d, const T *ein, T *eout, const double *X, const double *dinA,
                              const SweepItem *items, int item0, int count, int zseg, int na_oct, int nchunk_oct,
                              double *part, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (!sweep3d_fits(d, zseg, sizeof(T))) return hipErrorInvalidValue;
    sweep3d_launch<T, LIM_NONE, true, false>(d, ein, eout, nullptr, X, dinA, items, item0, count, zseg, na_oct,
                                             nchunk_oct, part, s);
    return hipGetLastError();
}

template hipError_t launch_sweep3d<float>(const Dev &, const float *, float *, const double *, const double *,
                                          const double *, const SweepItem *, int, int, int, int, int, double *,
                                          hipStream_t);
template hipError_t launch_sweep3d<double>(const Dev &, const double *, double *, const double *, const double *,
                                           const double *, const SweepItem *, int, int, int, int, int, double *,
                                           hipStream_t);
template hipError_t launch_sweep3d_adj<float>(const Dev &, const float *, float *, const double *, const double *,
                                              const SweepItem *, int, int, int, int, int, double *, hipStream_t);
template hipError_t launch_sweep3d_adj<double>(const Dev &, const double *, double *, const double *,
                                               const double *, const SweepItem *, int, int, int, int, int, double *,
                                               hipStream_t);

}  // namespace bte
