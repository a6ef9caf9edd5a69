// bte_transient3d.hip -- explicit transient step (Sec. 4.1, the forward-Euler
// second-order finite-volume update of the BTE) on three-dimensional
// geometries.
//
// One wavefront per (x, y) column of cells, octant and chunk of 64
// (direction, band) lanes.  The wavefront walks its column along z in the
// flow direction of the octant, so the z stencil (two upwind cells, the
// cell, the downwind cell) is a window of four registers that shifts by one
// load per cell, and the limited z slope of the upwind cell is carried from
// the previous cell.  The x and y neighbours are read from the cache
// hierarchy: neighbouring columns are walked by neighbouring wavefronts of
// the same XCD at the same time.  The cell itself is the same for all 64
// lanes, so its geometry code, T_L, scattering rate and source are scalar
// values, one cell per lane for runs of 64 cells, broadcast with readlane.
// The FP64 partial sum w e/tau of the T_L update is reduced over the 64
// lanes (a transposed reduction through LDS every eight cells) and written
// per (octant, chunk, cell).
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tilelds.h"
#include "bte_col3d.h"

namespace bte {


// JMP = false when no geometry has a periodic temperature drop: the jump
// terms are then zero and are not added.
template <typename T, int LIM, bool JMP>
__global__ __launch_bounds__(256) void k_transient3d(Dev d, const T *__restrict__ ein, T *__restrict__ eout,
                                                     const double *__restrict__ TLdev,
                                                     const double *__restrict__ din,
                                                     const ColItem *__restrict__ items, int nitems, int na_oct,
                                                     int nchunk_oct, double src, double dt,
                                                     double *__restrict__ part)
{
    // T_L partials of eight consecutive cells of each wavefront, reduced
    // transposed (lane = 8 cell + part) every eight cells
    __shared__ double red[4][8][64];
    // four wavefronts per block; logical blocks are contiguous per XCD so
    // that neighbouring columns share an L2
    const int nb = gridDim.x, bb = blockIdx.x;
    const int lb = (bb & 7) * (nb >> 3) + (bb >> 3);
    const int wi = lb * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wi >= nitems) return;
    const int lane = threadIdx.x & 63;
    const ColItem it = items[wi];
    const Film &fm = d.film[it.film];
    const int sg0 = octant_sign(d, it.oct, na_oct, 0), sg1 = octant_sign(d, it.oct, na_oct, 1),
              sg2 = octant_sign(d, it.oct, na_oct, 2);
    const int nl = d.nl, nk = d.nk, nc = d.nc;
    const int kbeg = it.oct * na_oct * nl, kend = kbeg + na_oct * nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const int kk = active ? k : kbeg;
    const LaneT<T> L = lane_make<T>(d, fm, kk);
    const T C4 = L.C4;
    const int n0 = fm.n[0], n1 = fm.n[1], n2 = fm.n[2], plane = n0 * n1;
    const int x = it.col % n0, y = it.col / n0;
    const int cb = fm.cell0 + x + n0 * y;   // cell of (x, y, 0)
    const T *zrow = static_cast<const T *>(d.zrow);
    const double *zd = static_cast<const double *>(d.zrow);
    const unsigned koff = (unsigned)kk * (unsigned)sizeof(T);
    // uniform row base, 32-bit lane offset; a missing cell reads the zero row
    auto ld = [&](const T *base, int c) -> T {
        const bool ok = c >= 0;
        const char *row = reinterpret_cast<const char *>((ok ? base : zrow) + (size_t)(ok ? c : 0) * nk);
        return *reinterpret_cast<const T *>(row + koff);
    };

    // x and y stencil columns (fixed along z): cell at z = 0 or -1, and the
    // periodic jump of their values
    int jx1, jx2, jxd, jy1, jy2, jyd;
    const int px1 = wrap_pos(x - sg0, n0, fm.periodic[0], jx1), px2 = wrap_pos(x - 2 * sg0, n0, fm.periodic[0], jx2),
              pxd = wrap_pos(x + sg0, n0, fm.periodic[0], jxd);
    const int py1 = wrap_pos(y - sg1, n1, fm.periodic[1], jy1), py2 = wrap_pos(y - 2 * sg1, n1, fm.periodic[1], jy2),
              pyd = wrap_pos(y + sg1, n1, fm.periodic[1], jyd);
    const int bx1 = px1 >= 0 ? fm.cell0 + px1 + n0 * y : -1, bx2 = px2 >= 0 ? fm.cell0 + px2 + n0 * y : -1,
              bxd = pxd >= 0 ? fm.cell0 + pxd + n0 * y : -1;
    const int by1 = py1 >= 0 ? fm.cell0 + x + n0 * py1 : -1, by2 = py2 >= 0 ? fm.cell0 + x + n0 * py2 : -1,
              byd = pyd >= 0 ? fm.cell0 + x + n0 * pyd : -1;
    auto jump = [&](int j, double pdT) -> T { return JMP ? C4 * (T)(j * pdT) : (T)0; };
    const T kx1 = jump(jx1, fm.pdT[0]), kx2 = jump(jx2, fm.pdT[0]), kxd = jump(jxd, fm.pdT[0]);
    const T ky1 = jump(jy1, fm.pdT[1]), ky2 = jump(jy2, fm.pdT[1]), kyd = jump(jyd, fm.pdT[1]);
    // cell of the column at flow index f (geometric z = f or n2 - 1 - f),
    // -1 outside a non-periodic column; its jump in units of C dT / 4pi
    auto zcell = [&](int f, int &jz) -> int {
        const int zg = wrap_pos(sg2 > 0 ? f : n2 - 1 - f, n2, fm.periodic[2], jz);
        return zg >= 0 ? cb + plane * zg : -1;
    };
    auto zval = [&](int f) -> T {
        int jz;
        const int c = zcell(f, jz);
        return JMP ? ld(ein, c) + jump(jz, fm.pdT[2]) : ld(ein, c);
    };
    auto plus = [](int base, int off) { return base >= 0 ? base + off : -1; };

    // z window (flow order) with its jumps
    T ez2 = zval(-2), ez1 = zval(-1), ec = zval(0), ezd = zval(1);
    // limited z slope of the upwind cell (carried from cell to cell)
    T lz_up = (LIM == LIM_NONE) ? (T)0 : lim_diff<T, LIM>(ez1 - ez2, ec - ez1);

    const T tdt = (T)dt, tsrc = (T)src;
    const T itau = L.itau;
    const T cp0 = L.cpl[0], cp1 = L.cpl[1], cp2 = L.cpl[2];
    double *__restrict__ pout = part + (size_t)(it.oct * nchunk_oct + it.chunk) * nc;

    // Values prefetched one cell ahead: the six x / y neighbours of the
    // next plane and the column value three cells downstream (it enters the
    // window after the next cell).  Two sets alternate (the loop is unrolled
    // by hand) so that no register copy has to wait for a load in flight.
    struct Pre {
        T nz, x1, x2, xd, y1, y2, yd;
    };
    // x / y neighbour rows of flow index 0 and the step between planes
    // (absent neighbours: the zero row, step 0), advanced cell by cell
    const long long zstep = (long long)(sg2 > 0 ? plane : -plane) * nk;
    const int z0 = sg2 > 0 ? 0 : n2 - 1;
    auto row0 = [&](int b) -> const T * { return b >= 0 ? ein + (size_t)(b + plane * z0) * nk : zrow; };
    const T *rx1 = row0(bx1), *rx2 = row0(bx2), *rxd = row0(bxd);   // rows of the cell being prefetched
    const T *ry1 = row0(by1), *ry2 = row0(by2), *ryd = row0(byd);
    const long long sx1 = bx1 >= 0 ? zstep : 0, sx2 = bx2 >= 0 ? zstep : 0, sxd = bxd >= 0 ? zstep : 0;
    const long long sy1 = by1 >= 0 ? zstep : 0, sy2 = by2 >= 0 ? zstep : 0, syd = byd >= 0 ? zstep : 0;
    const T *rc0 = ein + (size_t)(cb + plane * z0) * nk;   // the column's own row at flow index 0
    const T *rzr = rc0 + zstep;                            // row at flow index f + 3, before the advance
    auto at = [&](const T *row) -> T { return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + koff); };
    // loads for the cell after flow index f (x / y neighbours: the running
    // row pointers are advanced by one plane per cell, not past the column)
    // and the column value at flow index f + 3
    auto prefetch = [&](int f, Pre &q) {
        if (f + 1 < n2 && f >= 0) {
            rx1 += sx1;
            rx2 += sx2;
            rxd += sxd;
            ry1 += sy1;
            ry2 += sy2;
            ryd += syd;
        }
        q.x1 = at(rx1);
        q.x2 = at(rx2);
        q.xd = at(rxd);
        q.y1 = at(ry1);
        q.y2 = at(ry2);
        q.yd = at(ryd);
        // inside the column: plain row (a running pointer); past its end
        // (last three cells): periodic image with its jump, or zero
        rzr += zstep;
        const T *rz;
        T jz = (T)0;
        if (f + 3 < n2) {
            rz = rzr;
        } else {
            int j;
            const int c = zcell(f + 3, j);
            rz = c >= 0 ? ein + (size_t)c * nk : zrow;
            jz = jump(j, fm.pdT[2]);
        }
        q.nz = JMP ? at(rz) + jz : at(rz);
    };
    // Per-cell records, one cell of a run of 64 along the column per lane
    // (unconditional loads: an absent neighbour reads the cell's own code
    // and is masked), broadcast with readlane.
    // r_mode: bit 0 solid, bit 1 every axis has both upwind cells and the
    // downwind cell (the interior stencil), computed here once per cell so
    // that a cell's uniform decision is one broadcast and one branch.
    uint32_t r_code = 0, r_cxu = 0, r_cyu = 0, r_czu = 0, r_mode = 0;
    double r_gam = 0;
    T r_tlT = (T)0, r_gamT = (T)0, r_qsT = (T)0;
    auto records = [&](int f0) {
        const int fl = min(f0 + lane, n2 - 1);
        const int o = plane * (sg2 > 0 ? fl : n2 - 1 - fl);
        const int c = cb + o;
        r_code = d.code[c];
        const uint32_t cxu = d.code[bx1 >= 0 ? bx1 + o : c], cyu = d.code[by1 >= 0 ? by1 + o : c];
        r_cxu = bx1 >= 0 ? cxu : 0u;
        r_cyu = by1 >= 0 ? cyu : 0u;
        {
            int jz;
            const int cu = zcell(fl - 1, jz);
            const uint32_t v = d.code[cu >= 0 ? cu : c];
            r_czu = cu >= 0 ? v : 0u;
        }
        {
            const uint32_t ab0 = axis_bits(r_code, 0), ab1 = axis_bits(r_code, 1), ab2 = axis_bits(r_code, 2);
            const bool fx = side_is_cell(ab0, -sg0) && side_is_cell(ab0, sg0) &&
                            side_is_cell(axis_bits(r_cxu, 0), -sg0);
            const bool fy = side_is_cell(ab1, -sg1) && side_is_cell(ab1, sg1) &&
                            side_is_cell(axis_bits(r_cyu, 1), -sg1);
            const bool fz = side_is_cell(ab2, -sg2) && side_is_cell(ab2, sg2) &&
                            side_is_cell(axis_bits(r_czu, 2), -sg2);
            r_mode = ((r_code & kSolidBit) ? 1u : 0u) | ((fx && fy && fz) ? 2u : 0u);
        }
        r_gam = d.gamma[c];
        r_tlT = (T)TLdev[c];
        r_gamT = (T)r_gam;
        r_qsT = (T)(*(d.P ? d.P + c : zd) / fm.Ctot);   // P is null without a heat source
    };
    auto rlt = [&](T v, int q) -> T {
        if constexpr (sizeof(T) == 4) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
        else return rl_d(v, q);
    };
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    auto step = [&](int f, const Pre &in, Pre &out) {
        const int z = sg2 > 0 ? f : n2 - 1 - f;
        const int zo = plane * z;
        const int c = cb + zo;
        prefetch(f, out);
        const int q = f & 63;
        const uint32_t mode = (uint32_t)__builtin_amdgcn_readlane((int)r_mode, q);
        const T tlT = rlt(r_tlT, q), gamT = rlt(r_gamT, q), qsT = rlt(r_qsT, q);
        const bool solid = mode & 1u;
        const T ex1 = JMP ? in.x1 + kx1 : in.x1, ex2 = JMP ? in.x2 + kx2 : in.x2, exd = JMP ? in.xd + kxd : in.xd;
        const T ey1 = JMP ? in.y1 + ky1 : in.y1, ey2 = JMP ? in.y2 + ky2 : in.y2, eyd = JMP ? in.yd + kyd : in.yd;
        // z slope of this cell (also the upwind slope of the next cell)
        const T lz = (LIM == LIM_NONE) ? (T)0 : lim_diff<T, LIM>(ec - ez1, ezd - ec);
        T en = ec;
        double acc = 0.0;
        if (solid) {
          T dx, dy, dz;
          if (mode & 2u) {
            // interior stencil on every axis
            dx = delta_fast<T, LIM>(ex2, ex1, ec, exd);
            dy = delta_fast<T, LIM>(ey2, ey1, ec, eyd);
            if (LIM == LIM_NONE) dz = delta_fast<T, LIM>(ez2, ez1, ec, ezd);
            else dz = (ec - ez1) + (T)0.5 * (lz - lz_up);
          } else {
            const uint32_t code = (uint32_t)__builtin_amdgcn_readlane((int)r_code, q);
            const uint32_t code_xu = (uint32_t)__builtin_amdgcn_readlane((int)r_cxu, q);
            const uint32_t code_yu = (uint32_t)__builtin_amdgcn_readlane((int)r_cyu, q);
            const uint32_t code_zu = (uint32_t)__builtin_amdgcn_readlane((int)r_czu, q);
            const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1), ab2 = axis_bits(code, 2);
            const bool hu0 = side_is_cell(ab0, -sg0), hd0 = side_is_cell(ab0, sg0);
            const bool hu1 = side_is_cell(ab1, -sg1), hd1 = side_is_cell(ab1, sg1);
            const bool hu2 = side_is_cell(ab2, -sg2), hd2 = side_is_cell(ab2, sg2);
            const bool hu20 = hu0 && side_is_cell(axis_bits(code_xu, 0), -sg0);
            const bool hu21 = hu1 && side_is_cell(axis_bits(code_yu, 1), -sg1);
            const bool hu22 = hu2 && side_is_cell(axis_bits(code_zu, 2), -sg2);
            if (hu0 && hu20 && hd0) {
                dx = delta_fast<T, LIM>(ex2, ex1, ec, exd);
            } else {
                dx = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 0, sg0, hu0, hu20, hd0, ex2, ex1, ec, exd,
                                         plus(bxd, zo), kxd, L.al, L.l, C4, L.hh[0], L.ih[0]);
            }
            if (hu1 && hu21 && hd1) {
                dy = delta_fast<T, LIM>(ey2, ey1, ec, eyd);
            } else {
                dy = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 1, sg1, hu1, hu21, hd1, ey2, ey1, ec, eyd,
                                         plus(byd, zo), kyd, L.al, L.l, C4, L.hh[1], L.ih[1]);
            }
            if (hu2 && hu22 && hd2) {
                if (LIM == LIM_NONE) dz = delta_fast<T, LIM>(ez2, ez1, ec, ezd);
                else dz = (ec - ez1) + (T)0.5 * (lz - lz_up);
            } else {
                int jd;
                const int cdz = zcell(f + 1, jd);
                dz = delta_wall3<T, LIM>(d, fm, ein, din, c, code, 2, sg2, hu2, hu22, hd2, ez2, ez1, ec, ezd, cdz,
                                         jump(jd, fm.pdT[2]), L.al, L.l, C4, L.hh[2], L.ih[2]);
            }
          }
            const T D = cp0 * dx + cp1 * dy + cp2 * dz;
            const T itc = itau + gamT;
            en = ec + tdt * (-D - (ec - C4 * tlT) * itc + C4 * tsrc * qsT);
            acc = active ? (L.witau + L.w * rl_d(r_gam, q)) * (double)en : 0.0;
        }
        // streamed out (nontemporal): the step never reads its output back
        if (active) __builtin_nontemporal_store(en, &eout[(size_t)c * nk + k]);
        // partial of this cell into the transposed buffer; every eighth cell
        // (and at the end of the column) the eight cells are reduced
        red[wv][f & 7][lane] = acc;
        if ((f & 7) == 7 || f == n2 - 1) {
            const int j = lane >> 3, pp = lane & 7, fb = f & ~7;
            double v = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) v += red[wv][j][8 * pp + i];
            v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
            v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
            v += dpp_f64<0x141>(v);   // row_half_mirror
            const int fj = fb + j;
            // (pores get a zero partial: the T_L update ignores them)
            if (pp == 0 && fj <= f) __builtin_nontemporal_store(v, &pout[cb + plane * (sg2 > 0 ? fj : n2 - 1 - fj)]);
        }
        // shift the window to the next cell (the value two cells ahead was
        // prefetched by the previous cell, into `in`)
        ez2 = ez1;
        ez1 = ec;
        ec = ezd;
        ezd = in.nz;
        lz_up = lz;
    };

    Pre A, B;
    prefetch(-1, A);   // the first cell's x / y neighbours and the value at flow index 2
    for (int f0 = 0; f0 < n2; f0 += 64) {
        records(f0);
        const int f1 = min(f0 + 64, n2);
        int f = f0;
        for (; f + 1 < f1; f += 2) {
            step(f, A, B);
            step(f + 1, B, A);
        }
        if (f < f1) {
            step(f, A, B);
            A = B;
        }
    }
}

// Transposed explicit step of the transient adjoint (reverse mode of
// e^{k+1} = e^k + dt R(e^k)) on three-dimensional geometries, column by
// column like k_transient3d:  lam^k = lam^{k+1} + dt J^T lam^{k+1} with the
// forward state e^k read alongside for the gradient.  The item's octant
// fixes the frame; the lanes are those of the opposite octant, so in this
// frame the transposed stencil has the forward shape (two cells "upwind",
// one "downwind") and the same interior coefficients (central slopes, no
// limiter, no jumps: the transposed operator is linear).  Walls: a specular
// wall feeds the mirror lane's lam, a diffuse wall the record dinA (k_walls_adj)
// with weight w |s_a|, at the wall cell (3/2 or 1) and at its neighbour (-1/2).
// TLk = T_L(e^k), the lattice temperature the forward step of e^k used.
// Per (octant, chunk, cell) two partial sums go to
// part[((octant * nchunk + chunk) * 2 + q) * nc + cell]:
//   q = 0: sum C/(4 pi) (1/tau) lam^k,
//   q = 1: sum lam^{k+1} (C/(4 pi) T_L - e^k) + w X e^k  (the gradient's sums
//          over (direction, band), combined as in k_adj_step).

// RES: the transposed residual of the steady adjoint iteration instead of a
// transposed step (no output field, no forward state):
//   y = J^T psi - psi / tau_c + w X / tau_c + g,  g = w v_x L_x / (dT N_cells)
// (the k_eff objective of a geometry with a drop along x), and per
// (octant, chunk, cell) the two partials sum C/(4 pi) y and sum y^2 at
// part[((octant * nchunk + chunk) * 2 + q) * nc + cell].
template <typename T, bool RES>
__global__ __launch_bounds__(256) void k_adj_step3d(Dev d, const T *__restrict__ lam, T *__restrict__ lout,
                                                    const T *__restrict__ ek, const double *__restrict__ X,
                                                    const double *__restrict__ TLk, const double *__restrict__ dinA,
                                                    const ColItem *__restrict__ items, int nitems, int na_oct,
                                                    int nchunk_oct, double dt, double *__restrict__ part)
{
    // two partials of four consecutive cells per wavefront, reduced
    // transposed (lane = 16 cell + part) every four cells
    constexpr int NP = 2;
    __shared__ double red[4][NP][4][64];
    const int nb = gridDim.x, bb = blockIdx.x;
    const int lb = (bb & 7) * (nb >> 3) + (bb >> 3);
    const int wi = lb * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wi >= nitems) return;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ColItem it = items[wi];
    const Film &fm = d.film[it.film];
    const int sg0 = octant_sign(d, it.oct, na_oct, 0), sg1 = octant_sign(d, it.oct, na_oct, 1),
              sg2 = octant_sign(d, it.oct, na_oct, 2);
    const int nl = d.nl, nk = d.nk, nc = d.nc;
    const int loct = it.oct ^ 7;
    const int kbeg = loct * na_oct * nl, kend = kbeg + na_oct * nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const int kk = active ? k : kbeg;
    const LaneT<T> L = lane_make<T>(d, fm, kk);
    T wsa[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) wsa[a] = (T)(L.w * fabs(d.s[3 * L.al + a]));
    const double c4 = d.C4[L.l], it0 = d.itau[L.l];
    const int n0 = fm.n[0], n1 = fm.n[1], n2 = fm.n[2], plane = n0 * n1;
    const int x = it.col % n0, y = it.col / n0;
    const int cb = fm.cell0 + x + n0 * y;
    const T *zrow = static_cast<const T *>(d.zrow);
    const unsigned koff = (unsigned)kk * (unsigned)sizeof(T);
    auto at = [&](const T *row) -> T { return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + koff); };
    int jx;
    const int px1 = wrap_pos(x - sg0, n0, fm.periodic[0], jx), px2 = wrap_pos(x - 2 * sg0, n0, fm.periodic[0], jx),
              pxd = wrap_pos(x + sg0, n0, fm.periodic[0], jx);
    const int py1 = wrap_pos(y - sg1, n1, fm.periodic[1], jx), py2 = wrap_pos(y - 2 * sg1, n1, fm.periodic[1], jx),
              pyd = wrap_pos(y + sg1, n1, fm.periodic[1], jx);
    const int bx1 = px1 >= 0 ? fm.cell0 + px1 + n0 * y : -1, bx2 = px2 >= 0 ? fm.cell0 + px2 + n0 * y : -1,
              bxd = pxd >= 0 ? fm.cell0 + pxd + n0 * y : -1;
    const int by1 = py1 >= 0 ? fm.cell0 + x + n0 * py1 : -1, by2 = py2 >= 0 ? fm.cell0 + x + n0 * py2 : -1,
              byd = pyd >= 0 ? fm.cell0 + x + n0 * pyd : -1;
    auto zcell = [&](int f) -> int {
        int jz;
        const int zg = wrap_pos(sg2 > 0 ? f : n2 - 1 - f, n2, fm.periodic[2], jz);
        return zg >= 0 ? cb + plane * zg : -1;
    };
    auto zval = [&](int f) -> T {
        const int c = zcell(f);
        return at(c >= 0 ? lam + (size_t)c * nk : zrow);
    };
    auto plus = [](int base, int off) { return base >= 0 ? base + off : -1; };

    T z2 = zval(-2), z1 = zval(-1), zc = zval(0), zd = zval(1);
    const T tdt = (T)dt;
    const T itau = L.itau;

    struct Pre {
        T nz, x1, x2, xd, y1, y2, yd, e;
    };
    const long long zstep = (long long)(sg2 > 0 ? plane : -plane) * nk;
    const int z0 = sg2 > 0 ? 0 : n2 - 1;
    auto row0 = [&](const T *base, int b) -> const T * { return b >= 0 ? base + (size_t)(b + plane * z0) * nk : zrow; };
    const T *rx1 = row0(lam, bx1), *rx2 = row0(lam, bx2), *rxd = row0(lam, bxd);
    const T *ry1 = row0(lam, by1), *ry2 = row0(lam, by2), *ryd = row0(lam, byd);
    const T *re = RES ? lam : row0(ek, cb);
    const long long sx1 = bx1 >= 0 ? zstep : 0, sx2 = bx2 >= 0 ? zstep : 0, sxd = bxd >= 0 ? zstep : 0;
    const long long sy1 = by1 >= 0 ? zstep : 0, sy2 = by2 >= 0 ? zstep : 0, syd = byd >= 0 ? zstep : 0;
    const T *rc0 = lam + (size_t)(cb + plane * z0) * nk;
    auto prefetch = [&](int f, Pre &q) {
        if (f + 1 < n2 && f >= 0) {
            rx1 += sx1;
            rx2 += sx2;
            rxd += sxd;
            ry1 += sy1;
            ry2 += sy2;
            ryd += syd;
            if constexpr (!RES) re += zstep;
        }
        q.x1 = at(rx1);
        q.x2 = at(rx2);
        q.xd = at(rxd);
        q.y1 = at(ry1);
        q.y2 = at(ry2);
        q.yd = at(ryd);
        if constexpr (!RES) q.e = at(re);
        else q.e = (T)0;
        const T *rz;
        if (f + 3 < n2) {
            rz = rc0 + (long long)(f + 3) * zstep;
        } else {
            const int c = zcell(f + 3);
            rz = c >= 0 ? lam + (size_t)c * nk : zrow;
        }
        q.nz = at(rz);
    };
    // per-cell records of a run of 64 cells, one per lane: codes of the cell
    // and of its frame-upwind / frame-downwind neighbours along x, y, z,
    // the closure term X and gamma
    uint32_t r_code = 0, r_cxu = 0, r_cyu = 0, r_cxd = 0, r_cyd = 0, r_czu = 0, r_czd = 0, r_mode = 0;
    double r_X = 0, r_gam = 0, r_tl = 0;
    auto records = [&](int f0) {
        const int fl = min(f0 + lane, n2 - 1);
        const int o = plane * (sg2 > 0 ? fl : n2 - 1 - fl);
        const int c = cb + o;
        r_code = d.code[c];
        const uint32_t cxu = d.code[bx1 >= 0 ? bx1 + o : c], cyu = d.code[by1 >= 0 ? by1 + o : c];
        const uint32_t cxd = d.code[bxd >= 0 ? bxd + o : c], cyd = d.code[byd >= 0 ? byd + o : c];
        r_cxu = bx1 >= 0 ? cxu : 0u;
        r_cyu = by1 >= 0 ? cyu : 0u;
        r_cxd = bxd >= 0 ? cxd : 0u;
        r_cyd = byd >= 0 ? cyd : 0u;
        const int cu = zcell(fl - 1), cd = zcell(fl + 1);
        const uint32_t czu = d.code[cu >= 0 ? cu : c], czd = d.code[cd >= 0 ? cd : c];
        r_czu = cu >= 0 ? czu : 0u;
        r_czd = cd >= 0 ? czd : 0u;
        r_X = X[c];
        r_gam = d.gamma[c];
        if constexpr (!RES) r_tl = TLk[c];
        // bit 0 solid, bit 1 the interior transposed stencil on every axis
        // (two cells on each side where the forward stencil reaches)
        auto inner = [&](int a, int sg, uint32_t cu_, uint32_t cd_) {
            const uint32_t ab = axis_bits(r_code, a);
            return side_is_cell(ab, -sg) && side_is_cell(ab, sg) && side_is_cell(axis_bits(cu_, a), -sg) &&
                   side_is_cell(axis_bits(cd_, a), sg);
        };
        const bool all = inner(0, sg0, r_cxu, r_cxd) && inner(1, sg1, r_cyu, r_cyd) && inner(2, sg2, r_czu, r_czd);
        r_mode = ((r_code & kSolidBit) ? 1u : 0u) | (all ? 2u : 0u);
    };
    auto rlu = [&](uint32_t v, int q) -> uint32_t { return (uint32_t)__builtin_amdgcn_readlane((int)v, q); };
    double *__restrict__ pbase = part + (size_t)((it.oct * nchunk_oct + it.chunk) * NP) * nc;
    const double gfac = fm.pdT[0] != 0.0 ? fm.len[0] / (fm.pdT[0] * fm.ncell) : 0.0;
    const T gl = (T)(gfac * L.wv[0]);

    auto step = [&](int f, const Pre &in, Pre &out) {
        const int zo = plane * (sg2 > 0 ? f : n2 - 1 - f);
        const int c = cb + zo;
        prefetch(f, out);
        const int q = f & 63;
        const uint32_t mode = rlu(r_mode, q);
        const bool solid = mode & 1u;
        T ln = (T)0;
        double acc[NP] = {0, 0};
        if (solid) {
          const double Xc = rl_d(r_X, q), gam = rl_d(r_gam, q);
          T tf;
          if (mode & 2u) {
            // interior transposed stencil on every axis
            const T tx = L.cpl[0] * ((in.x1 - zc) + (T)0.25 * ((zc - in.xd) - (in.x2 - in.x1)));
            const T ty = L.cpl[1] * ((in.y1 - zc) + (T)0.25 * ((zc - in.yd) - (in.y2 - in.y1)));
            const T tz = L.cpl[2] * ((z1 - zc) + (T)0.25 * ((zc - zd) - (z2 - z1)));
            tf = (tx + ty) + tz;
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
            {
                T tx;
                if (hu0 && hu20 && hd0 && hd20) tx = L.cpl[0] * ((in.x1 - zc) + (T)0.25 * ((zc - in.xd) - (in.x2 - in.x1)));
                else
                    tx = adj_axis3<T>(d, lam, dinA, c, code, plus(bx1, zo), cxu, 0, sg0, hu0, hu20, hd0, hd20, zc,
                                      in.x1, in.x2, in.xd, L.al, L.l, L.cpl[0], wsa[0]);
                T ty;
                if (hu1 && hu21 && hd1 && hd21) ty = L.cpl[1] * ((in.y1 - zc) + (T)0.25 * ((zc - in.yd) - (in.y2 - in.y1)));
                else
                    ty = adj_axis3<T>(d, lam, dinA, c, code, plus(by1, zo), cyu, 1, sg1, hu1, hu21, hd1, hd21, zc,
                                      in.y1, in.y2, in.yd, L.al, L.l, L.cpl[1], wsa[1]);
                T tz;
                if (hu2 && hu22 && hd2 && hd22) tz = L.cpl[2] * ((z1 - zc) + (T)0.25 * ((zc - zd) - (z2 - z1)));
                else
                    tz = adj_axis3<T>(d, lam, dinA, c, code, zcell(f - 1), czu, 2, sg2, hu2, hu22, hd2, hd22, zc, z1,
                                      z2, zd, L.al, L.l, L.cpl[2], wsa[2]);
                tf = (tx + ty) + tz;
            }
          }
            const T itc = itau + (T)gam;
            if constexpr (RES) {
                const T yr = tf - zc * itc + (T)L.w * itc * (T)Xc + gl;
                if (active) {
                    acc[0] = c4 * (double)yr;
                    acc[1] = (double)yr * (double)yr;
                }
            } else {
                ln = zc + tdt * (tf - zc * itc + (T)L.w * itc * (T)Xc);
                if (active) {
                    const double xe = (double)in.e;
                    acc[0] = c4 * (it0 + gam) * (double)ln;
                    acc[1] = (double)zc * (c4 * rl_d(r_tl, q) - xe) + L.w * Xc * xe;
                }
            }
        }
        if constexpr (!RES)
            if (active) lout[(size_t)c * nk + k] = ln;
#pragma unroll
        for (int m = 0; m < NP; ++m) red[wv][m][f & 3][lane] = acc[m];
        if ((f & 3) == 3 || f == n2 - 1) {
            const int j = lane >> 4, pp = lane & 15, fb = f & ~3;
            const int fj = fb + j;
            double v[NP];
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) t += red[wv][m][j][4 * pp + i];
                t += dpp_f64<0xB1>(t);    // quad_perm [1,0,3,2]
                t += dpp_f64<0x4E>(t);    // quad_perm [2,3,0,1]
                t += dpp_f64<0x141>(t);   // row_half_mirror
                t += dpp_f64<0x140>(t);   // row_mirror
                v[m] = t;
            }
            if (pp == 0 && fj <= f) {
                const int cj = cb + plane * (sg2 > 0 ? fj : n2 - 1 - fj);
#pragma unroll
                for (int m = 0; m < NP; ++m) pbase[(size_t)m * nc + cj] = v[m];
            }
        }
        z2 = z1;
        z1 = zc;
        zc = zd;
        zd = in.nz;
    };

    Pre A, B;
    prefetch(-1, A);
    for (int f0 = 0; f0 < n2; f0 += 64) {
        records(f0);
        const int f1 = min(f0 + 64, n2);
        int f = f0;
        for (; f + 1 < f1; f += 2) {
            step(f, A, B);
            step(f + 1, B, A);
        }
        if (f < f1) {
            step(f, A, B);
            A = B;
        }
    }
}

template <typename T>
hipError_t launch_adj_step3d(const Dev &d, const T *lam, T *lout, const T *ek, const double *X, const double *TLk,
                             const double *dinA, const ColItem *items, int nitems, int na_oct, int nchunk_oct,
                             double dt, double *part, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int blocks = ((nitems + 3) / 4 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_adj_step3d<T, false>), dim3(blocks), dim3(256), 0, s, d, lam, lout, ek, X, TLk, dinA,
                       items, nitems, na_oct, nchunk_oct, dt, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_res3d(const Dev &d, const T *psi, const double *X, const double *dinA, const ColItem *items,
                            int nitems, int na_oct, int nchunk_oct, double *part, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int blocks = ((nitems + 3) / 4 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_adj_step3d<T, true>), dim3(blocks), dim3(256), 0, s, d, psi, nullptr, nullptr, X, nullptr,
                       dinA, items, nitems, na_oct, nchunk_oct, 0.0, part);
    return hipGetLastError();
}

template hipError_t launch_adj_res3d<float>(const Dev &, const float *, const double *, const double *,
                                            const ColItem *, int, int, int, double *, hipStream_t);
template hipError_t launch_adj_res3d<double>(const Dev &, const double *, const double *, const double *,
                                             const ColItem *, int, int, int, double *, hipStream_t);

template hipError_t launch_adj_step3d<float>(const Dev &, const float *, float *, const float *, const double *,
                                             const double *, const double *, const ColItem *, int, int, int, double,
                                             double *, hipStream_t);
template hipError_t launch_adj_step3d<double>(const Dev &, const double *, double *, const double *, const double *,
                                              const double *, const double *, const ColItem *, int, int, int, double,
                                              double *, hipStream_t);

template <typename T, int LIM>
void transient3d_launch(const Dev &d, const T *ein, T *eout, const double *TLdev, const double *din,
                        const ColItem *items, int nitems, int na_oct, int nchunk_oct, double src, double dt,
                        double *part, hipStream_t s)
{
    const int blocks = ((nitems + 3) / 4 + 7) / 8 * 8;
    if (d.jumps)
        hipLaunchKernelGGL((k_transient3d<T, LIM, true>), dim3(blocks), dim3(256), 0, s, d, ein, eout, TLdev, din,
                           items, nitems, na_oct, nchunk_oct, src, dt, part);
    else
        hipLaunchKernelGGL((k_transient3d<T, LIM, false>), dim3(blocks), dim3(256), 0, s, d, ein, eout, TLdev, din,
                           items, nitems, na_oct, nchunk_oct, src, dt, part);
}

template <typename T>
hipError_t launch_transient3d(const Dev &d, const T *ein, T *eout, const double *TLdev, const double *din,
                              const ColItem *items, int nitems, int na_oct, int nchunk_oct, double src, double dt,
                              double *part, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (d.limiter == LIM_NONE)
        transient3d_launch<T, LIM_NONE>(d, ein, eout, TLdev, din, items, nitems, na_oct, nchunk_oct, src, dt, part, s);
    else if (d.limiter == LIM_MC)
        transient3d_launch<T, LIM_MC>(d, ein, eout, TLdev, din, items, nitems, na_oct, nchunk_oct, src, dt, part, s);
    else
        transient3d_launch<T, LIM_MINMOD>(d, ein, eout, TLdev, din, items, nitems, na_oct, nchunk_oct, src, dt, part,
                                          s);
    return hipGetLastError();
}

template hipError_t launch_transient3d<float>(const Dev &, const float *, float *, const double *, const double *,
                                              const ColItem *, int, int, int, double, double, double *, hipStream_t);
template hipError_t launch_transient3d<double>(const Dev &, const double *, double *, const double *, const double *,
                                               const ColItem *, int, int, int, double, double, double *,
                                               hipStream_t);

}  // namespace bte
