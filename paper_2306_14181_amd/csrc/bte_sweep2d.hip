// bte_sweep2d.hip -- register-resident tile sweep for two-dimensional
// geometries (the steady transport sweep of Sec. 3.3-3.5, Algorithm 1, in
// delta form with the first-order upwind implicit operator).
//
// One block per work item (tile of up to 8 x 8 cells, octant, chunk of 64
// (direction, band) lanes) with 8 / kRW wavefronts of kRW tile rows each
// (kRW = 1, 2 or 4; two by default).  A
// wavefront keeps the window of its rows in registers (two upwind rows, its
// rows with their x halo, the next row), so the stencil of every cell is
// read from registers, and forms the right-hand side of its rows; the upwind
// recurrence (serial along x and y) then runs wavefront after wavefront,
// each handing the increments of its last row to the next through LDS.
// Everything that depends only on the cell (global index, geometry code,
// T_L, scattering rate, source, pending correction) is loaded once, one
// cell per lane, and read back with readlane or broadcast LDS loads.  The
// FP64 moment partials of a row are reduced through a small LDS transpose.
// With two rows per wavefront, at 124 VGPRs and 26 KiB of LDS (FP32), four
// blocks share a compute unit.
#include "bte_internal.h"
#include "bte_stencil.h"
#include "bte_tile.h"
#include "bte_tilelds.h"

namespace bte {

namespace {

constexpr int kTX = 8, kTY = 8;
constexpr int kWS = 65;   // row stride of a staged row in the moment transpose

struct Frame2 {
    int o0, o1, e0, e1, sg0, sg1, n0, n1, cell0, per0, per1;
    double pdT0, pdT1;
};

__device__ inline Frame2 frame2(const Sweep2Item &it)
{
    Frame2 F;
    F.o0 = it.o0;
    F.o1 = it.o1;
    F.e0 = it.e0;
    F.e1 = it.e1;
    F.n0 = it.n0;
    F.n1 = it.n1;
    F.cell0 = it.cell0;
    F.per0 = it.flags & 1;
    F.per1 = (it.flags >> 1) & 1;
    F.sg0 = (it.flags & 4) ? 1 : -1;
    F.sg1 = (it.flags & 8) ? 1 : -1;
    F.pdT0 = it.pdT0;
    F.pdT1 = it.pdT1;
    return F;
}

// The cell at flow position (f0, f1) whatever it holds (its value is only
// used where the codes of the neighbours say it is solid) and the periodic
// jump of the value there (units of C/4pi); -1 outside a non-periodic domain.
__device__ inline int cell2_any(const Frame2 &F, int f0, int f1, double &jump)
{
    int i0 = F.o0 + (F.sg0 > 0 ? f0 : F.e0 - 1 - f0);
    int i1 = F.o1 + (F.sg1 > 0 ? f1 : F.e1 - 1 - f1);
    jump = 0.0;
    // each crossing of the low face adds +C dT/4pi (two on an axis of one cell)
    if (i0 < 0 || i0 >= F.n0) {
        if (!F.per0) return -1;
        const int w = periods(i0, F.n0);
        jump -= w * F.pdT0;
        i0 -= w * F.n0;
    }
    if (i1 < 0 || i1 >= F.n1) {
        if (!F.per1) return -1;
        const int w = periods(i1, F.n1);
        jump -= w * F.pdT1;
        i1 -= w * F.n1;
    }
    return F.cell0 + i0 + F.n0 * i1;
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

// Queue words of a one-launch sweep: ticket counter, abort word, then one
// completion flag per item; all zeroed by k_queue_reset before the launch.
//
// Ordering without per-block cache maintenance: every new value a block
// writes is a device-scope store (coherent beyond the XCD's L2), and every
// wavefront waits for all its memory operations to complete (s_waitcnt 0)
// before the block's last barrier, after which the flag is written; a
// waiting block polls the flag with device-scope loads, passes a barrier,
// and reads the values it needs from its upwind tiles with device-scope
// loads.  (An agent-scope release / acquire pair per block instead writes
// back and invalidates the whole L2 each time, which made the sweep 2.4x
// slower than one launch per diagonal.)
constexpr int kQueueTicket = 0, kQueueAbort = 1, kQueueDone = 2;
constexpr int kQueueSpin = 1 << 20;   // polls before a wait gives up (about a second)

// Wait until item u is published.  The wait is bounded: after kQueueSpin
// polls (or once any block has given up) it sets the abort word and
// returns, so the launch always ends; the host reports the abort as an
// error.  The polls are device-scope loads, issued in the loop.
__device__ inline void queue_wait(unsigned *q, int u)
{
    for (int n = 0; n < kQueueSpin; ++n) {
        if (__hip_atomic_load(q + kQueueDone + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
        if ((n & 63) == 63 && __hip_atomic_load(q + kQueueAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(q + kQueueAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish item u (called after the barrier that follows every wavefront's
// completed stores).
__device__ inline void queue_publish(unsigned *q, int u)
{
    __hip_atomic_store(q + kQueueDone + u, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-scope load and store of a state value (the one-launch sweep's
// values that other blocks of the same launch read).
template <typename T> __device__ inline T dev_load(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ inline void dev_store(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_queue_reset(unsigned *q, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n + kQueueDone) q[i] = 0u;
}

}  // namespace

// Face-value difference of one axis on the general path (missing
// neighbours, walls).  fin_wall is the inflow face value when the upwind
// side is a wall (thermalizing, diffuse: prepared by the caller); a specular
// wall reads the mirror lane here.
template <typename T, int LIM>
__device__ inline T delta_general(const Dev &d, const T *__restrict__ e, int c, uint32_t code, int a, int sg,
                                  bool hu, bool hu2, bool hd, T e2, T e1, T ec, T ed, T fin_wall, int cd, double xd,
                                  double xc, int al, int l, bool active, T C4, T hh, T ih, int nk)
{
    const T fout = ec + hh * slope_flow<T>(LIM, hu, hd, e1, ec, ed, ih);
    T fin;
    if (hu) {
        fin = e1 + hh * slope_flow<T>(LIM, hu2, true, e2, e1, ec, ih);
    } else if (side_wall(axis_bits(code, a), -sg) == 1) {
        // specular: outgoing face value of the mirror direction, whose
        // upwind side is this lane's downwind side
        const int km = d.mirror[a * d.na + al] * d.nl + l;
        const T em = active ? e[(size_t)c * nk + km] + C4 * (T)xc : (T)0;
        T gm = (T)0;
        if (LIM == LIM_NONE && hd && active) gm = (em - (e[(size_t)cd * nk + km] + C4 * (T)xd)) * ih;
        fin = em + hh * gm;
    } else {
        fin = fin_wall;
    }
    return fout - fin;
}

// Number of diffuse-wall records of a cell that precede face f (records are
// numbered cell by cell in face order -x, +x, -y, +y).
__device__ inline int diffuse_rank2(uint32_t code, int f)
{
    int n = 0;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const uint32_t ab = axis_bits(code, g >> 1);
        const int side = (g & 1) ? 1 : -1;
        n += (g < f && !side_is_cell(ab, side) && side_record(ab, side)) ? 1 : 0;
    }
    return n;
}

// Per tile cell mode word (built once per wave, read as a uniform value)
enum : uint32_t {
    W_SOLID = 1u, W_FX = 2u, W_FY = 4u,        // solid; interior stencil along x / y
    W_CX = 8u, W_CY = 16u,                     // implicit coupling to the upwind cell along x / y
    W_HU20 = 32u, W_HU21 = 64u,                // second upwind cell exists along x / y
    W_DX = 128u, W_DY = 256u                   // diffuse wall on the upwind side along x / y
};

// Occupancy the compiler is held to (waves per SIMD) for kRW rows per
// wavefront, FP32: four waves per SIMD at one or two rows (four blocks of
// four wavefronts per compute unit at two rows), two at four rows; the
// one-launch form, which keeps a few more values across its wait, three
// (four would spill).  FP64: two (its registers allow no more without spills).
template <typename T, int kRW, bool QUEUE> constexpr int sweep2d_waves()
{
    return sizeof(T) == 8 ? 2 : (kRW == 4 ? 2 : (QUEUE ? 3 : 4));
}

// QUEUE: the whole sweep in one launch, one block per item: a block takes
// a ticket (items in sweep order), does everything that reads only the
// previous iterate, then waits for the items of its x- and y-upwind tiles
// (queue_wait) before it reads their new values, and publishes its own
// after its stores.  Otherwise the launch covers one tile diagonal.
template <typename T, int LIM, int kRW, bool QUEUE>
__global__ __launch_bounds__(64 * (kTY / kRW), (sweep2d_waves<T, kRW, QUEUE>())) void k_sweep2d(
    Dev d, const T *__restrict__ ein, T *__restrict__ eout, const double *__restrict__ dpend,
    const double *__restrict__ TLdev, const double *__restrict__ din, const Sweep2Item *__restrict__ items,
    int item0, int na_oct, int nchunk_oct, double *__restrict__ part, unsigned *__restrict__ queue)
{
    constexpr int kWT = kTY / kRW;   // wavefronts per tile (one block)
    // moment weights of lane l2 = 8 p + q at lc[q][m][p]: the lanes of the
    // row transpose below read the eight p of one (q, m) at once, eight
    // consecutive doubles (no bank conflicts)
    __shared__ double lc[8][kMomN][8];
    // increments of the last row of wavefront w, read by wavefront w + 1
    __shared__ T sH[64][kTX];
    // Per wavefront: a staging area of one row (diffuse inflow values, slot
    // 2 j + axis; then the row's new values for the moment transpose) and
    // the per-cell scalars of the tile (x = pending correction plus jump,
    // gamma, T_L, source; halo x), read back as broadcast LDS loads rather
    // than lane-by-lane register broadcasts.
    __shared__ T sStg[kWT][16][64];
    __shared__ T sPC[kWT][4][64];
    __shared__ T sHX[kWT][64];
    int item = item0 + (int)blockIdx.x;
    if constexpr (QUEUE) {
        // the ticket is taken first, by a running block: every item this
        // block waits for has a smaller ticket, i.e. a block already running
        __shared__ int s_ticket;
        if (threadIdx.x == 0) s_ticket = (int)atomicAdd(queue + kQueueTicket, 1u);
        __syncthreads();
        item = s_ticket;
    }
    const Sweep2Item it = items[item];
    // converged geometry of a batch (uniform over the block); a single
    // geometry is never swept once converged, so its blocks skip this load
    // and reach their stencil loads one round trip earlier
    if (d.nfilm > 1 && d.fdone[it.film]) {
        if constexpr (QUEUE)
            if (threadIdx.x == 0) queue_publish(queue, item);
        return;
    }
    // wavefront w owns tile rows r0 .. r0 + kRW - 1 (readfirstlane: w is
    // known to be uniform, so everything derived from it stays scalar)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r0 = kRW * w;
    const int nl = d.nl, nk = d.nk;
    const int kbeg = it.oct * na_oct * nl, kend = kbeg + na_oct * nl;
    const int k = kbeg + it.chunk * 64 + lane;
    const bool active = k < kend;
    const int kk = active ? k : kbeg;
    const int al = kk / nl, l = kk - al * nl;
    // lane constants (direction al, band l)
    const int mb = it.moff + l;   // the band in the geometry's material
    const double wq = d.w[al], vq = d.v[mb], itq = d.itau[mb];
    const double s0 = d.s[3 * al], s1 = d.s[3 * al + 1], s2 = d.s[3 * al + 2];
    const T C4 = (T)d.C4[mb], itau = (T)itq;
    const T cp0 = (T)(vq * fabs(s0) * it.ih0), cp1 = (T)(vq * fabs(s1) * it.ih1);
    const T hh0 = (T)(0.5 * it.h0), hh1 = (T)(0.5 * it.h1), ih0 = (T)it.ih0, ih1 = (T)it.ih1;
    if (w == 0) {
        double *lq = &lc[lane & 7][0][lane >> 3];
        lq[0] = active ? wq : 0.0;
        lq[8] = active ? wq * itq : 0.0;
        lq[16] = active ? wq * vq * s0 : 0.0;
        lq[24] = active ? wq * vq * s1 : 0.0;
        lq[32] = active ? wq * vq * s2 : 0.0;
    }
    const Frame2 F = frame2(it);
    const int e0 = F.e0, e1 = F.e1;
    const int sg0 = F.sg0, sg1 = F.sg1;
    const int sx = sg0 > 0 ? 1 : -1;
    const int rowstep = sg1 > 0 ? F.n0 : -F.n0;
    const int cbase = F.cell0 + (sg0 > 0 ? F.o0 : F.o0 + e0 - 1) + F.n0 * (sg1 > 0 ? F.o1 : F.o1 + e1 - 1);
    // rows of this wavefront inside the tile, and the first of them clamped
    // to the tile (a wavefront past the tile loads, and then skips)
    const int nrow = e1 - r0 < 0 ? 0 : (e1 - r0 > kRW ? kRW : e1 - r0);
    const int rb = r0 < e1 ? r0 : e1 - 1;

    // ---- cell records, one cell per lane (every wavefront builds the same),
    // read back with readlane: tile cell t = f0 + 8 f1 in lane t; halo cell
    // h (see halo_pos) in lane h.  Indices are arithmetic, so the stencil
    // loads below need no record; every load of the block depends on the
    // work item only and is issued unconditionally (a missing cell reads the
    // zero row, an absent field a zero), so the whole batch is in flight at
    // once: a load under a branch is waited for before the branch joins.
    int t_c = -1, h_c = -1;
    double h_j = 0;
    {
        const int f0 = lane & 7, f1 = lane >> 3;
        if (f0 < e0 && f1 < e1) t_c = cbase + rowstep * f1 + sx * f0;
        int h0, h1;
        if (halo_pos(F, lane, h0, h1)) h_c = cell2_any(F, h0, h1, h_j);
    }
    // cell records first (the mode words need them), then the raw stencil
    // values of this wavefront's row window, which are waited for only when
    // the right-hand side is formed
    const T *zrow = static_cast<const T *>(d.zrow);
    const double *zd = static_cast<const double *>(d.zrow);
    const int tcl = t_c >= 0 ? t_c : F.cell0, hcl = h_c >= 0 ? h_c : F.cell0;
    const uint32_t t_code = t_c >= 0 ? d.code[tcl] : 0u, h_code = h_c >= 0 ? d.code[hcl] : 0u;
    const double t_xd = *(dpend ? dpend + tcl : zd), h_xd = *(dpend ? dpend + hcl : zd);
    const double t_tld = *(TLdev ? TLdev + tcl : zd);
    const double t_gamd = d.gamma[tcl];
    const double t_qsd = *(d.P ? d.P + tcl : zd);   // P is null without a heat source
    const int t_db = d.dbase[tcl];
    auto row_c = [&](int q, int j) -> int {
        const int tc = j < e0 ? cbase + rowstep * q + sx * j : -1;
        const int hcv = rl(h_c, q == -2 ? j : (q == -1 ? 8 + j : 16 + j));
        return (q >= 0 && q < e1) ? tc : hcv;
    };
    // the row base is uniform and the lane offset a 32-bit byte count, so
    // these are scalar-base loads with one offset register
    const unsigned koff = (unsigned)kk * (unsigned)sizeof(T);
    auto ldc = [&](const T *base, int c) -> T {
        const bool ok = c >= 0;
        const char *row = reinterpret_cast<const char *>((ok ? base : zrow) + (size_t)(ok ? c : 0) * nk);
        return *reinterpret_cast<const T *>(row + koff);
    };
    // The cells of a row (tile row or halo row) are consecutive along x: a
    // row is addressed by the scalar address of its lowest-x cell, the cell
    // j by a per-lane byte offset (j clamped to the tile's extent, so a
    // ragged tile re-reads its last cell); a missing row, or a row past the
    // downwind halo, is the zero row, 8 cells long.  No scalar work per load.
    const char *zc = reinterpret_cast<const char *>(zrow);
    const int lo = sx > 0 ? 0 : -(e0 - 1);   // lowest-x cell relative to the row's flow-first cell
    auto rowp = [&](const T *base, int q) -> const char * {
        if (q > e1) return zc;
        const int c = (q >= 0 && q < e1) ? cbase + rowstep * q : rl(h_c, q == -2 ? 0 : (q == -1 ? 8 : 16));
        return c >= 0 ? reinterpret_cast<const char *>(base + (size_t)(c + lo) * nk) : zc;
    };
    // window: rows rb - 2 .. rb + kRW (y[i] holds row rb - 2 + i), the x
    // halo of this wavefront's rows, the new x-upwind values of its rows and
    // (first wavefront) the new values of the row upwind of the tile
    constexpr int kWin = kRW + 3;
    T y[kWin][kTX], dr[kTX];
    {
        const char *pr[kWin];
#pragma unroll
        for (int i = 0; i < kWin; ++i) pr[i] = rowp(ein, rb - 2 + i);
        const char *pdr = rb == 0 ? rowp(eout, -1) : zc;
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            const int jc = j < e0 ? j : e0 - 1;
            const unsigned o = koff + (unsigned)((sx > 0 ? jc : e0 - 1 - jc) * nk) * (unsigned)sizeof(T);
#pragma unroll
            for (int i = 0; i < kWin; ++i) y[i][j] = *reinterpret_cast<const T *>(pr[i] + o);
            if constexpr (!QUEUE) dr[j] = *reinterpret_cast<const T *>(pdr + o);
        }
    }
    T xh[kRW][3], dxr[kRW];
#pragma unroll
    for (int i = 0; i < kRW; ++i) {
        const int hx = 24 + 3 * (rb + i);   // lanes past the tile's halo hold no cell (zero row)
        const int c0 = rl(h_c, hx), c1 = rl(h_c, hx + 1), c2 = rl(h_c, hx + 2);
        xh[i][0] = ldc(ein, c0);
        xh[i][1] = ldc(ein, c1);
        xh[i][2] = ldc(ein, c2);
        if constexpr (!QUEUE) dxr[i] = ldc(eout, c1);
    }

    // mode words (needs the codes of the upwind neighbours: lanes t - 1 /
    // t - 8 of the tile, or the x-halo / row -1 halo lanes)
    uint32_t t_w = 0;
    T t_tl, t_gam, t_qs, t_x, h_x;
    {
        const int f0 = lane & 7, f1 = lane >> 3;
        const uint32_t cxa = (uint32_t)__shfl((int)t_code, lane - 1, 64);
        const uint32_t cxb = (uint32_t)__shfl((int)h_code, 24 + 3 * f1 + 1, 64);
        const uint32_t cya = (uint32_t)__shfl((int)t_code, lane - 8, 64);
        const uint32_t cyb = (uint32_t)__shfl((int)h_code, 8 + f0, 64);
        const uint32_t cu0 = f0 >= 1 ? cxa : cxb, cu1 = f1 >= 1 ? cya : cyb;
        const uint32_t code = t_code;
        if (t_c >= 0 && (code & kSolidBit)) {
            const uint32_t ab0 = axis_bits(code, 0), ab1 = axis_bits(code, 1);
            const bool hu0 = side_is_cell(ab0, -sg0), hu1 = side_is_cell(ab1, -sg1);
            const bool hu20 = hu0 && side_is_cell(axis_bits(cu0, 0), -sg0);
            const bool hu21 = hu1 && side_is_cell(axis_bits(cu1, 1), -sg1);
            uint32_t wd = W_SOLID;
            if (hu20) wd |= W_HU20;
            if (hu21) wd |= W_HU21;
            if (hu20 && side_is_cell(ab0, sg0)) wd |= W_FX;
            if (hu21 && side_is_cell(ab1, sg1)) wd |= W_FY;
            if (hu0 && !side_wraps(ab0, -sg0)) wd |= W_CX;
            if (hu1 && !side_wraps(ab1, -sg1)) wd |= W_CY;
            if (!hu0 && side_record(ab0, -sg0)) wd |= W_DX;   // diffuse wall or interface
            if (!hu1 && side_record(ab1, -sg1)) wd |= W_DY;
            t_w = wd;
        }
        const bool sol = t_w & W_SOLID;
        t_tl = sol ? (T)t_tld : (T)0;
        t_gam = sol ? (T)t_gamd : (T)0;
        t_qs = sol ? (T)(t_qsd / it.Ctot) : (T)0;
        t_x = sol ? (T)t_xd : (T)0;
        h_x = (T)(h_xd + h_j);
    }
    T *const px = &sPC[w][0][0], *const pgam = &sPC[w][1][0], *const ptl = &sPC[w][2][0],
            *const pqs = &sPC[w][3][0], *const phx = &sHX[w][0];
    px[lane] = t_x;
    pgam[lane] = t_gam;
    ptl[lane] = t_tl;
    pqs[lane] = t_qs;
    phx[lane] = h_x;
    const T A0 = cp0 + cp1 + itau;
    // x of the cells of row q (tile row, or halo row -2, -1, e1)
    auto row_xp = [&](int q) -> const T * {
        return (q >= 0 && q < e1) ? px + 8 * q : phx + (q == -2 ? 0 : (q == -1 ? 8 : 16));
    };
    auto row_x = [&](int q, int j) -> T { return row_xp(q)[j]; };
    T *const wl = &sStg[w][0][0];   // staging of one row of this wavefront

    // corrected window and x halo
#pragma unroll
    for (int i = 0; i < kWin; ++i) {
        const T *xr = row_xp(rb - 2 + i);
#pragma unroll
        for (int j = 0; j < kTX; ++j) y[i][j] += C4 * xr[j];
    }
    // the first wavefront's seeds: increments of the row upwind of the tile
    // (the previous launch's values; an uncoupled one is dropped by a select:
    // across a periodic face it is the other buffer), handed over like the
    // increments of the other wavefronts
    T dupx[kRW];
#pragma unroll
    for (int i = 0; i < kRW; ++i) {
        const int hx = 24 + 3 * (rb + i);
#pragma unroll
        for (int m = 0; m < 3; ++m) xh[i][m] += C4 * phx[hx + m];
    }
    // seeds of the recurrence (the increments upwind of the tile), in two
    // halves: the previous iterate's corrected values now (the row upwind
    // of the tile into sH by the first wavefront, the x halo into dupx),
    // the new values added once they are read (seeds_new): dr - ym1 and
    // dxr - xh1, exactly as one subtraction
    if (w == 0) {
#pragma unroll
        for (int j = 0; j < kTX; ++j) sH[lane][j] = -y[1][j];
    }
#pragma unroll
    for (int i = 0; i < kRW; ++i) dupx[i] = -xh[i][1];
    // (an uncoupled row seed is dropped by a select: across a periodic face
    // it is the other buffer's value)
    auto seeds_new = [&]() {
        if (w == 0) {
#pragma unroll
            for (int j = 0; j < kTX; ++j) {
                const uint32_t wd = (uint32_t)rl((int)t_w, j);
                sH[lane][j] = (wd & W_CY) ? sH[lane][j] + dr[j] : (T)0;
            }
        }
#pragma unroll
        for (int i = 0; i < kRW; ++i) dupx[i] += dxr[i];
    };
    if constexpr (!QUEUE) seeds_new();
    // thermalizing wall inflow per axis (upwind face of this octant)
    const T Tw0 = C4 * (T)(sg0 > 0 ? it.wallT[0] : it.wallT[1]);
    const T Tw1 = C4 * (T)(sg1 > 0 ? it.wallT[2] : it.wallT[3]);
    const T Tp = C4 * (T)d.poreT;

    // ---- right-hand side of this wavefront's rows and the operands of
    // their recurrence, dv = aa + ry dv(y-upwind) + rx dv(x-upwind) with
    // rx = cp0 rden, ry = cp1 rden where the face is implicitly coupled.  An
    // uncoupled upwind increment is dropped by a zero factor (inside the
    // tile every increment is finite; the seeds are selected)
    T aa[kRW][kTX], rdn[kRW][kTX];
#pragma unroll
    for (int i = 0; i < kRW; ++i) {
        if (i >= nrow) break;
        const int r = rb + i;
        // diffuse-wall inflow values of this row, in groups of eight loads
        // in flight (rows without such walls skip this)
        {
            const uint64_t bx = __ballot((t_w & W_DX) != 0), by = __ballot((t_w & W_DY) != 0);
            uint32_t need = 0;
#pragma unroll
            for (int j = 0; j < kTX; ++j)
                need |= (uint32_t)(((bx >> (8 * r + j)) & 1) << (2 * j)) |
                        (uint32_t)(((by >> (8 * r + j)) & 1) << (2 * j + 1));
            while (need) {
                int sl[8];
                const __attribute__((address_space(1))) double *adr[8];
                const auto *gzd = (const __attribute__((address_space(1))) double *)zd;
                const auto *gdin = (const __attribute__((address_space(1))) double *)din;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    sl[q] = -1;
                    adr[q] = gzd + l;
                    if (need) {
                        const int slot = __builtin_ctz(need);
                        need &= need - 1;
                        const int j = slot >> 1, a = slot & 1, t = 8 * r + j;
                        const uint32_t code = (uint32_t)rl((int)t_code, t);
                        const int f = face_of(a, a == 0 ? -sg0 : -sg1);
                        const int rec = rl(t_db, t) + diffuse_rank2(code, f);
                        sl[q] = slot;
                        adr[q] = gdin + (size_t)rec * nl + l;
                    }
                }
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = *adr[q];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (sl[q] >= 0) wl[sl[q] * 64 + lane] = (T)v[q];
            }
        }
        const T *ym2 = y[i], *ym1 = y[i + 1], *ec = y[i + 2], *yp1 = y[i + 3];
        const T xh0 = xh[i][0], xh1 = xh[i][1], xh2 = xh[i][2];
        const int hx = 24 + 3 * r;
        const int cx2 = rl(h_c, hx + 2);
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            const int t = 8 * r + j;
            const uint32_t wd = (uint32_t)rl((int)t_w, t);
            T num = (T)0, rden = (T)0;
            if (wd & W_SOLID) {
                const T ex2 = j >= 2 ? ec[j - 2] : (j == 1 ? xh1 : xh0);
                const T ex1 = j >= 1 ? ec[j - 1] : xh1;
                const T exd = j + 1 < e0 ? ec[j + 1] : xh2;
                T dx, dy;
                if (wd & W_FX) {
                    dx = delta_fast<T, LIM>(ex2, ex1, ec[j], exd);
                } else {
                    const int c = rl(t_c, t);
                    const uint32_t code = (uint32_t)rl((int)t_code, t);
                    const uint32_t ab0 = axis_bits(code, 0);
                    const bool hu0 = side_is_cell(ab0, -sg0), hd0 = side_is_cell(ab0, sg0);
                    const int cd = hd0 ? (j + 1 < e0 ? rl(t_c, t + 1) : cx2) : -1;
                    const double xd = j + 1 < e0 ? (double)px[t + 1] : (double)phx[hx + 2];
                    T fw = (side_wall(ab0, -sg0) == 0) ? (side_outer(code, 0, -sg0) ? Tw0 : Tp) : (T)0;
                    if (wd & W_DX) fw = wl[(2 * j) * 64 + lane];
                    dx = delta_general<T, LIM>(d, ein, c, code, 0, sg0, hu0, (wd & W_HU20) != 0, hd0, ex2, ex1,
                                               ec[j], exd, fw, cd, xd, (double)px[t], al, l, active, C4, hh0,
                                               ih0, nk);
                }
                if (wd & W_FY) {
                    dy = delta_fast<T, LIM>(ym2[j], ym1[j], ec[j], yp1[j]);
                } else {
                    const int c = rl(t_c, t);
                    const uint32_t code = (uint32_t)rl((int)t_code, t);
                    const uint32_t ab1 = axis_bits(code, 1);
                    const bool hu1 = side_is_cell(ab1, -sg1), hd1 = side_is_cell(ab1, sg1);
                    const int cd = hd1 ? row_c(r + 1, j) : -1;
                    const double xd = (double)row_x(r + 1, j);
                    T fw = (side_wall(ab1, -sg1) == 0) ? (side_outer(code, 1, -sg1) ? Tw1 : Tp) : (T)0;
                    if (wd & W_DY) fw = wl[(2 * j + 1) * 64 + lane];
                    dy = delta_general<T, LIM>(d, ein, c, code, 1, sg1, hu1, (wd & W_HU21) != 0, hd1, ym2[j],
                                               ym1[j], ec[j], yp1[j], fw, cd, xd, (double)px[t], al, l, active,
                                               C4, hh1, ih1, nk);
                }
                const T gam = pgam[t];
                const T itc = itau + gam;
                num = -(cp0 * dx + cp1 * dy) - (ec[j] - C4 * ptl[t]) * itc + C4 * pqs[t];
                const T den = A0 + gam;
                if constexpr (sizeof(T) == 4) rden = __builtin_amdgcn_rcpf(den);
                else rden = (T)1 / den;
            }
            aa[i][j] = num * rden;
            rdn[i][j] = rden;
        }
    }

    if constexpr (QUEUE) {
        // the new values of the upwind tiles: wait for their items, then read
        // (device scope, after the barrier) the row upwind of the tile (first
        // wavefront) and the x halo
        if (threadIdx.x == 0) {
            if (it.upx >= 0) queue_wait(queue, it.upx);
            if (it.upy >= 0) queue_wait(queue, it.upy);
        }
        __syncthreads();
        if (rb == 0) {
            const char *pdr = rowp(eout, -1);
#pragma unroll
            for (int j = 0; j < kTX; ++j) {
                const int jc = j < e0 ? j : e0 - 1;
                const unsigned o = koff + (unsigned)((sx > 0 ? jc : e0 - 1 - jc) * nk) * (unsigned)sizeof(T);
                dr[j] = dev_load(reinterpret_cast<const T *>(pdr + o));
            }
        }
#pragma unroll
        for (int i = 0; i < kRW; ++i) {
            const int c1 = rl(h_c, 24 + 3 * (rb + i) + 1);
            const bool ok = c1 >= 0;
            const char *row =
                reinterpret_cast<const char *>((ok ? static_cast<const T *>(eout) : zrow) + (size_t)(ok ? c1 : 0) * nk);
            dxr[i] = dev_load(reinterpret_cast<const T *>(row + koff));
        }
        seeds_new();
    }

    // ---- upwind recurrence over the tile, handed from wavefront to
    // wavefront (the only serial part; one FMA pair per cell)
    T dv[kRW][kTX];
#pragma unroll
    for (int s = 0; s < kWT; ++s) {
        if (w == s && nrow > 0) {
            T up[kTX];
#pragma unroll
            for (int j = 0; j < kTX; ++j) up[j] = sH[lane][j];
#pragma unroll
            for (int i = 0; i < kRW; ++i) {
                if (i >= nrow) break;
                const uint32_t w0 = (uint32_t)rl((int)t_w, 8 * (rb + i));
                T dl = (w0 & W_CX) ? dupx[i] : (T)0;
#pragma unroll
                for (int j = 0; j < kTX; ++j) {
                    // inside the tile the only uncoupled upwind neighbour is
                    // a pore (or a cell past a ragged edge), whose increment
                    // is exactly zero (aa = rden = 0): no per-cell coupling
                    // test; the seeds on the tile's edges are selected
                    const T rxv = cp0 * rdn[i][j], ryv = cp1 * rdn[i][j];
                    dl = aa[i][j] + ryv * up[j] + rxv * dl;
                    up[j] = dl;
                    dv[i][j] = dl;
                }
            }
#pragma unroll
            for (int j = 0; j < kTX; ++j) sH[lane][j] = up[j];
        }
        if (s + 1 < kWT) __syncthreads();
    }

    // ---- new values, moment partials of the rows (a pore cell keeps its
    // value: its increment is zero and it has no correction).  Both are
    // streamed out (nontemporal stores): no launch reads them back through
    // this L2, and dirty lines left in it would be written back at the end
    // of the launch, in the gap before the next diagonal.
#pragma unroll
    for (int i = 0; i < kRW; ++i) {
        if (i >= nrow) break;
        const int r = rb + i;
        const int b = cbase + rowstep * r;
#pragma unroll
        for (int j = 0; j < kTX; ++j) {
            T en = (T)0;
            if (j < e0) {
                en = y[i + 2][j] + dv[i][j];
                if (active) {
                    if constexpr (QUEUE) dev_store(&eout[(size_t)(b + sx * j) * nk + k], en);
                    else __builtin_nontemporal_store(en, &eout[(size_t)(b + sx * j) * nk + k]);
                }
            }
            wl[j * kWS + lane] = active ? en : (T)0;
        }
        // lane = 8 cell + part: part sums 8 of the 64 lanes (the staged row
        // has a stride of 65 values: the 64 lanes read 64 distinct banks)
        const int j = lane >> 3, p = lane & 7;
        double acc[kMomN] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double x = (double)wl[j * kWS + 8 * p + q];
#pragma unroll
            for (int m = 0; m < kMomN; ++m) acc[m] += lc[q][m][p] * x;
        }
#pragma unroll
        for (int m = 0; m < kMomN; ++m) {
            // sum of the 8 lanes of a cell: quad butterflies, then the two
            // quads of each half row (data-parallel-primitive moves, no LDS)
            double v = acc[m];
            v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
            v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
            v += dpp_f64<0x141>(v);   // row_half_mirror
            acc[m] = v;
        }
        const int t = 8 * r + j;
        const int c = __shfl(t_c, t, 64);
        const uint32_t wd = (uint32_t)__shfl((int)t_w, t, 64);
        const double gm = __shfl(t_gamd, t, 64);
        if (p == 0 && j < e0 && c >= 0) {
            double *o = part + ((size_t)(it.oct * nchunk_oct + it.chunk) * d.nc + c) * kMomN;
            const bool sol = wd & W_SOLID;
            __builtin_nontemporal_store(sol ? acc[0] : 0.0, &o[0]);
            __builtin_nontemporal_store(sol ? acc[1] + gm * acc[0] : 0.0, &o[1]);
            __builtin_nontemporal_store(sol ? acc[2] : 0.0, &o[2]);
            __builtin_nontemporal_store(sol ? acc[3] : 0.0, &o[3]);
            __builtin_nontemporal_store(sol ? acc[4] : 0.0, &o[4]);
        }
    }
    if constexpr (QUEUE) {
        // every wavefront's stores have completed (device scope), then the
        // barrier, then the flag
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) queue_publish(queue, item);
    }
}

template <typename T, int LIM, int RW>
void sweep2d_launch(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev, const double *din,
                    const Sweep2Item *items, int item0, int count, int na_oct, int nchunk_oct, double *part,
                    unsigned *queue, hipStream_t s)
{
    if (queue)
        hipLaunchKernelGGL((k_sweep2d<T, LIM, RW, true>), dim3(count), dim3(64 * (kTY / RW)), 0, s, d, ein, eout,
                           dpend, TLdev, din, items, 0, na_oct, nchunk_oct, part, queue);
    else
        hipLaunchKernelGGL((k_sweep2d<T, LIM, RW, false>), dim3(count), dim3(64 * (kTY / RW)), 0, s, d, ein, eout,
                           dpend, TLdev, din, items, item0, na_oct, nchunk_oct, part, queue);
}

// Sweep of the items [item0, item0 + count) (one tile diagonal) with rw
// tile rows per wavefront (1, 2 or 4).
// queue: null for one tile diagonal (items [item0, item0 + count)); else
// the whole sweep in one launch (items [0, count) in sweep order, queue
// words zeroed by launch_queue_reset on the same stream).
template <typename T>
hipError_t launch_sweep2d(const Dev &d, const T *ein, T *eout, const double *dpend, const double *TLdev,
                          const double *din, const Sweep2Item *items, int item0, int count, int rw, int na_oct,
                          int nchunk_oct, double *part, unsigned *queue, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (rw != 1 && rw != 2 && rw != 4) return hipErrorInvalidValue;
#define BTE_S2(LIM, RW)                                                                                              \
    if (d.limiter == LIM && rw == RW)                                                                                \
        sweep2d_launch<T, LIM, RW>(d, ein, eout, dpend, TLdev, din, items, item0, count, na_oct, nchunk_oct, part,   \
                                   queue, s);
    BTE_S2(LIM_NONE, 1) BTE_S2(LIM_NONE, 2) BTE_S2(LIM_NONE, 4)
    BTE_S2(LIM_MC, 1) BTE_S2(LIM_MC, 2) BTE_S2(LIM_MC, 4)
    BTE_S2(LIM_MINMOD, 1) BTE_S2(LIM_MINMOD, 2) BTE_S2(LIM_MINMOD, 4)
#undef BTE_S2
    return hipGetLastError();
}

template hipError_t launch_sweep2d<float>(const Dev &, const float *, float *, const double *, const double *,
                                          const double *, const Sweep2Item *, int, int, int, int, int, double *,
                                          unsigned *, hipStream_t);
template hipError_t launch_sweep2d<double>(const Dev &, const double *, double *, const double *, const double *,
                                           const double *, const Sweep2Item *, int, int, int, int, int, double *,
                                           unsigned *, hipStream_t);

// Zero the queue words of a one-launch sweep of n items (a kernel, not a
// memset: the sweep launches are replayed from graphs).
hipError_t launch_queue_reset(unsigned *queue, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_reset, dim3((n + kQueueDone + 255) / 256), dim3(256), 0, s, queue, n);
    return hipGetLastError();
}

}  // namespace bte
