// bte_mesh.hip -- the BTE on unstructured meshes: two-dimensional meshes of
// triangles and quadrilaterals, three-dimensional meshes of tetrahedra
// (Sec. 3.3, eq. disretized_BTE: second-order
// upwind face values from least-squares gradients on the right-hand side,
// the first-order upwind stiffness matrix of Sec. 3.5 on the left; the
// sequential scheme of Sec. 3.4).
//
// Host: per-cell areas and centroids, face lengths / normals / offsets, the
// least-squares stencils (cells sharing a vertex, or the face neighbours)
// and matrices (pseudo-inverse where the offsets do not span the plane),
// diffuse-wall records, directions, and the sweep schedule:
// for every direction the cells' upwind dependency graph is levelled (Kahn
// order; a cycle is broken at its smallest-index cell, whose unresolved
// upwind couplings are lagged), and the (direction, cell) items of all
// directions are launched level by level.
//
// Device: e[cell][direction][band] as for the structured grids.  One
// iteration = moments (T_L) -> gradients -> diffuse-wall inflow ->
// residual R -> level launches, each thread one (direction, cell, band)
// item: de = (R + sum_upwind v |s.n| S/V de_j) / (1/tau + sum_out v s.n S/V)
// with the geometric sums and the upwind cells of the (direction, cell)
// item precomputed on the host, the increments replacing R in place,
// e += de.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"

namespace bte {
namespace {

// doubles per face slot: S/V, n (3), l = x_f - x_i (3), d = x_j - x_i (3)
// (two-dimensional meshes: z components zero)
constexpr int kFG = 10;

struct MeshDev {
    int nc, na, nl, nk;
    const int *fptr;       // [nc + 1] face slots of each cell
    const int *fnb;        // [nf] neighbour across the face, -1 at a boundary
    const int *ftag;       // [nf] boundary tag, -1 inside
    const int *frec;       // [nf] diffuse-wall record, -1 otherwise
    const double *fgeo;    // [nf][kFG]
    const double *xinv;    // [nc][6] symmetric X^+: 00, 01, 02, 11, 12, 22
    const int *lsptr;      // [nc + 1] least-squares stencil of each cell
    const int *lsnb;       // [nls] stencil cells
    const int *vorder;     // [nc] cell visited by the i-th block group
    const double *lsd;     // [nls][3] offsets x_j - x_i
    const int *tag_bc;     // [ntag]
    const double *tag_dT;  // [ntag] wall temperature - T_ref
    const double *s;       // [na][3]
    const double *w;       // [na]
    const int *mirror;     // [3][na]: flip s_x, s_y, s_z
    const double *C4, *v, *itau;   // [nl]
    double Ctot, Ssum;
    const double *P;       // [nc] heat source or null
    const int *rec_cell, *rec_face;   // [nrec]
    const double *rec_den;            // [nrec] sum_{s.n<0} w |s.n|
    // sweep items by level: cell, direction, the outflow sum
    // sum_{s.n>0} s.n S/V, and up to four upwind couplings (interior inflow
    // faces not lagged): upwind cell (-1: none) and |s.n| S/V
    const int *item_c, *item_al;
    const double *item_out;
    const int4 *item_up;
    const double4 *item_coef;
};

// Lane k of a cell's row.  BUF (FP32 states below 2 GiB): one buffer
// descriptor over the whole state, the row's byte offset as the scalar
// offset and the lane's as the vector offset, so that a row costs no vector
// address arithmetic; otherwise a plain load.
template <typename T, bool BUF>
struct RowReader {
    const T *e;
    int nk, k;
    __amdgpu_buffer_rsrc_t r;
    __device__ RowReader(const T *e_, int nk_, int k_, int nc) : e(e_), nk(nk_), k(k_)
    {
        if constexpr (BUF) r = __builtin_amdgcn_make_buffer_rsrc((void *)e_, (short)0, nk_ * nc * 4, 0x00020000);
    }
    __device__ T operator()(int c) const
    {
        if constexpr (BUF && sizeof(T) == 4)
            return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, k * 4, c * nk * 4, 0));
        else
            return e[(size_t)c * nk + k];
    }
};

// gradient of lane k of cell c: D components at g[(c * D + q) * nk + k]
template <typename T, int D, bool BUF>
__global__ __launch_bounds__(kBlock) void k_mesh_grad(MeshDev d, const T *__restrict__ e, T *__restrict__ g, int nkb)
{
    // block = (cell, block of 256 lanes); cells in the Morton visit order
    const int i = blockIdx.x / nkb;
    const int c = d.vorder[i];
    const int k = (blockIdx.x - i * nkb) * kBlock + threadIdx.x;
    if (k >= d.nk) return;
    const RowReader<T, BUF> row(e, d.nk, k, d.nc);
    const double ec = (double)row(c);
    double y[3] = {0.0, 0.0, 0.0};
    // stencil rows eight, then four at a time in flight (the loads do not
    // wait on each other's sums), summed in stencil order; the row indices
    // and offsets are read through pointers that step by whole groups, so
    // that each group costs one scalar address computation; a row's load is
    // read by RowReader
    const int j0 = d.lsptr[c];
    int n = d.lsptr[c + 1] - j0;
    const int *nbp = d.lsnb + j0;
    const double *ldp = d.lsd + 3 * (size_t)j0;
    const size_t nk = (size_t)d.nk;
    for (; n >= 8; n -= 8, nbp += 8, ldp += 24) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = row(nbp[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double diff = (double)v[u] - ec;
#pragma unroll
            for (int q = 0; q < D; ++q) y[q] += ldp[3 * u + q] * diff;
        }
    }
    if (n >= 4) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = row(nbp[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double diff = (double)v[u] - ec;
#pragma unroll
            for (int q = 0; q < D; ++q) y[q] += ldp[3 * u + q] * diff;
        }
        n -= 4;
        nbp += 4;
        ldp += 12;
    }
    for (; n > 0; --n, ++nbp, ldp += 3) {
        const double diff = (double)row(*nbp) - ec;
#pragma unroll
        for (int q = 0; q < D; ++q) y[q] += ldp[q] * diff;
    }
    const double *xi = d.xinv + 6 * (size_t)c;
    const double gx = xi[0] * y[0] + xi[1] * y[1] + xi[2] * y[2];
    const double gy = xi[1] * y[0] + xi[3] * y[1] + xi[4] * y[2];
    g[((size_t)c * D) * d.nk + k] = (T)gx;
    g[((size_t)c * D + 1) * d.nk + k] = (T)gy;
    if constexpr (D == 3) g[((size_t)c * D + 2) * d.nk + k] = (T)(xi[2] * y[0] + xi[4] * y[1] + xi[5] * y[2]);
}

// outgoing second-order face value of lane k of cell c at the offset l of
// the face centre from the cell centre
template <typename T, int D>
__device__ inline double face_out(const MeshDev &d, const T *__restrict__ e, const T *__restrict__ g, int c, int k,
                                  double lx, double ly, double lz)
{
    double v = (double)e[(size_t)c * d.nk + k] + (double)g[((size_t)c * D) * d.nk + k] * lx +
               (double)g[((size_t)c * D + 1) * d.nk + k] * ly;
    if constexpr (D == 3) v += (double)g[((size_t)c * D + 2) * d.nk + k] * lz;
    return v;
}

// Diffuse-wall inflow per record and band: outgoing energy flux of the face
// over the incoming quadrature weight (one block per record).
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_mesh_walls(MeshDev d, const T *__restrict__ e, const T *__restrict__ g,
                                                       double *__restrict__ din)
{
    __shared__ double sh[kBlock];
    const int r = blockIdx.x;
    const int c = d.rec_cell[r], f = d.rec_face[r];
    const double *fg = d.fgeo + (size_t)f * kFG;
    const int G = kBlock / d.nl;
    const int grp = threadIdx.x / d.nl, l = threadIdx.x - grp * d.nl;
    double sum = 0.0;
    if (grp < G)
        for (int al = grp; al < d.na; al += G) {
            const double sn = d.s[3 * al] * fg[1] + d.s[3 * al + 1] * fg[2] + d.s[3 * al + 2] * fg[3];
            if (sn > 0.0) sum += d.w[al] * sn * face_out<T, D>(d, e, g, c, al * d.nl + l, fg[4], fg[5], fg[6]);
        }
    sh[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x < d.nl) {
        double t = 0.0;
        for (int g2 = 0; g2 < G; ++g2) t += sh[g2 * d.nl + threadIdx.x];
        din[(size_t)r * d.nl + threadIdx.x] = t / d.rec_den[r];
    }
}

// Face sum of a cell whose NF faces are all interior (the common cell):
// every face's loads are issued before the sums, which run in face order,
// and the upwind side is picked per lane without branches (a lane with
// s.n = 0 adds zero).
template <typename T, int D, int NF>
__device__ inline double interior_flux(const MeshDev &d, const T *__restrict__ e, const T *__restrict__ g, int c,
                                       int k, int f0, const int *nbv, double sx, double sy, double sz)
{
    double sn[NF], ev[NF], gv[NF][3], lo[NF][3];
#pragma unroll
    for (int u = 0; u < NF; ++u) {
        const double *fg = d.fgeo + (size_t)(f0 + u) * kFG;
        sn[u] = sx * fg[1] + sy * fg[2] + sz * fg[3];
        const bool own = sn[u] > 0.0;
        const int src = own ? c : nbv[u];
        // offset of the face centre from the upwind cell's centre
        const double m = own ? 0.0 : 1.0;
#pragma unroll
        for (int q = 0; q < D; ++q) lo[u][q] = fg[4 + q] - m * fg[7 + q];
        ev[u] = (double)e[(size_t)src * d.nk + k];
#pragma unroll
        for (int q = 0; q < D; ++q) gv[u][q] = (double)g[((size_t)src * D + q) * d.nk + k];
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < NF; ++u) {
        double ef = ev[u] + gv[u][0] * lo[u][0] + gv[u][1] * lo[u][1];
        if constexpr (D == 3) ef += gv[u][2] * lo[u][2];
        acc += sn[u] * d.fgeo[(size_t)(f0 + u) * kFG] * ef;
    }
    return acc;
}

// R = -(1/V) sum_f v (s.n) S e_f - (e - C4 T_L) / tau + C4 P / C_tot
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_mesh_residual(MeshDev d, const T *__restrict__ e, const T *__restrict__ g,
                                                          const double *__restrict__ din,
                                                          const double *__restrict__ TLdev, T *__restrict__ R,
                                                          int nkb)
{
    const int i = blockIdx.x / nkb;
    const int c = d.vorder[i];
    const int k = (blockIdx.x - i * nkb) * kBlock + threadIdx.x;
    if (k >= d.nk) return;
    const int al = k / d.nl, l = k - al * d.nl;
    const double sx = d.s[3 * al], sy = d.s[3 * al + 1], sz = d.s[3 * al + 2];
    double acc = 0.0;
    const int f0 = d.fptr[c], f1 = d.fptr[c + 1];
    const int nf = f1 - f0;
    int nbv[4] = {-1, -1, -1, -1};
    // tetrahedra: four faces; polygons: triangles and quadrilaterals
    bool inner = nf == 4 || (D == 2 && nf == 3);
    if (inner) {
#pragma unroll
        for (int u = 0; u < 3; ++u) nbv[u] = d.fnb[f0 + u];
        if (nf == 4) nbv[3] = d.fnb[f0 + 3];
        inner = nbv[0] >= 0 && nbv[1] >= 0 && nbv[2] >= 0 && (nf == 3 || nbv[3] >= 0);
    }
    if (inner) {
        if constexpr (D == 3)
            acc = interior_flux<T, D, 4>(d, e, g, c, k, f0, nbv, sx, sy, sz);
        else
            acc = nf == 4 ? interior_flux<T, D, 4>(d, e, g, c, k, f0, nbv, sx, sy, sz)
                          : interior_flux<T, D, 3>(d, e, g, c, k, f0, nbv, sx, sy, sz);
    }
    for (int f = inner ? f1 : f0; f < f1; ++f) {
        const double *fg = d.fgeo + (size_t)f * kFG;
        const double sn = sx * fg[1] + sy * fg[2] + sz * fg[3];
        const int nb = d.fnb[f];
        double ef;
        if (nb >= 0) {
            // interior face: the upwind cell per lane, so that the lanes of
            // a wave issue one set of loads whichever side is upwind (a lane
            // with s.n = 0 adds zero)
            const bool own = sn > 0.0;
            ef = face_out<T, D>(d, e, g, own ? c : nb, k, own ? fg[4] : fg[4] - fg[7], own ? fg[5] : fg[5] - fg[8],
                                own ? fg[6] : fg[6] - fg[9]);
        } else if (sn > 0.0) {
            ef = face_out<T, D>(d, e, g, c, k, fg[4], fg[5], fg[6]);
        } else if (sn < 0.0) {
            const int tag = d.ftag[f];
            const int kind = d.tag_bc[tag];
            if (kind == BTE_BC_THERMAL) {
                ef = d.C4[l] * d.tag_dT[tag];
            } else if (kind == BTE_BC_SPECULAR) {
                // the wall's normal axis (the face is normal to x, y or z)
                const int axis = fabs(fg[1]) > 0.5 ? 0 : (fabs(fg[2]) > 0.5 ? 1 : 2);
                const int km = d.mirror[axis * d.na + al] * d.nl + l;
                ef = face_out<T, D>(d, e, g, c, km, fg[4], fg[5], fg[6]);
            } else {
                ef = din[(size_t)d.frec[f] * d.nl + l];
            }
        } else {
            continue;
        }
        acc += sn * fg[0] * ef;
    }
    const double ec = (double)e[(size_t)c * d.nk + k];
    double r = -d.v[l] * acc - (ec - d.C4[l] * TLdev[c]) * d.itau[l];
    if (d.P) r += d.C4[l] * d.P[c] / d.Ctot;
    R[(size_t)c * d.nk + k] = (T)r;
}

// One level of the sweep: thread = (item, band).  b holds R on entry and the
// increment de once the item is done (read by the downwind items of later
// levels); e += de.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mesh_sweep_level(MeshDev d, T *__restrict__ e, T *__restrict__ b,
                                                             int item0, int nitems)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= nitems * d.nl) return;
    const int q = t / d.nl;
    const int i = item0 + q, l = t - q * d.nl;
    const int c = d.item_c[i];
    const int k = d.item_al[i] * d.nl + l;
    const int4 up = d.item_up[i];
    const double4 cf = d.item_coef[i];
    const double vl = d.v[l], den = d.itau[l] + vl * d.item_out[i];
    const size_t nk = (size_t)d.nk, ck = (size_t)c * nk + k;
    // an absent coupling (-1) reads the item's own slot with weight zero, so
    // that every load of the item issues at once, without branches
    const T b0 = b[ck], e0 = e[ck];
    const T bx = b[(size_t)(up.x >= 0 ? up.x : c) * nk + k];
    const T by = b[(size_t)(up.y >= 0 ? up.y : c) * nk + k];
    const T bz = b[(size_t)(up.z >= 0 ? up.z : c) * nk + k];
    const T bw = b[(size_t)(up.w >= 0 ? up.w : c) * nk + k];
    double num = (double)b0;
    num += (up.x >= 0 ? vl * cf.x : 0.0) * (double)bx;
    num += (up.y >= 0 ? vl * cf.y : 0.0) * (double)by;
    num += (up.z >= 0 ? vl * cf.z : 0.0) * (double)bz;
    num += (up.w >= 0 ? vl * cf.w : 0.0) * (double)bw;
    const double de = num / den;
    b[ck] = (T)de;
    e[ck] = (T)((double)e0 + de);
}

// Moments per cell: T - T_ref, T_L - T_ref and q.  A block takes
// kMomCells cells, so that each lane's direction and band weights serve all
// of them; wave sums by shuffles, then one pass over the block's waves.
constexpr int kMomCells = 4;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mesh_moments(MeshDev d, const T *__restrict__ e, double *__restrict__ Tdev,
                                                         double *__restrict__ TLdev, double *__restrict__ q)
{
    __shared__ double sh[kBlock / 64][kMomCells][5];
    const int c0 = blockIdx.x * kMomCells;
    double a[kMomCells][5] = {};
    for (int k = threadIdx.x; k < d.nk; k += kBlock) {
        const int al = k / d.nl, l = k - al * d.nl;
        const double w = d.w[al], wv = w * d.v[l];
        const double cw[5] = {w, w * d.itau[l], wv * d.s[3 * al], wv * d.s[3 * al + 1], wv * d.s[3 * al + 2]};
        T ev[kMomCells];
        // past the last cell the loads repeat it and the sums are dropped
#pragma unroll
        for (int m = 0; m < kMomCells; ++m) ev[m] = e[(size_t)min(c0 + m, d.nc - 1) * d.nk + k];
#pragma unroll
        for (int m = 0; m < kMomCells; ++m)
#pragma unroll
            for (int j = 0; j < 5; ++j) a[m][j] += cw[j] * (double)ev[m];
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < kMomCells; ++m)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            double x = a[m][j];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            if (lane == 0) sh[wv][m][j] = x;
        }
    __syncthreads();
    if ((int)threadIdx.x < kMomCells * 5) {
        const int m = threadIdx.x / 5, j = threadIdx.x - 5 * m, c = c0 + m;
        double t = 0.0;
        for (int u = 0; u < kBlock / 64; ++u) t += sh[u][m][j];
        if (c < d.nc) {
            if (j == 0 && Tdev) Tdev[c] = t / d.Ctot;
            if (j == 1 && TLdev) TLdev[c] = t / d.Ssum;
            if (j >= 2 && q) q[3 * c + j - 2] = t;
        }
    }
}

// grid of k_mesh_moments over nc cells
static inline dim3 mom_grid(int nc) { return dim3((unsigned)((nc + kMomCells - 1) / kMomCells)); }

// explicit step e += dt R
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mesh_axpy(size_t n, T *__restrict__ e, const T *__restrict__ R, double dt)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        e[i] = (T)((double)e[i] + dt * (double)R[i]);
}

// max |T1 - T0| and max |T1| (deviations) in two passes: kEpsBlocks blocks
// write their maxima to part[2 * block + {0, 1}], then one block of kBlock
// (= kEpsBlocks) threads reduces those into out[0], out[1]
constexpr int kEpsBlocks = kBlock;
__device__ inline void block_max2(double &a, double &b, double *out)
{
    __shared__ double sh[2][kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a = fmax(a, __shfl_xor(a, off, 64));
        b = fmax(b, __shfl_xor(b, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = a;
        sh[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = sh[0][0], y = sh[1][0];
        for (int w = 1; w < kBlock / 64; ++w) {
            x = fmax(x, sh[0][w]);
            y = fmax(y, sh[1][w]);
        }
        out[0] = x;
        out[1] = y;
    }
}

__global__ __launch_bounds__(kBlock) void k_mesh_eps(int nc, const double *__restrict__ T0,
                                                     const double *__restrict__ T1, double *__restrict__ part)
{
    double a = 0.0, b = 0.0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < nc; c += kEpsBlocks * kBlock) {
        a = fmax(a, fabs(T1[c] - T0[c]));
        b = fmax(b, fabs(T1[c]));
    }
    block_max2(a, b, part + 2 * blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_mesh_eps_final(const double *__restrict__ part, double *__restrict__ out)
{
    double a = part[2 * threadIdx.x], b = part[2 * threadIdx.x + 1];
    block_max2(a, b, out);
}

// T_abs = T_ref + dev
__global__ void k_mesh_abs(int n, double Tref, const double *__restrict__ dev, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = Tref + dev[i];
}

}  // namespace
}  // namespace bte

using namespace bte;

struct bte_mesh_problem {
    bte_control ctl{};
    std::string err;
    int nc = 0, na = 0, nl = 0, nk = 0, nf = 0, nrec = 0, ntag = 0, nlev = 0, nlag = 0, dim = 2;
    double Tref = 0;
    // host tables
    std::vector<int> fptr, fnb, ftag, frec, tag_bc, mirror, rec_cell, rec_face, lev_off, lsptr, lsnb, vorder;
    std::vector<int> item_c, item_al;
    std::vector<int4> item_up;
    std::vector<double4> item_coef;
    std::vector<double> fgeo, xinv, lsd, tag_dT, s, w, C4, v, itau, rec_den, item_out;
    double Ctot = 0, Ssum = 0;
    double vmax = 0, itau_max = 0, sv_max = 0;   // stability bound of the explicit step
    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    MeshDev dev{};
    void *g = nullptr, *b = nullptr;
    double *din = nullptr, *Tdev = nullptr, *Tprev = nullptr, *TLdev = nullptr, *P = nullptr, *eps = nullptr, *eps_part = nullptr;
    bool hasP = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // phase timers of the steady solve
    ~bte_mesh_problem()
    {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
    }
    size_t esize() const { return ctl.precision == BTE_F64 ? 8 : 4; }
    size_t nelem() const { return (size_t)nc * nk; }
};

namespace {

#define MFAIL(p, st, ...)                                                                                              \
    do {                                                                                                               \
        char _b[512];                                                                                                  \
        snprintf(_b, sizeof _b, __VA_ARGS__);                                                                          \
        (p)->err = _b;                                                                                                 \
        return st;                                                                                                     \
    } while (0)

#define MHIP(p, x)                                                                                                     \
    do {                                                                                                               \
        hipError_t _e = (x);                                                                                           \
        if (_e != hipSuccess) MFAIL(p, BTE_ERR_HIP, "%s: %s", #x, hipGetErrorString(_e));                              \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Symmetric pseudo-inverse, eigenvalues below 1e-10 of the largest dropped.
// 2 x 2 [[xx, xy], [xy, yy]] in closed form; out = 00, 01, 02, 11, 12, 22.
void pinv2(double xx, double xy, double yy, double out[6])
{
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    const double h = 0.5 * (xx + yy), r = std::sqrt(0.25 * (xx - yy) * (xx - yy) + xy * xy);
    const double l1 = h + r, l2 = h - r;
    if (!(l1 > 0)) return;
    if (l2 > 1e-10 * l1) {
        const double det = xx * yy - xy * xy;
        out[0] = yy / det;
        out[1] = -xy / det;
        out[3] = xx / det;
        return;
    }
    // rank one: X^+ = u u^T / l1 with u the unit eigenvector of l1
    double ux = xy, uy = l1 - xx, vx = l1 - yy, vy = xy;
    if (vx * vx + vy * vy > ux * ux + uy * uy) ux = vx, uy = vy;
    const double n = std::sqrt(ux * ux + uy * uy);
    ux /= n;
    uy /= n;
    out[0] = ux * ux / l1;
    out[1] = ux * uy / l1;
    out[3] = uy * uy / l1;
}

// 3 x 3 by cyclic Jacobi rotations (to machine precision), then
// X^+ = sum over kept eigenpairs of u u^T / lambda.
void pinv3(const double X[3][3], double out[6])
{
    double A[3][3], U[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = X[i][j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-32 * dia) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int pi = pq == 2 ? 1 : 0, qi = pq == 0 ? 1 : 2;
            if (A[pi][qi] == 0.0) continue;
            const double th = 0.5 * (A[qi][qi] - A[pi][pi]) / A[pi][qi];
            const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
            const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
            for (int k = 0; k < 3; ++k) {   // A <- A R (columns pi, qi)
                const double akp = A[k][pi], akq = A[k][qi];
                A[k][pi] = cs * akp - sn * akq;
                A[k][qi] = sn * akp + cs * akq;
            }
            for (int k = 0; k < 3; ++k) {   // A <- R^T A (rows pi, qi)
                const double apk = A[pi][k], aqk = A[qi][k];
                A[pi][k] = cs * apk - sn * aqk;
                A[qi][k] = sn * apk + cs * aqk;
            }
            for (int k = 0; k < 3; ++k) {   // U <- U R
                const double ukp = U[k][pi], ukq = U[k][qi];
                U[k][pi] = cs * ukp - sn * ukq;
                U[k][qi] = sn * ukp + cs * ukq;
            }
        }
    }
    const double lmax = std::max(A[0][0], std::max(A[1][1], A[2][2]));
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    if (!(lmax > 0)) return;
    const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int m = 0; m < 3; ++m) {
        const double lm = A[m][m];
        if (!(lm > 1e-10 * lmax)) continue;
        for (int i = 0; i < 6; ++i) out[i] += U[idx[i][0]][m] * U[idx[i][1]][m] / lm;
    }
}

bte_status mesh_tags(bte_mesh_problem *p, int n_tags, const int *tag_bc, const double *tag_T,
                     const bte_material *mat)
{
    if (n_tags < 0 || (n_tags > 0 && (!tag_bc || !tag_T))) MFAIL(p, BTE_ERR_ARG, "mesh: bad tags");
    p->ntag = n_tags;
    p->Tref = mat->T_ref;
    for (int t = 0; t < n_tags; ++t) {
        const int k = tag_bc[t];
        if (k != BTE_BC_THERMAL && k != BTE_BC_SPECULAR && k != BTE_BC_DIFFUSE)
            MFAIL(p, BTE_ERR_ARG, "mesh: tag %d: boundary condition must be thermal, specular or diffuse", t);
        p->tag_bc.push_back(k);
        p->tag_dT.push_back(tag_T[t] - mat->T_ref);
    }
    return BTE_OK;
}

// Cells sorted by the Morton (Z-order) code of their centroids, quantised to
// 2^10 steps per axis of the bounding box: consecutive blocks of the
// gradient and residual launches then read the rows of nearby cells, which
// the previous blocks have just brought into the L2 cache (the stored cell
// numbering may follow one axis, putting a neighbour across the slowest axis
// a whole layer of cells away).  Ties keep the stored order.
static void morton_order(const std::vector<double> &xc, int nc, int D, std::vector<int> &order)
{
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int q = 0; q < D; ++q) {
        lo[q] = hi[q] = nc > 0 ? xc[q] : 0.0;
        for (int c = 1; c < nc; ++c) {
            lo[q] = std::min(lo[q], xc[3 * (size_t)c + q]);
            hi[q] = std::max(hi[q], xc[3 * (size_t)c + q]);
        }
    }
    std::vector<unsigned long long> key(nc);
    for (int c = 0; c < nc; ++c) {
        unsigned long long code = 0;
        unsigned u[3] = {0, 0, 0};
        for (int q = 0; q < D; ++q) {
            const double span = hi[q] - lo[q];
            const double t = span > 0.0 ? (xc[3 * (size_t)c + q] - lo[q]) / span : 0.0;
            u[q] = (unsigned)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)));
        }
        for (int b = 9; b >= 0; --b)
            for (int q = 0; q < D; ++q) code = (code << 1) | ((u[q] >> b) & 1u);
        key[c] = code;
    }
    order.resize(nc);
    for (int c = 0; c < nc; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
}

// Everything after the cells' geometry: least-squares stencils and
// matrices, directions, bands, diffuse-wall records and the sweep schedule.
// V, xc (3 per cell), the face slots in p, and the vertices of each cell
// (cptr / cvtx, for the vertex stencil) are given.
bte_status mesh_finish(bte_mesh_problem *p, const bte_material *mat, int stencil, const std::vector<double> &xc,
                       const std::vector<int> &cptr, const std::vector<int> &cvtx, int nvert)
{
    const int nc = p->nc, D = p->dim;
    if (stencil != 0 && stencil != 1) MFAIL(p, BTE_ERR_ARG, "mesh: gradient_stencil 0 or 1");
    std::vector<std::vector<int>> vcells;
    if (stencil == 0) {
        vcells.assign(nvert, {});
        for (int c = 0; c < nc; ++c)
            for (int f = cptr[c]; f < cptr[c + 1]; ++f) vcells[cvtx[f]].push_back(c);
    }
    p->lsptr.assign(1, 0);
    for (int c = 0; c < nc; ++c) {
        std::vector<int> near;
        if (stencil == 0) {
            for (int f = cptr[c]; f < cptr[c + 1]; ++f)
                for (int j : vcells[cvtx[f]])
                    if (j != c) near.push_back(j);
        } else {
            for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f)
                if (p->fnb[f] >= 0) near.push_back(p->fnb[f]);
        }
        std::sort(near.begin(), near.end());
        near.erase(std::unique(near.begin(), near.end()), near.end());
        for (int j : near) {
            p->lsnb.push_back(j);
            for (int q = 0; q < 3; ++q) p->lsd.push_back(xc[3 * j + q] - xc[3 * c + q]);
        }
        p->lsptr.push_back((int)p->lsnb.size());
    }
    p->xinv.assign(6 * (size_t)nc, 0.0);
    for (int c = 0; c < nc; ++c) {
        double X[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int j = p->lsptr[c]; j < p->lsptr[c + 1]; ++j)
            for (int a = 0; a < 3; ++a)
                for (int b2 = 0; b2 < 3; ++b2) X[a][b2] += p->lsd[3 * (size_t)j + a] * p->lsd[3 * (size_t)j + b2];
        if (D == 2) pinv2(X[0][0], X[0][1], X[1][1], &p->xinv[6 * (size_t)c]);
        else pinv3(X, &p->xinv[6 * (size_t)c]);
    }
    morton_order(xc, nc, D, p->vorder);
    // directions (bulk material: on the sphere, 4 pi)
    if (mat->n_theta < 1 || mat->n_phi < 1) MFAIL(p, BTE_ERR_ARG, "n_theta and n_phi must be >= 1");
    sphere_directions(mat->n_theta, mat->n_phi, 4.0 * M_PI, p->s, p->w);
    p->na = (int)p->w.size();
    p->nl = mat->n_bands;
    p->nk = p->na * p->nl;
    if ((double)p->na * nc >= 2147483647.0) MFAIL(p, BTE_ERR_ARG, "mesh: directions x cells must stay below 2^31");
    p->mirror.assign(3 * (size_t)p->na, 0);
    for (int a = 0; a < 3; ++a)
        for (int al = 0; al < p->na; ++al) {
            double t[3] = {p->s[3 * al], p->s[3 * al + 1], p->s[3 * al + 2]};
            t[a] = -t[a];
            int best = -1;
            double bd = 1e300;
            for (int b2 = 0; b2 < p->na; ++b2) {
                const double dd = std::fabs(p->s[3 * b2] - t[0]) + std::fabs(p->s[3 * b2 + 1] - t[1]) +
                                  std::fabs(p->s[3 * b2 + 2] - t[2]);
                if (dd < bd) bd = dd, best = b2;
            }
            if (bd > 1e-9) MFAIL(p, BTE_ERR_ARG, "quadrature without mirror directions");
            p->mirror[(size_t)a * p->na + al] = best;
        }
    for (int l = 0; l < p->nl; ++l) {
        const double C = mat->C[l], v = mat->v[l], tau = mat->tau[l];
        if (!(C > 0) || !(v >= 0) || !(tau > 0)) MFAIL(p, BTE_ERR_ARG, "band %d: C > 0, v >= 0, tau > 0 required", l);
        p->C4.push_back(C / (4.0 * M_PI));
        p->v.push_back(v);
        p->itau.push_back(1.0 / tau);
        p->Ctot += C;
        p->Ssum += C / tau;
        p->vmax = std::max(p->vmax, v);
        p->itau_max = std::max(p->itau_max, 1.0 / tau);
    }
    for (int c = 0; c < nc; ++c) {
        double sv = 0;
        for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f) sv += p->fgeo[(size_t)f * kFG];
        p->sv_max = std::max(p->sv_max, sv);
    }
    auto sdotn = [&](int al, int f) {
        const double *fg = &p->fgeo[(size_t)f * kFG];
        return p->s[3 * al] * fg[1] + p->s[3 * al + 1] * fg[2] + p->s[3 * al + 2] * fg[3];
    };
    // diffuse-wall records
    std::vector<int> slot_cell(p->nf);
    for (int c = 0; c < nc; ++c)
        for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f) slot_cell[f] = c;
    for (int f = 0; f < p->nf; ++f) {
        if (p->fnb[f] >= 0 || p->tag_bc[p->ftag[f]] != BTE_BC_DIFFUSE) continue;
        double den = 0;
        for (int al = 0; al < p->na; ++al) {
            const double sn = sdotn(al, f);
            if (sn < 0) den += p->w[al] * (-sn);
        }
        p->frec[f] = p->nrec++;
        p->rec_cell.push_back(slot_cell[f]);
        p->rec_face.push_back(f);
        p->rec_den.push_back(den);
    }
    // sweep schedule: per direction, Kahn order with the lagging rule, the
    // level of a cell one more than its deepest non-lagged upwind cell
    std::vector<int> level((size_t)p->na * nc);
    std::vector<uint8_t> lagm((size_t)p->na * nc, 0);
    p->nlag = 0;
    int maxlev = 0;
    for (int al = 0; al < p->na; ++al) {
        std::vector<std::vector<int>> down(nc), deps(nc);
        std::vector<int> indeg(nc, 0);
        for (int c = 0; c < nc; ++c)
            for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f) {
                const int nb = p->fnb[f];
                if (nb < 0) continue;
                if (sdotn(al, f) < 0 && std::find(deps[c].begin(), deps[c].end(), nb) == deps[c].end()) {
                    deps[c].push_back(nb);
                    down[nb].push_back(c);
                }
            }
        for (int c = 0; c < nc; ++c) indeg[c] = (int)deps[c].size();
        std::vector<char> done(nc, 0);
        std::vector<int> ready;
        std::vector<std::pair<int, int>> lagged;
        auto is_lagged = [&](int c, int j) {
            return std::find(lagged.begin(), lagged.end(), std::make_pair(c, j)) != lagged.end();
        };
        for (int c = 0; c < nc; ++c)
            if (indeg[c] == 0) ready.push_back(c);
        size_t head = 0;
        int ndone = 0, lowest = 0;
        while (ndone < nc) {
            if (head == ready.size()) {
                while (done[lowest]) ++lowest;
                const int c = lowest;
                for (int j : deps[c])
                    if (!done[j]) lagged.push_back({c, j});
                indeg[c] = 0;
                ready.push_back(c);
            }
            const int c = ready[head++];
            done[c] = 1;
            ++ndone;
            int lv = 0;
            for (int j : deps[c])
                if (!is_lagged(c, j)) lv = std::max(lv, level[(size_t)al * nc + j] + 1);
            level[(size_t)al * nc + c] = lv;
            maxlev = std::max(maxlev, lv);
            for (int dd : down[c]) {
                if (is_lagged(dd, c)) continue;
                if (--indeg[dd] == 0 && !done[dd]) ready.push_back(dd);
            }
        }
        for (auto &pr : lagged) {
            const int c = pr.first;
            for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f)
                if (p->fnb[f] == pr.second) lagm[(size_t)al * nc + c] |= (uint8_t)(1u << (f - p->fptr[c]));
        }
        p->nlag += (int)lagged.size();
    }
    p->nlev = maxlev + 1;
    std::vector<int> cnt(p->nlev + 1, 0);
    for (size_t i = 0; i < level.size(); ++i) ++cnt[level[i] + 1];
    for (int L = 0; L < p->nlev; ++L) cnt[L + 1] += cnt[L];
    p->lev_off = cnt;
    const size_t ni = level.size();
    p->item_c.assign(ni, 0);
    p->item_al.assign(ni, 0);
    p->item_out.assign(ni, 0.0);
    p->item_up.assign(ni, make_int4(-1, -1, -1, -1));
    p->item_coef.assign(ni, make_double4(0, 0, 0, 0));
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (int al = 0; al < p->na; ++al)
        for (int c = 0; c < nc; ++c) {
            const size_t i = (size_t)al * nc + c;
            const int at = pos[level[i]]++;
            p->item_c[at] = c;
            p->item_al[at] = al;
            int upc[4] = {-1, -1, -1, -1};
            double cof[4] = {0, 0, 0, 0};
            int nu = 0;
            double aout = 0;
            for (int f = p->fptr[c]; f < p->fptr[c + 1]; ++f) {
                const double sn = sdotn(al, f), sv = p->fgeo[(size_t)f * kFG];
                if (sn > 0) {
                    aout += sn * sv;
                } else if (sn < 0 && p->fnb[f] >= 0 && !((lagm[i] >> (f - p->fptr[c])) & 1u)) {
                    upc[nu] = p->fnb[f];
                    cof[nu] = -sn * sv;
                    ++nu;
                }
            }
            p->item_out[at] = aout;
            p->item_up[at] = make_int4(upc[0], upc[1], upc[2], upc[3]);
            p->item_coef[at] = make_double4(cof[0], cof[1], cof[2], cof[3]);
        }
    return BTE_OK;
}

bte_status mesh_build(bte_mesh_problem *p, const bte_mesh *m, const bte_material *mat)
{
    const int nc = m->n_cells;
    if (nc < 1 || m->n_vertices < 3 || !m->xy || !m->cell_ptr || !m->cell_vtx || !m->edge_tag)
        MFAIL(p, BTE_ERR_ARG, "mesh: empty or null arrays");
    if (m->cell_ptr[0] != 0) MFAIL(p, BTE_ERR_ARG, "mesh: cell_ptr[0] must be 0");
    p->nc = nc;
    p->dim = 2;
    bte_status st = mesh_tags(p, m->n_tags, m->tag_bc, m->tag_T, mat);
    if (st != BTE_OK) return st;
    std::vector<double> V(nc), xc(3 * (size_t)nc, 0.0);
    for (int c = 0; c < nc; ++c) {
        const int a = m->cell_ptr[c], b = m->cell_ptr[c + 1], nv = b - a;
        if (nv != 3 && nv != 4) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d has %d vertices (3 or 4)", c, nv);
        double A = 0, cx = 0, cy = 0;
        for (int k = 0; k < nv; ++k) {
            const int i = m->cell_vtx[a + k], j = m->cell_vtx[a + (k + 1) % nv];
            if (i < 0 || i >= m->n_vertices || j < 0 || j >= m->n_vertices)
                MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: vertex index out of range", c);
            const double x0 = m->xy[2 * i], y0 = m->xy[2 * i + 1], x1 = m->xy[2 * j], y1 = m->xy[2 * j + 1];
            const double cr = x0 * y1 - x1 * y0;
            A += cr;
            cx += (x0 + x1) * cr;
            cy += (y0 + y1) * cr;
        }
        A *= 0.5;
        if (!(A > 0)) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d is not counter-clockwise with positive area", c);
        V[c] = A;
        xc[3 * c] = cx / (6.0 * A);
        xc[3 * c + 1] = cy / (6.0 * A);
    }
    const int nf = m->cell_ptr[nc];
    p->nf = nf;
    std::map<std::pair<int, int>, std::vector<int>> owner;   // edge -> face slots
    for (int c = 0; c < nc; ++c) {
        const int a = m->cell_ptr[c], nv = m->cell_ptr[c + 1] - a;
        for (int k = 0; k < nv; ++k) {
            const int i = m->cell_vtx[a + k], j = m->cell_vtx[a + (k + 1) % nv];
            owner[{std::min(i, j), std::max(i, j)}].push_back(a + k);
        }
    }
    std::vector<int> slot_cell(nf);
    for (int c = 0; c < nc; ++c)
        for (int f = m->cell_ptr[c]; f < m->cell_ptr[c + 1]; ++f) slot_cell[f] = c;
    p->fptr.assign(m->cell_ptr, m->cell_ptr + nc + 1);
    p->fnb.assign(nf, -1);
    p->ftag.assign(nf, -1);
    p->frec.assign(nf, -1);
    p->fgeo.assign((size_t)nf * kFG, 0.0);
    for (auto &kv : owner) {
        if (kv.second.size() > 2) MFAIL(p, BTE_ERR_ARG, "mesh: an edge is shared by more than two cells");
        if (kv.second.size() == 2) {
            p->fnb[kv.second[0]] = slot_cell[kv.second[1]];
            p->fnb[kv.second[1]] = slot_cell[kv.second[0]];
        }
    }
    for (int c = 0; c < nc; ++c) {
        const int a = m->cell_ptr[c], nv = m->cell_ptr[c + 1] - a;
        for (int k = 0; k < nv; ++k) {
            const int f = a + k;
            const int i = m->cell_vtx[f], j = m->cell_vtx[a + (k + 1) % nv];
            const double dx = m->xy[2 * j] - m->xy[2 * i], dy = m->xy[2 * j + 1] - m->xy[2 * i + 1];
            const double S = std::hypot(dx, dy);
            if (!(S > 0)) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d has an edge of zero length", c);
            const double nx = dy / S, ny = -dx / S;
            const double xf = 0.5 * (m->xy[2 * i] + m->xy[2 * j]), yf = 0.5 * (m->xy[2 * i + 1] + m->xy[2 * j + 1]);
            double *fg = &p->fgeo[(size_t)f * kFG];
            fg[0] = S / V[c];
            fg[1] = nx;
            fg[2] = ny;
            fg[4] = xf - xc[3 * c];
            fg[5] = yf - xc[3 * c + 1];
            const int nb = p->fnb[f], tag = m->edge_tag[f];
            if (nb >= 0) {
                if (tag >= 0) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: a shared edge carries a boundary tag", c);
                fg[7] = xc[3 * nb] - xc[3 * c];
                fg[8] = xc[3 * nb + 1] - xc[3 * c + 1];
            } else {
                if (tag < 0 || tag >= m->n_tags) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: boundary edge without a valid tag", c);
                p->ftag[f] = tag;
                if (p->tag_bc[tag] == BTE_BC_SPECULAR && std::min(std::fabs(nx), std::fabs(ny)) > 1e-12)
                    MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: specular edge not parallel to x or y", c);
            }
        }
    }
    std::vector<int> cptr(m->cell_ptr, m->cell_ptr + nc + 1), cvtx(m->cell_vtx, m->cell_vtx + nf);
    return mesh_finish(p, mat, m->gradient_stencil, xc, cptr, cvtx, m->n_vertices);
}

// Tetrahedra: face k of a cell is the triangle opposite its vertex k.
bte_status mesh_build_tet(bte_mesh_problem *p, const bte_tet_mesh *m, const bte_material *mat)
{
    const int nc = m->n_cells;
    if (nc < 1 || m->n_vertices < 4 || !m->xyz || !m->cell_vtx || !m->face_tag)
        MFAIL(p, BTE_ERR_ARG, "mesh: empty or null arrays");
    p->nc = nc;
    p->dim = 3;
    bte_status st = mesh_tags(p, m->n_tags, m->tag_bc, m->tag_T, mat);
    if (st != BTE_OK) return st;
    const double *X = m->xyz;
    std::vector<double> V(nc), xc(3 * (size_t)nc);
    for (int c = 0; c < nc; ++c) {
        const int *t = m->cell_vtx + 4 * (size_t)c;
        for (int k = 0; k < 4; ++k)
            if (t[k] < 0 || t[k] >= m->n_vertices) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: vertex index out of range", c);
        double e1[3], e2[3], e3[3];
        for (int q = 0; q < 3; ++q) {
            e1[q] = X[3 * t[1] + q] - X[3 * t[0] + q];
            e2[q] = X[3 * t[2] + q] - X[3 * t[0] + q];
            e3[q] = X[3 * t[3] + q] - X[3 * t[0] + q];
            xc[3 * c + q] = 0.25 * (X[3 * t[0] + q] + X[3 * t[1] + q] + X[3 * t[2] + q] + X[3 * t[3] + q]);
        }
        const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                           e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
        V[c] = std::fabs(det) / 6.0;
        if (!(V[c] > 0)) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d has zero volume", c);
    }
    const int nf = 4 * nc;
    p->nf = nf;
    std::map<std::array<int, 3>, std::vector<int>> owner;   // face -> face slots
    auto face_key = [&](int c, int k) {
        std::array<int, 3> f;
        int q = 0;
        for (int r = 0; r < 4; ++r)
            if (r != k) f[q++] = m->cell_vtx[4 * (size_t)c + r];
        std::sort(f.begin(), f.end());
        return f;
    };
    for (int c = 0; c < nc; ++c)
        for (int k = 0; k < 4; ++k) owner[face_key(c, k)].push_back(4 * c + k);
    p->fptr.resize(nc + 1);
    for (int c = 0; c <= nc; ++c) p->fptr[c] = 4 * c;
    p->fnb.assign(nf, -1);
    p->ftag.assign(nf, -1);
    p->frec.assign(nf, -1);
    p->fgeo.assign((size_t)nf * kFG, 0.0);
    for (auto &kv : owner) {
        if (kv.second.size() > 2) MFAIL(p, BTE_ERR_ARG, "mesh: a face is shared by more than two cells");
        if (kv.second.size() == 2) {
            p->fnb[kv.second[0]] = kv.second[1] / 4;
            p->fnb[kv.second[1]] = kv.second[0] / 4;
        }
    }
    for (int c = 0; c < nc; ++c)
        for (int k = 0; k < 4; ++k) {
            const int f = 4 * c + k;
            int v3[3], q = 0;
            for (int r = 0; r < 4; ++r)
                if (r != k) v3[q++] = m->cell_vtx[4 * (size_t)c + r];
            double a[3], b[3], xf[3];
            for (int i = 0; i < 3; ++i) {
                a[i] = X[3 * v3[1] + i] - X[3 * v3[0] + i];
                b[i] = X[3 * v3[2] + i] - X[3 * v3[0] + i];
                xf[i] = (X[3 * v3[0] + i] + X[3 * v3[1] + i] + X[3 * v3[2] + i]) / 3.0;
            }
            double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            if (!(nn > 0)) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d has a face of zero area", c);
            const int opp = m->cell_vtx[4 * (size_t)c + k];
            double side = 0;
            for (int i = 0; i < 3; ++i) side += n[i] * (xf[i] - X[3 * opp + i]);
            const double sg = side < 0 ? -1.0 : 1.0;   // away from the opposite vertex
            double *fg = &p->fgeo[(size_t)f * kFG];
            fg[0] = 0.5 * nn / V[c];
            for (int i = 0; i < 3; ++i) {
                fg[1 + i] = sg * n[i] / nn;
                fg[4 + i] = xf[i] - xc[3 * c + i];
            }
            const int nb = p->fnb[f], tag = m->face_tag[f];
            if (nb >= 0) {
                if (tag >= 0) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: a shared face carries a boundary tag", c);
                for (int i = 0; i < 3; ++i) fg[7 + i] = xc[3 * nb + i] - xc[3 * c + i];
            } else {
                if (tag < 0 || tag >= m->n_tags) MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: boundary face without a valid tag", c);
                p->ftag[f] = tag;
                double an[3] = {std::fabs(fg[1]), std::fabs(fg[2]), std::fabs(fg[3])};
                std::sort(an, an + 3);
                if (p->tag_bc[tag] == BTE_BC_SPECULAR && an[1] > 1e-12)
                    MFAIL(p, BTE_ERR_ARG, "mesh: cell %d: specular face not normal to x, y or z", c);
            }
        }
    std::vector<int> cptr(nc + 1), cvtx(m->cell_vtx, m->cell_vtx + 4 * (size_t)nc);
    for (int c = 0; c <= nc; ++c) cptr[c] = 4 * c;
    return mesh_finish(p, mat, m->gradient_stencil, xc, cptr, cvtx, m->n_vertices);
}

template <typename T>
void mesh_iteration_rhs(bte_mesh_problem *p, const T *e, const double *TLdev, T *R, hipStream_t s)
{
    const MeshDev &d = p->dev;
    const int nkb = (p->nk + kBlock - 1) / kBlock;
    const dim3 grid((unsigned)((size_t)nkb * p->nc));
    const bool buf = sizeof(T) == 4 && p->nelem() * 4 < (size_t(1) << 31);
    if (p->dim == 3) {
        if (buf)
            hipLaunchKernelGGL((k_mesh_grad<T, 3, true>), grid, dim3(kBlock), 0, s, d, e, (T *)p->g, nkb);
        else
            hipLaunchKernelGGL((k_mesh_grad<T, 3, false>), grid, dim3(kBlock), 0, s, d, e, (T *)p->g, nkb);
        if (p->nrec > 0)
            hipLaunchKernelGGL((k_mesh_walls<T, 3>), dim3(p->nrec), dim3(kBlock), 0, s, d, e, (const T *)p->g, p->din);
        hipLaunchKernelGGL((k_mesh_residual<T, 3>), grid, dim3(kBlock), 0, s, d, e, (const T *)p->g, p->din, TLdev,
                           R, nkb);
    } else {
        if (buf)
            hipLaunchKernelGGL((k_mesh_grad<T, 2, true>), grid, dim3(kBlock), 0, s, d, e, (T *)p->g, nkb);
        else
            hipLaunchKernelGGL((k_mesh_grad<T, 2, false>), grid, dim3(kBlock), 0, s, d, e, (T *)p->g, nkb);
        if (p->nrec > 0)
            hipLaunchKernelGGL((k_mesh_walls<T, 2>), dim3(p->nrec), dim3(kBlock), 0, s, d, e, (const T *)p->g, p->din);
        hipLaunchKernelGGL((k_mesh_residual<T, 2>), grid, dim3(kBlock), 0, s, d, e, (const T *)p->g, p->din, TLdev,
                           R, nkb);
    }
}

template <typename T>
bte_status mesh_solve(bte_mesh_problem *p, T *e, int init, bte_solve_stats *stats, hipStream_t s)
{
    const auto h0 = std::chrono::steady_clock::now();
    const MeshDev &d = p->dev;
    if (init) MHIP(p, hipMemsetAsync(e, 0, p->esize() * p->nelem(), s));
    hipLaunchKernelGGL(k_mesh_moments<T>, mom_grid(p->nc), dim3(kBlock), 0, s, d, e, p->Tprev, p->TLdev, nullptr);
    const int max_iter = p->ctl.max_iter > 0 ? p->ctl.max_iter : 10000;
    for (hipEvent_t &x : p->ev)
        if (!x) MHIP(p, hipEventCreate(&x));
    bte_solve_stats st{};
    bool conv = false;
    double eps = 0;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        MHIP(p, hipEventRecord(p->ev[0], s));
        mesh_iteration_rhs<T>(p, e, p->TLdev, (T *)p->b, s);
        MHIP(p, hipEventRecord(p->ev[1], s));
        for (int L = 0; L < p->nlev; ++L) {
            const int i0 = p->lev_off[L], n = p->lev_off[L + 1] - i0;
            const int blocks = (int)(((size_t)n * p->nl + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(k_mesh_sweep_level<T>, dim3(blocks), dim3(kBlock), 0, s, d, e, (T *)p->b, i0, n);
        }
        MHIP(p, hipEventRecord(p->ev[2], s));
        hipLaunchKernelGGL(k_mesh_moments<T>, mom_grid(p->nc), dim3(kBlock), 0, s, d, e, p->Tdev, p->TLdev, nullptr);
        hipLaunchKernelGGL(k_mesh_eps, dim3(kEpsBlocks), dim3(kBlock), 0, s, p->nc, p->Tprev, p->Tdev, p->eps_part);
        hipLaunchKernelGGL(k_mesh_eps_final, dim3(1), dim3(kBlock), 0, s, p->eps_part, p->eps);
        MHIP(p, hipEventRecord(p->ev[3], s));
        double h[2];
        MHIP(p, hipMemcpyAsync(h, p->eps, 16, hipMemcpyDeviceToHost, s));
        MHIP(p, hipStreamSynchronize(s));
        float ms[3];
        for (int i = 0; i < 3; ++i) MHIP(p, hipEventElapsedTime(&ms[i], p->ev[i], p->ev[i + 1]));
        st.ms_walls += ms[0];
        st.ms_sweep += ms[1];
        st.ms_post += ms[2];
        std::swap(p->Tprev, p->Tdev);
        eps = h[1] > 0 ? h[0] / h[1] : h[0];
        if (!std::isfinite(eps)) MFAIL(p, BTE_ERR_NONFINITE, "non-finite temperature at iteration %d", it);
        if (eps <= p->ctl.residual_temp) {
            conv = true;
            break;
        }
    }
    if (it > max_iter) it = max_iter;
    MHIP(p, hipGetLastError());
    st.iters = it;
    st.eps_T = eps;
    st.converged = conv;
    st.sweep_launches = it * p->nlev;
    st.updates = (double)it * (double)p->nelem();
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
    if (stats) *stats = st;
    if (!conv) MFAIL(p, BTE_ERR_NOT_CONVERGED, "not converged after %d iterations (eps_T %.3g)", it, eps);
    return BTE_OK;
}

}  // namespace

extern "C" {

bte_status bte_mesh_setup(const bte_mesh *mesh, const bte_material *mat, const bte_control *ctl,
                          bte_mesh_problem **out)
{
    if (!out) return BTE_ERR_ARG;
    *out = nullptr;
    bte_mesh_problem *p = new (std::nothrow) bte_mesh_problem();
    if (!p) return BTE_ERR_ARG;
    *out = p;
    if (!mesh || !mat || !ctl) MFAIL(p, BTE_ERR_ARG, "null argument");
    p->ctl = *ctl;
    if (ctl->precision != BTE_F32 && ctl->precision != BTE_F64) MFAIL(p, BTE_ERR_ARG, "bad precision");
    if (ctl->scheme != BTE_SEQUENTIAL) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes run the sequential scheme");
    if (ctl->limiter != BTE_LIM_NONE) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes take the unlimited gradient");
    if (mat->material_dim == 2) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes take bulk materials");
    if (mat->n_bands < 1 || mat->n_bands > kBlock || !mat->C || !mat->v || !mat->tau)
        MFAIL(p, BTE_ERR_ARG, "n_bands must be 1 .. %d with C, v, tau given", kBlock);
    return mesh_build(p, mesh, mat);
}

bte_status bte_mesh_setup_tet(const bte_tet_mesh *mesh, const bte_material *mat, const bte_control *ctl,
                              bte_mesh_problem **out)
{
    if (!out) return BTE_ERR_ARG;
    *out = nullptr;
    bte_mesh_problem *p = new (std::nothrow) bte_mesh_problem();
    if (!p) return BTE_ERR_ARG;
    *out = p;
    if (!mesh || !mat || !ctl) MFAIL(p, BTE_ERR_ARG, "null argument");
    p->ctl = *ctl;
    if (ctl->precision != BTE_F32 && ctl->precision != BTE_F64) MFAIL(p, BTE_ERR_ARG, "bad precision");
    if (ctl->scheme != BTE_SEQUENTIAL) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes run the sequential scheme");
    if (ctl->limiter != BTE_LIM_NONE) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes take the unlimited gradient");
    if (mat->material_dim == 2) MFAIL(p, BTE_ERR_UNSUPPORTED, "meshes take bulk materials");
    if (mat->n_bands < 1 || mat->n_bands > kBlock || !mat->C || !mat->v || !mat->tau)
        MFAIL(p, BTE_ERR_ARG, "n_bands must be 1 .. %d with C, v, tau given", kBlock);
    return mesh_build_tet(p, mesh, mat);
}

size_t bte_mesh_workspace_bytes(const bte_mesh_problem *p)
{
    if (!p || p->nc == 0) return 0;
    size_t b = 0;
    auto add = [&](size_t n) { b += al256(n); };
    add(4 * p->fptr.size());
    add(4 * (size_t)p->nf * 3);
    add(8 * p->fgeo.size());
    add(8 * p->xinv.size());
    add(4 * p->lsptr.size());
    add(4 * p->lsnb.size() + 4);
    add(4 * p->vorder.size());
    add(8 * p->lsd.size() + 8);
    add(4 * p->tag_bc.size() + 8);
    add(8 * p->tag_dT.size() + 8);
    add(8 * p->s.size());
    add(8 * p->w.size());
    add(4 * p->mirror.size());
    add(8 * 3 * (size_t)p->nl);
    add(4 * p->rec_cell.size() + 4);
    add(4 * p->rec_face.size() + 4);
    add(8 * p->rec_den.size() + 8);
    add(4 * p->item_c.size());
    add(4 * p->item_al.size());
    add(8 * p->item_out.size());
    add(sizeof(int4) * p->item_up.size());
    add(sizeof(double4) * p->item_coef.size());
    add((size_t)p->dim * p->esize() * p->nelem());   // gradients
    add(p->esize() * p->nelem());       // residual / increments
    add(8 * ((size_t)p->nrec * p->nl + 1));
    add(8 * 5 * (size_t)p->nc + 16);    // Tdev, Tprev, TLdev, P, eps
    add(8 * 2 * (size_t)kEpsBlocks);    // per-block maxima of the eps test
    return b;
}

bte_status bte_mesh_bind(bte_mesh_problem *p, void *ws_dev, size_t bytes)
{
    if (!p) return BTE_ERR_ARG;
    if (p->nc == 0) MFAIL(p, BTE_ERR_STATE, "setup failed");
    if (!ws_dev || ((uintptr_t)ws_dev & 255)) MFAIL(p, BTE_ERR_ARG, "workspace must be non-null and 256-byte aligned");
    if (bytes < bte_mesh_workspace_bytes(p)) MFAIL(p, BTE_ERR_ARG, "workspace too small");
    char *q = static_cast<char *>(ws_dev);
    auto take = [&](size_t n) {
        char *r = q;
        q += al256(n);
        return r;
    };
    auto up = [&](const void *src, size_t n, char *dst) -> hipError_t {
        return n ? hipMemcpy(dst, src, n, hipMemcpyHostToDevice) : hipSuccess;
    };
    MeshDev &d = p->dev;
    d.nc = p->nc;
    d.na = p->na;
    d.nl = p->nl;
    d.nk = p->nk;
    char *x;
    x = take(4 * p->fptr.size()); MHIP(p, up(p->fptr.data(), 4 * p->fptr.size(), x)); d.fptr = (const int *)x;
    x = take(4 * (size_t)p->nf * 3);
    MHIP(p, up(p->fnb.data(), 4 * (size_t)p->nf, x));
    MHIP(p, up(p->ftag.data(), 4 * (size_t)p->nf, x + 4 * (size_t)p->nf));
    MHIP(p, up(p->frec.data(), 4 * (size_t)p->nf, x + 8 * (size_t)p->nf));
    d.fnb = (const int *)x;
    d.ftag = (const int *)(x + 4 * (size_t)p->nf);
    d.frec = (const int *)(x + 8 * (size_t)p->nf);
    x = take(8 * p->fgeo.size()); MHIP(p, up(p->fgeo.data(), 8 * p->fgeo.size(), x)); d.fgeo = (const double *)x;
    x = take(8 * p->xinv.size()); MHIP(p, up(p->xinv.data(), 8 * p->xinv.size(), x)); d.xinv = (const double *)x;
    x = take(4 * p->lsptr.size()); MHIP(p, up(p->lsptr.data(), 4 * p->lsptr.size(), x)); d.lsptr = (const int *)x;
    x = take(4 * p->lsnb.size() + 4); MHIP(p, up(p->lsnb.data(), 4 * p->lsnb.size(), x)); d.lsnb = (const int *)x;
    x = take(4 * p->vorder.size()); MHIP(p, up(p->vorder.data(), 4 * p->vorder.size(), x)); d.vorder = (const int *)x;
    x = take(8 * p->lsd.size() + 8); MHIP(p, up(p->lsd.data(), 8 * p->lsd.size(), x)); d.lsd = (const double *)x;
    x = take(4 * p->tag_bc.size() + 8); MHIP(p, up(p->tag_bc.data(), 4 * p->tag_bc.size(), x)); d.tag_bc = (const int *)x;
    x = take(8 * p->tag_dT.size() + 8); MHIP(p, up(p->tag_dT.data(), 8 * p->tag_dT.size(), x)); d.tag_dT = (const double *)x;
    x = take(8 * p->s.size()); MHIP(p, up(p->s.data(), 8 * p->s.size(), x)); d.s = (const double *)x;
    x = take(8 * p->w.size()); MHIP(p, up(p->w.data(), 8 * p->w.size(), x)); d.w = (const double *)x;
    x = take(4 * p->mirror.size()); MHIP(p, up(p->mirror.data(), 4 * p->mirror.size(), x)); d.mirror = (const int *)x;
    x = take(8 * 3 * (size_t)p->nl);
    MHIP(p, up(p->C4.data(), 8 * (size_t)p->nl, x));
    MHIP(p, up(p->v.data(), 8 * (size_t)p->nl, x + 8 * (size_t)p->nl));
    MHIP(p, up(p->itau.data(), 8 * (size_t)p->nl, x + 16 * (size_t)p->nl));
    d.C4 = (const double *)x;
    d.v = (const double *)(x + 8 * (size_t)p->nl);
    d.itau = (const double *)(x + 16 * (size_t)p->nl);
    const size_t nr = p->rec_cell.size();
    x = take(4 * nr + 4); MHIP(p, up(p->rec_cell.data(), 4 * nr, x)); d.rec_cell = (const int *)x;
    x = take(4 * nr + 4); MHIP(p, up(p->rec_face.data(), 4 * nr, x)); d.rec_face = (const int *)x;
    x = take(8 * nr + 8); MHIP(p, up(p->rec_den.data(), 8 * nr, x)); d.rec_den = (const double *)x;
    {
        const size_t ni = p->item_c.size();
        x = take(4 * ni); MHIP(p, up(p->item_c.data(), 4 * ni, x)); d.item_c = (const int *)x;
        x = take(4 * ni); MHIP(p, up(p->item_al.data(), 4 * ni, x)); d.item_al = (const int *)x;
        x = take(8 * ni); MHIP(p, up(p->item_out.data(), 8 * ni, x)); d.item_out = (const double *)x;
        x = take(sizeof(int4) * ni); MHIP(p, up(p->item_up.data(), sizeof(int4) * ni, x)); d.item_up = (const int4 *)x;
        x = take(sizeof(double4) * ni);
        MHIP(p, up(p->item_coef.data(), sizeof(double4) * ni, x));
        d.item_coef = (const double4 *)x;
    }
    d.Ctot = p->Ctot;
    d.Ssum = p->Ssum;
    p->g = take((size_t)p->dim * p->esize() * p->nelem());
    p->b = take(p->esize() * p->nelem());
    p->din = (double *)take(8 * ((size_t)p->nrec * p->nl + 1));
    x = take(8 * 5 * (size_t)p->nc + 16);
    p->Tdev = (double *)x;
    p->Tprev = p->Tdev + p->nc;
    p->TLdev = p->Tprev + p->nc;
    p->P = p->TLdev + p->nc;
    p->eps = p->P + p->nc;
    p->eps_part = (double *)take(8 * 2 * (size_t)kEpsBlocks);
    d.P = p->hasP ? p->P : nullptr;
    p->ws = static_cast<char *>(ws_dev);
    p->ws_bytes = bytes;
    return BTE_OK;
}

int bte_mesh_num_cells(const bte_mesh_problem *p) { return p ? p->nc : 0; }
int bte_mesh_num_directions(const bte_mesh_problem *p) { return p ? p->na : 0; }
int bte_mesh_num_levels(const bte_mesh_problem *p) { return p ? p->nlev : 0; }
int bte_mesh_num_lagged(const bte_mesh_problem *p) { return p ? p->nlag : 0; }

bte_status bte_mesh_set_source(bte_mesh_problem *p, const double *P_dev, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) MFAIL(p, BTE_ERR_STATE, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    if (P_dev) {
        MHIP(p, hipMemcpyAsync(p->P, P_dev, 8 * (size_t)p->nc, hipMemcpyDeviceToDevice, s));
        p->hasP = true;
        p->dev.P = p->P;
    } else {
        p->hasP = false;
        p->dev.P = nullptr;
    }
    return BTE_OK;
}

bte_status bte_mesh_moments(bte_mesh_problem *p, const void *e_dev, double *T_dev, double *TL_dev, double *q_dev,
                            void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) MFAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) MFAIL(p, BTE_ERR_ARG, "null e");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64)
        hipLaunchKernelGGL(k_mesh_moments<double>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const double *)e_dev,
                           p->Tdev, p->TLdev, q_dev);
    else
        hipLaunchKernelGGL(k_mesh_moments<float>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const float *)e_dev,
                           p->Tdev, p->TLdev, q_dev);
    const dim3 gr((p->nc + kBlock - 1) / kBlock);
    if (T_dev) hipLaunchKernelGGL(k_mesh_abs, gr, dim3(kBlock), 0, s, p->nc, p->Tref, p->Tdev, T_dev);
    if (TL_dev) hipLaunchKernelGGL(k_mesh_abs, gr, dim3(kBlock), 0, s, p->nc, p->Tref, p->TLdev, TL_dev);
    MHIP(p, hipGetLastError());
    return BTE_OK;
}

bte_status bte_mesh_residual(bte_mesh_problem *p, const void *e_dev, const double *TLdev_dev, void *R_dev,
                             void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) MFAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev || !R_dev) MFAIL(p, BTE_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const double *tl = TLdev_dev;
    if (!tl) {
        if (p->ctl.precision == BTE_F64)
            hipLaunchKernelGGL(k_mesh_moments<double>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const double *)e_dev,
                               nullptr, p->TLdev, nullptr);
        else
            hipLaunchKernelGGL(k_mesh_moments<float>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const float *)e_dev,
                               nullptr, p->TLdev, nullptr);
        tl = p->TLdev;
    }
    if (p->ctl.precision == BTE_F64)
        mesh_iteration_rhs<double>(p, (const double *)e_dev, tl, (double *)R_dev, s);
    else
        mesh_iteration_rhs<float>(p, (const float *)e_dev, tl, (float *)R_dev, s);
    MHIP(p, hipGetLastError());
    return BTE_OK;
}

bte_status bte_mesh_steady_solve(bte_mesh_problem *p, void *e_dev, int init, bte_solve_stats *stats, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) MFAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) MFAIL(p, BTE_ERR_ARG, "null e");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64) return mesh_solve<double>(p, (double *)e_dev, init, stats, s);
    return mesh_solve<float>(p, (float *)e_dev, init, stats, s);
}

bte_status bte_mesh_transient_step(bte_mesh_problem *p, void *e_dev, int n_steps, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) MFAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev || n_steps < 0) MFAIL(p, BTE_ERR_ARG, "null e or negative n_steps");
    const double dt = p->ctl.dt;
    if (!(dt > 0)) MFAIL(p, BTE_ERR_ARG, "control.dt must be > 0");
    if (dt * p->itau_max >= 1.0 || 0.5 * dt * p->vmax * p->sv_max >= 1.0)
        MFAIL(p, BTE_ERR_CFL, "dt violates dt/tau_min < 1 or dt v_max max_i sum_f S/V / 2 < 1");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = p->nelem();
    const int blocks = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    for (int it = 0; it < n_steps; ++it) {
        if (p->ctl.precision == BTE_F64) {
            hipLaunchKernelGGL(k_mesh_moments<double>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const double *)e_dev,
                               nullptr, p->TLdev, nullptr);
            mesh_iteration_rhs<double>(p, (const double *)e_dev, p->TLdev, (double *)p->b, s);
            hipLaunchKernelGGL(k_mesh_axpy<double>, dim3(blocks), dim3(kBlock), 0, s, n, (double *)e_dev,
                               (const double *)p->b, dt);
        } else {
            hipLaunchKernelGGL(k_mesh_moments<float>, mom_grid(p->nc), dim3(kBlock), 0, s, p->dev, (const float *)e_dev,
                               nullptr, p->TLdev, nullptr);
            mesh_iteration_rhs<float>(p, (const float *)e_dev, p->TLdev, (float *)p->b, s);
            hipLaunchKernelGGL(k_mesh_axpy<float>, dim3(blocks), dim3(kBlock), 0, s, n, (float *)e_dev,
                               (const float *)p->b, dt);
        }
    }
    MHIP(p, hipGetLastError());
    return BTE_OK;
}

const char *bte_mesh_last_error(const bte_mesh_problem *p) { return p ? p->err.c_str() : "null handle"; }

void bte_mesh_destroy(bte_mesh_problem *p) { delete p; }

}  // extern "C"
