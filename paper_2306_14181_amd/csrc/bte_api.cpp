// bte_api.cpp -- host runtime and C ABI of the phonon-BTE library.
//
// Setup precomputes everything that does not change during a solve
// (Algorithm 1 precomputes its matrices once, Sec. 3.5): the angular
// quadrature, mirror-direction table, per-cell neighbour codes, diffuse-wall
// records and the tile-wavefront schedule of the sweep.  All device memory
// is a caller-provided workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"

namespace bte {
template <typename T> void launch_moments(const Dev &, const T *, const double *, double *, hipStream_t);
template <typename T>
void launch_walls(const Dev &, const T *, const double *, const int *, const double *, double *, int, hipStream_t);
template <typename T>
void launch_residual(const Dev &, const T *, T *, const double *, const double *, int, hipStream_t);
template <typename T>
hipError_t launch_sweep_tile(const Dev &, const T *, T *, const double *, const double *, const double *,
                             const SweepItem *, int, int, int3, int, int, int, double *, hipStream_t);
template <typename T>
hipError_t launch_transient_tile(const Dev &, const T *, T *, const double *, const double *, const TileItem *, int,
                                 int3, int, int, int, double, double, double *, hipStream_t);
hipError_t tile_kernels_init(size_t);
template <typename T>
hipError_t launch_sweep_adj(const Dev &, const T *, T *, const double *, const double *, const SweepItem *, int, int,
                            int3, int, int, int, double *, hipStream_t);
template <typename T>
void launch_walls_adj(const Dev &, const T *, const int *, const double *, double *, int, hipStream_t);
template <typename T>
hipError_t launch_adj_res(const Dev &, const T *, const double *, const double *, const TileItem *, int, int3, int, int,
                          int, double *, hipStream_t);
void launch_adj_post(const Dev &, const double *, int, double *, double *, hipStream_t);
void launch_adj_phi(const Dev &, const double *, int, double *, hipStream_t);
template <typename T>
void launch_adj_grad(const Dev &, const T *, const T *, const double *, const double *, const double *, double *,
                     hipStream_t);
hipError_t adj_kernels_init(size_t);
template <typename T>
hipError_t launch_sweep2d(const Dev &, const T *, T *, const double *, const double *, const double *,
                          const Sweep2Item *, int, int, int, int, int, double *, unsigned *, hipStream_t);
hipError_t launch_queue_reset(unsigned *, int, hipStream_t);
template <typename T>
hipError_t launch_transient3d(const Dev &, const T *, T *, const double *, const double *, const ColItem *, int, int,
                              int, double, double, double *, hipStream_t);
template <typename T>
hipError_t launch_adj_step(const Dev &, const T *, T *, const T *, const double *, const double *, const double *,
                           const TileItem *, int, int3, int, int, int, double, double *, hipStream_t);
template <typename T>
hipError_t launch_adj_step3d(const Dev &, const T *, T *, const T *, const double *, const double *, const double *,
                             const ColItem *, int, int, int, double, double *, hipStream_t);
template <typename T>
hipError_t launch_adj_res3d(const Dev &, const T *, const double *, const double *, const ColItem *, int, int, int,
                            double *, hipStream_t);
void launch_adj_step_post(const Dev &, const double *, int, const double *, const double *, double *, double *,
                          double, hipStream_t);
template <typename T> void launch_adj_tave_init(const Dev &, const double *, double, T *, hipStream_t);
template <typename T> void launch_adj_phi_cell(const Dev &, const T *, double *, hipStream_t);
void launch_tave(const Dev &, const double *, const double *, double *, hipStream_t);
size_t tile_smem_size(int, int, int);
template <typename T> void launch_set_equilibrium(const Dev &, T *, const double *, hipStream_t);
template <typename T> void launch_apply_shift(const Dev &, const T *, T *, const double *, const double *, hipStream_t);
void launch_keff(const Dev &, const double *, double *, hipStream_t);
void launch_cell_setup(const Dev &, double *, double *, double *, const double[3], const double[3], hipStream_t);
void launch_finalize(const Dev &, const double *, int, double, double *, double *, double *, double *, double *,
                     double *, hipStream_t);
void launch_finalize_tl(const Dev &, const double *, int, double *, hipStream_t);
void launch_steady_post(const Dev &, const double *, int, const double *, double *, double *, double *, double *, int,
                        hipStream_t);
int film_segments(int max_cells);
void launch_film_eps(const Dev &, const double *, const double *, const double *, const double *, double *, double *,
                     int, hipStream_t);
void launch_film_mean(const Dev &, const double *, double *, double *, int, hipStream_t);
void launch_sub_film_mean(const Dev &, double *, const double *, hipStream_t);
void launch_tl_update(int, const double *, const double *, double *, double *, const int *, const int *,
                      hipStream_t);
void launch_cg_coef(const Dev &, const CgArgs &, double *, double *, hipStream_t);
void launch_diff_rhs(const Dev &, const CgArgs &, double *, hipStream_t);
void launch_cg_begin(const Dev &, const CgArgs &, const double *, hipStream_t);
void launch_cg_iters(const Dev &, const CgArgs &, int, int, hipStream_t);
// Gauss-Legendre nodes/weights on [-1, 1], ascending (Newton on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = z;
                p0 = 1.0;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) p0 = 1.0, p1 = z;
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}


// Directions on the sphere for two- and three-dimensional geometries
// (Sec. 3.2, eq. directiondis): Gauss-Legendre nodes of theta and phi on the
// first octant, weight w_theta w_phi sin(theta), mirrored to the eight
// octants (bits 1 = s_x < 0, 2 = s_y < 0, 4 = s_z < 0), then theta, then
// phi; weights scaled to sum to omega exactly.
void sphere_directions(int n_theta, int n_phi, double omega, std::vector<double> &s, std::vector<double> &w)
{
    std::vector<double> xt, wt, xp, wp;
    gauss_legendre(n_theta, xt, wt);
    gauss_legendre(n_phi, xp, wp);
    s.clear();
    w.clear();
    for (int o = 0; o < 8; ++o)
        for (int i = 0; i < n_theta; ++i)
            for (int j = 0; j < n_phi; ++j) {
                const double th = (xt[i] + 1.0) * M_PI / 4.0, wth = wt[i] * M_PI / 4.0;
                const double ph = (xp[j] + 1.0) * M_PI / 4.0, wph = wp[j] * M_PI / 4.0, st = std::sin(th);
                s.push_back((o & 1 ? -1.0 : 1.0) * st * std::cos(ph));
                s.push_back((o & 2 ? -1.0 : 1.0) * st * std::sin(ph));
                s.push_back((o & 4 ? -1.0 : 1.0) * std::cos(th));
                w.push_back(wth * wph * st);
            }
    double sw = 0;
    for (double x : w) sw += x;
    for (double &x : w) x *= omega / sw;
}

}  // namespace bte

using namespace bte;

namespace {

// Width (in columns) of the strips in which the three-dimensional column
// walks are ordered.
constexpr int kColStrip = 16;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct bte_problem {
    std::string err;
    int dim = 0, nfilm = 0, nc = 0, na = 0, nl = 0, nk = 0, noct = 0, na_oct = 0;
    bte_control ctl{};
    double Tref = 0, Ctot = 0, vmax = 0, itau_max = 0;
    double omega = 4.0 * M_PI;   // total angle: 2 pi for a two-dimensional material
    std::vector<Film> films;
    std::vector<uint32_t> code;
    std::vector<int> nb, fid, dbase, wrec, mirror;
    std::vector<double> s, w, C4, v, itau;   // band tables, [nmat][nl]
    int nmat = 1, nifc = 0;
    std::vector<double> Ctot_m;    // sum_lambda C per material
    std::vector<int> wpart;        // per wall record: the cell across an interface, -1 for a diffuse wall
    std::vector<double> wbeta;     // per wall record: [2][nl] transmittance into the cell, out of it
    struct IfcEnd {
        int film = -1, face = -1, ifc = -1, is_a = 0;   // the facing geometry and face
    };
    std::vector<IfcEnd> ifc_end;   // [nfilm * 6]
    std::vector<bte_interface> ifcs;
    std::vector<std::vector<double>> ifc_beta;   // per interface: [2][nl] beta_ab, beta_ba
    double wden[6] = {0, 0, 0, 0, 0, 0};
    double M[3] = {0, 0, 0}, H[3] = {0, 0, 0};
    int nw = 0;
    // sweep schedule
    int3 tdim{1, 1, 1};      // sweep tiles
    int3 tdim_tr{1, 1, 1};   // transient tiles
    size_t items_cap = 0, titems_cap = 0;   // work-list room for every candidate tile shape
    int tile_cap_tr = 0;
    int nchunk_oct = 0;
    std::vector<SweepItem> items;
    std::vector<Sweep2Item> items2;   // two-dimensional sweep: self-contained items, same order
    std::vector<int> diag_off;
    std::vector<TileItem> titems;   // transient: (geometry, octant, tile)
    std::vector<ColItem> citems;    // three-dimensional transient: (geometry, octant, chunk, column)
    int tile_cap = 0;               // star slots of a full tile
    int floating_any = 0, thermal_any = 0;
    // workspace
    size_t ws_bytes = 0;
    char *ws = nullptr;
    size_t off_tables = 0;
    struct Buf {
        size_t off, bytes;
    };
    std::vector<std::pair<std::string, Buf>> layout;
    Dev dev{};
    bool fields_set = false;
    // device pointers
    double *S = nullptr, *kdif = nullptr, *kcor = nullptr, *gamma = nullptr, *P = nullptr;
    double *cdif = nullptr, *ccor = nullptr, *ddif = nullptr, *dcor = nullptr;
    double *TL = nullptr, *TLkin = nullptr, *T0 = nullptr, *T1 = nullptr, *q0 = nullptr, *q1 = nullptr;
    double *r = nullptr, *delta = nullptr, *dpend = nullptr, *fmean = nullptr, *feps = nullptr;
    double *fpart = nullptr;   // per-geometry reduction partials, 5 x nfilm x fseg
    int fseg = 1;              // segments of the largest geometry
    double *cg_x = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_Ap = nullptr;
    double *cg_w0 = nullptr, *cg_w1 = nullptr, *cg_s1 = nullptr;
    double *cg_part = nullptr, *cg_scal = nullptr;
    double *din = nullptr, *part = nullptr;
    void *e2 = nullptr;
    void *psi = nullptr, *psi2 = nullptr;                       // adjoint iterates (ctl.adjoint)
    double *adjX = nullptr, *adjT = nullptr, *adjTL = nullptr;   // adjoint closure term, forward T and T_L
    double *adju = nullptr, *adjr2 = nullptr;
    SweepItem *d_items = nullptr;
    Sweep2Item *d_items2 = nullptr;
    unsigned *d_queue = nullptr;   // one-launch 2D sweep: ticket, abort word, item flags
    TileItem *d_titems = nullptr;
    ColItem *d_citems = nullptr;
    int *d_wrec = nullptr;
    double *d_wden = nullptr;
    int npart_max = 0;
    // optional device timers of the transient step (bte_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> tev;
    bte_solve_stats last{};

    // HIP graphs of the steady iteration (bte_set_graphs), captured on a
    // private stream (the caller's may be the null stream, which cannot be
    // captured) and replayed on the caller's stream
    bool graphs = true;
    bool persistent = false;   // 2D register-tile sweeps in one launch (bte_set_persistent)
    bool queue_ok = false;     // every item's upwind items precede it (build_schedule)
    hipStream_t cstream = nullptr;
    ~bte_problem()
    {
        for (hipEvent_t e : tev) (void)hipEventDestroy(e);
        if (cstream) (void)hipStreamDestroy(cstream);
    }
    size_t esize() const { return ctl.precision == BTE_F64 ? 8 : 4; }
    size_t nelem() const { return (size_t)nc * nk; }
};

#define FAIL(p, st, ...)                                                                                               \
    do {                                                                                                               \
        char _b[512];                                                                                                  \
        snprintf(_b, sizeof _b, __VA_ARGS__);                                                                          \
        (p)->err = _b;                                                                                                 \
        return st;                                                                                                     \
    } while (0)

#define HIPCHK(p, x)                                                                                                   \
    do {                                                                                                               \
        hipError_t _e = (x);                                                                                           \
        if (_e != hipSuccess) FAIL(p, BTE_ERR_HIP, "%s: %s", #x, hipGetErrorString(_e));                               \
    } while (0)

namespace {

bte_status build_geometry(bte_problem *p, const bte_geometry *geo, int n_geo)
{
    p->dim = geo[0].dim;
    p->nfilm = n_geo;
    int cell0 = 0;
    for (int f = 0; f < n_geo; ++f) {
        const bte_geometry &g = geo[f];
        if (g.dim != p->dim) FAIL(p, BTE_ERR_ARG, "geometry %d: all geometries must share dim", f);
        Film fm{};
        long long ncell = 1;
        for (int a = 0; a < 3; ++a) {
            fm.n[a] = a < g.dim ? g.n[a] : 1;
            if (fm.n[a] < 1) FAIL(p, BTE_ERR_ARG, "geometry %d: n[%d] < 1", f, a);
            fm.len[a] = a < g.dim ? g.len[a] : 1.0;
            if (!(fm.len[a] > 0)) FAIL(p, BTE_ERR_ARG, "geometry %d: len[%d] must be > 0", f, a);
            fm.h[a] = fm.len[a] / fm.n[a];
            fm.ih[a] = 1.0 / fm.h[a];
            fm.pdT[a] = a < g.dim ? g.periodic_dT[a] : 0.0;
            fm.periodic[a] = a < g.dim && g.bc[2 * a] == BTE_BC_PERIODIC;
            ncell *= fm.n[a];
        }
        if (ncell + cell0 > 0x7fffffffLL / 8) FAIL(p, BTE_ERR_ARG, "too many cells");
        for (int a = 0; a < g.dim; ++a) {
            bool p0 = g.bc[2 * a] == BTE_BC_PERIODIC, p1 = g.bc[2 * a + 1] == BTE_BC_PERIODIC;
            if (p0 != p1) FAIL(p, BTE_ERR_ARG, "geometry %d: periodic faces of axis %d must come in pairs", f, a);
            for (int s = 0; s < 2; ++s) {
                if (g.bc[2 * a + s] < 0 || g.bc[2 * a + s] > 4) FAIL(p, BTE_ERR_ARG, "geometry %d: bad bc", f);
                if (g.bc[2 * a + s] == BTE_BC_INTERFACE && p->ifc_end[6 * f + 2 * a + s].film < 0)
                    FAIL(p, BTE_ERR_ARG, "geometry %d: face %d is an interface of no bte_interface", f, 2 * a + s);
            }
            if (!p0 && g.periodic_dT[a] != 0.0)
                FAIL(p, BTE_ERR_ARG, "geometry %d: periodic_dT on a non-periodic axis", f);
        }
        if (g.pore_bc != BTE_BC_DIFFUSE && g.pore_bc != BTE_BC_SPECULAR && g.pore_bc != BTE_BC_THERMAL)
            FAIL(p, BTE_ERR_ARG, "geometry %d: pore_bc must be thermalizing, specular or diffuse", f);
        for (int q = 0; q < 6; ++q) fm.wallT[q] = g.bc_T[q] - p->Tref;
        fm.cell0 = cell0;
        fm.ncell = (int)ncell;
        cell0 += (int)ncell;
        p->films.push_back(fm);
    }
    p->nc = cell0;
    const int nc = p->nc;
    p->code.assign(nc, 0);
    p->nb.assign(6 * (size_t)nc, -1);
    p->fid.assign(nc, 0);
    p->dbase.assign(nc, -1);
    int nw = 0;
    for (int f = 0; f < n_geo; ++f) {
        const bte_geometry &g = geo[f];
        Film &fm = p->films[f];
        auto solid_at = [&](int i) { return g.solid ? g.solid[i] != 0 : true; };
        int nsolid = 0, thermal = 0;
        for (int i = 0; i < fm.ncell; ++i) {
            const int c = fm.cell0 + i;
            p->fid[c] = f;
            if (!solid_at(i)) continue;
            ++nsolid;
            uint32_t code = kSolidBit;
            int idx[3] = {i % fm.n[0], (i / fm.n[0]) % fm.n[1], i / (fm.n[0] * fm.n[1])};
            for (int a = 0; a < p->dim; ++a) {
                for (int side = -1; side <= 1; side += 2) {
                    int k = idx[a] + side;
                    int fidx = face_of(a, side);
                    bool wraps = false, outer = false;
                    int kind = -1;
                    int partner = -1;
                    if (k < 0 || k >= fm.n[a]) {
                        if (g.bc[fidx] == BTE_BC_PERIODIC) {
                            k = (k + fm.n[a]) % fm.n[a];
                            wraps = true;
                        } else if (g.bc[fidx] == BTE_BC_INTERFACE) {
                            // the facing cell of the other geometry (same
                            // indices along the other axes); a pore there is
                            // a pore wall of this geometry
                            const bte_problem::IfcEnd &ie = p->ifc_end[6 * f + fidx];
                            const Film &fo = p->films[ie.film];
                            int jj[3] = {idx[0], idx[1], idx[2]};
                            jj[a] = side > 0 ? 0 : fo.n[a] - 1;
                            const int li = jj[0] + fo.n[0] * (jj[1] + fo.n[1] * jj[2]);
                            const uint8_t *so = geo[ie.film].solid;
                            if (!so || so[li]) {
                                kind = kWallInterface;
                                partner = fo.cell0 + li;
                            } else {
                                kind = g.pore_bc;
                            }
                        } else {
                            kind = g.bc[fidx];
                            outer = true;
                        }
                    }
                    int j = -1;
                    if (kind < 0) {
                        int jj[3] = {idx[0], idx[1], idx[2]};
                        jj[a] = k;
                        int li = jj[0] + fm.n[0] * (jj[1] + fm.n[1] * jj[2]);
                        if (solid_at(li)) j = fm.cell0 + li;
                        else {
                            kind = g.pore_bc;
                            wraps = false;
                        }
                    }
                    uint32_t bits = 0;
                    if (j >= 0) {
                        bits |= side > 0 ? 2u : 1u;
                        if (wraps) bits |= side > 0 ? 8u : 4u;
                        p->nb[(size_t)fidx * nc + c] = j;
                    } else {
                        bits |= (uint32_t)kind << (side > 0 ? 6 : 4);
                        if (outer) code |= 1u << ((side > 0 ? 28 : 25) + a);
                        if (kind == BTE_BC_THERMAL) thermal = 1;
                        if (kind == BTE_BC_DIFFUSE || kind == kWallInterface) {
                            // one inflow record per diffuse or interface face
                            if (p->dbase[c] < 0) p->dbase[c] = nw;
                            p->wrec.push_back(c);
                            p->wrec.push_back(fidx);
                            p->wpart.push_back(partner);
                            // the diffusion operators couple across the interface
                            if (partner >= 0) p->nb[(size_t)fidx * nc + c] = partner;
                            ++nw;
                        }
                    }
                    code |= bits << (8 * a);
                }
            }
            p->code[c] = code;
        }
        if (nsolid == 0) FAIL(p, BTE_ERR_ARG, "geometry %d has no solid cell", f);
        fm.nsolid = nsolid;
        fm.floating = thermal ? 0 : 1;
        p->floating_any |= fm.floating;
        p->thermal_any |= thermal;
    }
    p->nw = nw;
    return BTE_OK;
}

bte_status build_quadrature(bte_problem *p, int n_theta, int n_phi, bool planar)
{
    if (n_theta < 1 || (p->dim > 1 && !planar && n_phi < 1)) FAIL(p, BTE_ERR_ARG, "n_theta/n_phi must be >= 1");
    std::vector<double> xt, wt, xp, wp;
    gauss_legendre(n_theta, xt, wt);
    std::vector<double> th(n_theta), wth(n_theta);
    for (int i = 0; i < n_theta; ++i) {
        th[i] = (xt[i] + 1.0) * M_PI / 4.0;
        wth[i] = wt[i] * M_PI / 4.0;
    }
    p->s.clear();
    p->w.clear();
    if (planar) {
        // two-dimensional material: in-plane directions at angle th from x,
        // quadrant bits 1 = s_x < 0, 2 = s_y < 0; a slab merges the two
        // signs of s_y (weight 2 w_th per hemisphere)
        const int nq = p->dim == 1 ? 2 : 4;
        for (int o = 0; o < nq; ++o)
            for (int i = 0; i < n_theta; ++i) {
                p->s.push_back((o & 1 ? -1.0 : 1.0) * std::cos(th[i]));
                p->s.push_back(p->dim == 1 ? 0.0 : (o & 2 ? -1.0 : 1.0) * std::sin(th[i]));
                p->s.push_back(0.0);
                p->w.push_back(p->dim == 1 ? 2.0 * wth[i] : wth[i]);
            }
        p->noct = nq;
    } else if (p->dim == 1) {
        for (int h = 0; h < 2; ++h)
            for (int i = 0; i < n_theta; ++i) {
                p->s.push_back((h ? -1.0 : 1.0) * std::cos(th[i]));
                p->s.push_back(0.0);
                p->s.push_back(0.0);
                p->w.push_back(2.0 * M_PI * wth[i] * std::sin(th[i]));
            }
        p->noct = 2;
    } else {
        sphere_directions(n_theta, n_phi, p->omega, p->s, p->w);
        p->noct = 8;
    }
    p->na = (int)p->w.size();
    p->na_oct = p->na / p->noct;
    double sw = 0;
    for (double x : p->w) sw += x;
    for (double &x : p->w) x *= p->omega / sw;   // exact total angle: equilibrium is a fixed point
    p->mirror.assign(3 * (size_t)p->na, 0);
    for (int a = 0; a < 3; ++a)
        for (int al = 0; al < p->na; ++al) {
            if (a >= p->dim) {
                p->mirror[a * p->na + al] = al;
                continue;
            }
            int best = -1;
            double bd = 1e300;
            for (int b = 0; b < p->na; ++b) {
                double dd = 0;
                for (int q = 0; q < 3; ++q) {
                    double t = p->s[3 * al + q] * (q == a ? -1.0 : 1.0);
                    dd += std::fabs(p->s[3 * b + q] - t);
                }
                if (dd < bd) bd = dd, best = b;
            }
            p->mirror[a * p->na + al] = best;
        }
    for (int a = 0; a < 3; ++a) {
        double m = 0, h = 0;
        for (int al = 0; al < p->na; ++al) {
            double sa = p->s[3 * al + a];
            m += p->w[al] * sa * sa;
            if (sa > 0) h += p->w[al] * sa;
        }
        p->M[a] = m / p->omega;
        p->H[a] = h;
    }
    for (int f = 0; f < 6; ++f) {
        int a = f / 2, side = (f & 1) ? 1 : -1;
        double den = 0;
        for (int al = 0; al < p->na; ++al) {
            double sn = p->s[3 * al + a] * side;
            if (sn < 0) den += p->w[al] * (-sn);
        }
        p->wden[f] = den > 0 ? den : 1.0;
    }
    return BTE_OK;
}

// star slots of a tile: the tile and, per axis, two upwind and one downwind layer
int tile_cap_of(const bte_problem *p, int3 td)
{
    const int e[3] = {td.x, td.y, td.z};
    const int cells = e[0] * e[1] * e[2];
    int halo = 0;
    for (int a = 0; a < p->dim; ++a) halo += 3 * cells / e[a];
    return cells + halo;
}

// Two-dimensional sweeps with 8 x 8 tiles run the register-tile kernel
// (tdim.z = its tile rows per wavefront; a 2D geometry has one cell along z,
// so the tiling is that of 8 x 8 x 1); any other shape runs the LDS-tile
// kernel.  The LDS-tile kernels (and the 2D adjoint sweep, which has no
// register form) take the shape with z = 1 then.
bool reg2d(const bte_problem *p) { return p->dim == 2 && p->tdim.x == 8 && p->tdim.y == 8; }
int3 lds_tdim(const bte_problem *p) { return reg2d(p) ? make_int3(8, 8, 1) : p->tdim; }

// Tile shapes the LDS-tile kernels may use for one kind (bte_tune_kind), the
// default shape first: at most 64 cells (the kernels keep 64-entry per-cell
// tables), a star within the 160 KiB of LDS of a compute unit and, for the
// sweep, at most 48 cells in the first upwind halo layers of all axes (the
// LDS buffer of upwind increments has 48 rows).
// A 3D sweep segment addresses its rows by 32-bit byte offsets from the
// lowest row of the plane below the segment: (zseg + 2) planes of every
// geometry must span less than 4 GiB, and one plane less than 2 GiB.
bool seg_fits(const bte_problem *p, int zseg)
{
    for (const Film &fm : p->films) {
        const double plane = (double)fm.n[0] * fm.n[1] * p->nk * (double)p->esize();
        if (plane >= 2147483648.0 || (zseg + 2) * plane >= 4294967296.0) return false;
    }
    return true;
}

std::vector<int3> tile_candidates(const bte_problem *p, int kind)
{
    std::vector<int3> c;
    if (kind == BTE_TUNE_SWEEP_ONE_LAUNCH) {
        // the register-tile shapes of a 2D sweep, in one launch per sweep
        if (p->dim == 2) {
            c = {make_int3(8, 8, 2), make_int3(8, 8, 1)};
            if (p->esize() == 4) c.push_back(make_int3(8, 8, 4));
        }
        return c;
    }
    if (kind == BTE_TUNE_SWEEP) {
        if (p->dim == 1) c = {make_int3(64, 1, 1), make_int3(32, 1, 1), make_int3(16, 1, 1)};
        else if (p->dim == 2) c = {make_int3(16, 4, 1), make_int3(4, 16, 1), make_int3(8, 4, 1)};   // LDS tiles
        else {
            // column segments of 1 x 1 x z cells (k_sweep3d, at most 48 cells):
            // shorter segments shorten each hyperplane launch, longer ones
            // need fewer launches; lengths past the tallest geometry are the same
            int nz = 1;
            for (const Film &fm : p->films) nz = std::max(nz, fm.n[2]);
            for (int z : {16, 8, 12, 24, 32, 48, 4, 2, 1}) {
                const int zz = std::min(z, nz);
                bool dup = false;
                for (const int3 &t : c) dup = dup || t.z == zz;
                if (!dup && seg_fits(p, zz) && (zz > 1 || c.empty())) c.push_back(make_int3(1, 1, zz));
            }
            if (c.empty()) c.push_back(make_int3(1, 1, 1));   // too large: refused by the solves
            return c;
        }
    } else {
        if (p->dim == 1)
            c = {make_int3(64, 1, 1), make_int3(32, 1, 1), make_int3(16, 1, 1), make_int3(8, 1, 1),
                 make_int3(4, 1, 1)};
        else if (p->dim == 2)
            c = {make_int3(8, 8, 1), make_int3(16, 4, 1), make_int3(4, 16, 1), make_int3(8, 4, 1),
                 make_int3(16, 2, 1)};
        else c = {make_int3(4, 4, 2)};   // unused by the column walk; the transposed 1D/2D form only
    }
    const bool sweep = kind == BTE_TUNE_SWEEP;
    std::vector<int3> ok;
    // two-dimensional sweeps: the register-tile kernel first (8 x 8 tiles,
    // z = tile rows per wavefront: 2, 1, and 4 in FP32, where it needs no
    // scratch), then the LDS-tile shapes
    if (sweep && p->dim == 2) {
        ok = {make_int3(8, 8, 2), make_int3(8, 8, 1)};
        if (p->esize() == 4) ok.push_back(make_int3(8, 8, 4));
    }
    for (const int3 &t : c) {
        const int e[3] = {t.x, t.y, t.z}, cells = t.x * t.y * t.z;
        int up1 = 0;
        for (int a = 0; a < p->dim; ++a) up1 += cells / e[a];
        if (cells <= 64 && (!sweep || up1 <= 48) &&
            tile_smem_size(tile_cap_of(p, t), (int)p->esize(), sweep) <= 160 * 1024)
            ok.push_back(t);
    }
    return ok;
}

// work items of a tile shape: sweep (per octant and chunk) and transient (per octant)
size_t count_tiles(const bte_problem *p, int3 td)
{
    size_t n = 0;
    for (const Film &fm : p->films)
        n += (size_t)((fm.n[0] + td.x - 1) / td.x) * ((fm.n[1] + td.y - 1) / td.y) * ((fm.n[2] + td.z - 1) / td.z);
    return n;
}

// default shapes (the first candidates) and the work-list room for all candidates
void choose_default_tiles(bte_problem *p)
{
    const int lanes_oct = p->na_oct * p->nl;
    const int nchunk = (lanes_oct + 63) / 64;
    p->tdim = tile_candidates(p, BTE_TUNE_SWEEP)[0];
    // explicit steps in 1D: each block walks its octant's chunks in turn, so
    // a short domain needs short tiles to give the chip enough blocks; take
    // the largest tile that still yields two blocks per compute unit
    const std::vector<int3> tc = tile_candidates(p, BTE_TUNE_TRANSIENT);
    p->tdim_tr = tc[0];
    if (p->dim == 1)
        for (const int3 &t : tc) {
            p->tdim_tr = t;
            if (count_tiles(p, t) * (size_t)p->noct >= 512) break;
        }
    p->items_cap = p->titems_cap = 0;
    for (const int3 &t : tile_candidates(p, BTE_TUNE_SWEEP))
        p->items_cap = std::max(p->items_cap, count_tiles(p, t) * p->noct * nchunk);
    for (const int3 &t : tile_candidates(p, BTE_TUNE_TRANSIENT))
        p->titems_cap = std::max(p->titems_cap, count_tiles(p, t) * p->noct);
}

// Work lists of the current tile shapes (p->tdim, p->tdim_tr)
void build_schedule(bte_problem *p)
{
    const int lanes_oct = p->na_oct * p->nl;
    p->nchunk_oct = (lanes_oct + 63) / 64;
    struct Rec {
        int d;
        SweepItem it;
    };
    std::vector<Rec> recs;
    int maxd = 0;
    for (int f = 0; f < p->nfilm; ++f) {
        const Film &fm = p->films[f];
        const int nt[3] = {(fm.n[0] + p->tdim.x - 1) / p->tdim.x, (fm.n[1] + p->tdim.y - 1) / p->tdim.y,
                           (fm.n[2] + p->tdim.z - 1) / p->tdim.z};
        for (int o = 0; o < p->noct; ++o) {
            int sg[3];
            for (int a = 0; a < 3; ++a) sg[a] = p->s[3 * (o * p->na_oct) + a] > 0 ? 1 : -1;
            for (int tz = 0; tz < nt[2]; ++tz)
                for (int ty = 0; ty < nt[1]; ++ty)
                    for (int tx = 0; tx < nt[0]; ++tx) {
                        const int fx = sg[0] > 0 ? tx : nt[0] - 1 - tx;
                        const int fy = sg[1] > 0 ? ty : nt[1] - 1 - ty;
                        const int fz = sg[2] > 0 ? tz : nt[2] - 1 - tz;
                        const int dg = fx + fy + (p->dim > 2 ? fz : tz);
                        maxd = std::max(maxd, dg);
                        for (int ch = 0; ch < p->nchunk_oct; ++ch)
                            recs.push_back({dg, {f, o, ch, tx + nt[0] * (ty + nt[1] * tz)}});
                    }
        }
    }
    std::stable_sort(recs.begin(), recs.end(), [](const Rec &a, const Rec &b) { return a.d < b.d; });
    p->titems.clear();
    for (int f = 0; f < p->nfilm; ++f) {
        const Film &fm = p->films[f];
        const int ntile = ((fm.n[0] + p->tdim_tr.x - 1) / p->tdim_tr.x) *
                          ((fm.n[1] + p->tdim_tr.y - 1) / p->tdim_tr.y) * ((fm.n[2] + p->tdim_tr.z - 1) / p->tdim_tr.z);
        for (int o = 0; o < p->noct; ++o)
            for (int t = 0; t < ntile; ++t) p->titems.push_back({f, o, t, 0});
    }
    // Columns of one (geometry, octant, chunk) in strips of kColStrip along
    // x, each strip row by row: the y neighbours of a column are then walked
    // kColStrip and 2 kColStrip items earlier or later, close enough that
    // their values are still in the XCD's L2 (row by row over the whole
    // width they were 64 and 128 columns apart, and were fetched again).
    p->citems.clear();
    if (p->dim == 3)
        for (int f = 0; f < p->nfilm; ++f) {
            const Film &fm = p->films[f];
            for (int o = 0; o < p->noct; ++o)
                for (int ch = 0; ch < p->nchunk_oct; ++ch)
                    for (int x0 = 0; x0 < fm.n[0]; x0 += kColStrip)
                        for (int y = 0; y < fm.n[1]; ++y)
                            for (int x = x0; x < std::min(x0 + kColStrip, fm.n[0]); ++x)
                                p->citems.push_back({f, o, ch, x + fm.n[0] * y});
        }
    p->tile_cap = tile_cap_of(p, lds_tdim(p));
    p->tile_cap_tr = tile_cap_of(p, p->tdim_tr);
    p->items.clear();
    p->diag_off.assign(maxd + 2, 0);
    for (auto &r : recs) {
        p->items.push_back(r.it);
        p->diag_off[r.d + 1]++;
    }
    for (int d = 0; d <= maxd; ++d) p->diag_off[d + 1] += p->diag_off[d];
    p->items2.clear();
    if (reg2d(p)) {
        for (const SweepItem &it : p->items) {
            const Film &fm = p->films[it.film];
            Sweep2Item q{};
            q.oct = it.oct;
            q.chunk = it.chunk;
            q.film = it.film;
            const bool pos0 = p->s[3 * (it.oct * p->na_oct) + 0] > 0, pos1 = p->s[3 * (it.oct * p->na_oct) + 1] > 0;
            q.flags = (fm.periodic[0] ? 1 : 0) | (fm.periodic[1] ? 2 : 0) | (pos0 ? 4 : 0) | (pos1 ? 8 : 0);
            const int nt0 = (fm.n[0] + p->tdim.x - 1) / p->tdim.x;
            q.o0 = (it.tile % nt0) * p->tdim.x;
            q.o1 = (it.tile / nt0) * p->tdim.y;
            q.e0 = std::min(p->tdim.x, fm.n[0] - q.o0);
            q.e1 = std::min(p->tdim.y, fm.n[1] - q.o1);
            q.n0 = fm.n[0];
            q.n1 = fm.n[1];
            q.cell0 = fm.cell0;
            q.pdT0 = fm.pdT[0];
            q.pdT1 = fm.pdT[1];
            q.h0 = fm.h[0];
            q.h1 = fm.h[1];
            q.ih0 = fm.ih[0];
            q.ih1 = fm.ih[1];
            for (int f = 0; f < 4; ++f) q.wallT[f] = fm.wallT[f];
            q.upx = q.upy = -1;
            q.moff = fm.moff;
            q.Ctot = fm.Ctot;
            p->items2.push_back(q);
        }
        // Items of the x- and y-upwind tiles (same geometry, octant and
        // chunk; none across the domain edge, where the coupling is a wall or
        // a lagged periodic face) for the one-launch sweep, which waits for
        // them.  They lie on earlier tile diagonals, hence earlier in the
        // order; the queue form is refused if that ever fails.
        std::vector<size_t> foff(p->nfilm + 1, 0);
        for (int f = 0; f < p->nfilm; ++f) {
            const Film &fm = p->films[f];
            const size_t nt = (size_t)((fm.n[0] + 7) / 8) * ((fm.n[1] + 7) / 8);
            foff[f + 1] = foff[f] + nt * p->noct * p->nchunk_oct;
        }
        std::vector<int> at(foff[p->nfilm], -1);
        auto key = [&](int f, int o, int ch, int tile) {
            const Film &fm = p->films[f];
            const size_t nt = (size_t)((fm.n[0] + 7) / 8) * ((fm.n[1] + 7) / 8);
            return foff[f] + ((size_t)o * p->nchunk_oct + ch) * nt + tile;
        };
        for (size_t i = 0; i < p->items.size(); ++i) {
            const SweepItem &it = p->items[i];
            at[key(it.film, it.oct, it.chunk, it.tile)] = (int)i;
        }
        p->queue_ok = true;
        for (size_t i = 0; i < p->items.size(); ++i) {
            const SweepItem &it = p->items[i];
            Sweep2Item &q = p->items2[i];
            const Film &fm = p->films[it.film];
            const int nt0 = (fm.n[0] + 7) / 8, nt1 = (fm.n[1] + 7) / 8;
            const int tx = it.tile % nt0, ty = it.tile / nt0;
            const int ux = tx - ((q.flags & 4) ? 1 : -1), uy = ty - ((q.flags & 8) ? 1 : -1);
            if (ux >= 0 && ux < nt0) q.upx = at[key(it.film, it.oct, it.chunk, ux + nt0 * ty)];
            if (uy >= 0 && uy < nt1) q.upy = at[key(it.film, it.oct, it.chunk, tx + nt0 * uy)];
            if (q.upx >= (int)i || q.upy >= (int)i) p->queue_ok = false;
        }
    }
}

// Per geometry: the wall emission conductance of the correction operator
// (2 sum C v H_a / Omega of its material) and the interface conductance of
// each interface face (sum_lambda beta C v H_a / Omega, the mean of the two
// directions); per wall record the transmittances into and out of its cell
// (zero for a diffuse wall).
void finish_materials(bte_problem *p)
{
    std::vector<double> cv(p->nmat, 0.0);
    for (int m = 0; m < p->nmat; ++m)
        for (int l = 0; l < p->nl; ++l) {
            const size_t i = (size_t)m * p->nl + l;
            cv[m] += p->C4[i] * p->omega * p->v[i];
        }
    for (int f = 0; f < p->nfilm; ++f) {
        Film &fm = p->films[f];
        for (int a = 0; a < 3; ++a) fm.Hm[a] = 2.0 * cv[fm.mat] * p->H[a] / p->omega;
        for (int q = 0; q < 6; ++q) {
            fm.gif[q] = 0.0;
            const bte_problem::IfcEnd &ie = p->ifc_end[6 * f + q];
            if (ie.film < 0) continue;
            const Film &fo = p->films[ie.film];
            const std::vector<double> &bt = p->ifc_beta[ie.ifc];
            double g = 0.0;
            for (int l = 0; l < p->nl; ++l) {
                const double b_out = ie.is_a ? bt[l] : bt[p->nl + l], b_in = ie.is_a ? bt[p->nl + l] : bt[l];
                const size_t i = (size_t)fm.moff + l, o = (size_t)fo.moff + l;
                g += b_out * p->C4[i] * p->omega * p->v[i] + b_in * p->C4[o] * p->omega * p->v[o];
            }
            fm.gif[q] = 0.5 * g * p->H[q >> 1] / p->omega;
        }
    }
    p->wbeta.assign(2 * (size_t)p->nl * std::max(p->nw, 1), 0.0);
    for (int r = 0; r < p->nw; ++r) {
        if (p->wpart[r] < 0) continue;
        const int c = p->wrec[2 * r], fidx = p->wrec[2 * r + 1];
        const bte_problem::IfcEnd &ie = p->ifc_end[6 * p->fid[c] + fidx];
        const std::vector<double> &bt = p->ifc_beta[ie.ifc];
        for (int l = 0; l < p->nl; ++l) {
            p->wbeta[2 * (size_t)r * p->nl + l] = ie.is_a ? bt[p->nl + l] : bt[l];          // into the cell
            p->wbeta[(2 * (size_t)r + 1) * p->nl + l] = ie.is_a ? bt[l] : bt[p->nl + l];    // out of it
        }
    }
    if (p->wpart.empty()) p->wpart.assign(1, -1);
}

void plan_workspace(bte_problem *p)
{
    p->layout.clear();
    size_t off = 0;
    auto add = [&](const char *name, size_t bytes) {
        p->layout.push_back({name, {off, bytes}});
        off = align256(off + std::max<size_t>(bytes, 8));
    };
    const size_t nc = p->nc;
    add("s", 8 * p->s.size());
    add("w", 8 * p->w.size());
    add("mirror", 4 * p->mirror.size());
    add("C4", 8 * p->C4.size());
    add("v", 8 * p->v.size());
    add("itau", 8 * p->itau.size());
    add("wpart", 4 * p->wpart.size());
    add("wbeta", 8 * p->wbeta.size());
    add("film", sizeof(Film) * p->nfilm);
    add("code", 4 * nc);
    add("nb", 4 * 6 * nc);
    add("fid", 4 * nc);
    add("dbase", 4 * nc);
    add("wrec", 4 * p->wrec.size());
    add("wden", 8 * 6);
    add("items", sizeof(SweepItem) * p->items_cap);
    add("items2", sizeof(Sweep2Item) * (p->dim == 2 ? p->items_cap : 0));
    add("queue", 4 * (p->dim == 2 ? p->items_cap + 2 : 0));
    add("titems", sizeof(TileItem) * p->titems_cap);
    add("citems", sizeof(ColItem) * p->citems.size());
    for (const char *n : {"gamma", "P", "S", "TL", "TLkin", "T0", "T1", "q0", "q1", "r", "delta", "dpend", "cg_x",
                          "cg_r", "cg_z", "cg_p", "cg_Ap", "cg_w0", "cg_w1", "cg_s1"})
        add(n, 8 * nc);
    add("kdif", 8 * 3 * nc);
    add("kcor", 8 * 3 * nc);
    add("cdif", 8 * 6 * nc);
    add("ccor", 8 * 6 * nc);
    add("ddif", 8 * nc);
    add("dcor", 8 * nc);
    add("fmean", 8 * p->nfilm);
    add("feps", 8 * 5 * p->nfilm);
    {
        int mx = 1;
        for (const Film &fm : p->films) mx = std::max(mx, fm.ncell);
        p->fseg = film_segments(mx);
    }
    add("fpart", 8 * 5 * (size_t)p->nfilm * p->fseg);
    add("fdone", 4 * (size_t)p->nfilm);
    add("cg_part", 8 * 6 * (size_t)((nc + kBlock - 1) / kBlock));
    add("cg_scal", 8 * 16);
    add("din", 8 * (size_t)p->nw * p->nl);
    const int nchunk_stream = (p->nk + kBlock - 1) / kBlock;
    p->npart_max = std::max(nchunk_stream, p->noct * p->nchunk_oct);
    add("part", 8 * (size_t)kMomN * nc * p->npart_max);
    add("e2", p->esize() * p->nelem());
    add("zrow", 8 * 8 * (size_t)p->nk);   // 8 cells of zeros (a missing row of a tile)
    for (const char *n : {"adjX", "adjT", "adjTL", "adju", "adjr2"}) add(n, 8 * nc);
    if (p->ctl.adjoint) {
        add("psi", p->esize() * p->nelem());
        add("psi2", p->esize() * p->nelem());
    }
    p->ws_bytes = off;
}

template <typename X> X *wsptr(bte_problem *p, const char *name)
{
    for (auto &l : p->layout)
        if (l.first == name) return reinterpret_cast<X *>(p->ws + l.second.off);
    return nullptr;
}

}  // namespace

namespace {
void cell_setup(bte_problem *p, hipStream_t s);
}

extern "C" {

bte_status bte_setup(const bte_geometry *geo, int n_geo, const bte_material *mat, const bte_control *ctl,
                     bte_problem **out)
{
    return bte_setup_multi(geo, n_geo, mat, 1, nullptr, nullptr, 0, ctl, out);
}

bte_status bte_setup_multi(const bte_geometry *geo, int n_geo, const bte_material *mats, int n_mat,
                           const int *geo_mat, const bte_interface *ifc, int n_ifc, const bte_control *ctl,
                           bte_problem **out)
{
    if (!out) return BTE_ERR_ARG;
    *out = nullptr;
    bte_problem *p = new (std::nothrow) bte_problem();
    if (!p) return BTE_ERR_ARG;
    bte_status st = BTE_OK;
    auto bail = [&](bte_status s) {
        // keep the handle so the caller can read the message
        *out = p;
        return s;
    };
    if (!geo || n_geo < 1 || !mats || n_mat < 1 || !ctl || n_ifc < 0 || (n_ifc > 0 && !ifc)) {
        p->err = "null argument, n_geo < 1, n_mat < 1 or n_ifc < 0";
        return bail(BTE_ERR_ARG);
    }
    const bte_material *mat = &mats[0];
    if (geo[0].dim < 1 || geo[0].dim > 3) {
        p->err = "dim must be 1, 2 or 3";
        return bail(BTE_ERR_ARG);
    }
    for (int m = 0; m < n_mat; ++m) {
        const bte_material &mm = mats[m];
        if (mm.n_bands < 1 || mm.n_bands > 256 || !mm.C || !mm.v || !mm.tau) {
            p->err = "n_bands must be in [1, 256] with C, v, tau given";
            return bail(BTE_ERR_ARG);
        }
        if (mm.n_bands != mat->n_bands || mm.n_theta != mat->n_theta || mm.n_phi != mat->n_phi ||
            mm.T_ref != mat->T_ref || mm.material_dim != mat->material_dim) {
            p->err = "materials must share n_bands, n_theta, n_phi, T_ref and material_dim";
            return bail(BTE_ERR_ARG);
        }
    }
    for (int f = 0; f < n_geo; ++f)
        if (geo_mat && (geo_mat[f] < 0 || geo_mat[f] >= n_mat)) {
            p->err = "geo_mat out of range";
            return bail(BTE_ERR_ARG);
        }
    p->ctl = *ctl;
    if (p->ctl.precision != BTE_F32 && p->ctl.precision != BTE_F64) {
        p->err = "precision must be BTE_F32 or BTE_F64";
        return bail(BTE_ERR_ARG);
    }
    if (p->ctl.scheme != BTE_SEQUENTIAL && p->ctl.scheme != BTE_SYNTHETIC) {
        p->err = "scheme must be sequential or synthetic";
        return bail(BTE_ERR_ARG);
    }
    if (p->ctl.limiter < 0 || p->ctl.limiter > 2) {
        p->err = "bad limiter";
        return bail(BTE_ERR_ARG);
    }
    if (p->ctl.max_iter <= 0) p->ctl.max_iter = 10000;
    if (p->ctl.cg_max_iter <= 0) p->ctl.cg_max_iter = 2000;
    if (!(p->ctl.cg_rtol > 0)) p->ctl.cg_rtol = 1e-10;
    if (mat->material_dim != 0 && mat->material_dim != 2 && mat->material_dim != 3) {
        p->err = "material_dim must be 0, 2 or 3";
        return bail(BTE_ERR_ARG);
    }
    const bool planar = mat->material_dim == 2;
    if (planar && geo[0].dim == 3) {
        p->err = "a two-dimensional material takes a 1D or 2D geometry";
        return bail(BTE_ERR_ARG);
    }
    p->omega = planar ? 2.0 * M_PI : 4.0 * M_PI;
    p->Tref = mat->T_ref;
    p->nl = mat->n_bands;
    p->nmat = n_mat;
    const size_t nml = (size_t)n_mat * p->nl;
    p->C4.resize(nml);
    p->v.resize(nml);
    p->itau.resize(nml);
    p->Ctot_m.assign(n_mat, 0.0);
    for (int m = 0; m < n_mat; ++m)
        for (int l = 0; l < p->nl; ++l) {
            const bte_material &mm = mats[m];
            if (!(mm.C[l] > 0) || !(mm.v[l] >= 0) || !(mm.tau[l] > 0)) {
                p->err = "band properties must satisfy C > 0, v >= 0, tau > 0";
                return bail(BTE_ERR_ARG);
            }
            const size_t i = (size_t)m * p->nl + l;
            p->C4[i] = mm.C[l] / p->omega;
            p->v[i] = mm.v[l];
            p->itau[i] = 1.0 / mm.tau[l];
            p->Ctot_m[m] += mm.C[l];
            p->vmax = std::max(p->vmax, mm.v[l]);
            p->itau_max = std::max(p->itau_max, p->itau[i]);
        }
    p->Ctot = p->Ctot_m[0];
    // interfaces: which face of which geometry faces which
    p->nifc = n_ifc;
    p->ifc_end.assign(6 * (size_t)n_geo, bte_problem::IfcEnd{});
    for (int i = 0; i < n_ifc; ++i) {
        const bte_interface &q = ifc[i];
        if (q.geo_a < 0 || q.geo_a >= n_geo || q.geo_b < 0 || q.geo_b >= n_geo || q.face_a < 0 ||
            q.face_a >= 2 * geo[0].dim || q.face_b < 0 || q.face_b >= 2 * geo[0].dim || !q.beta_ab || !q.beta_ba) {
            p->err = "interface " + std::to_string(i) + ": bad geometry, face or beta";
            return bail(BTE_ERR_ARG);
        }
        const int ax = q.face_a >> 1;
        if ((q.face_b >> 1) != ax || q.face_b == q.face_a) {
            p->err = "interface " + std::to_string(i) + ": the faces must be opposite faces of one axis";
            return bail(BTE_ERR_ARG);
        }
        const bte_geometry &ga = geo[q.geo_a], &gb = geo[q.geo_b];
        if (ga.bc[q.face_a] != BTE_BC_INTERFACE || gb.bc[q.face_b] != BTE_BC_INTERFACE) {
            p->err = "interface " + std::to_string(i) + ": both faces must be BTE_BC_INTERFACE";
            return bail(BTE_ERR_ARG);
        }
        for (int a = 0; a < ga.dim; ++a) {
            const double ha = ga.len[a] / ga.n[a], hb = gb.len[a] / gb.n[a];
            const bool same_n = a == ax || ga.n[a] == gb.n[a];
            if (!same_n || std::fabs(ha - hb) > 1e-12 * std::max(ha, hb)) {
                p->err = "interface " + std::to_string(i) + ": the faces do not match cell for cell";
                return bail(BTE_ERR_ARG);
            }
        }
        bte_problem::IfcEnd &ea = p->ifc_end[6 * q.geo_a + q.face_a], &eb = p->ifc_end[6 * q.geo_b + q.face_b];
        if (ea.film >= 0 || eb.film >= 0) {
            p->err = "interface " + std::to_string(i) + ": a face is used twice";
            return bail(BTE_ERR_ARG);
        }
        ea = {q.geo_b, q.face_b, i, 1};
        eb = {q.geo_a, q.face_a, i, 0};
        std::vector<double> bt(2 * (size_t)p->nl);
        for (int l = 0; l < p->nl; ++l) {
            bt[l] = q.beta_ab[l];
            bt[p->nl + l] = q.beta_ba[l];
            if (!(bt[l] >= 0 && bt[l] <= 1) || !(bt[p->nl + l] >= 0 && bt[p->nl + l] <= 1)) {
                p->err = "interface " + std::to_string(i) + ": beta outside [0, 1]";
                return bail(BTE_ERR_ARG);
            }
        }
        p->ifcs.push_back(q);
        p->ifc_beta.push_back(bt);
    }
    if ((st = build_geometry(p, geo, n_geo)) != BTE_OK) return bail(st);
    for (int f = 0; f < n_geo; ++f) {
        Film &fm = p->films[f];
        fm.mat = geo_mat ? geo_mat[f] : 0;
        fm.moff = fm.mat * p->nl;
        fm.Ctot = p->Ctot_m[fm.mat];
    }
    if ((st = build_quadrature(p, mat->n_theta, mat->n_phi, planar)) != BTE_OK) return bail(st);
    finish_materials(p);
    if (n_ifc > 0)
        for (int f = 0; f < n_geo; ++f)
            if (p->films[f].floating) {
                p->err = "with interfaces every geometry needs a thermalizing wall";
                return bail(BTE_ERR_UNSUPPORTED);
            }
    p->nk = p->na * p->nl;
    choose_default_tiles(p);
    build_schedule(p);
    plan_workspace(p);
    *out = p;
    return BTE_OK;
}

bte_status bte_set_control(bte_problem *p, const bte_control *ctl)
{
    if (!p) return BTE_ERR_ARG;
    if (!ctl) FAIL(p, BTE_ERR_ARG, "null control");
    if (ctl->precision != p->ctl.precision) FAIL(p, BTE_ERR_ARG, "precision cannot change after setup");
    if (ctl->scheme != BTE_SEQUENTIAL && ctl->scheme != BTE_SYNTHETIC) FAIL(p, BTE_ERR_ARG, "bad scheme");
    if (ctl->limiter < 0 || ctl->limiter > 2) FAIL(p, BTE_ERR_ARG, "bad limiter");
    if ((ctl->adjoint != 0) != (p->ctl.adjoint != 0)) FAIL(p, BTE_ERR_ARG, "adjoint cannot change after setup");
    p->ctl = *ctl;
    if (p->ctl.max_iter <= 0) p->ctl.max_iter = 10000;
    if (p->ctl.cg_max_iter <= 0) p->ctl.cg_max_iter = 2000;
    if (!(p->ctl.cg_rtol > 0)) p->ctl.cg_rtol = 1e-10;
    p->dev.limiter = p->ctl.limiter;
    return BTE_OK;
}

size_t bte_workspace_bytes(const bte_problem *p) { return p ? p->ws_bytes : 0; }
size_t bte_num_unknowns(const bte_problem *p) { return p ? p->nelem() : 0; }
int bte_num_cells(const bte_problem *p) { return p ? p->nc : 0; }
int bte_num_directions(const bte_problem *p) { return p ? p->na : 0; }

bte_status bte_bind(bte_problem *p, void *ws, size_t bytes)
{
    if (!p) return BTE_ERR_ARG;
    if (!ws || bytes < p->ws_bytes) FAIL(p, BTE_ERR_ARG, "workspace too small (%zu < %zu)", bytes, p->ws_bytes);
    if ((uintptr_t)ws & 255) FAIL(p, BTE_ERR_ARG, "workspace must be 256-byte aligned");
    p->ws = (char *)ws;
    auto up = [&](const char *name, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpy(wsptr<char>(p, name), src, n, hipMemcpyHostToDevice);
    };
    HIPCHK(p, up("s", p->s.data(), 8 * p->s.size()));
    HIPCHK(p, up("w", p->w.data(), 8 * p->w.size()));
    HIPCHK(p, up("mirror", p->mirror.data(), 4 * p->mirror.size()));
    HIPCHK(p, up("C4", p->C4.data(), 8 * p->C4.size()));
    HIPCHK(p, up("v", p->v.data(), 8 * p->v.size()));
    HIPCHK(p, up("itau", p->itau.data(), 8 * p->itau.size()));
    HIPCHK(p, up("wpart", p->wpart.data(), 4 * p->wpart.size()));
    HIPCHK(p, up("wbeta", p->wbeta.data(), 8 * p->wbeta.size()));
    HIPCHK(p, up("film", p->films.data(), sizeof(Film) * p->nfilm));
    HIPCHK(p, up("code", p->code.data(), 4 * (size_t)p->nc));
    HIPCHK(p, up("nb", p->nb.data(), 4 * p->nb.size()));
    HIPCHK(p, up("fid", p->fid.data(), 4 * (size_t)p->nc));
    HIPCHK(p, up("dbase", p->dbase.data(), 4 * (size_t)p->nc));
    HIPCHK(p, up("wrec", p->wrec.data(), 4 * p->wrec.size()));
    HIPCHK(p, up("wden", p->wden, 8 * 6));
    HIPCHK(p, up("items", p->items.data(), sizeof(SweepItem) * p->items.size()));
    if (!p->items2.empty()) HIPCHK(p, up("items2", p->items2.data(), sizeof(Sweep2Item) * p->items2.size()));
    HIPCHK(p, up("titems", p->titems.data(), sizeof(TileItem) * p->titems.size()));
    if (!p->citems.empty()) HIPCHK(p, up("citems", p->citems.data(), sizeof(ColItem) * p->citems.size()));
    if (tile_smem_size(p->tile_cap, (int)p->esize(), 1) > 160 * 1024) FAIL(p, BTE_ERR_UNSUPPORTED, "tile LDS");
    HIPCHK(p, tile_kernels_init(160 * 1024));
    HIPCHK(p, adj_kernels_init(160 * 1024));
    Dev &d = p->dev;
    d.dim = p->dim;
    d.nc = p->nc;
    d.na = p->na;
    d.nl = p->nl;
    d.nk = p->nk;
    d.nfilm = p->nfilm;
    d.jumps = 0;
    for (const Film &fm : p->films)
        for (int a = 0; a < 3; ++a) d.jumps |= (fm.periodic[a] && fm.pdT[a] != 0.0) ? 1 : 0;
    d.limiter = p->ctl.limiter;
    d.Ctot = p->Ctot;
    d.omega = p->omega;
    d.poreT = 0.0;
    d.s = wsptr<double>(p, "s");
    d.w = wsptr<double>(p, "w");
    d.mirror = wsptr<int>(p, "mirror");
    d.C4 = wsptr<double>(p, "C4");
    d.v = wsptr<double>(p, "v");
    d.itau = wsptr<double>(p, "itau");
    d.nmat = p->nmat;
    d.wpart = wsptr<int>(p, "wpart");
    d.wbeta = wsptr<double>(p, "wbeta");
    d.film = wsptr<Film>(p, "film");
    d.code = wsptr<uint32_t>(p, "code");
    d.nb = wsptr<int>(p, "nb");
    d.fid = wsptr<int>(p, "fid");
    d.dbase = wsptr<int>(p, "dbase");
    p->gamma = wsptr<double>(p, "gamma");
    p->P = wsptr<double>(p, "P");
    p->S = wsptr<double>(p, "S");
    d.gamma = p->gamma;
    d.P = nullptr;
    d.S = p->S;
    d.zrow = wsptr<void>(p, "zrow");
    d.fdone = wsptr<int>(p, "fdone");
    p->kdif = wsptr<double>(p, "kdif");
    p->kcor = wsptr<double>(p, "kcor");
    p->cdif = wsptr<double>(p, "cdif");
    p->ccor = wsptr<double>(p, "ccor");
    p->ddif = wsptr<double>(p, "ddif");
    p->dcor = wsptr<double>(p, "dcor");
    p->TL = wsptr<double>(p, "TL");
    p->TLkin = wsptr<double>(p, "TLkin");
    p->T0 = wsptr<double>(p, "T0");
    p->T1 = wsptr<double>(p, "T1");
    p->q0 = wsptr<double>(p, "q0");
    p->q1 = wsptr<double>(p, "q1");
    p->r = wsptr<double>(p, "r");
    p->delta = wsptr<double>(p, "delta");
    p->dpend = wsptr<double>(p, "dpend");
    p->fmean = wsptr<double>(p, "fmean");
    p->feps = wsptr<double>(p, "feps");
    p->fpart = wsptr<double>(p, "fpart");
    p->cg_x = wsptr<double>(p, "cg_x");
    p->cg_r = wsptr<double>(p, "cg_r");
    p->cg_z = wsptr<double>(p, "cg_z");
    p->cg_p = wsptr<double>(p, "cg_p");
    p->cg_Ap = wsptr<double>(p, "cg_Ap");
    p->cg_w0 = wsptr<double>(p, "cg_w0");
    p->cg_w1 = wsptr<double>(p, "cg_w1");
    p->cg_s1 = wsptr<double>(p, "cg_s1");
    p->cg_part = wsptr<double>(p, "cg_part");
    p->cg_scal = wsptr<double>(p, "cg_scal");
    p->din = wsptr<double>(p, "din");
    p->part = wsptr<double>(p, "part");
    p->e2 = wsptr<void>(p, "e2");
    p->psi = wsptr<void>(p, "psi");
    p->psi2 = wsptr<void>(p, "psi2");
    p->adjX = wsptr<double>(p, "adjX");
    p->adjT = wsptr<double>(p, "adjT");
    p->adjTL = wsptr<double>(p, "adjTL");
    p->adju = wsptr<double>(p, "adju");
    p->adjr2 = wsptr<double>(p, "adjr2");
    p->d_items = wsptr<SweepItem>(p, "items");
    p->d_items2 = wsptr<Sweep2Item>(p, "items2");
    p->d_queue = wsptr<unsigned>(p, "queue");
    p->d_titems = wsptr<TileItem>(p, "titems");
    p->d_citems = wsptr<ColItem>(p, "citems");
    p->d_wrec = wsptr<int>(p, "wrec");
    p->d_wden = wsptr<double>(p, "wden");
    // default fields: no source, no extra scattering
    HIPCHK(p, hipMemset(wsptr<void>(p, "zrow"), 0, 8 * 8 * (size_t)p->nk));
    HIPCHK(p, hipMemset(wsptr<void>(p, "fdone"), 0, 4 * (size_t)p->nfilm));
    HIPCHK(p, hipMemset(p->gamma, 0, 8 * (size_t)p->nc));
    HIPCHK(p, hipMemset(p->P, 0, 8 * (size_t)p->nc));
    cell_setup(p, nullptr);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipDeviceSynchronize());
    p->fields_set = true;
    return BTE_OK;
}

bte_status bte_set_fields(bte_problem *p, const double *P_dev, const double *gamma_dev, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = 8 * (size_t)p->nc;
    if (P_dev) HIPCHK(p, hipMemcpyAsync(p->P, P_dev, nb, hipMemcpyDeviceToDevice, s));
    else HIPCHK(p, hipMemsetAsync(p->P, 0, nb, s));
    if (gamma_dev) HIPCHK(p, hipMemcpyAsync(p->gamma, gamma_dev, nb, hipMemcpyDeviceToDevice, s));
    else HIPCHK(p, hipMemsetAsync(p->gamma, 0, nb, s));
    p->dev.P = P_dev ? p->P : nullptr;
    cell_setup(p, s);
    HIPCHK(p, hipGetLastError());
    return BTE_OK;
}

}  // extern "C"

// ------------------------------------------------------------- device flows

namespace {

// CG arguments of the heat-diffusion (corr = 0) or correction (corr = 1) operator
CgArgs cg_args(bte_problem *p, int corr)
{
    CgArgs g{};
    g.kax = corr ? p->kcor : p->kdif;
    g.coef = corr ? p->ccor : p->cdif;
    g.dg = corr ? p->dcor : p->ddif;
    g.corr = corr;
    g.p = p->cg_p;
    g.rb[0] = p->cg_r;
    g.rb[1] = p->cg_z;
    g.wb[0] = p->cg_w0;
    g.wb[1] = p->cg_w1;
    g.sb[0] = p->cg_Ap;
    g.sb[1] = p->cg_s1;
    g.part = p->cg_part;
    g.scal = p->cg_scal;
    return g;
}

// per-cell quantities that depend on gamma: S, conductivities, CG couplings
void cell_setup(bte_problem *p, hipStream_t s)
{
    launch_cell_setup(p->dev, p->S, p->kdif, p->kcor, p->M, p->H, s);
    for (int corr = 0; corr < 2; ++corr) {
        CgArgs g = cg_args(p, corr);
        launch_cg_coef(p->dev, g, corr ? p->ccor : p->cdif, corr ? p->dcor : p->ddif, s);
    }
}

template <typename T> bte_status moments_to(bte_problem *p, const T *e, const double *dpend, hipStream_t s)
{
    // one partial per cell in part[0]
    launch_moments<T>(p->dev, e, dpend, p->part, s);
    return BTE_OK;
}

// Jacobi-preconditioned CG on the heat-diffusion (corr = 0) or correction
// (corr = 1) operator, two launches per iteration; b is projected per
// floating geometry beforehand, x afterwards.  Asynchronous when maxit fits
// one chunk of launches; the iteration count is accumulated on the device
// (cg_scal[9]).  Returns false on a HIP error.
constexpr int kCgChunk = 64;

bool run_cg(bte_problem *p, int corr, double *b, double *x_out, double rtol, int maxit, hipStream_t s)
{
    const Dev &d = p->dev;
    if (p->floating_any) {
        launch_film_mean(d, b, p->fmean, p->fpart, p->fseg, s);
        launch_sub_film_mean(d, b, p->fmean, s);
    }
    CgArgs g = cg_args(p, corr);
    g.x = x_out;
    g.rtol2 = rtol * rtol;
    // one launch per iteration, enqueued in chunks; between chunks the host
    // reads the done flag (one synchronisation per chunk)
    launch_cg_begin(d, g, b, s);
    constexpr int kChunk = kCgChunk;
    for (int it0 = 0; it0 < maxit; it0 += kChunk) {
        launch_cg_iters(d, g, it0, std::min(kChunk, maxit - it0), s);
        if (it0 + kChunk < maxit) {
            double done = 0;
            if (hipMemcpyAsync(&done, p->cg_scal + 5, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
            if (hipStreamSynchronize(s) != hipSuccess) return false;
            if (done != 0.0) break;
        }
    }
    if (p->floating_any) {
        launch_film_mean(d, x_out, p->fmean, p->fpart, p->fseg, s);
        launch_sub_film_mean(d, x_out, p->fmean, s);
    }
    return hipGetLastError() == hipSuccess;
}

// A captured launch sequence, instantiated once and replayed.
struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipStream_t s = nullptr;
    ~Graph()
    {
        if (x) {
            (void)hipStreamSynchronize(s);   // no replay of it is left in flight
            (void)hipGraphExecDestroy(x);
        }
        if (g) (void)hipGraphDestroy(g);
    }
};

// Capture the work `enqueue(cs)` puts on the capture stream cs into `gr`
// (first call) and replay it on stream s (every call).  Kernels only:
// nothing here records a memset.
template <typename F> hipError_t graph_run(Graph &gr, hipStream_t cs, hipStream_t s, F &&enqueue)
{
    hipError_t r;
    if (!gr.x) {
        gr.s = s;
        if ((r = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return r;
        const bool ok = enqueue(cs);
        r = hipStreamEndCapture(cs, &gr.g);
        if (!ok && r == hipSuccess) r = hipErrorUnknown;
        if (r != hipSuccess) return r;
        if ((r = hipGraphInstantiate(&gr.x, gr.g, nullptr, nullptr, 0)) != hipSuccess) return r;
    }
    return hipGraphLaunch(gr.x, s);
}

// One forward sweep (every tile-diagonal launch) from ein into eout: the
// register-tile kernel for 2D geometries with 8 x 8 tiles, the column
// segments in 3D, the LDS tiles otherwise.
template <typename T> hipError_t sweep_launches(bte_problem *p, const T *ein, T *eout, hipStream_t q)
{
    const Dev &d = p->dev;
    const bool reg = reg2d(p);
    const int3 lt = lds_tdim(p);
    if (reg && p->persistent && p->queue_ok) {
        // the whole sweep in one launch: every item waits for its upwind items
        const int n = (int)p->items2.size();
        hipError_t r = launch_queue_reset(p->d_queue, n, q);
        if (r == hipSuccess)
            r = launch_sweep2d<T>(d, ein, eout, p->dpend, p->TL, p->din, p->d_items2, 0, n, p->tdim.z, p->na_oct,
                                  p->nchunk_oct, p->part, p->d_queue, q);
        return r;
    }
    for (size_t dg = 0; dg + 1 < p->diag_off.size(); ++dg) {
        const int i0 = p->diag_off[dg], cnt = p->diag_off[dg + 1] - i0;
        const hipError_t r =
            reg ? launch_sweep2d<T>(d, ein, eout, p->dpend, p->TL, p->din, p->d_items2, i0, cnt, p->tdim.z, p->na_oct,
                                    p->nchunk_oct, p->part, nullptr, q)
                : launch_sweep_tile<T>(d, ein, eout, p->dpend, p->TL, p->din, p->d_items, i0, cnt, lt, p->na_oct,
                                       p->nchunk_oct, p->tile_cap, p->part, q);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

template <typename T>
bte_status steady_impl(bte_problem *p, T *e, int init, bte_solve_stats *stats, hipStream_t s)
{
    if (p->dim == 3 && !seg_fits(p, p->tdim.z))
        FAIL(p, BTE_ERR_UNSUPPORTED, "a z plane of a geometry is too large for the 3D sweep's 32-bit row offsets");
    auto t0 = std::chrono::steady_clock::now();
    const Dev &d = p->dev;
    const int nc = p->nc;
    const int synthetic = p->ctl.scheme == BTE_SYNTHETIC;
    bte_solve_stats st{};
    T *buf[2] = {e, (T *)p->e2};
    int cur = 0;
    HIPCHK(p, hipMemsetAsync(p->dpend, 0, 8 * (size_t)nc, s));
    HIPCHK(p, hipMemsetAsync(p->cg_scal, 0, 8 * 16, s));
    if (init) {
        CgArgs g = cg_args(p, 0);
        launch_diff_rhs(d, g, p->r, s);
        if (!run_cg(p, 0, p->r, p->T0, 1e-13, 200000, s)) FAIL(p, BTE_ERR_HIP, "CG failed");
        launch_set_equilibrium<T>(d, e, p->T0, s);
        HIPCHK(p, hipMemsetAsync(p->cg_scal, 0, 8 * 16, s));   // count correction CG only
    }
    // moments of the start field
    launch_moments<T>(d, e, nullptr, p->part, s);
    launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->TL, p->T0, p->q0, s);
    std::vector<double> feps(5 * (size_t)p->nfilm);
    // per-geometry convergence: a converged geometry is no longer swept or
    // corrected (its field, T_L and pending correction stay as they were
    // when it met the tolerances)
    std::vector<int> fdone(p->nfilm, 0);
    int ndone = 0;
    int *fdone_dev = const_cast<int *>(d.fdone);
    const int np = p->noct * p->nchunk_oct;
    bte_status ret = BTE_ERR_NOT_CONVERGED;
    // phase timers: events on the solve stream, read after the per-iteration sync
    hipEvent_t ev[5];
    for (auto &x : ev) HIPCHK(p, hipEventCreate(&x));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    double active_cells = 0;
    for (const Film &fm : p->films) active_cells += fm.ncell;
    Graph gsweep[2], gcg;   // captured in this call, replayed by its iterations
    if (p->graphs && !p->cstream) HIPCHK(p, hipStreamCreateWithFlags(&p->cstream, hipStreamNonBlocking));
    for (int iter = 1; iter <= p->ctl.max_iter; ++iter) {
        const T *ein = buf[cur];
        T *eout = buf[1 - cur];
        st.updates += active_cells * (double)p->nk;
        HIPCHK(p, hipEventRecord(ev[0], s));
        launch_walls<T>(d, ein, p->dpend, p->d_wrec, p->d_wden, p->din, p->nw, s);
        HIPCHK(p, hipEventRecord(ev[1], s));
        auto sweep = [&](hipStream_t q) -> bool { return sweep_launches<T>(p, ein, eout, q) == hipSuccess; };
        if (p->graphs) {
            HIPCHK(p, graph_run(gsweep[cur], p->cstream, s, sweep));
        } else if (!sweep(s)) {
            FAIL(p, BTE_ERR_HIP, "sweep launch failed");
        }
        if (reg2d(p) && p->persistent && p->queue_ok) st.sweep_launches += 1;
        else
            for (size_t dg = 0; dg + 1 < p->diag_off.size(); ++dg)
                st.sweep_launches += p->diag_off[dg + 1] > p->diag_off[dg];
        HIPCHK(p, hipEventRecord(ev[2], s));
        launch_steady_post(d, p->part, np, p->TL, p->TLkin, p->T1, p->q1, p->r, synthetic, s);
        launch_film_eps(d, p->T0, p->T1, p->q0, p->q1, p->feps, p->fpart, p->fseg, s);
        HIPCHK(p, hipEventRecord(ev[3], s));
        HIPCHK(p, hipGetLastError());
        if (synthetic) {
            // a CG solve without host checks (cg_max_iter <= one chunk) is a
            // fixed launch sequence: replayed from a graph
            if (p->graphs && p->ctl.cg_max_iter <= kCgChunk) {
                HIPCHK(p, graph_run(gcg, p->cstream, s, [&](hipStream_t q) {
                    return run_cg(p, 1, p->r, p->delta, p->ctl.cg_rtol, p->ctl.cg_max_iter, q);
                }));
            } else if (!run_cg(p, 1, p->r, p->delta, p->ctl.cg_rtol, p->ctl.cg_max_iter, s)) {
                FAIL(p, BTE_ERR_HIP, "CG failed");
            }
            launch_tl_update(nc, p->TLkin, p->delta, p->TL, p->dpend, d.fid, d.fdone, s);
        } else {
            launch_tl_update(nc, p->TLkin, nullptr, p->TL, nullptr, d.fid, d.fdone, s);
        }
        HIPCHK(p, hipEventRecord(ev[4], s));
        HIPCHK(p, hipMemcpyAsync(feps.data(), p->feps, 8 * feps.size(), hipMemcpyDeviceToHost, s));
        unsigned qabort = 0;
        if (reg2d(p) && p->persistent && p->queue_ok)
            HIPCHK(p, hipMemcpyAsync(&qabort, p->d_queue + 1, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(p, hipStreamSynchronize(s));
        if (qabort) FAIL(p, BTE_ERR_HIP, "one-launch sweep: a wait for an upwind tile gave up");
        {
            float ms[4];
            for (int i = 0; i < 4; ++i) HIPCHK(p, hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
            st.ms_walls += ms[0];
            st.ms_sweep += ms[1];
            st.ms_post += ms[2];
            st.ms_cg += ms[3];
        }
        double eT = 0, eq = 0;
        bool finite = true;
        std::vector<int> newly;
        for (int f = 0; f < p->nfilm; ++f) {
            if (fdone[f]) continue;
            const Film &fm = p->films[f];
            const double *o = &feps[5 * f];
            double a = std::sqrt(o[0] / fm.nsolid) / (o[1] > 1e-300 ? o[1] : 1.0);
            double b = std::sqrt(o[2] / fm.nsolid) / (o[3] > 1e-300 ? o[3] : 1.0);
            if (!std::isfinite(a) || !std::isfinite(b)) finite = false;
            eT = std::max(eT, a);
            eq = std::max(eq, b);
            if (a <= p->ctl.residual_temp && b <= p->ctl.residual_flux) newly.push_back(f);
        }
        // geometries joined by interfaces converge together: no masks
        if (p->nifc > 0 && (int)newly.size() < p->nfilm) newly.clear();
        std::swap(p->T0, p->T1);
        std::swap(p->q0, p->q1);
        cur = 1 - cur;
        st.iters = iter;
        st.eps_T = eT;
        st.eps_q = eq;
        if (!finite) {
            ret = BTE_ERR_NONFINITE;
            break;
        }
        if (ndone + (int)newly.size() == p->nfilm) {
            st.converged = 1;
            ret = BTE_OK;
            break;
        }
        if (!newly.empty()) {
            // both buffers hold the converged field of these geometries from now on
            for (int f : newly) {
                const Film &fm = p->films[f];
                const size_t off = (size_t)fm.cell0 * p->nk, cnt = (size_t)fm.ncell * p->nk;
                HIPCHK(p, hipMemcpyAsync(buf[1 - cur] + off, buf[cur] + off, cnt * sizeof(T), hipMemcpyDeviceToDevice,
                                         s));
                fdone[f] = 1;
                ++ndone;
                active_cells -= fm.ncell;
            }
            HIPCHK(p, hipMemcpyAsync(fdone_dev, fdone.data(), 4 * fdone.size(), hipMemcpyHostToDevice, s));
        }
    }
    // later calls (and the adjoint) sweep every geometry again
    HIPCHK(p, hipMemsetAsync(fdone_dev, 0, 4 * (size_t)p->nfilm, s));
    // final field: pending correction and, for floating geometries, the gauge
    // shift to zero mean T - T_ref (T0 now holds the last moments)
    double *fshift = nullptr;
    if (p->floating_any) {
        launch_film_mean(d, p->T0, p->fmean, p->fpart, p->fseg, s);
        // only floating films are shifted: zero the others on the host side
        std::vector<double> fm(p->nfilm);
        HIPCHK(p, hipMemcpyAsync(fm.data(), p->fmean, 8 * fm.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(p, hipStreamSynchronize(s));
        for (int f = 0; f < p->nfilm; ++f)
            if (!p->films[f].floating) fm[f] = 0.0;
        HIPCHK(p, hipMemcpyAsync(p->fmean, fm.data(), 8 * fm.size(), hipMemcpyHostToDevice, s));
        fshift = p->fmean;
    }
    launch_apply_shift<T>(d, buf[cur], e, synthetic ? p->dpend : nullptr, fshift, s);
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipStreamSynchronize(s));
    {
        double sc[16];
        HIPCHK(p, hipMemcpy(sc, p->cg_scal, sizeof sc, hipMemcpyDeviceToHost));
        st.cg_iters = (int)sc[9];
    }
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    p->last = st;
    if (stats) *stats = st;
    if (ret == BTE_ERR_NOT_CONVERGED) p->err = "not converged within max_iter";
    if (ret == BTE_ERR_NONFINITE) p->err = "non-finite convergence measure";
    return ret;
}

// Source factor of the pulse {t_centre, FWHM} at time t (1 without a pulse)
double pulse_factor(const double *pulse, double t)
{
    if (!pulse) return 1.0;
    const double x = t - pulse[0];
    return std::exp(-4.0 * std::log(2.0) * x * x / (pulse[1] * pulse[1]));
}

// One explicit step ein -> eout (Sec. 4.1); p->TL holds T_L of ein on entry
// and of eout on exit.  ev: 4 events (before walls, before and after the
// transport kernel, after T_L) or null.
template <typename T>
hipError_t one_step(bte_problem *p, const T *ein, T *eout, double src, hipEvent_t *ev, hipStream_t s)
{
    const Dev &d = p->dev;
    hipError_t r;
    if (ev && (r = hipEventRecord(ev[0], s)) != hipSuccess) return r;
    launch_walls<T>(d, ein, nullptr, p->d_wrec, p->d_wden, p->din, p->nw, s);
    if (ev && (r = hipEventRecord(ev[1], s)) != hipSuccess) return r;
    // three-dimensional geometries: column kernel, partials per (octant,
    // chunk); otherwise the tile kernel, partials per octant
    int np = p->noct;
    if (p->dim == 3) {
        r = launch_transient3d<T>(d, ein, eout, p->TL, p->din, p->d_citems, (int)p->citems.size(), p->na_oct,
                                  p->nchunk_oct, src, p->ctl.dt, p->part, s);
        np = p->noct * p->nchunk_oct;
    } else {
        r = launch_transient_tile<T>(d, ein, eout, p->TL, p->din, p->d_titems, (int)p->titems.size(), p->tdim_tr,
                                     p->na_oct, p->nchunk_oct, p->tile_cap_tr, src, p->ctl.dt, p->part, s);
    }
    if (r != hipSuccess) return r;
    if (ev && (r = hipEventRecord(ev[2], s)) != hipSuccess) return r;
    launch_finalize_tl(d, p->part, np, p->TL, s);
    if (ev && (r = hipEventRecord(ev[3], s)) != hipSuccess) return r;
    return hipGetLastError();
}

template <typename T>
bte_status transient_impl(bte_problem *p, T *e, int n_steps, double t0, const double *pulse, hipStream_t s)
{
    const Dev &d = p->dev;
    const double dt = p->ctl.dt;
    T *buf[2] = {e, (T *)p->e2};
    int cur = 0;
    const auto h0 = std::chrono::steady_clock::now();
    // with timing on: events before the walls, before and after the transport
    // kernel and after the T_L update of every step
    const bool timing = p->timing && n_steps > 0;
    if (timing)
        while (p->tev.size() < 4 * (size_t)n_steps) {
            hipEvent_t x;
            HIPCHK(p, hipEventCreate(&x));
            p->tev.push_back(x);
        }
    launch_moments<T>(d, e, nullptr, p->part, s);
    launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->TL, nullptr, nullptr, s);
    for (int n = 0; n < n_steps; ++n) {
        const double src = pulse_factor(pulse, t0 + n * dt);
        HIPCHK(p, one_step<T>(p, buf[cur], buf[1 - cur], src, timing ? &p->tev[4 * n] : nullptr, s));
        cur = 1 - cur;
    }
    if (cur != 0) HIPCHK(p, hipMemcpyAsync(e, buf[cur], p->esize() * p->nelem(), hipMemcpyDeviceToDevice, s));
    HIPCHK(p, hipGetLastError());
    if (timing) {
        bte_solve_stats st{};
        HIPCHK(p, hipEventSynchronize(p->tev[4 * (size_t)n_steps - 1]));
        for (int n = 0; n < n_steps; ++n) {
            float ms[3];
            for (int i = 0; i < 3; ++i) HIPCHK(p, hipEventElapsedTime(&ms[i], p->tev[4 * n + i], p->tev[4 * n + i + 1]));
            st.ms_walls += ms[0];
            st.ms_sweep += ms[1];
            st.ms_post += ms[2];
        }
        st.iters = n_steps;
        st.sweep_launches = n_steps;
        st.updates = (double)n_steps * (double)p->nelem();
        st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
        p->last = st;
    }
    return BTE_OK;
}

// Adjoint of the steady problem for J = k_eff (x): transposed synthetic
// iteration (see bte_adjoint.hip), then the gradient pass.  Stops when the
// residual |J^T psi + g| / |g| of every geometry is <= ctl.residual_temp.
template <typename T>
bte_status adjoint_impl(bte_problem *p, const T *e, double *grad, bte_solve_stats *stats, hipStream_t s)
{
    if (p->dim == 3 && !seg_fits(p, p->tdim.z))
        FAIL(p, BTE_ERR_UNSUPPORTED, "a z plane of a geometry is too large for the 3D sweep's 32-bit row offsets");
    auto t0 = std::chrono::steady_clock::now();
    const Dev &d = p->dev;
    const int nc = p->nc;
    const int synthetic = p->ctl.scheme == BTE_SYNTHETIC;
    bte_solve_stats st{};
    T *buf[2] = {(T *)p->psi, (T *)p->psi2};
    int cur = 0;
    // forward T and T_L deviations of e
    launch_moments<T>(d, e, nullptr, p->part, s);
    launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->adjTL, p->adjT, nullptr, s);
    HIPCHK(p, hipMemsetAsync(buf[0], 0, p->esize() * p->nelem(), s));
    HIPCHK(p, hipMemsetAsync(p->adjX, 0, 8 * (size_t)nc, s));
    HIPCHK(p, hipMemsetAsync(p->cg_scal, 0, 8 * 16, s));
    // |g|^2 per geometry: g = (L_x / (dT_x N_cells)) w v s_x on solid cells
    double sws = 0, svv = 0;
    for (int al = 0; al < p->na; ++al) sws += p->w[al] * p->w[al] * p->s[3 * al] * p->s[3 * al];
    for (int l = 0; l < p->nl; ++l) svv += p->v[l] * p->v[l];
    std::vector<double> g2(p->nfilm), mres(p->nfilm);
    for (int f = 0; f < p->nfilm; ++f) {
        const Film &fm = p->films[f];
        const double gf = fm.len[0] / (fm.pdT[0] * fm.ncell);
        g2[f] = gf * gf * fm.nsolid * sws * svv;
    }
    const int np = p->noct * p->nchunk_oct;
    bte_status ret = BTE_ERR_NOT_CONVERGED;
    hipEvent_t ev[5];
    for (auto &x : ev) HIPCHK(p, hipEventCreate(&x));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    for (int iter = 0;; ++iter) {
        const T *pin = buf[cur];
        T *pout = buf[1 - cur];
        HIPCHK(p, hipEventRecord(ev[0], s));
        launch_walls_adj<T>(d, pin, p->d_wrec, p->d_wden, p->din, p->nw, s);
        HIPCHK(p, hipEventRecord(ev[1], s));
        if (p->dim == 3) {
            // column walk: partials per (octant, chunk, cell)
            HIPCHK(p, launch_adj_res3d<T>(d, pin, p->adjX, p->din, p->d_citems, (int)p->citems.size(), p->na_oct,
                                          p->nchunk_oct, p->part, s));
            launch_adj_post(d, p->part, np, p->adju, p->adjr2, s);
        } else {
            HIPCHK(p, launch_adj_res<T>(d, pin, p->adjX, p->din, p->d_titems, (int)p->titems.size(), p->tdim_tr,
                                        p->na_oct, p->nchunk_oct, p->tile_cap_tr, p->part, s));
            launch_adj_post(d, p->part, p->noct, p->adju, p->adjr2, s);
        }
        launch_film_mean(d, p->adjr2, p->fmean, p->fpart, p->fseg, s);
        HIPCHK(p, hipEventRecord(ev[2], s));
        HIPCHK(p, hipMemcpyAsync(mres.data(), p->fmean, 8 * mres.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(p, hipStreamSynchronize(s));
        {
            float ms[2];
            for (int i = 0; i < 2; ++i) HIPCHK(p, hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
            st.ms_walls += ms[0];
            st.ms_post += ms[1];
        }
        double eps = 0;
        bool finite = true;
        for (int f = 0; f < p->nfilm; ++f) {
            const double r = std::sqrt(mres[f] * p->films[f].nsolid / g2[f]);
            if (!std::isfinite(r)) finite = false;
            eps = std::max(eps, r);
        }
        st.eps_T = eps;
        if (!finite) {
            ret = BTE_ERR_NONFINITE;
            p->err = "non-finite adjoint residual";
            break;
        }
        if (eps <= p->ctl.residual_temp) {
            st.converged = 1;
            ret = BTE_OK;
            break;
        }
        if (iter >= p->ctl.max_iter) {
            p->err = "adjoint: max_iter reached";
            break;
        }
        const double *X = p->adjX;
        HIPCHK(p, hipEventRecord(ev[2], s));
        if (synthetic) {
            // v = L^-1 P^T y; the sweep's isotropic term becomes X + v
            if (!run_cg(p, 1, p->adju, p->delta, p->ctl.cg_rtol, p->ctl.cg_max_iter, s))
                FAIL(p, BTE_ERR_HIP, "CG failed");
            launch_tl_update(nc, p->adjX, p->delta, p->TL, nullptr, nullptr, nullptr, s);
            X = p->TL;
        }
        HIPCHK(p, hipEventRecord(ev[3], s));
        for (size_t dg = 0; dg + 1 < p->diag_off.size(); ++dg) {
            const int i0 = p->diag_off[dg], cnt = p->diag_off[dg + 1] - i0;
            HIPCHK(p, launch_sweep_adj<T>(d, pin, pout, X, p->din, p->d_items, i0, cnt, lds_tdim(p), p->na_oct,
                                          p->nchunk_oct, p->tile_cap, p->part, s));
            st.sweep_launches += cnt > 0;
        }
        launch_adj_phi(d, p->part, np, p->adjX, s);
        HIPCHK(p, hipEventRecord(ev[4], s));
        HIPCHK(p, hipEventSynchronize(ev[4]));
        {
            float ms[2];
            for (int i = 0; i < 2; ++i) HIPCHK(p, hipEventElapsedTime(&ms[i], ev[2 + i], ev[3 + i]));
            st.ms_cg += ms[0];
            st.ms_sweep += ms[1];
        }
        cur = 1 - cur;
        st.iters = iter + 1;
        st.updates += (double)p->nelem();
    }
    launch_adj_grad<T>(d, e, buf[cur], p->adjT, p->adjTL, p->adjX, grad, s);
    HIPCHK(p, hipGetLastError());
    double cgit = 0;
    HIPCHK(p, hipMemcpyAsync(&cgit, p->cg_scal + 9, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    st.cg_iters = (int)cgit;
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    p->last = st;
    if (stats) *stats = st;
    return ret;
}

// Transient adjoint (reverse mode of the explicit steps, Sec. 4.1) for
// J = sum_c a_c T_c(e^N) / sum_c a_c.  The forward pass keeps e every `every`
// steps (ck[0 .. nseg)); the backward pass recomputes one segment at a time
// into ck[nseg .. nseg + every) and runs the transposed steps on it.
template <typename T>
bte_status tadj_impl(bte_problem *p, const T *e0, int n_steps, double t0, const double *pulse, const double *a,
                     int every, char *ck, double *J_host, double *grad, bte_solve_stats *stats, hipStream_t s)
{
    auto h0 = std::chrono::steady_clock::now();
    const Dev &d = p->dev;
    const size_t bytes = p->esize() * p->nelem();
    const int nseg = (n_steps + every - 1) / every;
    const double dt = p->ctl.dt;
    // checkpoints 1 .. nseg - 1 (the state after i * every steps; checkpoint
    // 0 is e0 itself, read in place), then the recomputed states
    // 1 .. every - 1 of the current segment
    auto CK = [&](int i) -> T * { return reinterpret_cast<T *>(ck + (size_t)(i - 1) * bytes); };
    auto SG = [&](int j) -> T * { return reinterpret_cast<T *>(ck + (size_t)(nseg - 2 + j) * bytes); };
    // T_L of each checkpoint 0 .. nseg - 1, so that a recomputed segment
    // repeats the forward pass bit for bit, then T_L of the recomputed
    // states 1 .. every - 1 (the lattice temperature each transposed step
    // needs)
    auto CTL = [&](int i) {
        return reinterpret_cast<double *>(ck + (size_t)(nseg + every - 2) * bytes) + (size_t)i * p->nc;
    };
    auto STL = [&](int j) { return CTL(nseg - 1 + j); };
    const size_t tlb = 8 * (size_t)p->nc;
    T *buf[2] = {(T *)p->psi, (T *)p->psi2};
    while (p->tev.size() < 3) {
        hipEvent_t x;
        HIPCHK(p, hipEventCreate(&x));
        p->tev.push_back(x);
    }
    HIPCHK(p, hipEventRecord(p->tev[0], s));
    // forward pass: a step whose result is a checkpoint writes it in place
    launch_moments<T>(d, e0, nullptr, p->part, s);
    launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->TL, nullptr, nullptr, s);
    HIPCHK(p, hipMemcpyAsync(CTL(0), p->TL, tlb, hipMemcpyDeviceToDevice, s));
    const T *cur = e0;
    for (int n = 0; n < n_steps; ++n) {
        const bool keep = (n + 1) % every == 0 && n + 1 < n_steps;
        T *dst = keep ? CK((n + 1) / every) : (cur == buf[0] ? buf[1] : buf[0]);
        HIPCHK(p, one_step<T>(p, cur, dst, pulse_factor(pulse, t0 + n * dt), nullptr, s));
        cur = dst;
        if (keep) HIPCHK(p, hipMemcpyAsync(CTL((n + 1) / every), p->TL, tlb, hipMemcpyDeviceToDevice, s));
    }
    // J from the final state
    launch_moments<T>(d, cur, nullptr, p->part, s);
    launch_finalize(d, p->part, 1, p->Tref, p->T1, nullptr, nullptr, nullptr, nullptr, nullptr, s);
    launch_tave(d, a, p->T1, p->fmean, s);
    HIPCHK(p, hipEventRecord(p->tev[1], s));
    double jt[2];
    HIPCHK(p, hipMemcpyAsync(jt, p->fmean, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    if (!(jt[1] > 0)) FAIL(p, BTE_ERR_ARG, "weights must have a positive sum");
    if (J_host) *J_host = jt[0];
    // backward pass (the two step buffers now hold lambda)
    T *lam[2] = {buf[0], buf[1]};
    double *X[2] = {p->adjX, p->adju};
    launch_adj_tave_init<T>(d, a, 1.0 / jt[1], lam[0], s);
    launch_adj_phi_cell<T>(d, lam[0], X[0], s);
    HIPCHK(p, hipMemsetAsync(grad, 0, 8 * (size_t)p->nc, s));
    int lc = 0;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int start = sg * every, len = std::min(every, n_steps - start);
        const T *first = sg == 0 ? e0 : CK(sg);
        auto state = [&](int j) -> const T * { return j == 0 ? first : SG(j); };
        HIPCHK(p, hipMemcpyAsync(p->TL, CTL(sg), tlb, hipMemcpyDeviceToDevice, s));
        for (int j = 1; j < len; ++j) {
            HIPCHK(p, one_step<T>(p, state(j - 1), SG(j), pulse_factor(pulse, t0 + (start + j - 1) * dt), nullptr, s));
            HIPCHK(p, hipMemcpyAsync(STL(j), p->TL, tlb, hipMemcpyDeviceToDevice, s));
        }
        for (int j = len - 1; j >= 0; --j) {
            const double *tlk = j == 0 ? CTL(sg) : STL(j);
            launch_walls_adj<T>(d, lam[lc], p->d_wrec, p->d_wden, p->din, p->nw, s);
            int np = p->noct;
            if (p->dim == 3) {
                HIPCHK(p, launch_adj_step3d<T>(d, lam[lc], lam[1 - lc], state(j), X[lc], tlk, p->din, p->d_citems,
                                               (int)p->citems.size(), p->na_oct, p->nchunk_oct, dt, p->part, s));
                np = p->noct * p->nchunk_oct;
            } else {
                HIPCHK(p, launch_adj_step<T>(d, lam[lc], lam[1 - lc], state(j), X[lc], tlk, p->din, p->d_titems,
                                             (int)p->titems.size(), p->tdim_tr, p->na_oct, p->nchunk_oct,
                                             p->tile_cap_tr, dt, p->part, s));
            }
            launch_adj_step_post(d, p->part, np, X[lc], tlk, X[1 - lc], grad, dt, s);
            lc = 1 - lc;
        }
    }
    HIPCHK(p, hipEventRecord(p->tev[2], s));
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipStreamSynchronize(s));
    bte_solve_stats st{};
    st.iters = n_steps;
    st.updates = (double)(2 * n_steps - nseg + n_steps) * (double)p->nelem();   // forward, recompute, transposed
    st.converged = 1;
    float ms[2];
    HIPCHK(p, hipEventElapsedTime(&ms[0], p->tev[0], p->tev[1]));
    HIPCHK(p, hipEventElapsedTime(&ms[1], p->tev[1], p->tev[2]));
    st.ms_sweep = ms[0];
    st.ms_post = ms[1];
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
    p->last = st;
    if (stats) *stats = st;
    return BTE_OK;
}

// dt stability check shared by the transient calls
bte_status check_cfl(bte_problem *p)
{
    if (!(p->ctl.dt > 0)) FAIL(p, BTE_ERR_ARG, "control.dt must be > 0");
    double adv = 0;
    for (const Film &fm : p->films) {
        double x = 0;
        for (int q = 0; q < p->dim; ++q) x += fm.ih[q];
        adv = std::max(adv, x);
    }
    if (p->ctl.dt * p->itau_max >= 1.0 || p->ctl.dt * p->vmax * adv >= 1.0)
        FAIL(p, BTE_ERR_CFL, "dt violates dt/tau_min < 1 or dt v_max sum_a 1/h_a < 1");
    return BTE_OK;
}

}  // namespace

extern "C" {

bte_status bte_moments(bte_problem *p, const void *e_dev, double *T_dev, double *TL_dev, double *q_dev, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) FAIL(p, BTE_ERR_ARG, "e is null");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64) launch_moments<double>(p->dev, (const double *)e_dev, nullptr, p->part, s);
    else launch_moments<float>(p->dev, (const float *)e_dev, nullptr, p->part, s);
    launch_finalize(p->dev, p->part, 1, p->Tref, T_dev, TL_dev, q_dev, nullptr, nullptr, nullptr, s);
    HIPCHK(p, hipGetLastError());
    return BTE_OK;
}

}  // extern "C"

namespace {
// Scratch of bte_moments_static: the FP64 moment partials (kMomN per cell)
// in a static device array, one copy on every GPU the library runs on, held
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): the address
// is looked up once per device with hipGetSymbolAddress and kept.
constexpr size_t kStaticScratchBytes = (size_t)BTE_STATIC_MAX_CELLS * kMomN * sizeof(double);
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call on each device), or null with the HIP error in *err
double *static_scratch(hipError_t *err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

bte_status bte_moments_static(bte_problem *p, const void *e_dev, double *T_dev, double *TL_dev, double *q_dev,
                              void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) FAIL(p, BTE_ERR_ARG, "e is null");
    if (p->nc > BTE_STATIC_MAX_CELLS)
        FAIL(p, BTE_ERR_ARG, "%d cells exceed the static scratch of bte_moments_static (%d cells)", p->nc,
             BTE_STATIC_MAX_CELLS);
    hipError_t herr = hipSuccess;
    double *part = static_scratch(&herr);
    if (!part) FAIL(p, BTE_ERR_HIP, "static scratch: %s", hipGetErrorString(herr));
    hipStream_t s = (hipStream_t)stream;
    // every partial the finalize kernel reads is written first: nothing has
    // to be cleared
    if (p->ctl.precision == BTE_F64) launch_moments<double>(p->dev, (const double *)e_dev, nullptr, part, s);
    else launch_moments<float>(p->dev, (const float *)e_dev, nullptr, part, s);
    launch_finalize(p->dev, part, 1, p->Tref, T_dev, TL_dev, q_dev, nullptr, nullptr, nullptr, s);
    HIPCHK(p, hipGetLastError());
    return BTE_OK;
}

bte_status bte_residual(bte_problem *p, const void *e_dev, void *R_dev, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev || !R_dev) FAIL(p, BTE_ERR_ARG, "null e or R");
    if (e_dev == R_dev) FAIL(p, BTE_ERR_ARG, "R must not alias e");
    hipStream_t s = (hipStream_t)stream;
    const Dev &d = p->dev;
    if (p->ctl.precision == BTE_F64) {
        launch_moments<double>(d, (const double *)e_dev, nullptr, p->part, s);
        launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->TL, nullptr, nullptr, s);
        launch_walls<double>(d, (const double *)e_dev, nullptr, p->d_wrec, p->d_wden, p->din, p->nw, s);
        launch_residual<double>(d, (const double *)e_dev, (double *)R_dev, p->TL, p->din, 4, s);
    } else {
        launch_moments<float>(d, (const float *)e_dev, nullptr, p->part, s);
        launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, nullptr, p->TL, nullptr, nullptr, s);
        launch_walls<float>(d, (const float *)e_dev, nullptr, p->d_wrec, p->d_wden, p->din, p->nw, s);
        launch_residual<float>(d, (const float *)e_dev, (float *)R_dev, p->TL, p->din, 4, s);
    }
    HIPCHK(p, hipGetLastError());
    return BTE_OK;
}

bte_status bte_transient_step(bte_problem *p, void *e_dev, int n_steps, double t0, const double *pulse, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) FAIL(p, BTE_ERR_ARG, "e is null");
    if (n_steps < 0) FAIL(p, BTE_ERR_ARG, "n_steps < 0");
    if (pulse && !(pulse[1] > 0)) FAIL(p, BTE_ERR_ARG, "pulse FWHM must be > 0");
    {
        const bte_status cs = check_cfl(p);
        if (cs != BTE_OK) return cs;
    }
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64) return transient_impl<double>(p, (double *)e_dev, n_steps, t0, pulse, s);
    return transient_impl<float>(p, (float *)e_dev, n_steps, t0, pulse, s);
}

bte_status bte_steady_solve(bte_problem *p, void *e_dev, int init, bte_solve_stats *stats, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev) FAIL(p, BTE_ERR_ARG, "e is null");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64) return steady_impl<double>(p, (double *)e_dev, init, stats, s);
    return steady_impl<float>(p, (float *)e_dev, init, stats, s);
}

bte_status bte_keff(bte_problem *p, const void *e_dev, double *keff_dev, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev || !keff_dev) FAIL(p, BTE_ERR_ARG, "null argument");
    for (const Film &fm : p->films)
        if (fm.pdT[0] == 0.0) FAIL(p, BTE_ERR_ARG, "k_eff needs periodic_dT[0] != 0");
    hipStream_t s = (hipStream_t)stream;
    const Dev &d = p->dev;
    if (p->ctl.precision == BTE_F64) launch_moments<double>(d, (const double *)e_dev, nullptr, p->part, s);
    else launch_moments<float>(d, (const float *)e_dev, nullptr, p->part, s);
    // q[nc][3] after the first partial set (part holds >= 2 sets of kMomN per cell)
    double *q = p->part + (size_t)kMomN * p->nc;
    launch_finalize(d, p->part, 1, p->Tref, nullptr, nullptr, q, nullptr, nullptr, nullptr, s);
    launch_keff(d, q, keff_dev, s);
    HIPCHK(p, hipGetLastError());
    return BTE_OK;
}

bte_status bte_adjoint(bte_problem *p, const void *e_dev, int objective, double *dJ_dgamma_dev,
                       bte_solve_stats *stats, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e_dev || !dJ_dgamma_dev) FAIL(p, BTE_ERR_ARG, "null e or gradient");
    if (objective != BTE_OBJ_KEFF_X) FAIL(p, BTE_ERR_ARG, "unknown objective %d", objective);
    if (p->nmat > 1 || p->nifc > 0) FAIL(p, BTE_ERR_UNSUPPORTED, "the adjoint: one material, no interface");
    if (!p->ctl.adjoint) FAIL(p, BTE_ERR_STATE, "control.adjoint was 0 at setup: no adjoint workspace");
    if (p->ctl.limiter != BTE_LIM_NONE) FAIL(p, BTE_ERR_UNSUPPORTED, "the adjoint needs limiter NONE");
    for (const Film &fm : p->films)
        if (fm.pdT[0] == 0.0) FAIL(p, BTE_ERR_ARG, "k_eff needs periodic_dT[0] != 0");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64)
        return adjoint_impl<double>(p, (const double *)e_dev, dJ_dgamma_dev, stats, s);
    return adjoint_impl<float>(p, (const float *)e_dev, dJ_dgamma_dev, stats, s);
}

size_t bte_transient_adjoint_bytes(const bte_problem *p, int n_steps, int every)
{
    if (!p || n_steps < 1 || every < 1) return 0;
    every = std::min(every, n_steps);
    const size_t nseg = (size_t)(n_steps + every - 1) / every;
    return (nseg + (size_t)every - 2) * p->esize() * p->nelem() + (nseg + (size_t)every - 1) * 8 * (size_t)p->nc;
}

int bte_transient_adjoint_interval(const bte_problem *p, int n_steps, size_t max_bytes)
{
    if (!p || n_steps < 1) return 0;
    // the recompute costs n_steps - ceil(n_steps / every) steps: the
    // smallest interval that fits is the fastest (the size is not monotonic
    // in the interval, hence the scan)
    for (int every = 1; every <= n_steps; ++every)
        if (bte_transient_adjoint_bytes(p, n_steps, every) <= max_bytes) return every;
    return 0;
}

bte_status bte_transient_adjoint(bte_problem *p, const void *e0_dev, int n_steps, double t0, const double *pulse,
                                 const double *weights_dev, int every, void *ckpt_dev, size_t ckpt_bytes,
                                 double *J_host, double *dJ_dgamma_dev, bte_solve_stats *stats, void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    if (!e0_dev || !weights_dev || !ckpt_dev || !dJ_dgamma_dev) FAIL(p, BTE_ERR_ARG, "null argument");
    if (n_steps < 1 || every < 1) FAIL(p, BTE_ERR_ARG, "n_steps and every must be >= 1");
    if (p->nmat > 1 || p->nifc > 0) FAIL(p, BTE_ERR_UNSUPPORTED, "the adjoint: one material, no interface");
    if (!p->ctl.adjoint) FAIL(p, BTE_ERR_STATE, "control.adjoint was 0 at setup: no adjoint workspace");
    if (p->ctl.limiter != BTE_LIM_NONE) FAIL(p, BTE_ERR_UNSUPPORTED, "the adjoint needs limiter NONE");
    if (pulse && !(pulse[1] > 0)) FAIL(p, BTE_ERR_ARG, "pulse FWHM must be > 0");
    {
        const bte_status cs = check_cfl(p);
        if (cs != BTE_OK) return cs;
    }
    every = std::min(every, n_steps);
    const size_t need = bte_transient_adjoint_bytes(p, n_steps, every);
    if (ckpt_bytes < need) FAIL(p, BTE_ERR_ARG, "checkpoint buffer too small (%zu < %zu)", ckpt_bytes, need);
    if ((uintptr_t)ckpt_dev & 255) FAIL(p, BTE_ERR_ARG, "checkpoint buffer must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    if (p->ctl.precision == BTE_F64)
        return tadj_impl<double>(p, (const double *)e0_dev, n_steps, t0, pulse, weights_dev, every, (char *)ckpt_dev,
                                 J_host, dJ_dgamma_dev, stats, s);
    return tadj_impl<float>(p, (const float *)e0_dev, n_steps, t0, pulse, weights_dev, every, (char *)ckpt_dev,
                            J_host, dJ_dgamma_dev, stats, s);
}

bte_status bte_get_directions(const bte_problem *p, double *s_host, double *w_host)
{
    if (!p) return BTE_ERR_ARG;
    if (s_host) std::memcpy(s_host, p->s.data(), 8 * p->s.size());
    if (w_host) std::memcpy(w_host, p->w.data(), 8 * p->w.size());
    return BTE_OK;
}

const char *bte_last_error(const bte_problem *p) { return p ? p->err.c_str() : "null handle"; }

bte_status bte_set_graphs(bte_problem *p, int on)
{
    if (!p) return BTE_ERR_ARG;
    p->graphs = on != 0;
    return BTE_OK;
}

bte_status bte_set_persistent(bte_problem *p, int on)
{
    if (!p) return BTE_ERR_ARG;
    if (on && p->dim != 2) FAIL(p, BTE_ERR_UNSUPPORTED, "the one-launch sweep is the 2D register-tile sweep's");
    if (on && !p->queue_ok) FAIL(p, BTE_ERR_STATE, "sweep order: an item precedes one of its upwind items");
    p->persistent = on != 0;
    return BTE_OK;
}

bte_status bte_tile_candidates(const bte_problem *p, int kind, int *tiles, int cap, int *n)
{
    if (!p || !n || (kind != BTE_TUNE_SWEEP && kind != BTE_TUNE_TRANSIENT && kind != BTE_TUNE_SWEEP_ONE_LAUNCH) ||
        cap < 0 || (cap > 0 && !tiles))
        return BTE_ERR_ARG;
    const std::vector<int3> c = tile_candidates(p, kind);
    for (int i = 0; i < (int)c.size() && i < cap; ++i) {
        tiles[3 * i] = c[i].x;
        tiles[3 * i + 1] = c[i].y;
        tiles[3 * i + 2] = c[i].z;
    }
    *n = (int)c.size();
    return BTE_OK;
}

}  // extern "C"

namespace {

// switch one kind to tile shape t (a candidate) and upload the new work lists
bte_status use_tiles(bte_problem *p, int kind, int3 t)
{
    if (kind == BTE_TUNE_SWEEP || kind == BTE_TUNE_SWEEP_ONE_LAUNCH) {
        p->tdim = t;
        p->persistent = kind == BTE_TUNE_SWEEP_ONE_LAUNCH;
    } else {
        p->tdim_tr = t;
    }
    build_schedule(p);
    if (p->items.size() > p->items_cap || p->titems.size() > p->titems_cap)
        FAIL(p, BTE_ERR_STATE, "work list larger than its reserved room");
    if (p->persistent && !p->queue_ok) {
        p->persistent = false;
        FAIL(p, BTE_ERR_STATE, "sweep order: an item precedes one of its upwind items");
    }
    HIPCHK(p, hipMemcpy(p->d_items, p->items.data(), sizeof(SweepItem) * p->items.size(), hipMemcpyHostToDevice));
    HIPCHK(p, hipMemcpy(p->d_titems, p->titems.data(), sizeof(TileItem) * p->titems.size(), hipMemcpyHostToDevice));
    if (!p->items2.empty())
        HIPCHK(p, hipMemcpy(p->d_items2, p->items2.data(), sizeof(Sweep2Item) * p->items2.size(),
                            hipMemcpyHostToDevice));
    return BTE_OK;
}

// one sweep (kind 0) or one explicit step (kind 1) from ein into e2,
// nothing else
template <typename T> hipError_t tune_run(bte_problem *p, int kind, const T *ein, hipStream_t s)
{
    const Dev &d = p->dev;
    T *eout = static_cast<T *>(p->e2);
    if (kind == BTE_TUNE_TRANSIENT)
        return launch_transient_tile<T>(d, ein, eout, p->TL, p->din, p->d_titems, (int)p->titems.size(),
                                        p->tdim_tr, p->na_oct, p->nchunk_oct, p->tile_cap_tr, 0.0, p->ctl.dt,
                                        p->part, s);
    return sweep_launches<T>(p, ein, eout, s);
}

template <typename T>
bte_status autotune_impl(bte_problem *p, const T *ein, int reps, bte_tune_entry *out, int cap, int *n,
                         hipStream_t s)
{
    hipEvent_t ev[2];
    for (auto &x : ev) HIPCHK(p, hipEventCreate(&x));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard()
        {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evg{ev};
    int m = 0;
    // the two sweep kinds are one choice (shape and launch form); the
    // explicit-step shapes another
    struct Best {
        int kind = -1;
        int3 t{};
        double ms = 0.0;
        int entry = -1;
    } best_sweep;
    for (int kind : {BTE_TUNE_SWEEP, BTE_TUNE_SWEEP_ONE_LAUNCH, BTE_TUNE_TRANSIENT}) {
        const std::vector<int3> c = tile_candidates(p, kind);
        const bool sweep = kind != BTE_TUNE_TRANSIENT;
        if (c.empty() || (!sweep && c.size() < 2)) continue;
        // the column walk takes the three-dimensional steps: no shape to time
        if (kind == BTE_TUNE_TRANSIENT && p->dim == 3) continue;
        if (kind == BTE_TUNE_SWEEP && c.size() < 2 && tile_candidates(p, BTE_TUNE_SWEEP_ONE_LAUNCH).empty()) continue;
        std::vector<double> ms(c.size());
        size_t best = 0;
        for (size_t i = 0; i < c.size(); ++i) {
            bte_status st = use_tiles(p, kind, c[i]);
            if (st != BTE_OK) return st;
            HIPCHK(p, tune_run<T>(p, kind, ein, s));
            HIPCHK(p, hipEventRecord(ev[0], s));
            for (int r = 0; r < reps; ++r) HIPCHK(p, tune_run<T>(p, kind, ein, s));
            HIPCHK(p, hipEventRecord(ev[1], s));
            HIPCHK(p, hipEventSynchronize(ev[1]));
            float t = 0;
            HIPCHK(p, hipEventElapsedTime(&t, ev[0], ev[1]));
            ms[i] = t / reps;
            if (ms[i] < ms[best]) best = i;
        }
        for (size_t i = 0; i < c.size(); ++i, ++m)
            if (m < cap) out[m] = bte_tune_entry{kind, {c[i].x, c[i].y, c[i].z}, ms[i], 0};
        const int first = m - (int)c.size();
        if (sweep) {
            if (best_sweep.kind < 0 || ms[best] < best_sweep.ms)
                best_sweep = Best{kind, c[best], ms[best], first + (int)best};
        } else {
            bte_status st = use_tiles(p, kind, c[best]);
            if (st != BTE_OK) return st;
            if (first + (int)best < cap) out[first + best].chosen = 1;
        }
    }
    if (best_sweep.kind >= 0) {
        bte_status st = use_tiles(p, best_sweep.kind, best_sweep.t);
        if (st != BTE_OK) return st;
        if (best_sweep.entry < cap) out[best_sweep.entry].chosen = 1;
    }
    *n = m;
    return BTE_OK;
}

}  // namespace

extern "C" {

bte_status bte_set_tiles(bte_problem *p, int kind, const int *tile)
{
    if (!p) return BTE_ERR_ARG;
    if (!tile || (kind != BTE_TUNE_SWEEP && kind != BTE_TUNE_TRANSIENT && kind != BTE_TUNE_SWEEP_ONE_LAUNCH))
        FAIL(p, BTE_ERR_ARG, "bad tile request");
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    for (const int3 &t : tile_candidates(p, kind))
        if (t.x == tile[0] && t.y == tile[1] && t.z == tile[2]) return use_tiles(p, kind, t);
    FAIL(p, BTE_ERR_ARG, "tile %dx%dx%d is not a candidate", tile[0], tile[1], tile[2]);
}

bte_status bte_autotune(bte_problem *p, void *e_scratch, int reps, bte_tune_entry *entries, int cap, int *n,
                        void *stream)
{
    if (!p) return BTE_ERR_ARG;
    if (!e_scratch || !n || reps < 1 || cap < 0 || (cap > 0 && !entries)) FAIL(p, BTE_ERR_ARG, "bad arguments");
    if (!p->ws) FAIL(p, BTE_ERR_STATE, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    // defined inputs for the timed runs
    HIPCHK(p, hipMemsetAsync(e_scratch, 0, p->esize() * p->nelem(), s));
    HIPCHK(p, hipMemsetAsync(p->TL, 0, 8 * (size_t)p->nc, s));
    HIPCHK(p, hipMemsetAsync(p->dpend, 0, 8 * (size_t)p->nc, s));
    if (p->nw) HIPCHK(p, hipMemsetAsync(p->din, 0, 8 * (size_t)p->nw * p->nl, s));
    if (p->ctl.precision == BTE_F64)
        return autotune_impl<double>(p, static_cast<const double *>(e_scratch), reps, entries, cap, n, s);
    return autotune_impl<float>(p, static_cast<const float *>(e_scratch), reps, entries, cap, n, s);
}

bte_status bte_set_timing(bte_problem *p, int on)
{
    if (!p) return BTE_ERR_ARG;
    p->timing = on != 0;
    return BTE_OK;
}

bte_status bte_last_stats(const bte_problem *p, bte_solve_stats *out)
{
    if (!p || !out) return BTE_ERR_ARG;
    *out = p->last;
    return BTE_OK;
}

void bte_destroy(bte_problem *p) { delete p; }

}  // extern "C"
