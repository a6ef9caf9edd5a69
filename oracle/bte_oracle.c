/*
 * bte_oracle.c -- plain FP64 CPU oracle for the non-gray phonon BTE hot path
 * (discrete-ordinates transport step, moment reduction, steady source iteration
 * with synthetic correction, explicit transient step, steady/transient adjoint).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code with
 * the HIP path and must never be used as a fallback for it.
 *
 * Everything is written from the paper (Hu et al., "GiftBTE: An efficient
 * deterministic solver for non-gray phonon Boltzmann transport equation"):
 *   - energy-based deviational BTE with RTA closure      Sec. 2.1, eqs. BTE_origin, BTE_get_e0
 *   - boundary conditions (thermalizing, specular,
 *     diffuse, periodic with temperature jump,
 *     interfacial between two materials)                  Sec. 2.2 (i)-(v)
 *   - angular quadrature (computed by the Python side
 *     with numpy's Gauss-Legendre nodes)                  Sec. 3.2, eq. directiondis
 *   - delta-form finite volume discretisation with
 *     first-order implicit / second-order explicit faces  Sec. 3.3, eq. disretized_BTE
 *   - least-squares cell gradient                         Sec. 3.5 (X^{-1} y)
 *   - stiffness matrix / right-hand side of the sweep     Sec. 3.5, eqs. Linear system, B_BTE
 *   - sequential and synthetic iterative schemes          Sec. 3.4, Algorithm 1
 *   - heat-diffusion initial guess                        Sec. 3.5, eq. diff
 *   - explicit forward-Euler transient step               Sec. 4.1, eq. disretized_transientBTE, Algorithm 2
 *   - temperature, lattice temperature and heat flux      eqs. BTE_get_e0, getTQ
 *
 * Readings of silent / garbled passages are those listed in the design notes
 * of this repository (renormalised quadrature, upwind-cell face vector,
 * lagged boundary values, harmonic face conductivity, corrected transient
 * update, consistent correction form of the synthetic scheme, ...).
 *
 * Geometry: structured Cartesian grid (dim 1, 2 or 3), cells indexed
 * c = ix + nx*(iy + ny*iz); an optional solid mask marks pores.
 * Layout of the energy deviation e: e[c][alpha][lambda] (lambda fastest).
 * Temperatures passed in/out as deviations from Tref unless stated.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { BC_THERMAL = 0, BC_SPECULAR = 1, BC_DIFFUSE = 2, BC_PERIODIC = 3, BC_INTERFACE = 4 };
enum { LIM_NONE = 0, LIM_MC = 1, LIM_MINMOD = 2 };

typedef struct {
    int dim;
    int n[3];
    double len[3];
    const uint8_t *solid;   /* [nc] or NULL (all solid) */
    int bc[6];              /* faces -x,+x,-y,+y,-z,+z */
    double bcT[6];          /* absolute wall temperatures (K) */
    double pdT[3];          /* periodic jump per axis: T(low side) - T(high side) */
    int pore_bc;            /* BC applied on solid/pore faces */
    double pore_T;          /* wall temperature if pore_bc is thermalizing */
    int na;
    const double *s;        /* [na][3] unit directions */
    const double *w;        /* [na] angular weights (sum omega) */
    int nl;
    const double *C, *v, *tau;  /* [nmat][nl] band heat capacity, speed, relaxation time */
    double Tref;
    const double *gamma;    /* [nc] extra scattering rate (1/s) or NULL */
    const double *P;        /* [nc] volumetric heat (W/m^3) or NULL */
    int limiter;
    double omega;           /* total angle of the direction set: 4 pi (bulk
                               material, 0 means 4 pi) or 2 pi (two-dimensional
                               material: in-plane directions, Sec. 2.1) */
    int nmat;               /* materials (0 or 1: a single one) */
    const int *mat;         /* [nc] material of each cell, or NULL (all 0) */
    const double *beta;     /* [nmat][nmat][nl]: beta[(a nmat + b) nl + l] is the
                               fraction of band l's energy flux arriving at an
                               interface from material a that crosses into b
                               (Sec. 2.2 (v)); NULL: no transmission */
} orc_case;

/* ------------------------------------------------------------------ basics */

static int nc_of(const orc_case *p) { return p->n[0] * p->n[1] * p->n[2]; }
/* Omega: the angular integral that replaces 4 pi in the equilibrium
 * e0 = C T / Omega (eq. BTE_get_e0 and the remark on two-dimensional
 * materials after it) and everywhere an isotropic value is formed */
static double omega(const orc_case *p) { return p->omega > 0 ? p->omega : 4.0 * M_PI; }
static double hx(const orc_case *p, int a) { return p->len[a] / p->n[a]; }
static int is_solid(const orc_case *p, int c) { return p->solid ? p->solid[c] != 0 : 1; }
static size_t nal(const orc_case *p) { return (size_t)p->na * p->nl; }
static double E(const orc_case *p, const double *e, int c, int al, int l)
{
    return e[((size_t)c * p->na + al) * p->nl + l];
}

/* band properties of the material of cell c */
static int mat_of(const orc_case *p, int c) { return p->mat ? p->mat[c] : 0; }
static double Cc(const orc_case *p, int c, int l) { return p->C[(size_t)mat_of(p, c) * p->nl + l]; }
static double vc(const orc_case *p, int c, int l) { return p->v[(size_t)mat_of(p, c) * p->nl + l]; }

/* effective relaxation time in cell c (Matthiessen rule with the extra rate) */
static double tau_cl(const orc_case *p, int c, int l)
{
    double g = p->gamma ? p->gamma[c] : 0.0;
    return 1.0 / (1.0 / p->tau[(size_t)mat_of(p, c) * p->nl + l] + g);
}

/* sum_lambda C of the material of cell c */
static double Ctot(const orc_case *p, int c)
{
    double s = 0;
    for (int l = 0; l < p->nl; l++) s += Cc(p, c, l);
    return s;
}

/* S_i = sum_lambda C/tau_i,lambda : denominator of the lattice temperature */
static double S_of(const orc_case *p, int c)
{
    double s = 0;
    for (int l = 0; l < p->nl; l++) s += Cc(p, c, l) / tau_cl(p, c, l);
    return s;
}

/* transmittance of band l from the material of cell a into that of cell b */
static double beta_of(const orc_case *p, int a, int b, int l)
{
    if (!p->beta) return 0.0;
    int nm = p->nmat > 0 ? p->nmat : 1;
    return p->beta[((size_t)mat_of(p, a) * nm + mat_of(p, b)) * p->nl + l];
}

typedef struct {
    int is_cell;   /* 1: neighbouring solid cell of the same material; 0: wall */
    int cell;      /* the neighbour (also the cell across an interface) */
    int wrapped;   /* reached through a periodic face */
    int jump;      /* +1/-1: neighbour value gets +/- C*pdT/Omega */
    int bc;        /* wall type */
    double Tw;     /* wall temperature (absolute) */
} nbr_t;

static nbr_t neighbour(const orc_case *p, int c, int a, int side)
{
    int idx[3];
    idx[0] = c % p->n[0];
    idx[1] = (c / p->n[0]) % p->n[1];
    idx[2] = c / (p->n[0] * p->n[1]);
    nbr_t r;
    memset(&r, 0, sizeof r);
    int k = idx[a] + side;
    int f = 2 * a + (side > 0);
    if (k < 0 || k >= p->n[a]) {
        if (p->bc[f] != BC_PERIODIC) {
            r.is_cell = 0; r.bc = p->bc[f]; r.Tw = p->bcT[f];
            return r;
        }
        k = (k + p->n[a]) % p->n[a];
        r.wrapped = 1;
        /* crossing the high face lands on the low side: e(x+L) = e(x) - C dT/Omega */
        r.jump = side > 0 ? -1 : +1;
    }
    idx[a] = k;
    int j = idx[0] + p->n[0] * (idx[1] + p->n[1] * idx[2]);
    if (!is_solid(p, j)) {
        r.is_cell = 0; r.bc = p->pore_bc; r.Tw = p->pore_T; r.wrapped = 0; r.jump = 0;
        return r;
    }
    r.cell = j;
    if (mat_of(p, j) != mat_of(p, c)) {
        /* a face between two materials is an interface (Sec. 2.2 (v)) */
        r.is_cell = 0; r.bc = BC_INTERFACE;
        return r;
    }
    r.is_cell = 1;
    return r;
}

/* value of a neighbour cell as seen from across the face (periodic jump applied) */
static double nval(const orc_case *p, const double *e, nbr_t nb, int a, int al, int l)
{
    return E(p, e, nb.cell, al, l) + nb.jump * Cc(p, nb.cell, l) * p->pdT[a] / omega(p);
}

/* ---------------------------------------------------------- reconstruction */

/* Least-squares gradient component along axis a.  On a Cartesian grid the
 * least-squares normal equations over the face neighbours decouple per axis:
 * central difference with both neighbours, one-sided with one, zero with none.
 * Optional limiters replace it by MC / minmod slopes (zero when a neighbour
 * is missing). */
static double slope(const orc_case *p, const double *e, int c, int a, int al, int l)
{
    double h = hx(p, a);
    nbr_t m = neighbour(p, c, a, -1), q = neighbour(p, c, a, +1);
    double ec = E(p, e, c, al, l);
    double em = m.is_cell ? nval(p, e, m, a, al, l) : 0.0;
    double ep = q.is_cell ? nval(p, e, q, a, al, l) : 0.0;
    if (p->limiter == LIM_NONE) {
        if (m.is_cell && q.is_cell) return (ep - em) / (2.0 * h);
        if (q.is_cell) return (ep - ec) / h;
        if (m.is_cell) return (ec - em) / h;
        return 0.0;
    }
    if (!(m.is_cell && q.is_cell)) return 0.0;
    double dl = (ec - em) / h, dr = (ep - ec) / h;
    if (dl * dr <= 0.0) return 0.0;
    double sg = dl > 0 ? 1.0 : -1.0;
    if (p->limiter == LIM_MC) {
        double t = fmin(2.0 * fabs(dl), 2.0 * fabs(dr));
        return sg * fmin(t, 0.5 * fabs(dl + dr));
    }
    return sg * fmin(fabs(dl), fabs(dr));
}

/* face value on side `side` of cell c along axis a: e_m + grad e_m . l_{m,f}
 * where the face centre lies h/2 away from the cell centre */
static double face_val(const orc_case *p, const double *e, int c, int a, int side, int al, int l)
{
    return E(p, e, c, al, l) + side * 0.5 * hx(p, a) * slope(p, e, c, a, al, l);
}

/* ------------------------------------------------------------------- walls */

typedef struct {
    int *wid;        /* [nc*6] diffuse wall or interface record index or -1 */
    int nw;
    double *din;     /* [nw][nl] incoming diffuse value */
    int *mirror;     /* [3][na] index of the mirror direction w.r.t. axis a */
} walls_t;

static int find_mirror(const orc_case *p, int al, int a)
{
    double t[3] = { p->s[3 * al], p->s[3 * al + 1], p->s[3 * al + 2] };
    t[a] = -t[a];
    int best = -1;
    double bd = 1e300;
    for (int b = 0; b < p->na; b++) {
        double d = fabs(p->s[3 * b] - t[0]) + fabs(p->s[3 * b + 1] - t[1]) + fabs(p->s[3 * b + 2] - t[2]);
        if (d < bd) { bd = d; best = b; }
    }
    return bd < 1e-9 ? best : -1;
}

static int walls_init(const orc_case *p, walls_t *W)
{
    int nc = nc_of(p);
    W->wid = (int *)malloc(sizeof(int) * (size_t)nc * 6);
    W->mirror = (int *)malloc(sizeof(int) * 3 * (size_t)p->na);
    if (!W->wid || !W->mirror) return -1;
    W->nw = 0;
    for (int c = 0; c < nc; c++)
        for (int f = 0; f < 6; f++) {
            W->wid[c * 6 + f] = -1;
            int a = f / 2, side = (f & 1) ? 1 : -1;
            if (a >= p->dim || !is_solid(p, c)) continue;
            nbr_t nb = neighbour(p, c, a, side);
            if (!nb.is_cell && (nb.bc == BC_DIFFUSE || nb.bc == BC_INTERFACE)) W->wid[c * 6 + f] = W->nw++;
        }
    for (int a = 0; a < 3; a++)
        for (int al = 0; al < p->na; al++) {
            W->mirror[a * p->na + al] = a < p->dim ? find_mirror(p, al, a) : al;
            if (a < p->dim && W->mirror[a * p->na + al] < 0) return -2;
        }
    W->din = (double *)calloc((size_t)(W->nw > 0 ? W->nw : 1) * p->nl, sizeof(double));
    return W->din ? 0 : -1;
}

static void walls_free(walls_t *W)
{
    free(W->wid); free(W->din); free(W->mirror);
}

/* Diffuse wall (Sec. 2.2 (iii), eq. diff_bound), discrete normalisation: the
 * incoming value per band equals the outgoing energy flux through the face
 * divided by the quadrature's incoming |s.n| weight, so the net flux is zero.
 *
 * Interface (Sec. 2.2 (v)) between cell c (material A) and cell j across
 * the face (material B): the value entering A is the diffuse part of what
 * comes back, the fraction beta_BA of B's outgoing flux that crosses plus
 * the fraction 1 - beta_AB of A's own outgoing flux that is reflected:
 *   e_in,A = [beta_BA (v_B / v_A) F_B + (1 - beta_AB) F_A] / sum_{s.n<0} w |s.n|
 * with F_X = sum over X's outgoing directions of w |s.n| e_face.  The
 * fractions act on energy fluxes (v e), hence the ratio v_B / v_A (the
 * printed equation omits it; with it the flux leaving A through the face
 * equals the flux entering B for any beta and any state, without it only
 * for equal speeds).  Face values are the second-order outgoing face
 * values of each side, as for the diffuse wall. */
static void walls_update(const orc_case *p, const double *e, walls_t *W)
{
    int nc = nc_of(p);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++)
        for (int f = 0; f < 6; f++) {
            int id = W->wid[c * 6 + f];
            if (id < 0) continue;
            int a = f / 2, side = (f & 1) ? 1 : -1;
            nbr_t nb = neighbour(p, c, a, side);
            for (int l = 0; l < p->nl; l++) {
                double num = 0, den = 0, numb = 0;
                for (int al = 0; al < p->na; al++) {
                    double sn = p->s[3 * al + a] * side;   /* s . n */
                    if (sn > 0) num += p->w[al] * sn * face_val(p, e, c, a, side, al, l);
                    else if (sn < 0) {
                        den += p->w[al] * (-sn);
                        if (nb.bc == BC_INTERFACE)
                            numb += p->w[al] * (-sn) * face_val(p, e, nb.cell, a, -side, al, l);
                    }
                }
                double din = num / den;
                if (nb.bc == BC_INTERFACE) {
                    double bab = beta_of(p, c, nb.cell, l), bba = beta_of(p, nb.cell, c, l);
                    din = (bba * vc(p, nb.cell, l) / vc(p, c, l) * numb + (1.0 - bab) * num) / den;
                }
                W->din[(size_t)id * p->nl + l] = din;
            }
        }
}

/* incoming value at the wall on side `side` of cell c, axis a (s.n < 0) */
static double wall_in(const orc_case *p, const double *e, const walls_t *W, nbr_t nb,
                      int c, int a, int side, int al, int l)
{
    switch (nb.bc) {
    case BC_THERMAL:
        return Cc(p, c, l) * (nb.Tw - p->Tref) / omega(p);
    case BC_SPECULAR:
        /* s' = s - 2(s.n)n : flip the normal component */
        return face_val(p, e, c, a, side, W->mirror[a * p->na + al], l);
    case BC_DIFFUSE:
    case BC_INTERFACE:
        return W->din[(size_t)W->wid[c * 6 + 2 * a + (side > 0)] * p->nl + l];
    default:
        return 0.0;
    }
}

/* value entering cell c through its face on side `side` of axis a */
static double inflow(const orc_case *p, const double *e, const walls_t *W, int c, int a, int side,
                     int al, int l)
{
    nbr_t nb = neighbour(p, c, a, side);
    if (nb.is_cell) {
        double jumpv = nb.jump * Cc(p, nb.cell, l) * p->pdT[a] / omega(p);
        return face_val(p, e, nb.cell, a, -side, al, l) + jumpv;
    }
    return wall_in(p, e, W, nb, c, a, side, al, l);
}

/* (1/V) sum_faces e_f v s.n S  for one (cell, direction, band) */
static double flux_div(const orc_case *p, const double *e, const walls_t *W, int c, int al, int l)
{
    double D = 0.0;
    for (int a = 0; a < p->dim; a++) {
        double sa = p->s[3 * al + a];
        if (sa == 0.0) continue;
        double fp, fm;
        if (sa > 0) {
            fp = face_val(p, e, c, a, +1, al, l);
            fm = inflow(p, e, W, c, a, -1, al, l);
        } else {
            fp = inflow(p, e, W, c, a, +1, al, l);
            fm = face_val(p, e, c, a, -1, al, l);
        }
        D += vc(p, c, l) * sa / hx(p, a) * (fp - fm);
    }
    return D;
}

/* ----------------------------------------------------------------- moments */

/* lattice temperature deviation (eq. BTE_get_e0, discrete form) */
static double TL_cell(const orc_case *p, const double *e, int c)
{
    double num = 0;
    for (int al = 0; al < p->na; al++)
        for (int l = 0; l < p->nl; l++)
            num += p->w[al] * E(p, e, c, al, l) / tau_cl(p, c, l);
    return num / S_of(p, c);
}

/* T (absolute), T_L (absolute), q[3] per cell (eqs. BTE_get_e0, getTQ).
 * Pores get T = T_L = Tref and q = 0. */
int orc_moments(const orc_case *p, const double *e, double *T, double *TL, double *q)
{
    int nc = nc_of(p);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) {
            if (T) T[c] = p->Tref;
            if (TL) TL[c] = p->Tref;
            if (q) q[3 * c] = q[3 * c + 1] = q[3 * c + 2] = 0;
            continue;
        }
        double se = 0, sq[3] = { 0, 0, 0 };
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) {
                double x = p->w[al] * E(p, e, c, al, l);
                se += x;
                for (int a = 0; a < 3; a++) sq[a] += x * vc(p, c, l) * p->s[3 * al + a];
            }
        if (T) T[c] = p->Tref + se / Ctot(p, c);
        if (TL) TL[c] = p->Tref + TL_cell(p, e, c);
        if (q) for (int a = 0; a < 3; a++) q[3 * c + a] = sq[a];
    }
    return 0;
}

/* --------------------------------------------------------------- residual */

static double src_term(const orc_case *p, int c, int l, double scale)
{
    /* heat split over bands by heat capacity and over Omega (total sum_{alpha,lambda} w Q = P) */
    if (!p->P) return 0.0;
    return scale * p->P[c] * Cc(p, c, l) / (omega(p) * Ctot(p, c));
}

/* R = -(1/V) sum_f F - (e - e0)/tau + Q, with e0 = C T_L/Omega.
 * TLdev: per-cell lattice temperature deviation to use in e0 (NULL: from e). */
int orc_residual(const orc_case *p, const double *e, const double *TLdev, double src_scale, double *R)
{
    walls_t W;
    if (walls_init(p, &W)) return -1;
    walls_update(p, e, &W);
    int nc = nc_of(p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; c++) {
        size_t base = (size_t)c * nal(p);
        if (!is_solid(p, c)) { memset(R + base, 0, sizeof(double) * nal(p)); continue; }
        double tl = TLdev ? TLdev[c] : TL_cell(p, e, c);
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) {
                double t = tau_cl(p, c, l);
                double e0 = Cc(p, c, l) * tl / omega(p);
                R[base + (size_t)al * p->nl + l] = -flux_div(p, e, &W, c, al, l)
                    - (E(p, e, c, al, l) - e0) / t + src_term(p, c, l, src_scale);
            }
    }
    walls_free(&W);
    return 0;
}

/* flux divergence only (boundary values taken from e) */
int orc_flux_div(const orc_case *p, const double *e, double *D)
{
    walls_t W;
    if (walls_init(p, &W)) return -1;
    walls_update(p, e, &W);
    int nc = nc_of(p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < nc; c++)
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++)
                D[((size_t)c * p->na + al) * p->nl + l] = is_solid(p, c) ? flux_div(p, e, &W, c, al, l) : 0.0;
    walls_free(&W);
    return 0;
}

/* ------------------------------------------------------------------ sweep */

/* One source-iteration transport solve in delta form (eq. disretized_BTE,
 * stiffness matrix and right-hand side of Sec. 3.5):
 *   A de = b,  b = R(e^n) with e0 from TLdev,
 *   A_ii = 1/tau + sum_out v s.n S/V,  A_ij = -|v s.n| S/V for the upwind
 *   neighbour j across an interior face (boundary and periodic inflow is
 *   lagged, i.e. it enters b only).
 * A is lower-triangular in upwind order, so each (alpha,lambda) system is
 * solved by marching the cells in that order.  e_out = e_in + de.
 * lanes/nlanes select a subset of (alpha*nl + lambda) lanes (NULL: all); the
 * other lanes of e_out are left untouched. */
int orc_sweep(const orc_case *p, const double *e_in, const double *TLdev, double *e_out,
              const int *lanes, int nlanes)
{
    int nc = nc_of(p);
    double *b = (double *)malloc(sizeof(double) * (size_t)nc * nal(p));
    if (!b) return -1;
    if (orc_residual(p, e_in, TLdev, 1.0, b)) { free(b); return -1; }
    int nlane = lanes ? nlanes : (int)nal(p);
#pragma omp parallel
    {
        double *de = (double *)malloc(sizeof(double) * (size_t)nc);
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < nlane; k++) {
            int lane = lanes ? lanes[k] : k;
            int al = lane / p->nl, l = lane % p->nl;
            const double *s = p->s + 3 * al;
            int dir[3];
            for (int a = 0; a < 3; a++) dir[a] = (a < p->dim && s[a] < 0) ? -1 : 1;
            for (int t2 = 0; t2 < p->n[2]; t2++)
                for (int t1 = 0; t1 < p->n[1]; t1++)
                    for (int t0 = 0; t0 < p->n[0]; t0++) {
                        int ix = dir[0] > 0 ? t0 : p->n[0] - 1 - t0;
                        int iy = dir[1] > 0 ? t1 : p->n[1] - 1 - t1;
                        int iz = dir[2] > 0 ? t2 : p->n[2] - 1 - t2;
                        int c = ix + p->n[0] * (iy + p->n[1] * iz);
                        if (!is_solid(p, c)) { de[c] = 0; continue; }
                        double A = 1.0 / tau_cl(p, c, l);
                        double num = b[((size_t)c * p->na + al) * p->nl + l];
                        for (int a = 0; a < p->dim; a++) {
                            if (s[a] == 0.0) continue;
                            double ca = vc(p, c, l) * fabs(s[a]) / hx(p, a);
                            A += ca;
                            nbr_t up = neighbour(p, c, a, s[a] > 0 ? -1 : +1);
                            if (up.is_cell && !up.wrapped) num += ca * de[up.cell];
                        }
                        de[c] = num / A;
                    }
            for (int c = 0; c < nc; c++) {
                size_t ix = ((size_t)c * p->na + al) * p->nl + l;
                e_out[ix] = e_in[ix] + (is_solid(p, c) ? de[c] : 0.0);
            }
        }
        free(de);
    }
    free(b);
    return 0;
}

/* ------------------------------------------------------- diffusion / CG */

static double hemi_flux(const orc_case *p, int a)
{
    double h = 0;
    for (int al = 0; al < p->na; al++) if (p->s[3 * al + a] > 0) h += p->w[al] * p->s[3 * al + a];
    return h;
}

/* sum_lambda C v of the material of cell c */
static double sum_Cv(const orc_case *p, int c)
{
    double g = 0;
    for (int l = 0; l < p->nl; l++) g += Cc(p, c, l) * vc(p, c, l);
    return g;
}

/* Per-axis conductivity.
 * Heat diffusion (corr = 0): k_a,i = sum_lambda C v^2 tau_i,lambda M_aa with
 * M_aa = sum_alpha w s_a^2 / Omega (bulk conductivity of the discrete quadrature).
 * Synthetic correction (corr = 1): the same plus the conduction that the
 * first-order upwind increment of the delta-form sweep gives an isotropic
 * change, sum_lambda C v h_a H_a / Omega with H_a = sum_{s_a > 0} w s_a. */
static double k_axis(const orc_case *p, int c, int a, int corr)
{
    double m = 0;
    for (int al = 0; al < p->na; al++) m += p->w[al] * p->s[3 * al + a] * p->s[3 * al + a];
    m /= omega(p);
    double k = 0;
    for (int l = 0; l < p->nl; l++) k += Cc(p, c, l) * vc(p, c, l) * vc(p, c, l) * tau_cl(p, c, l);
    k *= m;
    if (corr) k += sum_Cv(p, c) * hx(p, a) * hemi_flux(p, a) / omega(p);
    return k;
}

/* Conductance (per unit area) between cell c and a thermalizing wall on axis a:
 * half-cell conduction 2k/h; for the correction in series with the wall's
 * emission conductance 2 sum C v H_a / Omega (first-moment / Marshak closure). */
static double wall_cond(const orc_case *p, int c, int a, int corr)
{
    double kd = 2.0 * k_axis(p, c, a, corr) / hx(p, a);
    if (!corr) return kd;
    double g = 2.0 * sum_Cv(p, c) * hemi_flux(p, a) / omega(p);
    return 1.0 / (1.0 / kd + 1.0 / g);
}

static int has_thermal_wall(const orc_case *p)
{
    for (int f = 0; f < 2 * p->dim; f++)
        if (p->bc[f] == BC_THERMAL) return 1;
    if (p->pore_bc == BC_THERMAL && p->solid) {
        for (int c = 0; c < nc_of(p); c++) if (!p->solid[c]) return 1;
    }
    return 0;
}

/* face conductance between neighbouring cells: harmonic mean */
static double face_k(const orc_case *p, int c, int j, int a, int corr)
{
    double ki = k_axis(p, c, a, corr), kj = k_axis(p, j, a, corr);
    return 2.0 * ki * kj / (ki + kj);
}

/* Conductance per unit area across an interface between cell c and cell j
 * on axis a, for the diffusion operators only (initial guess and
 * correction: they change the path to the fixed point, not the fixed
 * point): the two half cells in series with the interface's own
 * conductance G = (G_AB + G_BA) / 2, G_XY = sum_lambda beta_XY C_X v_X H_a
 * / Omega (the flux crossing per kelvin of difference between the two
 * sides' emitted equilibria).  Returned times h, the form face_k has. */
static double iface_k(const orc_case *p, int c, int j, int a, int corr)
{
    double h = hx(p, a), H = hemi_flux(p, a);
    double gab = 0, gba = 0;
    for (int l = 0; l < p->nl; l++) {
        gab += beta_of(p, c, j, l) * Cc(p, c, l) * vc(p, c, l);
        gba += beta_of(p, j, c, l) * Cc(p, j, l) * vc(p, j, l);
    }
    double G = 0.5 * (gab + gba) * H / omega(p);
    if (!(G > 0)) return 0.0;
    double r = 0.5 * h / k_axis(p, c, a, corr) + 1.0 / G + 0.5 * h / k_axis(p, j, a, corr);
    return h / r;
}

/* y = L x for the finite-volume operator -div(k grad x) per unit volume with
 * harmonic-mean face conductivity; thermalizing walls through wall_cond
 * (homogeneous here), other walls zero flux, periodic faces wrap (jumps enter
 * the right-hand side). */
static void diff_apply(const orc_case *p, int corr, const double *x, double *y)
{
    int nc = nc_of(p);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) { y[c] = 0; continue; }
        double acc = 0;
        for (int a = 0; a < p->dim; a++) {
            double h = hx(p, a);
            for (int side = -1; side <= 1; side += 2) {
                nbr_t nb = neighbour(p, c, a, side);
                if (nb.is_cell) acc += face_k(p, c, nb.cell, a, corr) / (h * h) * (x[c] - x[nb.cell]);
                else if (nb.bc == BC_INTERFACE) acc += iface_k(p, c, nb.cell, a, corr) / (h * h) * (x[c] - x[nb.cell]);
                else if (nb.bc == BC_THERMAL) acc += wall_cond(p, c, a, corr) / h * x[c];
            }
        }
        y[c] = acc;
    }
}

static double diff_diag(const orc_case *p, int corr, int c)
{
    double d = 0;
    for (int a = 0; a < p->dim; a++) {
        double h = hx(p, a);
        for (int side = -1; side <= 1; side += 2) {
            nbr_t nb = neighbour(p, c, a, side);
            if (nb.is_cell) d += face_k(p, c, nb.cell, a, corr) / (h * h);
            else if (nb.bc == BC_INTERFACE) d += iface_k(p, c, nb.cell, a, corr) / (h * h);
            else if (nb.bc == BC_THERMAL) d += wall_cond(p, c, a, corr) / h;
        }
    }
    return d;
}

static void project_mean(const orc_case *p, double *x)
{
    int nc = nc_of(p), ns = 0;
    double m = 0;
    for (int c = 0; c < nc; c++) if (is_solid(p, c)) { m += x[c]; ns++; }
    m /= ns;
    for (int c = 0; c < nc; c++) if (is_solid(p, c)) x[c] -= m;
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned conjugate gradients on L x = rhs (corr selects the
 * correction operator), x0 = 0; stops when ||r||_2 <= rtol ||rhs||_2, after
 * maxit iterations, or on breakdown (p.Ap <= 0: the residual is roundoff).
 * For domains with no thermalizing wall the right-hand side and the result
 * are projected to zero solid mean.  Returns the iteration count. */
static int cg_solve(const orc_case *p, int corr, const double *rhs_in, double *x, double rtol, int maxit)
{
    int nc = nc_of(p);
    int floating = !has_thermal_wall(p);
    double *r = malloc(sizeof(double) * nc), *z = malloc(sizeof(double) * nc),
           *pp = malloc(sizeof(double) * nc), *Ap = malloc(sizeof(double) * nc),
           *dg = malloc(sizeof(double) * nc);
    for (int c = 0; c < nc; c++) {
        r[c] = is_solid(p, c) ? rhs_in[c] : 0.0;
        x[c] = 0;
        dg[c] = is_solid(p, c) ? diff_diag(p, corr, c) : 1.0;
    }
    if (floating) project_mean(p, r);
    double bn = sqrt(dot(nc, r, r));
    int it = 0;
    if (bn > 0) {
        for (int c = 0; c < nc; c++) { z[c] = r[c] / dg[c]; pp[c] = z[c]; }
        double rz = dot(nc, r, z);
        for (it = 1; it <= maxit; it++) {
            diff_apply(p, corr, pp, Ap);
            double pAp = dot(nc, pp, Ap);
            if (!(pAp > 0.0) || !(rz > 0.0)) { it--; break; }
            double alpha = rz / pAp;
            for (int c = 0; c < nc; c++) { x[c] += alpha * pp[c]; r[c] -= alpha * Ap[c]; }
            if (sqrt(dot(nc, r, r)) <= rtol * bn) break;
            for (int c = 0; c < nc; c++) z[c] = r[c] / dg[c];
            double rz2 = dot(nc, r, z);
            double beta = rz2 / rz;
            rz = rz2;
            for (int c = 0; c < nc; c++) pp[c] = z[c] + beta * pp[c];
        }
        if (it > maxit) it = maxit;
    }
    if (floating) project_mean(p, x);
    free(r); free(z); free(pp); free(Ap); free(dg);
    return it;
}

int orc_cg(const orc_case *p, int corr, const double *rhs, double *x, double rtol, int maxit)
{
    return cg_solve(p, corr, rhs, x, rtol, maxit);
}

/* Heat-diffusion initial guess (Sec. 3.5, eq. diff): L T = P with Dirichlet
 * wall temperatures and periodic jumps; returns the temperature deviation. */
int orc_diffusion_T(const orc_case *p, double *Tdev, double rtol, int maxit)
{
    int nc = nc_of(p);
    double *rhs = calloc(nc, sizeof(double));
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) continue;
        double acc = p->P ? p->P[c] : 0.0;
        for (int a = 0; a < p->dim; a++) {
            double h = hx(p, a);
            for (int side = -1; side <= 1; side += 2) {
                nbr_t nb = neighbour(p, c, a, side);
                if (nb.is_cell && nb.jump) {
                    /* flux term kf/h^2 (T_c - (T_j + jump*dT)) moves the jump to the rhs */
                    acc += face_k(p, c, nb.cell, a, 0) / (h * h) * nb.jump * p->pdT[a];
                } else if (!nb.is_cell && nb.bc == BC_THERMAL) {
                    acc += wall_cond(p, c, a, 0) / h * (nb.Tw - p->Tref);
                }
            }
        }
        rhs[c] = acc;
    }
    int it = cg_solve(p, 0, rhs, Tdev, rtol, maxit);
    free(rhs);
    return it;
}

/* ----------------------------------------------------------- steady solve */

typedef struct {
    int iters;
    int cg_iters;
    double eps_T, eps_q;
    int converged;
} orc_stats;

static void eps_of(const orc_case *p, const double *T0, const double *q0, const double *T1,
                   const double *q1, double *eT, double *eq)
{
    int nc = nc_of(p), ns = 0;
    double sT = 0, sq = 0, mT = 0, mq = 0;
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) continue;
        ns++;
        double a0 = sqrt(q0[3 * c] * q0[3 * c] + q0[3 * c + 1] * q0[3 * c + 1] + q0[3 * c + 2] * q0[3 * c + 2]);
        double a1 = sqrt(q1[3 * c] * q1[3 * c] + q1[3 * c + 1] * q1[3 * c + 1] + q1[3 * c + 2] * q1[3 * c + 2]);
        sT += (T0[c] - T1[c]) * (T0[c] - T1[c]);
        sq += (a0 - a1) * (a0 - a1);
        if (fabs(T1[c] - p->Tref) > mT) mT = fabs(T1[c] - p->Tref);
        if (a1 > mq) mq = a1;
    }
    *eT = sqrt(sT / ns) / (mT > 1e-300 ? mT : 1.0);
    *eq = sqrt(sq / ns) / (mq > 1e-300 ? mq : 1.0);
}

/* isotropic equilibrium e = C Tdev/Omega for every direction */
static void set_equilibrium(const orc_case *p, const double *Tdev, double *e)
{
    int nc = nc_of(p);
    for (int c = 0; c < nc; c++)
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++)
                e[((size_t)c * p->na + al) * p->nl + l] = is_solid(p, c) ? Cc(p, c, l) * Tdev[c] / omega(p) : 0.0;
}

/* Steady solve (Algorithm 1).
 *   scheme 0 = sequential: e0 <- C T_L(e^{n+1})/Omega
 *   scheme 1 = synthetic, in correction form:
 *        T_L^{n+1} = T_L^kin(e^{n+1}) + delta,   L_corr delta = P - div q^{n+1},
 *     where the face flux of iterate n+1 is that of the delta-form equation
 *     (second order on e^n, first-order upwind on the increment), so that the
 *     defect equals S_i (T_L^kin(e^{n+1}) - T_L^n) per cell.  The correction
 *     shifts the isotropic part of the distribution too: e^{n+1} += C delta/Omega.
 *     L_corr is the diffusion operator with the sweep's upwind conduction
 *     added to k and a first-moment wall conductance at thermalizing walls;
 *     these only change the path to the fixed point (delta = 0 there), and
 *     without them the correction diverges for optically thick cells and in
 *     ballistic films next to thermalizing walls.
 *   init: 1 = start from the heat-diffusion solution, 0 = start from e.
 * Stops when eps_T <= tol_T and eps_q <= tol_q, or after max_iter sweeps.
 * If the domain has no thermalizing wall the result is shifted by an
 * equilibrium distribution so that the mean local temperature is Tref. */
int orc_steady(const orc_case *p, int scheme, double tol_T, double tol_q, int max_iter,
               double cg_rtol, int cg_maxit, int init, double *e, orc_stats *st)
{
    int nc = nc_of(p);
    size_t N = (size_t)nc * nal(p);
    double *e1 = malloc(sizeof(double) * N);
    double *TL = malloc(sizeof(double) * nc), *TLk = malloc(sizeof(double) * nc);
    double *T0 = malloc(sizeof(double) * nc), *T1 = malloc(sizeof(double) * nc);
    double *q0 = malloc(sizeof(double) * 3 * nc), *q1 = malloc(sizeof(double) * 3 * nc);
    double *r = malloc(sizeof(double) * nc), *dl = malloc(sizeof(double) * nc);
    if (!e1 || !TL || !TLk || !T0 || !T1 || !q0 || !q1 || !r || !dl) return -1;
    memset(st, 0, sizeof *st);
    if (init) {
        orc_diffusion_T(p, T0, 1e-14, 100000);
        set_equilibrium(p, T0, e);
    }
    orc_moments(p, e, T0, TL, q0);
    for (int c = 0; c < nc; c++) TL[c] -= p->Tref;
    int floating = !has_thermal_wall(p);
    for (int it = 1; it <= max_iter; it++) {
        orc_sweep(p, e, TL, e1, NULL, 0);
        orc_moments(p, e1, T1, TLk, q1);
        for (int c = 0; c < nc; c++) TLk[c] -= p->Tref;
        if (scheme == 1) {
            for (int c = 0; c < nc; c++) r[c] = is_solid(p, c) ? S_of(p, c) * (TLk[c] - TL[c]) : 0.0;
            st->cg_iters += cg_solve(p, 1, r, dl, cg_rtol, cg_maxit);
            for (int c = 0; c < nc; c++) TL[c] = TLk[c] + dl[c];
            /* the correction moves the isotropic part of the whole distribution */
            for (int c = 0; c < nc; c++)
                    for (size_t k = 0; k < nal(p); k++)
                        if (is_solid(p, c)) e1[(size_t)c * nal(p) + k] += Cc(p, c, (int)(k % p->nl)) * dl[c] / omega(p);
        } else {
            memcpy(TL, TLk, sizeof(double) * nc);
        }
        eps_of(p, T0, q0, T1, q1, &st->eps_T, &st->eps_q);
        memcpy(e, e1, sizeof(double) * N);
        memcpy(T0, T1, sizeof(double) * nc);
        memcpy(q0, q1, sizeof(double) * 3 * nc);
        st->iters = it;
        if (st->eps_T <= tol_T && st->eps_q <= tol_q) { st->converged = 1; break; }
    }
    if (floating) {
        int ns = 0;
        double m = 0;
        for (int c = 0; c < nc; c++) if (is_solid(p, c)) { m += T0[c] - p->Tref; ns++; }
        m /= ns;
        for (int c = 0; c < nc; c++)
            for (size_t k = 0; k < nal(p); k++)
                if (is_solid(p, c)) e[(size_t)c * nal(p) + k] -= Cc(p, c, (int)(k % p->nl)) * m / omega(p);
    }
    free(e1); free(TL); free(TLk); free(T0); free(T1); free(q0); free(q1); free(r); free(dl);
    return 0;
}

/* k_eff = (L_x / dT) * (1/N_cells) * sum_solid q_x  (pores count as zero flux) */
double orc_keff(const orc_case *p, const double *e)
{
    int nc = nc_of(p);
    double *q = malloc(sizeof(double) * 3 * nc);
    orc_moments(p, e, NULL, NULL, q);
    double s = 0;
    for (int c = 0; c < nc; c++) s += q[3 * c];
    free(q);
    return p->len[0] / p->pdT[0] * s / nc;
}

/* ---------------------------------------------------------- transient step */

static double pulse_factor(const double *pulse, double t)
{
    /* Gaussian in time: pulse = {t_centre, FWHM}; NULL = constant source */
    if (!pulse) return 1.0;
    double d = t - pulse[0];
    return exp(-4.0 * log(2.0) * d * d / (pulse[1] * pulse[1]));
}

/* Explicit forward-Euler step (Sec. 4.1, eq. disretized_transientBTE with the
 * volume and time-step factors placed dimensionally):
 *   e^{n+1} = e^n - dt (1/V) sum_f e_f^n v s.n S + dt [-(e^n - e0^n)/tau + Q(t_n)],
 * with e0^n from the lattice temperature of e^n and boundary values from e^n.
 * Runs n_steps steps starting at time t0 (t_n = t0 + n dt).  If hist is not
 * NULL, hist[k] receives the weighted mean of T(absolute) over cells with
 * weight hw[c] after step k+1. */
int orc_transient(const orc_case *p, double *e, int n_steps, double dt, double t0,
                  const double *pulse, const double *hw, double *hist)
{
    int nc = nc_of(p);
    size_t N = (size_t)nc * nal(p);
    double *R = malloc(sizeof(double) * N);
    double *T = hist ? malloc(sizeof(double) * nc) : NULL;
    if (!R) return -1;
    for (int n = 0; n < n_steps; n++) {
        double t = t0 + n * dt;
        orc_residual(p, e, NULL, pulse_factor(pulse, t), R);
        for (size_t k = 0; k < N; k++) e[k] += dt * R[k];
        if (hist) {
            orc_moments(p, e, T, NULL, NULL);
            double sw = 0, st = 0;
            for (int c = 0; c < nc; c++) { sw += hw[c]; st += hw[c] * T[c]; }
            hist[n] = st / sw;
        }
    }
    free(R); free(T);
    return 0;
}

/* ------------------------------------------------------------------ adjoint
 * Transposed Jacobian of R (limiter NONE, so R is affine in e), built by
 * enumerating each row's linear dependence on e as (column, coefficient)
 * pairs and scattering; the rank-one-per-cell lattice-temperature closure
 * is handled separately.  Only the linear part is transposed: wall
 * temperatures, periodic jumps and the source are constants. */

typedef struct { size_t idx[3]; double cf[3]; int n; } lform;

static size_t IX(const orc_case *p, int c, int al, int l) { return ((size_t)c * p->na + al) * p->nl + l; }

/* linear form of the face value of cell c on side `side` of axis a */
static lform face_form(const orc_case *p, int c, int a, int side, int al, int l)
{
    lform f;
    double h = hx(p, a), half = side * 0.5 * h;
    nbr_t m = neighbour(p, c, a, -1), q = neighbour(p, c, a, +1);
    f.n = 1; f.idx[0] = IX(p, c, al, l); f.cf[0] = 1.0;
    if (m.is_cell && q.is_cell) {
        f.idx[1] = IX(p, q.cell, al, l); f.cf[1] = half / (2 * h);
        f.idx[2] = IX(p, m.cell, al, l); f.cf[2] = -half / (2 * h);
        f.n = 3;
    } else if (q.is_cell) {
        f.idx[1] = IX(p, q.cell, al, l); f.cf[1] = half / h;
        f.cf[0] -= half / h; f.n = 2;
    } else if (m.is_cell) {
        f.idx[1] = IX(p, m.cell, al, l); f.cf[1] = -half / h;
        f.cf[0] += half / h; f.n = 2;
    }
    return f;
}

static void scatter_form(double *y, lform f, double x)
{
    for (int k = 0; k < f.n; k++) {
        double *dst = y + f.idx[k];
#pragma omp atomic
        *dst += f.cf[k] * x;
    }
}

/* y = (dR/de)^T x */
int orc_apply_jac_T(const orc_case *p, const double *x, double *y)
{
    if (p->limiter != LIM_NONE) return -3;
    if (p->nmat > 1) return -4;   /* the adjoint covers one material */
    int nc = nc_of(p);
    size_t N = (size_t)nc * nal(p);
    walls_t W;
    if (walls_init(p, &W)) return -1;
    memset(y, 0, sizeof(double) * N);
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) continue;
        double Sc = S_of(p, c);
        /* closure: row (c,al,l) has + C_l/(Omega tau_cl) * T_L, T_L = sum w e/tau / S */
        double acc = 0;
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++)
                acc += x[IX(p, c, al, l)] * p->C[l] / (omega(p) * tau_cl(p, c, l));
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) {
                double v = acc * p->w[al] / tau_cl(p, c, l) / Sc - x[IX(p, c, al, l)] / tau_cl(p, c, l);
#pragma omp atomic
                y[IX(p, c, al, l)] += v;
            }
        /* streaming: row gets -v s_a/h (F+ - F-) */
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) {
                double xr = x[IX(p, c, al, l)];
                if (xr == 0.0) continue;
                for (int a = 0; a < p->dim; a++) {
                    double sa = p->s[3 * al + a];
                    if (sa == 0.0) continue;
                    double k = -p->v[l] * sa / hx(p, a) * xr;
                    for (int side = -1; side <= 1; side += 2) {
                        double sgn = side > 0 ? k : -k;   /* +F+ , -F- */
                        if (sa * side > 0) { scatter_form(y, face_form(p, c, a, side, al, l), sgn); continue; }
                        nbr_t nb = neighbour(p, c, a, side);
                        if (nb.is_cell) { scatter_form(y, face_form(p, nb.cell, a, -side, al, l), sgn); continue; }
                        if (nb.bc == BC_SPECULAR) {
                            scatter_form(y, face_form(p, c, a, side, W.mirror[a * p->na + al], l), sgn);
                        } else if (nb.bc == BC_DIFFUSE) {
                            double den = 0;
                            for (int b = 0; b < p->na; b++) {
                                double sn = p->s[3 * b + a] * side;
                                if (sn < 0) den += p->w[b] * (-sn);
                            }
                            for (int b = 0; b < p->na; b++) {
                                double sn = p->s[3 * b + a] * side;
                                if (sn > 0) scatter_form(y, face_form(p, c, a, side, b, l), sgn * p->w[b] * sn / den);
                            }
                        }
                    }
                }
            }
    }
    walls_free(&W);
    return 0;
}

/* dR_{c,al,l}/dgamma_c, contracted with psi:  out[c] = sum_{al,l} psi dR/dgamma_c
 *   dR/dgamma_c = -(e - e0) + C/(Omega tau) dT_L/dgamma_c,
 *   dT_L/dgamma_c = Ctot (T_c - T_L,c)/S_c  (both as deviations). */
int orc_dR_dgamma(const orc_case *p, const double *e, const double *psi, double *out)
{
    if (p->nmat > 1) return -4;   /* the adjoint covers one material */
    int nc = nc_of(p);
    double ct = Ctot(p, 0);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; c++) {
        if (!is_solid(p, c)) { out[c] = 0; continue; }
        double se = 0;
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) se += p->w[al] * E(p, e, c, al, l);
        double Tdev = se / ct, tl = TL_cell(p, e, c), Sc = S_of(p, c);
        double dTL = ct * (Tdev - tl) / Sc;
        double acc = 0;
        for (int al = 0; al < p->na; al++)
            for (int l = 0; l < p->nl; l++) {
                double t = tau_cl(p, c, l);
                double d = -(E(p, e, c, al, l) - p->C[l] * tl / omega(p)) + p->C[l] / (omega(p) * t) * dTL;
                acc += psi[IX(p, c, al, l)] * d;
            }
        out[c] = acc;
    }
    return 0;
}

/* transposed first-order sweep operator: solves A^T z = rhs (A as in orc_sweep),
 * marching each lane against the upwind order; used as the preconditioner of
 * the oracle's adjoint Krylov solve */
int orc_sweep_T(const orc_case *p, const double *rhs, double *z)
{
    if (p->nmat > 1) return -4;   /* the adjoint covers one material */
    int nc = nc_of(p);
    int nlane = (int)nal(p);
#pragma omp parallel
    {
        double *zz = (double *)malloc(sizeof(double) * (size_t)nc);
#pragma omp for schedule(dynamic, 1)
        for (int lane = 0; lane < nlane; lane++) {
            int al = lane / p->nl, l = lane % p->nl;
            const double *s = p->s + 3 * al;
            int dir[3];
            for (int a = 0; a < 3; a++) dir[a] = (a < p->dim && s[a] < 0) ? -1 : 1;
            for (int t2 = p->n[2] - 1; t2 >= 0; t2--)
                for (int t1 = p->n[1] - 1; t1 >= 0; t1--)
                    for (int t0 = p->n[0] - 1; t0 >= 0; t0--) {
                        int ix = dir[0] > 0 ? t0 : p->n[0] - 1 - t0;
                        int iy = dir[1] > 0 ? t1 : p->n[1] - 1 - t1;
                        int iz = dir[2] > 0 ? t2 : p->n[2] - 1 - t2;
                        int c = ix + p->n[0] * (iy + p->n[1] * iz);
                        if (!is_solid(p, c)) { zz[c] = 0; continue; }
                        double A = 1.0 / tau_cl(p, c, l);
                        double num = rhs[IX(p, c, al, l)];
                        for (int a = 0; a < p->dim; a++) {
                            if (s[a] == 0.0) continue;
                            double ca = p->v[l] * fabs(s[a]) / hx(p, a);
                            A += ca;
                            /* cells whose upwind neighbour is c: the downwind neighbour */
                            nbr_t dn = neighbour(p, c, a, s[a] > 0 ? +1 : -1);
                            if (dn.is_cell && !dn.wrapped) num += ca * zz[dn.cell];
                        }
                        zz[c] = num / A;
                    }
            for (int c = 0; c < nc; c++) z[IX(p, c, al, l)] = zz[c];
        }
        free(zz);
    }
    return 0;
}
