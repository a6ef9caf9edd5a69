// bte_internal.h -- device data structures shared by the gfx950 kernels and
// the host runtime of the phonon-BTE library.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>
#include <stddef.h>
#include <stdint.h>

namespace bte {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kMomN = 5;             // moment partials: sum w e, sum w e/tau, q_x, q_y, q_z

// Per-cell geometry code.  For each axis a the byte at bit 8a holds
//   bit0 minus neighbour is a solid cell, bit1 plus neighbour is a solid cell,
//   bit2 minus neighbour reached through a periodic face, bit3 plus ditto,
//   bits4-5 wall kind on the minus side, bits6-7 wall kind on the plus side
//   (bte_bc: 0 thermal, 1 specular, 2 diffuse) when that side is not a cell.
// bit24 solid, bits 25+a: minus-side wall is an outer face (else a pore),
// bits 28+a: plus-side wall is an outer face.
constexpr uint32_t kSolidBit = 1u << 24;

__host__ __device__ inline uint32_t axis_bits(uint32_t code, int a) { return (code >> (8 * a)) & 0xffu; }
__host__ __device__ inline bool side_is_cell(uint32_t ab, int side) { return ab & (side > 0 ? 2u : 1u); }
__host__ __device__ inline bool side_wraps(uint32_t ab, int side) { return ab & (side > 0 ? 8u : 4u); }
__host__ __device__ inline int side_wall(uint32_t ab, int side) { return (ab >> (side > 0 ? 6 : 4)) & 3; }
// Wall kinds in a cell code: 0 thermalizing, 1 specular, 2 diffuse,
// 3 interface (its inflow, like a diffuse wall's, comes from a wall record).
constexpr int kWallInterface = 3;
__host__ __device__ inline bool side_record(uint32_t ab, int side) { return side_wall(ab, side) >= 2; }
__host__ __device__ inline bool side_outer(uint32_t code, int a, int side)
{
    return code & (1u << ((side > 0 ? 28 : 25) + a));
}
__host__ __device__ inline int face_of(int a, int side) { return 2 * a + (side > 0 ? 1 : 0); }

// One geometry of a batch.
struct Film {
    double h[3], ih[3];      // cell size and its inverse per axis
    double pdT[3];           // periodic temperature drop per axis
    double wallT[6];         // thermalizing wall temperature minus T_ref, per face
    double len[3];
    int n[3];
    int cell0, ncell;        // first cell and number of cells in the global numbering
    int nsolid;
    int floating;            // no thermalizing wall: gauge fixed by zero mean T - T_ref
    int periodic[3];         // axis is periodic
    int moff;                // material: its band tables start at C4[moff], v[moff], itau[moff]
    int mat;                 // material index
    double Ctot;             // sum_lambda C of the material
    double Hm[3];            // wall emission conductance 2 sum C v H_a / Omega (correction operator)
    double gif[6];           // interface conductance per face (W m^-2 K^-1; 0: not an interface)
};

// Everything a kernel needs to evaluate the discrete operators.
struct Dev {
    int dim, nc, na, nl, nk, nfilm;
    int jumps;               // 1: some geometry has a periodic axis with a temperature drop
    int limiter;
    double Ctot;             // sum_lambda C of material 0 (single-material paths; Film::Ctot otherwise)
    double omega;            // total angle of the direction set: 4 pi, or 2 pi for a two-dimensional material
    double poreT;            // thermalizing pore wall temperature minus T_ref
    const double *s;         // [na][3]
    const double *w;         // [na]
    const int *mirror;       // [3][na]
    const double *C4;        // [nmat][nl] C/omega (C/(4 pi) for a bulk material)
    const double *v;         // [nmat][nl]
    const double *itau;      // [nmat][nl] 1/tau
    int nmat;                // materials (a geometry's are at Film::moff)
    const double *wbeta;     // [nw][2][nl] interface record: transmittance into its cell, out of it
    const int *wpart;        // [nw] the cell across an interface record's face, -1 for a diffuse wall
    const Film *film;        // [nfilm]
    const uint32_t *code;    // [nc]
    const int *nb;           // [6][nc] neighbour cell per face (or -1)
    const int *fid;          // [nc] geometry index
    const int *dbase;        // [nc] first diffuse-wall record of the cell or -1
    const double *gamma;     // [nc]
    const double *P;         // [nc]
    const double *S;         // [nc] sum_lambda C (1/tau + gamma)
    const void *zrow;        // [8][nk] zeros of the working precision (8 cells): loads of a
                             // missing cell read here instead of branching
    const int *fdone;        // [nfilm] 1: geometry converged, its steady sweep is skipped
};

// One work item of the sweep: a tile of one geometry for 64 lanes of one octant.
struct SweepItem {
    int film, oct, chunk, tile;
};

// Self-contained work item of the two-dimensional sweep: the tile frame and
// the geometry constants it needs, so that a block reaches its stencil
// loads after a single dependent load.
struct Sweep2Item {
    int oct, chunk, film, flags;   // flags: bit0/1 periodic x/y, bit2/3 octant sign of x/y positive
    int o0, o1, e0, e1;            // tile origin and extent (cells) in the geometry
    int n0, n1, cell0;             // geometry size and first cell
    int upx, upy, moff;            // items of the x- / y-upwind tiles in the sweep order (-1: none); material
    double Ctot;                   // sum_lambda C of the geometry's material
    double pdT0, pdT1;             // periodic temperature drops along x, y
    double h0, h1, ih0, ih1;       // cell size and inverse along x, y
    double wallT[4];               // thermalizing wall temperatures minus T_ref, faces -x, +x, -y, +y
};

// One work item of the three-dimensional transient step: one (x, y) column
// of a geometry (col = x + n_x y) for 64 lanes of one octant.
struct ColItem {
    int film, oct, chunk, col;
};

// One work item of the transient step: a tile of one geometry for every lane of one octant.
struct TileItem {
    int film, oct, tile, pad;
};

// Arguments of the conjugate-gradient kernels.
struct CgArgs {
    const double *kax;      // [3][nc] per-axis conductivity
    const double *coef;     // [6][nc] coupling to the neighbour across each face (0: none)
    const double *dg;       // [nc] diagonal (faces plus thermalizing walls)
    int corr;               // 1: correction operator, 0: heat diffusion
    double *x, *p;
    double *rb[2], *wb[2], *sb[2];   // r, w = A r/diag and s = A p by iteration parity
    double *part;           // [2][nblk][3] block partial sums by parity
    double *scal;           // [1] |b|^2, [5] done, [6] iterations, [9] total iterations, [10..13] gamma, alpha by parity
    double rtol2;
};

// Gauss-Legendre nodes / weights on [-1, 1], ascending.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
// Directions and weights on the sphere (two- and three-dimensional
// geometries), weights summing to omega.
void sphere_directions(int n_theta, int n_phi, double omega, std::vector<double> &s, std::vector<double> &w);

}  // namespace bte
