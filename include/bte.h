/*
 * bte.h -- C ABI of the MI355X (gfx950) phonon-BTE hot-path library.
 *
 * The library solves the energy-based, deviational phonon Boltzmann
 * transport equation in the relaxation-time approximation (Hu et al.,
 * GiftBTE, Sec. 2.1, eqs. BTE_origin / BTE_get_e0) with the discrete-
 * ordinates method on structured Cartesian grids:
 *   - steady state: implicit source iteration in delta form with a
 *     second-order upwind finite-volume flux (Sec. 3.3, eq. disretized_BTE;
 *     Sec. 3.5, stiffness matrix / right-hand side eq. B_BTE), sequential or
 *     synthetic scheme (Sec. 3.4, Algorithm 1);
 *   - transient: explicit forward-Euler step (Sec. 4.1,
 *     eq. disretized_transientBTE, Algorithm 2);
 *   - moments: temperature, lattice temperature, heat flux (eqs. BTE_get_e0,
 *     getTQ);
 *   - adjoint: gradient of the effective conductivity with respect to a
 *     per-cell extra scattering rate.
 *
 * Conventions shared by every call
 *   - Every call returns a bte_status and never throws or aborts.  On a
 *     validation error nothing is written to any output.  bte_last_error()
 *     returns a text description of the last failure on a handle.
 *   - Device pointers are HIP device addresses (e.g. the data pointer of a
 *     torch tensor on cuda:0); host pointers are ordinary CPU memory.  The
 *     caller owns every buffer; the library allocates no device memory: its
 *     scratch lives in a caller-provided workspace (bte_workspace_bytes /
 *     bte_bind).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     All device work of a call is enqueued on that stream.
 *   - A handle may be used by one host thread and one stream at a time.
 *
 * Layout of the energy deviation e (J m^-3 sr^-1 relative to the
 * equilibrium at T_ref):  e[cell][alpha][lambda], lambda fastest, cells
 * c = ix + nx*(iy + ny*iz), element type float (BTE_F32) or double
 * (BTE_F64).  For a batch of geometries the per-geometry arrays are
 * concatenated in batch order.  Directions alpha are ordered octant-major
 * (octant bits 1: s_x<0, 2: s_y<0, 4: s_z<0), then polar index (ascending
 * theta), then azimuthal index (ascending phi); in one dimension there are
 * two hemispheres (s_x>0 first), polar axis x.  bte_get_directions()
 * returns the table.
 */
#ifndef BTE_H
#define BTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BTE_OK = 0,
    BTE_ERR_ARG = 1,            /* invalid argument (nothing written)              */
    BTE_ERR_UNSUPPORTED = 2,    /* valid but not supported combination             */
    BTE_ERR_HIP = 3,            /* HIP runtime error                               */
    BTE_ERR_NOT_CONVERGED = 4,  /* max_iter reached; last iterate and stats written */
    BTE_ERR_NONFINITE = 5,      /* NaN/Inf detected in the iteration               */
    BTE_ERR_CFL = 6,            /* time step violates the explicit stability bound  */
    BTE_ERR_STATE = 7           /* call order (e.g. no workspace bound)            */
} bte_status;

typedef enum { BTE_F32 = 0, BTE_F64 = 1 } bte_precision;          /* storage of e      */
typedef enum { BTE_BC_THERMAL = 0, BTE_BC_SPECULAR = 1,
               BTE_BC_DIFFUSE = 2, BTE_BC_PERIODIC = 3,
               BTE_BC_INTERFACE = 4 } bte_bc;                     /* Sec. 2.2 (i)-(v)  */
typedef enum { BTE_SEQUENTIAL = 0, BTE_SYNTHETIC = 1 } bte_scheme; /* Sec. 3.4          */
typedef enum { BTE_LIM_NONE = 0, BTE_LIM_MC = 1, BTE_LIM_MINMOD = 2 } bte_limiter;
typedef enum { BTE_OBJ_KEFF_X = 0 } bte_objective;

/* Geometry (the GEOMETRY input of Sec. 5: dimension, scales, boundary
 * conditions).  Faces are ordered -x,+x,-y,+y,-z,+z; faces of axes beyond
 * `dim` are ignored.  Periodic faces come in pairs.  periodic_dT[a] is the
 * temperature drop imposed across a periodic axis (Sec. 2.2 (iv)): incoming
 * values on the low face get +C dT/4pi, on the high face -C dT/4pi (2 pi in
 * place of 4 pi for a two-dimensional material, see bte_material).
 * Faces between solid cells and pores (solid[c] == 0) use pore_bc. */
typedef struct {
    int dim;                 /* 1, 2 or 3                                  */
    int n[3];                /* cells per axis (unused axes: 1)            */
    double len[3];           /* domain length per axis (m)                 */
    const uint8_t *solid;    /* host, n0*n1*n2 bytes, NULL = all solid      */
    int bc[6];               /* bte_bc per face                            */
    double bc_T[6];          /* wall temperature of thermalizing faces (K) */
    double periodic_dT[3];   /* K                                          */
    int pore_bc;             /* BTE_BC_DIFFUSE or BTE_BC_SPECULAR          */
} bte_geometry;

/* Phonon bands (PHONON input: BandNumber, Ntheta, Nphi, MaterialDimension;
 * Sec. 3.1-3.2, Sec. 5).  material_dim 0 or 3: bulk material, directions on
 * the sphere, total angle 4 pi.  material_dim 2: two-dimensional material
 * (Sec. 2.1, the remark after eq. BTE_get_e0: the solid angle becomes the
 * in-plane polar angle): n_theta Gauss-Legendre directions per quadrant in
 * the x-y plane (n_phi ignored), total angle 2 pi, e0 = C T_L / 2 pi and
 * 2 pi in place of 4 pi in every isotropic value (wall emission, source
 * split, periodic jump); accepted for 1D and 2D geometries only
 * (BTE_ERR_ARG for 3D). */
typedef struct {
    int n_bands;
    const double *C;         /* host [n_bands] heat capacity, J m^-3 K^-1 */
    const double *v;         /* host [n_bands] group speed, m/s           */
    const double *tau;       /* host [n_bands] relaxation time, s         */
    int n_theta, n_phi;      /* Gauss-Legendre nodes per octant (1D: per hemisphere, n_phi ignored) */
    double T_ref;            /* reference temperature, K                  */
    int material_dim;        /* 0 or 3: bulk; 2: two-dimensional material */
} bte_material;

/* Control (CONTROL input, Sec. 5: IterativeScheme, MaxNumIter,
 * ResidualTemp, ResidualFlux, TimeStep) */
typedef struct {
    int precision;           /* bte_precision                               */
    int scheme;              /* bte_scheme                                  */
    int limiter;             /* bte_limiter                                 */
    double residual_temp;    /* stop when eps_T <= residual_temp ...       */
    double residual_flux;    /* ... and eps_q <= residual_flux             */
    int max_iter;            /* source iterations (<= 0: 10000)            */
    double cg_rtol;          /* relative residual of the CG solves          */
    int cg_max_iter;         /* CG iteration cap per solve (<= 0: 2000)     */
    double dt;               /* transient time step, s (0: steady only)     */
    int adjoint;             /* != 0: reserve workspace for bte_adjoint (two
                                more buffers the size of e); fixed at setup */
} bte_control;

typedef struct {
    int iters;               /* source iterations performed                */
    int cg_iters;            /* total CG iterations                        */
    double eps_T, eps_q;     /* last convergence measures                  */
    int converged;
    double ms_total;         /* wall time of the call (host clock)         */
    double ms_sweep;         /* device time of the transport sweeps (HIP events on the stream) */
    double ms_walls;         /* device time of the wall-inflow kernels     */
    double ms_post;          /* device time of moments/defect/eps kernels  */
    double ms_cg;            /* device time of the synthetic correction    */
    int sweep_launches;      /* kernel launches issued for the sweeps      */
    double updates;          /* (cell, direction, band) updates performed by the
                                sweeps or steps: converged geometries of a
                                batch are no longer swept                   */
} bte_solve_stats;

typedef struct bte_problem bte_problem;

/* Build a problem for n_geo geometries of identical dimension sharing one
 * material and control (n_geo > 1: a batch of independent films, solved
 * together).  Follows the inputs of Sec. 5 (CONTROL, GEOMETRY, PHONON) and
 * the precomputation of Algorithm 1 (Sec. 3.5): the band table (Sec. 3.1),
 * the direction set and weights of eq. directiondis (Sec. 3.2), per-cell
 * relaxation times and boundary tables (Sec. 2.2).  All inputs are host
 * memory and are copied.  Errors: BTE_ERR_ARG for an invalid dimension,
 * cell count, length, boundary code, unpaired periodic face, band table or
 * quadrature size (*out is still set so bte_last_error can report; destroy
 * it); nothing is allocated on the device.  On success *out receives the
 * handle; bind a workspace before any device call. */
bte_status bte_setup(const bte_geometry *geo, int n_geo, const bte_material *mat,
                     const bte_control *ctl, bte_problem **out);

/* An interface between two geometries of different materials (Sec. 2.2 (v)
 * and the Ge-Si verification case of Sec. 3.6): face face_a of geometry
 * geo_a (0..5: -x, +x, -y, +y, -z, +z) touches face face_b of geometry geo_b,
 * the opposite face of the same axis; both faces are set to
 * BTE_BC_INTERFACE in their geometries and hold the same cells along the
 * other axes (same n and len there) with the same cell size along the
 * axis too.  Cell i of one face touches cell i of the other (the other
 * axes' indices equal).  beta_ab[l] is the fraction of band l's energy flux
 * arriving at the interface from geo_a that crosses into geo_b, beta_ba[l]
 * the reverse (host arrays of n_bands values in [0, 1], copied).  The
 * value entering each side is diffuse: the crossing fraction of the other
 * side's outgoing flux plus the reflected fraction (1 - beta) of its own,
 * over the quadrature's incoming weight (the diffuse wall's normalisation),
 * the fractions applied to energy fluxes (v e): energy is conserved across
 * the face for any beta.  A solid cell facing a pore across the interface
 * sees its own geometry's pore_bc. */
typedef struct {
    int geo_a, face_a;
    int geo_b, face_b;
    const double *beta_ab;   /* host [n_bands] */
    const double *beta_ba;   /* host [n_bands] */
} bte_interface;

/* bte_setup with several materials: geometry g is made of material
 * mats[geo_mat[g]] (geo_mat NULL: all of mats[0]); n_ifc interfaces join
 * geometries of different (or equal) materials.  The materials share
 * n_bands, n_theta, n_phi, T_ref and material_dim (band l of one is
 * matched with band l of the other across an interface); their C, v and
 * tau differ.  Every geometry joined by an interface needs a thermalizing
 * wall (BTE_ERR_UNSUPPORTED otherwise).  The synthetic correction and the
 * initial guess couple the geometries across the interfaces through the
 * half cells in series with the interface conductance
 * sum_l beta C v H / Omega, averaged over the two directions.
 * Supported on such a problem: steady solves (both schemes, every
 * limiter, both 2D launch forms), transient steps, bte_moments,
 * bte_residual and bte_keff, in 1D, 2D and 3D; BTE_ERR_UNSUPPORTED for the
 * two adjoints.  BTE_ERR_ARG for an invalid interface (face not set to
 * BTE_BC_INTERFACE or used twice, faces that do not match, beta outside
 * [0, 1]), a BTE_BC_INTERFACE face without an interface, or materials that
 * differ in what they must share; otherwise as bte_setup.  bte_setup(geo,
 * n, mat, ctl, out) is bte_setup_multi(geo, n, mat, 1, NULL, NULL, 0, ctl,
 * out). */
bte_status bte_setup_multi(const bte_geometry *geo, int n_geo, const bte_material *mats, int n_mat,
                           const int *geo_mat, const bte_interface *ifc, int n_ifc,
                           const bte_control *ctl, bte_problem **out);

/* Replace the control of a handle (scheme, limiter, tolerances, iteration
 * caps, dt).  The precision must stay the same (it fixes the workspace). */
bte_status bte_set_control(bte_problem *p, const bte_control *ctl);

/* Size in bytes of the device workspace the handle needs. */
size_t bte_workspace_bytes(const bte_problem *p);

/* Number of elements of e (all geometries), cells, directions and bands. */
size_t bte_num_unknowns(const bte_problem *p);
int bte_num_cells(const bte_problem *p);
int bte_num_directions(const bte_problem *p);

/* Attach a device workspace (>= bte_workspace_bytes, 256-byte aligned) and
 * upload the tables; synchronous.  The workspace must stay alive and
 * untouched by the caller while the handle is used. */
bte_status bte_bind(bte_problem *p, void *workspace_dev, size_t bytes);

/* Per-cell fields (device, double, all cells of all geometries; NULL = 0):
 * P = volumetric heat generation sum_lambda Q (W/m^3), split over bands by
 * C_lambda/C_tot and over solid angle (Sec. 2.1 source term); gamma = extra
 * scattering rate (1/s) added to every band, 1/tau_i = 1/tau + gamma_i. */
bte_status bte_set_fields(bte_problem *p, const double *P_dev, const double *gamma_dev, void *stream);

/* Moments of e (eqs. BTE_get_e0, getTQ): T and T_L in K (pores: T_ref),
 * q[cell][3] in W/m^2.  Any output may be NULL.  Asynchronous. */
bte_status bte_moments(bte_problem *p, const void *e_dev, double *T_dev, double *TL_dev,
                       double *q_dev, void *stream);

/* No-allocation moments, for callers that cannot allocate device memory or
 * grow a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, outputs and
 * asynchrony as bte_moments; the FP64 moment partials (5 doubles per cell)
 * live in a static device array of BTE_STATIC_MAX_CELLS * 40 bytes (32 MiB)
 * that the library holds on every GPU it runs on until the process ends,
 * and the call allocates nothing.  Errors: BTE_ERR_ARG if the problem has
 * more than BTE_STATIC_MAX_CELLS cells (nothing written), BTE_ERR_STATE
 * without a bound workspace (the problem's tables live there).  Every call
 * on a GPU shares that GPU's array, which keeps the last call's contents;
 * every partial a call reads it writes first, so nothing needs clearing, but
 * calls that overlap on one GPU (other streams or host threads) race. */
#define BTE_STATIC_MAX_CELLS 838860
bte_status bte_moments_static(bte_problem *p, const void *e_dev, double *T_dev, double *TL_dev,
                              double *q_dev, void *stream);

/* Steady residual R(e) = -(1/V) sum_f e_f v s.n S - (e - C T_L/4pi)/tau + Q
 * (right-hand side of eq. B_BTE with T_L from e), same layout/precision
 * as e.  Asynchronous. */
bte_status bte_residual(bte_problem *p, const void *e_dev, void *R_dev, void *stream);

/* n_steps explicit steps (Sec. 4.1) of size ctl.dt, in place on e, starting
 * at time t0.  pulse (host, may be NULL) = {t_centre, FWHM}: the source P is
 * multiplied by exp(-4 ln2 (t - t_centre)^2 / FWHM^2) at t_n = t0 + n dt.
 * Returns BTE_ERR_CFL if dt * (1/tau_min + sum_a v_max/h_a) >= 1.
 * Asynchronous. */
bte_status bte_transient_step(bte_problem *p, void *e_dev, int n_steps, double t0,
                              const double *pulse, void *stream);

/* Steady solve (Algorithm 1), in place on e.  init != 0 starts from the
 * heat-diffusion solution (Sec. 3.5, eq. diff), else from e.  Synchronous
 * (reads one convergence flag per iteration).  Returns BTE_ERR_NOT_CONVERGED
 * with the last iterate if max_iter is reached.  stats may be NULL. */
bte_status bte_steady_solve(bte_problem *p, void *e_dev, int init, bte_solve_stats *stats,
                            void *stream);

/* Effective conductivity along x (W/m/K) of each geometry from e: the
 * conductivity kappa = q_x L / (T_1 - T_2) of the verification cases
 * (Sec. 3.6) with the mean flux of a porous film (Sec. 6.1):
 * k = (L_x / dT_x) * (1/N_cells) * sum_solid q_x (pores count as zero),
 * q from eq. getTQ.  keff_dev: device double[n_geo], written
 * asynchronously on `stream`.  BTE_ERR_ARG if periodic_dT[0] == 0 for a
 * geometry (nothing written). */
bte_status bte_keff(bte_problem *p, const void *e_dev, double *keff_dev, void *stream);

/* Adjoint of the steady problem for J = k_eff (objective BTE_OBJ_KEFF_X,
 * the functional of bte_keff, summed over the geometries of a batch):
 * solves (dR/de)^T psi = -dJ/de, where R is the steady residual of
 * bte_residual (Sec. 3.3 / 3.5 with the closures of Sec. 2.2), by the
 * transpose of the forward iteration: sweeps in the reversed direction of
 * every lane with the transposed boundary and scattering closures and, for
 * the synthetic scheme, the same CG correction.  Writes dJ/dgamma per cell
 * (device double[n_cells], pores 0) for the extra scattering rate of
 * bte_set_fields.  e must be a converged steady solution for the current
 * fields.  Requires control.adjoint != 0 at setup, limiter NONE and
 * periodic_dT[0] != 0.  Stops when |J^T psi + g| <= residual_temp |g| for
 * every geometry (2-norms over all unknowns) or after max_iter sweeps
 * (BTE_ERR_NOT_CONVERGED, gradient of the last iterate written).
 * stats: iters = sweeps, eps_T = final relative residual.  Synchronous. */
bte_status bte_adjoint(bte_problem *p, const void *e_dev, int objective, double *dJ_dgamma_dev,
                       bte_solve_stats *stats, void *stream);

/* Transient adjoint (reverse mode of n_steps explicit steps, Sec. 4.1,
 * Algorithm 2) for J = sum_c a_c T_c(e^N) / sum_c a_c, the weighted mean
 * local temperature after the last step.  e0_dev: start state (not
 * modified; read again by the backward pass); weights_dev: device
 * double[n_cells] a_c >= 0 with a positive sum; pulse as in
 * bte_transient_step.  The forward pass writes e every `every` steps into
 * ckpt_dev (device memory of at least bte_transient_adjoint_bytes(p,
 * n_steps, every) bytes, 256-byte aligned, owned by the caller and
 * overwritten); the backward pass recomputes one segment of `every` states
 * at a time and runs the transposed steps with the gradient accumulated on
 * the fly.  Writes J (host, may be NULL) and dJ/dgamma per cell (device
 * double[n_cells]).  stats: iters = n_steps, updates = forward, recomputed
 * and transposed steps times the unknowns, ms_sweep = device time of the
 * forward pass (with J), ms_post = device time of the backward pass.
 * Requires control.adjoint != 0 at setup, limiter NONE and a stable dt
 * (BTE_ERR_CFL).  Synchronous. */
bte_status bte_transient_adjoint(bte_problem *p, const void *e0_dev, int n_steps, double t0,
                                 const double *pulse, const double *weights_dev, int every,
                                 void *ckpt_dev, size_t ckpt_bytes, double *J_host,
                                 double *dJ_dgamma_dev, bte_solve_stats *stats, void *stream);

/* Bytes of the checkpoint buffer of bte_transient_adjoint, with
 * m = ceil(n_steps / every) (every clamped to n_steps):
 * (m + every - 2) states of e (checkpoints 1 .. m - 1, the recomputed
 * states of one segment) plus (m + every - 1) doubles per cell (T_L of the
 * checkpoints and of the recomputed states); 0 on invalid arguments. */
size_t bte_transient_adjoint_bytes(const bte_problem *p, int n_steps, int every);

/* The smallest checkpoint interval whose buffer fits in max_bytes (0 if
 * none, or on invalid arguments).  The backward pass recomputes
 * n_steps - ceil(n_steps / every) forward steps, so the smallest interval
 * that fits is the fastest: with the state in HBM-sized buffers, every = 1
 * (nothing recomputed) needs n_steps - 1 states, every = 2 about half. */
int bte_transient_adjoint_interval(const bte_problem *p, int n_steps, size_t max_bytes);

/* Device timers of bte_transient_step (off by default).  With on != 0 every
 * step records HIP events around its wall, transport and T_L kernels, and
 * the call waits for its own work to finish before it returns, so that the
 * times can be read; the call is then synchronous. */
bte_status bte_set_timing(bte_problem *p, int on);

/* HIP graphs in bte_steady_solve (on by default).  With on != 0 the
 * tile-diagonal launches of one sweep (one graph per buffer parity) and, when
 * control.cg_max_iter <= 64, the launches of one synthetic-correction CG solve
 * are captured once per solve call and replayed every source iteration; the
 * results are the same as with plain launches. */
bte_status bte_set_graphs(bte_problem *p, int on);

/* Launch form of the two-dimensional steady sweep (the transport sweep of
 * Algorithm 1, Sec. 3.3-3.5) with the register-tile kernel (8 x 8 tiles).
 * on == 0: one launch per tile diagonal (the default).  on != 0: one launch
 * per sweep; each block takes a ticket (the work items in sweep order),
 * does everything that reads only the previous iterate, then waits for the
 * items of its x- and y-upwind tiles and reads their new values.  The
 * results are bitwise those of the launch-per-diagonal form.  Every wait is
 * bounded: a wait that gives up (about a second) sets an abort word, the
 * launch ends, and bte_steady_solve returns BTE_ERR_HIP.  Errors:
 * BTE_ERR_UNSUPPORTED for a one- or three-dimensional problem (on != 0);
 * the LDS-tile shapes of a 2D problem keep one launch per diagonal. */
bte_status bte_set_persistent(bte_problem *p, int on);

/* Tile shapes (work decomposition) of the kernels.  The paper's solver runs
 * on CPUs (Sec. 3.5: MPI ranks over directions, then bands) and has no
 * counterpart; these calls only choose how the same arithmetic is blocked on
 * the GPU:
 *   BTE_TUNE_SWEEP     steady sweeps, one launch per tile diagonal: LDS
 *                      tiles in 1D; in 2D the register tile 8 x 8 x r (r =
 *                      tile rows per wavefront: 2, 1, and 4 in FP32) and
 *                      LDS tiles (other shapes); column segments 1 x 1 x z
 *                      in 3D;
 *   BTE_TUNE_SWEEP_ONE_LAUNCH  2D steady sweeps in one launch per sweep
 *                      (bte_set_persistent): the register-tile shapes;
 *                      choosing one sets the launch form too (an empty list
 *                      in 1D and 3D);
 *   BTE_TUNE_TRANSIENT tiles of the explicit step and its transpose in one
 *                      and two dimensions (three-dimensional steps walk
 *                      columns and have no choice).
 * LDS tiles hold at most 64 cells and their LDS star fits one compute unit;
 * the results of a sweep or step do not depend on the shape beyond
 * floating-point summation order (not at all on the launch form). */
typedef enum { BTE_TUNE_SWEEP = 0, BTE_TUNE_TRANSIENT = 1, BTE_TUNE_SWEEP_ONE_LAUNCH = 2 } bte_tune_kind;

typedef struct {
    int kind;        /* bte_tune_kind                                     */
    int tile[3];     /* cells per tile along x, y, z                      */
    double ms;       /* mean device time of one sweep / step (ms)        */
    int chosen;      /* 1: the shape kept                                  */
} bte_tune_entry;

/* Candidate shapes of one kind (at most `cap` written to tiles[3 * i ..]);
 * *n = number of candidates (0 or 1: nothing to choose).  Host only. */
bte_status bte_tile_candidates(const bte_problem *p, int kind, int *tiles, int cap, int *n);

/* Use tile shape tile[3] for `kind` from now on.  The shape must be one of
 * bte_tile_candidates (else BTE_ERR_ARG, nothing changed).  Needs a bound
 * workspace (the work lists are rebuilt and uploaded; synchronous). */
bte_status bte_set_tiles(bte_problem *p, int kind, const int *tile);

/* Autotuner: for every kind with more than one candidate, time `reps`
 * sweeps (or steps) with each candidate after one untimed run, keep the
 * fastest and report every candidate in entries[0 .. *n) (at most cap).
 * The two sweep kinds are one choice: the fastest candidate of either is
 * kept (with its launch form) and is the one marked chosen.
 * e_scratch: device buffer of bte_num_unknowns() elements of the problem's
 * precision, overwritten (it is the input state of the timed runs); the
 * diffuse-wall records, T_L and pending-correction fields are cleared.
 * Needs a bound workspace; synchronous on `stream`. */
bte_status bte_autotune(bte_problem *p, void *e_scratch, int reps, bte_tune_entry *entries, int cap, int *n,
                        void *stream);

/* Statistics of the last bte_steady_solve, or of the last timed
 * bte_transient_step (iters = steps, ms_sweep = transport kernels, ms_walls =
 * wall kernels, ms_post = T_L updates). */
bte_status bte_last_stats(const bte_problem *p, bte_solve_stats *out);

/* Mean-free-path band discretisation (Sec. 3.1, eq. banddis): from a
 * mode-level list (heat capacity C >= 0 in J m^-3 K^-1, group speed v >= 0
 * in m/s, relaxation time tau > 0 in s, all host arrays of n_modes) to
 * n_bands bands of the PHONON input.  The mean free path Lambda = v tau of
 * the modes with Lambda > 0 spans [Lambda_min, Lambda_max]; that range is
 * cut into n_bands intervals of equal width in log(Lambda) (band k holds
 * Lambda_k <= v tau < Lambda_{k+1}, the last interval also Lambda_max;
 * modes with v = 0 join band 0).  Per band:
 *   C_b = sum C,  v_b = sum C v / sum C,  tau_b = sum C v^2 tau / (v_b sum C v),
 * so that C_b, C_b v_b and C_b v_b^2 tau_b are the band's sums of C, C v and
 * C v^2 tau.  Empty intervals are dropped: *n_out (<= n_bands) bands are
 * written to C_out, v_out, tau_out (host arrays of n_bands), in ascending
 * mean free path; band_of_mode (host, n_modes, may be NULL) receives each
 * mode's band index in that numbering (-1 for a mode of an interval dropped
 * because its sum C v is zero).  BTE_ERR_ARG: n_modes < 1,
 * n_bands < 1, a null array, a negative C or v, a non-positive tau, or no
 * mode with Lambda > 0.  Host computation: no problem handle, no device. */
bte_status bte_band_discretize(const double *C, const double *v, const double *tau, long long n_modes,
                               int n_bands, double *C_out, double *v_out, double *tau_out, int *n_out,
                               int *band_of_mode);

/* Mean-free-path band discretisation on the device (Sec. 3.1, eq. banddis):
 * the computation of bte_band_discretize with the mode list and the results
 * in device memory, for mode lists produced or kept on the GPU.
 * C, v, tau: device double[n_modes] (1 <= n_modes <= 2^31 - 1);
 * C_out, v_out, tau_out: device double[n_bands]; band_of_mode: device
 * int[n_modes], required (it holds each mode's interval during the call and
 * each mode's band index, or -1, at the end); scratch: device memory of at
 * least bte_band_discretize_scratch_bytes(n_bands) bytes, 256-byte aligned,
 * owned by the caller.  *n_out (host) receives the number of bands.  The
 * intervals and band values are those of bte_band_discretize (the interval
 * of a mode from the FP64 logarithm of its mean free path; band sums over
 * the modes of an interval in a fixed order, so repeated calls give
 * identical bits; the order differs from the host routine's, so values agree
 * to rounding).  The list is validated on the device first: BTE_ERR_ARG for a
 * null pointer, n_modes or n_bands out of range, a small or misaligned
 * scratch, a negative C or v, a non-positive tau or no mode with v tau > 0,
 * with nothing written to C_out, v_out, tau_out or band_of_mode.
 * Synchronous on `stream` (two small device-to-host reads). */
bte_status bte_band_discretize_dev(const double *C, const double *v, const double *tau, long long n_modes,
                                   int n_bands, double *C_out, double *v_out, double *tau_out, int *n_out,
                                   int *band_of_mode, void *scratch, size_t scratch_bytes, void *stream);

/* Bytes of the scratch of bte_band_discretize_dev (0 if n_bands < 1). */
size_t bte_band_discretize_scratch_bytes(int n_bands);

/* Host copy of the direction table: s[n_dir][3], w[n_dir]. */
bte_status bte_get_directions(const bte_problem *p, double *s_host, double *w_host);

const char *bte_last_error(const bte_problem *p);
void bte_destroy(bte_problem *p);

/* ------------------------------------------------------------------------
 * Unstructured meshes: two-dimensional meshes of triangles and
 * quadrilaterals (bte_mesh_setup), tetrahedral meshes (bte_mesh_setup_tet)
 * (Sec. 3.3, eq. disretized_BTE, with the least-squares gradient and the
 * first-order upwind stiffness matrix of Sec. 3.5), steady (sequential
 * scheme, Sec. 3.4) and explicit transient steps (Sec. 4.1), bulk
 * materials (directions on the sphere, in-plane fluxes).  Cell i: area V_i, centre = area centroid x_i; face ij: length
 * S_ij, exterior unit normal n_ij, centre x_f.  Gradient
 * grad e_i = X_i^+ sum_j d_ij (e_j - e_i), d_ij = x_j - x_i, X_i =
 * sum_j d_ij d_ij^T over the stencil of i (the pseudo-inverse drops
 * eigenvalues below 1e-10 of the largest: a cell with one stencil neighbour
 * gets the derivative along it only).  Stencil (the paper names none):
 * every cell sharing a vertex with i (gradient_stencil 0), or the face
 * neighbours (1: on a Cartesian grid the central / one-sided difference of
 * bte_problem; on triangle meshes the sequential iteration then diverges).  Face value e_ij = e_m + grad e_m . (x_f -
 * x_m), m upwind; at a boundary edge the incoming value is the wall's:
 * thermalizing C (T_w - T_ref) / 4 pi, specular the mirror direction's
 * outgoing face value (edges parallel to x or y), diffuse
 * sum_{s.n>0} w s.n e_f / sum_{s.n<0} w |s.n|.  One iteration: T_L from the
 * moments, R = -(1/V) sum_j v (s.n) S e_ij - (e - C T_L / 4 pi) / tau +
 * C P / (4 pi C_tot), then A de = R with A_ii = 1/tau + (1/V) sum_{s.n>0}
 * v s.n S and A_ij = -(1/V) v |s.n| S for the interior upwind neighbour j,
 * solved in per-direction upwind (dependency-graph) order, one launch per
 * level of all directions together; on a cyclic graph the smallest-index
 * cell left is taken with its unresolved upwind couplings lagged (their
 * increments count as zero).  e layout and moments as for bte_problem:
 * e[cell][direction][band], direction-major within a cell. */
typedef struct {
    int n_vertices;
    const double *xy;        /* host [n_vertices][2] vertex coordinates, m       */
    int n_cells;
    const int *cell_ptr;     /* host [n_cells + 1]: cell c has the vertices
                                cell_vtx[cell_ptr[c] .. cell_ptr[c + 1])         */
    const int *cell_vtx;     /* counter-clockwise, 3 or 4 vertices per cell      */
    const int *edge_tag;     /* host [cell_ptr[n_cells]]: boundary tag of the edge
                                from vertex k to vertex k + 1 of each cell, -1
                                for an edge shared with another cell             */
    int n_tags;
    const int *tag_bc;       /* host [n_tags]: BTE_BC_THERMAL, BTE_BC_SPECULAR or
                                BTE_BC_DIFFUSE                                   */
    const double *tag_T;     /* host [n_tags]: wall temperature, K (thermalizing) */
    int gradient_stencil;    /* 0: cells sharing a vertex, 1: face neighbours     */
} bte_mesh;

/* Tetrahedral meshes (three dimensions): cell volume |det| / 6, centre =
 * vertex mean, face k of a cell = the triangle opposite its vertex k (area
 * |cross| / 2, centre = vertex mean, normal away from vertex k); the
 * least-squares fit is 3 x 3; specular faces must be normal to x, y or z.
 * Everything else as for bte_mesh. */
typedef struct {
    int n_vertices;
    const double *xyz;       /* host [n_vertices][3] vertex coordinates, m       */
    int n_cells;
    const int *cell_vtx;     /* host [n_cells][4] vertices of each tetrahedron   */
    const int *face_tag;     /* host [n_cells][4]: boundary tag of the face
                                opposite vertex k, -1 for a shared face          */
    int n_tags;
    const int *tag_bc;       /* host [n_tags]: BTE_BC_THERMAL, BTE_BC_SPECULAR or
                                BTE_BC_DIFFUSE                                   */
    const double *tag_T;     /* host [n_tags]: wall temperature, K (thermalizing) */
    int gradient_stencil;    /* 0: cells sharing a vertex, 1: face neighbours     */
} bte_tet_mesh;

typedef struct bte_mesh_problem bte_mesh_problem;

/* Builds the geometry, least-squares matrices, wall records, directions and
 * the per-level sweep schedule on the host.  Errors: BTE_ERR_ARG (null
 * pointers, a cell that is not 3 or 4 vertices, counter-clockwise and of
 * positive area, an edge shared by more than two cells, a boundary edge
 * without a tag or an interior edge with one, a tag out of range, a
 * specular edge not parallel to x or y, bad bands), BTE_ERR_UNSUPPORTED
 * (synthetic scheme, a limiter, two-dimensional materials).  The control's
 * precision, max_iter, residual_temp and dt are used.  *out is set whenever
 * allocation succeeded (destroy it also on error). */
bte_status bte_mesh_setup(const bte_mesh *mesh, const bte_material *mat, const bte_control *ctl,
                          bte_mesh_problem **out);
/* The same for a tetrahedral mesh (errors as above: zero volume or area,
 * a face shared by more than two cells, tags, a specular face not normal
 * to an axis); the problem takes every bte_mesh_* call below. */
bte_status bte_mesh_setup_tet(const bte_tet_mesh *mesh, const bte_material *mat, const bte_control *ctl,
                              bte_mesh_problem **out);
/* Device workspace the caller provides (256-byte aligned) and binds. */
size_t bte_mesh_workspace_bytes(const bte_mesh_problem *p);
bte_status bte_mesh_bind(bte_mesh_problem *p, void *ws_dev, size_t bytes);
int bte_mesh_num_cells(const bte_mesh_problem *p);
int bte_mesh_num_directions(const bte_mesh_problem *p);
/* Level launches of one sweep (the depth of the deepest direction's
 * dependency graph) and the number of lagged couplings over all directions. */
int bte_mesh_num_levels(const bte_mesh_problem *p);
int bte_mesh_num_lagged(const bte_mesh_problem *p);
/* Heat source P per cell (device double[n_cells], W/m^3; NULL: none). */
bte_status bte_mesh_set_source(bte_mesh_problem *p, const double *P_dev, void *stream);
/* T, T_L (K) and q (W/m^2, [n_cells][3]) of e, device doubles; any may be
 * NULL. */
bte_status bte_mesh_moments(bte_mesh_problem *p, const void *e_dev, double *T_dev, double *TL_dev, double *q_dev,
                            void *stream);
/* R(e) with e0 from TLdev (device double[n_cells], T_L - T_ref; NULL: from
 * the moments of e), into R_dev (same type and size as e). */
bte_status bte_mesh_residual(bte_mesh_problem *p, const void *e_dev, const double *TLdev_dev, void *R_dev,
                             void *stream);
/* Source iterations on e in place (init != 0: start from e = 0, i.e.
 * T = T_ref) until max |T^{n+1} - T^n| <= residual_temp max |T^{n+1} - T_ref|
 * or max_iter iterations (BTE_ERR_NOT_CONVERGED).  stats: iters, eps_T,
 * converged, ms_total, sweep_launches, updates and the device times (HIP
 * events on the stream, summed over the iterations) of the level sweeps
 * (ms_sweep), of gradients + wall inflow + residual (ms_walls) and of the
 * moments and convergence test (ms_post).  Synchronous. */
bte_status bte_mesh_steady_solve(bte_mesh_problem *p, void *e_dev, int init, bte_solve_stats *stats,
                                 void *stream);
/* n_steps explicit steps on e in place (Sec. 4.1, Algorithm 2):
 * e^{n+1} = e^n + dt R(e^n), T_L from the moments of e^n, dt =
 * control.dt.  BTE_ERR_CFL unless dt / tau_min < 1 and
 * dt v_max max_i (sum_f S_f / V_i) / 2 < 1 (on a square cell the structured
 * grids' dt v_max sum_a 1/h_a < 1).  Asynchronous on the stream. */
bte_status bte_mesh_transient_step(bte_mesh_problem *p, void *e_dev, int n_steps, void *stream);
const char *bte_mesh_last_error(const bte_mesh_problem *p);
void bte_mesh_destroy(bte_mesh_problem *p);

#ifdef __cplusplus
}
#endif
#endif /* BTE_H */
