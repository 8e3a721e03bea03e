/*
 * sph.h -- C-ABI of the MI355X (gfx950) strength-SPH hot path.
 *
 * Method: "SPH in pkdgrav3 for Shock Physics Simulations. II. Shear
 * Strength" (Meier et al., arXiv 2603.19764), sec. 2: kernel-sum density
 * with grad-h term (sec. 2.1), Cauchy stress with deviatoric part and
 * Jaumann rate (sec. 2.2), corrected velocity gradient (Velocity_Gradient,
 * Correction_Tensor, Corrected_Gradients eqs.), Collins yield with thermal
 * softening and plastic rescaling (sec. 2.3), momentum and energy equations
 * with the full stress tensor and Monaghan artificial viscosity (sec. 2.1,
 * 2.2), predictor-corrector time integration of S (sec. 2.4).
 *
 * Conventions that hold for every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, in
 *     structure-of-arrays layout: one row of n values per component.
 *     Deviatoric stress S has 5 rows (xx, yy, xy, xz, yz) with
 *     S_zz = -S_xx - S_yy; the velocity gradient G has 9 rows, row 3a+b
 *     holding dv^a/dx^b.  Rows of a multi-row array are n_stride = n
 *     elements apart.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     null stream) and allocates nothing; a call sequence can be captured
 *     into a hipGraph.  Scalars that change from step to step (the time
 *     step) are read from device memory for that reason.  Exceptions, which
 *     synchronise and are not capturable: sph_sync_status, sph_timing_read,
 *     sph_bound_mass, and the first call with a new run layout
 *     (sph_state.run_start), which uploads it.
 *   - Argument errors are returned synchronously (SPH_EINVAL, SPH_ESTATE,
 *     SPH_ECAPACITY).  Conditions found on the device (neighbour list
 *     overflow, cell table overflow, a NaN or infinite value) raise a
 *     device flag that sph_sync_status() reports after synchronising the
 *     stream.
 *   - After sph_build_cells the pair passes expect every per-particle array
 *     in the cell order the call produced: the caller permutes its arrays
 *     with sph_reorder (perm[k] = input index of the k-th particle).
 *   - sph_ctx owns only internal scratch (cell tables, sorted positions,
 *     neighbour lists), sized once by sph_create.  One ctx per stream.
 *   - No exception crosses the boundary; sph_last_error() describes the
 *     last failure of a ctx.
 */
#ifndef SPH_ABI_H_
#define SPH_ABI_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;
typedef void *sph_stream; /* hipStream_t */

typedef enum {
    SPH_OK = 0,
    SPH_EINVAL = 1,     /* bad argument (null pointer, size out of range)        */
    SPH_EHIP = 2,       /* a HIP runtime call failed                              */
    SPH_ENOMEM = 3,     /* device allocation failed in sph_create                 */
    SPH_ECAPACITY = 4,  /* n above the ctx capacity, or a device-side overflow    */
    SPH_ENONFINITE = 5, /* non-finite value met by a kernel                       */
    SPH_ESTATE = 6      /* call out of order (pair pass before sph_build_cells)   */
} sph_status;

/* Arithmetic of the pair passes.  SPH_FP64: every pair term in IEEE double on
 * absolute positions.  SPH_FP32_CELLREL: pair terms in float on positions
 * stored relative to the origin of each particle's cell, per-particle
 * epilogues (EOS, yield, correction-tensor inverse, stress update, kicks) in
 * double.  Neighbour sets are the same in both (FP64 test). */
typedef enum { SPH_FP64 = 0, SPH_FP32_CELLREL = 1 } sph_precision;

/* Material parameters (sec. 2.2 shear modulus, sec. 2.3 yield; Tillotson
 * EOS constants since EOSlib tables are not part of this library). */
typedef struct {
    double rho0, A, B, E0, Eiv, Ecv, a, b, alpha, beta; /* Tillotson              */
    double cv, T_ref, c_min;      /* T = T_ref + u/cv; sound-speed floor          */
    double shear_modulus, nu;     /* > 0: constant; otherwise 3(1-2nu)/(2(1+nu)) rho c^2 */
    double Y0, Ym, mu_i, mu_d, xi, T_melt; /* Collins yield, thermal softening    */
    int32_t strength_on, thermal_softening_on;
    /* Melting temperature as a table of density (sec. 2.3 gives T_melt as a
     * tabulated function of rho): with tmelt_n >= 2 nodes (ascending rho),
     * T_melt(rho) is interpolated linearly and held at the end values
     * outside the table; otherwise the constant T_melt above is used. */
    int32_t tmelt_n, tmelt_pad;
    double tmelt_rho[8], tmelt_T[8];
    /* Tabulated EOS (sec. 2.3 takes P, c and T from M-ANEOS tables): with
     * eos_nrho >= 2 and eos_nu >= 2 the state comes from a table instead of
     * Tillotson.  eos_rho[eos_nrho] and eos_u[eos_nu] are the node
     * coordinates, strictly ascending; eos_P, eos_c, eos_T hold the values
     * at the nodes, row-major [i_rho * eos_nu + i_u].  All five are DEVICE
     * pointers owned by the caller and must stay valid while calls that use
     * the material run.  Between nodes each value is the bilinear
     * interpolant in (rho, u); rho and u outside the grid are moved to its
     * edge; c is floored at c_min.  The Tillotson constants, cv and T_ref
     * are then unused.  Both counts at most 2^20, their product at most
     * 2^26; nodes that are not ascending give wrong values, never an
     * out-of-bounds read. */
    int32_t eos_nrho, eos_nu;
    const double *eos_rho, *eos_u, *eos_P, *eos_c, *eos_T;
    /* Tillotson only: the cold (compressed-branch) formula gives zero
     * pressure, with zero derivatives, for rho < rho_limit * rho0, so that
     * strongly expanded cold material (a free surface, a crack) carries no
     * tension; the blend with the hot branch keeps its form.  0 <= rho_limit
     * <= 1; 0 keeps the formula's tension everywhere. */
    double rho_limit;
} sph_material;

/* Run parameters: Monaghan AV (sec. 2.1), Courant factor (courant_condition
 * eq.), rotation sign of the Jaumann term (+1: R S - S R, the objective
 * rate; -1: the index order as printed), external gravity, correction
 * tensor switch (Corrected_Gradients eq.), Omega = 1 switch, and the
 * self-gravity of each run added by sph_step when grav_G > 0 (see
 * sph_gravity for the meaning of the three grav_ fields), and adaptive
 * smoothing lengths (kernel-mass equation of sec. 2.1) when adapt_ngb > 0. */
typedef struct {
    double av_alpha, av_beta, av_eps, eta_C, rot_sign;
    double g[3];
    int32_t use_correction_tensor, omega_one;
    double grav_G, grav_eps_over_h, grav_theta;
    double adapt_ngb;   /* > 0: sph_init / sph_step adapt h to constant kernel
                           mass (sph_adapt_h) before each evaluation          */
    double adapt_skin;  /* cap of one adaptation: h <= adapt_skin h_old (>= 1) */
    double eta_a;       /* > 0: a particle's step is also capped by the
                           acceleration criterion eta_a sqrt(h_i / |a_i|)
                           (time-integration section)                        */
    int32_t rungs;      /* > 0: hierarchical individual steps dt0 2^-r,
                           r = 0 .. rungs-1 (<= 40), dt0 = sph_state.dt_max;
                           0: one step per run                              */
    int32_t rungs_pad;
    double far_factor;  /* > 0: sph_init fixes for each run the cube centred
                           on its bounding box, of half-edge far_factor times
                           the box's largest half-extent; from then on the
                           run's search grid covers only that cube, and a
                           particle outside it (ejecta far from a collision)
                           enters no pair set, feels no pair force and no
                           self-gravity, is no source of self-gravity, drifts
                           with its velocity, and counts as unbound in
                           sph_bound_mass.  The grid of a dispersing run then
                           stays bounded.  0: the grid covers every particle */
} sph_params;

/* ---------------------------------------------------------------- context */

/* Create a context on device `device` for up to `capacity` particles, at
 * most `max_neighbors` pair-set members per particle, a cell table of at
 * most `max_cells` entries (summed over runs) and `max_runs` independent
 * particle sets.  capacity <= 2^26.  Returns SPH_ENOMEM if the scratch does
 * not fit. */
sph_status sph_create(sph_ctx **ctx, int64_t capacity, int32_t max_neighbors,
                      int64_t max_cells, int32_t max_runs, int32_t device);
sph_status sph_destroy(sph_ctx *ctx);
/* Message of the last failure of `ctx`; with ctx = NULL, of the last failed
 * context-free call (sph_diagnostics_noalloc) on the calling thread. */
const char *sph_last_error(const sph_ctx *ctx);

/* Synchronise `stream` and report (then clear) device-side flags:
 * SPH_ECAPACITY after a neighbour-list, cell-table or gravity-list overflow
 * or a step below the shortest rung; SPH_ENONFINITE after a kernel met a NaN
 * or infinite value in what it computes: a position or smoothing length
 * binned by the neighbour search (after the drift of sph_step), density or
 * Omega, EOS state (P, c, T, Y, Gamma), predicted or kicked stress, velocity
 * gradient, stress rate, acceleration, energy rate, CFL step, drifted,
 * predicted or kicked position, velocity or energy.  Each kernel raises the
 * flag with one atomic per wavefront; the values themselves are written as
 * computed (NaN propagates; a NaN CFL step is left out of the step minimum).
 * When several flags are up, the first in the order above is returned and
 * all are cleared. */
sph_status sph_sync_status(sph_ctx *ctx, sph_stream stream);

/* ---------------------------------------------------- neighbour search (a1) */

/* Bin particles into a uniform cell grid per run, sort them by the Morton
 * key of their cell, and build the pair sets
 *    N_i = { j != i : |x_i - x_j|^2 < max((2h_i)^2, (2h_j)^2) }
 * (support H = 2h; the density set uses (2h_i)^2 alone and is flagged per
 * entry).  The squared separation is ((dx dx + dy dy) + dz dz) in IEEE double
 * with no fused operation, dx = x_i - x_j, so membership is exact.
 *   x, y, z, h : n input positions and smoothing lengths (input order)
 *   run_start  : n_runs + 1 host integers, particles of run r occupy
 *                [run_start[r], run_start[r+1]) in input order; NULL means
 *                one run.  Runs never interact.
 *   cell_min   : lower bound of the cell edge; the edge used per run is
 *                max(cell_min, 2 max h) (grown if the table would overflow)
 *   perm_out   : n int32, perm_out[k] = input index of sorted particle k
 * Errors: SPH_EINVAL (null pointer, n < 0), SPH_ECAPACITY (n > capacity or
 * n_runs > max_runs); device overflow of the lists is reported later by
 * sph_sync_status. */
sph_status sph_build_cells(sph_ctx *ctx, int64_t n, const double *x, const double *y,
                           const double *z, const double *h, int32_t n_runs,
                           const int64_t *run_start, double cell_min, int32_t *perm_out,
                           sph_stream stream);

/* Permute `nfields` arrays: dst[f][k] = src[f][perm[k]] for k < n, each
 * element `elem_bytes[f]` bytes (4 or 8) and rows[f] rows of n elements.
 * src and dst must not overlap.  Pointer arrays are host arrays of at most
 * 64 entries. */
sph_status sph_reorder(sph_ctx *ctx, int64_t n, const int32_t *perm, int32_t nfields,
                       const void *const *src, void *const *dst, const int32_t *elem_bytes,
                       const int32_t *rows, sph_stream stream);

/* Export the pair sets of the last build as CSR in sorted order:
 * offsets (n+1, int64), nbr (sorted index of j), dflag (1 if j is in the
 * density set of i).  nbr/dflag must hold offsets[n] entries; pass NULL for
 * nbr and dflag to get offsets only.  Test and diagnostic use. */
sph_status sph_neighbors_csr(sph_ctx *ctx, int64_t *offsets, int32_t *nbr, uint8_t *dflag,
                             sph_stream stream);

/* Copy (asynchronously, on `stream`) the running total of ordered pairs
 * sum_i |N_i|, accumulated over every build since sph_create, into the
 * device uint64 *out. */
sph_status sph_pair_count(sph_ctx *ctx, uint64_t *out, sph_stream stream);

/* ---------------------------------------------------------- density (a2) */

/* rho_i = sum_j m_j W(r_ij, h_i) over the density set and the self term;
 * Omega_i = 1 + h_i/(3 rho_i) sum_j m_j dW(r_ij, h_i)/dh_i (sec. 2.1,
 * Density_estimate eq. and the grad-h term), Wendland C2 kernel with
 * support 2h.  Epilogue per particle in double: Tillotson P and c with
 * energy u, T = T_ref + u/cv, yield Y = min(Y_i, Y_d) with the thermal
 * softening factor (sec. 2.3), shear modulus Gamma (sec. 2.2).
 *   m, h, u, mat : sorted inputs (mat indexes mats[0..n_materials))
 *   outputs      : rho, omega, P, cs, T, Y, Gmod, n doubles each. */
sph_status sph_density(sph_ctx *ctx, int64_t n, const double *m, const double *h,
                       const double *u, const int32_t *mat, const sph_material *mats,
                       int32_t n_materials, const sph_params *prm, sph_precision prec,
                       double *rho, double *omega, double *P, double *cs, double *T,
                       double *Y, double *Gmod, sph_stream stream);

/* --------------------------------------------------------- gradients (a4) */

/* F_i = -1/2 sum_j m_j v_ij (x) (dW_ij(h_i)/(Omega_i rho_i) + dW_ij(h_j)/(Omega_j rho_j)),
 * C_i^-1 the same sum with x_ij in place of v_ij, G_i = F_i C_i
 * (Velocity_Gradient, Correction_Tensor, Corrected_Gradients eqs.).  The
 * 3x3 inverse is taken in double from the adjugate; a singular C^-1
 * (|det| < 1e-12 |C^-1|_F^3 or fewer than 4 neighbours) or
 * use_correction_tensor = 0 gives C = identity.
 *   vx, vy, vz : sorted (predicted) velocities;  rho, omega from sph_density
 *   G          : 9 rows of n doubles;  n_singular: device int64 counter,
 *                incremented by the number of singular particles (may be NULL). */
sph_status sph_gradients(sph_ctx *ctx, int64_t n, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *h,
                         const double *rho, const double *omega, const sph_params *prm,
                         sph_precision prec, double *G, int64_t *n_singular,
                         sph_stream stream);

/* --------------------------------------------------- stress update (a3, a5, a7) */

enum {
    SPH_STRESS_PREDICT = 1, /* S_pred = f(S_half + dt/2 Sdot), f = min(Y/sqrt(J2), 1)    */
    SPH_STRESS_RATE = 2,    /* Sdot = 2 Gamma (eps - tr(eps)/3) + rot_sign (R S_pred - S_pred R) */
    SPH_STRESS_KICK = 4,    /* S_half = f(S_half + dt/2 Sdot) + dt_next/2 Sdot; eps2 += dt eps:eps/2 */
    SPH_STRESS_OPEN = 8     /* S_half = S_pred + dt_next/2 Sdot (first opening kick of a run)      */
};

/* Per-particle stress phases of sec. 2.4 (Predict_S eq., the closing and
 * opening kicks) and the stress rate of Deviatoric_Stress_derivative eq.
 * with eps = (G + G^T)/2, R = (G - G^T)/2.  `phase` is one of the values
 * above.  dt and dt_next point to device doubles.  Fixed particles are left
 * untouched.  Arrays: S_half, S_pred, Sdot 5 rows; G 9 rows; Y, Gmod, eps2
 * one row; fixed (int32 0/1) may be NULL. */
sph_status sph_stress_update(sph_ctx *ctx, int32_t phase, int64_t n, const double *dt,
                             const double *dt_next, const double *G, const double *Y,
                             const double *Gmod, const int32_t *fixed, const sph_params *prm,
                             double *S_half, double *S_pred, double *Sdot, double *eps2,
                             sph_stream stream);

/* ------------------------------------------------------------ forces (a6) */

/* a_i = sum_j m_j (K_i A_i + K_j A_j) x_ij with A = (-P I + S)/(Omega rho^2) and
 * grad_i W_ij(h) = K(r,h) x_ij (momentum equation of sec. 2.2), minus the
 * Monaghan AV term with the mean kernel gradient for approaching pairs
 * (sec. 2.1), plus g.  du_i/dt = -A_i : sum_j m_j v_ij (x) grad_i W_ij(h_i)
 * (compatible hydro term plus the strength term of the energy equation)
 * plus the AV heating of AV_heating eq.  dt_cfl_i = eta_C min_j
 * h_i/((1+0.6 alpha) c_i + 0.6 beta |min(0, mu_ij)|) (courant_condition eq.).
 *   S : predicted, rescaled deviatoric stress (5 rows);  outputs n doubles. */
sph_status sph_forces_stress(sph_ctx *ctx, int64_t n, const double *vx, const double *vy,
                             const double *vz, const double *m, const double *h,
                             const double *rho, const double *omega, const double *P,
                             const double *cs, const double *S, const sph_params *prm,
                             sph_precision prec, double *ax, double *ay, double *az,
                             double *dudt, double *dt_cfl, sph_stream stream);

/* ------------------------------------------------------ kicks and drift (a7) */

enum {
    SPH_KD_DRIFT = 1,   /* x += dt v_half                                          */
    SPH_KD_PREDICT = 2, /* v_pred = v_half + dt/2 a, u_pred = u_half + dt/2 dudt   */
    SPH_KD_KICK = 4,    /* v_half += dt/2 a + dt_next/2 a, same for u              */
    SPH_KD_OPEN = 8     /* v_half += dt_next/2 a, same for u (start of a run)      */
};

/* Kick-drift-kick updates of sec. 2.4 for positions, velocities and
 * energies; fixed particles are left untouched.  dt, dt_next are device
 * doubles.  v_pred/u_pred are written by SPH_KD_PREDICT only. */
sph_status sph_kick_drift(sph_ctx *ctx, int32_t phase, int64_t n, const double *dt,
                          const double *dt_next, const int32_t *fixed, double *x, double *y,
                          double *z, double *vx, double *vy, double *vz, double *u,
                          const double *ax, const double *ay, const double *az,
                          const double *dudt, double *vpx, double *vpy, double *vpz,
                          double *up, sph_stream stream);

/* dt_out = min over non-fixed particles of dt_cfl (device double). */
sph_status sph_dt_min(sph_ctx *ctx, int64_t n, const double *dt_cfl, const int32_t *fixed,
                      double *dt_out, sph_stream stream);

/* Conservation diagnostics (device doubles, 13 values): sum m a (3),
 * sum m x x a (3), sum m (v . a + dudt), sum m v (3), sum m x x v (3). */
sph_status sph_diagnostics(sph_ctx *ctx, int64_t n, const double *x, const double *y,
                           const double *z, const double *vx, const double *vy,
                           const double *vz, const double *m, const double *ax,
                           const double *ay, const double *az, const double *dudt,
                           double *out13, sph_stream stream);

/* The diagnostics above without a context, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, hosts
 * that forbid hipMalloc): the same kernels and the same 13 results, bit for
 * bit, with the partial sums kept in a fixed device array of the library
 * (256 x 13 doubles, 26,624 bytes) that each GPU holds from the first call
 * on it until the process ends.  Runs on the current device; `stream` must
 * belong to it.  Allocates nothing and needs no initialisation by the
 * caller (the first call on a device looks up the array's address).  Every
 * call on a GPU shares its array, so calls that overlap on one GPU (two
 * streams, two host threads) race and may return wrong sums; calls in
 * sequence on one stream are safe (each call overwrites every partial sum it
 * reads).  n at most SPH_NOALLOC_MAX_N (the library's particle limit);
 * SPH_EINVAL for a larger n or a null array, with the reason in
 * sph_last_error(NULL). */
#define SPH_NOALLOC_MAX_N ((int64_t)1 << 26)
sph_status sph_diagnostics_noalloc(int64_t n, const double *x, const double *y,
                                   const double *z, const double *vx, const double *vy,
                                   const double *vz, const double *m, const double *ax,
                                   const double *ay, const double *az, const double *dudt,
                                   double *out13, sph_stream stream);

/* ------------------------------------------------- adaptive smoothing length */

/* Smoothing lengths at constant kernel mass (the kernel-mass equation of
 * sec. 2.1): for every particle, Newton-Raphson on
 *     (4/3) pi (2 h_i)^3 rho_i(h_i) = n_ngb m_i
 * with rho and drho/dh summed over the pair list of the last neighbour
 * search (self term included), each step limited to a factor 2, until
 * |dh| <= tol h or max_iter steps.  The search must have been done with
 * lengths h_search at least as large as the answer: a step past a
 * particle's h_search is held at h_search, and a particle whose next step
 * would leave it again stops there and is counted in *n_clamped (device
 * int64, may be NULL; not reset by the call).  Sorted order.  m, h_start:
 * masses and starting lengths (n doubles); h_out: result (n doubles, may
 * equal h_start); *iterations: device int32 raised to the largest number of
 * steps taken (may be NULL; not reset).  FP64. */
sph_status sph_adapt_h(sph_ctx *ctx, int64_t n, const double *m, const double *h_start,
                       double n_ngb, double tol, int32_t max_iter, double *h_out,
                       int64_t *n_clamped, int32_t *iterations, sph_stream stream);

/* ------------------------------------------------------------ self-gravity */

/* Softened self-gravity of every run (the gravitational term of the
 * momentum equation, sec. 2.2) at the positions of the last neighbour
 * search, in its sorted order: Barnes-Hut over a pyramid of the search
 * cells (level 0 = the cells, level k = 2x2x2 blocks of level k-1, level -1
 * = the octants of each cell), monopole moments, FP32 arithmetic on
 * positions relative to each run's grid origin.  The targets of each 2x2x2
 * block of cells share one walk: a node whose box is disjoint from the
 * block's and for which b < theta d (b: distance from the node's centre of
 * mass to its farthest corner; d: from the centre of mass to the block)
 * acts on all of them as a point mass; other nodes are opened down to
 * single particles.
 * Plummer softening of length eps_r = eps_over_h x max_i h_i of run r:
 *   a_i = G sum_j m_j (x_j - x_i) / (r^2 + eps_r^2)^(3/2),
 *   phi_i = -G sum_j m_j / (r^2 + eps_r^2)^(1/2),  j != i, same run.
 * m: masses (n doubles, sorted order); active: int32 0/1 per particle or
 * NULL (all): inactive particles exert no gravity but receive it.
 * ax, ay, az: outputs, overwritten (accumulate = 0) or added to (1); phi:
 * output or NULL.  G >= 0, eps_over_h > 0, theta in [0.3, 1].  A walk that
 * outgrows its lists is reported by sph_sync_status (SPH_ECAPACITY) and
 * leaves NaN in the outputs of its particles. */
sph_status sph_gravity(sph_ctx *ctx, int64_t n, const double *m, const int32_t *active, double G,
                       double eps_over_h, double theta, int32_t accumulate, double *ax,
                       double *ay, double *az, double *phi, sph_stream stream);

/* Bound mass of every run (sec. 3, catastrophic disruption: the bound mass
 * found by removing unbound particles until none is left), at the positions
 * of the last neighbour search, sorted order.  Starting from every particle
 * of its run: v_c = mass-weighted mean velocity of the bound set, phi =
 * potential of the bound set (sph_gravity with the bound flags as the active
 * set), and particles with |v - v_c|^2 / 2 + phi > 0 leave the set for good;
 * repeated until no particle leaves or max_iter passes.  bound: int32 flags
 * (n), m_bound: bound mass per run (n_runs doubles), work: 4 n doubles of
 * scratch (the last potential is left in its first n).  Synchronises the
 * stream once per pass (the test for convergence); not capturable.
 * iterations: passes done (host, may be NULL). */
sph_status sph_bound_mass(sph_ctx *ctx, int64_t n, const double *vx, const double *vy,
                          const double *vz, const double *m, double G, double eps_over_h,
                          double theta, int32_t max_iter, int32_t *bound, double *m_bound,
                          double *work, int32_t *iterations, sph_stream stream);

/* ------------------------------------------------------- whole step (a1-a8) */

/* Rows of the persistent double state buffer (each row n_cap doubles).
 * v, u and S hold half-step values, a, dudt and Sdot the derivatives of the
 * last evaluation. */
enum {
    SPH_X = 0, SPH_Y, SPH_Z, SPH_VX, SPH_VY, SPH_VZ, SPH_U,
    SPH_S = 7,                      /* 5 rows */
    SPH_AX = 12, SPH_AY, SPH_AZ, SPH_DUDT,
    SPH_SDOT = 16,                  /* 5 rows */
    SPH_M = 21, SPH_H, SPH_EPS2,
    SPH_DTP = 24,                   /* individual steps: the particle's step and   */
    SPH_EL = 25,                    /* the time elapsed in it, in ticks (exact);
                                       kept (and carried through the sorts) only
                                       while sph_params.rungs > 0               */
    SPH_NF64 = 26
};
/* Rows of the persistent int32 state buffer: material id, particle id (any
 * caller label, carried through the sorts), fixed flag (0/1), run id. */
enum { SPH_MAT = 0, SPH_ID, SPH_FIXED, SPH_RUN, SPH_NI32 = 4 };

/* Rows of the work buffer (each n_cap doubles) written by sph_step.  With
 * individual steps, rows that hold derivatives or their sums (G, DT) are
 * valid only where SPH_W_ACT is 1 (the particles whose step ended). */
enum {
    SPH_W_RHO = 0, SPH_W_OMEGA, SPH_W_P, SPH_W_CS, SPH_W_T, SPH_W_Y, SPH_W_GMOD,
    SPH_W_VP = 7,                   /* 3 rows */
    SPH_W_UP = 10,
    SPH_W_SP = 11,                  /* 5 rows */
    SPH_W_G = 16,                   /* 9 rows */
    SPH_W_DT = 25,
    SPH_W_PERM = 26,                /* int32 view of one row */
    SPH_W_TAU = 27,                 /* predictor interval of the step, then (with
                                       rungs) the time to the end of the step      */
    SPH_W_ACT = 28,                 /* int32 view: 1 where the step ends now        */
    SPH_NW = 29
};

typedef struct {
    int64_t n, n_cap;            /* particles, row stride                         */
    double *f64[2];              /* two buffers of SPH_NF64 x n_cap doubles; [cur] holds the state */
    int32_t *i32[2];             /* two buffers of SPH_NI32 x n_cap int32          */
    double *work;                /* SPH_NW x n_cap doubles                          */
    double *dt;                  /* device, one double per run (n_runs of them when
                                    run_start is set, else one): the step of the
                                    coming drift of that run                       */
    double *dt_next;             /* device scratch of the same length               */
    int64_t *n_singular;         /* device counter (may be NULL)                    */
    int32_t cur;                 /* 0 or 1; flipped by every sph_step               */
    int32_t n_runs;
    const int64_t *run_start;    /* host, n_runs + 1 offsets (NULL: one run).  Runs
                                    are independent simulations concatenated in the
                                    buffers: no pair crosses a run, and each run
                                    takes its own CFL step (batched scans)          */
    double cell_min;
    double dt_max;               /* > 0: upper bound of the step; with individual
                                    steps (sph_params.rungs > 0) the base step dt0  */
    double *clock;               /* device, one double per run (individual steps
                                    only, else may be NULL): the run's time in ticks
                                    of the shortest rung, dt0 2^-(rungs-1)           */
    double *time;                /* device, one double per run, or NULL: the run's
                                    simulated time, set to 0 by sph_init and advanced
                                    by every sph_step by the step (substep) the run
                                    took                                            */
} sph_state;

/* Start a run: neighbour search and reorder (buffers flip), derivatives at
 * the current state (predicted values = current values, S rescaled),
 * dt[r] = min of dt_cfl over the particles of run r (capped by dt_max) and
 * the first opening kick.  With individual steps (prm->rungs > 0, dt_max =
 * the base step dt0, clock set): each particle takes the longest step
 * dt0 2^-r not above its own (CFL, and acceleration criterion when
 * eta_a > 0), its opening kick uses it, clock[r] = 0 and dt[r] is the
 * shortest step of run r. */
sph_status sph_init(sph_ctx *ctx, sph_state *st, const sph_material *mats, int32_t n_materials,
                    const sph_params *prm, sph_precision prec, sph_stream stream);

/* One step: drift, neighbour search and reorder (buffers flip), predictor,
 * density + EOS + yield, stress predict and rescale, gradients, stress rate,
 * forces, closing kick with rescale, next step of each run from its CFL
 * minimum, opening kick.  With individual steps it is one substep of each
 * run, to the nearest end of a particle's step: every particle drifts and
 * is predicted from the start of its own step (time elapsed less half its
 * step); density, EOS, yield and the rescaled predicted stress for all;
 * gradients, stress rate, forces, closing kick, new step (lengthened only
 * at a multiple of the new step; below the shortest rung is reported by
 * sph_sync_status) and opening kick for the particles whose step ends
 * (SPH_W_ACT); clock[r] advances by the substep in ticks.  All on `stream`, no host synchronisation, no
 * allocation and no memset: a fixed sequence of kernel launches whose device
 * pointers repeat every two steps, so an even number of steps can be
 * captured in a hipGraph and replayed.  Particle masses must be positive
 * (the fused sweep stores each particle's mass-weighted terms and divides
 * its own by its mass). */
sph_status sph_step(sph_ctx *ctx, sph_state *st, const sph_material *mats, int32_t n_materials,
                    const sph_params *prm, sph_precision prec, sph_stream stream);

/* ------------------------------------------------- Q_RD* proposal network */

/* Multilayer perceptron 4 -> 64 -> 64 -> 1 (tanh, tanh, logistic) used to
 * propose impact speeds when bracketing the catastrophic disruption threshold
 * (the paper's Q_RD* bisection of sec. 3 is the fallback).  Float32 device
 * arrays; parameters in one flat array of sph_mlp_num_params() = 4545 values
 * laid out W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3.  These are for the
 * batched scan driver, outside the per-step hot path. */
int32_t sph_mlp_num_params(void);

/* out[s] = network(X[s][0..3]) for s < batch; h1, h2 (batch x 64 each) keep
 * the hidden activations for sph_mlp_backward (may be NULL otherwise). */
sph_status sph_mlp_forward(int32_t batch, const float *X, const float *params, float *out,
                           float *h1, float *h2, sph_stream stream);

/* Gradient of (1/batch) sum_s (out_s - Y_s)^2 with respect to the parameters
 * into grads (4545), from a forward pass with h1, h2 kept.  work: device
 * scratch of batch * 129 floats.  Deterministic (fixed summation order). */
sph_status sph_mlp_backward(int32_t batch, const float *X, const float *Y, const float *params,
                            const float *out, const float *h1, const float *h2, float *work,
                            float *grads, sph_stream stream);

/* *loss = (1/batch) sum_s (out_s - Y_s)^2 (device float), summed in a fixed
 * order (deterministic). */
sph_status sph_mlp_loss(int32_t batch, const float *out, const float *Y, float *loss,
                        sph_stream stream);

/* One bias-corrected Adam step (step >= 1) on params with moments m, v. */
sph_status sph_mlp_adam(float *params, const float *grads, float *m, float *v, int32_t step,
                        float lr, float beta1, float beta2, float eps, sph_stream stream);

/* ------------------------------------------------------ kernel timing */

/* Pass kernels whose launches can be timed with HIP events. */
enum { SPH_T_BUILD = 0, SPH_T_DENSITY, SPH_T_GRADIENTS, SPH_T_FORCES, SPH_T_COUNT };

/* enable = 1: from now on record a pair of hipEvents on the launch stream
 * around every launch of the kernels above and reset the totals; 0: stop.
 * Not for use while a stream is being captured into a graph. */
sph_status sph_timing(sph_ctx *ctx, int32_t enable);

/* Synchronise the recorded events and return the summed duration (ms) and
 * the number of timed launches of kernel `which` since sph_timing(ctx, 1). */
sph_status sph_timing_read(sph_ctx *ctx, int32_t which, double *total_ms, int64_t *launches);

/* ------------------------------------------------------ launch tuning */

/* Launch-shape knobs of a context, chosen by an autotuner that times them on
 * a sample of the workload.  None changes a result beyond the summation
 * order of the pair sums (lanes) or the cell grid (cell scale: the neighbour
 * sets themselves are exact for any cell edge >= 2 h_max).
 *   SPH_TUNE_LANES_*   lanes per particle i of a pair pass: 4, 8 or 16
 *                      (per precision);
 *   SPH_TUNE_CELL_SCALE cell edge = max(cell_min, scale * 2 h_max), scale in
 *                      permille, 1000..2000 (precision ignored);
 *   SPH_TUNE_BUILD_RANGE sorted particles per work-group of the pair-list
 *                      build: 32, 64, 96 or 128 (precision ignored);
 *   SPH_TUNE_SWEEP_DEPTH neighbour records in flight per lane of the fused
 *                      gradient + force sweep of sph_step: 1 or 2 (per
 *                      precision; 2 hides more latency, 1 needs fewer
 *                      registers and so runs more waves per SIMD; default
 *                      2 in the FP32 form, 1 in the FP64 form);
 *   SPH_TUNE_BUILD_TILE candidates held in the local-memory tile of the
 *                      pair-list build: 128, 192 or 256 (precision ignored;
 *                      a smaller tile lets more work-groups share a CU). */
enum {
    SPH_TUNE_LANES_DENSITY = 0,   /* density sweep                         */
    SPH_TUNE_LANES_GRADIENTS = 1, /* public gradient pass                  */
    SPH_TUNE_LANES_FORCES = 2,    /* public force pass                     */
    SPH_TUNE_LANES_STEP = 3,      /* fused gradient + force sweep of sph_step */
    SPH_TUNE_CELL_SCALE = 4,
    SPH_TUNE_BUILD_RANGE = 5,
    SPH_TUNE_SWEEP_DEPTH = 6,
    SPH_TUNE_BUILD_TILE = 7,
    SPH_TUNE_COUNT = 8
};
sph_status sph_set_tuning(sph_ctx *ctx, int32_t knob, sph_precision prec, int32_t value);
sph_status sph_get_tuning(sph_ctx *ctx, int32_t knob, sph_precision prec, int32_t *value);

#ifdef __cplusplus
}
#endif
#endif /* SPH_ABI_H_ */
