/*
 * FP64 CPU oracle for the strength-SPH hot path of
 * "SPH in pkdgrav3 for Shock Physics Simulations. II. Shear Strength"
 * (Meier, Reinhardt, Jutzi, Potter, Stadel; arXiv 2603.19764).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Design rules of this file
 *   - plain C99, every value in IEEE double, built with -ffp-contract=off so
 *     that no expression is fused into an FMA;
 *   - neighbours are found by brute force over all j for every target i
 *     (O(N^2)), with the strict criterion r^2 < H^2 on the FP64 squared
 *     separation ((dx*dx + dy*dy) + dz*dz), dx = x_i - x_j;
 *   - every sum runs over ascending j, so the result does not depend on the
 *     number of OpenMP threads;
 *   - each function names the passage of the paper it writes out.  Where the
 *     paper is silent the reading used is stated at the function.
 *
 * Readings of the paper used here (paper passage in brackets):
 *   K1  kernel support H = 2h for the Wendland C2 kernel [sec. 3, kernel and
 *       neighbour number; Density_estimate eq.].
 *   K2  the self term j = i is part of the density sum and of the sum in the
 *       grad-h term Omega [Density_estimate eq.; Omega eq. of sec. 2.1].
 *   K3  the artificial-viscosity constants alpha, beta, epsilon are inputs
 *       (Paper I holds their values; this paper does not print them).
 *   K4  the hydrodynamic du/dt is the compatible form
 *       du_i/dt|_H = P_i/(Omega_i rho_i^2) sum_j m_j v_ij . grad_i W_ij(h_i);
 *       the paper uses the entropy-conserving scheme of Paper I instead,
 *       whose formula is not in this paper [sec. 2.1 last paragraph].
 *   K5  the rotation term of the stress rate is rot_sign * (R S - S R).
 *       rot_sign = +1 is the objective (co-rotational) Jaumann rate the
 *       paper says it adopts; rot_sign = -1 reproduces the index order as
 *       printed in Deviatoric_Stress_derivative eq. and in the five
 *       component equations, which equals S R - R S [sec. 2.2].
 *   K6  a correction tensor whose inverse is singular (|det| below
 *       1e-12 |C^-1|_F^3, or fewer than 4 neighbours) is replaced by the
 *       identity, and counted [Correction_Tensor eq.; paper silent].
 *   K7  the EOS is Tillotson; temperature is T = T_ref + u / c_v; the sound
 *       speed follows c^2 = (dP/drho)_u + P/rho^2 (dP/du)_rho, floored at
 *       c_min [sec. 2.3 uses EOSlib / M-ANEOS, which are not available].
 *   K7b an EOS given as a table (sec. 2.3 takes P, c and T from M-ANEOS
 *       tables) holds P, c and T at the nodes of a rectangular grid in
 *       (rho, u); between nodes the values are bilinear in (rho, u), rho
 *       and u outside the grid are moved to its edge, and c is floored at
 *       c_min as for Tillotson.
 *   K7c optionally (rho_limit > 0) the cold Tillotson formula is cut to
 *       zero pressure for rho < rho_limit rho0: material expanded that far
 *       carries no tension, the usual treatment of cold expanded states in
 *       Tillotson codes; the blend with the hot branch keeps its form.
 *   K8  the thermal-softening factor is clamped at zero for T >= T_melt,
 *       and strength switched off for a material means Gamma = 0, Y = 0.
 *   K8b a melting temperature given as a table of density (sec. 2.3) is
 *       interpolated piecewise-linearly and held at its end values.
 *   H1  adaptive smoothing length: the constant kernel mass of the
 *       kernel-mass equation (sec. 2.1) is written N_ngb m_i with N_ngb a
 *       run parameter; Newton-Raphson steps limited to a factor 2.
 *   K9  time integration: kick-drift-kick with the predictor of Predict_S
 *       eq. applied to v, u and S; the closing kick is followed by the
 *       plastic rescaling, the opening kick is not [sec. 2.4].  A particle's
 *       step is the smaller of the CFL step (courant_condition eq.) and,
 *       with eta_a > 0, the acceleration criterion eta_a sqrt(h_i/|a_i|)
 *       (reading T2: the length in that criterion is h_i).  Without rungs
 *       the particles share one step, the minimum over them.
 *   T1  hierarchical individual steps [sec. 2.4 defers the scheme to Paper
 *       I]: particle steps are dt0 2^-r, r = 0 .. rungs-1, dt0 the base
 *       step; a particle takes the longest of these not above its own step,
 *       and may lengthen it only at a time that is a multiple of the new
 *       step.  The simulation advances to the next end of any particle's
 *       step; every particle drifts, and is predicted to that time from the
 *       start of its own step with its last derivatives (v, u and S as in
 *       the predictor above, with the time elapsed in its step in place of
 *       half a step).  Density, EOS, yield and the rescaled predicted stress
 *       are evaluated for all particles (they are the neighbour values);
 *       gradients, stress rates and forces, the closing kick and the new
 *       step for the particles whose step ends there, followed by their
 *       opening kick.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ----------------------------------------------------------------------- */
/* Parameter blocks (own definitions; the GPU library has its own).        */
/* ----------------------------------------------------------------------- */
typedef struct {
    /* Tillotson EOS */
    double rho0, A, B, E0, Eiv, Ecv, a, b, alpha, beta;
    /* temperature model and sound-speed floor */
    double cv, T_ref, c_min;
    /* shear modulus: > 0 constant, otherwise Poisson route with nu */
    double shear_modulus, nu;
    /* Collins yield and thermal softening */
    double Y0, Ym, mu_i, mu_d, xi, T_melt;
    int32_t strength_on, thermal_softening_on;
    /* melting temperature as a table of density (reading K8b): used when
     * tmelt_n >= 2, nodes in ascending density */
    int32_t tmelt_n, tmelt_pad;
    double tmelt_rho[8], tmelt_T[8];
    /* tabulated EOS (reading K7b): used when eos_nrho >= 2 and eos_nu >= 2;
     * grid eos_rho x eos_u (ascending), values [i_rho * eos_nu + i_u] */
    int32_t eos_nrho, eos_nu;
    const double *eos_rho, *eos_u, *eos_P, *eos_c, *eos_T;
    /* Tillotson: the cold formula gives no pressure below rho_limit rho0
     * (reading K7c; 0 keeps the tension of the formula) */
    double rho_limit;
} or_material;

typedef struct {
    double av_alpha, av_beta, av_eps, eta_C, rot_sign;
    double g[3];
    double box[3];          /* periodic box lengths; 0 = open along that axis */
    int32_t use_correction; /* 1: G = F C, 0: G = F                            */
    int32_t omega_one;      /* 1: Omega = 1; 0: Omega as defined               */
    double adapt_ngb;       /* > 0: adapt h to this kernel mass / m each step   */
    double adapt_skin;      /* cap of one adaptation: h <= adapt_skin * h_old   */
    double eta_a;           /* > 0: acceleration criterion eta_a sqrt(h/|a|)    */
    int32_t rungs;          /* > 0: individual steps dt0 2^-r, r < rungs (T1)  */
    int32_t rungs_pad;
} or_params;

/* ----------------------------------------------------------------------- */
/* Wendland C2 kernel in 3D, support H = 2h (reading K1).                  */
/*   W(r,h)      = 21/(2 pi H^3) (1-q)^4 (1+4q),  q = r/H < 1               */
/*   grad_i W    = K(r,h) x_ij,  K = -210/(pi H^5) (1-q)^3                  */
/*   dW/dh       = -21/(pi H^4) (1-q)^3 (3 + 9q - 32 q^2)                   */
/* ----------------------------------------------------------------------- */
double or_W(double r, double h)
{
    double H = 2.0 * h;
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    return 21.0 / (2.0 * OR_PI * H * H * H) * (t * t * t * t) * (1.0 + 4.0 * q);
}

double or_K(double r, double h)
{
    double H = 2.0 * h;
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    return -210.0 / (OR_PI * H * H * H * H * H) * (t * t * t);
}

double or_dWdh(double r, double h)
{
    double H = 2.0 * h;
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    return -21.0 / (OR_PI * H * H * H * H) * (t * t * t) * (3.0 + 9.0 * q - 32.0 * q * q);
}

/* Squared separation of i and j with dx = x_i - x_j (minimum image along
 * periodic axes), summed as ((dx*dx + dy*dy) + dz*dz). */
static double sep2(const double *x, const double *y, const double *z,
                   int64_t i, int64_t j, const double *box, double d[3])
{
    double dx = x[i] - x[j];
    double dy = y[i] - y[j];
    double dz = z[i] - z[j];
    if (box[0] > 0.0) dx -= box[0] * nearbyint(dx / box[0]);
    if (box[1] > 0.0) dy -= box[1] * nearbyint(dy / box[1]);
    if (box[2] > 0.0) dz -= box[2] * nearbyint(dz / box[2]);
    d[0] = dx; d[1] = dy; d[2] = dz;
    return dx * dx + dy * dy + dz * dz;
}

static double supp2(double h) { double H = 2.0 * h; return H * H; }

/* ----------------------------------------------------------------------- */
/* Neighbour sets by brute force.                                          */
/*   density set  D_i = { j != i : r^2 < H_i^2 }  (plus the self term)      */
/*   pair set     N_i = { j != i : r^2 < max(H_i^2, H_j^2) }                */
/* The pair set is the set over which both kernels W(h_i), W(h_j) of the   */
/* symmetrised sums (acceleration eq., Velocity_Gradient eq.) may be       */
/* non-zero.                                                                */
/* ----------------------------------------------------------------------- */

/* Count |N_i| for every target. */
void or_pair_counts(int64_t n, const double *x, const double *y, const double *z,
                    const double *h, const or_params *p,
                    int64_t nt, const int64_t *tar, int64_t *cnt)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double Hi2 = supp2(h[i]);
        int64_t c = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (r2 < (Hi2 > Hj2 ? Hi2 : Hj2)) ++c;
        }
        cnt[k] = c;
    }
}

/* Fill the pair lists (CSR rows given by off[k]..off[k+1]) in ascending j,
 * with dflag = 1 when j is also in the density set of i. */
void or_pair_lists(int64_t n, const double *x, const double *y, const double *z,
                   const double *h, const or_params *p,
                   int64_t nt, const int64_t *tar, const int64_t *off,
                   int64_t *nbr, uint8_t *dflag)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double Hi2 = supp2(h[i]);
        int64_t c = off[k];
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (r2 < (Hi2 > Hj2 ? Hi2 : Hj2)) {
                nbr[c] = j;
                dflag[c] = (uint8_t)(r2 < Hi2);
                ++c;
            }
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Density and grad-h term (sec. 2.1, Density_estimate eq. and the Omega   */
/* eq. that follows it):                                                   */
/*   rho_i   = sum_j m_j W(r_ij, h_i)                                      */
/*   Omega_i = 1 + h_i/(3 rho_i) sum_j m_j dW(r_ij, h_i)/dh_i              */
/* The sums run over j in D_i and the self term j = i (reading K2).  When  */
/* D_i holds no particle but i, Omega as defined vanishes (the self term's  */
/* dW/dh cancels the 1): such a particle takes Omega = 1 (reading K2b).    */
/* ----------------------------------------------------------------------- */
void or_density(int64_t n, const double *x, const double *y, const double *z,
                const double *m, const double *h, const or_params *p,
                int64_t nt, const int64_t *tar, double *rho, double *omega)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double Hi2 = supp2(h[i]);
        double sum_w = 0.0, sum_dh = 0.0;
        int64_t others = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            double r;
            if (j == i) {
                r = 0.0;
            } else {
                double r2 = sep2(x, y, z, i, j, p->box, d);
                if (!(r2 < Hi2)) continue;
                r = sqrt(r2);
                ++others;
            }
            sum_w += m[j] * or_W(r, h[i]);
            sum_dh += m[j] * or_dWdh(r, h[i]);
        }
        rho[i] = sum_w;
        omega[i] = (p->omega_one || others == 0) ? 1.0
                                                 : 1.0 + h[i] / (3.0 * sum_w) * sum_dh;
    }
}

/* ----------------------------------------------------------------------- */
/* Adaptive smoothing length (sec. 2.1, the kernel-mass equation): h_i is   */
/* chosen so that the mass inside the kernel support stays constant,       */
/*    (4/3) pi (2 h_i)^3 rho_i(h_i) = N_ngb m_i,                           */
/* solved by Newton-Raphson with the density and its h-derivative:          */
/*    f(h)  = (32 pi / 3) h^3 rho(h) - N_ngb m_i,                           */
/*    f'(h) = 32 pi h^2 rho(h) + (32 pi / 3) h^3 drho/dh                    */
/*          = 32 pi h^2 rho Omega.                                          */
/* Each Newton step is limited to a factor of 2 either way; the iteration   */
/* stops when |dh| <= tol h or after max_iter steps (reading H1: the target  */
/* mass is written N_ngb m_i, N_ngb a run parameter).  With a cap h_cap_i    */
/* (the length a neighbour search covered), a step past the cap is held at   */
/* it, and a particle whose next step would leave it again stops there.     */
/* Fixed particles (fixed[i] != 0) keep h_in.  Returns the largest number   */
/* of steps any particle took.                                              */
/* ----------------------------------------------------------------------- */
int32_t or_adapt_h(int64_t n, const double *x, const double *y, const double *z,
                   const double *m, const double *h_in, const double *h_cap,
                   const uint8_t *fixed, const or_params *p, double n_ngb, double tol,
                   int32_t max_iter, double *h_out)
{
    int32_t worst = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(max:worst)
    for (int64_t i = 0; i < n; ++i) {
        double h = h_cap ? fmin(h_in[i], h_cap[i]) : h_in[i];
        int32_t it = 0;
        if (fixed && fixed[i]) {
            h_out[i] = h_in[i];
            continue;
        }
        for (; it < max_iter; ++it) {
            const double H2 = supp2(h);
            double rho = 0.0, drho = 0.0, d[3];
            for (int64_t j = 0; j < n; ++j) {
                double r;
                if (j == i) {
                    r = 0.0;
                } else {
                    double r2 = sep2(x, y, z, i, j, p->box, d);
                    if (!(r2 < H2)) continue;
                    r = sqrt(r2);
                }
                rho += m[j] * or_W(r, h);
                drho += m[j] * or_dWdh(r, h);
            }
            const double f = (32.0 * OR_PI / 3.0) * h * h * h * rho - n_ngb * m[i];
            const double fp = 32.0 * OR_PI * h * h * rho + (32.0 * OR_PI / 3.0) * h * h * h * drho;
            double hn = fp > 0.0 ? h - f / fp : 2.0 * h;
            if (hn > 2.0 * h) hn = 2.0 * h;
            if (hn < 0.5 * h) hn = 0.5 * h;
            if (h_cap && hn > h_cap[i]) {
                if (h == h_cap[i]) {
                    ++it;
                    break;
                }
                hn = h_cap[i];
            }
            const double dh = hn - h;
            h = hn;
            if (fabs(dh) <= tol * h) {
                ++it;
                break;
            }
        }
        h_out[i] = h;
        if (it > worst) worst = it;
    }
    return worst;
}

/* ----------------------------------------------------------------------- */
/* Tillotson equation of state (reading K7).                               */
/*   eta = rho/rho0, mu = eta - 1, w = u/(E0 eta^2) + 1, z = 1/eta - 1      */
/*   compressed or cold (eta >= 1 or u <= Eiv):                             */
/*      Pc = (a + b/w) rho u + A mu + B mu^2                                */
/*   hot expanded (eta < 1 and u >= Ecv):                                   */
/*      Pe = a rho u + (b rho u / w + A mu exp(-beta z)) exp(-alpha z^2)    */
/*   otherwise the linear blend in u of Pe and Pc.                          */
/*   Pc = 0 (with zero derivatives) for eta < rho_limit (reading K7c).      */
/* Sound speed from the partial derivatives of the active branch.           */
/* ----------------------------------------------------------------------- */
static void till_compressed(const or_material *M, double rho, double u,
                            double *P, double *dPdrho, double *dPdu)
{
    double eta = rho / M->rho0;
    if (eta < M->rho_limit) {
        *P = 0.0;
        *dPdrho = 0.0;
        *dPdu = 0.0;
        return;
    }
    double mu = eta - 1.0;
    double w = u / (M->E0 * eta * eta) + 1.0;
    *P = (M->a + M->b / w) * rho * u + M->A * mu + M->B * mu * mu;
    /* dw/drho = -2 (w-1)/rho,  dw/du = (w-1)/u = 1/(E0 eta^2) */
    *dPdrho = M->a * u + M->b * u / w + 2.0 * M->b * u * (w - 1.0) / (w * w)
            + (M->A + 2.0 * M->B * mu) / M->rho0;
    *dPdu = M->a * rho + M->b * rho / w
          - M->b * rho * u / (w * w) / (M->E0 * eta * eta);
}

static void till_expanded(const or_material *M, double rho, double u,
                          double *P, double *dPdrho, double *dPdu)
{
    double eta = rho / M->rho0;
    double mu = eta - 1.0;
    double w = u / (M->E0 * eta * eta) + 1.0;
    double z = 1.0 / eta - 1.0;
    double eb = exp(-M->beta * z);
    double ea = exp(-M->alpha * z * z);
    double brace = M->b * rho * u / w + M->A * mu * eb;
    *P = M->a * rho * u + brace * ea;
    /* dz/drho = -rho0/rho^2 */
    double dz = -M->rho0 / (rho * rho);
    double dbrace = M->b * u / w + 2.0 * M->b * u * (w - 1.0) / (w * w)
                  + M->A / M->rho0 * eb + M->A * mu * eb * (-M->beta) * dz;
    *dPdrho = M->a * u + dbrace * ea + brace * ea * (-2.0 * M->alpha * z) * dz;
    *dPdu = M->a * rho + ea * (M->b * rho / w
          - M->b * rho * u / (w * w) / (M->E0 * eta * eta));
}

void or_tillotson(const or_material *M, double rho, double u,
                  double *P_out, double *c_out, double *dPdrho_out, double *dPdu_out)
{
    double eta = rho / M->rho0;
    double P, dPdrho, dPdu;
    if (eta >= 1.0 || u <= M->Eiv) {
        till_compressed(M, rho, u, &P, &dPdrho, &dPdu);
    } else if (u >= M->Ecv) {
        till_expanded(M, rho, u, &P, &dPdrho, &dPdu);
    } else {
        double Pc, Pe, dc_r, de_r, dc_u, de_u;
        till_compressed(M, rho, u, &Pc, &dc_r, &dc_u);
        till_expanded(M, rho, u, &Pe, &de_r, &de_u);
        double span = M->Ecv - M->Eiv;
        P = ((u - M->Eiv) * Pe + (M->Ecv - u) * Pc) / span;
        dPdrho = ((u - M->Eiv) * de_r + (M->Ecv - u) * dc_r) / span;
        dPdu = ((u - M->Eiv) * de_u + Pe + (M->Ecv - u) * dc_u - Pc) / span;
    }
    double c2 = dPdrho + P / (rho * rho) * dPdu;
    double c = c2 > 0.0 ? sqrt(c2) : 0.0;
    if (c < M->c_min) c = M->c_min;
    *P_out = P;
    *c_out = c;
    if (dPdrho_out) *dPdrho_out = dPdrho;
    if (dPdu_out) *dPdu_out = dPdu;
}

/* ----------------------------------------------------------------------- */
/* Yield strength (sec. 2.3):                                               */
/*   Y_i = Y0 + mu_i P / (1 + mu_i P / (Ym - Y0))   intact, P clipped >= 0  */
/*   Y_d = mu_d P                                    damaged                */
/*   Y   = min(Y_i, Y_d)                                                    */
/*   Y  <- Y tanh(xi (T_melt/T - 1))                 thermal softening      */
/* T_melt is the material constant, or, with a table (sec. 2.3: T_melt as a */
/* tabulated function of density), the piecewise-linear interpolation of   */
/* the table at rho, held at the end values outside it (reading K8b).       */
/* ----------------------------------------------------------------------- */
double or_tmelt(const or_material *M, double rho)
{
    if (M->tmelt_n < 2) return M->T_melt;
    const int n = M->tmelt_n;
    if (rho <= M->tmelt_rho[0]) return M->tmelt_T[0];
    if (rho >= M->tmelt_rho[n - 1]) return M->tmelt_T[n - 1];
    int k = 0;
    while (rho >= M->tmelt_rho[k + 1]) ++k;
    const double w = (rho - M->tmelt_rho[k]) / (M->tmelt_rho[k + 1] - M->tmelt_rho[k]);
    return M->tmelt_T[k] + w * (M->tmelt_T[k + 1] - M->tmelt_T[k]);
}

double or_yield(const or_material *M, double rho, double P, double T)
{
    if (!M->strength_on) return 0.0;
    double Pp = P > 0.0 ? P : 0.0;
    double Yi = M->Y0 + M->mu_i * Pp / (1.0 + M->mu_i * Pp / (M->Ym - M->Y0));
    double Yd = M->mu_d * Pp;
    double Y = Yi < Yd ? Yi : Yd;
    if (M->thermal_softening_on) {
        double s = tanh(M->xi * (or_tmelt(M, rho) / T - 1.0));
        Y *= (s > 0.0 ? s : 0.0);            /* reading K8 */
    }
    return Y;
}

/* Shear modulus (sec. 2.2): constant, or Gamma = 3(1-2nu)/(2(1+nu)) K with
 * K = rho c^2. */
double or_shear_modulus(const or_material *M, double rho, double c)
{
    if (!M->strength_on) return 0.0;
    if (M->shear_modulus > 0.0) return M->shear_modulus;
    double K = rho * c * c;
    return 3.0 * (1.0 - 2.0 * M->nu) / (2.0 * (1.0 + M->nu)) * K;
}

/* ----------------------------------------------------------------------- */
/* Tabulated EOS (reading K7b).  The cell is the one whose lower node is   */
/* the last node not above the (clamped) coordinate, so a coordinate on an */
/* interior node takes the cell above it; the top node belongs to the last */
/* cell.  Within the cell, with weights w_r, w_u in [0, 1]:                 */
/*   f = f0 + w_r (f1 - f0),  f0 = f00 + w_u (f01 - f00),                   */
/*                            f1 = f10 + w_u (f11 - f10),                   */
/* the bilinear interpolant of the four corner values.                      */
/* ----------------------------------------------------------------------- */
static int table_cell(const double *node, int n, double *x)
{
    if (*x < node[0]) *x = node[0];
    if (*x > node[n - 1]) *x = node[n - 1];
    int k = 0;
    while (k + 2 < n && *x >= node[k + 1]) ++k;
    return k;
}

static double bilinear(const double *f, int nu, int kr, int ku, double wr, double wu)
{
    const double f00 = f[kr * nu + ku], f01 = f[kr * nu + ku + 1];
    const double f10 = f[(kr + 1) * nu + ku], f11 = f[(kr + 1) * nu + ku + 1];
    const double f0 = f00 + wu * (f01 - f00);
    const double f1 = f10 + wu * (f11 - f10);
    return f0 + wr * (f1 - f0);
}

void or_eos_table(const or_material *M, double rho, double u, double *P, double *c, double *T)
{
    const int nr = M->eos_nrho, nu = M->eos_nu;
    double r = rho, e = u;
    const int kr = table_cell(M->eos_rho, nr, &r);
    const int ku = table_cell(M->eos_u, nu, &e);
    const double wr = (r - M->eos_rho[kr]) / (M->eos_rho[kr + 1] - M->eos_rho[kr]);
    const double wu = (e - M->eos_u[ku]) / (M->eos_u[ku + 1] - M->eos_u[ku]);
    *P = bilinear(M->eos_P, nu, kr, ku, wr, wu);
    double cc = bilinear(M->eos_c, nu, kr, ku, wr, wu);
    *c = cc < M->c_min ? M->c_min : cc;
    *T = bilinear(M->eos_T, nu, kr, ku, wr, wu);
}

/* P, c and T of one particle: the table when the material has one, else
 * Tillotson with T = T_ref + u / c_v (reading K7). */
void or_eos(const or_material *M, double rho, double u, double *P, double *c, double *T)
{
    if (M->eos_nrho >= 2 && M->eos_nu >= 2) {
        or_eos_table(M, rho, u, P, c, T);
        return;
    }
    or_tillotson(M, rho, u, P, c, NULL, NULL);
    *T = M->T_ref + u / M->cv;
}

/* Per-particle state after the density: P, c, T, Y, Gamma. */
void or_state(int64_t nt, const int64_t *tar, const double *rho, const double *u,
              const int32_t *mat, const or_material *mats,
              double *P, double *c, double *T, double *Y, double *Gam)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        const or_material *M = &mats[mat[i]];
        double Pi, ci, Ti;
        or_eos(M, rho[i], u[i], &Pi, &ci, &Ti);
        P[i] = Pi;
        c[i] = ci;
        T[i] = Ti;
        Y[i] = or_yield(M, rho[i], Pi, Ti);
        Gam[i] = or_shear_modulus(M, rho[i], ci);
    }
}

/* ----------------------------------------------------------------------- */
/* Deviatoric stress: 5 stored components (xx, yy, xy, xz, yz), with       */
/* S_zz = -S_xx - S_yy (sec. 2.2, matrix form of the stress tensor).       */
/* ----------------------------------------------------------------------- */
static void S_full(const double s5[5], double S[3][3])
{
    S[0][0] = s5[0]; S[1][1] = s5[1]; S[2][2] = -s5[0] - s5[1];
    S[0][1] = S[1][0] = s5[2];
    S[0][2] = S[2][0] = s5[3];
    S[1][2] = S[2][1] = s5[4];
}

/* J2 = 1/2 S:S over the full tensor (sec. 2.3). */
double or_J2(const double s5[5])
{
    double S[3][3];
    S_full(s5, S);
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            ss += S[a][b] * S[a][b];
    return 0.5 * ss;
}

/* Plastic rescaling S -> f S, f = min(Y / sqrt(J2), 1) (sec. 2.3,
 * Deviatoric_stress_rescaling eq.).  Operates on one particle. */
void or_plastic_return(double s5[5], double Y)
{
    double J2 = or_J2(s5);
    if (J2 > 0.0) {
        double f = Y / sqrt(J2);
        if (f < 1.0)
            for (int k = 0; k < 5; ++k) s5[k] *= f;
    }
}

/* Array form: S is component-major (5 rows of length n). */
void or_plastic_return_all(int64_t n, int64_t nt, const int64_t *tar, double *S,
                           const double *Y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double s5[5];
        for (int c = 0; c < 5; ++c) s5[c] = S[c * n + i];
        or_plastic_return(s5, Y[i]);
        for (int c = 0; c < 5; ++c) S[c * n + i] = s5[c];
    }
}

/* ----------------------------------------------------------------------- */
/* Velocity gradient with correction tensor (sec. 2.2,                     */
/* Velocity_Gradient, Correction_Tensor and Corrected_Gradients eqs.):     */
/*   F^ab    = -1/2 sum_j m_j v_ij^a (d_b W_ij(h_i)/(Om_i rho_i)            */
/*                                  + d_b W_ij(h_j)/(Om_j rho_j))           */
/*   (C^-1)^ab = the same sum with x_ij^a in place of v_ij^a                */
/*   G^ab    = F^ag C^gb                                                    */
/* with d_b W_ij(h) = K(r,h) x_ij^b.  G, Cinv and F are 9 rows of length n  */
/* (row-major component index 3a+b).                                        */
/* ----------------------------------------------------------------------- */
static int inverse3(const double A[3][3], double Ainv[3][3], double *det_out)
{
    double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    *det_out = det;
    if (det == 0.0) return 0;
    double id = 1.0 / det;
    Ainv[0][0] = c00 * id;
    Ainv[1][0] = c01 * id;
    Ainv[2][0] = c02 * id;
    Ainv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    Ainv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    Ainv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    Ainv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    Ainv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    Ainv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return 1;
}

void or_gradients(int64_t n, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz,
                  const double *m, const double *h, const double *rho,
                  const double *omega, const or_params *p,
                  int64_t nt, const int64_t *tar,
                  double *G, double *Cinv_out, double *F_out, int64_t *n_singular)
{
    int64_t nsing = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:nsing)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double F[3][3] = {{0}}, Ci[3][3] = {{0}};
        double Hi2 = supp2(h[i]);
        double wi = 1.0 / (omega[i] * rho[i]);
        int64_t cnt = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (!(r2 < (Hi2 > Hj2 ? Hi2 : Hj2))) continue;
            ++cnt;
            double r = sqrt(r2);
            double Ki = or_K(r, h[i]);
            double Kj = or_K(r, h[j]);
            double wj = 1.0 / (omega[j] * rho[j]);
            double v[3] = { vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j] };
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) {
                    double gw = Ki * d[b] * wi + Kj * d[b] * wj;
                    F[a][b] -= 0.5 * m[j] * v[a] * gw;
                    Ci[a][b] -= 0.5 * m[j] * d[a] * gw;
                }
            }
        }
        double C[3][3];
        int ok = 0;
        if (p->use_correction) {
            double fro = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) fro += Ci[a][b] * Ci[a][b];
            fro = sqrt(fro);
            double det;
            ok = inverse3(Ci, C, &det);
            if (!ok || cnt < 4 || fabs(det) < 1e-12 * fro * fro * fro) ok = 0;
            if (!ok) ++nsing;                                 /* reading K6 */
        }
        if (!ok) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) C[a][b] = (a == b) ? 1.0 : 0.0;
        }
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) {
                double g = 0.0;
                for (int c = 0; c < 3; ++c) g += F[a][c] * C[c][b];
                G[(3 * a + b) * n + i] = g;
                if (Cinv_out) Cinv_out[(3 * a + b) * n + i] = Ci[a][b];
                if (F_out) F_out[(3 * a + b) * n + i] = F[a][b];
            }
        }
    }
    if (n_singular) *n_singular = nsing;
}

/* ----------------------------------------------------------------------- */
/* Stress rate, tensor form (sec. 2.2, Deviatoric_Stress_derivative eq.,   */
/* Strain_rate_tensor and Rotation_rate_tensor from G):                     */
/*   eps = (G + G^T)/2,  R = (G - G^T)/2                                    */
/*   dS  = 2 Gamma (eps - tr(eps)/3 I) + rot_sign (R S - S R)   (K5)        */
/* Also returns the rate of the strain-rate invariant 1/2 eps:eps (end of   */
/* sec. 2.4).                                                               */
/* ----------------------------------------------------------------------- */
void or_stress_rate_one(const double G9[9], const double s5[5], double Gam,
                        double rot_sign, double ds5[5], double *eps2_rate)
{
    double S[3][3], E[3][3], R[3][3], D[3][3];
    S_full(s5, S);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            E[a][b] = 0.5 * (G9[3 * a + b] + G9[3 * b + a]);
            R[a][b] = 0.5 * (G9[3 * a + b] - G9[3 * b + a]);
        }
    double tr = E[0][0] + E[1][1] + E[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double rs = 0.0, sr = 0.0;
            for (int c = 0; c < 3; ++c) {
                rs += R[a][c] * S[c][b];
                sr += S[a][c] * R[c][b];
            }
            D[a][b] = 2.0 * Gam * (E[a][b] - (a == b ? tr / 3.0 : 0.0))
                    + rot_sign * (rs - sr);
        }
    ds5[0] = D[0][0]; ds5[1] = D[1][1]; ds5[2] = D[0][1]; ds5[3] = D[0][2]; ds5[4] = D[1][2];
    if (eps2_rate) {
        double ee = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) ee += E[a][b] * E[a][b];
        *eps2_rate = 0.5 * ee;
    }
}

/* The five component equations as printed at the end of sec. 2.2, written
 * out term by term.  Used by tests only, to show that they equal the tensor
 * form with rot_sign = -1. */
void or_stress_rate_printed(const double G9[9], const double s5[5], double Gam, double ds5[5])
{
#define GG(a, b) G9[3 * (a) + (b)]
    const int X = 0, Y = 1, Z = 2;
    double Sxx = s5[0], Syy = s5[1], Sxy = s5[2], Sxz = s5[3], Syz = s5[4];
    ds5[0] = Sxy * (GG(Y, X) - GG(X, Y)) + Sxz * (GG(Z, X) - GG(X, Z))
           - 2.0 / 3.0 * Gam * (GG(Y, Y) + GG(Z, Z) - 2.0 * GG(X, X));
    ds5[1] = Sxy * (GG(X, Y) - GG(Y, X)) + Syz * (GG(Z, Y) - GG(Y, Z))
           - 2.0 / 3.0 * Gam * (GG(X, X) + GG(Z, Z) - 2.0 * GG(Y, Y));
    ds5[2] = Gam * (GG(X, Y) + GG(Y, X))
           + 0.5 * (Sxx * (GG(X, Y) - GG(Y, X)) + Syy * (GG(Y, X) - GG(X, Y))
                    + Syz * (GG(Z, X) - GG(X, Z)) + Sxz * (GG(Z, Y) - GG(Y, Z)));
    ds5[3] = Gam * (GG(X, Z) + GG(Z, X))
           + 0.5 * ((Sxx + Syy) * (GG(X, Z) - GG(Z, X)) + Sxx * (GG(X, Z) - GG(Z, X))
                    + Syz * (GG(Y, X) - GG(X, Y)) + Sxy * (GG(Y, Z) - GG(Z, Y)));
    ds5[4] = Gam * (GG(Y, Z) + GG(Z, Y))
           + 0.5 * ((Sxx + Syy) * (GG(Y, Z) - GG(Z, Y)) + Sxz * (GG(X, Y) - GG(Y, X))
                    + Sxy * (GG(X, Z) - GG(Z, X)) + Syy * (GG(Y, Z) - GG(Z, Y)));
#undef GG
}

/* Array form of the tensor stress rate. */
void or_stress_rate(int64_t n, int64_t nt, const int64_t *tar, const double *G,
                    const double *S, const double *Gam, double rot_sign,
                    double *dS, double *eps2_rate)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double g9[9], s5[5], d5[5], e2;
        for (int c = 0; c < 9; ++c) g9[c] = G[c * n + i];
        for (int c = 0; c < 5; ++c) s5[c] = S[c * n + i];
        or_stress_rate_one(g9, s5, Gam[i], rot_sign, d5, &e2);
        for (int c = 0; c < 5; ++c) dS[c * n + i] = d5[c];
        if (eps2_rate) eps2_rate[i] = e2;
    }
}

/* ----------------------------------------------------------------------- */
/* Accelerations, internal-energy rate and CFL time step (sec. 2.1 and     */
/* 2.2: hydrodynamic acceleration, artificial viscosity Pi_ij with mu_ij,  */
/* AV_heating eq., the strength terms of the acceleration and energy       */
/* equations, and courant_condition eq. of sec. 2.4):                      */
/*  dv_i/dt = - sum_j m_j [P_i/(Om_i rho_i^2) dW(h_i) + P_j/(..)_j dW(h_j)] */
/*            - sum_j m_j Pi_ij dWbar                                       */
/*            + sum_j m_j [S_i/(Om_i rho_i^2) . dW(h_i) + S_j/(..)_j . dW(h_j)]*/
/*            + g                                                            */
/*  du_i/dt = P_i/(Om_i rho_i^2) sum_j m_j v_ij . dW(h_i)       (K4)         */
/*            + 1/2 sum_j m_j Pi_ij v_ij . dWbar                             */
/*            - S_i/(Om_i rho_i^2) : sum_j m_j v_ij (x) dW(h_i)              */
/*  dt_i    = eta_C min_j h_i / ((1 + 0.6 alpha) c_i + 0.6 beta |min(0,mu_ij)|)*/
/* AV acts only when v_ij . x_ij < 0; bars are arithmetic means of i and j. */
/* ----------------------------------------------------------------------- */
void or_forces(int64_t n, const double *x, const double *y, const double *z,
               const double *vx, const double *vy, const double *vz,
               const double *m, const double *h, const double *rho,
               const double *omega, const double *P, const double *cs,
               const double *S, const or_params *p,
               int64_t nt, const int64_t *tar,
               double *ax, double *ay, double *az, double *dudt, double *dt)
{
    const double al = p->av_alpha, be = p->av_beta, eps = p->av_eps;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double Si[3][3], s5[5];
        for (int c = 0; c < 5; ++c) s5[c] = S[c * n + i];
        S_full(s5, Si);
        double Hi2 = supp2(h[i]);
        double oi = omega[i] * rho[i] * rho[i];
        double acc_H[3] = {0, 0, 0}, acc_S[3] = {0, 0, 0}, acc_V[3] = {0, 0, 0};
        double du_H = 0.0, du_S = 0.0, du_V = 0.0;
        double denom_max = (1.0 + 0.6 * al) * cs[i];
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (!(r2 < (Hi2 > Hj2 ? Hi2 : Hj2))) continue;
            double r = sqrt(r2);
            double Ki = or_K(r, h[i]);
            double Kj = or_K(r, h[j]);
            double oj = omega[j] * rho[j] * rho[j];
            double Sj[3][3], t5[5];
            for (int c = 0; c < 5; ++c) t5[c] = S[c * n + j];
            S_full(t5, Sj);
            double v[3] = { vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j] };
            double dWi[3] = { Ki * d[0], Ki * d[1], Ki * d[2] };
            double dWj[3] = { Kj * d[0], Kj * d[1], Kj * d[2] };
            /* hydrodynamic pressure term */
            for (int a = 0; a < 3; ++a)
                acc_H[a] -= m[j] * (P[i] / oi * dWi[a] + P[j] / oj * dWj[a]);
            /* deviatoric stress term */
            for (int a = 0; a < 3; ++a) {
                double sum = 0.0;
                for (int b = 0; b < 3; ++b)
                    sum += Si[a][b] / oi * dWi[b] + Sj[a][b] / oj * dWj[b];
                acc_S[a] += m[j] * sum;
            }
            /* energy: compatible hydro part and strength part, kernel h_i */
            double vdw = v[0] * dWi[0] + v[1] * dWi[1] + v[2] * dWi[2];
            du_H += P[i] / oi * m[j] * vdw;
            {
                double ss = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        ss += Si[a][b] / oi * m[j] * v[a] * dWi[b];
                du_S -= ss;
            }
            /* artificial viscosity */
            double vr = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
            double hb = 0.5 * (h[i] + h[j]);
            double mu = hb * vr / (r2 + eps * hb * hb);
            if (vr < 0.0) {
                double cb = 0.5 * (cs[i] + cs[j]);
                double rb = 0.5 * (rho[i] + rho[j]);
                double Pi = (-al * cb * mu + be * mu * mu) / rb;
                double dWb[3];
                for (int a = 0; a < 3; ++a) dWb[a] = 0.5 * (dWi[a] + dWj[a]);
                for (int a = 0; a < 3; ++a) acc_V[a] -= m[j] * Pi * dWb[a];
                du_V += 0.5 * m[j] * Pi * (v[0] * dWb[0] + v[1] * dWb[1] + v[2] * dWb[2]);
            }
            double mneg = mu < 0.0 ? -mu : 0.0;
            double den = (1.0 + 0.6 * al) * cs[i] + 0.6 * be * mneg;
            if (den > denom_max) denom_max = den;
        }
        ax[i] = acc_H[0] + acc_S[0] + acc_V[0] + p->g[0];
        ay[i] = acc_H[1] + acc_S[1] + acc_V[1] + p->g[1];
        az[i] = acc_H[2] + acc_S[2] + acc_V[2] + p->g[2];
        dudt[i] = du_H + du_S + du_V;
        dt[i] = p->eta_C * h[i] / denom_max;
    }
}

/* ----------------------------------------------------------------------- */
/* Scales of the pair sums, for per-particle error metrics: for each target */
/* the sum over its pair set of the magnitude of each pair's contribution   */
/* to the result,                                                           */
/*   sa_i  = sum_j | m_j [-(P_i/o_i dW_i + P_j/o_j dW_j)                    */
/*                        + (S_i/o_i dW_i + S_j/o_j dW_j)] - m_j Pi dWbar | */
/*   sdu_i = sum_j | P_i/o_i m_j v.dW_i - S_i/o_i : m_j v (x) dW_i          */
/*                   + 1/2 m_j Pi v.dWbar |                                 */
/*   sG_i  = sum_j | g_ij |_F,  g_ij = -1/2 m_j v (x) gw_ij C_i, the pair's */
/*           share of G_i = F_i C_i (Velocity_Gradient, Corrected_Gradients)*/
/*   sdS_i = sum_j | dS(g_ij) |, the same share of the stress rate (the     */
/*           rate is linear in G at fixed S; 5 stored components)           */
/* with o = Omega rho^2 and the AV term only for approaching pairs, as in   */
/* or_forces and or_gradients.  Triangle inequality: |a_i - g| <= sa_i etc. */
/* ----------------------------------------------------------------------- */
void or_term_scales(int64_t n, const double *x, const double *y, const double *z,
                    const double *vx, const double *vy, const double *vz,
                    const double *m, const double *h, const double *rho,
                    const double *omega, const double *P, const double *cs,
                    const double *S, const double *Gam, const or_params *p,
                    int64_t nt, const int64_t *tar,
                    double *sa, double *sdu, double *sG, double *sdS)
{
    const double al = p->av_alpha, be = p->av_beta, eps = p->av_eps;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tar[k];
        double Si[3][3], s5[5];
        for (int c = 0; c < 5; ++c) s5[c] = S[c * n + i];
        S_full(s5, Si);
        double Hi2 = supp2(h[i]);
        double oi = omega[i] * rho[i] * rho[i];
        double wi = 1.0 / (omega[i] * rho[i]);
        double d[3];
        /* the correction tensor of i, as in or_gradients */
        double Ci[3][3] = {{0}};
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (!(r2 < (Hi2 > Hj2 ? Hi2 : Hj2))) continue;
            ++cnt;
            double r = sqrt(r2);
            double Ki = or_K(r, h[i]), Kj = or_K(r, h[j]);
            double wj = 1.0 / (omega[j] * rho[j]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    Ci[a][b] -= 0.5 * m[j] * d[a] * (Ki * d[b] * wi + Kj * d[b] * wj);
        }
        double Cm[3][3];
        int ok = 0;
        if (p->use_correction) {
            double fro = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) fro += Ci[a][b] * Ci[a][b];
            fro = sqrt(fro);
            double det;
            ok = inverse3(Ci, Cm, &det);
            if (!ok || cnt < 4 || fabs(det) < 1e-12 * fro * fro * fro) ok = 0;
        }
        if (!ok)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Cm[a][b] = (a == b) ? 1.0 : 0.0;
        double ta = 0.0, tdu = 0.0, tG = 0.0, tdS = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = sep2(x, y, z, i, j, p->box, d);
            double Hj2 = supp2(h[j]);
            if (!(r2 < (Hi2 > Hj2 ? Hi2 : Hj2))) continue;
            double r = sqrt(r2);
            double Ki = or_K(r, h[i]), Kj = or_K(r, h[j]);
            double oj = omega[j] * rho[j] * rho[j];
            double wj = 1.0 / (omega[j] * rho[j]);
            double Sj[3][3], t5[5];
            for (int c = 0; c < 5; ++c) t5[c] = S[c * n + j];
            S_full(t5, Sj);
            double v[3] = { vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j] };
            double dWi[3] = { Ki * d[0], Ki * d[1], Ki * d[2] };
            double dWj[3] = { Kj * d[0], Kj * d[1], Kj * d[2] };
            double ta3[3], tu = 0.0;
            for (int a = 0; a < 3; ++a) {
                double sum = 0.0;
                for (int b = 0; b < 3; ++b)
                    sum += Si[a][b] / oi * dWi[b] + Sj[a][b] / oj * dWj[b];
                ta3[a] = -m[j] * (P[i] / oi * dWi[a] + P[j] / oj * dWj[a]) + m[j] * sum;
            }
            tu += P[i] / oi * m[j] * (v[0] * dWi[0] + v[1] * dWi[1] + v[2] * dWi[2]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) tu -= Si[a][b] / oi * m[j] * v[a] * dWi[b];
            double vr = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
            if (vr < 0.0) {
                double hb = 0.5 * (h[i] + h[j]);
                double mu = hb * vr / (r2 + eps * hb * hb);
                double cb = 0.5 * (cs[i] + cs[j]);
                double rb = 0.5 * (rho[i] + rho[j]);
                double Pi = (-al * cb * mu + be * mu * mu) / rb;
                double dWb[3];
                for (int a = 0; a < 3; ++a) dWb[a] = 0.5 * (dWi[a] + dWj[a]);
                for (int a = 0; a < 3; ++a) ta3[a] -= m[j] * Pi * dWb[a];
                tu += 0.5 * m[j] * Pi * (v[0] * dWb[0] + v[1] * dWb[1] + v[2] * dWb[2]);
            }
            ta += sqrt(ta3[0] * ta3[0] + ta3[1] * ta3[1] + ta3[2] * ta3[2]);
            tdu += fabs(tu);
            /* the pair's share of G: -1/2 m_j v (x) gw, times C */
            double g9[9], gg = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0.0;
                    for (int c = 0; c < 3; ++c)
                        acc += -0.5 * m[j] * v[a] * (Ki * d[c] * wi + Kj * d[c] * wj) * Cm[c][b];
                    g9[3 * a + b] = acc;
                    gg += acc * acc;
                }
            tG += sqrt(gg);
            double ds5[5];
            or_stress_rate_one(g9, s5, Gam[i], p->rot_sign, ds5, NULL);
            tdS += sqrt(ds5[0] * ds5[0] + ds5[1] * ds5[1] + ds5[2] * ds5[2] + ds5[3] * ds5[3] +
                        ds5[4] * ds5[4]);
        }
        sa[i] = ta;
        sdu[i] = tdu;
        sG[i] = tG;
        sdS[i] = tdS;
    }
}

/* ----------------------------------------------------------------------- */
/* Full state integrator (used by multi-step tests).                        */
/* ----------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    double *x, *y, *z;          /* positions at the current time            */
    double *vx, *vy, *vz;       /* velocity at the half step                */
    double *u;                  /* internal energy at the half step         */
    double *S;                  /* deviatoric stress at the half step, 5n   */
    double *ax, *ay, *az;       /* derivatives of the last evaluation       */
    double *dudt, *dS;          /* dS is 5n                                  */
    double *eps2;               /* accumulated strain-rate invariant        */
    const double *m;
    double *h;                  /* smoothing lengths (changed only when adapted) */
    const int32_t *mat;
    const uint8_t *fixed;
    /* outputs of the last evaluation */
    double *rho, *omega, *P, *cs, *T, *Y, *Gam, *G, *dt_i;
    double dt;                  /* current global step (the next substep with
                                   rungs)                                    */
    int64_t n_singular, pairs;
    /* individual steps (reading T1), in ticks of the shortest rung
     * (tick = dt0 2^-(rungs-1)): each particle's step and the time elapsed
     * in it, the simulation time; the number of particles whose step was
     * cut to the shortest rung; the simulation time in seconds */
    int64_t *dtp, *el;
    int64_t ticks;
    double tick;
    int64_t n_clamped;
    double time;
} or_state_t;

/* One derivative evaluation at the current positions with the predicted
 * velocity vp, energy up and stress Sp (Sp is rescaled in place). */
static void eval_derivs(or_state_t *s, const or_material *mats, const or_params *p,
                        const double *vpx, const double *vpy, const double *vpz,
                        const double *up, double *Sp, int64_t *tar, int64_t nt,
                        int64_t *act, int64_t na, double *e2rate)
{
    /* density, state and rescaled predicted stress for the targets tar,
     * gradients, stress rates and forces for the targets act */
    int64_t n = s->n;
    or_density(n, s->x, s->y, s->z, s->m, s->h, p, nt, tar, s->rho, s->omega);
    or_state(nt, tar, s->rho, up, s->mat, mats, s->P, s->cs, s->T, s->Y, s->Gam);
    or_plastic_return_all(n, nt, tar, Sp, s->Y);
    or_gradients(n, s->x, s->y, s->z, vpx, vpy, vpz, s->m, s->h, s->rho, s->omega, p,
                 na, act, s->G, NULL, NULL, &s->n_singular);
    or_stress_rate(n, na, act, s->G, Sp, s->Gam, p->rot_sign, s->dS, e2rate);
    or_forces(n, s->x, s->y, s->z, vpx, vpy, vpz, s->m, s->h, s->rho, s->omega,
              s->P, s->cs, Sp, p, na, act, s->ax, s->ay, s->az, s->dudt, s->dt_i);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    or_pair_counts(n, s->x, s->y, s->z, s->h, p, n, tar, cnt);
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) tot += cnt[i];
    free(cnt);
    s->pairs = tot;
}

/* Own step of particle i: the CFL step and, with eta_a > 0, the
 * acceleration criterion (reading T2). */
static double own_step(const or_state_t *s, const or_params *p, int64_t i)
{
    double d = s->dt_i[i];
    if (p->eta_a > 0.0) {
        double a = sqrt((s->ax[i] * s->ax[i] + s->ay[i] * s->ay[i]) + s->az[i] * s->az[i]);
        if (a > 0.0) {
            double da = p->eta_a * sqrt(s->h[i] / a);
            if (da < d) d = da;
        }
    }
    return d;
}

static double min_dt(const or_state_t *s, const or_params *p)
{
    double d = INFINITY;
    for (int64_t i = 0; i < s->n; ++i) {
        if (s->fixed[i]) continue;
        double di = own_step(s, p, i);
        if (di < d) d = di;
    }
    return d;
}

/* Rung step in ticks (reading T1): the longest 2^(rungs-1-r) ticks whose
 * duration is not above d, the shortest rung if none is (counted); longer
 * than the current step cur only where the time t is a multiple of it. */
static int64_t rung_step(int rungs, double tick, double d, int64_t t, int64_t cur,
                         int64_t *clamped)
{
    int64_t st = (int64_t)1 << (rungs - 1);
    while (st > 1 && (double)st * tick > d) st >>= 1;
    if ((double)st * tick > d) ++*clamped;
    while (st > cur && t % st != 0) st >>= 1;
    return st;
}

/* Initial evaluation at t = 0 (predicted values = current values), choice
 * of the first step from the CFL condition (or dt_fixed > 0), and the
 * first opening kick. */
/* Adaptive smoothing lengths before an evaluation (reading H1), capped at
 * adapt_skin times the lengths on entry, fixed particles unchanged. */
#define OR_ADAPT_TOL 1e-10
#define OR_ADAPT_ITER 30
static void adapt_lengths(or_state_t *s, const or_params *p)
{
    if (!(p->adapt_ngb > 0.0)) return;
    int64_t n = s->n;
    double *cap = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) cap[i] = p->adapt_skin * s->h[i];
    or_adapt_h(n, s->x, s->y, s->z, s->m, s->h, cap, s->fixed, p, p->adapt_ngb, OR_ADAPT_TOL,
               OR_ADAPT_ITER, s->h);
    free(cap);
}

void or_init(or_state_t *s, const or_material *mats, const or_params *p, double dt_fixed)
{
    int64_t n = s->n;
    int64_t *tar = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) tar[i] = i;
    double *Sp = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    double *e2 = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(Sp, s->S, sizeof(double) * 5 * (size_t)n);
    adapt_lengths(s, p);
    eval_derivs(s, mats, p, s->vx, s->vy, s->vz, s->u, Sp, tar, n, tar, n, e2);
    s->time = 0.0;
    s->ticks = 0;
    s->n_clamped = 0;
    if (p->rungs > 0) {
        /* individual steps: dt_fixed is the base step dt0 */
        const int64_t top = (int64_t)1 << (p->rungs - 1);
        s->tick = ldexp(dt_fixed, -(p->rungs - 1));
        int64_t next = top;
        for (int64_t i = 0; i < n; ++i) {
            s->el[i] = 0;
            s->dtp[i] = top;
            if (s->fixed[i]) continue;
            s->dtp[i] = rung_step(p->rungs, s->tick, own_step(s, p, i), 0, top, &s->n_clamped);
            if (s->dtp[i] < next) next = s->dtp[i];
        }
        s->dt = (double)next * s->tick;
    } else {
        s->dt = dt_fixed > 0.0 ? dt_fixed : min_dt(s, p);
    }
    for (int64_t i = 0; i < n; ++i) {
        if (s->fixed[i]) continue;
        double hd = 0.5 * (p->rungs > 0 ? (double)s->dtp[i] * s->tick : s->dt);
        s->vx[i] += hd * s->ax[i];
        s->vy[i] += hd * s->ay[i];
        s->vz[i] += hd * s->az[i];
        s->u[i] += hd * s->dudt[i];
        for (int c = 0; c < 5; ++c) s->S[c * n + i] = Sp[c * n + i] + hd * s->dS[c * n + i];
    }
    free(Sp); free(e2); free(tar);
}

/* One step of the kick-drift-kick scheme with the predictor of
 * Predict_S eq. (reading K9), or, with rungs, one substep of the individual
 * steps (reading T1) to the next end of a particle's step.  On entry v, u,
 * S hold the values kicked at the start of each particle's step and a,
 * dudt, dS the derivatives of its last evaluation. */
void or_step(or_state_t *s, const or_material *mats, const or_params *p, double dt_fixed)
{
    int64_t n = s->n;
    const int hier = p->rungs > 0;
    double dt = s->dt;
    int64_t sub = hier ? (int64_t)llround(dt / s->tick) : 0;   /* substep in ticks */
    int64_t *tar = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *act = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) tar[i] = i;
    double *vpx = (double *)malloc(sizeof(double) * (size_t)n);
    double *vpy = (double *)malloc(sizeof(double) * (size_t)n);
    double *vpz = (double *)malloc(sizeof(double) * (size_t)n);
    double *up = (double *)malloc(sizeof(double) * (size_t)n);
    double *Sp = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    double *e2 = (double *)malloc(sizeof(double) * (size_t)n);
    /* drift */
    for (int64_t i = 0; i < n; ++i) {
        if (s->fixed[i]) continue;
        s->x[i] += dt * s->vx[i];
        s->y[i] += dt * s->vy[i];
        s->z[i] += dt * s->vz[i];
    }
    if (hier) {
        s->ticks += sub;
        s->time = (double)s->ticks * s->tick;
    } else {
        s->time += dt;
    }
    /* predictor: from the kicked values with the last derivatives, over the
     * time elapsed in each particle's step less half of it (half a step
     * for a particle whose step ends now) */
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (s->fixed[i]) {
            vpx[i] = s->vx[i]; vpy[i] = s->vy[i]; vpz[i] = s->vz[i]; up[i] = s->u[i];
            for (int c = 0; c < 5; ++c) Sp[c * n + i] = s->S[c * n + i];
            if (!hier) act[na++] = i;   /* shared step: derivatives of every particle */
            continue;
        }
        double tau = 0.5 * dt;
        if (hier) {
            s->el[i] += sub;
            tau = ((double)s->el[i] - 0.5 * (double)s->dtp[i]) * s->tick;
            if (s->el[i] == s->dtp[i]) act[na++] = i;
        } else {
            act[na++] = i;
        }
        vpx[i] = s->vx[i] + tau * s->ax[i];
        vpy[i] = s->vy[i] + tau * s->ay[i];
        vpz[i] = s->vz[i] + tau * s->az[i];
        up[i] = s->u[i] + tau * s->dudt[i];
        for (int c = 0; c < 5; ++c) Sp[c * n + i] = s->S[c * n + i] + tau * s->dS[c * n + i];
    }
    adapt_lengths(s, p);
    eval_derivs(s, mats, p, vpx, vpy, vpz, up, Sp, tar, n, act, na, e2);
    /* closing kick of the particles whose step ends, rescaling of S */
    for (int64_t k = 0; k < na; ++k) {
        int64_t i = act[k];
        if (s->fixed[i]) continue;
        double own = hier ? (double)s->dtp[i] * s->tick : dt;
        double hd = 0.5 * own;
        s->vx[i] += hd * s->ax[i];
        s->vy[i] += hd * s->ay[i];
        s->vz[i] += hd * s->az[i];
        s->u[i] += hd * s->dudt[i];
        double s5[5];
        for (int c = 0; c < 5; ++c) s5[c] = s->S[c * n + i] + hd * s->dS[c * n + i];
        or_plastic_return(s5, s->Y[i]);
        for (int c = 0; c < 5; ++c) s->S[c * n + i] = s5[c];
        s->eps2[i] += own * e2[i];
    }
    /* their next steps, opening kick (no rescaling) */
    double dtn = 0.0;
    if (hier) {
        for (int64_t k = 0; k < na; ++k) {
            int64_t i = act[k];
            s->dtp[i] = rung_step(p->rungs, s->tick, own_step(s, p, i), s->ticks, s->dtp[i],
                                  &s->n_clamped);
            s->el[i] = 0;
        }
    } else {
        dtn = dt_fixed > 0.0 ? dt_fixed : min_dt(s, p);
    }
    for (int64_t k = 0; k < na; ++k) {
        int64_t i = act[k];
        if (s->fixed[i]) continue;
        double hn = 0.5 * (hier ? (double)s->dtp[i] * s->tick : dtn);
        s->vx[i] += hn * s->ax[i];
        s->vy[i] += hn * s->ay[i];
        s->vz[i] += hn * s->az[i];
        s->u[i] += hn * s->dudt[i];
        for (int c = 0; c < 5; ++c) s->S[c * n + i] += hn * s->dS[c * n + i];
    }
    /* the next substep: to the next end of any particle's step */
    if (hier) {
        int64_t next = (int64_t)1 << (p->rungs - 1);
        for (int64_t i = 0; i < n; ++i) {
            if (s->fixed[i]) continue;
            int64_t rem = s->dtp[i] - s->el[i];
            if (rem < next) next = rem;
        }
        s->dt = (double)next * s->tick;
    } else {
        s->dt = dtn;
    }
    free(vpx); free(vpy); free(vpz); free(up); free(Sp); free(e2); free(tar); free(act);
}

/* The rung rule on its own, for the tests. */
int64_t or_rung_step(int32_t rungs, double tick, double d, int64_t t, int64_t cur,
                     int64_t *clamped)
{
    return rung_step(rungs, tick, d, t, cur, clamped);
}

/* ----------------------------------------------------------------------- */
/* Array helpers for the tests.                                             */
/* ----------------------------------------------------------------------- */
void or_kernel_arr(int64_t n, const double *r, const double *h,
                   double *W, double *K, double *dWdh)
{
    for (int64_t i = 0; i < n; ++i) {
        if (W) W[i] = or_W(r[i], h[i]);
        if (K) K[i] = or_K(r[i], h[i]);
        if (dWdh) dWdh[i] = or_dWdh(r[i], h[i]);
    }
}

void or_tillotson_arr(const or_material *M, int64_t n, const double *rho, const double *u,
                      double *P, double *c, double *dPdrho, double *dPdu)
{
    for (int64_t i = 0; i < n; ++i)
        or_tillotson(M, rho[i], u[i], &P[i], &c[i], dPdrho ? &dPdrho[i] : NULL,
                     dPdu ? &dPdu[i] : NULL);
}

void or_eos_arr(const or_material *M, int64_t n, const double *rho, const double *u,
                double *P, double *c, double *T)
{
    for (int64_t i = 0; i < n; ++i) or_eos(M, rho[i], u[i], &P[i], &c[i], &T[i]);
}

void or_yield_arr(const or_material *M, int64_t n, const double *rho, const double *P,
                  const double *T, double *Y)
{
    for (int64_t i = 0; i < n; ++i) Y[i] = or_yield(M, rho ? rho[i] : M->rho0, P[i], T[i]);
}

/* Rows of 9 (G) and 5 (S) per entry, entry-major. */
void or_stress_rate_rows(int64_t n, const double *G, const double *S, const double *Gam,
                         double rot_sign, int32_t printed, double *dS, double *e2)
{
    for (int64_t i = 0; i < n; ++i) {
        if (printed)
            or_stress_rate_printed(&G[9 * i], &S[5 * i], Gam[i], &dS[5 * i]);
        else
            or_stress_rate_one(&G[9 * i], &S[5 * i], Gam[i], rot_sign, &dS[5 * i],
                               e2 ? &e2[i] : NULL);
    }
}

void or_plastic_return_rows(int64_t n, double *S, const double *Y)
{
    for (int64_t i = 0; i < n; ++i) or_plastic_return(&S[5 * i], Y[i]);
}

/* y_pred = y + 1/2 dt dy for non-fixed entries (Predict_S eq. applied to a
 * component-major array of ncomp rows). */
void or_predict(int64_t n, int32_t ncomp, const uint8_t *fixed, double dt,
                const double *y, const double *dy, double *out)
{
    for (int c = 0; c < ncomp; ++c)
        for (int64_t i = 0; i < n; ++i)
            out[c * n + i] = (fixed && fixed[i]) ? y[c * n + i]
                                                 : y[c * n + i] + 0.5 * dt * dy[c * n + i];
}
