// Per-particle physics of the strength-SPH step as device functions, in
// double: Tillotson EOS with sound speed, Collins yield with thermal
// softening, shear modulus, plastic rescaling, Jaumann stress rate.  Shared
// by the separate pass kernels and the fused whole-step kernels.
#pragma once

#include "sph_internal.h"

namespace sph {

constexpr double kPiD = 3.14159265358979323846;

// Material table passed by value to the kernels.
struct MatTable {
    sph_material m[8];
    int32_t n;
};

__device__ __forceinline__ const sph_material &material_of(const MatTable &mt, const int32_t *mat,
                                                           int64_t i) {
    int id = mat ? mat[i] : 0;
    id = id < 0 ? 0 : (id >= mt.n ? mt.n - 1 : id);
    return mt.m[id];
}

// Tillotson, compressed or cold branch: P and its partial derivatives (zero
// below rho_limit rho0).
__device__ inline void till_cold(const sph_material &M, double rho, double u, double &P,
                                 double &dr, double &du) {
    const double eta = rho / M.rho0, mu = eta - 1.0;
    if (eta < M.rho_limit) {  // expanded below the limit: no tension
        P = dr = du = 0.0;
        return;
    }
    const double w = u / (M.E0 * eta * eta) + 1.0;
    P = (M.a + M.b / w) * rho * u + M.A * mu + M.B * mu * mu;
    dr = M.a * u + M.b * u / w + 2.0 * M.b * u * (w - 1.0) / (w * w) +
         (M.A + 2.0 * M.B * mu) / M.rho0;
    du = M.a * rho + M.b * rho / w - M.b * rho * (w - 1.0) / (w * w);
}

// Tillotson, hot expanded branch.
__device__ inline void till_hot(const sph_material &M, double rho, double u, double &P,
                                double &dr, double &du) {
    const double eta = rho / M.rho0, mu = eta - 1.0;
    const double w = u / (M.E0 * eta * eta) + 1.0;
    const double z = 1.0 / eta - 1.0;
    const double eb = exp(-M.beta * z), ea = exp(-M.alpha * z * z);
    const double br = M.b * rho * u / w + M.A * mu * eb;
    P = M.a * rho * u + br * ea;
    const double dz = -M.rho0 / (rho * rho);
    const double dbr = M.b * u / w + 2.0 * M.b * u * (w - 1.0) / (w * w) + M.A / M.rho0 * eb -
                       M.A * mu * eb * M.beta * dz;
    dr = M.a * u + dbr * ea - br * ea * 2.0 * M.alpha * z * dz;
    du = M.a * rho + ea * (M.b * rho / w - M.b * rho * (w - 1.0) / (w * w));
}

// Tillotson P and sound speed c (c^2 = dP/drho + P/rho^2 dP/du, floored).
__device__ inline void tillotson(const sph_material &M, double rho, double u, double &P,
                                 double &c) {
    double dr, du;
    if (rho >= M.rho0 || u <= M.Eiv) {
        till_cold(M, rho, u, P, dr, du);
    } else if (u >= M.Ecv) {
        till_hot(M, rho, u, P, dr, du);
    } else {
        double Pc, drc, duc, Ph, drh, duh;
        till_cold(M, rho, u, Pc, drc, duc);
        till_hot(M, rho, u, Ph, drh, duh);
        const double span = M.Ecv - M.Eiv;
        P = ((u - M.Eiv) * Ph + (M.Ecv - u) * Pc) / span;
        dr = ((u - M.Eiv) * drh + (M.Ecv - u) * drc) / span;
        du = ((u - M.Eiv) * duh + Ph + (M.Ecv - u) * duc - Pc) / span;
    }
    const double c2 = dr + P / (rho * rho) * du;
    c = c2 > 0.0 ? sqrt(c2) : 0.0;
    c = c < M.c_min ? M.c_min : c;
}

// Melting temperature: the constant, or the linear interpolation of the
// material's density table, held at its end values outside it.
__device__ inline double melt_temperature(const sph_material &M, double rho) {
    const int n = M.tmelt_n;
    if (n < 2) return M.T_melt;
    if (rho <= M.tmelt_rho[0]) return M.tmelt_T[0];
    if (rho >= M.tmelt_rho[n - 1]) return M.tmelt_T[n - 1];
    int k = 0;
    while (k + 2 < n && rho >= M.tmelt_rho[k + 1]) ++k;
    const double w = (rho - M.tmelt_rho[k]) / (M.tmelt_rho[k + 1] - M.tmelt_rho[k]);
    return M.tmelt_T[k] + w * (M.tmelt_T[k + 1] - M.tmelt_T[k]);
}

// Cell of a coordinate on ascending table nodes: x is clamped to the node
// range and the result is the largest k in [0, n-2] with node[k] <= x, by
// bisection (every probe is inside node[0..n-2]).
__device__ inline int table_cell(const double *node, int n, double &x) {
    const double lo = node[0], hi = node[n - 1];
    x = x < lo ? lo : (x > hi ? hi : x);
    int a = 0, b = n - 2;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (node[mid] <= x)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

// Bilinear interpolant of one value grid in cell (kr, ku) at weights wr, wu.
__device__ inline double table_bilinear(const double *f, int nu, int kr, int ku, double wr,
                                        double wu) {
    const double *r0 = f + (int64_t)kr * nu + ku, *r1 = r0 + nu;
    const double f0 = r0[0] + wu * (r0[1] - r0[0]);
    const double f1 = r1[0] + wu * (r1[1] - r1[0]);
    return f0 + wr * (f1 - f0);
}

// Tabulated EOS: P, c (floored at c_min) and T from the material's table.
__device__ inline void table_eos(const sph_material &M, double rho, double u, double &P,
                                 double &c, double &T) {
    const int nu = M.eos_nu;
    const int kr = table_cell(M.eos_rho, M.eos_nrho, rho);
    const int ku = table_cell(M.eos_u, nu, u);
    const double wr = (rho - M.eos_rho[kr]) / (M.eos_rho[kr + 1] - M.eos_rho[kr]);
    const double wu = (u - M.eos_u[ku]) / (M.eos_u[ku + 1] - M.eos_u[ku]);
    P = table_bilinear(M.eos_P, nu, kr, ku, wr, wu);
    c = table_bilinear(M.eos_c, nu, kr, ku, wr, wu);
    c = c < M.c_min ? M.c_min : c;
    T = table_bilinear(M.eos_T, nu, kr, ku, wr, wu);
}

// EOS, temperature, Collins yield (intact fit, Coulomb friction, minimum,
// pressure clipped at 0) with thermal softening, and shear modulus.
__device__ inline void material_state(const sph_material &M, double rho, double u, double &P,
                                      double &c, double &T, double &Y, double &Gm) {
    if (M.eos_nrho >= 2 && M.eos_nu >= 2) {
        table_eos(M, rho, u, P, c, T);
    } else {
        tillotson(M, rho, u, P, c);
        T = M.T_ref + u / M.cv;
    }
    Y = 0.0;
    Gm = 0.0;
    if (M.strength_on) {
        const double pp = P > 0.0 ? P : 0.0;
        const double yi = M.Y0 + M.mu_i * pp / (1.0 + M.mu_i * pp / (M.Ym - M.Y0));
        const double yd = M.mu_d * pp;
        Y = yi < yd ? yi : yd;
        if (M.thermal_softening_on) {
            const double s = tanh(M.xi * (melt_temperature(M, rho) / T - 1.0));
            Y *= s > 0.0 ? s : 0.0;
        }
        Gm = M.shear_modulus > 0.0 ? M.shear_modulus
                                   : 3.0 * (1.0 - 2.0 * M.nu) / (2.0 * (1.0 + M.nu)) * rho * c * c;
    }
}

// S -> f S, f = min(Y / sqrt(J2), 1), J2 = 1/2 S:S over the full tensor.
__device__ __forceinline__ void plastic_return(double s[5], double Y) {
    const double szz = -s[0] - s[1];
    const double J2 = 0.5 * (s[0] * s[0] + s[1] * s[1] + szz * szz) + s[2] * s[2] +
                      s[3] * s[3] + s[4] * s[4];
    if (J2 > 0.0) {
        const double f = Y / sqrt(J2);
        if (f < 1.0)
            for (int c = 0; c < 5; ++c) s[c] *= f;
    }
}

// Stress rate 2 Gamma (eps - tr(eps)/3 I) + rot (R S - S R) with
// eps = (G + G^T)/2, R = (G - G^T)/2; returns 1/2 eps:eps as well.
__device__ inline void stress_rate(const double g[9], const double s5[5], double gm, double rot,
                                   double ds[5], double &e2) {
    const double S[3][3] = {{s5[0], s5[2], s5[3]},
                            {s5[2], s5[1], s5[4]},
                            {s5[3], s5[4], -s5[0] - s5[1]}};
    double E[3][3], R[3][3];
    double ee = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            E[a][b] = 0.5 * (g[3 * a + b] + g[3 * b + a]);
            R[a][b] = 0.5 * (g[3 * a + b] - g[3 * b + a]);
            ee += E[a][b] * E[a][b];
        }
    e2 = 0.5 * ee;
    const double tr3 = (E[0][0] + E[1][1] + E[2][2]) / 3.0;
    const int ia[5] = {0, 1, 0, 0, 1}, ib[5] = {0, 1, 1, 2, 2};
    for (int c = 0; c < 5; ++c) {
        const int a = ia[c], b = ib[c];
        double rs = 0.0, sr = 0.0;
        for (int k = 0; k < 3; ++k) {
            rs += R[a][k] * S[k][b];
            sr += S[a][k] * R[k][b];
        }
        ds[c] = 2.0 * gm * (E[a][b] - (a == b ? tr3 : 0.0)) + rot * (rs - sr);
    }
}

// Corrected gradient G = F C from the raw sums (C^-1 symmetric: xx, yy, zz,
// xy, xz, yz; F row-major).  Returns false (C = identity) when C^-1 is
// singular or the particle has fewer than 4 neighbours.
__device__ inline bool corrected_gradient(const double ci[6], const double F[9], int nnb,
                                          int use_corr, double G[9]) {
    const double A[3][3] = {{ci[0], ci[3], ci[4]}, {ci[3], ci[1], ci[5]}, {ci[4], ci[5], ci[2]}};
    double C[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    bool ok = true;
    if (use_corr) {
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
        double fro = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) fro += A[a][b] * A[a][b];
        fro = sqrt(fro);
        if (det != 0.0 && nnb >= 4 && fabs(det) >= 1e-12 * fro * fro * fro) {
            const double id = 1.0 / det;
            C[0][0] = c00 * id;
            C[1][0] = c01 * id;
            C[2][0] = c02 * id;
            C[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
            C[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
            C[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
            C[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
            C[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
            C[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
        } else {
            ok = false;
        }
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            G[3 * a + b] = F[3 * a + 0] * C[0][b] + F[3 * a + 1] * C[1][b] + F[3 * a + 2] * C[2][b];
    return ok;
}

}  // namespace sph
