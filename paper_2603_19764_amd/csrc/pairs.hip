// Pair passes of the strength-SPH hot path on gfx950: density with the
// grad-h term, corrected velocity gradient, forces with the full stress
// tensor and artificial viscosity.  Each particle i is served by a group of
// L consecutive lanes that split i's pair list; per-particle sums are
// combined with cross-lane shuffles.  Templates select the arithmetic of
// the pair terms: double on absolute positions, or float on positions
// relative to each particle's cell origin (the separation of a pair is
// (d_i - d_j) - s L with s the stencil offset of j's cell).
//
// Kernel: Wendland C2 with support H = 2h,
//   W = 21/(2 pi H^3) t^4 (1 + 4q),  t = 1 - q,  q = r/H
//   grad_i W = K x_ij,  K = -210/(pi H^5) t^3
//   dW/dh = -21/(pi H^4) t^3 (3 + 9q - 32 q^2)
#include "sph_internal.h"

namespace sph {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;

// ---------------------------------------------------------- common helpers
__device__ __forceinline__ void stencil_offsets(float *sh) {
    // sh[3t + a] = offset of stencil cell t along axis a, t = 9(dz+1) + 3(dy+1) + (dx+1)
    for (int t = threadIdx.x; t < 27; t += blockDim.x) {
        sh[3 * t + 0] = (float)(t % 3 - 1);
        sh[3 * t + 1] = (float)((t / 3) % 3 - 1);
        sh[3 * t + 2] = (float)(t / 9 - 1);
    }
}

template <bool F32>
struct Real;
template <>
struct Real<true> {
    using T = float;
    using T4 = float4;
};
template <>
struct Real<false> {
    using T = double;
    using T4 = double4;
};

// Separation x_i - x_j of pair entry e.
template <bool F32>
__device__ __forceinline__ void separation(const typename Real<F32>::T4 &pi,
                                           const typename Real<F32>::T4 &pj, uint32_t e,
                                           const float *shs, float L32, typename Real<F32>::T &dx,
                                           typename Real<F32>::T &dy, typename Real<F32>::T &dz) {
    if constexpr (F32) {
        const int t = (int)((e >> kCodeShift) & 31u);
        dx = fmaf(-shs[3 * t + 0], L32, pi.x - pj.x);
        dy = fmaf(-shs[3 * t + 1], L32, pi.y - pj.y);
        dz = fmaf(-shs[3 * t + 2], L32, pi.z - pj.z);
    } else {
        dx = pi.x - pj.x;
        dy = pi.y - pj.y;
        dz = pi.z - pj.z;
    }
}

template <bool F32>
__device__ __forceinline__ typename Real<F32>::T4 load_pos(const double4 *p64, const float4 *p32,
                                                           int64_t k) {
    if constexpr (F32) return p32[k];
    else return p64[k];
}

__device__ __forceinline__ float rsqrt_sqrt(float r2) { return sqrtf(r2); }
__device__ __forceinline__ double rsqrt_sqrt(double r2) { return sqrt(r2); }

// ================================================================ density
template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_density(
    int64_t n, const double4 *__restrict__ posh64, const float4 *__restrict__ posh32,
    const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const double *__restrict__ m, double *__restrict__ rho, double *__restrict__ omega,
    int32_t omega_one) {
    using R = typename Real<F32>::T;
    using R4 = typename Real<F32>::T4;
    __shared__ float shs[81];
    if constexpr (F32) {
        stencil_offsets(shs);
        __syncthreads();
    }
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lg = threadIdx.x % L;
    const bool active = i < n;
    double sw = 0.0, sd = 0.0;
    double hi = 0.0;
    if (active) {
        const R4 pi = load_pos<F32>(posh64, posh32, i);
        hi = posh64[i].w;
        const R Hinv = (R)(0.5 / hi);
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        for (int k = lg; k < c; k += L) {
            const uint32_t e = row[k];
            if (!(e & kDensityBit)) continue;
            const int64_t j = e & kIdxMask;
            const R4 pj = load_pos<F32>(posh64, posh32, j);
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R q = rsqrt_sqrt(r2) * Hinv;
            R t = (R)1 - q;
            t = t > (R)0 ? t : (R)0;
            const R t3 = t * t * t;
            const R mj = (R)m[j];
            const R w = mj * (t3 * t * ((R)1 + (R)4 * q));
            const R dh = mj * (t3 * ((R)3 + q * ((R)9 - (R)32 * q)));
            sw += (double)w;
            sd += (double)dh;
        }
    }
    sw = group_sum<L>(sw);
    sd = group_sum<L>(sd);
    if (active && lg == 0) {
        const double H = 2.0 * hi;
        const double Wn = 21.0 / (2.0 * kPi * H * H * H);
        const double Dn = -21.0 / (kPi * H * H * H * H);
        const double mi = m[i];
        const double r = Wn * (mi + sw);           // self term W(0) = Wn
        const double dsum = Dn * (3.0 * mi + sd);  // self term dW/dh(0) = 3 Dn
        rho[i] = r;
        omega[i] = omega_one ? 1.0 : 1.0 + hi / (3.0 * r) * dsum;
    }
}

// -------------------------------------------- EOS, yield, shear modulus
struct MatTable {
    sph_material m[8];
    int32_t n;
};

__device__ static void till_cold(const sph_material &M, double rho, double u, double &P,
                                 double &dr, double &du) {
    const double eta = rho / M.rho0, mu = eta - 1.0;
    const double w = u / (M.E0 * eta * eta) + 1.0;
    P = (M.a + M.b / w) * rho * u + M.A * mu + M.B * mu * mu;
    dr = M.a * u + M.b * u / w + 2.0 * M.b * u * (w - 1.0) / (w * w) +
         (M.A + 2.0 * M.B * mu) / M.rho0;
    du = M.a * rho + M.b * rho / w - M.b * rho * (w - 1.0) / (w * w);
}

__device__ static void till_hot(const sph_material &M, double rho, double u, double &P,
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
__device__ static void tillotson(const sph_material &M, double rho, double u, double &P,
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

__global__ void k_eos(int64_t n, const double *__restrict__ rho, const double *__restrict__ u,
                      const int32_t *__restrict__ mat, MatTable mt, double *P, double *cs,
                      double *T, double *Y, double *Gmod) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int id = mat ? mat[i] : 0;
    id = id < 0 ? 0 : (id >= mt.n ? mt.n - 1 : id);
    const sph_material &M = mt.m[id];
    const double r = rho[i], e = u[i];
    double p, c;
    tillotson(M, r, e, p, c);
    const double t = M.T_ref + e / M.cv;
    double y = 0.0, gm = 0.0;
    if (M.strength_on) {
        // Collins yield: intact fit, Coulomb friction, minimum; P clipped at 0
        const double pp = p > 0.0 ? p : 0.0;
        const double yi = M.Y0 + M.mu_i * pp / (1.0 + M.mu_i * pp / (M.Ym - M.Y0));
        const double yd = M.mu_d * pp;
        y = yi < yd ? yi : yd;
        if (M.thermal_softening_on) {
            const double s = tanh(M.xi * (M.T_melt / t - 1.0));
            y *= s > 0.0 ? s : 0.0;
        }
        gm = M.shear_modulus > 0.0
                 ? M.shear_modulus
                 : 3.0 * (1.0 - 2.0 * M.nu) / (2.0 * (1.0 + M.nu)) * r * c * c;
    }
    P[i] = p;
    cs[i] = c;
    T[i] = t;
    Y[i] = y;
    Gmod[i] = gm;
}

// ============================================================== gradients
// Records: rec0 = (vx, vy, vz, m), rec1 = (1/H, K_norm/(Omega rho)),
// K_norm = -210/(pi H^5).
template <bool F32>
__global__ void k_pack_grad(int64_t n, const double *vx, const double *vy, const double *vz,
                            const double *m, const double *h, const double *rho,
                            const double *omega, typename Real<F32>::T4 *rec0, void *rec1v) {
    using R = typename Real<F32>::T;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double H = 2.0 * h[i];
    const double kn = -210.0 / (kPi * H * H * H * H * H);
    rec0[i] = {(R)vx[i], (R)vy[i], (R)vz[i], (R)m[i]};
    if constexpr (F32)
        ((float2 *)rec1v)[i] = make_float2((float)(1.0 / H), (float)(kn / (omega[i] * rho[i])));
    else
        ((double2 *)rec1v)[i] = make_double2(1.0 / H, kn / (omega[i] * rho[i]));
}

// Raw sums per particle (15 rows): C^-1 (xx, yy, zz, xy, xz, yz) and F (row-major 9).
template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_gradients(
    int64_t n, const double4 *__restrict__ posh64, const float4 *__restrict__ posh32,
    const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const typename Real<F32>::T4 *__restrict__ rec0, const void *__restrict__ rec1v,
    double *__restrict__ gsum) {
    using R = typename Real<F32>::T;
    using R4 = typename Real<F32>::T4;
    using R2 = typename std::conditional<F32, float2, double2>::type;
    const R2 *rec1 = (const R2 *)rec1v;
    __shared__ float shs[81];
    if constexpr (F32) {
        stencil_offsets(shs);
        __syncthreads();
    }
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lg = threadIdx.x % L;
    const bool active = i < n;
    R c_xx = 0, c_yy = 0, c_zz = 0, c_xy = 0, c_xz = 0, c_yz = 0;
    R f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
        const R4 pi = load_pos<F32>(posh64, posh32, i);
        const R4 vi = rec0[i];
        const R2 ai = rec1[i];
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        for (int k = lg; k < c; k += L) {
            const uint32_t e = row[k];
            const int64_t j = e & kIdxMask;
            const R4 pj = load_pos<F32>(posh64, posh32, j);
            const R4 vj = rec0[j];
            const R2 aj = rec1[j];
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R r = rsqrt_sqrt(dx * dx + dy * dy + dz * dz);
            R ti = (R)1 - r * ai.x, tj = (R)1 - r * aj.x;
            ti = ti > (R)0 ? ti : (R)0;
            tj = tj > (R)0 ? tj : (R)0;
            // -w = -1/2 m_j (K_i/(Om rho)_i + K_j/(Om rho)_j)
            const R nw = (R)(-0.5) * vj.w * (ai.y * ti * ti * ti + aj.y * tj * tj * tj);
            const R ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
            const R wx = nw * dx, wy = nw * dy, wz = nw * dz;
            c_xx += wx * dx; c_yy += wy * dy; c_zz += wz * dz;
            c_xy += wx * dy; c_xz += wx * dz; c_yz += wy * dz;
            f[0] += ux * wx; f[1] += ux * wy; f[2] += ux * wz;
            f[3] += uy * wx; f[4] += uy * wy; f[5] += uy * wz;
            f[6] += uz * wx; f[7] += uz * wy; f[8] += uz * wz;
        }
    }
    c_xx = group_sum<L>(c_xx); c_yy = group_sum<L>(c_yy); c_zz = group_sum<L>(c_zz);
    c_xy = group_sum<L>(c_xy); c_xz = group_sum<L>(c_xz); c_yz = group_sum<L>(c_yz);
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = group_sum<L>(f[a]);
    if (active && lg == 0) {
        double *o = gsum + i;
        o[0 * n] = c_xx; o[1 * n] = c_yy; o[2 * n] = c_zz;
        o[3 * n] = c_xy; o[4 * n] = c_xz; o[5 * n] = c_yz;
#pragma unroll
        for (int a = 0; a < 9; ++a) o[(6 + a) * n] = f[a];
    }
}

// C = (C^-1)^-1 from the adjugate (identity if singular), G = F C.
__global__ void k_grad_epilogue(int64_t n, const double *__restrict__ gsum,
                                const int32_t *__restrict__ ncount, int32_t use_corr,
                                double *__restrict__ G, int64_t *n_singular) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int sing = 0;
    if (i < n) {
        const double *s = gsum + i;
        const double A[3][3] = {{s[0], s[3 * n], s[4 * n]},
                                {s[3 * n], s[1 * n], s[5 * n]},
                                {s[4 * n], s[5 * n], s[2 * n]}};
        double F[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) F[a][b] = s[(6 + 3 * a + b) * n];
        double C[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        if (use_corr) {
            const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
            const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
            const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
            const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
            double fro = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) fro += A[a][b] * A[a][b];
            fro = sqrt(fro);
            if (det != 0.0 && ncount[i] >= 4 && fabs(det) >= 1e-12 * fro * fro * fro) {
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
                sing = 1;
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                G[(3 * a + b) * n + i] = F[a][0] * C[0][b] + F[a][1] * C[1][b] + F[a][2] * C[2][b];
    }
    if (n_singular) {
        const uint64_t m = __ballot(sing);
        if (m && (threadIdx.x % kWave) == 0) atomicAdd((unsigned long long *)n_singular,
                                                       (unsigned long long)__popcll(m));
    }
}

// ================================================================= forces
// Records: rec0 = (vx, vy, vz, m); rec1 = Kn (Axx, Ayy, Azz, Axy); rec2 =
// (Kn Axz, Kn Ayz, rho, c); rec3 = (1/H, Kn, h, 0) with A = (-P I + S)/(Omega
// rho^2) and Kn = -210/(pi H^5): K(r,h) A = t^3 (Kn A).
template <bool F32>
__global__ void k_pack_forces(int64_t n, const double *vx, const double *vy, const double *vz,
                              const double *m, const double *h, const double *rho,
                              const double *omega, const double *P, const double *cs,
                              const double *S, typename Real<F32>::T4 *rec) {
    using R = typename Real<F32>::T;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double H = 2.0 * h[i];
    const double kn = -210.0 / (kPi * H * H * H * H * H);
    const double sc = kn / (omega[i] * rho[i] * rho[i]);
    const double sxx = S[i], syy = S[n + i], sxy = S[2 * n + i], sxz = S[3 * n + i],
                 syz = S[4 * n + i];
    const double p = P[i];
    rec[i] = {(R)vx[i], (R)vy[i], (R)vz[i], (R)m[i]};
    rec[n + i] = {(R)(sc * (sxx - p)), (R)(sc * (syy - p)), (R)(sc * (-sxx - syy - p)), (R)(sc * sxy)};
    rec[2 * n + i] = {(R)(sc * sxz), (R)(sc * syz), (R)rho[i], (R)cs[i]};
    rec[3 * n + i] = {(R)(1.0 / H), (R)kn, (R)h[i], (R)0};
}

template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_forces(
    int64_t n, const double4 *__restrict__ posh64, const float4 *__restrict__ posh32,
    const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const typename Real<F32>::T4 *__restrict__ rec, double al, double be, double eps,
    double etaC, double gx, double gy, double gz, double *__restrict__ ax,
    double *__restrict__ ay, double *__restrict__ az, double *__restrict__ dudt,
    double *__restrict__ dtc) {
    using R = typename Real<F32>::T;
    using R4 = typename Real<F32>::T4;
    __shared__ float shs[81];
    if constexpr (F32) {
        stencil_offsets(shs);
        __syncthreads();
    }
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lg = threadIdx.x % L;
    const bool active = i < n;
    R acx = 0, acy = 0, acz = 0, du = 0, mumax = 0;
    if (active) {
        const R4 pi = load_pos<F32>(posh64, posh32, i);
        const R4 vi = rec[i], Ai = rec[n + i], Bi = rec[2 * n + i], Hi = rec[3 * n + i];
        const R ral = (R)al, rbe = (R)be, reps = (R)eps;
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        for (int k = lg; k < c; k += L) {
            const uint32_t e = row[k];
            const int64_t j = e & kIdxMask;
            const R4 pj = load_pos<F32>(posh64, posh32, j);
            const R4 vj = rec[j], Aj = rec[n + j], Bj = rec[2 * n + j], Hj = rec[3 * n + j];
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R r = rsqrt_sqrt(r2);
            R ti = (R)1 - r * Hi.x, tj = (R)1 - r * Hj.x;
            ti = ti > (R)0 ? ti : (R)0;
            tj = tj > (R)0 ? tj : (R)0;
            const R ti3 = ti * ti * ti, tj3 = tj * tj * tj;
            // y_k = (Kn A)_k x_ij
            const R yix = Ai.x * dx + Ai.w * dy + Bi.x * dz;
            const R yiy = Ai.w * dx + Ai.y * dy + Bi.y * dz;
            const R yiz = Bi.x * dx + Bi.y * dy + Ai.z * dz;
            const R yjx = Aj.x * dx + Aj.w * dy + Bj.x * dz;
            const R yjy = Aj.w * dx + Aj.y * dy + Bj.y * dz;
            const R yjz = Bj.x * dx + Bj.y * dy + Aj.z * dz;
            const R mj = vj.w;
            acx += mj * (ti3 * yix + tj3 * yjx);
            acy += mj * (ti3 * yiy + tj3 * yjy);
            acz += mj * (ti3 * yiz + tj3 * yjz);
            const R ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
            du -= mj * ti3 * (ux * yix + uy * yiy + uz * yiz);
            const R vr = ux * dx + uy * dy + uz * dz;
            if (vr < (R)0) {
                const R hb = (R)0.5 * (Hi.z + Hj.z);
                const R mu = hb * vr / (r2 + reps * hb * hb);
                const R cb = (R)0.5 * (Bi.w + Bj.w);
                const R rb = (R)0.5 * (Bi.z + Bj.z);
                const R Pi = (-ral * cb * mu + rbe * mu * mu) / rb;
                const R gw = (R)0.5 * (Hi.y * ti3 + Hj.y * tj3);  // mean K
                const R s = mj * Pi * gw;
                acx -= s * dx;
                acy -= s * dy;
                acz -= s * dz;
                du += (R)0.5 * s * vr;
                mumax = mumax > -mu ? mumax : -mu;
            }
        }
    }
    acx = group_sum<L>(acx);
    acy = group_sum<L>(acy);
    acz = group_sum<L>(acz);
    du = group_sum<L>(du);
    mumax = group_max<L>(mumax);
    if (active && lg == 0) {
        const double hi = posh64[i].w;
        const double ci = (double)rec[2 * n + i].w;
        ax[i] = (double)acx + gx;
        ay[i] = (double)acy + gy;
        az[i] = (double)acz + gz;
        dudt[i] = (double)du;
        dtc[i] = etaC * hi / ((1.0 + 0.6 * al) * ci + 0.6 * be * (double)mumax);
    }
}

// =============================================================== launches
template <int L>
static void density_launch(Ctx *ctx, int64_t n, const double *m, sph_precision prec,
                           const sph_params *prm, double *rho, double *omega, hipStream_t s) {
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    if (prec == SPH_FP32_CELLREL)
        hipLaunchKernelGGL((k_density<L, true>), dim3(nb), dim3(kBlock), 0, s, n, ctx->posh64,
                           ctx->posh32, ctx->runid, ctx->grid, ctx->nbr, ctx->ncount,
                           ctx->max_nbr, m, rho, omega, prm->omega_one);
    else
        hipLaunchKernelGGL((k_density<L, false>), dim3(nb), dim3(kBlock), 0, s, n, ctx->posh64,
                           ctx->posh32, ctx->runid, ctx->grid, ctx->nbr, ctx->ncount,
                           ctx->max_nbr, m, rho, omega, prm->omega_one);
}

int g_lanes_density = 8, g_lanes_gradients = 8, g_lanes_forces = 8;

sph_status launch_density(Ctx *ctx, int64_t n, const double *m, const double *h,
                          const double *u, const int32_t *mat, int32_t nmat,
                          const sph_params *prm, sph_precision prec, double *rho,
                          double *omega, double *P, double *cs, double *T, double *Y,
                          double *Gmod, hipStream_t s) {
    (void)h;
    if (n == 0) return SPH_OK;
    TimedLaunch tl(ctx, SPH_T_DENSITY, s);
    switch (g_lanes_density) {
        case 4: density_launch<4>(ctx, n, m, prec, prm, rho, omega, s); break;
        case 16: density_launch<16>(ctx, n, m, prec, prm, rho, omega, s); break;
        default: density_launch<8>(ctx, n, m, prec, prm, rho, omega, s); break;
    }
    MatTable mt;
    mt.n = nmat;
    for (int k = 0; k < nmat; ++k) mt.m[k] = ctx->mats[k].m;
    hipLaunchKernelGGL(k_eos, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rho, u,
                       mat, mt, P, cs, T, Y, Gmod);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

template <int L, bool F32>
static void grad_launch(Ctx *ctx, int64_t n, hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    R4 *rec0 = (R4 *)ctx->rec;
    void *rec1 = (char *)ctx->rec + sizeof(R4) * (size_t)ctx->capacity;
    hipLaunchKernelGGL((k_gradients<L, F32>), dim3(nb), dim3(kBlock), 0, s, n, ctx->posh64,
                       ctx->posh32, ctx->runid, ctx->grid, ctx->nbr, ctx->ncount, ctx->max_nbr,
                       rec0, rec1, ctx->gsum);
}

sph_status launch_gradients(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                            const double *vz, const double *m, const double *h,
                            const double *rho, const double *omega, const sph_params *prm,
                            sph_precision prec, double *G, int64_t *n_singular, hipStream_t s) {
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const bool f32 = prec == SPH_FP32_CELLREL;
    if (f32) {
        float4 *rec0 = (float4 *)ctx->rec;
        void *rec1 = (char *)ctx->rec + sizeof(float4) * (size_t)ctx->capacity;
        hipLaunchKernelGGL((k_pack_grad<true>), dim3(nb), dim3(256), 0, s, n, vx, vy, vz, m, h,
                           rho, omega, rec0, rec1);
    } else {
        double4 *rec0 = (double4 *)ctx->rec;
        void *rec1 = (char *)ctx->rec + sizeof(double4) * (size_t)ctx->capacity;
        hipLaunchKernelGGL((k_pack_grad<false>), dim3(nb), dim3(256), 0, s, n, vx, vy, vz, m, h,
                           rho, omega, rec0, rec1);
    }
    {
        TimedLaunch tl(ctx, SPH_T_GRADIENTS, s);
        switch (g_lanes_gradients) {
            case 4: f32 ? grad_launch<4, true>(ctx, n, s) : grad_launch<4, false>(ctx, n, s); break;
            case 16: f32 ? grad_launch<16, true>(ctx, n, s) : grad_launch<16, false>(ctx, n, s); break;
            default: f32 ? grad_launch<8, true>(ctx, n, s) : grad_launch<8, false>(ctx, n, s); break;
        }
    }
    hipLaunchKernelGGL(k_grad_epilogue, dim3(nb), dim3(256), 0, s, n, ctx->gsum, ctx->ncount,
                       prm->use_correction_tensor, G, n_singular);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

template <int L, bool F32>
static void forces_launch(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                          double *az, double *dudt, double *dtc, hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_forces<L, F32>), dim3(nb), dim3(kBlock), 0, s, n, ctx->posh64,
                       ctx->posh32, ctx->runid, ctx->grid, ctx->nbr, ctx->ncount, ctx->max_nbr,
                       (const R4 *)ctx->rec, prm->av_alpha, prm->av_beta, prm->av_eps,
                       prm->eta_C, prm->g[0], prm->g[1], prm->g[2], ax, ay, az, dudt, dtc);
}

sph_status launch_forces(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *h, const double *rho,
                         const double *omega, const double *P, const double *cs,
                         const double *S, const sph_params *prm, sph_precision prec,
                         double *ax, double *ay, double *az, double *dudt, double *dtc,
                         hipStream_t s) {
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const bool f32 = prec == SPH_FP32_CELLREL;
    if (f32)
        hipLaunchKernelGGL((k_pack_forces<true>), dim3(nb), dim3(256), 0, s, n, vx, vy, vz, m, h,
                           rho, omega, P, cs, S, (float4 *)ctx->rec);
    else
        hipLaunchKernelGGL((k_pack_forces<false>), dim3(nb), dim3(256), 0, s, n, vx, vy, vz, m,
                           h, rho, omega, P, cs, S, (double4 *)ctx->rec);
    TimedLaunch tl(ctx, SPH_T_FORCES, s);
    switch (g_lanes_forces) {
        case 4:
            f32 ? forces_launch<4, true>(ctx, n, prm, ax, ay, az, dudt, dtc, s)
                : forces_launch<4, false>(ctx, n, prm, ax, ay, az, dudt, dtc, s);
            break;
        case 16:
            f32 ? forces_launch<16, true>(ctx, n, prm, ax, ay, az, dudt, dtc, s)
                : forces_launch<16, false>(ctx, n, prm, ax, ay, az, dudt, dtc, s);
            break;
        default:
            f32 ? forces_launch<8, true>(ctx, n, prm, ax, ay, az, dudt, dtc, s)
                : forces_launch<8, false>(ctx, n, prm, ax, ay, az, dudt, dtc, s);
            break;
    }
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
