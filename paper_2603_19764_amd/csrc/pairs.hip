// Pair passes of the strength-SPH hot path on gfx950: density with the
// grad-h term, corrected velocity gradient, forces with the full stress
// tensor and artificial viscosity.  Each particle i is served by a group of
// L consecutive lanes that split i's pair list; per-particle sums are
// combined with cross-lane shuffles.  Before each pass a pack kernel writes
// one record per particle (array of structures, 16-byte slots) holding the
// position and every per-particle value the pair term needs, so a
// neighbour's data is one contiguous gather.  Templates select the
// arithmetic of the pair terms: double on absolute positions, or float on
// positions relative to each particle's cell origin (the separation of a
// pair is (d_i - d_j) - s L with s the stencil offset of j's cell).
//
// Kernel: Wendland C2 with support H = 2h,
//   W = 21/(2 pi H^3) t^4 (1 + 4q),  t = 1 - q,  q = r/H
//   grad_i W = K x_ij,  K = -210/(pi H^5) t^3
//   dW/dh = -21/(pi H^4) t^3 (3 + 9q - 32 q^2)
#include "physics.h"
#include "records.h"

namespace sph {

constexpr double kPi = kPiD;
constexpr int kBlock = 256;

// Record sizes in 16-byte (float) or 32-byte (double) slots.
constexpr int kRecDensity = 1;    // (p, m)
// gradient, force and fused records: slot counts and the (v, m) slots in records.h

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

// Position of sorted particle k: cell-relative float or absolute double.
template <bool F32>
__device__ __forceinline__ void load_p(const double4 *p64, const float4 *p32, int64_t k,
                                       typename Real<F32>::T &x, typename Real<F32>::T &y,
                                       typename Real<F32>::T &z) {
    if constexpr (F32) {
        const float4 q = p32[k];
        x = q.x; y = q.y; z = q.z;
    } else {
        const double4 q = p64[k];
        x = q.x; y = q.y; z = q.z;
    }
}

// Square root and quotient of the pair terms: the hardware instructions
// (v_sqrt_f32, v_rcp_f32; within 1 ulp) in float, IEEE-correct in double.
__device__ __forceinline__ float root(float r2) { return __builtin_amdgcn_sqrtf(r2); }
__device__ __forceinline__ double root(double r2) { return sqrt(r2); }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }

// ================================================================ density
template <bool F32>
__global__ void k_pack_density(int64_t n, const double4 *p64, const float4 *p32,
                               const double *m, typename Real<F32>::T4 *rec) {
    using R = typename Real<F32>::T;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    R x, y, z;
    load_p<F32>(p64, p32, i, x, y, z);
    rec[i] = {x, y, z, (R)m[i]};
}

constexpr int kDensStep = 2;  // pairs per lane evaluated per iteration

template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_density(
    int64_t n, const double4 *__restrict__ posh64, const int16_t *__restrict__ runid,
    const GridDesc *__restrict__ grid, const uint32_t *__restrict__ nbr,
    const int32_t *__restrict__ ncount, int32_t K, const typename Real<F32>::T4 *__restrict__ rec,
    double *__restrict__ rho, double *__restrict__ omega, int32_t omega_one,
    int32_t *__restrict__ flags) {
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
    int nd = 0;  // members of the density set other than i
    double hi = 0.0;
    R4 pi = {0, 0, 0, 0};
    if (active) {
        pi = rec[i];
        hi = posh64[i].w;
        const R Hinv = (R)(0.5 / hi);
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        // An iteration takes kDensStep pairs (k, k + L, ...): their records
        // are loaded together and the next iteration's entries are loaded
        // while they are evaluated.  Entry indices are clamped into the row;
        // a pair past the list is i itself, whose entry has no density flag
        // and adds exact zeros, so every pair of an iteration is evaluated
        // and no branch separates the record loads (their latencies overlap).
        auto body = [&](uint32_t e, const R4 &pj) {
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R q = root(dx * dx + dy * dy + dz * dz) * Hinv;
            R t = (R)1 - q;
            t = t > (R)0 ? t : (R)0;
            const R t3 = t * t * t;
            const bool in_d = (e & kDensityBit) != 0;
            const R mj = in_d ? pj.w : (R)0;
            const R w = mj * (t3 * t * ((R)1 + (R)4 * q));
            const R dh = mj * (t3 * ((R)3 + q * ((R)9 - (R)32 * q)));
            sw += (double)w;
            sd += (double)dh;
            nd += in_d ? 1 : 0;
        };
        auto entry = [&](int k) -> uint32_t {
            const uint32_t v = row[k < K ? k : K - 1];
            return k < c ? v : (uint32_t)i;
        };
        uint32_t e[kDensStep];
#pragma unroll
        for (int u = 0; u < kDensStep; ++u) e[u] = entry(lg + u * L);
        for (int k = lg; k < c; k += kDensStep * L) {
            R4 P[kDensStep];
#pragma unroll
            for (int u = 0; u < kDensStep; ++u) P[u] = rec[e[u] & kIdxMask];
            uint32_t en[kDensStep];
#pragma unroll
            for (int u = 0; u < kDensStep; ++u) en[u] = entry(k + (kDensStep + u) * L);
#pragma unroll
            for (int u = 0; u < kDensStep; ++u) body(e[u], P[u]);
#pragma unroll
            for (int u = 0; u < kDensStep; ++u) e[u] = en[u];
        }
    }
    sw = group_sum<L>(sw);
    sd = group_sum<L>(sd);
    nd = group_sum<L>(nd);
    bool bad = false;
    if (active && lg == 0) {
        const double H = 2.0 * hi;
        const double Wn = 21.0 / (2.0 * kPi * H * H * H);
        const double Dn = -21.0 / (kPi * H * H * H * H);
        const double mi = (double)pi.w;
        const double r = Wn * (mi + sw);           // self term W(0) = Wn
        const double dsum = Dn * (3.0 * mi + sd);  // self term dW/dh(0) = 3 Dn
        // a density set of i alone gives Omega = 0 by the definition (the
        // self term cancels the 1): such a particle takes Omega = 1
        const double om = (omega_one || nd == 0) ? 1.0 : 1.0 + hi / (3.0 * r) * dsum;
        rho[i] = r;
        omega[i] = om;
        bad = nonfinite(r, om);
    }
    flag_if(bad, flags, FLAG_NONFINITE);
}

// -------------------------------------------- EOS, yield, shear modulus
__global__ void k_eos(int64_t n, const double *__restrict__ rho, const double *__restrict__ u,
                      const int32_t *__restrict__ mat, MatTable mt, double *P, double *cs,
                      double *T, double *Y, double *Gmod, int32_t *__restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p, c, t, y, gm;
    material_state(material_of(mt, mat, i), rho[i], u[i], p, c, t, y, gm);
    P[i] = p;
    cs[i] = c;
    T[i] = t;
    Y[i] = y;
    Gmod[i] = gm;
    flag_if(nonfinite(p, c, t, y, gm), flags, FLAG_NONFINITE);
}

// ============================================================== gradients
template <bool F32>
__global__ void k_pack_grad(int64_t n, const double4 *p64, const float4 *p32, const double *vx,
                            const double *vy, const double *vz, const double *m,
                            const double *rho, const double *omega,
                            typename Real<F32>::T4 *rec) {
    using R = typename Real<F32>::T;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    R x, y, z;
    load_p<F32>(p64, p32, i, x, y, z);
    const double H = 2.0 * p64[i].w;
    const double kn = -210.0 / (kPi * H * H * H * H * H);
    typename Real<F32>::T4 *r = rec + kRecGradSlots<F32> * i;
    r[0] = {x, y, z, (R)(1.0 / H)};
    store_vm<F32>(r + 1, vx[i], vy[i], vz[i], m[i]);
    r[1 + kVelSlots<F32>] = {(R)(kn / (omega[i] * rho[i])), (R)0, (R)0, (R)0};
}

// Raw sums per particle (15 rows): C^-1 (xx, yy, zz, xy, xz, yz) and F (row-major 9).
template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_gradients(
    int64_t n, const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const typename Real<F32>::T4 *__restrict__ rec, double *__restrict__ gsum) {
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
    R c_xx = 0, c_yy = 0, c_zz = 0, c_xy = 0, c_xz = 0, c_yz = 0;
    R f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
        const R4 pi = rec[kRecGradSlots<F32> * i];
        const VM<R> vi = load_vm<F32, R>(rec + kRecGradSlots<F32> * i + 1);
        const R ai = rec[kRecGradSlots<F32> * i + 1 + kVelSlots<F32>].x;
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        uint32_t en = lg < c ? row[lg] : 0u;
        for (int k = lg; k < c; k += L) {
            const uint32_t e = en;
            en = k + L < c ? row[k + L] : 0u;  // next entry in flight
            const R4 *rj = rec + kRecGradSlots<F32> * (int64_t)(e & kIdxMask);
            const R4 pj = rj[0];
            const VM<R> vj = load_vm<F32, R>(rj + 1);
            const R aj = rj[1 + kVelSlots<F32>].x;
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R r = root(dx * dx + dy * dy + dz * dz);
            R ti = (R)1 - r * pi.w, tj = (R)1 - r * pj.w;
            ti = ti > (R)0 ? ti : (R)0;
            tj = tj > (R)0 ? tj : (R)0;
            // -w = -1/2 m_j (K_i/(Om rho)_i + K_j/(Om rho)_j)
            const R nw = (R)(-0.5) * vj.m * (ai * ti * ti * ti + aj * tj * tj * tj);
            const R ux = (R)(vi.x - vj.x), uy = (R)(vi.y - vj.y), uz = (R)(vi.z - vj.z);
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
                                double *__restrict__ G, int64_t *n_singular,
                                int32_t *__restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int sing = 0;
    bool bad = false;
    if (i < n) {
        double ci[6], F[9], g[9];
        for (int k = 0; k < 6; ++k) ci[k] = gsum[k * n + i];
        for (int k = 0; k < 9; ++k) F[k] = gsum[(6 + k) * n + i];
        sing = corrected_gradient(ci, F, ncount[i], use_corr, g) ? 0 : (use_corr ? 1 : 0);
        for (int k = 0; k < 9; ++k) G[k * n + i] = g[k];
        bad = nonfinite(g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7], g[8]);
    }
    flag_if(bad, flags, FLAG_NONFINITE);
    if (n_singular) {
        const uint64_t m = __ballot(sing);
        if (m && (threadIdx.x % kWave) == 0) atomicAdd((unsigned long long *)n_singular,
                                                       (unsigned long long)__popcll(m));
    }
}

// ================================================================= forces
// A = (-P I + S)/(Omega rho^2) and Kn = -210/(pi H^5): K(r,h) A = t^3 (Kn A).
template <bool F32>
__global__ void k_pack_forces(int64_t n, const double4 *p64, const float4 *p32, const double *vx,
                              const double *vy, const double *vz, const double *m,
                              const double *rho, const double *omega, const double *P,
                              const double *cs, const double *S, typename Real<F32>::T4 *rec) {
    using R = typename Real<F32>::T;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    R x, y, z;
    load_p<F32>(p64, p32, i, x, y, z);
    const double h = p64[i].w;
    const double H = 2.0 * h;
    const double kn = -210.0 / (kPi * H * H * H * H * H);
    const double sc = kn / (omega[i] * rho[i] * rho[i]);
    const double sxx = S[i], syy = S[n + i], sxy = S[2 * n + i], sxz = S[3 * n + i],
                 syz = S[4 * n + i];
    const double p = P[i];
    typename Real<F32>::T4 *r = rec + kRecForceSlots<F32> * i;
    constexpr int o = kVelSlots<F32>;
    r[0] = {x, y, z, (R)(1.0 / H)};
    store_vm<F32>(r + 1, vx[i], vy[i], vz[i], m[i]);
    r[1 + o] = {(R)(sc * (sxx - p)), (R)(sc * (syy - p)), (R)(sc * (-sxx - syy - p)), (R)(sc * sxy)};
    r[2 + o] = {(R)(sc * sxz), (R)(sc * syz), (R)rho[i], (R)cs[i]};
    r[3 + o] = {(R)kn, (R)h, (R)0, (R)0};
}

template <int L, bool F32>
__global__ __launch_bounds__(kBlock) void k_forces(
    int64_t n, const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const typename Real<F32>::T4 *__restrict__ rec, double al, double be, double eps,
    double etaC, double gx, double gy, double gz, double *__restrict__ ax,
    double *__restrict__ ay, double *__restrict__ az, double *__restrict__ dudt,
    double *__restrict__ dtc, int32_t *__restrict__ flags) {
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
    R4 Bi = {0, 0, 0, 0}, Hi = {0, 0, 0, 0};
    if (active) {
        constexpr int o = kVelSlots<F32>;
        const R4 *ri = rec + kRecForceSlots<F32> * i;
        const R4 pi = ri[0], Ai = ri[1 + o];
        const VM<R> vi = load_vm<F32, R>(ri + 1);
        Bi = ri[2 + o];
        Hi = ri[3 + o];
        const R ral = (R)al, rbe = (R)be, reps = (R)eps;
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        uint32_t en = lg < c ? row[lg] : 0u;
        for (int k = lg; k < c; k += L) {
            const uint32_t e = en;
            en = k + L < c ? row[k + L] : 0u;  // next entry in flight
            const R4 *rj = rec + kRecForceSlots<F32> * (int64_t)(e & kIdxMask);
            const R4 pj = rj[0], Aj = rj[1 + o], Bj = rj[2 + o], Hj = rj[3 + o];
            const VM<R> vj = load_vm<F32, R>(rj + 1);
            R dx, dy, dz;
            separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
            const R r2 = dx * dx + dy * dy + dz * dz;
            const R r = root(r2);
            R ti = (R)1 - r * pi.w, tj = (R)1 - r * pj.w;
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
            const R mj = vj.m;
            acx += mj * (ti3 * yix + tj3 * yjx);
            acy += mj * (ti3 * yiy + tj3 * yjy);
            acz += mj * (ti3 * yiz + tj3 * yjz);
            const R ux = (R)(vi.x - vj.x), uy = (R)(vi.y - vj.y), uz = (R)(vi.z - vj.z);
            du -= mj * ti3 * (ux * yix + uy * yiy + uz * yiz);
            const R vr = ux * dx + uy * dy + uz * dz;
            if (vr < (R)0) {
                const R hb = (R)0.5 * (Hi.y + Hj.y);
                const R mu = quot(hb * vr, r2 + reps * hb * hb);
                const R cb = (R)0.5 * (Bi.w + Bj.w);
                const R rb = (R)0.5 * (Bi.z + Bj.z);
                const R Pi = quot(-ral * cb * mu + rbe * mu * mu, rb);
                const R gw = (R)0.5 * (Hi.x * ti3 + Hj.x * tj3);  // mean K
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
    bool bad = false;
    if (active && lg == 0) {
        const double hi = (double)Hi.y;
        const double ci = (double)Bi.w;
        const double d = etaC * hi / ((1.0 + 0.6 * al) * ci + 0.6 * be * (double)mumax);
        ax[i] = (double)acx + gx;
        ay[i] = (double)acy + gy;
        az[i] = (double)acz + gz;
        dudt[i] = (double)du;
        dtc[i] = d;
        bad = nonfinite((double)acx, (double)acy, (double)acz, (double)du, d);
    }
    flag_if(bad, flags, FLAG_NONFINITE);
}

// ==================================================== gradients + forces
// The force pass needs only density-pass quantities and the rescaled
// predicted stress, not the velocity gradient, so the whole-step path
// evaluates both sums in one sweep over the pair lists.  Record (5 slots,
// written by the whole-step state kernel; A = sigma/(Omega rho^2)):
//   (p, 1/H) (v, m) (m Kn A: xx yy zz xy) (m Kn A: xz yz, rho/2, c/2)
//   (-m Kn/(2 Omega rho), m Kn/2, h/2, 1/m).
// Depth 1 keeps one neighbour record in registers: 79 VGPRs in float (six
// waves per SIMD, against four at 104 with two records) and 138 in double
// (three waves against two).
// Neighbour j's factors are used as stored; particle i's are divided by m_i
// once, so every pair term carries m_j without a product of its own:
//   -w_ij    = (m_j t_i^3) G_i + t_j^3 G'_j          (G = -Kn/(2 Omega rho))
//   dv_i    += (m_j t_i^3) (Kn A)_i x_ij + t_j^3 (m Kn A)_j x_ij
//   du_i    -= (m_j t_i^3) v_ij . (Kn A)_i x_ij
// and the viscosity term takes one reciprocal, of D rho_bar with
// D = r^2 + eps h_bar^2:  mu = h_bar v.x rho_bar / (D rho_bar),
// Pi = mu (beta mu - alpha c_bar) D / (D rho_bar).

template <int L, bool F32, int Depth>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(Depth == 1 ? (F32 ? 6 : 3) : 1, 8))) void k_grad_forces(
    int64_t n, const int16_t *__restrict__ runid, const GridDesc *__restrict__ grid,
    const uint32_t *__restrict__ nbr, const int32_t *__restrict__ ncount, int32_t K,
    const typename Real<F32>::T4 *__restrict__ rec, double al, double be, double eps,
    double etaC, double gx, double gy, double gz, void *__restrict__ gsum_v,
    double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az,
    double *__restrict__ dudt, double *__restrict__ dtc, const int32_t *__restrict__ act,
    int32_t *__restrict__ flags) {
    using R = typename Real<F32>::T;
    using R4 = typename Real<F32>::T4;
    __shared__ float shs[81];
    if constexpr (F32) {
        stencil_offsets(shs);
        __syncthreads();
    }
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kBlock / L) + threadIdx.x / L;
    const int lg = threadIdx.x % L;
    const bool active = i < n && (!act || act[i]);
    R c_xx = 0, c_yy = 0, c_zz = 0, c_xy = 0, c_xz = 0, c_yz = 0;
    R f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    R acx = 0, acy = 0, acz = 0, du = 0, mumax = 0;
    R hi2 = 0, ci2 = 0;
    if (active) {
        constexpr int o = kVelSlots<F32>;
        const R4 *ri = rec + kRecBothStride<F32> * i;
        const R4 pi = ri[0], A2 = ri[1 + o], B2 = ri[2 + o], H2 = ri[3 + o];
        const VM<R> vi = load_vm<F32, R>(ri + 1);
        const R im = H2.w;
        const R4 Ai = {A2.x * im, A2.y * im, A2.z * im, A2.w * im};
        const R bix = B2.x * im, biy = B2.y * im;
        const R Gi = H2.x * im, Xi = H2.y * im;
        hi2 = H2.z;
        ci2 = B2.w;
        const R ri2 = B2.z;
        const R ral = (R)al, rbe = (R)be, reps = (R)eps;
        float L32 = 0.f;
        if constexpr (F32) L32 = grid[runid[i]].L32;
        const int c = ncount[i];
        const uint32_t *row = nbr + i * (int64_t)K;
        // Depth 2: software pipeline (see k_density): entry two ahead, record
        // one ahead, unconditional loads; two record sets take turns, so no
        // copies between iterations.  Depth 1: one record set, the next
        // entry in flight (fewer registers, more waves per SIMD).
        auto body = [&](uint32_t e, const R4 &pj, const VM<R> &vj, const R4 &Aj, const R4 &Bj,
                        const R4 &Hj) {
                R dx, dy, dz;
                separation<F32>(pi, pj, e, shs, L32, dx, dy, dz);
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R r = root(r2);
                R ti = (R)1 - r * pi.w, tj = (R)1 - r * pj.w;
                ti = ti > (R)0 ? ti : (R)0;
                tj = tj > (R)0 ? tj : (R)0;
                const R ti3 = ti * ti * ti, tj3 = tj * tj * tj;
                const R mti = vj.m * ti3;
                const R ux = (R)(vi.x - vj.x), uy = (R)(vi.y - vj.y), uz = (R)(vi.z - vj.z);
                // gradient sums
                const R nw = mti * Gi + tj3 * Hj.x;
                const R wx = nw * dx, wy = nw * dy, wz = nw * dz;
                c_xx += wx * dx; c_yy += wy * dy; c_zz += wz * dz;
                c_xy += wx * dy; c_xz += wx * dz; c_yz += wy * dz;
                f[0] += ux * wx; f[1] += ux * wy; f[2] += ux * wz;
                f[3] += uy * wx; f[4] += uy * wy; f[5] += uy * wz;
                f[6] += uz * wx; f[7] += uz * wy; f[8] += uz * wz;
                // forces
                const R yix = Ai.x * dx + Ai.w * dy + bix * dz;
                const R yiy = Ai.w * dx + Ai.y * dy + biy * dz;
                const R yiz = bix * dx + biy * dy + Ai.z * dz;
                const R yjx = Aj.x * dx + Aj.w * dy + Bj.x * dz;
                const R yjy = Aj.w * dx + Aj.y * dy + Bj.y * dz;
                const R yjz = Bj.x * dx + Bj.y * dy + Aj.z * dz;
                acx += mti * yix; acx += tj3 * yjx;
                acy += mti * yiy; acy += tj3 * yjy;
                acz += mti * yiz; acz += tj3 * yjz;
                du -= mti * (ux * yix + uy * yiy + uz * yiz);
                const R vr = ux * dx + uy * dy + uz * dz;
                if (vr < (R)0) {
                    const R hb = hi2 + Hj.z;
                    const R D = r2 + reps * hb * hb;
                    const R rb = ri2 + Bj.z;
                    const R inv = quot((R)1, D * rb);
                    const R mu = hb * vr * rb * inv;
                    const R Pi = mu * (rbe * mu - ral * (ci2 + Bj.w)) * (D * inv);
                    const R sv = (mti * Xi + tj3 * Hj.y) * Pi;  // m_j Pi mean K
                    acx -= sv * dx;
                    acy -= sv * dy;
                    acz -= sv * dz;
                    du += (R)0.5 * sv * vr;
                    mumax = mumax > -mu ? mumax : -mu;
                }
        };
        auto entry = [&](int k) -> uint32_t {
            const uint32_t v = row[k < K ? k : K - 1];
            return k < c ? v : (uint32_t)i;
        };
        if constexpr (Depth == 2) {
            uint32_t e0 = entry(lg), e1 = entry(lg + L);
            R4 P0, A0, B0, H0, P1, A1, B1, H1;
            VM<R> V0, V1;
            {
                const R4 *rj = rec + kRecBothStride<F32> * (int64_t)(e0 & kIdxMask);
                P0 = rj[0]; V0 = load_vm<F32, R>(rj + 1); A0 = rj[1 + o]; B0 = rj[2 + o]; H0 = rj[3 + o];
            }
            for (int k = lg; k < c; k += 2 * L) {
                const uint32_t e2 = entry(k + 2 * L);
                {
                    const R4 *rj = rec + kRecBothStride<F32> * (int64_t)(e1 & kIdxMask);
                    P1 = rj[0]; V1 = load_vm<F32, R>(rj + 1); A1 = rj[1 + o]; B1 = rj[2 + o]; H1 = rj[3 + o];
                }
                body(e0, P0, V0, A0, B0, H0);
                if (k + L >= c) break;
                const uint32_t e3 = entry(k + 3 * L);
                {
                    const R4 *rj = rec + kRecBothStride<F32> * (int64_t)(e2 & kIdxMask);
                    P0 = rj[0]; V0 = load_vm<F32, R>(rj + 1); A0 = rj[1 + o]; B0 = rj[2 + o]; H0 = rj[3 + o];
                }
                body(e1, P1, V1, A1, B1, H1);
                e0 = e2;
                e1 = e3;
            }
    
        } else {
            uint32_t en = entry(lg);
            for (int k = lg; k < c; k += L) {
                const uint32_t e = en;
                en = entry(k + L);  // next entry in flight
                const R4 *rj = rec + kRecBothStride<F32> * (int64_t)(e & kIdxMask);
                const R4 Pj = rj[0], Aj = rj[1 + o], Bj = rj[2 + o], Hj = rj[3 + o];
                const VM<R> Vj = load_vm<F32, R>(rj + 1);
                body(e, Pj, Vj, Aj, Bj, Hj);
            }
        }
    }
    c_xx = group_sum<L>(c_xx); c_yy = group_sum<L>(c_yy); c_zz = group_sum<L>(c_zz);
    c_xy = group_sum<L>(c_xy); c_xz = group_sum<L>(c_xz); c_yz = group_sum<L>(c_yz);
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = group_sum<L>(f[a]);
    acx = group_sum<L>(acx);
    acy = group_sum<L>(acy);
    acz = group_sum<L>(acz);
    du = group_sum<L>(du);
    mumax = group_max<L>(mumax);
    bool bad = false;
    if (active && lg == 0) {
        // the raw sums in the sweep's own precision (exact: they are
        // accumulated in it)
        R *o = (R *)gsum_v + i;
        o[0 * n] = c_xx; o[1 * n] = c_yy; o[2 * n] = c_zz;
        o[3 * n] = c_xy; o[4 * n] = c_xz; o[5 * n] = c_yz;
#pragma unroll
        for (int a = 0; a < 9; ++a) o[(6 + a) * n] = f[a];
        const double hi = 2.0 * (double)hi2;
        const double ci = 2.0 * (double)ci2;
        const double d = etaC * hi / ((1.0 + 0.6 * al) * ci + 0.6 * be * (double)mumax);
        ax[i] = (double)acx + gx;
        ay[i] = (double)acy + gy;
        az[i] = (double)acz + gz;
        dudt[i] = (double)du;
        dtc[i] = d;
        // non-finite gradient sums show in G (checked with the stress rate)
        bad = nonfinite((double)acx, (double)acy, (double)acz, (double)du, d);
    }
    flag_if(bad, flags, FLAG_NONFINITE);
}

// =============================================================== launches
static int lanes_of(const Ctx *ctx, int knob, bool f32) { return ctx->lanes[knob][f32 ? 1 : 0]; }

template <int L, bool F32>
static void density_launch(Ctx *ctx, int64_t n, const sph_params *prm, double *rho,
                           double *omega, hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_density<L, F32>), dim3(nb), dim3(kBlock), 0, s, n, ctx->posh64,
                       ctx->runid, ctx->grid, ctx->nbr, ctx->ncount, nbr_stride(ctx),
                       (const R4 *)ctx->rec_d, rho, omega, prm->omega_one, ctx->flags);
}

template <bool F32>
static void density_dispatch(Ctx *ctx, int64_t n, const sph_params *prm, double *rho,
                             double *omega, hipStream_t s) {
    switch (lanes_of(ctx, SPH_TUNE_LANES_DENSITY, F32)) {
        case 4: density_launch<4, F32>(ctx, n, prm, rho, omega, s); break;
        case 16: density_launch<16, F32>(ctx, n, prm, rho, omega, s); break;
        default: density_launch<8, F32>(ctx, n, prm, rho, omega, s); break;
    }
}

sph_status launch_density_pairs(Ctx *ctx, int64_t n, const sph_params *prm, sph_precision prec,
                                double *rho, double *omega, hipStream_t s) {
    if (n == 0) return SPH_OK;
    TimedLaunch tl(ctx, SPH_T_DENSITY, s);
    prec == SPH_FP32_CELLREL ? density_dispatch<true>(ctx, n, prm, rho, omega, s)
                             : density_dispatch<false>(ctx, n, prm, rho, omega, s);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_density(Ctx *ctx, int64_t n, const double *m, const double *h,
                          const double *u, const int32_t *mat, int32_t nmat,
                          const sph_params *prm, sph_precision prec, double *rho,
                          double *omega, double *P, double *cs, double *T, double *Y,
                          double *Gmod, hipStream_t s) {
    (void)h;
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const bool f32 = prec == SPH_FP32_CELLREL;
    if (f32)
        hipLaunchKernelGGL((k_pack_density<true>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, m, (float4 *)ctx->rec_d);
    else
        hipLaunchKernelGGL((k_pack_density<false>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, m, (double4 *)ctx->rec_d);
    sph_status st = launch_density_pairs(ctx, n, prm, prec, rho, omega, s);
    if (st != SPH_OK) return st;
    MatTable mt;
    mt.n = nmat;
    for (int k = 0; k < nmat; ++k) mt.m[k] = ctx->mats[k].m;
    hipLaunchKernelGGL(k_eos, dim3(nb), dim3(256), 0, s, n, rho, u, mat, mt, P, cs, T, Y, Gmod,
                       ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

template <int L, bool F32>
static void grad_launch(Ctx *ctx, int64_t n, hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_gradients<L, F32>), dim3(nb), dim3(kBlock), 0, s, n, ctx->runid,
                       ctx->grid, ctx->nbr, ctx->ncount, nbr_stride(ctx), (const R4 *)ctx->rec_g,
                       ctx->gsum);
}

template <bool F32>
static void grad_dispatch(Ctx *ctx, int64_t n, hipStream_t s) {
    switch (lanes_of(ctx, SPH_TUNE_LANES_GRADIENTS, F32)) {
        case 4: grad_launch<4, F32>(ctx, n, s); break;
        case 16: grad_launch<16, F32>(ctx, n, s); break;
        default: grad_launch<8, F32>(ctx, n, s); break;
    }
}

sph_status launch_gradient_pairs(Ctx *ctx, int64_t n, sph_precision prec, hipStream_t s) {
    if (n == 0) return SPH_OK;
    TimedLaunch tl(ctx, SPH_T_GRADIENTS, s);
    prec == SPH_FP32_CELLREL ? grad_dispatch<true>(ctx, n, s) : grad_dispatch<false>(ctx, n, s);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_gradients(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                            const double *vz, const double *m, const double *h,
                            const double *rho, const double *omega, const sph_params *prm,
                            sph_precision prec, double *G, int64_t *n_singular, hipStream_t s) {
    (void)h;
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const bool f32 = prec == SPH_FP32_CELLREL;
    if (f32)
        hipLaunchKernelGGL((k_pack_grad<true>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, vx, vy, vz, m, rho, omega, (float4 *)ctx->rec_g);
    else
        hipLaunchKernelGGL((k_pack_grad<false>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, vx, vy, vz, m, rho, omega, (double4 *)ctx->rec_g);
    sph_status st = launch_gradient_pairs(ctx, n, prec, s);
    if (st != SPH_OK) return st;
    hipLaunchKernelGGL(k_grad_epilogue, dim3(nb), dim3(256), 0, s, n, ctx->gsum, ctx->ncount,
                       prm->use_correction_tensor, G, n_singular, ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

template <int L, bool F32>
static void forces_launch(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                          double *az, double *dudt, double *dtc, hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_forces<L, F32>), dim3(nb), dim3(kBlock), 0, s, n, ctx->runid, ctx->grid,
                       ctx->nbr, ctx->ncount, nbr_stride(ctx), (const R4 *)ctx->rec_f, prm->av_alpha,
                       prm->av_beta, prm->av_eps, prm->eta_C, prm->g[0], prm->g[1], prm->g[2], ax,
                       ay, az, dudt, dtc, ctx->flags);
}

template <bool F32>
static void forces_dispatch(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                            double *az, double *dudt, double *dtc, hipStream_t s) {
    switch (lanes_of(ctx, SPH_TUNE_LANES_FORCES, F32)) {
        case 4: forces_launch<4, F32>(ctx, n, prm, ax, ay, az, dudt, dtc, s); break;
        case 16: forces_launch<16, F32>(ctx, n, prm, ax, ay, az, dudt, dtc, s); break;
        default: forces_launch<8, F32>(ctx, n, prm, ax, ay, az, dudt, dtc, s); break;
    }
}

sph_status launch_forces(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *h, const double *rho,
                         const double *omega, const double *P, const double *cs,
                         const double *S, const sph_params *prm, sph_precision prec,
                         double *ax, double *ay, double *az, double *dudt, double *dtc,
                         hipStream_t s) {
    (void)h;
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)((n + 255) / 256);
    const bool f32 = prec == SPH_FP32_CELLREL;
    if (f32)
        hipLaunchKernelGGL((k_pack_forces<true>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, vx, vy, vz, m, rho, omega, P, cs, S, (float4 *)ctx->rec_f);
    else
        hipLaunchKernelGGL((k_pack_forces<false>), dim3(nb), dim3(256), 0, s, n, ctx->posh64,
                           ctx->posh32, vx, vy, vz, m, rho, omega, P, cs, S, (double4 *)ctx->rec_f);
    return launch_force_pairs(ctx, n, prm, prec, ax, ay, az, dudt, dtc, s);
}

template <int L, bool F32, int D>
static void both_launch(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                        double *az, double *dudt, double *dtc, const int32_t *act,
                        hipStream_t s) {
    using R4 = typename Real<F32>::T4;
    const int nb = (int)((n * L + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_grad_forces<L, F32, D>), dim3(nb), dim3(kBlock), 0, s, n, ctx->runid,
                       ctx->grid, ctx->nbr, ctx->ncount, nbr_stride(ctx), (const R4 *)ctx->rec_f,
                       prm->av_alpha, prm->av_beta, prm->av_eps, prm->eta_C, prm->g[0], prm->g[1],
                       prm->g[2], ctx->gsum, ax, ay, az, dudt, dtc, act, ctx->flags);
}

template <bool F32, int D>
static void both_dispatch_d(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                            double *az, double *dudt, double *dtc, const int32_t *act,
                            hipStream_t s) {
    switch (lanes_of(ctx, SPH_TUNE_LANES_STEP, F32)) {
        case 4: both_launch<4, F32, D>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s); break;
        case 16: both_launch<16, F32, D>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s); break;
        default: both_launch<8, F32, D>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s); break;
    }
}

template <bool F32>
static void both_dispatch(Ctx *ctx, int64_t n, const sph_params *prm, double *ax, double *ay,
                          double *az, double *dudt, double *dtc, const int32_t *act,
                          hipStream_t s) {
    if (ctx->sweep_depth[F32 ? 1 : 0] == 1)
        both_dispatch_d<F32, 1>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s);
    else
        both_dispatch_d<F32, 2>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s);
}

// Gradient raw sums and forces in one sweep (records written by the
// whole-step state kernel into rec_f).
sph_status launch_grad_force_pairs(Ctx *ctx, int64_t n, const sph_params *prm,
                                   sph_precision prec, double *ax, double *ay, double *az,
                                   double *dudt, double *dtc, hipStream_t s,
                                   const int32_t *act) {
    if (n == 0) return SPH_OK;
    TimedLaunch tl(ctx, SPH_T_FORCES, s);
    prec == SPH_FP32_CELLREL ? both_dispatch<true>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s)
                             : both_dispatch<false>(ctx, n, prm, ax, ay, az, dudt, dtc, act, s);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_force_pairs(Ctx *ctx, int64_t n, const sph_params *prm, sph_precision prec,
                              double *ax, double *ay, double *az, double *dudt, double *dtc,
                              hipStream_t s) {
    if (n == 0) return SPH_OK;
    TimedLaunch tl(ctx, SPH_T_FORCES, s);
    prec == SPH_FP32_CELLREL ? forces_dispatch<true>(ctx, n, prm, ax, ay, az, dudt, dtc, s)
                             : forces_dispatch<false>(ctx, n, prm, ax, ay, az, dudt, dtc, s);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
