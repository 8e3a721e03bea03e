// Fused per-particle kernels of the whole strength-SPH step (sec. 2.4
// sequence).  The public pass entry points keep their own kernels; the step
// path merges the per-particle work around the three pair passes so that
// each particle's state is read from HBM once per phase:
//   reorder + predictor          (Predict_S eq. applied to v, u)
//   state                        (EOS, T, yield, Gamma, stress predictor and
//                                 rescaling, gradient and force records)
//   gradient epilogue + rate     (Corrected_Gradients eq., Jaumann rate,
//                                 strain-rate invariant)
//   kicks                        (closing kick with rescaling, opening kick)
#include "physics.h"
#include "records.h"

namespace sph {

// --------------------------------------------------- reorder + predictor
// The predictor interval tau of each particle: half the run's step with one
// step per run; with individual steps (hier) the time elapsed in the
// particle's own step (advanced here by the run's substep; predict = 2: not
// advanced, a repeated reorder of the same step) less half of that step,
// and act = 1 where the step ends now.  predict = 0 (start of a run):
// tau = 0, every particle evaluated.
// The rows of the individual steps (SPH_DTP, SPH_EL, the last two) are
// carried only when they are in use (hier).
__global__ void k_reorder_predict(int64_t n, const int32_t *__restrict__ perm, StepRows r,
                                  const double *__restrict__ dtp,
                                  const int16_t *__restrict__ runid, int32_t predict,
                                  int32_t hier, double tick, double *__restrict__ vpx,
                                  double *__restrict__ vpy, double *__restrict__ vpz,
                                  double *__restrict__ up, double *__restrict__ tau,
                                  int32_t *__restrict__ act) {
    static_assert(SPH_DTP == SPH_NF64 - 2 && SPH_EL == SPH_NF64 - 1, "step rows last");
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t o = perm[k];
    double f[SPH_NF64];
#pragma unroll
    for (int c = 0; c < SPH_NF64; ++c) {
        if (c < SPH_DTP || hier) {
            f[c] = r.f_src[c][o];
            r.f_dst[c][k] = f[c];
        } else {
            f[c] = 0.0;
        }
    }
    int32_t fx = 0;
#pragma unroll
    for (int c = 0; c < SPH_NI32; ++c) {
        const int32_t v = r.i_src[c][o];
        r.i_dst[c][k] = v;
        if (c == SPH_FIXED) fx = v;
    }
    double hd = 0.0;
    int32_t a = 1;
    if (predict && hier) {
        a = 0;
        if (!fx) {
            const double el = f[SPH_EL] + (predict == 1 ? rint(dt_of(dtp, runid, k) / tick) : 0.0);
            r.f_dst[SPH_EL][k] = el;
            hd = (el - 0.5 * f[SPH_DTP]) * tick;
            a = el == f[SPH_DTP] ? 1 : 0;
        }
    } else if (predict && !fx) {
        hd = 0.5 * dt_of(dtp, runid, k);
    }
    tau[k] = hd;
    act[k] = a;
    vpx[k] = f[SPH_VX] + hd * f[SPH_AX];
    vpy[k] = f[SPH_VY] + hd * f[SPH_AY];
    vpz[k] = f[SPH_VZ] + hd * f[SPH_AZ];
    up[k] = f[SPH_U] + hd * f[SPH_DUDT];
}

// ------------------------------------------------------------------ state
// Record of the fused gradient + force pass (5 slots, 6 in the FP32 form
// whose (v, m) takes two, see records.h): (p, 1/H) (v, m)
// (m Kn A xx yy zz xy) (m Kn A xz yz, rho/2, c/2)
// (-m Kn/(2 Omega rho), m Kn/2, h/2, 1/m) with
// A = (-P I + S_pred)/(Omega rho^2), Kn = -210/(pi H^5).
// threads of a k_state block (its records staged in LDS: 24 KB in the
// FP32 form, 20 KB in the FP64 form)
template <bool F32>
constexpr int kStateBlock = F32 ? 256 : 128;

template <bool F32>
__global__ __launch_bounds__(kStateBlock<F32>) void k_state(int64_t n, const double4 *__restrict__ posh64,
                        const float4 *__restrict__ posh32, const double *__restrict__ rho,
                        const double *__restrict__ omega, const double *__restrict__ up,
                        const double *__restrict__ vpx, const double *__restrict__ vpy,
                        const double *__restrict__ vpz, const double *__restrict__ m,
                        const int32_t *__restrict__ mat, const int32_t *__restrict__ fixed,
                        MatTable mt, const double *__restrict__ tau,
                        const double *__restrict__ S_half, const double *__restrict__ Sdot,
                        double *__restrict__ P, double *__restrict__ cs, double *__restrict__ T,
                        double *__restrict__ Y, double *__restrict__ Gmod,
                        double *__restrict__ S_pred, void *rec_f_v,
                        int32_t *__restrict__ flags) {
    using R = typename std::conditional<F32, float, double>::type;
    using R4 = typename std::conditional<F32, float4, double4>::type;
    constexpr int kS = kRecBothStride<F32>;
    constexpr int kB = kStateBlock<F32>;
    // records (96 B in the FP32 form, 160 B in the FP64 form) are assembled
    // in LDS and written by the block as one contiguous span (each lane's
    // slot stores would otherwise fall a record apart)
    __shared__ R4 stg[kB * kS];
    const int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x;
    if (i < n) {
    const sph_material &M = material_of(mt, mat, i);
    const double r = rho[i], om = omega[i];
    double p, c, t, y, gm;
    material_state(M, r, up[i], p, c, t, y, gm);
    P[i] = p;
    cs[i] = c;
    T[i] = t;
    Y[i] = y;
    Gmod[i] = gm;
    const double hd = tau[i];
    double s[5];
    for (int k = 0; k < 5; ++k) s[k] = S_half[k * n + i] + hd * Sdot[k * n + i];
    plastic_return(s, y);
    for (int k = 0; k < 5; ++k) S_pred[k * n + i] = s[k];
    flag_if(nonfinite(p, c, t, y, gm, s[0], s[1], s[2], s[3], s[4]), flags, FLAG_NONFINITE);
    // records
    const double4 q64 = posh64[i];
    R px, py, pz;
    if constexpr (F32) {
        const float4 q = posh32[i];
        px = q.x; py = q.y; pz = q.z;
    } else {
        px = q64.x; py = q64.y; pz = q64.z;
    }
    // (p, 1/H) (v, m) (m Kn A: xx yy zz xy) (m Kn A: xz yz, rho/2, c/2)
    // (-m Kn/(2 Omega rho), m Kn/2, h/2, 1/m), A = sigma/(Omega rho^2): the
    // sweep uses j's terms as stored and i's divided by m_i once
    const double H = 2.0 * q64.w;
    const double mi = m[i];
    const double kn = -210.0 / (kPiD * H * H * H * H * H);
    const double sc = mi * kn / (om * r * r);
    R4 *rf = stg + kS * threadIdx.x;
    constexpr int o = kVelSlots<F32>;
    rf[0] = {px, py, pz, (R)(1.0 / H)};
    store_vm<F32>(rf + 1, vpx[i], vpy[i], vpz[i], mi);
    rf[1 + o] = {(R)(sc * (s[0] - p)), (R)(sc * (s[1] - p)), (R)(sc * (-s[0] - s[1] - p)),
                 (R)(sc * s[2])};
    rf[2 + o] = {(R)(sc * s[3]), (R)(sc * s[4]), (R)(0.5 * r), (R)(0.5 * c)};
    rf[3 + o] = {(R)(-0.5 * mi * kn / (om * r)), (R)(0.5 * mi * kn), (R)(0.5 * q64.w),
                 (R)(mi > 0.0 ? 1.0 / mi : 0.0)};
    }
    __syncthreads();
    const int64_t b0 = blockIdx.x * (int64_t)kB;
    const int64_t left = n - b0;
    const int cnt = kS * (int)(left < kB ? left : kB);
    R4 *dst = (R4 *)rec_f_v + kS * b0;
    for (int q = threadIdx.x; q < cnt; q += kB) dst[q] = stg[q];
}

// ------------------------------------------- gradient epilogue + stress rate
__global__ void k_grad_rate(int64_t n, const void *__restrict__ gsum_v, int32_t gsum_f32,
                            const int32_t *__restrict__ ncount, int32_t use_corr,
                            const double *__restrict__ S_pred, const double *__restrict__ Gmod,
                            const int32_t *__restrict__ fixed, double rot,
                            const double *__restrict__ tau, const int32_t *__restrict__ act,
                            double *__restrict__ G, double *__restrict__ Sdot,
                            double *__restrict__ eps2, int64_t *n_singular,
                            int32_t *__restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int sing = 0;
    bool bad = false;
    if (i < n && (!act || act[i])) {
        double ci[6], F[9], g[9], s[5], ds[5], e2;
        // raw sums of the fused sweep: float in the FP32 form, else double
        const float *g32 = (const float *)gsum_v;
        const double *g64 = (const double *)gsum_v;
        for (int k = 0; k < 15; ++k) {
            const double v = gsum_f32 ? (double)g32[k * n + i] : g64[k * n + i];
            if (k < 6) ci[k] = v; else F[k - 6] = v;
        }
        sing = corrected_gradient(ci, F, ncount[i], use_corr, g) ? 0 : (use_corr ? 1 : 0);
        for (int k = 0; k < 9; ++k) G[k * n + i] = g[k];
        for (int k = 0; k < 5; ++k) s[k] = S_pred[k * n + i];
        stress_rate(g, s, Gmod[i], rot, ds, e2);
        for (int k = 0; k < 5; ++k) Sdot[k * n + i] = ds[k];
        bad = nonfinite(g[0], g[1], g[2], g[3], g[4], g[5], g[6], g[7], g[8]) |
              nonfinite(ds[0], ds[1], ds[2], ds[3], ds[4]);
        // the step that ends here is twice the predictor interval
        if (eps2 && !(fixed && fixed[i])) eps2[i] += 2.0 * tau[i] * e2;
    }
    flag_if(bad, flags, FLAG_NONFINITE);
    if (n_singular) {
        const uint64_t mk = __ballot(sing);
        if (mk && (threadIdx.x % kWave) == 0)
            atomicAdd((unsigned long long *)n_singular, (unsigned long long)__popcll(mk));
    }
}

// ------------------------------------------------------------------ kicks
// mode 0: closing kick with rescaling then opening kick (a step);
// mode 1: opening kick from the predicted stress (start of a run).
// The next step of a run is its CFL minimum (bit pattern, capped) read
// here directly; threads r < nr also store it to dt_next[r] for the next
// step's drift and clear bits_clear[r] for the next reduction.
__device__ __forceinline__ double dt_from_bits(unsigned long long b, double cap) {
    double d = __longlong_as_double((long long)b);
    return (cap > 0.0 && !(d <= cap)) ? cap : d;
}

__global__ void k_kick_all(int64_t n, int32_t mode, const double *__restrict__ dtp,
                           const unsigned long long *__restrict__ bits_cur, double dt_cap,
                           double *__restrict__ dt_next, unsigned long long *__restrict__ bits_clear,
                           int32_t nr, const int16_t *__restrict__ runid,
                           const int32_t *__restrict__ fixed,
                           double *vx, double *vy, double *vz, double *u,
                           const double *__restrict__ ax, const double *__restrict__ ay,
                           const double *__restrict__ az, const double *__restrict__ dudt,
                           double *S_half, const double *__restrict__ S_pred,
                           const double *__restrict__ Sdot, const double *__restrict__ Y,
                           int32_t *__restrict__ flags, double *__restrict__ time) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nr) {
        dt_next[i] = dt_from_bits(bits_cur[i], dt_cap);
        bits_clear[i] = 0x7ff0000000000000ull;
        // the run's time: 0 at the start of a run, else advanced by its step
        if (time) time[i] = mode == 0 ? time[i] + dtp[i] : 0.0;
    }
    if (i >= n) return;
    if (fixed && fixed[i]) return;
    const double hn = 0.5 * dt_from_bits(bits_cur[runid ? (int)runid[i] : 0], dt_cap);
    if (mode == 0) {
        const double hd = 0.5 * dt_of(dtp, runid, i);
        vx[i] = (vx[i] + hd * ax[i]) + hn * ax[i];
        vy[i] = (vy[i] + hd * ay[i]) + hn * ay[i];
        vz[i] = (vz[i] + hd * az[i]) + hn * az[i];
        u[i] = (u[i] + hd * dudt[i]) + hn * dudt[i];
        double s[5], d[5];
        for (int k = 0; k < 5; ++k) {
            d[k] = Sdot[k * n + i];
            s[k] = S_half[k * n + i] + hd * d[k];
        }
        plastic_return(s, Y[i]);
        for (int k = 0; k < 5; ++k) S_half[k * n + i] = s[k] + hn * d[k];
    } else {
        vx[i] += hn * ax[i];
        vy[i] += hn * ay[i];
        vz[i] += hn * az[i];
        u[i] += hn * dudt[i];
        for (int k = 0; k < 5; ++k) S_half[k * n + i] = S_pred[k * n + i] + hn * Sdot[k * n + i];
    }
    flag_if(nonfinite(vx[i], vy[i], vz[i], u[i], S_half[i], S_half[n + i], S_half[2 * n + i],
                      S_half[3 * n + i], S_half[4 * n + i]),
            flags, FLAG_NONFINITE);
}

// ------------------------------------------------ acceleration criterion
// dt_i <- min(dt_i, eta_a sqrt(h_i / |a_i|)) once a is complete (after
// gravity), for the particles evaluated.
__global__ void k_accel_limit(int64_t n, double eta_a, const double *__restrict__ ax,
                              const double *__restrict__ ay, const double *__restrict__ az,
                              const double *__restrict__ h, const int32_t *__restrict__ act,
                              double *__restrict__ dtc) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || (act && !act[i])) return;
    const double a = sqrt((ax[i] * ax[i] + ay[i] * ay[i]) + az[i] * az[i]);
    if (a > 0.0) {
        const double d = eta_a * sqrt(h[i] / a);
        if (d < dtc[i]) dtc[i] = d;
    }
}

// --------------------------------------------------- individual steps
// Step of a particle in ticks: the longest 2^(rungs-1-r) ticks whose
// duration does not exceed its own step d (the shortest rung if none,
// flagged), longer than its current step cur only where the run's time t
// (ticks) is a multiple of it.
__device__ __forceinline__ double rung_ticks(int rungs, double tick, double d, double t,
                                             double cur, int32_t *flags) {
    double st = ldexp(1.0, rungs - 1);
    while (st > 1.0 && st * tick > d) st *= 0.5;
    if (st * tick > d) flags[FLAG_RUNG_CLAMP] = 1;
    while (st > cur && fmod(t, st) != 0.0) st *= 0.5;
    return st;
}

// Particles whose step ends (act): closing kick with rescaling (not at the
// start of a run), the next step, opening kick, elapsed time reset.  Every
// particle that is not fixed then leaves the duration to the end of its
// step in rem (the next substep of its run is the minimum).
__global__ void k_kick_hier(int64_t n, int32_t init, int32_t rungs, double tick,
                            const double *__restrict__ dtp, const double *__restrict__ clock,
                            const int16_t *__restrict__ runid, const int32_t *__restrict__ fixed,
                            const int32_t *__restrict__ act, double *vx, double *vy, double *vz,
                            double *u, const double *__restrict__ ax, const double *__restrict__ ay,
                            const double *__restrict__ az, const double *__restrict__ dudt,
                            double *S_half, const double *__restrict__ S_pred,
                            const double *__restrict__ Sdot, const double *__restrict__ Y,
                            const double *__restrict__ dtc, double *step, double *elapsed,
                            double *rem, int32_t *flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (fixed && fixed[i]) {
        rem[i] = 0.0;
        return;
    }
    if (!act[i]) {
        rem[i] = (step[i] - elapsed[i]) * tick;
        return;
    }
    const int r = runid ? (int)runid[i] : 0;
    const double top = ldexp(1.0, rungs - 1);
    double s[5], d[5];
    for (int k = 0; k < 5; ++k) d[k] = Sdot[k * n + i];
    double cur = top, t = 0.0;
    if (init) {
        for (int k = 0; k < 5; ++k) s[k] = S_pred[k * n + i];
    } else {
        const double hd = 0.5 * step[i] * tick;
        vx[i] += hd * ax[i];
        vy[i] += hd * ay[i];
        vz[i] += hd * az[i];
        u[i] += hd * dudt[i];
        for (int k = 0; k < 5; ++k) s[k] = S_half[k * n + i] + hd * d[k];
        plastic_return(s, Y[i]);
        cur = step[i];
        t = clock[r] + rint(dtp[r] / tick);
    }
    const double st = rung_ticks(rungs, tick, dtc[i], t, cur, flags);
    const double hn = 0.5 * st * tick;
    vx[i] += hn * ax[i];
    vy[i] += hn * ay[i];
    vz[i] += hn * az[i];
    u[i] += hn * dudt[i];
    for (int k = 0; k < 5; ++k) S_half[k * n + i] = s[k] + hn * d[k];
    step[i] = st;
    elapsed[i] = 0.0;
    rem[i] = st * tick;
    flag_if(nonfinite(vx[i], vy[i], vz[i], u[i], S_half[i], S_half[n + i], S_half[2 * n + i],
                      S_half[3 * n + i], S_half[4 * n + i]),
            flags, FLAG_NONFINITE);
}

// Per run: the next substep from the reduced minimum, the run's clock
// advanced by the substep just taken (set to 0 at the start of a run), the
// other minima buffer cleared.
__global__ void k_hier_next(int32_t nr, int32_t init, double tick,
                            const unsigned long long *__restrict__ bits_cur,
                            unsigned long long *bits_clear, const double *__restrict__ dt,
                            double *dt_next, double *clock, double *time) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    dt_next[r] = __longlong_as_double((long long)bits_cur[r]);
    clock[r] = init ? 0.0 : clock[r] + rint(dt[r] / tick);
    if (time) time[r] = clock[r] * tick;   // whole ticks: exact
    bits_clear[r] = 0x7ff0000000000000ull;
}

// -------------------------------------------------------------- launches
sph_status launch_step_reorder(Ctx *ctx, int64_t n, const int32_t *perm, const StepRows &r,
                               const double *dt, const int16_t *runid, int32_t predict,
                               int32_t hier, double tick, double *vpx, double *vpy, double *vpz,
                               double *up, double *tau, int32_t *act, hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_reorder_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       perm, r, dt, runid, predict, hier, tick, vpx, vpy, vpz, up, tau, act);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_step_state(Ctx *ctx, int64_t n, sph_precision prec, const double *rho,
                             const double *omega, const double *up, const double *vpx,
                             const double *vpy, const double *vpz, const double *m,
                             const int32_t *mat, int32_t nmat, const int32_t *fixed,
                             const double *tau, const double *S_half,
                             const double *Sdot, double *P, double *cs, double *T, double *Y,
                             double *Gmod, double *S_pred, hipStream_t s) {
    if (n == 0) return SPH_OK;
    MatTable mt;
    mt.n = nmat;
    for (int k = 0; k < nmat; ++k) mt.m[k] = ctx->mats[k].m;
    if (prec == SPH_FP32_CELLREL)
        hipLaunchKernelGGL((k_state<true>), dim3((unsigned)((n + 255) / 256)),
                           dim3(kStateBlock<true>), 0, s, n, ctx->posh64,
                           ctx->posh32, rho, omega, up, vpx, vpy, vpz, m, mat, fixed, mt, tau,
                           S_half, Sdot, P, cs, T, Y, Gmod, S_pred, ctx->rec_f, ctx->flags);
    else
        hipLaunchKernelGGL((k_state<false>), dim3((unsigned)((n + 127) / 128)),
                           dim3(kStateBlock<false>), 0, s, n, ctx->posh64,
                           ctx->posh32, rho, omega, up, vpx, vpy, vpz, m, mat, fixed, mt, tau,
                           S_half, Sdot, P, cs, T, Y, Gmod, S_pred, ctx->rec_f, ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_step_grad_rate(Ctx *ctx, int64_t n, const sph_params *prm, int32_t gsum_f32,
                                 const double *S_pred, const double *Gmod, const int32_t *fixed,
                                 const double *tau, const int32_t *act, double *G,
                                 double *Sdot, double *eps2,
                                 int64_t *n_singular, hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_grad_rate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (const void *)ctx->gsum, gsum_f32, ctx->ncount, prm->use_correction_tensor, S_pred, Gmod, fixed,
                       prm->rot_sign, tau, act, G, Sdot, eps2, n_singular, ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_step_kick(Ctx *ctx, int64_t n, int32_t mode, const double *dt,
                            const unsigned long long *bits_cur, double dt_cap,
                            double *dt_next, unsigned long long *bits_clear, int32_t nr,
                            const int16_t *runid, const int32_t *fixed, double *vx, double *vy,
                            double *vz, double *u, const double *ax, const double *ay,
                            const double *az, const double *dudt, double *S_half,
                            const double *S_pred, const double *Sdot, const double *Y,
                            double *time, hipStream_t s) {
    const int64_t m = n > nr ? n : nr;
    if (m == 0) return SPH_OK;
    hipLaunchKernelGGL(k_kick_all, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, n, mode,
                       dt, bits_cur, dt_cap, dt_next, bits_clear, nr, runid, fixed, vx, vy, vz, u,
                       ax, ay, az, dudt, S_half, S_pred, Sdot, Y, ctx->flags, time);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_accel_limit(Ctx *ctx, int64_t n, double eta_a, const double *ax,
                              const double *ay, const double *az, const double *h,
                              const int32_t *act, double *dtc, hipStream_t s) {
    (void)ctx;
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_accel_limit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       eta_a, ax, ay, az, h, act, dtc);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_kick_hier(Ctx *ctx, int64_t n, int32_t init, int32_t rungs, double tick,
                            const double *dt, const double *clock, const int16_t *runid,
                            const int32_t *fixed, const int32_t *act, double *vx, double *vy,
                            double *vz, double *u, const double *ax, const double *ay,
                            const double *az, const double *dudt, double *S_half,
                            const double *S_pred, const double *Sdot, const double *Y,
                            const double *dtc, double *step, double *elapsed, double *rem,
                            hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_kick_hier, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, init,
                       rungs, tick, dt, clock, runid, fixed, act, vx, vy, vz, u, ax, ay, az, dudt,
                       S_half, S_pred, Sdot, Y, dtc, step, elapsed, rem, ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_hier_next(Ctx *ctx, int32_t nr, int32_t init, double tick,
                            const unsigned long long *bits_cur, unsigned long long *bits_clear,
                            const double *dt, double *dt_next, double *clock, double *time,
                            hipStream_t s) {
    (void)ctx;
    hipLaunchKernelGGL(k_hier_next, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, nr,
                       init, tick, bits_cur, bits_clear, dt, dt_next, clock, time);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
