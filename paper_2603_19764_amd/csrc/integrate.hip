// Per-particle phases of the strength-SPH step on gfx950 (HBM-bound
// streams, one thread per particle, all in double): predictor and plastic
// rescaling of the deviatoric stress (Predict_S eq., Deviatoric_stress_
// rescaling eq.), Jaumann stress rate (Deviatoric_Stress_derivative eq.),
// closing and opening kicks (sec. 2.4), drift, global time step from the
// CFL condition, and conservation diagnostics.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "physics.h"

namespace sph {

__global__ void k_stress(int32_t phase, int64_t n, const double *__restrict__ dtp,
                         const double *__restrict__ dtnp, const double *__restrict__ G,
                         const double *__restrict__ Y, const double *__restrict__ Gmod,
                         const int32_t *__restrict__ fixed, double rot, double *S_half,
                         double *S_pred, double *Sdot, double *eps2,
                         int32_t *__restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fx = fixed && fixed[i];
    if (phase == SPH_STRESS_PREDICT) {
        const double hd = 0.5 * *dtp;
        double s[5];
        for (int c = 0; c < 5; ++c)
            s[c] = fx ? S_half[c * n + i] : S_half[c * n + i] + hd * Sdot[c * n + i];
        plastic_return(s, Y[i]);
        for (int c = 0; c < 5; ++c) S_pred[c * n + i] = s[c];
        flag_if(nonfinite(s[0], s[1], s[2], s[3], s[4]), flags, FLAG_NONFINITE);
    } else if (phase == SPH_STRESS_RATE) {
        double g[9];
        for (int c = 0; c < 9; ++c) g[c] = G[c * n + i];
        const double sxx = S_pred[i], syy = S_pred[n + i], sxy = S_pred[2 * n + i],
                     sxz = S_pred[3 * n + i], syz = S_pred[4 * n + i];
        const double S[3][3] = {{sxx, sxy, sxz}, {sxy, syy, syz}, {sxz, syz, -sxx - syy}};
        double E[3][3], R[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                E[a][b] = 0.5 * (g[3 * a + b] + g[3 * b + a]);
                R[a][b] = 0.5 * (g[3 * a + b] - g[3 * b + a]);
            }
        const double tr3 = (E[0][0] + E[1][1] + E[2][2]) / 3.0;
        const double gm = Gmod[i];
        const int ia[5] = {0, 1, 0, 0, 1}, ib[5] = {0, 1, 1, 2, 2};
        bool bad = false;
        for (int c = 0; c < 5; ++c) {
            const int a = ia[c], b = ib[c];
            double rs = 0.0, sr = 0.0;
            for (int k = 0; k < 3; ++k) {
                rs += R[a][k] * S[k][b];
                sr += S[a][k] * R[k][b];
            }
            const double d = 2.0 * gm * (E[a][b] - (a == b ? tr3 : 0.0)) + rot * (rs - sr);
            Sdot[c * n + i] = d;
            bad |= nonfinite(d);
        }
        flag_if(bad, flags, FLAG_NONFINITE);
    } else if (phase == SPH_STRESS_KICK) {
        if (fx) return;
        const double dt = *dtp, hd = 0.5 * dt, hn = 0.5 * *dtnp;
        double s[5], d[5];
        for (int c = 0; c < 5; ++c) {
            d[c] = Sdot[c * n + i];
            s[c] = S_half[c * n + i] + hd * d[c];
        }
        plastic_return(s, Y[i]);
        bool bad = false;
        for (int c = 0; c < 5; ++c) {
            S_half[c * n + i] = s[c] + hn * d[c];
            bad |= nonfinite(s[c] + hn * d[c]);
        }
        flag_if(bad, flags, FLAG_NONFINITE);
        if (eps2) {
            double ee = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double e = 0.5 * (G[(3 * a + b) * n + i] + G[(3 * b + a) * n + i]);
                    ee += e * e;
                }
            eps2[i] += dt * (0.5 * ee);
        }
    } else {  // opening kick from the predicted stress (start of a run)
        if (fx) return;
        const double hn = 0.5 * *dtnp;
        bool bad = false;
        for (int c = 0; c < 5; ++c) {
            const double v = S_pred[c * n + i] + hn * Sdot[c * n + i];
            S_half[c * n + i] = v;
            bad |= nonfinite(v);
        }
        flag_if(bad, flags, FLAG_NONFINITE);
    }
}

sph_status launch_stress(Ctx *ctx, int32_t phase, int64_t n, const double *dt,
                         const double *dt_next, const double *G, const double *Y,
                         const double *Gmod, const int32_t *fixed, const sph_params *prm,
                         double *S_half, double *S_pred, double *Sdot, double *eps2,
                         hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_stress, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phase, n, dt,
                       dt_next, G, Y, Gmod, fixed, prm->rot_sign, S_half, S_pred, Sdot, eps2,
                       ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

__global__ void k_kick_drift(int32_t phase, int64_t n, const double *__restrict__ dtp,
                             const double *__restrict__ dtnp, const int32_t *__restrict__ fixed,
                             double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, double *u, const double *ax, const double *ay,
                             const double *az, const double *dudt, double *vpx, double *vpy,
                             double *vpz, double *up, int32_t *__restrict__ flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fx = fixed && fixed[i];
    if (phase == SPH_KD_DRIFT) {
        if (fx) return;
        const double dt = *dtp;
        x[i] += dt * vx[i];
        y[i] += dt * vy[i];
        z[i] += dt * vz[i];
        flag_if(nonfinite(x[i], y[i], z[i]), flags, FLAG_NONFINITE);
    } else if (phase == SPH_KD_PREDICT) {
        const double hd = fx ? 0.0 : 0.5 * *dtp;
        if (fx) {
            vpx[i] = vx[i]; vpy[i] = vy[i]; vpz[i] = vz[i]; up[i] = u[i];
        } else {
            vpx[i] = vx[i] + hd * ax[i];
            vpy[i] = vy[i] + hd * ay[i];
            vpz[i] = vz[i] + hd * az[i];
            up[i] = u[i] + hd * dudt[i];
        }
        flag_if(nonfinite(vpx[i], vpy[i], vpz[i], up[i]), flags, FLAG_NONFINITE);
    } else if (phase == SPH_KD_KICK) {
        if (fx) return;
        const double hd = 0.5 * *dtp, hn = 0.5 * *dtnp;
        vx[i] = (vx[i] + hd * ax[i]) + hn * ax[i];
        vy[i] = (vy[i] + hd * ay[i]) + hn * ay[i];
        vz[i] = (vz[i] + hd * az[i]) + hn * az[i];
        u[i] = (u[i] + hd * dudt[i]) + hn * dudt[i];
        flag_if(nonfinite(vx[i], vy[i], vz[i], u[i]), flags, FLAG_NONFINITE);
    } else {  // opening kick only (start of a run)
        if (fx) return;
        const double hn = 0.5 * *dtnp;
        vx[i] += hn * ax[i];
        vy[i] += hn * ay[i];
        vz[i] += hn * az[i];
        u[i] += hn * dudt[i];
        flag_if(nonfinite(vx[i], vy[i], vz[i], u[i]), flags, FLAG_NONFINITE);
    }
}

sph_status launch_kick_drift(Ctx *ctx, int32_t phase, int64_t n, const double *dt,
                             const double *dt_next, const int32_t *fixed, double *x, double *y,
                             double *z, double *vx, double *vy, double *vz, double *u,
                             const double *ax, const double *ay, const double *az,
                             const double *dudt, double *vpx, double *vpy, double *vpz,
                             double *up, hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phase, n,
                       dt, dt_next, fixed, x, y, z, vx, vy, vz, u, ax, ay, az, dudt, vpx, vpy,
                       vpz, up, ctx->flags);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

// ------------------------------------------------------------ dt minimum
// Positive doubles order like their bit patterns, so an integer atomicMin on
// the bits is an exact, order-independent minimum.
// One minimum per run: blockIdx.y is the run, whose particles are the
// contiguous range [run_p[r], run_p[r+1]) of the sorted order (the whole
// range [0, n) when run_p is null).
constexpr int kDtUnroll = 4;

__global__ void k_dt_reduce(int64_t n, const int32_t *__restrict__ run_p,
                            const double *__restrict__ dtc, const int32_t *__restrict__ fixed,
                            const GridDesc *__restrict__ far_grid,
                            const int32_t *__restrict__ cell_count,
                            unsigned long long *bits_all, int32_t *__restrict__ flags) {
    const int r = blockIdx.y;
    const int64_t a = run_p ? run_p[r] : 0;
    int64_t b = run_p ? run_p[r + 1] : n;
    if (far_grid) {  // the run's particles outside its far cube (sorted last) take no part,
                     // unless no other is left (then they set the step of their flight)
        const GridDesc g = far_grid[r];
        if (g.sink && b - cell_count[far_key(g)] > a) b -= cell_count[far_key(g)];
    }
    unsigned long long *bits = bits_all + r;
    unsigned long long best = 0x7ff0000000000000ull;
    bool bad = false;  // a NaN step (skipped by the minimum, reported)
    // kDtUnroll independent loads in flight per thread
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < b;
         i0 += kDtUnroll * stride) {
        double d[kDtUnroll];
#pragma unroll
        for (int u = 0; u < kDtUnroll; ++u) {
            const int64_t i = i0 + u * stride;
            const bool ok = i < b && !(fixed && fixed[i]);
            d[u] = ok ? dtc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kDtUnroll; ++u) {
            bad |= d[u] != d[u];
            if (d[u] > 0.0) {
                const unsigned long long v = (unsigned long long)__double_as_longlong(d[u]);
                best = v < best ? v : best;
            }
        }
    }
    flag_if(bad, flags, FLAG_NONFINITE);
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = __shfl_xor(best, o);
        best = v < best ? v : best;
    }
    __shared__ unsigned long long wmin[16];
    if ((threadIdx.x % kWave) == 0) wmin[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (unsigned w = 1; w < blockDim.x / kWave; ++w) best = wmin[w] < best ? wmin[w] : best;
        if (best != 0x7ff0000000000000ull) atomicMin(bits, best);
    }
}

__global__ void k_dt_final(int nr, unsigned long long *bits, double cap, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double d = __longlong_as_double((long long)bits[r]);
    if (cap > 0.0 && !(d <= cap)) d = cap;
    out[r] = d;
    bits[r] = 0x7ff0000000000000ull;  // ready for the next reduction
}

sph_status launch_dt_reduce(Ctx *ctx, int64_t n, const double *dtc, const int32_t *fixed,
                            unsigned long long *bits, hipStream_t s, int32_t nr,
                            const int32_t *run_p, bool skip_far) {
    if (nr < 1 || nr > ctx->max_runs || (nr > 1 && !run_p)) return SPH_EINVAL;
    if (n > 0) {
        // about kDtUnroll elements per thread, at most 64 blocks (one atomic
        // each) per run
        int nb = (int)((n / nr + 1024 * kDtUnroll - 1) / (1024 * kDtUnroll));
        const int cap_b = 64;
        nb = nb < 1 ? 1 : (nb > cap_b ? cap_b : nb);
        hipLaunchKernelGGL(k_dt_reduce, dim3(nb, nr), dim3(1024), 0, s, n, nr > 1 ? run_p : nullptr,
                           dtc, fixed, (skip_far && ctx->far_built) ? ctx->grid : nullptr,
                           ctx->cell_count, bits, ctx->flags);
    }
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_dt_min(Ctx *ctx, int64_t n, const double *dtc, const int32_t *fixed,
                         double cap, double *out, hipStream_t s, int32_t nr,
                         const int32_t *run_p) {
    sph_status e = launch_dt_reduce(ctx, n, dtc, fixed, ctx->dtbits, s, nr, run_p);
    if (e != SPH_OK) return e;
    hipLaunchKernelGGL(k_dt_final, dim3((nr + 255) / 256), dim3(256), 0, s, nr, ctx->dtbits, cap,
                       out);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

__global__ void k_copy_scalar(const double *src, double *dst) { *dst = *src; }

// ------------------------------------------------------------ diagnostics
constexpr int kDiagBlocks = 256;
__global__ void k_diag(int64_t n, const double *x, const double *y, const double *z,
                       const double *vx, const double *vy, const double *vz, const double *m,
                       const double *ax, const double *ay, const double *az, const double *du,
                       double *part) {
    double acc[13] = {0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double mi = m[i];
        const double X[3] = {x[i], y[i], z[i]}, V[3] = {vx[i], vy[i], vz[i]},
                     A[3] = {ax[i], ay[i], az[i]};
        for (int d = 0; d < 3; ++d) acc[d] += mi * A[d];
        acc[3] += mi * (X[1] * A[2] - X[2] * A[1]);
        acc[4] += mi * (X[2] * A[0] - X[0] * A[2]);
        acc[5] += mi * (X[0] * A[1] - X[1] * A[0]);
        acc[6] += mi * (V[0] * A[0] + V[1] * A[1] + V[2] * A[2] + du[i]);
        for (int d = 0; d < 3; ++d) acc[7 + d] += mi * V[d];
        acc[10] += mi * (X[1] * V[2] - X[2] * V[1]);
        acc[11] += mi * (X[2] * V[0] - X[0] * V[2]);
        acc[12] += mi * (X[0] * V[1] - X[1] * V[0]);
    }
    __shared__ double sh[13][256];
    for (int k = 0; k < 13; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            for (int k = 0; k < 13; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 13) part[blockIdx.x * 13 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_diag_final(const double *part, double *out) {
    const int k = threadIdx.x;
    if (k >= 13) return;
    double s = 0.0;
    for (int b = 0; b < kDiagBlocks; ++b) s += part[b * 13 + k];
    out[k] = s;
}

// The two kernels of the diagnostics with the partial sums in `part`
// (kDiagBlocks x 13 doubles, every entry written before it is read).
static void diag_kernels(int64_t n, const double *x, const double *y, const double *z,
                         const double *vx, const double *vy, const double *vz, const double *m,
                         const double *ax, const double *ay, const double *az,
                         const double *dudt, double *part, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag, dim3(kDiagBlocks), dim3(256), 0, s, n, x, y, z, vx, vy, vz, m, ax,
                       ay, az, dudt, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, part, out);
}

sph_status launch_diag(Ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                       const double *vx, const double *vy, const double *vz, const double *m,
                       const double *ax, const double *ay, const double *az,
                       const double *dudt, double *out, hipStream_t s) {
    diag_kernels(n, x, y, z, vx, vy, vz, m, ax, ay, az, dudt, ctx->diag, out, s);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

// ------------------------------------- diagnostics without a context
// The partial sums of sph_diagnostics_noalloc live in this array (26,624
// bytes).  Host code never passes its name to a kernel: the device address
// of each GPU's copy is looked up once per device, with that device
// current, and kept in g_scratch.
constexpr int kNoAllocDoubles = kDiagBlocks * 13;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch[kNoAllocMaxDevices];
static thread_local char g_noalloc_err[256];

static sph_status noalloc_fail(sph_status code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_noalloc_err, sizeof g_noalloc_err, fmt, ap);
    va_end(ap);
    return code;
}

const char *noalloc_last_error() { return g_noalloc_err[0] ? g_noalloc_err : nullptr; }

// Device address of the current device's scratch (looked up on first use).
static sph_status noalloc_scratch(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return noalloc_fail(SPH_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return noalloc_fail(SPH_EINVAL, "device %d beyond the %d supported", dev,
                            kNoAllocMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(SPH_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                hipGetErrorString(e));
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return SPH_OK;
}

}  // namespace sph

extern "C" sph_status sph_diagnostics_noalloc(int64_t n, const double *x, const double *y,
                                              const double *z, const double *vx,
                                              const double *vy, const double *vz,
                                              const double *m, const double *ax,
                                              const double *ay, const double *az,
                                              const double *dudt, double *out13,
                                              sph_stream stream) {
    using namespace sph;
    g_noalloc_err[0] = 0;
    if (n < 0 || n > SPH_NOALLOC_MAX_N)
        return noalloc_fail(SPH_EINVAL, "sph_diagnostics_noalloc: n = %lld outside [0, %lld]",
                            (long long)n, (long long)SPH_NOALLOC_MAX_N);
    if (!out13 || (n > 0 && !(x && y && z && vx && vy && vz && m && ax && ay && az && dudt)))
        return noalloc_fail(SPH_EINVAL, "sph_diagnostics_noalloc: null array");
    double *part = nullptr;
    sph_status st = noalloc_scratch(&part);
    if (st != SPH_OK) return st;
    diag_kernels(n, x, y, z, vx, vy, vz, m, ax, ay, az, dudt, part, out13, (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return noalloc_fail(SPH_EHIP, "sph_diagnostics_noalloc launch: %s", hipGetErrorString(e));
    return SPH_OK;
}

namespace sph {

__global__ void k_copy_u64(const unsigned long long *src, unsigned long long *dst) { *dst = *src; }

sph_status launch_copy_u64(Ctx *ctx, const unsigned long long *src, unsigned long long *dst,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(1), 0, s, src, dst);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

sph_status launch_copy_scalar(Ctx *ctx, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, src, dst);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
