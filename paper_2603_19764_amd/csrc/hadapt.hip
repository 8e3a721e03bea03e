// Adaptive smoothing lengths (the kernel-mass equation of sec. 2.1): h_i
// such that (4/3) pi (2 h_i)^3 rho_i(h_i) = N_ngb m_i, by Newton-Raphson on
//   f(h) = (32 pi / 3) h^3 rho(h) - N_ngb m_i,
//   f'(h) = 32 pi h^2 rho(h) + (32 pi / 3) h^3 drho/dh  (= 32 pi h^2 rho Omega),
// each step limited to a factor 2 and to the searched length.  The sums run
// over the pair lists of the last neighbour search, built with lengths
// h_search >= the answer; every j closer than 2h <= 2 h_search is on i's
// list.  FP64 throughout, the membership test r^2 < (2h)^2 on the exact
// squared separation.
#include "sph_internal.h"

namespace sph {

constexpr int kAdaptL = 8;
constexpr int kAdaptBlock = 256;
constexpr double kPiA = 3.14159265358979323846;

__global__ __launch_bounds__(kAdaptBlock) void k_adapt_h(
    int64_t n, const double4 *__restrict__ posh64, const uint32_t *__restrict__ nbr,
    const int32_t *__restrict__ ncount, int32_t K, const double *__restrict__ m,
    const double *__restrict__ h_start, const int32_t *__restrict__ fixed, double n_ngb,
    double tol, int32_t max_iter, double *__restrict__ h_out, unsigned long long *n_clamped,
    int32_t *iterations) {
    constexpr int L = kAdaptL;
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (kAdaptBlock / L) + threadIdx.x / L;
    const int lg = threadIdx.x % L;
    const bool active = i < n;
    double xi = 0.0, yi = 0.0, zi = 0.0, hs = 0.0, mi = 0.0, h = 0.0;
    int c = 0;
    const uint32_t *row = nbr;
    if (active) {
        const double4 p = posh64[i];
        xi = p.x; yi = p.y; zi = p.z; hs = p.w;
        mi = m[i];
        h = fmin(h_start[i], hs);
        c = ncount[i];
        row = nbr + i * (int64_t)K;
    }
    bool done = !active || (fixed && fixed[i]);  // fixed particles keep h_start
    int it = 0;
    // every lane runs the same number of rounds so that the group shuffles
    // stay converged; finished groups add zeros
    for (int round = 0; round < max_iter; ++round) {
        const bool any = __ballot(!done) != 0;
        if (!any) break;
        double rho = 0.0, drho = 0.0;
        if (!done) {
            const double H = 2.0 * h;
            const double H2 = __dmul_rn(H, H);
            const double invH = 1.0 / H;
            for (int k = lg; k < c; k += L) {
                const uint32_t e = row[k];
                const double4 q = posh64[e & kIdxMask];
                const double r2 = sep2_exact(xi, yi, zi, q.x, q.y, q.z);
                if (!(r2 < H2)) continue;
                const double r = sqrt(r2);
                const double s = r * invH;
                const double t = 1.0 - s;
                const double t3 = t * t * t;
                const double mj = m[e & kIdxMask];
                rho += mj * (t3 * t * (1.0 + 4.0 * s));
                drho += mj * (t3 * (3.0 + s * (9.0 - 32.0 * s)));
            }
        }
        rho = group_sum<L>(rho);
        drho = group_sum<L>(drho);
        if (!done) {
            // normalisations: W = 21/(2 pi H^3) (...), dW/dh = -21/(pi H^4) (...)
            const double H = 2.0 * h;
            const double Wn = 21.0 / (2.0 * kPiA * H * H * H);
            const double Dn = -21.0 / (kPiA * H * H * H * H);
            const double rh = Wn * (mi + rho);          // self term W(0) = Wn
            const double dr = Dn * (3.0 * mi + drho);   // self term dW/dh(0) = 3 Dn
            const double f = (32.0 * kPiA / 3.0) * h * h * h * rh - n_ngb * mi;
            const double fp = 32.0 * kPiA * h * h * rh + (32.0 * kPiA / 3.0) * h * h * h * dr;
            double hn = fp > 0.0 ? h - f / fp : 2.0 * h;
            hn = fmin(fmax(hn, 0.5 * h), 2.0 * h);
            ++it;
            if (hn > hs) {
                // beyond the searched range: continue from its edge, and stop
                // there if the next step wants to leave it again
                if (h == hs) {
                    done = true;
                    if (lg == 0 && n_clamped) atomicAdd(n_clamped, 1ull);
                }
                hn = hs;
            }
            const double dh = hn - h;
            h = hn;
            if (fabs(dh) <= tol * h) done = true;
        }
    }
    if (active && lg == 0) {
        h_out[i] = (fixed && fixed[i]) ? h_start[i] : h;
        if (iterations) atomicMax(iterations, it);
    }
}

sph_status launch_adapt_h(Ctx *ctx, int64_t n, const double *m, const double *h_start,
                          const int32_t *fixed, double n_ngb, double tol, int32_t max_iter,
                          double *h_out, int64_t *n_clamped, int32_t *iterations,
                          hipStream_t s) {
    if (n == 0) return SPH_OK;
    const int64_t per = kAdaptBlock / kAdaptL;
    hipLaunchKernelGGL(k_adapt_h, dim3((unsigned)((n + per - 1) / per)), dim3(kAdaptBlock), 0, s,
                       n, ctx->posh64, ctx->nbr, ctx->ncount, nbr_stride(ctx), m, h_start, fixed,
                       n_ngb, tol, max_iter, h_out, (unsigned long long *)n_clamped, iterations);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

__global__ void k_scale(int64_t n, const double *__restrict__ a, double f, double *__restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = f * a[i];
}

sph_status launch_scale(Ctx *ctx, int64_t n, const double *a, double f, double *b,
                        hipStream_t s) {
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, f, b);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
