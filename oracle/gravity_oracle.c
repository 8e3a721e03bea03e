/*
 * FP64 CPU oracle of the self-gravity and bound-mass support of the batched
 * Q_RD* scan (the gravitational term of the momentum equation in sec. 2.2,
 * and the bound mass of sec. 3 "Catastrophic disruption", found there with
 * SKID by removing unbound particles until nothing changes).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU tree gravity
 * and bound-mass kernels; shares no code with them.  Plain C99, IEEE double,
 * built with -ffp-contract=off; direct O(N^2) summation over ascending j.
 *
 * Readings:
 *   G1  softened Newtonian gravity with a Plummer kernel of length eps:
 *       a_i = G sum_j m_j (x_j - x_i) / (r^2 + eps^2)^(3/2),
 *       phi_i = -G sum_j m_j / (r^2 + eps^2)^(1/2), over j != i of the same
 *       run (runs are independent simulations) and active j only.  The paper
 *       uses pkdgrav3's softened tree gravity; the softening form is not
 *       printed there.
 *   G2  bound mass of a run: start with every particle of the run bound;
 *       repeat { v_c = mass-weighted mean velocity of the bound set,
 *       phi_i from the bound set (G1), particle i leaves the set when
 *       |v_i - v_c|^2 / 2 + phi_i > 0 } until no particle leaves.  Removal
 *       is final.  SKID first splits the particles into density groups; in
 *       a head-on collision the iteration started from the whole run
 *       converges to the largest remnant and what is bound to it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void or_gravity(int64_t n, const double *x, const double *y, const double *z, const double *m,
                const int32_t *active, int32_t nr, const int64_t *run_start, double G,
                double eps, double *ax, double *ay, double *az, double *phi)
{
    const double e2 = eps * eps;
    for (int32_t r = 0; r < nr; ++r) {
        const int64_t a = run_start ? run_start[r] : 0, b = run_start ? run_start[r + 1] : n;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = a; i < b; ++i) {
            double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
            for (int64_t j = a; j < b; ++j) {
                if (j == i || (active && !active[j])) continue;
                const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                const double q = ((dx * dx + dy * dy) + dz * dz) + e2;
                const double inv = 1.0 / sqrt(q);
                const double inv3 = inv / q;
                sx += m[j] * dx * inv3;
                sy += m[j] * dy * inv3;
                sz += m[j] * dz * inv3;
                sp += m[j] * inv;
            }
            if (ax) ax[i] = G * sx;
            if (ay) ay[i] = G * sy;
            if (az) az[i] = G * sz;
            if (phi) phi[i] = -G * sp;
        }
    }
}

/* Returns the number of iterations of the last run; bound[i] = 0/1,
 * m_bound[r] = bound mass of run r. */
int32_t or_bound_mass(int64_t n, const double *x, const double *y, const double *z,
                      const double *vx, const double *vy, const double *vz, const double *m,
                      int32_t nr, const int64_t *run_start, double G, double eps,
                      int32_t max_iter, int32_t *bound, double *m_bound)
{
    double *phi = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t it_last = 0;
    for (int64_t i = 0; i < n; ++i) bound[i] = 1;
    for (int32_t r = 0; r < nr; ++r) {
        const int64_t a = run_start ? run_start[r] : 0, b = run_start ? run_start[r + 1] : n;
        int64_t run_off[2] = {0, b - a};
        int32_t it = 0;
        for (; it < max_iter; ++it) {
            double M = 0.0, px = 0.0, py = 0.0, pz = 0.0;
            for (int64_t i = a; i < b; ++i)
                if (bound[i]) {
                    M += m[i];
                    px += m[i] * vx[i];
                    py += m[i] * vy[i];
                    pz += m[i] * vz[i];
                }
            if (M <= 0.0) break;
            const double cx = px / M, cy = py / M, cz = pz / M;
            or_gravity(b - a, x + a, y + a, z + a, m + a, bound + a, 1, run_off, G, eps, NULL,
                       NULL, NULL, phi + a);
            int64_t left = 0;
            for (int64_t i = a; i < b; ++i) {
                if (!bound[i]) continue;
                const double ux = vx[i] - cx, uy = vy[i] - cy, uz = vz[i] - cz;
                const double e = 0.5 * ((ux * ux + uy * uy) + uz * uz) + phi[i];
                if (e > 0.0) {
                    bound[i] = 0;
                    ++left;
                }
            }
            if (left == 0) break;
        }
        double M = 0.0;
        for (int64_t i = a; i < b; ++i)
            if (bound[i]) M += m[i];
        m_bound[r] = M;
        it_last = it;
    }
    free(phi);
    return it_last;
}
