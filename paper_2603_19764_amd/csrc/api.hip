// C-ABI entry points of the strength-SPH library: argument checks, context
// scratch, and the whole-step sequence of sec. 2.4 built from the pass
// launches.  Everything is asynchronous on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "sph_internal.h"

struct sph_ctx {
    sph::Ctx c;
    std::vector<int64_t> run_cache;  // host copy of the run layout on the device
};

namespace sph {

void set_error(Ctx *ctx, const char *fmt, ...) {
    if (!ctx) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
    va_end(ap);
}

sph_status launch_copy_u64(Ctx *ctx, const unsigned long long *src, unsigned long long *dst,
                           hipStream_t s);

static hipEvent_t take_event(Ctx *ctx) {
    if (!ctx->t_pool.empty()) {
        hipEvent_t e = ctx->t_pool.back();
        ctx->t_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold recorded pairs of kernel w into the totals (oldest first); keep at
// most `keep` pending pairs.
static void fold_events(Ctx *ctx, int w, size_t keep) {
    auto &v = ctx->t_pending[w];
    size_t drop = v.size() > keep ? v.size() - keep : 0;
    for (size_t k = 0; k < drop; ++k) {
        float ms = 0.f;
        if (hipEventSynchronize(v[k].second) == hipSuccess &&
            hipEventElapsedTime(&ms, v[k].first, v[k].second) == hipSuccess) {
            ctx->t_ms[w] += ms;
            ctx->t_count[w] += 1;
        }
        ctx->t_pool.push_back(v[k].first);
        ctx->t_pool.push_back(v[k].second);
    }
    v.erase(v.begin(), v.begin() + drop);
}

TimedLaunch::TimedLaunch(Ctx *c, int w, hipStream_t st) : ctx(c), which(w), s(st) {
    if (!ctx->timing) return;
    a = take_event(ctx);
    b = take_event(ctx);
    if (a && b) (void)hipEventRecord(a, s);
}

TimedLaunch::~TimedLaunch() {
    if (!ctx->timing || !a || !b) return;
    (void)hipEventRecord(b, s);
    ctx->t_pending[which].push_back({a, b});
    if (ctx->t_pending[which].size() > 4096) fold_events(ctx, which, 2048);
}

}  // namespace sph

using namespace sph;

#define CHECK_CTX()                                     \
    do {                                                \
        if (!h) return SPH_EINVAL;                      \
    } while (0)
#define REQUIRE(cond, code, ...)                        \
    do {                                                \
        if (!(cond)) {                                  \
            set_error(&h->c, __VA_ARGS__);              \
            return code;                                \
        }                                               \
    } while (0)

static hipStream_t S(sph_stream s) { return (hipStream_t)s; }

extern "C" {

sph_status sph_create(sph_ctx **out, int64_t capacity, int32_t max_neighbors, int64_t max_cells,
                      int32_t max_runs, int32_t device) {
    if (!out) return SPH_EINVAL;
    *out = nullptr;
    if (capacity < 1 || capacity > (int64_t)kIdxMask + 1 || max_neighbors < 1 ||
        max_neighbors > 4096 || max_cells < 1 || max_cells > (int64_t)1 << 30 || max_runs < 1 ||
        max_runs > 32767)
        return SPH_EINVAL;
    sph_ctx *h = new (std::nothrow) sph_ctx();
    if (!h) return SPH_ENOMEM;
    Ctx *ctx = &h->c;
    ctx->device = device;
    ctx->capacity = capacity;
    ctx->max_nbr = max_neighbors;
    ctx->max_cells = max_cells;
    ctx->max_runs = max_runs;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return SPH_EINVAL;
    }
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
        ctx->num_cu = cu;
    size_t cap = (size_t)capacity;
    struct A {
        void **p;
        size_t bytes;
    } allocs[] = {
        {(void **)&ctx->key, cap * 4},
        {(void **)&ctx->slot, cap * 4},
        {(void **)&ctx->perm, cap * 4},
        {(void **)&ctx->ptmp, cap * 4},
        {(void **)&ctx->octant, cap},
        {(void **)&ctx->skey, cap * 4},
        {(void **)&ctx->cell_count, ((size_t)max_cells + 1) * 4},
        {(void **)&ctx->cell_start, ((size_t)max_cells + 1) * 4},
        {(void **)&ctx->posh64, cap * sizeof(double4)},
        {(void **)&ctx->posh32, cap * sizeof(float4)},
        {(void **)&ctx->cellc, cap * 4},
        {(void **)&ctx->runid, cap * 2},
        {(void **)&ctx->nbr, cap * (size_t)(max_neighbors + kRowGuard) * 4},
        {(void **)&ctx->far_box, (size_t)max_runs * sizeof(BBox)},
        {(void **)&ctx->ncount, cap * 4},
        {(void **)&ctx->grid, (size_t)max_runs * sizeof(GridDesc)},
        {(void **)&ctx->bbox_part, (size_t)max_runs * kBBoxBlocks * sizeof(BBox)},
        {(void **)&ctx->run_p, ((size_t)max_runs + 1) * 4},
        {(void **)&ctx->total_keys, 4},
        {(void **)&ctx->scan_part, (kScanBlocks + 1) * 8},
        {(void **)&ctx->flags, FLAG_COUNT * 4},
        {(void **)&ctx->pairs, 8},
        {(void **)&ctx->dtbits, (size_t)max_runs * 3 * 8},
        {(void **)&ctx->diag, 256 * 13 * 8},
        {(void **)&ctx->rec_d, cap * 32},
        {(void **)&ctx->rec_g, cap * 96},
        {(void **)&ctx->rec_f, cap * 160},
        {(void **)&ctx->gsum, cap * 15 * 8},
        {(void **)&ctx->grav_lev, gravity_levels_bytes(max_runs)},
        {(void **)&ctx->grav_totals, 24},
        {(void **)&ctx->grav_groups, ((size_t)max_cells / 8 + 8 * (size_t)max_runs + 1024) * sizeof(int4)},
        {(void **)&ctx->grav_mom0, ((size_t)max_cells + 1) * sizeof(float4)},
        {(void **)&ctx->grav_mom8, ((size_t)max_cells + 1) * 8 * sizeof(float4)},
        {(void **)&ctx->grav_momU, ((size_t)max_cells + 1) * sizeof(float4)},
        {(void **)&ctx->bm_part, bound_mass_part_bytes(max_runs)},
        {(void **)&ctx->bm_vcm, (size_t)max_runs * 3 * 8},
        {(void **)&ctx->bm_removed, 4},
    };
    ctx->grav_cap_upper = max_cells;
    ctx->grav_cap_groups = (int64_t)max_cells / 8 + 8 * (int64_t)max_runs + 1024;
    for (auto &a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            sph_destroy(h);
            return SPH_ENOMEM;
        }
    }
    ctx->mats = new Mat[kMaxMaterials];
    std::vector<unsigned long long> inf_bits((size_t)max_runs * 3, 0x7ff0000000000000ull);
    if (hipMemset(ctx->flags, 0, FLAG_COUNT * 4) != hipSuccess ||
        hipMemset(ctx->pairs, 0, 8) != hipSuccess ||
        hipMemset(ctx->ncount, 0, cap * 4) != hipSuccess ||
        hipMemset(ctx->total_keys, 0, 4) != hipSuccess ||
        hipMemset(ctx->cell_count, 0, ((size_t)max_cells + 1) * 4) != hipSuccess ||
        hipMemcpy(ctx->dtbits, inf_bits.data(), (size_t)max_runs * 3 * 8, hipMemcpyHostToDevice) !=
            hipSuccess) {
        sph_destroy(h);
        return SPH_EHIP;
    }
    *out = h;
    return SPH_OK;
}

sph_status sph_destroy(sph_ctx *h) {
    if (!h) return SPH_EINVAL;
    Ctx *ctx = &h->c;
    void *ptrs[] = {ctx->ptmp, ctx->key,  ctx->slot,      ctx->perm,   ctx->skey,    ctx->cell_count,
                    ctx->cell_start, ctx->posh64, ctx->posh32, ctx->cellc, ctx->runid,
                    ctx->nbr,  ctx->ncount,    ctx->grid,   ctx->bbox_part, ctx->run_p,
                    ctx->total_keys, ctx->scan_part, ctx->flags, ctx->pairs, ctx->dtbits,
                    ctx->diag, ctx->rec_d, ctx->rec_g, ctx->rec_f, ctx->gsum,
                    ctx->grav_lev, ctx->grav_totals, ctx->grav_mom0, ctx->grav_momU,
                    ctx->bm_part, ctx->bm_vcm, ctx->bm_removed, ctx->octant, ctx->grav_mom8,
                    ctx->far_box, ctx->grav_groups};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int w = 0; w < SPH_T_COUNT; ++w) {
        for (auto &pr : ctx->t_pending[w]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    }
    for (hipEvent_t e : ctx->t_pool) (void)hipEventDestroy(e);
    delete[] ctx->mats;
    delete h;
    return SPH_OK;
}

const char *sph_last_error(const sph_ctx *h) {
    if (h) return h->c.err;
    const char *e = noalloc_last_error();
    return e ? e : "null context";
}

sph_status sph_sync_status(sph_ctx *h, sph_stream stream) {
    CHECK_CTX();
    Ctx *ctx = &h->c;
    SPH_HIP(hipStreamSynchronize(S(stream)));
    int32_t fl[FLAG_COUNT];
    SPH_HIP(hipMemcpy(fl, ctx->flags, sizeof(fl), hipMemcpyDeviceToHost));
    SPH_HIP(hipMemset(ctx->flags, 0, sizeof(fl)));
    if (fl[FLAG_NBR_OVERFLOW]) {
        set_error(ctx, "pair list overflow: a particle has more than %d neighbours", ctx->max_nbr);
        return SPH_ECAPACITY;
    }
    if (fl[FLAG_CELL_OVERFLOW]) {
        set_error(ctx, "cell table overflow: more than %lld cells", (long long)ctx->max_cells);
        return SPH_ECAPACITY;
    }
    if (fl[FLAG_GRAV_OVERFLOW]) {
        set_error(ctx, "self-gravity walk outgrew its lists (theta too small for the grid, or "
                       "too many pyramid nodes)");
        return SPH_ECAPACITY;
    }
    if (fl[FLAG_RUNG_CLAMP]) {
        set_error(ctx, "a particle's step is below the shortest rung (raise rungs or lower "
                       "the base step)");
        return SPH_ECAPACITY;
    }
    if (fl[FLAG_NONFINITE]) {
        set_error(ctx, "non-finite value");
        return SPH_ENONFINITE;
    }
    return SPH_OK;
}

static sph_status upload_runs(sph_ctx *h, int64_t n, int32_t nr, const int64_t *run_start,
                              hipStream_t s) {
    Ctx *ctx = &h->c;
    std::vector<int64_t> rs(nr + 1);
    if (run_start) {
        for (int r = 0; r <= nr; ++r) rs[r] = run_start[r];
    } else {
        rs[0] = 0;
        rs[1] = n;
    }
    if (rs[0] != 0 || rs[nr] != n) {
        set_error(ctx, "run_start must start at 0 and end at n");
        return SPH_EINVAL;
    }
    for (int r = 0; r < nr; ++r)
        if (rs[r + 1] < rs[r]) {
            set_error(ctx, "run_start must be non-decreasing");
            return SPH_EINVAL;
        }
    if (rs != h->run_cache) {
        std::vector<int32_t> rp(nr + 1);
        for (int r = 0; r <= nr; ++r) rp[r] = (int32_t)rs[r];
        SPH_HIP(hipMemcpyAsync(ctx->run_p, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s));
        SPH_HIP(hipStreamSynchronize(s));
        h->run_cache = rs;
    }
    return SPH_OK;
}

sph_status sph_build_cells(sph_ctx *h, int64_t n, const double *x, const double *y,
                           const double *z, const double *hh, int32_t n_runs,
                           const int64_t *run_start, double cell_min, int32_t *perm_out,
                           sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0, SPH_EINVAL, "n < 0");
    REQUIRE(n <= h->c.capacity, SPH_ECAPACITY, "n = %lld exceeds capacity %lld", (long long)n,
            (long long)h->c.capacity);
    REQUIRE(n == 0 || (x && y && z && hh && perm_out), SPH_EINVAL, "null array");
    if (!run_start) n_runs = 1;
    REQUIRE(n_runs >= 1 && n_runs <= h->c.max_runs, SPH_ECAPACITY, "n_runs out of range");
    REQUIRE(cell_min >= 0.0, SPH_EINVAL, "cell_min < 0");
    sph_status st = upload_runs(h, n, n_runs, run_start, S(stream));
    if (st != SPH_OK) return st;
    return launch_build_cells(&h->c, n, const_cast<double *>(x), const_cast<double *>(y),
                              const_cast<double *>(z), hh, n_runs, cell_min, perm_out, nullptr,
                              S(stream));
}

sph_status sph_reorder(sph_ctx *h, int64_t n, const int32_t *perm, int32_t nfields,
                       const void *const *src, void *const *dst, const int32_t *elem_bytes,
                       const int32_t *rows, sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0 && n <= h->c.capacity, SPH_EINVAL, "n out of range");
    REQUIRE(nfields >= 0 && nfields <= 64, SPH_EINVAL, "nfields out of range");
    if (n == 0 || nfields == 0) return SPH_OK;
    REQUIRE(perm && src && dst && elem_bytes, SPH_EINVAL, "null argument");
    for (int f = 0; f < nfields; ++f) {
        REQUIRE(src[f] && dst[f], SPH_EINVAL, "null field %d", f);
        REQUIRE(elem_bytes[f] == 4 || elem_bytes[f] == 8, SPH_EINVAL, "elem_bytes must be 4 or 8");
        REQUIRE(!rows || (rows[f] >= 1 && rows[f] <= 16), SPH_EINVAL, "rows out of range");
        REQUIRE(src[f] != dst[f], SPH_EINVAL, "src and dst overlap");
    }
    return launch_reorder(&h->c, n, perm, nfields, src, dst, elem_bytes, rows, S(stream));
}

sph_status sph_neighbors_csr(sph_ctx *h, int64_t *offsets, int32_t *nbr, uint8_t *dflag,
                             sph_stream stream) {
    CHECK_CTX();
    REQUIRE(h->c.n_built >= 0, SPH_ESTATE, "no neighbour search yet");
    REQUIRE(offsets, SPH_EINVAL, "null offsets");
    return launch_csr(&h->c, offsets, nbr, dflag, S(stream));
}

sph_status sph_pair_count(sph_ctx *h, uint64_t *out, sph_stream stream) {
    CHECK_CTX();
    REQUIRE(out, SPH_EINVAL, "null argument");
    return launch_copy_u64(&h->c, h->c.pairs, (unsigned long long *)out, S(stream));
}

static sph_status check_built(sph_ctx *h, int64_t n) {
    REQUIRE(h->c.n_built >= 0, SPH_ESTATE, "pair pass before sph_build_cells");
    REQUIRE(n == h->c.n_built, SPH_ESTATE, "n = %lld differs from the last build (%lld)",
            (long long)n, (long long)h->c.n_built);
    return SPH_OK;
}

static sph_status set_mats(sph_ctx *h, const sph_material *mats, int32_t nmat) {
    REQUIRE(mats && nmat >= 1 && nmat <= 8, SPH_EINVAL, "need 1..8 materials");
    for (int k = 0; k < nmat; ++k) {
        const sph_material &m = mats[k];
        const bool table = m.eos_nrho >= 2 || m.eos_nu >= 2;
        if (table) {
            REQUIRE(m.eos_nrho >= 2 && m.eos_nu >= 2 && m.eos_nrho <= (1 << 20) &&
                        m.eos_nu <= (1 << 20) && (int64_t)m.eos_nrho * m.eos_nu <= (1ll << 26),
                    SPH_EINVAL, "material %d: EOS table of %d x %d nodes", k, m.eos_nrho,
                    m.eos_nu);
            REQUIRE(m.eos_rho && m.eos_u && m.eos_P && m.eos_c && m.eos_T, SPH_EINVAL,
                    "material %d: null EOS table pointer", k);
        } else {
            REQUIRE(m.rho0 > 0 && m.E0 > 0 && m.cv > 0 && m.Ecv > m.Eiv, SPH_EINVAL,
                    "material %d: invalid Tillotson or temperature constants", k);
            REQUIRE(m.rho_limit >= 0.0 && m.rho_limit <= 1.0, SPH_EINVAL,
                    "material %d: rho_limit %g outside [0, 1]", k, m.rho_limit);
        }
        REQUIRE(!m.strength_on || m.Ym > m.Y0, SPH_EINVAL, "material %d: Ym must exceed Y0", k);
        REQUIRE(m.tmelt_n >= 0 && m.tmelt_n <= 8, SPH_EINVAL,
                "material %d: melting table with %d nodes (0..8)", k, m.tmelt_n);
        for (int q = 1; q < m.tmelt_n; ++q)
            REQUIRE(m.tmelt_rho[q] > m.tmelt_rho[q - 1], SPH_EINVAL,
                    "material %d: melting table densities must ascend", k);
        h->c.mats[k].m = m;
    }
    return SPH_OK;
}

sph_status sph_density(sph_ctx *h, int64_t n, const double *m, const double *hh,
                       const double *u, const int32_t *mat, const sph_material *mats,
                       int32_t n_materials, const sph_params *prm, sph_precision prec,
                       double *rho, double *omega, double *P, double *cs, double *T, double *Y,
                       double *Gmod, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(prm && (prec == SPH_FP64 || prec == SPH_FP32_CELLREL), SPH_EINVAL, "bad params");
    REQUIRE(n == 0 || (m && hh && u && rho && omega && P && cs && T && Y && Gmod), SPH_EINVAL,
            "null array");
    st = set_mats(h, mats, n_materials);
    if (st != SPH_OK) return st;
    return launch_density(&h->c, n, m, hh, u, mat, n_materials, prm, prec, rho, omega, P, cs, T,
                          Y, Gmod, S(stream));
}

sph_status sph_gradients(sph_ctx *h, int64_t n, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *hh, const double *rho,
                         const double *omega, const sph_params *prm, sph_precision prec,
                         double *G, int64_t *n_singular, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(prm && (prec == SPH_FP64 || prec == SPH_FP32_CELLREL), SPH_EINVAL, "bad params");
    REQUIRE(n == 0 || (vx && vy && vz && m && hh && rho && omega && G), SPH_EINVAL, "null array");
    return launch_gradients(&h->c, n, vx, vy, vz, m, hh, rho, omega, prm, prec, G, n_singular,
                            S(stream));
}

sph_status sph_stress_update(sph_ctx *h, int32_t phase, int64_t n, const double *dt,
                             const double *dt_next, const double *G, const double *Y,
                             const double *Gmod, const int32_t *fixed, const sph_params *prm,
                             double *S_half, double *S_pred, double *Sdot, double *eps2,
                             sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0 && n <= h->c.capacity, SPH_EINVAL, "n out of range");
    REQUIRE(prm, SPH_EINVAL, "null params");
    if (n == 0) return SPH_OK;
    switch (phase) {
        case SPH_STRESS_PREDICT:
            REQUIRE(dt && Y && S_half && S_pred && Sdot, SPH_EINVAL, "null array");
            break;
        case SPH_STRESS_RATE:
            REQUIRE(G && Gmod && S_pred && Sdot, SPH_EINVAL, "null array");
            break;
        case SPH_STRESS_KICK:
            REQUIRE(dt && dt_next && Y && S_half && Sdot && (!eps2 || G), SPH_EINVAL, "null array");
            break;
        case SPH_STRESS_OPEN:
            REQUIRE(dt_next && S_half && S_pred && Sdot, SPH_EINVAL, "null array");
            break;
        default:
            REQUIRE(false, SPH_EINVAL, "unknown stress phase %d", phase);
    }
    return launch_stress(&h->c, phase, n, dt, dt_next, G, Y, Gmod, fixed, prm, S_half, S_pred,
                         Sdot, eps2, S(stream));
}

sph_status sph_forces_stress(sph_ctx *h, int64_t n, const double *vx, const double *vy,
                             const double *vz, const double *m, const double *hh,
                             const double *rho, const double *omega, const double *P,
                             const double *cs, const double *Sd, const sph_params *prm,
                             sph_precision prec, double *ax, double *ay, double *az,
                             double *dudt, double *dt_cfl, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(prm && (prec == SPH_FP64 || prec == SPH_FP32_CELLREL), SPH_EINVAL, "bad params");
    REQUIRE(n == 0 || (vx && vy && vz && m && hh && rho && omega && P && cs && Sd && ax && ay &&
                       az && dudt && dt_cfl),
            SPH_EINVAL, "null array");
    return launch_forces(&h->c, n, vx, vy, vz, m, hh, rho, omega, P, cs, Sd, prm, prec, ax, ay, az,
                         dudt, dt_cfl, S(stream));
}

sph_status sph_kick_drift(sph_ctx *h, int32_t phase, int64_t n, const double *dt,
                          const double *dt_next, const int32_t *fixed, double *x, double *y,
                          double *z, double *vx, double *vy, double *vz, double *u,
                          const double *ax, const double *ay, const double *az,
                          const double *dudt, double *vpx, double *vpy, double *vpz,
                          double *up, sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0 && n <= h->c.capacity, SPH_EINVAL, "n out of range");
    if (n == 0) return SPH_OK;
    switch (phase) {
        case SPH_KD_DRIFT:
            REQUIRE(dt && x && y && z && vx && vy && vz, SPH_EINVAL, "null array");
            break;
        case SPH_KD_PREDICT:
            REQUIRE(dt && vx && vy && vz && u && ax && ay && az && dudt && vpx && vpy && vpz && up,
                    SPH_EINVAL, "null array");
            break;
        case SPH_KD_KICK:
            REQUIRE(dt && dt_next && vx && vy && vz && u && ax && ay && az && dudt, SPH_EINVAL,
                    "null array");
            break;
        case SPH_KD_OPEN:
            REQUIRE(dt_next && vx && vy && vz && u && ax && ay && az && dudt, SPH_EINVAL,
                    "null array");
            break;
        default:
            REQUIRE(false, SPH_EINVAL, "unknown kick/drift phase %d", phase);
    }
    return launch_kick_drift(&h->c, phase, n, dt, dt_next, fixed, x, y, z, vx, vy, vz, u, ax, ay,
                             az, dudt, vpx, vpy, vpz, up, S(stream));
}

sph_status sph_dt_min(sph_ctx *h, int64_t n, const double *dt_cfl, const int32_t *fixed,
                      double *dt_out, sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0 && n <= h->c.capacity, SPH_EINVAL, "n out of range");
    REQUIRE(dt_out && (n == 0 || dt_cfl), SPH_EINVAL, "null array");
    return launch_dt_min(&h->c, n, dt_cfl, fixed, 0.0, dt_out, S(stream));
}

sph_status sph_diagnostics(sph_ctx *h, int64_t n, const double *x, const double *y,
                           const double *z, const double *vx, const double *vy, const double *vz,
                           const double *m, const double *ax, const double *ay, const double *az,
                           const double *dudt, double *out13, sph_stream stream) {
    CHECK_CTX();
    REQUIRE(n >= 0 && n <= h->c.capacity, SPH_EINVAL, "n out of range");
    REQUIRE(out13 && (n == 0 || (x && y && z && vx && vy && vz && m && ax && ay && az && dudt)),
            SPH_EINVAL, "null array");
    return launch_diag(&h->c, n, x, y, z, vx, vy, vz, m, ax, ay, az, dudt, out13, S(stream));
}

sph_status sph_gravity(sph_ctx *h, int64_t n, const double *m, const int32_t *active, double G,
                       double eps_over_h, double theta, int32_t accumulate, double *ax,
                       double *ay, double *az, double *phi, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(G >= 0.0 && eps_over_h > 0.0, SPH_EINVAL, "G must be >= 0 and eps_over_h > 0");
    REQUIRE(theta >= 0.3 && theta <= 1.0, SPH_EINVAL, "theta %g outside [0.3, 1]", theta);
    REQUIRE(n == 0 || (m && ax && ay && az), SPH_EINVAL, "null array");
    return launch_gravity(&h->c, n, m, active, G, eps_over_h, theta, accumulate, ax, ay, az, phi,
                          S(stream));
}

sph_status sph_bound_mass(sph_ctx *h, int64_t n, const double *vx, const double *vy,
                          const double *vz, const double *m, double G, double eps_over_h,
                          double theta, int32_t max_iter, int32_t *bound, double *m_bound,
                          double *work, int32_t *iterations, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(G >= 0.0 && eps_over_h > 0.0, SPH_EINVAL, "G must be >= 0 and eps_over_h > 0");
    REQUIRE(theta >= 0.3 && theta <= 1.0, SPH_EINVAL, "theta %g outside [0.3, 1]", theta);
    REQUIRE(max_iter >= 1, SPH_EINVAL, "max_iter must be >= 1");
    REQUIRE(m_bound && (n == 0 || (vx && vy && vz && m && bound && work)), SPH_EINVAL,
            "null array");
    return launch_bound_mass(&h->c, n, vx, vy, vz, m, G, eps_over_h, theta, max_iter, bound,
                             m_bound, work, work + n, iterations, S(stream));
}

sph_status sph_adapt_h(sph_ctx *h, int64_t n, const double *m, const double *h_start,
                       double n_ngb, double tol, int32_t max_iter, double *h_out,
                       int64_t *n_clamped, int32_t *iterations, sph_stream stream) {
    CHECK_CTX();
    sph_status st = check_built(h, n);
    if (st != SPH_OK) return st;
    REQUIRE(n_ngb > 0.0 && tol > 0.0 && max_iter >= 1, SPH_EINVAL,
            "n_ngb and tol must be > 0 and max_iter >= 1");
    REQUIRE(n == 0 || (m && h_start && h_out), SPH_EINVAL, "null array");
    return launch_adapt_h(&h->c, n, m, h_start, nullptr, n_ngb, tol, max_iter, h_out, n_clamped,
                          iterations, S(stream));
}

// ------------------------------------------------------------ whole step
struct Rows {
    double *f[SPH_NF64];
    int32_t *i[SPH_NI32];
    double *w[SPH_NW];
};

static Rows rows_of(const sph_state *st, int buf) {
    Rows r;
    for (int k = 0; k < SPH_NF64; ++k) r.f[k] = st->f64[buf] + (size_t)k * st->n_cap;
    for (int k = 0; k < SPH_NI32; ++k) r.i[k] = st->i32[buf] + (size_t)k * st->n_cap;
    for (int k = 0; k < SPH_NW; ++k) r.w[k] = st->work + (size_t)k * st->n_cap;
    return r;
}

static int32_t n_runs_of(const sph_state *st) { return st->run_start ? st->n_runs : 1; }
static unsigned long long *step_bits(Ctx *ctx, int other);

static sph_status check_state(sph_ctx *h, const sph_state *st) {
    REQUIRE(st, SPH_EINVAL, "null state");
    REQUIRE(st->n >= 0 && st->n <= st->n_cap && st->n <= h->c.capacity, SPH_ECAPACITY,
            "state size out of range");
    REQUIRE(st->f64[0] && st->f64[1] && st->i32[0] && st->i32[1] && st->work && st->dt &&
                st->dt_next,
            SPH_EINVAL, "null state buffer");
    REQUIRE(st->cur == 0 || st->cur == 1, SPH_EINVAL, "cur must be 0 or 1");
    return SPH_OK;
}

// Neighbour search (with the drift fused in when `drift`), then the
// reorder of every state row into the other buffer with the predictor of v
// and u fused in (predict = 0 at the start of a run: predicted = current).
static double tick_of(const sph_state *st, const sph_params *prm) {
    return prm->rungs > 0 ? ldexp(st->dt_max, -(prm->rungs - 1)) : 0.0;
}

static sph_status search_and_sort(sph_ctx *h, sph_state *st, const sph_params *prm,
                                  sph_precision prec, bool drift, int32_t predict, hipStream_t s,
                                  const double *h_build = nullptr, bool far_init = false) {
    Ctx *ctx = &h->c;
    const int64_t n = st->n;
    const int cur = st->cur, alt = 1 - cur;
    Rows A = rows_of(st, cur), B = rows_of(st, alt);
    int32_t *perm = (int32_t *)B.w[SPH_W_PERM];
    const int32_t nr = n_runs_of(st);
    REQUIRE(nr >= 1 && nr <= ctx->max_runs, SPH_ECAPACITY, "n_runs out of range");
    sph_status e = upload_runs(h, n, nr, st->run_start, s);
    if (e) return e;
    BuildExtras ex;
    if (drift) {
        ex.dt = st->dt;
        ex.vx = A.f[SPH_VX];
        ex.vy = A.f[SPH_VY];
        ex.vz = A.f[SPH_VZ];
        ex.fixed = A.i[SPH_FIXED];
    }
    ex.m = A.f[SPH_M];  // the gather reads the unsorted state: records in sorted order
    ex.f32 = prec == SPH_FP32_CELLREL;
    ex.far_factor = prm->far_factor > 0.0 ? prm->far_factor : 0.0;
    ex.far_init = far_init ? 1 : 0;
    if ((e = launch_build_cells(ctx, n, A.f[SPH_X], A.f[SPH_Y], A.f[SPH_Z],
                                h_build ? h_build : A.f[SPH_H], nr, st->cell_min, perm, &ex, s)))
        return e;
    StepRows r;
    for (int k = 0; k < SPH_NF64; ++k) {
        r.f_src[k] = A.f[k];
        r.f_dst[k] = B.f[k];
    }
    for (int k = 0; k < SPH_NI32; ++k) {
        r.i_src[k] = A.i[k];
        r.i_dst[k] = B.i[k];
    }
    if ((e = launch_step_reorder(ctx, n, perm, r, st->dt, nr > 1 ? ctx->runid : nullptr, predict,
                                 prm->rungs > 0 ? 1 : 0, tick_of(st, prm), B.w[SPH_W_VP],
                                 B.w[SPH_W_VP + 1], B.w[SPH_W_VP + 2], B.w[SPH_W_UP],
                                 B.w[SPH_W_TAU], (int32_t *)B.w[SPH_W_ACT], s)))
        return e;
    st->cur = alt;
    return SPH_OK;
}

// Neighbour search of a step.  With adaptive smoothing lengths
// (prm->adapt_ngb > 0): search with the lengths enlarged by adapt_skin,
// Newton-Raphson to constant kernel mass over those lists (capped at the
// enlarged lengths, fixed particles unchanged), then the exact search with
// the new lengths.  The second search neither drifts nor changes the
// predictor inputs, so the state is the same as after one plain search.
constexpr double kAdaptTol = 1e-10;
constexpr int32_t kAdaptIter = 30;

static sph_status step_search(sph_ctx *h, sph_state *st, const sph_params *prm,
                              sph_precision prec, bool drift, int32_t predict, hipStream_t s,
                              bool far_init = false) {
    if (!(prm->adapt_ngb > 0.0))
        return search_and_sort(h, st, prm, prec, drift, predict, s, nullptr, far_init);
    Ctx *ctx = &h->c;
    const int64_t n = st->n;
    Rows A = rows_of(st, st->cur);
    double *hs = A.w[SPH_W_T];  // free until the state kernel of this step
    sph_status e;
    if ((e = launch_scale(ctx, n, A.f[SPH_H], prm->adapt_skin, hs, s))) return e;
    if ((e = search_and_sort(h, st, prm, prec, drift, predict, s, hs, far_init))) return e;
    Rows R = rows_of(st, st->cur);
    if ((e = launch_adapt_h(ctx, n, R.f[SPH_M], R.f[SPH_H], R.i[SPH_FIXED], prm->adapt_ngb,
                            kAdaptTol, kAdaptIter, R.f[SPH_H], nullptr, nullptr, s)))
        return e;
    // the second search repeats the first one's predictor; with individual
    // steps (predict = 2) without advancing the elapsed times again
    return search_and_sort(h, st, prm, prec, false, (predict && prm->rungs > 0) ? 2 : predict,
                           s);
}

// Derivatives at the sorted state: density pass, per-particle state (EOS,
// yield, stress predictor + rescaling, pass record), one sweep for the
// gradient sums and the forces, gradient epilogue + stress rate, CFL minimum
// into *dt_next.
static sph_status eval(sph_ctx *h, const sph_state *st, const Rows &R, int32_t nmat,
                       const sph_params *prm, sph_precision prec, int32_t predict,
                       bool accumulate_eps2, hipStream_t s) {
    const int64_t n = st->n;
    Ctx *ctx = &h->c;
    sph_status e;
    const int32_t *fixed = R.i[SPH_FIXED];
    const int32_t nr = n_runs_of(st);
    const bool hier = prm->rungs > 0;
    // with individual steps only the particles whose step ends are evaluated
    // past the per-particle state (every particle at the start of a run)
    const int32_t *act = (hier && predict) ? (const int32_t *)R.w[SPH_W_ACT] : nullptr;
    if ((e = launch_density_pairs(ctx, n, prm, prec, R.w[SPH_W_RHO], R.w[SPH_W_OMEGA], s)))
        return e;
    if ((e = launch_step_state(ctx, n, prec, R.w[SPH_W_RHO], R.w[SPH_W_OMEGA], R.w[SPH_W_UP],
                               R.w[SPH_W_VP], R.w[SPH_W_VP + 1], R.w[SPH_W_VP + 2], R.f[SPH_M],
                               R.i[SPH_MAT], nmat, fixed, R.w[SPH_W_TAU], R.f[SPH_S],
                               R.f[SPH_SDOT], R.w[SPH_W_P], R.w[SPH_W_CS], R.w[SPH_W_T],
                               R.w[SPH_W_Y], R.w[SPH_W_GMOD], R.w[SPH_W_SP], s)))
        return e;
    if ((e = launch_grad_force_pairs(ctx, n, prm, prec, R.f[SPH_AX], R.f[SPH_AY], R.f[SPH_AZ],
                                     R.f[SPH_DUDT], R.w[SPH_W_DT], s, act)))
        return e;
    if (prm->grav_G > 0.0 &&
        (e = launch_gravity(ctx, n, R.f[SPH_M], nullptr, prm->grav_G, prm->grav_eps_over_h,
                            prm->grav_theta, 1, R.f[SPH_AX], R.f[SPH_AY], R.f[SPH_AZ], nullptr,
                            s, act)))
        return e;
    if ((e = launch_step_grad_rate(ctx, n, prm, prec == SPH_FP32_CELLREL ? 1 : 0, R.w[SPH_W_SP],
                                   R.w[SPH_W_GMOD], fixed,
                                   R.w[SPH_W_TAU], act, R.w[SPH_W_G], R.f[SPH_SDOT],
                                   accumulate_eps2 ? R.f[SPH_EPS2] : nullptr, st->n_singular, s)))
        return e;
    if (prm->eta_a > 0.0 &&
        (e = launch_accel_limit(ctx, n, prm->eta_a, R.f[SPH_AX], R.f[SPH_AY], R.f[SPH_AZ],
                                R.f[SPH_H], act, R.w[SPH_W_DT], s)))
        return e;
    if (hier) return SPH_OK;  // the kick takes the new steps
    return launch_dt_reduce(ctx, n, R.w[SPH_W_DT], fixed, step_bits(ctx, 0), s, nr, ctx->run_p,
                            true);
}

// Individual steps: kicks and new steps of the particles whose step ended,
// then each run's next substep (the nearest end of a step) and its clock.
static sph_status kick_hier(sph_ctx *h, sph_state *st, const Rows &R, const sph_params *prm,
                            int32_t init, hipStream_t s) {
    Ctx *ctx = &h->c;
    const int32_t nr = n_runs_of(st);
    const int16_t *runid = nr > 1 ? ctx->runid : nullptr;
    const double tick = tick_of(st, prm);
    sph_status e = launch_kick_hier(
        ctx, st->n, init, prm->rungs, tick, st->dt, st->clock, runid, R.i[SPH_FIXED],
        (const int32_t *)R.w[SPH_W_ACT], R.f[SPH_VX], R.f[SPH_VY], R.f[SPH_VZ], R.f[SPH_U],
        R.f[SPH_AX], R.f[SPH_AY], R.f[SPH_AZ], R.f[SPH_DUDT], R.f[SPH_S], R.w[SPH_W_SP],
        R.f[SPH_SDOT], R.w[SPH_W_Y], R.w[SPH_W_DT], R.f[SPH_DTP], R.f[SPH_EL], R.w[SPH_W_TAU], s);
    if (e) return e;
    if ((e = launch_dt_reduce(ctx, st->n, R.w[SPH_W_TAU], R.i[SPH_FIXED], step_bits(ctx, 0), s,
                              nr, ctx->run_p)))
        return e;
    e = launch_hier_next(ctx, nr, init, tick, step_bits(ctx, 0), step_bits(ctx, 1), st->dt,
                         st->dt_next, st->clock, st->time, s);
    ctx->dt_parity ^= 1;
    return e;
}

static sph_status check_rungs(sph_ctx *h, const sph_state *st, const sph_params *prm) {
    if (prm->rungs == 0) return SPH_OK;
    REQUIRE(prm->rungs > 0 && prm->rungs <= 40, SPH_EINVAL, "rungs must be in 0..40");
    REQUIRE(st->dt_max > 0.0, SPH_EINVAL, "individual steps need the base step in dt_max");
    REQUIRE(st->clock, SPH_EINVAL, "individual steps need the per-run clock");
    return SPH_OK;
}

// The kick that follows an evaluation turns the minima into the next step
// and clears the other buffer; then the parity flips.
static sph_status kick(sph_ctx *h, sph_state *st, const Rows &R, int32_t mode, hipStream_t s) {
    Ctx *ctx = &h->c;
    const int32_t nr = n_runs_of(st);
    const int16_t *runid = nr > 1 ? ctx->runid : nullptr;
    sph_status e = launch_step_kick(
        ctx, st->n, mode, st->dt, step_bits(ctx, 0), st->dt_max, st->dt_next, step_bits(ctx, 1),
        nr, runid, R.i[SPH_FIXED], R.f[SPH_VX], R.f[SPH_VY], R.f[SPH_VZ], R.f[SPH_U],
        R.f[SPH_AX], R.f[SPH_AY], R.f[SPH_AZ], R.f[SPH_DUDT], R.f[SPH_S], R.w[SPH_W_SP],
        R.f[SPH_SDOT], R.w[SPH_W_Y], st->time, s);
    ctx->dt_parity ^= 1;
    return e;
}

// Minima buffers of the whole step: the current one (other = 0) and the one
// to clear (other = 1); see Ctx::dtbits.
static unsigned long long *step_bits(Ctx *ctx, int other) {
    return ctx->dtbits + (size_t)ctx->max_runs * (1 + (ctx->dt_parity ^ other));
}

static void swap_dt(sph_state *st) {
    double *t = st->dt;
    st->dt = st->dt_next;
    st->dt_next = t;
}

sph_status sph_init(sph_ctx *h, sph_state *st, const sph_material *mats, int32_t n_materials,
                    const sph_params *prm, sph_precision prec, sph_stream stream) {
    CHECK_CTX();
    sph_status e = check_state(h, st);
    if (e) return e;
    REQUIRE(prm, SPH_EINVAL, "null params");
    REQUIRE(prec == SPH_FP64 || prec == SPH_FP32_CELLREL, SPH_EINVAL, "bad precision");
    if ((e = set_mats(h, mats, n_materials))) return e;
    hipStream_t s = S(stream);
    REQUIRE(!(prm->adapt_ngb > 0.0) || prm->adapt_skin >= 1.0, SPH_EINVAL,
            "adapt_skin must be >= 1");
    REQUIRE(!(prm->far_factor > 0.0) || prm->far_factor >= 1.0, SPH_EINVAL,
            "far_factor must be 0 or >= 1");
    if ((e = check_rungs(h, st, prm))) return e;
    if ((e = step_search(h, st, prm, prec, false, 0, s, true))) return e;
    Rows R = rows_of(st, st->cur);
    // predicted values are the current ones: v, u as they are, S rescaled
    if ((e = eval(h, st, R, n_materials, prm, prec, 0, false, s))) return e;
    // the opening kick uses the new step only: it writes it to dt_next, and
    // the swap makes it the step of the first drift
    if ((e = prm->rungs > 0 ? kick_hier(h, st, R, prm, 1, s) : kick(h, st, R, 1, s))) return e;
    swap_dt(st);
    return SPH_OK;
}

sph_status sph_step(sph_ctx *h, sph_state *st, const sph_material *mats, int32_t n_materials,
                    const sph_params *prm, sph_precision prec, sph_stream stream) {
    CHECK_CTX();
    sph_status e = check_state(h, st);
    if (e) return e;
    REQUIRE(prm, SPH_EINVAL, "null params");
    REQUIRE(prec == SPH_FP64 || prec == SPH_FP32_CELLREL, SPH_EINVAL, "bad precision");
    if ((e = set_mats(h, mats, n_materials))) return e;
    hipStream_t s = S(stream);
    REQUIRE(!(prm->adapt_ngb > 0.0) || prm->adapt_skin >= 1.0, SPH_EINVAL,
            "adapt_skin must be >= 1");
    REQUIRE(!(prm->far_factor > 0.0) || prm->far_factor >= 1.0, SPH_EINVAL,
            "far_factor must be 0 or >= 1");
    if ((e = check_rungs(h, st, prm))) return e;
    if ((e = step_search(h, st, prm, prec, true, 1, s))) return e;
    Rows R = rows_of(st, st->cur);
    if ((e = eval(h, st, R, n_materials, prm, prec, 1, true, s))) return e;
    if ((e = prm->rungs > 0 ? kick_hier(h, st, R, prm, 0, s) : kick(h, st, R, 0, s))) return e;
    swap_dt(st);
    return SPH_OK;
}

sph_status sph_timing(sph_ctx *h, int32_t enable) {
    CHECK_CTX();
    Ctx *ctx = &h->c;
    for (int w = 0; w < SPH_T_COUNT; ++w) {
        fold_events(ctx, w, 0);
        ctx->t_ms[w] = 0.0;
        ctx->t_count[w] = 0;
    }
    ctx->timing = enable != 0;
    return SPH_OK;
}

sph_status sph_set_tuning(sph_ctx *h, int32_t knob, sph_precision prec, int32_t value) {
    CHECK_CTX();
    REQUIRE(knob >= 0 && knob < SPH_TUNE_COUNT, SPH_EINVAL, "unknown tuning knob %d", knob);
    REQUIRE(prec == SPH_FP64 || prec == SPH_FP32_CELLREL, SPH_EINVAL, "bad precision");
    Ctx *ctx = &h->c;
    if (knob == SPH_TUNE_CELL_SCALE) {
        REQUIRE(value >= 1000 && value <= 2000, SPH_EINVAL, "cell scale %d outside 1000..2000",
                value);
        ctx->cell_scale = value / 1000.0;
        return SPH_OK;
    }
    if (knob == SPH_TUNE_BUILD_RANGE) {
        REQUIRE(value == 32 || value == 64 || value == 96 || value == 128, SPH_EINVAL,
                "build range must be 32, 64, 96 or 128 (got %d)", value);
        ctx->build_range = value;
        return SPH_OK;
    }
    if (knob == SPH_TUNE_BUILD_TILE) {
        REQUIRE(value == 128 || value == 192 || value == 256, SPH_EINVAL,
                "build tile must be 128, 192 or 256 (got %d)", value);
        ctx->build_tile = value;
        return SPH_OK;
    }
    if (knob == SPH_TUNE_SWEEP_DEPTH) {
        REQUIRE(value == 1 || value == 2, SPH_EINVAL, "sweep depth must be 1 or 2 (got %d)",
                value);
        ctx->sweep_depth[prec == SPH_FP32_CELLREL ? 1 : 0] = value;
        return SPH_OK;
    }
    REQUIRE(value == 4 || value == 8 || value == 16, SPH_EINVAL,
            "lanes per particle must be 4, 8 or 16 (got %d)", value);
    ctx->lanes[knob][prec == SPH_FP32_CELLREL ? 1 : 0] = value;
    return SPH_OK;
}

sph_status sph_get_tuning(sph_ctx *h, int32_t knob, sph_precision prec, int32_t *value) {
    CHECK_CTX();
    REQUIRE(knob >= 0 && knob < SPH_TUNE_COUNT && value, SPH_EINVAL, "bad argument");
    REQUIRE(prec == SPH_FP64 || prec == SPH_FP32_CELLREL, SPH_EINVAL, "bad precision");
    const Ctx *ctx = &h->c;
    const int pi = prec == SPH_FP32_CELLREL ? 1 : 0;
    *value = knob == SPH_TUNE_CELL_SCALE    ? (int32_t)(ctx->cell_scale * 1000.0 + 0.5)
             : knob == SPH_TUNE_BUILD_RANGE ? ctx->build_range
             : knob == SPH_TUNE_SWEEP_DEPTH ? ctx->sweep_depth[pi]
             : knob == SPH_TUNE_BUILD_TILE  ? ctx->build_tile
                                            : ctx->lanes[knob][pi];
    return SPH_OK;
}

sph_status sph_timing_read(sph_ctx *h, int32_t which, double *total_ms, int64_t *launches) {
    CHECK_CTX();
    REQUIRE(which >= 0 && which < SPH_T_COUNT, SPH_EINVAL, "unknown kernel id");
    REQUIRE(total_ms && launches, SPH_EINVAL, "null argument");
    Ctx *ctx = &h->c;
    fold_events(ctx, which, 0);
    *total_ms = ctx->t_ms[which];
    *launches = ctx->t_count[which];
    return SPH_OK;
}

}  // extern "C"
