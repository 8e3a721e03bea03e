// Internal declarations of the gfx950 strength-SPH library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/sph.h"
#include "device_util.h"

namespace sph {

// Flags raised on the device (ctx->flags[...]).
enum {
    FLAG_NBR_OVERFLOW = 0,
    FLAG_CELL_OVERFLOW = 1,
    FLAG_NONFINITE = 2,
    FLAG_GRAV_OVERFLOW = 3,
    FLAG_RUNG_CLAMP = 4,
    FLAG_COUNT = 5
};

// Raise flags[which] when `bad` holds on any lane of the wave: one atomic
// per wave, issued by the first lane that saw it.  Lanes that already left
// the kernel take no part, so it may follow an early return.
__device__ __forceinline__ void flag_if(bool bad, int32_t *flags, int which) {
    const uint64_t m = __ballot(bad);
    if (m && (int)__lane_id() == __ffsll((long long)m) - 1) atomicOr(&flags[which], 1);
}

// True when any of the values is NaN or infinite.
__device__ __forceinline__ bool nonfinite(double a) { return !__builtin_isfinite(a); }
template <typename... T>
__device__ __forceinline__ bool nonfinite(double a, T... rest) {
    return nonfinite(a) | nonfinite(rest...);
}

// Uniform cell grid of one run.
struct GridDesc {
    double ox, oy, oz;      // origin
    double L, invL;         // cell edge
    float L32;              // cell edge in float (cell-relative pair arithmetic)
    int32_t nx, ny, nz;     // cells per axis
    int32_t bx, by, bz;     // Morton bits per axis
    int32_t key_off;        // first key of this run in the global cell table
    int32_t key_count;      // 2^(bx+by+bz)
    int32_t p0, p1;         // particle range of the run (input order == sorted order by run)
    int32_t sink;           // 1: key key_off + key_count holds the run's particles outside
                            // its far cube (sph_params.far_factor), sorted after its cells
    int32_t pad;
};

// Key of the far slot of run g (valid when g.sink).
__host__ __device__ inline uint32_t far_key(const GridDesc &g) {
    return (uint32_t)(g.key_off + g.key_count);
}

struct BBox {
    double lo[3], hi[3], hmax;
};

// Material block as the kernels read it (copy of the ABI struct).
struct Mat {
    sph_material m;
};

struct Ctx {
    int device = 0;
    int64_t capacity = 0;
    int32_t max_nbr = 0;
    int64_t max_cells = 0;
    int32_t max_runs = 0;
    int32_t num_cu = 256;
    // launch shapes chosen by the autotuner: lanes per particle of the pair
    // passes [knob][precision], and the cell edge as a multiple of 2 h_max
    int32_t lanes[4][2] = {{8, 8}, {8, 8}, {8, 8}, {8, 8}};
    double cell_scale = 1.0;
    int32_t build_range = 64;  // sorted particles per work-group of the pair-list build
    int32_t sweep_depth[2] = {1, 2};  // records in flight per lane of the fused sweep [FP64, FP32]
    int32_t build_tile = 256;         // candidates in the LDS tile of the pair-list build
    // self-gravity pyramid (allocated with the context)
    void *grav_lev = nullptr;        // per-run level layout (max_runs entries)
    int64_t *grav_totals = nullptr;  // [upper nodes, groups written, top-level group nodes]
    int4 *grav_groups = nullptr;     // target groups of the walk (run, level, node)
    int64_t grav_cap_groups = 0;
    float4 *grav_mom0 = nullptr;     // max_cells cell monopoles (by cell key)
    float4 *grav_mom8 = nullptr;     // 8 max_cells octant monopoles (by cell key, octant)
    float4 *grav_momU = nullptr;     // grav_cap_upper monopoles of levels >= 1
    int64_t grav_cap_upper = 0;
    double *bm_part = nullptr;       // bound mass: per-(run, block) partial sums
    double *bm_vcm = nullptr;        // centre-of-mass velocity per run
    int32_t *bm_removed = nullptr;   // particles removed in the last pass
    // scratch (device)
    uint32_t *key = nullptr;        // capacity: cell key, input order
    int32_t *slot = nullptr;        // capacity: arrival rank within the cell
    int32_t *perm = nullptr;        // capacity: sorted -> input
    int32_t *ptmp = nullptr;        // capacity: arrival order within cells
    uint8_t *octant = nullptr;      // capacity: octant of each sorted particle in its cell
    uint32_t *skey = nullptr;       // capacity: cell key, sorted order
    int32_t *cell_count = nullptr;  // max_cells + 1
    int32_t *cell_start = nullptr;  // max_cells + 1
    double4 *posh64 = nullptr;      // capacity: (x, y, z, h) sorted
    float4 *posh32 = nullptr;       // capacity: (dx, dy, dz, h) relative to the cell origin
    uint32_t *cellc = nullptr;      // capacity: packed cell coordinates (10 bits each) + run in bits 30..
    int16_t *runid = nullptr;       // capacity: run of the sorted particle
    uint32_t *nbr = nullptr;        // capacity rows of max_nbr + kRowGuard entries
    int32_t *ncount = nullptr;      // capacity
    GridDesc *grid = nullptr;       // max_runs
    BBox *bbox_part = nullptr;      // max_runs * kBBoxBlocks
    int32_t *run_p = nullptr;       // max_runs + 1 particle offsets (device copy)
    int32_t *total_keys = nullptr;  // 1
    int64_t *scan_part = nullptr;   // scan partials (kScanBlocks + 1)
    int32_t *flags = nullptr;       // FLAG_COUNT
    unsigned long long *pairs = nullptr;  // accumulated ordered pairs
    // per-run step minima as ordered bit patterns: [0] for sph_dt_min,
    // [1 + parity] for the whole step, which alternates between the two so
    // that a step's kick can read one while clearing the other
    unsigned long long *dtbits = nullptr;  // 3 * max_runs
    int32_t dt_parity = 0;
    double *diag = nullptr;         // diagnostics partial sums: 256 x 13 doubles
    BBox *far_box = nullptr;        // max_runs: far cube of each run (sph_params.far_factor)
    // pair-pass records (array of structures, see the pair kernels)
    void *rec_d = nullptr;          // density: capacity * 32 bytes
    void *rec_g = nullptr;          // gradients: capacity * 96 bytes
    void *rec_f = nullptr;          // forces: capacity * 160 bytes
    double *gsum = nullptr;         // capacity * 15 (gradient raw sums)
    Mat *mats = nullptr;            // up to kMaxMaterials
    // kernel timing (host side): event pairs recorded around pass kernels
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> t_pending[SPH_T_COUNT];
    std::vector<hipEvent_t> t_pool;
    double t_ms[SPH_T_COUNT] = {0};
    int64_t t_count[SPH_T_COUNT] = {0};
    // host state
    int64_t n_built = -1;           // particles of the last build
    bool far_built = false;         // the last build kept far slots (sph_params.far_factor)
    int32_t n_runs_built = 0;
    char err[512] = {0};
};

// Bounding-box partials: at most kBBoxBlocks blocks per run (enough waves to
// cover the loads' latency on every SIMD), threads per block.
constexpr int kBBoxBlocks = 1024;
constexpr int kBBoxThreads = 256;
constexpr int kBBoxUnroll = 2;  // elements per thread in flight together
constexpr int kScanBlocks = 1024;
constexpr int kMaxMaterials = 16;
// Slots past max_nbr in each pair-list row: the list build writes a column
// of up to 64 hits before it checks a row's length.
constexpr int kRowGuard = 64;

// ------------------------------------------------------------ host helpers
#define SPH_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t _e = (expr);                                                \
        if (_e != hipSuccess) {                                                \
            set_error(ctx, "%s: %s", #expr, hipGetErrorString(_e));            \
            return SPH_EHIP;                                                   \
        }                                                                      \
    } while (0)

void set_error(Ctx *ctx, const char *fmt, ...);

// Entries between consecutive pair-list rows.
inline int32_t nbr_stride(const Ctx *ctx) { return ctx->max_nbr + kRowGuard; }

// Timing bracket around a pass kernel launch (no-op unless enabled).
struct TimedLaunch {
    Ctx *ctx;
    int which;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(Ctx *c, int w, hipStream_t st);
    ~TimedLaunch();
};

// Optional work fused into the neighbour search by the whole-step path:
// drift of the positions before binning, and the density-pass records.
struct BuildExtras {
    const double *dt = nullptr;                  // drift x += dt v (non-fixed) when set
    const double *vx = nullptr, *vy = nullptr, *vz = nullptr;
    const int32_t *fixed = nullptr;
    const double *m = nullptr;                   // write density records when set
    int32_t f32 = 0;                             // record arithmetic
    double far_factor = 0.0;                     // > 0: far cubes in use (sph_params)
    int32_t far_init = 0;                        // set the far cubes from this search's boxes
};

// Launch helpers implemented in the .hip files.
sph_status launch_build_cells(Ctx *ctx, int64_t n, double *x, double *y, double *z,
                              const double *h, int32_t n_runs, double cell_min,
                              int32_t *perm_out, const BuildExtras *ex, hipStream_t s);
sph_status launch_reorder(Ctx *ctx, int64_t n, const int32_t *perm, int32_t nf,
                          const void *const *src, void *const *dst, const int32_t *eb,
                          const int32_t *rows, hipStream_t s);
sph_status launch_csr(Ctx *ctx, int64_t *off, int32_t *nbr, uint8_t *dflag, hipStream_t s);
sph_status launch_density(Ctx *ctx, int64_t n, const double *m, const double *h,
                          const double *u, const int32_t *mat, int32_t nmat,
                          const sph_params *prm, sph_precision prec, double *rho,
                          double *omega, double *P, double *cs, double *T, double *Y,
                          double *Gmod, hipStream_t s);
sph_status launch_gradients(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                            const double *vz, const double *m, const double *h,
                            const double *rho, const double *omega, const sph_params *prm,
                            sph_precision prec, double *G, int64_t *n_singular, hipStream_t s);
sph_status launch_forces(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                         const double *vz, const double *m, const double *h, const double *rho,
                         const double *omega, const double *P, const double *cs,
                         const double *S, const sph_params *prm, sph_precision prec,
                         double *ax, double *ay, double *az, double *dudt, double *dtc,
                         hipStream_t s);
sph_status launch_stress(Ctx *ctx, int32_t phase, int64_t n, const double *dt,
                         const double *dt_next, const double *G, const double *Y,
                         const double *Gmod, const int32_t *fixed, const sph_params *prm,
                         double *S_half, double *S_pred, double *Sdot, double *eps2,
                         hipStream_t s);
sph_status launch_kick_drift(Ctx *ctx, int32_t phase, int64_t n, const double *dt,
                             const double *dt_next, const int32_t *fixed, double *x, double *y,
                             double *z, double *vx, double *vy, double *vz, double *u,
                             const double *ax, const double *ay, const double *az,
                             const double *dudt, double *vpx, double *vpy, double *vpz,
                             double *up, hipStream_t s);
// Per-run minima (nr runs over run_p) into out[0..nr); nr = 1 with a null
// run_p is the whole range.
sph_status launch_dt_min(Ctx *ctx, int64_t n, const double *dtc, const int32_t *fixed,
                         double cap, double *out, hipStream_t s, int32_t nr = 1,
                         const int32_t *run_p = nullptr);
// Reduction only, into bits (the step's kick finishes it); see launch_step_kick.
sph_status launch_dt_reduce(Ctx *ctx, int64_t n, const double *dtc, const int32_t *fixed,
                            unsigned long long *bits, hipStream_t s, int32_t nr,
                            const int32_t *run_p, bool skip_far = false);

// Self-gravity of every run at the last build (sorted order); see sph_gravity.
// tmask (may be NULL): only the targets with tmask[i] != 0 receive outputs.
sph_status launch_gravity(Ctx *ctx, int64_t n, const double *m, const int32_t *active, double G,
                          double eps_over_h, double theta, int32_t accumulate, double *ax,
                          double *ay, double *az, double *phi, hipStream_t s,
                          const int32_t *tmask = nullptr);
size_t gravity_levels_bytes(int32_t max_runs);
sph_status launch_bound_mass(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                             const double *vz, const double *m, double G, double eps_over_h,
                             double theta, int32_t max_iter, int32_t *bound, double *m_bound,
                             double *phi, double *acc3, int32_t *iterations, hipStream_t s);
size_t bound_mass_part_bytes(int32_t max_runs);
// Adaptive smoothing lengths over the last build's lists; see sph_adapt_h.
sph_status launch_adapt_h(Ctx *ctx, int64_t n, const double *m, const double *h_start,
                          const int32_t *fixed, double n_ngb, double tol, int32_t max_iter,
                          double *h_out, int64_t *n_clamped, int32_t *iterations,
                          hipStream_t s);
// b = f a (n doubles)
sph_status launch_scale(Ctx *ctx, int64_t n, const double *a, double f, double *b,
                        hipStream_t s);

// Time step of sorted particle i: one per run when runid is given.
__device__ __forceinline__ double dt_of(const double *dtp, const int16_t *runid, int64_t i) {
    return dtp[runid ? (int)runid[i] : 0];
}
sph_status launch_diag(Ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                       const double *vx, const double *vy, const double *vz, const double *m,
                       const double *ax, const double *ay, const double *az,
                       const double *dudt, double *out, hipStream_t s);
sph_status launch_fill_i32(Ctx *ctx, int32_t *p, int32_t v, int64_t n, hipStream_t s);
// Message of the last failed context-free call on this thread (or NULL).
const char *noalloc_last_error();
// pair kernels alone (records already written)
sph_status launch_density_pairs(Ctx *ctx, int64_t n, const sph_params *prm, sph_precision prec,
                                double *rho, double *omega, hipStream_t s);
sph_status launch_gradient_pairs(Ctx *ctx, int64_t n, sph_precision prec, hipStream_t s);
sph_status launch_force_pairs(Ctx *ctx, int64_t n, const sph_params *prm, sph_precision prec,
                              double *ax, double *ay, double *az, double *dudt, double *dtc,
                              hipStream_t s);
// act (may be NULL): only the particles with act[i] != 0 are evaluated.
sph_status launch_grad_force_pairs(Ctx *ctx, int64_t n, const sph_params *prm,
                                   sph_precision prec, double *ax, double *ay, double *az,
                                   double *dudt, double *dtc, hipStream_t s,
                                   const int32_t *act = nullptr);
// fused whole-step kernels: source and destination rows of the reorder
struct StepRows {
    const double *f_src[SPH_NF64];
    double *f_dst[SPH_NF64];
    const int32_t *i_src[SPH_NI32];
    int32_t *i_dst[SPH_NI32];
};
sph_status launch_step_reorder(Ctx *ctx, int64_t n, const int32_t *perm, const StepRows &r,
                               const double *dt, const int16_t *runid, int32_t predict,
                               int32_t hier, double tick, double *vpx, double *vpy, double *vpz,
                               double *up, double *tau, int32_t *act, hipStream_t s);
sph_status launch_step_state(Ctx *ctx, int64_t n, sph_precision prec, const double *rho,
                             const double *omega, const double *up, const double *vpx,
                             const double *vpy, const double *vpz, const double *m,
                             const int32_t *mat, int32_t nmat, const int32_t *fixed,
                             const double *tau, const double *S_half, const double *Sdot,
                             double *P, double *cs, double *T, double *Y, double *Gmod,
                             double *S_pred, hipStream_t s);
sph_status launch_step_grad_rate(Ctx *ctx, int64_t n, const sph_params *prm, int32_t gsum_f32,
                                 const double *S_pred, const double *Gmod, const int32_t *fixed,
                                 const double *tau, const int32_t *act, double *G,
                                 double *Sdot, double *eps2, int64_t *n_singular, hipStream_t s);
sph_status launch_accel_limit(Ctx *ctx, int64_t n, double eta_a, const double *ax,
                              const double *ay, const double *az, const double *h,
                              const int32_t *act, double *dtc, hipStream_t s);
sph_status launch_kick_hier(Ctx *ctx, int64_t n, int32_t init, int32_t rungs, double tick,
                            const double *dt, const double *clock, const int16_t *runid,
                            const int32_t *fixed, const int32_t *act, double *vx, double *vy,
                            double *vz, double *u, const double *ax, const double *ay,
                            const double *az, const double *dudt, double *S_half,
                            const double *S_pred, const double *Sdot, const double *Y,
                            const double *dtc, double *step, double *elapsed, double *rem,
                            hipStream_t s);
sph_status launch_hier_next(Ctx *ctx, int32_t nr, int32_t init, double tick,
                            const unsigned long long *bits_cur, unsigned long long *bits_clear,
                            const double *dt, double *dt_next, double *clock, double *time,
                            hipStream_t s);
// Kicks; the next step of each run is taken from the minima in bits_cur
// (capped at dt_cap when > 0) and written to dt_next[0..nr); bits_clear is
// set to +inf for the following reduction.
sph_status launch_step_kick(Ctx *ctx, int64_t n, int32_t mode, const double *dt,
                            const unsigned long long *bits_cur, double dt_cap,
                            double *dt_next, unsigned long long *bits_clear, int32_t nr,
                            const int16_t *runid, const int32_t *fixed, double *vx, double *vy,
                            double *vz, double *u, const double *ax, const double *ay,
                            const double *az, const double *dudt, double *S_half,
                            const double *S_pred, const double *Sdot, const double *Y,
                            double *time, hipStream_t s);

}  // namespace sph
