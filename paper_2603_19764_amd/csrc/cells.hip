// Neighbour search of the strength-SPH hot path on gfx950: uniform cell
// grid per run, counting sort of particles by the Morton key of their cell,
// and the exact pair sets N_i built from LDS-staged candidate tiles.
//
// Pair set (symmetrised sums of the acceleration and Velocity_Gradient
// eqs.): N_i = { j != i : r_ij^2 < max((2h_i)^2, (2h_j)^2) }, kernel support
// H = 2h; density set: r_ij^2 < (2h_i)^2 (Density_estimate eq.).
#include <stdarg.h>
#include <stdio.h>

#include <type_traits>

#include "sph_internal.h"

namespace sph {

// ------------------------------------------------------------- utilities
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

sph_status launch_fill_i32(Ctx *ctx, int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return SPH_OK;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, p, v, n);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

// ------------------------------------------------ exclusive scan (device length)
// out[k] = sum_{l<k} in[l] for k <= len (out[len] = total).  Three phases:
// per-block sums over contiguous chunks, scan of the block sums, rescan.
template <typename Tin>
__global__ void k_scan_reduce(const Tin *in, const int32_t *len32_dev, int64_t len_host,
                              int64_t *part) {
    const int64_t len = len32_dev ? (int64_t)*len32_dev : len_host;
    const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const int64_t a = blockIdx.x * chunk, b = a + chunk < len ? a + chunk : len;
    int64_t s = 0;
    for (int64_t k = a + threadIdx.x; k < b; k += blockDim.x) s += (int64_t)in[k];
    __shared__ int64_t red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Each block adds the totals of the blocks before it (a short reduction of
// at most gridDim.x values, no inter-block signalling), then scans its chunk.
template <typename Tin, typename Tout>
__global__ void k_scan_final(const Tin *in, Tout *out, const int32_t *len32_dev, int64_t len_host,
                             const int64_t *part) {
    const int64_t len = len32_dev ? (int64_t)*len32_dev : len_host;
    const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const int64_t a = blockIdx.x * chunk, b = a + chunk < len ? a + chunk : len;
    __shared__ int64_t sh[256];
    int64_t pre = 0;
    for (unsigned q = threadIdx.x; q < blockIdx.x; q += blockDim.x) pre += part[q];
    sh[threadIdx.x] = pre;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    int64_t carry = sh[0];
    __syncthreads();
    for (int64_t base = a; base < b; base += blockDim.x) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < b ? (int64_t)in[k] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < b) out[k] = (Tout)(carry + sh[threadIdx.x] - v);
        const int64_t tot = sh[255];
        __syncthreads();
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[len] = (Tout)carry;
}

template <typename Tin, typename Tout>
static sph_status scan(Ctx *ctx, const Tin *in, Tout *out, const int32_t *len32_dev,
                       int64_t len_host, hipStream_t s) {
    const int nb = kScanBlocks;
    hipLaunchKernelGGL((k_scan_reduce<Tin>), dim3(nb), dim3(256), 0, s, in, len32_dev, len_host,
                       ctx->scan_part);
    hipLaunchKernelGGL((k_scan_final<Tin, Tout>), dim3(nb), dim3(256), 0, s, in, out, len32_dev,
                       len_host, ctx->scan_part);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

// ------------------------------------------------------------ grid set-up
__device__ __forceinline__ int run_of(const int32_t *run_p, int nr, int64_t k) {
    int lo = 0, hi = nr;  // run_p[lo] <= k < run_p[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (run_p[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

// Per-run bounding box and largest h (partials per block).  Also: optional
// drift x += dt v of the non-fixed particles before binning, and zeroing of
// the cell-count entries the previous build used (the only non-zero ones).
__global__ void k_bbox(double *x, double *y, double *z, const double *h, const int32_t *run_p,
                       BBox *part, int32_t *cell_count, const int32_t *total_keys_prev,
                       const double *dtp, const double *vx, const double *vy, const double *vz,
                       const int32_t *fixed, const BBox *far, int32_t *flags) {
    {
        const int64_t nz = *total_keys_prev;
        const int64_t nthr = (int64_t)gridDim.x * gridDim.y * blockDim.x;
        for (int64_t k = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
             k < nz; k += nthr)
            cell_count[k] = 0;
    }
    const int r = blockIdx.y;
    const int64_t a = run_p[r], b = run_p[r + 1];
    const double dt = dtp ? dtp[r] : 0.0;  // one time step per run
    // with far cubes, particles outside the run's cube stay out of its box
    BBox fb;
    if (far) fb = far[r];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hm = 0.0;
    bool bad = false;  // a non-finite position or length (binned at the grid's edge, reported)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k0 = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k0 < b;
         k0 += kBBoxUnroll * stride) {
        // kBBoxUnroll independent elements: their loads are in flight together
#pragma unroll
        for (int u = 0; u < kBBoxUnroll; ++u) {
            const int64_t k = k0 + u * stride;
            if (k < b) {
                double v[3] = {x[k], y[k], z[k]};
                if (dtp && !(fixed && fixed[k])) {
                    v[0] += dt * vx[k];
                    v[1] += dt * vy[k];
                    v[2] += dt * vz[k];
                    x[k] = v[0];
                    y[k] = v[1];
                    z[k] = v[2];
                }
                bool in = true;
                if (far)
                    for (int d = 0; d < 3; ++d) in = in && v[d] >= fb.lo[d] && v[d] <= fb.hi[d];
                if (in) {
                    for (int d = 0; d < 3; ++d) {
                        lo[d] = fmin(lo[d], v[d]);
                        hi[d] = fmax(hi[d], v[d]);
                    }
                    hm = fmax(hm, h[k]);
                }
                bad |= nonfinite(v[0], v[1], v[2], h[k]);
            }
        }
    }
    flag_if(bad, flags, FLAG_NONFINITE);
    // wave minima/maxima by shuffles, then across the block's waves in LDS
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], __shfl_xor(lo[d], o));
            hi[d] = fmax(hi[d], __shfl_xor(hi[d], o));
        }
        hm = fmax(hm, __shfl_xor(hm, o));
    }
    constexpr int kW = kBBoxThreads / kWave;
    __shared__ double sh[7][kW];
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        for (int d = 0; d < 3; ++d) {
            sh[d][w] = lo[d];
            sh[3 + d][w] = hi[d];
        }
        sh[6][w] = hm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BBox bb;
        for (int d = 0; d < 3; ++d) {
            bb.lo[d] = sh[d][0];
            bb.hi[d] = sh[3 + d][0];
        }
        bb.hmax = sh[6][0];
        for (int v = 1; v < kW; ++v) {
            for (int d = 0; d < 3; ++d) {
                bb.lo[d] = fmin(bb.lo[d], sh[d][v]);
                bb.hi[d] = fmax(bb.hi[d], sh[3 + d][v]);
            }
            bb.hmax = fmax(bb.hmax, sh[6][v]);
        }
        part[r * kBBoxBlocks + blockIdx.x] = bb;
    }
}

__device__ static int bits_for(int n) {
    int b = 0;
    while ((1 << b) < n) ++b;
    return b;
}

// Cell grid of one run over its bounding box for an edge L (raised where an
// axis would need more than 2^kMaxMortonBits - 2 cells): origin, cells and
// Morton bits per axis, dense key count.
__device__ static void size_grid(GridDesc &g, const BBox &bb, double L) {
    if (!(L > 0.0)) L = 1.0;
    for (int d = 0; d < 3; ++d) {
        const double ext = bb.hi[d] - bb.lo[d];
        if (ext / L > (double)((1 << kMaxMortonBits) - 2)) L = ext / (double)((1 << kMaxMortonBits) - 2);
    }
    int dims[3];
    for (int d = 0; d < 3; ++d) {
        const double ext = bb.hi[d] - bb.lo[d];
        const int nd = (int)floor(ext / L) + 1;
        dims[d] = nd < 1 ? 1 : nd;
    }
    g.ox = bb.lo[0]; g.oy = bb.lo[1]; g.oz = bb.lo[2];
    g.L = L;
    g.invL = 1.0 / L;
    g.L32 = (float)L;
    g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
    g.bx = bits_for(dims[0]); g.by = bits_for(dims[1]); g.bz = bits_for(dims[2]);
    g.key_count = 1 << (g.bx + g.by + g.bz);
    g.key_off = 0;
}

// Per-run grids that fit the cell table.  The block first reduces each
// run's bounding-box partials in parallel (into the first partial of the
// run), then one thread sizes the grids.
__global__ void k_grid(BBox *part, int nbb, const int32_t *run_p, int nr, double cell_min,
                       double cell_scale, int64_t max_cells, GridDesc *grid, int32_t *total_keys,
                       double far_factor, BBox *far_set, int32_t *flags) {
    // per run: the nbb block partials reduced by one wave (waves take runs
    // in turn); the result goes to the run's first partial
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    for (int r = w; r < nr; r += nw) {
        double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
        for (int b = lane; b < nbb; b += kWave) {
            const BBox o = part[r * kBBoxBlocks + b];
            for (int d = 0; d < 3; ++d) {
                v[d] = fmin(v[d], o.lo[d]);
                v[3 + d] = fmax(v[3 + d], o.hi[d]);
            }
            v[6] = fmax(v[6], o.hmax);
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) v[d] = fmin(v[d], __shfl_xor(v[d], o));
#pragma unroll
            for (int d = 3; d < 7; ++d) v[d] = fmax(v[d], __shfl_xor(v[d], o));
        }
        if (lane == 0) {
            BBox bb;
            for (int d = 0; d < 3; ++d) {
                bb.lo[d] = v[d];
                bb.hi[d] = v[3 + d];
            }
            bb.hmax = v[6];
            part[r * kBBoxBlocks] = bb;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // Every run at its natural edge first; while the dense key ranges do not
    // fit the table, the run holding the most keys (the one whose particles
    // spread widest, e.g. the ejecta of a disruptive impact) coarsens its own
    // grid by 1.25, so one dispersing run does not coarsen the others.  With
    // far cubes every run has one more key after its cells, for the particles
    // outside its cube.
    const int sink = far_factor > 0.0 ? 1 : 0;
    int64_t total = 0;
    for (int r = 0; r < nr; ++r) {
        BBox bb = part[r * kBBoxBlocks];
        GridDesc g;
        g.p0 = run_p[r];
        g.p1 = run_p[r + 1];
        g.sink = sink;
        g.pad = 0;
        if (g.p1 <= g.p0 || !(bb.lo[0] <= bb.hi[0])) {  // empty run (or no particle in its cube)
            for (int d = 0; d < 3; ++d) { bb.lo[d] = 0.0; bb.hi[d] = 0.0; }
            bb.hmax = 0.0;
        }
        if (far_set) {
            // the cube: centred on the box, half-edge far_factor times its
            // largest half-extent (at least one cell edge)
            double half = 0.0;
            for (int d = 0; d < 3; ++d) half = fmax(half, 0.5 * (bb.hi[d] - bb.lo[d]));
            half = far_factor * fmax(half, fmax(cell_min, 2.0 * bb.hmax));
            BBox c;
            for (int d = 0; d < 3; ++d) {
                const double mid = 0.5 * (bb.lo[d] + bb.hi[d]);
                c.lo[d] = mid - half;
                c.hi[d] = mid + half;
            }
            c.hmax = 0.0;
            far_set[r] = c;
        }
        part[r * kBBoxBlocks] = bb;
        // Edge at least the largest support 2h (so every pair lies in the
        // 27-cell stencil), slightly enlarged so that rounding of
        // (x - origin)/L can never separate a pair by two cells.
        const double L = fmax(cell_min, 2.0 * bb.hmax * cell_scale) * (1.0 + 1.0 / 1099511627776.0);
        size_grid(g, bb, L);
        grid[r] = g;
        total += g.key_count + sink;
    }
    // (the search for the largest run is a scan over the runs, done by one
    // thread: beyond 1024 runs every run coarsens together instead)
    for (int attempt = 0; nr > 1024 && attempt < 64 && total > max_cells; ++attempt) {
        total = 0;
        for (int r = 0; r < nr; ++r) {
            GridDesc g = grid[r];
            BBox bb = part[r * kBBoxBlocks];
            if (g.p1 <= g.p0) {
                for (int d = 0; d < 3; ++d) { bb.lo[d] = 0.0; bb.hi[d] = 0.0; }
            }
            size_grid(g, bb, g.L * 1.25);
            grid[r] = g;
            total += g.key_count + sink;
        }
    }
    for (int attempt = 0; attempt < 4096 && total > max_cells; ++attempt) {
        int big = 0;
        for (int r = 1; r < nr; ++r)
            if (grid[r].key_count > grid[big].key_count) big = r;
        GridDesc g = grid[big];
        if (g.key_count <= 1) break;
        BBox bb = part[big * kBBoxBlocks];
        if (g.p1 <= g.p0) {
            for (int d = 0; d < 3; ++d) { bb.lo[d] = 0.0; bb.hi[d] = 0.0; }
        }
        total -= g.key_count;
        size_grid(g, bb, g.L * 1.25);
        grid[big] = g;
        total += g.key_count;
    }
    if (total <= max_cells) {
        int64_t off = 0;
        for (int r = 0; r < nr; ++r) {
            grid[r].key_off = (int32_t)off;
            off += grid[r].key_count + sink;
        }
        *total_keys = (int32_t)total;
        return;
    }
    flags[FLAG_CELL_OVERFLOW] = 1;
    *total_keys = 0;
}

__device__ __forceinline__ void cell_of(const GridDesc &g, double x, double y, double z,
                                        int &cx, int &cy, int &cz) {
    cx = (int)floor((x - g.ox) * g.invL);
    cy = (int)floor((y - g.oy) * g.invL);
    cz = (int)floor((z - g.oz) * g.invL);
    cx = cx < 0 ? 0 : (cx >= g.nx ? g.nx - 1 : cx);
    cy = cy < 0 ? 0 : (cy >= g.ny ? g.ny - 1 : cy);
    cz = cz < 0 ? 0 : (cz >= g.nz ? g.nz - 1 : cz);
}

__global__ void k_keys(int64_t n, const double *x, const double *y, const double *z,
                       const int32_t *run_p, int nr, const GridDesc *grid,
                       const int32_t *total_keys, const BBox *far, uint32_t *key, int32_t *slot,
                       int32_t *cell_count) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool valid = k < n;
    if (*total_keys == 0) {  // table overflow: flagged, produce a valid (empty) permutation
        if (valid) {
            key[k] = 0;
            slot[k] = 0;
        }
        return;
    }
    uint32_t kk = 0xffffffffu;
    int oct = 0;
    if (valid) {
        const int r = nr > 1 ? run_of(run_p, nr, k) : 0;
        const GridDesc g = grid[r];
        const double tx = (x[k] - g.ox) * g.invL, ty = (y[k] - g.oy) * g.invL,
                     tz = (z[k] - g.oz) * g.invL;
        int cx = (int)floor(tx), cy = (int)floor(ty), cz = (int)floor(tz);
        cx = cx < 0 ? 0 : (cx >= g.nx ? g.nx - 1 : cx);
        cy = cy < 0 ? 0 : (cy >= g.ny ? g.ny - 1 : cy);
        cz = cz < 0 ? 0 : (cz >= g.nz ? g.nz - 1 : cz);
        kk = (uint32_t)g.key_off + morton(cx, cy, cz, g.bx, g.by, g.bz);
        // octant of the particle in its cell (the half-cells of the gravity
        // tree below the search cells)
        oct = (tx - cx >= 0.5 ? 1 : 0) | (ty - cy >= 0.5 ? 2 : 0) | (tz - cz >= 0.5 ? 4 : 0);
        if (far) {  // outside the run's far cube: the run's far slot
            const BBox fb = far[r];
            const double p[3] = {x[k], y[k], z[k]};
            bool in = true;
            for (int d = 0; d < 3; ++d) in = in && p[d] >= fb.lo[d] && p[d] <= fb.hi[d];
            if (!in) {
                kk = far_key(g);
                oct = 0;
            }
        }
        key[k] = kk;
    }
    // One atomic per distinct key of the wave: lanes with equal keys take
    // consecutive slots in lane order.  Each group's leader issues the
    // atomic; every lane reads its leader's result once all are issued.
    const int lane = threadIdx.x % kWave;
    uint64_t todo = __ballot(valid);
    int my_leader = 0, my_rank = 0, lead_base = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t lk = __shfl(kk, leader);
        const uint64_t peers = __ballot(valid && kk == lk);
        if (lane == leader) lead_base = atomicAdd(&cell_count[lk], __popcll(peers));
        if (valid && kk == lk) {
            my_leader = leader;
            my_rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        }
        todo &= ~peers;
    }
    const int my_slot = __shfl(lead_base, my_leader) + my_rank;
    if (valid) slot[k] = my_slot | (oct << kIdxBits);
}

__global__ void k_scatter(int64_t n, const uint32_t *key, const int32_t *slot,
                          const int32_t *cell_start, const int32_t *total_keys, int32_t *out) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (*total_keys == 0) {
        out[k] = (int32_t)k;
        return;
    }
    const int32_t sl = slot[k];
    out[cell_start[key[k]] + (sl & (int32_t)kIdxMask)] = (int32_t)k | (sl & ~(int32_t)kIdxMask);
}

// Arrival order inside a cell depends on atomics; placing each member at its
// rank by (octant, input index) makes the permutation deterministic and
// leaves the members of each octant contiguous.  One thread per particle
// counts the members of its cell that precede it; arrival entries hold the
// input index in the low kIdxBits bits and the octant above them.  The same
// thread then writes the sorted copies at the particle's place q: positions
// and h, cell-relative float offsets, packed cell coordinates, run id,
// sorted key, the density-pass record, perm (and perm_out for the caller).
__global__ void k_place(int64_t n, const int32_t *__restrict__ arrived,
                        const uint32_t *__restrict__ key, const int32_t *__restrict__ cell_start,
                        const int32_t *__restrict__ cell_count, const int32_t *total_keys,
                        int32_t *__restrict__ perm, uint8_t *__restrict__ octant,
                        const double *x, const double *y, const double *z, const double *h,
                        const int32_t *run_p, int nr, const GridDesc *grid, double4 *posh64,
                        float4 *posh32, uint32_t *cellc, int16_t *runid, uint32_t *skey,
                        int32_t *perm_out, const double *m, void *rec_d, int32_t f32) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t e = arrived[p];
    const int32_t o = e & (int32_t)kIdxMask;
    const uint32_t ko = key[o];
    // the particle's own data and run do not depend on its rank (a run's
    // particles take the same index range before and after the sort)
    const double xo = x[o], yo = y[o], zo = z[o], ho = h[o];
    const double mo = m ? m[o] : 0.0;
    const int r = nr > 1 ? run_of(run_p, nr, o) : 0;
    const GridDesc g = grid[r];
    int64_t q = p;
    uint8_t oct = 0;
    if (*total_keys != 0) {
        const int32_t cs = cell_start[ko], c = cell_count[ko];
        int rank = 0;
        // four loads in flight per step (a cell holds a few tens)
        int l = 0;
        for (; l + 4 <= c; l += 4) {
            const int32_t a0 = arrived[cs + l], a1 = arrived[cs + l + 1];
            const int32_t a2 = arrived[cs + l + 2], a3 = arrived[cs + l + 3];
            rank += (a0 < e) + (a1 < e) + (a2 < e) + (a3 < e);
        }
        for (; l < c; ++l) rank += arrived[cs + l] < e;
        q = cs + rank;
        oct = (uint8_t)(e >> kIdxBits);
    }
    perm[q] = o;
    octant[q] = oct;
    int cx, cy, cz;
    cell_of(g, xo, yo, zo, cx, cy, cz);
    posh64[q] = make_double4(xo, yo, zo, ho);
    const double dx = (xo - g.ox) - (double)cx * g.L;
    const double dy = (yo - g.oy) - (double)cy * g.L;
    const double dz = (zo - g.oz) - (double)cz * g.L;
    posh32[q] = make_float4((float)dx, (float)dy, (float)dz, (float)ho);
    if (m) {  // density-pass record (p, m) of the sorted particle
        if (f32)
            ((float4 *)rec_d)[q] = make_float4((float)dx, (float)dy, (float)dz, (float)mo);
        else
            ((double4 *)rec_d)[q] = make_double4(xo, yo, zo, mo);
    }
    cellc[q] = (uint32_t)cx | ((uint32_t)cy << 10) | ((uint32_t)cz << 20);
    runid[q] = (int16_t)r;
    skey[q] = ko;
    if (perm_out) perm_out[q] = o;
}

// ------------------------------------------------------ pair-set builder
// One wave per work-group.  The work-group owns a contiguous range of
// sorted particles and walks it cell by cell, in batches of up to 64
// particles i of one cell.  For each batch, the candidates of the 27
// neighbour cells (stencil order, then sorted index) are culled and
// compacted into an LDS tile: a candidate j farther from the bounding box of
// the batch than max(max_i H_i, H_j) can pair with none of them (the
// distance to the box bounds every |x_i - x_j| from below; the cut keeps a
// 2^-40 relative margin over rounding, so the exact criterion still decides
// every pair that can be one).  The tests then run four i at a time: their
// positions and running counts are wave-uniform (scalar registers) while
// each lane holds one candidate of a 64-wide column of the tile; one exact
// test per lane, a ballot, and the hits are appended to i's list in
// candidate order at offsets from mbcnt.  The lists are deterministic.
constexpr int kFillChunks = 3;  // raw-candidate chunks whose loads overlap
constexpr int kIBatch = 64;
constexpr double kCullMargin = 1.0 + 0x1p-40;

__device__ __forceinline__ uint64_t wave_ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }
// This lane's bit of a wave mask, as a lane predicate (no vector instruction).
__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }
// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Tile: candidates the LDS tile holds (36 B each): 256 entries take 9.4 KB per
// single-wave work-group (17 work-groups, 4.25 waves per SIMD), 192 take 7.1 KB
// (5 waves, the register limit), 128 take 4.8 KB.
template <int Tile>
__global__ __launch_bounds__(64) void k_build_pairs(
    int64_t n, const double4 *__restrict__ posh64, const uint32_t *__restrict__ skey,
    const uint32_t *__restrict__ cellc, const int16_t *__restrict__ runid,
    const GridDesc *__restrict__ grid, const int32_t *__restrict__ cell_start,
    const int32_t *__restrict__ cell_count, const int32_t *total_keys, uint32_t *nbr,
    int32_t *ncount, int32_t K, int32_t stride, int32_t *flags, unsigned long long *pairs) {
    __shared__ double4 tpos[Tile];  // x, y, z, H_j^2
    __shared__ uint32_t tj[Tile];   // j | stencil code
    __shared__ int32_t st_start[27];
    // first raw candidate index of each stencil cell; 27..31 hold INT_MAX so
    // that the cell search below reads whole groups of eight
    __shared__ __align__(16) int32_t st_off[32];

    const int lane = threadIdx.x;
    const uint32_t wg = xcd_block(blockIdx.x, gridDim.x);
    const int64_t p_begin = n * (int64_t)wg / gridDim.x;
    const int64_t p_end = n * (int64_t)(wg + 1) / gridDim.x;
    if (*total_keys == 0) {  // table overflow (flagged): leave empty, valid lists
        for (int64_t q = p_begin + lane; q < p_end; q += kWave) ncount[q] = 0;
        return;
    }
    unsigned long long my_pairs = 0;

    int64_t p = p_begin;
    while (p < p_end) {
        const uint32_t key = skey[p];
        const int64_t cs = cell_start[key];
        const int64_t ce = cs + cell_count[key];
        const int64_t i_lo = p;
        const int64_t i_hi = ce < p_end ? ce : p_end;
        if (i_hi <= i_lo) {  // inconsistent cell table: never loop without progress
            for (int64_t q = p + lane; q < p_end; q += kWave) ncount[q] = 0;
            if (lane == 0) atomicOr(&flags[FLAG_CELL_OVERFLOW], 2);
            break;
        }
        {
            const GridDesc gr = grid[runid[p]];
            if (gr.sink && key == far_key(gr)) {  // outside the far cube: no pair set
                for (int64_t q = i_lo + lane; q < i_hi; q += kWave) ncount[q] = 0;
                p = i_hi;
                continue;
            }
        }
        // ---- stencil: 27 neighbour cells (lane t handles cell t)
        const uint32_t cc = cellc[p];
        const GridDesc g = grid[runid[p]];
        int cnt_t = 0, start_t = 0;
        if (lane < 27) {
            const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
            const int cx = (int)(cc & 1023u) + dx;
            const int cy = (int)((cc >> 10) & 1023u) + dy;
            const int cz = (int)((cc >> 20) & 1023u) + dz;
            if (cx >= 0 && cx < g.nx && cy >= 0 && cy < g.ny && cz >= 0 && cz < g.nz) {
                const uint32_t kk = (uint32_t)g.key_off + morton(cx, cy, cz, g.bx, g.by, g.bz);
                start_t = cell_start[kk];
                cnt_t = cell_count[kk];
            }
        }
        int incl = cnt_t;  // inclusive scan of the 27 counts across the wave
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        const int T = __shfl(incl, 26);  // raw candidates of the stencil
        __syncthreads();
        if (lane < 27) {
            st_start[lane] = start_t;
            st_off[lane] = incl - cnt_t;
        } else if (lane < 32) {
            st_off[lane] = 0x7fffffff;
        }
        __syncthreads();

        for (int64_t ib = i_lo; ib < i_hi; ib += kIBatch) {
            const int ni = (int)((i_hi - ib) < kIBatch ? (i_hi - ib) : kIBatch);
            // bounding box and largest H^2 of the batch
            double lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
            double hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY, hm = 0.0;
            if (lane < ni) {
                const double4 q = posh64[ib + lane];
                const double H = 2.0 * q.w;
                lo0 = hi0 = q.x;
                lo1 = hi1 = q.y;
                lo2 = hi2 = q.z;
                hm = __dmul_rn(H, H);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                lo0 = fmin(lo0, __shfl_xor(lo0, o));
                lo1 = fmin(lo1, __shfl_xor(lo1, o));
                lo2 = fmin(lo2, __shfl_xor(lo2, o));
                hi0 = fmax(hi0, __shfl_xor(hi0, o));
                hi1 = fmax(hi1, __shfl_xor(hi1, o));
                hi2 = fmax(hi2, __shfl_xor(hi2, o));
                hm = fmax(hm, __shfl_xor(hm, o));
            }
            int cnt_reg = 0;  // lane q: running count of particle ib + q
            const double4 *ipos = posh64 + ib;

            int fill = 0;  // kept candidates in the tile (carried over between chunks)
            for (int r0 = 0; r0 < T || fill > 0;) {
                // ---- fill: cull raw candidates into the tile
                __syncthreads();
                for (; r0 < T && fill <= Tile - kWave;) {
                    // up to kFillChunks chunks of 64 raw candidates at once:
                    // their searches and loads overlap, then they are
                    // appended in order (as many as the tile has room for)
                    int nch = (Tile - fill) / kWave;
                    const int left = (T - r0 + kWave - 1) / kWave;
                    nch = nch < left ? nch : left;
                    nch = nch < kFillChunks ? nch : kFillChunks;
                    int g[kFillChunks], lo[kFillChunks];
#pragma unroll
                    for (int u = 0; u < kFillChunks; ++u) g[u] = r0 + u * kWave + lane;
                    // stencil cell of each raw candidate: the largest t with
                    // st_off[t] <= g, which (offsets do not decrease, st_off[0]
                    // = 0) is the number of t >= 1 with st_off[t] <= g; counted
                    // in two levels, first against st_off[8], [16], [24], then
                    // against the seven entries after the chosen group's first
#pragma unroll
                    for (int u = 0; u < kFillChunks; ++u) {
                        const int b = (st_off[8] <= g[u]) + (st_off[16] <= g[u]) +
                                      (st_off[24] <= g[u]);
                        const int4 q0 = *reinterpret_cast<const int4 *>(&st_off[8 * b]);
                        const int4 q1 = *reinterpret_cast<const int4 *>(&st_off[8 * b + 4]);
                        lo[u] = 8 * b + (q0.y <= g[u]) + (q0.z <= g[u]) + (q0.w <= g[u]) +
                                (q1.x <= g[u]) + (q1.y <= g[u]) + (q1.z <= g[u]) + (q1.w <= g[u]);
                    }
                    double4 c[kFillChunks];
                    uint32_t code[kFillChunks];
                    bool keep[kFillChunks];
#pragma unroll
                    for (int u = 0; u < kFillChunks; ++u) {
                        keep[u] = false;
                        c[u] = make_double4(0.0, 0.0, 0.0, 0.0);
                        code[u] = 0;
                        if (u < nch && g[u] < T) {
                            const int j = st_start[lo[u]] + (g[u] - st_off[lo[u]]);
                            c[u] = posh64[j];
                            code[u] = (uint32_t)j | ((uint32_t)lo[u] << kCodeShift);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kFillChunks; ++u) {
                        if (u < nch && g[u] < T) {
                            const double H = 2.0 * c[u].w;
                            c[u].w = __dmul_rn(H, H);
                            const double ex = fmax(fmax(lo0 - c[u].x, c[u].x - hi0), 0.0);
                            const double ey = fmax(fmax(lo1 - c[u].y, c[u].y - hi1), 0.0);
                            const double ez = fmax(fmax(lo2 - c[u].z, c[u].z - hi2), 0.0);
                            const double d2 = (ex * ex + ey * ey) + ez * ez;
                            keep[u] = !(d2 >= fmax(hm, c[u].w) * kCullMargin);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kFillChunks; ++u) {
                        if (u < nch) {
                            const uint64_t m = wave_ballot(keep[u]);
                            if (keep[u]) {
                                const int s = fill + (int)__builtin_amdgcn_mbcnt_hi(
                                                         (uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                                tpos[s] = c[u];
                                tj[s] = code[u];
                            }
                            fill += __popcll(m);
                        }
                    }
                    r0 += nch * kWave;
                }
                // full columns only while raw candidates remain; the ragged
                // rest is carried to the front of the tile for the next chunk.
                // After the last chunk the ragged column is padded with
                // entries that pair with nothing (NaN position), so every
                // lane of every column loads and tests without a bounds check.
                int cols = (fill / kWave) * kWave;
                if (r0 >= T && cols < fill) {
                    cols += kWave;
                    if (fill + lane < cols) {
                        tpos[fill + lane] = make_double4(NAN, NAN, NAN, -1.0);
                        tj[fill + lane] = 0u;
                    }
                }
                // wave-uniform (keeps the column loop and the running counts
                // in scalar registers)
                cols = __builtin_amdgcn_readfirstlane(cols);
                __syncthreads();
                // ---- tests: G = 4 particles i at a time against every column
                // of the tile (G = 2 or 1 for the last two or one of a batch).
                // The masks are wave ballots of the compares (scalar
                // registers); a lane stores when its bit is set, at the
                // particle's running count plus the hits below it.  A last
                // group of three repeats its last particle: the repeat tests
                // the same candidates and stores the same entries at the same
                // places, so no slot needs a branch.  Rows have a guard of
                // kRowGuard slots past K: a column adds at most 64 entries,
                // and once a row holds K or more the next column writes from K
                // again (the overflow is reported; the extra entries are never
                // read).
                auto test_group = [&](auto gsz, int q0) {
                    constexpr int G = decltype(gsz)::value;
                    const int l = ni - 1;
                    double4 P[G];
                    double H2[G];
                    int qq[G], base[G];
                    uint32_t self[G];
                    uint32_t *row[G];
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        qq[k] = q0 + k < l ? q0 + k : l;
                        P[k] = ipos[qq[k]];
                        const double H = 2.0 * P[k].w;
                        H2[k] = __dmul_rn(H, H);
                        base[k] = __builtin_amdgcn_readlane(cnt_reg, qq[k]);
                        self[k] = (uint32_t)(ib + qq[k]);
                        row[k] = nbr + (ib + qq[k]) * (int64_t)stride;
                    }
                    for (int col = 0; col < cols; col += kWave) {
                        const double4 c = tpos[col + lane];
                        const uint32_t e = tj[col + lane];
                        const uint32_t jj = e & kIdxMask;
                        const uint32_t ed = e | kDensityBit;
                        // all G tests first (their FP64 chains interleave),
                        // then the G appends
                        uint64_t md[G], m[G];
#pragma unroll
                        for (int k = 0; k < G; ++k) {
                            const double r2 = sep2_exact(P[k].x, P[k].y, P[k].z, c.x, c.y, c.z);
                            md[k] = wave_ballot(r2 < H2[k]);                // density set of i
                            const uint64_t mj = wave_ballot(r2 < c.w);     // support of j
                            const uint64_t ms = wave_ballot(jj == self[k]);
                            m[k] = (md[k] | mj) & ~ms;
                        }
#pragma unroll
                        for (int k = 0; k < G; ++k) {
                            const int b = base[k];
                            const int at = b < K ? b : K;
                            const uint32_t v = lane_bit(md[k]) ? ed : e;
                            // wave-uniform base, unsigned lane offset: the
                            // store takes a scalar base and a 32-bit offset
                            uint32_t *dst = row[k] + at;
                            if (lane_bit(m[k])) dst[lanes_below(m[k])] = v;
                            base[k] = b + (int)__popcll(m[k]);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < G; ++k)
                        if (lane == qq[k]) cnt_reg = base[k];
                };
                int q0 = 0;
                for (; q0 + 4 <= ni; q0 += 4) test_group(std::integral_constant<int, 4>{}, q0);
                if (ni - q0 == 3)
                    test_group(std::integral_constant<int, 4>{}, q0);
                else if (ni - q0 == 2)
                    test_group(std::integral_constant<int, 2>{}, q0);
                else if (ni - q0 == 1)
                    test_group(std::integral_constant<int, 1>{}, q0);
                // carry the kept candidates not tested yet (fewer than 64)
                const int rest = fill > cols ? fill - cols : 0;
                double4 cr = make_double4(0.0, 0.0, 0.0, 0.0);
                uint32_t er = 0;
                if (lane < rest) {
                    cr = tpos[cols + lane];
                    er = tj[cols + lane];
                }
                __syncthreads();
                if (lane < rest) {
                    tpos[lane] = cr;
                    tj[lane] = er;
                }
                fill = rest;
            }
            if (lane < ni) {
                ncount[ib + lane] = cnt_reg < K ? cnt_reg : K;
                if (cnt_reg > K) atomicOr(&flags[FLAG_NBR_OVERFLOW], 1);
                my_pairs += (unsigned long long)cnt_reg;
            }
        }
        p = i_hi;
    }
    // wave sum of the pair count, one atomic per work-group
    unsigned long long v = my_pairs;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0 && v) atomicAdd(pairs, v);
}

sph_status launch_build_cells(Ctx *ctx, int64_t n, double *x, double *y, double *z,
                              const double *h, int32_t nr, double cell_min, int32_t *perm_out,
                              const BuildExtras *ex, hipStream_t s) {
    if (n == 0) {
        ctx->n_built = 0;
        ctx->n_runs_built = nr;
        ctx->far_built = false;
        return SPH_OK;
    }
    BuildExtras none;
    if (!ex) ex = &none;
    const int tb = 256;
    const int nb = (int)((n + tb - 1) / tb);
    // blocks per run: about kBBoxUnroll elements per thread (a run's average
    // size), at most kBBoxBlocks
    int64_t nbb = (n / nr + kBBoxThreads * kBBoxUnroll - 1) / (kBBoxThreads * kBBoxUnroll);
    nbb = nbb < 1 ? 1 : (nbb > kBBoxBlocks ? kBBoxBlocks : nbb);
    const bool far = ex->far_factor > 0.0;
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)nbb, nr), dim3(kBBoxThreads), 0, s, x, y, z, h, ctx->run_p,
                       ctx->bbox_part, ctx->cell_count, ctx->total_keys, ex->dt, ex->vx, ex->vy,
                       ex->vz, ex->fixed, (far && !ex->far_init) ? ctx->far_box : nullptr,
                       ctx->flags);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(1024), 0, s, ctx->bbox_part, (int)nbb, ctx->run_p, nr, cell_min,
                       ctx->cell_scale, ctx->max_cells, ctx->grid, ctx->total_keys,
                       far ? ex->far_factor : 0.0, (far && ex->far_init) ? ctx->far_box : nullptr,
                       ctx->flags);
    hipLaunchKernelGGL(k_keys, dim3(nb), dim3(tb), 0, s, n, x, y, z, ctx->run_p, nr, ctx->grid,
                       ctx->total_keys, far ? ctx->far_box : nullptr, ctx->key, ctx->slot,
                       ctx->cell_count);
    sph_status st = scan<int32_t, int32_t>(ctx, ctx->cell_count, ctx->cell_start,
                                           ctx->total_keys, 0, s);
    if (st != SPH_OK) return st;
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(tb), 0, s, n, ctx->key, ctx->slot,
                       ctx->cell_start, ctx->total_keys, ctx->ptmp);
    hipLaunchKernelGGL(k_place, dim3(nb), dim3(tb), 0, s, n, ctx->ptmp, ctx->key,
                       ctx->cell_start, ctx->cell_count, ctx->total_keys, ctx->perm, ctx->octant,
                       x, y, z, h, ctx->run_p, nr, ctx->grid, ctx->posh64, ctx->posh32,
                       ctx->cellc, ctx->runid, ctx->skey, perm_out, ex->m, ctx->rec_d, ex->f32);
    const int64_t per = ctx->build_range;
    int64_t wgs = (n + per - 1) / per;
    if (wgs > 65536) wgs = 65536;
    {
        TimedLaunch tl(ctx, SPH_T_BUILD, s);
#define SPH_BUILD_LAUNCH(T)                                                                    \
    hipLaunchKernelGGL(k_build_pairs<T>, dim3((unsigned)wgs), dim3(64), 0, s, n, ctx->posh64, \
                       ctx->skey, ctx->cellc, ctx->runid, ctx->grid, ctx->cell_start,          \
                       ctx->cell_count, ctx->total_keys, ctx->nbr, ctx->ncount, ctx->max_nbr, \
                       nbr_stride(ctx), ctx->flags, ctx->pairs)
        switch (ctx->build_tile) {
            case 128: SPH_BUILD_LAUNCH(128); break;
            case 192: SPH_BUILD_LAUNCH(192); break;
            default: SPH_BUILD_LAUNCH(256); break;
        }
#undef SPH_BUILD_LAUNCH
    }
    SPH_HIP(hipGetLastError());
    ctx->n_built = n;
    ctx->n_runs_built = nr;
    ctx->far_built = far;
    return SPH_OK;
}

// ----------------------------------------------------------------- reorder
struct ReorderArgs {
    const void *src[32];
    void *dst[32];
    int32_t eb[32];
    int32_t nf;
};

__global__ void k_reorder(int64_t n, const int32_t *__restrict__ perm, ReorderArgs a) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t o = perm[k];
    for (int f = 0; f < a.nf; ++f) {
        if (a.eb[f] == 8)
            ((double *)a.dst[f])[k] = ((const double *)a.src[f])[o];
        else
            ((int32_t *)a.dst[f])[k] = ((const int32_t *)a.src[f])[o];
    }
}

sph_status launch_reorder(Ctx *ctx, int64_t n, const int32_t *perm, int32_t nf,
                          const void *const *src, void *const *dst, const int32_t *eb,
                          const int32_t *rows, hipStream_t s) {
    if (n == 0) return SPH_OK;
    ReorderArgs a;
    a.nf = 0;
    const int nb = (int)((n + 255) / 256);
    for (int f = 0; f < nf; ++f) {
        int nrow = rows ? rows[f] : 1;
        for (int r = 0; r < nrow; ++r) {
            a.src[a.nf] = (const char *)src[f] + (size_t)r * n * eb[f];
            a.dst[a.nf] = (char *)dst[f] + (size_t)r * n * eb[f];
            a.eb[a.nf] = eb[f];
            if (++a.nf == 32) {
                hipLaunchKernelGGL(k_reorder, dim3(nb), dim3(256), 0, s, n, perm, a);
                a.nf = 0;
            }
        }
    }
    if (a.nf) hipLaunchKernelGGL(k_reorder, dim3(nb), dim3(256), 0, s, n, perm, a);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

// ----------------------------------------------------------- CSR export
__global__ void k_csr(int64_t n, const uint32_t *nbr, const int32_t *ncount, int32_t K,
                      const int64_t *off, int32_t *out, uint8_t *dfl) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t o = off[i];
    for (int k = 0; k < ncount[i]; ++k) {
        uint32_t e = nbr[i * (int64_t)K + k];
        out[o + k] = (int32_t)(e & kIdxMask);
        if (dfl) dfl[o + k] = (uint8_t)(e >> 31);
    }
}

sph_status launch_csr(Ctx *ctx, int64_t *off, int32_t *nbr, uint8_t *dflag, hipStream_t s) {
    int64_t n = ctx->n_built;
    sph_status st = scan<int32_t, int64_t>(ctx, ctx->ncount, off, nullptr, n, s);
    if (st != SPH_OK) return st;
    if (nbr && n > 0)
        hipLaunchKernelGGL(k_csr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ctx->nbr,
                           ctx->ncount, nbr_stride(ctx), off, nbr, dflag);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

}  // namespace sph
