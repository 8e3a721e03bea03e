// Self-gravity of each run (the gravitational term of the momentum equation,
// sec. 2.2) for the batched impact scans: Barnes-Hut over a pyramid built on
// the search cells of the last neighbour search.
//
//   level 0   the search cells of the run (edge L >= 2 h_max), indexed by
//             their Morton key in the global cell table;
//   level k   dense grid of 2x2x2 blocks of level k-1, up to the first level
//             whose every dimension is <= 2.
//   level -1  the eight octants of each search cell (the cell build orders
//             the members of a cell by octant).
// Each node holds a monopole (mass and centre of mass, FP32, relative to the
// run's grid origin).  Targets are grouped by pyramid node: a node of level
// up to kGroupTop (4x4x4 cells) whose particles number at most kGroupMax is
// one group, a fuller one is split into its children, down to level 1 (2x2x2
// cells), so sparse debris makes few walks and dense matter groups of a
// few hundred (a larger top level lets the candidate lists of a group's walk
// outgrow their kCand entries).  A node's cells form one range of Morton keys, hence its
// particles one contiguous range of the sorted order.  A group walks the
// pyramid breadth first, one candidate node per lane: a
// node whose box is disjoint from the group's box and for which b < theta d
// is used for every target of the group (b: distance from the node's centre
// of mass to its farthest corner, d: from the centre of mass to the group's
// box); other nodes are opened.  An opened cell tests
// its octants the same way, and the particles of the octants it cannot
// accept are used one by one.  Plummer softening of length
// eps_r = eps_over_h * max_i h_i of the run; sources inside the near field
// exclude the target itself.
#include "sph_internal.h"
#include <type_traits>

namespace sph {

constexpr int kGravLevels = 12;
constexpr int kCand = 1024;   // candidates of one level (>= 1) of one group walk
constexpr int kIL = 128;      // accepted monopoles held before evaluation
constexpr int kStage = 64;    // near-field source particles held before evaluation
constexpr int kSlots = 8;     // targets per lane per pass
constexpr int kEvalStep = 2;  // list entries evaluated together
constexpr int kGroupTop = 2;    // highest pyramid level of a target group
constexpr int kGroupMax = 256;  // particles of a group above level 1

struct GravLevels {
    int32_t nlev;                      // levels 0 .. nlev-1
    int32_t nx[kGravLevels], ny[kGravLevels], nz[kGravLevels];
    int64_t off[kGravLevels];          // level k >= 1: first node in the upper array
    int32_t grp_top;                   // highest level of this run's groups (0: one cell)
    double eps;                        // softening length
};

__device__ __forceinline__ int ceil_half(int n, int k) { return (n + (1 << k) - 1) >> k; }

// One thread: level sizes and offsets of every run, group offsets, totals.
__global__ void k_grav_layout(int nr, const GridDesc *__restrict__ grid,
                              const BBox *__restrict__ bbox_part, double eps_over_h,
                              GravLevels *lev, int64_t *totals, int64_t cap_upper,
                              int32_t *flags) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t up = 0, groups = 0;
    for (int r = 0; r < nr; ++r) {
        const GridDesc g = grid[r];
        GravLevels L;
        L.nx[0] = g.nx; L.ny[0] = g.ny; L.nz[0] = g.nz;
        L.off[0] = 0;
        int k = 0;
        while (k + 1 < kGravLevels && (L.nx[k] > 2 || L.ny[k] > 2 || L.nz[k] > 2)) {
            ++k;
            L.nx[k] = ceil_half(g.nx, k);
            L.ny[k] = ceil_half(g.ny, k);
            L.nz[k] = ceil_half(g.nz, k);
            L.off[k] = up;
            up += (int64_t)L.nx[k] * L.ny[k] * L.nz[k];
        }
        L.nlev = k + 1;
        const int top = kGroupTop < L.nlev - 1 ? kGroupTop : L.nlev - 1;
        L.grp_top = top < 0 ? 0 : top;
        L.eps = eps_over_h * bbox_part[r * kBBoxBlocks].hmax;
        lev[r] = L;
        groups += (int64_t)L.nx[L.grp_top] * L.ny[L.grp_top] * L.nz[L.grp_top];
    }
    totals[0] = up;
    totals[1] = 0;       // groups written by k_grav_groups
    totals[2] = groups;  // nodes of the groups' top levels
    if (up > cap_upper) flags[FLAG_GRAV_OVERFLOW] = 1;
}

// Cells of the level-k node (x, y, z) of run g: the Morton keys [kb, kb +
// 2^nb).  Below bit level k every axis that has such a bit varies over the
// node, above it the node's coordinates fix the key, so the range is
// contiguous (an axis with fewer than k bits lies whole in the node).
__device__ __forceinline__ void node_keys(const GridDesc &g, int k, int x, int y, int z,
                                          uint32_t &kb, int &nb) {
    kb = (uint32_t)g.key_off + morton((uint32_t)x << k, (uint32_t)y << k, (uint32_t)z << k,
                                      g.bx, g.by, g.bz);
    nb = (k < g.bx ? k : g.bx) + (k < g.by ? k : g.by) + (k < g.bz ? k : g.bz);
}

// Particles of the level-k node (x, y, z) of run g: one contiguous range.
__device__ __forceinline__ int32_t node_count(const GridDesc &g, const int32_t *cell_start, int k,
                                              int x, int y, int z) {
    uint32_t kb;
    int nb;
    node_keys(g, k, x, y, z, kb, nb);
    return cell_start[kb + (1u << nb)] - cell_start[kb];
}

// Target groups: one thread per top-level node of a run.  A node of at most
// kGroupMax particles (or of level 1, or the single cell of a run of one
// cell) is a group; a fuller one hands over to its non-empty children.
// Groups are appended with one atomic per node (their order does not
// matter: each group's results are its own).
__global__ void k_grav_groups(int nr, const GridDesc *__restrict__ grid,
                              const GravLevels *__restrict__ lev, const int32_t *__restrict__ cell_start,
                              int64_t *totals, int64_t cap_upper, int4 *groups, int64_t cap_groups,
                              int32_t *flags) {
    if (totals[0] > cap_upper) return;  // layout overflow (flagged): nothing is evaluated
    const int64_t nodes = totals[2];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nodes;
         t += (int64_t)gridDim.x * blockDim.x) {
        // run of node t: the runs' top-level node counts in turn
        int r = 0;
        int64_t base = 0;
        for (;; ++r) {
            const GravLevels &L = lev[r];
            const int64_t c = (int64_t)L.nx[L.grp_top] * L.ny[L.grp_top] * L.nz[L.grp_top];
            if (t < base + c || r == nr - 1) break;
            base += c;
        }
        const GravLevels &L = lev[r];
        const GridDesc g = grid[r];
        const int top = L.grp_top;
        const int64_t loc = t - base;
        const int nx = L.nx[top], ny = L.ny[top];
        const int x0 = (int)(loc % nx), y0 = (int)((loc / nx) % ny), z0 = (int)(loc / ((int64_t)nx * ny));
        // the node's groups, visited twice: counted, then written at the
        // place one atomic reserves
        auto visit = [&](auto emit) {
            const int c0 = node_count(g, cell_start, top, x0, y0, z0);
            if (c0 == 0) return;
            if (top <= 1 || c0 <= kGroupMax) {
                emit(top, x0, y0, z0);
                return;
            }
            for (int d = 0; d < 8; ++d) {
                const int x1 = 2 * x0 + (d & 1), y1 = 2 * y0 + ((d >> 1) & 1), z1 = 2 * z0 + (d >> 2);
                if (x1 >= L.nx[top - 1] || y1 >= L.ny[top - 1] || z1 >= L.nz[top - 1]) continue;
                const int c1 = node_count(g, cell_start, top - 1, x1, y1, z1);
                if (c1 == 0) continue;
                if (top - 1 <= 1 || c1 <= kGroupMax) {
                    emit(top - 1, x1, y1, z1);
                    continue;
                }
                for (int e = 0; e < 8; ++e) {
                    const int x2 = 2 * x1 + (e & 1), y2 = 2 * y1 + ((e >> 1) & 1),
                              z2 = 2 * z1 + (e >> 2);
                    if (x2 >= L.nx[top - 2] || y2 >= L.ny[top - 2] || z2 >= L.nz[top - 2]) continue;
                    if (node_count(g, cell_start, top - 2, x2, y2, z2) > 0) emit(top - 2, x2, y2, z2);
                }
            }
        };
        int nout = 0;
        visit([&](int, int, int, int) { ++nout; });
        if (nout == 0) continue;
        const int64_t at = (int64_t)atomicAdd((unsigned long long *)&totals[1],
                                              (unsigned long long)nout);
        if (at + nout > cap_groups) {
            atomicOr(&flags[FLAG_GRAV_OVERFLOW], 1);
            continue;
        }
        int q = 0;
        visit([&](int k, int x, int y, int z) {
            groups[at + q++] = make_int4(r, k, x | (y << 10) | (z << 20), 0);
        });
    }
}

__device__ __forceinline__ int run_of_key(const GridDesc *grid, int nr, int64_t key) {
    int lo = 0, hi = nr;  // grid[lo].key_off <= key
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (grid[mid].key_off <= key) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float4 monopole(double M, double sx, double sy, double sz) {
    return M > 0.0 ? make_float4((float)(sx / M), (float)(sy / M), (float)(sz / M), (float)M)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Cell and octant monopoles: one thread per key of the global cell table.
// The members of a cell are ordered by octant, so each octant is one run of
// consecutive members.
__global__ void k_grav_leaf(int nr, const GridDesc *__restrict__ grid,
                            const int32_t *__restrict__ total_keys,
                            const int32_t *__restrict__ cell_start,
                            const int32_t *__restrict__ cell_count,
                            const uint8_t *__restrict__ octant,
                            const double4 *__restrict__ posh64, const double *__restrict__ m,
                            const int32_t *__restrict__ active, float4 *mom0, float4 *mom8) {
    const int64_t nk = *total_keys;
    for (int64_t key = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; key < nk;
         key += (int64_t)gridDim.x * blockDim.x) {
        const int cnt = cell_count[key];
        for (int o = 0; o < 8; ++o) mom8[key * 8 + o] = make_float4(0.f, 0.f, 0.f, 0.f);
        double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        if (cnt > 0) {
            const GridDesc g = grid[run_of_key(grid, nr, key)];
            const int s = cell_start[key];
            double Mo = 0.0, ox = 0.0, oy = 0.0, oz = 0.0;
            int cur = octant[s];
            for (int k = 0; k < cnt; ++k) {
                const int j = s + k;
                const int o = octant[j];
                if (o != cur) {
                    mom8[key * 8 + cur] = monopole(Mo, ox, oy, oz);
                    Mo = ox = oy = oz = 0.0;
                    cur = o;
                }
                const double mj = (active && !active[j]) ? 0.0 : m[j];
                const double4 p = posh64[j];
                const double px = mj * (p.x - g.ox), py = mj * (p.y - g.oy), pz = mj * (p.z - g.oz);
                Mo += mj;
                ox += px;
                oy += py;
                oz += pz;
                M += mj;
                sx += px;
                sy += py;
                sz += pz;
            }
            mom8[key * 8 + cur] = monopole(Mo, ox, oy, oz);
        }
        mom0[key] = monopole(M, sx, sy, sz);
    }
}

__device__ __forceinline__ float4 node_moment(const GridDesc &g, const GravLevels &L,
                                              const float4 *mom0, const float4 *momU, int k,
                                              int cx, int cy, int cz) {
    if (k == 0)
        return mom0[(uint32_t)g.key_off + morton(cx, cy, cz, g.bx, g.by, g.bz)];
    return momU[L.off[k] + ((int64_t)cz * L.ny[k] + cy) * L.nx[k] + cx];
}

// Level-k monopoles from the eight children at level k-1 (k >= 1).
__global__ void k_grav_up(int nr, int k, const GridDesc *__restrict__ grid,
                          const GravLevels *__restrict__ lev, const int64_t *__restrict__ totals,
                          int64_t cap_upper, const float4 *__restrict__ mom0, float4 *momU) {
    if (totals[0] > cap_upper) return;  // layout overflow (flagged): nothing fits
    for (int r = blockIdx.y; r < nr; r += gridDim.y) {
        const GravLevels &L = lev[r];
        if (k >= L.nlev) continue;
        const GridDesc g = grid[r];
        const int nx = L.nx[k], ny = L.ny[k], nz = L.nz[k];
        const int64_t cells = (int64_t)nx * ny * nz;
        for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < cells;
             c += (int64_t)gridDim.x * blockDim.x) {
            const int cx = (int)(c % nx), cy = (int)((c / nx) % ny), cz = (int)(c / ((int64_t)nx * ny));
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int d = 0; d < 8; ++d) {
                const int x = 2 * cx + (d & 1), y = 2 * cy + ((d >> 1) & 1), z = 2 * cz + (d >> 2);
                if (x >= L.nx[k - 1] || y >= L.ny[k - 1] || z >= L.nz[k - 1]) continue;
                const float4 q = node_moment(g, L, mom0, momU, k - 1, x, y, z);
                M += q.w;
                sx += (double)q.w * q.x;
                sy += (double)q.w * q.y;
                sz += (double)q.w * q.z;
            }
            momU[L.off[k] + c] = M > 0.0 ? make_float4((float)(sx / M), (float)(sy / M),
                                                       (float)(sz / M), (float)M)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// ------------------------------------------------------------ group walk
struct Acc {
    float ax[kSlots], ay[kSlots], az[kSlots], ph[kSlots];
    float tx[kSlots], ty[kSlots], tz[kSlots];
    int32_t ti[kSlots];
};

__global__ __launch_bounds__(64) void k_grav_walk(
    int nr, const GridDesc *__restrict__ grid, const GravLevels *__restrict__ lev,
    const int64_t *__restrict__ totals, int64_t cap_upper, const int4 *__restrict__ groups,
    int64_t cap_groups, const int32_t *__restrict__ cell_start,
    const int32_t *__restrict__ cell_count, const double4 *__restrict__ posh64,
    const uint8_t *__restrict__ octant, const double *__restrict__ m,
    const int32_t *__restrict__ active, const float4 *__restrict__ mom0,
    const float4 *__restrict__ mom8, const float4 *__restrict__ momU, float Gc, float theta,
    int32_t accumulate, double *ax, double *ay, double *az, double *phi, int32_t *flags,
    const int32_t *__restrict__ tmask) {
    __shared__ uint32_t cand[2][kCand];
    __shared__ float4 il[kIL];
    __shared__ float4 stg[kStage];
    __shared__ int32_t stg_j[kStage];
    __shared__ int32_t leaf_s[8], leaf_c[8];
    const int lane = threadIdx.x;
    const int64_t ngroups = totals[0] > cap_upper ? 0 : (totals[1] < cap_groups ? totals[1] : cap_groups);

    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        // ---- the group's run, level gl and node; its particles are one
        // contiguous range of the sorted order
        const int4 gd = groups[grp];
        const int r = gd.x, gl = gd.y;
        const GravLevels &L = lev[r];
        const GridDesc g = grid[r];
        const int gx = gd.z & 1023, gy = (gd.z >> 10) & 1023, gz = (gd.z >> 20) & 1023;
        __syncthreads();
        if (lane < 8) {
            int s = 0, c = 0;
            if (lane == 0) {
                uint32_t kb;
                int nb;
                node_keys(g, gl, gx, gy, gz, kb, nb);
                s = cell_start[kb];
                c = cell_start[kb + (1u << nb)] - s;
            }
            leaf_s[lane] = s;
            leaf_c[lane] = c;
        }
        __syncthreads();
        const int nt = leaf_c[0];
        if (nt == 0) continue;
        const float edge_g = (float)(g.L * (double)(1 << gl));
        const float blo[3] = {gx * edge_g, gy * edge_g, gz * edge_g};
        const float bhi[3] = {blo[0] + edge_g, blo[1] + edge_g, blo[2] + edge_g};
        const float e2 = (float)(L.eps * L.eps);

        for (int t0 = 0; t0 < nt; t0 += kWave * kSlots) {
            // slots holding targets in this pass (wave-uniform): empty slots
            // are skipped by the evaluation loops
            const int ns = (nt - t0 + kWave - 1) / kWave < kSlots ? (nt - t0 + kWave - 1) / kWave
                                                                   : kSlots;
            Acc A;
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                A.ax[s] = A.ay[s] = A.az[s] = A.ph[s] = 0.f;
                A.ti[s] = -1;
                A.tx[s] = A.ty[s] = A.tz[s] = 0.f;
                const int t = t0 + s * kWave + lane;
                if (t < nt) {
                    int q = 0, base = 0;
                    while (t >= base + leaf_c[q]) { base += leaf_c[q]; ++q; }
                    const int i = leaf_s[q] + (t - base);
                    const double4 p = posh64[i];
                    A.ti[s] = i;
                    A.tx[s] = (float)(p.x - g.ox);
                    A.ty[s] = (float)(p.y - g.oy);
                    A.tz[s] = (float)(p.z - g.oz);
                }
            }
            int n_il = 0, n_st = 0;
            // Entries are evaluated kEvalStep at a time: per slot their
            // contributions are independent and are added in list order.
            // Only near-field particles (pp) can be the target itself, whose
            // term is left out; softened 1/r with eps^2 taken first.
            auto rinv = [&](float dx, float dy, float dz) {
                return __frsqrt_rn(fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2))));
            };
            auto eval = [&](auto pp, const float4 *lst, const int32_t *lj, int cnt) {
                constexpr bool PP = decltype(pp)::value;
                int e = 0;
                for (; e + kEvalStep <= cnt; e += kEvalStep) {
                    float4 q[kEvalStep];
                    int j[kEvalStep];
#pragma unroll
                    for (int u = 0; u < kEvalStep; ++u) {
                        q[u] = lst[e + u];
                        j[u] = PP ? lj[e + u] : -1;
                    }
#pragma unroll
                    for (int s = 0; s < kSlots; ++s) {
                        if (s >= ns) break;
                        float dx[kEvalStep], dy[kEvalStep], dz[kEvalStep], mr[kEvalStep],
                            m3[kEvalStep];
#pragma unroll
                        for (int u = 0; u < kEvalStep; ++u) {
                            dx[u] = q[u].x - A.tx[s];
                            dy[u] = q[u].y - A.ty[s];
                            dz[u] = q[u].z - A.tz[s];
                            const float ri = rinv(dx[u], dy[u], dz[u]);
                            mr[u] = (PP && j[u] == A.ti[s]) ? 0.f : q[u].w * ri;
                            m3[u] = mr[u] * ri * ri;
                        }
#pragma unroll
                        for (int u = 0; u < kEvalStep; ++u) {
                            A.ax[s] += m3[u] * dx[u];
                            A.ay[s] += m3[u] * dy[u];
                            A.az[s] += m3[u] * dz[u];
                            A.ph[s] += mr[u];
                        }
                    }
                }
                for (; e < cnt; ++e) {
                    const float4 q = lst[e];
                    const int j = PP ? lj[e] : -1;
#pragma unroll
                    for (int s = 0; s < kSlots; ++s) {
                        if (s >= ns) break;
                        const float dx = q.x - A.tx[s], dy = q.y - A.ty[s], dz = q.z - A.tz[s];
                        const float ri = rinv(dx, dy, dz);
                        const float mr = (PP && j == A.ti[s]) ? 0.f : q.w * ri;
                        const float mr3 = mr * ri * ri;
                        A.ax[s] += mr3 * dx;
                        A.ay[s] += mr3 * dy;
                        A.az[s] += mr3 * dz;
                        A.ph[s] += mr;
                    }
                }
            };
            auto flush_il = [&]() {
                __syncthreads();
                eval(std::false_type{}, il, nullptr, n_il);
                n_il = 0;
                __syncthreads();
            };
            auto flush_st = [&]() {
                __syncthreads();
                eval(std::true_type{}, stg, stg_j, n_st);
                n_st = 0;
                __syncthreads();
            };
            // ---- breadth-first walk from the top level
            const int top = L.nlev - 1;
            int cur = 0, n_cur = 0;
            {
                const int tn = L.nx[top] * L.ny[top] * L.nz[top];  // <= 8
                if (lane < tn) cand[0][lane] = (uint32_t)lane;
                n_cur = tn;
            }
            bool overflow = false;
            // b < theta d with b from the centre of mass to the node's
            // farthest corner and d from it to the group's box; the node's
            // box must be disjoint from the group's
            auto accepts = [&](const float4 &q, float lx, float ly, float lz, float e) -> bool {
                const bool disjoint = lx >= bhi[0] || lx + e <= blo[0] || ly >= bhi[1] ||
                                      ly + e <= blo[1] || lz >= bhi[2] || lz + e <= blo[2];
                const float ex = fmaxf(fmaxf(blo[0] - q.x, q.x - bhi[0]), 0.f);
                const float ey = fmaxf(fmaxf(blo[1] - q.y, q.y - bhi[1]), 0.f);
                const float ez = fmaxf(fmaxf(blo[2] - q.z, q.z - bhi[2]), 0.f);
                const float bx = fmaxf(q.x - lx, lx + e - q.x);
                const float by = fmaxf(q.y - ly, ly + e - q.y);
                const float bz = fmaxf(q.z - lz, lz + e - q.z);
                return disjoint &&
                       bx * bx + by * by + bz * bz < theta * theta * (ex * ex + ey * ey + ez * ez);
            };
            // wave-wide: append the lanes' accepted monopoles to the list
            auto push_il = [&](bool acc, const float4 &q) {
                const uint64_t mk = __builtin_amdgcn_ballot_w64(acc);
                const int cnt = __popcll(mk);
                if (cnt == 0) return;
                if (n_il + cnt > kIL) flush_il();
                if (acc) {
                    const int rk = (int)__builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                    il[n_il + rk] = q;
                }
                n_il += cnt;
            };
            // wave-wide: one search cell per lane (valid lanes): the cell
            // as a monopole, else its octants, else the particles of the
            // octants it cannot accept
            auto handle_cell = [&](bool valid, int cx, int cy, int cz) {
                const float Lc = (float)g.L, half = 0.5f * Lc;
                uint32_t key0 = 0u;
                float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                bool acc = false, open = false;
                if (valid) {
                    key0 = (uint32_t)g.key_off + morton(cx, cy, cz, g.bx, g.by, g.bz);
                    q = mom0[key0];
                    if (q.w > 0.f) {
                        acc = accepts(q, cx * Lc, cy * Lc, cz * Lc, Lc);
                        open = !acc;
                    }
                }
                push_il(acc, q);
                if (!__builtin_amdgcn_ballot_w64(open)) return;
                uint32_t lmask = 0;
                for (int d = 0; d < 8; ++d) {
                    bool acc8 = false;
                    float4 q8 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (open) {
                        q8 = mom8[(size_t)key0 * 8 + d];
                        if (q8.w > 0.f) {
                            acc8 = accepts(q8, (float)(2 * cx + (d & 1)) * half,
                                           (float)(2 * cy + ((d >> 1) & 1)) * half,
                                           (float)(2 * cz + (d >> 2)) * half, half);
                            if (!acc8) lmask |= 1u << d;
                        }
                    }
                    push_il(acc8, q8);
                }
                uint64_t mk = __builtin_amdgcn_ballot_w64(lmask != 0);
                while (mk) {
                    const int src = __builtin_ctzll(mk);
                    mk &= mk - 1;
                    const uint32_t kk = (uint32_t)__shfl((int)key0, src);
                    const uint32_t lm = (uint32_t)__shfl((int)lmask, src);
                    const int s0 = cell_start[kk], cnt = cell_count[kk];
                    for (int b = 0; b < cnt; b += kWave) {
                        const int j = s0 + b + lane;
                        const bool in = b + lane < cnt && ((lm >> octant[j]) & 1u);
                        const uint64_t mj = __builtin_amdgcn_ballot_w64(in);
                        const int take = __popcll(mj);
                        if (take == 0) continue;
                        if (n_st + take > kStage) flush_st();
                        if (in) {
                            const int rk = (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(mj >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mj, 0u));
                            const double4 p = posh64[j];
                            const double mass = (active && !active[j]) ? 0.0 : m[j];
                            stg[n_st + rk] = make_float4((float)(p.x - g.ox), (float)(p.y - g.oy),
                                                         (float)(p.z - g.oz), (float)mass);
                            stg_j[n_st + rk] = j;
                        }
                        n_st += take;
                    }
                }
            };
            // levels top .. 1 breadth first through the candidate lists; the
            // children of opened level-1 nodes (search cells) are handled by
            // the lane that opened them; a run of a single level starts at
            // its cells
            for (int k = top; k >= 0 && !overflow; --k) {
                __syncthreads();
                const int nx = L.nx[k], ny = L.ny[k];
                const float edge = (float)(g.L * (double)(1 << k));
                int n_next = 0;
                for (int c0 = 0; c0 < n_cur; c0 += kWave) {
                    const int c = c0 + lane;
                    int cx = 0, cy = 0, cz = 0;
                    if (c < n_cur) {
                        const uint32_t id = cand[cur][c];
                        cx = (int)(id % (uint32_t)nx);
                        cy = (int)((id / (uint32_t)nx) % (uint32_t)ny);
                        cz = (int)(id / ((uint32_t)nx * (uint32_t)ny));
                    }
                    bool acc_node = false, open = false;
                    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (k > 0) {
                        if (c < n_cur) {
                            q = node_moment(g, L, mom0, momU, k, cx, cy, cz);
                            if (q.w > 0.f) {
                                acc_node = accepts(q, cx * edge, cy * edge, cz * edge, edge);
                                open = !acc_node;
                            }
                        }
                        push_il(acc_node, q);
                    }
                    if (k <= 1) {
                        // cells: the eight children of opened level-1 nodes,
                        // or the candidates themselves at level 0
                        const int cnx = L.nx[0], cny = L.ny[0], cnz = L.nz[0];
                        for (int d = 0; d < (k == 1 ? 8 : 1); ++d) {
                            const int x = k == 1 ? 2 * cx + (d & 1) : cx;
                            const int y = k == 1 ? 2 * cy + ((d >> 1) & 1) : cy;
                            const int z = k == 1 ? 2 * cz + (d >> 2) : cz;
                            const bool v = k == 1 ? open && x < cnx && y < cny && z < cnz
                                                  : c < n_cur;
                            handle_cell(v, x, y, z);
                        }
                        continue;
                    }
                    // children of opened nodes into the next level's list.  When
                    // they would overflow it, the opened nodes disjoint from the
                    // group's box are used as monopoles instead (the far field
                    // then rests on coarser nodes than the opening angle asks
                    // for) and only those overlapping the box are opened
                    {
                        if (n_next + 8 * __popcll(__builtin_amdgcn_ballot_w64(open)) > kCand) {
                            const float x0 = cx * edge, y0 = cy * edge, z0 = cz * edge;
                            const bool disj = x0 >= bhi[0] || x0 + edge <= blo[0] ||
                                              y0 >= bhi[1] || y0 + edge <= blo[1] ||
                                              z0 >= bhi[2] || z0 + edge <= blo[2];
                            push_il(open && disj, q);
                            open = open && !disj;
                        }
                        const uint64_t mk = __builtin_amdgcn_ballot_w64(open);
                        const int cnt = __popcll(mk);
                        if (n_next + 8 * cnt > kCand) {
                            overflow = true;
                        } else if (open) {
                            const int rk = (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                            const int cnx = L.nx[k - 1], cny = L.ny[k - 1], cnz = L.nz[k - 1];
                            for (int d = 0; d < 8; ++d) {
                                const int x = 2 * cx + (d & 1), y = 2 * cy + ((d >> 1) & 1),
                                          z = 2 * cz + (d >> 2);
                                const bool ok = x < cnx && y < cny && z < cnz;
                                cand[cur ^ 1][n_next + 8 * rk + d] =
                                    ok ? (uint32_t)((z * cny + y) * cnx + x) : 0xffffffffu;
                            }
                        }
                        if (!overflow) n_next += 8 * cnt;
                    }
                }
                // drop the out-of-range children appended above
                __syncthreads();
                int kept = 0;
                for (int c0 = 0; c0 < n_next; c0 += kWave) {
                    const int c = c0 + lane;
                    const uint32_t id = c < n_next ? cand[cur ^ 1][c] : 0xffffffffu;
                    const bool ok = id != 0xffffffffu;
                    const uint64_t mk = __builtin_amdgcn_ballot_w64(ok);
                    __syncthreads();
                    if (ok) {
                        const int rk = (int)__builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                        cand[cur ^ 1][kept + rk] = id;
                    }
                    kept += __popcll(mk);
                    __syncthreads();
                }
                cur ^= 1;
                n_cur = kept;
            }
            if (overflow) {
                if (lane == 0) atomicOr(&flags[FLAG_GRAV_OVERFLOW], 1);
                // leave the outputs of this group as NaN so that nothing uses them silently
#pragma unroll
                for (int s = 0; s < kSlots; ++s) A.ax[s] = A.ay[s] = A.az[s] = A.ph[s] = NAN;
                n_il = n_st = 0;
            }
            flush_il();
            flush_st();
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const int i = A.ti[s];
                if (i < 0 || (tmask && !tmask[i])) continue;
                const double fx = (double)Gc * A.ax[s], fy = (double)Gc * A.ay[s],
                             fz = (double)Gc * A.az[s];
                if (accumulate) {
                    ax[i] += fx;
                    ay[i] += fy;
                    az[i] += fz;
                } else {
                    ax[i] = fx;
                    ay[i] = fy;
                    az[i] = fz;
                }
                if (phi) phi[i] = -(double)Gc * A.ph[s];
            }
        }
    }
}

sph_status launch_gravity(Ctx *ctx, int64_t n, const double *m, const int32_t *active, double G,
                          double eps_over_h, double theta, int32_t accumulate, double *ax,
                          double *ay, double *az, double *phi, hipStream_t s,
                          const int32_t *tmask) {
    if (n == 0) return SPH_OK;
    const int nr = ctx->n_runs_built;
    hipLaunchKernelGGL(k_grav_layout, dim3(1), dim3(64), 0, s, nr, ctx->grid, ctx->bbox_part,
                       eps_over_h, (GravLevels *)ctx->grav_lev, ctx->grav_totals, ctx->grav_cap_upper,
                       ctx->flags);
    hipLaunchKernelGGL(k_grav_leaf, dim3(2048), dim3(256), 0, s, nr, ctx->grid, ctx->total_keys,
                       ctx->cell_start, ctx->cell_count, ctx->octant, ctx->posh64, m, active,
                       ctx->grav_mom0, ctx->grav_mom8);
    const int ry = nr < 64 ? nr : 64;
    for (int k = 1; k < kGravLevels; ++k)
        hipLaunchKernelGGL(k_grav_up, dim3(64, ry), dim3(256), 0, s, nr, k, ctx->grid,
                           (const GravLevels *)ctx->grav_lev, ctx->grav_totals,
                           ctx->grav_cap_upper, ctx->grav_mom0, ctx->grav_momU);
    hipLaunchKernelGGL(k_grav_groups, dim3(256), dim3(256), 0, s, nr, ctx->grid,
                       (const GravLevels *)ctx->grav_lev, ctx->cell_start, ctx->grav_totals,
                       ctx->grav_cap_upper, ctx->grav_groups, ctx->grav_cap_groups, ctx->flags);
    hipLaunchKernelGGL(k_grav_walk, dim3(8192), dim3(64), 0, s, nr, ctx->grid,
                       (const GravLevels *)ctx->grav_lev,
                       ctx->grav_totals, ctx->grav_cap_upper, ctx->grav_groups,
                       ctx->grav_cap_groups, ctx->cell_start, ctx->cell_count, ctx->posh64,
                       ctx->octant, m, active, ctx->grav_mom0, ctx->grav_mom8, ctx->grav_momU,
                       (float)G, (float)theta, accumulate, ax, ay,
                       az, phi, ctx->flags, tmask);
    SPH_HIP(hipGetLastError());
    return SPH_OK;
}

size_t gravity_levels_bytes(int32_t max_runs) { return (size_t)max_runs * sizeof(GravLevels); }

}  // namespace sph

// ------------------------------------------------------------ bound mass
namespace sph {

constexpr int kBmBlocks = 64;  // partial sums per run

// Every particle starts bound; the potential starts at zero, so a particle
// the walk does not reach (outside its run's far cube) counts as unbound.
__global__ void k_bm_fill(int64_t n, int32_t *bound, double *phi) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bound[i] = 1;
        phi[i] = 0.0;
    }
}

// Per (run, block) partial sums of m, m v over the bound particles; fixed
// order, so the totals are reproducible.
__global__ void k_bm_partial(const int32_t *__restrict__ run_p, const double *__restrict__ vx,
                             const double *__restrict__ vy, const double *__restrict__ vz,
                             const double *__restrict__ m, const int32_t *__restrict__ bound,
                             double *part) {
    const int r = blockIdx.y;
    const int64_t a = run_p[r], b = run_p[r + 1];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!bound[i]) continue;
        s[0] += m[i];
        s[1] += m[i] * vx[i];
        s[2] += m[i] * vy[i];
        s[3] += m[i] * vz[i];
    }
    __shared__ double sh[4][256];
    for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[((int64_t)r * kBmBlocks + blockIdx.x) * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Run totals: M_r and the centre-of-mass velocity of the bound set.
__global__ void k_bm_total(int nr, const double *__restrict__ part, double *m_bound,
                           double *vcm, int32_t *removed) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < kBmBlocks; ++b)
        for (int c = 0; c < 4; ++c) s[c] += part[((int64_t)r * kBmBlocks + b) * 4 + c];
    m_bound[r] = s[0];
    for (int c = 0; c < 3; ++c) vcm[r * 3 + c] = s[0] > 0.0 ? s[1 + c] / s[0] : 0.0;
    if (r == 0) *removed = 0;
}

// Remove the particles with |v - v_c|^2 / 2 + phi > 0 from the bound set.
__global__ void k_bm_update(const int32_t *__restrict__ run_p, const double *__restrict__ vx,
                            const double *__restrict__ vy, const double *__restrict__ vz,
                            const double *__restrict__ phi, const double *__restrict__ vcm,
                            int32_t *bound, int32_t *removed) {
    const int r = blockIdx.y;
    const int64_t a = run_p[r], b = run_p[r + 1];
    const double cx = vcm[r * 3], cy = vcm[r * 3 + 1], cz = vcm[r * 3 + 2];
    int out = 0;
    for (int64_t i = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!bound[i]) continue;
        const double ux = vx[i] - cx, uy = vy[i] - cy, uz = vz[i] - cz;
        if (0.5 * ((ux * ux + uy * uy) + uz * uz) + phi[i] > 0.0) {
            bound[i] = 0;
            ++out;
        }
    }
    const uint64_t mk = __ballot(out > 0);
    if (mk) {
        int v = out;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x % kWave) == 0) atomicAdd(removed, v);
    }
}

sph_status launch_bound_mass(Ctx *ctx, int64_t n, const double *vx, const double *vy,
                             const double *vz, const double *m, double G, double eps_over_h,
                             double theta, int32_t max_iter, int32_t *bound, double *m_bound,
                             double *phi, double *acc3, int32_t *iterations, hipStream_t s) {
    const int nr = ctx->n_runs_built;
    hipLaunchKernelGGL(k_bm_fill, dim3(1024), dim3(256), 0, s, n, bound, phi);
    int32_t it = 0;
    for (; it < max_iter; ++it) {
        hipLaunchKernelGGL(k_bm_partial, dim3(kBmBlocks, nr), dim3(256), 0, s, ctx->run_p, vx, vy,
                           vz, m, bound, ctx->bm_part);
        hipLaunchKernelGGL(k_bm_total, dim3((nr + 255) / 256), dim3(256), 0, s, nr, ctx->bm_part,
                           m_bound, ctx->bm_vcm, ctx->bm_removed);
        sph_status e = launch_gravity(ctx, n, m, bound, G, eps_over_h, theta, 0, acc3, acc3 + n,
                                      acc3 + 2 * n, phi, s);
        if (e != SPH_OK) return e;
        hipLaunchKernelGGL(k_bm_update, dim3(kBmBlocks, nr), dim3(256), 0, s, ctx->run_p, vx, vy,
                           vz, phi, ctx->bm_vcm, bound, ctx->bm_removed);
        SPH_HIP(hipGetLastError());
        int32_t removed = 0;
        SPH_HIP(hipMemcpyAsync(&removed, ctx->bm_removed, 4, hipMemcpyDeviceToHost, s));
        SPH_HIP(hipStreamSynchronize(s));
        if (removed == 0) break;
    }
    // bound mass of the final set
    hipLaunchKernelGGL(k_bm_partial, dim3(kBmBlocks, nr), dim3(256), 0, s, ctx->run_p, vx, vy, vz,
                       m, bound, ctx->bm_part);
    hipLaunchKernelGGL(k_bm_total, dim3((nr + 255) / 256), dim3(256), 0, s, nr, ctx->bm_part,
                       m_bound, ctx->bm_vcm, ctx->bm_removed);
    SPH_HIP(hipGetLastError());
    if (iterations) *iterations = it;
    return SPH_OK;
}

size_t bound_mass_part_bytes(int32_t max_runs) { return (size_t)max_runs * kBmBlocks * 4 * 8; }

}  // namespace sph
