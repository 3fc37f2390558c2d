// nbr.hip -- neighbour lists inside r_out (gfx950).
//
// The list of particle i is { j != i : r_ij^2 < r_out^2 } with unsoftened
// FP64 distances evaluated without FMA as ((dx*dx + dy*dy) + dz*dz), the
// constant neighbour radius of Section 2.3 of Arnold, Baumgardt & Wang (2021);
// empty lists are legal. One wave per group walks only the nodes whose box
// comes closer than r_out to the group box (box distances never exceed pair
// distances, also after rounding, so no neighbour is missed). Two passes with
// the same deterministic order: counts (in caller order, scanned on the host
// side of the library into CSR offsets), then indices.
#include "pbh_internal.hpp"

namespace pbh {

namespace {

struct NbrParams {
    const WNode* node;
    const double* x;
    const double* y;
    const double* z;
    const int32_t* perm;
    const int32_t* g_begin;
    const int32_t* g_count;
    const int32_t* g_root;
    const int32_t* g_cluster;
    const double* g_lo;
    const double* g_hi;
    const ClusterParams* cp;
    const unsigned long long* G;   // device-side group count
    int32_t* counts;        // count pass: per caller index
    const int64_t* off;     // fill pass: CSR offsets (caller order)
    int32_t* idx;           // fill pass
    int64_t cap;
    int32_t* stack;
    int stack_cap;
    unsigned long long* cnt;
    int queue;
    unsigned long long* wave_log;   // per workgroup: groups done, clock ticks (count pass)
};

// Wave-uniform helpers (see walk.hip): scalar copies of wave-uniform values
// and a branch-free work-queue fetch.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline int wave_next(unsigned long long* ctr, int lane) {
    const unsigned long long r = atomicAdd(ctr, lane == 0 ? 1ull : 0ull);
    return uni((int)r);
}

__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline double box_box_d2(const double* glo, const double* ghi, const double* lo,
                                    const double* hi) {
#pragma clang fp contract(off)
    double g[3];
    for (int k = 0; k < 3; ++k) {
        const double a = lo[k] - ghi[k];
        const double b = glo[k] - hi[k];
        const double v = a > b ? a : b;
        g[k] = v > 0.0 ? v : 0.0;
    }
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
}

__device__ inline bool within(double xi, double yi, double zi, double xj, double yj, double zj,
                              double rout2) {
#pragma clang fp contract(off)
    const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    const double r2 = dx * dx + dy * dy + dz * dz;
    return r2 < rout2;
}

template <bool FILL>
__global__ __launch_bounds__(64) void k_nbr(NbrParams p) {
    const int lane = threadIdx.x;
    int32_t* stack = p.stack + (int64_t)blockIdx.x * p.stack_cap;
    const int64_t G = (int64_t)*p.G;
    const unsigned long long t_start = wall_clock64();
    int n_done = 0;
    for (;;) {
        const int g = wave_next(&p.cnt[p.queue], lane);
        if (g >= G) break;
        ++n_done;
        const int gb = uni(p.g_begin[g]), gcnt = uni(p.g_count[g]), root = uni(p.g_root[g]);
        const double rout2 = p.cp[p.g_cluster[g]].rout2;
        double glo[3], ghi[3];
        for (int k = 0; k < 3; ++k) {
            glo[k] = p.g_lo[3 * g + k];
            ghi[k] = p.g_hi[3 * g + k];
        }
        const bool active = lane < gcnt;
        const int me = gb + (active ? lane : 0);
        const double xi = p.x[me], yi = p.y[me], zi = p.z[me];
        const int orig = p.perm[me];
        int64_t wpos = 0;
        if (FILL && active) wpos = p.off[orig];
        int count = 0;
        bool overflow = false;
        if (rout2 > 0.0) {
            stack[0] = root;   // every lane stores the same value
            int top = 1;
            while (top > 0) {
                __threadfence_block();
                const int npop = uni(top < 64 ? top : 64);
                top -= npop;
                const bool has = lane < npop;
                const int nd = has ? stack[top + lane] : root;
                const WNode w = p.node[nd];
                const bool near = has && box_box_d2(glo, ghi, w.lo, w.hi) < rout2;
                const bool leaf = w.nchild == 0;
                const int nch = (near && !leaf) ? w.nchild : 0;
                const int incl = wave_incl_scan(nch, lane);
                const int tot = uni(__shfl(incl, 63, 64));
                if (top + tot > p.stack_cap) {
                    overflow = true;
                    break;
                }
                for (int k = 0; k < nch; ++k) stack[top + incl - nch + k] = w.first_child + k;
                top = uni(top + tot);
                uint64_t lm = __ballot(near && leaf);
                while (lm) {
                    const int k = __ffsll((long long)lm) - 1;
                    lm &= lm - 1;
                    const int lb = uni(__shfl(w.begin, k, 64));
                    const int lc = uni(__shfl(w.count, k, 64));
                    for (int j = lb; j < lb + lc; ++j) {
                        const bool hit = active && j != me &&
                                         within(xi, yi, zi, p.x[j], p.y[j], p.z[j], rout2);
                        if (hit) {
                            if (FILL) {
                                const int64_t at = wpos + count;
                                if (at < p.cap) p.idx[at] = p.perm[j];
                                else overflow = true;
                            }
                            ++count;
                        }
                    }
                }
            }
        }
        if (!FILL && active) p.counts[orig] = count;
        const uint64_t ov = __ballot(overflow);
        if (ov) atomicOr(&p.cnt[kErr], lane == 0 ? (FILL ? kErrNbrOverflow : kErrNbrStack) : 0ull);
    }
    if (!FILL && p.wave_log) {
        p.wave_log[2 * blockIdx.x] = (unsigned long long)n_done;
        p.wave_log[2 * blockIdx.x + 1] = wall_clock64() - t_start;
    }
}

NbrParams make_params(Dev& d, const BuildCfg& c, int stack_cap) {
    NbrParams p;
    p.node = d.node;
    p.x = d.x; p.y = d.y; p.z = d.z;
    p.perm = d.perm;
    p.g_begin = d.g.begin; p.g_count = d.g.count; p.g_root = d.g.root; p.g_cluster = d.g.cluster;
    p.g_lo = d.g.lo; p.g_hi = d.g.hi;
    p.cp = d.cparams;
    p.G = d.cnt + kCntGroups;
    p.counts = d.nbr_cnt;
    p.off = nullptr;
    p.idx = nullptr;
    p.cap = 0;
    p.stack = d.stack;
    p.stack_cap = stack_cap;
    p.cnt = d.cnt;
    p.queue = kQueueNbrCount;
    p.wave_log = d.wave_log_nbr;
    return p;
}

}  // namespace

void launch_nbr_count(Dev& d, const BuildCfg& c, int grid, int stack_cap, hipStream_t s) {
    NbrParams p = make_params(d, c, stack_cap);
    hipLaunchKernelGGL(k_nbr<false>, dim3(grid), dim3(64), 0, s, p);
}

void launch_nbr_fill(Dev& d, const BuildCfg& c, int grid, int stack_cap, const int64_t* off,
                     int32_t* idx, int64_t cap, hipStream_t s) {
    NbrParams p = make_params(d, c, stack_cap);
    p.off = off;
    p.idx = idx;
    p.cap = cap;
    p.queue = kQueueNbrFill;
    hipLaunchKernelGGL(k_nbr<true>, dim3(grid), dim3(64), 0, s, p);
}

}  // namespace pbh
