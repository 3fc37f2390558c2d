// nbr.hip -- neighbour lists inside the list radius R (gfx950).
//
// The list of particle i is { j != i : r_ij^2 < R^2 } with unsoftened FP64
// distances evaluated without FMA as ((dx*dx + dy*dy) + dz*dz): the constant
// neighbour radius of Section 2.3 of Arnold, Baumgardt & Wang (2021), R =
// r_out + r_buff (r_buff = 0: R = r_out); empty lists are legal. One wave per
// group walks only the nodes whose box comes closer than R to the group box
// (box distances never exceed pair
// distances, also after rounding, so no neighbour is missed). The particles
// of those leaves are staged 64 at a time in an LDS tile (FP64 position and
// caller index, loaded lane-parallel) and every lane tests its own particle
// against each tile entry by LDS broadcast. The tree walk (walk.hip) counts
// the neighbours while it evaluates the near pairs and writes them into
// per-particle staging rows; the host library scans the counts into CSR
// offsets. k_nbr_copy then moves the staged rows into the CSR, and
// k_nbr_fill writes the lists of the groups whose rows overflowed, in its own
// deterministic traversal order. Either route yields the set the walk counted.
#include "pbh_internal.hpp"
#include "wave.hpp"

namespace pbh {

namespace {

constexpr int NCAP = 128;   // candidate tile: < 64 left over + 64 new

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
    const int32_t* fill_list;      // the groups whose lists this pass writes
    const double* g_lo;
    const double* g_hi;
    const ClusterParams* cp;
    const unsigned long long* G;   // device-side group count
    const int64_t* off;            // CSR offsets (caller order)
    int32_t* idx;                  // CSR indices
    int64_t cap;
    int32_t* stack;
    int stack_cap;
    unsigned long long* cnt;
    unsigned long long* queues;    // [kQueues] of this pass
    unsigned long long* wave_log;  // per workgroup: groups done, clock ticks
};

struct NTile {
    double x[NCAP], y[NCAP], z[NCAP];
    int orig[NCAP];
    int lf_ex[64];
    int lf_beg[64];
};

__device__ inline void test_tile(const NTile& T, int cnt, double xi, double yi, double zi, int me_orig,
                                 bool active, double rlist2, const NbrParams& p, int64_t wpos,
                                 int& count, bool& overflow) {
#pragma clang fp contract(off)
    for (int e = 0; e < cnt; ++e) {
        const double dx = T.x[e] - xi, dy = T.y[e] - yi, dz = T.z[e] - zi;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const int oj = T.orig[e];
        if (active && r2 < rlist2 && oj != me_orig) {
            const int64_t at = wpos + count;
            if (at < p.cap) p.idx[at] = oj;
            else overflow = true;
            ++count;
        }
    }
}

__global__ __launch_bounds__(64) void k_nbr_fill(NbrParams p) {
    __shared__ NTile T;
    __shared__ int s_stack[kStackLds];
    const int lane = threadIdx.x;
    const Stack stack{s_stack, p.stack + (int64_t)blockIdx.x * (p.stack_cap - kStackLds), p.stack_cap,
                      kStackLds};
    const int64_t G = (int64_t)*p.G;
    int home = blockIdx.x % kQueues;
    const unsigned long long t_start = wall_clock64();
    int n_done = 0;
    for (;;) {
        const int64_t q = queue_next(p.queues, G, home, lane);
        if (q < 0) break;
        ++n_done;
        const int64_t g = uni(p.fill_list[q]);
        const int gb = uni(p.g_begin[g]), gcnt = uni(p.g_count[g]), root = uni(p.g_root[g]);
        const double rlist2 = p.cp[uni(p.g_cluster[g])].rlist2;   // list radius R^2
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
        if (active) wpos = p.off[orig];
        int count = 0;
        bool overflow = false;
        if (rlist2 > 0.0) {
            stack.put(0, root);
            int top = 1;
            int fill = 0;
            while (top > 0) {
                __threadfence_block();
                const int npop = uni(top < 64 ? top : 64);
                top -= npop;
                const bool has = lane < npop;
                const int nd = has ? stack.get(top + lane) : root;
                __threadfence_block();
                const WNode w = p.node[nd];
                const bool near = has && box_box_d2(glo, ghi, w.lo, w.hi) < rlist2;
                const bool leaf = w.nchild == 0;
                const int nch = (near && !leaf) ? w.nchild : 0;
                const int incl = wave_incl_scan(nch, lane);
                const int tot = last_lane(incl);
                if (top + tot > p.stack_cap) {
                    overflow = true;
                    break;
                }
                for (int k = 0; k < nch; ++k) stack.put(top + incl - nch + k, w.first_child + k);
                top = uni(top + tot);
                // particles of near leaves into the candidate tile
                const bool flag = near && leaf;
                if (!__ballot(flag)) continue;
                const int v = flag ? w.count : 0;
                const int li = wave_incl_scan(v, lane);
                const int total = last_lane(li);
                __syncthreads();
                T.lf_ex[lane] = li - v;
                T.lf_beg[lane] = w.begin;
                __syncthreads();
                for (int base = 0; base < total; base += 64) {
                    const int s = base + lane;
                    int k = 0;
#pragma unroll
                    for (int st = 32; st > 0; st >>= 1)
                        if (T.lf_ex[k + st] <= s) k += st;
                    const int j = T.lf_beg[k] + (s - T.lf_ex[k]);
                    if (s < total) {
                        T.x[fill + lane] = p.x[j];
                        T.y[fill + lane] = p.y[j];
                        T.z[fill + lane] = p.z[j];
                        T.orig[fill + lane] = p.perm[j];
                    }
                    fill = uni(fill + ((total - base) < 64 ? (total - base) : 64));
                    if (fill >= 64) {
                        __syncthreads();
                        test_tile(T, fill, xi, yi, zi, orig, active, rlist2, p, wpos, count, overflow);
                        fill = 0;
                        __syncthreads();
                    }
                }
                __syncthreads();
            }
            __syncthreads();
            if (fill) test_tile(T, fill, xi, yi, zi, orig, active, rlist2, p, wpos, count, overflow);
            __syncthreads();
        }
        const uint64_t ov = __ballot(overflow);
        if (ov) atomicOr(&p.cnt[kErr], lane == 0 ? kErrNbrOverflow : 0ull);
    }
    if (p.wave_log) {
        p.wave_log[2 * blockIdx.x] = (unsigned long long)n_done;
        p.wave_log[2 * blockIdx.x + 1] = wall_clock64() - t_start;
    }
}

// Staged lists into the CSR. One wave per block of 64 consecutive sorted
// particles (the interleaving unit of the staging rows); stage_k[p] = 1 if
// the walk staged the list of p (0: the fill pass writes it). The block's
// lists pass through an LDS tile of 64 entries per particle: entry t of all
// 64 particles is one 256-byte load, and each store instruction writes 64
// consecutive CSR entries of one particle (lists in caller order lie
// scattered over the CSR; one lane per list would write 64 unrelated lines
// per instruction). Entries beyond the caller's capacity are dropped and
// flagged.
constexpr int kCopyTile = 64;   // 16 KB of LDS per block; 16, 32, 96 and 128 were slower at 2^20

__global__ __launch_bounds__(64) void k_nbr_copy(int64_t n, const int8_t* __restrict__ stage_k,
                                                 const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ stage, int scap,
                                                 const int64_t* __restrict__ off,
                                                 int32_t* __restrict__ idx, int64_t cap,
                                                 unsigned long long* __restrict__ cnt) {
    __shared__ int s_tile[kStageStride][kCopyTile + 1];
    __shared__ int s_cnt[kStageStride];
    __shared__ int64_t s_off[kStageStride];
    const int lane = threadIdx.x;
    const int64_t nblk = (n + kStageStride - 1) / kStageStride;
    bool overflow = false;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t i = blk * kStageStride + lane;
        const bool staged = i < n && stage_k[i] != 0;
        int c = 0;
        int64_t at = 0;
        if (staged) {
            const int orig = perm[i];
            at = off[orig];
            c = (int)(off[orig + 1] - at);
        }
        const int32_t* row = stage + stage_index(i, 0, scap);   // inside the buffer for every lane
        int maxc = c;
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(maxc, o, 64);
            maxc = v > maxc ? v : maxc;
        }
        maxc = __builtin_amdgcn_readfirstlane(maxc);
        __syncthreads();
        s_cnt[lane] = c;
        s_off[lane] = at;
        for (int t0 = 0; t0 < maxc; t0 += kCopyTile) {
            __syncthreads();
            // unconditional loads (index clamped into the row) so that all of
            // them are in flight together; unused tile entries are never read
#pragma unroll
            for (int u = 0; u < kCopyTile; ++u) {
                const int t = t0 + u < c ? t0 + u : 0;
                s_tile[lane][u] = row[(int64_t)t * kStageStride];
            }
            __syncthreads();
#pragma unroll 4
            for (int q = 0; q < kStageStride * kCopyTile / 64; ++q) {
                const int slot = q * 64 + lane;
                const int pp = slot / kCopyTile, u = slot % kCopyTile;
                if (t0 + u < s_cnt[pp]) {
                    const int64_t dst = s_off[pp] + t0 + u;
                    if (dst < cap) idx[dst] = s_tile[pp][u];
                    else overflow = true;
                }
            }
        }
    }
    const uint64_t ov = __ballot(overflow);
    if (ov) atomicOr(&cnt[kErr], lane == 0 ? kErrNbrOverflow : 0ull);
}

NbrParams make_params(Dev& d, const BuildCfg& c, int stack_cap) {
    NbrParams p;
    p.node = d.node;
    p.x = d.x; p.y = d.y; p.z = d.z;
    p.perm = d.perm;
    p.g_begin = d.g.begin; p.g_count = d.g.count; p.g_root = d.g.root; p.g_cluster = d.g.cluster;
    p.fill_list = d.fill_list;
    p.g_lo = d.g.lo; p.g_hi = d.g.hi;
    p.cp = d.cparams;
    p.G = d.cnt + kCntFill;
    p.off = nullptr;
    p.idx = nullptr;
    p.cap = 0;
    p.stack = d.stack;
    p.stack_cap = stack_cap;
    p.cnt = d.cnt;
    p.queues = d.queues + kQueues;
    p.wave_log = d.wave_log_nbr;
    (void)c;
    return p;
}

}  // namespace

void launch_nbr_copy(Dev& d, const BuildCfg& c, int stage_cap, const int64_t* off, int32_t* idx,
                     int64_t cap, hipStream_t s) {
    int64_t grid = (c.n + kStageStride - 1) / kStageStride;
    if (grid > 16384) grid = 16384;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_nbr_copy, dim3((unsigned)grid), dim3(64), 0, s, c.n, (const int8_t*)d.stage_k,
                       (const int32_t*)d.perm, (const int32_t*)d.nbr_stage, stage_cap, off, idx, cap,
                       d.cnt);
}

void launch_nbr_fill(Dev& d, const BuildCfg& c, int grid, int stack_cap, const int64_t* off,
                     int32_t* idx, int64_t cap, hipStream_t s) {
    NbrParams p = make_params(d, c, stack_cap);
    p.off = off;
    p.idx = idx;
    p.cap = cap;
    p.queues = d.queues + 2 * kQueues;
    hipLaunchKernelGGL(k_nbr_fill, dim3(grid), dim3(64), 0, s, p);
}

}  // namespace pbh
