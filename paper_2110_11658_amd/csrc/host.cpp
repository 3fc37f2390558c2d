// host.cpp -- the C ABI of libpbh (declared in include/pbh.h).
//
// Owns the device buffers of a context, validates arguments, computes the
// per-cluster changeover constants, and enqueues the kernels of build.hip,
// sort.hip, walk.hip, nbr.hip and kdk.hip on the caller's stream. Every
// numerical step runs on the GPU; the host only marshals sizes and constants.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pbh.h"
#include "pbh_internal.hpp"

using namespace pbh;

namespace {

constexpr int kBoxChunk = 2048;      // particles per bbox/key block (512 blocks per 2^20)
constexpr int kStackCap = 16384;     // traversal stack entries per persistent wave (LDS + spill)
constexpr int kCntKdkStep = 11;      // counter slot: KDK energy output index
constexpr int64_t kIrrPackRatio = 32;  // target lists of >= n/32 use the key-order records

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Layout of the scratch of pbh_irregular_noalloc: the flag word, then the key
// ranks (int32) and the key-order records of at most PBH_NOALLOC_MAX_N
// particles, each part on a 256-byte boundary.
constexpr size_t kNaRankOff = 256;
constexpr size_t kNaRecOff = kNaRankOff + ((sizeof(int32_t) * (size_t)PBH_NOALLOC_MAX_N + 255) / 256) * 256;
constexpr size_t kNaBytes = kNaRecOff + sizeof(IrrRec) * (size_t)PBH_NOALLOC_MAX_N;
constexpr int kNaMaxDevices = 64;

}  // namespace

// The scratch of pbh_irregular_noalloc. Each device holds its own copy while
// the library is loaded; host code reaches it only through the address that
// hipGetSymbolAddress returned for that device (na_scratch_ptr), never by this
// name, which on the host is a stand-in and not a device address.
static __device__ __align__(256) unsigned long long scratch[kNaBytes / sizeof(unsigned long long)];

namespace {

std::mutex na_mu;
void* na_scratch_ptr[kNaMaxDevices] = {};

// Once per device, with that device current: the device address of scratch.
bool na_scratch_setup(int device) {
    if (device < 0 || device >= kNaMaxDevices) return false;
    std::lock_guard<std::mutex> lock(na_mu);
    if (na_scratch_ptr[device]) return true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return false;
    }
    na_scratch_ptr[device] = ptr;
    return true;
}

void* na_scratch(int device) {
    if (device < 0 || device >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(na_mu);
    return na_scratch_ptr[device];
}

}  // namespace

struct pbh_ctx {
    int device = 0;
    pbh_params params{8, 0, 64, 0, 0, PBH_MIXED};
    std::string err;
    hipStream_t last = nullptr;
    hipStream_t cap_stream = nullptr;
    int cus = 0;

    // build state
    bool built = false;
    bool irr_rank_ok = false;   // d.irr_rank holds the inverse of the current build's permutation
    bool batched = false;
    const double* built_pos = nullptr;    // the caller's arrays of the last build
    const double* built_mass = nullptr;
    BuildCfg cfg;
    Dev d;
    std::vector<Buf> bufs;
    std::vector<int64_t> cl_off_h;
    int nblk_box = 0;
    // cluster offsets and buffer generation of the block tables now on the device
    std::vector<int64_t> tab_off;
    int64_t tab_gen = -1;
    // grid of the last walk launch (its per-workgroup clock record), 0 before any
    int64_t last_walk_grid = 0;
    // allocation sizes
    int64_t a_n = -1, a_cap = -1, a_G = -1, a_C = -1, a_nblk = -1, a_stack = -1;
    int64_t alloc_gen = 0;   // bumped whenever device buffers are reallocated
    int grid_mixed = 0, grid_fp64 = 0;   // persistent walk grids at the default tile (the largest)
    int grid_tile[2][3] = {{0, 0, 0}, {0, 0, 0}};   // [mixed][tile 64, 96, 128]

    // kdk
    double* k_acc = nullptr;
    double* k_pot = nullptr;
    double* k_epart = nullptr;
    int k_nblk = 0;
    int64_t k_n = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // the build's kernel sequence, captured once per (buffers, sizes, parameters)
    std::vector<int32_t> lvl_count;   // nodes per level of the last build (moment grids)
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    std::vector<double> bkey;
    std::vector<double> gkey;   // parameters the captured graph was made with

    // irregular-force calls: device flag word of the last call (kIrr* bits)
    unsigned long long* irr_err = nullptr;

    // Hermite / P3T state, kept apart from the build buffers (a rebuild inside
    // the P3T loop must not free it)
    struct {
        int64_t n = -1;
        int64_t last_n = 0;   // particles of the last integration
        double *a = nullptr, *j = nullptr, *xp = nullptr, *vp = nullptr;
        int64_t *tau = nullptr, *dt = nullptr, *dt0 = nullptr;
        int32_t* act = nullptr;
        unsigned long long* ctl = nullptr;
        unsigned long long* lev = nullptr;
        int32_t* bucket = nullptr;
        uint32_t* slot = nullptr;
        double *fr = nullptr, *potr = nullptr, *poti = nullptr, *pott = nullptr, *scr = nullptr,
               *epart = nullptr;
        int64_t* off = nullptr;
        int32_t* idx = nullptr;
        int64_t cap = 0;
        std::vector<void*> mem;
        // one batch of blocks, captured once per set of buffers and parameters
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        std::vector<double> gkey;
        unsigned long long* done = nullptr;   // host-coherent pinned: every particle at the end
        hipEvent_t ev[2] = {nullptr, nullptr};
    } herm;

    // phase timing: events 0/1 build, 2/3 walk, 4/5 neighbours
    bool timing = false;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ev_build = false, ev_walk = false, ev_nbr = false;
};

namespace {

pbh_status fail(pbh_ctx* c, pbh_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, PBH_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void free_all(pbh_ctx* ctx) {
    for (auto& b : ctx->bufs)
        if (b.p) (void)hipFree(b.p);
    ctx->bufs.clear();
    ctx->d = Dev();
    ctx->a_n = ctx->a_cap = ctx->a_G = ctx->a_C = ctx->a_nblk = ctx->a_stack = -1;
    ctx->last_walk_grid = 0;
}

template <typename T>
bool dalloc(pbh_ctx* ctx, T** p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return false;
    ctx->bufs.push_back({q, bytes});
    *p = (T*)q;
    return true;
}

int cluster_bits(int32_t C) {
    int b = 0;
    while ((1ll << b) < C) ++b;
    return b;
}

int64_t node_capacity(int64_t n, int D, int n_leaf, int C) {
    // leaves <= n, branching inner nodes < leaves, single-child inner nodes
    // <= one per (n_leaf+1) particles per level
    return 2 * n + (int64_t)D * ((n + n_leaf) / (n_leaf + 1)) + C + 64;
}

// persistent walk grid for the context's precision and tile: resident
// workgroups per compute unit (LDS and registers) times the compute units
int walk_grid(pbh_ctx* ctx, int mixed) {
    const int tile = ctx->params.walk_tile;
    const int t = tile == 128 ? 2 : (tile == 96 ? 1 : 0);
    int& g = ctx->grid_tile[mixed ? 1 : 0][t];
    if (g == 0) g = walk_blocks_per_cu(mixed, tile) * ctx->cus;
    const int gmax = mixed ? ctx->grid_mixed : ctx->grid_fp64;   // the stacks are sized for this
    return g < gmax ? g : gmax;
}

pbh_status ensure_buffers(pbh_ctx* ctx) {
    const BuildCfg& c = ctx->cfg;
    const int64_t n = c.n, cap = c.node_cap, G = c.n_groups, C = c.n_clusters;
    const int64_t nblk = ctx->nblk_box;
    const int64_t stack = (int64_t)std::max(ctx->grid_mixed, ctx->grid_fp64) * kStackCap;
    if (n <= ctx->a_n && cap <= ctx->a_cap && G <= ctx->a_G && C <= ctx->a_C &&
        nblk <= ctx->a_nblk && stack <= ctx->a_stack)
        return PBH_OK;
    free_all(ctx);
    Dev& d = ctx->d;
    const int64_t big = std::max(n, cap);
    const int64_t scan_len = scan_tmp_need(std::max(big, radix_hist_need(big)) + 1);
    bool ok = dalloc(ctx, &d.x, n) && dalloc(ctx, &d.y, n) && dalloc(ctx, &d.z, n) &&
              dalloc(ctx, &d.m, n) && dalloc(ctx, &d.perm, n) && dalloc(ctx, &d.keys, n) &&
              dalloc(ctx, &d.keys_alt, n) && dalloc(ctx, &d.vals_alt, big) &&
              dalloc(ctx, &d.cl_off, C + 1) && dalloc(ctx, &d.cl_box, 6 * C) &&
              dalloc(ctx, &d.blk_cluster, nblk + C + 1) && dalloc(ctx, &d.blk_range, 2 * nblk) &&
              dalloc(ctx, &d.blk_part, 6 * nblk) && dalloc(ctx, &d.blk_bad, nblk) &&
              dalloc(ctx, &d.cparams, C) && dalloc(ctx, &d.p_first, n) &&
              dalloc(ctx, &d.p_nn, n + 1) && dalloc(ctx, &d.pre_begin, cap) &&
              dalloc(ctx, &d.pre_count, cap) && dalloc(ctx, &d.pre_level, cap) &&
              dalloc(ctx, &d.pre_nchild, cap) && dalloc(ctx, &d.lvl_key, cap) &&
              dalloc(ctx, &d.lvl_key_alt, cap) && dalloc(ctx, &d.lvl_val, cap) &&
              dalloc(ctx, &d.bfs2pre, cap) && dalloc(ctx, &d.pre2bfs, cap) &&
              dalloc(ctx, &d.lvl_off, 32) && dalloc(ctx, &d.node, cap) &&
              dalloc(ctx, &d.q64, cap) && dalloc(ctx, &d.q32, cap) &&
              dalloc(ctx, &d.g_flag, n + 1) && dalloc(ctx, &d.g_len, n) &&
              dalloc(ctx, &d.g_hist, (int64_t)128 * C * group_hist_reps((int)C)) && dalloc(ctx, &d.cl_S, C) &&
              dalloc(ctx, &d.g.begin, G) && dalloc(ctx, &d.g.count, G) &&
              dalloc(ctx, &d.g.root, G) && dalloc(ctx, &d.g.cluster, G) &&
              dalloc(ctx, &d.g.lo, 3 * G) && dalloc(ctx, &d.g.hi, 3 * G) && dalloc(ctx, &d.fill_list, G) &&
              dalloc(ctx, &d.stage_k, n) &&
              dalloc(ctx, &d.scan_tmp, scan_len) &&
              dalloc(ctx, &d.rs_hist, radix_hist_need(big) + 1) && dalloc(ctx, &d.nbr_cnt, n) &&
              dalloc(ctx, &d.stack, stack) && dalloc(ctx, &d.cnt, kNumCounters) &&
              dalloc(ctx, &d.queues, 32) &&
              dalloc(ctx, &d.wave_log, 2 * (stack / kStackCap)) &&
              dalloc(ctx, &d.wave_log_nbr, 2 * (stack / kStackCap)) &&
              dalloc(ctx, &d.wave_cyc, stack / kStackCap);
    if (!ok) {
        free_all(ctx);
        return fail(ctx, PBH_E_OOM, "device allocation failed");
    }
    d.scan_tmp_len = scan_len;
    d.stack_len = stack;
    ++ctx->alloc_gen;
    ctx->a_n = n; ctx->a_cap = cap; ctx->a_G = G; ctx->a_C = C; ctx->a_nblk = nblk;
    ctx->a_stack = stack;
    return PBH_OK;
}

// Neighbour staging rows: `cap` entries per particle, within a fixed memory
// budget (a particle of a Plummer core holds about 5.4x the mean count; 512
// covers a mean of 64). Returns the row size in use, 0 when staging is off
// (too little memory: every list then goes through the fill pass).
constexpr int64_t kStageBudgetBytes = 8ll << 30;
constexpr int kStageMaxCap = 512;
constexpr int kStageMinCap = 32;

int ensure_stage(pbh_ctx* ctx) {
    Dev& d = ctx->d;
    const int64_t n = std::max<int64_t>(ctx->cfg.n, 1);
    int64_t cap = kStageBudgetBytes / (4 * n);
    if (cap > kStageMaxCap) cap = kStageMaxCap;
    cap &= ~(int64_t)31;
    if (cap < kStageMinCap) return 0;
    const int64_t need = ((n + kStageStride - 1) / kStageStride) * kStageStride * cap;
    if (d.nbr_stage && d.nbr_stage_len >= need) return (int)cap;
    if (d.nbr_stage) {
        for (size_t k = 0; k < ctx->bufs.size(); ++k)
            if (ctx->bufs[k].p == d.nbr_stage) {
                (void)hipFree(ctx->bufs[k].p);
                ctx->bufs.erase(ctx->bufs.begin() + (int64_t)k);
                break;
            }
        d.nbr_stage = nullptr;
        d.nbr_stage_len = 0;
    }
    if (!dalloc(ctx, &d.nbr_stage, need)) {
        (void)hipGetLastError();   // a failed allocation is not a launch error
        d.nbr_stage = nullptr;
        return 0;
    }
    d.nbr_stage_len = need;
    return (int)cap;
}

// Host part of a build: sizes, tables, uploads. No kernel runs here.
pbh_status setup_build(pbh_ctx* ctx, int64_t n, int32_t C, const int64_t* offsets, hipStream_t s) {
    BuildCfg& c = ctx->cfg;
    c.n = n;
    c.n_clusters = C;
    c.cbits = cluster_bits(C);
    int D = (63 - c.cbits) / 3;
    if (D > 21) D = 21;
    if (ctx->params.key_bits > 0 && ctx->params.key_bits < D) D = ctx->params.key_bits;
    c.D = D;
    c.n_leaf = ctx->params.leaf_size;
    // n_crit 0: 32 below 2^18 particles (more, smaller groups keep all CUs busy), else 64
    c.n_crit = ctx->params.n_crit ? ctx->params.n_crit : (n < (1 << 18) ? 32 : 64);
    c.node_cap = node_capacity(n, D, c.n_leaf, C);
    for (int l = 0; l < 32; ++l) {
        c.mom_grid[l] = 0;
        if (l < (int)ctx->lvl_count.size()) {
            // power-of-two bucket of 1.5x the last count (few distinct graphs)
            const int64_t want = (ctx->lvl_count[l] * 3 / 2 + kMomT - 1) / kMomT;
            int g = 1;
            while (g < want && g < 2048) g <<= 1;
            c.mom_grid[l] = g;
        }
    }
    c.mom_hi = D;
    c.mom_lo = -1;
    if (!ctx->lvl_count.empty()) {
        // deepest level that held nodes, and the top levels that held few
        int hi = 0;
        for (int l = 0; l < (int)ctx->lvl_count.size() && l <= D; ++l)
            if (ctx->lvl_count[l] > 0) hi = l;
        int lo = -1;
        while (lo + 1 <= hi && ctx->lvl_count[lo + 1] <= 128) ++lo;   // one node per thread
        if (lo >= hi) lo = hi - 1;   // at least the deepest non-empty level runs on its own
        c.mom_hi = hi;
        c.mom_lo = lo;
    }
    if (c.node_cap >= (1ll << 31)) return fail(ctx, PBH_E_ARG, "too many particles for int32 node indices");
    ctx->cl_off_h.assign(offsets, offsets + C + 1);
    std::vector<int32_t> blk_cluster;
    std::vector<int64_t> blk_range;
    std::vector<int32_t> cblk(C + 1, 0);
    for (int k = 0; k < C; ++k) {
        const int64_t a = offsets[k], b = offsets[k + 1];
        cblk[k] = (int32_t)blk_cluster.size();
        for (int64_t q = a; q < b; q += kBoxChunk) {
            blk_cluster.push_back(k);
            blk_range.push_back(q);
            blk_range.push_back(std::min(b, q + kBoxChunk));
        }
    }
    cblk[C] = (int32_t)blk_cluster.size();
    c.n_groups = n;   // capacity; the walk reads the actual count on the device
    ctx->nblk_box = (int)blk_cluster.size();
    if (ctx->grid_mixed == 0) {
        ctx->grid_mixed = walk_blocks_per_cu(1, 64) * ctx->cus;
        ctx->grid_fp64 = walk_blocks_per_cu(0, 64) * ctx->cus;
    }
    pbh_status st = ensure_buffers(ctx);
    if (st != PBH_OK) return st;
    // the tables on the device still hold these offsets: nothing to upload or wait for
    if (ctx->tab_gen == ctx->alloc_gen && ctx->tab_off == ctx->cl_off_h) return PBH_OK;
    ctx->tab_gen = -1;
    // block table: cluster of each block, then per-cluster block offsets
    std::vector<int32_t> tab(blk_cluster);
    tab.insert(tab.end(), cblk.begin(), cblk.end());
    HIP_TRY(hipMemcpyAsync(ctx->d.blk_cluster, tab.data(), tab.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->d.blk_range, blk_range.data(), blk_range.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ctx->d.cl_off, ctx->cl_off_h.data(), (C + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));   // the host tables above are temporaries
    ctx->tab_off = ctx->cl_off_h;
    ctx->tab_gen = ctx->alloc_gen;
    return PBH_OK;
}

void enqueue_build(pbh_ctx* ctx, const double* pos, const double* mass, hipStream_t s);

// The build issues about 90 small kernels; launched one by one, the host's
// launch rate rather than the GPU sets the build time. The sequence is captured
// into a graph once per set of buffers, sizes and parameters (the block tables
// it reads are uploaded before each launch) and replayed.
pbh_status launch_build(pbh_ctx* ctx, const double* pos, const double* mass, hipStream_t s) {
    ctx->irr_rank_ok = false;   // a new permutation
    const BuildCfg& c = ctx->cfg;
    const std::vector<double> key = {(double)(uintptr_t)pos, (double)(uintptr_t)mass, (double)c.n,
                                     (double)c.n_clusters, (double)c.D, (double)c.cbits,
                                     (double)c.n_leaf, (double)c.n_crit, (double)c.node_cap,
                                     (double)ctx->nblk_box, (double)ctx->alloc_gen,
                                     (double)c.mom_grid[0], (double)c.mom_grid[1], (double)c.mom_grid[2],
                                     (double)c.mom_grid[3], (double)c.mom_grid[4], (double)c.mom_grid[5],
                                     (double)c.mom_grid[6], (double)c.mom_grid[7], (double)c.mom_grid[8],
                                     (double)c.mom_grid[9], (double)c.mom_grid[10], (double)c.mom_grid[11],
                                     (double)c.mom_grid[12], (double)c.mom_grid[13], (double)c.mom_grid[14],
                                     (double)c.mom_grid[15], (double)c.mom_grid[16], (double)c.mom_grid[17],
                                     (double)c.mom_grid[18], (double)c.mom_grid[19], (double)c.mom_grid[20],
                                     (double)c.mom_grid[21], (double)c.mom_hi, (double)c.mom_lo};
    if (!ctx->bexec || ctx->bkey != key) {
        if (ctx->bexec) { (void)hipGraphExecDestroy(ctx->bexec); ctx->bexec = nullptr; }
        if (ctx->bgraph) { (void)hipGraphDestroy(ctx->bgraph); ctx->bgraph = nullptr; }
        hipStream_t cs = ctx->cap_stream;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        enqueue_build(ctx, pos, mass, cs);
        HIP_TRY(hipStreamEndCapture(cs, &ctx->bgraph));
        HIP_TRY(hipGraphInstantiate(&ctx->bexec, ctx->bgraph, nullptr, nullptr, 0));
        ctx->bkey = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->bexec, s));
    return PBH_OK;
}

// Device part of a build: kernels only (capturable).
void enqueue_build(pbh_ctx* ctx, const double* pos, const double* mass, hipStream_t s) {
    Dev& d = ctx->d;
    const BuildCfg& c = ctx->cfg;
    launch_zero_u64(d.cnt, kNumCounters - 5, s);   // keep the KDK slots (>= 11)
    launch_bbox(d, c, pos, mass, ctx->nblk_box, s);
    launch_keys(d, c, pos, ctx->nblk_box, s);
    launch_key_sort(d, c, s);
    launch_gather(d, c, pos, mass, s);
    launch_topology(d, c, s);
    launch_moments(d, c, s);
    launch_groups(d, c, s);
}

// Changeover constants of one cluster (see ClusterParams); lists reach r_out + r_buff.
ClusterParams cluster_params(double r_in, double r_out, double r_buff = 0.0) {
    ClusterParams p;
    std::memset(&p, 0, sizeof(p));
    p.r_in = r_in;
    p.r_out = r_out;
    p.rout2 = r_out * r_out;
    p.rlist = r_out + r_buff;
    p.rlist2 = p.rlist * p.rlist;
    const double delta = r_out - r_in;
    if (r_out > 0.0 && delta > 0.0) {
        // g(t - a) = sum_k dk t^k with g(x) = 35x^4 - 84x^5 + 70x^6 - 20x^7
        const double a = r_in / delta;
        const double cg[8] = {0, 0, 0, 0, 35.0, -84.0, 70.0, -20.0};
        double dk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = 4; q <= 7; ++q) {
            double binom = 1.0;   // C(q, k) built up from k = 0
            for (int k = 0; k <= q; ++k) {
                if (k > 0) binom = binom * (double)(q - k + 1) / (double)k;
                dk[k] += cg[q] * binom * std::pow(-a, (double)(q - k));
            }
        }
        // G(t) = -d0/t + d1 ln t + sum_{k>=2} dk t^(k-1)/(k-1);
        // Phi_R(s) = -1/r_out - (G(a+1) - G(s/delta))/delta
        auto Gt = [&](double t) {
            double g = 0.0;
            if (dk[0] != 0.0) g += -dk[0] / t;
            if (dk[1] != 0.0) g += dk[1] * std::log(t);
            for (int k = 2; k <= 7; ++k) g += dk[k] * std::pow(t, (double)(k - 1)) / (double)(k - 1);
            return g;
        };
        const double G1 = Gt(a + 1.0);
        p.inv_delta = 1.0 / delta;
        p.d0 = dk[0];
        p.l1 = dk[1] / delta;
        p.c0 = -1.0 / r_out - G1 / delta - (dk[1] != 0.0 ? p.l1 * std::log(delta) : 0.0);
        for (int k = 2; k <= 7; ++k) p.e[k - 2] = dk[k] / ((double)(k - 1) * delta);
        p.inner = -1.0 / r_out - (G1 - Gt(a)) / delta;
        if (r_in == 0.0) p.inner = -1.0 / r_out - (G1 - Gt(0.0)) / delta;
    } else if (r_out > 0.0) {
        p.inner = -1.0 / r_out;   // step: W = 0 below r_out
    }
    p.f_r_in = (float)p.r_in;
    p.f_r_out = (float)p.r_out;
    p.f_inv_delta = (float)p.inv_delta;
    p.f_c0 = (float)p.c0;
    p.f_d0 = (float)p.d0;
    p.f_l1 = (float)p.l1;
    p.f_inner = (float)p.inner;
    for (int k = 0; k < 6; ++k) p.f_e[k] = (float)p.e[k];
    return p;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

void mark(pbh_ctx* ctx, int k, hipStream_t s) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev[k], s);
}

constexpr int kParamsPerStore = 8;
struct ParamPack {
    ClusterParams p[kParamsPerStore];
};

__global__ void k_store_params(ParamPack pk, int n, ClusterParams* dst) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = pk.p[i];
}

// Copy per-cluster constants to the device. Small counts travel as kernel
// arguments (no host buffer outlives the call, and the copy can be captured);
// large counts use a copy followed by a wait.
pbh_status upload_cparams(pbh_ctx* ctx, const std::vector<ClusterParams>& cps, hipStream_t s) {
    const int C = (int)cps.size();
    if (C <= 64) {
        for (int b = 0; b < C; b += kParamsPerStore) {
            ParamPack pk;
            const int k = std::min(kParamsPerStore, C - b);
            for (int i = 0; i < k; ++i) pk.p[i] = cps[b + i];
            hipLaunchKernelGGL(k_store_params, dim3(1), dim3(kParamsPerStore), 0, s, pk, k,
                               ctx->d.cparams + b);
        }
        HIP_TRY(hipGetLastError());
        return PBH_OK;
    }
    HIP_TRY(hipMemcpyAsync(ctx->d.cparams, cps.data(), cps.size() * sizeof(ClusterParams),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PBH_OK;
}

pbh_status check_radii(pbh_ctx* ctx, double r_in, double r_out) {
    if (!finite_nonneg(r_in) || !finite_nonneg(r_out) || r_out < r_in)
        return fail(ctx, PBH_E_ARG, "need 0 <= r_in <= r_out, both finite");
    return PBH_OK;
}

pbh_status finish_build(pbh_ctx* ctx, hipStream_t s) {
    unsigned long long h[kNumCounters];
    int32_t lo[32];
    HIP_TRY(hipMemcpyAsync(h, ctx->d.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(lo, ctx->d.lvl_off, sizeof(lo), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int D = ctx->cfg.D;
    ctx->lvl_count.assign(D + 1, 0);
    for (int l = 0; l <= D; ++l) ctx->lvl_count[l] = lo[l + 1] - lo[l];
    if (h[kErr] & kErrNonFinite) {
        ctx->built = false;
        return fail(ctx, PBH_E_NONFINITE, "non-finite position or mass");
    }
    if (h[kErr] & kErrNodeCap) {
        ctx->built = false;
        return fail(ctx, PBH_E_INTERNAL, "node capacity exceeded");
    }
    ctx->built = true;
    return PBH_OK;
}

pbh_status do_force(pbh_ctx* ctx, const double* pos, const double* mass,
                    const std::vector<ClusterParams>& cps, double theta, double eps,
                    double* acc, double* pot, int64_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap,
                    int64_t* nbr_total, hipStream_t s) {
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "pbh_force called without a successful build");
    if (pos != ctx->built_pos || mass != ctx->built_mass)
        return fail(ctx, PBH_E_STATE, "pos and mass must be the arrays of the last build");
    if (!finite_nonneg(theta) || !finite_nonneg(eps)) return fail(ctx, PBH_E_ARG, "theta and eps must be finite and >= 0");
    if (!acc || !pot) return fail(ctx, PBH_E_ARG, "acc and pot are required");
    if (nbr_cap < 0 || (nbr_cap > 0 && !nbr_idx)) return fail(ctx, PBH_E_ARG, "bad neighbour buffer");
    Dev& d = ctx->d;
    const BuildCfg& c = ctx->cfg;
    pbh_status up = upload_cparams(ctx, cps, s);
    if (up != PBH_OK) return up;
    launch_rcrit(d, c, theta, s);
    WalkCfg w;
    w.theta = theta;
    w.eps = eps;
    w.mixed = ctx->params.prec == PBH_MIXED;
    w.tile = ctx->params.walk_tile;
    w.max_copies = ctx->params.lanes_per_particle ? ctx->params.lanes_per_particle : 64;
    w.cpos = pos;
    w.cmass = mass;
    w.grid = walk_grid(ctx, w.mixed);   // persistent: workgroups leave when the group queue is empty
    w.stack_cap = kStackCap;
    w.count_nbr = nbr_off != nullptr;   // the walk counts the neighbours of every particle
    w.stage_cap = w.count_nbr ? ensure_stage(ctx) : 0;
    mark(ctx, 2, s);
    launch_walk(d, c, w, acc, pot, s);
    ctx->last_walk_grid = w.grid;
    mark(ctx, 3, s);
    ctx->ev_walk = ctx->timing;
    ctx->ev_nbr = false;
    if (nbr_off) {
        const int grid = ctx->grid_mixed;
        mark(ctx, 4, s);
        exclusive_scan_i32_to_i64(d.nbr_cnt, nbr_off, c.n, d.scan_tmp, s);
        if (nbr_total) {
            int64_t tot = 0;
            HIP_TRY(hipMemcpyAsync(&tot, nbr_off + c.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            *nbr_total = tot;
            if (tot > nbr_cap)
                return fail(ctx, PBH_E_NBR_OVERFLOW, "neighbour capacity " + std::to_string(nbr_cap) +
                                                         " < needed " + std::to_string(tot));
        }
        if (w.stage_cap > 0) launch_nbr_copy(d, c, w.stage_cap, nbr_off, nbr_idx, nbr_cap, s);
        launch_nbr_fill(d, c, grid, kStackCap, nbr_off, nbr_idx, nbr_cap, s);
        mark(ctx, 5, s);
        ctx->ev_nbr = ctx->timing;
        if (nbr_total) {
            unsigned long long err = 0;
            HIP_TRY(hipMemcpyAsync(&err, d.cnt + kErr, sizeof(err), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (err & kErrStale)
                return fail(ctx, PBH_E_STATE, "pos or mass changed since the build");
            if (err & (kErrWalkStack | kErrNbrStack))
                return fail(ctx, PBH_E_INTERNAL, "traversal stack overflow");
        }
    }
    return PBH_OK;
}

pbh_status ensure_irr_err(pbh_ctx* ctx);

// Scratch of one irregular-force call: the flag word and, for the key-order
// route, ranks and records of up to `cap` particles.
struct IrrScratch {
    unsigned long long* err = nullptr;
    int32_t* rank = nullptr;
    IrrRec* rec = nullptr;
    int64_t cap = 0;
};

// Shared part of pbh_irregular, pbh_irregular_batched and
// pbh_irregular_noalloc: p already holds the cluster constants (C, cl_off,
// cps or cp0). fixed == nullptr: the context's buffers, allocated on first
// need; otherwise the given scratch, and nothing is allocated.
pbh_status do_irregular(pbh_ctx* ctx, IrrParams& p, int64_t n, const double* pos, const double* vel,
                        const double* mass, double eps, const int64_t* nbr_off,
                        const int32_t* nbr_idx, int64_t nbr_cap, int64_t n_targets,
                        const int32_t* targets, double* acc, double* jerk, double* pot,
                        int32_t check, hipStream_t s, const IrrScratch* fixed = nullptr) {
    if (n < 1 || n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "need 1 <= n < 2^31");
    if (targets && n_targets < 0) return fail(ctx, PBH_E_ARG, "n_targets must be >= 0");
    if (targets && n_targets == 0) return PBH_OK;   // an empty target list: nothing to do
    if (!pos || !mass || !acc || !nbr_off) return fail(ctx, PBH_E_ARG, "pos, mass, acc and nbr_off are required");
    if (jerk && !vel) return fail(ctx, PBH_E_ARG, "the jerk needs vel");
    if (nbr_cap < 0 || (nbr_cap > 0 && !nbr_idx)) return fail(ctx, PBH_E_ARG, "bad neighbour buffer");
    if (!finite_nonneg(eps)) return fail(ctx, PBH_E_ARG, "eps must be finite and >= 0");
    unsigned long long* err = nullptr;
    if (fixed) {
        err = fixed->err;
    } else {
        pbh_status ae = ensure_irr_err(ctx);
        if (ae != PBH_OK) return ae;
        err = ctx->irr_err;
    }
    launch_zero_u64(err, 1, s);   // a kernel, not a memset: callers may capture the call
    p.n = n;
    p.n_tgt = targets ? n_targets : n;
    p.tgt = targets;
    // With a build of the same particle count, all targets or a long target
    // list: pack the particles into key-order records and take the targets in
    // key order (a wave's gathers then stay in a compact, cached range; the
    // sums do not depend on it). Otherwise gather from the caller's arrays
    // (a short list does not pay for a pass over every particle).
    Dev& d = ctx->d;
    if (ctx->built && ctx->cfg.n == n && (!targets || n_targets * kIrrPackRatio >= n)) {
        if (fixed) {
            if (fixed->cap < n) return fail(ctx, PBH_E_ARG, "n exceeds the fixed scratch");
            p.rank = fixed->rank;
            p.rec = fixed->rec;
        } else {
            if (d.irr_len < n) {
                ctx->irr_rank_ok = false;
                if (!dalloc(ctx, &d.irr_rank, n) || !dalloc(ctx, &d.irr_rec, n)) {
                    (void)hipGetLastError();
                    return fail(ctx, PBH_E_OOM, "irregular-force records");
                }
                d.irr_len = n;
            }
            p.rank = d.irr_rank;
            p.rec = d.irr_rec;
            p.rank_fresh = !ctx->irr_rank_ok;
        }
        p.perm = d.perm;
        p.order = targets ? nullptr : d.perm;
    }
    p.pos = pos;
    p.vel = vel;
    p.mass = mass;
    p.off = nbr_off;
    p.idx = nbr_idx;
    p.cap = nbr_cap;
    p.eps2 = eps * eps;
    p.acc = acc;
    p.jerk = jerk;
    p.pot = pot;
    p.err = err;
    launch_irregular(p, s);
    HIP_TRY(hipGetLastError());
    if (p.rec && !fixed) ctx->irr_rank_ok = true;
    if (check) {
        unsigned long long bits = 0;
        HIP_TRY(hipMemcpyAsync(&bits, err, sizeof(bits), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bits & kIrrBadTarget) return fail(ctx, PBH_E_ARG, "a target index is outside [0, n)");
        if (bits & kIrrBadOffsets) return fail(ctx, PBH_E_ARG, "neighbour offsets decrease or pass nbr_cap");
        if (bits & kIrrBadIndex) return fail(ctx, PBH_E_ARG, "a neighbour index is outside [0, n)");
    }
    return PBH_OK;
}

pbh_status ensure_irr_err(pbh_ctx* ctx) {
    if (ctx->irr_err) return PBH_OK;
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(unsigned long long)) != hipSuccess)
        return fail(ctx, PBH_E_OOM, "irregular-force flag word");
    ctx->irr_err = (unsigned long long*)q;
    return PBH_OK;
}

template <typename T>
bool halloc(pbh_ctx* ctx, T** p, int64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    ctx->herm.mem.push_back(q);
    *p = (T*)q;
    return true;
}

pbh_status ensure_herm(pbh_ctx* ctx, int64_t n) {
    auto& h = ctx->herm;
    if (h.n >= n) return PBH_OK;
    for (void* q : h.mem) (void)hipFree(q);
    h.mem.clear();
    h.cap = 0;
    h.idx = nullptr;
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (!halloc(ctx, &h.a, 3 * n) || !halloc(ctx, &h.j, 3 * n) ||
        !halloc(ctx, &h.xp, 3 * n) || !halloc(ctx, &h.vp, 3 * n) ||
        !halloc(ctx, &h.tau, n) || !halloc(ctx, &h.dt, n) || !halloc(ctx, &h.dt0, n) ||
        !halloc(ctx, &h.act, n) ||
        !halloc(ctx, &h.ctl, kHermCtl) || !halloc(ctx, &h.lev, kLevLen) ||
        !halloc(ctx, &h.bucket, (int64_t)(kHermK + 1) * n) || !halloc(ctx, &h.slot, n) ||
        !halloc(ctx, &h.fr, 3 * n) || !halloc(ctx, &h.potr, n) ||
        !halloc(ctx, &h.poti, n) || !halloc(ctx, &h.pott, n) || !halloc(ctx, &h.scr, 3 * n) ||
        !halloc(ctx, &h.epart, nb) || !halloc(ctx, &h.off, n + 1)) {
        for (void* q : h.mem) (void)hipFree(q);
        h.mem.clear();
        h.n = -1;
        return fail(ctx, PBH_E_OOM, "Hermite state");
    }
    h.n = n;
    return PBH_OK;
}

// Irregular-force launch parameters of one cluster for the Hermite driver.
IrrParams herm_irr(pbh_ctx* ctx, int64_t n, double r_in, double r_out, double eps,
                   const double* mass, const int64_t* off, const int32_t* idx, int64_t cap) {
    IrrParams ip;
    ip.n = n;
    ip.n_tgt = n;
    ip.C = 1;
    ip.cp0 = cluster_params(r_in, r_out);
    ip.eps2 = eps * eps;
    ip.mass = mass;
    ip.off = off;
    ip.idx = idx;
    ip.cap = cap;
    ip.err = ctx->irr_err;
    return ip;
}

// One regular step of Hermite integration of F_I (see herm.hip), in place.
constexpr int64_t kHermMaxBlocks = 1ll << 20;
constexpr int kHermBatch = 16;   // blocks per graph launch
static_assert(kHermBatch % 2 == 0, "block parity restarts at each batch");

pbh_status do_hermite(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                      const double* fr, double r_in, double r_out, double eps,
                      const int64_t* off, const int32_t* idx, int64_t cap, double T, double eta,
                      int64_t* stats, hipStream_t s) {
    auto& h = ctx->herm;
    h.last_n = n;
    launch_zero_u64(ctx->irr_err, 1, s);
    IrrParams ip = herm_irr(ctx, n, r_in, r_out, eps, mass, off, idx, cap);
    ip.pos = pos;
    ip.vel = vel;
    ip.acc = h.a;
    ip.jerk = h.j;
    launch_irregular(ip, s);
    HermParams hp;
    hp.n = n;
    hp.x = pos;
    hp.v = vel;
    hp.a = h.a;
    hp.j = h.j;
    hp.xp = h.xp;
    hp.vp = h.vp;
    hp.fr = fr;
    hp.tau = h.tau;
    hp.dt = h.dt;
    hp.dt0 = h.dt0;
    hp.act = h.act;
    hp.ctl = h.ctl;
    if (!h.done) {
        HIP_TRY(hipHostMalloc((void**)&h.done, sizeof(unsigned long long), hipHostMallocCoherent));
        for (auto& e : h.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    HIP_TRY(hipHostGetDevicePointer((void**)&hp.done_host, h.done, 0));
    hp.lev = h.lev;
    hp.bucket = h.bucket;
    hp.slot = h.slot;
    hp.off = off;
    hp.idx = idx;
    hp.cap = cap;
    hp.tend = 1ull << (kHermK + 2);
    hp.unit = T / (double)(1ll << (kHermK + 2));
    hp.dtmax = T / 4.0;
    hp.eta = eta;
    launch_zero_u64(h.lev, kLevLen, s);
    launch_herm_start(hp, ip, s);
    launch_zero_u64(h.ctl, kHermCtl, s);
    ip.pos = h.xp;   // the block's force reads predicted states
    ip.vel = h.vp;
    ip.acc = ip.jerk = nullptr;
    // Blocks run in batches of kHermBatch, each batch one graph launch. The
    // front that finds every particle at the end sets a host flag; the host
    // reads it once a batch has finished, while the next batch runs, so the GPU
    // does not wait for the host; the batch after the last busy one is empty.
    const std::vector<double> key = {(double)n, (double)(uintptr_t)pos, (double)(uintptr_t)vel,
                                     (double)(uintptr_t)mass, (double)(uintptr_t)fr, (double)(uintptr_t)off,
                                     (double)(uintptr_t)idx, (double)cap, r_in, r_out, eps, T, eta,
                                     (double)(uintptr_t)h.a, (double)(uintptr_t)h.bucket,
                                     (double)(uintptr_t)ctx->irr_err};
    if (!h.gexec || h.gkey != key) {
        if (h.gexec) { (void)hipGraphExecDestroy(h.gexec); h.gexec = nullptr; }
        if (h.graph) { (void)hipGraphDestroy(h.graph); h.graph = nullptr; }
        h.gkey.clear();
        hipStream_t cs = ctx->cap_stream;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int b = 0; b < kHermBatch; ++b) {   // kHermBatch is even: block parity b & 1
            launch_herm_front(hp, b & 1, cs);
            launch_herm_force_correct(hp, ip, b & 1, cs);
        }
        HIP_TRY(hipStreamEndCapture(cs, &h.graph));
        HIP_TRY(hipGraphInstantiate(&h.gexec, h.graph, nullptr, nullptr, 0));
        h.gkey = key;
    }
    volatile unsigned long long* flag = h.done;
    *flag = 0ull;   // no launch of an earlier call is pending (each call ends with a wait)
    HIP_TRY(hipGraphLaunch(h.gexec, s));
    HIP_TRY(hipEventRecord(h.ev[0], s));
    for (int64_t batch = 0;; ++batch) {
        if ((batch + 1) * kHermBatch >= kHermMaxBlocks) {
            HIP_TRY(hipStreamSynchronize(s));
            return fail(ctx, PBH_E_INTERNAL, "Hermite block steps exceed the limit");
        }
        HIP_TRY(hipGraphLaunch(h.gexec, s));
        HIP_TRY(hipEventRecord(h.ev[(batch + 1) & 1], s));
        HIP_TRY(hipEventSynchronize(h.ev[batch & 1]));
        if (*flag) break;
    }
    unsigned long long c[kHermCtl], err = 0;
    HIP_TRY(hipMemcpyAsync(c, h.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, ctx->irr_err, sizeof(err), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) return fail(ctx, PBH_E_ARG, "malformed neighbour lists in the Hermite integration");
    if (stats) {
        stats[0] += (int64_t)c[kHermBlocks];
        stats[1] += (int64_t)c[kHermSteps];
        stats[2] = std::max<int64_t>(stats[2], (int64_t)c[kHermKmax]);
    }
    return PBH_OK;
}

}  // namespace

extern "C" {

const char* pbh_status_string(pbh_status s) {
    switch (s) {
        case PBH_OK: return "ok";
        case PBH_E_ARG: return "invalid argument";
        case PBH_E_OOM: return "out of device memory";
        case PBH_E_HIP: return "HIP runtime error";
        case PBH_E_NONFINITE: return "non-finite input";
        case PBH_E_NBR_OVERFLOW: return "neighbour capacity too small";
        case PBH_E_STATE: return "no matching build";
        case PBH_E_INTERNAL: return "device capacity guard tripped";
    }
    return "unknown status";
}

const char* pbh_last_error(const pbh_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static pbh_status resolve_params(pbh_ctx* ctx, const pbh_params* in, pbh_params* out) {
    pbh_params p{8, 0, 64, 0, 0, PBH_MIXED};   // n_crit 0: chosen per build from N
    if (in) {
        const int t = in->walk_tile;
        if (in->leaf_size < 0 || in->n_crit < 0 || in->n_crit > 64 || in->key_bits < 0 ||
            in->key_bits > 21 || (in->prec != PBH_FP64 && in->prec != PBH_MIXED) ||
            (t != 0 && t != 64 && t != 96 && t != 128) || in->lanes_per_particle < 0 ||
            in->lanes_per_particle > 64)
            return fail(ctx, PBH_E_ARG,
                        "bad parameters (n_crit <= 64, walk_tile 64/96/128, lanes_per_particle <= 64, "
                        "key_bits <= 21)");
        if (in->leaf_size) p.leaf_size = in->leaf_size;
        if (in->n_crit) p.n_crit = in->n_crit;
        if (t) p.walk_tile = t;
        p.lanes_per_particle = in->lanes_per_particle;
        p.key_bits = in->key_bits;
        p.prec = in->prec;
    }
    *out = p;
    return PBH_OK;
}

pbh_status pbh_create(int device, const pbh_params* params, pbh_ctx** out) {
    if (!out) return PBH_E_ARG;
    *out = nullptr;
    pbh_ctx* ctx = new pbh_ctx();
    pbh_status st = resolve_params(ctx, params, &ctx->params);
    if (st != PBH_OK) {
        delete ctx;
        return st;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete ctx;
        return PBH_E_ARG;
    }
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete ctx;
        return PBH_E_HIP;
    }
    // the allocation-free entry point's scratch on this device (set up once)
    if (!na_scratch_setup(device)) {
        (void)hipStreamDestroy(ctx->cap_stream);
        delete ctx;
        return PBH_E_HIP;
    }
    *out = ctx;
    return PBH_OK;
}

void pbh_destroy(pbh_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->bexec) (void)hipGraphExecDestroy(ctx->bexec);
    if (ctx->bgraph) (void)hipGraphDestroy(ctx->bgraph);
    free_all(ctx);
    if (ctx->k_acc) (void)hipFree(ctx->k_acc);
    if (ctx->k_pot) (void)hipFree(ctx->k_pot);
    if (ctx->k_epart) (void)hipFree(ctx->k_epart);
    if (ctx->irr_err) (void)hipFree(ctx->irr_err);
    for (void* q : ctx->herm.mem) (void)hipFree(q);
    if (ctx->herm.gexec) (void)hipGraphExecDestroy(ctx->herm.gexec);
    if (ctx->herm.graph) (void)hipGraphDestroy(ctx->herm.graph);
    if (ctx->herm.done) (void)hipHostFree(ctx->herm.done);
    for (auto& e : ctx->herm.ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

pbh_status pbh_set_params(pbh_ctx* ctx, const pbh_params* params) {
    if (!ctx) return PBH_E_ARG;
    pbh_params p;
    pbh_status st = resolve_params(ctx, params, &p);
    if (st != PBH_OK) return st;
    ctx->params = p;
    ctx->built = false;
    return PBH_OK;
}

pbh_status pbh_get_params(const pbh_ctx* ctx, pbh_params* out) {
    if (!ctx || !out) return PBH_E_ARG;
    *out = ctx->params;
    return PBH_OK;
}

pbh_status pbh_build(pbh_ctx* ctx, int64_t n, const double* pos, const double* mass,
                     pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n < 1 || !pos || !mass) return fail(ctx, PBH_E_ARG, "need n >= 1 and pos/mass");
    if (n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->built = false;
    ctx->batched = false;
    ctx->last = s;
    const int64_t offs[2] = {0, n};
    pbh_status st = setup_build(ctx, n, 1, offs, s);
    if (st != PBH_OK) return st;
    mark(ctx, 0, s);
    st = launch_build(ctx, pos, mass, s);
    if (st != PBH_OK) return st;
    mark(ctx, 1, s);
    ctx->ev_build = ctx->timing;
    ctx->built_pos = pos;
    ctx->built_mass = mass;
    return finish_build(ctx, s);
}

pbh_status pbh_build_batched(pbh_ctx* ctx, int32_t n_clusters, const int64_t* offsets,
                             const double* pos, const double* mass, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n_clusters < 1 || n_clusters > 65536 || !offsets || !pos || !mass)
        return fail(ctx, PBH_E_ARG, "need 1 <= n_clusters <= 65536, offsets, pos, mass");
    if (offsets[0] != 0) return fail(ctx, PBH_E_ARG, "offsets[0] must be 0");
    for (int k = 0; k < n_clusters; ++k)
        if (offsets[k + 1] <= offsets[k]) return fail(ctx, PBH_E_ARG, "every cluster must be non-empty");
    const int64_t n = offsets[n_clusters];
    if (n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->built = false;
    ctx->batched = true;
    ctx->last = s;
    pbh_status st = setup_build(ctx, n, n_clusters, offsets, s);
    if (st != PBH_OK) return st;
    mark(ctx, 0, s);
    st = launch_build(ctx, pos, mass, s);
    if (st != PBH_OK) return st;
    mark(ctx, 1, s);
    ctx->ev_build = ctx->timing;
    ctx->built_pos = pos;
    ctx->built_mass = mass;
    return finish_build(ctx, s);
}

pbh_status pbh_force_buffered(pbh_ctx* ctx, const double* pos, const double* mass, double r_in,
                              double r_out, double r_buff, double theta, double eps, double* acc,
                              double* pot, int64_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap,
                              int64_t* nbr_total, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    if (!finite_nonneg(r_buff)) return fail(ctx, PBH_E_ARG, "r_buff must be finite and >= 0");
    if (ctx->built && ctx->cfg.n_clusters != 1)
        return fail(ctx, PBH_E_STATE, "last build was batched: use pbh_force_batched");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    std::vector<ClusterParams> cps(1, cluster_params(r_in, r_out, r_buff));
    return do_force(ctx, pos, mass, cps, theta, eps, acc, pot, nbr_off, nbr_idx, nbr_cap, nbr_total, s);
}

pbh_status pbh_force(pbh_ctx* ctx, const double* pos, const double* mass, double r_in, double r_out,
                     double theta, double eps, double* acc, double* pot, int64_t* nbr_off,
                     int32_t* nbr_idx, int64_t nbr_cap, int64_t* nbr_total, pbh_stream_t stream) {
    return pbh_force_buffered(ctx, pos, mass, r_in, r_out, 0.0, theta, eps, acc, pot, nbr_off,
                              nbr_idx, nbr_cap, nbr_total, stream);
}

pbh_status pbh_force_batched_buffered(pbh_ctx* ctx, const double* pos, const double* mass,
                                      const double* r_in, const double* r_out,
                                      const double* r_buff, double theta, double eps, double* acc,
                                      double* pot, int64_t* nbr_off, int32_t* nbr_idx,
                                      int64_t nbr_cap, int64_t* nbr_total, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "no successful build");
    if (!r_in || !r_out) return fail(ctx, PBH_E_ARG, "r_in and r_out arrays are required");
    std::vector<ClusterParams> cps;
    for (int k = 0; k < ctx->cfg.n_clusters; ++k) {
        pbh_status st = check_radii(ctx, r_in[k], r_out[k]);
        if (st != PBH_OK) return st;
        const double rb = r_buff ? r_buff[k] : 0.0;
        if (!finite_nonneg(rb)) return fail(ctx, PBH_E_ARG, "r_buff must be finite and >= 0");
        cps.push_back(cluster_params(r_in[k], r_out[k], rb));
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    return do_force(ctx, pos, mass, cps, theta, eps, acc, pot, nbr_off, nbr_idx, nbr_cap, nbr_total, s);
}

pbh_status pbh_force_batched(pbh_ctx* ctx, const double* pos, const double* mass, const double* r_in,
                             const double* r_out, double theta, double eps, double* acc, double* pot,
                             int64_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap, int64_t* nbr_total,
                             pbh_stream_t stream) {
    return pbh_force_batched_buffered(ctx, pos, mass, r_in, r_out, nullptr, theta, eps, acc, pot,
                                      nbr_off, nbr_idx, nbr_cap, nbr_total, stream);
}

pbh_status pbh_irregular(pbh_ctx* ctx, int64_t n, const double* pos, const double* vel,
                         const double* mass, double r_in, double r_out, double eps,
                         const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap,
                         int64_t n_targets, const int32_t* targets, double* acc, double* jerk,
                         double* pot, int32_t check, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    IrrParams p;
    p.C = 1;
    p.cp0 = cluster_params(r_in, r_out);
    return do_irregular(ctx, p, n, pos, vel, mass, eps, nbr_off, nbr_idx, nbr_cap, n_targets,
                        targets, acc, jerk, pot, check, s);
}

pbh_status pbh_irregular_batched(pbh_ctx* ctx, const double* pos, const double* vel,
                                 const double* mass, const double* r_in, const double* r_out,
                                 double eps, const int64_t* nbr_off, const int32_t* nbr_idx,
                                 int64_t nbr_cap, int64_t n_targets, const int32_t* targets,
                                 double* acc, double* jerk, double* pot, int32_t check,
                                 pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "no successful build");
    if (!r_in || !r_out) return fail(ctx, PBH_E_ARG, "r_in and r_out arrays are required");
    const int C = ctx->cfg.n_clusters;
    std::vector<ClusterParams> cps;
    for (int k = 0; k < C; ++k) {
        pbh_status st = check_radii(ctx, r_in[k], r_out[k]);
        if (st != PBH_OK) return st;
        cps.push_back(cluster_params(r_in[k], r_out[k]));
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    IrrParams p;
    p.C = C;
    p.cp0 = cps[0];
    if (C > 1) {
        pbh_status up = upload_cparams(ctx, cps, s);
        if (up != PBH_OK) return up;
        p.cl_off = ctx->d.cl_off;
        p.cps = ctx->d.cparams;
    }
    return do_irregular(ctx, p, ctx->cfg.n, pos, vel, mass, eps, nbr_off, nbr_idx, nbr_cap,
                        n_targets, targets, acc, jerk, pot, check, s);
}

pbh_status pbh_irregular_noalloc(pbh_ctx* ctx, int64_t n, const double* pos, const double* vel,
                                 const double* mass, double r_in, double r_out, double eps,
                                 const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap,
                                 int64_t n_targets, const int32_t* targets, double* acc,
                                 double* jerk, double* pot, int32_t check, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n > PBH_NOALLOC_MAX_N)
        return fail(ctx, PBH_E_ARG, "n exceeds PBH_NOALLOC_MAX_N (2^20 particles), the size of "
                                    "the allocation-free scratch; use pbh_irregular");
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    char* base = (char*)na_scratch(ctx->device);
    if (!base) return fail(ctx, PBH_E_STATE, "no scratch address for this device");
    IrrScratch fixed;
    fixed.err = (unsigned long long*)base;
    fixed.rank = (int32_t*)(base + kNaRankOff);
    fixed.rec = (IrrRec*)(base + kNaRecOff);
    fixed.cap = PBH_NOALLOC_MAX_N;
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    IrrParams p;
    p.C = 1;
    p.cp0 = cluster_params(r_in, r_out);
    return do_irregular(ctx, p, n, pos, vel, mass, eps, nbr_off, nbr_idx, nbr_cap, n_targets,
                        targets, acc, jerk, pot, check, s, &fixed);
}

pbh_status pbh_core(pbh_ctx* ctx, const double* pos, const double* mass, int64_t n_sample,
                    const int32_t* sample, double eta, double* rho, pbh_core_info* out,
                    pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "pbh_core needs a build of these particles");
    if (ctx->cfg.n_clusters != 1) return fail(ctx, PBH_E_STATE, "pbh_core works on a single-cluster build");
    const int64_t n = ctx->cfg.n;
    if (n < 7) return fail(ctx, PBH_E_ARG, "need at least 7 particles (6 neighbours each)");
    if (!pos || !mass || !sample || !out) return fail(ctx, PBH_E_ARG, "pos, mass, sample and out are required");
    if (pos != ctx->built_pos || mass != ctx->built_mass)
        return fail(ctx, PBH_E_STATE, "pos and mass must be the arrays of the last build");
    if (n_sample < 1 || n_sample > n) return fail(ctx, PBH_E_ARG, "need 1 <= n_sample <= n");
    if (!(std::isfinite(eta) && eta > 0.0)) return fail(ctx, PBH_E_ARG, "eta must be finite and > 0");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    Dev& d = ctx->d;
    if (d.irr_len < n) {   // the rank array is shared with the irregular-force records
        ctx->irr_rank_ok = false;
        if (!dalloc(ctx, &d.irr_rank, n) || !dalloc(ctx, &d.irr_rec, n)) {
            (void)hipGetLastError();
            return fail(ctx, PBH_E_OOM, "rank array");
        }
        d.irr_len = n;
    }
    if (d.core_len < n) {
        if (!dalloc(ctx, &d.core_keys, n) || !dalloc(ctx, &d.core_keys_alt, n) ||
            !dalloc(ctx, &d.core_vals, n) || !dalloc(ctx, &d.core_vals_alt, n) ||
            !dalloc(ctx, &d.core_bsum, core_bsum_len(n)) || !dalloc(ctx, &d.core_stats, 16) ||
            !dalloc(ctx, &d.core_cnt, 2)) {
            (void)hipGetLastError();
            return fail(ctx, PBH_E_OOM, "core-quantity scratch");
        }
        d.core_len = n;
    }
    double* rho_d = rho;
    if (!rho_d) {
        if (d.core_rho_len < n_sample) {
            if (!dalloc(ctx, &d.core_rho, n_sample)) {
                (void)hipGetLastError();
                return fail(ctx, PBH_E_OOM, "sample densities");
            }
            d.core_rho_len = n_sample;
        }
        rho_d = d.core_rho;
    }
    launch_zero_u64(d.core_cnt, 2, s);
    CoreLaunch c;
    c.n = n;
    c.ns = n_sample;
    c.sample = sample;
    c.node = d.node;
    c.x = d.x; c.y = d.y; c.z = d.z;
    c.perm = d.perm;
    c.rank = d.irr_rank;
    c.pos = pos;
    c.mass = mass;
    c.rho = rho_d;
    c.stats = d.core_stats;
    c.keys = d.core_keys;
    c.keys_alt = d.core_keys_alt;
    c.vals = d.core_vals;
    c.vals_alt = d.core_vals_alt;
    c.hist = d.rs_hist;
    c.scan_tmp = d.scan_tmp;
    c.bsum = d.core_bsum;
    c.ncore = d.core_cnt;
    c.err = d.core_cnt + 1;
    c.eta = eta;
    launch_core(c, s);
    HIP_TRY(hipGetLastError());
    double st[9];
    unsigned long long err = 0;
    HIP_TRY(hipMemcpyAsync(st, d.core_stats, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, d.core_cnt + 1, sizeof(err), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & kCoreBadSample) return fail(ctx, PBH_E_ARG, "a sample index is outside [0, n)");
    if (err & kCoreStackFull) return fail(ctx, PBH_E_INTERNAL, "nearest-neighbour traversal stack full");
    for (int k = 0; k < 3; ++k) out->center[k] = st[k];
    out->rho_core = st[3];
    out->r_core = st[4];
    out->n_core = (int64_t)st[5];
    out->r_half = st[6];
    out->r_min = st[7];
    out->dt_min = st[8];
    return PBH_OK;
}

pbh_status pbh_hermite(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                       const double* fr, double r_in, double r_out, double eps,
                       const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap, double dt_reg,
                       double eta, int64_t* stats, pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n < 1 || n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "need 1 <= n < 2^31");
    if (!pos || !vel || !mass || !nbr_off) return fail(ctx, PBH_E_ARG, "pos, vel, mass and nbr_off are required");
    if (nbr_cap < 0 || (nbr_cap > 0 && !nbr_idx)) return fail(ctx, PBH_E_ARG, "bad neighbour buffer");
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    if (!finite_nonneg(eps)) return fail(ctx, PBH_E_ARG, "eps must be finite and >= 0");
    if (!(std::isfinite(dt_reg) && dt_reg > 0.0) || !(std::isfinite(eta) && eta > 0.0))
        return fail(ctx, PBH_E_ARG, "dt_reg and eta must be finite and > 0");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    if ((st = ensure_irr_err(ctx)) != PBH_OK) return st;
    if ((st = ensure_herm(ctx, n)) != PBH_OK) return st;
    if (stats) stats[0] = stats[1] = stats[2] = 0;
    return do_hermite(ctx, n, pos, vel, mass, fr, r_in, r_out, eps, nbr_off, nbr_idx, nbr_cap, dt_reg,
                      eta, stats, s);
}

// regular force and buffered lists at pos (library-owned list buffer, grown on demand)
static pbh_status p3t_regular(pbh_ctx* ctx, int64_t n, const double* pos, const double* mass,
                              double r_in, double r_out, double r_buff, double theta, double eps,
                              hipStream_t s) {
    auto& h = ctx->herm;
    pbh_status st = pbh_build(ctx, n, pos, mass, s);
    if (st != PBH_OK) return st;
    for (int attempt = 0; attempt < 3; ++attempt) {
        int64_t total = 0;
        st = pbh_force_buffered(ctx, pos, mass, r_in, r_out, r_buff, theta, eps, h.fr, h.potr, h.off,
                                h.idx, h.cap, &total, s);
        if (st != PBH_E_NBR_OVERFLOW) return st;
        const int64_t want = total + total / 4 + 1024;
        int32_t* q = nullptr;
        if (!halloc(ctx, &q, want)) return fail(ctx, PBH_E_OOM, "P3T neighbour lists");
        h.idx = q;   // the old buffer stays in herm.mem until the context is destroyed or resized
        h.cap = want;
    }
    return fail(ctx, PBH_E_INTERNAL, "neighbour capacity did not settle");
}

pbh_status pbh_p3t(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                   double r_in, double r_out, double r_buff, double theta, double eps, double dt_reg,
                   double eta, int32_t steps, double* energy_out, int64_t* stats,
                   pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n < 1 || n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "need 1 <= n < 2^31");
    if (!pos || !vel || !mass) return fail(ctx, PBH_E_ARG, "pos, vel and mass are required");
    if (steps < 0) return fail(ctx, PBH_E_ARG, "steps must be >= 0");
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    if (!finite_nonneg(r_buff) || !finite_nonneg(theta) || !finite_nonneg(eps))
        return fail(ctx, PBH_E_ARG, "r_buff, theta and eps must be finite and >= 0");
    if (!(std::isfinite(dt_reg) && dt_reg > 0.0) || !(std::isfinite(eta) && eta > 0.0))
        return fail(ctx, PBH_E_ARG, "dt_reg and eta must be finite and > 0");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    if ((st = ensure_irr_err(ctx)) != PBH_OK) return st;
    if ((st = ensure_herm(ctx, n)) != PBH_OK) return st;
    auto& h = ctx->herm;
    if (stats) stats[0] = stats[1] = stats[2] = 0;
    const int nb = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if ((st = p3t_regular(ctx, n, pos, mass, r_in, r_out, r_buff, theta, eps, s)) != PBH_OK) return st;
    for (int k = 0; k <= steps; ++k) {
        if (energy_out) {   // E = sum m v^2 / 2 + sum m (Phi_R + Phi_I) / 2
            launch_zero_u64(ctx->irr_err, 1, s);
            IrrParams ip = herm_irr(ctx, n, r_in, r_out, eps, mass, h.off, h.idx, h.cap);
            ip.pos = pos;
            ip.vel = vel;
            ip.acc = h.scr;
            ip.pot = h.poti;
            launch_irregular(ip, s);
            launch_add(n, h.potr, h.poti, h.pott, s);
            launch_energy(vel, mass, h.pott, n, h.epart, nb, energy_out + k, s);
        }
        if (k == steps) break;
        launch_kick(vel, h.fr, 0.5 * dt_reg, n, s);
        st = do_hermite(ctx, n, pos, vel, mass, h.fr, r_in, r_out, eps, h.off, h.idx, h.cap, dt_reg, eta,
                        stats, s);
        if (st != PBH_OK) return st;
        if ((st = p3t_regular(ctx, n, pos, mass, r_in, r_out, r_buff, theta, eps, s)) != PBH_OK) return st;
        launch_kick(vel, h.fr, 0.5 * dt_reg, n, s);
    }
    HIP_TRY(hipGetLastError());
    return PBH_OK;
}

static pbh_status kdk_prepare(pbh_ctx* ctx, int64_t n, double r_in, double r_out, double theta,
                              double eps, hipStream_t s) {
    if (n < 1 || n >= (1ll << 31) - 1) return fail(ctx, PBH_E_ARG, "bad n");
    pbh_status st = check_radii(ctx, r_in, r_out);
    if (st != PBH_OK) return st;
    if (!finite_nonneg(theta) || !finite_nonneg(eps)) return fail(ctx, PBH_E_ARG, "bad theta/eps");
    const int64_t offs[2] = {0, n};
    st = setup_build(ctx, n, 1, offs, s);
    if (st != PBH_OK) return st;
    if (ctx->k_n != n) {
        if (ctx->k_acc) (void)hipFree(ctx->k_acc);
        if (ctx->k_pot) (void)hipFree(ctx->k_pot);
        if (ctx->k_epart) (void)hipFree(ctx->k_epart);
        ctx->k_acc = ctx->k_pot = ctx->k_epart = nullptr;
        ctx->k_n = -1;
        ctx->k_nblk = (int)std::min<int64_t>(1024, (n + 255) / 256) + 1;
        HIP_TRY(hipMalloc(&ctx->k_acc, sizeof(double) * 3 * n));
        HIP_TRY(hipMalloc(&ctx->k_pot, sizeof(double) * n));
        HIP_TRY(hipMalloc(&ctx->k_epart, sizeof(double) * ctx->k_nblk));
        ctx->k_n = n;
    }
    ctx->batched = false;
    std::vector<ClusterParams> cps(1, cluster_params(r_in, r_out));
    return upload_cparams(ctx, cps, s);
}

// force of the current positions into k_acc / k_pot (kernels only)
static void kdk_force(pbh_ctx* ctx, const double* pos, const double* mass, double theta, double eps,
                      hipStream_t s) {
    enqueue_build(ctx, pos, mass, s);
    launch_rcrit(ctx->d, ctx->cfg, theta, s);
    WalkCfg w;
    w.theta = theta;
    w.eps = eps;
    w.mixed = ctx->params.prec == PBH_MIXED;
    w.tile = ctx->params.walk_tile;
    w.max_copies = ctx->params.lanes_per_particle ? ctx->params.lanes_per_particle : 64;
    w.grid = walk_grid(ctx, w.mixed);
    w.stack_cap = kStackCap;
    w.count_nbr = 0;
    w.stage_cap = 0;
    launch_walk(ctx->d, ctx->cfg, w, ctx->k_acc, ctx->k_pot, s);
    ctx->last_walk_grid = w.grid;
}

__global__ void k_energy_store(const double* e, double* out, unsigned long long* cnt) {
    // out[cnt[kCntKdkStep]] = *e, then advance the slot
    const unsigned long long k = cnt[kCntKdkStep];
    out[k] = *e;
    cnt[kCntKdkStep] = k + 1;
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

static void kdk_energy(pbh_ctx* ctx, const double* vel, const double* mass, double* energy_out,
                       hipStream_t s) {
    double* e_tmp = ctx->k_epart + ctx->k_nblk - 1;   // last partial slot reused as the result
    launch_energy(vel, mass, ctx->k_pot, ctx->cfg.n, ctx->k_epart, ctx->k_nblk - 1, e_tmp, s);
    hipLaunchKernelGGL(k_energy_store, dim3(1), dim3(1), 0, s, (const double*)e_tmp, energy_out,
                       ctx->d.cnt);
}

static void kdk_step(pbh_ctx* ctx, double* pos, double* vel, const double* mass, double dt,
                     double theta, double eps, double* energy_out, hipStream_t s) {
    const int64_t n = ctx->cfg.n;
    launch_kick(vel, ctx->k_acc, 0.5 * dt, n, s);
    launch_drift(pos, vel, dt, n, s);
    kdk_force(ctx, pos, mass, theta, eps, s);
    launch_kick(vel, ctx->k_acc, 0.5 * dt, n, s);
    kdk_energy(ctx, vel, mass, energy_out, s);
}

static pbh_status kdk_impl(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                           double dt, int32_t steps, double r_in, double r_out, double theta,
                           double eps, double* energy_out, hipStream_t s, bool graph) {
    if (!ctx) return PBH_E_ARG;
    if (!pos || !vel || !mass || !energy_out || steps < 0 || !std::isfinite(dt))
        return fail(ctx, PBH_E_ARG, "bad kdk arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->last = s;
    ctx->irr_rank_ok = false;   // every step rebuilds the tree
    pbh_status st = kdk_prepare(ctx, n, r_in, r_out, theta, eps, s);
    if (st != PBH_OK) return st;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, ctx->d.cnt + kCntKdkStep, 0ull);
    // initial force and energy
    kdk_force(ctx, pos, mass, theta, eps, s);
    kdk_energy(ctx, vel, mass, energy_out, s);
    if (!graph) {
        for (int k = 0; k < steps; ++k) kdk_step(ctx, pos, vel, mass, dt, theta, eps, energy_out, s);
    } else if (steps > 0) {
        const std::vector<double> key = {dt, theta, eps, r_in, r_out, (double)(uintptr_t)pos,
                                         (double)(uintptr_t)vel, (double)(uintptr_t)mass,
                                         (double)(uintptr_t)energy_out, (double)ctx->params.prec,
                                         (double)ctx->params.leaf_size, (double)ctx->params.n_crit,
                                         (double)ctx->params.key_bits, (double)ctx->alloc_gen,
                                         (double)(uintptr_t)ctx->k_acc, (double)n};
        if (!ctx->gexec || ctx->gkey != key) {
            if (ctx->gexec) { (void)hipGraphExecDestroy(ctx->gexec); ctx->gexec = nullptr; }
            if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
            hipStream_t cs = ctx->cap_stream;
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            kdk_step(ctx, pos, vel, mass, dt, theta, eps, energy_out, cs);
            HIP_TRY(hipStreamEndCapture(cs, &ctx->graph));
            HIP_TRY(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
            ctx->gkey = key;
        }
        for (int k = 0; k < steps; ++k) HIP_TRY(hipGraphLaunch(ctx->gexec, s));
    }
    ctx->built = true;   // the tree of the final positions
    ctx->built_pos = pos;
    ctx->built_mass = mass;
    return PBH_OK;
}

pbh_status pbh_kdk_graph(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                         double dt, int32_t steps, double r_in, double r_out, double theta,
                         double eps, double* energy_out, pbh_stream_t stream) {
    return kdk_impl(ctx, n, pos, vel, mass, dt, steps, r_in, r_out, theta, eps, energy_out,
                    (hipStream_t)stream, true);
}

pbh_status pbh_kdk_eager(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                         double dt, int32_t steps, double r_in, double r_out, double theta,
                         double eps, double* energy_out, pbh_stream_t stream) {
    return kdk_impl(ctx, n, pos, vel, mass, dt, steps, r_in, r_out, theta, eps, energy_out,
                    (hipStream_t)stream, false);
}

pbh_status pbh_set_timing(pbh_ctx* ctx, int32_t enable) {
    if (!ctx) return PBH_E_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    if (enable && !ctx->ev[0])
        for (auto& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
    ctx->timing = enable != 0;
    ctx->ev_build = ctx->ev_walk = ctx->ev_nbr = false;
    return PBH_OK;
}

static double event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
}

pbh_status pbh_get_stats(pbh_ctx* ctx, pbh_stats* out) {
    if (!ctx || !out) return PBH_E_ARG;
    std::memset(out, 0, sizeof(*out));
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    if (ctx->irr_err) {
        unsigned long long f = 0;
        HIP_TRY(hipMemcpy(&f, ctx->irr_err, sizeof(f), hipMemcpyDeviceToHost));
        out->error_flags = (int64_t)(f << 8);
    }
    if (!ctx->d.cnt) return PBH_OK;
    unsigned long long h[kNumCounters];
    HIP_TRY(hipMemcpy(h, ctx->d.cnt, sizeof(h), hipMemcpyDeviceToHost));
    out->n = ctx->cfg.n;
    out->n_clusters = ctx->cfg.n_clusters;
    out->n_nodes = (int64_t)h[kCntNodes];
    out->n_leaves = (int64_t)h[kCntLeaves];
    out->n_groups = (int64_t)h[kCntGroups];
    out->max_level = (int64_t)h[kCntMaxLevel];
    out->n_pn = (int64_t)h[kCntPN];
    out->n_pp_far = (int64_t)h[kCntFar];
    out->n_pp_near = (int64_t)h[kCntNear];
    out->lane_slots_pn = (int64_t)h[kCntSlotPN];
    out->lane_slots_far = (int64_t)h[kCntSlotFar];
    out->lane_slots_near = (int64_t)h[kCntSlotNear];
    out->error_flags |= (int64_t)h[kErr];
    if (ctx->ev_build) out->ms_build = event_ms(ctx->ev[0], ctx->ev[1]);
    if (ctx->ev_walk) out->ms_walk = event_ms(ctx->ev[2], ctx->ev[3]);
    if (ctx->ev_nbr) out->ms_nbr = event_ms(ctx->ev[4], ctx->ev[5]);
    return PBH_OK;
}

pbh_status pbh_debug_groups(pbh_ctx* ctx, int64_t cap, int32_t* begin, int32_t* count,
                            double* box, int64_t* n_groups) {
    if (!ctx) return PBH_E_ARG;
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "no successful build");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    unsigned long long G = 0;
    HIP_TRY(hipMemcpy(&G, ctx->d.cnt + kCntGroups, sizeof(G), hipMemcpyDeviceToHost));
    if (n_groups) *n_groups = (int64_t)G;
    if (!begin && !count && !box) return PBH_OK;
    if (cap < (int64_t)G) return fail(ctx, PBH_E_ARG, "group buffer too small");
    if (begin) HIP_TRY(hipMemcpy(begin, ctx->d.g.begin, sizeof(int32_t) * G, hipMemcpyDeviceToHost));
    if (count) HIP_TRY(hipMemcpy(count, ctx->d.g.count, sizeof(int32_t) * G, hipMemcpyDeviceToHost));
    if (box) {
        std::vector<double> lo(3 * G), hi(3 * G);
        HIP_TRY(hipMemcpy(lo.data(), ctx->d.g.lo, sizeof(double) * 3 * G, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hi.data(), ctx->d.g.hi, sizeof(double) * 3 * G, hipMemcpyDeviceToHost));
        for (unsigned long long g = 0; g < G; ++g)
            for (int k = 0; k < 3; ++k) {
                box[6 * g + k] = lo[3 * g + k];
                box[6 * g + 3 + k] = hi[3 * g + k];
            }
    }
    return PBH_OK;
}

pbh_status pbh_debug_valu_probe(pbh_ctx* ctx, int64_t blocks, int32_t iters, float* out,
                                pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (blocks < 1 || blocks > (1ll << 30) || iters < 0 || !out)
        return fail(ctx, PBH_E_ARG, "need 1 <= blocks <= 2^30, iters >= 0 and out");
    HIP_TRY(hipSetDevice(ctx->device));
    launch_valu_probe(blocks, iters, out, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return PBH_OK;
}

pbh_status pbh_debug_series_log(pbh_ctx* ctx, int64_t n, const double* x, double* y,
                                pbh_stream_t stream) {
    if (!ctx) return PBH_E_ARG;
    if (n < 0 || n >= (1ll << 40) || (n > 0 && (!x || !y)))
        return fail(ctx, PBH_E_ARG, "need 0 <= n < 2^40 and x, y");
    HIP_TRY(hipSetDevice(ctx->device));
    launch_series_log(n, x, y, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return PBH_OK;
}

pbh_status pbh_debug_wave_log(pbh_ctx* ctx, uint64_t* walk, uint64_t* nbr, int64_t cap,
                                         int64_t* n_walk, int64_t* n_nbr) {
    if (!ctx || !ctx->d.wave_log) return PBH_E_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    const int64_t gw = walk_grid(ctx, ctx->params.prec == PBH_MIXED);
    const int64_t gn = ctx->grid_mixed;
    if (n_walk) *n_walk = gw;
    if (n_nbr) *n_nbr = gn;
    if (walk && cap >= gw)
        HIP_TRY(hipMemcpy(walk, ctx->d.wave_log, 16 * gw, hipMemcpyDeviceToHost));
    if (nbr && cap >= gn)
        HIP_TRY(hipMemcpy(nbr, ctx->d.wave_log_nbr, 16 * gn, hipMemcpyDeviceToHost));
    return PBH_OK;
}

pbh_status pbh_walk_clock(pbh_ctx* ctx, double* mhz) {
    if (!ctx || !mhz) return PBH_E_ARG;
    const int64_t gw = ctx->last_walk_grid;
    if (gw <= 0 || !ctx->d.wave_log) return fail(ctx, PBH_E_STATE, "no walk yet");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    std::vector<uint64_t> lg(2 * gw), cy(gw);
    HIP_TRY(hipMemcpy(lg.data(), ctx->d.wave_log, 16 * gw, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(cy.data(), ctx->d.wave_cyc, 8 * gw, hipMemcpyDeviceToHost));
    int wall_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device));
    double ticks = 0.0, cycles = 0.0;
    for (int64_t b = 0; b < gw; ++b) {
        ticks += (double)lg[2 * b + 1];
        cycles += (double)cy[b];
    }
    if (wall_khz <= 0 || ticks <= 0.0) return fail(ctx, PBH_E_STATE, "no clock record");
    *mhz = cycles / (ticks / (1e3 * wall_khz)) / 1e6;
    return PBH_OK;
}

pbh_status pbh_debug_herm_first_steps(pbh_ctx* ctx, int64_t cap, int64_t* ticks, int64_t* n_out) {
    if (!ctx) return PBH_E_ARG;
    const auto& h = ctx->herm;
    if (h.last_n < 1) return fail(ctx, PBH_E_STATE, "no Hermite integration yet");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    if (n_out) *n_out = h.last_n;
    if (!ticks) return PBH_OK;
    if (cap < h.last_n) return fail(ctx, PBH_E_ARG, "buffer too small");
    HIP_TRY(hipMemcpy(ticks, h.dt0, sizeof(int64_t) * h.last_n, hipMemcpyDeviceToHost));
    return PBH_OK;
}

pbh_status pbh_debug_tree(pbh_ctx* ctx, int32_t* order, uint64_t* keys, int64_t cap,
                          int64_t* nodes_i, double* nodes_d, int64_t* n_nodes) {
    if (!ctx) return PBH_E_ARG;
    if (!ctx->built) return fail(ctx, PBH_E_STATE, "no successful build");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->last));
    const int64_t n = ctx->cfg.n;
    unsigned long long h[kNumCounters];
    HIP_TRY(hipMemcpy(h, ctx->d.cnt, sizeof(h), hipMemcpyDeviceToHost));
    const int64_t nn = (int64_t)h[kCntNodes];
    if (n_nodes) *n_nodes = nn;
    if (order) HIP_TRY(hipMemcpy(order, ctx->d.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (keys) HIP_TRY(hipMemcpy(keys, ctx->d.keys, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    if (!nodes_i && !nodes_d) return PBH_OK;
    if (cap < nn) return fail(ctx, PBH_E_ARG, "node buffer too small");
    std::vector<WNode> w(nn);
    std::vector<Mom64> q(nn);
    std::vector<int32_t> lvl(nn);
    HIP_TRY(hipMemcpy(w.data(), ctx->d.node, sizeof(WNode) * nn, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(q.data(), ctx->d.q64, sizeof(Mom64) * nn, hipMemcpyDeviceToHost));
    std::vector<uint64_t> lk(nn);
    HIP_TRY(hipMemcpy(lk.data(), ctx->d.lvl_key, sizeof(uint64_t) * nn, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < nn; ++k) {
        if (nodes_i) {
            nodes_i[4 * k] = w[k].begin;
            nodes_i[4 * k + 1] = w[k].count;
            nodes_i[4 * k + 2] = w[k].nchild;
            nodes_i[4 * k + 3] = (int64_t)lk[k];
        }
        if (nodes_d) {
            double* o = nodes_d + 16 * k;
            o[0] = q[k].M;
            for (int j = 0; j < 3; ++j) {
                o[1 + j] = w[k].com[j];
                o[10 + j] = w[k].lo[j];
                o[13 + j] = w[k].hi[j];
            }
            o[4] = q[k].qxx; o[5] = q[k].qyy; o[6] = q[k].qzz;
            o[7] = q[k].qxy; o[8] = q[k].qxz; o[9] = q[k].qyz;
        }
    }
    return PBH_OK;
}

}  // extern "C"
