// pbh_internal.hpp -- device data layout and kernel launchers of libpbh.
//
// Memory layout in HBM (all device arrays owned by the context):
//   particles, sorted by key:  x, y, z, m  FP64 SoA [n];  perm int32 [n]
//                              (sorted position -> caller index)
//   keys                       uint64 [n] (cluster id above D Morton bits/axis)
//   nodes (breadth-first, children of a node contiguous, levels contiguous):
//     WNode  [cap] 96 B  box lo/hi, centre of mass (FP64), rcrit^2, begin,
//                        count, first child, child count -- the walk's view
//     q64    [cap] 64 B  M and traceless quadrupole (FP64 master copy)
//     q32    [cap] 32 B  the same in FP32 for the mixed-precision walk
//   groups: begin, count, root node, cluster (int32) and tight box (FP64)
//   clusters: ClusterParams per cluster (radii and potential coefficients)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pbh {

constexpr int kMaxLevels = 22;     // levels 0..21
constexpr int kWave = 64;

// device error-flag bits (counters[kErr])
enum : unsigned long long {
    kErrNbrOverflow = 1ull,   // neighbour entry dropped: beyond nbr_cap
    kErrWalkStack = 2ull,     // walk traversal stack full
    kErrNodeCap = 4ull,       // node capacity exceeded in the build
    kErrNonFinite = 8ull,     // NaN/Inf in positions or masses
    kErrNbrStack = 16ull,     // neighbour traversal stack full
    kErrStale = 32ull,        // pos or mass changed since the build (force call)
};

// slots of the device counter array
// kCntSlot*: wave-instruction slots of the walk's evaluation loops (64 lanes
// per loop iteration), beside the interactions they carried (kCntPN, ...)
enum { kCntNodes = 0, kCntPN = 1, kCntFar = 2, kCntNear = 3, kCntNbrTotal = 4, kErr = 5,
       kCntSlotPN = 6, kCntSlotFar = 7, kCntSlotNear = 8,
       kCntMaxLevel = 9, kCntLeaves = 10, kCntGroups = 12, kCntFill = 13, kNumCounters = 16 };

struct alignas(16) WNode {
    double lo[3];
    double hi[3];
    double com[3];
    double rcrit2;       // (l/theta + delta)^2 of the current force call
    int32_t begin;       // first sorted particle
    int32_t count;       // particles
    int32_t first_child; // breadth-first index of the first child (-1 for a leaf)
    int32_t nchild;      // 0 for a leaf
};
static_assert(sizeof(WNode) == 96, "WNode layout");

struct alignas(16) Mom64 { double M, qxx, qyy, qzz, qxy, qxz, qyz, pad; };
struct alignas(16) Mom32 { float M, qxx, qyy, qzz, qxy, qxz, qyz, pad; };

// Per-cluster constants of the changeover split (computed on the host).
// Regular potential on [r_in, r_out):
//   Phi_R(s) = c0 - d0 / s + l1 * ln(s) + t * (e2 + t * (e3 + ... + t * e7)),
//   t = s / (r_out - r_in); beyond r_out -1/s; below r_in `inner`.
struct alignas(16) ClusterParams {
    double r_in, r_out, rout2, inv_delta;
    double c0, d0, l1, inner;
    double e[6];   // e2..e7
    double rlist, rlist2;   // neighbour-list radius R = r_out + r_buff and R^2
    float f_r_in, f_r_out, f_inv_delta, f_c0;
    float f_d0, f_l1, f_inner, f_pad;
    float f_e[6];
    float f_pad2[2];
};

struct GroupArrays {
    int32_t* begin = nullptr;
    int32_t* count = nullptr;
    int32_t* root = nullptr;
    int32_t* cluster = nullptr;
    double* lo = nullptr;  // [G][3]
    double* hi = nullptr;  // [G][3]
};

struct BuildCfg {
    int64_t n = 0;
    int32_t n_clusters = 1;
    int32_t D = 21;          // Morton bits per axis
    int32_t cbits = 0;       // cluster-id bits above the Morton bits
    int32_t n_leaf = 16;
    int32_t n_crit = 64;
    int64_t node_cap = 0;
    int64_t n_groups = 0;
    // workgroups of the moment pass per level (0: sized for the node capacity).
    // Taken from the previous build's level sizes; any size is correct (the
    // kernel strides), a good guess avoids dispatching thousands of idle groups.
    int32_t mom_grid[32] = {0};
    // levels [mom_hi+1, D] and [0, mom_lo] are each done by one workgroup that
    // walks its levels in order (they held few or no nodes last time);
    // mom_hi = D and mom_lo = -1 launch every level on its own
    int32_t mom_hi = 21, mom_lo = -1;
};

// Scratch and arrays of one built forest.
// The first group pass counts groups per box-size octave with global atomics.
// A single cluster puts all of them on a few bins; spreading them over
// `reps` copies of the histogram (summed afterwards) removes the contention.
inline int group_hist_reps(int n_clusters) {
    return n_clusters >= 256 ? 1 : (n_clusters > 4 ? 256 / n_clusters : 64);
}

// Staging rows are interleaved by 64 particles: entry t of sorted particle i
// sits at stage_index(i, t, cap). The walk's lanes append entries with
// similar t at the same time, and the copy kernel's wave reads entry t of 64
// consecutive particles from one 256-byte segment; rows laid end to end
// would put every lane of a wave on its own 2 KB-strided line.
constexpr int kStageStride = 64;
__host__ __device__ inline int64_t stage_index(int64_t i, int t, int cap) {
    return (i / kStageStride) * kStageStride * cap + (int64_t)t * kStageStride + (i % kStageStride);
}

// One particle of the irregular-force pass, packed in key order (64 B).
struct alignas(64) IrrRec {
    double x, y, z, m, vx, vy, vz, pad;
};

struct Dev {
    // particles
    double *x = nullptr, *y = nullptr, *z = nullptr, *m = nullptr;
    int32_t* perm = nullptr;
    uint64_t* keys = nullptr;
    uint64_t* keys_alt = nullptr;
    int32_t* vals_alt = nullptr;
    // clusters
    int64_t* cl_off = nullptr;       // [C+1]
    double* cl_box = nullptr;        // [C][6] lo xyz, hi xyz
    int32_t* blk_cluster = nullptr;  // bbox/key block table: cluster of block
    int64_t* blk_range = nullptr;    // [nblk][2]
    double* blk_part = nullptr;      // [nblk][6] partial boxes
    int32_t* blk_bad = nullptr;      // [nblk] non-finite flags
    ClusterParams* cparams = nullptr;
    // topology scratch (pre-order)
    int32_t* p_first = nullptr;      // [n] first level started at i
    int32_t* p_nn = nullptr;         // [n+1] nodes started at i, then exclusive scan
    int32_t* pre_begin = nullptr;    // [cap]
    int32_t* pre_count = nullptr;
    int32_t* pre_level = nullptr;
    int32_t* pre_nchild = nullptr;
    uint64_t* lvl_key = nullptr;     // [cap] level as a sort key
    int32_t* lvl_val = nullptr;      // [cap] pre-order index
    uint64_t* lvl_key_alt = nullptr;
    int32_t* bfs2pre = nullptr;      // [cap]
    int32_t* pre2bfs = nullptr;      // [cap]
    int32_t* lvl_off = nullptr;      // [kMaxLevels+1] breadth-first level offsets
    // nodes (breadth-first)
    WNode* node = nullptr;
    Mom64* q64 = nullptr;
    Mom32* q32 = nullptr;
    // groups (capacity n: the count is data dependent, kept in cnt[kCntGroups])
    GroupArrays g;
    int32_t* g_flag = nullptr;   // [n+1] 1 at the first particle of a group, then scanned
    int32_t* g_len = nullptr;    // [n] group length at its first particle
    unsigned* g_hist = nullptr;  // [reps][C][128] octave histograms of first-pass group sizes
    double* cl_S = nullptr;      // [C] group size limit per cluster
    // generic scan scratch
    int64_t* scan_tmp = nullptr;
    int64_t scan_tmp_len = 0;
    // radix-sort histogram scratch
    int64_t* rs_hist = nullptr;
    int64_t rs_hist_len = 0;
    // neighbour counts
    int32_t* nbr_cnt = nullptr;
    // neighbour staging: the walk writes every particle's list into a row of
    // stage_cap entries (per-copy sub-rows in split groups); stage_k[p] is the
    // group's copy count, or 0 when the group's lists are left to the fill pass,
    // whose groups are listed in fill_list[0 .. cnt[kCntFill])
    int32_t* nbr_stage = nullptr;   // layout: stage_index()
    int64_t nbr_stage_len = 0;
    int8_t* stage_k = nullptr;     // [n]
    int32_t* fill_list = nullptr;  // [G]
    // irregular force: caller index -> key position, key-order particle records
    int32_t* irr_rank = nullptr;
    IrrRec* irr_rec = nullptr;
    int64_t irr_len = 0;
    // core quantities: distance keys and their sort scratch, block sums, results
    uint64_t* core_keys = nullptr;
    uint64_t* core_keys_alt = nullptr;
    int32_t* core_vals = nullptr;
    int32_t* core_vals_alt = nullptr;
    double* core_bsum = nullptr;
    double* core_stats = nullptr;          // [16]
    unsigned long long* core_cnt = nullptr; // [2]: N_core, error flags
    int64_t core_len = 0;
    double* core_rho = nullptr;            // [core_rho_len] when the caller passes none
    int64_t core_rho_len = 0;
    // walk stacks
    int32_t* stack = nullptr;
    int64_t stack_len = 0;
    // counters
    unsigned long long* cnt = nullptr;
    // group work queues: walk [0, 8), neighbour count [8, 16), neighbour fill [16, 24)
    unsigned long long* queues = nullptr;
    // per persistent workgroup of the last walk / neighbour count: groups, clock ticks
    unsigned long long* wave_log = nullptr;
    unsigned long long* wave_log_nbr = nullptr;
    unsigned long long* wave_cyc = nullptr;   // walk: core clock cycles per workgroup
};

// ---- launchers (all enqueue on `s`, none waits) ----
// scan.hip / sort.hip
int64_t scan_tmp_need(int64_t n);
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s);
int64_t radix_hist_need(int64_t n);
// Stable LSD radix sort of (key, val) on bits [0, nbits). The input is in
// (keys, vals); the result ends in (keys, vals), or with to_alt in (keys_alt,
// vals_alt), the other pair being scratch of the same size. The passes
// alternate between the pairs, so the result needs no final copy when the
// pass count (radix_passes) is even and to_alt is false, or odd and to_alt is
// true. With vals_are_iota the input values are taken to be 0..n-1 (vals not
// read). If n_dev is given the element count is min(n, *n_dev), read on the
// device.
int radix_passes(int nbits);
void radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                      int64_t n, int nbits, int64_t* hist, int64_t* scan_tmp, hipStream_t s,
                      bool vals_are_iota, const int32_t* n_dev = nullptr, bool to_alt = false);

// threads per workgroup of the per-level moment kernels (the host sizes their grids)
constexpr int kMomT = 64;   // 32, 128 and 256 built slower at 2^20

// build.hip
void launch_bbox(Dev& d, const BuildCfg& c, const double* pos, const double* mass, int nblk,
                 hipStream_t s);
void launch_keys(Dev& d, const BuildCfg& c, const double* pos, int nblk, hipStream_t s);
// the key sort of a build: (keys, perm) sorted by key, perm the caller order
void launch_key_sort(Dev& d, const BuildCfg& c, hipStream_t s);
void launch_gather(Dev& d, const BuildCfg& c, const double* pos, const double* mass, hipStream_t s);
void launch_topology(Dev& d, const BuildCfg& c, hipStream_t s);
void launch_moments(Dev& d, const BuildCfg& c, hipStream_t s);
void launch_groups(Dev& d, const BuildCfg& c, hipStream_t s);

// walk.hip
struct WalkCfg {
    double theta;
    double eps;
    int mixed;
    int tile = 64;         // LDS tile capacity (64, 96 or 128)
    int max_copies = 64;   // most sub-wave copies of a small group
    const double* cpos = nullptr;    // caller's arrays for the stale-input check, or null
    const double* cmass = nullptr;
    int grid;
    int stack_cap;
    int count_nbr;   // also count neighbours per particle into Dev::nbr_cnt
    int stage_cap;   // > 0: stage neighbour indices in Dev::nbr_stage rows of this size
};
void launch_rcrit(Dev& d, const BuildCfg& c, double theta, hipStream_t s);
void launch_walk(Dev& d, const BuildCfg& c, const WalkCfg& w, double* acc, double* pot,
                 hipStream_t s);
int walk_blocks_per_cu(int mixed, int tile);

// nbr.hip
void launch_nbr_copy(Dev& d, const BuildCfg& c, int stage_cap, const int64_t* off, int32_t* idx,
                     int64_t cap, hipStream_t s);
void launch_nbr_fill(Dev& d, const BuildCfg& c, int grid, int stack_cap, const int64_t* off,
                     int32_t* idx, int64_t cap, hipStream_t s);

// irr.hip: irregular force, jerk and potential from neighbour lists
enum : unsigned long long {
    kIrrBadIndex = 1ull,     // a list entry outside [0, n)
    kIrrBadOffsets = 2ull,   // off[i] < 0, off[i+1] < off[i] or off[i+1] > cap
    kIrrBadTarget = 4ull,    // a target index outside [0, n)
};
struct IrrParams {
    int64_t n = 0;              // particles (caller order)
    int64_t n_tgt = 0;          // targets of this launch
    const int32_t* tgt = nullptr;    // target caller indices (outputs compact), or null = all
    const int32_t* order = nullptr;  // processing order of all targets (key order), or null
    // key-order records: perm [n] (key position -> caller index), rank [n]
    // (caller index -> key position, the inverse of perm) and rec [n], written
    // by the pre-passes; null rec: gather from pos/vel/mass directly
    const int32_t* perm = nullptr;
    int32_t* rank = nullptr;
    IrrRec* rec = nullptr;
    bool rank_fresh = true;          // recompute rank from perm (false: it already holds the inverse)
    const double* pos = nullptr;     // [n][3]
    const double* vel = nullptr;     // [n][3] (jerk only)
    const double* mass = nullptr;    // [n]
    const int64_t* off = nullptr;    // [n+1]
    const int32_t* idx = nullptr;    // [cap]
    int64_t cap = 0;
    int C = 1;                        // clusters; > 1: cluster of i from cl_off, constants from cps
    const int64_t* cl_off = nullptr;  // [C+1] caller-order cluster offsets
    const ClusterParams* cps = nullptr;
    ClusterParams cp0;                // constants when C == 1
    double eps2 = 0.0;
    double* acc = nullptr;            // outputs ([n_tgt] or [n] slots)
    double* jerk = nullptr;           // may be null
    double* pot = nullptr;            // may be null
    unsigned long long* err = nullptr;   // kIrr* flag bits (OR)
};
void launch_irregular(const IrrParams& p, hipStream_t s);
void launch_series_log(int64_t n, const double* x, double* y, hipStream_t s);   // debug export

// core.hip: core quantities from the 6 nearest neighbours of a sample
enum : unsigned long long {
    kCoreBadSample = 1ull,   // a sample index outside [0, n)
    kCoreStackFull = 2ull,   // traversal stack of a nearest-neighbour search full
};
struct CoreLaunch {
    int64_t n = 0, ns = 0;
    const int32_t* sample = nullptr;   // [ns] caller indices
    const WNode* node = nullptr;
    const double *x = nullptr, *y = nullptr, *z = nullptr;   // sorted coordinates
    const int32_t* perm = nullptr;
    int32_t* rank = nullptr;           // [n] written here
    const double* pos = nullptr;       // [n][3] caller order
    const double* mass = nullptr;      // [n] caller order
    double* rho = nullptr;             // [ns] out
    double* stats = nullptr;           // [9] x_d, rho_core, r_c, N_core, r_h, R_min, dT_min
    uint64_t* keys = nullptr;          // [n] scratch
    uint64_t* keys_alt = nullptr;
    int32_t* vals = nullptr;
    int32_t* vals_alt = nullptr;
    int64_t* hist = nullptr;           // radix-sort scratch of the build
    int64_t* scan_tmp = nullptr;
    double* bsum = nullptr;            // [core_bsum_len(n)]
    unsigned long long* ncore = nullptr;
    unsigned long long* err = nullptr;
    double eta = 0.02;
};
void launch_core(const CoreLaunch& c, hipStream_t s);
int64_t core_bsum_len(int64_t n);

// herm.hip: Hermite integration of F_I with block steps over one regular step
constexpr int kHermK = 40;   // block steps dt_max / 2^k, k <= kHermK; times in ticks of dt_max / 2^kHermK
enum { kHermTn = 0, kHermNact = 1, kHermSteps = 2, kHermKmax = 3, kHermDone = 4, kHermBlocks = 5,
       kHermCtl = 6 };
// level bookkeeping, two slots by block parity: bucket counts, appends of the
// last corrector, block time, k* of the last block
enum { kLevCnt = 0, kLevNew = 128, kLevT = 256, kLevKs = 258, kLevLen = 260 };
struct HermParams {
    int64_t n = 0;
    double* x = nullptr;         // [n][3] positions (caller's, updated in place)
    double* v = nullptr;         // [n][3] velocities (caller's, updated in place)
    double* a = nullptr;         // [n][3] F_I at tau_i
    double* j = nullptr;         // [n][3] dF_I/dt at tau_i
    double* xp = nullptr;        // [n][3] predicted
    double* vp = nullptr;
    const double* fr = nullptr;  // [n][3] regular force (step criterion), or null
    int64_t* tau = nullptr;      // [n] ticks
    int64_t* dt = nullptr;       // [n] ticks
    int64_t* dt0 = nullptr;      // [n] first step of the regular step (ticks), or null
    int32_t* act = nullptr;      // [n] active list
    unsigned long long* ctl = nullptr;   // [kHermCtl]
    unsigned long long* lev = nullptr;   // [kLevLen]
    int32_t* bucket = nullptr;           // [kHermK + 1][n] particles by level
    uint32_t* slot = nullptr;            // [n] per-item level and rank (bucket moves)
    unsigned long long* done_host = nullptr;   // host-coherent pinned flag, set once all are at tend
    const int64_t* off = nullptr;        // neighbour lists (members are predicted with the active)
    const int32_t* idx = nullptr;
    int64_t cap = 0;
    unsigned long long tend = 0; // ticks of one regular step: 2^(kHermK + 2)
    double unit = 0.0;           // seconds per tick: T / 2^(kHermK + 2)
    double dtmax = 0.0;          // T / 4
    double eta = 0.02;
};
// first steps (eq. dt with the computed second and third derivatives of F_I;
// ip: masses, radii and softening of the irregular force, and its error word)
void launch_herm_start(const HermParams& p, const IrrParams& ip, hipStream_t s);
// one block: front (next time, active list, prediction), then the irregular
// force of the active list with the corrector; parity = block number & 1
void launch_herm_front(const HermParams& p, int parity, hipStream_t s);
void launch_herm_force_correct(const HermParams& p, const IrrParams& ip, int parity, hipStream_t s);
void launch_add(int64_t n, const double* a, const double* b, double* out, hipStream_t s);

// kdk.hip
void launch_kick(double* vel, const double* acc, double h, int64_t n, hipStream_t s);
void launch_drift(double* pos, const double* vel, double dt, int64_t n, hipStream_t s);
void launch_energy(const double* vel, const double* mass, const double* pot, int64_t n,
                   double* partial, int nblk, double* out, hipStream_t s);
void launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// one wave per block, 32 * iters + 32 VALU instructions per wave (counted in
// the kernel's gfx950 assembly): a known count for instruction counters
void launch_valu_probe(int64_t blocks, int iters, float* out, hipStream_t s);

}  // namespace pbh
