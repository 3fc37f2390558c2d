// irr.hip -- irregular (neighbour) force, its time derivative and the
// irregular potential from neighbour lists, in FP64 (gfx950).
//
// For a target i with list N(i) of caller indices, d = x_j - x_i,
// u = v_j - v_i and s^2 = |d|^2 + eps^2 (Arnold, Baumgardt & Wang 2021,
// Section 2.1, eq. fi, eq. fidot, eq. duncan, eq. duncan2):
//   F_I     = sum_{j in N(i), j != i} m_j K(s) d / s^3
//   dF_I/dt = sum m_j { K(s) [u / s^3 - 3 (d.u) d / s^5] + (dK/dt) d / s^3 }
//   dK/dt   = -g'(x) (d.u) / (s (r_out - r_in)) on r_in <= s < r_out, else 0,
//             with x = (s - r_in)/(r_out - r_in), g'(x) = 140 x^3 (1 - x)^3
//   Phi_I   = sum m_j (-1/s - Phi_R(s))
// The jerk is the time derivative of F_I term by term (the printed eq. fidot
// drops m_j and K from its second term, and eq. duncan2 carries the opposite
// sign of dK/dt for K = 1 - g). Pairs with s >= r_out add nothing (K = 0), so
// any list that holds every j with r_ij < r_out gives the whole sums; lists of
// a larger search radius work unchanged.
//
// A group of kIrrLanes lanes per target: lane g sums list entries g,
// g + kIrrLanes, ... in order, and the group adds the lanes' partial sums in a
// fixed butterfly, so the sums do not depend on the route, the grid or the
// target order. A wave's list loads are then contiguous runs. For all targets
// (or a long target list) with a build of these n particles, a pre-pass packs
// every particle into a 64-byte record (x, y, z, m, vx, vy, vz) in the build's
// key order and stores each caller index's key rank; the targets of a wave are
// then consecutive in key order, and its gathers land in a spatially compact
// range of records that stays in cache. Otherwise (no build, or a short
// target list) the kernel gathers from the caller's arrays. A lane's entries
// are taken in batches whose loads issue together (a gather costs cache
// latency, not arithmetic). Lists, targets and offsets are range-checked: a
// bad entry is skipped and flagged, never dereferenced.
#include "irr_pair.hpp"
#include "pbh_internal.hpp"
#include "wave.hpp"

namespace pbh {

namespace {

// rank[perm[k]] = k: the key position of each caller index (once per build)
__global__ __launch_bounds__(256) void k_irr_rank(int64_t n, const int32_t* __restrict__ perm,
                                                  int32_t* __restrict__ rank) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) rank[perm[k]] = (int32_t)k;
}

// rec[rank[i]] = particle i (velocity only if given): the caller's arrays are
// read in order and each record is stored whole (64 bytes, aligned)
__global__ __launch_bounds__(256) void k_irr_pack(int64_t n, const int32_t* __restrict__ rank,
                                                  const double* __restrict__ pos,
                                                  const double* __restrict__ vel,
                                                  const double* __restrict__ mass, IrrRec* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    IrrRec r;
    r.x = pos[3 * i];
    r.y = pos[3 * i + 1];
    r.z = pos[3 * i + 2];
    r.m = mass[i];
    r.vx = vel ? vel[3 * i] : 0.0;
    r.vy = vel ? vel[3 * i + 1] : 0.0;
    r.vz = vel ? vel[3 * i + 2] : 0.0;
    r.pad = 0.0;
    rec[rank[i]] = r;
}

template <bool JERK, bool POT>
__device__ inline void store_sums(const IrrParams& p, int64_t slot, const IrrSums& S) {
    p.acc[3 * slot] = S.ax;
    p.acc[3 * slot + 1] = S.ay;
    p.acc[3 * slot + 2] = S.az;
    if (JERK) {
        p.jerk[3 * slot] = S.jx;
        p.jerk[3 * slot + 1] = S.jy;
        p.jerk[3 * slot + 2] = S.jz;
    }
    if (POT) p.pot[slot] = S.ph;
}

// Key-order route, records loaded cooperatively. A lane's pair needs one
// 64-byte record (32 bytes without the jerk); loaded by its own lane as
// 16-byte pieces, the 64 scattered lanes of each load cost the vector L1 64
// separate accesses. Here CH = 4 (or 2) neighbouring lanes load the CH pieces
// of one record together, one contiguous access per record, and the pieces
// reach the lane that owns the pair through a 64-record slot of LDS per wave.
// Each lane still sums its own entries in list order, so the sums equal those
// of the per-lane route bit for bit. Every lane of the wave runs the loop until
// no lane has entries left (the loads serve other lanes' pairs); lanes without
// a target or past their list take part with no record of their own.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte piece

// Entries per lane and round on the key-order route: 2 with the jerk (120
// registers, 4 waves per SIMD; 3 entries need 136 and drop to 3 waves), 6 for
// the force alone (94 registers, 5 waves). Measured at 2^20 against 1 to 3
// and 2 to 6.
template <bool JERK>
constexpr int coop_lane_batch() { return JERK ? 2 : 6; }

template <bool JERK>
struct CoopPieces {
    static constexpr int B = coop_lane_batch<JERK>();
    static constexpr int CH = JERK ? 4 : 2;   // 16-byte pieces per record
    static constexpr int RPI = 64 / CH;       // records per load instruction
    u32x4 piece[B][CH];
};

// Issues every record load of one round: for each entry u, the pieces
// lane % CH of the records of lanes RPI k + lane / CH (k < CH). rk holds the
// key rank of each lane's record, or 0 where the lane has no pair: those
// slots all load record 0, one shared line per instruction, and are ignored.
template <bool JERK>
__device__ inline void coop_load(const IrrRec* __restrict__ rec, const int32_t* rk, int lane,
                                 CoopPieces<JERK>& P) {
    using C = CoopPieces<JERK>;
    const int c = lane % C::CH;
    int rt[C::B][C::CH];
#pragma unroll
    for (int u = 0; u < C::B; ++u)
#pragma unroll
        for (int k = 0; k < C::CH; ++k)
            rt[u][k] = __builtin_amdgcn_ds_bpermute((C::RPI * k + lane / C::CH) << 2, rk[u]);
#pragma unroll
    for (int u = 0; u < C::B; ++u)
#pragma unroll
        for (int k = 0; k < C::CH; ++k)
            P.piece[u][k] = reinterpret_cast<const u32x4*>(rec + rt[u][k])[c];
}

// Entry u's record of this lane, passed through the wave's LDS slot.
template <bool JERK>
__device__ inline PartJ coop_take(const CoopPieces<JERK>& P, int u, IrrRec* xch, int lane) {
    using C = CoopPieces<JERK>;
    const int c = lane % C::CH;
#pragma unroll
    for (int k = 0; k < C::CH; ++k)
        reinterpret_cast<u32x4*>(xch + C::RPI * k + lane / C::CH)[c] = P.piece[u][k];
    __builtin_amdgcn_wave_barrier();
    const PartJ q = load_rec<JERK>(xch, lane);   // a lane without a pair reads a slot it ignores
    __builtin_amdgcn_wave_barrier();             // the slot is rewritten for the next entry
    return q;
}

template <bool JERK, bool POT, bool MULTI>
__device__ inline bool irr_sums_coop(const IrrParams& p, int64_t i, bool have, int g, IrrSums& S,
                                     unsigned long long& bad, IrrRec* xch) {
    const int lane = (int)(threadIdx.x & 63);
    const ClusterParams* cp = &p.cp0;
    int64_t b = 0, e = 0;
    const bool valid = have && target_setup(p, i, cp, b, e, bad);
    if (g != 0) bad = 0;   // target and offset flags once per group
    const IrrK K = irr_constants(MULTI ? *cp : p.cp0);
    PartJ me = {};
    if (valid) me = load_rec<JERK>(p.rec, p.rank[i]);
    constexpr int B = coop_lane_batch<JERK>();
    constexpr int64_t STEP = (int64_t)kIrrLanes * B;
    int64_t m = b + g;
    if (!valid) m = e = 0;
    // While any lane of the wave has entries left, some list holds an entry
    // (so idx[0] exists) and some target is valid (so rank[0] and rec[0] do):
    // a lane without an entry loads those, and its loads stay in bounds. A
    // lane with entries clamps to its own last one, e - 1 in [b, cap).
    const int64_t last = m < e ? e - 1 : 0;
    while (__builtin_amdgcn_ballot_w64(m < e) != 0) {
        int32_t jv[B], rk[B];
        bool ok[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int64_t q = m + (int64_t)kIrrLanes * u;
            jv[u] = p.idx[q < e ? q : last];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const bool live = m + (int64_t)kIrrLanes * u < e;
            const bool inr = (uint64_t)(int64_t)jv[u] < (uint64_t)p.n;
            if (live && !inr) bad |= kIrrBadIndex;
            ok[u] = live && inr && jv[u] != i;
            rk[u] = p.rank[ok[u] ? jv[u] : 0];
            if (!ok[u]) rk[u] = 0;
        }
        CoopPieces<JERK> P;
        coop_load<JERK>(p.rec, rk, lane, P);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const PartJ q = coop_take<JERK>(P, u, xch, lane);
            if (ok[u]) pair_irr<JERK, POT>(K, p.eps2, me, q, S);
        }
        m += STEP;
    }
    S.ax = group_sum(S.ax);
    S.ay = group_sum(S.ay);
    S.az = group_sum(S.az);
    if (JERK) {
        S.jx = group_sum(S.jx);
        S.jy = group_sum(S.jy);
        S.jz = group_sum(S.jz);
    }
    if (POT) S.ph = group_sum(S.ph);
    return valid;
}

// Blocks (of 256 / kIrrLanes = 32 key-order targets) per XCD chunk: 512 targets
// (chunks of 4 to 128 blocks measured at 2^20; 8 and 16 were fastest).
constexpr unsigned kIrrChunk = 16;

// One target k (a lane group, lane g of it): the group's sums over its list,
// stored at its output slot by lane 0.
template <bool JERK, bool POT, bool SORTED, bool MULTI>
__device__ inline void irr_target(const IrrParams& p, int64_t k, int g) {
    unsigned long long bad = 0;
    const int64_t i = p.tgt ? (int64_t)p.tgt[k] : (p.order ? (int64_t)p.order[k] : k);
    IrrSums S;
    const bool valid = irr_sums_lanes<JERK, POT, SORTED, MULTI>(p, i, g, S, bad);
    if (g == 0 && (valid || p.tgt)) store_sums<JERK, POT>(p, p.tgt ? k : i, S);   // no slot of its own otherwise
    if (bad) atomicOr(p.err, bad);
}

template <bool JERK, bool POT, bool SORTED, bool MULTI>
__global__ __launch_bounds__(256) void k_irregular(IrrParams p) {
    const int g = threadIdx.x % kIrrLanes;   // lane groups never straddle a workgroup
    if (SORTED) {
        // key-order targets in chunks per XCD (cache locality and load balance);
        // every lane takes part in the cooperative loads, with a target or not
        __shared__ IrrRec xch[256 / 64][64];
        const unsigned blk = xcd_chunk_block(blockIdx.x, kIrrChunk);
        const int64_t k = ((int64_t)blk * blockDim.x + threadIdx.x) / kIrrLanes;
        const bool have = k < p.n_tgt;   // group-uniform
        unsigned long long bad = 0;
        const int64_t kk = have ? k : 0;
        const int64_t i = p.tgt ? (int64_t)p.tgt[kk] : (p.order ? (int64_t)p.order[kk] : kk);
        IrrSums S;
        const bool valid = irr_sums_coop<JERK, POT, MULTI>(p, i, have, g, S, bad, xch[threadIdx.x / 64]);
        if (have && g == 0 && (valid || p.tgt)) store_sums<JERK, POT>(p, p.tgt ? k : i, S);
        if (bad) atomicOr(p.err, bad);
        return;
    }
    // caller-array route: grid-stride
    const int64_t nt = p.n_tgt;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nt * kIrrLanes;
         v += (int64_t)gridDim.x * blockDim.x)
        irr_target<JERK, POT, SORTED, MULTI>(p, v / kIrrLanes, g);
}

template <bool JERK, bool POT, bool MULTI>
void launch_route(const IrrParams& p, hipStream_t s) {
    const int64_t nb = (p.n_tgt * kIrrLanes + 255) / 256;
    const dim3 block(256);
    // the key-order route has one work-item per (target, lane): it needs a grid
    // below 2^31 work-items; the caller-array route is grid-stride (same sums)
    const bool fits = p.n_tgt <= ((int64_t)1 << 31) / kIrrLanes - (int64_t)kQueues * kIrrChunk * 256;
    if (p.rec && fits) {   // grid padded to whole rounds of chunks over the XCDs
        const int64_t round = (int64_t)kQueues * kIrrChunk;
        const dim3 grid((unsigned)((nb + round - 1) / round * round));
        hipLaunchKernelGGL((k_irregular<JERK, POT, true, MULTI>), grid, block, 0, s, p);
    } else {
        const int64_t g = nb < (1 << 16) ? nb : (1 << 16);
        hipLaunchKernelGGL((k_irregular<JERK, POT, false, MULTI>), dim3((unsigned)g), block, 0, s, p);
    }
}

template <bool JERK, bool POT>
void launch_multi(const IrrParams& p, hipStream_t s) {
    if (p.C > 1) launch_route<JERK, POT, true>(p, s);
    else launch_route<JERK, POT, false>(p, s);
}

// the logarithm of the pair terms over an array (debug export)
__global__ __launch_bounds__(256) void k_series_log(int64_t n, const double* __restrict__ x,
                                                    double* __restrict__ y) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = log_pos(x[k]);
}

}  // namespace

void launch_series_log(int64_t n, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_series_log, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
}

void launch_irregular(const IrrParams& p, hipStream_t s) {
    if (p.n_tgt <= 0) return;
    if (p.rec) {
        const dim3 grid((unsigned)((p.n + 255) / 256));
        if (p.rank_fresh) hipLaunchKernelGGL(k_irr_rank, grid, dim3(256), 0, s, p.n, p.perm, p.rank);
        hipLaunchKernelGGL(k_irr_pack, grid, dim3(256), 0, s, p.n, (const int32_t*)p.rank, p.pos,
                           p.jerk ? p.vel : nullptr, p.mass, p.rec);
    }
    const bool jerk = p.jerk != nullptr, pot = p.pot != nullptr;
    if (jerk && pot) launch_multi<true, true>(p, s);
    else if (jerk) launch_multi<true, false>(p, s);
    else if (pot) launch_multi<false, true>(p, s);
    else launch_multi<false, false>(p, s);
}

}  // namespace pbh
