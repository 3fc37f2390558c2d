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
// One lane per target, its list summed in list order. For all targets (or a
// long target list) with a build of these n particles, a pre-pass packs every
// particle into a 64-byte record (x, y, z, m, vx, vy, vz) in the build's key
// order and stores each caller index's key rank; the targets of a wave are
// then consecutive in key order, and its gathers land in a spatially compact
// range of records that stays in cache. Otherwise (no build, or a short
// target list) the kernel gathers from the caller's arrays. List entries are
// taken in batches whose loads issue together (a gather costs cache latency,
// not arithmetic); the pairs of a batch are then summed in list order, so the
// sums do not depend on the route or the order. Lists, targets and offsets are
// range-checked: a bad entry is skipped and flagged, never dereferenced.
#include "pbh_internal.hpp"
#include "wave.hpp"

namespace pbh {

namespace {

// Pair arithmetic is written with explicit fma() and contraction off, so every
// kernel that inlines it performs the same operations (the routes below give
// bit-identical sums).
// The cluster constants one target needs, held in registers for its loop.
struct IrrK {
    double rout2, r_in, inv_delta, c0, d0, l1, inner;
    double e[6];
};

__device__ inline IrrK irr_constants(const ClusterParams& c) {
    IrrK k;
    k.rout2 = c.rout2; k.r_in = c.r_in; k.inv_delta = c.inv_delta;
    k.c0 = c.c0; k.d0 = c.d0; k.l1 = c.l1; k.inner = c.inner;
    for (int q = 0; q < 6; ++q) k.e[q] = c.e[q];
    return k;
}

__device__ inline double phi_regular(const IrrK& cp, double s, double inv) {
#pragma clang fp contract(off)
    if (s < cp.r_in) return cp.inner;
    const double t = s * cp.inv_delta;
    double poly = fma(t, cp.e[5], cp.e[4]);
    poly = fma(t, poly, cp.e[3]);
    poly = fma(t, poly, cp.e[2]);
    poly = fma(t, poly, cp.e[1]);
    poly = fma(t, poly, cp.e[0]);
    double mid = fma(t, poly, cp.c0);
    if (cp.r_in > 0.0) mid = fma(cp.l1, log(s), fma(-cp.d0, inv, mid));
    return mid;
}

// rank[perm[k]] = k and rec[k] = particle perm[k] (velocity only if given)
__global__ __launch_bounds__(256) void k_irr_pack(int64_t n, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ pos,
                                                  const double* __restrict__ vel,
                                                  const double* __restrict__ mass,
                                                  int32_t* __restrict__ rank, IrrRec* __restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = perm[k];
    rank[i] = (int32_t)k;
    IrrRec r;
    r.x = pos[3 * i];
    r.y = pos[3 * i + 1];
    r.z = pos[3 * i + 2];
    r.m = mass[i];
    r.vx = vel ? vel[3 * i] : 0.0;
    r.vy = vel ? vel[3 * i + 1] : 0.0;
    r.vz = vel ? vel[3 * i + 2] : 0.0;
    r.pad = 0.0;
    rec[k] = r;
}

struct PartJ {
    double x, y, z, m, vx, vy, vz;
};

// particle j (caller index, range-checked) from the caller's arrays
template <bool JERK>
__device__ inline PartJ load_caller(const IrrParams& p, int64_t j) {
    PartJ q;
    q.x = p.pos[3 * j]; q.y = p.pos[3 * j + 1]; q.z = p.pos[3 * j + 2];
    q.m = p.mass[j];
    q.vx = q.vy = q.vz = 0.0;
    if (JERK) {
        q.vx = p.vel[3 * j]; q.vy = p.vel[3 * j + 1]; q.vz = p.vel[3 * j + 2];
    }
    return q;
}

// record at key position r
template <bool JERK>
__device__ inline PartJ load_rec(const IrrRec* rec, int64_t r) {
    PartJ q;
    const IrrRec* rp = rec + r;
    const double4 a = *reinterpret_cast<const double4*>(rp);
    q.x = a.x; q.y = a.y; q.z = a.z; q.m = a.w;
    q.vx = q.vy = q.vz = 0.0;
    if (JERK) {
        const double4 v = *reinterpret_cast<const double4*>(&rp->vx);
        q.vx = v.x; q.vy = v.y; q.vz = v.z;
    }
    return q;
}

struct IrrSums {
    double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, ph = 0;
};

// One pair (j != i): the terms of F_I, dF_I/dt and Phi_I.
template <bool JERK, bool POT>
__device__ inline void pair_irr(const IrrK& cp, double eps2, const PartJ& me, const PartJ& q,
                                IrrSums& S) {
#pragma clang fp contract(off)
    const double dx = q.x - me.x;
    const double dy = q.y - me.y;
    const double dz = q.z - me.z;
    const double s2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
    if (!(s2 < cp.rout2)) return;   // K = 0, Phi_I = 0
    const double m = q.m;
    const double inv = rsqrt(s2);
    const double s = s2 * inv;
    const double inv2 = inv * inv;
    const double inv3 = inv * inv2;
    double K = 1.0, slope = 0.0;
    if (s >= cp.r_in) {   // changeover band (a step changeover has inv_delta = 0: K = 1)
        const double x = (s - cp.r_in) * cp.inv_delta;
        const double omx = 1.0 - x;
        const double x2 = x * x;
        const double g = x2 * x2 * fma(x, fma(x, fma(-20.0, x, 70.0), -84.0), 35.0);
        K = 1.0 - g;
        const double o3 = omx * omx * omx;
        slope = 140.0 * (x2 * x) * o3 * cp.inv_delta;
    }
    const double mk3 = m * K * inv3;
    S.ax = fma(mk3, dx, S.ax);
    S.ay = fma(mk3, dy, S.ay);
    S.az = fma(mk3, dz, S.az);
    if (JERK) {
        const double ux = q.vx - me.vx;
        const double uy = q.vy - me.vy;
        const double uz = q.vz - me.vz;
        const double du = fma(dz, uz, fma(dy, uy, dx * ux));
        const double c3 = 3.0 * du * inv2;
        const double kd = -m * slope * du * inv * inv3;   // m (dK/dt) / s^3
        S.jx = fma(kd, dx, fma(mk3, fma(-c3, dx, ux), S.jx));
        S.jy = fma(kd, dy, fma(mk3, fma(-c3, dy, uy), S.jy));
        S.jz = fma(kd, dz, fma(mk3, fma(-c3, dz, uz), S.jz));
    }
    if (POT) S.ph = fma(m, -inv - phi_regular(cp, s, inv), S.ph);
}

// Target setup shared by both kernels: validates i and its list range, and
// finds its cluster constants. Returns false when i is out of range.
__device__ inline bool target_setup(const IrrParams& p, int64_t i, const ClusterParams*& cp,
                                    int64_t& b, int64_t& e, unsigned long long& bad) {
    b = e = 0;
    cp = &p.cp0;
    if ((uint64_t)i >= (uint64_t)p.n) {
        bad |= kIrrBadTarget;
        return false;
    }
    if (p.C > 1) {   // cluster of i: last c with cl_off[c] <= i
        int lo = 0, hi = p.C - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (p.cl_off[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        cp = p.cps + lo;
    }
    b = p.off[i];
    e = p.off[i + 1];
    if (b < 0 || e < b || e > p.cap) {
        bad |= kIrrBadOffsets;
        e = b;
    }
    return true;
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

// List entries per batch: their list, rank and particle loads are independent
// and issue together (one dependent chain per batch instead of per entry).
constexpr int kIrrBatch = 8;
// Blocks (of 256 key-order targets) per XCD chunk.
constexpr unsigned kIrrChunk = 16;

// MULTI: clusters with their own constants (per lane); otherwise one set, read
// from the kernel arguments (wave-uniform, so it stays in scalar registers).
// One target k (a lane): its sums over its list, stored at its output slot.
template <bool JERK, bool POT, bool SORTED, bool MULTI>
__device__ inline void irr_target(const IrrParams& p, int64_t k) {
    unsigned long long bad = 0;
    const int64_t i = p.tgt ? (int64_t)p.tgt[k] : (p.order ? (int64_t)p.order[k] : k);
    const ClusterParams* cp;
    int64_t b, e;
    IrrSums S;
    const bool valid = target_setup(p, i, cp, b, e, bad);
    if (valid) {
        const IrrK K = irr_constants(MULTI ? *cp : p.cp0);
        const PartJ me = SORTED ? load_rec<JERK>(p.rec, p.rank[i]) : load_caller<JERK>(p, i);
        for (; b < e; b += kIrrBatch) {
            int32_t jv[kIrrBatch];
            bool ok[kIrrBatch];
#pragma unroll
            for (int u = 0; u < kIrrBatch; ++u)   // clamped: inside the list whenever b < e
                jv[u] = p.idx[b + u < e ? b + u : e - 1];
#pragma unroll
            for (int u = 0; u < kIrrBatch; ++u) {
                const bool live = b + u < e;
                const bool inr = (uint64_t)(int64_t)jv[u] < (uint64_t)p.n;
                if (live && !inr) bad |= kIrrBadIndex;
                ok[u] = live && inr && jv[u] != i;
                if (!ok[u]) jv[u] = (int32_t)i;   // a valid index; its pair is not summed
            }
            PartJ q[kIrrBatch];
            if (SORTED) {
                int32_t rk[kIrrBatch];
#pragma unroll
                for (int u = 0; u < kIrrBatch; ++u) rk[u] = p.rank[jv[u]];
#pragma unroll
                for (int u = 0; u < kIrrBatch; ++u) q[u] = load_rec<JERK>(p.rec, rk[u]);
            } else {
#pragma unroll
                for (int u = 0; u < kIrrBatch; ++u) q[u] = load_caller<JERK>(p, jv[u]);
            }
#pragma unroll
            for (int u = 0; u < kIrrBatch; ++u)
                if (ok[u]) pair_irr<JERK, POT>(K, p.eps2, me, q[u], S);
        }
    }
    if (valid || p.tgt) store_sums<JERK, POT>(p, p.tgt ? k : i, S);   // no slot of its own otherwise
    if (bad) atomicOr(p.err, bad);
}

template <bool JERK, bool POT, bool SORTED, bool MULTI>
__global__ __launch_bounds__(256) void k_irregular(IrrParams p) {
    if (SORTED) {
        // key-order targets in chunks per XCD (cache locality and load balance)
        const unsigned blk = xcd_chunk_block(blockIdx.x, kIrrChunk);
        const int64_t k = (int64_t)blk * blockDim.x + threadIdx.x;
        if (k < p.n_tgt) irr_target<JERK, POT, SORTED, MULTI>(p, k);
        return;
    }
    // caller-array route: grid-stride, the count possibly held on the device
    int64_t nt = p.n_tgt;
    if (p.n_tgt_dev && (int64_t)*p.n_tgt_dev < nt) nt = (int64_t)*p.n_tgt_dev;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x)
        irr_target<JERK, POT, SORTED, MULTI>(p, k);
}

template <bool JERK, bool POT, bool MULTI>
void launch_route(const IrrParams& p, hipStream_t s) {
    const int64_t nb = (p.n_tgt + 255) / 256;
    const dim3 block(256);
    if (p.rec) {   // grid padded to whole rounds of chunks over the XCDs
        const int64_t round = (int64_t)kQueues * kIrrChunk;
        const dim3 grid((unsigned)((nb + round - 1) / round * round));
        hipLaunchKernelGGL((k_irregular<JERK, POT, true, MULTI>), grid, block, 0, s, p);
    } else {   // grid-stride: a count held on the device may be far below n_tgt
        const int64_t g = p.n_tgt_dev ? (nb < 1024 ? nb : 1024) : nb;
        hipLaunchKernelGGL((k_irregular<JERK, POT, false, MULTI>), dim3((unsigned)g), block, 0, s, p);
    }
}

template <bool JERK, bool POT>
void launch_multi(const IrrParams& p, hipStream_t s) {
    if (p.C > 1) launch_route<JERK, POT, true>(p, s);
    else launch_route<JERK, POT, false>(p, s);
}

}  // namespace

void launch_irregular(const IrrParams& p, hipStream_t s) {
    if (p.n_tgt <= 0) return;
    if (p.rec)
        hipLaunchKernelGGL(k_irr_pack, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p.n, p.perm,
                           p.pos, p.jerk ? p.vel : nullptr, p.mass, p.rank, p.rec);
    const bool jerk = p.jerk != nullptr, pot = p.pot != nullptr;
    if (jerk && pot) launch_multi<true, true>(p, s);
    else if (jerk) launch_multi<true, false>(p, s);
    else if (pot) launch_multi<false, true>(p, s);
    else launch_multi<false, false>(p, s);
}

}  // namespace pbh
