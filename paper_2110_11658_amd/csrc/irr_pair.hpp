// irr_pair.hpp -- the pair terms and per-target sums of the irregular force
// (F_I, its time derivative, Phi_I), shared by the irregular-force kernels and
// the Hermite corrector that consumes them. The formulas and their readings
// are stated in irr.hip.
#pragma once
#include "pbh_internal.hpp"

namespace pbh {

namespace {

// Pair arithmetic is written with explicit fma() and contraction off, so every
// kernel that inlines it performs the same operations per pair (the two routes
// of the irregular-force kernel, which also share a summation order, give
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

// Natural logarithm of a positive normal s. With s = m 2^e and m in
// [1/sqrt 2, sqrt 2), ln s = e ln 2 + 2 atanh(t) for t = (m - 1)/(m + 1),
// |t| <= 0.1716, and atanh t = t + t^3/3 + t^5/5 + ... (the terms through t^19
// leave a remainder below 2.3e-17 t). m - 1 is exact; 1/(m + 1) is the
// hardware reciprocal, good to about single precision, refined by two Newton
// steps (one leaves errors up to 21 ulp in ln s); ln 2 is split into a 32-bit
// head (e ln2_hi is exact) and the rest (Cody and Waite). On the device within
// 2.4 ulp of ln s (mean 0.34 ulp) over 2^20 values in [1e-13, 400] against a
// long-double reference; about 32 instructions against the 85 of the library's
// correctly rounded form.
__device__ inline double log_pos(double s) {
    double m = __builtin_amdgcn_frexp_mant(s);   // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(s);
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double num = m - 1.0, den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double t = num * r, t2 = t * t;
    double q = 1.0 / 19.0;
    q = fma(q, t2, 1.0 / 17.0);
    q = fma(q, t2, 1.0 / 15.0);
    q = fma(q, t2, 1.0 / 13.0);
    q = fma(q, t2, 1.0 / 11.0);
    q = fma(q, t2, 1.0 / 9.0);
    q = fma(q, t2, 1.0 / 7.0);
    q = fma(q, t2, 1.0 / 5.0);
    q = fma(q, t2, 1.0 / 3.0);
    const double at = fma(t * t2, q, t);
    const double ln2_hi = 0x1.62e42fee00000p-1, ln2_lo = 0x1.a39ef35793c76p-33;
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, 2.0 * at));
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
    if (cp.r_in > 0.0) mid = fma(cp.l1, log_pos(s), fma(-cp.d0, inv, mid));   // s >= r_in > 0
    return mid;
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

// List entries per batch: their list, rank and particle loads are independent
// and issue together (one dependent chain per batch instead of per entry).
constexpr int kIrrBatch = 8;

// The sums of target i (caller index) over its list, in list order; false when
// i is out of range. MULTI: clusters with their own constants (per lane);
// otherwise one set, read from the kernel arguments (wave-uniform, so it stays
// in scalar registers). SORTED: particles from the key-order records.
template <bool JERK, bool POT, bool SORTED, bool MULTI>
__device__ inline bool irr_sums(const IrrParams& p, int64_t i, IrrSums& S, unsigned long long& bad) {
    const ClusterParams* cp;
    int64_t b, e;
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
    return valid;
}


// Lane groups: kIrrLanes lanes share one target. Lane g takes list entries
// g, g + kIrrLanes, g + 2 kIrrLanes, ... in that order (irr_lane_batch of
// them per round, their loads issued together), and the group adds its partial
// sums with a fixed butterfly (xor 4, 2, 1), so every lane ends with the
// same total and the order does not depend on the launch. A wave's list loads
// are then contiguous runs, and its record loads fall on the neighbours of a
// few targets, close together in key order.
constexpr int kIrrLanes = 8;
// entries per lane and round on the caller-array route: 4 for the force
// alone; 3 with the jerk, whose records and terms would otherwise hold the
// kernel to 3 waves per SIMD
template <bool JERK>
constexpr int irr_lane_batch() { return JERK ? 3 : 4; }

__device__ inline double group_sum(double v) {
#pragma unroll
    for (int o = kIrrLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool JERK, bool POT, bool SORTED, bool MULTI>
__device__ inline bool irr_sums_lanes(const IrrParams& p, int64_t i, int g, IrrSums& S,
                                      unsigned long long& bad) {
    const ClusterParams* cp;
    int64_t b, e;
    const bool valid = target_setup(p, i, cp, b, e, bad);
    if (g != 0) bad = 0;   // target and offset flags once per group
    if (valid) {
        const IrrK K = irr_constants(MULTI ? *cp : p.cp0);
        const PartJ me = SORTED ? load_rec<JERK>(p.rec, p.rank[i]) : load_caller<JERK>(p, i);
        constexpr int kIrrLaneBatch = irr_lane_batch<JERK>();
        for (int64_t m = b + g; m < e; m += kIrrLanes * kIrrLaneBatch) {
            int32_t jv[kIrrLaneBatch];
            bool ok[kIrrLaneBatch];
#pragma unroll
            for (int u = 0; u < kIrrLaneBatch; ++u) {   // clamped: inside the list whenever m < e
                const int64_t q = m + (int64_t)kIrrLanes * u;
                jv[u] = p.idx[q < e ? q : e - 1];
            }
#pragma unroll
            for (int u = 0; u < kIrrLaneBatch; ++u) {
                const bool live = m + (int64_t)kIrrLanes * u < e;
                const bool inr = (uint64_t)(int64_t)jv[u] < (uint64_t)p.n;
                if (live && !inr) bad |= kIrrBadIndex;
                ok[u] = live && inr && jv[u] != i;
                if (!ok[u]) jv[u] = (int32_t)i;   // a valid index; its pair is not summed
            }
            PartJ q[kIrrLaneBatch];
            if (SORTED) {
                int32_t rk[kIrrLaneBatch];
#pragma unroll
                for (int u = 0; u < kIrrLaneBatch; ++u) rk[u] = p.rank[jv[u]];
#pragma unroll
                for (int u = 0; u < kIrrLaneBatch; ++u) q[u] = load_rec<JERK>(p.rec, rk[u]);
            } else {
#pragma unroll
                for (int u = 0; u < kIrrLaneBatch; ++u) q[u] = load_caller<JERK>(p, jv[u]);
            }
#pragma unroll
            for (int u = 0; u < kIrrLaneBatch; ++u)
                if (ok[u]) pair_irr<JERK, POT>(K, p.eps2, me, q[u], S);
        }
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

}  // namespace

}  // namespace pbh
