// herm.hip -- Hermite integration of the irregular force with block time
// steps over one regular step, the inner loop of the P3T scheme (gfx950).
//
// Arnold, Baumgardt & Wang (2021), Section 2.2: between two regular kicks
// every particle moves under its irregular force F_I, integrated with the
// Hermite scheme on individual block steps. Per particle the state is x, v,
// a = F_I, j = dF_I/dt, its time tau_i and step dt_i = dt_max / 2^k, with
// dt_max = T / 4 (eq. dtmax) for a regular step T. Times are integer ticks of
// dt_max / 2^kHermK, so block times add exactly. One block:
//   tau' = min(tau_i + dt_i); the active particles and the members of their
//   neighbour lists are predicted to tau' with the P3T predictor (eq.
//   p3t-jpred-x, -dx: no regular force, the kicks carry it)
//     x_p = x + d v + d^2/2 a + d^3/6 j,   v_p = v + d a + d^2/2 j;
//   the active particles (tau_i + dt_i = tau') get F_I and its derivative at
//   the predicted state from their neighbour lists, then the 4th-order Hermite
//   corrector (d = dt_i, da = a - a1)
//     a2 = (-6 da - d (4 j + 2 j1)) / d^2,  a3 = (12 da + 6 d (j + j1)) / d^3
//     x = x_p + d^4/24 a2 + d^5/120 a3,     v = v_p + d^3/6 a2 + d^4/24 a3
//   and a new step from eq. dt (eta) with a^(0) = a1 + F_R, a^(1) = j1,
//   a^(2) = a2 + d a3, a^(3) = a3: at most twice the old step and dt_max,
//   rounded down to dt_max / 2^k dividing tau'. The corrector is the standard
//   Hermite one (Makino & Aarseth 1992).
// First steps (Section 2.1, after eq. dt: the higher derivatives are computed
// and the fourth-order criterion sets the initial step; steps are set afresh
// after every regular kick): with a = F_I and j = dF_I/dt of every particle
// at the start, the second and third derivatives of F_I along the motion
// under F_I come from the neighbour lists (relative accelerations a_j - a_i,
// relative jerks j_j - j_i), and eq. dt with a^(0) = a + F_R, a^(1) = j and
// those derivatives gives the first step; dt_max where its denominator is 0
// (no pair inside r_out). Expressions are evaluated as written (no contraction).
//
// A block is two launches: the front (next block time, active list,
// prediction) and the force with the corrector; particles are kept in one
// bucket per level, so neither launch passes over all n particles.
#include "irr_pair.hpp"
#include "pbh_internal.hpp"

namespace pbh {

namespace {

__device__ inline double norm3(double x, double y, double z) {
#pragma clang fp contract(off)
    return sqrt(x * x + y * y + z * z);
}

// Block schedule by level. A particle at level k has dt_i = 2^(kHermK - k)
// ticks, and its time tau_i is a multiple of dt_i (the new step is chosen to
// divide the block time), with tau_i <= t < tau_i + dt_i at the current block
// time t. Its next time tau_i + dt_i is then the first multiple of dt_i after
// t, so the next block time tn = min(tau_i + dt_i) is the first multiple of
// the smallest occupied step after t, and particle i is active at tn exactly
// when dt_i divides tn, i.e. when k >= k* = kHermK - ctz(tn) (0 if that is
// negative). Particles are therefore kept in one bucket per level and a block
// takes whole buckets: no pass over all n particles per block. The corrected
// particles of a block (levels >= k*) move to their new levels, which are
// >= k* - 1 (the step at most doubles): buckets >= k* are refilled from zero
// and bucket k* - 1 is appended to.
//
// Level counts are double-buffered by block parity q: the front of a block
// reads the counts of slot q (cnt, plus the appends newcnt of the previous
// block, and that block's k*) and writes the merged counts to slot q ^ 1,
// where the corrector of the same block appends. Every launch of a block
// reads only what earlier launches wrote.
//
// Blocks are enqueued in batches without waiting; once every particle has
// reached the end of the regular step the remaining blocks are empty
// (kHermDone), and the front that finds it also sets a host-visible flag,
// which the host reads after a batch while the next one runs.
constexpr int kHermGrid = 1024;   // grid-stride launches
constexpr int kHermLanes = 32;    // lanes per active particle in the prediction (the particle and its list)
constexpr int kHermAllFrac = 8;   // predict all particles when n_active >= n / 8
constexpr int kSlotShift = 26;    // per-item scratch: level << 26 | rank in its workgroup
constexpr uint32_t kSlotMask = (1u << kSlotShift) - 1;
static_assert(kHermK < 63, "levels fit one wave");

__device__ inline unsigned long long* lev_cnt(const HermParams& p, int q) { return p.lev + kLevCnt + 64 * q; }
__device__ inline unsigned long long* lev_new(const HermParams& p, int q) { return p.lev + kLevNew + 64 * q; }

__device__ inline void predict_one(const HermParams& p, int64_t i, int64_t tn) {
#pragma clang fp contract(off)
    const double d = (double)(tn - p.tau[i]) * p.unit;
    const double d2 = d * d, d3 = d2 * d;
    for (int k = 0; k < 3; ++k) {
        const int64_t q = 3 * i + k;
        p.xp[q] = p.x[q] + d * p.v[q] + 0.5 * d2 * p.a[q] + d3 / 6.0 * p.j[q];
        p.vp[q] = p.v[q] + d * p.a[q] + 0.5 * d2 * p.j[q];
    }
}

// The count of level k (lane k of a wave) after merging the previous block's
// appends into slot q; `add` returns those appends.
__device__ inline long long merged_count(const HermParams& p, int q, int k, long long& add) {
    add = 0;
    if (k > kHermK) return 0;
    const int kp = (int)p.lev[kLevKs + q];   // k* of the previous block
    const long long old = (long long)lev_cnt(p, q)[k];
    add = (long long)lev_new(p, q)[k];
    return k >= kp ? add : (k == kp - 1 ? old + add : old);
}

// The next block from the level counts (one wave, lane k holding count c of
// level k) and the current time t: its time tn, k*, the number of active
// particles and lane k's offset in the active list (levels >= k* in order).
struct BlockPlan {
    long long tn, nact, off;
    int ks;
    bool done;
};

__device__ inline BlockPlan plan_block(long long c, long long t, unsigned long long tend) {
    const int k = threadIdx.x & 63;
    BlockPlan b;
    const int kmax = 63 - __clzll(__ballot(c > 0));   // deepest occupied level (n >= 1)
    b.done = t >= (long long)tend;
    const int sh = kHermK - kmax;
    b.tn = b.done ? (long long)tend : (((t >> sh) + 1) << sh);
    const int tz = __ffsll((unsigned long long)b.tn) - 1;
    b.ks = b.done ? kHermK + 1 : (tz >= kHermK ? 0 : kHermK - tz);
    const long long a = k >= b.ks ? c : 0;
    long long incl = a;
    for (int o = 1; o < 64; o <<= 1) {
        const long long w = __shfl_up(incl, o, 64);
        if (k >= o) incl += w;
    }
    b.nact = __shfl(incl, 63, 64);
    b.off = incl - a;
    return b;
}

// entry t of the active list: level buckets ks, ks + 1, ... in turn
__device__ inline int32_t active_at(const HermParams& p, const long long* off, const long long* cnt, int ks,
                                    long long t) {
    int k = ks;
    while (k < kHermK && t >= off[k] + cnt[k]) ++k;
    return p.bucket[(int64_t)k * p.n + (t - off[k])];
}

// predict the active particle i (item 0) or member g - 1, g - 1 + kHermLanes, ...
// of its list (items g, g + kHermLanes, ...): lane g of its lane group
__device__ inline void predict_items(const HermParams& p, int32_t i, int g, int64_t tn) {
    if (g == 0) predict_one(p, i, tn);
    const int64_t b0 = p.off[i], e = p.off[i + 1];
    if (b0 < 0 || e < b0 || e > p.cap) return;   // flagged by the force kernel
    for (int64_t m = b0 + (g == 0 ? kHermLanes - 1 : g - 1); m < e; m += kHermLanes) {
        const int64_t j = p.idx[m];
        if ((uint64_t)j < (uint64_t)p.n) predict_one(p, j, tn);
    }
}

// Block front: the next block time and the active buckets (computed by every
// workgroup from slot q; workgroup 0 publishes them), then the active list
// (bucket order) with the prediction of each active particle and its list
// members (a member shared by several lists is written with the same value
// by each) -- the only states the irregular force of the block reads.
__global__ __launch_bounds__(256) void k_herm_front(HermParams p, int q) {
    __shared__ long long s_cnt[64], s_off[64];
    __shared__ long long s_tn, s_nact;
    __shared__ int s_ks;
    if (threadIdx.x < 64) {
        const int k = threadIdx.x;
        long long add;
        const long long c = merged_count(p, q, k, add);
        // deepest new level of the previous corrector (its appends; the first
        // block's appends are the start levels, not counted)
        const uint64_t app = __ballot(add > 0);
        const long long t = (long long)p.lev[kLevT + q];
        const BlockPlan B = plan_block(c, t, p.tend);
        s_cnt[k] = c;
        s_off[k] = B.off;
        if (k == 0) {
            s_tn = B.tn;
            s_nact = B.nact;
            s_ks = B.ks;
        }
        if (blockIdx.x == 0) {
            if (k == 0 && t > 0 && app) {
                const unsigned long long dl = (unsigned long long)(63 - __clzll(app));
                if (dl > p.ctl[kHermKmax]) p.ctl[kHermKmax] = dl;
            }
            if (k <= kHermK) {
                lev_cnt(p, q ^ 1)[k] = (unsigned long long)c;
                lev_new(p, q ^ 1)[k] = 0ull;
            }
            if (k == 0) {
                p.lev[kLevT + (q ^ 1)] = (unsigned long long)B.tn;
                p.lev[kLevKs + (q ^ 1)] = (unsigned long long)B.ks;
                p.ctl[kHermTn] = B.done ? ~0ull : (unsigned long long)B.tn;
                p.ctl[kHermNact] = (unsigned long long)B.nact;
                if (B.done) {
                    p.ctl[kHermDone] = 1ull;
                    if (p.done_host) *p.done_host = 1ull;   // read by the host while later blocks run
                } else {
                    p.ctl[kHermBlocks] += 1ull;
                    p.ctl[kHermSteps] += (unsigned long long)B.nact;
                }
            }
        }
    }
    __syncthreads();
    const long long nact = s_nact, tn = s_tn;
    const int ks = s_ks;
    const long long stride = (long long)gridDim.x * 256;
    const long long t0 = (long long)blockIdx.x * 256 + threadIdx.x;
    if (nact * kHermAllFrac >= p.n) {
        // a large active set: predict every particle once, in order (the
        // others are not read by this block), and list the active ones
        for (long long t = t0; t < p.n; t += stride) predict_one(p, t, tn);
        for (long long t = t0; t < nact; t += stride) p.act[t] = active_at(p, s_off, s_cnt, ks, t);
        return;
    }
    // kHermLanes lanes per active particle: item 0 is the particle, item
    // m >= 1 the m-th member of its list
    for (long long t = t0; t < nact * kHermLanes; t += stride) {
        const long long a = t / kHermLanes;
        const int g = (int)(t % kHermLanes);
        const int32_t i = active_at(p, s_off, s_cnt, ks, a);
        if (g == 0) p.act[a] = i;
        predict_items(p, i, g, tn);
    }
}

// Each workgroup takes one contiguous chunk of the n_items items (a multiple of
// 256, so a small set is one workgroup): `step(k, i)` advances item k (the
// particle i = list[k], or k without a list) and returns its new level; the
// workgroup ranks its items per level in LDS, reserves room in each bucket
// with one device atomic per level (buckets >= ks restart from zero, bucket
// ks - 1 keeps its members), then stores the particles there. Same-address
// device atomics serialise, so one per workgroup and level, not per wave; a
// workgroup that holds every item stores its counts without atomics.
template <class Step>
__device__ inline void step_and_bucket(const HermParams& p, int q, int ks, int64_t n_items,
                                       const int32_t* list, int32_t first, Step step) {
    __shared__ int s_h[64];
    __shared__ long long s_b[64];
    const int64_t per = ((n_items + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    const int64_t c0 = (int64_t)blockIdx.x * per, c1 = c0 + per < n_items ? c0 + per : n_items;
    if (c0 >= c1) return;   // workgroup-uniform
    if (threadIdx.x < 64) s_h[threadIdx.x] = 0;
    __syncthreads();
    // a thread's first item stays in registers; later ones go through p.slot
    int lv0 = -1, r0 = 0;
    int32_t i0 = 0;
    for (int64_t k = c0 + threadIdx.x; k < c1; k += 256) {
        const bool head = k == c0 + threadIdx.x;
        // (workgroup 0's first items are k = threadIdx.x: `first` holds list[k])
        const int32_t i = list ? (head && c0 == 0 ? first : list[k]) : (int32_t)k;
        const int level = step(k, i);
        const int r = atomicAdd(&s_h[level], 1);
        if (head) {
            lv0 = level;
            r0 = r;
            i0 = i;
        } else {
            p.slot[k] = ((uint32_t)level << kSlotShift) | (uint32_t)r;
        }
    }
    __syncthreads();
    if (threadIdx.x <= kHermK && s_h[threadIdx.x] > 0) {
        const int k = threadIdx.x;
        const long long keep = k == ks - 1 ? (long long)lev_cnt(p, q)[k] : 0;
        if (c0 == 0 && c1 == n_items) {   // the only workgroup with items: no other appends
            s_b[k] = keep;
            lev_new(p, q)[k] = (unsigned long long)s_h[k];
        } else {
            s_b[k] = keep + (long long)atomicAdd(lev_new(p, q) + k, (unsigned long long)s_h[k]);
        }
    }
    __syncthreads();
    if (lv0 >= 0) p.bucket[(int64_t)lv0 * p.n + s_b[lv0] + r0] = i0;
    for (int64_t k = c0 + threadIdx.x + 256; k < c1; k += 256) {   // the same later items per thread
        const uint32_t v = p.slot[k];
        const int level = (int)(v >> kSlotShift);
        const int32_t i = list ? list[k] : (int32_t)k;
        p.bucket[(int64_t)level * p.n + s_b[level] + (int64_t)(v & kSlotMask)] = i;
    }
}

// block step in ticks: dt_max / 2^k not above `want`, dividing tau (the
// largest power of two dividing tau > 0 is its lowest set bit)
__device__ inline int64_t block_step(double want, double dtmax, int64_t tau) {
    double d = dtmax;
    int k = 0;
    while (d > want && k < kHermK) {
        d *= 0.5;
        ++k;
    }
    int64_t t = (int64_t)1 << (kHermK - k);
    const int64_t low = tau & -tau;
    if (tau != 0 && low < t) t = low;
    return t;
}

__device__ inline int step_level(int64_t t) { return kHermK - (63 - __clzll((unsigned long long)t)); }

// Second and third time derivatives of one pair term m K(s) d / s^3 of F_I,
// added to f2, f3. d, u, w, z: relative position, velocity, acceleration and
// jerk (j's minus i's); s^2 = |d|^2 + eps^2. The Newtonian part A = m d / s^3
// follows the usual recurrences in
//   al = d.u / s^2,  be = (u.u + d.w) / s^2 + al^2,
//   ga = (3 u.w + d.z) / s^2 + al (3 be - 4 al^2):
//   dA = m u / s^3 - 3 al A,  d2A = m w / s^3 - 6 al dA - 3 be A,
//   d3A = m z / s^3 - 9 al d2A - 9 be dA - 3 ga A;
// along the motion s has the derivatives al s, (be - 2 al^2) s and
// s ((3 u.w + d.z) / s^2 - 3 al (be - 2 al^2)); in the band the weight has
// dK/ds = -g1(x)/D, d2K/ds2 = -g2(x)/D^2, d3K/ds3 = -g3(x)/D^3 with
// g1 = 140 x^3 (1-x)^3, g2 = 420 x^2 (1-x)^2 (1-2x), g3 = 840 x (1-x) (1-5x+5x^2),
// and the product rule gives the second and third derivatives of K A.
__device__ inline void pair_d23(const ClusterParams& cp, double eps2, const double* d, const double* u,
                                const double* w, const double* z, double m, double* f2, double* f3) {
#pragma clang fp contract(off)
    const double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    if (!(s2 < cp.rout2)) return;   // K = 0 with all its derivatives
    const double s = sqrt(s2);
    const double i2 = 1.0 / s2;
    const double mi3 = m / (s2 * s);
    const double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
    const double uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    const double dz = d[0] * z[0] + d[1] * z[1] + d[2] * z[2];
    const double al = du * i2;
    const double be = (uu + dw) * i2 + al * al;
    const double ga = (3.0 * uw + dz) * i2 + al * (3.0 * be - 4.0 * al * al);
    double K = 1.0, K1 = 0.0, K2 = 0.0, K3 = 0.0;   // K and its time derivatives
    if (s >= cp.r_in && cp.inv_delta > 0.0) {
        const double x = (s - cp.r_in) * cp.inv_delta, o = 1.0 - x;
        const double x2 = x * x;
        const double id = cp.inv_delta;
        K = 1.0 - x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
        const double ks1 = -140.0 * x2 * x * o * o * o * id;
        const double ks2 = -420.0 * x2 * o * o * (1.0 - 2.0 * x) * id * id;
        const double ks3 = -840.0 * x * o * (1.0 - 5.0 * x + 5.0 * x2) * id * id * id;
        const double sd1 = al * s;
        const double q = be - 2.0 * al * al;
        const double sd2 = q * s;
        const double sd3 = s * ((3.0 * uw + dz) * i2 - 3.0 * al * q);
        K1 = ks1 * sd1;
        K2 = ks2 * sd1 * sd1 + ks1 * sd2;
        K3 = ks3 * sd1 * sd1 * sd1 + 3.0 * ks2 * sd1 * sd2 + ks1 * sd3;
    }
    for (int c = 0; c < 3; ++c) {
        const double A0 = mi3 * d[c];
        const double A1 = mi3 * u[c] - 3.0 * al * A0;
        const double A2 = mi3 * w[c] - 6.0 * al * A1 - 3.0 * be * A0;
        const double A3 = mi3 * z[c] - 9.0 * al * A2 - 9.0 * be * A1 - 3.0 * ga * A0;
        f2[c] += K * A2 + 2.0 * K1 * A1 + K2 * A0;
        f3[c] += K * A3 + 3.0 * K1 * A2 + 3.0 * K2 * A1 + K3 * A0;
    }
}

// First steps: one lane per particle sums the derivatives over its list (in
// list order; lists from the regular-force walk are short), then eq. dt.
__global__ __launch_bounds__(256) void k_herm_start(HermParams p, IrrParams ip) {
    // slot 0, every level refilled (ks = 0)
    step_and_bucket(p, 0, 0, p.n, nullptr, 0, [&](int64_t, int32_t i) {
#pragma clang fp contract(off)
        const int64_t i3 = 3 * (int64_t)i;
        double xi[3], vi[3], ai[3], ji[3], f2[3] = {0.0, 0.0, 0.0}, f3[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            xi[c] = p.x[i3 + c];
            vi[c] = p.v[i3 + c];
            ai[c] = p.a[i3 + c];
            ji[c] = p.j[i3 + c];
        }
        int64_t b = p.off[i], e = p.off[i + 1];
        if (b < 0 || e < b || e > p.cap) {   // malformed offsets: flagged, list not read
            atomicOr(ip.err, kIrrBadOffsets);
            e = b;
        }
        for (int64_t q = b; q < e; ++q) {
            const int32_t jj = p.idx[q];
            if ((uint64_t)(int64_t)jj >= (uint64_t)p.n) {
                atomicOr(ip.err, kIrrBadIndex);
                continue;
            }
            if (jj == i) continue;
            const int64_t j3 = 3 * (int64_t)jj;
            double d[3], u[3], w[3], z[3];
            for (int c = 0; c < 3; ++c) {
                d[c] = p.x[j3 + c] - xi[c];
                u[c] = p.v[j3 + c] - vi[c];
                w[c] = p.a[j3 + c] - ai[c];
                z[c] = p.j[j3 + c] - ji[c];
            }
            pair_d23(ip.cp0, ip.eps2, d, u, w, z, ip.mass[jj], f2, f3);
        }
        double at[3];
        for (int c = 0; c < 3; ++c) at[c] = ai[c] + (p.fr ? p.fr[i3 + c] : 0.0);
        const double n0 = norm3(at[0], at[1], at[2]);
        const double n1 = norm3(ji[0], ji[1], ji[2]);
        const double n2 = norm3(f2[0], f2[1], f2[2]);
        const double n3 = norm3(f3[0], f3[1], f3[2]);
        const double num = n0 * n2 + n1 * n1, den = n1 * n3 + n2 * n2;
        const double want = den > 0.0 ? sqrt(p.eta * num / den) : p.dtmax;
        const int64_t t = block_step(want, p.dtmax, 0);
        p.tau[i] = 0;
        p.dt[i] = t;
        if (p.dt0) p.dt0[i] = t;
        return step_level(t);
    });
}

// The irregular force of the block and the corrector, one lane per active
// particle: F_I and its derivative a1, j1 at the predicted state (the pair
// terms of the irregular-force kernel, summed over the list in order), then
// the 4th-order corrector and the new block step; returns the new level. The force reads only
// predicted states and masses; the corrector writes only the state of its own
// particle, so neither reads what the other writes.
__device__ inline int force_correct(const HermParams& p, const IrrParams& ip, int32_t i, int64_t tn) {
#pragma clang fp contract(off)
    // the corrector's own inputs first: their loads overlap the force's gathers
    const int64_t dti = p.dt[i];
    double a0[3], j0[3], fr[3], xp[3], vp[3];
    for (int c = 0; c < 3; ++c) {
        const int64_t q3 = 3 * (int64_t)i + c;
        a0[c] = p.a[q3];
        j0[c] = p.j[q3];
        fr[c] = p.fr ? p.fr[q3] : 0.0;
        xp[c] = p.xp[q3];
        vp[c] = p.vp[q3];
    }
    IrrSums S;   // (the pair sums carry their own contraction setting)
    unsigned long long bad = 0;
    irr_sums<true, false, false, false>(ip, i, S, bad);
    if (bad) atomicOr(ip.err, bad);
    const double a1v[3] = {S.ax, S.ay, S.az}, j1v[3] = {S.jx, S.jy, S.jz};
    const double d = (double)dti * p.unit, d2 = d * d, d3 = d2 * d, d4 = d3 * d, d5 = d4 * d;
    double a2[3], a3[3], a2e[3], at[3];
    for (int c = 0; c < 3; ++c) {
        const int64_t q3 = 3 * (int64_t)i + c;
        const double a1 = a1v[c], j1 = j1v[c];
        const double da = a0[c] - a1;
        a2[c] = (-6.0 * da - d * (4.0 * j0[c] + 2.0 * j1)) / d2;
        a3[c] = (12.0 * da + 6.0 * d * (j0[c] + j1)) / d3;
        p.x[q3] = xp[c] + d4 / 24.0 * a2[c] + d5 / 120.0 * a3[c];
        p.v[q3] = vp[c] + d3 / 6.0 * a2[c] + d4 / 24.0 * a3[c];
        p.a[q3] = a1;
        p.j[q3] = j1;
        a2e[c] = a2[c] + d * a3[c];
        at[c] = a1 + fr[c];
    }
    const double n0 = norm3(at[0], at[1], at[2]);
    const double n1 = norm3(j1v[0], j1v[1], j1v[2]);
    const double n2 = norm3(a2e[0], a2e[1], a2e[2]);
    const double n3 = norm3(a3[0], a3[1], a3[2]);
    const double num = n0 * n2 + n1 * n1, den = n1 * n3 + n2 * n2;
    double want = den > 0.0 ? sqrt(p.eta * num / den) : p.dtmax;
    if (want > 2.0 * d) want = 2.0 * d;
    const int64_t t = block_step(want, p.dtmax, tn);
    p.tau[i] = tn;
    p.dt[i] = t;
    return step_level(t);
}

__global__ __launch_bounds__(256) void k_herm_force_correct(HermParams p, IrrParams ip, int q) {
    // workgroup 0's first active entries, read alongside the block's counts
    // (act has n entries; an entry past n_active is never used)
    const int32_t first = blockIdx.x == 0 && (int64_t)threadIdx.x < p.n ? p.act[threadIdx.x] : 0;
    const int64_t nact = (int64_t)p.ctl[kHermNact];
    const int ks = (int)p.lev[kLevKs + (q ^ 1)];
    const int64_t tn = (int64_t)p.ctl[kHermTn];
    step_and_bucket(p, q ^ 1, ks, nact, p.act, first,
                    [&](int64_t, int32_t i) { return force_correct(p, ip, i, tn); });
}

// pot_tot = pot_r + pot_i
__global__ void k_add(int64_t n, const double* a, const double* b, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

}  // namespace

static unsigned herm_grid(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < kHermGrid ? (g < 1 ? 1 : g) : kHermGrid);
}

void launch_herm_start(const HermParams& p, const IrrParams& ip, hipStream_t s) {
    hipLaunchKernelGGL(k_herm_start, dim3(herm_grid(p.n)), dim3(256), 0, s, p, ip);
}

void launch_herm_front(const HermParams& p, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_herm_front, dim3(herm_grid(p.n)), dim3(256), 0, s, p, parity);
}

void launch_herm_force_correct(const HermParams& p, const IrrParams& ip, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_herm_force_correct, dim3(herm_grid(p.n)), dim3(256), 0, s, p, ip, parity);
}

void launch_add(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b, out);
}

}  // namespace pbh
