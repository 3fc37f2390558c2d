// walk.hip -- grouped Barnes-Hut walk for the regular force (gfx950).
//
// Regular acceleration of particle i (Arnold, Baumgardt & Wang 2021, Section
// 2.1, eq. fi with F_R = total - F_I and eq. duncan):
//   a_i = sum_j m_j W(s_ij) d_ij / s_ij^3,  d = x_j - x_i,  s^2 = r^2 + eps^2,
// and the regular potential Phi_R (dPhi_R/ds = W/s^2). Far nodes are taken as
// monopole + traceless quadrupole about their centre of mass (Section 2.4:
// Barnes-Hut with opening angle theta).
//
// One wavefront walks one group (a run of <= 64 sorted particles, one per
// lane). Persistent workgroups of one wave pull groups from a global counter.
// Per step the wave pops up to 64 nodes from its stack (one per lane) and
// classifies them in FP64 without FMA, exactly like the definition:
//   near   box-box distance^2 < R^2, or the boxes touch (R = r_out + r_buff,
//          the neighbour-list radius; R = r_out without a buffer)
//   accept not near, theta > 0, distance^2(group box, COM) > rcrit^2
//   open   otherwise: a leaf becomes particle-particle work, an inner node
//          pushes its children.
// Accepted nodes and leaf particles are compacted with ballot + prefix sums
// into LDS tiles of TC entries (64, 96 or 128; FP32 in the mixed path: positions
// relative to the group centre, formed in FP64 first); a tile is evaluated
// just before it would overflow, every lane reading each entry by LDS
// broadcast. Tile partial sums are
// folded into FP32 (hi, lo) pairs with TwoSum and returned in FP64.
#include <type_traits>

#include "pbh_internal.hpp"
#include "wave.hpp"

namespace pbh {

namespace {

// Tile capacity TC (a template parameter, 64, 96 or 128). A far or near tile
// is evaluated just before it would overflow; the multipole tile holds TC + 32
// entries and is evaluated at the start of a traversal step once it holds more
// than TC - 32 (one step adds at most 64), where the least state is live. One
// traversal step adds at most 64 entries of a kind, so TC >= 64.
//
// The first kWalkStackLds traversal stack entries live in LDS (the rest in the
// wave's spill region).
constexpr int kWalkStackLds = 640;
//
// Near entries of the FP64 walk keep their original coordinates for the
// neighbour test; the mixed walk keeps the sorted index instead and reads the
// coordinates from global memory in the rare case the FP64 test is needed
// (10 KB of LDS per wave with TC = 64: 16 waves per CU).
template <typename R, int TC>
struct NearExtra {
    double nx[TC], ny[TC], nz[TC];
};
template <int TC>
struct NearExtra<float, TC> {
    int nears[TC];     // sorted index
};

template <typename R, int TC>
struct alignas(16) Tiles : NearExtra<R, TC> {
    static_assert(TC >= 64, "one traversal step adds up to 64 entries");
    static constexpr int kCap = TC;
    R pn[TC + 32][12];   // cx cy cz M | qxx qyy qzz qxy | qxz qyz - -  (room for one more step)
    R far[TC][4];        // x y z m (relative to the group centre)
    R nearp[TC][4];
    int nearj[TC];       // caller index: skips the self pair, and is the neighbour index
    int lf_ex[64];       // leaf expansion: exclusive prefix of particle counts
    int lf_beg[64];
};

struct WalkParams {
    const WNode* node;
    const Mom32* q32;
    const Mom64* q64;
    const double* x;
    const double* y;
    const double* z;
    const double* m;
    const int32_t* perm;
    const int32_t* g_begin;
    const int32_t* g_count;
    const int32_t* g_root;
    const int32_t* g_cluster;
    const double* g_lo;
    const double* g_hi;
    const ClusterParams* cp;
    const unsigned long long* G;   // device-side group count
    int use_theta;
    double eps2;
    double* acc;
    double* pot;
    int32_t* stack;
    int stack_cap;
    unsigned long long* cnt;
    unsigned long long* queues;     // [kQueues] group queue heads
    unsigned long long* wave_log;   // per workgroup: groups walked, steady-clock ticks
    unsigned long long* wave_cyc;   // per workgroup: core clock cycles over the same span
    int32_t* nbr_cnt;               // neighbour counts per caller index, or null
    int32_t* stage;                 // neighbour staging rows per sorted particle, or null
    int scap;                       // entries per staging row
    int8_t* stage_k;                // per sorted particle: 1 = list staged, 0 = left to the fill pass
    int32_t* fill_list;             // groups left to the fill pass
    int max_copies;                 // most sub-wave copies of a small group (1..64)
    const double* cpos;             // caller's pos [n][3] and mass [n]: compared with the
    const double* cmass;            // build's sorted copy (changed in place: kErrStale), or null
};

__device__ inline void two_sum_acc(float& hi, float& lo, float v) {
    const float s = hi + v;
    const float bp = s - hi;
    const float e = (hi - (s - bp)) + (v - bp);
    hi = s;
    lo += e;
}

// Partial sums of one tile evaluation (one lane).
template <typename R>
struct Part {
    R x, y, z, p;
};

template <typename R>
struct Acc;

template <>
struct Acc<float> {
    float hx = 0, hy = 0, hz = 0, hp = 0, lx = 0, ly = 0, lz = 0, lp = 0;
    static constexpr int kWords = 8;
    __device__ void add(float ax, float ay, float az, float ph) {
        two_sum_acc(hx, lx, ax);
        two_sum_acc(hy, ly, ay);
        two_sum_acc(hz, lz, az);
        two_sum_acc(hp, lp, ph);
    }
    __device__ void add(const Part<float>& q) { add(q.x, q.y, q.z, q.p); }
    __device__ void store(float* w) const {
        w[0] = hx; w[1] = lx; w[2] = hy; w[3] = ly; w[4] = hz; w[5] = lz; w[6] = hp; w[7] = lp;
    }
    // adds another (hi, lo) set: TwoSum of the high parts, plain sum of the low parts
    __device__ void merge(const float* w) {
        two_sum_acc(hx, lx, w[0]); lx += w[1];
        two_sum_acc(hy, ly, w[2]); ly += w[3];
        two_sum_acc(hz, lz, w[4]); lz += w[5];
        two_sum_acc(hp, lp, w[6]); lp += w[7];
    }
    __device__ double gx() const { return (double)hx + (double)lx; }
    __device__ double gy() const { return (double)hy + (double)ly; }
    __device__ double gz() const { return (double)hz + (double)lz; }
    __device__ double gp() const { return (double)hp + (double)lp; }
};

template <>
struct Acc<double> {
    double x = 0, y = 0, z = 0, p = 0;
    static constexpr int kWords = 4;
    __device__ void add(double ax, double ay, double az, double ph) {
        x += ax; y += ay; z += az; p += ph;
    }
    __device__ void add(const Part<double>& q) { add(q.x, q.y, q.z, q.p); }
    __device__ void store(double* w) const { w[0] = x; w[1] = y; w[2] = z; w[3] = p; }
    __device__ void merge(const double* w) { x += w[0]; y += w[1]; z += w[2]; p += w[3]; }
    __device__ double gx() const { return x; }
    __device__ double gy() const { return y; }
    __device__ double gz() const { return z; }
    __device__ double gp() const { return p; }
};

// the value of lane L ^ 32: lane p < 32 receives lane p + 32's
template <typename R>
__device__ inline R shfl_down32(R v) { return __shfl_xor(v, 32, 64); }

__device__ inline float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ inline double rsq(double v) { return rsqrt(v); }
__device__ inline float lnr(float v) { return __logf(v); }
__device__ inline double lnr(double v) { return log(v); }

// Sub-wave split of the tile entries. A group of g <= 32 particles occupies
// ksub = 64 / g copies of itself in the wave (lane = sub * g + particle); the
// copy `sub` evaluates tile entries sub, sub + ksub, sub + 2 ksub, ... and the
// copies' partial sums are merged once per group. ksub = 1 is the plain
// one-particle-per-lane walk. `body(e)` evaluates entry e for this lane.
template <int U, typename F>
__device__ inline void for_entries(int cnt, int ksub, int sub, F&& body) {
    if (ksub == 1) {
#pragma unroll U
        for (int e = 0; e < cnt; ++e) body(e);
    } else {
        int e2 = 0;
#pragma unroll 2
        for (; e2 + ksub <= cnt; e2 += ksub) body(e2 + sub);
        if (e2 + sub < cnt) body(e2 + sub);
    }
}

// Loop iterations of for_entries, ceil(cnt / ksub), as a multiply and shift:
// with rcp = ceil(2^16 / ksub), floor(v * rcp / 2^16) = floor(v / ksub) for
// v < 2^16 / 64 (the error v * (rcp - 2^16 / ksub) / 2^16 stays below 1 / ksub).
__device__ inline unsigned rounds_rcp(int ksub) { return (65536u + (unsigned)ksub - 1u) / (unsigned)ksub; }
__device__ inline int entry_rounds(int cnt, int ksub, unsigned rcp) {
    return (int)(((unsigned)(cnt + ksub - 1) * rcp) >> 16);
}

// Monopole + traceless quadrupole: phi = -M/s - (R^T Q R)/(2 s^5), a = -grad phi
//   a = -(M/s^3 + (5/2) (R^T Q R)/s^7) R + Q R / s^5,   R = x_i - COM
template <typename R, int TC>
__device__ inline Part<R> eval_pn(const Tiles<R, TC>& T, int cnt, int ksub, int sub, R px, R py, R pz,
                                  R eps2) {
    R ax = 0, ay = 0, az = 0, ph = 0;
    for_entries<2>(cnt, ksub, sub, [&](int e) {
        const R* q = T.pn[e];
        const R Rx = px - q[0], Ry = py - q[1], Rz = pz - q[2];
        const R s2 = Rx * Rx + Ry * Ry + Rz * Rz + eps2;
        const R inv = rsq(s2);
        const R inv2 = inv * inv;
        const R inv3 = inv * inv2;
        const R inv5 = inv3 * inv2;
        const R inv7 = inv5 * inv2;
        const R qx = q[4] * Rx + q[7] * Ry + q[8] * Rz;
        const R qy = q[7] * Rx + q[5] * Ry + q[9] * Rz;
        const R qz = q[8] * Rx + q[9] * Ry + q[6] * Rz;
        const R rqr = Rx * qx + Ry * qy + Rz * qz;
        const R cr = -q[3] * inv3 - R(2.5) * rqr * inv7;
        ax += cr * Rx + qx * inv5;
        ay += cr * Ry + qy * inv5;
        az += cr * Rz + qz * inv5;
        ph += -q[3] * inv - R(0.5) * rqr * inv5;
    });
    return Part<R>{ax, ay, az, ph};
}

// FP32 form written as explicit FMA chains (33 VALU + 1 rsqrt per entry). The
// tile holds Q' = 2.5 Q, so with q' = Q' R and t' = R.q' / s^5 (= 2.5 t):
//   cr = M/s^3 + t'/s^2,  a += 0.4 q'/s^5 - cr R,  phi += -M/s - 0.2 t'.
// The q'/s^5 terms are summed apart and scaled by 0.4 once per tile.
template <int TC>
__device__ inline Part<float> eval_pn_f32(const Tiles<float, TC>& T, int cnt, int ksub, int sub, float px,
                                          float py, float pz, float eps2) {
    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
    float bx = 0.f, by = 0.f, bz = 0.f;
    for_entries<4>(cnt, ksub, sub, [&](int e) {
        const float4 a = *reinterpret_cast<const float4*>(&T.pn[e][0]);   // cx cy cz M
        const float4 b = *reinterpret_cast<const float4*>(&T.pn[e][4]);   // qxx qyy qzz qxy
        const float2 c = *reinterpret_cast<const float2*>(&T.pn[e][8]);   // qxz qyz
        const float Rx = px - a.x, Ry = py - a.y, Rz = pz - a.z;
        const float s2 = fmaf(Rz, Rz, fmaf(Ry, Ry, fmaf(Rx, Rx, eps2)));
        const float inv = __builtin_amdgcn_rsqf(s2);
        const float inv2 = inv * inv;
        const float qx = fmaf(c.x, Rz, fmaf(b.w, Ry, b.x * Rx));
        const float qy = fmaf(c.y, Rz, fmaf(b.y, Ry, b.w * Rx));
        const float qz = fmaf(b.z, Rz, fmaf(c.y, Ry, c.x * Rx));
        const float rqr = fmaf(Rz, qz, fmaf(Ry, qy, Rx * qx));
        const float inv3 = inv * inv2;
        const float inv5 = inv3 * inv2;
        const float t = rqr * inv5;
        const float cr = fmaf(t, inv2, a.w * inv3);
        bx = fmaf(qx, inv5, bx);
        by = fmaf(qy, inv5, by);
        bz = fmaf(qz, inv5, bz);
        ax = fmaf(-cr, Rx, ax);
        ay = fmaf(-cr, Ry, ay);
        az = fmaf(-cr, Rz, az);
        ph = fmaf(-a.w, inv, fmaf(-0.2f, t, ph));
    });
    return Part<float>{fmaf(0.4f, bx, ax), fmaf(0.4f, by, ay), fmaf(0.4f, bz, az), ph};
}

// Pairs of far leaves: every pair is at r >= R >= r_out, where W = 1.
template <typename R, int TC>
__device__ inline Part<R> eval_far(const Tiles<R, TC>& T, int cnt, int ksub, int sub, R px, R py, R pz,
                                   R eps2) {
    R ax = 0, ay = 0, az = 0, ph = 0;
    for_entries<4>(cnt, ksub, sub, [&](int e) {
        const R* q = T.far[e];
        const R dx = q[0] - px, dy = q[1] - py, dz = q[2] - pz;
        const R s2 = dx * dx + dy * dy + dz * dz + eps2;
        const R inv = rsq(s2);
        const R mi = q[3] * inv;
        const R mi3 = mi * inv * inv;
        ax += mi3 * dx;
        ay += mi3 * dy;
        az += mi3 * dz;
        ph -= mi;
    });
    return Part<R>{ax, ay, az, ph};
}

template <int TC>
__device__ inline Part<float> eval_far_f32(const Tiles<float, TC>& T, int cnt, int ksub, int sub,
                                           float px, float py, float pz, float eps2) {
    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
    for_entries<4>(cnt, ksub, sub, [&](int e) {
        const float4 q = *reinterpret_cast<const float4*>(&T.far[e][0]);
        const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
        const float s2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
        const float inv = __builtin_amdgcn_rsqf(s2);
        const float mi = q.w * inv;
        const float mi3 = mi * (inv * inv);
        ax = fmaf(mi3, dx, ax);
        ay = fmaf(mi3, dy, ay);
        az = fmaf(mi3, dz, az);
        ph -= mi;
    });
    return Part<float>{ax, ay, az, ph};
}

template <typename R>
struct NearK {
    R r_in, r_out, inv_delta, c0, d0, l1, inner;
    R e[6];
    bool pole;   // r_in > 0: the -d0/s and log terms are present
    // FP32 neighbour pre-test (mixed path): R^2 (list radius) in FP32 and the half-width
    // of the band around it inside which the FP64 test decides (infinite:
    // always FP64)
    float rlist2f, band;
    const double* x;   // sorted FP64 coordinates (the FP64 neighbour test of the mixed walk)
    const double* y;
    const double* z;
};

// Neighbour test of the CSR lists: r^2 < R^2 (list radius) in FP64 from the original
// coordinates, ((dx*dx + dy*dy) + dz*dz) without FMA.
__device__ inline bool is_neighbour(double xj, double yj, double zj, double xi, double yi, double zi,
                                    double rlist2) {
#pragma clang fp contract(off)
    const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    const double r2 = dx * dx + dy * dy + dz * dz;
    return r2 < rlist2;
}

// Pairs of near leaves: changeover weight W(s) and the regular potential;
// optionally also counts the neighbours inside the list radius R (FP64 test).
// optionally also stores them in the lane's staging row (`srow`, at most
// `scap` entries, kStageStride apart).
template <typename R, int TC>
__device__ inline Part<R> eval_near(const Tiles<R, TC>& T, int cnt, int ksub, int sub, R px, R py, R pz,
                                    R eps2, int self, const NearK<R>& K, bool count_nbr, int me,
                                    double rlist2, int& nbr, int32_t* srow, int scap) {
    const double xi = K.x[me], yi = K.y[me], zi = K.z[me];
    R ax = 0, ay = 0, az = 0, ph = 0;
    for_entries<1>(cnt, ksub, sub, [&](int e) {
        const R* q = T.nearp[e];
        const int oj = T.nearj[e];
        const bool is_self = oj == self;
        if (count_nbr) {
            const bool nb = !is_self && is_neighbour(T.nx[e], T.ny[e], T.nz[e], xi, yi, zi, rlist2);
            if (nb && nbr < scap) srow[nbr * kStageStride] = oj;
            nbr += nb ? 1 : 0;
        }
        const R dx = q[0] - px, dy = q[1] - py, dz = q[2] - pz;
        const R s2 = dx * dx + dy * dy + dz * dz + eps2;
        const R inv = rsq(s2);
        const R s = s2 > R(0) ? s2 * inv : R(0);
        const R xx = (s - K.r_in) * K.inv_delta;
        const R x2 = xx * xx;
        const R gpoly = x2 * x2 * (R(35) + xx * (R(-84) + xx * (R(70) - R(20) * xx)));
        const R W = s >= K.r_out ? R(1) : (s < K.r_in ? R(0) : gpoly);
        const R f = (W > R(0) && !is_self) ? q[3] * W * inv * inv * inv : R(0);
        ax += f * dx;
        ay += f * dy;
        az += f * dz;
        const R t = s * K.inv_delta;
        R mid = K.c0 + t * (K.e[0] + t * (K.e[1] + t * (K.e[2] + t * (K.e[3] + t * (K.e[4] + t * K.e[5])))));
        if (K.pole) mid += -K.d0 * inv + K.l1 * lnr(s);
        const R phi = s >= K.r_out ? -inv : (s < K.r_in ? K.inner : mid);
        ph += is_self ? R(0) : q[3] * phi;
    });
    return Part<R>{ax, ay, az, ph};
}

// FP32 form without per-lane branches: the neighbour count and the pole
// terms (-d0/s + l1 ln s, present when r_in > 0) are compile-time switches,
// ln s = log2(s) ln 2, and the boundary cases of W and Phi_R are selects.
// Each entry yields a force factor f and a potential term, taken either from
// the far-pair formula (every lane beyond the list radius) or from the
// changeover forms; the sums are updated in one place after either.
template <bool CNT, bool POLE, int TC>
__device__ inline Part<float> eval_near_f32(const Tiles<float, TC>& T, int cnt, int ksub, int sub,
                                            float px, float py, float pz, float eps2, int self,
                                            const NearK<float>& K, int me, double rlist2, int& nbr,
                                            int32_t* srow, int scap) {
    const double* __restrict__ gx = K.x;
    const double* __restrict__ gy = K.y;
    const double* __restrict__ gz = K.z;
    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
    const float l1 = K.l1 * 0.693147180559945309f;
    const float x0 = -K.r_in * K.inv_delta;   // x = (s - r_in) / delta = s / delta + x0
    // s^2 >= 1e-30 keeps 1/s and 1/s^2 finite: a pair at s = 0 only arises with
    // eps = 0 (where W = 0 and the self pair is masked); for eps^2 >= 2^-76 the
    // added term is below half an ulp of s^2 and changes nothing
    const float e2 = eps2 + 1e-30f;
    for_entries<2>(cnt, ksub, sub, [&](int e) {
        const float4 q = *reinterpret_cast<const float4*>(&T.nearp[e][0]);
        const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float s2 = r2 + e2;
        const float dr = r2 - K.rlist2f;
        const float inv = __builtin_amdgcn_rsqf(s2);
        float f, pt;
        if (__ballot(dr <= K.band) == 0) {
            // every lane's pair lies beyond R >= r_out by more than the rounding band:
            // no neighbour, W = 1 and Phi_R = -1/s (the far-pair formula)
            const float mi = q.w * inv;
            f = mi * (inv * inv);
            pt = -mi;
        } else {
            // changeover forms first (every lane evaluates them), then the
            // neighbour test, then the selects
            const float s = s2 * inv;
            const float xx = fmaf(s, K.inv_delta, x0);
            const float x2 = xx * xx;
            const float gp = (x2 * x2) * fmaf(xx, fmaf(xx, fmaf(-20.f, xx, 70.f), -84.f), 35.f);
            const float t = s * K.inv_delta;
            float mid = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, K.e[5], K.e[4]), K.e[3]), K.e[2]), K.e[1]),
                             K.e[0]);
            mid = fmaf(t, mid, K.c0);
            if (POLE) mid = fmaf(-K.d0, inv, fmaf(l1, __builtin_amdgcn_logf(s), mid));
            // (the empty asm statements keep the polynomial and the selects in
            // place: sunk under a divergent branch on s < r_out, they cost more in
            // exec-mask handling than they save)
            asm volatile("" : "+v"(mid));
            const bool outer = s >= K.r_out, inner = s < K.r_in;
            float phi = inner ? K.inner : mid;
            asm volatile("" : "+v"(phi));
            phi = outer ? -inv : phi;
            const int oj = T.nearj[e];
            const bool other = oj != self;
            if (CNT) {
                // FP32 decides outside the band (where it provably agrees with the
                // FP64 definition), the FP64 test inside it
                const bool band = fabsf(dr) <= K.band;
                bool nb = dr < 0.f;
                if (__ballot(band)) {
                    if (band) {
                        const int js = T.nears[e];
                        nb = is_neighbour(gx[js], gy[js], gz[js], gx[me], gy[me], gz[me], rlist2);
                    }
                }
                nb = nb & other;
                if (nb & (nbr < scap)) srow[nbr * kStageStride] = oj;
                nbr += nb ? 1 : 0;
            }
            const float mq = other ? q.w : 0.f;
            const float W = outer ? 1.f : (inner ? 0.f : gp);
            // W first: W = 0 gives f = 0 without forming m / s^3
            f = ((W * mq) * inv) * (inv * inv);
            pt = mq * phi;
        }
        ax = fmaf(f, dx, ax);
        ay = fmaf(f, dy, ay);
        az = fmaf(f, dz, az);
        ph += pt;
    });
    return Part<float>{ax, ay, az, ph};
}

// The mixed walk's forms (explicit FMA chains above), chosen per precision.
template <int TC>
__device__ inline Part<float> eval_pn(const Tiles<float, TC>& T, int cnt, int ksub, int sub, float px,
                                      float py, float pz, float eps2) {
    return eval_pn_f32<TC>(T, cnt, ksub, sub, px, py, pz, eps2);
}

template <int TC>
__device__ inline Part<float> eval_far(const Tiles<float, TC>& T, int cnt, int ksub, int sub, float px,
                                       float py, float pz, float eps2) {
    return eval_far_f32<TC>(T, cnt, ksub, sub, px, py, pz, eps2);
}

template <int TC>
__device__ inline Part<float> eval_near(const Tiles<float, TC>& T, int cnt, int ksub, int sub,
                                        float px, float py, float pz, float eps2, int self,
                                        const NearK<float>& K, bool count_nbr, int me, double rlist2,
                                        int& nbr, int32_t* srow, int scap) {
    if (count_nbr) {
        if (K.pole)
            return eval_near_f32<true, true, TC>(T, cnt, ksub, sub, px, py, pz, eps2, self, K, me, rlist2,
                                                 nbr, srow, scap);
        return eval_near_f32<true, false, TC>(T, cnt, ksub, sub, px, py, pz, eps2, self, K, me, rlist2,
                                              nbr, srow, scap);
    }
    if (K.pole)
        return eval_near_f32<false, true, TC>(T, cnt, ksub, sub, px, py, pz, eps2, self, K, me, rlist2,
                                              nbr, srow, scap);
    return eval_near_f32<false, false, TC>(T, cnt, ksub, sub, px, py, pz, eps2, self, K, me, rlist2, nbr,
                                           srow, scap);
}

// Four waves per SIMD (16 per compute unit, which the 64-entry mixed walk's
// LDS allows): the register budget is held to 128, which this kernel fits
// without spilling; left free, the compiler takes more and halves nothing but
// occupancy. Larger tiles and the FP64 walk are held lower by their LDS.
template <bool MIXED, int TC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_walk(WalkParams p) {
    using R = typename std::conditional<MIXED, float, double>::type;
    constexpr int TCAP = TC;
    __shared__ Tiles<R, TC> T;
    __shared__ int s_stack[kWalkStackLds];
    const int lane = threadIdx.x;
    const Stack stack{s_stack, p.stack + (int64_t)blockIdx.x * (p.stack_cap - kWalkStackLds), p.stack_cap,
                      kWalkStackLds};
    int home = blockIdx.x % kQueues;
    const R eps2 = (R)p.eps2;
    const int64_t G = (int64_t)*p.G;
    const unsigned long long t_start = wall_clock64();
    const unsigned long long c_start = clock64();
    int n_walked = 0;

    for (;;) {
        const int64_t g = queue_next(p.queues, G, home, lane);
        if (g < 0) break;
        ++n_walked;

        const int gb = uni(p.g_begin[g]), gcnt = uni(p.g_count[g]), root = uni(p.g_root[g]);
        const int cl = uni(p.g_cluster[g]);
        double glo[3], ghi[3], ctr[3];
        for (int k = 0; k < 3; ++k) {
            glo[k] = p.g_lo[3 * g + k];
            ghi[k] = p.g_hi[3 * g + k];
            ctr[k] = (glo[k] + ghi[k]) * 0.5;
        }
        const ClusterParams& cp = p.cp[cl];
        const double rlist2 = cp.rlist2;   // neighbour-list radius R = r_out + r_buff, squared
        NearK<R> K;
        if (MIXED) {
            K.r_in = cp.f_r_in; K.r_out = cp.f_r_out; K.inv_delta = cp.f_inv_delta;
            K.c0 = cp.f_c0; K.d0 = cp.f_d0; K.l1 = cp.f_l1; K.inner = cp.f_inner;
            for (int k = 0; k < 6; ++k) K.e[k] = cp.f_e[k];
        } else {
            K.r_in = cp.r_in; K.r_out = cp.r_out; K.inv_delta = cp.inv_delta;
            K.c0 = cp.c0; K.d0 = cp.d0; K.l1 = cp.l1; K.inner = cp.inner;
            for (int k = 0; k < 6; ++k) K.e[k] = cp.e[k];
        }
        K.pole = cp.d0 != 0.0;
        {
            // Band of the FP32 neighbour pre-test against the list radius R.
            // Relative coordinates are FP64 differences rounded once to FP32, so
            // with |p| <= h (group box half side) and a pair at r <= 2 R each
            // component of d errs by at most 2^-24 (2h + 2.01 r); with h <= 64 R
            // the error of r^2 (squares, FMA rounding, R^2 in FP32) stays below
            // 928 * 2^-24 R^2, and for r > 2 R far below r^2 - R^2. The band is
            // 2048 * 2^-24 R^2; larger groups always take the FP64 test.
            double h = 0.0;
            for (int k = 0; k < 3; ++k) h = fmax(h, (ghi[k] - glo[k]) * 0.5);
            K.rlist2f = (float)rlist2;
            K.x = p.x; K.y = p.y; K.z = p.z;
            K.band = (h <= 64.0 * cp.rlist) ? (float)(2048.0 * 0x1p-24 * rlist2) : INFINITY;
        }

        // Lane roles. By default a group of g particles takes one pass over
        // every tile with ksub = min(64 / g, cap) copies, lane = copy * g +
        // particle (see for_entries; lanes beyond ksub * g repeat copy 0 and
        // are ignored at the merge), and the copies are merged once per group.
        // A group of 33..53 particles takes two passes over every multipole
        // tile instead (split): pass A holds particles 0..31 in two copies
        // (particle lane & 31, copy lane >> 5), pass B the other rB = g - 32
        // in kB = min(64 / rB, cap, 8) >= 3 copies counted from lane 32, so
        // that lane 32 + q holds particle 32 + q in copy 0. Their copies are
        // merged after every tile into lane p < g, which owns particle p and
        // takes the group's far and near tiles in one pass.
        const bool active = lane < gcnt;
        const int rB = gcnt - 32;
        int kB = 0;
        if (rB >= 1 && rB <= 21) {
            const int kfit = 64 / rB;
            kB = kfit < p.max_copies ? kfit : p.max_copies;
            kB = kB < 8 ? kB : 8;
        }
        const bool split = kB >= 3;
        int ksubA, subA, plA, copyA;
        int subB = 0, plB = 0;
        if (split) {
            ksubA = 2;
            copyA = lane >> 5;
            subA = copyA;
            plA = lane & 31;
            const int q = (lane - 32) & 63;
            const int cB = q / rB;
            plB = 32 + (q - cB * rB);
            subB = cB < kB ? cB : 0;
        } else {
            const int kfit = 64 / gcnt;
            ksubA = kfit < p.max_copies ? kfit : p.max_copies;
            copyA = lane / gcnt;
            plA = lane - copyA * gcnt;
            subA = copyA < ksubA ? copyA : 0;
        }
        // the particle whose far and near pairs, neighbour list and outputs
        // this lane handles (a stand-in for the idle lanes of a split group)
        const int own = split ? (active ? lane : 0) : plA;
        const int ksubN = split ? 1 : ksubA;
        const int subN = split ? 0 : subA;
        const int me = gb + own;
        const int orig_me = p.perm[me];
        if (p.cpos) {
            // the caller's arrays must still hold what the build sorted
            const int64_t o3 = 3 * (int64_t)orig_me;
            const bool stale = active && (p.cpos[o3] != p.x[me] || p.cpos[o3 + 1] != p.y[me] ||
                                          p.cpos[o3 + 2] != p.z[me] || p.cmass[orig_me] != p.m[me]);
            if (__ballot(stale)) atomicOr(&p.cnt[kErr], lane == 0 ? kErrStale : 0ull);
        }
        // Neighbour staging. A particle's row holds p.scap entries; a lane
        // that holds it whole (ksubN = 1) uses it whole, copies of a small group
        // each get a sub-row of wrow = p.scap / ksubN entries (joined into one
        // list after the walk). Lanes that hold no particle of their own, or
        // repeat copy 0, store nothing (scap = 0).
        const bool real = split ? active : copyA < ksubA;
        const int wrow = p.scap / ksubN;
        const int scap = (p.stage == nullptr || !real) ? 0 : (ksubN == 1 ? p.scap : wrow);
        int32_t* srow = p.stage != nullptr
                            ? p.stage + stage_index(me, (ksubN == 1 ? 0 : subN * wrow), p.scap)
                            : nullptr;
        // positions relative to the group centre: pass A (also the far and
        // near tiles, except on lanes >= 32 of a split group) and pass B
        const R pAx = (R)(p.x[gb + plA] - ctr[0]);
        const R pAy = (R)(p.y[gb + plA] - ctr[1]);
        const R pAz = (R)(p.z[gb + plA] - ctr[2]);
        const int pbi = split ? gb + plB : me;
        const R pBx = (R)(p.x[pbi] - ctr[0]);
        const R pBy = (R)(p.y[pbi] - ctr[1]);
        const R pBz = (R)(p.z[pbi] - ctr[2]);
        const unsigned rcpA = rounds_rcp(ksubA), rcpB = split ? rounds_rcp(kB) : 0u,
                       rcpN = rounds_rcp(ksubN);
        const bool hiB = split && lane >= 32;   // lanes whose own particle is pass B's copy 0
        const bool ownerB = hiB && active;
        const bool count_nbr = p.nbr_cnt != nullptr;
        int npn = 0, nfar = 0, nnear = 0;
        unsigned c_pn = 0, c_far = 0, c_near = 0;   // per group: far below 2^32
        // loop iterations of the evaluations (each occupies all 64 lanes)
        unsigned it_pn = 0, it_far = 0, it_near = 0;
        int nbr = 0;
        Acc<R> A;
        // one flush of each tile kind; every lane runs it (it_* counts the
        // loop iterations, each of which occupies the 64 lanes)
        auto flush_pn = [&](int cnt) {
            it_pn += entry_rounds(cnt, ksubA, rcpA);
            Part<R> pa = eval_pn(T, cnt, ksubA, subA, pAx, pAy, pAz, eps2);
            if (split) {
                it_pn += entry_rounds(cnt, kB, rcpB);
                const Part<R> pb = eval_pn(T, cnt, kB, subB, pBx, pBy, pBz, eps2);
                // pass A: copy 1 (lane p + 32) into lane p
                pa.x += shfl_down32(pa.x);
                pa.y += shfl_down32(pa.y);
                pa.z += shfl_down32(pa.z);
                pa.p += shfl_down32(pa.p);
                // pass B: copies in copy order into lane 32 + q, through the
                // tile's storage (every lane has read the tile)
                __syncthreads();
                Part<R>* red = reinterpret_cast<Part<R>*>(&T.pn[0][0]);
                red[lane] = pb;
                __syncthreads();
                Part<R> sb{R(0), R(0), R(0), R(0)};
                if (ownerB) {
                    for (int c = 0; c < kB; ++c) {
                        const Part<R> v = red[(lane + c * rB) & 63];
                        sb.x += v.x; sb.y += v.y; sb.z += v.z; sb.p += v.p;
                    }
                }
                __syncthreads();
                if (hiB) pa = sb;   // idle lanes add zero
            }
            A.add(pa);
        };
        auto flush_far = [&](int cnt) {
            it_far += entry_rounds(cnt, ksubN, rcpN);
            A.add(eval_far(T, cnt, ksubN, subN, hiB ? pBx : pAx, hiB ? pBy : pAy, hiB ? pBz : pAz, eps2));
        };
        auto flush_near = [&](int cnt) {
            it_near += entry_rounds(cnt, ksubN, rcpN);
            A.add(eval_near(T, cnt, ksubN, subN, hiB ? pBx : pAx, hiB ? pBy : pAy, hiB ? pBz : pAz, eps2,
                            orig_me, K, count_nbr, me, rlist2, nbr, srow, scap));
        };
        stack.put(0, root);   // every lane stores the same value
        int top = 1;
        bool overflow = false;

        while (top > 0) {
            // multipole tile: evaluated here, where no node state is live,
            // once it could not take another step's entries (up to 64)
            if (npn > TCAP - 32) {
                __syncthreads();
                flush_pn(npn);
                npn = 0;
                __syncthreads();
            }
            __threadfence_block();
            const int npop = uni(top < 64 ? top : 64);
            top -= npop;
            const bool has = lane < npop;
            const int nd = has ? stack.get(top + lane) : root;
            __threadfence_block();
            const WNode w = p.node[nd];
            const double dbox2 = box_box_d2(glo, ghi, w.lo, w.hi);
            const bool near = (dbox2 < rlist2) || (dbox2 == 0.0);
            const bool accept = has && !near && p.use_theta && (box_pt_d2(glo, ghi, w.com) > w.rcrit2);
            const bool open = has && !accept;
            const bool leaf = w.nchild == 0;

            // multipole entries
            const uint64_t mk = __ballot(accept);
            if (mk) {
                const int k = uni(__popcll(mk));
                if (accept) {
                    R* e = T.pn[npn + popc_below(mk)];
                    e[0] = (R)(w.com[0] - ctr[0]);
                    e[1] = (R)(w.com[1] - ctr[1]);
                    e[2] = (R)(w.com[2] - ctr[2]);
                    if (MIXED) {
                        // quadrupole scaled by 2.5 (see eval_pn<float>)
                        const Mom32 q = p.q32[nd];
                        e[3] = q.M; e[4] = 2.5f * q.qxx; e[5] = 2.5f * q.qyy; e[6] = 2.5f * q.qzz;
                        e[7] = 2.5f * q.qxy; e[8] = 2.5f * q.qxz; e[9] = 2.5f * q.qyz;
                    } else {
                        const Mom64 q = p.q64[nd];
                        e[3] = q.M; e[4] = q.qxx; e[5] = q.qyy; e[6] = q.qzz;
                        e[7] = q.qxy; e[8] = q.qxz; e[9] = q.qyz;
                    }
                }
                npn = uni(npn + k);
                c_pn += k;
            }

            // children of opened inner nodes
            const int nch = (open && !leaf) ? w.nchild : 0;
            const int incl = wave_incl_scan(nch, lane);
            const int tot = last_lane(incl);
            if (top + tot > p.stack_cap) {
                overflow = true;
                break;
            }
            for (int k = 0; k < nch; ++k) stack.put(top + incl - nch + k, w.first_child + k);
            top = uni(top + tot);

            // leaves: far ones (W = 1) and near ones (changeover)
            for (int cls = 0; cls < 2; ++cls) {
                const bool flag = open && leaf && (cls == 0 ? !near : near);
                const uint64_t lm = __ballot(flag);
                if (!lm) continue;
                const int v = flag ? w.count : 0;
                const int li = wave_incl_scan(v, lane);
                const int total = last_lane(li);
                __syncthreads();
                T.lf_ex[lane] = li - v;
                T.lf_beg[lane] = w.begin;
                __syncthreads();
                if (cls == 0) c_far += total; else c_near += total;
                for (int base = 0; base < total; base += 64) {
                    const int s = base + lane;
                    int k = 0;
#pragma unroll
                    for (int st = 32; st > 0; st >>= 1)
                        if (T.lf_ex[k + st] <= s) k += st;
                    const int j = T.lf_beg[k] + (s - T.lf_ex[k]);
                    int& fill = cls == 0 ? nfar : nnear;
                    const int add = (total - base) < 64 ? (total - base) : 64;
                    if (fill + add > TCAP) {
                        __syncthreads();
                        if (cls == 0) flush_far(fill);
                        else flush_near(fill);
                        fill = 0;
                        __syncthreads();
                    }
                    if (s < total) {
                        R* e = cls == 0 ? T.far[fill + lane] : T.nearp[fill + lane];
                        e[0] = (R)(p.x[j] - ctr[0]);
                        e[1] = (R)(p.y[j] - ctr[1]);
                        e[2] = (R)(p.z[j] - ctr[2]);
                        e[3] = (R)p.m[j];
                        if (cls == 1) {
                            T.nearj[fill + lane] = p.perm[j];
                            if constexpr (MIXED) {
                                T.nears[fill + lane] = j;
                            } else {
                                T.nx[fill + lane] = p.x[j];
                                T.ny[fill + lane] = p.y[j];
                                T.nz[fill + lane] = p.z[j];
                            }
                        }
                    }
                    fill = uni(fill + add);
                }
                __syncthreads();
            }
        }
        __syncthreads();
        if (npn) flush_pn(npn);
        if (nfar) flush_far(nfar);
        if (nnear) flush_near(nnear);
        __syncthreads();

        // a row that overflowed sends the group's lists to the fill pass
        const bool row_full = count_nbr && real && nbr > scap;
        const bool need_fill = count_nbr && (p.stage == nullptr || __ballot(row_full) != 0);
        if (!split && ksubA > 1) {
            const int ksub = ksubA;
            // merge the copies' partial sums in copy order, into copy 0
            R* red = &T.pn[0][0];
            constexpr int W = Acc<R>::kWords + 1;   // odd stride: no LDS bank conflicts
            A.store(red + W * lane);
            T.nearj[lane] = nbr;
            __syncthreads();
            // (the barrier also makes the copies' staged entries visible)
            if (active) {
                const bool join = count_nbr && !need_fill;
                int32_t* base = join ? p.stage + stage_index(me, 0, p.scap) : nullptr;
                for (int c = 1; c < ksub; ++c) {
                    A.merge(red + W * (c * gcnt + lane));
                    const int nc = T.nearj[c * gcnt + lane];
                    // move copy c's sub-row down to follow the list so far;
                    // targets lie below sources, loads of a batch precede its stores
                    if (join) {
                        for (int t0 = 0; t0 < nc; t0 += 8) {
                            int v[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int t = t0 + u < nc ? t0 + u : nc - 1;
                                v[u] = base[(int64_t)(c * wrow + t) * kStageStride];
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                if (t0 + u < nc) base[(int64_t)(nbr + t0 + u) * kStageStride] = v[u];
                        }
                    }
                    nbr += nc;
                }
            }
            __syncthreads();
        }
        if (overflow) atomicOr(&p.cnt[kErr], lane == 0 ? kErrWalkStack : 0ull);
        if (count_nbr) {
            // lists this walk did not stage completely go to the fill pass
            if (need_fill) {
                // all lanes issue the atomic (lane 0 adds 1): no lane-0-only branch
                const unsigned long long slot =
                    atomicAdd(&p.cnt[kCntFill], lane == 0 ? 1ull : 0ull);
                if (lane == 0) p.fill_list[slot] = (int32_t)g;
            }
            if (active) p.stage_k[me] = (int8_t)(need_fill ? 0 : 1);
        }
        if (active) {
            const int orig = orig_me;
            if (count_nbr) p.nbr_cnt[orig] = nbr;
            p.acc[3 * (int64_t)orig] = A.gx();
            p.acc[3 * (int64_t)orig + 1] = A.gy();
            p.acc[3 * (int64_t)orig + 2] = A.gz();
            p.pot[orig] = A.gp();
        }
        // interaction counters: one contribution per wave (lane 0), others add 0
        const unsigned long long l0 = lane == 0 ? (unsigned long long)gcnt : 0ull;
        atomicAdd(&p.cnt[kCntPN], (unsigned long long)c_pn * l0);
        atomicAdd(&p.cnt[kCntFar], (unsigned long long)c_far * l0);
        atomicAdd(&p.cnt[kCntNear], (unsigned long long)c_near * l0);
        const unsigned long long w0 = lane == 0 ? 64ull : 0ull;
        atomicAdd(&p.cnt[kCntSlotPN], (unsigned long long)it_pn * w0);
        atomicAdd(&p.cnt[kCntSlotFar], (unsigned long long)it_far * w0);
        atomicAdd(&p.cnt[kCntSlotNear], (unsigned long long)it_near * w0);
    }
    if (p.wave_log) {
        const unsigned long long c_end = clock64();
        p.wave_log[2 * blockIdx.x] = (unsigned long long)n_walked;
        p.wave_log[2 * blockIdx.x + 1] = wall_clock64() - t_start;
        p.wave_cyc[blockIdx.x] = c_end - c_start;
    }
}

// rcrit^2 = (l/theta + delta)^2 per node, l = largest box extent, delta =
// |COM - box centre|; also clears the per-call counters and queues.
__global__ void k_rcrit(WNode* __restrict__ node, const unsigned long long* __restrict__ n_dev,
                        double theta, unsigned long long* __restrict__ cnt,
                        unsigned long long* __restrict__ queues) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)*n_dev;
    if (blockIdx.x == 0 && threadIdx.x < 3 * kQueues) queues[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt[kCntPN] = 0; cnt[kCntFar] = 0; cnt[kCntNear] = 0; cnt[kCntFill] = 0;
        cnt[kCntSlotPN] = 0; cnt[kCntSlotFar] = 0; cnt[kCntSlotNear] = 0;
    }
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n;
         b += (int64_t)gridDim.x * blockDim.x) {
        WNode& w = node[b];
        double l = 0.0;
        for (int k = 0; k < 3; ++k)
            if (w.hi[k] - w.lo[k] > l) l = w.hi[k] - w.lo[k];
        double dd[3];
        for (int k = 0; k < 3; ++k) dd[k] = w.com[k] - (w.lo[k] + w.hi[k]) * 0.5;
        const double delta = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
        const double rc = theta > 0.0 ? l / theta + delta : 0.0;
        w.rcrit2 = rc * rc;
    }
}

}  // namespace

void launch_rcrit(Dev& d, const BuildCfg& c, double theta, hipStream_t s) {
    int64_t nb = (c.node_cap + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_rcrit, dim3(nb), dim3(256), 0, s, d.node,
                       (const unsigned long long*)(d.cnt + kCntNodes), theta, d.cnt, d.queues);
}

template <bool MIXED>
static auto walk_kernel(int tile) {
    return tile == 128 ? k_walk<MIXED, 128> : (tile == 96 ? k_walk<MIXED, 96> : k_walk<MIXED, 64>);
}

int walk_blocks_per_cu(int mixed, int tile) {
    int nb = 0;
    if (mixed) hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kernel<true>(tile), 64, 0);
    else hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kernel<false>(tile), 64, 0);
    return nb > 0 ? nb : 1;
}

void launch_walk(Dev& d, const BuildCfg& c, const WalkCfg& w, double* acc, double* pot,
                 hipStream_t s) {
    WalkParams p;
    p.node = d.node;
    p.q32 = d.q32;
    p.q64 = d.q64;
    p.x = d.x; p.y = d.y; p.z = d.z; p.m = d.m;
    p.perm = d.perm;
    p.g_begin = d.g.begin; p.g_count = d.g.count; p.g_root = d.g.root; p.g_cluster = d.g.cluster;
    p.g_lo = d.g.lo; p.g_hi = d.g.hi;
    p.cp = d.cparams;
    p.G = d.cnt + kCntGroups;
    p.use_theta = w.theta > 0.0;
    p.eps2 = w.eps * w.eps;
    p.acc = acc;
    p.pot = pot;
    p.stack = d.stack;
    p.stack_cap = w.stack_cap;
    p.cnt = d.cnt;
    p.queues = d.queues;
    p.wave_log = d.wave_log;
    p.wave_cyc = d.wave_cyc;
    p.nbr_cnt = w.count_nbr ? d.nbr_cnt : nullptr;
    p.stage = (w.count_nbr && w.stage_cap > 0) ? d.nbr_stage : nullptr;
    p.scap = w.stage_cap;
    p.stage_k = d.stage_k;
    p.fill_list = d.fill_list;
    p.max_copies = w.max_copies;
    p.cpos = w.cpos;
    p.cmass = w.cmass;
    if (w.mixed) hipLaunchKernelGGL(walk_kernel<true>(w.tile), dim3(w.grid), dim3(64), 0, s, p);
    else hipLaunchKernelGGL(walk_kernel<false>(w.tile), dim3(w.grid), dim3(64), 0, s, p);
}

}  // namespace pbh
