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
// One lane per target; the targets of a wave are consecutive in the tree's
// key order when the context holds a build of these n particles, so the
// neighbours a wave gathers overlap and stay in cache (the results do not
// depend on the order). Lists, targets and offsets are range-checked: a bad
// entry is skipped and flagged, never dereferenced.
#include "pbh_internal.hpp"

namespace pbh {

namespace {

__device__ inline double phi_regular(const ClusterParams& cp, double s, double inv) {
    if (s < cp.r_in) return cp.inner;
    const double t = s * cp.inv_delta;
    double mid = cp.c0 + t * (cp.e[0] + t * (cp.e[1] + t * (cp.e[2] + t * (cp.e[3] + t * (cp.e[4] + t * cp.e[5])))));
    if (cp.r_in > 0.0) mid += -cp.d0 * inv + cp.l1 * log(s);
    return mid;
}

template <bool JERK, bool POT>
__global__ __launch_bounds__(256) void k_irregular(IrrParams p) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_tgt) return;
    unsigned long long bad = 0;
    int64_t i = p.tgt ? (int64_t)p.tgt[k] : (p.order ? (int64_t)p.order[k] : k);
    const int64_t slot = p.tgt ? k : i;
    double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, ph = 0;
    if ((uint64_t)i >= (uint64_t)p.n) {
        bad |= kIrrBadTarget;
        if (!p.tgt) {   // no output slot of its own to clear
            atomicOr(p.err, bad);
            return;
        }
    } else {
        int c = 0;
        if (p.C > 1) {   // cluster of i: last c with cl_off[c] <= i
            int lo = 0, hi = p.C - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (p.cl_off[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            c = lo;
        }
        const ClusterParams& cp = p.C > 1 ? p.cps[c] : p.cp0;
        const double rout2 = cp.rout2;
        const double r_in = cp.r_in, inv_delta = cp.inv_delta;
        const double xi = p.pos[3 * i], yi = p.pos[3 * i + 1], zi = p.pos[3 * i + 2];
        double vxi = 0, vyi = 0, vzi = 0;
        if (JERK) {
            vxi = p.vel[3 * i];
            vyi = p.vel[3 * i + 1];
            vzi = p.vel[3 * i + 2];
        }
        int64_t b = p.off[i], e = p.off[i + 1];
        if (b < 0 || e < b || e > p.cap) {
            bad |= kIrrBadOffsets;
            e = b;
        }
        for (; b < e; ++b) {
            const int32_t j = p.idx[b];
            if ((uint64_t)(int64_t)j >= (uint64_t)p.n) {
                bad |= kIrrBadIndex;
                continue;
            }
            if (j == i) continue;
            const double dx = p.pos[3 * (int64_t)j] - xi;
            const double dy = p.pos[3 * (int64_t)j + 1] - yi;
            const double dz = p.pos[3 * (int64_t)j + 2] - zi;
            const double s2 = dx * dx + dy * dy + dz * dz + p.eps2;
            if (!(s2 < rout2)) continue;   // K = 0, Phi_I = 0
            const double m = p.mass[j];
            const double inv = rsqrt(s2);
            const double s = s2 * inv;
            const double inv2 = inv * inv;
            const double inv3 = inv * inv2;
            double K = 1.0, slope = 0.0;
            if (s >= r_in) {   // changeover band (a step changeover has inv_delta = 0: K = 1)
                const double x = (s - r_in) * inv_delta;
                const double omx = 1.0 - x;
                const double x2 = x * x;
                K = 1.0 - x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
                slope = 140.0 * x2 * x * omx * omx * omx * inv_delta;
            }
            const double mk3 = m * K * inv3;
            ax += mk3 * dx;
            ay += mk3 * dy;
            az += mk3 * dz;
            if (JERK) {
                const double ux = p.vel[3 * (int64_t)j] - vxi;
                const double uy = p.vel[3 * (int64_t)j + 1] - vyi;
                const double uz = p.vel[3 * (int64_t)j + 2] - vzi;
                const double du = dx * ux + dy * uy + dz * uz;
                const double c3 = 3.0 * du * inv2;
                const double kd = -m * slope * du * inv * inv3;   // m (dK/dt) / s^3
                jx += mk3 * (ux - c3 * dx) + kd * dx;
                jy += mk3 * (uy - c3 * dy) + kd * dy;
                jz += mk3 * (uz - c3 * dz) + kd * dz;
            }
            if (POT) ph += m * (-inv - phi_regular(cp, s, inv));
        }
    }
    p.acc[3 * slot] = ax;
    p.acc[3 * slot + 1] = ay;
    p.acc[3 * slot + 2] = az;
    if (JERK) {
        p.jerk[3 * slot] = jx;
        p.jerk[3 * slot + 1] = jy;
        p.jerk[3 * slot + 2] = jz;
    }
    if (POT) p.pot[slot] = ph;
    if (bad) atomicOr(p.err, bad);
}

}  // namespace

void launch_irregular(const IrrParams& p, hipStream_t s) {
    if (p.n_tgt <= 0) return;
    const dim3 grid((unsigned)((p.n_tgt + 255) / 256)), block(256);
    const bool jerk = p.jerk != nullptr, pot = p.pot != nullptr;
    if (jerk && pot) hipLaunchKernelGGL((k_irregular<true, true>), grid, block, 0, s, p);
    else if (jerk) hipLaunchKernelGGL((k_irregular<true, false>), grid, block, 0, s, p);
    else if (pot) hipLaunchKernelGGL((k_irregular<false, true>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((k_irregular<false, false>), grid, block, 0, s, p);
}

}  // namespace pbh
