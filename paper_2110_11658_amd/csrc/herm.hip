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
//   rounded down to dt_max / 2^k dividing tau'. The start step is
//   eta_s |a + F_R| / |j| with eta_s = 0.01. The corrector and the start step
//   are the standard Hermite ones (Makino & Aarseth 1992); the paper defers
//   both to NBODY6. Expressions are evaluated as written (no contraction).
#include "pbh_internal.hpp"

namespace pbh {

namespace {

__device__ inline double norm3(double x, double y, double z) {
#pragma clang fp contract(off)
    return sqrt(x * x + y * y + z * z);
}

// block step in ticks: dt_max / 2^k not above `want`, dividing tau
__device__ inline int64_t block_step(double want, double dtmax, int64_t tau) {
    double d = dtmax;
    int k = 0;
    while (d > want && k < kHermK) {
        d *= 0.5;
        ++k;
    }
    int64_t t = (int64_t)1 << (kHermK - k);
    while (tau % t != 0) t >>= 1;
    return t;
}

__device__ inline int step_level(int64_t t) {
    int k = 0;
    for (int64_t q = (int64_t)1 << kHermK; q > t; q >>= 1) ++k;
    return k;
}

__global__ __launch_bounds__(256) void k_herm_start(HermParams p) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    double at[3];
    for (int k = 0; k < 3; ++k) at[k] = p.a[3 * i + k] + (p.fr ? p.fr[3 * i + k] : 0.0);
    const double jn = norm3(p.j[3 * i], p.j[3 * i + 1], p.j[3 * i + 2]);
    const double want = jn > 0.0 ? 0.01 * norm3(at[0], at[1], at[2]) / jn : p.dtmax;
    p.tau[i] = 0;
    p.dt[i] = block_step(want, p.dtmax, 0);
}

// Blocks are enqueued in batches without waiting; once every particle has
// reached the end of the regular step the remaining blocks of a batch are
// empty (kHermDone), so the host waits once per batch.
// Block front, in two passes over the per-particle times (16 bytes each):
// the next block time tn = min(tau_i + dt_i) (exact: integer ticks) by a
// two-level reduction, then the list of active particles (tau_i + dt_i = tn)
// with the prediction of each active particle and of every member of its
// neighbour list -- the only states the irregular force of the block reads
// (the other particles keep x, v until their own block).
constexpr int kHermGrid = 1024;   // grid-stride launches

__global__ __launch_bounds__(256) void k_herm_min_part(HermParams p) {
    __shared__ unsigned long long red[4];
    unsigned long long v = ~0ull;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long t = (unsigned long long)(p.tau[i] + p.dt[i]);
        v = t < v ? t : v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) v = red[w] < v ? red[w] : v;
        p.part[blockIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_herm_min_final(HermParams p, int nparts) {
    __shared__ unsigned long long red[4];
    unsigned long long v = ~0ull;
    for (int b = threadIdx.x; b < nparts; b += 256) v = p.part[b] < v ? p.part[b] : v;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) v = red[w] < v ? red[w] : v;
        // past the end of the regular step (every particle at tend): nothing
        // matches the sentinel time, and the block does no work
        const bool done = v > p.tend;
        p.ctl[kHermTn] = done ? ~0ull : v;
        p.ctl[kHermNact] = 0ull;
        if (done) p.ctl[kHermDone] = 1ull;
        else p.ctl[kHermBlocks] += 1ull;
    }
}

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

// the active particle i and the members of its list
__device__ inline void predict_with_list(const HermParams& p, int64_t i, int64_t tn) {
    predict_one(p, i, tn);
    int64_t b = p.off[i], e = p.off[i + 1];
    if (b < 0 || e < b || e > p.cap) return;   // flagged by the force kernel
    for (; b < e; ++b) {
        const int64_t j = p.idx[b];
        if ((uint64_t)j < (uint64_t)p.n) predict_one(p, j, tn);
    }
}

// List the active particles and predict them with their list members (a
// member shared by several lists is written with the same value by each).
__global__ __launch_bounds__(256) void k_herm_active(HermParams p) {
    const int64_t tn = (int64_t)p.ctl[kHermTn];
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < p.n; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        const bool act = i < p.n && p.tau[i] + p.dt[i] == tn;
        const uint64_t b = __ballot(act);
        if (!b) continue;
        const unsigned long long at =
            __shfl(atomicAdd(p.ctl + kHermNact, lane == 0 ? (unsigned long long)__popcll(b) : 0ull), 0, 64);
        if (act) {
            const uint64_t below = lane ? (b & ((~0ull) >> (64 - lane))) : 0ull;
            p.act[at + __popcll(below)] = (int32_t)i;
            predict_with_list(p, i, tn);
        }
    }
}

// Hermite corrector and new block step of the active particles
__global__ __launch_bounds__(256) void k_herm_correct(HermParams p) {
#pragma clang fp contract(off)
    const int64_t nact = (int64_t)p.ctl[kHermNact];
    for (int64_t k0 = (int64_t)blockIdx.x * 256; k0 < nact; k0 += (int64_t)gridDim.x * 256) {
    const int64_t k = k0 + threadIdx.x;
    int level = 0;
    if (k < nact) {
        const int64_t i = p.act[k];
        const int64_t tn = (int64_t)p.ctl[kHermTn];
        const double d = (double)p.dt[i] * p.unit, d2 = d * d, d3 = d2 * d, d4 = d3 * d, d5 = d4 * d;
        double a2[3], a3[3], a2e[3], at[3];
        for (int c = 0; c < 3; ++c) {
            const int64_t q = 3 * i + c;
            const double a1 = p.a1[3 * k + c], j1 = p.j1[3 * k + c];
            const double da = p.a[q] - a1;
            a2[c] = (-6.0 * da - d * (4.0 * p.j[q] + 2.0 * j1)) / d2;
            a3[c] = (12.0 * da + 6.0 * d * (p.j[q] + j1)) / d3;
            p.x[q] = p.xp[q] + d4 / 24.0 * a2[c] + d5 / 120.0 * a3[c];
            p.v[q] = p.vp[q] + d3 / 6.0 * a2[c] + d4 / 24.0 * a3[c];
            p.a[q] = a1;
            p.j[q] = j1;
            a2e[c] = a2[c] + d * a3[c];
            at[c] = a1 + (p.fr ? p.fr[q] : 0.0);
        }
        const double n0 = norm3(at[0], at[1], at[2]);
        const double n1 = norm3(p.j[3 * i], p.j[3 * i + 1], p.j[3 * i + 2]);
        const double n2 = norm3(a2e[0], a2e[1], a2e[2]);
        const double n3 = norm3(a3[0], a3[1], a3[2]);
        const double num = n0 * n2 + n1 * n1, den = n1 * n3 + n2 * n2;
        double want = den > 0.0 ? sqrt(p.eta * num / den) : p.dtmax;
        if (want > 2.0 * d) want = 2.0 * d;
        p.tau[i] = tn;
        p.dt[i] = block_step(want, p.dtmax, tn);
        level = step_level(p.dt[i]);
    }
    // block statistics: particle steps and the deepest level (wave-combined)
    const uint64_t b = __ballot(k < nact);
    int lv = level;
    for (int o = 32; o > 0; o >>= 1) {
        const int w = __shfl_xor(lv, o, 64);
        lv = w > lv ? w : lv;
    }
    if (b) {
        const int lane = threadIdx.x & 63;
        atomicAdd(p.ctl + kHermSteps, lane == 0 ? (unsigned long long)__popcll(b) : 0ull);
        atomicMax(p.ctl + kHermKmax, lane == 0 ? (unsigned long long)lv : 0ull);
    }
    }
}

// pot_tot = pot_r + pot_i
__global__ void k_add(int64_t n, const double* a, const double* b, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

}  // namespace

void launch_herm_start(const HermParams& p, hipStream_t s) {
    hipLaunchKernelGGL(k_herm_start, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p);
}

static unsigned herm_grid(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < kHermGrid ? (g < 1 ? 1 : g) : kHermGrid);
}

int herm_part_len() { return kHermGrid; }

void launch_herm_block_front(const HermParams& p, hipStream_t s) {
    const unsigned g = herm_grid(p.n);
    hipLaunchKernelGGL(k_herm_min_part, dim3(g), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_herm_min_final, dim3(1), dim3(256), 0, s, p, (int)g);
    hipLaunchKernelGGL(k_herm_active, dim3(g), dim3(256), 0, s, p);
}

void launch_herm_correct(const HermParams& p, hipStream_t s) {
    hipLaunchKernelGGL(k_herm_correct, dim3(herm_grid(p.n)), dim3(256), 0, s, p);
}

void launch_add(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b, out);
}

}  // namespace pbh
