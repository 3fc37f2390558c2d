// core.hip -- core quantities from the 6 nearest neighbours of a particle
// sample (gfx950).
//
// Arnold, Baumgardt & Wang (2021) replace the neighbour-list based core
// estimate with a uniform sample of min(N, sqrt(5000 N)) particles whose 6
// nearest neighbours are found directly (Section 3.2), and feed the core
// density to the regularisation parameters R_min = 4 r_h / (N
// rho_core^(1/3)) and dT_min = 0.01 sqrt(eta / 0.02) sqrt(R_min^3)
// (Section 2.5). With the estimator of Casertano & Hut (1985), per
// sampled particle i:
//   rho_i = (sum of the masses of its 5 nearest neighbours) / ((4 pi/3) r_6^3)
// and over the sample x_d = sum rho x / sum rho, r_c^2 = sum rho^2 |x - x_d|^2
// / sum rho^2, rho_core = sum rho^2 / sum rho; N_core counts all particles
// inside r_c, r_h is the half-mass radius about x_d.
//
// The 6 nearest neighbours are exact (ordered by r^2 = (dx*dx + dy*dy) + dz*dz
// in FP64 without FMA, ties to the lower caller index), but found through the
// octree of the last build instead of a scan over all N: one wave per sampled
// particle seeds its list from the 64 particles around it in key order, then
// walks the tree and opens a node only if its box comes within the current
// 6th distance. The box distance is rounded exactly like a pair distance
// (monotone in every step), so it never exceeds the distance of a particle
// inside the box and no neighbour is pruned.
#include "pbh_internal.hpp"
#include "wave.hpp"

namespace pbh {

namespace {

constexpr int kCoreStack = 2048;   // LDS traversal stack of one wave (overflow is flagged)

struct CoreParams {
    int64_t n;
    int64_t ns;
    const int32_t* sample;   // [ns] caller indices
    const WNode* node;       // breadth-first nodes of the last build, root 0
    const double* x;         // sorted coordinates
    const double* y;
    const double* z;
    const int32_t* perm;     // key position -> caller index
    const int32_t* rank;     // caller index -> key position
    const double* mass;      // caller order
    double* rho;             // [ns] out
    unsigned long long* err; // kCore* flag bits
};

__device__ inline double pair_r2(double xj, double yj, double zj, double xi, double yi, double zi) {
#pragma clang fp contract(off)
    const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    return dx * dx + dy * dy + dz * dz;
}

__device__ inline unsigned long long wave_min_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

__device__ inline int wave_min_i32(int v) {
    for (int o = 32; o > 0; o >>= 1) {
        const int w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// The wave's current 6 nearest (wave-uniform), ascending by (r^2, index).
struct Top6 {
    double d[6];
    int id[6];
    int cnt;
    __device__ double bound() const { return cnt < 6 ? __builtin_inf() : d[5]; }
    // (r2, j) would enter the list
    __device__ bool better(double r2, int j) const {
        if (cnt < 6) return true;
        return r2 < d[5] || (r2 == d[5] && j < id[5]);
    }
    __device__ bool has(int j) const {
        bool h = false;
        for (int t = 0; t < 6; ++t) h |= (t < cnt) && id[t] == j;
        return h;
    }
    // insert at the rank of (r2, j), shifting the rest up (static indices only,
    // so the list stays in registers); the 7th entry falls off
    __device__ void insert(double r2, int j) {
        int pos = 0;
#pragma unroll
        for (int t = 0; t < 6; ++t)
            pos += (t < cnt && (d[t] < r2 || (d[t] == r2 && id[t] < j))) ? 1 : 0;
#pragma unroll
        for (int t = 5; t > 0; --t) {
            d[t] = t > pos ? d[t - 1] : (t == pos ? r2 : d[t]);
            id[t] = t > pos ? id[t - 1] : (t == pos ? j : id[t]);
        }
        if (pos == 0) {
            d[0] = r2;
            id[0] = j;
        }
        cnt = cnt < 6 ? cnt + 1 : 6;
    }
    // merge the lanes' candidates (valid lanes with distance r2, index j):
    // the wave minimum enters until no candidate beats the 6th entry
    __device__ void merge(bool valid, double r2, int j) {
        bool c = valid && !has(j);
        for (int it = 0; it < 6; ++it) {
            c = c && better(r2, j);
            if (!__ballot(c)) return;
            const unsigned long long key = c ? (unsigned long long)__double_as_longlong(r2) : ~0ull;
            const unsigned long long mk = wave_min_u64(key);
            const int mj = wave_min_i32((c && key == mk) ? j : 0x7fffffff);
            insert(__longlong_as_double((long long)mk), mj);
            c = c && !(key == mk && j == mj);
        }
    }
};

__global__ __launch_bounds__(64) void k_core_knn(CoreParams p) {
    __shared__ int s_stack[kCoreStack];
    __shared__ int s_ex[64];
    __shared__ int s_beg[64];
    const int lane = threadIdx.x;
    const int64_t s = blockIdx.x;
    const int64_t i = p.sample[s];
    if ((uint64_t)i >= (uint64_t)p.n) {   // wave-uniform
        if (lane == 0) p.rho[s] = __builtin_nan("");
        atomicOr(p.err, lane == 0 ? kCoreBadSample : 0ull);
        return;
    }
    const int64_t k = p.rank[i];
    const double xi = p.x[k], yi = p.y[k], zi = p.z[k];
    Top6 T;
    T.cnt = 0;
    for (int t = 0; t < 6; ++t) {
        T.d[t] = 0.0;
        T.id[t] = 0;
    }
    // seed: the 64 key positions around i (n >= 7 gives at least 6 others)
    {
        int64_t lo = k - 32;
        if (lo + 64 > p.n) lo = p.n - 64;
        if (lo < 0) lo = 0;
        const int64_t q = lo + lane;
        const bool ok = q < p.n && q != k;
        const int64_t qq = q < p.n ? q : k;
        const double r2 = pair_r2(p.x[qq], p.y[qq], p.z[qq], xi, yi, zi);
        T.merge(ok, r2, p.perm[qq]);
    }
    // tree walk from the root, opening nodes within the current 6th distance
    bool overflow = false;
    s_stack[0] = 0;
    int top = 1;
    while (top > 0) {
        __syncthreads();
        const int npop = uni(top < 64 ? top : 64);
        top -= npop;
        const bool has = lane < npop;
        const int nd = has ? s_stack[top + lane] : 0;
        __syncthreads();
        const WNode w = p.node[nd];
        const double c[3] = {xi, yi, zi};
        const bool open = has && !(box_pt_d2(w.lo, w.hi, c) > T.bound());
        const bool leaf = w.nchild == 0;
        const int nch = (open && !leaf) ? w.nchild : 0;
        const int incl = wave_incl_scan(nch, lane);
        const int tot = last_lane(incl);
        if (top + tot > kCoreStack) {
            overflow = true;
            break;
        }
        for (int q = 0; q < nch; ++q) s_stack[top + incl - nch + q] = w.first_child + q;
        top = uni(top + tot);
        // particles of opened leaves, 64 at a time
        const int v = (open && leaf) ? w.count : 0;
        const int li = wave_incl_scan(v, lane);
        const int total = last_lane(li);
        if (total == 0) continue;
        __syncthreads();
        s_ex[lane] = li - v;
        s_beg[lane] = w.begin;
        __syncthreads();
        for (int base = 0; base < total; base += 64) {
            const int sidx = base + lane;
            int f = 0;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1)
                if (s_ex[f + st] <= sidx) f += st;
            const bool ok = sidx < total;
            const int64_t q = ok ? (int64_t)s_beg[f] + (sidx - s_ex[f]) : k;
            const double r2 = pair_r2(p.x[q], p.y[q], p.z[q], xi, yi, zi);
            T.merge(ok && q != k, r2, p.perm[q]);
        }
    }
    if (overflow) atomicOr(p.err, lane == 0 ? kCoreStackFull : 0ull);
    if (lane == 0) {
#pragma clang fp contract(off)
        double m5 = 0.0;
        for (int t = 0; t < 5; ++t) m5 += p.mass[T.id[t]];
        const double r6 = sqrt(T.d[5]);
        p.rho[s] = overflow ? __builtin_nan("") : m5 / (4.0 / 3.0 * 3.14159265358979323846 * (T.d[5] * r6));
    }
}

// rank[perm[k]] = k
__global__ void k_core_rank(int64_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ rank) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) rank[perm[k]] = (int32_t)k;
}

// Sums over the sample in two levels, each in a fixed order: a workgroup of
// kStatT threads sums a chunk of kStatCh consecutive samples (thread t takes
// samples t, t + kStatT, ... of the chunk in that order, loads issued
// together, then a fixed tree over the threads), and one workgroup sums the
// chunk totals in chunk order the same way. First the density centre
// (sum rho, sum rho x), then the core density and radius (sum rho^2,
// sum rho^2 |x - x_d|^2). out: [0..2] x_d, [3] rho_core, [4] r_c, ...
// part: [0] the sum of rho; [8 + 4 c ..] the totals of chunk c.
constexpr int kStatT = 256;
constexpr int kStatB = 8;
constexpr int kStatCh = kStatT * kStatB;   // samples per chunk

__device__ inline double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int h = kStatT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    return red[0];
}

// the samples of thread t in chunk c: caller index (-1: none or out of range,
// flagged by the search and never read), density and position
__device__ inline void chunk_samples(int64_t n, int64_t ns, const int32_t* __restrict__ sample,
                                     const double* __restrict__ pos, const double* __restrict__ rho,
                                     int64_t c, int t, int64_t (&iv)[kStatB], double (&rv)[kStatB],
                                     double (&xv)[kStatB], double (&yv)[kStatB], double (&zv)[kStatB]) {
#pragma unroll
    for (int u = 0; u < kStatB; ++u) {
        const int64_t s = c * kStatCh + t + (int64_t)kStatT * u;
        iv[u] = s < ns ? (int64_t)sample[s] : -1;
    }
#pragma unroll
    for (int u = 0; u < kStatB; ++u) {
        const int64_t s = c * kStatCh + t + (int64_t)kStatT * u;
        const bool ok = (uint64_t)iv[u] < (uint64_t)n;
        if (!ok) iv[u] = -1;
        const int64_t i = ok ? iv[u] : 0;
        rv[u] = ok ? rho[s] : 0.0;
        xv[u] = pos[3 * i];
        yv[u] = pos[3 * i + 1];
        zv[u] = pos[3 * i + 2];
    }
}

__global__ __launch_bounds__(kStatT) void k_core_sum1(int64_t n, int64_t ns, const int32_t* __restrict__ sample,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ rho, double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[kStatT];
    int64_t iv[kStatB];
    double rv[kStatB], xv[kStatB], yv[kStatB], zv[kStatB];
    chunk_samples(n, ns, sample, pos, rho, blockIdx.x, threadIdx.x, iv, rv, xv, yv, zv);
    double sr = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int u = 0; u < kStatB; ++u) {
        if (iv[u] < 0) continue;
        sr += rv[u];
        sx += rv[u] * xv[u];
        sy += rv[u] * yv[u];
        sz += rv[u] * zv[u];
    }
    sr = block_sum(sr, red);
    sx = block_sum(sx, red);
    sy = block_sum(sy, red);
    sz = block_sum(sz, red);
    if (threadIdx.x == 0) {
        double* q = part + 8 + 4 * (int64_t)blockIdx.x;
        q[0] = sr; q[1] = sx; q[2] = sy; q[3] = sz;
    }
}

// totals of the first k (<= 4) values of every chunk, in chunk order
template <int K>
__device__ inline void chunk_totals(int64_t nc, const double* __restrict__ part, double* red, double (&tot)[K]) {
    double v[K];
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int64_t c = threadIdx.x; c < nc; c += kStatT)
        for (int k = 0; k < K; ++k) v[k] += part[8 + 4 * c + k];
    for (int k = 0; k < K; ++k) tot[k] = block_sum(v[k], red);
}

__global__ __launch_bounds__(kStatT) void k_core_centre(int64_t nc, double* __restrict__ part,
                                                        double* __restrict__ out) {
#pragma clang fp contract(off)
    __shared__ double red[kStatT];
    double tot[4];
    chunk_totals<4>(nc, part, red, tot);
    if (threadIdx.x == 0) {
        part[0] = tot[0];
        out[0] = tot[1] / tot[0];
        out[1] = tot[2] / tot[0];
        out[2] = tot[3] / tot[0];
    }
}

__global__ __launch_bounds__(kStatT) void k_core_sum2(int64_t n, int64_t ns, const int32_t* __restrict__ sample,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ rho,
                                                      const double* __restrict__ out, double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double red[kStatT];
    const double xd = out[0], yd = out[1], zd = out[2];
    int64_t iv[kStatB];
    double rv[kStatB], xv[kStatB], yv[kStatB], zv[kStatB];
    chunk_samples(n, ns, sample, pos, rho, blockIdx.x, threadIdx.x, iv, rv, xv, yv, zv);
    double s2 = 0, s2d = 0;
#pragma unroll
    for (int u = 0; u < kStatB; ++u) {
        if (iv[u] < 0) continue;
        const double r = rv[u];
        const double dx = xv[u] - xd, dy = yv[u] - yd, dz = zv[u] - zd;
        const double dd = dx * dx + dy * dy + dz * dz;
        s2 += r * r;
        s2d += r * r * dd;
    }
    s2 = block_sum(s2, red);
    s2d = block_sum(s2d, red);
    if (threadIdx.x == 0) {
        double* q = part + 8 + 4 * (int64_t)blockIdx.x;
        q[0] = s2; q[1] = s2d;
    }
}

__global__ __launch_bounds__(kStatT) void k_core_radius(int64_t nc, const double* __restrict__ part,
                                                        double* __restrict__ out) {
#pragma clang fp contract(off)
    __shared__ double red[kStatT];
    double tot[2];
    chunk_totals<2>(nc, part, red, tot);
    if (threadIdx.x == 0) {
        out[3] = tot[0] / part[0];        // rho_core
        out[4] = sqrt(tot[1] / tot[0]);   // r_c
    }
}

// distance keys about x_d for the half-mass radius, and the core count (one
// device atomic per workgroup: atomics on one address serialise)
constexpr int kDistGrid = 1024;

__global__ __launch_bounds__(256) void k_core_dist(int64_t n, const double* __restrict__ pos,
                                                   const double* __restrict__ st,
                                                   uint64_t* __restrict__ key,
                                                   unsigned long long* __restrict__ ncore) {
#pragma clang fp contract(off)
    __shared__ unsigned long long s_cnt[4];
    const double xd = st[0], yd = st[1], zd = st[2], rc = st[4];
    unsigned long long cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double dx = pos[3 * i] - xd, dy = pos[3 * i + 1] - yd, dz = pos[3 * i + 2] - zd;
        const double dd = dx * dx + dy * dy + dz * dz;
        cnt += dd < rc * rc ? 1ull : 0ull;
        key[i] = (uint64_t)__double_as_longlong(dd);   // dd >= 0: bit order is numeric order
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_cnt[w] = cnt;
    __syncthreads();
    if (w == 0) {   // all lanes of wave 0 take part; lane 0 adds the workgroup's count
        const unsigned long long tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        if (tot) atomicAdd(ncore, lane == 0 ? tot : 0ull);
    }
}

// masses in distance order, summed per block of kCrossBlk (fixed order)
constexpr int kCrossBlk = 1024;

__global__ __launch_bounds__(kCrossBlk) void k_core_bsum(int64_t n, const int32_t* __restrict__ order,
                                                         const double* __restrict__ mass,
                                                         double* __restrict__ bsum) {
    __shared__ double red[kCrossBlk];
    const int64_t i = (int64_t)blockIdx.x * kCrossBlk + threadIdx.x;
    red[threadIdx.x] = i < n ? mass[order[i]] : 0.0;
    __syncthreads();
    for (int h = kCrossBlk / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Half-mass radius (first distance at which the running mass reaches half the
// total, scanning blocks then one block in order) and the regularisation
// parameters. The scans are serial (thread 0, in order) over values that the
// workgroup first stages in LDS, kCrossBlk at a time.
__global__ __launch_bounds__(kCrossBlk) void k_core_final(int64_t n, int64_t nblk, const int32_t* __restrict__ order,
                                                          const uint64_t* __restrict__ key,
                                                          const double* __restrict__ mass,
                                                          const double* __restrict__ bsum,
                                                          const unsigned long long* ncore, double eta,
                                                          double* __restrict__ st) {
#pragma clang fp contract(off)
    __shared__ double v[kCrossBlk];
    __shared__ double s_tot, s_acc;
    __shared__ int64_t s_b;
    __shared__ int s_found;
    const int t = threadIdx.x;
    if (t == 0) {
        s_tot = 0.0;
        s_acc = 0.0;   // running mass of whole blocks before s_b
        s_b = 0;
        s_found = 0;
    }
    for (int64_t c0 = 0; c0 < nblk; c0 += kCrossBlk) {   // total mass
        __syncthreads();
        v[t] = c0 + t < nblk ? bsum[c0 + t] : 0.0;
        __syncthreads();
        if (t == 0) {
            double m = s_tot;
            const int64_t e = nblk - c0 < kCrossBlk ? nblk - c0 : kCrossBlk;
            for (int64_t k = 0; k < e; ++k) m += v[k];
            s_tot = m;
        }
    }
    __syncthreads();
    const double half = 0.5 * s_tot;
    for (int64_t c0 = 0; c0 < nblk; c0 += kCrossBlk) {   // block holding the half-mass point
        __syncthreads();
        if (s_found) break;   // workgroup-uniform
        v[t] = c0 + t < nblk ? bsum[c0 + t] : 0.0;
        __syncthreads();
        if (t == 0) {
            double cum = s_acc;
            int64_t b = c0;
            const int64_t e = c0 + kCrossBlk < nblk ? c0 + kCrossBlk : nblk;
            while (b < nblk - 1 && b < e && cum + v[b - c0] < half) cum += v[(b++) - c0];
            s_acc = cum;
            s_b = b;
            s_found = b < e;   // stopped inside this chunk (or at the last block)
        }
    }
    __syncthreads();
    const int64_t b = s_b;
    const int64_t beg = b * kCrossBlk, end = (b + 1) * kCrossBlk < n ? (b + 1) * kCrossBlk : n;
    v[t] = beg + t < end ? mass[order[beg + t]] : 0.0;
    __syncthreads();
    if (t == 0) {
        double cum = s_acc;
        int64_t kk = beg;
        for (; kk < end - 1; ++kk) {
            cum += v[kk - beg];
            if (cum >= half) break;
        }
        const double rh = sqrt(__longlong_as_double((long long)key[kk]));
        const double rmin = 4.0 * rh / ((double)n * cbrt(st[3]));
        st[5] = (double)*ncore;
        st[6] = rh;
        st[7] = rmin;
        st[8] = 0.01 * sqrt(eta / 0.02) * sqrt(rmin * rmin * rmin);
    }
}

}  // namespace

void launch_core(const CoreLaunch& c, hipStream_t s) {
    const int64_t n = c.n;
    hipLaunchKernelGGL(k_core_rank, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, c.perm, c.rank);
    CoreParams p;
    p.n = n;
    p.ns = c.ns;
    p.sample = c.sample;
    p.node = c.node;
    p.x = c.x; p.y = c.y; p.z = c.z;
    p.perm = c.perm;
    p.rank = c.rank;
    p.mass = c.mass;
    p.rho = c.rho;
    p.err = c.err;
    hipLaunchKernelGGL(k_core_knn, dim3((unsigned)c.ns), dim3(64), 0, s, p);
    const int64_t nc = (c.ns + kStatCh - 1) / kStatCh;   // sample chunks (ns >= 1)
    hipLaunchKernelGGL(k_core_sum1, dim3((unsigned)nc), dim3(kStatT), 0, s, n, c.ns, c.sample, c.pos,
                       (const double*)c.rho, c.bsum);
    hipLaunchKernelGGL(k_core_centre, dim3(1), dim3(kStatT), 0, s, nc, c.bsum, c.stats);
    hipLaunchKernelGGL(k_core_sum2, dim3((unsigned)nc), dim3(kStatT), 0, s, n, c.ns, c.sample, c.pos,
                       (const double*)c.rho, (const double*)c.stats, c.bsum);
    hipLaunchKernelGGL(k_core_radius, dim3(1), dim3(kStatT), 0, s, nc, (const double*)c.bsum, c.stats);
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_core_dist, dim3((unsigned)(nb < kDistGrid ? nb : kDistGrid)), dim3(256), 0, s, n, c.pos,
                       (const double*)c.stats, c.keys, c.ncore);
    radix_sort_pairs(c.keys, c.vals, c.keys_alt, c.vals_alt, n, 64, c.hist, c.scan_tmp, s, true);
    const int64_t nblk = (n + kCrossBlk - 1) / kCrossBlk;
    hipLaunchKernelGGL(k_core_bsum, dim3((unsigned)nblk), dim3(kCrossBlk), 0, s, n, (const int32_t*)c.vals,
                       c.mass, c.bsum);
    hipLaunchKernelGGL(k_core_final, dim3(1), dim3(kCrossBlk), 0, s, n, nblk, (const int32_t*)c.vals,
                       (const uint64_t*)c.keys, c.mass, (const double*)c.bsum,
                       (const unsigned long long*)c.ncore, c.eta, c.stats);
}

// the cross-block sums of the half-mass search, and before them the sample
// sums' chunk totals (n >= the sample size)
int64_t core_bsum_len(int64_t n) {
    const int64_t a = (n + kCrossBlk - 1) / kCrossBlk, b = 8 + 4 * ((n + kStatCh - 1) / kStatCh);
    return a > b ? a : b;
}

}  // namespace pbh
