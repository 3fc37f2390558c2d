// build.hip -- octree construction on gfx950.
//
// Steps (Barnes-Hut tree of Section 2.4 of Arnold, Baumgardt & Wang 2021):
//   bbox     per-cluster bounding box and NaN/Inf check (two-level reduction)
//   keys     cluster id above D-bit-per-axis Morton codes (x, y, z interleaved)
//   sort     stable radix sort (sort.hip) -> sorted keys and permutation
//   gather   sorted FP64 SoA copies of x, y, z, m
//   topology a node is a run of sorted particles sharing a key prefix whose
//            parent holds more than n_leaf particles; each particle knows the
//            levels of the nodes it starts, so one scan numbers the nodes in
//            pre-order; a one-pass counting sort by level then gives the
//            breadth-first order in which every node's children are contiguous
//   moments  bottom-up, one launch per level: M, centre of mass, traceless
//            quadrupole about it (parallel-axis sums over children), tight box
//   groups   tree-bounded runs of <= n_crit sorted particles (rule at k_group_pass)
//
// FP64 arithmetic that decides the tree (keys, moments) is evaluated without
// fused multiply-add so it rounds exactly as written.
#include "pbh_internal.hpp"

namespace pbh {

namespace {

constexpr int BB_T = 256;

// ------------------------------------------------------------------ bbox
__global__ __launch_bounds__(BB_T) void k_bbox_part(const double* __restrict__ pos,
                                                    const double* __restrict__ mass,
                                                    const int64_t* __restrict__ range,
                                                    double* __restrict__ part,
                                                    int32_t* __restrict__ bad) {
    __shared__ double s_v[6][BB_T];
    __shared__ int s_bad;
    const int t = threadIdx.x;
    if (t == 0) s_bad = 0;
    const int64_t b0 = range[2 * blockIdx.x], b1 = range[2 * blockIdx.x + 1];
    double lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    double hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    int nf = 0;
    for (int64_t i = b0 + t; i < b1; i += BB_T) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2], mm = mass[i];
        nf |= !(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(mm));
        lo0 = fmin(lo0, x); lo1 = fmin(lo1, y); lo2 = fmin(lo2, z);
        hi0 = fmax(hi0, x); hi1 = fmax(hi1, y); hi2 = fmax(hi2, z);
    }
    s_v[0][t] = lo0; s_v[1][t] = lo1; s_v[2][t] = lo2;
    s_v[3][t] = hi0; s_v[4][t] = hi1; s_v[5][t] = hi2;
    __syncthreads();
    if (nf) atomicOr(&s_bad, 1);
    for (int o = BB_T / 2; o > 0; o >>= 1) {
        if (t < o) {
            for (int k = 0; k < 3; ++k) s_v[k][t] = fmin(s_v[k][t], s_v[k][t + o]);
            for (int k = 3; k < 6; ++k) s_v[k][t] = fmax(s_v[k][t], s_v[k][t + o]);
        }
        __syncthreads();
    }
    if (t < 6) part[6 * blockIdx.x + t] = s_v[t][0];
    if (t == 0) bad[blockIdx.x] = s_bad;
}

// one block per cluster; blocks of cluster c are [cblk[c], cblk[c+1]). min and
// max are exact, so the reduction order does not matter.
__global__ __launch_bounds__(BB_T) void k_bbox_final(const double* __restrict__ part,
                                                     const int32_t* __restrict__ bad,
                                                     const int32_t* __restrict__ cblk, int nc,
                                                     double* __restrict__ box,
                                                     unsigned long long* __restrict__ cnt) {
    __shared__ double s_v[6][BB_T];
    __shared__ int s_bad;
    const int c = blockIdx.x, t = threadIdx.x;
    if (t == 0) s_bad = 0;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int nf = 0;
    for (int b = cblk[c] + t; b < cblk[c + 1]; b += BB_T) {
        for (int k = 0; k < 3; ++k) v[k] = fmin(v[k], part[6 * b + k]);
        for (int k = 3; k < 6; ++k) v[k] = fmax(v[k], part[6 * b + k]);
        nf |= bad[b];
    }
    for (int k = 0; k < 6; ++k) s_v[k][t] = v[k];
    __syncthreads();
    if (nf) atomicOr(&s_bad, 1);
    for (int o = BB_T / 2; o > 0; o >>= 1) {
        if (t < o) {
            for (int k = 0; k < 3; ++k) s_v[k][t] = fmin(s_v[k][t], s_v[k][t + o]);
            for (int k = 3; k < 6; ++k) s_v[k][t] = fmax(s_v[k][t], s_v[k][t + o]);
        }
        __syncthreads();
    }
    if (t < 6) box[6 * c + t] = s_v[t][0];
    if (t == 0 && s_bad) atomicOr(&cnt[kErr], kErrNonFinite);
}

// ------------------------------------------------------------------ keys
__device__ inline uint64_t spread_bits3(uint64_t v) {
    // spread the low 21 bits of v to every third bit
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ __launch_bounds__(BB_T) void k_keys(const double* __restrict__ pos,
                                               const int64_t* __restrict__ range,
                                               const int32_t* __restrict__ blk_cluster,
                                               const double* __restrict__ box, int D,
                                               uint64_t* __restrict__ keys) {
#pragma clang fp contract(off)
    const int c = blk_cluster[blockIdx.x];
    const int64_t b0 = range[2 * blockIdx.x], b1 = range[2 * blockIdx.x + 1];
    const double lo0 = box[6 * c], lo1 = box[6 * c + 1], lo2 = box[6 * c + 2];
    double L = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double e = box[6 * c + 3 + k] - box[6 * c + k];
        if (e > L) L = e;
    }
    if (L == 0.0) L = 1.0;
    const double scale = ldexp(1.0, D) / L;
    const int64_t maxc = ((int64_t)1 << D) - 1;
    const uint64_t cid = (uint64_t)c << (3 * D);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += BB_T) {
        const double v[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        const double lo[3] = {lo0, lo1, lo2};
        uint64_t key = 0;
        for (int k = 0; k < 3; ++k) {
            int64_t q = (int64_t)floor((v[k] - lo[k]) * scale);
            q = q > maxc ? maxc : (q < 0 ? 0 : q);
            key |= spread_bits3((uint64_t)q) << (2 - k);
        }
        keys[i] = cid | key;
    }
}

__global__ void k_gather(const double* __restrict__ pos, const double* __restrict__ mass,
                         const int32_t* __restrict__ perm, int64_t n, double* __restrict__ x,
                         double* __restrict__ y, double* __restrict__ z, double* __restrict__ m) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[k];
        x[k] = pos[3 * i];
        y[k] = pos[3 * i + 1];
        z[k] = pos[3 * i + 2];
        m[k] = mass[i];
    }
}

// -------------------------------------------------------------- topology
// Key layout: [cluster id | D levels of 3 bits]. Level l >= 1 prefix = key >> 3(D-l).
__device__ inline uint64_t prefix(uint64_t key, int l, int D) { return key >> (3 * (D - l)); }

__device__ inline int cluster_of(uint64_t key, int D) { return (int)(key >> (3 * D)); }

// Number of nodes started by sorted particle i and the first level.
__global__ void k_topo_count(const uint64_t* __restrict__ keys, const int64_t* __restrict__ cl_off,
                             int64_t n, int D, int n_leaf, int32_t* __restrict__ p_first,
                             int32_t* __restrict__ p_nn) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[i];
        const int c = cluster_of(key, D);
        const int64_t cs = cl_off[c], ce = cl_off[c + 1];
        int lf;
        if (i == cs) {
            lf = 0;
        } else {
            const uint64_t x = key ^ keys[i - 1];
            if (x == 0) {
                p_first[i] = D + 1;
                p_nn[i] = 0;
                continue;
            }
            const int h = 63 - __clzll(x);
            lf = D - h / 3;
            // the parent run (level lf-1) contains i-1 and i: it must hold more than n_leaf
            const uint64_t pp = prefix(key, lf - 1, D);
            int64_t a = i - 1, b = i + 1;
            while (a > cs && b - a <= n_leaf && prefix(keys[a - 1], lf - 1, D) == pp) --a;
            while (b < ce && b - a <= n_leaf && prefix(keys[b], lf - 1, D) == pp) ++b;
            if (b - a <= n_leaf) {
                p_first[i] = lf;
                p_nn[i] = 0;
                continue;
            }
        }
        // levels lf+1.. exist while the run of level l-1 starting at i holds > n_leaf
        int last = lf;
        for (int l = lf + 1; l <= D; ++l) {
            const int64_t j = i + n_leaf;
            if (j < ce && prefix(keys[j], l - 1, D) == prefix(key, l - 1, D)) last = l;
            else break;
        }
        p_first[i] = lf;
        p_nn[i] = last - lf + 1;
    }
}

// end of the level-l run that starts at i (exclusive)
__device__ inline int64_t run_end(const uint64_t* keys, int64_t i, int64_t ce, int l, int D) {
    if (l == 0) return ce;
    const uint64_t p = prefix(keys[i], l, D);
    int64_t step = 1, lo = i, hi;
    // exponential search for the first index with a different prefix
    for (;;) {
        hi = lo + step;
        if (hi >= ce || prefix(keys[hi], l, D) != p) break;
        lo = hi;
        step <<= 1;
    }
    if (hi > ce) hi = ce;
    // invariant: keys[lo] has prefix p; keys[hi] (if < ce) does not
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (prefix(keys[mid], l, D) == p) lo = mid; else hi = mid;
    }
    return hi;
}

// start of the level-l run containing i
__device__ inline int64_t run_start(const uint64_t* keys, int64_t i, int64_t cs, int l, int D) {
    if (l == 0) return cs;
    const uint64_t p = prefix(keys[i], l, D);
    int64_t step = 1, hi = i, lo;
    for (;;) {
        lo = hi - step;
        if (lo < cs || prefix(keys[lo], l, D) != p) break;
        hi = lo;
        step <<= 1;
    }
    if (lo < cs - 1) lo = cs - 1;
    // keys[hi] has prefix p; keys[lo] (if >= cs) does not
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (prefix(keys[mid], l, D) == p) hi = mid; else lo = mid;
    }
    return hi;
}

// One thread per node (pre-order index v): its first particle i is the last
// with p_base[i] <= v (binary search), and it is i's (v - p_base[i])-th node
// from level p_first[i] down. (A particle that starts nodes on many levels --
// the first of a cluster starts one on every level -- would otherwise search
// the runs of all of them in turn.)
__global__ void k_topo_emit(const uint64_t* __restrict__ keys, const int64_t* __restrict__ cl_off,
                            int64_t n, int D, int n_leaf, const int32_t* __restrict__ p_first,
                            const int32_t* __restrict__ p_base, int64_t cap,
                            int32_t* __restrict__ pre_begin, int32_t* __restrict__ pre_count,
                            int32_t* __restrict__ pre_level, int32_t* __restrict__ pre_nchild,
                            uint64_t* __restrict__ lvl_key, unsigned long long* __restrict__ cnt) {
    const int64_t total = p_base[n];
    if (total > cap && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&cnt[kErr], kErrNodeCap);
    const int64_t m = total < cap ? total : cap;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < m;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;   // p_base[lo] <= v < p_base[hi]
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)p_base[mid] <= v) lo = mid;
            else hi = mid;
        }
        const int64_t i = lo;
        const int k = (int)(v - p_base[i]);
        const uint64_t key = keys[i];
        const int c = cluster_of(key, D);
        const int64_t cs = cl_off[c], ce = cl_off[c + 1];
        const int l = p_first[i] + k;
        const int64_t e = run_end(keys, i, ce, l, D);
        pre_begin[v] = (int32_t)i;
        pre_count[v] = (int32_t)(e - i);
        pre_level[v] = l;
        lvl_key[v] = (uint64_t)l;
        // register with the parent: its node index is known from the particle
        // that starts it (i itself for k > 0)
        if (l > 0) {
            int64_t parent;
            if (k > 0) {
                parent = v - 1;
            } else {
                const int64_t s = run_start(keys, i, cs, l - 1, D);
                parent = (int64_t)p_base[s] + (l - 1 - p_first[s]);
            }
            if (parent < cap) atomicAdd(&pre_nchild[parent], 1);
        }
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_i32(int32_t* __restrict__ p, const int32_t* __restrict__ n_dev, int64_t cap) {
    const int64_t n = min(cap, (int64_t)*n_dev);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// breadth-first level offsets: lvl_off[l] = first sorted slot with level >= l
__global__ void k_level_offsets(const uint64_t* __restrict__ lvl_sorted,
                                const int32_t* __restrict__ n_dev, int64_t cap,
                                int32_t* __restrict__ lvl_off, unsigned long long* __restrict__ cnt) {
    const int l = threadIdx.x;
    const int64_t n = min(cap, (int64_t)*n_dev);
    if (l <= kMaxLevels) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (lvl_sorted[mid] < (uint64_t)l) lo = mid + 1; else hi = mid;
        }
        lvl_off[l] = (int32_t)lo;
    }
    if (l == 0) {
        cnt[kCntNodes] = (unsigned long long)n;
        cnt[kCntMaxLevel] = n ? lvl_sorted[n - 1] : 0ull;
    }
}

__global__ void k_invert(const int32_t* __restrict__ bfs2pre, const int32_t* __restrict__ n_dev,
                         int64_t cap, int32_t* __restrict__ pre2bfs) {
    const int64_t n = min(cap, (int64_t)*n_dev);
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n;
         b += (int64_t)gridDim.x * blockDim.x)
        pre2bfs[bfs2pre[b]] = (int32_t)b;
}

__global__ void k_nodes_init(const int32_t* __restrict__ bfs2pre, const int32_t* __restrict__ pre2bfs,
                             const int32_t* __restrict__ n_dev, int64_t cap,
                             const int32_t* __restrict__ pre_begin, const int32_t* __restrict__ pre_count,
                             const int32_t* __restrict__ pre_nchild, WNode* __restrict__ node,
                             unsigned long long* __restrict__ cnt) {
    const int64_t n = min(cap, (int64_t)*n_dev);
    unsigned long long leaves = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = bfs2pre[b];
        // pre-order: the first child follows its parent (guarded for a truncated node list)
        const int32_t nc = (p + 1 < n) ? pre_nchild[p] : 0;
        WNode& w = node[b];
        w.begin = pre_begin[p];
        w.count = pre_count[p];
        w.nchild = nc;
        w.first_child = nc ? pre2bfs[p + 1] : -1;
        leaves += (nc == 0);
    }
    // one atomic per block: a single counter serialises same-address atomics
    __shared__ unsigned long long s_leaves;
    if (threadIdx.x == 0) s_leaves = 0;
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) leaves += __shfl_xor(leaves, o, 64);
    if ((threadIdx.x & 63) == 0 && leaves) atomicAdd(&s_leaves, leaves);
    __syncthreads();
    if (threadIdx.x == 0 && s_leaves) atomicAdd(&cnt[kCntLeaves], s_leaves);
}

// ----------------------------------------------------------------- moments
// One node per thread for the nodes of one level. Leaves sum their particles,
// inner nodes their (contiguous) children, in order: M, the mass-weighted
// centre, the tight box, then the traceless quadrupole about the new centre
// (children's own quadrupoles shifted by the parallel-axis terms).
//
// A node with at most 8 parts (every inner node; leaves up to n_leaf = 8)
// loads all parts first, with indices clamped into the node so every load is
// valid and can be issued at once; the sums then run over the parts in order,
// exactly as in the general loop below, so both paths round alike.
constexpr int kMomFast = 8;

struct MomOut {
    double M, com[3], lo[3], hi[3], q[6];
};

__device__ inline void moments_small(const WNode& w, bool leaf, int nsub, const double* __restrict__ x,
                                     const double* __restrict__ y, const double* __restrict__ z,
                                     const double* __restrict__ m, const WNode* __restrict__ node,
                                     const Mom64* __restrict__ q64, MomOut& o) {
#pragma clang fp contract(off)
    double mu[kMomFast], cu[3][kMomFast], lu[3][kMomFast], hu[3][kMomFast];
#pragma unroll
    for (int k = 0; k < kMomFast; ++k) {
        const int u = k < nsub ? k : nsub - 1;
        if (leaf) {
            const int j = w.begin + u;
            mu[k] = m[j]; cu[0][k] = x[j]; cu[1][k] = y[j]; cu[2][k] = z[j];
            for (int d = 0; d < 3; ++d) { lu[d][k] = cu[d][k]; hu[d][k] = cu[d][k]; }
        } else {
            const int c = w.first_child + u;
            mu[k] = q64[c].M;
            for (int d = 0; d < 3; ++d) {
                cu[d][k] = node[c].com[d];
                lu[d][k] = node[c].lo[d];
                hu[d][k] = node[c].hi[d];
            }
        }
    }
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int k = 0; k < kMomFast; ++k) {
        if (k < nsub) {
            M = M + mu[k];
            sx = sx + mu[k] * cu[0][k];
            sy = sy + mu[k] * cu[1][k];
            sz = sz + mu[k] * cu[2][k];
            for (int d = 0; d < 3; ++d) {
                if (k == 0 || lu[d][k] < o.lo[d]) o.lo[d] = lu[d][k];
                if (k == 0 || hu[d][k] > o.hi[d]) o.hi[d] = hu[d][k];
            }
        }
    }
    if (M > 0.0) {
        o.com[0] = sx / M; o.com[1] = sy / M; o.com[2] = sz / M;
    } else {
        for (int d = 0; d < 3; ++d) o.com[d] = (o.lo[d] + o.hi[d]) * 0.5;
    }
    o.M = M;
    double qc[6][kMomFast];
#pragma unroll
    for (int k = 0; k < kMomFast; ++k) {
        const int u = k < nsub ? k : nsub - 1;
        if (leaf) {
            for (int e = 0; e < 6; ++e) qc[e][k] = 0.0;
        } else {
            const Mom64 mc = q64[w.first_child + u];
            qc[0][k] = mc.qxx; qc[1][k] = mc.qyy; qc[2][k] = mc.qzz;
            qc[3][k] = mc.qxy; qc[4][k] = mc.qxz; qc[5][k] = mc.qyz;
        }
    }
    double q[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kMomFast; ++k) {
        if (k < nsub) {
            const double dx = cu[0][k] - o.com[0], dy = cu[1][k] - o.com[1], dz = cu[2][k] - o.com[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            q[0] = q[0] + (qc[0][k] + mu[k] * (3.0 * dx * dx - r2));
            q[1] = q[1] + (qc[1][k] + mu[k] * (3.0 * dy * dy - r2));
            q[2] = q[2] + (qc[2][k] + mu[k] * (3.0 * dz * dz - r2));
            q[3] = q[3] + (qc[3][k] + mu[k] * (3.0 * dx * dy));
            q[4] = q[4] + (qc[4][k] + mu[k] * (3.0 * dx * dz));
            q[5] = q[5] + (qc[5][k] + mu[k] * (3.0 * dy * dz));
        }
    }
    for (int e = 0; e < 6; ++e) o.q[e] = q[e];
}

__device__ inline void moments_loop(const WNode& w, bool leaf, int nsub, const double* __restrict__ x,
                                    const double* __restrict__ y, const double* __restrict__ z,
                                    const double* __restrict__ m, const WNode* __restrict__ node,
                                    const Mom64* __restrict__ q64, MomOut& o) {
#pragma clang fp contract(off)
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int u = 0; u < nsub; ++u) {
        double mu, cu[3], lu[3], hu[3];
        if (leaf) {
            const int j = w.begin + u;
            mu = m[j]; cu[0] = x[j]; cu[1] = y[j]; cu[2] = z[j];
            for (int k = 0; k < 3; ++k) { lu[k] = cu[k]; hu[k] = cu[k]; }
        } else {
            const int c = w.first_child + u;
            mu = q64[c].M;
            for (int k = 0; k < 3; ++k) {
                cu[k] = node[c].com[k];
                lu[k] = node[c].lo[k];
                hu[k] = node[c].hi[k];
            }
        }
        M = M + mu;
        sx = sx + mu * cu[0];
        sy = sy + mu * cu[1];
        sz = sz + mu * cu[2];
        for (int k = 0; k < 3; ++k) {
            if (u == 0 || lu[k] < o.lo[k]) o.lo[k] = lu[k];
            if (u == 0 || hu[k] > o.hi[k]) o.hi[k] = hu[k];
        }
    }
    if (M > 0.0) {
        o.com[0] = sx / M; o.com[1] = sy / M; o.com[2] = sz / M;
    } else {
        for (int k = 0; k < 3; ++k) o.com[k] = (o.lo[k] + o.hi[k]) * 0.5;
    }
    o.M = M;
    double q[6] = {0, 0, 0, 0, 0, 0};
    for (int u = 0; u < nsub; ++u) {
        double mu, cu[3], qc[6];
        if (leaf) {
            const int j = w.begin + u;
            mu = m[j]; cu[0] = x[j]; cu[1] = y[j]; cu[2] = z[j];
            for (int e = 0; e < 6; ++e) qc[e] = 0.0;
        } else {
            const int c = w.first_child + u;
            const Mom64 mc = q64[c];
            mu = mc.M;
            for (int k = 0; k < 3; ++k) cu[k] = node[c].com[k];
            qc[0] = mc.qxx; qc[1] = mc.qyy; qc[2] = mc.qzz;
            qc[3] = mc.qxy; qc[4] = mc.qxz; qc[5] = mc.qyz;
        }
        const double dx = cu[0] - o.com[0], dy = cu[1] - o.com[1], dz = cu[2] - o.com[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        q[0] = q[0] + (qc[0] + mu * (3.0 * dx * dx - r2));
        q[1] = q[1] + (qc[1] + mu * (3.0 * dy * dy - r2));
        q[2] = q[2] + (qc[2] + mu * (3.0 * dz * dz - r2));
        q[3] = q[3] + (qc[3] + mu * (3.0 * dx * dy));
        q[4] = q[4] + (qc[4] + mu * (3.0 * dx * dz));
        q[5] = q[5] + (qc[5] + mu * (3.0 * dy * dz));
    }
    for (int e = 0; e < 6; ++e) o.q[e] = q[e];
}

__device__ inline void moments_node(int64_t b, const double* __restrict__ x, const double* __restrict__ y,
                                    const double* __restrict__ z, const double* __restrict__ m,
                                    WNode* __restrict__ node, Mom64* __restrict__ q64,
                                    Mom32* __restrict__ q32) {
    const WNode w = node[b];
    const bool leaf = w.nchild == 0;
    const int nsub = leaf ? w.count : w.nchild;
    MomOut o;
    if (nsub <= kMomFast) moments_small(w, leaf, nsub, x, y, z, m, node, q64, o);
    else moments_loop(w, leaf, nsub, x, y, z, m, node, q64, o);
    for (int k = 0; k < 3; ++k) {
        node[b].lo[k] = o.lo[k];
        node[b].hi[k] = o.hi[k];
        node[b].com[k] = o.com[k];
    }
    Mom64 r;
    r.M = o.M; r.qxx = o.q[0]; r.qyy = o.q[1]; r.qzz = o.q[2]; r.qxy = o.q[3]; r.qxz = o.q[4];
    r.qyz = o.q[5];
    r.pad = 0.0;
    q64[b] = r;
    Mom32 f;
    f.M = (float)o.M; f.qxx = (float)o.q[0]; f.qyy = (float)o.q[1]; f.qzz = (float)o.q[2];
    f.qxy = (float)o.q[3]; f.qxz = (float)o.q[4]; f.qyz = (float)o.q[5]; f.pad = 0.0f;
    q32[b] = f;
}

__global__ __launch_bounds__(kMomT) void k_moments_level(const int32_t* __restrict__ lvl_off, int level,
                                const double* __restrict__ x, const double* __restrict__ y,
                                const double* __restrict__ z, const double* __restrict__ m,
                                WNode* __restrict__ node, Mom64* __restrict__ q64,
                                Mom32* __restrict__ q32) {
    const int64_t b0 = lvl_off[level], b1 = lvl_off[level + 1];
    for (int64_t b = b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < b1;
         b += (int64_t)gridDim.x * blockDim.x)
        moments_node(b, x, y, z, m, node, q64, q32);
}

// one workgroup, levels l_hi down to l_lo in order (a barrier between levels)
__global__ __launch_bounds__(kMomT) void k_moments_levels(const int32_t* __restrict__ lvl_off, int l_hi,
                                 int l_lo, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ z,
                                 const double* __restrict__ m, WNode* __restrict__ node,
                                 Mom64* __restrict__ q64, Mom32* __restrict__ q32) {
    for (int l = l_hi; l >= l_lo; --l) {
        const int64_t b0 = lvl_off[l], b1 = lvl_off[l + 1];
        for (int64_t b = b0 + threadIdx.x; b < b1; b += blockDim.x)
            moments_node(b, x, y, z, m, node, q64, q32);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ groups
// A node is "big" if it holds more than n_crit particles or its tight box is
// larger (largest side) than the cluster's size limit S. Every big node splits
// into walk groups: a big leaf into runs of n_crit particles, or into single
// particles if its box exceeds S; an inner node packs its consecutive
// children that are not big, greedily in order, into groups of at most
// n_crit particles whose joint box stays within S (a big child interrupts the
// run). A root that is not big is one group. S = 2^5 x 2^e for the octave e
// (2^e <= x < 2^(e+1)) holding the median box size of the groups formed with
// S = infinity (first pass, histogram only). The first particle of each group
// is flagged; a scan of the flags numbers the groups in particle order.
constexpr int kOctaves = 128;
constexpr int kGroupLimitLog2 = 5;

__device__ inline double box_extent(const double* lo, const double* hi) {
    double e = 0.0;
    for (int k = 0; k < 3; ++k)
        if (hi[k] - lo[k] > e) e = hi[k] - lo[k];
    return e;
}

__device__ inline int octave_index(double x) {
    if (!(x > 0.0)) return 0;
    int e = ilogb(x);   // 2^e <= x < 2^(e+1)
    e = e < -64 ? -64 : (e > 63 ? 63 : e);
    return e + 64;
}

// emit one group: first pass -> octave histogram of its box size; second
// pass -> flag its first particle and store its length
template <bool HIST>
__device__ inline void emit_group(int begin, int count, double ext, unsigned* hist, int32_t* flag,
                                  int32_t* len) {
    if (HIST) {
        atomicAdd(&hist[octave_index(ext)], 1u);
    } else {
        flag[begin] = 1;
        len[begin] = count;
    }
}

template <bool HIST>
__global__ __launch_bounds__(256) void k_group_pass(const WNode* __restrict__ node, const uint64_t* __restrict__ lvl,
                             const unsigned long long* __restrict__ n_dev,
                             const uint64_t* __restrict__ keys, int D, int n_crit,
                             const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, const double* __restrict__ cl_S,
                             unsigned* __restrict__ hist, int nc, int reps, int32_t* __restrict__ flag,
                             int32_t* __restrict__ len) {
    const int64_t nn = (int64_t)*n_dev;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nn;
         b += (int64_t)gridDim.x * blockDim.x) {
        const WNode w = node[b];
        const int c = cluster_of(keys[w.begin], D);
        const double S = HIST ? INFINITY : cl_S[c];
        unsigned* h = hist + ((int64_t)(b % reps) * nc + c) * kOctaves;
        const double ext = box_extent(w.lo, w.hi);
        const bool big = w.count > n_crit || ext > S;
        if (lvl[b] == 0 && !big) emit_group<HIST>(w.begin, w.count, ext, h, flag, len);
        if (!big) continue;
        if (w.nchild == 0) {
            if (ext > S) {
                for (int j = w.begin; j < w.begin + w.count; ++j) emit_group<HIST>(j, 1, 0.0, h, flag, len);
            } else {
                for (int s0 = w.begin; s0 < w.begin + w.count; s0 += n_crit) {
                    const int e0 = min(s0 + n_crit, w.begin + w.count);
                    double lo[3], hi[3];
                    for (int j = s0; j < e0; ++j) {
                        const double v[3] = {x[j], y[j], z[j]};
                        for (int k = 0; k < 3; ++k) {
                            if (j == s0 || v[k] < lo[k]) lo[k] = v[k];
                            if (j == s0 || v[k] > hi[k]) hi[k] = v[k];
                        }
                    }
                    emit_group<HIST>(s0, e0 - s0, box_extent(lo, hi), h, flag, len);
                }
            }
            continue;
        }
        int run_begin = 0, run_count = 0;
        double rlo[3] = {0, 0, 0}, rhi[3] = {0, 0, 0};
        // the children's boxes and counts are loaded together (one memory
        // latency per node, not one per child); the loops are unrolled so the
        // arrays stay in registers
        const int nch = w.nchild;
        double alo[8][3], ahi[8][3];
        int acnt[8], abeg[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u < nch) {
                const WNode& ch = node[w.first_child + u];
                for (int k = 0; k < 3; ++k) { alo[u][k] = ch.lo[k]; ahi[u][k] = ch.hi[k]; }
                acnt[u] = ch.count;
                abeg[u] = ch.begin;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u >= nch) break;
            const double clo[3] = {alo[u][0], alo[u][1], alo[u][2]};
            const double chi[3] = {ahi[u][0], ahi[u][1], ahi[u][2]};
            const int cc = acnt[u];
            if (cc > n_crit || box_extent(clo, chi) > S) {
                if (run_count > 0) emit_group<HIST>(run_begin, run_count, box_extent(rlo, rhi), h, flag, len);
                run_count = 0;
                continue;
            }
            double ulo[3], uhi[3];
            for (int k = 0; k < 3; ++k) {
                ulo[k] = (run_count > 0 && rlo[k] < clo[k]) ? rlo[k] : clo[k];
                uhi[k] = (run_count > 0 && rhi[k] > chi[k]) ? rhi[k] : chi[k];
            }
            if (run_count > 0 && (run_count + cc > n_crit || box_extent(ulo, uhi) > S)) {
                emit_group<HIST>(run_begin, run_count, box_extent(rlo, rhi), h, flag, len);
                run_count = 0;
                for (int k = 0; k < 3; ++k) { ulo[k] = clo[k]; uhi[k] = chi[k]; }
            }
            if (run_count == 0) run_begin = abeg[u];
            run_count += cc;
            for (int k = 0; k < 3; ++k) { rlo[k] = ulo[k]; rhi[k] = uhi[k]; }
        }
        if (run_count > 0) emit_group<HIST>(run_begin, run_count, box_extent(rlo, rhi), h, flag, len);
    }
}

// one block per cluster: 8 threads per octave sum the histogram copies (one
// batch of loads each), then the size limit from the median octave of the
// first pass (the first octave whose running count reaches half the groups,
// found by a scan over the octaves)
constexpr int kLimitT = 8 * kOctaves;
__global__ __launch_bounds__(kLimitT) void k_group_limit(const unsigned* __restrict__ hist, int nc,
                                                         int reps, double* __restrict__ cl_S) {
    static_assert(kOctaves == 128, "two waves scan the octaves");
    __shared__ int64_t s_part[8][kOctaves];
    __shared__ int64_t s_w[2];
    const int c = blockIdx.x, t = threadIdx.x, oct = t & (kOctaves - 1), part = t / kOctaves;
    int64_t v = 0;
#pragma unroll 8
    for (int r = part; r < reps; r += 8) v += hist[((int64_t)r * nc + c) * kOctaves + oct];
    s_part[part][oct] = v;
    __syncthreads();
    // the first two waves scan the octaves; every wave reaches both barriers
    const int i = t, lane = i & 63, w = i >> 6;
    int64_t inc = 0;
    v = 0;
    if (i < kOctaves) {
        for (int k = 0; k < 8; ++k) v += s_part[k][i];
        inc = v;   // inclusive running count over octaves 0..i
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) s_w[w] = inc;
    }
    __syncthreads();
    if (i >= kOctaves) return;
    if (w == 1) inc += s_w[0];
    const int64_t total = s_w[0] + s_w[1];
    const int64_t need = (total + 1) / 2;
    // the first octave whose running count reaches need (octave 0 when empty)
    if (inc >= need && inc - v < need) cl_S[c] = ldexp(1.0, i - 64 + kGroupLimitLog2);
    else if (i == 0 && need == 0) cl_S[c] = ldexp(1.0, -64 + kGroupLimitLog2);
}

__global__ void k_fill_u32(unsigned* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_group_fill(const int32_t* __restrict__ gid, const int32_t* __restrict__ len,
                             const uint64_t* __restrict__ keys, const int64_t* __restrict__ cl_off,
                             int64_t n, int D, const int32_t* __restrict__ p_base,
                             const int32_t* __restrict__ pre2bfs, GroupArrays g,
                             unsigned long long* __restrict__ cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (gid[i + 1] == gid[i]) continue;   // not the first particle of a group
        const int32_t k = gid[i];
        const int c = cluster_of(keys[i], D);
        g.begin[k] = (int32_t)i;
        g.count[k] = len[i];
        g.cluster[k] = c;
        g.root[k] = pre2bfs[p_base[cl_off[c]]];   // level-0 node started by the cluster's first particle
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[kCntGroups] = (unsigned long long)gid[n];
}

// One wave per group (persistent over the device-side group count): tight box.
__global__ __launch_bounds__(64) void k_group_box(const unsigned long long* __restrict__ g_dev,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ z, GroupArrays g) {
    const int64_t G = (int64_t)*g_dev;
    const int lane = threadIdx.x;
    for (int64_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
        const int b = g.begin[gi];
        const int cntg = g.count[gi];
        double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int k = lane; k < cntg; k += 64) {
            const double p[3] = {x[b + k], y[b + k], z[b + k]};
            for (int d = 0; d < 3; ++d) {
                v[d] = fmin(v[d], p[d]);
                v[3 + d] = fmax(v[3 + d], p[d]);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            for (int d = 0; d < 3; ++d) {
                v[d] = fmin(v[d], __shfl_xor(v[d], o, 64));
                v[3 + d] = fmax(v[3 + d], __shfl_xor(v[3 + d], o, 64));
            }
        }
        if (lane < 3) {
            g.lo[3 * gi + lane] = lane == 0 ? v[0] : (lane == 1 ? v[1] : v[2]);
            g.hi[3 * gi + lane] = lane == 0 ? v[3] : (lane == 1 ? v[4] : v[5]);
        }
    }
}

inline int grid_for(int64_t n, int threads, int maxb = 4096) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > maxb) b = maxb;
    return (int)b;
}

}  // namespace

void launch_bbox(Dev& d, const BuildCfg& c, const double* pos, const double* mass, int nblk,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_part, dim3(nblk), dim3(BB_T), 0, s, pos, mass,
                       (const int64_t*)d.blk_range, d.blk_part, d.blk_bad);
    // d.blk_cluster is followed by the per-cluster block offsets (see host setup)
    const int32_t* cblk = d.blk_cluster + nblk;
    hipLaunchKernelGGL(k_bbox_final, dim3(c.n_clusters), dim3(BB_T), 0, s,
                       (const double*)d.blk_part, (const int32_t*)d.blk_bad, cblk, c.n_clusters,
                       d.cl_box, d.cnt);
}

void launch_keys(Dev& d, const BuildCfg& c, const double* pos, int nblk, hipStream_t s) {
    // with an odd number of sort passes the keys start in keys_alt, so that the
    // sorted keys and permutation end in (keys, perm) without a copy
    uint64_t* out = (radix_passes(3 * c.D + c.cbits) & 1) ? d.keys_alt : d.keys;
    hipLaunchKernelGGL(k_keys, dim3(nblk), dim3(BB_T), 0, s, pos, (const int64_t*)d.blk_range,
                       (const int32_t*)d.blk_cluster, (const double*)d.cl_box, c.D, out);
}

void launch_key_sort(Dev& d, const BuildCfg& c, hipStream_t s) {
    const int nbits = 3 * c.D + c.cbits;
    if (radix_passes(nbits) & 1)
        radix_sort_pairs(d.keys_alt, d.vals_alt, d.keys, d.perm, c.n, nbits, d.rs_hist, d.scan_tmp, s,
                         true, nullptr, true);
    else
        radix_sort_pairs(d.keys, d.perm, d.keys_alt, d.vals_alt, c.n, nbits, d.rs_hist, d.scan_tmp, s,
                         true);
}

void launch_gather(Dev& d, const BuildCfg& c, const double* pos, const double* mass, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid_for(c.n, 256)), dim3(256), 0, s, pos, mass,
                       (const int32_t*)d.perm, c.n, d.x, d.y, d.z, d.m);
}

void launch_topology(Dev& d, const BuildCfg& c, hipStream_t s) {
    const int64_t n = c.n;
    const int64_t cap = c.node_cap;
    hipLaunchKernelGGL(k_topo_count, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       (const uint64_t*)d.keys, (const int64_t*)d.cl_off, n, c.D, c.n_leaf,
                       d.p_first, d.p_nn);
    exclusive_scan_i32(d.p_nn, d.p_nn, n, d.scan_tmp, s);   // p_nn[n] = node count
    const int32_t* n_nodes = d.p_nn + n;
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(cap, 256)), dim3(256), 0, s, d.pre_nchild,
                       n_nodes, cap);
    hipLaunchKernelGGL(k_topo_emit, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       (const uint64_t*)d.keys, (const int64_t*)d.cl_off, n, c.D, c.n_leaf,
                       (const int32_t*)d.p_first, (const int32_t*)d.p_nn, cap, d.pre_begin,
                       d.pre_count, d.pre_level, d.pre_nchild, d.lvl_key_alt, d.cnt);
    // breadth-first order: stable sort of pre-order nodes by level (one 8-bit
    // pass, from lvl_key_alt into (lvl_key, bfs2pre))
    radix_sort_pairs(d.lvl_key_alt, d.lvl_val, d.lvl_key, d.bfs2pre, cap, 8, d.rs_hist, d.scan_tmp,
                     s, true, n_nodes, true);
    hipLaunchKernelGGL(k_level_offsets, dim3(1), dim3(64), 0, s, (const uint64_t*)d.lvl_key,
                       n_nodes, cap, d.lvl_off, d.cnt);
    hipLaunchKernelGGL(k_invert, dim3(grid_for(cap, 256)), dim3(256), 0, s,
                       (const int32_t*)d.bfs2pre, n_nodes, cap, d.pre2bfs);
    hipLaunchKernelGGL(k_nodes_init, dim3(grid_for(cap, 256, 1024)), dim3(256), 0, s,
                       (const int32_t*)d.bfs2pre, (const int32_t*)d.pre2bfs, n_nodes, cap,
                       (const int32_t*)d.pre_begin, (const int32_t*)d.pre_count,
                       (const int32_t*)d.pre_nchild, d.node, d.cnt);
}

void launch_moments(Dev& d, const BuildCfg& c, hipStream_t s) {
    const int hi = c.mom_hi < c.D ? c.mom_hi : c.D;
    const int lo = c.mom_lo;
    if (hi < c.D)
        hipLaunchKernelGGL(k_moments_levels, dim3(1), dim3(kMomT), 0, s, (const int32_t*)d.lvl_off, c.D,
                           hi + 1, (const double*)d.x, (const double*)d.y, (const double*)d.z,
                           (const double*)d.m, d.node, d.q64, d.q32);
    for (int l = hi; l > lo; --l) {
        const int grid = c.mom_grid[l] > 0 ? c.mom_grid[l] : grid_for(c.node_cap, kMomT, 2048);
        hipLaunchKernelGGL(k_moments_level, dim3(grid), dim3(kMomT), 0, s,
                           (const int32_t*)d.lvl_off, l, (const double*)d.x, (const double*)d.y,
                           (const double*)d.z, (const double*)d.m, d.node, d.q64, d.q32);
    }
    if (lo >= 0)
        hipLaunchKernelGGL(k_moments_levels, dim3(1), dim3(kMomT), 0, s, (const int32_t*)d.lvl_off, lo, 0,
                           (const double*)d.x, (const double*)d.y, (const double*)d.z,
                           (const double*)d.m, d.node, d.q64, d.q32);
}

void launch_groups(Dev& d, const BuildCfg& c, hipStream_t s) {
    const int64_t n = c.n;
    const unsigned long long* n_nodes = d.cnt + kCntNodes;
    const int gb = grid_for(c.node_cap, 256, 2048);
    const int reps = group_hist_reps(c.n_clusters);
    const int64_t hist_len = (int64_t)reps * c.n_clusters * kOctaves;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(hist_len, 256)), dim3(256), 0, s, d.g_hist, hist_len);
    hipLaunchKernelGGL(k_group_pass<true>, dim3(gb), dim3(256), 0, s, (const WNode*)d.node,
                       (const uint64_t*)d.lvl_key, n_nodes, (const uint64_t*)d.keys, c.D, c.n_crit,
                       (const double*)d.x, (const double*)d.y, (const double*)d.z,
                       (const double*)d.cl_S, d.g_hist, c.n_clusters, reps, d.g_flag, d.g_len);
    hipLaunchKernelGGL(k_group_limit, dim3(c.n_clusters), dim3(kLimitT), 0, s,
                       (const unsigned*)d.g_hist, c.n_clusters, reps, d.cl_S);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, d.g_flag, n + 1, 0);
    hipLaunchKernelGGL(k_group_pass<false>, dim3(gb), dim3(256), 0, s, (const WNode*)d.node,
                       (const uint64_t*)d.lvl_key, n_nodes, (const uint64_t*)d.keys, c.D, c.n_crit,
                       (const double*)d.x, (const double*)d.y, (const double*)d.z,
                       (const double*)d.cl_S, d.g_hist, c.n_clusters, reps, d.g_flag, d.g_len);
    exclusive_scan_i32(d.g_flag, d.g_flag, n, d.scan_tmp, s);   // g_flag[n] = group count
    hipLaunchKernelGGL(k_group_fill, dim3(grid_for(n, 256)), dim3(256), 0, s,
                       (const int32_t*)d.g_flag, (const int32_t*)d.g_len, (const uint64_t*)d.keys,
                       (const int64_t*)d.cl_off, n, c.D, (const int32_t*)d.p_nn,
                       (const int32_t*)d.pre2bfs, d.g, d.cnt);
    hipLaunchKernelGGL(k_group_box, dim3(grid_for(n, 64, 32768)), dim3(64), 0, s,
                       (const unsigned long long*)(d.cnt + kCntGroups), (const double*)d.x,
                       (const double*)d.y, (const double*)d.z, d.g);
}

}  // namespace pbh
