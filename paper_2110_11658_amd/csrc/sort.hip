// sort.hip -- device-wide exclusive scan and stable LSD radix sort (gfx950).
//
// Scan: launches of fixed size (so they can be captured in a graph): per-tile
// sums, then per-tile scans, each tile adding the sums of the tiles before it
// (summed by its own workgroup while there are at most kScanFuseTiles tiles;
// beyond that a single workgroup scans the tile sums in a launch between).
//
// Radix sort: 8-bit digits. Per pass a tile
// histogram (LDS atomics), a scan of the digit-major histogram table, and a
// stable scatter in which each wave ranks equal digits with one ballot per
// digit bit (match by bits) and the waves of a workgroup are ordered through
// LDS.
#include "pbh_internal.hpp"

namespace pbh {

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_I = 4;   // 1024 elements per tile (2, 8 and 16 built slower at 2^20; 2 leaves the fused path at 4M)
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

__device__ inline int64_t wave_incl_scan64(int64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over a 256-thread block; returns the exclusive prefix, total in *tot
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* s_wave, int64_t* tot) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t inc = wave_incl_scan64(v, lane);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    int64_t base = 0, all = 0;
    for (int k = 0; k < SCAN_T / 64; ++k) {
        if (k < w) base += s_wave[k];
        all += s_wave[k];
    }
    *tot = all;
    __syncthreads();
    return base + inc - v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const T* __restrict__ in, int64_t n,
                                                        int64_t* __restrict__ tmp) {
    __shared__ int64_t s_wave[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k * SCAN_T + threadIdx.x;
        if (i < n) v += (int64_t)in[i];
    }
    int64_t tot;
    block_excl_scan(v, s_wave, &tot);
    if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ tmp, int64_t nb) {
    __shared__ int64_t s_wave[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per;
    int64_t sum = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) sum += tmp[b0 + k];
    int64_t inc = wave_incl_scan64(sum, lane);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    int64_t base = 0, all = 0;
    for (int k = 0; k < 16; ++k) {
        if (k < w) base += s_wave[k];
        all += s_wave[k];
    }
    int64_t run = base + inc - sum;
    for (int64_t k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            int64_t v = tmp[b0 + k];
            tmp[b0 + k] = run;
            run += v;
        }
    }
    if (t == 0) tmp[nb] = all;
}

template <typename T, typename O>
__global__ __launch_bounds__(SCAN_T) void k_scan_down(const T* in, int64_t n,
                                                      const int64_t* __restrict__ tmp, O* out,
                                                      int64_t nb) {
    __shared__ int64_t s_val[SCAN_TILE];
    __shared__ int64_t s_wave[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k * SCAN_T + threadIdx.x;
        s_val[k * SCAN_T + threadIdx.x] = (i < n) ? (int64_t)in[i] : 0;
    }
    __syncthreads();
    int64_t v[SCAN_I];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        v[k] = s_val[threadIdx.x * SCAN_I + k];
        sum += v[k];
    }
    int64_t tot;
    int64_t run = block_excl_scan(sum, s_wave, &tot) + tmp[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        s_val[threadIdx.x * SCAN_I + k] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k * SCAN_T + threadIdx.x;
        if (i < n) out[i] = (O)s_val[k * SCAN_T + threadIdx.x];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (O)tmp[nb];
}

// Per-tile scan with the tile's offset summed here from the tile sums before
// it (tmp[0 .. blockIdx.x), in index order per thread, then across the
// workgroup); the last tile also writes the total to out[n].
constexpr int64_t kScanFuseTiles = 4096;

template <typename T, typename O>
__global__ __launch_bounds__(SCAN_T) void k_scan_down_fused(const T* in, int64_t n,
                                                            const int64_t* __restrict__ tmp, O* out,
                                                            int64_t nb) {
    __shared__ int64_t s_val[SCAN_TILE];
    __shared__ int64_t s_wave[SCAN_T / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t part = 0;
    for (int64_t k = t; k < (int64_t)blockIdx.x; k += SCAN_T) part += tmp[k];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if (lane == 0) s_wave[w] = part;
    __syncthreads();
    int64_t off = 0;
    for (int k = 0; k < SCAN_T / 64; ++k) off += s_wave[k];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k * SCAN_T + t;
        s_val[k * SCAN_T + t] = (i < n) ? (int64_t)in[i] : 0;
    }
    __syncthreads();
    int64_t v[SCAN_I];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        v[k] = s_val[t * SCAN_I + k];
        sum += v[k];
    }
    int64_t tot;
    int64_t run = block_excl_scan(sum, s_wave, &tot) + off;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        s_val[t * SCAN_I + k] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + k * SCAN_T + t;
        if (i < n) out[i] = (O)s_val[k * SCAN_T + t];
    }
    if (blockIdx.x == nb - 1 && t == 0) out[n] = (O)(off + tot);
}

template <typename T, typename O>
void scan_impl(const T* in, O* out, int64_t n, int64_t* tmp, hipStream_t s) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb >= 1 && nb <= kScanFuseTiles) {
        hipLaunchKernelGGL((k_scan_reduce<T>), dim3(nb), dim3(SCAN_T), 0, s, in, n, tmp);
        hipLaunchKernelGGL((k_scan_down_fused<T, O>), dim3(nb), dim3(SCAN_T), 0, s, in, n,
                           (const int64_t*)tmp, out, nb);
        return;
    }
    if (nb == 0) {
        // n == 0: out[0] = 0 through the top kernel with nb = 0
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, (int64_t)0);
        hipLaunchKernelGGL((k_scan_down<T, O>), dim3(1), dim3(SCAN_T), 0, s, in, (int64_t)0,
                           (const int64_t*)tmp, out, (int64_t)0);
        return;
    }
    hipLaunchKernelGGL((k_scan_reduce<T>), dim3(nb), dim3(SCAN_T), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, nb);
    hipLaunchKernelGGL((k_scan_down<T, O>), dim3(nb), dim3(SCAN_T), 0, s, in, n,
                       (const int64_t*)tmp, out, nb);
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_T = 256;
constexpr int RS_R = 16;            // rounds per tile (4096 keys; 4, 8, 12, 20, 24 and 32 built slower at 2^20)
constexpr int RS_TILE = RS_T * RS_R;
constexpr int RS_MAX_BINS = 256;    // bins of the widest digit used

// Tile histogram of one digit (BITS wide, at `shift`), digit-major table.
template <int BITS>
__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                  const int32_t* __restrict__ n_dev, int shift,
                                                  int64_t* __restrict__ hist, int64_t nblk) {
    constexpr int BINS = 1 << BITS;
    constexpr unsigned MASK = BINS - 1;
    __shared__ int s_h[BINS];
    if (n_dev) n = min(n, (int64_t)*n_dev);
    for (int d = threadIdx.x; d < BINS; d += RS_T) s_h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    uint64_t k[RS_R];
#pragma unroll
    for (int r = 0; r < RS_R; ++r) {
        const int64_t i = base + r * RS_T + threadIdx.x;
        k[r] = i < n ? keys[i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < RS_R; ++r) {
        const int64_t i = base + r * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&s_h[(unsigned)(k[r] >> shift) & MASK], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < BINS; d += RS_T) hist[(int64_t)d * nblk + blockIdx.x] = s_h[d];
}

__device__ inline uint64_t lanes_below(int lane) {
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

template <int BITS>
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                     const int32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout,
                                                     int32_t* __restrict__ vout, int64_t n,
                                                     const int32_t* __restrict__ n_dev, int shift,
                                                     const int64_t* __restrict__ hist,
                                                     int64_t nblk, int iota) {
    constexpr int BINS = 1 << BITS;
    constexpr unsigned MASK = BINS - 1;
    constexpr int PER = BINS / RS_T;   // bins per thread
    if (n_dev) n = min(n, (int64_t)*n_dev);
    __shared__ int64_t s_goff[BINS];
    __shared__ int s_run[BINS];
    __shared__ int s_wc[RS_T / 64][BINS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        s_goff[t + u * RS_T] = hist[(int64_t)(t + u * RS_T) * nblk + blockIdx.x];
        s_run[t + u * RS_T] = 0;
    }
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t below = lanes_below(lane);
    // every round's key and value are loaded up front: one memory latency per
    // tile instead of one per round (the rounds are separated by barriers)
    uint64_t keys[RS_R];
    int32_t vals[RS_R];
#pragma unroll
    for (int r = 0; r < RS_R; ++r) {
        const int64_t i = base + r * RS_T + t;
        const bool valid = i < n;
        keys[r] = valid ? kin[i] : 0ull;
        vals[r] = valid ? (iota ? (int32_t)i : vin[i]) : 0;
    }
#pragma unroll
    for (int r = 0; r < RS_R; ++r) {
        const int64_t i = base + r * RS_T + t;
        const bool valid = i < n;
        const uint64_t key = keys[r];
        const int32_t val = vals[r];
        const unsigned d = (unsigned)(key >> shift) & MASK;
#pragma unroll
        for (int u = 0; u < PER; ++u)
            for (int k = 0; k < RS_T / 64; ++k) s_wc[k][t + u * RS_T] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) s_wc[w][d] = __popcll(peers);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int bin = t + u * RS_T;
            int run = s_run[bin];
            for (int k = 0; k < RS_T / 64; ++k) {
                int c = s_wc[k][bin];
                s_wc[k][bin] = run;
                run += c;
            }
            s_run[bin] = run;
        }
        __syncthreads();
        if (valid) {
            const int64_t dst = s_goff[d] + s_wc[w][d] + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
    }
}

__global__ void k_copy_pairs(const uint64_t* __restrict__ ks, const int32_t* __restrict__ vs,
                             uint64_t* __restrict__ kd, int32_t* __restrict__ vd, int64_t n,
                             const int32_t* __restrict__ n_dev) {
    if (n_dev) n = min(n, (int64_t)*n_dev);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        kd[i] = ks[i];
        vd[i] = vs[i];
    }
}

}  // namespace

int64_t scan_tmp_need(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 2; }

void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp,
                               hipStream_t s) {
    scan_impl<int32_t, int64_t>(in, out, n, tmp, s);
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
    scan_impl<int32_t, int32_t>(in, out, n, tmp, s);
}

int64_t radix_hist_need(int64_t n) {
    const int64_t nblk = (n + RS_TILE - 1) / RS_TILE;
    return nblk * RS_MAX_BINS + 1;
}

// 8-bit digits (9-bit digits would save a pass on 63-bit keys, 7 instead of 8,
// but cost more per pass than that pass at 2^20)
constexpr int RS_BITS = 8;

int radix_passes(int nbits) { return (nbits + RS_BITS - 1) / RS_BITS; }

void radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                      int64_t n, int nbits, int64_t* hist, int64_t* scan_tmp, hipStream_t s,
                      bool vals_are_iota, const int32_t* n_dev, bool to_alt) {
    if (n <= 0) return;
    const int64_t nblk = (n + RS_TILE - 1) / RS_TILE;
    const int passes = radix_passes(nbits);
    uint64_t* ki = keys;
    int32_t* vi = vals;
    uint64_t* ko = keys_alt;
    int32_t* vo = vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = RS_BITS * p;
        const int iota = (int)(vals_are_iota && p == 0);
        hipLaunchKernelGGL(k_rs_hist<RS_BITS>, dim3(nblk), dim3(RS_T), 0, s, (const uint64_t*)ki, n, n_dev,
                           shift, hist, nblk);
        scan_impl<int64_t, int64_t>(hist, hist, nblk << RS_BITS, scan_tmp, s);
        hipLaunchKernelGGL(k_rs_scatter<RS_BITS>, dim3(nblk), dim3(RS_T), 0, s, (const uint64_t*)ki,
                           (const int32_t*)vi, ko, vo, n, n_dev, shift, (const int64_t*)hist, nblk, iota);
        uint64_t* tk = ki; ki = ko; ko = tk;
        int32_t* tv = vi; vi = vo; vo = tv;
    }
    uint64_t* kd = to_alt ? keys_alt : keys;
    int32_t* vd = to_alt ? vals_alt : vals;
    if (ki != kd) {
        const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_copy_pairs, dim3(nb), dim3(256), 0, s, (const uint64_t*)ki,
                           (const int32_t*)vi, kd, vd, n, n_dev);
    }
}

}  // namespace pbh
