// wave.hpp -- wavefront-level helpers shared by the walk and neighbour kernels.
#pragma once

#include "pbh_internal.hpp"

namespace pbh {

// A value every lane holds equally, moved to a scalar register so that loops
// and branches on it are wave-uniform in the generated code.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline int popc_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes (all lanes active) with DPP moves:
// shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the last lane of row
// 0 is added into row 1 and row 3 (row_bcast:15, row mask 0b1010) and the last
// lane of row 1 into rows 2 and 3 (row_bcast:31, row mask 0b1100). Lanes whose
// source lies outside the row, and rows outside the mask, add 0.
__device__ inline int wave_incl_scan(int v, int /*lane*/) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// value of lane 63, in a scalar register
__device__ inline int last_lane(int v) { return __builtin_amdgcn_readlane(v, 63); }

// Work queue of groups split into kQueues contiguous ranges, one per XCD:
// workgroups are dispatched round-robin over the XCDs, so a workgroup takes
// its XCD's range first (neighbouring groups share tree nodes in that XCD's
// L2) and then helps the other ranges. All lanes issue the atomic (lane 0
// adds 1, the others 0): no lane-0-only branch precedes the broadcast.
constexpr int kQueues = 8;

// Workgroup id -> logical block in chunks of `chunk` consecutive blocks:
// workgroups go to XCDs round-robin by id, and XCD x runs the chunks
// x, x + 8, x + 16, ... in order, so every XCD's L2 serves a few compact
// stretches at a time while dense and sparse stretches spread over all XCDs.
// A bijection on [0, nb) when nb is a multiple of 8 * chunk (pad the grid;
// blocks mapped past the real count have no work).
__device__ inline unsigned xcd_chunk_block(unsigned b, unsigned chunk) {
    const unsigned x = b % kQueues, j = b / kQueues;
    return ((j / chunk) * kQueues + x) * chunk + j % chunk;
}

__device__ inline int64_t queue_next(unsigned long long* q /* [kQueues] */, int64_t G, int& home,
                                     int lane) {
    for (int k = 0; k < kQueues; ++k) {
        const int qi = (home + k) % kQueues;
        const int64_t lo = G * qi / kQueues, hi = G * (qi + 1) / kQueues;
        if (hi <= lo) continue;   // empty range (G < kQueues, or nothing queued)
        if (k > 0 && (int64_t)__builtin_amdgcn_readfirstlane((int)(q[qi] < (unsigned long long)(hi - lo))) == 0)
            continue;   // range already drained: skip the atomic
        const unsigned long long r = atomicAdd(&q[qi], lane == 0 ? 1ull : 0ull);
        const int64_t t = lo + (int64_t)uni((int)r);
        if (t < hi) {
            home = qi;
            return t;
        }
    }
    return -1;
}

// squared distance between two boxes (per-axis gap >= 0), FP64 without FMA
__device__ inline double box_box_d2(const double* alo, const double* ahi, const double* blo,
                                    const double* bhi) {
#pragma clang fp contract(off)
    double g[3];
    for (int k = 0; k < 3; ++k) {
        const double a = blo[k] - ahi[k];
        const double b = alo[k] - bhi[k];
        const double v = a > b ? a : b;
        g[k] = v > 0.0 ? v : 0.0;
    }
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
}

// squared distance from point c to the box [lo, hi], FP64 without FMA
__device__ inline double box_pt_d2(const double* lo, const double* hi, const double* c) {
#pragma clang fp contract(off)
    double g[3];
    for (int k = 0; k < 3; ++k) {
        const double a = lo[k] - c[k];
        const double b = c[k] - hi[k];
        const double v = a > b ? a : b;
        g[k] = v > 0.0 ? v : 0.0;
    }
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
}

// Traversal stack: the first lcap entries live in LDS, deeper entries in a
// per-wave spill region of global memory (the walk of a 2^20-particle Plummer
// sphere needs < 900 entries). kStackLds is the LDS part of the neighbour
// fill pass; the force walk keeps a smaller one (its LDS holds larger tiles).
constexpr int kStackLds = 1024;

struct Stack {
    int* lds;        // [lcap]
    int32_t* spill;  // [cap - lcap]
    int cap;
    int lcap;
    __device__ int get(int i) const { return i < lcap ? lds[i] : spill[i - lcap]; }
    __device__ void put(int i, int v) const {
        if (i < lcap) lds[i] = v;
        else spill[i - lcap] = v;
    }
};

}  // namespace pbh
