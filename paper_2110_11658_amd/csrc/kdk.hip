// kdk.hip -- leapfrog kick and drift under the regular force, and the energy
// sum (Arnold, Baumgardt & Wang 2021, Section 2.2, eq. kick: v += dt/2 F_R).
// All FP64. The energy is E = sum m v^2/2 + sum m Phi_R/2, reduced in a fixed
// order (per-block partial sums, then one block) so it is reproducible.
#include "pbh_internal.hpp"

namespace pbh {

namespace {

__global__ void k_kick(double* __restrict__ vel, const double* __restrict__ acc, double h,
                       int64_t n3) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x)
        vel[i] += h * acc[i];
}

__global__ void k_drift(double* __restrict__ pos, const double* __restrict__ vel, double dt,
                        int64_t n3) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x)
        pos[i] += dt * vel[i];
}

constexpr int E_T = 256;

__global__ __launch_bounds__(E_T) void k_energy_part(const double* __restrict__ vel,
                                                     const double* __restrict__ mass,
                                                     const double* __restrict__ pot, int64_t n,
                                                     double* __restrict__ part) {
    __shared__ double s[E_T];
    double e = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * E_T + threadIdx.x; i < n; i += (int64_t)gridDim.x * E_T) {
        const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
        e += 0.5 * mass[i] * (vx * vx + vy * vy + vz * vz) + 0.5 * mass[i] * pot[i];
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = E_T / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(E_T) void k_energy_final(const double* __restrict__ part, int nb,
                                                      double* __restrict__ out) {
    __shared__ double s[E_T];
    double e = 0.0;
    for (int b = threadIdx.x; b < nb; b += E_T) e += part[b];
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = E_T / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

inline int grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

// Counter calibration: every lane runs `iters` rounds of 32 FP32 FMAs in
// eight independent chains (the count a VALU instruction counter must see).
__global__ __launch_bounds__(64) void k_valu_probe(int iters, float seed, float* out) {
    float a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = seed + (float)(threadIdx.x + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) a[c] = __builtin_fmaf(a[c], 0.999f, 0.5f);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += a[c];
    if (s == 1234.5f) out[blockIdx.x] = s;   // keeps the chains live; never true for the seeds used
}

}  // namespace

void launch_valu_probe(int64_t blocks, int iters, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_valu_probe, dim3((unsigned)blocks), dim3(64), 0, s, iters, 0.25f, out);
}

void launch_kick(double* vel, const double* acc, double h, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_kick, dim3(grid_for(3 * n)), dim3(256), 0, s, vel, acc, h, 3 * n);
}

void launch_drift(double* pos, const double* vel, double dt, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_drift, dim3(grid_for(3 * n)), dim3(256), 0, s, pos, vel, dt, 3 * n);
}

void launch_energy(const double* vel, const double* mass, const double* pot, int64_t n,
                   double* partial, int nblk, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_part, dim3(nblk), dim3(E_T), 0, s, vel, mass, pot, n, partial);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(E_T), 0, s, (const double*)partial, nblk, out);
}

void launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

}  // namespace pbh
