// Internal helpers shared by the gfx950 kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sigsep.h"

#define SS_RETURN_IF_LAUNCH_FAILED()                    \
    do {                                                \
        if (hipGetLastError() != hipSuccess) return SS_EHIP; \
    } while (0)

namespace ss {

constexpr int kWave = 64;

// Butterfly sum over the 64 lanes of a wavefront; every lane gets the total.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum N doubles over the work-group; every thread gets the totals.
// `part` holds N * (BLOCK / 64) doubles and `tot` N doubles; the two regions
// let consecutive calls run with two barriers each.  The summation order is
// fixed, so results are reproducible run to run.
template <int N, int BLOCK>
__device__ inline void block_sum(double (&v)[N], double *part, double *tot) {
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) part[k * NW + wid] = v[k];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double x = lane < NW ? part[k * NW + lane] : 0.0;
#pragma unroll
            for (int off = NW / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
            if (lane == 0) tot[k] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = tot[k];
}

// Lanes below this one whose bit is set in a 64-bit wave mask.
__device__ inline int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// Raw buffer resource over `bytes` bytes at p (gfx9-family data format
// word).  Buffer loads through it are range-checked by the hardware: an
// offset at or beyond `bytes` reads 0 instead of touching memory.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, int(bytes), 0x00020000);
}

__device__ inline float buffer_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}

__device__ inline int32_t buffer_load_i32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0);
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t value);

}  // namespace ss
