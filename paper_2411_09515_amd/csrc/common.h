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

// Move a double across lanes with a DPP control (both 32-bit halves).
template <int CTRL>
__device__ inline double dpp_move(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane(double x, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                            __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Row broadcast (row_bcast:15 / row_bcast:31) into the rows of ROWS; lanes
// of the other rows get 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_bcast(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront, left in lane 63.  Within each row of
// 16 lanes quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and
// row_mirror leave the row's sum in every lane; row_bcast:15 then adds row 0
// into row 1 and row 2 into row 3, and row_bcast:31 adds rows 0-1 into row
// 3.  The order is fixed, so the result is reproducible.
__device__ inline double wave_sum_last(double x) {
    x += dpp_move<0xB1>(x);
    x += dpp_move<0x4E>(x);
    x += dpp_move<0x141>(x);
    x += dpp_move<0x140>(x);
    x += dpp_bcast<0x142, 0xA>(x);
    x += dpp_bcast<0x143, 0xC>(x);
    return x;
}

// wave_sum_last of N values, taken stage by stage over groups of up to
// five of them so that their dependency chains overlap (each result is the
// same as alone; larger groups would hold more registers for the moves).
template <int N>
__device__ inline void wave_sum_last_n(double (&x)[N]) {
    constexpr int G = 5;
#pragma unroll
    for (int k0 = 0; k0 < N; k0 += G) {
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_move<0xB1>(x[k]);
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_move<0x4E>(x[k]);
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_move<0x141>(x[k]);
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_move<0x140>(x[k]);
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_bcast<0x142, 0xA>(x[k]);
#pragma unroll
        for (int k = k0; k < N && k < k0 + G; ++k) x[k] += dpp_bcast<0x143, 0xC>(x[k]);
    }
}

// The same total, given to every lane.
__device__ inline double wave_sum(double x) { return readlane(wave_sum_last(x), kWave - 1); }

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
    for (int k = 0; k < N; ++k) v[k] = wave_sum_last(v[k]);
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < N; ++k) part[k * NW + wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) x += part[threadIdx.x * NW + w];
        tot[threadIdx.x] = x;
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

// Word offsets of pixels in a frame of an ss_layout: row-major (sw < 0),
// or tiles of 2^sw x 2^sh pixels, tiles row-major, pixels row-major inside
// a tile.
struct Layout {
    int32_t height, width;
    int32_t sw, sh;   // log2 of the tile width and height; sw < 0: row-major
    int32_t tiles_x;
    int64_t words;    // words per frame

    __host__ __device__ bool tiled() const { return sw >= 0; }
    __host__ __device__ int64_t offset(int y, int x) const {
        if (sw < 0) return int64_t(y) * width + x;
        return ((int64_t(y >> sh) * tiles_x + (x >> sw)) << (sw + sh)) + ((y & ((1 << sh) - 1)) << sw) +
               (x & ((1 << sw) - 1));
    }
};

// The Layout of frames of height x width pixels in tiles of tile_w x tile_h
// (0 x 0: row-major); false for a layout ss_layout_words refuses.
bool make_layout(int32_t height, int32_t width, int32_t tile_w, int32_t tile_h, Layout &out);

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t value);

}  // namespace ss
