// The learned clip surrogate's network on gfx950: batched forward, the loss
// gradient and Adam, with the per-bin training targets.
//
// Network: 19 -> 64 -> 64 -> 2 with GELU (erf form) after both hidden
// layers; parameters are float16 (the layout of SS_MLP_OFF_*), arithmetic is
// float32.  The batched kernels work on tiles of 16 samples per wavefront
// with v_mfma_f32_16x16x4_f32 (D[16x16] += A[16x4] B[4x16]); the parameters
// are staged once per work-group in LDS as float32.
//
// MFMA operand layout (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element i of lane l is D[4 (l / 16) + i][l % 16].
//
// The gradient is that of the summed squared error over the used samples;
// the reduction kernel divides by their count, in a fixed order, so the
// result is reproducible.

#include <hip/hip_fp16.h>

#include <cmath>

#include "common.h"

namespace ss {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kIn = SS_MLP_IN;
constexpr int kHid = SS_MLP_HID;
constexpr int kK1 = SS_MLP_K1;
constexpr int kOutPad = SS_MLP_OUT_PAD;
constexpr int kParams = SS_MLP_PARAMS;
constexpr int kTile = 16;                 // samples per wavefront tile
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWavesPerBlock * kWave;
constexpr int kMaxGradWaves = 1024;       // partial gradients reduced at the end

__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

__device__ inline float gelu(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float u) {
    return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * expf(-0.5f * u * u) * 0.39894228040143268f;
}

__device__ inline float half_bits(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// Parameters (float16 bits) into LDS as float32, by the whole work-group.
__device__ inline void stage_params(const uint16_t *__restrict__ w16, float *p_s) {
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) p_s[i] = half_bits(w16[i]);
}

// Per-wave LDS scratch for one tile.
struct TileLds {
    float x[kTile][kK1];
    float z1[kTile][kHid];
    float h1[kTile][kHid];
    float z2[kTile][kHid];
    float h2[kTile][kHid];
    float dz[kTile][kHid];
};

// out[16][N] = in[16][K] . W[K][N] + b over N-tiles nt (W row-major with
// row stride ldw); returns the accumulators of N-tile nt.
template <int K>
__device__ inline f4 tile_gemm(const float (*in)[K], const float *W, int ldw, int nt, int lane) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
    for (int ks = 0; ks < K / 4; ++ks) {
        const float a = in[lane % 16][ks * 4 + lane / 16];
        const float b = W[(ks * 4 + lane / 16) * ldw + nt * 16 + lane % 16];
        acc = mfma(a, b, acc);
    }
    return acc;
}

// Forward pass of one tile; leaves z1, h1, z2, h2 in LDS and returns the two
// outputs of row (lane) for lanes < 16 in y0, y1.
__device__ inline void tile_forward(const float *p_s, TileLds &t, int lane) {
    const float *W1 = p_s + SS_MLP_OFF_W1, *b1 = p_s + SS_MLP_OFF_B1;
    const float *W2 = p_s + SS_MLP_OFF_W2, *b2 = p_s + SS_MLP_OFF_B2;
#pragma unroll
    for (int nt = 0; nt < kHid / 16; ++nt) {
        const f4 acc = tile_gemm<kK1>(t.x, W1, kHid, nt, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * (lane / 16) + i, c = nt * 16 + lane % 16;
            const float z = acc[i] + b1[c];
            t.z1[r][c] = z;
            t.h1[r][c] = gelu(z);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int nt = 0; nt < kHid / 16; ++nt) {
        const f4 acc = tile_gemm<kHid>(t.h1, W2, kHid, nt, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * (lane / 16) + i, c = nt * 16 + lane % 16;
            const float z = acc[i] + b2[c];
            t.z2[r][c] = z;
            t.h2[r][c] = gelu(z);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Output layer: accumulators of the 16 x 16 tile (2 live columns).
__device__ inline f4 tile_output(const float *p_s, TileLds &t, int lane) {
    const float *W3 = p_s + SS_MLP_OFF_W3, *b3 = p_s + SS_MLP_OFF_B3;
    f4 acc = tile_gemm<kHid>(t.h2, W3, kOutPad, 0, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += b3[lane % 16];
    return acc;
}

__device__ inline void load_x(TileLds &t, const float *__restrict__ x, int64_t n, int64_t row0, int lane) {
    for (int i = lane; i < kTile * kK1; i += kWave) {
        const int r = i / kK1, c = i % kK1;
        const int64_t s = row0 + r;
        t.x[r][c] = (c < kIn && s < n) ? x[s * kIn + c] : 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBlock) void k_mlp_forward(const uint16_t *__restrict__ w16, const float *__restrict__ x,
                                                       int64_t n, float *__restrict__ y) {
    __shared__ float p_s[kParams];
    __shared__ TileLds tl[kWavesPerBlock];
    stage_params(w16, p_s);
    __syncthreads();
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    for (int64_t tile = int64_t(blockIdx.x) * kWavesPerBlock + wid; tile < n_tiles;
         tile += int64_t(gridDim.x) * kWavesPerBlock) {
        TileLds &t = tl[wid];
        load_x(t, x, n, tile * kTile, lane);
        tile_forward(p_s, t, lane);
        const f4 acc = tile_output(p_s, t, lane);
        const int c = lane % 16;
        if (c < SS_MLP_OUT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t s = tile * kTile + 4 * (lane / 16) + i;
                if (s < n) y[s * SS_MLP_OUT + c] = acc[i];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Partial gradient of the summed squared error over this wavefront's tiles,
// written to part[wave][kParams]; the used-sample count and partial loss go
// to part_n[wave] and part_l[wave].
__global__ __launch_bounds__(kBlock) void k_mlp_grad(const uint16_t *__restrict__ w16, const float *__restrict__ x,
                                                    const float *__restrict__ target, const uint8_t *__restrict__ use,
                                                    int64_t n, float *__restrict__ part, float *__restrict__ part_l,
                                                    int32_t *__restrict__ part_n) {
    __shared__ float p_s[kParams];
    __shared__ TileLds tl[kWavesPerBlock];
    __shared__ float dy_s[kWavesPerBlock][kTile][kOutPad];
    stage_params(w16, p_s);
    __syncthreads();
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int gw = blockIdx.x * kWavesPerBlock + wid;
    const int n_waves = gridDim.x * kWavesPerBlock;
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    const float *W2 = p_s + SS_MLP_OFF_W2, *W3 = p_s + SS_MLP_OFF_W3;
    TileLds &t = tl[wid];
    float (*dy)[kOutPad] = dy_s[wid];

    // gradient accumulators, MFMA layout: gW1 2 x 4 tiles, gW2 4 x 4, gW3 4 x 1
    f4 g1[2][4], g2[4][4], g3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        g3[a] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            g2[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            if (a < 2) g1[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
    float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;  // lane c holds column c (c < 64)
    float loss = 0.0f;
    int used = 0;

    for (int64_t tile = gw; tile < n_tiles; tile += n_waves) {
        const int64_t row0 = tile * kTile;
        load_x(t, x, n, row0, lane);
        tile_forward(p_s, t, lane);
        const f4 out = tile_output(p_s, t, lane);
        // dy = 2 (y - t) on used rows, columns 0 and 1; zero elsewhere
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * (lane / 16) + i, c = lane % 16;
            const int64_t s = row0 + r;
            float d = 0.0f;
            if (c < SS_MLP_OUT && s < n && (use == nullptr || use[s])) {
                const float e = out[i] - target[s * SS_MLP_OUT + c];
                d = 2.0f * e;
                loss += e * e;
                if (c == 0) ++used;
            }
            dy[r][c] = d;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW3 += h2^T dy  (M = 64, N = 16, K = 16 samples); gb3 = column sums of dy
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                g3[mt] = mfma(t.h2[ks * 4 + lane / 16][mt * 16 + lane % 16], dy[ks * 4 + lane / 16][lane % 16], g3[mt]);
        if (lane < kOutPad)
            for (int r = 0; r < kTile; ++r) gb3 += dy[r][lane];
        // dz2 = (dy W3^T) * gelu'(z2)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < kOutPad / 4; ++ks)
                acc = mfma(dy[lane % 16][ks * 4 + lane / 16], W3[(nt * 16 + lane % 16) * kOutPad + ks * 4 + lane / 16],
                           acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * (lane / 16) + i, c = nt * 16 + lane % 16;
                t.dz[r][c] = acc[i] * gelu_grad(t.z2[r][c]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW2 += h1^T dz2; gb2 += column sums of dz2
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    g2[mt][nt] = mfma(t.h1[ks * 4 + lane / 16][mt * 16 + lane % 16],
                                      t.dz[ks * 4 + lane / 16][nt * 16 + lane % 16], g2[mt][nt]);
        for (int r = 0; r < kTile; ++r) gb2 += t.dz[r][lane];
        // dz1 = (dz2 W2^T) * gelu'(z1), written over z1 (z1 is not needed after)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
            for (int ks = 0; ks < kHid / 4; ++ks)
                acc = mfma(t.dz[lane % 16][ks * 4 + lane / 16], W2[(nt * 16 + lane % 16) * kHid + ks * 4 + lane / 16],
                           acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * (lane / 16) + i, c = nt * 16 + lane % 16;
                t.h2[r][c] = acc[i] * gelu_grad(t.z1[r][c]);  // h2 is free now: holds dz1
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW1 += x^T dz1; gb1 += column sums of dz1
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    g1[mt][nt] = mfma(t.x[ks * 4 + lane / 16][mt * 16 + lane % 16],
                                      t.h2[ks * 4 + lane / 16][nt * 16 + lane % 16], g1[mt][nt]);
        for (int r = 0; r < kTile; ++r) gb1 += t.h2[r][lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    float *out = part + int64_t(gw) * kParams;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = 4 * (lane / 16) + i, cc = lane % 16;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                out[SS_MLP_OFF_W1 + (mt * 16 + rr) * kHid + nt * 16 + cc] = g1[mt][nt][i];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                out[SS_MLP_OFF_W2 + (mt * 16 + rr) * kHid + nt * 16 + cc] = g2[mt][nt][i];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) out[SS_MLP_OFF_W3 + (mt * 16 + rr) * kOutPad + cc] = g3[mt][i];
    }
    out[SS_MLP_OFF_B1 + lane] = gb1;
    out[SS_MLP_OFF_B2 + lane] = gb2;
    if (lane < kOutPad) out[SS_MLP_OFF_B3 + lane] = gb3;
    // the wave's loss and count (summed over lanes in a fixed order)
    double l = wave_sum(double(loss));
    const int u = wave_sum(used);
    if (lane == 0) {
        part_l[gw] = float(l);
        part_n[gw] = u;
    }
}

// grad[p] = (sum over waves of part[w][p]) / n_used; loss likewise.
__global__ void k_mlp_grad_reduce(const float *__restrict__ part, const float *__restrict__ part_l,
                                  const int32_t *__restrict__ part_n, int n_waves, float *__restrict__ grad,
                                  float *__restrict__ loss) {
    int64_t used = 0;
    for (int w = 0; w < n_waves; ++w) used += part_n[w];
    const double inv = used > 0 ? 1.0 / double(used) : 0.0;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        double s = 0.0;
        for (int w = 0; w < n_waves; ++w) s += double(part[int64_t(w) * kParams + p]);
        grad[p] = float(s * inv);
    }
    if (p == 0 && loss) {
        double s = 0.0;
        for (int w = 0; w < n_waves; ++w) s += double(part_l[w]);
        *loss = float(s * inv);
    }
}

__global__ void k_mlp_adam(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ grad, float lr, float beta1, float beta2, float eps, float c1,
                           float c2, uint16_t *__restrict__ w16) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float w = params[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    params[p] = w;
    w16[p] = __half_as_ushort(__float2half(w));
}

// Training targets from the unclipped statistics and a converged clip.
__global__ void k_surrogate_targets(const double *__restrict__ stats0, const double *__restrict__ mean,
                                    const double *__restrict__ std, const int32_t *__restrict__ n_members,
                                    const int32_t *__restrict__ converged, int64_t count, float *__restrict__ target,
                                    uint8_t *__restrict__ use) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double n0 = stats0[3 * i], m0 = stats0[3 * i + 1], s0 = stats0[3 * i + 2];
    const bool ok = n0 >= 2.0 && s0 > 0.0 && converged[i] == 1 && n_members[i] >= 2 && std[i] > 0.0;
    target[2 * i] = ok ? float((mean[i] - m0) / s0) : 0.0f;
    target[2 * i + 1] = ok ? float(log(std[i] / s0)) : 0.0f;
    use[i] = ok ? 1 : 0;
}

int grad_waves(int64_t n) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t w = tiles < kMaxGradWaves ? tiles : kMaxGradWaves;
    return int(((w + kWavesPerBlock - 1) / kWavesPerBlock) * kWavesPerBlock);
}

}  // namespace
}  // namespace ss

extern "C" int ss_mlp_forward(const uint16_t *w16, const float *x, int64_t n, float *y, hipStream_t stream) {
    if (n < 0) return SS_ESIZE;
    if (n == 0) return SS_OK;
    if (!w16 || !x || !y) return SS_EINVAL;
    const int64_t tiles = (n + ss::kTile - 1) / ss::kTile;
    int64_t blocks = (tiles + ss::kWavesPerBlock - 1) / ss::kWavesPerBlock;
    if (blocks > 2048) blocks = 2048;
    ss::k_mlp_forward<<<dim3(uint32_t(blocks)), ss::kBlock, 0, stream>>>(w16, x, n, y);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

extern "C" size_t ss_mlp_grad_workspace(int64_t n) {
    if (n <= 0) return 0;
    const size_t w = size_t(ss::grad_waves(n));
    return w * size_t(ss::kParams) * sizeof(float) + w * sizeof(float) + w * sizeof(int32_t) + 256;
}

extern "C" int ss_mlp_grad(const uint16_t *w16, const float *x, const float *target, const uint8_t *use, int64_t n,
                           float *grad, float *loss, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (n <= 0) return SS_ESIZE;
    if (!w16 || !x || !target || !grad || !workspace) return SS_EINVAL;
    if (workspace_bytes < ss_mlp_grad_workspace(n)) return SS_ESIZE;
    const int waves = ss::grad_waves(n);
    char *ws = static_cast<char *>(workspace);
    float *part = reinterpret_cast<float *>(ws);
    float *part_l = part + size_t(waves) * ss::kParams;
    int32_t *part_n = reinterpret_cast<int32_t *>(part_l + waves);
    ss::k_mlp_grad<<<dim3(uint32_t(waves / ss::kWavesPerBlock)), ss::kBlock, 0, stream>>>(w16, x, target, use, n,
                                                                                          part, part_l, part_n);
    ss::k_mlp_grad_reduce<<<dim3((ss::kParams + 255) / 256), 256, 0, stream>>>(part, part_l, part_n, waves, grad, loss);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

extern "C" int ss_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr, float beta1,
                           float beta2, float eps, uint16_t *w16, hipStream_t stream) {
    if (!params || !m || !v || !grad || !w16) return SS_EINVAL;
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return SS_EINVAL;
    const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
    const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
    ss::k_mlp_adam<<<dim3((ss::kParams + 255) / 256), 256, 0, stream>>>(params, m, v, grad, lr, beta1, beta2, eps, c1,
                                                                       c2, w16);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

extern "C" int ss_surrogate_targets(const double *stats0, const ss_profile *ref, int64_t count, float *target,
                                    uint8_t *use, hipStream_t stream) {
    if (count < 0) return SS_ESIZE;
    if (count == 0) return SS_OK;
    if (!stats0 || !ref || !ref->mean || !ref->std || !ref->n_members || !ref->converged || !target || !use)
        return SS_EINVAL;
    const int64_t blocks = (count + 255) / 256;
    if (blocks >= (int64_t(1) << 31)) return SS_ESIZE;
    ss::k_surrogate_targets<<<dim3(uint32_t(blocks)), 256, 0, stream>>>(stats0, ref->mean, ref->std, ref->n_members,
                                                                       ref->converged, count, target, use);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}
