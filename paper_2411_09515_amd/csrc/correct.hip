// Jungfrau pre-processing and normalisation (Sec. 1.2, eq. norm).
//
// One thread owns 8 consecutive pixels and walks all frames of the batch, so
// the level-0 calibration and the normalisation of its pixels are read once
// per batch while the raw words stream through with 16-byte loads.  Levels 1
// and 2 (about 5 % of pixels) are gathered when a word selects them.
//
// The arithmetic is float64 and each stored value is rounded once to
// float32: signal = f32((adc - ped) / gain), out = f32(signal / norm).

#include "common.h"

namespace ss {

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t value) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = value;
}

namespace {

constexpr int kVec = 8;
constexpr int kCorrectBlock = 256;

__device__ inline float correct_one(uint32_t word, int64_t i, int64_t n_pix, float ped0, float gain0,
                                    const float *__restrict__ ped, const float *__restrict__ gain,
                                    int &invalid) {
    const uint32_t code = (word >> 14) & 3u;
    const double adc = double(word & 0x3FFFu);
    float p = ped0, k = gain0;
    if (code == 2u) {
        invalid += 1;
        return __builtin_nanf("");
    }
    if (code != 0u) {
        const int64_t off = (code == 1u ? 1 : 2) * n_pix + i;
        p = ped[off];
        k = gain[off];
    }
    return float((adc - double(p)) / double(k));
}

__device__ inline float normalise(float s, float nrm, bool has_norm) {
    return has_norm ? float(double(s) / double(nrm)) : s;
}

// Vector path: n_pix % 8 == 0 and 16-byte aligned buffers.
__global__ __launch_bounds__(kCorrectBlock) void k_correct_vec(
    const uint16_t *__restrict__ raw, int n_frames, int64_t n_pix, const float *__restrict__ ped,
    const float *__restrict__ gain, const float *__restrict__ norm, float *__restrict__ out,
    int64_t *__restrict__ n_invalid) {
    const int64_t p0 = (int64_t(blockIdx.x) * kCorrectBlock + threadIdx.x) * kVec;
    if (p0 >= n_pix) return;
    const bool has_norm = norm != nullptr;
    float p0v[kVec], g0v[kVec], nv[kVec];
    {
        const float4 *pp = reinterpret_cast<const float4 *>(ped + p0);
        const float4 *gp = reinterpret_cast<const float4 *>(gain + p0);
        float4 a = pp[0], b = pp[1], c = gp[0], d = gp[1];
        p0v[0] = a.x; p0v[1] = a.y; p0v[2] = a.z; p0v[3] = a.w;
        p0v[4] = b.x; p0v[5] = b.y; p0v[6] = b.z; p0v[7] = b.w;
        g0v[0] = c.x; g0v[1] = c.y; g0v[2] = c.z; g0v[3] = c.w;
        g0v[4] = d.x; g0v[5] = d.y; g0v[6] = d.z; g0v[7] = d.w;
        if (has_norm) {
            const float4 *np = reinterpret_cast<const float4 *>(norm + p0);
            float4 e = np[0], f = np[1];
            nv[0] = e.x; nv[1] = e.y; nv[2] = e.z; nv[3] = e.w;
            nv[4] = f.x; nv[5] = f.y; nv[6] = f.z; nv[7] = f.w;
        } else {
#pragma unroll
            for (int k = 0; k < kVec; ++k) nv[k] = 1.0f;
        }
    }
    for (int f = 0; f < n_frames; ++f) {
        const int64_t base = int64_t(f) * n_pix + p0;
        const uint4 w = *reinterpret_cast<const uint4 *>(raw + base);
        const uint32_t words[kVec] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16,
                                      w.z & 0xFFFFu, w.z >> 16, w.w & 0xFFFFu, w.w >> 16};
        int invalid = 0;
        float o[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k)
            o[k] = normalise(correct_one(words[k], p0 + k, n_pix, p0v[k], g0v[k], ped, gain, invalid),
                             nv[k], has_norm);
        float4 *op = reinterpret_cast<float4 *>(out + base);
        op[0] = make_float4(o[0], o[1], o[2], o[3]);
        op[1] = make_float4(o[4], o[5], o[6], o[7]);
        if (invalid && n_invalid) atomicAdd(reinterpret_cast<unsigned long long *>(n_invalid + f),
                                            (unsigned long long)invalid);
    }
}

// Scalar path for any size and alignment: one thread per pixel, all frames.
__global__ __launch_bounds__(kCorrectBlock) void k_correct_scalar(
    const uint16_t *__restrict__ raw, int n_frames, int64_t n_pix, const float *__restrict__ ped,
    const float *__restrict__ gain, const float *__restrict__ norm, float *__restrict__ out,
    int64_t *__restrict__ n_invalid) {
    const int64_t i = int64_t(blockIdx.x) * kCorrectBlock + threadIdx.x;
    if (i >= n_pix) return;
    const bool has_norm = norm != nullptr;
    const float p0 = ped[i], g0 = gain[i], nr = has_norm ? norm[i] : 1.0f;
    for (int f = 0; f < n_frames; ++f) {
        const int64_t at = int64_t(f) * n_pix + i;
        int invalid = 0;
        out[at] = normalise(correct_one(raw[at], i, n_pix, p0, g0, ped, gain, invalid), nr, has_norm);
        if (invalid && n_invalid) atomicAdd(reinterpret_cast<unsigned long long *>(n_invalid + f),
                                            (unsigned long long)invalid);
    }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace ss

extern "C" int ss_correct(const uint16_t *raw, int32_t n_frames, int64_t n_pix, const float *pedestal,
                          const float *gain, const float *norm, float *out, int64_t *n_invalid,
                          hipStream_t stream) {
    using namespace ss;
    if (n_frames < 0 || n_pix < 0 || n_pix >= (int64_t(1) << 31)) return SS_ESIZE;
    if (n_frames == 0) return SS_OK;
    if (!raw || !pedestal || !gain || !out) return SS_EINVAL;
    if (n_invalid) {
        k_fill_i64<<<1, 64, 0, stream>>>(n_invalid, n_frames, 0);
        SS_RETURN_IF_LAUNCH_FAILED();
    }
    if (n_pix == 0) return SS_OK;
    const bool vec = (n_pix % kVec == 0) && aligned16(raw) && aligned16(pedestal) && aligned16(gain) &&
                     aligned16(out) && (!norm || aligned16(norm));
    if (vec) {
        const int64_t threads = n_pix / kVec;
        const int64_t blocks = (threads + kCorrectBlock - 1) / kCorrectBlock;
        k_correct_vec<<<dim3(uint32_t(blocks)), kCorrectBlock, 0, stream>>>(
            raw, n_frames, n_pix, pedestal, gain, norm, out, n_invalid);
    } else {
        const int64_t blocks = (n_pix + kCorrectBlock - 1) / kCorrectBlock;
        k_correct_scalar<<<dim3(uint32_t(blocks)), kCorrectBlock, 0, stream>>>(
            raw, n_frames, n_pix, pedestal, gain, norm, out, n_invalid);
    }
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}
