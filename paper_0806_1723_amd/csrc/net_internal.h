// Internal interface of the learned-form kernels (net_kernels.hip) and the
// network runtime (net.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lasto {
namespace net {

enum ConvMode { CONV_SAME = 0, CONV_DOWN = 1, CONV_ADJ = 2, CONV_ADJD = 3 };

// BF16 <-> FP32. BF16 is the top half of an FP32; rounding is to nearest,
// ties to even (the low half decides, the kept half's last bit breaks ties).
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));   // inf / nan
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Shapes of one convolution launch: output grid (nx, ny, nz) with cout
// channels, input grid (ix, iy, iz) with cin channels, channels-last BF16
// tensors [z][y][x][c]; kpad = 27 cin rounded up to a multiple of 32 (the
// packed weight row length).
struct ConvGeom {
    int nx, ny, nz;
    int ix, iy, iz;
    int cin, cout;
    int kpad;
    int mode;
};

// What the convolution does with its FP32 accumulator at each output value,
// in this order: + bias[co]; ReLU; + addend (BF16, same shape as the output);
// zero where mask (BF16, same shape) is not > 0; store FP32 and/or BF16.
struct ConvEpilogue {
    const float* bias = nullptr;
    int relu = 0;
    const uint16_t* addend = nullptr;
    const uint16_t* mask = nullptr;
    float* out_f32 = nullptr;
    uint16_t* out_bf16 = nullptr;
};

inline int kpad_of(int cin) { return (27 * cin + 31) / 32 * 32; }

hipError_t launch_conv(const ConvGeom& g, const uint16_t* in, const uint16_t* wp, const ConvEpilogue& ep,
                       hipStream_t s);
// partials part[splits][cout][kpad] of dW^T for a forward layer g (CONV_SAME or CONV_DOWN)
hipError_t launch_conv_wgrad(const ConvGeom& g, const uint16_t* in, const uint16_t* gout, float* part, int splits,
                             hipStream_t s);
hipError_t launch_sum_splits(const float* part, int splits, long n, float* out, int accumulate, hipStream_t s);
hipError_t launch_chan_sum(const uint16_t* a, long nvox, int c, float* part, int splits, hipStream_t s);
hipError_t launch_upsample_add(const uint16_t* coarse, int cx, int cy, int cz, const uint16_t* skip, uint16_t* out,
                               int nx, int ny, int nz, int c, hipStream_t s);
hipError_t launch_upsample_adj(const uint16_t* fine, int nx, int ny, int nz, uint16_t* out, int cx, int cy, int cz, int c,
                               const uint16_t* act, hipStream_t s);
// inference: y = w . BF16(up(coarse) + skip) + b without storing the sum
hipError_t launch_upsample_head(const uint16_t* coarse, int cx, int cy, int cz, const uint16_t* skip, int nx, int ny,
                                int nz, int c, const float* w, float* y, hipStream_t s);
hipError_t launch_head(const uint16_t* a, long nvox, int c, const float* w, float* y, hipStream_t s);
hipError_t launch_head_loss_bwd(const uint16_t* a, long nvox, int c, const float* w, const float* y, const float* tgt,
                                const float* wt, uint16_t* da, double* lossp, float* pw, int splits, hipStream_t s);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, long n, float lr, int step, hipStream_t s);
hipError_t launch_pack_weights(const float* W, int cin, int cout, uint16_t* wp, int kpad, uint16_t* wa, int kpad_adj,
                               int cin_rows, hipStream_t s);
hipError_t launch_unpack_wgrad(const float* dwt, int cin, int cout, int kpad, float* dw, hipStream_t s);
hipError_t launch_to_bf16(const float* a, uint16_t* b, long n, hipStream_t s);
hipError_t launch_to_f32(const uint16_t* a, float* b, long n, hipStream_t s);

}  // namespace net
}  // namespace lasto
