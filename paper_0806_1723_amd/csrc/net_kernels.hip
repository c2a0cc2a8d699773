// Kernels of the learned initial guess and coarse correction: a small 3-D
// U-Net on the grid's index space, channels-last BF16 activations, FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// A 3x3x3 convolution is an implicit GEMM: out[v][co] = sum_k A[v][k] B[k][co]
// with k = tap * cin + ci, A[v][k] = in[g(v, tap)][ci] gathered on the fly
// and B the packed weights. g depends on the mode:
//   CONV_SAME  g = v + off          (stride 1, same size)
//   CONV_DOWN  g = 2 v + off        (stride 2: output node v sits on input node 2v)
//   CONV_ADJ   g = v - off          (adjoint of CONV_SAME: the backward pass to the input)
//   CONV_ADJD  g = (v - off) / 2    (adjoint of CONV_DOWN; only where v - off is even)
// off = (dx, dy, dz) in {-1, 0, 1}^3, tap = 9 (dz+1) + 3 (dy+1) + (dx+1);
// nodes outside the input grid read as zero. Grid sizes: a stride-2 level of
// an n-node axis has (n + 1) / 2 nodes.
//
// MFMA 16x16x32 (bf16 in, f32 accumulate), wave64: lane l supplies
//   A[m = l % 16][k = 8 (l / 16) + i], B[k = 8 (l / 16) + i][n = l % 16], i < 8,
// and receives C[m = 4 (l / 16) + i][n = l % 16], i < 4.
#include <algorithm>
#include <cstdint>

#include "net_internal.h"

namespace lasto {
namespace net {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 q) { return __builtin_bit_cast(bf16x8, q); }

struct Off {
    int dx, dy, dz;
};
__device__ __forceinline__ Off tap_off(int t) { return Off{t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1}; }

// input node of output node (x, y, z) for one tap; false when it is outside
template <int MODE>
__device__ __forceinline__ bool gather_node(int x, int y, int z, Off o, const ConvGeom& g, int& xi, int& yi, int& zi)
{
    if (MODE == CONV_SAME) {
        xi = x + o.dx; yi = y + o.dy; zi = z + o.dz;
    } else if (MODE == CONV_DOWN) {
        xi = 2 * x + o.dx; yi = 2 * y + o.dy; zi = 2 * z + o.dz;
    } else if (MODE == CONV_ADJ) {
        xi = x - o.dx; yi = y - o.dy; zi = z - o.dz;
    } else {
        const int ax = x - o.dx, ay = y - o.dy, az = z - o.dz;
        if ((ax | ay | az) & 1) return false;
        xi = ax >> 1; yi = ay >> 1; zi = az >> 1;   // ax may be -1 only when odd, so >> 1 of an even value
    }
    return xi >= 0 && yi >= 0 && zi >= 0 && xi < g.ix && yi < g.iy && zi < g.iz;
}

// ------------------------------------------------------------ forward
// One wave computes MT*16 consecutive output nodes (in the flat [z][y][x]
// order, so rows of any length pack without waste) times all NT*16 output
// channels; four waves per workgroup. Each 32-wide K chunk's weight
// fragment is loaded once per wave and used for all MT node tiles. The K
// loop runs in groups of KB chunks: all gathers and weight loads of a group
// are issued before its MFMAs. A lane's position in K advances by 32 per
// chunk; its tap t and channel ci are updated incrementally (no division).
constexpr int CONV_KB = 2;

template <int MODE, int NT, int MT>
__global__ __launch_bounds__(256) void k_conv(ConvGeom g, const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ wp, ConvEpilogue ep)
{
    const int lane = threadIdx.x & 63;
    const long tile = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long nvox = (long)g.nx * g.ny * g.nz;
    const long v0 = tile * 16 * MT;
    if (v0 >= nvox) return;
    const int m = lane & 15, kq = lane >> 4;
    // this lane's node in each of the MT tiles (A rows)
    int xs[MT], ys[MT], zs[MT];
    bool vok[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const long v = v0 + 16 * u + m;
        vok[u] = v < nvox;
        const long vv = vok[u] ? v : nvox - 1;
        xs[u] = (int)(vv % g.nx);
        ys[u] = (int)((vv / g.nx) % g.ny);
        zs[u] = (int)(vv / ((long)g.nx * g.ny));
    }
    const int K = 27 * g.cin;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[u][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int t = (8 * kq) / g.cin, ci = 8 * kq - t * g.cin;   // this lane's tap and channel at chunk 0
    for (int kc0 = 0; kc0 < g.kpad; kc0 += 32 * CONV_KB) {
        uint4 a[CONV_KB][MT], b[CONV_KB][NT];
#pragma unroll
        for (int q = 0; q < CONV_KB; ++q) {
            const int kc = kc0 + 32 * q;
            const int k = kc + 8 * kq;
#pragma unroll
            for (int u = 0; u < MT; ++u) a[q][u] = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < NT; ++j) b[q][j] = make_uint4(0, 0, 0, 0);
            if (kc < g.kpad) {
                if (k < K) {
                    const Off o = tap_off(t);
#pragma unroll
                    for (int u = 0; u < MT; ++u) {
                        int xi, yi, zi;
                        if (vok[u] && gather_node<MODE>(xs[u], ys[u], zs[u], o, g, xi, yi, zi))
                            a[q][u] = *(const uint4*)(in + (((size_t)zi * g.iy + yi) * g.ix + xi) * g.cin + ci);
                    }
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) b[q][j] = *(const uint4*)(wp + (size_t)(j * 16 + m) * g.kpad + k);
            }
            ci += 32;
            while (ci >= g.cin) {
                ci -= g.cin;
                ++t;
            }
        }
#pragma unroll
        for (int q = 0; q < CONV_KB; ++q) {
            if (kc0 + 32 * q >= g.kpad) break;
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const bf16x8 av = as_bf16x8(a[q][u]);
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf16x8(b[q][j]), acc[u][j], 0, 0, 0);
            }
        }
    }
    // epilogue: C[m' = 4 kq + i][n = lane % 16] of tile (u, j) is node
    // v0 + 16 u + m', channel 16 j + n. The operands it reads are loaded for
    // all four nodes before any is used.
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = j * 16 + m;
        const float bias = ep.bias ? ep.bias[co] : 0.f;
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            uint16_t add[4] = {0, 0, 0, 0}, msk[4] = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long v = min(v0 + 16 * u + 4 * kq + i, nvox - 1);
                if (ep.addend) add[i] = ep.addend[(size_t)v * g.cout + co];
                if (ep.mask) msk[i] = ep.mask[(size_t)v * g.cout + co];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long v = v0 + 16 * u + 4 * kq + i;
                if (v >= nvox) continue;
                const size_t at = (size_t)v * g.cout + co;
                float val = acc[u][j][i] + bias;
                if (ep.relu) val = fmaxf(val, 0.f);
                if (ep.addend) val += bf2f(add[i]);
                if (ep.mask && !(bf2f(msk[i]) > 0.f)) val = 0.f;
                if (ep.out_f32) ep.out_f32[at] = val;
                if (ep.out_bf16) ep.out_bf16[at] = f2bf(val);
            }
        }
    }
}

// Stride-1 convolution through LDS: a workgroup owns a 16 (x) x 4 (y) x 4
// (z) brick of output nodes (wave w: plane z0 + w; its MT = 4 tiles: rows
// y0 .. y0+3; lane m: x0 + m) and first copies the 18 x 6 x 6 input box
// with its halo into LDS, 16 bytes (8 channels) per load, zero outside the
// grid. The A operands then come from LDS; K order, MFMA order and the
// epilogue are those of k_conv, so the results are the same bit for bit.
constexpr int CL_BX = 16, CL_BY = 4, CL_BZ = 4;
constexpr int CL_HX = CL_BX + 2, CL_HY = CL_BY + 2, CL_HZ = CL_BZ + 2;
constexpr int CL_CMAX = 32;   // input channels the largest box holds
#ifndef LASTO_CONV_LDS_MIN_NODES
#define LASTO_CONV_LDS_MIN_NODES 100000   // levels from this many nodes use the LDS form
#endif

// CM: input channels the box holds (8, 16 or 32: 10, 21 or 41 KB of LDS)
template <int NT, int CM>
__global__ __launch_bounds__(256) void k_conv_same_lds(ConvGeom g, const uint16_t* __restrict__ in,
                                                       const uint16_t* __restrict__ wp, ConvEpilogue ep)
{
    constexpr int MT = CL_BY;
    __shared__ __align__(16) uint16_t box[CL_HZ * CL_HY * CL_HX * CM];
    const int nbx = (g.nx + CL_BX - 1) / CL_BX, nby = (g.ny + CL_BY - 1) / CL_BY;
    const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * CL_BX, y0 = by * CL_BY, z0 = bz * CL_BZ;
    const int cq = g.cin / 8;   // 16-byte chunks per node
    {
        // fill: box node (hx, hy, hz) <- input (x0 - 1 + hx, y0 - 1 + hy, z0 - 1 + hz)
        constexpr int B = 8;
        const int n = CL_HZ * CL_HY * CL_HX * cq;
        for (int e0 = threadIdx.x; e0 < n; e0 += B * 256) {
            uint4 v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * 256;
                const int c = e % cq, node = e / cq;
                const int hx = node % CL_HX, hy = (node / CL_HX) % CL_HY, hz = node / (CL_HX * CL_HY);
                const int xi = x0 - 1 + hx, yi = y0 - 1 + hy, zi = z0 - 1 + hz;
                v[u] = make_uint4(0, 0, 0, 0);
                if (e < n && xi >= 0 && yi >= 0 && zi >= 0 && xi < g.ix && yi < g.iy && zi < g.iz)
                    v[u] = *(const uint4*)(in + (((size_t)zi * g.iy + yi) * g.ix + xi) * g.cin + 8 * c);
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * 256;
                if (e < n) *(uint4*)(box + (size_t)e * 8) = v[u];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int z = z0 + w;
    const int K = 27 * g.cin;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[u][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    int t = (8 * kq) / g.cin, ci = 8 * kq - t * g.cin;   // this lane's tap and channel at chunk 0
    for (int kc = 0; kc < g.kpad; kc += 32) {
        const int k = kc + 8 * kq;
        uint4 b[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) b[j] = *(const uint4*)(wp + (size_t)(j * 16 + m) * g.kpad + k);
        uint4 a[MT];
        if (k < K) {
            const Off o = tap_off(t);
            // box node of output (x0 + m, y0 + u, z) plus the tap offset
            const int base = ((w + 1 + o.dz) * CL_HY + 1 + o.dy) * CL_HX + m + 1 + o.dx;
#pragma unroll
            for (int u = 0; u < MT; ++u) a[u] = *(const uint4*)(box + (size_t)(base + u * CL_HX) * g.cin + ci);
        } else {
#pragma unroll
            for (int u = 0; u < MT; ++u) a[u] = make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const bf16x8 av = as_bf16x8(a[u]);
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf16x8(b[j]), acc[u][j], 0, 0, 0);
        }
        ci += 32;
        while (ci >= g.cin) {
            ci -= g.cin;
            ++t;
        }
    }
    if (z >= g.nz) return;
    // epilogue: C[m' = 4 kq + i][n = lane % 16] of tile (u, j) is node
    // (x0 + m', y0 + u, z), channel 16 j + n
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = j * 16 + m;
        const float bias = ep.bias ? ep.bias[co] : 0.f;
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int y = y0 + u;
            if (y >= g.ny) continue;
            uint16_t add[4] = {0, 0, 0, 0}, msk[4] = {0, 0, 0, 0};
            const size_t rowv = ((size_t)z * g.ny + y) * g.nx;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = min(x0 + 4 * kq + i, g.nx - 1);
                if (ep.addend) add[i] = ep.addend[(rowv + x) * g.cout + co];
                if (ep.mask) msk[i] = ep.mask[(rowv + x) * g.cout + co];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * kq + i;
                if (x >= g.nx) continue;
                const size_t at = (rowv + x) * g.cout + co;
                float val = acc[u][j][i] + bias;
                if (ep.relu) val = fmaxf(val, 0.f);
                if (ep.addend) val += bf2f(add[i]);
                if (ep.mask && !(bf2f(msk[i]) > 0.f)) val = 0.f;
                if (ep.out_f32) ep.out_f32[at] = val;
                if (ep.out_bf16) ep.out_bf16[at] = f2bf(val);
            }
        }
    }
}

template <int MODE>
static hipError_t launch_conv_mode(const ConvGeom& g, const uint16_t* in, const uint16_t* wp, const ConvEpilogue& ep,
                                   hipStream_t s)
{
    // several node tiles per wave share the weight loads on large levels;
    // small levels keep one tile per wave so that enough waves exist
    const long nvox = (long)g.nx * g.ny * g.nz;
    auto grid = [&](int mt) { return dim3((unsigned)((nvox + 64L * mt - 1) / (64L * mt))); };
    const bool big = nvox >= 64L * 4 * 2048;
    switch ((g.cout / 16) * 2 + (big ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((k_conv<MODE, 1, 1>), grid(1), dim3(256), 0, s, g, in, wp, ep); break;
        case 3: hipLaunchKernelGGL((k_conv<MODE, 1, 4>), grid(4), dim3(256), 0, s, g, in, wp, ep); break;
        case 4: hipLaunchKernelGGL((k_conv<MODE, 2, 1>), grid(1), dim3(256), 0, s, g, in, wp, ep); break;
        case 5: hipLaunchKernelGGL((k_conv<MODE, 2, 4>), grid(4), dim3(256), 0, s, g, in, wp, ep); break;
        case 6: hipLaunchKernelGGL((k_conv<MODE, 3, 1>), grid(1), dim3(256), 0, s, g, in, wp, ep); break;
        case 7: hipLaunchKernelGGL((k_conv<MODE, 3, 2>), grid(2), dim3(256), 0, s, g, in, wp, ep); break;
        case 8: hipLaunchKernelGGL((k_conv<MODE, 4, 1>), grid(1), dim3(256), 0, s, g, in, wp, ep); break;
        case 9: hipLaunchKernelGGL((k_conv<MODE, 4, 2>), grid(2), dim3(256), 0, s, g, in, wp, ep); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_conv(const ConvGeom& g, const uint16_t* in, const uint16_t* wp, const ConvEpilogue& ep,
                       hipStream_t s)
{
    if (g.cin % 8 || g.cout % 16 || g.cout > 64 || g.kpad % 32 || g.kpad < 27 * g.cin) return hipErrorInvalidValue;
    // (on small levels the one-tile-per-wave gathers keep more waves busy
    // than the bricks do, so the LDS form serves the large ones)
    if (g.mode == CONV_SAME && g.cin <= CL_CMAX && g.ix == g.nx && g.iy == g.ny && g.iz == g.nz &&
        (long)g.nx * g.ny * g.nz >= LASTO_CONV_LDS_MIN_NODES) {
        const unsigned nb = (unsigned)(((g.nx + CL_BX - 1) / CL_BX) * ((g.ny + CL_BY - 1) / CL_BY) *
                                       ((g.nz + CL_BZ - 1) / CL_BZ));
        const int cm = g.cin <= 8 ? 8 : (g.cin <= 16 ? 16 : 32);
#define CL_CASE(nt, cmv)                                                                                  \
    case (nt) * 64 + (cmv):                                                                               \
        hipLaunchKernelGGL((k_conv_same_lds<nt, cmv>), dim3(nb), dim3(256), 0, s, g, in, wp, ep);       \
        break;
        switch ((g.cout / 16) * 64 + cm) {
            CL_CASE(1, 8) CL_CASE(1, 16) CL_CASE(1, 32)
            CL_CASE(2, 8) CL_CASE(2, 16) CL_CASE(2, 32)
            CL_CASE(3, 8) CL_CASE(3, 16) CL_CASE(3, 32)
            CL_CASE(4, 8) CL_CASE(4, 16) CL_CASE(4, 32)
            default: return hipErrorInvalidValue;
        }
#undef CL_CASE
        return hipGetLastError();
    }
    switch (g.mode) {
        case CONV_SAME: return launch_conv_mode<CONV_SAME>(g, in, wp, ep, s);
        case CONV_DOWN: return launch_conv_mode<CONV_DOWN>(g, in, wp, ep, s);
        case CONV_ADJ: return launch_conv_mode<CONV_ADJ>(g, in, wp, ep, s);
        case CONV_ADJD: return launch_conv_mode<CONV_ADJD>(g, in, wp, ep, s);
        default: return hipErrorInvalidValue;
    }
}

// ----------------------------------------------------- weight gradient
// dW[co][k] = sum_v gout[v][co] in[g(v, tap(k))][ci(k)] over the output
// nodes v of the forward layer (modes CONV_SAME and CONV_DOWN): a GEMM with
// M = co, N = k and the reduction over nodes. A workgroup takes one 16-wide
// column block of k and a contiguous share of the nodes, its four waves
// interleave 32-node steps, and the four waves' tiles are summed in LDS in a
// fixed order into one FP32 partial per workgroup: part[s][co][k].
template <int MODE, int MT>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvGeom g, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ gout, float* __restrict__ part,
                                                    long per_split)
{
    __shared__ float red[4][MT * 16 * 16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int nblk = blockIdx.x;          // 16 k-columns
    const int split = blockIdx.y;
    const long nvox = (long)g.nx * g.ny * g.nz;
    const long v_begin = split * per_split;
    const long v_end = v_begin + per_split < nvox ? v_begin + per_split : nvox;
    const int K = 27 * g.cin;
    const int kcol = nblk * 16 + m;        // this lane's B column
    const bool kok = kcol < K;
    const int t = kok ? kcol / g.cin : 0, ci = kok ? kcol - t * g.cin : 0;
    const Off o = tap_off(t);
    f32x4 acc[MT];
#pragma unroll
    for (int j = 0; j < MT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (long v0 = v_begin + 32 * w; v0 < v_end; v0 += 128) {
        // B[r][n]: in[g(v0 + 8 kq + i)][ci]; A[m][r]: gout[v0 + 8 kq + i][16 j + m]
        uint16_t bv[8], av[MT][8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const long v = v0 + 8 * kq + i;
            bv[i] = 0;
#pragma unroll
            for (int j = 0; j < MT; ++j) av[j][i] = 0;
            if (v >= v_end) continue;
            const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((long)g.nx * g.ny));
#pragma unroll
            for (int j = 0; j < MT; ++j) av[j][i] = gout[(size_t)v * g.cout + 16 * j + m];
            int xi, yi, zi;
            if (kok && gather_node<MODE>(x, y, z, o, g, xi, yi, zi))
                bv[i] = in[(((size_t)zi * g.iy + yi) * g.ix + xi) * g.cin + ci];
        }
        bf16x8 b;
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = __builtin_bit_cast(__bf16, bv[i]);
#pragma unroll
        for (int j = 0; j < MT; ++j) {
            bf16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = __builtin_bit_cast(__bf16, av[j][i]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
    }
    // C[m' = 4 kq + i][n = m] of tile j: co = 16 j + 4 kq + i, k = 16 nblk + m
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[w][(16 * j + 4 * kq + i) * 16 + m] = acc[j][i];
    __syncthreads();
    for (int e = threadIdx.x; e < MT * 256; e += 256) {
        const float sum = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        const int co = e / 16, kk = nblk * 16 + e % 16;
        if (kk < g.kpad) part[((size_t)split * g.cout + co) * g.kpad + kk] = sum;
    }
}

hipError_t launch_conv_wgrad(const ConvGeom& g, const uint16_t* in, const uint16_t* gout, float* part, int splits,
                             hipStream_t s)
{
    if (g.cin % 8 || g.cout % 16 || g.cout > 64 || (g.mode != CONV_SAME && g.mode != CONV_DOWN)) return hipErrorInvalidValue;
    const long nvox = (long)g.nx * g.ny * g.nz;
    const long per = ((nvox + splits - 1) / splits + 127) / 128 * 128;
    const dim3 grid((unsigned)(g.kpad / 16), (unsigned)splits);
#define WG(MODE, MT) hipLaunchKernelGGL((k_conv_wgrad<MODE, MT>), grid, dim3(256), 0, s, g, in, gout, part, per)
    if (g.mode == CONV_SAME) {
        switch (g.cout / 16) {
            case 1: WG(CONV_SAME, 1); break;
            case 2: WG(CONV_SAME, 2); break;
            case 3: WG(CONV_SAME, 3); break;
            case 4: WG(CONV_SAME, 4); break;
        }
    } else {
        switch (g.cout / 16) {
            case 1: WG(CONV_DOWN, 1); break;
            case 2: WG(CONV_DOWN, 2); break;
            case 3: WG(CONV_DOWN, 3); break;
            case 4: WG(CONV_DOWN, 4); break;
        }
    }
#undef WG
    return hipGetLastError();
}

// out[e] = sum_s part[s * n + e] in split order (+ out[e] when accumulate)
__global__ void k_sum_splits(const float* __restrict__ part, int splits, long n, float* __restrict__ out,
                             int accumulate)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        float a = 0.f;
        for (int s = 0; s < splits; ++s) a += part[(size_t)s * n + e];
        out[e] = accumulate ? out[e] + a : a;
    }
}

hipError_t launch_sum_splits(const float* part, int splits, long n, float* out, int accumulate, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, part, splits, n, out, accumulate);
    return hipGetLastError();
}

// per-channel sums (bias gradients): part[b][c] over node chunks, in order
__global__ __launch_bounds__(256) void k_chan_sum(const uint16_t* __restrict__ a, long nvox, int c, long per,
                                                  float* __restrict__ part)
{
    __shared__ float sh[256];
    const long v0 = blockIdx.x * per, v1 = v0 + per < nvox ? v0 + per : nvox;
    const int ch = threadIdx.x % c, lanes = 256 / c * c;   // threads ch, ch + c, ... sum channel ch
    float s = 0.f;
    if ((int)threadIdx.x < lanes)
        for (long v = v0 + threadIdx.x / c; v < v1; v += 256 / c) s += bf2f(a[(size_t)v * c + ch]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < c) {
        float t = 0.f;
        for (int q = threadIdx.x; q < lanes; q += c) t += sh[q];
        part[(size_t)blockIdx.x * c + threadIdx.x] = t;
    }
}

hipError_t launch_chan_sum(const uint16_t* a, long nvox, int c, float* part, int splits, hipStream_t s)
{
    if (c > 256) return hipErrorInvalidValue;
    const long per = (nvox + splits - 1) / splits;
    hipLaunchKernelGGL(k_chan_sum, dim3(splits), dim3(256), 0, s, a, nvox, c, per, part);
    return hipGetLastError();
}

// ------------------------------------------------------------ sampling
// Linear up-sampling in index space from a (n+1)/2 level to n: fine node i
// takes coarse i/2 when i is even, the mean of (i-1)/2 and (i+1)/2 when odd
// (per axis; the last coarse node stands in when i+1 falls outside), plus skip.
__device__ __forceinline__ void up_taps(int i, int nc, int& a, int& b, float& wa, float& wb)
{
    a = i >> 1;
    if (i & 1) {
        b = min(a + 1, nc - 1);
        wa = 0.5f;
        wb = 0.5f;
    } else {
        b = a;
        wa = 1.f;
        wb = 0.f;
    }
}

// One thread per fine node and group of 8 channels (16-byte loads and
// stores); a workgroup covers 64 x-consecutive nodes of one (y, z) row, so
// the row's index arithmetic is done once per thread, not per channel.
__device__ __forceinline__ void add8(float* acc, uint4 q, float w)
{
    const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        acc[2 * h] += w * __uint_as_float(u[h] << 16);
        acc[2 * h + 1] += w * __uint_as_float(u[h] & 0xffff0000u);
    }
}

__global__ __launch_bounds__(256) void k_upsample_add(const uint16_t* __restrict__ coarse, int cx, int cy, int cz,
                                                      const uint16_t* __restrict__ skip, uint16_t* __restrict__ out,
                                                      int nx, int ny, int nz, int c)
{
    const int g8 = c / 8;   // channel groups
    const int lanes = 64 * g8;
    const int t = blockIdx.x * 256 + threadIdx.x;   // within the row segment of this block
    const int y = blockIdx.y, z = blockIdx.z;
    const int x = t / g8, grp = t - x * g8;
    if (x >= nx || t >= lanes * ((nx + 63) / 64)) return;
    int xa, xb, ya, yb, za, zb;
    float wxa, wxb, wya, wyb, wza, wzb;
    up_taps(x, cx, xa, xb, wxa, wxb);
    up_taps(y, cy, ya, yb, wya, wyb);
    up_taps(z, cz, za, zb, wza, wzb);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int zz[2] = {za, zb}, yy[2] = {ya, yb}, xx[2] = {xa, xb};
    const float wz[2] = {wza, wzb}, wy[2] = {wya, wyb}, wx[2] = {wxa, wxb};
#pragma unroll
    for (int cz2 = 0; cz2 < 2; ++cz2)
#pragma unroll
        for (int cy2 = 0; cy2 < 2; ++cy2)
#pragma unroll
            for (int cx2 = 0; cx2 < 2; ++cx2) {
                const float w = wz[cz2] * wy[cy2] * wx[cx2];
                const uint4 q = *(const uint4*)(coarse + (((size_t)zz[cz2] * cy + yy[cy2]) * cx + xx[cx2]) * c + 8 * grp);
                add8(acc, q, w);
            }
    const size_t at = (((size_t)z * ny + y) * nx + x) * c + 8 * grp;
    if (skip) add8(acc, *(const uint4*)(skip + at), 1.f);
    uint32_t o[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) o[h] = (uint32_t)f2bf(acc[2 * h]) | ((uint32_t)f2bf(acc[2 * h + 1]) << 16);
    *(uint4*)(out + at) = make_uint4(o[0], o[1], o[2], o[3]);
}

hipError_t launch_upsample_add(const uint16_t* coarse, int cx, int cy, int cz, const uint16_t* skip, uint16_t* out,
                               int nx, int ny, int nz, int c, hipStream_t s)
{
    if (c % 8) return hipErrorInvalidValue;
    const long per_row = (long)((nx + 63) / 64) * 64 * (c / 8);
    const dim3 grid((unsigned)((per_row + 255) / 256), (unsigned)ny, (unsigned)nz);
    hipLaunchKernelGGL(k_upsample_add, grid, dim3(256), 0, s, coarse, cx, cy, cz, skip, out, nx, ny, nz, c);
    return hipGetLastError();
}

// The net's last two steps for inference, fused: u0 = BF16(up(coarse) +
// skip) and y = w . u0 + b at each fine node, without storing u0. The
// arithmetic (tap order, BF16 rounding of u0, the head's summation order) is
// that of k_upsample_add followed by k_head, so y is the same bit for bit.
__global__ __launch_bounds__(256) void k_upsample_head(const uint16_t* __restrict__ coarse, int cx, int cy, int cz,
                                                       const uint16_t* __restrict__ skip, int nx, int ny, int nz,
                                                       int c, const float* __restrict__ w, float* __restrict__ y)
{
    const int x = blockIdx.x * 256 + threadIdx.x, yq = blockIdx.y, z = blockIdx.z;
    if (x >= nx) return;
    int xa, xb, ya, yb, za, zb;
    float wxa, wxb, wya, wyb, wza, wzb;
    up_taps(x, cx, xa, xb, wxa, wxb);
    up_taps(yq, cy, ya, yb, wya, wyb);
    up_taps(z, cz, za, zb, wza, wzb);
    const int zz[2] = {za, zb}, yy[2] = {ya, yb}, xx[2] = {xa, xb};
    const float wz[2] = {wza, wzb}, wy[2] = {wya, wyb}, wx[2] = {wxa, wxb};
    const size_t node = ((size_t)z * ny + yq) * nx + x;
    float s = w[c];
    for (int q0 = 0; q0 < c; q0 += 8) {
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int cz2 = 0; cz2 < 2; ++cz2)
#pragma unroll
            for (int cy2 = 0; cy2 < 2; ++cy2)
#pragma unroll
                for (int cx2 = 0; cx2 < 2; ++cx2) {
                    const float wt = wz[cz2] * wy[cy2] * wx[cx2];
                    const uint4 q =
                        *(const uint4*)(coarse + (((size_t)zz[cz2] * cy + yy[cy2]) * cx + xx[cx2]) * c + q0);
                    add8(acc, q, wt);
                }
        add8(acc, *(const uint4*)(skip + node * c + q0), 1.f);
#pragma unroll
        for (int h = 0; h < 8; ++h) s += w[q0 + h] * bf2f(f2bf(acc[h]));
    }
    y[node] = s;
}

hipError_t launch_upsample_head(const uint16_t* coarse, int cx, int cy, int cz, const uint16_t* skip, int nx, int ny,
                                int nz, int c, const float* w, float* y, hipStream_t s)
{
    if (c % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_upsample_head, dim3((unsigned)((nx + 255) / 256), (unsigned)ny, (unsigned)nz), dim3(256), 0,
                       s, coarse, cx, cy, cz, skip, nx, ny, nz, c, w, y);
    return hipGetLastError();
}

// adjoint of the up-sampling: coarse node I gathers the fine nodes whose taps
// name it, with the same weights; out (FP32) then optionally masked by the
// ReLU of act (> 0) and rounded to BF16
__device__ __forceinline__ float up_adj_w(int I, int i, int nc)
{
    int a, b;
    float wa, wb;
    up_taps(i, nc, a, b, wa, wb);
    return (a == I ? wa : 0.f) + (b == I ? wb : 0.f);
}

__global__ void k_upsample_adj(const uint16_t* __restrict__ fine, int nx, int ny, int nz, uint16_t* __restrict__ out,
                               int cx, int cy, int cz, int c, const uint16_t* __restrict__ act)
{
    const long n = (long)cx * cy * cz * c;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c);
        const long v = e / c;
        const int X = (int)(v % cx), Y = (int)((v / cx) % cy), Z = (int)(v / ((long)cx * cy));
        float s = 0.f;
        for (int dz = -1; dz <= 2; ++dz) {
            const int z = 2 * Z + dz;
            if (z < 0 || z >= nz) continue;
            const float wz = up_adj_w(Z, z, cz);
            if (wz == 0.f) continue;
            for (int dy = -1; dy <= 2; ++dy) {
                const int y = 2 * Y + dy;
                if (y < 0 || y >= ny) continue;
                const float wy = up_adj_w(Y, y, cy);
                if (wy == 0.f) continue;
                for (int dx = -1; dx <= 2; ++dx) {
                    const int x = 2 * X + dx;
                    if (x < 0 || x >= nx) continue;
                    const float wx = up_adj_w(X, x, cx);
                    if (wx == 0.f) continue;
                    s += wz * wy * wx * bf2f(fine[(((size_t)z * ny + y) * nx + x) * c + ch]);
                }
            }
        }
        if (act && !(bf2f(act[e]) > 0.f)) s = 0.f;
        out[e] = f2bf(s);
    }
}

hipError_t launch_upsample_adj(const uint16_t* fine, int nx, int ny, int nz, uint16_t* out, int cx, int cy, int cz, int c,
                               const uint16_t* act, hipStream_t s)
{
    const long n = (long)cx * cy * cz * c;
    hipLaunchKernelGGL(k_upsample_adj, dim3((unsigned)std::min<long>((n + 255) / 256, 16384)), dim3(256), 0, s, fine, nx,
                       ny, nz, out, cx, cy, cz, c, act);
    return hipGetLastError();
}

// ------------------------------------------------------ output and loss
// y[v] = sum_c w[c] a[v][c] + w[c] (the 1x1x1 output layer, FP32 result;
// the bias is the last weight); one node per thread, channels in 16-byte loads
__global__ __launch_bounds__(256) void k_head(const uint16_t* __restrict__ a, long nvox, int c,
                                              const float* __restrict__ w, float* __restrict__ y)
{
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long)gridDim.x * blockDim.x) {
        float s = w[c];
        for (int q0 = 0; q0 < c; q0 += 8) {
            float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            add8(acc, *(const uint4*)(a + (size_t)v * c + q0), 1.f);
#pragma unroll
            for (int h = 0; h < 8; ++h) s += w[q0 + h] * acc[h];
        }
        y[v] = s;
    }
}

hipError_t launch_head(const uint16_t* a, long nvox, int c, const float* w, float* y, hipStream_t s)
{
    if (c % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_head, dim3((unsigned)std::min<long>((nvox + 255) / 256, 16384)), dim3(256), 0, s, a, nvox, c, w,
                       y);
    return hipGetLastError();
}

// loss = sum_v wt[v] (y[v] - t[v])^2 (partials per block); dy = 2 wt (y - t);
// da[v][c] = w[c] dy[v] (BF16); head-weight partials pw[b][q] = sum_v a[v][q] dy[v]
// for q < c and pw[b][c] = sum_v dy[v] (the bias).
constexpr int HEAD_CMAX = 16;

__global__ __launch_bounds__(256) void k_head_loss_bwd(const uint16_t* __restrict__ a, long nvox, int c,
                                                       const float* __restrict__ w, const float* __restrict__ y,
                                                       const float* __restrict__ tgt, const float* __restrict__ wt,
                                                       uint16_t* __restrict__ da, double* __restrict__ lossp,
                                                       float* __restrict__ pw, long per)
{
    __shared__ double shl[256];
    __shared__ float shw[256];
    const long v0 = blockIdx.x * per, v1 = v0 + per < nvox ? v0 + per : nvox;
    double l = 0.0;
    float hp[HEAD_CMAX + 1];
#pragma unroll
    for (int q = 0; q <= HEAD_CMAX; ++q) hp[q] = 0.f;
    for (long v = v0 + threadIdx.x; v < v1; v += 256) {
        const float d = y[v] - tgt[v];
        l += (double)wt[v] * (double)d * (double)d;
        const float dy = 2.f * wt[v] * d;
#pragma unroll
        for (int q = 0; q < HEAD_CMAX; ++q) {
            if (q < c) {
                hp[q] += bf2f(a[(size_t)v * c + q]) * dy;
                da[(size_t)v * c + q] = f2bf(w[q] * dy);
            }
        }
        hp[HEAD_CMAX] += dy;
    }
    shl[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 256; ++q) t += shl[q];
        lossp[blockIdx.x] = t;
    }
#pragma unroll
    for (int q = 0; q <= HEAD_CMAX; ++q) {
        if (q < c || q == HEAD_CMAX) {
            __syncthreads();
            shw[threadIdx.x] = hp[q];
            __syncthreads();
            if (threadIdx.x == 0) {
                float t = 0.f;
                for (int r = 0; r < 256; ++r) t += shw[r];
                pw[(size_t)blockIdx.x * (c + 1) + (q < c ? q : c)] = t;
            }
        }
    }
}

hipError_t launch_head_loss_bwd(const uint16_t* a, long nvox, int c, const float* w, const float* y, const float* tgt,
                                const float* wt, uint16_t* da, double* lossp, float* pw, int splits, hipStream_t s)
{
    if (c > HEAD_CMAX) return hipErrorInvalidValue;
    const long per = (nvox + splits - 1) / splits;
    hipLaunchKernelGGL(k_head_loss_bwd, dim3(splits), dim3(256), 0, s, a, nvox, c, w, y, tgt, wt, da, lossp, pw, per);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Adam
// FP32 master weights w (natural [27][cin][cout] order for convolutions),
// moments m, v; step t (1-based). Bias-corrected Adam.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, long n, float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, s, w, m, v, g, n, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// Packed BF16 weights of a convolution from its FP32 master W[t][ci][co]:
//   forward  wp[co][k],  k = t cin + ci          (kpad columns, zero-padded)
//   adjoint  wa[ci][k'], k' = t cout + co        (kpad_adj columns)
// The adjoint applies W[t]^T to the output gradient at the same tap.
__global__ void k_pack_weights(const float* __restrict__ W, int cin, int cout, uint16_t* __restrict__ wp, int kpad,
                               uint16_t* __restrict__ wa, int kpad_adj, int cin_rows)
{
    const long nf = (long)cout * kpad;
    const long na = wa ? (long)cin_rows * kpad_adj : 0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nf + na; e += (long)gridDim.x * blockDim.x) {
        if (e < nf) {
            const int co = (int)(e / kpad), k = (int)(e % kpad);
            float val = 0.f;
            if (k < 27 * cin) {
                const int t = k / cin, ci = k % cin;
                val = W[((size_t)t * cin + ci) * cout + co];
            }
            wp[e] = f2bf(val);
        } else {
            const long f = e - nf;
            const int ci = (int)(f / kpad_adj), k = (int)(f % kpad_adj);
            float val = 0.f;
            if (ci < cin && k < 27 * cout) {
                const int t = k / cout, co = k % cout;
                val = W[((size_t)t * cin + ci) * cout + co];
            }
            wa[f] = f2bf(val);
        }
    }
}

hipError_t launch_pack_weights(const float* W, int cin, int cout, uint16_t* wp, int kpad, uint16_t* wa, int kpad_adj,
                               int cin_rows, hipStream_t s)
{
    const long n = (long)cout * kpad + (wa ? (long)cin_rows * kpad_adj : 0);
    hipLaunchKernelGGL(k_pack_weights, dim3((unsigned)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, s, W, cin, cout,
                       wp, kpad, wa, kpad_adj, cin_rows);
    return hipGetLastError();
}

// dW in the master order [t][ci][co] from the GEMM result dWt[co][k]
__global__ void k_unpack_wgrad(const float* __restrict__ dwt, int cin, int cout, int kpad, float* __restrict__ dw)
{
    const long n = 27L * cin * cout;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int co = (int)(e % cout);
        const long tk = e / cout;   // t * cin + ci
        dw[e] = dwt[(size_t)co * kpad + tk];
    }
}

hipError_t launch_unpack_wgrad(const float* dwt, int cin, int cout, int kpad, float* dw, hipStream_t s)
{
    const long n = 27L * cin * cout;
    hipLaunchKernelGGL(k_unpack_wgrad, dim3((unsigned)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, s, dwt, cin,
                       cout, kpad, dw);
    return hipGetLastError();
}

// FP32 -> BF16 and BF16 -> FP32 copies
__global__ void k_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b, long n)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) b[e] = f2bf(a[e]);
}
__global__ void k_to_f32(const uint16_t* __restrict__ a, float* __restrict__ b, long n)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) b[e] = bf2f(a[e]);
}

hipError_t launch_to_bf16(const float* a, uint16_t* b, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)std::min<long>((n + 255) / 256, 16384)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}
hipError_t launch_to_f32(const uint16_t* a, float* b, long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<long>((n + 255) / 256, 16384)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

}  // namespace net
}  // namespace lasto
