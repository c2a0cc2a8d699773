// Device helpers shared by the multigrid kernel files (gfx950, wave64).
#pragma once

#include "internal.h"

namespace lasto {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum (fixed tree); result valid in thread 0. Every
// thread of the block must call it.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NT / 64; ++w) t += sh[w];
    }
    return t;
}

// Workgroups are dispatched to the eight XCDs in turn; tile (id % 8) * per +
// id / 8 hands each XCD a contiguous run of tiles, so tiles that share halo
// rows share an L2. Ids past the last tile only contribute a zero partial.
__device__ __forceinline__ int xcd_tile(int id, int per) { return (id & 7) * per + (id >> 3); }

// 16 bytes of one colour row: VEC consecutive entries (4 FP32, 2 FP64)
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <> struct Vec16<double> {
    typedef double V __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

template <typename T> __device__ __forceinline__ const T* tab_am(const Axis& a);
template <typename T> __device__ __forceinline__ const T* tab_ap(const Axis& a);
template <> __device__ __forceinline__ const float* tab_am<float>(const Axis& a) { return a.amf; }
template <> __device__ __forceinline__ const float* tab_ap<float>(const Axis& a) { return a.apf; }
template <> __device__ __forceinline__ const double* tab_am<double>(const Axis& a) { return a.am; }
template <> __device__ __forceinline__ const double* tab_ap<double>(const Axis& a) { return a.ap; }

// 1/d: the hardware reciprocal refined by Newton steps r <- r + r (1 - d r)
// (one in FP32, two in FP64), within about half an ulp of the quotient
__device__ __forceinline__ float recip(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(fmaf(-d, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// Gauss-Seidel update of one node, (sum_d am_d u_{n-e_d} + ap_d u_{n+e_d} -
// bscale f_n) / sum_d (am_d + ap_d), with every rounding step written out
// (explicit fused multiply-adds in a fixed order), so that any kernel that
// calls it gets the same bits for the same operands.
template <typename T>
__device__ __forceinline__ T gs_update(T cxm, T cxp, T xl, T xr, T cym, T cyp, T ym, T yp, T czm, T czp, T zm, T zp,
                                       T bscale, T f)
{
    const T d = cxm + cxp + cym + cyp + czm + czp;
    T s = fma(cxm, xl, cxp * xr);
    s = fma(cym, ym, s);
    s = fma(cyp, yp, s);
    s = fma(czm, zm, s);
    s = fma(czp, zp, s);
    return fma(-bscale, f, s) * recip(d);
}
// the same with every neighbour zero (the first half-sweep from zero)
template <typename T>
__device__ __forceinline__ T gs_update0(T cxm, T cxp, T cym, T cyp, T czm, T czp, T bscale, T f)
{
    const T d = cxm + cxp + cym + cyp + czm + czp;
    return fma(-bscale, f, T(0)) * recip(d);
}

}  // namespace lasto
