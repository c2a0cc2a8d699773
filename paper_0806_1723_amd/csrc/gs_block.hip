// Red-black Gauss-Seidel half-sweeps fused into one pass over a level
// (gfx950, wave64): the smoother of the multigrid cycle for the finite
// difference form of eq. (3.2), on correction arrays whose faces are zero.
//
// A half-sweep reads one colour and writes the other, about 12 bytes per
// updated node, and the cycle runs several in a row (pre- and post-smoothing).
// Here S of them (colours c0, 1 - c0, c0, ...) share one pass over the level.
//
// A workgroup is 16 waves; wave w holds row j0 - S + w of the tile and lane l
// colour entry m0 - S + l of it (64 entries). It marches up a chunk of planes:
// at step t half-sweep s updates plane t - s. In the colour-split layout all
// the nodes a lane updates at one step lie in one physical column i = 2 m + o
// (o = (c0 + j + t) & 1 for every s), and their neighbours are
//   z:  (i, j, t - s + 1), half-sweep s - 1 at this step, and (i, j, t - s - 1),
//       half-sweep s - 1 two steps ago: both in the lane's registers;
//   x:  the other column of the lane's entry pair, half-sweep s - 1 one step
//       ago (registers), and the adjacent lane's value of the same (a DPP
//       lane shift, its direction uniform over the wave);
//   y:  rows j -+ 1, half-sweep s - 1 one step ago: the only values that go
//       through LDS, published once per step, so a step has one barrier.
// Half-sweep -1 stands for the input: plane t + 1 of colour 1 - c0, loaded.
// Half-sweep s is exact on lanes s + 1 .. 62 - s of waves s + 1 .. 14 - s
// (each one needs its neighbours' values of the one before), so the output
// tile is GbShape::TX entries by TY rows; neighbouring workgroups recompute
// the halo rather than exchange it. The pass reads one colour of its input
// and f once and writes both colours once, and its result is that of S
// separate half-sweeps bit for bit (gs_update: the same operations in the
// same order per node).
//
// The input is read from `uin` and the result written to `uout`, distinct
// arrays: a workgroup writes planes that its neighbours read as halo. With
// ZERO_IN the input is zero and nothing is read.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include "internal.h"
#include "kern_util.h"

namespace lasto {

constexpr int GB_ROWS = 16;      // waves (rows) of a workgroup
constexpr int GB_NT = 64 * GB_ROWS;
constexpr int GB_DEPTH = 4;      // steps the global loads run ahead
constexpr int GB_KC_MAX = 128;   // planes of a chunk

template <typename T, int S> struct GbShape {
    static constexpr int TX = 64 - 2 * S;        // output entries of a row
    static constexpr int TY = GB_ROWS - 2 * S;   // output rows
    static constexpr int LDS_BYTES =
        2 * S * GB_NT * (int)sizeof(T) + (2 * (int)sizeof(T) + 12) * (GB_KC_MAX + 2 * S) + 8 * GB_ROWS;
};

// the pass lengths built: FP32 up to 6, FP64 up to 4 (beyond, its registers
// would spill at 16 waves per workgroup)
template <typename T, int S> constexpr bool gb_fits()
{
    return GbShape<T, S>::LDS_BYTES <= 160 * 1024 - 64 && (sizeof(T) == 4 || S <= 4);
}

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& fn)
{
    if constexpr (I < N) {
        fn(std::integral_constant<int, I>{});
        static_for<I + 1, N>(fn);
    }
}

// lane l takes lane l - 1's value (UP) or lane l + 1's (zero past the ends)
template <bool UP>
__device__ __forceinline__ float lane_shift(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), UP ? 0x138 : 0x130, 0xf, 0xf, false));
}
template <bool UP>
__device__ __forceinline__ double lane_shift(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), UP ? 0x138 : 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), UP ? 0x138 : 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <typename T, int S, bool ZERO_IN, bool DOT, bool TOP>
__global__ __launch_bounds__(GB_NT) void k_gs_block(LevelView L, const T* __restrict__ uin, const T* __restrict__ f,
                                                    T* __restrict__ uout, int c0, T bscale, double* __restrict__ dotp,
                                                    int nbx, int nby, int nb, int per, int kc)
{
    using G = GbShape<T, S>;
    static_assert(gb_fits<T, S>(), "the published values exceed the LDS of a compute unit");
    constexpr int D = sizeof(T) == 8 ? GB_DEPTH / 2 : GB_DEPTH;
    // values of half-sweeps -1 .. S - 2 published at a step, for the y
    // neighbours at the next: [step & 1][half-sweep + 1][wave][lane]
    __shared__ T pub[2 * S * GB_NT];
    // z coefficients, interior-plane flags and (dot products) z volume
    // factors of planes lo0 .. hi0
    __shared__ T zam[GB_KC_MAX + 2 * S], zap[GB_KC_MAX + 2 * S];
    __shared__ int zok[GB_KC_MAX + 2 * S];
    __shared__ double zvol[DOT ? GB_KC_MAX + 2 * S : 1];
    __shared__ double red[GB_NT / 64];
    const int t = xcd_tile(blockIdx.x, per);
    if (t >= nb) {
        if (DOT && threadIdx.x == 0) dotp[blockIdx.x] = 0.0;
        return;
    }
    const int nx = L.nx, ny = L.ny, nz = L.nz, W = L.W;
    const size_t plane = (size_t)ny * W, cs = L.cs;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m0 = (t % nbx) * G::TX;
    const int j0 = 1 + ((t / nbx) % nby) * G::TY;
    const int k0 = 1 + (t / (nbx * nby)) * kc;
    const int k1 = min(k0 + kc, nz - 1);
    const int cin = 1 - c0;
    const int j = j0 - S + w, m = m0 - S + lane;
    const bool row_in = j >= 0 && j < ny, ent_in = m >= 0 && m < W;
    const bool iy = j >= 1 && j <= ny - 2;
    const bool ix0 = ent_in && 2 * m >= 1 && 2 * m <= nx - 2;
    const bool ix1 = ent_in && 2 * m + 1 >= 1 && 2 * m + 1 <= nx - 2;
    const bool tile_row = w >= S && w < S + G::TY && j <= ny - 2;
    const bool tile = tile_row && lane >= S && lane < S + G::TX && ent_in;
    const int jc = min(max(j, 1), ny - 2), mc = min(max(m, 0), W - 1);
    const T* __restrict__ xp = XPar<T>::get(L);
    const T cxm0 = xp[(size_t)0 * W + mc], cxp0 = xp[(size_t)1 * W + mc];
    const T cxm1 = xp[(size_t)3 * W + mc], cxp1 = xp[(size_t)4 * W + mc];
    const T cym = tab_am<T>(L.ax[1])[jc], cyp = tab_ap<T>(L.ax[1])[jc];
    const T* __restrict__ amz = tab_am<T>(L.ax[2]);
    const T* __restrict__ apz = tab_ap<T>(L.ax[2]);
    T vx0 = T(0), vx1 = T(0);
    double vy = 0.0;
    if (DOT) {
        vx0 = xp[(size_t)2 * W + mc];
        vx1 = xp[(size_t)5 * W + mc];
        vy = L.ax[1].m[jc];
    }
    // this lane's entry of a colour plane (clamped into the arrays: loads are
    // unconditional and masked when used)
    const size_t at = (size_t)min(max(j, 0), ny - 1) * W + min(max(m, 0), W - 1);

    // planes half-sweep s updates: [lo(s), hi(s)]
    auto lo = [&](int s) { return max(1, k0 - (S - 1 - s)); };
    auto hi = [&](int s) { return min(nz - 2, k1 - 1 + (S - 1 - s)); };
    const int lo0 = lo(0), hi0 = hi(0);

    // values of half-sweeps -1 .. S - 1 (index s + 1): this step, one and
    // two steps ago
    T cur[S + 1], p1[S + 1], p2[S + 1];
#pragma unroll
    for (int k = 0; k <= S; ++k) cur[k] = p1[k] = p2[k] = T(0);
    // f of the even half-sweeps' colour c0 on planes t - i (qa[i]) and of the
    // odd ones' colour 1 - c0 on planes t - 1 - i (qb[i])
    T qa[S], qb[S];
#pragma unroll
    for (int k = 0; k < S; ++k) qa[k] = qb[k] = T(0);
    // loads in flight, one set per step of the unrolled loop: the input on
    // plane t + 1, f (c0) on plane t and f (1 - c0) on plane t - 1
    T lin[D], lfa[D], lfb[D];
    auto issue = [&](auto uc, int tt) {
        constexpr int u = decltype(uc)::value;
        const size_t pin = (size_t)min(max(tt + 1, 0), nz - 1) * plane;
        const size_t pfa = (size_t)min(max(tt, 0), nz - 1) * plane;
        const size_t pfb = (size_t)min(max(tt - 1, 0), nz - 1) * plane;
        lin[u] = ZERO_IN ? T(0) : uin[cin * cs + pin + at];
        lfa[u] = f[c0 * cs + pfa + at];
        lfb[u] = f[cin * cs + pfb + at];
    };
    const bool node_in = row_in && ent_in;
    // the input on plane p, zero outside the arrays
    auto input_at = [&](T v, int p) { return (!ZERO_IN && node_in && p >= 0 && p <= nz - 1) ? v : T(0); };

    for (int i = threadIdx.x; i <= hi0 - lo0; i += GB_NT) {
        zam[i] = amz[lo0 + i];
        zap[i] = apz[lo0 + i];
        zok[i] = L.zint[lo0 + i];
        if (DOT) zvol[DOT ? i : 0] = L.ax[2].m[lo0 + i];
    }
    double dot = 0.0;
    // prologue: the input on planes lo0 - 1 and lo0 (half-sweep -1 two and
    // one steps before lo0), published for the y neighbours of lo0
    {
        const size_t pa = (size_t)min(max(lo0 - 1, 0), nz - 1) * plane, pb = (size_t)min(lo0, nz - 1) * plane;
        T a = ZERO_IN ? T(0) : uin[cin * cs + pa + at];
        T b = ZERO_IN ? T(0) : uin[cin * cs + pb + at];
        p2[0] = input_at(a, lo0 - 1);
        p1[0] = input_at(b, lo0);
        pub[(((lo0 - 1) & 1) * S + 0) * GB_NT + threadIdx.x] = p1[0];
    }
    static_for<0, D>([&](auto uc) { issue(uc, lo0 + decltype(uc)::value); });
    __syncthreads();

    const int last = k1 + S - 2;   // half-sweep S - 1 reaches plane k1 - 1
    for (int base = lo0; base <= last; base += D) {
        static_for<0, D>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            const int tt = base + u;
            const int o = (c0 + j + tt) & 1;   // uniform over the wave
            const T cxm = o ? cxm1 : cxm0, cxp = o ? cxp1 : cxp0;
            const bool ix = o ? ix1 : ix0;
            // half-sweep -1: the input on plane tt + 1; f entering the queues
            cur[0] = input_at(lin[u], tt + 1);
#pragma unroll
            for (int k = S - 1; k > 0; --k) {
                qa[k] = qa[k - 1];
                qb[k] = qb[k - 1];
            }
            qa[0] = lfa[u];
            qb[0] = lfb[u];
            issue(uc, tt + D);
            // y neighbours of every half-sweep: published one step ago
            const T* prev = pub + ((tt - 1) & 1) * S * GB_NT;
            T ym[S], yp[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                ym[s] = prev[s * GB_NT + max(w - 1, 0) * 64 + lane];
                yp[s] = prev[s * GB_NT + min(w + 1, GB_ROWS - 1) * 64 + lane];
            }
            // z coefficients of every half-sweep's plane
            T czm[S], czp[S];
            int zk[S];
            double zv[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int zi = min(max(tt - s - lo0, 0), hi0 - lo0);
                czm[s] = zam[zi];
                czp[s] = zap[zi];
                zk[s] = zok[zi];
                zv[s] = DOT ? zvol[DOT ? zi : 0] : 0.0;
            }
            // x neighbours from the adjacent lane: one step old values
            T xn[S];
#pragma unroll
            for (int s = 0; s < S; ++s) xn[s] = o ? lane_shift<false>(p1[s]) : lane_shift<true>(p1[s]);
            static_for<0, S>([&](auto sc) {
                constexpr int s = decltype(sc)::value;
                const int p = tt - s;
                T r = T(0);
                if (p >= lo(s) && p <= hi(s) && w >= s + 1 && w <= GB_ROWS - 2 - s) {
                    T fv;
                    if constexpr ((s & 1) != 0)
                        fv = qb[s - 1];
                    else
                        fv = qa[s];
                    const T xl = o ? p1[s] : xn[s], xr = o ? xn[s] : p1[s];
                    if (ZERO_IN && s == 0)
                        r = gs_update0(cxm, cxp, cym, cyp, czm[s], czp[s], bscale, fv);
                    else
                        r = gs_update(cxm, cxp, xl, xr, cym, cyp, ym[s], yp[s], czm[s], czp[s], p2[s], cur[s], bscale,
                                      fv);
                    const bool ok = zk[s] && iy && ix;
                    r = ok ? r : T(0);
                    if (DOT && s >= S - 2 && tile && p >= k0 && p < k1) {
                        dot += (double)(o ? vx1 : vx0) * (vy * zv[s]) * (double)fv * (double)r;
                    }
                }
                cur[s + 1] = r;
            });
            // publish for the next step (half-sweeps -1 .. S - 2)
            T* mine = pub + (tt & 1) * S * GB_NT;
#pragma unroll
            for (int s = 0; s < S; ++s) mine[s * GB_NT + threadIdx.x] = cur[s];
            // plane tt - S + 1 is final: colour c_{S-1} now, c_{S-2} one step ago
            const int q = tt - S + 1;
            if (tile && q >= k0 && q < k1) {
                uout[((c0 + S - 1) & 1) * cs + (size_t)q * plane + at] = cur[S];
                uout[((c0 + S - 2) & 1) * cs + (size_t)q * plane + at] = p1[S - 1];
            }
#pragma unroll
            for (int k = 0; k <= S; ++k) {
                p2[k] = p1[k];
                p1[k] = cur[k];
            }
            __syncthreads();
        });
    }
    if (DOT) {
        const double sm = block_sum<GB_NT>(dot, red);
        if (threadIdx.x == 0) dotp[blockIdx.x] = sm;
    }
}

struct GbLaunch {
    int nbx, nby, nbz, nb, per, kc;
};

// Planes per chunk: a workgroup takes kc + 2 S - 2 steps, and the launch
// about rounds x that, rounds being how many tiles the busiest of the cap
// resident workgroups takes; kc minimises it (the larger on a tie, which
// recomputes fewer halo planes).
static GbLaunch gb_shape(const LevelView& L, int S, int tx, int ty, int cap)
{
    GbLaunch g;
    g.nbx = ((L.nx - 2) / 2) / tx + 1;
    g.nby = (L.ny - 2 + ty - 1) / ty;
    const long tiles = (long)g.nbx * g.nby;
    const int planes = L.nz - 2;
    long best = -1;
    g.kc = 1;
    for (int k = 1; k <= std::min(planes, GB_KC_MAX); ++k) {
        const long n = tiles * ((planes + k - 1) / k);
        const long cost = ((n + cap - 1) / cap) * (k + 2 * S - 2);
        if (best < 0 || cost <= best) {
            best = cost;
            g.kc = k;
        }
    }
    g.nbz = (planes + g.kc - 1) / g.kc;
    g.nb = g.nbx * g.nby * g.nbz;
    g.per = (g.nb + 7) / 8;
    return g;
}

template <typename T, int S, bool ZERO_IN, bool DOT, bool TOP>
static int gb_cap()
{
    static const int cap = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 8;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 8;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gs_block<T, S, ZERO_IN, DOT, TOP>, GB_NT, 0) !=
            hipSuccess)
            return 8;
        return std::max(8, per_cu * cus / 8 * 8);
    }();
    return cap;
}

template <typename T, int S, bool ZERO_IN, bool DOT, bool TOP>
static hipError_t launch_gb(const LevelView& L, const T* uin, const T* f, T* uout, int c0, T bscale, double* dotp,
                            hipStream_t st, int* nparts, hipEvent_t ev0, hipEvent_t ev1)
{
    const GbLaunch g = gb_shape(L, S, GbShape<T, S>::TX, GbShape<T, S>::TY, gb_cap<T, S, ZERO_IN, DOT, TOP>());
    const dim3 grid(8 * g.per), block(GB_NT);
    if (ev0 && ev1)
        hipExtLaunchKernelGGL((k_gs_block<T, S, ZERO_IN, DOT, TOP>), grid, block, 0, st, ev0, ev1, 0, L, uin, f, uout,
                              c0, bscale, dotp, g.nbx, g.nby, g.nb, g.per, g.kc);
    else
        hipLaunchKernelGGL((k_gs_block<T, S, ZERO_IN, DOT, TOP>), grid, block, 0, st, L, uin, f, uout, c0, bscale,
                           dotp, g.nbx, g.nby, g.nb, g.per, g.kc);
    if (nparts) *nparts = 8 * g.per;
    return hipGetLastError();
}

template <> int gs_block_max<float>() { return 6; }
template <> int gs_block_max<double>() { return 4; }

template <typename T, int S, bool TOP>
static hipError_t launch_gb_s(const LevelView& L, const T* uin, const T* f, T* uout, int c0, int zero_in, T bscale,
                              double* dotp, hipStream_t st, int* nparts, hipEvent_t ev0, hipEvent_t ev1)
{
    if constexpr (!gb_fits<T, S>()) {
        return hipErrorInvalidValue;
    } else {
        if (zero_in)
            return launch_gb<T, S, true, false, TOP>(L, uin, f, uout, c0, bscale, nullptr, st, nparts, ev0, ev1);
        if (dotp) return launch_gb<T, S, false, true, TOP>(L, uin, f, uout, c0, bscale, dotp, st, nparts, ev0, ev1);
        return launch_gb<T, S, false, false, TOP>(L, uin, f, uout, c0, bscale, nullptr, st, nparts, ev0, ev1);
    }
}

template <typename T>
hipError_t launch_gs_block(const LevelView& L, const T* uin, const T* f, T* uout, int c0, int nsweeps, int zero_in,
                           T bscale, double* dotp, hipStream_t st, int* nparts, int top, hipEvent_t ev0,
                           hipEvent_t ev1)
{
    if (zero_in && dotp) return hipErrorInvalidValue;
    if (!zero_in && (void*)uin == (void*)uout) return hipErrorInvalidValue;
    if (c0 != 0 && c0 != 1) return hipErrorInvalidValue;
#define GB_CASE(NS)                                                                                             \
    case NS:                                                                                                    \
        return top ? launch_gb_s<T, NS, true>(L, uin, f, uout, c0, zero_in, bscale, dotp, st, nparts, ev0, ev1) \
                   : launch_gb_s<T, NS, false>(L, uin, f, uout, c0, zero_in, bscale, dotp, st, nparts, ev0, ev1);
    switch (nsweeps) {
        GB_CASE(2)
        GB_CASE(4)
        GB_CASE(6)
    default:
        return hipErrorInvalidValue;
    }
#undef GB_CASE
}

// partials a dot-product pass of launch_gs_block may write on this level
// (the most over the pass lengths and precisions)
template <typename T, int S>
static int gb_parts_t(const LevelView& L)
{
    if constexpr (!gb_fits<T, S>())
        return 0;
    else
        return 8 * std::max(gb_shape(L, S, GbShape<T, S>::TX, GbShape<T, S>::TY, gb_cap<T, S, false, true, false>()).per,
                            gb_shape(L, S, GbShape<T, S>::TX, GbShape<T, S>::TY, gb_cap<T, S, false, true, true>()).per);
}

int gs_block_parts(const LevelView& L)
{
    int n = 0;
    n = std::max(n, gb_parts_t<float, 2>(L));
    n = std::max(n, gb_parts_t<float, 4>(L));
    n = std::max(n, gb_parts_t<float, 6>(L));
    n = std::max(n, gb_parts_t<double, 2>(L));
    n = std::max(n, gb_parts_t<double, 4>(L));
    return n;
}

template <typename A, typename B>
__global__ void k_cast(const A* __restrict__ a, B* __restrict__ b, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        b[t] = (B)a[t];
}

template <typename A, typename B>
static hipError_t cast_t(const A* a, B* b, size_t n, hipStream_t s)
{
    const int blocks = (int)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL((k_cast<A, B>), dim3(blocks), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_cast(const double* a, float* b, size_t n, hipStream_t s) { return cast_t(a, b, n, s); }
hipError_t launch_cast(const float* a, double* b, size_t n, hipStream_t s) { return cast_t(a, b, n, s); }

template hipError_t launch_gs_block<float>(const LevelView&, const float*, const float*, float*, int, int, int, float,
                                           double*, hipStream_t, int*, int, hipEvent_t, hipEvent_t);
template hipError_t launch_gs_block<double>(const LevelView&, const double*, const double*, double*, int, int, int,
                                            double, double*, hipStream_t, int*, int, hipEvent_t, hipEvent_t);

}  // namespace lasto
