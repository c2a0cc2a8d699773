// Multigrid and Krylov kernels of the Poisson solve (eq. (3.2)) on the graded
// tensor-product mesh, gfx950 (wave64). All of these are HBM-bound stencils
// and streams; none uses MFMA.
//
// Operator (interior node n, per axis d):
//   (A u)_n = sum_d am_d (u_{n-e_d} - u_n) + ap_d (u_{n+e_d} - u_n)
// with am = 1/(h_- m), ap = 1/(h_+ m), m = (h_- + h_+)/2: the three-point
// second difference on a nonuniform mesh. Equation A u = bscale * f.
//
// Multigrid arrays use the colour-split layout of internal.h (sidx). Natural
// [nz][ny][nx] arrays appear only at the fine level (the caller's rho and v).
#include <algorithm>

#include <hip/hip_ext.h>

#include "internal.h"
#include "kern_util.h"

namespace lasto {

// ------------------------------------------------------------- helpers
__device__ __forceinline__ int block_linear()
{
    return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

__device__ __forceinline__ double vol_at(const LevelView& L, int i, int j, int k)
{
    return L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k];
}

size_t split_elems(const LevelView& L) { return 2 * L.cs; }

// Solve of one node's equation from its six neighbours (GS update).
template <typename T>
__device__ __forceinline__ T gs_point(const LevelView& L, const T* __restrict__ u, int i, int j, int k, T fb)
{
    const T cxm = (T)L.ax[0].am[i], cxp = (T)L.ax[0].ap[i];
    const T cym = (T)L.ax[1].am[j], cyp = (T)L.ax[1].ap[j];
    const T czm = (T)L.ax[2].am[k], czp = (T)L.ax[2].ap[k];
    T s = cxm * u[sidx(L, i - 1, j, k)] + cxp * u[sidx(L, i + 1, j, k)];
    s += cym * u[sidx(L, i, j - 1, k)] + cyp * u[sidx(L, i, j + 1, k)];
    s += czm * u[sidx(L, i, j, k - 1)] + czp * u[sidx(L, i, j, k + 1)];
    return (s - fb) / (cxm + cxp + cym + cyp + czm + czp);
}

// (A u) at interior (i,j,k) of a split array
template <typename T>
__device__ __forceinline__ T apply_split(const LevelView& L, const T* __restrict__ u, int i, int j, int k, T c)
{
    T a = (T)L.ax[0].am[i] * (u[sidx(L, i - 1, j, k)] - c) + (T)L.ax[0].ap[i] * (u[sidx(L, i + 1, j, k)] - c);
    a += (T)L.ax[1].am[j] * (u[sidx(L, i, j - 1, k)] - c) + (T)L.ax[1].ap[j] * (u[sidx(L, i, j + 1, k)] - c);
    a += (T)L.ax[2].am[k] * (u[sidx(L, i, j, k - 1)] - c) + (T)L.ax[2].ap[k] * (u[sidx(L, i, j, k + 1)] - c);
    return a;
}

// Restriction R = M_c^-1 P^T M_f gathers, per axis, the fine nodes rf-1..rf+1
// of coarse node I with weights rw. The solver restricts only residuals that
// vanish on black nodes (right after a black half-sweep), so only red fine
// nodes are read. In a fine row of parity q = (jj + kk) & 1 the red nodes are
// those with i = q (mod 2), at entry i >> 1 of the red colour row; the red
// taps of coarse I in that row are therefore entries m0 = (fi - 1) >> 1 and
// m0 + 1, weighted (wx1 on fi alone) when fi = q (mod 2), else (wx0, wx2 on
// fi - 1, fi + 1). RTaps holds both weight pairs of one coarse I.
template <typename T> struct RTaps {
    T s0, s1;   // fi red
    T d0, d1;   // fi black
    int m0, e;  // first entry, parity of fi
};

template <typename T>
__device__ __forceinline__ RTaps<T> restrict_taps(const LevelView& C, int I)
{
    RTaps<T> x;
    const int fi = C.ax[0].rf[I];
    const double* w = C.ax[0].rw + 3 * I;
    x.e = fi & 1;
    x.m0 = (fi - 1) >> 1;
    x.s0 = x.e ? (T)w[1] : T(0);
    x.s1 = x.e ? T(0) : (T)w[1];
    x.d0 = (T)w[0];
    x.d1 = (T)w[2];
    return x;
}

// restricted red residual at coarse (I, J, K), I given by its taps. The 18
// loads are unconditional (zero weights included, every index inside the fine
// array) so that they are all in flight at once.
template <typename T>
__device__ __forceinline__ T restrict_red_at(const LevelView& F, const LevelView& C, const T* __restrict__ r,
                                             const RTaps<T>& x, int J, int K)
{
    const int fj = C.ax[1].rf[J], fk = C.ax[2].rf[K];
    const double* wy = C.ax[1].rw + 3 * J;
    const double* wz = C.ax[2].rw + 3 * K;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T plane = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int jj = fj - 1 + b, kk = fk - 1 + c;
            const bool same = ((jj + kk) & 1) == x.e;
            const T* row = r + ((size_t)kk * F.ny + jj) * F.W + x.m0;   // red colour: the first half of r
            plane += (T)wy[b] * ((same ? x.s0 : x.d0) * row[0] + (same ? x.s1 : x.d1) * row[1]);
        }
        acc += (T)wz[c] * plane;
    }
    return acc;
}

// Prolongation: fine node i lies in coarse cell (pc_i, pc_i + 1) with linear
// weights in physical coordinates (1 and 0 at a kept node). For an interior
// fine node pc_i + 1 is still a coarse node (possibly on a face), so all eight
// coarse values can be loaded unconditionally.
template <typename T> struct PTaps {
    int I;
    T w0, w1;
};

template <typename T>
__device__ __forceinline__ PTaps<T> prolong_taps(const Axis& a, int i)
{
    PTaps<T> t;
    t.I = a.pc[i];
    t.w0 = (T)a.pw[2 * i];
    t.w1 = (T)a.pw[2 * i + 1];
    return t;
}

// interpolated coarse correction at fine (i, j, k), i given by its taps
template <typename T>
__device__ __forceinline__ T prolong_at(const LevelView& C, const T* __restrict__ e, const PTaps<T>& x, int j, int k)
{
    const PTaps<T> y = prolong_taps<T>(C.ax[1], j), z = prolong_taps<T>(C.ax[2], k);
    const int ma = x.I >> 1, mb = (x.I + 1) >> 1;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        T s = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int Jb = y.I + b, Kc = z.I + c;
            const size_t row = ((size_t)Kc * C.ny + Jb) * C.W;
            const int ca = (x.I + Jb + Kc) & 1;   // colour of coarse node I; I + 1 has the other
            const T va = e[(size_t)ca * C.cs + row + ma];
            const T vb = e[(size_t)(ca ^ 1) * C.cs + row + mb];
            s += (b ? y.w1 : y.w0) * (x.w0 * va + x.w1 * vb);
        }
        acc += (c ? z.w1 : z.w0) * s;
    }
    return acc;
}

// --------------------------------------------------------- half-sweep
enum HalfMode { HM_GS = 0, HM_RESID = 1, HM_APPLY = 2, HM_APPLY2 = 3 };

// Over the nodes of colour c (VEC neighbouring entries m0 .. m0+VEC-1 of a
// colour row per thread, 16 bytes, loaded as one vector):
//   HM_GS    out_n = (sum_d am_d u_{n-e_d} + ap_d u_{n+e_d} - bscale f_n) / sum_d (am_d + ap_d)
//            (the Gauss-Seidel update of a red-black half-sweep; dot += vol f out)
//   HM_RESID out_n = bscale f_n - (A u)_n
//   HM_APPLY out_n = (A u)_n                                     (dot += vol u out)
//   HM_APPLY2 HM_APPLY on both colours in one launch: tile ids 2t and 2t+1
//            are the two colours of spatial tile t, side by side in an
//            XCD's run, so the colour each reads as its neighbours is the
//            one the other has just read (launched with c = 0: uo colour 1,
//            ucen colour 0, out colour 0 of out's two colours)
// The neighbours all have the other colour: entry m of the other colour on
// planes k-1 and k+1 holds the z neighbours, entries m-1+o and m+o the x
// neighbours (o = (c+j+k) & 1), rows j-1 and j+1 the y neighbours; the x
// neighbours of a group are its own vector of the other colour plus one
// entry past its left (o = 0) or right (o = 1) end. A thread marches over a
// chunk of planes keeping the z neighbours in a register queue and loading
// plane k+1's operands while it computes plane k. `uo` (other colour), `fc`,
// `ucen` and `out` (this colour) are distinct arrays, so the loads may run
// ahead of the stores. A workgroup is 32 groups (a 512-byte run of a row)
// by 8 rows.
constexpr int H2_X = 32, H2_Y = 8, H2_NT = H2_X * H2_Y, H2_KC_MAX = 16, H2_BLOCKS = 2048;

struct HalfShape {
    int nbx, nby, nbz, nb, per, grid, kc;
};

// Planes per thread (kc): the march saves re-reads, but a workgroup's
// planes form a serial chain and its first planes are start-up, so the
// cost of a launch is about rounds x (kc + 2), rounds being how many tiles
// the busiest of the cap resident workgroups takes. kc minimises that (the
// smaller on a tie).
static int chunk_planes(long tiles, int planes, int cap, int kmax)
{
    int best = 1;
    long best_cost = -1;
    for (int k = 1; k <= kmax; ++k) {
        const long nb = tiles * ((planes + k - 1) / k);
        const long rounds = (nb + cap - 1) / cap;
        const long cost = rounds * (k + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = k;
        }
    }
    return best;
}

static HalfShape half_shape(const LevelView& L, int vec, int cap = H2_BLOCKS)
{
    HalfShape h;
    // groups of VEC entries m0 = VEC g with m0 <= (nx-2)/2 (the last entry
    // that can hold an interior node)
    const int ngroups = ((L.nx - 2) / 2) / vec + 1;
    h.nbx = (ngroups + H2_X - 1) / H2_X;
    h.nby = (L.ny - 2 + H2_Y - 1) / H2_Y;
    const long tiles = (long)h.nbx * h.nby;
    h.kc = chunk_planes(tiles, L.nz - 2, std::max(cap, 8), H2_KC_MAX);
    h.nbz = (L.nz - 2 + h.kc - 1) / h.kc;
    h.nb = h.nbx * h.nby * h.nbz;
    h.per = (h.nb + 7) / 8;
    h.grid = 8 * h.per;
    return h;
}

int half_blocks(const LevelView& L) { return half_shape(L, 2).grid; }

template <typename T> struct HalfOps {
    typename Vec16<T>::V ym, yp, fv, cv;   // y neighbours, f and centre of a group
    T xe;                                  // the x neighbour outside the z queue
};

// TOP marks finest-level launches; it changes no code, only the kernel's name,
// so that a kernel trace separates the finest level from the coarse ones.
template <typename T, int MODE, bool ZERO_IN, bool DOT, bool ZERO_FACES, bool TOP>
__global__ __launch_bounds__(H2_NT) void k_half2(LevelView L, const T* __restrict__ uo, const T* __restrict__ fc,
                                                 const T* __restrict__ ucen, T* __restrict__ out, int c, T bscale,
                                                 double* __restrict__ dotp, int nbx, int nby, int nb, int per, int kc)
{
    typedef typename Vec16<T>::V VT;
    constexpr int VEC = Vec16<T>::N;
    __shared__ double red[H2_NT / 64];
    constexpr bool BOTH = MODE == HM_APPLY2;
    constexpr int M = BOTH ? HM_APPLY : MODE;   // the node arithmetic
    constexpr bool NEED_U = !ZERO_IN || M != HM_GS;
    double dot = 0.0;
    const int nx = L.nx, nz = L.nz, W = L.W;
    const size_t plane = (size_t)L.ny * W;
    const T* __restrict__ xp = XPar<T>::get(L);
    const T* __restrict__ amz = tab_am<T>(L.ax[2]);
    const T* __restrict__ apz = tab_ap<T>(L.ax[2]);
    // Persistent workgroups: workgroup b takes ids b, b + G, ... (G =
    // gridDim.x, a multiple of 8, so every id it takes maps to a tile of the
    // XCD it runs on).
    for (int id = blockIdx.x; id < 8 * per; id += gridDim.x) {
        const int tt = xcd_tile(id, per);
        const int t = BOTH ? tt >> 1 : tt;          // the spatial tile
        const int cc = BOTH ? (c ^ (tt & 1)) : c;   // and its colour
        const T* __restrict__ po = BOTH && cc != c ? ucen : uo;   // other colour
        const T* __restrict__ pc = BOTH && cc != c ? uo : ucen;   // this colour
        T* __restrict__ pq = BOTH && cc != c ? out + L.cs : out;
        const int m0 = VEC * ((t % nbx) * H2_X + (threadIdx.x & (H2_X - 1)));
        const int j = 1 + ((t / nbx) % nby) * H2_Y + (threadIdx.x / H2_X);
        if (!(t < nb && j <= L.ny - 2 && m0 <= (nx - 2) / 2)) continue;
        const int k0 = 1 + (t / (nbx * nby)) * kc;
        const int k1 = min(k0 + kc, nz - 1);
        const size_t row = (size_t)j * W + m0;
        // both parities' x coefficients, picked per plane by select (named
        // values, not an array indexed at run time, so they stay in registers)
        const VT axm0 = *(const VT*)(xp + (size_t)0 * W + m0), axm1 = *(const VT*)(xp + (size_t)3 * W + m0);
        const VT axp0 = *(const VT*)(xp + (size_t)1 * W + m0), axp1 = *(const VT*)(xp + (size_t)4 * W + m0);
        VT axv0 = VT(T(0)), axv1 = VT(T(0));
        if (DOT) {
            axv0 = *(const VT*)(xp + (size_t)2 * W + m0);
            axv1 = *(const VT*)(xp + (size_t)5 * W + m0);
        }
        const T cym = tab_am<T>(L.ax[1])[j], cyp = tab_ap<T>(L.ax[1])[j];
        const double vy = DOT ? L.ax[1].m[j] : 0.0;
        // the x neighbour not in the z queue: entry m0+VEC (o = 1) or m0-1
        // (o = 0; m0 = 0 has no interior node there)
        const int xoff1 = VEC, xoff0 = m0 > 0 ? -1 : 0;
        auto load_plane = [&](int k, HalfOps<T>& q) {
            const size_t at = (size_t)k * plane + row;
            const int o = (cc + j + k) & 1;
            if (M != HM_APPLY) q.fv = *(const VT*)(fc + at);
            if (M != HM_GS) q.cv = *(const VT*)(pc + at);
            if (NEED_U) {
                q.ym = *(const VT*)(po + at - W);
                q.yp = *(const VT*)(po + at + W);
                q.xe = po[at + (o ? xoff1 : xoff0)];
            }
        };
        auto load_z = [&](int k) -> VT {
            VT z = VT(T(0));
            if (NEED_U) z = *(const VT*)(po + (size_t)k * plane + row);
            return z;
        };
        // plane k from its operands and the z neighbours (zm, zc, zp)
        auto compute = [&](int k, const HalfOps<T>& q, const VT& zm, const VT& zc, const VT& zp) {
            const int o = (cc + j + k) & 1;
            const int i0 = o + 2 * m0;
            const bool okz = L.zint[k];   // planes next to another copy of a batch are faces
            const VT cxm = o ? axm1 : axm0, cxp = o ? axp1 : axp0;
            const T czm = amz[k], czp = apz[k];
            VT r;
            bool ok[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                ok[e] = okz && i0 + 2 * e >= 1 && i0 + 2 * e <= nx - 2;
                // x neighbours of entry e: o = 1: (zc[e], zc[e+1] or xe); o = 0: (zc[e-1] or xe, zc[e])
                const T xl = o ? zc[e] : (e > 0 ? zc[e > 0 ? e - 1 : 0] : q.xe);
                const T xr = o ? (e + 1 < VEC ? zc[e + 1 < VEC ? e + 1 : e] : q.xe) : zc[e];
                if (M == HM_GS) {
                    if (NEED_U)
                        r[e] = gs_update(cxm[e], cxp[e], xl, xr, cym, cyp, q.ym[e], q.yp[e], czm, czp, zm[e], zp[e],
                                         bscale, q.fv[e]);
                    else
                        r[e] = gs_update0(cxm[e], cxp[e], cym, cyp, czm, czp, bscale, q.fv[e]);
                } else {
                    // (A u) in difference form, which keeps FP32 free of cancellation
                    const T c0 = q.cv[e];
                    T a = cxm[e] * (xl - c0) + cxp[e] * (xr - c0);
                    a += cym * (q.ym[e] - c0) + cyp * (q.yp[e] - c0);
                    a += czm * (zm[e] - c0) + czp * (zp[e] - c0);
                    r[e] = M == HM_RESID ? bscale * q.fv[e] - a : a;
                }
            }
            const size_t at = (size_t)k * plane + row;
            if (ZERO_FACES) {
                // face and padding entries of this array are zero: store the
                // group unconditionally, with zero where a node is not interior
                VT w;
#pragma unroll
                for (int e = 0; e < VEC; ++e) w[e] = ok[e] ? r[e] : T(0);
                *(VT*)(pq + at) = w;
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (ok[e]) pq[at + e] = r[e];
            }
            if (DOT) {
                const double vz = okz ? vy * L.ax[2].m[k] : 0.0;
                const VT av = o ? axv1 : axv0;   // zero off the interior
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T a = M == HM_APPLY ? q.cv[e] : q.fv[e];
                    dot += (double)av[e] * vz * (double)a * (double)(ok[e] ? r[e] : T(0));
                }
            }
        };
        // two planes per step with alternating operand sets (A: even steps,
        // B: odd), so the next plane's loads are in flight while one plane is
        // computed and no register copies wait on them
        HalfOps<T> A{}, B{};
        VT z0 = load_z(k0 - 1), z1 = load_z(k0), z2 = load_z(k0 + 1);
        load_plane(k0, A);
        for (int k = k0; k < k1; k += 2) {
            load_plane(min(k + 1, k1 - 1), B);
            const VT z3 = load_z(min(k + 2, nz - 1));
            compute(k, A, z0, z1, z2);
            if (k + 1 < k1) {
                load_plane(min(k + 2, k1 - 1), A);
                const VT z4 = load_z(min(k + 3, nz - 1));
                compute(k + 1, B, z1, z2, z3);
                z0 = z2;
                z1 = z3;
                z2 = z4;
            }
        }
    }
    if (DOT) {
        const double s = block_sum<H2_NT>(dot, red);
        if (threadIdx.x == 0) dotp[blockIdx.x] = s;
    }
}

// Resident workgroups of one half-sweep variant on the whole device (a
// multiple of 8, at least 8); the persistent launch never exceeds it, so no
// workgroup waits for a second round.
template <typename T, int MODE, bool ZERO_IN, bool DOT, bool ZERO_FACES, bool TOP>
static int half_cap()
{
    static const int cap = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 8;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 8;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_half2<T, MODE, ZERO_IN, DOT, ZERO_FACES, TOP>, H2_NT,
                                                         0) != hipSuccess)
            return 8;
        return std::max(8, per_cu * cus / 8 * 8);
    }();
    return cap;
}

// ev0/ev1 (optional): events that take the dispatch's own start and end
// timestamps (hipExtLaunchKernelGGL), i.e. the kernel's execution time alone.
template <typename T, int MODE, bool ZERO_IN, bool DOT, bool ZERO_FACES, bool TOP = false>
static hipError_t launch_half2(const LevelView& L, const T* u, const T* f, T* out, int colour, T bscale,
                               double* dotp, hipStream_t s, int* nparts, hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr)
{
    const int cap = half_cap<T, MODE, ZERO_IN, DOT, ZERO_FACES, TOP>();
    const HalfShape h = half_shape(L, Vec16<T>::N, cap);
    const int G = std::min(h.grid, cap);
    const size_t own = (size_t)colour * L.cs, other = (size_t)(1 - colour) * L.cs;
    const T* fo = f ? f + own : (const T*)nullptr;
    if (ev0 && ev1)
        hipExtLaunchKernelGGL((k_half2<T, MODE, ZERO_IN, DOT, ZERO_FACES, TOP>), dim3(G), dim3(H2_NT), 0, s, ev0, ev1,
                              0, L, u + other, fo, u + own, out + own, colour, bscale, dotp, h.nbx, h.nby, h.nb, h.per,
                              h.kc);
    else
        hipLaunchKernelGGL((k_half2<T, MODE, ZERO_IN, DOT, ZERO_FACES, TOP>), dim3(G), dim3(H2_NT), 0, s, L,
                           u + other, fo, u + own, out + own, colour, bscale, dotp, h.nbx, h.nby, h.nb, h.per, h.kc);
    if (nparts) *nparts = G;
    return hipGetLastError();
}

// In the multigrid arrays (corrections, right-hand sides, residuals) faces
// and padding are zero, so the sweeps store pairs unconditionally.
template <typename T, bool TOP>
static hipError_t launch_half_t(const LevelView& L, T* u, const T* f, int colour, int zero_in, T bscale,
                                double* dotp, hipStream_t s, int* nparts, hipEvent_t ev0, hipEvent_t ev1)
{
    if (zero_in) {
        if (dotp)
            return launch_half2<T, HM_GS, true, true, true, TOP>(L, u, f, u, colour, bscale, dotp, s, nparts, ev0, ev1);
        return launch_half2<T, HM_GS, true, false, true, TOP>(L, u, f, u, colour, bscale, nullptr, s, nparts, ev0, ev1);
    }
    if (dotp)
        return launch_half2<T, HM_GS, false, true, true, TOP>(L, u, f, u, colour, bscale, dotp, s, nparts, ev0, ev1);
    return launch_half2<T, HM_GS, false, false, true, TOP>(L, u, f, u, colour, bscale, nullptr, s, nparts, ev0, ev1);
}

template <typename T>
hipError_t launch_half(const LevelView& L, T* u, const T* f, int colour, int zero_in, T bscale, double* dotp,
                       hipStream_t s, int* nparts, int top, hipEvent_t ev0, hipEvent_t ev1)
{
    if (top) return launch_half_t<T, true>(L, u, f, colour, zero_in, bscale, dotp, s, nparts, ev0, ev1);
    return launch_half_t<T, false>(L, u, f, colour, zero_in, bscale, dotp, s, nparts, ev0, ev1);
}

// the same half-sweep on an array whose faces hold Dirichlet data (kept)
template <typename T>
hipError_t launch_half_keep_faces(const LevelView& L, T* u, const T* f, int colour, T bscale, hipStream_t s)
{
    return launch_half2<T, HM_GS, false, false, false>(L, u, f, u, colour, bscale, nullptr, s, nullptr);
}

// residual f - A u at the nodes of one colour only (written into that
// colour of r; the other colour of r is not touched)
template <typename T>
hipError_t launch_residual_colour(const LevelView& L, const T* u, const T* f, T* r, int colour, hipStream_t s)
{
    return launch_half2<T, HM_RESID, false, false, true>(L, u, f, r, colour, T(1), nullptr, s, nullptr);
}

// q = A p on both colours in one launch (HM_APPLY2), with partials of
// <p, q>_W
template <typename T>
hipError_t launch_apply_both(const LevelView& L, const T* p, T* q, double* dotp, hipStream_t s, int* nparts)
{
    const int cap = half_cap<T, HM_APPLY2, false, true, true, false>();
    const HalfShape h = half_shape(L, Vec16<T>::N, cap);
    const int per = (2 * h.nb + 7) / 8;   // ids over both colours of every tile
    const int G = std::min(8 * per, cap);
    hipLaunchKernelGGL((k_half2<T, HM_APPLY2, false, true, true, false>), dim3(G), dim3(H2_NT), 0, s, L, p + L.cs,
                       (const T*)nullptr, p, q, 0, T(1), dotp, h.nbx, h.nby, h.nb, per, h.kc);
    if (nparts) *nparts = G;
    return hipGetLastError();
}

// ------------------------------------------------- pointwise 3-D launches
// A workgroup covers a 64 x 4 tile of (i, j) interior columns over a chunk
// of kp planes (kp chosen to keep about PT_BLOCKS workgroups); split arrays
// are read through sidx, so a wavefront touches two contiguous runs (one per
// colour). Reducing kernels write one partial per tile.
//
// The grid is 1-D, eight runs of `per` workgroups: xcd_tile hands each XCD
// a contiguous run of the gx x gy x gz tiles (x fastest), so tiles that
// share the cache lines at their x ends and the rows next to them (the y
// neighbours of a march) are read through one L2 instead of eight.
constexpr int PT_X = 64, PT_Y = 4, PT_NT = PT_X * PT_Y, PT_BLOCKS = 4096, PT_KP_MAX = 32;

struct PtShape {
    dim3 grid;
    int kp;
};

static dim3 pt_grid(int gx, int gy, int gz)
{
    const long tiles = (long)gx * gy * gz;
    return dim3((unsigned)(8 * ((tiles + 7) / 8)));
}

static PtShape pt_shape(const LevelView& L)
{
    PtShape p;
    const int gx = (L.nx - 2 + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    const long tiles = (long)gx * gy;
    p.kp = (int)std::min<long>(PT_KP_MAX, std::max<long>(1, (long)(L.nz - 2) * tiles / PT_BLOCKS));
    p.grid = pt_grid(gx, gy, (L.nz - 2 + p.kp - 1) / p.kp);
    return p;
}

// This workgroup's tile (bx, by, bz) and its linear index t = bx + gx (by +
// gy bz); ok is false for the few ids past the last tile.
struct PtTile {
    int bx, by, bz, t;
    bool ok;
};

__device__ __forceinline__ PtTile pt_tile(const LevelView& L, int kp)
{
    const int gx = (L.nx - 2 + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    const int gz = (L.nz - 2 + kp - 1) / kp;
    PtTile p;
    p.t = xcd_tile(blockIdx.x, gridDim.x >> 3);
    p.ok = p.t < gx * gy * gz;
    p.bx = p.t % gx;
    p.by = (p.t / gx) % gy;
    p.bz = p.t / (gx * gy);
    return p;
}

// zint of the planes kb-1 .. kb+62 as the bits of a wave-uniform mask (bit
// k - kb + 1 is zint[k]; one byte load per lane, once). Must be reached by
// every lane of the wave. A byte load inside a plane loop goes through the
// vector memory path, and the wait for it also waits for every load issued
// before it, which undoes any prefetch.
static_assert(PT_KP_MAX + 2 <= 64, "a chunk's planes and their neighbours fit one mask");
__device__ __forceinline__ unsigned long long zint_mask(const LevelView& L, int kb)
{
    const int k = kb - 1 + (int)(threadIdx.x & 63);
    return __ballot(k < L.nz && L.zint[k]);
}

__device__ __forceinline__ bool zbit(unsigned long long m, int k, int kb) { return (m >> (k - kb + 1)) & 1ull; }

// Resident workgroups of 256 threads on the device when each takes at most
// 64 VGPRs (eight per compute unit), at least 8
static int resident_256()
{
    static const int cap = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 8;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 8;
        return std::max(8, 8 * cus);
    }();
    return cap;
}

static int chunk_planes(long tiles, int planes, int cap, int kmax);

// The residual kernels march up their planes (z-queue, one plane of loads
// ahead): their chunk follows the same cost model as the half-sweeps.
static PtShape residual_shape(const LevelView& L)
{
    PtShape p;
    const int gx = (L.nx - 2 + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    p.kp = chunk_planes((long)gx * gy, L.nz - 2, resident_256(), PT_KP_MAX);
    p.grid = pt_grid(gx, gy, (L.nz - 2 + p.kp - 1) / p.kp);
    return p;
}

// partials of a residual norm (one per tile of residual_shape)
int interior_blocks(const LevelView& L)
{
    const int gx = (L.nx - 2 + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    const int kp = residual_shape(L).kp;
    return gx * gy * ((L.nz - 2 + kp - 1) / kp);
}

// (bodies skip planes that are faces of a batch copy: !ZINT(k))
#define INTERIOR_LOOP                                                 \
    const PtTile tl_ = pt_tile(L, kp);                                \
    if (!tl_.ok) return;                                              \
    const int i = 1 + tl_.bx * PT_X + (threadIdx.x % PT_X);           \
    const int j = 1 + tl_.by * PT_Y + (threadIdx.x / PT_X);           \
    const bool inside = (i <= L.nx - 2) && (j <= L.ny - 2);           \
    const int kb_ = 1 + tl_.bz * kp;                                  \
    const int ke_ = min(kb_ + kp, L.nz - 1);                          \
    const unsigned long long zm_ = zint_mask(L, kb_);                 \
    for (int k = kb_; k < ke_; ++k)

// zint[k] of a plane of this INTERIOR_LOOP's or ROW_LOOP's chunk
#define ZINT(k) zbit(zm_, (k), kb_)

#define PT_LAUNCH(kernel, L, s, ...)                                                         \
    do {                                                                                     \
        const PtShape ps_ = pt_shape(L);                                                     \
        hipLaunchKernelGGL(kernel, ps_.grid, dim3(PT_NT), 0, s, L, ps_.kp, __VA_ARGS__);      \
    } while (0)

// Fine level, natural v and rho: r = bscale rho - A v (r in the split
// layout, FP64 or FP32, when given) and partials of ||r||_W^2. Each thread
// marches its (i, j) column up its chunk of planes: the centre values of
// planes k-1, k, k+1 stay in registers, a wave covers 64 consecutive nodes
// of a row, so the x neighbours are the adjacent lanes' centres (a lane at
// either end of the wave loads its outer neighbour), and plane k+1's y
// neighbours and rho are loaded before plane k is computed.
template <typename TO>
__global__ __launch_bounds__(PT_NT) void k_residual_march(LevelView L, int kp, const double* __restrict__ v,
                                                          const double* __restrict__ rho, double bscale,
                                                          TO* __restrict__ r, double* __restrict__ part)
{
    static_assert(PT_X == 64, "a wave covers one row segment");
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    const PtTile tl = pt_tile(L, kp);
    if (!tl.ok) return;   // (the whole workgroup)
    const int lane = threadIdx.x % PT_X;
    const int i = 1 + tl.bx * PT_X + lane;
    const int j = 1 + tl.by * PT_Y + (threadIdx.x / PT_X);
    const int kb = 1 + tl.bz * kp;
    const int ke = min(kb + kp, L.nz - 1);
    const int nx = L.nx;
    // every lane of a row that exists takes part in the shuffles: lanes past
    // the row's last interior node hold the face value (or a clamped copy)
    const bool row_ok = j <= L.ny - 2;
    const bool inside = row_ok && i <= nx - 2;
    const int ic = min(i, nx - 1);
    const size_t sxy = (size_t)nx * L.ny;
    const size_t col = (size_t)min(j, L.ny - 1) * nx + ic;
    const double cxm = L.ax[0].am[min(i, nx - 2)], cxp = L.ax[0].ap[min(i, nx - 2)];
    const double cym = L.ax[1].am[min(j, L.ny - 2)], cyp = L.ax[1].ap[min(j, L.ny - 2)];
    const double vxy = L.ax[0].m[min(i, nx - 2)] * L.ax[1].m[min(j, L.ny - 2)];
    const bool first = lane == 0, last = lane == PT_X - 1;
    struct Ops {
        double ym, yp, b, xo;   // xo: the outer x neighbour of an end lane
    };
    auto load = [&](int k) {
        Ops o;
        const size_t idx = (size_t)k * sxy + col;
        o.b = inside ? rho[idx] : 0.0;
        o.ym = inside ? v[idx - nx] : 0.0;
        o.yp = inside ? v[idx + nx] : 0.0;
        o.xo = (inside && (first || last)) ? v[first ? idx - 1 : idx + 1] : 0.0;
        return o;
    };
    // centres of planes k-1, k, k+1
    auto centre = [&](int k) -> double { return row_ok ? v[(size_t)k * sxy + col] : 0.0; };
    const unsigned long long zm_ = zint_mask(L, kb);
    double zm = centre(kb - 1), zc = centre(kb);
    Ops A = load(kb);
    for (int k = kb; k < ke; ++k) {
        const double zp = centre(k + 1);
        Ops B = A;
        if (k + 1 < ke) B = load(k + 1);
        // x neighbours from the adjacent lanes' centres
        const double sl = __shfl_up(zc, 1, 64), sr = __shfl_down(zc, 1, 64);
        const double xm = first ? A.xo : sl, xp = last ? A.xo : sr;
        if (inside && zbit(zm_, k, kb)) {
            double a = cxm * (xm - zc) + cxp * (xp - zc);
            a += cym * (A.ym - zc) + cyp * (A.yp - zc);
            a += L.ax[2].am[k] * (zm - zc) + L.ax[2].ap[k] * (zp - zc);
            const double res = bscale * A.b - a;
            if (r) r[sidx(L, i, j, k)] = (TO)res;
            acc += vxy * L.ax[2].m[k] * res * res;
        }
        zm = zc;
        zc = zp;
        A = B;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[tl.t] = t;
}

// The reference residual of the face data alone: the interior of v is read
// as zero, so only rho and the face values next to a node are read. With no
// neighbours to share there is no march: a thread takes RF planes of its
// column at a time and issues all their loads together (the tiles and
// partials are k_residual_march's).
template <typename TO>
__global__ __launch_bounds__(PT_NT) void k_residual_faces(LevelView L, int kp, const double* __restrict__ v,
                                                          const double* __restrict__ rho, double bscale,
                                                          TO* __restrict__ r, double* __restrict__ part)
{
    constexpr int RF = 2;
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    const PtTile tl = pt_tile(L, kp);
    if (!tl.ok) return;   // (the whole workgroup)
    const int i = 1 + tl.bx * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + tl.by * PT_Y + (threadIdx.x / PT_X);
    const int kb = 1 + tl.bz * kp;
    const int ke = min(kb + kp, L.nz - 1);
    const int nx = L.nx, ny = L.ny;
    const bool inside = i <= nx - 2 && j <= ny - 2;
    const size_t sxy = (size_t)nx * ny;
    const size_t col = (size_t)min(j, ny - 1) * nx + min(i, nx - 1);
    const double cxm = L.ax[0].am[min(i, nx - 2)], cxp = L.ax[0].ap[min(i, nx - 2)];
    const double cym = L.ax[1].am[min(j, ny - 2)], cyp = L.ax[1].ap[min(j, ny - 2)];
    const double vxy = L.ax[0].m[min(i, nx - 2)] * L.ax[1].m[min(j, ny - 2)];
    const bool fxm = i == 1, fxp = i == nx - 2, fym = j == 1, fyp = j == ny - 2;
    const unsigned long long zm_ = zint_mask(L, kb);
    for (int k0 = kb; k0 < ke; k0 += RF) {
        double b[RF], xm[RF], xp[RF], ym[RF], yp[RF], zm[RF], zp[RF];
        bool ok[RF], fzm[RF], fzp[RF];
#pragma unroll
        for (int u = 0; u < RF; ++u) {
            const int k = k0 + u;
            ok[u] = inside && k < ke && zbit(zm_, k, kb);
            fzm[u] = ok[u] && !zbit(zm_, k - 1, kb);
            fzp[u] = ok[u] && !zbit(zm_, k + 1, kb);
            const size_t idx = (size_t)k * sxy + col;
            b[u] = ok[u] ? rho[idx] : 0.0;
            xm[u] = ok[u] && fxm ? v[idx - 1] : 0.0;
            xp[u] = ok[u] && fxp ? v[idx + 1] : 0.0;
            ym[u] = ok[u] && fym ? v[idx - nx] : 0.0;
            yp[u] = ok[u] && fyp ? v[idx + nx] : 0.0;
            zm[u] = fzm[u] ? v[idx - sxy] : 0.0;
            zp[u] = fzp[u] ? v[idx + sxy] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RF; ++u) {
            if (!ok[u]) continue;
            const int k = k0 + u;
            // only neighbours on a face (of this copy) keep their values
            double a = (fxm ? cxm * xm[u] : 0.0) + (fxp ? cxp * xp[u] : 0.0);
            a += (fym ? cym * ym[u] : 0.0) + (fyp ? cyp * yp[u] : 0.0);
            a += (fzm[u] ? L.ax[2].am[k] * zm[u] : 0.0) + (fzp[u] ? L.ax[2].ap[k] * zp[u] : 0.0);
            const double res = bscale * b[u] - a;
            if (r) r[sidx(L, i, j, k)] = (TO)res;
            acc += vxy * L.ax[2].m[k] * res * res;
        }
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[tl.t] = t;
}

hipError_t launch_residual_nat(const LevelView& L, const double* v, const double* rho, double bscale, double* r_split,
                               double* partials, int interior_zero, hipStream_t s)
{
    const PtShape ps = residual_shape(L);
    if (interior_zero)
        hipLaunchKernelGGL((k_residual_faces<double>), ps.grid, dim3(PT_NT), 0, s, L, ps.kp, v, rho, bscale,
                           r_split, partials);
    else
        hipLaunchKernelGGL((k_residual_march<double>), ps.grid, dim3(PT_NT), 0, s, L, ps.kp, v, rho, bscale,
                           r_split, partials);
    return hipGetLastError();
}

hipError_t launch_residual_nat32(const LevelView& L, const double* v, const double* rho, double bscale, float* r32,
                                 double* partials, hipStream_t s)
{
    const PtShape ps = residual_shape(L);
    hipLaunchKernelGGL((k_residual_march<float>), ps.grid, dim3(PT_NT), 0, s, L, ps.kp, v, rho, bscale, r32,
                       partials);
    return hipGetLastError();
}

// Au = A u, natural layout (the diagnostic lasto_apply)
__global__ __launch_bounds__(PT_NT) void k_apply_nat(LevelView L, int kp, const double* __restrict__ u,
                                                     double* __restrict__ Au)
{
    INTERIOR_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        const int nx = L.nx;
        const size_t sxy = (size_t)nx * L.ny;
        const size_t idx = (size_t)k * sxy + (size_t)j * nx + i;
        const double c = u[idx];
        double a = L.ax[0].am[i] * (u[idx - 1] - c) + L.ax[0].ap[i] * (u[idx + 1] - c);
        a += L.ax[1].am[j] * (u[idx - nx] - c) + L.ax[1].ap[j] * (u[idx + nx] - c);
        a += L.ax[2].am[k] * (u[idx - sxy] - c) + L.ax[2].ap[k] * (u[idx + sxy] - c);
        Au[idx] = a;
    }
}

hipError_t launch_apply_nat(const LevelView& L, const double* u, double* Au, hipStream_t s)
{
    PT_LAUNCH(k_apply_nat, L, s, u, Au);
    return hipGetLastError();
}

// Elementwise Krylov kernels walk the split storage row by row: a
// workgroup covers 64 entries x 4 rows of one colour over a chunk of planes.
// Entries off the interior (faces, padding) are zero in every vector these
// kernels touch and stay zero; their volume weight (parity table) is zero.
struct RowShape {
    dim3 grid;
    int kp;
};

static RowShape row_shape(const LevelView& L)
{
    RowShape r;
    const int gx = (L.W + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    const long tiles = 2L * gx * gy;
    r.kp = (int)std::min<long>(PT_KP_MAX, std::max<long>(1, (long)(L.nz - 2) * tiles / PT_BLOCKS));
    r.grid = dim3(gx, gy, 2 * ((L.nz - 2 + r.kp - 1) / r.kp));
    return r;
}

int row_blocks(const LevelView& L)
{
    const dim3 g = row_shape(L).grid;
    return (int)(g.x * g.y * g.z);
}

#define ROW_LOOP                                                          \
    const int m = blockIdx.x * PT_X + (threadIdx.x % PT_X);               \
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);           \
    const int c = blockIdx.z & 1;                                         \
    const bool inside = (m < L.W) && (j <= L.ny - 2);                     \
    const int kb_ = 1 + (blockIdx.z >> 1) * kp;                           \
    const int ke_ = min(kb_ + kp, L.nz - 1);                              \
    const unsigned long long zm_ = zint_mask(L, kb_);                     \
    for (int k = kb_; k < ke_; ++k)

#define ROW_AT ((size_t)c * L.cs + ((size_t)k * L.ny + j) * L.W + m)
#define ROW_VOL (L.xpar[(size_t)(((c + j + k) & 1) * 3 + 2) * L.W + m] * L.ax[1].m[j] * L.ax[2].m[k])

#define ROW_LAUNCH(kernel, L, s, ...)                                                        \
    do {                                                                                     \
        const RowShape rs_ = row_shape(L);                                                   \
        hipLaunchKernelGGL(kernel, rs_.grid, dim3(PT_NT), 0, s, L, rs_.kp, __VA_ARGS__);      \
    } while (0)

template <typename T>
__global__ __launch_bounds__(PT_NT) void k_dot(LevelView L, int kp, const T* __restrict__ a, const T* __restrict__ b,
                                               double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    ROW_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        const size_t at = ROW_AT;
        acc += ROW_VOL * (double)a[at] * (double)b[at];
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_dot(const LevelView& L, const T* a, const T* b, double* partials, hipStream_t s)
{
    ROW_LAUNCH(k_dot<T>, L, s, a, b, partials);
    return hipGetLastError();
}

// ---- Krylov updates over whole split arrays
// Each array is one flat run of 2 cs entries in rows of W (a multiple of 16),
// so a thread moves 16 bytes per access without leaving its row and keeps
// FL_U such accesses of every operand in flight before it stores any. Rows
// of interior (j, k) are updated whole, as every split kernel treats them;
// face rows and planes of other copies' faces are left alone. The norm
// partials use one fixed workgroup count per array size (deterministic).

constexpr int FL_NT = 256, FL_U = 4, FL_MAX_BLOCKS = 2048;

struct RowPos {
    int c, k, j, m;
    bool live;
};

// position of split entry q (32-bit: the grid limits 2 cs below 2^32)
__device__ __forceinline__ RowPos row_pos(const LevelView& L, unsigned q)
{
    RowPos p;
    const unsigned row = q / (unsigned)L.W;
    p.m = (int)(q - row * (unsigned)L.W);
    const unsigned ck = row / (unsigned)L.ny;
    p.j = (int)(row - ck * (unsigned)L.ny);
    p.c = ck >= (unsigned)L.nz ? 1 : 0;
    p.k = (int)ck - p.c * L.nz;
    p.live = p.j >= 1 && p.j <= L.ny - 2 && p.k >= 1 && p.k <= L.nz - 2 && L.zint[p.k];
    return p;
}

template <typename T>
static unsigned flat_vectors(const LevelView& L)
{
    return (unsigned)(2 * L.cs / Vec16<T>::N);
}

// Workgroups of a flat launch: as many passes (iters) per thread as the
// kernel's resident workgroups (cap) need to cover the array, then the
// fewest workgroups that cover it in that many passes, so every workgroup
// is resident from the start and all take the same number of passes.
static int flat_grid(unsigned nvec, int cap)
{
    const unsigned per = FL_NT * FL_U;
    const unsigned c = (unsigned)std::max(1, std::min(cap, FL_MAX_BLOCKS));
    const unsigned iters = std::max(1u, (nvec + c * per - 1) / (c * per));
    return (int)std::max(1u, std::min<unsigned>(c, (nvec + per * iters - 1) / (per * iters)));
}

template <typename KernelPtr>
static int kernel_cap(KernelPtr k)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 8;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 8;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, FL_NT, 0) != hipSuccess) return 8;
    return std::max(8, per_cu * cus);
}

// an upper bound of the partials of any flat launch
template <typename T>
int flat_blocks(const LevelView& L)
{
    (void)L;
    return FL_MAX_BLOCKS;
}

// pnew = z + beta pold, beta = scal[i_num]/scal[i_den] (0 on the first step)
template <typename T>
__global__ __launch_bounds__(FL_NT) void k_update_p(LevelView L, unsigned nvec, const T* __restrict__ z,
                                                    const T* __restrict__ pold, T* __restrict__ pnew,
                                                    const double* __restrict__ scal, int i_num, int i_den, int first)
{
    typedef typename Vec16<T>::V V;
    constexpr int N = Vec16<T>::N;
    const T beta = first ? T(0) : (T)(scal[i_num] / scal[i_den]);
    const unsigned stride = gridDim.x * FL_NT;
    for (unsigned e0 = blockIdx.x * FL_NT + threadIdx.x; e0 < nvec; e0 += stride * FL_U) {
        V zv[FL_U], pv[FL_U];
        bool lv[FL_U];
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            const unsigned e = e0 + u * stride;
            lv[u] = e < nvec && row_pos(L, e * N).live;
            zv[u] = V(T(0));
            pv[u] = V(T(0));
            if (lv[u]) {
                zv[u] = reinterpret_cast<const V*>(z)[e];
                if (!first) pv[u] = reinterpret_cast<const V*>(pold)[e];
            }
        }
#pragma unroll
        for (int u = 0; u < FL_U; ++u)
            if (lv[u]) reinterpret_cast<V*>(pnew)[e0 + u * stride] = first ? zv[u] : zv[u] + beta * pv[u];
    }
}

template <typename T>
hipError_t launch_update_p(const LevelView& L, const T* z, const T* pold, T* pnew, const double* scal, int i_num,
                           int i_den, int first, hipStream_t s)
{
    static const int cap = kernel_cap(k_update_p<T>);
    hipLaunchKernelGGL(k_update_p<T>, dim3(flat_grid(flat_vectors<T>(L), cap)), dim3(FL_NT), 0, s, L,
                       flat_vectors<T>(L), z, pold, pnew, scal, i_num, i_den, first);
    return hipGetLastError();
}

// The inner FP32 PCG defers x += alpha p by one step into the next p update,
// which reads the old p anyway (8 array passes a step instead of 9):
// pnew = z + beta pold, beta = scal[i_num]/scal[i_den], and with XM 1
// x = alpha pold, with XM 2 x += alpha pold, alpha = scal[i_anum]/scal[i_aden]
// (the previous step's); a non-finite alpha leaves x untouched.
template <typename T, int XM>
__global__ __launch_bounds__(FL_NT) void k_update_px(LevelView L, unsigned nvec, const T* __restrict__ z,
                                                     const T* __restrict__ pold, T* __restrict__ pnew,
                                                     T* __restrict__ x, const double* __restrict__ scal, int i_num,
                                                     int i_den, int i_anum, int i_aden)
{
    typedef typename Vec16<T>::V V;
    constexpr int N = Vec16<T>::N;
    const T beta = (T)(scal[i_num] / scal[i_den]);
    const double ad = scal[i_anum] / scal[i_aden];
    const bool ok = isfinite(ad);
    const T alpha = (T)ad;
    const unsigned stride = gridDim.x * FL_NT;
    for (unsigned e0 = blockIdx.x * FL_NT + threadIdx.x; e0 < nvec; e0 += stride * FL_U) {
        V zv[FL_U], pv[FL_U], xv[FL_U];
        bool lv[FL_U];
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            const unsigned e = e0 + u * stride;
            lv[u] = e < nvec && row_pos(L, e * N).live;
            zv[u] = pv[u] = xv[u] = V(T(0));
            if (lv[u]) {
                zv[u] = reinterpret_cast<const V*>(z)[e];
                pv[u] = reinterpret_cast<const V*>(pold)[e];
                if (XM == 2 && ok) xv[u] = reinterpret_cast<const V*>(x)[e];
            }
        }
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            if (!lv[u]) continue;
            const unsigned e = e0 + u * stride;
            reinterpret_cast<V*>(pnew)[e] = zv[u] + beta * pv[u];
            if (ok) reinterpret_cast<V*>(x)[e] = xv[u] + alpha * pv[u];
            else if (XM == 1) reinterpret_cast<V*>(x)[e] = V(T(0));
        }
    }
}

template <typename T>
hipError_t launch_update_px(const LevelView& L, const T* z, const T* pold, T* pnew, T* x, const double* scal,
                            int i_num, int i_den, int i_anum, int i_aden, int accumulate, hipStream_t s)
{
    if (accumulate) {
        static const int cap = kernel_cap(k_update_px<T, 2>);
        hipLaunchKernelGGL((k_update_px<T, 2>), dim3(flat_grid(flat_vectors<T>(L), cap)), dim3(FL_NT), 0, s, L,
                           flat_vectors<T>(L), z, pold, pnew, x, scal, i_num, i_den, i_anum, i_aden);
    } else {
        static const int cap = kernel_cap(k_update_px<T, 1>);
        hipLaunchKernelGGL((k_update_px<T, 1>), dim3(flat_grid(flat_vectors<T>(L), cap)), dim3(FL_NT), 0, s, L,
                           flat_vectors<T>(L), z, pold, pnew, x, scal, i_num, i_den, i_anum, i_aden);
    }
    return hipGetLastError();
}

// r -= alpha q (split), alpha = scal[i_num]/scal[i_den]; a non-finite alpha
// leaves r untouched
template <typename T>
__global__ __launch_bounds__(FL_NT) void k_update_r(LevelView L, unsigned nvec, T* __restrict__ r,
                                                    const T* __restrict__ q, const double* __restrict__ scal,
                                                    int i_num, int i_den)
{
    typedef typename Vec16<T>::V V;
    constexpr int N = Vec16<T>::N;
    const double ad = scal[i_num] / scal[i_den];
    if (!isfinite(ad)) return;
    const T alpha = (T)ad;
    const unsigned stride = gridDim.x * FL_NT;
    for (unsigned e0 = blockIdx.x * FL_NT + threadIdx.x; e0 < nvec; e0 += stride * FL_U) {
        V rv[FL_U], qv[FL_U];
        bool lv[FL_U];
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            const unsigned e = e0 + u * stride;
            lv[u] = e < nvec && row_pos(L, e * N).live;
            rv[u] = qv[u] = V(T(0));
            if (lv[u]) {
                rv[u] = reinterpret_cast<const V*>(r)[e];
                qv[u] = reinterpret_cast<const V*>(q)[e];
            }
        }
#pragma unroll
        for (int u = 0; u < FL_U; ++u)
            if (lv[u]) reinterpret_cast<V*>(r)[e0 + u * stride] = rv[u] - alpha * qv[u];
    }
}

template <typename T>
hipError_t launch_update_r(const LevelView& L, T* r, const T* q, const double* scal, int i_num, int i_den,
                           hipStream_t s)
{
    static const int cap = kernel_cap(k_update_r<T>);
    hipLaunchKernelGGL(k_update_r<T>, dim3(flat_grid(flat_vectors<T>(L), cap)), dim3(FL_NT), 0, s, L,
                       flat_vectors<T>(L), r, q, scal, i_num, i_den);
    return hipGetLastError();
}

// x += alpha p (x = alpha p on the first step), r -= alpha q (all split),
// alpha = scal[i_num]/scal[i_den]; with NORM, partials of <r,r>_W. A non-finite alpha leaves
// x and r untouched (the caller then reports the breakdown with x still the
// last finite iterate).
template <typename T, bool NORM>
__global__ __launch_bounds__(FL_NT) void k_update_xr(LevelView L, unsigned nvec, T* __restrict__ x,
                                                     T* __restrict__ r, const T* __restrict__ p,
                                                     const T* __restrict__ q, const double* __restrict__ scal,
                                                     int i_num, int i_den, double* __restrict__ part, int first)
{
    typedef typename Vec16<T>::V V;
    constexpr int N = Vec16<T>::N;
    __shared__ double red[FL_NT / 64];
    const double ad = scal[i_num] / scal[i_den];
    const bool ok = isfinite(ad);
    const T alpha = (T)ad;
    double acc = 0.0;
    const unsigned stride = gridDim.x * FL_NT;
    for (unsigned e0 = blockIdx.x * FL_NT + threadIdx.x; e0 < nvec; e0 += stride * FL_U) {
        V xv[FL_U], rv[FL_U], pv[FL_U], qv[FL_U];
        RowPos ps[FL_U];
        bool lv[FL_U];
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            const unsigned e = e0 + u * stride;
            ps[u] = row_pos(L, e * N);
            lv[u] = e < nvec && ps[u].live;
            xv[u] = rv[u] = pv[u] = qv[u] = V(T(0));
            if (lv[u]) {
                rv[u] = reinterpret_cast<const V*>(r)[e];
                if (ok) {
                    if (!first) xv[u] = reinterpret_cast<const V*>(x)[e];
                    pv[u] = reinterpret_cast<const V*>(p)[e];
                    qv[u] = reinterpret_cast<const V*>(q)[e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            if (!lv[u]) continue;
            const unsigned e = e0 + u * stride;
            if (ok) {
                xv[u] = xv[u] + alpha * pv[u];
                rv[u] = rv[u] - alpha * qv[u];
                reinterpret_cast<V*>(x)[e] = xv[u];
                reinterpret_cast<V*>(r)[e] = rv[u];
            } else if (first) {
                reinterpret_cast<V*>(x)[e] = V(T(0));   // the iterate is still e = 0
            }
            if (!NORM) continue;
            // dual volume: x width by parity of i (zero off the interior), y, z widths
            const double* wx = L.xpar + (size_t)(((ps[u].c + ps[u].j + ps[u].k) & 1) * 3 + 2) * L.W + ps[u].m;
            const double wyz = L.ax[1].m[ps[u].j] * L.ax[2].m[ps[u].k];
            double a = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) a += wx[l] * ((double)rv[u][l] * (double)rv[u][l]);
            acc += wyz * a;
        }
    }
    if (!NORM) return;
    const double t = block_sum<FL_NT>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = ok ? t : __builtin_nan("");
}

template <typename T>
hipError_t launch_update_xr(const LevelView& L, T* x, T* r, const T* p, const T* q, const double* scal, int i_num,
                            int i_den, double* partials, hipStream_t s, int* nparts, int first)
{
    if (partials) {
        static const int cap = kernel_cap(k_update_xr<T, true>);
        const int nb = flat_grid(flat_vectors<T>(L), cap);
        hipLaunchKernelGGL((k_update_xr<T, true>), dim3(nb), dim3(FL_NT), 0, s, L, flat_vectors<T>(L), x, r, p, q,
                           scal, i_num, i_den, partials, first);
        if (nparts) *nparts = nb;
    } else {
        static const int cap = kernel_cap(k_update_xr<T, false>);
        const int nb = flat_grid(flat_vectors<T>(L), cap);
        hipLaunchKernelGGL((k_update_xr<T, false>), dim3(nb), dim3(FL_NT), 0, s, L, flat_vectors<T>(L), x, r, p, q,
                           scal, i_num, i_den, partials, first);
        if (nparts) *nparts = 0;
    }
    return hipGetLastError();
}

// v (natural) += e (split), interior
__global__ __launch_bounds__(PT_NT) void k_add_nat(LevelView L, int kp, double* __restrict__ v,
                                                   const double* __restrict__ e)
{
    INTERIOR_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        v[((size_t)k * L.ny + j) * L.nx + i] += e[sidx(L, i, j, k)];
    }
}

hipError_t launch_add_nat(const LevelView& L, double* v, const double* e_split, hipStream_t s)
{
    PT_LAUNCH(k_add_nat, L, s, v, e_split);
    return hipGetLastError();
}

// v (natural) += s * y (FP32, natural), interior
__global__ __launch_bounds__(PT_NT) void k_add_f32_nat(LevelView L, int kp, double* __restrict__ v,
                                                       const float* __restrict__ y, double s)
{
    INTERIOR_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        const size_t at = ((size_t)k * L.ny + j) * L.nx + i;
        v[at] += s * (double)y[at];
    }
}

hipError_t launch_add_f32_nat(const LevelView& L, double* v, const float* y, double s, hipStream_t st)
{
    PT_LAUNCH(k_add_f32_nat, L, st, v, y, s);
    return hipGetLastError();
}

// v (natural) += e (FP32, split) and, with p given, + alpha p, alpha =
// scal[i_num]/scal[i_den] (the last step of an inner PCG folded into v; a
// non-finite alpha adds e alone), interior. A thread takes AD planes of its
// column at a time: their loads are issued together, then the updates.
template <bool FLAG>
__global__ __launch_bounds__(PT_NT) void k_add32_nat(LevelView L, int kp, double* __restrict__ v,
                                                     const float* __restrict__ e, const float* __restrict__ p,
                                                     double* __restrict__ scal, int i_num, int i_den)
{
    constexpr int AD = 4;
    float alpha = 0.0f;
    if (p) {
        const double ad = scal[i_num] / scal[i_den];
        alpha = isfinite(ad) ? (float)ad : 0.0f;
    }
    const PtTile tl = pt_tile(L, kp);
    if (!tl.ok) return;
    const int i = 1 + tl.bx * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + tl.by * PT_Y + (threadIdx.x / PT_X);
    const int kb = 1 + tl.bz * kp, ke = min(kb + kp, L.nz - 1);
    const unsigned long long zm_ = zint_mask(L, kb);
    if (i > L.nx - 2 || j > L.ny - 2) return;   // (no barrier follows)
    for (int k0 = kb; k0 < ke; k0 += AD) {
        double vv[AD];
        float d[AD];
        bool ok[AD];
#pragma unroll
        for (int u = 0; u < AD; ++u) {
            const int k = k0 + u;
            ok[u] = k < ke && zbit(zm_, k, kb);
            vv[u] = 0.0;
            d[u] = 0.0f;
            if (ok[u]) {
                const size_t at = sidx(L, i, j, k);
                vv[u] = v[((size_t)k * L.ny + j) * L.nx + i];
                d[u] = p ? e[at] + alpha * p[at] : e[at];
            }
        }
#pragma unroll
        for (int u = 0; u < AD; ++u) {
            if (!ok[u]) continue;
            double& dst = v[((size_t)(k0 + u) * L.ny + j) * L.nx + i];
            if (FLAG) {
                // a broken-down FP32 correction never reaches v: the node keeps
                // its value and the solve is told (every writer stores the same 1)
                const double nv = vv[u] + (double)d[u];
                if (isfinite(nv)) dst = nv;
                else scal[S_BAD] = 1.0;
            } else {
                dst = vv[u] + (double)d[u];
            }
        }
    }
}

hipError_t launch_add32_nat(const LevelView& L, double* v, const float* e32, const float* p32, double* scal,
                            int i_num, int i_den, hipStream_t s, bool flag_bad)
{
    if (flag_bad) PT_LAUNCH(k_add32_nat<true>, L, s, v, e32, p32, scal, i_num, i_den);
    else PT_LAUNCH(k_add32_nat<false>, L, s, v, e32, p32, scal, i_num, i_den);
    return hipGetLastError();
}

// layout conversions
__global__ __launch_bounds__(PT_NT) void k_nat_to_split(LevelView L, const double* __restrict__ a,
                                                        double* __restrict__ out)
{
    const int i = blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = blockIdx.z;
    if (i >= L.nx || j >= L.ny) return;
    out[sidx(L, i, j, k)] = a[((size_t)k * L.ny + j) * L.nx + i];
}

__global__ __launch_bounds__(PT_NT) void k_split_to_nat(LevelView L, int kp, const double* __restrict__ in,
                                                        double* __restrict__ a)
{
    INTERIOR_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        a[((size_t)k * L.ny + j) * L.nx + i] = in[sidx(L, i, j, k)];
    }
}

hipError_t launch_nat_to_split(const LevelView& L, const double* a, double* s_out, hipStream_t s)
{
    // every node, faces included
    const dim3 g((L.nx + PT_X - 1) / PT_X, (L.ny + PT_Y - 1) / PT_Y, L.nz);
    hipLaunchKernelGGL(k_nat_to_split, g, dim3(PT_NT), 0, s, L, a, s_out);
    return hipGetLastError();
}

hipError_t launch_split_to_nat(const LevelView& L, const double* s_in, double* a, hipStream_t s)
{
    PT_LAUNCH(k_split_to_nat, L, s, s_in, a);
    return hipGetLastError();
}

// fill a whole array (n elements) with zeros (a kernel, never a memset)
template <typename T>
__global__ void k_fill_zero(T* __restrict__ a, size_t n)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) a[t] = T(0);
}

template <typename T>
hipError_t launch_fill_zero(T* a, size_t n, hipStream_t s)
{
    int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(blocks), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

template <typename T>
__global__ void k_inject_nan(T* r, size_t idx)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) r[idx] = (T)__builtin_nan("");
}

hipError_t launch_inject_nan(double* r, size_t idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_inject_nan<double>, dim3(1), dim3(64), 0, s, r, idx);
    return hipGetLastError();
}

hipError_t launch_inject_nan(float* r, size_t idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_inject_nan<float>, dim3(1), dim3(64), 0, s, r, idx);
    return hipGetLastError();
}

// ---------------------------------------------------------- transfers
// Both transfers tile their level like the half-sweeps: a workgroup covers
// 64 x 4 (x, y) columns, and tiles go to the XCDs in contiguous runs
// (xcd_tile), so fine rows shared by neighbouring tiles are mostly read from
// one L2. A thread marches a chunk of planes (sized like the residual's), and
// since both operators are products of per-axis weights, each plane's x-y sum
// is formed once and reused by the neighbouring planes of the other level.

struct TileShape {
    int nbx, nby, nb, per;
};

// two consecutive elements, aligned to one (a pair starting at any entry)
template <typename T> struct Pair;
template <> struct Pair<float> {
    typedef float P __attribute__((ext_vector_type(2), aligned(4)));
};
template <> struct Pair<double> {
    typedef double P __attribute__((ext_vector_type(2), aligned(8)));
};

static TileShape tile_shape(int cols_x, int rows_y, int planes, int ku)
{
    TileShape t;
    t.nbx = (cols_x + PT_X - 1) / PT_X;
    t.nby = (rows_y + PT_Y - 1) / PT_Y;
    t.nb = t.nbx * t.nby * ((planes + ku - 1) / ku);
    t.per = (t.nb + 7) / 8;
    return t;
}

// f_coarse = R r on the interior of the coarse level, r vanishing on black
// fine nodes. One coarse (I, J) column per thread, marching a chunk of kc
// coarse planes: R is a product of per-axis weights, so the x-y sum of fine
// plane kk at the column is formed once (three two-entry loads) and kept
// while the coarse planes that use it pass (a coarse step spans one or two
// fine steps, so each coarse plane adds one or two fine planes). The sums are
// taken in the order of the per-plane form (y inside z), so the result does
// not depend on the chunking.
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_restrict_red(LevelView F, LevelView C, const T* __restrict__ r,
                                                        T* __restrict__ rc, int nbx, int nby, int nb, int per, int kc)
{
    const int t = xcd_tile(blockIdx.x, per);
    const int I = 1 + (t % nbx) * PT_X + (threadIdx.x & (PT_X - 1));
    const int J = 1 + ((t / nbx) % nby) * PT_Y + (threadIdx.x >> 6);
    if (t >= nb || J > C.ny - 2) return;
    const bool inside = I <= C.nx - 2;
    const int K0 = 1 + (t / (nbx * nby)) * kc;
    const int K1 = min(K0 + kc, C.nz - 1);
    const RTaps<T> x = restrict_taps<T>(C, inside ? I : C.nx - 2);
    const int fj = C.ax[1].rf[J];
    const T wy0 = (T)C.ax[1].rw[3 * J], wy1 = (T)C.ax[1].rw[3 * J + 1], wy2 = (T)C.ax[1].rw[3 * J + 2];
    // the x-y sum of fine plane kk: two consecutive red entries of each of
    // the three fine rows, as one load (aligned to one element only)
    auto pxy = [&](int kk) -> T {
        T g0[3], g1[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T* row = r + ((size_t)kk * F.ny + (fj - 1 + b)) * F.W + x.m0;
            const typename Pair<T>::P q = *(const typename Pair<T>::P*)row;
            g0[b] = q.x;
            g1[b] = q.y;
        }
        T plane = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const bool same = ((fj - 1 + b + kk) & 1) == x.e;
            const T wy = b == 0 ? wy0 : (b == 1 ? wy1 : wy2);
            plane += wy * ((same ? x.s0 : x.d0) * g0[b] + (same ? x.s1 : x.d1) * g1[b]);
        }
        return plane;
    };
    // sums of fine planes fk - 1, fk, fk + 1 of the previous coarse plane
    int fprev = -8;
    T w0 = T(0), w1 = T(0), w2 = T(0);
    for (int K = K0; K < K1; ++K) {
        const int fk = C.ax[2].rf[K];
        if (fk == fprev + 1) {
            w0 = w1;
            w1 = w2;
            w2 = pxy(fk + 1);
        } else if (fk == fprev + 2) {
            const T a = pxy(fk), b = pxy(fk + 1);
            w0 = w2;
            w1 = a;
            w2 = b;
        } else {
            const T a = pxy(fk - 1), b = pxy(fk), c = pxy(fk + 1);
            w0 = a;
            w1 = b;
            w2 = c;
        }
        fprev = fk;
        T acc = T(0);
        acc += (T)C.ax[2].rw[3 * K] * w0;
        acc += (T)C.ax[2].rw[3 * K + 1] * w1;
        acc += (T)C.ax[2].rw[3 * K + 2] * w2;
        if (inside && C.zint[K]) rc[sidx(C, I, J, K)] = acc;
    }
}

template <typename T>
hipError_t launch_restrict_red(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s)
{
    const int gx = (C.nx - 2 + PT_X - 1) / PT_X, gy = (C.ny - 2 + PT_Y - 1) / PT_Y;
    const int kc = chunk_planes((long)gx * gy, C.nz - 2, resident_256(), PT_KP_MAX);
    const TileShape ts = tile_shape(C.nx - 2, C.ny - 2, C.nz - 2, kc);
    hipLaunchKernelGGL(k_restrict_red<T>, dim3(8 * ts.per), dim3(PT_NT), 0, s, F, C, r, rc, ts.nbx, ts.nby, ts.nb,
                       ts.per, kc);
    return hipGetLastError();
}

// u + P e on the red nodes only: when a black half-sweep follows, it
// overwrites every black value, so correcting them would be wasted work. Two
// consecutive red entries m, m+1 of a row per thread (fine nodes i0 = o + 2m
// and i1 = i0 + 2, o = (j + k) & 1), marching a chunk of kc fine planes.
// Their coarse nodes lie in Ix0 .. Ix0 + 3 (Ix0 = pc(i0); a coarse step spans
// at most two fine steps), which in each coarse row are two consecutive
// entries of each colour: two pair loads per row serve both fine nodes. P is
// a product of per-axis weights, so the x-y sums of a coarse plane (for both
// row parities and both nodes) are formed once and kept while the fine
// planes between it and the next pass (one or two of them); the sums are
// taken in the order of the per-plane form (y inside z). The result goes to
// uout, which is uin (in place) or another array (its red entries written,
// the rest untouched); each thread reads its own entries before it writes
// them.
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_prolong_red(LevelView F, LevelView C, const T* __restrict__ e,
                                                       const T* uin, T* uout, int nbx, int nby, int nb, int per, int kc)
{
    typedef typename Pair<T>::P P2;
    const int t = xcd_tile(blockIdx.x, per);
    const int m = 2 * ((t % nbx) * PT_X + (threadIdx.x & (PT_X - 1)));
    const int j = 1 + ((t / nbx) % nby) * PT_Y + (threadIdx.x >> 6);
    if (t >= nb || j > F.ny - 2 || m > (F.nx - 2) / 2) return;
    const int mlast = (F.nx - 2) / 2;
    // taps of both nodes for both row parities (o = 0: i = 2m, 2m + 2; o = 1: 2m + 1, 2m + 3)
    PTaps<T> xa[2], xb[2];
    bool oka[2], okb[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const int i0 = o + 2 * m, i1 = i0 + 2;
        oka[o] = i0 >= 1 && i0 <= F.nx - 2;
        okb[o] = m + 1 <= mlast && i1 <= F.nx - 2;
        xa[o] = prolong_taps<T>(C.ax[0], min(max(i0, 1), F.nx - 2));
        xb[o] = prolong_taps<T>(C.ax[0], min(max(i1, 1), F.nx - 2));
    }
    const PTaps<T> y = prolong_taps<T>(C.ax[1], j);
    const int k0 = 1 + (t / (nbx * nby)) * kc;
    const int k1 = min(k0 + kc, F.nz - 1);
    const size_t plane = (size_t)F.ny * F.W;
    const size_t row = (size_t)j * F.W + m;
    // the x-y sums of coarse plane Kc: sv[o][0] for node i0, sv[o][1] for i1
    auto sums = [&](int Kc, T (&sv)[2][2]) {
        T cv[2][2][4];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const int I0 = xa[o].I;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int Jb = y.I + b;
                const size_t crow = ((size_t)Kc * C.ny + Jb) * C.W;
                const int c0 = (I0 + Jb + Kc) & 1;   // colour of I0 (and I0 + 2); I0 + 1, I0 + 3 have the other
                const P2 p0 = *(const P2*)(e + (size_t)c0 * C.cs + crow + (I0 >> 1));
                const P2 p1 = *(const P2*)(e + (size_t)(c0 ^ 1) * C.cs + crow + ((I0 + 1) >> 1));
                cv[o][b][0] = p0.x;
                cv[o][b][1] = p1.x;
                cv[o][b][2] = p0.y;
                cv[o][b][3] = p1.y;
            }
        }
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const PTaps<T>& A = xa[o];
            const PTaps<T>& B = xb[o];
            const int d = B.I - A.I;   // 0, 1 or 2
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const T* v = cv[o][b];
                const T wyb = b ? y.w1 : y.w0;
                s0 += wyb * (A.w0 * v[0] + A.w1 * v[1]);
                const T b0 = d == 0 ? v[0] : (d == 1 ? v[1] : v[2]);
                const T b1 = d == 0 ? v[1] : (d == 1 ? v[2] : v[3]);
                s1 += wyb * (B.w0 * b0 + B.w1 * b1);
            }
            sv[o][0] = s0;
            sv[o][1] = s1;
        }
    };
    // sums of coarse planes kcur and kcur + 1 (the cell of the previous plane)
    T sa[2][2], sb[2][2];
    int kcur = -8;
    for (int k = k0; k < k1; ++k) {
        const PTaps<T> z = prolong_taps<T>(C.ax[2], k);
        const P2 uo = *(const P2*)(uin + (size_t)k * plane + row);
        if (z.I == kcur + 1) {
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                sa[o][0] = sb[o][0];
                sa[o][1] = sb[o][1];
            }
            sums(z.I + 1, sb);
        } else if (z.I != kcur) {
            sums(z.I, sa);
            sums(z.I + 1, sb);
        }
        kcur = z.I;
        if (!F.zint[k]) continue;
        const int o = (j + k) & 1;
        T acc0 = T(0), acc1 = T(0);
        acc0 += z.w0 * sa[o][0];
        acc1 += z.w0 * sa[o][1];
        acc0 += z.w1 * sb[o][0];
        acc1 += z.w1 * sb[o][1];
        const bool s_a = o ? oka[1] : oka[0], s_b = o ? okb[1] : okb[0];
        T* out = uout + (size_t)k * plane + row;
        if (s_a && s_b) {
            P2 w;
            w.x = uo.x + acc0;
            w.y = uo.y + acc1;
            *(P2*)out = w;
        } else {
            if (s_a) out[0] = uo.x + acc0;
            if (s_b) out[1] = uo.y + acc1;
        }
    }
}

template <typename T>
hipError_t launch_prolong_red(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s)
{
    return launch_prolong_red_to<T>(F, C, e, u, u, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_red_to(const LevelView& F, const LevelView& C, const T* e, const T* uin, T* out,
                                 hipStream_t s)
{
    // pairs of red entries m = 0, 2, ... <= (nx - 2) / 2
    const int cols = ((F.nx - 2) / 2) / 2 + 1;
    const int gx = (cols + PT_X - 1) / PT_X, gy = (F.ny - 2 + PT_Y - 1) / PT_Y;
    const int kc = chunk_planes((long)gx * gy, F.nz - 2, resident_256(), PT_KP_MAX);
    const TileShape ts = tile_shape(cols, F.ny - 2, F.nz - 2, kc);
    hipLaunchKernelGGL(k_prolong_red<T>, dim3(8 * ts.per), dim3(PT_NT), 0, s, F, C, e, uin, out, ts.nbx, ts.nby,
                       ts.nb, ts.per, kc);
    return hipGetLastError();
}

// u += P e on every interior node (a V-cycle without post-smoothing)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_prolong_add(LevelView F, int kp, LevelView C, const T* __restrict__ e,
                                                       T* __restrict__ u)
{
    const LevelView& L = F;
    INTERIOR_LOOP
    {
        if (!inside || !ZINT(k)) continue;
        u[sidx(F, i, j, k)] += prolong_at<T>(C, e, prolong_taps<T>(C.ax[0], i), j, k);
    }
}

template <typename T>
hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s)
{
    PT_LAUNCH(k_prolong_add<T>, F, s, C, e, u);
    return hipGetLastError();
}

// -------------------------------------------------------------- tail
// The V-cycle below a small level in ONE workgroup: every step is a loop of
// the workgroup's threads over the level's nodes followed by a barrier. On
// levels of a few thousand nodes a launch costs more than the work, so this
// replaces about a dozen launches per level by one.
//
// Threads are assigned to (x, y) columns once per step (ncols columns, ng
// threads per column taking every ng-th plane), so no node needs an integer
// division to find its indices; a thread computes TL_BATCH planes before
// storing any of them, so their loads are in flight together.
constexpr int TL_NT = 1024, TL_BATCH = 4;

struct Cols {
    int ncols, ng, col, grp;
    bool active;
};

__device__ __forceinline__ Cols tail_cols(int ncols)
{
    Cols c;
    c.ncols = ncols;
    c.ng = max(1, TL_NT / max(ncols, 1));
    c.active = (int)threadIdx.x < ncols * c.ng;
    c.col = (int)threadIdx.x % max(ncols, 1);
    c.grp = (int)threadIdx.x / max(ncols, 1);
    return c;
}

// half-sweep of colour c (RESID: residual of colour c into r instead)
template <typename T, bool RESID>
__device__ void t_half(const LevelView& V, T* __restrict__ u, const T* __restrict__ f, T* __restrict__ r, int c,
                       int zero_in)
{
    const int mcount = (V.nx - 2) / 2 + 1;
    const Cols cl = tail_cols(mcount * (V.ny - 2));
    if (!cl.active) return;
    const int m = cl.col % mcount, j = 1 + cl.col / mcount;
    for (int kb = 1 + cl.grp; kb <= V.nz - 2; kb += cl.ng * TL_BATCH) {
        T val[TL_BATCH];
        size_t at[TL_BATCH];
        bool ok[TL_BATCH];
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int k = kb + b * cl.ng;
            const int i = ((c + j + k) & 1) + 2 * m;
            ok[b] = k <= V.nz - 2 && i >= 1 && i <= V.nx - 2 && V.zint[k];
            at[b] = 0;
            val[b] = T(0);
            if (!ok[b]) continue;
            at[b] = sidx(V, i, j, k);
            if (RESID) {
                val[b] = f[at[b]] - apply_split(V, (const T*)u, i, j, k, u[at[b]]);
            } else if (zero_in) {
                const T d = (T)(V.ax[0].am[i] + V.ax[0].ap[i] + V.ax[1].am[j] + V.ax[1].ap[j] + V.ax[2].am[k] +
                                V.ax[2].ap[k]);
                val[b] = -f[at[b]] / d;
            } else {
                val[b] = gs_point(V, (const T*)u, i, j, k, f[at[b]]);
            }
        }
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b)
            if (ok[b]) (RESID ? r : u)[at[b]] = val[b];
    }
}

template <typename T>
__device__ void t_restrict_red(const LevelView& F, const LevelView& C, const T* __restrict__ r, T* __restrict__ fc)
{
    const Cols cl = tail_cols((C.nx - 2) * (C.ny - 2));
    if (!cl.active) return;
    const int I = 1 + cl.col % (C.nx - 2), J = 1 + cl.col / (C.nx - 2);
    const RTaps<T> x = restrict_taps<T>(C, I);
    for (int kb = 1 + cl.grp; kb <= C.nz - 2; kb += cl.ng * TL_BATCH) {
        T val[TL_BATCH];
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int K = kb + b * cl.ng;
            val[b] = K <= C.nz - 2 && C.zint[K] ? restrict_red_at<T>(F, C, r, x, J, K) : T(0);
        }
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int K = kb + b * cl.ng;
            if (K <= C.nz - 2 && C.zint[K]) fc[sidx(C, I, J, K)] = val[b];
        }
    }
}

template <typename T>
__device__ void t_prolong(const LevelView& F, const LevelView& C, const T* __restrict__ e, T* __restrict__ u,
                          bool red_only)
{
    const Cols cl = tail_cols((F.nx - 2) * (F.ny - 2));
    if (!cl.active) return;
    const int i = 1 + cl.col % (F.nx - 2), j = 1 + cl.col / (F.nx - 2);
    const PTaps<T> x = prolong_taps<T>(C.ax[0], i);
    for (int kb = 1 + cl.grp; kb <= F.nz - 2; kb += cl.ng * TL_BATCH) {
        T val[TL_BATCH];
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int k = kb + b * cl.ng;
            const bool ok = k <= F.nz - 2 && F.zint[k] && !(red_only && ((i + j + k) & 1));
            val[b] = ok ? prolong_at<T>(C, e, x, j, k) : T(0);
        }
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int k = kb + b * cl.ng;
            if (k <= F.nz - 2 && F.zint[k] && !(red_only && ((i + j + k) & 1))) u[sidx(F, i, j, k)] += val[b];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(TL_NT) void k_tail(const TailLevel* __restrict__ lv, int nl, int nu1, int nu2,
                                                int csweeps, int top_zero)
{
    // descent
    for (int l = 0; l + 1 < nl; ++l) {
        const LevelView& V = lv[l].V;
        T* u = TailBuf<T>::u(lv[l]);
        const T* f = TailBuf<T>::f(lv[l]);
        T* r = TailBuf<T>::r(lv[l]);
        for (int s = 0; s < nu1; ++s) {
            t_half<T, false>(V, u, f, r, 0, s == 0 && (l > 0 || top_zero));
            __syncthreads();
            t_half<T, false>(V, u, f, r, 1, 0);
            __syncthreads();
        }
        // residual on red nodes only (the black half-sweep just zeroed it on black)
        t_half<T, true>(V, u, f, r, 0, 0);
        __syncthreads();
        t_restrict_red<T>(V, lv[l + 1].V, r, TailBuf<T>::f(lv[l + 1]));
        __syncthreads();
    }
    // coarsest: csweeps sweeps (red, black), then csweeps (black, red), from zero
    {
        const LevelView& V = lv[nl - 1].V;
        T* u = TailBuf<T>::u(lv[nl - 1]);
        const T* f = TailBuf<T>::f(lv[nl - 1]);
        for (int pass = 0; pass < 2 * csweeps; ++pass) {
            for (int h = 0; h < 2; ++h) {
                const int colour = (pass < csweeps) ? h : 1 - h;
                t_half<T, false>(V, u, f, (T*)nullptr, colour, pass == 0 && h == 0);
                __syncthreads();
            }
        }
    }
    // ascent
    for (int l = nl - 2; l >= 0; --l) {
        const LevelView& V = lv[l].V;
        T* u = TailBuf<T>::u(lv[l]);
        const T* f = TailBuf<T>::f(lv[l]);
        // correction on red nodes only when a black half-sweep follows
        t_prolong<T>(V, lv[l + 1].V, TailBuf<T>::u(lv[l + 1]), u, nu2 > 0);
        __syncthreads();
        for (int s = 0; s < nu2; ++s) {
            t_half<T, false>(V, u, f, (T*)nullptr, 1, 0);
            __syncthreads();
            t_half<T, false>(V, u, f, (T*)nullptr, 0, 0);
            __syncthreads();
        }
    }
}

template <typename T>
hipError_t launch_tail(const TailLevel* lv, int nl, int nu1, int nu2, int csweeps, int top_zero, hipStream_t s)
{
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(TL_NT), 0, s, lv, nl, nu1, nu2, csweeps, top_zero);
    return hipGetLastError();
}

// ------------------------------------------------------ LDS tail (FP32)
// The same cycle with every level's correction, right-hand side and FP32
// coefficient tables held in one workgroup's LDS. On one compute unit the
// cycle is bound by instruction issue, not by memory, so each step is a flat
// loop over its items with 32-bit LDS offsets, table lookups instead of
// per-node coefficient conversions, and index division by a float
// reciprocal (exact after one correction for the small counts here). The
// fine residual is formed where the restriction reads it instead of being
// stored. Only the top level's right-hand side (and its correction when the
// cycle continues from one) comes in from global memory, and only its
// correction goes back.

// q = a / d, r = a - q d for 0 <= a < 2^24 with inv = 1/d rounded: the float
// quotient is off by at most one, which the two corrections remove
__device__ __forceinline__ int lh_divmod(int a, int d, float inv, int& r)
{
    int q = (int)((float)a * inv);
    r = a - q * d;
    if (r >= d) {
        ++q;
        r -= d;
    }
    if (r < 0) {
        --q;
        r += d;
    }
    return q;
}

struct LhLevel {
    int nx, ny, nz, W, cs, P;   // P = ny W, one plane of one colour
    LdsTab t;
};

__device__ __forceinline__ LhLevel lh_level(float* lds, const LdsPlan* __restrict__ P, int q)
{
    LhLevel L;
    L.nx = P->dims[q][0];
    L.ny = P->dims[q][1];
    L.nz = P->dims[q][2];
    L.W = P->dims[q][3];
    L.cs = P->dims[q][4];
    L.P = L.ny * L.W;
    const int f = q > 0 ? q - 1 : q;
    L.t = lds_tab(lds + P->off[q][2], L.nx, L.ny, L.nz, P->dims[f][0], P->dims[f][1], P->dims[f][2], q > 0);
    return L;
}

// half-sweep of colour c (zero_in: the other colour is read as zero)
__device__ __forceinline__ void lh_half(const LhLevel& L, float* u, const float* f, int c, bool zero_in)
{
    const int mc = (L.nx - 2) / 2 + 1, ry = L.ny - 2;
    const int total = mc * ry * (L.nz - 2);
    const float im = 1.0f / (float)mc, iy = 1.0f / (float)ry;
    float* uc = u + c * L.cs;
    const float* uo = u + (1 - c) * L.cs;
    const float* fc = f + c * L.cs;
    for (int t = threadIdx.x; t < total; t += TL_NT) {
        int m, jj;
        const int row = lh_divmod(t, mc, im, m);
        const int k = 1 + lh_divmod(row, ry, iy, jj);
        const int j = 1 + jj;
        const int o = (c + j + k) & 1, i = o + 2 * m;
        if (i < 1 || i > L.nx - 2 || L.t.zin[k] == 0.0f) continue;
        const int at = (k * L.ny + j) * L.W + m;
        const float cxm = L.t.cxm[i], cxp = L.t.cxp[i], cym = L.t.cym[j], cyp = L.t.cyp[j];
        const float czm = L.t.czm[k], czp = L.t.czp[k];
        const float d = cxm + cxp + cym + cyp + czm + czp;
        float sum = 0.0f;
        if (!zero_in) {
            const float* q = uo + at;
            sum = cxm * q[o - 1] + cxp * q[o];
            sum += cym * q[-L.W] + cyp * q[L.W];
            sum += czm * q[-L.P] + czp * q[L.P];
        }
        uc[at] = (sum - fc[at]) * recip(d);
    }
}

// residual f - A u at a red node (zero off the interior)
__device__ __forceinline__ float lh_resid_red(const LhLevel& L, const float* u, const float* f, int i, int j, int k)
{
    if (i < 1 || i > L.nx - 2 || j < 1 || j > L.ny - 2 || k < 1 || k > L.nz - 2 || L.t.zin[k] == 0.0f) return 0.0f;
    const int at = (k * L.ny + j) * L.W + (i >> 1);
    const int o = i & 1;
    const float cen = u[at];
    const float* q = u + L.cs + at;   // black neighbours
    float a = L.t.cxm[i] * (q[o - 1] - cen) + L.t.cxp[i] * (q[o] - cen);
    a += L.t.cym[j] * (q[-L.W] - cen) + L.t.cyp[j] * (q[L.W] - cen);
    a += L.t.czm[k] * (q[-L.P] - cen) + L.t.czp[k] * (q[L.P] - cen);
    return f[at] - a;
}

// fc = R r, r = f - A u of the fine level on its red nodes (black residuals
// vanish after the black half-sweep that ends the pre-smoothing)
__device__ __forceinline__ void lh_restrict(const LhLevel& F, const float* u, const float* f, const LhLevel& C, float* fcoarse)
{
    const int rx = C.nx - 2, ry = C.ny - 2;
    const int total = rx * ry * (C.nz - 2);
    const float ix = 1.0f / (float)rx, iy = 1.0f / (float)ry;
    for (int t = threadIdx.x; t < total; t += TL_NT) {
        int I0, J0;
        const int row = lh_divmod(t, rx, ix, I0);
        const int K = 1 + lh_divmod(row, ry, iy, J0);
        const int I = 1 + I0, J = 1 + J0;
        if (C.t.zin[K] == 0.0f) continue;
        const int fi = (int)C.t.rfx[I], fj = (int)C.t.rfy[J], fk = (int)C.t.rfz[K];
        float acc = 0.0f;
        for (int cz = 0; cz < 3; ++cz) {
            const float wz = C.t.rwz[3 * K + cz];
            if (wz == 0.0f) continue;
            const int kk = fk - 1 + cz;
            for (int by = 0; by < 3; ++by) {
                const float wy = C.t.rwy[3 * J + by];
                if (wy == 0.0f) continue;
                const int jj = fj - 1 + by;
                float sx = 0.0f;
                for (int ax = 0; ax < 3; ++ax) {
                    const int ii = fi - 1 + ax;
                    const float wx = C.t.rwx[3 * I + ax];
                    if (wx == 0.0f || ((ii + jj + kk) & 1)) continue;
                    sx += wx * lh_resid_red(F, u, f, ii, jj, kk);
                }
                acc += (wz * wy) * sx;
            }
        }
        fcoarse[(K * C.ny + J) * C.W + (I >> 1) + ((I + J + K) & 1) * C.cs] = acc;
    }
}

// u += P e on the fine nodes of colour c (P: trilinear in the coordinates)
__device__ __forceinline__ void lh_prolong(const LhLevel& F, float* u, const LhLevel& C, const float* e, int c)
{
    const int mc = (F.nx - 2) / 2 + 1, ry = F.ny - 2;
    const int total = mc * ry * (F.nz - 2);
    const float im = 1.0f / (float)mc, iy = 1.0f / (float)ry;
    for (int t = threadIdx.x; t < total; t += TL_NT) {
        int m, jj;
        const int row = lh_divmod(t, mc, im, m);
        const int k = 1 + lh_divmod(row, ry, iy, jj);
        const int j = 1 + jj;
        const int o = (c + j + k) & 1, i = o + 2 * m;
        if (i < 1 || i > F.nx - 2 || F.t.zin[k] == 0.0f) continue;
        const int Ix = (int)C.t.pcx[i], Jy = (int)C.t.pcy[j], Kz = (int)C.t.pcz[k];
        const float wx0 = C.t.pwx[2 * i], wx1 = C.t.pwx[2 * i + 1];
        const float wy0 = C.t.pwy[2 * j], wy1 = C.t.pwy[2 * j + 1];
        const float wz0 = C.t.pwz[2 * k], wz1 = C.t.pwz[2 * k + 1];
        float acc = 0.0f;
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
            float sy = 0.0f;
#pragma unroll
            for (int by = 0; by < 2; ++by) {
                const int Jb = Jy + by, Kc = Kz + cz;
                const int rowc = (Kc * C.ny + Jb) * C.W;
                const int ca = (Ix + Jb + Kc) & 1;   // colour of coarse Ix; Ix + 1 has the other
                const float va = e[ca * C.cs + rowc + (Ix >> 1)];
                const float vb = e[(ca ^ 1) * C.cs + rowc + ((Ix + 1) >> 1)];
                sy += (by ? wy1 : wy0) * (wx0 * va + wx1 * vb);
            }
            acc += (cz ? wz1 : wz0) * sy;
        }
        u[c * F.cs + (k * F.ny + j) * F.W + m] += acc;
    }
}

__global__ __launch_bounds__(TL_NT) void k_tail_lds(float* __restrict__ utop, const float* __restrict__ ftop,
                                                    const float* __restrict__ tabs, int nu1, int nu2, int csweeps,
                                                    int top_zero, const LdsPlan* __restrict__ P)
{
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int nl = P->nl;
    // every correction to zero (faces and padding stay zero), the tables in,
    // the top level's right-hand side (and correction) in: 16-byte accesses,
    // four in flight per thread
    for (int q = 0; q < nl; ++q) {
        float4* u4 = reinterpret_cast<float4*>(lds + P->off[q][0]);
        const int n4 = P->dims[q][4] / 2;   // 2 cs / 4
        for (int e = threadIdx.x; e < n4; e += TL_NT) u4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    {
        const int n4 = P->dims[0][4] / 2;
        const float4* f4 = reinterpret_cast<const float4*>(ftop);
        const float4* g4 = reinterpret_cast<const float4*>(utop);
        float4* lf = reinterpret_cast<float4*>(lds + P->off[0][1]);
        float4* lu = reinterpret_cast<float4*>(lds + P->off[0][0]);
        for (int e0 = threadIdx.x; e0 < n4; e0 += 4 * TL_NT) {
            const int e1 = e0 + TL_NT, e2 = e0 + 2 * TL_NT, e3 = e0 + 3 * TL_NT;
            const float4 f0 = f4[e0];
            const float4 f1 = f4[min(e1, n4 - 1)];   // clamped: in bounds, stored only below n4
            const float4 f2 = f4[min(e2, n4 - 1)];
            const float4 f3 = f4[min(e3, n4 - 1)];
            lf[e0] = f0;
            if (e1 < n4) lf[e1] = f1;
            if (e2 < n4) lf[e2] = f2;
            if (e3 < n4) lf[e3] = f3;
        }
        if (!top_zero) {
            for (int e0 = threadIdx.x; e0 < n4; e0 += 4 * TL_NT) {
                const int e1 = e0 + TL_NT, e2 = e0 + 2 * TL_NT, e3 = e0 + 3 * TL_NT;
                const float4 a0 = g4[e0];
                const float4 a1 = g4[min(e1, n4 - 1)];   // clamped: in bounds, stored only below n4
                const float4 a2 = g4[min(e2, n4 - 1)];
                const float4 a3 = g4[min(e3, n4 - 1)];
                lu[e0] = a0;
                if (e1 < n4) lu[e1] = a1;
                if (e2 < n4) lu[e2] = a2;
                if (e3 < n4) lu[e3] = a3;
            }
        }
        for (int e = threadIdx.x; e < P->ntab; e += TL_NT) lds[P->tab0 + e] = tabs[e];
    }
    __syncthreads();
    for (int q = 0; q + 1 < nl; ++q) {
        const LhLevel L = lh_level(lds, P, q);
        float* u = lds + P->off[q][0];
        const float* f = lds + P->off[q][1];
        for (int s = 0; s < nu1; ++s) {
            lh_half(L, u, f, 0, s == 0 && (q > 0 || top_zero));
            __syncthreads();
            lh_half(L, u, f, 1, false);
            __syncthreads();
        }
        lh_restrict(L, u, f, lh_level(lds, P, q + 1), lds + P->off[q + 1][1]);
        __syncthreads();
    }
    {
        // coarsest: csweeps sweeps (red, black), then csweeps (black, red)
        const LhLevel L = lh_level(lds, P, nl - 1);
        float* u = lds + P->off[nl - 1][0];
        const float* f = lds + P->off[nl - 1][1];
        for (int pass = 0; pass < 2 * csweeps; ++pass) {
            for (int h = 0; h < 2; ++h) {
                const int colour = (pass < csweeps) ? h : 1 - h;
                lh_half(L, u, f, colour, pass == 0 && h == 0 && (nl > 1 || top_zero));
                __syncthreads();
            }
        }
    }
    for (int q = nl - 2; q >= 0; --q) {
        const LhLevel L = lh_level(lds, P, q), C = lh_level(lds, P, q + 1);
        float* u = lds + P->off[q][0];
        const float* f = lds + P->off[q][1];
        // only red nodes take the correction when a black half-sweep follows
        lh_prolong(L, u, C, lds + P->off[q + 1][0], 0);
        if (nu2 == 0) lh_prolong(L, u, C, lds + P->off[q + 1][0], 1);
        __syncthreads();
        for (int s = 0; s < nu2; ++s) {
            lh_half(L, u, f, 1, false);
            __syncthreads();
            lh_half(L, u, f, 0, false);
            __syncthreads();
        }
    }
    {
        const int n4 = P->dims[0][4] / 2;
        float4* g4 = reinterpret_cast<float4*>(utop);
        const float4* lu = reinterpret_cast<const float4*>(lds + P->off[0][0]);
        for (int e = threadIdx.x; e < n4; e += TL_NT) g4[e] = lu[e];
    }
}

hipError_t launch_tail_lds(float* u, const float* f, const float* tabs, int nu1, int nu2, int csweeps, int top_zero,
                           const LdsPlan& P, const LdsPlan* P_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_tail_lds, dim3(1), dim3(TL_NT), sizeof(float) * (size_t)P.total, s, u, f, tabs, nu1, nu2,
                       csweeps, top_zero, P_dev);
    return hipGetLastError();
}

// Device limit on one workgroup's LDS, set as the LDS tail's ceiling once
int tail_lds_limit()
{
    static const int lim = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
        if (hipFuncSetAttribute((const void*)k_tail_lds, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess)
            return 0;
        return v;
    }();
    return lim;
}

// ------------------------------------------------------------ reduction
// out[c] = sum_b partials[b * stride + c], c < stride, in a fixed order:
// thread t adds entries t, t + 256, ... of its column, each wave combines its
// lanes by a butterfly, and thread 0 adds the four wave sums in order, so a
// given count always gives the same bits. One workgroup of 256 per column
// (a launch of this size is latency-bound: few threads, no tree of
// barriers, and the columns side by side rather than one after another).
constexpr int RD_NT = 256;

__global__ __launch_bounds__(RD_NT) void k_reduce(const double* __restrict__ part, int stride, int count,
                                                  double* __restrict__ out)
{
    __shared__ double sh[RD_NT / 64];
    const int c = blockIdx.x;
    double a = 0.0;
    for (int t = threadIdx.x; t < count; t += RD_NT) a += part[(size_t)t * stride + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RD_NT / 64; ++w) t += sh[w];
        out[c] = t;
    }
}

hipError_t launch_reduce(const double* partials, int stride, int count, double* out, hipStream_t s)
{
    if (stride < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3(stride), dim3(RD_NT), 0, s, partials, stride, count, out);
    return hipGetLastError();
}

// ------------------------------------------------- explicit instantiation
#define INST(T)                                                                                                  \
    template hipError_t launch_half<T>(const LevelView&, T*, const T*, int, int, T, double*, hipStream_t, int*, int, \
                                       hipEvent_t, hipEvent_t);                                                   \
    template hipError_t launch_half_keep_faces<T>(const LevelView&, T*, const T*, int, T, hipStream_t);          \
    template hipError_t launch_prolong_add<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);      \
    template hipError_t launch_prolong_red<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);      \
    template hipError_t launch_prolong_red_to<T>(const LevelView&, const LevelView&, const T*, const T*, T*,        \
                                                 hipStream_t);                                                  \
    template hipError_t launch_restrict_red<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);     \
    template hipError_t launch_residual_colour<T>(const LevelView&, const T*, const T*, T*, int, hipStream_t);    \
    template hipError_t launch_apply_both<T>(const LevelView&, const T*, T*, double*, hipStream_t, int*);          \
    template hipError_t launch_tail<T>(const TailLevel*, int, int, int, int, int, hipStream_t);                    \
    template hipError_t launch_dot<T>(const LevelView&, const T*, const T*, double*, hipStream_t);                 \
    template hipError_t launch_update_p<T>(const LevelView&, const T*, const T*, T*, const double*, int, int, int,  \
                                           hipStream_t);                                                          \
    template hipError_t launch_update_px<T>(const LevelView&, const T*, const T*, T*, T*, const double*, int, int, \
                                            int, int, int, hipStream_t);                                       \
    template hipError_t launch_update_r<T>(const LevelView&, T*, const T*, const double*, int, int, hipStream_t); \
    template hipError_t launch_update_xr<T>(const LevelView&, T*, T*, const T*, const T*, const double*, int, int, \
                                            double*, hipStream_t, int*, int);                                     \
    template int flat_blocks<T>(const LevelView&);                                                                \
    template hipError_t launch_fill_zero<T>(T*, size_t, hipStream_t);
INST(double)
INST(float)
#undef INST
template hipError_t launch_fill_zero<unsigned char>(unsigned char*, size_t, hipStream_t);

}  // namespace lasto

namespace lasto {

// Flexible (Polak-Ribiere) CG with a preconditioner that changes from step
// to step: beta = <z_new, r_new - r_old> / <z_old, r_old>, where
// r_new - r_old = -alpha_old q_old, so its numerator is
// -alpha_old <z_new, q_old>, alpha_old = <z_old, r_old> / <p_old, q_old> (with
// a fixed symmetric preconditioner <z_new, r_old> = 0 and this is <z_new, r_new>).
__global__ void k_flex_beta(double* scal, int i_rz_old, int i_pq, int i_zq, int i_out)
{
    if (threadIdx.x == 0) {
        const double alpha = scal[i_rz_old] / scal[i_pq];
        scal[i_out] = -alpha * scal[i_zq];
    }
}

hipError_t launch_flex_beta(double* scal, int i_rz_old, int i_pq, int i_zq, int i_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_flex_beta, dim3(1), dim3(64), 0, s, scal, i_rz_old, i_pq, i_zq, i_out);
    return hipGetLastError();
}

}  // namespace lasto

// ------------------------------------------------- streaming ceiling probes
// The rate a plain stream reaches on this device, the ceiling the stencils
// are measured against: dst = src (one read, one write) or dst = a + b (two
// reads, one write, the half-sweep's mix), 16-byte accesses, four per thread
// in flight before any store, grid-stride over resident workgroups.
namespace lasto {

typedef double sp_dbl2 __attribute__((ext_vector_type(2)));

template <int READS>
__global__ __launch_bounds__(256) void k_stream(const sp_dbl2* __restrict__ a, const sp_dbl2* __restrict__ b,
                                                sp_dbl2* __restrict__ d, size_t n)
{
    const size_t stride = (size_t)gridDim.x * 256;
    size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; t + 3 * stride < n; t += 4 * stride) {
        sp_dbl2 x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = a[t + u * stride];
        if (READS == 2) {
#pragma unroll
            for (int u = 0; u < 4; ++u) y[u] = b[t + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) d[t + u * stride] = READS == 2 ? x[u] + y[u] : x[u];
    }
    for (; t < n; t += stride) d[t] = READS == 2 ? a[t] + b[t] : a[t];
}

}  // namespace lasto

// dst = a (b NULL) or dst = a + b over `bytes` (a multiple of 16) of FP64 data
extern "C" lasto_status lasto_stream_probe(const double* a, const double* b, double* dst, size_t bytes,
                                           void* hip_stream)
{
    if (!a || !dst || bytes % 16 != 0) return lasto::fail(LASTO_ERR_ARG, "lasto_stream_probe: NULL or bytes % 16");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return lasto::fail(LASTO_ERR_HIP, "lasto_stream_probe: device query");
    const size_t n = bytes / 16;
    const unsigned grid = (unsigned)std::max(8, cus * 8);
    hipStream_t s = (hipStream_t)hip_stream;
    typedef lasto::sp_dbl2 V;
    if (b)
        hipLaunchKernelGGL(lasto::k_stream<2>, dim3(grid), dim3(256), 0, s, (const V*)a, (const V*)b, (V*)dst, n);
    else
        hipLaunchKernelGGL(lasto::k_stream<1>, dim3(grid), dim3(256), 0, s, (const V*)a, (const V*)nullptr, (V*)dst, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lasto::fail(LASTO_ERR_HIP, std::string("lasto_stream_probe: ") + hipGetErrorString(e));
    return LASTO_OK;
}
