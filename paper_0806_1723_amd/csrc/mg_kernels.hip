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

#include "internal.h"

namespace lasto {

// ------------------------------------------------------------- helpers
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

// restricted value at coarse (I,J,K): the up-to-3x3x3 fine nodes around
// (rf[I], rf[J], rf[K]) weighted by rw_x rw_y rw_z (M_c^-1 P^T M_f).
// RED_ONLY: the fine residual is known to vanish on black nodes (as it does
// right after a black half-sweep), so they are not read.
template <typename T, bool RED_ONLY>
__device__ __forceinline__ T restrict_point(const LevelView& F, const LevelView& C, const T* __restrict__ r, int I,
                                            int J, int K)
{
    const int fi = C.ax[0].rf[I], fj = C.ax[1].rf[J], fk = C.ax[2].rf[K];
    const double* wx = C.ax[0].rw + 3 * I;
    const double* wy = C.ax[1].rw + 3 * J;
    const double* wz = C.ax[2].rw + 3 * K;
    T acc = T(0);
    for (int c = 0; c < 3; ++c) {
        const T z = (T)wz[c];
        if (z == T(0)) continue;
        for (int b = 0; b < 3; ++b) {
            const T y = (T)wy[b];
            if (y == T(0)) continue;
            const int jj = fj - 1 + b, kk = fk - 1 + c;
            T sx = T(0);
            for (int a = 0; a < 3; ++a) {
                const T x = (T)wx[a];
                if (RED_ONLY && ((fi - 1 + a + jj + kk) & 1)) continue;
                if (x != T(0)) sx += x * r[sidx(F, fi - 1 + a, jj, kk)];
            }
            acc += z * y * sx;
        }
    }
    return acc;
}

// interpolated coarse correction at fine (i,j,k): the 2x2x2 coarse values
// around it with linear weights in physical coordinates (weight 1 at kept
// nodes); coarse neighbours with zero weight are not read
template <typename T>
__device__ __forceinline__ T prolong_point(const LevelView& C, const T* __restrict__ e, int i, int j, int k)
{
    const int I = C.ax[0].pc[i], J = C.ax[1].pc[j], K = C.ax[2].pc[k];
    const T wx[2] = {(T)C.ax[0].pw[2 * i], (T)C.ax[0].pw[2 * i + 1]};
    const T wy[2] = {(T)C.ax[1].pw[2 * j], (T)C.ax[1].pw[2 * j + 1]};
    const T wz[2] = {(T)C.ax[2].pw[2 * k], (T)C.ax[2].pw[2 * k + 1]};
    T w = T(0);
    for (int c = 0; c < 2; ++c) {
        if (wz[c] == T(0)) continue;
        T v = T(0);
        for (int b = 0; b < 2; ++b) {
            if (wy[b] == T(0)) continue;
            T a = T(0);
            for (int q = 0; q < 2; ++q)
                if (wx[q] != T(0)) a += wx[q] * e[sidx(C, I + q, J + b, K + c)];
            v += wy[b] * a;
        }
        w += wz[c] * v;
    }
    return w;
}

// --------------------------------------------------------- half-sweep
// Workgroups are dispatched to the eight XCDs in turn; tile (id % 8) * per +
// id / 8 hands each XCD a contiguous run of tiles, so tiles that share halo
// rows share an L2. Ids past the last tile only contribute a zero partial.
__device__ __forceinline__ int xcd_tile(int id, int per) { return (id & 7) * per + (id >> 3); }

constexpr int HS_X = 64, HS_Y = 4, HS_NT = HS_X * HS_Y, HS_KC_MAX = 16, HS_BLOCKS = 2048;

struct HalfShape {
    int nbx, nby, nbz, nb, per, grid, kc;
};

// Planes per thread: as many as keep about HS_BLOCKS workgroups (the z-march
// saves re-reads, but its planes are a serial chain of loads, so small levels
// march one plane per thread).
static HalfShape half_shape(const LevelView& L)
{
    HalfShape h;
    const int mcount = (L.nx - 2) / 2 + 1;   // i >> 1 over every interior i
    h.nbx = (mcount + HS_X - 1) / HS_X;
    h.nby = (L.ny - 2 + HS_Y - 1) / HS_Y;
    const long tiles = (long)h.nbx * h.nby;
    h.kc = (int)std::min<long>(HS_KC_MAX, std::max<long>(1, (long)(L.nz - 2) * tiles / HS_BLOCKS));
    h.nbz = (L.nz - 2 + h.kc - 1) / h.kc;
    h.nb = h.nbx * h.nby * h.nbz;
    h.per = (h.nb + 7) / 8;
    h.grid = 8 * h.per;
    return h;
}

int half_blocks(const LevelView& L) { return half_shape(L).grid; }

// Nodes of colour c solve their own equation with the other colour's values
// (RESID = false):
//   u_n = (sum_d am_d u_{n-e_d} + ap_d u_{n+e_d} - bscale f_n) / sum_d (am_d + ap_d),
// or (RESID = true) get their residual out_n = bscale f_n - (A u)_n.
// A thread owns the entries [c][k][j][m] for one (j, m) and marches over a
// chunk of planes, keeping the other colour's z-neighbours in a register
// queue (entry m of the other colour on planes k-1, k, k+1 holds both z
// neighbours and one x neighbour) and loading plane k+1's operands while it
// computes plane k. `uo` (the other colour), `fc` and `out` (this colour) are
// distinct arrays, so the loads may run ahead of the store.
template <typename T, bool RESID>
__global__ __launch_bounds__(HS_NT) void k_half(LevelView L, const T* __restrict__ uo, const T* __restrict__ fc,
                                                const T* __restrict__ ucen, T* __restrict__ out, int c, int zero_in,
                                                T bscale, double* __restrict__ dotp, int nbx, int nby, int nb, int per,
                                                int kc)
{
    __shared__ double red[HS_NT / 64];
    const int t = xcd_tile(blockIdx.x, per);
    double dot = 0.0;
    const int m = (t % nbx) * HS_X + (threadIdx.x & (HS_X - 1));
    const int j = 1 + ((t / nbx) % nby) * HS_Y + (threadIdx.x >> 6);
    if (t < nb && j <= L.ny - 2 && m <= (L.nx - 2) / 2) {
        const int k0 = 1 + (t / (nbx * nby)) * kc;
        const int k1 = min(k0 + kc, L.nz - 1);
        const int nx = L.nx;
        const int W = L.W;
        const size_t plane = (size_t)L.ny * W;
        const size_t row = (size_t)j * W + m;
        const T cym = (T)L.ax[1].am[j], cyp = (T)L.ax[1].ap[j];
        const double* __restrict__ amx = L.ax[0].am;
        const double* __restrict__ apx = L.ax[0].ap;
        // operands of plane k: z queue, the other x neighbour, y neighbours, f, centre
        T zm = T(0), zc = T(0), zp = T(0), xo = T(0), ym = T(0), yp = T(0), fv, cv = T(0);
        auto load_plane = [&](int k, T& x_o, T& y_m, T& y_p, T& f_v, T& c_v) {
            const size_t at = (size_t)k * plane + row;
            const int o = (c + j + k) & 1;
            f_v = fc[at];
            if (RESID) c_v = ucen[at];
            if (!zero_in) {
                x_o = o ? uo[at + 1] : uo[at - (m > 0 ? 1 : 0)];
                y_m = uo[at - W];
                y_p = uo[at + W];
            }
        };
        if (!zero_in) {
            zm = uo[(size_t)(k0 - 1) * plane + row];
            zc = uo[(size_t)k0 * plane + row];
            zp = uo[(size_t)(k0 + 1) * plane + row];
        }
        load_plane(k0, xo, ym, yp, fv, cv);
        for (int k = k0; k < k1; ++k) {
            // prefetch plane k+1 (and the z queue's next entry)
            T xo_n = T(0), ym_n = T(0), yp_n = T(0), fv_n = T(0), cv_n = T(0), znext = T(0);
            if (k + 1 < k1) {
                load_plane(k + 1, xo_n, ym_n, yp_n, fv_n, cv_n);
                if (!zero_in) znext = uo[(size_t)(k + 2) * plane + row];
            }
            const int o = (c + j + k) & 1;
            const int i = o + 2 * m;
            if (i >= 1 && i <= nx - 2) {
                const size_t at = (size_t)k * plane + row;
                const T cxm = (T)amx[i], cxp = (T)apx[i];
                const T czm = (T)L.ax[2].am[k], czp = (T)L.ax[2].ap[k];
                T s = T(0);
                if (!zero_in) {
                    // x neighbours i-1, i+1 of the other colour sit at m-1+o and m+o
                    const T xl = o ? zc : xo;
                    const T xr = o ? xo : zc;
                    s = cxm * xl + cxp * xr;
                    s += cym * ym + cyp * yp;
                    s += czm * zm + czp * zp;
                }
                const T d = cxm + cxp + cym + cyp + czm + czp;
                T res;
                if (RESID) res = bscale * fv - (s - d * cv);
                else res = (s - bscale * fv) / d;
                out[at] = res;
                if (dotp) dot += vol_at(L, i, j, k) * (double)fv * (double)res;
            }
            zm = zc;
            zc = zp;
            zp = znext;
            xo = xo_n;
            ym = ym_n;
            yp = yp_n;
            fv = fv_n;
            cv = cv_n;
        }
    }
    if (dotp) {
        const double s = block_sum<HS_NT>(dot, red);
        if (threadIdx.x == 0) dotp[blockIdx.x] = s;
    }
}

template <typename T>
hipError_t launch_half(const LevelView& L, T* u, const T* f, int colour, int zero_in, T bscale, double* dotp,
                       hipStream_t s)
{
    const HalfShape h = half_shape(L);
    hipLaunchKernelGGL((k_half<T, false>), dim3(h.grid), dim3(HS_NT), 0, s, L, u + (size_t)(1 - colour) * L.cs,
                       f + (size_t)colour * L.cs, (const T*)nullptr, u + (size_t)colour * L.cs, colour, zero_in, bscale,
                       dotp, h.nbx, h.nby, h.nb, h.per, h.kc);
    return hipGetLastError();
}

// residual f - A u at the nodes of one colour only (written into that
// colour of r; the other colour of r is not touched)
template <typename T>
hipError_t launch_residual_colour(const LevelView& L, const T* u, const T* f, T* r, int colour, hipStream_t s)
{
    const HalfShape h = half_shape(L);
    hipLaunchKernelGGL((k_half<T, true>), dim3(h.grid), dim3(HS_NT), 0, s, L, u + (size_t)(1 - colour) * L.cs,
                       f + (size_t)colour * L.cs, u + (size_t)colour * L.cs, r + (size_t)colour * L.cs, colour, 0,
                       T(1), (double*)nullptr, h.nbx, h.nby, h.nb, h.per, h.kc);
    return hipGetLastError();
}

// ------------------------------------------------- pointwise 3-D launches
// A workgroup covers a 64 x 4 tile of (i, j) interior columns over a chunk
// of kp planes (kp chosen to keep about PT_BLOCKS workgroups); split arrays
// are read through sidx, so a wavefront touches two contiguous runs (one per
// colour). Reducing kernels write one partial per workgroup.
constexpr int PT_X = 64, PT_Y = 4, PT_NT = PT_X * PT_Y, PT_BLOCKS = 4096, PT_KP_MAX = 32;

struct PtShape {
    dim3 grid;
    int kp;
};

static PtShape pt_shape(const LevelView& L)
{
    PtShape p;
    const int gx = (L.nx - 2 + PT_X - 1) / PT_X, gy = (L.ny - 2 + PT_Y - 1) / PT_Y;
    const long tiles = (long)gx * gy;
    p.kp = (int)std::min<long>(PT_KP_MAX, std::max<long>(1, (long)(L.nz - 2) * tiles / PT_BLOCKS));
    p.grid = dim3(gx, gy, (L.nz - 2 + p.kp - 1) / p.kp);
    return p;
}

int interior_blocks(const LevelView& L)
{
    const dim3 g = pt_shape(L).grid;
    return (int)(g.x * g.y * g.z);
}

#define INTERIOR_LOOP                                                 \
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);       \
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);       \
    const bool inside = (i <= L.nx - 2) && (j <= L.ny - 2);           \
    const int kb_ = 1 + blockIdx.z * kp;                              \
    const int ke_ = min(kb_ + kp, L.nz - 1);                          \
    for (int k = kb_; k < ke_; ++k)

#define PT_LAUNCH(kernel, L, s, ...)                                                         \
    do {                                                                                     \
        const PtShape ps_ = pt_shape(L);                                                     \
        hipLaunchKernelGGL(kernel, ps_.grid, dim3(PT_NT), 0, s, L, ps_.kp, __VA_ARGS__);      \
    } while (0)

// r = f - A u (split arrays)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_residual(LevelView L, int kp, const T* __restrict__ u,
                                                    const T* __restrict__ f, T* __restrict__ r)
{
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        r[at] = f[at] - apply_split(L, u, i, j, k, u[at]);
    }
}

template <typename T>
hipError_t launch_residual(const LevelView& L, const T* u, const T* f, T* r, hipStream_t s)
{
    PT_LAUNCH(k_residual<T>, L, s, u, f, r);
    return hipGetLastError();
}

// Fine level, natural v and rho: r = bscale rho - A v (r in the split layout
// when given) and partials of ||r||_W^2. interior_zero: the interior of v is
// read as zero (the reference residual of the face data alone).
__global__ __launch_bounds__(PT_NT) void k_residual_nat(LevelView L, int kp, const double* __restrict__ v,
                                                        const double* __restrict__ rho, double bscale,
                                                        double* __restrict__ r, double* __restrict__ part,
                                                        int interior_zero)
{
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        const size_t sxy = (size_t)nx * ny;
        const size_t idx = (size_t)k * sxy + (size_t)j * nx + i;
        double a;
        if (!interior_zero) {
            const double c = v[idx];
            a = L.ax[0].am[i] * (v[idx - 1] - c) + L.ax[0].ap[i] * (v[idx + 1] - c);
            a += L.ax[1].am[j] * (v[idx - nx] - c) + L.ax[1].ap[j] * (v[idx + nx] - c);
            a += L.ax[2].am[k] * (v[idx - sxy] - c) + L.ax[2].ap[k] * (v[idx + sxy] - c);
        } else {
            a = 0.0;
            if (i == 1) a += L.ax[0].am[i] * v[idx - 1];
            if (i == nx - 2) a += L.ax[0].ap[i] * v[idx + 1];
            if (j == 1) a += L.ax[1].am[j] * v[idx - nx];
            if (j == ny - 2) a += L.ax[1].ap[j] * v[idx + nx];
            if (k == 1) a += L.ax[2].am[k] * v[idx - sxy];
            if (k == nz - 2) a += L.ax[2].ap[k] * v[idx + sxy];
        }
        const double res = bscale * rho[idx] - a;
        if (r) r[sidx(L, i, j, k)] = res;
        acc += vol_at(L, i, j, k) * res * res;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

hipError_t launch_residual_nat(const LevelView& L, const double* v, const double* rho, double bscale, double* r_split,
                               double* partials, int interior_zero, hipStream_t s)
{
    PT_LAUNCH(k_residual_nat, L, s, v, rho, bscale, r_split, partials, interior_zero);
    return hipGetLastError();
}

// Au = A u, natural layout (the diagnostic lasto_apply)
__global__ __launch_bounds__(PT_NT) void k_apply_nat(LevelView L, int kp, const double* __restrict__ u,
                                                     double* __restrict__ Au)
{
    INTERIOR_LOOP
    {
        if (!inside) continue;
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

// q = A p and partial <p, q>_W (split arrays)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_apply_dot(LevelView L, int kp, const T* __restrict__ p,
                                                     T* __restrict__ q, double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        const T c = p[at];
        const T a = apply_split(L, p, i, j, k, c);
        q[at] = a;
        acc += vol_at(L, i, j, k) * (double)c * (double)a;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_apply_dot(const LevelView& L, const T* p, T* q, double* partials, hipStream_t s)
{
    PT_LAUNCH(k_apply_dot<T>, L, s, p, q, partials);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(PT_NT) void k_dot(LevelView L, int kp, const T* __restrict__ a, const T* __restrict__ b,
                                               double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    double acc = 0.0;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        acc += vol_at(L, i, j, k) * (double)a[at] * (double)b[at];
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_dot(const LevelView& L, const T* a, const T* b, double* partials, hipStream_t s)
{
    PT_LAUNCH(k_dot<T>, L, s, a, b, partials);
    return hipGetLastError();
}

// pnew = z + beta pold, beta = scal[i_num]/scal[i_den] (0 on the first step)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_update_p(LevelView L, int kp, const T* __restrict__ z,
                                                    const T* __restrict__ pold, T* __restrict__ pnew,
                                                    const double* __restrict__ scal, int i_num, int i_den, int first)
{
    const T beta = first ? T(0) : (T)(scal[i_num] / scal[i_den]);
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        pnew[at] = first ? z[at] : z[at] + beta * pold[at];
    }
}

template <typename T>
hipError_t launch_update_p(const LevelView& L, const T* z, const T* pold, T* pnew, const double* scal, int i_num,
                           int i_den, int first, hipStream_t s)
{
    PT_LAUNCH(k_update_p<T>, L, s, z, pold, pnew, scal, i_num, i_den, first);
    return hipGetLastError();
}

// x += alpha p, r -= alpha q, alpha = scal[i_num]/scal[i_den]; partial <r,r>_W.
// A non-finite alpha leaves x and r untouched (the caller then reports the
// breakdown with x still the last finite iterate).
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_update_xr(LevelView L, int kp, void* __restrict__ xv, int x_nat,
                                                     T* __restrict__ r, const T* __restrict__ p,
                                                     const T* __restrict__ q, const double* __restrict__ scal,
                                                     int i_num, int i_den, double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    const double ad = scal[i_num] / scal[i_den];
    const bool ok = isfinite(ad);
    const T alpha = (T)ad;
    double acc = 0.0;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        T rv = r[at];
        if (ok) {
            if (x_nat) {
                double* x = (double*)xv;
                const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
                x[idx] = x[idx] + ad * (double)p[at];
            } else {
                T* x = (T*)xv;
                x[at] = x[at] + alpha * p[at];
            }
            rv = rv - alpha * q[at];
            r[at] = rv;
        }
        acc += vol_at(L, i, j, k) * (double)rv * (double)rv;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = ok ? t : __builtin_nan("");
}

template <typename T>
hipError_t launch_update_xr(const LevelView& L, void* x, int x_nat, T* r, const T* p, const T* q, const double* scal,
                            int i_num, int i_den, double* partials, hipStream_t s)
{
    PT_LAUNCH(k_update_xr<T>, L, s, x, x_nat, r, p, q, scal, i_num, i_den, partials);
    return hipGetLastError();
}

// v (natural) += e (split), interior
__global__ __launch_bounds__(PT_NT) void k_add_nat(LevelView L, int kp, double* __restrict__ v,
                                                   const double* __restrict__ e)
{
    INTERIOR_LOOP
    {
        if (!inside) continue;
        v[((size_t)k * L.ny + j) * L.nx + i] += e[sidx(L, i, j, k)];
    }
}

hipError_t launch_add_nat(const LevelView& L, double* v, const double* e_split, hipStream_t s)
{
    PT_LAUNCH(k_add_nat, L, s, v, e_split);
    return hipGetLastError();
}

// r32 = r / sqrt(scal[i_norm2]) (scaled FP32 copy of the FP64 residual, split)
__global__ __launch_bounds__(PT_NT) void k_scale_to32(LevelView L, int kp, const double* __restrict__ r,
                                                      float* __restrict__ r32, const double* __restrict__ scal,
                                                      int i_norm2)
{
    const double inv = 1.0 / sqrt(scal[i_norm2]);
    INTERIOR_LOOP
    {
        if (!inside) continue;
        const size_t at = sidx(L, i, j, k);
        r32[at] = (float)(r[at] * inv);
    }
}

hipError_t launch_scale_to32(const LevelView& L, const double* r, float* r32, const double* scal, int i_norm2,
                             hipStream_t s)
{
    PT_LAUNCH(k_scale_to32, L, s, r, r32, scal, i_norm2);
    return hipGetLastError();
}

// v (natural) += sqrt(scal[i_norm2]) * e32 (split): the defect correction
__global__ __launch_bounds__(PT_NT) void k_add_scaled32_nat(LevelView L, int kp, double* __restrict__ v,
                                                            const float* __restrict__ e,
                                                            const double* __restrict__ scal, int i_norm2)
{
    const double sc = sqrt(scal[i_norm2]);
    if (!isfinite(sc)) return;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        v[((size_t)k * L.ny + j) * L.nx + i] += sc * (double)e[sidx(L, i, j, k)];
    }
}

hipError_t launch_add_scaled32_nat(const LevelView& L, double* v, const float* e32, const double* scal, int i_norm2,
                                   hipStream_t s)
{
    PT_LAUNCH(k_add_scaled32_nat, L, s, v, e32, scal, i_norm2);
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
        if (!inside) continue;
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

__global__ void k_inject_nan(double* r, size_t idx)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) r[idx] = __builtin_nan("");
}

hipError_t launch_inject_nan(double* r, size_t idx, hipStream_t s)
{
    hipLaunchKernelGGL(k_inject_nan, dim3(1), dim3(64), 0, s, r, idx);
    return hipGetLastError();
}

// ---------------------------------------------------------- transfers
template <typename T, bool RED_ONLY>
__global__ __launch_bounds__(PT_NT) void k_restrict(LevelView C, int kp, LevelView F, const T* __restrict__ r,
                                                    T* __restrict__ rc)
{
    const LevelView& L = C;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        rc[sidx(C, i, j, k)] = restrict_point<T, RED_ONLY>(F, C, r, i, j, k);
    }
}

template <typename T>
hipError_t launch_restrict(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s)
{
    PT_LAUNCH((k_restrict<T, false>), C, s, F, r, rc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_red(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s)
{
    PT_LAUNCH((k_restrict<T, true>), C, s, F, r, rc);
    return hipGetLastError();
}

// u += P e on the red nodes only: when a black half-sweep follows, it
// overwrites every black value, so correcting them would be wasted work.
template <typename T>
__global__ __launch_bounds__(HS_NT) void k_prolong_red(LevelView F, LevelView C, const T* __restrict__ e,
                                                       T* __restrict__ u, int nbx, int nby, int nb, int per, int kc)
{
    const int t = xcd_tile(blockIdx.x, per);
    const int m = (t % nbx) * HS_X + (threadIdx.x & (HS_X - 1));
    const int j = 1 + ((t / nbx) % nby) * HS_Y + (threadIdx.x >> 6);
    if (t >= nb || j > F.ny - 2 || m > (F.nx - 2) / 2) return;
    const int k0 = 1 + (t / (nbx * nby)) * kc;
    const int k1 = min(k0 + kc, F.nz - 1);
    const size_t plane = (size_t)F.ny * F.W;
    const size_t row = (size_t)j * F.W + m;
    for (int k = k0; k < k1; ++k) {
        const int i = ((j + k) & 1) + 2 * m;
        if (i < 1 || i > F.nx - 2) continue;
        u[(size_t)k * plane + row] += prolong_point(C, e, i, j, k);
    }
}

template <typename T>
hipError_t launch_prolong_red(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s)
{
    const HalfShape h = half_shape(F);
    hipLaunchKernelGGL(k_prolong_red<T>, dim3(h.grid), dim3(HS_NT), 0, s, F, C, e, u, h.nbx, h.nby, h.nb, h.per, h.kc);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(PT_NT) void k_prolong_add(LevelView F, int kp, LevelView C, const T* __restrict__ e,
                                                       T* __restrict__ u)
{
    const LevelView& L = F;
    INTERIOR_LOOP
    {
        if (!inside) continue;
        u[sidx(F, i, j, k)] += prolong_point(C, e, i, j, k);
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
constexpr int TL_NT = 1024;

// One half-sweep of colour c by the whole workgroup. A thread takes up to
// TL_BATCH nodes at a time and computes all their new values before storing
// any (nodes of one colour never read each other), so the loads of a batch
// are in flight together instead of forming a chain.
constexpr int TL_BATCH = 8;

template <typename T>
__device__ void t_half(const LevelView& V, T* __restrict__ u, const T* __restrict__ f, int c, int zero_in)
{
    const int mcount = (V.nx - 2) / 2 + 1, nyi = V.ny - 2;
    const int total = mcount * nyi * (V.nz - 2);
    for (int base = 0; base < total; base += TL_NT * TL_BATCH) {
        T val[TL_BATCH];
        size_t at[TL_BATCH];
        bool ok[TL_BATCH];
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b) {
            const int t = base + b * TL_NT + threadIdx.x;
            const int m = t % mcount, j = 1 + (t / mcount) % nyi, k = 1 + t / (mcount * nyi);
            const int i = ((c + j + k) & 1) + 2 * m;
            ok[b] = t < total && i >= 1 && i <= V.nx - 2;
            at[b] = 0;
            val[b] = T(0);
            if (!ok[b]) continue;
            at[b] = sidx(V, i, j, k);
            if (zero_in) {
                const T d = (T)(V.ax[0].am[i] + V.ax[0].ap[i] + V.ax[1].am[j] + V.ax[1].ap[j] + V.ax[2].am[k] +
                                V.ax[2].ap[k]);
                val[b] = -f[at[b]] / d;
            } else {
                val[b] = gs_point(V, u, i, j, k, f[at[b]]);
            }
        }
#pragma unroll
        for (int b = 0; b < TL_BATCH; ++b)
            if (ok[b]) u[at[b]] = val[b];
    }
}

template <typename T>
__global__ __launch_bounds__(TL_NT) void k_tail(const TailLevel* __restrict__ lv, int nl, int nu1, int nu2,
                                                int csweeps)
{
    // descent
    for (int l = 0; l + 1 < nl; ++l) {
        const LevelView& V = lv[l].V;
        T* u = TailBuf<T>::u(lv[l]);
        const T* f = TailBuf<T>::f(lv[l]);
        for (int s = 0; s < nu1; ++s) {
            t_half<T>(V, u, f, 0, s == 0);
            __syncthreads();
            t_half<T>(V, u, f, 1, 0);
            __syncthreads();
        }
        // residual on red nodes only (the black half-sweep just zeroed it on black)
        T* r = TailBuf<T>::r(lv[l]);
        const int ni = (V.nx - 2) * (V.ny - 2) * (V.nz - 2);
        for (int t = threadIdx.x; t < ni; t += TL_NT) {
            const int i = 1 + t % (V.nx - 2), j = 1 + (t / (V.nx - 2)) % (V.ny - 2), k = 1 + t / ((V.nx - 2) * (V.ny - 2));
            if ((i + j + k) & 1) continue;
            const size_t at = sidx(V, i, j, k);
            r[at] = f[at] - apply_split(V, u, i, j, k, u[at]);
        }
        __syncthreads();
        const LevelView& C = lv[l + 1].V;
        T* fc = TailBuf<T>::f(lv[l + 1]);
        const int nc = (C.nx - 2) * (C.ny - 2) * (C.nz - 2);
        for (int t = threadIdx.x; t < nc; t += TL_NT) {
            const int I = 1 + t % (C.nx - 2), J = 1 + (t / (C.nx - 2)) % (C.ny - 2), K = 1 + t / ((C.nx - 2) * (C.ny - 2));
            fc[sidx(C, I, J, K)] = restrict_point<T, true>(V, C, (const T*)r, I, J, K);
        }
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
                t_half<T>(V, u, f, colour, pass == 0 && h == 0);
                __syncthreads();
            }
        }
    }
    // ascent
    for (int l = nl - 2; l >= 0; --l) {
        const LevelView& V = lv[l].V;
        const LevelView& C = lv[l + 1].V;
        T* u = TailBuf<T>::u(lv[l]);
        const T* f = TailBuf<T>::f(lv[l]);
        const T* e = TailBuf<T>::u(lv[l + 1]);
        // correction on red nodes only when a black half-sweep follows
        const int ni = (V.nx - 2) * (V.ny - 2) * (V.nz - 2);
        for (int t = threadIdx.x; t < ni; t += TL_NT) {
            const int i = 1 + t % (V.nx - 2), j = 1 + (t / (V.nx - 2)) % (V.ny - 2), k = 1 + t / ((V.nx - 2) * (V.ny - 2));
            if (nu2 > 0 && ((i + j + k) & 1)) continue;
            u[sidx(V, i, j, k)] += prolong_point(C, e, i, j, k);
        }
        __syncthreads();
        for (int s = 0; s < nu2; ++s) {
            t_half<T>(V, u, f, 1, 0);
            __syncthreads();
            t_half<T>(V, u, f, 0, 0);
            __syncthreads();
        }
    }
}

template <typename T>
hipError_t launch_tail(const TailLevel* lv, int nl, int nu1, int nu2, int csweeps, hipStream_t s)
{
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(TL_NT), 0, s, lv, nl, nu1, nu2, csweeps);
    return hipGetLastError();
}

// ------------------------------------------------------------ reduction
// out[c] = sum_b partials[b * stride + c], c < stride, in a fixed order
// (thread t takes t, t+1024, ..., then a fixed tree): a given launch shape
// always gives the same bits.
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ part, int stride, int count,
                                                 double* __restrict__ out)
{
    __shared__ double sh[1024];
    for (int c = 0; c < stride; ++c) {
        double a = 0.0;
        for (int t = threadIdx.x; t < count; t += 1024) a += part[(size_t)t * stride + c];
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = sh[0];
        __syncthreads();
    }
}

hipError_t launch_reduce(const double* partials, int stride, int count, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partials, stride, count, out);
    return hipGetLastError();
}

// ------------------------------------------------- explicit instantiation
#define INST(T)                                                                                                  \
    template hipError_t launch_half<T>(const LevelView&, T*, const T*, int, int, T, double*, hipStream_t);         \
    template hipError_t launch_residual<T>(const LevelView&, const T*, const T*, T*, hipStream_t);                 \
    template hipError_t launch_restrict<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);         \
    template hipError_t launch_prolong_add<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);      \
    template hipError_t launch_prolong_red<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);      \
    template hipError_t launch_restrict_red<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);     \
    template hipError_t launch_residual_colour<T>(const LevelView&, const T*, const T*, T*, int, hipStream_t);    \
    template hipError_t launch_tail<T>(const TailLevel*, int, int, int, int, hipStream_t);                         \
    template hipError_t launch_apply_dot<T>(const LevelView&, const T*, T*, double*, hipStream_t);                 \
    template hipError_t launch_dot<T>(const LevelView&, const T*, const T*, double*, hipStream_t);                 \
    template hipError_t launch_update_p<T>(const LevelView&, const T*, const T*, T*, const double*, int, int, int,  \
                                           hipStream_t);                                                          \
    template hipError_t launch_update_xr<T>(const LevelView&, void*, int, T*, const T*, const T*, const double*,   \
                                            int, int, double*, hipStream_t);                                      \
    template hipError_t launch_fill_zero<T>(T*, size_t, hipStream_t);
INST(double)
INST(float)
#undef INST
template hipError_t launch_fill_zero<unsigned char>(unsigned char*, size_t, hipStream_t);

}  // namespace lasto
