// Multigrid and Krylov kernels of the Poisson solve (eq. (3.2)) on the graded
// tensor-product mesh, gfx950 (wave64). All of these are HBM-bound stencils
// and streams; none uses MFMA.
//
// Operator (interior node n, per axis d):
//   (A u)_n = sum_d am_d (u_{n-e_d} - u_n) + ap_d (u_{n+e_d} - u_n)
// with am = 1/(h_- m), ap = 1/(h_+ m), m = (h_- + h_+)/2: the three-point
// second difference on a nonuniform mesh. Equation A u = bscale * f.
#include "internal.h"

namespace lasto {

// ------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Deterministic block sum (fixed tree); result valid in thread 0.
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

// ---------------------------------------------------------- smoother
// One fused red-black Gauss-Seidel sweep, out of place: uout = S(uin).
// Nodes of parity `first` ((i+j+k)&1 == first) are updated from uin; the
// other colour is then updated from those new values. Because the sweep reads
// only uin and writes only uout, every tile recomputes the first-colour
// values it needs on its one-node ring, and the result does not depend on
// the tiling or on the order in which tiles run.
//
// A workgroup owns a TX x TY tile of (i,j) columns and marches in z over a
// chunk of KC planes, keeping three planes of uin (tile + 2-node ring) and
// three planes of the half-updated field H (tile + 1-node ring) in LDS.
constexpr int SM_TX = 64, SM_TY = 4, SM_KC = 16, SM_NT = SM_TX * SM_TY;

template <typename T>
__global__ __launch_bounds__(SM_NT) void k_smooth(LevelView L, const T* __restrict__ uin,
                                                   const T* __restrict__ f, T* __restrict__ uout, T bscale,
                                                   int first, int zero_in, double* __restrict__ dotp)
{
    __shared__ T Us[3][SM_TY + 4][SM_TX + 4];
    __shared__ T Hs[3][SM_TY + 2][SM_TX + 2];
    __shared__ double red[SM_NT / 64];

    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int i0 = 1 + blockIdx.x * SM_TX, j0 = 1 + blockIdx.y * SM_TY;
    const int k0 = 1 + blockIdx.z * SM_KC;
    const int k1 = min(k0 + SM_KC, nz - 1);
    const int tid = threadIdx.x;
    const size_t sxy = (size_t)nx * ny;
    const double* __restrict__ amx = L.ax[0].am;
    const double* __restrict__ apx = L.ax[0].ap;
    const double* __restrict__ amy = L.ax[1].am;
    const double* __restrict__ apy = L.ax[1].ap;
    const double* __restrict__ amz = L.ax[2].am;
    const double* __restrict__ apz = L.ax[2].ap;

    auto loadU = [&](int k) {
        T(*dst)[SM_TX + 4] = Us[(k + 3) % 3];
        for (int e = tid; e < (SM_TY + 4) * (SM_TX + 4); e += SM_NT) {
            const int a = e % (SM_TX + 4), b = e / (SM_TX + 4);
            const int i = i0 - 2 + a, j = j0 - 2 + b;
            T val = T(0);
            if (!zero_in && i >= 0 && i < nx && j >= 0 && j < ny) val = uin[(size_t)k * sxy + (size_t)j * nx + i];
            dst[b][a] = val;
        }
    };

    const int kstart = k0 - 1;
    if (kstart - 1 >= 0) loadU(kstart - 1);
    loadU(kstart);

    // tile point owned by this thread for the output step
    const int tx = tid % SM_TX, ty = tid / SM_TX;
    const int io = i0 + tx, jo = j0 + ty;
    const bool own = (io <= nx - 2) && (jo <= ny - 2);
    double dot = 0.0;

    for (int kk = kstart; kk <= k1; ++kk) {
        if (kk + 1 <= nz - 1) loadU(kk + 1);
        __syncthreads();
        // H at plane kk over the tile and its one-node ring
        {
            T(*H)[SM_TX + 2] = Hs[(kk + 3) % 3];
            T(*U)[SM_TX + 4] = Us[(kk + 3) % 3];
            const bool bplane = (kk == 0) || (kk == nz - 1);
            for (int e = tid; e < (SM_TY + 2) * (SM_TX + 2); e += SM_NT) {
                const int a = e % (SM_TX + 2), b = e / (SM_TX + 2);
                const int i = i0 - 1 + a, j = j0 - 1 + b;
                if (i > nx - 1 || j > ny - 1) continue;
                T uc = U[b + 1][a + 1];
                const bool bnode = bplane || i == 0 || i == nx - 1 || j == 0 || j == ny - 1;
                if (!bnode && (((i + j + kk) & 1) == first)) {
                    T(*Um)[SM_TX + 4] = Us[(kk + 2) % 3];
                    T(*Up)[SM_TX + 4] = Us[(kk + 1) % 3];
                    const T cxm = (T)amx[i], cxp = (T)apx[i], cym = (T)amy[j], cyp = (T)apy[j];
                    const T czm = (T)amz[kk], czp = (T)apz[kk];
                    T s = cxm * U[b + 1][a] + cxp * U[b + 1][a + 2];
                    s += cym * U[b][a + 1] + cyp * U[b + 2][a + 1];
                    s += czm * Um[b + 1][a + 1] + czp * Up[b + 1][a + 1];
                    const T d = cxm + cxp + cym + cyp + czm + czp;
                    uc = (s - bscale * f[(size_t)kk * sxy + (size_t)j * nx + i]) / d;
                }
                H[b][a] = uc;
            }
        }
        __syncthreads();
        const int ko = kk - 1;
        if (ko >= k0 && own) {
            T(*H)[SM_TX + 2] = Hs[(ko + 3) % 3];
            const size_t idx = (size_t)ko * sxy + (size_t)jo * nx + io;
            T out = H[ty + 1][tx + 1];
            const T fv = f[idx];
            if (((io + jo + ko) & 1) != first) {
                T(*Hm)[SM_TX + 2] = Hs[(ko + 2) % 3];
                T(*Hp)[SM_TX + 2] = Hs[(ko + 1) % 3];
                const T cxm = (T)amx[io], cxp = (T)apx[io], cym = (T)amy[jo], cyp = (T)apy[jo];
                const T czm = (T)amz[ko], czp = (T)apz[ko];
                T s = cxm * H[ty + 1][tx] + cxp * H[ty + 1][tx + 2];
                s += cym * H[ty][tx + 1] + cyp * H[ty + 2][tx + 1];
                s += czm * Hm[ty + 1][tx + 1] + czp * Hp[ty + 1][tx + 1];
                const T d = cxm + cxp + cym + cyp + czm + czp;
                out = (s - bscale * fv) / d;
            }
            uout[idx] = out;
            if (dotp) dot += L.ax[0].m[io] * L.ax[1].m[jo] * L.ax[2].m[ko] * (double)fv * (double)out;
        }
    }
    if (dotp) {
        const double t = block_sum<SM_NT>(dot, red);
        if (tid == 0) dotp[block_linear()] = t;
    }
}

static dim3 smooth_grid(const LevelView& L)
{
    return dim3((L.nx - 2 + SM_TX - 1) / SM_TX, (L.ny - 2 + SM_TY - 1) / SM_TY, (L.nz - 2 + SM_KC - 1) / SM_KC);
}

template <typename T>
hipError_t launch_smooth(const LevelView& L, const T* uin, const T* f, T* uout, T bscale, int first, int zero_in,
                         double* dot_partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_smooth<T>, smooth_grid(L), dim3(SM_NT), 0, s, L, uin, f, uout, bscale, first, zero_in,
                       dot_partials);
    return hipGetLastError();
}

int smooth_blocks(const LevelView& L)
{
    dim3 g = smooth_grid(L);
    return (int)(g.x * g.y * g.z);
}

// ------------------------------------------------- pointwise 3-D launches
constexpr int PT_X = 64, PT_Y = 4, PT_NT = PT_X * PT_Y;

static dim3 interior_grid(const LevelView& L)
{
    return dim3((L.nx - 2 + PT_X - 1) / PT_X, (L.ny - 2 + PT_Y - 1) / PT_Y, L.nz - 2);
}

int interior_blocks(const LevelView& L)
{
    dim3 g = interior_grid(L);
    return (int)(g.x * g.y * g.z);
}

template <typename T>
__device__ __forceinline__ T apply_at(const LevelView& L, const T* __restrict__ u, int i, int j, int k, size_t idx,
                                      size_t sxy, int nx)
{
    const T c = u[idx];
    T a = (T)L.ax[0].am[i] * (u[idx - 1] - c) + (T)L.ax[0].ap[i] * (u[idx + 1] - c);
    a += (T)L.ax[1].am[j] * (u[idx - nx] - c) + (T)L.ax[1].ap[j] * (u[idx + nx] - c);
    a += (T)L.ax[2].am[k] * (u[idx - sxy] - c) + (T)L.ax[2].ap[k] * (u[idx + sxy] - c);
    return a;
}

// r = bscale f - A u at interior nodes (faces of r untouched, kept zero)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_residual(LevelView L, const T* __restrict__ u, const T* __restrict__ f,
                                                    T bscale, T* __restrict__ r)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t sxy = (size_t)L.nx * L.ny;
    const size_t idx = (size_t)k * sxy + (size_t)j * L.nx + i;
    r[idx] = bscale * f[idx] - apply_at(L, u, i, j, k, idx, sxy, L.nx);
}

template <typename T>
hipError_t launch_residual(const LevelView& L, const T* u, const T* f, T bscale, T* r, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual<T>, interior_grid(L), dim3(PT_NT), 0, s, L, u, f, bscale, r);
    return hipGetLastError();
}

// r = bscale f - A u (FP64 arithmetic; u = v with faces = Dirichlet data),
// stored as T; W-norm^2 partials. interior_zero: the interior of u is read as
// zero (the reference residual of the face data alone).
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_residual_norm(LevelView L, const double* __restrict__ u,
                                                         const double* __restrict__ f, double bscale,
                                                         T* __restrict__ r, double* __restrict__ part,
                                                         int interior_zero)
{
    __shared__ double red[PT_NT / 64];
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    double acc = 0.0;
    if (i <= L.nx - 2 && j <= L.ny - 2) {
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        const size_t sxy = (size_t)nx * ny;
        const size_t idx = (size_t)k * sxy + (size_t)j * nx + i;
        double res;
        if (!interior_zero) {
            res = bscale * f[idx] - apply_at(L, u, i, j, k, idx, sxy, nx);
        } else {
            // only face neighbours carry values
            double a = 0.0;
            if (i == 1) a += L.ax[0].am[i] * u[idx - 1];
            if (i == nx - 2) a += L.ax[0].ap[i] * u[idx + 1];
            if (j == 1) a += L.ax[1].am[j] * u[idx - nx];
            if (j == ny - 2) a += L.ax[1].ap[j] * u[idx + nx];
            if (k == 1) a += L.ax[2].am[k] * u[idx - sxy];
            if (k == nz - 2) a += L.ax[2].ap[k] * u[idx + sxy];
            res = bscale * f[idx] - a;
        }
        if (r) r[idx] = (T)res;
        acc = L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] * res * res;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_residual_norm(const LevelView& L, const double* u, const double* f, double bscale, T* r,
                                double* partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_norm<T>, interior_grid(L), dim3(PT_NT), 0, s, L, u, f, bscale, r, partials, 0);
    return hipGetLastError();
}

hipError_t launch_reference_norm(const LevelView& L, const double* u, const double* f, double bscale,
                                 double* partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_norm<double>, interior_grid(L), dim3(PT_NT), 0, s, L, u, f, bscale,
                       (double*)nullptr, partials, 1);
    return hipGetLastError();
}

// q = A p and partial <p, q>_W
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_apply_dot(LevelView L, const T* __restrict__ p, T* __restrict__ q,
                                                     double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    double acc = 0.0;
    if (i <= L.nx - 2 && j <= L.ny - 2) {
        const size_t sxy = (size_t)L.nx * L.ny;
        const size_t idx = (size_t)k * sxy + (size_t)j * L.nx + i;
        const T a = apply_at(L, p, i, j, k, idx, sxy, L.nx);
        q[idx] = a;
        acc = L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] * (double)p[idx] * (double)a;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_apply_dot(const LevelView& L, const T* p, T* q, double* partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply_dot<T>, interior_grid(L), dim3(PT_NT), 0, s, L, p, q, partials);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(PT_NT) void k_dot(LevelView L, const T* __restrict__ a, const T* __restrict__ b,
                                               double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    double acc = 0.0;
    if (i <= L.nx - 2 && j <= L.ny - 2) {
        const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
        acc = L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] * (double)a[idx] * (double)b[idx];
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = t;
}

template <typename T>
hipError_t launch_dot(const LevelView& L, const T* a, const T* b, double* partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot<T>, interior_grid(L), dim3(PT_NT), 0, s, L, a, b, partials);
    return hipGetLastError();
}

// pnew = z + beta pold, beta = scal[i_num]/scal[i_den] (0 on the first step)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_update_p(LevelView L, const T* __restrict__ z, const T* __restrict__ pold,
                                                    T* __restrict__ pnew, const double* __restrict__ scal, int i_num,
                                                    int i_den, int first)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
    if (first) {
        pnew[idx] = z[idx];
    } else {
        const T beta = (T)(scal[i_num] / scal[i_den]);
        pnew[idx] = z[idx] + beta * pold[idx];
    }
}

template <typename T>
hipError_t launch_update_p(const LevelView& L, const T* z, const T* pold, T* pnew, const double* scal, int i_num,
                           int i_den, int first, hipStream_t s)
{
    hipLaunchKernelGGL(k_update_p<T>, interior_grid(L), dim3(PT_NT), 0, s, L, z, pold, pnew, scal, i_num, i_den, first);
    return hipGetLastError();
}

// x += alpha p, r -= alpha q, alpha = scal[i_num]/scal[i_den]; partial <r,r>_W.
// A non-finite alpha leaves x and r untouched (the caller then reports the
// breakdown with x still the last finite iterate).
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_update_xr(LevelView L, T* __restrict__ x, T* __restrict__ r,
                                                     const T* __restrict__ p, const T* __restrict__ q,
                                                     const double* __restrict__ scal, int i_num, int i_den,
                                                     double* __restrict__ part)
{
    __shared__ double red[PT_NT / 64];
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    const double ad = scal[i_num] / scal[i_den];
    const bool ok = isfinite(ad);
    double acc = 0.0;
    if (i <= L.nx - 2 && j <= L.ny - 2) {
        const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
        T rv = r[idx];
        if (ok) {
            const T alpha = (T)ad;
            x[idx] = x[idx] + alpha * p[idx];
            rv = rv - alpha * q[idx];
            r[idx] = rv;
        }
        acc = L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] * (double)rv * (double)rv;
    }
    const double t = block_sum<PT_NT>(acc, red);
    if (threadIdx.x == 0) part[block_linear()] = ok ? t : __builtin_nan("");
}

template <typename T>
hipError_t launch_update_xr(const LevelView& L, T* x, T* r, const T* p, const T* q, const double* scal, int i_num,
                            int i_den, double* partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_update_xr<T>, interior_grid(L), dim3(PT_NT), 0, s, L, x, r, p, q, scal, i_num, i_den, partials);
    return hipGetLastError();
}

// u += e (interior), FP32 correction into an FP64 iterate (plain V-cycle mode, FP64 e)
__global__ __launch_bounds__(PT_NT) void k_add64(LevelView L, double* __restrict__ u, const double* __restrict__ e)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
    u[idx] += e[idx];
}

hipError_t launch_add64(const LevelView& L, double* u, const double* e, hipStream_t s)
{
    hipLaunchKernelGGL(k_add64, interior_grid(L), dim3(PT_NT), 0, s, L, u, e);
    return hipGetLastError();
}

__global__ __launch_bounds__(PT_NT) void k_scale_inplace(LevelView L, double* __restrict__ u, double a)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
    u[idx] *= a;
}

hipError_t launch_scale_inplace(const LevelView& L, double* u, double a, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_inplace, interior_grid(L), dim3(PT_NT), 0, s, L, u, a);
    return hipGetLastError();
}

// r32 = r / sqrt(scal[i_norm2])  (scaled FP32 copy of the FP64 residual)
__global__ __launch_bounds__(PT_NT) void k_scale_to32(LevelView L, const double* __restrict__ r, float* __restrict__ r32,
                                                      const double* __restrict__ scal, int i_norm2)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
    const double inv = 1.0 / sqrt(scal[i_norm2]);
    r32[idx] = (float)(r[idx] * inv);
}

hipError_t launch_scale_f64_to_f32(const LevelView& L, const double* r, float* r32, const double* scal, int i_norm2,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_to32, interior_grid(L), dim3(PT_NT), 0, s, L, r, r32, scal, i_norm2);
    return hipGetLastError();
}

// u += sqrt(scal[i_norm2]) * e  (defect correction with the scaled FP32 solution)
__global__ __launch_bounds__(PT_NT) void k_add_scaled32(LevelView L, double* __restrict__ u, const float* __restrict__ e,
                                                        const double* __restrict__ scal, int i_norm2)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    const size_t idx = ((size_t)k * L.ny + j) * L.nx + i;
    const double s = sqrt(scal[i_norm2]);
    if (!isfinite(s)) return;
    u[idx] += s * (double)e[idx];
}

hipError_t launch_add_scaled_f32_to_f64(const LevelView& L, double* u, const float* e, const double* scal, int i_norm2,
                                        hipStream_t s)
{
    hipLaunchKernelGGL(k_add_scaled32, interior_grid(L), dim3(PT_NT), 0, s, L, u, e, scal, i_norm2);
    return hipGetLastError();
}

// fill the interior with zeros (a kernel rather than a memset so that a
// captured graph never records a memset node)
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_zero_interior(LevelView L, T* __restrict__ u)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > L.nx - 2 || j > L.ny - 2) return;
    u[((size_t)k * L.ny + j) * L.nx + i] = T(0);
}

template <typename T>
hipError_t launch_zero_interior(const LevelView& L, T* u, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_interior<T>, interior_grid(L), dim3(PT_NT), 0, s, L, u);
    return hipGetLastError();
}

// fill a whole array (n elements) with zeros
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
// rc(I,J,K) = sum over the up-to-3x3x3 fine nodes around (rf[I],rf[J],rf[K])
// of rw_x rw_y rw_z r: the restriction M_c^-1 P^T M_f, adjoint of the
// interpolation in the volume-weighted inner product.
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_restrict(LevelView F, LevelView C, const T* __restrict__ r,
                                                    T* __restrict__ rc)
{
    const int I = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int J = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int K = 1 + blockIdx.z;
    if (I > C.nx - 2 || J > C.ny - 2) return;
    const int fi = C.ax[0].rf[I], fj = C.ax[1].rf[J], fk = C.ax[2].rf[K];
    const double* wx = C.ax[0].rw + 3 * I;
    const double* wy = C.ax[1].rw + 3 * J;
    const double* wz = C.ax[2].rw + 3 * K;
    const size_t sxy = (size_t)F.nx * F.ny;
    T acc = T(0);
    for (int c = 0; c < 3; ++c) {
        const T z = (T)wz[c];
        if (z == T(0)) continue;
        for (int b = 0; b < 3; ++b) {
            const T y = (T)wy[b];
            if (y == T(0)) continue;
            const T* row = r + (size_t)(fk - 1 + c) * sxy + (size_t)(fj - 1 + b) * F.nx + (fi - 1);
            const T sx = (T)wx[0] * row[0] + (T)wx[1] * row[1] + (T)wx[2] * row[2];
            acc += z * y * sx;
        }
    }
    rc[((size_t)K * C.ny + J) * C.nx + I] = acc;
}

template <typename T>
hipError_t launch_restrict(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s)
{
    hipLaunchKernelGGL(k_restrict<T>, interior_grid(C), dim3(PT_NT), 0, s, F, C, r, rc);
    return hipGetLastError();
}

// u(i,j,k) += sum of the 2x2x2 coarse values around it times the linear
// interpolation weights in physical coordinates (weight 1 at kept nodes).
template <typename T>
__global__ __launch_bounds__(PT_NT) void k_prolong_add(LevelView F, LevelView C, const T* __restrict__ e,
                                                       T* __restrict__ u)
{
    const int i = 1 + blockIdx.x * PT_X + (threadIdx.x % PT_X);
    const int j = 1 + blockIdx.y * PT_Y + (threadIdx.x / PT_X);
    const int k = 1 + blockIdx.z;
    if (i > F.nx - 2 || j > F.ny - 2) return;
    const int I = C.ax[0].pc[i], J = C.ax[1].pc[j], K = C.ax[2].pc[k];
    const T x0 = (T)C.ax[0].pw[2 * i], x1 = (T)C.ax[0].pw[2 * i + 1];
    const T y0 = (T)C.ax[1].pw[2 * j], y1 = (T)C.ax[1].pw[2 * j + 1];
    const T z0 = (T)C.ax[2].pw[2 * k], z1 = (T)C.ax[2].pw[2 * k + 1];
    const size_t csxy = (size_t)C.nx * C.ny;
    const T* e0 = e + (size_t)K * csxy + (size_t)J * C.nx + I;
    // neighbours with zero weight may sit one past the last coarse node:
    // read them only when the weight is nonzero
    T a = x0 * e0[0];
    if (x1 != T(0)) a += x1 * e0[1];
    T v = y0 * a;
    if (y1 != T(0)) {
        T b = x0 * e0[C.nx];
        if (x1 != T(0)) b += x1 * e0[C.nx + 1];
        v += y1 * b;
    }
    T w = z0 * v;
    if (z1 != T(0)) {
        const T* e1 = e0 + csxy;
        T a2 = x0 * e1[0];
        if (x1 != T(0)) a2 += x1 * e1[1];
        T v2 = y0 * a2;
        if (y1 != T(0)) {
            T b2 = x0 * e1[C.nx];
            if (x1 != T(0)) b2 += x1 * e1[C.nx + 1];
            v2 += y1 * b2;
        }
        w += z1 * v2;
    }
    const size_t idx = ((size_t)k * F.ny + j) * F.nx + i;
    u[idx] += w;
}

template <typename T>
hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s)
{
    hipLaunchKernelGGL(k_prolong_add<T>, interior_grid(F), dim3(PT_NT), 0, s, F, C, e, u);
    return hipGetLastError();
}

// --------------------------------------------------------- coarsest level
// One workgroup: `sweeps` red-black sweeps (red, black) then `sweeps` in the
// reverse order (black, red), from zero, in LDS; symmetric, so the V-cycle
// stays a symmetric preconditioner. At most 4096 nodes.
constexpr int CS_MAX = 4096;

template <typename T>
__global__ __launch_bounds__(256) void k_coarse(LevelView L, T* __restrict__ u, const T* __restrict__ f, int sweeps)
{
    __shared__ T us[CS_MAX];
    __shared__ T fs[CS_MAX];
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int n = nx * ny * nz;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        us[t] = T(0);
        fs[t] = f[t];
    }
    __syncthreads();
    for (int pass = 0; pass < 2 * sweeps; ++pass) {
        for (int half = 0; half < 2; ++half) {
            const int colour = (pass < sweeps) ? half : 1 - half;
            for (int t = threadIdx.x; t < n; t += blockDim.x) {
                const int i = t % nx, j = (t / nx) % ny, k = t / (nx * ny);
                if (i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1) continue;
                if (((i + j + k) & 1) != colour) continue;
                const T cxm = (T)L.ax[0].am[i], cxp = (T)L.ax[0].ap[i];
                const T cym = (T)L.ax[1].am[j], cyp = (T)L.ax[1].ap[j];
                const T czm = (T)L.ax[2].am[k], czp = (T)L.ax[2].ap[k];
                T s = cxm * us[t - 1] + cxp * us[t + 1];
                s += cym * us[t - nx] + cyp * us[t + nx];
                s += czm * us[t - nx * ny] + czp * us[t + nx * ny];
                us[t] = (s - fs[t]) / (cxm + cxp + cym + cyp + czm + czp);
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < n; t += blockDim.x) u[t] = us[t];
}

template <typename T>
hipError_t launch_coarse_solve(const LevelView& L, T* u, const T* f, int sweeps, hipStream_t s)
{
    if ((size_t)L.nx * L.ny * L.nz > (size_t)CS_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(256), 0, s, L, u, f, sweeps);
    return hipGetLastError();
}

// ------------------------------------------------------------ reduction
// out[c] = sum_b partials[b * stride + c] for c < stride... here stride 1:
// out[0] = sum of count partials in a fixed order (thread t takes t, t+1024,
// ..., then a fixed tree), so a given launch shape always gives the same bits.
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
#define INST(T)                                                                                               \
    template hipError_t launch_smooth<T>(const LevelView&, const T*, const T*, T*, T, int, int, double*,         \
                                         hipStream_t);                                                         \
    template hipError_t launch_residual<T>(const LevelView&, const T*, const T*, T, T*, hipStream_t);           \
    template hipError_t launch_restrict<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);      \
    template hipError_t launch_prolong_add<T>(const LevelView&, const LevelView&, const T*, T*, hipStream_t);   \
    template hipError_t launch_coarse_solve<T>(const LevelView&, T*, const T*, int, hipStream_t);               \
    template hipError_t launch_apply_dot<T>(const LevelView&, const T*, T*, double*, hipStream_t);              \
    template hipError_t launch_residual_norm<T>(const LevelView&, const double*, const double*, double, T*,     \
                                                double*, hipStream_t);                                         \
    template hipError_t launch_dot<T>(const LevelView&, const T*, const T*, double*, hipStream_t);              \
    template hipError_t launch_update_p<T>(const LevelView&, const T*, const T*, T*, const double*, int, int,   \
                                           int, hipStream_t);                                                  \
    template hipError_t launch_update_xr<T>(const LevelView&, T*, T*, const T*, const T*, const double*, int,   \
                                            int, double*, hipStream_t);                                        \
    template hipError_t launch_zero_interior<T>(const LevelView&, T*, hipStream_t);                             \
    template hipError_t launch_fill_zero<T>(T*, size_t, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace lasto

namespace lasto {
template hipError_t launch_fill_zero<unsigned char>(unsigned char*, size_t, hipStream_t);
}  // namespace lasto
