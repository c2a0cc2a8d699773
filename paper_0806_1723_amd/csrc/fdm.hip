// Fast diagonalisation: a direct solve of the discrete eq. (3.2) on the
// tensor-product mesh.
//
// The 7-point operator is a Kronecker sum A = A_z (+) A_y (+) A_x of 1-D
// three-point operators A_d = M_d^-1 T_d (T_d symmetric tridiagonal with
// off-diagonals 1/h, M_d the dual widths). Each A_d = S_d L_d S_d^-1 with
// S_d = M_d^-1/2 Q_d, S_d^-1 = Q_d^T M_d^1/2, where Q_d L_d Q_d^T is the
// eigen-decomposition of the symmetric M_d^-1/2 T_d M_d^-1/2. The interior
// solution of A u = b is then
//   u = (S_z x S_y x S_x) [ (S_z^-1 x S_y^-1 x S_x^-1) b / (l_z + l_y + l_x) ],
// three dense contractions along the axes, a division, three more: about
// 12 n^4 flops on the FP64 matrix cores (rocBLAS GEMMs) where a multigrid
// cycle is bandwidth-bound, and exact up to rounding. b is the residual of
// the face data, 4 pi rho - A v_bc; the result fills the interior of v.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"
#include "internal.h"

namespace lasto {

struct FdmState {
    int m[3] = {0, 0, 0};                          // interior nodes per axis (one copy)
    double* S[3] = {nullptr, nullptr, nullptr};    // device [m][m] row-major
    double* Si[3] = {nullptr, nullptr, nullptr};   // device inverses
    double* lam[3] = {nullptr, nullptr, nullptr};  // device eigenvalues
    double* buf[2] = {nullptr, nullptr};           // device [mz][my][mx]
    rocblas_handle blas = nullptr;
};

void free_fdm(lasto_grid g)
{
    FdmState* f = g->fdm;
    if (!f) return;
    for (int d = 0; d < 3; ++d) {
        (void)hipFree(f->S[d]);
        (void)hipFree(f->Si[d]);
        (void)hipFree(f->lam[d]);
    }
    (void)hipFree(f->buf[0]);
    (void)hipFree(f->buf[1]);
    if (f->blas) (void)rocblas_destroy_handle(f->blas);
    delete f;
    g->fdm = nullptr;
}

// ------------------------------------------------------------------ kernels
// b = bscale rho - A v_bc at the interior nodes, packed [mz][my][mx]: with a
// zero interior only face neighbours contribute
__global__ __launch_bounds__(256) void k_fdm_rhs(LevelView L, const double* __restrict__ v,
                                                 const double* __restrict__ rho, double bscale, double* __restrict__ b)
{
    const int mx = L.nx - 2, my = L.ny - 2, mz = L.nz - 2;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)mx * my * mz) return;
    const int i = (int)(t % mx) + 1;
    const size_t rest = t / mx;
    const int j = (int)(rest % my) + 1, k = (int)(rest / my) + 1;
    const size_t plane = (size_t)L.nx * L.ny;
    const size_t at = (size_t)k * plane + (size_t)j * L.nx + i;
    double s = bscale * rho[at];
    if (i == 1) s -= L.ax[0].am[i] * v[at - 1];
    if (i == L.nx - 2) s -= L.ax[0].ap[i] * v[at + 1];
    if (j == 1) s -= L.ax[1].am[j] * v[at - L.nx];
    if (j == L.ny - 2) s -= L.ax[1].ap[j] * v[at + L.nx];
    if (k == 1) s -= L.ax[2].am[k] * v[at - plane];
    if (k == L.nz - 2) s -= L.ax[2].ap[k] * v[at + plane];
    b[t] = s;
}

// u /= l_z[k] + l_y[j] + l_x[i] in the eigenbasis
__global__ __launch_bounds__(256) void k_fdm_divide(double* __restrict__ u, const double* __restrict__ lx,
                                                    const double* __restrict__ ly, const double* __restrict__ lz,
                                                    int mx, int my, int mz)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)mx * my * mz) return;
    const int i = (int)(t % mx);
    const size_t rest = t / mx;
    const int j = (int)(rest % my), k = (int)(rest / my);
    u[t] = u[t] / (lz[k] + ly[j] + lx[i]);
}

// interior of v from the packed solution
__global__ __launch_bounds__(256) void k_fdm_unpack(LevelView L, const double* __restrict__ u, double* __restrict__ v)
{
    const int mx = L.nx - 2, my = L.ny - 2, mz = L.nz - 2;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)mx * my * mz) return;
    const int i = (int)(t % mx) + 1;
    const size_t rest = t / mx;
    const int j = (int)(rest % my) + 1, k = (int)(rest / my) + 1;
    v[((size_t)k * L.ny + j) * L.nx + i] = u[t];
}

static lasto_status fdm_init(lasto_grid g)
{
    if (g->fdm) return LASTO_OK;
    const LevelView& V = g->cview;
    const int n[3] = {V.nx, V.ny, V.nz};
    FdmState* f = new FdmState;
    g->fdm = f;
    for (int d = 0; d < 3; ++d) {
        const int m = n[d] - 2;
        f->m[d] = m;
        std::vector<double> lam(m), S((size_t)m * m), Si((size_t)m * m);
        if (!axis_decomposition(g->lev[0].hx[d].data(), n[d], lam.data(), S.data(), Si.data())) {
            free_fdm(g);
            return fail(LASTO_ERR_STATE, "lasto_fdm_solve: the 1-D eigen-decomposition did not converge");
        }
        if (hipMalloc(&f->S[d], sizeof(double) * m * m) != hipSuccess ||
            hipMalloc(&f->Si[d], sizeof(double) * m * m) != hipSuccess ||
            hipMalloc(&f->lam[d], sizeof(double) * m) != hipSuccess) {
            free_fdm(g);
            return fail(LASTO_ERR_ALLOC, "lasto_fdm_solve: tables");
        }
        hipError_t e = hipMemcpy(f->S[d], S.data(), sizeof(double) * m * m, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(f->Si[d], Si.data(), sizeof(double) * m * m, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(f->lam[d], lam.data(), sizeof(double) * m, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_fdm(g);
            return fail(LASTO_ERR_HIP, std::string("lasto_fdm_solve: ") + hipGetErrorString(e));
        }
    }
    const size_t cells = (size_t)f->m[0] * f->m[1] * f->m[2];
    if (hipMalloc(&f->buf[0], sizeof(double) * cells) != hipSuccess ||
        hipMalloc(&f->buf[1], sizeof(double) * cells) != hipSuccess) {
        free_fdm(g);
        return fail(LASTO_ERR_ALLOC, "lasto_fdm_solve: work arrays");
    }
    if (rocblas_create_handle(&f->blas) != rocblas_status_success ||
        rocblas_set_stream(f->blas, g->stream) != rocblas_status_success) {
        free_fdm(g);
        return fail(LASTO_ERR_HIP, "lasto_fdm_solve: rocBLAS handle");
    }
    return LASTO_OK;
}

// out[r][line] = sum_k P[r][k] in[line][k] for the m = f->m[d] entries of
// each line of the packed interior (axis d fastest): the new axis is written
// slowest, so column-major this is one GEMM, C (L x m) = A^T B, with A the
// input (m x L) and B the row-major P read as column-major. Contracting x, y,
// z in turn takes [z][y][x] to [x'][z][y], [y'][x'][z] and [z'][y'][x'] (the
// original order); the same three steps take it back.
static rocblas_status contract(FdmState* f, int d, const double* P, const double* in, double* out)
{
    const int m = f->m[d];
    const int L = f->m[0] * f->m[1] * f->m[2] / m;
    const double one = 1.0, zero = 0.0;
    return rocblas_dgemm(f->blas, rocblas_operation_transpose, rocblas_operation_none, L, m, m, &one, in, m, P, m,
                         &zero, out, L);
}

// ---------------------------------------------- coarsest solve of the cycle
// The multigrid cycle's correction equation A e = f (zero faces) at one small
// level, solved exactly by the same diagonalisation in one workgroup. The
// level's interior is copied from the split layout into a dense
// [copy][z][y][x] block in LDS, with the axis tables beside it (copied in
// once per call: the large sweeps between calls evict them from the caches).
// Each contraction step gives one thread one grid line, held in registers,
// which it replaces by the line times an axis matrix, two rows at a time
// (each pair read into registers by 16-byte LDS reads before its products);
// every lane of a wave reads the same matrix entry, an LDS broadcast. Rows are
// padded with zeros to MX entries. All six contractions run through one
// rolled loop over the same code, so a call fetches a few KB of instructions
// rather than a fully unrolled pass each (the code runs once per call, from a
// cold instruction cache). A batched level solves each copy on its own
// planes with the same z tables.
// lanes of the workgroup (a line and two matrix rows in registers need more
// than the 128 registers per lane that 1024 lanes allow)
constexpr int CF_NT = 512;

// element offsets of each axis's blocks in the table: S^-1 [m][MX],
// S [m][MX], eigenvalues [m], each block starting on a multiple of 4
struct CfTab {
    int si[3], s[3], lam[3];
    int total;
};

static CfTab cf_layout(const int m[3], int MX)
{
    CfTab t{};
    int o = 0;
    auto take = [&](int n) {
        const int at = o;
        o += (n + 3) & ~3;
        return at;
    };
    for (int d = 0; d < 3; ++d) {
        t.si[d] = take(m[d] * MX);
        t.s[d] = take(m[d] * MX);
        t.lam[d] = take(m[d]);
    }
    t.total = o;
    return t;
}

template <typename T> struct CfVec;
template <> struct CfVec<float> { using type = float4; };
template <> struct CfVec<double> { using type = double2; };

// row[0..MX) into registers by 16-byte LDS reads, all issued before use
template <typename T, int MX>
__device__ __forceinline__ void cf_load_row(const T* row, T (&a)[MX])
{
    using V = typename CfVec<T>::type;
    constexpr int E = 16 / sizeof(T);
#pragma unroll
    for (int i = 0; i < MX; i += E) *reinterpret_cast<V*>(&a[i]) = *reinterpret_cast<const V*>(row + i);
}

// rows r and r + 1 of a matrix (row points at row r) times the register line v
template <typename T, int MX>
__device__ __forceinline__ void cf_rows2(const T* row, const T (&v)[MX], T& y0, T& y1)
{
    T a[MX], b[MX];
    cf_load_row<T, MX>(row, a);
    cf_load_row<T, MX>(row + MX, b);
    T a0 = T(0), a1 = T(0), b0 = T(0), b1 = T(0);
#pragma unroll
    for (int i = 0; i < MX; i += 2) {
        a0 = fma(a[i], v[i], a0);
        a1 = fma(a[i + 1], v[i + 1], a1);
        b0 = fma(b[i], v[i], b0);
        b1 = fma(b[i + 1], v[i + 1], b1);
    }
    y0 = a0 + a1;
    y1 = b0 + b1;
}

template <typename T, int MX>
__device__ __forceinline__ T cf_row(const T* row, const T (&v)[MX])
{
    T a[MX];
    cf_load_row<T, MX>(row, a);
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int i = 0; i < MX; i += 2) {
        a0 = fma(a[i], v[i], a0);
        a1 = fma(a[i + 1], v[i + 1], a1);
    }
    return a0 + a1;
}

// dense block index t (x fastest, copies stacked in z) -> split-layout index
__device__ __forceinline__ size_t cf_split(const LevelView& V, int t, int mx, int my, int mz)
{
    const int i = t % mx, r = t / mx;
    const int j = r % my, kb = r / my;
    return sidx(V, i + 1, j + 1, (kb / mz) * V.nzc + 1 + kb % mz);
}

template <typename T, int MX>
__global__ __launch_bounds__(CF_NT) void k_coarse_fdm(LevelView V, const T* __restrict__ f, T* __restrict__ u,
                                                      const T* __restrict__ tab, CfTab tl)
{
    extern __shared__ unsigned char cf_smem[];
    const int mx = V.nx - 2, my = V.ny - 2, mz = V.nzc - 2, nb = V.nz / V.nzc;
    const int pxy = mx * my, pc = pxy * mz;   // nodes of a plane, of a copy
    const int n = pc * nb;
    T* w = reinterpret_cast<T*>(cf_smem);
    T* tb = w + ((n + 3) & ~3);
    // tables and f into LDS, eight loads in flight per lane
    for (int t0 = 0; t0 < tl.total; t0 += 8 * CF_NT) {
        T tmp[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int t = t0 + b * CF_NT + (int)threadIdx.x;
            tmp[b] = t < tl.total ? tab[t] : T(0);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int t = t0 + b * CF_NT + (int)threadIdx.x;
            if (t < tl.total) tb[t] = tmp[b];
        }
    }
    for (int t0 = 0; t0 < n; t0 += 8 * CF_NT) {
        T tmp[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int t = t0 + b * CF_NT + (int)threadIdx.x;
            tmp[b] = t < n ? f[cf_split(V, t, mx, my, mz)] : T(0);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int t = t0 + b * CF_NT + (int)threadIdx.x;
            if (t < n) w[t] = tmp[b];
        }
    }
    __syncthreads();
    // Seven steps on the block: S_x^-1, S_y^-1, S_z^-1, the division, S_z,
    // S_y, S_x. A line of axis d starts at (line / A) B + (line % A) C with
    // stride st: x lines (A, B, C, st) = (my, pxy, mx, 1), y lines
    // (mx, pxy, 1, mx), z lines (pxy, pc, 1, pxy). A lane owns its line
    // for the step, so it may overwrite it in place.
    T v[MX];
    for (int step = 0; step < 7; ++step) {
        if (step == 3) {
            for (int t = threadIdx.x; t < n; t += CF_NT) {
                const int i = t % mx, r = t / mx;
                w[t] = w[t] / (tb[tl.lam[0] + i] + tb[tl.lam[1] + r % my] + tb[tl.lam[2] + (r / my) % mz]);
            }
        } else {
            const int d = step < 3 ? step : 6 - step;
            const T* M = tb + (step < 3 ? tl.si[d] : tl.s[d]);
            const int m = d == 0 ? mx : d == 1 ? my : mz;
            const int A = d == 0 ? my : d == 1 ? mx : pxy;
            const int B = d == 2 ? pc : pxy;
            const int C = d == 0 ? mx : 1;
            const int st = d == 0 ? 1 : d == 1 ? mx : pxy;
            for (int line = threadIdx.x; line < n / m; line += CF_NT) {
                T* base = w + (line / A) * B + (line % A) * C;
#pragma unroll
                for (int k = 0; k < MX; ++k) v[k] = k < m ? base[k * st] : T(0);
                int r = 0;
                for (; r + 1 < m; r += 2) {
                    T y0, y1;
                    cf_rows2<T, MX>(M + r * MX, v, y0, y1);
                    base[r * st] = y0;
                    base[(r + 1) * st] = y1;
                }
                if (r < m) base[r * st] = cf_row<T, MX>(M + r * MX, v);
            }
        }
        __syncthreads();
    }
    // the block into e
    for (int t = threadIdx.x; t < n; t += CF_NT) u[cf_split(V, t, mx, my, mz)] = w[t];
}

template <typename T, int MX>
static hipError_t cf_allow_lds(int bytes)
{
    return hipFuncSetAttribute((const void*)k_coarse_fdm<T, MX>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

static size_t cf_lds_bytes(size_t elem, const int m[3], int nb, const CfTab& tl)
{
    const size_t cells = ((size_t)m[0] * m[1] * m[2] * nb + 3) & ~(size_t)3;
    return elem * (cells + tl.total);
}

lasto_status build_coarse_fdm(lasto_grid g)
{
    g->cfdm_level = -1;
    const int t = g->tail_top;
    if (t < 1) return LASTO_OK;   // at the finest level the cycle would be the direct solve itself
    const Level& L = g->lev[t];
    int m[3], mmax = 0;
    for (int d = 0; d < 3; ++d) {
        m[d] = L.n[d] - 2;
        if (m[d] < 1) return LASTO_OK;
        mmax = std::max(mmax, m[d]);
    }
    if (mmax > 32) return LASTO_OK;   // (a line of at most 32 in registers)
    const int MX = mmax <= 16 ? 16 : 32;
    const CfTab tl = cf_layout(m, MX);
    const int lim = tail_lds_limit();
    if (lim <= 0 || cf_lds_bytes(sizeof(double), m, g->n_batch, tl) > (size_t)lim) return LASTO_OK;
    std::vector<double> tab((size_t)tl.total, 0.0);
    for (int d = 0; d < 3; ++d) {
        const int n = m[d];
        std::vector<double> lam(n), S((size_t)n * n), Si((size_t)n * n);
        if (!axis_decomposition(L.hx[d].data(), L.n[d], lam.data(), S.data(), Si.data()))
            return fail(LASTO_ERR_STATE, "lasto_grid_create: coarse-level eigen-decomposition did not converge");
        for (int r = 0; r < n; ++r) {
            for (int c = 0; c < n; ++c) {
                tab[tl.si[d] + (size_t)r * MX + c] = Si[(size_t)r * n + c];
                tab[tl.s[d] + (size_t)r * MX + c] = S[(size_t)r * n + c];
            }
            tab[tl.lam[d] + r] = lam[r];
        }
    }
    std::vector<float> tabf(tab.begin(), tab.end());
    hipError_t e = hipSuccess;
    switch (MX) {
        case 16: e = cf_allow_lds<double, 16>(lim); if (e == hipSuccess) e = cf_allow_lds<float, 16>(lim); break;
        default: e = cf_allow_lds<double, 32>(lim); if (e == hipSuccess) e = cf_allow_lds<float, 32>(lim); break;
    }
    if (e == hipSuccess) e = hipMalloc(&g->cfdm_tab64, sizeof(double) * tab.size());
    if (e == hipSuccess) e = hipMalloc(&g->cfdm_tab32, sizeof(float) * tabf.size());
    if (e == hipSuccess) e = hipMemcpy(g->cfdm_tab64, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->cfdm_tab32, tabf.data(), sizeof(float) * tabf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(LASTO_ERR_HIP, std::string("lasto_grid_create: coarse tables: ") + hipGetErrorString(e));
    g->cfdm_level = t;
    g->cfdm_mx = MX;
    return LASTO_OK;
}

void free_coarse_fdm(lasto_grid g)
{
    (void)hipFree(g->cfdm_tab64);
    (void)hipFree(g->cfdm_tab32);
    g->cfdm_tab64 = nullptr;
    g->cfdm_tab32 = nullptr;
    g->cfdm_level = -1;
}

template <typename T>
hipError_t launch_coarse_fdm(lasto_grid g, const T* f, T* u, hipStream_t s)
{
    const Level& L = g->lev[g->cfdm_level];
    const LevelView& V = L.view;
    const T* tab = sizeof(T) == 8 ? (const T*)g->cfdm_tab64 : (const T*)g->cfdm_tab32;
    const int m[3] = {L.n[0] - 2, L.n[1] - 2, L.n[2] - 2};
    const CfTab tl = cf_layout(m, g->cfdm_mx);
    const size_t lds = cf_lds_bytes(sizeof(T), m, g->n_batch, tl);
    switch (g->cfdm_mx) {
        case 16: hipLaunchKernelGGL((k_coarse_fdm<T, 16>), dim3(1), dim3(CF_NT), lds, s, V, f, u, tab, tl); break;
        default: hipLaunchKernelGGL((k_coarse_fdm<T, 32>), dim3(1), dim3(CF_NT), lds, s, V, f, u, tab, tl); break;
    }
    return hipGetLastError();
}
template hipError_t launch_coarse_fdm<double>(lasto_grid, const double*, double*, hipStream_t);
template hipError_t launch_coarse_fdm<float>(lasto_grid, const float*, float*, hipStream_t);

// ------------------------------------ coarsest solve by GEMMs (a larger level)
// The same exact solve on a level of up to kGemmCoarseMaxPts nodes per copy
// (90^3 under the 257^3 mesh), where the block no longer fits in LDS: the
// level's interior is packed into a dense [copy][z][y][x] array, contracted
// along x, y, z by rocBLAS GEMMs in the cycle's precision (each a single
// GEMM per copy: the axes rotate, see contract_rot), divided by the
// eigenvalue sums, contracted back and unpacked. Below that level nothing
// runs, so the launch-bound sweeps and transfers of the small levels are
// replaced by nine launches. rocBLAS runs with atomics off (fixed summation
// order, so repeated solves give the same bits).
struct CoarseGemm {
    int m[3] = {0, 0, 0};
    int nb = 1;
    double* S64[3] = {nullptr, nullptr, nullptr};
    double* Si64[3] = {nullptr, nullptr, nullptr};
    double* lam64[3] = {nullptr, nullptr, nullptr};
    float* S32[3] = {nullptr, nullptr, nullptr};
    float* Si32[3] = {nullptr, nullptr, nullptr};
    float* lam32[3] = {nullptr, nullptr, nullptr};
    double* buf64[2] = {nullptr, nullptr};
    float* buf32[2] = {nullptr, nullptr};
    rocblas_handle blas = nullptr;   // the FP32 contractions
};

void free_coarse_gemm(lasto_grid g)
{
    CoarseGemm* c = g->cg;
    if (!c) return;
    for (int d = 0; d < 3; ++d) {
        (void)hipFree(c->S64[d]);
        (void)hipFree(c->Si64[d]);
        (void)hipFree(c->lam64[d]);
        (void)hipFree(c->S32[d]);
        (void)hipFree(c->Si32[d]);
        (void)hipFree(c->lam32[d]);
    }
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(c->buf64[b]);
        (void)hipFree(c->buf32[b]);
    }
    if (c->blas) (void)rocblas_destroy_handle(c->blas);
    delete c;
    g->cg = nullptr;
}

// the level the GEMM solve would take (set at grid creation; -1: none). It
// must lie below the finest level and above the LDS solve's level.
void choose_coarse_gemm_level(lasto_grid g)
{
    g->cg_level = -1;
    for (int l = 1; l < g->nlev; ++l) {
        const Level& L = g->lev[l];
        const size_t per_copy = (size_t)L.n[0] * L.n[1] * L.n[2];
        if (per_copy > kGemmCoarseMaxPts) continue;
        if (L.npts > kTailMaxPts && L.n[0] >= 3 && L.n[1] >= 3 && L.n[2] >= 3) g->cg_level = l;
        return;
    }
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<double>& src)
{
    std::vector<T> h(src.begin(), src.end());
    hipError_t e = hipMalloc(dst, sizeof(T) * h.size());
    if (e == hipSuccess) e = hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    return e;
}

lasto_status coarse_gemm_init(lasto_grid g)
{
    if (g->cg || g->cg_level < 0) return LASTO_OK;
    const Level& L = g->lev[g->cg_level];
    CoarseGemm* c = new CoarseGemm;
    g->cg = c;
    c->nb = g->n_batch;
    hipError_t e = hipSuccess;
    for (int d = 0; d < 3 && e == hipSuccess; ++d) {
        const int m = L.n[d] - 2;
        c->m[d] = m;
        std::vector<double> lam(m), S((size_t)m * m), Si((size_t)m * m);
        if (!axis_decomposition(L.hx[d].data(), L.n[d], lam.data(), S.data(), Si.data())) {
            free_coarse_gemm(g);
            return fail(LASTO_ERR_STATE, "lasto_poisson_solve: coarse-level eigen-decomposition did not converge");
        }
        e = upload(&c->S64[d], S);
        if (e == hipSuccess) e = upload(&c->Si64[d], Si);
        if (e == hipSuccess) e = upload(&c->lam64[d], lam);
        if (e == hipSuccess) e = upload(&c->S32[d], S);
        if (e == hipSuccess) e = upload(&c->Si32[d], Si);
        if (e == hipSuccess) e = upload(&c->lam32[d], lam);
    }
    const size_t cells = (size_t)c->m[0] * c->m[1] * c->m[2] * c->nb;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipMalloc(&c->buf64[b], sizeof(double) * cells);
        if (e == hipSuccess) e = hipMalloc(&c->buf32[b], sizeof(float) * cells);
    }
    if (e != hipSuccess) {
        free_coarse_gemm(g);
        return fail(LASTO_ERR_ALLOC, std::string("lasto_poisson_solve: coarse-level tables: ") + hipGetErrorString(e));
    }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success ||
        rocblas_set_stream(c->blas, g->stream) != rocblas_status_success ||
        rocblas_set_atomics_mode(c->blas, rocblas_atomics_not_allowed) != rocblas_status_success) {
        free_coarse_gemm(g);
        return fail(LASTO_ERR_HIP, "lasto_poisson_solve: rocBLAS handle");
    }
    return LASTO_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void k_split_to_dense(LevelView V, const T* __restrict__ a, T* __restrict__ d)
{
    const int mx = V.nx - 2, my = V.ny - 2, mz = V.nzc - 2;
    const int n = mx * my * mz * (V.nz / V.nzc);
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) d[t] = a[cf_split(V, t, mx, my, mz)];
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_to_split(LevelView V, const T* __restrict__ d, T* __restrict__ a)
{
    const int mx = V.nx - 2, my = V.ny - 2, mz = V.nzc - 2;
    const int n = mx * my * mz * (V.nz / V.nzc);
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < n) a[cf_split(V, t, mx, my, mz)] = d[t];
}

template <typename T>
__global__ __launch_bounds__(256) void k_divide_dense(T* __restrict__ d, const T* __restrict__ lx,
                                                      const T* __restrict__ ly, const T* __restrict__ lz, int mx,
                                                      int my, int mz, int n)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const int i = t % mx, r = t / mx;
    d[t] = d[t] / (lx[i] + ly[r % my] + lz[(r / my) % mz]);
}

// One contraction with the axes rotated, on the matrix cores: each copy's
// block holds L = cells / m lines of m contiguous entries ([line][k], the
// contracted axis fastest); the output is out[r][line] = sum_k P[r][k]
// in[line][k], the new axis slowest. Three of them take [z][y][x] to
// [x'][z][y], [y'][x'][z] and [z'][y'][x'] (the original order), three more
// back to [z][y][x]. Each wave computes one 16 x 16 tile (16 rows r by 16
// lines) by 16 x 16 x 4 matrix-core steps in the cycle's precision
// (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32): A 16 x 4 from lane
// (row = lane % 16, k-slot = lane / 16), B 4 x 16 from lane (k-slot =
// lane / 16, col = lane % 16). The k axis is taken in chunks of 16 in a
// permuted order so that each lane reads four consecutive entries of its row
// of P and of its line at once: in chunk c, step s, lane group g holds
// k = 16 c + 4 g + s (the four steps of a chunk cover its 16 k once, A and B
// alike). Both operands come straight from memory (P stays in the L2; each
// lane's line is a contiguous run); for m <= 16 NCH every load of the whole
// k range is issued before the first matrix-core step. The summation order
// is fixed: the same bits every time.
constexpr int CT_NT = 256;
typedef double ct_dbl4 __attribute__((ext_vector_type(4)));
typedef float ct_flt4 __attribute__((ext_vector_type(4)));

template <typename T> struct CtMfma;
template <> struct CtMfma<double> {
    typedef ct_dbl4 Acc;
    static __device__ __forceinline__ Acc step(double a, double b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // lane l holds rows l / 16 + 4 j of column l % 16
    static __device__ __forceinline__ int row(int grp, int j) { return grp + 4 * j; }
};
template <> struct CtMfma<float> {
    typedef ct_flt4 Acc;
    static __device__ __forceinline__ Acc step(float a, float b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // lane l holds rows 4 (l / 16) + j of column l % 16
    static __device__ __forceinline__ int row(int grp, int j) { return 4 * grp + j; }
};

// four consecutive entries p[k .. k + 3] (zero past n), one load when all are in range
template <typename T>
__device__ __forceinline__ void ct_load4(const T* __restrict__ p, int k, int n, bool ok, T* v)
{
    if (ok && k + 3 < n) {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = p[k + s];
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = (ok && k + s < n) ? p[k + s] : T(0);
    }
}

template <typename T, int NCH, int RT>
__global__ __launch_bounds__(CT_NT) void k_contract(const T* __restrict__ P, const T* __restrict__ in,
                                                    T* __restrict__ out, int m, int L, int rtiles, int ctiles)
{
    typedef typename CtMfma<T>::Acc Acc;
    constexpr int NC = NCH > 0 ? NCH : 2;   // 16-k chunks held in registers at once
    const int lane = threadIdx.x & 63;
    // (column tile, group of RT row tiles) of copy blockIdx.y: the wave's
    // line operands are loaded once for its RT row tiles
    const int task = blockIdx.x * (CT_NT / 64) + (threadIdx.x >> 6);
    const int rgroups = (rtiles + RT - 1) / RT;
    if (task >= rgroups * ctiles) return;   // the last workgroup's spare waves
    const int rg = task % rgroups, ct = task / rgroups;
    const int p16 = lane & 15, grp = lane >> 4;
    const size_t per = (size_t)m * L;
    const T* __restrict__ inc = in + blockIdx.y * per;
    T* __restrict__ outc = out + blockIdx.y * per;
    const int ln = ct * 16 + p16;
    const bool lok = ln < L;
    const T* __restrict__ il = inc + (size_t)(lok ? ln : 0) * m;
    Acc acc[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) acc[q] = Acc{T(0), T(0), T(0), T(0)};
    const int kend = NCH > 0 ? 16 * NC : m;
    for (int k0 = 0; k0 < kend; k0 += 16 * NC) {
        T bv[NC][4];
#pragma unroll
        for (int c = 0; c < NC; ++c) ct_load4(il, k0 + 16 * c + 4 * grp, m, lok, bv[c]);
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const int r = (rg * RT + q) * 16 + p16;
            const bool rok = r < m;
            const T* __restrict__ prow = P + (size_t)(rok ? r : 0) * m;
            T a[NC][4];
#pragma unroll
            for (int c = 0; c < NC; ++c) ct_load4(prow, k0 + 16 * c + 4 * grp, m, rok, a[c]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int st = 0; st < 4; ++st) acc[q] = CtMfma<T>::step(a[c][st], bv[c][st], acc[q]);
        }
    }
    if (!lok) return;
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = (rg * RT + q) * 16 + CtMfma<T>::row(grp, j);
            if (row < m) outc[(size_t)row * L + ln] = acc[q][j];
        }
}

template <typename T>
static hipError_t contract_rot_mfma(const CoarseGemm* c, int m, const T* P, const T* in, T* out, hipStream_t s)
{
    // one row tile per wave (two, sharing the line loads, measured slower:
    // 10.9 against 9.7 us FP32, 14.5 against 13.5 us FP64 at 90^3, fewer
    // waves to hide the loads' latency)
    constexpr int RT = 1;
    const int per = c->m[0] * c->m[1] * c->m[2];
    const int L = per / m;
    const int rtiles = (m + 15) / 16, ctiles = (L + 15) / 16;
    const int waves = ((rtiles + RT - 1) / RT) * ctiles;   // per copy
    const dim3 grid((unsigned)((waves + CT_NT / 64 - 1) / (CT_NT / 64)), (unsigned)c->nb);
    const int nch = (m + 15) / 16;
    switch (nch) {
        case 1: hipLaunchKernelGGL((k_contract<T, 1, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        case 2: hipLaunchKernelGGL((k_contract<T, 2, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        case 3: hipLaunchKernelGGL((k_contract<T, 3, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        case 4: hipLaunchKernelGGL((k_contract<T, 4, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        case 5: hipLaunchKernelGGL((k_contract<T, 5, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        case 6: hipLaunchKernelGGL((k_contract<T, 6, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
        default: hipLaunchKernelGGL((k_contract<T, 0, RT>), grid, dim3(CT_NT), 0, s, P, in, out, m, L, rtiles, ctiles); break;
    }
    return hipGetLastError();
}

// Which contraction each precision takes (measured at 90^3, one right-hand
// side, 7744 x 88 x 88 per contraction): FP64 on the matrix cores above
// (rocBLAS dgemm takes 19.5 us); FP32 through rocBLAS sgemm (strided batch
// over the copies, atomics off, so the bits repeat), 6.9 us against 9.7 us
// for the kernel above on the FP32 matrix cores.
static hipError_t contract_rot(const CoarseGemm* c, int m, const double* const* P64, int d, const double* in,
                               double* out, hipStream_t s)
{
    return contract_rot_mfma<double>(c, m, P64[d], in, out, s);
}

static hipError_t contract_rot(const CoarseGemm* c, int m, const float* const* P32, int d, const float* in, float* out,
                               hipStream_t)
{
    const int per = c->m[0] * c->m[1] * c->m[2];
    const int L = per / m;
    const float one = 1.0f, zero = 0.0f;
    // column-major C (L x m) = A^T B, A the input (m x L), B the row-major P
    // read as column-major (B(k, r) = P[r][k]): out[r][line] = sum_k P[r][k] in[line][k]
    const rocblas_status st = rocblas_sgemm_strided_batched(c->blas, rocblas_operation_transpose,
                                                            rocblas_operation_none, L, m, m, &one, in, m, per, P32[d], m,
                                                            0, &zero, out, L, per, c->nb);
    return st == rocblas_status_success ? hipSuccess : hipErrorUnknown;
}

// (the axis tables are FP64 in both precisions; the eigenvalue sums of the
// division are the cycle's precision)
template <typename T> struct CgTab;
template <> struct CgTab<double> {
    static double* const* S(const CoarseGemm* c) { return c->S64; }
    static double* const* Si(const CoarseGemm* c) { return c->Si64; }
    static double* const* lam(const CoarseGemm* c) { return c->lam64; }
    static double* buf(const CoarseGemm* c, int b) { return c->buf64[b]; }
};
template <> struct CgTab<float> {
    static float* const* S(const CoarseGemm* c) { return c->S32; }
    static float* const* Si(const CoarseGemm* c) { return c->Si32; }
    static float* const* lam(const CoarseGemm* c) { return c->lam32; }
    static float* buf(const CoarseGemm* c, int b) { return c->buf32[b]; }
};

// the stream the FP32 contractions (rocBLAS) are issued on
void coarse_gemm_set_stream(lasto_grid g, hipStream_t s)
{
    if (g->cg && g->cg->blas) (void)rocblas_set_stream(g->cg->blas, s);
}

template <typename T>
lasto_status coarse_gemm_solve(lasto_grid g, const T* f, T* u, hipStream_t s)
{
    const CoarseGemm* c = g->cg;
    const LevelView& V = g->lev[g->cg_level].view;
    const int n = c->m[0] * c->m[1] * c->m[2] * c->nb;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    T* b0 = CgTab<T>::buf(c, 0);
    T* b1 = CgTab<T>::buf(c, 1);
    auto lam = CgTab<T>::lam(c);
    hipLaunchKernelGGL(k_split_to_dense<T>, dim3(blocks), dim3(256), 0, s, V, f, b0);
    LASTO_LAUNCH_CHECK("k_split_to_dense");
    auto Si = CgTab<T>::Si(c);
    auto S = CgTab<T>::S(c);
    LASTO_HIP(contract_rot(c, c->m[0], Si, 0, b0, b1, s));
    LASTO_HIP(contract_rot(c, c->m[1], Si, 1, b1, b0, s));
    LASTO_HIP(contract_rot(c, c->m[2], Si, 2, b0, b1, s));
    hipLaunchKernelGGL(k_divide_dense<T>, dim3(blocks), dim3(256), 0, s, b1, lam[0], lam[1], lam[2], c->m[0],
                       c->m[1], c->m[2], n);
    LASTO_LAUNCH_CHECK("k_divide_dense");
    LASTO_HIP(contract_rot(c, c->m[0], S, 0, b1, b0, s));
    LASTO_HIP(contract_rot(c, c->m[1], S, 1, b0, b1, s));
    LASTO_HIP(contract_rot(c, c->m[2], S, 2, b1, b0, s));
    hipLaunchKernelGGL(k_dense_to_split<T>, dim3(blocks), dim3(256), 0, s, V, b0, u);
    LASTO_LAUNCH_CHECK("k_dense_to_split");
    return LASTO_OK;
}
template lasto_status coarse_gemm_solve<double>(lasto_grid, const double*, double*, hipStream_t);
template lasto_status coarse_gemm_solve<float>(lasto_grid, const float*, float*, hipStream_t);

}  // namespace lasto

using namespace lasto;

extern "C" lasto_status lasto_fdm_axis(const double* x, int n, double* lam, double* S, double* Sinv)
{
    if (!x || !lam || !S || !Sinv || n < 3) return fail(LASTO_ERR_ARG, "lasto_fdm_axis: NULL argument or n < 3");
    for (int i = 0; i + 1 < n; ++i)
        if (!(x[i + 1] > x[i])) return fail(LASTO_ERR_ARG, "lasto_fdm_axis: coordinates must increase");
    if (!axis_decomposition(x, n, lam, S, Sinv)) return fail(LASTO_ERR_STATE, "lasto_fdm_axis: no convergence");
    return LASTO_OK;
}

extern "C" lasto_status lasto_fdm_solve(lasto_grid g, const double* rho, double* v, int bc, int lmax_bc,
                                        lasto_solve_info* info)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!g || !rho || !v) return fail(LASTO_ERR_ARG, "lasto_fdm_solve: NULL argument");
    if (bc < 0 || bc > 2 || lmax_bc < 0 || lmax_bc > 4) return fail(LASTO_ERR_ARG, "lasto_fdm_solve: bad bc/lmax_bc");
    const LevelView& V = g->cview;
    if (V.nx < 3 || V.ny < 3 || V.nz < 3) return fail(LASTO_ERR_ARG, "lasto_fdm_solve: needs 3 nodes per axis");
    if (lasto_status st = fdm_init(g); st != LASTO_OK) return st;
    FdmState* f = g->fdm;
    const size_t N = (size_t)V.nx * V.ny * V.nz;
    const size_t cells = (size_t)f->m[0] * f->m[1] * f->m[2];
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    hipStream_t s = g->stream;
    for (int b = 0; b < g->n_batch; ++b) {
        const double* rb = rho + b * N;
        double* vb = v + b * N;
        if (bc == 1) {
            LASTO_HIP(launch_moments(g, rb, g->moments + 25 * b));
            LASTO_HIP(launch_bc(g, 1, g->moments + 25 * b, lmax_bc, vb));
        } else if (bc == 0) {
            LASTO_HIP(launch_bc(g, 0, g->moments, 0, vb));
        }   // bc 2: the faces of v as given
        hipLaunchKernelGGL(k_fdm_rhs, dim3(blocks), dim3(256), 0, s, V, vb, rb, 4.0 * kPi, f->buf[0]);
        LASTO_LAUNCH_CHECK("k_fdm_rhs");
        rocblas_status e = contract(f, 0, f->Si[0], f->buf[0], f->buf[1]);
        if (e == rocblas_status_success) e = contract(f, 1, f->Si[1], f->buf[1], f->buf[0]);
        if (e == rocblas_status_success) e = contract(f, 2, f->Si[2], f->buf[0], f->buf[1]);
        if (e != rocblas_status_success) return fail(LASTO_ERR_HIP, "lasto_fdm_solve: rocBLAS GEMM");
        hipLaunchKernelGGL(k_fdm_divide, dim3(blocks), dim3(256), 0, s, f->buf[1], f->lam[0], f->lam[1], f->lam[2],
                           f->m[0], f->m[1], f->m[2]);
        LASTO_LAUNCH_CHECK("k_fdm_divide");
        e = contract(f, 0, f->S[0], f->buf[1], f->buf[0]);
        if (e == rocblas_status_success) e = contract(f, 1, f->S[1], f->buf[0], f->buf[1]);
        if (e == rocblas_status_success) e = contract(f, 2, f->S[2], f->buf[1], f->buf[0]);
        if (e != rocblas_status_success) return fail(LASTO_ERR_HIP, "lasto_fdm_solve: rocBLAS GEMM");
        hipLaunchKernelGGL(k_fdm_unpack, dim3(blocks), dim3(256), 0, s, V, f->buf[0], vb);
        LASTO_LAUNCH_CHECK("k_fdm_unpack");
    }
    // ||4 pi rho - A v||_W against the face data's, per right-hand side
    const int nparts = interior_blocks(V);
    for (int b = 0; b < g->n_batch; ++b) {
        for (int zero = 1; zero >= 0; --zero) {
            LASTO_HIP(launch_residual_nat(V, v + b * N, rho + b * N, 4.0 * kPi, nullptr, g->partials, zero, s));
            LASTO_HIP(launch_reduce(g->partials, 1, nparts, g->scalars + (zero ? S_BR0 : S_BRR) + b, s));
        }
    }
    LASTO_HIP(hipMemcpyAsync(g->h_scalars, g->scalars, sizeof(double) * kNumScalars, hipMemcpyDeviceToHost, s));
    LASTO_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    if (info) std::memset(info, 0, sizeof(*info));
    for (int b = 0; b < g->n_batch; ++b) {
        const double r0 = g->h_scalars[S_BR0 + b], rr = g->h_scalars[S_BRR + b];
        const double rel = r0 > 0.0 ? std::sqrt(rr / r0) : std::sqrt(rr);
        worst = std::max(worst, rel);
        if (info && b < kMaxBatch) info->batch_rel_resid[b] = rel;
    }
    if (info) {
        info->iters = 1;
        info->rel_resid = worst;
        info->resid_hist[0] = worst;
        info->n_batch = g->n_batch;
        info->coarse_level = -1;
        if (bc == 1) {
            LASTO_HIP(hipMemcpy(info->moments, g->moments, sizeof(double) * 25, hipMemcpyDeviceToHost));
        }
        info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!std::isfinite(worst)) return fail(LASTO_ERR_DIVERGED, "lasto_fdm_solve: non-finite residual");
    return LASTO_OK;
}
