// Internal declarations of the LASTO Hartree-step library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lasto.h"

namespace lasto {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxLevels = 40;
constexpr int kCoarseMax = 5;         // coarsening stops when every axis has <= 5 nodes
constexpr double kCoarsenTheta = 4.0; // merge cell pairs up to theta * (smallest spacing)
constexpr int kReduceBlocks = 1024;   // fixed partial count of every reduction (determinism)
constexpr int kMaxBatch = 16;          // right-hand sides of one batched grid
constexpr int kInnerHist = 32;        // inner FP32 PCG steps whose <r, z>_W are kept (a ring)
constexpr int kNumScalars = 32 + 3 * kMaxBatch + kInnerHist;

// scalar slots of the device scalar array
enum Scalar {
    S_RZ0 = 0, S_RZ1 = 1,   // <r, z>_W of the current / previous PCG step (ping-pong)
    S_PQ = 2,               // <p, A p>_W
    S_RR = 3,               // <r, r>_W after the update
    S_R0 = 4,               // reference ||b - A v_bc||_W^2
    S_TMP = 5,
    S_BAD = 6,              // nonzero once an FP32 correction held a non-finite value (not added to v)
    S_PQ32 = 10,            // inner FP32 PCG: <p, A p>_W (its <r, z>_W are S_RZH + step)
    S_LC_R = 12, S_LC_E = 13,  // learned coarse correction: ||f_c||_W^2 and ||f_c - A_c e||_W^2
    S_LC_ACC = 14,          // learned coarse corrections accepted in this solve
    S_LC_SCALE = 15,        // (spare)
    S_ZQ = 16, S_FNUM = 17,     // flexible CG: <z_new, q_old>_W and its beta numerator (FP64)
    S_ZQ32 = 18, S_FNUM32 = 19, // the same in the inner FP32 PCG
    S_BR0 = 32,                        // per right-hand side: reference norm^2 [kMaxBatch]
    S_BRR = 32 + kMaxBatch,            // per right-hand side: residual norm^2 [kMaxBatch]
    S_BJ = 32 + 2 * kMaxBatch,         // per right-hand side: a second residual norm^2 [kMaxBatch]
    S_RZH = 32 + 3 * kMaxBatch,        // inner FP32 PCG: <r, z>_W of step k at S_RZH + k % kInnerHist
};

void set_error(const std::string& msg);
lasto_status fail(lasto_status s, const std::string& msg);

#define LASTO_HIP(call)                                                               \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::lasto::fail(LASTO_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LASTO_LAUNCH_CHECK(name)                                                      \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess)                                                         \
            return ::lasto::fail(LASTO_ERR_HIP, std::string("launch ") + name + ": " + hipGetErrorString(e_)); \
    } while (0)

// Per-axis device tables of one level.
//   am[i] = 1/(h_{i-1} m_i), ap[i] = 1/(h_i m_i) at interior i (0 at the ends)
//   m[i]  = dual width (half spacings at the ends)
//   x[i]  = coordinate
// Transfer tables toward the next finer level (level > 0):
//   rf[I]   = fine index of coarse node I
//   rw[3*I + s], s = 0,1,2: restriction weight of fine node rf[I]-1+s,
//             already multiplied by m_fine/m_coarse (zero if that fine node
//             is kept by another coarse node)
//   pc[i]   = coarse index at or left of fine node i
//   pw[2*i + s]: interpolation weights of coarse nodes pc[i], pc[i]+1
struct Axis {
    int n;
    const double* am;
    const double* ap;
    const double* m;
    const double* x;
    const int* rf;
    const double* rw;
    const int* pc;
    const double* pw;
    const float* amf;   // FP32 copies of am, ap
    const float* apf;
};

// x coefficients by parity for the half-sweeps: entry [p][q][m] (q = 0 am,
// 1 ap, 2 dual width) of node i = p + 2m, zero where i is not interior;
// rows of W entries. One block per precision.
template <typename T> struct XPar;

// Colour-split storage of multigrid arrays: node (i,j,k) of colour
// c = (i+j+k) & 1 lives at [c][k][j][i >> 1] in rows of W (padded) entries,
// cs = nz*ny*W apart between colours. A red-black half-sweep then reads one
// colour array and writes the other, both contiguous in x.
//
// A batched grid stacks its n_batch right-hand sides along z: copy b owns
// planes b*nzc .. b*nzc + nzc - 1, its first and last planes are its own
// Dirichlet faces, and the z tables repeat per copy. zint[k] marks the planes
// interior to their copy; stencils never couple two copies because every
// plane next to another copy is a face.
struct LevelView {
    int nx, ny, nz;
    int nzc;        // planes per copy (nz = n_batch * nzc)
    int W;          // padded row length of one colour (>= (nx+1)/2)
    size_t cs;      // colour stride = nz * ny * W
    Axis ax[3];
    const double* xpar;   // [2][3][W] x coefficients by parity (FP64)
    const float* xparf;   // the same in FP32
    const unsigned char* zint;   // [nz] 1 on planes interior to their copy
};

template <> struct XPar<double> {
    __host__ __device__ static const double* get(const LevelView& L) { return L.xpar; }
};
template <> struct XPar<float> {
    __host__ __device__ static const float* get(const LevelView& L) { return L.xparf; }
};

__host__ __device__ __forceinline__ size_t sidx(const LevelView& L, int i, int j, int k)
{
    return (size_t)((i + j + k) & 1) * L.cs + ((size_t)k * L.ny + j) * L.W + (i >> 1);
}

struct Level {
    int n[3];
    size_t npts;       // nx*ny*nz
    size_t nsplit;     // 2*cs elements of a split array
    std::vector<double> hx[3];     // host copies of coordinates
    std::vector<int> keep[3];      // index in the finer level (level > 0)
    double* dtab = nullptr;        // device table block
    int* dtabi = nullptr;
    double* dxpar = nullptr;       // device x-parity table (FP64)
    unsigned char* dzint = nullptr;   // device [nz] interior-plane flags
    float* dtabf = nullptr;        // device FP32 tables (am, ap per axis; x-parity)
    LevelView view;
    // V-cycle work arrays (split layout): correction, right-hand side, residual
    double* u64 = nullptr;
    double* f64 = nullptr;
    double* r64 = nullptr;
    float* u32 = nullptr;
    float* f32 = nullptr;
    float* r32 = nullptr;
};

// A level as the single-workgroup tail kernel sees it (an array of these
// lives in device memory). Level 0's correction and right-hand side are the
// fine-level Krylov vectors z and r.
struct TailLevel {
    LevelView V;
    double *u64, *f64, *r64;
    float *u32, *f32, *r32;
};

template <typename T> struct TailBuf;
template <> struct TailBuf<double> {
    __host__ __device__ static double* u(const TailLevel& t) { return t.u64; }
    __host__ __device__ static double* f(const TailLevel& t) { return t.f64; }
    __host__ __device__ static double* r(const TailLevel& t) { return t.r64; }
};
template <> struct TailBuf<float> {
    __host__ __device__ static float* u(const TailLevel& t) { return t.u32; }
    __host__ __device__ static float* f(const TailLevel& t) { return t.f32; }
    __host__ __device__ static float* r(const TailLevel& t) { return t.r32; }
};

constexpr size_t kTailMaxPts = 16384;   // levels at or below this size run in the tail kernel
constexpr size_t kGemmCoarseMaxPts = 3000000;   // per copy: the largest level the GEMM coarsest solve takes

// LDS layout of the FP32 tail. Per level q (0 = the first level it takes):
// dims nx, ny, nz, W, cs; offsets (floats) of its correction and right-hand
// side (split layout, 2 cs each, 16-byte aligned) and of its table block.
// The table blocks are one run of ntab floats at tab0, copied in from a
// device table the grid builds (layout: lds_tab).
constexpr int kLdsMaxLevels = 12;
struct LdsPlan {
    int nl;
    int total;                      // floats of LDS
    int tab0, ntab;
    int dims[kLdsMaxLevels][5];
    int off[kLdsMaxLevels][3];
};

// Table block of one level of the LDS tail (FP32): am and ap of x, y, z,
// interior-plane flags of z (1 or 0); below the first level also the
// restriction from the finer level (rf as values, rw) and the interpolation
// back to it (pc as values, pw), indexed as in Axis. fn*: the finer level's
// sizes.
struct LdsTab {
    const float *cxm, *cxp, *cym, *cyp, *czm, *czp, *zin;
    const float *rfx, *rfy, *rfz, *rwx, *rwy, *rwz;
    const float *pcx, *pcy, *pcz, *pwx, *pwy, *pwz;
};

__host__ __device__ __forceinline__ int lds_tab_size(int nx, int ny, int nz, int fnx, int fny, int fnz, bool coarse)
{
    int s = 2 * nx + 2 * ny + 3 * nz;
    if (coarse) s += 4 * (nx + ny + nz) + 3 * (fnx + fny + fnz);
    return (s + 3) / 4 * 4;
}

template <typename P>
__host__ __device__ __forceinline__ LdsTab lds_tab(P* b, int nx, int ny, int nz, int fnx, int fny, int fnz,
                                                   bool coarse)
{
    LdsTab t{};
    t.cxm = b;
    t.cxp = t.cxm + nx;
    t.cym = t.cxp + nx;
    t.cyp = t.cym + ny;
    t.czm = t.cyp + ny;
    t.czp = t.czm + nz;
    t.zin = t.czp + nz;
    if (coarse) {
        t.rfx = t.zin + nz;
        t.rfy = t.rfx + nx;
        t.rfz = t.rfy + ny;
        t.rwx = t.rfz + nz;
        t.rwy = t.rwx + 3 * nx;
        t.rwz = t.rwy + 3 * ny;
        t.pcx = t.rwz + 3 * nz;
        t.pcy = t.pcx + fnx;
        t.pcz = t.pcy + fny;
        t.pwx = t.pcz + fnz;
        t.pwy = t.pwx + 2 * fnx;
        t.pwz = t.pwy + 2 * fny;
    }
    return t;
}

}  // namespace lasto

namespace lasto {
struct FdmState;     // fast-diagonalisation tables and work arrays (fdm.hip)
struct CoarseGemm;   // the same for the cycle's coarsest level (fdm.hip)
}

struct lasto_grid_s {
    int nlev = 0;
    int n_batch = 1;
    hipStream_t stream = nullptr;
    int device = 0;
    lasto::Level lev[lasto::kMaxLevels];
    int tail_top = 0;                      // first level handled by the tail kernel
    int tail32_top = -1;                   // first level of the FP32 LDS tail (-1: none)
    lasto::LdsPlan lds_plan{};
    float* lds_tabs = nullptr;             // device copy of the LDS tail's tables
    lasto::LdsPlan* lds_plan_dev = nullptr;   // device copy of lds_plan
    lasto::TailLevel* tail_dev = nullptr;  // device [nlev]
    // fine-level Krylov vectors (FP64, split layout): residual, preconditioned
    // residual, search direction (ping-pong), A p
    double* r = nullptr;
    double* z = nullptr;
    double* p[2] = {nullptr, nullptr};
    double* q = nullptr;
    double* x = nullptr;       // PCG correction to v, added to v at convergence
    // FP32 inner-solve vectors on the fine level (split layout)
    float* r32 = nullptr;
    float* z32 = nullptr;
    float* p32[2] = {nullptr, nullptr};
    float* q32 = nullptr;
    float* e32 = nullptr;
    // reductions
    double* partials = nullptr;
    double* scalars = nullptr;      // [kNumScalars]
    double* h_scalars = nullptr;    // pinned host mirror (then 25 moments at h_scalars + kNumScalars)
    double* moments = nullptr;      // device [25 * n_batch]
    lasto::LevelView cview;         // the finest level as one copy of the batch sees it
    // scratch of the learned entry points (finest-level size, allocated on
    // first use): natural residual, natural zeros, the two kept candidates,
    // and the split iterate and source of their judging sweep
    double* lscr[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // interpolation / atom staging
    double* stage = nullptr;
    size_t stage_bytes = 0;
    void* stage_host = nullptr;       // pinned host copy of the staged atom table (an async upload)
    size_t stage_host_bytes = 0;
    double box_center[3] = {0, 0, 0};
    lasto::FdmState* fdm = nullptr;   // built on the first lasto_fdm_solve
    // coarsest solve of the cycle by fast diagonalisation (cfdm_level -1: the
    // level does not allow it, and the red-black tail runs instead)
    int cfdm_level = -1;
    int cfdm_mx = 0;                  // padded row length of its axis tables
    double* cfdm_tab64 = nullptr;     // device: per axis S^-1, S, eigenvalues
    float* cfdm_tab32 = nullptr;
    int coarse_mode = 0;              // the current solve's opts.coarse
    int nu_coarse = 0;                // the current solve's opts.nu_coarse
    int fused_sweeps = 0;             // the current solve's opts.fused_sweeps
    // the exact coarsest solve by GEMMs on a larger level (tables built on
    // first use; cg_level -1: no level qualifies)
    int cg_level = -1;
    lasto::CoarseGemm* cg = nullptr;
    // optional event timing of the finest-level sweeps (solve opts.profile)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;   // start/stop pairs
    // launch sequences captured into HIP graphs (the finest-level V-cycle,
    // a step of the inner FP32 PCG) and replayed in place of their launches,
    // keyed by what they do and the arrays they touch; captured on a stream
    // of the library's own at their second use
    struct VGraph {
        int key[8];
        const void* ptr[4];
        int uses = 0;
        hipGraphExec_t exec = nullptr;
        int aux = 0;          // an int the sequence reports (the V-cycle's partial count)
        double bytes = 0.0;   // algorithmic bytes it counts
    };
    std::vector<VGraph> vgraphs;
    hipStream_t cap_stream = nullptr;
    int prof_used = 0;
    double prof_bytes = 0.0;
    int prof_fp32 = 0;
    // algorithmic bytes of the current solve's finest-level launches
    double alg_bytes = 0.0;
    // phase stamps of a solve (start, faces done, guess done, end)
    hipEvent_t ph_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // tables of the learned guess on a coarse level (lg_level -1: none built)
    int lg_level = -1;
    const int* lg_idx[3] = {nullptr, nullptr, nullptr};     // fine index of each coarse node
    const int* lg_pi[3] = {nullptr, nullptr, nullptr};      // coarse interval of each fine node
    const double* lg_pw[3] = {nullptr, nullptr, nullptr};   // its linear weight
    std::vector<void*> lg_alloc;
    // the current solve's learned coarse correction (lc_net NULL: none)
    lasto_net lc_net = nullptr;
    int lc_level = -1;
    int lc_applied = 0;
};

namespace lasto {

// ----------------------------------------------------------------- kernels
// Block counts of the reducing launches (each writes one partial per block).
int half_blocks(const LevelView& L);       // one half-sweep
int interior_blocks(const LevelView& L);   // partials of a residual-norm launch (launch_residual_nat*)
size_t split_elems(const LevelView& L);

// Red-black half-sweep on A u = bscale f, in place in the split layout:
// nodes of colour c solve their equation from the other colour's values.
// zero_in: the other colour is read as zero. dotp (optional): per-block
// partials of sum vol * f * u_new over the updated nodes.
// *nparts (optional): partials written (one per workgroup; at most half_blocks(L)).
// top: finest-level launch (a kernel of its own name, same code).
// ev0, ev1 (optional): events stamped with the dispatch's own start and end.
template <typename T>
hipError_t launch_half(const LevelView& L, T* u, const T* f, int colour, int zero_in, T bscale, double* dotp,
                       hipStream_t s, int* nparts = nullptr, int top = 0, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// nsweeps (2, 4 or 6; at most gs_block_max<T>()) consecutive half-sweeps, colours c0, 1 - c0, ..., in
// one pass (zero faces): colour 1 - c0 of uin is read (nothing with zero_in)
// and both colours of the result written to uout, which must differ from uin
// unless zero_in. dotp (not with zero_in): per-block partials of
// sum vol * f * u over the nodes of the last two half-sweeps (*nparts of them).
template <typename T>
hipError_t launch_gs_block(const LevelView& L, const T* uin, const T* f, T* uout, int c0, int nsweeps, int zero_in,
                           T bscale, double* dotp, hipStream_t st, int* nparts = nullptr, int top = 0,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int gs_block_parts(const LevelView& L);   // partials a launch_gs_block with dotp may write
template <typename T> int gs_block_max();   // the longest pass launch_gs_block takes (FP32 6, FP64 4)
// whole-array precision changes (n elements, rounding to nearest)
hipError_t launch_cast(const double* a, float* b, size_t n, hipStream_t s);
hipError_t launch_cast(const float* a, double* b, size_t n, hipStream_t s);
// the same on an array whose faces carry Dirichlet data (written back unchanged)
template <typename T>
hipError_t launch_half_keep_faces(const LevelView& L, T* u, const T* f, int colour, T bscale, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s);
// Transfers exploiting the red-black ordering of the cycle: after a
// pre-smoothing that ends with a black half-sweep the residual vanishes on
// black nodes (residual_colour computes one colour; restrict_red reads red
// fine nodes only), and before a post-smoothing that starts with a black
// half-sweep only red nodes need the coarse correction (prolong_red).
template <typename T>
hipError_t launch_residual_colour(const LevelView& L, const T* u, const T* f, T* r, int colour, hipStream_t s);
// q = A p on both colours in one launch, partials of <p, q>_W
template <typename T>
hipError_t launch_apply_both(const LevelView& L, const T* p, T* q, double* dotp, hipStream_t s, int* nparts);
template <typename T>
hipError_t launch_restrict_red(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s);
template <typename T>
hipError_t launch_prolong_red(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s);
// the same interpolation, from uin, written to another array: out (red) = uin (red) + P e
template <typename T>
hipError_t launch_prolong_red_to(const LevelView& F, const LevelView& C, const T* e, const T* uin, T* out,
                                 hipStream_t s);
// V(nu1, nu2) on levels lv[0..nl-1] in one workgroup, from zero (lv[0]
// from its current u unless top_zero); the coarsest runs csweeps (red,
// black) sweeps then csweeps (black, red).
template <typename T>
hipError_t launch_tail(const TailLevel* lv, int nl, int nu1, int nu2, int csweeps, int top_zero, hipStream_t s);
// the FP32 cycle from level P's first with every level in LDS: u, f that
// level's correction and right-hand side (split), tabs the grid's table run
hipError_t launch_tail_lds(float* u, const float* f, const float* tabs, int nu1, int nu2, int csweeps, int top_zero,
                           const LdsPlan& P, const LdsPlan* P_dev, hipStream_t s);
int tail_lds_limit();   // bytes of LDS one workgroup may use (0 if unknown)
// exact solve of A e = f (zero faces) at level g->cfdm_level, split layout
template <typename T>
hipError_t launch_coarse_fdm(lasto_grid g, const T* f, T* e, hipStream_t s);
lasto_status build_coarse_fdm(lasto_grid g);   // tables of the tail's top level, if it qualifies
void free_coarse_fdm(lasto_grid g);
// exact solve of A e = f (zero faces) at level g->cg_level by GEMMs, split layout
void choose_coarse_gemm_level(lasto_grid g);
lasto_status coarse_gemm_init(lasto_grid g);    // tables, buffers and rocBLAS handle on first use
void coarse_gemm_set_stream(lasto_grid g, hipStream_t s);   // the stream of its rocBLAS calls
template <typename T>
lasto_status coarse_gemm_solve(lasto_grid g, const T* f, T* e, hipStream_t s);
void free_coarse_gemm(lasto_grid g);

hipError_t launch_reduce(const double* partials, int stride, int count, double* out, hipStream_t s);
template <typename T>
hipError_t launch_dot(const LevelView& L, const T* a, const T* b, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_update_p(const LevelView& L, const T* z, const T* pold, T* pnew, const double* scal,
                           int i_num, int i_den, int first, hipStream_t s);
// x += alpha p, r -= alpha q (all split), alpha = scal[i_num]/scal[i_den];
// partials of <r, r>_W when partials is given (count in *nparts, at most
// flat_blocks<T>(L))
// the inner FP32 PCG's deferred form: pnew = z + beta pold with x = (or +=,
// accumulate) alpha_prev pold in the same pass; then r -= alpha q
template <typename T>
hipError_t launch_update_px(const LevelView& L, const T* z, const T* pold, T* pnew, T* x, const double* scal,
                            int i_num, int i_den, int i_anum, int i_aden, int accumulate, hipStream_t s);
template <typename T>
hipError_t launch_update_r(const LevelView& L, T* r, const T* q, const double* scal, int i_num, int i_den,
                           hipStream_t s);
template <typename T>
hipError_t launch_update_xr(const LevelView& L, T* x, T* r, const T* p, const T* q, const double* scal, int i_num,
                            int i_den, double* partials, hipStream_t s, int* nparts, int first = 0);
template <typename T>
int flat_blocks(const LevelView& L);
int row_blocks(const LevelView& L);   // partials of the row-wise split dot
// natural-layout fine-level helpers
hipError_t launch_residual_nat(const LevelView& L, const double* v, const double* rho, double bscale, double* r_split,
                               double* partials, int interior_zero, hipStream_t s);
hipError_t launch_apply_nat(const LevelView& L, const double* u, double* Au, hipStream_t s);
hipError_t launch_add_nat(const LevelView& L, double* v, const double* e_split, hipStream_t s);
// r32 = bscale rho - A v in FP32 (split), partials of ||r||_W^2 (FP64)
hipError_t launch_residual_nat32(const LevelView& L, const double* v, const double* rho, double bscale, float* r32,
                                 double* partials, hipStream_t s);
// v (natural) += e32 (+ alpha p32 when p32 is given, alpha = scal[i_num]/scal[i_den]); a node
// whose new value would not be finite keeps its value and sets scal[S_BAD] (bad = true)
hipError_t launch_add32_nat(const LevelView& L, double* v, const float* e32, const float* p32, double* scal,
                            int i_num, int i_den, hipStream_t s, bool flag_bad = false);
hipError_t launch_nat_to_split(const LevelView& L, const double* a, double* s_out, hipStream_t s);
hipError_t launch_split_to_nat(const LevelView& L, const double* s_in, double* a, hipStream_t s);
template <typename T>
hipError_t launch_fill_zero(T* a, size_t n, hipStream_t s);
hipError_t launch_inject_nan(double* r, size_t idx, hipStream_t s);
hipError_t launch_inject_nan(float* r, size_t idx, hipStream_t s);

// source, boundary, interpolation
struct AtomDev {
    double c[3];
    double R;
    double q;
    double w;
    double alpha;
    double rho_R, drho_R;
    double coef[3];   // kind 1 quartic a, b, c (filled on the device)
    double s;         // kind 0 renormalisation (filled on the device)
    int kind;
    int lmax;
    double clm[24];
    // filled on the device by k_atom_prep:
    double pre;       // kind 0: q s (pi w^2)^(-3/2)
    double iw2;       // kind 0: 1 / w^2
    double cut2;      // squared radius of the l = 0 term (kind 0: (7 w)^2, kind 1: R^2)
    double lcut2;     // squared radius of the l >= 1 terms (alpha r^2 < 42.25), -1 without them
    double cull2;     // squared radius beyond which the atom adds nothing (and is not "inside")
    double cn[24];    // clm times the r^l y_lm normalisation
};
hipError_t launch_atom_prep(lasto_grid g, AtomDev* atoms, int n_atoms, int renormalize);
hipError_t launch_pseudo(lasto_grid g, const AtomDev* atoms, int n_atoms, const double* rho_inter, double* rho);
hipError_t launch_moments(lasto_grid g, const double* rho, double* Q);
hipError_t launch_bc(lasto_grid g, int mode, const double* Q, int lmax_bc, double* v);
hipError_t launch_guess(lasto_grid g, const AtomDev* atoms, int n_atoms, double* v);
// every right-hand side's guess (one pass for copies that share their geometry)
hipError_t launch_guess_all(lasto_grid g, const AtomDev* dev_atoms, const lasto_atom* host_atoms, int n_atoms,
                            double* v);
// validate an atom table, copy it to the grid's staging buffer and prepare it on the device
lasto_status stage_atoms(lasto_grid g, int n_atoms, const lasto_atom* atoms, int renormalize, const char* who,
                         AtomDev** out);
// v (natural, interior) += s * y (FP32, natural)
hipError_t launch_add_f32_nat(const LevelView& L, double* v, const float* y, double s, hipStream_t st);
// learned guess: features of (rho, v) and the net's forward pass on the grid's
// stream; *y is the net's output buffer (finest-level nodes, FP32)
lasto_status net_guess_forward(lasto_grid g, lasto_net n, const double* rho, const double* v, const float** y,
                               double* out_scale, double rho_mul = 1.0);
lasto_status net_features_async(lasto_grid g, lasto_net n, const double* rho, const double* v, uint16_t* x,
                                double rho_mul);
// v += the learned correction of one right-hand side (finest-level net, or a
// net on a coarse level with its output interpolated to the finest)
lasto_status net_guess_apply(lasto_grid g, lasto_net n, const double* rho, double* v);
// learned coarse correction at level l of a cycle: u = the net's proposal for
// A_l u = f if it lowers the residual, else 0 (r: the level's residual scratch,
// zero again on return); g->lc_net must be set
template <typename T>
lasto_status learned_coarse_start(lasto_grid g, int l, const T* f, T* u, T* r);
// `cycles` FP64 V-cycles of level c on A_c u = f from zero (no learned correction)
lasto_status coarse_cycles(lasto_grid g, int c, int cycles, const double* f, double* u);
// the node grid a net was created for (its largest), out[3] = nx, ny, nz
lasto_status net_capacity(lasto_net n, int* out);
lasto_status coarse_pair(lasto_grid g, lasto_net n, const double* rho, const double* v, int c, int nu1, int cycles,
                         uint16_t* x, float* t, double* r_scale);
hipError_t launch_flex_beta(double* scal, int i_rz_old, int i_pq, int i_zq, int i_out, hipStream_t s);
hipError_t launch_interp(lasto_grid g, const double* v, const double* pts, int npts, double* out);

// inside the spheres: one entry per atom (device table of a lasto_spheres)
struct SphereAtom {
    double c[3];   // centre
    double R;      // sphere radius
    double Z;      // nuclear charge
    double D;      // log step of the radial mesh, ln(R / r_min) / (n_rad - 1)
    double pad[2];
};
hipError_t launch_sphere_project(lasto_grid g, const double* v, const SphereAtom* atoms, int n_atoms,
                                 const double4* rule, int npts, double* vlmR);
hipError_t launch_radial_solve(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* vlmR,
                               const double* rho_lm, double* v_lm);
// per (atom, LM) row of each copy: int_0^R V_LM rho_LM r^2 dr into e_row [n_batch][n_atoms][25]
hipError_t launch_sphere_energy(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* v_lm,
                                const double* rho_lm, double* e_row);
int energy_grid_blocks(const LevelView& L);   // partials per copy of launch_energy_grid
hipError_t launch_sphere_terms(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* rho_lm,
                               int lmin, double* rho);
hipError_t launch_energy_grid(lasto_grid g, const double* v, const double* rho, const SphereAtom* atoms, int n_atoms,
                              double* partials);
// interstitial output density: atoms [n][4] (centre, sphere radius), shells
// [n_shells][4] (n, l, offset within the atom's basis, zeta), coef
// [n_atoms * nbpa][n_occ], occ [n_occ] (device)
hipError_t launch_interstitial(lasto_grid g, const double4* atoms, int n_atoms, const double4* shells, int n_shells,
                               int lmax, int nbpa, const double* coef, int n_occ, const double* occ, double* rho);
// interstitial matrix elements: node weights vol * (outside every sphere),
// then the 64 x 64 blocks (r <= c) of S and H over n_chunks node chunks
hipError_t launch_node_weights(lasto_grid g, const double4* atoms, int n_atoms, double* w);
int matrix_block_count(int n_basis);
size_t matrix_partial_doubles(int n_pairs, int n_chunks);
hipError_t launch_matrix_elements(lasto_grid g, const double* w, const double* v, const double4* atoms, int n_atoms,
                                  const double4* shells, int n_shells, int lmax, int nbpa, int n_basis,
                                  const int2* pairs, int n_pairs, int n_chunks, double* partials, double* S, double* H);
void free_fdm(lasto_grid g);
hipError_t launch_energy_final(lasto_grid g, const double* partials, int nparts, const double* e_row, int nrows,
                               double* out);

// device table block builder
lasto_status build_level_tables(lasto_grid g, int l);

}  // namespace lasto
