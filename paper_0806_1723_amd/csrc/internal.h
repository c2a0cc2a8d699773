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
constexpr int kNumScalars = 32;

// scalar slots of the device scalar array
enum Scalar {
    S_RZ0 = 0, S_RZ1 = 1,   // <r, z>_W of the current / previous PCG step (ping-pong)
    S_PQ = 2,               // <p, A p>_W
    S_RR = 3,               // <r, r>_W after the update
    S_R0 = 4,               // reference ||b - A v_bc||_W^2
    S_TMP = 5,
    S_RZ32_0 = 8, S_RZ32_1 = 9, S_PQ32 = 10, S_RR32 = 11,   // inner FP32 PCG
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
};

struct LevelView {
    int nx, ny, nz;
    Axis ax[3];
};

struct Level {
    int n[3];
    size_t npts;
    std::vector<double> hx[3];     // host copies of coordinates
    std::vector<int> keep[3];      // index in the finer level (level > 0)
    double* dtab = nullptr;        // device table block
    int* dtabi = nullptr;
    LevelView view;
    // work arrays (level 0: fine-level PCG/V-cycle vectors; coarse: V-cycle vectors)
    double* u64[2] = {nullptr, nullptr};
    double* f64 = nullptr;
    double* r64 = nullptr;
    float* u32[2] = {nullptr, nullptr};
    float* f32 = nullptr;
    float* r32 = nullptr;
};

}  // namespace lasto

struct lasto_grid_s {
    int nlev = 0;
    int n_batch = 1;
    hipStream_t stream = nullptr;
    int device = 0;
    lasto::Level lev[lasto::kMaxLevels];
    // fine-level Krylov vectors (FP64): residual, search direction (ping-pong), A p, z
    double* r = nullptr;
    double* p[2] = {nullptr, nullptr};
    double* q = nullptr;
    double* z = nullptr;
    // FP32 inner-solve vectors on the fine level
    float* r32 = nullptr;
    float* p32[2] = {nullptr, nullptr};
    float* q32 = nullptr;
    float* e32 = nullptr;
    float* z32 = nullptr;
    // reductions
    double* partials = nullptr;     // [kReduceBlocks * 32]
    double* scalars = nullptr;      // [kNumScalars]
    double* h_scalars = nullptr;    // pinned host mirror
    double* moments = nullptr;      // device [25]
    // interpolation / atom staging
    double* stage = nullptr;        // device staging for points / atoms
    size_t stage_bytes = 0;
    double box_center[3] = {0, 0, 0};
    // optional event timing of the finest-level sweeps (solve opts.profile)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;   // start/stop pairs
    int prof_used = 0;
    double prof_bytes = 0.0;
    int prof_fp32 = 0;
};

namespace lasto {

// ----------------------------------------------------------------- kernels
// blocks of the smoother and of the pointwise interior launches (each writes
// one reduction partial per block)
int smooth_blocks(const LevelView& L);
int interior_blocks(const LevelView& L);
// smoother / transfer / krylov launchers (stream-ordered, no host sync)
template <typename T>
hipError_t launch_smooth(const LevelView& L, const T* uin, const T* f, T* uout, T bscale, int first,
                         int zero_in, double* dot_partials, hipStream_t s);
template <typename T>
hipError_t launch_residual(const LevelView& L, const T* u, const T* f, T bscale, T* r, hipStream_t s);
template <typename T>
hipError_t launch_restrict(const LevelView& F, const LevelView& C, const T* r, T* rc, hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, const T* e, T* u, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(const LevelView& L, T* u, const T* f, int sweeps, hipStream_t s);

hipError_t launch_reduce(const double* partials, int stride, int count, double* out, hipStream_t s);
template <typename T>
hipError_t launch_apply_dot(const LevelView& L, const T* p, T* q, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_residual_norm(const LevelView& L, const double* u, const double* f, double bscale, T* r,
                                double* partials, hipStream_t s);
template <typename T>
hipError_t launch_dot(const LevelView& L, const T* a, const T* b, double* partials, hipStream_t s);
template <typename T>
hipError_t launch_update_p(const LevelView& L, const T* z, const T* pold, T* pnew, const double* scal,
                           int i_num, int i_den, int first, hipStream_t s);
template <typename T>
hipError_t launch_update_xr(const LevelView& L, T* x, T* r, const T* p, const T* q, const double* scal,
                            int i_num, int i_den, double* partials, hipStream_t s);
hipError_t launch_add_f32_to_f64(const LevelView& L, double* u, const float* e, hipStream_t s);
hipError_t launch_scale_f64_to_f32(const LevelView& L, const double* r, float* r32, const double* scal,
                                   int i_norm2, hipStream_t s);
hipError_t launch_add_scaled_f32_to_f64(const LevelView& L, double* u, const float* e, const double* scal,
                                        int i_norm2, hipStream_t s);
hipError_t launch_inject_nan(double* r, size_t idx, hipStream_t s);

// V-cycle (preconditioner): solve A e = f approximately from e = 0, zero faces.
template <typename T>
lasto_status vcycle(lasto_grid g, int nu1, int nu2, T* e_out, const T* f, double* rz_partials);

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
};
hipError_t launch_atom_prep(lasto_grid g, AtomDev* atoms, int n_atoms, int renormalize);
hipError_t launch_pseudo(lasto_grid g, const AtomDev* atoms, int n_atoms, const double* rho_inter, double* rho);
hipError_t launch_moments(lasto_grid g, const double* rho, double* Q);
hipError_t launch_bc(lasto_grid g, int mode, const double* Q, int lmax_bc, double* v);
hipError_t launch_interp(lasto_grid g, const double* v, const double* pts, int npts, double* out);

// device table block builder
lasto_status build_level_tables(lasto_grid g, int l);

}  // namespace lasto
