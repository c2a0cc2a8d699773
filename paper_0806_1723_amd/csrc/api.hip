// C-ABI entry points: errors, the graded mesh helper, the pseudo-density
// and the sphere-boundary interpolation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "internal.h"

namespace lasto {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

lasto_status fail(lasto_status s, const std::string& msg)
{
    set_error(msg);
    return s;
}

}  // namespace lasto

using namespace lasto;

extern "C" const char* lasto_status_string(lasto_status s)
{
    switch (s) {
    case LASTO_OK: return "ok";
    case LASTO_ERR_ARG: return "invalid argument";
    case LASTO_ERR_ALLOC: return "allocation failed";
    case LASTO_ERR_HIP: return "HIP error";
    case LASTO_ERR_NOT_CONVERGED: return "not converged";
    case LASTO_ERR_DIVERGED: return "diverged";
    case LASTO_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

extern "C" const char* lasto_last_error(void) { return g_last_error.c_str(); }

extern "C" lasto_status lasto_mesh_graded_1d(double lo, double hi, int n, const double* planes, int n_planes,
                                             double hmin, double hmax, double gmax, double hmin_step, double* x_out,
                                             double* g_out, double* hmin_used)
{
    const char* err = lasto::mesh_graded_1d(lo, hi, n, planes, n_planes, hmin, hmax, gmax, hmin_step, x_out, g_out,
                                            hmin_used);
    return err ? fail(LASTO_ERR_ARG, std::string("lasto_mesh_graded_1d: ") + err) : LASTO_OK;
}

// Validate an atom table, copy it to the grid's staging buffer and derive the
// per-atom constants on the device (k_atom_prep). The staging buffer is reused
// by the next call, so callers finish their kernels before returning.
lasto_status lasto::stage_atoms(lasto_grid g, int n_atoms, const lasto_atom* atoms, int renormalize, const char* who,
                         AtomDev** out)
{
    std::vector<AtomDev> hv((size_t)std::max(n_atoms, 1));
    const std::string w(who);
    for (int a = 0; a < n_atoms; ++a) {
        const lasto_atom& A = atoms[a];
        AtomDev& D = hv[a];
        std::memset(&D, 0, sizeof(D));
        if (A.kind != 0 && A.kind != 1) return fail(LASTO_ERR_ARG, w + ": kind must be 0 or 1");
        if (A.lmax < 0 || A.lmax > 4) return fail(LASTO_ERR_ARG, w + ": lmax must be 0..4");
        if (A.kind == 0 && !(A.width > 0.0)) return fail(LASTO_ERR_ARG, w + ": width must be > 0");
        if (A.kind == 1 && !(A.radius > 0.0)) return fail(LASTO_ERR_ARG, w + ": radius must be > 0");
        if (A.lmax >= 1 && !(A.alpha > 0.0)) return fail(LASTO_ERR_ARG, w + ": alpha must be > 0");
        double chk = A.q + A.width + A.radius + A.alpha + A.rho_R + A.drho_R + A.center[0] + A.center[1] + A.center[2];
        for (int c = 0; c < 24; ++c) chk += A.clm[c];
        if (!std::isfinite(chk)) return fail(LASTO_ERR_ARG, w + ": non-finite atom data");
        for (int d = 0; d < 3; ++d) D.c[d] = A.center[d];
        D.R = A.radius;
        D.q = A.q;
        D.w = A.width;
        D.alpha = A.alpha;
        D.rho_R = A.rho_R;
        D.drho_R = A.drho_R;
        D.kind = A.kind;
        D.lmax = A.lmax;
        for (int c = 0; c < 24; ++c) D.clm[c] = (c < (A.lmax + 1) * (A.lmax + 1) - 1) ? A.clm[c] : 0.0;
    }
    const size_t bytes = sizeof(AtomDev) * (size_t)std::max(n_atoms, 1);
    if (bytes > g->stage_bytes) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipFree(g->stage);
        g->stage = nullptr;
        LASTO_HIP(hipMalloc(&g->stage, bytes));
        g->stage_bytes = bytes;
    }
    // the upload goes from pinned memory, so it does not wait for the
    // stream's earlier work (the previous call finished before returning, so
    // the pinned copy is free)
    if (bytes > g->stage_host_bytes) {
        (void)hipStreamSynchronize(g->stream);
        if (g->stage_host) (void)hipHostFree(g->stage_host);
        g->stage_host = nullptr;
        g->stage_host_bytes = 0;
        LASTO_HIP(hipHostMalloc(&g->stage_host, std::max(bytes, (size_t)1 << 16)));
        g->stage_host_bytes = std::max(bytes, (size_t)1 << 16);
    }
    std::memcpy(g->stage_host, hv.data(), bytes);
    AtomDev* dat = (AtomDev*)g->stage;
    LASTO_HIP(hipMemcpyAsync(dat, g->stage_host, bytes, hipMemcpyHostToDevice, g->stream));
    if (n_atoms > 0) LASTO_HIP(launch_atom_prep(g, dat, n_atoms, renormalize));
    *out = dat;
    return LASTO_OK;
}

extern "C" lasto_status lasto_pseudo_density(lasto_grid g, int n_atoms, const lasto_atom* atoms,
                                             const double* rho_interstitial, int renormalize, double* rho_out,
                                             double* moments_out)
{
    if (!g || !rho_out || n_atoms < 0 || (n_atoms > 0 && !atoms))
        return fail(LASTO_ERR_ARG, "lasto_pseudo_density: NULL argument");
    // a batch has one atom table of n_atoms per right-hand side, back to back
    const int nb = g->n_batch;
    AtomDev* dat = nullptr;
    if (lasto_status st = stage_atoms(g, nb * n_atoms, atoms, renormalize, "lasto_pseudo_density", &dat);
        st != LASTO_OK)
        return st;
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    for (int b = 0; b < nb; ++b) {
        LASTO_HIP(launch_pseudo(g, dat + (size_t)b * n_atoms, n_atoms, rho_interstitial ? rho_interstitial + b * N : nullptr,
                                rho_out + b * N));
        if (moments_out) LASTO_HIP(launch_moments(g, rho_out + b * N, g->moments + 25 * b));
    }
    if (moments_out)
        LASTO_HIP(hipMemcpyAsync(moments_out, g->moments, sizeof(double) * 25 * nb, hipMemcpyDeviceToHost, g->stream));
    // the staging buffer is reused by the next call: finish before returning
    LASTO_HIP(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_analytic_guess(lasto_grid g, int n_atoms, const lasto_atom* atoms, double* v)
{
    if (!g || !v || n_atoms < 0 || (n_atoms > 0 && !atoms))
        return fail(LASTO_ERR_ARG, "lasto_analytic_guess: NULL argument");
    const int nb = g->n_batch;
    AtomDev* dat = nullptr;
    if (lasto_status st = stage_atoms(g, nb * n_atoms, atoms, 1, "lasto_analytic_guess", &dat); st != LASTO_OK)
        return st;
    LASTO_HIP(launch_guess_all(g, dat, atoms, n_atoms, v));
    LASTO_HIP(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

// The 64 default directions of the sphere values: 8 Gauss-Legendre nodes in
// cos(theta) (roots of P_8 by Newton, ascending) times 8 azimuths
// 2 pi (b + 1/2)/8, theta-major; d[3 k + c].
static void default_directions(double* d)
{
    double t[8];
    for (int a = 0; a < 8; ++a) {
        double xx = std::cos(kPi * (a + 0.75) / 8.5);
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = xx;
            for (int k = 2; k <= 8; ++k) {
                const double p2 = ((2.0 * k - 1.0) * xx * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = 8.0 * (xx * p1 - p0) / (xx * xx - 1.0);
            const double dx = p1 / dp;
            xx -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        t[a] = xx;
    }
    std::sort(t, t + 8);
    for (int a = 0; a < 8; ++a) {
        const double st = std::sqrt(std::max(0.0, 1.0 - t[a] * t[a]));
        for (int b = 0; b < 8; ++b) {
            const double ph = 2.0 * kPi * (b + 0.5) / 8.0;
            double* o = d + 3 * (8 * a + b);
            o[0] = st * std::cos(ph);
            o[1] = st * std::sin(ph);
            o[2] = t[a];
        }
    }
}

// sphere point C_a + R_a d_k, component c (the product rounded, then the sum)
static inline double sphere_point(const double* centers, const double* radii, const double* d, int a, int k, int c)
{
    return centers[3 * a + c] + radii[a] * d[3 * k + c];
}

// every sphere point inside the box of level 0
static lasto_status check_sphere_points(lasto_grid g, int n_atoms, const double* centers, const double* radii,
                                        int n_dir, const double* d, const char* who)
{
    const Level& L0 = g->lev[0];
    for (int a = 0; a < n_atoms; ++a)
        for (int k = 0; k < n_dir; ++k)
            for (int c = 0; c < 3; ++c) {
                const double p = sphere_point(centers, radii, d, a, k, c);
                if (!std::isfinite(p) || p < L0.hx[c].front() || p > L0.hx[c].back())
                    return fail(LASTO_ERR_ARG, std::string(who) + ": point outside the box");
            }
    return LASTO_OK;
}

extern "C" lasto_status lasto_sphere_interp(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                            const double* radii, int n_dir, const double* dirs, double* out)
{
    if (!g || !v || !out || n_atoms < 0 || (n_atoms > 0 && (!centers || !radii)))
        return fail(LASTO_ERR_ARG, "lasto_sphere_interp: NULL argument");
    std::vector<double> d;
    if (dirs) {
        if (n_dir < 1) return fail(LASTO_ERR_ARG, "lasto_sphere_interp: n_dir must be >= 1");
        d.assign(dirs, dirs + 3 * (size_t)n_dir);
    } else {
        if (n_dir != 64) return fail(LASTO_ERR_ARG, "lasto_sphere_interp: default directions need n_dir = 64");
        d.resize(3 * 64);
        default_directions(d.data());
    }
    const size_t np = (size_t)n_atoms * n_dir;
    if (np == 0) return LASTO_OK;
    if (lasto_status e = check_sphere_points(g, n_atoms, centers, radii, n_dir, d.data(), "lasto_sphere_interp");
        e != LASTO_OK)
        return e;
    std::vector<double> pts(3 * np);
    for (int a = 0; a < n_atoms; ++a)
        for (int k = 0; k < n_dir; ++k)
            for (int c = 0; c < 3; ++c) pts[3 * ((size_t)a * n_dir + k) + c] = sphere_point(centers, radii, d.data(), a, k, c);
    const size_t bytes = sizeof(double) * 4 * np;
    if (bytes > g->stage_bytes) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipFree(g->stage);
        g->stage = nullptr;
        LASTO_HIP(hipMalloc(&g->stage, bytes));
        g->stage_bytes = bytes;
    }
    double* dpts = g->stage;
    double* dout = g->stage + 3 * np;
    LASTO_HIP(hipMemcpyAsync(dpts, pts.data(), sizeof(double) * 3 * np, hipMemcpyHostToDevice, g->stream));
    // each right-hand side of a batch in turn (same points, its own values)
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    for (int b = 0; b < g->n_batch; ++b) {
        LASTO_HIP(launch_interp(g, v + b * N, dpts, (int)np, dout));
        LASTO_HIP(hipMemcpyAsync(out + b * np, dout, sizeof(double) * np, hipMemcpyDeviceToHost, g->stream));
        LASTO_HIP(hipStreamSynchronize(g->stream));
    }
    return LASTO_OK;
}

// ------------------------------------------- allocation-free sphere values
// Staging of lasto_sphere_interp_noalloc in one static device array per GPU:
// [points 3P][values P][directions 3P][centres 3P][radii P] doubles,
// P = LASTO_NOALLOC_MAX_POINTS (n_dir <= P and n_atoms <= P, since both are at
// least 1 and their product is at most P). Every region is written before it
// is read, so nothing needs clearing between calls.
constexpr size_t kNaPts = 0, kNaVals = 3 * (size_t)LASTO_NOALLOC_MAX_POINTS,
                 kNaDirs = 4 * (size_t)LASTO_NOALLOC_MAX_POINTS, kNaCent = 7 * (size_t)LASTO_NOALLOC_MAX_POINTS,
                 kNaRad = 10 * (size_t)LASTO_NOALLOC_MAX_POINTS, kNaTotal = 11 * (size_t)LASTO_NOALLOC_MAX_POINTS;
static __device__ __align__(256) double scratch[kNaTotal];

// The device address of `scratch` on each device, taken once per device with
// that device current (the host-side name is not a device address).
constexpr int kNaMaxDevices = 64;
static std::mutex g_na_mutex;
static double* g_na_ptr[kNaMaxDevices] = {};

static lasto_status noalloc_scratch(int device, double** out)
{
    if (device < 0 || device >= kNaMaxDevices) return fail(LASTO_ERR_ARG, "noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[device]) {
        int cur = 0;
        LASTO_HIP(hipGetDevice(&cur));
        if (cur != device) LASTO_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(LASTO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_na_ptr[device] = (double*)p;
    }
    *out = g_na_ptr[device];
    return LASTO_OK;
}

// p[3 t + c] = centre[3 a + c] + radius[a] dir[3 k + c], t = a n_dir + k: the
// points the host path forms (product rounded, then the sum; no fused multiply-add)
__global__ __launch_bounds__(64) void k_sphere_points(const double* __restrict__ cen, const double* __restrict__ rad,
                                                      const double* __restrict__ dir, int n_dir, int np,
                                                      double* __restrict__ pts)
{
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    const int a = t / n_dir, k = t - a * n_dir;
    for (int c = 0; c < 3; ++c) {
        const double prod = rad[a] * dir[3 * k + c];
        pts[3 * t + c] = cen[3 * a + c] + prod;
    }
}

extern "C" lasto_status lasto_sphere_interp_noalloc(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                                    const double* radii, int n_dir, const double* dirs, double* out)
{
    const char* who = "lasto_sphere_interp_noalloc";
    if (!g || !v || !out || n_atoms < 0 || (n_atoms > 0 && (!centers || !radii)))
        return fail(LASTO_ERR_ARG, std::string(who) + ": NULL argument");
    double dflt[3 * 64];
    const double* d = dirs;
    if (dirs) {
        if (n_dir < 1) return fail(LASTO_ERR_ARG, std::string(who) + ": n_dir must be >= 1");
    } else {
        if (n_dir != 64) return fail(LASTO_ERR_ARG, std::string(who) + ": default directions need n_dir = 64");
        default_directions(dflt);
        d = dflt;
    }
    const long long np = (long long)n_atoms * n_dir;
    if (np == 0) return LASTO_OK;
    if (np > LASTO_NOALLOC_MAX_POINTS)
        return fail(LASTO_ERR_ARG, std::string(who) + ": n_atoms * n_dir exceeds LASTO_NOALLOC_MAX_POINTS (" +
                                       std::to_string(LASTO_NOALLOC_MAX_POINTS) + ")");
    if (lasto_status e = check_sphere_points(g, n_atoms, centers, radii, n_dir, d, who); e != LASTO_OK) return e;
    double* S = nullptr;
    if (lasto_status e = noalloc_scratch(g->device, &S); e != LASTO_OK) return e;
    hipStream_t s = g->stream;
    LASTO_HIP(hipMemcpyAsync(S + kNaDirs, d, sizeof(double) * 3 * n_dir, hipMemcpyHostToDevice, s));
    LASTO_HIP(hipMemcpyAsync(S + kNaCent, centers, sizeof(double) * 3 * n_atoms, hipMemcpyHostToDevice, s));
    LASTO_HIP(hipMemcpyAsync(S + kNaRad, radii, sizeof(double) * n_atoms, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sphere_points, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, s, (const double*)(S + kNaCent),
                       (const double*)(S + kNaRad), (const double*)(S + kNaDirs), n_dir, (int)np, S + kNaPts);
    LASTO_HIP(hipGetLastError());
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    for (int b = 0; b < g->n_batch; ++b) {
        LASTO_HIP(launch_interp(g, v + b * N, S + kNaPts, (int)np, S + kNaVals));
        LASTO_HIP(hipMemcpyAsync(out + b * np, S + kNaVals, sizeof(double) * np, hipMemcpyDeviceToHost, s));
        // the values region is reused by the next copy; the host inputs
        // (default directions on this stack frame) stay alive until here
        LASTO_HIP(hipStreamSynchronize(s));
    }
    return LASTO_OK;
}
