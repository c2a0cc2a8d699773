// Sphere sets: the interior solve of eq. (3.4)-(3.7) and the energy integral
// (host side of the C ABI; the kernels live in src_kernels.hip).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

using namespace lasto;

struct lasto_spheres_s {
    lasto_grid g = nullptr;
    int n_atoms = 0;
    int npts = 0;
    int n_rad = 0;
    SphereAtom* atoms = nullptr;   // device [n_atoms]
    double4* rule = nullptr;       // device [npts]: direction, weight
    int nparts = 0;                // grid partials per copy
    double* partials = nullptr;    // device [n_batch][nparts]
    double* e_row = nullptr;       // device [n_batch][n_atoms][25]
    double* e_dev = nullptr;       // device [n_batch][2]
    double* e_host = nullptr;      // pinned [n_batch][2]
};

namespace {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton on P_n from
// cos(pi (n - a - 1/4) / (n + 1/2)); weights 2 / ((1 - t^2) P_n'(t)^2).
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w)
{
    t.resize(n);
    w.resize(n);
    for (int a = 0; a < n; ++a) {
        double x = std::cos(kPi * (n - a - 0.25) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        t[a] = x;
        w[a] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

void free_spheres(lasto_spheres s)
{
    if (!s) return;
    (void)hipFree(s->atoms);
    (void)hipFree(s->rule);
    (void)hipFree(s->partials);
    (void)hipFree(s->e_row);
    (void)hipFree(s->e_dev);
    if (s->e_host) (void)hipHostFree(s->e_host);
    delete s;
}

}  // namespace

extern "C" lasto_status lasto_spheres_create(lasto_grid g, int n_atoms, const double* centers, const double* radii,
                                             const double* Z, int n_theta, int n_phi, int n_rad, double r_min,
                                             lasto_spheres* out)
{
    if (!g || !out || !centers || !radii || n_atoms < 1)
        return fail(LASTO_ERR_ARG, "lasto_spheres_create: NULL argument or no atoms");
    *out = nullptr;
    if (n_atoms > 65535) return fail(LASTO_ERR_ARG, "lasto_spheres_create: at most 65535 atoms");
    if (n_theta < 5 || n_theta > 64 || n_phi < 9 || n_phi > 1024 || n_theta * n_phi > 8192)
        return fail(LASTO_ERR_ARG, "lasto_spheres_create: need 5 <= n_theta <= 64, 9 <= n_phi <= 1024, "
                                   "n_theta * n_phi <= 8192");
    if (n_rad < 8 || n_rad > 1024) return fail(LASTO_ERR_ARG, "lasto_spheres_create: need 8 <= n_rad <= 1024");
    if (!(r_min > 0.0) || !std::isfinite(r_min)) return fail(LASTO_ERR_ARG, "lasto_spheres_create: r_min must be > 0");
    const Level& L0 = g->lev[0];
    std::vector<SphereAtom> at(n_atoms);
    for (int a = 0; a < n_atoms; ++a) {
        SphereAtom& A = at[a];
        A = SphereAtom{};
        A.R = radii[a];
        A.Z = Z ? Z[a] : 0.0;
        if (!std::isfinite(A.R) || !(A.R > r_min) || !std::isfinite(A.Z))
            return fail(LASTO_ERR_ARG, "lasto_spheres_create: radius must exceed r_min, Z finite");
        for (int c = 0; c < 3; ++c) {
            A.c[c] = centers[3 * a + c];
            if (!std::isfinite(A.c[c]) || A.c[c] - A.R < L0.hx[c].front() || A.c[c] + A.R > L0.hx[c].back())
                return fail(LASTO_ERR_ARG, "lasto_spheres_create: a sphere reaches outside the box");
        }
        A.D = std::log(A.R / r_min) / (n_rad - 1);
    }
    for (int a = 0; a < n_atoms; ++a)
        for (int b = a + 1; b < n_atoms; ++b) {
            const double dx = at[a].c[0] - at[b].c[0], dy = at[a].c[1] - at[b].c[1], dz = at[a].c[2] - at[b].c[2];
            if (std::sqrt(dx * dx + dy * dy + dz * dz) < at[a].R + at[b].R)
                return fail(LASTO_ERR_ARG, "lasto_spheres_create: spheres overlap");
        }
    std::vector<double> t, w;
    gauss_legendre(n_theta, t, w);
    std::vector<double4> rule((size_t)n_theta * n_phi);
    for (int a = 0; a < n_theta; ++a) {
        const double st = std::sqrt(1.0 - t[a] * t[a]);
        for (int b = 0; b < n_phi; ++b) {
            const double ph = 2.0 * kPi * (b + 0.5) / n_phi;
            rule[(size_t)a * n_phi + b] = double4{st * std::cos(ph), st * std::sin(ph), t[a], w[a] * 2.0 * kPi / n_phi};
        }
    }
    const LevelView& V = g->cview;
    if ((double)V.nx * V.ny * V.nz >= 2147483647.0)
        return fail(LASTO_ERR_ARG, "lasto_spheres_create: a copy of the grid must hold fewer than 2^31 nodes");
    lasto_spheres s = new lasto_spheres_s;
    s->g = g;
    s->n_atoms = n_atoms;
    s->npts = n_theta * n_phi;
    s->n_rad = n_rad;
    s->nparts = energy_grid_blocks(V);
    const int nb = g->n_batch;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&s->atoms, sizeof(SphereAtom) * n_atoms);
    if (e == hipSuccess) e = hipMalloc(&s->rule, sizeof(double4) * rule.size());
    if (e == hipSuccess) e = hipMalloc(&s->partials, sizeof(double) * (size_t)nb * s->nparts);
    if (e == hipSuccess) e = hipMalloc(&s->e_row, sizeof(double) * (size_t)nb * n_atoms * 25);
    if (e == hipSuccess) e = hipMalloc(&s->e_dev, sizeof(double) * 2 * nb);
    if (e == hipSuccess) e = hipHostMalloc(&s->e_host, sizeof(double) * 2 * nb, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_spheres(s);
        return fail(LASTO_ERR_ALLOC, std::string("lasto_spheres_create: ") + hipGetErrorString(e));
    }
    e = hipMemcpyAsync(s->atoms, at.data(), sizeof(SphereAtom) * n_atoms, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->rule, rule.data(), sizeof(double4) * rule.size(), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        free_spheres(s);
        return fail(LASTO_ERR_HIP, std::string("lasto_spheres_create: ") + hipGetErrorString(e));
    }
    *out = s;
    return LASTO_OK;
}

extern "C" lasto_status lasto_spheres_destroy(lasto_spheres s)
{
    if (!s) return LASTO_OK;
    (void)hipStreamSynchronize(s->g->stream);
    free_spheres(s);
    return LASTO_OK;
}

extern "C" lasto_status lasto_sphere_project(lasto_spheres s, const double* v, double* vlm_R)
{
    if (!s || !v || !vlm_R) return fail(LASTO_ERR_ARG, "lasto_sphere_project: NULL argument");
    LASTO_HIP(launch_sphere_project(s->g, v, s->atoms, s->n_atoms, s->rule, s->npts, vlm_R));
    return LASTO_OK;
}

extern "C" lasto_status lasto_sphere_radial(lasto_spheres s, const double* vlm_R, const double* rho_lm, double* v_lm)
{
    if (!s || !vlm_R || !rho_lm || !v_lm) return fail(LASTO_ERR_ARG, "lasto_sphere_radial: NULL argument");
    const size_t rows = (size_t)s->g->n_batch * s->n_atoms * 25;
    const char* o0 = (const char*)v_lm;
    const char* o1 = o0 + sizeof(double) * rows * s->n_rad;
    auto overlaps = [&](const void* p, size_t bytes) {
        const char* c = (const char*)p;
        return c < o1 && o0 < c + bytes;
    };
    if (overlaps(vlm_R, sizeof(double) * rows) || overlaps(rho_lm, sizeof(double) * rows * s->n_rad))
        return fail(LASTO_ERR_ARG, "lasto_sphere_radial: v_lm overlaps an input");
    LASTO_HIP(launch_radial_solve(s->g, s->atoms, s->n_atoms, s->n_rad, vlm_R, rho_lm, v_lm));
    return LASTO_OK;
}

extern "C" lasto_status lasto_sphere_energy(lasto_spheres s, const double* v, const double* rho, const double* v_lm,
                                            const double* rho_lm, double* e_out)
{
    if (!s || !v || !rho || !v_lm || !rho_lm || !e_out) return fail(LASTO_ERR_ARG, "lasto_sphere_energy: NULL argument");
    lasto_grid g = s->g;
    const int nb = g->n_batch;
    LASTO_HIP(launch_energy_grid(g, v, rho, s->atoms, s->n_atoms, s->partials));
    LASTO_HIP(launch_sphere_energy(g, s->atoms, s->n_atoms, s->n_rad, v_lm, rho_lm, s->e_row));
    LASTO_HIP(launch_energy_final(g, s->partials, s->nparts, s->e_row, s->n_atoms * 25, s->e_dev));
    LASTO_HIP(hipMemcpyAsync(s->e_host, s->e_dev, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, g->stream));
    LASTO_HIP(hipStreamSynchronize(g->stream));
    std::copy(s->e_host, s->e_host + 2 * nb, e_out);
    return LASTO_OK;
}

extern "C" lasto_status lasto_sphere_density_terms(lasto_spheres s, const double* rho_lm, int lmin, double* rho)
{
    if (!s || !rho_lm || !rho) return fail(LASTO_ERR_ARG, "lasto_sphere_density_terms: NULL argument");
    if (lmin < 0 || lmin > 4) return fail(LASTO_ERR_ARG, "lasto_sphere_density_terms: lmin must be 0..4");
    LASTO_HIP(launch_sphere_terms(s->g, s->atoms, s->n_atoms, s->n_rad, rho_lm, lmin, rho));
    return LASTO_OK;
}
