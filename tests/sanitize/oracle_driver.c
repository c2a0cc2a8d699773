/* Runs every oracle entry point once on small synthetic inputs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds
 * access, use after free, leak or undefined operation aborts the program.
 * Exit status 0 when every call returned success and finite output. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_mesh_graded_1d(double lo, double hi, int n, const double* planes, int np, double hmin, double hmax,
                          double gmax, double hmin_step, double* x, double* g_out, double* hmin_out);
int oracle_pseudo_density(const double* x, int nx, const double* y, int ny, const double* z, int nz, int n_atoms,
                          const double* centers, const double* q, const double* width, const double* radius,
                          const double* alpha, const int* lmax, const double* clm, const int* kind,
                          const double* rho_R, const double* drho_R, const double* rho_inter, int renormalize,
                          double* rho);
void oracle_moments(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* rho,
                    int lmax_bc, const double* c, double* Q);
void oracle_boundary_values(const double* x, int nx, const double* y, int ny, const double* z, int nz, int bc_mode,
                            const double* Q, int lmax_bc, const double* c, double* v);
void oracle_apply(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* u,
                  double* Au);
int oracle_hierarchy_sizes(const double* x, int nx, const double* y, int ny, const double* z, int nz, double theta,
                           int coarse_max, int* sizes, int max_levels);
int oracle_solve(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* rho,
                 double* v, double rtol, int max_cycles, int nu1, int nu2, double theta, int coarse_max, double* rel,
                 double* hist);
double oracle_rel_residual(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                           const double* rho, const double* v);
int oracle_interp(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* v,
                  int npts, const double* pts, double* out);
void oracle_rb_sweep(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* u,
                     const double* rho, int first, double* out);
int oracle_sphere_rule(int n_theta, int n_phi, double* dirs, double* weights);
int oracle_sphere_project(int n_atoms, int n_theta, int n_phi, const double* values, double* out);
int oracle_sphere_radial(int n_atoms, const double* radii, const double* Z, int n_rad, double r_min,
                         const double* vlm_R, const double* rho_lm, double* vlm);
int oracle_sphere_energy(int n_atoms, const double* radii, int n_rad, double r_min, const double* vlm,
                         const double* rho_lm, double* out);
double oracle_energy_grid(const double* x, int nx, const double* y, int ny, const double* z, int nz, const double* v,
                          const double* rho, int n_atoms, const double* centers, const double* radii);
int oracle_sphere_density_terms(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                                int n_atoms, const double* centers, const double* radii, int n_rad, double r_min,
                                const double* rho_lm, int lmin, double* rho);
int oracle_density_points(int n_atoms, const double* centers, int n_shells, const int* n, const int* l,
                          const double* zeta, int n_occ, const double* coef, const double* occ, int npts,
                          const double* pts, double* out);
int oracle_interstitial_density(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                                int n_atoms, const double* centers, const double* radii, int n_shells, const int* n,
                                const int* l, const double* zeta, int n_occ, const double* coef, const double* occ,
                                double* rho);
int oracle_basis_points(int n_atoms, const double* centers, int n_shells, const int* n, const int* l,
                        const double* zeta, int npts, const double* pts, const double* vpts, double* phi,
                        double* tphi);
int oracle_matrix_elements(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                           const double* v, int n_atoms, const double* centers, const double* radii, int n_shells,
                           const int* n, const int* l, const double* zeta, double* S, double* H);

static int failures = 0;

static void check(int ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static int all_finite(const double* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static double* zeros(size_t n)
{
    double* p = calloc(n, sizeof(double));
    if (!p) abort();
    return p;
}

enum { NA = 2, NX = 19, NY = 17, NZ = 21, NLM = 25, NRAD = 40, NT = 8, NP = 16 };

int main(void)
{
    const double L = 8.0;
    const double centers[NA * 3] = {-1.0, 0.3, -0.2, 1.1, -0.4, 0.5};
    double x[NX], y[NY], z[NZ], g, hmin;
    const double px[NA] = {-1.0, 1.1}, py[NA] = {0.3, -0.4}, pz[NA] = {-0.2, 0.5};
    check(oracle_mesh_graded_1d(-L, L, NX, px, NA, 0.4, 1.5, 1.3, 0.05, x, &g, &hmin) == 0, "graded mesh x");
    check(oracle_mesh_graded_1d(-L, L, NY, py, NA, 0.4, 1.5, 1.3, 0.05, y, &g, &hmin) == 0, "graded mesh y");
    check(oracle_mesh_graded_1d(-L, L, NZ, pz, 0, 0.0, 0.0, 0.0, 0.0, z, &g, &hmin) == 0, "uniform mesh z");
    check(oracle_mesh_graded_1d(-L, L, 2, px, NA, 0.4, 1.5, 1.3, 0.0, x, &g, &hmin) != 0, "mesh rejects n < 3");

    const size_t N = (size_t)NX * NY * NZ;
    const double q[NA] = {2.0, 3.0}, width[NA] = {0.5, 0.6}, radius[NA] = {1.2, 1.3}, alpha[NA] = {1.0, 1.1};
    const int lmax[NA] = {2, 4}, kind[NA] = {0, 1};
    double clm[NA * 24];
    for (int i = 0; i < NA * 24; ++i) clm[i] = 0.01 * (double)((i % 7) - 3);
    const double rho_R[NA] = {0.0, 0.02}, drho_R[NA] = {0.0, -0.05};
    double* rho_inter = zeros(N);
    for (size_t t = 0; t < N; ++t) rho_inter[t] = 1e-3 * (double)(t % 5);
    double* rho = zeros(N);
    check(oracle_pseudo_density(x, NX, y, NY, z, NZ, NA, centers, q, width, radius, alpha, lmax, clm, kind, rho_R,
                                drho_R, rho_inter, 1, rho) == 0 && all_finite(rho, N), "pseudo-density");

    const double c[3] = {0.0, 0.0, 0.0};
    double Q[NLM];
    oracle_moments(x, NX, y, NY, z, NZ, rho, 4, c, Q);
    check(all_finite(Q, NLM), "moments");
    double* v = zeros(N);
    oracle_boundary_values(x, NX, y, NY, z, NZ, 1, Q, 4, c, v);
    check(all_finite(v, N), "boundary values");

    int sizes[3 * 16];
    const int nl = oracle_hierarchy_sizes(x, NX, y, NY, z, NZ, 4.0, 5, sizes, 16);
    check(nl >= 1 && nl <= 16, "hierarchy sizes");

    double rel = 1.0, hist[128];
    const int cyc = oracle_solve(x, NX, y, NY, z, NZ, rho, v, 1e-10, 60, 2, 2, 4.0, 5, &rel, hist);
    check(cyc > 0 && rel <= 1e-10 && all_finite(v, N), "solve");
    check(oracle_rel_residual(x, NX, y, NY, z, NZ, rho, v) <= 1e-10, "relative residual");

    double* Au = zeros(N);
    oracle_apply(x, NX, y, NY, z, NZ, v, Au);
    check(all_finite(Au, N), "apply");
    oracle_rb_sweep(x, NX, y, NY, z, NZ, v, rho, 0, Au);
    oracle_rb_sweep(x, NX, y, NY, z, NZ, v, rho, 1, Au);
    check(all_finite(Au, N), "red-black sweep");

    double dirs[NT * NP * 3], w[NT * NP];
    check(oracle_sphere_rule(NT, NP, dirs, w) == 0, "sphere rule");
    double pts[NA * NT * NP * 3];
    for (int a = 0; a < NA; ++a)
        for (int k = 0; k < NT * NP; ++k)
            for (int d = 0; d < 3; ++d)
                pts[(a * NT * NP + k) * 3 + d] = centers[a * 3 + d] + radius[a] * dirs[k * 3 + d];
    double vs[NA * NT * NP];
    check(oracle_interp(x, NX, y, NY, z, NZ, v, NA * NT * NP, pts, vs) == 0 && all_finite(vs, NA * NT * NP),
          "sphere interpolation");
    double vlm_R[NA * NLM];
    check(oracle_sphere_project(NA, NT, NP, vs, vlm_R) == 0 && all_finite(vlm_R, NA * NLM), "sphere projection");

    const double Z[NA] = {46.0, 46.0};
    double* rho_lm = zeros((size_t)NA * NLM * NRAD);
    for (size_t i = 0; i < (size_t)NA * NLM * NRAD; ++i) rho_lm[i] = 0.05 * exp(-0.01 * (double)(i % NRAD));
    double* vlm = zeros((size_t)NA * NLM * NRAD);
    check(oracle_sphere_radial(NA, radius, Z, NRAD, 1e-5, vlm_R, rho_lm, vlm) == 0 &&
              all_finite(vlm, (size_t)NA * NLM * NRAD),
          "radial solve");
    double e[NA];
    check(oracle_sphere_energy(NA, radius, NRAD, 1e-5, vlm, rho_lm, e) == 0 && all_finite(e, NA), "sphere energy");
    check(isfinite(oracle_energy_grid(x, NX, y, NY, z, NZ, v, rho, NA, centers, radius)), "grid energy");
    check(oracle_sphere_density_terms(x, NX, y, NY, z, NZ, NA, centers, radius, NRAD, 1e-5, rho_lm, 1, rho) == 0 &&
              all_finite(rho, N),
          "sphere density terms");

    /* interstitial basis: shells (n, l, zeta) on every atom */
    enum { NS = 3, NOCC = 4 };
    const int sn[NS] = {1, 2, 3}, sl[NS] = {0, 1, 2};
    const double sz[NS] = {1.3, 0.9, 0.7};
    const int nb = NA * (1 + 3 + 5);
    double* coef = zeros((size_t)nb * NOCC);
    for (int i = 0; i < nb * NOCC; ++i) coef[i] = 0.1 * (double)((i % 9) - 4);
    const double occ[NOCC] = {2.0, 2.0, 1.0, 0.5};
    double dens[NA * NT * NP];
    check(oracle_density_points(NA, centers, NS, sn, sl, sz, NOCC, coef, occ, NA * NT * NP, pts, dens) == 0 &&
              all_finite(dens, NA * NT * NP),
          "density at points");
    double* rint = zeros(N);
    check(oracle_interstitial_density(x, NX, y, NY, z, NZ, NA, centers, radius, NS, sn, sl, sz, NOCC, coef, occ,
                                      rint) == 0 &&
              all_finite(rint, N),
          "interstitial density");
    double* phi = zeros((size_t)NA * NT * NP * nb);
    double* tphi = zeros((size_t)NA * NT * NP * nb);
    check(oracle_basis_points(NA, centers, NS, sn, sl, sz, NA * NT * NP, pts, vs, phi, tphi) == 0 &&
              all_finite(phi, (size_t)NA * NT * NP * nb) && all_finite(tphi, (size_t)NA * NT * NP * nb),
          "basis at points");
    double* S = zeros((size_t)nb * nb);
    double* H = zeros((size_t)nb * nb);
    check(oracle_matrix_elements(x, NX, y, NY, z, NZ, v, NA, centers, radius, NS, sn, sl, sz, S, H) == 0 &&
              all_finite(S, (size_t)nb * nb) && all_finite(H, (size_t)nb * nb),
          "matrix elements");

    free(rho_inter); free(rho); free(v); free(Au); free(rho_lm); free(vlm); free(coef); free(rint);
    free(phi); free(tphi); free(S); free(H);
    if (failures) return 1;
    printf("oracle driver: every entry point ran clean\n");
    return 0;
}
