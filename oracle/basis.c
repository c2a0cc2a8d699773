/*
 * CPU oracle, part three: the output density in the interstitial region --
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c: plain FP64 C, loaded only
 * by the tests, the smoke check and the benchmark's CPU-baseline leg; no code
 * shared with the GPU path).
 *
 * What it computes (Section 3, the density update after the eigenproblem,
 * and the basis of eq. (3.13)):
 *   rho_out(x) = sum_k f_k psi_k(x)^2,   psi_k(x) = sum_mu c_(mu,k) phi_mu(x),
 *   phi_(i n l m)(x) = r_i^(n-1) exp(-zeta r_i) y_lm(r_i / |r_i|),  r_i = x - C_i,
 * at the grid nodes outside every sphere (|x - C_i|^2 >= R_i^2, squares and
 * sums rounded as written), zero at nodes inside one. Written with the solid
 * harmonic S_lm(r) = |r|^l y_lm(r/|r|) as |r|^(n-1-l) exp(-zeta |r|) S_lm(r)
 * (n >= l + 1), which is defined at r = 0 too.
 *
 * Readings: the paper sums |phi_k|^2 over the states below the Fermi level;
 * here each state carries an occupation f_k (2 for a doubly occupied state),
 * the coefficients are real (real basis, real symmetric H and S), and the
 * basis is the same list of shells (n, l, zeta) on every atom, ordered
 * atom-major, then shell, then m = -l..l.
 *
 * Layouts: coef [n_basis][n_occ] (a basis function's coefficients over the
 * states are contiguous), occ [n_occ], rho [nz][ny][nx].
 */
#include <math.h>
#include <stdlib.h>

void oracle_solid_harmonics(double x, double y, double z, double* S);   /* oracle.c */

static int basis_per_atom(int n_shells, const int* l)
{
    int s = 0;
    for (int t = 0; t < n_shells; ++t) s += 2 * l[t] + 1;
    return s;
}

/* phi_mu at point p for every basis function mu (out: [n_atoms * per atom]) */
static void basis_values(double px, double py, double pz, int n_atoms, const double* centers, int n_shells,
                         const int* n, const int* l, const double* zeta, double* out)
{
    int mu = 0;
    for (int a = 0; a < n_atoms; ++a) {
        double dx = px - centers[3 * a], dy = py - centers[3 * a + 1], dz = pz - centers[3 * a + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double S[25];
        oracle_solid_harmonics(dx, dy, dz, S);
        for (int t = 0; t < n_shells; ++t) {
            double radial = pow(r, n[t] - 1 - l[t]) * exp(-zeta[t] * r);
            for (int m = -l[t]; m <= l[t]; ++m) out[mu++] = radial * S[l[t] * l[t] + l[t] + m];
        }
    }
}

/* rho_out at arbitrary points (no sphere test): pts [npts][3], out [npts] */
int oracle_density_points(int n_atoms, const double* centers, int n_shells, const int* n, const int* l,
                          const double* zeta, int n_occ, const double* coef, const double* occ, int npts,
                          const double* pts, double* out)
{
    for (int t = 0; t < n_shells; ++t)
        if (l[t] < 0 || l[t] > 4 || n[t] < l[t] + 1) return 1;
    int nb = n_atoms * basis_per_atom(n_shells, l);
    double* phi = malloc(sizeof(double) * (nb > 0 ? nb : 1));
    for (int p = 0; p < npts; ++p) {
        basis_values(pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], n_atoms, centers, n_shells, n, l, zeta, phi);
        double rho = 0.0;
        for (int k = 0; k < n_occ; ++k) {
            double psi = 0.0;
            for (int mu = 0; mu < nb; ++mu) psi += coef[(size_t)mu * n_occ + k] * phi[mu];
            rho += occ[k] * psi * psi;
        }
        out[p] = rho;
    }
    free(phi);
    return 0;
}

/* rho_out on the grid nodes, zero inside the spheres (radii may be all zero) */
int oracle_interstitial_density(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                                int n_atoms, const double* centers, const double* radii, int n_shells,
                                const int* n, const int* l, const double* zeta, int n_occ, const double* coef,
                                const double* occ, double* rho)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t at = ((size_t)k * ny + j) * nx + i;
                int outside = 1;
                for (int a = 0; a < n_atoms; ++a) {
                    double dx = x[i] - centers[3 * a], dy = y[j] - centers[3 * a + 1], dz = z[k] - centers[3 * a + 2];
                    volatile double sx = dx * dx, sy = dy * dy, sz = dz * dz;   /* no contraction */
                    if (sx + sy + sz < radii[a] * radii[a]) { outside = 0; break; }
                }
                rho[at] = 0.0;
                if (outside) {
                    double p[3] = {x[i], y[j], z[k]};
                    int rc = oracle_density_points(n_atoms, centers, n_shells, n, l, zeta, n_occ, coef, occ, 1, p,
                                                   &rho[at]);
                    if (rc) return rc;
                }
            }
    return 0;
}
