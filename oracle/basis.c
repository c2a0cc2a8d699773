/*
 * CPU oracle, part three: the output density in the interstitial region --
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c: plain FP64 C, loaded only
 * by the tests, the smoke check and the benchmark's CPU-baseline leg; no code
 * shared with the GPU path).
 *
 * What it computes (Section 3, the density update after the eigenproblem,
 * and the basis of eq. (3.13); the interstitial matrix elements of
 * eq. (3.11)-(3.14) at the end of the file):
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

/* ------------------------------------------------ matrix elements on the grid */

/* -1/2 Laplacian of phi_(n l m) about its centre (eq. (3.14)):
 *   1/2 [ (l(l+1) - n(n-1)) r^(n-3) + 2 zeta n r^(n-2) - zeta^2 r^(n-1) ] exp(-zeta r) y_lm,
 * written with S_lm = r^l y_lm (the first term vanishes for n = l + 1). */
static double kinetic_radial(int n, int l, double zeta, double r)
{
    double e = exp(-zeta * r);
    double t = -zeta * zeta * pow(r, n - 1 - l) + 2.0 * zeta * n * pow(r, n - 2 - l);
    if (n != l + 1) t += (double)(l * (l + 1) - n * (n - 1)) * pow(r, n - 3 - l);
    return 0.5 * t * e;
}

/* phi_mu and (-1/2 Laplacian + V) phi_mu at points (V given per point):
 * phi, tphi [npts][n_basis] */
int oracle_basis_points(int n_atoms, const double* centers, int n_shells, const int* n, const int* l,
                        const double* zeta, int npts, const double* pts, const double* vpts, double* phi,
                        double* tphi)
{
    for (int t = 0; t < n_shells; ++t)
        if (l[t] < 0 || l[t] > 4 || n[t] < l[t] + 1) return 1;
    int nb = n_atoms * basis_per_atom(n_shells, l);
    for (int p = 0; p < npts; ++p) {
        double* ph = phi + (size_t)p * nb;
        double* tp = tphi + (size_t)p * nb;
        basis_values(pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], n_atoms, centers, n_shells, n, l, zeta, ph);
        int mu = 0;
        for (int a = 0; a < n_atoms; ++a) {
            double dx = pts[3 * p] - centers[3 * a], dy = pts[3 * p + 1] - centers[3 * a + 1];
            double dz = pts[3 * p + 2] - centers[3 * a + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double S[25];
            oracle_solid_harmonics(dx, dy, dz, S);
            for (int t = 0; t < n_shells; ++t) {
                double kr = kinetic_radial(n[t], l[t], zeta[t], r);
                for (int m = -l[t]; m <= l[t]; ++m, ++mu)
                    tp[mu] = kr * S[l[t] * l[t] + l[t] + m] + vpts[p] * ph[mu];
            }
        }
    }
    return 0;
}

/* The interstitial parts of S and H by grid quadrature (eq. (3.11)-(3.12)
 * with the nodes of the graded grid and their dual volumes, the form S^1 /
 * H^1 under eq. (3.14)):
 *   S[mu][nu] = sum_P vol_P phi_mu(P) phi_nu(P),
 *   H[mu][nu] = 1/2 sum_P vol_P (phi_mu(P) tphi_nu(P) + phi_nu(P) tphi_mu(P)),
 * over the nodes P outside every sphere, tphi = (-1/2 Laplacian + V) phi.
 * v [nz][ny][nx]; S, H [n_basis][n_basis]. */
int oracle_matrix_elements(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                           const double* v, int n_atoms, const double* centers, const double* radii, int n_shells,
                           const int* n, const int* l, const double* zeta, double* S, double* H)
{
    for (int t = 0; t < n_shells; ++t)
        if (l[t] < 0 || l[t] > 4 || n[t] < l[t] + 1) return 1;
    int nb = n_atoms * basis_per_atom(n_shells, l);
    double* ph = malloc(sizeof(double) * nb);
    double* tp = malloc(sizeof(double) * nb);
    for (size_t e = 0; e < (size_t)nb * nb; ++e) { S[e] = 0.0; H[e] = 0.0; }
    for (int k = 0; k < nz; ++k) {
        double mz = 0.5 * ((k + 1 < nz ? z[k + 1] : z[k]) - (k > 0 ? z[k - 1] : z[k]));
        for (int j = 0; j < ny; ++j) {
            double my = 0.5 * ((j + 1 < ny ? y[j + 1] : y[j]) - (j > 0 ? y[j - 1] : y[j]));
            for (int i = 0; i < nx; ++i) {
                double mx = 0.5 * ((i + 1 < nx ? x[i + 1] : x[i]) - (i > 0 ? x[i - 1] : x[i]));
                int outside = 1;
                for (int a = 0; a < n_atoms; ++a) {
                    double dx = x[i] - centers[3 * a], dy = y[j] - centers[3 * a + 1], dz = z[k] - centers[3 * a + 2];
                    volatile double sx = dx * dx, sy = dy * dy, sz = dz * dz;   /* no contraction */
                    if (sx + sy + sz < radii[a] * radii[a]) { outside = 0; break; }
                }
                if (!outside) continue;
                double p[3] = {x[i], y[j], z[k]};
                double vp = v[((size_t)k * ny + j) * nx + i];
                oracle_basis_points(n_atoms, centers, n_shells, n, l, zeta, 1, p, &vp, ph, tp);
                double vol = mx * my * mz;
                for (int mu = 0; mu < nb; ++mu)
                    for (int nu = 0; nu < nb; ++nu) {
                        S[(size_t)mu * nb + nu] += vol * ph[mu] * ph[nu];
                        H[(size_t)mu * nb + nu] += 0.5 * vol * (ph[mu] * tp[nu] + ph[nu] * tp[mu]);
                    }
            }
        }
    }
    free(ph);
    free(tp);
    return 0;
}
