/*
 * CPU oracle, part two: inside the muffin-tin spheres -- TEST INFRASTRUCTURE
 * ONLY (same rules as oracle.c: plain FP64 C, loaded only by the tests, the
 * smoke check and the benchmark's CPU-baseline leg; no code shared with the
 * GPU path).
 *
 * What it computes (Section 3, eq. (3.4)-(3.7); the energy of Section 4,
 * eq. (4.1)):
 *   - the projection of V_C on a sphere boundary onto the real orthonormal
 *     harmonics y_LM, eq. (3.6), by a product rule on the unit sphere;
 *   - the interior solution of the radial equation (3.4) with that
 *     projection as Dirichlet data, written as the radial Green's function
 *     integrals under (3.4)-(3.5);
 *   - the tabulated non-spherical density put on the grid inside each sphere
 *     (the paper places the non-spherical terms directly on the grid; here
 *     from the same radial tables the interior solve uses);
 *   - the bilinear integral of V against the density over the whole domain:
 *     grid quadrature at nodes outside every sphere plus radial quadrature
 *     of sum_LM V_LM rho_LM inside each sphere (orthonormal y_LM turn the
 *     angular integral into that sum); half of it is the Hartree term of
 *     eq. (4.1) when V is the Hartree potential.
 *
 * Readings where the paper is silent or garbled:
 *   - Sign: eq. (3.2)/(3.4) solved literally, Laplacian(V) = +4 pi (rho - Z delta).
 *     The paper's printed interior formula carries the opposite overall sign;
 *     the form used here solves (3.4) as written: for L = 0 the nucleus adds
 *     sqrt(4 pi) Z (1/r - 1/R) (V = +Z/r near a nucleus of charge -Z in the
 *     rho - Z delta convention).
 *   - The garbled integrands "rho_LM(r')^(L+2)" and "rho_LM(r')^(L-l)" are
 *     read as rho_LM(r') r'^(L+2) and rho_LM(r') r'^(1-L), the radial
 *     Green's function of (3.4):
 *       V_LM(r) = V_LM(R) (r/R)^L
 *               - 4 pi/(2L+1) [ r^-(L+1) P(r) + r^L Q(r) - r^L P(R) / R^(2L+1) ]
 *               + delta_L0 sqrt(4 pi) Z (1/r - 1/R),
 *       P(r) = int_0^r rho_LM r'^(L+2) dr',  Q(r) = int_r^R rho_LM r'^(1-L) dr'.
 *   - eq. (3.6) integrates over the unit sphere (dOmega) against orthonormal
 *     y_LM; the rule is n_theta Gauss-Legendre nodes in cos(theta) times
 *     n_phi azimuths 2 pi (b + 1/2)/n_phi, theta-major. It integrates
 *     y_LM y_L'M' exactly for L, L' <= 4 when n_theta >= 5 and n_phi >= 9
 *     (eight azimuths would alias M = +-4 products).
 *   - Radial mesh (Section 4: logarithmic, 429 points; origin not given):
 *     r_k = R exp((k - (n - 1)) D), D = ln(R / r_min) / (n - 1), so r_0 = r_min
 *     and r_(n-1) = R. In t = ln r the mesh is uniform and dr = r dt.
 *   - Quadrature in t: each mesh interval [t_k, t_k+1] takes the integral of
 *     the cubic through four consecutive samples (k-1..k+2 inside,
 *     0..3 on the first interval, n-4..n-1 on the last), fourth order.
 *     The piece [0, r_0] is taken with rho_LM ~ r^L there:
 *     int_0^r0 rho r^(L+2) dr = rho(r_0) r_0^(L+3) / (2L+3); for the energy,
 *     int_0^r0 V rho r^2 dr = V(r_0) rho(r_0) r_0^3 / 3.
 *   - A node belongs to sphere a when |x_n - C_a|^2 < R_a^2 (the squares and
 *     sums in that order, no fused multiply-add); spheres do not overlap.
 *
 * LM index: L*L + L + M (M = -L..L), L <= 4, 25 entries; y_LM real,
 * orthonormal on the unit sphere, no Condon-Shortley phase (oracle.c).
 */
#include <math.h>
#include <stdlib.h>

#define PI 3.14159265358979323846
#define NLM 25

void oracle_solid_harmonics(double x, double y, double z, double* S);   /* oracle.c */

static int lm_degree(int lm)
{
    int L = 0;
    while ((L + 1) * (L + 1) <= lm) ++L;
    return L;
}

/* --------------------------------------------------------- angular rule */

/* Legendre P_n(t) and its derivative by the three-term recurrence */
static void legendre(int n, double t, double* p, double* dp)
{
    double p0 = 1.0, p1 = t;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (t * p1 - p0) / (t * t - 1.0);
}

/* Gauss-Legendre nodes (ascending) and weights on [-1, 1]: the roots of P_n
 * by Newton's method, weights 2 / ((1 - t^2) P_n'(t)^2). */
static void gauss_legendre(int n, double* t, double* w)
{
    for (int a = 0; a < n; ++a) {
        double x = cos(PI * (n - a - 0.25) / (n + 0.5));   /* ascending start values */
        double p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, x, &p, &dp);
            double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        legendre(n, x, &p, &dp);
        t[a] = x;
        w[a] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* Directions and weights of the product rule: point p = a * n_phi + b has
 * cos(theta) = t_a (Gauss-Legendre, ascending), phi = 2 pi (b + 1/2)/n_phi,
 * d = (sin cos phi, sin sin phi, cos theta), weight w_a 2 pi / n_phi. */
int oracle_sphere_rule(int n_theta, int n_phi, double* dirs, double* weights)
{
    if (n_theta < 1 || n_theta > 64 || n_phi < 1) return 1;
    double t[64], w[64];
    gauss_legendre(n_theta, t, w);
    for (int a = 0; a < n_theta; ++a) {
        double st = sqrt(1.0 - t[a] * t[a]);
        for (int b = 0; b < n_phi; ++b) {
            double ph = 2.0 * PI * (b + 0.5) / n_phi;
            int p = a * n_phi + b;
            dirs[3 * p] = st * cos(ph);
            dirs[3 * p + 1] = st * sin(ph);
            dirs[3 * p + 2] = t[a];
            weights[p] = w[a] * 2.0 * PI / n_phi;
        }
    }
    return 0;
}

/* eq. (3.6): V_LM(R_a) = int V(C_a + R_a d) y_LM(d) dOmega by the product
 * rule. values: [n_atoms][n_theta * n_phi] (V at C_a + R_a d_p, for
 * instance oracle_interp of the grid field); out: [n_atoms][25]. */
int oracle_sphere_project(int n_atoms, int n_theta, int n_phi, const double* values, double* out)
{
    int np = n_theta * n_phi;
    double* d = malloc(sizeof(double) * 3 * np);
    double* w = malloc(sizeof(double) * np);
    if (oracle_sphere_rule(n_theta, n_phi, d, w)) { free(d); free(w); return 1; }
    for (int a = 0; a < n_atoms; ++a) {
        for (int lm = 0; lm < NLM; ++lm) out[NLM * a + lm] = 0.0;
        for (int p = 0; p < np; ++p) {
            double y[NLM];
            oracle_solid_harmonics(d[3 * p], d[3 * p + 1], d[3 * p + 2], y);   /* |d| = 1: S_LM(d) = y_LM(d) */
            for (int lm = 0; lm < NLM; ++lm) out[NLM * a + lm] += w[p] * values[(size_t)a * np + p] * y[lm];
        }
    }
    free(d);
    free(w);
    return 0;
}

/* ---------------------------------------------------------- radial part */

double oracle_radial_node(double R, double r_min, int n, int k)
{
    double D = log(R / r_min) / (n - 1);
    return R * exp((k - (n - 1)) * D);
}

/* integral over [t_k, t_k+1] of the cubic through four samples of g (step D) */
static double interval(const double* g, int n, int k, double D)
{
    if (k == 0) return D / 24.0 * (9.0 * g[0] + 19.0 * g[1] - 5.0 * g[2] + g[3]);
    if (k == n - 2) return D / 24.0 * (g[n - 4] - 5.0 * g[n - 3] + 19.0 * g[n - 2] + 9.0 * g[n - 1]);
    return D / 24.0 * (-g[k - 1] + 13.0 * g[k] + 13.0 * g[k + 1] - g[k + 2]);
}

/* Interior solution of eq. (3.4) in every sphere (formula in the header).
 *   radii, Z: [n_atoms]; vlm_R: [n_atoms][25] the Dirichlet data (eq. (3.6));
 *   rho_lm: [n_atoms][25][n_rad] the density's rho_LM(r_k) on atom a's mesh;
 *   vlm: [n_atoms][25][n_rad] out. n_rad >= 4. */
int oracle_sphere_radial(int n_atoms, const double* radii, const double* Z, int n_rad, double r_min,
                         const double* vlm_R, const double* rho_lm, double* vlm)
{
    if (n_rad < 4) return 1;
    int n = n_rad;
    double* r = malloc(sizeof(double) * n);
    double* g1 = malloc(sizeof(double) * n);
    double* g2 = malloc(sizeof(double) * n);
    for (int a = 0; a < n_atoms; ++a) {
        double R = radii[a];
        double D = log(R / r_min) / (n - 1);
        for (int k = 0; k < n; ++k) r[k] = oracle_radial_node(R, r_min, n, k);
        for (int lm = 0; lm < NLM; ++lm) {
            int L = lm_degree(lm);
            const double* rho = rho_lm + ((size_t)a * NLM + lm) * n;
            double* out = vlm + ((size_t)a * NLM + lm) * n;
            /* integrands in t: rho r^(L+2) dr = rho r^(L+3) dt, rho r^(1-L) dr = rho r^(2-L) dt */
            for (int k = 0; k < n; ++k) {
                g1[k] = rho[k] * pow(r[k], L + 3);
                g2[k] = rho[k] * pow(r[k], 2 - L);
            }
            double head = rho[0] * pow(r[0], L + 3) / (2 * L + 3);
            double PR = head;
            for (int j = 0; j < n - 1; ++j) PR += interval(g1, n, j, D);
            double c = 4.0 * PI / (2 * L + 1);
            for (int k = 0; k < n; ++k) {
                double P = head, Q = 0.0;
                for (int j = 0; j < k; ++j) P += interval(g1, n, j, D);
                for (int j = k; j < n - 1; ++j) Q += interval(g2, n, j, D);
                double v = vlm_R[NLM * a + lm] * pow(r[k] / R, L)
                         - c * (P / pow(r[k], L + 1) + pow(r[k], L) * Q - pow(r[k], L) * PR / pow(R, 2 * L + 1));
                if (L == 0) v += sqrt(4.0 * PI) * Z[a] * (1.0 / r[k] - 1.0 / R);
                out[k] = v;
            }
        }
    }
    free(r);
    free(g1);
    free(g2);
    return 0;
}

/* Sphere part of the energy integral: out[a] = sum_LM int_0^R_a V_LM rho_LM r^2 dr
 * on atom a's mesh (quadrature in the header). vlm, rho_lm: [n_atoms][25][n_rad]. */
int oracle_sphere_energy(int n_atoms, const double* radii, int n_rad, double r_min, const double* vlm,
                         const double* rho_lm, double* out)
{
    if (n_rad < 4) return 1;
    int n = n_rad;
    double* g = malloc(sizeof(double) * n);
    for (int a = 0; a < n_atoms; ++a) {
        double R = radii[a];
        double D = log(R / r_min) / (n - 1);
        double s = 0.0;
        for (int lm = 0; lm < NLM; ++lm) {
            const double* v = vlm + ((size_t)a * NLM + lm) * n;
            const double* rho = rho_lm + ((size_t)a * NLM + lm) * n;
            for (int k = 0; k < n; ++k) g[k] = v[k] * rho[k] * pow(oracle_radial_node(R, r_min, n, k), 3);
            double r0 = oracle_radial_node(R, r_min, n, 0);
            s += v[0] * rho[0] * r0 * r0 * r0 / 3.0;
            for (int j = 0; j < n - 1; ++j) s += interval(g, n, j, D);
        }
        out[a] = s;
    }
    free(g);
    return 0;
}

/* ------------------------------------------------------------ grid part */

/* Grid part of the energy integral: sum over nodes outside every sphere of
 * vol_n v_n rho_n, vol_n the product of the dual widths (half a spacing at
 * an end). v, rho: [nz][ny][nx]. */
double oracle_energy_grid(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                          const double* v, const double* rho, int n_atoms, const double* centers,
                          const double* radii)
{
    double s = 0.0;
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
                if (outside) {
                    size_t n = ((size_t)k * ny + j) * nx + i;
                    s += mx * my * mz * v[n] * rho[n];
                }
            }
        }
    }
    return s;
}

/* ------------------------------------------- tabulated density on the grid */

/* The paper puts the non-spherical part of the sphere density directly on
 * the grid. Here it is read from the radial tables: at each node inside
 * sphere a (|x - C|^2 < R^2),
 *   rho += sum_(LM, L >= lmin) rho_LM(r) y_LM(x - C),
 * with rho_LM(r) the cubic Lagrange interpolant in t = ln r through the four
 * mesh samples around t (window start clamp(floor((t - t_0)/D) - 1, 0, n - 4),
 * t_k = ln R + (k - (n-1)) D), and below r_0, rho_LM(r_0) (r / r_0)^L (the
 * r^L behaviour at the centre). y_LM(x - C) = S_LM(x - C) / r^L.
 * rho_lm [n_atoms][25][n_rad]; rho [nz][ny][nx] is added to. */
int oracle_sphere_density_terms(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                                int n_atoms, const double* centers, const double* radii, int n_rad, double r_min,
                                const double* rho_lm, int lmin, double* rho)
{
    if (n_rad < 4 || lmin < 0 || lmin > 4) return 1;
    int n = n_rad;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int a = 0; a < n_atoms; ++a) {
                    double dx = x[i] - centers[3 * a], dy = y[j] - centers[3 * a + 1], dz = z[k] - centers[3 * a + 2];
                    volatile double sx = dx * dx, sy = dy * dy, sz = dz * dz;   /* no contraction */
                    double R = radii[a];
                    if (!(sx + sy + sz < R * R)) continue;
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    double S[25];
                    oracle_solid_harmonics(dx, dy, dz, S);
                    double D = log(R / r_min) / (n - 1);
                    double r0 = oracle_radial_node(R, r_min, n, 0);
                    double add = 0.0;
                    for (int lm = lmin * lmin; lm < NLM; ++lm) {
                        int L = lm_degree(lm);
                        const double* tab = rho_lm + ((size_t)a * NLM + lm) * n;
                        double val;
                        if (r < r0) {
                            val = tab[0] * S[lm] / pow(r0, L);   /* rho(r_0) (r/r_0)^L y_LM, y_LM = S / r^L */
                        } else {
                            double t = log(r);
                            double t0 = log(R) - (n - 1) * D;
                            double u0 = (t - t0) / D;
                            int i0 = (int)floor(u0) - 1;
                            if (i0 < 0) i0 = 0;
                            if (i0 > n - 4) i0 = n - 4;
                            double u = u0 - i0;
                            double w[4] = {-(u - 1) * (u - 2) * (u - 3) / 6.0, u * (u - 2) * (u - 3) / 2.0,
                                           -u * (u - 1) * (u - 3) / 2.0, u * (u - 1) * (u - 2) / 6.0};
                            double f = w[0] * tab[i0] + w[1] * tab[i0 + 1] + w[2] * tab[i0 + 2] + w[3] * tab[i0 + 3];
                            val = f * S[lm] / pow(r, L);
                        }
                        add += val;
                    }
                    rho[((size_t)k * ny + j) * nx + i] += add;
                    break;   /* spheres do not overlap */
                }
    return 0;
}
