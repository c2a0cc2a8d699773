// Host-side numerics of the library: the graded mesh, the coarsening of the
// hierarchy, the dual widths and the 1-D eigen-decompositions of the direct
// solve. Plain C++ with no HIP header, so that it also builds with the host
// compiler alone (the sanitizer build of the tests).
#include "host.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

namespace lasto {

// ---------------------------------------------------------------- mesh
// Spacing rule h(d) = min(hmax, hmin + (g-1) d), d = distance to the nearest
// plane. Phi(d) = int_0^d dt/h(t) in closed form and its inverse.
struct Spacing {
    double g, hmin, hmax;
    double dsat() const { return (hmax - hmin) / (g - 1.0); }
    double phi(double d) const
    {
        if (g <= 1.0) return d / hmin;
        const double ds = dsat();
        if (d <= ds) return std::log1p((g - 1.0) * d / hmin) / (g - 1.0);
        return std::log1p((g - 1.0) * ds / hmin) / (g - 1.0) + (d - ds) / hmax;
    }
    double phi_inv(double v) const
    {
        if (g <= 1.0) return v * hmin;
        const double ds = dsat();
        const double vs = std::log1p((g - 1.0) * ds / hmin) / (g - 1.0);
        if (v <= vs) return hmin * std::expm1((g - 1.0) * v) / (g - 1.0);
        return ds + (v - vs) * hmax;
    }
};

// Pieces of [lo, hi] on which the distance to the nearest plane is linear:
// breaks at planes and at midpoints between neighbouring planes.
struct Piece {
    double a, b, plane;
};

static std::vector<Piece> mesh_pieces(double lo, double hi, std::vector<double> planes)
{
    std::sort(planes.begin(), planes.end());
    std::vector<double> br{lo};
    for (size_t j = 0; j < planes.size(); ++j) {
        if (j > 0) {
            const double mid = 0.5 * (planes[j - 1] + planes[j]);
            if (mid > br.back() && mid < hi) br.push_back(mid);
        }
        if (planes[j] > br.back() && planes[j] < hi) br.push_back(planes[j]);
    }
    br.push_back(hi);
    std::vector<Piece> out;
    for (size_t k = 0; k + 1 < br.size(); ++k) {
        const double mid = 0.5 * (br[k] + br[k + 1]);
        double best = planes[0];
        for (double p : planes)
            if (std::fabs(p - mid) < std::fabs(best - mid)) best = p;
        out.push_back({br[k], br[k + 1], best});
    }
    return out;
}

static double piece_length(const Piece& P, const Spacing& S)
{
    return std::fabs(S.phi(std::fabs(P.b - P.plane)) - S.phi(std::fabs(P.a - P.plane)));
}

static double total_length(const std::vector<Piece>& pcs, const Spacing& S)
{
    double t = 0.0;
    for (const Piece& P : pcs) t += piece_length(P, S);
    return t;
}

const char* mesh_graded_1d(double lo, double hi, int n, const double* planes, int n_planes, double hmin, double hmax,
                           double gmax, double hmin_step, double* x_out, double* g_out, double* hmin_used)
{
    if (!x_out || n < 3 || !(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi) || n_planes < 0 ||
        (n_planes > 0 && !planes))
        return "bad n, range or arrays";
    if (n_planes == 0) {
        for (int i = 0; i < n; ++i) x_out[i] = lo + (hi - lo) * (double)i / (double)(n - 1);
        x_out[0] = lo;
        x_out[n - 1] = hi;
        if (g_out) *g_out = 1.0;
        if (hmin_used) *hmin_used = (hi - lo) / (double)(n - 1);
        return nullptr;
    }
    if (!(hmin > 0.0) || hmax < hmin || !(gmax > 1.0))
        return "need hmin > 0, hmax >= hmin, gmax > 1";
    std::vector<double> pl(planes, planes + n_planes);
    for (double p : pl)
        if (!std::isfinite(p)) return "non-finite plane";
    const std::vector<Piece> pcs = mesh_pieces(lo, hi, pl);
    const double cells = (double)(n - 1);
    Spacing S{1.0, hmin, hmax};
    for (;;) {
        S.g = 1.0;
        if (total_length(pcs, S) <= cells) break;
        S.g = gmax;
        if (total_length(pcs, S) <= cells) {
            double a = 1.0, b = gmax;
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (a + b);
                if (m <= a || m >= b) break;
                S.g = m;
                if (total_length(pcs, S) > cells) a = m;
                else b = m;
            }
            S.g = b;
            break;
        }
        if (hmin_step <= 0.0 || S.hmin + hmin_step > hmax)
            return "no growth factor <= gmax fits n nodes";
        S.hmin += hmin_step;
    }
    const double T = total_length(pcs, S);
    std::vector<double> start(pcs.size() + 1, 0.0);
    for (size_t k = 0; k < pcs.size(); ++k) start[k + 1] = start[k] + piece_length(pcs[k], S);
    x_out[0] = lo;
    x_out[n - 1] = hi;
    size_t k = 0;
    for (int i = 1; i < n - 1; ++i) {
        const double t = T * (double)i / (double)(n - 1);
        while (k + 1 < pcs.size() && start[k + 1] < t) ++k;
        const Piece& P = pcs[k];
        const double pa = S.phi(std::fabs(P.a - P.plane));
        double x;
        if (P.plane <= P.a) x = P.plane + S.phi_inv(pa + (t - start[k]));
        else x = P.plane - S.phi_inv(pa - (t - start[k]));
        x_out[i] = std::min(std::max(x, P.a), P.b);
    }
    if (g_out) *g_out = S.g;
    if (hmin_used) *hmin_used = S.hmin;
    return nullptr;
}

// ---------------------------------------------------------------- hierarchy
// Pair-merging coarsening of one axis: walking up from node 0, the pair of
// cells [x_i, x_{i+2}] merges (node i+1 dropped) when x_{i+2} - x_i <= tau.
// An axis with at most 3 nodes is kept as it is.
std::vector<int> coarsen_axis(const std::vector<double>& x, double tau)
{
    const int n = (int)x.size();
    std::vector<int> keep;
    keep.push_back(0);
    if (n <= 3) {
        for (int t = 1; t < n; ++t) keep.push_back(t);
        return keep;
    }
    int i = 0;
    while (i < n - 1) {
        if (i + 2 <= n - 1 && x[i + 2] - x[i] <= tau) {
            keep.push_back(i + 2);
            i += 2;
        } else {
            keep.push_back(i + 1);
            i += 1;
        }
    }
    return keep;
}

void dual_widths(const std::vector<double>& x, std::vector<double>& m)
{
    const int n = (int)x.size();
    m.assign(n, 0.0);
    m[0] = 0.5 * (x[1] - x[0]);
    m[n - 1] = 0.5 * (x[n - 1] - x[n - 2]);
    for (int i = 1; i < n - 1; ++i) m[i] = 0.5 * (x[i + 1] - x[i - 1]);
}

// ---------------------------------------------------------------- direct solve
// Eigen-decomposition T = Q diag(a) Q^T of a symmetric tridiagonal matrix
// (diagonal a[0..n-1], off-diagonal b[k] between k and k+1) by implicit
// symmetric QR steps with the Wilkinson shift, as the bulge-chasing sweep of
// Golub and Van Loan (Matrix Computations, Section 8.3): on the unreduced
// block [lo, hi] ending at the bottom, a plane rotation on (lo, lo+1) set by
// the first column of T - mu I starts a bulge, and rotations on (k, k+1) for
// k = lo+1 .. hi-1 chase it down and out; the rotations are accumulated into
// Q. An off-diagonal below eps (|a_k| + |a_k+1|) is set to zero, which splits
// the matrix. On return a holds the eigenvalues and column k of Q
// (q[i * n + k]) the eigenvector of a[k]. False if the iteration has not
// converged after 40 n steps.
bool tridiagonal_eigen(int n, std::vector<double>& a, std::vector<double>& b, std::vector<double>& q)
{
    q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
    b.resize(std::max(n - 1, 0));
    auto negligible = [&](int k) { return std::fabs(b[k]) <= DBL_EPSILON * (std::fabs(a[k]) + std::fabs(a[k + 1])); };
    // plane rotation of columns k, k+1 of Q (Q <- Q R, R^T = [[c, s], [-s, c]])
    auto rotate_q = [&](int k, double c, double s) {
        for (int i = 0; i < n; ++i) {
            double* row = &q[(size_t)i * n];
            const double u = row[k], w = row[k + 1];
            row[k] = c * u + s * w;
            row[k + 1] = -s * u + c * w;
        }
    };
    long steps = 0;
    int hi = n - 1;
    while (hi > 0) {
        if (negligible(hi - 1)) {
            b[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(lo - 1)) --lo;
        if (++steps > 40L * n) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer a[hi]
        const double dl = 0.5 * (a[hi - 1] - a[hi]);
        const double bb = b[hi - 1];
        const double mu = a[hi] - bb * bb / (dl + std::copysign(std::hypot(dl, bb), dl));
        double x = a[lo] - mu, y = b[lo], bulge = 0.0;
        for (int k = lo; k < hi; ++k) {
            // rotation (c, s) with -s x + c y = 0: it zeroes the bulge (or, at
            // k = lo, the second entry of the shifted first column)
            const double r = std::hypot(x, y);
            const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? y / r : 0.0;
            if (k > lo) b[k - 1] = r;
            // the 2 x 2 block on (k, k+1) under R^T . R
            const double ak = a[k], ak1 = a[k + 1], bk = b[k];
            a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
            a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
            b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
            // the entry below the block becomes the new bulge
            if (k + 1 < hi) {
                bulge = s * b[k + 1];
                b[k + 1] = c * b[k + 1];
            }
            rotate_q(k, c, s);
            x = b[k];
            y = bulge;
        }
    }
    return true;
}

// 1-D operator of the interior nodes of coordinates x[0..n-1]:
// (A u)_i = am_i (u_i-1 - u_i) + ap_i (u_i+1 - u_i), am = 1/(h_i-1 m_i),
// ap = 1/(h_i m_i). Fills lam[n-2], S and Si [n-2][n-2] row-major.
bool axis_decomposition(const double* x, int n, double* lam, double* S, double* Si)
{
    const int m = n - 2;
    std::vector<double> w(m), d(m), e(m), z;
    for (int t = 0; t < m; ++t) {
        const int i = t + 1;
        const double hm = x[i] - x[i - 1], hp = x[i + 1] - x[i];
        w[t] = 0.5 * (hm + hp);
        d[t] = -(1.0 / (hm * w[t]) + 1.0 / (hp * w[t]));
    }
    for (int t = 0; t + 1 < m; ++t) e[t] = 1.0 / ((x[t + 2] - x[t + 1]) * std::sqrt(w[t] * w[t + 1]));
    if (!tridiagonal_eigen(m, d, e, z)) return false;
    for (int t = 0; t < m; ++t) lam[t] = d[t];
    for (int i = 0; i < m; ++i) {
        const double sq = std::sqrt(w[i]);
        for (int k = 0; k < m; ++k) {
            S[(size_t)i * m + k] = z[(size_t)i * m + k] / sq;    // M^-1/2 Q
            Si[(size_t)k * m + i] = z[(size_t)i * m + k] * sq;   // Q^T M^1/2
        }
    }
    return true;
}

}  // namespace lasto
