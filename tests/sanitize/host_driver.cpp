// Runs the library's host-side numerics (graded mesh, coarsening, dual
// widths, 1-D eigen-decompositions) on small inputs, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer. Exit status 0 when every
// result holds its defining property.
#include <cmath>
#include <cstdio>
#include <vector>

#include "host.h"

static int failures = 0;

static void check(bool ok, const char* what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

int main()
{
    using namespace lasto;
    const double planes[3] = {-2.0, 0.5, 3.0};
    for (int n : {3, 33, 64, 129}) {
        std::vector<double> x(n);
        double g = 0.0, hmin = 0.0;
        // three nodes: the uniform mesh (no planes); more: graded towards the planes
        const char* err = mesh_graded_1d(-10.0, 10.0, n, planes, n > 3 ? 3 : 0, 0.2, 1.0, 1.2, 0.05, x.data(), &g,
                                         &hmin);
        check(err == nullptr, "graded mesh");
        bool increasing = true;
        for (int i = 1; i < n; ++i) increasing = increasing && x[i] > x[i - 1];
        check(increasing && x[0] == -10.0 && x[n - 1] == 10.0, "graded mesh is increasing from lo to hi");

        std::vector<double> m;
        dual_widths(x, m);
        double total = 0.0;
        for (double w : m) total += w;
        check(std::fabs(total - 20.0) < 1e-12, "dual widths sum to the length");

        const std::vector<int> keep = coarsen_axis(x, 4.0 * 0.2);
        check(!keep.empty() && keep.front() == 0 && keep.back() == n - 1, "coarsening keeps both ends");

        if (n > 3) {
            const int k = n - 2;
            std::vector<double> lam(k), S((size_t)k * k), Si((size_t)k * k);
            check(axis_decomposition(x.data(), n, lam.data(), S.data(), Si.data()), "axis decomposition");
            double err_id = 0.0;
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) {
                    double s = 0.0;
                    for (int t = 0; t < k; ++t) s += S[(size_t)i * k + t] * Si[(size_t)t * k + j];
                    err_id = std::fmax(err_id, std::fabs(s - (i == j ? 1.0 : 0.0)));
                }
            check(err_id < 1e-10, "S Si = I");
        }
    }
    std::vector<double> x(5);
    check(mesh_graded_1d(1.0, -1.0, 5, planes, 3, 0.2, 1.0, 1.2, 0.0, x.data(), nullptr, nullptr) != nullptr,
          "mesh rejects hi < lo");
    check(mesh_graded_1d(-1.0, 1.0, 5, nullptr, 2, 0.2, 1.0, 1.2, 0.0, x.data(), nullptr, nullptr) != nullptr,
          "mesh rejects missing planes");
    if (failures) return 1;
    std::printf("host driver: every routine ran clean\n");
    return 0;
}
