// Host-side numerics shared by the entry points (no HIP types), built into
// the library and, on their own, by the host compiler for sanitizer runs.
#pragma once

#include <vector>

namespace lasto {

// Graded 1-D mesh of n nodes on [lo, hi] refined towards the given planes
// (spacing min(hmax, hmin + (g - 1) d), d the distance to the nearest plane,
// g <= gmax chosen so that n nodes fit; hmin raised by hmin_step when no g
// fits). Null on success, else a message naming the bad argument.
const char* mesh_graded_1d(double lo, double hi, int n, const double* planes, int n_planes, double hmin, double hmax,
                           double gmax, double hmin_step, double* x_out, double* g_out, double* hmin_used);

// Indices of the nodes of x kept by one pair-merging coarsening with width tau.
std::vector<int> coarsen_axis(const std::vector<double>& x, double tau);

// Dual (control-volume) widths of the nodes of x, half cells at the ends.
void dual_widths(const std::vector<double>& x, std::vector<double>& m);

// Eigen-decomposition of a symmetric tridiagonal matrix: a (diagonal, n)
// and b (off-diagonal, n - 1) in, eigenvalues in a and eigenvectors in the
// columns of q (q[i * n + k]) out. False if the iteration does not converge.
bool tridiagonal_eigen(int n, std::vector<double>& a, std::vector<double>& b, std::vector<double>& q);

// Eigenvalues lam[n - 2] and the transforms S, Si ([n - 2][n - 2] row-major)
// of the 1-D interior operator on the nodes x[0 .. n - 1]. False if the
// eigen-decomposition does not converge.
bool axis_decomposition(const double* x, int n, double* lam, double* S, double* Si);

}  // namespace lasto
