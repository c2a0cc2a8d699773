// The output density in the interstitial region (host side of the C ABI;
// the kernel lives in src_kernels.hip).
#include <cmath>
#include <vector>

#include "internal.h"

using namespace lasto;

extern "C" lasto_status lasto_interstitial_density(lasto_grid g, int n_atoms, const double* centers,
                                                   const double* radii, int n_shells, const lasto_shell* shells,
                                                   int n_occ, const double* coef, const double* occ, double* rho_out)
{
    if (!g || !centers || !shells || !coef || !occ || !rho_out || n_atoms < 1 || n_shells < 1 || n_occ < 1)
        return fail(LASTO_ERR_ARG, "lasto_interstitial_density: NULL argument or empty basis");
    if (n_shells > 64) return fail(LASTO_ERR_ARG, "lasto_interstitial_density: at most 64 shells");
    std::vector<double4> sh(n_shells);
    int nbpa = 0;
    for (int s = 0; s < n_shells; ++s) {
        const lasto_shell& S = shells[s];
        if (S.l < 0 || S.l > 4 || S.n < S.l + 1 || S.n > 16 || !(S.zeta > 0.0) || !std::isfinite(S.zeta))
            return fail(LASTO_ERR_ARG, "lasto_interstitial_density: shells need 0 <= l <= 4, l + 1 <= n <= 16, "
                                       "zeta > 0");
        sh[s] = double4{(double)S.n, (double)S.l, (double)nbpa, S.zeta};
        nbpa += 2 * S.l + 1;
    }
    if (nbpa > 64) return fail(LASTO_ERR_ARG, "lasto_interstitial_density: at most 64 basis functions per atom");
    const LevelView& V = g->cview;
    if ((double)V.nx * V.ny * V.nz >= 2147483647.0)
        return fail(LASTO_ERR_ARG, "lasto_interstitial_density: a copy of the grid must hold fewer than 2^31 nodes");
    std::vector<double4> at(n_atoms);
    for (int a = 0; a < n_atoms; ++a) {
        const double R = radii ? radii[a] : 0.0;
        at[a] = double4{centers[3 * a], centers[3 * a + 1], centers[3 * a + 2], R};
        if (!std::isfinite(at[a].x) || !std::isfinite(at[a].y) || !std::isfinite(at[a].z) || !std::isfinite(R) ||
            R < 0.0)
            return fail(LASTO_ERR_ARG, "lasto_interstitial_density: centres finite, radii >= 0");
    }
    for (int k = 0; k < n_occ; ++k)
        if (!std::isfinite(occ[k])) return fail(LASTO_ERR_ARG, "lasto_interstitial_density: occupations finite");
    // device tables: atoms, shells, occupations (one staged block)
    const size_t bytes = sizeof(double4) * (n_atoms + n_shells) + sizeof(double) * n_occ;
    if (bytes > g->stage_bytes) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipFree(g->stage);
        g->stage = nullptr;
        LASTO_HIP(hipMalloc(&g->stage, bytes));
        g->stage_bytes = bytes;
    }
    double4* d_at = (double4*)g->stage;
    double4* d_sh = d_at + n_atoms;
    double* d_occ = (double*)(d_sh + n_shells);
    LASTO_HIP(hipMemcpyAsync(d_at, at.data(), sizeof(double4) * n_atoms, hipMemcpyHostToDevice, g->stream));
    LASTO_HIP(hipMemcpyAsync(d_sh, sh.data(), sizeof(double4) * n_shells, hipMemcpyHostToDevice, g->stream));
    LASTO_HIP(hipMemcpyAsync(d_occ, occ, sizeof(double) * n_occ, hipMemcpyHostToDevice, g->stream));
    LASTO_HIP(hipStreamSynchronize(g->stream));   // the host tables may go once copied
    LASTO_HIP(launch_interstitial(g, d_at, n_atoms, d_sh, n_shells, nbpa, coef, n_occ, d_occ, rho_out));
    return LASTO_OK;
}
