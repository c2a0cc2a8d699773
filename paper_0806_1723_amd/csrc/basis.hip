// The output density and the matrix elements in the interstitial region
// (host side of the C ABI; the kernels live in src_kernels.hip).
#include <algorithm>
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
    int nbpa = 0, lmax = 0;
    for (int s = 0; s < n_shells; ++s) {
        const lasto_shell& S = shells[s];
        lmax = std::max(lmax, S.l);
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
    LASTO_HIP(launch_interstitial(g, d_at, n_atoms, d_sh, n_shells, lmax, nbpa, coef, n_occ, d_occ, rho_out));
    return LASTO_OK;
}

extern "C" lasto_status lasto_matrix_elements(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                              const double* radii, int n_shells, const lasto_shell* shells, double* S,
                                              double* H)
{
    if (!g || !v || !centers || !radii || !shells || !S || !H || n_atoms < 1 || n_shells < 1)
        return fail(LASTO_ERR_ARG, "lasto_matrix_elements: NULL argument or empty basis");
    if (n_shells > 64) return fail(LASTO_ERR_ARG, "lasto_matrix_elements: at most 64 shells");
    std::vector<double4> sh(n_shells);
    int nbpa = 0, lmax = 0;
    for (int s = 0; s < n_shells; ++s) {
        const lasto_shell& Q = shells[s];
        lmax = std::max(lmax, Q.l);
        if (Q.l < 0 || Q.l > 4 || Q.n < Q.l + 1 || Q.n > 16 || !(Q.zeta > 0.0) || !std::isfinite(Q.zeta))
            return fail(LASTO_ERR_ARG, "lasto_matrix_elements: shells need 0 <= l <= 4, l + 1 <= n <= 16, zeta > 0");
        sh[s] = double4{(double)Q.n, (double)Q.l, (double)nbpa, Q.zeta};
        nbpa += 2 * Q.l + 1;
    }
    const long long nbl = (long long)nbpa * n_atoms;
    if (nbl > 32768) return fail(LASTO_ERR_ARG, "lasto_matrix_elements: at most 32768 basis functions");
    const int n_basis = (int)nbl;
    const LevelView& V = g->cview;
    const size_t N = (size_t)V.nx * V.ny * V.nz;
    if ((double)N >= 2147483647.0)
        return fail(LASTO_ERR_ARG, "lasto_matrix_elements: a copy of the grid must hold fewer than 2^31 nodes");
    std::vector<double4> at(n_atoms);
    for (int a = 0; a < n_atoms; ++a) {
        at[a] = double4{centers[3 * a], centers[3 * a + 1], centers[3 * a + 2], radii[a]};
        if (!std::isfinite(at[a].x) || !std::isfinite(at[a].y) || !std::isfinite(at[a].z) || !(radii[a] > 0.0) ||
            !std::isfinite(radii[a]))
            return fail(LASTO_ERR_ARG, "lasto_matrix_elements: centres finite, every radius > 0 (the kinetic term "
                                       "is singular at a centre)");
    }
    // block pairs (r <= c) and node chunks: about 2048 workgroups, chunks of >= 4096 nodes
    const int nblk = (n_basis + 63) / 64;
    std::vector<int2> pr;
    for (int r = 0; r < nblk; ++r)
        for (int c = r; c < nblk; ++c) pr.push_back(int2{r, c});
    const int n_pairs = (int)pr.size();
    int n_chunks = std::max(1, (2048 + n_pairs - 1) / n_pairs);
    n_chunks = (int)std::max<size_t>(1, std::min<size_t>(n_chunks, (N + 4095) / 4096));
    double* w = nullptr;
    double* partials = nullptr;
    void* tab = nullptr;
    const size_t tab_bytes = sizeof(double4) * (n_atoms + n_shells) + sizeof(int2) * n_pairs;
    auto release = [&]() {
        (void)hipFree(w);
        (void)hipFree(partials);
        (void)hipFree(tab);
    };
    if (hipMalloc(&w, sizeof(double) * N) != hipSuccess ||
        hipMalloc(&partials, sizeof(double) * matrix_partial_doubles(n_pairs, n_chunks)) != hipSuccess ||
        hipMalloc(&tab, tab_bytes) != hipSuccess) {
        release();
        return fail(LASTO_ERR_ALLOC, "lasto_matrix_elements: device scratch");
    }
    double4* d_at = (double4*)tab;
    double4* d_sh = d_at + n_atoms;
    int2* d_pr = (int2*)(d_sh + n_shells);
    hipError_t e = hipMemcpyAsync(d_at, at.data(), sizeof(double4) * n_atoms, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_sh, sh.data(), sizeof(double4) * n_shells, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pr, pr.data(), sizeof(int2) * n_pairs, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = launch_node_weights(g, d_at, n_atoms, w);
    if (e == hipSuccess)
        e = launch_matrix_elements(g, w, v, d_at, n_atoms, d_sh, n_shells, lmax, nbpa, n_basis, d_pr, n_pairs,
                                   n_chunks, partials, S, H);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    release();
    if (e != hipSuccess) return fail(LASTO_ERR_HIP, std::string("lasto_matrix_elements: ") + hipGetErrorString(e));
    return LASTO_OK;
}
