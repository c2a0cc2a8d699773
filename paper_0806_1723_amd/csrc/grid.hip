// Grid creation: the multigrid hierarchy of the graded tensor-product mesh,
// its per-axis device tables, and the device work arrays.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"
#include "internal.h"

namespace lasto {

hipError_t init_harmonic_constants();
template <typename T>
hipError_t launch_fill_zero(T* a, size_t n, hipStream_t s);

// Per-axis tables of one copy: stencil coefficients, dual widths,
// coordinates, restriction (rf, rw) and prolongation (pc, pw from the finer
// level; level > 0 only).
struct AxisTables {
    std::vector<double> am, ap, m, x, rw, pw;
    std::vector<int> rf, pc;
};

static AxisTables axis_tables(lasto_grid g, int l, int d)
{
    const Level& L = g->lev[l];
    const int n = L.n[d];
    const std::vector<double>& x = L.hx[d];
    AxisTables t;
    dual_widths(x, t.m);
    t.x = x;
    t.am.assign(n, 0.0);
    t.ap.assign(n, 0.0);
    for (int i = 1; i < n - 1; ++i) {
        t.am[i] = 1.0 / ((x[i] - x[i - 1]) * t.m[i]);
        t.ap[i] = 1.0 / ((x[i + 1] - x[i]) * t.m[i]);
    }
    t.rf.assign(n, 0);
    t.rw.assign(3 * (size_t)n, 0.0);
    if (l == 0) {
        for (int I = 0; I < n; ++I) {
            t.rf[I] = I;
            t.rw[3 * I + 1] = 1.0;
        }
        return t;
    }
    const Level& F = g->lev[l - 1];
    const std::vector<double>& xf = F.hx[d];
    const int nf = F.n[d];
    std::vector<double> mf;
    dual_widths(xf, mf);
    const std::vector<int>& keep = L.keep[d];
    t.pc.assign(nf, 0);
    t.pw.assign(2 * (size_t)nf, 0.0);
    // interpolation: kept fine node -> weight 1 on its coarse node; a
    // dropped node between coarse c and c+1 -> linear weights in x
    int c = 0;
    for (int i = 0; i < nf; ++i) {
        while (c + 1 < n && keep[c + 1] <= i) ++c;
        t.pc[i] = c;
        if (keep[c] == i) {
            t.pw[2 * i] = 1.0;
        } else {
            const double xa = xf[keep[c]], xb = xf[keep[c + 1]];
            const double w = (xb - xf[i]) / (xb - xa);
            t.pw[2 * i] = w;
            t.pw[2 * i + 1] = 1.0 - w;
        }
    }
    // restriction: coarse node I gathers fine nodes keep[I]-1..keep[I]+1
    // with the transposed interpolation weight times m_fine/m_coarse
    for (int I = 0; I < n; ++I) {
        t.rf[I] = keep[I];
        for (int s2 = 0; s2 < 3; ++s2) {
            const int fi = keep[I] - 1 + s2;
            double w = 0.0;
            if (fi >= 0 && fi < nf) {
                if (t.pc[fi] == I) w = t.pw[2 * fi];
                else if (t.pc[fi] + 1 == I) w = t.pw[2 * fi + 1];
                w *= mf[fi] / t.m[I];
            }
            t.rw[3 * I + s2] = w;
        }
    }
    return t;
}

// The z tables of a batch: the copy's tables repeated, with the restriction
// and prolongation indices shifted to each copy's planes.
static AxisTables stack_copies(const AxisTables& t, int nb, int n, int nf)
{
    if (nb == 1) return t;
    AxisTables s;
    for (int b = 0; b < nb; ++b) {
        s.am.insert(s.am.end(), t.am.begin(), t.am.end());
        s.ap.insert(s.ap.end(), t.ap.begin(), t.ap.end());
        s.m.insert(s.m.end(), t.m.begin(), t.m.end());
        s.x.insert(s.x.end(), t.x.begin(), t.x.end());
        s.rw.insert(s.rw.end(), t.rw.begin(), t.rw.end());
        s.pw.insert(s.pw.end(), t.pw.begin(), t.pw.end());
        for (int v : t.rf) s.rf.push_back(v + b * nf);
        for (int v : t.pc) s.pc.push_back(v + b * n);
    }
    return s;
}

// Device table layout of level l (doubles): per axis d, am[n] ap[n] m[n] x[n]
// rw[3n]; then, for l > 0, per axis pw[2 nf] (nf = the finer level's length).
// Ints: per axis rf[n]; then, for l > 0, per axis pc[nf]. For z, n and nf
// count all copies of a batch.
lasto_status build_level_tables(lasto_grid g, int l)
{
    Level& L = g->lev[l];
    const int nb = g->n_batch;
    AxisTables T[3];
    int nst[3], nfst[3];
    for (int d = 0; d < 3; ++d) {
        const int copies = d == 2 ? nb : 1;
        const int nf = l > 0 ? g->lev[l - 1].n[d] : 0;
        T[d] = stack_copies(axis_tables(g, l, d), copies, L.n[d], nf);
        nst[d] = copies * L.n[d];
        nfst[d] = copies * nf;
    }
    size_t od_own[3], oi_own[3], od_fine[3], oi_fine[3];
    size_t nd = 0, ni = 0;
    for (int d = 0; d < 3; ++d) {
        od_own[d] = nd;
        oi_own[d] = ni;
        nd += 7 * (size_t)nst[d];
        ni += (size_t)nst[d];
    }
    for (int d = 0; d < 3; ++d) {
        od_fine[d] = nd;
        oi_fine[d] = ni;
        nd += 2 * (size_t)nfst[d];
        ni += (size_t)nfst[d];
    }
    std::vector<double> hd(nd, 0.0);
    std::vector<int> hi(ni, 0);
    LASTO_HIP(hipMalloc(&L.dtab, sizeof(double) * nd));
    LASTO_HIP(hipMalloc(&L.dtabi, sizeof(int) * ni));
    for (int d = 0; d < 3; ++d) {
        const int n = nst[d];
        const size_t o = od_own[d];
        std::copy(T[d].am.begin(), T[d].am.end(), hd.begin() + o);
        std::copy(T[d].ap.begin(), T[d].ap.end(), hd.begin() + o + n);
        std::copy(T[d].m.begin(), T[d].m.end(), hd.begin() + o + 2 * n);
        std::copy(T[d].x.begin(), T[d].x.end(), hd.begin() + o + 3 * n);
        std::copy(T[d].rw.begin(), T[d].rw.end(), hd.begin() + o + 4 * n);
        std::copy(T[d].rf.begin(), T[d].rf.end(), hi.begin() + oi_own[d]);
        Axis& A = L.view.ax[d];
        A.n = n;
        A.am = L.dtab + o;
        A.ap = L.dtab + o + n;
        A.m = L.dtab + o + 2 * n;
        A.x = L.dtab + o + 3 * n;
        A.rw = L.dtab + o + 4 * n;
        A.rf = L.dtabi + oi_own[d];
        A.pc = nullptr;
        A.pw = nullptr;
        if (l > 0) {
            std::copy(T[d].pw.begin(), T[d].pw.end(), hd.begin() + od_fine[d]);
            std::copy(T[d].pc.begin(), T[d].pc.end(), hi.begin() + oi_fine[d]);
            A.pc = L.dtabi + oi_fine[d];
            A.pw = L.dtab + od_fine[d];
        }
    }
    LASTO_HIP(hipMemcpy(L.dtab, hd.data(), sizeof(double) * nd, hipMemcpyHostToDevice));
    LASTO_HIP(hipMemcpy(L.dtabi, hi.data(), sizeof(int) * ni, hipMemcpyHostToDevice));
    L.view.nx = L.n[0];
    L.view.ny = L.n[1];
    L.view.nz = nst[2];
    L.view.nzc = L.n[2];
    // split-layout row: entries 0..nx/2 of one colour plus two spare entries
    // (a half-sweep pair at the row's end reads one past it), padded to 16
    // (128 B in FP64)
    L.view.W = ((L.n[0] / 2 + 3) + 15) / 16 * 16;
    L.view.cs = (size_t)L.view.nz * L.n[1] * L.view.W;
    L.nsplit = 2 * L.view.cs;
    // the Krylov kernels address split entries with 32-bit indices
    if (L.nsplit >= ((size_t)1 << 32))
        return fail(LASTO_ERR_ARG, "lasto_grid_create: a split array of 2^32 or more entries is not supported");
    // planes interior to their copy
    std::vector<unsigned char> zi(nst[2], 0);
    for (int k = 0; k < nst[2]; ++k) {
        const int kk = k % L.n[2];
        zi[k] = (kk >= 1 && kk <= L.n[2] - 2) ? 1 : 0;
    }
    LASTO_HIP(hipMalloc(&L.dzint, zi.size()));
    LASTO_HIP(hipMemcpy(L.dzint, zi.data(), zi.size(), hipMemcpyHostToDevice));
    L.view.zint = L.dzint;

    // x coefficients by parity ([p][q][m], node i = p + 2m; zero off the
    // interior) in FP64 and FP32, and FP32 copies of every axis' am/ap
    const int W = L.view.W, nx = L.n[0];
    std::vector<double> xp(6 * (size_t)W, 0.0);
    for (int p = 0; p < 2; ++p)
        for (int m = 0; m < W; ++m) {
            const int i = p + 2 * m;
            if (i < 1 || i > nx - 2) continue;
            xp[(p * 3 + 0) * (size_t)W + m] = hd[od_own[0] + i];
            xp[(p * 3 + 1) * (size_t)W + m] = hd[od_own[0] + nx + i];
            xp[(p * 3 + 2) * (size_t)W + m] = hd[od_own[0] + 2 * nx + i];
        }
    size_t nfl = 6 * (size_t)W;
    for (int d = 0; d < 3; ++d) nfl += 2 * (size_t)nst[d];
    std::vector<float> hf(nfl, 0.0f);
    for (size_t t = 0; t < 6 * (size_t)W; ++t) hf[t] = (float)xp[t];
    size_t of = 6 * (size_t)W;
    size_t ofs[3];
    for (int d = 0; d < 3; ++d) {
        ofs[d] = of;
        for (int i = 0; i < nst[d]; ++i) {
            hf[of + i] = (float)hd[od_own[d] + i];
            hf[of + nst[d] + i] = (float)hd[od_own[d] + nst[d] + i];
        }
        of += 2 * (size_t)nst[d];
    }
    LASTO_HIP(hipMalloc(&L.dxpar, sizeof(double) * xp.size()));
    LASTO_HIP(hipMalloc(&L.dtabf, sizeof(float) * hf.size()));
    LASTO_HIP(hipMemcpy(L.dxpar, xp.data(), sizeof(double) * xp.size(), hipMemcpyHostToDevice));
    LASTO_HIP(hipMemcpy(L.dtabf, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice));
    L.view.xpar = L.dxpar;
    L.view.xparf = L.dtabf;
    for (int d = 0; d < 3; ++d) {
        L.view.ax[d].amf = L.dtabf + ofs[d];
        L.view.ax[d].apf = L.dtabf + ofs[d] + nst[d];
    }
    return LASTO_OK;
}

static lasto_status alloc_zero(lasto_grid g, void** p, size_t bytes)
{
    LASTO_HIP(hipMalloc(p, bytes));
    LASTO_HIP(launch_fill_zero<unsigned char>((unsigned char*)*p, bytes, g->stream));
    return LASTO_OK;
}

static void free_grid(lasto_grid g)
{
    for (auto& e : g->vgraphs)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    g->vgraphs.clear();
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
    free_fdm(g);
    free_coarse_fdm(g);
    free_coarse_gemm(g);
    for (int l = 0; l < g->nlev; ++l) {
        Level& L = g->lev[l];
        (void)hipFree(L.dtab);
        (void)hipFree(L.dtabi);
        (void)hipFree(L.dxpar);
        (void)hipFree(L.dzint);
        (void)hipFree(L.dtabf);
        (void)hipFree(L.u64);
        (void)hipFree(L.u32);
        (void)hipFree(L.f64);
        (void)hipFree(L.r64);
        (void)hipFree(L.f32);
        (void)hipFree(L.r32);
    }
    (void)hipFree(g->r);
    (void)hipFree(g->p[0]);
    (void)hipFree(g->p[1]);
    (void)hipFree(g->q);
    (void)hipFree(g->z);
    (void)hipFree(g->x);
    (void)hipFree(g->r32);
    (void)hipFree(g->p32[0]);
    (void)hipFree(g->p32[1]);
    (void)hipFree(g->q32);
    (void)hipFree(g->e32);
    (void)hipFree(g->z32);
    (void)hipFree(g->partials);
    (void)hipFree(g->scalars);
    (void)hipFree(g->moments);
    (void)hipFree(g->stage);
    (void)hipFree(g->tail_dev);
    (void)hipFree(g->lds_tabs);
    (void)hipFree(g->lds_plan_dev);
    for (double*& a : g->lscr) {
        (void)hipFree(a);
        a = nullptr;
    }
    if (g->h_scalars) (void)hipHostFree(g->h_scalars);
    if (g->stage_host) (void)hipHostFree(g->stage_host);
    g->stage_host = nullptr;
    for (hipEvent_t e : g->prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->ph_ev)
        if (e) (void)hipEventDestroy(e);
    for (void* p : g->lg_alloc) (void)hipFree(p);
    g->lg_alloc.clear();
    g->prof_ev.clear();
}

}  // namespace lasto

using namespace lasto;

// FP32 LDS tail: from the first level whose corrections, right-hand sides
// and tables, with those of every coarser level, fit in one workgroup's LDS
// (keeping 8 KB spare), and only where it takes over at least the levels of
// the global-memory tail (a later start would run those by separate
// launches). Builds the plan and the device table run it copies in.
static lasto_status build_lds_tail(lasto_grid g)
{
    g->tail32_top = -1;
    const int lim = tail_lds_limit() - 8192;
    if (lim <= 0) return LASTO_OK;
    auto dims_of = [&](int l, int d) { return d == 2 ? g->lev[l].view.nz : g->lev[l].n[d]; };
    auto tab_of = [&](int l, bool coarse) {
        const int f = coarse ? l - 1 : l;
        return (size_t)lds_tab_size(dims_of(l, 0), dims_of(l, 1), dims_of(l, 2), dims_of(f, 0), dims_of(f, 1),
                                    dims_of(f, 2), coarse);
    };
    for (int t = g->nlev - 1; t >= 0 && g->nlev - t <= kLdsMaxLevels; --t) {
        size_t need = 0;
        for (int l = t; l < g->nlev; ++l) need += 2 * g->lev[l].nsplit + tab_of(l, l > t);
        if (need * sizeof(float) > (size_t)lim) break;
        g->tail32_top = t;
    }
    if (g->tail32_top > g->tail_top) g->tail32_top = -1;
    if (g->tail32_top < 0) return LASTO_OK;
    const int top = g->tail32_top;
    LdsPlan& P = g->lds_plan;
    P = LdsPlan{};
    P.nl = g->nlev - top;
    int o = 0;
    for (int q = 0; q < P.nl; ++q) {
        const LevelView& V = g->lev[top + q].view;
        P.dims[q][0] = V.nx;
        P.dims[q][1] = V.ny;
        P.dims[q][2] = V.nz;
        P.dims[q][3] = V.W;
        P.dims[q][4] = (int)V.cs;
        P.off[q][0] = o;
        P.off[q][1] = o + (int)(2 * V.cs);
        o += (int)(4 * V.cs);
    }
    P.tab0 = o;
    std::vector<float> tab;
    for (int q = 0; q < P.nl; ++q) {
        const int l = top + q;
        const LevelView& V = g->lev[l].view;
        P.off[q][2] = o + (int)tab.size();
        const size_t base = tab.size();
        tab.resize(base + tab_of(l, q > 0), 0.0f);
        const int n[3] = {V.nx, V.ny, V.nz};
        const int fn[3] = {q > 0 ? dims_of(l - 1, 0) : 0, q > 0 ? dims_of(l - 1, 1) : 0, q > 0 ? dims_of(l - 1, 2) : 0};
        float* b0 = tab.data() + base;
        LdsTab t = lds_tab(b0, n[0], n[1], n[2], fn[0], fn[1], fn[2], q > 0);
        auto w = [&](const float* at) { return const_cast<float*>(at); };
        float* am[3] = {w(t.cxm), w(t.cym), w(t.czm)};
        float* ap[3] = {w(t.cxp), w(t.cyp), w(t.czp)};
        float* rf[3] = {w(t.rfx), w(t.rfy), w(t.rfz)};
        float* rw[3] = {w(t.rwx), w(t.rwy), w(t.rwz)};
        float* pc[3] = {w(t.pcx), w(t.pcy), w(t.pcz)};
        float* pw[3] = {w(t.pwx), w(t.pwy), w(t.pwz)};
        for (int d = 0; d < 3; ++d) {
            LASTO_HIP(hipMemcpy(am[d], V.ax[d].amf, sizeof(float) * n[d], hipMemcpyDeviceToHost));
            LASTO_HIP(hipMemcpy(ap[d], V.ax[d].apf, sizeof(float) * n[d], hipMemcpyDeviceToHost));
            if (q == 0) continue;
            std::vector<int> vi(std::max(n[d], fn[d]));
            std::vector<double> vd(3 * (size_t)std::max(n[d], fn[d]));
            LASTO_HIP(hipMemcpy(vi.data(), V.ax[d].rf, sizeof(int) * n[d], hipMemcpyDeviceToHost));
            LASTO_HIP(hipMemcpy(vd.data(), V.ax[d].rw, sizeof(double) * 3 * n[d], hipMemcpyDeviceToHost));
            for (int e = 0; e < n[d]; ++e) rf[d][e] = (float)vi[e];
            for (int e = 0; e < 3 * n[d]; ++e) rw[d][e] = (float)vd[e];
            LASTO_HIP(hipMemcpy(vi.data(), V.ax[d].pc, sizeof(int) * fn[d], hipMemcpyDeviceToHost));
            LASTO_HIP(hipMemcpy(vd.data(), V.ax[d].pw, sizeof(double) * 2 * fn[d], hipMemcpyDeviceToHost));
            for (int e = 0; e < fn[d]; ++e) pc[d][e] = (float)vi[e];
            for (int e = 0; e < 2 * fn[d]; ++e) pw[d][e] = (float)vd[e];
        }
        std::vector<unsigned char> zi(n[2]);
        LASTO_HIP(hipMemcpy(zi.data(), V.zint, n[2], hipMemcpyDeviceToHost));
        for (int k = 0; k < n[2]; ++k) w(t.zin)[k] = zi[k] ? 1.0f : 0.0f;
    }
    P.ntab = (int)tab.size();
    P.total = o + P.ntab;
    LASTO_HIP(hipMalloc((void**)&g->lds_tabs, sizeof(float) * tab.size()));
    LASTO_HIP(hipMemcpy(g->lds_tabs, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice));
    LASTO_HIP(hipMalloc((void**)&g->lds_plan_dev, sizeof(LdsPlan)));
    LASTO_HIP(hipMemcpy(g->lds_plan_dev, &P, sizeof(LdsPlan), hipMemcpyHostToDevice));
    return LASTO_OK;
}

extern "C" lasto_status lasto_grid_create(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                                          int n_batch, void* hip_stream, lasto_grid* out)
{
    if (!out) return fail(LASTO_ERR_ARG, "lasto_grid_create: out is NULL");
    *out = nullptr;
    if (!x || !y || !z) return fail(LASTO_ERR_ARG, "lasto_grid_create: NULL coordinates");
    const double* xs[3] = {x, y, z};
    const int ns[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d) {
        if (ns[d] < 4) return fail(LASTO_ERR_ARG, "lasto_grid_create: every axis needs at least 4 nodes");
        if (ns[d] > (1 << 16)) return fail(LASTO_ERR_ARG, "lasto_grid_create: axis too long");
        for (int i = 0; i < ns[d]; ++i)
            if (!std::isfinite(xs[d][i])) return fail(LASTO_ERR_ARG, "lasto_grid_create: non-finite coordinate");
        for (int i = 0; i + 1 < ns[d]; ++i)
            if (!(xs[d][i + 1] > xs[d][i])) return fail(LASTO_ERR_ARG, "lasto_grid_create: coordinates must increase");
    }
    if (n_batch < 1 || n_batch > kMaxBatch) return fail(LASTO_ERR_ARG, "lasto_grid_create: n_batch must be 1..16");
    if (hipError_t e = init_harmonic_constants(); e != hipSuccess)
        return fail(LASTO_ERR_HIP, std::string("harmonic constants: ") + hipGetErrorString(e));

    lasto_grid g = new (std::nothrow) lasto_grid_s();
    if (!g) return fail(LASTO_ERR_ALLOC, "lasto_grid_create: host allocation");
    g->stream = (hipStream_t)hip_stream;
    g->n_batch = n_batch;
    (void)hipGetDevice(&g->device);
    for (int d = 0; d < 3; ++d) g->box_center[d] = 0.5 * (xs[d][0] + xs[d][ns[d] - 1]);

    // hierarchy
    Level& L0 = g->lev[0];
    for (int d = 0; d < 3; ++d) {
        L0.n[d] = ns[d];
        L0.hx[d].assign(xs[d], xs[d] + ns[d]);
    }
    g->nlev = 1;
    for (;;) {
        Level& F = g->lev[g->nlev - 1];
        if (F.n[0] <= kCoarseMax && F.n[1] <= kCoarseMax && F.n[2] <= kCoarseMax) break;
        if (g->nlev == kMaxLevels) break;
        double hmin = 1e300, hmax = 0.0;
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i + 1 < F.n[d]; ++i) {
                const double h = F.hx[d][i + 1] - F.hx[d][i];
                hmin = std::min(hmin, h);
                hmax = std::max(hmax, h);
            }
        std::vector<int> kp[3];
        bool changed = false;
        for (int d = 0; d < 3; ++d) {
            kp[d] = coarsen_axis(F.hx[d], kCoarsenTheta * hmin * (1.0 + 1e-12));
            if ((int)kp[d].size() < F.n[d]) changed = true;
        }
        if (!changed)
            for (int d = 0; d < 3; ++d) kp[d] = coarsen_axis(F.hx[d], 2.0 * hmax * (1.0 + 1e-12));
        Level& C = g->lev[g->nlev];
        for (int d = 0; d < 3; ++d) {
            C.n[d] = (int)kp[d].size();
            C.keep[d] = kp[d];
            C.hx[d].resize(C.n[d]);
            for (int t = 0; t < C.n[d]; ++t) C.hx[d][t] = F.hx[d][kp[d][t]];
        }
        g->nlev++;
    }
    lasto_status st = LASTO_OK;
    for (int l = 0; l < g->nlev && st == LASTO_OK; ++l) {
        Level& L = g->lev[l];
        L.npts = (size_t)L.n[0] * L.n[1] * L.n[2] * n_batch;
        st = build_level_tables(g, l);
        if (st != LASTO_OK) break;
        // V-cycle arrays in the split layout (level 0 uses the Krylov vectors
        // below for its correction and right-hand side)
        const size_t ns = L.nsplit;
        if (l > 0) {
            st = alloc_zero(g, (void**)&L.u64, sizeof(double) * ns);
            if (st == LASTO_OK) st = alloc_zero(g, (void**)&L.u32, sizeof(float) * ns);
            if (st == LASTO_OK) st = alloc_zero(g, (void**)&L.f64, sizeof(double) * ns);
            if (st == LASTO_OK) st = alloc_zero(g, (void**)&L.f32, sizeof(float) * ns);
        }
        if (st == LASTO_OK) st = alloc_zero(g, (void**)&L.r64, sizeof(double) * ns);
        if (st == LASTO_OK) st = alloc_zero(g, (void**)&L.r32, sizeof(float) * ns);
    }
    const size_t N = g->lev[0].nsplit;
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->r, sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->p[0], sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->p[1], sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->q, sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->z, sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->x, sizeof(double) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->r32, sizeof(float) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->p32[0], sizeof(float) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->p32[1], sizeof(float) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->q32, sizeof(float) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->e32, sizeof(float) * N);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->z32, sizeof(float) * N);
    // one partial per block of any reducing launch on any level (the finest
    // level's pointwise launch has the most blocks; a fused dot spans two
    // half-sweeps), and 25 per block of the moment reduction
    size_t nparts = (size_t)25 * kReduceBlocks;
    for (int l = 0; l < g->nlev; ++l) {
        nparts = std::max(nparts, (size_t)interior_blocks(g->lev[l].view));
        nparts = std::max(nparts, (size_t)2 * half_blocks(g->lev[l].view));
        nparts = std::max(nparts, (size_t)gs_block_parts(g->lev[l].view));
        nparts = std::max(nparts, (size_t)row_blocks(g->lev[l].view));
        nparts = std::max(nparts, (size_t)flat_blocks<float>(g->lev[l].view));
        nparts = std::max(nparts, (size_t)flat_blocks<double>(g->lev[l].view));
    }
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->partials, sizeof(double) * nparts);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->scalars, sizeof(double) * kNumScalars);
    if (st == LASTO_OK) st = alloc_zero(g, (void**)&g->moments, sizeof(double) * 25 * kMaxBatch);
    if (st == LASTO_OK) {
        // one copy of the finest level (natural-layout kernels that work per right-hand side)
        g->cview = g->lev[0].view;
        g->cview.nz = g->cview.nzc;
        g->cview.cs = (size_t)g->cview.nz * g->cview.ny * g->cview.W;
        g->cview.ax[2].n = g->cview.nzc;
    }
    if (st == LASTO_OK) {
        g->stage_bytes = 1 << 20;
        st = alloc_zero(g, (void**)&g->stage, g->stage_bytes);
    }
    if (st == LASTO_OK) {
        // the scalars, then the first right-hand side's moments (copied while a solve runs)
        if (hipHostMalloc((void**)&g->h_scalars, sizeof(double) * (kNumScalars + 25)) != hipSuccess)
            st = fail(LASTO_ERR_ALLOC, "lasto_grid_create: pinned host scalars");
    }
    if (st == LASTO_OK) {
        // level descriptors of the single-workgroup tail: every level from the
        // first one with at most kTailMaxPts nodes down to the coarsest
        g->tail_top = g->nlev - 1;
        for (int l = 0; l < g->nlev; ++l)
            if (g->lev[l].npts <= kTailMaxPts) {
                g->tail_top = l;
                break;
            }
        st = build_lds_tail(g);
        if (st == LASTO_OK) st = build_coarse_fdm(g);
        if (st == LASTO_OK) choose_coarse_gemm_level(g);
    }
    if (st == LASTO_OK) {
        std::vector<TailLevel> tl(g->nlev);
        for (int l = 0; l < g->nlev; ++l) {
            Level& L = g->lev[l];
            tl[l].V = L.view;
            tl[l].u64 = l ? L.u64 : g->z;
            tl[l].f64 = l ? L.f64 : g->r;
            tl[l].r64 = L.r64;
            tl[l].u32 = l ? L.u32 : g->z32;
            tl[l].f32 = l ? L.f32 : g->r32;
            tl[l].r32 = L.r32;
        }
        if (hipMalloc((void**)&g->tail_dev, sizeof(TailLevel) * g->nlev) != hipSuccess ||
            hipMemcpy(g->tail_dev, tl.data(), sizeof(TailLevel) * g->nlev, hipMemcpyHostToDevice) != hipSuccess)
            st = fail(LASTO_ERR_HIP, "lasto_grid_create: tail level table");
    }
    if (st == LASTO_OK) {
        if (hipError_t e = hipStreamSynchronize(g->stream); e != hipSuccess)
            st = fail(LASTO_ERR_HIP, std::string("lasto_grid_create: ") + hipGetErrorString(e));
    }
    if (st != LASTO_OK) {
        free_grid(g);
        delete g;
        return st;
    }
    *out = g;
    return LASTO_OK;
}

extern "C" lasto_status lasto_grid_destroy(lasto_grid g)
{
    if (!g) return LASTO_OK;
    (void)hipStreamSynchronize(g->stream);
    free_grid(g);
    delete g;
    return LASTO_OK;
}

extern "C" lasto_status lasto_grid_levels(lasto_grid g, int* n_levels)
{
    if (!g || !n_levels) return fail(LASTO_ERR_ARG, "lasto_grid_levels: NULL argument");
    *n_levels = g->nlev;
    return LASTO_OK;
}

extern "C" lasto_status lasto_grid_level_shape(lasto_grid g, int level, int* out3)
{
    if (!g || !out3) return fail(LASTO_ERR_ARG, "lasto_grid_level_shape: NULL argument");
    if (level < 0 || level >= g->nlev) return fail(LASTO_ERR_ARG, "lasto_grid_level_shape: level out of range");
    for (int d = 0; d < 3; ++d) out3[d] = g->lev[level].n[d];
    return LASTO_OK;
}

extern "C" lasto_status lasto_grid_level_nodes(lasto_grid g, int level, int* ix, int* iy, int* iz)
{
    if (!g || !ix || !iy || !iz) return fail(LASTO_ERR_ARG, "lasto_grid_level_nodes: NULL argument");
    if (level < 0 || level >= g->nlev) return fail(LASTO_ERR_ARG, "lasto_grid_level_nodes: level out of range");
    int* out[3] = {ix, iy, iz};
    for (int d = 0; d < 3; ++d) {
        const std::vector<double>& xf = g->lev[0].hx[d];
        const std::vector<double>& xc = g->lev[level].hx[d];
        for (size_t I = 0; I < xc.size(); ++I) {
            const auto it = std::lower_bound(xf.begin(), xf.end(), xc[I]);
            if (it == xf.end() || *it != xc[I]) return fail(LASTO_ERR_STATE, "lasto_grid_level_nodes: not nested");
            out[d][I] = (int)(it - xf.begin());
        }
    }
    return LASTO_OK;
}
