// Solver drivers for eq. (3.2) on the graded mesh: the V-cycle
// preconditioner, MG-preconditioned CG (FP64), plain V-cycle iteration, and
// FP32 inner solves inside FP64 defect-correction refinement.
//
// Every step is a kernel on the grid's stream; dot products and norms are
// reduced on the device into a scalar array that later kernels read (so CG's
// alpha and beta never travel to the host). The host reads one 8-byte norm
// per outer iteration to decide convergence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace lasto {

// symmetric sweep pairs on the coarsest level (at most 5^3 nodes, 27 unknowns)
constexpr int kCoarseSweeps = 4;

template <typename T> struct Buf;
template <> struct Buf<double> {
    static double* u(Level& L) { return L.u64; }
    static double* f(Level& L) { return L.f64; }
    static double* r(Level& L) { return L.r64; }
};
template <> struct Buf<float> {
    static float* u(Level& L) { return L.u32; }
    static float* f(Level& L) { return L.f32; }
    static float* r(Level& L) { return L.r32; }
};

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(LASTO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// interior nodes of a level, all copies of a batch
static double interior_pts(const LevelView& V)
{
    return (double)(V.nx - 2) * (V.ny - 2) * (V.nzc - 2) * (V.nz / V.nzc);
}

// algorithmic bytes of a finest-level launch: `per_node` bytes per interior node
static void count(lasto_grid g, int l, double per_node)
{
    if (l == 0) g->alg_bytes += per_node * interior_pts(g->lev[0].view);
}

// A half-sweep at level l. With profiling on, each finest-level half-sweep
// is launched with a pair of events that take the dispatch's own start and
// end timestamps, so their difference is the kernel's execution time.
template <typename T>
static hipError_t half(lasto_grid g, int l, T* u, const T* f, int colour, int zero_in, double* dotp,
                       int* nparts = nullptr)
{
    const LevelView& V = g->lev[l].view;
    const bool timed = g->prof_on && l == 0;
    // half the interior nodes read f and (unless the other colour is zero)
    // one other-colour value, and write their own value
    count(g, l, 0.5 * sizeof(T) * (zero_in ? 2.0 : 3.0));
    if (!timed) return launch_half<T>(V, u, f, colour, zero_in, T(1), dotp, g->stream, nparts, l == 0);
    if ((size_t)(2 * g->prof_used + 2) > g->prof_ev.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            g->prof_ev.push_back(e);
        }
    }
    hipError_t err = launch_half<T>(V, u, f, colour, zero_in, T(1), dotp, g->stream, nparts, 1,
                                    g->prof_ev[2 * g->prof_used], g->prof_ev[2 * g->prof_used + 1]);
    if (err != hipSuccess) return err;
    // algorithmic bytes: half the interior nodes read f and (unless the
    // other colour is zero) one other-colour value, and write their own value
    const double pts = 0.5 * (double)(V.nx - 2) * (V.ny - 2) * (V.nzc - 2) * (V.nz / V.nzc);
    g->prof_bytes += pts * sizeof(T) * (zero_in ? 2.0 : 3.0);
    if (sizeof(T) == 4) g->prof_fp32++;
    g->prof_used++;
    return hipSuccess;
}

// nsw half-sweeps at level l in one pass (launch_gs_block), timed and
// counted as half() does: from zero it reads f and writes u (both colours),
// otherwise it also reads one colour of uin.
template <typename T>
static hipError_t sweeps(lasto_grid g, int l, const T* uin, const T* f, T* u, int c0, int nsw, int zero_in,
                         double* dotp, int* nparts = nullptr)
{
    const LevelView& V = g->lev[l].view;
    const bool timed = g->prof_on && l == 0;
    const double per_node = sizeof(T) * (zero_in ? 2.0 : 2.5);
    count(g, l, per_node);
    if (!timed) return launch_gs_block<T>(V, uin, f, u, c0, nsw, zero_in, T(1), dotp, g->stream, nparts, l == 0);
    if ((size_t)(2 * g->prof_used + 2) > g->prof_ev.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            g->prof_ev.push_back(e);
        }
    }
    hipError_t err = launch_gs_block<T>(V, uin, f, u, c0, nsw, zero_in, T(1), dotp, g->stream, nparts, 1,
                                        g->prof_ev[2 * g->prof_used], g->prof_ev[2 * g->prof_used + 1]);
    if (err != hipSuccess) return err;
    g->prof_bytes += per_node * interior_pts(V);
    if (sizeof(T) == 4) g->prof_fp32++;
    g->prof_used++;
    return hipSuccess;
}

// half-sweeps per pass at level l: opts.fused_sweeps when it sets a length
// (every level that sweeps), else one launch each (measured faster at 257^3:
// the half-sweep streams at the copy ceiling, while the fused pass is bound by
// its per-step latency)
static int pass_sweeps(lasto_grid g, int l)
{
    (void)l;
    return g->fused_sweeps > 1 ? g->fused_sweeps : 1;
}

// V(nu1, nu2) at level l on A u = f with zero faces, in place in the split
// layout, starting from u = 0 (zero_start) or from the u given (level 0
// only; coarse levels always start from zero). Pre-smoothing sweeps update
// red then black, post-smoothing black then red, and the coarsest level runs
// a symmetric sweep sequence, so the cycle from zero is a symmetric operator
// (a valid CG preconditioner). With dotp, partials of <f, u>_W over the
// result are written (count in *ndot).
template <typename T>
static lasto_status vcycle_level(lasto_grid g, int l, int nu1, int nu2, const T* f, T* u, double* dotp, int* ndot,
                                 bool zero_start = true)
{
    Level& L = g->lev[l];
    const LevelView& V = L.view;
    hipStream_t s = g->stream;
    if (g->coarse_mode == 0 && g->cg && l == g->cg_level) {
        // exact coarsest solve by GEMMs (nothing below this level runs)
        if (lasto_status e = coarse_gemm_solve<T>(g, f, u, s); e != LASTO_OK) return e;
        if (dotp) {
            HIPCHK(launch_dot<T>(V, f, u, dotp, s));
            *ndot = row_blocks(V);
        }
        return LASTO_OK;
    }
    if (g->coarse_mode != 1 && l == g->cfdm_level) {
        // exact coarsest solve (its result does not depend on a start)
        HIPCHK(launch_coarse_fdm<T>(g, f, u, s));
        if (dotp) {
            HIPCHK(launch_dot<T>(V, f, u, dotp, s));
            *ndot = row_blocks(V);
        }
        return LASTO_OK;
    }
    if (sizeof(T) == 4 && l == g->tail32_top) {
        // the rest of the FP32 cycle in one workgroup, all levels in LDS
        HIPCHK(launch_tail_lds((float*)u, (const float*)f, g->lds_tabs, nu1, nu2, kCoarseSweeps, zero_start ? 1 : 0,
                               g->lds_plan, g->lds_plan_dev, s));
        if (dotp) {
            HIPCHK(launch_dot<T>(V, f, u, dotp, s));
            *ndot = row_blocks(V);
        }
        return LASTO_OK;
    }
    if (l == g->tail_top) {
        // the rest of the cycle in one workgroup; its level-0 buffers are the
        // Krylov vectors, which are the only ones a level-0 cycle is given
        if (l == 0 && !((void*)u == (void*)g->z || (void*)u == (void*)g->z32))
            return fail(LASTO_ERR_STATE, "vcycle: level-0 tail needs the grid's Krylov vectors");
        HIPCHK(launch_tail<T>(g->tail_dev + l, g->nlev - l, nu1, nu2, kCoarseSweeps, zero_start ? 1 : 0, s));
        if (dotp) {
            HIPCHK(launch_dot<T>(V, f, u, dotp, s));
            *ndot = row_blocks(V);
        }
        return LASTO_OK;
    }
    if (g->lc_net && l == g->lc_level) {
        // the learned coarse correction proposes this level's start (kept
        // only if it lowers the level's residual, else zero)
        if (lasto_status e = learned_coarse_start<T>(g, l, f, u, Buf<T>::r(L)); e != LASTO_OK) return e;
        zero_start = false;
    }
    // pre-smoothing: half-sweep h updates colour h & 1 (red first); from a
    // zero start the first blk of them share one pass (in place: nothing is
    // read from u)
    const int blk = std::min(pass_sweeps(g, l), gs_block_max<T>());
    int h0 = 0;
    if (zero_start && blk >= 2) {
        h0 = std::min(blk, 2 * nu1);
        HIPCHK(sweeps<T>(g, l, u, f, u, 0, h0, 1, nullptr));
    }
    for (int h = h0; h < 2 * nu1; ++h) HIPCHK(half<T>(g, l, u, f, h & 1, h == 0 && zero_start, nullptr));
    // The pre-smoothing ended with a black half-sweep, so the residual is zero
    // on black nodes: compute and restrict the red part only. (The black part
    // of r is never written and stays zero.)
    Level& C = g->lev[l + 1];
    T* r = Buf<T>::r(L);
    HIPCHK(launch_residual_colour<T>(V, u, f, r, 0, s));
    HIPCHK(launch_restrict_red<T>(V, C.view, r, Buf<T>::f(C), s));
    // red residual: read u (both colours) and f, write r at red nodes;
    // restriction: read the red residual, write the coarse right-hand side
    const double cfrac = l == 0 ? interior_pts(C.view) / interior_pts(V) : 0.0;
    count(g, l, 0.5 * 4 * sizeof(T));
    count(g, l, (0.5 + cfrac) * sizeof(T));
    // levels below the finest take nu_coarse sweeps each way when it is set
    const int nc1 = g->nu_coarse > 0 ? g->nu_coarse : nu1, nc2 = g->nu_coarse > 0 ? g->nu_coarse : nu2;
    lasto_status st = vcycle_level<T>(g, l + 1, nc1, nc2, Buf<T>::f(C), Buf<T>::u(C), nullptr, nullptr);
    if (st != LASTO_OK) return st;
    // a post-smoothing that starts with a black half-sweep recomputes every
    // black value, so only red nodes take the interpolated correction. With
    // a fused first pass the corrected red values go to r (free since the
    // restriction) and the pass reads them there and writes u.
    const int h1 = nu2 > 0 && blk >= 2 ? std::min(blk, 2 * nu2) : 0;
    if (h1 > 0) HIPCHK(launch_prolong_red_to<T>(V, C.view, Buf<T>::u(C), u, r, s));
    else if (nu2 > 0) HIPCHK(launch_prolong_red<T>(V, C.view, Buf<T>::u(C), u, s));
    else HIPCHK(launch_prolong_add<T>(V, C.view, Buf<T>::u(C), u, s));
    // read-modify-write of u at red (or all) nodes plus the coarse correction
    count(g, l, (nu2 > 0 ? 0.5 : 1.0) * 2 * sizeof(T) + cfrac * sizeof(T));
    // post-smoothing: half-sweep h updates colour 1 - (h & 1) (black first);
    // the last two carry the partials of <f, u>_W
    int nb1 = 0, nb2 = 0, nbf = 0;
    const bool dot_fused = dotp && h1 == 2 * nu2 && h1 > 0;
    if (h1 > 0) HIPCHK(sweeps<T>(g, l, r, f, u, 1, h1, 0, dot_fused ? dotp : nullptr, &nbf));
    for (int h = h1; h < 2 * nu2; ++h) {
        const bool second_last = dotp && h == 2 * nu2 - 2, last = dotp && h == 2 * nu2 - 1;
        // the last half-sweep's partials follow the second last's
        HIPCHK(half<T>(g, l, u, f, (h & 1) ? 0 : 1, 0, second_last ? dotp : (last ? dotp + nb1 : nullptr),
                       (h & 1) ? &nb2 : &nb1));
    }
    if (dotp) {
        if (dot_fused) {
            *ndot = nbf;
        } else if (nu2 > 0) {
            *ndot = nb1 + nb2;
        } else {
            HIPCHK(launch_dot<T>(V, f, u, dotp, s));
            *ndot = row_blocks(V);
        }
    }
    return LASTO_OK;
}

// A launch sequence `body` (launches on g->stream only, no host reads)
// replayed from a HIP graph: the first use for a key runs eagerly (lazy
// tables, library workspaces and static launch shapes are set up outside any
// capture), the second captures the sequence on the library's own stream and
// replays it, and later uses replay. The int the body reports and the
// algorithmic bytes it counts are those of the capture.
template <typename Body>
static lasto_status graphed(lasto_grid g, const int (&key)[8], const void* const (&ptr)[4], Body body, int* aux)
{
    lasto_grid_s::VGraph* e = nullptr;
    for (auto& v : g->vgraphs)
        if (std::equal(key, key + 8, v.key) && std::equal(ptr, ptr + 4, v.ptr)) e = &v;
    if (!e) {
        lasto_grid_s::VGraph v;
        std::copy(key, key + 8, v.key);
        std::copy(ptr, ptr + 4, v.ptr);
        g->vgraphs.push_back(v);
        e = &g->vgraphs.back();
    }
    int tmp = 0;
    if (!aux) aux = &tmp;
    if (e->exec) {
        HIPCHK(hipGraphLaunch(e->exec, g->stream));
        g->alg_bytes += e->bytes;
        *aux = e->aux;
        return LASTO_OK;
    }
    if (e->uses++ == 0) return body(aux);
    if (!g->cap_stream) HIPCHK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    hipStream_t keep = g->stream;
    const double b0 = g->alg_bytes;
    HIPCHK(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
    g->stream = g->cap_stream;
    coarse_gemm_set_stream(g, g->cap_stream);
    int got = 0;
    const lasto_status st = body(&got);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->cap_stream, &graph);
    g->stream = keep;
    coarse_gemm_set_stream(g, keep);
    if (st != LASTO_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != LASTO_OK) return st;
        return fail(LASTO_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(LASTO_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
    e->exec = exec;
    e->aux = got;
    e->bytes = g->alg_bytes - b0;   // counted while capturing: this use's share
    HIPCHK(hipGraphLaunch(exec, g->stream));
    *aux = got;
    return LASTO_OK;
}

// whether launch sequences may go through graphs in this solve
static bool graphs_on(lasto_grid g, const lasto_solve_opts& o) { return o.graphs && !g->prof_on && !g->lc_net; }

// The finest-level V-cycle of the CG forms (fixed operands every step),
// through a graph when `graphs` is set
template <typename T>
static lasto_status vcycle0(lasto_grid g, const lasto_solve_opts& o, const T* f, T* u, double* dotp, int* ndot)
{
    auto body = [&](int* nd) { return vcycle_level<T>(g, 0, o.nu1, o.nu2, f, u, dotp, nd); };
    if (!graphs_on(g, o)) return body(ndot);
    const int key[8] = {1, (int)sizeof(T), o.nu1, o.nu2, g->coarse_mode, g->nu_coarse, g->fused_sweeps, 0};
    const void* const ptr[4] = {f, u, dotp, nullptr};
    return graphed(g, key, ptr, body, ndot);
}

static lasto_status reduce_to(lasto_grid g, int count, int slot)
{
    HIPCHK(launch_reduce(g->partials, 1, count, g->scalars + slot, g->stream));
    return LASTO_OK;
}

// q = A p over both colours; partials of <p, q>_W (count returned)
template <typename T>
static lasto_status apply_dot(lasto_grid g, const T* p, T* q, int* count)
{
    const LevelView& V = g->lev[0].view;
    HIPCHK(launch_apply_both<T>(V, p, q, g->partials, g->stream, count));
    // each colour reads p's other colour and centre, writes q
    lasto::count(g, 0, 3.0 * sizeof(T));
    return LASTO_OK;
}

static lasto_status read_scalars(lasto_grid g, int first, int n)
{
    HIPCHK(hipMemcpyAsync(g->h_scalars + first, g->scalars + first, sizeof(double) * n, hipMemcpyDeviceToHost,
                          g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

// Inner FP32 multigrid on A e = r32 (the FP64 residual rounded to FP32):
// `cycles` V-cycles in z32, the first from e = 0, each later one continuing
// from the current e (a stationary iteration needs no residual of its own:
// the cycle computes it after its pre-smoothing); then v += e.
static lasto_status mg32_inner(lasto_grid g, const lasto_solve_opts& o, int cycles, int* vcycles, double* v)
{
    for (int c = 0; c < cycles; ++c) {
        lasto_status st = vcycle_level<float>(g, 0, o.nu1, o.nu2, g->r32, g->z32, nullptr, nullptr, c == 0);
        if (st != LASTO_OK) return st;
        ++*vcycles;
    }
    HIPCHK(launch_add32_nat(g->lev[0].view, v, g->z32, nullptr, g->scalars, 0, 0, g->stream, true));
    count(g, 0, 4.0 + 16.0);
    return LASTO_OK;
}

// one step `it` of the inner FP32 PCG (the last when it + 1 == iters)
static lasto_status pcg32_step(lasto_grid g, const lasto_solve_opts& o, int it, int iters, double* v)
{
    const LevelView& V = g->lev[0].view;
    hipStream_t s = g->stream;
    float* rr = g->r32;   // working residual, updated in place
    int nd = 0;
    lasto_status st = vcycle_level<float>(g, 0, o.nu1, o.nu2, rr, g->z32, g->partials, &nd);
    if (st != LASTO_OK) return st;
    // <r, z>_W of every step is kept (the refinement reads the inner
    // solve's convergence from them)
    const int srz = S_RZH + it % kInnerHist, srz_old = S_RZH + (it + kInnerHist - 1) % kInnerHist;
    if (lasto_status e = reduce_to(g, nd, srz); e != LASTO_OK) return e;
    float* pn = g->p32[it & 1];
    float* po = g->p32[(it + 1) & 1];
    if (it == 0) {
        HIPCHK(launch_update_p<float>(V, g->z32, po, pn, g->scalars, srz, srz_old, 1, s));
        count(g, 0, 2 * 4.0);
    } else {
        int beta_num = srz;
        if (g->lc_net) {
            // flexible (Polak-Ribiere) beta under the learned coarse correction
            HIPCHK(launch_dot<float>(V, g->z32, g->q32, g->partials, s));
            if (lasto_status e = reduce_to(g, row_blocks(V), S_ZQ32); e != LASTO_OK) return e;
            HIPCHK(launch_flex_beta(g->scalars, srz_old, S_PQ32, S_ZQ32, S_FNUM32, s));
            count(g, 0, 8.0);
            beta_num = S_FNUM32;
        }
        // e (=, then +=) alpha_prev p_old, alpha_prev = (r,z) / (p,q) of the previous step
        HIPCHK(launch_update_px<float>(V, g->z32, po, pn, g->e32, g->scalars, beta_num, srz_old, srz_old, S_PQ32,
                                       it >= 2, s));
        count(g, 0, (it >= 2 ? 5 : 4) * 4.0);
    }
    int npq = 0;
    if (lasto_status e = apply_dot<float>(g, pn, g->q32, &npq); e != LASTO_OK) return e;
    if (lasto_status e = reduce_to(g, npq, S_PQ32); e != LASTO_OK) return e;
    if (it + 1 == iters) {
        if (it == 0) {
            HIPCHK(launch_fill_zero<float>(g->e32, split_elems(V), s));
            count(g, 0, 4.0);
        }
        HIPCHK(launch_add32_nat(V, v, g->e32, pn, g->scalars, srz, S_PQ32, s, true));
        count(g, 0, 8.0 + 16.0);
        return LASTO_OK;
    }
    // (the inner loop never reads its own residual norm)
    HIPCHK(launch_update_r<float>(V, rr, g->q32, g->scalars, srz, S_PQ32, s));
    count(g, 0, 3 * 4.0);
    return LASTO_OK;
}

// Inner FP32 PCG on A e = r32 from e = 0, `iters` steps, then v += e. The
// update e += alpha p of each step is deferred into the next step's update
// of p (which reads the old p anyway); the last step's goes straight into v
// (v += e + alpha p): its residual is not needed, since the refinement
// recomputes the true one in FP64. Each step (its V-cycle, reductions and
// updates) goes through a graph keyed by its index and whether it is the
// last, when `graphs` is set.
static lasto_status pcg32_inner(lasto_grid g, const lasto_solve_opts& o, int iters, int* vcycles, double* v)
{
    for (int it = 0; it < iters; ++it) {
        const bool last = it + 1 == iters;
        auto body = [&](int*) { return pcg32_step(g, o, it, iters, v); };
        lasto_status st;
        if (graphs_on(g, o)) {
            const int key[8] = {2, it % kInnerHist, last ? 1 : 0, o.nu1 * 64 + o.nu2, g->fused_sweeps,
                                g->coarse_mode, g->nu_coarse, it >= 2 ? 2 : it};
            const void* const ptr[4] = {v, g->r32, g->z32, nullptr};
            st = graphed(g, key, ptr, body, nullptr);
        } else {
            st = body(nullptr);
        }
        if (st != LASTO_OK) return st;
        ++*vcycles;
    }
    return LASTO_OK;
}

}  // namespace lasto

using namespace lasto;

// Dirichlet data on the faces of every right-hand side of the grid (bc 1:
// multipole field of its own moments, kept in g->moments[25 b]; bc 0: zero)
static lasto_status set_faces(lasto_grid g, const double* rho, int bc, int lmax_bc, double* v)
{
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    for (int b = 0; b < g->n_batch; ++b) {
        if (bc == 1) {
            HIPCHK(launch_moments(g, rho + b * N, g->moments + 25 * b));
            HIPCHK(launch_bc(g, 1, g->moments + 25 * b, lmax_bc, v + b * N));
        } else {
            HIPCHK(launch_bc(g, 0, g->moments, 0, v + b * N));
        }
    }
    return LASTO_OK;
}

// squared W-norm of 4 pi rho - A v for each right-hand side into slot
// base + b (default: S_BR0 + b with interior_zero, of the face data alone;
// S_BRR + b otherwise)
static lasto_status batch_norms(lasto_grid g, const double* rho, const double* v, int interior_zero, int base = -1)
{
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    const int nb = interior_blocks(g->cview);
    if (base < 0) base = interior_zero ? S_BR0 : S_BRR;
    for (int b = 0; b < g->n_batch; ++b) {
        HIPCHK(launch_residual_nat(g->cview, v + b * N, rho + b * N, 4.0 * kPi, nullptr, g->partials, interior_zero,
                                   g->stream));
        if (lasto_status e = reduce_to(g, nb, base + b); e != LASTO_OK) return e;
    }
    return LASTO_OK;
}

extern "C" void lasto_solve_opts_default(lasto_solve_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-10;
    o->max_iters = 100;
    o->nu1 = 2;
    o->nu2 = 2;
    o->method = 0;
    o->precision = 0;
    o->inner_iters = 6;
    o->guess = 0;
    o->bc = 1;
    o->lmax_bc = 4;
    o->debug_nan_iter = -1;
    o->profile = 0;
    o->fallback = 1;
}

static lasto_status judge_batch(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel, int* accepted);
static lasto_status coarse_net_check(lasto_grid g, const lasto_solve_opts& o);

// milliseconds between two recorded events (0 if either is missing)
static double event_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.0f;
    if (!a || !b || hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

extern "C" lasto_status lasto_poisson_solve(lasto_grid g, const double* rho, double* v, const lasto_solve_opts* opts,
                                            lasto_solve_info* info)
{
    const auto t_start = std::chrono::steady_clock::now();
    if (!g) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: NULL grid");
    if (!rho || !v) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: NULL rho or v");
    lasto_solve_opts o;
    if (opts) o = *opts;
    else lasto_solve_opts_default(&o);
    if (!(o.rtol > 0.0) || o.max_iters < 1 || o.nu1 < 1 || o.nu2 < 0 || o.nu1 > 16 || o.nu2 > 16)
        return fail(LASTO_ERR_ARG, "lasto_poisson_solve: bad rtol/max_iters/nu1/nu2");
    if (o.method < 0 || o.method > 1 || o.precision < 0 || o.precision > 1 || o.bc < 0 || o.bc > 2 ||
        o.lmax_bc < 0 || o.lmax_bc > 4 || o.guess < 0 || o.guess > 3 || (o.precision == 1 && o.inner_iters < 1) ||
        o.inner_first < 0 || o.coarse < 0 || o.coarse > 2 || o.fallback < 0 || o.fallback > 1 ||
        !(o.inner_rate >= 0.0 && o.inner_rate < 1.0) || o.nu_coarse < 0 ||
        !(o.fused_sweeps == 0 || o.fused_sweeps == 1 || o.fused_sweeps == 2 || o.fused_sweeps == 4 ||
          o.fused_sweeps == 6))
        return fail(LASTO_ERR_ARG,
                    "lasto_poisson_solve: bad method/precision/bc/lmax_bc/guess/inner_iters/coarse/fallback/"
                    "inner_rate/nu_coarse/fused_sweeps");
    if (o.guess >= 2 && (o.n_atoms < 1 || !o.atoms))
        return fail(LASTO_ERR_ARG, "lasto_poisson_solve: guess 2 and 3 need the atom tables");
    if (o.guess == 3 && !o.guess_net) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: guess 3 needs guess_net");
    lasto_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    hipStream_t s = g->stream;
    g->prof_on = (o.profile == 1);
    g->coarse_mode = o.coarse;
    if (o.coarse == 0) {
        if (lasto_status e = coarse_gemm_init(g); e != LASTO_OK) return e;
    }
    if (o.coarse == 0 && g->cg) {
        inf.coarse_level = g->cg_level;
    } else {
        // the FP32 cycle reaches the LDS solve unless its LDS tail starts above it
        const bool lds_first = o.precision == 1 && g->tail32_top >= 0 && g->tail32_top < g->cfdm_level;
        inf.coarse_level = (o.coarse != 1 && !lds_first) ? g->cfdm_level : -1;
    }
    if (o.coarse_net) {
        if (lasto_status e = coarse_net_check(g, o); e != LASTO_OK) return e;
    }
    g->lc_net = o.coarse_net;
    g->lc_level = o.coarse_net ? o.coarse_net_level : -1;
    g->lc_applied = 0;
    struct LcOff {
        lasto_grid g;
        ~LcOff()
        {
            g->lc_net = nullptr;
            g->lc_level = -1;
        }
    } lc_off{g};
    g->prof_used = 0;
    g->prof_bytes = 0.0;
    g->prof_fp32 = 0;
    g->alg_bytes = 0.0;
    struct ProfOff {
        lasto_grid g;
        ~ProfOff()
        {
            g->prof_on = false;
            g->nu_coarse = 0;
            g->fused_sweeps = 0;
        }
    } prof_off{g};
    g->nu_coarse = o.nu_coarse;
    g->fused_sweeps = o.fused_sweeps;
    for (hipEvent_t& e : g->ph_ev)
        if (!e) HIPCHK(hipEventCreate(&e));
    Level& L0 = g->lev[0];
    const LevelView& V = L0.view;
    const int nb_i = interior_blocks(V);
    const double fourpi = 4.0 * kPi;
    const int nbat = g->n_batch;
    HIPCHK(hipEventRecord(g->ph_ev[0], s));

    // face values (every right-hand side of a batch from its own moments)
    if (o.bc == 0 || o.bc == 1) {
        if (lasto_status e = set_faces(g, rho, o.bc, o.lmax_bc, v); e != LASTO_OK) return e;
        // the first right-hand side's moments for info, copied to pinned host
        // memory while the solve runs (read after the solve's last wait)
        if (o.bc == 1)
            HIPCHK(hipMemcpyAsync(g->h_scalars + kNumScalars, g->moments, sizeof(double) * 25, hipMemcpyDeviceToHost,
                                  s));
    }
    HIPCHK(hipEventRecord(g->ph_ev[1], s));
    // the start inside
    if (o.guess == 1) {
        // zero interior: copy an all-zero split array onto the interior of v
        HIPCHK(launch_fill_zero<double>(g->q, split_elems(V), s));
        HIPCHK(launch_split_to_nat(V, g->q, v, s));
    } else if (o.guess >= 2) {
        AtomDev* dat = nullptr;
        if (lasto_status e = stage_atoms(g, nbat * o.n_atoms, o.atoms, 1, "lasto_poisson_solve", &dat); e != LASTO_OK)
            return e;
        HIPCHK(launch_guess_all(g, dat, o.atoms, o.n_atoms, v));
        if (o.guess == 3) {
            int acc = 0;
            if (lasto_status e = judge_batch(g, o.guess_net, rho, v, nullptr, &acc); e != LASTO_OK) return e;
            inf.guess_accepted = acc;
            if (acc < nbat) inf.fallback_used |= 1;
        }
    }
    HIPCHK(hipEventRecord(g->ph_ev[2], s));

    // reference norm ||b - A v_bc||_W and initial residual r (split)
    HIPCHK(launch_residual_nat(V, v, rho, fourpi, nullptr, g->partials, 1, s));
    if (lasto_status e = reduce_to(g, nb_i, S_R0); e != LASTO_OK) return e;
    // (the mixed form keeps only the FP32 rounding of r, which is all its
    // inner solve reads)
    if (o.precision == 1) HIPCHK(launch_residual_nat32(V, v, rho, fourpi, g->r32, g->partials, s));
    else HIPCHK(launch_residual_nat(V, v, rho, fourpi, g->r, g->partials, 0, s));
    count(g, 0, 8.0 + (o.precision == 1 ? 20.0 : 24.0));
    if (lasto_status e = reduce_to(g, nb_i, S_RR); e != LASTO_OK) return e;
    HIPCHK(launch_fill_zero<double>(g->scalars + S_BAD, 1, s));
    HIPCHK(launch_fill_zero<double>(g->scalars + S_LC_ACC, 1, s));
    if (lasto_status e = read_scalars(g, 0, kNumScalars); e != LASTO_OK) return e;
    const double r0sq = g->h_scalars[S_R0];
    const double r0 = std::sqrt(r0sq);
    double rel = (r0 > 0.0) ? std::sqrt(g->h_scalars[S_RR]) / r0 : 0.0;
    inf.rel_start = rel;
    // rel is the true residual of v with no CG correction pending (the mixed
    // form and the stationary cycles recompute it every step; CG only when it
    // folds its correction into v), so the exit need not compute it again
    bool true_resid = true;
    // A batch iterates on the stacked system (one norm, one set of CG
    // coefficients for all copies, which is CG on the block-diagonal system)
    // and then checks every copy against its own reference norm.
    double br0[kMaxBatch] = {0.0};
    if (nbat > 1) {
        if (lasto_status e = batch_norms(g, rho, v, 1); e != LASTO_OK) return e;
        if (lasto_status e = read_scalars(g, S_BR0, nbat); e != LASTO_OK) return e;
        for (int b = 0; b < nbat; ++b) br0[b] = std::sqrt(g->h_scalars[S_BR0 + b]);
    }
    double target = o.rtol;
    if (!std::isfinite(r0) || !std::isfinite(rel)) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: non-finite rho or v");
    if (r0 == 0.0) {
        // the face data alone satisfy every interior equation exactly (for
        // instance rho = 0 with zero faces): the solution is the zero interior
        HIPCHK(launch_fill_zero<double>(g->q, split_elems(V), s));
        HIPCHK(launch_split_to_nat(V, g->q, v, s));
        HIPCHK(hipStreamSynchronize(s));
        inf.n_batch = nbat;
        inf.ms_bc = event_ms(g->ph_ev[0], g->ph_ev[1]);
        inf.ms_guess = event_ms(g->ph_ev[1], g->ph_ev[2]);
        if (o.bc == 1) std::memcpy(inf.moments, g->h_scalars + kNumScalars, sizeof(double) * 25);
        inf.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        if (info) *info = inf;
        return LASTO_OK;
    }

    lasto_status result = LASTO_OK;
    const char* why = "";
    double best = rel;
    int grow = 0;
    int it = 0, cg_it = 0;
    int max_it = o.max_iters;
    // the form running now: the mixed form can hand over to FP64 MG-PCG
    int prec = o.precision;
    int method = o.method;
    // adaptive inner step counts of the mixed form: q is the expected
    // per-step reduction, first the option's, then the inner PCG's own
    // (the decrease of sqrt(<r, z>_W) over a refinement's steps, which runs
    // a little slower than the true residual's), raised to the true
    // residual's per-step reduction over a later
    // refinement when that is slower (a refinement reducing by 1e-5 or more
    // may have stopped at FP32 rounding, so it does not count)
    double q_rate = o.inner_rate;
    int pending_rate = 0, rz_steps = 0;
    double rate_from = 0.0;
    // CG accumulates its correction in the split array x (zero now) and adds
    // it to v when it stops or restarts
    bool cg = (prec == 0 && method == 0);
    if (cg) {
        HIPCHK(launch_fill_zero<double>(g->x, split_elems(V), s));
        count(g, 0, 8.0);
    }
  for (;;) {
    while (rel > target && it < max_it) {
        if (o.debug_nan_iter == it) {
            const size_t at = sidx(V, V.nx / 2, V.ny / 2, V.nz / 2);
            if (prec == 1) HIPCHK(launch_inject_nan(g->r32, at, s));
            else HIPCHK(launch_inject_nan(g->r, at, s));
        }
        if (prec == 1) {
            // FP32 inner solve on the FP32 rounding of the FP64 residual (the
            // equation is linear, so the residual's scale does not matter
            // while it stays far inside the FP32 range), then v += e in FP64
            const int cap = (inf.refinements == 0 && o.inner_first > 0) ? o.inner_first : o.inner_iters;
            int inner = cap;
            if (o.inner_rate > 0.0 && rel > target) {
                // just enough steps at the expected rate to reach the target
                // (planned against 0.7 of it, so that a refinement that
                // lands a hair above it does not cost another)
                const double want = std::log(0.7 * target / rel) / std::log(q_rate);
                inner = std::max(1, std::min(cap, (int)std::ceil(want - 1e-9)));
            }
            const double rel_before = rel;
            if (method == 1) {
                if (lasto_status e = mg32_inner(g, o, inner, &inf.vcycles, v); e != LASTO_OK) return e;
            } else {
                if (lasto_status e = pcg32_inner(g, o, inner, &inf.vcycles, v); e != LASTO_OK) return e;
            }
            HIPCHK(launch_residual_nat32(V, v, rho, fourpi, g->r32, g->partials, s));
            count(g, 0, 20.0);
            if (lasto_status e = reduce_to(g, nb_i, S_RR); e != LASTO_OK) return e;
            inf.refinements++;
            pending_rate = o.inner_rate > 0.0 && inf.refinements > 1 && inner > 1 ? inner : 0;
            rate_from = rel_before;
            inf.inner_rate = q_rate;
            rz_steps = (o.inner_rate > 0.0 && method == 0) ? std::min(inner, kInnerHist) : 0;
        } else if (method == 1) {
            // plain V-cycle iteration: v += V(r), r = b - A v
            lasto_status st = vcycle_level<double>(g, 0, o.nu1, o.nu2, g->r, g->z, nullptr, nullptr);
            if (st != LASTO_OK) return st;
            inf.vcycles++;
            HIPCHK(launch_add_nat(V, v, g->z, s));
            HIPCHK(launch_residual_nat(V, v, rho, fourpi, g->r, g->partials, 0, s));
            count(g, 0, 24.0 + 24.0);
            if (lasto_status e = reduce_to(g, nb_i, S_RR); e != LASTO_OK) return e;
        } else {
            // one MG-preconditioned CG step
            int nd = 0;
            lasto_status st = vcycle0<double>(g, o, g->r, g->z, g->partials, &nd);
            if (st != LASTO_OK) return st;
            inf.vcycles++;
            const int srz = S_RZ0 + (cg_it & 1), srz_old = S_RZ0 + ((cg_it + 1) & 1);
            if (lasto_status e = reduce_to(g, nd, srz); e != LASTO_OK) return e;
            double* pn = g->p[cg_it & 1];
            double* po = g->p[(cg_it + 1) & 1];
            int beta_num = srz;
            if (g->lc_net && cg_it > 0) {
                // the learned coarse correction makes the preconditioner vary
                // from step to step: flexible (Polak-Ribiere) beta
                HIPCHK(launch_dot<double>(V, g->z, g->q, g->partials, s));
                if (lasto_status e = reduce_to(g, row_blocks(V), S_ZQ); e != LASTO_OK) return e;
                HIPCHK(launch_flex_beta(g->scalars, srz_old, S_PQ, S_ZQ, S_FNUM, s));
                count(g, 0, 16.0);
                beta_num = S_FNUM;
            }
            HIPCHK(launch_update_p<double>(V, g->z, po, pn, g->scalars, beta_num, srz_old, cg_it == 0, s));
            count(g, 0, (cg_it == 0 ? 2 : 3) * 8.0);
            int npq = 0;
            if (lasto_status e = apply_dot<double>(g, pn, g->q, &npq); e != LASTO_OK) return e;
            if (lasto_status e = reduce_to(g, npq, S_PQ); e != LASTO_OK) return e;
            int nb_r = 0;
            HIPCHK(launch_update_xr<double>(V, g->x, g->r, pn, g->q, g->scalars, srz, S_PQ, g->partials, s, &nb_r));
            count(g, 0, 6 * 8.0);
            if (lasto_status e = reduce_to(g, nb_r, S_RR); e != LASTO_OK) return e;
            cg_it++;
        }
        true_resid = !cg;
        // the residual norm, and (mixed form) whether an FP32 correction broke
        // down; with adaptive inner steps also the inner PCG's <r, z>_W
        const int last_slot = rz_steps > 0 ? S_RZH + kInnerHist - 1 : S_BAD;
        if (lasto_status e = read_scalars(g, S_RR, last_slot - S_RR + 1); e != LASTO_OK) return e;
        rel = std::sqrt(g->h_scalars[S_RR]) / r0;
        if (it < 128) inf.resid_hist[it] = rel;
        ++it;
        if (rz_steps >= 2) {
            // (A and the cycle are negative definite: <r, z>_W < 0)
            const int last = rz_steps - 1;
            const double a = std::fabs(g->h_scalars[S_RZH]), b = std::fabs(g->h_scalars[S_RZH + last]);
            if (a > 0.0 && b > 0.0 && std::isfinite(a) && std::isfinite(b) && b < a)
                q_rate = std::min(0.9, std::max(1e-3, std::pow(b / a, 0.5 / last)));
        }
        rz_steps = 0;
        if (pending_rate > 0 && std::isfinite(rel) && rel > 0.0 && rate_from > 0.0) {
            const double red = rel / rate_from;
            if (red > 1e-5 && red < 1.0) q_rate = std::max(q_rate, std::pow(red, 1.0 / pending_rate));
        }
        pending_rate = 0;
        if (prec == 1 && g->h_scalars[S_BAD] != 0.0) {
            result = LASTO_ERR_DIVERGED;
            why = "lasto_poisson_solve: the FP32 inner solve produced non-finite values (v kept finite)";
            break;
        }
        if (!std::isfinite(rel)) {
            result = LASTO_ERR_DIVERGED;
            why = "lasto_poisson_solve: residual not finite";
            break;
        }
        if (rel < best) {
            best = rel;
            grow = 0;
        } else if (rel > 1e3 * best && ++grow >= 3) {
            result = LASTO_ERR_DIVERGED;
            why = "lasto_poisson_solve: residual growing";
            break;
        }
        if (rel <= target && cg) {
            // the CG residual is a recurrence: fold the correction into v,
            // confirm with the true residual, and restart CG from it if the
            // two have drifted apart
            HIPCHK(launch_add_nat(V, v, g->x, s));
            HIPCHK(launch_fill_zero<double>(g->x, split_elems(V), s));
            HIPCHK(launch_residual_nat(V, v, rho, fourpi, g->r, g->partials, 0, s));
            count(g, 0, 24.0 + 8.0 + 24.0);
            if (lasto_status e = reduce_to(g, nb_i, S_RR); e != LASTO_OK) return e;
            if (lasto_status e = read_scalars(g, S_RR, 1); e != LASTO_OK) return e;
            rel = std::sqrt(g->h_scalars[S_RR]) / r0;
            true_resid = true;
            cg_it = 0;
        }
    }
    if (result == LASTO_OK && rel > target && it >= max_it) {
        result = LASTO_ERR_NOT_CONVERGED;
        why = "lasto_poisson_solve: tolerance not reached within max_iters";
    }
    if (result != LASTO_OK && prec == 1 && o.fallback == 1) {
        // the mixed form failed: finish as FP64 MG-PCG from the current
        // iterate (finite: a broken-down correction never reaches v), with
        // max_iters more iterations
        inf.fallback_used |= 2;
        prec = 0;
        method = 0;
        cg = true;
        cg_it = 0;
        grow = 0;
        result = LASTO_OK;
        why = "";
        max_it = it + o.max_iters;
        HIPCHK(launch_fill_zero<double>(g->x, split_elems(V), s));
        HIPCHK(launch_residual_nat(V, v, rho, fourpi, g->r, g->partials, 0, s));
        count(g, 0, 8.0 + 24.0);
        if (lasto_status e = reduce_to(g, nb_i, S_RR); e != LASTO_OK) return e;
        if (lasto_status e = read_scalars(g, S_RR, 1); e != LASTO_OK) return e;
        rel = std::sqrt(g->h_scalars[S_RR]) / r0;
        best = rel;
        true_resid = true;
        if (!std::isfinite(rel)) {
            result = LASTO_ERR_DIVERGED;
            why = "lasto_poisson_solve: residual not finite";
            break;
        }
        continue;
    }
    if (nbat > 1 && result == LASTO_OK && rel <= target && it < max_it) {
        // every copy against its own reference norm; tighten the stacked
        // target while one of them is still above the tolerance
        if (lasto_status e = batch_norms(g, rho, v, 0); e != LASTO_OK) return e;
        if (lasto_status e = read_scalars(g, S_BRR, nbat); e != LASTO_OK) return e;
        double worst = 0.0;
        for (int b = 0; b < nbat; ++b)
            if (br0[b] > 0.0) worst = std::max(worst, std::sqrt(g->h_scalars[S_BRR + b]) / br0[b]);
        if (std::isfinite(worst) && worst > o.rtol) {
            target *= 0.5 * o.rtol / worst;
            continue;
        }
    }
    break;
  }
    // fold any CG correction not yet in v (the loop stopped on max_iters or
    // a breakdown; x holds the last finite correction), then the true
    // residual of the returned iterate, unless the loop ended on it (the same
    // kernel and launch shape: the same bits)
    if (true_resid) {
        inf.rel_resid = rel;
    } else {
        if (cg) HIPCHK(launch_add_nat(V, v, g->x, s));
        HIPCHK(launch_residual_nat(V, v, rho, fourpi, nullptr, g->partials, 0, s));
        if (lasto_status e = reduce_to(g, nb_i, S_TMP); e != LASTO_OK) return e;
        if (lasto_status e = read_scalars(g, S_TMP, 1); e != LASTO_OK) return e;
        inf.rel_resid = std::sqrt(g->h_scalars[S_TMP]) / r0;
    }
    HIPCHK(hipEventRecord(g->ph_ev[3], s));
    inf.iters = it;
    inf.n_batch = nbat;
    if (nbat > 1) {
        if (lasto_status e = batch_norms(g, rho, v, 0); e != LASTO_OK) return e;
        if (lasto_status e = read_scalars(g, S_BRR, nbat); e != LASTO_OK) return e;
        double worst = 0.0;
        for (int b = 0; b < nbat; ++b) {
            inf.batch_rel_resid[b] = br0[b] > 0.0 ? std::sqrt(g->h_scalars[S_BRR + b]) / br0[b] : 0.0;
            worst = std::max(worst, inf.batch_rel_resid[b]);
        }
        inf.rel_resid = std::max(inf.rel_resid, worst);
    } else {
        inf.batch_rel_resid[0] = inf.rel_resid;
    }
    // learned coarse corrections accepted on the device
    if (g->lc_applied > 0) {
        if (lasto_status e = read_scalars(g, S_LC_ACC, 1); e != LASTO_OK) return e;
        inf.coarse_applied = g->lc_applied;
        inf.coarse_accepted = (int)g->h_scalars[S_LC_ACC];
    }
    HIPCHK(hipStreamSynchronize(s));
    if (g->prof_on) {
        // the stream is synchronised: every event has completed
        double ms = 0.0;
        for (int k = 0; k < g->prof_used; ++k) {
            float e = 0.0f;
            HIPCHK(hipEventElapsedTime(&e, g->prof_ev[2 * k], g->prof_ev[2 * k + 1]));
            ms += e;
        }
        inf.smooth_launches = g->prof_used;
        inf.smooth_ms = ms;
        inf.smooth_bytes = g->prof_bytes;
        inf.smooth_fp32 = g->prof_fp32;
    }
    inf.ms_bc = event_ms(g->ph_ev[0], g->ph_ev[1]);
    inf.ms_guess = event_ms(g->ph_ev[1], g->ph_ev[2]);
    inf.ms_cycles = event_ms(g->ph_ev[2], g->ph_ev[3]);
    inf.alg_bytes = g->alg_bytes;
    if (result == LASTO_OK && !(inf.rel_resid <= o.rtol)) {
        result = LASTO_ERR_NOT_CONVERGED;
        why = "lasto_poisson_solve: tolerance not reached within max_iters";
    }
    if (!std::isfinite(inf.rel_resid)) {
        result = LASTO_ERR_DIVERGED;
        why = "lasto_poisson_solve: residual not finite";
    }
    if (o.bc == 1) std::memcpy(inf.moments, g->h_scalars + kNumScalars, sizeof(double) * 25);
    inf.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (info) *info = inf;
    if (result != LASTO_OK) return fail(result, why);
    return LASTO_OK;
}

extern "C" lasto_status lasto_boundary_values(lasto_grid g, const double* rho, int bc, int lmax_bc, double* v,
                                              double* moments_out)
{
    if (!g || !v || (bc == 1 && !rho)) return fail(LASTO_ERR_ARG, "lasto_boundary_values: NULL argument");
    if ((bc != 0 && bc != 1) || lmax_bc < 0 || lmax_bc > 4)
        return fail(LASTO_ERR_ARG, "lasto_boundary_values: bc must be 0 or 1, lmax_bc 0..4");
    if (lasto_status e = set_faces(g, rho, bc, lmax_bc, v); e != LASTO_OK) return e;
    if (moments_out && bc == 1)
        HIPCHK(hipMemcpyAsync(moments_out, g->moments, sizeof(double) * 25 * g->n_batch, hipMemcpyDeviceToHost,
                              g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

// ||4 pi rho - A v||_W (interior_zero: of the face data alone), squared, into slot
static lasto_status resid_norm2(lasto_grid g, const double* rho, const double* v, int interior_zero, int slot)
{
    const LevelView& V = g->lev[0].view;
    HIPCHK(launch_residual_nat(V, v, rho, 4.0 * kPi, nullptr, g->partials, interior_zero, g->stream));
    return reduce_to(g, interior_blocks(V), slot);
}

// Scratch of the learned entry points (zero-filled once, on first use).
enum { LS_R = 0, LS_ZERO = 1, LS_PLAIN = 2, LS_LEARNED = 3, LS_SU = 4, LS_SF = 5 };

static lasto_status learned_scratch(lasto_grid g)
{
    const size_t n = split_elems(g->lev[0].view);
    for (double*& a : g->lscr) {
        if (a) continue;
        HIPCHK(hipMalloc(&a, sizeof(double) * n));
        HIPCHK(launch_fill_zero<double>(a, n, g->stream));
    }
    return LASTO_OK;
}

// rho in the split layout in the learned scratch, for smooth_nat
static lasto_status stage_rho_split(lasto_grid g, const double* rho)
{
    HIPCHK(launch_nat_to_split(g->lev[0].view, rho, g->lscr[LS_SF], g->stream));
    return LASTO_OK;
}

// one red-black sweep on A v = 4 pi rho in place on natural v (faces kept),
// through the split layout in the learned scratch (rho staged there first)
static lasto_status smooth_nat(lasto_grid g, double* v)
{
    const LevelView& V = g->lev[0].view;
    double* su = g->lscr[LS_SU];
    double* sf = g->lscr[LS_SF];
    HIPCHK(launch_nat_to_split(V, v, su, g->stream));
    HIPCHK(launch_half_keep_faces<double>(V, su, sf, 0, 4.0 * kPi, g->stream));
    HIPCHK(launch_half_keep_faces<double>(V, su, sf, 1, 4.0 * kPi, g->stream));
    HIPCHK(launch_split_to_nat(V, su, v, g->stream));
    return LASTO_OK;
}

// Plain multigrid judges a learned candidate: v (the plain one) and
// v_learned = v + cscale * y each get one red-black sweep (which removes the
// grid-scale roughness any cycle removes cheaply, leaving the smooth error
// that decides how many cycles remain), and v receives the one with the
// smaller residual.
static lasto_status judge(lasto_grid g, const double* rho, double* v, const float* y, double cscale, double* rel,
                          int* accepted)
{
    const LevelView& V = g->lev[0].view;
    hipStream_t s = g->stream;
    const size_t nn = (size_t)V.nx * V.ny * V.nz;
    // the plain candidate is swept in a copy, the learned one in v itself,
    // and the plain one goes back to v only if it wins
    double* keep_plain = g->lscr[LS_PLAIN];
    if (lasto_status e = resid_norm2(g, rho, v, 1, S_R0); e != LASTO_OK) return e;
    HIPCHK(hipMemcpyAsync(keep_plain, v, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    if (lasto_status e = stage_rho_split(g, rho); e != LASTO_OK) return e;
    if (y) HIPCHK(launch_add_f32_nat(V, v, y, cscale, s));
    if (lasto_status e = smooth_nat(g, v); e != LASTO_OK) return e;
    if (lasto_status e = resid_norm2(g, rho, v, 0, S_TMP); e != LASTO_OK) return e;
    if (lasto_status e = smooth_nat(g, keep_plain); e != LASTO_OK) return e;
    if (lasto_status e = resid_norm2(g, rho, keep_plain, 0, S_RR); e != LASTO_OK) return e;
    if (lasto_status e = read_scalars(g, 0, kNumScalars); e != LASTO_OK) return e;
    const double r0 = std::sqrt(g->h_scalars[S_R0]);
    const double plain = r0 > 0.0 ? std::sqrt(g->h_scalars[S_RR]) / r0 : 0.0;
    const double learned = r0 > 0.0 ? std::sqrt(g->h_scalars[S_TMP]) / r0 : 0.0;
    const bool keep = y && std::isfinite(learned) && learned < plain;
    if (!keep) HIPCHK(hipMemcpyAsync(v, keep_plain, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (rel) {
        rel[0] = plain;
        rel[1] = learned;
    }
    if (accepted) *accepted = keep ? 1 : 0;
    return LASTO_OK;
}

// The learned guess on every right-hand side of the grid: per copy the
// net's correction of v (features of that copy's rho and v), then both
// candidates of every copy get one red-black sweep (all copies in one
// launch) and each copy keeps the one with the smaller residual relative to
// its face data alone. rel (host [2 n_batch] or NULL): plain, learned per
// copy; *accepted: copies that kept the learned candidate.
static lasto_status judge_batch(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel, int* accepted)
{
    if (lasto_status e = learned_scratch(g); e != LASTO_OK) return e;
    const int nb = g->n_batch;
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    hipStream_t s = g->stream;
    // the plain candidates are swept in a copy, the learned ones in v
    // itself, and a plain one goes back to v only where it wins
    double* keep_plain = g->lscr[LS_PLAIN];
    if (lasto_status e = batch_norms(g, rho, v, 1, S_BR0); e != LASTO_OK) return e;
    HIPCHK(hipMemcpyAsync(keep_plain, v, sizeof(double) * N * nb, hipMemcpyDeviceToDevice, s));
    if (lasto_status e = stage_rho_split(g, rho); e != LASTO_OK) return e;
    for (int b = 0; b < nb; ++b)
        if (lasto_status e = net_guess_apply(g, n, rho + b * N, v + b * N); e != LASTO_OK) return e;
    if (lasto_status e = smooth_nat(g, v); e != LASTO_OK) return e;
    if (lasto_status e = batch_norms(g, rho, v, 0, S_BRR); e != LASTO_OK) return e;
    if (lasto_status e = smooth_nat(g, keep_plain); e != LASTO_OK) return e;
    if (lasto_status e = batch_norms(g, rho, keep_plain, 0, S_BJ); e != LASTO_OK) return e;
    if (lasto_status e = read_scalars(g, 0, kNumScalars); e != LASTO_OK) return e;
    int acc = 0;
    for (int b = 0; b < nb; ++b) {
        const double r0 = std::sqrt(g->h_scalars[S_BR0 + b]);
        const double plain = r0 > 0.0 ? std::sqrt(g->h_scalars[S_BJ + b]) / r0 : 0.0;
        const double learned = r0 > 0.0 ? std::sqrt(g->h_scalars[S_BRR + b]) / r0 : 0.0;
        if (rel) {
            rel[2 * b] = plain;
            rel[2 * b + 1] = learned;
        }
        if (std::isfinite(learned) && learned < plain) ++acc;
        else HIPCHK(hipMemcpyAsync(v + b * N, keep_plain + b * N, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (accepted) *accepted = acc;
    return LASTO_OK;
}

// The first level a cycle in precision T does not treat level by level (an
// exact coarsest solve or a one-workgroup tail), under coarse mode `mode`.
static int first_special_level(lasto_grid g, int mode, bool fp32)
{
    int lev = g->tail_top;
    if (fp32 && g->tail32_top >= 0) lev = std::min(lev, g->tail32_top);
    if (mode != 1 && g->cfdm_level >= 0) lev = std::min(lev, g->cfdm_level);
    if (mode == 0 && g->cg) lev = std::min(lev, g->cg_level);
    return lev;
}

static lasto_status coarse_net_check(lasto_grid g, const lasto_solve_opts& o)
{
    const int c = o.coarse_net_level;
    if (g->n_batch != 1) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: coarse_net needs one right-hand side");
    if (c < 1 || c >= g->nlev) return fail(LASTO_ERR_ARG, "lasto_poisson_solve: coarse_net_level out of range");
    if (c >= first_special_level(g, o.coarse, false) || (o.precision == 1 && c >= first_special_level(g, o.coarse, true)))
        return fail(LASTO_ERR_ARG, "lasto_poisson_solve: coarse_net_level must lie above the cycle's exact coarsest "
                                   "solve (choose a coarser exact solve with coarse = 2 or 1)");
    const LevelView& V = g->lev[c].view;
    int cap[3];
    if (lasto_status e = net_capacity(o.coarse_net, cap); e != LASTO_OK) return e;
    if (V.nx < 8 || V.ny < 8 || V.nz < 8 || V.nx > cap[0] || V.ny > cap[1] || V.nz > cap[2])
        return fail(LASTO_ERR_ARG, "lasto_poisson_solve: coarse_net_level's grid does not fit the net");
    return LASTO_OK;
}

// `cycles` FP64 V(2,2)-cycles of level c on A_c u = f, the first from zero
// (the exact LDS solve below when the level allows it, else the tail)
lasto_status lasto::coarse_cycles(lasto_grid g, int c, int cycles, const double* f, double* u)
{
    const int mode = g->coarse_mode, nuc = g->nu_coarse;
    lasto_net lc = g->lc_net;
    g->coarse_mode = (g->cfdm_level > c) ? 2 : 1;
    g->lc_net = nullptr;
    g->nu_coarse = 0;
    lasto_status st = LASTO_OK;
    for (int k = 0; k < cycles && st == LASTO_OK; ++k)
        st = vcycle_level<double>(g, c, 2, 2, f, u, nullptr, nullptr, k == 0);
    g->coarse_mode = mode;
    g->nu_coarse = nuc;
    g->lc_net = lc;
    return st;
}

extern "C" lasto_status lasto_learned_guess(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel,
                                            int* accepted)
{
    if (!g || !n || !rho || !v) return fail(LASTO_ERR_ARG, "lasto_learned_guess: NULL argument");
    return judge_batch(g, n, rho, v, rel, accepted);
}

// The residual r = 4 pi rho - A v in natural layout (LS_R, faces zero) and
// its RMS over the interior, s = ||r||_W / sqrt(sum vol); the correction
// net's potential channel reads the zero array LS_ZERO.
static lasto_status correction_input(lasto_grid g, const double* rho, const double* v, double* s_r)
{
    const LevelView& V = g->lev[0].view;
    hipStream_t s = g->stream;
    HIPCHK(launch_residual_nat(V, v, rho, 4.0 * kPi, g->r, g->partials, 0, s));
    if (lasto_status e = reduce_to(g, interior_blocks(V), S_TMP); e != LASTO_OK) return e;
    HIPCHK(launch_split_to_nat(V, g->r, g->lscr[LS_R], s));
    if (lasto_status e = read_scalars(g, S_TMP, 1); e != LASTO_OK) return e;
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) {
        const std::vector<double>& x = g->lev[0].hx[d];
        vol *= x[x.size() - 2] - x[1] + 0.5 * (x[1] - x[0]) + 0.5 * (x[x.size() - 1] - x[x.size() - 2]);
    }
    *s_r = std::sqrt(g->h_scalars[S_TMP] / vol);
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_correction_features(lasto_grid g, lasto_net n, const double* rho, const double* v,
                                                      uint16_t* x, double* r_scale)
{
    if (!g || !n || !rho || !v || !x || !r_scale)
        return fail(LASTO_ERR_ARG, "lasto_net_correction_features: NULL argument");
    if (g->n_batch != 1) return fail(LASTO_ERR_ARG, "lasto_net_correction_features: one right-hand side per grid");
    if (lasto_status e = learned_scratch(g); e != LASTO_OK) return e;
    double sr = 0.0;
    if (lasto_status e = correction_input(g, rho, v, &sr); e != LASTO_OK) return e;
    if (!(sr > 0.0) || !std::isfinite(sr)) return fail(LASTO_ERR_ARG, "lasto_net_correction_features: zero residual");
    if (lasto_status e = net_features_async(g, n, g->lscr[LS_R], g->lscr[LS_ZERO], x, 1.0 / sr); e != LASTO_OK)
        return e;
    HIPCHK(hipStreamSynchronize(g->stream));
    *r_scale = sr;
    return LASTO_OK;
}

extern "C" lasto_status lasto_learned_correction(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel,
                                                 int* accepted)
{
    if (!g || !n || !rho || !v) return fail(LASTO_ERR_ARG, "lasto_learned_correction: NULL argument");
    if (g->n_batch != 1) return fail(LASTO_ERR_ARG, "lasto_learned_correction: one right-hand side per grid");
    if (lasto_status e = learned_scratch(g); e != LASTO_OK) return e;
    double sr = 0.0;
    if (lasto_status e = correction_input(g, rho, v, &sr); e != LASTO_OK) return e;
    const float* y = nullptr;
    double out_scale = 0.0;
    if (sr > 0.0 && std::isfinite(sr)) {
        if (lasto_status e = net_guess_forward(g, n, g->lscr[LS_R], g->lscr[LS_ZERO], &y, &out_scale, 1.0 / sr);
            e != LASTO_OK)
            return e;
    }
    return judge(g, rho, v, y, out_scale * sr, rel, accepted);
}

extern "C" lasto_status lasto_apply(lasto_grid g, const double* u, double* Au)
{
    if (!g || !u || !Au || u == Au) return fail(LASTO_ERR_ARG, "lasto_apply: NULL or aliased buffers");
    HIPCHK(launch_apply_nat(g->lev[0].view, u, Au, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

// nsw half-sweeps at level l on split arrays, fused or one launch each
template <typename T>
static lasto_status smooth_split(lasto_grid g, int l, const T* uin, const T* f, T* u, int c0, int nsw, int zero_in,
                                 int fused, double* dotp, int* ndot)
{
    const LevelView& V = g->lev[l].view;
    hipStream_t s = g->stream;
    if (fused) {
        HIPCHK(launch_gs_block<T>(V, uin, f, u, c0, nsw, zero_in, T(1), dotp, s, ndot, l == 0));
        return LASTO_OK;
    }
    HIPCHK(hipMemcpyAsync(u, uin, sizeof(T) * split_elems(V), hipMemcpyDeviceToDevice, s));
    int off = 0;
    for (int h = 0; h < nsw; ++h) {
        const bool d = dotp && h >= nsw - 2;
        int nb = 0;
        HIPCHK(launch_half<T>(V, u, f, (c0 + h) & 1, h == 0 && zero_in, T(1), d ? dotp + off : nullptr, s, &nb,
                              l == 0));
        if (d) off += nb;
    }
    if (ndot) *ndot = off;
    return LASTO_OK;
}

extern "C" lasto_status lasto_smooth(lasto_grid g, int level, int precision, const double* f, double* u, int nsweeps,
                                     int first_colour, int zero_in, int fused, double* dot)
{
    if (!g || !f || !u || f == u) return fail(LASTO_ERR_ARG, "lasto_smooth: NULL or aliased buffers");
    if (level < 0 || level >= g->nlev || precision < 0 || precision > 1 ||
        !(nsweeps == 2 || nsweeps == 4 || nsweeps == 6) || (first_colour != 0 && first_colour != 1) ||
        zero_in < 0 || zero_in > 1 || fused < 0 || fused > 1 || (dot && zero_in) ||
        (fused && precision == 0 && nsweeps > gs_block_max<double>()))
        return fail(LASTO_ERR_ARG, "lasto_smooth: bad level/precision/nsweeps/colour/zero_in/fused/dot");
    Level& L = g->lev[level];
    const LevelView& V = L.view;
    hipStream_t s = g->stream;
    const size_t n = split_elems(V);
    // the level's own work arrays serve as scratch (level 0: the Krylov vectors)
    double* U = level ? L.u64 : g->z;
    double* F = level ? L.f64 : g->q;
    double* I = L.r64;
    HIPCHK(launch_nat_to_split(V, u, I, s));
    HIPCHK(launch_nat_to_split(V, f, F, s));
    int nd = 0;
    double* dp = dot ? g->partials : nullptr;
    if (precision == 0) {
        if (lasto_status e = smooth_split<double>(g, level, I, F, U, first_colour, nsweeps, zero_in, fused, dp, &nd);
            e != LASTO_OK)
            return e;
    } else {
        float* U32 = level ? L.u32 : g->z32;
        float* F32 = level ? L.f32 : g->q32;
        float* I32 = L.r32;
        HIPCHK(launch_cast(I, I32, n, s));
        HIPCHK(launch_cast(F, F32, n, s));
        if (lasto_status e = smooth_split<float>(g, level, I32, F32, U32, first_colour, nsweeps, zero_in, fused, dp,
                                                 &nd);
            e != LASTO_OK)
            return e;
        HIPCHK(launch_cast(U32, U, n, s));
        HIPCHK(launch_fill_zero<float>(U32, n, s));
        HIPCHK(launch_fill_zero<float>(F32, n, s));
        HIPCHK(launch_fill_zero<float>(I32, n, s));
    }
    HIPCHK(launch_split_to_nat(V, U, u, s));
    if (dot) {
        HIPCHK(launch_reduce(g->partials, 1, nd, g->scalars + S_TMP, s));
        if (lasto_status e = read_scalars(g, S_TMP, 1); e != LASTO_OK) return e;
        *dot = g->h_scalars[S_TMP];
    }
    // the solver's arrays must come back with zero faces and padding
    HIPCHK(launch_fill_zero<double>(U, n, s));
    HIPCHK(launch_fill_zero<double>(F, n, s));
    HIPCHK(launch_fill_zero<double>(I, n, s));
    HIPCHK(hipStreamSynchronize(s));
    return LASTO_OK;
}

extern "C" lasto_status lasto_rb_sweep(lasto_grid g, const double* u_in, const double* rho, double* u_out,
                                       int first_colour)
{
    if (!g || !u_in || !rho || !u_out || u_in == u_out || (first_colour != 0 && first_colour != 1))
        return fail(LASTO_ERR_ARG, "lasto_rb_sweep: NULL/aliased buffers or bad colour");
    const LevelView& V = g->lev[0].view;
    hipStream_t s = g->stream;
    // the sweep runs in the solver's split layout on grid scratch
    HIPCHK(launch_nat_to_split(V, u_in, g->z, s));
    HIPCHK(launch_nat_to_split(V, rho, g->q, s));
    HIPCHK(launch_half_keep_faces<double>(V, g->z, g->q, first_colour, 4.0 * kPi, s));
    HIPCHK(launch_half_keep_faces<double>(V, g->z, g->q, 1 - first_colour, 4.0 * kPi, s));
    HIPCHK(launch_split_to_nat(V, g->z, u_out, s));
    // the solver's vectors must come back with zero faces and padding
    HIPCHK(launch_fill_zero<double>(g->z, split_elems(V), s));
    HIPCHK(launch_fill_zero<double>(g->q, split_elems(V), s));
    HIPCHK(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}
