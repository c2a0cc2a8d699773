/*
 * lasto.h -- C ABI of the MI355X (gfx950) Hartree step of the LASTO method.
 *
 * Paper: Kang, Davenport, Glimm, Keyes, McGuigan, "Linear Augmented
 * Slater-Type Orbital Method for Free Standing Clusters".
 *
 * The Hartree step (the paper's "computation of the potential", Section 3):
 *   1. a smoothed monopole pseudo-density with the charge of the true sphere
 *      density, plus the non-spherical terms put directly on the grid
 *      (Section 1; eq. (3.2) and the three constraints under it);
 *   2. a finite-difference multigrid solution of the Poisson problem
 *      Laplacian(V_C) = 4 pi rho~ (eq. (3.2)) on a graded tensor-product mesh
 *      (Section 3: finite adaptive domain, Dirichlet data at its edge; the
 *      edge data is the multipole field of the source, or zero as in
 *      eq. (3.3));
 *   3. interpolation of V_C onto the atom-sphere boundaries as Dirichlet
 *      data for the interior problem (Section 1; eq. (3.5)-(3.6)).
 *
 * Conventions shared by every call:
 *   - Every call returns a lasto_status; no C++ exception crosses the ABI.
 *     On failure lasto_last_error() returns a thread-local message.
 *   - Grid arrays are dense FP64 [nz][ny][nx], x fastest, boundary nodes
 *     included, in device memory owned by the caller (for example a torch
 *     tensor's data_ptr()). The library never frees caller memory.
 *   - Lengths in bohr, charges in e, potentials in hartree; the equation is
 *     solved with the sign of eq. (3.2): Laplacian(V) = +4 pi rho, so a
 *     positive charge q gives V -> -q/r.
 *   - All device work is enqueued on the grid's HIP stream, ordered after the
 *     caller's earlier work on that stream. lasto_poisson_solve and
 *     lasto_sphere_interp return only after their work has completed.
 *   - A grid owns its multigrid hierarchy and scratch; it is not thread-safe
 *     (use one grid per host thread).
 */
#ifndef LASTO_H
#define LASTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lasto_grid_s* lasto_grid;
/* a learned-form network (see lasto_net_create) */
typedef struct lasto_net_s* lasto_net;

typedef enum {
    LASTO_OK = 0,
    LASTO_ERR_ARG = 1,            /* invalid argument (sizes, NaN, ordering, NULL) */
    LASTO_ERR_ALLOC = 2,          /* device or host allocation failed */
    LASTO_ERR_HIP = 3,            /* a HIP runtime call or kernel launch failed */
    LASTO_ERR_NOT_CONVERGED = 4,  /* tolerance not met within max_iters; v and info hold the last iterate */
    LASTO_ERR_DIVERGED = 5,       /* residual became NaN/Inf or grew; v holds the last finite iterate */
    LASTO_ERR_STATE = 6           /* call not valid in the current state */
} lasto_status;

/* Text of a status code (static storage). */
const char* lasto_status_string(lasto_status s);
/* Detail of the last failure on this host thread ("" if none). */
const char* lasto_last_error(void);

/*
 * Graded 1-D node coordinates (host only, no device work).
 *
 * Section 3 asks for a finite domain with fine meshes near the atoms and
 * coarse meshes far from them, without fixing a rule. The rule used here:
 * spacing h(x) = min(hmax, hmin + (g - 1) d(x)), d(x) the distance to the
 * nearest entry of `planes` (atom coordinates on this axis); the node map
 * xi(x) = int_lo^x dt/h(t) is integrated in closed form, g in (1, gmax] is
 * found by bisection so that xi(hi) = n - 1 (g = 1 when even hmin leaves
 * nodes to spare), and node i is placed at xi^-1(i xi(hi)/(n-1)); x[0] = lo
 * and x[n-1] = hi exactly. With n_planes = 0 the nodes are uniform.
 * If no g <= gmax fits and hmin_step > 0, hmin is raised by hmin_step until
 * one does (hmin_used reports it).
 *   x_out [n] host, caller-owned. g_out, hmin_used may be NULL.
 * Errors: LASTO_ERR_ARG for n < 3, hi <= lo, hmin <= 0, hmax < hmin,
 * gmax <= 1, or an infeasible request.
 */
lasto_status lasto_mesh_graded_1d(double lo, double hi, int n, const double* planes, int n_planes,
                                  double hmin, double hmax, double gmax, double hmin_step,
                                  double* x_out, double* g_out, double* hmin_used);

/*
 * Create a grid on the tensor-product mesh x[nx] * y[ny] * z[nz] (host
 * arrays, strictly increasing, each n >= 4), build the multigrid hierarchy
 * and allocate its device scratch on the current HIP device.
 *   hip_stream: a hipStream_t (NULL = the default stream) on which all of
 *   this grid's work runs.
 *   n_batch: right-hand sides the grid carries, 1..16. A batched grid holds
 *     n_batch independent problems on the same mesh: every device array of
 *     the calls below is then [n_batch][nz][ny][nx] (copies back to back),
 *     every kernel launch of a solve covers all copies at once (they are
 *     stacked along z, each copy's first and last planes being its own
 *     faces), and host outputs gain a leading n_batch dimension.
 * The hierarchy: per axis, a pair of cells merges (its middle node is
 * dropped) when its merged width is at most 4 times the level's smallest
 * spacing; when no axis can merge, every pair merges. Coarsening stops when
 * every axis has at most 5 nodes.
 * Errors: LASTO_ERR_ARG (sizes, ordering, NaN), LASTO_ERR_ALLOC, LASTO_ERR_HIP.
 */
lasto_status lasto_grid_create(const double* x, int nx, const double* y, int ny, const double* z, int nz,
                               int n_batch, void* hip_stream, lasto_grid* out);
lasto_status lasto_grid_destroy(lasto_grid g);
/* Number of levels and the node counts of level l (out[3] = nx, ny, nz). */
lasto_status lasto_grid_levels(lasto_grid g, int* n_levels);
lasto_status lasto_grid_level_shape(lasto_grid g, int level, int* out3);
/* The finest-level index of each node of level l per axis (every coarse node
 * is a fine node): ix [nx_l], iy [ny_l], iz [nz_l], host. */
lasto_status lasto_grid_level_nodes(lasto_grid g, int level, int* ix, int* iy, int* iz);

/*
 * One atom of the pseudo-density (host struct, passed by pointer).
 * kind 0: monopole q s (pi w^2)^(-3/2) exp(-r^2/w^2) for r < 7 w, with s
 *         making the discrete charge sum_n vol_n rho_n exactly q when
 *         renormalize != 0 (s = 1 otherwise); vol_n is the product of the
 *         nodes' dual widths.
 * kind 1: the paper's pseudo-density (eq. (3.2) and its constraints): inside
 *         R the even quartic a + b r^2 + c r^4 with 4 pi int_0^R rho~ r^2 dr = q,
 *         rho~(R) = rho_R and rho~'(R) = drho_R; zero outside R.
 * Both kinds add the non-spherical terms directly on the grid:
 *         sum_{l=1..lmax} sum_m clm[l*l+l+m-1] r^l y_lm exp(-alpha r^2) for
 *         alpha r^2 < 42.25, y_lm the real orthonormal harmonics of eq. (3.1)
 *         without the Condon-Shortley phase (lmax <= 4, the paper's L <= 4).
 */
typedef struct {
    double center[3];
    double radius;     /* sphere radius R (kind 1 support; interpolation radius) */
    double q;          /* charge of the monopole part */
    int kind;          /* 0 Gaussian, 1 quartic */
    int lmax;          /* 0..4 */
    double width;      /* kind 0: w */
    double rho_R;      /* kind 1: spherical density at R */
    double drho_R;     /* kind 1: its radial derivative at R */
    double alpha;      /* radial factor of the l >= 1 terms */
    double clm[24];    /* (l,m) = (1,-1),(1,0),(1,1),(2,-2),...,(4,4); unused entries ignored */
} lasto_atom;

/*
 * Pseudo-density on every grid node (Section 1 and eq. (3.2)).
 *   atoms: host array [n_atoms].
 *   rho_interstitial: device [nz][ny][nx] added at nodes outside every
 *     sphere (|x - C_a| >= R_a), or NULL.
 *   rho_out: device [nz][ny][nx], overwritten.
 *   Batched grids: atoms holds n_batch tables of n_atoms back to back (copy
 *   b uses atoms[b * n_atoms ...]); moments_out is [n_batch][25].
 *   moments_out: host [25] (l <= 4 moments about the box centre, see
 *     lasto_poisson_solve) or NULL.
 * Errors: LASTO_ERR_ARG (lmax > 4, kind not 0/1, width <= 0, NaN), LASTO_ERR_HIP.
 */
lasto_status lasto_pseudo_density(lasto_grid g, int n_atoms, const lasto_atom* atoms,
                                  const double* rho_interstitial, int renormalize,
                                  double* rho_out, double* moments_out);

typedef struct {
    double rtol;        /* stop when ||b - A v||_W <= rtol ||b - A v_bc||_W (default 1e-10) */
    int max_iters;      /* outer iterations (PCG steps or V-cycles), default 100 */
    int nu1, nu2;       /* pre/post red-black sweeps per level (default 2, 2) */
    int method;         /* 0 MG-preconditioned CG (default), 1 plain V-cycle iteration; with
                           precision 1 it selects the inner FP32 solver the same way */
    int precision;      /* 0 FP64 throughout (default); 1 FP32 V-cycles inside FP64 refinement */
    int inner_iters;    /* precision 1: FP32 PCG steps or V-cycles per FP64 refinement (default 6) */
    int guess;          /* interior start: 0 v as given (default), 1 zero, 2 the analytic superposition of
                           the atoms' monopole fields (lasto_analytic_guess), 3 that plus the learned
                           correction of guess_net, judged as lasto_learned_guess (the analytic start is
                           kept when the learned one is no better: info->fallback_used bit 0) */
    int bc;             /* 0 zero faces (eq. (3.3)), 1 multipole faces (default), 2 faces of v as given */
    int lmax_bc;        /* multipole order of the face values, 0..4 (default 4) */
    int debug_nan_iter; /* >= 0: inject a NaN into the residual at that iteration (tests only); default -1 */
    int profile;        /* 1: time every finest-level smoother launch with HIP events (default 0) */
    int inner_first;    /* precision 1: inner steps of the first refinement, 0 = inner_iters (default 0);
                           its reduction is bounded by FP32 rounding of the operator sooner than later ones */
    int coarse;         /* coarsest solve of the cycle, exact by fast diagonalisation of the level's
                           tensor-product operator: 0 (default) on the first level below the finest with
                           at most 3e6 nodes per right-hand side if that level has more than 16384 nodes
                           (by GEMMs), else as 2; 2 on the first level with at most 16384 nodes (each axis
                           at most 34 nodes, the level below the finest, its block in one workgroup's LDS),
                           else as 1; 1 red-black sweeps on every level down to the coarsest */
    int fallback;       /* precision 1: 1 (default) when the FP32 inner solve breaks down (a non-finite
                           correction, which is never added to v), the residual keeps growing, or max_iters
                           pass, the solve restarts as FP64 MG-PCG from the current iterate with max_iters
                           more iterations (info->fallback_used bit 1); 0 returns the failure */
    int n_atoms;        /* guess 2, 3: atoms per right-hand side in `atoms` */
    const lasto_atom* atoms;   /* guess 2, 3: host atom tables as for lasto_pseudo_density */
    lasto_net guess_net;       /* guess 3: the learned-guess net (its grid: one copy of the finest level) */
    lasto_net coarse_net;      /* learned coarse correction (NULL: none): a net trained to map a coarse
                                  level's restricted residual to its correction; see lasto_poisson_solve */
    int coarse_net_level;      /* the level it acts on (>= 1, above the exact coarsest solve) */
    double inner_rate;  /* precision 1: 0 (default) fixed inner step counts (inner_first, inner_iters); in
                           (0, 1) adaptive: each refinement takes just enough steps to reach 0.7 rtol from
                           the current relative residual rel at a per-step reduction q,
                           ceil(log(0.7 rtol / rel) / log(q)), at least 1 and at most inner_first (first
                           refinement, when set) or inner_iters. q starts at inner_rate; after a refinement
                           of two or more PCG steps it becomes that refinement's own per-step decrease of
                           sqrt(<r, z>_W); after a later refinement that reduced the true residual by less
                           than 1e-5 it rises to that reduction per step when slower */
    int graphs;         /* 1: the inner FP32 PCG's steps (their V-cycle, reductions and updates) and the FP64
                           CG's finest-level V-cycle are captured into HIP graphs at their second use on a
                           grid (keyed by what they launch; on a stream of the library's own) and replayed
                           after, one host call in place of each sequence's launches; same kernels in the same
                           order, so the same bits. 0 (default): every launch from the host, which measured as
                           fast or faster at 257^3 and 513^3 (the GPU, not the host, bounds these solves).
                           profile = 1 and a learned coarse correction always launch from the host */
    int nu_coarse;      /* > 0: red-black sweeps before and after the coarse correction on every level below
                           the finest (the finest keeps nu1, nu2); 0 (default): nu1, nu2 on every level */
    int fused_sweeps;   /* red-black half-sweeps that share one pass over a level (lasto_smooth): 0 (default) or
                           1 one launch per half-sweep; 2, 4 or 6 (FP64: at most 4) at most that many per pass on
                           every level that sweeps: the pre-smoothing from zero and the start of the
                           post-smoothing. The results are the same bits either way, apart from the order in
                           which <r, z>_W sums its terms; the fused pass measured slower at 257^3 (its time is
                           bound by latency per plane step, not by HBM) */
} lasto_solve_opts;

typedef struct {
    int iters;              /* outer iterations run */
    int vcycles;            /* V-cycles run (all precisions) */
    int refinements;        /* FP64 refinement steps (precision 1) */
    double rel_resid;       /* true ||b - A v||_W / ||b - A v_bc||_W at exit */
    double resid_hist[128]; /* relative residual after each outer iteration */
    double moments[25];     /* Q_lm used for the face values (bc = 1) */
    double ms_total;        /* wall time of the call, ms */
    /* profile = 1: finest-level red-black sweeps (the dominant kernel) */
    int smooth_launches;    /* sweeps timed */
    double smooth_ms;       /* summed event-timed duration of those sweeps, ms */
    double smooth_bytes;    /* their algorithmic HBM bytes: (read u, f + write u) per interior node */
    int smooth_fp32;        /* launches among them that ran in FP32 */
    int n_batch;            /* right-hand sides solved (the grid's n_batch) */
    double batch_rel_resid[16]; /* rel_resid of each right-hand side (rel_resid is their maximum) */
    int coarse_level;       /* level the cycle solved exactly by fast diagonalisation, -1 if none */
    int fallback_used;      /* bit 0: guess 3 kept the analytic start; bit 1: FP64 finished a failed mixed solve */
    int guess_accepted;     /* guess 3: right-hand sides whose learned start was kept */
    int coarse_applied;     /* learned coarse corrections proposed (one per visit of coarse_net_level) */
    int coarse_accepted;    /* ... and accepted by the coarse residual test */
    double ms_bc;           /* moments and face values (HIP events on the grid's stream), ms */
    double ms_guess;        /* the initial guess (analytic superposition, net and judge), ms */
    double ms_cycles;       /* the iteration to the exit residual, ms */
    double alg_bytes;       /* algorithmic HBM bytes of the iteration's finest-level launches (each launch's
                               compulsory reads and writes of whole arrays) */
    double inner_rate;      /* precision 1 with opts->inner_rate > 0: the per-step reduction q the last
                               refinement was planned with */
    double rel_start;       /* relative residual of the start (after the guess), as rel_resid */
} lasto_solve_info;

void lasto_solve_opts_default(lasto_solve_opts* o);

/*
 * Solve eq. (3.2), Laplacian(V_C) = 4 pi rho, on the grid by finite
 * differences and multigrid (Section 3).
 *   rho: device [nz][ny][nx] source.
 *   v: device [nz][ny][nx], in: initial guess (interior) and, for bc = 2,
 *      the face values; out: the iterate, faces holding the Dirichlet data.
 * Discretisation: at interior node n, sum over axes of
 *   [(v_{n+e} - v_n)/h_+ - (v_n - v_{n-e})/h_-] / m = 4 pi rho_n,
 * h_-/h_+ the adjacent spacings and m = (h_- + h_+)/2.
 * Face values for bc = 1: V(x) = -sum_{l<=lmax_bc, m} 4 pi/(2l+1) Q_lm
 * r^l y_lm(x') / |x'|^(2l+1), x' = x - c, Q_lm = sum_n vol_n rho_n
 * r_n^l y_lm(x_n - c), c the box centre.
 * W-norm: ||r||_W^2 = sum over interior nodes of vol_n r_n^2.
 * Batched grids solve all copies together (one norm and one set of CG
 * coefficients for the stacked system, i.e. CG on the block-diagonal
 * operator) until every copy meets rtol against its own reference norm
 * (info->batch_rel_resid); each copy's faces come from its own moments.
 * Learned coarse correction (opts->coarse_net, one right-hand side): each
 * time a cycle reaches level c = coarse_net_level, the net reads that level's
 * restricted residual f_c at unit RMS s (s = ||f_c||_W / sqrt(sum of the
 * interior dual volumes)) with the level's spacings, and proposes
 * e^ = s out_scale net(f_c / s) for A_c e = f_c; e^ starts the level's cycle
 * if ||f_c - A_c e^||_W < ||f_c||_W, otherwise it starts from zero as without
 * the net (the test runs on the device; info->coarse_applied / _accepted
 * count the proposals). The preconditioner then varies from step to step, so
 * the CG forms take the flexible (Polak-Ribiere) beta. Level c must lie above
 * the cycle's exact coarsest solve or one-workgroup tail (coarse = 2 or 1
 * make room) and fit the net's creation size.
 * Returns LASTO_OK, or LASTO_ERR_NOT_CONVERGED / LASTO_ERR_DIVERGED with v
 * and info filled, or LASTO_ERR_ARG / LASTO_ERR_HIP.
 */
lasto_status lasto_poisson_solve(lasto_grid g, const double* rho, double* v,
                                 const lasto_solve_opts* opts, lasto_solve_info* info);

/*
 * V_C on the sphere boundaries (Section 1; eq. (3.5)-(3.6)): the value at
 * C_a + R_a d_k for every atom a and direction d_k, by tricubic Lagrange
 * interpolation of the grid values (per axis the 4-node window starts at
 * clamp(upper_bound(x, p) - 2, 0, n - 4)).
 *   v: device grid values. centers: host [n_atoms][3]. radii: host [n_atoms].
 *   dirs: host [n_dir][3] unit vectors, or NULL for the default 64 (8
 *     Gauss-Legendre nodes in cos(theta) times 8 azimuths 2 pi (b + 1/2)/8,
 *     theta-major; n_dir must then be 64).
 *   out: host [n_atoms][n_dir] ([n_batch][n_atoms][n_dir] for a batch; the
 *     points are the same for every copy).
 * Errors: LASTO_ERR_ARG (a point outside the box, n_dir mismatch), LASTO_ERR_HIP.
 */
lasto_status lasto_sphere_interp(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                 const double* radii, int n_dir, const double* dirs, double* out);

/*
 * lasto_sphere_interp for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same values, bit for bit, with no hipMalloc or hipFree. Its
 * staging (the points, the device values, and copies of the directions,
 * centres and radii) lives in a static device array of the library, sized for
 * LASTO_NOALLOC_MAX_POINTS points (11 doubles per point, 2.75 MiB), which each
 * GPU the library runs on holds until the process ends; its device address is
 * looked up once per device, on the first call there.
 *   Arguments, layout and ownership as lasto_sphere_interp.
 *   n_atoms * n_dir > LASTO_NOALLOC_MAX_POINTS -> LASTO_ERR_ARG (nothing runs).
 * Every call on one GPU shares that array: calls that overlap on one GPU (from
 * two host threads, or on two streams) race; serialise them. Each call writes
 * every part of the array it reads, so no clearing is needed between calls.
 * Errors: as lasto_sphere_interp.
 */
#define LASTO_NOALLOC_MAX_POINTS 32768
lasto_status lasto_sphere_interp_noalloc(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                         const double* radii, int n_dir, const double* dirs, double* out);

/* ------------------------------------------------------------------------
 * Inside the muffin-tin spheres (Section 3, eq. (3.4)-(3.7)) and the energy
 * integral of Section 4. The grid solution gives V_C on each sphere boundary;
 * its projection onto the real orthonormal harmonics y_LM (L <= 4, index
 * L*L + L + M, no Condon-Shortley phase) is the Dirichlet datum of the radial
 * equation (3.4) inside, whose solution with the sphere's own density
 * rho_LM(r) and nuclear charge Z is
 *   V_LM(r) = V_LM(R) (r/R)^L
 *           - 4 pi/(2L+1) [ r^-(L+1) P(r) + r^L Q(r) - r^L P(R)/R^(2L+1) ]
 *           + (L = 0) sqrt(4 pi) Z (1/r - 1/R),
 *   P(r) = int_0^r rho_LM r'^(L+2) dr',  Q(r) = int_r^R rho_LM r'^(1-L) dr'
 * (the printed integrands read as rho r'^(L+2) and rho r'^(1-L); the sign is
 * that of eq. (3.2) as written, Laplacian V = +4 pi (rho - Z delta), the
 * printed formula having the opposite overall sign).
 *
 * Radial mesh (Section 4: logarithmic, 429 points in the paper): atom a uses
 *   r_k = R_a exp((k - (n_rad - 1)) D_a), D_a = ln(R_a / r_min) / (n_rad - 1),
 * k = 0..n_rad-1, so r_0 = r_min and r_(n_rad-1) = R_a. Radial integrals are
 * taken in t = ln r interval by interval, each as the integral of the cubic
 * through four consecutive samples (fourth order); the piece [0, r_0] as
 * rho(r_0) r_0^(L+3)/(2L+3) (rho_LM ~ r^L there) and, for the energy,
 * V(r_0) rho(r_0) r_0^3 / 3.
 *
 * Angular rule of eq. (3.6): n_theta Gauss-Legendre nodes t_a in cos(theta)
 * (ascending) times n_phi azimuths 2 pi (b + 1/2)/n_phi, point p = a n_phi + b,
 * direction (sin cos, sin sin, cos), weight w_a 2 pi / n_phi. With
 * n_theta >= 5 and n_phi >= 9 it integrates every product y_LM y_L'M' with
 * L, L' <= 4 exactly.
 *
 * Batches: arrays of a batched grid carry a leading [n_batch] dimension; the
 * geometry is the same for every copy.
 */
typedef struct lasto_spheres_s* lasto_spheres;

/*
 * A set of non-overlapping spheres on grid g: device tables of the atoms,
 * the angular rule and the reduction scratch (owned by the set; destroy it
 * before its grid).
 *   centers: host [n_atoms][3]; radii, Z: host [n_atoms] (Z may be NULL: 0).
 *   Each sphere lies inside the box; |C_a - C_b| >= R_a + R_b.
 *   n_theta in 5..64, n_phi in 9..1024 (n_theta * n_phi <= 8192),
 *   n_rad in 8..1024, 0 < r_min < min R_a.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_ALLOC, LASTO_ERR_HIP.
 */
lasto_status lasto_spheres_create(lasto_grid g, int n_atoms, const double* centers, const double* radii,
                                  const double* Z, int n_theta, int n_phi, int n_rad, double r_min,
                                  lasto_spheres* out);
lasto_status lasto_spheres_destroy(lasto_spheres s);

/*
 * The non-spherical density put on the grid inside the spheres (Section 1
 * places the non-spherical terms of the sphere densities directly on the
 * grid; here from the radial tables the interior solve uses): at every node
 * inside sphere a (|x - C_a|^2 < R_a^2),
 *   rho += sum_(LM, L >= lmin) rho_LM(r) y_LM(x - C_a),
 * rho_LM(r) the cubic in t = ln r through the four mesh samples around t
 * (window start clamp(floor((t - t_0)/D) - 1, 0, n_rad - 4)); below r_0,
 * rho_LM(r_0) (r / r_0)^L. With kind-1 atoms of lmax 0 in
 * lasto_pseudo_density, lmin = 1 here and the interstitial density outside,
 * this is the paper-mode source.
 *   rho_lm: device [n_atoms][25][n_rad]; rho: device grid array, added to.
 * Enqueued on the grid's stream. Errors: LASTO_ERR_ARG, LASTO_ERR_HIP.
 */
lasto_status lasto_sphere_density_terms(lasto_spheres s, const double* rho_lm, int lmin, double* rho);

/*
 * eq. (3.6): vlm_R[a][LM] = sum_p w_p V(C_a + R_a d_p) y_LM(d_p), V(x) by
 * tricubic Lagrange interpolation of the grid values (as lasto_sphere_interp).
 *   v: device grid values [nz][ny][nx]. vlm_R: device [n_atoms][25].
 * Enqueued on the grid's stream; returns without waiting.
 * Errors: LASTO_ERR_ARG (NULL), LASTO_ERR_HIP.
 */
lasto_status lasto_sphere_project(lasto_spheres s, const double* v, double* vlm_R);

/*
 * Interior solution of eq. (3.4) (formula above) in every sphere.
 *   vlm_R: device [n_atoms][25] the Dirichlet data (lasto_sphere_project).
 *   rho_lm: device [n_atoms][25][n_rad] rho_LM(r_k) of the density inside
 *     sphere a on its mesh (the electron density; the nucleus enters by Z).
 *   v_lm: device [n_atoms][25][n_rad] out, V_LM(r_k); v_lm[.][.][n_rad-1] = vlm_R.
 * Enqueued on the grid's stream; returns without waiting.
 * Errors: LASTO_ERR_ARG (NULL, v_lm aliasing an input), LASTO_ERR_HIP.
 */
lasto_status lasto_sphere_radial(lasto_spheres s, const double* vlm_R, const double* rho_lm, double* v_lm);

/*
 * The integral of V against the density over the domain (Section 4: half of
 * it is the Hartree term of eq. (4.1) when V is the Hartree potential):
 *   e_out[0] = sum over grid nodes outside every sphere (|x_n - C_a|^2 >= R_a^2,
 *              squares and sums rounded as written) of vol_n v_n rho_n,
 *              vol_n the product of the dual widths;
 *   e_out[1] = sum over atoms and LM of int_0^R_a V_LM rho_LM r^2 dr on the
 *              radial mesh (orthonormal y_LM turn the angular integral into
 *              the sum over LM).
 *   v, rho: device grid arrays; v_lm, rho_lm: device [n_atoms][25][n_rad].
 *   e_out: host [2] ([n_batch][2] for a batch). Waits for the result.
 * Errors: LASTO_ERR_ARG (NULL), LASTO_ERR_HIP.
 */
lasto_status lasto_sphere_energy(lasto_spheres s, const double* v, const double* rho, const double* v_lm,
                                 const double* rho_lm, double* e_out);

/* ------------------------------------------------------------------------
 * The output density in the interstitial region (Section 3, the density
 * update after the eigenproblem H c = e S c): at the grid nodes outside every
 * sphere
 *   rho_out(x) = sum_k f_k psi_k(x)^2,  psi_k(x) = sum_mu c(mu, k) phi_mu(x),
 * over the basis of eq. (3.13), phi_(i n l m)(x) = r_i^(n-1) exp(-zeta r_i)
 * y_lm(r_i / |r_i|), r_i = x - C_i, the same shells on every atom; zero at
 * nodes inside a sphere (|x - C_i|^2 < R_i^2). The paper sums |psi_k|^2 over
 * the states below the Fermi level; f_k carries their occupations (2 for a
 * doubly occupied state). Computed on the FP64 matrix cores (the contraction
 * of nodes x basis with basis x states), then squared and summed.
 */
typedef struct {
    int n;          /* principal quantum number, l + 1 <= n <= 16 */
    int l;          /* 0..4; the shell holds 2l + 1 functions, m = -l..l */
    double zeta;    /* exponent > 0 */
} lasto_shell;

/*
 *   centers: host [n_atoms][3]; radii: host [n_atoms] (0: no sphere), or NULL.
 *   shells: host [n_shells], at most 64 functions per atom; basis function
 *     index mu = atom * (functions per atom) + (shell offset) + (m + l).
 *   coef: device [n_basis][n_occ] (a function's coefficients over the states
 *     contiguous). occ: host [n_occ].
 *   rho_out: device [nz][ny][nx], one copy of a batched grid per call.
 * Enqueued on the grid's stream; returns once the small tables are on the
 * device, without waiting for the result.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_ALLOC, LASTO_ERR_HIP.
 */
lasto_status lasto_interstitial_density(lasto_grid g, int n_atoms, const double* centers, const double* radii,
                                        int n_shells, const lasto_shell* shells, int n_occ, const double* coef,
                                        const double* occ, double* rho_out);

/*
 * The interstitial parts of the overlap and Hamiltonian matrices by grid
 * quadrature (Section 3, eq. (3.11)-(3.12) in the nodal form under
 * eq. (3.14), with the nodes of this grid and their dual volumes vol_P):
 *   S[mu][nu] = sum_P vol_P phi_mu(P) phi_nu(P),
 *   H[mu][nu] = 1/2 sum_P vol_P (phi_mu(P) tphi_nu(P) + tphi_mu(P) phi_nu(P)),
 * over the nodes P outside every sphere, tphi = (-1/2 Laplacian + V) phi with
 * the kinetic term in closed form, eq. (3.14):
 *   -1/2 Laplacian phi = 1/2 [(l(l+1) - n(n-1)) r^(n-3) + 2 zeta n r^(n-2)
 *                             - zeta^2 r^(n-1)] exp(-zeta r) y_lm.
 * Basis as for lasto_interstitial_density.
 *   v: device [nz][ny][nx] the potential V at the nodes (one copy).
 *   centers: host [n_atoms][3]; radii: host [n_atoms], every radius > 0 (the
 *     kinetic term is singular at a centre, which a sphere must cover).
 *   S, H: device [n_basis][n_basis] (both triangles written), n_basis <= 32768.
 * Computed on the FP64 matrix cores in 64 x 64 blocks (upper triangle) over
 * node chunks, the chunks summed in a fixed order. Allocates its scratch
 * (a node weight per node, the partial blocks) and waits for the result.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_ALLOC, LASTO_ERR_HIP.
 */
lasto_status lasto_matrix_elements(lasto_grid g, const double* v, int n_atoms, const double* centers,
                                   const double* radii, int n_shells, const lasto_shell* shells, double* S, double* H);

/*
 * A direct solve of the discrete eq. (3.2) by fast diagonalisation (Lynch,
 * Rice and Thomas, 1964), beside the multigrid of lasto_poisson_solve: the
 * 7-point operator on a tensor-product mesh is the Kronecker sum of three
 * 1-D operators A_d = M_d^-1 T_d, each diagonalised once per grid as
 * S_d L_d S_d^-1 (S_d = M_d^-1/2 Q_d from the symmetric tridiagonal
 * M_d^-1/2 T_d M_d^-1/2 = Q_d L_d Q_d^T), so that the interior solution is
 *   u = (S_z x S_y x S_x) [ (S_z^-1 x S_y^-1 x S_x^-1) b / (l_z + l_y + l_x) ],
 * b = 4 pi rho - A v_bc: six dense contractions along the axes on the FP64
 * matrix cores (rocBLAS GEMMs). Exact up to rounding; no iteration.
 *   rho, v: as lasto_poisson_solve (v's faces are set from bc/lmax_bc as
 *     there: 0 zero, 1 multipole, 2 the faces of v as given; its interior is
 *     overwritten; a batched grid solves every copy).
 *   info (may be NULL): iters = 1, rel_resid = max over copies of
 *     ||4 pi rho - A v||_W / ||4 pi rho - A v_bc||_W, batch_rel_resid, moments,
 *     ms_total.
 * The first call on a grid builds the 1-D decompositions on the host (O(n^3)
 * per axis) and allocates two work arrays of the interior's size, kept until
 * lasto_grid_destroy. Waits for the result.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_ALLOC, LASTO_ERR_HIP, LASTO_ERR_STATE (no
 * convergence of a 1-D decomposition), LASTO_ERR_DIVERGED (non-finite result).
 */
lasto_status lasto_fdm_solve(lasto_grid g, const double* rho, double* v, int bc, int lmax_bc,
                             lasto_solve_info* info);
/* The 1-D decomposition on its own (host only, no device work): for
 * coordinates x[0..n-1] (increasing, n >= 3) and the interior operator
 * (A u)_i = am_i (u_(i-1) - u_i) + ap_i (u_(i+1) - u_i), i = 1..n-2, fills
 * lam[n-2] and S, Sinv [n-2][n-2] (row-major) with A = S diag(lam) Sinv. */
lasto_status lasto_fdm_axis(const double* x, int n, double* lam, double* S, double* Sinv);

/*
 * The discrete operator of eq. (3.2) on the finest level: Au[n] = (A u)_n at
 * interior nodes (the three-point nonuniform second difference per axis, as
 * in lasto_poisson_solve); faces of Au are left untouched.
 *   u, Au: device [nz][ny][nx], distinct buffers.
 * Errors: LASTO_ERR_ARG (NULL or aliasing), LASTO_ERR_HIP.
 */
lasto_status lasto_apply(lasto_grid g, const double* u, double* Au);

/*
 * One red-black Gauss-Seidel sweep on A u = 4 pi rho at the finest level,
 * out of place: u_out = S(u_in). Nodes with (i+j+k) % 2 == first_colour are
 * updated first from u_in, the other colour then from those new values. On a
 * batched grid k counts planes of the stacked copies (copy b starts at plane
 * b nz), so with an odd nz the copies at odd b take the colours in the other
 * order (every solve form converges to the same solution either way).
 * Faces of u_out are left untouched (copy them from u_in when needed).
 * This is the smoother of the multigrid solve, exposed for testing.
 *   u_in, rho, u_out: device [nz][ny][nx]; u_out must not alias u_in.
 */
lasto_status lasto_rb_sweep(lasto_grid g, const double* u_in, const double* rho, double* u_out, int first_colour);

/*
 * Red-black Gauss-Seidel half-sweeps of the multigrid smoother (eq. (3.2)'s
 * seven-point operator; the smoother of the multigrid solve the paper names)
 * on the correction equation A u = f with zero faces at `level` of the grid:
 * nsweeps half-sweeps (2, 4 or 6; a fused FP64 pass at most 4, its u and f
 * rings filling a compute unit's LDS) updating colours first_colour,
 * 1 - first_colour, ... in turn, starting from u (zero_in 0) or from zero
 * (zero_in 1). fused 1 runs them as one pass over the level (a workgroup
 * marches a ring of planes through LDS and recomputes its halo), fused 0 as
 * one launch per half-sweep; both give the same bits. precision 1 runs in
 * FP32 (u and f rounded on entry, the result widened on exit). dot (host,
 * optional, not with zero_in): the sum over the nodes of the last two
 * half-sweeps of vol * f * u (the smoother's share of <f, u>_W). Exposed for
 * testing.
 *   f, u: device [nz][ny][nx] of the level (lasto_grid_level_shape), FP64,
 *   distinct; u in/out (interior nodes written, faces untouched). Faces of f
 *   and u must be zero.
 * Errors: LASTO_ERR_ARG (NULL or aliased buffers, bad level, precision,
 * nsweeps, colour, zero_in or fused, dot with zero_in), LASTO_ERR_HIP.
 */
lasto_status lasto_smooth(lasto_grid g, int level, int precision, const double* f, double* u, int nsweeps,
                          int first_colour, int zero_in, int fused, double* dot);

/*
 * Streaming ceiling (measurement, not part of the method): dst = a over
 * `bytes` (b NULL) or dst = a + b elementwise in FP64 (two reads and one
 * write, the red-black half-sweep's mix), 16-byte accesses, four per thread in
 * flight. Enqueued on hip_stream (NULL: the default stream); returns without
 * waiting. a, b, dst: device, bytes a multiple of 16.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_HIP.
 */
lasto_status lasto_stream_probe(const double* a, const double* b, double* dst, size_t bytes, void* hip_stream);

/*
 * Dirichlet data on the six faces of v, the boundary step of
 * lasto_poisson_solve on its own (eq. (3.3) for bc = 0; bc = 1 the multipole
 * field of the grid moments, as documented at lasto_poisson_solve).
 *   rho: device source (read for bc = 1). v: device, only faces written.
 *   moments_out: host [25] Q_lm (bc = 1) or NULL.
 * Errors: LASTO_ERR_ARG (bc not 0/1, lmax_bc outside 0..4), LASTO_ERR_HIP.
 */
lasto_status lasto_boundary_values(lasto_grid g, const double* rho, int bc, int lmax_bc, double* v,
                                   double* moments_out);

/*
 * Analytic initial guess: the interior of v becomes the sum over atoms of the
 * free-space potential of each atom's monopole under eq. (3.2)'s sign
 * (kind 0: -q erf(r/w)/r; kind 1: the uniform ball of charge q and radius R).
 * Faces are not touched. Atoms as for lasto_pseudo_density.
 * Errors: LASTO_ERR_ARG, LASTO_ERR_HIP.
 */
lasto_status lasto_analytic_guess(lasto_grid g, int n_atoms, const lasto_atom* atoms, double* v);

/* ------------------------------------------------------------------------
 * Learned form. The paper's solver has no learned part; this is the learned
 * initial guess grown beside the multigrid solver: a four-level 3-D U-Net on
 * the finest grid's index space (channels 16, c1, c2, c3; 3x3x3 convolutions,
 * stride-2 down-sampling, linear up-sampling with skip sums, a 1x1x1 head),
 * BF16 activations and FP32 accumulation on the matrix cores, FP32 master
 * weights trained with Adam by the library's own forward and backward
 * kernels. Plain multigrid stays the judge: lasto_learned_guess keeps the
 * correction only if it lowers the residual.
 */
typedef struct {
    int nx, ny, nz;              /* node grid the net runs on: the grid's finest level or, for the learned
                                    guess, one of its coarse levels (features at that level's nodes, the
                                    output interpolated linearly to the finest); each >= 8 */
    int ch[4];                   /* channels per level: ch[0] = 16, the others 16, 32, 48 or 64 */
    unsigned long long seed;     /* initial weights: He-normal from a splitmix64 / Box-Muller stream */
    double rho_scale;            /* feature 0 = rho * rho_scale */
    double pot_scale;            /* feature 4 = v * pot_scale */
    double h_ref;                /* features 1..3 = log(m_d / h_ref), m_d the dual width along axis d */
    double out_scale;            /* the correction is out_scale times the net's output */
} lasto_net_config;

/* Create a net on a stream (NULL: the default stream). Errors: LASTO_ERR_ARG,
 * LASTO_ERR_ALLOC, LASTO_ERR_HIP. The net owns all its device memory. */
lasto_status lasto_net_create(const lasto_net_config* cfg, void* hip_stream, lasto_net* out);
lasto_status lasto_net_destroy(lasto_net n);
/* Run the net on a node grid of nx * ny * nz (each 8 .. its creation size; every
 * buffer was allocated for the creation size): the learned coarse correction
 * meets a different coarse-level shape on each graded mesh. Errors: LASTO_ERR_ARG. */
lasto_status lasto_net_set_grid(lasto_net n, int nx, int ny, int nz);
/* Flat FP32 parameter vector: per convolution W[27][cin][cout] then b[cout]
 * (8 convolutions in forward order), then the head w[16] and its bias. */
lasto_status lasto_net_param_count(lasto_net n, long long* count);
lasto_status lasto_net_get_params(lasto_net n, float* host, long long count);
lasto_status lasto_net_set_params(lasto_net n, const float* host, long long count);
/* gradients of the last lasto_net_backward, same layout */
lasto_status lasto_net_get_grads(lasto_net n, float* host, long long count);
/*
 * Checkpoint and resume of training: the file holds the FP32 masters, Adam's
 * first and second moments and step count, the seed and the feature and
 * output scales (not the grid size, which is the loading net's own). A net
 * loaded from a checkpoint continues training with the same bits as the net
 * that wrote it, given the same data and learning rates (every reduction of
 * the forward and backward kernels runs in a fixed order).
 *   path: host file name; lasto_net_save writes "<path>.tmp" and renames it.
 * Errors: LASTO_ERR_ARG (NULL, unreadable or foreign file, channel counts
 * that differ from the net's), LASTO_ERR_STATE (a write failed), LASTO_ERR_HIP.
 */
lasto_status lasto_net_save(lasto_net n, const char* path);
lasto_status lasto_net_load(lasto_net n, const char* path);
/* the net's configuration (its scales and seed as loaded) and Adam step count (step may be NULL) */
lasto_status lasto_net_get_config(lasto_net n, lasto_net_config* cfg, long long* step);
/*
 * Read access to the net's stored BF16 tensors, for checking each kernel on
 * the operands it read: after lasto_net_forward the activations e_l (level l,
 * ch[l] channels), m_3 (level 3, ch[3]), d_l (conv output on level l + 1,
 * ch[l]) and u_l = up(d_l) + e_l (level l, ch[l]); after lasto_net_backward
 * the gradient of each convolution's pre-activation output (G0..G7, on its
 * output level with its output channels) and of u_l (DU0..DU2).
 *   out: device [nz_l][ny_l][nx_l][c] BF16 bit patterns, count its length, or
 *   NULL to query the shape; dims: host [4] out: nx_l, ny_l, nz_l, c.
 * Errors: LASTO_ERR_ARG (NULL dims, unknown tensor, count mismatch), LASTO_ERR_HIP.
 */
enum {
    LASTO_NET_E0 = 0, LASTO_NET_E1, LASTO_NET_E2, LASTO_NET_E3, LASTO_NET_M3,
    LASTO_NET_D2, LASTO_NET_D1, LASTO_NET_D0, LASTO_NET_U2, LASTO_NET_U1, LASTO_NET_U0,
    LASTO_NET_G0, LASTO_NET_G1, LASTO_NET_G2, LASTO_NET_G3, LASTO_NET_G4, LASTO_NET_G5, LASTO_NET_G6, LASTO_NET_G7,
    LASTO_NET_DU0, LASTO_NET_DU1, LASTO_NET_DU2
};
lasto_status lasto_net_tensor(lasto_net n, int which, uint16_t* out, long long count, int* dims);

/*
 * Net input features from a source and a potential on grid g (whose finest
 * level must match the net's grid): x = device [nz][ny][nx][8] BF16 (bit
 * patterns as uint16), channels rho * rho_scale, log(m_x / h_ref),
 * log(m_y / h_ref), log(m_z / h_ref), v * pot_scale, face indicator, 0, 0.
 */
lasto_status lasto_net_features(lasto_grid g, lasto_net n, const double* rho, const double* v, uint16_t* x);
/* y = device [nz][ny][nx] FP32: the net's output for features x */
lasto_status lasto_net_forward(lasto_net n, const uint16_t* x, float* y);
/* After lasto_net_forward(x): gradients of L = sum_v weight[v] (y[v] - target[v])^2
 * (target, weight device FP32 [nz][ny][nx]); *loss (host, may be NULL) = L. */
lasto_status lasto_net_backward(lasto_net n, const uint16_t* x, const float* target, const float* weight,
                                double* loss);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) with the last gradients */
lasto_status lasto_net_adam_step(lasto_net n, float lr);
/* forward + backward + Adam */
lasto_status lasto_net_train_step(lasto_net n, const uint16_t* x, const float* target, const float* weight,
                                  float lr, double* loss);

/*
 * Learned initial guess: v holds the Dirichlet data on its faces and an
 * initial guess inside (for instance lasto_analytic_guess). Two candidates
 * are formed: v and v + out_scale * net(features(rho, v)); each gets one
 * red-black sweep of eq. (3.2)'s discrete form (red, then black; faces kept),
 * and the one with the smaller relative residual
 * ||4 pi rho - A v||_W / ||4 pi rho - A v_bc||_W is returned in v. On a
 * batched grid every right-hand side is judged on its own (the net runs per
 * copy; the sweeps and norms of all copies share launches), with the same
 * bits as a grid holding that copy alone.
 *   rel: host [2 n_batch] or NULL: per copy, that residual for the plain and
 *     the learned candidate.
 *   accepted: host, may be NULL: how many copies kept the learned candidate.
 * Uses the grid's solver scratch (not to be called during a solve on the same grid).
 * Errors: LASTO_ERR_ARG (the net's grid differs from one copy of the finest level), LASTO_ERR_HIP.
 */
lasto_status lasto_learned_guess(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel,
                                 int* accepted);

/*
 * Learned correction of an iterate (the learned coarse correction): a net
 * maps the residual r = 4 pi rho - A v, scaled to unit RMS s = ||r||_W /
 * sqrt(sum vol), to the error; the candidate v + s * out_scale * net(r / s)
 * and v itself each get one red-black sweep, and the one with the smaller
 * relative residual is returned in v (rel, accepted as for
 * lasto_learned_guess). Between cycles of a stationary solve this removes
 * the smooth error a V-cycle reduces slowly, when the net has learned it.
 * Features: channel 0 = (r / s) * rho_scale, 1..3 as lasto_net_features,
 * 4 = 0, 5 = face indicator. One right-hand side per grid; uses the grid's
 * solver scratch. Errors: LASTO_ERR_ARG, LASTO_ERR_HIP.
 */
lasto_status lasto_learned_correction(lasto_grid g, lasto_net n, const double* rho, double* v, double* rel,
                                      int* accepted);
/*
 * A training pair of the learned coarse correction for iterate v (one
 * right-hand side): the restricted residual f_c that a cycle's descent
 * produces at level c (nu1 red-black pre-smoothing sweeps from zero on each
 * finer level, the red residual, the restriction), as the net's features
 * (x: device [nz_c][ny_c][nx_c][8] BF16, as the solve forms them), and the
 * target e_c / (s out_scale) (target: device FP32 [nz_c][ny_c][nx_c], zero
 * on faces), e_c the solution of A_c e = f_c by 40 V-cycles of level c.
 *   r_scale: host out s; dims: host [3] out nx_c, ny_c, nz_c.
 * Uses the grid's solver vectors (zero again on return).
 * Errors: LASTO_ERR_ARG (level outside 1 .. levels - 1, a level that does not
 * fit the net, a zero residual), LASTO_ERR_HIP.
 */
lasto_status lasto_coarse_pair(lasto_grid g, lasto_net n, const double* rho, const double* v, int level, int nu1,
                               uint16_t* x, float* target, double* r_scale, int* dims);
/* the correction net's features for iterate v (x as for lasto_net_features);
 * *r_scale (host) receives s. Errors: LASTO_ERR_ARG (zero residual), LASTO_ERR_HIP. */
lasto_status lasto_net_correction_features(lasto_grid g, lasto_net n, const double* rho, const double* v,
                                           uint16_t* x, double* r_scale);

#ifdef __cplusplus
}
#endif
#endif /* LASTO_H */
