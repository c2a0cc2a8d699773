// Source, boundary and interpolation kernels of the Hartree step.
//   k_atom_prep : per-atom constants (Gaussian renormalisation, quartic fit)
//   k_pseudo    : pseudo-density on every node (Section 1; eq. (3.2) and its
//                 three constraints)
//   k_moments   : Q_lm = sum_n vol_n rho_n r^l y_lm(x_n - c), l <= 4 (the
//                 paper's L <= 4 of eq. (3.1))
//   k_bc        : multipole field of Q on the six faces (zero: eq. (3.3))
//   k_interp    : tricubic Lagrange values at the sphere points
//                 (eq. (3.5)-(3.6) take V_C on the sphere boundaries)
#include <algorithm>

#include "internal.h"

namespace lasto {

// r^l y_lm normalisation: sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times sqrt(2)
// for m != 0; index l*l + l + m. Filled once per process.
__constant__ double c_ynorm[25];
static bool g_ynorm_ready = false;

// The solid harmonic r^l y_lm is a homogeneous polynomial of degree l in
// (x, y, z): c_mono[lm][p] is its coefficient of the monomial p = (a, b, c),
// a + b + c <= 4, numbered a-major (mono_index). Filled with c_ynorm.
constexpr int kMono = 35;
__constant__ double c_mono[25 * kMono];

static int mono_index(int a, int b, int c)
{
    int p = 0;
    for (int a2 = 0; a2 <= 4; ++a2)
        for (int b2 = 0; b2 <= 4 - a2; ++b2)
            for (int c2 = 0; c2 <= 4 - a2 - b2; ++c2) {
                if (a2 == a && b2 == b && c2 == c) return p;
                ++p;
            }
    return -1;
}

// polynomials of degree <= 4 in x, y, z: coefficient [a][b][c] of x^a y^b z^c
struct Poly4 {
    double c[5][5][5] = {};
    Poly4 shifted(int d) const   // times x (d 0), y (1) or z (2)
    {
        Poly4 r;
        for (int a = 0; a <= 4; ++a)
            for (int b = 0; b <= 4; ++b)
                for (int e = 0; e <= 4; ++e) {
                    if (c[a][b][e] == 0.0) continue;
                    const int a2 = a + (d == 0), b2 = b + (d == 1), e2 = e + (d == 2);
                    if (a2 > 4 || b2 > 4 || e2 > 4) continue;   // (degree stays <= 4)
                    r.c[a2][b2][e2] += c[a][b][e];
                }
        return r;
    }
    Poly4 lin(double s, const Poly4& o, double t) const   // s this + t o
    {
        Poly4 r;
        for (int a = 0; a <= 4; ++a)
            for (int b = 0; b <= 4; ++b)
                for (int e = 0; e <= 4; ++e) r.c[a][b][e] = s * c[a][b][e] + t * o.c[a][b][e];
        return r;
    }
};

// the recurrence of solid_harmonics (below) carried out on polynomials
static void harmonic_polys(const double* ynorm, double* mono)
{
    Poly4 S[25];
    Poly4 mre, mim;
    mre.c[0][0][0] = 1.0;
    for (int m = 0; m <= 4; ++m) {
        if (m > 0) {
            const Poly4 nre = mre.shifted(0).lin(1.0, mim.shifted(1), -1.0);
            const Poly4 nim = mre.shifted(1).lin(1.0, mim.shifted(0), 1.0);
            mre = nre.lin(2.0 * m - 1.0, nre, 0.0);
            mim = nim.lin(2.0 * m - 1.0, nim, 0.0);
        }
        Poly4 pre, pim, cre = mre, cim = mim;
        for (int l = m; l <= 4; ++l) {
            if (l > m) {
                const double a = (2.0 * (l - 1) + 1.0) / (double)(l - m);
                const double b = (double)(l - 1 + m) / (double)(l - m);
                const Poly4 r2re = pre.shifted(0).shifted(0).lin(1.0, pre.shifted(1).shifted(1), 1.0)
                                       .lin(1.0, pre.shifted(2).shifted(2), 1.0);
                const Poly4 r2im = pim.shifted(0).shifted(0).lin(1.0, pim.shifted(1).shifted(1), 1.0)
                                       .lin(1.0, pim.shifted(2).shifted(2), 1.0);
                const Poly4 nre = cre.shifted(2).lin(a, r2re, -b);
                const Poly4 nim = cim.shifted(2).lin(a, r2im, -b);
                pre = cre; pim = cim;
                cre = nre; cim = nim;
            }
            S[l * l + l + m] = cre.lin(ynorm[l * l + l + m], cre, 0.0);
            if (m > 0) S[l * l + l - m] = cim.lin(ynorm[l * l + l - m], cim, 0.0);
        }
    }
    for (int q = 0; q < 25; ++q)
        for (int a = 0; a <= 4; ++a)
            for (int b = 0; b <= 4 - a; ++b)
                for (int e = 0; e <= 4 - a - b; ++e) mono[q * kMono + mono_index(a, b, e)] = S[q].c[a][b][e];
}

hipError_t init_harmonic_constants()
{
    if (g_ynorm_ready) return hipSuccess;
    double h[25];
    for (int l = 0; l <= 4; ++l)
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            double ratio = 1.0;   // (l-|m|)!/(l+|m|)!
            for (int t = l - am + 1; t <= l + am; ++t) ratio /= (double)t;
            double nrm = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * ratio);
            if (m != 0) nrm *= std::sqrt(2.0);
            h[l * l + l + m] = nrm;
        }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_ynorm), h, sizeof(h));
    if (e != hipSuccess) return e;
    static double mono[25 * kMono];
    harmonic_polys(h, mono);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_mono), mono, sizeof(mono));
    if (e == hipSuccess) g_ynorm_ready = true;
    return e;
}

// Real solid harmonics r^l y_lm(x,y,z), l <= lmax <= 4, without the
// Condon-Shortley phase. Built from the complex Q_l^m = r^l P_l^m(cos t) e^{i m p}:
//   Q_m^m = (2m-1)!! (x + i y)^m,  Q_{m+1}^m = (2m+1) z Q_m^m,
//   (l-m+1) Q_{l+1}^m = (2l+1) z Q_l^m - (l+m) r^2 Q_{l-1}^m;
// then S_l,m = N Re Q_l^m (m >= 0), S_l,-m = N Im Q_l^m.
__device__ __forceinline__ void solid_harmonics(double x, double y, double z, int lmax, double* S)
{
    const double r2 = x * x + y * y + z * z;
    double mre = 1.0, mim = 0.0;   // Q_m^m
    double dfact = 1.0;            // (2m-1)!!
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            // (x+iy)^m = (x+iy)^(m-1) (x+iy); (2m-1)!! = (2m-3)!! (2m-1)
            const double nre = mre * x - mim * y;
            const double nim = mre * y + mim * x;
            mre = nre * (2.0 * m - 1.0);
            mim = nim * (2.0 * m - 1.0);
        }
        (void)dfact;
        double pre = 0.0, pim = 0.0;     // Q_{l-1}^m
        double cre = mre, cim = mim;     // Q_l^m at l = m
        for (int l = m; l <= lmax; ++l) {
            if (l > m) {
                // Q_l^m from Q_{l-1}^m (c) and Q_{l-2}^m (p)
                const double a = (2.0 * (l - 1) + 1.0) / (double)(l - m);
                const double b = (double)(l - 1 + m) / (double)(l - m);
                const double nre = a * z * cre - b * r2 * pre;
                const double nim = a * z * cim - b * r2 * pim;
                pre = cre; pim = cim;
                cre = nre; cim = nim;
            }
            S[l * l + l + m] = c_ynorm[l * l + l + m] * cre;
            if (m > 0) S[l * l + l - m] = c_ynorm[l * l + l - m] * cim;
        }
    }
}

// ---------------------------------------------------------------- atoms
// One workgroup per atom.
// kind 0: s = 1/((pi w^2)^(-3/2) prod_d sum_i m_d,i exp(-(x_d,i - c_d)^2/w^2))
//         (the discrete integral of the normalised Gaussian is separable;
//         each 1-D sum is split over the workgroup and reduced in a fixed order)
// kind 1: quartic a + b r^2 + c r^4 from value, slope and charge at R, by
//         Cramer's rule on
//           [1, R^2, R^4; 0, 2R, 4R^3; 4piR^3/3, 4piR^5/5, 4piR^7/7] (a,b,c) = (rho_R, drho_R, q)
// Then the per-atom constants the density kernel uses.
constexpr int AP_NT = 256;

__global__ __launch_bounds__(AP_NT) void k_atom_prep(LevelView L, AtomDev* atoms, int n_atoms, int renormalize)
{
    __shared__ double red[AP_NT];
    const int a = blockIdx.x;
    if (a >= n_atoms) return;
    AtomDev& A = atoms[a];
    double s = 1.0;
    if (A.kind == 0 && renormalize) {
        const double w2 = A.w * A.w;
        double prod = pow(kPi * w2, -1.5);
        for (int d = 0; d < 3; ++d) {
            double sum = 0.0;
            for (int i = threadIdx.x; i < L.ax[d].n; i += AP_NT) {
                const double t = L.ax[d].x[i] - A.c[d];
                sum += L.ax[d].m[i] * exp(-t * t / w2);
            }
            red[threadIdx.x] = sum;
            __syncthreads();
            for (int h = AP_NT / 2; h > 0; h >>= 1) {
                if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                __syncthreads();
            }
            prod *= red[0];
            __syncthreads();
        }
        s = 1.0 / prod;
    }
    if (threadIdx.x != 0) return;
    if (A.kind == 0) {
        A.s = s;
        A.pre = A.q * s * pow(kPi * A.w * A.w, -1.5);
        A.iw2 = 1.0 / (A.w * A.w);
        A.cut2 = (7.0 * A.w) * (7.0 * A.w);
    } else {
        const double R = A.R, R2 = R * R;
        const double m00 = 1.0, m01 = R2, m02 = R2 * R2;
        const double m10 = 0.0, m11 = 2.0 * R, m12 = 4.0 * R * R2;
        const double f = 4.0 * kPi * R * R2;
        const double m20 = f / 3.0, m21 = f * R2 / 5.0, m22 = f * R2 * R2 / 7.0;
        const double r0 = A.rho_R, r1 = A.drho_R, r2 = A.q;
        const double det = m00 * (m11 * m22 - m12 * m21) - m01 * (m10 * m22 - m12 * m20) + m02 * (m10 * m21 - m11 * m20);
        const double da = r0 * (m11 * m22 - m12 * m21) - m01 * (r1 * m22 - m12 * r2) + m02 * (r1 * m21 - m11 * r2);
        const double db = m00 * (r1 * m22 - m12 * r2) - r0 * (m10 * m22 - m12 * m20) + m02 * (m10 * r2 - r1 * m20);
        const double dc = m00 * (m11 * r2 - r1 * m21) - m01 * (m10 * r2 - r1 * m20) + r0 * (m10 * m21 - m11 * m20);
        A.coef[0] = da / det;
        A.coef[1] = db / det;
        A.coef[2] = dc / det;
        A.s = 1.0;
        A.pre = 0.0;
        A.iw2 = 0.0;
        A.cut2 = R2;
    }
    A.lcut2 = A.lmax >= 1 ? 42.25 / A.alpha * (1.0 + 1e-12) : -1.0;   // culling only (a little wide)
    A.cull2 = fmax(fmax(A.cut2, A.R * A.R), A.lcut2) * (1.0 + 1e-12);
    for (int l = 1; l <= 4; ++l)
        for (int m = -l; m <= l; ++m) A.cn[l * l + l + m - 1] = A.clm[l * l + l + m - 1] * c_ynorm[l * l + l + m];
}

hipError_t launch_atom_prep(lasto_grid g, AtomDev* atoms, int n_atoms, int renormalize)
{
    hipLaunchKernelGGL(k_atom_prep, dim3(n_atoms), dim3(AP_NT), 0, g->stream, g->cview, atoms, n_atoms,
                       renormalize);
    return hipGetLastError();
}

// sum_{1 <= l <= lmax, m} cn_lm Q-recurrence values: the l >= 1 part of
// sum c_lm r^l y_lm at (x, y, z), with cn = c_lm times the normalisation.
// Same recurrences as solid_harmonics, unrolled so every term has a fixed
// register (no array indexed at run time).
__device__ __forceinline__ double clm_sum(double x, double y, double z, int lmax, const double* __restrict__ cn)
{
    const double r2 = x * x + y * y + z * z;
    double s = 0.0;
    double mre = 1.0, mim = 0.0;   // Q_m^m
#pragma unroll
    for (int m = 0; m <= 4; ++m) {
        if (m > lmax) break;
        if (m > 0) {
            const double nre = mre * x - mim * y;
            const double nim = mre * y + mim * x;
            mre = nre * (2.0 * m - 1.0);
            mim = nim * (2.0 * m - 1.0);
        }
        double pre = 0.0, pim = 0.0;
        double cre = mre, cim = mim;
#pragma unroll
        for (int l = m; l <= 4; ++l) {
            if (l > lmax) break;
            if (l > m) {
                const double a = (2.0 * (l - 1) + 1.0) / (double)(l - m);
                const double b = (double)(l - 1 + m) / (double)(l - m);
                const double nre = a * z * cre - b * r2 * pre;
                const double nim = a * z * cim - b * r2 * pim;
                pre = cre;
                pim = cim;
                cre = nre;
                cim = nim;
            }
            if (l >= 1) {
                s += cn[l * l + l + m - 1] * cre;
                if (m > 0) s += cn[l * l + l - m - 1] * cim;
            }
        }
    }
    return s;
}

// --------------------------------------------------------------- density
// A workgroup covers 64 x 4 x 4 nodes. It first lists, in atom order, the
// atoms whose cut-off sphere reaches its box (a block-wide ordered
// compaction), then each thread sums only those atoms at its 4 nodes.
constexpr int PS_X = 64, PS_Y = 4, PS_Z = 4, PS_NT = PS_X * PS_Y, PS_LIST = 1024;

__global__ __launch_bounds__(PS_NT) void k_pseudo(LevelView L, const AtomDev* __restrict__ atoms, int n_atoms,
                                                  const double* __restrict__ rho_inter, double* __restrict__ rho)
{
    __shared__ int list[PS_LIST];
    __shared__ int wcount[PS_NT / 64];
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int i0 = blockIdx.x * PS_X, j0 = blockIdx.y * PS_Y, k0 = blockIdx.z * PS_Z;
    const int i1 = min(i0 + PS_X, nx) - 1, j1 = min(j0 + PS_Y, ny) - 1, k1 = min(k0 + PS_Z, nz) - 1;
    const double bx0 = L.ax[0].x[i0], bx1 = L.ax[0].x[i1];
    const double by0 = L.ax[1].x[j0], by1 = L.ax[1].x[j1];
    const double bz0 = L.ax[2].x[k0], bz1 = L.ax[2].x[k1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int count = 0;
    bool all = n_atoms > PS_LIST;   // too many to list: every atom is tested per node
    for (int base = 0; base < n_atoms && !all; base += PS_NT) {
        const int a = base + (int)threadIdx.x;
        bool hit = false;
        if (a < n_atoms) {
            const AtomDev& A = atoms[a];
            const double dx = fmax(fmax(bx0 - A.c[0], A.c[0] - bx1), 0.0);
            const double dy = fmax(fmax(by0 - A.c[1], A.c[1] - by1), 0.0);
            const double dz = fmax(fmax(bz0 - A.c[2], A.c[2] - bz1), 0.0);
            hit = dx * dx + dy * dy + dz * dz < A.cull2;
        }
        const unsigned long long mask = __ballot(hit);
        if (lane == 0) wcount[wid] = __popcll(mask);
        __syncthreads();
        int off = count;
        for (int w = 0; w < wid; ++w) off += wcount[w];
        if (hit) list[off + __popcll(mask & ((1ull << lane) - 1ull))] = a;
        for (int w = 0; w < PS_NT / 64; ++w) count += wcount[w];
        __syncthreads();
    }
    const int i = i0 + lane, j = j0 + wid;
    if (i > i1 || j > j1) return;
    const double px = L.ax[0].x[i], py = L.ax[1].x[j];
    const int na = all ? n_atoms : count;
    for (int k = k0; k <= k1; ++k) {
        const double pz = L.ax[2].x[k];
        double acc = 0.0;
        bool outside = true;
        for (int t = 0; t < na; ++t) {
            const AtomDev& A = atoms[all ? t : list[t]];
            const double dx = px - A.c[0], dy = py - A.c[1], dz = pz - A.c[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= A.cull2) continue;
            if (r2 < A.R * A.R) outside = false;
            if (r2 < A.cut2) acc += A.kind == 0 ? A.pre * exp(-r2 * A.iw2) : A.coef[0] + r2 * (A.coef[1] + r2 * A.coef[2]);
            if (A.lmax >= 1 && A.alpha * r2 < 42.25) acc += clm_sum(dx, dy, dz, A.lmax, A.cn) * exp(-A.alpha * r2);
        }
        const size_t at = ((size_t)k * ny + j) * nx + i;
        if (rho_inter && outside) acc += rho_inter[at];
        rho[at] = acc;
    }
}

hipError_t launch_pseudo(lasto_grid g, const AtomDev* atoms, int n_atoms, const double* rho_inter, double* rho)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    const dim3 grid((L.nx + PS_X - 1) / PS_X, (L.ny + PS_Y - 1) / PS_Y, (L.nz + PS_Z - 1) / PS_Z);
    hipLaunchKernelGGL(k_pseudo, grid, dim3(PS_NT), 0, g->stream, L, atoms, n_atoms, rho_inter, rho);
    return hipGetLastError();
}

// ------------------------------------------------------ analytic guess
// Interior of v = the sum over atoms of the free-space potential of each
// atom's monopole under Laplacian(V) = 4 pi rho (so a positive charge gives
// V -> -q/r): kind 0 (Gaussian of width w) -q erf(r/w)/r, with the limit
// -2 q / (sqrt(pi) w) at r = 0 and erf taken as 1 beyond 6w; kind 1 (the
// quartic inside R) the uniform ball, -q (3R^2 - r^2)/(2R^3) inside and -q/r
// outside. Faces are left as they are.
//
// A guess only starts the iteration, so it is summed in FP32: coordinates
// relative to the workgroup's first node (exact to about 1e-7 bohr near
// it), the far field -q/r (beyond 6w, or R for kind 1: most node-atom pairs)
// by the hardware reciprocal square root, the near field (erf, the ball) by
// FP32 formulas, in partial sums over at most 32 atoms added in FP64. Every
// term has the sign of its charge, so with positive charges the result is
// within about 32 * 2^-24 (plus a few ulp per term) of the FP64 sum,
// relative: far below what the guess itself misses (the l >= 1 terms, the
// discretisation).
constexpr int GU_X = 64, GU_Y = 4, GU_Z = 4, GU_NT = GU_X * GU_Y, GU_CHUNK = 512, GU_PART = 32;
constexpr float kTwoOverSqrtPi = 1.12837916709551257f;

// an atom's LDS entry (near-field radius^2 and the near-field constants):
// kind 0 (Gaussian): (36 w^2, 1/w, the radius below which erf(r/w)/r takes
// its r -> 0 limit, that limit 2/(sqrt(pi) w)); kind 1 (uniform ball):
// (R^2, 0, 3 R^2, 1/(2 R^3))
__device__ __forceinline__ float4 guess_params(const AtomDev& A)
{
    if (A.kind == 0) {
        const float iw = (float)(1.0 / A.w);
        return make_float4((float)(36.0 * A.w * A.w), iw, 1e-6f / iw, kTwoOverSqrtPi * iw);
    }
    return make_float4((float)(A.R * A.R), 0.0f, (float)(3.0 * A.R * A.R), (float)(0.5 / (A.R * A.R * A.R)));
}

// The workgroup's nodes as FP32 offsets from its origin (the same roundings
// as the nodes' own offsets), and whether an atom's near field (squared
// radius r2n) may reach one of them: the squared distance from the centre to
// the box, taken a little short (a relative 1e-4 and 1e-30), below r2n. An
// atom it clears is beyond r2n from every node by more than any rounding of
// the nodes' own r^2, so those take the far field whichever path they run.
struct GuessBox {
    float xl, xh, yl, yh, zl, zh;
    __device__ int reaches(const float4& c, float r2n) const
    {
        const float dx = fmaxf(fmaxf(xl - c.x, c.x - xh), 0.0f);
        const float dy = fmaxf(fmaxf(yl - c.y, c.y - yh), 0.0f);
        const float dz = fmaxf(fmaxf(zl - c.z, c.z - zh), 0.0f);
        const float d2 = dx * dx + dy * dy + dz * dz;
        return d2 * (1.0f - 1e-4f) - 1e-30f < r2n ? 1 : 0;
    }
};

__device__ __forceinline__ GuessBox guess_box(const LevelView& L, int i0, int j0, int k0, int nzp, double ox, double oy,
                                              double oz)
{
    GuessBox b;
    const int i1 = min(i0 + GU_X - 1, L.nx - 2), j1 = min(j0 + GU_Y - 1, L.ny - 2), k1 = min(k0 + nzp - 1, L.nz - 2);
    b.xl = (float)(L.ax[0].x[i0] - ox);
    b.xh = (float)(L.ax[0].x[i1] - ox);
    b.yl = (float)(L.ax[1].x[j0] - oy);
    b.yh = (float)(L.ax[1].x[j1] - oy);
    b.zl = (float)(L.ax[2].x[min(k0, L.nz - 2)] - oz);
    b.zh = (float)(L.ax[2].x[k1] - oz);
    return b;
}

// the potential shape at squared distance r2 < p.x from the atom (near field)
__device__ __forceinline__ float guess_near(float r2, const float4& p)
{
    if (p.y > 0.0f) {
        const float r = sqrtf(r2);
        return r > p.z ? erff(r * p.y) / r : p.w;   // erf(r/w)/r, its limit at r = 0
    }
    return (p.z - r2) * p.w;                         // (3R^2 - r^2)/(2R^3)
}

__global__ __launch_bounds__(GU_NT) void k_guess(LevelView L, const AtomDev* __restrict__ atoms, int n_atoms,
                                                 double* __restrict__ v)
{
    __shared__ float4 sc[GU_CHUNK];   // atom centre relative to the origin, and charge
    __shared__ float4 sp[GU_CHUNK];   // guess_params
    __shared__ int sn[GU_CHUNK];      // 1: the atom's near field may reach this workgroup's nodes
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int i0 = 1 + blockIdx.x * GU_X, j0 = 1 + blockIdx.y * GU_Y, k0 = 1 + blockIdx.z * GU_Z;
    const int i = i0 + (threadIdx.x & (GU_X - 1)), j = j0 + (int)(threadIdx.x / GU_X);
    const bool live = i <= nx - 2 && j <= ny - 2;
    // origin: the workgroup's first node
    const double ox = L.ax[0].x[i0], oy = L.ax[1].x[j0], oz = L.ax[2].x[k0];
    const float fx = (float)(L.ax[0].x[min(i, nx - 2)] - ox), fy = (float)(L.ax[1].x[min(j, ny - 2)] - oy);
    float fz[GU_Z];
#pragma unroll
    for (int t = 0; t < GU_Z; ++t) fz[t] = (float)(L.ax[2].x[min(k0 + t, nz - 2)] - oz);
    double acc[GU_Z];
#pragma unroll
    for (int t = 0; t < GU_Z; ++t) acc[t] = 0.0;
    const GuessBox box = guess_box(L, i0, j0, k0, GU_Z, ox, oy, oz);
    for (int a0 = 0; a0 < n_atoms; a0 += GU_CHUNK) {
        const int na = min(GU_CHUNK, n_atoms - a0);
        __syncthreads();
        for (int t = threadIdx.x; t < na; t += GU_NT) {
            const AtomDev& A = atoms[a0 + t];
            sc[t] = make_float4((float)(A.c[0] - ox), (float)(A.c[1] - oy), (float)(A.c[2] - oz), (float)A.q);
            sp[t] = guess_params(A);
            sn[t] = box.reaches(sc[t], sp[t].x);
        }
        __syncthreads();
        for (int a1 = 0; a1 < na; a1 += GU_PART) {
            float part[GU_Z];
#pragma unroll
            for (int t = 0; t < GU_Z; ++t) part[t] = 0.0f;
            const int a2 = min(a1 + GU_PART, na);
            for (int a = a1; a < a2; ++a) {
                const float4 c = sc[a];
                const float4 p = sp[a];
                const float dx = fx - c.x, dy = fy - c.y;
                const float dxy = fmaf(dx, dx, dy * dy);
                // the far field 1/r on every plane, then the near field
                // where a lane needs it (only for atoms whose near field may
                // reach the workgroup, a test uniform over it)
                float r2[GU_Z], f[GU_Z];
#pragma unroll
                for (int t = 0; t < GU_Z; ++t) {
                    const float dz = fz[t] - c.z;
                    r2[t] = fmaf(dz, dz, dxy);
                    f[t] = __builtin_amdgcn_rsqf(r2[t]);
                }
                if (sn[a]) {
                    bool near = false;
#pragma unroll
                    for (int t = 0; t < GU_Z; ++t) near |= !(r2[t] >= p.x);
                    if (near) {
#pragma unroll
                        for (int t = 0; t < GU_Z; ++t)
                            if (!(r2[t] >= p.x)) f[t] = guess_near(r2[t], p);
                    }
                }
#pragma unroll
                for (int t = 0; t < GU_Z; ++t) part[t] = fmaf(-c.w, f[t], part[t]);
            }
#pragma unroll
            for (int t = 0; t < GU_Z; ++t) acc[t] += (double)part[t];
        }
    }
    if (!live) return;
#pragma unroll
    for (int t = 0; t < GU_Z; ++t)
        if (k0 + t <= nz - 2) v[((size_t)(k0 + t) * ny + j) * nx + i] = acc[t];
}

hipError_t launch_guess(lasto_grid g, const AtomDev* atoms, int n_atoms, double* v)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    const dim3 grid((L.nx - 2 + GU_X - 1) / GU_X, (L.ny - 2 + GU_Y - 1) / GU_Y, (L.nz - 2 + GU_Z - 1) / GU_Z);
    hipLaunchKernelGGL(k_guess, grid, dim3(GU_NT), 0, g->stream, L, atoms, n_atoms, v);
    return hipGetLastError();
}

// The same guess for NB right-hand sides whose atoms share every centre,
// width, radius and kind and differ only in charge (the perturbations of one
// structure): each node-atom pair's potential shape is evaluated once and
// scaled by the NB charges, the same FP32 operations per copy as k_guess in
// the same order from the same origins (so the same bits). atoms:
// [NB][n_atoms] (copy-major);
// copy b of v at v + b * N.
constexpr int GB_Z = 2;

template <int NB>
__global__ __launch_bounds__(GU_NT) void k_guess_shared(LevelView L, const AtomDev* __restrict__ atoms, int n_atoms,
                                                        size_t N, double* __restrict__ v)
{
    __shared__ float4 sc[GU_CHUNK];     // atom centre relative to the origin; w unused
    __shared__ float4 sp[GU_CHUNK];     // as in k_guess
    __shared__ float sq[GU_CHUNK][NB];  // the charge of the atom in each copy
    __shared__ int sn[GU_CHUNK];        // as in k_guess
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int i0 = 1 + blockIdx.x * GU_X, j0 = 1 + blockIdx.y * GU_Y, k0 = 1 + blockIdx.z * GB_Z;
    const int i = i0 + (threadIdx.x & (GU_X - 1)), j = j0 + (int)(threadIdx.x / GU_X);
    const bool live = i <= nx - 2 && j <= ny - 2;
    // the origin of k_guess's workgroup holding these planes (same roundings)
    static_assert(GU_Z % GB_Z == 0, "a guess workgroup's planes split evenly");
    const int ko = 1 + (blockIdx.z / (GU_Z / GB_Z)) * GU_Z;
    const double ox = L.ax[0].x[i0], oy = L.ax[1].x[j0], oz = L.ax[2].x[ko];
    const float fx = (float)(L.ax[0].x[min(i, nx - 2)] - ox), fy = (float)(L.ax[1].x[min(j, ny - 2)] - oy);
    float fz[GB_Z];
#pragma unroll
    for (int t = 0; t < GB_Z; ++t) fz[t] = (float)(L.ax[2].x[min(k0 + t, nz - 2)] - oz);
    double acc[GB_Z][NB];
#pragma unroll
    for (int t = 0; t < GB_Z; ++t)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[t][b] = 0.0;
    const GuessBox box = guess_box(L, i0, j0, k0, GB_Z, ox, oy, oz);
    for (int a0 = 0; a0 < n_atoms; a0 += GU_CHUNK) {
        const int na = min(GU_CHUNK, n_atoms - a0);
        __syncthreads();
        for (int t = threadIdx.x; t < na; t += GU_NT) {
            const AtomDev& A = atoms[a0 + t];
            sc[t] = make_float4((float)(A.c[0] - ox), (float)(A.c[1] - oy), (float)(A.c[2] - oz), 0.0f);
            sp[t] = guess_params(A);
            sn[t] = box.reaches(sc[t], sp[t].x);
#pragma unroll
            for (int b = 0; b < NB; ++b) sq[t][b] = (float)atoms[(size_t)b * n_atoms + a0 + t].q;
        }
        __syncthreads();
        for (int a1 = 0; a1 < na; a1 += GU_PART) {
            float part[GB_Z][NB];
#pragma unroll
            for (int t = 0; t < GB_Z; ++t)
#pragma unroll
                for (int b = 0; b < NB; ++b) part[t][b] = 0.0f;
            const int a2 = min(a1 + GU_PART, na);
            for (int a = a1; a < a2; ++a) {
                const float4 c = sc[a];
                const float4 p = sp[a];
                const float dx = fx - c.x, dy = fy - c.y;
                const float dxy = fmaf(dx, dx, dy * dy);
                float r2[GB_Z], f[GB_Z];
#pragma unroll
                for (int t = 0; t < GB_Z; ++t) {
                    const float dz = fz[t] - c.z;
                    r2[t] = fmaf(dz, dz, dxy);
                    f[t] = __builtin_amdgcn_rsqf(r2[t]);
                }
                if (sn[a]) {
                    bool near = false;
#pragma unroll
                    for (int t = 0; t < GB_Z; ++t) near |= !(r2[t] >= p.x);
                    if (near) {
#pragma unroll
                        for (int t = 0; t < GB_Z; ++t)
                            if (!(r2[t] >= p.x)) f[t] = guess_near(r2[t], p);
                    }
                }
#pragma unroll
                for (int t = 0; t < GB_Z; ++t)
#pragma unroll
                    for (int b = 0; b < NB; ++b) part[t][b] = fmaf(-sq[a][b], f[t], part[t][b]);
            }
#pragma unroll
            for (int t = 0; t < GB_Z; ++t)
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[t][b] += (double)part[t][b];
        }
    }
    if (!live) return;
#pragma unroll
    for (int t = 0; t < GB_Z; ++t)
        if (k0 + t <= nz - 2) {
            const size_t at = ((size_t)(k0 + t) * ny + j) * nx + i;
#pragma unroll
            for (int b = 0; b < NB; ++b) v[(size_t)b * N + at] = acc[t][b];
        }
}

template <int NB>
static hipError_t launch_guess_shared(lasto_grid g, const AtomDev* atoms, int n_atoms, double* v)
{
    const LevelView& L = g->cview;
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    const dim3 grid((L.nx - 2 + GU_X - 1) / GU_X, (L.ny - 2 + GU_Y - 1) / GU_Y, (L.nz - 2 + GB_Z - 1) / GB_Z);
    hipLaunchKernelGGL(k_guess_shared<NB>, grid, dim3(GU_NT), 0, g->stream, L, atoms, n_atoms, N, v);
    return hipGetLastError();
}

// the guess of every right-hand side of the grid: copies whose atoms share
// their geometry with copy 0 of their group of up to 8 go through one pass
hipError_t launch_guess_all(lasto_grid g, const AtomDev* dev_atoms, const lasto_atom* host_atoms, int n_atoms,
                            double* v)
{
    const int nb = g->n_batch;
    const size_t N = (size_t)g->cview.nx * g->cview.ny * g->cview.nz;
    auto same_geometry = [&](int b) {
        for (int a = 0; a < n_atoms; ++a) {
            const lasto_atom& x = host_atoms[(size_t)b * n_atoms + a];
            const lasto_atom& y = host_atoms[a];
            if (x.center[0] != y.center[0] || x.center[1] != y.center[1] || x.center[2] != y.center[2] ||
                x.kind != y.kind || x.width != y.width || x.radius != y.radius)
                return false;
        }
        return true;
    };
    bool shared = nb > 1;
    for (int b = 1; b < nb && shared; ++b) shared = same_geometry(b);
    int b = 0;
    if (shared) {
        for (; b + 8 <= nb; b += 8) {
            hipError_t e = launch_guess_shared<8>(g, dev_atoms + (size_t)b * n_atoms, n_atoms, v + b * N);
            if (e != hipSuccess) return e;
        }
        for (; b + 4 <= nb; b += 4) {
            hipError_t e = launch_guess_shared<4>(g, dev_atoms + (size_t)b * n_atoms, n_atoms, v + b * N);
            if (e != hipSuccess) return e;
        }
        for (; b + 2 <= nb; b += 2) {
            hipError_t e = launch_guess_shared<2>(g, dev_atoms + (size_t)b * n_atoms, n_atoms, v + b * N);
            if (e != hipSuccess) return e;
        }
    }
    for (; b < nb; ++b) {
        hipError_t e = launch_guess(g, dev_atoms + (size_t)b * n_atoms, n_atoms, v + b * N);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


// --------------------------------------------------------------- moments
// Q_lm = sum_n w_n S_lm(x_n - c), w_n = m_x,i m_y,j m_z,k rho_n. S_lm is a
// polynomial of degree l, so Q_lm = sum_p c_mono[lm][p] M_p over the 35 raw
// moments M_abc = sum_n w_n x^a y^b z^c, and on the tensor-product mesh
// M_abc = sum_rows (m_y y^b)(m_z z^c) X_a(row), X_a = sum_i m_x,i x_i^a rho.
// A wave takes whole rows (its lanes the nodes i = lane + 64 u, the loads of
// up to 64 MO_AHEAD nodes of a row in flight together); each lane folds its X_a into its 35 M's with the
// row's y-z factors, so no lane-crossing sum is needed until the end. Each
// workgroup then turns its M's into the 25 partials of Q.
constexpr int MO_NT = 256, MO_AHEAD = 6;

__global__ __launch_bounds__(MO_NT) void k_moments(LevelView L, const double* __restrict__ rho, double cx, double cy,
                                                   double cz, double* __restrict__ part)
{
    constexpr int NW = MO_NT / 64;
    __shared__ double sm[NW][kMono];
    __shared__ double mb[kMono];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nx = L.nx, ny = L.ny;
    const int rows = ny * L.nz;   // (node counts fit 32 bits per row index)
    double M[kMono];
#pragma unroll
    for (int p = 0; p < kMono; ++p) M[p] = 0.0;
    for (int row = blockIdx.x * NW + wid; row < rows; row += gridDim.x * NW) {
        const double* rr = rho + (size_t)row * nx;
        double X[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        bool any = false;
        for (int i0 = lane; i0 < nx; i0 += 64 * MO_AHEAD) {
            double f[MO_AHEAD];
#pragma unroll
            for (int u = 0; u < MO_AHEAD; ++u) {
                const int i = i0 + 64 * u;
                f[u] = i < nx ? rr[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < MO_AHEAD; ++u) {
                if (f[u] == 0.0) continue;
                const int i = i0 + 64 * u;
                const double x = L.ax[0].x[i] - cx;
                double t = L.ax[0].m[i] * f[u];
                X[0] += t;
                t *= x; X[1] += t;
                t *= x; X[2] += t;
                t *= x; X[3] += t;
                t *= x; X[4] += t;
                any = true;
            }
        }
        if (!__any(any)) continue;   // (a row of zeros adds nothing)
        const int j = row % ny, k = row / ny;
        const double y = L.ax[1].x[j] - cy, z = L.ax[2].x[k] - cz;
        double Y[5], Z[5];
        Y[0] = L.ax[1].m[j];
        Z[0] = L.ax[2].m[k];
#pragma unroll
        for (int d = 1; d <= 4; ++d) {
            Y[d] = Y[d - 1] * y;
            Z[d] = Z[d - 1] * z;
        }
        int p = 0;
#pragma unroll
        for (int ea = 0; ea <= 4; ++ea)
#pragma unroll
            for (int eb = 0; eb <= 4 - ea; ++eb) {
                const double xy = X[ea] * Y[eb];
#pragma unroll
                for (int ec = 0; ec <= 4 - ea - eb; ++ec) M[p++] += xy * Z[ec];
            }
    }
    // lanes, then waves in order, then the 25 partials of Q
#pragma unroll
    for (int p = 0; p < kMono; ++p) {
        double v = M[p];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sm[wid][p] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMono) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += sm[w][threadIdx.x];
        mb[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x < 25) {
        double q = 0.0;
        for (int p = 0; p < kMono; ++p) q += c_mono[threadIdx.x * kMono + p] * mb[p];
        part[(size_t)blockIdx.x * 25 + threadIdx.x] = q;
    }
}

hipError_t launch_moments(lasto_grid g, const double* rho, double* Q)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    hipLaunchKernelGGL(k_moments, dim3(kReduceBlocks), dim3(MO_NT), 0, g->stream, L, rho, g->box_center[0],
                       g->box_center[1], g->box_center[2], g->partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(g->partials, 25, kReduceBlocks, Q, g->stream);
}

// ---------------------------------------------------------- face values
__global__ __launch_bounds__(256) void k_bc(LevelView L, int mode, const double* __restrict__ Q, int lmax_bc, double cx,
                                            double cy, double cz, double* __restrict__ v)
{
    // face node counts fit 32 bits (the launcher checks): 32-bit index math
    const unsigned nx = L.nx, ny = L.ny, nz = L.nz;
    const unsigned nxy = nx * ny, nxz = nx * nz, nyz = ny * nz;
    const unsigned total = 2 * (nxy + nxz + nyz);
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    unsigned i, j, k;
    unsigned u = t;
    if (u < 2 * nxy) {
        const unsigned face = u / nxy;
        u -= face * nxy;
        j = u / nx; i = u - j * nx; k = face ? nz - 1 : 0;
    } else if ((u -= 2 * nxy) < 2 * nxz) {
        const unsigned face = u / nxz;
        u -= face * nxz;
        k = u / nx; i = u - k * nx; j = face ? ny - 1 : 0;
    } else {
        u -= 2 * nxz;
        const unsigned face = u / nyz;
        u -= face * nyz;
        k = u / ny; j = u - k * ny; i = face ? nx - 1 : 0;
    }
    double val = 0.0;
    if (mode == 1) {
        const double dx = L.ax[0].x[i] - cx, dy = L.ax[1].x[j] - cy, dz = L.ax[2].x[k] - cz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double rinv = 1.0 / sqrt(r2);
        const double r2inv = rinv * rinv;
        // every l <= 4 (the recurrence of each l uses only lower ones, so
        // the values are those of a shorter call), the sum up to lmax_bc
        double S[25];
        solid_harmonics(dx, dy, dz, 4, S);
        double pw = rinv;   // 1/r^(2l+1)
#pragma unroll
        for (int l = 0; l <= 4; ++l) {
            if (l > lmax_bc) break;
            double s = 0.0;
#pragma unroll
            for (int m = -l; m <= l; ++m) s += Q[l * l + l + m] * S[l * l + l + m];
            val -= 4.0 * kPi / (2.0 * l + 1.0) * s * pw;
            pw *= r2inv;
        }
    }
    v[((size_t)k * ny + j) * nx + i] = val;
}

hipError_t launch_bc(lasto_grid g, int mode, const double* Q, int lmax_bc, double* v)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    const size_t total = 2 * ((size_t)L.nx * L.ny + (size_t)L.nx * L.nz + (size_t)L.ny * L.nz);
    if (total >= (size_t)1 << 31) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bc, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, g->stream, L, mode, Q, lmax_bc,
                       g->box_center[0], g->box_center[1], g->box_center[2], v);
    return hipGetLastError();
}

// -------------------------------------------------------- interpolation
__device__ __forceinline__ int upper_bound_dev(const double* x, int n, double p)
{
    int lo = 0, hi = n;   // first index with x[idx] > p
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] <= p) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int window_start(const double* x, int n, double p)
{
    int i0 = upper_bound_dev(x, n, p) - 2;
    if (i0 < 0) i0 = 0;
    if (i0 > n - 4) i0 = n - 4;
    return i0;
}

__device__ __forceinline__ void lagrange_weights(const double* x, int i0, double p, double* w)
{
    const double x0 = x[i0], x1 = x[i0 + 1], x2 = x[i0 + 2], x3 = x[i0 + 3];
    const double d0 = p - x0, d1 = p - x1, d2 = p - x2, d3 = p - x3;
    w[0] = (d1 * d2 * d3) / ((x0 - x1) * (x0 - x2) * (x0 - x3));
    w[1] = (d0 * d2 * d3) / ((x1 - x0) * (x1 - x2) * (x1 - x3));
    w[2] = (d0 * d1 * d3) / ((x2 - x0) * (x2 - x1) * (x2 - x3));
    w[3] = (d0 * d1 * d2) / ((x3 - x0) * (x3 - x1) * (x3 - x2));
}

// tricubic Lagrange value of grid field v (one copy) at point p
__device__ __forceinline__ double interp_point(const LevelView& L, const double* __restrict__ v, double px,
                                              double py, double pz)
{
    const int i0 = window_start(L.ax[0].x, L.nx, px);
    const int j0 = window_start(L.ax[1].x, L.ny, py);
    const int k0 = window_start(L.ax[2].x, L.nz, pz);
    double wx[4], wy[4], wz[4];
    lagrange_weights(L.ax[0].x, i0, px, wx);
    lagrange_weights(L.ax[1].x, j0, py, wy);
    lagrange_weights(L.ax[2].x, k0, pz, wz);
    double s = 0.0;
    for (int c = 0; c < 4; ++c) {
        double sy = 0.0;
        for (int b = 0; b < 4; ++b) {
            const double* row = v + ((size_t)(k0 + c) * L.ny + (j0 + b)) * L.nx + i0;
            sy += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2] + wx[3] * row[3]);
        }
        s += wz[c] * sy;
    }
    return s;
}

__global__ __launch_bounds__(64) void k_interp(LevelView L, const double* __restrict__ v, const double* __restrict__ pts,
                                               int npts, double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    out[t] = interp_point(L, v, pts[3 * t], pts[3 * t + 1], pts[3 * t + 2]);
}

hipError_t launch_interp(lasto_grid g, const double* v, const double* pts, int npts, double* out)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    hipLaunchKernelGGL(k_interp, dim3((npts + 63) / 64), dim3(64), 0, g->stream, L, v, pts, npts, out);
    return hipGetLastError();
}

// ------------------------------------------------------ inside the spheres
// eq. (3.6): V_LM(R) = int V(C + R d) y_LM(d) dOmega by a product rule
// (rule[p] = direction, weight); eq. (3.4): the radial Green's-function
// solution on each atom's logarithmic mesh; and the two parts of the
// integral of V rho over the domain (grid nodes outside every sphere, radial
// quadrature inside).

// C + R d, rounded as written (no fused multiply-add), so the sphere points
// are the products and sums of their definition
__device__ __forceinline__ double axpy_exact(double c, double R, double d)
{
#pragma clang fp contract(off)
    return c + R * d;
}

// |p - C|^2 with each square and sum rounded as written
__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

constexpr int SP_NT = 128;

// one workgroup per (atom, right-hand side): every thread takes points
// p = tid, tid + SP_NT, ..., accumulates w_p V_p y_LM(d_p) for the 25 LM,
// then waves reduce in a fixed order
__global__ __launch_bounds__(SP_NT) void k_sphere_project(LevelView L, const double* __restrict__ v, size_t copy_stride,
                                                          const SphereAtom* __restrict__ atoms, int n_atoms,
                                                          const double4* __restrict__ rule, int npts,
                                                          double* __restrict__ vlmR)
{
    __shared__ double part[SP_NT / 64][25];
    const int a = blockIdx.x, b = blockIdx.y;
    const SphereAtom A = atoms[a];
    const double* vb = v + (size_t)b * copy_stride;
    double acc[25];
    for (int t = 0; t < 25; ++t) acc[t] = 0.0;
    for (int p = threadIdx.x; p < npts; p += SP_NT) {
        const double4 d = rule[p];
        const double val = d.w * interp_point(L, vb, axpy_exact(A.c[0], A.R, d.x), axpy_exact(A.c[1], A.R, d.y),
                                              axpy_exact(A.c[2], A.R, d.z));
        double S[25];
        solid_harmonics(d.x, d.y, d.z, 4, S);   // |d| = 1: r^L y_LM(d) = y_LM(d)
        for (int t = 0; t < 25; ++t) acc[t] += val * S[t];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int t = 0; t < 25; ++t) {
        double s = acc[t];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
        if (lane == 0) part[wid][t] = s;
    }
    __syncthreads();
    if (threadIdx.x < 25) {
        double s = 0.0;
        for (int w = 0; w < SP_NT / 64; ++w) s += part[w][threadIdx.x];
        vlmR[((size_t)b * n_atoms + a) * 25 + threadIdx.x] = s;
    }
}

hipError_t launch_sphere_project(lasto_grid g, const double* v, const SphereAtom* atoms, int n_atoms,
                                 const double4* rule, int npts, double* vlmR)
{
    const LevelView& L = g->cview;
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_sphere_project, dim3(n_atoms, g->n_batch), dim3(SP_NT), 0, g->stream, L, v, N, atoms, n_atoms,
                       rule, npts, vlmR);
    return hipGetLastError();
}

__device__ __forceinline__ int lm_degree(int lm)
{
    return lm < 1 ? 0 : lm < 4 ? 1 : lm < 9 ? 2 : lm < 16 ? 3 : 4;
}

__device__ __forceinline__ double ipow(double r, int e)
{
    double p = 1.0;
    for (int t = 0; t < e; ++t) p *= r;
    return p;
}

// integral over [t_k, t_k+1] of the cubic through four samples of g (uniform
// step D in t = ln r): samples k-1..k+2 inside, 0..3 on the first interval,
// n-4..n-1 on the last
__device__ __forceinline__ double cubic_interval(const double* g, int n, int k, double D)
{
    double s;
    if (k == 0)
        s = 9.0 * g[0] + 19.0 * g[1] - 5.0 * g[2] + g[3];
    else if (k == n - 2)
        s = g[n - 4] - 5.0 * g[n - 3] + 19.0 * g[n - 2] + 9.0 * g[n - 1];
    else
        s = -g[k - 1] + 13.0 * g[k] + 13.0 * g[k + 1] - g[k + 2];
    return D / 24.0 * s;
}

__device__ __forceinline__ double wave_prefix(double x, int lane)
{
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(x, off);
        if (lane >= off) x += t;
    }
    return x;
}

__device__ __forceinline__ double wave_suffix(double x, int lane)
{
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_down(x, off);
        if (lane + off < 64) x += t;
    }
    return x;
}

// Atom a's mesh: r_k = R exp((k - (n-1)) D), k = 0..n-1 (r_0 = r_min, r_(n-1) = R).
__device__ __forceinline__ double radial_node(const SphereAtom& A, int n, int k)
{
    return A.R * exp((double)(k - (n - 1)) * A.D);
}

// One wave per (LM, atom, right-hand side). Interior solution of eq. (3.4):
//   V(r) = V(R) (r/R)^L - 4 pi/(2L+1) [r^-(L+1) P(r) + r^L Q(r) - r^L P(R)/R^(2L+1)]
//          + (L = 0) sqrt(4 pi) Z (1/r - 1/R),
//   P(r) = int_0^r rho r'^(L+2) dr',  Q(r) = int_r^R rho r'^(1-L) dr'.
// In t = ln r the integrands are g1 = rho r^(L+3) and g2 = rho r^(2-L);
// P(r_k) = g1(r_0)/(2L+3) + sum_(j<k) I_j(g1), Q(r_k) = sum_(j>=k) I_j(g2).
// Lane l owns points [l c, l c + c) and the intervals that start there; a
// wave prefix sum of the lanes' P-increments and a suffix sum of their
// Q-increments give each lane its starting values.
__global__ __launch_bounds__(64) void k_radial_solve(const SphereAtom* __restrict__ atoms, int n_atoms, int n,
                                                     const double* __restrict__ vlmR, const double* __restrict__ rho_lm,
                                                     double* __restrict__ v_lm)
{
    extern __shared__ double rs_lds[];   // r, g1, g2, P: n each
    double* r = rs_lds;
    double* g1 = r + n;
    double* g2 = g1 + n;
    double* P = g2 + n;
    const int lm = blockIdx.x, a = blockIdx.y, b = blockIdx.z, lane = threadIdx.x;
    const int L = lm_degree(lm);
    const SphereAtom A = atoms[a];
    const size_t row = ((size_t)b * n_atoms + a) * 25 + lm;
    const double* rho = rho_lm + row * n;
    for (int k = lane; k < n; k += 64) {
        const double rk = radial_node(A, n, k);
        const double rl = ipow(rk, L);
        r[k] = rk;
        g1[k] = rho[k] * (rl * rk * rk * rk);
        g2[k] = rho[k] * (rk * rk / rl);
    }
    __syncthreads();
    const int c = (n + 63) / 64;
    const int lo = min(n, lane * c), hi = min(n, lo + c), ihi = min(hi, n - 1);
    double sI = 0.0, sJ = 0.0;
    for (int k = lo; k < ihi; ++k) {
        sI += cubic_interval(g1, n, k, A.D);
        sJ += cubic_interval(g2, n, k, A.D);
    }
    const double head = g1[0] / (2 * L + 3);
    const double inI = wave_prefix(sI, lane);
    double exI = __shfl_up(inI, 1);
    if (lane == 0) exI = 0.0;
    const double PR = head + __shfl(inI, 63);
    const double inJ = wave_suffix(sJ, lane);
    double exJ = __shfl_down(inJ, 1);
    if (lane == 63) exJ = 0.0;
    double p = head + exI;
    for (int k = lo; k < hi; ++k) {
        P[k] = p;
        if (k < n - 1) p += cubic_interval(g1, n, k, A.D);
    }
    const double cL = 4.0 * kPi / (2 * L + 1);
    const double vR = vlmR[row];
    const double R = A.R;
    const double PRn = PR / ipow(R, 2 * L + 1);
    const double zt = L == 0 ? sqrt(4.0 * kPi) * A.Z : 0.0;
    double q = exJ;
    double* out = v_lm + row * n;
    for (int k = hi - 1; k >= lo; --k) {
        if (k < n - 1) q += cubic_interval(g2, n, k, A.D);
        const double rk = r[k];
        const double rl = ipow(rk, L);
        out[k] = vR * ipow(rk / R, L) - cL * (P[k] / (rl * rk) + rl * q - rl * PRn) + zt * (1.0 / rk - 1.0 / R);
    }
}

hipError_t launch_radial_solve(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* vlmR,
                               const double* rho_lm, double* v_lm)
{
    hipLaunchKernelGGL(k_radial_solve, dim3(25, n_atoms, g->n_batch), dim3(64), sizeof(double) * 4 * n_rad, g->stream,
                       atoms, n_atoms, n_rad, vlmR, rho_lm, v_lm);
    return hipGetLastError();
}

// One wave per (LM, atom, right-hand side): int_0^R V_LM rho_LM r^2 dr, in
// t: g = V rho r^3, the piece [0, r_0] as g(r_0)/3, then the intervals
// (each lane sums its strided intervals, the wave adds the lanes in a fixed
// tree). e_row [n_batch][n_atoms][25].
__global__ __launch_bounds__(64) void k_sphere_energy(const SphereAtom* __restrict__ atoms, int n_atoms, int n,
                                                      const double* __restrict__ v_lm,
                                                      const double* __restrict__ rho_lm, double* __restrict__ e_row)
{
    extern __shared__ double se_lds[];   // [n]
    const int lm = blockIdx.x, a = blockIdx.y, b = blockIdx.z, lane = threadIdx.x;
    const SphereAtom A = atoms[a];
    const size_t row = ((size_t)b * n_atoms + a) * 25 + lm;
    const double* v = v_lm + row * n;
    const double* rho = rho_lm + row * n;
    for (int k = lane; k < n; k += 64) {
        const double rk = radial_node(A, n, k);
        se_lds[k] = v[k] * rho[k] * (rk * rk * rk);
    }
    __syncthreads();
    double s = 0.0;
    for (int k = lane; k < n - 1; k += 64) s += cubic_interval(se_lds, n, k, A.D);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if (lane == 0) e_row[row] = se_lds[0] / 3.0 + s;
}

hipError_t launch_sphere_energy(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* v_lm,
                                const double* rho_lm, double* e_row)
{
    hipLaunchKernelGGL(k_sphere_energy, dim3(25, n_atoms, g->n_batch), dim3(64), sizeof(double) * n_rad, g->stream,
                       atoms, n_atoms, n_rad, v_lm, rho_lm, e_row);
    return hipGetLastError();
}

// Grid part: sum over nodes outside every sphere of vol_n v_n rho_n. A
// workgroup takes EG_NT * EG_PER consecutive nodes of one copy (each wave
// reads 64 consecutive doubles per load); the atoms whose sphere meets the
// bounding box of those nodes are listed first (the box test can only
// under-estimate a node's distance, so no node inside a sphere is missed).
// One partial per workgroup.
constexpr int EG_NT = 256;
constexpr int EG_PER = 8;
constexpr int EG_LIST = 512;

int energy_grid_blocks(const LevelView& L)
{
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    return (int)((N + (size_t)EG_NT * EG_PER - 1) / ((size_t)EG_NT * EG_PER));
}

__global__ __launch_bounds__(EG_NT) void k_energy_grid(LevelView L, const double* __restrict__ v,
                                                       const double* __restrict__ rho, const SphereAtom* __restrict__ atoms,
                                                       int n_atoms, double* __restrict__ partials)
{
    __shared__ int list[EG_LIST];
    __shared__ int wcount[EG_NT / 64];
    __shared__ double wsum[EG_NT / 64];
    __shared__ double box[6];
    const int b = blockIdx.y;
    const unsigned nx = L.nx, ny = L.ny, nz = L.nz, plane = nx * ny, N = plane * nz;
    const unsigned first = blockIdx.x * (unsigned)(EG_NT * EG_PER);
    const unsigned last = min(first + (unsigned)(EG_NT * EG_PER), N) - 1u;
    const double* X = L.ax[0].x;
    const double* Y = L.ax[1].x;
    const double* Zc = L.ax[2].x;
    if (threadIdx.x == 0) {
        const unsigned kf = first / plane, kl = last / plane;
        const unsigned jf = (first - kf * plane) / nx, jl = (last - kl * plane) / nx;
        const unsigned i_f = first - kf * plane - jf * nx, il = last - kl * plane - jl * nx;
        const bool one_plane = kf == kl, one_row = one_plane && jf == jl;
        box[0] = one_row ? X[i_f] : X[0];
        box[1] = one_row ? X[il] : X[nx - 1];
        box[2] = one_plane ? Y[jf] : Y[0];
        box[3] = one_plane ? Y[jl] : Y[ny - 1];
        box[4] = Zc[kf];
        box[5] = Zc[kl];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int count = 0;
    bool all = false;
    for (int a0 = 0; a0 < n_atoms; a0 += EG_NT) {
        const int a = a0 + threadIdx.x;
        bool hit = false;
        if (a < n_atoms) {
            const SphereAtom& A = atoms[a];
            const double ex = fmax(fmax(box[0] - A.c[0], A.c[0] - box[1]), 0.0);
            const double ey = fmax(fmax(box[2] - A.c[1], A.c[1] - box[3]), 0.0);
            const double ez = fmax(fmax(box[4] - A.c[2], A.c[2] - box[5]), 0.0);
            hit = dist2_exact(ex, ey, ez) < A.R * A.R;
        }
        const unsigned long long mask = __ballot(hit);
        if (lane == 0) wcount[wid] = __popcll(mask);
        __syncthreads();
        int off = count;
        for (int w = 0; w < wid; ++w) off += wcount[w];
        if (hit && off + __popcll(mask & ((1ull << lane) - 1ull)) < EG_LIST)
            list[off + __popcll(mask & ((1ull << lane) - 1ull))] = a;
        for (int w = 0; w < EG_NT / 64; ++w) count += wcount[w];
        __syncthreads();
    }
    if (count > EG_LIST) all = true;
    const int na = all ? n_atoms : count;
    const double* vb = v + (size_t)b * N;
    const double* rb = rho + (size_t)b * N;
    double vv[EG_PER], rr[EG_PER];
#pragma unroll
    for (int s = 0; s < EG_PER; ++s) {
        const unsigned n = first + threadIdx.x + s * EG_NT;
        vv[s] = n < N ? vb[n] : 0.0;
        rr[s] = n < N ? rb[n] : 0.0;
    }
    double acc = 0.0;
    // the thread's first node decoded once, then stepped by EG_NT with carries
    unsigned n = first + threadIdx.x;
    unsigned k = n / plane, j = (n - k * plane) / nx, i = n - k * plane - j * nx;
#pragma unroll
    for (int s = 0; s < EG_PER; ++s) {
        if (n < N) {
            const double px = X[i], py = Y[j], pz = Zc[k];
            bool outside = true;
            for (int t = 0; t < na; ++t) {
                const SphereAtom& A = atoms[all ? t : list[t]];
                if (dist2_exact(px - A.c[0], py - A.c[1], pz - A.c[2]) < A.R * A.R) outside = false;
            }
            if (outside) acc += L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] * vv[s] * rr[s];
        }
        n += EG_NT;
        i += EG_NT;
        while (i >= nx) {
            i -= nx;
            if (++j == ny) {
                j = 0;
                ++k;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if (lane == 0) wsum[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < EG_NT / 64; ++w) s += wsum[w];
        partials[(size_t)b * gridDim.x + blockIdx.x] = s;
    }
}

hipError_t launch_energy_grid(lasto_grid g, const double* v, const double* rho, const SphereAtom* atoms, int n_atoms,
                              double* partials)
{
    const LevelView& L = g->cview;
    hipLaunchKernelGGL(k_energy_grid, dim3(energy_grid_blocks(L), g->n_batch), dim3(EG_NT), 0, g->stream, L, v, rho,
                       atoms, n_atoms, partials);
    return hipGetLastError();
}

// The tabulated non-spherical density on the grid: at every node inside a
// sphere, rho += sum_(L >= lmin) rho_LM(r) y_LM, rho_LM by the cubic in
// t = ln r through the four radial samples around t (window start
// clamp(floor((t - t_0)/D) - 1, 0, n - 4)); below r_0, rho_LM(r_0) (r/r_0)^L.
// Workgroups take EG_NT * EG_PER consecutive nodes and the spheres meeting
// their box, as for the energy's grid part.
__global__ __launch_bounds__(EG_NT) void k_sphere_terms(LevelView L, const SphereAtom* __restrict__ atoms, int n_atoms,
                                                        int n, const double* __restrict__ rho_lm, int lmin,
                                                        double* __restrict__ rho)
{
    __shared__ int list[EG_LIST];
    __shared__ int wcount[EG_NT / 64];
    __shared__ double box[6];
    const int b = blockIdx.y;
    const unsigned nx = L.nx, ny = L.ny, nz = L.nz, plane = nx * ny, N = plane * nz;
    const unsigned first = blockIdx.x * (unsigned)(EG_NT * EG_PER);
    const unsigned last = min(first + (unsigned)(EG_NT * EG_PER), N) - 1u;
    const double* X = L.ax[0].x;
    const double* Y = L.ax[1].x;
    const double* Zc = L.ax[2].x;
    if (threadIdx.x == 0) {
        const unsigned kf = first / plane, kl = last / plane;
        const unsigned jf = (first - kf * plane) / nx, jl = (last - kl * plane) / nx;
        const unsigned i_f = first - kf * plane - jf * nx, il = last - kl * plane - jl * nx;
        const bool one_plane = kf == kl, one_row = one_plane && jf == jl;
        box[0] = one_row ? X[i_f] : X[0];
        box[1] = one_row ? X[il] : X[nx - 1];
        box[2] = one_plane ? Y[jf] : Y[0];
        box[3] = one_plane ? Y[jl] : Y[ny - 1];
        box[4] = Zc[kf];
        box[5] = Zc[kl];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int count = 0;
    for (int a0 = 0; a0 < n_atoms; a0 += EG_NT) {
        const int a = a0 + threadIdx.x;
        bool hit = false;
        if (a < n_atoms) {
            const SphereAtom& A = atoms[a];
            const double ex = fmax(fmax(box[0] - A.c[0], A.c[0] - box[1]), 0.0);
            const double ey = fmax(fmax(box[2] - A.c[1], A.c[1] - box[3]), 0.0);
            const double ez = fmax(fmax(box[4] - A.c[2], A.c[2] - box[5]), 0.0);
            hit = dist2_exact(ex, ey, ez) < A.R * A.R;
        }
        const unsigned long long mask = __ballot(hit);
        if (lane == 0) wcount[wid] = __popcll(mask);
        __syncthreads();
        int off = count;
        for (int w = 0; w < wid; ++w) off += wcount[w];
        if (hit && off + __popcll(mask & ((1ull << lane) - 1ull)) < EG_LIST)
            list[off + __popcll(mask & ((1ull << lane) - 1ull))] = a;
        for (int w = 0; w < EG_NT / 64; ++w) count += wcount[w];
        __syncthreads();
    }
    if (count == 0) return;
    const bool all = count > EG_LIST;
    const int na = all ? n_atoms : count;
    double* rb = rho + (size_t)b * N;
    unsigned node = first + threadIdx.x;
    unsigned k = node / plane, j = (node - k * plane) / nx, i = node - k * plane - j * nx;
    for (int s = 0; s < EG_PER; ++s) {
        if (node < N) {
            const double px = X[i], py = Y[j], pz = Zc[k];
            int hit_a = -1;
            double dx = 0.0, dy = 0.0, dz = 0.0, d2 = 0.0;
            for (int t = 0; t < na && hit_a < 0; ++t) {
                const int a = all ? t : list[t];
                const SphereAtom& A = atoms[a];
                const double ex = px - A.c[0], ey = py - A.c[1], ez = pz - A.c[2];
                const double q = dist2_exact(ex, ey, ez);
                if (q < A.R * A.R) {
                    hit_a = a;
                    dx = ex;
                    dy = ey;
                    dz = ez;
                    d2 = q;
                }
            }
            if (hit_a >= 0) {
                const SphereAtom& A = atoms[hit_a];
                const double r = sqrt(d2);
                double S[25];
                solid_harmonics(dx, dy, dz, 4, S);
                const double r0 = radial_node(A, n, 0);
                const double* tab = rho_lm + ((size_t)b * n_atoms + hit_a) * 25 * n;
                double add = 0.0;
                if (r < r0) {
                    double ir0[5] = {1.0, 1.0 / r0, 0.0, 0.0, 0.0};
                    ir0[2] = ir0[1] * ir0[1];
                    ir0[3] = ir0[2] * ir0[1];
                    ir0[4] = ir0[3] * ir0[1];
#pragma unroll
                    for (int lm = 0; lm < 25; ++lm)
                        if (lm >= lmin * lmin) add += tab[(size_t)lm * n] * S[lm] * ir0[lm_degree(lm)];
                } else {
                    const double t0 = log(A.R) - (n - 1) * A.D;
                    const double u0 = (log(r) - t0) / A.D;
                    int i0 = (int)floor(u0) - 1;
                    i0 = i0 < 0 ? 0 : (i0 > n - 4 ? n - 4 : i0);
                    const double u = u0 - i0;
                    const double w0 = -(u - 1) * (u - 2) * (u - 3) / 6.0, w1 = u * (u - 2) * (u - 3) / 2.0;
                    const double w2 = -u * (u - 1) * (u - 3) / 2.0, w3 = u * (u - 1) * (u - 2) / 6.0;
                    double ir[5] = {1.0, 1.0 / r, 0.0, 0.0, 0.0};
                    ir[2] = ir[1] * ir[1];
                    ir[3] = ir[2] * ir[1];
                    ir[4] = ir[3] * ir[1];
#pragma unroll
                    for (int lm = 0; lm < 25; ++lm)
                        if (lm >= lmin * lmin) {
                            const double* tl = tab + (size_t)lm * n + i0;
                            add += (w0 * tl[0] + w1 * tl[1] + w2 * tl[2] + w3 * tl[3]) * S[lm] * ir[lm_degree(lm)];
                        }
                }
                rb[node] += add;
            }
        }
        node += EG_NT;
        i += EG_NT;
        while (i >= nx) {
            i -= nx;
            if (++j == ny) {
                j = 0;
                ++k;
            }
        }
    }
}

hipError_t launch_sphere_terms(lasto_grid g, const SphereAtom* atoms, int n_atoms, int n_rad, const double* rho_lm,
                               int lmin, double* rho)
{
    const LevelView& L = g->cview;
    hipLaunchKernelGGL(k_sphere_terms, dim3(energy_grid_blocks(L), g->n_batch), dim3(EG_NT), 0, g->stream, L, atoms,
                       n_atoms, n_rad, rho_lm, lmin, rho);
    return hipGetLastError();
}

// out[b][0] = sum of the grid partials of copy b, out[b][1] = sum of the
// sphere rows of copy b (fixed orders: strided per thread, then a tree).
__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ partials, int nparts,
                                                      const double* __restrict__ e_row, int nrows,
                                                      double* __restrict__ out)
{
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    double s = 0.0, e = 0.0;
    for (int t = threadIdx.x; t < nparts; t += 256) s += partials[(size_t)b * nparts + t];
    for (int t = threadIdx.x; t < nrows; t += 256) e += e_row[(size_t)b * nrows + t];
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * b] = red[0][0];
        out[2 * b + 1] = red[1][0];
    }
}

hipError_t launch_energy_final(lasto_grid g, const double* partials, int nparts, const double* e_row, int nrows,
                               double* out)
{
    hipLaunchKernelGGL(k_energy_final, dim3(g->n_batch), dim3(256), 0, g->stream, partials, nparts, e_row, nrows, out);
    return hipGetLastError();
}

// -------------------------------------------- interstitial output density
// rho_out(x) = sum_k f_k psi_k(x)^2, psi_k = sum_mu c_(mu,k) phi_mu(x), the
// Slater-type basis phi = r^(n-1) exp(-zeta r) y_lm = r^(n-1-l) exp(-zeta r)
// S_lm(x - C) of eq. (3.13), at the nodes outside every sphere (zero inside).
// psi for 64 nodes x 16 NT states per workgroup is a dense contraction
// (nodes x basis) . (basis x states) on the FP64 matrix cores
// (v_mfma_f64_16x16x4: A 16 x 4 from lane (row = lane % 16, k = lane / 16),
// B 4 x 16 from lane (k = lane / 16, col = lane % 16), D 16 x 16 with lane
// holding rows lane / 16 + 4 j, j = 0..3, of column lane % 16, as measured on
// gfx950). Per atom the
// workgroup stages that atom's coefficient rows in LDS and each wave writes the
// basis values of its 16 nodes to LDS; the squares are summed in registers.
constexpr int ID_NT = 256;
constexpr int ID_PTS = 64;    // nodes per workgroup, 16 per wave

typedef double dbl4v __attribute__((ext_vector_type(4)));

// LDS row of the staged coefficients: 16 NT doubles, plus 16 when NT is even,
// so that the four k-rows one matrix-core operand reads start 32 banks apart
__host__ __device__ constexpr int id_ldb(int nt)
{
    return 16 * nt + ((nt & 1) ? 0 : 16);
}

size_t interstitial_lds_bytes(int nt, int kpa)
{
    return sizeof(double) * ((size_t)kpa * id_ldb(nt) + (size_t)(ID_NT / 64) * 16 * kpa);
}

// PF > 0: the next atom's coefficient rows are fetched into PF registers per
// thread while the current atom's products run (kpa * 16 NT <= PF * ID_NT)
template <int NT, int PF, int LMAX>
__global__ __launch_bounds__(ID_NT) void k_interstitial(LevelView L, const double4* __restrict__ atoms, int n_atoms,
                                                        const double4* __restrict__ shells, int n_shells, int nbpa,
                                                        int kpa, const double* __restrict__ coef, int n_occ, int c0,
                                                        const double* __restrict__ occ, int accumulate,
                                                        double* __restrict__ rho)
{
    constexpr int NC = 16 * NT;
    constexpr int LDB = id_ldb(NT);
    extern __shared__ double id_lds[];
    double* Bs = id_lds;                          // [kpa][LDB] coefficient rows of one atom
    double* Ph = id_lds + (size_t)kpa * LDB;      // [waves][16 nodes][kpa] basis values
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int p16 = lane & 15, grp = lane >> 4;
    const unsigned nx = L.nx, ny = L.ny, plane = nx * ny, N = plane * L.nz;
    const unsigned node0 = blockIdx.x * ID_PTS + wid * 16;
    const unsigned me = min(node0 + p16, N - 1u);
    const unsigned mk = me / plane, mj = (me - mk * plane) / nx, mi = me - mk * plane - mj * nx;
    const double px = L.ax[0].x[mi], py = L.ax[1].x[mj], pz = L.ax[2].x[mk];
    dbl4v acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dbl4v{0.0, 0.0, 0.0, 0.0};
    double* ph = Ph + ((size_t)wid * 16 + p16) * kpa;
    const double* phw = Ph + (size_t)wid * 16 * kpa;
    // staging: wave w takes rows w, w + 4, ..., each lane columns lane,
    // lane + 64, ... (NC is a multiple of 16, so the last pass may be partial)
    constexpr int CPL = (NC + 63) / 64;   // column passes per row
    double pre[PF > 0 ? PF : 1];
    auto fetch = [&](int a) {
        const double* crow = coef + (size_t)a * nbpa * n_occ + c0;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int r = wid + 4 * (q / CPL), c = lane + 64 * (q % CPL);
            pre[q] = (r < nbpa && c < NC && c0 + c < n_occ) ? crow[(size_t)r * n_occ + c] : 0.0;
        }
    };
    if (PF > 0) fetch(0);
    for (int a = 0; a < n_atoms; ++a) {
        __syncthreads();   // the previous atom's products are done with Bs and Ph
        if (PF > 0) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int r = wid + 4 * (q / CPL), c = lane + 64 * (q % CPL);
                if (r < kpa && c < NC) Bs[r * LDB + c] = pre[q];
            }
            if (a + 1 < n_atoms) fetch(a + 1);   // in flight during this atom's work
        } else {
            const double* crow = coef + (size_t)a * nbpa * n_occ + c0;
            for (int r = wid; r < kpa; r += 4)
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    const int c = lane + 64 * q;
                    if (c < NC) Bs[r * LDB + c] = (r < nbpa && c0 + c < n_occ) ? crow[(size_t)r * n_occ + c] : 0.0;
                }
        }
        const double4 A = atoms[a];
        const double dx = px - A.x, dy = py - A.y, dz = pz - A.z;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double S[25];
        solid_harmonics(dx, dy, dz, LMAX, S);   // the shells' largest l is LMAX
        for (int s = grp; s < n_shells; s += 4) {
            const double4 sh = shells[s];   // n, l, offset within the atom, zeta
            const int n = (int)sh.x, l = (int)sh.y, off = (int)sh.z;
            const double radial = ipow(r, n - 1 - l) * exp(-sh.w * r);
#pragma unroll
            for (int ll = 0; ll <= LMAX; ++ll)
                if (ll == l) {
#pragma unroll
                    for (int m = 0; m <= 2 * ll; ++m) ph[off + m] = radial * S[ll * ll + m];
                }
        }
        if (grp == 0)
            for (int q = nbpa; q < kpa; ++q) ph[q] = 0.0;
        __syncthreads();
        for (int ks = 0; ks < kpa; ks += 4) {
            const double av = phw[p16 * kpa + ks + grp];
            const double* brow = Bs + (size_t)(ks + grp) * LDB + p16;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, brow[16 * t], acc[t], 0, 0, 0);
        }
    }
    // rows grp + 4 j of this wave's 16 nodes, state c0 + 16 t + p16
    double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = c0 + 16 * t + p16;
        const double f = col < n_occ ? occ[col] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] += f * (acc[t][j] * acc[t][j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        for (int o = 1; o < 16; o <<= 1) part[j] += __shfl_xor(part[j], o);
    if (p16 < 4) {
        const int j = p16;
        const unsigned node = node0 + grp + 4 * j;
        double val = j == 0 ? part[0] : j == 1 ? part[1] : j == 2 ? part[2] : part[3];
        if (node < N) {
            const unsigned k = node / plane, jj = (node - k * plane) / nx, i = node - k * plane - jj * nx;
            const double qx = L.ax[0].x[i], qy = L.ax[1].x[jj], qz = L.ax[2].x[k];
            for (int a = 0; a < n_atoms; ++a) {
                const double4 A = atoms[a];
                if (dist2_exact(qx - A.x, qy - A.y, qz - A.z) < A.w * A.w) val = 0.0;
            }
            rho[node] = accumulate ? rho[node] + val : val;
        }
    }
}

template <int NT, int PF, int LMAX>
static hipError_t launch_interstitial_kernel(lasto_grid g, const double4* atoms, int n_atoms, const double4* shells,
                                             int n_shells, int nbpa, int kpa, const double* coef, int n_occ, int c0,
                                             const double* occ, int accumulate, double* rho)
{
    const LevelView& L = g->cview;
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    const size_t lds = interstitial_lds_bytes(NT, kpa);
    if (lds > 65536)
        if (hipError_t e = hipFuncSetAttribute((const void*)k_interstitial<NT, PF, LMAX>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            e != hipSuccess)
            return e;
    hipLaunchKernelGGL((k_interstitial<NT, PF, LMAX>), dim3((unsigned)((N + ID_PTS - 1) / ID_PTS)), dim3(ID_NT), lds,
                       g->stream, L, atoms, n_atoms, shells, n_shells, nbpa, kpa, coef, n_occ, c0, occ, accumulate,
                       rho);
    return hipGetLastError();
}

// up to 32 functions per atom (kpa <= 32) the next atom's rows are
// prefetched into registers; more take the plain staging
template <int NT, int LMAX>
static hipError_t launch_interstitial_nt(lasto_grid g, const double4* atoms, int n_atoms, const double4* shells,
                                         int n_shells, int nbpa, int kpa, const double* coef, int n_occ, int c0,
                                         const double* occ, int accumulate, double* rho)
{
    // (more than eight tiles with the prefetch exceed 256 registers per lane)
    // rows per wave (kpa <= 32: 8) times column passes per row
    constexpr int PF = NT <= 8 ? 8 * ((16 * NT + 63) / 64) : 0;
    if (PF > 0 && kpa <= 32)
        return launch_interstitial_kernel<NT, PF, LMAX>(g, atoms, n_atoms, shells, n_shells, nbpa, kpa, coef, n_occ, c0,
                                                        occ, accumulate, rho);
    return launch_interstitial_kernel<NT, 0, LMAX>(g, atoms, n_atoms, shells, n_shells, nbpa, kpa, coef, n_occ, c0,
                                                   occ, accumulate, rho);
}

// The states in chunks of at most LASTO_ID_CHUNK (160: ten column tiles, two
// waves per SIMD; launches of at most eight tiles also prefetch the next
// atom's rows); the first chunk writes rho, the others add.
#ifndef LASTO_ID_CHUNK
#define LASTO_ID_CHUNK 160
#endif
template <int LMAX>
static hipError_t launch_interstitial_l(lasto_grid g, const double4* atoms, int n_atoms, const double4* shells,
                                        int n_shells, int nbpa, const double* coef, int n_occ, const double* occ,
                                        double* rho)
{
    const int kpa = (nbpa + 3) & ~3;
    constexpr int CHUNK = LASTO_ID_CHUNK;
    static_assert(CHUNK % 16 == 0 && CHUNK <= 288, "state chunk: a multiple of 16, at most 288");
    for (int c0 = 0; c0 < n_occ; c0 += CHUNK) {
        const int tiles = std::min(CHUNK / 16, (n_occ - c0 + 15) / 16);
        const int acc = c0 > 0;
        hipError_t e;
#define LASTO_ID_CASE(T) \
    e = launch_interstitial_nt<T, LMAX>(g, atoms, n_atoms, shells, n_shells, nbpa, kpa, coef, n_occ, c0, occ, acc, rho)
        if (tiles <= 1) LASTO_ID_CASE(1);
        else if (tiles <= 2) LASTO_ID_CASE(2);
        else if (tiles <= 4) LASTO_ID_CASE(4);
        else if (tiles <= 6) LASTO_ID_CASE(6);
        else if (tiles <= 8) LASTO_ID_CASE(8);
        else if (tiles <= 10) LASTO_ID_CASE(10);
        else if (tiles <= 12) LASTO_ID_CASE(12);
        else if (tiles <= 14) LASTO_ID_CASE(14);
        else if (tiles <= 16) LASTO_ID_CASE(16);
        else LASTO_ID_CASE(18);
#undef LASTO_ID_CASE
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// harmonics up to l = 3 when no shell goes higher (the Table 1 basis), else 4
hipError_t launch_interstitial(lasto_grid g, const double4* atoms, int n_atoms, const double4* shells, int n_shells,
                               int lmax, int nbpa, const double* coef, int n_occ, const double* occ, double* rho)
{
    if (lmax <= 3) return launch_interstitial_l<3>(g, atoms, n_atoms, shells, n_shells, nbpa, coef, n_occ, occ, rho);
    return launch_interstitial_l<4>(g, atoms, n_atoms, shells, n_shells, nbpa, coef, n_occ, occ, rho);
}

// ------------------------------------------ interstitial matrix elements
// S[mu][nu] = sum_P w_P phi_mu phi_nu, H[mu][nu] = 1/2 sum_P w_P (phi_mu tphi_nu
// + tphi_mu phi_nu), w_P = vol_P at nodes outside every sphere (0 inside),
// tphi = (-1/2 Laplacian + V) phi with the kinetic term in closed form
// (eq. (3.14)). A workgroup owns one 64 x 64 block (rows r0.., columns c0..,
// r0 <= c0) and one chunk of nodes; per batch of 32 nodes it writes w phi and
// w tphi of its rows and phi and tphi of its columns to LDS (one task per
// (node, atom) evaluates that atom's harmonics once), then each wave runs
// its 2 x 2 tiles of 16 x 16 through v_mfma_f64_16x16x4f64 (S: one product;
// H: two into one accumulator). One partial block per workgroup, summed over
// the chunks in a fixed order afterwards.
constexpr int ME_NT = 256;
constexpr int ME_B = 64;     // block of basis functions
constexpr int ME_K = 32;     // nodes per batch
constexpr int ME_LD = ME_B + 1;   // padded LDS row (doubles)

__global__ __launch_bounds__(256) void k_node_weights(LevelView L, const double4* __restrict__ atoms, int n_atoms,
                                                      double* __restrict__ w)
{
    const unsigned nx = L.nx, ny = L.ny, plane = nx * ny, N = plane * L.nz;
    const unsigned node = blockIdx.x * 256u + threadIdx.x;
    if (node >= N) return;
    const unsigned k = node / plane, j = (node - k * plane) / nx, i = node - k * plane - j * nx;
    const double px = L.ax[0].x[i], py = L.ax[1].x[j], pz = L.ax[2].x[k];
    bool outside = true;
    for (int a = 0; a < n_atoms; ++a) {
        const double4 A = atoms[a];
        if (dist2_exact(px - A.x, py - A.y, pz - A.z) < A.w * A.w) outside = false;
    }
    w[node] = outside ? L.ax[0].m[i] * L.ax[1].m[j] * L.ax[2].m[k] : 0.0;
}

hipError_t launch_node_weights(lasto_grid g, const double4* atoms, int n_atoms, double* w)
{
    const LevelView& L = g->cview;
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k_node_weights, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, g->stream, L, atoms, n_atoms, w);
    return hipGetLastError();
}

// -1/2 Laplacian of r^(n-1) exp(-zeta r) y_lm, over S_lm = r^l y_lm (eq. (3.14)):
// 1/2 [(l(l+1) - n(n-1)) r^(n-3-l) + 2 zeta n r^(n-2-l) - zeta^2 r^(n-1-l)] e,
// from p = r^(n-1-l) and ir = 1/r (the first term vanishes for n = l + 1, so
// no power below -1 of r appears)
__device__ __forceinline__ double kinetic_radial(int n, int l, double zeta, double p, double ir, double e)
{
    double t = (-zeta * zeta + 2.0 * zeta * n * ir) * p;
    if (n != l + 1) t += (double)(l * (l + 1) - n * (n - 1)) * p * ir * ir;
    return 0.5 * t * e;
}

template <int LMAX>
__global__ __launch_bounds__(ME_NT) void k_matrix_elements(LevelView L, const double* __restrict__ w,
                                                           const double* __restrict__ v,
                                                           const double4* __restrict__ atoms, int n_atoms,
                                                           const double4* __restrict__ shells, int n_shells, int nbpa,
                                                           int n_basis, const int2* __restrict__ pairs, int n_chunks,
                                                           unsigned chunk_nodes, double* __restrict__ partials)
{
    __shared__ double WPR[ME_K * ME_LD], WTR[ME_K * ME_LD], PC[ME_K * ME_LD], TC[ME_K * ME_LD];
    const int pair = blockIdx.x / n_chunks, chunk = blockIdx.x - pair * n_chunks;
    const int r0 = pairs[pair].x * ME_B, c0 = pairs[pair].y * ME_B;
    const unsigned nx = L.nx, ny = L.ny, plane = nx * ny, N = plane * L.nz;
    const unsigned n_begin = chunk * chunk_nodes, n_end = min(N, n_begin + chunk_nodes);
    // atoms touching the row and the column block
    const int ra0 = r0 / nbpa, ra1 = min(n_atoms - 1, (r0 + ME_B - 1) / nbpa);
    const int ca0 = c0 / nbpa, ca1 = min(n_atoms - 1, (c0 + ME_B - 1) / nbpa);
    const int nra = ra1 - ra0 + 1, nta = nra + (ca1 - ca0 + 1);
    for (int e = threadIdx.x; e < ME_K * ME_LD; e += ME_NT) {
        WPR[e] = 0.0;
        WTR[e] = 0.0;
        PC[e] = 0.0;
        TC[e] = 0.0;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int p16 = lane & 15, grp = lane >> 4;
    const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;   // this wave's 32 x 32 quarter
    dbl4v accS[2][2], accH[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accS[a][b] = dbl4v{0.0, 0.0, 0.0, 0.0};
            accH[a][b] = dbl4v{0.0, 0.0, 0.0, 0.0};
        }
    for (unsigned base = n_begin; base < n_end; base += ME_K) {
        __syncthreads();   // the previous batch's products are done with the tables
        for (int task = threadIdx.x; task < ME_K * nta; task += ME_NT) {
            const int t = task % ME_K, ti = task / ME_K;
            const bool row = ti < nra;
            const int a = row ? ra0 + ti : ca0 + (ti - nra);
            const int lo = row ? r0 : c0;
            const unsigned node = min(base + t, N - 1u);
            const double wt = base + t < n_end ? w[node] : 0.0;
            double* P1 = row ? WPR : PC;
            double* P2 = row ? WTR : TC;
            const unsigned k = node / plane, j = (node - k * plane) / nx, i = node - k * plane - j * nx;
            const double4 A = atoms[a];
            const double dx = L.ax[0].x[i] - A.x, dy = L.ax[1].x[j] - A.y, dz = L.ax[2].x[k] - A.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double vp = v[node];
            double S[25];
            solid_harmonics(dx, dy, dz, LMAX, S);   // the shells' largest l is LMAX
            const double ir = wt != 0.0 ? 1.0 / r : 0.0;
            double zeta_prev = -1.0, e = 0.0;   // consecutive shells of one exponent share exp
            for (int s = 0; s < n_shells; ++s) {
                const double4 sh = shells[s];
                const int n = (int)sh.x, l = (int)sh.y;
                const int mu0 = a * nbpa + (int)sh.z;
                if (mu0 + 2 * l < lo || mu0 >= lo + ME_B) continue;
                // nodes of zero weight (inside a sphere, past the chunk) get zeros
                // on both sides, so no singular column value meets a zero weight
                double phr = 0.0, kr = 0.0;
                if (wt != 0.0) {
                    if (sh.w != zeta_prev) {
                        e = exp(-sh.w * r);
                        zeta_prev = sh.w;
                    }
                    const double p = ipow(r, n - 1 - l);
                    phr = p * e;
                    kr = kinetic_radial(n, l, sh.w, p, ir, e);
                }
                const double f = row ? wt : 1.0;
#pragma unroll
                for (int ll = 0; ll <= LMAX; ++ll)
                    if (ll == l) {
#pragma unroll
                        for (int m = 0; m <= 2 * ll; ++m) {
                            const int col = mu0 + m - lo;
                            if (col >= 0 && col < ME_B) {
                                const double ph = phr * S[ll * ll + m];
                                P1[t * ME_LD + col] = wt != 0.0 ? f * ph : 0.0;
                                P2[t * ME_LD + col] = wt != 0.0 ? f * (kr * S[ll * ll + m] + vp * ph) : 0.0;
                            }
                        }
                    }
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < ME_K; ks += 4) {
            const int kn = ks + grp;
            double aP[2], aT[2], bP[2], bT[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                aP[q] = WPR[kn * ME_LD + wr + 16 * q + p16];
                aT[q] = WTR[kn * ME_LD + wr + 16 * q + p16];
                bP[q] = PC[kn * ME_LD + wc + 16 * q + p16];
                bT[q] = TC[kn * ME_LD + wc + 16 * q + p16];
            }
            // the two H products of a tile are seven instructions apart, so
            // no product waits on the one before it
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    accS[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aP[a], bP[b], accS[a][b], 0, 0, 0);
                    accH[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aP[a], bT[b], accH[a][b], 0, 0, 0);
                }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    accH[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aT[a], bP[b], accH[a][b], 0, 0, 0);
        }
    }
    // partial block: [2][64][64] (S, then H), row-major
    double* out = partials + (size_t)blockIdx.x * 2 * ME_B * ME_B;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int rr = wr + 16 * a + grp + 4 * j, cc = wc + 16 * b + p16;
                out[rr * ME_B + cc] = accS[a][b][j];
                out[ME_B * ME_B + rr * ME_B + cc] = 0.5 * accH[a][b][j];
            }
}

// S and H [n_basis][n_basis] (both triangles) from the partial blocks
__global__ __launch_bounds__(256) void k_matrix_reduce(const double* __restrict__ partials, const int2* __restrict__ pairs,
                                                       int n_chunks, int n_basis, double* __restrict__ S,
                                                       double* __restrict__ H)
{
    const int pair = blockIdx.x;
    const int r0 = pairs[pair].x * ME_B, c0 = pairs[pair].y * ME_B;
    for (int e = threadIdx.x; e < ME_B * ME_B; e += 256) {
        const int rr = e / ME_B, cc = e - rr * ME_B;
        const int mu = r0 + rr, nu = c0 + cc;
        if (mu >= n_basis || nu >= n_basis || (r0 == c0 && rr > cc)) continue;   // a diagonal block: its upper half
        double s = 0.0, h = 0.0;
        for (int c = 0; c < n_chunks; ++c) {
            const double* p = partials + ((size_t)pair * n_chunks + c) * 2 * ME_B * ME_B;
            s += p[e];
            h += p[ME_B * ME_B + e];
        }
        S[(size_t)mu * n_basis + nu] = s;
        S[(size_t)nu * n_basis + mu] = s;
        H[(size_t)mu * n_basis + nu] = h;
        H[(size_t)nu * n_basis + mu] = h;
    }
}

int matrix_block_count(int n_basis)
{
    const int nblk = (n_basis + ME_B - 1) / ME_B;
    return nblk * (nblk + 1) / 2;
}

size_t matrix_partial_doubles(int n_pairs, int n_chunks)
{
    return (size_t)n_pairs * n_chunks * 2 * ME_B * ME_B;
}

hipError_t launch_matrix_elements(lasto_grid g, const double* w, const double* v, const double4* atoms, int n_atoms,
                                  const double4* shells, int n_shells, int lmax, int nbpa, int n_basis,
                                  const int2* pairs, int n_pairs, int n_chunks, double* partials, double* S, double* H)
{
    const LevelView& L = g->cview;
    const size_t N = (size_t)L.nx * L.ny * L.nz;
    const unsigned chunk = (unsigned)((N + n_chunks - 1) / n_chunks);
    if (lmax <= 3)
        hipLaunchKernelGGL(k_matrix_elements<3>, dim3((unsigned)(n_pairs * n_chunks)), dim3(ME_NT), 0, g->stream, L, w,
                           v, atoms, n_atoms, shells, n_shells, nbpa, n_basis, pairs, n_chunks, chunk, partials);
    else
        hipLaunchKernelGGL(k_matrix_elements<4>, dim3((unsigned)(n_pairs * n_chunks)), dim3(ME_NT), 0, g->stream, L, w,
                           v, atoms, n_atoms, shells, n_shells, nbpa, n_basis, pairs, n_chunks, chunk, partials);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    hipLaunchKernelGGL(k_matrix_reduce, dim3(n_pairs), dim3(256), 0, g->stream, partials, pairs, n_chunks, n_basis, S, H);
    return hipGetLastError();
}

}  // namespace lasto
