// Network runtime of the learned initial guess and coarse correction: a
// four-level 3-D U-Net on a node grid's index space (the paper has no learned
// part; this is the learned form grown beside the multigrid solver).
//
//   e0 = relu(conv(x))            level 0, c0 channels (x: 8 input features)
//   e1 = relu(conv_s2(e0))        level 1, c1
//   e2 = relu(conv_s2(e1))        level 2, c2
//   e3 = relu(conv_s2(e2))        level 3, c3
//   m3 = relu(conv(e3))           level 3, c3
//   d2 = relu(conv(m3)); u2 = up(d2) + e2     level 2, c2
//   d1 = relu(conv(u2)); u1 = up(d1) + e1     level 1, c1
//   d0 = relu(conv(u1)); u0 = up(d0) + e0     level 0, c0
//   y  = w . u0 + b               level 0, one FP32 value per node
//
// Level l + 1 has (n + 1) / 2 nodes per axis; conv is 3x3x3 with zero
// padding; conv_s2 samples every other node; up is linear in index space.
// Parameters live as FP32 masters in one flat vector (per convolution
// W[27][cin][cout] then b[cout]; then the head w[c0], b); Adam updates them and
// re-packs the BF16 copies the matrix-core kernels read.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "net_internal.h"

using namespace lasto::net;

namespace {

constexpr int kSplits = 64;     // node shares of the weight-gradient reductions
constexpr int kInFeatures = 8;  // padded input channels

struct Layer {
    int cin, cout, mode;   // forward mode CONV_SAME / CONV_DOWN
    int lin, lout;         // input and output levels
    int kpad, kpad_adj, cin_rows;
    size_t w_off, b_off;   // in the parameter vector
    uint16_t* wp = nullptr;   // packed forward weights [cout][kpad]
    uint16_t* wa = nullptr;   // packed adjoint weights [cin_rows][kpad_adj] (not for layer 0)
};

uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// standard normal deviates by the Box-Muller transform of two uniforms
double normal(uint64_t& s)
{
    const double u1 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * lasto::kPi * u2);
}

}  // namespace

struct lasto_net_s {
    lasto_net_config cfg;
    hipStream_t stream = nullptr;
    int dim[4][3];
    long nvox[4];
    int c[4];
    std::vector<Layer> layers;   // 8 convolutions
    size_t nparam = 0, head_off = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    // activations (BF16 channels-last)
    uint16_t *e[4] = {}, *m3 = nullptr, *d[3] = {}, *u[3] = {};
    // gradients
    uint16_t *du[3] = {}, *gg[8] = {};
    float* y = nullptr;
    uint16_t* xin = nullptr;   // features for the learned guess (allocated on first use)
    float* part = nullptr;
    size_t part_n = 0;
    float* dwt = nullptr;   // [cout][kpad] of the largest layer
    double* lossp = nullptr;
    float* hpart = nullptr;
    int step = 0;
    bool fwd_done = false;
    std::vector<void*> allocs;
};

namespace {

lasto_status net_fail(lasto_status s, const std::string& msg) { return lasto::fail(s, msg); }

#define NCHK(expr)                                                                                      \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return net_fail(LASTO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
lasto_status nalloc(lasto_net n, T** p, size_t count)
{
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return net_fail(LASTO_ERR_ALLOC, "lasto_net: device allocation failed");
    n->allocs.push_back(q);
    *p = (T*)q;
    return LASTO_OK;
}

// the node grid the net runs on (at most its creation size per axis, for
// which every buffer is allocated): level l + 1 has (n + 1) / 2 nodes per axis
void set_dims(lasto_net n, int nx, int ny, int nz)
{
    int nn[3] = {nx, ny, nz};
    for (int l = 0; l < 4; ++l) {
        for (int d = 0; d < 3; ++d) {
            n->dim[l][d] = nn[d];
            nn[d] = (nn[d] + 1) / 2;
        }
        n->nvox[l] = (long)n->dim[l][0] * n->dim[l][1] * n->dim[l][2];
    }
}

ConvGeom fwd_geom(const lasto_net_s* n, const Layer& L)
{
    ConvGeom g;
    g.nx = n->dim[L.lout][0];
    g.ny = n->dim[L.lout][1];
    g.nz = n->dim[L.lout][2];
    g.ix = n->dim[L.lin][0];
    g.iy = n->dim[L.lin][1];
    g.iz = n->dim[L.lin][2];
    g.cin = L.cin;
    g.cout = L.cout;
    g.kpad = L.kpad;
    g.mode = L.mode;
    return g;
}

// the adjoint launch: gradient of the layer's output (lout, cout channels) to
// its input (lin, cin channels)
ConvGeom adj_geom(const lasto_net_s* n, const Layer& L)
{
    ConvGeom g;
    g.nx = n->dim[L.lin][0];
    g.ny = n->dim[L.lin][1];
    g.nz = n->dim[L.lin][2];
    g.ix = n->dim[L.lout][0];
    g.iy = n->dim[L.lout][1];
    g.iz = n->dim[L.lout][2];
    g.cin = L.cout;
    g.cout = L.cin;
    g.kpad = L.kpad_adj;
    g.mode = L.mode == CONV_SAME ? CONV_ADJ : CONV_ADJD;
    return g;
}

lasto_status pack_all(lasto_net n)
{
    for (size_t i = 0; i < n->layers.size(); ++i) {
        const Layer& L = n->layers[i];
        NCHK(launch_pack_weights(n->w + L.w_off, L.cin, L.cout, L.wp, L.kpad, L.wa, L.kpad_adj, L.cin_rows, n->stream));
    }
    return LASTO_OK;
}

void free_net(lasto_net n)
{
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
}

// weight and bias gradients of layer i from its input activation and the
// gradient of its (pre-ReLU) output, into the gradient vector
lasto_status layer_grads(lasto_net n, int i, const uint16_t* in, const uint16_t* gout)
{
    const Layer& L = n->layers[i];
    const ConvGeom g = fwd_geom(n, L);
    NCHK(launch_conv_wgrad(g, in, gout, n->part, kSplits, n->stream));
    NCHK(launch_sum_splits(n->part, kSplits, (long)L.cout * L.kpad, n->dwt, 0, n->stream));
    NCHK(launch_unpack_wgrad(n->dwt, L.cin, L.cout, L.kpad, n->g + L.w_off, n->stream));
    NCHK(launch_chan_sum(gout, n->nvox[L.lout], L.cout, n->part, kSplits, n->stream));
    NCHK(launch_sum_splits(n->part, kSplits, L.cout, n->g + L.b_off, 0, n->stream));
    return LASTO_OK;
}

}  // namespace

extern "C" lasto_status lasto_net_create(const lasto_net_config* cfg, void* hip_stream, lasto_net* out)
{
    if (!cfg || !out) return net_fail(LASTO_ERR_ARG, "lasto_net_create: NULL argument");
    *out = nullptr;
    for (int d = 0; d < 3; ++d)
        if ((&cfg->nx)[d] < 8) return net_fail(LASTO_ERR_ARG, "lasto_net_create: each axis needs >= 8 nodes");
    for (int l = 0; l < 4; ++l)
        if (cfg->ch[l] < 16 || cfg->ch[l] > 64 || cfg->ch[l] % 16)
            return net_fail(LASTO_ERR_ARG, "lasto_net_create: channels must be 16, 32, 48 or 64");
    if (cfg->ch[0] > 16) return net_fail(LASTO_ERR_ARG, "lasto_net_create: level-0 channels must be 16");
    if (!(cfg->rho_scale > 0.0) || !(cfg->pot_scale > 0.0) || !(cfg->h_ref > 0.0) || !(cfg->out_scale > 0.0))
        return net_fail(LASTO_ERR_ARG, "lasto_net_create: scales must be > 0");
    lasto_net n = new lasto_net_s();
    n->cfg = *cfg;
    n->stream = (hipStream_t)hip_stream;
    set_dims(n, cfg->nx, cfg->ny, cfg->nz);
    for (int l = 0; l < 4; ++l) n->c[l] = cfg->ch[l];
    const int* c = n->c;
    // (cin, cout, mode, lin, lout)
    const int spec[8][5] = {{kInFeatures, c[0], CONV_SAME, 0, 0}, {c[0], c[1], CONV_DOWN, 0, 1},
                            {c[1], c[2], CONV_DOWN, 1, 2},       {c[2], c[3], CONV_DOWN, 2, 3},
                            {c[3], c[3], CONV_SAME, 3, 3},       {c[3], c[2], CONV_SAME, 3, 3},
                            {c[2], c[1], CONV_SAME, 2, 2},       {c[1], c[0], CONV_SAME, 1, 1}};
    size_t off = 0, max_part = 0, max_dwt = 0;
    for (int i = 0; i < 8; ++i) {
        Layer L;
        L.cin = spec[i][0];
        L.cout = spec[i][1];
        L.mode = spec[i][2];
        L.lin = spec[i][3];
        L.lout = spec[i][4];
        L.kpad = kpad_of(L.cin);
        L.kpad_adj = kpad_of(L.cout);
        L.cin_rows = (L.cin + 15) / 16 * 16;
        L.w_off = off;
        off += 27 * (size_t)L.cin * L.cout;
        L.b_off = off;
        off += L.cout;
        max_part = std::max(max_part, (size_t)kSplits * L.cout * L.kpad);
        max_dwt = std::max(max_dwt, (size_t)L.cout * L.kpad);
        n->layers.push_back(L);
    }
    n->head_off = off;
    off += c[0] + 1;
    n->nparam = off;
    lasto_status st = LASTO_OK;
    auto A = [&](auto** p, size_t cnt) {
        if (st == LASTO_OK) st = nalloc(n, p, cnt);
    };
    A(&n->w, n->nparam);
    A(&n->m, n->nparam);
    A(&n->v, n->nparam);
    A(&n->g, n->nparam);
    for (Layer& L : n->layers) {
        A(&L.wp, (size_t)L.cout * L.kpad);
        if (&L != &n->layers[0]) A(&L.wa, (size_t)L.cin_rows * L.kpad_adj);
    }
    for (int l = 0; l < 4; ++l) A(&n->e[l], n->nvox[l] * c[l]);
    A(&n->m3, n->nvox[3] * c[3]);
    for (int l = 0; l < 3; ++l) {
        A(&n->d[l], n->nvox[l + 1] * c[l]);   // d_l lives on level l + 1 with c_l channels
        A(&n->u[l], n->nvox[l] * c[l]);
        A(&n->du[l], n->nvox[l] * c[l]);
    }
    // per-layer output gradients (pre-ReLU), on the layer's output level
    for (int i = 0; i < 8; ++i) A(&n->gg[i], n->nvox[n->layers[i].lout] * n->layers[i].cout);
    A(&n->y, n->nvox[0]);
    A(&n->part, std::max(max_part, (size_t)kSplits * 64));
    A(&n->dwt, max_dwt);
    A(&n->lossp, kSplits);
    A(&n->hpart, (size_t)kSplits * (c[0] + 1));
    if (st != LASTO_OK) {
        free_net(n);
        return st;
    }
    n->part_n = max_part;
    // He-normal convolution weights, zero biases, a small head
    std::vector<float> h(n->nparam, 0.0f);
    uint64_t s = cfg->seed;
    for (const Layer& L : n->layers) {
        const double sd = std::sqrt(2.0 / (27.0 * L.cin));
        for (size_t e = 0; e < 27 * (size_t)L.cin * L.cout; ++e) h[L.w_off + e] = (float)(sd * normal(s));
    }
    for (int q = 0; q < c[0]; ++q) h[n->head_off + q] = (float)(0.01 * normal(s));
    if (hipMemcpy(n->w, h.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, sizeof(float) * n->nparam) != hipSuccess ||
        hipMemset(n->v, 0, sizeof(float) * n->nparam) != hipSuccess ||
        hipMemset(n->g, 0, sizeof(float) * n->nparam) != hipSuccess) {
        free_net(n);
        return net_fail(LASTO_ERR_HIP, "lasto_net_create: initial upload failed");
    }
    st = pack_all(n);
    if (st == LASTO_OK && hipStreamSynchronize(n->stream) != hipSuccess) st = net_fail(LASTO_ERR_HIP, "lasto_net_create: sync");
    if (st != LASTO_OK) {
        free_net(n);
        return st;
    }
    *out = n;
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_destroy(lasto_net n)
{
    if (!n) return net_fail(LASTO_ERR_ARG, "lasto_net_destroy: NULL net");
    free_net(n);
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_param_count(lasto_net n, long long* count)
{
    if (!n || !count) return net_fail(LASTO_ERR_ARG, "lasto_net_param_count: NULL argument");
    *count = (long long)n->nparam;
    return LASTO_OK;
}

static lasto_status copy_vec(lasto_net n, float* dev, float* host, long long count, bool to_host, const char* who)
{
    if (!n || !host) return net_fail(LASTO_ERR_ARG, std::string(who) + ": NULL argument");
    if (count != (long long)n->nparam) return net_fail(LASTO_ERR_ARG, std::string(who) + ": count != parameter count");
    NCHK(hipStreamSynchronize(n->stream));
    if (to_host) NCHK(hipMemcpy(host, dev, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    else NCHK(hipMemcpy(dev, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_get_params(lasto_net n, float* host, long long count)
{
    return copy_vec(n, n ? n->w : nullptr, host, count, true, "lasto_net_get_params");
}

extern "C" lasto_status lasto_net_set_params(lasto_net n, const float* host, long long count)
{
    lasto_status st = copy_vec(n, n ? n->w : nullptr, const_cast<float*>(host), count, false, "lasto_net_set_params");
    if (st != LASTO_OK) return st;
    st = pack_all(n);
    if (st != LASTO_OK) return st;
    NCHK(hipStreamSynchronize(n->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_get_grads(lasto_net n, float* host, long long count)
{
    return copy_vec(n, n ? n->g : nullptr, host, count, true, "lasto_net_get_grads");
}

namespace lasto {

// forward pass on the net's stream; y (device, nvox[0] FP32) receives the output
// keep_acts: store every activation the backward pass reads (training);
// otherwise the last up-sampling and the head are fused (inference)
lasto_status net_forward_async(lasto_net n, const uint16_t* x, float* y, bool keep_acts)
{
    const int* c = n->c;
    auto conv = [&](int i, const uint16_t* in, uint16_t* out) -> hipError_t {
        const Layer& L = n->layers[i];
        ConvEpilogue ep;
        ep.bias = n->w + L.b_off;
        ep.relu = 1;
        ep.out_bf16 = out;
        return launch_conv(fwd_geom(n, L), in, L.wp, ep, n->stream);
    };
    NCHK(conv(0, x, n->e[0]));
    NCHK(conv(1, n->e[0], n->e[1]));
    NCHK(conv(2, n->e[1], n->e[2]));
    NCHK(conv(3, n->e[2], n->e[3]));
    NCHK(conv(4, n->e[3], n->m3));
    NCHK(conv(5, n->m3, n->d[2]));
    const int* D = &n->dim[0][0];
    NCHK(launch_upsample_add(n->d[2], D[9], D[10], D[11], n->e[2], n->u[2], D[6], D[7], D[8], c[2], n->stream));
    NCHK(conv(6, n->u[2], n->d[1]));
    NCHK(launch_upsample_add(n->d[1], D[6], D[7], D[8], n->e[1], n->u[1], D[3], D[4], D[5], c[1], n->stream));
    NCHK(conv(7, n->u[1], n->d[0]));
    if (!keep_acts) {
        NCHK(launch_upsample_head(n->d[0], D[3], D[4], D[5], n->e[0], D[0], D[1], D[2], c[0], n->w + n->head_off,
                                  y ? y : n->y, n->stream));
        n->fwd_done = false;
        return LASTO_OK;
    }
    NCHK(launch_upsample_add(n->d[0], D[3], D[4], D[5], n->e[0], n->u[0], D[0], D[1], D[2], c[0], n->stream));
    NCHK(launch_head(n->u[0], n->nvox[0], c[0], n->w + n->head_off, y ? y : n->y, n->stream));
    n->fwd_done = true;
    return LASTO_OK;
}

// Input features of the net at every node of the grid's finest level
// (channels-last BF16, 8 per node):
//   0: rho * rho_scale
//   1..3: log(m_d / h_ref), m_d the dual width along axis d
//   4: v * pot_scale (an initial guess inside, the Dirichlet data on faces)
//   5: 1 on faces, 0 inside;  6, 7: 0
__global__ __launch_bounds__(128) void k_features(LevelView L, const double* __restrict__ rho,
                                                  const double* __restrict__ v, double s_rho, double s_pot,
                                                  float h_ref, uint16_t* __restrict__ x)
{
    const int i = blockIdx.x * 128 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= L.nx) return;
    const size_t e = ((size_t)k * L.ny + j) * L.nx + i;
    const bool face = i == 0 || j == 0 || k == 0 || i == L.nx - 1 || j == L.ny - 1 || k == L.nz - 1;
    // the width channels are rounded to BF16 (8 significant bits), so FP32
    // logarithms carry more than enough precision
    const float inv = 1.0f / h_ref;
    uint4 o;
    o.x = (uint32_t)f2bf((float)(rho[e] * s_rho)) | ((uint32_t)f2bf(logf((float)L.ax[0].m[i] * inv)) << 16);
    o.y = (uint32_t)f2bf(logf((float)L.ax[1].m[j] * inv)) | ((uint32_t)f2bf(logf((float)L.ax[2].m[k] * inv)) << 16);
    o.z = (uint32_t)f2bf((float)(v[e] * s_pot)) | ((uint32_t)f2bf(face ? 1.0f : 0.0f) << 16);
    o.w = 0;
    *(uint4*)(x + e * 8) = o;
}

// The learned guess on a coarse level l of the hierarchy: the features are
// taken at that level's nodes (every coarse node is a fine node: injection of
// rho and v, the level's own dual widths), and the net's output, a correction
// at the coarse nodes, is brought to the finest level by linear
// interpolation in physical coordinates along each axis (the multigrid's
// prolongation composed down the levels). Tables per axis: the fine index of
// each coarse node, and for each fine node its coarse interval and weight.
__global__ __launch_bounds__(128) void k_features_inject(LevelView F, LevelView C, const int* __restrict__ ix,
                                                         const int* __restrict__ iy, const int* __restrict__ iz,
                                                         const double* __restrict__ rho, const double* __restrict__ v,
                                                         double s_rho, double s_pot, float h_ref,
                                                         uint16_t* __restrict__ x)
{
    const int I = blockIdx.x * 128 + threadIdx.x, J = blockIdx.y, K = blockIdx.z;
    if (I >= C.nx) return;
    const size_t e = ((size_t)K * C.ny + J) * C.nx + I;
    const size_t f = ((size_t)iz[K] * F.ny + iy[J]) * F.nx + ix[I];
    const bool face = I == 0 || J == 0 || K == 0 || I == C.nx - 1 || J == C.ny - 1 || K == C.nz - 1;
    const float inv = 1.0f / h_ref;
    uint4 o;
    o.x = (uint32_t)f2bf((float)(rho[f] * s_rho)) | ((uint32_t)f2bf(logf((float)C.ax[0].m[I] * inv)) << 16);
    o.y = (uint32_t)f2bf(logf((float)C.ax[1].m[J] * inv)) | ((uint32_t)f2bf(logf((float)C.ax[2].m[K] * inv)) << 16);
    o.z = (uint32_t)f2bf((float)(v[f] * s_pot)) | ((uint32_t)f2bf(face ? 1.0f : 0.0f) << 16);
    o.w = 0;
    *(uint4*)(x + e * 8) = o;
}

// v += s * (linear interpolation of y from the coarse nodes), interior fine nodes
__global__ __launch_bounds__(128) void k_prolong_add_nat(LevelView F, int cnx, int cny, const int* __restrict__ px,
                                                         const double* __restrict__ wx, const int* __restrict__ py,
                                                         const double* __restrict__ wy, const int* __restrict__ pz,
                                                         const double* __restrict__ wz, const float* __restrict__ y,
                                                         double s, double* __restrict__ v)
{
    const int i = blockIdx.x * 128 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i < 1 || i > F.nx - 2 || j < 1 || j > F.ny - 2 || k < 1 || k > F.nz - 2) return;
    const int I = px[i], J = py[j], K = pz[k];
    const double ax = wx[i], ay = wy[j], az = wz[k];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float* row = y + ((size_t)(K + c) * cny + (J + b)) * cnx + I;
            const double w = (c ? az : 1.0 - az) * (b ? ay : 1.0 - ay);
            acc += w * ((1.0 - ax) * (double)row[0] + ax * (double)row[1]);
        }
    v[((size_t)k * F.ny + j) * F.nx + i] += s * acc;
}

// the level whose node grid the net runs on (0: the finest), -1 if none
static int net_level(lasto_grid g, lasto_net n)
{
    for (int l = 0; l < g->nlev; ++l) {
        const Level& L = g->lev[l];
        if (L.n[0] == n->dim[0][0] && L.n[1] == n->dim[0][1] && L.n[2] == n->dim[0][2]) return l;
    }
    return -1;
}

// device tables of level l against the finest level (built once per level)
static lasto_status coarse_guess_tables(lasto_grid g, int l)
{
    if (g->lg_level == l) return LASTO_OK;
    for (void* p : g->lg_alloc) (void)hipFree(p);
    g->lg_alloc.clear();
    g->lg_level = -1;
    const Level& F = g->lev[0];
    const Level& C = g->lev[l];
    for (int d = 0; d < 3; ++d) {
        const std::vector<double>& xf = F.hx[d];
        const std::vector<double>& xc = C.hx[d];
        const int nf = (int)xf.size(), nc = (int)xc.size();
        std::vector<int> idx(nc), pi(nf);
        std::vector<double> pw(nf);
        for (int I = 0; I < nc; ++I) {
            const auto it = std::lower_bound(xf.begin(), xf.end(), xc[I]);
            if (it == xf.end() || *it != xc[I]) return fail(LASTO_ERR_STATE, "lasto_net: a coarse node is not a fine node");
            idx[I] = (int)(it - xf.begin());
        }
        for (int i = 0, I = 0; i < nf; ++i) {
            while (I + 2 < nc && xc[I + 1] <= xf[i]) ++I;
            pi[i] = I;
            pw[i] = (xf[i] - xc[I]) / (xc[I + 1] - xc[I]);
        }
        int* d_idx = nullptr;
        int* d_pi = nullptr;
        double* d_pw = nullptr;
        if (hipMalloc(&d_idx, sizeof(int) * nc) != hipSuccess || hipMalloc(&d_pi, sizeof(int) * nf) != hipSuccess ||
            hipMalloc(&d_pw, sizeof(double) * nf) != hipSuccess)
            return fail(LASTO_ERR_ALLOC, "lasto_net: coarse guess tables");
        g->lg_alloc.push_back(d_idx);
        g->lg_alloc.push_back(d_pi);
        g->lg_alloc.push_back(d_pw);
        NCHK(hipMemcpy(d_idx, idx.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
        NCHK(hipMemcpy(d_pi, pi.data(), sizeof(int) * nf, hipMemcpyHostToDevice));
        NCHK(hipMemcpy(d_pw, pw.data(), sizeof(double) * nf, hipMemcpyHostToDevice));
        g->lg_idx[d] = d_idx;
        g->lg_pi[d] = d_pi;
        g->lg_pw[d] = d_pw;
    }
    g->lg_level = l;
    return LASTO_OK;
}

lasto_status net_features_async(lasto_grid g, lasto_net n, const double* rho, const double* v, uint16_t* x,
                                double rho_mul)
{
    const LevelView& L = g->cview;   // one right-hand side of a batch
    const int l = net_level(g, n);
    if (l < 0) return fail(LASTO_ERR_ARG, "lasto_net: the net's grid matches no level of the grid");
    if (l == 0) {
        hipLaunchKernelGGL(k_features, dim3((L.nx + 127) / 128, L.ny, L.nz), dim3(128), 0, g->stream, L, rho, v,
                           n->cfg.rho_scale * rho_mul, n->cfg.pot_scale, (float)n->cfg.h_ref, x);
    } else {
        if (lasto_status e = coarse_guess_tables(g, l); e != LASTO_OK) return e;
        LevelView C = g->lev[l].view;
        C.nz = C.nzc;   // one copy
        hipLaunchKernelGGL(k_features_inject, dim3((C.nx + 127) / 128, C.ny, C.nz), dim3(128), 0, g->stream, L, C,
                           g->lg_idx[0], g->lg_idx[1], g->lg_idx[2], rho, v, n->cfg.rho_scale * rho_mul,
                           n->cfg.pot_scale, (float)n->cfg.h_ref, x);
    }
    NCHK(hipGetLastError());
    return LASTO_OK;
}

// the learned correction of one right-hand side: v += out_scale net(features(rho, v)),
// on the finest level or, for a net on a coarse level, interpolated from it
lasto_status net_guess_apply(lasto_grid g, lasto_net n, const double* rho, double* v)
{
    const float* y = nullptr;
    double out_scale = 0.0;
    if (lasto_status st = net_guess_forward(g, n, rho, v, &y, &out_scale); st != LASTO_OK) return st;
    const LevelView& L = g->cview;
    const int l = net_level(g, n);
    if (l == 0) {
        NCHK(launch_add_f32_nat(L, v, y, out_scale, g->stream));
    } else {
        hipLaunchKernelGGL(k_prolong_add_nat, dim3((L.nx + 127) / 128, L.ny, L.nz), dim3(128), 0, g->stream, L,
                           n->dim[0][0], n->dim[0][1], g->lg_pi[0], g->lg_pw[0], g->lg_pi[1], g->lg_pw[1],
                           g->lg_pi[2], g->lg_pw[2], y, out_scale, v);
        NCHK(hipGetLastError());
    }
    return LASTO_OK;
}

// features and forward pass on the grid's stream (the net's own stream is
// synchronised first); *y receives the net's output buffer
lasto_status net_guess_forward(lasto_grid g, lasto_net n, const double* rho, const double* v, const float** y,
                               double* out_scale, double rho_mul)
{
    if (!n->xin) {
        const size_t cap = (size_t)n->cfg.nx * n->cfg.ny * n->cfg.nz;
        if (lasto_status st = nalloc(n, &n->xin, cap * kInFeatures); st != LASTO_OK) return st;
    }
    NCHK(hipStreamSynchronize(n->stream));
    if (lasto_status st = net_features_async(g, n, rho, v, n->xin, rho_mul); st != LASTO_OK) return st;
    hipStream_t keep = n->stream;
    n->stream = g->stream;
    lasto_status st = net_forward_async(n, n->xin, n->y, false);
    n->stream = keep;
    if (st != LASTO_OK) return st;
    *y = n->y;
    *out_scale = n->cfg.out_scale;
    return LASTO_OK;
}

}  // namespace lasto

extern "C" lasto_status lasto_net_features(lasto_grid g, lasto_net n, const double* rho, const double* v, uint16_t* x)
{
    if (!g || !n || !rho || !v || !x) return net_fail(LASTO_ERR_ARG, "lasto_net_features: NULL argument");
    if (lasto_status st = lasto::net_features_async(g, n, rho, v, x, 1.0); st != LASTO_OK) return st;
    NCHK(hipStreamSynchronize(g->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_forward(lasto_net n, const uint16_t* x, float* y)
{
    if (!n || !x || !y) return net_fail(LASTO_ERR_ARG, "lasto_net_forward: NULL argument");
    lasto_status st = lasto::net_forward_async(n, x, y, true);
    if (st != LASTO_OK) return st;
    NCHK(hipMemcpyAsync(n->y, y, sizeof(float) * n->nvox[0], hipMemcpyDeviceToDevice, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    return LASTO_OK;
}

// gradients of sum_v weight[v] (y[v] - target[v])^2 for the last forward
// input; *loss receives that sum
extern "C" lasto_status lasto_net_backward(lasto_net n, const uint16_t* x, const float* target, const float* weight,
                                           double* loss)
{
    if (!n || !x || !target || !weight) return net_fail(LASTO_ERR_ARG, "lasto_net_backward: NULL argument");
    if (!n->fwd_done) return net_fail(LASTO_ERR_STATE, "lasto_net_backward: no forward pass to differentiate");
    const int* c = n->c;
    const int* D = &n->dim[0][0];
    hipStream_t s = n->stream;
    // head: loss, du0 = dL/du0, head-weight gradient
    NCHK(launch_head_loss_bwd(n->u[0], n->nvox[0], c[0], n->w + n->head_off, n->y, target, weight, n->du[0], n->lossp,
                              n->hpart, kSplits, s));
    NCHK(launch_sum_splits(n->hpart, kSplits, c[0] + 1, n->g + n->head_off, 0, s));
    // u0 = up(d0) + e0: layer 7's output gradient is up^T(du0), masked by its ReLU
    NCHK(launch_upsample_adj(n->du[0], D[0], D[1], D[2], n->gg[7], D[3], D[4], D[5], c[0], n->d[0], s));
    if (lasto_status e = layer_grads(n, 7, n->u[1], n->gg[7]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;
        ep.out_bf16 = n->du[1];
        NCHK(launch_conv(adj_geom(n, n->layers[7]), n->gg[7], n->layers[7].wa, ep, s));
    }
    NCHK(launch_upsample_adj(n->du[1], D[3], D[4], D[5], n->gg[6], D[6], D[7], D[8], c[1], n->d[1], s));
    if (lasto_status e = layer_grads(n, 6, n->u[2], n->gg[6]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;
        ep.out_bf16 = n->du[2];
        NCHK(launch_conv(adj_geom(n, n->layers[6]), n->gg[6], n->layers[6].wa, ep, s));
    }
    NCHK(launch_upsample_adj(n->du[2], D[6], D[7], D[8], n->gg[5], D[9], D[10], D[11], c[2], n->d[2], s));
    if (lasto_status e = layer_grads(n, 5, n->m3, n->gg[5]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;   // through layer 5 to m3, masked by m3's ReLU
        ep.mask = n->m3;
        ep.out_bf16 = n->gg[4];
        NCHK(launch_conv(adj_geom(n, n->layers[5]), n->gg[5], n->layers[5].wa, ep, s));
    }
    if (lasto_status e = layer_grads(n, 4, n->e[3], n->gg[4]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;   // to e3
        ep.mask = n->e[3];
        ep.out_bf16 = n->gg[3];
        NCHK(launch_conv(adj_geom(n, n->layers[4]), n->gg[4], n->layers[4].wa, ep, s));
    }
    if (lasto_status e = layer_grads(n, 3, n->e[2], n->gg[3]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;   // to e2: through the stride-2 layer 3 plus the skip into u2
        ep.addend = n->du[2];
        ep.mask = n->e[2];
        ep.out_bf16 = n->gg[2];
        NCHK(launch_conv(adj_geom(n, n->layers[3]), n->gg[3], n->layers[3].wa, ep, s));
    }
    if (lasto_status e = layer_grads(n, 2, n->e[1], n->gg[2]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;
        ep.addend = n->du[1];
        ep.mask = n->e[1];
        ep.out_bf16 = n->gg[1];
        NCHK(launch_conv(adj_geom(n, n->layers[2]), n->gg[2], n->layers[2].wa, ep, s));
    }
    if (lasto_status e = layer_grads(n, 1, n->e[0], n->gg[1]); e != LASTO_OK) return e;
    {
        ConvEpilogue ep;
        ep.addend = n->du[0];
        ep.mask = n->e[0];
        ep.out_bf16 = n->gg[0];
        NCHK(launch_conv(adj_geom(n, n->layers[1]), n->gg[1], n->layers[1].wa, ep, s));
    }
    if (lasto_status e = layer_grads(n, 0, x, n->gg[0]); e != LASTO_OK) return e;
    std::vector<double> lp(kSplits);
    NCHK(hipMemcpyAsync(lp.data(), n->lossp, sizeof(double) * kSplits, hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    double l = 0.0;
    for (double q : lp) l += q;
    if (loss) *loss = l;
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_adam_step(lasto_net n, float lr)
{
    if (!n || !(lr > 0.0f)) return net_fail(LASTO_ERR_ARG, "lasto_net_adam_step: NULL net or lr <= 0");
    n->step++;
    NCHK(launch_adam(n->w, n->m, n->v, n->g, (long)n->nparam, lr, n->step, n->stream));
    if (lasto_status e = pack_all(n); e != LASTO_OK) return e;
    NCHK(hipStreamSynchronize(n->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_train_step(lasto_net n, const uint16_t* x, const float* target, const float* weight,
                                             float lr, double* loss)
{
    if (!n || !x) return net_fail(LASTO_ERR_ARG, "lasto_net_train_step: NULL argument");
    lasto_status st = lasto::net_forward_async(n, x, n->y, true);
    if (st != LASTO_OK) return st;
    st = lasto_net_backward(n, x, target, weight, loss);
    if (st != LASTO_OK) return st;
    return lasto_net_adam_step(n, lr);
}

// ------------------------------------------------------------ checkpoints
// File layout (little-endian): "LASTONET" | u32 version (1) | i32 ch[4] |
// u64 seed | f64 rho_scale, pot_scale, h_ref, out_scale | i32 nx, ny, nz |
// i64 step | u64 nparam | f32 w[nparam] | f32 m[nparam] | f32 v[nparam].
// The masters w and Adam's moments m, v and step count are all the state a
// training step reads besides its data, so a net loaded from a checkpoint
// continues training with the same bits as the net that wrote it.
namespace {

constexpr char kNetMagic[8] = {'L', 'A', 'S', 'T', 'O', 'N', 'E', 'T'};
constexpr uint32_t kNetVersion = 1;

struct NetFileHead {
    char magic[8];
    uint32_t version;
    int32_t ch[4];
    uint64_t seed;
    double rho_scale, pot_scale, h_ref, out_scale;
    int32_t nx, ny, nz;
    int64_t step;
    uint64_t nparam;
};

struct FileCloser {
    FILE* f;
    ~FileCloser()
    {
        if (f) fclose(f);
    }
};

}  // namespace

extern "C" lasto_status lasto_net_save(lasto_net n, const char* path)
{
    if (!n || !path) return net_fail(LASTO_ERR_ARG, "lasto_net_save: NULL argument");
    NCHK(hipStreamSynchronize(n->stream));
    NetFileHead h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kNetMagic, 8);
    h.version = kNetVersion;
    for (int l = 0; l < 4; ++l) h.ch[l] = n->cfg.ch[l];
    h.seed = n->cfg.seed;
    h.rho_scale = n->cfg.rho_scale;
    h.pot_scale = n->cfg.pot_scale;
    h.h_ref = n->cfg.h_ref;
    h.out_scale = n->cfg.out_scale;
    h.nx = n->cfg.nx;
    h.ny = n->cfg.ny;
    h.nz = n->cfg.nz;
    h.step = n->step;
    h.nparam = n->nparam;
    std::vector<float> buf(3 * n->nparam);
    NCHK(hipMemcpy(buf.data(), n->w, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    NCHK(hipMemcpy(buf.data() + n->nparam, n->m, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    NCHK(hipMemcpy(buf.data() + 2 * n->nparam, n->v, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    const std::string tmp = std::string(path) + ".tmp";
    {
        FileCloser fc{fopen(tmp.c_str(), "wb")};
        if (!fc.f) return net_fail(LASTO_ERR_ARG, "lasto_net_save: cannot open " + tmp);
        if (fwrite(&h, sizeof(h), 1, fc.f) != 1 || fwrite(buf.data(), sizeof(float), buf.size(), fc.f) != buf.size())
            return net_fail(LASTO_ERR_STATE, "lasto_net_save: write failed");
        if (fclose(fc.f) != 0) {
            fc.f = nullptr;
            return net_fail(LASTO_ERR_STATE, "lasto_net_save: write failed");
        }
        fc.f = nullptr;
    }
    if (std::rename(tmp.c_str(), path) != 0) return net_fail(LASTO_ERR_STATE, "lasto_net_save: rename failed");
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_load(lasto_net n, const char* path)
{
    if (!n || !path) return net_fail(LASTO_ERR_ARG, "lasto_net_load: NULL argument");
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return net_fail(LASTO_ERR_ARG, std::string("lasto_net_load: cannot open ") + path);
    NetFileHead h;
    if (fread(&h, sizeof(h), 1, fc.f) != 1 || std::memcmp(h.magic, kNetMagic, 8) != 0 || h.version != kNetVersion)
        return net_fail(LASTO_ERR_ARG, "lasto_net_load: not a net checkpoint of this version");
    for (int l = 0; l < 4; ++l)
        if (h.ch[l] != n->cfg.ch[l]) return net_fail(LASTO_ERR_ARG, "lasto_net_load: channel counts differ");
    if (h.nparam != n->nparam) return net_fail(LASTO_ERR_ARG, "lasto_net_load: parameter count differs");
    if (!(h.rho_scale > 0.0) || !(h.pot_scale > 0.0) || !(h.h_ref > 0.0) || !(h.out_scale > 0.0) || h.step < 0)
        return net_fail(LASTO_ERR_ARG, "lasto_net_load: corrupt header");
    std::vector<float> buf(3 * n->nparam);
    if (fread(buf.data(), sizeof(float), buf.size(), fc.f) != buf.size())
        return net_fail(LASTO_ERR_ARG, "lasto_net_load: truncated file");
    char extra;
    if (fread(&extra, 1, 1, fc.f) != 0) return net_fail(LASTO_ERR_ARG, "lasto_net_load: trailing bytes");
    NCHK(hipStreamSynchronize(n->stream));
    NCHK(hipMemcpy(n->w, buf.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    NCHK(hipMemcpy(n->m, buf.data() + n->nparam, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    NCHK(hipMemcpy(n->v, buf.data() + 2 * n->nparam, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    // the grid size the net runs on is the caller's; the weights, moments,
    // step, seed and feature scales are the checkpoint's
    n->cfg.seed = h.seed;
    n->cfg.rho_scale = h.rho_scale;
    n->cfg.pot_scale = h.pot_scale;
    n->cfg.h_ref = h.h_ref;
    n->cfg.out_scale = h.out_scale;
    n->step = (int)h.step;
    if (lasto_status e = pack_all(n); e != LASTO_OK) return e;
    NCHK(hipStreamSynchronize(n->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_get_config(lasto_net n, lasto_net_config* cfg, long long* step)
{
    if (!n || !cfg) return net_fail(LASTO_ERR_ARG, "lasto_net_get_config: NULL argument");
    *cfg = n->cfg;
    if (step) *step = n->step;
    return LASTO_OK;
}

// ------------------------------------------------------------ test access
// The stored BF16 tensors of the last forward (with activations kept) and
// backward pass, for checking each kernel on exactly the operands it read.
extern "C" lasto_status lasto_net_tensor(lasto_net n, int which, uint16_t* out, long long count, int* dims)
{
    if (!n || !dims) return net_fail(LASTO_ERR_ARG, "lasto_net_tensor: NULL argument");
    const uint16_t* src = nullptr;
    int level = 0, ch = 0;
    if (which >= LASTO_NET_E0 && which <= LASTO_NET_E3) {
        level = which - LASTO_NET_E0;
        ch = n->c[level];
        src = n->e[level];
    } else if (which == LASTO_NET_M3) {
        level = 3;
        ch = n->c[3];
        src = n->m3;
    } else if (which >= LASTO_NET_D2 && which <= LASTO_NET_D0) {
        const int l = 2 - (which - LASTO_NET_D2);   // d_l lives on level l + 1 with ch[l] channels
        level = l + 1;
        ch = n->c[l];
        src = n->d[l];
    } else if (which >= LASTO_NET_U2 && which <= LASTO_NET_U0) {
        const int l = 2 - (which - LASTO_NET_U2);
        level = l;
        ch = n->c[l];
        src = n->u[l];
    } else if (which >= LASTO_NET_G0 && which <= LASTO_NET_G7) {
        const Layer& L = n->layers[which - LASTO_NET_G0];
        level = L.lout;
        ch = L.cout;
        src = n->gg[which - LASTO_NET_G0];
    } else if (which >= LASTO_NET_DU0 && which <= LASTO_NET_DU2) {
        level = which - LASTO_NET_DU0;
        ch = n->c[level];
        src = n->du[level];
    } else {
        return net_fail(LASTO_ERR_ARG, "lasto_net_tensor: unknown tensor");
    }
    dims[0] = n->dim[level][0];
    dims[1] = n->dim[level][1];
    dims[2] = n->dim[level][2];
    dims[3] = ch;
    const long long size = (long long)n->nvox[level] * ch;
    if (!out) return LASTO_OK;   // dims only
    if (count != size) return net_fail(LASTO_ERR_ARG, "lasto_net_tensor: count != the tensor's size");
    NCHK(hipMemcpyAsync(out, src, sizeof(uint16_t) * size, hipMemcpyDeviceToDevice, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    return LASTO_OK;
}

extern "C" lasto_status lasto_net_set_grid(lasto_net n, int nx, int ny, int nz)
{
    if (!n) return net_fail(LASTO_ERR_ARG, "lasto_net_set_grid: NULL net");
    if (nx < 8 || ny < 8 || nz < 8 || nx > n->cfg.nx || ny > n->cfg.ny || nz > n->cfg.nz)
        return net_fail(LASTO_ERR_ARG, "lasto_net_set_grid: each axis must be 8 .. the net's creation size");
    NCHK(hipStreamSynchronize(n->stream));
    set_dims(n, nx, ny, nz);
    n->fwd_done = false;
    return LASTO_OK;
}

// -------------------------------------------- learned coarse correction
// Inside a V-cycle, at one coarse level c: the net reads the restricted
// residual f_c (scaled to unit RMS s = ||f_c||_W / sqrt(sum vol)) and the
// level's spacings, and proposes the correction e^ = s out_scale net(f_c / s)
// of A_c e = f_c. It becomes the start of the level's own cycle only if it
// lowers the residual, ||f_c - A_c e^||_W < ||f_c||_W (the residual of the
// zero start); otherwise the cycle starts from zero as without the net. The
// test runs on the device (no host read inside the cycle).
namespace lasto {

template <typename T>
__global__ __launch_bounds__(128) void k_lc_features(LevelView L, const T* __restrict__ f,
                                                     const double* __restrict__ scal, double inv_vol, double rho_scale,
                                                     float h_ref, uint16_t* __restrict__ x)
{
    const int i = blockIdx.x * 128 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= L.nx) return;
    const double sr = sqrt(scal[S_LC_R] * inv_vol);
    const double mul = sr > 0.0 ? rho_scale / sr : 0.0;
    const size_t e = ((size_t)k * L.ny + j) * L.nx + i;
    const bool face = i == 0 || j == 0 || k == 0 || i == L.nx - 1 || j == L.ny - 1 || k == L.nz - 1;
    const double fv = face ? 0.0 : (double)f[sidx(L, i, j, k)];
    const float inv = 1.0f / h_ref;
    uint4 o;
    o.x = (uint32_t)f2bf((float)(fv * mul)) | ((uint32_t)f2bf(logf((float)L.ax[0].m[i] * inv)) << 16);
    o.y = (uint32_t)f2bf(logf((float)L.ax[1].m[j] * inv)) | ((uint32_t)f2bf(logf((float)L.ax[2].m[k] * inv)) << 16);
    o.z = (uint32_t)f2bf(face ? 1.0f : 0.0f) << 16;
    o.w = 0;
    *(uint4*)(x + e * 8) = o;
}

// u = s out_scale y at interior nodes, zero on faces (split layout)
template <typename T>
__global__ __launch_bounds__(128) void k_lc_candidate(LevelView L, const float* __restrict__ y,
                                                      const double* __restrict__ scal, double inv_vol,
                                                      double out_scale, T* __restrict__ u)
{
    const int i = blockIdx.x * 128 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= L.nx) return;
    const bool face = i == 0 || j == 0 || k == 0 || i == L.nx - 1 || j == L.ny - 1 || k == L.nz - 1;
    const double sr = sqrt(scal[S_LC_R] * inv_vol);
    const double val = face ? 0.0 : sr * out_scale * (double)y[((size_t)k * L.ny + j) * L.nx + i];
    u[sidx(L, i, j, k)] = (T)val;
}

// keep u if ||f - A u||_W < ||f||_W, else zero it; count acceptances
template <typename T>
__global__ __launch_bounds__(256) void k_lc_select(T* __restrict__ u, size_t n, double* __restrict__ scal)
{
    const double r = scal[S_LC_R], e = scal[S_LC_E];
    const bool keep = e < r;   // false for NaN
    if (blockIdx.x == 0 && threadIdx.x == 0 && keep) scal[S_LC_ACC] += 1.0;
    if (keep) return;
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (size_t)gridDim.x * 256) u[t] = T(0);
}

// sum of the dual volumes over the interior of a level
static double interior_volume(const Level& L)
{
    double v = 1.0;
    for (int d = 0; d < 3; ++d) {
        const std::vector<double>& x = L.hx[d];
        v *= 0.5 * (x[x.size() - 1] + x[x.size() - 2]) - 0.5 * (x[0] + x[1]);
    }
    return v;
}

lasto_status net_capacity(lasto_net n, int* out)
{
    if (!n) return fail(LASTO_ERR_ARG, "lasto_net: NULL net");
    out[0] = n->cfg.nx;
    out[1] = n->cfg.ny;
    out[2] = n->cfg.nz;
    return LASTO_OK;
}

template <typename T>
lasto_status learned_coarse_start(lasto_grid g, int l, const T* f, T* u, T* r)
{
    lasto_net n = g->lc_net;
    Level& Lv = g->lev[l];
    const LevelView& V = Lv.view;
    hipStream_t s = g->stream;
    const double inv_vol = 1.0 / interior_volume(Lv);
    // ||f||_W^2
    NCHK(launch_dot<T>(V, f, f, g->partials, s));
    NCHK(launch_reduce(g->partials, 1, row_blocks(V), g->scalars + S_LC_R, s));
    if (!n->xin) {
        const size_t cap = (size_t)n->cfg.nx * n->cfg.ny * n->cfg.nz;
        if (lasto_status st = nalloc(n, &n->xin, cap * kInFeatures); st != LASTO_OK) return st;
    }
    set_dims(n, V.nx, V.ny, V.nz);
    const dim3 grid3((V.nx + 127) / 128, V.ny, V.nz);
    hipLaunchKernelGGL(k_lc_features<T>, grid3, dim3(128), 0, s, V, f, (const double*)g->scalars, inv_vol,
                       n->cfg.rho_scale, (float)n->cfg.h_ref, n->xin);
    NCHK(hipGetLastError());
    hipStream_t keep = n->stream;
    n->stream = s;
    lasto_status st = net_forward_async(n, n->xin, n->y, false);
    n->stream = keep;
    if (st != LASTO_OK) return st;
    hipLaunchKernelGGL(k_lc_candidate<T>, grid3, dim3(128), 0, s, V, (const float*)n->y, (const double*)g->scalars,
                       inv_vol, n->cfg.out_scale, u);
    NCHK(hipGetLastError());
    // ||f - A e^||_W^2 (r is the level's residual scratch: zero again afterwards)
    NCHK(launch_residual_colour<T>(V, u, f, r, 0, s));
    NCHK(launch_residual_colour<T>(V, u, f, r, 1, s));
    NCHK(launch_dot<T>(V, r, r, g->partials, s));
    NCHK(launch_reduce(g->partials, 1, row_blocks(V), g->scalars + S_LC_E, s));
    NCHK(launch_fill_zero<T>(r, split_elems(V), s));
    const size_t ne = split_elems(V);
    const unsigned nbk = (unsigned)std::min<size_t>((ne + 255) / 256, 2048);
    hipLaunchKernelGGL(k_lc_select<T>, dim3(nbk), dim3(256), 0, s, u, ne, g->scalars);
    NCHK(hipGetLastError());
    g->lc_applied++;
    return LASTO_OK;
}

template lasto_status learned_coarse_start<float>(lasto_grid, int, const float*, float*, float*);
template lasto_status learned_coarse_start<double>(lasto_grid, int, const double*, double*, double*);

// natural FP32 copy of a split FP64 level array (faces included)
__global__ __launch_bounds__(128) void k_split_to_f32_nat(LevelView L, const double* __restrict__ a, float* __restrict__ t)
{
    const int i = blockIdx.x * 128 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i >= L.nx) return;
    t[((size_t)k * L.ny + j) * L.nx + i] = (float)a[sidx(L, i, j, k)];
}

__global__ __launch_bounds__(256) void k_scale_f32(float* __restrict__ t, long n, double mul)
{
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) t[e] = (float)(t[e] * mul);
}

static hipError_t launch_split_to_f32_nat(const LevelView& L, const double* a, float* t, hipStream_t s)
{
    hipLaunchKernelGGL(k_split_to_f32_nat, dim3((L.nx + 127) / 128, L.ny, L.nz), dim3(128), 0, s, L, a, t);
    return hipGetLastError();
}

static hipError_t launch_scale_f32(float* t, long n, double mul, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, s, t, n, mul);
    return hipGetLastError();
}

// Training pair of the coarse net at level c for iterate v: the restricted
// residual the cycle's descent produces there (nu1 pre-smoothing sweeps from
// zero on each finer level, red residual, restriction) and the solution of
// A_c e = f_c by `cycles` V-cycles of level c (FP64).
lasto_status coarse_pair(lasto_grid g, lasto_net n, const double* rho, const double* v, int c, int nu1, int cycles,
                         uint16_t* x, float* t, double* r_scale)
{
    hipStream_t s = g->stream;
    const LevelView& V0 = g->lev[0].view;
    NCHK(launch_residual_nat(V0, v, rho, 4.0 * kPi, g->r, g->partials, 0, s));
    const double* f = g->r;
    for (int l = 0; l < c; ++l) {
        const LevelView& V = g->lev[l].view;
        double* u = l == 0 ? g->z : g->lev[l].u64;
        for (int k = 0; k < nu1; ++k) {
            NCHK(launch_half<double>(V, u, f, 0, k == 0, 1.0, nullptr, s, nullptr, 0));
            NCHK(launch_half<double>(V, u, f, 1, 0, 1.0, nullptr, s, nullptr, 0));
        }
        NCHK(launch_residual_colour<double>(V, u, f, g->lev[l].r64, 0, s));
        NCHK(launch_restrict_red<double>(V, g->lev[l + 1].view, g->lev[l].r64, g->lev[l + 1].f64, s));
        f = g->lev[l + 1].f64;
    }
    Level& Lc = g->lev[c];
    const LevelView& Vc = Lc.view;
    if (lasto_status e = coarse_cycles(g, c, cycles, Lc.f64, Lc.u64); e != LASTO_OK) return e;
    NCHK(launch_dot<double>(Vc, Lc.f64, Lc.f64, g->partials, s));
    NCHK(launch_reduce(g->partials, 1, row_blocks(Vc), g->scalars + S_LC_R, s));
    const double inv_vol = 1.0 / interior_volume(Lc);
    set_dims(n, Vc.nx, Vc.ny, Vc.nz);
    const dim3 grid3((Vc.nx + 127) / 128, Vc.ny, Vc.nz);
    hipLaunchKernelGGL(k_lc_features<double>, grid3, dim3(128), 0, s, Vc, (const double*)Lc.f64,
                       (const double*)g->scalars, inv_vol, n->cfg.rho_scale, (float)n->cfg.h_ref, x);
    NCHK(hipGetLastError());
    // the target e_c / (s out_scale) in natural layout, zero on faces
    NCHK(launch_split_to_f32_nat(Vc, Lc.u64, t, s));
    double sr2 = 0.0;
    NCHK(hipMemcpyAsync(&sr2, g->scalars + S_LC_R, sizeof(double), hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    const double sr = std::sqrt(sr2 * inv_vol);
    if (!(sr > 0.0) || !std::isfinite(sr)) return fail(LASTO_ERR_ARG, "lasto_coarse_pair: zero residual");
    NCHK(launch_scale_f32(t, (long)Vc.nx * Vc.ny * Vc.nz, 1.0 / (sr * n->cfg.out_scale), s));
    // the solver's vectors go back with zero faces and padding (and zero)
    for (int l = 0; l <= c; ++l) {
        const LevelView& V = g->lev[l].view;
        NCHK(launch_fill_zero<double>(l == 0 ? g->z : g->lev[l].u64, split_elems(V), s));
        NCHK(launch_fill_zero<double>(g->lev[l].r64, split_elems(V), s));
        if (l > 0) NCHK(launch_fill_zero<double>(g->lev[l].f64, split_elems(V), s));
    }
    NCHK(launch_fill_zero<double>(g->r, split_elems(V0), s));
    NCHK(hipStreamSynchronize(s));
    *r_scale = sr;
    return LASTO_OK;
}

}  // namespace lasto

extern "C" lasto_status lasto_coarse_pair(lasto_grid g, lasto_net n, const double* rho, const double* v, int level,
                                          int nu1, uint16_t* x, float* target, double* r_scale, int* dims)
{
    if (!g || !n || !rho || !v || !x || !target || !r_scale || !dims)
        return net_fail(LASTO_ERR_ARG, "lasto_coarse_pair: NULL argument");
    if (g->n_batch != 1) return net_fail(LASTO_ERR_ARG, "lasto_coarse_pair: one right-hand side per grid");
    if (level < 1 || level >= g->nlev || nu1 < 1 || nu1 > 16)
        return net_fail(LASTO_ERR_ARG, "lasto_coarse_pair: level must be 1 .. levels - 1, nu1 1 .. 16");
    const lasto::LevelView& Vc = g->lev[level].view;
    if (Vc.nx < 8 || Vc.ny < 8 || Vc.nz < 8 || Vc.nx > n->cfg.nx || Vc.ny > n->cfg.ny || Vc.nz > n->cfg.nz)
        return net_fail(LASTO_ERR_ARG, "lasto_coarse_pair: the level does not fit the net (8 .. its size per axis)");
    NCHK(hipStreamSynchronize(n->stream));
    dims[0] = Vc.nx;
    dims[1] = Vc.ny;
    dims[2] = Vc.nz;
    return lasto::coarse_pair(g, n, rho, v, level, nu1, 40, x, target, r_scale);
}
