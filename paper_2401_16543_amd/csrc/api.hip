// C-ABI of the KFVM-WENO library: context life cycle, argument checking,
// workspace ownership and dispatch to the HIP kernels.  See include/kfvm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kfvm.h"
#include "kernels.hpp"
#include "stencil.hpp"

struct kfvm_ctx {
    int dim = 0, R = 0, nvar = 0;
    kfvm::Geom geom{};
    kfvm::Limiter lim{1, 0.5, 0.0};
    int riemann = KFVM_HLLC;
    int precision = KFVM_FP64;
    int checking = 0;
    hipStream_t stream = nullptr;
    double *d_tables = nullptr;
    double *d_wch = nullptr;          // chunk-major copy of the tables (3D R = 3 FP64 path)
    kfvm::Work work{};
    double *d_dt = nullptr;
    double min_rho = NAN, min_p = NAN;       // of the state of the last kfvm_cfl_dt
    double *cfl_scratch = nullptr;           // device address of the static CFL scratch on this context's GPU
    std::vector<void *> allocs;
    std::string msg;
    // per-kernel timing (kfvm_set_timing): event pairs per launch, summed on query
    int timing = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
    hipEvent_t pending[kfvm::KT_COUNT] = {};
    // split-precision path
    std::vector<double> host_tables;
    uint4 *d_mix_full = nullptr, *d_mix_lin = nullptr;
    int mix_sw = 0, mix_mode = -1;
    // learned gate (fused into the split-precision reconstruction)
    uint4 *d_gate_w = nullptr;
    uint8_t *d_gate_raw = nullptr;   // per-cell decision bits ahead of dilation (3D order 7)
    float *d_gate_vec = nullptr;
    uint8_t *d_flags_out = nullptr;
    float gate_thr = 0.f;
    int gate_on = 0;
    // gate-network training workspace
    float *d_mlp_ws = nullptr;
    size_t mlp_ws_floats = 0;
    // KXRCF indicator (two-pass reconstruction)
    int indicator = KFVM_IND_NONE;
    double kx_m = 1.5;
    double *d_kx_w = nullptr;       // S0 face rows as [axis][side][member][Gauss point]
    double *d_kx_jump = nullptr;    // [dim][ncell] largest entropy jump on each upper face
    double *d_kx_jlo = nullptr;     // [dim][plane] jumps on the lower faces of non-periodic boundaries
    const uint8_t *last_flags = nullptr;   // the per-(variable, cell) choices of the last reconstruction
    int recon_done = 0;                    // a reconstruction has filled the limiter factors
};

namespace {

thread_local std::string g_init_msg;

int fail(kfvm_ctx *c, int code, const std::string &m)
{
    if (c) c->msg = m; else g_init_msg = m;
    return code;
}

int hip_fail(kfvm_ctx *c, hipError_t e, const char *where)
{
    return fail(c, KFVM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                           \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);     \
    } while (0)

template <int D, int R>
bool layout_matches(const kfvm_weights *w)
{
    constexpr kfvm::Stencil<D, R> st{};
    using S = kfvm::Stencil<D, R>;
    if (w->dim != D || w->R != R || w->n0 != S::N0 || w->n_stencils != S::NST) return false;
    if (w->n_pts != S::NPTS || w->n_der != S::NDER) return false;
    if (!w->offsets || !w->stencil_ptr || !w->members || !w->tables) return false;
    for (int h = 0; h < S::N0; ++h)
        for (int a = 0; a < D; ++a)
            if (w->offsets[h * D + a] != st.off[h][a]) return false;
    if (w->stencil_ptr[0] != 0) return false;
    for (int q = 0; q < S::NST; ++q) {
        if (w->stencil_ptr[q + 1] - w->stencil_ptr[q] != st.nmem[q]) return false;
        for (int j = 0; j < st.nmem[q]; ++j)
            if (w->members[w->stencil_ptr[q] + j] != st.mem[q][j]) return false;
    }
    return true;
}

bool layout_matches(int dim, int R, const kfvm_weights *w)
{
    if (dim == 2 && R == 2) return layout_matches<2, 2>(w);
    if (dim == 2 && R == 3) return layout_matches<2, 3>(w);
    if (dim == 3 && R == 2) return layout_matches<3, 2>(w);
    if (dim == 3 && R == 3) return layout_matches<3, 3>(w);
    return false;
}

int npts_of(int dim, int R)
{
    if (dim == 2 && R == 2) return kfvm::Stencil<2, 2>::NPTS;
    if (dim == 2 && R == 3) return kfvm::Stencil<2, 3>::NPTS;
    if (dim == 3 && R == 2) return kfvm::Stencil<3, 2>::NPTS;
    return kfvm::Stencil<3, 3>::NPTS;
}

int alloc(kfvm_ctx *c, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    c->allocs.push_back(*p);
    return KFVM_OK;
}

int sync_check(kfvm_ctx *c)
{
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int err = 0;
    HIP_TRY(c, hipMemcpy(&err, c->work.err, sizeof(int), hipMemcpyDeviceToHost));
    if (err != 0) {
        int zero = 0;
        HIP_TRY(c, hipMemcpy(c->work.err, &zero, sizeof(int), hipMemcpyHostToDevice));
        return fail(c, err, "non-physical state (rho <= 0, p <= 0 or non-finite) met on the device");
    }
    return KFVM_OK;
}

uint16_t to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}

double from_bf16(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

uint16_t to_f16(double x)
{
    _Float16 h = (_Float16)x;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

double from_f16(uint16_t u)
{
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return (double)h;
}

// Lay the float64 tables out as matrix-core operands (see rhs_mixed.hip):
// slot (tile t, k-step ks, hi/lo, lane) holds A[32 t + lane % 32][16 ks + 8 (lane / 32) + i], i < 8.
template <int D, int R>
void build_operands(const double *tab, bool bf16, int sw, std::vector<uint16_t> &full, std::vector<uint16_t> &lin)
{
    constexpr kfvm::Stencil<D, R> st{};
    using S = kfvm::Stencil<D, R>;
    constexpr int NK = S::N0 - 1;        // contraction slots: S0 less its centre
    constexpr int KS = (NK + 15) / 16, NTF = (S::NROWS * 8 + 31) / 32, NTL = (S::NPTS + 31) / 32;
    int pos[S::NST][S::N0];
    for (int q = 0; q < S::NST; ++q) {
        for (int h = 0; h < S::N0; ++h) pos[q][h] = -1;
        for (int j = 0; j < st.nmem[q]; ++j) pos[q][st.mem[q][j]] = j;
    }
    auto put = [&](std::vector<uint16_t> &dst, int t, int ks, int lane, int i, double w) {
        const double x = std::ldexp(w, sw);
        const uint16_t hi = bf16 ? to_bf16(x) : to_f16(x);
        const double xh = bf16 ? from_bf16(hi) : from_f16(hi);
        const uint16_t lo = bf16 ? to_bf16(x - xh) : to_f16(x - xh);
        dst[((((size_t)t * KS + ks) * 2 + 0) * 64 + lane) * 8 + i] = hi;
        dst[((((size_t)t * KS + ks) * 2 + 1) * 64 + lane) * 8 + i] = lo;
    };
    full.assign((size_t)NTF * KS * 2 * 64 * 8, 0);
    lin.assign((size_t)NTL * KS * 2 * 64 * 8, 0);
    for (int t = 0; t < NTF; ++t)
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int row = 32 * t + lane % 32, k = 16 * ks + 8 * (lane / 32) + i;
                    const int tau = row / 8, q = row % 8;
                    double w = 0.0;
                    const int h = k < NK ? kfvm::slot_point<D, R>(k) : -1;
                    if (q < S::NST && tau < S::NROWS && h >= 0 && pos[q][h] >= 0)
                        w = tab[st.tab[q] + tau * st.nmem[q] + pos[q][h]];
                    put(full, t, ks, lane, i, w);
                }
    for (int t = 0; t < NTL; ++t)
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int tau = 32 * t + lane % 32, k = 16 * ks + 8 * (lane / 32) + i;
                    const double w = (tau < S::NPTS && k < NK) ? tab[st.tab[0] + tau * S::N0 + kfvm::slot_point<D, R>(k)]
                                                               : 0.0;
                    put(lin, t, ks, lane, i, w);
                }
}

int prepare_mixed(kfvm_ctx *c, int mode)
{
    if (c->mix_mode == mode) return KFVM_OK;
    // the kernels address the face buffer with 32-bit per-lane byte offsets
    // the reconstruction stores through 32-bit lane offsets of up to 32 bytes per cell
    if (c->geom.ncell >= (1L << 27)) return fail(c, KFVM_ERR_ARG, "the split-precision path takes fewer than 2^27 cells");
    const bool bf16 = mode == KFVM_SPLIT_BF16;
    double wmax = 0.0;
    for (double x : c->host_tables) wmax = std::fmax(wmax, std::fabs(x));
    // largest power-of-two scale that keeps every scaled weight below 30000 (fp16 max 65504)
    const int sw = (int)std::floor(std::log2(30000.0 / wmax));
    std::vector<uint16_t> full, lin;
    if (c->dim == 2 && c->R == 2) build_operands<2, 2>(c->host_tables.data(), bf16, sw, full, lin);
    else if (c->dim == 2 && c->R == 3) build_operands<2, 3>(c->host_tables.data(), bf16, sw, full, lin);
    else if (c->dim == 3 && c->R == 2) build_operands<3, 2>(c->host_tables.data(), bf16, sw, full, lin);
    else build_operands<3, 3>(c->host_tables.data(), bf16, sw, full, lin);
    if (!c->d_mix_full) {
        int rc = alloc(c, (void **)&c->d_mix_full, full.size() * 2);
        if (rc == KFVM_OK) rc = alloc(c, (void **)&c->d_mix_lin, lin.size() * 2);
        if (rc == KFVM_OK) rc = alloc(c, (void **)&c->work.inc32,
                                      sizeof(float) * (size_t)kfvm::inc_points(npts_of(c->dim, c->R)) * c->nvar *
                                          c->geom.ncell);
        if (rc != KFVM_OK) return rc;
    }
    HIP_TRY(c, hipMemcpy(c->d_mix_full, full.data(), full.size() * 2, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_mix_lin, lin.data(), lin.size() * 2, hipMemcpyHostToDevice));
    c->mix_sw = sw;
    c->mix_mode = mode;
    return KFVM_OK;
}

}  // namespace

extern "C" {

static int init_context(kfvm_ctx **out, const kfvm_mesh *mesh, int order, double gamma, const kfvm_weights *weights,
                        double ell_hat)
{
    if (!out || !mesh) return fail(nullptr, KFVM_ERR_ARG, "null argument");
    *out = nullptr;
    if (mesh->dim != 2 && mesh->dim != 3) return fail(nullptr, KFVM_ERR_ARG, "dim must be 2 or 3");
    if (order != 5 && order != 7) return fail(nullptr, KFVM_ERR_ARG, "order must be 5 (R = 2) or 7 (R = 3)");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(nullptr, KFVM_ERR_ARG, "gamma must exceed 1");
    const int dim = mesh->dim, R = order == 5 ? 2 : 3;
    long ncell = 1;
    for (int a = 0; a < dim; ++a) {
        if (mesh->n[a] < 2 * R + 2) return fail(nullptr, KFVM_ERR_ARG, "every n must be at least 2R + 2");
        if (!(mesh->dx[a] > 0.0) || !std::isfinite(mesh->dx[a])) return fail(nullptr, KFVM_ERR_ARG, "bad dx");
        ncell *= mesh->n[a];
    }
    if (ncell > (1L << 31)) return fail(nullptr, KFVM_ERR_ARG, "grid too large");

    kfvm_ctx *c = new kfvm_ctx();
    c->dim = dim;
    c->R = R;
    c->nvar = dim + 2;
    for (int a = 0; a < 3; ++a) {
        c->geom.n[a] = a < dim ? mesh->n[a] : 1;
        c->geom.dx[a] = a < dim ? mesh->dx[a] : 1.0;
    }
    c->geom.ncell = ncell;
    c->geom.gamma = gamma;
    c->geom.periodic = 1;
    for (int a = 0; a < 3; ++a) c->work.plane = std::max(c->work.plane, ncell / c->geom.n[a]);

    const int ntab = kfvm_weights_size(dim, R);
    std::vector<double> host(ntab);
    if (weights) {
        if (!layout_matches(dim, R, weights)) {
            delete c;
            return fail(nullptr, KFVM_ERR_ARG, "weights layout does not match the library's stencils");
        }
        std::memcpy(host.data(), weights->tables, sizeof(double) * ntab);
    } else {
        if (kfvm_weights_build(dim, R, ell_hat, host.data(), ntab) != ntab) {
            delete c;
            return fail(nullptr, KFVM_ERR_STATE, "weight build failed");
        }
    }

    const int nv = c->nvar;
    int rc = KFVM_OK;
    auto A = [&](void **p, size_t bytes) { if (rc == KFVM_OK) rc = alloc(c, p, bytes); };
    A((void **)&c->d_tables, sizeof(double) * ntab);
    A((void **)&c->work.theta, sizeof(double) * 2 * (size_t)ncell);
    A((void **)&c->work.fbar, sizeof(double) * (size_t)dim * nv * ncell);
    A((void **)&c->work.stage[0], sizeof(double) * (size_t)nv * ncell);
    A((void **)&c->work.stage[1], sizeof(double) * (size_t)nv * ncell);
    A((void **)&c->work.cfl_part, sizeof(double) * kfvm::CFL_SCRATCH_DOUBLES);
    A((void **)&c->work.err, sizeof(int) * 4);
    A((void **)&c->work.counts, sizeof(unsigned long long) * 2);
    A((void **)&c->d_dt, sizeof(double) * 3);
    if (rc != KFVM_OK) {
        g_init_msg = c->msg;
        kfvm_destroy(c);
        return rc;
    }
    c->host_tables = host;
    hipError_t e = hipMemcpy(c->d_tables, host.data(), sizeof(double) * ntab, hipMemcpyHostToDevice);
    if (e == hipSuccess && dim == 3 && R == 3) {
        // chunk-major copy for the chunked FP64 reconstruction: per chunk a [row][CH]
        // block of its stencil's weights, zeros in the padding
        using L = kfvm::ChunkLayout<3, 3, kfvm::FP64_CHUNK>;
        using S = kfvm::Stencil<3, 3>;
        static constexpr L lay{};
        static constexpr S st{};
        std::vector<double> wch((size_t)L::NCH * S::NROWS * L::CH, 0.0);
        for (int q = 0; q < S::NST; ++q)
            for (int k = lay.cb[q]; k < lay.cb[q + 1]; ++k)
                for (int row = 0; row < S::NROWS; ++row)
                    for (int j = 0; j < L::CH; ++j) {
                        const int m = (k - lay.cb[q]) * L::CH + j;
                        if (m < st.nmem[q])
                            wch[((size_t)k * S::NROWS + row) * L::CH + j] = host[st.tab[q] + row * st.nmem[q] + m];
                    }
        if (alloc(c, (void **)&c->d_wch, sizeof(double) * wch.size()) != KFVM_OK) {
            g_init_msg = c->msg;
            kfvm_destroy(c);
            return KFVM_ERR_HIP;
        }
        e = hipMemcpy(c->d_wch, wch.data(), sizeof(double) * wch.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(c->work.err, 0, sizeof(int) * 4);
    // the allocation-free CFL call's scratch on this GPU (looked up once per device)
    if (e == hipSuccess) e = kfvm::cfl_scratch_address(&c->cfl_scratch);
    if (e != hipSuccess) {
        hip_fail(nullptr, e, "upload");
        kfvm_destroy(c);
        return KFVM_ERR_HIP;
    }
    *out = c;
    return KFVM_OK;
}

int kfvm_init(kfvm_ctx **out, const kfvm_mesh *mesh, int order, double gamma, const kfvm_weights *weights)
{
    return init_context(out, mesh, order, gamma, weights, 5.0);
}

int kfvm_init_length_scale(kfvm_ctx **out, const kfvm_mesh *mesh, int order, double gamma, double ell_hat)
{
    if (out) *out = nullptr;
    if (!(ell_hat > 0.0 && ell_hat <= 100.0))
        return fail(nullptr, KFVM_ERR_ARG, "ell_hat must lie in (0, 100]");
    return init_context(out, mesh, order, gamma, nullptr, ell_hat);
}

static void record_event(void *self, int kind, hipStream_t s, int begin)
{
    kfvm_ctx *c = (kfvm_ctx *)self;
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return;
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return;
    }
    if (begin) {
        c->pending[kind] = ev;
    } else {
        c->events.push_back({kind, {c->pending[kind], ev}});
        c->pending[kind] = nullptr;
    }
}

static kfvm::Timing timing_of(kfvm_ctx *c) { return kfvm::Timing{c->timing, record_event, c}; }

static kfvm::GateArgs gate_of(kfvm_ctx *c)
{
    return kfvm::GateArgs{c->gate_on ? c->d_gate_w : nullptr, c->d_gate_vec, c->gate_thr, c->d_flags_out,
                          c->d_gate_raw};
}

// The FP64 face buffer (n_pts * nvar float64 per cell: 122 GB at 384^3 R = 3)
// is allocated on the first use of the FP64 reconstruction.
static int ensure_face64(kfvm_ctx *c)
{
    if (c->work.face) return KFVM_OK;
    return alloc(c, (void **)&c->work.face, sizeof(double) * (size_t)npts_of(c->dim, c->R) * c->nvar * c->geom.ncell);
}

// The KXRCF operands: the S0 face-point rows regrouped per (axis, side) so that
// the rows one thread needs for a member are contiguous, and the buffers of
// the indicator's output.
extern "C++" template <int D, int R>
static void kxrcf_rows(const double *tab, std::vector<double> &kw)
{
    using S = kfvm::Stencil<D, R>;
    constexpr int N0 = S::N0, NG = S::NG;
    kw.assign((size_t)kfvm::kxrcf_table_size(D, R), 0.0);
    if constexpr (kfvm::kx_all_axes(D, R)) {
        // [member][axis][point] upper-face rows over S0, then per member of the
        // neighbours' union and per axis it belongs to, the n_g lower-face rows
        using Un = kfvm::KxUnion<D, R>;
        static constexpr Un un{};
        for (int j = 0; j < N0; ++j)
            for (int a = 0; a < D; ++a)
                for (int p = 0; p < NG; ++p) kw[((size_t)j * D + a) * NG + p] = tab[((2 * a + 1) * NG + p) * N0 + j];
        double *kn = kw.data() + (size_t)N0 * D * NG;
        for (int m = 0; m < Un::NU; ++m) {
            int k = un.woff[m];
            for (int a = 0; a < D; ++a) {
                if (un.j[m][a] < 0) continue;
                for (int p = 0; p < NG; ++p) kn[k + p] = tab[((2 * a) * NG + p) * N0 + un.j[m][a]];
                k += NG;
            }
        }
        return;
    }
    for (int a = 0; a < D; ++a)
        for (int side = 0; side < 2; ++side)
            for (int j = 0; j < N0; ++j)
                for (int p = 0; p < NG; ++p) {
                    // side 0: the cell's upper face (2a + 1); side 1: the neighbour's lower face (2a)
                    const int row = (2 * a + (side == 0 ? 1 : 0)) * NG + p;
                    kw[((size_t)(a * 2 + side) * N0 + j) * NG + p] = tab[row * N0 + j];   // stencil 0 leads the tables
                }
}

static int ensure_kxrcf(kfvm_ctx *c)
{
    if (!c->d_kx_w) {
        std::vector<double> kw;
        if (c->dim == 2 && c->R == 2) kxrcf_rows<2, 2>(c->host_tables.data(), kw);
        else if (c->dim == 2 && c->R == 3) kxrcf_rows<2, 3>(c->host_tables.data(), kw);
        else if (c->dim == 3 && c->R == 2) kxrcf_rows<3, 2>(c->host_tables.data(), kw);
        else kxrcf_rows<3, 3>(c->host_tables.data(), kw);
        int rc = alloc(c, (void **)&c->d_kx_w, sizeof(double) * kw.size());
        if (rc != KFVM_OK) return rc;
        HIP_TRY(c, hipMemcpy(c->d_kx_w, kw.data(), sizeof(double) * kw.size(), hipMemcpyHostToDevice));
    }
    if (!c->d_kx_jump) {
        const int rc = alloc(c, (void **)&c->d_kx_jump, sizeof(double) * (size_t)c->dim * c->geom.ncell);
        if (rc != KFVM_OK) return rc;
    }
    if (!c->d_flags_out) return alloc(c, (void **)&c->d_flags_out, (size_t)c->nvar * c->geom.ncell);
    return KFVM_OK;
}

// Delta^m, Delta the cell width (the largest spacing when they differ)
static double kxrcf_threshold(const kfvm_ctx *c, double m)
{
    double delta = c->geom.dx[0];
    for (int a = 1; a < c->dim; ++a) delta = std::fmax(delta, c->geom.dx[a]);
    return std::pow(delta, m);
}

static int run_kxrcf(kfvm_ctx *c, const double *U, double m, double *J, uint8_t *flags)
{
    kfvm::Timing tm = timing_of(c);
    if (tm.on) tm.record(tm.self, kfvm::KT_INDICATOR, c->stream, 1);
    if (!c->geom.periodic && !c->d_kx_jlo) {
        const int rc = alloc(c, (void **)&c->d_kx_jlo, sizeof(double) * (size_t)c->dim * c->work.plane);
        if (rc != KFVM_OK) return rc;
    }
    hipError_t e = kfvm::launch_kxrcf(c->dim, c->R, c->geom, c->d_kx_w, c->d_tables, U, J, c->d_kx_jlo, c->work.plane,
                                      flags, kxrcf_threshold(c, m), c->stream);
    if (tm.on) tm.record(tm.self, kfvm::KT_INDICATOR, c->stream, 0);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return KFVM_OK;
}

// The reconstruction's per-(variable, cell) choices for input U: with the KXRCF
// indicator on, its first pass runs here and its flags replace any others.
static int prepare_flags(kfvm_ctx *c, const double *U, kfvm::Work &w)
{
    w = c->work;
    c->recon_done = 1;
    c->last_flags = c->gate_on ? c->d_flags_out : c->work.flags_in;
    if (c->indicator != KFVM_IND_KXRCF) return KFVM_OK;
    c->last_flags = c->d_flags_out;
    const int rc = run_kxrcf(c, U, c->kx_m, c->d_kx_jump, c->d_flags_out);
    w.flags_in = c->d_flags_out;
    return rc;
}

// err (optional): the error word this stage's kernels raise instead of the
// sticky one; guard (optional): the update writes nothing while *guard != 0
static int stage_call(kfvm_ctx *c, const double *U0, const double *Uin, double *out, int stage, double dt,
                      int *err = nullptr, const int *guard = nullptr)
{
    hipError_t e;
    kfvm::Work w;
    int rc = prepare_flags(c, Uin, w);
    if (rc != KFVM_OK) return rc;
    if (err) w.err = err;
    w.guard = guard;
    if (c->precision == KFVM_FP64) {
        rc = ensure_face64(c);
        if (rc != KFVM_OK) return rc;
        w.face = c->work.face;
        kfvm::Tables t{c->d_tables, c->d_wch};
        e = kfvm::launch_rhs_fp64(c->dim, c->R, c->geom, t, w, c->lim, c->riemann, U0, Uin, out, stage, dt,
                                  c->stream, timing_of(c));
    } else {
        kfvm::MixTables t{c->d_mix_full, c->d_mix_lin, c->mix_sw};
        e = kfvm::launch_rhs_mixed(c->dim, c->R, c->precision == KFVM_SPLIT_BF16, c->geom, t, w, c->lim,
                                   c->riemann, U0, Uin, out, stage, dt, nullptr, c->stream, timing_of(c), gate_of(c));
    }
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return KFVM_OK;
}

int kfvm_rhs(kfvm_ctx *c, const double *U, double *dUdt)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !dUdt) return fail(c, KFVM_ERR_ARG, "null buffer");
    if (U == dUdt) return fail(c, KFVM_ERR_ARG, "U and dUdt must not alias");
    int rc = stage_call(c, U, U, dUdt, 0, 0.0);
    if (rc == KFVM_OK && c->checking) rc = sync_check(c);
    return rc;
}

int kfvm_step(kfvm_ctx *c, double *U, double dt)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U) return fail(c, KFVM_ERR_ARG, "null buffer");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, KFVM_ERR_ARG, "dt must be positive and finite");
    double *U1 = c->work.stage[0], *U2 = c->work.stage[1];
    // the step's own error word: cleared first, raised by any stage, read by the
    // last stage's update (which then leaves U as it was), then merged into the
    // sticky word; all stream-ordered, no host synchronisation
    int *step_err = c->work.err + 1;
    hipError_t e = kfvm::launch_err_reset(step_err, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    int rc = stage_call(c, U, U, U1, 1, dt, step_err);
    if (rc == KFVM_OK) rc = stage_call(c, U, U1, U2, 2, dt, step_err);
    if (rc == KFVM_OK) rc = stage_call(c, U, U2, U, 3, dt, step_err, step_err);
    e = kfvm::launch_err_merge(c->work.err, step_err, c->stream);
    if (rc == KFVM_OK && e != hipSuccess) return hip_fail(c, e, "launch");
    if (rc == KFVM_OK && c->checking) rc = sync_check(c);
    return rc;
}

int kfvm_step_ssp432(kfvm_ctx *c, const double *U, double *U_out, double dt, double atol, double rtol,
                     double *err_host)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !U_out || !err_host) return fail(c, KFVM_ERR_ARG, "null pointer");
    if (U == U_out) return fail(c, KFVM_ERR_ARG, "U and U_out must not alias");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, KFVM_ERR_ARG, "dt must be positive and finite");
    if (!(atol >= 0.0) || !(rtol >= 0.0) || !(atol + rtol > 0.0)) return fail(c, KFVM_ERR_ARG, "bad tolerances");
    const double h = 0.5 * dt;
    double *S0 = c->work.stage[0], *S1 = c->work.stage[1];
    int rc = stage_call(c, U, U, S0, 1, h);                      // U1 = U + h L(U)
    if (rc == KFVM_OK) rc = stage_call(c, U, S0, S1, 1, h);      // U2 = U1 + h L(U1)
    if (rc == KFVM_OK) rc = stage_call(c, U, S1, S0, 4, h);      // U3 = 2/3 U + 1/3 (U2 + h L(U2))
    if (rc == KFVM_OK) rc = stage_call(c, U, S0, U_out, 1, h);   // U+ = U3 + h L(U3)
    if (rc != KFVM_OK) return rc;
    hipError_t e = kfvm::launch_ssp_error(U, S0, U_out, c->geom.ncell * c->nvar, atol, rtol, c->work.cfl_part,
                                          c->d_dt, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    HIP_TRY(c, hipMemcpyAsync(err_host, c->d_dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync_check(c);
}

int kfvm_cfl_dt(kfvm_ctx *c, const double *U, double cfl, double *dt_host)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !dt_host) return fail(c, KFVM_ERR_ARG, "null pointer");
    if (!(cfl > 0.0)) return fail(c, KFVM_ERR_ARG, "cfl must be positive");
    hipError_t e = kfvm::launch_cfl(c->dim, c->geom, c->work, U, cfl, c->d_dt, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    double r[3];
    HIP_TRY(c, hipMemcpyAsync(r, c->d_dt, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    const int rc = sync_check(c);
    *dt_host = r[0];
    c->min_rho = r[1];
    c->min_p = r[2];
    return rc;
}

int kfvm_cfl_dt_noalloc(kfvm_ctx *c, const double *U, double cfl, double *out_dev)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !out_dev) return fail(c, KFVM_ERR_ARG, "null pointer");
    if (!(cfl > 0.0)) return fail(c, KFVM_ERR_ARG, "cfl must be positive");
    if (!c->cfl_scratch) return fail(c, KFVM_ERR_STATE, "no CFL scratch on this device");
    const hipError_t e = kfvm::launch_cfl_scratch(c->dim, c->geom, c->cfl_scratch, c->work.err, U, cfl, out_dev,
                                                  c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return KFVM_OK;
}

int kfvm_set_stream(kfvm_ctx *c, void *s)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    c->stream = (hipStream_t)s;
    return KFVM_OK;
}

int kfvm_set_precision(kfvm_ctx *c, int mode)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (mode != KFVM_FP64 && mode != KFVM_SPLIT_F16 && mode != KFVM_SPLIT_BF16)
        return fail(c, KFVM_ERR_ARG, "unknown precision mode");
    if (mode != KFVM_FP64) {
        if (!kfvm::mixed_supported(c->dim, c->R))
            return fail(c, KFVM_ERR_ARG, "split precision is not available for this dimension and order");
        const int rc = prepare_mixed(c, mode);
        if (rc != KFVM_OK) return rc;
    }
    c->precision = mode;
    return KFVM_OK;
}

int kfvm_set_limiter(kfvm_ctx *c, int enabled, double kappa)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!(kappa >= 0.0 && kappa < 1.0)) return fail(c, KFVM_ERR_ARG, "kappa must lie in [0, 1)");
    c->lim.on = enabled != 0;
    c->lim.kappa = kappa;
    return KFVM_OK;
}

int kfvm_set_cfl_form(kfvm_ctx *c, int form)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (form != KFVM_CFL_SUM && form != KFVM_CFL_MAX_AXIS) return fail(c, KFVM_ERR_ARG, "unknown CFL form");
    c->geom.cfl_max_axis = form == KFVM_CFL_MAX_AXIS;
    return KFVM_OK;
}

int kfvm_set_flattener(kfvm_ctx *c, double k1)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!(k1 >= 0.0 && k1 < INFINITY)) return fail(c, KFVM_ERR_ARG, "the flattener onset k1 must be finite and >= 0");
    c->lim.flat_k1 = k1;
    return KFVM_OK;
}

int kfvm_set_riemann(kfvm_ctx *c, int solver)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (solver != KFVM_HLLC && solver != KFVM_HLL) return fail(c, KFVM_ERR_ARG, "unknown Riemann solver");
    c->riemann = solver;
    return KFVM_OK;
}

int kfvm_set_checking(kfvm_ctx *c, int checking)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    c->checking = checking != 0;
    return KFVM_OK;
}

int kfvm_status(kfvm_ctx *c)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    return sync_check(c);
}

int kfvm_stats(kfvm_ctx *c, kfvm_stats_t *out)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!out) return fail(c, KFVM_ERR_ARG, "null pointer");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int err = 0;
    HIP_TRY(c, hipMemcpy(&err, c->work.err, sizeof(int), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->cell_vars = (long long)c->geom.ncell * c->nvar;
    out->min_rho = c->min_rho;
    out->min_p = c->min_p;
    // counted from the limiter factors and the choices the last reconstruction left
    unsigned long long cnt[2] = {0, 0};
    if (!c->recon_done) {
        out->error = err;
        return KFVM_OK;
    }
    HIP_TRY(c, hipMemsetAsync(c->work.counts, 0, sizeof(cnt), c->stream));
    hipError_t e = kfvm::launch_count_stats(c->work.theta, c->last_flags, c->geom.ncell, c->nvar, c->work.counts,
                                            c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    HIP_TRY(c, hipMemcpyAsync(cnt, c->work.counts, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out->limiter_cells = (long long)cnt[0];
    out->weno_cell_vars = c->last_flags ? (long long)cnt[1] : out->cell_vars;
    out->error = err;
    return KFVM_OK;
}

int kfvm_face_states(kfvm_ctx *c, const double *U, double *states)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !states) return fail(c, KFVM_ERR_ARG, "null buffer");
    hipError_t e;
    kfvm::Work w;
    int rc = prepare_flags(c, U, w);
    if (rc != KFVM_OK) return rc;
    if (c->precision == KFVM_FP64) {
        rc = ensure_face64(c);
        if (rc != KFVM_OK) return rc;
        w.face = c->work.face;
        kfvm::Tables t{c->d_tables, c->d_wch};
        e = kfvm::launch_face_states(c->dim, c->R, c->geom, t, w, c->lim, U, states, c->stream);
    } else {
        kfvm::MixTables t{c->d_mix_full, c->d_mix_lin, c->mix_sw};
        e = kfvm::launch_rhs_mixed(c->dim, c->R, c->precision == KFVM_SPLIT_BF16, c->geom, t, w, c->lim,
                                   c->riemann, U, U, nullptr, 0, 0.0, states, c->stream, kfvm::Timing{0, nullptr, nullptr},
                                   gate_of(c));
    }
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return c->checking ? sync_check(c) : KFVM_OK;
}

int kfvm_set_flags(kfvm_ctx *c, const uint8_t *flags)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    c->work.flags_in = flags;
    if (flags) {
        c->gate_on = 0;
        c->indicator = KFVM_IND_NONE;
    }
    return KFVM_OK;
}

int kfvm_set_boundary(kfvm_ctx *c, int axis, int lower, int upper, const double *lower_state,
                      const double *upper_state)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (axis < 0 || axis >= c->dim) return fail(c, KFVM_ERR_ARG, "axis out of range");
    const int kinds[2] = {lower, upper};
    const double *states[2] = {lower_state, upper_state};
    for (int side = 0; side < 2; ++side)
        if (kinds[side] < KFVM_BC_PERIODIC || kinds[side] > KFVM_BC_INFLOW)
            return fail(c, KFVM_ERR_ARG, "unknown boundary condition");
    if ((lower == KFVM_BC_PERIODIC) != (upper == KFVM_BC_PERIODIC))
        return fail(c, KFVM_ERR_ARG, "periodic must be set on both sides of an axis");
    for (int side = 0; side < 2; ++side) {
        if (kinds[side] != KFVM_BC_INFLOW) continue;
        if (!states[side]) return fail(c, KFVM_ERR_ARG, "an inflow side needs its state");
        const double *u = states[side];
        double ke = 0.0;
        for (int a = 0; a < c->dim; ++a) ke += u[1 + a] * u[1 + a];
        bool fin = true;
        for (int v = 0; v < c->nvar; ++v) fin = fin && std::isfinite(u[v]);
        if (!fin || !(u[0] > 0.0) || !((c->geom.gamma - 1.0) * (u[c->dim + 1] - 0.5 * ke / u[0]) > 0.0))
            return fail(c, KFVM_ERR_NONPHYSICAL, "inflow state with rho <= 0 or p <= 0");
    }
    if (lower != KFVM_BC_PERIODIC && !c->work.fbar_top) {
        const int rc = alloc(c, (void **)&c->work.fbar_top, sizeof(double) * (size_t)c->dim * c->nvar * c->work.plane);
        if (rc != KFVM_OK) return rc;
    }
    for (int side = 0; side < 2; ++side) {
        c->geom.bc[axis][side] = kinds[side];
        for (int v = 0; v < 5; ++v)
            c->geom.bc_state[axis][side][v] = kinds[side] == KFVM_BC_INFLOW && v < c->nvar ? states[side][v] : 0.0;
    }
    int periodic = 1;
    for (int a = 0; a < c->dim; ++a) periodic = periodic && c->geom.bc[a][0] == KFVM_BC_PERIODIC;
    c->geom.periodic = periodic;
    return KFVM_OK;
}

int kfvm_set_indicator(kfvm_ctx *c, int kind, double m)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (kind != KFVM_IND_NONE && kind != KFVM_IND_KXRCF) return fail(c, KFVM_ERR_ARG, "unknown indicator");
    if (kind == KFVM_IND_NONE) {
        c->indicator = KFVM_IND_NONE;
        return KFVM_OK;
    }
    if (!(m > 0.0) || !std::isfinite(m)) return fail(c, KFVM_ERR_ARG, "m must be positive and finite");
    const int rc = ensure_kxrcf(c);
    if (rc != KFVM_OK) return rc;
    c->indicator = kind;
    c->kx_m = m;
    c->gate_on = 0;
    c->work.flags_in = nullptr;
    return KFVM_OK;
}

int kfvm_kxrcf(kfvm_ctx *c, const double *U, double m, double *jumps, uint8_t *flags)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U) return fail(c, KFVM_ERR_ARG, "null buffer");
    if (!(m > 0.0) || !std::isfinite(m)) return fail(c, KFVM_ERR_ARG, "m must be positive and finite");
    const int rc = ensure_kxrcf(c);
    if (rc != KFVM_OK) return rc;
    return run_kxrcf(c, U, m, jumps ? jumps : c->d_kx_jump, flags ? flags : c->d_flags_out);
}

int kfvm_mlp_sizes(int dim, int *n_in, int *n_params)
{
    if ((dim != 2 && dim != 3) || !n_in || !n_params) return KFVM_ERR_ARG;
    *n_in = kfvm::mlp_n_in(dim);
    *n_params = kfvm::mlp_n_params(dim);
    return KFVM_OK;
}

int kfvm_set_gate(kfvm_ctx *c, const float *params, float threshold)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!params) {
        c->gate_on = 0;
        return KFVM_OK;
    }
    if (!kfvm::mixed_supported(c->dim, c->R)) return fail(c, KFVM_ERR_ARG, "the gate needs the split-precision path");
    const int nin = kfvm::mlp_n_in(c->dim), P = kfvm::mlp_n_params(c->dim), H = 32;
    std::vector<float> p(P);
    HIP_TRY(c, hipMemcpy(p.data(), params, sizeof(float) * P, hipMemcpyDeviceToHost));
    const int slots = kfvm::gate_operand_slots(c->dim), ksg = slots / 64 - 2, w1e = kfvm::gate_w1_exp(c->dim);
    std::vector<uint16_t> w((size_t)slots * 8, 0);
    // W1 as the A operand of k-step ks: lane l holds W1[l % 32][input of column 16 ks + 8 (l / 32) + i],
    // times 2^w1e (an exact exponent shift of the BF16 value)
    for (int ks = 0; ks < ksg; ++ks)
        for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 8; ++i) {
                const int m = l % 32, in = kfvm::gate_slot_input(c->dim, 16 * ks + 8 * (l / 32) + i);
                w[((size_t)ks * 64 + l) * 8 + i] = in >= 0 ? to_bf16(std::ldexp((double)p[m * nin + in], w1e)) : 0;
            }
    const float *W2 = p.data() + H * nin + H;
    for (int ks = 0; ks < 2; ++ks)
        for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 8; ++i) {
                const int m = l % 32, k = 16 * ks + 8 * (l / 32) + i;
                w[((size_t)(ksg + ks) * 64 + l) * 8 + i] = to_bf16(W2[m * H + k]);
            }
    std::vector<float> vec(97);
    for (int m = 0; m < H; ++m) {
        vec[m] = p[H * nin + m];                       // b1
        vec[32 + m] = p[H * nin + H + H * H + m];      // b2
        vec[64 + m] = p[H * nin + H + H * H + H + m];  // w3
    }
    vec[96] = p[P - 1];                                 // b3
    if (!c->d_gate_w) {
        int rc = alloc(c, (void **)&c->d_gate_w, w.size() * 2);
        if (rc == KFVM_OK) rc = alloc(c, (void **)&c->d_gate_vec, sizeof(float) * 97);
        if (rc == KFVM_OK && !c->d_flags_out) rc = alloc(c, (void **)&c->d_flags_out, (size_t)c->nvar * c->geom.ncell);
        if (rc == KFVM_OK) rc = alloc(c, (void **)&c->d_gate_raw, (size_t)c->geom.ncell);
        if (rc != KFVM_OK) return rc;
    }
    HIP_TRY(c, hipMemcpy(c->d_gate_w, w.data(), w.size() * 2, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_gate_vec, vec.data(), sizeof(float) * 97, hipMemcpyHostToDevice));
    c->gate_thr = threshold;
    c->gate_on = 1;
    c->work.flags_in = nullptr;
    c->indicator = KFVM_IND_NONE;
    return KFVM_OK;
}

int kfvm_get_flags(kfvm_ctx *c, uint8_t *flags)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!flags) return fail(c, KFVM_ERR_ARG, "null buffer");
    if (!c->d_flags_out) return fail(c, KFVM_ERR_STATE, "neither the gate nor the indicator has run");
    HIP_TRY(c, hipMemcpyAsync(flags, c->d_flags_out, (size_t)c->nvar * c->geom.ncell, hipMemcpyDeviceToDevice,
                              c->stream));
    return KFVM_OK;
}

int kfvm_gate_samples(kfvm_ctx *c, const double *U, float *x, float *ratio)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!U || !ratio) return fail(c, KFVM_ERR_ARG, "null buffer");
    const int rc = ensure_face64(c);
    if (rc != KFVM_OK) return rc;
    hipError_t e = x ? kfvm::launch_gate_inputs(c->dim, c->geom, U, x, c->stream) : hipSuccess;
    kfvm::Tables t{c->d_tables, c->d_wch};
    if (e == hipSuccess) e = kfvm::launch_recon_ratio(c->dim, c->R, c->geom, t, c->work, c->lim, U, ratio, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return c->checking ? sync_check(c) : KFVM_OK;
}

int kfvm_mlp_train_step(kfvm_ctx *c, const float *x, const float *y, int B, float *params, float *adam_m,
                        float *adam_v, int t, float lr, float pos_weight, float *loss, float *grad, float *logits)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!x || !params || B <= 0) return fail(c, KFVM_ERR_ARG, "null buffer or empty batch");
    if (lr > 0.f && (!adam_m || !adam_v || !y || t < 1)) return fail(c, KFVM_ERR_ARG, "an update needs y, m, v, t >= 1");
    const size_t need = kfvm::mlp_workspace_floats(c->dim, B);
    if (need > c->mlp_ws_floats) {
        if (c->d_mlp_ws) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipFree(c->d_mlp_ws));
            for (auto &p : c->allocs)
                if (p == c->d_mlp_ws) p = nullptr;
        }
        int rc = alloc(c, (void **)&c->d_mlp_ws, need * sizeof(float));
        if (rc != KFVM_OK) return rc;
        c->mlp_ws_floats = need;
    }
    hipError_t e = kfvm::launch_mlp_train(c->dim, x, y, B, params, adam_m, adam_v, t, lr, pos_weight, loss, grad,
                                          logits, c->d_mlp_ws, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launch");
    return KFVM_OK;
}

int kfvm_set_timing(kfvm_ctx *c, int on)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    c->timing = on != 0;
    return KFVM_OK;
}

int kfvm_kernel_times(kfvm_ctx *c, double *ms, long long *launches, int n)
{
    if (!c) return fail(nullptr, KFVM_ERR_STATE, "null context");
    if (!ms || !launches || n < kfvm::KT_COUNT) return fail(c, KFVM_ERR_ARG, "need room for every kernel class");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) { ms[k] = 0.0; launches[k] = 0; }
    for (auto &e : c->events) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.second.first, e.second.second) == hipSuccess) {
            ms[e.first] += t;
            launches[e.first] += 1;
        }
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    c->events.clear();
    return KFVM_OK;
}

const char *kfvm_last_error(const kfvm_ctx *c)
{
    return c ? c->msg.c_str() : g_init_msg.c_str();
}

void kfvm_destroy(kfvm_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (void *p : c->allocs)
        if (p) (void)hipFree(p);
    delete c;
}

}  // extern "C"
