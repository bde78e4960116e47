// Troubled-cell gate network: sample export, training and batch inference.
//
// Network n_in -> 32 -> 32 -> 1 with GELU (tanh form) after the hidden layers.
// n_in = 25 in 2D (5 x 5 window of one reconstruction variable around the cell)
// and 33 in 3D (the radius-2 sphere S0).  Inputs are the increments W_h - W_c,
// divided by the power of two 2^(e+1) with max |W_h - W_c| in [2^e, 2^(e+1)).
// Flat float32 parameters: W1 [32][n_in], b1 [32], W2 [32][32], b2 [32], w3 [32], b3.
//
// The hidden layers are evaluated as the matrix cores do in the gated
// reconstruction: inputs, W1, W2 and the first hidden activations rounded to
// BF16, products accumulated in float32.  Training keeps float32 master
// weights, differentiates straight through the roundings, minimises a
// positive-weighted binary cross-entropy and updates with Adam.  Weight
// gradients are reduced over fixed batch chunks in a fixed order (no atomics),
// so a training step is deterministic.
#include "device_common.hpp"

namespace kfvm {
namespace {
using namespace dev;

constexpr int H = 32;
constexpr int CHUNK = 256;     // samples per partial-gradient block
constexpr int SUB = 32;        // samples staged in LDS at a time

template <int NIN>
struct MlpLayout {
    static constexpr int W1 = 0, B1 = H * NIN, W2 = B1 + H, B2 = W2 + H * H, W3 = B2 + H, B3 = W3 + H;
    static constexpr int P = B3 + 1;
};

__device__ __forceinline__ float bf16r(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// ----------------------------------------------------------- sample export ---
// Gate inputs of every (variable, cell): x[v][cell][NIN] (float32), from the
// conserved averages with the cell's own Phi (the same W the reconstruction uses).
template <int D>
__global__ __launch_bounds__(256) void k_gate_inputs(const double *__restrict__ U, float *__restrict__ x, Geom g)
{
    constexpr int NV = D + 2;
    constexpr int NIN = D == 2 ? 25 : 33;
    constexpr Stencil<3, 2> s3{};
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const int cx = (int)(cell % g.n[0]), cy = (int)((cell / g.n[0]) % g.n[1]);
    const int cz = (int)(cell / ((long)g.n[0] * g.n[1]));
    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = U[v * g.ncell + cell];
    PhiRows<D> ph;
    ph.init(ref, g.gamma);
#pragma unroll 1
    for (int k = 0; k < NV; ++k) {
        double dl[NIN], amax = 0.0;
        double uc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) uc[v] = ref[v];
        const double wc = ph.row(k, uc);
#pragma unroll
        for (int h = 0; h < NIN; ++h) {
            int ox, oy, oz;
            if constexpr (D == 2) { ox = h / 5 - 2; oy = h % 5 - 2; oz = 0; }
            else { ox = s3.off[h][0]; oy = s3.off[h][1]; oz = s3.off[h][2]; }
            const long nb = wrap_any(cx + ox, g.n[0]) +
                            (long)g.n[0] * (wrap_any(cy + oy, g.n[1]) + (long)g.n[1] * (D == 3 ? wrap_any(cz + oz, g.n[2]) : 0));
            double un[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) un[v] = U[v * g.ncell + nb];
            dl[h] = ph.row(k, un) - wc;
            amax = fmax(amax, fabs(dl[h]));
        }
        int ex = 0;
        if (amax > 0.0) frexp(amax, &ex);       // amax in [2^(ex-1), 2^ex)
#pragma unroll
        for (int h = 0; h < NIN; ++h) x[((long)k * g.ncell + cell) * NIN + h] = (float)ldexp(dl[h], -ex);
    }
}

// --------------------------------------------------------------- training ---
// Per sample: forward pass and the backpropagated deltas.
template <int NIN>
__global__ __launch_bounds__(128) void k_mlp_fwd_bwd(const float *__restrict__ prm, const float *__restrict__ x,
                                                     const float *__restrict__ y, int B, float pos_weight,
                                                     float *__restrict__ h1r_o, float *__restrict__ h2_o,
                                                     float *__restrict__ dz1_o, float *__restrict__ dz2_o,
                                                     float *__restrict__ dz3_o, float *__restrict__ loss_o,
                                                     float *__restrict__ logit_o)
{
    using L = MlpLayout<NIN>;
    __shared__ float W1r[H * NIN], W2r[H * H], b1[H], b2[H], w3[H];
    __shared__ float b3;
    for (int i = threadIdx.x; i < H * NIN; i += blockDim.x) W1r[i] = bf16r(prm[L::W1 + i]);
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) W2r[i] = bf16r(prm[L::W2 + i]);
    for (int i = threadIdx.x; i < H; i += blockDim.x) { b1[i] = prm[L::B1 + i]; b2[i] = prm[L::B2 + i]; w3[i] = prm[L::W3 + i]; }
    if (threadIdx.x == 0) b3 = prm[L::B3];
    __syncthreads();
    const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float xr[NIN], z1[H], h1r[H], z2[H];
#pragma unroll
    for (int k = 0; k < NIN; ++k) xr[k] = bf16r(x[b * NIN + k]);
#pragma unroll
    for (int m = 0; m < H; ++m) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NIN; ++k) s = fmaf(W1r[m * NIN + k], xr[k], s);
        z1[m] = s + b1[m];
        h1r[m] = bf16r(gelu_f(z1[m]));
    }
    float z3 = b3;
#pragma unroll
    for (int m = 0; m < H; ++m) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < H; ++k) s = fmaf(W2r[m * H + k], h1r[k], s);
        z2[m] = s + b2[m];
        const float h2 = gelu_f(z2[m]);
        h2_o[b * H + m] = h2;
        z3 = fmaf(w3[m], h2, z3);
    }
    const float yy = y ? y[b] : 0.f;
    const float sp_pos = fmaxf(z3, 0.f) + log1pf(__expf(-fabsf(z3)));   // softplus(z)
    const float sp_neg = sp_pos - z3;                                     // softplus(-z)
    loss_o[b] = pos_weight * yy * sp_neg + (1.f - yy) * sp_pos;
    logit_o[b] = z3;
    const float sg = 1.f / (1.f + __expf(-z3));
    const float dz3 = (-pos_weight * yy * (1.f - sg) + (1.f - yy) * sg) / (float)B;
    dz3_o[b] = dz3;
    float dz2[H];
#pragma unroll
    for (int m = 0; m < H; ++m) {
        dz2[m] = dz3 * w3[m] * gelu_grad_f(z2[m]);
        dz2_o[b * H + m] = dz2[m];
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        float s = 0.f;
#pragma unroll
        for (int m = 0; m < H; ++m) s = fmaf(W2r[m * H + k], dz2[m], s);
        dz1_o[b * H + k] = s * gelu_grad_f(z1[k]);
        h1r_o[b * H + k] = h1r[k];
    }
}

// Partial weight gradients over one chunk of CHUNK samples (fixed order).
template <int NIN>
__global__ __launch_bounds__(256) void k_mlp_grad_partial(const float *__restrict__ x, const float *__restrict__ h1r,
                                                          const float *__restrict__ h2, const float *__restrict__ dz1,
                                                          const float *__restrict__ dz2, const float *__restrict__ dz3,
                                                          int B, float *__restrict__ part)
{
    using L = MlpLayout<NIN>;
    __shared__ float sx[SUB][NIN], sh1[SUB][H], sh2[SUB][H], sd1[SUB][H], sd2[SUB][H], sd3[SUB];
    constexpr int PER = (L::P + 255) / 256;
    float acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = 0.f;
    const long b0 = (long)blockIdx.x * CHUNK;
    for (int s0 = 0; s0 < CHUNK; s0 += SUB) {
        __syncthreads();
        for (int i = threadIdx.x; i < SUB * NIN; i += 256) {
            const long b = b0 + s0 + i / NIN;
            sx[i / NIN][i % NIN] = b < B ? bf16r(x[b * NIN + i % NIN]) : 0.f;
        }
        for (int i = threadIdx.x; i < SUB * H; i += 256) {
            const long b = b0 + s0 + i / H;
            const bool ok = b < B;
            sh1[i / H][i % H] = ok ? h1r[b * H + i % H] : 0.f;
            sh2[i / H][i % H] = ok ? h2[b * H + i % H] : 0.f;
            sd1[i / H][i % H] = ok ? dz1[b * H + i % H] : 0.f;
            sd2[i / H][i % H] = ok ? dz2[b * H + i % H] : 0.f;
        }
        for (int i = threadIdx.x; i < SUB; i += 256) sd3[i] = (b0 + s0 + i) < B ? dz3[b0 + s0 + i] : 0.f;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int p = threadIdx.x + 256 * r;
            if (p >= L::P) continue;
            float a = acc[r];
            if (p < L::B1) {
                const int m = p / NIN, k = p % NIN;
                for (int s = 0; s < SUB; ++s) a = fmaf(sd1[s][m], sx[s][k], a);
            } else if (p < L::W2) {
                const int m = p - L::B1;
                for (int s = 0; s < SUB; ++s) a += sd1[s][m];
            } else if (p < L::B2) {
                const int m = (p - L::W2) / H, k = (p - L::W2) % H;
                for (int s = 0; s < SUB; ++s) a = fmaf(sd2[s][m], sh1[s][k], a);
            } else if (p < L::W3) {
                const int m = p - L::B2;
                for (int s = 0; s < SUB; ++s) a += sd2[s][m];
            } else if (p < L::B3) {
                const int m = p - L::W3;
                for (int s = 0; s < SUB; ++s) a = fmaf(sd3[s], sh2[s][m], a);
            } else {
                for (int s = 0; s < SUB; ++s) a += sd3[s];
            }
            acc[r] = a;
        }
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int p = threadIdx.x + 256 * r;
        if (p < L::P) part[(long)blockIdx.x * L::P + p] = acc[r];
    }
}

// Sum the partials in chunk order; optional gradient output; Adam (lr > 0).
__global__ __launch_bounds__(256) void k_mlp_adam(const float *__restrict__ part, int nchunk, int P,
                                                  float *__restrict__ prm, float *__restrict__ m,
                                                  float *__restrict__ v, float *__restrict__ grad_o, int t, float lr)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float g = 0.f;
    for (int c = 0; c < nchunk; ++c) g += part[(long)c * P + p];
    if (grad_o) grad_o[p] = g;
    if (lr > 0.f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mm = b1 * m[p] + (1.f - b1) * g;
        const float vv = b2 * v[p] + (1.f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / (1.f - powf(b1, (float)t)), vh = vv / (1.f - powf(b2, (float)t));
        prm[p] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ __launch_bounds__(256) void k_sum(const float *__restrict__ a, int n, float *__restrict__ out)
{
    __shared__ float red[4];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1] + red[2] + red[3]) / (float)n;
}

template <int NIN>
hipError_t train_impl(const float *x, const float *y, int B, float *prm, float *m, float *v, int t, float lr,
                      float pos_weight, float *loss, float *grad, float *logits, float *ws, hipStream_t s)
{
    using L = MlpLayout<NIN>;
    float *h1r = ws, *h2 = h1r + (size_t)B * H, *dz1 = h2 + (size_t)B * H, *dz2 = dz1 + (size_t)B * H;
    float *dz3 = dz2 + (size_t)B * H, *lss = dz3 + B, *lg = lss + B, *part = lg + B;
    const int nchunk = (B + CHUNK - 1) / CHUNK;
    hipLaunchKernelGGL((k_mlp_fwd_bwd<NIN>), dim3((B + 127) / 128), dim3(128), 0, s, prm, x, y, B, pos_weight, h1r, h2,
                       dz1, dz2, dz3, lss, logits ? logits : lg);
    hipLaunchKernelGGL((k_mlp_grad_partial<NIN>), dim3(nchunk), dim3(256), 0, s, x, h1r, h2, dz1, dz2, dz3, B, part);
    hipLaunchKernelGGL(k_mlp_adam, dim3((L::P + 255) / 256), dim3(256), 0, s, part, nchunk, L::P, prm, m, v, grad, t,
                       lr);
    if (loss) hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, lss, B, loss);
    return hipGetLastError();
}

}  // namespace

int mlp_n_in(int dim) { return dim == 2 ? 25 : 33; }
int mlp_n_params(int dim) { return dim == 2 ? MlpLayout<25>::P : MlpLayout<33>::P; }

size_t mlp_workspace_floats(int dim, int B)
{
    const int P = mlp_n_params(dim);
    return (size_t)B * (4 * H + 3) + (size_t)((B + CHUNK - 1) / CHUNK) * P;
}

hipError_t launch_gate_inputs(int dim, const Geom &g, const double *U, float *x, hipStream_t s)
{
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (dim == 2) hipLaunchKernelGGL((k_gate_inputs<2>), dim3(nb), dim3(256), 0, s, U, x, g);
    else hipLaunchKernelGGL((k_gate_inputs<3>), dim3(nb), dim3(256), 0, s, U, x, g);
    return hipGetLastError();
}

hipError_t launch_mlp_train(int dim, const float *x, const float *y, int B, float *prm, float *m, float *v, int t,
                            float lr, float pos_weight, float *loss, float *grad, float *logits, float *ws,
                            hipStream_t s)
{
    if (dim == 2) return train_impl<25>(x, y, B, prm, m, v, t, lr, pos_weight, loss, grad, logits, ws, s);
    return train_impl<33>(x, y, B, prm, m, v, t, lr, pos_weight, loss, grad, logits, ws, s);
}

}  // namespace kfvm
