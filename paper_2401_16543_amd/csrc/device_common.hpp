// Device helpers shared by the FP64 and mixed-precision right-hand-side
// kernels: tiling, periodic wrap, the ideal-gas law, the linearised primitive
// variables (section 3.4.2), the positivity-limited Riemann states (section 4),
// the HLLC / HLL Riemann solvers and the face Gauss weights.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "stencil.hpp"

namespace kfvm {
namespace dev {

constexpr double EPS_WENO = 1e-40;
constexpr int ERR_NONPHYSICAL = -3;

// Tile of cells per workgroup plus its R-cell halo (3D depth selectable).
template <int D, int R, int TZ_ = (D == 2 ? 1 : 4)>
struct Cfg {
    using S = Stencil<D, R>;
    static constexpr S st{};
    static constexpr int TX = D == 2 ? 16 : 8;
    static constexpr int TY = D == 2 ? 16 : 8;
    static constexpr int TZ = D == 2 ? 1 : TZ_;
    static constexpr int NT = TX * TY * TZ;
    static constexpr int HX = TX + 2 * R, HY = TY + 2 * R, HZ = D == 3 ? TZ + 2 * R : 1;
    static constexpr int HN = HX * HY * HZ;
    static constexpr int NV = D + 2;
};

// linear weights, evaluated as (1 - g_hi) g_lo and (1 - g_hi)(1 - g_lo) / (2 D)
template <int D>
__host__ __device__ constexpr double lin_w(int q)
{
    constexpr double ghi = 0.8, glo = 0.8;
    return q == 0 ? ghi : (q == 1 ? (1.0 - ghi) * glo : (1.0 - ghi) * (1.0 - glo) / (2 * D));
}

// gamma_q / gamma_0 and 1 / gamma_0 (folded at compile time)
template <int D>
__host__ __device__ constexpr double lin_ratio(int q) { return lin_w<D>(q) / lin_w<D>(0); }
template <int D>
__host__ __device__ constexpr double inv_lin0() { return 1.0 / lin_w<D>(0); }

// Blocks are handed to the 8 XCDs round-robin; give XCD k the k-th contiguous
// eighth of the tiles so neighbouring tiles share an L2.
__device__ __forceinline__ long xcd_tile(long bid, long nblk)
{
    const long per = (nblk + 7) / 8;
    const long xcd = bid % 8, local = bid / 8;
    const long t = xcd * per + local;
    return t;    // may exceed nblk - 1 for the last XCD: caller checks
}

// i in [-n, 2n): one wrap (neighbour indices of in-range cells)
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// any i: full periodic reduction (halo of a tile can reach past 2n on small grids)
__device__ __forceinline__ int wrap_any(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Average of the cell at grid coordinates (x, y, z), which may lie outside the
// grid, through the boundary conditions (the ghost fill of section 5.3, step 1):
// along a periodic axis the index wraps; past a non-periodic boundary the ghost
// is the nearest interior cell (outflow), the mirror image (reflecting) or the
// given state (inflow).  At a corner ghost the first inflow axis in x, y, z
// order gives the state, otherwise every axis clamps or mirrors; the normal
// momentum of every reflecting axis is then negated.
template <int D>
__device__ __forceinline__ void ghost_load(const double *__restrict__ U, const Geom &g, int x, int y, int z,
                                           double *u)
{
    int idx[3] = {x, y, z}, fixed = -1;
    bool flip[3] = {false, false, false};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int i = idx[a], n = g.n[a];
        if (i >= 0 && i < n) continue;
        const int side = i < 0 ? 0 : 1, kind = g.bc[a][side];
        if (kind == BC_PERIODIC) {
            const int r = i % n;
            idx[a] = r < 0 ? r + n : r;
        } else if (kind == BC_REFLECTING) {
            // (a tile's unused far corner can lie past the mirror image: clamp)
            idx[a] = min(max(side ? 2 * n - 1 - i : -1 - i, 0), n - 1);
            flip[a] = true;
        } else {
            idx[a] = side ? n - 1 : 0;
            if (kind == BC_INFLOW && fixed < 0) fixed = 2 * a + side;
        }
    }
    if (D == 2) idx[2] = 0;
    const long cell = idx[0] + (long)g.n[0] * (idx[1] + (long)g.n[1] * idx[2]);
#pragma unroll
    for (int v = 0; v < D + 2; ++v) u[v] = fixed >= 0 ? g.bc_state[fixed / 2][fixed % 2][v] : U[v * g.ncell + cell];
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (flip[a]) u[1 + a] = -u[1 + a];
}

// The cell a ghost coordinate i of axis a copies (inflow ghosts: the nearest
// interior cell), for per-cell data other than the averages.
__device__ __forceinline__ int ghost_index(const Geom &g, int a, int i)
{
    const int n = g.n[a];
    if (i >= 0 && i < n) return i;
    const int side = i < 0 ? 0 : 1, kind = g.bc[a][side];
    if (kind == BC_PERIODIC) {
        const int r = i % n;
        return r < 0 ? r + n : r;
    }
    if (kind == BC_REFLECTING) return min(max(side ? 2 * n - 1 - i : -1 - i, 0), n - 1);
    return side ? n - 1 : 0;
}

// Riemann state outside the domain at a boundary face of axis a (section 5.3,
// step 4) from the inner one: the same (outflow), normal momentum negated
// (reflecting) or the given state (inflow).
template <int D>
__device__ __forceinline__ void boundary_state(const Geom &g, int a, int side, const double *in, double *out)
{
    const int kind = g.bc[a][side];
#pragma unroll
    for (int v = 0; v < D + 2; ++v) out[v] = kind == BC_INFLOW ? g.bc_state[a][side][v] : in[v];
    if (kind == BC_REFLECTING) out[1 + a] = -in[1 + a];
}

// 1/x from the hardware estimate and two Newton-Raphson steps r <- r + r (1 - x r)
// (each squares the relative error): within an ulp or so of the rounded
// quotient, for positive normal x, at half the cost of an IEEE division.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

template <int D>
__device__ __forceinline__ double pressure(const double *u, double gam)
{
    double ke = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) ke += u[1 + a] * u[1 + a];
    return (gam - 1.0) * (u[D + 1] - 0.5 * ke * rcp64(u[0]));
}

template <int D>
__device__ __forceinline__ bool admissible(const double *u, double gam)
{
    bool ok = true;
#pragma unroll
    for (int v = 0; v < D + 2; ++v) ok = ok && isfinite(u[v]);
    return ok && u[0] > 0.0 && pressure<D>(u, gam) > 0.0;
}

// Phi^-1 at a reference state (eq. primMat; dE/du_i = rho u_i), applied to a
// vector of reconstruction variables in the row order of the dense product.
template <int D>
struct PhiInv {
    double rho, vel[D], rvel[D], uu2, inv_gm1;
    __device__ __forceinline__ void init(const double *ref, double gam)
    {
        rho = ref[0];
        const double ir = rcp64(rho);
        double uu = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) { vel[a] = ref[1 + a] * ir; uu += vel[a] * vel[a]; rvel[a] = rho * vel[a]; }
        uu2 = uu / 2.0;
        inv_gm1 = 1.0 / (gam - 1.0);
    }
    __device__ __forceinline__ void apply(const double *w, double *u) const
    {
        u[0] = w[0];
        double e = uu2 * w[0];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            u[1 + a] = vel[a] * w[0] + rho * w[1 + a];
            e += rvel[a] * w[1 + a];
        }
        u[D + 1] = e + inv_gm1 * w[D + 1];
    }
};

// Limited Riemann state: u = Phi^-1 w, then the density and pressure scalings
// about the cell average, each only when it is active (section 4.2).
template <int D>
__device__ __forceinline__ void limited_state(const double *ref, const PhiInv<D> &pi, const double *w, double th_rho,
                                              double th_p, double *u)
{
    constexpr int NV = D + 2;
    pi.apply(w, u);
    if (th_rho < 1.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = ref[v] + th_rho * (u[v] - ref[v]);
    }
    if (th_p < 1.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = ref[v] + th_p * (u[v] - ref[v]);
    }
}

// ------------------------------------------------------------------ recon ---
// Nonzero entries of Phi = dV/dU at the reference state (eq. consToLPMat).
template <int D>
struct PhiRows {
    double inv_rho, m_vel[D], e0, e_mom[D], e_e;
    __device__ __forceinline__ void init(const double *ref, double gam)
    {
        const double rho = ref[0];
        inv_rho = rcp64(rho);
        double vel[D], uu = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) { vel[a] = ref[1 + a] * inv_rho; uu += vel[a] * vel[a]; }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            m_vel[a] = -vel[a] * inv_rho;
            e_mom[a] = (1.0 - gam) * vel[a];
        }
        e0 = (gam - 1.0) * uu / 2.0;
        e_e = gam - 1.0;
    }
    // component k (runtime) of Phi u, same summation order as w_component
    __device__ __forceinline__ double row(int k, const double *u) const
    {
        if (k == 0) return u[0];
        if (k == D + 1) {
            double s = e0 * u[0];
#pragma unroll
            for (int a = 0; a < D; ++a) s += e_mom[a] * u[1 + a];
            return s + e_e * u[D + 1];
        }
        double mv = 0.0, ua = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            mv = (k == 1 + a) ? m_vel[a] : mv;
            ua = (k == 1 + a) ? u[1 + a] : ua;
        }
        const double s = mv * u[0];
        return s + inv_rho * ua;
    }
};

// Component K of W = Phi U at LDS index o, summed in the column order of the
// dense product (zero entries skipped: adding an exact zero changes nothing).
template <int D, int K, int HN>
__device__ __forceinline__ double w_component(const double (*tile)[HN], int o, const PhiRows<D> &ph)
{
    if constexpr (K == 0) {
        return tile[0][o];
    } else if constexpr (K <= D) {
        double s = ph.m_vel[K - 1] * tile[0][o];
        return s + ph.inv_rho * tile[K][o];
    } else {
        double s = ph.e0 * tile[0][o];
#pragma unroll
        for (int a = 0; a < D; ++a) s += ph.e_mom[a] * tile[1 + a][o];
        return s + ph.e_e * tile[D + 1][o];
    }
}

// ----------------------------------------------------------------- Riemann ---
// HLLC (Toro ch. 10) or HLL, wavespeeds of Batten et al. from Roe averages.
// Quotients by the densities and wave-speed differences go through rcp64.
//
// WS32 (the split-precision paths): the wave-speed estimates S_L and S_R (sound
// speeds, Roe averages) in float32 with the hardware square root and
// reciprocal; the fluxes, S* and the star state stay float64.  Both fluxes
// equal the physical flux when u_L = u_R whatever S_L and S_R are, and move by
// a perturbation of either times the jump u_R - u_L: on smooth data a change
// far below the update's float64 rounding, at a discontinuity a relative 1e-7
// of the dissipative term.  (Four float64 square roots per point are most of
// the face-flux kernel's non-FMA work.)
template <int D, int A, bool WS32 = false>
__device__ __forceinline__ void riemann(const double *uL, const double *uR, double gam, int hll, double *F)
{
    constexpr int NV = D + 2, E = D + 1;
    const double rL = uL[0], rR = uR[0];
    const double irL = rcp64(rL), irR = rcp64(rR);
    double vL[D], vR[D], qL = 0.0, qR = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        vL[b] = uL[1 + b] * irL;
        vR[b] = uR[1 + b] * irR;
        qL += uL[1 + b] * vL[b];
        qR += uR[1 + b] * vR[b];
    }
    const double pL = (gam - 1.0) * (uL[E] - 0.5 * qL), pR = (gam - 1.0) * (uR[E] - 0.5 * qR);
    const double HL = (uL[E] + pL) * irL, HR = (uR[E] + pR) * irR;
    double SL, SR;
    if constexpr (WS32) {
        const float cL = __builtin_amdgcn_sqrtf((float)(gam * pL * irL));
        const float cR = __builtin_amdgcn_sqrtf((float)(gam * pR * irR));
        const float sq = __builtin_amdgcn_sqrtf((float)(rR * irL));
        const float wL = __builtin_amdgcn_rcpf(1.f + sq), wR = sq * wL;
        float qt = 0.f, vtA = 0.f;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const float vt = wL * (float)vL[b] + wR * (float)vR[b];
            qt += vt * vt;
            if (b == A) vtA = vt;
        }
        const float Ht = wL * (float)HL + wR * (float)HR;
        const float ct = __builtin_amdgcn_sqrtf((float)(gam - 1.0) * (Ht - 0.5f * qt));
        SL = (double)fminf((float)vL[A] - cL, vtA - ct);
        SR = (double)fmaxf((float)vR[A] + cR, vtA + ct);
    } else {
        const double cL = sqrt(gam * pL * irL), cR = sqrt(gam * pR * irR);
        // Roe weights sqrt(rL) / (sqrt(rL) + sqrt(rR)) and its complement
        const double sq = sqrt(rR * irL);
        const double wL = rcp64(1.0 + sq), wR = sq * wL;
        double qt = 0.0, vtA = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const double vt = wL * vL[b] + wR * vR[b];
            qt += vt * vt;
            if (b == A) vtA = vt;
        }
        const double Ht = wL * HL + wR * HR;
        const double ct = sqrt((gam - 1.0) * (Ht - 0.5 * qt));
        SL = fmin(vL[A] - cL, vtA - ct);
        SR = fmax(vR[A] + cR, vtA + ct);
    }
    double FL[NV], FR[NV];
    FL[0] = uL[1 + A];
    FR[0] = uR[1 + A];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        FL[1 + b] = uL[1 + b] * vL[A] + (b == A ? pL : 0.0);
        FR[1 + b] = uR[1 + b] * vR[A] + (b == A ? pR : 0.0);
    }
    FL[E] = vL[A] * (uL[E] + pL);
    FR[E] = vR[A] * (uR[E] + pR);
    if (SL >= 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = FL[v];
        return;
    }
    if (SR <= 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = FR[v];
        return;
    }
    if (hll) {
        const double id = rcp64(SR - SL);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (uR[v] - uL[v])) * id;
        return;
    }
    const double dL = SL - vL[A], dR = SR - vR[A];
    const double Ss = (pR - pL + rL * vL[A] * dL - rR * vR[A] * dR) / (rL * dL - rR * dR);
    const bool left = Ss >= 0.0;
    const double SK = left ? SL : SR, rK = left ? rL : rR, pK = left ? pL : pR, irK = left ? irL : irR;
    const double dK = left ? dL : dR;
    double uK[NV], FK[NV], vK[D];
#pragma unroll
    for (int v = 0; v < NV; ++v) { uK[v] = left ? uL[v] : uR[v]; FK[v] = left ? FL[v] : FR[v]; }
#pragma unroll
    for (int b = 0; b < D; ++b) vK[b] = left ? vL[b] : vR[b];
    const double fac = rK * dK * rcp64(SK - Ss);
    double us[NV];
    us[0] = fac;
#pragma unroll
    for (int b = 0; b < D; ++b) us[1 + b] = fac * (b == A ? Ss : vK[b]);
    us[E] = fac * (uK[E] * irK + (Ss - vK[A]) * (Ss + pK * irK * rcp64(dK)));
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = FK[v] + SK * (us[v] - uK[v]);
}

// Gauss weight of transverse index gi: product over the transverse axes,
// first factor from the fastest-varying index
template <int D, int R>
__device__ __forceinline__ double face_weight(int gi)
{
    const double w2[2] = {0.5, 0.5};
    const double w3[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};
    double w = 1.0;
#pragma unroll
    for (int t = 0; t < D - 1; ++t) {
        w *= R == 2 ? w2[gi % R] : w3[gi % R];
        gi /= R;
    }
    return w;
}


// Flattener of the positivity limiter's bounds (section 4: rho_max (1 + kappa -
// kappa eta), rho_min and p_min (1 - kappa + kappa eta)).  The paper takes eta
// from a cited rule it does not state; here eta rises from 0 to 1 with the
// compression at the cell: d is the undivided velocity divergence
// sum_a (v_a(c + e_a) - v_a(c - e_a)) / 2 and c2min the least squared sound
// speed gamma p / rho of the 3^d block, and
//   eta = min(1, max(0, -d / (k1 c_min) - 1)),
// zero down to d = -k1 c_min, one from d = -2 k1 c_min.
__device__ __forceinline__ double flattener_eta(double d, double c2min, double k1)
{
    const double e = -d / (k1 * sqrt(c2min)) - 1.0;
    return fmin(1.0, fmax(0.0, e));
}

// undivided velocity divergence at tile cell lc (strides 1, sy, sz of the axes)
template <int D, typename T>
__device__ __forceinline__ double undivided_divergence(const T &tile, int lc, int sy, int sz)
{
    double d = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int s = a == 0 ? 1 : (a == 1 ? sy : sz);
        d += 0.5 * (tile[1 + a][lc + s] / tile[0][lc + s] - tile[1 + a][lc - s] / tile[0][lc - s]);
    }
    return d;
}

// GELU, tanh form (Hendrycks & Gimpel 2016), float32: 0.5 z (1 + tanh a) with
// a = sqrt(2/pi) (z + 0.044715 z^3) equals z / (1 + 2^(-2 a log2 e)), taken with
// the hardware base-2 exponential and reciprocal
__device__ __forceinline__ float gelu_f(float z)
{
    constexpr float k0 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;   // -2 sqrt(2/pi) log2(e)
    constexpr float k1 = k0 * 0.044715f;
    const float a = z * fmaf(z * z, k1, k0);
    return z * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(a));
}

__device__ __forceinline__ float gelu_grad_f(float z)
{
    const float a = 0.7978845608028654f * (z + 0.044715f * z * z * z);
    const float t = 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + __expf(2.f * a));
    const float da = 0.7978845608028654f * (1.f + 3.f * 0.044715f * z * z);
    return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * da;
}

}  // namespace dev
}  // namespace kfvm
