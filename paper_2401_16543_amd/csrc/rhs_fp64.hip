// FP64 KFVM-WENO right-hand side for gfx950.
//
// One Runge-Kutta stage is three kernels:
//   recon   one thread per cell.  The workgroup stages its tile of conserved
//           averages plus an R-cell periodic halo in LDS (the ghost fill of
//           section 5.3 is the index wrap).  Per reconstruction variable the
//           thread forms W = Phi U over S0 (section 3.4.2) in registers, applies
//           the derivative rows of every stencil's table (weights are uniform
//           across the wave: scalar loads, FP64 FMA with an SGPR operand), the
//           smoothness indicators and WENO-JS weights in FP64 (section 3.3), then
//           the point rows blended by WENO-AO (eq. wenoAOrec).  The blended
//           values go to the face buffer in reconstruction variables; the
//           positivity limiter of section 4 takes its factors from running
//           bounds of those values (re-reading them only for a cell whose
//           pressure bound fails) and stores the cell's two scaling factors.
//           3D R = 3 walks each stencil's members in chunks instead of holding
//           all 123 S0 values (recon_var_chunked).
//   flux    one thread per cell, Riemann problem at the Gauss points of each
//           of its lower faces (states rebuilt as U~ + theta (Phi^-1 w - U~)),
//           HLLC or HLL with Batten wavespeeds, Gauss sum; one flux per face.
//   update  flux difference divided by the spacing and the SSP-RK3 stage
//           combination (or the plain right-hand side).
// All arrays are struct-of-arrays over cells so that every global access is
// coalesced along x.  Blocks are remapped so that each XCD owns a contiguous
// run of tiles, which keeps halo re-reads in that XCD's L2.
#include <algorithm>
#include <mutex>

#include "device_common.hpp"

namespace kfvm {
namespace {
using namespace dev;

// Running bounds of a cell's face-point values for the positivity limiter:
// least and largest density, and, as increments over the cell's own W, the
// least pressure-row value and the sum over the velocity rows of their
// largest square.
struct FaceBounds {
    double rlo = INFINITY, rhi = -INFINITY, plo = INFINITY, v2 = 0.0;
};

// Partial sums of a weight row's dot product with the members (members
// j = 0, 1, .. mod NPS in turn), added pairwise.  A float64 FMA's result reaches
// the next FMA only after several cycles, and a single chain per row left the
// VALU waiting on it (3D 256^3, R = 2: 30.3 ms per launch with one chain, 26.8
// with two, 23.1 with four, 24.1 with eight).  The order differs from the
// left-to-right sum only in rounding.
template <int NPS>
__device__ __forceinline__ double pairwise(const double (&pa)[NPS])
{
    static_assert(NPS == 1 || NPS == 2 || NPS == 4, "partial sums combined pairwise");
    if constexpr (NPS == 4) return (pa[0] + pa[1]) + (pa[2] + pa[3]);
    else if constexpr (NPS == 2) return pa[0] + pa[1];
    else return pa[0];
}

// Reconstruction of variable K of W at every face point of one cell: smoothness
// indicators (eq. smoothIndic), nonlinear weights (eq. nlinWts) and the WENO-AO
// blend (eq. wenoAOrec), or the linear S0 value when the gate says so.
template <int D, int R, int K>
__device__ __forceinline__ void recon_var(const double (*tile)[Cfg<D, R>::HN], int lc, const double *__restrict__ wt,
                                          const PhiRows<D> &ph, const uint8_t *__restrict__ flags,
                                          double *__restrict__ face, long cell, long ncell, float *__restrict__ ratio,
                                          FaceBounds &fb)
{
    using C = Cfg<D, R>;
    using S = typename C::S;
    constexpr int NV = C::NV, N0 = S::N0, NST = S::NST, NPTS = S::NPTS, NDER = S::NDER;
    double gv[N0];
    int lcc = lc;
#pragma unroll
    for (int h = 0; h < N0; ++h) {
        const int o = lcc + C::st.off[h][0] + C::HX * (C::st.off[h][1] + C::HY * C::st.off[h][2]);
        gv[h] = w_component<D, K, C::HN>(tile, o, ph);
        // Each value is pinned where it is computed and the next group's LDS
        // index depends on it (empty asm), so at most a group of reads is in
        // flight: otherwise all N0 x NV reads are issued up front, their
        // arithmetic is sunk to the first use, and the VGPRs run out.
        asm volatile("" : "+v"(gv[h]));
        if (h % 4 == 3) asm volatile("" : "+v"(lcc) : "v"(gv[h]));
    }
    const bool use_weno = flags ? flags[(long)K * ncell + cell] != 0 : true;
    double cq[NST];
#pragma unroll
    for (int q = 0; q < NST; ++q) cq[q] = q == 0 ? 1.0 : 0.0;
    // partial sums per row dot product (pairwise): four in 3D; in 2D the extra
    // registers cost more occupancy than the shorter chains gain
    constexpr int NPS = D == 3 ? 4 : 1;
    if (use_weno) {
        double beta[NST];
#pragma unroll
        for (int q = 0; q < NST; ++q) beta[q] = 0.0;
#pragma unroll 1
        for (int a = 0; a < NDER; ++a) {
#pragma unroll
            for (int q = 0; q < NST; ++q) {
                const double *row = wt + C::st.tab[q] + (NPTS + a) * C::st.nmem[q];
                double pa[NPS] = {};
#pragma unroll
                for (int j = 0; j < C::st.nmem[q]; ++j) pa[j % NPS] += row[j] * gv[C::st.mem[q][j]];
                const double acc = pairwise<NPS>(pa);
                beta[q] += acc * acc;
            }
        }
        double om[NST], sum = 0.0;
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            om[q] = lin_w<D>(q) * rcp64(beta[q] * beta[q] + EPS_WENO);
            sum += om[q];
        }
        const double isum = rcp64(sum);
#pragma unroll
        for (int q = 0; q < NST; ++q) om[q] *= isum;
        cq[0] = om[0] * inv_lin0<D>();
#pragma unroll
        for (int q = 1; q < NST; ++q) cq[q] = om[q] - om[0] * lin_ratio<D>(q);
    }
    if (ratio) ratio[(long)K * ncell + cell] = (float)cq[0];   // omega_0 / gamma_0 (1 when linear)
    const double Wc = gv[N0 / 2];                                // the cell's own W (S0 centre)
    double v2k = 0.0;
#pragma unroll 1
    for (int s = 0; s < NPTS; ++s) {
        double v[NST];
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            v[q] = 0.0;
            if (q == 0 || use_weno) {
                const double *row = wt + C::st.tab[q] + s * C::st.nmem[q];
                double pa[NPS] = {};
#pragma unroll
                for (int j = 0; j < C::st.nmem[q]; ++j) pa[j % NPS] += row[j] * gv[C::st.mem[q][j]];
                v[q] = pairwise<NPS>(pa);
            }
        }
        double f = v[0];
        if (use_weno) {
            f = cq[0] * v[0];
#pragma unroll
            for (int q = 1; q < NST; ++q) f += cq[q] * v[q];
        }
        face[(s * NV + K) * ncell + cell] = f;
        if constexpr (K == 0) {
            fb.rlo = fmin(fb.rlo, f);
            fb.rhi = fmax(fb.rhi, f);
        } else if constexpr (K == D + 1) {
            fb.plo = fmin(fb.plo, f - Wc);
        } else {
            v2k = fmax(v2k, (f - Wc) * (f - Wc));
        }
    }
    if constexpr (K >= 1 && K <= D) fb.v2 += v2k;
    // settle the bounds here: sunk to their use they would keep every face value
    // of the variable live through the later passes
    asm volatile("" : "+v"(fb.rlo), "+v"(fb.rhi), "+v"(fb.plo), "+v"(fb.v2));
}

// 3D R = 3 holds too many S0 values per variable for the register-blocked form
constexpr bool chunked_fp64(int dim, int R) { return dim == 3 && R == 3; }

// LDS offsets (in the FP64 tile) of the chunked member slots; padding reads the centre
template <int D, int R>
struct ChunkOffsets {
    using L = ChunkLayout<D, R, FP64_CHUNK>;
    int off[L::NCH * L::CH];
    constexpr ChunkOffsets() : off{}
    {
        using C = Cfg<D, R>;
        constexpr L lay{};
        constexpr typename C::S st{};
        for (int i = 0; i < L::NCH * L::CH; ++i) {
            const int h = lay.member[i];
            off[i] = h < 0 ? 0 : st.off[h][0] + C::HX * (st.off[h][1] + C::HY * st.off[h][2]);
        }
    }
};

// Reconstruction of variable K for stencils too large to hold in VGPRs (3D
// R = 3: 123 S0 values per variable).  The members of every stencil are walked
// in chunks of FP64_CHUNK: the first pass accumulates each stencil's derivative
// rows and its smoothness indicator (eq. smoothIndic, members in the oracle's
// order), the second the WENO-AO blend (eq. wenoAOrec) of the point rows
// directly, each chunk's values scaled by its stencil's coefficient.  Weights
// come through scalar loads, one [row][chunk] block of the chunk-major table per
// chunk; stencil indices run in rolled loops, the per-stencil values move
// through small shift registers.
template <int D, int R, int K>
__device__ __forceinline__ void recon_var_chunked(const double (*tile)[Cfg<D, R>::HN], int lc,
                                                  const double *__restrict__ wch, const PhiRows<D> &ph,
                                                  const uint8_t *__restrict__ flags, double *__restrict__ face,
                                                  long cell, long ncell, float *__restrict__ ratio, FaceBounds &fb)
{
    using C = Cfg<D, R>;
    using S = typename C::S;
    using L = ChunkLayout<D, R, FP64_CHUNK>;
    constexpr int NV = C::NV, NST = S::NST, NPTS = S::NPTS, NDER = S::NDER, NROWS = S::NROWS, CH = L::CH;
    static constexpr L lay{};
    static constexpr ChunkOffsets<D, R> co{};
    const bool use_weno = flags ? flags[(long)K * ncell + cell] != 0 : true;
    double cq[NST];
#pragma unroll
    for (int q = 0; q < NST; ++q) cq[q] = q == 0 ? 1.0 : 0.0;
    if (use_weno) {
        double beta[NST];
#pragma unroll 1
        for (int q = 0; q < NST; ++q) {
            double acc[NDER];
#pragma unroll
            for (int a = 0; a < NDER; ++a) acc[a] = 0.0;
#pragma unroll 1
            for (int k = lay.cb[q]; k < lay.cb[q + 1]; ++k) {
                double gv[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) gv[j] = w_component<D, K, C::HN>(tile, lc + co.off[k * CH + j], ph);
                const double *blk = wch + (long)k * NROWS * CH + NPTS * CH;
#pragma unroll
                for (int a = 0; a < NDER; ++a)
#pragma unroll
                    for (int j = 0; j < CH; ++j) acc[a] += blk[a * CH + j] * gv[j];
            }
            double b = 0.0;
#pragma unroll
            for (int a = 0; a < NDER; ++a) b += acc[a] * acc[a];
#pragma unroll
            for (int i = 0; i + 1 < NST; ++i) beta[i] = beta[i + 1];
            beta[NST - 1] = b;
        }
        double om[NST], sum = 0.0;
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            om[q] = lin_w<D>(q) * rcp64(beta[q] * beta[q] + EPS_WENO);
            sum += om[q];
        }
        const double isum = rcp64(sum);
#pragma unroll
        for (int q = 0; q < NST; ++q) om[q] *= isum;
        cq[0] = om[0] * inv_lin0<D>();
#pragma unroll
        for (int q = 1; q < NST; ++q) cq[q] = om[q] - om[0] * lin_ratio<D>(q);
    }
    if (ratio) ratio[(long)K * ncell + cell] = (float)cq[0];   // omega_0 / gamma_0 (1 when linear)
    const double Wc = w_component<D, K, C::HN>(tile, lc, ph);
    double f[NPTS];
#pragma unroll
    for (int s = 0; s < NPTS; ++s) f[s] = 0.0;
    const int qend = use_weno ? NST : 1;
#pragma unroll 1
    for (int q = 0; q < qend; ++q) {
        const double c = cq[0];
#pragma unroll
        for (int i = 0; i + 1 < NST; ++i) cq[i] = cq[i + 1];
#pragma unroll 1
        for (int k = lay.cb[q]; k < lay.cb[q + 1]; ++k) {
            double gv[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) gv[j] = c * w_component<D, K, C::HN>(tile, lc + co.off[k * CH + j], ph);
            const double *blk = wch + (long)k * NROWS * CH;
#pragma unroll
            for (int s = 0; s < NPTS; ++s)
#pragma unroll
                for (int j = 0; j < CH; ++j) f[s] += blk[s * CH + j] * gv[j];
        }
    }
    double v2k = 0.0;
#pragma unroll
    for (int s = 0; s < NPTS; ++s) {
        face[(s * NV + K) * ncell + cell] = f[s];
        if constexpr (K == 0) {
            fb.rlo = fmin(fb.rlo, f[s]);
            fb.rhi = fmax(fb.rhi, f[s]);
        } else if constexpr (K == D + 1) {
            fb.plo = fmin(fb.plo, f[s] - Wc);
        } else {
            v2k = fmax(v2k, (f[s] - Wc) * (f[s] - Wc));
        }
    }
    if constexpr (K >= 1 && K <= D) fb.v2 += v2k;
    // settle the bounds here: sunk to their use they would keep every face value
    // of the variable live through the later passes
    asm volatile("" : "+v"(fb.rlo), "+v"(fb.rhi), "+v"(fb.plo), "+v"(fb.v2));
}

template <int D, int R, int... K>
__device__ __forceinline__ void recon_all_vars(const double (*tile)[Cfg<D, R>::HN], int lc, const double *__restrict__ wt,
                                               const double *__restrict__ wch, const PhiRows<D> &ph,
                                               const uint8_t *__restrict__ flags, double *__restrict__ face, long cell,
                                               long ncell, float *ratio, FaceBounds &fb,
                                               std::integer_sequence<int, K...>)
{
    // one pass per variable; the empty asm keeps each pass's LDS reads from
    // being hoisted into a single register-hungry prologue
    if constexpr (chunked_fp64(D, R))
        ((recon_var_chunked<D, R, K>(tile, [&] { int l = lc; asm volatile("" : "+v"(l)); return l; }(), wch, ph,
                                     flags, face, cell, ncell, ratio, fb)),
         ...);
    else
        ((recon_var<D, R, K>(tile, [&] { int l = lc; asm volatile("" : "+v"(l)); return l; }(), wt, ph, flags, face,
                             cell, ncell, ratio, fb)),
         ...);
}

template <int D, int R>
__global__ __launch_bounds__((Cfg<D, R>::NT)) void k_recon(const double *__restrict__ U, const double *__restrict__ wt,
                                                         const double *__restrict__ wch,
                                                         double *__restrict__ face, double *__restrict__ theta,
                                                         int *__restrict__ err, const uint8_t *__restrict__ flags,
                                                         Geom g, Limiter lim, float *__restrict__ ratio)
{
    using C = Cfg<D, R>;
    using S = typename C::S;
    constexpr int NV = C::NV, NPTS = S::NPTS;
    __shared__ double tile[NV][C::HN];

    const int nbx = (g.n[0] + C::TX - 1) / C::TX, nby = (g.n[1] + C::TY - 1) / C::TY;
    const int nbz = D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1;
    const long nblk = (long)nbx * nby * nbz;
    const long t = xcd_tile(blockIdx.x, nblk);
    if (t >= nblk) return;
    const int bx = (int)(t % nbx), by = (int)((t / nbx) % nby), bz = (int)(t / ((long)nbx * nby));
    const int x0 = bx * C::TX - R, y0 = by * C::TY - R, z0 = D == 3 ? bz * C::TZ - R : 0;

    // tile + halo, periodic wrap (the ghost fill)
    // a single conditional wrap reaches every halo index once the grid is at
    // least a tile plus R wide along each axis; smaller grids take the modulo
    const bool near = g.n[0] >= C::TX + R && g.n[1] >= C::TY + R && (D == 2 || g.n[2] >= C::TZ + R);
    // only a tile whose halo crosses a non-periodic boundary needs the ghost fill
    bool ghosts = false;
    if (!g.periodic) {
        const int o[3] = {x0, y0, z0}, h[3] = {C::HX, C::HY, C::HZ};
#pragma unroll
        for (int a = 0; a < D; ++a)
            ghosts = ghosts || (g.bc[a][0] != BC_PERIODIC && (o[a] < 0 || o[a] + h[a] > g.n[a]));
    }
    for (int i = threadIdx.x; i < C::HN; i += C::NT) {
        const int hx = i % C::HX, hy = (i / C::HX) % C::HY, hz = i / (C::HX * C::HY);
        if (ghosts) {
            // non-periodic axes: ghost cells by the boundary conditions
            double u[NV];
            ghost_load<D>(U, g, x0 + hx, y0 + hy, D == 3 ? z0 + hz : 0, u);
#pragma unroll
            for (int v = 0; v < NV; ++v) tile[v][i] = u[v];
            continue;
        }
        const int gx = near ? wrapi(x0 + hx, g.n[0]) : wrap_any(x0 + hx, g.n[0]);
        const int gy = near ? wrapi(y0 + hy, g.n[1]) : wrap_any(y0 + hy, g.n[1]);
        const int gz = D == 3 ? (near ? wrapi(z0 + hz, g.n[2]) : wrap_any(z0 + hz, g.n[2])) : 0;
        const long cell = gx + (long)g.n[0] * (gy + (long)g.n[1] * gz);
#pragma unroll
        for (int v = 0; v < NV; ++v) tile[v][i] = U[v * g.ncell + cell];
    }
    __syncthreads();

    const int tx = threadIdx.x % C::TX, ty = (threadIdx.x / C::TX) % C::TY, tz = threadIdx.x / (C::TX * C::TY);
    const int cx = bx * C::TX + tx, cy = by * C::TY + ty, cz = D == 3 ? bz * C::TZ + tz : 0;
    if (cx >= g.n[0] || cy >= g.n[1] || (D == 3 && cz >= g.n[2])) return;
    const long cell = cx + (long)g.n[0] * (cy + (long)g.n[1] * cz);
    const int lc = (tx + R) + C::HX * ((ty + R) + C::HY * (D == 3 ? tz + R : 0));

    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = tile[v][lc];
    const double gam = g.gamma;
    if (!admissible<D>(ref, gam)) {
        *err = ERR_NONPHYSICAL;
        theta[cell] = 1.0;
        theta[g.ncell + cell] = 1.0;
#pragma unroll 1
        for (int s = 0; s < NPTS * NV; ++s) face[s * g.ncell + cell] = 0.0;
        return;
    }

    // Phi = dV/dU at the cell's own average (eq. consToLPMat): its nonzero
    // entries, applied row by row with one compile-time pass per variable
    PhiRows<D> ph;
    ph.init(ref, gam);
    FaceBounds fb;
    recon_all_vars<D, R>(tile, lc, wt, wch, ph, flags, face, cell, g.ncell, ratio, fb,
                         std::make_integer_sequence<int, NV>{});

    // positivity limiter (section 4) on the cell's Riemann states
    double th_rho = 1.0, th_p = 1.0;
    if (lim.on) {
        double rmax = -INFINITY, rmin = INFINITY, pmin = INFINITY, c2min = INFINITY;
        const bool flat = lim.flat_k1 > 0.0;
        bool ok = true;
#pragma unroll 1
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll 1
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll 1
                for (int dx = -1; dx <= 1; ++dx) {
                    const int o = lc + dx + C::HX * (dy + C::HY * dz);
                    double un[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) un[v] = tile[v][o];
                    ok = ok && admissible<D>(un, gam);
                    const double pn = pressure<D>(un, gam);
                    rmax = fmax(rmax, un[0]);
                    rmin = fmin(rmin, un[0]);
                    pmin = fmin(pmin, pn);
                    if (flat) c2min = fmin(c2min, gam * pn / un[0]);
                }
        if (!ok) *err = ERR_NONPHYSICAL;
        // bounds widened by kappa (1 - eta)
        const double f =
            flat ? lim.kappa * (1.0 - flattener_eta(undivided_divergence<D>(tile, lc, C::HX, C::HX * C::HY), c2min,
                                                    lim.flat_k1))
                 : lim.kappa;
        rmax *= 1.0 + f;
        rmin *= 1.0 - f;
        pmin *= 1.0 - f;
        PhiInv<D> pi;
        pi.init(ref, gam);
        // density scaling (eq. ppThetaRho), only the violated side of each bound;
        // the smallest ratio of a side is taken at its extreme point value (row
        // 0 of Phi^-1 is e_0: the reconstructed density itself)
        const double r0 = ref[0];
        if (fb.rlo < rmin) th_rho = fmin(th_rho, (r0 - rmin) / (r0 - fb.rlo));
        if (fb.rhi > rmax) th_rho = fmin(th_rho, (rmax - r0) / (fb.rhi - r0));
        // pressure at a point, exactly: p = p~ + th dw_p - (gamma-1)/2 th^2 rho~^2 |dw_u|^2 / rho
        // (dw: its increments in reconstruction variables).  The least dw_p and
        // rho and the largest |dw_u|^2 bound every point from below; only a cell
        // whose bound falls under pmin takes the per-point test and bisection.
        const double rlo = r0 + th_rho * (fb.rlo - r0);
        const double plow = pressure<D>(ref, gam) + th_rho * fb.plo -
                            0.5 * (gam - 1.0) * th_rho * th_rho * r0 * r0 * fb.v2 * rcp64(rlo);
        // pressure scaling (eq. thetapRoot, eq. thetaP): 60 bisection steps
#pragma unroll 1
        for (int s = 0; s < (rlo > 0.0 && plow >= pmin ? 0 : NPTS); ++s) {
            double w[NV], u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = face[(s * NV + v) * g.ncell + cell];
            limited_state<D>(ref, pi, w, th_rho, 1.0, u);
            if (pressure<D>(u, gam) >= pmin) continue;
            double lo = 0.0, hi = 1.0;
#pragma unroll 1
            for (int it = 0; it < 60; ++it) {
                const double m = 0.5 * (lo + hi);
                double um[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) um[v] = ref[v] + m * (u[v] - ref[v]);
                if (pressure<D>(um, gam) >= pmin) lo = m; else hi = m;
            }
            th_p = fmin(th_p, lo);
        }
    }
    theta[cell] = th_rho;
    theta[g.ncell + cell] = th_p;
}

// ------------------------------------------------------------------- flux ---
template <int D, int R, int A>
__device__ __forceinline__ void lower_face_flux(const double *__restrict__ U, const double *__restrict__ face,
                                                const double *__restrict__ theta, const Geom &g, long cell,
                                                long lower, int hll, double *Fbar)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NG = S::NG;
    double refL[NV], refR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { refL[v] = U[v * g.ncell + lower]; refR[v] = U[v * g.ncell + cell]; }
    const double trL = theta[lower], tpL = theta[g.ncell + lower];
    const double trR = theta[cell], tpR = theta[g.ncell + cell];
    PhiInv<D> piL, piR;
    piL.init(refL, g.gamma);
    piR.init(refR, g.gamma);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fbar[v] = 0.0;
#pragma unroll 1
    for (int gi = 0; gi < NG; ++gi) {
        double wL[NV], wR[NV], uL[NV], uR[NV], F[NV];
        const int sL = (2 * A + 1) * NG + gi, sR = (2 * A + 0) * NG + gi;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            wL[v] = face[(sL * NV + v) * g.ncell + lower];
            wR[v] = face[(sR * NV + v) * g.ncell + cell];
        }
        limited_state<D>(refL, piL, wL, trL, tpL, uL);
        limited_state<D>(refR, piR, wR, trR, tpR, uR);
        riemann<D, A>(uL, uR, g.gamma, hll, F);
        const double w = face_weight<D, R>(gi);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[v] += w * F[v];
    }
}

// Flux through the face of `cell` on this side of axis A when it lies on a
// non-periodic boundary: the cell's limited state inside, the state the
// boundary condition gives outside (section 5.3, step 4).
template <int D, int R, int A>
__device__ __forceinline__ void boundary_face_flux(const double *__restrict__ U, const double *__restrict__ face,
                                                   const double *__restrict__ theta, const Geom &g, long cell,
                                                   int side, int hll, double *Fbar)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NG = S::NG;
    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = U[v * g.ncell + cell];
    const double tr = theta[cell], tp = theta[g.ncell + cell];
    PhiInv<D> pi;
    pi.init(ref, g.gamma);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fbar[v] = 0.0;
#pragma unroll 1
    for (int gi = 0; gi < NG; ++gi) {
        double w[NV], in[NV], out[NV], F[NV];
        const int s = (2 * A + side) * NG + gi;
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = face[(s * NV + v) * g.ncell + cell];
        limited_state<D>(ref, pi, w, tr, tp, in);
        boundary_state<D>(g, A, side, in, out);
        if (side) riemann<D, A>(in, out, g.gamma, hll, F);
        else riemann<D, A>(out, in, g.gamma, hll, F);
        const double wt = face_weight<D, R>(gi);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[v] += wt * F[v];
    }
}

// The fluxes of axis A at `cell`: through its lower face into fbar and, on an
// upper non-periodic boundary, through its upper face into fbar_top.
template <int D, int R, int A>
__device__ __forceinline__ bool axis_fluxes(const double *__restrict__ U, const double *__restrict__ face,
                                            const double *__restrict__ theta, double *__restrict__ fbar,
                                            double *__restrict__ fbar_top, long plane, const Geom &g, long cell,
                                            const int *c, int hll)
{
    constexpr int NV = D + 2;
    double F[NV];
    bool ok = true;
    if (!g.periodic && c[A] == 0 && g.bc[A][0] != BC_PERIODIC) {
        boundary_face_flux<D, R, A>(U, face, theta, g, cell, 0, hll, F);
    } else {
        int lc[3] = {c[0], c[1], c[2]};
        lc[A] = wrapi(c[A] - 1, g.n[A]);
        const long lower = lc[0] + (long)g.n[0] * (lc[1] + (long)g.n[1] * lc[2]);
        lower_face_flux<D, R, A>(U, face, theta, g, cell, lower, hll, F);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) { fbar[(A * NV + v) * g.ncell + cell] = F[v]; ok = ok && isfinite(F[v]); }
    if (!g.periodic && c[A] == g.n[A] - 1 && g.bc[A][1] != BC_PERIODIC) {
        boundary_face_flux<D, R, A>(U, face, theta, g, cell, 1, hll, F);
        const long pi = plane_index(A, c[0], c[1], c[2], g.n);
#pragma unroll
        for (int v = 0; v < NV; ++v) { fbar_top[(A * NV + v) * plane + pi] = F[v]; ok = ok && isfinite(F[v]); }
    }
    return ok;
}

template <int D, int R>
__global__ __launch_bounds__(256) void k_flux(const double *__restrict__ U, const double *__restrict__ face,
                                              const double *__restrict__ theta, double *__restrict__ fbar,
                                              double *__restrict__ fbar_top, long plane, int *__restrict__ err,
                                              Geom g, int hll)
{
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const int c[3] = {(int)(cell % g.n[0]), (int)((cell / g.n[0]) % g.n[1]), (int)(cell / ((long)g.n[0] * g.n[1]))};
    bool ok = axis_fluxes<D, R, 0>(U, face, theta, fbar, fbar_top, plane, g, cell, c, hll);
    ok = axis_fluxes<D, R, 1>(U, face, theta, fbar, fbar_top, plane, g, cell, c, hll) && ok;
    if constexpr (D == 3) ok = axis_fluxes<D, R, 2>(U, face, theta, fbar, fbar_top, plane, g, cell, c, hll) && ok;
    if (!ok) *err = ERR_NONPHYSICAL;
}

// ----------------------------------------------------------------- update ---
// U0 and out may be the same array (the last stage of a step in place): each
// thread reads U0[i] before it writes out[i], so they carry no __restrict__.
// guard (optional): nothing is written while *guard != 0, which leaves `out`
// as it was when an earlier kernel of the step met a non-physical state.
template <int D>
__global__ __launch_bounds__(256) void k_update(const double *__restrict__ fbar, const double *__restrict__ fbar_top,
                                                long plane, const double *U0, const double *__restrict__ Uin,
                                                double *out, Geom g, int stage, double dt, const int *guard)
{
    constexpr int NV = D + 2;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    if (guard && *guard != 0) return;
    const int cx = (int)(cell % g.n[0]), cy = (int)((cell / g.n[0]) % g.n[1]);
    const int cz = (int)(cell / ((long)g.n[0] * g.n[1]));
    const int c[3] = {cx, cy, cz};
    long up[3];
    up[0] = wrapi(cx + 1, g.n[0]) + (long)g.n[0] * (cy + (long)g.n[1] * cz);
    up[1] = cx + (long)g.n[0] * (wrapi(cy + 1, g.n[1]) + (long)g.n[1] * cz);
    up[2] = D == 3 ? cx + (long)g.n[0] * (cy + (long)g.n[1] * wrapi(cz + 1, g.n[2])) : 0;
    // an upper non-periodic boundary face has its own flux
    bool top[3];
    long ptop[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        top[a] = !g.periodic && c[a] == g.n[a] - 1 && g.bc[a][1] != BC_PERIODIC;
        ptop[a] = top[a] ? plane_index(a, cx, cy, cz, g.n) : 0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double Fp = top[a] ? fbar_top[(a * NV + v) * plane + ptop[a]] : fbar[(a * NV + v) * g.ncell + up[a]];
            const double Fm = fbar[(a * NV + v) * g.ncell + cell];
            acc -= (Fp - Fm) / g.dx[a];
        }
        const long i = v * g.ncell + cell;
        double r;
        if (stage == 0) r = acc;
        else if (stage == 1) r = Uin[i] + dt * acc;
        else if (stage == 2) r = 0.75 * U0[i] + 0.25 * (Uin[i] + dt * acc);
        else if (stage == 3) r = U0[i] / 3.0 + 2.0 / 3.0 * (Uin[i] + dt * acc);
        else r = 2.0 / 3.0 * U0[i] + 1.0 / 3.0 * (Uin[i] + dt * acc);   // third stage of SSP(4,3)
        out[i] = r;
    }
}

// ------------------------------------------------------------ face states ---
template <int D, int R>
__global__ __launch_bounds__(256) void k_states(const double *__restrict__ U, const double *__restrict__ face,
                                                const double *__restrict__ theta, double *__restrict__ states,
                                                Geom g)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NPTS = S::NPTS;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = U[v * g.ncell + cell];
    const double tr = theta[cell], tp = theta[g.ncell + cell];
    PhiInv<D> pi;
    pi.init(ref, g.gamma);
#pragma unroll 1
    for (int s = 0; s < NPTS; ++s) {
        double w[NV], u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = face[(s * NV + v) * g.ncell + cell];
        limited_state<D>(ref, pi, w, tr, tp, u);
#pragma unroll
        for (int v = 0; v < NV; ++v) states[(cell * NPTS + s) * NV + v] = u[v];
    }
}

// -------------------------------------------------------------------- CFL ---
template <int D>
__global__ __launch_bounds__(256) void k_cfl_partial(const double *__restrict__ U, double *__restrict__ part,
                                                     int *__restrict__ err, Geom g)
{
    constexpr int NV = D + 2;
    __shared__ double red[3][256 / 64];
    double m = 0.0, rmin = INFINITY, pmin = INFINITY;    // also the least density and pressure
    for (long cell = (long)blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncell;
         cell += (long)gridDim.x * blockDim.x) {
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + cell];
        if (!admissible<D>(u, g.gamma)) { *err = ERR_NONPHYSICAL; continue; }
        const double p = pressure<D>(u, g.gamma);
        rmin = fmin(rmin, u[0]);
        pmin = fmin(pmin, p);
        const double cs = sqrt(g.gamma * p / u[0]);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double r = (fabs(u[1 + a] / u[0]) + cs) / g.dx[a];
            s = g.cfl_max_axis ? fmax(s, r) : s + r;
        }
        m = fmax(m, s);
    }
    // wave64 max (min), then across the block's waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_xor(m, off, 64));
        rmin = fmin(rmin, __shfl_xor(rmin, off, 64));
        pmin = fmin(pmin, __shfl_xor(pmin, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = m;
        red[1][threadIdx.x >> 6] = rmin;
        red[2][threadIdx.x >> 6] = pmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0][0], a = red[1][0], b = red[2][0];
#pragma unroll
        for (int i = 1; i < 256 / 64; ++i) {
            r = fmax(r, red[0][i]);
            a = fmin(a, red[1][i]);
            b = fmin(b, red[2][i]);
        }
        part[blockIdx.x] = r;
        part[gridDim.x + blockIdx.x] = a;
        part[2 * gridDim.x + blockIdx.x] = b;
    }
}

// dt[0] = cfl / (largest ratio), dt[1] the least density, dt[2] the least pressure
__global__ __launch_bounds__(256) void k_cfl_final(const double *__restrict__ part, int nparts, double cfl,
                                                   double *__restrict__ dt)
{
    __shared__ double red[3][256 / 64];
    double m = 0.0, a = INFINITY, b = INFINITY;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        m = fmax(m, part[i]);
        a = fmin(a, part[nparts + i]);
        b = fmin(b, part[2 * nparts + i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_xor(m, off, 64));
        a = fmin(a, __shfl_xor(a, off, 64));
        b = fmin(b, __shfl_xor(b, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = m;
        red[1][threadIdx.x >> 6] = a;
        red[2][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0][0], ra = red[1][0], rb = red[2][0];
#pragma unroll
        for (int i = 1; i < 256 / 64; ++i) {
            r = fmax(r, red[0][i]);
            ra = fmin(ra, red[1][i]);
            rb = fmin(rb, red[2][i]);
        }
        dt[0] = cfl / r;
        dt[1] = ra;
        dt[2] = rb;
    }
}

// --------------------------------------------------- SSP(4,3,2) error norm ---
// Sum over (variable, cell) of ((U+ - (2 U3 - U)) / (atol + rtol max(|U|, |U+|)))^2:
// per-block partial sums in a fixed order (grid-stride, then a tree in LDS),
// then one block adds the partials, so the norm does not depend on timing.
__global__ __launch_bounds__(256) void k_err_partial(const double *__restrict__ U, const double *__restrict__ U3,
                                                     const double *__restrict__ Up, long M, double atol, double rtol,
                                                     double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x) {
        const double uhat = 2.0 * U3[i] - U[i];
        const double sc = atol + rtol * fmax(fabs(U[i]), fabs(Up[i]));
        const double e = (Up[i] - uhat) / sc;
        acc += e * e;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_err_final(const double *__restrict__ part, int nparts, long M,
                                                   double *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0] / (double)M);
}

// ------------------------------------------------------------ statistics ---
__global__ __launch_bounds__(256) void k_count_stats(const double *__restrict__ theta,
                                                     const uint8_t *__restrict__ flags, long ncell, int nvar,
                                                     unsigned long long *__restrict__ counts)
{
    unsigned long long lim = 0, weno = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += (long)gridDim.x * blockDim.x) {
        lim += (theta[i] < 1.0 || theta[ncell + i] < 1.0) ? 1 : 0;
        if (flags)
            for (int v = 0; v < nvar; ++v) weno += flags[(long)v * ncell + i] != 0 ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lim += __shfl_xor(lim, off, 64);
        weno += __shfl_xor(weno, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], lim);
        atomicAdd(&counts[1], weno);
    }
}

template <int D, int R>
hipError_t rhs_impl(const Geom &g, const Tables &t, const Work &w, const Limiter &lim, int riemann,
                    const double *U0, const double *Uin, double *out, int stage, double dt, hipStream_t s,
                    const Timing &tm)
{
    auto mark = [&](int kind, int begin) { if (tm.on) tm.record(tm.self, kind, s, begin); };
    using C = Cfg<D, R>;
    const long nblk = (long)((g.n[0] + C::TX - 1) / C::TX) * ((g.n[1] + C::TY - 1) / C::TY) *
                      (D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1);
    const long grid = ((nblk + 7) / 8) * 8;   // every XCD gets the same number of slots
    mark(KT_RECON, 1);
    hipLaunchKernelGGL((k_recon<D, R>), dim3((unsigned)grid), dim3(C::NT), 0, s, Uin, t.w, t.wch, w.face, w.theta, w.err,
                       w.flags_in, g, lim, (float *)nullptr);
    mark(KT_RECON, 0);
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    mark(KT_FLUX, 1);
    hipLaunchKernelGGL((k_flux<D, R>), dim3(nb), dim3(256), 0, s, Uin, w.face, w.theta, w.fbar, w.fbar_top, w.plane,
                       w.err, g, riemann);
    mark(KT_FLUX, 0);
    mark(KT_UPDATE, 1);
    hipLaunchKernelGGL((k_update<D>), dim3(nb), dim3(256), 0, s, w.fbar, w.fbar_top, w.plane, U0, Uin, out, g, stage,
                       dt, w.guard);
    mark(KT_UPDATE, 0);
    return hipGetLastError();
}

template <int D, int R>
hipError_t states_impl(const Geom &g, const Tables &t, const Work &w, const Limiter &lim, const double *U,
                       double *states, hipStream_t s)
{
    using C = Cfg<D, R>;
    const long nblk = (long)((g.n[0] + C::TX - 1) / C::TX) * ((g.n[1] + C::TY - 1) / C::TY) *
                      (D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1);
    const long grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_recon<D, R>), dim3((unsigned)grid), dim3(C::NT), 0, s, U, t.w, t.wch, w.face, w.theta, w.err,
                       w.flags_in, g, lim, (float *)nullptr);
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    hipLaunchKernelGGL((k_states<D, R>), dim3(nb), dim3(256), 0, s, U, w.face, w.theta, states, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_fp64(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                           int riemann, const double *U0, const double *Uin, double *out, int stage, double dt,
                           hipStream_t s, const Timing &tm)
{
    if (dim == 2 && R == 2) return rhs_impl<2, 2>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, s, tm);
    if (dim == 2 && R == 3) return rhs_impl<2, 3>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, s, tm);
    if (dim == 3 && R == 2) return rhs_impl<3, 2>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, s, tm);
    if (dim == 3 && R == 3) return rhs_impl<3, 3>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, s, tm);
    return hipErrorInvalidValue;
}

template <int D, int R>
hipError_t ratio_impl(const Geom &g, const Tables &t, const Work &w, const Limiter &lim, const double *U, float *ratio,
                      hipStream_t s)
{
    using C = Cfg<D, R>;
    const long nblk = (long)((g.n[0] + C::TX - 1) / C::TX) * ((g.n[1] + C::TY - 1) / C::TY) *
                      (D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1);
    const long grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_recon<D, R>), dim3((unsigned)grid), dim3(C::NT), 0, s, U, t.w, t.wch, w.face, w.theta, w.err,
                       (const uint8_t *)nullptr, g, lim, ratio);
    return hipGetLastError();
}

hipError_t launch_recon_ratio(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                              const double *U, float *ratio, hipStream_t s)
{
    if (dim == 2 && R == 2) return ratio_impl<2, 2>(g, t, w, lim, U, ratio, s);
    if (dim == 2 && R == 3) return ratio_impl<2, 3>(g, t, w, lim, U, ratio, s);
    if (dim == 3 && R == 2) return ratio_impl<3, 2>(g, t, w, lim, U, ratio, s);
    if (dim == 3 && R == 3) return ratio_impl<3, 3>(g, t, w, lim, U, ratio, s);
    return hipErrorInvalidValue;
}

hipError_t launch_ssp_error(const double *U, const double *U3, const double *Up, long M, double atol, double rtol,
                            double *part, double *out, hipStream_t s)
{
    const int nb = (int)std::min<long>((M + 255) / 256, 1024);
    hipLaunchKernelGGL(k_err_partial, dim3((unsigned)nb), dim3(256), 0, s, U, U3, Up, M, atol, rtol, part);
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(256), 0, s, part, nb, M, out);
    return hipGetLastError();
}

hipError_t launch_count_stats(const double *theta, const uint8_t *flags, long ncell, int nvar,
                              unsigned long long *counts, hipStream_t s)
{
    const long nb = std::min<long>((ncell + 255) / 256, 4096);
    hipLaunchKernelGGL(k_count_stats, dim3((unsigned)nb), dim3(256), 0, s, theta, flags, ncell, nvar, counts);
    return hipGetLastError();
}

hipError_t launch_update(int dim, const Geom &g, const Work &w, const double *U0, const double *Uin, double *out,
                         int stage, double dt, hipStream_t s)
{
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (dim == 2)
        hipLaunchKernelGGL((k_update<2>), dim3(nb), dim3(256), 0, s, w.fbar, w.fbar_top, w.plane, U0, Uin, out, g,
                           stage, dt, w.guard);
    else
        hipLaunchKernelGGL((k_update<3>), dim3(nb), dim3(256), 0, s, w.fbar, w.fbar_top, w.plane, U0, Uin, out, g,
                           stage, dt, w.guard);
    return hipGetLastError();
}

namespace {
__global__ void k_err_reset(int *word) { *word = 0; }
__global__ void k_err_merge(int *sticky, const int *word)
{
    if (*word != 0) *sticky = *word;
}
}  // namespace

hipError_t launch_err_reset(int *word, hipStream_t s)
{
    hipLaunchKernelGGL(k_err_reset, dim3(1), dim3(1), 0, s, word);
    return hipGetLastError();
}

hipError_t launch_err_merge(int *sticky, const int *word, hipStream_t s)
{
    hipLaunchKernelGGL(k_err_merge, dim3(1), dim3(1), 0, s, sticky, word);
    return hipGetLastError();
}

hipError_t launch_face_states(int dim, int R, const Geom &g, const Tables &t, const Work &w, const Limiter &lim,
                              const double *U, double *states, hipStream_t s)
{
    if (dim == 2 && R == 2) return states_impl<2, 2>(g, t, w, lim, U, states, s);
    if (dim == 2 && R == 3) return states_impl<2, 3>(g, t, w, lim, U, states, s);
    if (dim == 3 && R == 2) return states_impl<3, 2>(g, t, w, lim, U, states, s);
    if (dim == 3 && R == 3) return states_impl<3, 3>(g, t, w, lim, U, states, s);
    return hipErrorInvalidValue;
}

static hipError_t cfl_launch(int dim, const Geom &g, double *part, int *err, const double *U, double cfl,
                             double *dt_dev, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL((k_cfl_partial<2>), dim3(CFL_PARTS), dim3(256), 0, s, U, part, err, g);
    else
        hipLaunchKernelGGL((k_cfl_partial<3>), dim3(CFL_PARTS), dim3(256), 0, s, U, part, err, g);
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, s, part, CFL_PARTS, cfl, dt_dev);
    return hipGetLastError();
}

hipError_t launch_cfl(int dim, const Geom &g, const Work &w, const double *U, double cfl, double *dt_dev,
                      hipStream_t s)
{
    return cfl_launch(dim, g, w.cfl_part, w.err, U, cfl, dt_dev, s);
}

// ---------------------------------------------- allocation-free CFL reduction ---
// The per-block partials of the allocation-free CFL call live in this
// file-scope device array rather than in context memory: every GPU that loads
// the library holds its own copy until the process ends, and every call on
// that GPU shares it.  Each call overwrites all 3 x CFL_PARTS entries before
// reading any, so nothing needs clearing; calls that overlap on one GPU race.
// In host code the array's name is only a stand-in: kernels are given the
// device address that cfl_scratch_address looks up once per device.
static __device__ __align__(256) double scratch[CFL_SCRATCH_DOUBLES];

hipError_t cfl_scratch_address(double **ptr)
{
    static std::mutex mu;
    static double *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_cfl_scratch(int dim, const Geom &g, double *scratch_dev, int *err, const double *U, double cfl,
                              double *out_dev, hipStream_t s)
{
    static_assert(3 * CFL_PARTS <= CFL_SCRATCH_DOUBLES, "the partials must fit the scratch array");
    return cfl_launch(dim, g, scratch_dev, err, U, cfl, out_dev, s);
}

}  // namespace kfvm
