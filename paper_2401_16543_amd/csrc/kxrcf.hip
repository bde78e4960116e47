// KXRCF troubled-cell indicator (section 3.5, eq. kxrcf) for gfx950, FP64: the
// first pass of the two-pass Riemann-state procedure of section 5.3.
//
//   jump   one thread per cell.  The workgroup stages its tile of conserved
//          averages in LDS with a periodic halo of R cells below and R + 1
//          above (the upper neighbour's stencil).  Per axis the thread forms the
//          unlimited states (the S0 point rows applied to the conserved averages
//          themselves) at the Gauss points of the face it shares with its upper
//          neighbour, from both sides in turn: its own upper-face rows over its
//          S0, then the neighbour's lower-face rows over the neighbour's S0.  Each
//          average read from LDS feeds the n_g point accumulators of that side;
//          the weights are uniform across the wave (scalar loads from a table
//          laid out [axis][side][member][point]).  The face keeps the largest
//          |q+ - q-| of the entropy q = p / rho^gamma, or infinity when a state
//          is not admissible.  Both sides' q are formed as p (rho / rho_c)^-gamma
//          with rho_c the cell's average density, by a binomial series when
//          rho is within 1/32 of rho_c (pow otherwise), and the face maximum is
//          scaled by rho_c^-gamma once.  Reads of a member group are issued one
//          group ahead of the FMAs that use them.
//   boundary  (non-periodic grids) one thread per boundary face: the jump
//          between the cell's unlimited state and the outer state the
//          boundary condition gives.
//   flags  one thread per cell: the largest jump over its 2d faces against
//          Delta^m times the entropy of its own average.  Every variable of a
//          flagged cell takes WENO-AO in the reconstruction that follows, the
//          other cells the linear S0 value.
#include "device_common.hpp"

namespace kfvm {
namespace {
using namespace dev;

constexpr int KX_SERIES_K = 15;
struct KxSeries {
    double a[KX_SERIES_K];   // a_k = (1 - k - gamma) / k
    double xmax;             // 1/32 for gamma <= 10, else -1 (pow everywhere)
};

template <int D, int R>
struct KxCfg {
    using S = Stencil<D, R>;
    static constexpr S st{};
    // 3D order 7: a wider tile (512 threads, 152 KB of LDS) for a better halo
    // ratio and two waves per SIMD
    static constexpr int TX = D == 2 ? 16 : (R == 3 ? 16 : 8);
    static constexpr int TY = D == 2 ? 16 : 8;
    static constexpr int TZ = D == 2 ? 1 : 4;
    static constexpr int NT = TX * TY * TZ;
    static constexpr int HX = TX + 2 * R + 1, HY = TY + 2 * R + 1, HZ = D == 3 ? TZ + 2 * R + 1 : 1;
    static constexpr int HN = HX * HY * HZ;
    static constexpr int NV = D + 2, NG = S::NG, N0 = S::N0;
    static constexpr int MG = NG >= 9 ? 1 : 2;   // members per group of reads
    static constexpr bool PIN_W = NG * MG <= 8;   // two groups of weights fit the scalar registers
};

// q = p / rho^gamma of a point state; false when the state is not admissible
template <int D>
__device__ __forceinline__ bool point_entropy(const double *u, double gam, double &q)
{
    if (!admissible<D>(u, gam)) return false;
    q = pressure<D>(u, gam) * pow(u[0], -gam);
    return true;
}

// (1 + x)^-gamma for |x| <= 1/32 by its binomial series, nested as
// 1 + a_1 x (1 + a_2 x (1 + ... (1 + a_K x))), a_k = (1 - k - gamma) / k: for
// gamma <= 10 the first omitted term is below 2e-18.
__device__ __forceinline__ double binomial_pow(double x, const KxSeries &ser)
{
    double t = 1.0;
#pragma unroll
    for (int k = KX_SERIES_K; k >= 1; --k) t = fma(ser.a[k - 1] * x, t, 1.0);
    return t;
}

// q / rho_ref^-gamma = p (rho / rho_ref)^-gamma of a point state; false when the
// state is not admissible.  The series covers densities within 1/32 of the
// reference (every point of smooth data), pow the rest.
template <int D>
__device__ __forceinline__ bool scaled_entropy(const double *u, double gam, double irho_ref, const KxSeries &ser,
                                               double &q)
{
    if (!admissible<D>(u, gam)) return false;
    const double r = u[0] * irho_ref, x = r - 1.0;
    const double y = fabs(x) <= ser.xmax ? binomial_pow(x, ser) : pow(r, -gam);
    q = pressure<D>(u, gam) * y;
    return true;
}

// Pin every accumulator (empty asm): the FMAs that feed them are complete here.
template <int NP, int NV>
__device__ __forceinline__ void pin_acc(double (&acc)[NP][NV])
{
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if constexpr (NV == 4)
            asm volatile("" : "+v"(acc[p][0]), "+v"(acc[p][1]), "+v"(acc[p][2]), "+v"(acc[p][3]));
        else
            asm volatile("" : "+v"(acc[p][0]), "+v"(acc[p][1]), "+v"(acc[p][2]), "+v"(acc[p][3]), "+v"(acc[p][4]));
    }
}

// The upper-face jumps of every axis (infinity where a state is not admissible)
// in two passes over LDS: the cell's own
// upper-face rows of all axes over S0 (each average read feeds d n_g points),
// then the upper neighbours' lower-face rows over the union of their stencils
// (an average shared by several neighbours' stencils is read once).  Weights:
// [member][axis][point] for the first pass, then the union's layout.
template <int D, int R>
__device__ __forceinline__ void jumps_all_axes(const double (*tile)[KxCfg<D, R>::HN], int lc,
                                               const double *__restrict__ kw, double gam, double irho_ref,
                                               const KxSeries &ser, double (&jump)[D])
{
    using C = KxCfg<D, R>;
    using Un = KxUnion<D, R>;
    constexpr int NV = C::NV, NG = C::NG, N0 = C::N0, NP = D * NG;
    constexpr Un un{};
    double acc[NP][NV], q0[NP];
    bool bad[D];
#pragma unroll
    for (int a = 0; a < D; ++a) bad[a] = false;
    int base = lc;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[p][v] = 0.0;
    // the next member's LDS index depends on the pinned accumulators, so one
    // member's reads are in flight at a time (not all of them hoisted up front)
#pragma unroll
    for (int j = 0; j < N0; ++j) {
        const int o = base + C::st.off[j][0] + C::HX * (C::st.off[j][1] + C::HY * C::st.off[j][2]);
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = tile[v][o];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const double w = kw[j * NP + p];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[p][v] = fma(w, u[v], acc[p][v]);
        }
        pin_acc(acc);
        asm volatile("" : "+v"(base) : "v"(acc[NP - 1][NV - 1]));
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        q0[p] = 0.0;
        bad[p / NG] = bad[p / NG] || !scaled_entropy<D>(acc[p], gam, irho_ref, ser, q0[p]);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[p][v] = 0.0;
    }
    const double *kn = kw + N0 * NP;
#pragma unroll
    for (int m = 0; m < Un::NU; ++m) {
        const int o = base + un.off[m][0] + C::HX * (un.off[m][1] + C::HY * un.off[m][2]);
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = tile[v][o];
        int k = un.woff[m];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (un.j[m][a] < 0) continue;
#pragma unroll
            for (int p = 0; p < NG; ++p) {
                const double w = kn[k + p];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[a * NG + p][v] = fma(w, u[v], acc[a * NG + p][v]);
            }
            k += NG;
        }
        pin_acc(acc);
        asm volatile("" : "+v"(base) : "v"(acc[NP - 1][NV - 1]));
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double jm = 0.0;
#pragma unroll
        for (int p = 0; p < NG; ++p) {
            double q = 0.0;
            bad[a] = bad[a] || !scaled_entropy<D>(acc[a * NG + p], gam, irho_ref, ser, q);
            jm = fmax(jm, fabs(q - q0[a * NG + p]));
        }
        jump[a] = bad[a] ? INFINITY : jm;
    }
}

template <int D, int R>
__global__ __launch_bounds__((KxCfg<D, R>::NT)) void k_kxrcf_jump(const double *__restrict__ U,
                                                                const double *__restrict__ kw,
                                                                double *__restrict__ J, Geom g, KxSeries ser)
{
    using C = KxCfg<D, R>;
    constexpr int NV = C::NV, NG = C::NG, N0 = C::N0, MG = C::MG;
    __shared__ double tile[NV][C::HN];

    const int nbx = (g.n[0] + C::TX - 1) / C::TX, nby = (g.n[1] + C::TY - 1) / C::TY;
    const int nbz = D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1;
    const long nblk = (long)nbx * nby * nbz;
    const long t = xcd_tile(blockIdx.x, nblk);
    if (t >= nblk) return;
    const int bx = (int)(t % nbx), by = (int)((t / nbx) % nby), bz = (int)(t / ((long)nbx * nby));
    const int x0 = bx * C::TX - R, y0 = by * C::TY - R, z0 = D == 3 ? bz * C::TZ - R : 0;

    // one conditional wrap reaches every halo index once each axis holds a tile
    // plus R + 1 cells; smaller grids take the full modulo
    const bool near = g.n[0] >= C::TX + R + 1 && g.n[1] >= C::TY + R + 1 && (D == 2 || g.n[2] >= C::TZ + R + 1);
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
            // non-periodic axes: ghost cells by the boundary conditions (the
            // jumps of boundary faces are redone by k_kxrcf_boundary)
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
    const double gam = g.gamma;
    // the entropies of both sides are formed relative to this cell's average
    // density and scaled back once per cell
    const double rho_ref = tile[0][lc], irho_ref = rcp64(rho_ref);
    const double qscale = rho_ref > 0.0 ? pow(rho_ref, -gam) : 0.0;

    if constexpr (kx_all_axes(D, R)) {
        double jump[D];
        jumps_all_axes<D, R>(tile, lc, kw, gam, irho_ref, ser, jump);
#pragma unroll
        for (int a = 0; a < D; ++a) J[(long)a * g.ncell + cell] = !(rho_ref > 0.0) ? INFINITY : jump[a] * qscale;
        return;
    }
    // 3D order 7 (nine points per face): one axis and one side at a time
#pragma unroll 1
    for (int a = 0; a < D; ++a) {
        const int step = a == 0 ? 1 : (a == 1 ? C::HX : C::HX * C::HY);
        double q0[NG], jmax = 0.0;
        bool bad = false;
        // side 0: this cell, rows of its upper face along a; side 1: the upper
        // neighbour, rows of its lower face (the same physical points)
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const double *wk = kw + (long)(a * 2 + side) * N0 * NG;
            int base = lc + side * step;
            asm volatile("" : "+v"(base));
            double acc[NG][NV];
#pragma unroll
            for (int p = 0; p < NG; ++p)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[p][v] = 0.0;
            // Members in groups of MG, software-pipelined: the LDS reads and the
            // weight loads (scalar) of group k + 1 are issued before the FMAs of
            // group k, and the weights are pinned only after those FMAs, which is
            // where the wave waits for both.  After each group's FMAs the
            // accumulators are pinned too and the LDS index of the reads that
            // follow depends on them (empty asm), so at most two groups' values
            // are live instead of all N0 x NV reads hoisted up front.
            double u[2][MG][NV], wb[2][MG][NG];
            auto load_group = [&](int j0, double (&dst)[MG][NV], double (&w)[MG][NG]) {
#pragma unroll
                for (int m = 0; m < MG; ++m) {
                    const int j = j0 + m < N0 ? j0 + m : N0 - 1;
                    const int o = base + C::st.off[j][0] + C::HX * (C::st.off[j][1] + C::HY * C::st.off[j][2]);
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[m][v] = tile[v][o];
#pragma unroll
                    for (int p = 0; p < NG; ++p) w[m][p] = wk[j * NG + p];
                }
            };
            auto pin_weights = [&](double (&w)[MG][NG]) {
                if constexpr (!C::PIN_W) return;
#pragma unroll
                for (int m = 0; m < MG; ++m)
#pragma unroll
                    for (int p = 0; p < NG; ++p) asm volatile("" : "+s"(w[m][p]));
            };
            // (without room for two groups of weights in scalar registers the
            // weight loads sit right before their FMAs and the wave waits there
            // for everything in flight: the reads are then not issued ahead)
            load_group(0, u[0], wb[0]);
            pin_weights(wb[0]);
#pragma unroll
            for (int j0 = 0; j0 < N0; j0 += MG) {
                const int cur = C::PIN_W ? (j0 / MG) & 1 : 0;
                const bool more = j0 + MG < N0;
                if (C::PIN_W && more) load_group(j0 + MG, u[cur ^ 1], wb[cur ^ 1]);
                if (!C::PIN_W && j0 > 0) load_group(j0, u[0], wb[0]);
#pragma unroll
                for (int m = 0; m < MG; ++m) {
                    if (j0 + m >= N0) break;
#pragma unroll
                    for (int p = 0; p < NG; ++p)
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[p][v] = fma(wb[cur][m][p], u[cur][m][v], acc[p][v]);
                }
#pragma unroll
                for (int p = 0; p < NG; ++p) {
                    if constexpr (NV == 4)
                        asm volatile("" : "+v"(acc[p][0]), "+v"(acc[p][1]), "+v"(acc[p][2]), "+v"(acc[p][3]));
                    else
                        asm volatile("" : "+v"(acc[p][0]), "+v"(acc[p][1]), "+v"(acc[p][2]), "+v"(acc[p][3]),
                                     "+v"(acc[p][4]));
                }
                if (C::PIN_W && more) pin_weights(wb[cur ^ 1]);
                asm volatile("" : "+v"(base) : "v"(acc[NG - 1][NV - 1]));
            }
#pragma unroll
            for (int p = 0; p < NG; ++p) {
                double q = 0.0;
                bad = bad || !scaled_entropy<D>(acc[p], gam, irho_ref, ser, q);
                if (side == 0) q0[p] = q;
                else jmax = fmax(jmax, fabs(q - q0[p]));
            }
        }
        J[(long)a * g.ncell + cell] = bad || !(rho_ref > 0.0) ? INFINITY : jmax * qscale;
    }
}

// Jumps at the faces of non-periodic boundaries, between the cell's unlimited
// state and the outer state the boundary condition gives (section 5.3, step 4):
// upper faces overwrite J, lower faces go to Jlo.  One thread per boundary
// face, the faces of axis A and side SIDE; the stencil is read through the
// ghost fill and the S0 rows of the FP64 tables.
template <int D, int R, int A, int SIDE>
__global__ __launch_bounds__(256) void k_kxrcf_boundary(const double *__restrict__ U, const double *__restrict__ w0,
                                                      double *__restrict__ J, double *__restrict__ Jlo, long plane,
                                                      Geom g)
{
    using S = Stencil<D, R>;
    constexpr S st{};
    constexpr int NV = D + 2, NG = S::NG, N0 = S::N0;
    constexpr int B0 = A == 0 ? 1 : 0, B1 = A == 2 ? 1 : 2;          // the plane's axes, lower first
    const long pi = (long)blockIdx.x * 256 + threadIdx.x;
    const long np = g.ncell / g.n[A];
    if (pi >= np) return;
    int c[3] = {0, 0, 0};
    c[B0] = (int)(pi % g.n[B0]);
    c[B1] = D == 3 ? (int)(pi / g.n[B0]) : 0;
    c[A] = SIDE ? g.n[A] - 1 : 0;
    const long cell = c[0] + (long)g.n[0] * (c[1] + (long)g.n[1] * c[2]);
    double jm = 0.0;
    bool bad = false;
#pragma unroll 1
    for (int p = 0; p < NG; ++p) {
        const double *row = w0 + ((2 * A + SIDE) * NG + p) * N0;
        double in[NV], out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) in[v] = 0.0;
        int cx = c[0];
#pragma unroll
        for (int j = 0; j < N0; ++j) {
            double u[NV];
            ghost_load<D>(U, g, cx + st.off[j][0], c[1] + st.off[j][1], c[2] + st.off[j][2], u);
#pragma unroll
            for (int v = 0; v < NV; ++v) in[v] = fma(row[j], u[v], in[v]);
            // the next member's address depends on this one's sums (empty asm):
            // one member's loads in flight, not all N0 hoisted
            asm volatile("" : "+v"(cx) : "v"(in[NV - 1]));
        }
        boundary_state<D>(g, A, SIDE, in, out);
        double qi = 0.0, qo = 0.0;
        bad = bad || !point_entropy<D>(in, g.gamma, qi) || !point_entropy<D>(out, g.gamma, qo);
        jm = fmax(jm, fabs(qo - qi));
    }
    const double j = bad ? INFINITY : jm;
    if (SIDE) J[(long)A * g.ncell + cell] = j;
    else Jlo[(long)A * plane + pi] = j;
}

template <int D, int R, int A>
void launch_boundary_axis(const Geom &g, const double *U, const double *w0, double *J, double *Jlo, long plane,
                          hipStream_t s)
{
    if (A >= D || g.bc[A][0] == BC_PERIODIC) return;
    const unsigned nb = (unsigned)((g.ncell / g.n[A] + 255) / 256);
    hipLaunchKernelGGL((k_kxrcf_boundary<D, R, A, 0>), dim3(nb), dim3(256), 0, s, U, w0, J, Jlo, plane, g);
    hipLaunchKernelGGL((k_kxrcf_boundary<D, R, A, 1>), dim3(nb), dim3(256), 0, s, U, w0, J, Jlo, plane, g);
}

template <int D>
__global__ __launch_bounds__(256) void k_kxrcf_flags(const double *__restrict__ U, const double *__restrict__ J,
                                                   const double *__restrict__ Jlo, long plane,
                                                   uint8_t *__restrict__ flags, Geom g, double thr)
{
    constexpr int NV = D + 2;
    const long cell = (long)blockIdx.x * 256 + threadIdx.x;
    if (cell >= g.ncell) return;
    const int c[3] = {(int)(cell % g.n[0]), (int)((cell / g.n[0]) % g.n[1]), (int)(cell / ((long)g.n[0] * g.n[1]))};
    const long stride[3] = {1, g.n[0], (long)g.n[0] * g.n[1]};
    double jm = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const long lower = cell + (c[a] == 0 ? (long)(g.n[a] - 1) * stride[a] : -stride[a]);
        const double jl = c[a] == 0 && g.bc[a][0] != BC_PERIODIC
                              ? Jlo[(long)a * plane + plane_index(a, c[0], c[1], c[2], g.n)]
                              : J[(long)a * g.ncell + lower];
        jm = fmax(jm, fmax(J[(long)a * g.ncell + cell], jl));
    }
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + cell];
    double Q = 0.0;
    const bool ok = point_entropy<D>(u, g.gamma, Q);
    // smooth (linear S0 value) only when eq. kxrcf holds: jump / <Q> < Delta^m
    const uint8_t f = (ok && jm < thr * Q) ? 0 : 1;
#pragma unroll
    for (int v = 0; v < NV; ++v) flags[(long)v * g.ncell + cell] = f;
}

template <int D, int R>
hipError_t kxrcf_impl(const Geom &g, const double *kw, const double *w0, const double *U, double *J, double *Jlo,
                      long plane, uint8_t *flags, double thr, hipStream_t s)
{
    using C = KxCfg<D, R>;
    KxSeries ser;
    for (int k = 1; k <= KX_SERIES_K; ++k) ser.a[k - 1] = (1.0 - k - g.gamma) / k;
    ser.xmax = g.gamma <= 10.0 ? 1.0 / 32 : -1.0;
    const long nblk = (long)((g.n[0] + C::TX - 1) / C::TX) * ((g.n[1] + C::TY - 1) / C::TY) *
                      (D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1);
    hipLaunchKernelGGL((k_kxrcf_jump<D, R>), dim3((unsigned)(((nblk + 7) / 8) * 8)), dim3(C::NT), 0, s, U, kw, J, g,
                       ser);
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (!g.periodic) {
        launch_boundary_axis<D, R, 0>(g, U, w0, J, Jlo, plane, s);
        launch_boundary_axis<D, R, 1>(g, U, w0, J, Jlo, plane, s);
        launch_boundary_axis<D, R, 2>(g, U, w0, J, Jlo, plane, s);
    }
    if (flags)
        hipLaunchKernelGGL((k_kxrcf_flags<D>), dim3(nb), dim3(256), 0, s, U, J, Jlo, plane, flags, g, thr);
    return hipGetLastError();
}

}  // namespace

int kxrcf_table_size(int dim, int R)
{
    if (dim == 2 && R == 2) return 2 * 2 * Stencil<2, 2>::N0 * Stencil<2, 2>::NG;
    if (dim == 2 && R == 3) return 2 * 2 * Stencil<2, 3>::N0 * Stencil<2, 3>::NG;
    if (dim == 3 && R == 2) return 3 * 2 * Stencil<3, 2>::N0 * Stencil<3, 2>::NG;
    if (dim == 3 && R == 3) return 3 * 2 * Stencil<3, 3>::N0 * Stencil<3, 3>::NG;
    return -1;
}

hipError_t launch_kxrcf(int dim, int R, const Geom &g, const double *kw, const double *w0, const double *U, double *J,
                        double *Jlo, long plane, uint8_t *flags, double thr, hipStream_t s)
{
    if (dim == 2 && R == 2) return kxrcf_impl<2, 2>(g, kw, w0, U, J, Jlo, plane, flags, thr, s);
    if (dim == 2 && R == 3) return kxrcf_impl<2, 3>(g, kw, w0, U, J, Jlo, plane, flags, thr, s);
    if (dim == 3 && R == 2) return kxrcf_impl<3, 2>(g, kw, w0, U, J, Jlo, plane, flags, thr, s);
    if (dim == 3 && R == 3) return kxrcf_impl<3, 3>(g, kw, w0, U, J, Jlo, plane, flags, thr, s);
    return hipErrorInvalidValue;
}

}  // namespace kfvm
