// Compile-time description of the KFVM-WENO stencils (paper section 3.1) and
// of the per-cell reconstruction targets (section 5.1), for radius R in d
// dimensions.  Used by the host weight builder and by the HIP kernels, which
// unroll every loop over these tables so that offsets and member indices
// become immediate operands.
//
//  * S0 = { i in Z^d : |i|^2 <= R^2 }, cells in lexicographic order of the
//    offset tuple (x, y[, z]) with x slowest;
//  * stencil 0 is S0, stencil 1 the ball of radius R-1, stencils 2.. the
//    biased cones along +x, -x, +y, -y, +z, -z: the cells of S0 whose other
//    coordinates are bounded in magnitude by the signed leading coordinate;
//  * each stencil's table has n_pts face-point rows then n_der derivative
//    rows, N_q columns in the stencil's member order;
//  * face point s = (2 a + side) * R^(d-1) + g (normal axis a, side 0 = lower
//    face, g the Gauss index over the transverse axes, first one slowest);
//  * derivative multi-indices 0 < |alpha| <= R (section 3.3), by degree, then
//    lexicographically descending.
#pragma once

namespace kfvm {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

constexpr int count_ball(int d, int r2, int R)
{
    int c = 0;
    for (int i = -R; i <= R; ++i)
        for (int j = -R; j <= R; ++j)
            for (int k = (d == 3 ? -R : 0); k <= (d == 3 ? R : 0); ++k)
                if (i * i + j * j + k * k <= r2) ++c;
    return c;
}

constexpr int count_derivs(int d, int R)
{
    int c = 0;
    for (int i = 0; i <= R; ++i)
        for (int j = 0; j <= R; ++j)
            for (int k = 0; k <= (d == 3 ? R : 0); ++k) {
                int s = i + j + k;
                if (s > 0 && s <= R) ++c;
            }
    return c;
}

template <int D, int R>
struct Stencil {
    static constexpr int N0 = count_ball(D, R * R, R);
    static constexpr int NST = 2 + 2 * D;
    static constexpr int NG = ipow(R, D - 1);        // Gauss points per face
    static constexpr int NPTS = 2 * D * NG;          // face points per cell
    static constexpr int NDER = count_derivs(D, R);  // derivative rows
    static constexpr int NROWS = NPTS + NDER;
    static constexpr int NV = D + 2;                 // conserved variables

    int off[N0][3];          // unit-cell offsets (z = 0 in 2D)
    int nmem[NST];           // cells per stencil
    int mem[NST][N0];        // member indices into S0
    int tab[NST];            // start of each stencil's table in the packed array
    int tab_total;           // doubles in the packed array
    int der[NDER][3];        // derivative multi-indices
    int degree[NST];         // polynomial degree of the augmentation

    constexpr Stencil() : off{}, nmem{}, mem{}, tab{}, tab_total(0), der{}, degree{}
    {
        int c = 0;
        for (int i = -R; i <= R; ++i)
            for (int j = -R; j <= R; ++j)
                for (int k = (D == 3 ? -R : 0); k <= (D == 3 ? R : 0); ++k)
                    if (i * i + j * j + k * k <= R * R) {
                        off[c][0] = i; off[c][1] = j; off[c][2] = k;
                        ++c;
                    }
        for (int q = 0; q < NST; ++q) {
            int m = 0;
            for (int h = 0; h < N0; ++h) {
                int o[3] = {off[h][0], off[h][1], off[h][2]};
                bool in = false;
                if (q == 0) {
                    in = true;
                } else if (q == 1) {
                    in = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] <= (R - 1) * (R - 1);
                } else {
                    int a = (q - 2) / 2, sg = ((q - 2) % 2 == 0) ? 1 : -1;
                    int lead = sg * o[a];
                    in = true;
                    for (int b = 0; b < D; ++b)
                        if (b != a && (o[b] < 0 ? -o[b] : o[b]) > lead) in = false;
                    if (lead < 0) in = false;
                }
                if (in) mem[q][m++] = h;
            }
            nmem[q] = m;
        }
        int t = 0;
        for (int q = 0; q < NST; ++q) {
            tab[q] = t;
            t += NROWS * nmem[q];
        }
        tab_total = t;
        int n = 0;
        for (int deg = 1; deg <= R; ++deg)
            for (int i = deg; i >= 0; --i)
                for (int j = deg - i; j >= 0; --j) {
                    int k = deg - i - j;
                    if (D == 2 && k != 0) continue;
                    der[n][0] = i; der[n][1] = j; der[n][2] = k;
                    ++n;
                }
        // largest unisolvent degree: 2R-1 on S0, 2R-3 on the inner ball and
        // R-1 on the cones (exact-rank result for R = 2, 3 in 2D and 3D)
        degree[0] = 2 * R - 1;
        degree[1] = 2 * R - 3;
        for (int q = 2; q < NST; ++q) degree[q] = R - 1;
    }
};

// Contraction slot k of the split-precision path -> S0 index.  The centre is
// the middle of the lexicographic order of S0 and, its increment W_c - W_c
// being zero, takes no slot: slots 0 .. N0 - 2.
template <int D, int R>
constexpr int slot_point(int k)
{
    return k < Stencil<D, R>::N0 / 2 ? k : k + 1;
}

template <int D, int R>
constexpr bool centre_is_middle()
{
    constexpr Stencil<D, R> s{};
    constexpr int c = Stencil<D, R>::N0 / 2;
    return s.off[c][0] == 0 && s.off[c][1] == 0 && s.off[c][2] == 0;
}
static_assert(centre_is_middle<2, 2>() && centre_is_middle<2, 3>() && centre_is_middle<3, 2>() &&
                  centre_is_middle<3, 3>(),
              "S0 centre must sit in the middle of the lexicographic order");

// Members of every stencil in chunks of CH (the FP64 reconstruction of large
// stencils walks them chunk by chunk): stencil q's members padded with -1 to a
// multiple of CH; chunk k covers member slots [CH k, CH k + CH) and belongs to
// stencil q for cb[q] <= k < cb[q + 1].  The padded weights are laid out per
// chunk as [row][CH] (rows: face points, then derivatives), zeros in padding.
template <int D, int R, int CH_>
struct ChunkLayout {
    using S = Stencil<D, R>;
    static constexpr int CH = CH_;
    static constexpr int total_chunks()
    {
        constexpr S st{};
        int n = 0;
        for (int q = 0; q < S::NST; ++q) n += (st.nmem[q] + CH - 1) / CH;
        return n;
    }
    static constexpr int NCH = total_chunks();
    int cb[S::NST + 1];       // first chunk of each stencil
    int member[NCH * CH];     // S0 index of each padded member slot, -1 for padding
    constexpr ChunkLayout() : cb{}, member{}
    {
        constexpr S st{};
        int k = 0;
        for (int q = 0; q < S::NST; ++q) {
            cb[q] = k;
            const int nc = (st.nmem[q] + CH - 1) / CH;
            for (int m = 0; m < nc * CH; ++m) member[k * CH + m] = m < st.nmem[q] ? st.mem[q][m] : -1;
            k += nc;
        }
        cb[S::NST] = k;
    }
};

// Members of the KXRCF indicator's neighbour pass: the union over the axes a of
// S0 + e_a (the stencils of the upper neighbours), in lexicographic order of the
// offset with x slowest; per member the S0 index of (offset - e_a) for each axis
// (-1 outside S0) and where its weights start in the pass's table, which holds
// for each member, for each axis it belongs to, the n_g lower-face rows.
template <int D, int R>
struct KxUnion {
    using S = Stencil<D, R>;
    static constexpr int count()
    {
        constexpr S st{};
        int c = 0;
        for (int i = -R; i <= R + 1; ++i)
            for (int j = -R; j <= R + 1; ++j)
                for (int k = (D == 3 ? -R : 0); k <= (D == 3 ? R + 1 : 0); ++k) {
                    bool in = false;
                    for (int a = 0; a < D; ++a) {
                        const int o[3] = {i - (a == 0), j - (a == 1), k - (a == 2)};
                        for (int h = 0; h < S::N0; ++h)
                            if (st.off[h][0] == o[0] && st.off[h][1] == o[1] && st.off[h][2] == o[2]) in = true;
                    }
                    if (in) ++c;
                }
        return c;
    }
    static constexpr int NU = count();
    int off[NU][3];
    int j[NU][3];
    int woff[NU + 1];
    constexpr KxUnion() : off{}, j{}, woff{}
    {
        constexpr S st{};
        int c = 0, w = 0;
        for (int i = -R; i <= R + 1; ++i)
            for (int jj = -R; jj <= R + 1; ++jj)
                for (int k = (D == 3 ? -R : 0); k <= (D == 3 ? R + 1 : 0); ++k) {
                    int idx[3] = {-1, -1, -1};
                    bool in = false;
                    for (int a = 0; a < D; ++a) {
                        const int o[3] = {i - (a == 0), jj - (a == 1), k - (a == 2)};
                        for (int h = 0; h < S::N0; ++h)
                            if (st.off[h][0] == o[0] && st.off[h][1] == o[1] && st.off[h][2] == o[2]) idx[a] = h;
                        in = in || idx[a] >= 0;
                    }
                    if (!in) continue;
                    off[c][0] = i; off[c][1] = jj; off[c][2] = k;
                    woff[c] = w;
                    for (int a = 0; a < 3; ++a) {
                        j[c][a] = idx[a];
                        if (idx[a] >= 0) w += S::NG;
                    }
                    ++c;
                }
        woff[c] = w;
    }
};

// The KXRCF first pass takes every axis at once where the accumulators of all
// upper-face points fit (d n_g <= 12); 3D order 7 takes one axis and side at a time.
constexpr bool kx_all_axes(int D, int R) { return D * ipow(R, D - 1) <= 12; }

// linear weights of section 3.2 (gamma_hi = gamma_lo = 0.8)
template <int D>
constexpr double linear_weight(int q)
{
    return q == 0 ? 0.8 : (q == 1 ? 0.2 * 0.8 : 0.2 * 0.2 / (2 * D));
}

}  // namespace kfvm
