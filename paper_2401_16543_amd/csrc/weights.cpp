// Host-side builder of the KFVM-WENO reconstruction vectors (paper section 2.1,
// eq. recVec1; section 3.3 for the derivative rows; section 5.1 for the face
// Gauss points and l = 5 Delta), in IEEE binary128 arithmetic (libquadmath).
//
// For every (sub)stencil the (N + D) x (N + D) saddle matrix
//     M = [ Q  P ; P^T 0 ],   Q_hl = cell average over cell h of K(x, x_l),
//                              P_hv = cell average over cell h of x^alpha_v,
// is assembled in unit-cell coordinates with the squared-exponential kernel
// K(x, y) = exp(-|x - y|^2 / (2 l^2)), l = ell_hat (section 3.1: the unit-cell
// rescaling replaces l by l / Delta).  One LU factorisation of M^T with partial
// pivoting then serves every target: face points (T_l = K(x*, x_l),
// S_v = x*^alpha_v) and derivatives at the cell centre (D_l = d^alpha K(x, x_l)
// at 0, S_v = alpha! delta).  The first N entries of each solution are the
// reconstruction vector, rounded once to binary64.
//
// Binary128 keeps about 34 significant digits; the worst S0 system (3D, R = 3)
// has a condition number near 3e17, which leaves the rounded result within an
// ulp or so of the exact one.  Binary64 elimination would lose it entirely.
#include <quadmath.h>

#include <cstring>
#include <vector>

#include "stencil.hpp"

namespace {

typedef __float128 q128;

// integral over [t - 1/2, t + 1/2] of exp(-x^2 / (2 l^2)) dx
q128 kernel_avg_1d(q128 t, q128 ell)
{
    q128 s = sqrtq((q128)2) * ell;
    return ell * sqrtq(M_PIq / 2) * (erfq((t + 0.5Q) / s) - erfq((t - 0.5Q) / s));
}

// n-th derivative of exp(-(x - c)^2 / (2 l^2)) at x = 0 through the Hermite
// recurrence H_{k+1}(z) = 2 z H_k(z) - 2 k H_{k-1}(z):
//     d^n/dx^n e^{-z^2} = (-1)^n H_n(z) e^{-z^2} / s^n,  z = (x - c) / s,  s = sqrt(2) l
q128 kernel_deriv_1d(int n, q128 c, q128 ell)
{
    q128 s = sqrtq((q128)2) * ell, z = -c / s;
    q128 h0 = 1, h1 = 2 * z, hn = (n == 0) ? h0 : h1;
    for (int k = 1; k < n; ++k) {
        hn = 2 * z * h1 - 2 * k * h0;
        h0 = h1;
        h1 = hn;
    }
    q128 sign = (n % 2) ? -1 : 1;
    return sign * hn * expq(-z * z) / powq(s, n);
}

q128 avg_monomial_1d(int c, int a)
{
    q128 hi = c + 0.5Q, lo = c - 0.5Q;
    return (powq(hi, a + 1) - powq(lo, a + 1)) / (a + 1);
}

// Gauss-Legendre nodes on [-1/2, 1/2], ascending (R = 2 or 3)
void gauss_nodes(int R, q128 *x)
{
    if (R == 2) {
        x[0] = -0.5Q / sqrtq((q128)3);
        x[1] = -x[0];
    } else {
        x[0] = -0.5Q * sqrtq((q128)3 / 5);
        x[1] = 0;
        x[2] = -x[0];
    }
}

struct Mono {
    int e[3];
};

std::vector<Mono> monomials(int d, int p)
{
    std::vector<Mono> m;
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j)
            for (int k = 0; k <= (d == 3 ? p : 0); ++k)
                if (i + j + k <= p) m.push_back(Mono{{i, j, k}});
    return m;
}

// LU with partial pivoting, in place, row-major n x n.  Returns false if singular.
bool lu_factor(std::vector<q128> &A, std::vector<int> &piv, int n)
{
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        q128 best = fabsq(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabsq(A[i * n + k]) > best) { best = fabsq(A[i * n + k]); p = i; }
        if (best == 0) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) { q128 t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            q128 f = A[i * n + k] / A[k * n + k];
            A[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
        }
    }
    return true;
}

void lu_solve(const std::vector<q128> &A, const std::vector<int> &piv, int n, std::vector<q128> &b)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { q128 t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 1; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= A[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= A[i * n + j] * b[j];
        b[i] /= A[i * n + i];
    }
}

q128 factorial(int n) { q128 f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

template <int D, int R>
int build(double ell_hat, double *out, int capacity)
{
    constexpr kfvm::Stencil<D, R> st{};
    using S = kfvm::Stencil<D, R>;
    if (capacity < st.tab_total) return -1;
    const q128 ell = ell_hat;
    q128 gx[3];
    gauss_nodes(R, gx);
    // face points (section 5.1)
    q128 pts[S::NPTS][3];
    for (int a = 0; a < D; ++a)
        for (int side = 0; side < 2; ++side)
            for (int g = 0; g < S::NG; ++g) {
                q128 *x = pts[(2 * a + side) * S::NG + g];
                x[0] = x[1] = x[2] = 0;
                x[a] = side ? 0.5Q : -0.5Q;
                int gi = g, t = 0;
                int trans[2] = {0, 0};
                for (int b = 0; b < D; ++b)
                    if (b != a) trans[t++] = b;
                // first transverse axis slowest
                for (int tt = D - 2; tt >= 0; --tt) {
                    x[trans[tt]] = gx[gi % R];
                    gi /= R;
                }
            }
    for (int q = 0; q < S::NST; ++q) {
        const int N = st.nmem[q];
        std::vector<Mono> mons = monomials(D, st.degree[q]);
        const int Dm = (int)mons.size(), n = N + Dm;
        std::vector<q128> MT((size_t)n * n, 0);   // M^T, row-major
        for (int h = 0; h < N; ++h) {
            const int *ch = st.off[st.mem[q][h]];
            for (int l = 0; l < N; ++l) {
                const int *cl = st.off[st.mem[q][l]];
                q128 v = 1;
                for (int k = 0; k < D; ++k) v *= kernel_avg_1d((q128)(ch[k] - cl[k]), ell);
                MT[l * n + h] = v;                 // M[h][l]
            }
            for (int v = 0; v < Dm; ++v) {
                q128 pv = 1;
                for (int k = 0; k < D; ++k) pv *= avg_monomial_1d(ch[k], mons[v].e[k]);
                MT[(N + v) * n + h] = pv;          // M[h][N + v]
                MT[h * n + N + v] = pv;            // M[N + v][h]
            }
        }
        std::vector<int> piv;
        if (!lu_factor(MT, piv, n)) return -2;
        std::vector<q128> b(n);
        double *tab = out + st.tab[q];
        for (int row = 0; row < S::NROWS; ++row) {
            if (row < S::NPTS) {
                const q128 *x = pts[row];
                for (int l = 0; l < N; ++l) {
                    const int *cl = st.off[st.mem[q][l]];
                    q128 r2 = 0;
                    for (int k = 0; k < D; ++k) r2 += (x[k] - cl[k]) * (x[k] - cl[k]);
                    b[l] = expq(-r2 / (2 * ell * ell));
                }
                for (int v = 0; v < Dm; ++v) {
                    q128 m = 1;
                    for (int k = 0; k < D; ++k) m *= powq(x[k], mons[v].e[k]);
                    b[N + v] = m;
                }
            } else {
                const int *al = st.der[row - S::NPTS];
                for (int l = 0; l < N; ++l) {
                    const int *cl = st.off[st.mem[q][l]];
                    q128 m = 1;
                    for (int k = 0; k < D; ++k) m *= kernel_deriv_1d(al[k], (q128)cl[k], ell);
                    b[l] = m;
                }
                for (int v = 0; v < Dm; ++v) {
                    bool same = true;
                    for (int k = 0; k < D; ++k) same = same && mons[v].e[k] == al[k];
                    q128 f = 1;
                    for (int k = 0; k < D; ++k) f *= factorial(al[k]);
                    b[N + v] = same ? f : 0;
                }
            }
            lu_solve(MT, piv, n, b);
            for (int j = 0; j < N; ++j) tab[row * N + j] = (double)b[j];
        }
    }
    return st.tab_total;
}

}  // namespace

// Exported through the C-ABI (declared in include/kfvm.h).
extern "C" int kfvm_weights_build(int dim, int R, double ell_hat, double *tables, int capacity)
{
    if (!tables || ell_hat <= 0) return -1;
    if (dim == 2 && R == 2) return build<2, 2>(ell_hat, tables, capacity);
    if (dim == 2 && R == 3) return build<2, 3>(ell_hat, tables, capacity);
    if (dim == 3 && R == 2) return build<3, 2>(ell_hat, tables, capacity);
    if (dim == 3 && R == 3) return build<3, 3>(ell_hat, tables, capacity);
    return -1;
}

extern "C" int kfvm_weights_size(int dim, int R)
{
    if (dim == 2 && R == 2) return kfvm::Stencil<2, 2>{}.tab_total;
    if (dim == 2 && R == 3) return kfvm::Stencil<2, 3>{}.tab_total;
    if (dim == 3 && R == 2) return kfvm::Stencil<3, 2>{}.tab_total;
    if (dim == 3 && R == 3) return kfvm::Stencil<3, 3>{}.tab_total;
    return -1;
}
