"""Oracle: stencils and kernel reconstruction vectors for KFVM-WENO, in 50-digit arithmetic.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this module;
only tests/, the smoke check and the CPU-baseline leg of the benchmark do.

What it computes (paper, section 2.1 "Asymmetric reconstruction", section 3.1
"Stencils and substencils", section 3.3 "Smoothness indicators and weights",
section 5.1 "Stencils and weight vectors"):

* the full spherical stencil S0 = {|i|^2 <= R^2} and its substencils
  S1 = {|i|^2 <= (R-1)^2} and the 2d axis-biased cones (section 3.1);
* for each (sub)stencil the largest polynomial degree p_q for which the cell
  averages of the monomials of total degree <= p_q are linearly independent over
  the stencil (unisolvence, section 2.1), found by exact rational rank;
* the saddle-point matrix [[Q, P], [P^T, 0]] with Q_hl the cell average over
  cell h of the squared-exponential kernel centred on cell l (eq. kernelMat) and
  P_hv the cell average of monomial v (the P matrix of section 2.1), in unit-cell
  coordinates with length scale l/Delta = 5 (sections 3.1 and 5.1);
* reconstruction vectors r solving [[Q^T, P], [P^T, 0]] (r, w) = (T, S)
  (eq. recVec1) for every face Gauss-Legendre point (section 5.1, R points per
  transverse dimension) and, with the differential sample vector D and the
  derivatives of the monomials in place of T and S (section 3.3), for every
  derivative multi-index 0 < |alpha| <= R (section 3.3: p = R);
* the linear weights gamma_q (section 3.2).

The solve runs in mpmath at 50 significant digits and each r is rounded once to
binary64.  Float64 Gaussian elimination is not accurate enough at l/Delta = 5
(the S0 Gram systems have condition numbers up to ~1e17 in 3D, R = 3).

Conventions shared with the C-ABI (data layout, not code):
* S0 cells are ordered lexicographically by their offset tuple (x, y[, z]),
  x slowest; a substencil lists its cells in that same order.
* stencil q = 0 is S0, q = 1 the central S1, q = 2.. the biased cones in the
  order +x, -x, +y, -y, +z, -z (section 3.1).
* rows of a stencil's table: first the face points, then the derivatives.
  Face point index s = (2*a + side) * R^(d-1) + g, with a the face normal axis,
  side 0 for the lower face (x_a = -1/2) and 1 for the upper face (+1/2), and g
  the Gauss-Legendre index over the transverse axes in ascending axis order,
  first transverse axis slowest, nodes ascending on [-1/2, 1/2].
* derivative multi-indices ordered by total degree, then lexicographically
  descending in (alpha_x, alpha_y, alpha_z).
"""
from __future__ import annotations

import functools
import itertools
import math
import os
from fractions import Fraction

import mpmath
import numpy as np

DPS = 50          # working precision of every solve, in decimal digits
ELL_HAT = 5       # l / Delta: the kernel length scale in unit-cell coordinates (section 5.1)
GAMMA_HI = 0.8    # linear-weight constants of section 3.2
GAMMA_LO = 0.8


# ---------------------------------------------------------------------------
# Stencils (section 3.1)
# ---------------------------------------------------------------------------
def full_stencil(d: int, R: int) -> list[tuple[int, ...]]:
    """S0 = {i in Z^d : |i|^2 <= R^2}, lexicographic order, x slowest."""
    rng = range(-R, R + 1)
    return [o for o in itertools.product(rng, repeat=d) if sum(c * c for c in o) <= R * R]


def substencils(d: int, R: int) -> list[list[int]]:
    """Member lists (indices into S0) of S0, S1 and the 2d biased cones.

    S1 is the ball of radius R-1.  The biased cone along +axis a keeps the cells
    of S0 whose every other coordinate is bounded in magnitude by the a-th
    coordinate; the -axis cone by minus the a-th coordinate (section 3.1).
    """
    s0 = full_stencil(d, R)
    out = [list(range(len(s0)))]
    out.append([h for h, o in enumerate(s0) if sum(c * c for c in o) <= (R - 1) ** 2])
    for a in range(d):
        for sgn in (1, -1):
            mem = []
            for h, o in enumerate(s0):
                lead = sgn * o[a]
                if all(abs(o[b]) <= lead for b in range(d) if b != a):
                    mem.append(h)
            out.append(mem)
    return out


def monomials(d: int, p: int) -> list[tuple[int, ...]]:
    """Exponent tuples of all monomials of total degree <= p."""
    return [a for a in itertools.product(range(p + 1), repeat=d) if sum(a) <= p]


def derivative_indices(d: int, R: int) -> list[tuple[int, ...]]:
    """Multi-indices 0 < |alpha| <= R (section 3.3), by degree then descending."""
    out = []
    for k in range(1, R + 1):
        out += sorted([a for a in itertools.product(range(k + 1), repeat=d) if sum(a) == k],
                      reverse=True)
    return out


# ---------------------------------------------------------------------------
# Unisolvence: exact rank of the cell-averaged monomial matrix (section 2.1)
# ---------------------------------------------------------------------------
def _avg_monomial_1d_exact(c: int, a: int) -> Fraction:
    # average of x^a over the unit cell [c - 1/2, c + 1/2]
    hi, lo = Fraction(2 * c + 1, 2), Fraction(2 * c - 1, 2)
    return (hi ** (a + 1) - lo ** (a + 1)) / (a + 1)


def _rank_exact(rows: list[list[Fraction]]) -> int:
    m = [r[:] for r in rows]
    rank, ncol = 0, len(m[0]) if m else 0
    for col in range(ncol):
        piv = next((i for i in range(rank, len(m)) if m[i][col] != 0), None)
        if piv is None:
            continue
        m[rank], m[piv] = m[piv], m[rank]
        for i in range(len(m)):
            if i != rank and m[i][col] != 0:
                f = m[i][col] / m[rank][col]
                m[i] = [x - f * y for x, y in zip(m[i], m[rank])]
        rank += 1
    return rank


def max_unisolvent_degree(cells: list[tuple[int, ...]]) -> int:
    """Largest p such that the averaged monomials of degree <= p are independent."""
    d = len(cells[0])
    p = 0
    while True:
        mons = monomials(d, p + 1)
        if len(mons) > len(cells):
            return p
        rows = [[math.prod(_avg_monomial_1d_exact(c[k], a[k]) for k in range(d)) for a in mons]
                for c in cells]
        if _rank_exact(rows) < len(mons):
            return p
        p += 1


# ---------------------------------------------------------------------------
# Gauss-Legendre points on [-1/2, 1/2]
# ---------------------------------------------------------------------------
def gauss_legendre_unit(n: int) -> tuple[list, list]:
    """n-point Gauss-Legendre nodes (ascending) and weights (summing to 1) on [-1/2, 1/2]."""
    with mpmath.workdps(DPS):
        nodes, weights = [], []
        # roots of P_n by Newton from the Chebyshev guesses, in DPS digits
        for i in range(n):
            x = mpmath.cos(mpmath.pi * (i + mpmath.mpf(3) / 4) / (n + mpmath.mpf(1) / 2))
            for _ in range(200):
                p = mpmath.legendre(n, x)
                dp = n * (x * p - mpmath.legendre(n - 1, x)) / (x * x - 1)
                dx = p / dp
                x -= dx
                if abs(dx) < mpmath.mpf(10) ** (-DPS + 3):
                    break
            p = mpmath.legendre(n, x)
            dp = n * (x * p - mpmath.legendre(n - 1, x)) / (x * x - 1)
            w = 2 / ((1 - x * x) * dp * dp)
            if abs(x) < mpmath.mpf(10) ** (-DPS + 3):
                x = mpmath.mpf(0)     # the odd-n middle root is exactly zero
            nodes.append(x / 2)
            weights.append(w / 2)
        order = sorted(range(n), key=lambda i: nodes[i])
        return [nodes[i] for i in order], [weights[i] for i in order]


def face_points(d: int, R: int) -> list[tuple]:
    """Face Gauss points x* in unit-cell coordinates (mpf), in face-point index order."""
    nodes, _ = gauss_legendre_unit(R)
    half = mpmath.mpf(1) / 2
    pts = []
    for a in range(d):
        trans = [b for b in range(d) if b != a]
        for side in (0, 1):
            for g in itertools.product(range(R), repeat=d - 1):
                x = [None] * d
                x[a] = -half if side == 0 else half
                for b, gi in zip(trans, g):
                    x[b] = nodes[gi]
                pts.append(tuple(x))
    return pts


# ---------------------------------------------------------------------------
# Kernel, its cell averages and derivatives (eq. kernSE, eq. kernelMat)
# ---------------------------------------------------------------------------
def _kernel_avg_1d(t, ell):
    # integral over [t - 1/2, t + 1/2] of exp(-x^2 / (2 ell^2)) dx (unit cell: average = integral)
    s = mpmath.sqrt(2) * ell
    return ell * mpmath.sqrt(mpmath.pi / 2) * (mpmath.erf((t + mpmath.mpf(1) / 2) / s)
                                               - mpmath.erf((t - mpmath.mpf(1) / 2) / s))


def _kernel_deriv_1d(n: int, c, ell):
    # n-th derivative in x of exp(-(x - c)^2 / (2 ell^2)), evaluated at x = 0,
    # via the physicists' Hermite polynomials: d^n/dx^n e^{-z^2} = (-1)^n H_n(z) e^{-z^2}
    s = mpmath.sqrt(2) * ell
    z = (0 - c) / s
    return (-1) ** n * mpmath.hermite(n, z) * mpmath.exp(-z * z) / s ** n


def _avg_monomial_1d(c, a):
    half = mpmath.mpf(1) / 2
    return ((c + half) ** (a + 1) - (c - half) ** (a + 1)) / (a + 1)


def reconstruction_vectors(cells, p, points, derivs, ell_hat=ELL_HAT, dps=DPS) -> list:
    """Reconstruction vectors on an arbitrary stencil of unit cells (section 2.1).

    cells: cell-centre offsets; p: polynomial degree of the augmentation;
    points: evaluation points x* (eq. sampleVec); derivs: multi-indices alpha for
    the differential sample vectors (section 3.3).  Returns mpf rows, one per
    point then one per derivative, each of length len(cells).
    """
    d = len(cells[0])
    mons = monomials(d, p)
    N, D = len(cells), len(mons)
    with mpmath.workdps(dps):
        ell = mpmath.mpf(ell_hat)
        M = mpmath.zeros(N + D, N + D)
        for h, ch in enumerate(cells):
            for l, cl in enumerate(cells):
                M[h, l] = mpmath.fprod(_kernel_avg_1d(mpmath.mpf(ch[k] - cl[k]), ell)
                                       for k in range(d))
            for v, a in enumerate(mons):
                pv = mpmath.fprod(_avg_monomial_1d(mpmath.mpf(ch[k]), a[k]) for k in range(d))
                M[h, N + v] = pv
                M[N + v, h] = pv
        # reconstruction vectors solve the transposed system (eq. recVec1);
        # one LU factorisation (partial pivoting, 10 guard digits) serves every target
        rows = []
        with mpmath.extradps(10):
            LU, perm = mpmath.mp.LU_decomp(M.T)

        def solve(rhs):
            with mpmath.extradps(10):
                sol = mpmath.mp.U_solve(LU, mpmath.mp.L_solve(LU, rhs, perm))
            return [sol[h] for h in range(N)]

        for x in points:
            rhs = mpmath.zeros(N + D, 1)
            for l, cl in enumerate(cells):
                rhs[l] = mpmath.exp(-mpmath.fsum((mpmath.mpf(x[k]) - cl[k]) ** 2 for k in range(d))
                                    / (2 * ell ** 2))
            for v, a in enumerate(mons):
                rhs[N + v] = mpmath.fprod(mpmath.mpf(x[k]) ** a[k] for k in range(d))
            rows.append(solve(rhs))
        for al in derivs:
            rhs = mpmath.zeros(N + D, 1)
            for l, cl in enumerate(cells):
                rhs[l] = mpmath.fprod(_kernel_deriv_1d(al[k], mpmath.mpf(cl[k]), ell) for k in range(d))
            for v, a in enumerate(mons):
                # d^alpha x^a at 0 is alpha! when a == alpha, else 0
                rhs[N + v] = (mpmath.mpf(math.prod(math.factorial(t) for t in al))
                              if tuple(a) == tuple(al) else 0)
            rows.append(solve(rhs))
    return rows


@functools.lru_cache(maxsize=None)
def stencil_weights(d: int, R: int, q: int, ell_hat=ELL_HAT, dps=DPS) -> np.ndarray:
    """Reconstruction vectors of (sub)stencil q: float64 array [n_pts + n_der, N_q]."""
    s0 = full_stencil(d, R)
    cells = [s0[h] for h in substencils(d, R)[q]]
    p = max_unisolvent_degree(cells)
    rows = reconstruction_vectors(cells, p, face_points(d, R), derivative_indices(d, R), ell_hat, dps)
    with mpmath.workdps(dps):
        return np.array([[float(x) for x in r] for r in rows], dtype=np.float64)


def linear_weights(d: int) -> np.ndarray:
    """gamma_q of section 3.2: S0, S1, then 2d biased cones."""
    nb = 2 * d
    g = [GAMMA_HI, (1 - GAMMA_HI) * GAMMA_LO] + [(1 - GAMMA_HI) * (1 - GAMMA_LO) / nb] * nb
    return np.array(g, dtype=np.float64)


# ---------------------------------------------------------------------------
# Bundle, with the rounded tables cached under oracle/tables/ (written by
# oracle/build_tables.py, which calls only this module)
# ---------------------------------------------------------------------------
_CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")


def tables(d: int, R: int) -> dict:
    """Everything the oracle RHS needs for (d, R)."""
    s0 = full_stencil(d, R)
    subs = substencils(d, R)
    fname = os.path.join(_CACHE_DIR, f"weights_d{d}_R{R}_ell{ELL_HAT}.npz")
    W = None
    if os.path.exists(fname):
        with np.load(fname, allow_pickle=False) as z:
            W = [z[f"q{q}"] for q in range(len(subs))]
    if W is None:
        W = [stencil_weights(d, R, q) for q in range(len(subs))]
        os.makedirs(_CACHE_DIR, exist_ok=True)
        tmp = fname + f".tmp{os.getpid()}.npz"
        np.savez(tmp, **{f"q{q}": w for q, w in enumerate(W)})
        os.replace(tmp, fname)
    nodes, wts = gauss_legendre_unit(R)
    return dict(
        d=d, R=R, s0=np.array(s0, dtype=np.int32), members=[np.array(m, dtype=np.int32) for m in subs],
        weights=W, gamma=linear_weights(d), n_pts=2 * d * R ** (d - 1),
        n_der=len(derivative_indices(d, R)), gl_nodes=np.array([float(x) for x in nodes]),
        gl_weights=np.array([float(w) for w in wts]),
        degrees=[max_unisolvent_degree([s0[h] for h in m]) for m in subs],
    )
