"""Pins of the oracle's stencils and reconstruction vectors against what the
paper prints and what the mathematics fixes (no GPU)."""
import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import weights as W

GOLDEN = {}
with open(__file__.rsplit("/", 1)[0] + "/golden/paper_constants.txt") as f:
    for line in f:
        line = line.split("#")[0].split()
        if line:
            GOLDEN[line[0]] = float(line[1])


def test_stencil_sizes_match_paper():
    s = [len(m) for m in W.substencils(2, 2)]
    assert s[0] == GOLDEN["stencil_size_2d_R2_S0"]
    assert all(x == GOLDEN["stencil_size_2d_R2_sub"] for x in s[1:])
    assert len(s) - 1 == GOLDEN["n_substencils_2d"]
    s = [len(m) for m in W.substencils(2, 3)]
    assert s[0] == GOLDEN["stencil_size_2d_R3_S0"]
    assert s[1] == GOLDEN["stencil_size_2d_R3_S1"]
    assert all(x == GOLDEN["stencil_size_2d_R3_biased"] for x in s[2:])
    assert len(W.substencils(3, 2)) - 1 == GOLDEN["n_substencils_3d"]


def test_stencils_brute_force_3d():
    # brute-force recount of the set definitions of section 3.1
    for R in (2, 3):
        pts = [p for p in itertools.product(range(-R, R + 1), repeat=3) if sum(c * c for c in p) <= R * R]
        subs = W.substencils(3, R)
        s0 = W.full_stencil(3, R)
        assert sorted(pts) == sorted(s0)
        assert [s0[h] for h in subs[1]] == [p for p in s0 if sum(c * c for c in p) <= (R - 1) ** 2]
        # +y cone: |i| <= j and |k| <= j
        assert [s0[h] for h in subs[4]] == [p for p in s0 if abs(p[0]) <= p[1] and abs(p[2]) <= p[1]]
        # -z cone
        assert [s0[h] for h in subs[7]] == [p for p in s0 if abs(p[0]) <= -p[2] and abs(p[1]) <= -p[2]]


def test_degrees_and_derivative_counts():
    for d, R, key in [(2, 2, "degree_S0_R2"), (2, 3, "degree_S0_R3"),
                      (3, 2, "degree_S0_R2"), (3, 3, "degree_S0_R3")]:
        assert W.max_unisolvent_degree(W.full_stencil(d, R)) == GOLDEN[key]
    for d, R in [(2, 2), (2, 3), (3, 2), (3, 3)]:
        assert len(W.derivative_indices(d, R)) == GOLDEN[f"n_derivs_{d}d_R{R}"]


def test_paper_constants_used_by_oracle():
    """The oracle's epsilon of the nonlinear weights (section 3.3) and its kernel
    length scale in cells (l = 5 Delta, sections 5.1 and 6) are the printed ones."""
    from oracle import core
    assert core.EPS_WENO == GOLDEN["eps_weno"]
    assert W.ELL_HAT == GOLDEN["ell_over_dx"]


def test_linear_weights():
    g2, g3 = W.linear_weights(2), W.linear_weights(3)
    assert g2[0] == GOLDEN["gamma_hi"]
    assert math.isclose(g2[1], (1 - GOLDEN["gamma_hi"]) * GOLDEN["gamma_lo"])
    assert math.isclose(g2.sum(), 1.0) and math.isclose(g3.sum(), 1.0)
    assert len(g2) == 6 and len(g3) == 8


def test_polynomial_interpolant_closed_form():
    # when the stencil has exactly as many cells as monomials the kernel part
    # drops out: 1D cells -1, 0, 1 with p = 2 give the parabola through the
    # three averages, whose value at x = 1/2 is (-g_-1 + 5 g_0 + 2 g_1) / 6,
    # whatever the length scale
    for ell in (1, 5, 20):
        r = W.reconstruction_vectors([(-1,), (0,), (1,)], 2, [(0.5,)], [(1,)], ell_hat=ell)
        assert [float(x) for x in r[0]] == pytest.approx([-1 / 6, 5 / 6, 2 / 6], abs=1e-30)
        # derivative of that parabola at 0: (g_1 - g_-1) / 2
        assert [float(x) for x in r[1]] == pytest.approx([-0.5, 0.0, 0.5], abs=1e-30)


def _gl_avg(f, cell, d, q=10):
    # cell average by a q-point tensor Gauss-Legendre rule (independent of the
    # closed forms the oracle uses)
    x, w = np.polynomial.legendre.leggauss(q)
    x, w = 0.5 * x, 0.5 * w
    tot = 0.0
    for idx in itertools.product(range(q), repeat=d):
        pt = np.array([cell[k] + x[i] for k, i in enumerate(idx)])
        tot += np.prod([w[i] for i in idx]) * f(pt)
    return tot


@pytest.mark.parametrize("d,R", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_polynomial_exactness(d, R):
    """r . (cell averages of a polynomial of degree <= p_q) equals its value at x*
    and the derivatives at 0 (the constraint P^T r = S, section 2.1)."""
    rng = np.random.default_rng(7)
    T = W.tables(d, R)
    s0 = T["s0"]
    pts = [tuple(float(c) for c in x) for x in W.face_points(d, R)]
    ders = W.derivative_indices(d, R)
    for q, mem in enumerate(T["members"]):
        p = T["degrees"][q]
        mons = W.monomials(d, p)
        coef = rng.normal(size=len(mons))

        def f(x):
            return sum(c * np.prod([x[k] ** a[k] for k in range(d)]) for c, a in zip(coef, mons))

        g = np.array([_gl_avg(f, s0[h], d, q=max(3, p)) for h in mem])
        tab = T["weights"][q]
        got = tab @ g
        want = [f(np.array(x)) for x in pts]
        for al in ders:
            val = 0.0
            for c, a in zip(coef, mons):
                if all(a[k] == al[k] for k in range(d)):
                    val += c * np.prod([math.factorial(t) for t in al])
            want.append(val)
        scale = np.abs(tab).sum(1) * np.abs(g).max()
        assert np.all(np.abs(got - np.array(want)) <= 1e-13 * scale + 1e-14)


def test_kernel_part_reproduced_2d():
    """Data from f = sum_l a_l K(x, x_l) + poly with P^T a = 0 lie in the
    approximation space, so r . g must equal f(x*) and the derivatives of f at 0.
    Averages and targets are computed by quadrature and by mpmath
    differentiation, independently of the closed forms in the oracle."""
    d, R = 2, 2
    T = W.tables(d, R)
    s0 = T["s0"]
    rng = np.random.default_rng(3)
    for q in (0, 1, 2):
        mem = T["members"][q]
        cells = [tuple(int(c) for c in s0[h]) for h in mem]
        p = T["degrees"][q]
        mons = W.monomials(d, p)
        # P from quadrature, a in the null space of P^T
        P = np.array([[_gl_avg(lambda x, a=a: np.prod([x[k] ** a[k] for k in range(d)]), c, d, 6)
                       for a in mons] for c in cells])
        _, _, vt = np.linalg.svd(P.T)
        a = vt[len(mons):].T @ rng.normal(size=len(cells) - len(mons))
        b = rng.normal(size=len(mons))
        ell = 5.0

        def f(x):
            k = sum(al * math.exp(-((x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2) / (2 * ell ** 2))
                    for al, c in zip(a, cells))
            return k + sum(bb * x[0] ** m[0] * x[1] ** m[1] for bb, m in zip(b, mons))

        g = np.array([_gl_avg(f, c, d, 12) for c in cells])
        got = T["weights"][q] @ g
        want = [f(np.array(x, dtype=float)) for x in W.face_points(d, R)]
        for al in W.derivative_indices(d, R):
            with mpmath.workdps(30):
                fm = lambda x, y: sum(aa * mpmath.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2 * ell ** 2))
                                      for aa, c in zip(a, cells)) + \
                    sum(bb * x ** m[0] * y ** m[1] for bb, m in zip(b, mons))
                want.append(float(mpmath.diff(fm, (0, 0), tuple(al))))
        assert np.allclose(got, want, rtol=0, atol=1e-9 * max(1.0, np.abs(g).max()))


def test_brute_force_high_precision_2d_r2():
    # an 80-digit solve of every 2D R = 2 stencil at the paper's length scale
    # (l = 5 Delta, from the golden file) agrees with the 50-digit tables the
    # oracle uses to within rounding of the float64 result
    T = W.tables(2, 2)
    ell = GOLDEN["ell_over_dx"]
    for q in range(len(T["members"])):
        hi = W.stencil_weights.__wrapped__(2, 2, q, ell, 80)
        lo = T["weights"][q]
        scale = np.abs(hi).max(axis=1, keepdims=True)
        assert np.all(np.abs(hi - lo) <= 2 * np.finfo(float).eps * scale)


@pytest.mark.parametrize("d,R", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_row_sums(d, R):
    # constants are reproduced (point rows sum to 1) and have no derivatives
    T = W.tables(d, R)
    npt = T["n_pts"]
    for tab in T["weights"]:
        s = np.abs(tab).sum(1)
        assert np.all(np.abs(tab[:npt].sum(1) - 1) <= 1e-15 * s[:npt] * tab.shape[1])
        assert np.all(np.abs(tab[npt:].sum(1)) <= 1e-15 * s[npt:] * tab.shape[1])


@pytest.mark.parametrize("d,R", [(2, 2), (3, 2), (2, 3), (3, 3)])
def test_mirror_and_rotation_symmetry(d, R):
    """Mirroring x -> -x maps S0 to itself, the +x cone to the -x cone and the
    upper x-face points to the lower ones (section 3.1); permuting x and y does
    the same for the y faces.  The tables must follow."""
    T = W.tables(d, R)
    s0 = [tuple(int(c) for c in o) for o in T["s0"]]
    pos = {o: h for h, o in enumerate(s0)}
    pts = [tuple(float(c) for c in x) for x in W.face_points(d, R)]
    ders = W.derivative_indices(d, R)
    npt = T["n_pts"]

    def check(cellmap, ptmap, dermap, qmap):
        for q, mem in enumerate(T["members"]):
            q2 = qmap(q)
            mem2 = list(T["members"][q2])
            tab, tab2 = T["weights"][q], T["weights"][q2]
            for row in range(tab.shape[0]):
                if row < npt:
                    row2, sgn = pts.index(ptmap(pts[row])), 1.0
                else:
                    al = ders[row - npt]
                    al2, sgn = dermap(al)
                    row2 = npt + ders.index(al2)
                for j, h in enumerate(mem):
                    j2 = mem2.index(pos[cellmap(s0[h])])
                    assert abs(tab[row, j] - sgn * tab2[row2, j2]) <= 1e-13 * np.abs(tab[row]).max()

    flip = lambda o: (-o[0],) + tuple(o[1:])
    check(flip, lambda x: (-x[0],) + tuple(x[1:]) if abs(x[0]) == 0.5 else (x[0] if x[0] == 0 else -x[0],) + tuple(x[1:]),
          lambda al: (al, (-1.0) ** al[0]),
          lambda q: q if q < 2 else (q ^ 1 if q in (2, 3) else q))
    swap = lambda o: (o[1], o[0]) + tuple(o[2:])
    check(swap, lambda x: (x[1], x[0]) + tuple(x[2:]), lambda al: ((al[1], al[0]) + tuple(al[2:]), 1.0),
          lambda q: {2: 4, 3: 5, 4: 2, 5: 3}.get(q, q))


def test_kernel_matrix_symmetric_on_unit_cells():
    # on identical unit cells the averaged kernel depends on the offset only
    # through even functions, so Q = Q^T (the asymmetric form of section 2.2
    # coincides with its transpose here)
    with mpmath.workdps(30):
        for t in range(-4, 5):
            assert abs(W._kernel_avg_1d(mpmath.mpf(t), 5) - W._kernel_avg_1d(mpmath.mpf(-t), 5)) < 1e-28


def _max_fourier_growth(R, a):
    """Largest real part (times the spacing) of the semi-discrete linear-advection
    symbol of the linear S0 scheme in 2D: upwind fluxes at the face Gauss points
    of the cell's own reconstruction, a = advection velocity."""
    T = W.tables(2, R)
    pts = [tuple(float(v) for v in p) for p in W.face_points(2, R)]
    s0 = np.asarray(T["s0"])
    r = np.asarray(T["weights"][0])[:len(pts)]
    nodes, gw = np.asarray(T["gl_nodes"]), np.asarray(T["gl_weights"])
    th = np.linspace(-np.pi, np.pi, 181)
    TX, TY = np.meshgrid(th, th, indexing="ij")
    ph = np.exp(1j * (TX[..., None] * s0[None, None, :, 0] + TY[..., None] * s0[None, None, :, 1]))
    sym = []
    for axis in (0, 1):
        face = [i for i, p in enumerate(pts) if abs(p[axis] - 0.5) < 1e-12]
        sym.append(sum(gw[np.argmin(np.abs(nodes - pts[i][1 - axis]))] * (ph @ r[i]) for i in face))
    lam = -(a[0] * (1 - np.exp(-1j * TX)) * sym[0] + a[1] * (1 - np.exp(-1j * TY)) * sym[1])
    return lam.real.max()


def test_linear_scheme_fourier_growth():
    """A property of the tables, not a paper pin: the R = 2 linear scheme has no
    growing Fourier mode for linear advection (up to 3e-4 / spacing for a flow
    along an axis), while the R = 3 one has modes odd in the transverse index that
    grow at up to 0.19 / spacing (flow along x), 0.011 / spacing diagonally.  They
    are what the linear R = 3 scheme shows on the 256^2 vortex (design notes);
    WENO-AO damps them."""
    assert _max_fourier_growth(2, (1.0, 1.0)) <= 1e-12
    assert _max_fourier_growth(2, (1.0, 0.0)) <= 5e-4
    assert _max_fourier_growth(3, (1.0, 0.0)) > 0.15
    assert 0.005 < _max_fourier_growth(3, (1.0, 1.0)) < 0.05
