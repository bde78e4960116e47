"""Pins of the oracle's boundary conditions (section 5.3: ghost cells filled by the
boundary conditions, Riemann states outside the domain from the inner ones).

A reflecting wall is a mirror: a field on [0, 1] with reflecting walls evolves as
its mirror-doubled extension on the periodic [0, 2], so the right-hand side and
the KXRCF measure must agree with that periodic computation to rounding.  An
outflow boundary in a region the waves have not reached leaves the solution
equal to the periodic mirror-image computation.  A uniform inflow into the same
uniform state is steady."""
import numpy as np
import pytest

from paper_2401_16543_amd import inputs


def _field(n, seed=3):
    U = inputs.cell_averages(inputs.smooth(seed, 2, 3), 2 * n, 1.4, rule="gauss", q=3).numpy()
    return U[:, :n, :n].copy()           # any admissible field on [0, 1)^2 (not periodic)


def _mirror_x(U):
    """The field on [0, 2) x [0, 1): U on [0, 1), its mirror image (x -> 2 - x,
    x-momentum negated) on [1, 2)."""
    M = U[:, :, ::-1].copy()
    M[1] = -M[1]
    return np.concatenate([U, M], axis=2)


@pytest.mark.parametrize("R", [2, 3])
def test_reflecting_walls_are_mirrors(oracle_mod, R):
    n = 16
    U = _field(n)
    dx = [1.0 / n] * 2
    wall = oracle_mod.Oracle(2, R, (n, n), dx=dx)
    wall.set_boundary(0, "reflecting", "reflecting")
    per = oracle_mod.Oracle(2, R, (2 * n, n), dx=dx)
    D = _mirror_x(U)
    L_wall = wall.rhs(U)
    L_per = per.rhs(D)[:, :, :n]
    scale = np.abs(L_per).reshape(4, -1).max(axis=1)
    err = (np.abs(L_wall - L_per).reshape(4, -1).max(axis=1) / scale).max()
    assert err <= 1e-12, err
    # the indicator sees the mirror too: the wall faces' jumps vanish
    m_wall = wall.kxrcf(U, 1.5)[1]
    m_per = per.kxrcf(D, 1.5)[1].reshape(n, 2 * n)[:, :n].reshape(-1)
    assert np.abs(m_wall - m_per).max() <= 1e-12 * max(1.0, m_per.max())


def test_reflecting_box_conserves_mass_and_energy(oracle_mod):
    n, R = 16, 2
    U = _field(n, seed=8)
    o = oracle_mod.Oracle(2, R, (n, n))
    for a in (0, 1):
        o.set_boundary(a, "reflecting", "reflecting")
    L = o.rhs(U).reshape(4, -1)
    tot = np.abs(L.sum(axis=1)) / np.abs(L).sum(axis=1)
    assert tot[0] <= 1e-13 and tot[3] <= 1e-13        # no mass or energy through the walls


def test_outflow_ahead_of_the_waves_matches_mirror(oracle_mod):
    """Sod tube on [0, 1] with outflow ends: until the waves reach the ends it is
    the periodic mirror-image computation on [0, 2)."""
    R = 2
    D, m = inputs.sod("aligned", R)
    D = D.numpy()
    nx, ny = m["n"]
    per = oracle_mod.Oracle(2, R, (nx, ny), dx=[m["dx"]] * 2, gamma=1.4)
    out = oracle_mod.Oracle(2, R, (nx // 2, ny), dx=[m["dx"]] * 2, gamma=1.4)
    out.set_boundary(0, "outflow", "outflow")
    U = D[:, :, :nx // 2].copy()
    t = 0.0
    for _ in range(60):
        dt = per.cfl_dt(D, 0.4)
        D = per.step(D, dt)
        U = out.step(U, dt)
        t += dt
    assert t > 0.05
    assert np.abs(U - D[:, :, :nx // 2]).max() <= 1e-13


@pytest.mark.parametrize("u0", [0.5, 2.0])
def test_uniform_inflow_is_steady(oracle_mod, u0):
    """A uniform flow entering through an inflow side with its own state and
    leaving through an outflow side (subsonic and supersonic), reflecting walls
    across: steady to rounding."""
    n, R, gamma = 12, 2, 1.4
    rho, p = 1.0, 1.0
    state = np.array([rho, rho * u0, 0.0, p / (gamma - 1.0) + 0.5 * rho * u0 * u0])
    U = np.broadcast_to(state[:, None, None], (4, n, n)).copy()
    o = oracle_mod.Oracle(2, R, (n, n), gamma=gamma)
    o.set_boundary(0, "inflow", "outflow", lower_state=state)
    o.set_boundary(1, "reflecting", "reflecting")
    L = o.rhs(U)
    assert np.abs(L).max() <= 1e-12
    # a different inflow state is felt in the cells within reach of the ghosts
    # (stencil radius R plus the face), not beyond
    o.set_boundary(0, "inflow", "outflow", lower_state=state * np.array([1.1, 1.1, 1.0, 1.1]))
    L = o.rhs(U)
    assert np.abs(L[[0, 1, 3], :, 0]).min() > 1e-3
    assert np.abs(L[:, :, R + 1:]).max() <= 1e-12
    assert np.abs(L[2]).max() <= 1e-12                 # nothing pushes across the flow


@pytest.mark.parametrize("kind", ["outflow", "reflecting", "inflow"])
def test_ghost_fill_matches_explicit_extension(oracle_mod, kind):
    """The ghost cells of each kind written out: the field extended by R + 1
    explicit layers on both x sides (copies of the boundary cell, mirror images
    with x-momentum negated, or the inflow state) on a periodic domain gives the
    same limited Riemann states in the original cells (their stencils and
    limiter neighbourhoods never reach the far layers)."""
    n, R = 14, 2
    U = _field(n, seed=21)
    dx = [1.0 / n] * 2
    inflow = np.array([1.3, 0.4, -0.1, 3.0])
    e = R + 1
    if kind == "outflow":
        lo = np.repeat(U[:, :, :1], e, axis=2)
        hi = np.repeat(U[:, :, -1:], e, axis=2)
    elif kind == "reflecting":
        lo = U[:, :, e - 1::-1].copy()
        hi = U[:, :, :-e - 1:-1].copy()
        lo[1], hi[1] = -lo[1], -hi[1]
    else:
        lo = np.broadcast_to(inflow[:, None, None], (4, n, e)).copy()
        hi = lo.copy()
    X = np.concatenate([lo, U, hi], axis=2)
    bc = oracle_mod.Oracle(2, R, (n, n), dx=dx)
    bc.set_boundary(0, kind, kind, lower_state=inflow if kind == "inflow" else None,
                    upper_state=inflow if kind == "inflow" else None)
    ext = oracle_mod.Oracle(2, R, (n + 2 * e, n), dx=dx)
    s_bc = bc.states(U).reshape(n, n, -1, 4)
    s_ext = ext.states(X).reshape(n, n + 2 * e, -1, 4)[:, e:e + n]
    assert np.abs(s_bc - s_ext).max() <= 1e-13 * np.abs(s_ext).max()
