"""Pins of the oracle's limiter flattener eta (section 4: the bounds
rho_max (1 + kappa - kappa eta), rho_min (1 - kappa + kappa eta),
p_min (1 - kappa + kappa eta), with eta tending to one only where the flow
compresses).  The paper defers eta's rule to a reference it does not reproduce;
the oracle's reading is a ramp in the undivided velocity divergence against the
least sound speed of the 3^d block.  These tests pin what that reading must
satisfy whatever its constants: the two ends of the ramp reduce the limiter to
the kappa-widened and to the unwidened bounds; eta is zero under expansion,
invariant under a Galilean boost, under scaling velocity and sound speed
together, and under a transpose of the field; it grows with compression, falls
under refinement (an undivided difference), and sees the coldest state of the
block, not the cell's own."""
import numpy as np
import pytest

GAMMA = 1.4
K1 = 0.25


def _state(rho, u, v, p):
    """Conserved 2D state [4, ny, nx] from primitive fields."""
    return np.stack([rho, rho * u, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])


def _grid(n):
    x = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(x, x, indexing="ij")
    return X, Y


def _oracle(oracle_mod, n, R=2, k1=K1, kappa=0.5, bcs=("outflow", "outflow")):
    o = oracle_mod.Oracle(2, R, (n, n), dx=[1.0 / n] * 2, gamma=GAMMA, kappa=kappa, flattener=k1)
    for a in (0, 1):
        if bcs[a] != "periodic":
            o.set_boundary(a, bcs[a], bcs[a])
    return o


def _jumpy(n, a):
    """A density and pressure jump across x = 0.5 carried by the linear velocity
    u = a (x - 1/2), v = 0 (a > 0 expands, a < 0 compresses)."""
    X, Y = _grid(n)
    rho = np.where(X < 0.5 + 0.1 * np.sin(2 * np.pi * Y), 1.0, 0.125)
    p = np.where(X < 0.5 + 0.1 * np.sin(2 * np.pi * Y), 1.0, 0.1)
    return _state(rho, a * (X - 0.5), 0.0 * X, p)


def test_expansion_leaves_the_kappa_bounds(oracle_mod):
    n = 24
    U = _jumpy(n, 3.0)
    on, off = _oracle(oracle_mod, n), _oracle(oracle_mod, n, k1=None)
    assert np.all(on.flattener(U) == 0.0)
    assert np.array_equal(on.rhs(U), off.rhs(U))


def test_strong_compression_gives_the_unwidened_bounds(oracle_mod):
    """eta = 1 everywhere: the limiter with kappa = 0.5 acts as with kappa = 0."""
    n = 24
    U = _jumpy(n, -200.0)
    on = _oracle(oracle_mod, n)
    assert np.all(on.flattener(U) == 1.0)
    L_on = on.rhs(U)
    L_k0 = _oracle(oracle_mod, n, k1=None, kappa=0.0).rhs(U)
    L_k5 = _oracle(oracle_mod, n, k1=None).rhs(U)
    assert np.array_equal(L_on, L_k0)
    assert np.abs(L_k5 - L_k0).max() > 1e-6 * np.abs(L_k0).max()      # the limiter bites here


def _smooth_flow(n, seed=4, amp=1.0):
    X, Y = _grid(n)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, 6)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * X + ph[0]) * np.cos(2 * np.pi * Y + ph[1])
    u = amp * np.sin(2 * np.pi * X + ph[2]) * np.cos(2 * np.pi * Y + ph[3])
    v = amp * np.cos(2 * np.pi * X + ph[4]) * np.sin(2 * np.pi * Y + ph[5])
    p = 1.0 + 0.2 * np.cos(2 * np.pi * (X + Y) + ph[0])
    return rho, u, v, p


def test_eta_range_and_galilean_invariance(oracle_mod):
    n = 32
    rho, u, v, p = _smooth_flow(n, amp=3.0)
    o = _oracle(oracle_mod, n, k1=0.05, bcs=("periodic", "periodic"))
    eta = o.flattener(_state(rho, u, v, p))
    assert eta.min() == 0.0 and eta.max() == 1.0 and np.any((eta > 0) & (eta < 1))
    boosted = o.flattener(_state(rho, u + 0.7, v - 1.3, p))
    assert np.abs(boosted - eta).max() <= 1e-12


def test_eta_invariant_under_velocity_and_sound_speed_scaling(oracle_mod):
    n = 32
    rho, u, v, p = _smooth_flow(n, seed=5, amp=3.0)
    o = _oracle(oracle_mod, n, k1=0.05, bcs=("periodic", "periodic"))
    eta = o.flattener(_state(rho, u, v, p))
    assert np.any((eta > 0) & (eta < 1))
    s = 2.5
    assert np.abs(o.flattener(_state(rho, s * u, s * v, s * s * p)) - eta).max() <= 1e-12


def test_eta_transposes_with_the_field(oracle_mod):
    n = 32
    rho, u, v, p = _smooth_flow(n, seed=6, amp=3.0)
    o = _oracle(oracle_mod, n, k1=0.05, bcs=("periodic", "periodic"))
    eta = o.flattener(_state(rho, u, v, p)).reshape(n, n)
    eta_t = o.flattener(_state(rho.T, v.T, u.T, p.T)).reshape(n, n)
    assert np.any((eta > 0) & (eta < 1))
    assert np.abs(eta_t - eta.T).max() <= 1e-12


def test_eta_grows_with_compression(oracle_mod):
    n = 16
    X, Y = _grid(n)
    o = _oracle(oracle_mod, n)
    prev = None
    for a in [2.0, 0.0, -1.0, -2.0, -3.0, -4.0, -6.0, -10.0, -20.0]:
        eta = o.flattener(_state(1.0 + 0 * X, a * (X - 0.5), 0 * X, 1.0 + 0 * X))
        if a >= 0:
            assert np.all(eta == 0.0)
        if prev is not None:
            assert np.all(eta >= prev)
        prev = eta
    assert np.all(prev == 1.0)


def test_eta_is_undivided(oracle_mod):
    """On a linear velocity field the undivided divergence halves under refinement:
    on the ramp, eta + 1 halves with the grid spacing."""
    X, Y = _grid(16)
    c = np.sqrt(GAMMA)
    a = -1.5 * K1 * c * 16          # eta = 0.5 on the 16^2 grid's interior
    o16, o32 = _oracle(oracle_mod, 16, bcs=("periodic", "periodic")), _oracle(oracle_mod, 32, bcs=("periodic", "periodic"))
    one = 1.0 + 0 * X
    e16 = o16.flattener(_state(one, a * X, 0 * X, one)).reshape(16, 16)[:, 4:12]
    X2, _ = _grid(32)
    one2 = 1.0 + 0 * X2
    e32 = o32.flattener(_state(one2, a * X2, 0 * X2, one2)).reshape(32, 32)[:, 8:24]
    # periodic wrap breaks the linear field only at the seam, far from these columns
    assert np.abs(e16 - 0.5).max() <= 1e-12
    assert np.all(e32 == 0.0)                # (0.5 + 1) / 2 - 1 < 0: below the onset


def test_eta_takes_the_coldest_state_of_the_block(oracle_mod):
    """A colder diagonal neighbour (lower sound speed) raises eta; a hotter one
    leaves it; neither changes the divergence."""
    n = 16
    X, Y = _grid(n)
    one = 1.0 + 0 * X
    a = -1.2 * K1 * np.sqrt(GAMMA) * n    # eta = 0.2 on uniform sound speed
    o = _oracle(oracle_mod, n, bcs=("periodic", "periodic"))
    base = o.flattener(_state(one, a * (X - 0.5), 0 * X, one)).reshape(n, n)
    i, j = 8, 8
    assert abs(base[j, i] - 0.2) <= 1e-12
    for scale, rises in [(0.25, True), (4.0, False)]:
        p = one.copy()
        p[j + 1, i + 1] = scale                  # sound speed sqrt(gamma p / rho) at a corner
        eta = o.flattener(_state(one, a * (X - 0.5), 0 * X, p)).reshape(n, n)
        if rises:
            # c_min halves: -d / (k1 c_min) - 1 = 2 (1.2) - 1 > 1, clamped to 1
            assert abs(eta[j, i] - 1.0) <= 1e-12
        else:
            assert eta[j, i] == base[j, i]


@pytest.mark.parametrize("R", [2, 3])
def test_flattener_only_narrows_bounds(oracle_mod, R):
    """eta in [0, 1] moves each bound between its kappa-widened and unwidened
    values, so on a compressive jump the flattened limiter scales each cell's
    states toward its average at least as much as the kappa limiter: no face
    state deviates more from the cell average, and some deviate less."""
    n = 24
    U = _jumpy(n, -20.0)
    on = _oracle(oracle_mod, n, R=R)
    eta = on.flattener(U)
    assert np.any((eta > 0) & (eta < 1)) or np.any(eta == 1.0)
    s_on = on.states(U)
    s_off = _oracle(oracle_mod, n, R=R, k1=None).states(U)
    Uc = U.reshape(4, -1).T[:, None, :]
    dev_on = np.abs(s_on - Uc).max(axis=(1, 2))
    dev_off = np.abs(s_off - Uc).max(axis=(1, 2))
    assert np.all(dev_on <= dev_off * (1 + 1e-12) + 1e-15)
    assert np.any(dev_on < dev_off * (1 - 1e-6))
