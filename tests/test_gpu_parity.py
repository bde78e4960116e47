"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Bar (spec tolerance): for every conserved variable k,
    max |X_gpu[k] - X_oracle[k]| / max |X_oracle[k]| <= 1e-12,
on the same seeded inputs.  Small grids are compared element by element; the
full-size workloads on sampled cells, in the launch configuration the benchmark
times."""
import sys

import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nv = a.shape[0]
    a, b = a.reshape(nv, -1), b.reshape(nv, -1)
    return max(float(np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300)) for k in range(nv))


@pytest.fixture(scope="module")
def K():
    from paper_2401_16543_amd import kfvm
    kfvm.load_library()
    return kfvm


def _state(kind, d, n, seed, gamma=1.4, q=3):
    if kind == "smooth":
        spec = inputs.smooth(seed, d, 8)
        return inputs.cell_averages(spec, n, gamma, rule="gauss", q=q)
    spec = inputs.discontinuous(seed, d, 6 if d == 2 else 4, 10.0, 100.0)
    return inputs.cell_averages(spec, n, gamma, rule="midpoint", q=4)


def _shape_state(U, n):
    # inputs are cubic; crop to a ragged box by taking a sub-block (still a valid state)
    d = len(n)
    sl = (slice(None),) + tuple(slice(0, x) for x in reversed(n))
    return U[sl].contiguous()


CASES = [
    # (dim, R, n per axis, kind, riemann)
    (2, 2, (64, 64), "smooth", "hllc"),
    (2, 2, (37, 29), "jumps", "hllc"),
    (2, 2, (48, 40), "jumps", "hll"),
    (2, 3, (40, 36), "jumps", "hllc"),
    (3, 2, (16, 16, 16), "smooth", "hllc"),
    (3, 2, (13, 11, 9), "jumps", "hllc"),
    (3, 3, (12, 10, 9), "jumps", "hllc"),
]


@pytest.mark.parametrize("d,R,n,kind,riemann", CASES)
def test_rhs_and_states_match_oracle(K, oracle_mod, d, R, n, kind, riemann):
    say(f"case rhs d={d} R={R} n={n} {kind} {riemann}")
    gamma = 1.4
    U = _shape_state(_state(kind, d, max(n), 100 + d * 10 + R, gamma), n)
    # a non-cubic box keeps the unit spacing of the cubic field it was cut from
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx, gamma=gamma, riemann=riemann)
    ref = orc.rhs(U.numpy())
    ref_states = orc.states(U.numpy())
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1, gamma=gamma)
    dev.set_riemann(riemann)
    dev.set_checking(True)
    Ud = U.cuda()
    got = dev.rhs(Ud).cpu().numpy()
    st = dev.face_states(Ud).cpu().numpy()
    e_rhs = rel_err(got, ref)
    e_st = rel_err(np.moveaxis(st, -1, 0), np.moveaxis(ref_states, -1, 0))
    say(f"  rhs rel err {e_rhs:.3e}  states rel err {e_st:.3e}")
    assert e_st <= TOL
    assert e_rhs <= TOL


def test_limiter_engaged_case_matches(K, oracle_mod):
    """Strong jumps so the positivity limiter acts; parity still holds."""
    d, R, n, gamma = 2, 3, 32, 1.4
    say("case limiter d=2 R=3 n=32")
    U = inputs.cell_averages(inputs.discontinuous(9, d, 6, 100.0, 1000.0), n, gamma, rule="midpoint", q=4)
    orc = oracle_mod.Oracle(d, R, (n, n), gamma=gamma, kappa=0.1)
    free = oracle_mod.Oracle(d, R, (n, n), gamma=gamma, limiter=False).states(U.numpy())
    ref_states = orc.states(U.numpy())
    assert np.abs(free - ref_states).max() > 1e-6          # the limiter acted
    dev = K.KFVM(d, (n, n), order=7, gamma=gamma)
    dev.set_limiter(True, 0.1)
    dev.set_checking(True)
    Ud = U.cuda()
    st = dev.face_states(Ud).cpu().numpy()
    assert rel_err(np.moveaxis(st, -1, 0), np.moveaxis(ref_states, -1, 0)) <= TOL
    assert rel_err(dev.rhs(Ud).cpu().numpy(), orc.rhs(U.numpy())) <= TOL


def test_ssp_rk3_trajectory_2d_64(K, oracle_mod):
    """The small 2D workload: 64^2 smooth seeded field, R = 2, 10 SSP-RK3 steps at CFL 0.4."""
    say("case trajectory 2d_smooth_64")
    U0, cfg = inputs.config_state("2d_smooth_64")
    d, n, gamma = cfg["d"], cfg["n"], cfg["gamma"]
    orc = oracle_mod.Oracle(d, 2, (n, n), gamma=gamma)
    dev = K.KFVM(d, (n, n), order=5, gamma=gamma)
    dev.set_checking(True)
    Uo, Ug = U0.numpy().copy(), U0.cuda()
    for _ in range(cfg["steps"]):
        dt_o = orc.cfl_dt(Uo, cfg["cfl"])
        dt_g = dev.cfl_dt(Ug, cfg["cfl"])
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o
        Uo = orc.step(Uo, dt_o)
        dev.step(Ug, dt_o)
    e = rel_err(Ug.cpu().numpy(), Uo)
    say(f"  10-step rel err {e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("d,n", [(2, (40, 24)), (3, (20, 12, 16))])
@pytest.mark.parametrize("form", ["sum", "max_axis"])
def test_cfl_dt_forms(K, oracle_mod, d, n, form):
    """Both CFL formulas against the oracle on a field with unequal spacings."""
    say(f"case cfl form {form} d={d}")
    U = inputs.cell_averages(inputs.discontinuous(4, d, 4, 10.0, 100.0), max(n), 1.4, rule="midpoint", q=2)
    U = U[(slice(None),) + tuple(slice(0, x) for x in reversed(n))].contiguous()
    dx = [0.5 / n[a] * (1 + a) for a in range(d)]
    orc = oracle_mod.Oracle(d, 2, n, dx=dx)
    dev = K.KFVM(d, n, dx=dx, order=5)
    orc.set_cfl_form(form)
    dev.set_cfl_form(form)
    assert np.isnan(dev.stats()["min_rho"])                  # no CFL reduction yet
    dt_o, dt_g = orc.cfl_dt(U.numpy(), 0.7), dev.cfl_dt(U.cuda(), 0.7)
    say(f"  dt {dt_g:.6e} (oracle {dt_o:.6e})")
    assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    # the same reduction reports the least density and pressure of the state
    Un = U.numpy().reshape(d + 2, -1)
    p = 0.4 * (Un[-1] - 0.5 * (Un[1:1 + d] ** 2).sum(0) / Un[0])
    st = dev.stats()
    assert st["min_rho"] == Un[0].min()
    assert abs(st["min_p"] - p.min()) <= 1e-13 * p.min()
    with pytest.raises(K.KfvmError):
        dev._check(dev.lib.kfvm_set_cfl_form(dev._h, 7))      # an unknown form


@pytest.mark.parametrize("name,nsample", [("2d_jumps_1024", 600), ("3d_smooth_256", 160), ("3d_jumps_384_r3", 60)])
def test_full_size_sampled(K, oracle_mod, name, nsample):
    """Full-size workloads: the GPU RHS over the whole grid (the benchmark's
    launch configuration) against the oracle at sampled cells, plus conservation."""
    say(f"case full-size {name}")
    U, cfg = inputs.config_state(name, device="cuda")
    d, n, R, gamma = cfg["d"], cfg["n"], cfg["R"], cfg["gamma"]
    dev = K.KFVM(d, (n,) * d, order=2 * R + 1, gamma=gamma)
    dev.set_checking(True)
    L = dev.rhs(U)
    torch.cuda.synchronize()
    Lh = L.cpu().numpy().reshape(d + 2, -1)
    Uh = U.cpu().numpy()
    rng = np.random.default_rng(5)
    ncell = n ** d
    cells = np.concatenate([[0, ncell - 1, n - 1, ncell - n], rng.integers(0, ncell, nsample)])
    orc = oracle_mod.Oracle(d, R, (n,) * d, gamma=gamma)
    ref = orc.rhs_cells(Uh, cells)
    scale = np.abs(Lh).max(axis=1)
    err = (np.abs(Lh[:, cells].T - ref) / scale).max()
    say(f"  sampled rel err {err:.3e}")
    assert err <= TOL
    # periodic conservation over the whole grid
    tot = np.abs(Lh.sum(axis=1)) / np.abs(Lh).sum(axis=1)
    assert np.all(tot <= 1e-13)


def test_weights_passed_in_match_built(K):
    """Tables handed over at init (the oracle's 50-digit ones) and the library's
    own binary128 tables give the same RHS to rounding."""
    from oracle import weights as W
    say("case weights in")
    d, R, n = 2, 2, 32
    U = _state("jumps", d, n, 3).cuda()
    a = K.KFVM(d, (n, n), order=5, weights=W.tables(d, R)).rhs(U)
    b = K.KFVM(d, (n, n), order=5).rhs(U)
    assert rel_err(a.cpu().numpy(), b.cpu().numpy()) <= 1e-14


def test_length_scale_entry_point(K, oracle_mod):
    """Tables at another kernel length scale (l = 20 cells): the library's own
    binary128 build through kfvm_init_length_scale against the oracle with its
    50-digit tables at the same l, RHS to 1e-12; l = 5 through the entry point
    is the default init, bit for bit."""
    from oracle import weights as W
    say("case length scale")
    d, R, n = 2, 2, 32
    U = _state("jumps", d, n, 3)
    a = K.KFVM(d, (n, n), order=5, ell_hat=5.0).rhs(U.cuda())
    b = K.KFVM(d, (n, n), order=5).rhs(U.cuda())
    assert torch.equal(a, b)
    T = dict(W.tables(d, R))
    T["weights"] = [W.stencil_weights(d, R, q, ell_hat=20) for q in range(len(T["weights"]))]
    ref = oracle_mod.Oracle(d, R, (n, n), tables=T).rhs(U.numpy())
    got = K.KFVM(d, (n, n), order=5, ell_hat=20.0).rhs(U.cuda()).cpu().numpy()
    e, moved = rel_err(got, ref), rel_err(got, b.cpu().numpy())
    say(f"  rel err vs oracle at l = 20: {e:.3e}; change from l = 5: {moved:.3e}")
    assert e <= TOL and moved > 1e-8


def test_deterministic(K):
    say("case determinism")
    d, n = 3, 16
    U = _state("jumps", d, n, 4).cuda()
    dev = K.KFVM(d, (n,) * d, order=5)
    a = dev.rhs(U).clone()
    b = dev.rhs(U)
    assert torch.equal(a, b)


def test_nonphysical_input_is_reported(K):
    say("case nonphysical")
    d, n = 2, 16
    U = _state("smooth", d, n, 6)
    U[3, 4, 5] = 0.0                 # negative pressure in one cell
    dev = K.KFVM(d, (n, n), order=5)
    dev.set_checking(True)
    with pytest.raises(K.KfvmError) as ei:
        dev.rhs(U.cuda())
    assert ei.value.code == K.KFVM_ERR_NONPHYSICAL
    assert dev.status() == K.KFVM_OK        # cleared


@pytest.mark.parametrize("precision", ["fp64", "split_f16"])
def test_step_leaves_state_on_nonphysical(K, precision):
    """The non-physical contract of kfvm_step: when a stage meets a non-physical
    state, U is left unmodified (bitwise) and the error is reported, with the
    check on (returned by the step) and off (kfvm_status afterwards); a later
    step from an admissible state runs normally."""
    say(f"case step nonphysical {precision}")
    d, n = 2, 16
    U = _state("smooth", d, n, 6)
    U[3, 4, 5] = 0.0                 # negative pressure in one cell
    dev = K.KFVM(d, (n, n), order=5)
    dev.set_precision(precision)
    Ud = U.cuda()
    before = Ud.clone()
    dev.set_checking(True)
    with pytest.raises(K.KfvmError) as ei:
        dev.step(Ud, 1e-3)
    assert ei.value.code == K.KFVM_ERR_NONPHYSICAL
    assert torch.equal(Ud, before)
    dev.set_checking(False)
    dev.step(Ud, 1e-3)
    assert dev.status() == K.KFVM_ERR_NONPHYSICAL
    assert torch.equal(Ud, before)
    assert dev.status() == K.KFVM_OK        # cleared
    good = _state("smooth", d, n, 6).cuda()
    g0 = good.clone()
    dev.step(good, 1e-3)
    assert dev.status() == K.KFVM_OK
    assert not torch.equal(good, g0) and bool(torch.isfinite(good).all())


def test_bad_arguments_are_rejected(K):
    say("case bad args")
    with pytest.raises(K.KfvmError):
        K.KFVM(2, (5, 64), order=5)          # n < 2R + 2
    with pytest.raises(K.KfvmError):
        K.KFVM(2, (64, 64), order=6)
    dev = K.KFVM(2, (16, 16), order=5)
    U = _state("smooth", 2, 16, 1).cuda()
    rc = dev.lib.kfvm_rhs(dev._h, dev._state(U), dev._state(U))
    assert rc == K.KFVM_ERR_ARG


def test_split_path_cell_limit(K):
    """The split path stores through 32-bit lane offsets of up to 32 bytes per
    cell: a grid of 2^27 cells is refused by kfvm_set_precision (the FP64 path
    still takes it); one cell fewer along a row is accepted."""
    say("case split-path cell limit")
    dev = K.KFVM(2, (16384, 8192), order=5)
    with pytest.raises(K.KfvmError):
        dev.set_precision("split_f16")
    dev.close()
    dev = K.KFVM(2, (16383, 8192), order=5)
    dev.set_precision("split_f16")
    dev.close()
