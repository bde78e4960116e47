"""The KXRCF troubled-cell indicator and the two-pass reconstruction on the GPU
(through the C-ABI) against the FP64 CPU oracle.

Jumps are continuous: they match to rounding.  Flags are integers decided in
float64 on both sides from values that differ by rounding, so they must agree
except at cells whose measure lies within 1e-9 of the threshold (relative).
Right-hand sides of the FP64 path match the oracle's two-pass scheme to 1e-12
(the oracle replays the GPU's decisions where a near-threshold cell differs);
the split-precision path keeps its own accuracy bar."""
import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu
M = 1.5            # the paper's power of Delta
NEAR = 1e-9        # relative band around Delta^m where the two sides may decide differently


def say(*a):
    print(*a, flush=True)


def rel_err(a, b):
    nv = a.shape[0]
    a, b = np.asarray(a).reshape(nv, -1), np.asarray(b).reshape(nv, -1)
    return max(float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in range(nv))


@pytest.fixture(scope="module")
def K():
    from paper_2401_16543_amd import kfvm
    kfvm.load_library()
    return kfvm


def _entropy(U, d, gamma):
    U = U.reshape(d + 2, -1)
    p = (gamma - 1.0) * (U[d + 1] - 0.5 * (U[1:1 + d] ** 2).sum(0) / U[0])
    return p / U[0] ** gamma


def _cell_avg(fun, n, q=3):
    """Cell averages on the periodic unit box (spacing 1 / max(n)) by q-point Gauss rules."""
    g, w = np.polynomial.legendre.leggauss(q)
    h = 1.0 / max(n)
    axes = [(np.arange(x) + 0.5) * h for x in n]
    acc = 0.0
    for idx in np.ndindex(*([q] * len(n))):
        pts = [axes[a] + 0.5 * g[idx[a]] * h for a in range(len(n))]
        X = np.meshgrid(*pts[::-1], indexing="ij")[::-1]          # x, y[, z] on a (z,) y, x grid
        acc = acc + np.prod([0.5 * w[i] for i in idx]) * fun(*X)
    return acc


def _wave_block(d, n, seed, gamma=1.4):
    """A smooth wave (one density and one pressure mode, uniform velocity) with a
    denser block whose faces are contacts: part of the grid flagged, part smooth."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 3, size=(2, 3))
    ph = rng.random(2) * 2 * np.pi
    tw = 2 * np.pi
    rho = _cell_avg(lambda *X: 1.0 + 0.2 * np.sin(tw * sum(k[0, a] * X[a] for a in range(d)) + ph[0]), n)
    p = _cell_avg(lambda *X: 1.0 + 0.1 * np.cos(tw * sum(k[1, a] * X[a] for a in range(d)) + ph[1]), n)
    u = np.array([0.3, -0.2, 0.1])[:d]
    U = np.stack([rho] + [rho * u[a] for a in range(d)] + [p / (gamma - 1.0) + 0.5 * rho * (u ** 2).sum()])
    blk = (slice(None),) + tuple(slice(x // 4, x // 2) for x in reversed(n))
    U[blk] *= 1.6
    return torch.from_numpy(np.ascontiguousarray(U))


def _jumps_state(d, n, seed):
    U = inputs.cell_averages(inputs.discontinuous(seed, d, 6 if d == 2 else 4, 10.0, 100.0), max(n), 1.4,
                             rule="midpoint", q=4 if d == 2 else 2)
    return U[(slice(None),) + tuple(slice(0, x) for x in reversed(n))].contiguous()


CASES = [
    (2, 2, (64, 64), "wave"),
    (2, 2, (37, 29), "jumps"),
    (2, 3, (40, 36), "wave"),
    (3, 2, (16, 16, 16), "wave"),
    (3, 2, (13, 11, 9), "jumps"),
    (3, 3, (16, 12, 10), "wave"),
    (3, 3, (12, 10, 9), "jumps"),
]


def _state(d, n, kind, seed):
    return _wave_block(d, n, seed) if kind == "wave" else _jumps_state(d, n, seed)


def _compare_decisions(flags_gpu, meas, thr):
    """Flags equal except within NEAR of the threshold; returns the count of such cells."""
    want = ~(meas < thr)
    got = flags_gpu[0].astype(bool)
    assert np.all(flags_gpu == flags_gpu[:1])           # one decision per cell, every variable
    diff = got != want
    assert np.all(np.abs(meas[diff] / thr - 1.0) <= NEAR), meas[diff] / thr
    return int(diff.sum())


@pytest.mark.parametrize("d,R,n,kind", CASES)
def test_jumps_and_flags_match_oracle(K, oracle_mod, d, R, n, kind):
    say(f"case kxrcf d={d} R={R} n={n} {kind}")
    U = _state(d, n, kind, 40 + d * 10 + R)
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    f_o, meas, J_o = orc.kxrcf(U.numpy(), M)
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    J, fl = dev.kxrcf(U.cuda(), M)
    J, fl = J.cpu().numpy(), fl.cpu().numpy()
    Jup = np.stack([J_o[:, 2 * a + 1] for a in range(d)])
    inf_o, inf_g = ~np.isfinite(Jup), ~np.isfinite(J)
    assert np.array_equal(inf_o, inf_g)
    # rounding of q = p / rho^gamma at a point grows with q itself (a point
    # state near vacuum has a large q and an ill-conditioned one), so the error
    # is measured against the larger of the jump and the largest cell entropy
    scale = _entropy(U.numpy(), d, 1.4).max()
    fin = ~inf_g
    err = (np.abs(J[fin] - Jup[fin]) / (scale + Jup[fin])).max() if fin.any() else 0.0
    ndiff = _compare_decisions(fl, meas, orc.kxrcf_threshold(M))
    say(f"  flagged {fl[0].mean():.3f}  non-admissible faces {inf_g.mean():.3f}  jump err {err:.2e}  "
        f"near-threshold differences {ndiff}")
    assert err <= 1e-11
    if kind == "wave":
        assert 0.0 < fl[0].mean() < 0.9


@pytest.mark.parametrize("d,R,n,kind", CASES)
def test_two_pass_fp64_matches_oracle(K, oracle_mod, d, R, n, kind):
    """The FP64 right-hand side and limited states with the indicator on, against
    the oracle's two-pass scheme (section 5.3)."""
    say(f"case two-pass fp64 d={d} R={R} n={n} {kind}")
    U = _state(d, n, kind, 40 + d * 10 + R)
    dx = [1.0 / max(n)] * d
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    dev.set_indicator("kxrcf", M)
    dev.set_checking(True)
    Ud = U.cuda()
    got = dev.rhs(Ud).cpu().numpy()
    fl = dev.get_flags().cpu().numpy()
    st = dev.face_states(Ud).cpu().numpy()
    orc = oracle_mod.Oracle(d, R, n, dx=dx, kxrcf_m=M)
    f_o = orc.kxrcf(U.numpy(), M)[0]
    if not np.array_equal(f_o, fl):              # near-threshold cells: replay the GPU's choice
        _compare_decisions(fl, orc.kxrcf(U.numpy(), M)[1], orc.kxrcf_threshold(M))
        orc.set_kxrcf(None)
        orc.set_flags(fl)
    e_rhs = rel_err(got, orc.rhs(U.numpy()))
    e_st = rel_err(np.moveaxis(st, -1, 0), np.moveaxis(orc.states(U.numpy()), -1, 0))
    say(f"  flagged {fl[0].mean():.3f}  rhs rel err {e_rhs:.3e}  states rel err {e_st:.3e}")
    assert e_rhs <= 1e-12 and e_st <= 1e-12


@pytest.mark.parametrize("d,R,n,kind,mode,tol", [(2, 2, (37, 29), "jumps", "split_f16", 2e-5),
                                                  (2, 3, (40, 36), "wave", "split_f16", 2e-5),
                                                  (3, 2, (16, 16, 16), "wave", "split_f16", 2e-5),
                                                  (3, 2, (13, 11, 9), "jumps", "split_bf16", 2e-2),
                                                  (3, 3, (16, 12, 10), "wave", "split_f16", 2e-5)])
def test_two_pass_split_precision(K, oracle_mod, d, R, n, kind, mode, tol):
    """The indicator (FP64) driving the split-precision reconstruction; the oracle
    replays the decisions."""
    say(f"case two-pass {mode} d={d} R={R} n={n} {kind}")
    U = _state(d, n, kind, 40 + d * 10 + R)
    dx = [1.0 / max(n)] * d
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    dev.set_precision(mode)
    dev.set_indicator("kxrcf", M)
    dev.set_checking(True)
    got = dev.rhs(U.cuda()).cpu().numpy()
    fl = dev.get_flags().cpu().numpy()
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    _compare_decisions(fl, orc.kxrcf(U.numpy(), M)[1], orc.kxrcf_threshold(M))
    orc.set_flags(fl)
    e = rel_err(got, orc.rhs(U.numpy()))
    say(f"  flagged {fl[0].mean():.3f}  rhs rel err {e:.3e}")
    assert e <= tol


@pytest.mark.parametrize("name,mode,tol,nsample", [("3d_smooth_256", "fp64", 1e-12, 120),
                                                   ("3d_smooth_256", "split_f16", 2e-6, 120),
                                                   ("2d_jumps_1024", "fp64", 1e-12, 400),
                                                   ("3d_jumps_384_r3", "split_f16", 2e-5, 40)])
def test_two_pass_full_size_sampled(K, oracle_mod, name, mode, tol, nsample):
    """Full-size workloads in the benchmark's launch configuration: the indicator
    and the reconstruction over the whole grid; at sampled cells the oracle's
    measure against the GPU's decision, and the right-hand side against the
    oracle replaying the GPU's decisions; conservation over the grid."""
    say(f"case two-pass full-size {name} {mode}")
    U, cfg = inputs.config_state(name, device="cuda")
    d, n, R, gamma = cfg["d"], cfg["n"], cfg["R"], cfg["gamma"]
    dev = K.KFVM(d, (n,) * d, order=2 * R + 1, gamma=gamma)
    dev.set_precision(mode)
    dev.set_indicator("kxrcf", M)
    dev.set_checking(True)
    L = dev.rhs(U)
    torch.cuda.synchronize()
    fl = dev.get_flags().cpu().numpy()
    Lh = L.cpu().numpy().reshape(d + 2, -1)
    Uh = U.cpu().numpy()
    del U, L
    ncell = n ** d
    rng = np.random.default_rng(12)
    cells = np.concatenate([[0, ncell - 1, n - 1, ncell - n], rng.integers(0, ncell, nsample)])
    # bias part of the sample towards flagged cells
    flagged = np.flatnonzero(fl[0])
    if flagged.size:
        cells = np.concatenate([cells, rng.choice(flagged, min(nsample // 4, flagged.size), replace=False)])
    orc = oracle_mod.Oracle(d, R, (n,) * d, gamma=gamma)
    meas = orc.kxrcf_cells(Uh, cells)
    thr = orc.kxrcf_threshold(M)
    want = ~(meas < thr)
    diff = fl[0, cells].astype(bool) != want
    assert np.all(np.abs(meas[diff] / thr - 1.0) <= NEAR)
    orc.set_flags(fl)
    ref = orc.rhs_cells(Uh, cells)
    err = (np.abs(Lh[:, cells].T - ref) / np.abs(Lh).max(axis=1)).max()
    say(f"  flagged {fl[0].mean():.4f}  sampled rel err {err:.3e}")
    assert err <= tol
    tot = np.abs(Lh.sum(axis=1)) / np.abs(Lh).sum(axis=1)
    assert np.all(tot <= 1e-13)


def test_two_pass_trajectory_matches_oracle(K, oracle_mod):
    """10 SSP-RK3 steps with the indicator deciding at every stage (FP64 path)."""
    say("case two-pass trajectory")
    d, R, n = 2, 2, 48
    U0 = _wave_block(d, (n, n), 7)
    orc = oracle_mod.Oracle(d, R, (n, n), kxrcf_m=M)
    dev = K.KFVM(d, (n, n), order=5)
    dev.set_indicator("kxrcf", M)
    dev.set_checking(True)
    Uo, Ug = U0.numpy().copy(), U0.cuda()
    for _ in range(10):
        dt = orc.cfl_dt(Uo, 0.4)
        Uo = orc.step(Uo, dt)
        dev.step(Ug, dt)
    e = rel_err(Ug.cpu().numpy(), Uo)
    say(f"  10-step rel err {e:.3e}")
    assert e <= 1e-11


def test_indicator_settings_interplay(K):
    """Enabling the gate or caller flags turns the indicator off, and back."""
    from paper_2401_16543_amd import gate
    say("case indicator settings")
    d, n = 3, 16
    U = _wave_block(d, (n,) * d, 3).cuda()
    dev = K.KFVM(d, (n,) * d, order=5)
    dev.set_precision("split_f16")
    dev.set_indicator("kxrcf", M)
    a = dev.rhs(U).clone()
    fa = dev.get_flags().clone()
    params, thr, _ = gate.load(d)
    dev.set_gate(torch.from_numpy(params).cuda(), thr)
    dev.rhs(U)
    fg = dev.get_flags().clone()
    dev.set_flags(fa)                       # replaying the indicator's decisions gives its RHS
    assert torch.equal(dev.rhs(U), a)
    dev.set_indicator("kxrcf", M)
    assert torch.equal(dev.rhs(U), a)
    assert not torch.equal(fa, fg)
    with pytest.raises(K.KfvmError):
        dev.set_indicator("kxrcf", 0.0)


@pytest.mark.parametrize("case", ["3d_density_wave", "2d_vortex"])
def test_two_pass_accuracy_on_exact_solution(K, case):
    """What the two-pass procedure is for (section 5.3): WENO-AO only on the cells
    the indicator flags, at no loss of accuracy on smooth flow.  Density error
    against the exact cell averages, FP64 both ways, from the same state and dt."""
    say(f"case two-pass accuracy {case}")
    if case == "3d_density_wave":
        d, n, gamma, steps, vel = 3, 64, 5.0 / 3.0, 40, (0.5, 0.3, -0.2)
        spec = lambda t: inputs.density_wave(31, d, 6, vel, t)
        dx = 1.0 / n
    else:
        d, n, gamma, steps = 2, 64, 1.4, 80
        spec = lambda t: inputs.isentropic_vortex(gamma, t)
        dx = 20.0 / n
    U0 = inputs.cell_averages(spec(0.0), n, gamma, rule="gauss", q=4, device="cuda")
    plain = K.KFVM(d, (n,) * d, dx=[dx] * d, order=5, gamma=gamma)
    kx = K.KFVM(d, (n,) * d, dx=[dx] * d, order=5, gamma=gamma)
    kx.set_indicator("kxrcf", M)
    dt = plain.cfl_dt(U0, 0.4)
    Up, Uk = U0.clone(), U0.clone()
    flagged = 0.0
    for _ in range(steps):
        plain.step(Up, dt)
        kx.step(Uk, dt)
        flagged += float(kx.get_flags()[0].float().mean()) / steps
    Ue = inputs.cell_averages(spec(steps * dt), n, gamma, rule="gauss", q=4, device="cuda")
    ep = float((Up[0] - Ue[0]).abs().mean())
    ek = float((Uk[0] - Ue[0]).abs().mean())
    say(f"  t={steps * dt:.4f}: L1 rho error WENO-AO everywhere {ep:.3e}, two-pass {ek:.3e}, "
        f"cells flagged {flagged:.4f}")
    assert kx.status() == K.KFVM_OK and plain.status() == K.KFVM_OK
    assert ek <= 1.05 * ep
    assert flagged < 0.5


def test_stats_count_limited_cells_and_weno_pairs(K, oracle_mod):
    """kfvm_stats after a two-pass RHS: the WENO-AO pairs are the indicator's
    flags; the limited cells are those whose states the oracle's limiter changes."""
    say("case stats")
    d, R, n = 2, 3, (32, 32)
    U = inputs.cell_averages(inputs.discontinuous(9, d, 6, 100.0, 1000.0), 32, 1.4, rule="midpoint", q=4)
    dev = K.KFVM(d, n, order=7)
    assert dev.stats()["limiter_cells"] == 0                  # nothing reconstructed yet
    dev.set_limiter(True, 0.1)
    dev.set_indicator("kxrcf", M)
    dev.rhs(U.cuda())
    st = dev.stats()
    fl = dev.get_flags().cpu().numpy()
    assert st["weno_cell_vars"] == int(fl.astype(np.int64).sum())
    orc = oracle_mod.Oracle(d, R, n, kappa=0.1, kxrcf_m=M)
    free = oracle_mod.Oracle(d, R, n, limiter=False, kxrcf_m=M)
    changed = (np.abs(orc.states(U.numpy()) - free.states(U.numpy())) > 0).any(axis=(1, 2))
    say(f"  limited cells {st['limiter_cells']} (oracle {int(changed.sum())}), WENO pairs {st['weno_cell_vars']}")
    assert changed.sum() > 0
    assert abs(st["limiter_cells"] - int(changed.sum())) <= 2 + 0.01 * changed.sum()
    dev.set_indicator(None)
    dev.rhs(U.cuda())
    assert dev.stats()["weno_cell_vars"] == 4 * 32 * 32
