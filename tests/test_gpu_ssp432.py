"""SSP(4,3,2) steps on the GPU (through the C-ABI) against the oracle, and the
error-controlled integration driver on the isentropic vortex."""
import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("d,R,n,kind,mode,tol", [(2, 2, (37, 29), "jumps", "fp64", 1e-12),
                                                  (3, 2, (16, 16, 16), "smooth", "fp64", 1e-12),
                                                  (2, 3, (40, 36), "jumps", "fp64", 1e-12),
                                                  (3, 2, (16, 16, 16), "smooth", "split_f16", 2e-6)])
def test_step_ssp432_matches_oracle(K, oracle_mod, d, R, n, kind, mode, tol):
    say(f"case ssp432 d={d} R={R} n={n} {kind} {mode}")
    if kind == "jumps":
        U = inputs.cell_averages(inputs.discontinuous(12, d, 6, 10.0, 100.0), max(n), 1.4, rule="midpoint", q=4)
    else:
        U = inputs.cell_averages(inputs.smooth(12, d, 4), max(n), 1.4, rule="gauss", q=3)
    U = U[(slice(None),) + tuple(slice(0, x) for x in reversed(n))].contiguous()
    dx = [1.0 / max(n)] * d
    orc = oracle_mod.Oracle(d, R, n, dx=dx)
    dt = 0.8 * orc.cfl_dt(U.numpy(), 1.0)
    ref, e_ref = orc.step_ssp432(U.numpy(), dt, atol=1e-6, rtol=1e-6)
    dev = K.KFVM(d, n, dx=dx, order=2 * R + 1)
    dev.set_precision(mode)
    Ud = U.cuda()
    out = torch.empty_like(Ud)
    e = dev.step_ssp432(Ud, out, dt, 1e-6, 1e-6)
    err_state = rel_err(out.cpu().numpy(), ref)
    say(f"  state rel err {err_state:.3e}  error norm {e:.6e} (oracle {e_ref:.6e})")
    assert err_state <= tol
    assert torch.equal(Ud, U.cuda())                          # the input is kept
    if mode == "fp64":
        assert abs(e - e_ref) <= 1e-8 * e_ref
    with pytest.raises(K.KfvmError):
        dev.step_ssp432(Ud, Ud, dt)


def test_error_controlled_vortex(K):
    """The isentropic vortex (section 6.1, 64^2, R = 2) to t = 2 with atol = rtol =
    1e-6: the controller keeps the temporal error below the spatial one, so the
    density error against the exact solution matches SSP-RK3 at a small CFL."""
    from paper_2401_16543_amd import integrate
    say("case ssp432 vortex")
    n, gamma, T = 64, 1.4, 2.0
    spec = lambda t: inputs.isentropic_vortex(gamma, t)
    U0 = inputs.cell_averages(spec(0.0), n, gamma, rule="gauss", q=4, device="cuda")
    dx = [20.0 / n] * 2
    dev = K.KFVM(2, (n, n), dx=dx, order=5, gamma=gamma)
    U = U0.clone()
    st = integrate.integrate(dev, U, T, atol=1e-6, rtol=1e-6, cfl_max=1.0)
    Ue = inputs.cell_averages(spec(T), n, gamma, rule="gauss", q=4, device="cuda")
    e_ssp = float((U[0] - Ue[0]).abs().mean())
    V = U0.clone()
    t = 0.0
    while t < T - 1e-14:
        dt = min(dev.cfl_dt(V, 0.2), T - t)
        dev.step(V, dt)
        t += dt
    e_rk3 = float((V[0] - Ue[0]).abs().mean())
    say(f"  {st}: L1 rho error {e_ssp:.3e} (SSP-RK3 at CFL 0.2: {e_rk3:.3e})")
    assert abs(st["t"] - T) <= 1e-12
    assert st["accepted"] > 0 and st["rejected"] <= st["accepted"]
    assert e_ssp <= 1.05 * e_rk3


@pytest.mark.parametrize("integrator", ["ssp3", "ssp432"])
def test_richtmyer_meshkov_driver_short_run(K, oracle_mod, integrator):
    """The Richtmyer-Meshkov driver on a coarse grid (1/32 spacing, 192 x 32
    cells): a few steps of either integrator match the oracle taking the same
    step sizes (WENO-AO everywhere: a trajectory cannot replay the indicator's
    decisions, and one taken at its threshold would differ; the two-pass
    reconstruction of this setup is checked cell by cell in test_gpu_boundary)."""
    from paper_2401_16543_amd import rmi
    say(f"case rmi driver {integrator}")
    out = rmi.run(R=2, cells_per_unit=32, t_end=1.0, cfl=0.5 if integrator == "ssp3" else 1.0, indicator=False,
                  max_steps=4, keep_state=True, integrator=integrator, tol=1e-3)
    assert out["status"] == 0 and out["steps"] == 4
    assert len(out["dts"]) == (4 if integrator == "ssp3" else out["accepted"]) > 0
    U0, m = inputs.rmi(2, 32)
    nx, ny = m["n"]
    orc = oracle_mod.Oracle(2, 2, (nx, ny), dx=[m["dx"]] * 2, gamma=inputs.RMI_GAMMA)
    orc.set_boundary(0, "inflow", "outflow", lower_state=m["inflow"])
    orc.set_boundary(1, "reflecting", "reflecting")
    U = U0.numpy().copy()
    if integrator == "ssp3":
        for dt in out["dts"]:
            U = orc.step(U, dt)
    else:                        # a rejected attempt leaves U as it was
        for dt in out["dts"]:
            U, _ = orc.step_ssp432(U, dt, 1e-3, 1e-3)
    e = rel_err(out["U"].cpu().numpy(), U)
    say(f"  {out['steps']} steps, t = {out['t']:.4f}, rel err vs oracle {e:.2e}")
    assert e <= 1e-10
