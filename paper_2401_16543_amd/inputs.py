"""Seeded synthetic initial states for the KFVM-WENO right-hand side.

This module holds no part of the method's arithmetic: it only draws random
fields and averages them over cells.  Both the GPU path and the CPU oracle are
fed from it; it imports neither.

Domain: the periodic unit box [0, 1)^d with n cells per axis.  Primitive fields
(rho, u_1..u_d, p) are evaluated at quadrature points and converted to the
conserved variables (rho, rho u, E = p/(gamma-1) + rho |u|^2 / 2) before
averaging, so cell averages are those of the conserved variables.

* smooth(seed, d, M): every primitive variable gets its own M Fourier modes with
  integer wavevectors k in [-4, 4]^d \\ {0}, amplitudes a ~ U(0,1) normalised to
  sum 1 and phases ~ U(0, 2 pi):
      rho = 1 + 0.2 S_rho,  u_i = 0.5 S_ui,  p = 1 + 0.2 S_p,
  with S = sum_m a_m sin(2 pi k_m . x + phi_m).
* discontinuous(seed, d, n_disc, r_rho_max, r_p_max): the smooth field with its
  velocity amplitude scaled by s ~ U(0, 1), then n_disc regions applied in turn,
  each a (periodic) ball with centre ~ U[0,1)^d and radius ~ U(0.05, 0.25) or a
  periodic slab with a small-integer normal and half-width ~ U(0.05, 0.15); inside
  a region rho is multiplied by r_rho and p by r_p, each log-uniform on
  [1, r_max] and inverted with probability 1/2.
* density_wave(seed, d, M, vel, t): rho = 1 + 0.2 S_rho(x - vel t) with constant
  velocity vel and p = 1, an exact solution of the Euler equations at every t
  (for accuracy checks against the exact cell averages).
* isentropic_vortex(gamma, t): the vortex of the paper's convergence study on
  [-10, 10]^2 (section 6.1), for validation runs.

Cell averages use a tensor Gauss-Legendre rule (smooth fields) or sub-cell
midpoints (fields with jumps), evaluated with torch in float64 on any device,
in slabs along the slowest axis to bound memory.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

_SLAB_POINTS = 1 << 22   # quadrature points evaluated per slab


@dataclass
class FieldSpec:
    d: int
    modes: list                     # per primitive variable: (k [M, d], a [M], phi [M])
    base: list
    amp: list
    regions: list = field(default_factory=list)   # (kind, params, r_rho, r_p)
    domain_lo: float = 0.0
    domain_hi: float = 1.0
    vortex: bool = False
    t: float = 0.0                  # vortex: advected by (1, 1) over time t


_SLAB_NORMALS_2D = [(1, 0), (0, 1), (1, 1), (1, -1), (1, 2), (2, 1)]
_SLAB_NORMALS_3D = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1),
                    (1, -1, 0), (1, 1, 1), (1, 2, 0), (2, 1, 1)]


def _draw_modes(rng, d, M):
    out = []
    for _ in range(d + 2):
        ks = []
        while len(ks) < M:
            k = rng.integers(-4, 5, size=d)
            if np.any(k != 0):
                ks.append(k)
        a = rng.uniform(0.0, 1.0, size=M)
        a = a / a.sum()
        phi = rng.uniform(0.0, 2 * np.pi, size=M)
        out.append((np.array(ks, dtype=np.float64), a, phi))
    return out


def smooth(seed: int, d: int, M: int) -> FieldSpec:
    rng = np.random.default_rng(seed)
    return FieldSpec(d=d, modes=_draw_modes(rng, d, M), base=[1.0] + [0.0] * d + [1.0],
                     amp=[0.2] + [0.5] * d + [0.2])


def discontinuous(seed: int, d: int, n_disc: int, r_rho_max: float, r_p_max: float,
                  M: int = 8) -> FieldSpec:
    rng = np.random.default_rng(seed)
    modes = _draw_modes(rng, d, M)
    s = rng.uniform(0.0, 1.0)
    spec = FieldSpec(d=d, modes=modes, base=[1.0] + [0.0] * d + [1.0],
                     amp=[0.2] + [0.5 * s] * d + [0.2])
    normals = _SLAB_NORMALS_2D if d == 2 else _SLAB_NORMALS_3D
    for _ in range(n_disc):
        r_rho = math.exp(rng.uniform(0.0, math.log(r_rho_max)))
        r_p = math.exp(rng.uniform(0.0, math.log(r_p_max)))
        if rng.uniform() < 0.5:
            r_rho = 1.0 / r_rho
        if rng.uniform() < 0.5:
            r_p = 1.0 / r_p
        if rng.uniform() < 0.5:
            centre = rng.uniform(0.0, 1.0, size=d)
            radius = rng.uniform(0.05, 0.25)
            spec.regions.append(("ball", (centre, radius), r_rho, r_p))
        else:
            nrm = np.array(normals[rng.integers(len(normals))], dtype=np.float64)
            offset = rng.uniform(0.0, 1.0)
            half = rng.uniform(0.05, 0.15)
            spec.regions.append(("slab", (nrm, offset, half), r_rho, r_p))
    return spec


def density_wave(seed: int, d: int, M: int, vel, t: float = 0.0) -> FieldSpec:
    rng = np.random.default_rng(seed)
    k, a, phi = _draw_modes(rng, d, M)[0]
    shift = 2.0 * np.pi * (k @ np.asarray(vel, dtype=np.float64)) * t     # sin(2 pi k.(x - vel t) + phi)
    zero = (np.zeros((1, d), dtype=np.int64), np.zeros(1), np.zeros(1))
    modes = [(k, a, phi - shift)] + [zero] * (d + 1)
    base = [1.0] + [float(v) for v in vel] + [1.0]
    amp = [0.2] + [0.0] * (d + 1)
    return FieldSpec(d=d, modes=modes, base=base, amp=amp)


def isentropic_vortex(gamma: float = 1.4, t: float = 0.0) -> FieldSpec:
    return FieldSpec(d=2, modes=[], base=[], amp=[], domain_lo=-10.0, domain_hi=10.0, vortex=True, t=t)


# ---------------------------------------------------------------------------
def _primitive(spec: FieldSpec, X: torch.Tensor, gamma: float):
    """Primitive variables [d + 2, P] at points X [P, d] (domain coordinates)."""
    d = spec.d
    if spec.vortex:
        # the vortex centre moves with the mean flow (1, 1); periodic image in [-10, 10)
        x = torch.remainder(X[:, 0] - spec.t + 10.0, 20.0) - 10.0
        y = torch.remainder(X[:, 1] - spec.t + 10.0, 20.0) - 10.0
        om = 5.0 * math.sqrt(2.0 * math.e) / (4.0 * math.pi) * torch.exp(-0.5 * (x * x + y * y))
        base = 1.0 + (1.0 - gamma) / 2.0 * om * om
        rho = base ** (1.0 / (gamma - 1.0))
        p = base ** (gamma / (gamma - 1.0)) / gamma
        return torch.stack([rho, 1.0 - y * om, 1.0 + x * om, p])
    out = []
    for j in range(d + 2):
        k, a, phi = (torch.as_tensor(t, dtype=torch.float64, device=X.device) for t in spec.modes[j])
        # elementwise products and sums (no BLAS: its gemv rejects very tall operands)
        arg = 2.0 * math.pi * (X[:, None, :] * k[None, :, :]).sum(-1) + phi   # [P, M]
        out.append(spec.base[j] + spec.amp[j] * (torch.sin(arg) * a).sum(-1))
    V = torch.stack(out)
    for kind, prm, r_rho, r_p in spec.regions:
        if kind == "ball":
            centre, radius = prm
            c = torch.as_tensor(centre, dtype=torch.float64, device=X.device)
            dd = X - c
            dd = dd - torch.round(dd)                    # periodic minimal image
            inside = (dd * dd).sum(1) < radius * radius
        else:
            nrm, offset, half = prm
            nv = torch.as_tensor(nrm, dtype=torch.float64, device=X.device)
            s = (X * nv).sum(-1) - offset
            s = s - torch.round(s)
            inside = s.abs() < half
        V[0] = torch.where(inside, V[0] * r_rho, V[0])
        V[d + 1] = torch.where(inside, V[d + 1] * r_p, V[d + 1])
    return V


def _conserved(V: torch.Tensor, d: int, gamma: float):
    rho, u, p = V[0], V[1:d + 1], V[d + 1]
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0)
    return torch.cat([rho[None], rho[None] * u, E[None]])


def _rule(kind: str, q: int):
    if kind == "gauss":
        x, w = np.polynomial.legendre.leggauss(q)
        return 0.5 * x, 0.5 * w                          # on [-1/2, 1/2], weights sum to 1
    x = (np.arange(q) + 0.5) / q - 0.5
    return x, np.full(q, 1.0 / q)


def cell_averages(spec: FieldSpec, n: int, gamma: float, *, rule: str = "gauss", q: int = 3,
                  device="cpu") -> torch.Tensor:
    """Conserved cell averages, float64 tensor [d + 2, (n,)*d] on `device`."""
    d = spec.d
    h = (spec.domain_hi - spec.domain_lo) / n
    xq, wq = _rule(rule, q)
    xq = torch.as_tensor(xq, dtype=torch.float64, device=device)
    wq = torch.as_tensor(wq, dtype=torch.float64, device=device)
    # tensor rule offsets [Q^d, d] and weights [Q^d]
    grids = torch.meshgrid(*([xq] * d), indexing="ij")
    off = torch.stack([g.reshape(-1) for g in grids], 1) * h
    wg = torch.meshgrid(*([wq] * d), indexing="ij")
    wts = torch.ones_like(wg[0]).reshape(-1)
    for g in wg:
        wts = wts * g.reshape(-1)
    out = torch.empty((d + 2,) + (n,) * d, dtype=torch.float64, device=device)
    idx = torch.arange(n, dtype=torch.float64, device=device)
    centres_1d = spec.domain_lo + (idx + 0.5) * h
    per_slab = max(1, _SLAB_POINTS // (off.shape[0] * n ** (d - 1)))
    for s0 in range(0, n, per_slab):
        s1 = min(n, s0 + per_slab)
        # numpy layout (z, y, x) for 3D, (y, x) for 2D; coordinates (x, y[, z])
        axes = [centres_1d[s0:s1]] + [centres_1d] * (d - 1)
        mesh = torch.meshgrid(*axes, indexing="ij")      # slowest axis first
        C = torch.stack([m.reshape(-1) for m in reversed(mesh)], 1)   # [cells, d] as (x, y[, z])
        X = (C[:, None, :] + off[None, :, :]).reshape(-1, d)
        U = _conserved(_primitive(spec, X, gamma), d, gamma)          # [nv, cells * Q^d]
        U = (U.reshape(d + 2, C.shape[0], -1) * wts).sum(-1)
        out[:, s0:s1] = U.reshape((d + 2, s1 - s0) + (n,) * (d - 1))
    return out


def config_state(name: str, device="cpu", n: int | None = None) -> tuple[torch.Tensor, dict]:
    """Initial state of a named workload, optionally at another resolution n."""
    cfg = WORKLOADS[name]
    nn = n or cfg["n"]
    spec = cfg["spec"]()
    rule, q = ("gauss", cfg["R"] + 1) if not spec.regions else ("midpoint", 4 if cfg["d"] == 2 else 2)
    U = cell_averages(spec, nn, cfg["gamma"], rule=rule, q=q, device=device)
    return U, dict(cfg, n=nn)


WORKLOADS = {
    "2d_smooth_64": dict(d=2, n=64, R=2, gamma=1.4, cfl=0.4, steps=10,
                         spec=lambda: smooth(1, 2, 8)),
    "2d_jumps_1024": dict(d=2, n=1024, R=2, gamma=1.4, cfl=0.4, steps=200,
                          spec=lambda: discontinuous(2, 2, 6, 10.0, 100.0)),
    "3d_smooth_256": dict(d=3, n=256, R=2, gamma=5.0 / 3.0, cfl=0.4, steps=50,
                          spec=lambda: smooth(3, 3, 16)),
    "2d_jumps_2048": dict(d=2, n=2048, R=2, gamma=1.4, cfl=0.4, steps=100,
                          spec=lambda: discontinuous(4, 2, 6, 10.0, 100.0)),
    "3d_jumps_384_r3": dict(d=3, n=384, R=3, gamma=1.4, cfl=0.4, steps=30,
                            spec=lambda: discontinuous(5, 3, 4, 10.0, 50.0, M=16)),
}


# ----------------------------------------------------------------- Sod tube ---
SOD_GAMMA = 1.4
SOD_LEFT = (1.0, 1.0)        # (rho, p), at rest
SOD_RIGHT = (0.125, 0.1)


def sod_parallel_coordinate(config: str, x, y):
    """The coordinate along which the Sod solution varies: x itself (aligned) or
    x_par = (2x + y) / sqrt 5 (tilted, tan theta = 1/2)."""
    return x if config == "aligned" else (2.0 * x + y) / math.sqrt(5.0)


def sod(config: str, R: int, device="cpu"):
    """Cell averages of the Sod shock tube on a periodic grid, by the tensor
    Gauss-Legendre rule with R points per axis (the rule of the paper's initial
    conditions).  Left state (rho, p) = (1, 1), right (0.125, 0.1), at rest,
    gamma = 1.4; the left state fills the coordinate s in [-1/2, 1/2] modulo 2.

    "aligned": [0, 2) x [0, 0.08), spacing 1/100 (200 x 8 cells): the grid-aligned
    tube on [0, 1] and its mirror image on [1, 2), which stand in for the
    outflow boundaries until the waves of the two interfaces meet (after
    t = 0.2); s = x.  "tilted": [0, sqrt 5) x [0, 2 sqrt 5), spacing sqrt(5)/250
    (250 x 500 cells), s = (2x + y) / sqrt 5.

    Returns (U [4, ny, nx] float64 tensor, dict(n=(nx, ny), dx))."""
    if config == "aligned":
        nx, ny, h = 200, 8, 0.01
    elif config == "tilted":
        nx, ny, h = 250, 500, math.sqrt(5.0) / 250
    else:
        raise ValueError(config)
    g, w = np.polynomial.legendre.leggauss(R)
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    rho = np.zeros((ny, nx))
    p = np.zeros((ny, nx))
    for gy, wy in zip(g, w):
        for gx, wx in zip(g, w):
            s = sod_parallel_coordinate(config, X + 0.5 * gx * h, Y + 0.5 * gy * h)
            left = np.abs(np.mod(s + 0.5, 2.0) - 0.5) <= 0.5
            ww = 0.25 * wx * wy
            rho += ww * np.where(left, SOD_LEFT[0], SOD_RIGHT[0])
            p += ww * np.where(left, SOD_LEFT[1], SOD_RIGHT[1])
    U = np.stack([rho, np.zeros_like(rho), np.zeros_like(rho), p / (SOD_GAMMA - 1.0)])
    return torch.from_numpy(U).to(device), {"n": (nx, ny), "dx": h}


# ----------------------------------------------- Richtmyer-Meshkov instability ---
RMI_MA, RMI_RHO_D, RMI_GAMMA = 3.0, 2.0, 1.4
RMI_X0, RMI_X1 = -0.5, 5.5          # domain [-1/2, 11/2] x [0, 1]


def rmi_primitive(x, y, gamma=RMI_GAMMA, ma=RMI_MA, rho_d=RMI_RHO_D):
    """(rho, u, v, p) of the Richtmyer-Meshkov initial state (section 6.3): the
    post-shock state of a Mach-ma shock for x < 0.2, then density 1 for x < y and
    rho_d for x >= y at rest with p = 1."""
    post = x < 0.2
    rho_s = 1.0 / (1.0 - 2.0 / (gamma + 1.0) * (1.0 - 1.0 / ma ** 2))
    rho = np.where(post, rho_s, np.where(x < y, 1.0, rho_d))
    p = np.where(post, 1.0 + 2.0 * gamma / (gamma + 1.0) * (ma ** 2 - 1.0), 1.0)
    u = np.where(post, ma * math.sqrt(gamma) * (1.0 - 1.0 / rho_s), 0.0)
    return rho, u, np.zeros_like(rho), p


def rmi_inflow_state(gamma=RMI_GAMMA):
    """Conserved post-shock state fixed at the inflow boundary x = -1/2."""
    rho, u, v, p = (float(a) for a in rmi_primitive(np.array(-0.5), np.array(0.5), gamma))
    return np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def rmi(R: int, cells_per_unit: int = 512, device="cpu"):
    """Cell averages of the Richtmyer-Meshkov problem on [-1/2, 11/2] x [0, 1] with
    spacing 1 / cells_per_unit (the paper's 1/512: 3072 x 512 cells), by the
    tensor Gauss rule with R points per axis.  Boundaries: fixed inflow at
    x = -1/2, extrapolation (outflow) at x = 11/2, reflecting in y.
    Returns (U [4, ny, nx] float64 tensor, dict(n, dx, inflow))."""
    h = 1.0 / cells_per_unit
    nx, ny = int(round((RMI_X1 - RMI_X0) * cells_per_unit)), cells_per_unit
    g, w = np.polynomial.legendre.leggauss(R)
    xc = RMI_X0 + (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    acc = np.zeros((4, ny, nx))
    for gy, wy in zip(g, w):
        for gx, wx in zip(g, w):
            rho, u, v, p = rmi_primitive(X + 0.5 * gx * h, Y + 0.5 * gy * h)
            ww = 0.25 * wx * wy
            acc += ww * np.stack([rho, rho * u, rho * v, p / (RMI_GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])
    return torch.from_numpy(acc).to(device), {"n": (nx, ny), "dx": h, "inflow": rmi_inflow_state()}
