"""The seeded input generators against closed forms and invariants: the exact
cell average of one Fourier mode (a product of sinc factors over the axes),
the zero mean of integer-wavevector modes on the periodic box, the vortex's
period of 20 along (1, 1), positivity of the jump fields, and seeding."""
import math

import numpy as np
import pytest
import torch

from paper_2401_16543_amd import inputs


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_density_wave_cell_average_is_the_sinc_product(d, n):
    spec = inputs.density_wave(5, d, 1, [0.3] * d)
    k, a, phi = spec.modes[0]
    U = inputs.cell_averages(spec, n, 1.4, rule="gauss", q=8)
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X = np.stack(np.meshgrid(*([c] * d), indexing="ij")[::-1], -1)     # (x, y[, z]) in numpy layout
    sinc = np.prod([np.sinc(k[0, i] * h) for i in range(d)])           # np.sinc(t) = sin(pi t)/(pi t)
    exact = 1.0 + 0.2 * a[0] * np.sin(2 * np.pi * (X @ k[0]) + phi[0]) * sinc
    assert np.abs(U[0].numpy() - exact).max() < 1e-11
    # momentum: rho u with constant u; energy: p/(gamma-1) + rho |u|^2 / 2 with p = 1
    assert np.abs(U[1].numpy() - 0.3 * exact).max() < 1e-11
    ke = 0.5 * exact * 0.09 * d
    assert np.abs(U[d + 1].numpy() - (1.0 / 0.4 + ke)).max() < 1e-11


@pytest.mark.parametrize("d,n", [(2, 24), (3, 10)])
def test_smooth_density_has_unit_mean(d, n):
    U = inputs.cell_averages(inputs.smooth(3, d, 4), n, 1.4, rule="gauss", q=3)
    assert abs(float(U[0].mean()) - 1.0) < 1e-13


def test_vortex_returns_after_one_period():
    a = inputs.cell_averages(inputs.isentropic_vortex(1.4, 0.0), 32, 1.4, rule="gauss", q=4)
    b = inputs.cell_averages(inputs.isentropic_vortex(1.4, 20.0), 32, 1.4, rule="gauss", q=4)
    c = inputs.cell_averages(inputs.isentropic_vortex(1.4, 5.0), 32, 1.4, rule="gauss", q=4)
    assert torch.allclose(a, b, rtol=0, atol=1e-12)
    assert not torch.allclose(a, c, rtol=0, atol=1e-3)
    # far field: rho = 1, velocity (1, 1), p = 1/gamma
    corner = a[:, 0, 0].numpy()
    assert np.allclose(corner, [1.0, 1.0, 1.0, 1.0 / (1.4 * 0.4) + 1.0], atol=1e-6)


@pytest.mark.parametrize("d,n", [(2, 32), (3, 12)])
def test_jump_fields_are_positive_and_seeded(d, n):
    spec = inputs.discontinuous(11, d, 4, 10.0, 100.0)
    U = inputs.cell_averages(spec, n, 1.4, rule="midpoint", q=3)
    V = inputs.cell_averages(inputs.discontinuous(11, d, 4, 10.0, 100.0), n, 1.4, rule="midpoint", q=3)
    W = inputs.cell_averages(inputs.discontinuous(12, d, 4, 10.0, 100.0), n, 1.4, rule="midpoint", q=3)
    assert torch.equal(U, V) and not torch.equal(U, W)
    rho = U[0]
    kinetic = 0.5 * (U[1:d + 1] ** 2).sum(0) / rho
    assert float(rho.min()) > 0 and float((U[d + 1] - kinetic).min()) > 0
    assert float(rho.max() / rho.min()) > 5.0                        # the regions carry real jumps
