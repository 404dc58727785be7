"""Pins of the evaluation-loop oracle (Sec. 2 Eq. 1, Appendix A exchange and
demagnetizing rows, Sec. 7 RK4), none of which come from the oracle itself:

* one cubic cell in a static field: its demagnetizing field is -M/3, parallel
  to m, and it has no exchange, so RK4 must follow the closed-form precession
  (alpha = 0) and damped relaxation (alpha > 0) of a single moment;
* the Neumann Laplacian has the cosine modes cos(pi k (i + 1/2) / n) as exact
  eigenvectors with eigenvalues -(2 / h^2)(1 - cos(pi k / n));
* with damping the total energy decreases step by step; without it, a single
  moment keeps its angle to the field;
* the two-sublattice demagnetizing input is the field of the mean
  magnetization.
"""
import math

import numpy as np
import pytest

from oracle import conv, llg
from oracle.newell import tensor_full
from paper_2008_02478_amd import inputs


@pytest.mark.parametrize("alpha", [0.0, 0.02, 0.5])
def test_single_cell_follows_closed_form(alpha):
    h = (2e-9, 2e-9, 2e-9)
    H = 8e4
    th0, ph0 = 1.1, 0.3
    m = llg.single_spin(th0, ph0, H, 0.0, 0.0).reshape(3, 1, 1, 1)
    dt = 2e-14
    steps = 200
    Nf = tensor_full((1, 1, 1), h)
    for _ in range(steps):
        m = llg.rk4_step(m, dt, 8e5, 1.3e-11, alpha, (0.0, 0.0, H), h, Nfull=Nf)
    want = llg.single_spin(th0, ph0, H, alpha, steps * dt)
    assert np.max(np.abs(m.reshape(3) - want)) < 1e-9


def test_cubic_cell_demag_is_parallel():
    h = (3e-9, 3e-9, 3e-9)
    m = inputs.unit_sphere((1, 1, 1), seed=3).astype(np.float64)
    Hd = conv.fft_conv(7e5 * m, h)
    assert np.max(np.abs(Hd + 7e5 * m / 3.0)) < 1e-9 * 7e5


@pytest.mark.parametrize("n,h,k,ax", [((12, 5, 3), (2e-9, 3e-9, 1e-9), 3, 3),
                                      ((7, 9, 1), (5e-9, 4e-9, 3e-9), 4, 2),
                                      ((4, 3, 10), (1e-9, 1e-9, 2e-9), 7, 1)])
def test_neumann_laplacian_modes(n, h, k, ax):
    nax = n[3 - ax]
    hh = h[3 - ax]
    i = np.arange(nax) + 0.5
    mode = np.cos(math.pi * k * i / nax)
    shape = [1, 1, 1, 1]
    shape[ax] = nax
    m = np.broadcast_to(mode.reshape(shape), (3, n[2], n[1], n[0])).copy()
    lam = -2.0 / hh ** 2 * (1.0 - math.cos(math.pi * k / nax))
    assert np.max(np.abs(llg.laplacian_neumann(m, h) - lam * m)) < 1e-9 * abs(lam)


def test_damping_dissipates_energy():
    n, h = (16, 8, 1), (5e-9, 5e-9, 3e-9)
    Ms, A, Hext = 8e5, 1.3e-11, (2e4, -1e4, 3e4)
    m = inputs.unit_sphere(n, seed=81).astype(np.float64)
    Nf = tensor_full(n, h)
    E = [llg.total_energy(m, Ms, A, Hext, h, Nf)]
    for _ in range(5):
        m = llg.rk4_step(m, 5e-14, Ms, A, 0.3, Hext, h, Nfull=Nf)
        E.append(llg.total_energy(m, Ms, A, Hext, h, Nf))
    assert all(b < a for a, b in zip(E, E[1:]))


def test_two_sublattice_input_is_mean():
    n, h = (10, 6, 2), (2e-9, 2e-9, 1e-9)
    mA = inputs.unit_sphere(n, seed=82).astype(np.float64)
    mB = inputs.unit_sphere(n, seed=83).astype(np.float64)
    H2 = llg.two_sublattice_demag(mA, mB, 6e5, 9e5, h)
    # linearity: mean of the two sublattice fields
    Hm = 0.5 * (conv.fft_conv(6e5 * mA, h) + conv.fft_conv(9e5 * mB, h))
    assert np.max(np.abs(H2 - Hm)) < 1e-9 * np.max(np.abs(Hm))


def test_gamma_matches_electron_gyromagnetic_ratio():
    # CODATA electron gyromagnetic ratio |gamma_e| = 1.76085963e11 1/(s T)
    assert abs(llg.GAMMA - conv.MU0 * 1.76085963023e11) / llg.GAMMA < 1e-8


def test_periodic_laplacian_modes():
    # periodic axis: exp modes cos(2 pi k i / n) with eigenvalue -(2/h^2)(1 - cos(2 pi k / n))
    n, h, k = (10, 4, 1), (2e-9, 3e-9, 1e-9), 3
    i = np.arange(n[0])
    mode = np.cos(2 * math.pi * k * i / n[0])
    m = np.broadcast_to(mode.reshape(1, 1, 1, n[0]), (3, n[2], n[1], n[0])).copy()
    lam = -2.0 / h[0] ** 2 * (1.0 - math.cos(2 * math.pi * k / n[0]))
    assert np.max(np.abs(llg.laplacian_neumann(m, h, (True, False, False)) - lam * m)) < 1e-9 * abs(lam)
