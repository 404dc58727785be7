"""Pins of the Oersted oracle (Table 1, row "Oersted"; Sec. 4) against facts
fixed by the mathematics rather than by the oracle itself:

  * the reduction's premise, d^2/dY^2 d^2/dZ^2 f = 1/R for Newell's f, and the
    path integral Q against 30-digit quadrature;
  * the gradient identity: moving the target cell by d changes g at the rate
    dg_a/dd_b = 4 pi N_ab(d), the demagnetizing tensor at the same continuous
    offset (itself pinned in test_oracle_newell.py);
  * the point-source limit g -> V d / |d|^3 with O((h/r)^2) error;
  * the refinement identity (a coarse cell is the union of fine cells);
  * g(0) = 0 and the parities;
  * the Biot-Savart field of a long straight wire (right-hand rule, I/(2 pi rho));
  * FFT convolution == direct sum, and self-adjointness of J -> H.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import newell, oersted as oe
from paper_2008_02478_amd import inputs


def _mp_f(x, y, z):
    x, y, z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = mp.sqrt(x2 + y2 + z2)
    s = (2 * x2 - y2 - z2) * R / 6
    if x2 + z2 > 0:
        s += y / 2 * (z2 - x2) * mp.asinh(y / mp.sqrt(x2 + z2))
    if x2 + y2 > 0:
        s += z / 2 * (y2 - x2) * mp.asinh(z / mp.sqrt(x2 + y2))
    if x != 0:
        s -= x * y * z * mp.atan(y * z / (x * R))
    return s


def test_newell_f_fourth_derivative_is_inverse_distance():
    mp.mp.dps = 40
    for p in [(0.7, 1.3, 0.4), (1.9, 0.3, 2.2), (0.2, 2.5, 1.1)]:
        d = mp.diff(lambda y, z: _mp_f(p[0], y, z), (p[1], p[2]), (2, 2))
        assert abs(d * mp.sqrt(sum(mp.mpf(v) ** 2 for v in p)) - 1) < mp.mpf(10) ** -30


@pytest.mark.parametrize("X,Y,Z", [(1.0, 0.0, 0.0), (2.5, 1.0, 0.0), (3.0, 0.0, 2.0), (-1.5, 2.0, 1.0),
                                   (4.0, 3.0, 2.0), (0.5, 0.0, 0.0)])
def test_q_integral_matches_30_digit_quadrature(X, Y, Z):
    mp.mp.dps = 30
    ref = mp.quad(lambda s: _mp_f(s, Y, Z), [0, X / 4, X / 2, X])
    got = oe.q_integral(X, Y, Z)
    assert abs(got - float(ref)) <= 1e-14 * max(1.0, abs(float(ref)))


H = (2e-9, 2e-9, 1e-9)


def _jacobian(d, h, dl):
    J = np.zeros((3, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = dl
        f = lambda s: oe.g_at(*(np.asarray(d) + s * e), h).ravel()
        J[:, b] = (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * dl)
    return J


@pytest.mark.parametrize("d", [(1.3e-9, 0.7e-9, 2.1e-9), (3.1e-9, 2.2e-9, 0.4e-9), (0.2e-9, 0.1e-9, 0.3e-9),
                               (9e-9, 4e-9, 3e-9), (-2.6e-9, 5.1e-9, -0.8e-9)])
def test_gradient_is_4pi_demag_tensor(d):
    Jg = _jacobian(d, H, 1e-11)
    N = newell.tensor_at(*d, H).ravel()
    Nm = 4 * math.pi * np.array([[N[0], N[3], N[4]], [N[3], N[1], N[5]], [N[4], N[5], N[2]]])
    assert np.max(np.abs(Jg - Nm)) <= 1e-7 * np.max(np.abs(Nm))


def test_point_source_limit_is_second_order():
    V = H[0] * H[1] * H[2]
    u = np.array([0.6, -0.48, 0.64])
    errs = []
    for r in (32, 128):
        d = r * max(H) * u
        g = oe.g_at(*d, H).ravel()
        pt = V * d / np.linalg.norm(d) ** 3
        errs.append(np.linalg.norm(g - pt) / np.linalg.norm(pt))
    assert errs[0] < 1e-3 and errs[1] < 1e-4
    assert 12.0 < errs[0] / errs[1] < 20.0          # (128/32)^2 = 16


@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 0, 1), (2, 1, 1), (4, 3, 2)])
def test_refinement_identity(D):
    hf = (1e-9, 1e-9, 0.5e-9)
    hc = tuple(2 * v for v in hf)
    gc = oe.g_at(*(np.array(D) * hc), hc).ravel()
    subs = [np.array(s) for s in np.ndindex(2, 2, 2)]
    acc = np.zeros(3)
    for a in subs:
        for b in subs:
            acc += oe.g_at(*(np.array(D) * hc + (a - b) * hf), hf).ravel()
    acc /= 8.0
    scale = max(np.max(np.abs(gc)), hc[0])          # g is O(h) next to the source
    assert np.max(np.abs(acc - gc)) <= 1e-11 * scale


def test_self_term_zero_and_parities():
    g0 = oe.g_at(0.0, 0.0, 0.0, H).ravel()
    assert np.max(np.abs(g0)) < 1e-14 * H[0]
    d = np.array([2.6e-9, 1.1e-9, 0.7e-9])
    g = oe.g_at(*d, H).ravel()
    for b in range(3):
        m = d.copy()
        m[b] = -m[b]
        gm = oe.g_at(*m, H).ravel()
        for a in range(3):
            assert gm[a] == pytest.approx(oe.PARITY[a][b] * g[a], rel=1e-13, abs=1e-25)


def test_long_wire_biot_savart():
    """A straight bar of one-cell cross-section and 2L+1 cells along z with
    current density J along z: at rho cells along x, mid-length, the field is
    I/(4 pi rho) * 2 cos(theta) along +y (I = J dx dy), the finite-filament
    Biot-Savart result, up to O((h/rho)^2) from the finite cross-section."""
    h = (1e-9, 1e-9, 1e-9)
    J, L, rho = 1e12, 400, 12
    k = np.arange(-L, L + 1)
    g = oe.g_at(rho * h[0], 0.0, k * h[2], h)          # target minus source offsets
    Jv = np.array([0.0, 0.0, J])
    Hs = np.cross(Jv[:, None], g, axis=0).sum(axis=1) / (4 * math.pi)
    I = J * h[0] * h[1]
    r = rho * h[0]
    half = (L + 0.5) * h[2]
    expect = I / (4 * math.pi * r) * 2 * half / math.hypot(half, r)
    assert abs(Hs[0]) < 1e-12 * expect and abs(Hs[2]) < 1e-12 * expect
    assert Hs[1] > 0
    assert abs(Hs[1] / expect - 1) < 2e-3


@pytest.mark.parametrize("n,h", [((5, 3, 2), (2e-9, 3e-9, 1e-9)), ((4, 4, 1), (5e-9, 5e-9, 3e-9)),
                                 ((3, 5, 3), (1e-9, 1e-9, 2e-9))])
def test_fft_matches_direct_sum(n, h):
    J = inputs.gaussian(n, seed=91)
    Hd = oe.field_direct(J, h)
    Hf = oe.field_fft(J, h)
    assert np.linalg.norm(Hf - Hd) <= 1e-12 * np.linalg.norm(Hd)


def test_self_adjoint():
    n, h = (6, 5, 3), (2e-9, 2e-9, 1e-9)
    J = inputs.gaussian(n, seed=92)
    G = inputs.gaussian(n, seed=93)
    a = float(np.sum(G * oe.field_fft(J, h)))
    b = float(np.sum(J * oe.field_fft(G, h)))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


@pytest.mark.parametrize("n,h,pbc,K", [
    ((5, 4, 2), (2e-9, 3e-9, 1e-9), (True, False, False), 2),
    ((4, 3, 2), (2e-9, 2e-9, 1e-9), (True, True, False), 1),
    ((4, 3, 2), (5e-9, 5e-9, 3e-9), (False, False, True), 2),
    ((3, 3, 2), (2e-9, 2e-9, 2e-9), (True, True, True), 1),
])
def test_periodic_images_equal_repeated_mesh(n, h, pbc, K):
    """Multiple images (Sec. 3): the image-summed kernel gives exactly the
    open-boundary field of the (2K+1)-times repeated mesh in its central copy."""
    J = inputs.gaussian(n, seed=94)
    Hp = oe.field_direct(J, h, oe.g_full(n, h, pbc, K))
    reps = [2 * K + 1 if p else 1 for p in pbc]
    big = tuple(n[a] * reps[a] for a in range(3))
    Hbig = oe.field_direct(np.tile(J, (1, reps[2], reps[1], reps[0])), h, oe.g_full(big, h))
    c = [K * n[a] if pbc[a] else 0 for a in range(3)]
    Hc = Hbig[:, c[2]:c[2] + n[2], c[1]:c[1] + n[1], c[0]:c[0] + n[0]]
    assert np.linalg.norm(Hp - Hc) <= 1e-12 * np.linalg.norm(Hc)
    assert np.linalg.norm(oe.field_fft(J, h, oe.g_full(n, h, pbc, K)) - Hp) <= 1e-12 * np.linalg.norm(Hp)


def test_periodic_film_tends_to_current_sheet():
    """A film of two layers periodic in x and y carrying a uniform current
    density J along x is an infinite slab: by Ampere's law H_y = -J z inside
    (z from the mid-plane), so the layers average -+J dz/2, and H_x = H_z = 0.
    The image sum approaches this as K grows."""
    n, h, J0 = (4, 4, 2), (2e-9, 2e-9, 1e-9), 1e11
    J = np.zeros((3, 2, 4, 4))
    J[0] = J0
    errs = []
    for K in (5, 20):
        H = oe.field_direct(J, h, oe.g_full(n, h, (True, True, False), K))
        expect = np.array([J0 * h[2] / 2, -J0 * h[2] / 2])[:, None, None]
        assert np.max(np.abs(H[0])) < 1e-9 * J0 * h[2]
        errs.append(max(np.max(np.abs(H[1] - expect)), np.max(np.abs(H[2]))) / (J0 * h[2] / 2))
    assert errs[0] < 0.1 and errs[1] < 0.03 and errs[1] < errs[0] / 3
