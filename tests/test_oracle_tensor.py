"""Pins of the oracle's demagnetizing tensor against facts that do not come
from the oracle itself (Sec. 3 Eq. 4 and Table 1 define N as the
cell-averaged Newell tensor; the paper prints no values of it)."""
import math

import numpy as np
import pytest

from oracle import newell
from oracle.newell import COMPONENTS, tensor_at, tensor_full, tensor_octant


def aharoni_Dz(A, B, C):
    """Demagnetizing factor along z of a uniformly magnetized rectangular
    prism of edges A x B x C (Aharoni, J. Appl. Phys. 83, 3432 (1998)); a
    closed form derived independently of Newell's f/g functions."""
    a, b, c = A / 2.0, B / 2.0, C / 2.0
    r = math.sqrt(a * a + b * b + c * c)
    ab, bc, ac = math.sqrt(a * a + b * b), math.sqrt(b * b + c * c), math.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c)) * math.log((r - a) / (r + a)) \
        + ((a * a - c * c) / (2 * a * c)) * math.log((r - b) / (r + b)) \
        + b / (2 * c) * math.log((ab + a) / (ab - a)) + a / (2 * c) * math.log((ab + b) / (ab - b)) \
        + c / (2 * a) * math.log((bc - b) / (bc + b)) + c / (2 * b) * math.log((ac - a) / (ac + a)) \
        + 2 * math.atan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c) \
        + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + c / (a * b) * (ac + bc) \
        - ((a * a + b * b) ** 1.5 + (b * b + c * c) ** 1.5 + (c * c + a * a) ** 1.5) / (3 * a * b * c)
    return s / math.pi


def aharoni_diag(A, B, C):
    """(Nxx, Nyy, Nzz) of an A x B x C prism by permuting the z formula."""
    return (aharoni_Dz(B, C, A), aharoni_Dz(C, A, B), aharoni_Dz(A, B, C))


CELLS = [(5e-9, 5e-9, 3e-9), (4e-9, 4e-9, 4e-9), (2e-9, 2e-9, 1e-9),
         (5e-9, 5e-9, 2e-9), (1e-9, 1.3e-9, 0.7e-9), (3e-9, 1e-9, 2e-9)]


@pytest.mark.parametrize("h", CELLS)
def test_self_term_matches_aharoni_prism(h):
    N0 = tensor_at(0.0, 0.0, 0.0, h)
    for got, want in zip(N0[:3], aharoni_diag(*h)):
        assert abs(got - want) < 1e-13
    assert np.all(np.abs(N0[3:]) < 1e-15)
    assert abs(N0[0] + N0[1] + N0[2] - 1.0) < 1e-14


def test_cube_self_term_is_one_third():
    N0 = tensor_at(0.0, 0.0, 0.0, (1.0, 1.0, 1.0))
    assert np.allclose(N0[:3], 1.0 / 3.0, atol=1e-15, rtol=0)


def test_thin_film_limit():
    # a wide flat cell approaches the infinite film: Nzz -> 1, Nxx, Nyy -> 0
    prev = 0.0
    for ratio in (10.0, 100.0, 1000.0, 1e4):
        N0 = tensor_at(0.0, 0.0, 0.0, (ratio, ratio, 1.0))
        assert N0[2] > prev
        prev = N0[2]
        assert abs(N0[2] - aharoni_Dz(ratio, ratio, 1.0)) < 1e-11
    assert prev > 0.999


@pytest.mark.parametrize("h", CELLS)
def test_trace_vanishes_off_the_self_term(h):
    # N is the Hessian of a harmonic potential away from the source cell
    rng = np.random.default_rng(0)
    off = rng.integers(-40, 41, size=(200, 3)).astype(float)
    off = off[np.any(off != 0, axis=1)]
    N = tensor_at(off[:, 0] * h[0], off[:, 1] * h[1], off[:, 2] * h[2], h)
    scale = np.max(np.abs(N), axis=0)
    assert np.all(np.abs(N[0] + N[1] + N[2]) <= 1e-10 * scale)


@pytest.mark.parametrize("h", CELLS)
def test_quadrature_and_closed_form_agree_in_overlap_band(h):
    # two independent evaluations of the same definition: Newell's closed form
    # and Gauss-Legendre quadrature of the dipole kernel over the tent weight
    hm = max(h)
    rng = np.random.default_rng(1)
    dirs = rng.standard_normal((60, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for rad in (3.5, 5.0, 8.0):
        pts = np.round(dirs * rad * hm / np.array(h)) * np.array(h)
        cf = newell.newell_near(pts[:, 0], pts[:, 1], pts[:, 2], h)
        gl = newell.gl_far(pts[:, 0], pts[:, 1], pts[:, 2], h, 10)
        scale = np.max(np.abs(cf), axis=0)
        # the closed form loses about eps (r/h_min)^6 to cancellation
        tol = {3.5: 1e-10, 5.0: 1e-9, 8.0: 1e-8}[rad]
        assert np.all(np.abs(cf - gl) <= tol * scale)


def test_adaptive_integration_of_definition():
    # scipy's adaptive cubature of the defining integral, independent of both
    # the closed form and the Gauss-Legendre rule
    from scipy.integrate import nquad
    h = (1.0, 1.3, 0.7)
    V = h[0] * h[1] * h[2]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for off in [(2.0, 1.3, 0.0), (1.0, 2.6, 1.4), (0.0, 0.0, 1.4)]:
        want = tensor_at(*off, h)
        for c, (a, b) in enumerate(pairs):
            def integrand(ux, uy, uz):
                v = (off[0] + ux, off[1] + uy, off[2] + uz)
                r2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
                w = (h[0] - abs(ux)) * (h[1] - abs(uy)) * (h[2] - abs(uz))
                return w * ((r2 if a == b else 0.0) - 3.0 * v[a] * v[b]) / r2 ** 2.5
            if off == (0.0, 0.0, 1.4):
                continue   # face neighbour: integrand singular at a corner; covered by refinement
            val, _ = nquad(integrand, [(-h[0], h[0]), (-h[1], h[1]), (-h[2], h[2])],
                           opts=[{"points": [0.0], "epsabs": 1e-13, "epsrel": 1e-11}] * 3)
            val /= 4.0 * math.pi * V
            assert abs(val - want[c]) < 1e-9 * max(1e-3, abs(want[c]))


@pytest.mark.parametrize("blk,h", [((2, 2, 2), (1.0, 1.0, 1.0)),
                                   ((4, 4, 4), (1.0, 1.0, 1.0)),
                                   ((3, 2, 1), (2.0, 2.0, 1.0)),
                                   ((6, 3, 2), (1.0, 1.5, 0.5)),
                                   ((12, 12, 1), (5.0, 5.0, 3.0))])
def test_refinement_identity(blk, h):
    # a big cell made of p*q*s fine cells: its self term is the mean over all
    # ordered fine-cell pairs of the fine tensor (exact), and Aharoni's formula
    # gives the big cell's self term independently
    p, q, s = blk
    Nfull = tensor_full((p, q, s), h)
    # number of ordered pairs with each offset = prod_a (n_a - |o_a|)
    wz = s - np.abs(np.arange(-(s - 1), s))
    wy = q - np.abs(np.arange(-(q - 1), q))
    wx = p - np.abs(np.arange(-(p - 1), p))
    w = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    mean = np.array([np.sum(w * Nfull[c]) for c in range(6)]) / (p * q * s)
    want = aharoni_diag(p * h[0], q * h[1], s * h[2])
    assert np.allclose(mean[:3], want, atol=2e-13, rtol=0)
    assert np.all(np.abs(mean[3:]) < 1e-13)


def test_parity_reflection_matches_direct_evaluation():
    # the closed form and the quadrature hold for any sign of the offset, so
    # evaluating directly at negative offsets checks the reflection signs
    h = (1.0, 1.3, 0.7)
    n = (9, 7, 5)
    full = tensor_full(n, h)
    oz, oy, ox = np.meshgrid(np.arange(-4, 5), np.arange(-6, 7), np.arange(-8, 9), indexing="ij")
    direct = tensor_at(ox * h[0], oy * h[1], oz * h[2], h)
    sub = full[:, 0:9, 0:13, 0:17]
    assert np.allclose(sub, direct, atol=1e-15, rtol=1e-12)


def test_dipole_limit():
    # far away the cell looks like a point dipole: N -> V/(4 pi) (I r^2 - 3 r r^T)/r^5
    h = (2.0, 2.0, 1.0)
    V = 4.0
    for r in [(200.0, 0.0, 0.0), (0.0, 0.0, 300.0), (150.0, 120.0, 60.0)]:
        N = tensor_at(*r, h)
        v = np.array(r)
        d = np.linalg.norm(v)
        D = V / (4 * math.pi) * (np.eye(3) * d * d - 3 * np.outer(v, v)) / d ** 5
        want = np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])
        rel = np.max(np.abs(N - want)) / np.max(np.abs(want))
        assert rel < 2 * (max(h) / d) ** 2     # O((h/r)^2) correction


def test_octant_layout():
    h = (5e-9, 5e-9, 3e-9)
    octn = tensor_octant((4, 3, 2), h)
    assert octn.shape == (6, 2, 3, 4)
    direct = tensor_at(3 * h[0], 2 * h[1], 1 * h[2], h)
    assert np.allclose(octn[:, 1, 2, 3], direct, rtol=0, atol=0)
