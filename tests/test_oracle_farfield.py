"""Far-field pins of the oracle's kernels at the tensor accuracy contract.

Beyond a few cell sizes the oracle evaluates the demagnetizing tensor, the
inter-mesh tensor and the Oersted vector g by Gauss-Legendre quadrature of
their defining integrals, with fewer nodes the farther the offset (Table 1,
demagnetizing and Oersted rows; Sec. 3 Eq. 4 for unequal cells).  These tests
hold every distance band to 1e-10 relative per entry against an evaluation
that shares nothing with that quadrature: the closed forms (Newell's f and g
under the 27-point or the 4-point stencil; for g the second difference of
Q = int_0^X f ds) carried out in 50-digit arithmetic, where the stencils'
cancellation (about (r/h)^6 at distance r) costs no accuracy that matters.
The closed forms themselves are pinned near the source elsewhere (Aharoni's
prism, adaptive cubature of the definition, the fourth-derivative identity of
f and the path integral Q against adaptive quadrature).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import multilayer, newell, oersted

DPS = 50
TOL = 1e-10

# every cell shape of the benchmark configurations (nm)
CELLS = [(5.0, 5.0, 3.0), (4.0, 4.0, 4.0), (2.0, 2.0, 1.0), (5.0, 5.0, 2.0), (1.0, 1.0, 1.0), (2.0, 2.0, 2.0)]
# distances in units of the largest cell edge, one or more per quadrature band
# (4-6: 8 nodes, 6-16: 6, 16-40: 4, beyond: 3 per half-axis)
DISTANCES = [4.5, 9.0, 23.0, 60.0, 140.0]
# directions: generic, in-plane diagonal, along z
DIRECTIONS = [(0.62, 0.47, 0.63), (0.70710678, 0.70710678, 0.0), (0.0, 0.0, 1.0)]


def _mf(x, y, z):
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


def _mg(x, y, z):
    x2, y2, z2 = x * x, y * y, z * z
    R = mp.sqrt(x2 + y2 + z2)
    s = -x * y * R / 3
    if x2 + y2 > 0:
        s += x * y * z * mp.asinh(z / mp.sqrt(x2 + y2))
    if y2 + z2 > 0:
        s += y / 6 * (3 * z2 - y2) * mp.asinh(x / mp.sqrt(y2 + z2))
    if x2 + z2 > 0:
        s += x / 6 * (3 * z2 - x2) * mp.asinh(y / mp.sqrt(x2 + z2))
    if z != 0:
        s -= z * z2 / 6 * mp.atan(x * y / (z * R))
    if y != 0:
        s -= z * y2 / 2 * mp.atan(x * z / (y * R))
    if x != 0:
        s -= z * x2 / 2 * mp.atan(y * z / (x * R))
    return s


def _points(t, s):
    """Stencil points and weights along one axis for target size t and
    source size s: X +- (t+s)/2 with -1 and X +- (t-s)/2 with +1 (the
    27-point weights -1, 2, -1 when t == s)."""
    return [((t + s) / 2, -1), (-(t + s) / 2, -1), ((t - s) / 2, 1), (-(t - s) / 2, 1)]


def _mp_stencil(phi, X, Y, Z, ht, hs):
    acc = mp.mpf(0)
    for ox, wx in _points(ht[0], hs[0]):
        for oy, wy in _points(ht[1], hs[1]):
            for oz, wz in _points(ht[2], hs[2]):
                acc += wx * wy * wz * phi(X + ox, Y + oy, Z + oz)
    return acc / (4 * mp.pi * ht[0] * ht[1] * ht[2])


def mp_tensor(r, ht, hs=None):
    """Six components (xx yy zz xy xz yz) of the (inter-mesh) tensor at
    offset r from the closed forms in DPS-digit arithmetic."""
    hs = ht if hs is None else hs
    with mp.workdps(DPS):
        X, Y, Z = (mp.mpf(v) for v in r)
        t = [mp.mpf(v) for v in ht]
        s = [mp.mpf(v) for v in hs]
        perm = lambda a, b, c, v: (v[a], v[b], v[c])
        return np.array([float(v) for v in (
            _mp_stencil(_mf, X, Y, Z, t, s),
            _mp_stencil(_mf, Y, X, Z, perm(1, 0, 2, t), perm(1, 0, 2, s)),
            _mp_stencil(_mf, Z, Y, X, perm(2, 1, 0, t), perm(2, 1, 0, s)),
            _mp_stencil(_mg, X, Y, Z, t, s),
            _mp_stencil(_mg, X, Z, Y, perm(0, 2, 1, t), perm(0, 2, 1, s)),
            _mp_stencil(_mg, Y, Z, X, perm(1, 2, 0, t), perm(1, 2, 0, s)),
        )])


def _offsets(h):
    hmax = max(h)
    for d in DISTANCES:
        for u in DIRECTIONS:
            yield tuple(d * hmax * c for c in u)


def _check(got, want, what):
    scale = np.max(np.abs(want))
    err = np.abs(got - want)
    # per entry: relative to the entry, with a floor at 1e-13 of the largest
    # entry for components that vanish by symmetry (e.g. xy along z)
    bad = err > TOL * np.abs(want) + 1e-13 * scale
    assert not bad.any(), f"{what}: rel err {err / np.maximum(np.abs(want), 1e-300)} (want {want}, got {got})"


@pytest.mark.parametrize("h", CELLS)
def test_tensor_far_bands_match_50_digit_closed_form(h):
    for r in _offsets(h):
        want = mp_tensor(r, h)
        got = newell.tensor_at(*r, h)
        _check(got, want, f"N at {r} for cell {h}")


@pytest.mark.parametrize("ht,hs", [((1.0, 1.0, 1.0), (2.0, 2.0, 2.0)), ((2.0, 2.0, 2.0), (1.0, 1.0, 1.0)),
                                   ((1.0, 1.0, 1.0), (1.0, 1.0, 1.0)), ((2.0, 2.0, 1.0), (4.0, 4.0, 2.0))])
def test_unequal_tensor_far_bands_match_50_digit_closed_form(ht, hs):
    hmax = max(max(ht), max(hs))
    for d in DISTANCES:
        for u in DIRECTIONS[:2]:
            # offsets off the lattice (the coupled-layer case: half-cell and
            # layer-spacing shifts)
            r = (d * hmax * u[0] + 0.5, d * hmax * u[1] - 0.25, d * hmax * u[2] + 3.5)
            want = mp_tensor(r, ht, hs)
            got = multilayer.tensor_unequal(*r, ht, hs)
            _check(got, want, f"N({r}; {ht}, {hs})")


def _mq(X, Y, Z):
    """Q(X, Y, Z) = int_0^X f(s, Y, Z) ds by mpmath's Gauss-Legendre
    quadrature at working precision (degree raised until it converges).  At
    these offsets every stencil point has Y and Z away from 0, so f is
    analytic along the path."""
    if X == 0:
        return mp.mpf(0)
    return mp.quad(lambda s: _mf(s, Y, Z), [0, X], method="gauss-legendre")


def mp_g(r, h):
    """The Oersted vector g at offset r: -(1/V) times the 27-point second
    difference (weights 1, -2, 1) of Q, in DPS-digit arithmetic."""
    with mp.workdps(DPS):
        X, Y, Z = (mp.mpf(v) for v in r)
        a, b, c = (mp.mpf(v) for v in h)
        w = {-1: 1, 0: -2, 1: 1}

        def comp(P, Q_, R_, p, q, s):
            acc = mp.mpf(0)
            for i in (-1, 0, 1):
                for j in (-1, 0, 1):
                    for k in (-1, 0, 1):
                        acc += w[i] * w[j] * w[k] * _mq(P + i * p, Q_ + j * q, R_ + k * s)
            return -acc / (a * b * c)

        return np.array([float(comp(X, Y, Z, a, b, c)), float(comp(Y, X, Z, b, a, c)),
                         float(comp(Z, X, Y, c, a, b))])


@pytest.mark.parametrize("h", [(2.0, 2.0, 1.0), (5.0, 5.0, 3.0)])
def test_oersted_far_bands_match_50_digit_reduction(h):
    hmax = max(h)
    for d in DISTANCES:
        r = tuple(d * hmax * c for c in DIRECTIONS[0])
        want = mp_g(r, h)
        got = oersted.g_at(*r, h)
        _check(got, want, f"g at {r} for cell {h}")


def test_band_edges_are_the_documented_ones():
    # the pins above sample every band the oracle uses
    edges = [newell.NEAR_RADIUS] + [hi for hi, _ in newell.GL_BANDS[:-1]]
    for lo, hi in zip(edges, edges[1:] + [math.inf]):
        assert any(lo <= d < hi for d in DISTANCES)
    assert oersted.GL_BANDS is newell.GL_BANDS and multilayer.GL_BANDS == newell.GL_BANDS
