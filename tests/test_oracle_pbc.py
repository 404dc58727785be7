"""Pins of the periodic-boundary oracle (Sec. 3, multiple images), none of
which come from the oracle itself:

* the image-summed field equals the open-boundary field of the (2K+1)-times
  repeated mesh read in its central copy (exact: the direct sum over the
  repeated mesh uses only the open-boundary tensor);
* the zero-padded FFT route and the direct sum agree with the image-summed
  tensor;
* a film periodic in x and y, magnetized uniformly, tends to the infinite-film
  limit: H = -M for M normal to the film, H = 0 in plane (demagnetizing
  factors 1 and 0);
* the image sum converges as K grows (1D periodicity).
"""
import numpy as np
import pytest

from oracle import conv
from oracle.newell import tensor_full
from oracle.pbc import tensor_full_pbc, tensor_octant_pbc
from paper_2008_02478_amd import inputs


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("n,h,pbc,K", [
    ((5, 4, 2), (2e-9, 3e-9, 1e-9), (True, False, False), 2),
    ((5, 4, 2), (2e-9, 3e-9, 1e-9), (False, True, False), 2),
    ((4, 3, 2), (2e-9, 2e-9, 1e-9), (True, True, False), 1),
    ((4, 3, 2), (5e-9, 5e-9, 3e-9), (False, False, True), 2),
    ((3, 3, 2), (2e-9, 2e-9, 2e-9), (True, True, True), 1),
])
def test_images_equal_repeated_mesh(n, h, pbc, K):
    M = 8e5 * inputs.unit_sphere(n, seed=41).astype(np.float64)
    Hp = conv.direct_sum(M, h, tensor_full_pbc(n, h, pbc, K))
    reps = [2 * K + 1 if p else 1 for p in pbc]
    big = tuple(n[a] * reps[a] for a in range(3))
    Mbig = np.tile(M, (1, reps[2], reps[1], reps[0]))
    Hbig = conv.direct_sum(Mbig, h, tensor_full(big, h))
    c = [K * n[a] if pbc[a] else 0 for a in range(3)]
    Hc = Hbig[:, c[2]:c[2] + n[2], c[1]:c[1] + n[1], c[0]:c[0] + n[0]]
    assert _rel(Hp, Hc) < 1e-12


@pytest.mark.parametrize("pbc", [(True, False, False), (True, True, False), (False, True, True)])
def test_fft_route_equals_direct_sum(pbc):
    n, h = (6, 5, 3), (2e-9, 2.5e-9, 1e-9)
    M = 1e6 * inputs.unit_sphere(n, seed=42).astype(np.float64)
    Nf = tensor_full_pbc(n, h, pbc, 3)
    assert _rel(conv.fft_conv(M, h, Nf), conv.direct_sum(M, h, Nf)) < 1e-12


def test_film_tends_to_infinite_film():
    # one layer of 4x4 cells (8x8x1 nm), periodic in x and y
    n, h = (4, 4, 1), (2e-9, 2e-9, 1e-9)
    Ms = 1e6
    errs = []
    for K in (5, 40):
        Nf = tensor_full_pbc(n, h, (True, True, False), K)
        for axis, want in ((2, -1.0), (0, 0.0)):
            M = np.zeros((3,) + n[::-1])
            M[axis] = Ms
            H = conv.direct_sum(M, h, Nf)
            errs.append((K, axis, float(np.max(np.abs(H[axis] / Ms - want)))))
    e = {(K, a): v for K, a, v in errs}
    assert e[(40, 2)] < 0.01 and e[(40, 0)] < 0.01
    assert e[(40, 2)] < e[(5, 2)] and e[(40, 0)] < e[(5, 0)]


def test_image_sum_converges():
    n, h = (6, 4, 2), (2e-9, 2e-9, 1e-9)
    pbc = (True, False, False)
    d = []
    prev = tensor_octant_pbc(n, h, pbc, 4)
    for K in (8, 16):
        cur = tensor_octant_pbc(n, h, pbc, K)
        d.append(_rel(cur, prev))
        prev = cur
    assert d[1] < d[0] < 1e-3


def test_no_images_is_open_boundary():
    n, h = (5, 3, 2), (2e-9, 2e-9, 1e-9)
    assert _rel(tensor_full_pbc(n, h, (True, True, True), 0), tensor_full(n, h)) < 1e-15
