"""Pins of the oracle's field, energy and gradients (Table 1 demagnetizing
field, Sec. 3 Eq. 4, Sec. 7 convolution theorem with zero padding, the
field/energy relation of Appendix A)."""
import math

import numpy as np
import pytest

from oracle import conv
from oracle.newell import tensor_at, tensor_full
from paper_2008_02478_amd import inputs
from tests.test_oracle_tensor import aharoni_diag


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_padded_length():
    assert [conv.padded_len(n) for n in (1, 2, 3, 4, 5, 64, 65, 512, 1024)] == \
        [1, 4, 8, 8, 16, 128, 256, 1024, 2048]


def test_single_cell_field_is_self_term():
    h = (5e-9, 5e-9, 3e-9)
    M = np.array([1.0, -2.0, 0.5]).reshape(3, 1, 1, 1) * 8e5
    N0 = tensor_at(0.0, 0.0, 0.0, h)
    H = conv.fft_conv(M, h)
    assert np.allclose(H[:, 0, 0, 0], -N0[:3] * M[:, 0, 0, 0], rtol=1e-14, atol=0)


def test_two_cells_by_hand():
    h = (2e-9, 3e-9, 1e-9)
    rng = np.random.default_rng(3)
    M = rng.standard_normal((3, 1, 1, 2))
    N0 = tensor_at(0.0, 0.0, 0.0, h)
    N1 = tensor_at(h[0], 0.0, 0.0, h)      # target 0 sees source 1 at offset -dx
    def mat(N, sx):
        xx, yy, zz, xy, xz, yz = N
        return np.array([[xx, sx * xy, sx * xz], [sx * xy, yy, yz], [sx * xz, yz, zz]])
    want0 = -(mat(N0, 1) @ M[:, 0, 0, 0] + mat(N1, -1) @ M[:, 0, 0, 1])
    want1 = -(mat(N0, 1) @ M[:, 0, 0, 1] + mat(N1, 1) @ M[:, 0, 0, 0])
    for route in (conv.direct_sum, conv.fft_conv):
        H = route(M, h)
        assert np.allclose(H[:, 0, 0, 0], want0, rtol=1e-13, atol=0)
        assert np.allclose(H[:, 0, 0, 1], want1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,h", [((5, 3, 2), (1e-9, 1.3e-9, 0.7e-9)),
                                 ((7, 6, 1), (5e-9, 5e-9, 3e-9)),
                                 ((1, 9, 3), (2e-9, 2e-9, 1e-9)),
                                 ((16, 16, 1), (5e-9, 5e-9, 3e-9)),
                                 ((12, 5, 4), (4e-9, 4e-9, 4e-9)),
                                 ((3, 3, 3), (3e-9, 1e-9, 2e-9))])
def test_fft_convolution_equals_direct_sum(n, h):
    # two routes to one result: zero-padded FFT convolution is exact
    M = inputs.unit_sphere(n, seed=11).astype(np.float64) * 8e5
    Nfull = tensor_full(n, h)
    Hd = conv.direct_sum(M, h, Nfull)
    Hf = conv.fft_conv(M, h, Nfull)
    assert rel_l2(Hf, Hd) < 1e-12


def test_fft_convolution_equals_direct_sum_64x64():
    n, h = (64, 64, 1), (5e-9, 5e-9, 3e-9)
    M = inputs.unit_sphere(n, seed=1).astype(np.float64) * 8e5
    Nfull = tensor_full(n, h)
    assert rel_l2(conv.fft_conv(M, h, Nfull), conv.direct_sum(M, h, Nfull)) < 1e-12


@pytest.mark.parametrize("blk,h", [((4, 4, 4), (1e-9, 1e-9, 1e-9)),
                                   ((6, 3, 2), (1e-9, 1.5e-9, 0.5e-9)),
                                   ((12, 12, 1), (5e-9, 5e-9, 3e-9))])
def test_uniform_box_mean_field_and_energy(blk, h):
    # a uniformly magnetized box: mean field = -N_box M with N_box the prism's
    # demagnetizing factors (Aharoni), energy = (mu0/2) V_box M.N_box M
    p, q, s = blk
    Mv = np.array([3e5, -4e5, 5e5])
    M = np.broadcast_to(Mv[:, None, None, None], (3, s, q, p)).copy()
    H = conv.fft_conv(M, h)
    Nbox = np.array(aharoni_diag(p * h[0], q * h[1], s * h[2]))
    assert np.allclose(H.mean(axis=(1, 2, 3)), -Nbox * Mv, rtol=1e-12, atol=1e-9)
    Vbox = p * q * s * h[0] * h[1] * h[2]
    E = conv.energy(M, H, h)
    assert math.isclose(E, 0.5 * conv.MU0 * Vbox * float(np.sum(Mv * Nbox * Mv)), rel_tol=1e-12)


def test_energy_positive_and_self_adjoint():
    n, h = (9, 7, 3), (2e-9, 3e-9, 1e-9)
    M = inputs.unit_sphere(n, seed=5).astype(np.float64) * 1.1e6
    G = inputs.gaussian(n, seed=6).astype(np.float64)
    HM = conv.fft_conv(M, h)
    HG = conv.fft_conv(G, h)
    assert conv.energy(M, HM, h) > 0
    assert conv.energy(G, HG, h) > 0
    a, b = float(np.sum(G * HM)), float(np.sum(M * HG))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


@pytest.mark.parametrize("per_cell_ms", [False, True])
def test_gradients_match_central_differences(per_cell_ms):
    # E is quadratic and <G, H> linear in m, so central differences are exact
    # up to rounding
    n, h = (6, 5, 3), (5e-9, 5e-9, 2e-9)
    m = inputs.unit_sphere(n, seed=4).astype(np.float64)
    G = inputs.gaussian(n, seed=5).astype(np.float64)
    if per_cell_ms:
        Ms = inputs.uniform(n[0] * n[1] * n[2], 5e5, 1.4e6, seed=7).reshape(n[2], n[1], n[0])
    else:
        Ms = 8e5
    Nfull = tensor_full(n, h)
    def cv(M, hh):
        return conv.fft_conv(M, hh, Nfull)
    def E(mm):
        M = Ms * mm
        return conv.energy(M, cv(M, h), h)
    def L(mm):
        return float(np.sum(G * cv(Ms * mm, h)))
    gE = conv.grad_energy_m(m, Ms, h, conv=cv)
    gL = conv.grad_inner_m(m, Ms, G, h, conv=cv)
    rng = np.random.default_rng(6)
    step = 1e-3
    for _ in range(64):
        idx = tuple(int(rng.integers(0, s)) for s in m.shape)
        mp_, mm_ = m.copy(), m.copy()
        mp_[idx] += step
        mm_[idx] -= step
        fdE = (E(mp_) - E(mm_)) / (2 * step)
        fdL = (L(mp_) - L(mm_)) / (2 * step)
        assert abs(fdE - gE[idx]) <= 1e-9 * np.max(np.abs(gE)) + 1e-12 * abs(gE[idx])
        assert abs(fdL - gL[idx]) <= 1e-9 * np.max(np.abs(gL))


def test_translation_invariance():
    # a pattern shifted inside a larger mesh produces the shifted field
    h = (2e-9, 2e-9, 1e-9)
    small = inputs.unit_sphere((4, 3, 2), seed=8).astype(np.float64)
    big = np.zeros((3, 4, 6, 9))
    big[:, 1:3, 2:5, 3:7] = small
    Hs = conv.fft_conv(small, h)
    Hb = conv.fft_conv(big, h)
    big2 = np.zeros_like(big)
    big2[:, 2:4, 3:6, 5:9] = small
    Hb2 = conv.fft_conv(big2, h)
    assert np.allclose(Hb[:, 1:3, 2:5, 3:7], Hs, rtol=0, atol=1e-13)
    assert np.allclose(Hb2[:, 2:4, 3:6, 5:9], Hs, rtol=0, atol=1e-13)


def test_sampled_direct_sum_matches_full_direct_sum():
    from oracle.newell import tensor_octant
    n, h = (9, 6, 4), (2e-9, 3e-9, 1e-9)
    M = inputs.unit_sphere(n, seed=12).astype(np.float64)
    Hd = conv.direct_sum(M, h)
    targets = [(0, 0, 0), (3, 5, 8), (1, 2, 4), (2, 0, 7)]
    Hs = conv.direct_sum_at(M, h, targets, tensor_octant(n, h))
    for q, (tz, ty, tx) in enumerate(targets):
        assert np.allclose(Hs[q], Hd[:, tz, ty, tx], rtol=1e-13, atol=0)
