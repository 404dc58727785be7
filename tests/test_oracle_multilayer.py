"""Pins of the oracle's inter-mesh tensor and multi-mesh direct sum (Sec. 3,
Eq. 4: tensors N(r, h_k, h_i) between cells of different sizes, summed over
a collection of meshes).  None of these values comes from the oracle's own
formulas: equal-cell reduction to the pinned single-mesh tensor, exact
superposition of sub-cells, reciprocity, the overlap-volume trace, the
dipole limit and the split-mesh identity."""
import math

import numpy as np
import pytest

from oracle import conv, multilayer as ml
from oracle.newell import tensor_at
from paper_2008_02478_amd import inputs


def test_equal_cells_reduce_to_single_mesh_tensor():
    h = (2e-9, 3e-9, 1e-9)
    rng = np.random.default_rng(0)
    off = rng.integers(-30, 31, size=(80, 3)) * np.array(h)
    off = np.vstack([off, [[0, 0, 0], [h[0], 0, 0], [0, h[1], h[2]]]])
    a = ml.tensor_unequal(off[:, 0], off[:, 1], off[:, 2], h, h)
    b = tensor_at(off[:, 0], off[:, 1], off[:, 2], h)
    assert np.all(np.abs(a - b) <= 1e-12 * np.max(np.abs(b), axis=0))


@pytest.mark.parametrize("ht,sub,reps", [((1e-9, 1e-9, 1e-9), (1e-9, 1e-9, 1e-9), (2, 2, 2)),
                                         ((2e-9, 1e-9, 1e-9), (1e-9, 1e-9, 2e-9), (2, 1, 3)),
                                         ((1e-9, 3e-9, 2e-9), (1.5e-9, 1e-9, 1e-9), (2, 3, 1))])
def test_superposition_of_subcells(ht, sub, reps):
    # a source cell made of sub-cells produces the sum of their fields
    big = tuple(s * r for s, r in zip(sub, reps))
    for R in [(0.3e-9, 0.2e-9, 0.1e-9), (3e-9, -1e-9, 2e-9), (12e-9, 5e-9, -4e-9), (80e-9, 20e-9, 10e-9)]:
        want = ml.tensor_unequal(*R, ht, big)
        got = 0.0
        for ix in range(reps[0]):
            for iy in range(reps[1]):
                for iz in range(reps[2]):
                    c = [(i + 0.5) * s - 0.5 * b for i, s, b in zip((ix, iy, iz), sub, big)]
                    got = got + ml.tensor_unequal(R[0] - c[0], R[1] - c[1], R[2] - c[2], ht, sub)
        # the closed form loses ~1e-10 to cancellation at a few cells; still exact otherwise
        assert np.max(np.abs(got - want)) <= 3e-10 * np.max(np.abs(want))


def test_reciprocity():
    ha, hb = (1e-9, 1e-9, 1e-9), (2e-9, 2e-9, 3e-9)
    Va, Vb = 1e-27, 12e-27
    for R in [(0.5e-9, 0.5e-9, 1e-9), (4e-9, 1e-9, -3e-9), (25e-9, -10e-9, 6e-9), (90e-9, 0, 40e-9)]:
        a = Va * ml.tensor_unequal(*R, ha, hb)
        b = Vb * ml.tensor_unequal(-R[0], -R[1], -R[2], hb, ha)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_trace_is_overlap_fraction():
    # the Laplacian of 1/r is -4 pi delta: the trace of the cell-averaged
    # tensor is the overlap volume of the two cells over the target volume
    ht, hs = (1e-9, 1e-9, 1e-9), (2e-9, 2e-9, 2e-9)
    N = ml.tensor_unequal(0.0, 0.0, 0.0, ht, hs)
    assert abs(N[0] + N[1] + N[2] - 1.0) < 1e-13
    N = ml.tensor_unequal(0.0, 0.0, 0.0, hs, ht)
    assert abs(N[0] + N[1] + N[2] - 1.0 / 8.0) < 1e-13
    # half overlapping along x: overlap 0.5 x 1 x 1 nm^3 of a 1 nm^3 target
    N = ml.tensor_unequal(1.0e-9, 0.0, 0.0, ht, hs)
    assert abs(N[0] + N[1] + N[2] - 0.5) < 1e-13
    N = ml.tensor_unequal(5e-9, 1e-9, 0.0, ht, hs)
    assert abs(N[0] + N[1] + N[2]) < 1e-12 * np.max(np.abs(N))


def test_dipole_limit():
    ht, hs = (1e-9, 1e-9, 1e-9), (2e-9, 2e-9, 3e-9)
    Vs = 12e-27
    for r in [(300e-9, 0, 0), (0, 0, 250e-9), (150e-9, 120e-9, 60e-9)]:
        N = ml.tensor_unequal(*r, ht, hs)
        v = np.array(r)
        d = np.linalg.norm(v)
        D = Vs / (4 * math.pi) * (np.eye(3) * d * d - 3 * np.outer(v, v)) / d ** 5
        want = np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])
        assert np.max(np.abs(N - want)) / np.max(np.abs(want)) < 2 * (3e-9 / d) ** 2


def test_split_mesh_equals_single_mesh():
    # one mesh of nz = 3 equals three single-layer meshes stacked at zero gap
    n, h = (5, 4, 3), (2e-9, 3e-9, 1e-9)
    M = inputs.unit_sphere(n, seed=9).astype(np.float64) * 8e5
    Hs = conv.direct_sum(M, h)
    layers = [((5, 4, 1), h, (0.0, 0.0, k * h[2])) for k in range(3)]
    H = ml.field(layers, [M[:, k:k + 1] for k in range(3)])
    for k in range(3):
        assert np.allclose(H[k][:, 0], Hs[:, k], rtol=1e-11, atol=1e-6)


def test_coarse_cell_equals_its_fine_cells():
    # a layer of 2 nm cells with the magnetization of a layer of 1 nm cells
    # (uniform within each 2x2x2 block) gives the same field at other layers
    rng = np.random.default_rng(4)
    Mc = rng.standard_normal((3, 1, 2, 3)) * 1e5
    Mf = np.repeat(np.repeat(np.repeat(Mc, 2, axis=1), 2, axis=2), 2, axis=3)
    target = ((4, 3, 1), (1e-9, 1.5e-9, 1e-9), (0.5e-9, -1e-9, 3.0e-9))
    coarse = [target, ((3, 2, 1), (2e-9, 2e-9, 2e-9), (0.0, 0.0, 0.0))]
    fine = [target, ((6, 4, 2), (1e-9, 1e-9, 1e-9), (0.0, 0.0, 0.0))]
    Mt = np.zeros((3, 1, 3, 4))
    Hc = ml.field(coarse, [Mt, Mc])[0]
    Hf = ml.field(fine, [Mt, Mf])[0]
    assert np.allclose(Hc, Hf, rtol=1e-11, atol=1e-6)


def test_gradient_matches_central_differences():
    # <G, H> is linear in M: exact differences pin the adjoint, which follows
    # from reciprocity: d<G,H>/dM_q = V_q H_q[G_p / V_p]
    meshes = [((3, 2, 1), (1e-9, 1e-9, 1e-9), (0.0, 0.0, 0.0)),
              ((2, 1, 2), (2e-9, 2e-9, 1.5e-9), (0.0, 0.0, 2e-9))]
    rng = np.random.default_rng(5)
    M = [rng.standard_normal((3, n[2], n[1], n[0])) for n, _, _ in meshes]
    G = [rng.standard_normal((3, n[2], n[1], n[0])) for n, _, _ in meshes]
    V = [h[0] * h[1] * h[2] for _, h, _ in meshes]
    def L(Mx):
        H = ml.field(meshes, Mx)
        return sum(float(np.sum(g * hh)) for g, hh in zip(G, H))
    HG = ml.field(meshes, [g / v for g, v in zip(G, V)])
    grad = [v * hg for v, hg in zip(V, HG)]
    for q in range(2):
        for idx in [(0, 0, 0, 0), (1, 0, 0, 1), (2, 1, 0, 0)] if q == 1 else [(0, 0, 1, 2), (2, 0, 0, 0)]:
            Mp = [x.copy() for x in M]
            Mm = [x.copy() for x in M]
            Mp[q][idx] += 1.0
            Mm[q][idx] -= 1.0
            fd = (L(Mp) - L(Mm)) / 2.0
            assert abs(fd - grad[q][idx]) <= 1e-9 * max(1.0, abs(fd))


# --- periodic in-plane axes (Sec. 3, multiple images, on a coupled stack) ---

STACK = [((4, 2, 2), (1e-9, 1e-9, 1e-9), (0.0, 0.0, 0.0)),
         ((4, 2, 1), (1e-9, 1e-9, 1e-9), (0.0, 0.0, 3e-9)),
         ((2, 1, 1), (2e-9, 2e-9, 2e-9), (0.0, 0.0, 5e-9))]


def test_periodic_collection_equals_the_repeated_collection():
    # the image-summed field is the open-boundary field of the collection
    # repeated (2K+1)^2 times in the plane, read in its central copy
    K, pbc = 1, (True, True, False)
    Ms = [8e5 * inputs.unit_sphere(n, seed=40 + i).astype(np.float64) for i, (n, _, _) in enumerate(STACK)]
    got = ml.field_periodic(STACK, Ms, pbc, K)
    P = ml.periods(STACK, pbc)
    assert P == pytest.approx((4e-9, 2e-9, 0.0), rel=1e-12)
    tiled, tiled_M = [], []
    for i in range(-K, K + 1):
        for j in range(-K, K + 1):
            for (n, h, o), M in zip(STACK, Ms):
                tiled.append((n, h, (o[0] + i * P[0], o[1] + j * P[1], o[2])))
                tiled_M.append(M)
    central = 3 * ((2 * K + 1) * K + K)              # index of the (0, 0) copy of the first mesh
    want = ml.field(tiled, tiled_M, only=[central, central + 1, central + 2])
    for g, w in zip(got, want):
        assert np.max(np.abs(g - w)) <= 1e-12 * np.max(np.abs(w))


def test_periodic_axes_need_a_common_span():
    with pytest.raises(ValueError):
        ml.periods([((4, 4, 1), (1e-9, 1e-9, 1e-9), (0, 0, 0)), ((3, 4, 1), (1e-9, 1e-9, 1e-9), (0, 0, 2e-9))],
                   (True, False, False))


@pytest.mark.parametrize("axis", [2, 0])
def test_periodic_stack_tends_to_the_infinite_slab(axis):
    # a stack of layers periodic in x and y and uniformly magnetized is, as
    # K grows, a set of infinite slabs: perpendicular M gives H = -M inside
    # every layer, in-plane M gives H = 0 (coarse layer with 2x in-plane cells)
    stack = [((2, 2, 2), (5e-9, 5e-9, 1e-9), (0.0, 0.0, 0.0)),
             ((2, 2, 1), (5e-9, 5e-9, 1e-9), (0.0, 0.0, 3e-9)),
             ((1, 1, 2), (10e-9, 10e-9, 2e-9), (0.0, 0.0, 6e-9))]
    Ms = 1e6
    errs = []
    for K in (3, 12):
        Mlist = []
        for n, _, _ in stack:
            M = np.zeros((3, n[2], n[1], n[0]))
            M[axis] = Ms
            Mlist.append(M)
        H = ml.field_periodic(stack, Mlist, (True, True, False), K)
        want = np.zeros(3)
        want[axis] = -Ms if axis == 2 else 0.0
        err = max(np.max(np.abs(Hp - want[:, None, None, None])) for Hp in H) / Ms
        # a finite film of side L = (2K+1) P deviates by O(thickness / L)
        assert err < 4 * 4e-9 / ((2 * K + 1) * 10e-9), (K, err)
        errs.append(err)
    assert errs[1] < 0.5 * errs[0]
