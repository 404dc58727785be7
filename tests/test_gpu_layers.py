"""Coupled layers (Sec. 3, Eq. 4): meshes with their own cell sizes and
positions, fields coupled through inter-mesh tensors and summed in the
transform space, against the FP64 oracle's direct sum of Eq. 4."""
import numpy as np
import pytest

from oracle import conv, multilayer as ml
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu
MU0 = 4e-7 * np.pi


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def run(torch, meshes, origins, Ms, seed0, energy=True, G=None, gE=None):
    from paper_2008_02478_amd.demag import DemagBatch
    b = DemagBatch([(n, h) for n, h in meshes], origins=origins, groups=[0] * len(meshes))
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    ms_np = []
    for i, (n, h) in enumerate(meshes):
        x = inputs.unit_sphere(n, seed=seed0 + i)
        b.view(m, i).copy_(to_dev(x, torch))
        ms_np.append(x)
    Msd = torch.tensor(Ms, dtype=torch.float32, device="cuda")
    H, E = b.field(m, Msd, energy=True)
    out = {"b": b, "m": ms_np, "H": [b.view(H, i).cpu().numpy() for i in range(len(meshes))], "E": E.cpu().numpy()}
    if G is not None:
        Gd = torch.empty_like(m)
        for i in range(len(meshes)):
            b.view(Gd, i).copy_(to_dev(G[i], torch))
        gEd = torch.tensor(gE, dtype=torch.float64, device="cuda")
        grad = b.backward(Gd, Msd, H=H, gE=gEd)
        out["grad"] = [b.view(grad, i).cpu().numpy() for i in range(len(meshes))]
    torch.cuda.synchronize()
    return out


TINY = [((8, 6, 2), (1e-9, 1e-9, 1e-9)), ((8, 6, 1), (1e-9, 1e-9, 1e-9)), ((4, 3, 1), (2e-9, 2e-9, 2e-9))]
TINY_ORIG = [(0.0, 0.0, 0.0), (0.0, 0.0, 3e-9), (0.0, 0.0, 6e-9)]


def test_tiny_group_against_direct_sum_with_energy_and_gradient(torch):
    Ms = [8e5, 1.1e6, 6e5]
    G = [inputs.gaussian(n, seed=50 + i).astype(np.float64) for i, (n, _) in enumerate(TINY)]
    gE = [1e18, 2e18, 3e18]
    say("tiny coupled group (3 layers, unequal cells)")
    r = run(torch, TINY, TINY_ORIG, Ms, 40, G=G, gE=gE)
    meshes = [(n, h, o) for (n, h), o in zip(TINY, TINY_ORIG)]
    M = [Ms[i] * r["m"][i].astype(np.float64) for i in range(3)]
    Hr = ml.field(meshes, M)
    err = rel_l2(np.concatenate([x.ravel() for x in r["H"]]), np.concatenate([x.ravel() for x in Hr]))
    say(f"  field rel-L2 {err:.2e}")
    assert err < TOL
    for i, (n, h) in enumerate(TINY):
        V = h[0] * h[1] * h[2]
        Er = -0.5 * MU0 * V * float(np.sum(M[i] * Hr[i]))
        assert abs(r["E"][i] - Er) < TOL * abs(Er) + 1e-3 * TOL * max(abs(x) for x in r["E"]), (i, r["E"][i], Er)
    # d<G,H>/dm_i + gE_i dE_i/dm_i with the reciprocity adjoint V_i H_i[G/V]
    Vs = [h[0] * h[1] * h[2] for _, h in TINY]
    HG = ml.field(meshes, [G[i] / Vs[i] for i in range(3)])
    want = [Ms[i] * Vs[i] * (HG[i] - MU0 * gE[i] * Hr[i]) for i in range(3)]
    errg = rel_l2(np.concatenate([x.ravel() for x in r["grad"]]), np.concatenate([x.ravel() for x in want]))
    say(f"  gradient rel-L2 {errg:.2e}")
    assert errg < TOL


def test_group_with_in_plane_offsets_and_stride_four(torch):
    """Planes on the fine in-plane lattice at offsets of whole fine cells, one
    layer with cells four times the finest: the embedding and decimation of
    the layer x passes (cells found on a stride with an offset) against the
    Eq. 4 direct sum, field and energies."""
    meshes = [((12, 9, 1), (1e-9, 1e-9, 1e-9)), ((3, 2, 2), (4e-9, 4e-9, 1e-9)), ((5, 4, 1), (1e-9, 1e-9, 1e-9))]
    orig = [(0.0, 0.0, 0.0), (1e-9, 2e-9, 2e-9), (3e-9, 1e-9, 5e-9)]
    Ms = [8e5, 1.0e6, 6e5]
    say("coupled group with in-plane offsets and a stride-4 layer")
    r = run(torch, meshes, orig, Ms, 60)
    M = [Ms[i] * r["m"][i].astype(np.float64) for i in range(3)]
    Hr = ml.field([(n, h, o) for (n, h), o in zip(meshes, orig)], M)
    err = rel_l2(np.concatenate([x.ravel() for x in r["H"]]), np.concatenate([x.ravel() for x in Hr]))
    say(f"  field rel-L2 {err:.2e}")
    assert err < TOL
    for i, (n, h) in enumerate(meshes):
        V = h[0] * h[1] * h[2]
        Er = -0.5 * MU0 * V * float(np.sum(M[i] * Hr[i]))
        assert abs(r["E"][i] - Er) < TOL * abs(Er) + 1e-3 * TOL * max(abs(x) for x in r["E"]), (i, r["E"][i], Er)


def test_split_layers_equal_single_mesh(torch):
    # two single-plane layers stacked at zero gap reproduce one two-plane mesh
    from paper_2008_02478_amd.demag import DemagPlan
    n, h = (40, 24, 2), (2e-9, 3e-9, 1e-9)
    x = inputs.unit_sphere(n, seed=61)
    plan = DemagPlan(n, h)
    Hs = plan.field(to_dev(x, torch), 8e5).cpu().numpy()
    meshes = [((40, 24, 1), h), ((40, 24, 1), h)]
    from paper_2008_02478_amd.demag import DemagBatch
    b = DemagBatch(meshes, origins=[(0, 0, 0), (0, 0, h[2])], groups=[0, 0])
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    b.view(m, 0).copy_(to_dev(x[:, 0:1], torch))
    b.view(m, 1).copy_(to_dev(x[:, 1:2], torch))
    H = b.field(m, 8e5)
    torch.cuda.synchronize()
    Hl = np.concatenate([b.view(H, 0).cpu().numpy(), b.view(H, 1).cpu().numpy()], axis=1)
    say(f"  split vs single rel-L2 {rel_l2(Hl, Hs):.2e}")
    assert rel_l2(Hl, Hs) < TOL


def test_medium_group_sampled_direct_sum(torch):
    meshes = [((64, 64, 2), (1e-9, 1e-9, 1e-9)), ((64, 64, 1), (1e-9, 1e-9, 1e-9)), ((32, 32, 3), (2e-9, 2e-9, 2e-9))]
    orig = [(0.0, 0.0, 0.0), (0.0, 0.0, 3e-9), (0.0, 0.0, 7e-9)]
    Ms = [7e5, 1.2e6, 9e5]
    say("medium coupled group 64x64x2 + 64x64x1 + 32x32x3")
    r = run(torch, meshes, orig, Ms, 70)
    M = [Ms[i] * r["m"][i].astype(np.float64) for i in range(3)]
    rng = np.random.default_rng(3)
    targets = []
    for i, (n, _) in enumerate(meshes):
        for _ in range(4):
            targets.append((i, (int(rng.integers(n[2])), int(rng.integers(n[1])), int(rng.integers(n[0])))))
        targets.append((i, (0, 0, 0)))
        targets.append((i, (n[2] - 1, n[1] - 1, n[0] - 1)))
    Hr = ml.field_at([(n, h, o) for (n, h), o in zip(meshes, orig)], M, targets)
    got = np.array([r["H"][i][:, k, j, x] for i, (k, j, x) in targets])
    err = rel_l2(got, Hr)
    say(f"  sampled rel-L2 {err:.2e}")
    assert err < TOL


def test_mixed_batch(torch):
    # a coupled group and independent meshes in one plan: independent meshes
    # match their own single-mesh plans bit for bit
    from paper_2008_02478_amd.demag import DemagBatch, DemagPlan
    meshes = TINY + [((64, 64, 1), (5e-9, 5e-9, 3e-9))] * 4
    origins = TINY_ORIG + [(0.0, 0.0, 0.0)] * 4
    groups = [0, 0, 0, -1, -1, -1, -1]
    b = DemagBatch(meshes, origins=origins, groups=groups)
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(meshes):
        b.view(m, i).copy_(to_dev(inputs.unit_sphere(n, seed=80 + i), torch))
    H = b.field(m, 8e5)
    plan = DemagPlan((64, 64, 1), (5e-9, 5e-9, 3e-9))
    for i in range(3, 7):
        Hi = plan.field(b.view(m, i).contiguous(), 8e5)
        torch.cuda.synchronize()
        assert torch.equal(Hi, b.view(H, i))
    meshes3 = [(n, h, o) for (n, h), o in zip(TINY, TINY_ORIG)]
    Hr = ml.field(meshes3, [8e5 * b.view(m, i).cpu().numpy().astype(np.float64) for i in range(3)])
    err = rel_l2(np.concatenate([b.view(H, i).cpu().numpy().ravel() for i in range(3)]),
                 np.concatenate([x.ravel() for x in Hr]))
    assert err < TOL


C5_LAYERS = [((512, 512, 2), (1e-9, 1e-9, 1e-9)), ((512, 512, 1), (1e-9, 1e-9, 1e-9)),
             ((256, 256, 3), (2e-9, 2e-9, 2e-9))]
C5_ORIG = [(0.0, 0.0, 0.0), (0.0, 0.0, 3e-9), (0.0, 0.0, 7e-9)]


def test_full_size_layers_and_small_meshes(torch):
    # three coupled layers (1 nm and 3 nm spacings) plus 64 independent
    # 64x64x1 meshes, one plan; sampled direct sums of Eq. 4 for the layers
    from paper_2008_02478_amd.demag import DemagBatch
    meshes = C5_LAYERS + [((64, 64, 1), (5e-9, 5e-9, 3e-9))] * 64
    origins = C5_ORIG + [(0.0, 0.0, 0.0)] * 64
    groups = [0, 0, 0] + [-1] * 64
    Ms = inputs.uniform(len(meshes), 5e5, 1.4e6, seed=7).astype(np.float32)
    say("full-size layers + 64 small meshes")
    b = DemagBatch(meshes, origins=origins, groups=groups)
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    host = []
    for i, (n, _) in enumerate(meshes):
        x = inputs.unit_sphere(n, seed=100 + i)
        host.append(x)
        b.view(m, i).copy_(to_dev(x, torch))
    H, E = b.field(m, torch.from_numpy(Ms).cuda(), energy=True)
    torch.cuda.synchronize()
    Hl = [b.view(H, i).cpu().numpy() for i in range(3)]
    M = [float(Ms[i]) * host[i].astype(np.float64) for i in range(3)]
    targets = [(0, (1, 100, 200)), (1, (0, 511, 3)), (2, (2, 128, 17)), (2, (0, 0, 255))]
    say("  oracle direct sums at 4 cells")
    Hr = ml.field_at([(n, h, o) for (n, h), o in zip(C5_LAYERS, C5_ORIG)], M, targets)
    got = np.array([Hl[i][:, k, j, x] for i, (k, j, x) in targets])
    err = rel_l2(got, Hr)
    say(f"  sampled rel-L2 {err:.2e}")
    assert err < TOL
    for i in (3, 40, 66):
        n, h = meshes[i]
        Hs = conv.fft_conv(float(Ms[i]) * host[i].astype(np.float64), h)
        assert rel_l2(b.view(H, i).cpu().numpy(), Hs) < TOL
