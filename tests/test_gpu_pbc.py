"""GPU parity with periodic boundaries (Sec. 3, multiple images): field,
energy and backward against the FP64 oracle's image-summed tensor, and
batches of periodic meshes against single-mesh plans."""
import numpy as np
import pytest

from oracle import conv
from oracle.pbc import tensor_full_pbc
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

X, Y, Z = 1, 2, 4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _flags(f):
    return (bool(f & X), bool(f & Y), bool(f & Z))


CASES = [
    ((40, 30, 3), (2e-9, 2e-9, 1e-9), X, 3),
    ((32, 48, 2), (5e-9, 4e-9, 3e-9), Y, 5),
    ((24, 20, 1), (2e-9, 2e-9, 1e-9), X | Y, 4),
    ((20, 16, 1), (4e-9, 4e-9, 2e-9), X | Y, 0),     # library default: 10 images
    ((16, 12, 4), (3e-9, 3e-9, 2e-9), Z, 3),
    ((12, 10, 3), (2e-9, 2e-9, 2e-9), X | Y | Z, 2),
    ((33, 7, 5), (1e-9, 2e-9, 1e-9), X | Z, 2),
]


@pytest.mark.parametrize("n,h,flags,K", CASES)
def test_periodic_field_energy_backward(torch, n, h, flags, K):
    from paper_2008_02478_amd.demag import DemagPlan
    Ms = 8e5
    say(f"pbc {n} flags={flags} K={K}")
    Nf = tensor_full_pbc(n, h, _flags(flags), K if K > 0 else 10)
    m = inputs.unit_sphere(n, seed=51)
    G = inputs.gaussian(n, seed=52)
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, h, Nf)
    Er = conv.energy(M, Hr, h)
    gr = Ms * conv.fft_conv(G.astype(np.float64), h, Nf)
    plan = DemagPlan(n, h, pbc=flags, images=K)
    H, E = plan.field(to_dev(m, torch), Ms, energy=True)
    g = plan.backward(to_dev(G, torch), Ms)
    torch.cuda.synchronize()
    err, eerr, gerr = rel_l2(H.cpu().numpy(), Hr), abs(float(E) - Er) / abs(Er), rel_l2(g.cpu().numpy(), gr)
    say(f"  field {err:.2e} energy {eerr:.2e} backward {gerr:.2e}")
    assert err < TOL and eerr < TOL and gerr < TOL


def test_periodic_batch_equals_single_plans(torch):
    from paper_2008_02478_amd.demag import DemagBatch, DemagPlan
    meshes = [((24, 20, 1), (2e-9, 2e-9, 1e-9))] * 3 + [((16, 12, 2), (3e-9, 3e-9, 2e-9))] * 2
    Ms = inputs.uniform(len(meshes), 5e5, 1.4e6, seed=53).astype(np.float32)
    say("periodic batch")
    b = DemagBatch(meshes, pbc=X | Y, images=4)
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(meshes):
        b.view(m, i).copy_(to_dev(inputs.unit_sphere(n, seed=60 + i), torch))
    H = b.field(m, torch.from_numpy(Ms).cuda())
    for i, (n, h) in enumerate(meshes):
        p = DemagPlan(n, h, pbc=X | Y, images=4)
        Hs = p.field(b.view(m, i).contiguous(), float(Ms[i]))
        torch.cuda.synchronize()
        assert torch.equal(Hs, b.view(H, i))


def test_film_limit_on_device(torch):
    # a single-layer film periodic in x and y: uniform Mz gives H close to -M
    from paper_2008_02478_amd.demag import DemagPlan
    n, h, Ms = (64, 64, 1), (2e-9, 2e-9, 1e-9), 1e6
    plan = DemagPlan(n, h, pbc=X | Y, images=40)
    m = np.zeros((3,) + n[::-1], np.float32)
    m[2] = 1.0
    H = plan.field(to_dev(m, torch), Ms).cpu().numpy()
    say(f"film Hz/M in [{H[2].min() / Ms:.5f}, {H[2].max() / Ms:.5f}]")
    assert np.all(np.abs(H[2] / Ms + 1.0) < 0.01)
    assert np.all(np.abs(H[:2] / Ms) < 1e-6)
