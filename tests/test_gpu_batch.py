"""Batches of independent meshes (Sec. 3: a collection of meshes, each with its
own discretization) in one launch sequence, and its HIP-graph capture."""
import numpy as np
import pytest

from oracle import conv
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def batch_meshes():
    meshes = [((64, 64, 1), (5e-9, 5e-9, 3e-9))] * 64
    meshes += [((40, 24, 6), (2e-9, 3e-9, 1e-9)), ((17, 33, 3), (2e-9, 2e-9, 1e-9)),
               ((40, 24, 6), (2e-9, 3e-9, 1e-9)), ((128, 64, 4), (5e-9, 5e-9, 2e-9))]
    return meshes


def fill(batch, torch, seed0):
    x = torch.empty(batch.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(batch.meshes):
        batch.view(x, i).copy_(to_dev(inputs.unit_sphere(n, seed=seed0 + i), torch))
    return x


def test_batch_equals_single_mesh_launches_and_oracle(torch):
    from paper_2008_02478_amd.demag import DemagBatch, DemagPlan
    meshes = batch_meshes()
    say(f"batch of {len(meshes)} meshes")
    b = DemagBatch(meshes)
    m = fill(b, torch, 100)
    Ms = torch.from_numpy(inputs.uniform(len(meshes), 5e5, 1.4e6, seed=7).astype(np.float32)).cuda()
    H, E = b.field(m, Ms, energy=True)
    G = torch.randn(b.total, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    gE = torch.linspace(1e17, 2e17, len(meshes), dtype=torch.float64, device="cuda")
    grad = b.backward(G, Ms, H=H, gE=gE)
    torch.cuda.synchronize()
    plans = {}
    for i, (n, h) in enumerate(meshes):
        key = (n, h)
        if key not in plans:
            plans[key] = DemagPlan(n, h)
        p = plans[key]
        mi = b.view(m, i).contiguous()
        Hi, Ei = p.field(mi, float(Ms[i]), energy=True)
        gi = p.backward(b.view(G, i).contiguous(), float(Ms[i]), H=Hi, gE=gE[i:i + 1])
        torch.cuda.synchronize()
        assert torch.equal(Hi, b.view(H, i)), i          # same kernels, same arithmetic
        assert torch.equal(Ei, E[i]), i
        assert torch.equal(gi, b.view(grad, i)), i
    for i in (0, 37, 64, 65, 67):
        n, h = meshes[i]
        M = float(Ms[i]) * b.view(m, i).cpu().numpy().astype(np.float64)
        Hr = conv.fft_conv(M, h)
        err = rel_l2(b.view(H, i).cpu().numpy(), Hr)
        Er = conv.energy(M, Hr, h)
        say(f"  mesh {i} {n}: rel-L2 {err:.2e}, energy {abs(float(E[i]) - Er) / Er:.2e}")
        assert err < TOL and abs(float(E[i]) - Er) < TOL * Er


def test_graph_capture_replays(torch):
    from paper_2008_02478_amd.demag import DemagBatch
    meshes = batch_meshes()
    say(f"graph capture of a batch of {len(meshes)} meshes")
    b = DemagBatch(meshes)
    m = fill(b, torch, 200)
    H = torch.empty_like(m)
    E = torch.empty(len(meshes), dtype=torch.float64, device="cuda")
    H0, E0 = b.field(m, 8e5, energy=True)
    H0, E0 = H0.clone(), E0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.field(m, 8e5, out=H, energy=False)          # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    import ctypes
    from paper_2008_02478_amd import lib as L
    with torch.cuda.graph(g):
        L.check(L.load().demag_field_batch(b._p, ctypes.c_void_p(m.data_ptr()), None, 8e5,
                                           ctypes.c_void_p(H.data_ptr()), 0, ctypes.c_void_p(E.data_ptr()),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    for k in range(4):
        H.zero_()
        E.zero_()
        m.mul_(1.0)                                    # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(H, H0) and torch.equal(E, E0), f"replay {k}"
