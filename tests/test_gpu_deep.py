"""GPU parity for meshes with more than 16 cells along z (padded z length 64
or 128):
the z transforms stay fused with the x transforms while the z rows of a y
line fit in LDS (Sec. 7; the pipelined form of the paper applies up to 16
cells, longer lines are the general 3D case).  Field, energy and backward
against the FP64 oracle."""
import numpy as np
import pytest

from oracle import conv
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("n,h", [
    ((40, 30, 20), (2e-9, 2e-9, 1e-9)),
    ((17, 9, 17), (3e-9, 2e-9, 1e-9)),
    ((64, 48, 32), (4e-9, 4e-9, 4e-9)),
    ((1, 1, 32), (5e-9, 5e-9, 3e-9)),
    ((256, 256, 32), (4e-9, 4e-9, 4e-9)),
    ((40, 24, 33), (3e-9, 3e-9, 2e-9)),
    ((256, 256, 64), (4e-9, 4e-9, 4e-9)),
])
def test_deep_meshes(torch, n, h):
    from paper_2008_02478_amd.demag import DemagPlan
    Ms = 8e5
    say(f"deep {n}")
    m = inputs.unit_sphere(n, seed=71)
    G = inputs.gaussian(n, seed=72)
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, h)
    Er = conv.energy(M, Hr, h)
    gr = Ms * conv.fft_conv(G.astype(np.float64), h)
    plan = DemagPlan(n, h)
    assert plan.padded[2] == (64 if n[2] <= 32 else 128)
    H, E = plan.field(to_dev(m, torch), Ms, energy=True)
    g = plan.backward(to_dev(G, torch), Ms)
    torch.cuda.synchronize()
    err, eerr, gerr = rel_l2(H.cpu().numpy(), Hr), abs(float(E) - Er) / abs(Er), rel_l2(g.cpu().numpy(), gr)
    say(f"  field {err:.2e} energy {eerr:.2e} backward {gerr:.2e}")
    assert err < TOL and eerr < TOL and gerr < TOL
