"""GPU parity for every compile-time class of the x passes.

The x passes (x transform with the z transform fused in, Sec. 7) are
instantiated per (log2 Nx, log2 Nz); each class has its own LDS footprint and
occupancy.  One ragged mesh per class the library accepts runs the field,
the fused energy and the backward against the FP64 oracle's FFT convolution
(Table 1 demag row).  tests/test_abi.py checks on the host that the classes
skipped here are the ones the library rejects for every mesh in them."""
import ctypes

import numpy as np
import pytest

from oracle import conv
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev
from tests.xpass_classes import representatives

pytestmark = pytest.mark.gpu

H = (3e-9, 2e-9, 1e-9)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _accepted(n):
    from paper_2008_02478_amd import lib as L
    lib = L.load()
    p = ctypes.c_void_p()
    rc = lib.demag_setup(ctypes.byref(p), *n, *H, 0, 0)
    if rc == L.OK:
        lib.demag_destroy(p)
    return rc == L.OK


@pytest.mark.parametrize("cls,n", representatives(), ids=[f"lnx{a}-lnz{b}" for (a, b), _ in representatives()])
def test_xpass_class(torch, cls, n):
    from paper_2008_02478_amd.demag import DemagPlan
    if not _accepted(n):
        pytest.skip(f"class {cls} is rejected by demag_setup")
    Ms = 8e5
    say(f"x-pass class {cls} mesh {n}")
    m = inputs.unit_sphere(n, seed=91)
    G = inputs.gaussian(n, seed=92)
    plan = DemagPlan(n, H)
    assert plan.padded[0] == 1 << cls[0] and plan.padded[2] == 1 << cls[1]
    Hd, E = plan.field(to_dev(m, torch), Ms, energy=True)
    g = plan.backward(to_dev(G, torch), Ms)
    torch.cuda.synchronize()
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, H)
    Er = conv.energy(M, Hr, H)
    gr = Ms * conv.fft_conv(G.astype(np.float64), H)
    e1, e2, e3 = rel_l2(Hd.cpu().numpy(), Hr), abs(float(E) - Er) / abs(Er), rel_l2(g.cpu().numpy(), gr)
    say(f"  field {e1:.2e} energy {e2:.2e} backward {e3:.2e}")
    assert e1 < TOL and e2 < TOL and e3 < TOL
