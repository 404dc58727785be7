"""GPU parity of the demagnetizing field, energy and backward against the
FP64 oracle (Table 1 demagnetizing field; Sec. 3 Eq. 4; Sec. 7 zero-padded
FFT convolution; Appendix A field/energy relation).  Inputs are drawn on the
host, rounded to FP32 and given to both sides; the oracle upcasts them."""
import math

import numpy as np
import pytest

from oracle import conv
from oracle.newell import tensor_full
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, max_cell, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def gpu_field(torch, n, h, m, Ms, energy=True):
    from paper_2008_02478_amd.demag import DemagPlan
    plan = DemagPlan(n, h)
    msarg = to_dev(Ms, torch) if isinstance(Ms, np.ndarray) else Ms
    H, E = plan.field(to_dev(m, torch), msarg, energy=True)
    torch.cuda.synchronize()
    return plan, H.cpu().numpy(), float(E)


def test_c1_against_direct_sum(torch):
    n, h, Ms = (64, 64, 1), (5e-9, 5e-9, 3e-9), 8e5
    say(f"C1 {n} seed 1")
    m = inputs.unit_sphere(n, seed=1)
    _, H, E = gpu_field(torch, n, h, m, Ms)
    M = Ms * m.astype(np.float64)
    Nfull = tensor_full(n, h)
    Hd = conv.direct_sum(M, h, Nfull)
    Hf = conv.fft_conv(M, h, Nfull)
    say(f"  rel-L2 vs direct sum {rel_l2(H, Hd):.2e}, oracle routes differ by {rel_l2(Hf, Hd):.1e}")
    assert rel_l2(Hf, Hd) < 1e-12
    assert rel_l2(H, Hd) < TOL
    assert max_cell(H, Hd) < TOL
    assert abs(E - conv.energy(M, Hd, h)) < TOL * abs(conv.energy(M, Hd, h))


RAGGED = [
    ((1, 1, 1), (5e-9, 5e-9, 3e-9)), ((2, 1, 1), (5e-9, 5e-9, 3e-9)), ((1, 2, 1), (5e-9, 5e-9, 3e-9)),
    ((1, 1, 2), (5e-9, 5e-9, 3e-9)), ((3, 1, 1), (2e-9, 2e-9, 1e-9)), ((1, 1, 16), (2e-9, 2e-9, 1e-9)),
    ((5, 3, 2), (1e-9, 1.3e-9, 0.7e-9)), ((7, 6, 1), (5e-9, 5e-9, 3e-9)), ((1, 9, 3), (2e-9, 2e-9, 1e-9)),
    ((12, 5, 4), (4e-9, 4e-9, 4e-9)), ((33, 17, 5), (3e-9, 1e-9, 2e-9)), ((17, 33, 9), (2e-9, 2e-9, 1e-9)),
    ((100, 3, 16), (2e-9, 2e-9, 1e-9)), ((3, 100, 7), (5e-9, 5e-9, 2e-9)), ((65, 65, 1), (5e-9, 5e-9, 3e-9)),
    ((130, 70, 3), (2e-9, 3e-9, 1e-9)), ((257, 9, 2), (2e-9, 2e-9, 2e-9)), ((20, 129, 1), (5e-9, 5e-9, 3e-9)),
]


@pytest.mark.parametrize("n,h", RAGGED)
def test_ragged_meshes(torch, n, h):
    Ms = 8e5
    say(f"ragged {n} {h}")
    m = inputs.unit_sphere(n, seed=21)
    _, H, E = gpu_field(torch, n, h, m, Ms)
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, h)
    err = rel_l2(H, Hr)
    Er = conv.energy(M, Hr, h)
    say(f"  rel-L2 {err:.2e}  max cell {max_cell(H, Hr):.2e}  energy rel {abs(E - Er) / abs(Er):.2e}")
    assert err < TOL
    assert max_cell(H, Hr) < TOL
    assert abs(E - Er) < TOL * abs(Er)


def test_c4_field_energy_and_gradients(torch):
    n, h, Ms = (256, 128, 4), (5e-9, 5e-9, 2e-9), 8e5
    say(f"C4 {n} seeds 4/5")
    from paper_2008_02478_amd.demag import DemagPlan
    m = inputs.unit_sphere(n, seed=4)
    G = inputs.gaussian(n, seed=5)
    plan = DemagPlan(n, h)
    md, Gd = to_dev(m, torch), to_dev(G, torch)
    H, E = plan.field(md, Ms, energy=True)
    gE = torch.tensor(0.37e18, dtype=torch.float64, device="cuda")
    grad = plan.backward(Gd, Ms, H=H, gE=gE)
    Econ = plan.energy(md, Ms, H)
    torch.cuda.synchronize()
    Nfull = tensor_full(n, h)
    cv = lambda X, hh: conv.fft_conv(X, hh, Nfull)
    M = Ms * m.astype(np.float64)
    Hr = cv(M, h)
    Er = conv.energy(M, Hr, h)
    gr = conv.grad_inner_m(m, Ms, G, h, conv=cv) + 0.37e18 * conv.grad_energy_m(m, Ms, h, conv=cv)
    errs = (rel_l2(H.cpu().numpy(), Hr), abs(float(E) - Er) / Er, abs(float(Econ) - Er) / Er,
            rel_l2(grad.cpu().numpy(), gr))
    say("  rel-L2 H %.2e  E(parseval) %.2e  E(cells) %.2e  grad %.2e" % errs)
    assert all(e < TOL for e in errs)
    assert max_cell(H.cpu().numpy(), Hr) < TOL and max_cell(grad.cpu().numpy(), gr) < TOL


@pytest.mark.parametrize("core,seed", [(1, 2), (-1, 3)])
def test_c2_vortex_field_and_energy(torch, core, seed):
    n, h, Ms = (256, 256, 8), (4e-9, 4e-9, 4e-9), 8e5
    say(f"C2 {n} core {core} seed {seed}")
    m = inputs.vortex(n, (4.0, 4.0, 4.0), core, seed)
    _, H, E = gpu_field(torch, n, h, m, Ms)
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, h)
    Er = conv.energy(M, Hr, h)
    say(f"  rel-L2 {rel_l2(H, Hr):.2e}  max cell {max_cell(H, Hr):.2e}  energy rel {abs(E - Er) / Er:.2e}")
    assert rel_l2(H, Hr) < TOL and max_cell(H, Hr) < TOL
    assert abs(E - Er) < TOL * Er


def test_per_cell_ms_and_accumulate(torch):
    n, h = (40, 24, 6), (2e-9, 3e-9, 1e-9)
    say(f"per-cell Ms + accumulate {n}")
    from paper_2008_02478_amd.demag import DemagPlan
    m = inputs.unit_sphere(n, seed=30)
    Ms = inputs.uniform(n[0] * n[1] * n[2], 5e5, 1.4e6, seed=31).astype(np.float32).reshape(n[2], n[1], n[0])
    base = inputs.gaussian(n, seed=32) * 1e4
    plan = DemagPlan(n, h)
    Hd = to_dev(base, torch)
    plan.field(to_dev(m, torch), to_dev(Ms, torch), out=Hd, accumulate=True)
    torch.cuda.synchronize()
    Hr = conv.fft_conv(Ms.astype(np.float64) * m.astype(np.float64), h)
    err = rel_l2(Hd.cpu().numpy() - base, Hr)
    say(f"  rel-L2 {err:.2e}")
    assert err < TOL


def test_autograd_function(torch):
    n, h, Ms = (48, 40, 5), (5e-9, 5e-9, 2e-9), 8e5
    say(f"autograd {n}")
    from paper_2008_02478_amd.demag import DemagPlan, demag
    m = inputs.unit_sphere(n, seed=40)
    G = inputs.gaussian(n, seed=41)
    plan = DemagPlan(n, h)
    md = to_dev(m, torch).requires_grad_(True)
    H, E = demag(md, plan, Ms)
    loss = (to_dev(G, torch) * H).sum() + 2e18 * E
    loss.backward()
    torch.cuda.synchronize()
    gr = conv.grad_inner_m(m, Ms, G, h) + 2e18 * conv.grad_energy_m(m, Ms, h)
    err = rel_l2(md.grad.cpu().numpy(), gr)
    say(f"  rel-L2 grad {err:.2e}")
    assert err < TOL
    # only the energy: the field gradient is absent
    md.grad = None
    H, E = demag(md, plan, Ms)
    (3e18 * E).backward()
    torch.cuda.synchronize()
    gr = 3e18 * conv.grad_energy_m(m, Ms, h)
    assert rel_l2(md.grad.cpu().numpy(), gr) < TOL


def test_deterministic(torch):
    n, h, Ms = (96, 80, 6), (2e-9, 2e-9, 1e-9), 1.1e6
    say(f"determinism {n}")
    from paper_2008_02478_amd.demag import DemagPlan
    plan = DemagPlan(n, h)
    md = to_dev(inputs.voronoi(n, (2, 2, 1), seed=50), torch)
    H1, E1 = plan.field(md, Ms, energy=True)
    H1 = H1.clone(); E1 = E1.clone()
    H2, E2 = plan.field(md, Ms, energy=True)
    torch.cuda.synchronize()
    assert torch.equal(H1, H2) and torch.equal(E1, E2)


def test_self_adjoint_on_gpu(torch):
    n, h = (100, 60, 7), (3e-9, 2e-9, 1e-9)
    say(f"self-adjoint {n}")
    from paper_2008_02478_amd.demag import DemagPlan
    plan = DemagPlan(n, h)
    A = to_dev(inputs.gaussian(n, seed=60), torch)
    B = to_dev(inputs.gaussian(n, seed=61), torch)
    HA = plan.field(A, 1.0)
    HB = plan.field(B, 1.0)
    a = float((B.double() * HA.double()).sum())
    b = float((A.double() * HB.double()).sum())
    assert abs(a - b) < 1e-5 * max(abs(a), abs(b))
