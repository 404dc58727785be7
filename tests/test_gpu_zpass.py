"""GPU parity of the separate z passes (the non-pipelined form for long z
lines, Sec. 7): every padded z length 4..512 forced onto them, the default
for meshes too deep for the fused x+z passes, both forms on one mesh,
periodic z, batches, the Oersted kernel, and a 1024x1024x32 mesh at full size
against sampled direct sums and the uniform-box identity.  Field, fused
energy and backward against the FP64 oracle (Table 1 demag row)."""
import numpy as np
import pytest

from oracle import conv
from oracle.newell import tensor_at
from oracle.pbc import tensor_full_pbc
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev
from tests.test_oracle_tensor import aharoni_diag

pytestmark = pytest.mark.gpu

MS = 8e5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _check(torch, plan, n, h, seed, Nfull=None):
    m = inputs.unit_sphere(n, seed=seed)
    G = inputs.gaussian(n, seed=seed + 1)
    H, E = plan.field(to_dev(m, torch), MS, energy=True)
    g = plan.backward(to_dev(G, torch), MS)
    torch.cuda.synchronize()
    M = MS * m.astype(np.float64)
    Hr = conv.fft_conv(M, h, Nfull)
    Er = conv.energy(M, Hr, h)
    gr = MS * conv.fft_conv(G.astype(np.float64), h, Nfull)
    e1, e2, e3 = rel_l2(H.cpu().numpy(), Hr), abs(float(E) - Er) / abs(Er), rel_l2(g.cpu().numpy(), gr)
    say(f"  field {e1:.2e} energy {e2:.2e} backward {e3:.2e}")
    assert e1 < TOL and e2 < TOL and e3 < TOL
    return H.cpu().numpy()


# one mesh per padded z length (smallest nz of each), and the longest
@pytest.mark.parametrize("n", [(13, 5, 2), (13, 5, 3), (13, 5, 5), (13, 5, 9), (13, 5, 17), (13, 5, 33),
                               (11, 4, 65), (9, 3, 129), (9, 3, 256)])
def test_forced_separate_z_passes(torch, n):
    from paper_2008_02478_amd.demag import DemagPlan
    h = (3e-9, 2e-9, 1e-9)
    say(f"separate z passes {n}")
    plan = DemagPlan(n, h)
    plan.set_z_passes(True)
    assert plan.z_passes()
    _check(torch, plan, n, h, 141)


@pytest.mark.parametrize("n,h", [
    ((64, 48, 100), (4e-9, 4e-9, 4e-9)),        # nz > 64
    ((600, 6, 20), (2e-9, 2e-9, 1e-9)),         # nx > 512 with nz > 16
    ((300, 5, 40), (3e-9, 3e-9, 2e-9)),         # nx > 256 with nz > 32
    ((40, 24, 130), (2e-9, 2e-9, 2e-9)),        # padded z length 512
])
def test_deep_meshes_default_to_separate_z_passes(torch, n, h):
    from paper_2008_02478_amd.demag import DemagPlan
    say(f"deep default {n}")
    plan = DemagPlan(n, h)
    assert plan.z_passes()
    _check(torch, plan, n, h, 143)


def test_fused_and_separate_forms_agree(torch):
    from paper_2008_02478_amd.demag import DemagPlan
    n, h = (40, 30, 20), (2e-9, 2e-9, 1e-9)
    plan = DemagPlan(n, h)
    assert not plan.z_passes()
    say("fused form")
    a = _check(torch, plan, n, h, 145)
    plan.set_z_passes(True)
    say("separate form")
    b = _check(torch, plan, n, h, 145)
    assert rel_l2(b, a) < TOL


@pytest.mark.parametrize("n,h,flags,K", [((16, 12, 40), (3e-9, 3e-9, 2e-9), 4, 3),
                                         ((12, 10, 70), (2e-9, 2e-9, 2e-9), 3, 2)])
def test_periodic_with_separate_z_passes(torch, n, h, flags, K):
    from paper_2008_02478_amd.demag import DemagPlan
    say(f"periodic {n} flags={flags}")
    Nf = tensor_full_pbc(n, h, (bool(flags & 1), bool(flags & 2), bool(flags & 4)), K)
    plan = DemagPlan(n, h, pbc=flags, images=K)
    plan.set_z_passes(True)
    _check(torch, plan, n, h, 147, Nf)


def test_batch_with_separate_z_passes_equals_single_plans(torch):
    from paper_2008_02478_amd.demag import DemagBatch, DemagPlan
    meshes = [((24, 20, 70), (2e-9, 2e-9, 1e-9)), ((24, 20, 70), (2e-9, 2e-9, 1e-9)),
              ((16, 8, 3), (1e-9, 1e-9, 1e-9))]
    say("batch with separate z passes")
    b = DemagBatch(meshes)
    m = torch.empty(b.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(meshes):
        b.view(m, i).copy_(to_dev(inputs.unit_sphere(n, seed=150 + i), torch))
    Ms = torch.tensor([6e5, 8e5, 1e6], dtype=torch.float32, device="cuda")
    H, E = b.field(m, Ms, energy=True)
    torch.cuda.synchronize()
    for i, (n, h) in enumerate(meshes):
        p = DemagPlan(n, h)
        Hi, Ei = p.field(b.view(m, i).contiguous(), float(Ms[i]), energy=True)
        torch.cuda.synchronize()
        assert torch.equal(b.view(H, i).reshape(-1), Hi.reshape(-1)) and torch.equal(E[i], Ei)


def test_oersted_with_separate_z_passes(torch):
    from oracle import oersted
    from paper_2008_02478_amd.demag import OerstedPlan
    n, h = (24, 20, 70), (3e-9, 3e-9, 2e-9)
    say("Oersted, separate z passes")
    J = (1e11 * inputs.gaussian(n, seed=152)).astype(np.float32)
    plan = OerstedPlan(n, h)
    assert plan.z_passes()
    H = plan.field(to_dev(J, torch))
    torch.cuda.synchronize()
    Hr = oersted.field_fft(J.astype(np.float64), h)
    err = rel_l2(H.cpu().numpy(), Hr)
    say(f"  field {err:.2e}")
    assert err < TOL


def test_tuner_chooses_between_the_forms(torch, tmp_path):
    from paper_2008_02478_amd.demag import DemagPlan
    n, h = (64, 48, 32), (4e-9, 4e-9, 4e-9)
    say("tuner over both forms")
    plan = DemagPlan(n, h)
    plan.autotune(cache=tmp_path / "sched.json")
    say(f"  picked separate={plan.z_passes()} {plan.schedules()[0]}")
    _check(torch, plan, n, h, 155)
    text = (tmp_path / "sched.json").read_text()
    assert '"zsep": ' in text
    # a forced form survives tuning with keep_form
    other = not plan.z_passes()
    plan.set_z_passes(other)
    plan.autotune(cache=tmp_path / "sched.json", keep_form=True)
    assert plan.z_passes() == other
    _check(torch, plan, n, h, 156)


def test_full_size_1024x1024x32(torch):
    """The mesh that does not fit the fused passes, at its real size: sampled
    targets of a compact source against the direct sum, and a uniform
    magnetization against the prism factors (mean field = -N_box M)."""
    from paper_2008_02478_amd.demag import DemagPlan
    n, h = (1024, 1024, 32), (2e-9, 2e-9, 1e-9)
    nx, ny, nz = n
    say("full size 1024x1024x32")
    plan = DemagPlan(n, h)
    assert plan.z_passes()
    # compact random source block
    src = (slice(0, nz), slice(500, 516), slice(300, 324))
    m = np.zeros((3, nz, ny, nx), np.float32)
    blk = inputs.unit_sphere((24, 16, nz), seed=157)
    m[:, src[0], src[1], src[2]] = blk
    H = plan.field(to_dev(m, torch), MS).cpu().numpy()
    rng = np.random.default_rng(158)
    targets = [(int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))) for _ in range(6)]
    targets += [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (5, 508, 310)]
    zs, ys, xs = np.meshgrid(np.arange(nz), np.arange(500, 516), np.arange(300, 324), indexing="ij")
    Ms_blk = MS * blk.astype(np.float64)
    scale = np.linalg.norm(H) / np.sqrt(H[0].size)
    for (tz, ty, tx) in targets:
        N = tensor_at((tx - xs) * h[0], (ty - ys) * h[1], (tz - zs) * h[2], h)
        xx, yy, zz, xy, xz, yz = N
        Mx, My, Mz = Ms_blk
        want = -np.array([np.sum(xx * Mx + xy * My + xz * Mz), np.sum(xy * Mx + yy * My + yz * Mz),
                          np.sum(xz * Mx + yz * My + zz * Mz)])
        got = H[:, tz, ty, tx]
        assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want) + 1e-6 * scale, (tz, ty, tx, got, want)
    # uniform magnetization: exact mean field
    u = np.zeros((3, nz, ny, nx), np.float32)
    u[0], u[1], u[2] = 0.6, -0.48, 0.64
    Hu = plan.field(to_dev(u, torch), MS).cpu().numpy()
    Nbox = np.array(aharoni_diag(nx * h[0], ny * h[1], nz * h[2]))
    mean = Hu.mean(axis=(1, 2, 3)) / MS
    want = -Nbox * u[:, 0, 0, 0]
    say(f"  uniform box mean field {mean} vs {want}")
    assert np.allclose(mean, want, rtol=2e-5, atol=2e-6)
