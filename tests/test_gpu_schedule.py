"""Launch schedules and the schedule tuner on the GPU.  Every schedule a plan
offers computes the same convolution (Sec. 3, Eq. 4; Sec. 7 zero-padded FFT
convolution), so each one is held to the FP64 oracle at the stated tolerance;
the tuner must pick a valid schedule, write it to its JSON cache and apply it
from there without measuring again."""
import json

import numpy as np
import pytest

from oracle import conv
from paper_2008_02478_amd import inputs
from tests.gpu_common import TOL, rel_l2, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


# (mesh, cell): y lines of 256 points (radix 4 / 8 / 16), of 512 points
# (radix 8 / 16), of 1024 points (radix 16, and radix 8 with lines spanning
# two wavefronts), and a short-line mesh with several z planes per x row
CASES = [
    ((150, 200, 3), (2e-9, 2e-9, 1e-9)),
    ((40, 300, 2), (5e-9, 5e-9, 3e-9)),
    ((40, 600, 2), (4e-9, 2e-9, 3e-9)),
    ((70, 30, 5), (3e-9, 3e-9, 2e-9)),
]


def _all_schedules(plan):
    base = plan.schedules()[0]
    out = []
    for kw in (2, 4, 8):
        for r in (4, 8, 16):
            try:
                plan.set_schedule(0, kw=kw, radix=r)
            except Exception:
                continue
            out.append((base["yg"], kw, r))
    ny = plan.n[1]
    for yg in (1, 2, 3, 5, 8):
        if yg <= ny and yg != base["yg"]:
            try:
                plan.set_schedule(0, yg=yg, kw=base["kw"], radix=base["radix"])
            except Exception:
                continue
            out.append((yg, base["kw"], base["radix"]))
    plan.set_schedule(0, yg=base["yg"], kw=base["kw"], radix=base["radix"])
    return out


@pytest.mark.parametrize("n,h", CASES)
def test_every_schedule_matches_oracle(torch, n, h):
    from paper_2008_02478_amd.demag import DemagPlan
    Ms = 8e5
    m = inputs.unit_sphere(n, seed=21)
    M = Ms * m.astype(np.float64)
    Hr = conv.fft_conv(M, h)
    Er = conv.energy(M, Hr, h)
    plan = DemagPlan(n, h)
    md = to_dev(m, torch)
    scheds = _all_schedules(plan)
    say(f"schedules {n}: {len(scheds)}")
    assert len(scheds) >= 3
    for yg, kw, r in scheds:
        plan.set_schedule(0, yg=yg, kw=kw, radix=r)
        assert plan.schedules()[0] == {"yg": yg, "kw": kw, "radix": r}
        H, E = plan.field(md, Ms, energy=True)
        G = plan.backward(md, Ms)
        torch.cuda.synchronize()
        err = rel_l2(H.cpu().numpy(), Hr)
        eerr = abs(float(E) - Er) / abs(Er)
        gerr = rel_l2(G.cpu().numpy(), Hr)   # Ms (-N * G) with G = m
        say(f"  yg={yg} kw={kw} radix={r}: field {err:.2e} energy {eerr:.2e} backward {gerr:.2e}")
        assert err < TOL and eerr < TOL and gerr < TOL


def test_autotune_cache_round_trip(torch, tmp_path):
    from paper_2008_02478_amd.demag import DemagPlan
    n, h, Ms = (150, 200, 3), (2e-9, 2e-9, 1e-9), 8e5
    cache = tmp_path / "sched.json"
    say(f"autotune {n}")
    p1 = DemagPlan(n, h)
    assert p1.autotune(cache=cache) == 1
    data = json.loads(cache.read_text())
    assert data["format"] == "demag-schedule-cache/1"
    (key, ent), = data["entries"].items()
    assert "mesh 150x200x3 nb=1" in key
    s1 = p1.schedules()[0]
    assert s1 == {"yg": ent["yg"], "kw": ent["kw"], "radix": ent["radix"]}
    assert ent["x_us"] > 0 and ent["mid_us"] > 0
    say(f"  picked {s1}, x {ent['x_us']:.1f} us, middle {ent['mid_us']:.1f} us")
    p2 = DemagPlan(n, h)
    assert p2.autotune(cache=cache) == 0          # applied from the cache
    assert p2.schedules()[0] == s1
    assert p2.autotune(cache=cache, force=True) == 1
    m = inputs.unit_sphere(n, seed=22)
    Hr = conv.fft_conv(Ms * m.astype(np.float64), h)
    H = p2.field(to_dev(m, torch), Ms)
    torch.cuda.synchronize()
    assert rel_l2(H.cpu().numpy(), Hr) < TOL


def test_autotune_batch_with_layers(torch, tmp_path):
    from paper_2008_02478_amd.demag import DemagBatch
    meshes = [((64, 64, 1), (5e-9, 5e-9, 3e-9))] * 4 + [((48, 40, 2), (2e-9, 2e-9, 1e-9)),
                                                      ((24, 20, 1), (4e-9, 4e-9, 2e-9))]
    origins = [(0.0, 0.0, 0.0)] * 4 + [(0.0, 0.0, 0.0), (0.0, 0.0, 3e-9)]
    groups = [-1] * 4 + [0, 0]
    Ms = inputs.uniform(len(meshes), 5e5, 1.4e6, seed=23).astype(np.float32)
    say("autotune batch: 4 small meshes + a 2-layer group")
    a = DemagBatch(meshes, origins=origins, groups=groups)
    b = DemagBatch(meshes, origins=origins, groups=groups)
    assert len(a.schedules()) == 2
    m = torch.empty(a.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(meshes):
        a.view(m, i).copy_(to_dev(inputs.unit_sphere(n, seed=300 + i), torch))
    msd = torch.from_numpy(Ms).cuda()
    H0, E0 = a.field(m, msd, energy=True)
    assert b.autotune(cache=tmp_path / "c.json") == 2
    H1, E1 = b.field(m, msd, energy=True)
    torch.cuda.synchronize()
    say(f"  schedules {b.schedules()}")
    for i in range(len(meshes)):
        assert rel_l2(b.view(H1, i).cpu().numpy(), a.view(H0, i).cpu().numpy()) < 1e-6
    assert np.allclose(E1.cpu().numpy(), E0.cpu().numpy(), rtol=1e-6, atol=0)
