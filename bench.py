#!/usr/bin/env python3
"""Benchmark of the demagnetizing-field hot path on one MI355X.

One step = the whole path on one batch: the field H_d = -N * (Ms m) with the
demag energy (forward), then the gradient of <G, H_d> with respect to m
(backward, the same convolution applied to G).  Workload: a 512x512x16 mesh of
2x2x1 nm cells, Ms = 1.1e6 A/m, random-domain magnetization (Voronoi grains of
~50 cells, seed 10) and a Gaussian upstream gradient (seed 110), open
boundaries, FP32.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  Per-pass durations come from HIP events recorded by the
library between its passes inside the timed region; the middle pass (y FFT,
kernel product, inverse y FFT) moves the most bytes and is the one reported
against the HBM roofline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: each of the 256 compute units issues one wave64 VALU
# instruction per clock (four SIMDs, 16 lanes, 4 cycles per instruction) at
# 2.4 GHz; packed FP32 is not used.
VALU_INSTS_PER_S = 256 * 2.4e9
# FP32 vector peak without packed FP32: 256 CUs x 64 lanes x 2 (fused
# multiply-add) x 2.4 GHz
FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
WORKLOADS = {
    "512x512x16": dict(n=(512, 512, 16), h=(2e-9, 2e-9, 1e-9), Ms=1.1e6, seed=10),
    "1024x1024x4": dict(n=(1024, 1024, 4), h=(2e-9, 2e-9, 1e-9), Ms=1.1e6, seed=11),
    "256x256x8": dict(n=(256, 256, 8), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=2),
    "256x128x4": dict(n=(256, 128, 4), h=(5e-9, 5e-9, 2e-9), Ms=8e5, seed=4),
    "256x256x64": dict(n=(256, 256, 64), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=12),
    "64x64x1": dict(n=(64, 64, 1), h=(5e-9, 5e-9, 3e-9), Ms=8e5, seed=1),
    # z-form crossover (fused x+z passes vs separate z passes) and deep meshes
    "256x256x4": dict(n=(256, 256, 4), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=13),
    "256x256x16": dict(n=(256, 256, 16), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=14),
    "256x256x32": dict(n=(256, 256, 32), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=15),
    "256x256x128": dict(n=(256, 256, 128), h=(4e-9, 4e-9, 4e-9), Ms=8e5, seed=16),
    "512x512x32": dict(n=(512, 512, 32), h=(2e-9, 2e-9, 1e-9), Ms=1.1e6, seed=17),
    "1024x1024x32": dict(n=(1024, 1024, 32), h=(2e-9, 2e-9, 1e-9), Ms=1.1e6, seed=18),
}


def _dims(n, padded):
    """Padded lengths (the plan's, from demag_padded_dims) and the stored
    half/octant extents Kx = Nx/2+1, Ky = Ny/2+1, Kz = Nz/2+1 (1 for unit
    lengths)."""
    Nx, Ny, Nz = padded
    half = lambda N: N // 2 + 1 if N > 1 else 1
    return Nx, Ny, Nz, half(Nx), half(Ny), half(Nz)


def mid_pass_bytes(n, padded):
    """Algorithmic HBM bytes of one middle-pass launch of this library's pass
    order (z transformed in the x passes): read and write the x/z-transformed
    spectrum of the three components (3 * Nz * (Nx/2+1) * ny complex FP32)
    and read the kernel-spectrum octant once (6 * (Nz/2+1) * (Ny/2+1) *
    (Nx/2+1) FP32)."""
    nx, ny, nz = n
    Nx, Ny, Nz, Kx, Ky, Kz = _dims(n, padded)
    spec = 3 * Nz * Kx * ny * 8
    return 2 * spec + 6 * Kz * Ky * Kx * 4


def model_mid_bytes(n, padded):
    """Algorithmic HBM bytes of the fused middle step in the three-pass byte
    model the measurement is held to (x / fused y-z-y / x): read and write
    the x-transformed spectrum (3 * nz * (Nx/2+1) * ny complex FP32, z not yet
    padded) and read the kernel octant once."""
    nx, ny, nz = n
    Nx, Ny, Nz, Kx, Ky, Kz = _dims(n, padded)
    xspec = 3 * nz * Kx * ny * 8
    return 2 * xspec + 6 * Kz * Ky * Kx * 4


def mid_pass_flops(n, padded):
    """Algorithmic FP32 operations of one middle-pass launch, counting a
    complex M-point FFT as 5 M log2 M: per (kz, kx) line and component the two
    residue FFTs forward and inverse (M = Ny/2), the odd residue's twiddle each
    way (6 per point) and the residue sum (2 per point); per frequency the
    3x3 real-by-complex product (30)."""
    import math
    Nx, Ny, Nz, Kx, Ky, Kz = _dims(n, padded)
    M = Ny // 2 if Ny > 1 else 1
    fft = 5 * M * math.log2(M) if M > 1 else 0
    per_line = 3 * (4 * fft + 12 * M + 2 * M) + 30 * Ny
    return per_line * Nz * Kx


def path_bytes(n, padded):
    """Per field evaluation: (algorithmic, compulsory, three-pass model) HBM
    bytes.  Algorithmic: this library's three passes' reads and writes (M in,
    x/z spectrum out; that spectrum in and out plus the kernel octant;
    spectrum in, H out).  Compulsory: read M and the kernel octant once, write
    H.  Three-pass model: M in, x spectrum out; x spectrum in and out plus the
    kernel octant; x spectrum in, H out."""
    nx, ny, nz = n
    Nx, Ny, Nz, Kx, Ky, Kz = _dims(n, padded)
    vec = 3 * nx * ny * nz * 4
    spec = 3 * Nz * Kx * ny * 8
    xspec = 3 * nz * Kx * ny * 8
    kern = 6 * Kz * Ky * Kx * 4
    return 2 * vec + 4 * spec + kern, 2 * vec + kern, 2 * vec + 4 * xspec + kern


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_copy(torch, mib=1024, reps=10):
    """Read + write rate (GB/s) of the library's plain streaming copy, and of
    torch's copy for reference, over 1 GiB buffers."""
    import ctypes
    from paper_2008_02478_amd import lib
    L = lib.load()
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    call = lambda: lib.check(L.demag_stream_copy(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                                 x.numel() * 4, st))
    call()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        call()
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * x.numel() * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    torch_gbs = 2 * x.numel() * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    return gbs, torch_gbs


def bench_batch(torch, reps=10, tune=True, cache=None):
    """Batched multi-mesh workload: three coupled layers (512x512x2 and
    512x512x1 of 1 nm cells, 256x256x3 of 2 nm cells, 1 nm and 3 nm
    spacings) plus 64 independent 64x64x1 meshes of 5x5x3 nm cells; Ms uniform
    in [5e5, 1.4e6] A/m (seed 7), random unit fields (seeds 100+i); energies
    included.  B0: the plain launches, 64 demag_field calls plus the coupled
    group's own batch call, on one stream.  B1: one batched call for all 67
    meshes replayed from a HIP graph."""
    import ctypes
    from paper_2008_02478_amd import inputs, lib
    from paper_2008_02478_amd.demag import DemagBatch, DemagPlan
    L = lib.load()
    layers = [((512, 512, 2), (1e-9, 1e-9, 1e-9)), ((512, 512, 1), (1e-9, 1e-9, 1e-9)),
              ((256, 256, 3), (2e-9, 2e-9, 2e-9))]
    lorig = [(0.0, 0.0, 0.0), (0.0, 0.0, 3e-9), (0.0, 0.0, 7e-9)]
    small, k = ((64, 64, 1), (5e-9, 5e-9, 3e-9)), 64
    meshes = layers + [small] * k
    Ms = inputs.uniform(len(meshes), 5e5, 1.4e6, seed=7).astype(np.float32)
    full = DemagBatch(meshes, origins=lorig + [(0.0, 0.0, 0.0)] * k, groups=[0, 0, 0] + [-1] * k)
    grp = DemagBatch(layers, origins=lorig, groups=[0, 0, 0])
    plan = DemagPlan(*small)
    if tune:
        for x in (full, grp, plan):
            x.autotune(cache=cache)
    mf = torch.empty(full.total, dtype=torch.float32, device="cuda")
    for i, (n, _) in enumerate(meshes):
        full.view(mf, i).copy_(torch.from_numpy(inputs.unit_sphere(n, seed=100 + i)).cuda())
    Hf = torch.empty_like(mf)
    Ef = torch.empty(len(meshes), dtype=torch.float64, device="cuda")
    Msf = torch.from_numpy(Ms).cuda()
    mg = mf[:grp.total].clone()
    Hg = torch.empty_like(mg)
    Eg = torch.empty(3, dtype=torch.float64, device="cuda")
    Msg = Msf[:3].clone()
    ms = [full.view(mf, 3 + i).contiguous() for i in range(k)]
    Hs = [torch.empty_like(x) for x in ms]
    Es = torch.empty(k, dtype=torch.float64, device="cuda")
    st = lambda: ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())

    def b0():
        lib.check(L.demag_field_batch(grp._p, P(mg), P(Msg), 0.0, P(Hg), 0, P(Eg), st()))
        for i in range(k):
            lib.check(L.demag_field(plan._p, P(ms[i]), None, float(Ms[3 + i]), P(Hs[i]), 0,
                                    ctypes.c_void_p(Es.data_ptr() + 8 * i), st()))

    def b1_call():
        lib.check(L.demag_field_batch(full._p, P(mf), P(Msf), 0.0, P(Hf), 0, P(Ef), st()))

    for _ in range(2):
        b0()
        b1_call()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b1_call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b1_call()
    t = {}
    for name, fn in (("B0", b0), ("B1", graph.replay)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t[name] = e0.elapsed_time(e1) / reps
    same = (torch.equal(Hg, Hf[:grp.total]) and torch.equal(Eg, Ef[:3]) and torch.equal(Es, Ef[3:])
            and all(torch.equal(Hs[i].reshape(-1), full.view(Hf, 3 + i).reshape(-1)) for i in range(k)))
    return {"workload": "3 coupled layers (512x512x2 + 512x512x1 of 1 nm, 256x256x3 of 2 nm) + 64 independent "
                        "64x64x1 meshes, energies included",
            "per_mesh_calls_ms": t["B0"], "batched_graph_ms": t["B1"], "speedup": t["B0"] / t["B1"],
            "identical_results": bool(same), "schedules": full.schedules()}


def bench_llg(torch, plan, m_np, steps=10):
    """RK4 steps of the LLG equation on the benchmark mesh (demagnetizing,
    exchange and a perpendicular applied field; four field evaluations per
    step): time per step and per evaluation."""
    m = torch.from_numpy(m_np).to(plan.device)
    kw = dict(Ms=1.1e6, A=1.3e-11, alpha=0.02, dt=1e-13, Hext=(0.0, 0.0, 1e5))
    plan.llg_rk4(m, steps=2, **kw)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    plan.llg_rk4(m, steps=steps, **kw)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {"workload": "RK4 steps of the LLG equation (demagnetizing + exchange + perpendicular applied field) "
                        "on the benchmark mesh, 4 field evaluations per step",
            "ms_per_step": ms, "us_per_evaluation": 1e3 * ms / 4, "steps": steps,
            "params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in kw.items()}}


def oersted_mid_bytes(n, padded):
    """Algorithmic HBM bytes of one Oersted middle-pass launch: the spectrum
    read and written as for the demagnetizing field, and 3 kernel rows
    (instead of 6) per (kz, kx) of the octant."""
    nx, ny, nz = n
    Nx, Ny, Nz, Kx, Ky, Kz = _dims(n, padded)
    return 2 * 3 * Nz * Kx * ny * 8 + 3 * Kz * Ky * Kx * 4


def bench_oersted(torch, n, h, seed, steps=30, tune=True, cache=None):
    """Oersted field H = K * J of a random current density on the benchmark
    mesh: time per evaluation, per pass, and the middle pass against HBM."""
    import ctypes
    from paper_2008_02478_amd import inputs, lib
    from paper_2008_02478_amd.demag import OerstedPlan
    L = lib.load()
    t0 = time.time()
    plan = OerstedPlan(n, h)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    if tune:
        plan.autotune(cache=cache)
    J = torch.from_numpy((1e11 * inputs.gaussian(n, seed=seed)).astype(np.float32)).to(plan.device)
    H = torch.empty_like(J)
    for _ in range(5):
        plan.field(J, out=H)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for s in evs:           # a torch event has a HIP event only once recorded
        for e in s:
            e.record()
    torch.cuda.synchronize()
    handles = [(ctypes.c_void_p * 4)(*[e.cuda_event for e in s]) for s in evs]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for k in range(steps):
        lib.check(L.demag_set_timing_events(plan._p, handles[k], 4))
        plan.field(J, out=H)
    b.record()
    torch.cuda.synchronize()
    lib.check(L.demag_set_timing_events(plan._p, None, 0))
    ms = a.elapsed_time(b) / steps
    pass_us = {"fwd_xz": 1e3 * float(np.mean([s[0].elapsed_time(s[1]) for s in evs])),
               "mid_y": 1e3 * float(np.mean([s[1].elapsed_time(s[2]) for s in evs])),
               "inv_zx": 1e3 * float(np.mean([s[2].elapsed_time(s[3]) for s in evs]))}
    mb = oersted_mid_bytes(n, plan.padded)
    ach = mb / (pass_us["mid_y"] * 1e-6) / 1e9
    return {"workload": f"Oersted field of a random current density on the {n[0]}x{n[1]}x{n[2]} mesh "
                        "(cell-averaged Biot-Savart kernel, open boundaries)",
            "ms_per_eval": ms, "cell_updates_per_s": n[0] * n[1] * n[2] / (ms * 1e-3), "pass_us": pass_us,
            "setup_s": setup_s, "schedule": plan.schedules()[0],
            "mid_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": mb}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1300)   # about 1 s of timed field + backward steps
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="512x512x16", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch schedules")
    ap.add_argument("--schedule-cache", default=None, help="JSON schedule cache to apply (and extend)")
    ap.add_argument("--z-form", choices=("auto", "fused", "separate"), default="auto",
                    help="z transform inside the x passes (fused) or in separate passes; auto: the tuner's choice")
    ap.add_argument("--schedule", default=None, metavar="YG,KW,RADIX",
                    help="launch schedule of the mesh after tuning (0 keeps a field)")
    ap.add_argument("--legs", default="batch,llg,oersted",
                    help="comma-separated secondary legs to run after the main step (batch, llg, oersted)")
    ap.add_argument("--main-only", action="store_true",
                    help="time the field + backward step only (no batch, RK4 or Oersted legs), e.g. under a profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2008_02478_amd import inputs, lib
    from paper_2008_02478_amd.demag import DemagPlan
    if not os.path.exists(lib.LIB_PATH):
        from paper_2008_02478_amd import build_lib
        build_lib.build()

    wl = WORKLOADS[args.workload]
    n, h, Ms = wl["n"], wl["h"], wl["Ms"]
    ncell = n[0] * n[1] * n[2]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if h == (2e-9, 2e-9, 1e-9):
        m_np = inputs.voronoi(n, (h[0] * 1e9, h[1] * 1e9, h[2] * 1e9), seed=wl["seed"])
    else:
        m_np = inputs.unit_sphere(n, seed=wl["seed"])
    G_np = inputs.gaussian(n, seed=wl["seed"] + 100)
    t0 = time.time()
    plan = DemagPlan(n, h, device=dev)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    if args.z_form != "auto":
        plan.set_z_passes(args.z_form == "separate")
    t0 = time.time()
    if not args.no_tune:
        plan.autotune(cache=args.schedule_cache, keep_form=args.z_form != "auto")
    tune_s = time.time() - t0
    if args.schedule:
        yg, kw, radix = (int(v) for v in args.schedule.split(","))
        plan.set_schedule(0, yg, kw, radix)
    m = torch.from_numpy(m_np).to(dev)
    G = torch.from_numpy(G_np).to(dev)
    H = torch.empty_like(m)
    grad = torch.empty_like(m)
    E = torch.empty((), dtype=torch.float64, device=dev)

    import ctypes
    L = lib.load()

    def step():
        plan.field(m, Ms, out=H, energy=False)
        plan.backward(G, Ms, out=grad)

    # field with energy: done through the C ABI so the energy lands in E
    def step_energy():
        lib.check(L.demag_field(plan._p, ctypes.c_void_p(m.data_ptr()), None, Ms, ctypes.c_void_p(H.data_ptr()), 0,
                                ctypes.c_void_p(E.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        plan.backward(G, Ms, out=grad)

    for _ in range(args.warmup):
        step_energy()
    torch.cuda.synchronize()

    # per-pass events: 4 per call, 2 calls per step
    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(2 * K)]
    for s in evs:
        for e in s:
            e.record()
    torch.cuda.synchronize()
    handles = [(ctypes.c_void_p * 4)(*[e.cuda_event for e in s]) for s in evs]

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(K):
        lib.check(L.demag_set_timing_events(plan._p, handles[2 * k], 4))
        lib.check(L.demag_field(plan._p, ctypes.c_void_p(m.data_ptr()), None, Ms, ctypes.c_void_p(H.data_ptr()), 0,
                                ctypes.c_void_p(E.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        lib.check(L.demag_set_timing_events(plan._p, handles[2 * k + 1], 4))
        plan.backward(G, Ms, out=grad)
    stop.record()
    torch.cuda.synchronize()
    lib.check(L.demag_set_timing_events(plan._p, None, 0))
    ms_step = start.elapsed_time(stop) / K

    passes = {"fwd_xz": [], "mid_y": [], "inv_zx": []}
    for s in evs:
        passes["fwd_xz"].append(s[0].elapsed_time(s[1]))
        passes["mid_y"].append(s[1].elapsed_time(s[2]))
        passes["inv_zx"].append(s[2].elapsed_time(s[3]))
    pass_us = {k: 1e3 * float(np.mean(v)) for k, v in passes.items()}
    padded = plan.padded
    mid_bytes = mid_pass_bytes(n, padded)
    model_bytes = model_mid_bytes(n, padded)
    t_mid = pass_us["mid_y"] * 1e-6
    achieved = model_bytes / t_mid / 1e9
    flops = mid_pass_flops(n, padded)
    traffic = None
    valu = None
    side = os.path.join(ROOT, "profiles", f"k_mid_{args.workload}.json")
    if os.path.exists(side):
        from paper_2008_02478_amd.profiling import source_hash
        with open(side) as f:
            prof = json.load(f)
        if prof.get("source_hash") == source_hash():   # counters of this very kernel build
            traffic = prof["traffic_bytes"]
            insts = prof.get("extra_counters", {}).get("SQ_INSTS_VALU")
            if insts:
                floor_us = insts / VALU_INSTS_PER_S * 1e6
                valu = {"insts_per_launch": insts, "issue_floor_us": floor_us,
                        "issue_frac": floor_us / pass_us["mid_y"],
                        "lds_bank_conflict_cycles": prof["extra_counters"].get("SQ_LDS_BANK_CONFLICT")}

    out = {
        "metric": "demag field evals/sec and cell-updates/s (fwd+bwd) at 512x512x16 FP32; HBM GB/s",
        "value": ncell / (ms_step * 1e-3),
        "unit": "cell-updates/s (fwd+bwd)",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n[0]}x{n[1]}x{n[2]} mesh of {h[0]*1e9:g}x{h[1]*1e9:g}x{h[2]*1e9:g} nm cells, "
                        f"Ms={Ms:g} A/m, open boundaries; step = field+energy forward and <G,H> backward",
            "mesh": list(n), "cell_m": list(h), "padded": list(padded),
        },
        "evals_per_s_fwd_bwd_pairs": 1e3 / ms_step,
        "pass_us": pass_us,
        "setup_s": setup_s,
        "tune_s": tune_s,
        "schedule": plan.schedules()[0],
        "z_form": "separate" if plan.z_passes() else "fused",
        "roofline": {
            "bound": "hbm",
            "kernel": "k_mid (y FFT + kernel product + inverse y FFT)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": model_bytes,
            "bytes_model": "three-pass model: x-transformed spectrum (3 nz (Nx/2+1) ny complex FP32) read and "
                           "written once, kernel octant read once",
            "this_pass_order": {
                "algorithmic_bytes_per_launch": mid_bytes,
                "achieved": mid_bytes / t_mid / 1e9,
                "frac": mid_bytes / t_mid / 1e9 / HBM_PEAK_GBS,
                "note": "z is transformed in the x passes, so the middle pass moves the z-padded spectrum "
                        "(3 Nz (Nx/2+1) ny complex FP32) each way"},
            "valu": valu,
            "alu": {"algorithmic_flop_per_launch": flops,
                    "achieved_tflops": flops / t_mid / 1e12,
                    "peak_tflops": FP32_PEAK_TFLOPS,
                    "frac": flops / t_mid / 1e12 / FP32_PEAK_TFLOPS},
        },
    }

    alg, comp, model = path_bytes(n, padded)
    copy_gbs, torch_copy_gbs = bench_copy(torch)
    step_gbs = 2 * alg / (ms_step * 1e-3) / 1e9
    model_gbs = 2 * model / (ms_step * 1e-3) / 1e9
    out["path"] = {
        "model_bytes_per_eval": model, "model_gbs": model_gbs, "model_frac_of_peak": model_gbs / HBM_PEAK_GBS,
        "algorithmic_bytes_per_eval": alg, "compulsory_bytes_per_eval": comp,
        "achieved_gbs": step_gbs, "frac_of_peak": step_gbs / HBM_PEAK_GBS,
        "copy_gbs": copy_gbs, "frac_of_copy": step_gbs / copy_gbs, "torch_copy_gbs": torch_copy_gbs,
        "compulsory_gbs": 2 * comp / (ms_step * 1e-3) / 1e9,
        "note": "two field evaluations (forward with energy, backward) per step; whole-step time"}
    legs = set() if args.main_only else {x for x in args.legs.split(",") if x}
    if legs - {"batch", "llg", "oersted"}:
        ap.error(f"unknown legs {sorted(legs - {'batch', 'llg', 'oersted'})}")
    if "batch" in legs:
        out["batched_multi_mesh"] = bench_batch(torch, tune=not args.no_tune, cache=args.schedule_cache)
    if "llg" in legs:
        out["llg_rk4"] = bench_llg(torch, plan, m_np)
    if "oersted" in legs:
        out["oersted"] = bench_oersted(torch, n, h, wl["seed"] + 200, tune=not args.no_tune,
                                       cache=args.schedule_cache)

    if not args.no_cpu_baseline:
        from oracle import conv
        from oracle.newell import tensor_full
        t0 = time.time()
        Nfull = tensor_full(n, h)
        tensor_s = time.time() - t0
        M = Ms * m_np.astype(np.float64)
        times = []
        for _ in range(3):
            t0 = time.time()
            Hr = conv.fft_conv(M, h, Nfull)
            gr = Ms * conv.fft_conv(G_np.astype(np.float64), h, Nfull)
            times.append(time.time() - t0)
        cpu_s = float(np.median(times))
        Hg = H.cpu().numpy().astype(np.float64)
        gg = grad.cpu().numpy().astype(np.float64)
        out["cpu_baseline"] = {
            "value": ncell / cpu_s,
            "unit": "cell-updates/s (fwd+bwd)",
            "cores": conv.fft_workers(),
            "kind": "oracle",
            "sample": "one forward + backward step of the same workload by the FP64 oracle's FFT convolution, "
                      f"median of 3 ({', '.join(f'{t:.2f}' for t in times)} s; tensor set-up excluded, "
                      f"{tensor_s:.1f} s)",
            "seconds": cpu_s,
            "threads": conv.fft_workers(),
            "host_cpus": os.cpu_count(),
            "cpu_model": cpu_model(),
        }
        out["accuracy"] = {
            "H_rel_l2_vs_fp64_oracle": float(np.linalg.norm(Hg - Hr) / np.linalg.norm(Hr)),
            "grad_rel_l2_vs_fp64_oracle": float(np.linalg.norm(gg - gr) / np.linalg.norm(gr)),
            "E_rel_vs_fp64_oracle": abs(float(E) - conv.energy(M, Hr, h)) / abs(conv.energy(M, Hr, h)),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
