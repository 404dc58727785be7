"""Host-side pieces of bench.py: the byte and operation counts it reports
against the rooflines, and its refusal of more than one GPU."""
import subprocess
import sys

import bench

P = (1024, 1024, 32)   # padded lengths of the 512x512x16 mesh (powers of two >= 2n - 1)


def test_middle_pass_bytes_at_the_benchmark_size():
    # spectrum 3 x Nz x (Nx/2+1) x ny complex FP32, read and written; kernel
    # octant 6 x (Nz/2+1) x (Ny/2+1) x (Nx/2+1) FP32, read once
    spec = 3 * 32 * 513 * 512 * 8
    kern = 6 * 17 * 513 * 513 * 4
    assert bench.mid_pass_bytes((512, 512, 16), P) == 2 * spec + kern == 510812568
    assert bench.oersted_mid_bytes((512, 512, 16), P) == 2 * spec + kern // 2


def test_path_bytes_are_the_sum_of_the_passes():
    alg, comp, model = bench.path_bytes((512, 512, 16), P)
    vec = 3 * 512 * 512 * 16 * 4
    spec = 3 * 32 * 513 * 512 * 8
    kern = 6 * 17 * 513 * 513 * 4
    x_pass = vec + spec                      # each x pass: the vector one way, the spectrum the other
    assert alg == 2 * x_pass + bench.mid_pass_bytes((512, 512, 16), P)
    assert comp == 2 * vec + kern
    # three-pass model: x spectrum (nz planes, z not padded) each way
    xspec = 3 * 16 * 513 * 512 * 8
    assert model == 2 * (vec + xspec) + bench.model_mid_bytes((512, 512, 16), P)
    assert bench.model_mid_bytes((512, 512, 16), P) == 2 * xspec + kern == 309092760
    assert round(model / 1e6, 1) == 611.5


def test_middle_pass_flops():
    # per (kz, kx) line: 3 components x (4 FFTs of 512 points at 5 M log2 M,
    # two residue twiddles of 6 per point, a residue sum of 2 per point) and
    # a 30-operation 3x3 product per frequency
    per_line = 3 * (4 * 5 * 512 * 9 + 12 * 512 + 2 * 512) + 30 * 1024
    assert bench.mid_pass_flops((512, 512, 16), P) == per_line * 32 * 513


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_padded_lengths_come_from_the_library():
    import ctypes
    from paper_2008_02478_amd import lib as L
    lib = L.load()
    p = ctypes.c_void_p()
    assert lib.demag_setup(ctypes.byref(p), 512, 512, 16, 2e-9, 2e-9, 1e-9, 0, 0) == L.OK
    try:
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert lib.demag_padded_dims(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == L.OK
        assert (a.value, b.value, c.value) == P
    finally:
        lib.demag_destroy(p)


def test_source_hash_covers_every_library_source():
    from paper_2008_02478_amd import profiling
    srcs = profiling.kernel_sources()
    for f in ("csrc/xrows.hpp", "csrc/k_field.hip", "csrc/fft_core.hpp", "csrc/plan.hpp", "csrc/demag_api.cpp",
              "csrc/k_layers.hip", "csrc/launch.hpp"):
        assert f in srcs
