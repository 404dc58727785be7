"""Host-side pieces of bench.py: the byte and operation counts it reports
against the rooflines, and its refusal of more than one GPU."""
import subprocess
import sys

import bench


def test_middle_pass_bytes_at_the_benchmark_size():
    # spectrum 3 x Nz x (Nx/2+1) x ny complex FP32, read and written; kernel
    # octant 6 x (Nz/2+1) x (Ny/2+1) x (Nx/2+1) FP32, read once
    spec = 3 * 32 * 513 * 512 * 8
    kern = 6 * 17 * 513 * 513 * 4
    assert bench.mid_pass_bytes((512, 512, 16)) == 2 * spec + kern == 510812568
    assert bench.oersted_mid_bytes((512, 512, 16)) == 2 * spec + kern // 2


def test_path_bytes_are_the_sum_of_the_passes():
    alg, comp = bench.path_bytes((512, 512, 16))
    vec = 3 * 512 * 512 * 16 * 4
    spec = 3 * 32 * 513 * 512 * 8
    kern = 6 * 17 * 513 * 513 * 4
    x_pass = vec + spec                      # each x pass: the vector one way, the spectrum the other
    assert alg == 2 * x_pass + bench.mid_pass_bytes((512, 512, 16))
    assert comp == 2 * vec + kern


def test_middle_pass_flops():
    # per (kz, kx) line: 3 components x (4 FFTs of 512 points at 5 M log2 M,
    # two residue twiddles of 6 per point, a residue sum of 2 per point) and
    # a 30-operation 3x3 product per frequency
    per_line = 3 * (4 * 5 * 512 * 9 + 12 * 512 + 2 * 512) + 30 * 1024
    assert bench.mid_pass_flops((512, 512, 16)) == per_line * 32 * 513


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
