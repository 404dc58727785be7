"""Build of libdemag with AddressSanitizer and UndefinedBehaviorSanitizer in
its host code (the C ABI, plans, validation, the schedule cache), for the CPU
tests of the ABI.  The device code is linked unchanged from the normal build;
sanitizers apply to the host pass only.

    python tests/sanitize_host.py     # writes _build/asan/libdemag_asan.so
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2008_02478_amd import build_lib  # noqa: E402

OUT = os.path.join(ROOT, "_build", "asan")
LIB = os.path.join(OUT, "libdemag_asan.so")
HOST_SOURCES = ["demag_api.cpp", "tune_cache.cpp"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def runtime():
    """The shared ASan runtime of the ROCm clang (it carries the UBSan
    handlers too); preloaded into an uninstrumented python."""
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not c:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return c[-1]


def build():
    os.makedirs(OUT, exist_ok=True)
    dev = [os.path.join(build_lib.BUILD, os.path.splitext(s)[0] + ".o")
           for s in build_lib.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in dev):
        build_lib.build(verbose=False)
    objs = list(dev)
    for src in HOST_SOURCES:
        obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        cmd = [build_lib._hipcc(), *build_lib.FLAGS, *SAN, "-c", os.path.join(build_lib.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized build of {src} failed:\n{r.stderr}")
        objs.append(obj)
    cmd = [build_lib._hipcc(), f"--offload-arch={build_lib.ARCH}", "-shared", "-fPIC", *objs, "-o", LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return LIB


def env():
    e = dict(os.environ)
    e["LD_PRELOAD"] = runtime()
    e["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    e["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    e["DEMAG_LIB"] = LIB
    return e


if __name__ == "__main__":
    print(build())
