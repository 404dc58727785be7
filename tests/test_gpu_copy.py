"""The streaming copy the benchmark measures the HBM ceiling with: an exact
copy of aligned buffers, and nothing for zero bytes."""
import ctypes

import pytest

from tests.gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu


def test_stream_copy_is_exact():
    torch = require_gpu()
    from paper_2008_02478_amd import lib
    L = lib.load()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n in (4, 1000, (1 << 22) + 12):                     # floats: one float4, a ragged size, several MiB
        x = torch.randn(n, device="cuda")
        y = torch.zeros(n + 4, device="cuda")
        say(f"stream copy of {n} floats")
        lib.check(L.demag_stream_copy(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      (n // 4) * 16, st))
        torch.cuda.synchronize()
        m = (n // 4) * 4
        assert torch.equal(y[:m], x[:m]) and bool((y[m:] == 0).all())
    lib.check(L.demag_stream_copy(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0, st))
