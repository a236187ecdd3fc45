"""The calibration kernels: argument checks and that fill/copy/fma write what they say."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


def test_probe_kernels_write_their_buffers():
    import torch
    from paper_1302_7203_amd import binding
    L = binding.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    buf = torch.zeros(4096, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.arrow_probe_fill(p, 16 * 1000, 2.5, st) == 0
    torch.cuda.synchronize()
    assert bool((buf[:2000] == 2.5).all()) and bool((buf[2000:] == 0).all())
    src = torch.arange(4096, dtype=torch.float64, device="cuda")
    assert L.arrow_probe_copy(p, ctypes.c_void_p(src.data_ptr()), 8 * 4096, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(buf, src)
    out = torch.full((2 * 256,), float("nan"), dtype=torch.float64, device="cuda")
    assert L.arrow_probe_fma(ctypes.c_void_p(out.data_ptr()), 2, 10, st) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    # argument errors are synchronous and launch nothing
    assert L.arrow_probe_fill(p, 24, 1.0, st) == -2
    assert L.arrow_probe_fill(ctypes.c_void_p(buf.data_ptr() + 8), 16, 1.0, st) == -1
    assert L.arrow_probe_copy(p, None, 16, st) == -2
    assert L.arrow_probe_fma(None, 1, 1, st) == -1
    assert L.arrow_probe_fma(ctypes.c_void_p(out.data_ptr()), 0, 1, st) == -2
