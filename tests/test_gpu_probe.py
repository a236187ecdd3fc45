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


def test_reciprocal_accuracy_the_solver_relies_on():
    """The solver's reciprocals: the hardware estimate to about 2^-24 (used where only a sign
    matters), one Newton step within 16 ulps (the double-double b pass, whose remainder digit
    corrects it), two steps correctly rounded (every other pass)."""
    import numpy as np
    import torch
    from paper_1302_7203_amd import binding
    L = binding.lib()
    rng = np.random.default_rng(11)
    n = 1 << 20
    x = rng.uniform(1.0, 2.0, n) * np.exp2(np.floor(rng.uniform(-300.0, 300.0, n))) * rng.choice([-1.0, 1.0], n)
    x[:4] = [1.0, -1.0, 3.0, np.nextafter(2.0, 1.0)]
    xd = torch.from_numpy(x).cuda()
    out = torch.full((3 * n,), float("nan"), dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.arrow_probe_rcp(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, st) == 0
    torch.cuda.synchronize()
    r = out.cpu().numpy().reshape(3, n)
    ref = 1.0 / x
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(r[0] - ref) <= 2.0 ** -22 * np.abs(ref))
    assert np.all(np.abs(r[1] - ref) <= 16 * ulp)
    assert np.array_equal(r[2], ref)
    assert L.arrow_probe_rcp(None, ctypes.c_void_p(out.data_ptr()), n, st) == -1
    assert L.arrow_probe_rcp(ctypes.c_void_p(xd.data_ptr()), None, n, st) == -2
    assert L.arrow_probe_rcp(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(out.data_ptr()), 0, st) == -3
