"""The FP32 issue-rate helper computes what it states: per lane, 8 chains of x <- x * a + b as a
float32 multiply then a float32 add (no fused form), summed in chain order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_peak_fp32_values_and_flop_count():
    import torch
    from paper_2410_00425_amd import ms
    n_waves, iters = 3, 257
    out = torch.full((n_waves * 64,), np.nan, dtype=torch.float32, device="cuda")
    flop = ms.peak_fp32(out, n_waves, iters)
    torch.cuda.synchronize()
    assert flop == 16 * iters * 64 * n_waves
    a, b = np.float32(0.999), np.float32(1e-3)
    lane = np.arange(64, dtype=np.float32)
    x = np.stack([lane * np.float32(1e-3) + np.float32(k) for k in range(8)]).astype(np.float32)
    for _ in range(iters):
        x = (x * a).astype(np.float32) + b
    s = np.zeros(64, np.float32)
    for k in range(8):
        s = (s + x[k]).astype(np.float32)
    got = out.cpu().numpy().reshape(n_waves, 64)
    for w in range(n_waves):
        assert np.array_equal(got[w], s)


def test_peak_fp32_rejects_bad_arguments():
    import torch
    from paper_2410_00425_amd import ms
    out = torch.empty(64, dtype=torch.float32, device="cuda")
    with pytest.raises(ms.MsError):
        ms.peak_fp32(out, 0, 10)
    with pytest.raises(ValueError):
        ms.peak_fp32(out, 2, 10)
