"""The tracklet filter's shorter square root (catpc_fp32_probe op 5) equals the
correctly rounded binary32 square root (op 4, which the host-rounding test
pins to numpy) for every binary32 value of its domain, the normal values from
2^-96 to the largest finite one: an exhaustive comparison on the device."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_short_sqrt_equals_sqrtf_on_its_whole_domain():
    from paper_1712_09430_amd import catpc as C
    lo, hi = 0x0F800000, 0x7F800000  # bit patterns of 2^-96 and +inf (exclusive)
    chunk = 1 << 27
    buf = torch.empty(chunk, dtype=torch.int32, device="cuda")
    a = torch.empty(chunk, dtype=torch.float32, device="cuda")
    b = torch.empty(chunk, dtype=torch.float32, device="cuda")
    checked = 0
    for start in range(lo, hi, chunk):
        n = min(chunk, hi - start)
        torch.arange(start, start + n, dtype=torch.int32, device="cuda", out=buf[:n])
        x = buf[:n].view(torch.float32)
        C.catpc_fp32_probe(4, x.data_ptr(), x.data_ptr(), a.data_ptr(), n, None)
        C.catpc_fp32_probe(5, x.data_ptr(), x.data_ptr(), b.data_ptr(), n, None)
        diff = torch.ne(a[:n].view(torch.int32), b[:n].view(torch.int32))
        bad = int(diff.sum().item())
        if bad:
            i = int(torch.nonzero(diff)[0].item())
            pytest.fail(f"{bad} mismatches in [{start:#x}, {start + n:#x}); first x bits {start + i:#x}")
        checked += n
    assert checked == hi - lo


def test_short_sqrt_on_the_transport_domain_matches_numpy():
    """Spot check against the host on the domain the transport uses,
    1 - s^2 for |s| < 0.999."""
    from paper_1712_09430_amd import catpc as C
    rng = np.random.default_rng(3)
    s = rng.uniform(-0.999, 0.999, 1 << 20).astype(np.float32)
    x = (np.float32(1.0) - s * s).astype(np.float32)
    x[:4] = [np.float32(1.0) - np.float32(0.999) * np.float32(0.999), 1.0, 0.5, 0.25]
    dx = torch.from_numpy(x).cuda()
    out = torch.empty_like(dx)
    C.catpc_fp32_probe(5, dx.data_ptr(), dx.data_ptr(), out.data_ptr(), len(x), None)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), np.sqrt(x).view(np.uint32))
