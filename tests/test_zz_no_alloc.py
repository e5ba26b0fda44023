"""The allocation-free scan (mgs_scan_noalloc, the library's fixed per-GPU
scratch) against mgs_scan (caller scratch) through the C ABI: bit for bit on
two calls in a row, the second with a smaller input, at the largest size it
serves, on an empty input, and refused beyond that size."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _scan(M, ctx, x, noalloc):
    out = torch.full_like(x, -1)
    total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    if noalloc:
        M.mgs_scan_noalloc(ctx, x, out, total)
    else:
        M.mgs_scan(ctx, x, out, total)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), int(total.item())


def test_noalloc_scan_equals_scan():
    from paper_2412_20522_amd import maskgs as M
    ctx = M.mgs_create(0)
    try:
        rng = np.random.default_rng(77)
        for n in (5_000_001, 123_457, M.SCAN_NOALLOC_MAX_N, 1, 4097):
            h = rng.integers(0, 100, n).astype(np.int32)
            x = torch.from_numpy(h).cuda()
            a, ta = _scan(M, ctx, x, True)
            b, tb = _scan(M, ctx, x, False)
            assert np.array_equal(a, b), n
            assert ta == tb == int(h.astype(np.int64).sum()), n
            want = np.zeros(n, np.uint64)
            np.cumsum(h[:-1].astype(np.uint64), out=want[1:])
            assert np.array_equal(a, want.astype(np.uint32)), n
        # an empty input: total 0, nothing written
        empty = torch.zeros(0, dtype=torch.int32, device="cuda")
        total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        M.mgs_scan_noalloc(ctx, empty, empty, total)
        torch.cuda.synchronize()
        assert int(total.item()) == 0
        # beyond the fixed scratch: refused on the host, nothing launched
        big = torch.zeros(M.SCAN_NOALLOC_MAX_N + 1, dtype=torch.int32, device="cuda")
        out = torch.empty_like(big)
        with pytest.raises(M.MaskGSError) as e:
            M.mgs_scan_noalloc(ctx, big, out)
        assert e.value.status == 1
        assert "exceeds" in str(e.value)
    finally:
        M.mgs_destroy(ctx)
