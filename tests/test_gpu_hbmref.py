"""GPU checks of the streaming reference kernels (include/couple_hbmref.h), the
HBM ceiling the coupling kernels are measured against: the copy reproduces its
source bit for bit, the write fills every element, the read (a scan for
non-finite values) flags a buffer exactly when it holds a NaN or an infinity,
wherever it sits, on sizes with a ragged last workgroup."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_11834_amd as cpl
    return torch, cpl


@pytest.mark.parametrize("n16", [1, 63, 255, 256, 257, 100_003])
def test_copy_write_read(env, n16):
    torch, cpl = env
    print(f"case hbmref n16={n16}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(n16)
    src = torch.randn(4 * n16, generator=g, device="cuda") * 1e30
    dst = torch.full_like(src, float("nan"))
    cpl.hbmref(cpl.COUPLE_HBMREF_COPY, src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    cpl.hbmref(cpl.COUPLE_HBMREF_WRITE, None, dst, value=-2.5)
    torch.cuda.synchronize()
    assert bool((dst == -2.5).all())
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    cpl.hbmref(cpl.COUPLE_HBMREF_READ, src, flag)            # large finite values only
    torch.cuda.synchronize()
    assert int(flag) == 0
    for pos, bad in ((0, float("nan")), (4 * n16 - 1, float("inf")), ((4 * n16) // 2, float("-inf"))):
        x = src.clone()
        x[pos] = bad
        flag.zero_()
        cpl.hbmref(cpl.COUPLE_HBMREF_READ, x, flag)
        torch.cuda.synchronize()
        assert int(flag) == 1, (pos, bad)


def test_argument_checks(env):
    torch, cpl = env
    a = torch.zeros(16, device="cuda")
    with pytest.raises(ValueError):
        cpl.hbmref(cpl.COUPLE_HBMREF_COPY, a, torch.zeros(12, device="cuda"))        # size mismatch
    with pytest.raises(ValueError):
        cpl.hbmref(cpl.COUPLE_HBMREF_COPY, a, torch.zeros(16, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        cpl.hbmref(cpl.COUPLE_HBMREF_READ, a, torch.zeros(1, device="cuda"))         # the flag is int32
    with pytest.raises(ValueError):
        cpl.hbmref(7, a, a)
