"""The measurement helpers behind the measured peaks: the streaming copy copies, and the FMA chains compute
their closed form (x <- x + 1 from x = 0..7 gives 28 + 8 iters per thread, exactly in FP32)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge
    lodge.lib()
    return lodge


@pytest.mark.parametrize("n", [4, 4 * 1000 + 4, 1 << 22])
def test_stream_copy(L, n):
    import torch
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    L.lodge_microbench_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_fma_chains_closed_form_and_arguments(L):
    import torch
    out = torch.zeros(4 * 256, dtype=torch.float32, device="cuda")
    ops = L.lodge_microbench_fma(out, 1000)
    torch.cuda.synchronize()
    assert ops == 8 * 1000 * 4 * 256
    assert bool((out == 28.0 + 8 * 1000).all())
    with pytest.raises(ValueError):
        L.lodge_microbench_fma(torch.zeros(100, device="cuda"), 10)
    odd = torch.zeros(5, dtype=torch.float32, device="cuda")   # 20 bytes: not a multiple of 16
    with pytest.raises(L.LodgeError):
        L.lodge_microbench_copy(odd, torch.zeros_like(odd))


def test_stream_read_sums_what_it_reads(L):
    import torch
    src = torch.ones(1 << 22, dtype=torch.float32, device="cuda")
    sums = L.lodge_microbench_read(src)
    torch.cuda.synchronize()
    assert float(sums.double().sum()) == float(src.numel())


def test_fp32_division_and_sqrt_are_correctly_rounded(L):
    """The bit-exact stages (selection bounds, rectangles, depth keys) assume the device's FP32 division and
    square root round correctly, as the host's IEEE ones do: 1.0e8 random operands (random signs and
    mantissas, exponents in [-60, 60], so no result is subnormal or overflows), every quotient and root
    equal bit for bit to numpy's."""
    import numpy as np
    import torch
    rng = np.random.default_rng(2505)
    n = 1 << 24
    mism_q = mism_r = 0
    for chunk in range(6):
        def draw():
            exp = rng.integers(127 - 60, 127 + 61, size=n, dtype=np.uint32)
            man = rng.integers(0, 1 << 23, size=n, dtype=np.uint32)
            sgn = rng.integers(0, 2, size=n, dtype=np.uint32)
            return ((sgn << 31) | (exp << 23) | man).view(np.float32)
        a, b = draw(), draw()
        da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        dq, dr = torch.empty_like(da), torch.empty_like(da)
        L.lodge_fp32_div_sqrt(da, db, dq, dr)
        q_ref = a / b
        with np.errstate(invalid="ignore"):
            r_ref = np.sqrt(a)
        q, r = dq.cpu().numpy(), dr.cpu().numpy()
        mism_q += int(np.count_nonzero(q.view(np.uint32) != q_ref.view(np.uint32)))
        neg = a < 0   # sqrt of a negative operand: NaN on both sides (payloads may differ)
        ok_r = (r.view(np.uint32) == r_ref.view(np.uint32)) | (neg & np.isnan(r) & np.isnan(r_ref))
        mism_r += int(np.count_nonzero(~ok_r))
    assert mism_q == 0 and mism_r == 0, (mism_q, mism_r)
