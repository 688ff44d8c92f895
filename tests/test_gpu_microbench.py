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
