"""The measurement kernels (include/wmd_bench.h) compute what they claim, so
the ceilings bench.py reports come from kernels that did their reads."""
import numpy as np
import pytest
import torch

from paper_2107_06433_amd import wmd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S", [4, 8, 12, 20, 32, 100, 512])
def test_gather_sums_the_named_rows(S):
    lib = wmd.lib()
    rng = np.random.default_rng(S)
    U, nids = 777, 5003  # not a multiple of any pass size
    table = torch.from_numpy(rng.standard_normal(U * S).astype(np.float32)).cuda()
    ids = torch.from_numpy(rng.integers(0, U, nids).astype(np.int32)).cuda()
    out = torch.full((nids,), float("nan"), dtype=torch.float32, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    for blocks in (1, 7, 64):
        out.fill_(float("nan"))
        assert lib.wmd_bench_gather(table.data_ptr(), S, ids.data_ptr(), nids, out.data_ptr(), blocks, sh) == 0
        torch.cuda.synchronize()
        ref = table.cpu().double().view(U, S)[ids.cpu().long()].sum(1)
        np.testing.assert_allclose(out.cpu().double().numpy(), ref.numpy(), rtol=1e-5, atol=1e-4 * np.sqrt(S))


def test_stream_copy_and_read():
    lib = wmd.lib()
    n = (1 << 20) + 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    sink = torch.full((1,), 7.0, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    assert lib.wmd_bench_stream(src.data_ptr(), dst.data_ptr(), n * 4, 1, 97, None, sh) == 0
    assert lib.wmd_bench_stream(src.data_ptr(), None, n * 4, 0, 97, sink.data_ptr(), sh) == 0
    assert lib.wmd_bench_tiles(src.data_ptr(), n * 4 // 1280, 1280, sink.data_ptr(), sh) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert sink.item() == 7.0  # written only in a case that cannot occur


def test_valu_modes_finish():
    lib = wmd.lib()
    out = torch.full((4 * 256,), float("nan"), device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    for mode in (0, 1, 2):
        out.fill_(float("nan"))
        assert lib.wmd_bench_valu(out.data_ptr(), 4, 16, mode, sh) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
