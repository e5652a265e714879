"""The streaming copy probe (include/probe.h) copies exactly, in both cache
policies, one element per thread and at odd block counts, and rejects bad
arguments on the host."""
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu


def test_probe_copy_is_exact():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import probe
    st = torch.cuda.current_stream().cuda_stream
    n = (1 << 22) + 192                                # bytes: not a multiple of the grid
    src = torch.randint(0, 1 << 30, (n // 4,), dtype=torch.int32, device="cuda")
    for nt in (False, True):
        for blocks in (0, 1, 7, 4096):
            say(f"[probe] copy {n} B nontemporal={nt} blocks={blocks}")
            dst = torch.zeros_like(src)
            probe.probe_copy(src, dst, n, nt, blocks, st)
            torch.cuda.synchronize()
            assert torch.equal(src, dst)
    with pytest.raises(RuntimeError):
        probe.probe_copy(src, src, n, False, 8, st)   # overlapping ranges
    with pytest.raises(RuntimeError):
        probe.probe_copy(src, dst, n - 16, False, 8, st)  # not a multiple of 64
    with pytest.raises(RuntimeError):
        probe.probe_copy(src, dst, n, False, -1, st)  # negative block count
