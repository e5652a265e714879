"""sur_checks_noalloc (the per-window checks for callers that cannot
allocate device memory) against sur_checks with a caller's scratch, through
the C ABI: the same seven FP64 results bit for bit, on two calls in a row,
the second on a smaller state (so the shared buffer holds the first call's
partials when the second runs), and sizes beyond the buffer rejected."""
import numpy as np
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import surrogate
    surrogate.load_library()
    return surrogate


def _state(torch, grid, seed):
    nx, ny, nz = grid
    rng = np.random.default_rng(seed)
    s = np.zeros((nx * ny * nz, 16), dtype=np.float32)
    s[:, 0] = rng.uniform(-0.1, 1.1, nx * ny * nz)
    s[:, 1:5] = rng.standard_normal((nx * ny * nz, 4))
    return torch.as_tensor(s).cuda()


def _with_scratch(sur, torch, st, grid):
    P = grid[0] * grid[1] * grid[2]
    scr = torch.empty(7 * (P // 256 + 1), dtype=torch.float64, device="cuda")
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    sur.sur_checks(st, grid, scr, out)
    return out.cpu().numpy()


def _noalloc(sur, torch, st, grid):
    out = torch.full((7,), np.nan, dtype=torch.float64, device="cuda")
    sur.sur_checks_noalloc(st, grid, out)
    return out.cpu().numpy()


def test_noalloc_checks_equal_scratch_checks_twice(sur):
    import torch
    for grid, seed in (((128, 128, 128), 1), ((40, 24, 18), 2)):
        say(f"[noalloc] sur_checks_noalloc on {grid}")
        st = _state(torch, grid, seed)
        a = _noalloc(sur, torch, st, grid)
        b = _with_scratch(sur, torch, st, grid)
        say(f"   {a.tolist()}")
        assert np.array_equal(a, b), (a, b)
        assert a[5] == grid[0] * grid[1] * grid[2]


def test_noalloc_checks_at_the_size_limit_and_beyond(sur):
    import torch
    grid = (256, 128, 128)                     # exactly the maximum, 2^22 points
    say(f"[noalloc] sur_checks_noalloc at the limit {grid}")
    st = _state(torch, grid, 3)
    assert np.array_equal(_noalloc(sur, torch, st, grid), _with_scratch(sur, torch, st, grid))
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        sur.sur_checks_noalloc(st, (256, 128, 129), out)   # one plane too many: rejected
    assert sur.CHECKS_NOALLOC_MAX_POINTS == 256 * 128 * 128
