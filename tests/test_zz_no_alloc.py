"""The allocation-free banded solve (ctd_kernel_band_solve_noalloc) against
the allocating entry point (ctd_kernel_band_solve) through the C-ABI: the
same kernels, so results must be bitwise equal.  Two calls in a row, the
second smaller, so the shared static workspace is reused with stale data
from the first call; sizes cover block data in LDS, split LDS/workspace and
all-workspace storage.  The oversize request is refused before any launch."""
import numpy as np
import pytest

from oracle.cfe1d import Axis

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_15519_amd import ctd as mod
    return mod


def _system(s, n, count, seed):
    import torch
    ax = Axis(n, 0.0, 1.0, s=s, p=min(s, 2), a=12.0, ng=5)
    Mb, Kb = ax.banded(ax.M), ax.banded(ax.K)
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    return (dev(Mb), dev(Kb), dev(rng.uniform(10.0, 3000.0, count)),
            dev(rng.uniform(1e-6, 1e-2, count)), dev(rng.standard_normal((count, n))))


@pytest.mark.parametrize("big,small", [((2, 2600, 7), (2, 1800, 3)),     # all-workspace, then split
                                       ((3, 1300, 6), (3, 515, 2)),      # split, then LDS only
                                       ((1, 3000, 9), (1, 2900, 4))])    # all-workspace twice
def test_noalloc_equals_allocating(ctd, big, small):
    import torch
    for (s, n, count), seed in ((big, 1), (small, 2)):
        print(f"noalloc band solve s={s} n={n} count={count}", flush=True)
        Mb, Kb, al, be, b = _system(s, n, count, seed)
        x_ref = torch.zeros((count, n), dtype=torch.float64, device="cuda")
        x_na = torch.full((count, n), float("nan"), dtype=torch.float64, device="cuda")
        ctd.band_solve(n, 2 * s + 1, Mb, Kb, al, be, b, x_ref, count)
        ctd.band_solve_noalloc(n, 2 * s + 1, Mb, Kb, al, be, b, x_na, count)
        torch.cuda.synchronize()
        assert torch.equal(x_na, x_ref)


def test_noalloc_refuses_oversize(ctd):
    import torch
    n, s = 4000, 3
    count = 64            # 64 systems of ~0.5 MB block data each: beyond 16 MiB
    Mb, Kb, al, be, b = _system(s, n, count, 3)
    x = torch.zeros((count, n), dtype=torch.float64, device="cuda")
    with pytest.raises(ctd.CtdError) as ei:
        ctd.band_solve_noalloc(n, 2 * s + 1, Mb, Kb, al, be, b, x, count)
    assert "ENOMEM" in str(ei.value)
    torch.cuda.synchronize()
    assert not bool(x.any())
