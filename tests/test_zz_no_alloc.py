"""The allocation-free re-initialisation (lsmg_reinitialize_noalloc) against the
allocating entry point (lsmg_reinitialize): the same kernels on scratch from a
fixed device array instead of hipMalloc, so the same bits.  Two calls in a row,
the second on a smaller grid, then the first again; a grid beyond the scratch
is refused before any GPU work."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I

pytestmark = pytest.mark.gpu


def _ellipse(n):
    # a level set that is not a distance function: its zero set is an ellipse
    x, y = I.grid_points(n, 2)
    return (x / 0.6) ** 2 + (y / 0.35) ** 2 - 1.0


def _ellipsoid(n):
    x, y, z = I.grid_points(n, 3)
    return (x / 0.6) ** 2 + (y / 0.4) ** 2 + (z / 0.5) ** 2 - 1.0


def test_noalloc_reinitialize_equals_allocating_one():
    from paper_1902_07029_amd import lsmg
    cases = [(2, 1025, _ellipse(1025), 60), (3, 65, _ellipsoid(65), 40), (2, 1025, _ellipse(1025), 60)]
    for dim, n, phi, iters in cases:
        print(f"no-alloc reinitialisation dim={dim} n={n} iterations={iters}", flush=True)
        p0 = torch.from_numpy(phi).cuda()
        a = p0.clone()
        b = p0.clone()
        lsmg.reinitialize(a, dim, n, iters)
        lsmg.reinitialize_noalloc(b, dim, n, iters)
        torch.cuda.synchronize()
        assert not torch.equal(b, p0)
        assert torch.equal(a, b)


def test_noalloc_reinitialize_refuses_grids_beyond_its_scratch():
    from paper_1902_07029_amd import lsmg
    n = 2049   # 4.2 M nodes > 2^21
    phi = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    with pytest.raises(lsmg.LsmgError) as e:
        lsmg.reinitialize_noalloc(phi, 2, n, 5)
    assert e.value.code == lsmg.EINVAL
    assert torch.count_nonzero(phi).item() == 0
