"""The caller's allocator at the boundary (lsmg_allocator): a hierarchy, its state
and a batch built with torch's caching allocator hold their buffers in torch's
pool (torch.cuda.memory_allocated counts them) and hand them back when
destroyed; results do not depend on where the memory comes from."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I

pytestmark = pytest.mark.gpu


def _mb(x):
    return x / 2 ** 20


def test_hierarchy_bytes_live_in_torch_pool():
    from paper_1902_07029_amd import lsmg
    from tests._gpu import say
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    n = 257
    H = lsmg.Hierarchy(torch.from_numpy(I.star(n)), 2, n, params=lsmg.default_params(coarsest_n=9, precision=1))
    torch.cuda.synchronize()
    hb, sb = H.memory_bytes()
    held = torch.cuda.memory_allocated() - base
    say(f"star {n}^2 mixed: hierarchy {_mb(hb):.2f} MiB, torch pool grew {_mb(held):.2f} MiB")
    # every buffer rounded up to torch's 512-byte blocks; the phi copy made by the binding is freed
    assert hb <= held <= 1.1 * hb + (1 << 20)
    st = lsmg.State(H)
    torch.cuda.synchronize()
    held2 = torch.cuda.memory_allocated() - base
    assert sb <= held2 - held <= sb + 4096
    st.close()
    H.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_step_and_batch_same_bits_with_either_allocator():
    from paper_1902_07029_amd import lsmg
    n, dt = 129, 1e-4
    phi = torch.from_numpy(I.star(n))
    out = []
    for alloc in ("torch", None):
        p = lsmg.default_params(coarsest_n=9, precision=1)
        H = lsmg.Hierarchy(phi, 2, n, params=p, allocator=alloc)
        H2 = lsmg.Hierarchy(torch.from_numpy(I.star(n, 0.45, 0.1, 3, 0.5)), 2, n, params=p, allocator=alloc)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        B = lsmg.Batch([H, H2], allocator=alloc)
        torch.cuda.synchronize()
        grew = torch.cuda.memory_allocated() - before
        if alloc == "torch":
            assert grew > 0, "batch buffers must come from torch's pool"
        else:
            assert grew == 0
        sts = []
        for h in (H, H2):
            st = lsmg.State(h)
            s0, c0 = I.initial_state(n, 2)
            st.set_grid(torch.from_numpy(s0).cuda(), torch.from_numpy(c0).cuda())
            sts.append(st)
        for _ in range(2):
            B.step(sts, dt)
        single = lsmg.State(H)
        s0, c0 = I.initial_state(n, 2)
        single.set_grid(torch.from_numpy(s0).cuda(), torch.from_numpy(c0).cuda())
        for _ in range(2):
            single.step(dt)
        out.append([st.get().cpu().numpy() for st in sts] + [single.get().cpu().numpy()])
        B.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(out[0][0], out[0][2])
