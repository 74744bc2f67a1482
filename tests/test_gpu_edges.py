"""Degenerate and boundary cases of the GPU path: domains of one inside node, domains
touching the box edge, empty domains in 2-D and 3-D, an empty member in a batch,
and the argument checks of the boundary (all refused on the host before any GPU
work, or by the build's own classification)."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
from _gpu import cuda, host, pair, rel, say
from paper_1902_07029_amd import lsmg

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _steps(H, O, n, dim, dt, steps):
    info = O.level_info(0)
    na = info["na"]
    s, c = I.initial_state(n, dim)
    W = O.to_compact(0, s, c)
    st = lsmg.State(H)
    st.set(cuda(W))
    sb = np.ones(info["ng"])
    for k in range(steps):
        st.step(dt)
        rc, W, _ = O.newton_cn_step(W, dt, sb)
        assert rc == 0
        G = host(st.get())
        assert rel(G[:na], W[:na]) <= TOL and rel(G[na:], W[na:]) <= TOL, k


@pytest.mark.parametrize("r", [0.05, 0.07])
def test_domain_of_one_or_few_inside_nodes(r):
    # r = 0.05 on a 33^2 grid: one inside node on every level; r = 0.07: five on the finest
    n = 33
    H, O = pair("disk", n, 5, phi=I.disk(n, r=r))
    say(f"tiny disk r={r}: active nodes per level {[O.level_info(l)['na'] for l in range(O.nlev)]}")
    _steps(H, O, n, 2, 1e-3, 3)


def test_domain_next_to_the_box_edge():
    # a disk whose inside nodes reach the last column but one: its ghosts lie on the box edge
    n = 65
    phi = I.disk(n, r=0.12, x0=0.85)
    H, O = pair("disk", n, 5, phi=phi)
    _steps(H, O, n, 2, 1e-3, 3)


def test_inside_node_on_the_box_edge_is_refused():
    n = 33
    with pytest.raises(lsmg.LsmgError) as e:
        lsmg.Hierarchy(torch.from_numpy(-np.ones(n * n)), 2, n, params=lsmg.default_params(coarsest_n=5))
    assert e.value.code == lsmg.EGEOM


def test_bad_grids_are_refused():
    p = lsmg.default_params(coarsest_n=5)
    for dim, n, lo, hi in ((2, 34, -1.0, 1.0), (2, 33, 1.0, -1.0), (4, 17, -1.0, 1.0), (2, 2, -1.0, 1.0)):
        phi = torch.ones(n ** dim, dtype=torch.float64)
        with pytest.raises(lsmg.LsmgError) as e:
            lsmg.Hierarchy(phi, dim, n, lo, hi, params=p)
        assert e.value.code == lsmg.EINVAL, (dim, n, lo, hi)


def test_empty_domain_3d():
    n = 17
    H = lsmg.Hierarchy(torch.ones(n ** 3, dtype=torch.float64), 3, n, params=lsmg.default_params(coarsest_n=5))
    assert H.level_info(0)["na"] == 0
    st = lsmg.State(H)
    rc, stats = st.step(1e-4)
    assert rc == 0


def test_batch_with_an_empty_member():
    n, dt = 129, 1e-4
    p = lsmg.default_params(coarsest_n=9, precision=1)
    Hs = [lsmg.Hierarchy(torch.from_numpy(I.star(n)), 2, n, params=p),
          lsmg.Hierarchy(torch.ones(n * n, dtype=torch.float64), 2, n, params=p)]
    B = lsmg.Batch(Hs)
    sts = []
    for H in Hs:
        st = lsmg.State(H)
        s0, c0 = I.initial_state(n, 2)
        st.set_grid(cuda(s0), cuda(c0))
        sts.append(st)
    alone = lsmg.State(lsmg.Hierarchy(torch.from_numpy(I.star(n)), 2, n, params=p))
    s0, c0 = I.initial_state(n, 2)
    alone.set_grid(cuda(s0), cuda(c0))
    for _ in range(2):
        status, _ = B.step(sts, dt)
        assert status == [0, 0]
        alone.step(dt)
    assert np.array_equal(host(sts[0].get()), host(alone.get()))
    assert sts[1].get().numel() == 0
