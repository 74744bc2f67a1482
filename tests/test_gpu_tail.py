"""The coarse tail held in LDS against the same tail read from HBM (hierarchies built
with LSMG_TAIL_LDS=0): the two apply the same row arithmetic to the same values in the
same order, and on these shapes whole cycles and whole steps agree bit for bit.  V- and
W-cycles, 2-D and 3-D, Dirichlet and Neumann rows, FP64 and mixed precision, single
hierarchies and a batch.  (Compiled separately, the two kernels may pair a product
with an addition differently somewhere; a batch therefore runs each member's tail in
the kernel the member runs alone, which the last test checks.)"""
import os

import numpy as np
import pytest
import torch

import lsmg_inputs as I
from _gpu import cuda, pair, random_state, say
from paper_1902_07029_amd import lsmg


def _both(kind, n, coarsest, **params):
    os.environ["LSMG_TAIL_LDS"] = "0"
    try:
        Hh, O = pair(kind, n, coarsest, **params)
    finally:
        del os.environ["LSMG_TAIL_LDS"]
    Hl, _ = pair(kind, n, coarsest, **params)
    assert not Hh.tail_in_lds(0) and not Hh.tail_in_lds(1)
    return Hh, Hl, O


CASES = [("disk", 65, 5, {}), ("star", 257, 9, {}), ("star", 1025, 9, {}), ("star", 257, 9, dict(bc=1)),
         ("paper3", 257, 9, dict(nu1=2, nu2=1, cycle_gamma=2)), ("torus", 65, 9, {}), ("torus", 33, 5, dict(bc=1)),
         ("torus", 257, 9, {})]


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,params", CASES)
def test_tail_in_lds_cycles_bitwise(kind, n, coarsest, params):
    say(f"LDS tail cycles {kind} n={n} {params}")
    Hh, Hl, O = _both(kind, n, coarsest, **params)
    assert Hl.tail_in_lds(0), "the tail of this domain should fit in LDS"
    rng = np.random.default_rng(4)
    W = random_state(O, 0, rng)
    na = O.level_info(0)["na"]
    rhs = cuda(rng.standard_normal(2 * na))
    xs = []
    for H in (Hh, Hl):
        H.set_linearization(cuda(W), 1e-3)
        x = cuda(np.zeros(2 * na))
        norms = []
        for _ in range(3):
            x, r = H.vcycle(0, rhs, x)
            norms.append(r)
        xs.append((x, norms))
    assert torch.equal(xs[0][0], xs[1][0])
    assert xs[0][1] == xs[1][1]


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,precision,params",
                         [("star", 257, 9, 1, {}), ("torus", 65, 9, 1, {}), ("star", 513, 9, 0, dict(bc=1))])
def test_tail_in_lds_steps_bitwise(kind, n, coarsest, precision, params):
    Hh, Hl, O = _both(kind, n, coarsest, precision=precision, **params)
    assert Hl.tail_in_lds(precision)
    states = []
    for H in (Hh, Hl):
        st = lsmg.State(H)
        s, c = I.initial_state(n, H.dim)
        st.set_grid(cuda(s), cuda(c))
        stats = [st.step(1e-4)[1] for _ in range(2)]
        states.append((st.get(), [(x["newton_iters"], x["vcycles"]) for x in stats]))
    say(f"LDS tail steps {kind} n={n} prec {precision}: (newton, cycles) {states[1][1]}")
    assert torch.equal(states[0][0], states[1][0])
    assert states[0][1] == states[1][1]


@pytest.mark.gpu
def test_tail_in_lds_batch_bitwise():
    doms = [dict(n=129, a=0.45, b=0.1, k=4, p=0.3), dict(n=257, a=0.5, b=0.15, k=5, p=0.0),
            dict(n=65, a=0.55, b=0.08, k=3, p=1.0)]
    out = []
    for lds in ("0", None):
        if lds is not None:
            os.environ["LSMG_TAIL_LDS"] = lds
        try:
            Hs = [lsmg.Hierarchy(torch.from_numpy(I.star(d["n"], d["a"], d["b"], d["k"], d["p"])), 2, d["n"],
                                 params=lsmg.default_params(coarsest_n=9, precision=1)) for d in doms]
        finally:
            os.environ.pop("LSMG_TAIL_LDS", None)
        assert all(H.tail_in_lds(1) == (lds is None) for H in Hs)
        sts = []
        for H, d in zip(Hs, doms):
            st = lsmg.State(H)
            s, c = I.initial_state(d["n"], 2)
            st.set_grid(cuda(s), cuda(c))
            sts.append(st)
        B = lsmg.Batch(Hs)
        for _ in range(2):
            status, _ = B.step(sts, 1e-4)
            assert all(x == lsmg.OK for x in status)
        out.append([st.get() for st in sts])
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.gpu
def test_batch_members_run_their_own_tail_kind():
    # the 3-D domains of the serving test (unions of ellipsoids, 33^3 and 65^3, mixed
    # precision): one member's tail does not fit LDS, the others' do; each member runs in
    # the batch the tail kernel it runs alone (the two kernels agree only to rounding on
    # some of these domains), so the batch equals stepping alone bit for bit
    from test_gpu_serve import _requests
    params = lsmg.default_params(coarsest_n=9, precision=1)
    reqs = _requests(6, 3, steps=(8, 15), gap=0.01)

    def hier(r):
        return lsmg.Hierarchy(torch.from_numpy(r.phi), r.dim, r.n, params=params)

    def state(H, r):
        st = lsmg.State(H)
        nn = r.n ** r.dim
        st.set_grid(torch.full((nn,), r.s0, dtype=torch.float64, device="cuda"),
                    torch.full((nn,), r.c0, dtype=torch.float64, device="cuda"))
        return st

    alone = [(hier(r), r) for r in reqs]
    kinds = [H.tail_in_lds(1) for H, _ in alone]
    assert any(kinds) and not all(kinds), kinds
    ref = []
    for H, r in alone:
        st = state(H, r)
        for _ in range(3):
            st.step(r.dt, sb_const=r.sb)
        ref.append(st.get())
    Hs = [hier(r) for r in reqs]
    sts = [state(H, r) for H, r in zip(Hs, reqs)]
    B = lsmg.Batch(Hs)
    for _ in range(3):
        status, _ = B.step(sts, reqs[0].dt, sb_const=[r.sb for r in reqs])
        assert all(x == lsmg.OK for x in status)
    say(f"tail kinds (LDS) per member: {kinds}")
    for k in range(len(reqs)):
        assert torch.equal(sts[k].get(), ref[k]), k
