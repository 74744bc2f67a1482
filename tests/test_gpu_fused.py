"""The fused 2-D sweep (both colours of a smoothing sweep in one launch over tiles of
rows, the red half-sweep recomputed on a one-node halo, the corrections alternating
between two copies) against one launch per colour: both apply the same row
arithmetic to the same values, so smoothing sweeps, cycles and whole steps must agree
bit for bit.  Covered: odd sweep counts (the last step per colour), V- and W-cycles,
Dirichlet and Neumann rows, FP64 and mixed precision, grids whose rows are not a
multiple of the 64-position tile width, and a disc reaching the nodes next to the box
edge (tiles on the edge rows and positions).  Where a launch moves more than 1 MiB
of node values the fused sweep is not used (lsmg_sweep_fused)."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
from _gpu import cuda, pair, random_state, say
from paper_1902_07029_amd import lsmg


def _both(kind, n, coarsest, phi=None, **params):
    Hu, O = pair(kind, n, coarsest, phi=phi, fused_sweep=0, **params)
    Hf, _ = pair(kind, n, coarsest, phi=phi, **params)
    assert Hu.params.fused_sweep == 0 and Hf.params.fused_sweep == 1
    return Hu, Hf, O


# (kind, n, coarsest, levelset override, params)
CASES = [("disk", 65, 5, None, {}), ("star", 257, 9, None, {}), ("star", 1025, 9, None, {}),
         ("star", 257, 9, None, dict(bc=1)), ("paper3", 257, 9, None, dict(nu1=2, nu2=1, cycle_gamma=2)),
         ("disk", 129, 5, "edge", {}), ("star", 129, 9, None, dict(nu1=3, nu2=3))]


def _phi(kind, n, override):
    # a disc of radius 0.99 in [-1, 1]^2: inside nodes on the rows and columns next to the box edge
    return I.disk(n, r=0.99) if override == "edge" else None


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,override,params", CASES)
def test_fused_sweep_cycles_bitwise(kind, n, coarsest, override, params):
    say(f"fused sweep cycles {kind} n={n} {override} {params}")
    Hu, Hf, O = _both(kind, n, coarsest, phi=_phi(kind, n, override), **params)
    rng = np.random.default_rng(11)
    W = random_state(O, 0, rng)
    na = O.level_info(0)["na"]
    rhs = cuda(rng.standard_normal(2 * na))
    out = []
    for H in (Hu, Hf):
        H.set_linearization(cuda(W), 1e-3)
        x = cuda(np.zeros(2 * na))
        norms = []
        for _ in range(3):
            x, r = H.vcycle(0, rhs, x)
            norms.append(r)
        out.append((x, norms))
    say(f"  residuals {out[1][1]}")
    assert torch.equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,override", [("star", 257, 9, None), ("disk", 129, 5, "edge")])
@pytest.mark.parametrize("nsweeps", [1, 2, 3, 4])
def test_fused_sweep_smoothing_bitwise(kind, n, coarsest, override, nsweeps):
    Hu, Hf, O = _both(kind, n, coarsest, phi=_phi(kind, n, override))
    rng = np.random.default_rng(5)
    W = random_state(O, 0, rng)
    for level in (0, 1):
        na = O.level_info(level)["na"]
        rhs = cuda(rng.standard_normal(2 * na))
        x0 = cuda(rng.standard_normal(2 * na))
        got = []
        for H in (Hu, Hf):
            H.set_linearization(cuda(W), 1e-3)
            got.append(H.smooth(level, rhs, x0.clone(), nsweeps))
        assert torch.equal(got[0], got[1]), (level, nsweeps)


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,precision,params",
                         [("star", 257, 9, 1, {}), ("star", 513, 9, 0, dict(bc=1)), ("star", 1025, 9, 0, {})])
def test_fused_sweep_steps_bitwise(kind, n, coarsest, precision, params):
    Hu, Hf, _ = _both(kind, n, coarsest, precision=precision, **params)
    states = []
    for H in (Hu, Hf):
        st = lsmg.State(H)
        s, c = I.initial_state(n, 2)
        st.set_grid(cuda(s), cuda(c))
        stats = [st.step(1e-4)[1] for _ in range(2)]
        states.append((st.get(), [(x["newton_iters"], x["vcycles"]) for x in stats]))
    say(f"fused sweep steps {kind} n={n} prec {precision}: (newton, cycles) {states[1][1]}")
    assert torch.equal(states[0][0], states[1][0])
    assert states[0][1] == states[1][1]


@pytest.mark.gpu
def test_fused_sweep_switch_by_set_params():
    # the same hierarchy stepped with fused sweeps, then switched off through
    # lsmg_set_params (the captured cycles are rebuilt), against a reference without
    n = 257
    Hu, Hf, _ = _both("star", n, 9)
    sts = []
    for H in (Hu, Hf):
        st = lsmg.State(H)
        s, c = I.initial_state(n, 2)
        st.set_grid(cuda(s), cuda(c))
        sts.append(st)
    sts[0].step(1e-4)
    sts[1].step(1e-4)
    p = Hf.params
    p.fused_sweep = 0
    Hf.set_params(p)
    assert Hf.params.fused_sweep == 0
    sts[0].step(1e-4)
    sts[1].step(1e-4)
    assert torch.equal(sts[0].get(), sts[1].get())


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_fused_sweep_batch_bitwise(precision):
    # a batch of stars of three grid sizes with fused sweeps against the same batch with
    # one launch per colour
    doms = [dict(n=129, a=0.45, b=0.1, k=4, p=0.3), dict(n=257, a=0.5, b=0.15, k=5, p=0.0),
            dict(n=65, a=0.55, b=0.08, k=3, p=1.0), dict(n=257, a=0.38, b=0.18, k=7, p=2.5)]
    out = []
    for fused in (0, 1):
        Hs, sts = [], []
        for d in doms:
            p = lsmg.default_params(coarsest_n=9, precision=precision, fused_sweep=fused)
            H = lsmg.Hierarchy(torch.from_numpy(I.star(d["n"], d["a"], d["b"], d["k"], d["p"])), 2, d["n"], params=p)
            st = lsmg.State(H)
            s, c = I.initial_state(d["n"], 2)
            st.set_grid(cuda(s), cuda(c))
            Hs.append(H)
            sts.append(st)
        B = lsmg.Batch(Hs)
        stats = []
        for _ in range(2):
            status, st_ = B.step(sts, 1e-4)
            assert all(x == lsmg.OK for x in status)
            stats.append([(x["newton_iters"], x["vcycles"]) for x in st_])
        out.append(([st.get() for st in sts], stats))
    say(f"fused batch prec {precision}: (newton, cycles) {out[1][1]}")
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)
    assert out[0][1] == out[1][1]


@pytest.mark.gpu
def test_sweep_fused_rule():
    # fused where active nodes x value size <= 1 MiB: the 1025^2 star level (217 k active
    # nodes) runs one launch per colour in FP64 and fused in FP32; coarser levels fused
    p = lsmg.default_params(coarsest_n=9, precision=1)
    H = lsmg.Hierarchy(torch.from_numpy(I.star(1025)), 2, 1025, params=p)
    na = H.level_info(0)["na"]
    assert na * 8 > (1 << 20) >= na * 4
    assert not H.sweep_fused(0, 0) and H.sweep_fused(0, 1)
    assert all(H.sweep_fused(l, 0) for l in range(1, H.nlev))
    q = lsmg.default_params(coarsest_n=9, fused_sweep=0)
    Hu = lsmg.Hierarchy(torch.from_numpy(I.star(257)), 2, 257, params=q)
    assert not any(Hu.sweep_fused(l, 0) for l in range(Hu.nlev))
    T = lsmg.Hierarchy(torch.from_numpy(I.torus(33)), 3, 33, params=lsmg.default_params(coarsest_n=9))
    assert not T.sweep_fused(0, 0)
    B = lsmg.Batch([H, lsmg.Hierarchy(torch.from_numpy(I.star(257)), 2, 257, params=p)])
    assert not B.sweep_fused(1025, 0) and B.sweep_fused(1025, 1) and B.sweep_fused(257, 0)
    assert not B.sweep_fused(1000, 0)
