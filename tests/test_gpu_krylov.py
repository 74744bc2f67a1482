"""The Krylov option of the linear solves (krylov_m > 0: flexible GMRES preconditioned by
one V-cycle) on the GPU against the oracle's, step by step: the same status and, when
both converge, ||x_gpu - x_oracle||_inf / ||x_oracle||_inf <= 1e-10 for s and for c,
in FP64 and in mixed precision, in 2-D and 3-D, with restarts, under the paper's
W-cycle, with Neumann rows, and on a creased union
of ellipsoids where plain cycles need ten times as many cycles.  Batches refuse
members with the option."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
import oracle
from _gpu import cuda, host, oracle_params, pair, rel, say
from paper_1902_07029_amd import lsmg

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _steps(H, O, n, dim, dt, steps, label):
    info = O.level_info(0)
    na = info["na"]
    s0, c0 = I.initial_state(n, dim)
    W = O.to_compact(0, s0, c0)
    st = lsmg.State(H)
    st.set_grid(cuda(s0), cuda(c0))
    sb = np.ones(info["ng"])
    counts = []
    for k in range(steps):
        rc, gs = st.step(dt, check=False)
        orc, W, os_ = O.newton_cn_step(W, dt, sb)
        assert rc == orc == 0, (label, k, rc, orc)
        G = host(st.get())
        e = max(rel(G[:na], W[:na]), rel(G[na:], W[na:]))
        say(f"{label} step {k}: err {e:.2e} newton {gs['newton_iters']}/{os_['newton_iters']} "
            f"cycles {gs['vcycles']}/{os_['vcycles']}")
        assert e <= TOL, (label, k, e)
        counts.append(gs["vcycles"])
    return counts


@pytest.mark.parametrize("kind,n,coarsest,precision,m,extra", [
    ("disk", 65, 5, 0, 30, {}), ("star", 129, 9, 1, 30, {}), ("star", 129, 9, 0, 3, {}), ("torus", 33, 9, 0, 20, {}),
    ("torus", 65, 9, 1, 4, {}), ("star", 65, 9, 1, 10, dict(cycle_gamma=2)), ("disk", 65, 5, 0, 20, dict(bc=1)),
    ("torus", 33, 9, 1, 20, dict(bc=1))])
def test_krylov_steps_match_oracle(kind, n, coarsest, precision, m, extra):
    # also with the paper's W-cycle as the preconditioner, and with Neumann rows
    label = f"krylov m={m} {kind} {n} precision {precision} {extra}"
    say(label)
    H, O = pair(kind, n, coarsest, precision=precision, krylov_m=m, **extra)
    _steps(H, O, n, 2 if kind != "torus" else 3, 1e-4, 3, label)


@pytest.mark.parametrize("precision", [0, 1])
def test_krylov_on_a_creased_union(precision):
    # request 10 of the served stream on its plain (creased) union at 65^3: plain
    # cycles need about 212 per step, the Krylov solves about 20
    r = [q for q in I.serving_requests(24, seed=0) if q["id"] == 10][0]
    n = r["n"]
    label = f"krylov creased union, request 10 (65^3), precision {precision}"
    say(label)
    phi = I.ellipsoids(n, r["centres"], r["semi"], smooth=0.0)
    H = lsmg.Hierarchy(torch.from_numpy(phi), 3, n,
                       params=lsmg.default_params(coarsest_n=9, precision=precision, krylov_m=30))
    O = oracle.Hierarchy(phi, 3, n, coarsest_n=9, params=oracle_params(H.params))
    counts = _steps(H, O, n, 3, r["dt"], 2, label)
    assert max(counts) <= 40, counts


def test_batch_refuses_krylov_members():
    n = 33
    Hs = [lsmg.Hierarchy(torch.from_numpy(I.star(n)), 2, n, params=lsmg.default_params(coarsest_n=5, krylov_m=10)),
          lsmg.Hierarchy(torch.from_numpy(I.disk(n)), 2, n, params=lsmg.default_params(coarsest_n=5, krylov_m=10))]
    with pytest.raises(lsmg.LsmgError) as e:
        lsmg.Batch(Hs)
    assert e.value.code == lsmg.ENOTIMPL
