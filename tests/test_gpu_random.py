"""Seeded random configurations stepped on the GPU beside the oracle, each on its own
inputs: 2-D star domains of random shape, size, time step, precision and boundary rows
(Dirichlet or Neumann), 3-D unions of random ellipsoids, and a batch of random stars of
different sizes.  After every Crank-Nicolson step the two sides must end with the same
status and, when both converged, ||x_gpu - x_oracle||_inf / ||x_oracle||_inf <= 1e-10 for
s and for c over the active nodes.  Each case prints its draws before any GPU work."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
import oracle
from _gpu import cuda, host, oracle_params, pair, rel, say
from paper_1902_07029_amd import lsmg

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _star_draw(rng):
    return dict(a=float(rng.uniform(0.35, 0.6)), b=float(rng.uniform(0.03, 0.2)), k=int(rng.integers(2, 9)),
                p=float(rng.uniform(0.0, 2.0 * np.pi)))


def _step_both(H, O, n, dim, dt, steps, label, flux=1.0):
    info = O.level_info(0)
    na = info["na"]
    s0, c0 = I.initial_state(n, dim)
    W = O.to_compact(0, s0, c0)
    st = lsmg.State(H)
    st.set_grid(cuda(s0), cuda(c0))
    sb = np.full(info["ng"], flux)
    for k in range(steps):
        rc, gs = st.step(dt, sb_const=flux, check=False)
        orc, W, os_ = O.newton_cn_step(W, dt, sb)
        assert rc == orc, (label, k, rc, orc)
        if orc != 0:
            say(f"{label} step {k}: both sides end with status {orc}")
            return
        G = host(st.get())
        e = max(rel(G[:na], W[:na]), rel(G[na:], W[na:]))
        say(f"{label} step {k}: err {e:.2e} newton {gs['newton_iters']}/{os_['newton_iters']} "
            f"cycles {gs['vcycles']}/{os_['vcycles']}")
        assert e <= TOL, (label, k, e)


@pytest.mark.parametrize("seed", range(5))
def test_random_star(seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.choice([33, 65, 129]))
    shape = _star_draw(rng)
    dt = float(rng.choice([1e-4, 1e-3, 2.0 / (n - 1)]))
    precision = int(rng.integers(0, 2))
    bc = int(rng.integers(0, 2))
    coarsest = 5 if n == 33 else 9
    label = f"random star {seed}: n={n} {shape} dt={dt:.3g} precision={precision} bc={bc}"
    say(label)
    H, O = pair("star", n, coarsest, phi=I.star(n, **shape), precision=precision, bc=bc)
    _step_both(H, O, n, 2, dt, 3, label)


@pytest.mark.parametrize("seed", range(2))
def test_random_ellipsoid_union(seed):
    rng = np.random.default_rng(7100 + seed)
    n = int(rng.choice([33, 65]))
    m = int(rng.integers(1, 4))
    centres = [tuple(float(v) for v in rng.uniform(-0.4, 0.4, 3)) for _ in range(m)]
    semi = [tuple(float(v) for v in rng.uniform(0.15, 0.4, 3)) for _ in range(m)]
    precision = int(rng.integers(0, 2))
    label = f"random ellipsoids {seed}: n={n} m={m} precision={precision}"
    say(label)
    phi = I.ellipsoids(n, centres, semi)
    H = lsmg.Hierarchy(torch.from_numpy(phi), 3, n, params=lsmg.default_params(coarsest_n=9, precision=precision))
    O = oracle.Hierarchy(phi, 3, n, coarsest_n=9, params=oracle_params(H.params))
    _step_both(H, O, n, 3, 1e-4, 2, label)


def test_random_batch():
    rng = np.random.default_rng(7200)
    sizes = [129, 33, 65]
    shapes = [_star_draw(rng) for _ in sizes]
    dt = 1e-4
    say(f"random batch: sizes {sizes} shapes {shapes}")
    Hs, Os, sts, Ws = [], [], [], []
    for n, sh in zip(sizes, shapes):
        phi = I.star(n, **sh)
        # batch members share their parameters: a 9 x 9 coarsest grid for every size
        H = lsmg.Hierarchy(torch.from_numpy(phi), 2, n, params=lsmg.default_params(coarsest_n=9, precision=1))
        Hs.append(H)
        Os.append(oracle.Hierarchy(phi, 2, n, coarsest_n=9, params=oracle_params(H.params)))
        st = lsmg.State(H)
        s0, c0 = I.initial_state(n, 2)
        st.set_grid(cuda(s0), cuda(c0))
        sts.append(st)
        Ws.append(Os[-1].to_compact(0, s0, c0))
    B = lsmg.Batch(Hs)
    for k in range(3):
        status, _ = B.step(sts, dt)
        for m, (O, st) in enumerate(zip(Os, sts)):
            orc, Ws[m], _ = O.newton_cn_step(Ws[m], dt, np.ones(O.level_info(0)["ng"]))
            assert status[m] == orc == 0, (k, m, status[m], orc)
            na = O.level_info(0)["na"]
            G = host(st.get())
            e = max(rel(G[:na], Ws[m][:na]), rel(G[na:], Ws[m][na:]))
            assert e <= TOL, (k, m, e)
        say(f"random batch step {k}: members within {TOL:g} of the oracle")
