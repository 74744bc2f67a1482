"""Seeded random configurations stepped on the GPU beside the oracle, each on its own
inputs: 2-D star domains of random shape, size, time step, precision and boundary rows
(Dirichlet or Neumann), the same stars under W-cycles with full multigrid, 3-D unions of
random ellipsoids with Dirichlet and with Neumann rows, and batches of random stars and
of random unions of different sizes.  After every Crank-Nicolson step the two sides must
end with the same status and, when both converged,
||x_gpu - x_oracle||_inf / ||x_oracle||_inf <= 1e-10 for s and for c over the active
nodes.  Each case prints its draws before any GPU work."""
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


def _union_draw(rng):
    m = int(rng.integers(1, 4))
    centres = [tuple(float(v) for v in rng.uniform(-0.4, 0.4, 3)) for _ in range(m)]
    semi = [tuple(float(v) for v in rng.uniform(0.15, 0.4, 3)) for _ in range(m)]
    return m, centres, semi


@pytest.mark.parametrize("seed", range(3))
def test_random_neumann_union(seed):
    # Neumann rows (section 3.6) on a random union; a ghost with no admissible row is
    # refused by the build, and then both sides must refuse it
    rng = np.random.default_rng(7300 + seed)
    n = int(rng.choice([33, 65]))
    m, centres, semi = _union_draw(rng)
    precision = int(rng.integers(0, 2))
    label = f"random Neumann union {seed}: n={n} m={m} precision={precision}"
    say(label)
    phi = I.ellipsoids(n, centres, semi)
    p = lsmg.default_params(coarsest_n=9, precision=precision, bc=1)
    try:
        H = lsmg.Hierarchy(torch.from_numpy(phi), 3, n, params=p)
    except lsmg.LsmgError as e:
        assert e.code == lsmg.EGEOM, (label, e.code)
        with pytest.raises(oracle.OracleError) as eo:
            oracle.Hierarchy(phi, 3, n, coarsest_n=9, bc=1)
        assert eo.value.code == oracle.EGEOM
        say(f"{label}: refused by both sides")
        return
    O = oracle.Hierarchy(phi, 3, n, coarsest_n=9, params=oracle_params(H.params), bc=1)
    _step_both(H, O, n, 3, 1e-4, 2, label)


@pytest.mark.parametrize("seed", range(3))
def test_random_star_w_cycle(seed):
    # the paper's cycle index (gamma = 2), with full multigrid drawn on or off
    rng = np.random.default_rng(7400 + seed)
    n = int(rng.choice([33, 65, 129]))
    shape = _star_draw(rng)
    precision = int(rng.integers(0, 2))
    fmg = int(rng.integers(0, 2))
    dt = float(rng.choice([1e-4, 2.0 / (n - 1)]))
    coarsest = 5 if n == 33 else 9
    label = f"random star, W-cycle {seed}: n={n} {shape} dt={dt:.3g} precision={precision} fmg={fmg}"
    say(label)
    H, O = pair("star", n, coarsest, phi=I.star(n, **shape), precision=precision, cycle_gamma=2, fmg=fmg)
    _step_both(H, O, n, 2, dt, 2, label)


def _batch_against_oracle(phis, dim, sizes, dt, steps, label, **params):
    Hs, Os, sts, Ws = [], [], [], []
    for n, phi in zip(sizes, phis):
        H = lsmg.Hierarchy(torch.from_numpy(phi), dim, n, params=lsmg.default_params(coarsest_n=9, **params))
        Hs.append(H)
        Os.append(oracle.Hierarchy(phi, dim, n, coarsest_n=9, params=oracle_params(H.params), bc=H.params.bc))
        st = lsmg.State(H)
        s0, c0 = I.initial_state(n, dim)
        st.set_grid(cuda(s0), cuda(c0))
        sts.append(st)
        Ws.append(Os[-1].to_compact(0, s0, c0))
    B = lsmg.Batch(Hs)
    for k in range(steps):
        status, _ = B.step(sts, dt)
        for m, (O, st) in enumerate(zip(Os, sts)):
            orc, Ws[m], _ = O.newton_cn_step(Ws[m], dt, np.ones(O.level_info(0)["ng"]))
            assert status[m] == orc == 0, (label, k, m, status[m], orc)
            na = O.level_info(0)["na"]
            G = host(st.get())
            e = max(rel(G[:na], Ws[m][:na]), rel(G[na:], Ws[m][na:]))
            assert e <= TOL, (label, k, m, e)
        say(f"{label} step {k}: members within {TOL:g} of the oracle")


def test_random_batch_3d():
    # unions of random ellipsoids at two grid sizes, batched in mixed precision
    rng = np.random.default_rng(7500)
    sizes = [33, 65, 33]
    draws = [_union_draw(rng) for _ in sizes]
    say(f"random 3-D batch: sizes {sizes} ellipsoids per member {[d[0] for d in draws]}")
    phis = [I.ellipsoids(n, c, s) for n, (_, c, s) in zip(sizes, draws)]
    _batch_against_oracle(phis, 3, sizes, 1e-4, 2, "random 3-D batch", precision=1)


def test_random_batch_neumann_2d():
    # random stars of three sizes with Neumann rows, batched in FP64
    rng = np.random.default_rng(7600)
    sizes = [65, 129, 33]
    shapes = [_star_draw(rng) for _ in sizes]
    say(f"random Neumann batch: sizes {sizes} shapes {shapes}")
    phis = [I.star(n, **sh) for n, sh in zip(sizes, shapes)]
    _batch_against_oracle(phis, 2, sizes, 1e-4, 2, "random Neumann batch", precision=0, bc=1)
