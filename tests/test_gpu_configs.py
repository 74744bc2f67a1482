"""Each configuration over its whole stated length, GPU against the oracle after
every Crank-Nicolson step (||x_gpu - x_oracle||_inf / ||x_oracle||_inf <= 1e-10
for s and for c), with the GPU on its own inputs (its own hierarchy from the
level set, its own boundary points):

* configuration 2, the star at 1025^2: all 100 steps in FP64, the oracle live;
* configuration 3, the torus at 257^3: all 20 steps, FP64 and mixed precision,
  against the oracle's stored trajectory (tests/golden/trajectory_torus257.npz,
  written by tests/golden/make_oracle_trajectories.py: 512 seeded active nodes
  per step and the norms over all of them);
* configuration 4: one member of each grid size of the 64-star batch, batched
  together in mixed precision, all 50 steps, the oracle live;
* configuration 5: served requests to completion in mixed precision, request 12
  (129^3) and request 17 (257^3) of the seeded stream, against stored oracle
  trajectories; and requests on the domains as stated, the plain (creased) minimum
  of their ellipsoids, where the V-cycles converge on it (request 18 at 65^3 and
  request 19 at 129^3), stepped beside the live oracle."""
import os

import numpy as np
import pytest
import torch

import lsmg_inputs as I
from _gpu import cuda, host, oracle_params, rel, say
from paper_1902_07029_amd import lsmg

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu


def _state(H, n, dim):
    st = lsmg.State(H)
    s0, c0 = I.initial_state(n, dim)
    st.set_grid(cuda(s0), cuda(c0))
    return st


def test_star_1025_config_all_steps():
    import oracle
    n, dt, steps = 1025, 1e-4, 100
    phi = I.star(n)
    H = lsmg.Hierarchy(torch.from_numpy(phi), 2, n, params=lsmg.default_params(coarsest_n=9, precision=0))
    O = oracle.Hierarchy(phi, 2, n, coarsest_n=9, params=oracle_params(H.params))
    na = O.level_info(0)["na"]
    st = _state(H, n, 2)
    s0, c0 = I.initial_state(n, 2)
    W = O.to_compact(0, s0, c0)
    sb = np.ones(O.level_info(0)["ng"])
    worst = 0.0
    for k in range(steps):
        _, gs = st.step(dt)
        rc, W, os_ = O.newton_cn_step(W, dt, sb)
        assert rc == 0
        G = host(st.get())
        e = max(rel(G[:na], W[:na]), rel(G[na:], W[na:]))
        worst = max(worst, e)
        if k % 10 == 9 or e > TOL:
            say(f"star 1025^2 FP64 step {k + 1}/{steps}: err {e:.2e} (worst {worst:.2e}) "
                f"cycles {gs['vcycles']}/{os_['vcycles']}")
        assert e <= TOL, (k, e)


def _golden(case):
    return np.load(os.path.join(GOLDEN, f"trajectory_{case}.npz"))


def _check_against_golden(case, phi, precision):
    g = _golden(case)
    n, steps, dt = int(g["n"]), int(g["steps"]), float(g["dt"])
    p = lsmg.default_params(coarsest_n=9, precision=precision)
    H = lsmg.Hierarchy(torch.from_numpy(phi), 3, n, params=p)
    eff = H.params
    assert (eff.ghost_sweeps, eff.ghost_sweeps_coarse) == tuple(int(v) for v in g["params"])
    assert eff.sweeps_lambda == float(g["sweeps_lambda"])
    info = H.level_info(0)
    assert (info["na"], info["ng"]) == (int(g["na"]), int(g["ng"]))
    na, idx = info["na"], g["idx"]
    st = _state(H, n, 3)
    worst = 0.0
    for k in range(steps):
        rc, gs = st.step(dt)
        assert rc == 0
        G = host(st.get())
        errs = []
        for b, blk in enumerate((slice(0, na), slice(na, 2 * na))):
            ref = g["norms"][k, b]
            errs.append(np.max(np.abs(G[blk][idx] - g["vals"][k, b])) / ref)
            errs.append(abs(np.max(np.abs(G[blk])) - ref) / ref)
        e = max(errs)
        worst = max(worst, e)
        if k % 5 == 4 or e > TOL or k == steps - 1:
            say(f"{case} precision {precision} step {k + 1}/{steps}: err {e:.2e} (worst {worst:.2e}) "
                f"newton {gs['newton_iters']}/{g['counts'][k, 0]} cycles {gs['vcycles']}/{g['counts'][k, 1]}")
        assert e <= TOL, (k, e)
    return worst


@pytest.mark.parametrize("precision", [0, 1])
def test_torus_257_config_all_steps(precision):
    _check_against_golden("torus257", I.torus(257), precision)


def _request(rid):
    return [r for r in I.serving_requests(24, seed=0) if r["id"] == rid][0]


@pytest.mark.parametrize("rid", [12, 17])
def test_served_request_to_completion(rid):
    r = _request(rid)
    _check_against_golden(f"serve_r{rid}", I.ellipsoids(r["n"], r["centres"], r["semi"]), 1)


def test_batch_one_member_per_size_all_steps():
    import oracle
    doms = I.batch_domains(64, 0)
    dt, steps = doms[0]["dt"], doms[0]["steps"]
    pick = [next(k for k, d in enumerate(doms) if d["n"] == n) for n in (129, 257, 513, 1025)]
    Hs, Os, sts, Ws, sbs = [], [], [], [], []
    for k in pick:
        d = doms[k]
        phi = I.star(d["n"], **d["shape"])
        H = lsmg.Hierarchy(torch.from_numpy(phi), 2, d["n"], params=lsmg.default_params(coarsest_n=9, precision=1))
        O = oracle.Hierarchy(phi, 2, d["n"], coarsest_n=9, params=oracle_params(H.params))
        Hs.append(H)
        Os.append(O)
        sts.append(_state(H, d["n"], 2))
        s0, c0 = I.initial_state(d["n"], 2)
        Ws.append(O.to_compact(0, s0, c0))
        sbs.append(np.ones(O.level_info(0)["ng"]))
    B = lsmg.Batch(Hs)
    worst = 0.0
    for j in range(steps):
        status, stats = B.step(sts, dt)
        assert all(s == 0 for s in status)
        for m, (O, st) in enumerate(zip(Os, sts)):
            rc, Ws[m], os_ = O.newton_cn_step(Ws[m], dt, sbs[m])
            assert rc == 0
            na = O.level_info(0)["na"]
            G = host(st.get())
            e = max(rel(G[:na], Ws[m][:na]), rel(G[na:], Ws[m][na:]))
            worst = max(worst, e)
            assert e <= TOL, (j, pick[m], e)
        if j % 10 == 9:
            say(f"batch members {pick} step {j + 1}/{steps}: worst err {worst:.2e}")


@pytest.mark.parametrize("rid", [18, 19])
def test_plain_union_request_against_oracle(rid):
    import oracle
    r = _request(rid)
    n, dt = r["n"], r["dt"]
    phi = I.ellipsoids(n, r["centres"], r["semi"], smooth=0.0)
    H = lsmg.Hierarchy(torch.from_numpy(phi), 3, n, params=lsmg.default_params(coarsest_n=9, precision=1))
    O = oracle.Hierarchy(phi, 3, n, coarsest_n=9, params=oracle_params(H.params))
    info = O.level_info(0)
    na = info["na"]
    assert H.level_info(0)["na"] == na
    st = _state(H, n, 3)
    s0, c0 = I.initial_state(n, 3)
    W = O.to_compact(0, s0, c0)
    sb = np.ones(info["ng"])
    for k in range(3):
        rc, gs = st.step(dt)
        assert rc == 0
        orc, W, os_ = O.newton_cn_step(W, dt, sb)
        assert orc == 0
        G = host(st.get())
        e = max(rel(G[:na], W[:na]), rel(G[na:], W[na:]))
        say(f"plain union, request {rid} ({n}^3) step {k + 1}: err {e:.2e} "
            f"newton {gs['newton_iters']}/{os_['newton_iters']} cycles {gs['vcycles']}/{os_['vcycles']}")
        assert e <= TOL, (k, e)
