"""Continuous batching (paper_1902_07029_amd.serve): requests that arrive while
others run join the batch at step boundaries; each result must be bitwise the
result of the same simulation run alone with lsmg_newton_cn_step; admission must
respect the memory budget."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
from _gpu import say
from paper_1902_07029_amd import lsmg
from paper_1902_07029_amd.serve import Request, Server


def _requests(count, seed, sizes=(33, 65), steps=(3, 7), gap=0.02):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(count):
        t += gap * rng.uniform(0.5, 1.5)
        m = int(rng.integers(1, 3))
        centres = [tuple(rng.uniform(-0.3, 0.3, 3)) for _ in range(m)]
        semi = [tuple(rng.uniform(0.25, 0.4, 3)) for _ in range(m)]
        n = int(rng.choice(sizes))
        out.append(Request(i, t, 3, n, int(rng.integers(*steps)), 1e-4, I.ellipsoids(n, centres, semi)))
    return out


def _alone(req, params):
    H = lsmg.Hierarchy(torch.from_numpy(req.phi), req.dim, req.n, params=params)
    st = lsmg.State(H)
    nn = req.n ** req.dim
    st.set_grid(torch.full((nn,), req.s0, dtype=torch.float64, device="cuda"),
                torch.full((nn,), req.c0, dtype=torch.float64, device="cuda"))
    for _ in range(req.steps):
        st.step(req.dt, sb_const=req.sb)
    return st.get().cpu().numpy()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [1, 0])
def test_served_results_equal_alone(precision):
    params = lsmg.default_params(coarsest_n=9, precision=precision)
    reqs = _requests(6, 3, steps=(8, 15), gap=0.01)
    rep = Server(params, keep_states=True).run(reqs)
    assert rep["completed"] == len(reqs), rep["errors"]
    say(f"served {len(reqs)} requests in {rep['ticks']} ticks, up to {rep['max_members']} "
        f"members at once, p50 {rep['p50_step_ms']:.2f} ms p99 {rep['p99_step_ms']:.2f} ms")
    # requests overlapped on the device: some batched step held several members
    assert rep["max_members"] >= 2
    by_id = {f["id"]: f for f in rep["finished"]}
    for r in reqs:
        f = by_id[r.id]
        assert f["steps"] == r.steps
        assert np.array_equal(f["state"], _alone(r, params)), r.id


@pytest.mark.gpu
def test_admission_respects_budget():
    params = lsmg.default_params(coarsest_n=9, precision=1)
    reqs = _requests(5, 5, sizes=(65,), steps=(3, 5), gap=0.0)
    est = sum(lsmg.estimate_bytes(3, 65, params))
    # room for two simulations at a time
    rep = Server(params, budget_bytes=int(2.5 * est)).run(reqs)
    assert rep["completed"] == len(reqs)
    say(f"budget for 2.5 estimates: up to {rep['max_members']} members at once")
    assert rep["max_members"] <= 2
    for f in rep["finished"]:
        assert f["bytes"] <= f["est_bytes"], (f["bytes"], f["est_bytes"])


@pytest.mark.gpu
def test_failing_request_is_evicted_others_unchanged():
    # one request starts from a non-finite state (forced from the host): its first step
    # fails with LSMG_ENONFINITE and it leaves the batch; the others finish with the
    # bits they have when run alone
    params = lsmg.default_params(coarsest_n=9, precision=1)
    reqs = _requests(4, 7, steps=(5, 9), gap=0.0)
    bad = reqs[1]
    bad.s0 = float("nan")
    rep = Server(params, keep_states=True).run(reqs)
    by_id = {f["id"]: f for f in rep["finished"]}
    say(f"served {len(reqs)} requests, one failing: statuses "
        f"{[by_id[r.id]['status'] for r in reqs]}, up to {rep['max_members']} members at once")
    assert by_id[bad.id]["status"] == lsmg.ENONFINITE and by_id[bad.id]["steps"] == 0
    assert rep["completed"] == len(reqs) - 1
    assert rep["max_members"] >= 2
    for r in reqs:
        if r is bad:
            continue
        f = by_id[r.id]
        assert f["status"] == lsmg.OK and f["steps"] == r.steps
        assert np.array_equal(f["state"], _alone(r, params)), r.id


def _alone_with_lane(req, params, krylov_m, krylov_cycles):
    # the lane's rule applied to one simulation on its own: after a first step of more
    # than krylov_cycles V-cycles, the remaining steps use Krylov solves
    H = lsmg.Hierarchy(torch.from_numpy(req.phi), req.dim, req.n, params=params)
    st = lsmg.State(H)
    nn = req.n ** req.dim
    st.set_grid(torch.full((nn,), req.s0, dtype=torch.float64, device="cuda"),
                torch.full((nn,), req.c0, dtype=torch.float64, device="cuda"))
    lane = False
    for k in range(req.steps):
        _, stats = st.step(req.dt, sb_const=req.sb)
        if k == 0 and stats["vcycles"] > krylov_cycles:
            p = type(params).from_buffer_copy(params)
            p.krylov_m = krylov_m
            H.set_params(p)
            lane = True
    return st.get().cpu().numpy(), lane


@pytest.mark.gpu
def test_slow_request_moves_to_the_krylov_lane():
    # request 10 of the served stream on its plain (creased) union needs about 212
    # V-cycles in its first step: it leaves the batch after that step and finishes with
    # Krylov solves beside two ordinary requests.  Every result equals the same
    # simulation run alone under the same rule, and the slow one is within 1e-10 of the
    # oracle stepping it the same way.
    import oracle
    from _gpu import oracle_params, rel
    params = lsmg.default_params(coarsest_n=9, precision=1)
    r10 = [q for q in I.serving_requests(24, seed=0) if q["id"] == 10][0]
    n = r10["n"]
    slow = Request(100, 0.0, 3, n, 3, r10["dt"], I.ellipsoids(n, r10["centres"], r10["semi"], smooth=0.0))
    reqs = [slow] + _requests(2, 11, sizes=(33,), steps=(4, 6), gap=0.0)
    rep = Server(params, keep_states=True, krylov_m=30, krylov_cycles=60).run(reqs)
    assert rep["completed"] == len(reqs), rep["errors"]
    say(f"Krylov lane: {rep['krylov_lane']}, p99 {rep['p99_step_ms']:.2f} ms, up to {rep['max_members']} in the batch")
    assert rep["krylov_lane"] == [100]
    by_id = {f["id"]: f for f in rep["finished"]}
    for r in reqs:
        state, lane = _alone_with_lane(r, params, 30, 60)
        assert lane == (r.id == 100)
        assert np.array_equal(by_id[r.id]["state"], state), r.id
    # the effective parameters (automatic ghost sweep counts resolved) of a hierarchy of the domain
    eff = lsmg.Hierarchy(torch.from_numpy(slow.phi), 3, n, params=params).params
    O = oracle.Hierarchy(slow.phi, 3, n, coarsest_n=9, params=oracle_params(eff))
    info = O.level_info(0)
    s0, c0 = I.initial_state(n, 3)
    W = O.to_compact(0, s0, c0)
    sb = np.ones(info["ng"])
    for k in range(slow.steps):
        if k == 1:
            O.set_params(krylov_m=30)
        rc, W, _ = O.newton_cn_step(W, slow.dt, sb)
        assert rc == 0
    G = by_id[100]["state"]
    na = info["na"]
    e = max(rel(G[:na], W[:na]), rel(G[na:], W[na:]))
    say(f"request 10 through the lane against the oracle: {e:.2e}")
    assert e <= 1e-10
