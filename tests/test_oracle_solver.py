"""Pins of the oracle's solvers against references that share none of its solver code.

* Linear solve: V-cycles iterated to convergence equal scipy's sparse direct
  solve of the assembled Jacobian.
* Crank-Nicolson step: Newton with V-cycles gives the same W^{n+1} as Newton
  with direct solves.
* d = 0: every node is an independent 2x2 nonlinear Crank-Nicolson system,
  solved here node by node with scipy's root finder.
* Manufactured solution of section 4.1: second-order convergence in s and c
  (the paper's Tables 1-2 report orders close to 2).
* Multigrid convergence factor (section 4.2 metric) stays small and does not
  grow under refinement.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse
import scipy.sparse.linalg

import lsmg_inputs as I

SOLVER = dict(ghost_sweeps=5, ghost_sweeps_coarse=20, sweeps_lambda=0.3)


def _hier(oracle_mod, kind, n, coarsest, **params):
    phi = {"disk": I.disk, "star": I.star}[kind](n)
    p = dict(SOLVER)
    p.update(params)
    return oracle_mod.Hierarchy(phi, 2, n, coarsest_n=coarsest, params=p)


def _initial(H, s0=0.0, c0=1.0):
    na = H.level_info(0)["na"]
    return np.concatenate([np.full(na, s0), np.full(na, c0)])


def _coo(H):
    rows, cols, vals = H.assemble_coo(0)
    N = 2 * H.level_info(0)["na"]
    return scipy.sparse.csc_matrix((vals, (rows, cols)), shape=(N, N))


@pytest.mark.parametrize("kind,n,coarsest", [("disk", 65, 5), ("star", 129, 9)])
def test_vcycles_converge_to_direct_solve(oracle_mod, kind, n, coarsest):
    H = _hier(oracle_mod, kind, n, coarsest)
    info = H.level_info(0)
    rng = np.random.default_rng(5)
    W = np.concatenate([rng.uniform(0, 1, info["na"]), rng.uniform(0.5, 1.5, info["na"])])
    dt = 1e-3
    H.set_linearization(W, dt)
    rhs = rng.standard_normal(W.size)
    x_direct = scipy.sparse.linalg.spsolve(_coo(H), rhs)
    x = np.zeros_like(rhs)
    for _ in range(40):
        x, res = H.vcycle(0, rhs, x)
        if res < 1e-13 * np.max(np.abs(rhs)):
            break
    assert np.max(np.abs(x - x_direct)) <= 1e-10 * np.max(np.abs(x_direct))


def test_newton_with_vcycles_equals_newton_with_direct_solves(oracle_mod):
    H = _hier(oracle_mod, "star", 129, 9)
    info = H.level_info(0)
    dt = 1e-3
    sb = np.ones(info["ng"])
    W0 = _initial(H)
    rc, W_mg, st = H.newton_cn_step(W0, dt, sb, newton_tol=1e-12)
    assert rc == 0
    W = W0.copy()
    for _ in range(30):
        F, nF = H.residual(W, W0, dt, sb)
        H.set_linearization(W, dt)
        D = scipy.sparse.linalg.spsolve(_coo(H), F)
        W = W - D
        if np.max(np.abs(D)) < 1e-14 * np.max(np.abs(W)):
            break
    scale = np.max(np.abs(W))
    assert np.max(np.abs(W_mg - W)) < 1e-11 * scale


def test_pointwise_cn_systems_without_diffusion(oracle_mod):
    # with d = 0 each inside node evolves by the two reaction ODEs; Crank-Nicolson gives one
    # 2x2 nonlinear system per node, solved here independently of the oracle
    H = _hier(oracle_mod, "disk", 33, 5, d=0.0)
    info = H.level_info(0)
    na, ni = info["na"], info["ni"]
    rng = np.random.default_rng(2)
    W0 = np.concatenate([rng.uniform(0, 1, na), rng.uniform(0.5, 1.5, na)])
    dt = 1e-3
    rc, W1, _ = H.newton_cn_step(W0, dt, np.ones(info["ng"]), newton_tol=1e-13)
    assert rc == 0
    M = I.MODEL
    ks, kc = M["a"] / M["m_c"], M["a"] / M["m_s"]
    por = lambda c: M["alpha"] * c + M["beta"]
    for r in range(0, ni, 7):
        s0, c0 = W0[r], W0[na + r]

        def eqs(v):
            s, c = v
            return [(por(c) * s - por(c0) * s0) / dt + 0.5 * (ks * por(c) * s * c + ks * por(c0) * s0 * c0),
                    (c - c0) / dt + 0.5 * (kc * por(c) * s * c + kc * por(c0) * s0 * c0)]

        sol = scipy.optimize.fsolve(eqs, [s0, c0], xtol=1e-13)
        assert abs(W1[r] - sol[0]) < 1e-11 and abs(W1[na + r] - sol[1]) < 1e-11


def _mms_run(oracle_mod, n, T=1.0):
    H = _hier(oracle_mod, "disk", n, 5)
    info = H.level_info(0)
    na, ni = info["na"], info["ni"]
    h = info["h"]
    dt = h
    steps = int(round(T / dt))
    x, y = I.grid_points(n, 2)
    g = H.compact_to_grid(0)
    xa, ya = x[g], y[g]
    B = H.ghost_table(0)["B"]
    W = np.concatenate([I.s_exact(xa, ya, 0.0), I.c_exact(xa, ya, 0.0)])

    def forcing(t):
        f1, f2 = I.mms_sources(xa, ya, t)
        return np.concatenate([f1, f2])

    for k in range(steps):
        t0, t1 = k * dt, (k + 1) * dt
        sb = I.s_exact(B[:, 0], B[:, 1], t1)
        rc, W, _ = H.newton_cn_step(W, dt, sb, forcing(t0), forcing(t1))
        assert rc == 0
    t = steps * dt
    es = np.abs(W[:ni] - I.s_exact(xa[:ni], ya[:ni], t))
    ec = np.abs(W[na:na + ni] - I.c_exact(xa[:ni], ya[:ni], t))
    sx = np.abs(I.s_exact(xa[:ni], ya[:ni], t)); cx = np.abs(I.c_exact(xa[:ni], ya[:ni], t))
    return es.max() / sx.max(), ec.max() / cx.max(), es.sum() / sx.sum(), ec.sum() / cx.sum()


def test_manufactured_solution_second_order(oracle_mod):
    errs = [_mms_run(oracle_mod, n) for n in (17, 33, 65, 129)]
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    # L-infinity and L1 orders of s and c between successive grids
    assert np.all(orders[1:] > 1.85), orders
    assert np.all(errs[-1] < 1e-5), errs[-1]


def _rho(oracle_mod, kind, n, coarsest, dt):
    H = _hier(oracle_mod, kind, n, coarsest)
    info = H.level_info(0)
    W = _initial(H)
    sb = np.ones(info["ng"])
    rc, W, st = H.newton_cn_step(W, dt, sb, rho_cap=200)
    assert rc == 0
    rho = st["rho"]
    return np.median(rho[1:])


def test_multigrid_convergence_factor(oracle_mod):
    r65 = _rho(oracle_mod, "disk", 65, 5, 1e-3)
    assert r65 < 0.05
    r257 = _rho(oracle_mod, "star", 257, 9, 1e-4)
    r513 = _rho(oracle_mod, "star", 513, 9, 1e-4)
    assert r257 < 0.1 and r513 < 0.2


@pytest.mark.parametrize("member", [36, 47, 14])
def test_batch_star_domains_converge(oracle_mod, member):
    # 129^2 stars of the 64-domain batch (seed 0) with thin arms and concave corners: with the
    # axis rows for negative ghost weights and the extra ghost relaxations on mass-dominated
    # levels, Newton converges in the same few iterations as on the smooth domains and the
    # V-cycle factor stays well below 1
    d = I.batch_domains(64, 0)[member]
    n = d["n"]
    H = oracle_mod.Hierarchy(I.star(n, **d["shape"]), 2, n, coarsest_n=9, params=dict(SOLVER))
    W = _initial(H)
    sb = np.ones(H.level_info(0)["ng"])
    for _ in range(2):
        rc, W, st = H.newton_cn_step(W, 1e-4, sb, rho_cap=200)
        assert rc == 0
        assert st["newton_iters"] <= 5
        assert np.median(st["rho"][1:st["vcycles"]]) < 0.5


def _mms_star_run(oracle_mod, shape, n, T):
    H = oracle_mod.Hierarchy(I.star(n, **shape), 2, n, coarsest_n=9, params=dict(SOLVER))
    info = H.level_info(0)
    na, ni, h = info["na"], info["ni"], info["h"]
    dt = h
    x, y = I.grid_points(n, 2)
    g = H.compact_to_grid(0)
    xa, ya = x[g], y[g]
    gt = H.ghost_table(0)
    B = gt["B"]
    W = np.concatenate([I.s_exact(xa, ya, 0.0), I.c_exact(xa, ya, 0.0)])

    def forcing(t):
        return np.concatenate(I.mms_sources(xa, ya, t))

    steps = int(round(T / dt))
    for k in range(steps):
        t0, t1 = k * dt, (k + 1) * dt
        rc, W, _ = H.newton_cn_step(W, dt, I.s_exact(B[:, 0], B[:, 1], t1), forcing(t0), forcing(t1))
        assert rc == 0
    t = steps * dt
    sx, cx = I.s_exact(xa[:ni], ya[:ni], t), I.c_exact(xa[:ni], ya[:ni], t)
    es, ec = np.abs(W[:ni] - sx), np.abs(W[na:na + ni] - cx)
    return (np.array([es.max() / np.abs(sx).max(), ec.max() / np.abs(cx).max(),
                      es.sum() / np.abs(sx).sum(), ec.sum() / np.abs(cx).sum()]),
            int(np.sum(gt["bfallback"] == 2)))


def test_manufactured_solution_second_order_on_thin_armed_star(oracle_mod):
    # member 36 of the 64-star batch (seed 0): on the 129^2 grid four ghosts at its concave
    # corners would take a negative biquadratic self-weight; their axis rows keep the scheme
    # second order there (with the constant rule s_G = s_b the 129^2 error was 1.7e-3, four
    # orders above the trend; measured now 6.0e-7, 1.5e-7, 3.8e-8, orders 1.98-2.01)
    shape = I.batch_domains(64, 0)[36]["shape"]
    runs = [_mms_star_run(oracle_mod, shape, n, 0.25) for n in (129, 257, 513)]
    errs = np.array([e for e, _ in runs])
    assert runs[0][1] == 4
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 1.9), orders
    assert np.all(errs[0] < 2e-6), errs[0]
