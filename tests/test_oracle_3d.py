"""Pins of the oracle's three-dimensional discretisation and solvers.

The 3-D rules are the tensor-product extension of section 3.3 (7-point
eq. FDs/FDc, triquadratic eq. BCs/JssD) and of section 3.5.  Each pin compares
the oracle with something fixed outside its code:

* the section 4.1 manufactured solution with a cos z factor on a sphere: the
  errors of s and c at t = 1/2 fall at second order (a wrong z stride, a wrong
  triquadratic weight or a dropped z term of the sources breaks the order);
* B on an analytic sphere: its distance to the sphere is an interpolation
  error of the triquadratic level-set interpolant, O(h^3);
* the boxed diagonal coefficient of eq. (JssD) in tensor form,
  prod_a theta_a (1 + theta_a) / 2, recomputed from B alone;
* V-cycles converge to scipy's sparse direct solve of the assembled Jacobian,
  and Newton with V-cycles reaches the step that Newton with direct solves does;
* F = 0 at a steady constant state.
"""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import lsmg_inputs as I

SOLVER3 = dict(ghost_sweeps=15, ghost_sweeps_coarse=30, sweeps_lambda=0.1)


def _hier(oracle_mod, phi, n, coarsest=5, **params):
    p = dict(SOLVER3)
    p.update(params)
    return oracle_mod.Hierarchy(phi, 3, n, coarsest_n=coarsest, params=p)


def _coo(H):
    rows, cols, vals = H.assemble_coo(0)
    N = 2 * H.level_info(0)["na"]
    return scipy.sparse.csc_matrix((vals, (rows, cols)), shape=(N, N))


def _mms3_run(oracle_mod, n, T=0.5, r=0.6):
    H = _hier(oracle_mod, I.sphere(n, r), n)
    info = H.level_info(0)
    na, ni, h = info["na"], info["ni"], info["h"]
    dt = h
    steps = int(round(T / dt))
    x, y, z = I.grid_points(n, 3)
    g = H.compact_to_grid(0)
    xa, ya, za = x[g], y[g], z[g]
    B = H.ghost_table(0)["B"]
    W = np.concatenate([I.s_exact3(xa, ya, za, 0.0), I.c_exact3(xa, ya, za, 0.0)])

    def forcing(t):
        return np.concatenate(I.mms_sources3(xa, ya, za, t))

    for k in range(steps):
        t0, t1 = k * dt, (k + 1) * dt
        sb = I.s_exact3(B[:, 0], B[:, 1], B[:, 2], t1)
        rc, W, _ = H.newton_cn_step(W, dt, sb, forcing(t0), forcing(t1))
        assert rc == 0
    t = steps * dt
    sx = I.s_exact3(xa[:ni], ya[:ni], za[:ni], t)
    cx = I.c_exact3(xa[:ni], ya[:ni], za[:ni], t)
    es = np.abs(W[:ni] - sx)
    ec = np.abs(W[na:na + ni] - cx)
    return es.max() / np.abs(sx).max(), ec.max() / np.abs(cx).max(), es.sum() / np.abs(sx).sum(), \
        ec.sum() / np.abs(cx).sum()


def test_manufactured_solution_second_order_3d(oracle_mod):
    errs = np.array([_mms3_run(oracle_mod, n) for n in (17, 33, 65)])
    orders = np.log2(errs[:-1] / errs[1:])
    # L-infinity and L1 orders of s and c; measured 1.88-1.97 and 1.92-1.98
    assert np.all(orders > 1.8), orders
    assert np.all(orders[-1] > 1.85), orders
    assert np.all(errs[-1] < 2e-5), errs[-1]


def test_mms_sources_3d_match_symbolic_derivatives():
    sp = pytest.importorskip("sympy")
    x, y, z, t = sp.symbols("x y z t")
    M = I.MODEL
    s = 2 + sp.sin(x) * sp.cos(y) * sp.cos(z) * sp.sin(t + sp.sqrt(2))
    c = 3 + sp.sin(x / 2) * sp.cos(3 * y) * sp.cos(z) * sp.sin(2 * t + sp.sqrt(3))
    por = M["alpha"] * c + M["beta"]
    div = sum(sp.diff(por * sp.diff(s, v), v) for v in (x, y, z))
    f1 = sp.diff(por * s, t) + M["a"] / M["m_c"] * por * s * c - M["d"] * div
    f2 = sp.diff(c, t) + M["a"] / M["m_s"] * por * s * c
    F1 = sp.lambdify((x, y, z, t), f1, "numpy")
    F2 = sp.lambdify((x, y, z, t), f2, "numpy")
    S = sp.lambdify((x, y, z, t), [sp.diff(s, v) for v in (x, y, z)], "numpy")
    rng = np.random.default_rng(1)
    X, Y, Z, T = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), rng.uniform(0, 1, 50)
    g1, g2 = I.mms_sources3(X, Y, Z, T)
    assert np.allclose(g1, F1(X, Y, Z, T), rtol=1e-13, atol=1e-12)
    assert np.allclose(g2, F2(X, Y, Z, T), rtol=1e-13, atol=1e-12)
    for a, b in zip(I.s_exact3_grad(X, Y, Z, T), S(X, Y, Z, T)):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


def test_boundary_point_on_sphere(oracle_mod):
    # distance of B to the sphere of radius 0.6: measured 1.0e-3, 1.2e-4, 1.8e-5 (ratios 8.4, 7.0)
    errs = []
    for n in (17, 33, 65):
        H = _hier(oracle_mod, I.sphere(n), n)
        B = H.ghost_table(0)["B"]
        errs.append(np.max(np.abs(np.linalg.norm(B, axis=1) - 0.6)))
    assert errs[0] < 2e-3
    assert errs[1] < errs[0] / 6 and errs[2] < errs[1] / 6


def test_triquadratic_diagonal_coefficient_and_cfl(oracle_mod):
    # the ghost's own weight is prod_a theta_a (1 + theta_a) / 2 with theta_a measured from the
    # first inner stencil node along SIGN(n_a); |1 - 0.9 w| < 1 (eq. CFLcond)
    n = 33
    H = _hier(oracle_mod, I.sphere(n, 0.55, (0.03, -0.02, 0.05)), n)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    x, y, z = I.grid_points(n, 3)
    h = info["h"]
    checked = 0
    for q in range(info["ng"]):
        g = c2g[info["ni"] + q]
        if gt["order"][q] != 2:
            continue
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        G = np.array([x[g], y[g], z[g]])
        th = m * (gt["B"][q] - (G - m * h)) / h
        w0 = np.prod(th * (1 + th) / 2)
        assert abs(gt["w"][q][0] - w0) < 1e-14
        assert abs(1 - 0.9 * w0) < 1
        checked += 1
    assert checked > 0.9 * info["ng"]


def test_ghost_stencil_offsets_3d(oracle_mod):
    # the 27 stencil nodes of a ghost G are G - m_a k_a e_a, k_a in {0,1,2}, with the first
    # node G itself; checked against the grid coordinates (a wrong z stride moves them)
    n = 33
    H = _hier(oracle_mod, I.torus(n), n, coarsest=9)
    info = H.level_info(0)
    gt = H.ghost_table(0)
    c2g = H.compact_to_grid(0)
    h = info["h"]
    x, y, z = I.grid_points(n, 3)
    P = np.stack([x, y, z], axis=1)
    for q in range(0, info["ng"], 7):
        if gt["order"][q] != 2:
            continue
        st = gt["st"][q]
        # inactive stencil nodes (index -1) are allowed only under exactly zero weights
        assert np.all(gt["w"][q][st < 0] == 0.0)
        if np.any(st < 0):
            continue
        g = c2g[info["ni"] + q]
        m = np.where(gt["normal"][q] >= 0, 1, -1)
        pts = P[c2g[st]]
        assert c2g[st[0]] == g
        offs = np.rint((P[g] - pts) / h).astype(int) * m
        assert sorted(map(tuple, offs)) == sorted((i, j, k) for k in range(3) for j in range(3) for i in range(3))


@pytest.mark.parametrize("kind,n", [("sphere", 17), ("torus", 33), ("sphere", 33)])
def test_vcycles_converge_to_direct_solve_3d(oracle_mod, kind, n):
    phi = I.sphere(n) if kind == "sphere" else I.torus(n)
    H = _hier(oracle_mod, phi, n)
    info = H.level_info(0)
    rng = np.random.default_rng(5)
    W = np.concatenate([rng.uniform(0, 1, info["na"]), rng.uniform(0.5, 1.5, info["na"])])
    H.set_linearization(W, 1e-3)
    rhs = rng.standard_normal(W.size)
    x_direct = scipy.sparse.linalg.spsolve(_coo(H), rhs)
    x = np.zeros_like(rhs)
    for _ in range(60):
        x, res = H.vcycle(0, rhs, x)
        if res < 1e-13 * np.max(np.abs(rhs)):
            break
    assert np.max(np.abs(x - x_direct)) <= 1e-10 * np.max(np.abs(x_direct))


def test_newton_with_vcycles_equals_newton_with_direct_solves_3d(oracle_mod):
    n = 33
    H = _hier(oracle_mod, I.torus(n), n)
    info = H.level_info(0)
    na = info["na"]
    dt = 1e-3
    sb = np.ones(info["ng"])
    W0 = np.concatenate([np.zeros(na), np.ones(na)])
    rc, W_mg, _ = H.newton_cn_step(W0, dt, sb, newton_tol=1e-12)
    assert rc == 0
    W = W0.copy()
    for _ in range(30):
        F, _ = H.residual(W, W0, dt, sb)
        H.set_linearization(W, dt)
        D = scipy.sparse.linalg.spsolve(_coo(H), F)
        W = W - D
        if np.max(np.abs(D)) < 1e-14 * np.max(np.abs(W)):
            break
    assert np.max(np.abs(W_mg - W)) < 1e-11 * np.max(np.abs(W))


def test_residual_vanishes_at_steady_constant_state_3d(oracle_mod):
    n = 33
    H = _hier(oracle_mod, I.torus(n), n, a=0.0)
    info = H.level_info(0)
    na = info["na"]
    W = np.concatenate([np.full(na, 0.7), np.full(na, 1.3)])
    _, nrm = H.residual(W, W, 1e-3, np.full(info["ng"], 0.7))
    assert nrm < 1e-11
