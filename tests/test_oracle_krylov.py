"""Pins of the oracle's Krylov option (krylov_m > 0: flexible GMRES preconditioned by one
V-cycle, in place of the paper's plain cycles) against references that share none of
its code:

* the Krylov solve alone reaches scipy's sparse direct solve of the assembled
  Jacobian, with and without restarts, in 2-D and in 3-D;
* a Crank-Nicolson step with Krylov solves gives the same W^{n+1} as Newton with
  direct solves (the nonlinear system and its stopping rule are unchanged);
* on a creased union of ellipsoids, where a few ghost rows with a tiny self-weight
  make plain V-cycles converge at rho ~ 0.9, the Krylov solves need a tenth of the
  cycles: a solver that fell back to a plain preconditioned iteration fails this.
"""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import lsmg_inputs as I

SOLVER_2D = dict(ghost_sweeps=5, ghost_sweeps_coarse=20, sweeps_lambda=0.3)
SOLVER_3D = dict(ghost_sweeps=15, ghost_sweeps_coarse=30, sweeps_lambda=0.1)


def _coo(H):
    rows, cols, vals = H.assemble_coo(0)
    N = 2 * H.level_info(0)["na"]
    return scipy.sparse.csc_matrix((vals, (rows, cols)), shape=(N, N))


def _linearised(oracle_mod, dim, n, seed):
    if dim == 2:
        H = oracle_mod.Hierarchy(I.star(n), 2, n, coarsest_n=9, params=SOLVER_2D)
    else:
        H = oracle_mod.Hierarchy(I.torus(n), 3, n, coarsest_n=9, params=SOLVER_3D)
    info = H.level_info(0)
    rng = np.random.default_rng(seed)
    W = np.concatenate([rng.uniform(0, 1, info["na"]), rng.uniform(0.5, 1.5, info["na"])])
    H.set_linearization(W, 1e-3)
    return H, rng.standard_normal(W.size)


@pytest.mark.parametrize("dim,n,m", [(2, 65, 30), (2, 65, 3), (3, 17, 30), (3, 33, 4)])
def test_krylov_solve_reaches_direct_solve(oracle_mod, dim, n, m):
    # m = 3 and 4 restart several times before the tolerance is met
    H, rhs = _linearised(oracle_mod, dim, n, 11 + n)
    x_direct = scipy.sparse.linalg.spsolve(_coo(H), rhs)
    x, cycles = H.krylov_solve(rhs, m=m, rtol=1e-12, cycles_max=400)
    assert 0 < cycles < 400
    assert np.max(np.abs(x - x_direct)) <= 1e-9 * np.max(np.abs(x_direct))


def test_krylov_solve_is_exact_in_few_steps_on_a_tiny_grid(oracle_mod):
    # on a 9 x 9 grid (the coarsest level only) the V-cycle is the exact solve, so GMRES
    # preconditioned by it ends after one iteration with the direct solution
    H = oracle_mod.Hierarchy(I.disk(9, r=0.6), 2, 9, coarsest_n=9, params=SOLVER_2D)
    na = H.level_info(0)["na"]
    H.set_linearization(np.concatenate([np.full(na, 0.3), np.full(na, 1.0)]), 1e-3)
    rhs = np.random.default_rng(3).standard_normal(2 * na)
    x, cycles = H.krylov_solve(rhs, m=10, rtol=1e-13, cycles_max=10)
    assert cycles == 1
    x_direct = scipy.sparse.linalg.spsolve(_coo(H), rhs)
    assert np.max(np.abs(x - x_direct)) <= 1e-12 * np.max(np.abs(x_direct))


def test_newton_with_krylov_solves_equals_newton_with_direct_solves(oracle_mod):
    n, dt = 129, 1e-3
    H = oracle_mod.Hierarchy(I.star(n), 2, n, coarsest_n=9, params=dict(SOLVER_2D, krylov_m=30))
    info = H.level_info(0)
    sb = np.ones(info["ng"])
    W0 = np.concatenate([np.zeros(info["na"]), np.ones(info["na"])])
    rc, W_k, st = H.newton_cn_step(W0, dt, sb, newton_tol=1e-12)
    assert rc == 0
    W = W0.copy()
    for _ in range(30):
        F, _ = H.residual(W, W0, dt, sb)
        H.set_linearization(W, dt)
        D = scipy.sparse.linalg.spsolve(_coo(H), F)
        W = W - D
        if np.max(np.abs(D)) < 1e-14 * np.max(np.abs(W)):
            break
    assert np.max(np.abs(W_k - W)) < 1e-11 * np.max(np.abs(W))


def test_krylov_removes_the_slow_ghost_modes_of_a_creased_union(oracle_mod):
    r = [q for q in I.serving_requests(24, seed=0) if q["id"] == 10][0]
    n = r["n"]
    phi = I.ellipsoids(n, r["centres"], r["semi"], smooth=0.0)
    sb = None
    counts = {}
    for m in (0, 30):
        H = oracle_mod.Hierarchy(phi, 3, n, coarsest_n=9, params=dict(SOLVER_3D, krylov_m=m))
        info = H.level_info(0)
        sb = np.ones(info["ng"])
        s0, c0 = I.initial_state(n, 3)
        rc, _, st = H.newton_cn_step(H.to_compact(0, s0, c0), r["dt"], sb,
                                     cycles_max=400 if m == 0 else 30)
        assert rc == 0
        counts[m] = st["vcycles"]
    # plain cycles: 212 on this step (rho ~ 0.88); Krylov: 21
    assert counts[0] > 150 and counts[30] <= 30, counts
