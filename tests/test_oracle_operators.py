"""Pins of the oracle's discrete operators.

* Jacobian: F is a cubic polynomial of W along any line, so the five-point
  central difference is exact up to rounding; it must equal J v.  This fixes
  every Jacobian entry (section 3.4) against the residual (eqs. FDs, FDc, BCs).
* Residual: a constant state equal to the boundary value with no reaction is a
  steady state, so F = 0.
* Restriction: the three stencils printed in Fig. Neigh (section 3.5.2).
* Prolongation: bilinear interpolation reproduces linear functions (3.5.3).
* Band extension: constant transport keeps a constant ghost defect constant.
* Dense LU: agrees with numpy's solver, including a system that needs pivoting.
* Manufactured sources: agree with sympy's derivatives of the section 4.1
  solutions.
"""
import os

import numpy as np
import pytest

import lsmg_inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "restriction_stencils.txt")


def _state(H, rng, l=0):
    info = H.level_info(l)
    na = info["na"]
    s = rng.uniform(0.0, 1.0, na)
    c = rng.uniform(0.5, 1.5, na)
    return np.concatenate([s, c])


@pytest.mark.parametrize("dim,kind,n,coarsest", [(2, "disk", 33, 5), (2, "star", 65, 9), (3, "torus", 33, 9)])
def test_jacobian_matches_exact_difference_of_F(oracle_mod, dim, kind, n, coarsest):
    phi = {"disk": I.disk, "star": I.star, "torus": I.torus}[kind](n)
    H = oracle_mod.Hierarchy(phi, dim, n, coarsest_n=coarsest)
    rng = np.random.default_rng(1)
    info = H.level_info(0)
    W = _state(H, rng)
    Wn = _state(H, rng)
    sb = rng.uniform(0.5, 1.5, info["ng"])
    dt = 1e-3
    v = rng.standard_normal(W.size)
    eps = 0.5

    def F(x):
        return H.residual(x, Wn, dt, sb)[0]

    fd = (-F(W + 2 * eps * v) + 8 * F(W + eps * v) - 8 * F(W - eps * v) + F(W - 2 * eps * v)) / (12 * eps)
    H.set_linearization(W, dt)
    Jv = H.apply_J(0, v)
    scale = np.max(np.abs(Jv))
    assert np.max(np.abs(Jv - fd)) < 1e-10 * scale
    # the dense and sparse assemblies are the same operator
    A = H.assemble_dense(0)
    assert np.max(np.abs(A @ v - Jv)) < 1e-12 * scale


def test_residual_vanishes_at_steady_constant_state(oracle_mod):
    H = oracle_mod.Hierarchy(I.star(129), 2, 129, coarsest_n=9,
                             params=dict(a=0.0))
    info = H.level_info(0)
    na = info["na"]
    W = np.concatenate([np.full(na, 0.7), np.full(na, 1.3)])
    F, nrm = H.residual(W, W, 1e-3, np.full(info["ng"], 0.7))
    assert nrm < 1e-11


def _read_golden():
    cases = {}
    cur = None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("case"):
            cur = line
            cases[cur] = []
        else:
            cases[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) / 16.0 for k, v in cases.items()}


def _square(n, a):
    x, y = I.grid_points(n, 2)
    return np.maximum(np.abs(x), np.abs(y)) - a


def test_restriction_reproduces_printed_stencils(oracle_mod):
    gold = _read_golden()
    n = 17
    H = oracle_mod.Hierarchy(_square(n, 0.56), 2, n, coarsest_n=5)
    fine = H.level_info(0)
    c2g_f = H.compact_to_grid(0)
    c2g_c = H.compact_to_grid(1)
    nc = H.level_info(1)["n"]

    def stencil_at(ci, cj):
        gc = ci + nc * cj
        rc = int(np.where(c2g_c == gc)[0][0])
        out = np.zeros((3, 3))
        for dj in (1, 0, -1):
            for di in (-1, 0, 1):
                gf = (2 * ci + di) + n * (2 * cj + dj)
                hit = np.where(c2g_f == gf)[0]
                if len(hit) == 0:
                    continue
                r = np.zeros(2 * fine["na"])
                r[hit[0]] = 1.0
                out[1 - dj, di + 1] = H.restrict(0, r)[rc]
        return out

    # coarse grid 9x9 on [-1,1]: node (4,4) is the origin, node (6,4) is x = 0.5, node (6,6) is (0.5, 0.5)
    assert np.allclose(stencil_at(4, 4), gold["case1"], atol=1e-15)
    assert np.allclose(stencil_at(6, 4), gold["case2"], atol=1e-15)
    assert np.allclose(stencil_at(6, 6), gold["case3"], atol=1e-15)


def test_restriction_preserves_constants(oracle_mod):
    H = oracle_mod.Hierarchy(I.star(129), 2, 129, coarsest_n=9)
    for l in range(H.nlev - 1):
        f = H.level_info(l)
        c = H.level_info(l + 1)
        r = np.concatenate([np.full(f["ni"], 2.0), np.full(f["ng"], 3.0), np.full(f["na"], 5.0)])
        rc, band = H.restrict(l, r, return_band=True)
        # inside equations see only inside defects, boundary equations only ghost/band defects
        assert np.allclose(rc[:c["ni"]], 2.0, rtol=1e-14)
        assert np.allclose(rc[c["ni"]:c["na"]], 3.0, rtol=1e-14)
        assert np.allclose(rc[c["na"]:], 5.0, rtol=1e-14)
        # band nodes reached by the transport carry the ghost value (NaN: not reached)
        reached = ~np.isnan(band)
        assert np.all(np.abs(band[reached] - 3.0) < 1e-14)
        assert reached.mean() > 0.9


def test_prolongation_reproduces_linear_functions(oracle_mod):
    H = oracle_mod.Hierarchy(I.disk(65), 2, 65, coarsest_n=5)
    for l in range(H.nlev - 1):
        f = H.level_info(l); c = H.level_info(l + 1)
        xf, yf = I.grid_points(f["n"], 2)
        xc, yc = I.grid_points(c["n"], 2)
        gf = H.compact_to_grid(l); gc = H.compact_to_grid(l + 1)
        lin = lambda x, y: 0.3 + 1.7 * x - 0.9 * y
        ec = np.concatenate([lin(xc[gc], yc[gc]), 2 * lin(xc[gc], yc[gc])])
        out = H.prolong_add(l, ec, np.zeros(2 * f["na"]))
        # fine nodes whose coarse contributors are all active get the exact linear value
        ctype = np.zeros(c["n"] ** 2, dtype=bool)
        ctype[gc] = True
        ok = 0
        for r, g in enumerate(gf):
            i, j = g % f["n"], g // f["n"]
            cis = {i // 2, (i + 1) // 2}
            cjs = {j // 2, (j + 1) // 2}
            if all(ctype[ci + c["n"] * cj] for ci in cis for cj in cjs):
                assert abs(out[r] - lin(xf[g], yf[g])) < 1e-13
                assert abs(out[f["na"] + r] - 2 * lin(xf[g], yf[g])) < 1e-13
                ok += 1
        if f["na"] > 200:
            assert ok > 0.7 * f["na"]


def test_dense_lu_matches_numpy(oracle_mod):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40)) + 10 * np.eye(40)
    b = rng.standard_normal(40)
    assert np.allclose(oracle_mod.lu_solve_dense(A, b), np.linalg.solve(A, b), rtol=1e-12, atol=1e-12)
    P = np.array([[0.0, 2.0, 1.0], [1.0, 0.0, 3.0], [4.0, 1.0, 0.0]])
    b = np.array([1.0, 2.0, 3.0])
    assert np.allclose(oracle_mod.lu_solve_dense(P, b), np.linalg.solve(P, b), rtol=1e-13)


def test_mms_sources_match_symbolic_derivatives():
    sp = pytest.importorskip("sympy")
    x, y, t = sp.symbols("x y t")
    M = I.MODEL
    s = 2 + sp.sin(x) * sp.cos(y) * sp.sin(t + sp.sqrt(2))
    c = 3 + sp.sin(x / 2) * sp.cos(3 * y) * sp.sin(2 * t + sp.sqrt(3))
    por = M["alpha"] * c + M["beta"]
    f1 = sp.diff(por * s, t) + M["a"] / M["m_c"] * por * s * c - M["d"] * (sp.diff(por * sp.diff(s, x), x) + sp.diff(por * sp.diff(s, y), y))
    f2 = sp.diff(c, t) + M["a"] / M["m_s"] * por * s * c
    F1 = sp.lambdify((x, y, t), f1, "numpy")
    F2 = sp.lambdify((x, y, t), f2, "numpy")
    rng = np.random.default_rng(0)
    X, Y, T = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50), rng.uniform(0, 1, 50)
    g1, g2 = I.mms_sources(X, Y, T)
    assert np.allclose(g1, F1(X, Y, T), rtol=1e-13, atol=1e-12)
    assert np.allclose(g2, F2(X, Y, T), rtol=1e-13, atol=1e-12)
