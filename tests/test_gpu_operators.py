"""Each component of the V-cycle on the GPU against the oracle on identical inputs:
residual F, J x, one smoothing step, the defect, restriction, prolongation, the
coarse linearisation point, the coarsest solve and a whole V-cycle, on every level."""
import numpy as np
import pytest

import lsmg_inputs as I
from _gpu import cuda, host, pair, random_state, rel, say

CASES = [("disk", 65, 5), ("star", 257, 9), ("torus", 33, 9)]
TOL = 1e-12


def _setup(kind, n, coarsest, seed=7):
    H, O = pair(kind, n, coarsest)
    rng = np.random.default_rng(seed)
    W = random_state(O, 0, rng)
    dt = 1e-3
    H.set_linearization(cuda(W), dt)
    O.set_linearization(W, dt)
    return H, O, rng, dt, W


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest", CASES)
def test_residual(kind, n, coarsest):
    say(f"residual {kind} n={n}")
    H, O = pair(kind, n, coarsest)
    rng = np.random.default_rng(3)
    W, Wn = random_state(O, 0, rng), random_state(O, 0, rng)
    info = O.level_info(0)
    sb = rng.uniform(0.5, 1.5, info["ng"])
    fn, fnp1 = rng.standard_normal(2 * info["na"]), rng.standard_normal(2 * info["na"])
    for dt in (1e-3, 1e-4):
        Fg, ng = H.residual(cuda(W), cuda(Wn), dt, sb=cuda(sb), fn=cuda(fn), fnp1=cuda(fnp1))
        Fo, no = O.residual(W, Wn, dt, sb, fn, fnp1)
        assert rel(host(Fg), Fo) <= TOL
        assert abs(ng - no) <= TOL * no
    Fg, _ = H.residual(cuda(W), cuda(Wn), 1e-3, sb=None, sb_const=0.7)
    Fo, _ = O.residual(W, Wn, 1e-3, np.full(info["ng"], 0.7))
    assert rel(host(Fg), Fo) <= TOL


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest", CASES)
def test_linearization_and_operators(kind, n, coarsest):
    say(f"operators {kind} n={n}")
    H, O, rng, dt, W = _setup(kind, n, coarsest)
    for l in range(O.nlev):
        na = O.level_info(l)["na"]
        assert rel(host(H.level_state(l)), O.level_state(l)) <= TOL, ("state", l)
        x = rng.standard_normal(2 * na)
        rhs = rng.standard_normal(2 * na)
        assert rel(host(H.apply_J(l, cuda(x))), O.apply_J(l, x)) <= TOL, ("J", l)
        rg, ng = H.defect(l, cuda(rhs), cuda(x))
        ro, no = O.defect(l, rhs, x)
        assert rel(host(rg), ro) <= TOL and abs(ng - no) <= TOL * no, ("defect", l)
        for sweeps in (1, 2):
            assert rel(host(H.smooth(l, cuda(rhs), cuda(x), sweeps)), O.smooth(l, rhs, x, sweeps)) <= 1e-11, \
                ("smooth", l, sweeps)
        if l + 1 < O.nlev:
            nc = O.level_info(l + 1)["na"]
            r = rng.standard_normal(2 * na)
            assert rel(host(H.restrict(l, cuda(r))), O.restrict(l, r)) <= TOL, ("restrict", l)
            e = rng.standard_normal(2 * nc)
            assert rel(host(H.prolong_add(l, cuda(e), cuda(x))), O.prolong_add(l, e, x)) <= TOL, ("prolong", l)
    lc = O.nlev - 1
    rhs = rng.standard_normal(2 * O.level_info(lc)["na"])
    assert rel(host(H.coarse_solve(cuda(rhs))), O.coarse_solve(rhs)) <= 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest", CASES)
def test_vcycle(kind, n, coarsest):
    say(f"vcycle {kind} n={n}")
    H, O, rng, dt, W = _setup(kind, n, coarsest)
    na = O.level_info(0)["na"]
    rhs = rng.standard_normal(2 * na)
    xg = cuda(np.zeros(2 * na))
    xo = np.zeros(2 * na)
    for q in range(3):
        xg, rg = H.vcycle(0, cuda(rhs), xg)
        xo, ro = O.vcycle(0, rhs, xo)
        assert rel(host(xg), xo) <= 1e-10, q
        # the defect of a nearly converged iterate is a difference of terms of the size of
        # rhs: its rounding is a few ulps of |rhs|, whatever the size of the defect itself
        assert abs(rg - ro) <= 1e-8 * ro + 1e-12 * np.max(np.abs(rhs)), q


# coarsest operators on either side of the sizes where the factorisation changes
# kernel: up to 96 unknowns two LDS copies with one barrier per pivot, up to 138 one
# LDS copy, beyond that the matrix in HBM (radius: a disc of that radius instead)
COARSE_CASES = [("star", 129, 17, None, 88), ("disk", 129, 33, 0.28, 97), ("disk", 129, 33, None, 165),
                ("torus", 33, 17, None, 480)]


@pytest.mark.gpu
@pytest.mark.parametrize("kind,n,coarsest,radius,na", COARSE_CASES)
def test_coarse_solve_sizes(kind, n, coarsest, radius, na):
    say(f"coarse solve {kind} n={n} coarsest={coarsest} na={na}")
    H, O = pair(kind, n, coarsest, phi=I.disk(n, r=radius) if radius else None)
    lc = O.nlev - 1
    assert O.level_info(lc)["na"] == na
    rng = np.random.default_rng(3)
    W = random_state(O, 0, rng)
    H.set_linearization(cuda(W), 1e-3)
    O.set_linearization(W, 1e-3)
    for _ in range(2):
        rhs = rng.standard_normal(2 * na)
        assert rel(host(H.coarse_solve(cuda(rhs))), O.coarse_solve(rhs)) <= 1e-11
