"""Input preparation on the GPU (sections 2 and 3.3) against the oracle: level set from
a mask, re-initialisation and second-order extrapolation on full grids in 2-D and
3-D (the same operations in the same order, so the same bits up to the square root),
and a whole run prepared that way: a pixel mask made a level set and re-initialised,
non-constant initial data extrapolated to the ghosts, then Crank-Nicolson steps of
the manufactured problem, each within 1e-10 of the oracle's."""
import numpy as np
import pytest
import torch

import lsmg_inputs as I
import oracle
from _gpu import cuda, host, oracle_params, rel, say
from paper_1902_07029_amd import lsmg


@pytest.mark.gpu
@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33)])
def test_levelset_from_mask_matches_oracle(dim, n):
    if dim == 2:
        mask = I.necklace_mask(n)
    else:
        mask = I.torus(n) < 0
    g = lsmg.levelset_from_mask(cuda(mask.astype(np.uint8)), dim, n, 6)
    o = oracle.levelset_from_mask(mask, dim, n, 6)
    assert np.array_equal(host(g), o)


@pytest.mark.gpu
@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33)])
def test_reinitialize_matches_oracle(dim, n):
    h = 2 / (n - 1)
    pts = I.grid_points(n, dim)
    r2 = sum(p * p for p in pts)
    phi0 = r2 - 0.25
    g = lsmg.reinitialize(cuda(phi0), dim, n, 80)
    o = oracle.reinitialize(phi0, dim, n, h, 80)
    say(f"reinitialize dim {dim}: max |gpu - oracle| {np.max(np.abs(host(g) - o)):.2e}")
    assert np.max(np.abs(host(g) - o)) <= 1e-13


@pytest.mark.gpu
@pytest.mark.parametrize("dim,n", [(2, 129), (3, 33)])
def test_extrapolate_matches_oracle(dim, n):
    h = 2 / (n - 1)
    pts = I.grid_points(n, dim)
    phi = I.disk(n) if dim == 2 else I.torus(n)
    q = 2.0 + np.sin(pts[0]) * np.cos(pts[1]) + (0.3 * pts[2] if dim == 3 else 0.0)
    g = lsmg.extrapolate(cuda(phi), cuda(q), dim, n, 40)
    o = oracle.extrapolate(phi, dim, n, h, q, 40)
    say(f"extrapolate dim {dim}: max |gpu - oracle| {np.max(np.abs(host(g) - o)):.2e}")
    assert np.max(np.abs(host(g) - o)) <= 1e-13 * np.max(np.abs(o))
    assert np.array_equal(host(g)[phi < 0], q[phi < 0])


@pytest.mark.gpu
def test_prepared_run_matches_oracle():
    n = 129
    h = 2 / (n - 1)
    mask = I.necklace_mask(n)
    phi_g = lsmg.reinitialize(lsmg.levelset_from_mask(cuda(mask.astype(np.uint8)), 2, n, 4), 2, n, 30)
    phi = oracle.reinitialize(oracle.levelset_from_mask(mask, 2, n, 4), 2, n, h, 30)
    assert np.array_equal(host(phi_g), phi)
    # each side builds from its own prepared level set and extrapolates its own data
    p = lsmg.default_params(coarsest_n=9)
    H = lsmg.Hierarchy(phi_g, 2, n, params=p)
    O = oracle.Hierarchy(phi, 2, n, coarsest_n=9, params=oracle_params(H.params))
    x, y = I.grid_points(n, 2)
    phi_gh = host(phi_g)
    s0, c0 = I.s_exact(x, y, 0.0), I.c_exact(x, y, 0.0)
    s0g, c0g = s0.copy(), c0.copy()
    s0[phi >= 0] = 0.0
    c0[phi >= 0] = 0.0
    s0g[phi_gh >= 0] = 0.0
    c0g[phi_gh >= 0] = 0.0
    sg = lsmg.extrapolate(phi_g, cuda(s0g), 2, n, 40)
    cg = lsmg.extrapolate(phi_g, cuda(c0g), 2, n, 40)
    so = oracle.extrapolate(phi, 2, n, h, s0, 40)
    co = oracle.extrapolate(phi, 2, n, h, c0, 40)
    st = lsmg.State(H)
    st.set_grid(sg, cg)
    W = O.to_compact(0, so, co)
    na = O.level_info(0)["na"]
    assert rel(host(st.get()), W) <= 1e-13
    g, gg = O.compact_to_grid(0), host(H.compact_to_grid(0))
    B, Bg = O.ghost_table(0)["B"], host(H.ghost_table(0)["B"])
    dt = 1e-3

    def forcing(t, idx):
        return np.concatenate(I.mms_sources(x[idx], y[idx], t))

    for k in range(3):
        t0, t1 = k * dt, (k + 1) * dt
        st.step(dt, sb=cuda(I.s_exact(Bg[:, 0], Bg[:, 1], t1)), fn=cuda(forcing(t0, gg)),
                fnp1=cuda(forcing(t1, gg)))
        rc, W, _ = O.newton_cn_step(W, dt, I.s_exact(B[:, 0], B[:, 1], t1), forcing(t0, g), forcing(t1, g))
        assert rc == 0
        G = host(st.get())
        es, ec = rel(G[:na], W[:na]), rel(G[na:], W[na:])
        say(f"prepared necklace run step {k}: err s {es:.2e} c {ec:.2e}")
        assert es <= 1e-10 and ec <= 1e-10
