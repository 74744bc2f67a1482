"""Pins of the oracle's input preparation (sections 2 and 3.3), against facts fixed by
the mathematics:

* re-initialisation: a signed distance to a straight line is a fixed point; from
  phi0 = r^2 - R^2 (not a distance) it approaches r - R near the interface, with an
  error that halves under refinement; the sign of phi0 is kept at every node, also
  for a disc of 11 cells made a level set from its mask;
* level set from a mask: keeps the mask's inside where the mask is not within a
  couple of cells of its edge, and is symmetric for a symmetric mask;
* second-order extrapolation: exact for a linear function across a straight
  interface (normal derivative constant, second derivative zero); second-order
  convergence at the ghost nodes of a circle for a smooth function; values inside
  unchanged bit for bit.
"""
import numpy as np

import lsmg_inputs as I


def _ghosts(phi, n):
    P = phi.reshape(n, n)
    ins = P < 0
    nb = np.zeros_like(ins)
    nb[1:, :] |= ins[:-1, :]
    nb[:-1, :] |= ins[1:, :]
    nb[:, 1:] |= ins[:, :-1]
    nb[:, :-1] |= ins[:, 1:]
    return (~ins & nb).reshape(-1)


def test_reinitialize_fixed_point_and_distance(oracle_mod):
    n = 65
    h = 2 / (n - 1)
    x, y = I.grid_points(n, 2)
    p = x - 0.3
    assert np.max(np.abs(oracle_mod.reinitialize(p, 2, n, h, 60) - p)) <= 1e-14
    errs = []
    for n in (65, 129, 257):
        h = 2 / (n - 1)
        x, y = I.grid_points(n, 2)
        r = np.hypot(x, y)
        p0 = r ** 2 - 0.25
        p = oracle_mod.reinitialize(p0, 2, n, h, int(4.4 / h))
        errs.append(np.max(np.abs(p - (r - 0.5))[np.abs(r - 0.5) < 0.25]))
        assert np.array_equal(np.sign(p), np.sign(p0))
    assert errs[0] < 1e-2 and errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_reinitialize_keeps_small_shapes(oracle_mod):
    # a disc of radius 0.17 (11 cells at 129^2) made a level set from its mask: the zero
    # level set stays where the mask put it, and the values approach r - R
    n = 129
    h = 2 / (n - 1)
    x, y = I.grid_points(n, 2)
    r = np.hypot(x, y)
    p1 = oracle_mod.levelset_from_mask(r < 0.17, 2, n, 4)
    p2 = oracle_mod.reinitialize(p1, 2, n, h, int(2.0 / h))
    assert np.array_equal(np.sign(p2), np.sign(p1))
    assert np.max(np.abs(p2 - (r - 0.17))[np.abs(r - 0.17) < 0.1]) < 1e-2


def test_levelset_from_mask(oracle_mod):
    n = 65
    x, y = I.grid_points(n, 2)
    mask = (np.abs(x) < 0.5) & (np.abs(y) < 0.3)
    p = oracle_mod.levelset_from_mask(mask, 2, n, 5)
    h = 2 / (n - 1)
    deep = (np.abs(x) < 0.5 - 3 * h) & (np.abs(y) < 0.3 - 3 * h)
    far = (np.abs(x) > 0.5 + 3 * h) | (np.abs(y) > 0.3 + 3 * h)
    assert np.all(p[deep] < 0) and np.all(p[far] > 0)
    P = p.reshape(n, n)
    assert np.array_equal(P, P[:, ::-1]) and np.array_equal(P, P[::-1, :])


def test_extrapolation_exact_for_linear_data_across_a_line(oracle_mod):
    n = 65
    h = 2 / (n - 1)
    x, y = I.grid_points(n, 2)
    phi = x - 0.1
    q = 2 + 3 * x - y
    out = oracle_mod.extrapolate(phi, 2, n, h, q, 120)
    assert np.array_equal(out[phi < 0], q[phi < 0])
    # rows at the box edge have no central difference across them: left out
    off_edge = np.abs(np.abs(y) - 1) > 1e-12
    band = (phi >= 0) & (phi < 4 * h) & off_edge
    assert np.max(np.abs(out - q)[band]) <= 1e-12


def test_extrapolation_second_order_at_ghosts(oracle_mod):
    errs = []
    for n in (65, 129, 257):
        h = 2 / (n - 1)
        x, y = I.grid_points(n, 2)
        phi = I.disk(n)
        q = I.s_exact(x, y, 0.3)
        out = oracle_mod.extrapolate(phi, 2, n, h, q, 40)
        assert np.array_equal(out[phi < 0], q[phi < 0])
        errs.append(np.max(np.abs(out - q)[_ghosts(phi, n)]))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), orders
    assert errs[-1] < 3e-5
